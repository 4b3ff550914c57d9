"""The steps either side of the deblur and the Hessian accuracy test.

Paper: the multiplier-based extended FWI algorithm, per source: the residual
dd = d - S b, the multipliers dd^e = Q^{-1} dd computed in the frequency domain,
the source extension db = S^T dd^e, and the extended wavefield
u^e = A^{-1}(b + db), whose traces are P u^e = S b + S db; the Hessian
accuracy test (numerical examples) scores RelErr = ||d - P u^e||^2 / ||d||^2,
and d - P u^e = dd - S S^T dd^e equals mu dd^e when the deblurring system is
solved exactly.

Every step is a call into the library (argument marshalling only): the 2nt-point
transform of the residuals, the resident factors' deblur, the inverse transform
cropped to the record, the adjoint and forward runs on the subgrid sources,
and the misfit reduction.
"""
from __future__ import annotations

from typing import Optional

from . import ehi


def deblur_time(sv: "ehi.Survey", dd, stream=None):
    """dd^e in time for time-domain residuals ``dd`` float32 [ns][nr][nt]:
    residual spectra at the survey's frequencies (bins of the 2nt-point
    transform), X = Qhat^{-1} R per frequency, inverse transform cropped to
    samples 1..nt.  Requires a factored survey."""
    R = sv.residual_spectra(dd, stream=stream)
    X = sv.apply_multipliers(R, stream=stream)
    return sv.multipliers_to_time(X, stream=stream)


def accuracy_test(sv: "ehi.Survey", dd, d_obs, db_out: Optional[object] = None) -> dict:
    """The accuracy test for a batch of sources.

    ``dd``: residuals d - S b, float32 [ns][nr][nt]; ``d_obs``: the observed
    data d (the normaliser), same shape.  Returns the multipliers ``dde``, the
    source extension ``db`` [ns][nt][nzs][nxs], the predicted change ``pred``
    = S db, the misfit ``err`` = dd - pred = d - P u^e and ``relerr`` [ns]
    (float64), all on the device.
    """
    dde = deblur_time(sv, dd)
    db = sv.backpropagate(dde, out=db_out)
    pred = sv.forward_subgrid(db)
    err, rel = ehi.misfit(dd, pred, d_obs)
    return {"dde": dde, "db": db, "pred": pred, "err": err, "relerr": rel}
