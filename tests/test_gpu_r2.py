"""The finite-record weighting on the GPU against the oracle.

Hhat_W(w) = (1/Nt) sum_p Ghat_p Ghat_p^H with Ghat_p the DFT truncated after
sample p (the paper's weighting function W(m, n) = min(Nt - m, Nt - n) kept
exactly, as the oracle's running-DFT Gram, pinned against the literal
algorithm).  Cases: tiny with nt = 300 (one full 256-sample window and a
partial one), ragged with stride 2 and odd sizes, and tiny end to end with the
1e-5 multiplier target.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fd, hessian, solve

pytestmark = pytest.mark.gpu


from parity import check, rel  # noqa: E402


@pytest.fixture(scope="module")
def ehi():
    from paper_2512_16642_amd import ehi as mod
    mod.lib()
    return mod


def _oracle_r2(s, v):
    gt = fd.green_samples_c(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, s.stride)
    return hessian.hessian_r2(gt.reshape(s.nr, s.nt, -1), s.freqs_hz, s.dt)


def _gpu_r2(ehi, s, v):
    sv = ehi.survey_from(s, precision="split_bf16", weighting="finite_record")
    sv.build_green(torch.from_numpy(v).cuda())
    sv.build_hessian()
    H = sv.copy_hessian().cpu().numpy()
    return sv, H


@pytest.mark.parametrize("case", ["tiny_nt300", "ragged"])
def test_finite_record_hessian(ehi, case):
    s = synth.tiny().with_(nt=300) if case == "tiny_nt300" else synth.ragged()
    v = s.velocity()
    ref = _oracle_r2(s, v)
    sv, H = _gpu_r2(ehi, s, v)
    sv.close()
    for f in range(s.nf):
        np.testing.assert_array_equal(H[f], H[f].conj().T)
    check(H, ref, 5e-6, 5e-6, 1e-5, f"{case} finite-record Hhat")
    # the weighting changes the result: it is not the final-spectrum Gram
    r1 = hessian.hessian_r1(fd.green_dft(s, v))
    assert min(rel(H[f], r1[f] / s.nt) for f in range(s.nf)) > 1e-3


def test_finite_record_end_to_end_tiny(ehi):
    s = synth.tiny()
    v = s.velocity()
    ref = _oracle_r2(s, v)
    mu = 1e-3 * solve.lambda_max(ref)
    R = s.residuals()
    Xr = solve.multipliers(ref, mu, R.astype(np.complex128))
    sv, H = _gpu_r2(ehi, s, v)
    sv.factor(mu)
    X = sv.apply_multipliers(torch.from_numpy(R).cuda()).cpu().numpy()
    sv.close()
    check(X, Xr, 1e-5, 1e-5, 2e-5, "finite-record multipliers")


def test_finite_record_refuses_given_spectra(ehi):
    s = synth.ragged()
    sv = ehi.survey_from(s, weighting="finite_record")
    g = torch.zeros((s.nf, s.nr, s.nzs, s.nxs), dtype=torch.complex64, device="cuda")
    with pytest.raises(ehi.EhiError) as ei:
        sv.load_green_dft(g)
    assert ei.value.status == ehi.EHI_ESTATE
    sv.close()
