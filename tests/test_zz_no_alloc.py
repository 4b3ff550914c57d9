"""The batched factorisation's no-allocation entry point (static job table)
against the entry point with a caller-provided job table, through the C ABI.

Two calls in a row on the same device, the second with a smaller batch (fewer
surveys, fewer frequencies, fewer receivers), each compared bitwise with
ehi_factor_batch on an identical set of surveys: factors, the triangular
inverses' effect on the deblur (multipliers), and the FP64 factor against the
oracle's Cholesky (1e-12).  Also: a batch beyond the table is refused with
EHI_EINVAL, and a non-positive pivot is reported with its survey and frequency.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import hessian, solve
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ehi():
    from paper_2512_16642_amd import ehi as mod
    mod.lib()
    return mod


def _surveys(ehi, specs):
    out = []
    for k, (nr, nf) in enumerate(specs):
        s = synth.ragged(nz=41, nx=67, nb=6, nt=40, nr=1, stride=1).with_(
            rec_iz=tuple(k2 % 3 for k2 in range(nr)), rec_ix=tuple((5 * k2) % 67 for k2 in range(nr)),
            freqs_hz=tuple(3.0 + 2.0 * f for f in range(nf)), ns=12)
        G = synth.spectra(nf, nr, s.nsub, seed=700 + 10 * k + nr)
        H = hessian.hessian_r1(G.astype(np.complex128))
        mu = 1e-3 * solve.lambda_max(H)
        out.append((s, H, mu))
    return out


def _run(ehi, cases, static):
    svs, mus = [], []
    for s, H, mu in cases:
        sv = ehi.survey_from(s, precision="split_bf16")
        sv.load_hessian(torch.from_numpy(H).cuda())
        svs.append(sv)
        mus.append(mu)
    (ehi.factor_batch_static if static else ehi.factor_batch)(svs, mus)
    res = []
    for (s, H, mu), sv in zip(cases, svs):
        R = torch.from_numpy(s.residuals()).cuda()
        res.append((sv.copy_factor().cpu().numpy(), sv.apply_multipliers(R).cpu().numpy()))
        sv.close()
    return res


def test_static_job_table_matches_workspace_table_twice(ehi):
    for specs in ([(40, 5), (33, 3), (70, 4)], [(17, 2), (25, 3)]):
        cases = _surveys(ehi, specs)
        a = _run(ehi, cases, static=True)
        b = _run(ehi, cases, static=False)
        for (s, H, mu), (La, Xa), (Lb, Xb) in zip(cases, a, b):
            np.testing.assert_array_equal(La, Lb)
            np.testing.assert_array_equal(Xa, Xb)
            check(La, solve.cholesky(solve.penalize(H, mu)), 1e-12, 1e-12, 1e-11, f"static factor nr={s.nr}")


def test_static_job_table_limits_and_pivots(ehi):
    cases = _surveys(ehi, [(16, 4)])
    s, H, mu = cases[0]
    sv = ehi.survey_from(s)
    Hb = np.array(H)
    Hb[1] = -np.eye(s.nr)
    sv.load_hessian(torch.from_numpy(Hb).cuda())
    with pytest.raises(ehi.EhiError) as e:
        ehi.factor_batch_static([sv], [1e-3])
    assert e.value.status == ehi.EHI_ENOTPD and e.value.bad_freq == 1 and e.value.bad_survey == 0
    # more (survey, frequency) jobs than the static table holds: 65 surveys x 64 frequencies
    big = s.with_(freqs_hz=tuple(1.0 + f for f in range(64)))
    many = [ehi.survey_from(big) for _ in range(65)]
    for m in many:
        m.load_hessian(torch.zeros((64, s.nr, s.nr), dtype=torch.complex128, device="cuda"))
    with pytest.raises(ehi.EhiError) as e:
        ehi.factor_batch_static(many, [1.0] * len(many))
    assert e.value.status == ehi.EHI_EINVAL
    for m in many:
        m.close()
    sv.close()
