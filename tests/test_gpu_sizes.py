"""Parity of the contraction and of the factor + solve at every receiver count
the surveys use, from given inputs (the stage isolated from the stepping).

Seeded spectra (synth.spectra: rows mixed by a random unitary matrix, singular
values over four decades, so the Hessians' eigenvalues span eight) are loaded
through ehi_load_green_dft; the Hessian comes back through ehi_copy_hessian and
is compared with the oracle's FP64 contraction of the same complex64 values.
The receiver counts cover every form of the kernel: a single receiver (1), one
32 x 32 block (16), a ragged block count (33), the whole-matrix split-BF16 form
with every row staged (200, 224) and with 4 x 4 tiles of block pairs past it
(225, 256, 400, the largest batch survey, and 1024, the descriptor's limit),
in both precision modes; the 64 x 64 tile-pair form at 400 receivers too.  The subgrid (61 x 203 = 12,383 points) spans several
grid partitions and ends on a ragged tail.

Factor + solve from a given Hessian (the oracle's FP64 Hhat of the same
spectra, mu = 1e-3 lambda_max, so cond(Qhat) ~ 1e3 as in the surveys' low
frequencies) at 1, 33, 200, 256, 400 and 1024 receivers: the FP64 factor against scipy's, the
multipliers of 64 sources against the oracle's solve (a single source at 33
receivers, 47 sources at 200 receivers for a ragged source tile, 1408 at 256
receivers for a wide grid of source tiles).

Tolerances: 1e-6 per frequency for the split-BF16 Hessian at the default
partition counts (2e-6 for the forms and partition counts the autotuner may
choose, as for the tiny survey, tests/test_gpu_parity.py), 2.5e-7 for the
plain FP32 contraction, 1e-12 for the FP64 factor, and for the refined solve
1e-7 (the complex64 output's rounding is 6e-8 per element); the element-wise
and per-row measures of tests/parity.py beside them.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import hessian, solve
from parity import check

pytestmark = pytest.mark.gpu

NZ, NX, NF = 61, 203, 3


def _survey(nr, ns=64):
    s = synth.ragged(nz=NZ, nx=NX, nb=4, nt=16, nr=1, stride=1)
    return s.with_(rec_iz=tuple(k % 3 for k in range(nr)), rec_ix=tuple((7 * k) % NX for k in range(nr)),
                   freqs_hz=(4.0, 7.5, 11.0)[:NF], ns=ns)


@pytest.fixture(scope="module")
def ehi():
    from paper_2512_16642_amd import ehi as mod
    mod.lib()
    return mod


_CACHE = {}


def _spectra(nr):
    if nr not in _CACHE:
        G = synth.spectra(NF, nr, NZ * NX, seed=500 + nr)
        _CACHE[nr] = (G, hessian.hessian_r1(G.astype(np.complex128)))
    return _CACHE[nr]


@pytest.mark.parametrize("prec", ["split_bf16", "plain_fp32"])
@pytest.mark.parametrize("nr", [1, 16, 33, 200, 224, 225, 256, 400, 1024])
def test_hessian_from_given_spectra_sizes(ehi, nr, prec):
    s = _survey(nr)
    G, ref = _spectra(nr)
    sv = ehi.survey_from(s, precision=prec, nr_batch=8)
    sv.load_green_dft(torch.from_numpy(G.reshape(NF, nr, NZ, NX)).cuda())
    sv.build_hessian()
    H = sv.copy_hessian().cpu().numpy()
    sv.close()
    # split-BF16 (four hi/lo products, FP32 running sums per partition): up to
    # 3.3e-7 measured at 1024 receivers; FP32 operands on the FP32 matrix
    # cores: up to 1.3e-7 per row
    if prec == "split_bf16":
        check(H, ref, 1e-6, 1e-6, 1.5e-6, f"nr={nr} {prec} hessian")
    else:
        check(H, ref, 2.5e-7, 4e-7, 6e-7, f"nr={nr} {prec} hessian")
    for f in range(NF):
        np.testing.assert_array_equal(H[f], H[f].conj().T)
        d = np.diagonal(H[f])
        assert np.all(d.imag == 0) and np.all(d.real > 0)


@pytest.mark.parametrize("nr,ns", [(1, 64), (33, 1), (33, 64), (200, 64), (200, 47), (256, 64), (256, 1408),
                                   (400, 64), (1024, 64)])
def test_factor_and_solve_from_given_hessian_sizes(ehi, nr, ns):
    s = _survey(nr, ns)
    _, H = _spectra(nr)
    mu = 1e-3 * solve.lambda_max(H)
    R = synth.residuals(NF, s.ns, nr, seed=900 + nr)
    L = solve.cholesky(solve.penalize(H, mu))
    X = solve.solve(L, R.astype(np.complex128))
    sv = ehi.survey_from(s, precision="split_bf16", nr_batch=8)
    sv.load_hessian(torch.from_numpy(H).cuda())
    sv.factor(mu)
    Lg = sv.copy_factor().cpu().numpy()
    Xg = sv.apply_multipliers(torch.from_numpy(R).cuda()).cpu().numpy()
    sv.close()
    check(Lg, L, 1e-12, 1e-12, 1e-11, f"nr={nr} FP64 factor")
    # FP64 factor + one FP64 refinement step: the multipliers to the rounding
    # of their complex64 output (2^-24 = 6e-8 per element); without the
    # refinement step the error is several times larger
    check(Xg, X, 1e-7, 1.5e-7, 2e-7, f"nr={nr} ns={ns} solve")


@pytest.mark.parametrize("nr,form,split", [(200, 1, 1), (200, 1, 7), (200, 2, 3), (200, 2, 12), (200, 0, 64),
                                            (400, 2, 8), (400, 1, 5)])
def test_hessian_contraction_shapes(ehi, nr, form, split):
    # every form and partition count the autotuner may choose: the same
    # Hessian to rounding (partitions change only the order of FP32 partial
    # sums), within the contraction's tolerance of the oracle
    s = _survey(nr)
    G, ref = _spectra(nr)
    sv = ehi.survey_from(s, precision="split_bf16", nr_batch=8, herk_form=form, herk_split=split)
    sv.load_green_dft(torch.from_numpy(G.reshape(NF, nr, NZ, NX)).cuda())
    sv.build_hessian()
    H = sv.copy_hessian().cpu().numpy()
    sv.close()
    check(H, ref, 2e-6, 2e-6, 4e-6, f"nr={nr} form {form} split {split} hessian")
    for f in range(NF):
        np.testing.assert_array_equal(H[f], H[f].conj().T)


@pytest.mark.parametrize("form", [0, 3])
def test_plain_contraction_forms(ehi, form):
    # the plain FP32 form on the FP32 matrix cores (0) and on the vector units (3)
    nr = 225
    s = _survey(nr)
    G, ref = _spectra(nr)
    sv = ehi.survey_from(s, precision="plain_fp32", nr_batch=8, herk_form=form)
    sv.load_green_dft(torch.from_numpy(G.reshape(NF, nr, NZ, NX)).cuda())
    sv.build_hessian()
    H = sv.copy_hessian().cpu().numpy()
    sv.close()
    check(H, ref, 2e-6, 2e-6, 4e-6, f"plain form {form} hessian")
