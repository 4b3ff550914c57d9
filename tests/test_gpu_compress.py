"""Spatially compressed contraction on the GPU against the oracle.

Each spectrum row (an nzs x nxs image) is transformed by the orthonormal 2D
DCT-II and cropped to the leading keep_z x keep_x coefficients before the
contraction (FP32 products, FP64 sums, in either precision mode).  The spectra are the oracle's own (loaded into the survey), so the
comparison isolates the transform and the contraction; keeping every
coefficient must reproduce the uncompressed Hessian.
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


def _gpu_hessian(ehi, s, G, keep, precision="split_bf16"):
    sv = ehi.survey_from(s, precision=precision, keep=keep)
    sv.load_green_dft(torch.from_numpy(np.ascontiguousarray(G.astype(np.complex64)).reshape(
        s.nf, s.nr, s.nzs, s.nxs)).cuda())
    sv.build_hessian()
    return sv, sv.copy_hessian().cpu().numpy()


@pytest.mark.parametrize("case,keep", [("tiny", (50, 40)), ("tiny", (101, 101)), ("ragged", (7, 13))])
def test_compressed_hessian(ehi, case, keep):
    s = synth.tiny() if case == "tiny" else synth.ragged()
    G = fd.green_dft(s, s.velocity()).astype(np.complex64)
    ref = hessian.hessian_compressed(G.astype(np.complex128), s.nzs, s.nxs, *keep)
    sv, H = _gpu_hessian(ehi, s, G, keep)
    sv.close()
    full = hessian.hessian_r1(G.astype(np.complex128))
    approx = [rel(ref[f], full[f]) for f in range(s.nf)]
    print(case, keep, "compression error of the method", approx)
    check(H, ref, 5e-7, 5e-7, 1e-6, f"{case} {keep} compressed Hhat")
    if keep == (s.nzs, s.nxs):
        check(H, full, 5e-7, 5e-7, 1e-6, f"{case} all coefficients vs uncompressed Hhat")


def test_compressed_end_to_end_plain_and_split(ehi):
    s = synth.tiny()
    G = fd.green_dft(s, s.velocity()).astype(np.complex64)
    keep = (60, 60)
    ref = hessian.hessian_compressed(G.astype(np.complex128), s.nzs, s.nxs, *keep)
    mu = 1e-3 * solve.lambda_max(ref)
    R = s.residuals()
    Xr = solve.multipliers(ref, mu, R.astype(np.complex128))
    sv, _ = _gpu_hessian(ehi, s, G, keep)
    sv.factor(mu)
    X = sv.apply_multipliers(torch.from_numpy(R).cuda()).cpu().numpy()
    sv.close()
    check(X, Xr, 1e-6, 1e-6, 2e-6, "compressed multipliers")


def test_compressed_build_in_receiver_batches(ehi):
    # build_green on a compressed survey transforms each receiver batch's
    # spectra as soon as they are complete (batches of 3 and 2 receivers): the
    # compressed spectra against the oracle's transform of its own spectra,
    # the Hessian end to end; the full spectra are not held
    s = synth.ragged()
    keep = (9, 17)
    v = s.velocity()
    G = fd.green_dft(s, v)
    Cref = hessian.compress_spectra(G, s.nzs, s.nxs, *keep)
    Href = hessian.hessian_r1(Cref)
    sv = ehi.survey_from(s, precision="split_bf16", keep=keep, nr_batch=3)
    sv.build_green(torch.from_numpy(v).cuda())
    sv.build_hessian()
    C = sv.copy_compressed().reshape(s.nf, s.nr, -1).cpu().numpy()
    H = sv.copy_hessian().cpu().numpy()
    with pytest.raises(ehi.EhiError):
        sv.copy_green_dft()
    sv.close()
    check(C, Cref, 5e-6, 5e-6, 2e-5, "compressed spectra, built in batches")
    check(H, Href, 1e-5, 1e-5, 2e-5, "compressed Hhat end to end")

