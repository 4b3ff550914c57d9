"""The finite-record weighting on the GPU against the oracle.

Hhat_W(w) = (1/Nt) sum_p Ghat_p Ghat_p^H with Ghat_p the DFT truncated after
sample p (the paper's weighting function W(m, n) = min(Nt - m, Nt - n) kept
exactly, as the oracle's running-DFT Gram, pinned against the literal
algorithm).  Cases: tiny with nt = 300 (one full 256-sample window and a
partial one), ragged with stride 2 and odd sizes, 70 receivers (several
32-row blocks and block pairs), and tiny end to end with the 1e-5 multiplier
target.
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


def _wide():
    # 70 receivers: three 32-row blocks, six block pairs (two workgroups, the
    # second partial), a partial last block
    return synth.micro(nz=40, nx=80, nb=6, nt=300, nr=70)


@pytest.mark.parametrize("case", ["tiny_nt300", "ragged", "wide"])
def test_finite_record_hessian(ehi, case):
    s = {"tiny_nt300": lambda: synth.tiny().with_(nt=300), "ragged": synth.ragged, "wide": _wide}[case]()
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


# ---------------------------------------------------------------------------
# time-axis resampling of the record (descriptor field decim)
# ---------------------------------------------------------------------------

def _oracle_r2_dec(s, v, D):
    gt = fd.green_samples_c(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, s.stride).reshape(s.nr, s.nt, -1)
    return gt, hessian.hessian_r2_decimated(gt, s.freqs_hz, s.dt, D)


def _gpu_r2_dec(ehi, s, v, D, chunk=256):
    sv = ehi.survey_from(s, precision="split_bf16", weighting="finite_record", decim=D, chunk=chunk)
    sv.build_green(torch.from_numpy(v).cuda())
    sv.build_hessian()
    return sv, sv.copy_hessian().cpu().numpy(), sv.copy_green_dft().reshape(s.nf, s.nr, -1).cpu().numpy()


@pytest.mark.parametrize("case,D,chunk", [("tiny", 10, 256), ("tiny", 4, 512), ("ragged", 3, 256),
                                          ("ragged_long", 8, 256), ("wide", 5, 256)])
def test_resampled_finite_record_hessian(ehi, case, D, chunk):
    # against the oracle's finite-record Hessian on the same resampled record
    # (same filter design, kept times and D / H(w) correction); several
    # windows, kept samples straddling window edges, a partial last window
    if case == "tiny":
        s = synth.tiny()
    elif case == "ragged":
        s = synth.ragged()
    elif case == "wide":
        s = _wide()
    else:
        s = synth.ragged(nt=1157)
    v = s.velocity()
    gt, ref = _oracle_r2_dec(s, v, D)
    sv, H, G = _gpu_r2_dec(ehi, s, v, D, chunk)
    sv.close()
    for f in range(s.nf):
        np.testing.assert_array_equal(H[f], H[f].conj().T)
    check(H, ref, 5e-6, 5e-6, 1e-5, f"{case} D={D} resampled finite-record Hhat")
    # the corrected running spectra at the end are the record's spectra
    check(G, fd.dft(gt, s.freqs_hz, s.dt), 5e-6, 5e-6, 2e-5, f"{case} D={D} resampled spectra")


def test_resampled_finite_record_end_to_end_tiny(ehi):
    s = synth.tiny()
    v = s.velocity()
    _, ref = _oracle_r2_dec(s, v, 10)
    mu = 1e-3 * solve.lambda_max(ref)
    R = s.residuals()
    Xr = solve.multipliers(ref, mu, R.astype(np.complex128))
    sv, H, _ = _gpu_r2_dec(ehi, s, v, 10)
    sv.factor(mu)
    X = sv.apply_multipliers(torch.from_numpy(R).cuda()).cpu().numpy()
    sv.close()
    check(X, Xr, 1e-5, 1e-5, 2e-5, "resampled finite-record multipliers")


def test_resampling_factor_one_is_the_whole_record(ehi):
    s = synth.ragged()
    v = s.velocity()
    _, H1, G1 = _gpu_r2_dec(ehi, s, v, 1)
    sv, H0 = _gpu_r2(ehi, s, v)
    G0 = sv.copy_green_dft().reshape(s.nf, s.nr, -1).cpu().numpy()
    sv.close()
    np.testing.assert_array_equal(H1, H0)
    np.testing.assert_array_equal(G1, G0)


def test_resampling_descriptor_checks(ehi):
    s = synth.tiny()
    with pytest.raises(ehi.EhiError):       # long-record weighting
        ehi.survey_from(s, decim=4)
    with pytest.raises(ehi.EhiError):       # stopband below the passband: 1/(D dt) < 2 f_max
        ehi.survey_from(s, weighting="finite_record", decim=60)
    with pytest.raises(ehi.EhiError):       # filter longer than the window allows
        ehi.survey_from(s, weighting="finite_record", decim=40, chunk=256)
