"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances, derived from the arithmetic of each stage:
  * Green-function spectra: FP32 increment-form stepping (~1e-6 relative,
    measured on FP32 emulations of the recurrence) plus FP32 chunked DFT sums:
    5e-6 per frequency (relative Frobenius).
  * Hessian from given spectra: FP32 products, two-level FP32 accumulation and
    an FP64 reduction of the grid partitions: 2e-6.
  * Factor + solve from a given Hessian, split-BF16 mode: FP64 Cholesky, FP32
    solves refined once in FP64 (the default), output rounded to complex64: 2e-6.
  * End to end (split-BF16 mode): the multiplier target 1e-5.
Beside each relative Frobenius bound, the largest element-wise difference is
bounded relative to the largest reference entry of the frequency slice, and
per row (receiver spectrum, Hessian row, source) relative to that row's largest
entry (tests/parity.py).
Inputs are the seeded synthetic surveys of ``synth``; the oracle sees the same
float32 velocity and complex64 residuals, upcast.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fd, hessian, solve

pytestmark = pytest.mark.gpu

DEV = "cuda"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


from parity import check  # noqa: E402


@pytest.fixture(scope="module")
def ehi():
    from paper_2512_16642_amd import ehi as mod
    mod.lib()
    return mod


@pytest.fixture(scope="module")
def tiny_ref():
    s = synth.tiny()
    v = s.velocity()
    G = fd.green_dft(s, v)                       # [nf][nr][nsub] c128
    H = hessian.hessian_r1(G)
    mu = 1e-3 * solve.lambda_max(H)
    R = s.residuals()
    X = solve.multipliers(H, mu, R.astype(np.complex128))
    return dict(s=s, v=v, G=G, H=H, mu=mu, R=R, X=X)


def _gpu_green(ehi, s, v, precision="split_bf16", nr_batch=0):
    sv = ehi.survey_from(s, precision=precision, nr_batch=nr_batch)
    sv.build_green(dev(v))
    G = sv.copy_green_dft().reshape(s.nf, s.nr, -1)
    torch.cuda.synchronize()
    return sv, G.cpu().numpy()


def test_green_dft_tiny(ehi, tiny_ref):
    s = tiny_ref["s"]
    sv, G = _gpu_green(ehi, s, tiny_ref["v"])
    check(G, tiny_ref["G"], 5e-6, 5e-6, 2e-5, "tiny ghat")


def test_green_dft_ragged_stride2(ehi):
    s = synth.ragged()
    v = s.velocity()
    ref = fd.green_dft(s, v)
    sv, G = _gpu_green(ehi, s, v)
    check(G, ref, 5e-6, 5e-6, 2e-5, "ragged ghat")


def test_green_receiver_batches_identical(ehi):
    s = synth.ragged()
    v = s.velocity()
    _, G_all = _gpu_green(ehi, s, v)
    _, G_b2 = _gpu_green(ehi, s, v, nr_batch=2)
    np.testing.assert_array_equal(G_all, G_b2)


def test_launch_shapes_bitwise_identical(ehi):
    # every (time levels, band width, segment rows) gives the same bits; the grid
    # spans several bands for every width, the receivers sit near band edges and
    # nt = 121 ends on a partial launch
    s = synth.ragged(nz=45, nx=1100, nb=9, nt=121, nr=4).with_(
        rec_iz=(1, 2, 3, 1), rec_ix=(215, 440, 700, 1090))
    v = s.velocity()
    ref = None
    for tb in (4, 8):
        for band in (256, 384, 448, 512):
            for seg in (16, 256):
                sv = ehi.survey_from(s)
                sv.set_launch(tb, seg, band)
                assert sv.get_launch() == (tb, seg, band)
                sv.build_green(dev(v))
                G = sv.copy_green_dft().reshape(s.nf, s.nr, -1).cpu().numpy()
                sv.close()
                if ref is None:
                    ref = G
                else:
                    np.testing.assert_array_equal(G, ref, err_msg=f"T={tb} band={band} seg={seg}")
    check(ref, fd.green_dft(s, v), 5e-6, 5e-6, 2e-5, "wide ragged ghat")


@pytest.mark.parametrize("chunk", [512, 1024])
def test_green_dft_longer_sample_windows(ehi, tiny_ref, chunk):
    # a longer staging window changes only the grouping of the DFT sums (1024 >
    # nt = 1000: one partial window)
    s = tiny_ref["s"]
    sv = ehi.survey_from(s, chunk=chunk)
    sv.build_green(dev(tiny_ref["v"]))
    G = sv.copy_green_dft().reshape(s.nf, s.nr, -1).cpu().numpy()
    sv.close()
    check(G, tiny_ref["G"], 5e-6, 5e-6, 2e-5, f"{chunk}-sample window ghat")


@pytest.mark.parametrize("chunk,nr_batch", [(256, 0), (256, 2), (512, 3), (1024, 0)])
def test_two_staging_windows_bitwise_identical(ehi, chunk, nr_batch):
    # the DFT of each window on the second stream, overlapped with the steps of
    # the next: same kernels, same order of accumulation, so the same bits;
    # nt = 1157 leaves a partial last window, receiver batches restart the
    # windows
    s = synth.ragged(nt=1157)
    v = s.velocity()
    out = []
    for windows in (1, 2):
        sv = ehi.survey_from(s, chunk=chunk, nr_batch=nr_batch, windows=windows)
        sv.build_green(dev(v))
        sv.build_green(dev(v))       # a second build on the same handle
        out.append(sv.copy_green_dft().cpu().numpy())
        sv.close()
    np.testing.assert_array_equal(out[1], out[0])


def test_two_staging_windows_finite_record_identical(ehi):
    s = synth.ragged(nt=700)
    v = s.velocity()
    out = []
    for windows in (1, 2):
        sv = ehi.survey_from(s, chunk=256, weighting="finite_record", windows=windows)
        sv.build_green(dev(v))
        sv.build_hessian()
        out.append(sv.copy_hessian().cpu().numpy())
        sv.close()
    np.testing.assert_array_equal(out[1], out[0])


def test_green_single_step_and_chunk_edges(ehi):
    # nt = 1 (only the impulse sample), nt = 64 and 65 (DFT chunk edge)
    base = synth.ragged(nt=1)
    for nt in (1, 64, 65):
        s = base.with_(nt=nt)
        v = s.velocity()
        ref = fd.green_dft(s, v)
        _, G = _gpu_green(ehi, s, v)
        check(G, ref, 5e-6, 5e-6, 2e-5, f"nt={nt} ghat")


def test_hessian_from_given_spectra(ehi, tiny_ref):
    s = tiny_ref["s"]
    G64 = np.ascontiguousarray(tiny_ref["G"].astype(np.complex64))
    ref = hessian.hessian_r1(G64.astype(np.complex128))
    for prec in ("split_bf16", "plain_fp32"):
        sv = ehi.survey_from(s, precision=prec)
        sv.load_green_dft(dev(G64.reshape(s.nf, s.nr, s.nzs, s.nxs)))
        sv.build_hessian()
        H = sv.copy_hessian().cpu().numpy()
        check(H, ref, 2e-6, 2e-6, 4e-6, f"{prec} hessian")
        for f in range(s.nf):
            np.testing.assert_array_equal(H[f], H[f].conj().T)
            assert np.all(np.diag(H[f]).imag == 0) and np.all(np.diag(H[f]).real > 0)


def test_factor_and_solve_from_given_hessian(ehi, tiny_ref):
    s = tiny_ref["s"]
    H = tiny_ref["H"]
    mu = tiny_ref["mu"]
    R = tiny_ref["R"]
    Lref = solve.cholesky(solve.penalize(H, mu))
    Xref = tiny_ref["X"]
    sv = ehi.survey_from(s, precision="split_bf16")
    sv.load_hessian(dev(H))
    sv.factor(mu)
    Lg = sv.copy_factor().cpu().numpy()
    check(Lg, Lref, 1e-12, 1e-12, 1e-11, "FP64 factor")
    X = sv.apply_multipliers(dev(R)).cpu().numpy()
    check(X, Xref, 2e-6, 2e-6, 4e-6, "split mode solve")
    # plain FP32 mode: FP32 Cholesky and solves, error ~ cond(Qhat) * 2^-24
    sp = ehi.survey_from(s, precision="plain_fp32")
    sp.load_hessian(dev(H))
    sp.factor(mu)
    Xp = sp.apply_multipliers(dev(R)).cpu().numpy()
    check(Xp, Xref, 1e-2, 1e-2, None, "plain mode solve")


def test_end_to_end_tiny(ehi, tiny_ref):
    s = tiny_ref["s"]
    sv = ehi.survey_from(s, precision="split_bf16")
    sv.build_green(dev(tiny_ref["v"]))
    sv.build_hessian()
    sv.factor(tiny_ref["mu"])
    X = sv.apply_multipliers(dev(tiny_ref["R"])).cpu().numpy()
    check(X, tiny_ref["X"], 1e-5, 1e-5, 2e-5, "end-to-end multipliers")


def test_end_to_end_tiny_plain_form(ehi, tiny_ref):
    # the plain FP32 form (FP32 contraction, FP32 Cholesky, no refinement): its
    # error is bounded by cond(Qhat) * 2^-24-sized terms, far looser than the
    # split form's; recorded for the comparison of the two forms
    s = tiny_ref["s"]
    sv = ehi.survey_from(s, precision="plain_fp32")
    sv.build_green(dev(tiny_ref["v"]))
    sv.build_hessian()
    sv.factor(tiny_ref["mu"])
    X = sv.apply_multipliers(dev(tiny_ref["R"])).cpu().numpy()
    check(X, tiny_ref["X"], 1e-2, 1e-2, None, "plain-form end-to-end multipliers")


def test_lambda_max(ehi, tiny_ref):
    s = tiny_ref["s"]
    sv = ehi.survey_from(s)
    sv.load_hessian(dev(tiny_ref["H"]))
    lam = sv.lambda_max()
    ref = solve.lambda_max(tiny_ref["H"])
    assert abs(lam - ref) <= 1e-9 * ref


def test_apply_source_chunks_and_zero(ehi, tiny_ref):
    # more sources than max_ns: processed in chunks; ns = 0 is a no-op
    s = tiny_ref["s"]
    sv = ehi.survey_from(s, precision="split_bf16", max_ns=3)
    sv.load_hessian(dev(tiny_ref["H"]))
    sv.factor(tiny_ref["mu"])
    X = sv.apply_multipliers(dev(tiny_ref["R"])).cpu().numpy()
    check(X, tiny_ref["X"], 2e-6, 2e-6, 4e-6, "chunked sources")
    empty = torch.zeros((s.nf, 0, s.nr), dtype=torch.complex64, device=DEV)
    sv.apply_multipliers(empty)


def test_deterministic(ehi, tiny_ref):
    s = tiny_ref["s"]
    outs = []
    for _ in range(2):
        sv = ehi.survey_from(s)
        sv.build_green(dev(tiny_ref["v"]))
        sv.build_hessian()
        sv.factor(tiny_ref["mu"])
        outs.append(sv.apply_multipliers(dev(tiny_ref["R"])).cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])


def test_error_paths(ehi, tiny_ref):
    s = tiny_ref["s"]
    sv = ehi.survey_from(s)
    with pytest.raises(ehi.EhiError) as e:
        sv.build_hessian()
    assert e.value.status == ehi.EHI_ESTATE
    with pytest.raises(ehi.EhiError) as e:
        sv.factor(1.0)
    assert e.value.status == ehi.EHI_ESTATE
    R = dev(tiny_ref["R"])
    with pytest.raises(ehi.EhiError) as e:
        sv.apply_multipliers(R)
    assert e.value.status == ehi.EHI_ESTATE
    # not positive definite: -I at frequency 2, small mu
    H = np.array(tiny_ref["H"])
    H[2] = -np.eye(s.nr)
    sv.load_hessian(dev(H))
    with pytest.raises(ehi.EhiError) as e:
        sv.factor(1e-3)
    assert e.value.status == ehi.EHI_ENOTPD and e.value.bad_freq == 2
    with pytest.raises(ehi.EhiError) as e:
        sv.apply_multipliers(R)
    assert e.value.status == ehi.EHI_ESTATE
    with pytest.raises(ehi.EhiError) as e:
        sv.factor(-1.0)
    assert e.value.status == ehi.EHI_EINVAL
    sv.load_hessian(dev(tiny_ref["H"]))
    sv.factor(tiny_ref["mu"])
    with pytest.raises(ehi.EhiError) as e:
        ehi._check(ehi.lib().ehi_apply_multipliers(sv._h, R.data_ptr(), R.data_ptr(), s.ns, None))
    assert e.value.status == ehi.EHI_EINVAL
    with pytest.raises(ValueError):
        sv.apply_multipliers(R[:, :, :3].contiguous())
    with pytest.raises(TypeError):
        sv.apply_multipliers(R.to(torch.complex128))


def test_refinement_steps(ehi, tiny_ref):
    # no refinement leaves the FP32 solve's error (~cond x 2^-24); one step
    # (the default) reaches the complex64 output's rounding, and a second one
    # changes nothing above it
    s = tiny_ref["s"]
    out = {}
    for steps in (0, 1, 2):
        sv = ehi.survey_from(s, precision="split_bf16")
        sv.load_hessian(dev(tiny_ref["H"]))
        sv.factor(tiny_ref["mu"])
        sv.set_refinement(steps)
        out[steps] = sv.apply_multipliers(dev(tiny_ref["R"])).cpu().numpy()
        sv.close()
    check(out[1], tiny_ref["X"], 1e-7, 1.5e-7, 2e-7, "one refinement step")
    check(out[2], tiny_ref["X"], 1e-7, 1.5e-7, 2e-7, "two refinement steps")
    check(out[0], tiny_ref["X"], 1e-3, 1e-3, None, "no refinement")
    sp = ehi.survey_from(s, precision="plain_fp32")
    with pytest.raises(ehi.EhiError):
        sp.set_refinement(1)
    sp.close()


@pytest.fixture(scope="module")
def many_freq_ref():
    # 4 receivers on a 48 x 64 grid, 300 steps: with 256-sample windows the
    # second window is partial (44 samples: a partial 32-sample group and a
    # partial twiddle stage); up to 64 frequencies over 2-60 Hz
    base = synth.micro(nz=48, nx=64, nb=8, nt=300, nr=4)
    v = base.velocity()
    out = {}
    for nf in (10, 20, 30, 36, 64):
        s = base.with_(freqs_hz=tuple(2.0 + 58.0 * k / (nf - 1) for k in range(nf)))
        out[nf] = (s, fd.green_dft(s, v))
    return v, out


@pytest.mark.parametrize("form", [1, 0])
@pytest.mark.parametrize("nf", [10, 20, 30, 36, 64])
def test_green_dft_row_tiles(ehi, many_freq_ref, monkeypatch, nf, form):
    # 2 nf rows of twiddles make 2, 3, 4, 6 (5 rounded up) and 8 row tiles of 16
    # in the DFT kernels: every instantiation of both forms (three-part BF16 on
    # the BF16 matrix cores, and FP32 matrix cores) against the oracle
    monkeypatch.setenv("EHI_DFT_FORM", str(form))
    v, refs = many_freq_ref
    s, ref = refs[nf]
    sv = ehi.survey_from(s, chunk=256)
    sv.build_green(dev(v))
    G = sv.copy_green_dft().reshape(s.nf, s.nr, -1).cpu().numpy()
    sv.close()
    check(G, ref, 5e-6, 5e-6, 2e-5, f"nf={nf} form {form} ghat")


@pytest.mark.parametrize("nt", [1, 2, 7, 9])
def test_green_dft_short_records(ehi, nt):
    # records shorter than one 8-level launch, or one level past it: the first
    # launch advances fewer levels than it holds, and nt = 1 is the impulse alone
    s = synth.ragged(nt=nt)
    v = s.velocity()
    sv, G = _gpu_green(ehi, s, v)
    sv.close()
    check(G, fd.green_dft(s, v), 5e-6, 5e-6, 2e-5, f"nt={nt} ghat")


def test_single_receiver_end_to_end(ehi):
    # one receiver: one 32-row block of one row in the contraction, 1 x 1
    # factors, every source's multiplier a scalar division per frequency
    s = synth.ragged(nr=1)
    v = s.velocity()
    G = fd.green_dft(s, v)
    H = hessian.hessian_r1(G)
    mu = 1e-3 * solve.lambda_max(H)
    R = s.residuals()
    X = solve.multipliers(H, mu, R.astype(np.complex128))
    sv = ehi.survey_from(s)
    sv.build_green(dev(v))
    sv.build_hessian()
    sv.factor(mu)
    Xg = sv.apply_multipliers(dev(R)).cpu().numpy()
    Hg = sv.copy_hessian().cpu().numpy()
    sv.close()
    check(Hg, H, 1e-5, 1e-5, 1e-5, "one receiver Hhat")
    check(Xg, X, 1e-5, 1e-5, 1e-5, "one receiver multipliers")
