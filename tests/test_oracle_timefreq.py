"""Pins of the oracle's time/frequency transfer and the accuracy test (CPU only).

The forward and inverse 2nt-point transforms are checked against numpy's FFT
of the zero-padded record; the frequency-domain Hessian product, carried back
to time, against a brute-force correlation sum over the Green functions; the
accuracy test's PDE product against the explicit Toeplitz-block Hessian.
"""
import numpy as np
import pytest

import synth
from oracle import fd, hessian, solve, timefreq


def _padded_fft(x):
    """FFT of length 2nt with sample n (1..nt) at position n."""
    nt = x.shape[-1]
    z = np.zeros(x.shape[:-1] + (2 * nt,))
    z[..., 1:nt + 1] = x
    return np.fft.fft(z, axis=-1)


def test_residual_spectra_match_padded_fft_at_bins():
    rng = np.random.default_rng(0)
    nt, dt = 37, 2e-3
    dd = rng.standard_normal((2, 3, nt))
    k = np.arange(nt + 1)
    R = timefreq.residual_spectra(dd, timefreq.bin_freqs(k, nt, dt), dt)
    ref = _padded_fft(dd)[..., k]                     # [ns][nr][nf]
    np.testing.assert_allclose(R, ref.transpose(2, 0, 1), rtol=1e-12, atol=1e-12)


def test_to_time_matches_inverse_fft():
    rng = np.random.default_rng(1)
    nt, dt = 40, 1e-3
    k = np.array([0, 3, 4, 11, 39, 40])
    X = rng.standard_normal((len(k), 2, 3)) + 1j * rng.standard_normal((len(k), 2, 3))
    X[k == 0] = X[k == 0].real                        # bins of a real record
    X[k == nt] = X[k == nt].real
    x = timefreq.to_time(X, timefreq.bin_freqs(k, nt, dt), dt, nt)
    F = np.zeros((2, 3, 2 * nt), dtype=complex)
    for b, kk in enumerate(k):
        F[..., kk] = X[b]
        if 0 < kk < nt:
            F[..., 2 * nt - kk] = np.conj(X[b])
    ref = np.fft.ifft(F, axis=-1)
    assert np.abs(ref.imag).max() < 1e-12
    np.testing.assert_allclose(x, ref.real[..., 1:nt + 1], rtol=1e-12, atol=1e-13)


def test_round_trip_over_all_bins():
    rng = np.random.default_rng(2)
    nt, dt = 29, 4e-3
    dd = rng.standard_normal((3, 2, nt))
    f = timefreq.bin_freqs(np.arange(nt + 1), nt, dt)
    back = timefreq.to_time(timefreq.residual_spectra(dd, f, dt), f, dt, nt)
    np.testing.assert_allclose(back, dd, rtol=1e-12, atol=1e-12)


def test_bins_rejects_off_grid_and_repeats():
    with pytest.raises(ValueError):
        timefreq.bins([3.0], 100, 1e-3)               # 0.6 of a bin
    with pytest.raises(ValueError):
        timefreq.bins([timefreq.bin_freqs(101, 100, 1e-3)], 100, 1e-3)
    f = timefreq.bin_freqs([5, 5], 100, 1e-3)
    with pytest.raises(ValueError):
        timefreq.to_time(np.zeros((2, 1, 1), complex), f, 1e-3, 100)


@pytest.fixture(scope="module")
def micro():
    s = synth.micro(nz=12, nx=14, nb=3, nt=24, nr=3)
    v = s.velocity()
    gt = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1).reshape(s.nr, s.nt, -1)
    f = timefreq.bin_freqs(np.arange(s.nt + 1), s.nt, s.dt)
    H = hessian.hessian_r1(fd.dft(gt, f, s.dt))
    op = fd.ForwardOperator(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    return s, gt, f, H, op


def test_frequency_hessian_product_is_circular_correlation(micro):
    s, gt, f, H, _ = micro
    x = np.random.default_rng(3).standard_normal((s.nr, s.nt))
    R = timefreq.residual_spectra(x[None], f, s.dt)           # [nf][1][nr]
    HX = np.einsum("fij,fsj->fsi", H, R)
    y = timefreq.to_time(HX, f, s.dt, s.nt)[0]
    ref = timefreq.correlation_product(gt, x)
    np.testing.assert_allclose(y, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_frequency_solve_identity_in_time(micro):
    # frequency by frequency (Hhat + mu) X = R, so over the whole 2nt period
    # dd - (circular correlation product of x) = mu x, x the inverse of X; the
    # cropped multipliers dd^e are x on samples 1..nt
    s, gt, f, H, _ = micro
    nt = s.nt
    dd = np.random.default_rng(4).standard_normal((1, s.nr, nt))
    mu = 1e-2 * solve.lambda_max(H)
    X = solve.multipliers(H, mu, timefreq.residual_spectra(dd, f, s.dt))[:, 0]   # [nf][nr]
    F = np.zeros((s.nr, 2 * nt), dtype=complex)                                # bins 0..nt present
    F[:, :nt + 1] = X.T
    F[:, nt + 1:] = np.conj(X.T[:, 1:nt][:, ::-1])
    x = np.fft.ifft(F, axis=-1)
    assert np.abs(x.imag).max() < 1e-12 * np.abs(x.real).max()
    x = x.real
    np.testing.assert_allclose(timefreq.to_time(X[:, None], f, s.dt, nt)[0], x[:, 1:nt + 1],
                               rtol=1e-10, atol=1e-13)
    lhs = dd[0] - timefreq.correlation_product(gt, x)
    np.testing.assert_allclose(lhs, mu * x[:, 1:nt + 1], rtol=1e-9, atol=1e-11 * np.abs(dd).max())


def test_accuracy_test_prediction_is_toeplitz_hessian_product(micro):
    s, gt, f, H, op = micro
    rng = np.random.default_rng(5)
    dd = rng.standard_normal((2, s.nr, s.nt))
    d_obs = dd + rng.standard_normal(dd.shape)
    mu = 1e-2 * solve.lambda_max(H)
    dde, db, pred, err, relerr = timefreq.accuracy_test(op, H, mu, dd, d_obs, f, s.dt)
    Q0 = hessian.time_domain_matrix(gt, 0.0)                   # receiver-major vec
    for k in range(2):
        ref = (Q0 @ dde[k].reshape(-1)).reshape(s.nr, s.nt)
        np.testing.assert_allclose(pred[k], ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())
        assert relerr[k] == pytest.approx(np.sum((dd[k] - ref) ** 2) / np.sum(d_obs[k] ** 2), rel=1e-9)
    assert db.shape == (2, s.nt, s.nsub)
