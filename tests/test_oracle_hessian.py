"""Pins of the oracle's Hessian forms (CPU only).

The time-domain blocks are checked against S S^T assembled from PDE solves; the
diagonal-sum structure of each block is written out independently; the literal
Fourier-diagonal algorithm is checked against the diagonal of the 2Nt-point
transform of the zero-embedded block (numpy's FFT matrix); the R1 and R2 forms
are checked against the literal algorithm; the penalty normalisation is pinned
by the transform of the embedded identity.
"""
import math

import numpy as np

import synth
from oracle import fd, hessian


def _rand_g(nr=3, nt=7, nsub=5, seed=0):
    return np.random.default_rng(seed).standard_normal((nr, nt, nsub))


def test_blocks_diagonal_sum_structure():
    # Q^{ij}[m, n] = sum_{k=0}^{min(m,n)} G^{ij}[m-k, n-k]  (structure of the block
    # equation: sums along diagonals of the outer-product matrix)
    g = _rand_g()
    Q = hessian.time_domain_blocks(g)
    nr, nt, _ = g.shape
    for i in range(nr):
        for j in range(nr):
            G = g[i] @ g[j].T
            ref = np.zeros((nt, nt))
            for m in range(nt):
                for n in range(nt):
                    ref[m, n] = sum(G[m - k, n - k] for k in range(min(m, n) + 1))
            np.testing.assert_allclose(Q[i, j], ref, rtol=1e-13, atol=1e-13)


def test_blocks_equal_explicit_s_st():
    s = synth.micro(nz=14, nx=15, nb=3, nt=24, nr=3)
    v = s.velocity()
    op = fd.ForwardOperator(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    gt = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1).reshape(3, s.nt, -1)
    Qt = hessian.time_domain_matrix(gt, 0.0)
    n = op.nr * s.nt
    SSt = np.zeros((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        SSt[:, col] = op.apply(op.adjoint(e.reshape(op.nr, s.nt))).reshape(-1)
    scale = np.abs(SSt).max()
    np.testing.assert_allclose(Qt, SSt, rtol=0, atol=1e-12 * scale)


def _dft_matrix(N):
    return np.fft.fft(np.eye(N), axis=0)      # F[k, m] = exp(-i 2 pi k m / N)


def test_alg2_literal_matches_transformed_embedding():
    g = _rand_g(nr=3, nt=7, nsub=4, seed=1)
    nr, nt, _ = g.shape
    Q = hessian.time_domain_blocks(g)
    N = 2 * nt
    F = _dft_matrix(N)
    bins = list(range(N))
    lit = hessian.alg2_literal(g, bins, use_w=True)
    for i in range(nr):
        for j in range(nr):
            E = np.zeros((N, N))
            E[:nt, :nt] = Q[i, j]
            # diagonal of the 2Nt-point representation; the sign follows xi = n - m
            ref = np.diag(F @ E @ F.conj().T) / N
            np.testing.assert_allclose(lit[:, i, j], ref, rtol=1e-12, atol=1e-12)


def test_identity_block_maps_to_one_half():
    nt = 9
    N = 2 * nt
    F = _dft_matrix(N)
    E = np.zeros((N, N))
    E[:nt, :nt] = np.eye(nt)
    d = np.diag(F @ E @ F.conj().T) / N
    np.testing.assert_allclose(d, 0.5 * np.ones(N), atol=1e-14)


def test_r1_equals_unweighted_literal():
    g = _rand_g(nr=4, nt=11, nsub=6, seed=2)
    nr, nt, _ = g.shape
    dt = 1e-3
    bins = [0, 1, 3, 8, 11]
    freqs = [k / (2 * nt * dt) for k in bins]
    ghat = fd.dft(g, freqs, dt)
    r1 = hessian.hessian_r1(ghat)
    lit = hessian.alg2_literal(g, bins, use_w=False)
    np.testing.assert_allclose(r1, 2 * nt * lit, rtol=1e-12, atol=1e-12 * np.abs(r1).max())


def test_r2_equals_weighted_literal():
    g = _rand_g(nr=4, nt=11, nsub=6, seed=3)
    nr, nt, _ = g.shape
    dt = 1e-3
    bins = [0, 2, 5, 10]
    freqs = [k / (2 * nt * dt) for k in bins]
    r2 = hessian.hessian_r2(g, freqs, dt)
    lit = hessian.alg2_literal(g, bins, use_w=True)
    np.testing.assert_allclose(r2, 2 * lit, rtol=1e-12, atol=1e-12 * np.abs(r2).max())


def test_weighting_function_values():
    W = hessian.weighting(4)
    ref = np.array([[4, 3, 2, 1], [3, 3, 2, 1], [2, 2, 2, 1], [1, 1, 1, 1]], dtype=float)
    np.testing.assert_array_equal(W, ref)


def test_r1_hermitian_positive_semidefinite():
    rng = np.random.default_rng(4)
    ghat = rng.standard_normal((3, 6, 40)) + 1j * rng.standard_normal((3, 6, 40))
    H = hessian.hessian_r1(ghat)
    for f in range(3):
        np.testing.assert_allclose(H[f], H[f].conj().T, rtol=0, atol=1e-13 * np.abs(H[f]).max())
        assert np.linalg.eigvalsh(H[f]).min() > -1e-12 * np.abs(H[f]).max()


def test_block_diagonal_after_permutation():
    # Fig. 1 structure (Nt = 7, Nr = 5): with the Fourier diagonal of every block
    # kept, reordering frequency-major gives one Nr x Nr block per frequency.
    rng = np.random.default_rng(6)
    nr, nt = 5, 7
    N = 2 * nt
    qhat = rng.standard_normal((N, nr, nr)) + 1j * rng.standard_normal((N, nr, nr))
    big = np.zeros((nr * N, nr * N), dtype=complex)   # receiver-major, blocks diagonal
    for i in range(nr):
        for j in range(nr):
            big[i * N:(i + 1) * N, j * N:(j + 1) * N] = np.diag(qhat[:, i, j])
    perm = np.array([i * N + k for k in range(N) for i in range(nr)])
    P = big[np.ix_(perm, perm)]
    for k in range(N):
        blk = P[k * nr:(k + 1) * nr, k * nr:(k + 1) * nr]
        np.testing.assert_array_equal(blk, qhat[k])
        off = P[k * nr:(k + 1) * nr].copy()
        off[:, k * nr:(k + 1) * nr] = 0
        assert not off.any()


def test_dct_matrix_is_the_definition_and_orthonormal():
    # against scipy's orthonormal DCT-II of the identity (an independent routine)
    import scipy.fft
    for n in (1, 5, 16, 33):
        D = hessian.dct_matrix(n, n)
        ref = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
        np.testing.assert_allclose(D, ref, atol=1e-13)
        np.testing.assert_allclose(D @ D.T, np.eye(n), atol=1e-13)


def test_compression_exact_with_all_coefficients_and_converges():
    rng = np.random.default_rng(4)
    nf, nr, nzs, nxs = 2, 5, 9, 12
    # smooth fields (decaying spectrum) plus a little noise
    z = np.arange(nzs)[:, None] / nzs
    x = np.arange(nxs)[None, :] / nxs
    g = np.empty((nf, nr, nzs * nxs), dtype=np.complex128)
    for f in range(nf):
        for r in range(nr):
            a, b = rng.uniform(0.5, 2.0, 2)
            field = np.exp(-((z - 0.3 * a) ** 2 + (x - 0.2 * b) ** 2) * 8) * np.exp(1j * (a * z + b * x))
            g[f, r] = (field + 1e-3 * rng.standard_normal((nzs, nxs))).ravel()
    full = hessian.hessian_r1(g)
    np.testing.assert_allclose(hessian.hessian_compressed(g, nzs, nxs, nzs, nxs), full, rtol=1e-12, atol=1e-12)
    errs = [np.linalg.norm(hessian.hessian_compressed(g, nzs, nxs, k, k + 3) - full) / np.linalg.norm(full)
            for k in (2, 4, 6, 8)]
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    # Parseval: the kept energy never exceeds the full energy (diagonal of H)
    for k in (2, 5):
        c = hessian.hessian_compressed(g, nzs, nxs, k, k)
        assert np.all(np.diagonal(c, axis1=1, axis2=2).real <= np.diagonal(full, axis1=1, axis2=2).real + 1e-12)


# ---------------------------------------------------------------------------
# time-axis resampling before the finite-record Hessian
# ---------------------------------------------------------------------------

def _response(h, dt, nfft=1 << 16):
    # H(f) of the zero-phase taps h_{-K..K}, evaluated with numpy's FFT
    K = (len(h) - 1) // 2
    x = np.zeros(nfft)
    x[:K + 1] = h[K:]
    x[nfft - K:] = h[:K]
    return np.fft.fftfreq(nfft, dt), np.fft.fft(x)


def test_decimation_filter_response():
    # passband (|f| <= f_max) within 5e-6 of one, stopband (|f| >= fs/D - f_max,
    # everything that folds onto the passband) below 5e-6 (the 120 dB design)
    dt, fmax = 0.8e-3, 15.0
    for D in (2, 5, 10, 16):
        h = hessian.decimation_filter(D, dt, fmax)
        assert np.allclose(h, h[::-1]) and abs(h.sum() - 1.0) < 1e-12
        f, H = _response(h, dt)
        fs = 1.0 / dt
        assert np.abs(H[np.abs(f) <= fmax] - 1.0).max() < 5e-6, D
        assert np.abs(H[np.abs(f) >= fs / D - fmax]).max() < 5e-6, D
    assert np.array_equal(hessian.decimation_filter(1, dt, fmax), np.ones(1))


def test_decimate_matches_convolution():
    rng = np.random.default_rng(11)
    g = rng.standard_normal((2, 137, 3))
    D = 5
    h = hessian.decimation_filter(D, 1e-3, 20.0)
    K = (len(h) - 1) // 2
    y = hessian.decimate(g, D, h)
    n, qa, qb = hessian.decimation_times(137, D, K)
    for r in range(2):
        for x in range(3):
            full = np.convolve(g[r, :, x], h)            # full[i] = sum h[k] g[i - k], g index 0 = n 1
            # y_q = sum_j h_j g(n_q + j) = full[n_q - 1 + K]  (h symmetric)
            idx = n - 1 + K
            ok = (idx >= 0) & (idx < len(full))
            ref = np.where(ok, full[np.clip(idx, 0, len(full) - 1)], 0.0)
            np.testing.assert_allclose(y[r, :, x], ref, rtol=1e-12, atol=1e-14)
    assert n[qa] >= 1 and n[qb] <= 137 and (qa == 0 or n[qa - 1] < 1) and (qb == len(n) - 1 or n[qb + 1] > 137)
    assert n[0] + K <= 1 + D - 1 and n[-1] - K <= 137      # every kept sample whose support meets the record


def test_decimated_transform_matches_the_whole_record():
    # (D / H(w)) sum_q y_q exp(-i w n_q dt) equals the DFT of the whole record
    # up to the stopband's folding (5e-6 of the aliased content)
    s = synth.micro(nz=30, nx=36, nb=6, nt=400, nr=2)
    gt = fd.green_samples(s.velocity(), s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1).reshape(2, s.nt, -1)
    G = fd.dft(gt, s.freqs_hz, s.dt)
    for D in (2, 10):
        h = hessian.decimation_filter(D, s.dt, max(s.freqs_hz))
        K = (len(h) - 1) // 2
        y = hessian.decimate(gt, D, h)
        n, _, _ = hessian.decimation_times(s.nt, D, K)
        for f, fr in enumerate(s.freqs_hz):
            w = 2 * math.pi * fr
            Hw = np.real(np.sum(h * np.exp(-1j * w * np.arange(-K, K + 1) * s.dt)))
            Gd = (D / Hw) * np.einsum("q,rqx->rx", np.exp(-1j * w * n * s.dt), y)
            assert np.linalg.norm(Gd - G[f]) <= 1e-6 * np.linalg.norm(G[f]), (D, f)


def test_decimated_hessian_reduces_to_r2():
    g = _rand_g(nr=3, nt=40, nsub=6, seed=4)
    freqs = (3.0, 7.0, 11.0)
    a = hessian.hessian_r2_decimated(g, freqs, 1e-3, 1)
    b = hessian.hessian_r2(g, freqs, 1e-3)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())
    # on a Green-function record, keeping every 5th sample changes the
    # time average by the resampling's approximation only (recorded: ~5e-3)
    s = synth.micro(nz=30, nx=36, nb=6, nt=400, nr=3)
    gt = fd.green_samples(s.velocity(), s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1).reshape(3, s.nt, -1)
    full = hessian.hessian_r2(gt, s.freqs_hz, s.dt)
    dec = hessian.hessian_r2_decimated(gt, s.freqs_hz, s.dt, 5)
    err = max(np.linalg.norm(dec[f] - full[f]) / np.linalg.norm(full[f]) for f in range(len(s.freqs_hz)))
    print("decimated (D = 5) vs whole-record finite-record Hessian", err)
    assert err < 5e-2
    for f in range(len(s.freqs_hz)):
        np.testing.assert_allclose(dec[f], dec[f].conj().T, atol=1e-12 * np.abs(dec[f]).max())
