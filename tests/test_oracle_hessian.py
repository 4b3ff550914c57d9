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
