"""Pins of the oracle's penalty, factorisation, solves and Krylov baseline (CPU)."""
import numpy as np
import pytest

import synth
from oracle import fd, hessian, krylov, solve


def _spd_batch(nf=3, nr=7, seed=0):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nf, nr, 30)) + 1j * rng.standard_normal((nf, nr, 30))
    return hessian.hessian_r1(g)


def test_cholesky_reconstructs_and_is_lower():
    H = _spd_batch()
    Q = solve.penalize(H, 0.1)
    L = solve.cholesky(Q)
    for f in range(Q.shape[0]):
        assert np.allclose(np.triu(L[f], 1), 0)
        d = np.diag(L[f])
        assert np.all(np.abs(d.imag) == 0) and np.all(d.real > 0)
        np.testing.assert_allclose(L[f] @ L[f].conj().T, Q[f], rtol=1e-13, atol=1e-13 * np.abs(Q[f]).max())


def test_solve_matches_dense_inverse():
    H = _spd_batch(seed=1)
    mu = 1e-3 * solve.lambda_max(H)
    R = synth.residuals(3, 5, 7, 9).astype(np.complex128)
    X = solve.multipliers(H, mu, R)
    for f in range(3):
        Qinv = np.linalg.inv(H[f] + mu * np.eye(7))
        ref = (Qinv @ R[f].T).T
        np.testing.assert_allclose(X[f], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_penalty_bounds_spectrum():
    H = _spd_batch(seed=2)
    mu = 0.37
    Q = solve.penalize(H, mu)
    for f in range(3):
        assert np.linalg.eigvalsh(Q[f]).min() >= mu * (1 - 1e-12)


def test_lambda_max_vs_power_iteration():
    H = _spd_batch(seed=3)
    best = 0.0
    for f in range(3):
        v = np.ones(7, dtype=complex)
        for _ in range(2000):
            v = H[f] @ v
            v /= np.linalg.norm(v)
        best = max(best, float(np.real(np.vdot(v, H[f] @ v))))
    assert abs(solve.lambda_max(H) - best) <= 1e-10 * best


@pytest.fixture(scope="module")
def micro_system():
    s = synth.micro(nz=12, nx=14, nb=3, nt=24, nr=3)
    v = s.velocity()
    op = fd.ForwardOperator(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    gt = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1).reshape(s.nr, s.nt, -1)
    Q0 = hessian.time_domain_matrix(gt, 0.0)
    mu = 1e-2 * np.linalg.eigvalsh(Q0)[-1]
    rng = np.random.default_rng(8)
    d = rng.standard_normal((s.nr, s.nt))
    return s, op, Q0, mu, d


def test_exact_solve_identity(micro_system):
    # Hessian accuracy test: at the exact solution, d - S S^T x = mu x
    s, op, Q0, mu, d = micro_system
    x = np.linalg.solve(Q0 + mu * np.eye(Q0.shape[0]), d.reshape(-1)).reshape(d.shape)
    lhs = d - op.apply(op.adjoint(x))
    np.testing.assert_allclose(lhs, mu * x, rtol=1e-9, atol=1e-10 * np.abs(d).max())


def test_cg_converges_to_dense_solve(micro_system):
    s, op, Q0, mu, d = micro_system
    x, it, solves = krylov.cg(op, d, mu, tol=1e-11, maxiter=400)
    ref = np.linalg.solve(Q0 + mu * np.eye(Q0.shape[0]), d.reshape(-1)).reshape(d.shape)
    assert solves == 2 * it
    np.testing.assert_allclose(x, ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())


def test_gmres_converges_to_dense_solve(micro_system):
    s, op, Q0, mu, d = micro_system
    ref = np.linalg.solve(Q0 + mu * np.eye(Q0.shape[0]), d.reshape(-1)).reshape(d.shape)
    x, it, solves, hist = krylov.gmres(op, d, mu, m=30, tol=1e-11, maxiter=300)
    assert solves == 2 * it
    np.testing.assert_allclose(x, ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())


def test_gmres_minimal_residual_and_exact_in_n_steps(micro_system):
    # without restarts GMRES minimises |d - Q x| over the Krylov space, so after
    # k iterations its residual is never above CG's; in n iterations it is exact
    s, op, Q0, mu, d = micro_system
    Q = Q0 + mu * np.eye(Q0.shape[0])
    b = d.reshape(-1)
    for k in (3, 8, 15):
        xg, _, _, _ = krylov.gmres(op, d, mu, m=k, tol=0.0, maxiter=k)
        xc, _, _ = krylov.cg(op, d, mu, tol=0.0, maxiter=k)
        rg = np.linalg.norm(b - Q @ xg.reshape(-1))
        rc = np.linalg.norm(b - Q @ xc.reshape(-1))
        assert rg <= rc * (1 + 1e-9), (k, rg, rc)
    # the Krylov space of a small system fills up: residual at rounding level
    small = synth.micro(nz=8, nx=9, nb=2, nt=6, nr=2)
    v = small.velocity()
    op2 = fd.ForwardOperator(v, small.nb, small.h, small.dt, small.nt, small.rec_iz, small.rec_ix, 1)
    gt = fd.green_samples(v, small.nb, small.h, small.dt, small.nt, small.rec_iz, small.rec_ix, 1)
    Q2 = hessian.time_domain_matrix(gt.reshape(small.nr, small.nt, -1), 0.1)
    d2 = np.random.default_rng(9).standard_normal((small.nr, small.nt))
    n = Q2.shape[0]
    x2, _, _, _ = krylov.gmres(op2, d2, 0.1, m=n, tol=0.0, maxiter=n)
    np.testing.assert_allclose(Q2 @ x2.reshape(-1), d2.reshape(-1), rtol=1e-8, atol=1e-9 * np.abs(d2).max())

