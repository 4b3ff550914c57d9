"""Oracle: the paper's iterative baseline, CG on the time-domain system (FP64).

Test infrastructure only (see the package docstring).

Solves Q delta d^e = delta d with Q = S S^T + mu I (Theory: the deblurring
system and the Hessian definition) by conjugate gradients, applying Q through
one adjoint and one forward PDE solve per iteration (Introduction: iterative
methods need two PDE solves per inner iteration per source; Hessian accuracy
test: CG with two PDE solves per iteration).

GMRES (the paper's second iterative baseline, also two PDE solves per
iteration): restarted GMRES(m) on the same system, Arnoldi with modified
Gram-Schmidt, the least-squares problem of the Hessenberg matrix solved with
Givens rotations (Saad and Schultz's algorithm, written out from its
definition).

Pins (tests/test_oracle_solve.py): convergence to the dense solve of the
explicit time-domain Q on a micro grid, the exact-solve identity
d - S S^T x = mu x, GMRES's minimal residual over the Krylov space (never
above CG's after the same number of iterations), and its exact solution in
n iterations.
"""
from __future__ import annotations

import numpy as np


def apply_q(op, x: np.ndarray, mu: float) -> np.ndarray:
    """Q x = S (S^T x) + mu x for data x ``[nr][nt]`` (two PDE solves)."""
    return op.apply(op.adjoint(x)) + mu * x


def cg(op, d: np.ndarray, mu: float, tol: float = 1e-10, maxiter: int = 500):
    """Conjugate gradients on Q x = d.  Returns (x, iterations, pde_solves)."""
    d = np.asarray(d, dtype=np.float64)
    x = np.zeros_like(d)
    r = d.copy()
    p = r.copy()
    rr = float(np.vdot(r, r))
    d_norm = float(np.sqrt(np.vdot(d, d)))
    it = 0
    solves = 0
    while it < maxiter and np.sqrt(rr) > tol * d_norm:
        Ap = apply_q(op, p, mu)
        solves += 2
        alpha = rr / float(np.vdot(p, Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, solves


def gmres(op, d: np.ndarray, mu: float, m: int = 50, tol: float = 1e-10, maxiter: int = 500):
    """Restarted GMRES(m) on Q x = d.  Returns (x, iterations, pde_solves,
    residual norms after every iteration, relative to |d|)."""
    d = np.asarray(d, dtype=np.float64)
    shape = d.shape
    b = d.reshape(-1)
    x = np.zeros_like(b)
    bn = float(np.linalg.norm(b))
    hist = []
    it = 0
    while it < maxiter:
        r = b - apply_q(op, x.reshape(shape), mu).reshape(-1) if it else b.copy()
        beta = float(np.linalg.norm(r))
        if beta <= tol * bn:
            break
        k = min(m, maxiter - it)
        V = np.zeros((k + 1, b.size))
        H = np.zeros((k + 1, k))
        V[0] = r / beta
        g = np.zeros(k + 1)
        g[0] = beta
        cs, sn = np.zeros(k), np.zeros(k)
        j_done = 0
        for j in range(k):
            w = apply_q(op, V[j].reshape(shape), mu).reshape(-1)
            it += 1
            for i in range(j + 1):                     # modified Gram-Schmidt
                H[i, j] = float(np.dot(V[i], w))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                         # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            hist.append(abs(g[j + 1]) / bn)
            j_done = j + 1
            if abs(g[j + 1]) <= tol * bn:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + V[:j_done].T @ y
        if hist and hist[-1] <= tol:
            break
    return x.reshape(shape), it, 2 * it, hist

