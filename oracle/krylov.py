"""Oracle: the paper's iterative baseline, CG on the time-domain system (FP64).

Test infrastructure only (see the package docstring).

Solves Q delta d^e = delta d with Q = S S^T + mu I (Theory: the deblurring
system and the Hessian definition) by conjugate gradients, applying Q through
one adjoint and one forward PDE solve per iteration (Introduction: iterative
methods need two PDE solves per inner iteration per source; Hessian accuracy
test: CG with two PDE solves per iteration).

Pins (tests/test_oracle_krylov.py): convergence to the dense solve of the
explicit time-domain Q on a micro grid, and the exact-solve identity
d - S S^T x = mu x.
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
