"""Oracle: penalty, factorisation and the per-frequency multi-source solve (FP64).

Test infrastructure only (see the package docstring).

* ``penalize``: Qhat(w) = Hhat(w) + mu I (the Hessian definition Q = S S^T + mu I,
  mapped to each frequency block of the block-diagonal system).
* ``cholesky``: Qhat(w) = L(w) L(w)^H with L lower triangular and a real
  positive diagonal.  The paper inverts each Qhat(w) and stores the inverse
  (frequency-domain inversion; last step of its Fourier block-diagonal Hessian
  algorithm); a Cholesky factorisation gives the same solves and is used instead.
* ``solve``: delta d^e(w) = Qhat(w)^{-1} delta d(w) for every source at once
  (frequency-domain inversion: one Nr x Nr system per frequency).
* ``mu_from_eps``: mu = eps * max_w lambda_max(Hhat(w)) (numerical examples: mu
  is chosen as a fraction 1e-2..1e-4 of the largest eigenvalue of S S^T).

Pins (tests/test_oracle_solve.py): the factor against numpy's eigenvalues and
L L^H reconstruction; the solve against the explicit dense inverse; the
identity d - S S^T x = mu x at the exact solution (Hessian accuracy test).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def penalize(H: np.ndarray, mu: float) -> np.ndarray:
    """Qhat = Hhat + mu I for every frequency (``[nf][nr][nr]``)."""
    H = np.asarray(H, dtype=np.complex128)
    nr = H.shape[-1]
    return H + mu * np.eye(nr)[None]


def cholesky(Q: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor per frequency; raises LinAlgError if not HPD."""
    Q = np.asarray(Q, dtype=np.complex128)
    return np.stack([sla.cholesky(Q[f], lower=True) for f in range(Q.shape[0])])


def solve(L: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X(w) = (L L^H)^{-1} R(w); ``R`` is ``[nf][ns][nr]`` (one row per source).

    Forward substitution with L, then back substitution with L^H.
    """
    R = np.asarray(R, dtype=np.complex128)
    X = np.empty_like(R)
    for f in range(R.shape[0]):
        y = sla.solve_triangular(L[f], R[f].T, lower=True)
        X[f] = sla.solve_triangular(L[f].conj().T, y, lower=False).T
    return X


def lambda_max(H: np.ndarray) -> float:
    """max over frequencies of the largest eigenvalue of Hhat(w)."""
    H = np.asarray(H, dtype=np.complex128)
    return float(max(np.linalg.eigvalsh(H[f])[-1] for f in range(H.shape[0])))


def mu_from_eps(H: np.ndarray, eps: float = 1e-3) -> float:
    return eps * lambda_max(H)


def multipliers(H: np.ndarray, mu: float, R: np.ndarray) -> np.ndarray:
    """End to end from the Hessian: penalty, factor, solve."""
    return solve(cholesky(penalize(H, mu)), R)
