"""Oracle: the steps either side of the deblur and the Hessian accuracy test (FP64).

Test infrastructure only (see the package docstring).

What is computed, and where the paper defines it:

* Residual spectra in (frequency-domain inversion: the data residuals are
  carried to the frequency domain by a transform of length 2 Nt, so that the
  correlation with the Green functions does not wrap around):
      R_s(w, r) = sum_{n=1}^{nt} dd_s(r, n) exp(-i w n dt),
  the same sign and sample origin as the Green-function spectra.  At the bins
  w_k = 2 pi k / (2 nt dt) this is bin k of the 2nt-point DFT of the record
  placed at positions 1..nt of a zero-padded sequence.
* Multipliers out: the inverse 2nt-point transform, cropped to samples
  1..nt.  The records are real, so only bins k = 0..nt are carried (the others
  are their conjugates); bins that were not computed count as zero:
      x(n) = (1 / 2nt) [X_0 + (-1)^n X_nt + 2 Re sum_{0<k<nt} X_k exp(+i w_k n dt)].
* Hessian accuracy test (numerical examples, Hessian accuracy test): the
  multipliers dd^e are back-propagated as adjoint sources, db = S^T dd^e, the
  extended source predicts the data change S db, and
      RelErr = ||d - P u^e||^2 / ||d||^2,   d - P u^e = dd - S S^T dd^e
  (with dd = d - S b, so P u^e = S b + S db).  An exact solve of
  Q dd^e = dd with Q = S S^T + mu I gives d - P u^e = mu dd^e.

Pins (tests/test_oracle_timefreq.py): the forward transform against numpy's
FFT of the zero-padded record at every bin, the inverse against numpy's
inverse FFT, the round trip over all bins, the frequency-domain Hessian
product against a brute-force time-domain correlation sum, the frequency
solve's identity over the whole 2nt period (dd - correlation product = mu x),
and the accuracy test's PDE prediction against the explicit Toeplitz-block
Hessian.
"""
from __future__ import annotations

import math

import numpy as np


def bins(freqs_hz, nt: int, dt: float) -> np.ndarray:
    """Bin index k of each frequency on the 2nt-point grid (k = f 2 nt dt);
    raises ValueError if a frequency is not a bin in 0..nt."""
    k = np.asarray(freqs_hz, dtype=np.float64) * 2.0 * nt * dt
    kr = np.rint(k)
    if np.any(np.abs(k - kr) > 1e-6) or np.any(kr < 0) or np.any(kr > nt):
        raise ValueError("frequencies are not bins 0..nt of the 2nt-point transform")
    return kr.astype(np.int64)


def bin_freqs(k, nt: int, dt: float) -> np.ndarray:
    """Frequencies (Hz) of bins k of the 2nt-point grid."""
    return np.asarray(k, dtype=np.float64) / (2.0 * nt * dt)


def residual_spectra(dd: np.ndarray, freqs_hz, dt: float) -> np.ndarray:
    """R[f][s][r] = sum_{n=1}^{nt} dd[s][r][n-1] exp(-i w_f n dt).

    ``dd`` is real ``[ns][nr][nt]``; returns complex128 ``[nf][ns][nr]``.
    Twiddles in FP64, the sum as a matrix product over n.
    """
    dd = np.asarray(dd, dtype=np.float64)
    ns, nr, nt = dd.shape
    n = np.arange(1, nt + 1, dtype=np.float64)
    w = 2.0 * math.pi * np.asarray(freqs_hz, dtype=np.float64)
    tw = np.exp(-1j * np.outer(w, n) * dt)                # [nf][nt]
    flat = dd.reshape(ns * nr, nt)
    return (flat @ tw.T).T.reshape(len(w), ns, nr)


def to_time(X: np.ndarray, freqs_hz, dt: float, nt: int) -> np.ndarray:
    """Inverse 2nt-point transform of the bins held in ``X`` (complex
    ``[nf][ns][nr]``, frequencies that must be bins 0..nt, each at most once),
    cropped to samples 1..nt: real ``[ns][nr][nt]``."""
    k = bins(freqs_hz, nt, dt)
    if len(set(k.tolist())) != len(k):
        raise ValueError("a bin occurs twice")
    X = np.asarray(X, dtype=np.complex128)
    n = np.arange(1, nt + 1, dtype=np.float64)
    w = 2.0 * math.pi * bin_freqs(k, nt, dt)
    c = np.where((k == 0) | (k == nt), 1.0, 2.0) / (2.0 * nt)   # weight of each bin
    e = np.exp(1j * np.outer(w, n) * dt) * c[:, None]           # [nf][nt]
    nf, ns, nr = X.shape
    out = np.einsum("fn,fq->qn", e, X.reshape(nf, ns * nr)).real
    return out.reshape(ns, nr, nt)


def correlation_product(gt: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Brute-force time-domain counterpart of to_time(Hhat X) at full band:
    y_i(n) = sum_j sum_x' sum_{l1, l2 = 1..nt} g_i(l1, x') g_j(l2, x') x_j(m),
    m = n - l1 + l2 modulo 2nt, for output samples n = 1..nt.

    ``gt``: Green-function samples ``[nr][nt][nsub]`` (g(l) at index l - 1);
    ``x``: ``[nr][nt]`` (samples 1..nt, zero elsewhere in the period) or
    ``[nr][2nt]`` (a whole period, positions 0..2nt-1).  Returns ``[nr][nt]``.
    Small sizes only.
    """
    nr, nt, _ = gt.shape
    P = 2 * nt
    if x.shape[1] == nt:
        xp = np.zeros((nr, P))
        xp[:, 1:nt + 1] = x
    elif x.shape[1] == P:
        xp = np.asarray(x)
    else:
        raise ValueError("x must hold nt or 2nt samples per receiver")
    # c_ij(lag) = sum_x' sum_{l1 - l2 = lag} g_i(l1) g_j(l2), lag in -(nt-1)..nt-1
    c = np.zeros((nr, nr, P))
    for l1 in range(1, nt + 1):
        for l2 in range(1, nt + 1):
            c[:, :, (l1 - l2) % P] += gt[:, l1 - 1, :] @ gt[:, l2 - 1, :].T
    y = np.zeros((nr, nt))
    for n in range(1, nt + 1):
        for m in range(P):
            y[:, n - 1] += c[:, :, (n - m) % P] @ xp[:, m]
    return y


def accuracy_test(op, H: np.ndarray, mu: float, dd: np.ndarray, d_obs: np.ndarray,
                  freqs_hz, dt: float):
    """The Hessian accuracy test with the frequency-domain direct inversion.

    ``op``: an ``fd.ForwardOperator`` (S on the subgrid sources); ``H``: Hhat
    ``[nf][nr][nr]`` at the bins ``freqs_hz``; ``dd``: residuals
    ``[ns][nr][nt]``; ``d_obs``: observed data of the same shape (the
    normaliser).  Returns (dde, db, pred, err, relerr): the time-domain
    multipliers, the back-propagated source ``[ns][nt][nsub]``, the predicted
    change S db, the misfit dd - S db and RelErr per source.
    """
    from . import solve
    ns, nr, nt = dd.shape
    R = residual_spectra(dd, freqs_hz, dt)
    X = solve.multipliers(H, mu, R)
    dde = to_time(X, freqs_hz, dt, nt)
    db = np.stack([op.adjoint(dde[s]) for s in range(ns)])
    pred = np.stack([op.apply(db[s]) for s in range(ns)])
    err = dd - pred
    relerr = np.array([np.sum(err[s] ** 2) / np.sum(np.asarray(d_obs[s], dtype=np.float64) ** 2)
                       for s in range(ns)])
    return dde, db, pred, err, relerr
