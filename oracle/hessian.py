"""Oracle: the data-space Hessian in time and frequency (FP64).

Test infrastructure only (see the package docstring).

Forms computed here (all for one survey; receivers i, j; grid points x):

* ``time_domain_blocks``: block (i, j) of Q without the penalty, as the sum over
  x of products of lower-triangular Toeplitz matrices built from the Green
  functions (Direct Hessian-inverse computation, block equation of the
  Hessian).  Brute force, micro grids only.
* ``alg2_literal``: the Fourier block-diagonal approximation exactly in the
  order of the paper's algorithm for the Fourier block-diagonal Hessian:
  weighting function W(m, n) = min(Nt - m, Nt - n); for i and j >= i form
  G^{ij} = sum_x g^i g^{jT}; sum W o G^{ij} along descending diagonals into
  q^{ij}_xi, xi = n - m; 2Nt-length transform with the paper's normalisation
  qhat_k = (1/2Nt) sum_xi q_xi exp(+i 2 pi k xi / 2Nt); Hermitian fill.  Only on
  frequencies that are bins of the 2Nt-point transform.
* ``hessian_r1``: Hhat(w) = Ghat(w) Ghat(w)^H, Ghat the final DFT of each Green
  function.  This is the algorithm with W replaced by a constant (the long-record
  Toeplitz limit the paper invokes when it lets t grow), written with the
  transfer-function normalisation (no 1/2Nt, and W = 1): Hhat = 2Nt qhat|_{W=1}.
* ``hessian_compressed``: Ĝ Ψᵀ (Ĝ Ψᵀ)ᴴ with Ψ the leading rows of the
  orthonormal 2D DCT-II of the subgrid (the spatial compression the discussion
  proposes); every coefficient kept gives ``hessian_r1`` exactly.
* ``hessian_r2``: the finite-record weighting kept exactly, evaluated without
  the 2Nt transform as the time average of running-DFT Gram matrices:
  Hhat_W(w) = (1/Nt) sum_{p=1}^{Nt} Ghat_p(w) Ghat_p(w)^H with Ghat_p the DFT
  truncated after sample p.  Equals 2 qhat of the literal algorithm with W.
* ``hessian_r2_decimated``: the same time average on the record resampled in
  time (the numerical examples resample the Green functions and data to the
  Nyquist rate before forming the Hessian): every D-th sample of the record
  low-pass filtered by ``decimation_filter``, the running spectra taken at the
  kept samples and corrected by D / H(w), the Gram average over the kept
  samples that fall inside the record, each weighted D / Nt.

Pins (tests/test_oracle_hessian.py): the decimation filter's response
(numpy FFT of the taps) in the passband and the stopband, the decimated record
against numpy's convolution, the decimated transform against the DFT of the
whole record, and the decimated Hessian at D = 1 against ``hessian_r2``; the
Toeplitz blocks against S S^T built
column by column from PDE solves; the diagonal-sum structure of Q; the literal
algorithm against the diagonal of the 2Nt-point transform of the zero-embedded
brute-force Q (computed with numpy's FFT); R1 and R2 against the literal
algorithm (W = 1 and W as defined); Hermitian positive-definiteness.
"""
from __future__ import annotations

import math

import numpy as np


def toeplitz_lower(v: np.ndarray) -> np.ndarray:
    """T(v): lower-triangular Toeplitz matrix with first column v."""
    n = len(v)
    T = np.zeros((n, n))
    for k in range(n):
        T[k:, k] = v[: n - k]
    return T


def time_domain_blocks(gt: np.ndarray) -> np.ndarray:
    """Q^{ij} = sum_x T(g^i(:, x)) T(g^j(:, x))^T for all i, j.

    ``gt`` holds time samples ``[nr][nt][nsub]``.  Returns ``[nr][nr][nt][nt]``
    (the penalty is not included).  Cost O(nr^2 nsub nt^3): micro sizes only.
    """
    nr, nt, nsub = gt.shape
    T = np.zeros((nr, nsub, nt, nt))
    for i in range(nr):
        for x in range(nsub):
            T[i, x] = toeplitz_lower(gt[i, :, x])
    Q = np.zeros((nr, nr, nt, nt))
    for i in range(nr):
        for j in range(nr):
            Q[i, j] = np.einsum("xab,xcb->ac", T[i], T[j])
    return Q


def time_domain_matrix(gt: np.ndarray, mu: float) -> np.ndarray:
    """The full (nr nt) x (nr nt) Hessian Q = S S^T + mu I, receiver-major
    (vec of the Nt x Nr gather stacks one receiver's trace after another)."""
    nr, nt, _ = gt.shape
    B = time_domain_blocks(gt)
    Q = B.transpose(0, 2, 1, 3).reshape(nr * nt, nr * nt)
    return Q + mu * np.eye(nr * nt)


def weighting(nt: int) -> np.ndarray:
    """W(m, n) = min(Nt - m, Nt - n), m, n = 0..Nt-1 (weighting function)."""
    m = np.arange(nt)
    return np.minimum(nt - m[:, None], nt - m[None, :]).astype(np.float64)


def alg2_literal(gt: np.ndarray, bins, use_w: bool = True) -> np.ndarray:
    """The Fourier block-diagonal Hessian, step by step as the paper's algorithm.

    ``gt``: time samples ``[nr][Nt][nsub]`` (vector index m = 0..Nt-1 holds the
    sample after m+1 steps).  ``bins``: indices k of the 2Nt-point transform.
    Returns qhat ``[len(bins)][nr][nr]`` complex (paper normalisation, no
    penalty).  ``use_w=False`` replaces W by ones.
    """
    nr, nt, _ = gt.shape
    W = weighting(nt) if use_w else np.ones((nt, nt))
    L = 2 * nt
    out = np.zeros((len(bins), nr, nr), dtype=np.complex128)
    for i in range(nr):
        for j in range(i, nr):
            Gij = gt[i] @ gt[j].T                       # [m][n] = sum_x g^i(m,x) g^j(n,x)
            WG = W * Gij
            q = np.zeros(L)                             # q[xi mod 2Nt], xi = n - m
            for xi in range(-nt + 1, nt):
                q[xi % L] = np.trace(WG, offset=xi)     # entries (m, m + xi)
            # qhat_k = (1/2Nt) sum_xi q_xi exp(+i 2 pi k xi / 2Nt)
            spec = np.fft.ifft(q)                       # = (1/L) sum q e^{+i2pi k xi/L}
            for b, k in enumerate(bins):
                out[b, i, j] = spec[k]
                out[b, j, i] = np.conj(spec[k])
    return out


def hessian_r1(ghat: np.ndarray) -> np.ndarray:
    """Hhat(w)[i][j] = sum_x ghat_i(w, x) conj(ghat_j(w, x)); ``ghat`` is
    ``[nf][nr][nsub]`` complex.  Returns ``[nf][nr][nr]`` complex128."""
    g = np.asarray(ghat, dtype=np.complex128)
    return np.stack([g[f] @ g[f].conj().T for f in range(g.shape[0])])


def dct_matrix(n: int, keep: int) -> np.ndarray:
    """Leading ``keep`` rows of the orthonormal DCT-II matrix of size n:
    D[k][m] = s_k cos(pi k (2m + 1) / (2n)), s_0 = sqrt(1/n), s_k = sqrt(2/n)."""
    k = np.arange(keep)[:, None]
    m = np.arange(n)[None, :]
    s = np.where(k == 0, math.sqrt(1.0 / n), math.sqrt(2.0 / n))
    return s * np.cos(math.pi * k * (2 * m + 1) / (2.0 * n))


def compress_spectra(ghat: np.ndarray, nzs: int, nxs: int, keep_z: int, keep_x: int) -> np.ndarray:
    """Spatially compressed spectra (Discussion: an orthonormal transform Psi
    of the spatial axis, keeping the leading coefficients): each spectrum row,
    seen as an nzs x nxs image, is transformed by the 2D DCT-II and cropped to
    the leading keep_z x keep_x coefficients.  ``ghat`` is ``[nf][nr][nzs*nxs]``;
    returns ``[nf][nr][keep_z*keep_x]`` (kz-major)."""
    g = np.asarray(ghat, dtype=np.complex128).reshape(ghat.shape[0], ghat.shape[1], nzs, nxs)
    Dz = dct_matrix(nzs, keep_z)
    Dx = dct_matrix(nxs, keep_x)
    c = np.einsum("az,frzx,bx->frab", Dz, g, Dx, optimize=True)
    return c.reshape(ghat.shape[0], ghat.shape[1], keep_z * keep_x)


def hessian_compressed(ghat: np.ndarray, nzs: int, nxs: int, keep_z: int, keep_x: int) -> np.ndarray:
    """Hhat ~ (Ghat Psi^T)(Ghat Psi^T)^H with Psi the cropped 2D DCT-II; exact
    (= hessian_r1) when every coefficient is kept."""
    return hessian_r1(compress_spectra(ghat, nzs, nxs, keep_z, keep_x))


def running_dft_gram(gt: np.ndarray, freqs_hz, dt: float) -> np.ndarray:
    """(1/Nt) sum_{p=1}^{Nt} Ghat_p Ghat_p^H at each frequency (the R2 form).

    Ghat_p(w, x) = sum_{n=1}^{p} g(n, x) exp(-i w n dt).  ``gt`` is
    ``[nr][Nt][nsub]``.  Cost O(nf nr^2 nsub Nt): small sizes only.
    """
    nr, nt, nsub = gt.shape
    w = 2.0 * math.pi * np.asarray(freqs_hz, dtype=np.float64)
    out = np.zeros((len(w), nr, nr), dtype=np.complex128)
    for f, wf in enumerate(w):
        acc = np.zeros((nr, nsub), dtype=np.complex128)
        for p in range(1, nt + 1):
            acc += gt[:, p - 1, :] * np.exp(-1j * wf * p * dt)
            out[f] += acc @ acc.conj().T
    return out / nt


def hessian_r2(gt: np.ndarray, freqs_hz, dt: float) -> np.ndarray:
    """Finite-record (W-weighted) Hessian without penalty, ``[nf][nr][nr]``."""
    return running_dft_gram(gt, freqs_hz, dt)


# ---------------------------------------------------------------------------
# time-axis resampling of the record before the finite-record Hessian
# ---------------------------------------------------------------------------

def _bessel_i0(x: np.ndarray) -> np.ndarray:
    return np.i0(x)


def decimation_filter(D: int, dt: float, f_max: float, atten_db: float = 120.0) -> np.ndarray:
    """Zero-phase low-pass taps h_j, j = -K..K, for keeping every D-th sample.

    Kaiser-windowed sinc (Kaiser's design rules): the passband ends at f_max
    (the highest frequency the Hessian needs), the stopband starts at
    fs/D - f_max (the lowest frequency that folds onto the passband once every
    D-th sample is kept), the cutoff fc = fs/(2D) lies halfway;
    beta = 0.1102 (A - 8.7), filter order N = (A - 7.95) / (14.36 df / fs)
    with df = fs/D - 2 f_max, half-length K = ceil(N / 2); taps
    (1/D) sinc(j / D) I0(beta sqrt(1 - (j/K)^2)) / I0(beta), scaled to unit
    sum.  D = 1 gives the single tap 1.
    """
    if D <= 1:
        return np.ones(1)
    fs = 1.0 / dt
    df = fs / D - 2.0 * f_max
    if df <= 0:
        raise ValueError("decimation factor too large for the highest frequency")
    beta = 0.1102 * (atten_db - 8.7)
    order = (atten_db - 7.95) / (14.36 * df / fs)
    K = int(math.ceil(order / 2.0))
    j = np.arange(-K, K + 1, dtype=np.float64)
    w = _bessel_i0(beta * np.sqrt(np.maximum(0.0, 1.0 - (j / K) ** 2))) / _bessel_i0(np.array(beta))
    h = np.sinc(j / D) / D * w
    return h / h.sum()


def decimation_times(nt: int, D: int, K: int):
    """Times (sample indices) n_q = 1 - K + q D of the kept samples, q = 0..M-1,
    M the count whose filter support [n_q - K, n_q + K] meets the record
    1..nt; and the range [qa, qb] of those inside the record (1 <= n_q <= nt)."""
    if D <= 1:
        n = np.arange(1, nt + 1)
        return n, 0, nt - 1
    M = (nt - 1 + 2 * K) // D + 1
    n = 1 - K + D * np.arange(M)
    inside = np.nonzero((n >= 1) & (n <= nt))[0]
    return n, int(inside[0]), int(inside[-1])


def decimate(gt: np.ndarray, D: int, h: np.ndarray) -> np.ndarray:
    """y_q(x) = sum_{j=-K}^{K} h_j g(n_q + j, x) at the kept times n_q of
    ``decimation_times``, with g(n) = 0 outside 1..nt.  ``gt`` is
    ``[nr][nt][...]``; returns ``[nr][M][...]``."""
    K = (len(h) - 1) // 2
    nr, nt = gt.shape[:2]
    n, _, _ = decimation_times(nt, D, K)
    out = np.zeros((nr, len(n)) + gt.shape[2:])
    for q, nq in enumerate(n):
        for jj, hj in enumerate(h):
            m = nq + jj - K                  # sample index 1..nt
            if 1 <= m <= nt:
                out[:, q] += hj * gt[:, m - 1]
    return out


def hessian_r2_decimated(gt: np.ndarray, freqs_hz, dt: float, D: int, atten_db: float = 120.0) -> np.ndarray:
    """Finite-record Hessian on the record resampled to every D-th sample.

    With h = decimation_filter(D, dt, max f), y = decimate(g), the kept times
    n_q and H(w) = sum_j h_j exp(-i w j dt) (real), the running spectra are
    Gt_q(w) = (D / H(w)) sum_{m <= q} y_m exp(-i w n_m dt) and
        Hhat_W^D(w) = (D / Nt) sum_{q: 1 <= n_q <= Nt} Gt_q(w) Gt_q(w)^H.
    ``gt`` is ``[nr][Nt][nsub]``; returns ``[nf][nr][nr]``.  D = 1 is
    ``hessian_r2``."""
    nr, nt, nsub = gt.shape
    fmax = float(np.max(freqs_hz))
    h = decimation_filter(D, dt, fmax, atten_db)
    K = (len(h) - 1) // 2
    y = decimate(gt, D, h)
    n, qa, qb = decimation_times(nt, D, K)
    w = 2.0 * math.pi * np.asarray(freqs_hz, dtype=np.float64)
    j = np.arange(-K, K + 1)
    out = np.zeros((len(w), nr, nr), dtype=np.complex128)
    for f, wf in enumerate(w):
        Hw = float(np.real(np.sum(h * np.exp(-1j * wf * j * dt))))
        c = D / Hw
        acc = np.zeros((nr, nsub), dtype=np.complex128)
        for q in range(len(n)):
            acc += y[:, q, :] * np.exp(-1j * wf * n[q] * dt)
            if qa <= q <= qb:
                g = c * acc
                out[f] += g @ g.conj().T
    return out * (D / nt)
