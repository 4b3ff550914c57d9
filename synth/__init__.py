"""Seeded synthetic survey generators shared by the HIP path, its tests and the oracle.

This module draws inputs only: velocity models, receiver positions, frequency
lists and data residuals.  It holds none of the method's arithmetic (no
coefficients, sponge, time stepping, transforms or linear algebra), so the
oracle and the GPU path can both consume it without sharing any computation.

All randomness uses ``numpy.random.default_rng(seed)`` (PCG64).  Velocities are
returned as float32 arrays, exactly the values the GPU receives; the oracle
upcasts the same array to float64.  Residuals are complex64 for the same reason.

The surveys stand in for the paper's Marmousi II and 2004 BP benchmark models
(numerical-examples section), which are not reproduced here: layered and smooth
synthetic media of comparable size, receiver count and record length.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Survey:
    """One survey: medium, acquisition, time axis, frequencies and sources.

    Grid conventions: the interior grid is ``[nz][nx]`` (row-major, z down),
    spacing ``h`` metres, surrounded by an ``nb``-cell absorbing layer on all four
    sides.  Receivers sit at interior indices ``(rec_iz[k], rec_ix[k])``.
    ``nt`` time steps of ``dt`` seconds give samples u^1..u^nt.  The Hessian
    contraction runs over interior cells with stride ``stride`` in both axes.
    """

    name: str
    nz: int
    nx: int
    h: float
    nb: int
    nt: int
    dt: float
    freqs_hz: tuple
    rec_iz: tuple
    rec_ix: tuple
    ns: int
    stride: int
    model_seed: int
    resid_seed: int
    model_kind: str  # "linear_anomaly" | "layered" | "homogeneous"
    v_const: float = 2000.0
    n_interfaces: int = 12
    v_min: float = 1500.0
    v_max: float = 4700.0

    @property
    def nr(self) -> int:
        return len(self.rec_ix)

    @property
    def nf(self) -> int:
        return len(self.freqs_hz)

    @property
    def nzs(self) -> int:
        return (self.nz + self.stride - 1) // self.stride

    @property
    def nxs(self) -> int:
        return (self.nx + self.stride - 1) // self.stride

    @property
    def nsub(self) -> int:
        return self.nzs * self.nxs

    @property
    def padded_shape(self):
        return (self.nz + 2 * self.nb, self.nx + 2 * self.nb)

    def velocity(self) -> np.ndarray:
        return velocity_model(self)

    def residuals(self, ns: int | None = None, seed: int | None = None) -> np.ndarray:
        return residuals(self.nf, self.ns if ns is None else ns, self.nr,
                         self.resid_seed if seed is None else seed)

    def with_(self, **kw) -> "Survey":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# velocity models
# ---------------------------------------------------------------------------

def _linear_anomaly(nz, nx, h, seed):
    """v(z) rising linearly 1500 -> 3000 m/s over 1000 m plus one Gaussian anomaly.

    The anomaly has amplitude +-300 m/s and sigma 80 m; its centre (z, x) is
    drawn uniformly in [200, 800] m (both axes) and its sign uniformly from
    {-1, +1}, in that order, from ``default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    zc = rng.uniform(200.0, 800.0)
    xc = rng.uniform(200.0, 800.0)
    sign = -1.0 if rng.integers(0, 2) == 0 else 1.0
    z = np.arange(nz, dtype=np.float64)[:, None] * h
    x = np.arange(nx, dtype=np.float64)[None, :] * h
    v = 1500.0 + 1500.0 * z / 1000.0 + 0.0 * x
    r2 = (z - zc) ** 2 + (x - xc) ** 2
    v = v + sign * 300.0 * np.exp(-r2 / (2.0 * 80.0 ** 2))
    return v


def _layered(nz, nx, h, seed, n_if, v_min, v_max):
    """Layered medium with ``n_if`` randomly dipping planar interfaces.

    Interface k: z_k(x) = z0_k + tan(theta_k) (x - x_mid), z0_k drawn as sorted
    U(0.05, 0.95) * depth, theta_k ~ U(-15, 15) degrees.  Layer velocities:
    v_0 = v_min, v_1..v_{n-1} sorted U(v_min, v_max), v_n = v_max; a point lies in
    layer #{k : z > z_k(x)}.  Draw order: z0, theta, inner velocities.
    """
    rng = np.random.default_rng(seed)
    depth = nz * h
    z0 = np.sort(rng.uniform(0.05, 0.95, size=n_if)) * depth
    theta = np.deg2rad(rng.uniform(-15.0, 15.0, size=n_if))
    inner = np.sort(rng.uniform(v_min, v_max, size=n_if - 1))
    vel = np.concatenate([[v_min], inner, [v_max]])
    z = np.arange(nz, dtype=np.float64)[:, None] * h
    x = np.arange(nx, dtype=np.float64)[None, :] * h
    x_mid = 0.5 * nx * h
    count = np.zeros((nz, nx), dtype=np.int64)
    for k in range(n_if):
        zk = z0[k] + np.tan(theta[k]) * (x - x_mid)
        count += (z > zk).astype(np.int64)
    return vel[count]


def velocity_model(s: Survey) -> np.ndarray:
    """Interior velocity ``[nz][nx]`` in m/s, float32 (the exact GPU input)."""
    if s.model_kind == "linear_anomaly":
        v = _linear_anomaly(s.nz, s.nx, s.h, s.model_seed)
    elif s.model_kind == "layered":
        v = _layered(s.nz, s.nx, s.h, s.model_seed, s.n_interfaces, s.v_min, s.v_max)
    elif s.model_kind == "homogeneous":
        v = np.full((s.nz, s.nx), s.v_const)
    else:
        raise ValueError(f"unknown model kind {s.model_kind!r}")
    return np.ascontiguousarray(v, dtype=np.float32)


# ---------------------------------------------------------------------------
# residuals
# ---------------------------------------------------------------------------

def residuals(nf: int, ns: int, nr: int, seed: int) -> np.ndarray:
    """Frequency-domain data residuals ``[nf][ns][nr]`` complex64.

    i.i.d. circular complex Gaussian (N(0,1) + i N(0,1)) / sqrt(2) per
    (frequency, source, receiver): real parts are drawn first, then imaginary.
    """
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nf, ns, nr))
    im = rng.standard_normal((nf, ns, nr))
    return ((re + 1j * im) / math.sqrt(2.0)).astype(np.complex64)


def residuals_device(nf: int, ns: int, nr: int, seed: int, device) -> "torch.Tensor":
    """Residuals ``[nf][ns][nr]`` complex64 drawn on the device (for request
    streams, where a host draw per request would stall the scheduler).

    torch's device generator seeded with ``seed``: real parts then imaginary
    parts, each N(0, 1/2).  A different stream of numbers from ``residuals``
    for the same seed; the same seed always gives the same tensor.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    z = torch.randn((2, nf, ns, nr), generator=g, device=device, dtype=torch.float32)
    z.mul_(math.sqrt(0.5))
    return torch.complex(z[0], z[1])


def spectra(nf: int, nr: int, nsub: int, seed: int, decades: float = 4.0) -> np.ndarray:
    """Seeded stand-in for Green-function spectra, complex64 ``[nf][nr][nsub]``:
    per frequency U diag(s) V with U a random unitary nr x nr matrix (QR of a
    complex Gaussian), s_k = 10^(-decades k / nr) and V complex Gaussian rows
    scaled by 1/sqrt(nsub), so the Gram matrix of the rows spans about
    2 * decades decades (the spread of a survey's low-frequency Hessians).
    Draw order per frequency: the Gaussian for U (real, imaginary), then V."""
    rng = np.random.default_rng(seed)
    out = np.empty((nf, nr, nsub), dtype=np.complex64)
    sv = 10.0 ** (-decades * np.arange(nr) / nr)
    for f in range(nf):
        a = rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))
        q, _ = np.linalg.qr(a)
        v = (rng.standard_normal((nr, nsub)) + 1j * rng.standard_normal((nr, nsub))) / math.sqrt(2.0 * nsub)
        out[f] = ((q * sv[None, :]) @ v).astype(np.complex64)
    return out


def time_residuals(ns: int, nr: int, nt: int, seed: int) -> np.ndarray:
    """Time-domain data residuals ``[ns][nr][nt]`` float32, i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ns, nr, nt), dtype=np.float32)


def subgrid_sources(ns: int, nt: int, nzs: int, nxs: int, seed: int) -> np.ndarray:
    """Source fields on the subgrid ``[ns][nt][nzs][nxs]`` float32, i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ns, nt, nzs, nxs), dtype=np.float32)


def ricker(nt: int, dt: float, f0: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet of peak frequency f0 at samples n = 0..nt-1 (time n dt),
    centred at t0 (default 1.5 / f0), float32."""
    t0 = 1.5 / f0 if t0 is None else t0
    a = (math.pi * f0 * (np.arange(nt) * dt - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def smoothed(vel: np.ndarray, radius: int) -> np.ndarray:
    """Box-filtered copy of a velocity model (edges replicated): a starting
    model for the accuracy test."""
    from scipy.ndimage import uniform_filter
    return uniform_filter(np.asarray(vel, dtype=np.float64), size=2 * radius + 1,
                          mode="nearest").astype(np.float32)


def nearest_bins(nt: int, dt: float, freqs_hz) -> tuple:
    """The bins of the 2nt-point transform nearest to the given frequencies
    (distinct, ascending)."""
    k = sorted({int(round(f * 2.0 * nt * dt)) for f in freqs_hz})
    return transform_bins(nt, dt, k)


def transform_bins(nt: int, dt: float, k) -> tuple:
    """Frequencies (Hz) of bins k of the 2nt-point transform: k / (2 nt dt)."""
    return tuple(float(kk) / (2.0 * nt * dt) for kk in k)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def tiny() -> Survey:
    """101 x 101 at 10 m, 20-cell sponge, v(z) 1500->3000 m/s + anomaly,
    16 surface receivers, nt = 1000 at 1 ms, f = {3,5,7,9} Hz, Ns = 8, stride 1."""
    return Survey(
        name="tiny-101x101-nr16-nt1000-nf4",
        nz=101, nx=101, h=10.0, nb=20, nt=1000, dt=1.0e-3,
        freqs_hz=(3.0, 5.0, 7.0, 9.0),
        rec_iz=(2,) * 16, rec_ix=tuple(5 + 6 * k for k in range(16)),
        ns=8, stride=1, model_seed=1000, resid_seed=2000,
        model_kind="linear_anomaly")


def layered_1000x300() -> Survey:
    """1000 x 300 at 10 m, 40-cell sponge, 12 dipping interfaces 1500-4700 m/s,
    200 receivers every 50 m, nt = 4000 at 0.8 ms, 30 frequencies over 3-15 Hz,
    Ns = 200, stride 2 (complex64 Green-function spectra: 3.6 GB)."""
    return Survey(
        name="layered-1000x300-nr200-nt4000-nf30-ns200",
        nz=300, nx=1000, h=10.0, nb=40, nt=4000, dt=0.8e-3,
        freqs_hz=tuple(3.0 + 12.0 * k / 29.0 for k in range(30)),
        rec_iz=(2,) * 200, rec_ix=tuple(2 + 5 * k for k in range(200)),
        ns=200, stride=2, model_seed=1001, resid_seed=2001,
        model_kind="layered")


# (nx, nz, Nr, nf, Ns) of the eight uneven surveys of the batched workload.
BATCH_SPECS = (
    (400, 150, 96, 10, 64),
    (1700, 350, 400, 40, 400),
    (600, 200, 300, 20, 128),
    (1200, 250, 160, 30, 256),
    (900, 300, 128, 40, 96),
    (1500, 180, 350, 15, 320),
    (500, 320, 220, 25, 200),
    (1100, 280, 256, 35, 160),
)


def batch_survey(k: int, nt: int = 4000) -> Survey:
    """Survey k (0..7) of the batched uneven workload: layered model seed 1300+k,
    residual seed 2300+k, h = 10 m, 40-cell sponge, dt = 0.8 ms, nf frequencies
    evenly spaced over 3-20 Hz, receivers at iz = 2, ix = 2 + j*floor((nx-4)/Nr)."""
    nx, nz, nr, nf, ns = BATCH_SPECS[k]
    step = (nx - 4) // nr
    freqs = tuple(3.0 + 17.0 * i / (nf - 1) for i in range(nf))
    return Survey(
        name=f"batch{k}-{nx}x{nz}-nr{nr}-nf{nf}-ns{ns}",
        nz=nz, nx=nx, h=10.0, nb=40, nt=nt, dt=0.8e-3,
        freqs_hz=freqs, rec_iz=(2,) * nr, rec_ix=tuple(2 + j * step for j in range(nr)),
        ns=ns, stride=2, model_seed=1300 + k, resid_seed=2300 + k,
        model_kind="layered")


def batch_surveys(nt: int = 4000) -> List[Survey]:
    return [batch_survey(k, nt) for k in range(len(BATCH_SPECS))]


def homogeneous(n: int = 161, nb: int = 20, h: float = 10.0, v: float = 2000.0,
                nt: int = 1200, dt: float = 1.0e-3, freqs: Sequence[float] = (3.0, 5.0, 7.0, 9.0),
                rec=((80, 80),), stride: int = 1) -> Survey:
    """Homogeneous square medium, used against closed-form Green functions."""
    return Survey(
        name=f"homog-{n}", nz=n, nx=n, h=h, nb=nb, nt=nt, dt=dt,
        freqs_hz=tuple(freqs), rec_iz=tuple(r[0] for r in rec), rec_ix=tuple(r[1] for r in rec),
        ns=1, stride=stride, model_seed=0, resid_seed=0,
        model_kind="homogeneous", v_const=v)


def micro(nz: int = 31, nx: int = 31, nb: int = 8, nt: int = 120, nr: int = 4,
          seed: int = 7, stride: int = 1) -> Survey:
    """A micro survey small enough for the explicit time-domain Hessian."""
    freqs = (5.0, 10.0, 15.0, 20.0)
    step = max(1, (nx - 4) // nr)
    return Survey(
        name=f"micro-{nz}x{nx}-nt{nt}-nr{nr}", nz=nz, nx=nx, h=10.0, nb=nb, nt=nt, dt=1.0e-3,
        freqs_hz=freqs, rec_iz=(2,) * nr, rec_ix=tuple(2 + j * step for j in range(nr)),
        ns=3, stride=stride, model_seed=seed, resid_seed=seed + 1,
        model_kind="layered", n_interfaces=3, v_min=1500.0, v_max=2500.0)


def ragged(nz: int = 45, nx: int = 77, nb: int = 9, nt: int = 157, nr: int = 5,
           stride: int = 2, seed: int = 11) -> Survey:
    """Odd sizes everywhere, for tile-edge coverage (ragged subgrid tails)."""
    freqs = (4.0, 7.5, 11.0)
    return Survey(
        name=f"ragged-{nz}x{nx}-nt{nt}-nr{nr}-s{stride}", nz=nz, nx=nx, h=10.0, nb=nb, nt=nt,
        dt=1.0e-3, freqs_hz=freqs, rec_iz=tuple(1 + (k % 3) for k in range(nr)),
        rec_ix=tuple(3 + 13 * k for k in range(nr)), ns=5, stride=stride,
        model_seed=seed, resid_seed=seed + 1, model_kind="layered", n_interfaces=4,
        v_min=1500.0, v_max=3000.0)


def accuracy_micro(nt: int = 60) -> Survey:
    """A survey whose frequencies are every bin 0..nt of the 2nt-point
    transform (24 x 30 grid, 6-cell sponge, 4 surface receivers, stride 1), for
    the accuracy test at full band."""
    s = micro(nz=24, nx=30, nb=6, nt=nt, nr=4, seed=21)
    return s.with_(name=f"accuracy-micro-nt{nt}", freqs_hz=transform_bins(nt, s.dt, range(nt + 1)))


def accuracy_tiny() -> Survey:
    """The tiny survey with the 21 bins of the 2nt-point transform in 2-12 Hz
    (0.5 Hz apart), for the accuracy-test workload."""
    t = tiny()
    return t.with_(name="accuracy-tiny-101x101-nr16-nt1000-nf21",
                   freqs_hz=transform_bins(t.nt, t.dt, range(4, 25)))


WORKLOADS = {
    "tiny": tiny,
    "layered_1000x300": layered_1000x300,
}
