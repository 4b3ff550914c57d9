"""Pins of the oracle's finite-difference Green functions and DFT (CPU only).

Each test checks the oracle against something other than itself: the 2D
closed-form Green function, exactness of the stencil on polynomials, discrete
reciprocity, energy conservation, numpy's FFT, and adjointness.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import fd

ALPHA = 12.0  # damping of the DFT (1/s) so that the finite record is negligible


def _hankel_errors(n, nb, h, dt, nt, freqs=(3.0, 6.0, 9.0), radii=(100.0, 200.0, 300.0)):
    c = n // 2
    s = synth.homogeneous(n=n, nb=nb, h=h, nt=nt, dt=dt, rec=((c, c),))
    gt = fd.green_samples(s.velocity(), s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    t = np.arange(1, nt + 1) * dt
    errs = []
    for f in freqs:
        w = 2.0 * math.pi * f
        damp = np.exp(-(1j * w + ALPHA) * t)
        for r in radii:
            ir = int(round(r / h))
            g = np.dot(damp, gt[0, :, c, c + ir]) / (h * h)
            # outgoing 2D Green function of m u_tt - lap u = delta(x) delta(t) with the
            # forward transform exp(-i w t): (lap + k^2) G = -delta, G = (-i/4) H0^(2)(k r)
            k = (w - 1j * ALPHA) / 2000.0
            ref = -0.25j * sp.hankel2(0, k * r)
            errs.append(abs(g - ref) / abs(ref))
    return np.array(errs)


def test_green_matches_hankel_and_converges():
    coarse = _hankel_errors(161, 30, 10.0, 1.0e-3, 1500)
    assert coarse.max() < 2e-3, coarse
    fine = _hankel_errors(321, 60, 5.0, 0.5e-3, 3000)
    assert fine.max() < 6e-4, fine
    # halving h and dt must cut the error by ~4 (2nd order in time dominates)
    assert np.all(coarse / fine > 2.0), coarse / fine


def test_laplacian_exact_on_quartic():
    # the 4th-order stencil is exact for polynomials of degree <= 5
    Z, X, h = 12, 14, 2.0
    z = np.arange(Z)[:, None] * h
    x = np.arange(X)[None, :] * h
    u = z ** 4 - 3.0 * x ** 3 + z * x ** 2 + 7.0
    lap = fd.laplacian(u, h)
    exact = 12.0 * z ** 2 - 18.0 * x + 2.0 * z + 0.0 * x
    np.testing.assert_allclose(lap[2:-2, 2:-2], exact[2:-2, 2:-2], rtol=1e-12, atol=1e-9)


def test_reciprocity_tiny():
    s = synth.tiny().with_(nt=300)
    v = s.velocity()
    recs = [0, 5, 11, 15]
    gt = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, [s.rec_iz[i] for i in recs],
                          [s.rec_ix[i] for i in recs], 1)
    scale = np.abs(gt).max()
    for a, i in enumerate(recs):
        for b, j in enumerate(recs):
            gij = gt[a, :, s.rec_iz[j], s.rec_ix[j]]
            gji = gt[b, :, s.rec_iz[i], s.rec_ix[i]]
            assert np.abs(gij - gji).max() <= 1e-13 * scale


def test_energy_conserved_without_sponge():
    s = synth.micro(nz=40, nx=50, nb=0, nt=400)
    med = fd.Medium(s.velocity(), 0, s.h, s.dt)
    src = np.zeros((1,) + med.shape)
    src[0, 10, 20] = 1.0
    hist = []

    def inject(n):
        return src if n == 0 else None

    prev = [np.zeros((1,) + med.shape)]

    def record(n, u):
        # E^{n-1/2} = sum (u^n - u^{n-1})^2 / kappa - sum u^n L4 u^{n-1}
        up = prev[0]
        if n >= 2:
            e = np.sum((u - up) ** 2 / med.kappa) - np.sum(u * fd.laplacian(up, med.h))
            hist.append(e)
        prev[0] = u.copy()

    fd.propagate(med, s.nt, 1, inject, record)
    hist = np.array(hist)
    assert hist[0] > 0
    assert np.abs(hist - hist[0]).max() <= 1e-11 * hist[0]


def test_dft_matches_fft_on_bins():
    rng = np.random.default_rng(5)
    nt, dt = 64, 2e-3
    g = rng.standard_normal((3, nt, 7))
    bins = [0, 1, 5, 17, 63, 64]
    freqs = [k / (2 * nt * dt) for k in bins]
    got = fd.dft(g, freqs, dt)
    x = np.zeros((3, 2 * nt, 7))
    x[:, 1:nt + 1] = g                      # sample n sits at time index n
    ref = np.fft.fft(x, axis=1)[:, bins]    # [nr][k][x]
    np.testing.assert_allclose(got, ref.transpose(1, 0, 2), rtol=1e-12, atol=1e-12)


def test_forward_adjoint_are_transposes():
    s = synth.micro(nz=16, nx=18, nb=4, nt=30, nr=3)
    op = fd.ForwardOperator(s.velocity(), s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((s.nt, op.nsub))
    d = rng.standard_normal((op.nr, s.nt))
    lhs = np.vdot(op.apply(f), d)
    rhs = np.vdot(f, op.adjoint(d))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300) + 1e-300


def test_forward_operator_reproduces_green_functions():
    # S applied to a unit impulse at (step 0, subgrid point of receiver j) gives
    # g_j at the receivers: the Green functions are the impulse responses of S.
    s = synth.micro(nz=16, nx=18, nb=4, nt=30, nr=3)
    v = s.velocity()
    op = fd.ForwardOperator(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    gt = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, 1)
    for j in range(op.nr):
        f = np.zeros((s.nt, s.nz, s.nx))
        f[0, s.rec_iz[j], s.rec_ix[j]] = 1.0
        d = op.apply(f.reshape(s.nt, -1))
        for i in range(op.nr):
            np.testing.assert_allclose(d[i], gt[j, :, s.rec_iz[i], s.rec_ix[i]], rtol=1e-13,
                                       atol=1e-15 * np.abs(gt).max())


def test_c_recurrence_matches_numpy():
    # the plain-C loops (fdcore.c) reproduce the NumPy recurrence
    if fd._core() is None:
        pytest.skip("oracle/_fdcore.so not built")
    for s in (synth.ragged(nt=120), synth.tiny().with_(nt=150)):
        v = s.velocity()
        a = fd.green_samples(v, s.nb, s.h, s.dt, s.nt, s.rec_iz[:3], s.rec_ix[:3], s.stride)
        b = fd.green_samples_c(v, s.nb, s.h, s.dt, s.nt, s.rec_iz[:3], s.rec_ix[:3], s.stride)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


# ---------------------------------------------------------------------------
# the absorbing layer (reading of "appropriate boundary conditions"): a
# quadratic damping profile eta(d) = eta_max (d/nb)^2 with
# eta_max = 3 vmax ln(1000) / (2 nb h), entering the wave equation as the
# centred term m eta du/dt, over an edge-replicated extension of the model
# ---------------------------------------------------------------------------

def _plane_wave_trace(vel, nb, h, dt, nt, src_row, rec_row, f0=25.0):
    """Trace at the centre column of ``rec_row`` for a Ricker line source along
    the whole padded row ``src_row`` (interior row indices): a plane wave
    travelling up and down, away from the side layers."""
    med = fd.Medium(vel, nb, h, dt)
    w = synth.ricker(nt, dt, f0)
    f = np.zeros((1,) + med.shape)
    out = []

    def inject(n):
        f[0, src_row + nb, :] = w[n]
        return f

    cx = vel.shape[1] // 2 + nb
    fd.propagate(med, nt, 1, inject, lambda n, u: out.append(u[0, rec_row + nb, cx]))
    return np.array(out)


def test_sponge_absorbs_as_the_damped_wave_equation_predicts():
    # u_tt + eta u_t = v^2 lap u damps a wave travelling through the layer by
    # exp(-int eta / (2 v) ds) (WKB, eta << w, eta slowly varying).  A plane
    # wave going up into the top layer, reflected by the zero field beyond the
    # grid and coming back therefore returns with
    #   exp(-sum_{d=1}^{nb} eta(d) h / v)
    # of its amplitude.  The record ends before the side layers' disturbance or
    # the bottom layer's return reaches the receiver.  A wrong eta_max (say a
    # dropped factor 3, or twice the damping) or a linear profile moves the
    # ratio by a factor of 3 or more.
    nz, nx, nb, h, dt, v0 = 150, 401, 40, 10.0, 1.0e-3, 2000.0
    src_row, rec_row, nt = 40, 20, 1000
    vel = np.full((nz, nx), v0, dtype=np.float32)
    g = _plane_wave_trace(vel, nb, h, dt, nt, src_row, rec_row)
    t = np.arange(1, nt + 1) * dt
    t_inc = (src_row - rec_row) * h / v0
    t_ret = t_inc + 2.0 * (rec_row + nb + 1) * h / v0      # the zero field starts one cell beyond the layer
    inc = g[(t > t_inc - 0.02) & (t < t_inc + 0.15)]
    ret = g[(t > t_ret - 0.02) & (t < t_ret + 0.15)]
    ratio = np.ptp(ret) / np.ptp(inc)
    eta_max = 3.0 * v0 * math.log(1000.0) / (2.0 * nb * h)
    expected = math.exp(-sum(eta_max * (d / nb) ** 2 * h for d in range(1, nb + 1)) / v0)
    print("returned / incident amplitude", ratio, "WKB", expected)
    assert 0.75 * expected < ratio < 1.15 * expected


def test_layer_carries_the_edge_velocity():
    # v(z) = 2000 + 0.5 z in the interior; the layer above it must hold the top
    # row's velocity, so the pulse that goes up through the layer to the zero
    # field and back returns after 2 (int_0^{z_r} dz / v + (nb + 1) h / v(0)).
    # Mirrored or ramped extensions change that delay by 12-16 ms.
    nz, nx, nb, h, dt = 150, 401, 40, 10.0, 1.0e-3
    src_row, rec_row, nt = 40, 20, 1150
    grad = 0.5
    z = np.arange(nz) * h
    vel = np.ascontiguousarray(np.broadcast_to((2000.0 + grad * z)[:, None], (nz, nx)), dtype=np.float32)
    g = _plane_wave_trace(vel, nb, h, dt, nt, src_row, rec_row)
    t = np.arange(1, nt + 1) * dt
    v = lambda zz: 2000.0 + grad * zz
    t_inc = math.log(v(src_row * h) / v(rec_row * h)) / grad
    delay = 2.0 * (math.log(v(rec_row * h) / v(0.0)) / grad + (nb + 1) * h / v(0.0))
    inc = np.where((t > t_inc - 0.02) & (t < t_inc + 0.15), g, 0.0)
    ret = np.where((t > t_inc + delay - 0.02) & (t < t_inc + delay + 0.15), g, 0.0)
    # the zero field inverts the pulse: the returned pulse is the negative of a
    # delayed copy of the incident one
    cc = np.correlate(ret, inc, mode="full")
    lag = (int(np.argmax(-cc)) - (nt - 1)) * dt
    print("measured delay", lag, "travel time", delay)
    assert abs(lag - delay) <= 7.0e-3


def test_windowed_c_spectra_match_numpy():
    # the C recurrence advanced window by window with the DFT of each window
    # added to the running spectra equals the NumPy recurrence followed by the
    # DFT of the whole record (windows of 64 with a partial last one)
    if fd._core() is None:
        pytest.skip("oracle/_fdcore.so not built")
    for s in (synth.ragged(nt=157), synth.tiny().with_(nt=150)):
        v = s.velocity()
        ref = fd.green_dft(s, v, engine="numpy")
        got = fd.green_dft_windowed(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, s.freqs_hz,
                                    s.stride, window=64)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        # receivers in groups of 2 (a ragged last group)
        got = fd.green_dft_windowed(v, s.nb, s.h, s.dt, s.nt, s.rec_iz, s.rec_ix, s.freqs_hz,
                                    s.stride, window=64, max_window_bytes=8 * 64 * s.nsub * 2)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
