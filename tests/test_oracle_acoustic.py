"""Pins for the oracle's acoustic solver (Eq. (Acou), Algorithm 1).

Each test checks the oracle against something other than itself:
  * a dense-matrix brute force assembled from independently solved weights;
  * the exact discrete plane-wave solution (the dispersion relation of the
    leapfrog scheme) in the region the walls have not yet reached;
  * the stability threshold given by the spectral radius of the dense
    operator, and the CFL condition of Eq. (stability) being sufficient;
  * the homogeneous 3D Green's function q(t - r/v) / (4 pi r) of Eq. (Acou);
  * exact mirror symmetry, and bitwise resume from a saved state.
The damping term has no pin in the paper (it leaves boundary treatment out
of its model); beyond the brute force it is checked only for energy decay.
"""
import numpy as np
import pytest

import oracle
from tests import _bruteforce as bf
from workloads import ricker


def brute_acoustic(ndim, shape_zyx, nbl, h, dt, so, vel, eta, src, q, rec, nt, u0=None, u1=None):
    """Dense-matrix leapfrog with damping, source and receivers."""
    N = int(np.prod(shape_zyx))
    D2 = bf.second_derivative_ops(shape_zyx, so, h)
    L = D2[0] + D2[2] + (D2[1] if ndim == 3 else 0.0)
    v = vel.astype(np.float64).ravel()
    A = dt * dt * v * v
    s = 0.5 * dt * eta.astype(np.float64).ravel() if eta is not None else np.zeros(N)
    hp = h[0] * h[2] * (h[1] if ndim == 3 else 1.0)
    S = np.array([bf.interp_row(shape_zyx, nbl, h, c, ndim) for c in src]).reshape(len(src), N)
    R = np.array([bf.interp_row(shape_zyx, nbl, h, c, ndim) for c in rec]).reshape(len(rec), N)
    up = np.zeros(N) if u0 is None else u0.ravel().copy()
    uc = np.zeros(N) if u1 is None else u1.ravel().copy()
    traces = np.zeros((nt, len(rec)))
    for t in range(nt):
        un = (2 * uc - (1 - s) * up + A * (L @ uc)) / (1 + s)
        un = un + (A / (1 + s)) * (S.T @ q[t].astype(np.float64)) / hp
        traces[t] = R @ un
        up, uc = uc, un
    return traces, up.reshape(shape_zyx), uc.reshape(shape_zyx)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("so", [2, 4, 8])
def test_bruteforce_2d(so):
    rng = np.random.default_rng(11 + so)
    nz, nx, nbl = 13, 16, 3
    h = (10.0, 1.0, 7.5)
    vel = (1500 + 500 * rng.random((nz, nx))).astype(np.float32)
    eta = (30 * rng.random((nz, nx))).astype(np.float32)
    dt = 0.5 * oracle.cfl_dt(2, so, h, float(vel.max()))
    src = np.array([[37.0, 21.3], [0.0, 0.0]])           # off-grid and on-grid
    rec = np.array([[13.1, 40.0], [50.0, 7.5], [-30.0, -22.5]])
    nt = 12
    q = rng.standard_normal((nt, 2)).astype(np.float32)
    tr, up, uc = oracle.acoustic_forward(2, nbl, h, dt, so, vel, eta, src, q, rec, nt)
    tb, ub_p, ub_c = brute_acoustic(2, (nz, 1, nx), nbl, h, dt, so, vel, eta, src, q, rec, nt)
    assert rel(tr, tb) < 1e-10
    assert rel(uc, ub_c.reshape(nz, nx)) < 1e-10
    assert rel(up, ub_p.reshape(nz, nx)) < 1e-10


@pytest.mark.parametrize("so", [2, 4, 6])
def test_bruteforce_3d(so):
    rng = np.random.default_rng(21 + so)
    nz, ny, nx, nbl = 7, 6, 8, 2
    h = (10.0, 12.0, 8.0)
    vel = (1800 + 400 * rng.random((nz, ny, nx))).astype(np.float32)
    eta = (20 * rng.random((nz, ny, nx))).astype(np.float32)
    dt = 0.5 * oracle.cfl_dt(3, so, h, float(vel.max()))
    src = np.array([[11.0, 5.0, 3.3]])
    rec = np.array([[1.0, 2.0, 3.0], [-20.0, -24.0, -16.0], [30.0, 30.0, 20.0]])
    nt = 8
    q = rng.standard_normal((nt, 1)).astype(np.float32)
    tr, up, uc = oracle.acoustic_forward(3, nbl, h, dt, so, vel, eta, src, q, rec, nt)
    tb, ub_p, ub_c = brute_acoustic(3, (nz, ny, nx), nbl, h, dt, so, vel, eta, src, q, rec, nt)
    assert rel(tr, tb) < 1e-10
    assert rel(uc, ub_c) < 1e-10


def _symbol(w, theta):
    """Second-derivative symbol W(theta) = w0 + 2 sum_j w_j cos(j theta)."""
    return w[0] + 2 * sum(w[j] * np.cos(j * theta) for j in range(1, len(w)))


@pytest.mark.parametrize("ndim,so", [(2, 2), (2, 4), (2, 8), (3, 4), (3, 8)])
def test_plane_wave_exact(ndim, so):
    """cos(k.x - n w dt) with sin^2(w dt/2) = (v dt/2)^2 sum_a -W(k_a h_a)/h_a^2
    is an exact solution of the scheme; after n steps it must hold to
    rounding wherever the zero walls have not yet reached (n r points)."""
    r = so // 2
    w = oracle.weights_d2(so)
    v = 2000.0
    if ndim == 2:
        shape = (72, 80)               # [nz][nx]
        h = (10.0, 1.0, 7.0)
        k = np.array([2 * np.pi / (9.3 * h[0]), 0.0, 2 * np.pi / (13.7 * h[2])])
        nsteps = 24 // r
    else:
        shape = (40, 38, 42)
        h = (10.0, 12.0, 8.0)
        k = np.array([2 * np.pi / (7.1 * h[0]), 2 * np.pi / (11.3 * h[1]),
                      -2 * np.pi / (8.9 * h[2])])
        nsteps = 12 // r
    dt = 0.8 * oracle.cfl_dt(ndim, so, h, v)
    X2 = sum(-_symbol(w, k[a] * h[a]) / h[a] ** 2 for a in range(3) if ndim == 3 or a != 1)
    om = 2.0 / dt * np.arcsin(0.5 * v * dt * np.sqrt(X2))
    if ndim == 2:
        z, x = np.meshgrid(np.arange(shape[0]) * h[2], np.arange(shape[1]) * h[0], indexing="ij")
        phase = k[0] * x + k[2] * z
    else:
        z, y, x = np.meshgrid(np.arange(shape[0]) * h[2], np.arange(shape[1]) * h[1],
                              np.arange(shape[2]) * h[0], indexing="ij")
        phase = k[0] * x + k[1] * y + k[2] * z
    u_prev = np.cos(phase + om * dt)
    u_cur = np.cos(phase)
    vel = np.full(shape, v, dtype=np.float32)
    _, up, uc = oracle.acoustic_forward(ndim, 0, h, dt, so, vel, None, [], np.zeros((nsteps, 0)),
                                        [], nsteps, u_prev, u_cur)
    exact = np.cos(phase - nsteps * om * dt)
    d = nsteps * r
    sl = tuple(slice(d, n - d) for n in shape)
    assert exact[sl].size > 100
    err = np.max(np.abs(uc[sl] - exact[sl]))
    assert err < 1e-11, err
    # and the walls did change the solution outside that region
    assert np.max(np.abs(uc - exact)) > 1e-6


@pytest.mark.parametrize("ndim,so", [(2, 2), (2, 4), (2, 8), (3, 4)])
def test_cfl_threshold_dense_spectrum(ndim, so):
    """Leapfrog with constant v is stable iff dt <= 2 / (v sqrt(lambda_max(-L))).
    The CFL bound of Eq. (stability) must be below that threshold and close to
    it; the oracle must blow up just above it and stay bounded just below."""
    shape = (12, 1, 14) if ndim == 2 else (6, 7, 5)
    h = (10.0, 9.0, 11.0)
    D2 = bf.second_derivative_ops(shape, so, h)
    L = D2[0] + D2[2] + (D2[1] if ndim == 3 else 0.0)
    lam = np.max(np.abs(np.linalg.eigvalsh(0.5 * (L + L.T))))
    v = 1700.0
    dt_crit = 2.0 / (v * np.sqrt(lam))
    dt_cfl = oracle.cfl_dt(ndim, so, h, v)
    assert dt_cfl <= dt_crit * (1 + 1e-12)
    assert dt_crit / dt_cfl < 1.25
    fshape = (shape[0], shape[2]) if ndim == 2 else shape
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal(fshape)
    vel = np.full(fshape, v, dtype=np.float32)
    nt = 150
    _, _, ug = oracle.acoustic_forward(ndim, 0, h, 1.03 * dt_crit, so, vel, None, [],
                                       np.zeros((nt, 0)), [], nt, u0, u0)
    _, _, us = oracle.acoustic_forward(ndim, 0, h, 0.97 * dt_crit, so, vel, None, [],
                                       np.zeros((nt, 0)), [], nt, u0, u0)
    n0 = np.linalg.norm(u0)
    assert np.linalg.norm(ug) > 1e6 * n0
    assert np.linalg.norm(us) < 50 * n0


def test_greens_function_3d():
    """Homogeneous 3D medium: the trace at distance r must follow
    q(t - r/v) / (4 pi r) (Eq. (Acou) with constant m and a point source),
    which pins the source scaling and the injection/recording timing."""
    so = 8
    h = (10.0, 10.0, 10.0)
    n, nbl = 60, 10
    v = 1500.0
    pad = (n + 2 * nbl,) * 3
    vel = np.full(pad, v, dtype=np.float32)
    dt = 0.4 * oracle.cfl_dt(3, so, h, v)
    f0 = 10.0
    nt = int(0.36 / dt)
    q = ricker(f0, dt, nt)[:, None]
    src = np.array([[300.0, 300.0, 300.0]])
    rec = np.array([[500.0, 300.0, 300.0], [300.0, 300.0, 150.0], [420.0, 420.0, 420.0]])
    oracle.set_threads(8)
    try:
        tr, _, _ = oracle.acoustic_forward(3, nbl, h, dt, so, vel, None, src, q, rec, nt)
    finally:
        oracle.set_threads(1)
    # trace sample n is u^{n+1}, i.e. time (n + 1) dt, driven by q(t_n) at
    # the centre of the leapfrog difference
    t = (np.arange(nt) + 1) * dt
    for j, c in enumerate(rec):
        r = np.linalg.norm(c - src[0])
        # analytic trace, wavelet evaluated at the retarded time
        tt = t - r / v - 1.0 / f0
        a = (np.pi * f0 * tt) ** 2
        ana = (1 - 2 * a) * np.exp(-a) / (4 * np.pi * r)
        e = rel(tr[:, j], ana)
        assert e < 0.01, (j, r, e)
        assert abs(tr[:, j].max() / ana.max() - 1) < 0.005
        # a one-sample shift in either direction is clearly worse
        for s in (-1, 1):
            assert rel(np.roll(tr[:, j], s), ana) > 5 * e


def test_mirror_symmetry_bitwise():
    """A centred source in a medium symmetric under x -> -x gives a field
    that is bitwise mirror-symmetric (symmetric pairs are summed first)."""
    so, nbl = 8, 6
    nz, nx = 41, 37
    h = (10.0, 1.0, 10.0)
    rng = np.random.default_rng(3)
    half = 1500 + 800 * rng.random((nz, nx // 2 + 1))
    vel = np.concatenate([half, half[:, -2::-1]], axis=1).astype(np.float32)
    assert np.array_equal(vel, vel[:, ::-1])
    eta = np.zeros((nz, nx), np.float32)
    eta[:, :nbl] = np.linspace(50, 0, nbl)[None, :]
    eta[:, -nbl:] = np.linspace(0, 50, nbl)[None, :]
    dt = 0.4 * oracle.cfl_dt(2, so, h, float(vel.max()))
    xs = (nx // 2 - nbl) * h[0]
    src = np.array([[xs, 120.0]])
    rec = np.array([[xs - 50.0, 40.0], [xs + 50.0, 40.0]])
    nt = 60
    q = ricker(20.0, dt, nt)[:, None]
    tr, up, uc = oracle.acoustic_forward(2, nbl, h, dt, so, vel, eta, src, q, rec, nt)
    assert np.array_equal(uc, uc[:, ::-1])
    assert np.array_equal(tr[:, 0], tr[:, 1])
    assert np.max(np.abs(uc)) > 0


def test_resume_bitwise():
    so, nbl = 4, 5
    shape = (30, 33)
    h = (10.0, 1.0, 10.0)
    rng = np.random.default_rng(9)
    vel = (1500 + 1000 * rng.random(shape)).astype(np.float32)
    eta = (10 * rng.random(shape)).astype(np.float32)
    dt = 0.4 * oracle.cfl_dt(2, so, h, float(vel.max()))
    src = np.array([[100.0, 80.0]])
    rec = np.array([[20.0, 30.0], [150.0, 44.4]])
    nt = 40
    q = ricker(25.0, dt, nt)[:, None]
    tr, up, uc = oracle.acoustic_forward(2, nbl, h, dt, so, vel, eta, src, q, rec, nt)
    t1, p1, c1 = oracle.acoustic_forward(2, nbl, h, dt, so, vel, eta, src, q[:17], rec, 17)
    t2, p2, c2 = oracle.acoustic_forward(2, nbl, h, dt, so, vel, eta, src, q[17:], rec, 23, p1, c1)
    assert np.array_equal(np.concatenate([t1, t2]), tr)
    assert np.array_equal(c2, uc) and np.array_equal(p2, up)


def test_damping_energy_decays():
    """After the source stops, a damped layer removes energy monotonically
    (over windows), while the undamped box keeps it."""
    so, nbl = 4, 12
    n = 40
    shape = (n + 2 * nbl, n + 2 * nbl)
    h = (10.0, 1.0, 10.0)
    vel = np.full(shape, 2000.0, np.float32)
    from workloads import damping_profile
    eta = damping_profile(shape, nbl, h, 2000.0)
    dt = 0.4 * oracle.cfl_dt(2, so, h, 2000.0)
    nt = 800
    q = ricker(15.0, dt, nt)[:, None]
    src = np.array([[200.0, 200.0]])
    energies = []
    up = uc = None
    for k in range(8):
        _, up, uc = oracle.acoustic_forward(2, nbl, h, dt, so, vel, eta, src,
                                            q[k * 100:(k + 1) * 100], [], 100, up, uc)
        energies.append(np.sum(uc ** 2))
    tail = energies[3:]
    assert all(b < a for a, b in zip(tail, tail[1:]))
    assert tail[-1] < 1e-3 * max(energies)
