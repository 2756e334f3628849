"""Pins for the oracle's VTI solver (Eq. (vVTI); horizontal operator D_xx in
2D and D_xx + D_yy in 3D).

  * a dense block-matrix leapfrog with independently solved weights (2D and
    3D, damping, source into p and r, receivers on p);
  * in 3D the system is the TTI system with zero tilt and azimuth, against
    the (separately pinned) TTI oracle;
  * epsilon = delta = 0 reduces p and r to the acoustic field;
  * a homogeneous medium carries an exact discrete plane wave whose
    frequency and polarisation follow the 2 x 2 symbol of the system.
"""
import numpy as np
import pytest

import oracle
from tests import _bruteforce as bf
from workloads import ricker


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _model(shape, seed):
    rng = np.random.default_rng(seed)
    vel = (1800 + 600 * rng.random(shape)).astype(np.float32)
    eta = (15 * rng.random(shape)).astype(np.float32)
    eps = (0.3 * rng.random(shape)).astype(np.float32)
    delta = np.minimum(0.1 * rng.random(shape), eps).astype(np.float32)
    return rng, vel, eta, eps, delta


@pytest.mark.parametrize("ndim,so", [(2, 2), (2, 8), (3, 4)])
def test_dense_bruteforce_vti_run(ndim, so):
    nbl = 1
    shape_zyx = (7, 1, 9) if ndim == 2 else (6, 5, 7)
    fshape = (7, 9) if ndim == 2 else (6, 5, 7)
    h = (10.0, 11.0, 9.0)
    N = int(np.prod(shape_zyx))
    rng, vel, eta, eps, delta = _model(fshape, 31 + so + ndim)
    dt = 0.3 * oracle.cfl_dt(ndim, so, h, float(vel.max()) * np.sqrt(1.6))
    if ndim == 2:
        src = np.array([[20.0, 13.0]])
        rec = np.array([[0.0, 0.0], [30.0, 27.0], [-9.0, 31.5]])
    else:
        src = np.array([[20.0, 15.0, 13.0]])
        rec = np.array([[0.0, 0.0, 0.0], [30.0, 22.0, 27.0]])
    nt = 10
    q = rng.standard_normal((nt, 1)).astype(np.float32)
    tr, st = oracle.vti_forward(ndim, nbl, h, dt, so, vel, eta, eps, delta, src, q, rec, nt)

    D2 = bf.second_derivative_ops(shape_zyx, so, h)
    Hm = D2[0] + (D2[1] if ndim == 3 else 0.0)
    Zm = D2[2]
    A = dt * dt * vel.astype(np.float64).ravel() ** 2
    s = 0.5 * dt * eta.astype(np.float64).ravel()
    e2 = 1 + 2 * eps.astype(np.float64).ravel()
    sd = np.sqrt(1 + 2 * delta.astype(np.float64).ravel())
    S = bf.interp_row(shape_zyx, nbl, h, src[0], ndim)
    R = np.array([bf.interp_row(shape_zyx, nbl, h, c, ndim) for c in rec])
    hp = h[0] * h[2] * (h[1] if ndim == 3 else 1.0)
    pp = pc = rp = rc = np.zeros(N)
    tb = np.zeros((nt, len(rec)))
    for t in range(nt):
        hpv = Hm @ pc
        zr = Zm @ rc
        pn = (2 * pc - (1 - s) * pp + A * (e2 * hpv + sd * zr)) / (1 + s)
        rn = (2 * rc - (1 - s) * rp + A * (sd * hpv + zr)) / (1 + s)
        inj = A / (1 + s) * S * float(q[t, 0]) / hp
        pn, rn = pn + inj, rn + inj
        tb[t] = R @ pn
        pp, pc, rp, rc = pc, pn, rc, rn
    assert rel(tr, tb) < 1e-10
    assert rel(st[1].ravel(), pc) < 1e-10
    assert rel(st[3].ravel(), rc) < 1e-10


def test_vti_is_tti_without_tilt():
    so, nbl = 4, 3
    shape = (16, 14, 18)
    h = (10.0, 12.0, 9.0)
    rng, vel, eta, eps, delta = _model(shape, 8)
    z = np.zeros(shape, np.float32)
    dt = 0.4 * oracle.cfl_dt(3, so, h, float(vel.max()) * np.sqrt(1.6))
    src = np.array([[60.0, 50.0, 40.0]])
    rec = np.array([[10.0, 20.0, 30.0], [100.0, 80.0, 90.0]])
    nt = 25
    q = ricker(30.0, dt, nt)[:, None]
    tv, sv = oracle.vti_forward(3, nbl, h, dt, so, vel, eta, eps, delta, src, q, rec, nt)
    tt, stt = oracle.tti_forward(nbl, h, dt, so, vel, eta, eps, delta, z, z, src, q, rec, nt)
    assert rel(tv, tt) < 1e-12
    for a, b in zip(sv, stt):
        assert rel(a, b) < 1e-12


@pytest.mark.parametrize("ndim", [2, 3])
def test_isotropic_vti_equals_acoustic(ndim):
    so, nbl = 8, 4
    shape = (30, 34) if ndim == 2 else (16, 14, 18)
    h = (10.0, 10.0, 10.0)
    rng, vel, eta, _, _ = _model(shape, 9)
    z = np.zeros(shape, np.float32)
    dt = 0.4 * oracle.cfl_dt(ndim, so, h, float(vel.max()))
    src = np.array([[120.0, 90.0]]) if ndim == 2 else np.array([[70.0, 60.0, 55.0]])
    rec = np.array([[10.0, 30.0], [200.0, 150.0]]) if ndim == 2 else \
        np.array([[10.0, 20.0, 30.0], [100.0, 80.0, 90.0]])
    nt = 30
    q = ricker(30.0, dt, nt)[:, None]
    tv, sv = oracle.vti_forward(ndim, nbl, h, dt, so, vel, eta, z, z, src, q, rec, nt)
    ta, _, ua = oracle.acoustic_forward(ndim, nbl, h, dt, so, vel, eta, src, q, rec, nt)
    assert rel(sv[1], ua) < 1e-11 and rel(sv[3], ua) < 1e-11
    assert rel(tv, ta) < 1e-11


@pytest.mark.parametrize("ndim,so", [(2, 4), (3, 2), (3, 8)])
def test_vti_plane_wave_exact(ndim, so):
    """[p; r] = [a; b] cos(k.x - w t) with [a; b] an eigenvector of
    M = [[(1+2e) H, sqrt(1+2d) Z], [sqrt(1+2d) H, Z]] (H, Z the horizontal and
    vertical second-derivative symbols) and 4 sin^2(w dt/2) = dt^2 v^2 mu."""
    r = so // 2
    h = (10.0, 12.0, 9.0)
    w2 = oracle.weights_d2(so)
    v, e, d = (float(np.float32(c)) for c in (2500.0, 0.25, 0.1))
    if ndim == 2:
        shape = (40, 44)
        k = np.array([2 * np.pi / (7.3 * h[0]), 0.0, 2 * np.pi / (6.7 * h[2])])
    else:
        shape = (36, 34, 38)
        k = np.array([2 * np.pi / (7.3 * h[0]), -2 * np.pi / (9.1 * h[1]), 2 * np.pi / (6.7 * h[2])])
    X2 = np.array([-(w2[0] + 2 * sum(w2[j] * np.cos(j * k[a] * h[a]) for j in range(1, r + 1)))
                   / h[a] ** 2 for a in range(3)])
    Hs = X2[0] + (X2[1] if ndim == 3 else 0.0)
    Z = X2[2]
    M = np.array([[(1 + 2 * e) * Hs, np.sqrt(1 + 2 * d) * Z], [np.sqrt(1 + 2 * d) * Hs, Z]])
    mu, vec = np.linalg.eig(M)
    i = int(np.argmax(mu.real))
    mu, ab = mu[i].real, vec[:, i].real
    dt = 0.4 * oracle.cfl_dt(ndim, so, h, v * np.sqrt(1 + 2 * e))
    om = 2.0 / dt * np.arcsin(0.5 * v * dt * np.sqrt(mu))
    if ndim == 2:
        z, x = np.meshgrid(np.arange(shape[0]) * h[2], np.arange(shape[1]) * h[0], indexing="ij")
        phase = k[0] * x + k[2] * z
    else:
        z, y, x = np.meshgrid(np.arange(shape[0]) * h[2], np.arange(shape[1]) * h[1],
                              np.arange(shape[2]) * h[0], indexing="ij")
        phase = k[0] * x + k[1] * y + k[2] * z
    full = lambda c: np.full(shape, c, np.float32)
    state = (ab[0] * np.cos(phase + om * dt), ab[0] * np.cos(phase),
             ab[1] * np.cos(phase + om * dt), ab[1] * np.cos(phase))
    nsteps = 12 // r
    _, st = oracle.vti_forward(ndim, 0, h, dt, so, full(v), None, full(e), full(d), [],
                               np.zeros((nsteps, 0)), [], nsteps, state)
    c = np.cos(phase - nsteps * om * dt)
    sl = tuple(slice(nsteps * r, m - nsteps * r) for m in shape)
    assert c[sl].size > 100
    assert np.max(np.abs(st[1][sl] - ab[0] * c[sl])) < 1e-11
    assert np.max(np.abs(st[3][sl] - ab[1] * c[sl])) < 1e-11
