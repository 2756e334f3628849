"""More pins for the oracle's acoustic solver (Eq. (Acou), Algorithm 1):

  * the step's spatial operator converges to the Laplacian at order h^so on
    a smooth field (weights, 1/h^2 scaling and the sum over axes together);
  * the leapfrog time stepping converges at order dt^2 on an exact
    eigenvector of the second-order Dirichlet Laplacian (no spatial error);
  * source-receiver reciprocity: the scheme is symmetric in space for every
    frequency (diagonal mass and damping, symmetric Laplacian), so swapping a
    source and a receiver leaves the trace unchanged, off-grid points and
    damping included;
  * receiver interpolation reproduces affine fields exactly, which fixes the
    coordinate convention (metres from the physical origin, (x, y, z) order,
    the layer offset).
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("so", [2, 4, 6, 8])
def test_space_order_of_the_step(so):
    """One undamped step from u^{n-1} = u^n = f gives u^{n+1} = f + A L f; on
    f = sin(kx x + kz z) the error of L f against -|k|^2 f must fall like
    h^so when h is halved (2D, FP64 state)."""
    errs = []
    for m in (1, 2):
        h = 8.0 / m
        n = 48 * m
        k = np.array([2 * np.pi / 120.0, 2 * np.pi / 95.0])  # (x, z): 12-15 points per wavelength at h = 8
        z, x = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="ij")
        f = np.sin(k[0] * x + k[1] * z)
        v = 1000.0
        vel = np.full((n, n), v, dtype=np.float32)
        dt = 0.5 * oracle.cfl_dt(2, so, (h, 1.0, h), v)
        _, _, u1 = oracle.acoustic_forward(2, 0, (h, 1.0, h), dt, so, vel, None, [],
                                           np.zeros((1, 0)), [], 1, f, f)
        lap = (u1 - f) / (dt * dt * v * v)
        inner = slice(so, n - so)
        e = lap[inner, inner] + (k @ k) * f[inner, inner]
        errs.append(np.max(np.abs(e)))
    order = np.log2(errs[0] / errs[1])
    assert abs(order - so) < 0.3, (so, errs, order)


def test_time_order_of_leapfrog():
    """phi = sin(pi p (iz+1)/(nz+1)) sin(pi q (ix+1)/(nx+1)) is an eigenvector
    of the second-order Laplacian with zero ghosts (eigenvalue -lam), so the
    exact-in-time solution from u(0) = phi, u_t(0) = 0 is cos(v sqrt(lam) t)
    phi.  Started from that solution at t = -dt and 0, the scheme's error at a
    fixed time must fall by 4 when dt is halved."""
    nz, nx, h, v = 24, 30, 10.0, 1500.0
    p, q = 3, 2
    tz = np.pi * p / (nz + 1)
    tx = np.pi * q / (nx + 1)
    phi = np.outer(np.sin(tz * (np.arange(nz) + 1)), np.sin(tx * (np.arange(nx) + 1)))
    lam = 4.0 / h ** 2 * (np.sin(tz / 2) ** 2 + np.sin(tx / 2) ** 2)
    om = v * np.sqrt(lam)
    # 1.25 periods: cos(om T) = 0, where a phase error shows at first order
    # (at an extremum of the cosine it would show only at second order)
    T = 1.25 * 2 * np.pi / om
    vel = np.full((nz, nx), v, dtype=np.float32)
    errs = []
    for steps in (80, 160, 320):
        dt = T / steps
        assert v * dt / h < 0.5              # inside the CFL bound of order 2
        _, _, u = oracle.acoustic_forward(2, 0, (h, 1.0, h), dt, 2, vel, None, [],
                                          np.zeros((steps, 0)), [], steps,
                                          np.cos(om * dt) * phi, phi)
        errs.append(np.max(np.abs(u - np.cos(om * T) * phi)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, (errs, r1, r2)


def test_reciprocity_off_grid_with_damping():
    """Trace of a source at a recorded at b equals the trace of a source at b
    recorded at a (3D, heterogeneous velocity and damping, so 8, both points
    off the grid)."""
    rng = np.random.default_rng(31)
    nbl = 4
    phys = (20, 18, 16)                       # (x, y, z)
    shape = (phys[2] + 2 * nbl, phys[1] + 2 * nbl, phys[0] + 2 * nbl)
    h = (10.0, 12.0, 9.0)
    vel = (1500 + 1500 * rng.random(shape)).astype(np.float32)
    # damping everywhere and different at every corner, so that the 1/(1+s)
    # of the injection is exercised at both points
    eta = (20 + 40 * rng.random(shape)).astype(np.float32)
    dt = 0.4 * oracle.cfl_dt(3, 8, h, float(vel.max()))
    nt = 70
    q = rng.standard_normal((nt, 1)).astype(np.float32)
    a = np.array([[37.3, 41.9, 30.2]])
    b = np.array([[121.7, 150.2, 101.4]])
    dab, _, _ = oracle.acoustic_forward(3, nbl, h, dt, 8, vel, eta, a, q, b, nt)
    dba, _, _ = oracle.acoustic_forward(3, nbl, h, dt, 8, vel, eta, b, q, a, nt)
    assert np.max(np.abs(dab)) > 0
    assert np.linalg.norm(dab - dba) / np.linalg.norm(dab) < 1e-11


def test_reciprocity_fails_for_a_different_receiver():
    """Control for the reciprocity pin: moving the receiver by a fraction of
    a cell changes the trace well beyond rounding."""
    rng = np.random.default_rng(32)
    shape = (20, 22, 24)
    h = (10.0, 10.0, 10.0)
    vel = (1500 + 1000 * rng.random(shape)).astype(np.float32)
    dt = 0.4 * oracle.cfl_dt(3, 4, h, float(vel.max()))
    q = rng.standard_normal((40, 1)).astype(np.float32)
    a = np.array([[60.0, 70.0, 80.0]])
    b = np.array([[150.0, 120.0, 110.0]])
    dab, _, _ = oracle.acoustic_forward(3, 0, h, dt, 4, vel, None, a, q, b, 40)
    dba, _, _ = oracle.acoustic_forward(3, 0, h, dt, 4, vel, None, b, q, a + 2.5, 40)
    assert np.linalg.norm(dab - dba) / np.linalg.norm(dab) > 1e-3


@pytest.mark.parametrize("ndim", [2, 3])
def test_receivers_exact_on_affine_fields(ndim):
    """With zero velocity a step maps (u^{n-1}, u^n) = (f, f) to f, so the
    recorded values are the multilinear interpolation of f; for an affine f
    of the physical coordinates they must equal f at the receiver."""
    rng = np.random.default_rng(40 + ndim)
    nbl = 3
    if ndim == 2:
        phys = (17, 1, 13)
        shape = (phys[2] + 2 * nbl, phys[0] + 2 * nbl)
        h = (7.0, 1.0, 11.0)
    else:
        phys = (15, 12, 10)
        shape = (phys[2] + 2 * nbl, phys[1] + 2 * nbl, phys[0] + 2 * nbl)
        h = (7.0, 9.0, 11.0)
    c = np.array([0.3, -1.7, 2.9, 0.45])      # f = c0 + c1 x + c2 y + c3 z, metres
    hs = h if ndim == 3 else (h[0], h[2])
    axes = [(np.arange(n) - nbl) * hh for n, hh in zip(shape[::-1], hs)]
    if ndim == 2:
        z, x = np.meshgrid(axes[1], axes[0], indexing="ij")
        f = c[0] + c[1] * x + c[3] * z
        span = np.array([(phys[0] - 1) * h[0], (phys[2] - 1) * h[2]])
    else:
        z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        f = c[0] + c[1] * x + c[2] * y + c[3] * z
        span = np.array([(phys[0] - 1) * h[0], (phys[1] - 1) * h[1], (phys[2] - 1) * h[2]])
    rec = rng.random((25, ndim)) * span
    vel = np.zeros(shape, np.float32)
    tr, _, _ = oracle.acoustic_forward(ndim, nbl, h, 1e-3, 4, vel, None, [], np.zeros((1, 0)),
                                       rec, 1, f, f)
    if ndim == 2:
        exact = c[0] + c[1] * rec[:, 0] + c[3] * rec[:, 1]
    else:
        exact = c[0] + c[1] * rec[:, 0] + c[2] * rec[:, 1] + c[3] * rec[:, 2]
    assert np.max(np.abs(tr[0] - exact)) < 1e-10 * np.max(np.abs(exact))
