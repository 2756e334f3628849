"""Pins for the oracle's TTI solver (Eq. (TTI) with the operators of
Eq. (DiffOp)).

  * the three rotated operators sum to the Laplacian (an identity that holds
    only with the d2/dxdy coefficient of G_ybar_ybar read as -sin(2 phi));
  * each operator equals (n . grad)^2 for the rotated axis n, assembled as a
    dense matrix from independently solved weights (so the printed
    coefficient table is checked against its geometric definition);
  * epsilon = delta = 0 reduces the system to the acoustic equation;
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


def rotated_axes(theta, phi):
    """Unit vectors xbar, ybar, zbar (rows) of the tilted frame."""
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    xb = np.stack([ct * cp, ct * sp, -st])
    yb = np.stack([-sp, cp, np.zeros_like(sp)])
    zb = np.stack([st * cp, st * sp, ct])
    return xb, yb, zb


@pytest.mark.parametrize("so", [2, 4, 8])
def test_rotated_operators_sum_to_laplacian(so):
    rng = np.random.default_rng(so)
    shape = (9, 10, 11)
    h = (10.0, 12.0, 8.0)
    f = rng.standard_normal(shape)
    theta = rng.uniform(0, np.pi / 2, shape).astype(np.float32)
    phi = rng.uniform(0, np.pi, shape).astype(np.float32)
    gxx, gyy, gzz, lap = oracle.tti_operators(h, so, f, theta, phi)
    assert rel(gxx + gyy + gzz, lap) < 1e-13
    # the operators are genuinely different from each other
    assert rel(gzz, lap) > 0.1 and rel(gxx, lap) > 0.1


@pytest.mark.parametrize("so", [2, 4])
def test_rotated_operators_dense_geometric(so):
    """G_nn = sum_ab n_a n_b D_ab with D_aa the second-derivative matrix and
    D_ab = D1_a D1_b, for n = xbar, ybar, zbar of the tilted frame."""
    rng = np.random.default_rng(40 + so)
    shape = (5, 6, 7)
    h = (10.0, 12.0, 8.0)
    N = int(np.prod(shape))
    theta = rng.uniform(0, np.pi / 2, shape).astype(np.float32)
    phi = rng.uniform(0, np.pi, shape).astype(np.float32)
    f = rng.standard_normal(shape)
    D2 = bf.second_derivative_ops(shape, so, h)
    D1 = bf.first_derivative_ops(shape, so, h)
    axes = rotated_axes(theta.astype(np.float64).ravel(), phi.astype(np.float64).ravel())
    got = oracle.tti_operators(h, so, f, theta, phi)[:3]
    for n, g in zip(axes, got):
        G = np.zeros((N, N))
        for a in range(3):
            for b in range(3):
                Dab = D2[a] if a == b else D1[a] @ D1[b]
                G += (n[a] * n[b])[:, None] * Dab
        assert rel(g.ravel(), G @ f.ravel()) < 1e-11


def test_dense_bruteforce_tti_run():
    """Full TTI run (damping, source into p and r, receivers on p) against a
    dense block-matrix leapfrog built from the geometric operators."""
    so, nbl = 4, 1
    rng = np.random.default_rng(77)
    shape = (6, 5, 7)
    h = (10.0, 11.0, 9.0)
    N = int(np.prod(shape))
    vel = (1800 + 600 * rng.random(shape)).astype(np.float32)
    eta = (15 * rng.random(shape)).astype(np.float32)
    eps = (0.3 * rng.random(shape)).astype(np.float32)
    delta = np.minimum(0.1 * rng.random(shape), eps).astype(np.float32)
    theta = rng.uniform(0, np.pi / 4, shape).astype(np.float32)
    phi = rng.uniform(0, np.pi / 2, shape).astype(np.float32)
    dt = 0.3 * oracle.cfl_dt(3, so, h, float(vel.max()) * np.sqrt(1.6))
    src = np.array([[20.0, 15.0, 13.0]])
    rec = np.array([[0.0, 0.0, 0.0], [30.0, 22.0, 27.0]])
    nt = 10
    q = rng.standard_normal((nt, 1)).astype(np.float32)
    tr, st = oracle.tti_forward(nbl, h, dt, so, vel, eta, eps, delta, theta, phi, src, q, rec, nt)

    D2 = bf.second_derivative_ops(shape, so, h)
    D1 = bf.first_derivative_ops(shape, so, h)
    xb, yb, zb = rotated_axes(theta.astype(np.float64).ravel(), phi.astype(np.float64).ravel())

    def G(n):
        M = np.zeros((N, N))
        for a in range(3):
            for b in range(3):
                M += (n[a] * n[b])[:, None] * (D2[a] if a == b else D1[a] @ D1[b])
        return M

    Hm = G(xb) + G(yb)
    Zm = G(zb)
    A = dt * dt * vel.astype(np.float64).ravel() ** 2
    s = 0.5 * dt * eta.astype(np.float64).ravel()
    e2 = 1 + 2 * eps.astype(np.float64).ravel()
    sd = np.sqrt(1 + 2 * delta.astype(np.float64).ravel())
    S = bf.interp_row(shape, nbl, h, src[0], 3)
    R = np.array([bf.interp_row(shape, nbl, h, c, 3) for c in rec])
    hp = h[0] * h[1] * h[2]
    pp = pc = rp = rc = np.zeros(N)
    tb = np.zeros((nt, 2))
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


def test_isotropic_limit_equals_acoustic():
    """epsilon = delta = 0: p and r obey the same equation as the acoustic
    field (the operators sum to the Laplacian), whatever the angles."""
    so, nbl = 4, 4
    rng = np.random.default_rng(5)
    shape = (20, 18, 22)
    h = (10.0, 10.0, 10.0)
    vel = (2000 + 500 * rng.random(shape)).astype(np.float32)
    eta = (10 * rng.random(shape)).astype(np.float32)
    z = np.zeros(shape, np.float32)
    theta = rng.uniform(0, np.pi / 4, shape).astype(np.float32)
    phi = rng.uniform(0, np.pi / 2, shape).astype(np.float32)
    dt = 0.4 * oracle.cfl_dt(3, so, h, float(vel.max()))
    src = np.array([[70.0, 60.0, 55.0]])
    rec = np.array([[10.0, 20.0, 30.0], [100.0, 80.0, 90.0]])
    nt = 30
    q = ricker(30.0, dt, nt)[:, None]
    tr, st = oracle.tti_forward(nbl, h, dt, so, vel, eta, z, z, theta, phi, src, q, rec, nt)
    ta, _, ua = oracle.acoustic_forward(3, nbl, h, dt, so, vel, eta, src, q, rec, nt)
    assert rel(st[1], ua) < 1e-11
    assert rel(st[3], ua) < 1e-11
    assert rel(tr, ta) < 1e-11


def _symbols(so, k, h):
    """Per-axis second-derivative symbols X2_a >= 0 and first-derivative
    symbols s_a of the stencils for wavenumber k."""
    w2 = oracle.weights_d2(so)
    w1 = oracle.weights_d1(so)
    r = so // 2
    X2 = np.array([-(w2[0] + 2 * sum(w2[j] * np.cos(j * k[a] * h[a]) for j in range(1, r + 1)))
                   / h[a] ** 2 for a in range(3)])
    s1 = np.array([2 * sum(w1[j] * np.sin(j * k[a] * h[a]) for j in range(1, r + 1)) / h[a]
                   for a in range(3)])
    return X2, s1


@pytest.mark.parametrize("so", [2, 4, 8])
def test_tti_plane_wave_exact(so):
    """In a homogeneous medium, [p; r] = [a; b] cos(k.x - w t) is an exact
    solution of the scheme when [a; b] is an eigenvector of the symbol
    M = [[(1+2e) H, sqrt(1+2d) Z], [sqrt(1+2d) H, Z]] and
    4 sin^2(w dt/2) = dt^2 v^2 mu; checked where the walls have not reached."""
    r = so // 2
    h = (10.0, 12.0, 9.0)
    shape = (36, 34, 38)
    # the oracle reads FP32 inputs, so the symbol uses the rounded values
    v, e, d, th, ph = (float(np.float32(c)) for c in (2500.0, 0.25, 0.1, 0.6, 1.1))
    k = np.array([2 * np.pi / (7.3 * h[0]), -2 * np.pi / (9.1 * h[1]), 2 * np.pi / (6.7 * h[2])])
    X2, s1 = _symbols(so, k, h)
    n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    K = np.outer(s1, s1)
    np.fill_diagonal(K, X2)
    Z = n @ K @ n
    Hs = X2.sum() - Z
    M = np.array([[(1 + 2 * e) * Hs, np.sqrt(1 + 2 * d) * Z], [np.sqrt(1 + 2 * d) * Hs, Z]])
    mu, vec = np.linalg.eig(M)
    i = int(np.argmax(mu.real))                 # the quasi-P mode
    mu, ab = mu[i].real, vec[:, i].real
    dt = 0.4 * oracle.cfl_dt(3, so, h, v * np.sqrt(1 + 2 * e))
    om = 2.0 / dt * np.arcsin(0.5 * v * dt * np.sqrt(mu))
    z, y, x = np.meshgrid(np.arange(shape[0]) * h[2], np.arange(shape[1]) * h[1],
                          np.arange(shape[2]) * h[0], indexing="ij")
    phase = k[0] * x + k[1] * y + k[2] * z
    full = lambda c: np.full(shape, c, np.float32)
    state = (ab[0] * np.cos(phase + om * dt), ab[0] * np.cos(phase),
             ab[1] * np.cos(phase + om * dt), ab[1] * np.cos(phase))
    nsteps = 12 // r
    _, st = oracle.tti_forward(0, h, dt, so, full(v), None, full(e), full(d), full(th), full(ph),
                               [], np.zeros((nsteps, 0)), [], nsteps, state)
    c = np.cos(phase - nsteps * om * dt)
    sl = tuple(slice(nsteps * r, m - nsteps * r) for m in shape)
    assert c[sl].size > 100
    assert np.max(np.abs(st[1][sl] - ab[0] * c[sl])) < 1e-11
    assert np.max(np.abs(st[3][sl] - ab[1] * c[sl])) < 1e-11


@pytest.mark.parametrize("so", [2, 4, 8, 16])
def test_tti_symbol_bounded_by_scaled_laplacian(so):
    """The stability reading used for TTI: with 0 <= delta <= epsilon the
    symbol's eigenvalues are real, non-negative and at most (1 + 2 eps) times
    the Laplacian symbol, because the second-derivative symbol dominates the
    square of the first-derivative symbol on every axis (X2 >= s^2)."""
    rng = np.random.default_rng(so)
    h = (10.0, 12.0, 9.0)
    for _ in range(400):
        k = rng.uniform(-np.pi, np.pi, 3) / np.array(h)
        X2, s1 = _symbols(so, k, h)
        # X2 comes from a cancelling sum: rounding ~1e-16 sum|w| / h^2
        S = np.abs(oracle.weights_d2(so)).sum() * 2 / np.array(h) ** 2
        assert np.all(X2 - s1 ** 2 >= -1e-14 * S)
        th, ph = rng.uniform(0, np.pi / 2), rng.uniform(0, np.pi)
        e = rng.uniform(0, 0.3)
        d = rng.uniform(0, e)
        n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
        K = np.outer(s1, s1)
        np.fill_diagonal(K, X2)
        Z = n @ K @ n
        Hs = X2.sum() - Z
        assert Z >= -1e-9 * X2.sum() and Hs >= -1e-9 * X2.sum()
        M = np.array([[(1 + 2 * e) * Hs, np.sqrt(1 + 2 * d) * Z], [np.sqrt(1 + 2 * d) * Hs, Z]])
        mu = np.linalg.eigvals(M)
        assert np.all(np.abs(mu.imag) < 1e-9 * X2.sum())
        assert mu.real.max() <= (1 + 2 * e) * X2.sum() * (1 + 1e-12)
        assert mu.real.min() >= -1e-9 * X2.sum()
