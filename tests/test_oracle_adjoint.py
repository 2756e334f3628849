"""Pins for the oracle's adjoint and velocity gradient of the acoustic forward
map (Eq. (Acou) stepped by Algorithm 1, zero initial state).

The forward map q -> d (wavelet to traces) is linear; the oracle's adjoint
runs the transposed recurrence.  It is checked against
  * the transpose of the dense matrix of the map, assembled column by column
    from the dense-matrix brute force of the forward run (independent
    weights, explicit Kronecker operators);
  * the dot-product identity <F q, d> = <q, F^T d> with the oracle forward.
The gradient of J = 1/2 |F(m) q - dobs|^2 with respect to m = 1/v^2 is checked
against central differences of J, point by point on a tiny grid (brute
force) and along a smooth direction on a 3D grid, and vanishes at dobs = d.
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_acoustic import brute_acoustic, rel


def _small_2d(so, seed, nt=14):
    rng = np.random.default_rng(seed)
    nz, nx, nbl = 11, 13, 3
    h = (10.0, 1.0, 8.0)
    vel = (1500 + 600 * rng.random((nz, nx))).astype(np.float32)
    eta = np.zeros((nz, nx), np.float32)
    eta[:nbl], eta[-nbl:], eta[:, :nbl], eta[:, -nbl:] = 40.0, 40.0, 25.0, 25.0
    dt = 0.6 * oracle.cfl_dt(2, so, h, float(vel.max()))
    src = np.array([[31.0, 17.3], [0.0, 8.0]])
    rec = np.array([[13.1, 40.0], [50.0, 7.5], [-24.0, -20.0], [44.4, 0.0]])
    return dict(ndim=2, nbl=nbl, h=h, dt=dt, vel=vel, eta=eta, src=src, rec=rec, nt=nt,
                shape=(nz, 1, nx))


@pytest.mark.parametrize("so", [2, 4, 8])
def test_adjoint_equals_dense_transpose(so):
    c = _small_2d(so, 40 + so, nt=10)
    nt, ns, nr = c["nt"], len(c["src"]), len(c["rec"])
    # dense matrix of the map: one brute-force run per (time, source) impulse
    F = np.zeros((nt * nr, nt * ns))
    for t in range(nt):
        for s in range(ns):
            q = np.zeros((nt, ns), np.float32)
            q[t, s] = 1.0
            tr, _, _ = brute_acoustic(2, c["shape"], c["nbl"], c["h"], c["dt"], so, c["vel"],
                                      c["eta"], c["src"], q, c["rec"], nt)
            F[:, t * ns + s] = tr.ravel()
    rng = np.random.default_rng(so)
    d = rng.standard_normal((nt, nr))
    q_adj = oracle.acoustic_adjoint(2, c["nbl"], c["h"], c["dt"], so, c["vel"], c["eta"],
                                    c["src"], c["rec"], d, nt)
    assert rel(q_adj.ravel(), F.T @ d.ravel()) < 1e-10


@pytest.mark.parametrize("ndim,so", [(2, 4), (2, 16), (3, 2), (3, 8)])
def test_adjoint_dot_product(ndim, so):
    rng = np.random.default_rng(7 * so + ndim)
    if ndim == 2:
        c = _small_2d(so, so, nt=40)
        vel, eta = c["vel"], c["eta"]
    else:
        nz, ny, nx = 12, 10, 14
        vel = (1700 + 500 * rng.random((nz, ny, nx))).astype(np.float32)
        eta = (15 * rng.random((nz, ny, nx))).astype(np.float32)
        h = (10.0, 12.0, 9.0)
        c = dict(nbl=2, h=h, dt=0.5 * oracle.cfl_dt(3, so, h, float(vel.max())),
                 src=np.array([[11.0, 5.0, 3.3], [40.0, 20.0, 10.0]]),
                 rec=np.array([[1.0, 2.0, 3.0], [-10.0, -14.0, -8.0], [60.0, 30.0, 27.0]]),
                 nt=30)
    nt, ns, nr = c["nt"], len(c["src"]), len(c["rec"])
    q = rng.standard_normal((nt, ns)).astype(np.float32)
    d = rng.standard_normal((nt, nr))
    tr, _, _ = oracle.acoustic_forward(ndim, c["nbl"], c["h"], c["dt"], so, vel, eta, c["src"],
                                       q, c["rec"], nt)
    q_adj = oracle.acoustic_adjoint(ndim, c["nbl"], c["h"], c["dt"], so, vel, eta, c["src"],
                                    c["rec"], d, nt)
    lhs = float(np.sum(tr * d))
    rhs = float(np.sum(q.astype(np.float64) * q_adj))
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), np.linalg.norm(tr) * np.linalg.norm(d))


def _misfit(c, so, vel, q, dobs):
    return oracle.acoustic_misfit(c["ndim"], c["nbl"], c["h"], c["dt"], so, vel, c["eta"],
                                  c["src"], q, c["rec"], dobs, c["nt"])


def _observed(c, so, q, seed):
    """Data of a perturbed model (a smooth bump added to the velocity)."""
    rng = np.random.default_rng(seed)
    v = c["vel"].astype(np.float64) * (1.0 + 0.05 * rng.random(c["vel"].shape))
    tr, _, _ = oracle.acoustic_forward(c["ndim"], c["nbl"], c["h"], c["dt"], so,
                                       v.astype(np.float32), c["eta"], c["src"], q, c["rec"],
                                       c["nt"])
    return tr


@pytest.mark.parametrize("so", [2, 4])
def test_gradient_pointwise_central_differences(so):
    """Brute force: perturb m at every point of a tiny damped grid."""
    c = _small_2d(so, 90 + so, nt=30)
    from workloads import ricker
    q = np.stack([ricker(40.0, c["dt"], c["nt"]), 0.5 * ricker(30.0, c["dt"], c["nt"])],
                 axis=1).astype(np.float32) * 1e3
    dobs = _observed(c, so, q, 5)
    g, J = oracle.acoustic_gradient(2, c["nbl"], c["h"], c["dt"], so, c["vel"], c["eta"],
                                    c["src"], q, c["rec"], dobs, c["nt"])
    assert J == pytest.approx(_misfit(c, so, c["vel"], q, dobs), rel=1e-13)
    m = 1.0 / c["vel"].astype(np.float64) ** 2
    eps = 1e-3
    fd = np.zeros_like(g)
    for i in range(m.size):
        vp, vm = c["vel"].copy(), c["vel"].copy()
        vp.flat[i] = np.float32(1.0 / np.sqrt(m.flat[i] * (1 + eps)))
        vm.flat[i] = np.float32(1.0 / np.sqrt(m.flat[i] * (1 - eps)))
        dm = 1.0 / float(vp.flat[i]) ** 2 - 1.0 / float(vm.flat[i]) ** 2  # realised in FP32
        fd.flat[i] = (_misfit(c, so, vp, q, dobs) - _misfit(c, so, vm, q, dobs)) / dm
    assert rel(g, fd) < 1e-4
    assert np.abs(g).max() > 0


def test_gradient_directional_3d():
    rng = np.random.default_rng(3)
    nz, ny, nx, nbl, so = 14, 12, 16, 3, 4
    h = (10.0, 10.0, 10.0)
    vel = (2000 + 300 * rng.random((nz, ny, nx))).astype(np.float32)
    eta = np.zeros_like(vel)
    eta[:nbl] = eta[-nbl:] = 30.0
    c = dict(ndim=3, nbl=nbl, h=h, dt=0.5 * oracle.cfl_dt(3, so, h, 2300.0), vel=vel, eta=eta,
             src=np.array([[40.0, 35.0, 20.0]]),
             rec=np.array([[10.0, 10.0, 0.0], [80.0, 30.0, 1.0], [50.0, 55.0, 70.0]]), nt=60)
    from workloads import ricker
    q = (1e4 * ricker(60.0, c["dt"], c["nt"])).astype(np.float32)[:, None]
    dobs = _observed(c, so, q, 6)
    g, J = oracle.acoustic_gradient(3, nbl, h, c["dt"], so, vel, eta, c["src"], q, c["rec"],
                                    dobs, c["nt"])
    m = 1.0 / vel.astype(np.float64) ** 2
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    bump = np.exp(-((z - 7) ** 2 + (y - 6) ** 2 + (x - 8) ** 2) / 8.0)
    # central differences converge quadratically to <g, dm>
    for eps, tol in ((1e-3, 1e-5), (1e-4, 1e-7)):
        vp = (1.0 / np.sqrt(m * (1 + eps * bump))).astype(np.float32)
        vm = (1.0 / np.sqrt(m * (1 - eps * bump))).astype(np.float32)
        dmp = 1.0 / vp.astype(np.float64) ** 2 - m
        dmm = 1.0 / vm.astype(np.float64) ** 2 - m
        lhs = _misfit(c, so, vp, q, dobs) - _misfit(c, so, vm, q, dobs)
        rhs = float(np.sum(g * (dmp - dmm)))
        assert abs(lhs - rhs) < tol * abs(rhs)


def test_gradient_vanishes_at_the_data_model():
    c = _small_2d(4, 12, nt=20)
    from workloads import ricker
    q = (1e3 * ricker(40.0, c["dt"], c["nt"])).astype(np.float32)[:, None].repeat(2, 1)
    d, _, _ = oracle.acoustic_forward(2, c["nbl"], c["h"], c["dt"], 4, c["vel"], c["eta"],
                                      c["src"], q, c["rec"], c["nt"])
    g, J = oracle.acoustic_gradient(2, c["nbl"], c["h"], c["dt"], 4, c["vel"], c["eta"],
                                    c["src"], q, c["rec"], d, c["nt"])
    assert J == 0.0 and np.all(g == 0.0)
