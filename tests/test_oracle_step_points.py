"""Pins for the oracle's one-step entries (``*_step_points``).

Every one-step GPU parity test compares the library with
``acoustic_step_points``, ``vti_step_points`` or ``tti_step_points``: one
source-free step of Algorithm 1 evaluated at listed flat indices of the
padded array, from an FP32 state.  Here each of them must equal, bit for bit
and at every point (listed in a scrambled order), one step of the pinned full
forward run (``*_forward`` with no sources or receivers) started from the same
FP32 state up-cast to FP64.  Grids are non-cubic so that a wrong flat-index
decode, a swapped time level or a swapped field shows.
"""
import numpy as np
import pytest

import oracle


def _fields(rng, shape, aniso=False, tilt=False):
    vel = (1500 + 1500 * rng.random(shape)).astype(np.float32)
    eta = np.zeros(shape, np.float32)
    eta[..., :2] = 40.0 * rng.random(shape[:-1] + (2,))
    out = {"vel": vel, "eta": eta}
    if aniso:
        eps = (0.3 * rng.random(shape)).astype(np.float32)
        out["eps"] = eps
        out["delta"] = (eps * rng.random(shape)).astype(np.float32)
    if tilt:
        out["theta"] = (0.8 * rng.random(shape)).astype(np.float32)
        out["phi"] = (1.5 * rng.random(shape)).astype(np.float32)
    return out


def _state(rng, shape, k):
    return [rng.standard_normal(shape).astype(np.float32) for _ in range(k)]


def _scrambled(rng, n):
    return rng.permutation(n).astype(np.int64)


def check_acoustic(ndim, so):
    rng = np.random.default_rng(100 + 10 * ndim + so)
    shape = (9, 11) if ndim == 2 else (9, 7, 11)
    h = (10.0, 12.5, 15.0) if ndim == 3 else (10.0, 10.0, 15.0)
    f = _fields(rng, shape)
    up, uc = _state(rng, shape, 2)
    dt = 1e-3
    _, _, nxt = oracle.acoustic_forward(ndim, 0, h, dt, so, f["vel"], f["eta"], [], [], [], 1,
                                        u_prev=up.astype(np.float64), u_cur=uc.astype(np.float64))
    pts = _scrambled(rng, up.size)
    got = oracle.acoustic_step_points(ndim, h, dt, so, f["vel"], f["eta"], up, uc, pts)
    assert np.array_equal(got, nxt.ravel()[pts])


def check_vti(ndim, so):
    rng = np.random.default_rng(200 + 10 * ndim + so)
    shape = (9, 11) if ndim == 2 else (9, 7, 11)
    h = (10.0, 12.5, 15.0) if ndim == 3 else (10.0, 10.0, 15.0)
    f = _fields(rng, shape, aniso=True)
    st = _state(rng, shape, 4)
    dt = 1e-3
    _, nxt = oracle.vti_forward(ndim, 0, h, dt, so, f["vel"], f["eta"], f["eps"], f["delta"], [],
                                [], [], 1, state=[s.astype(np.float64) for s in st])
    pts = _scrambled(rng, st[0].size)
    gp, gr = oracle.vti_step_points(ndim, h, dt, so, f["vel"], f["eta"], f["eps"], f["delta"],
                                    st, pts)
    assert np.array_equal(gp, nxt[1].ravel()[pts])
    assert np.array_equal(gr, nxt[3].ravel()[pts])


def check_tti(so):
    rng = np.random.default_rng(300 + so)
    shape = (9, 7, 11)
    h = (10.0, 12.5, 15.0)
    f = _fields(rng, shape, aniso=True, tilt=True)
    st = _state(rng, shape, 4)
    dt = 1e-3
    _, nxt = oracle.tti_forward(0, h, dt, so, f["vel"], f["eta"], f["eps"], f["delta"],
                                f["theta"], f["phi"], [], [], [], 1,
                                state=[s.astype(np.float64) for s in st])
    pts = _scrambled(rng, st[0].size)
    gp, gr = oracle.tti_step_points(h, dt, so, f["vel"], f["eta"], f["eps"], f["delta"],
                                    f["theta"], f["phi"], st, pts)
    assert np.array_equal(gp, nxt[1].ravel()[pts])
    assert np.array_equal(gr, nxt[3].ravel()[pts])


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("so", [2, 8])
def test_acoustic_step_points_equal_one_forward_step(ndim, so):
    check_acoustic(ndim, so)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("so", [4, 8])
def test_vti_step_points_equal_one_forward_step(ndim, so):
    check_vti(ndim, so)


@pytest.mark.parametrize("so", [2, 8])
def test_tti_step_points_equal_one_forward_step(so):
    check_tti(so)
