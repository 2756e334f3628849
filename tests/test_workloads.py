"""The seeded input generators: time-step literals re-derived from the
oracle's CFL bound, shapes, ranges and the structure each recipe states."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("key", sorted(W.DT))
def test_time_step_literals_are_0p4_cfl(key):
    name, so = key
    h = {"acoustic_2d": 10.0, "acoustic_3d": 10.0, "tti_3d": 12.5, "fwi_3d": 15.0}[name]
    ndim = 2 if name == "acoustic_2d" else 3
    vmax = W.VMAX[name] * (np.sqrt(1 + 2 * W.EPS_MAX) if name == "tti_3d" else 1.0)
    assert W.DT[key] == pytest.approx(0.4 * oracle.cfl_dt(ndim, so, (h, h, h), vmax), rel=1e-14)


def test_acoustic_3d_replica_structure():
    p = W.acoustic_3d(so=8, phys=48, nbl=6, nt=10, receivers="surface")
    assert p.vel.shape == (60, 60, 60) and p.vel.dtype == np.float32
    assert p.eta.shape == p.vel.shape
    inner = p.eta[6:-6, 6:-6, 6:-6]
    assert np.all(inner == 0) and p.eta.max() > 0
    assert p.vel.max() <= W.VMAX["acoustic_3d"] * (1 + 1e-6)
    assert p.rec.shape == (48 * 48, 3)


def test_tti_delta_below_epsilon():
    p = W.tti_3d(so=8, phys=32, nbl=4, nt=4)
    assert np.all(p.delta <= p.eps)
    assert p.eps.max() <= W.EPS_MAX + 1e-6
    assert float(p.theta.max()) <= np.deg2rad(45.0) + 1e-6


def test_fwi_survey_layout():
    p = W.fwi_3d(so=8, phys=40, nbl=5, nt=20, nshots=16, receivers="surface")
    assert p.src.shape == (16, 3) and p.extra["nshots"] == 16
    assert np.all(p.src[:, 2] == 30.0)
    assert len(np.unique(p.src[:, 0])) == 4 and len(np.unique(p.src[:, 1])) == 4
    assert p.rec.shape == (40 * 40, 3)
    v0 = p.extra["vel_start"]
    assert v0.shape == p.vel.shape
    # the start model is smoother than the true one but keeps its range
    gt = np.abs(np.diff(p.vel.astype(np.float64), axis=0)).mean()
    g0 = np.abs(np.diff(v0.astype(np.float64), axis=0)).mean()
    assert g0 < gt
    assert v0.min() >= p.vel.min() - 1 and v0.max() <= p.vel.max() + 1
