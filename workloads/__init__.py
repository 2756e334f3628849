"""Seeded synthetic inputs for the finite-difference wave solver.

This module produces *inputs only*: grids, velocity / damping / anisotropy
fields, Ricker wavelets, source and receiver coordinates, and synthetic
wavefield states.  It holds none of the solver's arithmetic (no stencil
weights, no time stepping, no stability bound).  Both the GPU library's tests
and the CPU oracle consume what it returns, so the two see identical FP32
inputs.

Conventions shared with both solvers:
  * fields are float32, C-order ``[nz][ny][nx]`` (3D) or ``[nz][nx]`` (2D) on
    the padded array (physical points plus ``nbl`` layer points per side);
  * coordinates are float64 metres from the physical origin, ordered
    ``(x, y, z)`` in 3D and ``(x, z)`` in 2D;
  * the wavelet is ``[nt][nsrc]`` float32.

Workload recipes (the paper measures no run of its own, so every workload is
synthetic; random fields are white noise on a grid coarsened by ``COARSEN``,
Gaussian-smoothed there with the stated correlation length, trilinearly
upsampled, rescaled, and edge-replicated into the layer):

  * ``acoustic_2d``  -- 2D, 201 x 201 physical, h = 10 m, 20-point layer,
    v = 1500 m/s, 15 Hz Ricker at (1000, 1000) m, 101 receivers at z = 20 m,
    x = 0, 20, ..., 2000 m, 500 steps.
  * ``acoustic_3d``  -- 512^3 physical, h = 10 m, 40-point layer; v = 1500 m/s
    above z = 2560 m and 3500 m/s below, times (1 + p) with p a smooth random
    field (correlation 20 points) scaled to max|p| = 0.05; 10 Hz Ricker at
    (2560, 2560, 20) m; 512 x 512 receivers at z = 20 m on every physical
    (x, y) node; 1000 steps.  ``phys`` shrinks it to a replica of the same
    structure (interfaces and source at the same relative positions).
  * ``tti_3d``       -- 384^3 physical, h = 12.5 m, 40-point layer; v in four
    layers 1.5 / 2.3 / 3.2 / 4.0 km/s times (1 + p), |p| <= 0.05; Thomsen
    epsilon in [0, 0.3], delta in [0, 0.1] then delta <- min(delta, epsilon);
    tilt in [0, 45] deg, azimuth in [0, 90] deg; all smooth (correlation 16
    points); 10 Hz Ricker at the centre (x, y) and z = 25 m; 800 steps.
  * ``vti_3d``       -- the ``tti_3d`` model without tilt and azimuth (VTI
    pseudo-acoustic), same grid, time steps and source.
  * ``learned_model`` -- one training/evaluation model of the coarse-grid
    correction: random layered velocity (2-5 layers between 1.5 and 3.4 km/s,
    random interface depths) times (1 + p), |p| <= 0.05 (correlation 20 fine
    points); fine grid h = 10 m (256^3 physical, 40-point layer, space order
    16, dt = 0.4 CFL at 3675 m/s, 1000 steps), coarse grid h = 20 m (every
    second fine point, 20-point layer, space order 4, dt doubled, 500
    steps); 10 Hz Ricker source at a random on-grid (x, y) in the middle half
    at z = 40 m; receivers every 40 m at z = 20 m.
  * ``fwi_3d``       -- the many-shot survey of a full-waveform inversion:
    256^3 physical, h = 15 m, 40-point layer; true model of four layers
    1.5 / 2.0 / 2.7 / 3.5 km/s times (1 + p), |p| <= 0.05 (correlation 12
    points), start model the true model Gaussian-smoothed (sigma 10 points,
    applied on the grid coarsened by COARSEN and upsampled back);
    16 shots, one 8 Hz Ricker source each on a 4 x 4 grid at z = 30 m;
    256 x 256 receivers at z = 30 m shared by all shots; 1200 steps.

The time steps below are 0.4 times the CFL bound of Eq. (stability) at the
workload's maximum velocity (for TTI, at the maximum horizontal P velocity
v * sqrt(1 + 2 epsilon)); the tests re-derive each from the oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

COARSEN = 4  # random fields are drawn on a grid this many times coarser

# 0.4 x CFL time steps (seconds), keyed by (workload, space order).
DT = {
    ("acoustic_2d", 4): 1.632993161855452e-3,   # v_max 1500, h 10
    ("acoustic_3d", 4): 5.442176870748299e-4,   # v_max 3675, h 10
    ("acoustic_3d", 8): 4.929039709588243e-4,
    ("acoustic_3d", 12): 4.7257643591476446e-4,
    ("acoustic_3d", 16): 4.6117695896582113e-4,
    ("tti_3d", 4): 4.7057703276315164e-4,       # v_max 4200 * sqrt(1.6), h 12.5
    ("tti_3d", 8): 4.262068168671727e-4,
    ("fwi_3d", 4): 8.16326530612245e-4,         # v_max 3675, h 15
    ("fwi_3d", 8): 7.393559564382367e-4,
    ("fwi_3d", 16): 6.917654384487317e-4,
}
VMAX = {"acoustic_2d": 1500.0, "acoustic_3d": 3675.0, "tti_3d": 4200.0, "fwi_3d": 3675.0}
EPS_MAX = 0.3


@dataclass
class Problem:
    """One seeded problem: grid, model fields, wavelet and sparse points."""

    name: str
    ndim: int
    physics: str                 # "acoustic" or "tti"
    shape: tuple                 # physical points (nx, ny, nz); 2D has ny = 1
    spacing: tuple               # (hx, hy, hz) metres
    nbl: int
    so: int
    dt: float
    nt: int
    f0: float
    vel: np.ndarray
    eta: Optional[np.ndarray]
    src: np.ndarray              # [nsrc][ndim] float64 metres
    rec: np.ndarray              # [nrec][ndim] float64 metres
    wavelet: np.ndarray          # [nt][nsrc] float32
    eps: Optional[np.ndarray] = None
    delta: Optional[np.ndarray] = None
    theta: Optional[np.ndarray] = None
    phi: Optional[np.ndarray] = None
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def padded(self):
        """Padded field shape in array order ([nz][ny][nx] or [nz][nx])."""
        nx, ny, nz = self.shape
        b = self.nbl
        if self.ndim == 2:
            return (nz + 2 * b, nx + 2 * b)
        return (nz + 2 * b, ny + 2 * b, nx + 2 * b)

    @property
    def npoints(self):
        return int(np.prod(self.padded))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def ricker(f0: float, dt: float, nt: int, t0: Optional[float] = None) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 f^2 (t-t0)^2) exp(-pi^2 f^2 (t-t0)^2) sampled
    at t_n = n dt, t0 = 1/f0 by default; float32 [nt]."""
    t0 = 1.0 / f0 if t0 is None else t0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (np.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def damping_profile(padded_shape, nbl: int, spacing, vmax: float) -> np.ndarray:
    """Damping-rate field eta (1/s) that rises quadratically across the layer:
    eta = sum over axes of eta_max (d/nbl)^2, d = points into the layer,
    eta_max = 1.5 vmax ln(1000) / (nbl h).  Zero in the physical domain."""
    ndim = len(padded_shape)
    eta = np.zeros(padded_shape, dtype=np.float64)
    if nbl <= 0:
        return eta.astype(np.float32)
    hs = (spacing[2], spacing[0]) if ndim == 2 else (spacing[2], spacing[1], spacing[0])
    for ax, (n, h) in enumerate(zip(padded_shape, hs)):
        i = np.arange(n)
        d = np.maximum(np.maximum(nbl - i, i - (n - 1 - nbl)), 0).astype(np.float64)
        prof = 1.5 * vmax * np.log(1000.0) / (nbl * h) * (d / nbl) ** 2
        sh = [1] * ndim
        sh[ax] = n
        eta = eta + prof.reshape(sh)
    return eta.astype(np.float32)


def _gauss_kernel(sigma: float) -> np.ndarray:
    rad = max(1, int(np.ceil(3.0 * sigma)))
    x = np.arange(-rad, rad + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _smooth_axis(a: np.ndarray, sigma: float, axis: int) -> np.ndarray:
    k = _gauss_kernel(sigma)
    rad = (k.size - 1) // 2
    pad = [(0, 0)] * a.ndim
    pad[axis] = (rad, rad)
    ap = np.pad(a, pad, mode="reflect" if a.shape[axis] > rad else "edge")
    out = np.zeros_like(a)
    n = a.shape[axis]
    for j, kj in enumerate(k):
        sl = [slice(None)] * a.ndim
        sl[axis] = slice(j, j + n)
        out += kj * ap[tuple(sl)]
    return out


def _upsample_axis(a: np.ndarray, n: int, axis: int) -> np.ndarray:
    m = a.shape[axis]
    if m == 1:
        return np.repeat(a, n, axis=axis)
    pos = np.linspace(0.0, m - 1.0, n)
    i0 = np.minimum(np.floor(pos).astype(np.int64), m - 2)
    f = pos - i0
    sh = [1] * a.ndim
    sh[axis] = n
    f = f.reshape(sh)
    return np.take(a, i0, axis=axis) * (1.0 - f) + np.take(a, i0 + 1, axis=axis) * f


def smooth_random(shape, corr_pts: float, rng: np.random.Generator) -> np.ndarray:
    """Smooth random field on ``shape`` (array order), zero mean, max|.| = 1:
    white noise on a grid COARSEN times coarser, Gaussian-smoothed with
    sigma = corr_pts / COARSEN there, trilinearly upsampled."""
    cshape = tuple(max(2, int(np.ceil(n / COARSEN)) + 1) for n in shape)
    a = rng.standard_normal(cshape)
    for ax in range(a.ndim):
        a = _smooth_axis(a, max(corr_pts / COARSEN, 0.5), ax)
    for ax, n in enumerate(shape):
        a = _upsample_axis(a, n, ax)
    a = a - a.mean()
    return a / np.max(np.abs(a))


def _to_unit(a: np.ndarray) -> np.ndarray:
    lo, hi = a.min(), a.max()
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def _pad_edge(a: np.ndarray, nbl: int) -> np.ndarray:
    return np.pad(a, nbl, mode="edge") if nbl > 0 else a


def noise_state(padded_shape, seed: int) -> np.ndarray:
    """White-noise state N(0, 1), float32 (the harshest input for a stencil)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(padded_shape, dtype=np.float32)


def smooth_state(padded_shape, seed: int, corr_pts: float = 6.0) -> np.ndarray:
    """Synthetic wavefield-like state: a smooth random field plus 1 % white
    noise, float32, max|.| about 1.  Used as a common starting state for
    single-step comparisons."""
    rng = np.random.default_rng(seed)
    s = smooth_random(padded_shape, corr_pts, rng)
    s = s + 0.01 * rng.standard_normal(padded_shape)
    return s.astype(np.float32)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def acoustic_2d(nt: int = 500, seed: int = 1609) -> Problem:
    """2D isotropic acoustic, space order 4, 201 x 201 physical grid."""
    nx = nz = 201
    h = 10.0
    nbl = 20
    so = 4
    dt = DT[("acoustic_2d", so)]
    pad = (nz + 2 * nbl, nx + 2 * nbl)
    vel = np.full(pad, 1500.0, dtype=np.float32)
    eta = damping_profile(pad, nbl, (h, h, h), VMAX["acoustic_2d"])
    src = np.array([[1000.0, 1000.0]])
    rec = np.stack([np.arange(101) * 20.0, np.full(101, 20.0)], axis=1)
    w = ricker(15.0, dt, nt)[:, None]
    return Problem("acoustic_2d", 2, "acoustic", (nx, 1, nz), (h, h, h), nbl, so, dt, nt, 15.0,
                   vel, eta, src, rec, w, seed=seed)


def acoustic_3d(so: int = 8, phys: int = 512, nbl: int = 40, nt: int = 1000,
                seed: int = 1610, receivers: str = "surface") -> Problem:
    """3D isotropic acoustic: two-layer velocity with a smooth +-5 % random
    perturbation; ``phys`` physical points per axis (512 for the full size).

    ``receivers`` is "surface" (every physical (x, y) node at z = 20 m),
    "line" (every 8th node along y = centre) or "none"."""
    h = 10.0
    n = phys
    dt = DT[("acoustic_3d", so)]
    rng = np.random.default_rng(seed)
    z = np.arange(n) * h
    zi = n * h / 2.0                       # interface at half depth (2560 m at 512)
    vz = np.where(z < zi, 1500.0, 3500.0)
    p = 0.05 * smooth_random((n, n, n), 20.0, rng)
    vphys = vz[:, None, None] * (1.0 + p)
    vel = _pad_edge(vphys, nbl).astype(np.float32)
    pad = vel.shape
    eta = damping_profile(pad, nbl, (h, h, h), VMAX["acoustic_3d"])
    src = np.array([[n * h / 2.0, n * h / 2.0, 20.0]])
    if receivers == "surface":
        gx, gy = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="xy")
        rec = np.stack([gx.ravel(), gy.ravel(), np.full(n * n, 20.0)], axis=1)
    elif receivers == "line":
        xs = np.arange(0, n, 8) * h
        rec = np.stack([xs, np.full(xs.size, n * h / 2.0), np.full(xs.size, 20.0)], axis=1)
    else:
        rec = np.zeros((0, 3))
    w = ricker(10.0, dt, nt)[:, None]
    return Problem("acoustic_3d", 3, "acoustic", (n, n, n), (h, h, h), nbl, so, dt, nt, 10.0,
                   vel, eta, src, rec, w, seed=seed)


def tti_3d(so: int = 8, phys: int = 384, nbl: int = 40, nt: int = 800, seed: int = 1611,
           receivers: str = "line") -> Problem:
    """3D TTI pseudo-acoustic: layered velocity with a smooth perturbation and
    smooth Thomsen / angle fields (delta clipped to epsilon)."""
    h = 12.5
    n = phys
    dt = DT[("tti_3d", so)]
    rng = np.random.default_rng(seed)
    layers = np.array([1500.0, 2300.0, 3200.0, 4000.0])
    z = np.arange(n)
    vz = layers[np.minimum((4 * z) // n, 3)]
    p = 0.05 * smooth_random((n, n, n), 16.0, rng)
    vel = _pad_edge(vz[:, None, None] * (1.0 + p), nbl).astype(np.float32)
    eps = 0.3 * _to_unit(smooth_random((n, n, n), 16.0, rng))
    delta = np.minimum(0.1 * _to_unit(smooth_random((n, n, n), 16.0, rng)), eps)
    theta = np.deg2rad(45.0) * _to_unit(smooth_random((n, n, n), 16.0, rng))
    phi = np.deg2rad(90.0) * _to_unit(smooth_random((n, n, n), 16.0, rng))
    eps, delta, theta, phi = (_pad_edge(a, nbl).astype(np.float32)
                              for a in (eps, delta, theta, phi))
    delta = np.minimum(delta, eps)
    pad = vel.shape
    eta = damping_profile(pad, nbl, (h, h, h), VMAX["tti_3d"])
    src = np.array([[n * h / 2.0, n * h / 2.0, 25.0]])
    if receivers == "surface":
        gx, gy = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="xy")
        rec = np.stack([gx.ravel(), gy.ravel(), np.full(n * n, 25.0)], axis=1)
    elif receivers == "line":
        xs = np.arange(0, n, 4) * h
        rec = np.stack([xs, np.full(xs.size, n * h / 2.0), np.full(xs.size, 25.0)], axis=1)
    else:
        rec = np.zeros((0, 3))
    w = ricker(10.0, dt, nt)[:, None]
    return Problem("tti_3d", 3, "tti", (n, n, n), (h, h, h), nbl, so, dt, nt, 10.0,
                   vel, eta, src, rec, w, eps=eps, delta=delta, theta=theta, phi=phi, seed=seed)


def fwi_3d(so: int = 8, phys: int = 256, nbl: int = 40, nt: int = 1200, nshots: int = 16,
           seed: int = 1612, receivers: str = "surface") -> Problem:
    """Many-shot survey: true and smoothed start models, ``nshots`` single-
    source shots on a square grid at z = 30 m, receivers shared by all shots.

    ``src`` holds one source per shot ([nshots][3]); ``extra`` carries
    ``vel_start`` (the smoothed start model) and ``nshots``.  ``receivers``
    is "surface" (every physical (x, y) node) or "line" (every 8th node
    along y = centre)."""
    h = 15.0
    n = phys
    dt = DT[("fwi_3d", so)]
    rng = np.random.default_rng(seed)
    layers = np.array([1500.0, 2000.0, 2700.0, 3500.0])
    z = np.arange(n)
    vz = layers[np.minimum((4 * z) // n, 3)]
    p = 0.05 * smooth_random((n, n, n), 12.0, rng)
    vtrue = vz[:, None, None] * (1.0 + p)
    # smoothed on the coarse grid (every COARSEN-th point), then upsampled
    vstart = vtrue[::COARSEN, ::COARSEN, ::COARSEN]
    for ax in range(3):
        vstart = _smooth_axis(vstart, 10.0 / COARSEN, ax)
    for ax in range(3):
        vstart = _upsample_axis(vstart, n, ax)
    vel = _pad_edge(vtrue, nbl).astype(np.float32)
    vel0 = _pad_edge(vstart, nbl).astype(np.float32)
    eta = damping_profile(vel.shape, nbl, (h, h, h), VMAX["fwi_3d"])
    k = int(round(np.sqrt(nshots)))
    k = k if k * k == nshots else nshots
    side = np.linspace(0.125, 0.875, k) * (n - 1) * h
    if k * k == nshots:
        sx, sy = np.meshgrid(side, side, indexing="xy")
        src = np.stack([sx.ravel(), sy.ravel(), np.full(nshots, 30.0)], axis=1)
    else:
        src = np.stack([side, np.full(nshots, (n - 1) * h / 2.0), np.full(nshots, 30.0)], axis=1)
    if receivers == "surface":
        gx, gy = np.meshgrid(np.arange(n) * h, np.arange(n) * h, indexing="xy")
        rec = np.stack([gx.ravel(), gy.ravel(), np.full(n * n, 30.0)], axis=1)
    else:
        xs = np.arange(0, n, 8) * h
        rec = np.stack([xs, np.full(xs.size, n * h / 2.0), np.full(xs.size, 30.0)], axis=1)
    w = ricker(8.0, dt, nt)[:, None]
    return Problem("fwi_3d", 3, "acoustic", (n, n, n), (h, h, h), nbl, so, dt, nt, 8.0, vel, eta,
                   src, rec, w, seed=seed, extra={"vel_start": vel0, "nshots": nshots})


def vti_3d(so: int = 8, phys: int = 384, nbl: int = 40, nt: int = 800, seed: int = 1611,
           receivers: str = "line") -> Problem:
    """3D VTI pseudo-acoustic: the ``tti_3d`` velocity, epsilon and delta
    fields (delta <= epsilon) with no tilt or azimuth."""
    p = tti_3d(so=so, phys=phys, nbl=nbl, nt=nt, seed=seed, receivers=receivers)
    p.name, p.physics, p.theta, p.phi = "vti_3d", "vti", None, None
    return p


def learned_model(seed: int, phys_f: int = 256, nbl_f: int = 40, so_f: int = 16, so_c: int = 4,
                  nt_f: int = 1000, f0: float = 10.0, rec_every: int = 4) -> dict:
    """Fine / coarse pair of one random layered model (see the module notes).
    The coarse padded grid is every second point of the fine padded grid, so
    phys_f and nbl_f must be even."""
    assert phys_f % 2 == 0 and nbl_f % 2 == 0
    rng = np.random.default_rng(seed)
    h_f = 10.0
    n = phys_f
    nl = int(rng.integers(2, 6))
    depths = np.sort(rng.uniform(0.1, 0.9, nl - 1)) * n
    vels = np.sort(rng.uniform(1500.0, 3400.0, nl))
    z = np.arange(n)
    vz = vels[np.searchsorted(depths, z, side="right")]
    p = 0.05 * smooth_random((n, n, n), 20.0, rng)
    vel_f = _pad_edge(vz[:, None, None] * (1.0 + p), nbl_f).astype(np.float32)
    vel_c = np.ascontiguousarray(vel_f[::2, ::2, ::2])
    nbl_c = nbl_f // 2
    vmax = VMAX["acoustic_3d"]
    eta_f = damping_profile(vel_f.shape, nbl_f, (h_f,) * 3, vmax)
    eta_c = damping_profile(vel_c.shape, nbl_c, (2 * h_f,) * 3, vmax)
    dt_f = DT[("acoustic_3d", so_f)]
    dt_c = 2.0 * dt_f
    nt_c = nt_f // 2
    cx, cy = (rng.integers(n // 4, 3 * n // 4, 2) // 2) * 2 * h_f   # on the coarse grid
    src = np.array([[cx, cy, 40.0]])
    g = np.arange(0, n, rec_every) * h_f
    gx, gy = np.meshgrid(g, g, indexing="xy")
    rec = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 20.0)], axis=1)
    return {
        "shape_f": (n, n, n), "h_f": (h_f,) * 3, "nbl_f": nbl_f, "so_f": so_f, "dt_f": dt_f,
        "vel_f": vel_f, "eta_f": eta_f,
        "shape_c": (n // 2,) * 3, "h_c": (2 * h_f,) * 3, "nbl_c": nbl_c, "so_c": so_c,
        "dt_c": dt_c, "vel_c": vel_c, "eta_c": eta_c,
        "src": src, "rec": rec, "nt_f": nt_f, "nt_c": nt_c,
        "wav_f": ricker(f0, dt_f, nt_f)[:, None].astype(np.float32),
        "wav_c": ricker(f0, dt_c, nt_c)[:, None].astype(np.float32),
        "seed": seed,
    }
