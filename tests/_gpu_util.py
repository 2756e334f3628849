"""Helpers shared by the GPU parity tests (problem builders, norms, point
samples).  Inputs come from the seeded generators in ``workloads``; expected
values come only from the CPU oracle."""
import os
import sys

import numpy as np

import oracle
from workloads import Problem, damping_profile, ricker, smooth_random

THREADS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def acoustic_problem(ndim, phys, nbl, so, nt, seed, h=(10.0, 10.0, 10.0), damping=True,
                     nrec=24, f0=None):
    """Two-layer velocity with a smooth +-5 % perturbation, quadratic damping
    layer, one off-grid Ricker source and a line of receivers (alternately on
    and off grid).  ``phys`` = physical (nx, ny, nz); ny = 1 in 2D."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = phys
    pad = (nz + 2 * nbl, nx + 2 * nbl) if ndim == 2 else (nz + 2 * nbl, ny + 2 * nbl, nx + 2 * nbl)
    zz = np.arange(pad[0])[(slice(None),) + (None,) * (ndim - 1)]
    v = np.where(zz < pad[0] // 2, 1500.0, 3000.0) * (1 + 0.05 * smooth_random(pad, 6.0, rng))
    vel = v.astype(np.float32)
    vmax = float(vel.max())
    eta = damping_profile(pad, nbl, h, vmax) if damping else None
    dt = 0.4 * oracle.cfl_dt(ndim, so, h, vmax)
    f0 = f0 or 0.25 * 1500.0 / (6 * max(h))
    q = ricker(f0, dt, nt)[:, None]
    if ndim == 2:
        src = np.array([[0.37 * nx * h[0] + 3.3, 0.41 * nz * h[2] + 1.7]])
        xs = np.linspace(-nbl * h[0], (nx + nbl - 1) * h[0], nrec)
        rec = np.stack([xs, np.full(nrec, 2.0 * h[2])], 1)
        rec[::2, 0] = np.round(rec[::2, 0] / h[0]) * h[0]
    else:
        src = np.array([[0.37 * nx * h[0] + 3.3, 0.52 * ny * h[1] - 2.1, 0.41 * nz * h[2] + 1.7]])
        xs = np.linspace(-nbl * h[0], (nx + nbl - 1) * h[0], nrec)
        yr = 0.5 * (ny - 1) * h[1] + 0.25 * h[1] if ny > 1 else 0.0
        rec = np.stack([xs, np.full(nrec, yr), np.full(nrec, 2.0 * h[2])], 1)
        rec[::2, 0] = np.round(rec[::2, 0] / h[0]) * h[0]
    return Problem("test", ndim, "acoustic", (nx, ny if ndim == 3 else 1, nz), h, nbl, so, dt, nt,
                   f0, vel, eta, src, rec, q, seed=seed)


def oracle_run_with_peak(p, chunk=10):
    """Oracle forward run of p; also returns max over sampled times of the
    field norm (sampled every ``chunk`` steps)."""
    oracle.set_threads(THREADS)
    try:
        up = uc = None
        peak = 0.0
        traces = []
        done = 0
        while done < p.nt:
            k = min(chunk, p.nt - done)
            if p.physics == "acoustic":
                tr, up, uc = oracle.acoustic_forward(p.ndim, p.nbl, p.spacing, p.dt, p.so, p.vel,
                                                     p.eta, p.src, p.wavelet[done:done + k], p.rec,
                                                     k, up, uc)
                state = (up, uc)
            elif p.physics == "vti":
                tr, state = oracle.vti_forward(p.ndim, p.nbl, p.spacing, p.dt, p.so, p.vel,
                                               p.eta, p.eps, p.delta, p.src,
                                               p.wavelet[done:done + k], p.rec, k,
                                               None if uc is None else state)
                uc = state[1]
            else:
                tr, state = oracle.tti_forward(p.nbl, p.spacing, p.dt, p.so, p.vel, p.eta, p.eps,
                                               p.delta, p.theta, p.phi, p.src,
                                               p.wavelet[done:done + k], p.rec, k,
                                               None if uc is None else state)
                uc = state[1]
            traces.append(tr)
            peak = max(peak, float(np.linalg.norm(uc)))
            done += k
        return np.concatenate(traces), state, peak
    finally:
        oracle.set_threads(1)


def sample_points(shape, n_random, seed, radius):
    """Flat indices: every combination of per-axis edge/tile-boundary
    coordinates plus uniformly random points."""
    rng = np.random.default_rng(seed)
    axes = []
    for n in shape:
        c = {0, 1, radius - 1, radius, n // 2, n - radius - 1, n - radius, n - 2, n - 1, 7, 8,
             15, 16, 31, 32, 63, 64, 65, 127, 128}
        axes.append(sorted(v for v in c if 0 <= v < n))
    grid = np.array(np.meshgrid(*axes, indexing="ij")).reshape(len(shape), -1)
    rnd = np.stack([rng.integers(0, n, n_random) for n in shape])
    pts = np.concatenate([grid, rnd], axis=1)
    return np.ravel_multi_index(tuple(pts), shape)


def tti_problem(phys, nbl, so, nt, seed, h=(12.5, 12.5, 12.5), nrec=20):
    """Layered velocity, smooth Thomsen and angle fields (delta <= epsilon),
    damping layer, off-grid source into p and r, receivers on p."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = phys
    pad = (nz + 2 * nbl, ny + 2 * nbl, nx + 2 * nbl)
    zz = np.arange(pad[0])[:, None, None]
    v = (1500.0 + 2500.0 * zz / pad[0]) * (1 + 0.05 * smooth_random(pad, 6.0, rng))
    unit = lambda a: (a - a.min()) / (a.max() - a.min())
    eps = 0.3 * unit(smooth_random(pad, 6.0, rng))
    delta = np.minimum(0.1 * unit(smooth_random(pad, 6.0, rng)), eps)
    theta = np.deg2rad(45.0) * unit(smooth_random(pad, 6.0, rng))
    phi = np.deg2rad(90.0) * unit(smooth_random(pad, 6.0, rng))
    vel, eps, delta, theta, phi = (a.astype(np.float32) for a in (v, eps, delta, theta, phi))
    delta = np.minimum(delta, eps)
    vmax = float(np.max(vel.astype(np.float64) * np.sqrt(1 + 2 * eps.astype(np.float64))))
    eta = damping_profile(pad, nbl, h, float(vel.max()))
    dt = 0.4 * oracle.cfl_dt(3, so, h, vmax)
    f0 = 0.25 * 1500.0 / (6 * max(h))
    q = ricker(f0, dt, nt)[:, None]
    src = np.array([[0.45 * nx * h[0] + 1.1, 0.5 * ny * h[1] - 2.3, 0.4 * nz * h[2] + 0.7]])
    xs = np.linspace(-nbl * h[0], (nx + nbl - 1) * h[0], nrec)
    rec = np.stack([xs, np.full(nrec, 0.5 * ny * h[1]), np.full(nrec, 2.0 * h[2])], 1)
    rec[1::2, 0] -= 0.3 * h[0]   # odd receivers off grid, all inside the array
    return Problem("tti-test", 3, "tti", (nx, ny, nz), h, nbl, so, dt, nt, f0, vel, eta, src, rec,
                   q, eps=eps, delta=delta, theta=theta, phi=phi, seed=seed)


def vti_problem(ndim, phys, nbl, so, nt, seed, h=(12.5, 12.5, 12.5), nrec=20):
    """Layered velocity with smooth epsilon and delta (delta <= epsilon), no
    tilt: the VTI counterpart of ``tti_problem`` (2D uses the x-z plane)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = phys
    pad = (nz + 2 * nbl, nx + 2 * nbl) if ndim == 2 else (nz + 2 * nbl, ny + 2 * nbl, nx + 2 * nbl)
    zz = np.arange(pad[0])[(slice(None),) + (None,) * (ndim - 1)]
    v = (1500.0 + 2500.0 * zz / pad[0]) * (1 + 0.05 * smooth_random(pad, 6.0, rng))
    unit = lambda a: (a - a.min()) / (a.max() - a.min())
    eps = 0.3 * unit(smooth_random(pad, 6.0, rng))
    delta = np.minimum(0.1 * unit(smooth_random(pad, 6.0, rng)), eps)
    vel, eps, delta = (a.astype(np.float32) for a in (v, eps, delta))
    delta = np.minimum(delta, eps)
    vmax = float(np.max(vel.astype(np.float64) * np.sqrt(1 + 2 * eps.astype(np.float64))))
    eta = damping_profile(pad, nbl, h, float(vel.max()))
    dt = 0.4 * oracle.cfl_dt(ndim, so, h, vmax)
    f0 = 0.25 * 1500.0 / (6 * max(h))
    q = ricker(f0, dt, nt)[:, None]
    if ndim == 2:
        src = np.array([[0.45 * nx * h[0] + 1.1, 0.4 * nz * h[2] + 0.7]])
        xs = np.linspace(-nbl * h[0], (nx + nbl - 1) * h[0], nrec)
        rec = np.stack([xs, np.full(nrec, 2.0 * h[2])], 1)
    else:
        src = np.array([[0.45 * nx * h[0] + 1.1, 0.5 * ny * h[1] - 2.3, 0.4 * nz * h[2] + 0.7]])
        xs = np.linspace(-nbl * h[0], (nx + nbl - 1) * h[0], nrec)
        rec = np.stack([xs, np.full(nrec, 0.5 * ny * h[1]), np.full(nrec, 2.0 * h[2])], 1)
    rec[1::2, 0] -= 0.3 * h[0]
    return Problem("vti-test", ndim, "vti", (nx, ny if ndim == 3 else 1, nz), h, nbl, so, dt, nt,
                   f0, vel, eta, src, rec, q, eps=eps, delta=delta, seed=seed)
