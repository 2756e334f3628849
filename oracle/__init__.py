"""FP64 CPU oracle for the explicit finite-difference wave solver.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_1608_03984_amd``) never imports it, and it imports nothing from
the product: the two share no code.

The arithmetic lives in ``fd_oracle.c`` (plain C, IEEE double, scalar loops,
``-O2 -ffp-contract=off``); this module only marshals numpy arrays through
ctypes.  Inputs that a user supplies in FP32 (velocity, damping, Thomsen
parameters, angles, wavelet) are passed as float32 and up-cast inside the C
code, so a comparison against the GPU measures the solver and not input
rounding.  The evolving state of a forward run is FP64.

Shapes follow the C code: fields are C-order ``[nz][ny][nx]`` (x fastest) on
the padded array (physical points plus ``nbl`` layer points per side); 2D
problems have ``ny == 1``.  Coordinates are metres from the physical origin,
``(x, y, z)`` in 3D and ``(x, z)`` in 2D.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "fd_oracle.c"
_LIB = _HERE / "liboracle.so"

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_float_p = ctypes.POINTER(ctypes.c_float)
_c_long_p = ctypes.POINTER(ctypes.c_long)

_lib_handle = None


def build(force: bool = True) -> Path:
    """Compile ``liboracle.so`` with gcc (FP64, no contraction, OpenMP)."""
    if not force and _LIB.exists():
        return _LIB
    tmp = _LIB.with_suffix(".so.tmp")
    cmd = [
        "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", str(tmp), str(_SRC), "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not _LIB.exists():
            build()
        lib = ctypes.CDLL(str(_LIB))
        I, L, D = ctypes.c_int, ctypes.c_long, ctypes.c_double
        dp, fp, lp = _c_double_p, _c_float_p, _c_long_p
        sig = {
            "or_set_threads": (I, [I]),
            "or_weights_d2": (I, [I, dp]),
            "or_weights_d1": (I, [I, dp]),
            "or_cfl_dt": (D, [I, I, dp, D]),
            "or_a2": (D, [I, I]),
            "or_point_corners": (I, [I, lp, I, dp, dp, lp, dp]),
            "or_acoustic_forward": (I, [I, lp, I, dp, D, I, fp, fp, I, dp, fp, I, dp, dp,
                                        I, dp, dp]),
            "or_acoustic_step_points": (I, [I, lp, dp, D, I, fp, fp, fp, fp, L, lp, dp]),
            "or_tti_operators": (I, [lp, dp, I, dp, fp, fp, dp, dp, dp, dp]),
            "or_tti_forward": (I, [lp, I, dp, D, I, fp, fp, fp, fp, fp, fp, I, dp, fp, I, dp,
                                   dp, I, dp, dp, dp, dp]),
            "or_tti_step_points": (I, [lp, dp, D, I, fp, fp, fp, fp, fp, fp, fp, fp, fp, fp,
                                       L, lp, dp, dp]),
            "or_vti_forward": (I, [I, lp, I, dp, D, I, fp, fp, fp, fp, I, dp, fp, I, dp, dp, I,
                                   dp, dp, dp, dp]),
            "or_vti_step_points": (I, [I, lp, dp, D, I, fp, fp, fp, fp, fp, fp, fp, fp, L, lp,
                                       dp, dp]),
            "or_acoustic_adjoint": (I, [I, lp, I, dp, D, I, fp, fp, I, dp, dp, I, dp, dp, I]),
            "or_acoustic_gradient": (I, [I, lp, I, dp, D, I, fp, fp, I, dp, fp, I, dp, dp, I,
                                         dp, dp]),
            "or_acoustic_misfit": (I, [I, lp, I, dp, D, I, fp, fp, I, dp, fp, I, dp, dp, I, dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = lib
    return _lib_handle


def _d(a):
    return a.ctypes.data_as(_c_double_p)


def _f(a):
    return None if a is None else a.ctypes.data_as(_c_float_p)


def _l(a):
    return a.ctypes.data_as(_c_long_p)


def _as_f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _as_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> int:
    """OpenMP threads for the sweep loops (timing only)."""
    return int(_lib().or_set_threads(int(n)))


# --------------------------------------------------------------------------
# Weights and stability
# --------------------------------------------------------------------------

def weights_d2(so: int) -> np.ndarray:
    """Central second-derivative weights w[0..r] of order ``so`` (r = so/2)."""
    r = so // 2
    w = np.zeros(r + 1)
    if _lib().or_weights_d2(r, _d(w)) != 0:
        raise ValueError(so)
    return w


def weights_d1(so: int) -> np.ndarray:
    """Central first-derivative weights w[0..r] (w[0] = 0, w[-j] = -w[j])."""
    r = so // 2
    w = np.zeros(r + 1)
    if _lib().or_weights_d1(r, _d(w)) != 0:
        raise ValueError(so)
    return w


def a2(ndim: int, so: int) -> float:
    """Sum of absolute Laplacian weights (unit spacing), Eq. (stability)."""
    return float(_lib().or_a2(int(ndim), int(so)))


def cfl_dt(ndim: int, so: int, spacing, vmax: float) -> float:
    """Largest stable dt by the CFL condition of Eq. (stability), a1 = 4."""
    h = _as_f64(spacing)
    return float(_lib().or_cfl_dt(int(ndim), int(so), _d(h), float(vmax)))


def point_corners(ndim, shape_xyz, nbl, spacing, coord):
    """Flat corner indices and multilinear weights of one sparse point."""
    n = np.ascontiguousarray(shape_xyz, dtype=np.int64)
    h = _as_f64(spacing)
    c = _as_f64(coord)
    idx = np.zeros(8, dtype=np.int64)
    w = np.zeros(8)
    m = _lib().or_point_corners(int(ndim), _l(n), int(nbl), _d(h), _d(c), _l(idx), _d(w))
    return idx[:m], w[:m]


# --------------------------------------------------------------------------
# Acoustic
# --------------------------------------------------------------------------

def _pts(xyz, ndim):
    return _as_f64(np.reshape(xyz, (-1, ndim)) if len(xyz) else np.zeros((0, ndim)))


def _dims(ndim, field_shape):
    if ndim == 2:
        nz, nx = field_shape
        return np.array([nx, 1, nz], dtype=np.int64)
    nz, ny, nx = field_shape
    return np.array([nx, ny, nz], dtype=np.int64)


def acoustic_forward(ndim, nbl, spacing, dt, so, vel, eta, src_xyz, wavelet, rec_xyz, nt,
                     u_prev=None, u_cur=None):
    """Run ``nt`` damped leapfrog steps from the given (or zero) state.

    Returns ``(traces[nt][nrec], u_prev, u_cur)`` in FP64.
    """
    vel = _as_f32(vel)
    shape = vel.shape
    n = _dims(ndim, shape)
    h = _as_f64(spacing)
    eta = _as_f32(eta)
    src = _as_f64(np.reshape(src_xyz, (-1, ndim)) if len(src_xyz) else np.zeros((0, ndim)))
    rec = _as_f64(np.reshape(rec_xyz, (-1, ndim)) if len(rec_xyz) else np.zeros((0, ndim)))
    nsrc, nrec = src.shape[0], rec.shape[0]
    q = _as_f32(np.reshape(wavelet, (nt, nsrc)) if nsrc else np.zeros((nt, 0)))
    up = np.zeros(shape) if u_prev is None else np.array(u_prev, dtype=np.float64, copy=True)
    uc = np.zeros(shape) if u_cur is None else np.array(u_cur, dtype=np.float64, copy=True)
    tr = np.zeros((nt, max(nrec, 1)))
    rc = _lib().or_acoustic_forward(
        int(ndim), _l(n), int(nbl), _d(h), float(dt), int(so), _f(vel), _f(eta),
        int(nsrc), _d(src), _f(q), int(nrec), _d(rec), _d(tr), int(nt), _d(up), _d(uc))
    if rc != 0:
        raise ValueError("oracle rejected the acoustic problem (shape/order/points)")
    return tr[:, :nrec], up, uc


def acoustic_step_points(ndim, spacing, dt, so, vel, eta, u_prev, u_cur, pts):
    """One source-free acoustic step evaluated at flat indices ``pts`` from an
    FP32 state; returns FP64 values."""
    vel = _as_f32(vel)
    n = _dims(ndim, vel.shape)
    h = _as_f64(spacing)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.zeros(pts.size)
    rc = _lib().or_acoustic_step_points(
        int(ndim), _l(n), _d(h), float(dt), int(so), _f(vel), _f(_as_f32(eta)),
        _f(_as_f32(u_prev)), _f(_as_f32(u_cur)), int(pts.size), _l(pts), _d(out))
    if rc != 0:
        raise ValueError("oracle rejected the acoustic step")
    return out


# --------------------------------------------------------------------------
# TTI
# --------------------------------------------------------------------------

def tti_operators(spacing, so, f, theta, phi):
    """(G_xbar_xbar f, G_ybar_ybar f, G_zbar_zbar f, Laplacian f) on a 3D field."""
    f = _as_f64(f)
    n = _dims(3, f.shape)
    h = _as_f64(spacing)
    outs = [np.zeros(f.shape) for _ in range(4)]
    rc = _lib().or_tti_operators(_l(n), _d(h), int(so), _d(f), _f(_as_f32(theta)),
                                 _f(_as_f32(phi)), *[_d(o) for o in outs])
    if rc != 0:
        raise ValueError(so)
    return tuple(outs)


def tti_forward(nbl, spacing, dt, so, vel, eta, eps, delta, theta, phi, src_xyz, wavelet,
                rec_xyz, nt, state=None):
    """TTI forward run; ``state`` = (p_prev, p_cur, r_prev, r_cur) or None.

    Returns ``(traces[nt][nrec], (p_prev, p_cur, r_prev, r_cur))``.
    """
    vel = _as_f32(vel)
    shape = vel.shape
    n = _dims(3, shape)
    h = _as_f64(spacing)
    src = _as_f64(np.reshape(src_xyz, (-1, 3)) if len(src_xyz) else np.zeros((0, 3)))
    rec = _as_f64(np.reshape(rec_xyz, (-1, 3)) if len(rec_xyz) else np.zeros((0, 3)))
    nsrc, nrec = src.shape[0], rec.shape[0]
    q = _as_f32(np.reshape(wavelet, (nt, nsrc)) if nsrc else np.zeros((nt, 0)))
    if state is None:
        st = [np.zeros(shape) for _ in range(4)]
    else:
        st = [np.array(s, dtype=np.float64, copy=True) for s in state]
    tr = np.zeros((nt, max(nrec, 1)))
    rc = _lib().or_tti_forward(
        _l(n), int(nbl), _d(h), float(dt), int(so), _f(vel), _f(_as_f32(eta)),
        _f(_as_f32(eps)), _f(_as_f32(delta)), _f(_as_f32(theta)), _f(_as_f32(phi)),
        int(nsrc), _d(src), _f(q), int(nrec), _d(rec), _d(tr), int(nt), *[_d(s) for s in st])
    if rc != 0:
        raise ValueError("oracle rejected the TTI problem")
    return tr[:, :nrec], tuple(st)


def tti_step_points(spacing, dt, so, vel, eta, eps, delta, theta, phi, state, pts):
    """One source-free TTI step at flat indices ``pts`` from an FP32 state
    (p_prev, p_cur, r_prev, r_cur); returns (p_next, r_next) in FP64."""
    vel = _as_f32(vel)
    n = _dims(3, vel.shape)
    h = _as_f64(spacing)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    op = np.zeros(pts.size)
    orr = np.zeros(pts.size)
    st = [_as_f32(s) for s in state]
    rc = _lib().or_tti_step_points(
        _l(n), _d(h), float(dt), int(so), _f(vel), _f(_as_f32(eta)), _f(_as_f32(eps)),
        _f(_as_f32(delta)), _f(_as_f32(theta)), _f(_as_f32(phi)), *[_f(s) for s in st],
        int(pts.size), _l(pts), _d(op), _d(orr))
    if rc != 0:
        raise ValueError("oracle rejected the TTI step")
    return op, orr


# --------------------------------------------------------------------------
# VTI
# --------------------------------------------------------------------------

def vti_forward(ndim, nbl, spacing, dt, so, vel, eta, eps, delta, src_xyz, wavelet, rec_xyz, nt,
                state=None):
    """VTI forward run (2D or 3D); ``state`` = (p_prev, p_cur, r_prev, r_cur)
    or None.  Returns ``(traces[nt][nrec], (p_prev, p_cur, r_prev, r_cur))``."""
    vel = _as_f32(vel)
    shape = vel.shape
    n = _dims(ndim, shape)
    h = _as_f64(spacing)
    src = _pts(src_xyz, ndim)
    rec = _pts(rec_xyz, ndim)
    nsrc, nrec = src.shape[0], rec.shape[0]
    q = _as_f32(np.reshape(wavelet, (nt, nsrc)) if nsrc else np.zeros((nt, 0)))
    if state is None:
        st = [np.zeros(shape) for _ in range(4)]
    else:
        st = [np.array(x, dtype=np.float64, copy=True) for x in state]
    tr = np.zeros((nt, max(nrec, 1)))
    rc = _lib().or_vti_forward(
        int(ndim), _l(n), int(nbl), _d(h), float(dt), int(so), _f(vel), _f(_as_f32(eta)),
        _f(_as_f32(eps)), _f(_as_f32(delta)), int(nsrc), _d(src), _f(q), int(nrec), _d(rec),
        _d(tr), int(nt), *[_d(x) for x in st])
    if rc != 0:
        raise ValueError("oracle rejected the VTI problem")
    return tr[:, :nrec], tuple(st)


def vti_step_points(ndim, spacing, dt, so, vel, eta, eps, delta, state, pts):
    """One source-free VTI step at flat indices ``pts`` from an FP32 state
    (p_prev, p_cur, r_prev, r_cur); returns (p_next, r_next) in FP64."""
    vel = _as_f32(vel)
    n = _dims(ndim, vel.shape)
    h = _as_f64(spacing)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    op = np.zeros(pts.size)
    orr = np.zeros(pts.size)
    st = [_as_f32(x) for x in state]
    rc = _lib().or_vti_step_points(
        int(ndim), _l(n), _d(h), float(dt), int(so), _f(vel), _f(_as_f32(eta)),
        _f(_as_f32(eps)), _f(_as_f32(delta)), *[_f(x) for x in st], int(pts.size), _l(pts),
        _d(op), _d(orr))
    if rc != 0:
        raise ValueError("oracle rejected the VTI step")
    return op, orr


# --------------------------------------------------------------------------
# Adjoint and gradient (acoustic)
# --------------------------------------------------------------------------

def acoustic_adjoint(ndim, nbl, spacing, dt, so, vel, eta, src_xyz, rec_xyz, d, nt):
    """F^T d: the transpose of the (zero-initial-state) map wavelet -> traces,
    applied to receiver data d[nt][nrec]; returns q'[nt][nsrc] (FP64)."""
    vel = _as_f32(vel)
    n = _dims(ndim, vel.shape)
    h = _as_f64(spacing)
    src, rec = _pts(src_xyz, ndim), _pts(rec_xyz, ndim)
    d = _as_f64(np.reshape(d, (nt, rec.shape[0])))
    q = np.zeros((nt, max(src.shape[0], 1)))
    rc = _lib().or_acoustic_adjoint(int(ndim), _l(n), int(nbl), _d(h), float(dt), int(so), _f(vel),
                                    _f(_as_f32(eta)), int(src.shape[0]), _d(src), _d(q),
                                    int(rec.shape[0]), _d(rec), _d(d), int(nt))
    if rc != 0:
        raise ValueError("oracle rejected the adjoint problem")
    return q[:, :src.shape[0]]


def acoustic_gradient(ndim, nbl, spacing, dt, so, vel, eta, src_xyz, wavelet, rec_xyz, dobs, nt):
    """(dJ/dm field, J) for J = 1/2 sum (d - dobs)^2, m = 1/v^2 (FP64, full
    forward history in memory: small grids only)."""
    vel = _as_f32(vel)
    n = _dims(ndim, vel.shape)
    h = _as_f64(spacing)
    src, rec = _pts(src_xyz, ndim), _pts(rec_xyz, ndim)
    q = _as_f32(np.reshape(wavelet, (nt, src.shape[0])))
    dobs = _as_f64(np.reshape(dobs, (nt, rec.shape[0])))
    g = np.zeros(vel.shape)
    J = np.zeros(1)
    rc = _lib().or_acoustic_gradient(int(ndim), _l(n), int(nbl), _d(h), float(dt), int(so),
                                     _f(vel), _f(_as_f32(eta)), int(src.shape[0]), _d(src), _f(q),
                                     int(rec.shape[0]), _d(rec), _d(dobs), int(nt), _d(g), _d(J))
    if rc != 0:
        raise ValueError("oracle rejected the gradient problem")
    return g, float(J[0])


def acoustic_misfit(ndim, nbl, spacing, dt, so, vel, eta, src_xyz, wavelet, rec_xyz, dobs, nt):
    """J = 1/2 sum (d - dobs)^2 of an oracle forward run."""
    vel = _as_f32(vel)
    n = _dims(ndim, vel.shape)
    h = _as_f64(spacing)
    src, rec = _pts(src_xyz, ndim), _pts(rec_xyz, ndim)
    q = _as_f32(np.reshape(wavelet, (nt, src.shape[0])))
    dobs = _as_f64(np.reshape(dobs, (nt, rec.shape[0])))
    J = np.zeros(1)
    rc = _lib().or_acoustic_misfit(int(ndim), _l(n), int(nbl), _d(h), float(dt), int(so), _f(vel),
                                   _f(_as_f32(eta)), int(src.shape[0]), _d(src), _f(q),
                                   int(rec.shape[0]), _d(rec), _d(dobs), int(nt), _d(J))
    if rc != 0:
        raise ValueError("oracle rejected the misfit problem")
    return float(J[0])
