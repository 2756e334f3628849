"""ctypes binding of libfd (include/fd.h): the same entry points, argument
marshalling only.  Every step of the solver runs in the HIP kernels of
libfd.so; nothing here computes on the CPU.  Loading fails loudly when the
library has not been built."""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

_LIBPATH = Path(__file__).resolve().parent / "libfd.so"

FD_OK = 0
FD_ERR_INVALID_ARG = 1
FD_ERR_UNSTABLE_DT = 2
FD_ERR_UNSUPPORTED = 3
FD_ERR_WORKSPACE = 4
FD_ERR_DEVICE = 5
FD_ERR_NONFINITE = 6
FD_ERR_HOST = 7

FD_ACOUSTIC = 0
FD_TTI = 1
FD_VTI = 2

FD_FIELD_PREV = 0
FD_FIELD_CUR = 1
FD_FIELD_R_PREV = 2
FD_FIELD_R_CUR = 3

FD_ZERO_STATE = 1
FD_KEEP_POINTS = 2
FD_TRIAD_TEMPORAL = 1
FD_MAX_SPACE_ORDER = 16

FD_OPT_KERNEL = 1
FD_OPT_ZCHUNK = 2
FD_OPT_TILE = 3
FD_OPT_SHOTS_PER_BLOCK = 4
FD_OPT_DAMPING_PROFILE = 5
FD_OPT_FUSED_IMAGING = 6

FD_WRT_M = 0
FD_WRT_VEL = 1
FD_GRAD_ACCUMULATE = 256

FD_CNN_LAYER_FLOATS = 27 * 256 + 16
FD_CNN_RELU = 0
FD_CNN_LINEAR = 1
FD_CNN_MASKED = 2
FD_CNN_IDENTITY = 3
FD_CNN_UNMASKED = 4
FD_CNN_NOALLOC_SCRATCH_FLOATS = 12582912
FD_CNN_LOSS_FLOATS = 257
FD_MISFIT_DOUBLES = 1025

EXPORTS = (
    "fd_workspace_bytes", "fd_setup", "fd_forward", "fd_get_field", "fd_set_field",
    "fd_stencil_weights", "fd_cfl_dt", "fd_set_option", "fd_destroy", "fd_strerror",
    "fd_last_error", "fd_triad", "fd_checkpoint_bytes", "fd_forward_checkpointed", "fd_gradient",
    "fd_adjoint", "fd_misfit", "fd_workspace_bytes_shots", "fd_setup_shots", "fd_forward_shots",
    "fd_get_shot_field", "fd_set_shot_field", "fd_cnn_packed_elems", "fd_cnn_pack", "fd_cnn_conv",
    "fd_cnn_wgrad_scratch", "fd_cnn_wgrad", "fd_cnn_loss_grad", "fd_cnn_adam", "fd_cnn_features",
    "fd_cnn_correct", "fd_cnn_residual", "fd_restrict", "fd_triad_config",
    "fd_cnn_wgrad_noalloc", "fd_forward_checkpointed_shots", "fd_gradient_shots",
    "fd_get_option",
)


class FdGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("space_order", ctypes.c_int32),
        ("physics", ctypes.c_int32),
        ("nbl", ctypes.c_int32),
        ("shape", ctypes.c_int64 * 3),
        ("spacing", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
    ]


class FdModel(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("vel", "eta", "epsilon", "delta", "theta", "phi")]


class FdPoints(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("coords", ctypes.POINTER(ctypes.c_double)),
        ("data", ctypes.c_void_p),
    ]


class FdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        msg = f"{where}: {fd_strerror(code)} (status {code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib_handle = None


def lib() -> ctypes.CDLL:
    """The loaded libfd.so; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not _LIBPATH.exists():
            raise RuntimeError(f"{_LIBPATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_1608_03984_amd._build)")
        L = ctypes.CDLL(str(_LIBPATH))
        i32, u64p, vp = ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p
        gp, mp, pp = ctypes.POINTER(FdGrid), ctypes.POINTER(FdModel), ctypes.POINTER(FdPoints)
        sig = {
            "fd_workspace_bytes": (i32, [gp, i32, u64p]),
            "fd_setup": (i32, [gp, mp, vp, ctypes.c_uint64, i32, vp, ctypes.POINTER(vp)]),
            "fd_forward": (i32, [vp, i32, pp, pp, i32, vp]),
            "fd_get_field": (i32, [vp, i32, vp, vp]),
            "fd_set_field": (i32, [vp, i32, vp, vp]),
            "fd_stencil_weights": (i32, [i32, i32, ctypes.POINTER(ctypes.c_double)]),
            "fd_cfl_dt": (i32, [gp, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
            "fd_set_option": (i32, [vp, i32, ctypes.c_int64]),
            "fd_get_option": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int64)]),
            "fd_destroy": (i32, [vp]),
            "fd_strerror": (ctypes.c_char_p, [i32]),
            "fd_last_error": (ctypes.c_char_p, [vp]),
            "fd_triad": (i32, [vp, vp, vp, ctypes.c_float, ctypes.c_int64, vp]),
            "fd_triad_config": (i32, [vp, vp, vp, ctypes.c_float, ctypes.c_int64, i32, i32, i32,
                                      vp]),
            "fd_checkpoint_bytes": (i32, [vp, i32, i32, u64p, ctypes.POINTER(i32)]),
            "fd_forward_checkpointed": (i32, [vp, i32, pp, pp, i32, vp, ctypes.c_uint64, vp]),
            "fd_gradient": (i32, [vp, i32, pp, pp, i32, vp, ctypes.c_uint64, i32, vp, vp, vp]),
            "fd_forward_checkpointed_shots": (i32, [vp, i32, pp, ctypes.POINTER(i32), pp,
                                                    ctypes.POINTER(i32), i32, vp, ctypes.c_uint64,
                                                    vp]),
            "fd_gradient_shots": (i32, [vp, i32, pp, ctypes.POINTER(i32), pp, ctypes.POINTER(i32),
                                        i32, vp, ctypes.c_uint64, i32, vp, vp, vp]),
            "fd_adjoint": (i32, [vp, i32, pp, pp, vp]),
            "fd_misfit": (i32, [vp, vp, ctypes.c_int64, vp, vp, vp]),
            "fd_workspace_bytes_shots": (i32, [gp, i32, i32, u64p]),
            "fd_setup_shots": (i32, [gp, mp, i32, vp, ctypes.c_uint64, i32, vp,
                                     ctypes.POINTER(vp)]),
            "fd_forward_shots": (i32, [vp, i32, pp, ctypes.POINTER(i32), pp,
                                       ctypes.POINTER(i32), i32, vp]),
            "fd_get_shot_field": (i32, [vp, i32, i32, vp, vp]),
            "fd_set_shot_field": (i32, [vp, i32, i32, vp, vp]),
            "fd_cnn_packed_elems": (i32, [i32, ctypes.POINTER(ctypes.c_int64)]),
            "fd_cnn_pack": (i32, [vp, i32, i32, vp, vp]),
            "fd_cnn_conv": (i32, [vp, i32, ctypes.POINTER(ctypes.c_int64), vp, vp, i32, vp, i32,
                                  vp, vp, vp]),
            "fd_cnn_wgrad_scratch": (i32, [ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64)]),
            "fd_cnn_wgrad": (i32, [vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int64), vp,
                                   ctypes.c_int64, vp, vp]),
            "fd_cnn_wgrad_noalloc": (i32, [vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int64), vp,
                                           vp]),
            "fd_cnn_loss_grad": (i32, [vp, vp, vp, ctypes.c_int64, i32, i32, ctypes.c_float, vp,
                                       vp, vp]),
            "fd_cnn_adam": (i32, [vp, vp, vp, vp, ctypes.c_int64, i32, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]),
            "fd_cnn_features": (i32, [vp, ctypes.c_float, vp, vp, vp, vp]),
            "fd_cnn_correct": (i32, [vp, vp, vp, vp, vp]),
            "fd_cnn_residual": (i32, [vp, vp, vp, vp, vp, vp]),
            "fd_restrict": (i32, [vp, i32, i32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = L
    return _lib_handle


def make_grid(ndim, shape, spacing, nbl, space_order, dt, physics=FD_ACOUSTIC) -> FdGrid:
    """fd_grid from Python values; shape/spacing are (x, y, z) (ny = 1 in 2D)."""
    g = FdGrid()
    g.ndim = int(ndim)
    g.space_order = int(space_order)
    g.physics = int(physics)
    g.nbl = int(nbl)
    for a in range(3):
        g.shape[a] = int(shape[a])
        g.spacing[a] = float(spacing[a])
    g.dt = float(dt)
    return g


def _check(code: int, where: str, ctx=None):
    if code != FD_OK:
        detail = fd_last_error(ctx) if ctx else ""
        raise FdError(code, where, detail)


def fd_strerror(code: int) -> str:
    return lib().fd_strerror(int(code)).decode()


def fd_last_error(ctx) -> str:
    return lib().fd_last_error(ctx).decode() if ctx else ""


def fd_workspace_bytes(grid: FdGrid, max_points: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().fd_workspace_bytes(ctypes.byref(grid), int(max_points), ctypes.byref(out)),
           "fd_workspace_bytes")
    return int(out.value)


def fd_setup(grid: FdGrid, model: FdModel, workspace_ptr: int, workspace_bytes: int,
             max_points: int, stream: int):
    ctx = ctypes.c_void_p(0)
    _check(lib().fd_setup(ctypes.byref(grid), ctypes.byref(model), ctypes.c_void_p(workspace_ptr),
                          int(workspace_bytes), int(max_points), ctypes.c_void_p(stream),
                          ctypes.byref(ctx)), "fd_setup")
    return ctx


def _points(coords, data_ptr):
    """fd_points for host coordinates [n][ndim]; an int n instead gives n
    points with no coordinates (FD_KEEP_POINTS calls)."""
    if coords is None:
        return None, None
    if isinstance(coords, (int, np.integer)):
        p = FdPoints()
        p.n = int(coords)
        p.coords = None
        p.data = ctypes.c_void_p(int(data_ptr) if data_ptr else 0)
        return p, None
    c = np.ascontiguousarray(coords, dtype=np.float64)
    p = FdPoints()
    p.n = int(c.shape[0]) if c.size else 0
    p.coords = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.data = ctypes.c_void_p(int(data_ptr) if data_ptr else 0)
    return p, c


def fd_forward(ctx, nt: int, src_coords, src_data_ptr, rec_coords, rec_data_ptr, flags: int,
               stream: int):
    sp, keep_s = _points(src_coords, src_data_ptr)
    rp, keep_r = _points(rec_coords, rec_data_ptr)
    code = lib().fd_forward(ctx, int(nt), ctypes.byref(sp) if sp else None,
                            ctypes.byref(rp) if rp else None, int(flags), ctypes.c_void_p(stream))
    del keep_s, keep_r
    _check(code, "fd_forward", ctx)


def fd_get_field(ctx, which: int, dst_ptr: int, stream: int):
    _check(lib().fd_get_field(ctx, int(which), ctypes.c_void_p(dst_ptr), ctypes.c_void_p(stream)),
           "fd_get_field", ctx)


def fd_set_field(ctx, which: int, src_ptr: int, stream: int):
    _check(lib().fd_set_field(ctx, int(which), ctypes.c_void_p(src_ptr), ctypes.c_void_p(stream)),
           "fd_set_field", ctx)


def fd_set_option(ctx, option: int, value: int):
    _check(lib().fd_set_option(ctx, int(option), int(value)), "fd_set_option", ctx)


def fd_get_option(ctx, option: int) -> int:
    v = ctypes.c_int64(0)
    _check(lib().fd_get_option(ctx, int(option), ctypes.byref(v)), "fd_get_option", ctx)
    return int(v.value)


def fd_destroy(ctx):
    if ctx:
        lib().fd_destroy(ctx)


def fd_triad(a_ptr: int, b_ptr: int, c_ptr: int, s: float, n: int, stream: int):
    _check(lib().fd_triad(ctypes.c_void_p(a_ptr), ctypes.c_void_p(b_ptr), ctypes.c_void_p(c_ptr),
                          float(s), int(n), ctypes.c_void_p(stream)), "fd_triad")


def fd_triad_config(a_ptr: int, b_ptr: int, c_ptr: int, s: float, n: int, unroll: int,
                    blocks: int, flags: int, stream: int):
    _check(lib().fd_triad_config(ctypes.c_void_p(a_ptr), ctypes.c_void_p(b_ptr),
                                 ctypes.c_void_p(c_ptr), float(s), int(n), int(unroll),
                                 int(blocks), int(flags), ctypes.c_void_p(stream)),
           "fd_triad_config")


def fd_stencil_weights(space_order: int, deriv: int) -> np.ndarray:
    w = np.zeros(space_order // 2 + 1)
    _check(lib().fd_stencil_weights(int(space_order), int(deriv),
                                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "fd_stencil_weights")
    return w


def fd_cfl_dt(grid: FdGrid, vmax: float) -> float:
    out = ctypes.c_double(0.0)
    _check(lib().fd_cfl_dt(ctypes.byref(grid), float(vmax), ctypes.byref(out)), "fd_cfl_dt")
    return float(out.value)


def fd_checkpoint_bytes(ctx, nt: int, interval: int):
    """(bytes, interval used)."""
    out = ctypes.c_uint64(0)
    used = ctypes.c_int32(0)
    _check(lib().fd_checkpoint_bytes(ctx, int(nt), int(interval), ctypes.byref(out),
                                     ctypes.byref(used)), "fd_checkpoint_bytes", ctx)
    return int(out.value), int(used.value)


def fd_forward_checkpointed(ctx, nt: int, src_coords, src_data_ptr, rec_coords, rec_data_ptr,
                            interval: int, store_ptr: int, store_bytes: int, stream: int):
    sp, keep_s = _points(src_coords, src_data_ptr)
    rp, keep_r = _points(rec_coords, rec_data_ptr)
    code = lib().fd_forward_checkpointed(ctx, int(nt), ctypes.byref(sp) if sp else None,
                                         ctypes.byref(rp) if rp else None, int(interval),
                                         ctypes.c_void_p(store_ptr), int(store_bytes),
                                         ctypes.c_void_p(stream))
    del keep_s, keep_r
    _check(code, "fd_forward_checkpointed", ctx)


def fd_gradient(ctx, nt: int, src_coords, src_data_ptr, adj_coords, adj_data_ptr, interval: int,
                store_ptr: int, store_bytes: int, wrt: int, grad_ptr: int, wavelet_grad_ptr: int,
                stream: int):
    sp, keep_s = _points(src_coords, src_data_ptr)
    ap, keep_a = _points(adj_coords, adj_data_ptr)
    code = lib().fd_gradient(ctx, int(nt), ctypes.byref(sp) if sp else None,
                             ctypes.byref(ap) if ap else None, int(interval),
                             ctypes.c_void_p(store_ptr), int(store_bytes), int(wrt),
                             ctypes.c_void_p(grad_ptr), ctypes.c_void_p(wavelet_grad_ptr or 0),
                             ctypes.c_void_p(stream))
    del keep_s, keep_a
    _check(code, "fd_gradient", ctx)


def fd_misfit(d_ptr, dobs_ptr, n: int, res_ptr, J_ptr, stream: int):
    code = lib().fd_misfit(ctypes.c_void_p(d_ptr), ctypes.c_void_p(dobs_ptr), int(n),
                           ctypes.c_void_p(res_ptr), ctypes.c_void_p(J_ptr),
                           ctypes.c_void_p(stream))
    _check(code, "fd_misfit", None)


def fd_adjoint(ctx, nt: int, adj_coords, adj_data_ptr, out_coords, out_data_ptr, stream: int):
    ap, keep_a = _points(adj_coords, adj_data_ptr)
    op, keep_o = _points(out_coords, out_data_ptr)
    code = lib().fd_adjoint(ctx, int(nt), ctypes.byref(ap) if ap else None,
                            ctypes.byref(op) if op else None, ctypes.c_void_p(stream))
    del keep_a, keep_o
    _check(code, "fd_adjoint", ctx)


def fd_workspace_bytes_shots(grid: FdGrid, nshots: int, max_points: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().fd_workspace_bytes_shots(ctypes.byref(grid), int(nshots), int(max_points),
                                          ctypes.byref(out)), "fd_workspace_bytes_shots")
    return int(out.value)


def fd_setup_shots(grid: FdGrid, model: FdModel, nshots: int, workspace_ptr: int,
                   workspace_bytes: int, max_points: int, stream: int):
    ctx = ctypes.c_void_p(0)
    _check(lib().fd_setup_shots(ctypes.byref(grid), ctypes.byref(model), int(nshots),
                                ctypes.c_void_p(workspace_ptr), int(workspace_bytes),
                                int(max_points), ctypes.c_void_p(stream), ctypes.byref(ctx)),
           "fd_setup_shots")
    return ctx


def _counts(c):
    if c is None:
        return None, None
    a = np.ascontiguousarray(c, dtype=np.int32)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), a


def fd_forward_shots(ctx, nt: int, src_coords, src_counts, src_data_ptr, rec_coords, rec_counts,
                     rec_data_ptr, flags: int, stream: int):
    sp, keep_s = _points(src_coords, src_data_ptr)
    rp, keep_r = _points(rec_coords, rec_data_ptr)
    sc, keep_sc = _counts(src_counts)
    rc, keep_rc = _counts(rec_counts)
    code = lib().fd_forward_shots(ctx, int(nt), ctypes.byref(sp) if sp else None, sc,
                                  ctypes.byref(rp) if rp else None, rc, int(flags),
                                  ctypes.c_void_p(stream))
    del keep_s, keep_r, keep_sc, keep_rc
    _check(code, "fd_forward_shots", ctx)


def fd_forward_checkpointed_shots(ctx, nt: int, src_coords, src_counts, src_data_ptr,
                                  rec_coords, rec_counts, rec_data_ptr, interval: int,
                                  store_ptr: int, store_bytes: int, stream: int):
    sp, keep_s = _points(src_coords, src_data_ptr)
    rp, keep_r = _points(rec_coords, rec_data_ptr)
    sc, keep_sc = _counts(src_counts)
    rc, keep_rc = _counts(rec_counts)
    code = lib().fd_forward_checkpointed_shots(ctx, int(nt), ctypes.byref(sp) if sp else None, sc,
                                               ctypes.byref(rp) if rp else None, rc,
                                               int(interval), ctypes.c_void_p(store_ptr),
                                               int(store_bytes), ctypes.c_void_p(stream))
    del keep_s, keep_r, keep_sc, keep_rc
    _check(code, "fd_forward_checkpointed_shots", ctx)


def fd_gradient_shots(ctx, nt: int, src_coords, src_counts, src_data_ptr, adj_coords, adj_counts,
                      adj_data_ptr, interval: int, store_ptr: int, store_bytes: int, wrt: int,
                      grad_ptr: int, wavelet_grad_ptr: int, stream: int):
    sp, keep_s = _points(src_coords, src_data_ptr)
    ap, keep_a = _points(adj_coords, adj_data_ptr)
    sc, keep_sc = _counts(src_counts)
    ac, keep_ac = _counts(adj_counts)
    code = lib().fd_gradient_shots(ctx, int(nt), ctypes.byref(sp) if sp else None, sc,
                                   ctypes.byref(ap) if ap else None, ac, int(interval),
                                   ctypes.c_void_p(store_ptr), int(store_bytes), int(wrt),
                                   ctypes.c_void_p(grad_ptr), ctypes.c_void_p(wavelet_grad_ptr or 0),
                                   ctypes.c_void_p(stream))
    del keep_s, keep_a, keep_sc, keep_ac
    _check(code, "fd_gradient_shots", ctx)


def fd_get_shot_field(ctx, shot: int, which: int, dst_ptr: int, stream: int):
    _check(lib().fd_get_shot_field(ctx, int(shot), int(which), ctypes.c_void_p(dst_ptr),
                                   ctypes.c_void_p(stream)), "fd_get_shot_field", ctx)


def fd_set_shot_field(ctx, shot: int, which: int, src_ptr: int, stream: int):
    _check(lib().fd_set_shot_field(ctx, int(shot), int(which), ctypes.c_void_p(src_ptr),
                                   ctypes.c_void_p(stream)), "fd_set_shot_field", ctx)


def _shape3(shape):
    return (ctypes.c_int64 * 3)(*[int(v) for v in shape])


def _vp(ptr):
    return ctypes.c_void_p(int(ptr) if ptr else 0)


def fd_cnn_packed_elems(cin_pad: int) -> int:
    out = ctypes.c_int64(0)
    _check(lib().fd_cnn_packed_elems(int(cin_pad), ctypes.byref(out)), "fd_cnn_packed_elems")
    return int(out.value)


def fd_cnn_pack(layer_ptr, cin_pad, transpose, packed_ptr, stream):
    _check(lib().fd_cnn_pack(_vp(layer_ptr), int(cin_pad), int(transpose), _vp(packed_ptr),
                             _vp(stream)), "fd_cnn_pack")


def fd_cnn_conv(x_ptr, cin_pad, shape, packed_ptr, bias_ptr, mode, mask_ptr, cout_store, y_ptr,
                yf_ptr, stream):
    _check(lib().fd_cnn_conv(_vp(x_ptr), int(cin_pad), _shape3(shape), _vp(packed_ptr),
                             _vp(bias_ptr), int(mode), _vp(mask_ptr), int(cout_store), _vp(y_ptr),
                             _vp(yf_ptr), _vp(stream)), "fd_cnn_conv")


def fd_cnn_wgrad_scratch(shape) -> int:
    out = ctypes.c_int64(0)
    _check(lib().fd_cnn_wgrad_scratch(_shape3(shape), ctypes.byref(out)), "fd_cnn_wgrad_scratch")
    return int(out.value)


def fd_cnn_wgrad(x_ptr, cx, dz_ptr, cz, shape, scratch_ptr, scratch_floats, grad_ptr, stream):
    _check(lib().fd_cnn_wgrad(_vp(x_ptr), int(cx), _vp(dz_ptr), int(cz), _shape3(shape),
                              _vp(scratch_ptr), int(scratch_floats), _vp(grad_ptr), _vp(stream)),
           "fd_cnn_wgrad")


def fd_cnn_wgrad_noalloc(x_ptr, cx, dz_ptr, cz, shape, grad_ptr, stream):
    _check(lib().fd_cnn_wgrad_noalloc(_vp(x_ptr), int(cx), _vp(dz_ptr), int(cz), _shape3(shape),
                                      _vp(grad_ptr), _vp(stream)), "fd_cnn_wgrad_noalloc")


def fd_cnn_loss_grad(out_ptr, target_ptr, mask_ptr, nvox, cout, cpad, inv_n, dz_ptr, loss_ptr,
                     stream):
    _check(lib().fd_cnn_loss_grad(_vp(out_ptr), _vp(target_ptr), _vp(mask_ptr), int(nvox),
                                  int(cout), int(cpad), float(inv_n), _vp(dz_ptr), _vp(loss_ptr),
                                  _vp(stream)), "fd_cnn_loss_grad")


def fd_cnn_adam(p_ptr, g_ptr, m_ptr, v_ptr, n, t, lr, beta1, beta2, eps, stream):
    _check(lib().fd_cnn_adam(_vp(p_ptr), _vp(g_ptr), _vp(m_ptr), _vp(v_ptr), int(n), int(t),
                             float(lr), float(beta1), float(beta2), float(eps), _vp(stream)),
           "fd_cnn_adam")


def fd_cnn_features(ctx, vref, mask_ptr, bits_ptr, x_ptr, stream):
    _check(lib().fd_cnn_features(ctx, float(vref), _vp(mask_ptr), _vp(bits_ptr), _vp(x_ptr),
                                 _vp(stream)), "fd_cnn_features", ctx)


def fd_cnn_correct(ctx, d_ptr, mask_ptr, bits_ptr, stream):
    _check(lib().fd_cnn_correct(ctx, _vp(d_ptr), _vp(mask_ptr), _vp(bits_ptr), _vp(stream)),
           "fd_cnn_correct", ctx)


def fd_cnn_residual(ctx, ref_cur_ptr, ref_prev_ptr, bits_ptr, target_ptr, stream):
    _check(lib().fd_cnn_residual(ctx, _vp(ref_cur_ptr), _vp(ref_prev_ptr), _vp(bits_ptr),
                                 _vp(target_ptr), _vp(stream)), "fd_cnn_residual", ctx)


def fd_restrict(ctx, which, stride, dst_ptr, stream):
    _check(lib().fd_restrict(ctx, int(which), int(stride), _vp(dst_ptr), _vp(stream)),
           "fd_restrict", ctx)
