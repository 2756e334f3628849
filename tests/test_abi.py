"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/fd.h declares, and its host-side helpers and argument
validation behave (no call here reaches the device)."""
import ctypes
import re
import subprocess
from pathlib import Path

import numpy as np
import pytest

import oracle
import paper_1608_03984_amd as P

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "fd.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(fd_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("fd_workspace_bytes", "fd_setup", "fd_forward", "fd_destroy", "fd_strerror",
              "fd_last_error", "fd_get_field", "fd_set_field"):
        assert n in names
    assert set(names) == set(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", str(Path(P._binding._LIBPATH))],
                         capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in declared_functions():
        assert n in exported, n
        assert hasattr(lib, n)


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_library_weights_match_oracle(so):
    np.testing.assert_allclose(P.fd_stencil_weights(so, 2), oracle.weights_d2(so), rtol=0,
                               atol=1e-14)
    np.testing.assert_allclose(P.fd_stencil_weights(so, 1), oracle.weights_d1(so), rtol=0,
                               atol=1e-14)


def test_library_weights_reject_bad_orders():
    with pytest.raises(P.FdError) as e:
        P.fd_stencil_weights(18, 2)
    assert e.value.code == P.FD_ERR_UNSUPPORTED
    with pytest.raises(P.FdError):
        P.fd_stencil_weights(3, 2)
    with pytest.raises(P.FdError):
        P.fd_stencil_weights(4, 3)


@pytest.mark.parametrize("ndim,so,h", [(2, 4, (10, 1, 10)), (3, 8, (10, 12, 8)),
                                       (3, 16, (12.5, 12.5, 12.5))])
def test_library_cfl_matches_oracle(ndim, so, h):
    g = P.make_grid(ndim, (50, 1 if ndim == 2 else 40, 30), h, 10, so, 1e-3)
    assert abs(P.fd_cfl_dt(g, 3000.0) - oracle.cfl_dt(ndim, so, h, 3000.0)) < 1e-15


def _code(fn):
    try:
        fn()
    except P.FdError as e:
        return e.code
    return P.FD_OK


def test_workspace_validation_codes():
    ok = P.make_grid(3, (64, 64, 64), (10, 10, 10), 8, 8, 1e-4)
    assert P.fd_workspace_bytes(ok, 10) > 6 * 64 ** 3 * 4
    bad = [
        (P.make_grid(4, (8, 8, 8), (1, 1, 1), 0, 4, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (8, 8, 8), (1, 1, 1), 0, 18, 1e-3), P.FD_ERR_UNSUPPORTED),
        (P.make_grid(3, (8, 8, 8), (1, 1, 1), 0, 5, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (8, 8, 8), (1, 1, 1), 0, 0, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(2, (8, 1, 8), (1, 1, 1), 0, 4, 1e-3, P.FD_TTI), P.FD_ERR_UNSUPPORTED),
        (P.make_grid(2, (8, 2, 8), (1, 1, 1), 0, 4, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (8, 8, 8), (1, 0, 1), 0, 4, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (8, 8, 8), (1, 1, 1), 0, 4, 0.0), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (0, 8, 8), (1, 1, 1), 0, 4, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (8, 8, 8), (1, 1, 1), -1, 4, 1e-3), P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (8, 8, 8), (1, 1, 1), 0, 4, 1e-3, 7), P.FD_ERR_INVALID_ARG),
        # beyond 2^40 padded points (byte counts would approach 64-bit overflow)
        (P.make_grid(3, (1 << 20, 1 << 20, 1 << 20), (1, 1, 1), 0, 4, 1e-3),
         P.FD_ERR_INVALID_ARG),
        (P.make_grid(3, (1 << 14, 1 << 14, 1 << 13), (1, 1, 1), 0, 4, 1e-3),
         P.FD_ERR_INVALID_ARG),
    ]
    for g, code in bad:
        assert _code(lambda: P.fd_workspace_bytes(g, 1)) == code
    assert _code(lambda: P.fd_workspace_bytes(ok, -1)) == P.FD_ERR_INVALID_ARG
    # the injection plan codes a point index in 29 bits: at most 2^27 points
    assert P.fd_workspace_bytes(ok, 1 << 27) > 0
    assert _code(lambda: P.fd_workspace_bytes(ok, (1 << 27) + 1)) == P.FD_ERR_INVALID_ARG


def test_setup_rejects_before_device_work():
    """Argument errors are reported before any HIP call is made."""
    g = P.make_grid(3, (16, 16, 16), (10, 10, 10), 4, 4, 1e-4)
    need = P.fd_workspace_bytes(g, 4)
    m = P.FdModel()
    m.vel = None
    assert _code(lambda: P.fd_setup(g, m, 4096, need, 4, 0)) == P.FD_ERR_INVALID_ARG
    m.vel = 0x1000
    assert _code(lambda: P.fd_setup(g, m, 0, need, 4, 0)) == P.FD_ERR_INVALID_ARG
    assert _code(lambda: P.fd_setup(g, m, 4096 + 4, need, 4, 0)) == P.FD_ERR_WORKSPACE
    assert _code(lambda: P.fd_setup(g, m, 4096, need - 1, 4, 0)) == P.FD_ERR_WORKSPACE
    gt = P.make_grid(3, (16, 16, 16), (10, 10, 10), 4, 4, 1e-4, P.FD_TTI)
    assert _code(lambda: P.fd_setup(gt, m, 4096, 1 << 40, 4, 0)) == P.FD_ERR_INVALID_ARG


def test_null_context_and_strings():
    lib = P.lib()
    assert lib.fd_forward(None, 1, None, None, 0, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_get_field(None, 0, None, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_set_option(None, 1, 0) == P.FD_ERR_INVALID_ARG
    assert lib.fd_get_option(None, 1, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_destroy(None) == P.FD_OK
    assert P.fd_last_error(None) == ""
    for c in range(8):
        assert len(P.fd_strerror(c)) > 3 and P.fd_strerror(c) != "unknown status"
    assert "host" in P.fd_strerror(P.FD_ERR_HOST)
    assert P.fd_strerror(99) == "unknown status"


def test_binding_status_codes_match_the_header():
    """Every FD_ERR_* status the header defines has the same value in the
    binding."""
    hdr = (Path(__file__).resolve().parent.parent / "include" / "fd.h").read_text()
    codes = dict(re.findall(r"#define (FD_(?:OK|ERR_[A-Z_]+)) (\d+)", hdr))
    assert "FD_ERR_HOST" in codes
    for name, value in codes.items():
        assert getattr(P, name) == int(value), name


def test_triad_config_rejects_bad_shapes():
    lib = P.lib()
    a = ctypes.c_void_p(256)  # aligned dummies: rejected before any device work
    for unroll, blocks, flags in ((3, 0, 0), (0, 0, 0), (16, 0, 0), (4, -1, 0), (4, 0, 2)):
        assert lib.fd_triad_config(a, a, a, 1.0, 64, unroll, blocks, flags,
                                   None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_triad_config(ctypes.c_void_p(4), a, a, 1.0, 64, 1, 0, 0,
                               None) == P.FD_ERR_INVALID_ARG  # misaligned


def test_noalloc_wgrad_rejects_before_device_work():
    """The allocation-free weight gradient checks its arguments and its
    array's capacity on the host: shapes beyond FD_CNN_NOALLOC_SCRATCH_FLOATS
    give FD_ERR_WORKSPACE, bad channels or pointers FD_ERR_INVALID_ARG."""
    lib = P.lib()
    a = ctypes.c_void_p(256)
    big = (ctypes.c_int64 * 3)(256, 256, 256)
    ok = (ctypes.c_int64 * 3)(16, 16, 16)
    assert P.fd_cnn_wgrad_scratch((256, 256, 256)) > P.FD_CNN_NOALLOC_SCRATCH_FLOATS
    assert P.fd_cnn_wgrad_scratch((168, 168, 168)) <= P.FD_CNN_NOALLOC_SCRATCH_FLOATS
    assert lib.fd_cnn_wgrad_noalloc(a, 16, a, 16, big, a, None) == P.FD_ERR_WORKSPACE
    assert lib.fd_cnn_wgrad_noalloc(a, 8, a, 8, ok, a, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_cnn_wgrad_noalloc(None, 16, a, 16, ok, a, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_cnn_wgrad_noalloc(a, 16, a, 16, ok, None, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_cnn_wgrad_noalloc(a, 16, a, 16, None, a, None) == P.FD_ERR_INVALID_ARG


def test_gradient_entry_points_reject_null_context():
    lib = P.lib()
    u64 = ctypes.c_uint64(0)
    assert lib.fd_checkpoint_bytes(None, 10, 0, ctypes.byref(u64), None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_forward_checkpointed(None, 10, None, None, 0, None, 0, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_gradient(None, 10, None, None, 0, None, 0, P.FD_WRT_M, None, None,
                           None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_adjoint(None, 10, None, None, None) == P.FD_ERR_INVALID_ARG
    # the misfit: missing buffers and negative sizes are rejected, n = 0 is a no-op
    assert lib.fd_misfit(None, None, 5, None, None, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_misfit(None, None, -1, None, None, None) == P.FD_ERR_INVALID_ARG
    assert lib.fd_misfit(None, None, 0, None, None, None) == P.FD_OK
