"""The allocation-free weight gradient (fd_cnn_wgrad_noalloc, for callers
that cannot allocate device memory) against fd_cnn_wgrad with a caller
scratch buffer, through the C ABI: the same kernels and summation order, so
the results must be bitwise equal.  Two calls in a row share the library's
scratch array; the second is smaller than the first and must not see the
first call's partial sums."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1608_03984_amd as P  # noqa: E402
from tests._gpu_util import say  # noqa: E402

pytestmark = pytest.mark.gpu
LAYER = P.FD_CNN_LAYER_FLOATS


def _bf16_bits(shape, c, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    v = torch.randn(shape + (c,), generator=g, device="cuda", dtype=torch.float32)
    return v.to(torch.bfloat16).view(torch.int16).contiguous()


def _both(shape, cx, cz, seed):
    x = _bf16_bits(shape, cx, seed)
    dz = _bf16_bits(shape, cz, seed + 1)
    st = torch.cuda.current_stream().cuda_stream
    ns = P.fd_cnn_wgrad_scratch(shape)
    assert ns <= P.FD_CNN_NOALLOC_SCRATCH_FLOATS
    scratch = torch.empty(ns, dtype=torch.float32, device="cuda")
    ref = torch.full((LAYER,), float("nan"), dtype=torch.float32, device="cuda")
    got = torch.full((LAYER,), float("nan"), dtype=torch.float32, device="cuda")
    P.fd_cnn_wgrad(x.data_ptr(), cx, dz.data_ptr(), cz, shape, scratch.data_ptr(), ns,
                   ref.data_ptr(), st)
    P.fd_cnn_wgrad_noalloc(x.data_ptr(), cx, dz.data_ptr(), cz, shape, got.data_ptr(), st)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_wgrad_equals_scratch_entry_point_on_two_calls():
    # first call: the 168^3 grid of the learned correction (1512 of the 1816
    # partial slots the array holds), then a smaller ragged grid
    for shape, cx, cz, seed in (((168, 168, 168), 16, 16, 5), ((11, 7, 45), 8, 16, 9)):
        say(f"case: no-alloc weight gradient {shape} cx{cx} cz{cz}")
        ref, got = _both(shape, cx, cz, seed)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32)), shape


def test_noalloc_wgrad_rejects_shapes_beyond_its_array():
    shape = (256, 256, 256)
    assert P.fd_cnn_wgrad_scratch(shape) > P.FD_CNN_NOALLOC_SCRATCH_FLOATS
    x = torch.zeros(16, dtype=torch.int16, device="cuda")
    g = torch.zeros(LAYER, dtype=torch.float32, device="cuda")
    with pytest.raises(P.FdError) as e:
        P.fd_cnn_wgrad_noalloc(x.data_ptr(), 16, x.data_ptr(), 16, shape, g.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    assert e.value.code == P.FD_ERR_WORKSPACE
