"""The launch configuration a context chooses by itself, read back with
fd_get_option: tiles of one block per compute unit (acoustic 64 x 24 up to
so 8, TTI 64 x 15 up to so 8) only where their x-y tiles number 90-100 % of
the device's compute units, the smaller tiles otherwise; a setting is read
back as set, and -1 returns to the default."""
import pytest

torch = pytest.importorskip("torch")

import paper_1608_03984_amd as P  # noqa: E402
from paper_1608_03984_amd.solver import Solver  # noqa: E402
from tests._gpu_util import say  # noqa: E402

pytestmark = pytest.mark.gpu


def fills_once(n_xy, tile_y, ncu):
    blocks = -(-n_xy // 64) * -(-n_xy // tile_y)
    return 10 * blocks >= 9 * ncu and blocks <= ncu


def context(phys_xy, so, physics="acoustic", nshots=1, nz=8, nbl=40):
    n = phys_xy + 2 * nbl
    shape = (nz + 2 * nbl, n, n)
    vel = torch.full(shape, 2000.0, device="cuda")
    kw = {}
    if physics != "acoustic":
        zero = torch.zeros(shape, device="cuda")
        kw = dict(epsilon=zero, delta=zero)
        if physics == "tti":
            kw.update(theta=zero, phi=zero)
    return Solver(3, (phys_xy, phys_xy, nz), (10.0, 10.0, 10.0), nbl, so, 1e-4, vel,
                  physics=physics, nshots=nshots, max_points=4, **kw), n


@pytest.mark.parametrize("phys_xy,so", [(512, 4), (512, 6), (512, 8), (512, 16), (420, 4)])
def test_acoustic_default_tile(phys_xy, so):
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    s, n = context(phys_xy, so)
    say(f"case: acoustic default tile {n}^2 x-y so{so}, {ncu} CUs")
    want = 4 if so <= 8 and fills_once(n, 24, ncu) else 0
    assert s.get_option(P.FD_OPT_TILE) == want
    assert s.get_option(P.FD_OPT_SHOTS_PER_BLOCK) == 1
    assert s.get_option(P.FD_OPT_ZCHUNK) == 0
    assert s.get_option(P.FD_OPT_DAMPING_PROFILE) == 1
    assert s.get_option(P.FD_OPT_FUSED_IMAGING) == 1
    s.set_option(P.FD_OPT_TILE, 2)
    assert s.get_option(P.FD_OPT_TILE) == 2
    s.set_option(P.FD_OPT_TILE, -1)
    assert s.get_option(P.FD_OPT_TILE) == want
    s.close()


@pytest.mark.parametrize("phys_xy,so", [(384, 8), (384, 4), (384, 12), (300, 8)])
def test_tti_default_tile(phys_xy, so):
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    s, n = context(phys_xy, so, physics="tti")
    say(f"case: tti default tile {n}^2 x-y so{so}, {ncu} CUs")
    want = 2 if so <= 8 and fills_once(n, 15, ncu) else 0
    assert s.get_option(P.FD_OPT_TILE) == want
    s.set_option(P.FD_OPT_TILE, 1)
    assert s.get_option(P.FD_OPT_TILE) == 1
    s.set_option(P.FD_OPT_TILE, -1)
    assert s.get_option(P.FD_OPT_TILE) == want
    s.close()


def test_shots_and_vti_defaults():
    s, _ = context(120, 8, nshots=4)
    say("case: shots and vti defaults")
    assert s.get_option(P.FD_OPT_TILE) == 2          # 64 x 8 of 512 threads
    assert s.get_option(P.FD_OPT_SHOTS_PER_BLOCK) == 2
    s.close()
    v, _ = context(120, 8, physics="vti")
    assert v.get_option(P.FD_OPT_TILE) == 0
    with pytest.raises(P.FdError) as e:
        v.get_option(99)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    v.close()
