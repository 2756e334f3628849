"""GPU parity of the TTI path (libfd through its C ABI) against the FP64
CPU oracle (same tolerances as the acoustic path)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1608_03984_amd as P  # noqa: E402
from paper_1608_03984_amd.solver import Solver, from_problem  # noqa: E402
from tests._gpu_util import (THREADS, oracle_run_with_peak, rel, sample_points, say,  # noqa: E402
                             tti_problem)
from workloads import noise_state, tti_3d  # noqa: E402

pytestmark = pytest.mark.gpu


def gpu_run(p, variant=0, damping_profile=None, tile=None):
    s = from_problem(p)
    if variant:
        s.set_option(P.FD_OPT_KERNEL, variant)
    if tile is not None:
        s.set_option(P.FD_OPT_TILE, tile)
    if damping_profile is not None:
        s.set_option(P.FD_OPT_DAMPING_PROFILE, damping_profile)
    tr = s.forward(p.nt, p.src, p.wavelet, p.rec)
    u = s.get_field(P.FD_FIELD_CUR)
    r = s.get_field(P.FD_FIELD_R_CUR)
    torch.cuda.synchronize()
    out = tr.cpu().numpy(), u.cpu().numpy(), r.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("so", [2, 4, 8])
@pytest.mark.parametrize("variant,tile", [(0, 0), (0, 1), (0, 2), (1, 0)])
def test_tti_multi_tile_full_run(so, variant, tile):
    """60 steps on a grid of several tiles in x and y (ragged in both) with
    the damping layer: the tiled kernel with 64 x 8 (tile 0), 64 x 4 (tile 1)
    and 64 x 15 (tile 2) tiles and the direct kernel (variant 1)."""
    p = tti_problem((80, 26, 22), 6, so, 60, seed=200 + so)
    say(f"case: tti {p.padded} so{so} variant{variant} tile{tile}")
    tr, u, r = gpu_run(p, variant, tile=tile)
    tref, st, peak = oracle_run_with_peak(p, chunk=20)
    et = rel(tr, tref)
    eu = float(np.linalg.norm(u - st[1]) / peak)
    er = float(np.linalg.norm(r - st[3]) / max(np.linalg.norm(st[3]), 1e-30))
    say(f"  traces {et:.2e}  p/peak {eu:.2e}  r {er:.2e}")
    assert et < 1e-4 and eu < 1e-4 and er < 1e-4


@pytest.mark.parametrize("tile", [0, 1, 2])
def test_tti_damping_profiles(tile):
    """The tiled TTI kernel with the layer evaluated from its per-axis
    profiles matches the run that reads the damping field (through the
    per-tile damping flags), for every tile shape."""
    p = tti_problem((90, 37, 30), 6, 8, 60, seed=590)
    say(f"case: tti damping profiles {p.padded} tile{tile}")
    on, off = gpu_run(p, tile=tile), gpu_run(p, damping_profile=0, tile=tile)
    e = [rel(a, b) for a, b in zip(on, off)]
    say(f"  profiles vs field: traces {e[0]:.2e} p {e[1]:.2e} r {e[2]:.2e}")
    assert max(e) < 1e-6


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16])
@pytest.mark.parametrize("tile", [0, 1, 2])
def test_tti_one_step_from_common_state(so, tile):
    """One step from a common noise state at every point, for every tile
    shape of the tiled kernel (64 x 8, 64 x 4, and 64 x 15 up to so 8)."""
    if tile == 2 and so > 8:
        pytest.skip("the 64 x 15 tile is built for space orders up to 8")
    p = tti_problem((70, 18, 20), 4, so, 1, seed=so)
    shape = p.padded
    st = [noise_state(shape, 20 + k) for k in range(4)]
    say(f"case: tti one step so{so} {shape} tile{tile}")
    s = from_problem(p)
    s.set_option(P.FD_OPT_TILE, tile)
    for which, f in zip((P.FD_FIELD_PREV, P.FD_FIELD_CUR, P.FD_FIELD_R_PREV, P.FD_FIELD_R_CUR), st):
        s.set_field(which, f)
    s.forward(1, zero_state=False)
    gp = s.get_field(P.FD_FIELD_CUR).cpu().numpy().ravel()
    gr = s.get_field(P.FD_FIELD_R_CUR).cpu().numpy().ravel()
    torch.cuda.synchronize()
    s.close()
    pts = np.arange(gp.size)
    oracle.set_threads(THREADS)
    rp, rr = oracle.tti_step_points(p.spacing, p.dt, so, p.vel, p.eta, p.eps, p.delta, p.theta,
                                    p.phi, st, pts)
    oracle.set_threads(1)
    ep, er = rel(gp, rp), rel(gr, rr)
    say(f"  one-step rel L2 p {ep:.2e} r {er:.2e}")
    assert ep < 1e-5 and er < 1e-5


def test_tti_full_size_one_step_sampled():
    """464^3 (384^3 + 40-point layer), so 8: one step from a common state at
    sampled points, in the launch configuration the benchmark times."""
    say("generating the 384^3 (+40 layer) TTI workload model")
    p = tti_3d(so=8, phys=384, nbl=40, nt=1, receivers="none")
    shape = p.padded
    st = [noise_state(shape, 30 + k) for k in range(4)]
    say(f"case: tti full-size one step {shape}")
    s = Solver(3, p.shape, p.spacing, p.nbl, 8, p.dt, p.vel, p.eta, physics="tti",
               epsilon=p.eps, delta=p.delta, theta=p.theta, phi=p.phi, max_points=16)
    for which, f in zip((P.FD_FIELD_PREV, P.FD_FIELD_CUR, P.FD_FIELD_R_PREV, P.FD_FIELD_R_CUR), st):
        s.set_field(which, f)
    s.forward(1, zero_state=False)
    gp = s.get_field(P.FD_FIELD_CUR).cpu().numpy().ravel()
    gr = s.get_field(P.FD_FIELD_R_CUR).cpu().numpy().ravel()
    torch.cuda.synchronize()
    s.close()
    pts = sample_points(shape, 4000, seed=8, radius=4)
    oracle.set_threads(THREADS)
    rp, rr = oracle.tti_step_points(p.spacing, p.dt, 8, p.vel, p.eta, p.eps, p.delta, p.theta,
                                    p.phi, st, pts)
    oracle.set_threads(1)
    ep, er = rel(gp[pts], rp), rel(gr[pts], rr)
    say(f"  sampled one-step rel L2 p {ep:.2e} r {er:.2e}")
    assert ep < 1e-5 and er < 1e-5


def test_tti_tall_tile_limited_to_so8():
    """The 64 x 15 tile is refused above so 8 (its 960-thread blocks fit
    128 registers per lane only up to radius 4) and out-of-range tiles are
    refused; the context keeps its previous tile, and -1 (the default for
    the order) is accepted."""
    p = tti_problem((20, 20, 20), 2, 12, 1, seed=3)
    s = from_problem(p)
    with pytest.raises(P.FdError) as e:
        s.set_option(P.FD_OPT_TILE, 2)
    assert e.value.code == P.FD_ERR_UNSUPPORTED
    with pytest.raises(P.FdError) as e:
        s.set_option(P.FD_OPT_TILE, 3)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    s.set_option(P.FD_OPT_TILE, -1)
    s.forward(1)
    torch.cuda.synchronize()
    s.close()


def test_tti_rejects_delta_above_epsilon():
    p = tti_problem((20, 20, 20), 2, 4, 1, seed=1)
    bad = p.delta.copy()
    bad[5, 5, 5] = p.eps[5, 5, 5] + 0.05
    with pytest.raises(P.FdError) as e:
        Solver(3, p.shape, p.spacing, p.nbl, 4, p.dt, p.vel, p.eta, physics="tti",
               epsilon=p.eps, delta=bad, theta=p.theta, phi=p.phi)
    assert e.value.code == P.FD_ERR_INVALID_ARG
