"""GPU parity of the VTI path (libfd through its C ABI) against the FP64
CPU oracle (same tolerances as the acoustic path: one step 1e-5, full runs
1e-4)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1608_03984_amd as P  # noqa: E402
from paper_1608_03984_amd.solver import Solver, from_problem  # noqa: E402
from tests._gpu_util import (THREADS, oracle_run_with_peak, rel, sample_points, say,  # noqa: E402
                             vti_problem)
from workloads import noise_state, vti_3d  # noqa: E402

pytestmark = pytest.mark.gpu
FIELDS = (P.FD_FIELD_PREV, P.FD_FIELD_CUR, P.FD_FIELD_R_PREV, P.FD_FIELD_R_CUR)


def gpu_run(p, variant=0, damping_profile=None):
    s = from_problem(p)
    if variant:
        s.set_option(P.FD_OPT_KERNEL, variant)
    if damping_profile is not None:
        s.set_option(P.FD_OPT_DAMPING_PROFILE, damping_profile)
    tr = s.forward(p.nt, p.src, p.wavelet, p.rec)
    u = s.get_field(P.FD_FIELD_CUR)
    r = s.get_field(P.FD_FIELD_R_CUR)
    torch.cuda.synchronize()
    out = tr.cpu().numpy(), u.cpu().numpy(), r.cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("so", [2, 4, 8, 16])
@pytest.mark.parametrize("variant", [0, 1])
def test_vti_3d_multi_tile_full_run(so, variant):
    p = vti_problem(3, (90, 37, 30), 6, so, 70, seed=300 + so)
    say(f"case: vti {p.padded} so{so} variant{variant}")
    tr, u, r = gpu_run(p, variant)
    tref, st, peak = oracle_run_with_peak(p, chunk=35)
    et = rel(tr, tref)
    eu = float(np.linalg.norm(u - st[1]) / peak)
    er = float(np.linalg.norm(r - st[3]) / max(np.linalg.norm(st[3]), 1e-30))
    say(f"  traces {et:.2e}  p/peak {eu:.2e}  r {er:.2e}")
    assert et < 1e-4 and eu < 1e-4 and er < 1e-4


def test_vti_damping_profiles():
    """The tiled VTI kernel with the layer evaluated from its per-axis
    profiles matches the run that reads the damping field."""
    p = vti_problem(3, (90, 37, 30), 6, 8, 70, seed=390)
    say(f"case: vti damping profiles {p.padded}")
    on, off = gpu_run(p), gpu_run(p, damping_profile=0)
    e = [rel(a, b) for a, b in zip(on, off)]
    say(f"  profiles vs field: traces {e[0]:.2e} p {e[1]:.2e} r {e[2]:.2e}")
    assert max(e) < 1e-6


@pytest.mark.parametrize("so", [4, 8, 16])
def test_vti_2d_full_run(so):
    p = vti_problem(2, (150, 1, 90), 10, so, 120, seed=310 + so)
    say(f"case: vti 2d {p.padded} so{so}")
    tr, u, r = gpu_run(p)
    tref, st, peak = oracle_run_with_peak(p, chunk=60)
    et, eu = rel(tr, tref), float(np.linalg.norm(u - st[1]) / peak)
    say(f"  traces {et:.2e}  p/peak {eu:.2e}")
    assert et < 1e-4 and eu < 1e-4


@pytest.mark.parametrize("ndim,so", [(3, 2), (3, 4), (3, 6), (3, 8), (3, 12), (3, 16), (2, 8)])
def test_vti_one_step_from_common_state(ndim, so):
    phys = (70, 18, 20) if ndim == 3 else (80, 1, 60)
    p = vti_problem(ndim, phys, 4, so, 1, seed=so)
    shape = p.padded
    st = [noise_state(shape, 40 + k) for k in range(4)]
    say(f"case: vti one step {ndim}d so{so} {shape}")
    s = from_problem(p)
    for which, f in zip(FIELDS, st):
        s.set_field(which, f)
    s.forward(1, zero_state=False)
    gp = s.get_field(P.FD_FIELD_CUR).cpu().numpy().ravel()
    gr = s.get_field(P.FD_FIELD_R_CUR).cpu().numpy().ravel()
    torch.cuda.synchronize()
    s.close()
    pts = np.arange(gp.size)
    oracle.set_threads(THREADS)
    rp, rr = oracle.vti_step_points(ndim, p.spacing, p.dt, so, p.vel, p.eta, p.eps, p.delta, st,
                                    pts)
    oracle.set_threads(1)
    ep, er = rel(gp, rp), rel(gr, rr)
    say(f"  one-step rel L2 p {ep:.2e} r {er:.2e}")
    assert ep < 1e-5 and er < 1e-5


def test_vti_full_size_one_step_sampled():
    """464^3 (384^3 + 40-point layer), so 8: one step from a common state at
    sampled points, in the launch configuration the benchmark times."""
    p = vti_3d(so=8, phys=384, nbl=40, nt=1, receivers="none")
    shape = p.padded
    st = [noise_state(shape, 50 + k) for k in range(4)]
    say(f"case: vti full-size one step {shape}")
    s = Solver(3, p.shape, p.spacing, p.nbl, 8, p.dt, p.vel, p.eta, physics="vti",
               epsilon=p.eps, delta=p.delta, max_points=16)
    for which, f in zip(FIELDS, st):
        s.set_field(which, f)
    s.forward(1, zero_state=False)
    gp = s.get_field(P.FD_FIELD_CUR).cpu().numpy().ravel()
    gr = s.get_field(P.FD_FIELD_R_CUR).cpu().numpy().ravel()
    torch.cuda.synchronize()
    s.close()
    pts = sample_points(shape, 6000, seed=8, radius=4)
    oracle.set_threads(THREADS)
    rp, rr = oracle.vti_step_points(3, p.spacing, p.dt, 8, p.vel, p.eta, p.eps, p.delta, st, pts)
    oracle.set_threads(1)
    ep, er = rel(gp[pts], rp), rel(gr[pts], rr)
    say(f"  sampled one-step rel L2 p {ep:.2e} r {er:.2e}")
    assert ep < 1e-5 and er < 1e-5


def test_vti_equals_tti_without_tilt_on_gpu():
    """The VTI kernels against the TTI kernels with zero angles (same FP32
    coefficients; the operators differ only by exact zeros)."""
    p = vti_problem(3, (70, 24, 26), 5, 8, 50, seed=77)
    say("case: vti vs tti(0, 0)")
    tr, u, r = gpu_run(p)
    z = np.zeros_like(p.vel)
    s = Solver(3, p.shape, p.spacing, p.nbl, 8, p.dt, p.vel, p.eta, physics="tti", epsilon=p.eps,
               delta=p.delta, theta=z, phi=z, max_points=64)
    tt = s.forward(p.nt, p.src, p.wavelet, p.rec).cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    assert rel(tr, tt) < 1e-5


def test_vti_rejections():
    p = vti_problem(3, (20, 20, 20), 4, 4, 2, seed=3)
    say("case: vti rejections")
    bad = p.delta.copy()
    bad[5, 5, 5] = p.eps[5, 5, 5] + 0.05
    with pytest.raises(P.FdError) as e:
        Solver(3, p.shape, p.spacing, p.nbl, 4, p.dt, p.vel, p.eta, physics="vti", epsilon=p.eps,
               delta=bad)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    with pytest.raises(P.FdError) as e:
        Solver(3, p.shape, p.spacing, p.nbl, 4, p.dt, p.vel, p.eta, physics="vti", epsilon=p.eps,
               delta=p.delta, nshots=2)
    assert e.value.code == P.FD_ERR_UNSUPPORTED
    with pytest.raises(P.FdError) as e:   # CFL at the horizontal speed v sqrt(1 + 2 eps)
        Solver(3, p.shape, p.spacing, p.nbl, 4, p.dt * 2.6, p.vel, p.eta, physics="vti",
               epsilon=p.eps, delta=p.delta)
    assert e.value.code == P.FD_ERR_UNSTABLE_DT
