"""GPU parity of the adjoint and the velocity gradient (libfd's fd_adjoint,
fd_forward_checkpointed and fd_gradient through the C ABI) against the FP64
oracle.

Tolerances.  The adjoint run is a forward-type run of the same FP32 kernels,
so its output is held to the full-run bar of the forward path, relative L2
1e-4.  The gradient is a sum over time of products of two such FP32 fields
(adjoint state times the forward acceleration), each within 1e-4 of the
oracle's, summed in FP32 in two levels (partial sums of at most 32 steps):
relative L2 2e-4 (the sum of the two factors' bounds; the summation adds
rounding of order 32 eps relative to the sum of magnitudes).  The dot-product identity between the GPU forward and adjoint holds
to FP32 rounding of the two runs, 1e-5 relative to |Fq| |d|.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_1608_03984_amd as P  # noqa: E402
from paper_1608_03984_amd.solver import Solver, acoustic_modeling, from_problem  # noqa: E402
from tests._gpu_util import THREADS, acoustic_problem, rel, say  # noqa: E402
from workloads import smooth_random  # noqa: E402

pytestmark = pytest.mark.gpu


def observed(p, seed=99):
    """Oracle traces of the model with a smooth 4 % velocity perturbation
    (the 'observed' data of the misfit)."""
    rng = np.random.default_rng(seed)
    v = (p.vel.astype(np.float64) * (1 + 0.04 * smooth_random(p.vel.shape, 5.0, rng)))
    oracle.set_threads(THREADS)
    try:
        d, _, _ = oracle.acoustic_forward(p.ndim, p.nbl, p.spacing, p.dt, p.so,
                                          v.astype(np.float32), p.eta, p.src, p.wavelet, p.rec,
                                          p.nt)
    finally:
        oracle.set_threads(1)
    return d


def oracle_gradient(p, dobs):
    oracle.set_threads(THREADS)
    try:
        g, J = oracle.acoustic_gradient(p.ndim, p.nbl, p.spacing, p.dt, p.so, p.vel, p.eta, p.src,
                                        p.wavelet, p.rec, dobs, p.nt)
        tr, _, _ = oracle.acoustic_forward(p.ndim, p.nbl, p.spacing, p.dt, p.so, p.vel, p.eta,
                                           p.src, p.wavelet, p.rec, p.nt)
        qg = oracle.acoustic_adjoint(p.ndim, p.nbl, p.spacing, p.dt, p.so, p.vel, p.eta, p.src,
                                     p.rec, tr - dobs, p.nt)
    finally:
        oracle.set_threads(1)
    return g, J, qg


def with_sources(p, nsrc=3, seed=5):
    """The problem with several sources of distinct wavelets (so that the
    wavelet gradient has several columns)."""
    rng = np.random.default_rng(seed)
    src = np.repeat(p.src, nsrc, axis=0)
    span = np.array(p.shape, np.float64) * np.array(p.spacing)
    dims = [0, 2] if p.ndim == 2 else [0, 1, 2]
    src = src + (rng.random(src.shape) - 0.5) * 0.2 * span[dims]
    q = np.concatenate([p.wavelet * (1 + k) for k in range(nsrc)], axis=1).astype(np.float32)
    p.src, p.wavelet = src, q
    return p


@pytest.mark.parametrize("ndim,so", [(2, 4), (2, 16), (3, 2), (3, 8), (3, 16)])
def test_adjoint_vs_oracle(ndim, so):
    phys = (67, 1, 45) if ndim == 2 else (90, 37, 41)
    p = with_sources(acoustic_problem(ndim, phys, 6, so, 90, seed=200 + so))
    rng = np.random.default_rng(so)
    d = rng.standard_normal((p.nt, len(p.rec))).astype(np.float32)
    say(f"case: adjoint {ndim}d so{so} {p.padded}")
    s = from_problem(p)
    got = s.adjoint(p.nt, p.rec, d, p.src).cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    oracle.set_threads(THREADS)
    ref = oracle.acoustic_adjoint(ndim, p.nbl, p.spacing, p.dt, so, p.vel, p.eta, p.src, p.rec,
                                  d, p.nt)
    oracle.set_threads(1)
    e = rel(got, ref)
    say(f"  F^T d rel L2 {e:.2e}")
    assert e < 1e-4


@pytest.mark.parametrize("ndim,so", [(2, 8), (3, 4), (3, 12)])
def test_forward_adjoint_dot_product(ndim, so):
    phys = (70, 1, 50) if ndim == 2 else (80, 30, 33)
    p = with_sources(acoustic_problem(ndim, phys, 5, so, 70, seed=300 + so), nsrc=2)
    rng = np.random.default_rng(so + 1)
    q = rng.standard_normal(p.wavelet.shape).astype(np.float32)
    d = rng.standard_normal((p.nt, len(p.rec))).astype(np.float32)
    say(f"case: dot product {ndim}d so{so}")
    s = from_problem(p)
    fq = s.forward(p.nt, p.src, q, p.rec).cpu().numpy().astype(np.float64)
    ftd = s.adjoint(p.nt, p.rec, d, p.src).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    s.close()
    lhs, rhs = float(np.sum(fq * d)), float(np.sum(q * ftd))
    scale = np.linalg.norm(fq) * np.linalg.norm(d)
    say(f"  <Fq,d> {lhs:.6e}  <q,F^T d> {rhs:.6e}  gap/scale {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) < 1e-5 * scale


def gpu_gradient(p, dobs, interval=0, wrt="m"):
    s = from_problem(p)
    tr = s.forward_checkpointed(p.nt, p.src, p.wavelet, p.rec, interval=interval)
    res = tr - torch.from_numpy(dobs.astype(np.float32)).to(tr.device)
    g, qg = s.gradient(res, wrt=wrt)
    out = (g.cpu().numpy(), qg.cpu().numpy(), tr.cpu().numpy(), s.checkpoint_interval)
    torch.cuda.synchronize()
    s.close()
    return out


@pytest.mark.parametrize("ndim,so,interval", [(2, 4, 0), (2, 8, 13), (3, 2, 0), (3, 4, 1),
                                              (3, 8, 0), (3, 8, 7), (3, 8, 1000), (3, 16, 0)])
def test_gradient_vs_oracle(ndim, so, interval):
    """dJ/dm and dJ/dq of J = 1/2 |d - dobs|^2 on a damped multi-tile grid,
    for several checkpoint intervals (1 = checkpoint every step, 1000 = one
    segment, nothing recomputed)."""
    phys = (80, 1, 60) if ndim == 2 else (75, 30, 34)
    p = with_sources(acoustic_problem(ndim, phys, 6, so, 80, seed=400 + so), nsrc=2)
    dobs = observed(p)
    say(f"case: gradient {ndim}d so{so} interval {interval} {p.padded}")
    g, qg, tr, used = gpu_gradient(p, dobs, interval)
    gref, J, qref = oracle_gradient(p, dobs)
    eg, eq = rel(g, gref), rel(qg, qref)
    say(f"  interval used {used}  J {J:.4e}  grad rel L2 {eg:.2e}  wavelet grad {eq:.2e}")
    assert eg < 2e-4 and eq < 1e-4


def test_gradient_wrt_velocity_and_repeat():
    """The velocity gradient is dJ/dm * (-2 / v^3); a second fd_gradient call
    on the same store (the last segment now recomputed) gives the same bits."""
    p = acoustic_problem(3, (70, 24, 30), 5, 8, 60, seed=17)
    dobs = observed(p)
    say("case: gradient wrt v, repeated call")
    s = from_problem(p)
    tr = s.forward_checkpointed(p.nt, p.src, p.wavelet, p.rec, interval=9)
    res = tr - torch.from_numpy(dobs.astype(np.float32)).to(tr.device)
    gv1, q1 = s.gradient(res, wrt="vel")
    gv2, q2 = s.gradient(res, wrt="vel")
    gm, _ = s.gradient(res, wrt="m")
    gv1, gv2, q1, q2, gm = (t.cpu().numpy() for t in (gv1, gv2, q1, q2, gm))
    torch.cuda.synchronize()
    s.close()
    assert np.array_equal(gv1, gv2) and np.array_equal(q1, q2)
    gref, _, _ = oracle_gradient(p, dobs)
    v = p.vel.astype(np.float64)
    assert rel(gm, gref) < 2e-4
    assert rel(gv1, gref * (-2.0 / v ** 3)) < 2e-4


def test_misfit_vs_oracle():
    """fd_misfit: the residual is the FP32 difference of the traces and the
    observed data, and J matches the oracle's misfit of the same run."""
    p = acoustic_problem(3, (60, 20, 24), 5, 8, 50, seed=29)
    dobs = observed(p)
    say("case: misfit")
    s = from_problem(p)
    tr = s.forward(p.nt, p.src, p.wavelet, p.rec)
    do = torch.from_numpy(dobs.astype(np.float32)).to(tr.device)
    res = torch.empty_like(tr)
    J = torch.zeros(P.FD_MISFIT_DOUBLES, dtype=torch.float64, device=tr.device)
    st = torch.cuda.current_stream().cuda_stream
    P.fd_misfit(tr.data_ptr(), do.data_ptr(), tr.numel(), res.data_ptr(), J.data_ptr(), st)
    J1 = float(J[0].item())
    P.fd_misfit(tr.data_ptr(), do.data_ptr(), tr.numel(), res.data_ptr(), J.data_ptr(), st)
    torch.cuda.synchronize()
    got_res, got_J, d = res.cpu().numpy(), float(J[0].item()) / 2, tr.cpu().numpy()
    # the partials are summed in a fixed order: the second call adds the same bits
    assert float(J[0].item()) == 2 * J1
    s.close()
    assert np.array_equal(got_res, d - dobs.astype(np.float32))
    oracle.set_threads(THREADS)
    try:
        Jref = oracle.acoustic_misfit(p.ndim, p.nbl, p.spacing, p.dt, p.so, p.vel, p.eta, p.src,
                                      p.wavelet, p.rec, dobs, p.nt)
    finally:
        oracle.set_threads(1)
    say(f"  J {got_J:.6e} oracle {Jref:.6e}")
    assert abs(got_J - Jref) <= 2e-4 * Jref


@pytest.mark.parametrize("so,tile,interval", [(8, 0, 0), (8, 0, 7), (8, 0, 1), (4, 4, 7)])
def test_fused_imaging_gives_the_same_bits(so, tile, interval):
    """The imaging term fused into the adjoint stencil launch and the separate
    imaging kernel give bitwise equal gradients (same terms, same order, same
    fmaf), for several checkpoint intervals (1: every segment one step) and
    both single-shot tiles built with it (64 x 8 and 64 x 24)."""
    p = with_sources(acoustic_problem(3, (75, 30, 34), 6, so, 50, seed=77), nsrc=2)
    dobs = observed(p)
    say(f"case: fused imaging, so{so} tile{tile} interval {interval}")
    out = []
    for fused in (1, 0):
        s = from_problem(p)
        s.set_option(P.FD_OPT_TILE, tile)
        s.set_option(P.FD_OPT_FUSED_IMAGING, fused)
        tr = s.forward_checkpointed(p.nt, p.src, p.wavelet, p.rec, interval=interval)
        res = tr - torch.from_numpy(dobs.astype(np.float32)).to(tr.device)
        g, qg = s.gradient(res, wrt="m")
        out.append((g.cpu().numpy(), qg.cpu().numpy()))
        torch.cuda.synchronize()
        s.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_taylor_remainder_is_second_order():
    """Taylor test of the GPU gradient: R(e) = |J(v + e d) - J(v) - e <g, d>|
    falls as e^2 (ratio 4 per halving of e), J from fd_misfit of FP32 runs."""
    p = acoustic_problem(3, (60, 24, 30), 5, 8, 60, seed=31)
    dobs = torch.from_numpy(observed(p).astype(np.float32))
    say("case: Taylor test of the gradient")
    st = torch.cuda.current_stream().cuda_stream

    def J_of(vel, keep=None):
        s = Solver(3, p.shape, p.spacing, p.nbl, p.so, p.dt, vel, p.eta,
                   max_points=1 + p.rec.shape[0])
        if keep is None:
            tr = s.forward(p.nt, p.src, p.wavelet, p.rec)
        else:
            tr = s.forward_checkpointed(p.nt, p.src, p.wavelet, p.rec)
        J = torch.zeros(P.FD_MISFIT_DOUBLES, dtype=torch.float64, device=tr.device)
        do = dobs.to(tr.device)
        P.fd_misfit(tr.data_ptr(), do.data_ptr(), tr.numel(), tr.data_ptr(), J.data_ptr(), st)
        if keep is not None:
            g, _ = s.gradient(tr, wrt="vel", wavelet_grad=False)
            keep.append(g.cpu().numpy().astype(np.float64))
        torch.cuda.synchronize()
        s.close()
        return float(J[0].item())

    keep = []
    J0 = J_of(p.vel, keep)
    g = keep[0]
    d = smooth_random(p.vel.shape, 4.0, np.random.default_rng(7))
    d = (d / np.abs(d).max()).astype(np.float64)
    gd = float(np.sum(g * d))
    R = []
    for e in (8.0, 4.0, 2.0):
        Je = J_of((p.vel + e * d).astype(np.float32))
        R.append(abs(Je - J0 - e * gd))
    say(f"  J {J0:.4e}  <g,d> {gd:.4e}  remainders {R[0]:.3e} {R[1]:.3e} {R[2]:.3e}")
    assert 3.0 < R[0] / R[1] < 5.0 and 3.0 < R[1] / R[2] < 5.0


def test_gradient_accumulates_over_shots():
    """FD_GRAD_ACCUMULATE: the gradients of two shots (two source positions)
    summed into one buffer equal the FP32 sum of the separate gradients, and
    that sum matches the sum of the oracle's gradients."""
    import dataclasses
    p = acoustic_problem(3, (70, 24, 30), 5, 8, 60, seed=23)
    q = dataclasses.replace(p, src=p.src + np.array([[120.0, -30.0, 40.0]]))
    say("case: gradient accumulated over two shots")
    s = from_problem(p)
    gs, refs = [], []
    acc = torch.zeros(s.field_shape, dtype=torch.float32, device=s.device)
    for k, shot in enumerate((p, q)):
        dobs = observed(shot, seed=50 + k)
        tr = s.forward_checkpointed(shot.nt, shot.src, shot.wavelet, shot.rec, interval=7)
        res = tr - torch.from_numpy(dobs.astype(np.float32)).to(tr.device)
        g, _ = s.gradient(res, wrt="vel", wavelet_grad=False)
        gs.append(g.cpu().numpy())
        s.gradient(res, wrt="vel", wavelet_grad=False, accumulate_into=acc)
        refs.append(oracle_gradient(shot, dobs)[0] * (-2.0 / shot.vel.astype(np.float64) ** 3))
    got = acc.cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    assert np.array_equal(got, (gs[0] + gs[1]).astype(np.float32))
    e = rel(got, refs[0] + refs[1])
    say(f"  accumulated vs oracle sum: {e:.2e}")
    assert e < 2e-4


@pytest.mark.parametrize("so,sb,tile,nshots,interval",
                         [(8, 2, 2, 3, 7), (4, 0, 2, 5, 0), (16, 1, 0, 2, 11), (8, 2, 2, 4, 1),
                          (2, 4, 2, 3, 9)])
def test_gradient_shots_equal_single_shot_sum(so, sb, tile, nshots, interval):
    """A context of several shots forms its checkpointed forward runs,
    adjoints and imaging in shared launches (two shots per block where the
    tile configuration has that variant); its traces, wavelet gradients and
    the summed model gradient equal, bit for bit, one single-shot gradient
    per shot accumulated in shot order."""
    from tests.test_gpu_shots import survey
    p = acoustic_problem(3, (70, 24, 30), 5, so, 50, seed=600 + so)
    srcs, wavs, recs = survey(p, nshots, seed=so)
    rng = np.random.default_rng(so + nshots)
    adjs = [rng.standard_normal((p.nt, len(r))).astype(np.float32) for r in recs]
    say(f"case: gradient of {nshots} shots so{so} sb{sb} tile{tile} interval{interval}")
    npts = sum(len(a) for a in srcs) + sum(len(a) for a in recs) + 1
    s = Solver(3, p.shape, p.spacing, p.nbl, so, p.dt, p.vel, p.eta, nshots=nshots,
               max_points=npts)
    s.set_option(P.FD_OPT_TILE, tile)
    s.set_option(P.FD_OPT_SHOTS_PER_BLOCK, sb)
    trs = [t.cpu().numpy() for t in s.forward_checkpointed_shots(p.nt, srcs, wavs, recs,
                                                                  interval=interval)]
    g, qg = s.gradient_shots(adjs, wrt="vel", wavelet_grad=True)
    g, qg = g.cpu().numpy(), qg.cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    acc, col = None, 0
    for k in range(nshots):
        s1 = Solver(3, p.shape, p.spacing, p.nbl, so, p.dt, p.vel, p.eta, max_points=npts)
        t1 = s1.forward_checkpointed(p.nt, srcs[k], wavs[k], recs[k] if len(recs[k]) else None,
                                     interval=interval)
        assert np.array_equal(trs[k], t1.cpu().numpy()), f"shot {k} traces differ"
        g1, q1 = s1.gradient(adjs[k], wrt="vel", wavelet_grad=True, accumulate_into=acc)
        acc = g1
        ns = len(srcs[k])
        assert np.array_equal(qg[:, col:col + ns], q1.cpu().numpy()), f"shot {k} dJ/dq differs"
        col += ns
        torch.cuda.synchronize()
        s1.close()
    assert np.array_equal(g, acc.cpu().numpy())
    assert np.abs(g).max() > 0


def test_gradient_shots_errors():
    p = acoustic_problem(3, (30, 20, 20), 4, 8, 10, seed=77)
    say("case: gradient of several shots, error paths")
    s = Solver(3, p.shape, p.spacing, p.nbl, 8, p.dt, p.vel, p.eta, nshots=2, max_points=8)
    s1 = from_problem(p, max_points=8)
    nbytes, used = P.fd_checkpoint_bytes(s.ctx, p.nt, 0)
    one, used1 = P.fd_checkpoint_bytes(s1.ctx, p.nt, 0)
    assert used == used1 and 2 * one - 4096 <= nbytes <= 2 * one
    with pytest.raises(P.FdError) as e:   # a context of several shots needs the _shots calls
        s.forward_checkpointed(p.nt, p.src, p.wavelet, p.rec)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    s.forward_checkpointed_shots(p.nt, [p.src, p.src], [p.wavelet, p.wavelet],
                                 [p.rec[:1], p.rec[:1]])
    ck = s._ck
    grad = torch.empty(s.field_shape, device=s.device)
    with pytest.raises(P.FdError) as e:   # source counts that do not cover the points
        P.fd_gradient_shots(s.ctx, p.nt, ck["src"], np.array([1, 0]), ck["q"].data_ptr(), None,
                            None, 0, ck["interval"], ck["ptr"], ck["bytes"], P.FD_WRT_M,
                            grad.data_ptr(), 0, s.stream)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    with pytest.raises(P.FdError) as e:   # missing counts
        P.fd_gradient_shots(s.ctx, p.nt, ck["src"], None, ck["q"].data_ptr(), None, None, 0,
                            ck["interval"], ck["ptr"], ck["bytes"], P.FD_WRT_M, grad.data_ptr(),
                            0, s.stream)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    torch.cuda.synchronize()
    s.close()
    s1.close()


def test_autograd_function():
    """torch.autograd through AcousticModeling: vel.grad and wavelet.grad of
    1/2 |d - dobs|^2 against the oracle."""
    p = with_sources(acoustic_problem(3, (60, 26, 30), 5, 4, 70, seed=23), nsrc=2)
    dobs = observed(p)
    say("case: autograd")
    geom = dict(ndim=3, shape=p.shape, spacing=p.spacing, nbl=p.nbl, so=p.so, dt=p.dt, eta=p.eta,
                src=p.src, rec=p.rec)
    vel = torch.from_numpy(p.vel).cuda().requires_grad_(True)
    q = torch.from_numpy(p.wavelet.astype(np.float32)).cuda().requires_grad_(True)
    d = acoustic_modeling(vel, q, geom)
    loss = 0.5 * ((d - torch.from_numpy(dobs.astype(np.float32)).cuda()) ** 2).sum()
    loss.backward()
    gv, gq = vel.grad.cpu().numpy(), q.grad.cpu().numpy()
    torch.cuda.synchronize()
    gref, J, qref = oracle_gradient(p, dobs)
    say(f"  loss {loss.item():.6e} oracle J {J:.6e}")
    assert abs(loss.item() - J) < 1e-4 * J
    assert rel(gv, gref * (-2.0 / p.vel.astype(np.float64) ** 3)) < 2e-4
    assert rel(gq, qref) < 1e-4


def test_full_size_adjoint_dot_product():
    """The 592^3 grid (512^3 + 40-point layer) in the launch configuration of
    the benchmark: the forward/adjoint identity on a short run."""
    from workloads import acoustic_3d
    p = acoustic_3d(so=8, phys=512, nbl=40, nt=24, receivers="line")
    rng = np.random.default_rng(8)
    q = rng.standard_normal((p.nt, len(p.src))).astype(np.float32)
    d = rng.standard_normal((p.nt, len(p.rec))).astype(np.float32)
    say(f"case: full-size dot product {p.padded}")
    s = from_problem(p)
    fq = s.forward(p.nt, p.src, q, p.rec).cpu().numpy().astype(np.float64)
    ftd = s.adjoint(p.nt, p.rec, d, p.src).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    s.close()
    lhs, rhs = float(np.sum(fq * d)), float(np.sum(q * ftd))
    scale = np.linalg.norm(fq) * np.linalg.norm(d)
    say(f"  gap/scale {abs(lhs - rhs) / scale:.2e}")
    assert scale > 0 and abs(lhs - rhs) < 1e-5 * scale


def test_gradient_errors():
    p = acoustic_problem(3, (20, 20, 20), 4, 4, 10, seed=6)
    s = from_problem(p)
    say("case: gradient error paths")
    d = torch.zeros((p.nt, len(p.rec)), device="cuda")
    g = torch.empty(s.field_shape, device="cuda")
    # no checkpointed forward yet: rejected before any device work
    with pytest.raises(P.FdError) as e:
        P._binding.fd_gradient(s.ctx, p.nt, p.src, 0, p.rec, d.data_ptr(), 3, g.data_ptr(), 1 << 20,
                               P.FD_WRT_M, g.data_ptr(), 0, s.stream)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    s.forward_checkpointed(p.nt, p.src, p.wavelet, p.rec, interval=3)
    st = s._ck
    with pytest.raises(P.FdError) as e:   # a different interval than the forward run's
        P._binding.fd_gradient(s.ctx, p.nt, st["src"], st["q"].data_ptr(), st["rec"], d.data_ptr(),
                               4, st["ptr"], st["bytes"], P.FD_WRT_M, g.data_ptr(), 0, s.stream)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    with pytest.raises(P.FdError) as e:   # unknown wrt
        P._binding.fd_gradient(s.ctx, p.nt, st["src"], st["q"].data_ptr(), st["rec"], d.data_ptr(),
                               3, st["ptr"], st["bytes"], 7, g.data_ptr(), 0, s.stream)
    assert e.value.code == P.FD_ERR_INVALID_ARG
    with pytest.raises(P.FdError) as e:   # store too small
        P._binding.fd_forward_checkpointed(s.ctx, p.nt, st["src"], st["q"].data_ptr(), None, 0, 3,
                                           st["ptr"], 1024, s.stream)
    assert e.value.code == P.FD_ERR_WORKSPACE
    torch.cuda.synchronize()
    s.close()
    # TTI contexts have no gradient
    from tests._gpu_util import tti_problem
    t = tti_problem((20, 20, 20), 4, 4, 4, seed=3)
    st = from_problem(t)
    with pytest.raises(P.FdError) as e:
        st.forward_checkpointed(4, t.src, t.wavelet, t.rec)
    assert e.value.code == P.FD_ERR_UNSUPPORTED
    st.close()
