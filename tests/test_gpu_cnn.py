"""GPU parity of the correction network's kernels (libfd's fd_cnn_* through
the C ABI) against the FP64 oracle of oracle/cnn.py.

Tolerances.  Inputs and weights are rounded to BF16 the same way on both
sides (round to nearest even), so a single layer differs only by FP32
accumulation order (relative 1e-5 on FP32 outputs) and, for BF16 outputs, by
at most one BF16 unit (2^-7 relative) where the FP32 value straddles a
rounding boundary.  The weight gradient sums over every voxel in FP32:
relative L2 1e-4.  Through the whole network every intermediate BF16 rounding
(two activations, two back-propagated gradients) adds up to 2^-9 relative
error per element, so the end-to-end parameter gradient is held to relative
L2 3e-2 per layer.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1608_03984_amd as P  # noqa: E402
from oracle import cnn as C  # noqa: E402
from paper_1608_03984_amd.learned import CorrectionNet  # noqa: E402
from tests._gpu_util import say  # noqa: E402

pytestmark = pytest.mark.gpu
LAYER = P.FD_CNN_LAYER_FLOATS


def bf16_bits(a):
    """FP32 values -> BF16 bit patterns (RNE) as int16, and their values."""
    r = C.bf16_round(a)
    bits = (np.ascontiguousarray(r, np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return bits.view(np.int16), r


def from_bits(b):
    u = np.asarray(b).view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def layer_params(rng, cin, cout, scale=0.3):
    p = np.zeros(LAYER, np.float32)
    w = p[:27 * 256].reshape(27, 16, 16)
    w[:, :cin, :cout] = rng.standard_normal((27, cin, cout)) * scale
    p[27 * 256:27 * 256 + cout] = rng.standard_normal(cout) * 0.1
    return p


def st():
    return torch.cuda.current_stream().cuda_stream


SHAPES = [(3, 5, 70), (4, 9, 33), (2, 4, 130), (37, 6, 70)]


@pytest.mark.parametrize("cin,mode", [(8, 0), (8, 1), (16, 0), (16, 1), (8, 2), (16, 2), (16, 3),
                                      (8, 4), (16, 4)])
@pytest.mark.parametrize("shape", SHAPES)
def test_conv_vs_oracle(cin, mode, shape):
    rng = np.random.default_rng(cin * 10 + mode + shape[2])
    D, H, W = shape
    creal = 3 if cin == 8 else 16
    x = np.zeros(shape + (cin,), np.float32)
    x[..., :creal] = rng.standard_normal(shape + (creal,))
    xb, xv = bf16_bits(x)
    back = mode in (2, 4)
    if back:
        # backward-data: the layer maps 16 -> cin' channels in the forward
        # direction; its transpose takes cin channels (real ones) to 16
        p = layer_params(rng, 16, creal)
    else:
        p = layer_params(rng, creal, 2 if mode == 1 else 16)
    w = p[:27 * 256].reshape(27, 16, 16)
    wr = C.bf16_round(w)
    say(f"case: conv cin{cin} mode{mode} {shape}")
    pk = torch.empty(P.fd_cnn_packed_elems(cin), dtype=torch.int16, device="cuda")
    pd = dev(p)
    P.fd_cnn_pack(pd.data_ptr(), cin, 1 if back else 0, pk.data_ptr(), st())
    V = D * H * W
    xd = dev(xb.reshape(-1))
    mask_np = None
    if mode == 2:
        mvals = np.maximum(rng.standard_normal(shape + (16,)), 0).astype(np.float32)
        mb, mask_np = bf16_bits(mvals)
        md = dev(mb.reshape(-1))
    y = torch.zeros(V * 16, dtype=torch.int16, device="cuda")
    yf = torch.zeros(V * 2, dtype=torch.float32, device="cuda")
    P.fd_cnn_conv(xd.data_ptr(), cin, shape, pk.data_ptr(), pd.data_ptr() + 4 * 27 * 256, mode,
                  md.data_ptr() if mode == 2 else 0, 2, y.data_ptr(), yf.data_ptr(), st())
    torch.cuda.synchronize()
    if mode in (0, 3):
        ref = C.conv3d(xv, wr[:, :cin, :], p[27 * 256:27 * 256 + 16])
        if mode == 0:
            ref = np.maximum(ref, 0)
        got = from_bits(y.cpu().numpy()).reshape(ref.shape)
    elif mode == 1:
        ref = C.conv3d(xv, wr[:, :cin, :2], p[27 * 256:27 * 256 + 2])
        got = yf.cpu().numpy().reshape(ref.shape)
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        say(f"  FP32 output rel L2 {e:.2e}")
        assert e < 1e-5
        return
    else:
        # input channels of the transpose are the forward layer's outputs
        ref = C.conv3d_backward_data(xv[..., :creal] if cin == 8 else xv, wr[:, :, :creal]
                                     if cin == 8 else wr)
        if mode == 2:
            ref = ref * (mask_np > 0)
        got = from_bits(y.cpu().numpy()).reshape(ref.shape)
    # one BF16 unit and a half, plus FP32 accumulation noise near zero
    tol = 1.5 * 2.0 ** -7 * np.abs(ref) + 1e-5 * np.abs(ref).max()
    bad = np.abs(got - ref) > tol
    say(f"  BF16 outputs beyond one unit: {int(bad.sum())} of {ref.size}; rel L2 "
        f"{np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
    assert not bad.any()


@pytest.mark.parametrize("cx,cz", [(8, 16), (16, 16), (16, 8)])
def test_weight_gradient_vs_oracle(cx, cz):
    rng = np.random.default_rng(cx + cz)
    shape = (11, 7, 45)
    xr, zr = (3 if cx == 8 else 16), (2 if cz == 8 else 16)
    x = np.zeros(shape + (cx,), np.float32)
    x[..., :xr] = rng.standard_normal(shape + (xr,))
    dz = np.zeros(shape + (cz,), np.float32)
    dz[..., :zr] = rng.standard_normal(shape + (zr,))
    xb, xv = bf16_bits(x)
    zb, zv = bf16_bits(dz)
    say(f"case: weight gradient cx{cx} cz{cz}")
    ns = P.fd_cnn_wgrad_scratch(shape)
    scratch = torch.empty(ns, dtype=torch.float32, device="cuda")
    g = torch.zeros(LAYER, dtype=torch.float32, device="cuda")
    xd, zd = dev(xb.reshape(-1)), dev(zb.reshape(-1))
    P.fd_cnn_wgrad(xd.data_ptr(), cx, zd.data_ptr(), cz, shape, scratch.data_ptr(), ns,
                   g.data_ptr(), st())
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    dw, db = C.conv3d_backward_weight(xv, zv)
    gw = got[:27 * 256].reshape(27, 16, 16)[:, :cx, :cz]
    e = np.linalg.norm(gw - dw) / np.linalg.norm(dw)
    eb = np.linalg.norm(got[27 * 256:27 * 256 + cz] - db) / np.linalg.norm(db)
    say(f"  dW rel L2 {e:.2e}  db rel L2 {eb:.2e}")
    assert e < 1e-4 and eb < 1e-4
    # channels beyond the real ones stay exactly zero
    assert np.all(got[:27 * 256].reshape(27, 16, 16)[:, cx:, :] == 0)
    assert np.all(got[:27 * 256].reshape(27, 16, 16)[:, :, cz:] == 0)


def test_network_gradient_and_adam_vs_oracle():
    """End to end: forward, masked loss, backward and one Adam step of the
    three-layer network against the FP64 oracle on the same BF16 inputs and
    BF16-rounded weights."""
    rng = np.random.default_rng(9)
    shape = (6, 10, 40)
    V = int(np.prod(shape))
    net = CorrectionNet(seed=4, out_scale=1.0)
    # non-zero biases here, to check their gradients too
    net.params[:, 27 * 256:] = torch.from_numpy(
        rng.standard_normal((3, 16)).astype(np.float32) * 0.1).cuda()
    x = np.zeros(shape + (8,), np.float32)
    x[..., :4] = rng.standard_normal(shape + (4,))
    xb, xv = bf16_bits(x)
    target = rng.standard_normal(shape + (2,)).astype(np.float32)
    mask = np.zeros(shape, np.uint8)
    mask[1:-1, 1:-1, 1:-1] = 1
    n = int(mask.sum())
    say("case: network gradient + Adam")
    p0 = net.params.cpu().numpy().copy()
    xd = dev(xb.reshape(-1))
    net.pack(backward=True)
    out = net.forward(xd, shape)
    net.backward(xd, dev(target.reshape(-1)), dev(mask.reshape(-1)), shape, n)
    torch.cuda.synchronize()
    got_out = out.cpu().numpy().reshape(shape + (2,))
    grads = net.grads.cpu().numpy()
    loss_gpu = float(net.loss[0].item())
    # oracle with BF16-rounded weights (what the matrix cores multiply)
    W = [C.bf16_round(p0[k, :27 * 256].reshape(27, 16, 16)) for k in range(3)]
    bias = [p0[k, 27 * 256:].astype(np.float64) for k in range(3)]
    params = (W[0][:, :8, :], bias[0], W[1], bias[1], W[2][:, :, :2], bias[2][:2])
    ref_out, cache = C.net_forward(xv, params)
    eo = np.linalg.norm(got_out - ref_out) / np.linalg.norm(ref_out)
    say(f"  output rel L2 {eo:.2e}")
    assert eo < 2e-2
    L = C.loss(ref_out, target, mask)
    assert abs(loss_gpu - L) < 3e-2 * L
    g = C.net_backward(C.loss_grad(ref_out, target, mask), params, cache)
    pairs = [(grads[0, :27 * 256].reshape(27, 16, 16)[:, :8, :], g[0]),
             (grads[0, 27 * 256:], g[1]),
             (grads[1, :27 * 256].reshape(27, 16, 16), g[2]), (grads[1, 27 * 256:], g[3]),
             (grads[2, :27 * 256].reshape(27, 16, 16)[:, :, :2], g[4]),
             (grads[2, 27 * 256:27 * 256 + 2], g[5])]
    for k, (a, b) in enumerate(pairs):
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        say(f"  grad {k} rel L2 {e:.2e}")
        assert e < 3e-2, k
    # one Adam step on the GPU against the oracle's, from the GPU gradient
    # (weights only: the biases are not trained)
    net.adam(1e-3)
    torch.cuda.synchronize()
    p1 = net.params.cpu().numpy()
    ref, _, _ = C.adam_step(p0.astype(np.float64), grads.astype(np.float64), np.zeros(p0.shape),
                            np.zeros(p0.shape), 1, 1e-3)
    assert np.max(np.abs(p1[:, :27 * 256] - ref[:, :27 * 256])) < 1e-6
    assert np.array_equal(p1[:, 27 * 256:], p0[:, 27 * 256:])


def test_adam_carried_steps_vs_oracle():
    """fd_cnn_adam over five consecutive steps with the moments carried on
    the device (t = 1..5, a fresh gradient each step) against the oracle's
    Adam run in FP64 from the same FP32 start, element-wise (beyond t = 1 the
    bias corrections 1 - beta^t and the carried moments matter).  Parameters
    to 1e-6.  A moment is an FP32 running sum whose terms may cancel, so its
    error is bounded by the magnitudes summed, not by its value: each step
    rounds its two products and their sum (at most about 2 ulp of the
    operands) and carries the earlier error scaled by beta, so after t steps
    |m - m_ref| <= 4 t 2^-24 S_t with S_t = b1 S_{t-1} + (1 - b1)|g_t|
    (S_0 = 0), and the same for v with g^2 and b2."""
    rng = np.random.default_rng(77)
    n = 3000
    p0 = rng.standard_normal(n).astype(np.float32)
    grads = [rng.standard_normal(n).astype(np.float32) for _ in range(5)]
    # the oracle takes the hyperparameters as the kernel receives them, rounded
    # to FP32 (1 - beta2 differs by 1.3e-5 between 0.999 and its FP32 value)
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-2, 0.9, 0.999, 1e-8))
    say("case: Adam, five carried steps")
    pd, md, vd = dev(p0.copy()), dev(np.zeros(n, np.float32)), dev(np.zeros(n, np.float32))
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    sm, sv = np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        gd = dev(g)
        P.fd_cnn_adam(pd.data_ptr(), gd.data_ptr(), md.data_ptr(), vd.data_ptr(), n, t, lr,
                      b1, b2, eps, st())
        pr, mr, vr = C.adam_step(pr, g.astype(np.float64), mr, vr, t, lr, b1, b2, eps)
        torch.cuda.synchronize()
        g64 = g.astype(np.float64)
        sm = b1 * sm + (1 - b1) * np.abs(g64)
        sv = b2 * sv + (1 - b2) * g64 * g64
        np.testing.assert_allclose(pd.cpu().numpy(), pr, rtol=0, atol=1e-6)
        assert np.all(np.abs(md.cpu().numpy() - mr) <= 4 * t * 2.0**-24 * sm), t
        assert np.all(np.abs(vd.cpu().numpy() - vr) <= 4 * t * 2.0**-24 * sv), t


def test_restrict_features_correct_roundtrip():
    """fd_restrict samples every second point; features carry s u^n, s u^{n-1}
    and v / vref - 1; a correction by the residual restores the reference."""
    from workloads import learned_model
    from paper_1608_03984_amd.learned import VREF, make_pair
    m = learned_model(5, phys_f=32, nbl_f=8, nt_f=40)
    pair = make_pair(m)
    say("case: restrict / features / residual / correct")
    f, c = pair.fine, pair.coarse
    f.forward(30, pair.src, pair.wav_f[:30], None)
    fine_cur = f.get_field(P.FD_FIELD_CUR).cpu().numpy()
    V = int(np.prod(c.field_shape))
    r = torch.empty(V, dtype=torch.float32, device="cuda")
    P.fd_restrict(f.ctx, P.FD_FIELD_CUR, 2, r.data_ptr(), st())
    torch.cuda.synchronize()
    assert np.array_equal(r.cpu().numpy().reshape(c.field_shape), fine_cur[::2, ::2, ::2])
    c.forward(15, pair.src, pair.wav_c[:15], None)
    uc = c.get_field(P.FD_FIELD_CUR).cpu().numpy()
    up = c.get_field(P.FD_FIELD_PREV).cpu().numpy()
    bits = torch.zeros(1, dtype=torch.int32, device="cuda")
    x0 = torch.empty(V * 8, dtype=torch.int16, device="cuda")
    P.fd_cnn_features(c.ctx, VREF, 0, bits.data_ptr(), x0.data_ptr(), st())
    torch.cuda.synchronize()
    mx = np.abs(uc).max()
    assert np.frombuffer(bits.cpu().numpy().tobytes(), np.float32)[0] == np.float32(mx)
    feats = from_bits(x0.cpu().numpy()).reshape(c.field_shape + (8,))
    # s u in FP32, then rounded to BF16: within one BF16 unit of the exact value
    np.testing.assert_allclose(feats[..., 0], uc / mx, rtol=2.0 ** -7, atol=1e-30)
    np.testing.assert_allclose(feats[..., 1], up / mx, rtol=2.0 ** -7, atol=1e-30)
    vn = m["vel_c"].astype(np.float64) / VREF - 1
    np.testing.assert_allclose(feats[..., 2], uc / mx * vn, rtol=2.0 ** -6, atol=1e-7)
    np.testing.assert_allclose(feats[..., 3], up / mx * vn, rtol=2.0 ** -6, atol=1e-7)
    assert np.all(feats[..., 4:] == 0)
    # residual to a reference, applied as a correction, gives the reference
    ref_cur, ref_prev = dev(uc * 1.5 + 1e-3), dev(up * 0.5)
    t = torch.empty(V * 2, dtype=torch.float32, device="cuda")
    P.fd_cnn_residual(c.ctx, ref_cur.data_ptr(), ref_prev.data_ptr(), bits.data_ptr(),
                      t.data_ptr(), st())
    P.fd_cnn_correct(c.ctx, t.data_ptr(), 0, bits.data_ptr(), st())
    torch.cuda.synchronize()
    a = c.get_field(P.FD_FIELD_CUR).cpu().numpy()
    b = c.get_field(P.FD_FIELD_PREV).cpu().numpy()
    assert np.max(np.abs(a - (uc * 1.5 + 1e-3))) < 1e-6 * max(1.0, np.abs(a).max())
    assert np.max(np.abs(b - up * 0.5)) < 1e-6 * max(1.0, np.abs(b).max())
    pair.close()
