"""Learned coarse-grid correction: a coarse, low-order acoustic solver whose
state is corrected every few steps by a three-layer 3D convolution network
trained to track a fine, high-order solution sampled at the coarse points.

Every operation on the network and the wavefields runs in libfd's kernels
(fd_cnn_* and fd_restrict through the C ABI): the BF16 matrix-core
convolutions and their backward passes, the loss gradient, Adam, the
feature extraction and the correction.  PyTorch provides device memory, and
this module orchestrates: it builds the training pairs from solver runs,
loops over them, and runs the corrected solver.

The cost study of the paper (section 6) trades space order against grid
spacing at a fixed physical problem; the plain solvers stay available as the
fallback and as the reference for the learned solver's error.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _binding as B
from .solver import Solver

LAYER = B.FD_CNN_LAYER_FLOATS
VREF = 2500.0          # velocity normalisation of the network's third input channel


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


class CorrectionNet:
    """Three 3x3x3 convolution layers, 4 (padded to 8) -> 16 -> 16 -> 2
    channels, ReLU between them.  Parameters are FP32 [3][LAYER] with each
    layer stored padded as [27][16 ci][16 co] + bias[16] (unused channels stay
    zero: their gradients are zero).  The biases stay zero (Adam updates the
    weights only), which keeps the network positively homogeneous: inputs
    scaled by a > 0 give outputs scaled by a, and no input gives no
    correction.

    The correction is small against the field (about 1e-3 of it), so the last
    layer is parametrised as w3 = out_scale * v with v He-initialised and
    trained: Adam on v with learning rate lr is Adam on w3 with learning rate
    out_scale * lr (Adam's step does not depend on the gradient's scale, up to
    its epsilon), which is how the last layer is updated here."""

    NIN = 4

    def __init__(self, device="cuda", seed=0, out_scale=0.01, relu=True):
        self.device = torch.device(device)
        self.relu = relu
        rng = np.random.default_rng(seed)
        p = np.zeros((3, LAYER), np.float32)
        w = [p[k, :27 * 256].reshape(27, 16, 16) for k in range(3)]
        w[0][:, :self.NIN, :] = (rng.standard_normal((27, self.NIN, 16))
                                 * np.sqrt(2.0 / (27 * self.NIN)))
        w[1][:, :, :] = rng.standard_normal((27, 16, 16)) * np.sqrt(2.0 / (27 * 16))
        w[2][:, :, :2] = rng.standard_normal((27, 16, 2)) * np.sqrt(1.0 / (27 * 16)) * out_scale
        self.out_scale = out_scale
        self.params = torch.from_numpy(p).to(self.device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        e8, e16 = B.fd_cnn_packed_elems(8), B.fd_cnn_packed_elems(16)
        mk = lambda n: torch.empty(n, dtype=torch.int16, device=self.device)
        self.pk = [mk(e8), mk(e16), mk(e16)]           # forward operands
        self.pkT = [None, mk(e16), mk(e8)]             # backward-data operands (layers 2, 3)
        # loss[0] accumulates; the rest are the loss kernel's per-block partials
        self.loss = torch.zeros(B.FD_CNN_LOSS_FLOATS, dtype=torch.float32, device=self.device)
        self._shape = None

    # -- buffers -------------------------------------------------------------
    def _buffers(self, shape):
        if self._shape == tuple(shape):
            return
        V = int(np.prod(shape))
        i16 = lambda c: torch.empty(V * c, dtype=torch.int16, device=self.device)
        self.y1, self.y2 = i16(16), i16(16)
        self.dz3, self.dz2, self.dz1 = i16(8), i16(16), i16(16)
        self.d = torch.empty(V * 2, dtype=torch.float32, device=self.device)
        ns = B.fd_cnn_wgrad_scratch(shape)
        self.scratch = torch.empty(ns, dtype=torch.float32, device=self.device)
        self._shape = tuple(shape)

    def _ptr(self, k, off=0):
        return self.params[k].data_ptr() + 4 * off

    def pack(self, backward=False):
        st = _stream(self.device)
        for k, cin in enumerate((8, 16, 16)):
            B.fd_cnn_pack(self._ptr(k), cin, 0, self.pk[k].data_ptr(), st)
        if backward:
            B.fd_cnn_pack(self._ptr(1), 16, 1, self.pkT[1].data_ptr(), st)
            B.fd_cnn_pack(self._ptr(2), 8, 1, self.pkT[2].data_ptr(), st)

    # -- forward / backward ----------------------------------------------------
    def forward(self, x0, shape):
        """x0: BF16 bit patterns [shape][8] (int16 tensor); returns the FP32
        output [V][2] (a view of an internal buffer)."""
        self._buffers(shape)
        st = _stream(self.device)
        act = B.FD_CNN_RELU if self.relu else B.FD_CNN_IDENTITY
        B.fd_cnn_conv(x0.data_ptr(), 8, shape, self.pk[0].data_ptr(), self._ptr(0, 27 * 256),
                      act, 0, 0, self.y1.data_ptr(), 0, st)
        B.fd_cnn_conv(self.y1.data_ptr(), 16, shape, self.pk[1].data_ptr(),
                      self._ptr(1, 27 * 256), act, 0, 0, self.y2.data_ptr(), 0, st)
        B.fd_cnn_conv(self.y2.data_ptr(), 16, shape, self.pk[2].data_ptr(),
                      self._ptr(2, 27 * 256), B.FD_CNN_LINEAR, 0, 2, 0, self.d.data_ptr(), st)
        return self.d

    def backward(self, x0, target, mask, shape, n_mask):
        """Gradients of the masked mean square into self.grads (after a
        forward on the same x0); adds the loss to self.loss."""
        st = _stream(self.device)
        V = int(np.prod(shape))
        B.fd_cnn_loss_grad(self.d.data_ptr(), target.data_ptr(), mask.data_ptr(), V, 2, 8,
                           1.0 / max(n_mask, 1), self.dz3.data_ptr(), self.loss.data_ptr(), st)
        ns = self.scratch.numel()
        g = self.grads
        B.fd_cnn_wgrad(self.y2.data_ptr(), 16, self.dz3.data_ptr(), 8, shape,
                       self.scratch.data_ptr(), ns, g[2].data_ptr(), st)
        back = B.FD_CNN_MASKED if self.relu else B.FD_CNN_UNMASKED
        B.fd_cnn_conv(self.dz3.data_ptr(), 8, shape, self.pkT[2].data_ptr(), 0, back,
                      self.y2.data_ptr(), 0, self.dz2.data_ptr(), 0, st)
        B.fd_cnn_wgrad(self.y1.data_ptr(), 16, self.dz2.data_ptr(), 16, shape,
                       self.scratch.data_ptr(), ns, g[1].data_ptr(), st)
        B.fd_cnn_conv(self.dz2.data_ptr(), 16, shape, self.pkT[1].data_ptr(), 0, back,
                      self.y1.data_ptr(), 0, self.dz1.data_ptr(), 0, st)
        B.fd_cnn_wgrad(x0.data_ptr(), 8, self.dz1.data_ptr(), 16, shape, self.scratch.data_ptr(),
                       ns, g[0].data_ptr(), st)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam on the weights of the three layers (the biases stay zero)."""
        self.t += 1
        st = _stream(self.device)
        nw = 27 * 256
        for k in range(3):
            lr_k = lr * (self.out_scale if k == 2 else 1.0)
            B.fd_cnn_adam(self.params[k].data_ptr(), self.grads[k].data_ptr(),
                          self.m[k].data_ptr(), self.v[k].data_ptr(), nw, self.t, lr_k, beta1,
                          beta2, eps, st)

    def state_dict(self):
        return {"params": self.params.detach().cpu().numpy().copy(), "t": self.t}


# ---------------------------------------------------------------------------
# Solvers of one fine / coarse pair
# ---------------------------------------------------------------------------

@dataclass
class PairSetup:
    """A fine (so_f, h) and a coarse (so_c, 2h) solver of the same physical
    model; the coarse padded grid is every second point of the fine one
    (nbl_f = 2 nbl_c).  `region` (uint8 over the coarse padded grid) marks
    where the correction acts and is trained: outside the absorbing layer
    and away from the source, whose grid-dependent near field differs
    between any two grids and is not the coarse solver's error to correct."""
    fine: Solver
    coarse: Solver
    src: np.ndarray
    rec: np.ndarray
    wav_f: np.ndarray
    wav_c: np.ndarray
    nt_c: int
    region: torch.Tensor = None
    n_region: int = 0

    def close(self):
        self.fine.close()
        self.coarse.close()


def region_mask(field_shape, nbl, spacing, src, src_radius, device="cuda"):
    """uint8 [V]: 1 outside the absorbing layer and farther than src_radius
    points from every source, 0 elsewhere; and the number of ones."""
    nz, ny, nx = field_shape
    m = np.zeros(field_shape, np.uint8)
    m[nbl:nz - nbl, nbl:ny - nbl, nbl:nx - nbl] = 1
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for c in np.reshape(src, (-1, 3)):
        gx, gy, gz = (c[0] / spacing[0] + nbl, c[1] / spacing[1] + nbl, c[2] / spacing[2] + nbl)
        m[(x - gx) ** 2 + (y - gy) ** 2 + (z - gz) ** 2 <= src_radius ** 2] = 0
    t = torch.from_numpy(m.reshape(-1)).to(device)
    return t, int(m.sum())


SRC_RADIUS = 4       # coarse points of the source ball left out of the correction


def make_pair(model, device="cuda", src_radius=SRC_RADIUS):
    """Solvers for a workloads.learned_model() dictionary."""
    m = model
    fine = Solver(3, m["shape_f"], m["h_f"], m["nbl_f"], m["so_f"], m["dt_f"], m["vel_f"],
                  m["eta_f"], max_points=1 + len(m["rec"]), device=device)
    coarse = Solver(3, m["shape_c"], m["h_c"], m["nbl_c"], m["so_c"], m["dt_c"], m["vel_c"],
                    m["eta_c"], max_points=1 + len(m["rec"]), device=device)
    region, n = region_mask(coarse.field_shape, m["nbl_c"], m["h_c"], m["src"], src_radius,
                            device)
    return PairSetup(fine, coarse, m["src"], m["rec"], m["wav_f"], m["wav_c"], m["nt_c"],
                     region, n)


def training_pairs(pair, times, K, device="cuda"):
    """Training samples of one model: for each coarse time m in `times`
    (m >= K), the coarse state at m - K is set from the fine solution sampled
    at the coarse points, the coarse solver runs K steps, and the sample is
    (network input of the result, target = scaled difference to the sampled
    fine solution at m).  Returns a list of (x0 int16 [V*8], target f32
    [V*2], region mask, mask count)."""
    f, c = pair.fine, pair.coarse
    st = lambda: _stream(torch.device(device))
    shape_c = c.field_shape
    V = int(np.prod(shape_c))
    need = sorted({s for m in times for s in (2 * (m - K) - 2, 2 * (m - K), 2 * m - 2, 2 * m)})
    snaps = {}
    done = 0
    f.forward(0, zero_state=True)
    for s in need:
        if s < 0:
            snaps[s] = torch.zeros(V, dtype=torch.float32, device=device)
            continue
        if s > done:
            f.forward(s - done, pair.src, pair.wav_f[done:s], None, zero_state=False)
            done = s
        buf = torch.empty(V, dtype=torch.float32, device=device)
        B.fd_restrict(f.ctx, B.FD_FIELD_CUR, 2, buf.data_ptr(), st())
        snaps[s] = buf
    out = []
    bits = torch.zeros(1, dtype=torch.int32, device=device)
    for m in times:
        m0 = m - K
        c.set_field(B.FD_FIELD_PREV, snaps[2 * m0 - 2].view(shape_c))
        c.set_field(B.FD_FIELD_CUR, snaps[2 * m0].view(shape_c))
        c.forward(K, pair.src, pair.wav_c[m0:m], None, zero_state=False)
        x0 = torch.empty(V * 8, dtype=torch.int16, device=device)
        tgt = torch.empty(V * 2, dtype=torch.float32, device=device)
        B.fd_cnn_features(c.ctx, VREF, pair.region.data_ptr(), bits.data_ptr(), x0.data_ptr(),
                          st())
        B.fd_cnn_residual(c.ctx, snaps[2 * m].data_ptr(), snaps[2 * m - 2].data_ptr(),
                          bits.data_ptr(), tgt.data_ptr(), st())
        out.append((x0, tgt, pair.region, pair.n_region))
    torch.cuda.synchronize()
    return out


def train(net, samples, shape_c, iters, lr=1e-3, lr_end=1e-4, log=None, seed=0):
    """Adam on the masked mean square over the samples (one sample per
    iteration, each with its own region mask; cosine-decayed learning rate).
    Returns the loss history."""
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(iters):
        x0, tgt, mask, n_mask = samples[int(rng.integers(len(samples)))]
        lr_it = lr_end + 0.5 * (lr - lr_end) * (1 + np.cos(np.pi * it / max(iters - 1, 1)))
        net.pack(backward=True)
        net.loss.zero_()
        net.forward(x0, shape_c)
        net.backward(x0, tgt, mask, shape_c, n_mask)
        net.adam(lr_it)
        if (it + 1) % 50 == 0 or it == iters - 1:
            hist.append((it + 1, float(net.loss[0].item())))
            if log:
                log(f"  iter {it + 1}: loss {hist[-1][1]:.4e}")
    return hist


def sample_loss(net, samples, shape_c):
    """Mean masked loss of the network over samples (no parameter update);
    with net=None the loss of no correction."""
    if net is None:
        net = CorrectionNet(device=samples[0][0].device, out_scale=0.0)
    net.pack(backward=True)
    tot = 0.0
    for x0, tgt, mask, n in samples:
        net.loss.zero_()
        net.forward(x0, shape_c)
        net.backward(x0, tgt, mask, shape_c, n)
        tot += float(net.loss[0].item())
    return tot / max(len(samples), 1)


def correction_start(model, src_radius=SRC_RADIUS, periods=1.0, f0=10.0, vmin=1500.0):
    """First coarse step at which corrections apply: after the source wavelet
    (`periods` / f0) and the travel time out of the excluded source ball."""
    t = periods / f0 + src_radius * model["h_c"][0] / vmin
    return int(round(t / model["dt_c"]))


def solve_coarse(pair, nt_c, K=0, net=None, rec=None, start=0):
    """Coarse run of nt_c steps from the zero state; with a network, the
    state is corrected after every K steps from coarse step `start` on (before
    it, the source is still radiating and the field outside the source region
    is too weak to carry the coarse solver's error).  Returns traces
    [nt_c][nrec]."""
    c = pair.coarse
    rec = pair.rec if rec is None else rec
    dev = c.device
    st = _stream(dev)
    if net is None or K <= 0:
        return c.forward(nt_c, pair.src, pair.wav_c[:nt_c], rec)
    net.pack()
    V = int(np.prod(c.field_shape))
    x0 = torch.empty(V * 8, dtype=torch.int16, device=dev)
    bits = torch.zeros(1, dtype=torch.int32, device=dev)
    traces = torch.empty((nt_c, len(rec)), dtype=torch.float32, device=dev)
    done = 0
    while done < nt_c:
        k = min(K, nt_c - done)
        c.forward(k, pair.src, pair.wav_c[done:done + k], rec, zero_state=(done == 0),
                  traces=traces[done:done + k])
        done += k
        if k == K and done >= start:
            B.fd_cnn_features(c.ctx, VREF, pair.region.data_ptr(), bits.data_ptr(),
                              x0.data_ptr(), st)
            d = net.forward(x0, c.field_shape)
            B.fd_cnn_correct(c.ctx, d.data_ptr(), pair.region.data_ptr(), bits.data_ptr(), st)
    return traces


def solve_coarse_exact(pair, nt_c, K, start=0):
    """The best case of the correction scheme: the coarse run of
    solve_coarse() with the network's output replaced by the exact residual
    (the fine solution sampled at the coarse points minus the coarse state,
    over the same region, every K steps from `start` on).  The fine solver
    advances in step; returns the coarse traces [nt_c][nrec]."""
    f, c = pair.fine, pair.coarse
    dev = c.device
    st = _stream(dev)
    V = int(np.prod(c.field_shape))
    ref_cur = torch.empty(V, dtype=torch.float32, device=dev)
    ref_prev = torch.empty(V, dtype=torch.float32, device=dev)
    bits = torch.zeros(1, dtype=torch.int32, device=dev)
    x0 = torch.empty(V * 8, dtype=torch.int16, device=dev)
    res = torch.empty(V * 2, dtype=torch.float32, device=dev)
    traces = torch.empty((nt_c, len(pair.rec)), dtype=torch.float32, device=dev)
    f.forward(0, zero_state=True)
    done = done_f = 0
    while done < nt_c:
        k = min(K, nt_c - done)
        c.forward(k, pair.src, pair.wav_c[done:done + k], pair.rec, zero_state=(done == 0),
                  traces=traces[done:done + k])
        done += k
        if k == K and done >= start:
            f.forward(2 * done - 2 - done_f, pair.src, pair.wav_f[done_f:2 * done - 2], None,
                      zero_state=False)
            B.fd_restrict(f.ctx, B.FD_FIELD_CUR, 2, ref_prev.data_ptr(), st)
            f.forward(2, pair.src, pair.wav_f[2 * done - 2:2 * done], None, zero_state=False)
            B.fd_restrict(f.ctx, B.FD_FIELD_CUR, 2, ref_cur.data_ptr(), st)
            done_f = 2 * done
            B.fd_cnn_features(c.ctx, VREF, pair.region.data_ptr(), bits.data_ptr(),
                              x0.data_ptr(), st)
            B.fd_cnn_residual(c.ctx, ref_cur.data_ptr(), ref_prev.data_ptr(), bits.data_ptr(),
                              res.data_ptr(), st)
            B.fd_cnn_correct(c.ctx, res.data_ptr(), pair.region.data_ptr(), bits.data_ptr(), st)
    return traces


def solve_fine(pair, nt_f, rec=None):
    rec = pair.rec if rec is None else rec
    return pair.fine.forward(nt_f, pair.src, pair.wav_f[:nt_f], rec)


def trace_error(coarse_tr, fine_tr, receivers=None, t0=0):
    """Relative L2 error of coarse traces (sample n at time (n+1) dt_c)
    against fine traces at the same times (every second fine sample); with
    `receivers` (bool per receiver) and t0, over those receivers and coarse
    samples t0 on only."""
    f = fine_tr[1::2][:coarse_tr.shape[0]]
    d = coarse_tr - f
    if receivers is not None:
        sel = torch.as_tensor(receivers, device=f.device)
        d, f = d[:, sel], f[:, sel]
    return float(torch.linalg.norm(d[t0:]) / torch.linalg.norm(f[t0:]))


def far_receivers(pair, radius):
    """Receivers farther (horizontally) than `radius` metres from the source
    -- with the radius of the region mask's source ball, the ones whose
    traces the correction can act on."""
    r = radius
    off = np.hypot(pair.rec[:, 0] - pair.src[0, 0], pair.rec[:, 1] - pair.src[0, 1])
    return off > r


def timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
