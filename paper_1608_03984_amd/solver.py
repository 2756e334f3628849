"""Torch-facing convenience wrapper over the libfd C ABI.

PyTorch supplies device memory (the workspace and every field/trace tensor)
and the current HIP stream; all arithmetic runs in libfd's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B

PHYSICS = {"acoustic": B.FD_ACOUSTIC, "tti": B.FD_TTI, "vti": B.FD_VTI}


def _dev(a, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float32).contiguous()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)


class Solver:
    """One problem set up in libfd: grid, model coefficients and wavefields.

    ``shape`` and ``spacing`` are (x, y, z) physical sizes (ny = 1 in 2D);
    model fields are float32 arrays/tensors of the padded shape in array order
    ([Nz][Ny][Nx] or [Nz][Nx])."""

    def __init__(self, ndim, shape, spacing, nbl, space_order, dt, vel, eta=None, *,
                 physics="acoustic", epsilon=None, delta=None, theta=None, phi=None,
                 max_points=1024, device="cuda", nshots=1):
        self.device = torch.device(device)
        self.ndim = int(ndim)
        self.grid = B.make_grid(ndim, shape, spacing, nbl, space_order, dt, PHYSICS[physics])
        self.physics = physics
        nb = int(nbl)
        if self.ndim == 2:
            self.field_shape = (int(shape[2]) + 2 * nb, int(shape[0]) + 2 * nb)
        else:
            self.field_shape = tuple(int(shape[a]) + 2 * nb for a in (2, 1, 0))
        self.max_points = int(max_points)
        self.nshots = int(nshots)
        nbytes = B.fd_workspace_bytes_shots(self.grid, self.nshots, self.max_points)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.workspace_bytes = nbytes
        fields = {"vel": vel, "eta": eta, "epsilon": epsilon, "delta": delta, "theta": theta,
                  "phi": phi}
        keep = {k: _dev(v, self.device) for k, v in fields.items()}
        for k, v in keep.items():
            if v is not None and tuple(v.shape) != self.field_shape:
                raise ValueError(f"{k} has shape {tuple(v.shape)}, expected {self.field_shape}")
        m = B.FdModel()
        for k, v in keep.items():
            setattr(m, k, v.data_ptr() if v is not None else None)
        self.ctx = B.fd_setup_shots(self.grid, m, self.nshots, self._ws_ptr, nbytes,
                                    self.max_points, self.stream)
        del keep  # fd_setup synchronised its stream: the model buffers are no longer read

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def forward(self, nt, src_coords=None, wavelet=None, rec_coords=None, zero_state=True,
                traces=None, keep_points=False):
        """Run nt steps; returns the receiver traces [nt][nrec] (device tensor).
        keep_points: the points are the previous call's (FD_KEEP_POINTS; the
        coordinates are only counted, not passed)."""
        src = None if src_coords is None else np.asarray(src_coords, np.float64).reshape(-1, self.ndim)
        rec = None if rec_coords is None else np.asarray(rec_coords, np.float64).reshape(-1, self.ndim)
        q = None
        if src is not None and src.shape[0]:
            q = _dev(wavelet, self.device).reshape(nt, src.shape[0])
        nrec = 0 if rec is None else rec.shape[0]
        if traces is None and nrec:
            traces = torch.empty((nt, nrec), dtype=torch.float32, device=self.device)
        flags = (B.FD_ZERO_STATE if zero_state else 0) | (B.FD_KEEP_POINTS if keep_points else 0)
        if keep_points:
            src = None if src is None else src.shape[0]
            rec = None if rec is None else rec.shape[0]
        B.fd_forward(self.ctx, nt, src, q.data_ptr() if q is not None else 0, rec,
                     traces.data_ptr() if nrec else 0, flags, self.stream)
        self._keep_q = q  # the wavelet must outlive the asynchronous launches
        return traces

    def _coords(self, c):
        return None if c is None else np.asarray(c, np.float64).reshape(-1, self.ndim)

    def forward_checkpointed(self, nt, src_coords, wavelet, rec_coords, interval=0):
        """Zero-state forward run (same traces as ``forward``) that keeps the
        checkpoints ``gradient`` needs; the store is allocated here."""
        src, rec = self._coords(src_coords), self._coords(rec_coords)
        nbytes, used = B.fd_checkpoint_bytes(self.ctx, nt, interval)
        store = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (store.data_ptr() + 255) // 256 * 256
        q = _dev(wavelet, self.device).reshape(nt, src.shape[0]) if src is not None and len(src) else None
        nrec = 0 if rec is None else rec.shape[0]
        traces = torch.empty((nt, nrec), dtype=torch.float32, device=self.device)
        B.fd_forward_checkpointed(self.ctx, nt, src, q.data_ptr() if q is not None else 0, rec,
                                  traces.data_ptr() if nrec else 0, used, ptr, nbytes,
                                  self.stream)
        self._ck = dict(store=store, ptr=ptr, bytes=nbytes, interval=used, nt=nt, src=src, q=q,
                        rec=rec)
        return traces

    @property
    def checkpoint_interval(self):
        return self._ck["interval"] if getattr(self, "_ck", None) else None

    def gradient(self, adj_data, wrt="vel", wavelet_grad=True, accumulate_into=None):
        """(dJ/dmodel [padded field shape], dJ/dwavelet [nt][nsrc] or None) for
        the trace sensitivities ``adj_data`` [nt][nrec] of the last
        ``forward_checkpointed`` run.  With ``accumulate_into`` (a float32
        tensor of the field shape) the model gradient is added to it (the sum
        over the shots of a survey) and that tensor is returned."""
        ck = self._ck
        nt, src, rec = ck["nt"], ck["src"], ck["rec"]
        d = _dev(adj_data, self.device).reshape(nt, 0 if rec is None else rec.shape[0])
        if accumulate_into is not None:
            grad = accumulate_into
            if tuple(grad.shape) != self.field_shape or grad.dtype != torch.float32 \
                    or not grad.is_contiguous() or not grad.is_cuda:
                raise ValueError("accumulate_into: contiguous float32 tensor of the field shape")
        else:
            grad = torch.empty(self.field_shape, dtype=torch.float32, device=self.device)
        nsrc = 0 if src is None else src.shape[0]
        qg = torch.empty((nt, nsrc), dtype=torch.float32, device=self.device) \
            if wavelet_grad and nsrc else None
        B.fd_gradient(self.ctx, nt, src, ck["q"].data_ptr() if ck["q"] is not None else 0, rec,
                      d.data_ptr(), ck["interval"], ck["ptr"], ck["bytes"],
                      (B.FD_WRT_VEL if wrt == "vel" else B.FD_WRT_M)
                      | (B.FD_GRAD_ACCUMULATE if accumulate_into is not None else 0),
                      grad.data_ptr(),
                      qg.data_ptr() if qg is not None else 0, self.stream)
        self._keep_adj = d
        return grad, qg

    def adjoint(self, nt, adj_coords, adj_data, out_coords):
        """F^T d: the transpose of the zero-state map wavelet -> traces, for
        data ``adj_data`` [nt][nadj] at ``adj_coords``; returns [nt][nout]
        at ``out_coords``.  The held wavefields are overwritten."""
        a, o = self._coords(adj_coords), self._coords(out_coords)
        d = _dev(adj_data, self.device).reshape(nt, 0 if a is None else a.shape[0])
        nout = 0 if o is None else o.shape[0]
        out = torch.empty((nt, nout), dtype=torch.float32, device=self.device)
        B.fd_adjoint(self.ctx, nt, a, d.data_ptr(), o, out.data_ptr() if nout else 0, self.stream)
        self._keep_adj = d
        return out

    def forward_shots(self, nt, src_list, wavelet_list, rec_list, zero_state=True,
                      keep_points=False):
        """nt steps of every shot: ``src_list[k]`` / ``rec_list[k]`` are shot
        k's source and receiver coordinates, ``wavelet_list[k]`` its wavelets
        [nt][nsrc_k].  Returns the list of per-shot traces [nt][nrec_k].
        keep_points: the points are the previous call's (FD_KEEP_POINTS; the
        coordinates are only counted, not passed)."""
        ns = self.nshots
        srcs = [self._coords(c) if c is not None else np.zeros((0, self.ndim)) for c in src_list]
        recs = [self._coords(c) if c is not None else np.zeros((0, self.ndim)) for c in rec_list]
        if len(srcs) != ns or len(recs) != ns or len(wavelet_list) != ns:
            raise ValueError("one source set, wavelet and receiver set per shot")
        sc = np.array([len(c) for c in srcs], np.int32)
        rc = np.array([len(c) for c in recs], np.int32)
        if keep_points:
            src = int(sc.sum()) if sc.sum() else None
            rec = int(rc.sum()) if rc.sum() else None
        else:
            src = np.concatenate(srcs) if sc.sum() else None
            rec = np.concatenate(recs) if rc.sum() else None
        q = None
        if src is not None:
            q = torch.cat([_dev(w, self.device).reshape(nt, int(k))
                           for w, k in zip(wavelet_list, sc)], dim=1).contiguous()
        traces = torch.empty((nt, int(rc.sum())), dtype=torch.float32, device=self.device)
        B.fd_forward_shots(self.ctx, nt, src, sc if src is not None else None,
                           q.data_ptr() if q is not None else 0, rec,
                           rc if rec is not None else None,
                           traces.data_ptr() if rec is not None else 0,
                           (B.FD_ZERO_STATE if zero_state else 0)
                           | (B.FD_KEEP_POINTS if keep_points else 0), self.stream)
        self._keep_q = q
        bounds = np.concatenate([[0], np.cumsum(rc)])
        return [traces[:, bounds[k]:bounds[k + 1]] for k in range(ns)]

    def _shot_points(self, nt, src_list, wavelet_list, rec_list):
        ns = self.nshots
        srcs = [self._coords(c) if c is not None else np.zeros((0, self.ndim)) for c in src_list]
        recs = [self._coords(c) if c is not None else np.zeros((0, self.ndim)) for c in rec_list]
        if len(srcs) != ns or len(recs) != ns or len(wavelet_list) != ns:
            raise ValueError("one source set, wavelet and receiver set per shot")
        sc = np.array([len(c) for c in srcs], np.int32)
        rc = np.array([len(c) for c in recs], np.int32)
        src = np.concatenate(srcs) if sc.sum() else None
        rec = np.concatenate(recs) if rc.sum() else None
        q = None
        if src is not None:
            q = torch.cat([_dev(w, self.device).reshape(nt, int(k))
                           for w, k in zip(wavelet_list, sc)], dim=1).contiguous()
        return src, sc, rec, rc, q

    def forward_checkpointed_shots(self, nt, src_list, wavelet_list, rec_list, interval=0):
        """``forward_checkpointed`` for every shot of a context of several
        shots (per-shot lists as in ``forward_shots``); returns the per-shot
        traces and keeps the checkpoints ``gradient_shots`` needs."""
        src, sc, rec, rc, q = self._shot_points(nt, src_list, wavelet_list, rec_list)
        nbytes, used = B.fd_checkpoint_bytes(self.ctx, nt, interval)
        store = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (store.data_ptr() + 255) // 256 * 256
        traces = torch.empty((nt, int(rc.sum())), dtype=torch.float32, device=self.device)
        B.fd_forward_checkpointed_shots(self.ctx, nt, src, sc if src is not None else None,
                                        q.data_ptr() if q is not None else 0, rec,
                                        rc if rec is not None else None,
                                        traces.data_ptr() if rec is not None else 0, used, ptr,
                                        nbytes, self.stream)
        self._ck = dict(store=store, ptr=ptr, bytes=nbytes, interval=used, nt=nt, src=src, q=q,
                        rec=rec, sc=sc, rc=rc)
        self._ck_traces = traces
        bounds = np.concatenate([[0], np.cumsum(rc)])
        return [traces[:, bounds[k]:bounds[k + 1]] for k in range(self.nshots)]

    def gradient_shots(self, adj_list, wrt="vel", wavelet_grad=False, accumulate_into=None):
        """Sum over the shots of dJ/dmodel for per-shot trace sensitivities
        ``adj_list[k]`` [nt][nrec_k] (or one [nt][sum nrec_k] tensor, the
        layout of the traces) of the last ``forward_checkpointed_shots`` run;
        returns (gradient [padded field shape], dJ/dwavelet [nt][nsrc]
        over all sources, or None)."""
        ck = self._ck
        nt, src, rec, sc, rc = ck["nt"], ck["src"], ck["rec"], ck["sc"], ck["rc"]
        if isinstance(adj_list, torch.Tensor):   # already [nt][sum nrec_k]
            d = adj_list.to(device=self.device, dtype=torch.float32).reshape(nt, int(rc.sum()))
            d = d.contiguous()
        else:
            d = torch.cat([_dev(a, self.device).reshape(nt, int(k))
                           for a, k in zip(adj_list, rc)], dim=1).contiguous()
        if accumulate_into is not None:
            grad = accumulate_into
            if tuple(grad.shape) != self.field_shape or grad.dtype != torch.float32 \
                    or not grad.is_contiguous() or not grad.is_cuda:
                raise ValueError("accumulate_into: contiguous float32 tensor of the field shape")
        else:
            grad = torch.empty(self.field_shape, dtype=torch.float32, device=self.device)
        nsrc = 0 if src is None else src.shape[0]
        qg = torch.empty((nt, nsrc), dtype=torch.float32, device=self.device) \
            if wavelet_grad and nsrc else None
        B.fd_gradient_shots(self.ctx, nt, src, sc if src is not None else None,
                            ck["q"].data_ptr() if ck["q"] is not None else 0, rec,
                            rc if rec is not None else None, d.data_ptr(), ck["interval"],
                            ck["ptr"], ck["bytes"],
                            (B.FD_WRT_VEL if wrt == "vel" else B.FD_WRT_M)
                            | (B.FD_GRAD_ACCUMULATE if accumulate_into is not None else 0),
                            grad.data_ptr(), qg.data_ptr() if qg is not None else 0, self.stream)
        self._keep_adj = d
        return grad, qg

    def get_field(self, which=B.FD_FIELD_CUR, shot=0):
        out = torch.empty(self.field_shape, dtype=torch.float32, device=self.device)
        B.fd_get_shot_field(self.ctx, shot, which, out.data_ptr(), self.stream)
        return out

    def set_field(self, which, value, shot=0):
        v = _dev(value, self.device)
        if tuple(v.shape) != self.field_shape:
            raise ValueError("field shape mismatch")
        B.fd_set_shot_field(self.ctx, shot, which, v.data_ptr(), self.stream)
        self._keep_set = v

    def set_option(self, option, value):
        B.fd_set_option(self.ctx, option, value)

    def get_option(self, option):
        return B.fd_get_option(self.ctx, option)

    def close(self):
        if getattr(self, "ctx", None):
            B.fd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_problem(p, device="cuda", max_points=None) -> Solver:
    """Solver for a workloads.Problem."""
    mp = max_points if max_points is not None else max(1024, len(p.src) + len(p.rec))
    return Solver(p.ndim, p.shape, p.spacing, p.nbl, p.so, p.dt, p.vel, p.eta, physics=p.physics,
                  epsilon=p.eps, delta=p.delta, theta=p.theta, phi=p.phi, max_points=mp,
                  device=device)


class AcousticModeling(torch.autograd.Function):
    """Traces of the zero-state acoustic run as a differentiable function of
    the velocity model and the source wavelets.  The forward pass keeps
    checkpoints; the backward pass runs libfd's adjoint and imaging
    condition (fd_gradient) on the incoming trace sensitivities."""

    @staticmethod
    def forward(ctx, vel, wavelet, geometry):
        g = geometry
        s = Solver(g["ndim"], g["shape"], g["spacing"], g["nbl"], g["so"], g["dt"], vel.detach(),
                   g.get("eta"), max_points=len(g["src"]) + len(g["rec"]) + 1, device=vel.device)
        tr = s.forward_checkpointed(wavelet.shape[0], g["src"], wavelet.detach(), g["rec"],
                                    g.get("interval", 0))
        ctx.solver = s
        return tr

    @staticmethod
    def backward(ctx, gtr):
        s = ctx.solver
        need_v, need_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gv, gq = s.gradient(gtr.contiguous(), wrt="vel", wavelet_grad=need_q)
        ctx.solver = None
        s.close()
        return (gv if need_v else None), (gq if need_q else None), None


def acoustic_modeling(vel, wavelet, geometry):
    """Differentiable traces [nt][nrec] for ``vel`` (padded shape, float32 on
    the GPU) and ``wavelet`` [nt][nsrc].  ``geometry`` is a dict with ndim,
    shape (x, y, z physical), spacing, nbl, so, dt, src and rec coordinates and
    optionally eta (damping, padded shape) and interval (checkpoint spacing)."""
    return AcousticModeling.apply(vel, wavelet, geometry)
