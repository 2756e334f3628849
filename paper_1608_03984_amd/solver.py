"""Torch-facing convenience wrapper over the libfd C ABI.

PyTorch supplies device memory (the workspace and every field/trace tensor)
and the current HIP stream; all arithmetic runs in libfd's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B

PHYSICS = {"acoustic": B.FD_ACOUSTIC, "tti": B.FD_TTI}


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
                 max_points=1024, device="cuda"):
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
        nbytes = B.fd_workspace_bytes(self.grid, self.max_points)
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
        self.ctx = B.fd_setup(self.grid, m, self._ws_ptr, nbytes, self.max_points, self.stream)
        del keep  # fd_setup synchronised its stream: the model buffers are no longer read

    @property
    def stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def forward(self, nt, src_coords=None, wavelet=None, rec_coords=None, zero_state=True,
                traces=None):
        """Run nt steps; returns the receiver traces [nt][nrec] (device tensor)."""
        src = None if src_coords is None else np.asarray(src_coords, np.float64).reshape(-1, self.ndim)
        rec = None if rec_coords is None else np.asarray(rec_coords, np.float64).reshape(-1, self.ndim)
        q = None
        if src is not None and src.shape[0]:
            q = _dev(wavelet, self.device).reshape(nt, src.shape[0])
        nrec = 0 if rec is None else rec.shape[0]
        if traces is None and nrec:
            traces = torch.empty((nt, nrec), dtype=torch.float32, device=self.device)
        B.fd_forward(self.ctx, nt, src, q.data_ptr() if q is not None else 0, rec,
                     traces.data_ptr() if nrec else 0, B.FD_ZERO_STATE if zero_state else 0,
                     self.stream)
        self._keep_q = q  # the wavelet must outlive the asynchronous launches
        return traces

    def get_field(self, which=B.FD_FIELD_CUR):
        out = torch.empty(self.field_shape, dtype=torch.float32, device=self.device)
        B.fd_get_field(self.ctx, which, out.data_ptr(), self.stream)
        return out

    def set_field(self, which, value):
        v = _dev(value, self.device)
        if tuple(v.shape) != self.field_shape:
            raise ValueError("field shape mismatch")
        B.fd_set_field(self.ctx, which, v.data_ptr(), self.stream)
        self._keep_set = v

    def set_option(self, option, value):
        B.fd_set_option(self.ctx, option, value)

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
