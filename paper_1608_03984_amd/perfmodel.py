"""Roofline performance model of section 4 and the cost-to-solution set-up of
section 6 ("Cost-benefit analysis"), evaluated for MI355X.

Host arithmetic only (no device work): it predicts what the kernels of
libfd.so can reach and sizes the fixed-physics problems that the benchmark
then runs for real.

* FLOPs per point update (Table 1): acoustic 6k + 4, VTI 2(6k + 8),
  TTI 2(6k^2 - 6k + 50), with k = so + 1 points per 1D stencil.
* Bytes per point update (section 4.2, stream stores): 4 x (fields read +
  written): acoustic 16, VTI 36, TTI 60.
* Operational intensity I = FLOPs / bytes; attainable rate
  min(peak FLOP/s, I x bandwidth) (the roofline of section 3).
* Cost-to-solution (Tables 2 and 3): a fixed physical model of 500 points per
  axis at second order, p points per wavelength falling from 6 (order 2) to
  2 (order 24), h = 6 / p in units of the second-order spacing, dt at the CFL
  bound of Eq. (stability) with a1 = 4 and v = 1, and as many steps as reach
  the second-order run's final time of 1000 steps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

# MI355X published peaks
MI355X_HBM_GBS = 8000.0
MI355X_FP32_GFLOPS = 157300.0          # vector FP32 with packed FMA
MI355X_FP32_GFLOPS_NONPACKED = 78600.0

BYTES_PER_POINT = {"acoustic": 16, "vti": 36, "tti": 60}

# Table 2: points per wavelength for the printed orders
TABLE2_P = {2: 6.0, 6: 5.0, 12: 4.0, 18: 3.0, 24: 2.0}


def flops_per_point(physics: str, so: int) -> int:
    """Table 1 FLOP count per point update for stencils of k = so + 1 points."""
    k = so + 1
    if physics == "acoustic":
        return 6 * k + 4
    if physics == "vti":
        return 2 * (6 * k + 8)
    if physics == "tti":
        return 2 * (6 * k * k - 6 * k + 50)
    raise ValueError(physics)


def operational_intensity(physics: str, so: int) -> float:
    """I_alg(k) of section 4.2 (FLOP per byte)."""
    return flops_per_point(physics, so) / BYTES_PER_POINT[physics]


def attainable_gflops(oi: float, bandwidth_gbs: float, peak_gflops: float) -> float:
    """Roofline: min(peak, OI x bandwidth)."""
    return min(peak_gflops, oi * bandwidth_gbs)


def second_derivative_abs_sum(so: int) -> float:
    """Sum of |w| of the central second-derivative stencil of order so on unit
    spacing (exact rational arithmetic; any even order)."""
    r = so // 2
    w = []
    for j in range(1, r + 1):
        wj = Fraction(2 * (-1) ** (j + 1) * math.factorial(r) ** 2,
                      j * j * math.factorial(r - j) * math.factorial(r + j))
        w.append(wj)
    w0 = -2 * sum(w)
    return float(abs(w0) + 2 * sum(abs(x) for x in w))


def a2(ndim: int, so: int) -> float:
    """a2 of Eq. (stability): the sum of |w| of the discrete Laplacian."""
    return ndim * second_derivative_abs_sum(so)


def points_per_wavelength(order: int) -> float:
    """Table 2's p, linear between the printed orders."""
    if order in TABLE2_P:
        return TABLE2_P[order]
    keys = sorted(TABLE2_P)
    if not keys[0] <= order <= keys[-1]:
        raise ValueError(order)
    lo = max(k for k in keys if k < order)
    hi = min(k for k in keys if k > order)
    f = (order - lo) / (hi - lo)
    return TABLE2_P[lo] + f * (TABLE2_P[hi] - TABLE2_P[lo])


@dataclass
class CostRow:
    order: int
    a2: float
    p: float
    h: float          # grid spacing in units of the second-order spacing
    dt: float         # CFL time step at v = 1 in those units
    n_axis: int       # grid points per axis
    N: int            # grid points
    nt: int           # time steps to the common final time
    gflop: float      # Table 1 FLOPs x N x nt / 1e9

    def oi(self) -> float:
        return operational_intensity("acoustic", self.order)

    def runtime_s(self, bandwidth_gbs: float, peak_gflops: float) -> float:
        return self.gflop / attainable_gflops(self.oi(), bandwidth_gbs, peak_gflops)


def cost_row(order: int, base_points: int = 500, base_steps: int = 1000) -> CostRow:
    """One row of Tables 2 and 3 (3D acoustic)."""
    p = points_per_wavelength(order)
    h = TABLE2_P[2] / p
    aa = a2(3, order)
    dt = h * math.sqrt(4.0 / aa)
    t_end = base_steps * math.sqrt(4.0 / a2(3, 2))
    n_axis = int(round(base_points / h))
    N = int(round((base_points / h) ** 3))
    nt = int(math.ceil(t_end / dt - 1e-9))
    return CostRow(order, aa, p, h, dt, n_axis, N, nt,
                   flops_per_point("acoustic", order) * N * nt / 1e9)


def cost_table(orders=(2, 6, 12, 18, 24)):
    return [cost_row(o) for o in orders]
