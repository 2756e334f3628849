"""The roofline / cost-to-solution model (perfmodel) against the paper's
printed Tables 2 and 3 and its OI formulas (section 4.2)."""
import math
from pathlib import Path

import pytest

from paper_1608_03984_amd import perfmodel as M

GOLD = Path(__file__).resolve().parent / "golden"


def _rows(name):
    out = []
    for line in (GOLD / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            out.append([float(x) for x in line.split()])
    return out


@pytest.mark.parametrize("k", [3, 5, 9, 13, 17, 25])
def test_oi_formulas_of_section_4_2(k):
    so = k - 1
    assert M.operational_intensity("acoustic", so) == pytest.approx(3 * k / 8 + 1 / 4)
    assert M.operational_intensity("vti", so) == pytest.approx(k / 3 + 4 / 9)
    assert M.operational_intensity("tti", so) == pytest.approx(k * k / 5 - k / 5 + 5 / 3)


def test_table2_setup():
    for order, a2, p, h, dt, N, nt in _rows("table2_stability.txt"):
        r = M.cost_row(int(order))
        assert abs(r.a2 - a2) <= 0.005 + 1e-12
        assert r.p == p and r.h == pytest.approx(h)
        assert abs(r.dt - dt) <= 1.5e-4            # see the Table 2 dt pin for the tolerance
        assert abs(r.N - N) <= 0.005 * N
        # the printed step counts mix rounding directions (1024 for 1024.4,
        # 688 for 687.4): within one step of reaching the final time
        assert abs(r.nt - nt) <= 1


def test_table3_cost():
    """GFLOPs within the rounding of N and nt; attainable rates at the
    bandwidths the table implies (100 GB/s Xeon, 200 GB/s Xeon Phi, both far
    below their compute peaks); runtimes as printed (whole seconds, up)."""
    for order, oi, gflop, g_xeon, g_phi, t_xeon, t_phi in _rows("table3_cost.txt"):
        r = M.cost_row(int(order))
        assert r.oi() == pytest.approx(oi)
        assert r.gflop == pytest.approx(gflop, rel=5e-3)
        assert M.attainable_gflops(r.oi(), 100.0, 1e9) == pytest.approx(g_xeon)
        assert M.attainable_gflops(r.oi(), 200.0, 1e9) == pytest.approx(g_phi)
        assert math.ceil(gflop / g_xeon) == t_xeon
        assert math.ceil(gflop / g_phi) == t_phi


def test_mi355x_roofline_position():
    """Acoustic and VTI are bandwidth-bound at every built order on MI355X
    (ridge 9.8 FLOP/B non-packed); TTI so 8 lies right of the non-packed
    ridge and left of the packed one (19.7)."""
    ridge_np = M.MI355X_FP32_GFLOPS_NONPACKED / M.MI355X_HBM_GBS
    ridge_p = M.MI355X_FP32_GFLOPS / M.MI355X_HBM_GBS
    for so in range(2, 17, 2):
        assert M.operational_intensity("acoustic", so) < ridge_np
        assert M.operational_intensity("vti", so) < ridge_np
    assert ridge_np < M.operational_intensity("tti", 8) < ridge_p
