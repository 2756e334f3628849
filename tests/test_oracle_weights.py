"""Pins for the oracle's finite-difference weights and CFL bound.

Fixed by the paper: the k-point symmetric stencils of section 4.1 and the
a2 / dt columns of Table 2 (section 6).  Fixed by mathematics: polynomial
exactness up to the stencil's order, the Nyquist symbol, and agreement with
weights solved independently from the Taylor conditions.
"""
import math
from pathlib import Path

import numpy as np
import pytest

import oracle
from tests._bruteforce import taylor_weights

ORDERS = [2, 4, 6, 8, 10, 12, 14, 16]
GOLDEN = Path(__file__).parent / "golden" / "table2_stability.txt"


def full_stencil(w):
    """w[0..r] -> symmetric array indexed j + r."""
    return np.concatenate([w[:0:-1], w])


def antisym_stencil(w):
    return np.concatenate([-w[:0:-1], w])


@pytest.mark.parametrize("so", ORDERS + [24])
def test_second_derivative_polynomial_exactness(so):
    """sum_j w_j j^p equals d^2/dx^2 x^p at 0 (2 for p = 2, else 0) for every
    degree p <= so + 1 and fails at p = so + 2."""
    r = so // 2
    c = full_stencil(oracle.weights_d2(so))
    j = np.arange(-r, r + 1, dtype=np.float64)
    for p in range(so + 2):
        val = np.sum(c * j ** p)
        scale = np.sum(np.abs(c) * np.abs(j) ** p) + 1.0
        assert abs(val - (2.0 if p == 2 else 0.0)) <= 1e-12 * scale, (so, p, val)
    p = so + 2
    val = np.sum(c * j ** p)
    assert abs(val) > 1e-6 * np.sum(np.abs(c) * np.abs(j) ** p), (so, val)


@pytest.mark.parametrize("so", ORDERS)
def test_first_derivative_polynomial_exactness(so):
    """sum_j w1_j j^p equals 1 for p = 1 and 0 otherwise for p <= so, and fails
    at p = so + 1."""
    r = so // 2
    c = antisym_stencil(oracle.weights_d1(so))
    j = np.arange(-r, r + 1, dtype=np.float64)
    for p in range(so + 1):
        val = np.sum(c * j ** p)
        scale = np.sum(np.abs(c) * np.abs(j) ** p) + 1.0
        assert abs(val - (1.0 if p == 1 else 0.0)) <= 1e-12 * scale, (so, p, val)
    val = np.sum(c * j ** (so + 1))
    assert abs(val) > 1e-6 * np.sum(np.abs(c) * np.abs(j) ** (so + 1))


@pytest.mark.parametrize("so", ORDERS)
def test_weights_match_taylor_solve(so):
    """Closed-form weights equal the Vandermonde solution of the Taylor
    conditions (an independent derivation)."""
    r = so // 2
    # the Vandermonde system is ill-conditioned (cond ~ 1e13 at r = 8), so the
    # solved weights carry ~1e-10 absolute error
    np.testing.assert_allclose(full_stencil(oracle.weights_d2(so)), taylor_weights(2, r),
                               rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(antisym_stencil(oracle.weights_d1(so)), taylor_weights(1, r),
                               rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("so", ORDERS + [24])
def test_nyquist_symbol(so):
    """The symbol W(theta) = w0 + 2 sum w_j cos(j theta) reaches -sum|w| at
    theta = pi (alternating signs), and is non-positive everywhere."""
    w = oracle.weights_d2(so)
    r = so // 2
    S = abs(w[0]) + 2 * np.sum(np.abs(w[1:]))
    th = np.linspace(0, np.pi, 2001)
    W = w[0] + 2 * sum(w[j] * np.cos(j * th) for j in range(1, r + 1))
    assert abs(W[-1] + S) < 1e-12 * S
    assert np.all(W <= 1e-14)
    assert np.isclose(W.min(), -S, rtol=1e-12)


def _golden():
    rows = []
    for line in GOLDEN.read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


def test_table2_a2_column():
    """a2 (3D Laplacian, unit spacing) reproduces Table 2 to its two decimals."""
    for order, a2, p, h, dt, N, nt in _golden():
        assert abs(oracle.a2(3, int(order)) - a2) <= 0.005 + 1e-12, order


def test_table2_dt_column():
    """dt = h sqrt(a1/a2)/v with a1 = 4, v = 1 reproduces Table 2's dt column.
    The printed 24th-order value 1.2359 is h sqrt(4/23.57) with a2 already
    rounded to 23.57; the exact a2 gives 1.23576, so the tolerance is 1.5e-4
    (about 1.2e-4 relative) rather than half a unit of the last digit."""
    for order, a2, p, h, dt, N, nt in _golden():
        got = oracle.cfl_dt(3, int(order), [h, h, h], 1.0)
        assert abs(got - dt) <= 1.5e-4, (order, got, dt)
        # and the printed dt is consistent with the printed a2 to rounding
        assert abs(h * np.sqrt(4.0 / a2) - dt) <= 1.5e-4


def test_table2_grid_size_column():
    """N = (500 / h)^3 (fixed physical size of 500 points at 2nd order)."""
    for order, a2, p, h, dt, N, nt in _golden():
        assert abs((500.0 / h) ** 3 - N) <= 0.005 * N


def test_cfl_unequal_spacing_reduces_to_equal():
    for so in (4, 8):
        a = oracle.cfl_dt(3, so, [10, 10, 10], 2000.0)
        b = 10 * math.sqrt(4 / oracle.a2(3, so)) / 2000.0
        assert abs(a - b) < 1e-15
        # 2D uses hx, hz only
        c = oracle.cfl_dt(2, so, [10, 123.0, 10], 2000.0)
        d = 10 * math.sqrt(4 / oracle.a2(2, so)) / 2000.0
        assert abs(c - d) < 1e-15
