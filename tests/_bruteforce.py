"""Dense-matrix brute force: a third code path for pinning the oracle.

Nothing here shares code with the oracle or the GPU library.  Finite-difference
weights come from solving the Taylor (Vandermonde) conditions with
``numpy.linalg.solve``; operators are assembled as dense matrices from 1D
Toeplitz blocks with Kronecker products (truncated at the array edge, which
is the zero-ghost boundary); time stepping is a dense matrix-vector product.
Only tiny grids (a few hundred points) are practical.
"""
import math

import numpy as np


def taylor_weights(deriv: int, r: int) -> np.ndarray:
    """Weights c[-r..r] with sum_j c_j j^p = p! [p == deriv] for p = 0..2r.
    Returned as an array of length 2r + 1 indexed by j + r."""
    j = np.arange(-r, r + 1, dtype=np.float64)
    V = np.vstack([j ** p for p in range(2 * r + 1)])
    rhs = np.zeros(2 * r + 1)
    rhs[deriv] = math.factorial(deriv)
    return np.linalg.solve(V, rhs)


def toeplitz_1d(n: int, c: np.ndarray) -> np.ndarray:
    """n x n banded matrix applying stencil c (length 2r+1) with zero ghosts."""
    r = (c.size - 1) // 2
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(-r, r + 1):
            if 0 <= i + j < n:
                M[i, i + j] = c[j + r]
    return M


def axis_op(shape_zyx, axis_xyz: int, M1: np.ndarray) -> np.ndarray:
    """Embed a 1D operator acting along x (0), y (1) or z (2) of a C-order
    [nz][ny][nx] field as a dense N x N matrix."""
    nz, ny, nx = shape_zyx
    I = np.eye
    if axis_xyz == 0:
        return np.kron(I(nz), np.kron(I(ny), M1))
    if axis_xyz == 1:
        return np.kron(I(nz), np.kron(M1, I(nx)))
    return np.kron(M1, np.kron(I(ny), I(nx)))


def second_derivative_ops(shape_zyx, so, spacing):
    r = so // 2
    c2 = taylor_weights(2, r)
    nz, ny, nx = shape_zyx
    ns = (nx, ny, nz)
    return [axis_op(shape_zyx, a, toeplitz_1d(ns[a], c2)) / spacing[a] ** 2 for a in range(3)]


def first_derivative_ops(shape_zyx, so, spacing):
    r = so // 2
    c1 = taylor_weights(1, r)
    nz, ny, nx = shape_zyx
    ns = (nx, ny, nz)
    return [axis_op(shape_zyx, a, toeplitz_1d(ns[a], c1)) / spacing[a] for a in range(3)]


def interp_row(shape_zyx, nbl, spacing, coord, ndim):
    """Row vector of multilinear interpolation weights for one point."""
    nz, ny, nx = shape_zyx
    if ndim == 2:
        axes = [(coord[0], spacing[0], nx), (0.0, 1.0, 1), (coord[1], spacing[2], nz)]
        offs = [nbl, 0, nbl]
    else:
        axes = [(coord[0], spacing[0], nx), (coord[1], spacing[1], ny), (coord[2], spacing[2], nz)]
        offs = [nbl, nbl, nbl]
    per_axis = []
    for (c, h, n), o in zip(axes, offs):
        vec = np.zeros(n)
        if n == 1:
            vec[0] = 1.0
        else:
            g = c / h + o
            i = min(int(np.floor(g)), n - 2)
            f = g - i
            vec[i] += 1.0 - f
            vec[i + 1] += f
        per_axis.append(vec)
    vx, vy, vz = per_axis
    return np.kron(vz, np.kron(vy, vx))
