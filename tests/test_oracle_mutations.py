"""The oracle's pins must catch plausible mistakes.

Each case copies ``oracle/fd_oracle.c`` to a temporary directory, plants one
mistake by text substitution (a wrong sign, index, spacing, term or weight),
compiles the copy, points the oracle wrapper at it, and runs pin tests that
must now fail.  The committed oracle source is never modified.
"""
import contextlib
import subprocess
from pathlib import Path

import pytest

import oracle
from tests import test_oracle_acoustic as ta
from tests import test_oracle_adjoint as tadj
from tests import test_oracle_step_points as tsp
from tests import test_oracle_tti as tt
from tests import test_oracle_vti as tv
from tests import test_oracle_weights as tw

SRC = Path(oracle.__file__).resolve().parent / "fd_oracle.c"


@contextlib.contextmanager
def mutant(tmp_path, old, new):
    """Plant the substitution old -> new (first occurrence; a tuple of strings
    plants several)."""
    text = SRC.read_text()
    olds, news = (old, new) if isinstance(old, tuple) else ((old,), (new,))
    for o, n in zip(olds, news):
        assert text.count(o) >= 1, o
        text = text.replace(o, n, 1)
    so = tmp_path / "liboracle_mutant.so"
    c = tmp_path / "fd_oracle_mutant.c"
    c.write_text(text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(so), str(c), "-lm"], check=True)
    saved = (oracle._LIB, oracle._lib_handle)
    oracle._LIB, oracle._lib_handle = so, None
    try:
        yield
    finally:
        oracle._LIB, oracle._lib_handle = saved


def caught(checks):
    for fn in checks:
        try:
            fn()
        except Exception:
            return True
    return False


ACOUSTIC = [
    lambda: ta.test_bruteforce_2d(4),
    lambda: ta.test_bruteforce_3d(4),
    lambda: ta.test_plane_wave_exact(3, 4),
]
TTI = [
    lambda: tt.test_rotated_operators_sum_to_laplacian(4),
    lambda: tt.test_rotated_operators_dense_geometric(2),
    lambda: tt.test_tti_plane_wave_exact(4),
    tt.test_dense_bruteforce_tti_run,
]
VTI = [
    lambda: tv.test_dense_bruteforce_vti_run(2, 8),
    lambda: tv.test_dense_bruteforce_vti_run(3, 4),
    lambda: tv.test_vti_plane_wave_exact(3, 2),
]
ADJOINT = [
    lambda: tadj.test_adjoint_equals_dense_transpose(4),
    lambda: tadj.test_adjoint_dot_product(3, 8),
]
STEP_POINTS = [
    lambda: tsp.check_acoustic(3, 4),
    lambda: tsp.check_acoustic(2, 4),
    lambda: tsp.check_vti(3, 4),
    lambda: tsp.check_tti(4),
]
GRADIENT = [
    lambda: tadj.test_gradient_pointwise_central_differences(2),
    tadj.test_gradient_directional_3d,
]

MUTANTS = [
    # weights: wrong alternation of the second-derivative weights
    ("w2 sign", "double sgn = (j % 2 == 1) ? 1.0 : -1.0;\n        w[j] = 2.0",
     "double sgn = (j % 2 == 0) ? 1.0 : -1.0;\n        w[j] = 2.0",
     [lambda: tw.test_second_derivative_polynomial_exactness(8)]),
    # weights: first derivative divided by j^2 instead of j
    ("w1 power", "w[j] = sgn * fact_ratio(r, j) / (double)j;",
     "w[j] = sgn * fact_ratio(r, j) / ((double)j * (double)j);",
     [lambda: tw.test_first_derivative_polynomial_exactness(4)]),
    # CFL with a1 = 2
    ("cfl a1", "return sqrt(4.0 / denom) / vmax;", "return sqrt(2.0 / denom) / vmax;",
     [tw.test_table2_dt_column]),
    # Laplacian: z term scaled with the x spacing
    ("lap spacing", "L += sz / (h[2] * h[2]);", "L += sz / (h[0] * h[2]);", ACOUSTIC),
    # Laplacian: off-by-one neighbour along z
    ("lap z index", "sz += w[j] * (at(u, n, ix, iy, iz + j) + at(u, n, ix, iy, iz - j));",
     "sz += w[j] * (at(u, n, ix, iy, iz + j) + at(u, n, ix, iy, iz - j + 1));", ACOUSTIC),
    # Laplacian: y term dropped
    ("lap y dropped", "        L += sy / (h[1] * h[1]);\n", "", ACOUSTIC),
    # damping: wrong sign on the previous level
    ("damping sign", "return (2.0 * fget(uc, i) - (1.0 - s) * fget(up, i) + A * L) / (1.0 + s);",
     "return (2.0 * fget(uc, i) - (1.0 + s) * fget(up, i) + A * L) / (1.0 + s);", ACOUSTIC),
    # source: forgetting the cell volume
    ("source volume", "un[idx[c]] += w[c] * A * (double)q[s] / (hp * (1.0 + sg));",
     "un[idx[c]] += w[c] * A * (double)q[s] / (1.0 + sg);", ACOUSTIC),
    # interpolation: corner weights swapped along x
    ("interp swap", "w[m] = (dx ? fx : 1.0 - fx) * (dz ? fz : 1.0 - fz);",
     "w[m] = (dx ? 1.0 - fx : fx) * (dz ? fz : 1.0 - fz);", ACOUSTIC),
    # TTI: sign of the xy term of G_xbar_xbar
    ("Gxx xy sign", "+ s2p * ct * ct * d.dxy - sp * s2t * d.dyz",
     "- s2p * ct * ct * d.dxy - sp * s2t * d.dyz", TTI),
    # TTI: yz cross derivative taken along xz
    ("dyz axes", "syz += wa * wb * at(f, n, ix, iy + a, iz + b);",
     "syz += wa * wb * at(f, n, ix + a, iy, iz + b);", TTI),
    # TTI: the coupling factor sqrt(1 + 2 delta) dropped in the p equation
    ("tti coupling", "A * (e2 * hp + sd * gr.gzz)", "A * (e2 * hp + gr.gzz)", TTI),
    # TTI: Gzz coefficient of dzz uses sin instead of cos
    ("Gzz dzz", "+ ct * ct * d.dzz\n", "+ st * st * d.dzz\n", TTI),
    # VTI: anisotropy factors exchanged in the p equation
    ("vti factors", "A * (e2 * dh + sd * dzz)", "A * (sd * dh + e2 * dzz)", VTI),
    # VTI: D_yy missing from the horizontal operator in 3D
    ("vti dyy", "    if (ndim == 3) dh += d2_axis(pc, n, w, r, h, ix, iy, iz, 1);\n", "", VTI),
    # VTI: vertical derivative taken of p instead of r
    ("vti dzz field", "double dzz = d2_axis(rc, n, w, r, h, ix, iy, iz, 2);",
     "double dzz = d2_axis(pc, n, w, r, h, ix, iy, iz, 2);", VTI),
    # adjoint: wrong sign of the damping factor on lambda^{k+2}
    ("adjoint damping", "(1.0 - s) * l2[i];", "(1.0 + s) * l2[i];", ADJOINT),
    # adjoint: B L applied instead of its transpose L B
    ("adjoint operand order",
     ("bl[i] = dt * dt * v * v * l1[i];",
      "l0[i] = 2.0 * l1[i] + laplacian_at(fb, n, ndim, w, r, h, ix, iy, iz) -"),
     ("bl[i] = l1[i];",
      "l0[i] = 2.0 * l1[i] + dt * dt * (double)vel[i] * (double)vel[i] *"
      " laplacian_at(fb, n, ndim, w, r, h, ix, iy, iz) -"), ADJOINT),
    # adjoint: receiver data spread without the interpolation weights
    ("adjoint receiver weights", "l0[idx[c]] += wc[c] * dk[j];", "l0[idx[c]] += dk[j];",
     ADJOINT),
    # gradient: wrong history level in the imaging condition
    ("gradient level", "const double* uk2 = hist + (size_t)(k - 1) * (size_t)N;",
     "const double* uk2 = hist + (size_t)k * (size_t)N;", GRADIENT),
    # gradient: damping factor of u^k with the wrong sign
    ("gradient damping", "(1.0 + s) * uk[i]", "(1.0 - s) * uk[i]", GRADIENT),
    # one-step entries: y and z exchanged in the flat-index decode
    ("acoustic step decode",
     "long ix = i % n.nx, iy = (i / n.nx) % n.ny, iz = i / (n.nx * n.ny);\n        out[k] = acoustic_point",
     "long ix = i % n.nx, iz = (i / n.nx) % n.nz, iy = i / (n.nx * n.nz);\n        out[k] = acoustic_point",
     STEP_POINTS),
    # one-step entries: the two time levels exchanged
    ("acoustic step levels", "fld_t up = {NULL, u_prev}, uc = {NULL, u_cur};",
     "fld_t up = {NULL, u_cur}, uc = {NULL, u_prev};", STEP_POINTS),
    # one-step entries: x and y exchanged in the TTI decode
    ("tti step decode",
     "long ix = i % n.nx, iy = (i / n.nx) % n.ny, iz = i / (n.nx * n.ny);\n        tti_point",
     "long ix = i % n.ny, iy = (i / n.ny) % n.nx, iz = i / (n.nx * n.ny);\n        tti_point",
     STEP_POINTS),
    # one-step entries: the previous levels of p and r exchanged (TTI)
    ("tti step fields",
     "fld_t pp = {NULL, p_prev}, pc = {NULL, p_cur}, rp = {NULL, r_prev}, rc = {NULL, r_cur};",
     "fld_t pp = {NULL, r_prev}, pc = {NULL, p_cur}, rp = {NULL, p_prev}, rc = {NULL, r_cur};",
     STEP_POINTS),
    # one-step entries: the current p passed for r (VTI)
    ("vti step fields", "iz = i / (n.nx * n.ny);\n        vti_point(pp, pc, rp, rc,",
     "iz = i / (n.nx * n.ny);\n        vti_point(pp, pc, rp, pc,", STEP_POINTS),
]


@pytest.mark.parametrize("name,old,new,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, checks):
    with mutant(tmp_path, old, new):
        assert caught(checks), f"planted mistake '{name}' passed every pin"
    # the real oracle still passes the same checks
    assert not caught(checks)
