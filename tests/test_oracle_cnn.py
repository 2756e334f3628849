"""Pins for the FP64 oracle of the correction network (oracle/cnn.py).

  * the shift-and-matmul convolution equals the definition written as loops;
  * a one-hot tap with an identity matrix is a pure shift;
  * backward-data is the adjoint of the convolution (dot-product identity),
    backward-weight its adjoint in the weights;
  * the network gradient equals central differences of the FP64 loss;
  * Adam's first step has a closed form, and so have five steps of a
    constant and of a sign-alternating gradient (moments carried, bias
    corrections 1 - beta^t); bf16 rounding is exact on representable values
    and rounds half to even.
Planted mistakes in a copy of the module must fail these pins.
"""
import importlib.util
from pathlib import Path

import numpy as np
import pytest

import oracle
from oracle import cnn as C

SRC = Path(oracle.__file__).resolve().parent / "cnn.py"


def _params(rng, cin, c, cout):
    return (rng.standard_normal((27, cin, c)) * 0.3, rng.standard_normal(c) * 0.1,
            rng.standard_normal((27, c, c)) * 0.2, rng.standard_normal(c) * 0.1,
            rng.standard_normal((27, c, cout)) * 0.2, rng.standard_normal(cout) * 0.1)


def check_conv_matches_loops(M=C):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 5, 6, 3))
    w = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    np.testing.assert_allclose(M.conv3d(x, w, b), M.conv3d_loops(x, w, b), rtol=1e-12, atol=1e-12)


def check_adjoints(M=C):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((5, 4, 6, 4))
    w = rng.standard_normal((27, 4, 3))
    y = rng.standard_normal((5, 4, 6, 3))
    lhs = np.sum(M.conv3d(x, w) * y)
    assert np.sum(x * M.conv3d_backward_data(y, w)) == pytest.approx(lhs, rel=1e-12)
    dw, db = M.conv3d_backward_weight(x, y)
    assert np.sum(w * dw) == pytest.approx(lhs, rel=1e-12)
    assert np.allclose(db, y.reshape(-1, 3).sum(0))


def check_net_gradient(M=C):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 4, 5, 3))
    target = rng.standard_normal((4, 4, 5, 2))
    mask = np.zeros((4, 4, 5), bool)
    mask[1:3, 1:3, 1:4] = True
    params = [np.array(p) for p in _params(rng, 3, 4, 2)]
    out, cache = M.net_forward(x, params)
    grads = M.net_backward(M.loss_grad(out, target, mask), params, cache)
    h = 1e-6
    for k, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for i in rng.choice(flat.size, min(12, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + h
            lp = M.loss(M.net_forward(x, params)[0], target, mask)
            flat[i] = old - h
            lm = M.loss(M.net_forward(x, params)[0], target, mask)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g.reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, g.reshape(-1)[i])


def check_adam_sequence(M=C):
    """Five carried Adam steps against closed forms written from the
    recurrences m_t = b1 m + (1-b1) g_t, v_t = b2 v + (1-b2) g_t^2 with zero
    initial moments:
      constant g:            m_t = (1 - b1^t) g,  v_t = (1 - b2^t) g^2, so
                             every bias-corrected step is g / (|g| + eps);
      g_t = (-1)^(t+1) g:    m_t = (1-b1) g (-1)^(t+1) (1 - (-b1)^t) / (1 + b1),
                             v_t = (1 - b2^t) g^2."""
    rng = np.random.default_rng(6)
    b1, b2, eps, lr, T = 0.9, 0.999, 1e-8, 1e-2, 5
    g = rng.standard_normal(8) + np.sign(rng.standard_normal(8)) * 0.5
    p0 = rng.standard_normal(8)
    for alternating in (False, True):
        p, m, v = p0.copy(), np.zeros(8), np.zeros(8)
        ref = p0.copy()
        for t in range(1, T + 1):
            gt = g * (-1.0) ** (t + 1) if alternating else g
            p, m, v = M.adam_step(p, gt, m, v, t, lr, b1, b2, eps)
            if alternating:
                mt = (1 - b1) * g * (-1.0) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
            else:
                mt = (1 - b1 ** t) * g
            vt = (1 - b2 ** t) * g * g
            np.testing.assert_allclose(m, mt, rtol=1e-12, atol=1e-15)
            np.testing.assert_allclose(v, vt, rtol=1e-12, atol=1e-15)
            ref = ref - lr * (mt / (1 - b1 ** t)) / (np.abs(g) + eps)
            np.testing.assert_allclose(p, ref, rtol=1e-12, atol=1e-14)


def test_adam_sequence_closed_forms():
    check_adam_sequence()


def test_conv_matches_loops():
    check_conv_matches_loops()


def test_one_hot_tap_is_a_shift():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((5, 6, 7, 2))
    for t, (dz, dy, dx) in enumerate(C.OFFSETS):
        w = np.zeros((27, 2, 2))
        w[t] = np.eye(2)
        out = C.conv3d(x, w)
        ref = np.zeros_like(x)
        D, H, W = x.shape[:3]
        zs = slice(max(0, -dz), min(D, D - dz))
        ys = slice(max(0, -dy), min(H, H - dy))
        xs = slice(max(0, -dx), min(W, W - dx))
        ref[zs, ys, xs] = x[max(0, dz):D + min(0, dz), max(0, dy):H + min(0, dy),
                            max(0, dx):W + min(0, dx)]
        assert np.array_equal(out, ref), t


def test_backward_operators_are_adjoints():
    check_adjoints()


def test_net_gradient_equals_central_differences():
    check_net_gradient()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = C.adam_step(p, g, np.zeros(10), np.zeros(10), 1, 1e-3)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # a quadratic bowl is descended
    q = np.ones(4) * 3.0
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 400):
        q, m, v = C.adam_step(q, 2 * q, m, v, t, 0.05)
    assert np.abs(q).max() < 0.1


def test_bf16_rounding():
    exact = np.array([1.0, -2.5, 0.15625, 3.0 * 2.0 ** -20], np.float32)
    assert np.array_equal(C.bf16_round(exact), exact.astype(np.float64))
    one = np.float32(1.0)
    half = np.float32(1.0 + 2.0 ** -8)        # halfway between 1 and 1 + 2^-7
    assert C.bf16_round(np.array([half]))[0] == 1.0                  # ties to even
    odd_half = np.float32(1.0 + 3 * 2.0 ** -8)  # halfway between 1+2^-7 and 1+2^-6
    assert C.bf16_round(np.array([odd_half]))[0] == 1.0 + 2.0 ** -6
    assert C.bf16_round(np.array([np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)]))[0] == 1.0 + 2.0 ** -7
    assert one == 1.0


MUTANTS = [
    ("backward-data offset sign", "dx += _shift(dz, -oz, -oy, -ox) @ w[t].T",
     "dx += _shift(dz, oz, oy, ox) @ w[t].T", [check_adjoints, check_net_gradient]),
    ("backward-data flipped taps", "dx += _shift(dz, -oz, -oy, -ox) @ w[t].T",
     "dx += _shift(dz, -oz, -oy, -ox) @ w[26 - t].T", [check_adjoints, check_net_gradient]),
    ("backward-weight offset", "dw[t] = _shift(x, oz, oy, ox)", "dw[t] = _shift(x, -oz, -oy, -ox)",
     [check_adjoints, check_net_gradient]),
    ("relu mask on the wrong layer", "dz1 = conv3d_backward_data(dz2, w2) * (z1 > 0)",
     "dz1 = conv3d_backward_data(dz2, w2) * (z2 > 0)", [check_net_gradient]),
    ("loss without the 1/n", "g[m] = (out - np.asarray(target, np.float64))[m] / max(int(m.sum()), 1)",
     "g[m] = (out - np.asarray(target, np.float64))[m]", [check_net_gradient]),
    ("tap order", "OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]",
     "OFFSETS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]",
     [check_conv_matches_loops]),
    ("adam bias correction without the power", "vh = v / (1 - beta2 ** t)",
     "vh = v / (1 - beta2)", [check_adam_sequence]),
    ("adam first-moment correction without the power", "mh = m / (1 - beta1 ** t)",
     "mh = m / (1 - beta1)", [check_adam_sequence]),
    ("adam moments not carried", "return param - lr * mh / (np.sqrt(vh) + eps), m, v",
     "return param - lr * mh / (np.sqrt(vh) + eps), m * 0, v * 0", [check_adam_sequence]),
    ("adam second moment of the gradient, not its square",
     "v = beta2 * v + (1 - beta2) * grad * grad", "v = beta2 * v + (1 - beta2) * np.abs(grad)",
     [check_adam_sequence]),
]


@pytest.mark.parametrize("name,old,new,checks", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, checks):
    text = SRC.read_text()
    assert old in text, old
    path = tmp_path / "cnn_mutant.py"
    path.write_text(text.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location("cnn_mutant", path)
    M = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(M)
    caught = False
    for fn in checks:
        try:
            fn(M)
        except Exception:
            caught = True
            break
    assert caught, f"planted mistake '{name}' passed every pin"
