"""The learned coarse-grid correction end to end on small grids: training
pairs from the fine (space order 16, h) and coarse (space order 4, 2h)
solvers, training by libfd's own forward/backward kernels and Adam, and the
corrected coarse solver against the plain one, both measured against the fine
solve's receiver traces.

What is asserted:
  * training lowers the masked loss on its samples well below the loss of no
    correction, and the trained network also lowers it on held-out models
    (it has learned part of the coarse solver's one-window error, not the
    training models);
  * the correction scheme itself works: with the exact residual in place of
    the network, the late traces of receivers outside the source ball match
    the fine solve far better than the plain coarse solve's;
  * the corrected solver stays stable (finite traces, whole-run error within
    10 % of the plain coarse solver's: a trained network that makes the run
    worse than that is a regression).
What the trained network gains over the plain coarse solver over a whole run
is measured and printed; on these small models it is 1.06x on one held-out
model and 0.98x on the other, so it is reported, not asserted (the
learned-correction target is not met: its cost, not its accuracy, rules it
out against a higher-order plain solve).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1608_03984_amd import learned as Lm  # noqa: E402
from tests._gpu_util import say  # noqa: E402
from workloads import learned_model  # noqa: E402

pytestmark = pytest.mark.gpu

PHYS, NBL, NT_F, K = 48, 12, 800, 8


def _model(seed):
    return learned_model(seed, phys_f=PHYS, nbl_f=NBL, nt_f=NT_F)


def test_learned_correction_small():
    nt_c = NT_F // 2
    shape_c = (PHYS // 2 + NBL,) * 3
    m0 = _model(100)
    start = Lm.correction_start(m0)
    times = list(range(start + K, nt_c + 1, 6))
    say(f"case: learned correction {shape_c}, K {K}, corrections from step {start}")
    train_s, held_s = [], []
    for seed, dest in [(100 + i, train_s) for i in range(24)] + [(900, held_s), (901, held_s)]:
        pair = Lm.make_pair(_model(seed))
        dest += Lm.training_pairs(pair, times, K)
        pair.close()
    net = Lm.CorrectionNet(seed=1, out_scale=0.01)
    none_t = Lm.sample_loss(None, train_s, shape_c)
    Lm.train(net, train_s, shape_c, 1500, lr=1e-3, lr_end=1e-4)
    after = Lm.sample_loss(net, train_s, shape_c)
    none_h = Lm.sample_loss(None, held_s, shape_c)
    net_h = Lm.sample_loss(net, held_s, shape_c)
    say(f"  window loss: training no correction {none_t:.3e}, trained {after:.3e}; held-out "
        f"no correction {none_h:.3e}, trained {net_h:.3e} (gain {none_h / net_h:.2f}x)")
    assert after < 0.85 * none_t
    assert net_h < 0.85 * none_h
    for seed in (900, 901):
        m = _model(seed)
        pair = Lm.make_pair(m)
        far = Lm.far_receivers(pair, Lm.SRC_RADIUS * m["h_c"][0])
        tf = Lm.solve_fine(pair, NT_F).clone()
        tc = Lm.solve_coarse(pair, nt_c).clone()
        tl = Lm.solve_coarse(pair, nt_c, K, net, start=start).clone()
        tx = Lm.solve_coarse_exact(pair, nt_c, K, start=start).clone()
        pair.close()
        e0, e1 = Lm.trace_error(tc, tf), Lm.trace_error(tl, tf)
        l0 = Lm.trace_error(tc, tf, far, start)
        l1 = Lm.trace_error(tl, tf, far, start)
        lx = Lm.trace_error(tx, tf, far, start)
        say(f"  held-out model {seed}: trace error plain {e0:.4f}, learned {e1:.4f} "
            f"(gain {e0 / e1:.2f}x); far receivers after step {start}: plain {l0:.4f}, "
            f"learned {l1:.4f}, exact residual {lx:.4f}")
        assert bool(torch.isfinite(tl).all())
        assert e1 < 1.1 * e0
        assert lx < 0.1 * l0
