"""Full-length parity: the 3D workloads run for their whole step count.

The headline workloads run 1000 (acoustic, space orders 4 to 16) and 800
(TTI and VTI, space order 8) steps; FP32 rounding accumulates over the run,
so one-step parity does not bound the error at the end.  These tests run
reduced replicas of the same structure -- the same generators, spacing,
40-point layer, time step, source, wavelet and receiver line, 128^3 (acoustic)
and 96^3 (TTI, VTI) physical points -- for the full step count on the GPU and
compare with the FP64 oracle's run of the same inputs, stored in
tests/golden/replica_*.npz by tests/golden/make_replica_golden.py (oracle
only).  Bars: receiver traces within relative L2 1e-4 of the oracle's, and
the final field within relative L2 1e-4 of its own norm on a seeded sample
of 16384 points (also reported against the largest field norm of the run).
"""
import ast
from pathlib import Path

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1608_03984_amd as P  # noqa: E402
from paper_1608_03984_amd.solver import from_problem  # noqa: E402
from tests._gpu_util import rel, say  # noqa: E402
from tests.golden.make_replica_golden import GENERATORS, model_digest  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = Path(__file__).resolve().parent / "golden"


def _load(name):
    path = GOLDEN / f"replica_{name}.npz"
    g = np.load(path, allow_pickle=False)
    kw = dict(ast.literal_eval(str(g["kwargs"])))
    p = GENERATORS[str(g["generator"])](**kw)
    assert model_digest(p) == str(g["digest"]), "the input generator no longer makes these inputs"
    return p, g


@pytest.mark.parametrize("name", ["acoustic_so4", "acoustic_so16", "tti_so8", "vti_so8"])
def test_full_length_replica(name):
    p, g = _load(name)
    say(f"case: replica {name} {p.padded} so{p.so} {p.nt} steps")
    s = from_problem(p)
    tr = s.forward(p.nt, p.src, p.wavelet, p.rec)
    u = s.get_field(P.FD_FIELD_CUR)
    r = s.get_field(P.FD_FIELD_R_CUR) if p.physics != "acoustic" else None
    torch.cuda.synchronize()
    tr = tr.cpu().numpy()
    idx = g["index"]
    us = u.reshape(-1)[torch.from_numpy(idx).to(u.device)].cpu().numpy().astype(np.float64)
    s.close()
    et = rel(tr, g["traces"])
    eu = rel(us, g["final"])
    e_diff = float(np.linalg.norm(us - g["final"]))
    # the sample's error scaled to the whole field, against the run's peak norm
    scale = np.sqrt(p.npoints / idx.size)
    epk = e_diff * scale / float(g["max_norm"])
    msg = f"  traces {et:.2e}  final field {eu:.2e} (own norm)  {epk:.2e} (peak norm)"
    if r is not None:
        rs = r.reshape(-1)[torch.from_numpy(idx).to(r.device)].cpu().numpy().astype(np.float64)
        er = rel(rs, g["final_r"])
        msg += f"  r {er:.2e}"
    say(msg)
    assert np.all(np.isfinite(tr))
    assert et < 1e-4, et
    assert eu < 1e-4, eu
    if r is not None:
        assert er < 1e-4, er
