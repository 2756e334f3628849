"""Write the expected results of the full-length replica runs (oracle only).

The 3D workloads run for 1000 (acoustic) and 800 (VTI, TTI) steps; their
full-size oracle runs take hours, so parity over the whole run is checked on
reduced replicas with the same structure (same generator, spacing, layer,
time step, source and wavelet; fewer physical points).  Running the FP64
oracle on them takes minutes, longer than a GPU test should wait, so this
script runs it once and stores what the GPU run is compared with:

* the receiver traces [nt][nrec] (the workload's "line" receivers);
* the final wavefield u^nt (TTI/VTI: p^nt and r^nt) at a fixed seeded sample
  of flat indices of the padded array, with the full-field L2 norm of u^nt;
* the largest full-field L2 norm over the run (taken every 50 steps).

It calls only ``oracle`` and the seeded input generators of ``workloads``;
nothing here comes from the GPU path.  Usage (about 20 minutes on 8 cores):

    python tests/golden/make_replica_golden.py [case ...]
"""
from __future__ import annotations

import hashlib
import sys
import time
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent.parent
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from workloads import acoustic_3d, tti_3d, vti_3d  # noqa: E402

CHUNK = 50          # steps between the norms of the running maximum
NSAMPLE = 16384     # sampled points of the final field
SAMPLE_SEED = 1708

# name -> (generator, keyword arguments); the GPU test rebuilds the same
# problem from these arguments.
CASES = {
    "acoustic_so4": (acoustic_3d, dict(so=4, phys=128, nbl=40, nt=1000, receivers="line")),
    "acoustic_so16": (acoustic_3d, dict(so=16, phys=128, nbl=40, nt=1000, receivers="line")),
    "tti_so8": (tti_3d, dict(so=8, phys=96, nbl=40, nt=800, receivers="line")),
    "vti_so8": (vti_3d, dict(so=8, phys=96, nbl=40, nt=800, receivers="line")),
}
GENERATORS = {"acoustic_3d": acoustic_3d, "tti_3d": tti_3d, "vti_3d": vti_3d}


def model_digest(p) -> str:
    """sha256[:16] of the problem's FP32 model fields, wavelet and points."""
    h = hashlib.sha256()
    for a in (p.vel, p.eta, p.eps, p.delta, p.theta, p.phi, p.wavelet):
        if a is not None:
            h.update(np.ascontiguousarray(a, np.float32).tobytes())
    for a in (p.src, p.rec):
        h.update(np.ascontiguousarray(a, np.float64).tobytes())
    return h.hexdigest()[:16]


def sample_indices(npoints: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.unique(rng.integers(0, npoints, NSAMPLE)).astype(np.int64)


def run_case(name: str) -> None:
    gen, kw = CASES[name]
    p = gen(**kw)
    t0 = time.time()
    nt, so = p.nt, p.so
    traces = []
    maxnorm = 0.0
    state = None
    for n0 in range(0, nt, CHUNK):
        k = min(CHUNK, nt - n0)
        w = p.wavelet[n0:n0 + k]
        if p.physics == "acoustic":
            up, uc = (None, None) if state is None else state
            tr, up, uc = oracle.acoustic_forward(3, p.nbl, p.spacing, p.dt, so, p.vel, p.eta,
                                                 p.src, w, p.rec, k, u_prev=up, u_cur=uc)
            state = (up, uc)
            cur = uc
        elif p.physics == "tti":
            tr, state = oracle.tti_forward(p.nbl, p.spacing, p.dt, so, p.vel, p.eta, p.eps,
                                           p.delta, p.theta, p.phi, p.src, w, p.rec, k,
                                           state=state)
            cur = state[1]
        else:
            tr, state = oracle.vti_forward(3, p.nbl, p.spacing, p.dt, so, p.vel, p.eta, p.eps,
                                           p.delta, p.src, w, p.rec, k, state=state)
            cur = state[1]
        traces.append(tr)
        maxnorm = max(maxnorm, float(np.linalg.norm(cur)))
        print(f"{name}: step {n0 + k}/{nt} ({time.time() - t0:.0f} s)", flush=True)
    idx = sample_indices(p.npoints)
    out = dict(
        traces=np.concatenate(traces, axis=0),
        index=idx,
        final=state[1].reshape(-1)[idx],
        final_norm=np.float64(np.linalg.norm(state[1])),
        max_norm=np.float64(maxnorm),
        digest=np.array(model_digest(p)),
        generator=np.array(p.name),
        kwargs=np.array(repr(sorted(kw.items()))),
    )
    if p.physics != "acoustic":
        out["final_r"] = state[3].reshape(-1)[idx]
        out["final_r_norm"] = np.float64(np.linalg.norm(state[3]))
    np.savez_compressed(HERE / f"replica_{name}.npz", **out)
    print(f"{name}: wrote replica_{name}.npz in {time.time() - t0:.0f} s", flush=True)


def main(argv) -> None:
    oracle.set_threads(8)
    for name in (argv or list(CASES)):
        run_case(name)


if __name__ == "__main__":
    main(sys.argv[1:])
