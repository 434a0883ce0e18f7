"""Writes the full-size sampled-output fixtures: the FP64 oracle's outputs at
64 seeded nodes of the 400k-point 3-level ellipsoid (H = 128) and of the
4M-point 3-level car (H = 256), 15 layers, each evaluated through the node's
15-hop in-cone (an output depends on nothing else, Eq. 4), at the FP32
master weights and at the bfloat16-cast weights that the BF16 form multiplies
with.  A whole-graph FP64 run of these workloads is out of reach on a host
(its checkpoints alone would take tens to hundreds of GB), so the GPU tests
compare their full-size outputs with these.

Calls only oracle/, synth/ and the oracle-side helpers of tests/cases.py
(never the GPU path).  Each fixture records a digest of the inputs it was
computed from; the GPU test refuses a fixture whose digest no longer matches.

Run: python tests/golden/make_fullsize_golden.py [workload ...]   (about 20 min
for the car on 8 cores)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from cases import Case, cone_graph  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import partition as opart  # noqa: E402

WORKLOADS = {"ellipsoid-ms-400k": 3, "car-ms-4m-16p": 5}
N_SEEDS = 64


def fixture_path(workload: str) -> str:
    return os.path.join(HERE, f"fullsize_{workload}.json")


def inputs_digest(case: Case) -> str:
    """Digest of every input the outputs depend on."""
    h = hashlib.sha256()
    for a in (case.inp.pos, case.inp.node_in, case.params, np.asarray(case.inp.edge_norm, np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(json.dumps([case.levels, case.k_intra, case.k_cross, case.H, case.L, case.activation]).encode())
    return h.hexdigest()[:16]


def seeds_for(case: Case, cfg_idx: int) -> np.ndarray:
    rng = np.random.default_rng(1000 * cfg_idx + 99)
    return np.sort(rng.choice(case.N, N_SEEDS, replace=False))


def sampled(workload: str) -> dict:
    from scipy.spatial import cKDTree
    cfg_idx = WORKLOADS[workload]
    case = Case(cfg_idx, precision="bf16")
    pos64 = case.inp.pos.astype(np.float64)
    trees = {n_l: cKDTree(pos64[:n_l]) for n_l in case.levels}
    seeds = seeds_for(case, cfg_idx)
    blob = case.params.astype(np.float64)
    amp = om.amp_cast(case.desc, case.params)
    y_model, y_cast, cone = [], [], []
    t0 = time.time()
    for i, s in enumerate(seeds):
        G = cone_graph(case, int(s), trees)
        part = opart.in_cone(G, [int(s)], case.L)
        args = (part, case.inp.node_in[part.gid], case.inp.pos[part.gid], case.inp.edge_norm)
        y_model.append(om.forward_cone(case.desc, blob, *args)[0].tolist())
        y_cast.append(om.forward_cone(case.desc, amp, *args)[0].tolist())
        cone.append([len(part.gid), int(part.graph.n_edges)])
        print(f"{workload} seed {i + 1}/{len(seeds)} ({s}): cone {cone[-1]}, {time.time() - t0:.0f} s", flush=True)
    return {"workload": workload, "config": cfg_idx, "nodes": case.N, "levels": case.levels, "hidden": case.H,
            "layers": case.L, "activation": case.activation, "inputs_digest": inputs_digest(case),
            "seeds": [int(s) for s in seeds], "y_model": y_model, "y_cast": y_cast, "cone_nodes_edges": cone}


if __name__ == "__main__":
    for w in sys.argv[1:] or list(WORKLOADS):
        rec = sampled(w)
        with open(fixture_path(w), "w") as f:
            json.dump(rec, f)
        print(f"written {fixture_path(w)}")
