"""Writes the oracle regression fixtures in this folder.

The paper prints no worked example and no intermediate values, so every
fixture here is written by this script from oracle/ alone (never from the
GPU path).  They freeze the oracle's outputs on small seeded cases so that
an accidental change of its arithmetic is caught; the oracle itself is pinned
by the independent checks in tests/test_oracle_*.py.

Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import graph as og  # noqa: E402
from oracle import model as om  # noqa: E402
from synth import CONFIGS, init_params, make_inputs  # noqa: E402


def sphere_tiny():
    cfg = CONFIGS[1]
    inp = make_inputs(cfg, levels=(40, 160))
    G = og.build_graph(inp.pos, [40, 160], 4, 2)
    d = om.Desc(hidden=8, layers=2, activation="silu")
    p = init_params(om.param_entries(d), 7).astype(np.float64)
    loss, y, g = om.step_full(d, p, G, inp.node_in, inp.pos, inp.edge_norm, inp.targets)
    return {
        "case": "sphere 40/160 points, k=4 intra, k=2 cross, H=8, L=2, SiLU, params seed 7",
        "row_ptr": G.row_ptr.tolist(), "col": G.col.tolist(),
        "y_first_rows": y[:8].tolist(), "loss": loss,
        "grad_norm_per_tensor": [float(np.linalg.norm(g[sl])) for sl in _slices(d)],
    }


def _slices(d):
    out, off = [], 0
    for _, _, s in om.layout(d):
        n = int(np.prod(s))
        out.append(slice(off, off + n))
        off += n
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_sphere_tiny.json"), "w") as f:
        json.dump(sphere_tiny(), f, indent=0)
    print("written")
