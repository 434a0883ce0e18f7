"""Shared helpers for the GPU parity tests: seeded cases, the oracle side and
the library side of each comparison, and the error measures."""
from __future__ import annotations

import sys
import time

import numpy as np

from oracle import graph as og
from oracle import model as om
from synth import CONFIGS, init_params, make_inputs


def log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


class Case:
    """Inputs of one parity case: a config recipe at reduced or full size."""

    def __init__(self, cfg_idx, levels=None, hidden=None, layers=None, precision="fp32", activation="relu",
                 aggregate="message"):
        self.cfg = CONFIGS[cfg_idx]
        self.inp = make_inputs(self.cfg, levels=levels)
        self.levels = [int(x) for x in self.inp.level_end]
        self.H = hidden or self.cfg.hidden
        self.L = layers or self.cfg.layers
        self.k_intra, self.k_cross = self.cfg.k_intra, (self.cfg.k_cross if len(self.levels) > 1 else 0)
        self.precision = precision
        self.activation = activation
        self.aggregate = aggregate
        self.desc = om.Desc(hidden=self.H, layers=self.L, node_in=self.cfg.node_in, activation=activation,
                            aggregate=aggregate)
        self.params = init_params(om.param_entries(self.desc), self.cfg.seed("weights"))
        self.N = self.levels[-1]
        self._graph = None

    def oracle_graph(self):
        if self._graph is None:
            self._graph = og.build_graph(self.inp.pos, self.levels, self.k_intra, self.k_cross)
        return self._graph

    def model(self, api):
        return api.Model(self.H, self.L, node_in=self.cfg.node_in, activation=self.activation,
                         precision=self.precision, aggregate=self.aggregate)

    def tensor_slices(self):
        """(name, slice) of every parameter tensor, in blob order."""
        out, off = [], 0
        for b, k, s in om.layout(self.desc):
            n = int(np.prod(s))
            out.append((f"{b}.{k}{len(out)}", slice(off, off + n)))
            off += n
        return out


def per_tensor_errors(case: Case, got, ref):
    """rel-L2 of every parameter tensor's gradient."""
    return {name: rel_l2(got[sl], ref[sl]) for name, sl in case.tensor_slices()}


def oracle_refs(case: Case, G=None):
    """FP64 oracle steps on the whole graph: at the FP32 master weights and,
    for the BF16 form, also at the weights that form multiplies with
    (hidden-to-hidden weights cast to bfloat16, as mixed-precision training
    does).  Returns (base, amp); amp is None for FP32."""
    G = case.oracle_graph() if G is None else G
    args = (G, case.inp.node_in, case.inp.pos, case.inp.edge_norm, case.inp.targets)
    base = om.step_full(case.desc, case.params.astype(np.float64), *args)
    amp = om.step_full(case.desc, om.amp_cast(case.desc, case.params), *args) if case.precision == "bf16" else None
    return base, amp


def check_step(case: Case, out, loss, grad, refs) -> str:
    """The parity bar for one forward + backward; returns a summary line.

    FP32: outputs and loss <= 1e-4 relative.  Gradients: 1e-4 per tensor
    under SiLU; under ReLU the derivative is a 0/1 decision on the sign of a
    pre-activation and FP32-sized (1e-7) perturbations of the FP64 oracle
    itself move single tensors by ~1e-4 (a kink flips), so there the whole
    gradient is held to 1e-4 and each tensor to 1e-3.

    BF16: against the oracle at the cast weights (the arithmetic the form
    performs) every output and every gradient tensor <= 2e-2; against the
    oracle at the FP32 master weights (the model) the outputs, the loss and
    the whole gradient <= 2e-2, with the worst tensor reported.  The cast
    alone moves the deepest gradient tensors (encoder input layers and
    first-layer biases) by up to ~2.3e-2 at 5 layers."""
    (loss_r, y_r, g_r), amp = refs
    assert np.isfinite(out).all() and np.isfinite(grad).all()
    errs = per_tensor_errors(case, grad, g_r)
    worst = sorted(errs.items(), key=lambda kv: -kv[1])[:2]
    total = rel_l2(grad, g_r)
    e_out = rel_l2(out, y_r)
    e_loss = abs(loss - loss_r) / loss_r
    if case.precision == "fp32":
        assert e_out <= 1e-4, e_out
        assert e_loss <= 1e-4, e_loss
        if case.activation == "silu":
            assert worst[0][1] <= 1e-4, worst
        else:
            assert total <= 1e-4, (total, worst)
            assert worst[0][1] <= 1e-3, worst
        return f"out {e_out:.2e} loss {e_loss:.2e} grad {total:.2e} worst {worst}"
    loss_a, y_a, g_a = amp
    assert e_out <= 2e-2, e_out
    assert e_loss <= 2e-2, e_loss
    assert total <= 2e-2, (total, worst)
    errs_a = per_tensor_errors(case, grad, g_a)
    worst_a = sorted(errs_a.items(), key=lambda kv: -kv[1])[:2]
    e_out_a = rel_l2(out, y_a)
    assert e_out_a <= 2e-2, e_out_a
    assert worst_a[0][1] <= 2e-2, worst_a
    return (f"vs model: out {e_out:.2e} loss {e_loss:.2e} grad {total:.2e} worst {worst} | "
            f"vs cast weights: out {e_out_a:.2e} grad {rel_l2(grad, g_a):.2e} worst {worst_a}")


def cone_graph(case, seeds, trees):
    """The in-lists of every node within L - 1 hops of the seed node(s)
    (receiver = query), computed node set by node set with the oracle's kNN
    over the full cloud, as an oracle Graph over all N nodes whose other
    rows are empty.  The L-hop in-cone of the seeds in it (a sampled output,
    or a partition with its halo) equals their in-cone in the full
    multi-scale graph, whose whole construction takes minutes at 4M points.
    trees: {candidate count: cKDTree over those points} for every level."""
    pos, le = case.inp.pos, case.levels
    frontier = np.unique(np.atleast_1d(np.asarray(seeds, dtype=np.int64)))
    seen = np.zeros(case.N, dtype=bool)
    seen[frontier] = True
    recv, send = [], []
    for _ in range(case.L):  # rows of hops 0 .. L-1
        for lvl, n_l in enumerate(le):
            q = frontier[frontier < n_l]
            if len(q) == 0:
                continue
            nb = og.knn(pos, q, n_l, case.k_intra, trees[n_l])
            recv.append(np.repeat(q, case.k_intra))
            send.append(nb.reshape(-1).astype(np.int64))
            if lvl >= 1 and case.k_cross > 0:
                nb = og.knn(pos, q, le[lvl - 1], case.k_cross, trees[le[lvl - 1]])
                recv.append(np.repeat(q, case.k_cross))
                send.append(nb.reshape(-1).astype(np.int64))
        new = np.unique(np.concatenate(send))
        new = new[~seen[new]]
        seen[new] = True
        frontier = new
    return og.Graph(case.N, np.concatenate(recv), np.concatenate(send))
