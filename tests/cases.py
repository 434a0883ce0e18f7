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
        self.desc = om.Desc(hidden=self.H, layers=self.L, activation=activation, aggregate=aggregate)
        self.params = init_params(om.param_entries(self.desc), self.cfg.seed("weights"))
        self.N = self.levels[-1]
        self._graph = None

    def oracle_graph(self):
        if self._graph is None:
            self._graph = og.build_graph(self.inp.pos, self.levels, self.k_intra, self.k_cross)
        return self._graph

    def model(self, api):
        return api.Model(self.H, self.L, activation=self.activation, precision=self.precision,
                         aggregate=self.aggregate)

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
