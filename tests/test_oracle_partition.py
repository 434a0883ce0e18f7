"""Pins of the oracle's partitioner and halo (Sec. III.A).

* RCB sizes are exact and each cut separates the two halves along its axis.
* The halo equals the set reachable backwards within L hops, computed with a
  library shortest-path routine.
* With halo depth L, partitioned inner outputs equal the full graph; with
  depth L - 1 some boundary output differs (the empirical minimal-halo probe
  of Sec. VI).
* Partition gradients summed in order equal the full-graph gradient
  (Sec. III.A, gradient aggregation).
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from oracle import graph as og
from oracle import model as om
from oracle import partition as opart
from synth import init_params


def cloud(n, levels, seed=0):
    g = np.random.default_rng(seed)
    pos = g.standard_normal((n, 3)) * np.array([3.0, 1.0, 0.7])
    return pos.astype(np.float32)


def test_rcb_sizes_and_cuts():
    pos = cloud(1000, None)
    sizes = np.array([140, 260, 100, 300, 200])
    part = opart.rcb(pos, sizes)
    assert (np.bincount(part, minlength=5) == sizes).all()
    # the first cut splits parts {0,1} | {2,3,4} along x (largest extent)
    left = np.isin(part, [0, 1])
    assert pos[left, 0].max() <= pos[~left, 0].min()


def test_halo_is_backward_reachability():
    pos = cloud(400, None, 1)
    G = og.build_graph(pos, [100, 400], 5, 2)
    inner = np.flatnonzero(opart.rcb(pos, [150, 250]) == 0)
    A = sp.csr_matrix((np.ones(G.n_edges), G.col, G.row_ptr), shape=(G.n, G.n))
    # dist from any inner node along reversed edges: receiver r -> sender s
    dist = shortest_path(A, unweighted=True, indices=inner).min(axis=0)
    for L in (1, 2, 3):
        hop = opart.halo_hops(G, inner, L)
        expect = np.where(dist <= L, dist, -1)
        assert (hop == expect).all()


def setup_case(L=2, agg="message", seed=0):
    pos = cloud(500, None, seed)
    G = og.build_graph(pos, [120, 500], 5, 2)
    d = om.Desc(hidden=8, layers=L, activation="silu", aggregate=agg)
    blob = init_params(om.param_entries(d), 77).astype(np.float64)
    g = np.random.default_rng(seed + 10)
    node_in = g.standard_normal((500, 6)).astype(np.float32)
    tgt = g.standard_normal((500, 4)).astype(np.float32)
    en = np.array([[0, 0, 0, 0.4], [0.4, 0.4, 0.4, 0.2]], dtype=np.float32)
    return d, blob, G, pos, node_in, tgt, en


@pytest.mark.parametrize("agg", ["message", "edge"])
def test_partitioned_equals_full_with_halo_L(agg):
    L = 3
    d, blob, G, pos, node_in, tgt, en = setup_case(L, agg)
    loss_f, y_f, g_f = om.step_full(d, blob, G, node_in, pos, en, tgt)
    parts, _ = opart.partition(G, pos, [90, 160, 110, 140], L)
    loss_p, y_p, g_p = om.step_partitioned(d, blob, parts, node_in, pos, en, tgt)
    assert np.allclose(y_p, y_f, rtol=1e-12, atol=1e-12)
    assert loss_p == pytest.approx(loss_f, rel=1e-12)
    assert np.abs(g_p - g_f).max() <= 1e-12 * np.abs(g_f).max()


def test_halo_one_short_is_not_exact():
    L = 3
    d, blob, G, pos, node_in, tgt, en = setup_case(L)
    y_f = om.forward(d, blob, G, node_in, pos, en)
    parts, _ = opart.partition(G, pos, [250, 250], L - 1)
    worst = 0.0
    for p in parts:
        y = om.forward(d, blob, p.graph, node_in[p.gid], pos[p.gid], en)
        worst = max(worst, np.abs(y[: p.n_inner] - y_f[p.gid[: p.n_inner]]).max())
    assert worst > 1e-6


def test_in_cone_gives_single_outputs():
    L = 3
    d, blob, G, pos, node_in, tgt, en = setup_case(L)
    y_f = om.forward(d, blob, G, node_in, pos, en)
    seeds = [3, 77, 401]
    c = opart.in_cone(G, seeds, L)
    y = om.forward(d, blob, c.graph, node_in[c.gid], pos[c.gid], en)
    assert np.allclose(y[:3], y_f[seeds], rtol=1e-12, atol=1e-12)


def test_lazy_in_cone_equals_full_graph_cone():
    """The test helper that builds a seed's in-cone from kNN queries of the
    cone's own nodes (used at 4M points, where the whole graph is too slow
    to build) gives the same cone, node for node and edge for edge, as the
    full multi-scale graph."""
    from scipy.spatial import cKDTree
    from cases import Case, cone_graph
    case = Case(5, levels=(300, 1200, 4000), layers=4)
    G = case.oracle_graph()
    pos64 = case.inp.pos.astype(np.float64)
    trees = {n: cKDTree(pos64[:n]) for n in case.levels}
    for s in (0, 17, 3999):
        a = opart.in_cone(G, [s], case.L)
        b = opart.in_cone(cone_graph(case, s, trees), [s], case.L)
        assert (a.gid == b.gid).all() and (a.hop == b.hop).all()
        assert (a.graph.row_ptr == b.graph.row_ptr).all() and (a.graph.col == b.graph.col).all()
