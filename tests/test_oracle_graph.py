"""Pins of the oracle's kNN graph against brute force and invariants.

The paper connects every point to its k nearest neighbours (Sec. III.B) and
links nested levels (Sec. III.C); it prints no worked example, so the oracle
is pinned by an O(N^2) brute force with the same key, by lattice clouds full
of exact ties, and by structural invariants of the multi-scale union.
"""
import numpy as np
import pytest

from oracle import graph as og


def brute_knn(pos, queries, cand_end, k):
    """Full distance matrix and a lexicographic (d2, j) sort per row."""
    p = pos.astype(np.float64)
    out = []
    for q in queries:
        j = np.arange(cand_end)
        j = j[j != q]
        d = p[j] - p[q]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        o = np.lexsort((j, d2))
        out.append(j[o[:k]])
    return np.array(out, dtype=np.int32)


def test_knn_matches_brute_force_random():
    g = np.random.default_rng(0)
    pos = g.standard_normal((600, 3)).astype(np.float32)
    q = np.arange(600)
    assert (og.knn(pos, q, 600, 6) == brute_knn(pos, q, 600, 6)).all()
    # queries outside the candidate prefix (cross-level)
    q = np.arange(100, 600)
    assert (og.knn(pos, q, 100, 3) == brute_knn(pos, q, 100, 3)).all()


def test_knn_lattice_ties_go_to_lower_index():
    g = np.random.default_rng(1)
    ijk = np.stack(np.meshgrid(np.arange(7), np.arange(7), np.arange(7), indexing="ij"), -1).reshape(-1, 3)
    pos = (0.25 * ijk[g.permutation(len(ijk))]).astype(np.float32)
    q = np.arange(len(pos))
    got = og.knn(pos, q, len(pos), 6)
    assert (got == brute_knn(pos, q, len(pos), 6)).all()
    # an interior lattice point has 6 axis neighbours at the same distance:
    # they must come out in ascending index order
    d2 = ((pos[got] - pos[q][:, None]) ** 2).sum(-1)
    same = np.isclose(d2, d2[:, :1]).all(axis=1)
    assert same.sum() > 50
    assert (np.diff(got[same], axis=1) > 0).all()


def test_knn_duplicate_points_are_neighbours_self_is_not():
    pos = np.array([[0, 0, 0], [0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 3, 0]], dtype=np.float32)
    got = og.knn(pos, np.arange(5), 5, 2)
    assert got[0].tolist() == [1, 2]
    assert got[1].tolist() == [0, 2]
    assert got[3].tolist() == [2, 0]


def test_multiscale_nesting_degree_pattern_and_dedupe():
    g = np.random.default_rng(2)
    pos = g.standard_normal((800, 3))
    pos = (pos / np.linalg.norm(pos, axis=1, keepdims=True)).astype(np.float32)
    levels = [50, 200, 800]
    G = og.build_graph(pos, levels, 6, 3)
    deg = G.degree()
    # upper bounds 6+3 / 6+6+3 / 6+6+6 (cross lists of coarse points repeat
    # their own intra lists); duplicates between lists are removed
    assert (deg[200:] <= 9).all() and (deg[200:] >= 6).all()
    assert (deg[50:200] <= 15).all() and (deg[50:200] >= 6).all()
    assert (deg[:50] <= 18).all() and (deg[:50] >= 6).all()
    assert deg.max() > 9
    # each segment is exactly the set union of the node's lists
    lists = {}
    for l, n in enumerate(levels):
        nb = og.knn(pos, np.arange(n), n, 6)
        for r in range(n):
            lists.setdefault(r, set()).update(nb[r].tolist())
        if l >= 1:
            nb = og.knn(pos, np.arange(n), levels[l - 1], 3)
            for r in range(n):
                lists[r].update(nb[r].tolist())
    for r in range(800):
        assert G.col[G.row_ptr[r]:G.row_ptr[r + 1]].tolist() == sorted(lists[r])
    # every per-level 6-NN edge is present
    for l, n in enumerate(levels):
        nb = og.knn(pos, np.arange(n), n, 6)
        for r in range(0, n, 7):
            seg = set(G.col[G.row_ptr[r]:G.row_ptr[r + 1]].tolist())
            assert set(nb[r].tolist()) <= seg
    # segments sorted, no duplicate pairs, no self loops
    for r in range(800):
        seg = G.col[G.row_ptr[r]:G.row_ptr[r + 1]]
        assert (np.diff(seg) > 0).all()
        assert r not in seg


def test_cross_level_all_queries_equals_new_points_only():
    """A point inherited from level l-1 finds, among level l-1, exactly the
    first k_cross entries of its own level-(l-1) list, so querying every
    level-l point and querying only the new ones give the same edge set."""
    g = np.random.default_rng(3)
    pos = g.standard_normal((900, 3)).astype(np.float32)
    levels = [60, 240, 900]
    G = og.build_graph(pos, levels, 6, 3)
    recv, send = [], []
    for l, n in enumerate(levels):
        q = np.arange(n)
        recv.append(np.repeat(q, 6))
        send.append(og.knn(pos, q, n, 6).reshape(-1))
        if l >= 1:
            q = np.arange(levels[l - 1], n)
            recv.append(np.repeat(q, 3))
            send.append(og.knn(pos, q, levels[l - 1], 3).reshape(-1))
    G2 = og.Graph(900, np.concatenate(recv), np.concatenate(send))
    assert (G.row_ptr == G2.row_ptr).all() and (G.col == G2.col).all()


def test_csc_is_the_stable_transpose():
    g = np.random.default_rng(4)
    pos = g.standard_normal((300, 3)).astype(np.float32)
    G = og.build_graph(pos, [100, 300], 5, 2)
    perm = G.csc_perm
    assert sorted(perm.tolist()) == list(range(G.n_edges))
    s, r = G.col[perm], G.recv[perm]
    assert (np.diff(s) >= 0).all()
    same = np.diff(s) == 0
    assert (np.diff(r)[same] > 0).all()
    assert (np.diff(G.csc_ptr) == np.bincount(G.col, minlength=300)).all()


def test_translation_invariance_exact():
    """Coordinates on a 2^-16 grid, |x| < 8, shifted by a multiple of 2^-16:
    every difference is exact in float32, so graph and edge features are
    bitwise unchanged (the features use x_s - x_r only, Sec. II.E)."""
    from oracle import model as om
    g = np.random.default_rng(5)
    pos = (np.round(g.uniform(-2, 2, (400, 3)) * 65536) / 65536).astype(np.float32)
    shift = (np.array([1.5, -0.75, 3.0]) + np.round(g.uniform(-1, 1, 3) * 65536) / 65536).astype(np.float32)
    pos2 = (pos + shift).astype(np.float32)
    assert ((pos2.astype(np.float64) - pos.astype(np.float64)) == shift.astype(np.float64)).all()
    G1 = og.build_graph(pos, [100, 400], 6, 3)
    G2 = og.build_graph(pos2, [100, 400], 6, 3)
    assert (G1.col == G2.col).all() and (G1.row_ptr == G2.row_ptr).all()
    en = np.array([[0, 0, 0, 0.1], [0.2, 0.2, 0.2, 0.1]], dtype=np.float32)
    assert (om.edge_features(G1, pos, en) == om.edge_features(G2, pos2, en)).all()
