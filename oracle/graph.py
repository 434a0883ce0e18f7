"""Multi-scale kNN graph of a point cloud (Sec. III.B and III.C).

Reading of the paper taken here:
* A point is connected to its k nearest neighbours; the neighbour list of
  point i is N(i) of Eq. (2), so edges run sender j -> receiver i (the
  query).  Graphs are directed, with in-degree exactly k per level.
* The self match is excluded by index; other points at the same location
  remain candidates.
* Distances are squared Euclidean distances in float64 from float32
  coordinates, evaluated as ((dx*dx + dy*dy) + dz*dz) with no fused
  multiply-add.  Candidates are ranked by the key (d2, j): equal distances go
  to the lower index.
* Level l is the prefix [0, level_end[l]) of the point array, so every level
  is a superset of the coarser ones (Sec. III.C).  kNN runs within each
  level; for l >= 1 every point of level l also links to its k_cross nearest
  points of level l-1 (cross-level edges, coarse -> fine).
* The union of all lists is a set: a repeated (receiver, sender) pair is kept
  once.  Segments of the receiver-sorted CSR are ordered by sender id.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def sqdist(pos64: np.ndarray, q: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Squared distance between points q and j (index arrays), float64,
    in the fixed order ((dx*dx + dy*dy) + dz*dz)."""
    d = pos64[j] - pos64[q]
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def knn(pos: np.ndarray, queries: np.ndarray, cand_end: int, k: int, tree=None) -> np.ndarray:
    """The k nearest candidates j in [0, cand_end), j != q, of each query q,
    ranked by (d2, j).  Returns int32 [len(queries)][k].

    A k-d tree (library primitive) supplies, for each query, every candidate
    within a radius that is guaranteed to contain the k best; the exact key is
    then computed here and sorted.  `tree`: a cKDTree over the float64
    candidates pos[:cand_end], built here when not given (a caller querying
    the same candidates many times builds it once).
    """
    queries = np.asarray(queries, dtype=np.int64)
    nq = len(queries)
    if nq == 0 or k == 0:
        return np.zeros((nq, k), dtype=np.int32)
    if k >= cand_end:
        raise ValueError("k must be smaller than the candidate count")
    pos64 = pos.astype(np.float64)
    if tree is None:
        tree = cKDTree(pos64[:cand_end])
    elif tree.n != cand_end:
        raise ValueError("tree does not hold the candidates [0, cand_end)")
    kk = min(k + 1, cand_end)
    dist, _ = tree.query(pos64[queries], k=kk)
    dist = np.asarray(dist).reshape(nq, kk)
    radius = dist[:, -1] * (1.0 + 1e-9) + 1e-300
    lists = tree.query_ball_point(pos64[queries], radius)
    lens = np.fromiter((len(x) for x in lists), dtype=np.int64, count=nq)
    flat = np.fromiter((j for x in lists for j in x), dtype=np.int64, count=int(lens.sum()))
    qrow = np.repeat(np.arange(nq), lens)
    qid = queries[qrow]
    keep = flat != qid
    flat, qrow, qid = flat[keep], qrow[keep], qid[keep]
    d2 = sqdist(pos64, qid, flat)
    order = np.lexsort((flat, d2, qrow))
    flat, qrow = flat[order], qrow[order]
    start = np.searchsorted(qrow, np.arange(nq))
    take = start[:, None] + np.arange(k)[None, :]
    out = flat[take]
    assert (qrow[take] == np.arange(nq)[:, None]).all()
    return out.astype(np.int32)


def multiscale_edge_lists(pos, level_end, k_intra, k_cross):
    """Raw (receiver, sender) lists, level by level, before the union."""
    recv, send = [], []
    level_end = [int(x) for x in level_end]
    for l, n_l in enumerate(level_end):
        q = np.arange(n_l)
        nb = knn(pos, q, n_l, k_intra)
        recv.append(np.repeat(q, k_intra))
        send.append(nb.reshape(-1))
        if l >= 1 and k_cross > 0:
            nb = knn(pos, q, level_end[l - 1], k_cross)
            recv.append(np.repeat(q, k_cross))
            send.append(nb.reshape(-1))
    return np.concatenate(recv).astype(np.int64), np.concatenate(send).astype(np.int64)


class Graph:
    """Receiver-sorted CSR plus its sender-sorted transpose.

    row_ptr [n+1], col [E]      : in-edges of receiver r are col[row_ptr[r]:row_ptr[r+1]],
                                  ascending sender id.
    recv [E]                    : receiver of each CSR edge.
    csc_ptr [n+1], csc_perm [E] : out-edges of sender s are the CSR edges
                                  csc_perm[csc_ptr[s]:csc_ptr[s+1]], ascending receiver.
    """

    def __init__(self, n, recv, send):
        key = np.unique(recv.astype(np.int64) * n + send.astype(np.int64))
        self.n = int(n)
        self.recv = (key // n).astype(np.int32)
        self.col = (key % n).astype(np.int32)
        self.row_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.recv, minlength=n), out=self.row_ptr[1:])
        order = np.lexsort((self.recv, self.col))
        self.csc_perm = order.astype(np.int64)
        self.csc_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.col, minlength=n), out=self.csc_ptr[1:])

    @property
    def n_edges(self) -> int:
        return len(self.col)

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def build_graph(pos, level_end, k_intra, k_cross=0) -> Graph:
    """The multi-scale kNN graph: union of per-level and cross-level lists."""
    level_end = [int(x) for x in level_end]
    if sorted(level_end) != level_end or level_end[0] <= 0 or level_end[-1] != len(pos):
        raise ValueError("level_end must be increasing and end at the point count")
    recv, send = multiscale_edge_lists(pos, level_end, k_intra, k_cross)
    return Graph(len(pos), recv, send)
