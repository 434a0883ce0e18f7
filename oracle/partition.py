"""Graph partitions with an L-hop halo (Sec. III.A).

Reading of the paper taken here:
* The partitioner is recursive coordinate bisection (RCB) with given integer
  part sizes, standing in for METIS.  RCB(nodes, parts [a, b)): one part ->
  assign; otherwise split the parts at m = a + (b - a) // 2, cut along the
  axis of largest bounding-box extent (ties: x before y before z), order
  the nodes by (coordinate on that axis, node id) and give the first
  sum(size[a:m]) nodes to the left half.
* The halo is as deep as the number of message-passing layers.  It is found
  by breadth-first search over in-edges (sender of each in-edge), since an
  output after L layers depends only on its L-hop in-neighbourhood (Eq. 4).
  Inner nodes have hop 0, halo nodes hop 1..L.
* Local node order: inner nodes by ascending id, then halo nodes by
  ascending (hop, id).  Local edges: all in-edges of local nodes whose hop is
  below L, segments kept in ascending global sender id.  Nodes at hop L keep
  no in-edges; they only send.
"""
from __future__ import annotations

import numpy as np

from .graph import Graph


def rcb(pos: np.ndarray, sizes) -> np.ndarray:
    """Part id (int32 [n]) of every node."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n = len(pos)
    if sizes.sum() != n or (sizes <= 0).any():
        raise ValueError("part sizes must be positive and sum to the node count")
    pos64 = pos.astype(np.float64)
    part = np.empty(n, dtype=np.int32)

    def split(ids, a, b):
        if b - a == 1:
            part[ids] = a
            return
        m = a + (b - a) // 2
        ext = pos64[ids].max(axis=0) - pos64[ids].min(axis=0)
        axis = int(np.argmax(ext))
        order = np.lexsort((ids, pos64[ids, axis]))
        n_left = int(sizes[a:m].sum())
        split(ids[order[:n_left]], a, m)
        split(ids[order[n_left:]], m, b)

    split(np.arange(n, dtype=np.int64), 0, len(sizes))
    return part


def _ranges(lo: np.ndarray, cnt: np.ndarray) -> np.ndarray:
    """Concatenation of the index ranges [lo[i], lo[i] + cnt[i])."""
    if len(cnt) == 0:
        return np.zeros(0, dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    return np.repeat(lo - start, cnt) + np.arange(int(cnt.sum()))


def halo_hops(g: Graph, inner: np.ndarray, depth: int) -> np.ndarray:
    """hop[i] for every node: 0 inner, 1..depth halo, -1 outside."""
    hop = np.full(g.n, -1, dtype=np.int64)
    hop[inner] = 0
    frontier = np.asarray(inner, dtype=np.int64)
    for h in range(1, depth + 1):
        if len(frontier) == 0:
            break
        lo, hi = g.row_ptr[frontier], g.row_ptr[frontier + 1]
        idx = _ranges(lo, hi - lo)
        senders = np.unique(g.col[idx])
        new = senders[hop[senders] < 0]
        hop[new] = h
        frontier = new
    return hop


class Part:
    """One partition: local graph over inner + halo nodes."""

    def __init__(self, g: Graph, inner: np.ndarray, depth: int):
        inner = np.sort(np.asarray(inner, dtype=np.int64))
        hop = halo_hops(g, inner, depth)
        halo = np.flatnonzero(hop > 0)
        halo = halo[np.lexsort((halo, hop[halo]))]
        self.gid = np.concatenate([inner, halo])           # local -> global
        self.n_inner = len(inner)
        self.hop = hop[self.gid]
        self.depth = depth
        loc = np.full(g.n, -1, dtype=np.int64)
        loc[self.gid] = np.arange(len(self.gid))
        deg = np.where(self.hop < depth, np.diff(g.row_ptr)[self.gid], 0)
        self.row_ptr = np.zeros(len(self.gid) + 1, dtype=np.int64)
        np.cumsum(deg, out=self.row_ptr[1:])
        src = _ranges(g.row_ptr[self.gid], deg)
        self.edge_gid = src                                   # global CSR edge ids
        self.col = loc[g.col[src]]
        assert (self.col >= 0).all(), "halo is not closed under in-edges"
        self.recv = np.repeat(np.arange(len(self.gid)), deg)
        self.graph = Graph.__new__(Graph)
        lg = self.graph
        lg.n = len(self.gid)
        lg.recv = self.recv.astype(np.int32)
        lg.col = self.col.astype(np.int32)
        lg.row_ptr = self.row_ptr
        order = np.lexsort((lg.recv, lg.col))
        lg.csc_perm = order.astype(np.int64)
        lg.csc_ptr = np.zeros(lg.n + 1, dtype=np.int64)
        np.cumsum(np.bincount(lg.col, minlength=lg.n), out=lg.csc_ptr[1:])

    @property
    def n_halo(self) -> int:
        return len(self.gid) - self.n_inner


def partition(g: Graph, pos, sizes, depth: int):
    """RCB into len(sizes) parts, each extended by a depth-hop halo."""
    part = rcb(pos, sizes)
    return [Part(g, np.flatnonzero(part == p), depth) for p in range(len(sizes))], part


def in_cone(g: Graph, seeds, depth: int) -> Part:
    """The depth-hop in-cone of a set of seed nodes, as a partition whose
    inner nodes are the seeds (used to evaluate single outputs)."""
    return Part(g, np.asarray(seeds), depth)
