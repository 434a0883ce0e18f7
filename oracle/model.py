"""Encoder / processor / decoder of MeshGraphNet over a (partitioned) graph,
its masked MSE loss and the hand-written adjoint, all in float64.

Processor layer l (Eq. 1-4, with the MeshGraphNet edge and node MLPs):
  for every edge k = (s -> r):
     x_k  = [h_r ; h_s ; e_k]                          (3H, order of Eq. 1)
     a_k  = W1e x_k + b1e,  z_k = act(a_k)
     u_k  = W2e z_k + b2e
     v_k  = LN_e(u_k)                                  message of Eq. (1)
     e'_k = e_k + v_k                                  edge residual
  m_r  = sum over in-edges of r of v_k                 Eq. (2), sender order
         (aggregate="edge": sum of e'_k instead)
  y_r  = [h_r ; m_r],  a = W1n y + b1n,  z = act(a),  u = W2n z + b2n
  h'_r = h_r + LN_n(u)                                 Eq. (3) with residual

LN(u) = gamma * (u - mean) / sqrt(var + eps) + beta, biased variance.

Encoders: in -> H -> H -> H MLP followed by LN, for nodes (input [pos,
normal], z-scored) and for edges (input [x_s - x_r, |x_s - x_r|],
normalised with a caller-given affine).  Edge features follow Sec. II.E.
Decoder: H -> H -> H -> out, no LN.
Loss (Sec. II.E, III.D): mean squared error over inner nodes only, with the
global normaliser N_total * out_dim so that the partition losses add up to
the full-graph loss; halo rows are excluded.

BF16 form (training in bfloat16 with automatic mixed precision, Sec. V.D):
the products over the hidden width take bfloat16 copies of their weights,
and the gradient of the cast is passed through unchanged.  amp_cast gives
the parameters such a form multiplies with; the oracle run at them is the
exact counterpart of the BF16 form's arithmetic, while the run at the FP32
master weights is the model itself.

Parameter blob (float32 master, flat, this order; W stored [out][in]):
  node encoder  W1[H][6]  b1[H]  W2[H][H]  b2[H]  W3[H][H]  b3[H]  g[H]  be[H]
  edge encoder  W1[H][4]  b1[H]  W2[H][H]  b2[H]  W3[H][H]  b3[H]  g[H]  be[H]
  layer l = 0..L-1:
    edge  W1[H][3H] b1[H] W2[H][H] b2[H] g[H] be[H]
    node  W1[H][2H] b1[H] W2[H][H] b2[H] g[H] be[H]
  decoder W1[H][H] b1[H] W2[H][H] b2[H] W3[out][H] b3[out]
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .graph import Graph


@dataclass(frozen=True)
class Desc:
    hidden: int
    layers: int
    node_in: int = 6
    edge_in: int = 4
    out_dim: int = 4
    activation: str = "relu"      # "relu" | "silu"
    aggregate: str = "message"    # "message" (sum of v) | "edge" (sum of e')
    ln_eps: float = 1e-5


def _mlp_entries(dims, ln):
    out = []
    for i in range(len(dims) - 1):
        out.append(("weight", (dims[i + 1], dims[i])))
        out.append(("bias", (dims[i + 1],)))
    if ln:
        out.append(("gamma", (dims[-1],)))
        out.append(("beta", (dims[-1],)))
    return out


def layout(d: Desc):
    """[(block, kind, shape)] in blob order."""
    H = d.hidden
    blocks = [("enc_node", _mlp_entries([d.node_in, H, H, H], True)),
              ("enc_edge", _mlp_entries([d.edge_in, H, H, H], True))]
    for l in range(d.layers):
        blocks.append((f"edge{l}", _mlp_entries([3 * H, H, H], True)))
        blocks.append((f"node{l}", _mlp_entries([2 * H, H, H], True)))
    blocks.append(("dec", _mlp_entries([H, H, H, d.out_dim], False)))
    return [(b, k, s) for b, ents in blocks for (k, s) in ents]


def param_entries(d: Desc):
    """(kind, shape) list for the seeded initialiser."""
    return [(k, s) for (_, k, s) in layout(d)]


def n_params(d: Desc) -> int:
    return int(sum(np.prod(s) for (_, _, s) in layout(d)))


def unpack(d: Desc, blob: np.ndarray):
    """dict block -> list of float64 arrays (W1, b1, W2, b2, ..., [g, be])."""
    out = {}
    off = 0
    for b, _, s in layout(d):
        cnt = int(np.prod(s))
        out.setdefault(b, []).append(np.asarray(blob[off:off + cnt], dtype=np.float64).reshape(s))
        off += cnt
    assert off == len(blob), "blob size does not match the layout"
    return out


def pack(d: Desc, grads: dict) -> np.ndarray:
    parts = []
    names = []
    for b, _, _ in layout(d):
        if b not in names:
            names.append(b)
    for b in names:
        parts.extend(x.reshape(-1) for x in grads[b])
    return np.concatenate(parts)


def bf16_round(x) -> np.ndarray:
    """Each value of x, taken as float32, rounded to the nearest bfloat16
    (sign, 8 exponent bits and 7 stored significand bits: the upper half of
    the float32 bit pattern), ties to the even significand; as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    if not np.isfinite(f).all():
        raise ValueError("bf16_round takes finite values")
    u = f.view(np.uint32).astype(np.uint64)
    odd = (u >> 16) & 1
    r = ((u + 0x7FFF + odd) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def amp_cast(d: Desc, blob) -> np.ndarray:
    """The parameter blob with every hidden-to-hidden weight (both dimensions
    at least H: the encoders' second and third layers, the processor MLPs and
    the decoder's first two layers) rounded to bfloat16.  The encoders' input
    layers (6 and 4 inputs), the decoder's output layer, the biases and the
    LayerNorm affines stay float32."""
    out = np.asarray(blob, dtype=np.float64).copy()
    off = 0
    for _, kind, shape in layout(d):
        cnt = int(np.prod(shape))
        if kind == "weight" and min(shape) >= d.hidden:
            out[off:off + cnt] = bf16_round(out[off:off + cnt])
        off += cnt
    return out


# --- elementwise pieces -----------------------------------------------------

def act(d: Desc, a):
    if d.activation == "relu":
        return np.maximum(a, 0.0)
    return a / (1.0 + np.exp(-a))


def act_grad(d: Desc, a):
    if d.activation == "relu":
        return (a > 0).astype(np.float64)
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def layernorm(u, gamma, beta, eps):
    """Returns (y, xhat, inv_std) with biased variance per row."""
    mu = u.mean(axis=1, keepdims=True)
    var = ((u - mu) ** 2).mean(axis=1, keepdims=True)
    inv = 1.0 / np.sqrt(var + eps)
    xhat = (u - mu) * inv
    return gamma * xhat + beta, xhat, inv


def layernorm_bwd(dy, xhat, inv, gamma):
    """(du, dgamma, dbeta) of y = gamma * xhat + beta."""
    g = dy * gamma
    du = (g - g.mean(axis=1, keepdims=True) - xhat * (g * xhat).mean(axis=1, keepdims=True)) * inv
    return du, (dy * xhat).sum(axis=0), dy.sum(axis=0)


def segment_sum(g: Graph, rows: np.ndarray) -> np.ndarray:
    """out[r] = sum of rows[k] over the in-edges k of r, added one CSR slot at
    a time in ascending sender order."""
    deg = np.diff(g.row_ptr)
    out = np.zeros((g.n, rows.shape[1]))
    if g.n == 0 or len(rows) == 0:
        return out
    for t in range(int(deg.max())):
        r = np.flatnonzero(deg > t)
        out[r] += rows[g.row_ptr[r] + t]
    return out


def sender_sum(g: Graph, rows: np.ndarray) -> np.ndarray:
    """out[s] = sum of rows[k] over the out-edges k of s."""
    out = np.zeros((g.n, rows.shape[1]))
    np.add.at(out, g.col, rows)
    return out


# --- MLP with cached intermediates -------------------------------------------

def mlp_fwd(d: Desc, ps, x, ln: bool):
    """Dense MLP: hidden layers use act, the last layer is linear, then LN if
    ln.  ps = [W1, b1, W2, b2, ..., (g, be)].  Returns (y, cache)."""
    nlin = (len(ps) - (2 if ln else 0)) // 2
    cache = {"x": [x], "a": []}
    z = x
    for i in range(nlin):
        a = z @ ps[2 * i].T + ps[2 * i + 1]
        if i < nlin - 1:
            cache["a"].append(a)
            z = act(d, a)
            cache["x"].append(z)
        else:
            z = a
    if ln:
        y, xhat, inv = layernorm(z, ps[-2], ps[-1], d.ln_eps)
        cache["ln"] = (xhat, inv)
        return y, cache
    return z, cache


def mlp_bwd(d: Desc, ps, cache, dy, ln: bool):
    """Returns (dx, [grads in the order of ps])."""
    nlin = (len(ps) - (2 if ln else 0)) // 2
    grads = [None] * len(ps)
    g = dy
    if ln:
        xhat, inv = cache["ln"]
        g, grads[-2], grads[-1] = layernorm_bwd(dy, xhat, inv, ps[-2])
    for i in reversed(range(nlin)):
        xin = cache["x"][i]
        grads[2 * i] = g.T @ xin
        grads[2 * i + 1] = g.sum(axis=0)
        g = g @ ps[2 * i]
        if i > 0:
            g = g * act_grad(d, cache["a"][i - 1])
    return g, grads


# --- the model ---------------------------------------------------------------

def edge_features(g: Graph, pos, edge_norm):
    """[x_s - x_r, |x_s - x_r|] per CSR edge, then (f - mean) / std."""
    p = pos.astype(np.float64)
    dx = p[g.col] - p[g.recv]
    f = np.concatenate([dx, np.sqrt((dx * dx).sum(axis=1, keepdims=True))], axis=1)
    en = np.asarray(edge_norm, dtype=np.float64)
    return (f - en[0]) / en[1]


def processor_layer_fwd(d: Desc, g: Graph, pe, pn, h, e):
    H = d.hidden
    x = np.concatenate([h[g.recv], h[g.col], e], axis=1)
    v, ce = mlp_fwd(d, pe, x, True)
    e_new = e + v
    m = segment_sum(g, e_new if d.aggregate == "edge" else v)
    y = np.concatenate([h, m], axis=1)
    hn, cn = mlp_fwd(d, pn, y, True)
    assert x.shape[1] == 3 * H
    return h + hn, e_new, m


def forward(d: Desc, blob, g: Graph, node_in, pos, edge_norm, keep=False):
    """Outputs y [n][out_dim] for every node of graph g (a full graph or a
    partition's local graph with its node_in / pos rows).  With keep=True also
    returns the per-layer checkpoints (h^l, e^l) for the backward pass."""
    P = unpack(d, blob)
    h, _ = mlp_fwd(d, P["enc_node"], np.asarray(node_in, np.float64), True)
    e, _ = mlp_fwd(d, P["enc_edge"], edge_features(g, pos, edge_norm), True)
    tape = []
    for l in range(d.layers):
        tape.append((h, e))
        h, e, _ = processor_layer_fwd(d, g, P[f"edge{l}"], P[f"node{l}"], h, e)
    y, _ = mlp_fwd(d, P["dec"], h, False)
    if keep:
        return y, {"tape": tape, "hL": h, "P": P}
    return y


def forward_cone(d: Desc, blob, part, node_in, pos, edge_norm):
    """Outputs of a cone's inner nodes (its seeds), evaluating each layer only
    on the rows that can still reach them.

    `part` is an L-hop in-cone (partition.in_cone): local nodes ordered by
    hop, every node with hop < L keeping all its in-edges.  An output of
    layer l at a node with hop j feeds the seeds only if j <= L - 1 - l
    (Eq. 4: one hop per layer), so layer l updates the nodes with hop
    <= L - 1 - l from the edges into them: a prefix of the local nodes and
    of the local CSR edges.  Every row it computes is the same per-row
    arithmetic as forward() on the whole cone; the rows it skips never reach
    a seed."""
    P = unpack(d, blob)
    g = part.graph
    hop = np.asarray(part.hop)
    L = d.layers
    assert part.depth == L, "the cone must be L hops deep"
    n_upto = [int(np.searchsorted(hop, j, side="right")) for j in range(L + 1)]  # nodes with hop <= j
    h, _ = mlp_fwd(d, P["enc_node"], np.asarray(node_in, np.float64), True)
    e, _ = mlp_fwd(d, P["enc_edge"], edge_features(g, pos, edge_norm), True)
    for l in range(L):
        nr = n_upto[L - 1 - l]            # receivers updated by this layer
        ns = n_upto[L - l]                # rows of h it reads (their senders)
        ne = int(g.row_ptr[nr])           # their in-edges: a CSR prefix
        sub = Graph.__new__(Graph)
        sub.n = ns
        sub.recv = g.recv[:ne]
        sub.col = g.col[:ne]
        sub.row_ptr = np.concatenate([g.row_ptr[: nr + 1], np.full(ns - nr, ne, dtype=g.row_ptr.dtype)])
        h, e, _ = processor_layer_fwd(d, sub, P[f"edge{l}"], P[f"node{l}"], h[:ns], e[:ne])
        h = h[:nr]                        # rows past nr had no in-edges here and reach no seed
    y, _ = mlp_fwd(d, P["dec"], h[: part.n_inner], False)
    return y


def loss_and_grad(y, targets, n_inner, n_total):
    """Masked MSE: rows [0, n_inner) are inner nodes, the rest is halo.
    Returns (loss, d loss / d y) with halo rows zero."""
    C = y.shape[1]
    diff = y[:n_inner] - np.asarray(targets, np.float64)[:n_inner]
    scale = 1.0 / (n_total * C)
    dy = np.zeros_like(y)
    dy[:n_inner] = 2.0 * scale * diff
    return float(scale * (diff * diff).sum()), dy


def backward(d: Desc, g: Graph, node_in, pos, edge_norm, saved, dy):
    """Gradient of sum(dy * y) with respect to the parameter blob (float64),
    recomputing each layer from its checkpoint (h^l, e^l)."""
    P = saved["P"]
    G = {}
    H = d.hidden
    _, cdec = mlp_fwd(d, P["dec"], saved["hL"], False)
    dh, G["dec"] = mlp_bwd(d, P["dec"], cdec, dy, False)
    de = np.zeros((g.n_edges, H))
    for l in reversed(range(d.layers)):
        h, e = saved["tape"][l]
        pe, pn = P[f"edge{l}"], P[f"node{l}"]
        x = np.concatenate([h[g.recv], h[g.col], e], axis=1)
        v, ce = mlp_fwd(d, pe, x, True)
        e_new = e + v
        m = segment_sum(g, e_new if d.aggregate == "edge" else v)
        y = np.concatenate([h, m], axis=1)
        _, cn = mlp_fwd(d, pn, y, True)
        # node update h' = h + LN_n(...)
        dy_n, G[f"node{l}"] = mlp_bwd(d, pn, cn, dh, True)
        dh_new = dh + dy_n[:, :H]
        dm = dy_n[:, H:]
        # edge update: v feeds e' (residual) and, through m, the receiver
        dm_k = dm[g.recv]
        if d.aggregate == "edge":
            de_total = de + dm_k          # gradient reaching e'_k
            dv = de_total
            de_res = de_total
        else:
            dv = de + dm_k
            de_res = de
        dx, G[f"edge{l}"] = mlp_bwd(d, pe, ce, dv, True)
        dh_new += segment_sum(g, dx[:, :H])
        dh_new += sender_sum(g, dx[:, H:2 * H])
        de = de_res + dx[:, 2 * H:]
        dh = dh_new
    _, cen = mlp_fwd(d, P["enc_node"], np.asarray(node_in, np.float64), True)
    _, G["enc_node"] = mlp_bwd(d, P["enc_node"], cen, dh, True)
    _, cee = mlp_fwd(d, P["enc_edge"], edge_features(g, pos, edge_norm), True)
    _, G["enc_edge"] = mlp_bwd(d, P["enc_edge"], cee, de, True)
    return pack(d, G)


# --- whole-graph and partitioned training steps -------------------------------

def step_full(d: Desc, blob, g: Graph, node_in, pos, edge_norm, targets):
    """(loss, y, grad) on the whole graph."""
    y, saved = forward(d, blob, g, node_in, pos, edge_norm, keep=True)
    loss, dy = loss_and_grad(y, targets, g.n, g.n)
    return loss, y, backward(d, g, node_in, pos, edge_norm, saved, dy)


def step_part(d: Desc, blob, part, node_in, pos, edge_norm, targets, n_total):
    """(loss, y_inner, grad) of one partition: forward on its local graph,
    loss over its inner nodes with the global normaliser, backward."""
    gid = part.gid
    y, saved = forward(d, blob, part.graph, node_in[gid], pos[gid], edge_norm, keep=True)
    loss, dy = loss_and_grad(y, targets[gid], part.n_inner, n_total)
    grad = backward(d, part.graph, node_in[gid], pos[gid], edge_norm, saved, dy)
    return loss, y[: part.n_inner], grad


def step_partitioned(d: Desc, blob, parts, node_in, pos, edge_norm, targets):
    """Gradient aggregation over partitions: losses and gradients summed in
    ascending partition order; outputs re-assembled from inner rows."""
    n_total = sum(p.n_inner for p in parts)
    y = np.zeros((n_total, d.out_dim))
    loss = 0.0
    grad = np.zeros(n_params(d))
    for p in parts:
        lp, yp, gp = step_part(d, blob, p, node_in, pos, edge_norm, targets, n_total)
        loss += lp
        grad += gp
        y[p.gid[: p.n_inner]] = yp
    return loss, y, grad
