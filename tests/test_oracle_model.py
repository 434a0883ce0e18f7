"""Pins of the oracle's network, loss and hand-written adjoint.

The paper gives Eq. (1)-(4) and no numeric example.  The oracle is pinned by
closed forms where a layer collapses to textbook operations, by symmetry
(node-permutation equivariance), by LayerNorm's defining statistics, and by
central finite differences of the float64 loss for the adjoint.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import graph as og
from oracle import model as om
from synth import init_params


def small_case(n=120, levels=(30, 120), k=4, kc=2, H=8, L=2, act="silu", agg="message", seed=0):
    g = np.random.default_rng(seed)
    pos = g.standard_normal((n, 3))
    pos = (pos / np.linalg.norm(pos, axis=1, keepdims=True)).astype(np.float32)
    G = og.build_graph(pos, list(levels), k, kc)
    d = om.Desc(hidden=H, layers=L, activation=act, aggregate=agg)
    blob = init_params(om.param_entries(d), 1000 + seed).astype(np.float64)
    node_in = g.standard_normal((n, 6)).astype(np.float32)
    en = np.array([[0, 0, 0, 0.3], [0.3, 0.3, 0.3, 0.2]], dtype=np.float32)
    tgt = g.standard_normal((n, 4)).astype(np.float32)
    return d, blob, G, node_in, pos, en, tgt


def test_param_count_closed_form():
    for H, L in [(8, 2), (128, 15), (256, 15)]:
        d = om.Desc(hidden=H, layers=L)
        per_layer = (3 * H * H + H + H * H + H + 2 * H) + (2 * H * H + H + H * H + H + 2 * H)
        enc = 2 * (H * H + H) + 2 * H
        n = (6 * H + H + enc) + (4 * H + H + enc) + L * per_layer + (2 * (H * H + H) + 4 * H + 4)
        assert om.n_params(d) == n
        assert per_layer == 7 * H * H + 8 * H


def test_layernorm_statistics():
    g = np.random.default_rng(0)
    u = g.standard_normal((50, 16)) * 3 + 1
    y, xhat, inv = om.layernorm(u, np.ones(16), np.zeros(16), 1e-5)
    assert np.allclose(y.mean(axis=1), 0, atol=1e-12)
    assert np.allclose((y * y).mean(axis=1), u.var(axis=1) / (u.var(axis=1) + 1e-5), atol=1e-12)


def test_zero_edge_mlp_gives_degree_times_beta():
    """W2e = 0, b2e = 0: u is constant, LN returns beta_e, so every message
    is beta_e and m_r = deg(r) * beta_e."""
    d, blob, G, node_in, pos, en, _ = small_case()
    P = om.unpack(d, blob)
    pe = [x.copy() for x in P["edge0"]]
    pe[2][:] = 0
    pe[3][:] = 0
    h = np.random.default_rng(1).standard_normal((G.n, d.hidden))
    e = np.random.default_rng(2).standard_normal((G.n_edges, d.hidden))
    hn, en_, m = om.processor_layer_fwd(d, G, pe, P["node0"], h, e)
    assert np.allclose(m, G.degree()[:, None] * pe[5][None, :], atol=1e-12)
    assert np.allclose(en_ - e, pe[5][None, :], atol=1e-12)


def test_aggregation_is_the_sparse_adjacency_product():
    """W1e = [0 | I | 0], b1e = 0, W2e = I, b2e = 0, ReLU and positive h:
    the message of edge s -> r is LN(h_s), so m = A LN(h) with A[r, s] = 1
    for each edge (a scipy.sparse product).  A swapped gather (h_r for h_s)
    or a transposed adjacency fails this."""
    d, blob, G, _, _, _, _ = small_case(act="relu")
    H = d.hidden
    P = om.unpack(d, blob)
    pe = [x.copy() for x in P["edge0"]]
    pe[0][:] = 0
    pe[0][:, H:2 * H] = np.eye(H)
    pe[1][:] = 0
    pe[2][:] = np.eye(H)
    pe[3][:] = 0
    h = np.random.default_rng(3).uniform(0.1, 2.0, (G.n, H))
    e = np.random.default_rng(4).standard_normal((G.n_edges, H))
    _, _, m = om.processor_layer_fwd(d, G, pe, P["node0"], h, e)
    mu = h.mean(1, keepdims=True)
    lnh = pe[4] * (h - mu) / np.sqrt(h.var(1, keepdims=True) + d.ln_eps) + pe[5]
    A = sp.csr_matrix((np.ones(G.n_edges), G.col, G.row_ptr), shape=(G.n, G.n))
    assert np.allclose(m, A @ lnh, atol=1e-12)


def test_zero_node_mlp_adds_beta():
    d, blob, G, _, _, _, _ = small_case()
    P = om.unpack(d, blob)
    pn = [x.copy() for x in P["node0"]]
    pn[2][:] = 0
    pn[3][:] = 0
    h = np.random.default_rng(5).standard_normal((G.n, d.hidden))
    e = np.random.default_rng(6).standard_normal((G.n_edges, d.hidden))
    hn, _, _ = om.processor_layer_fwd(d, G, P["edge0"], pn, h, e)
    assert np.allclose(hn - h, pn[5][None, :], atol=1e-12)


def test_node_permutation_equivariance():
    d, blob, G, node_in, pos, en, _ = small_case(act="relu")
    y = om.forward(d, blob, G, node_in, pos, en)
    perm = np.random.default_rng(7).permutation(G.n)
    inv = np.argsort(perm)
    # relabel: new node i is old node perm[i]
    G2 = og.Graph(G.n, inv[G.recv], inv[G.col])
    y2 = om.forward(d, blob, G2, node_in[perm], pos[perm], en)
    assert np.allclose(y2, y[perm], rtol=1e-12, atol=1e-12)


def _loss(d, blob, G, node_in, pos, en, tgt):
    y = om.forward(d, blob, G, node_in, pos, en)
    return om.loss_and_grad(y, tgt, G.n, G.n)[0]


@pytest.mark.parametrize("agg", ["message", "edge"])
def test_adjoint_matches_central_differences(agg):
    d, blob, G, node_in, pos, en, tgt = small_case(agg=agg, L=2)
    loss, y, grad = om.step_full(d, blob, G, node_in, pos, en, tgt)
    g = np.random.default_rng(8)
    eps = 1e-6
    # random directions
    for _ in range(3):
        v = g.standard_normal(len(blob))
        fd = (_loss(d, blob + eps * v, G, node_in, pos, en, tgt)
              - _loss(d, blob - eps * v, G, node_in, pos, en, tgt)) / (2 * eps)
        assert abs(fd - grad @ v) <= 1e-7 * max(1.0, abs(fd))
    # single coordinates spread over every block of the layout
    idx = np.unique(np.concatenate([g.choice(len(blob), 150, replace=False),
                                    np.cumsum([0] + [int(np.prod(s)) for _, _, s in om.layout(d)])[:-1]]))
    errs = []
    for i in idx:
        bp = blob.copy()
        bp[i] += eps
        bm = blob.copy()
        bm[i] -= eps
        fd = (_loss(d, bp, G, node_in, pos, en, tgt) - _loss(d, bm, G, node_in, pos, en, tgt)) / (2 * eps)
        errs.append(abs(fd - grad[i]) / max(1e-3, abs(fd)))
    assert max(errs) < 1e-5


def test_loss_excludes_halo_rows():
    y = np.arange(12, dtype=np.float64).reshape(3, 4)
    t = np.zeros((3, 4))
    loss, dy = om.loss_and_grad(y, t, 2, 10)
    assert loss == pytest.approx((y[:2] ** 2).sum() / 40)
    assert (dy[2] == 0).all() and np.allclose(dy[:2], 2 * y[:2] / 40)


def test_bf16_round_against_torch_and_hand_values():
    """bf16_round agrees with torch's float32 -> bfloat16 conversion (round
    to nearest, ties to even) on random values, exact ties and values next
    to ties; and with hand-worked cases near 1."""
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(3)
    x = (g.standard_normal(20000) * np.exp(g.uniform(-30, 30, 20000))).astype(np.float32)
    bits = g.integers(0, 1 << 16, 5000, dtype=np.uint32) << 16
    ties = (bits | 0x8000).view(np.float32)           # exactly halfway between two bfloat16 values
    near = np.concatenate([(bits | 0x7FFF).view(np.float32), (bits | 0x8001).view(np.float32)])
    for v in (x, ties, near):
        v = v[np.isfinite(v)]
        ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert (om.bf16_round(v) == ref).all()
    one = 1.0
    assert om.bf16_round(np.float32(one + 2.0**-8)) == 1.0                 # tie, even neighbour is 1
    assert om.bf16_round(np.float32(one + 3 * 2.0**-8)) == one + 2.0**-6   # tie, even neighbour above
    assert om.bf16_round(np.float32(one + 2.0**-8 + 2.0**-20)) == one + 2.0**-7
    assert om.bf16_round(np.float32(-3.0)) == -3.0
    assert om.bf16_round(np.float32(0.0)) == 0.0


def test_amp_cast_rounds_only_hidden_products():
    d = om.Desc(hidden=16, layers=2)
    blob = init_params(om.param_entries(d), 7).astype(np.float32)
    c = om.amp_cast(d, blob)
    assert (om.amp_cast(d, c) == c).all()                                  # idempotent
    off = 0
    for b, kind, shape in om.layout(d):
        n = int(np.prod(shape))
        a, r = blob[off:off + n].astype(np.float64), c[off:off + n]
        hidden = kind == "weight" and min(shape) >= d.hidden
        if hidden:
            assert (np.abs(r - a) <= 2.0**-8 * np.abs(a)).all()        # unit roundoff of an 8-bit significand
            assert (r != a).any()
        else:
            assert (r == a).all(), (b, kind, shape)
        off += n
    names = [(b, s) for b, k, s in om.layout(d) if k == "weight" and min(s) < d.hidden]
    assert names == [("enc_node", (16, 6)), ("enc_edge", (16, 4)), ("dec", (4, 16))]
