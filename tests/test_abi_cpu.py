"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every declared symbol, the parameter layout agrees with the oracle's,
the host partitioner reproduces the oracle's partitions bit for bit, and bad
arguments are rejected before any device work."""
import numpy as np
import pytest

api = pytest.importorskip("paper_2411_17164_amd.api")
from paper_2411_17164_amd import _lib  # noqa: E402

from oracle import graph as og  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import partition as opart  # noqa: E402


def test_library_exports_every_header_symbol():
    names = _lib.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(_lib.lib, n)]
    assert missing == []
    assert b"gfx950" in _lib.lib.xmgn_version()


@pytest.mark.parametrize("H,L,nin,out", [(128, 2, 6, 4), (256, 15, 6, 4), (128, 3, 5, 7)])
def test_param_layout_matches_oracle(H, L, nin, out):
    m = api.Model(H, L, node_in=nin, out_dim=out)
    d = om.Desc(hidden=H, layers=L, node_in=nin, out_dim=out)
    lay = om.layout(d)
    mine = m.param_tensors()
    assert m.param_count() == om.n_params(d)
    assert len(mine) == len(lay)
    off = 0
    for (b, l, t, kind, shape, o), (_, okind, oshape) in zip(mine, lay):
        assert (kind, tuple(shape)) == (okind, tuple(oshape))
        assert o == off
        off += int(np.prod(shape))


def test_unsupported_hidden_and_bad_desc():
    with pytest.raises(api.XmgnError) as e:
        api.Model(96, 2).param_count()
    assert e.value.code == -5
    with pytest.raises(api.XmgnError):
        api.Model(128, 0).param_count()
    with pytest.raises(api.XmgnError):
        api.Model(128, 2, edge_in=3).param_count()
    # H = 512 runs in the BF16 form only; wide inputs come in multiples of 4
    with pytest.raises(api.XmgnError) as e:
        api.Model(512, 2, precision="fp32").param_count()
    assert e.value.code == -5
    assert api.Model(512, 2, precision="bf16", node_in=24).param_count() > 0
    with pytest.raises(api.XmgnError):
        api.Model(128, 2, node_in=10).param_count()
    with pytest.raises(api.XmgnError):
        api.Model(128, 2, node_in=36).param_count()


def _cloud(n, seed):
    g = np.random.default_rng(seed)
    return (g.standard_normal((n, 3)) * np.array([3.0, 1.0, 0.6])).astype(np.float32)


@pytest.mark.parametrize("halo", [1, 3])
def test_partition_matches_oracle_bitwise(halo):
    pos = _cloud(3000, 1)
    G = og.build_graph(pos, [300, 1000, 3000], 6, 3)
    g = api.Graph.from_csr(G.row_ptr, G.col)
    assert g.info() == (3000, G.n_edges)
    sizes = np.array([500, 800, 300, 700, 400, 300])
    ps = api.Partset.halo(g, pos, sizes, halo)
    parts, _ = opart.partition(G, pos, sizes, halo)
    assert ps.count() == (6, 3000)
    for p, P in enumerate(parts):
        x = ps.export(p)
        assert x["n_inner"] == P.n_inner
        assert (x["gid"] == P.gid).all()
        assert (x["hop"] == P.hop).all()
        assert (x["row_ptr"] == P.row_ptr).all()
        assert (x["col"] == P.col).all()


def test_explicit_in_cones_match_oracle():
    pos = _cloud(1500, 2)
    G = og.build_graph(pos, [200, 1500], 6, 3)
    g = api.Graph.from_csr(G.row_ptr, G.col)
    seeds = [[5], [17, 900, 1200], [1499]]
    ps = api.Partset.explicit(g, seeds, 4)
    for p, s in enumerate(seeds):
        c = opart.in_cone(G, s, 4)
        x = ps.export(p)
        assert (x["gid"] == c.gid).all() and (x["col"] == c.col).all() and (x["row_ptr"] == c.row_ptr).all()


def test_bad_graphs_and_partitions_are_rejected():
    with pytest.raises(api.XmgnError):  # self loop
        api.Graph.from_csr([0, 1, 1], [0])
    with pytest.raises(api.XmgnError):  # unsorted segment
        api.Graph.from_csr([0, 2, 2, 2], [2, 1])
    with pytest.raises(api.XmgnError):  # sender out of range
        api.Graph.from_csr([0, 1, 1], [5])
    pos = _cloud(100, 3)
    G = og.build_graph(pos, [100], 4, 0)
    g = api.Graph.from_csr(G.row_ptr, G.col)
    with pytest.raises(api.XmgnError):
        api.Partset.halo(g, pos, [50, 49], 2)  # sizes do not sum
    with pytest.raises(api.XmgnError):
        api.Partset.halo(g, pos, [50, 50], 0)  # halo must be >= 1
    bad = pos.copy()
    bad[3, 1] = np.nan
    with pytest.raises(api.XmgnError):
        api.Partset.halo(g, bad, [50, 50], 2)
    with pytest.raises(api.XmgnError):
        api.Partset.explicit(g, [[1, 1]], 2)


def test_context_calls_reject_null_handles():
    lib = _lib.lib
    b = _lib.C.c_int64()
    assert lib.xmgn_ctx_set_offload(None, 1) == -1
    assert lib.xmgn_ctx_host_memory(None, _lib.C.byref(b)) == -1
    assert lib.xmgn_ctx_memory(None, _lib.C.byref(b)) == -1
