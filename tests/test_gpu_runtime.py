"""GPU: the runtime around the kernels -- the tile autotuner and its cache
file, the tape policy, and the stream contract (a batch plan rebuilt while a
previous batch's kernels may still be running on a non-default stream)."""
import numpy as np
import pytest

from cases import Case, check_step, log, oracle_refs, per_tensor_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_17164_amd import api as a
    return a


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


class Step:
    """Device inputs of one case and a forward + MSE + backward through the C ABI."""

    def __init__(self, api, case):
        self.api, self.case = api, case
        self.model = case.model(api)
        self.p = dev(case.params)
        self.node_in, self.pos, self.tgt = dev(case.inp.node_in), dev(case.inp.pos), dev(case.inp.targets)

    def run(self, ctx, ps, part_ids):
        c = self.case
        out = torch.zeros(c.N, 4, device="cuda")
        ctx.forward(self.model, self.p, ps, part_ids, self.node_in, self.pos, c.inp.edge_norm, out, keep_tape=True)
        d_out = torch.zeros_like(out)
        loss = torch.zeros(1, device="cuda")
        ctx.mse_grad(out, self.tgt, c.N, d_out, loss)
        d_params = torch.full_like(self.p, float("nan"))
        ctx.backward(self.model, self.p, d_out, d_params)
        return out, loss, d_params


def test_autotune_and_cache(api, tmp_path):
    """The tuner picks one of its candidate configurations, leaves it set on
    the context, writes one cache line, and a second call reads the line
    back without timing anything; the tuned step still meets the bar."""
    case = Case(3, levels=(500, 2000, 6000), layers=2, precision="bf16", activation="silu")
    ctx = api.Context(0)
    g = ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    ps = api.Partset.halo(g, case.inp.pos, None, case.L)
    st = Step(api, case)
    out = torch.zeros(case.N, 4, device="cuda")
    d_out = torch.full_like(out, 1e-3)
    d_params = torch.zeros_like(st.p)
    cache = str(tmp_path / "tiles.txt")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    er, nr, gr, wv, ms = ctx.autotune(st.model, st.p, ps, [0], st.node_in, st.pos, case.inp.edge_norm, out, d_out,
                                      d_params, cache)
    log(f"autotune: edge_rows {er} node_rows {nr} grid {gr} waves {wv} ({ms:.3f} ms)")
    assert er in (32, 64) and nr in (32, 64) and wv in (4, 8) and ms > 0
    assert gr in {((cus * w + 7) // 8) * 8 for w in (4, 8)}
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1
    key, *vals = lines[0].split()
    assert [int(v) for v in vals[:4]] == [er, nr, gr, wv]
    br, bw = ctx.get_bwd_tiles()
    assert [int(v) for v in vals[4:6]] == [br, bw] and br in (0, 32, 64) and bw in (0, 4, 8)
    assert ":H128:L2:p1:a1:g0:" in key
    # the cached configuration comes back as is
    ctx2 = api.Context(0)
    assert ctx2.autotune(st.model, st.p, ps, [0], st.node_in, st.pos, case.inp.edge_norm, out, d_out, d_params,
                         cache) == (er, nr, gr, wv, pytest.approx(ms, rel=1e-4))
    assert len(open(cache).read().strip().splitlines()) == 1
    # the tuned context runs the step at the bar
    o, l, dp = st.run(ctx2, ps, [0])
    torch.cuda.synchronize()
    log("  " + check_step(case, o.cpu().numpy(), float(l.item()), dp.cpu().numpy(), oracle_refs(case)))


@pytest.mark.parametrize("precision,act", [("bf16", "relu"), ("bf16", "silu"), ("fp32", "relu"), ("fp32", "silu")])
def test_tape_policy(api, precision, act):
    """Keeping the edge MLPs' hidden activations or recomputing them: the
    forward is bitwise the same, the gradients agree to BF16 rounding, the
    recompute tape is smaller by the z (and a) tapes, and both meet the bar;
    the offloaded tape (which always recomputes) equals the recomputing
    resident tape bit for bit."""
    case = Case(3, levels=(500, 2000, 6000), layers=3, precision=precision, activation=act)
    keep, rec, off = api.Context(0), api.Context(0), api.Context(0)
    assert keep.get_tape() is True
    rec.set_tape(False)
    off.set_tape(False)
    off.set_offload(True)
    assert rec.get_tape() is False
    g = keep.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    ps = api.Partset.halo(g, case.inp.pos, None, case.L)
    st = Step(api, case)
    res = {}
    for name, c in (("keep", keep), ("recompute", rec), ("offload", off)):
        o, l, dp = st.run(c, ps, [0])
        torch.cuda.synchronize()
        res[name] = (o.cpu().numpy(), float(l.item()), dp.cpu().numpy(), c.memory())
    assert (res["keep"][0] == res["recompute"][0]).all() and (res["offload"][0] == res["recompute"][0]).all()
    assert (res["offload"][2] == res["recompute"][2]).all()
    n_in, n_h, E = ps.info(0)
    s = 2 if precision == "bf16" else 4
    ztape = case.L * E * case.H * s * (2 if act == "silu" else 1)
    assert res["keep"][3] - res["recompute"][3] == ztape
    errs = per_tensor_errors(case, res["keep"][2], res["recompute"][2])
    worst = sorted(errs.items(), key=lambda kv: -kv[1])[:3]
    log(f"tape policy {precision} {act}: keep vs recompute worst {worst}; z tape {ztape / 1e6:.1f} MB")
    assert worst[0][1] <= (5e-3 if precision == "bf16" else 1e-5), worst
    refs = oracle_refs(case)
    for name in ("keep", "recompute"):
        o, l, dp, _ = res[name]
        log(f"  {name}: " + check_step(case, o, l, dp, refs))


def test_side_stream_alternating_batches(api):
    """Two batches alternated on a non-default stream with no host
    synchronisation between the calls: every rebuild of the cached batch plan
    must wait for the previous batch's kernels, so each step equals the same
    step run alone on the default stream."""
    case = Case(4, levels=(500, 2000, 8000), layers=2, precision="bf16", activation="relu")
    ctx = api.Context(0)
    g = ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    torch.cuda.synchronize()
    ps = api.Partset.halo(g, case.inp.pos, [5000, 3000], case.L)
    st = Step(api, case)
    ref = []
    for i in (0, 1):
        o, l, dp = st.run(ctx, ps, [i])
        torch.cuda.synchronize()
        ref.append((o.cpu().numpy(), dp.cpu().numpy()))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    got = []
    with torch.cuda.stream(side):
        for _ in range(3):
            for i in (0, 1):
                o, l, dp = st.run(ctx, ps, [i])
                got.append((i, o, dp))
    side.synchronize()
    for i, o, dp in got:
        assert (o.cpu().numpy() == ref[i][0]).all()
        assert (dp.cpu().numpy() == ref[i][1]).all()
