"""GPU checks at the workloads' full sizes, in the launch configuration the
benchmark times.

* Outputs: the oracle evaluates sampled nodes one by one through their
  L-hop in-cones (an output depends only on its L-hop in-neighbourhood,
  Eq. 4), compared with the GPU's full-graph forward on the same rows.
* kNN: sampled receivers' segments against the oracle's exact lists.
* Gradients: properties that hold at any size -- a central directional
  difference of the GPU loss, and determinism of the whole step.
* Graph replay: the step captured into a HIP graph and replayed several
  times, with eager work in between, equals the eager step bit for bit.
"""
import numpy as np
import pytest

from cases import Case, check_step, cone_graph, log, rel_l2
from oracle import graph as og
from oracle import model as om
from oracle import partition as opart

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_17164_amd import api as a
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


class Run:
    def __init__(self, api, ctx, case, part_ids=(0,), ps=None, g=None):
        self.api, self.ctx, self.case = api, ctx, case
        self.g = g or ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
        self.ps = ps or api.Partset.halo(self.g, case.inp.pos, None, case.L)
        self.part_ids = list(part_ids)
        self.model = case.model(api)
        self.p = dev(case.params)
        self.node_in, self.pos, self.tgt = dev(case.inp.node_in), dev(case.inp.pos), dev(case.inp.targets)
        self.out = torch.zeros(case.N, 4, device="cuda")
        self.d_out = torch.zeros_like(self.out)
        self.loss = torch.zeros(1, device="cuda")
        self.dp = torch.zeros_like(self.p)

    def step(self, backward=True, params=None):
        p = self.p if params is None else params
        self.ctx.forward(self.model, p, self.ps, self.part_ids, self.node_in, self.pos, self.case.inp.edge_norm,
                         self.out, keep_tape=backward)
        self.ctx.mse_grad(self.out, self.tgt, self.case.N, self.d_out, self.loss)
        if backward:
            self.ctx.backward(self.model, p, self.d_out, self.dp)


def sampled_outputs(case, G, seeds):
    """Oracle outputs of the seed nodes from their L-hop in-cone."""
    c = opart.in_cone(G, seeds, case.L)
    y = om.forward(case.desc, case.params.astype(np.float64), c.graph, case.inp.node_in[c.gid],
                   case.inp.pos[c.gid], case.inp.edge_norm)
    return y[: len(seeds)], len(c.gid)


@pytest.mark.parametrize("cfg,precision,tol,n_seeds", [(2, "fp32", 1e-4, 6), (2, "bf16", 2e-2, 6),
                                                       (3, "bf16", 2e-2, 2), (3, "fp32", 1e-4, 2)])
def test_fullsize_sampled_outputs(api, ctx, cfg, precision, tol, n_seeds):
    case = Case(cfg, precision=precision)
    log(f"full-size cfg={cfg} {precision}: N={case.N}")
    r = Run(api, ctx, case)
    r.step(backward=False)
    torch.cuda.synchronize()
    y = r.out.cpu().numpy()
    assert np.isfinite(y).all()
    G = case.oracle_graph()
    rp, col = r.g.export()
    rng = np.random.default_rng(99)
    seeds = np.sort(rng.choice(case.N, n_seeds, replace=False))
    # kNN segments of sampled receivers, bit for bit
    for s in rng.choice(case.N, 200, replace=False):
        assert (col[rp[s]:rp[s + 1]] == G.col[G.row_ptr[s]:G.row_ptr[s + 1]]).all()
    errs = []
    for s in seeds:
        yo, cone = sampled_outputs(case, G, [s])
        errs.append(rel_l2(y[s], yo[0]))
        log(f"  seed {s}: in-cone {cone} nodes, rel-L2 {errs[-1]:.2e}")
    assert max(errs) <= tol, errs


def test_fullsize_directional_derivative(api, ctx):
    """(loss(p + eps v) - loss(p - eps v)) / 2 eps against grad . v, FP32,
    15 layers on the 200k-node ellipsoid."""
    case = Case(2, precision="fp32", activation="silu")
    r = Run(api, ctx, case)
    r.step()
    torch.cuda.synchronize()
    grad = r.dp.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(5)
    # direction half along the gradient, half random, so grad . v is large
    v = rng.standard_normal(len(case.params))
    v = v / np.linalg.norm(v) + grad / np.linalg.norm(grad)
    v = (v / np.linalg.norm(v)).astype(np.float32)
    eps = 1e-2
    losses = []
    for sgn in (1, -1):
        p = dev((case.params + sgn * eps * v).astype(np.float32))
        r.step(backward=False, params=p)
        torch.cuda.synchronize()
        losses.append(float(r.loss.item()))
    fd = (losses[0] - losses[1]) / (2 * eps)
    an = float(grad @ v.astype(np.float64))
    log(f"  fd {fd:.6e} analytic {an:.6e}")
    assert abs(fd - an) <= 1e-2 * max(abs(an), 1e-6)


def test_graph_replay_equals_eager(api, ctx):
    case = Case(3, levels=(2000, 8000, 32000), layers=4, precision="bf16")
    r = Run(api, ctx, case)
    r.step()
    torch.cuda.synchronize()
    y0, g0, l0 = r.out.clone(), r.dp.clone(), r.loss.clone()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        r.step()
    for i in range(3):
        r.out.zero_()
        r.dp.fill_(float("nan"))
        gr.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.out, y0), i
        assert torch.equal(r.dp, g0), i
        assert torch.equal(r.loss, l0), i
        # eager work between replays
        r.step()
        torch.cuda.synchronize()
        assert torch.equal(r.dp, g0)


def test_fullsize_car_4m_sampled_outputs(api, ctx):
    """The 4M-point car recipe at H = 256 (BF16, 15 layers) as one batch:
    outputs of sampled nodes against the oracle through their 15-hop
    in-cones, and the kNN rows of every node of those cones bit for bit."""
    from scipy.spatial import cKDTree
    case = Case(5, precision="bf16")
    log(f"full-size car: N={case.N}")
    r = Run(api, ctx, case)
    r.ctx.forward(r.model, r.p, r.ps, r.part_ids, r.node_in, r.pos, case.inp.edge_norm, r.out, keep_tape=False)
    torch.cuda.synchronize()
    y = r.out.cpu().numpy()
    assert np.isfinite(y).all()
    rp, col = r.g.export()
    pos64 = case.inp.pos.astype(np.float64)
    trees = {n_l: cKDTree(pos64[:n_l]) for n_l in case.levels}
    rng = np.random.default_rng(99)
    for s in np.sort(rng.choice(case.N, 2, replace=False)):
        G = cone_graph(case, int(s), trees)
        rows = np.flatnonzero(np.diff(G.row_ptr) > 0)
        for q in rows:
            assert (col[rp[q]:rp[q + 1]] == G.col[G.row_ptr[q]:G.row_ptr[q + 1]]).all(), q
        c = opart.in_cone(G, [s], case.L)
        yo = om.forward(case.desc, case.params.astype(np.float64), c.graph, case.inp.node_in[c.gid],
                        case.inp.pos[c.gid], case.inp.edge_norm)
        ya = om.forward(case.desc, om.amp_cast(case.desc, case.params), c.graph, case.inp.node_in[c.gid],
                        case.inp.pos[c.gid], case.inp.edge_norm)
        e, ea = rel_l2(y[s], yo[0]), rel_l2(y[s], ya[0])
        log(f"  seed {s}: in-cone {len(c.gid)} nodes, {len(rows)} kNN rows bit-exact, rel-L2 {e:.2e} "
            f"(cast weights {ea:.2e})")
        assert e <= 2e-2 and ea <= 2e-2


def test_fullsize_partition_gradient(api, ctx):
    """One partition of the 1M-point, 24-part workload (its smallest, with
    its 15-hop halo; FP32, 15 layers) in the configuration the benchmark
    runs it: the partition's nodes against the oracle's RCB and halo, and
    its outputs, loss and every gradient tensor G_p (before accumulation,
    with the global normaliser) against the oracle's step on it."""
    from scipy.spatial import cKDTree
    case = Case(4, precision="fp32")
    sizes = case.inp.part_sizes
    p = int(np.argmin(sizes))
    log(f"full-size partition {p} of {len(sizes)}: {sizes[p]} inner nodes of {case.N}")
    g = ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    ps = api.Partset.halo(g, case.inp.pos, sizes, case.L)
    r = Run(api, ctx, case, part_ids=(p,), ps=ps, g=g)
    r.step()
    torch.cuda.synchronize()
    inner = np.flatnonzero(opart.rcb(case.inp.pos, sizes) == p)
    pos64 = case.inp.pos.astype(np.float64)
    trees = {n_l: cKDTree(pos64[:n_l]) for n_l in case.levels}
    P = opart.Part(cone_graph(case, inner, trees), inner, case.L)
    x = ps.export(p)
    assert (x["gid"] == P.gid).all() and (x["col"] == P.graph.col).all()
    log(f"  {len(P.gid)} local nodes, {P.graph.n_edges} edges: partition bit-exact")
    refs = (om.step_part(case.desc, case.params.astype(np.float64), P, case.inp.node_in, case.inp.pos,
                         case.inp.edge_norm, case.inp.targets, case.N), None)
    y = r.out.cpu().numpy()[P.gid[: P.n_inner]]
    log("  " + check_step(case, y, float(r.loss.item()), r.dp.cpu().numpy(), refs))
