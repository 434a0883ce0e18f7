"""GPU: the torch.autograd.Function around the C ABI (api.ProcessorFn).

The hand-written adjoint (xmgn_backward, recomputing every layer from the
forward's checkpoints) sits behind autograd: loss.backward() must give the
FP64 oracle's gradient at the parity bar and the C ABI's own backward bit
for bit.  A context keeps the tape of its last forward only, so an
application whose tape a later forward replaced must refuse its backward;
applications on contexts of their own accumulate their partitions'
gradients in params.grad as the aggregation of Sec. III.A does."""
import numpy as np
import pytest

from cases import Case, check_step, log, oracle_refs, per_tensor_errors
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def setup(api, case):
    ctx = api.Context(0)
    g = ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    torch.cuda.synchronize()
    return ctx, g


@pytest.mark.parametrize("precision,act", [("fp32", "silu"), ("bf16", "relu")])
def test_processor_fn_backward(api, precision, act):
    """loss.backward() through ProcessorFn against the oracle gradient, and
    bitwise against xmgn_forward + xmgn_backward on the same d_out."""
    case = Case(3, levels=(500, 2000, 6000), layers=3, precision=precision, activation=act)
    log(f"ProcessorFn {precision} {act}")
    ctx, g = setup(api, case)
    ps = api.Partset.halo(g, case.inp.pos, None, case.L)
    model = case.model(api)
    p = dev(case.params).requires_grad_(True)
    node_in, pos, tgt = dev(case.inp.node_in), dev(case.inp.pos), dev(case.inp.targets)
    out = api.ProcessorFn.apply(p, node_in, pos, ctx, model, ps, [0], case.inp.edge_norm)
    # the masked MSE gradient from the library: sum(out * d_out) then has
    # exactly d_out as its gradient, so autograd hands xmgn_backward d_out
    d_out = torch.zeros_like(out)
    loss = torch.zeros(1, device="cuda")
    ctx.mse_grad(out.detach(), tgt, case.N, d_out, loss)
    (out * d_out).sum().backward()
    torch.cuda.synchronize()
    grad = p.grad.cpu().numpy()
    # the same step through the C ABI directly
    pd = p.detach()
    out2 = torch.zeros_like(out)
    ctx.forward(model, pd, ps, [0], node_in, pos, case.inp.edge_norm, out2, keep_tape=True)
    d_params = torch.full_like(pd, float("nan"))
    ctx.backward(model, pd, d_out, d_params)
    torch.cuda.synchronize()
    assert (out2 == out.detach()).all()
    assert (d_params.cpu().numpy() == grad).all()
    log("  " + check_step(case, out.detach().cpu().numpy(), float(loss.item()), grad, oracle_refs(case)))


def test_processor_fn_refuses_a_replaced_tape(api):
    """Two applications on one context: the first one's tape is gone when
    its backward runs, so loss.backward() raises instead of returning the
    second batch's gradient."""
    case = Case(3, levels=(500, 2000, 6000), layers=2, precision="fp32", activation="silu")
    ctx, g = setup(api, case)
    ps = api.Partset.halo(g, case.inp.pos, [3000, 3000], case.L)
    model = case.model(api)
    p = dev(case.params).requires_grad_(True)
    node_in, pos = dev(case.inp.node_in), dev(case.inp.pos)
    s0 = ctx.tape_serial()
    y0 = api.ProcessorFn.apply(p, node_in, pos, ctx, model, ps, [0], case.inp.edge_norm)
    s1 = ctx.tape_serial()
    y1 = api.ProcessorFn.apply(p, node_in, pos, ctx, model, ps, [1], case.inp.edge_norm)
    s2 = ctx.tape_serial()
    assert 0 == s0 < s1 < s2
    with pytest.raises(api.XmgnError, match="later forward"):
        (y0.sum() + y1.sum()).backward()
    # a forward without a tape leaves none to consume
    out = torch.zeros_like(y0)
    ctx.forward(model, p.detach(), ps, [0], node_in, pos, case.inp.edge_norm, out, keep_tape=False)
    assert ctx.tape_serial() == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_processor_fn_partitions_one_context_each(api, precision):
    """Each partition applied on its own context: autograd adds the
    partitions' gradients into params.grad, which must meet the parity bar
    against the oracle's partitioned step (Sec. III.A)."""
    case = Case(4, levels=(500, 2000, 8000), layers=3, precision=precision, activation="silu")
    log(f"ProcessorFn partitions {precision}")
    ctx0, g = setup(api, case)
    sizes = np.array([2500, 3500, 2000])
    ps = api.Partset.halo(g, case.inp.pos, sizes, case.L)
    model = case.model(api)
    p = dev(case.params).requires_grad_(True)
    node_in, pos, tgt = dev(case.inp.node_in), dev(case.inp.pos), dev(case.inp.targets)
    ctxs = [ctx0] + [api.Context(0) for _ in range(len(sizes) - 1)]
    total = None
    y = np.zeros((case.N, 4))
    loss_sum = 0.0
    for i, c in enumerate(ctxs):
        out = api.ProcessorFn.apply(p, node_in, pos, c, model, ps, [i], case.inp.edge_norm)
        d_out = torch.zeros_like(out)
        loss = torch.zeros(1, device="cuda")
        c.mse_grad(out.detach(), tgt, case.N, d_out, loss)
        term = (out * d_out).sum()
        total = term if total is None else total + term
        gid = ps.export(i)["gid"][: ps.info(i)[0]]
        y[gid] = out.detach().cpu().numpy()[gid]
        loss_sum += float(loss.item())
    total.backward()
    torch.cuda.synchronize()
    grad = p.grad.cpu().numpy()
    parts, _ = opart.partition(case.oracle_graph(), case.inp.pos, sizes, case.L)
    args = (parts, case.inp.node_in, case.inp.pos, case.inp.edge_norm, case.inp.targets)
    base = om.step_partitioned(case.desc, case.params.astype(np.float64), *args)
    amp = om.step_partitioned(case.desc, om.amp_cast(case.desc, case.params), *args) if precision == "bf16" else None
    log("  " + check_step(case, y, loss_sum, grad, (base, amp)))
    # the oracle's partitioned step is the full-graph step (pinned on the CPU)
    full = oracle_refs(case)[0]
    assert max(per_tensor_errors(case, base[2], full[2]).values()) <= 1e-10
