"""GPU: the steps on either side of the hot path (Sec. V.D, III.D).

The optimizer step (global-norm clipping + Adam) against the FP64 oracle's,
over several steps with clipping active and inactive; the inference loop
(forward without a tape over partitions, halo rows dropped, re-assembled)
against the training forward and the oracle; and a short training run
whose loss falls."""
import numpy as np
import pytest

from cases import Case, log, rel_l2
from oracle import model as om
from oracle import optim

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


@pytest.mark.parametrize("n", [1, 1000, 1_234_567])
def test_adam_step_matches_oracle(api, n):
    """Each step from the same state on both sides (the library's FP32
    parameters and moments after the previous step): moments and norm to
    FP32 rounding, parameters within two units in the last place plus 1e-6
    of the update's scale (lr times the moment terms over the root of the
    second moment; the update is a handful of FP32 operations)."""
    ctx = api.Context(0)
    rng = np.random.default_rng(n)
    params = dev(rng.standard_normal(n).astype(np.float32))
    opt = api.Adam(ctx, params, clip_norm=32.0)
    scales = [200.0, 0.3, 50.0, 1.0, 0.01]   # gradient norms around and across the threshold
    for t, sc in enumerate(scales, start=1):
        p0, m0, v0 = (x.cpu().numpy().astype(np.float64) for x in (params, opt.m, opt.v))
        g = (rng.standard_normal(n) * sc / np.sqrt(n) * 40).astype(np.float32)
        lr = optim.cosine_lr(t - 1, len(scales), 1e-3, 1e-6)
        opt.step(dev(g), lr)
        p, m, v, norm = optim.adam_step(p0, g, m0, v0, t, lr=lr, clip=32.0)
        torch.cuda.synchronize()
        got = params.cpu().numpy().astype(np.float64)
        ulp = np.spacing(np.abs(p).astype(np.float32)).astype(np.float64)
        # condition of the update: where b1 m0 and (1 - b1) g nearly cancel,
        # FP32 rounding of the two terms, not of their small sum, sets the error
        gc = g * min(1.0, 32.0 / (norm + 1e-6))
        terms = (0.9 * np.abs(m0) + 0.1 * np.abs(gc)) / (1 - 0.9 ** t)
        scale = lr * terms / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
        e_p = float(np.max(np.abs(got - p) / (ulp + 1e-6 * scale)))
        e_m = rel_l2(opt.m.cpu().numpy(), m)
        e_v = rel_l2(opt.v.cpu().numpy(), v)
        e_n = abs(float(opt.norm.item()) - norm) / norm
        log(f"n={n} t={t} norm {norm:.3g}: params {e_p:.2f} x (ulp + 1e-6 scale) m {e_m:.2e} v {e_v:.2e} "
            f"norm {e_n:.2e}")
        assert e_p <= 2.0 and e_m <= 1e-6 and e_v <= 1e-6 and e_n <= 1e-6


def test_adam_rejects_bad_arguments(api):
    ctx = api.Context(0)
    p = torch.zeros(10, device="cuda")
    opt = api.Adam(ctx, p)
    with pytest.raises(api.XmgnError):
        opt.step(torch.zeros(10, device="cuda"), float("nan"))
    with pytest.raises(ValueError):
        opt.step(torch.zeros(9, device="cuda"), 1e-3)
    from paper_2411_17164_amd._lib import lib
    assert lib.xmgn_adam_step(ctx._h, None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, 32.0, None, None) == 0
    assert lib.xmgn_adam_step(ctx._h, None, None, None, None, 0, 0, 1e-3, 0.9, 0.999, 1e-8, 32.0, None, None) == -1


def test_inference_over_partitions(api):
    """Inference (no tape) over 3 partitions in 2 batches re-assembles the
    full graph's output bit for bit (halo rows dropped), equal to the
    training forward and within the bound of the oracle."""
    case = Case(4, levels=(500, 2000, 8000), layers=3, precision="bf16", activation="silu")
    ctx = api.Context(0)
    g = ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    torch.cuda.synchronize()
    model = case.model(api)
    p = dev(case.params)
    node_in, pos = dev(case.inp.node_in), dev(case.inp.pos)
    full = api.Partset.halo(g, case.inp.pos, None, case.L)
    y_train = torch.zeros(case.N, 4, device="cuda")
    ctx.forward(model, p, full, [0], node_in, pos, case.inp.edge_norm, y_train, keep_tape=True)
    ps = api.Partset.halo(g, case.inp.pos, np.array([2500, 3000, 2500]), case.L)
    y_inf = torch.full((case.N, 4), float("nan"), device="cuda")
    for wave in ([0, 2], [1]):
        ctx.forward(model, p, ps, wave, node_in, pos, case.inp.edge_norm, y_inf, keep_tape=False)
    torch.cuda.synchronize()
    assert torch.equal(y_inf, y_train)
    y_r = om.forward(case.desc, case.params.astype(np.float64), case.oracle_graph(), case.inp.node_in,
                     case.inp.pos, case.inp.edge_norm)
    assert rel_l2(y_inf.cpu().numpy(), y_r) <= 2e-2


def test_training_loss_falls(api):
    """Twenty steps of the paper's recipe (two partitions per step, gradients
    aggregated, clip 32, Adam on a cosine schedule) on a small car: the loss
    falls."""
    case = Case(5, levels=(400, 1600, 5000), hidden=128, layers=4, precision="bf16", activation="silu")
    ctx = api.Context(0)
    g = ctx.build_knn(dev(case.inp.pos), case.levels, case.k_intra, case.k_cross)
    torch.cuda.synchronize()
    model = case.model(api)
    params = dev(case.params)
    node_in, pos, tgt = dev(case.inp.node_in), dev(case.inp.pos), dev(case.inp.targets)
    ps = api.Partset.halo(g, case.inp.pos, np.array([2000, 3000]), case.L)
    opt = api.Adam(ctx, params, clip_norm=32.0)
    out = torch.zeros(case.N, 4, device="cuda")
    d_out, loss = torch.zeros_like(out), torch.zeros(1, device="cuda")
    d_params, acc = torch.zeros_like(params), torch.zeros_like(params)
    losses = []
    steps = 20
    for t in range(steps):
        acc.zero_()
        total = 0.0
        for part in (0, 1):
            ctx.forward(model, params, ps, [part], node_in, pos, case.inp.edge_norm, out, keep_tape=True)
            ctx.mse_grad(out, tgt, case.N, d_out, loss)
            ctx.backward(model, params, d_out, d_params)
            api.grad_accumulate(acc, d_params)
            total += float(loss.item())
        opt.step(acc, api.cosine_lr(t, steps, 1e-3, 1e-6))
        losses.append(total)
    torch.cuda.synchronize()
    log(f"losses {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0]  # the FP64 oracle run of the same recipe: 3.41 -> 1.01
