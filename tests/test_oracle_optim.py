"""Pins of the oracle's optimizer: closed forms of Adam's first step and of
clipping, the schedule's end points, and agreement with torch's CPU Adam,
global-norm clipping and cosine schedule (library routines) over several
steps."""
import numpy as np
import pytest

from oracle import optim


def test_first_step_closed_form():
    g = np.random.default_rng(1).standard_normal(1000)
    p0 = np.random.default_rng(2).standard_normal(1000)
    p, m, v, norm = optim.adam_step(p0, g, np.zeros(1000), np.zeros(1000), 1, lr=1e-3, eps=1e-8)
    # m_hat = g, v_hat = g^2: the first step moves every entry by lr g / (|g| + eps)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    assert norm == pytest.approx(np.linalg.norm(g))


def test_clipping_closed_form():
    g = np.full(400, 3.0)                          # ||g|| = 60
    c, norm = optim.clip_by_global_norm(g, 32.0)
    assert norm == pytest.approx(60.0)
    assert np.linalg.norm(c) == pytest.approx(32.0 * 60.0 / (60.0 + 1e-6))
    small, _ = optim.clip_by_global_norm(g / 10, 32.0)
    assert (small == g / 10).all()                 # below the threshold: unchanged
    same, _ = optim.clip_by_global_norm(g, 0.0)
    assert (same == g).all()


def test_cosine_end_points():
    assert optim.cosine_lr(0, 100, 1e-3, 1e-6) == pytest.approx(1e-3)
    assert optim.cosine_lr(100, 100, 1e-3, 1e-6) == pytest.approx(1e-6)
    assert optim.cosine_lr(50, 100, 1e-3, 1e-6) == pytest.approx(0.5 * (1e-3 + 1e-6))
    assert optim.cosine_lr(250, 100, 1e-3, 1e-6) == pytest.approx(1e-6)


def test_against_torch_adam_clip_and_schedule():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    n, steps, T = 300, 6, 6
    p0 = rng.standard_normal(n)
    grads = [rng.standard_normal(n) * s for s in (40.0, 0.5, 20.0, 1.0, 100.0, 0.1)]
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=T, eta_min=1e-6)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, steps + 1):
        lr = optim.cosine_lr(t - 1, T, 1e-3, 1e-6)
        assert lr == pytest.approx(opt.param_groups[0]["lr"], rel=1e-12)
        w.grad = torch.tensor(grads[t - 1], dtype=torch.float64)
        torch.nn.utils.clip_grad_norm_([w], 32.0)
        opt.step()
        sched.step()
        p, m, v, _ = optim.adam_step(p, grads[t - 1], m, v, t, lr=lr, clip=32.0)
        assert np.allclose(p, w.detach().numpy(), rtol=1e-12, atol=1e-15), t
