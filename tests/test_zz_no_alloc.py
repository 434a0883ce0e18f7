"""GPU: the allocation-free optimizer step (xmgn_adam_step_noalloc), called
through the C ABI, against the context's step (xmgn_adam_step) on the same
inputs: two calls in a row on the same parameters, the second with a
smaller input, every output bit for bit (same kernels, same partial count;
only the home of the norm's partials differs)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_17164_amd import api as a
    return a


def _state(n, seed):
    rng = np.random.default_rng(seed)
    t = lambda x: torch.from_numpy(x.astype(np.float32)).cuda()  # noqa: E731
    return dict(p=t(rng.standard_normal(n)), g=t(rng.standard_normal(n) * 3.0),
                m=t(rng.standard_normal(n) * 0.1), v=t(np.abs(rng.standard_normal(n)) * 0.01))


def _clone(st):
    return {k: v.clone() for k, v in st.items()}


@pytest.mark.parametrize("clip", [4.0, 0.0])
def test_noalloc_adam_matches_context_step(api, clip):
    from paper_2411_17164_amd._lib import check, lib
    ctx = api.Context(0)
    stream = torch.cuda.current_stream().cuda_stream
    for call, (n, step, seed) in enumerate([(1_000_003, 1, 11), (4_097, 7, 12)]):
        a = _state(n, seed)
        b = _clone(a)
        na, nb = torch.zeros(1, device="cuda"), torch.full((1,), float("nan"), device="cuda")
        check(lib.xmgn_adam_step(ctx._h, a["p"].data_ptr(), a["g"].data_ptr(), a["m"].data_ptr(),
                                 a["v"].data_ptr(), n, step, 1e-3, 0.9, 0.999, 1e-8, clip, na.data_ptr(), stream))
        check(lib.xmgn_adam_step_noalloc(0, b["p"].data_ptr(), b["g"].data_ptr(), b["m"].data_ptr(),
                                         b["v"].data_ptr(), n, step, 1e-3, 0.9, 0.999, 1e-8, clip, nb.data_ptr(),
                                         stream))
        torch.cuda.synchronize()
        for k in ("p", "m", "v", "g"):
            assert torch.equal(a[k], b[k]), (call, k)
        assert torch.equal(na, nb), call
        norm = float(np.linalg.norm(a["g"].cpu().numpy().astype(np.float64)))
        assert abs(nb.item() - norm) <= 1e-6 * norm
        if clip > 0:
            assert norm > clip  # the clipping branch is taken
        changed = (b["p"] != _state(n, seed)["p"]).float().mean().item()
        assert changed > 0.99


def test_noalloc_adam_rejects_bad_arguments(api):
    from paper_2411_17164_amd._lib import lib
    x = torch.zeros(8, device="cuda")
    p = x.data_ptr()
    s = torch.cuda.current_stream().cuda_stream
    assert lib.xmgn_adam_step_noalloc(-1, p, p, p, p, 8, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0, None, s) == -1
    assert lib.xmgn_adam_step_noalloc(4096, p, p, p, p, 8, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0, None, s) == -1
    assert lib.xmgn_adam_step_noalloc(0, p, p, p, p, 8, 0, 1e-3, 0.9, 0.999, 1e-8, 0.0, None, s) == -1
    assert b"step" in lib.xmgn_last_error()
    assert lib.xmgn_adam_step_noalloc(0, p, p, p, p, -1, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0, None, s) == -1
    assert lib.xmgn_adam_step_noalloc(0, None, p, p, p, 8, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0, None, s) == -1
    assert b"NULL" in lib.xmgn_last_error()
    # n = 0 is a no-op that still succeeds
    assert lib.xmgn_adam_step_noalloc(0, None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, 0.0, None, s) == 0
    torch.cuda.synchronize()
