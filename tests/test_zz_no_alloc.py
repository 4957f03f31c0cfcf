"""The allocation-free training step (crk_hnet_train_step_noalloc, static
device scratch) against crk_hnet_train_step (context workspace): two calls
in a row, the second on a smaller batch, give bit-identical weights, Adam
moments, gradient and loss; batches beyond the static scratch are refused
on the host before any launch."""
import numpy as np
import pytest
import torch

import crk_inputs as ci
from paper_2202_02840_amd import Context, CrkError

pytestmark = pytest.mark.gpu


def _batch(seed, B):
    g = np.random.default_rng(seed)
    f = g.normal(0, 1, (B, 8))
    f[:, 7] = 1.0
    return (torch.as_tensor(np.ascontiguousarray(f.T, dtype=np.float32), device="cuda"),
            torch.as_tensor(g.normal(0, 0.3, B).astype(np.float32), device="cuda"))


def test_noalloc_train_step_matches_workspace_step():
    th0 = torch.as_tensor(ci.hnet_init(21).astype(np.float32), device="cuda")
    ref_ctx, ctx = Context(0), Context(0)
    th_r, m_r, v_r = th0.clone(), torch.zeros_like(th0), torch.zeros_like(th0)
    th_s, m_s, v_s = th0.clone(), torch.zeros_like(th0), torch.zeros_like(th0)
    grad = torch.empty_like(th0)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    # the first call fills the whole static scratch; the second, smaller one
    # must not see the rows the first left behind
    for step, (seed, B) in enumerate(((31, 8192), (32, 777)), start=1):
        print(f"[case] noalloc train step {step} nb={B}", flush=True)
        f, t = _batch(seed, B)
        g_r, l_r = ref_ctx.hnet_train_step(th_r, m_r, v_r, step, 1e-3, f, t, want_grad=True,
                                           want_loss=True)
        ctx.hnet_train_step_noalloc(th_s, m_s, v_s, step, 1e-3, f, t, grad=grad, loss=loss)
        torch.cuda.synchronize()
        assert torch.equal(grad, g_r), step
        assert float(loss.item()) == l_r, step
        assert torch.equal(th_s, th_r) and torch.equal(m_s, m_r) and torch.equal(v_s, v_r), step
    ctx.close()
    ref_ctx.close()


def test_noalloc_refuses_batches_beyond_the_scratch():
    ctx = Context(0)
    th = torch.as_tensor(ci.hnet_init(22).astype(np.float32), device="cuda")
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    f, t = _batch(33, 8193)
    before = th.clone()
    with pytest.raises(CrkError) as e:
        ctx.hnet_train_step_noalloc(th, m, v, 1, 1e-3, f, t)
    assert e.value.status == -1 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(th, before)
    ctx.close()
