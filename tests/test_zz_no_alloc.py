"""The allocation-free MLP backward (nvgs_mlp_backward_noalloc) against the
allocating entry point nvgs_mlp_backward: two calls in a row, the second
with a smaller batch, bit-identical gradients, and no device allocation
during the calls."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_19202_amd as nvgs
    ctx = nvgs.Context(0)
    yield nvgs, ctx, torch
    ctx.close()


def _allocations(torch):
    return torch.cuda.memory_stats(0).get("allocation.all.allocated", 0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_backward_equals_allocating_backward(env, prec):
    nvgs, ctx, torch = env
    p = torch.from_numpy(synth.mlp_params(64, synth.rng(31)).astype(np.float32)).cuda()
    g = np.random.default_rng(32)
    # the largest accepted batch first, then a smaller, ragged one
    for B in (65536, 1000):
        log(f"[noalloc] prec={prec} B={B}")
        X = torch.from_numpy(g.uniform(-1, 1, (B, 72)).astype(np.float32)).cuda()
        dlog = torch.from_numpy((g.standard_normal(B) / B).astype(np.float32)).cuda()
        dp = torch.full((nvgs.NUM_PARAMS_W64,), float("nan"), device="cuda")
        dx = torch.full((B, 72), float("nan"), device="cuda")
        torch.cuda.synchronize()
        before = _allocations(torch)
        ctx.mlp_backward_noalloc(p, X, dlog, dp, dx, precision=prec)
        torch.cuda.synchronize()
        assert _allocations(torch) == before, "the allocation-free entry point allocated device memory"
        dp_ref, dx_ref = ctx.mlp_backward(p, X, dlog, precision=prec)
        torch.cuda.synchronize()
        assert _allocations(torch) > before  # the probe sees the allocating entry point's buffers
        assert torch.equal(dp, dp_ref), float((dp - dp_ref).abs().max())
        assert torch.equal(dx, dx_ref), float((dx - dx_ref).abs().max())


def test_noalloc_backward_rejects_batches_beyond_the_workspace(env):
    nvgs, ctx, torch = env
    B = 65537
    p = torch.from_numpy(synth.mlp_params(64, synth.rng(33)).astype(np.float32)).cuda()
    X = torch.zeros((B, 72), device="cuda")
    dlog = torch.zeros(B, device="cuda")
    dp = torch.zeros(nvgs.NUM_PARAMS_W64, device="cuda")
    with pytest.raises(nvgs.NvgsError) as e:
        ctx.mlp_backward_noalloc(p, X, dlog, dp, None)
    assert e.value.status == 1 and "NVGS_NOALLOC_MAX_BATCH" in str(e.value)
