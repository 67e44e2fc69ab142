"""The context's device scratch served by a caller allocator (rtg_set_allocator),
here PyTorch's caching allocator: results equal those of the library's own
allocator, the memory is PyTorch's, and it goes back when the context closes."""
import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def raster():
    from paper_2409_18122_amd import raster as r
    return r


def step(raster, ctx, dev, cams, S):
    f = raster.Frame(ctx, dev, cams, S)
    f.bin_sort()
    out = f.render()
    loss, d_rgb, d_dep = f.loss(out["rgb"], out["depth"], torch.zeros_like(out["rgb"]),
                                torch.zeros_like(out["depth"]), 0.5)
    grads = f.backward(d_rgb, d_dep)
    torch.cuda.synchronize()
    return f, out, loss, grads


def test_torch_allocator_serves_scratch(raster):
    g, cams = scenes.config1(n=20_000)
    S = dict(scenes.DEFAULT_SETTINGS)
    dev = raster.to_device(g)
    ref_ctx = raster.Context(0)
    f, out_ref, loss_ref, grads_ref = step(raster, ref_ctx, dev, cams, S)
    f.close()
    ref_ctx.close()

    ctx = raster.Context(0)
    ctx.use_torch_allocator()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    f, out, loss, grads = step(raster, ctx, dev, cams, S)
    during = torch.cuda.memory_allocated()
    # the frame's records, pair lists and per-pixel state are PyTorch memory now
    assert during - before > f.info()["records"] * 64
    for k in out:
        assert torch.equal(out[k], out_ref[k]), k
    assert loss.item() == loss_ref.item()
    for k in grads_ref:
        a, b = grads[k].double(), grads_ref[k].double()
        assert torch.linalg.norm(a - b) <= 1e-6 * torch.linalg.norm(b), k
    # switching allocators while a frame holds scratch is refused
    with pytest.raises(raster.RtgError):
        ctx.use_hip_allocator()
    f.close()
    del out, grads
    ctx.use_hip_allocator()  # hands the cached blocks back to PyTorch
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + (1 << 20)
    ctx.close()
