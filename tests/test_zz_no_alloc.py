"""rtg_collision_check_noalloc, the entry point that allocates nothing (its
scratch is the library's fixed device array), against rtg_collision_check
through the C ABI: two calls in a row, the second with a smaller input, and
an input too large for the fixed array."""
import ctypes

import numpy as np
import pytest
import torch

import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _call(L, name, ctx, gs, pts, n_pts, hit, clr):
    return getattr(L, name)(ctx.handle, ctypes.byref(gs), ctypes.c_void_p(pts.data_ptr()), n_pts, 0.25, 3.0,
                            ctypes.c_void_p(hit.data_ptr()), ctypes.c_void_p(clr.data_ptr()), None)


def test_no_alloc_collision_matches_allocating_entry_point():
    from paper_2409_18122_amd import raster
    from paper_2409_18122_amd._lib import Gaussians, lib
    L = lib()
    ctx = raster.Context(0)
    lot = scenes.lot_scene()  # 3M Gaussians: 72 MB of the 96 MiB scratch
    dev = torch.device("cuda:0")
    cases = [(lot, 16, 7), (scenes.subset(lot, np.arange(0, 3_000_000, 7)), 2, 8)]
    for k, (scene, n_paths, seed) in enumerate(cases):
        means = torch.as_tensor(scene["means"]).to(dev).contiguous()
        ls = torch.as_tensor(scene["log_scales"]).to(dev).contiguous()
        n = int(means.shape[1])
        gs = Gaussians(n, ctypes.c_void_p(means.data_ptr()), ctypes.c_void_p(ls.data_ptr()), None, None, None, None)
        pts = torch.as_tensor(scenes.path_points(n_paths, seed)).to(dev).contiguous()
        npt = int(pts.shape[1])
        say(f"call {k}: {n} Gaussians, {npt} points")
        out = {}
        for name in ("rtg_collision_check", "rtg_collision_check_noalloc"):
            hit = torch.full((npt,), -7, device=dev, dtype=torch.int32)
            clr = torch.full((npt,), float("nan"), device=dev, dtype=torch.float32)
            rc = _call(L, name, ctx, gs, pts, npt, hit, clr)
            assert rc == 0, (name, L.rtg_last_error())
            torch.cuda.synchronize()
            out[name] = (hit.cpu().numpy(), clr.cpu().numpy())
        a, b = out["rtg_collision_check"], out["rtg_collision_check_noalloc"]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), k
        assert 0 < int(b[0].sum()) < npt
        say(f"call {k}: {int(b[0].sum())} of {npt} points collide; identical to the allocating entry point")
    # beyond the fixed scratch: refused before any launch, outputs untouched
    # (the arrays are allocated at full size all the same)
    big_n = (96 << 20) // 24 + 1
    big_m = torch.zeros((3, big_n), device=dev, dtype=torch.float32)
    big_l = torch.full((3, big_n), -3.0, device=dev, dtype=torch.float32)
    gs = Gaussians(big_n, ctypes.c_void_p(big_m.data_ptr()), ctypes.c_void_p(big_l.data_ptr()), None, None, None,
                   None)
    hit = torch.full((npt,), -7, device=dev, dtype=torch.int32)
    clr = torch.zeros(npt, device=dev, dtype=torch.float32)
    rc = _call(L, "rtg_collision_check_noalloc", ctx, gs, pts, npt, hit, clr)
    assert rc == -5 and b"fixed" in L.rtg_last_error()
    torch.cuda.synchronize()
    assert bool((hit == -7).all())
    ctx.close()
