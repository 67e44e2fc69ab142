"""Full-size parity of the HIP path with the oracle, in the launch configuration
the benchmark times: 1M Gaussians x 8 keyframes of 1280x720 (autotuned tile),
2M Gaussians x 256 uneven views (captured graph), and FP64 finite-difference
spot checks of GPU gradients.

The oracle computes what it can in seconds: whole images and adjoints of two
sampled keyframes (the other keyframes get zero image gradient, so the GPU's
8-frame batched backward must equal the oracle's two-frame adjoint), scores of
sampled views, and finite differences over the pixels a perturbed Gaussian
can reach.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import (GRAD_REL_TOL, SCORE_TOL_PER_PIXEL, assert_elementwise, assert_images_close, gpu_stack,
                      grad_rel_errors, grads_to_numpy)

pytestmark = pytest.mark.gpu

GROUPS = ("means", "log_scales", "quats", "opacity", "colors")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def raster():
    from paper_2409_18122_amd import raster as r
    return r


@pytest.fixture(scope="module")
def rctx(raster):
    oracle.set_threads(16)
    return raster.Context(0)


def S(tile=(16, 16), **kw):
    s = dict(scenes.DEFAULT_SETTINGS)
    s["tile_w"], s["tile_h"] = tile
    s.update(kw)
    return s


def fd_spot_checks(g, cams, weights, gpu_grads, pairs, settings, rng_seed=0):
    """FP64 central differences of sum_v <w_v, image_v> for (Gaussian, group,
    component) pairs.  Each objective is evaluated over the pixel window the
    Gaussian's support reaches (plus a margin), with only the Gaussians whose
    support meets that window - they are all that composite there, in the same
    order.  Returns (checked, worst ratio of error to tolerance)."""
    g64 = {k: np.asarray(v, np.float64) for k, v in g.items()}
    proj = [oracle.project(g64, c, settings) for c in cams]
    worst = 0.0
    checked = 0
    scale = {k: np.sqrt(np.mean(gpu_grads[k] ** 2)) for k in GROUPS}
    for (i, grp, comp) in pairs:
        views = []
        for v, c in enumerate(cams):
            p = proj[v]
            if not p["valid"][i]:
                continue
            u0, u1, v0, v1 = (int(x) for x in p["box"][:, i])
            m = 2
            roi = (max(u0 - m, 0), max(v0 - m, 0), min(u1 + m + 1, c["width"]), min(v1 + m + 1, c["height"]))
            bx = p["box"]
            sel = np.nonzero(p["valid"] & (bx[0] < roi[2]) & (bx[1] >= roi[0]) &
                             (bx[2] < roi[3]) & (bx[3] >= roi[1]))[0]
            sel = np.union1d(sel, [i])
            views.append((v, c, roi, sel))
        if not views:
            continue
        flat_idx = np.ravel_multi_index((comp, i), g64[grp].shape) if g64[grp].ndim == 2 else i
        theta = g64[grp].reshape(-1)[flat_idx]
        h = 1e-7 * max(1.0, abs(theta))
        vals, sigs = [], []
        for sgn in (1.0, -1.0):
            tot = 0.0
            sig = []
            for (v, c, roi, sel) in views:
                sub = scenes.subset(g64, sel)
                j = int(np.searchsorted(sel, i))
                arr = sub[grp]
                if arr.ndim == 2:
                    arr[comp, j] += sgn * h
                else:
                    arr[j] += sgn * h
                r = oracle.render(sub, c, settings, roi=roi)
                x0, y0, x1, y1 = roi
                img = np.concatenate([r["rgb"], r["depth"][None], r["alpha"][None], r["unc"][None]])
                tot += float((weights[v][:, y0:y1, x0:x1] * img[:, y0:y1, x0:x1]).sum())
                sig.append((r["ncontrib"][y0:y1, x0:x1].copy(), r["T"][y0:y1, x0:x1].copy()))
            vals.append(tot)
            sigs.append(sig)
        # a threshold decision that changes inside the stencil changes a
        # pixel's contributor count, or its final transmittance by a factor
        # (1 - alpha) with alpha >= alpha_min; smooth changes are ~1e-6
        if any(not np.array_equal(a[0], b[0]) or np.max(np.abs(a[1] - b[1]) / b[1], initial=0.0) > 1e-4
               for a, b in zip(sigs[0], sigs[1])):
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        got = gpu_grads[grp][comp, i] if gpu_grads[grp].ndim == 2 else gpu_grads[grp][i]
        tol = GRAD_REL_TOL * (abs(fd) + scale[grp]) + 1e-12
        worst = max(worst, abs(got - fd) / tol)
        checked += 1
    return checked, worst


def random_pairs(rng, visible, n):
    comps = {"means": 3, "log_scales": 3, "quats": 4, "opacity": 1, "colors": 3}
    out = []
    for _ in range(n):
        i = int(rng.choice(visible))
        grp = GROUPS[int(rng.integers(len(GROUPS)))]
        out.append((i, grp, int(rng.integers(comps[grp]))))
    return out


def test_c4_keyframes_full_size(raster, rctx):
    g, cams, _ = scenes.config4()
    dev = raster.to_device(g)
    say("C4: autotune (forward + backward) on 1M Gaussians x 8 x 1280x720")
    tuned = raster.autotune(rctx, dev, cams, 1, S())
    tile = (tuned["tile_w"], tuned["tile_h"])
    say(f"C4: tuned tile {tile}")
    assert tile in ((8, 8), (16, 16), (32, 8))
    st = S(tile)
    f = raster.Frame(rctx, dev, cams, st)
    f.bin_sort()
    out = f.render()
    views = raster.unpack_images(out, cams)
    rng = np.random.default_rng(44)
    checked_views = (0, 5)
    weights, d = [], {"rgb": [], "depth": [], "alpha": [], "unc": []}
    for v, c in enumerate(cams):
        H, W = c["height"], c["width"]
        w = rng.standard_normal((6, H, W)) * 1e-6 if v in checked_views else np.zeros((6, H, W))
        weights.append(w)
        d["rgb"].append(w[:3].astype(np.float32).reshape(-1))
        d["depth"].append(w[3].astype(np.float32).reshape(-1))
        d["alpha"].append(w[4].astype(np.float32).reshape(-1))
        d["unc"].append(w[5].astype(np.float32).reshape(-1))
    t = {k: torch.as_tensor(np.concatenate(x)).cuda() for k, x in d.items()}
    say("C4: batched backward over 8 keyframes")
    grads = grads_to_numpy(f.backward(t["rgb"], t["depth"], t["alpha"], t["unc"]))
    ref = {k: np.zeros_like(np.asarray(g[k], np.float64)) for k in GROUPS}
    touched = np.zeros(scenes.n_gaussians(g), bool)
    for v in checked_views:
        say(f"C4: oracle render + adjoint of keyframe {v}")
        r = oracle.render(g, cams[v], st)
        e, n_excl = assert_images_close(gpu_stack(views[v], cams[v]), r, label=f"C4 view {v}")
        say(f"C4 view {v}: max image err {e:.3g}, excluded {n_excl}")
        w = weights[v]
        a = oracle.adjoint(g, cams[v], st, g_rgb=w[:3], g_depth=w[3], g_alpha=w[4], g_unc=w[5], tile=tile)
        for k in GROUPS:
            ref[k] += a[k]
        touched |= a["touched"]
    rel = grad_rel_errors(grads, ref)
    say(f"C4 gradient relative errors {rel}")
    for k, val in rel.items():
        assert val <= GRAD_REL_TOL, (k, val)
    n_excl = assert_elementwise(grads, ref, touched, "C4")
    say(f"C4 element-wise bar met; {n_excl} Gaussians excluded (near-threshold decisions)")
    # FP64 finite-difference spot checks on (Gaussian, parameter) pairs; a
    # stencil is used only if no threshold decision changes inside it, so more
    # pairs are drawn than must be checked
    vis = np.nonzero(np.abs(ref["opacity"]) > 0)[0]
    pairs = random_pairs(np.random.default_rng(45), vis, 160)
    checked, worst = fd_spot_checks(g, [cams[v] for v in checked_views], [weights[v] for v in checked_views],
                                    grads, pairs, st)
    say(f"C4 FD spot checks: {checked} checked, worst error/tolerance {worst:.3f}")
    assert checked >= 48 and worst <= 1.0


def test_c2_finite_difference_spot_checks(raster, rctx):
    g, cams, _ = scenes.config2()
    dev = raster.to_device(g)
    f = raster.Frame(rctx, dev, cams, S())
    f.bin_sort()
    f.render()
    H, W = 480, 640
    w = np.random.default_rng(21).standard_normal((6, H, W)) * 1e-6
    say("C2: backward with random image weights")
    grads = grads_to_numpy(f.backward(torch.as_tensor(w[:3].astype(np.float32).reshape(-1)).cuda(),
                                      torch.as_tensor(w[3].astype(np.float32).reshape(-1)).cuda(),
                                      torch.as_tensor(w[4].astype(np.float32).reshape(-1)).cuda(),
                                      torch.as_tensor(w[5].astype(np.float32).reshape(-1)).cuda()))
    vis = np.nonzero(np.abs(grads["colors"]).sum(0) > 0)[0]
    pairs = random_pairs(np.random.default_rng(22), vis, 256)
    checked, worst = fd_spot_checks(g, cams, [w], grads, pairs, S())
    say(f"C2 FD spot checks: {checked} checked, worst error/tolerance {worst:.3f}")
    assert checked >= 200 and worst <= 1.0


def test_c5_uneven_graph_full_size(raster, rctx):
    g, cams = scenes.config5()
    dev = raster.to_device(g)
    say("C5: graph over 256 uneven views, 2M Gaussians")
    gr = raster.ScoreGraph(rctx, dev, 256, 640, 480, S(), probe=cams)
    got = gr.launch(cams).cpu().numpy()
    assert gr.status()
    again = gr.launch(cams).cpu().numpy()
    assert gr.status() and np.array_equal(got, again)
    eager = raster.score_views(rctx, dev, cams, S(), persistent=True).cpu().numpy()
    assert np.array_equal(got, eager)
    gr.close()
    say("C5: binary-J graph over the same views")
    grb = raster.ScoreGraph(rctx, dev, 256, 640, 480, S(), probe=cams, mode="binary")
    gotb = grb.launch(cams).cpu().numpy()
    assert grb.status()
    grb.close()
    eagerb = raster.score_views(rctx, dev, cams, S(), persistent=True, mode="binary").cpu().numpy()
    assert np.array_equal(gotb, eagerb) and np.all(gotb >= got)
    # 16 views, the first five or six of each resolution; the binary-J trace
    # on the first of each resolution
    by_size = {}
    for v, c in enumerate(cams):
        by_size.setdefault(c["width"], []).append(v)
    assert len(by_size) == 3
    sample = sorted(sum((vs[:6] if w == 160 else vs[:5] for w, vs in by_size.items()), []))
    assert len(sample) == 16
    refs = oracle.score(g, [cams[v] for v in sample], S())
    rel_max = 0.0
    for v, ref in zip(sample, refs):
        c = cams[v]
        P = c["width"] * c["height"]
        rel = abs(got[v] - ref) / max(abs(ref), 1e-30)
        rel_max = max(rel_max, rel)
        say(f"C5 view {v} ({c['width']}x{c['height']}): gpu {got[v]:.6f} oracle {ref:.6f} rel {rel:.2e}")
        assert abs(got[v] - ref) <= SCORE_TOL_PER_PIXEL * P
    say(f"C5: 16 views within the bar, max relative score error {rel_max:.2e}")
    firsts = [vs[0] for vs in by_size.values()]
    refb = oracle.score(g, [cams[v] for v in firsts], S(), mode=1)
    for v, rb in zip(firsts, refb):
        P = cams[v]["width"] * cams[v]["height"]
        say(f"C5 view {v} binary-J: gpu {gotb[v]:.4f} oracle {rb:.4f} diff {abs(gotb[v] - rb):.3g}")
        assert abs(gotb[v] - rb) <= SCORE_TOL_PER_PIXEL * P


def test_autotuner_choice_does_not_change_results(raster, rctx, tmp_path):
    g, cams = scenes.tiny_scene(800, 5, 160, 120)
    dev = raster.to_device(g)
    base, f0 = raster.render(rctx, dev, cams, S())
    f0.close()
    for mode in (0, 1, 2):
        say(f"autotune mode {mode}")
        tuned = raster.autotune(rctx, dev, cams, mode, S())
        assert (tuned["tile_w"], tuned["tile_h"]) in ((8, 8), (16, 16), (32, 8))
        assert tuned["batch"] in (0, 32, 64, 128) and tuned["batch"] < tuned["tile_w"] * tuned["tile_h"]
        out, f = raster.render(rctx, dev, cams, tuned)
        for k in base:
            assert torch.equal(base[k], out[k]), (mode, k)
        f.close()
    # settings 0x0 take the context's tuned tile and batch
    out, f = raster.render(rctx, dev, cams, dict(S(), tile_w=0, tile_h=0))
    assert f.info()["tile_w"] == tuned["tile_w"]
    for k in base:
        assert torch.equal(base[k], out[k])
    f.close()
    # the JSON cache: the first call tunes and stores, the second returns the
    # stored choice, keyed by mode, resolution, view count and N bucket
    cache = str(tmp_path / "tune.json")
    first = raster.autotune(rctx, dev, cams, 1, S(), cache=cache)
    import json
    with open(cache) as fh:
        table = json.load(fh)
    key = raster.tune_key(dev, cams, 1, S())
    # the key separates settings that change the work
    assert raster.tune_key(dev, cams, 1, S(alpha_min=0.01)) != key
    assert raster.tune_key(dev, cams, 1, S(isotropic=1)) != key
    assert table[key] == {"tile_w": first["tile_w"], "tile_h": first["tile_h"], "batch": first["batch"]}
    table[key] = {"tile_w": 32, "tile_h": 8, "batch": 64}  # a stored entry wins without timing
    with open(cache, "w") as fh:
        json.dump(table, fh)
    again = raster.autotune(rctx, dev, cams, 1, S(), cache=cache)
    assert (again["tile_w"], again["tile_h"], again["batch"]) == (32, 8, 64)
