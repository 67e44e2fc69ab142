"""GPU parity of the isotropic mode (the paper's 8-parameter Gaussians of
Sec. III, r_2D = f r / d) against the oracle, through the C ABI: images within
1e-4, keys bit-exact, gradients within 1e-3 relative, scores within 1e-4 per
pixel."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import (GRAD_REL_TOL, SCORE_TOL_PER_PIXEL, assert_images_close, gpu_stack, grads_to_numpy)

pytestmark = pytest.mark.gpu

TILES = [(8, 8), (16, 16), (32, 8)]
ISO_GROUPS = ("means", "log_scales", "opacity", "colors")


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
    s = dict(scenes.DEFAULT_SETTINGS, isotropic=1)
    s["tile_w"], s["tile_h"] = tile
    s.update(kw)
    return s


def gpu_render(raster, rctx, scene, cams, settings):
    g = raster.to_device(scene)
    out, frame = raster.render(rctx, g, cams, settings)
    views = raster.unpack_images(out, cams)
    return [gpu_stack(v, c) for v, c in zip(views, cams)], frame


def iso_rel_errors(gpu, ref):
    out = {}
    for k in ISO_GROUPS:
        a = np.asarray(gpu[k], np.float64).reshape(-1)
        b = np.asarray(ref[k], np.float64)
        b = (b[:1] if k == "log_scales" else b).reshape(-1)
        out[k] = float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))
    return out


@pytest.mark.parametrize("n", [1, 3, 50, 500])
def test_tiny_isotropic_vs_brute_force(raster, rctx, n):
    g, cams = scenes.tiny_scene(n, 400 + n, 48, 32)
    g = scenes.isotropic_scene(g)
    r = oracle.render(g, cams[0], S(), mode="brute")
    outs = []
    for tile in TILES:
        say(f"isotropic tiny n={n} tile={tile}")
        imgs, f = gpu_render(raster, rctx, g, cams, S(tile))
        f.close()
        assert_images_close(imgs[0], r, label=f"iso n={n} {tile}")
        outs.append(imgs[0])
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_c2_isotropic_forward_and_keys(raster, rctx):
    g, cams, _ = scenes.config2()
    g = scenes.isotropic_scene(g)
    say("isotropic C2 forward, 200k Gaussians, 640x480")
    imgs, f = gpu_render(raster, rctx, g, cams, S())
    r = oracle.render(g, cams[0], S())
    e, n_excl = assert_images_close(imgs[0], r, label="iso C2")
    say(f"  max err {e:.3g}, excluded {n_excl}, instances {f.n_instances}")
    f.close()
    # keys on a smaller map: the list is the oracle's pixel-box list restricted to the GPU's pairs
    g1, cams1 = scenes.config1()
    g1 = scenes.isotropic_scene(g1)
    f = raster.Frame(rctx, raster.to_device(g1), cams1, S())
    f.bin_sort()
    keys, vals, _ = f.export()
    keys = keys.cpu().numpy().view(np.uint64)
    vals = vals.cpu().numpy().view(np.uint32)
    k_box, v_box = oracle.keys(g1, cams1, S(), (16, 16))
    pid = lambda k, v: (k >> np.uint64(32)) << np.uint64(32) | v.astype(np.uint64)
    keep = np.isin(pid(k_box, v_box), pid(keys, vals))
    assert keep.sum() == len(keys)
    assert np.array_equal(keys, k_box[keep]) and np.array_equal(vals, v_box[keep])
    k_sup, v_sup = oracle.keys(g1, cams1, S(), (16, 16), support=True)
    assert np.isin(pid(k_sup, v_sup), pid(keys, vals)).all()
    f.close()


@pytest.mark.parametrize("which", ["tiny", "C2"])
def test_isotropic_gradients(raster, rctx, which):
    if which == "tiny":
        g, cams = scenes.tiny_scene(60, 451, 64, 48)
        target = scenes.perturbed(g, 451)
    else:
        g, cams, target = scenes.config2()
    g, target = scenes.isotropic_scene(g), scenes.isotropic_scene(target)
    say(f"isotropic gradients {which}")
    f = raster.Frame(rctx, raster.to_device(g), cams, S())
    f.bin_sort()
    f.render()
    c = cams[0]
    r = oracle.render(g, c, S())
    rt = oracle.render(target, c, S())
    _, gr, gd = oracle.loss(r["rgb"], r["depth"], rt["rgb"].astype(np.float32), rt["depth"].astype(np.float32), 0.5)
    ref = oracle.adjoint(g, c, S(), g_rgb=gr, g_depth=gd)
    t = lambda a: torch.as_tensor(a.astype(np.float32).reshape(-1)).cuda()
    grads = f.backward(t(gr), t(gd))
    assert "quats" not in grads
    gpu = grads_to_numpy(grads)
    rel = iso_rel_errors(gpu, ref)
    say(f"  relative errors {rel}")
    for k, v in rel.items():
        assert v <= GRAD_REL_TOL, (k, v)
    f.close()


def test_isotropic_autograd_without_quaternions(raster, rctx):
    g, cams = scenes.tiny_scene(40, 470, 64, 48)
    g = scenes.isotropic_scene(g)
    dev = raster.to_device(g)
    leaves = {k: dev[k].clone().requires_grad_(k != "uncert") for k in dev}
    rgb, depth, alpha, unc = raster.rasterize(rctx, leaves, cams, S())
    rng = np.random.default_rng(6)
    w = [torch.as_tensor(rng.standard_normal(x.shape).astype(np.float32)).cuda() for x in (rgb, depth, alpha, unc)]
    sum((wi * xi).sum() for wi, xi in zip(w, (rgb, depth, alpha, unc))).backward()
    H, W = 48, 64
    wn = [x.cpu().numpy().astype(np.float64) for x in w]
    ref = oracle.adjoint(g, cams[0], S(), g_rgb=wn[0].reshape(3, H, W), g_depth=wn[1].reshape(H, W),
                         g_alpha=wn[2].reshape(H, W), g_unc=wn[3].reshape(H, W))
    gpu = {k: leaves[k].grad.cpu().numpy() for k in ISO_GROUPS}
    for k, v in iso_rel_errors(gpu, ref).items():
        assert v <= GRAD_REL_TOL, (k, v)


def test_isotropic_scores(raster, rctx):
    g, cams = scenes.config3(n=100_000, n_views=4, width=160, height=120)
    g = scenes.isotropic_scene(g)
    say("isotropic scores")
    dev = raster.to_device(g)
    got = raster.score_views(rctx, dev, cams, S()).cpu().numpy()
    ref = oracle.score(g, cams, S())
    for v, c in enumerate(cams):
        assert abs(got[v] - ref[v]) <= SCORE_TOL_PER_PIXEL * c["width"] * c["height"]


def test_anisotropic_needs_quaternions(raster, rctx):
    g, cams = scenes.tiny_scene(5, 480, 32, 24)
    g = scenes.isotropic_scene(g)
    with pytest.raises(raster.RtgError):
        raster.Frame(rctx, raster.to_device(g), cams, dict(scenes.DEFAULT_SETTINGS))
    with pytest.raises(raster.RtgError):
        raster.Frame(rctx, raster.to_device(g), cams, S(isotropic=2))


def test_isotropic_graphs_match_eager(raster, rctx):
    # the captured mapping step and the captured scoring pipeline take the setting too
    g, cams, target = scenes.config4(n=60_000, n_views=2, width=256, height=144)
    g, target = scenes.isotropic_scene(g), scenes.isotropic_scene(target)
    dev = raster.to_device(g)
    timg, tf = raster.render(rctx, raster.to_device(target), cams, S(), want=("rgb", "depth"))
    tf.close()
    say("isotropic map graph vs eager")
    f = raster.Frame(rctx, dev, cams, S())
    f.bin_sort()
    out = f.render(("rgb", "depth"))
    loss, d_rgb, d_dep = f.loss(out["rgb"], out["depth"], timg["rgb"], timg["depth"], 0.5)
    ref = f.backward(d_rgb, d_dep)
    f.close()
    assert "quats" not in ref
    mg = raster.MapGraph(rctx, dev, cams, timg["rgb"], timg["depth"], 0.5, S())
    for rep in range(2):
        lv = mg.launch()
        assert mg.status()
        torch.cuda.synchronize()
        assert torch.equal(mg.rgb, out["rgb"]) and lv.item() == loss.item(), rep
    for k in ref:
        a = mg.grads[k].double().cpu().numpy()
        b = 2.0 * ref[k].double().cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-5 * (np.linalg.norm(b) + 1e-300), k
    mg.close()
    say("isotropic score graph vs eager")
    eager = raster.score_views(rctx, dev, cams, S()).cpu().numpy()
    gr = raster.ScoreGraph(rctx, dev, 4, 256, 144, S(), probe=cams)
    for rep in range(2):
        got = gr.launch(cams).cpu().numpy()
        assert gr.status()
        assert np.array_equal(got, eager), rep
    gr.close()
