"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Inputs are the seeded scenes of `scenes`; the oracle computes every expected
value on the CPU from the same float32 inputs.  Bars are in gpu_util.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import (GRAD_REL_TOL, SCORE_TOL_PER_PIXEL, assert_elementwise, assert_images_close, gpu_stack,
                      grad_rel_errors, grads_to_numpy)

pytestmark = pytest.mark.gpu

TILES = [(8, 8), (16, 16), (32, 8)]


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


def gpu_render(raster, rctx, scene, cams, settings):
    g = raster.to_device(scene)
    out, frame = raster.render(rctx, g, cams, settings)
    views = raster.unpack_images(out, cams)
    return [gpu_stack(v, c) for v, c in zip(views, cams)], frame, g, out


# ------------------------------------------------------------------ forward

def test_c1_forward(raster, rctx):
    g, cams = scenes.config1()
    say("C1 forward, 2000 Gaussians, 128x96, tile 16x16")
    imgs, frame, _, _ = gpu_render(raster, rctx, g, cams, S())
    r = oracle.render(g, cams[0], S())
    e, n_excl = assert_images_close(imgs[0], r, label="C1")
    say(f"C1 max err {e:.3g}, excluded {n_excl}, instances {frame.n_instances}")
    # the pairs are the support tiles (up to a tiny widening), never more than the box tiles
    assert oracle.count(g, cams[0], S(), support=True)[1] <= frame.n_instances <= oracle.count(g, cams[0], S())[1]


@pytest.mark.parametrize("n", [1, 2, 3, 10, 50, 500])
@pytest.mark.parametrize("size", [(32, 24), (64, 48)])
def test_tiny_scenes_vs_brute_force(raster, rctx, n, size):
    g, cams = scenes.tiny_scene(n, 100 + n, *size)
    r = oracle.render(g, cams[0], S(), mode="brute")
    for tile in TILES:
        say(f"tiny n={n} size={size} tile={tile}")
        imgs, _, _, _ = gpu_render(raster, rctx, g, cams, S(tile))
        assert_images_close(imgs[0], r, label=f"n={n} {size} {tile}")


BATCHES = {(8, 8): (0, 32, 64), (16, 16): (0, 32, 64, 128, 256), (32, 8): (0, 32, 64, 128, 256)}


def test_tile_and_batch_invariance(raster, rctx):
    g, cams = scenes.config1()
    outs = []
    for tile in TILES:
        for batch in BATCHES[tile]:
            say(f"C1 tile/batch invariance {tile} batch {batch}")
            imgs, _, _, _ = gpu_render(raster, rctx, g, cams, S(tile, batch=batch))
            outs.append(imgs[0])
    # the per-pixel sequence of splats does not depend on the tile or the
    # staging batch, so the float32 results are identical
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    # scores too (binary64 per-tile partials are summed in a fixed order per
    # tile size, so compare within a tile size)
    g3, cams3 = scenes.config3(n=20_000, n_views=3, width=96, height=64)
    dev3 = raster.to_device(g3)
    for tile in TILES:
        ref = None
        for batch in BATCHES[tile]:
            sc = raster.score_views(rctx, dev3, cams3, S(tile, batch=batch), persistent=True).cpu().numpy()
            if ref is None:
                ref = sc
            assert np.array_equal(sc, ref), (tile, batch)


def test_c2_forward_full_size(raster, rctx):
    g, cams, _ = scenes.config2()
    say("C2 forward, 200k Gaussians, 640x480")
    imgs, frame, _, _ = gpu_render(raster, rctx, g, cams, S())
    r = oracle.render(g, cams[0], S())
    e, n_excl = assert_images_close(imgs[0], r, label="C2")
    say(f"C2 max err {e:.3g}, excluded {n_excl}, instances {frame.n_instances}")


def test_multiview_forward(raster, rctx):
    g, cams, _ = scenes.config4(n=60_000, n_views=3, width=320, height=180)
    say("multi-view forward, 60k Gaussians, 3 views 320x180")
    imgs, _, _, _ = gpu_render(raster, rctx, g, cams, S())
    for v, c in enumerate(cams):
        r = oracle.render(g, c, S())
        assert_images_close(imgs[v], r, label=f"view {v}")


# --------------------------------------------------------------------- keys

def pair_ids(keys, vals):
    return (keys >> np.uint64(32)) << np.uint64(32) | vals.astype(np.uint64)


def test_sparse_visibility_records(raster, rctx):
    # one Gaussian in 40 in front of the camera, the rest behind it: 256
    # consecutive records then span ~10k Gaussians, more than a projection
    # block stages, so record emission takes its global-memory search
    g, cams = scenes.config1(n=100_000)
    g = {k: v.copy() for k, v in g.items()}
    behind = np.ones(100_000, bool)
    behind[::40] = False
    g["means"][2, behind] = -g["means"][2, behind]
    say("sparse visibility: 100k Gaussians, 2.5k in front")
    dev = raster.to_device(g)
    f = raster.Frame(rctx, dev, cams, S())
    f.bin_sort()
    keys, vals, _ = f.export()
    keys = keys.cpu().numpy().view(np.uint64)
    vals = vals.cpu().numpy().view(np.uint32)
    k_box, v_box = oracle.keys(g, cams, S(), (16, 16))
    keep = np.isin(pair_ids(k_box, v_box), pair_ids(keys, vals))
    assert keep.sum() == len(keys) > 0
    assert np.array_equal(keys, k_box[keep]) and np.array_equal(vals, v_box[keep])
    assert np.all(np.isin(vals, np.nonzero(~behind)[0]))
    out = f.render()
    f.close()
    imgs = raster.unpack_images(out, cams)
    r = oracle.render(g, cams[0], S())
    assert_images_close(gpu_stack(imgs[0], cams[0]), r, label="sparse")


@pytest.mark.parametrize("tile", TILES)
def test_keys_bit_exact(raster, rctx, tile):
    g, cams = scenes.config1(n=1500)
    # duplicates create equal depth keys; they must come out in index order
    idx = np.concatenate([np.arange(1500), np.arange(0, 1500, 29)])
    g = scenes.subset(g, idx)
    g3, cams3 = scenes.config3(n=20_000, n_views=3, width=96, height=64)
    # elongated, randomly rotated splats close to the camera, mixed resolutions
    g5, cams5 = scenes.config5(n=150_000, n_views=6)
    for scene, cs, label in ((g, cams, "C1+dups"), (g3, cams3, "3 views"), (g5, cams5, "C5-like 6 views")):
        say(f"keys {label} tile {tile}")
        dev = raster.to_device(scene)
        f = raster.Frame(rctx, dev, cs, S(tile))
        f.bin_sort()
        keys, vals, ranges = f.export()
        keys = keys.cpu().numpy().view(np.uint64)
        vals = vals.cpu().numpy().view(np.uint32)
        # a Gaussian is binned to the tiles its support meets (a conservative
        # binary32 test, so a few percent more): every exact support pair is
        # there, every pair is a pixel-box pair, and the list is the box list
        # restricted to its pairs (the same keys in the same order)
        k_box, v_box = oracle.keys(scene, cs, S(tile), tile)
        k_sup, v_sup = oracle.keys(scene, cs, S(tile), tile, support=True)
        got = pair_ids(keys, vals)
        assert len(np.unique(got)) == len(got), label
        keep = np.isin(pair_ids(k_box, v_box), got)
        assert keep.sum() == len(got), (label, keep.sum(), len(got))
        assert np.array_equal(keys, k_box[keep]), label
        assert np.array_equal(vals, v_box[keep]), label
        assert np.isin(pair_ids(k_sup, v_sup), got).all(), label
        say(f"keys {label}: box {len(k_box)} support {len(k_sup)} gpu {len(keys)}")
        assert len(keys) <= len(k_sup) + max(8, len(k_sup) // 20), label
        # tile ranges partition the sorted list
        rg = ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
        tiles = (keys >> np.uint64(32)).astype(np.int64)
        for t in np.unique(tiles)[:200]:
            pos = np.nonzero(tiles == t)[0]
            assert rg[t, 0] == pos[0] and rg[t, 1] == pos[-1] + 1
        f.close()


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_keys_tall_records(raster, rctx, tile):
    # five needle-thin, slightly tilted Gaussians spanning the whole height of
    # a 1024 x 16384 view: each record meets ~2 tiles on each of up to 2048
    # tile rows, so the pair-emission blocks that hold parts of two records
    # have more support rows than they tabulate and walk them per thread
    n = 5
    rng = np.random.default_rng(17)
    g = {"means": np.zeros((3, n), np.float32),
         "log_scales": np.tile(np.array([[-3.5], [2.0], [-3.5]], np.float32), (1, n)),
         "quats": np.zeros((4, n), np.float32), "opacity": np.full(n, 0.9, np.float32),
         "colors": rng.random((3, n)).astype(np.float32), "uncert": rng.random(n).astype(np.float32)}
    ang = np.array([0.004, -0.006, 0.01, 0.0025, -0.012])
    g["quats"][0] = np.cos(ang / 2)
    g["quats"][3] = np.sin(ang / 2)  # about the optical axis
    g["means"][0] = np.array([-0.8, -0.3, 0.1, 0.4, 0.9], np.float32)
    g["means"][2] = np.array([3.0, 3.2, 2.9, 3.1, 3.05], np.float32)
    cams = [scenes.make_camera(1024, 16384, 1000.0, 1000.0, 512.0, 8192.0)]
    say(f"tall records, tile {tile}")
    dev = raster.to_device(g)
    f = raster.Frame(rctx, dev, cams, S(tile))
    f.bin_sort()
    keys, vals, _ = f.export()
    f.close()
    keys = keys.cpu().numpy().view(np.uint64)
    vals = vals.cpu().numpy().view(np.uint32)
    k_box, v_box = oracle.keys(g, cams, S(tile), tile)
    k_sup, v_sup = oracle.keys(g, cams, S(tile), tile, support=True)
    got = pair_ids(keys, vals)
    keep = np.isin(pair_ids(k_box, v_box), got)
    assert keep.sum() == len(got) and len(np.unique(got)) == len(got)
    assert np.array_equal(keys, k_box[keep]) and np.array_equal(vals, v_box[keep])
    assert np.isin(pair_ids(k_sup, v_sup), got).all()
    say(f"tall records {tile}: box {len(k_box)} support {len(k_sup)} gpu {len(keys)}")
    assert len(keys) <= len(k_sup) + max(8, len(k_sup) // 20)


# ---------------------------------------------------------- loss, backward

def test_c2_loss_parity(raster, rctx):
    g, cams, target = scenes.config2()
    say("C2 loss")
    dev = raster.to_device(g)
    out, frame = raster.render(rctx, dev, cams, S())
    rt = oracle.render(target, cams[0], S())
    trgb = torch.as_tensor(rt["rgb"].astype(np.float32).reshape(-1)).cuda()
    tdep = torch.as_tensor(rt["depth"].astype(np.float32).reshape(-1)).cuda()
    loss, d_rgb, d_dep = frame.loss(out["rgb"], out["depth"], trgb, tdep, 0.5)
    L_ref, gr_ref, gd_ref = oracle.loss(out["rgb"].cpu().numpy().reshape(3, 480, 640),
                                        out["depth"].cpu().numpy().reshape(480, 640),
                                        rt["rgb"].astype(np.float32), rt["depth"].astype(np.float32), 0.5)
    assert abs(loss.item() - L_ref) <= 1e-6 * abs(L_ref)
    np.testing.assert_allclose(d_rgb.cpu().numpy().reshape(3, 480, 640), gr_ref, rtol=1e-6, atol=0)
    np.testing.assert_allclose(d_dep.cpu().numpy().reshape(480, 640), gd_ref, rtol=1e-6, atol=0)


def _backward_parity(raster, rctx, g, cams, target, tile=(16, 16), label=""):
    dev = raster.to_device(g)
    f = raster.Frame(rctx, dev, cams, S(tile))
    f.bin_sort()
    f.render()
    ref = {k: np.zeros_like(np.asarray(g[k], np.float64)) for k in
           ("means", "log_scales", "quats", "opacity", "colors")}
    touched = np.zeros(scenes.n_gaussians(g), bool)
    d_rgb_all, d_dep_all, d_a_all, d_u_all = [], [], [], []
    rng = np.random.default_rng(7)
    for c in cams:
        r = oracle.render(g, c, S(tile))
        rt = oracle.render(target, c, S(tile))
        _, gr, gd = oracle.loss(r["rgb"], r["depth"], rt["rgb"].astype(np.float32),
                                rt["depth"].astype(np.float32), 0.5)
        H, W = r["depth"].shape
        ga = rng.standard_normal((H, W)) * 1e-6
        gu = rng.standard_normal((H, W)) * 1e-6
        a = oracle.adjoint(g, c, S(tile), g_rgb=gr, g_depth=gd, g_alpha=ga, g_unc=gu, tile=tile)
        for k in ref:
            ref[k] += a[k]
        touched |= a["touched"]
        d_rgb_all.append(gr.astype(np.float32).reshape(-1))
        d_dep_all.append(gd.astype(np.float32).reshape(-1))
        d_a_all.append(ga.astype(np.float32).reshape(-1))
        d_u_all.append(gu.astype(np.float32).reshape(-1))
    t = lambda xs: torch.as_tensor(np.concatenate(xs)).cuda()
    say(f"backward {label}")
    grads = f.backward(t(d_rgb_all), t(d_dep_all), t(d_a_all), t(d_u_all))
    gpu = grads_to_numpy(grads)
    rel = grad_rel_errors(gpu, ref)
    say(f"{label} relative errors {rel}")
    for k, v in rel.items():
        assert v <= GRAD_REL_TOL, (label, k, v)
    n_excl = assert_elementwise(gpu, ref, touched, label)
    say(f"{label} element-wise bar met; {n_excl} of {touched.size} Gaussians excluded (near-threshold decisions)")
    return rel, n_excl


def test_c2_gradients_full_size(raster, rctx):
    g, cams, target = scenes.config2()
    _backward_parity(raster, rctx, g, cams, target, label="C2")


@pytest.mark.parametrize("tile", TILES)
def test_multiview_gradients(raster, rctx, tile):
    g, cams, target = scenes.config4(n=40_000, n_views=3, width=256, height=144)
    _backward_parity(raster, rctx, g, cams, target, tile=tile, label=f"3 views {tile}")


def test_tiny_gradients(raster, rctx):
    for n in (1, 5, 50):
        g, cams = scenes.tiny_scene(n, 300 + n, 48, 32)
        target = scenes.perturbed(g, 300 + n)
        _backward_parity(raster, rctx, g, cams, target, label=f"tiny n={n}")


def test_autograd_function(raster, rctx):
    g, cams = scenes.tiny_scene(40, 77, 64, 48)
    dev = raster.to_device(g)
    leaves = {k: dev[k].clone().requires_grad_(k != "uncert") for k in dev}
    rgb, depth, alpha, unc = raster.rasterize(rctx, leaves, cams, S())
    rng = np.random.default_rng(5)
    w = [torch.as_tensor(rng.standard_normal(x.shape).astype(np.float32)).cuda() for x in (rgb, depth, alpha, unc)]
    say("autograd backward")
    total = sum((wi * xi).sum() for wi, xi in zip(w, (rgb, depth, alpha, unc)))
    total.backward()
    H, W = 48, 64
    wn = [x.cpu().numpy().astype(np.float64) for x in w]
    ref = oracle.adjoint(g, cams[0], S(), g_rgb=wn[0].reshape(3, H, W), g_depth=wn[1].reshape(H, W),
                         g_alpha=wn[2].reshape(H, W), g_unc=wn[3].reshape(H, W))
    gpu = {k: leaves[k].grad.cpu().numpy() for k in ("means", "log_scales", "quats", "opacity", "colors")}
    rel = grad_rel_errors(gpu, ref)
    for k, v in rel.items():
        assert v <= GRAD_REL_TOL, (k, v)


# ------------------------------------------------------------------ scoring

def test_c3_scores(raster, rctx):
    g, cams = scenes.config3()
    say("C3 scoring, 500k Gaussians, 64 views 320x240")
    dev = raster.to_device(g)
    batched = raster.score_views(rctx, dev, cams, S(), persistent=True).cpu().numpy()
    plain = raster.score_views(rctx, dev, cams, S(), persistent=False).cpu().numpy()
    # same kernels, same per-tile sums, same fixed-order reductions
    assert np.array_equal(batched, plain)
    sample = list(range(0, 64, 4))  # 16 of the 64 views
    refs = oracle.score(g, [cams[v] for v in sample], S())
    for v, ref in zip(sample, refs):
        P = cams[v]["width"] * cams[v]["height"]
        say(f"view {v}: gpu {batched[v]:.6f} oracle {ref:.6f} rel {abs(batched[v] - ref) / max(ref, 1e-30):.2e}")
        assert abs(batched[v] - ref) <= SCORE_TOL_PER_PIXEL * P
    # batch invariance: a view scored alone equals its score inside the batch
    alone = raster.score_views(rctx, dev, [cams[17]], S(), persistent=True).cpu().numpy()
    assert alone[0] == batched[17]


def test_c3_binary_j_scores(raster, rctx):
    # the binary-J trace: per pixel the sum of u over the contributing
    # Gaussians.  A termination decision that flips between binary32 and
    # binary64 moves a pixel by one u (<= 1); such flips are rare (~1e-5 of
    # pixels), inside the per-pixel tolerance
    g, cams = scenes.config3(n=200_000, n_views=16)
    say("C3-like binary-J scoring, 200k Gaussians, 16 views 320x240")
    dev = raster.to_device(g)
    batched = raster.score_views(rctx, dev, cams, S(), persistent=True, mode="binary").cpu().numpy()
    plain = raster.score_views(rctx, dev, cams, S(), persistent=False, mode="binary").cpu().numpy()
    assert np.array_equal(batched, plain)
    rendered = raster.score_views(rctx, dev, cams, S(), persistent=True).cpu().numpy()
    assert np.all(batched >= rendered)
    ref = oracle.score(g, [cams[v] for v in (0, 7, 15)], S(), mode=1)
    for j, v in enumerate((0, 7, 15)):
        P = cams[v]["width"] * cams[v]["height"]
        say(f"binary view {v}: gpu {batched[v]:.4f} oracle {ref[j]:.4f} diff {abs(batched[v] - ref[j]):.3g}")
        assert abs(batched[v] - ref[j]) <= SCORE_TOL_PER_PIXEL * P
    # captured graph, same mode
    gr = raster.ScoreGraph(rctx, dev, 16, 320, 240, S(), probe=cams, mode="binary")
    got = gr.launch(cams).cpu().numpy()
    assert gr.status() and np.array_equal(got, batched)
    gr.close()
    # a mode other than 0 or 1 is an argument error
    import ctypes
    st = raster.make_settings(S())
    out = torch.empty(16, device="cuda", dtype=torch.float64)
    rc = raster.lib().rtg_score_views(rctx.handle, ctypes.byref(raster.make_gaussians(dev)),
                                      raster.make_cameras(cams), 16, ctypes.byref(st), out.data_ptr(), 1, 2, None)
    assert rc == -1


def test_score_graph_replay_uneven(raster, rctx):
    g, cams = scenes.config5(n=300_000, n_views=48)
    dev = raster.to_device(g)
    say("graph: create with probe views")
    gr = raster.ScoreGraph(rctx, dev, 48, 640, 480, S(), probe=cams)
    eager = raster.score_views(rctx, dev, cams, S(), persistent=True).cpu().numpy()
    for rep, sel in enumerate((slice(0, 48), slice(5, 37), slice(0, 48))):
        cs = cams[sel]
        say(f"graph replay {rep} with {len(cs)} views")
        got = gr.launch(cs).cpu().numpy()
        assert gr.status()
        assert np.array_equal(got, eager[sel]), rep
        torch.cuda.synchronize()
    for v in (3, 20):
        ref = oracle.score(g, [cams[v]], S())[0]
        P = cams[v]["width"] * cams[v]["height"]
        assert abs(eager[v] - ref) <= SCORE_TOL_PER_PIXEL * P
    gr.close()


def test_score_graph_capacity_flag(raster, rctx):
    g, cams = scenes.config3(n=50_000, n_views=4, width=160, height=120)
    dev = raster.to_device(g)
    say("graph with tiny capacity")
    gr = raster.ScoreGraph(rctx, dev, 4, 160, 120, S(max_instances=64))
    gr.launch(cams)
    assert gr.status() is False  # overflow reported, kernels exited cleanly
    gr.close()


# --------------------------------------------------------------- edge cases

def test_edge_cases(raster, rctx):
    base, cams = scenes.tiny_scene(30, 9, 64, 48)
    # NaN geometry, zero quaternion, behind the camera, too faint: all culled
    g = {k: v.copy() for k, v in base.items()}
    g["means"][1, 0] = np.nan
    g["quats"][:, 1] = 0.0
    g["means"][2, 2] = -1.0
    g["opacity"][3] = 0.001
    say("edge: culled Gaussians")
    imgs, frame, _, _ = gpu_render(raster, rctx, g, cams, S())
    r = oracle.render(g, cams[0], S())
    assert_images_close(imgs[0], r, label="culled")
    assert frame.info()["records"] == int(oracle.project(g, cams[0], S())["valid"].sum())
    # nothing visible
    g2 = {k: v.copy() for k, v in base.items()}
    g2["means"][2, :] = -5.0
    say("edge: nothing visible")
    imgs, frame, _, _ = gpu_render(raster, rctx, g2, cams, S())
    assert frame.n_instances == 0 and not imgs[0].any()
    # one Gaussian covering the whole image (many tiles)
    big = scenes.subset(base, [0])
    big["means"][:, 0] = [0.0, 0.0, 2.0]
    big["log_scales"][:, 0] = [0.5, 0.5, 0.5]
    big["opacity"][0] = 0.8
    say("edge: one huge Gaussian")
    imgs, frame, _, _ = gpu_render(raster, rctx, big, cams, S((8, 8)))
    assert frame.n_instances == 8 * 6
    assert_images_close(imgs[0], oracle.render(big, cams[0], S()), label="huge")
    # empty map
    empty = scenes.subset(base, np.array([], np.int64))
    say("edge: empty map")
    imgs, frame, _, _ = gpu_render(raster, rctx, empty, cams, S())
    assert frame.n_instances == 0 and not imgs[0].any()
    dev = raster.to_device(empty)
    s = raster.score_views(rctx, dev, cams, S()).cpu().numpy()
    assert s[0] == 0.0
    # ragged image size (not a multiple of any tile)
    g3, cams3 = scenes.tiny_scene(200, 11, 37, 29)
    for tile in TILES:
        say(f"edge: ragged 37x29 tile {tile}")
        imgs, _, _, _ = gpu_render(raster, rctx, g3, cams3, S(tile))
        assert_images_close(imgs[0], oracle.render(g3, cams3[0], S(), mode="brute"), label="ragged")


def test_invalid_arguments(raster, rctx):
    g, cams = scenes.tiny_scene(5, 1, 32, 24)
    dev = raster.to_device(g)
    with pytest.raises(raster.RtgError):
        raster.Frame(rctx, dev, cams, S((16, 8)))  # tile not supported
    bad = [dict(cams[0], width=0)]
    with pytest.raises(raster.RtgError):
        raster.Frame(rctx, dev, bad, S())
    nan = [dict(cams[0], fx=float("nan"))]
    with pytest.raises(raster.RtgError):
        raster.Frame(rctx, dev, nan, S())
    for tile, batch in (((16, 16), 48), ((16, 16), 512), ((8, 8), 128), ((16, 16), -1)):
        with pytest.raises(raster.RtgError):
            raster.Frame(rctx, dev, cams, S(tile, batch=batch))


# ------------------------------------------------------- captured mapping step

def test_map_graph_matches_eager(raster, rctx):
    g, cams, target = scenes.config4(n=80_000, n_views=2, width=320, height=180)
    dev = raster.to_device(g)
    tdev = raster.to_device(target)
    timg, tf = raster.render(rctx, tdev, cams, S(), want=("rgb", "depth"))
    tf.close()
    say("map graph: eager reference step")
    f = raster.Frame(rctx, dev, cams, S())
    f.bin_sort()
    out = f.render(("rgb", "depth"))
    loss, d_rgb, d_dep = f.loss(out["rgb"], out["depth"], timg["rgb"], timg["depth"], 0.5)
    ref = f.backward(d_rgb, d_dep)
    f.close()
    say("map graph: capture and replay 3 times")
    mg = raster.MapGraph(rctx, dev, cams, timg["rgb"], timg["depth"], 0.5, S())
    for rep in range(3):
        l = mg.launch()
        assert mg.status()
        torch.cuda.synchronize()
        # eager work between replays
        _ = (dev["means"] * 1.0).sum().item()
        assert torch.equal(mg.rgb, out["rgb"]) and torch.equal(mg.depth, out["depth"]), rep
        assert l.item() == loss.item(), rep
    for k in ref:
        a = mg.grads[k].double().cpu().numpy()
        b = 3.0 * ref[k].double().cpu().numpy()
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300)
        assert rel <= 1e-5, (k, rel)
    mg.close()


def test_map_graph_capacity_overflow_is_reported(raster, rctx):
    g, cams, target = scenes.config4(n=20_000, n_views=1, width=160, height=90)
    dev = raster.to_device(g)
    tdev = raster.to_device(target)
    timg, tf = raster.render(rctx, tdev, cams, S(), want=("rgb", "depth"))
    tf.close()
    say("map graph with a too small pair capacity")
    mg = raster.MapGraph(rctx, dev, cams, timg["rgb"], timg["depth"], 0.5, S(max_instances=100))
    mg.launch()
    assert mg.status() is False
    for k in mg.grads:
        assert not mg.grads[k].any()  # kernels past the overflow exited: nothing added
    mg.close()
