"""The C ABI's contracts beyond the images: the record export against the
oracle's projection, overflow reporting of the captured graphs, and counts
beyond the 32-bit list offsets."""
import numpy as np
import pytest
import torch

import oracle
import scenes

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("which", ["C1", "3 views"])
def test_export_records_match_oracle_projection(raster, rctx, which):
    if which == "C1":
        g, cams = scenes.config1()
    else:
        g, cams = scenes.config3(n=20_000, n_views=3, width=96, height=64)
    say(f"export records {which}")
    dev = raster.to_device(g)
    f = raster.Frame(rctx, dev, cams, S())
    f.bin_sort()
    rec = {k: v.cpu().numpy() for k, v in f.export_records().items()}
    f.close()
    gid = rec["gid"].view(np.uint32).astype(np.int64)
    view = rec["view"].view(np.uint32).astype(np.int64)
    # Gaussian-major, views ascending within a Gaussian
    order = gid * len(cams) + view
    assert np.all(np.diff(order) > 0)
    n_box_edge = 0
    for v, cam in enumerate(cams):
        p = oracle.project(g, cam, S())
        sel = view == v
        ids = gid[sel]
        assert np.array_equal(ids, np.nonzero(p["valid"])[0]), v
        assert np.array_equal(rec["depth_bits"][sel].view(np.uint32), p["depth_bits"][ids]), v
        np.testing.assert_allclose(rec["mean2d"][:, sel], p["mean2d"][:, ids], rtol=0, atol=1e-9)
        scale = np.abs(p["conic"][:, ids]).max(axis=0)
        assert np.all(np.abs(rec["conic"][:, sel] - p["conic"][:, ids]) <= 1e-9 * scale), v
        # the pixel box is exact; an edge may differ only where mu +- h lies
        # within 1e-6 px of a pixel centre (either rounding is then correct)
        box = rec["pbox"][:, sel]
        ref = p["box"][:, ids]
        diff = np.any(box != ref, axis=0)
        if diff.any():
            m, h = p["mean2d"][:, ids[diff]], p["half"][:, ids[diff]]
            edges = np.concatenate([m - h, m + h])
            near = np.min(np.abs(edges - np.round(edges)), axis=0) <= 1e-6
            assert near.all(), (v, np.nonzero(diff)[0][~near][:5])
            n_box_edge += int(diff.sum())
        assert np.all(rec["ntiles"][sel] >= 1)
    say(f"{which}: {len(gid)} records, {n_box_edge} box edges on a pixel centre")


def test_score_graph_overflow_makes_launch_fail(raster, rctx):
    g, cams = scenes.config3(n=50_000, n_views=4, width=160, height=120)
    dev = raster.to_device(g)
    say("score graph overflow: tiny pair capacity")
    gr = raster.ScoreGraph(rctx, dev, 4, 160, 120, S(max_instances=64))
    first = gr.launch(cams)
    assert gr.status() is False
    # the overflowed replay's scores are NaN, not stale
    assert torch.isnan(first).all()
    # the overflow is sticky and the next launch reports it without replaying
    with pytest.raises(raster.RtgError) as e:
        gr.launch(cams)
    assert e.value.code == raster.RTG_ERR_CAPACITY
    assert gr.status() is False
    gr.close()
    # a graph with room: launches back to back never report an error
    say("score graph without overflow: 6 launches back to back")
    gr = raster.ScoreGraph(rctx, dev, 4, 160, 120, S(), probe=cams)
    ref = raster.score_views(rctx, dev, cams, S()).cpu().numpy()
    outs = [gr.launch(cams) for _ in range(6)]
    assert gr.status()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), ref)
    gr.close()


def test_map_graph_overflow_makes_launch_fail(raster, rctx):
    g, cams, target = scenes.config4(n=20_000, n_views=1, width=160, height=90)
    dev = raster.to_device(g)
    tdev = raster.to_device(target)
    timg, tf = raster.render(rctx, tdev, cams, S(), want=("rgb", "depth"))
    tf.close()
    say("map graph overflow: tiny pair capacity")
    mg = raster.MapGraph(rctx, dev, cams, timg["rgb"], timg["depth"], 0.5, S(max_instances=100))
    mg.launch()
    assert mg.status() is False
    with pytest.raises(raster.RtgError) as e:
        mg.launch()
    assert e.value.code == raster.RTG_ERR_CAPACITY
    for k in mg.grads:
        assert not mg.grads[k].any()
    mg.close()


def test_pairs_beyond_32_bit_offsets_are_refused(raster, rctx):
    # 600 Gaussians that each cover a whole 16384 x 16384 view binned in 8x8
    # tiles: 600 x 2048^2 = 2.5e9 (tile, Gaussian) pairs, more than 2^31 - 1
    n = 600
    rng = np.random.default_rng(11)
    g = {"means": np.zeros((3, n), np.float32), "log_scales": np.full((3, n), 1.5, np.float32),
         "quats": np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
         "opacity": np.full(n, 0.8, np.float32), "colors": rng.random((3, n)).astype(np.float32),
         "uncert": rng.random(n).astype(np.float32)}
    g["means"][2] = np.linspace(2.0, 3.0, n, dtype=np.float32)
    cam = scenes.make_camera(16384, 16384, 8000.0, 8000.0, 8192.0, 8192.0)
    say("2.5e9 pairs on one 16384x16384 view, tile 8x8")
    dev = raster.to_device(g)
    f = raster.Frame(rctx, dev, [cam], S((8, 8)))
    assert f.info()["records"] == n
    with pytest.raises(raster.RtgError) as e:
        f.bin_sort()
    assert e.value.code == raster.RTG_ERR_UNSUPPORTED
    f.close()
    # half as many Gaussians (1.26e9 pairs, 20 GB of pair lists) still bin,
    # with every pair counted
    say("1.26e9 pairs: binned")
    half = {k: np.ascontiguousarray(v[..., :300]) for k, v in g.items()}
    f = raster.Frame(rctx, raster.to_device(half), [cam], S((8, 8)))
    assert f.info()["records"] == 300
    assert f.bin_sort() == 300 * 2048 * 2048
    f.close()
