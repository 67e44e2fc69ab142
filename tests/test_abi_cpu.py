"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/rtg.h, and validates arguments before
touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(rtg_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2409_18122_amd import _lib
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    from paper_2409_18122_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_default_settings(L):
    from paper_2409_18122_amd._lib import Settings
    s = Settings()
    assert L.rtg_default_settings(ctypes.byref(s)) == 0
    assert (s.tile_w, s.tile_h, s.batch) == (16, 16, 0)
    assert s.T_min == pytest.approx(1e-4) and s.alpha_max == pytest.approx(0.99)
    assert s.alpha_min == pytest.approx(1 / 255) and s.z_near == pytest.approx(0.2)
    assert s.isotropic == 0 and s.reserved == 0 and ctypes.sizeof(s) == 48
    assert L.rtg_default_settings(None) == -1


def test_no_device_is_reported(L):
    h = ctypes.c_void_p()
    n = L.rtg_device_count()
    if n == 0:
        assert L.rtg_create(0, ctypes.byref(h)) == -2
        assert b"no HIP device" in L.rtg_last_error()
    assert L.rtg_create(-1, ctypes.byref(h)) == -2
    assert L.rtg_create(0, None) == -1


def test_null_arguments_rejected_on_host(L):
    from paper_2409_18122_amd._lib import Camera, Gaussians, Settings
    out = ctypes.c_void_p()
    assert L.rtg_project(None, None, None, 1, None, ctypes.byref(out), None) == -1
    assert L.rtg_project(None, None, None, 1, None, None, None) == -1
    assert L.rtg_bin_sort(None, None, None, None) == -1
    assert L.rtg_render(None, None, None, None, None, None, None) == -1
    assert L.rtg_loss(None, None, None, None, None, None, 0.5, None, None, None, None) == -1
    assert L.rtg_loss_ssim(None, None, None, None, None, None, 1.0, 0.4, 0.1, None, None, None, None) == -1
    assert L.rtg_render_backward(None, None, None, None, None, None, None, None) == -1
    assert L.rtg_score_views(None, None, None, 1, None, None, 1, 0, None) == -1
    assert L.rtg_score_graph_create(None, None, 1, 1, 1, None, 0, None, 0, ctypes.byref(out), None) == -1
    assert L.rtg_score_graph_launch(None, None, 1, None, None) == -1
    assert L.rtg_score_graph_status(None) == -1
    assert L.rtg_frame_export(None, None, None, None, None, None) == -1
    assert L.rtg_frame_export_records(None, None, None, None, None, None, None, None, None, None) == -1
    info = (ctypes.c_int64 * 6)()
    assert L.rtg_frame_info(None, info) == -1
    assert L.rtg_autotune(None, None, None, 1, 0, None, None) == -1
    assert L.rtg_map_graph_create(None, None, None, 1, None, None, None, 0.5, None, None, None, None,
                                  ctypes.byref(out), None) == -1
    assert L.rtg_map_graph_create_ssim(None, None, None, 1, None, None, None, 1.0, 0.4, 0.1, None, None, None,
                                       None, ctypes.byref(out), None) == -1
    assert L.rtg_map_graph_launch(None, None) == -1
    assert L.rtg_map_graph_status(None) == -1
    assert L.rtg_view_utility(None, None, None, 1, None, 5.0, None, 1.0, None, None, None, None, None) == -1
    assert L.rtg_uncertainty_thresholds(None, None, 0, 0.5, None, None) == -1
    assert L.rtg_trajectory_select(None, None, None, 1, None, None, None) == -1
    assert L.rtg_uncertainty_update(None, 4, None, None, None, 0, None, None) == -1
    box = (ctypes.c_double * 6)(0, 0, 0, 10, 5, 2.5)
    assert L.rtg_region_utility(None, 4, None, None, box, 2.5, None, None, None, None) == -1
    assert L.rtg_collision_check(None, None, None, 4, 0.25, 3.0, None, None, None) == -1
    assert L.rtg_collision_check_noalloc(None, None, None, 4, 0.25, 3.0, None, None, None) == -1
    stats = (ctypes.c_int64 * 4)()
    assert L.rtg_frame_stats(None, None, stats, None) == -1
    from paper_2409_18122_amd._lib import ALLOC_FN, FREE_FN
    assert L.rtg_set_allocator(None, ALLOC_FN(), FREE_FN(), None) == -1
    assert L.rtg_timing_enable(None, 1) == -1
    assert L.rtg_timing_reset(None) == -1
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    assert L.rtg_timing_read(None, 0, ctypes.byref(ms), ctypes.byref(n)) == -1
    assert len(L.rtg_last_error()) > 0
    # destroy functions accept NULL
    L.rtg_destroy(None)
    L.rtg_frame_destroy(None)
    L.rtg_score_graph_destroy(None)
    L.rtg_map_graph_destroy(None)


def test_region_grid_on_host(L):
    # host-only: needs no device; same dims as the oracle's definition
    import oracle
    for box, size in (([0, 0, 0, 10, 5, 2.5], 2.5), ([-10, -10, 0, 10.1, 10, 4], 2.5), ([0, 0, 0, 1, 1, 1], 0.3)):
        b = (ctypes.c_double * 6)(*box)
        d = (ctypes.c_int32 * 3)()
        assert L.rtg_region_grid(b, size, d) == 0
        assert tuple(d) == oracle.region_grid(box, size)
    b = (ctypes.c_double * 6)(0, 0, 0, 0, 1, 1)
    d = (ctypes.c_int32 * 3)()
    assert L.rtg_region_grid(b, 2.5, d) == -1
    assert L.rtg_region_grid(None, 2.5, d) == -1
    b = (ctypes.c_double * 6)(0, 0, 0, 1, 1, 1)
    assert L.rtg_region_grid(b, 0.0, d) == -1


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2409_18122_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_librtg.so"))
    with pytest.raises(ImportError):
        _lib.lib()


def test_tune_key_separates_what_changes_the_work():
    import scenes
    from paper_2409_18122_amd import raster
    g, cams = scenes.config1()
    base = raster.tune_key(g, cams, 1, dict(scenes.DEFAULT_SETTINGS))
    assert base.startswith("host:mode1:")
    assert raster.tune_key(g, cams, 1, dict(scenes.DEFAULT_SETTINGS)) == base
    for k, v in (("alpha_min", 0.01), ("T_min", 1e-3), ("alpha_max", 0.9), ("eps2d", 0.1), ("isotropic", 1)):
        assert raster.tune_key(g, cams, 1, dict(scenes.DEFAULT_SETTINGS, **{k: v})) != base, k
    assert raster.tune_key(g, cams, 0, dict(scenes.DEFAULT_SETTINGS)) != base
    # tile, batch and capacity are what the tuner picks or bounds: not in the key
    assert raster.tune_key(g, cams, 1, dict(scenes.DEFAULT_SETTINGS, tile_w=32, tile_h=8, batch=64)) == base
