"""The seeded scene generators: determinism, shapes and value ranges."""
import numpy as np

from paper_1409_7474_amd import synth


def test_tiny_scene_deterministic_and_shaped():
    a = synth.scene_tiny(3)
    b = synth.scene_tiny(3)
    c = synth.scene_tiny(4)
    assert a.image.shape == (256, 256, 1) and a.image.dtype == np.float64
    assert synth.array_digest(a.image) == synth.array_digest(b.image)
    assert synth.array_digest(a.image) != synth.array_digest(c.image)
    assert a.init_region.sum() == 128 * 128
    assert a.init_region[64:192, 64:192].all()
    assert len(a.meta["rects"]) == 3
    for (y0, x0, rh, rw) in a.meta["rects"]:
        assert 20 <= rh <= 80 and 20 <= rw <= 80
        assert 0 <= y0 and y0 + rh <= 256 and 0 <= x0 and x0 + rw <= 256


def test_multiband_scene_ranges():
    sc = synth.scene_multiband(1, size=512)
    assert sc.image.shape == (512, 512, 4)
    assert sc.image.min() >= 0.0 and sc.image.max() <= 1.0
    assert sc.truth.any() and sc.init_edge.any()
    assert synth.array_digest(sc.image) == synth.array_digest(synth.scene_multiband(1, size=512).image)


def test_precision_scene_has_runway():
    sc = synth.scene_multiband(2, size=1024, n_roofs=20, n_roads=0, runway=True)
    assert sc.truth.mean() > 0.005


def test_batch_shapes_and_serving_trace():
    shapes = synth.batch_shapes(0)
    assert len(shapes) == 64
    assert all(512 <= h <= 2048 and 512 <= w <= 2048 for h, w in shapes)
    jobs = synth.serving_trace(0, n_jobs=200, qps=50.0)
    assert all(256 <= j.side <= 4096 and j.bands in (1, 4) and 100 <= j.iters <= 300 for j in jobs)
    arr = np.array([j.arrival_s for j in jobs])
    assert np.all(np.diff(arr) > 0)
    assert abs(arr[-1] / 200 - 1 / 50.0) < 0.01


def test_runway_sizes_are_given_at_8192():
    # the runway is 60-120 px wide and 2000-4000 px long at an 8192 px side,
    # scaled down (never up) for smaller scenes; its edge seeds lie inside it
    sc = synth.scene_multiband(4, size=2048, n_roofs=0, n_roads=0, runway=True, noise=0.0)
    cy, cx, theta, width, length = sc.meta["runway"]
    assert 60 / 4 <= width <= 120 / 4 and 2000 / 4 <= length <= 4000 / 4
    assert sc.init_edge.any() and not (sc.init_edge & (1 - sc.truth)).any()


def test_crop_scene_has_its_own_initial_curve():
    sc = synth.scene_multiband(1, size=512)
    c = synth.crop_scene(sc, 100, 50, 128, 200)
    assert c.image.shape == (128, 200, 4)
    assert np.array_equal(c.image, sc.image[100:228, 50:250])
    assert c.init_region.sum() == 64 * 100 and c.init_region[32:96, 50:150].all()
