"""GPU (HIP, gfx950) parity with the FP64 oracle, through the C ABI.

Bars:
  * one step from identical state: every binary decision equal to the
    oracle's except where the oracle's update value |u| is below
    1e-5 * max(1, dt) (a sign FP32 cannot decide like FP64; such pixels are
    counted and must stay below 1e-4 of the image), and the LSF after the step
    within 1e-5 max-abs outside the Gaussian footprint of those pixels;
  * whole runs: at most 1e-4 of the final mask's pixels differ in sign.
Inputs are handed to the oracle exactly as the GPU received them (the float32
or float16 values, promoted to float64).
"""
import numpy as np
import pytest

import oracle
from paper_1409_7474_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from parity_helpers import LSF_TOL, MASK_TOL, _as_gpu, _make, check_normaliser, mask_disagreement, one_step  # noqa: E402,F401


# ------------------------------------------------------------ one step ---

@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_tiny_workload_one_step_parity(dev, seed):
    """256 x 256 x 1, three rectangles, sigma 1 / 7 x 7, dt 15: every one of
    the first 12 iterations (the first starts from the binary LSF of eq. (13))."""
    sc = synth.scene_tiny(seed)
    img, img64 = _as_gpu(sc.image, dev)
    job = _make(dev, img, sc.init_region, sigma=1.0, ksize=7)
    for it in range(12):
        err, amb, ref = one_step(job, img64, sigma=1.0, ts=7)
        assert err <= LSF_TOL, (seed, it, err)
        st = job.stats()
        np.testing.assert_allclose(st["c_plus"], ref.c_plus, rtol=2e-6, atol=1e-7)
        np.testing.assert_allclose(st["c_minus"], ref.c_minus, rtol=2e-6, atol=1e-7)
        assert st["M"] == pytest.approx(ref.M, rel=5e-6)


@pytest.mark.parametrize("bands,h,w,ts,sigma", [
    (4, 200, 333, 11, 1.5), (2, 97, 130, 7, 1.0), (3, 150, 77, 13, 2.0), (1, 65, 257, 9, 3.0),
    (4, 130, 200, 31, 5.0), (4, 180, 250, 15, 2.5), (1, 300, 420, 9, 1.5),
])
def test_multiband_ragged_one_step_parity(dev, bands, h, w, ts, sigma):
    sc = synth.scene_multiband(7, size=max(h, w), bands=bands, n_roofs=12, n_roads=2, height=h, width=w)
    img, img64 = _as_gpu(sc.image, dev)
    job = _make(dev, img, sc.init_region, sigma=sigma, ksize=ts)
    for it in range(6):
        err, amb, ref = one_step(job, img64, sigma=sigma, ts=ts)
        assert err <= LSF_TOL, (it, err)
        # the normaliser of eq. (17) (pruned block scan for B > 1) is the full max
        check_normaliser(job.stats(), img64, ref.M)


@pytest.mark.parametrize("h,w,ts", [(2, 2, 3), (3, 5, 3), (5, 7, 31), (2, 100, 11), (40, 33, 7), (33, 65, 9),
                                    (31, 2, 5)])
def test_degenerate_shapes_one_step_parity(dev, h, w, ts):
    """Images smaller than the template, one-pixel tails in the last bit word
    and tile, two-pixel extents (one-sided gradients on both sides)."""
    rng = np.random.default_rng(h * 1000 + w)
    image = rng.random((h, w, 2))
    mask = (rng.random((h, w)) > 0.5).astype(np.uint8)
    mask[0, 0], mask[-1, -1] = 1, 0
    img, img64 = _as_gpu(image, dev)
    job = _make(dev, img, mask, sigma=1.0, ksize=ts)
    for it in range(4):
        err, _, _ = one_step(job, img64, sigma=1.0, ts=ts)
        assert err <= LSF_TOL, (it, err)


def test_edge_term_one_step_parity(dev):
    sc = synth.scene_multiband(3, size=300, bands=4, n_roofs=10, n_roads=2, height=260, width=300)
    img, img64 = _as_gpu(sc.image, dev)
    g = oracle.edge_map(img64, 1.0, 9, 255.0)
    job = _make(dev, img, sc.init_edge, term="edge", sigma=1.5, ksize=11, sigma_img=1.0, ksize_img=9)
    for it in range(8):
        err, amb, _ = one_step(job, img64, term="edge", sigma=1.5, ts=11, g=g)
        assert err <= LSF_TOL, (it, err)


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_half_precision_inputs(dev, dtype):
    sc = synth.scene_multiband(4, size=160, bands=4, n_roofs=6, n_roads=1)
    img, img64 = _as_gpu(sc.image, dev, dtype=dtype)
    job = _make(dev, img, sc.init_region, sigma=1.0, ksize=7)
    for it in range(4):
        err, _, _ = one_step(job, img64, sigma=1.0, ts=7)
        assert err <= LSF_TOL


# --------------------------------------------------------- trajectories ---

@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_tiny_workload_trajectory(dev, seed):
    """Tiny workload, 100 iterations: final masks agree within 1e-4."""
    sc = synth.scene_tiny(seed)
    img, img64 = _as_gpu(sc.image, dev)
    job = _make(dev, img, sc.init_region, sigma=1.0, ksize=7)
    job.run(100)
    got = job.mask().cpu().numpy()
    ref = oracle.run(img64, sc.init_region, iters=100, sigma=1.0, ts=7)
    assert mask_disagreement(got, ref.mask) <= MASK_TOL
    assert job.stats()["iters_done"] == 100


def test_multiband_trajectory_region_and_edge(dev):
    sc = synth.scene_multiband(5, size=384, bands=4, n_roofs=10, n_roads=2)
    img, img64 = _as_gpu(sc.image, dev)
    for term, mask in (("region", sc.init_region), ("edge", sc.init_edge)):
        job = _make(dev, img, mask, term=term, sigma=1.5, ksize=11)
        job.run(60)
        got = job.mask().cpu().numpy()
        ref = oracle.run(img64, mask, term=term, iters=60, sigma=1.5, ts=11)
        assert mask_disagreement(got, ref.mask) <= MASK_TOL, term


def test_noise_free_rectangle_exact_and_stops(dev):
    image, truth = synth.rectangle_scene()
    img, img64 = _as_gpu(image, dev)
    init = synth.centred_square(256, 256, 128, 128)
    job = _make(dev, img, init, sigma=1.0, ksize=7)
    job.run(300, stop_when_unchanged=True)
    st = job.stats()
    ref = oracle.run(img64, init, iters=300, stop_unchanged=True)
    assert st["converged"] and st["iters_done"] == ref.iters_done
    np.testing.assert_array_equal(job.mask().cpu().numpy(), truth)


# ------------------------------------------------------- state handling ---

def test_initial_lsf_and_mask_roundtrip(dev):
    sc = synth.scene_tiny(1, size=100, n_rects=2)
    img, _ = _as_gpu(sc.image, dev)
    job = _make(dev, img, sc.init_region)
    np.testing.assert_array_equal(job.mask().cpu().numpy(), sc.init_region)
    np.testing.assert_array_equal(job.lsf().cpu().numpy(), np.where(sc.init_region > 0, 1.0, -1.0))
    st = job.stats()
    assert st["iters_done"] == 0 and st["n_plus"] == int(sc.init_region.sum())


@pytest.mark.parametrize("w", [2, 15, 16, 17, 31, 33, 100, 129])
@pytest.mark.parametrize("off", [0, 1, 5])
def test_mask_packing_any_width_and_alignment(dev, w, off):
    """Mask -> bits (lse_init), bits -> mask (lse_mask) and sign(lsf) -> bits
    (lse_set_lsf) at widths around the 16-pixel segments and 32-pixel words
    of the packing kernels, with every buffer at an element offset that
    breaks 16-byte alignment (off > 0): nonzero bytes are inside, and
    lsf >= 0 is inside (eq. (15)'s tie rule, -0.0 included)."""
    h = 9
    rng = np.random.default_rng(100 * w + off)
    m = ((rng.random((h, w)) < 0.5) * rng.integers(1, 256, (h, w))).astype(np.uint8)
    img = torch.tensor(rng.random((h, w, 1), dtype=np.float32), device=dev)

    mbuf = torch.zeros(h * w + 64, dtype=torch.uint8, device=dev)
    mview = mbuf[off:off + h * w].view(h, w)
    mview.copy_(torch.tensor(m, device=dev))
    from paper_1409_7474_amd import lse
    job = lse.LSE(img, mview, reinit_every=2)  # the view itself: its pointer keeps the offset
    obuf = torch.full((h * w + 64,), 7, dtype=torch.uint8, device=dev)
    oview = obuf[off:off + h * w].view(h, w)
    job.mask(out=oview)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(oview.cpu().numpy(), (m != 0).astype(np.uint8))
    rest = torch.cat([obuf[:off], obuf[off + h * w:]]).cpu().numpy()
    assert (rest == 7).all()  # nothing written outside the mask

    lsf = rng.standard_normal((h, w)).astype(np.float32)
    lsf[rng.random((h, w)) < 0.1] = 0.0
    lsf[rng.random((h, w)) < 0.1] = -0.0
    fbuf = torch.zeros(h * w + 64, dtype=torch.float32, device=dev)
    fview = fbuf[off:off + h * w].view(h, w)
    fview.copy_(torch.tensor(lsf, device=dev))
    job.set_lsf(fview)
    np.testing.assert_array_equal(job.mask().cpu().numpy(), (lsf >= 0).astype(np.uint8))


def test_runs_are_bitwise_deterministic(dev):
    sc = synth.scene_multiband(6, size=256, bands=4, n_roofs=8, n_roads=2)
    img, _ = _as_gpu(sc.image, dev)
    outs = []
    for _ in range(2):
        job = _make(dev, img, sc.init_region, sigma=1.5, ksize=11)
        job.run(25)
        outs.append((job.lsf().cpu().numpy(), job.stats()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


def test_checkpoint_resume_is_bitwise(dev):
    sc = synth.scene_multiband(8, size=256, bands=4, n_roofs=8, n_roads=2)
    img, _ = _as_gpu(sc.image, dev)
    full = _make(dev, img, sc.init_region, sigma=1.5, ksize=11)
    full.run(9)
    part = _make(dev, img, sc.init_region, sigma=1.5, ksize=11)
    part.run(4)
    ckpt = part.mask()
    resumed = _make(dev, img, sc.init_region, sigma=1.5, ksize=11)
    resumed.set_mask(ckpt, smoothed=True)
    resumed.run(5)
    np.testing.assert_array_equal(resumed.lsf().cpu().numpy(), full.lsf().cpu().numpy())
    np.testing.assert_array_equal(resumed.mask().cpu().numpy(), full.mask().cpu().numpy())
    # set_mask(smoothed=False) restarts from the binary LSF of eq. (13)
    resumed.set_mask(torch.tensor(sc.init_region, device=dev), smoothed=False)
    resumed.run(9)
    np.testing.assert_array_equal(resumed.lsf().cpu().numpy(), full.lsf().cpu().numpy())


def test_bad_values_are_reported(dev):
    from paper_1409_7474_amd import lse
    sc = synth.scene_tiny(0, size=64, n_rects=1)
    image = sc.image.copy()
    image[10, 10, 0] = np.nan
    img, _ = _as_gpu(image, dev)
    job = _make(dev, img, sc.init_region)
    job.run(3)
    assert job.check() == lse.LSE_ERR_BAD_VALUE
    assert job.stats()["bad_value"] and job.stats()["iters_done"] == 0
    np.testing.assert_array_equal(job.mask().cpu().numpy(), sc.init_region)


def test_constant_image_moves_nothing(dev):
    """A dyadic constant image: c+ == c- exactly, R == 0; Table I order then
    only rounds corners (the square loses its 4 corner pixels)."""
    img, img64 = _as_gpu(np.full((256, 256, 1), 0.25), dev)
    sq = synth.centred_square(256, 256, 128, 128)
    job = _make(dev, img, sq, sigma=1.0, ksize=7)
    job.run(2)
    ref = oracle.run(img64, sq, iters=2)
    np.testing.assert_array_equal(job.mask().cpu().numpy(), ref.mask)
    assert job.stats()["M"] == 0.0


# ----------------------------------------------------------- full sizes ---

@pytest.mark.parametrize("term", ["region", "edge"])
def test_large_multiband_one_step_parity(dev, term):
    """4096 x 4096 x 4 scene (40 roofs, 6 roads), sigma 1.5 / 11 x 11, in the
    launch configuration the benchmark times: one step from the GPU state
    after 5 iterations, checked on every pixel."""
    sc = synth.scene_large(0)
    img, img64 = _as_gpu(sc.image, dev)
    del sc.image
    mask = sc.init_region if term == "region" else sc.init_edge
    job = _make(dev, img, mask, term=term, sigma=1.5, ksize=11)
    job.run(5)
    g = oracle.edge_map(img64, 1.0, 9, 255.0) if term == "edge" else None
    err, amb, ref = one_step(job, img64, term=term, sigma=1.5, ts=11, g=g)
    assert err <= LSF_TOL
    if term == "region":
        st = job.stats()
        check_normaliser(st, img64, ref.M)
        np.testing.assert_allclose(st["c_plus"], ref.c_plus, rtol=2e-6)
        np.testing.assert_allclose(st["c_minus"], ref.c_minus, rtol=2e-6)


def _quiet_inside_tiles(bits_prev, r, fx=96, fy=48):
    """Pixels of the region step kernel's quiet all-inside tiles: 96 x 48
    tiles away from the border whose previous binary state is all ones over
    every bit the tile reads (rows y0 - 2r - 1 .. + fy + 4r + 2, columns
    x0 - 1 - 2r .. x0 + 97 + 2r); their region sums come from init."""
    h, w = bits_prev.shape
    out = np.zeros((h, w), bool)
    for y0 in range(0, h, fy):
        for x0 in range(0, w, fx):
            by0, nr = y0 - 2 * r - 1, fy + 4 * r + 2
            if x0 - 2 * r - 2 < 0 or x0 + fx + 2 * r + 2 > w or by0 < 0 or by0 + nr > h:
                continue
            if bits_prev[by0:by0 + nr, x0 - 1 - 2 * r:x0 + fx + 1 + 2 * r].all():
                out[y0:y0 + fy, x0:x0 + fx] = True
    return out


def test_profile_counts_needed_pixels(dev):
    """The algorithmic-bytes count used for roofline figures: per step, the
    pixels on the + side of the new LSF (read for the region sums) except in
    quiet all-inside tiles, or with |grad phi| != 0 (read for the update),
    recomputed here from the exported LSFs and masks."""
    from paper_1409_7474_amd import lse
    sc = synth.scene_multiband(9, size=500, bands=4, n_roofs=6, n_roads=1, height=400, width=500)
    img, _ = _as_gpu(sc.image, dev)
    for term, mask in (("region", sc.init_region), ("edge", sc.init_edge)):
        job = _make(dev, img, mask, term=term, sigma=1.5, ksize=11)
        job.run(2)
        job.profile(lse.PROFILE_COUNT)
        expect, quiet_px = 0, 0
        for _ in range(3):
            phi_n = job.lsf().cpu().double().numpy()
            b_prev = job.mask().cpu().numpy().astype(bool)
            job.step()
            phi_n1 = job.lsf().cpu().double().numpy()
            gx, gy = oracle.gradient(phi_n)
            need = (gx != 0) | (gy != 0)
            if term == "region":
                q = _quiet_inside_tiles(b_prev, 5)
                quiet_px += int(q.sum())
                need |= (phi_n1 >= 0) & ~q
            expect += int(need.sum())
        p = job.profile_read()
        assert p["counted_steps"] == 3 and p["needed_pixels"] == expect, (term, p, expect)
        if term == "region":
            assert quiet_px > 0  # the case is exercised


def _heavy_tiles(bits_prev, r, edge):
    """Tile grid of the fast step kernel (96 x 48 region, 96 x 64 edge tiles)
    with True where the tile is heavy (not quiet) given the binary state it
    reads: quiet needs the tile and its whole halo inside the image and every
    staged bit it reads uniform (rows y0 - RU - 1 - r .. + FY + 2 RU + 2 + 2r,
    columns x0 - 1 - RU - r .. x0 + 96 + RU + r; RU = r for the region term,
    0 for the edge term)."""
    h, w = bits_prev.shape
    fy, ru = (64, 0) if edge else (48, r)
    nty, ntx = -(-h // fy), -(-w // 96)
    heavy = np.ones((nty, ntx), bool)
    for ty in range(nty):
        for tx in range(ntx):
            y0, x0 = ty * fy, tx * 96
            by0, nr = y0 - ru - 1 - r, fy + 2 * ru + 2 + 2 * r
            if x0 - 2 * r - 2 < 0 or x0 + 96 + 2 * r + 2 > w or by0 < 0 or by0 + nr > h:
                continue
            win = bits_prev[by0:by0 + nr, x0 - 1 - ru - r:x0 + 97 + ru + r]
            heavy[ty, tx] = not (win.all() or not win.any())
    return heavy


def _touched_tiles(prev, cur, r, edge):
    """Tiles whose bit window (the rows and columns _heavy_tiles reads: RU +
    r + 1 pixels beyond the tile, one more on the right) holds a pixel that
    flipped from prev to cur; the kernel marks them from each flipping tile's
    own pixels within RU + r + 2 of its sides, a superset of those windows."""
    h, w = prev.shape
    fy, ru = (64, 0) if edge else (48, r)
    hw = ru + r + 2
    nty, ntx = -(-h // fy), -(-w // 96)
    out = np.zeros((nty, ntx), bool)
    for y, x in zip(*np.nonzero(prev != cur)):
        ty, tx, ry, rx = y // fy, x // 96, y % fy, x % 96
        dys = [0] + ([-1] if ry < hw else []) + ([1] if ry >= fy - hw else [])
        dxs = [0] + ([-1] if rx < hw else []) + ([1] if rx >= 96 - hw else [])
        for dy in dys:
            for dx in dxs:
                if (dy or dx) and 0 <= ty + dy < nty and 0 <= tx + dx < ntx:
                    out[ty + dy, tx + dx] = True
    return out


@pytest.mark.parametrize("term", ["region", "edge"])
def test_profile_counts_visited_and_heavy_tiles(dev, term):
    """Profiling counts of the front-sparse schedule: the tiles a step visits
    are the heavy tiles of the previous iteration and the neighbours whose
    bit windows that iteration's flips reached (all tiles right after a
    restart), and its heavy tiles are those whose bit window is not uniform;
    both recomputed here from the exported masks."""
    from paper_1409_7474_amd import lse
    sc = synth.scene_multiband(4, size=1400, bands=4, n_roofs=12, n_roads=1, height=1100, width=1400)
    img, _ = _as_gpu(sc.image, dev)
    r = 6
    job = _make(dev, img, sc.init_region if term == "region" else sc.init_edge, term=term, sigma=2.0, ksize=2 * r + 1)
    job.profile(lse.PROFILE_COUNT)
    job.step()
    p = job.profile_read()
    assert p["tiles"] == p["visited_tiles"] > 0 and p["counted_steps"] == 1
    masks = [job.mask().cpu().numpy().astype(bool)]
    job.step()
    masks.append(job.mask().cpu().numpy().astype(bool))
    job.profile(lse.PROFILE_COUNT)
    want_vis = want_heavy = touched_only = 0
    for _ in range(4):
        heavy_prev = _heavy_tiles(masks[-2], r, term == "edge")
        touched = _touched_tiles(masks[-2], masks[-1], r, term == "edge")
        want_vis += int((heavy_prev | touched).sum())
        touched_only += int((touched & ~heavy_prev).sum())
        want_heavy += int(_heavy_tiles(masks[-1], r, term == "edge").sum())
        job.step()
        masks.append(job.mask().cpu().numpy().astype(bool))
    p = job.profile_read()
    print(f"{term}: visited {want_vis}, heavy {want_heavy}, touched only {touched_only}, tiles {p['tiles']}", flush=True)
    assert (p["visited_tiles"], p["heavy_tiles"]) == (want_vis, want_heavy), (p, want_vis, want_heavy)
    assert 0 < want_vis < 4 * p["tiles"]  # the schedule skips settled tiles here
    if term == "edge":
        assert touched_only > 0  # the edge front moves across tile sides: touched tiles are exercised
    job.close()


def test_profile_timing_samples(dev):
    """LSE_PROFILE_SAMPLE(k): one launch in 2^k of each kernel carries timing
    events (launches 2^k - 1, 2 * 2^k - 1, ...); every launch with k = 0."""
    from paper_1409_7474_amd import lse
    sc = synth.scene_tiny(1)
    img = torch.tensor(np.asarray(sc.image, np.float32), device=dev)
    for flags, want in ((lse.PROFILE_TIMING, 12), (lse.PROFILE_TIMING | lse.PROFILE_SAMPLE(2), 3)):
        job = _make(dev, img, sc.init_region)
        job.profile(flags)
        job.run(12)
        p = job.profile_read()
        assert p["step_launches"] == want and p["step_ms"] > 0.0, p
        job.close()
