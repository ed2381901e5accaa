"""GPU tests of 16-bit storage and of batched execution, through the C ABI.

Storage: the library rounds the image (region term) or the edge map (edge
term) once, at init, to FP16 or BF16 and computes in FP32.  One-step parity
is checked against the FP64 oracle fed the same rounded values, with the
bars of the FP32 path; the error of each storage type against the FP64
oracle on the unrounded image is measured over whole runs.

Batching: contexts advanced together by lse_batch_run (one launch per
iteration and kernel family, optionally replayed from a HIP graph) must give
bit for bit the results of each context run alone.
"""
import numpy as np
import pytest

import oracle
from paper_1409_7474_amd import synth
from parity_helpers import (LSF_TOL, _make, check_normaliser, iou, mask_disagreement, one_step,
                            round_storage)

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DT16 = {"f16": torch.float16, "bf16": torch.bfloat16}
# Relative rounding step (one ulp at 1) of the storage types.
ULP1 = {"f16": 2.0 ** -10, "bf16": 2.0 ** -7}


def _img(dev, image, dtype=torch.float32):
    return torch.tensor(np.asarray(image, np.float32), device=dev).to(dtype)


# ------------------------------------------------------------- storage ---

@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("bands,h,w,ts,sigma", [(4, 200, 333, 11, 1.5), (1, 150, 97, 7, 1.0),
                                                (2, 97, 130, 13, 2.0)])
def test_region_storage_one_step_parity(dev, storage, bands, h, w, ts, sigma):
    """Region term with the image stored in 16 bits: the oracle, given the
    rounded image, agrees to the FP32 bars (the rounding is the only
    difference, and it is applied identically on both sides)."""
    sc = synth.scene_multiband(11, size=max(h, w), bands=bands, n_roofs=10, n_roads=2, height=h, width=w)
    img64 = round_storage(sc.image, storage)
    job = _make(dev, _img(dev, sc.image), sc.init_region, sigma=sigma, ksize=ts, storage=storage)
    for it in range(6):
        err, _, ref = one_step(job, img64, sigma=sigma, ts=ts)
        assert err <= LSF_TOL, (storage, it, err)
        st = job.stats()
        np.testing.assert_allclose(st["c_plus"], ref.c_plus, rtol=2e-6, atol=1e-7)
        np.testing.assert_allclose(st["c_minus"], ref.c_minus, rtol=2e-6, atol=1e-7)
        check_normaliser(st, img64, ref.M)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_input_with_matching_storage_is_exact(dev, storage):
    """A 16-bit caller image stored in the same type is copied exactly: the
    run equals the run on the same values given as FP32."""
    sc = synth.scene_multiband(3, size=160, bands=4, n_roofs=6, n_roads=1)
    t16 = _img(dev, sc.image, DT16[storage])
    a = _make(dev, t16, sc.init_region, sigma=1.5, ksize=11, storage=storage)
    b = _make(dev, t16.float(), sc.init_region, sigma=1.5, ksize=11, storage=storage)
    a.run(25)
    b.run(25)
    assert torch.equal(a.lsf(), b.lsf())
    assert a.stats() == b.stats()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_edge_storage_one_step_parity(dev, storage):
    """Edge term with g stored in 16 bits.  The oracle takes its own FP64 g
    rounded to the storage type; the GPU rounds its FP32 g, so the two stored
    maps may differ by one storage ulp where FP32 and FP64 straddle a rounding
    boundary.  Decisions may then differ only where |u| is below
    dt * max|grad phi| * ulp(1) (max|grad phi| <= 2 sqrt 2 for phi in
    [-1, 1], one-sided differences at the border)."""
    sc = synth.scene_multiband(5, size=192, bands=3, n_roofs=8, n_roads=1)
    x = np.asarray(sc.image, np.float32).astype(np.float64)
    g = round_storage(oracle.edge_map(x, 1.0, 9, 255.0), storage)
    job = _make(dev, _img(dev, sc.image), sc.init_edge, term="edge", sigma=1.5, ksize=11, storage=storage)
    tau = 15.0 * 2.0 * np.sqrt(2.0) * ULP1[storage]
    for it in range(6):
        err, amb, _ = one_step(job, None, term="edge", sigma=1.5, ts=11, g=g, tau=tau)
        assert err <= LSF_TOL, (storage, it, err, amb)


def test_storage_precision_against_fp64(dev):
    """Whole runs (512 x 512 x 4, sigma 1.5 / TS 11, 150 iterations): each
    storage type against the FP64 oracle on the unrounded image -- final mask
    sign disagreement <= 1e-4 and IoU -- and the LSF max-abs error, printed
    per storage type."""
    sc = synth.scene_multiband(21, size=512, bands=4, n_roofs=10, n_roads=2)
    x = np.asarray(sc.image, np.float32).astype(np.float64)
    ref = oracle.run(x, sc.init_region, term="region", iters=150, sigma=1.5, ts=11)
    ref_mask = ref.b > 0
    report = {}
    for storage in ("f32", "f16", "bf16"):
        job = _make(dev, _img(dev, sc.image), sc.init_region, sigma=1.5, ksize=11, storage=storage)
        job.run(150)
        mask = job.mask().cpu().numpy().astype(bool)
        lsf = job.lsf().cpu().double().numpy()
        d = mask_disagreement(mask, ref_mask)
        report[storage] = (float(np.abs(lsf - ref.phi).max()), d, iou(mask, ref_mask))
        assert d <= 1e-4, (storage, report[storage])
    print("storage precision vs FP64 oracle (LSF max-abs, mask disagreement, IoU):", report)


# ------------------------------------------------------------- batches ---

def _jobs_spec():
    """Uneven images of every kernel family the batch groups by."""
    return [
        dict(h=300, w=211, bands=4, term="region", storage="f32", ts=7, sigma=1.0, seed=1),
        dict(h=97, w=450, bands=4, term="region", storage="f32", ts=7, sigma=1.0, seed=2),
        dict(h=256, w=256, bands=1, term="region", storage="f32", ts=7, sigma=1.0, seed=3),
        dict(h=180, w=140, bands=3, term="region", storage="f16", ts=11, sigma=1.5, seed=4),
        dict(h=210, w=333, bands=2, term="edge", storage="f32", ts=11, sigma=1.5, seed=5),
        dict(h=64, w=64, bands=4, term="region", storage="f32", ts=7, sigma=1.0, seed=6),
        dict(h=130, w=150, bands=1, term="edge", storage="bf16", ts=7, sigma=1.0, seed=7),
    ]


def _build(dev, spec):
    jobs, inputs = [], []
    for s in spec:
        sc = synth.scene_multiband(s["seed"], size=max(s["h"], s["w"]), bands=s["bands"], n_roofs=8, n_roads=1,
                                   height=s["h"], width=s["w"])
        init = sc.init_region if s["term"] == "region" else sc.init_edge
        jobs.append(_make(dev, _img(dev, sc.image), init, term=s["term"], storage=s["storage"], sigma=s["sigma"],
                          ksize=s["ts"]))
        inputs.append(sc)
    return jobs


def _state(job):
    return job.mask().cpu().numpy(), job.lsf().cpu().numpy(), job.stats()


def _assert_same(a, b, what):
    assert np.array_equal(a[0], b[0]), f"{what}: masks differ"
    assert np.array_equal(a[1], b[1]), f"{what}: LSFs differ"
    assert a[2] == b[2], f"{what}: statistics differ"


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_alone(dev, graph):
    """Seven uneven images (both terms, B = 1..4, three storage types, two
    template sizes; five kernel families, each on a stream of the batch's
    own), per-image iteration targets: the batch reproduces every image's
    solo run bit for bit, also when its launches replay from a graph.  The
    graph is replayed three times with host reads in between, and every
    image is checked after each replay (the third one is past every target
    and must change nothing)."""
    from paper_1409_7474_amd import lse
    spec = _jobs_spec()
    targets = [23, 17, 30, 23, 11, 30, 5]
    alone = _build(dev, spec)
    want15 = []
    for j, t in zip(alone, targets):
        j.run(min(15, t))
        want15.append(_state(j))
        j.run(t - min(15, t))
    want = [_state(j) for j in alone]

    stream = torch.cuda.Stream(dev)  # graphs need a non-default stream
    with torch.cuda.stream(stream):
        jobs = _build(dev, spec)
        for j in jobs:
            j.stream = stream
        batch = lse.Batch(jobs, targets=targets, stream=stream)
        for replay, expect in enumerate((want15, want, want)):
            batch.run(15, graph=graph)
            stream.synchronize()
            for i, (j, t) in enumerate(zip(jobs, targets)):
                got = _state(j)
                assert got[2]["iters_done"] == min(15 * (replay + 1), t), (replay, i, got[2]["iters_done"])
                _assert_same(got, expect[i], f"run {replay}, image {i}")
    batch.close()


@pytest.mark.parametrize("term", ["region", "region_intensity", "edge"])
def test_single_image_skipping_equals_batch(dev, term):
    """A single image visits only the tiles near the front, from a visit
    list built by the normaliser pass (region, B = 4) or by its own pass (the
    other terms, more than 4096 tiles here); small images let each workgroup
    scan the heavy record itself (every other test).  A batch of one builds
    its list in a separate pass over the whole group.  The independent
    builders must agree bit for bit after 40 iterations, and after a restart
    from a new mask."""
    from paper_1409_7474_amd import lse
    sc = synth.scene_multiband(11, size=4160, bands=4, n_roofs=30, n_roads=3, height=4160, width=6240)
    img = _img(dev, sc.image)
    init = sc.init_edge if term == "edge" else sc.init_region
    kw = dict(term=term, sigma=1.5, ksize=11)
    solo = _make(dev, img, init, **kw)
    solo.run(40)
    want = _state(solo)
    other = _make(dev, img, init, **kw)
    batch = lse.Batch([other])
    batch.run(40)
    _assert_same(_state(other), want, term)
    assert want[2]["iters_done"] == 40
    m = torch.tensor(sc.init_region, device=dev)
    solo.set_mask(m, smoothed=False)
    other.set_mask(m, smoothed=False)
    solo.run(12)
    batch.run(12)
    _assert_same(_state(other), _state(solo), term + " after set_mask")
    batch.close()
    solo.close()
    other.close()


@pytest.mark.parametrize("term,image,at", [("region", 8, 25), ("region", 10, 65), ("edge", 8, 40),
                                           ("edge", 12, 60)])
def test_uneven_image_late_step_parity(dev, term, image, at):
    """Images of the batched workload (4 bands, 7 x 7), deep into the run,
    where most tiles are settled and skipped: one-step parity with the FP64
    oracle, which evaluates every pixel.  The region cases are where the
    visited tiles once missed neighbours of the image's top tile row (record
    words next to the record's ends read as zero)."""
    shapes = synth.batch_shapes(0, n=64)
    sc = synth.scene_batch_image(0, image, *shapes[image])
    init = sc.init_region if term == "region" else sc.init_edge
    job = _make(dev, _img(dev, sc.image), init, term=term, sigma=1.0, ksize=7)
    job.run(at)
    x = np.asarray(sc.image, np.float32).astype(np.float64)
    g = oracle.edge_map(x, 1.0, 9, 255.0) if term == "edge" else None
    for _ in range(2):
        err, _, _ = one_step(job, x, term=term, sigma=1.0, ts=7, g=g)
        assert err <= LSF_TOL


@pytest.mark.parametrize("term", ["region", "edge"])
def test_uneven_images_alone_equal_batch(dev, term):
    """Eight uneven images of the batched workload, 150 iterations: each
    image's single-image run (visit list from the normaliser pass, or each
    workgroup's own scan of the heavy record) equals the batch (visit list
    over the group) bit for bit."""
    from paper_1409_7474_amd import lse
    shapes = synth.batch_shapes(0, n=64)
    pick = [8, 10, 12, 13, 17, 18, 19, 22]
    scs = [synth.scene_batch_image(0, i, *shapes[i]) for i in pick]
    init = [sc.init_region if term == "region" else sc.init_edge for sc in scs]
    alone = [_make(dev, _img(dev, sc.image), m, term=term, sigma=1.0, ksize=7) for sc, m in zip(scs, init)]
    for j in alone:
        j.run(150)
    jobs = [_make(dev, _img(dev, sc.image), m, term=term, sigma=1.0, ksize=7) for sc, m in zip(scs, init)]
    batch = lse.Batch(jobs)
    batch.run(150)
    for i in range(len(pick)):
        _assert_same(_state(jobs[i]), _state(alone[i]), f"image {pick[i]}")
    batch.close()


def test_batch_interleaves_with_single_steps(dev):
    """Batch runs, solo steps of one member and lse_set_mask between them keep
    every image identical to its solo history."""
    from paper_1409_7474_amd import lse
    spec = _jobs_spec()[:4]
    alone = _build(dev, spec)
    jobs = _build(dev, spec)
    batch = lse.Batch(jobs)
    batch.run(4)
    jobs[1].step()
    batch.run(3)
    for i, j in enumerate(alone):
        j.run(4)
        if i == 1:
            j.step()
        j.run(3)
    for i in range(len(jobs)):
        _assert_same(_state(jobs[i]), _state(alone[i]), f"image {i}")
    # restart one member from its initial mask: the batch follows
    sc = synth.scene_multiband(spec[2]["seed"], size=256, bands=1, n_roofs=8, n_roads=1, height=256, width=256)
    m = torch.tensor(sc.init_region, device=dev)
    jobs[2].set_mask(m, smoothed=False)
    alone[2].set_mask(m, smoothed=False)
    batch.run(6)
    for i, j in enumerate(alone):
        j.run(6)
    for i in range(len(jobs)):
        _assert_same(_state(jobs[i]), _state(alone[i]), f"image {i} after set_mask")
    batch.close()


def test_batch_update_equals_alone(dev):
    """lse_batch_update: members leave and join between runs (as in
    continuous batching), on new tables while the old ones are still alive;
    every image's state equals its run alone bit for bit."""
    from paper_1409_7474_amd import lse
    spec = _jobs_spec()
    jobs = _build(dev, spec)
    solo = _build(dev, spec)
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    batch = lse.Batch(jobs[:4], targets=[30, 25, 30, 12], stream=stream)
    batch.run(10)
    held = [batch.update(jobs[1:6], targets=[25, 30, 12, 40, 40])]  # job 0 leaves, 4 and 5 join
    batch.run(8)
    held.append(batch.update([jobs[5], jobs[6], jobs[2]], targets=[40, 9, 30]))  # only families 1, 3 left
    batch.run(9)
    torch.cuda.synchronize(dev)
    done = {0: 10, 1: 18, 2: 27, 3: 12, 4: 8, 5: 17, 6: 9}
    for i, n in done.items():
        solo[i].run(n)
        _assert_same(_state(jobs[i]), _state(solo[i]), f"image {i} after {n} iterations")
    batch.close()
    del held


def test_batch_update_refused_after_graph_runs(dev):
    """A batch that has replayed from a graph is not re-planned (its captured
    sequence names the old table): lse_batch_update returns LSE_ERR_STATE and
    leaves the batch as it was.  Host-side check; nothing is re-captured."""
    from paper_1409_7474_amd import lse
    jobs = _build(dev, _jobs_spec()[:3])
    stream = torch.cuda.Stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    batch = lse.Batch(jobs, stream=stream)
    batch.run(4, graph=True)
    with pytest.raises(lse.LSEError) as e:
        batch.update(jobs[:2])
    assert e.value.status == lse.LSE_ERR_STATE
    batch.run(4, graph=True)  # the same captured sequence replays
    stream.synchronize()
    assert all(j.stats()["iters_done"] == 8 for j in jobs)
    batch.close()


def test_batch_stop_when_unchanged(dev):
    """Step 5 inside a batch: the noise-free rectangle reaches its exact mask
    and stops; a noisy partner keeps iterating; both equal their solo runs."""
    from paper_1409_7474_amd import lse
    img, truth = synth.rectangle_scene()
    init = synth.centred_square(256, 256, 128, 128)
    sc = synth.scene_tiny(2)
    alone = [_make(dev, _img(dev, img), init), _make(dev, _img(dev, sc.image), sc.init_region)]
    for j in alone:
        j.run(80, stop_when_unchanged=True)
    jobs = [_make(dev, _img(dev, img), init), _make(dev, _img(dev, sc.image), sc.init_region)]
    batch = lse.Batch(jobs)
    batch.run(80, stop_when_unchanged=True)
    for i in range(2):
        _assert_same(_state(jobs[i]), _state(alone[i]), f"image {i}")
    assert jobs[0].stats()["converged"]
    assert np.array_equal(jobs[0].mask().cpu().numpy(), truth)
    batch.close()


def test_batch_many_small_images_parity(dev):
    """A batch of 24 small uneven tiny-workload images (region, B = 4, 7 x 7):
    after 10 iterations each image matches the FP64 oracle one step further
    (one-step parity from the batch's own state)."""
    from paper_1409_7474_amd import lse
    shapes = synth.batch_shapes(3, n=24, lo=40, hi=200)
    scenes = [synth.scene_batch_image(3, i, h, w) for i, (h, w) in enumerate(shapes)]
    jobs = [_make(dev, _img(dev, s.image), s.init_region, sigma=1.0, ksize=7) for s in scenes]
    batch = lse.Batch(jobs)
    batch.run(10)
    for s, j in zip(scenes, jobs):
        x = np.asarray(s.image, np.float32).astype(np.float64)
        err, _, _ = one_step(j, x, sigma=1.0, ts=7)
        assert err <= LSF_TOL
    batch.close()


def test_batch_rejects_repeated_context(dev):
    from paper_1409_7474_amd import lse
    sc = synth.scene_tiny(0, size=64, n_rects=1)
    j = _make(dev, _img(dev, sc.image), sc.init_region)
    with pytest.raises(lse.LSEError) as e:
        lse.Batch([j, j])
    assert e.value.status == lse.LSE_ERR_INVALID_ARG
    big = _make(dev, _img(dev, sc.image), sc.init_region, sigma=5.0, ksize=31)
    with pytest.raises(lse.LSEError) as e:
        lse.Batch([j, big])
    assert e.value.status == lse.LSE_ERR_UNSUPPORTED
