"""Step-kernel variants and the autotuner (lse_autotune), through the C ABI.

Every variant (edge term: 64, 48 or 80 tile rows; region terms: 4, 3 or 5
waves per SIMD) must give the same binary state, LSF and statistics bit for
bit as variant 0, whose results the parity tests check against the FP64
oracle; a batch whose images run different variants must equal their solo
runs; the tuner must time every candidate and enter the fastest."""
import numpy as np
import pytest

from paper_1409_7474_amd import lse, synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def clean_table():
    lse.lse_tuning_clear()
    yield
    lse.lse_tuning_clear()


def _scene(h, w, bands, seed):
    sc = synth.scene_multiband(seed, size=max(h, w), bands=bands, n_roofs=10, n_roads=2, height=h, width=w)
    return sc


def _state(job):
    return job.mask().cpu().numpy(), job.lsf().cpu().numpy(), job.stats()


FAMILIES = [
    # term, bands, TS, storage, shape, iterations
    ("region", 4, 7, "f32", (700, 900), 25),
    ("region", 4, 13, "f32", (640, 500), 20),
    ("region", 1, 11, "f16", (513, 777), 20),
    ("edge", 4, 11, "f32", (650, 800), 25),
    ("edge", 2, 13, "bf16", (401, 999), 20),
]


@pytest.mark.parametrize("term,bands,ts,storage,shape,iters", FAMILIES)
def test_variants_are_bitwise_equal(dev, term, bands, ts, storage, shape, iters):
    h, w = shape
    sc = _scene(h, w, bands, 3)
    img = torch.tensor(np.asarray(sc.image, np.float32), device=dev)
    init = torch.tensor(sc.init_region if term == "region" else sc.init_edge, device=dev)
    kw = dict(term=term, sigma=(ts // 2) / 3.0, ksize=ts, storage=storage)
    p = lse.make_params(h, w, bands, **kw)
    states = []
    for v in range(3):
        lse.lse_tuning_set(p, v)
        job = lse.LSE(img, init, **kw)
        t = job.tuning()
        assert t["variant"] == v
        rows = {"region": [48, 48, 48], "edge": [64, 48, 80]}[term][v]
        assert t["tile_rows"] == rows
        job.run(iters)
        states.append(_state(job))
        job.close()
    print(f"{term} B={bands} TS {ts} {storage} {shape}: variants 0-2 equal", flush=True)
    for v in (1, 2):
        assert np.array_equal(states[v][0], states[0][0]), f"variant {v}: masks differ"
        assert np.array_equal(states[v][1].view(np.uint32), states[0][1].view(np.uint32)), f"variant {v}: LSF"
        assert states[v][2] == states[0][2], f"variant {v}: statistics differ"


def test_batch_of_mixed_variants_equals_solo(dev):
    """Contexts of one family but different variants form separate groups of
    one batch; each image still equals its solo run."""
    jobs, solo, kws = [], [], []
    for i, (h, w, v) in enumerate([(300, 420, 0), (280, 500, 2), (333, 211, 1), (256, 256, 2)]):
        sc = _scene(h, w, 4, 10 + i)
        img = torch.tensor(np.asarray(sc.image, np.float32), device=dev)
        init = torch.tensor(sc.init_edge, device=dev)
        kw = dict(term="edge", sigma=1.5, ksize=11)
        lse.lse_tuning_set(lse.make_params(h, w, 4, **kw), v)
        jobs.append(lse.LSE(img, init, **kw))
        assert jobs[-1].tuning()["variant"] == v
        lse.lse_tuning_clear()
        solo.append(lse.LSE(img, init, **kw))  # variant 0
    batch = lse.Batch(jobs)
    batch.run(18)
    for j, s in zip(jobs, solo):
        s.run(18)
        a, b = _state(j), _state(s)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    batch.close()


def test_autotune_times_every_candidate_and_enters_the_fastest(dev):
    sc = synth.scene_large(0, size=1024)
    img = torch.tensor(np.asarray(sc.image, np.float32), device=dev)
    for term, init in (("region", sc.init_region), ("edge", sc.init_edge)):
        kw = dict(term=term, sigma=1.5, ksize=11)
        t = lse.autotune(img, torch.tensor(init, device=dev), iters=12, **kw)
        print(f"autotune {term} 1024^2: {t}", flush=True)
        assert t["candidates"] == 3 and all(m > 0 for m in t["ms"])
        ms = t["ms"]
        faster = [v for v in (1, 2) if ms[v] < 0.97 * ms[0]]
        assert t["variant"] == (min(faster, key=lambda v: ms[v]) if faster else 0)
        p = lse.make_params(1024, 1024, 4, **kw)
        assert lse.lse_tuning_lookup(p).as_dict() == t
        job = lse.LSE(img, torch.tensor(init, device=dev), **kw)
        assert job.tuning()["variant"] == t["variant"]
        job.close()
