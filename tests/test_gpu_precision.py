"""Storage precision against the FP64 oracle, per result (FP32, FP16 and BF16
storage of the image or edge map; all arithmetic FP32):

* on the full 8192 x 8192 x 4 runway scene (sigma 2 / 13 x 13), after the
  300 iterations the benchmark runs, one more step from the GPU's own state
  against the oracle step on the same stored values -- the bars of the
  one-step parity tests (binary decisions equal outside the FP32 ambiguity
  band, LSF within 1e-5 outside its footprint);
* on a 1024 x 1024 window centred on the runway, whole trajectories against
  the oracle on the unrounded image: the region term over 300 iterations, the
  edge term over 60 (at sigma 2 it leaks out of the runway later, the oracle
  too).  FP32 storage meets the 1e-4 mask bar; the 16-bit results are
  reported (their difference is the rounding of the input, which the oracle
  on the rounded input reproduces: checked below on a serving job).
"""
import numpy as np
import pytest

import oracle
from paper_1409_7474_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from parity_helpers import LSF_TOL, MASK_TOL, _make, iou, mask_disagreement, one_step, round_storage  # noqa: E402


@pytest.fixture(scope="module")
def precision_scene():
    return synth.scene_precision(0)


@pytest.mark.parametrize("term", ["region", "edge"])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_full_size_one_step_parity_after_300_iterations(dev, precision_scene, term, storage):
    sc = precision_scene
    x32 = np.asarray(sc.image, np.float32)
    img = torch.tensor(x32, device=dev)
    job = _make(dev, img, sc.init_region if term == "region" else sc.init_edge, term=term, sigma=2.0, ksize=13,
                storage=storage)
    job.run(300)
    stored = round_storage(x32, storage)
    g = round_storage(oracle.edge_map(x32.astype(np.float64), 1.0, 9, 255.0), storage) if term == "edge" else None
    # 16-bit edge maps: the GPU rounds its FP32 g, the oracle its FP64 g; they
    # may differ by one storage ulp, |grad phi| <= 2 sqrt(2): widen the band.
    ulp = {"f32": 0.0, "f16": 2.0 ** -10, "bf16": 2.0 ** -7}[storage]
    tau = 1e-5 * 15.0 + (15.0 * 2.0 * np.sqrt(2.0) * ulp if term == "edge" else 0.0)
    err, amb, ref = one_step(job, stored if term == "region" else None, term=term, sigma=2.0, ts=13, g=g, tau=tau)
    print(f"8192^2 {term} {storage}, step 301 vs FP64 oracle on the stored values: LSF max-abs {err:.3g}, "
          f"{amb} decisions in the ambiguity band differ", flush=True)
    assert err <= LSF_TOL
    job.close()


@pytest.mark.parametrize("term,iters", [("region", 300), ("edge", 60)])
def test_window_trajectories_against_fp64(dev, precision_scene, term, iters):
    full = precision_scene
    cy, cx = int(full.meta["runway"][0]), int(full.meta["runway"][1])
    y0, x0 = min(max(cy - 512, 0), 8192 - 1024), min(max(cx - 512, 0), 8192 - 1024)
    sc = synth.crop_scene(full, y0, x0, 1024, 1024)
    x32 = np.asarray(sc.image, np.float32)
    x64 = x32.astype(np.float64)
    m0 = sc.init_region if term == "region" else sc.init_edge
    g = oracle.edge_map(x64, 1.0, 9, 255.0) if term == "edge" else None
    ref = oracle.run(x64, m0, term=term, iters=iters, sigma=2.0, ts=13, g=g)
    ref_mask = ref.b > 0
    assert 0.01 < ref_mask.mean() < 0.9  # the front neither vanished nor flooded the window
    img = torch.tensor(x32, device=dev)
    report = {}
    for storage in ("f32", "f16", "bf16"):
        job = _make(dev, img, m0, term=term, sigma=2.0, ksize=13, storage=storage)
        job.run(iters)
        mask = job.mask().cpu().numpy().astype(bool)
        lsf = job.lsf().cpu().double().numpy()
        report[storage] = {"mask_disagreement": mask_disagreement(mask, ref_mask), "iou": iou(mask, ref_mask),
                           "lsf_max_abs": float(np.abs(lsf - ref.phi).max())}
        job.close()
    print(f"1024^2 window, {term} {iters} iterations vs FP64 oracle (inside {ref_mask.mean():.4f}): {report}",
          flush=True)
    assert report["f32"]["mask_disagreement"] <= MASK_TOL


def test_16bit_difference_is_the_rounding_of_the_input(dev):
    """Serving job 1995 of the serving trace (region term, 283 x 283, one
    band, 176 iterations; its front is still moving at the end): its FP16 mask
    differs from the FP32 one in about 0.85 % of the pixels.  The FP16 GPU
    run matches the FP64 oracle run on the FP16-rounded image, and the FP32
    GPU run the oracle on the FP32 image, each within the mask bar: the
    difference is the method's response to the rounding of its input, not an
    error of the kernels."""
    from paper_1409_7474_amd import serve
    pool = serve.PoolInputs(synth.serving_pool(0), dev)
    job = [j for j in synth.serving_trace(0, n_jobs=2000, qps=1.0) if j.job_id == 1995][0]
    assert (job.side, job.bands, job.term, job.iters) == (283, 1, "region", 176)
    img, init = pool(job)
    x64 = img.cpu().double().numpy()
    m0 = init.cpu().numpy()
    masks = {}
    for storage in ("f32", "f16"):
        j = _make(dev, img, m0, sigma=1.5, ksize=11, storage=storage)
        j.run(job.iters)
        masks[storage] = j.mask().cpu().numpy().astype(bool)
        j.close()
    ref32 = oracle.run(x64, m0, iters=job.iters, sigma=1.5, ts=11)
    ref16 = oracle.run(round_storage(x64, "f16"), m0, iters=job.iters, sigma=1.5, ts=11)
    d_gpu = mask_disagreement(masks["f16"], masks["f32"])
    d_oracle = mask_disagreement(ref16.b > 0, ref32.b > 0)
    d16 = mask_disagreement(masks["f16"], ref16.b > 0)
    d32 = mask_disagreement(masks["f32"], ref32.b > 0)
    print(f"serving job 1995: FP16 vs FP32 on the GPU {d_gpu:.4g}, oracle on the FP16-rounded vs FP32 image "
          f"{d_oracle:.4g}; GPU FP16 vs oracle (rounded) {d16:.3g}, GPU FP32 vs oracle {d32:.3g}", flush=True)
    assert d_gpu > 1e-3 and d_oracle > 1e-3
    assert d16 <= MASK_TOL and d32 <= MASK_TOL
