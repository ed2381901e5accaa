"""Throughput benchmark of the fast level set evolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]

One step = one whole job on the 4096 x 4096 x 4 multiband scene (40 roofs,
6 roads, noise 0.03; sigma 1.5, 11 x 11 template, dt 15): lse_init + 200
region-term iterations, then lse_init + 200 edge-term iterations, with the
image already resident in HBM.  `value` = pixel-iterations per second over
the K timed steps (2 x 200 x 4096^2 per step).  The line also carries
  * roofline -- algorithmic HBM bytes of the fused region step kernel per
    launch / its mean launch time (HIP events on the launch stream, over the
    timed region), against the MI355X HBM peak of 8 TB/s;
  * cpu_baseline -- the FP64 CPU oracle on a bounded sample of the same job
    (a few iterations of each term on the full image), on this host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "LSE Mpixel-iter/s + % HBM peak, batched vs plain FP32; p50/p99 job latency"

WORKLOADS = {
    # name: (generator kwargs, sigma, ksize, iterations, terms)
    "large": (dict(size=4096), 1.5, 11, 200, ("region", "edge")),
    "tiny": (dict(size=256), 1.0, 7, 100, ("region",)),
    "precision": (dict(size=8192), 2.0, 13, 300, ("region", "edge")),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8, help="oracle iterations per term in the CPU sample")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="instead of the benchmark, run a plain device copy of this many MiB (reads and writes "
                         "that many bytes) so that profiler byte counters can be scaled against a known size")
    return ap.parse_args()


def calibrate_copy(mib):
    """A plain copy kernel of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * 1024 * 1024 // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_read_per_launch": n * 4, "bytes_written_per_launch": n * 4,
                      "launches": 3}), flush=True)


def measured_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from a committed rocprofv3
    summary (profiles/*.md, FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel
    calibration), only if it was taken on the current kernel source."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1409_7474_amd", "csrc", "lse_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        for block in text.split("```json")[1:]:
            try:
                data = json.loads(block.split("```")[0])
            except ValueError:
                continue
            if data.get("kernel_source_sha256") != sha:
                continue
            t = data.get("per_launch_traffic", {}).get(kernel_name)
            if t:
                return t["read_bytes"] + t["write_bytes"], os.path.relpath(path, ROOT)
    return None, None


def make_scene(name):
    from paper_1409_7474_amd import synth
    if name == "large":
        return synth.scene_large(0)
    if name == "precision":
        return synth.scene_precision(0)
    return synth.scene_tiny(0)


def cpu_baseline(scene, sigma, ksize, iters, terms):
    """FP64 oracle on the full image, `iters` iterations of each term."""
    import numpy as np

    import oracle
    img = scene.image.astype(np.float32).astype(np.float64)
    h, w, _ = img.shape
    t_total = 0.0
    px_it = 0
    for term in terms:
        mask = scene.init_region if term == "region" else scene.init_edge
        g = oracle.edge_map(img, 1.0, 9, 255.0) if term == "edge" else None
        t0 = time.perf_counter()
        oracle.run(img, mask, term=term, iters=iters, sigma=sigma, ts=ksize, g=g)
        t_total += time.perf_counter() - t0
        px_it += h * w * iters
    return {"value": px_it / t_total / 1e6, "unit": "Mpixel-iter/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{iters} iterations of each of {list(terms)} on the full {h}x{w}x{img.shape[2]} image "
                      f"(edge map precompute excluded), {t_total:.1f} s"}


def main():
    args = parse()
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "see DESIGN.md for how the path would shard.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1409_7474_amd import lse

    gen_kw, sigma, ksize, iters, terms = WORKLOADS[args.workload]
    scene = make_scene(args.workload)
    h, w, b = scene.image.shape
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    s = int(stream.cuda_stream)
    img = torch.tensor(scene.image, dtype=torch.float32, device=dev)
    masks = {"region": torch.tensor(scene.init_region, device=dev),
             "edge": torch.tensor(scene.init_edge, device=dev)}
    params = {t: lse.make_params(h, w, b, term=t, sigma=sigma, ksize=ksize) for t in terms}
    for p in params.values():
        p.image_dtype = 0
    nbytes = max(lse.lse_workspace_bytes(p) for p in params.values())
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    ws_ptr = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    mask_out = torch.empty((h, w), dtype=torch.uint8, device=dev)

    def job(profile_into=None, flags=lse.PROFILE_TIMING):
        for t in terms:
            ctx = lse.lse_init(params[t], img.data_ptr(), masks[t].data_ptr(), ws_ptr, nbytes, s)
            if profile_into is not None:
                lse.lse_profile(ctx, flags)
            lse.lse_run(ctx, iters, False, s)
            lse.lse_mask(ctx, mask_out.data_ptr(), s)
            if profile_into is not None:
                p = lse.lse_profile_read(ctx)
                acc = profile_into.setdefault(t, {"step_ms": 0.0, "step_n": 0, "mpass_ms": 0.0, "mpass_n": 0,
                                                  "needed_px": 0, "counted": 0})
                acc["step_ms"] += p.step_ms
                acc["step_n"] += p.step_launches
                acc["mpass_ms"] += p.mpass_ms
                acc["mpass_n"] += p.mpass_launches
                acc["needed_px"] += p.needed_pixels
                acc["counted"] += p.counted_steps
                acc["dense_bytes_per_px"] = lse.lse_step_bytes_per_pixel(ctx)
            lse.lse_destroy(ctx)

    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()
    prof = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        job(prof)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    px_it = h * w * iters * len(terms) * args.steps
    value = px_it / elapsed / 1e6
    inside = float(mask_out.float().mean().item())

    # Algorithmic bytes of the step kernel: an untimed replay of the same
    # (deterministic) job counts, per step, the pixels whose image value the
    # step needs; each costs one pixel of image (region: B x 4 bytes) or edge
    # map (4 bytes); the binary state adds one bit read and one bit written.
    counted = {}
    job(counted, lse.PROFILE_COUNT)
    torch.cuda.synchronize()

    def step_bytes(t):
        c = counted[t]
        per_px = 4.0 * b if t == "region" else 4.0
        return per_px * c["needed_px"] / max(c["counted"], 1) + 2.0 * h * w / 8.0

    dom = "region" if "region" in prof else terms[0]
    pr = prof[dom]
    step_ms = pr["step_ms"] / max(pr["step_n"], 1)
    alg = step_bytes(dom)
    achieved = alg / (step_ms * 1e-3) / 1e9
    kname = f"lse::step_fast_kernel<{ksize // 2}, {4 if b == 3 else b if dom == 'region' else 1}, " \
            f"{'false' if dom == 'region' else 'true'}>"
    traffic, traffic_src = measured_traffic(kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
                "kernel": f"step_fast_kernel ({dom} term, B={b})", "mean_launch_us": round(step_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": int(alg),
                "needed_pixel_fraction": round(counted[dom]["needed_px"] / max(counted[dom]["counted"], 1) / (h * w),
                                               4)}
    per_term = {}
    for t, pr_t in prof.items():
        ms_t = pr_t["step_ms"] / max(pr_t["step_n"], 1)
        d = {"step_kernel_us": round(ms_t * 1e3, 2),
             "step_kernel_GBps": round(step_bytes(t) / (ms_t * 1e-3) / 1e9, 1),
             "step_dense_equiv_GBps": round(pr_t["dense_bytes_per_px"] * h * w / (ms_t * 1e-3) / 1e9, 1)}
        if pr_t["mpass_n"]:
            mp = pr_t["mpass_ms"] / pr_t["mpass_n"]
            d["mpass_kernel_us"] = round(mp * 1e3, 2)
        per_term[t] = d

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{h}x{w}x{b} multiband scene ({args.workload}), "
                               f"{'+'.join(terms)} terms, {iters} iterations each, "
                               f"sigma {sigma}, {ksize}x{ksize} template, dt 15, image resident in HBM",
                   "global_batch": 1, "parallelism": "single GPU"},
        "roofline": roofline, "per_term": per_term, "final_mask_inside_fraction": round(inside, 4),
        "gpu": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, sigma, ksize, args.cpu_iters, terms)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
