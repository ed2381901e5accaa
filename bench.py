"""Throughput benchmark of the fast level set evolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]
                    [--job both|concurrent|sequential]
                    [--sections batched,precision,serving]

One step = one whole job on the 4096 x 4096 x 4 multiband scene (40 roofs,
6 roads, noise 0.03; sigma 1.5, 11 x 11 template, dt 15): lse_init + 200
region-term iterations and lse_init + 200 edge-term iterations, with the
image already resident in HBM.  The two solves are independent and run on two
HIP streams at once (their latency-bound steps overlap on the device; the
edge solve's stream runs on 7/8 of the CUs, so the region solve, the longer
chain, always finds room); `sequential` times the same job with one solve
after the other on one stream.  --job concurrent or --job sequential times
one of the two only, so that a kernel trace of the run has one launch
configuration.  `value` = pixel-iterations per second over the K timed steps
of the two-stream job (2 x 200 x 4096^2 per step).  The line also carries
  * roofline -- algorithmic HBM bytes of the fused region step kernel per
    launch / its mean launch time (HIP events carried by the dispatch of one
    launch in 8 on the launch stream) in the timed sequential pass, where the
    kernel has the device to itself, against the MI355X HBM peak of 8 TB/s;
    roofline_concurrent -- the same in the timed two-stream job;
  * cpu_baseline -- the FP64 CPU oracle on a bounded sample of the same job
    (a few iterations of each term on the full image), on this host's cores;
  * batched -- 64 uneven images (sides 512-2048, 4 bands, sigma 1 / 7 x 7,
    150 iterations): one batched, graph-replayed launch sequence (FP32 and
    FP16 storage) against the 64 images run one after another (plain FP32);
  * precision -- 8192 x 8192 x 4 runway scene (sigma 2 / 13 x 13, 300
    iterations) with the image / edge map stored in FP32, FP16 and BF16:
    throughput, and agreement of the 16-bit runs with the FP32 run; and a
    1024 x 1024 window of it against the FP64 oracle;
  * serving -- 2000 jobs (sides log-uniform 256-4096, 1 or 4 bands, region or
    edge, 100-300 iterations) arriving as a Poisson stream at 80 % of the
    measured batched capacity: continuous batching with FP16 storage under a
    200 GB budget (and a 2 GB budget for queueing) against one-at-a-time
    plain FP32 solves of the same trace; throughput and p50 / p99 latency.
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
    ap.add_argument("--job", default="both", choices=["both", "concurrent", "sequential"],
                    help="timed job: solves on concurrent streams (both: and a timed sequential pass after it), "
                         "or one after the other on one stream")
    ap.add_argument("--sections", default="batched,precision,serving",
                    help="extra sections after the headline job: batched, precision, serving (comma-separated; "
                         "empty for none)")
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate as a fraction of batched capacity")
    ap.add_argument("--batch-images", type=int, default=64)
    ap.add_argument("--cpu-iters", type=int, default=24, help="oracle iterations per term in the CPU sample (~10-15 s)")
    ap.add_argument("--profile-summary", default="",
                    help="print the markdown summary of the rocprofv3 runs under this directory and exit")
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


def kernel_source_digest():
    """SHA-256 over the HIP sources of the library (kernels and their headers),
    in name order: profiler figures apply only to the code they were taken on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1409_7474_amd", "csrc", "*"))):
        if path.endswith((".hip", ".h")):
            h.update(os.path.basename(path).encode())
            h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel_name):
    """HBM bytes per launch of `kernel_name` from a committed rocprofv3
    summary (profiles/*.md, FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel
    calibration), only if it was taken on the current kernel source."""
    import glob
    sha = kernel_source_digest()
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


def _hip():
    import ctypes
    return ctypes.CDLL("libamdhip64.so")


def cu_masked_stream(ncu, first, count):
    """A HIP stream (default priority) whose kernels run only on CUs first ..
    first + count - 1 (hipExtStreamCreateWithCUMask); raises if the runtime
    refuses the mask.  Release it with destroy_stream."""
    import ctypes
    hip = _hip()
    words = (ncu + 31) // 32
    mask = (ctypes.c_uint32 * words)()
    for i in range(first, min(first + count, ncu)):
        mask[i // 32] |= 1 << (i % 32)
    s = ctypes.c_void_p()
    rc = hip.hipExtStreamCreateWithCUMask(ctypes.byref(s), ctypes.c_uint32(words), mask)
    if rc != 0:
        raise RuntimeError(f"hipExtStreamCreateWithCUMask failed ({rc}) for CUs {first}..{first + count - 1}")
    return s.value


def destroy_stream(s):
    import ctypes
    _hip().hipStreamDestroy(ctypes.c_void_p(s))


PROFILE_COMMANDS = [
    "rocprofv3 --kernel-trace --stats -d OUT/trace_concurrent -o run -- python3 $R/bench.py --steps 2 --warmup 1 "
    "--no-cpu-baseline --sections '' --job concurrent",
    "rocprofv3 --kernel-trace --stats -d OUT/trace_sequential -o run -- python3 $R/bench.py --steps 2 --warmup 1 "
    "--no-cpu-baseline --sections '' --job sequential",
    "rocprofv3 --pmc FETCH_SIZE --kernel-trace --stats -d OUT/FETCH_SIZE -o run -- python3 $R/bench.py --steps 1 "
    "--warmup 0 --no-cpu-baseline --sections '' --job sequential",
    "rocprofv3 --pmc WRITE_SIZE --kernel-trace --stats -d OUT/WRITE_SIZE -o run -- python3 $R/bench.py --steps 1 "
    "--warmup 0 --no-cpu-baseline --sections '' --job sequential",
    "rocprofv3 --pmc FETCH_SIZE --kernel-trace --stats -d OUT/cal_FETCH_SIZE -o run -- python3 $R/bench.py "
    "--calibrate-copy-mib 256",
    "rocprofv3 --pmc WRITE_SIZE --kernel-trace --stats -d OUT/cal_WRITE_SIZE -o run -- python3 $R/bench.py "
    "--calibrate-copy-mib 256",
    "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY "
    "SQ_INSTS_VMEM_RD --kernel-trace --stats -d OUT/sq -o run -- python3 $R/bench.py --steps 1 --warmup 0 "
    "--no-cpu-baseline --sections '' --job sequential",
]


def profile_summary(base):
    """Markdown summary of the rocprofv3 runs of PROFILE_COMMANDS under `base`
    (one directory per run, each holding run_results.db): kernel-trace
    statistics of both job configurations, per-dispatch byte counters scaled
    by the copy calibration, SQ counters of the step kernels, and the
    per-launch traffic that measured_traffic reads back."""
    import sqlite3

    def q(db, sql):
        return list(sqlite3.connect(db).execute(sql))

    def counters(run):
        rows = q(os.path.join(base, run, "run_results.db"),
                 "select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                 "group by kernel_name, counter_name")
        return {(k, c): v for k, c, v, n in rows}

    def short(k):
        return k.split("(")[0].replace("void ", "")

    sha = kernel_source_digest()
    f, w = counters("FETCH_SIZE"), counters("WRITE_SIZE")
    cal_f = [v for (k, c), v in counters("cal_FETCH_SIZE").items() if "copyBuffer" in k][0]
    cal_w = [v for (k, c), v in counters("cal_WRITE_SIZE").items() if "copyBuffer" in k][0]
    copy_kib = 256 * 1024
    fac_f, fac_w = copy_kib / cal_f, copy_kib / cal_w
    out = ["# rocprofv3: fast LSE step on 4096x4096x4 (region + edge, sigma 1.5, 11x11, 200 iterations each)\n",
           "Workload: `bench.py` default (the 4096 x 4096 x 4 multiband scene; one step = one region job of 200 "
           "iterations + one edge job of 200 iterations).\n",
           f"Kernel sources: `paper_1409_7474_amd/csrc/*.hip, *.h` (bench.kernel_source_digest) sha256 `{sha}`.\n",
           "## Commands (run from /tmp with TMPDIR=/tmp, repo at $R)\n", "```", *PROFILE_COMMANDS,
           "python3 $R/bench.py --profile-summary OUT", "```\n",
           "The step timing in the PMC runs includes the untimed counting replay of bench.py (count_needed_kernel); "
           "the trace runs are the reference for durations.  Every run traces the warm-up, the timed steps and the "
           "counting replay, all in the one launch configuration that --job names.\n"]
    for j in ("concurrent", "sequential"):
        what = ("the region and edge solves on two concurrent streams, the edge one on 7/8 of the CUs (the timed "
                "job of bench.py; its `roofline_concurrent`)" if j == "concurrent"
                else "the two solves one after the other on one stream (bench.py's timed `sequential` pass; its "
                     "`roofline`)")
        out.append(f"## Kernel trace (--stats), --job {j}: {what}\n")
        out.append("| kernel | calls | mean (us) | % of GPU time |\n|---|---:|---:|---:|")
        for n, c, t, a, p in q(os.path.join(base, f"trace_{j}", "run_results.db"),
                               "select name,total_calls,total_duration,average,percentage from top_kernels limit 14"):
            out.append(f"| `{short(n)}` | {c} | {a:.2f} | {p:.1f} |")
        out.append("")
    out.append("## Byte counters (per dispatch, scaled)\n")
    out.append(f"Calibration: a plain 256 MiB device copy reads FETCH_SIZE = {cal_f:.0f} KiB and WRITE_SIZE = "
               f"{cal_w:.0f} KiB per dispatch, so FETCH_SIZE is scaled by {fac_f:.3f} and WRITE_SIZE by {fac_w:.3f}.\n")
    out.append("| kernel | FETCH_SIZE (KiB, raw) | read (MB, scaled) | WRITE_SIZE (KiB, raw) | written (MB, scaled) |"
               "\n|---|---:|---:|---:|---:|")
    traffic = {}
    for (k, c), v in sorted(f.items()):
        if "lse::" not in k:
            continue
        wv = w.get((k, "WRITE_SIZE"), 0)
        out.append(f"| `{short(k)}` | {v:.1f} | {v * 1024 * fac_f / 1e6:.2f} | {wv:.1f} | {wv * 1024 * fac_w / 1e6:.2f} |")
        traffic[short(k)] = {"read_bytes": int(v * 1024 * fac_f), "write_bytes": int(wv * 1024 * fac_w)}
    out.append("\n## SQ counters (per dispatch)\n")
    out.append("| kernel | counter | value |\n|---|---|---:|")
    for (k, c), v in sorted(counters("sq").items()):
        if "step_fast" in k or "mpass" in k:
            out.append(f"| `{short(k)}` | {c} | {v:.0f} |")
    out.append("\n## Machine-readable traffic (read by bench.py when the kernel source hash matches)\n")
    out.append("```json")
    out.append(json.dumps({"kernel_source_sha256": sha, "per_launch_traffic": traffic}))
    out.append("```")
    return "\n".join(out)


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


def _sync():
    import torch
    torch.cuda.synchronize()


def _agreement(mask_a, mask_b, lsf_a, lsf_b):
    import numpy as np
    a, b = mask_a.astype(bool), mask_b.astype(bool)
    union = np.logical_or(a, b).sum()
    return {"mask_disagreement": float(np.mean(a != b)),
            "iou": 1.0 if union == 0 else float(np.logical_and(a, b).sum() / union),
            "lsf_max_abs": float(np.abs(lsf_a.astype(np.float64) - lsf_b.astype(np.float64)).max())}


def section_batched(args):
    """64 uneven images advanced together vs one after another."""
    import numpy as np
    import torch

    from paper_1409_7474_amd import lse, synth
    dev = torch.device("cuda:0")
    iters = 150
    shapes = synth.batch_shapes(0, n=args.batch_images)
    stream = torch.cuda.Stream(dev)
    jobs = {}
    with torch.cuda.stream(stream):
        masks = []
        imgs = []
        for i, (h, w) in enumerate(shapes):
            sc = synth.scene_batch_image(0, i, h, w)
            imgs.append(torch.tensor(sc.image, dtype=torch.float32, device=dev))
            masks.append(torch.tensor(sc.init_region, device=dev))
        for st in ("f32", "f16"):
            jobs[st] = [lse.LSE(im, m, sigma=1.0, ksize=7, storage=st, stream=stream) for im, m in zip(imgs, masks)]
    npx = sum(h * w for h, w in shapes)

    def reset(js):
        for j, m in zip(js, masks):
            j.set_mask(m, smoothed=False)
        stream.synchronize()

    def timed(fn, js, reps=3):
        best = None
        for _ in range(reps):
            reset(js)
            t0 = time.perf_counter()
            fn()
            stream.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    def plain_all(js):
        for j in js:
            j.run(iters)

    out = {"workload": f"{len(shapes)} images, sides U{{512..2048}} (non-square), 4 bands, region term, "
                       f"sigma 1.0 / 7x7, dt 15, {iters} iterations, {npx / 1e6:.1f} Mpx in total",
           "pixels": npx}
    t_plain = timed(lambda: plain_all(jobs["f32"]), jobs["f32"])
    ref_masks = [j.mask().cpu().numpy() for j in jobs["f32"]]
    out["plain_f32"] = {"ms": round(t_plain * 1e3, 2), "value": round(npx * iters / t_plain / 1e6, 1)}
    for st in ("f32", "f16"):
        batch = lse.Batch(jobs[st], targets=[iters] * len(shapes), stream=stream)
        for graph in (False, True):
            reset(jobs[st])
            batch.run(iters, graph=graph)  # warm-up (and graph capture)
            t = timed(lambda: batch.run(iters, graph=graph), jobs[st])
            key = f"batched_{st}" + ("_graph" if graph else "")
            out[key] = {"ms": round(t * 1e3, 2), "value": round(npx * iters / t / 1e6, 1),
                        "speedup_vs_plain_f32": round(t_plain / t, 3)}
        masks_b = [j.mask().cpu().numpy() for j in jobs[st]]
        dis = float(sum(np.sum(a != b) for a, b in zip(masks_b, ref_masks)) / npx)
        out[f"batched_{st}"]["mask_disagreement_vs_plain_f32"] = dis
        batch.close()
    out["unit"] = "Mpixel-iter/s"
    return out


def section_precision(args):
    """Storage precision on the 8192^2 x 4 runway scene (GPU, three storage
    types, against the FP32-storage run) and on a 1024^2 window of it centred
    on the runway (against the FP64 oracle)."""
    import numpy as np
    import torch

    import oracle
    from paper_1409_7474_amd import lse, synth
    dev = torch.device("cuda:0")
    iters, sigma, ts = 300, 2.0, 13
    out = {"workload": f"8192x8192x4 runway + 200 roofs, sigma {sigma} / {ts}x{ts}, dt 15, {iters} iterations, "
                       "region and edge terms; FP64 comparison on a 1024x1024 window centred on the runway "
                       "(its own centred initial square; edge also after 100 iterations)"}
    full = synth.scene_precision(0)
    cy, cx = int(full.meta["runway"][0]), int(full.meta["runway"][1])
    y0, x0 = min(max(cy - 512, 0), 8192 - 1024), min(max(cx - 512, 0), 8192 - 1024)
    window = synth.crop_scene(full, y0, x0, 1024, 1024)
    for sc, tag in ((full, "full"), (window, "window")):
        size = sc.image.shape[0]
        img = torch.tensor(sc.image, dtype=torch.float32, device=dev)
        res = {}
        cases = [("region", iters), ("edge", iters)] + ([("edge", 100)] if tag == "window" else [])
        for term, n_it in cases:
            init = torch.tensor(sc.init_region if term == "region" else sc.init_edge, device=dev)
            runs = {}
            for st in ("f32", "f16", "bf16"):
                job = lse.LSE(img, init, term=term, sigma=sigma, ksize=ts, storage=st)
                _sync()
                t0 = time.perf_counter()
                job.run(n_it)
                _sync()
                dt = time.perf_counter() - t0
                runs[st] = (job.mask().cpu().numpy(), job.lsf().cpu().numpy(), dt)
                job.close()
                del job
            r = {}
            for st in ("f32", "f16", "bf16"):
                r[st] = {"ms": round(runs[st][2] * 1e3, 2),
                         "value": round(size * size * n_it / runs[st][2] / 1e6, 1),
                         "inside_fraction": round(float(runs[st][0].mean()), 5)}
                if st != "f32":
                    r[st]["vs_f32_storage"] = _agreement(runs[st][0], runs["f32"][0], runs[st][1], runs["f32"][1])
            if tag == "window":
                x = np.asarray(sc.image, np.float32).astype(np.float64)
                g = oracle.edge_map(x, 1.0, 9, 255.0) if term == "edge" else None
                ref = oracle.run(x, sc.init_region if term == "region" else sc.init_edge, term=term, iters=n_it,
                                 sigma=sigma, ts=ts, g=g)
                for st in ("f32", "f16", "bf16"):
                    r[st]["vs_fp64_oracle"] = _agreement(runs[st][0], (ref.b > 0).astype(np.uint8), runs[st][1],
                                                         ref.phi)
            res[f"{term}_{n_it}"] = r
        out[tag] = res
        del img
        torch.cuda.empty_cache()
    out["unit"] = "Mpixel-iter/s"
    return out


def section_serving(args):
    """Continuous-batching server vs one-at-a-time plain solves on one trace."""
    import dataclasses

    import torch

    from paper_1409_7474_amd import serve, synth
    dev = torch.device("cuda:0")
    pool = serve.PoolInputs(synth.serving_pool(0), dev)
    base = synth.serving_trace(0, n_jobs=args.serve_jobs, qps=1.0)
    work = [j.side * j.side * j.iters for j in base]
    mean_work = sum(work) / len(work)
    budget = 200 << 30
    # Capacity: the first 300 jobs all present at t = 0 (saturated batching).
    probe = [dataclasses.replace(j, arrival_s=0.0) for j in base[:300]]
    serve.serve(probe[:20], pool, budget_bytes=budget, storage="f16")  # warm-up
    cap = serve.serve(probe, pool, budget_bytes=budget, storage="f16")
    cap_pxit = cap.pixel_iters / cap.makespan_s
    qps = args.serve_load * cap_pxit / mean_work
    trace = synth.serving_trace(0, n_jobs=args.serve_jobs, qps=qps)
    served = serve.serve(trace, pool, budget_bytes=budget, storage="f16", keep_masks=True)
    plain = serve.serve_plain(trace, pool, storage="f32", keep_masks=True)
    dis, px = 0, 0
    worst = 0.0
    for a, b in zip(served.records, plain.records):
        d = int((a.mask != b.mask).sum().item())
        dis += d
        px += a.pixels
        worst = max(worst, d / a.pixels)
        a.mask = b.mask = None
    small = serve.serve(trace[:300], pool, budget_bytes=2 << 30, storage="f16")
    return {"workload": f"{len(trace)} jobs, Poisson arrivals at {qps:.1f} jobs/s ({args.serve_load:.0%} of the "
                        f"measured batched capacity), side log-uniform 256-4096, 1 or 4 bands, region/edge 50/50, "
                        f"100-300 iterations, sigma 1.5 / 11x11; inputs cut from a resident 4096^2 pool scene",
            "capacity": {"Mpixel_iter_per_s": round(cap_pxit / 1e6, 1),
                         "jobs_per_s": round(cap_pxit / mean_work, 2), "probe_jobs": len(probe)},
            "batched_f16_200GB": served.summary(), "plain_f32": plain.summary(),
            "batched_f16_2GB_first300": small.summary(),
            "mask_disagreement_batched_f16_vs_plain_f32": {"all_pixels": dis / px, "worst_job": worst}}


def main():
    args = parse()
    if args.profile_summary:
        print(profile_summary(args.profile_summary))
        return
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
    img = torch.tensor(scene.image, dtype=torch.float32, device=dev)
    masks = {"region": torch.tensor(scene.init_region, device=dev),
             "edge": torch.tensor(scene.init_edge, device=dev)}
    params = {t: lse.make_params(h, w, b, term=t, sigma=sigma, ksize=ksize) for t in terms}
    for p in params.values():
        p.image_dtype = 0
    # The solves of the two terms are independent: each has its own workspace
    # and HIP stream (default priority), so their latency-bound steps overlap
    # on the device.  The region solve (step + normaliser per iteration, the
    # longer chain) may use every CU; the edge solve's stream is limited to
    # 7/8 of them, so some CUs always have room for the region tiles.  A
    # sequential pass on one stream (the region one) is timed as well.
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    edge_cus = ncu * 7 // 8
    streams = {t: torch.cuda.Stream(dev) for t in terms}
    sids = {t: int(streams[t].cuda_stream) for t in terms}
    if "edge" in sids and len(terms) > 1:
        try:
            sids["edge"] = cu_masked_stream(ncu, 0, edge_cus)
        except RuntimeError as e:  # the line then states the schedule that ran
            print(f"bench.py: {e}; the edge solve runs on all CUs", file=sys.stderr)
            edge_cus = ncu
    ws, ws_ptr, nbytes = {}, {}, {}
    for t in terms:
        nbytes[t] = lse.lse_workspace_bytes(params[t])
        ws[t] = torch.empty(nbytes[t] + 256, dtype=torch.uint8, device=dev)
        ws_ptr[t] = ws[t].data_ptr() + ((-ws[t].data_ptr()) % 256)
    mask_out = {t: torch.empty((h, w), dtype=torch.uint8, device=dev) for t in terms}
    chunk = 20  # iterations enqueued per term in turn, so both streams start at once

    # Kernel durations come from events carried by the dispatch of one step
    # and normaliser launch in 8 (iterations 7, 15, ...): the events of a
    # timed launch cost the device a few microseconds, so timing every launch
    # would lower the throughput being measured.
    def job(profile_into=None, flags=lse.PROFILE_TIMING | lse.PROFILE_SAMPLE(3), concurrent=True):
        one = sids[terms[0]]
        sid = {t: (sids[t] if concurrent else one) for t in terms}
        ctx = {}
        for t in terms:
            ctx[t] = lse.lse_init(params[t], img.data_ptr(), masks[t].data_ptr(), ws_ptr[t], nbytes[t], sid[t])
            if profile_into is not None:
                lse.lse_profile(ctx[t], flags)
        if concurrent:
            for k0 in range(0, iters, chunk):
                for t in terms:
                    lse.lse_run(ctx[t], min(chunk, iters - k0), False, sid[t])
        else:
            for t in terms:
                lse.lse_run(ctx[t], iters, False, sid[t])
        for t in terms:
            lse.lse_mask(ctx[t], mask_out[t].data_ptr(), sid[t])
        for t in terms:
            if profile_into is not None:
                p = lse.lse_profile_read(ctx[t])
                acc = profile_into.setdefault(t, {"step_ms": 0.0, "step_n": 0, "mpass_ms": 0.0, "mpass_n": 0,
                                                  "needed_px": 0, "counted": 0})
                acc["step_ms"] += p.step_ms
                acc["step_n"] += p.step_launches
                acc["mpass_ms"] += p.mpass_ms
                acc["mpass_n"] += p.mpass_launches
                acc["needed_px"] += p.needed_pixels
                acc["counted"] += p.counted_steps
                acc["dense_bytes_per_px"] = lse.lse_step_bytes_per_pixel(ctx[t])
        torch.cuda.synchronize()
        for t in terms:
            lse.lse_destroy(ctx[t])

    conc = args.job != "sequential"
    for _ in range(args.warmup):
        job(concurrent=conc)
    torch.cuda.synchronize()
    prof = {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        job(prof, concurrent=conc)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    px_it = h * w * iters * len(terms) * args.steps
    value = px_it / elapsed / 1e6
    inside = {t: round(float(mask_out[t].float().mean().item()), 4) for t in terms}
    concurrent_masks = {t: mask_out[t].clone() for t in terms}
    # The same job with the two solves one after the other on one stream.
    prof_seq, sequential = prof, None
    if args.job == "both":
        prof_seq = {}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            job(prof_seq, concurrent=False)
        torch.cuda.synchronize()
        seq_elapsed = time.perf_counter() - t0
        sequential = {"ms_per_step": round(seq_elapsed * 1e3 / args.steps, 3),
                      "value": round(px_it / seq_elapsed / 1e6, 1),
                      "masks_equal_to_concurrent": all(torch.equal(concurrent_masks[t], mask_out[t]) for t in terms)}

    # Algorithmic bytes of the step kernel: an untimed replay of the same
    # (deterministic) job counts, per step, the pixels whose image value the
    # step needs; each costs one pixel of image (region: B x 4 bytes) or edge
    # map (4 bytes); the binary state adds one bit read and one bit written.
    counted = {}
    job(counted, lse.PROFILE_COUNT, concurrent=conc)
    torch.cuda.synchronize()
    if sids.get("edge") not in (None, int(streams["edge"].cuda_stream)):
        destroy_stream(sids["edge"])

    def step_bytes(t):
        c = counted[t]
        per_px = 4.0 * b if t == "region" else 4.0
        return per_px * c["needed_px"] / max(c["counted"], 1) + 2.0 * h * w / 8.0

    dom = "region" if "region" in prof else terms[0]
    kname = f"lse::step_fast_kernel<{ksize // 2}, {(4 if b == 3 else b) if dom == 'region' else 1}, " \
            f"{'false' if dom == 'region' else 'true'}, float>"
    traffic, traffic_src = measured_traffic(kname)

    def roofline_of(pf):
        pr = pf[dom]
        step_ms = pr["step_ms"] / max(pr["step_n"], 1)
        alg = step_bytes(dom)
        achieved = alg / (step_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": traffic_src,
                "kernel": f"step_fast_kernel ({dom} term, B={b})", "mean_launch_us": round(step_ms * 1e3, 2),
                "algorithmic_bytes_per_launch": int(alg),
                "needed_pixel_fraction": round(counted[dom]["needed_px"] / max(counted[dom]["counted"], 1) / (h * w),
                                               4)}

    # roofline: the region step with the device to itself (the timed
    # sequential pass), where the dispatch-packet events and a rocprofv3
    # kernel trace agree.  roofline_concurrent: the same kernel in the timed
    # two-stream job; there the events of a launch also count time spent
    # waiting for CUs that the other stream's kernels hold, and read ~15 %
    # above the trace's kernel durations.
    conc_note = ("two concurrent solves: dispatch-packet events include waits for CUs held by the other "
                 "stream and read ~15 % above rocprofv3 kernel durations")
    if conc and prof_seq is not prof:
        roofline = dict(roofline_of(prof_seq), **{"pass": "sequential"})
        roofline_conc = dict(roofline_of(prof), **{"pass": "concurrent", "note": conc_note})
    elif conc:
        roofline = dict(roofline_of(prof), **{"pass": "concurrent", "note": conc_note})
        roofline_conc = None
    else:
        roofline = dict(roofline_of(prof), **{"pass": "sequential"})
        roofline_conc = None
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
                               f"sigma {sigma}, {ksize}x{ksize} template, dt 15, image resident in HBM; "
                               + (f"the {len(terms)} independent solves on concurrent HIP streams, "
                                  f"the edge one on {edge_cus} of the {ncu} CUs" if conc
                                  else f"the {len(terms)} solves one after the other on one HIP stream"),
                   "global_batch": 1, "parallelism": "single GPU"},
        "sequential": sequential,
        "roofline": roofline, "roofline_concurrent": roofline_conc, "per_term": per_term,
        "final_mask_inside_fraction": inside,
        "gpu": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, sigma, ksize, args.cpu_iters, terms)
    sections = [x for x in args.sections.split(",") if x]
    if "batched" in sections:
        out["batched"] = section_batched(args)
    if "precision" in sections:
        out["precision"] = section_precision(args)
    if "serving" in sections:
        out["serving"] = section_serving(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
