"""Serving loop: segmentation jobs of different sizes admitted by HBM budget
and advanced together with continuous batching.

Every iteration of every job runs in the HIP library (lse_init, lse_batch_*,
lse_mask); this module only schedules.  Jobs arrive on a timeline (seconds
from the start of the run).  A job is admitted, first come first served, when
it has arrived and its workspace (lse_workspace_bytes) fits in the remaining
budget and a slot is free; admitted jobs keep their binary state and
statistics resident until they finish.  The running jobs form one batch
(lse_batch_create, then lse_batch_update whenever jobs join or leave: the
batch keeps its streams and nothing synchronises); the batch advances in
chunks of iterations, each chunk ending at the next job completion or after
`chunk` iterations, and jobs that arrived meanwhile join at chunk
boundaries, so new work overlaps running work on the device.  At most two
chunks are in flight; memory is released when the chunk that last used it
has completed.  Each job's result equals its solo run bit for bit (the batch
keeps per-image state and exact fixed-point statistics).

serve_plain runs the same trace one job at a time with plain FP32 solves
(lse_init + lse_run + lse_mask per job, in arrival order), for comparison.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

from . import lse


@dataclass
class JobRecord:
    job_id: int
    arrival_s: float
    pixels: int
    iters: int
    admitted_s: float = -1.0
    completed_s: float = -1.0
    mask: object = None                       # H x W uint8 device tensor (keep_masks)

    @property
    def latency_s(self) -> float:
        return self.completed_s - self.arrival_s


@dataclass
class ServeStats:
    records: list
    makespan_s: float
    pixel_iters: int
    max_running: int = 0
    max_queue: int = 0
    batches_created: int = 0
    batch_updates: int = 0
    chunks: int = 0
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        import numpy as np
        lat = np.array([r.latency_s for r in self.records])
        wait = np.array([r.admitted_s - r.arrival_s for r in self.records])
        return {"jobs": len(self.records), "makespan_s": round(self.makespan_s, 4),
                "value": round(self.pixel_iters / self.makespan_s / 1e6, 1), "unit": "Mpixel-iter/s",
                "jobs_per_s": round(len(self.records) / self.makespan_s, 2),
                "latency_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "latency_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                "latency_max_ms": round(float(lat.max()) * 1e3, 2),
                "queue_wait_p50_ms": round(float(np.percentile(wait, 50)) * 1e3, 2),
                "max_running": self.max_running, "max_queue": self.max_queue,
                "batches_created": self.batches_created, "batch_updates": self.batch_updates,
                "chunks": self.chunks, **self.extra}


def _params(job, storage, sigma, ksize):
    return lse.make_params(job.side, job.side, job.bands, term=job.term, sigma=sigma, ksize=ksize, storage=storage)


def _table_bound(workspace_bytes: int) -> int:
    """Upper bound of the bytes one job adds to a batch table: its argument
    record (160 B), 4 B per step tile and per normaliser group, and map
    alignment.  A step tile covers at least 4608 pixels, whose workspace
    holds at least 2.25 B per pixel, so 4 B per tile is below 1/2048 of the
    workspace; 1/256 plus 1 KiB leaves a wide margin."""
    return workspace_bytes // 256 + 1024


def _tensor_bytes(*ts) -> int:
    return sum(int(t.numel()) * t.element_size() for t in ts if t is not None)


def serve(trace, make_input, *, budget_bytes: int, storage: str = "f16", sigma: float = 1.5, ksize: int = 11,
          chunk: int = 16, max_slots: int = 512, keep_masks: bool = False, stream=None, clock=None):
    """Continuous-batching server over `trace` (objects with job_id,
    arrival_s, side, bands, term, iters).  make_input(job) returns the job's
    image (H x W x B float tensor on the device) and initial mask (H x W
    uint8).  Returns ServeStats.

    Device memory held by the server never exceeds budget_bytes: the
    workspaces of admitted jobs, their input tensors until lse_init has run,
    and the batch tables (the current one and those still read by chunks in
    flight) are all counted, and each is released only when the chunk that
    last used it has completed (its event has been waited for)."""
    import torch
    dev = torch.device("cuda:0")
    stream = stream if stream is not None else torch.cuda.Stream(dev)
    clock = clock or time.perf_counter
    pending = collections.deque(sorted(trace, key=lambda j: j.arrival_s))
    queue = collections.deque()
    running = []            # [job, LSE, record, done_iters, workspace bytes]
    inflight = collections.deque()   # [event, finished entries, held tensors, bytes released at retire]
    records = []
    used = 0                # workspaces, held inputs and live tables
    peak = 0
    batch, members = None, None
    table_bytes = 0         # the current table
    next_hold, next_bytes = [], 0    # held until the next chunk completes (inputs of new jobs)
    st = ServeStats(records=records, makespan_s=0.0, pixel_iters=0)
    ws_need = {}
    with torch.cuda.stream(stream):
        t0 = clock()
        while pending or queue or running or inflight:
            now = clock() - t0
            while pending and pending[0].arrival_s <= now:
                queue.append(pending.popleft())
            st.max_queue = max(st.max_queue, len(queue))
            # Admission: first come first served, by budget and slots.  Room
            # is left for the new table (the old one stays until its last
            # chunk completes).
            grow = 0
            while queue and len(running) < max_slots:
                job = queue[0]
                need = ws_need.get(job.job_id)
                if need is None:
                    need = ws_need[job.job_id] = lse.lse_workspace_bytes(_params(job, storage, sigma, ksize))
                    if need == 0:
                        raise ValueError(f"job {job.job_id}: invalid parameters")
                in_bytes = job.side * job.side * (4 * job.bands + 1)
                g = _table_bound(need)
                if need + in_bytes + 2 * g > budget_bytes:
                    raise ValueError(f"job {job.job_id} cannot be served within the budget")
                if used + need + in_bytes + table_bytes + grow + g > budget_bytes:
                    break
                queue.popleft()
                img, init = make_input(job)
                ctx = lse.LSE(img, init, term=job.term, sigma=sigma, ksize=ksize, storage=storage, stream=stream)
                ctx._keep = None  # the next chunk's retirement releases the inputs
                next_hold += [img, init]
                b_in = _tensor_bytes(img, init)
                next_bytes += b_in
                rec = JobRecord(job.job_id, job.arrival_s, job.side * job.side, job.iters, admitted_s=clock() - t0)
                records.append(rec)
                running.append([job, ctx, rec, 0, need])
                used += need + b_in
                grow += g
            st.max_running = max(st.max_running, len(running))
            if running:
                ids = [e[0].job_id for e in running]
                if ids != members:
                    jobs, targets = [e[1] for e in running], [e[0].iters for e in running]
                    if batch is None:
                        batch = lse.Batch(jobs, targets=targets, stream=stream)
                        st.batches_created += 1
                        old = None
                    else:
                        old = batch.update(jobs, targets=targets)
                        st.batch_updates += 1
                    new_bytes = batch.table_bytes
                    if new_bytes > table_bytes + grow + 256:
                        raise AssertionError("batch table larger than its reserve")
                    used += new_bytes
                    if old is not None:
                        # Read by the chunks already enqueued: released with the last of them.
                        if inflight:
                            inflight[-1][2].append(old)
                            inflight[-1][3] += table_bytes
                        else:
                            used -= table_bytes
                        del old
                    table_bytes = new_bytes
                    members = ids
                peak = max(peak, used)
                c = min(chunk, min(e[0].iters - e[3] for e in running))
                batch.run(c)
                st.chunks += 1
                finished = []
                for e in running:
                    e[3] += c
                    if e[3] >= e[0].iters:
                        finished.append(e)
                for e in finished:
                    if keep_masks:
                        e[2].mask = e[1].mask()
                    running.remove(e)
                    st.pixel_iters += e[2].pixels * e[2].iters
                if finished:
                    # The batch object no longer references finished jobs;
                    # this chunk's entry keeps them until it completes.
                    batch.jobs = [e[1] for e in running]
                ev = torch.cuda.Event()
                ev.record(stream)
                inflight.append([ev, finished, next_hold, next_bytes + sum(e[4] for e in finished)])
                next_hold, next_bytes = [], 0
            # Retire chunks: keep at most two in flight while there is work to
            # enqueue; otherwise wait for the oldest.
            while inflight and (len(inflight) > 2 or not running or inflight[0][0].query()):
                ev, fin, held, freed = inflight.popleft()
                ev.synchronize()
                t = clock() - t0
                for e in fin:
                    e[2].completed_s = t
                    e[1].close()
                    e[1] = None
                del fin, held
                used -= freed
            if not running and not inflight and not queue and pending:
                wait = pending[0].arrival_s - (clock() - t0)
                if wait > 0:
                    time.sleep(wait)
        st.makespan_s = clock() - t0
    if batch is not None:
        batch.close()
    st.extra["peak_reserved_bytes"] = peak
    st.extra["budget_bytes"] = budget_bytes
    records.sort(key=lambda r: r.job_id)
    return st


def serve_plain(trace, make_input, *, storage: str = "f32", sigma: float = 1.5, ksize: int = 11,
                keep_masks: bool = False, stream=None, clock=None):
    """One job at a time in arrival order: lse_init, lse_run, lse_mask."""
    import torch
    dev = torch.device("cuda:0")
    stream = stream if stream is not None else torch.cuda.Stream(dev)
    clock = clock or time.perf_counter
    records = []
    st = ServeStats(records=records, makespan_s=0.0, pixel_iters=0, max_running=1)
    with torch.cuda.stream(stream):
        t0 = clock()
        for job in sorted(trace, key=lambda j: j.arrival_s):
            wait = job.arrival_s - (clock() - t0)
            if wait > 0:
                time.sleep(wait)
            rec = JobRecord(job.job_id, job.arrival_s, job.side * job.side, job.iters, admitted_s=clock() - t0)
            img, init = make_input(job)
            ctx = lse.LSE(img, init, term=job.term, sigma=sigma, ksize=ksize, storage=storage, stream=stream)
            ctx.run(job.iters)
            m = ctx.mask()
            stream.synchronize()
            rec.completed_s = clock() - t0
            if keep_masks:
                rec.mask = m
            ctx.close()
            records.append(rec)
            st.pixel_iters += rec.pixels * rec.iters
        st.makespan_s = clock() - t0
    records.sort(key=lambda r: r.job_id)
    return st


class PoolInputs:
    """Serving inputs cut from a resident pool scene (synth.serving_pool):
    job i takes the side x side window synth.serving_window(job); single-band
    jobs take the band mean; the region term starts from the window's centred
    half-size square, the edge term from the pool's seeds in the window."""

    def __init__(self, pool_scene, device):
        import torch
        from . import synth
        self._synth = synth
        self.size = pool_scene.image.shape[0]
        self.img4 = torch.tensor(pool_scene.image, dtype=torch.float32, device=device)
        self.img1 = self.img4.mean(dim=2, keepdim=True).contiguous()
        self.seeds = torch.tensor(pool_scene.init_edge, dtype=torch.uint8, device=device)
        self.device = device

    def __call__(self, job):
        import torch
        y0, x0 = self._synth.serving_window(job, self.size)
        s = job.side
        src = self.img4 if job.bands == 4 else self.img1
        img = src[y0:y0 + s, x0:x0 + s, :].contiguous()
        if job.term == "region":
            init = torch.zeros((s, s), dtype=torch.uint8, device=self.device)
            q = (s - s // 2) // 2  # centred square of half the side, as synth.centred_square
            init[q:q + s // 2, q:q + s // 2] = 1
        else:
            init = self.seeds[y0:y0 + s, x0:x0 + s].contiguous()
        return img, init
