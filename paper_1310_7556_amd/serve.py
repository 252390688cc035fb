"""Trigger-style serving loop with continuous batching.

Events (requests) arrive over time.  A request is admitted as soon as a
stream slot is free and the device bytes of everything in flight stay within
an HBM budget; all waiting requests that fit are admitted together as one
micro-batch, which runs the whole path (assembly, vote, peaks, rz) on that
slot's stream while other slots' micro-batches run on theirs.  Accumulators
and peak/rz buffers live on the device for the life of the server, so a
request never pays an allocation.  The paper motivates keeping data
resident on the accelerator across frames (Section 6.2, data persistence on
the coprocessor) and notes that small events cost a fixed overhead (the
small-event plateau of Section 7); batching arrivals removes that overhead.

The scheduler is plain Python and backend-agnostic, so its policy (FIFO
order, budget, slot reuse, latency bookkeeping) is tested on the CPU with a
fake clock and backend; the GPU backend drives libhough.so.
"""
import collections
import ctypes as C
import dataclasses
import os
import time

import numpy as np


class Roctx:
    """roctx ranges and marks for timelines of the serving loop (visible
    under `rocprofv3 --marker-trace`); every call is a no-op when ROCm's
    roctx library cannot be loaded."""

    def __init__(self):
        self.lib = None
        root = os.environ.get("ROCM_PATH", "/opt/rocm")
        for name in ("libroctx64.so", os.path.join(root, "lib", "libroctx64.so")):
            try:
                self.lib = C.CDLL(name)
                break
            except OSError:
                continue
        if self.lib is not None:
            self.lib.roctxRangePushA.argtypes = [C.c_char_p]
            self.lib.roctxMarkA.argtypes = [C.c_char_p]

    def push(self, msg):
        if self.lib is not None:
            self.lib.roctxRangePushA(msg.encode())

    def pop(self):
        if self.lib is not None:
            self.lib.roctxRangePop()

    def mark(self, msg):
        if self.lib is not None:
            self.lib.roctxMarkA(msg.encode())


ROCTX = Roctx()


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds on the trace clock
    event: int              # index into the event pool
    n_hits: int
    nbytes: int             # device bytes held while in flight
    admitted: float = None
    done: float = None
    slot: int = -1


class Scheduler:
    """FIFO admission of requests into stream slots under a byte budget.

    A slot holds one micro-batch at a time.  When a slot is free,
    next_batch() takes waiting requests in arrival order while the batch has
    at most max_batch events and max_batch_hits hits and the bytes of all
    in-flight requests stay within budget_bytes.  max_batch_hits is also the
    slots' hit capacity: a request with more hits can never be served and is
    refused when it arrives (ValueError).  A request whose bytes alone exceed
    the budget is admitted alone when nothing else is in flight, so the queue
    cannot stall."""

    def __init__(self, n_slots, max_batch, max_batch_hits, budget_bytes):
        self.queue = collections.deque()
        self.free = collections.deque(range(n_slots))
        self.max_batch = max_batch
        self.max_batch_hits = max_batch_hits
        self.budget = budget_bytes
        self.in_flight_bytes = 0
        self.batches = {}

    def arrive(self, req):
        if req.n_hits > self.max_batch_hits:
            raise ValueError(f"request {req.rid}: {req.n_hits} hits exceed the slot capacity of "
                             f"{self.max_batch_hits} hits")
        self.queue.append(req)

    @property
    def idle(self):
        return not self.batches

    def next_batch(self):
        if not self.free or not self.queue:
            return None, []
        batch, hits, nbytes = [], 0, 0
        while self.queue and len(batch) < self.max_batch:
            r = self.queue[0]
            alone = not batch and not self.batches
            if batch and hits + r.n_hits > self.max_batch_hits:
                break
            if self.in_flight_bytes + nbytes + r.nbytes > self.budget and not alone:
                break
            batch.append(self.queue.popleft())
            hits += r.n_hits
            nbytes += r.nbytes
            if alone and r.nbytes > self.budget:
                break
        if not batch:
            return None, []
        slot = self.free.popleft()
        self.in_flight_bytes += nbytes
        self.batches[slot] = (batch, nbytes)
        for r in batch:
            r.slot = slot
        return slot, batch

    def complete(self, slot):
        batch, nbytes = self.batches.pop(slot)
        self.in_flight_bytes -= nbytes
        self.free.append(slot)
        return batch


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def wait_until(self, t):
        # spin briefly: sleeps are far coarser than the service times here
        while self.now() < t:
            pass


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)


class FakeBackend:
    """Completes a micro-batch service_time(batch) after its launch."""

    def __init__(self, clock, service_time):
        self.clock = clock
        self.service_time = service_time
        self.finish = {}
        self.launches = []

    def launch(self, slot, batch):
        self.launches.append((slot, [r.rid for r in batch], self.clock.now()))
        self.finish[slot] = self.clock.now() + self.service_time(batch)

    def next_completion(self):
        return min(self.finish.values()) if self.finish else None

    def poll(self):
        now = self.clock.now()
        done = [(s, t) for s, t in self.finish.items() if t <= now]
        for s, _ in done:
            del self.finish[s]
        return done


def run_trace(requests, scheduler, backend, clock):
    """Serves `requests` (sorted by arrival) in real or simulated time and
    fills each request's admitted/done times (trace clock)."""
    n = len(requests)
    i = 0
    completed = 0
    while completed < n:
        now = clock.now()
        while i < n and requests[i].arrival <= now:
            scheduler.arrive(requests[i])
            i += 1
        for slot, t_done in backend.poll():
            for r in scheduler.complete(slot):
                r.done = t_done
                completed += 1
        while True:
            slot, batch = scheduler.next_batch()
            if slot is None:
                break
            t = clock.now()
            for r in batch:
                r.admitted = t
            backend.launch(slot, batch)
        if completed >= n:
            break
        # advance to the next thing that can happen
        nxt = [t for t in (requests[i].arrival if i < n else None, backend.next_completion()) if t is not None]
        if nxt:
            clock.wait_until(min(nxt))
    return requests


def latency_stats(requests):
    lat = np.array([r.done - r.arrival for r in requests])
    t_first = min(r.arrival for r in requests)
    t_last = max(r.done for r in requests)
    return dict(n=len(requests), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                events_per_s=len(requests) / (t_last - t_first))


# --------------------------------------------------------------------------
# GPU backend
# --------------------------------------------------------------------------

class GpuBackend:
    """Per-slot stream, library context and device-resident buffers; a
    micro-batch is assembled from a device-resident event pool by the
    library's gather kernel (hits pre-staged on the device) or copied from a
    pinned host pool (async H2D), then voted, peak-searched and rz-refined
    on the slot's stream.  Completion times come from HIP events."""

    def __init__(self, H, torch, spec, pool, n_slots, max_batch, max_batch_hits, clock,
                 staged=True, keep=None):
        self.H, self.torch, self.spec = H, torch, spec
        self.clock = clock
        self.staged = staged
        self.keep = set(keep or [])
        self.kept = {}
        self.pool_off = pool.offsets.astype(np.int64)
        self.pool_dev = H.DeviceHits.from_batch(pool) if staged else None
        if not staged:
            self.pool_host = [torch.from_numpy(np.ascontiguousarray(a).view(v)).pin_memory()
                              for a, v in ((pool.layer, np.uint8), (pool.phi, np.int32), (pool.z, np.int32))]
        dev = torch.device("cuda")
        self.slots = []
        self.cells = spec["n_d0"] * spec["n_qpt"] * spec["n_phi"]
        cap = spec["rz_max_candidates"]
        for _ in range(n_slots):
            ctx = H.HoughContext(spec, max_events=max_batch, max_hits=max_batch_hits)
            sl = dict(
                ctx=ctx, stream=torch.cuda.Stream(),
                layer=torch.empty(max_batch_hits, dtype=torch.uint8, device=dev),
                phi=torch.empty(max_batch_hits, dtype=torch.int32, device=dev),
                z=torch.empty(max_batch_hits, dtype=torch.int32, device=dev),
                idx_host=torch.empty((3, max_batch + 1), dtype=torch.int64).pin_memory(),
                idx=torch.empty((3, max_batch + 1), dtype=torch.int64, device=dev),
                acc=ctx.new_acc(max_batch),
                pcap=max_batch * self.cells,
                rcap=max_batch * (cap if cap else self.cells),
                done=torch.cuda.Event(enable_timing=True), batch=None)
            sl["pk"], sl["poff"] = ctx.new_peaks(sl["pcap"]), ctx.new_offsets(max_batch)
            sl["rz"], sl["roff"] = ctx.new_rz(sl["rcap"]), ctx.new_offsets(max_batch)
            self.slots.append(sl)
        self.ref = torch.cuda.Event(enable_timing=True)
        self.t_ref = None

    def start(self):
        """Pins the GPU timeline to the trace clock (call right before run_trace)."""
        self.torch.cuda.synchronize()
        self.ref.record(self.slots[0]["stream"])
        self.ref.synchronize()
        self.t_ref = self.clock.now()

    def launch(self, slot, batch):
        sl = self.slots[slot]
        n = len(batch)
        ev = np.array([r.event for r in batch], np.int64)
        lens = np.array([r.n_hits for r in batch], np.int64)
        ih = sl["idx_host"].numpy()
        ih[0, :n] = self.pool_off[ev]
        ih[1, :n] = lens
        ih[2, 0] = 0
        np.cumsum(lens, out=ih[2, 1:n + 1])
        total = int(ih[2, n])
        if total > sl["layer"].numel():
            # checked before anything is copied: the slot's arrays hold max_batch_hits
            raise ValueError(f"micro-batch of {total} hits exceeds the slot capacity of "
                             f"{sl['layer'].numel()} hits")
        s = sl["stream"]
        ROCTX.push(f"slot {slot}: micro-batch of {n} events, {total} hits")
        try:
            self._enqueue(sl, s, n, ih, total)
        finally:
            ROCTX.pop()
        sl["batch"] = batch

    def _enqueue(self, sl, s, n, ih, total):
        """Enqueue one micro-batch's assembly, vote, peaks and rz on slot
        stream s, then its completion event."""
        H, torch = self.H, self.torch
        with torch.cuda.stream(s):
            sl["idx"].copy_(sl["idx_host"], non_blocking=True)
            if self.staged:
                H.gather_events(self.pool_dev, sl["idx"][0], sl["idx"][1], sl["idx"][2], n,
                                sl["layer"], sl["phi"], sl["z"], stream=s)
            else:
                for i in range(n):
                    a, m, d = int(ih[0, i]), int(ih[1, i]), int(ih[2, i])
                    for dst, src in zip((sl["layer"], sl["phi"], sl["z"]), self.pool_host):
                        dst[d:d + m].copy_(src[a:a + m], non_blocking=True)
            h = H.Hits()
            h.layer, h.phi, h.z_um = sl["layer"].data_ptr(), sl["phi"].data_ptr(), sl["z"].data_ptr()
            h.event_offsets = sl["idx"][2].data_ptr()
            h.n_events, h.n_hits = n, total
            ctx, lib, sp = sl["ctx"], sl["ctx"].lib, C.c_void_p(s.cuda_stream)
            H._check(lib.hough_vote(ctx._h, C.byref(h), C.c_void_p(sl["acc"].data_ptr()), sp), ctx._h, "vote")
            H._check(lib.hough_peaks(ctx._h, C.c_void_p(sl["acc"].data_ptr()), n, C.c_void_p(sl["pk"].data_ptr()),
                                     sl["pcap"], C.c_void_p(sl["poff"].data_ptr()), sp), ctx._h, "peaks")
            if self.spec["n_z0"]:
                H._check(lib.hough_rz_refine(ctx._h, C.byref(h), C.c_void_p(sl["pk"].data_ptr()), sl["pcap"],
                                             C.c_void_p(sl["poff"].data_ptr()), C.c_void_p(sl["rz"].data_ptr()),
                                             sl["rcap"], C.c_void_p(sl["roff"].data_ptr()), sp), ctx._h, "rz")
            sl["done"].record(s)

    def next_completion(self):
        # completions are discovered by polling; report "now" while work is pending
        return self.clock.now() if any(sl["batch"] is not None for sl in self.slots) else None

    def poll(self):
        out = []
        for i, sl in enumerate(self.slots):
            if sl["batch"] is not None and sl["done"].query():
                t_done = self.t_ref + self.ref.elapsed_time(sl["done"]) * 1e-3
                ROCTX.mark(f"slot {i}: micro-batch of {len(sl['batch'])} events done")
                if self.keep:
                    self._keep_results(sl)
                sl["batch"] = None
                out.append((i, t_done))
        return out

    def _keep_results(self, sl):
        H = self.H
        n = len(sl["batch"])
        # a micro-batch of n events writes offsets[0..n] only
        poff, roff = sl["poff"][:n + 1], sl["roff"][:n + 1]
        for j, r in enumerate(sl["batch"]):
            if r.rid not in self.keep:
                continue
            acc = H.acc_numpy(sl["acc"][j:j + 1])[0].copy()
            pk = H.peaks_numpy(sl["pk"], poff, j).copy()
            rz = H.rz_numpy(sl["rz"], roff, j).copy() if self.spec["n_z0"] else None
            self.kept[r.rid] = (acc, pk, rz)


def make_requests(pool, rate_hz, n, arrivals, device_bytes):
    sizes = np.diff(pool.offsets.astype(np.int64))
    reqs = []
    for i in range(n):
        e = i % pool.n_events
        reqs.append(Request(rid=i, arrival=float(arrivals[i]), event=e, n_hits=int(sizes[e]),
                            nbytes=int(device_bytes(int(sizes[e])))))
    return reqs


def bench_serving(H, torch, log=print, rates=(250, 500, 1000, 2000, 5000, 10000, 20000, 50000, 100000),
                  modes=("staged", "h2d"), seconds=1.0, max_events=4000, plain_events=1000, pool_events=64,
                  n_slots=4, max_batch=16):
    """Latency/throughput sweep of the serving workload: continuous batching
    vs the plain one-event-per-launch FIFO path on the same arrival traces,
    for each mode: "staged" (the event pool resident on the device, a
    micro-batch assembled by the gather kernel) and "h2d" (the pool in pinned
    host memory, each micro-batch copied host-to-device asynchronously on its
    slot's stream)."""
    import synth
    name = "c5_serving"
    spec = synth.grid_spec(name)
    pool = synth.gen_batch(name, pool_events)
    sizes = np.diff(pool.offsets.astype(np.int64))
    cells = spec["n_d0"] * spec["n_qpt"] * spec["n_phi"]
    cap = spec["rz_max_candidates"]

    def device_bytes(n_hits):
        return 9 * n_hits + 2 * cells + 8 * cells + 16 * cap

    free, _ = torch.cuda.mem_get_info()
    budget = int(min(4 << 30, free // 4))
    max_hits = int(max(sizes.max(), min(sizes.sum(), max_batch * np.mean(sizes) * 2)))
    out = dict(workload=f"{name}: Poisson arrivals, pool of {pool_events} events "
                        f"(mean {sizes.mean():.0f} hits, max {sizes.max()}), 512x512 + rz, "
                        f"rz_max_candidates {cap}", budget_bytes=budget,
               slots=n_slots, max_batch=max_batch, modes={})
    clock = WallClock()
    for mode in modes:
        staged = mode == "staged"
        cb = GpuBackend(H, torch, spec, pool, n_slots, max_batch, max_hits, clock, staged=staged)
        plain = GpuBackend(H, torch, spec, pool, 1, 1, int(sizes.max()), clock, staged=staged)
        res = dict(hits_on_device=staged,
                   description=("event pool resident in HBM, micro-batches assembled on the device" if staged
                                else "event pool in pinned host memory, each micro-batch copied host to "
                                     "device asynchronously on its slot's stream"),
                   rates=[])
        for rate in rates:
            n = int(min(max_events, max(500, rate * seconds)))
            arr = synth.arrival_times(name, rate, n)
            row = dict(rate_hz=rate)
            for label, be, slots, mb, nreq in (("batched", cb, n_slots, max_batch, n),
                                                ("plain", plain, 1, 1, min(n, plain_events))):
                reqs = make_requests(pool, rate, nreq, arr, device_bytes)
                sched = Scheduler(slots, mb, max_hits if mb > 1 else int(sizes.max()), budget)
                be.start()
                t_start = clock.now()
                for r in reqs:
                    r.arrival += t_start
                run_trace(reqs, sched, be, clock)
                row[label] = latency_stats(reqs)
            log(f"serving [{mode}] {rate}/s: batched p50 {row['batched']['p50_ms']:.2f} ms p99 "
                f"{row['batched']['p99_ms']:.2f} ms {row['batched']['events_per_s']:.0f} ev/s | plain p50 "
                f"{row['plain']['p50_ms']:.2f} p99 {row['plain']['p99_ms']:.2f} "
                f"{row['plain']['events_per_s']:.0f} ev/s")
            res["rates"].append(row)
        out["modes"][mode] = res
        del cb, plain
        torch.cuda.empty_cache()
    return out
