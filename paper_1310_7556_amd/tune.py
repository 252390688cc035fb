"""Autotuner for the library's launch parameters on a given workload.

Swept: the vote's algorithm, tile rows, threads per workgroup and
workgroups per compute unit; the peak search's tile rows; the rz stage's
waves per compute unit and LDS counter width (the fields of
`hough_tuning`).

Stages are tuned one after another (vote, then peaks, then rz), each with
the earlier stages' winners in place.  A candidate is run `reps` times and
timed with the library's own per-kernel HIP-event timers (the sum over the
stage's kernels); it is accepted only if its output equals the default
configuration's output bit for bit -- every result is an integer -- and
the accepted candidate with the smallest mean time wins.  Winners are
cached in a JSON file keyed by device, grid spec and workload shape.

    python -m paper_1310_7556_amd.tune c4_batch_4096      # tune, cache, print
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")


def vote_space():
    c = [dict(vote_algo=5, vote_items=i) for i in (1, 2)]
    c += [dict(vote_algo=4, vote_rows=r, vote_threads=t, vote_wgs_per_cu=w)
          for r in (8, 16) for t in (128, 256) for w in (2, 4, 8, 16)]
    c += [dict(vote_algo=3, vote_threads=t) for t in (256, 512)]
    c += [dict(vote_algo=1)]
    return c


def peak_space():
    return ([dict(peak_algo=2, peak_rows=r) for r in (4, 8, 16, 32, 64, 128)] +
            [dict(peak_algo=1, peak_rows=r) for r in (2, 4, 8, 16, 32, 64)])


def rz_space():
    return [dict(rz_waves_per_cu=w, rz_counter_bits=b) for w in (4, 8, 12, 16) for b in (0, 4, 8, 16)]


STAGES = (("vote", vote_space), ("peaks", peak_space), ("rz", rz_space))


def workload_key(spec, n_events, n_hits, device):
    """Cache key: device name, a hash of the grid spec, the batch size and
    the mean hits per event rounded to a power of two."""
    h = hashlib.sha256(json.dumps(spec, sort_keys=True).encode()).hexdigest()[:16]
    mean = max(1, n_hits // max(n_events, 1))
    return f"{device}|{h}|E{n_events}|H{2 ** round(math.log2(mean))}"


def load_cache(path=CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(key, path=CACHE):
    entry = load_cache(path).get(key)
    return None if entry is None else dict(entry["tuning"])


def store(key, tuning, info, path=CACHE):
    cache = load_cache(path)
    cache[key] = dict(tuning=tuning, info=info)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(runner, stages=STAGES, reps=3, log=None):
    """Sweep `stages` on `runner` (see GpuRunner for the interface).
    Returns (tuning, report): the winning field values merged over the
    stages, and per stage the default time, the winner's time and the
    candidates rejected for differing output."""
    tuning = {}
    report = {}
    for name, space in stages:
        base_ms = runner.time_stage(name, tuning, reps)
        best, best_ms, rejected, failed = {}, base_ms, [], []
        for cand in space():
            trial = dict(tuning, **cand)
            try:
                ok = runner.same_output(name, trial)
            except Exception as ex:                      # invalid for this spec
                failed.append((cand, str(ex)))
                continue
            if not ok:
                rejected.append(cand)
                continue
            ms = runner.time_stage(name, trial, reps)
            if log:
                log(f"  {name} {cand}: {ms:.4f} ms")
            if ms < best_ms:
                best, best_ms = cand, ms
        tuning.update(best)
        report[name] = dict(default_ms=base_ms, best_ms=best_ms, best=best, rejected=rejected,
                            invalid=len(failed))
        if log:
            log(f"{name}: default {base_ms:.4f} ms -> {best_ms:.4f} ms with {best}")
    return tuning, report


class GpuRunner:
    """Runs one stage of the path on a fixed batch with a given tuning.

    The reference outputs come from the default tuning; a stage's inputs
    (accumulator for peaks, peak list for rz) are the reference ones, so
    stages are timed and compared in isolation."""

    def __init__(self, H, torch, spec, batch, peak_capacity=None):
        self.H, self.torch = H, torch
        self.E = batch.n_events
        self.ctx = H.HoughContext(spec, max_events=self.E, max_hits=max(batch.n_hits, 1))
        self.hits = H.DeviceHits.from_batch(batch)
        self.has_rz = bool(spec["n_z0"])
        self.cap = peak_capacity or self.E * self.ctx.cells
        c = self.ctx
        self.ref_acc = c.vote(self.hits)
        self.ref_pk, self.ref_poff = c.peaks(self.ref_acc, self.E, capacity=self.cap)
        if self.has_rz:
            self.ref_rz, self.ref_roff = c.rz_refine(self.hits, self.ref_pk, self.ref_poff,
                                                     peak_capacity=self.cap, capacity=self.cap)
        torch.cuda.synchronize()
        self.acc = c.new_acc(self.E)
        self.pk, self.poff = c.new_peaks(self.cap), c.new_offsets(self.E)
        if self.has_rz:
            self.rz, self.roff = c.new_rz(self.cap), c.new_offsets(self.E)

    def _apply(self, tuning):
        self.ctx.set_tuning(**tuning)

    def _run(self, stage):
        c = self.ctx
        if stage == "vote":
            c.vote(self.hits, self.acc)
        elif stage == "peaks":
            c.peaks(self.ref_acc, self.E, capacity=self.cap, peaks=self.pk, offsets=self.poff)
        elif stage == "rz" and self.has_rz:
            c.rz_refine(self.hits, self.ref_pk, self.ref_poff, peak_capacity=self.cap, capacity=self.cap,
                        out=self.rz, offsets=self.roff)

    def same_output(self, stage, tuning):
        torch = self.torch
        self._apply(tuning)
        self._run(stage)
        torch.cuda.synchronize()
        if stage == "vote":
            return bool(torch.equal(self.acc, self.ref_acc))
        if stage == "peaks":
            n = min(int(self.H.offsets_numpy(self.ref_poff)[-1]), self.cap)
            return bool(torch.equal(self.poff, self.ref_poff) and torch.equal(self.pk[:n], self.ref_pk[:n]))
        if not self.has_rz:
            return True
        n = min(int(self.H.offsets_numpy(self.ref_roff)[-1]), self.cap)
        return bool(torch.equal(self.roff, self.ref_roff) and torch.equal(self.rz[:n], self.ref_rz[:n]))

    def time_stage(self, stage, tuning, reps):
        if stage == "rz" and not self.has_rz:
            return 0.0
        self._apply(tuning)
        self._run(stage)
        self.torch.cuda.synchronize()
        self.ctx.kernel_times_reset()
        self.ctx.set_profiling(True)
        for _ in range(reps):
            self._run(stage)
        self.torch.cuda.synchronize()
        self.ctx.set_profiling(False)
        return sum(ms for _, ms in self.ctx.kernel_times().values()) / reps


def device_name(torch, device=0):
    """Device part of the cache key: marketing name, ISA and CU count."""
    p = torch.cuda.get_device_properties(device)
    arch = getattr(p, "gcnArchName", "").split(":")[0]
    return f"{p.name}/{arch}/{p.multi_processor_count}cu".replace("|", "/")


def cached(spec, n_events, n_hits, device=0, path=CACHE):
    """The cached tuning of this workload shape on the current device, or
    None when the cache has no entry for it.  When the device's name is not
    in the cache (a profiler can report another marketing name), an entry
    for the same ISA and workload shape is used if there is exactly one."""
    import torch
    dev = device_name(torch, device)
    key = workload_key(spec, n_events, n_hits, dev)
    t = lookup(key, path)
    if t is not None:
        return t
    arch = dev.split("/")[-2] if dev.count("/") >= 2 else None
    shape = key.split("|", 1)[1]
    alike = [v for k, v in load_cache(path).items()
             if k.split("|", 1)[1:] == [shape] and arch and k.split("|")[0].split("/")[-2:-1] == [arch]]
    return dict(alike[0]["tuning"]) if len(alike) == 1 else None


def tune_workload(name, n_events=None, reps=3, cache=CACHE, log=print):
    """Tune the named synthetic workload (see synth.CONFIGS) and cache the
    result; returns (key, tuning, report)."""
    import torch

    from . import hough as H
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    spec = synth.grid_spec(name)
    if n_events:
        batch = synth.gen_batch(name, n_events)
    else:
        batch = synth.gen_config(name)
    t0 = time.perf_counter()
    runner = GpuRunner(H, torch, spec, batch, peak_capacity=min(batch.n_events * spec["n_qpt"] * spec["n_phi"]
                                                                  * spec["n_d0"], 1 << 28))
    tuning, report = tune(runner, reps=reps, log=log)
    key = workload_key(spec, batch.n_events, batch.n_hits, device_name(torch))
    info = dict(workload=name, n_events=batch.n_events, n_hits=batch.n_hits, report=report,
                seconds=round(time.perf_counter() - t0, 1))
    store(key, tuning, info, cache)
    return key, tuning, report


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload", help="a synthetic workload name, e.g. c4_batch_4096")
    ap.add_argument("--n-events", type=int, default=None)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=CACHE)
    a = ap.parse_args()
    key, tuning, report = tune_workload(a.workload, a.n_events, a.reps, a.cache,
                                        log=lambda *x: print(*x, flush=True))
    print(json.dumps(dict(key=key, tuning=tuning), indent=1))


if __name__ == "__main__":
    main()
