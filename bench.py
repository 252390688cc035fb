"""Benchmark of the Hough-transform track finder on one MI355X.

Prints one JSON line.  The headline step is one pass of the whole hot path
(layer bucketing, vote, peak finding, rz refinement) over the 1000-track
event with 10,000 noise hits on a 1024 x 1024 (q/pT, phi0) grid plus the
256 x 256 (cot theta, z0) refinement, with its hits already resident in HBM.
`value` is Hough votes per second: rphi votes (hits x q/pT rows) per step
over the measured step time.  Per-kernel durations come from HIP events
recorded on the kernels' own stream inside the timed region.

Also reported, in the same line:
  single_events -- the 100-track event (256 x 256) and the displaced
              10,000-track event (512 x 512 x 64 d0): time per event, votes/s,
              peak volume, dominant kernel's HBM roofline, oracle beside it;
  batched  -- 4096 events (lognormal sizes) as one captured HIP graph vs a
              loop of per-event launches on the same GPU, with the vote
              kernel's HBM roofline;
  serving  -- the continuous-batching request loop against the plain
              one-event-per-launch path, with the event pool resident on the
              device and with async host-to-device copies, each labelled;
  cpu_baseline -- the CPU oracle timed on this host (bounded sample, median
              of several passes, CPU model recorded).
GPU step times are means over the timed steps, with per-step HIP-event
p10/p50/p90 beside them.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Hough votes/s and events/s (1k-track event); batched vs plain; serving p99 latency"
HBM_PEAK_GBS = 8000.0
# int32 vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# LDS atomics: 32 banks per CU, one read-modify-write per bank every two
# cycles (an estimate from the LDS width, not a published figure)
LDS_ATOMIC_PEAK = 256 * 32 / 2 * 2.4e9
# integer operations per rz (member, cot bin) vote: z - Z, - z0_lo, range
# test, * n_z0, / span, histogram increment, running-maximum compare
RZ_OPS_PER_VOTE = 7
# Algorithmic HBM bytes of the vote kernels for n_hits hits and `cells`
# accumulator cells: the per-hit scatter reads layer + phi (5 B) and writes
# each uint16 cell once; the bucket-bounds and gap forms split that into a
# scan that reads the hits and a tile kernel that writes the cells.
VOTE_KERNEL_BYTES = {
    "vote_lds": lambda n_hits, cells: 5 * n_hits + 2 * cells,
    "vote_bounds": lambda n_hits, cells: 5 * n_hits,
    "vote_direct": lambda n_hits, cells: 2 * cells,
    "vote_scan": lambda n_hits, cells: 5 * n_hits,
    "vote_gaps": lambda n_hits, cells: 2 * cells,
    # rank form: whole events per workgroup read their hits and write their
    # cells in one kernel; one tile per workgroup reads a bounds table
    # written by vote_bounds
    "vote_rank_event": lambda n_hits, cells: 5 * n_hits + 2 * cells,
    "vote_rank_tile": lambda n_hits, cells: 2 * cells,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_avg_ms(times, name):
    n, ms = times.get(name, (0, 0.0))
    return ms / n if n else float("nan")


def apply_cached_tuning(ctx, torch, spec, n_events, n_hits):
    """The autotuner's cached launch parameters for this workload, applied
    to ctx; returns them, or "default" when the cache has no entry."""
    from paper_1310_7556_amd import tune
    t = tune.cached(spec, n_events, n_hits)
    if not t:
        return "default"
    ctx.set_tuning(**t)
    return t


def bench_single(H, torch, steps, warmup):
    import synth
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    ev = synth.gen_config(name)
    ctx = H.HoughContext(spec, max_events=1, max_hits=ev.n_hits)
    tuning = apply_cached_tuning(ctx, torch, spec, 1, ev.n_hits)
    hits = H.DeviceHits.from_batch(ev)
    acc = ctx.new_acc(1)
    cap = ctx.cells
    pk, poff = ctx.new_peaks(cap), ctx.new_offsets(1)
    rz, roff = ctx.new_rz(cap), ctx.new_offsets(1)
    stream = torch.cuda.current_stream()

    def step():
        ctx.vote(hits, acc)
        ctx.peaks(acc, 1, capacity=cap, peaks=pk, offsets=poff)
        ctx.rz_refine(hits, pk, poff, peak_capacity=cap, capacity=cap, out=rz, offsets=roff)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times_reset()
    ctx.set_profiling(True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for i in range(steps):
        step()
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_profiling(False)
    times = ctx.kernel_times()
    per_step = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(steps)])
    n_peaks = int(H.offsets_numpy(poff)[-1])
    rzrec = H.rz_numpy(rz, roff)
    members = int(rzrec["n_members"].astype(np.int64).sum())
    rphi_votes = ev.n_hits * spec["n_qpt"] * spec["n_d0"]
    rz_votes = members * spec["n_cot"]
    ms = dt / steps * 1e3
    stage = {k: round(v[1] / v[0], 5) for k, v in times.items() if v[0]}
    dom = max(times, key=lambda k: times[k][1])
    out = dict(ms_per_step=ms, rphi_votes=rphi_votes, rz_votes=rz_votes, n_peaks=n_peaks,
               n_hits=ev.n_hits, stage_ms=stage, dominant=dom, stream=int(stream.cuda_stream), tuning=tuning,
               step_ms_percentiles=percentiles(per_step))
    # roofline of the dominant kernel
    if dom == "rz_vote":
        t = kernel_avg_ms(times, "rz_vote") * 1e-3
        achieved = rz_votes * RZ_OPS_PER_VOTE / t / 1e12
        out["roofline"] = dict(kernel="rz_vote", bound="alu", achieved=round(achieved, 4),
                               peak=round(ALU_PEAK_TOPS, 2), unit="TOP/s",
                               frac=round(achieved / ALU_PEAK_TOPS, 5), traffic=recorded_traffic("rz_vote"),
                               work_per_launch=f"{rz_votes} member x cot votes x {RZ_OPS_PER_VOTE} int ops")
    else:
        t = kernel_avg_ms(times, dom) * 1e-3
        byts = VOTE_KERNEL_BYTES.get(dom, lambda n_hits, cells: 2 * cells)(ev.n_hits, ctx.cells)
        gbs = byts / t / 1e9
        out["roofline"] = dict(kernel=dom, bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS,
                               unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 5), traffic=recorded_traffic(dom))
    out["rz_votes_per_s"] = rz_votes / (ms * 1e-3)
    # k_rz_vote_fast issues one LDS atomic add per (member, cot bin) vote of
    # the members that can vote in range in a 64-cot pass (the others are
    # skipped, their votes would all land in the trash counter); the count
    # of those atomics comes from the SQ counters in profiles/ (64 lanes
    # per SQ_INSTS_LDS_ATOMIC wave-instruction) while the kernel source is
    # unchanged, else it is not reported
    t_rz = kernel_avg_ms(times, "rz_vote") * 1e-3
    sq = recorded_counters("rz_vote")
    counted = int(sq["SQ_INSTS_LDS_ATOMIC"] * 64) if sq and "SQ_INSTS_LDS_ATOMIC" in sq else None
    out["atomics"] = dict(kernel="rz_vote", space="lds", votes_algorithmic=rz_votes,
                          per_launch_counted=counted,
                          per_s=(counted / t_rz) if counted else None, peak_estimate=LDS_ATOMIC_PEAK,
                          frac=round(counted / t_rz / LDS_ATOMIC_PEAK, 5) if counted else None,
                          valu_wave_instr_counted=int(sq["SQ_INSTS_VALU"]) if sq and "SQ_INSTS_VALU" in sq
                          else None)
    return out, (spec, ev)


def percentiles(ms):
    """p10 / p50 / p90 of per-step HIP-event durations (ms)."""
    ms = np.asarray(ms, np.float64)
    return dict(p10=round(float(np.percentile(ms, 10)), 5), p50=round(float(np.percentile(ms, 50)), 5),
                p90=round(float(np.percentile(ms, 90)), 5), n=int(ms.size))


# Algorithmic HBM bytes of the peak kernels: the count pass reads every
# cell once; the write pass reads every cell again and writes each 8-byte
# peak record.
PEAK_KERNEL_BYTES = {
    "peaks_count": lambda cells, peaks: 2 * cells,
    "peaks_write": lambda cells, peaks: 2 * cells + 8 * peaks,
}


def bench_event(H, torch, name, steps=20, warmup=3):
    """One single-event workload without an rz stage (vote + peaks per
    step): time per event with percentiles, votes/s, the peak volume and the
    dominant kernel's HBM roofline."""
    import synth
    spec = synth.grid_spec(name)
    ev = synth.gen_config(name)
    ctx = H.HoughContext(spec, max_events=1, max_hits=ev.n_hits)
    tuning = apply_cached_tuning(ctx, torch, spec, 1, ev.n_hits)
    hits = H.DeviceHits.from_batch(ev)
    acc = ctx.new_acc(1)
    cap = ctx.cells
    pk, poff = ctx.new_peaks(cap), ctx.new_offsets(1)
    stream = torch.cuda.current_stream()

    def step():
        ctx.vote(hits, acc)
        ctx.peaks(acc, 1, capacity=cap, peaks=pk, offsets=poff)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times_reset()
    ctx.set_profiling(True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    marks[0].record(stream)
    for i in range(steps):
        step()
        marks[i + 1].record(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ctx.set_profiling(False)
    times = ctx.kernel_times()
    per_step = [marks[i].elapsed_time(marks[i + 1]) for i in range(steps)]
    n_peaks = int(H.offsets_numpy(poff)[-1])
    votes = ev.n_hits * spec["n_qpt"] * spec["n_d0"]
    dom = max(times, key=lambda k: times[k][1])
    t = kernel_avg_ms(times, dom) * 1e-3
    if dom in VOTE_KERNEL_BYTES:
        byts = VOTE_KERNEL_BYTES[dom](ev.n_hits, ctx.cells)
    else:
        byts = PEAK_KERNEL_BYTES.get(dom, lambda cells, peaks: 2 * cells)(ctx.cells, n_peaks)
    return dict(workload=name, n_hits=ev.n_hits, cells=ctx.cells, votes=votes, peaks=n_peaks,
                ms_per_event=round(dt * 1e3, 5), step_ms_percentiles=percentiles(per_step),
                events_per_s=1.0 / dt, votes_per_s=votes / dt,
                stage_ms={k: round(v[1] / v[0], 5) for k, v in times.items() if v[0]}, tuning=tuning,
                roofline=dict(kernel=dom, bound="hbm", achieved=round(byts / t / 1e9, 2), peak=HBM_PEAK_GBS,
                              unit="GB/s", frac=round(byts / t / 1e9 / HBM_PEAK_GBS, 5), bytes_per_launch=byts))


def cpu_baseline_event(name, runs=3):
    """The oracle on a single-event workload without an rz stage, one
    thread: vote and peaks on the full event, or for the displaced 3D event
    (6.5e9 votes, over a minute of oracle time) the vote over every 32nd hit
    scaled to all hits plus the peak search; median of `runs` passes."""
    import oracle
    import synth
    spec = synth.grid_spec(name)
    ev = synth.gen_config(name)
    tab = oracle.Tables(spec)
    sub = 32 if spec["n_d0"] > 1 else 1
    est = []
    for _ in range(runs):
        t0 = time.perf_counter()
        A = oracle.vote_mask(tab, ev.layer[::sub], ev.phi[::sub])
        t1 = time.perf_counter()
        oracle.peaks(tab, A)
        t2 = time.perf_counter()
        est.append((t1 - t0) * ev.n_hits / max(len(ev.layer[::sub]), 1) + (t2 - t1))
    dt = float(np.median(est))
    votes = ev.n_hits * spec["n_qpt"] * spec["n_d0"]
    return dict(value=votes / dt, unit="votes/s", cores=1, cpu_model=cpu_model(), kind="oracle",
                seconds=round(dt, 4), runs=runs,
                sample=("the full event: vote and peaks, single thread" if sub == 1 else
                        f"vote over every {sub}th hit scaled to all {ev.n_hits} hits, plus the peak search, "
                        "single thread") + f"; median of {runs} passes")


def bench_batched(H, torch, reps=5):
    import synth
    name = "c4_batch_4096"
    spec = synth.grid_spec(name)
    t0 = time.perf_counter()
    batch = synth.gen_config(name)
    log(f"c4: generated {batch.n_events} events, {batch.n_hits} hits in {time.perf_counter() - t0:.1f}s")
    E = batch.n_events
    ctx = H.HoughContext(spec, max_events=E, max_hits=batch.n_hits)
    tuning = apply_cached_tuning(ctx, torch, spec, E, batch.n_hits)
    hits = H.DeviceHits.from_batch(batch)
    acc = ctx.new_acc(E)
    cap = E * ctx.cells
    pk, poff = ctx.new_peaks(cap), ctx.new_offsets(E)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = ctx.graph_capture(hits, acc, pk, cap, poff, stream=stream)
    g.launch(stream)
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.launch(stream)
    stream.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    total_peaks = int(H.offsets_numpy(poff)[-1])
    # per-kernel times of the batched path (eager, same kernels, events on stream)
    with torch.cuda.stream(stream):
        ctx.kernel_times_reset()
        ctx.set_profiling(True)
        for _ in range(2):
            ctx.vote(hits, acc, stream=stream)
            ctx.peaks(acc, E, capacity=cap, peaks=pk, offsets=poff, stream=stream)
        stream.synchronize()
        ctx.set_profiling(False)
        times = ctx.kernel_times()
    vk = next(k for k in ("vote_rank_event", "vote_rank_tile", "vote_direct", "vote_gaps", "vote_lds") if k in times)
    t_vote = kernel_avg_ms(times, vk) * 1e-3
    vote_bytes = VOTE_KERNEL_BYTES[vk](batch.n_hits, E * ctx.cells)
    gbs = vote_bytes / t_vote / 1e9
    stage_bytes = 5 * batch.n_hits + 2 * E * ctx.cells
    t_stage = sum(kernel_avg_ms(times, k) for k in ("vote_bounds", "vote_direct", "vote_scan", "vote_gaps",
                                                     "vote_lds", "bucket_layers", "vote_rank_event",
                                                     "vote_rank_tile")
                  if k in times) * 1e-3

    # the per-hit LDS-atomic form of the vote (the paper's recipe), timed once
    # for its atomic throughput: one LDS atomic OR per (hit, row)
    with torch.cuda.stream(stream):
        ctx.set_tuning(vote_algo=1)
        ctx.vote(hits, acc, stream=stream)
        stream.synchronize()
        ctx.kernel_times_reset()
        ctx.set_profiling(True)
        ctx.vote(hits, acc, stream=stream)
        stream.synchronize()
        ctx.set_profiling(False)
        t_atomic = kernel_avg_ms(ctx.kernel_times(), "vote_lds") * 1e-3
        if isinstance(tuning, dict):
            ctx.set_tuning(**tuning)
        else:
            ctx.set_tuning()
    n_atomics = batch.n_hits * spec["n_qpt"] * spec["n_d0"]
    atomics = dict(kernel="vote_lds", space="lds", per_launch=n_atomics, per_s=n_atomics / t_atomic,
                   peak_estimate=LDS_ATOMIC_PEAK, frac=round(n_atomics / t_atomic / LDS_ATOMIC_PEAK, 5),
                   ms=round(t_atomic * 1e3, 3))

    # plain path: one event per launch, same kernels, same GPU
    import ctypes as C
    lib = ctx.lib
    offs_dev = torch.zeros((E, 2), dtype=torch.int64, device="cuda")
    sizes = np.diff(batch.offsets.astype(np.int64))
    offs_dev[:, 1] = torch.from_numpy(sizes).cuda()
    pctx = H.HoughContext(spec, max_events=1, max_hits=int(sizes.max()))
    pacc = pctx.new_acc(1)
    ppk, ppoff = pctx.new_peaks(pctx.cells), pctx.new_offsets(1)
    structs = []
    for e in range(E):
        h = H.Hits()
        a = int(batch.offsets[e])
        h.layer = hits.layer.data_ptr() + a
        h.phi = hits.phi.data_ptr() + 4 * a
        h.z_um = None
        h.event_offsets = offs_dev.data_ptr() + 16 * e
        h.n_events = 1
        h.n_hits = int(sizes[e])
        structs.append(h)
    sp = C.c_void_p(stream.cuda_stream)
    acc_p, pk_p, poff_p = C.c_void_p(pacc.data_ptr()), C.c_void_p(ppk.data_ptr()), C.c_void_p(ppoff.data_ptr())

    def plain():
        for e in range(E):
            lib.hough_vote(pctx._h, C.byref(structs[e]), acc_p, sp)
            lib.hough_peaks(pctx._h, acc_p, 1, pk_p, pctx.cells, poff_p, sp)

    plain()
    stream.synchronize()
    t0 = time.perf_counter()
    plain()
    stream.synchronize()
    t_plain = time.perf_counter() - t0
    votes = batch.n_hits * spec["n_qpt"]
    g.close()
    return dict(
        workload=name, n_events=E, n_hits=batch.n_hits, votes=votes, peaks=total_peaks, tuning=tuning,
        per_hit_atomic_vote=atomics,
        graph_ms=round(t_graph * 1e3, 3), events_per_s=E / t_graph, votes_per_s=votes / t_graph,
        plain_ms=round(t_plain * 1e3, 3), plain_events_per_s=E / t_plain,
        speedup_vs_plain=round(t_plain / t_graph, 3),
        stage_ms={k: round(v[1] / v[0], 4) for k, v in times.items() if v[0]},
        roofline=dict(kernel=vk, bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS,
                      unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 5), traffic=recorded_traffic(vk),
                      bytes_per_launch=vote_bytes),
        vote_stage=dict(kernels_ms=round(t_stage * 1e3, 4), bytes=stage_bytes,
                        achieved_gbs=round(stage_bytes / t_stage / 1e9, 2),
                        frac=round(stage_bytes / t_stage / 1e9 / HBM_PEAK_GBS, 5)),
        vote_alu=vote_alu_view(vk, E * ctx.cells, spec["n_layers"], t_vote))


# --- HBM traffic of the dominant kernels ---------------------------------
# `--traffic-probe` runs, once each: a plain device-to-device copy of
# COPY_BYTES (the calibration kernel), one c2 step and one c4 vote + peaks.
# It is meant to run under `rocprofv3 --pmc FETCH_SIZE` and, separately,
# `--pmc WRITE_SIZE`; `--summarize-traffic FETCH_CSV WRITE_CSV` turns the two
# counter files into TRAFFIC_FILE.  A kernel's entry holds the SHA-256 of its
# source file, and the bench reports `traffic` only while it still matches.
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sq_counters.json")
TRAFFIC_KERNELS = {
    # bench name: (rocprofv3 kernel-name prefix, source file, workload); the
    # probe's largest dispatch of a prefix is the named workload's
    "rz_vote": ("hough::k_rz_vote_fast", "paper_1310_7556_amd/csrc/k_rz.hip", "c2_single_1ktrk_rz"),
    "vote_direct": ("hough::k_vote_direct", "paper_1310_7556_amd/csrc/k_vote_direct.hip", "c2_single_1ktrk_rz"),
    "vote_rank_tile": ("hough::k_vote_rank<2, 10, true, false>", "paper_1310_7556_amd/csrc/k_vote_rank.hip",
                       "c4_batch_4096"),
    "vote_rank_event": ("hough::k_vote_rank<2, 10, true, true>", "paper_1310_7556_amd/csrc/k_vote_rank.hip",
                        "c4_batch_4096"),
    "peaks_count": ("hough::(anonymous namespace)::k_peaks_rows<8, false, false>",
                    "paper_1310_7556_amd/csrc/k_peaks_rows.hip", "c4_batch_4096"),
    "peaks_write": ("hough::(anonymous namespace)::k_peaks_rows<8, true, false>",
                    "paper_1310_7556_amd/csrc/k_peaks_rows.hip", "c4_batch_4096"),
}
# SQ counters of the counter profiles: two passes of at most 8 SQ counters
COUNTER_PASSES = (
    "SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAIT_ANY "
    "SQ_ACTIVE_INST_VALU",
    "SQ_INSTS_VMEM SQ_INSTS_LDS_ATOMIC SQ_LDS_BANK_CONFLICT SQ_LDS_ADDR_CONFLICT SQ_WAIT_INST_LDS "
    "SQ_ACTIVE_INST_LDS SQ_INSTS_BRANCH SQ_INST_CYCLES_SALU",
)


def source_sha(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_probe(H, torch):
    import synth
    src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    log("probe: copy")
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    from paper_1310_7556_amd import tune
    log(f"probe: device {tune.device_name(torch)}")
    log("probe: c2 step")
    name = "c2_single_1ktrk_rz"
    spec, ev = synth.grid_spec(name), synth.gen_config(name)
    ctx = H.HoughContext(spec, max_events=1, max_hits=ev.n_hits)
    log(f"probe: c2 tuning {apply_cached_tuning(ctx, torch, spec, 1, ev.n_hits)}")
    hits = H.DeviceHits.from_batch(ev)
    acc = ctx.vote(hits)
    pk, poff = ctx.peaks(acc, 1, capacity=ctx.cells)
    ctx.rz_refine(hits, pk, poff, capacity=ctx.cells)
    torch.cuda.synchronize()
    del ctx, hits, acc, pk, poff
    log("probe: c4 vote + peaks")
    name = "c4_batch_4096"
    spec, batch = synth.grid_spec(name), synth.gen_config(name)
    E = batch.n_events
    ctx = H.HoughContext(spec, max_events=E, max_hits=batch.n_hits)
    log(f"probe: c4 tuning {apply_cached_tuning(ctx, torch, spec, E, batch.n_hits)}")
    hits = H.DeviceHits.from_batch(batch)
    acc = ctx.vote(hits)
    ctx.peaks(acc, E, capacity=E * ctx.cells)
    torch.cuda.synchronize()
    log("probe: done")


def summarize_counters(paths):
    """Per-dispatch SQ counter totals (summed over the XCDs' rows) of the
    probe's kernels from rocprofv3 counter CSVs: the largest dispatch of each
    TRAFFIC_KERNELS prefix, written to COUNTERS_FILE (with each kernel's
    source hash) and printed as a markdown table with derived rates."""
    import csv
    disp = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"][5:] if r["Kernel_Name"].startswith("void ") else r["Kernel_Name"]
            d = disp.setdefault((path, r["Dispatch_Id"]), dict(name=name, grid=int(r["Grid_Size"]),
                                                               wg=int(r["Workgroup_Size"]), c={}))
            d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    rows = {}
    for label, (prefix, _, workload) in TRAFFIC_KERNELS.items():
        merged = {}
        for path in paths:
            cands = [d for (p, _), d in disp.items() if p == path and d["name"].startswith(prefix)]
            if cands:
                big = max(cands, key=lambda d: d["grid"])
                merged.update(big["c"])
                merged["_grid"], merged["_wg"] = big["grid"], big["wg"]
        if merged:
            rows[label] = (workload, merged)
    record = {label: dict(workload=wl, source=TRAFFIC_KERNELS[label][1],
                          sha256=source_sha(TRAFFIC_KERNELS[label][1]),
                          grid=c["_grid"], workgroup=c["_wg"],
                          counters={k: v for k, v in c.items() if not k.startswith("_")})
              for label, (wl, c) in rows.items()}
    with open(COUNTERS_FILE, "w") as fh:
        json.dump(record, fh, indent=1)
    names = sorted({k for _, c in rows.values() for k in c if not k.startswith("_")})
    print("| kernel (workload) | " + " | ".join(names) + " |")
    print("|---|" + "---|" * len(names))
    for label, (wl, c) in rows.items():
        print(f"| {label} ({wl}) | " + " | ".join(f"{c[n]:.4g}" if n in c else "" for n in names) + " |")
    print()
    for label, (wl, c) in rows.items():
        out = []
        if "SQ_WAVE_CYCLES" in c and "SQ_WAIT_ANY" in c:
            out.append(f"waiting {c['SQ_WAIT_ANY'] / c['SQ_WAVE_CYCLES']:.2f} of wave cycles")
        if "SQ_BUSY_CYCLES" in c and "SQ_INSTS_VALU" in c:
            # VALU wave-instructions per SIMD per busy cycle (4 cycles each at full rate)
            out.append(f"VALU {c['SQ_INSTS_VALU']:.3g} wave-instr")
        if "SQ_INSTS_LDS_ATOMIC" in c:
            out.append(f"LDS atomics {c['SQ_INSTS_LDS_ATOMIC']:.3g} wave-instr")
        if "SQ_WAVES" in c:
            out.append(f"{c['SQ_WAVES']:.0f} waves, grid {c['_grid']}, workgroup {c['_wg']}")
        print(f"* {label}: " + "; ".join(out))


def summarize_traffic(fetch_csv, write_csv):
    import csv
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"][5:] if r["Kernel_Name"].startswith("void ") else r["Kernel_Name"]
            per.setdefault((counter, name), []).append(float(r["Counter_Value"]) * 1024.0)

    def largest(counter, prefix):
        # the probe's largest dispatch of the kernel is the named workload's
        vals = [v for (c, k), vs in per.items() if c == counter and k.startswith(prefix) for v in vs]
        return (max(vals), len(vals)) if vals else (None, 0)

    # the copy moves COPY_BYTES each way; blit launches of other copies are far smaller
    big_f = max(v for (c, k), vs in per.items() if c == "FETCH_SIZE" and k.startswith("__amd_rocclr_copyBuffer")
                for v in vs)
    big_w = max(v for (c, k), vs in per.items() if c == "WRITE_SIZE" and k.startswith("__amd_rocclr_copyBuffer")
                for v in vs)
    ff, fw = COPY_BYTES / big_f, COPY_BYTES / big_w
    out = dict(calibration=dict(copy_bytes=COPY_BYTES, fetch_counter_bytes=big_f, write_counter_bytes=big_w,
                                fetch_factor=ff, write_factor=fw),
               kernels={})
    for name, (prefix, src, workload) in TRAFFIC_KERNELS.items():
        f, nf = largest("FETCH_SIZE", prefix)
        w, nw = largest("WRITE_SIZE", prefix)
        if f is None or w is None:
            continue
        out["kernels"][name] = dict(source=src, sha256=source_sha(src), workload=workload, dispatches=[nf, nw],
                                    fetch_bytes=f * ff, write_bytes=w * fw, bytes_per_launch=f * ff + w * fw)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def recorded_counters(name):
    """SQ counters of kernel `name` from COUNTERS_FILE, or None when absent or
    when its source has changed since they were taken."""
    try:
        with open(COUNTERS_FILE) as fh:
            k = json.load(fh)[name]
    except (OSError, KeyError, ValueError):
        return None
    return k["counters"] if source_sha(k["source"]) == k["sha256"] else None


def recorded_traffic(name):
    """HBM bytes per launch of kernel `name` from TRAFFIC_FILE, or None when
    absent or when its source has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            k = json.load(fh)["kernels"][name]
    except (OSError, KeyError, ValueError):
        return None
    return round(k["bytes_per_launch"]) if source_sha(k["source"]) == k["sha256"] else None


# Lane operations per (cell, layer) decision of the vote forms that decide
# every cell: the direct form uses three VALU instructions per 64 decisions
# (subtract, subtract with borrow, add with carry); the rank form five per
# 4 x 64 (two subtracts, a three-input bit operation, a shift and a bit-field
# insert on four byte lanes).  Their ALU roof, beside the HBM one.
VOTE_LANE_OPS_PER_DECISION = {"vote_direct": 3.0, "vote_rank_event": 1.25, "vote_rank_tile": 1.25}


def vote_alu_view(kernel, cells, layers, seconds):
    """ALU roofline of a deciding vote form: cells x layers decisions per launch."""
    per = VOTE_LANE_OPS_PER_DECISION.get(kernel)
    if per is None:
        return None
    decisions = cells * layers
    ops = decisions * per                                  # lane operations
    alu_floor = ops / (ALU_PEAK_TOPS * 1e12)
    return dict(decisions_per_launch=decisions, lane_ops_per_decision=per,
                achieved_tops=round(ops / seconds / 1e12, 3), peak_tops=round(ALU_PEAK_TOPS, 2),
                frac=round(alu_floor / seconds, 5), alu_floor_ms=round(alu_floor * 1e3, 4),
                hbm_floor_ms=round(2 * cells / (HBM_PEAK_GBS * 1e9) * 1e3, 4))


def bench_count_form(H, torch, reps=5):
    """The paper's counting accumulator on its own detector and 2048 x 2048
    grid: time per event (count vote + count peaks) against the number of
    tracks, the shape of the paper's Figure 2 (no noise, 0.4 mm hits)."""
    import synth
    name = "p6_paper_2048_count"
    spec = synth.grid_spec(name)
    cfg = synth.CONFIGS[name]
    ctx = H.HoughContext(spec, max_events=1, max_hits=1 << 17)
    cnt = ctx.new_counts(1)
    cap = ctx.cells
    pk, poff = ctx.new_peaks(cap), ctx.new_offsets(1)
    sweep = []
    for n_tracks in (100, 300, 1000, 3000, 5000):
        rng = np.random.default_rng(np.random.SeedSequence(0, spawn_key=(cfg["index"], n_tracks)))
        layer, phi, z, _ = synth.gen_event(cfg, rng, n_tracks=n_tracks)
        hits = H.DeviceHits.from_batch(synth.concat_events([(layer, phi, z)]))
        ctx.vote_count(hits, cnt)
        ctx.peaks_count(cnt, 1, capacity=cap, peaks=pk, offsets=poff)
        torch.cuda.synchronize()
        ctx.kernel_times_reset()
        ctx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.vote_count(hits, cnt)
            ctx.peaks_count(cnt, 1, capacity=cap, peaks=pk, offsets=poff)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        ctx.set_profiling(False)
        kt = ctx.kernel_times()
        sweep.append(dict(tracks=n_tracks, hits=len(layer), ms_per_event=round(dt * 1e3, 4),
                          votes_per_s=len(layer) * spec["n_qpt"] / dt,
                          peaks=int(H.offsets_numpy(poff)[-1]),
                          kernel_ms={k: round(v[1] / v[0], 4) for k, v in kt.items() if v[0]}))
    return dict(workload=name + ": paper detector (10 layers, r = 11 i cm), 2048 x 2048 counts, "
                "0.4 mm hits, no noise", sweep=sweep)


def bench_confirmation(H, torch, reps=5, c4_events=512):
    """Candidate confirmation after the peak search: plateau clusters of the
    peak list and the track fit of every cluster, on the single-event c2
    workload and on the first c4_events events of the c4 batch.  Kernel times
    from the library's HIP-event timers, averaged over reps calls; the
    oracle's clusters + fit of the c2 event timed beside it."""
    import synth
    out = {}
    for name, n_ev in (("c2_single_1ktrk_rz", None), ("c4_batch_4096", c4_events)):
        spec = synth.grid_spec(name)
        batch = synth.gen_config(name) if n_ev is None else synth.gen_batch(name, n_ev)
        E = batch.n_events
        cap = E * spec["n_qpt"] * spec["n_phi"] * spec["n_d0"]
        ctx = H.HoughContext(spec, max_events=E, max_hits=batch.n_hits, max_peaks=cap)
        hits = H.DeviceHits.from_batch(batch)
        pk, poff = ctx.peaks(ctx.vote(hits), E, capacity=cap)
        ccap = min(cap, 1 << 25)
        lab, cl, coff = ctx.peak_clusters(pk, poff, E, capacity=ccap)
        fits = ctx.cluster_fit(hits, pk, poff, cl, coff, peak_capacity=cap, capacity=ccap)
        torch.cuda.synchronize()
        ctx.kernel_times_reset()
        ctx.set_profiling(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.peak_clusters(pk, poff, E, capacity=ccap, labels=lab, out=cl, offsets=coff)
            ctx.cluster_fit(hits, pk, poff, cl, coff, peak_capacity=cap, capacity=ccap, out=fits)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        ctx.set_profiling(False)
        kt = {k: round(v[1] / v[0], 4) for k, v in ctx.kernel_times().items() if v[0]}
        n_pk = int(H.offsets_numpy(poff)[-1])
        n_cl = int(H.offsets_numpy(coff)[-1])
        f = H.fits_numpy(fits, coff)
        r = dict(events=E, peaks=n_pk, clusters=n_cl, fitted=int(np.count_nonzero(f["status"])),
                 mean_members=round(float(f["n_hits"].mean()), 2) if len(f) else 0.0,
                 ms_per_call=round(wall * 1e3, 4), kernel_ms=kt,
                 clusters_ms=round(sum(v for k, v in kt.items() if k.startswith("cluster_") and
                                       k != "cluster_fit") + kt.get("scan_counts", 0.0), 4),
                 fit_ms=round(kt.get("cluster_fit", 0.0) + kt.get("bucket_layers", 0.0), 4))
        if n_ev is None:
            import oracle
            tab = oracle.Tables(spec)
            ev = batch.event(0)
            opk = oracle.peaks(tab, oracle.vote_mask(tab, ev.layer, ev.phi))
            t1 = time.perf_counter()
            _, ocl = oracle.clusters(tab, opk)
            oracle.fit(tab, ev.layer, ev.phi, opk, ocl)
            r["oracle_s"] = round(time.perf_counter() - t1, 3)
        out[name] = r
        del ctx, pk, lab, cl, fits
        torch.cuda.empty_cache()
    return out


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), for the baseline records."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_event(args):
    spec, layer, phi = args
    import oracle
    tab = oracle.Tables(spec)
    A = oracle.vote_mask(tab, layer, phi)
    oracle.peaks(tab, A)
    return len(layer)


def cpu_baseline_batched(n_events=128, runs=5):
    """The oracle on a sample of the 4096-event batch, one event per worker
    process across the host cores (vote and peaks, as in the batched path);
    the median of `runs` passes over the same sample, pool start-up excluded."""
    import multiprocessing as mp
    import synth
    name = "c4_batch_4096"
    spec = synth.grid_spec(name)
    batch = synth.gen_batch(name, n_events)
    work = [(spec, batch.event(e).layer, batch.event(e).phi) for e in range(n_events)]
    cores = min(16, os.cpu_count() or 1)
    secs = []
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_event, work[:cores], chunksize=1)          # workers started and warm
        for _ in range(runs):
            t0 = time.perf_counter()
            hits = sum(pool.map(_oracle_event, work, chunksize=1))
            secs.append(time.perf_counter() - t0)
    dt = float(np.median(secs))
    return dict(value=hits * spec["n_qpt"] / dt, unit="votes/s", events_per_s=n_events / dt, cores=cores,
                cpu_model=cpu_model(), kind="oracle", seconds=round(dt, 3),
                seconds_min_max=[round(min(secs), 3), round(max(secs), 3)], runs=runs,
                sample=f"the first {n_events} events of the 4096-event batch ({hits} hits): vote and peaks, "
                       f"one event per process on {cores} host cores; median of {runs} passes")


def cpu_baseline(spec, ev, runs=5):
    """The oracle on the headline event, one thread: each of `runs` passes
    does the whole vote and peak search and the rz stage on one fifth of the
    candidates (every runs-th peak, a different fifth each pass), and its
    step time is the vote and peak time plus the rz time scaled to all
    candidates; the value is the median of the passes' rates."""
    import oracle
    tab = oracle.Tables(spec)
    est, parts = [], []
    for r in range(runs):
        t0 = time.perf_counter()
        A = oracle.vote_mask(tab, ev.layer, ev.phi)
        t1 = time.perf_counter()
        pk = oracle.peaks(tab, A)
        t2 = time.perf_counter()
        sub = pk[r::runs]
        oracle.rz(tab, ev.layer, ev.phi, ev.z, sub)
        t3 = time.perf_counter()
        step = (t1 - t0) + (t2 - t1) + (t3 - t2) * len(pk) / max(len(sub), 1)
        est.append(step)
        parts.append((t1 - t0, t2 - t1, t3 - t2))
    votes = ev.n_hits * spec["n_qpt"] * spec["n_d0"]
    dt = float(np.median(est))
    med = np.median(np.array(parts), axis=0)
    return dict(value=votes / dt, unit="votes/s", cores=1, cpu_model=cpu_model(), kind="oracle",
                seconds=round(dt, 3), seconds_min_max=[round(min(est), 3), round(max(est), 3)], runs=runs,
                stage_seconds=dict(vote=round(med[0], 4), peaks=round(med[1], 4),
                                   rz_fifth=round(med[2], 4)),
                sample=f"the 1000-track event ({ev.n_hits} hits, {len(pk)} peaks), single thread: per pass "
                       f"the full vote and peak search plus rz on every {runs}th candidate (a different "
                       f"{runs}th each pass) scaled to all candidates; median of {runs} passes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the copy/c2/c4 kernels once each (for rocprofv3 --pmc runs) and exit")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic file from two rocprofv3 counter CSVs and exit")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the c5 serving sweep (for a kernel trace of it) and print its JSON")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV",
                    help="print the SQ counters of the probe's kernels from rocprofv3 counter CSVs and exit")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: events are independent, so more GPUs would "
              "shard whole events with no exchange; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1310_7556_amd import hough as H
    H.load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.traffic_probe:
        traffic_probe(H, torch)
        return
    if args.serving_only:
        from paper_1310_7556_amd import serve
        print(json.dumps(serve.bench_serving(H, torch, log=log)))
        return

    log("c2 single-event steps ...")
    single, (spec, ev) = bench_single(H, torch, args.steps, args.warmup)
    log(f"c2: {single['ms_per_step']:.3f} ms/step, dominant {single['dominant']}")
    res = dict(
        metric=METRIC, value=single["rphi_votes"] / (single["ms_per_step"] * 1e-3), unit="votes/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=round(single["ms_per_step"], 4),
        higher_is_better=True, scaling="weak", vs_baseline=None, dtype="u32", data="synthetic",
        config=dict(workload="c2_single_1ktrk_rz: 1000 prompt tracks + 10000 noise hits, 1024x1024 "
                             "(q/pT, phi0) uint16 layer masks, threshold 8, rz 256x256",
                    n_hits=single["n_hits"], grid=[1024, 1024], rz=[256, 256]),
        events_per_s=1e3 / single["ms_per_step"],
        rz_votes_per_s=single["rz_votes_per_s"],
        atomics=single["atomics"],
        paper_context=("the paper prints no absolute timings; its Figure 2 (2048x2048 grid, toy Monte "
                       "Carlo) has a Tesla K20c about as fast as 2x Xeon E5-2697v2, Xeon Phi 7120P 3x and "
                       "i7-3770 5x slower at 5000 tracks"),
        step_ms_percentiles=single["step_ms_percentiles"],
        peaks_per_event=single["n_peaks"],
        stage_ms=single["stage_ms"],
        tuning=single["tuning"],
        roofline=single["roofline"],
    )
    res["single_events"] = {}
    for name in ("c1_single_100trk", "c3_pileup_displaced_3d"):
        log(f"{name} ...")
        r = bench_event(H, torch, name)
        res["single_events"][name] = r
        log(f"{name}: {r['ms_per_event']} ms/event, dominant {r['roofline']['kernel']} "
            f"{r['roofline']['frac']:.3f} of HBM")
    if not args.no_batched:
        log("c4 batched vs plain ...")
        res["batched"] = bench_batched(H, torch)
        log(f"c4: graph {res['batched']['graph_ms']} ms, plain {res['batched']['plain_ms']} ms")
    if not args.no_batched:
        log("paper-detector counting form sweep ...")
        res["count_form"] = bench_count_form(H, torch)
        log("count form: " + ", ".join(f"{x['tracks']} trk {x['ms_per_event']} ms"
                                       for x in res["count_form"]["sweep"]))
    if not args.no_batched:
        log("candidate confirmation: clusters and fit ...")
        res["confirmation"] = bench_confirmation(H, torch)
        log("confirmation: " + ", ".join(f"{k.split('_')[0]} {v['clusters']} clusters "
                                          f"{v['clusters_ms']}+{v['fit_ms']} ms"
                                          for k, v in res["confirmation"].items()))
    if not args.no_serving:
        from paper_1310_7556_amd import serve
        log("c5 serving sweep ...")
        res["serving"] = serve.bench_serving(H, torch, log=log)
    if not args.no_cpu:
        log("cpu oracle baseline ...")
        res["cpu_baseline"] = cpu_baseline(spec, ev)
        for name, r in res["single_events"].items():
            log(f"cpu oracle baseline, {name} ...")
            r["cpu_baseline"] = cpu_baseline_event(name)
        if not args.no_batched:
            log("cpu oracle baseline, batched sample ...")
            res["batched"]["cpu_baseline"] = cpu_baseline_batched()
    print(json.dumps(res))


if __name__ == "__main__":
    main()
