"""Oracle runs spread over host processes, for full-size parity tests.

Test infrastructure only.  Workers regenerate the seeded events themselves
(from the workload name and the event index) and run the CPU oracle on them,
returning per-event digests of the exact result bytes, so a test can compare
every event of a 4096-event batch, or every rz record of a large event,
without shipping gigabytes between processes.  A digest mismatch names the
event; the test then recomputes that event in-process for a readable diff.
"""
import multiprocessing as mp
import os

import numpy as np

try:
    import xxhash

    def digest(*arrays):
        h = xxhash.xxh3_128()
        for a in arrays:
            h.update(np.ascontiguousarray(a).view(np.uint8).reshape(-1).data)
        return h.hexdigest()
except ImportError:                     # pragma: no cover - xxhash ships with this image
    import hashlib

    def digest(*arrays):
        h = hashlib.blake2b(digest_size=16)
        for a in arrays:
            h.update(np.ascontiguousarray(a).view(np.uint8).reshape(-1).data)
        return h.hexdigest()


PEAK_DTYPE = np.dtype([("cell", np.uint32), ("mask", np.uint16), ("popcount", np.uint16)])
RZ_DTYPE = np.dtype([("peak", np.uint32), ("cot_bin", np.uint16), ("z0_bin", np.uint16),
                     ("count", np.uint32), ("n_members", np.uint32)])


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def _event_digests(args):
    name, spec, events, with_rz = args
    import oracle
    import synth
    tab = oracle.Tables(spec)
    out = []
    for e in events:
        ev = synth.gen_batch(name, 1, first_event=e)
        A, pk, rz = oracle.run_event(tab, ev.layer, ev.phi, ev.z, with_rz=with_rz)
        out.append((e, digest(A), digest(pk.astype(PEAK_DTYPE)),
                    digest(rz.astype(RZ_DTYPE)) if with_rz else None))
    return out


def event_digests(name, spec, events, with_rz=False):
    """{event: (accumulator digest, peak-list digest, rz digest or None)} of
    the oracle on events `events` of workload `name` under grid `spec`."""
    events = list(events)
    n = workers()
    chunks = [events[i::n] for i in range(n)]
    with mp.get_context("spawn").Pool(n) as pool:
        res = pool.map(_event_digests, [(name, spec, c, with_rz) for c in chunks if c])
    return {e: (a, p, r) for part in res for e, a, p, r in part}


def _rz_chunk(args):
    name, spec, first, peaks = args
    import oracle
    import synth
    tab = oracle.Tables(spec)
    ev = synth.gen_batch(name, 1)
    r = oracle.rz(tab, ev.layer, ev.phi, ev.z, peaks)
    r["peak"] += np.uint32(first)
    return first, r.astype(RZ_DTYPE)


def rz_records(name, spec, peaks, chunk=16384):
    """The oracle's rz records of event 0 of workload `name` for every peak
    of `peaks` (candidates in list order, no cap), computed in chunks of
    consecutive peaks across the host's cores; `peak` indexes the full list."""
    assert spec["rz_max_candidates"] == 0
    jobs = [(name, spec, i, peaks[i:i + chunk]) for i in range(0, len(peaks), chunk)]
    with mp.get_context("spawn").Pool(workers()) as pool:
        res = sorted(pool.map(_rz_chunk, jobs), key=lambda t: t[0])
    return np.concatenate([r for _, r in res]) if res else np.zeros(0, RZ_DTYPE)
