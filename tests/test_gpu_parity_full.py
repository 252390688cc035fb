"""Full-size GPU parity, in the launch configuration the benchmark times.

* The 1000-track event: accumulator, peak list and every one of its rz
  records (all peaks are candidates), under the autotuner's cached tuning.
* The 4096-event batch: every event's accumulator and peak list, produced by
  replays of the captured HIP graph under the cached tuning.

The oracle runs across the host's cores (tests/oracle_pool.py); results are
compared bit for bit, per event through digests of the exact bytes, with an
in-process diff of the first differing event.
"""
import numpy as np
import pytest

import oracle
import oracle_pool
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_7556_amd import hough
    hough.load_library()
    return hough


def cached_tuning(spec, n_events, n_hits):
    from paper_1310_7556_amd import tune
    t = tune.cached(spec, n_events, n_hits)
    print(f"cached tuning: {t}", flush=True)
    return t


def test_c2_every_rz_record_under_cached_tuning(H):
    import torch
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    ev = synth.gen_config(name)
    ctx = H.HoughContext(spec, max_events=1, max_hits=ev.n_hits)
    t = cached_tuning(spec, 1, ev.n_hits)
    if t:
        ctx.set_tuning(**t)
    hits = H.DeviceHits.from_batch(ev)
    cap = ctx.cells
    acc = ctx.vote(hits)
    pk, poff = ctx.peaks(acc, 1, capacity=cap)
    rz, roff = ctx.rz_refine(hits, pk, poff, peak_capacity=cap, capacity=cap)
    torch.cuda.synchronize()
    tab = oracle.Tables(spec)
    A = oracle.vote_mask(tab, ev.layer, ev.phi)
    np.testing.assert_array_equal(H.acc_numpy(acc)[0], A)
    opk = oracle.peaks(tab, A)
    np.testing.assert_array_equal(H.peaks_numpy(pk, poff), opk.astype(H.PEAK_DTYPE))
    print(f"c2: {len(opk)} peaks; oracle rz over all of them ...", flush=True)
    orz = oracle_pool.rz_records(name, spec, opk)
    grz = H.rz_numpy(rz, roff)
    assert len(grz) == len(opk) == len(orz)
    diff = np.nonzero(grz != orz.astype(H.RZ_DTYPE))[0]
    assert len(diff) == 0, f"{len(diff)} rz records differ, first {diff[:5]}: {grz[diff[:3]]} vs {orz[diff[:3]]}"


def test_c4_graph_replays_every_event_under_cached_tuning(H):
    import torch
    name = "c4_batch_4096"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    E = batch.n_events
    ctx = H.HoughContext(spec, max_events=E, max_hits=batch.n_hits)
    t = cached_tuning(spec, E, batch.n_hits)
    if t:
        ctx.set_tuning(**t)
    hits = H.DeviceHits.from_batch(batch)
    acc = ctx.new_acc(E)
    cap = E * ctx.cells
    pk, poff = ctx.new_peaks(cap), ctx.new_offsets(E)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = ctx.graph_capture(hits, acc, pk, cap, poff, stream=stream)
    print("c4: oracle digests of all events ...", flush=True)
    want = oracle_pool.event_digests(name, spec, range(E))
    for rep in range(2):
        acc.fill_(-1)
        pk.fill_(-1)
        torch.cuda.synchronize()
        g.launch(stream)
        stream.synchronize()
        print(f"c4: replay {rep} done, comparing", flush=True)
        A = H.acc_numpy(acc)
        off = H.offsets_numpy(poff).astype(np.int64)
        assert off[-1] <= cap
        P = pk[:int(off[-1])].cpu().numpy().view(H.PEAK_DTYPE).reshape(-1)
        bad = [e for e in range(E)
               if (oracle_pool.digest(A[e]), oracle_pool.digest(P[off[e]:off[e + 1]])) != want[e][:2]]
        if bad:
            e = bad[0]
            ev = batch.event(e)
            tab = oracle.Tables(spec)
            OA, opk, _ = oracle.run_event(tab, ev.layer, ev.phi, with_rz=False)
            np.testing.assert_array_equal(A[e], OA, err_msg=f"replay {rep}: accumulator of event {e}")
            np.testing.assert_array_equal(P[off[e]:off[e + 1]], opk.astype(H.PEAK_DTYPE),
                                          err_msg=f"replay {rep}: peaks of event {e}")
        assert not bad, f"replay {rep}: {len(bad)} events differ"
        # eager work on the same context between the replays
        ctx.vote(hits, acc)
        torch.cuda.synchronize()
    g.close()
