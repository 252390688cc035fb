"""The paper's counting accumulator (A[B[i]] += 1) and its local maxima on
the GPU against the CPU oracle, bit for bit: the paper-detector 2048x2048
workload in full, ragged batches under several tunings, a displaced 3D grid,
and the relation between counts and layer masks."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_1310_7556_amd import hough
    hough.load_library()
    return hough


def run_counts(H, spec, batch, tuning=None):
    import torch
    ctx = H.HoughContext(spec, max_events=max(batch.n_events, 1), max_hits=max(batch.n_hits, 1))
    if tuning:
        ctx.set_tuning(**tuning)
    hits = H.DeviceHits.from_batch(batch)
    cnt = ctx.vote_count(hits)
    pk, poff = ctx.peaks_count(cnt, batch.n_events)
    torch.cuda.synchronize()
    return ctx, hits, cnt, pk, poff


def check(H, spec, batch, cnt, pk, poff):
    tab = oracle.Tables(spec)
    got = H.counts_numpy(cnt)
    for e in range(batch.n_events):
        ev = batch.event(e)
        Cc = oracle.vote_count(tab, ev.layer, ev.phi)
        np.testing.assert_array_equal(got[e], Cc, err_msg=f"counts of event {e}")
        np.testing.assert_array_equal(H.count_peaks_numpy(pk, poff, e), oracle.peaks_count(tab, Cc),
                                      err_msg=f"count peaks of event {e}")


def test_paper_detector_2048_grid_full(H):
    name = "p6_paper_2048_count"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    _, _, cnt, pk, poff = run_counts(H, spec, batch)
    check(H, spec, batch, cnt, pk, poff)
    # the P2 invariant on the device: every hit votes once per row
    assert int(H.counts_numpy(cnt).astype(np.int64).sum()) == batch.n_hits * spec["n_qpt"]


def ragged():
    evs = []
    for e, n in enumerate([0, 1, 2500, 0, 57, 9000]):
        rng = np.random.default_rng(300 + e)
        layer = rng.integers(0, 10, n).astype(np.uint8)
        layer[::53] = 11
        evs.append((layer, rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32), np.zeros(n, np.int32)))
    return synth.concat_events(evs)


@pytest.mark.parametrize("tuning", [None, dict(vote_rows=1), dict(vote_rows=4, vote_threads=64),
                                    dict(vote_algo=2), dict(peak_rows=1), dict(peak_rows=5)])
def test_ragged_batches_under_tunings(H, tuning):
    spec = synth.grid_spec("c1_single_100trk")
    spec.update(n_qpt=48, n_phi=512, threshold=4)
    batch = ragged()
    _, _, cnt, pk, poff = run_counts(H, spec, batch, tuning)
    check(H, spec, batch, cnt, pk, poff)


def test_displaced_3d_grid(H):
    spec = synth.grid_spec("c3_pileup_displaced_3d")
    spec.update(n_qpt=32, n_phi=64, n_d0=16, d0_lo_mm=-120.0, d0_hi_mm=120.0, threshold=3)
    batch = ragged()
    _, _, cnt, pk, poff = run_counts(H, spec, batch)
    check(H, spec, batch, cnt, pk, poff)


def test_counts_bound_the_layer_masks(H):
    spec = synth.grid_spec("c1_single_100trk")
    batch = synth.gen_config("c1_single_100trk")
    ctx, hits, cnt, _, _ = run_counts(H, spec, batch)
    acc = ctx.vote(hits)
    import torch
    torch.cuda.synchronize()
    m = H.acc_numpy(acc)
    pop = np.zeros(m.shape, np.int64)
    for b in range(10):
        pop += (m >> b) & 1
    c = H.counts_numpy(cnt).astype(np.int64)
    assert (c >= pop).all() and ((c > 0) == (m > 0)).all()
