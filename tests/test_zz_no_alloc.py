"""hough_peaks_noalloc (peak search with static device scratch) against
hough_peaks: the same offsets and peak records bit for bit, on two calls in a
row through the C ABI, the second with a smaller input; and its size limit
is refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _noalloc(H, ctx, acc, n_events, cap):
    import torch
    pk, off = ctx.new_peaks(cap), ctx.new_offsets(n_events)
    pk.fill_(-1)
    off.fill_(-1)
    rc = ctx.lib.hough_peaks_noalloc(ctx._h, C.c_void_p(acc.data_ptr()), n_events, C.c_void_p(pk.data_ptr()),
                                     cap, C.c_void_p(off.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    H._check(rc, ctx._h, "hough_peaks_noalloc")
    return pk, off


def test_noalloc_peaks_equal_peaks_on_two_calls():
    import torch
    from paper_1310_7556_amd import hough as H
    name = "c4_batch_4096"
    spec = synth.grid_spec(name)
    big = synth.gen_batch(name, 48)
    small = synth.gen_batch(name, 5, first_event=100)
    ctx = H.HoughContext(spec, max_events=big.n_events, max_hits=big.n_hits)
    ctx.set_tuning(peak_rows=2)           # 48 x 256 tiles: the multi-block scan; 5 x 256: one block
    tab = oracle.Tables(spec)
    for batch in (big, small):
        E = batch.n_events
        print(f"noalloc: {E} events", flush=True)
        hits = H.DeviceHits.from_batch(batch)
        acc = ctx.vote(hits)
        cap = E * ctx.cells
        ref_pk, ref_off = ctx.peaks(acc, E, capacity=cap)
        pk, off = _noalloc(H, ctx, acc, E, cap)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(H.offsets_numpy(off), H.offsets_numpy(ref_off))
        np.testing.assert_array_equal(H.peaks_numpy(pk, off), H.peaks_numpy(ref_pk, ref_off))
        # and the first event against the oracle
        ev = batch.event(0)
        opk = oracle.peaks(tab, oracle.vote_mask(tab, ev.layer, ev.phi))
        np.testing.assert_array_equal(H.peaks_numpy(pk, off, 0), opk.astype(H.PEAK_DTYPE))


def test_noalloc_peaks_equal_peaks_with_a_d0_axis():
    """The same comparison on a grid with a d0 axis (5 planes) under the
    row-window form, whose tiles are (event, plane, strip)."""
    import torch
    from paper_1310_7556_amd import hough as H
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    spec.update(n_qpt=40, n_phi=256, n_d0=5, d0_lo_mm=-120.0, d0_hi_mm=120.0, n_z0=0, n_cot=0)
    evs = []
    for e, n in enumerate([3000, 0, 9000, 57, 4000, 1]):
        rng = np.random.default_rng(400 + e)
        evs.append((rng.integers(0, 10, n).astype(np.uint8),
                    rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                    rng.integers(-1_200_000, 1_200_000, n).astype(np.int32)))
    big = synth.concat_events(evs)
    small = synth.concat_events(evs[2:4])
    ctx = H.HoughContext(spec, max_events=big.n_events, max_hits=big.n_hits)
    ctx.set_tuning(peak_algo=2, peak_rows=8)
    tab = oracle.Tables(spec)
    for batch in (big, small):
        E = batch.n_events
        print(f"noalloc d0 axis: {E} events", flush=True)
        hits = H.DeviceHits.from_batch(batch)
        acc = ctx.vote(hits)
        cap = E * ctx.cells
        ref_pk, ref_off = ctx.peaks(acc, E, capacity=cap)
        pk, off = _noalloc(H, ctx, acc, E, cap)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(H.offsets_numpy(off), H.offsets_numpy(ref_off))
        np.testing.assert_array_equal(H.peaks_numpy(pk, off), H.peaks_numpy(ref_pk, ref_off))
        ev = batch.event(0)
        _, opk, _ = oracle.run_event(tab, ev.layer, ev.phi, ev.z, with_rz=False)
        np.testing.assert_array_equal(H.peaks_numpy(pk, off, 0), opk.astype(H.PEAK_DTYPE))


def test_noalloc_peaks_refuses_more_tiles_than_its_scratch():
    import torch
    from paper_1310_7556_amd import hough as H
    spec = synth.grid_spec("c3_pileup_displaced_3d")
    E = 24                                   # 24 x 64 x 512 one-row tiles > 8 MiB of scratch
    ctx = H.HoughContext(spec, max_events=E, max_hits=16)
    ctx.set_tuning(peak_rows=1)
    acc = ctx.new_acc(E)
    acc.zero_()
    pk, off = ctx.new_peaks(16), ctx.new_offsets(E)
    torch.cuda.synchronize()
    rc = ctx.lib.hough_peaks_noalloc(ctx._h, C.c_void_p(acc.data_ptr()), E, C.c_void_p(pk.data_ptr()), 16,
                                     C.c_void_p(off.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == H.HOUGH_ELIMIT
    assert b"static scratch" in ctx.lib.hough_last_error(ctx._h)
