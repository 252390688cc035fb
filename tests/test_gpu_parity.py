"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer work, so the bar is bit-exact equality: accumulators, peak lists (in
order) and rz records.  Full-size workloads are compared in full where the
oracle finishes in seconds, else on sampled events or sampled candidates.
"""
import math

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


def run_gpu(H, spec, batch, tuning=None, rz=None, peak_capacity=None, rz_capacity=None):
    import torch
    ctx = H.HoughContext(spec, max_events=max(batch.n_events, 1), max_hits=max(batch.n_hits, 1))
    if tuning:
        ctx.set_tuning(**tuning)
    hits = H.DeviceHits.from_batch(batch)
    acc = ctx.vote(hits)
    pk, poff = ctx.peaks(acc, batch.n_events, capacity=peak_capacity)
    out = dict(ctx=ctx, hits=hits, acc=acc, pk=pk, poff=poff)
    want_rz = bool(spec["n_z0"]) if rz is None else rz
    if want_rz:
        r, roff = ctx.rz_refine(hits, pk, poff, capacity=rz_capacity)
        out.update(rz=r, roff=roff)
    torch.cuda.synchronize()
    return out


def check_event(H, tab, res, batch, e, rz=False):
    ev = batch.event(e)
    A, opk, _ = oracle.run_event(tab, ev.layer, ev.phi, ev.z, with_rz=False)
    acc = H.acc_numpy(res["acc"][e:e + 1])[0]
    np.testing.assert_array_equal(acc, A, err_msg=f"accumulator of event {e}")
    gpk = H.peaks_numpy(res["pk"], res["poff"], e)
    np.testing.assert_array_equal(gpk, opk.astype(H.PEAK_DTYPE), err_msg=f"peaks of event {e}")
    if rz:
        orz = oracle.rz(tab, ev.layer, ev.phi, ev.z, opk)
        grz = H.rz_numpy(res["rz"], res["roff"], e)
        np.testing.assert_array_equal(grz, orz.astype(H.RZ_DTYPE), err_msg=f"rz of event {e}")
    return A, opk


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def test_c1_full(H):
    name = "c1_single_100trk"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    res = run_gpu(H, spec, batch)
    check_event(H, oracle.Tables(spec), res, batch, 0)


def test_c2_full_vote_peaks_and_sampled_rz(H):
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    res = run_gpu(H, spec, batch)
    tab = oracle.Tables(spec)
    _, opk = check_event(H, tab, res, batch, 0)
    grz = H.rz_numpy(res["rz"], res["roff"], 0)
    assert len(grz) == len(opk)
    idx = np.arange(0, len(opk), 53)
    orz = oracle.rz(tab, batch.layer, batch.phi, batch.z, opk[idx])
    assert np.array_equal(grz["peak"][idx], idx)
    for f in ("cot_bin", "z0_bin", "count", "n_members"):
        np.testing.assert_array_equal(grz[f][idx], orz[f], err_msg=f)


def test_c3_full(H):
    name = "c3_pileup_displaced_3d"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    res = run_gpu(H, spec, batch)
    check_event(H, oracle.Tables(spec), res, batch, 0)


def test_c4_full_batch_sampled_events_and_batch_equals_single(H):
    name = "c4_batch_4096"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    assert batch.n_events == 4096
    res = run_gpu(H, spec, batch)
    tab = oracle.Tables(spec)
    sizes = np.diff(batch.offsets.astype(np.int64))
    sample = sorted(set([int(np.argmax(sizes)), int(np.argmin(sizes)), 0, 4095] +
                        list(np.random.default_rng(1).choice(4096, 12, replace=False))))
    for e in sample:
        check_event(H, tab, res, batch, e)
    # the same events launched alone give the same accumulators and peaks
    for e in sample[:4]:
        single = run_gpu(H, spec, batch.event(e))
        np.testing.assert_array_equal(H.acc_numpy(single["acc"])[0], H.acc_numpy(res["acc"][e:e + 1])[0])
        np.testing.assert_array_equal(H.peaks_numpy(single["pk"], single["poff"]),
                                      H.peaks_numpy(res["pk"], res["poff"], e))
    # every event's peak count matches its offsets; total is consistent
    off = H.offsets_numpy(res["poff"])
    assert off[0] == 0 and np.all(np.diff(off.astype(np.int64)) >= 0)


def test_c5_sampled_events_with_candidate_cap(H):
    name = "c5_serving"
    spec = synth.grid_spec(name)
    batch = synth.gen_batch(name, 6)
    res = run_gpu(H, spec, batch)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        ev = batch.event(e)
        A, opk, orz = oracle.run_event(tab, ev.layer, ev.phi, ev.z)
        np.testing.assert_array_equal(H.acc_numpy(res["acc"][e:e + 1])[0], A)
        np.testing.assert_array_equal(H.peaks_numpy(res["pk"], res["poff"], e), opk.astype(H.PEAK_DTYPE))
        grz = H.rz_numpy(res["rz"], res["roff"], e)
        assert len(grz) == min(len(opk), spec["rz_max_candidates"])
        np.testing.assert_array_equal(grz, orz.astype(H.RZ_DTYPE))


# --------------------------------------------------------------------------
# edge cases, ragged and degenerate inputs, knobs
# --------------------------------------------------------------------------

def small_spec(**kw):
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    spec.update(n_qpt=64, n_phi=128)
    spec.update(kw)
    return spec


def ragged_batch():
    evs = []
    for e, n in enumerate([0, 1, 3000, 0, 57, 12000, 2]):
        rng = np.random.default_rng(100 + e)
        layer = rng.integers(0, 10, n).astype(np.uint8)
        layer[::97] = 12                      # out-of-range layers are ignored
        evs.append((layer, rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                    rng.integers(-1_200_000, 1_200_000, n).astype(np.int32)))
    return synth.concat_events(evs)


@pytest.mark.parametrize("tuning", [None, dict(vote_rows=1), dict(vote_rows=4, vote_threads=64),
                                    dict(vote_algo=1), dict(vote_algo=1, vote_rows=4, vote_threads=64),
                                    dict(vote_algo=3, vote_rows=64, vote_threads=1024), dict(vote_algo=3),
                                    dict(vote_algo=4, vote_rows=64), dict(vote_algo=4, vote_rows=1, vote_threads=64),
                                    dict(vote_algo=2), dict(peak_rows=1), dict(peak_rows=7),
                                    dict(rz_slow_path=1), dict(vote_threads=1024, vote_wgs_per_cu=1)])
def test_ragged_batch_with_empty_events(H, tuning):
    spec = small_spec()
    batch = ragged_batch()
    res = run_gpu(H, spec, batch, tuning=tuning)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e, rz=True)


@pytest.mark.parametrize("kw", [dict(n_phi=2, n_qpt=3), dict(n_phi=4, n_qpt=1),
                                dict(n_phi=4096, n_qpt=8), dict(threshold=0, n_phi=8, n_qpt=4),
                                dict(threshold=11)])
def test_degenerate_grids(H, kw):
    spec = small_spec(**kw)
    batch = synth.concat_events([tuple(a[:500] for a in (b.layer, b.phi, b.z))
                                 for b in [synth.gen_config("c1_single_100trk")]])
    res = run_gpu(H, spec, batch)
    check_event(H, oracle.Tables(spec), res, batch, 0, rz=True)


def gap_layout_batch(n_phi):
    """Events whose layers stress the gap form of the vote: every hit of a
    layer in one azimuth bucket (one gap of almost a full turn), repeated
    hits, hits on bucket edges and at 0 and 2^32 - 1, exactly n_phi/2 and
    n_phi/2 + 1 hits in a layer (the sparse/dense switch), all gaps exactly
    one bin wide (full rows) and all gaps one unit wider than a bin."""
    W = 1 << (32 - int(math.log2(n_phi)))
    rng = np.random.default_rng(11)
    evs = []

    def add(parts):
        layer = np.concatenate([np.full(len(p), l, np.uint8) for l, p in parts])
        phi = np.concatenate([np.asarray(p, np.uint64) % (1 << 32) for _, p in parts]).astype(np.uint32)
        evs.append((layer, phi, np.zeros(len(phi), np.int32)))

    add([(2, [5 * W + 3] * (n_phi // 2) + [6 * W - 1] * 20 + [0, (1 << 32) - 1, W, W - 1])])
    add([(0, [k * W for k in range(n_phi) if not (n_phi // 8 <= k < n_phi // 4)] +
          [k * W + W // 2 for k in range(n_phi)])])
    add([(1, rng.integers(0, 1 << 32, n_phi // 2)), (3, rng.integers(0, 1 << 32, n_phi // 2 + 1)),
         (9, [12345])])
    add([(4, [k * W for k in range(n_phi)]), (5, [k * (W + 1) for k in range(n_phi - 1)]),
         (6, [k * W + W - 1 for k in range(n_phi)] * 2)])
    add([(l, rng.integers(0, 1 << 32, 3 * n_phi)) for l in range(10)])
    add([(l, rng.integers(0, 1 << 32, n_phi // 2)) for l in range(10)])
    return synth.concat_events(evs)


@pytest.mark.parametrize("kw", [dict(n_phi=64, n_qpt=16), dict(n_phi=1024, n_qpt=8), dict(n_phi=512, n_qpt=200),
                                dict(n_phi=64, n_qpt=8, n_d0=8, d0_lo_mm=-120.0, d0_hi_mm=120.0, n_z0=0)])
def test_vote_forms_on_layer_layouts(H, kw):
    spec = small_spec(**kw)
    batch = gap_layout_batch(spec["n_phi"])
    tab = oracle.Tables(spec)
    res = run_gpu(H, spec, batch, rz=False)
    per_hit = H.acc_numpy(run_gpu(H, spec, batch, tuning=dict(vote_algo=1), rz=False)["acc"])
    gaps = H.acc_numpy(run_gpu(H, spec, batch, tuning=dict(vote_algo=3), rz=False)["acc"])
    direct = H.acc_numpy(run_gpu(H, spec, batch, tuning=dict(vote_algo=4), rz=False)["acc"])
    np.testing.assert_array_equal(H.acc_numpy(res["acc"]), per_hit)
    np.testing.assert_array_equal(gaps, per_hit)
    np.testing.assert_array_equal(direct, per_hit)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e)


RANK_SPECS = [dict(n_phi=256, n_qpt=16), dict(n_phi=512, n_qpt=300), dict(n_phi=1024, n_qpt=129),
              dict(n_phi=256, n_qpt=64, n_d0=8, d0_lo_mm=-120.0, d0_hi_mm=120.0, n_z0=0)]


@pytest.mark.parametrize("kw", RANK_SPECS)
@pytest.mark.parametrize("items", [0, 1, 2])
def test_rank_vote_form(H, kw, items):
    """The rank form of the vote (four cells per operation in tile rank
    space), with whole events per workgroup (bounds in LDS) and one tile per
    workgroup (bounds table), on ragged events, the adversarial layer
    layouts and a displaced grid with unreachable rows."""
    spec = small_spec(**kw)
    tab = oracle.Tables(spec)
    for batch in (ragged_batch(), gap_layout_batch(spec["n_phi"])):
        res = run_gpu(H, spec, batch, tuning=dict(vote_algo=5, vote_items=items), rz=False)
        for e in range(batch.n_events):
            check_event(H, tab, res, batch, e)


PEAK_SPECS = [dict(n_phi=256, n_qpt=16), dict(n_phi=512, n_qpt=300), dict(n_phi=1024, n_qpt=129),
              dict(n_phi=256, n_qpt=1), dict(n_phi=512, n_qpt=2, threshold=0),
              dict(n_phi=256, n_qpt=70, threshold=0), dict(n_phi=512, n_qpt=33, threshold=11),
              dict(n_phi=1024, n_qpt=5, threshold=17),
              dict(n_phi=256, n_qpt=40, n_d0=5, d0_lo_mm=-120.0, d0_hi_mm=120.0),
              dict(n_phi=512, n_qpt=33, n_d0=3, d0_lo_mm=-60.0, d0_hi_mm=60.0, threshold=0),
              dict(n_phi=1024, n_qpt=17, n_d0=2, d0_lo_mm=-30.0, d0_hi_mm=30.0)]


@pytest.mark.parametrize("kw", PEAK_SPECS)
@pytest.mark.parametrize("tuning", [dict(peak_algo=1), dict(peak_algo=2), dict(peak_algo=2, peak_rows=1),
                                    dict(peak_algo=2, peak_rows=3), dict(peak_algo=2, peak_rows=4096)])
def test_peak_forms(H, kw, tuning):
    """The row-window peak form (a wavefront strip of rows in registers,
    neighbours across lanes by wave rotates; with a d0 axis the same rows of
    the planes on either side) and the LDS tile form against the oracle:
    one-row and two-row grids, 2, 3 and 5 d0 planes, strips of 1, 3 and all
    rows (ragged last strips), thresholds 0 (every plateau cell), 11 and 17
    (no peaks), on ragged events and the adversarial layer layouts."""
    spec = small_spec(n_z0=0, n_cot=0, **kw)
    tab = oracle.Tables(spec)
    for batch in (ragged_batch(), gap_layout_batch(spec["n_phi"])):
        res = run_gpu(H, spec, batch, tuning=tuning, rz=False)
        for e in range(batch.n_events):
            check_event(H, tab, res, batch, e)


@pytest.mark.parametrize("peak_algo", [1, 2])
def test_peak_capacity_overflow_both_forms(H, peak_algo):
    """A peak list shorter than the peaks: the offsets still count every
    peak, and the stored prefix equals the full run's."""
    spec = small_spec(n_phi=512, n_qpt=40, n_z0=0, n_cot=0, threshold=0)
    batch = ragged_batch()
    t = dict(peak_algo=peak_algo, peak_rows=7)
    full = run_gpu(H, spec, batch, tuning=t, rz=False)
    total = int(H.offsets_numpy(full["poff"])[-1])
    cap = total // 3 + 5
    res = run_gpu(H, spec, batch, tuning=t, rz=False, peak_capacity=cap)
    np.testing.assert_array_equal(H.offsets_numpy(res["poff"]), H.offsets_numpy(full["poff"]))
    np.testing.assert_array_equal(H.peaks_numpy(res["pk"], res["poff"])[:cap],
                                  H.peaks_numpy(full["pk"], full["poff"])[:cap])


def test_unaligned_accumulator_peaks_take_the_tile_form(H):
    """An accumulator 4- but not 8-byte aligned: the row-window form needs
    aligned rows, so the peak search takes the LDS tile form; results equal
    the oracle's."""
    import torch
    spec = small_spec(n_phi=256, n_qpt=24, n_z0=0, n_cot=0)
    batch = ragged_batch()
    ctx = H.HoughContext(spec, max_events=batch.n_events, max_hits=batch.n_hits)
    hits = H.DeviceHits.from_batch(batch)
    base = ctx.new_acc(batch.n_events + 1).view(-1)
    acc = base[2:2 + batch.n_events * ctx.cells].view(batch.n_events, -1)
    assert acc.data_ptr() % 8
    ctx.vote(hits, acc)
    pk, poff = ctx.peaks(acc, batch.n_events)
    torch.cuda.synchronize()
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        ev = batch.event(e)
        _, opk, _ = oracle.run_event(tab, ev.layer, ev.phi, ev.z, with_rz=False)
        np.testing.assert_array_equal(H.peaks_numpy(pk, poff, e), opk.astype(H.PEAK_DTYPE), err_msg=f"event {e}")


@pytest.mark.parametrize("tuning,n_phi,sizes", [
    (dict(vote_algo=4), 64, [40000, 0, 33333, 25000]),
    (dict(vote_algo=5, vote_items=2), 256, [120000, 0, 90000, 60000]),
])
def test_bucket_bounds_split_over_parts_of_dense_events(H, tuning, n_phi, sizes):
    """Few dense events (at least 16 hits per (layer, bucket) entry on
    average): the bucket bounds are found by several workgroups per event and
    merged with global atomic min/max; accumulators and peaks equal the
    oracle's."""
    spec = small_spec(n_phi=n_phi, n_qpt=24, n_z0=0, n_cot=0)
    assert sum(sizes) // len(sizes) >= 16 * spec["n_layers"] * n_phi
    evs = []
    for e, n in enumerate(sizes):
        rng = np.random.default_rng(900 + e)
        evs.append((rng.integers(0, 10, n).astype(np.uint8),
                    rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                    np.zeros(n, np.int32)))
    batch = synth.concat_events(evs)
    res = run_gpu(H, spec, batch, tuning=tuning, rz=False)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e)


def test_unaligned_hit_arrays_and_accumulator(H):
    """Hit arrays that start one element past an aligned address and an
    accumulator that is 4- but not 8-byte aligned take the scalar load paths
    and the fallback vote form; results are unchanged."""
    import torch
    spec = small_spec(n_phi=256, n_qpt=16)
    batch = ragged_batch()
    ctx = H.HoughContext(spec, max_events=batch.n_events, max_hits=batch.n_hits)
    n = batch.n_hits
    lay = torch.zeros(n + 1, dtype=torch.uint8, device="cuda")[1:]
    lay.copy_(torch.from_numpy(batch.layer.astype(np.uint8)))
    phi = torch.zeros(n + 1, dtype=torch.int32, device="cuda")[1:]
    phi.copy_(torch.from_numpy(batch.phi.astype(np.uint32).view(np.int32)))
    hits = H.DeviceHits(lay, phi, None, batch.offsets)
    assert hits.layer.data_ptr() % 4 and hits.phi.data_ptr() % 16
    base = ctx.new_acc(batch.n_events + 1).view(-1)
    acc = base[2:2 + batch.n_events * ctx.cells].view(batch.n_events, -1)
    assert acc.data_ptr() % 16
    ctx.vote(hits, acc)
    torch.cuda.synchronize()
    tab = oracle.Tables(spec)
    got = H.acc_numpy(acc)
    for e in range(batch.n_events):
        ev = batch.event(e)
        A = oracle.vote_mask(tab, ev.layer, ev.phi)
        np.testing.assert_array_equal(got[e].reshape(A.shape), A, err_msg=f"event {e}")


def test_displaced_small_grid_unreachable_rows(H):
    spec = synth.grid_spec("c3_pileup_displaced_3d")
    spec.update(n_qpt=32, n_phi=64, n_d0=16, d0_lo_mm=-120.0, d0_hi_mm=120.0)
    batch = ragged_batch()
    res = run_gpu(H, spec, batch, rz=False)
    tab = oracle.Tables(spec)
    assert not tab.V.all()
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e)


def test_peak_and_rz_capacity_overflow(H):
    spec = small_spec()
    batch = ragged_batch()
    full = run_gpu(H, spec, batch)
    total = int(H.offsets_numpy(full["poff"])[-1])
    cap = total // 3
    res = run_gpu(H, spec, batch, peak_capacity=cap, rz_capacity=cap // 2)
    np.testing.assert_array_equal(H.offsets_numpy(res["poff"]), H.offsets_numpy(full["poff"]))
    np.testing.assert_array_equal(H.peaks_numpy(res["pk"], res["poff"])[:cap],
                                  H.peaks_numpy(full["pk"], full["poff"])[:cap])
    # rz sees only the stored peaks; the first cap // 2 records are still exact
    roff = H.offsets_numpy(res["roff"])
    assert roff[-1] == cap
    tab = oracle.Tables(spec)
    gall = H.rz_numpy(res["rz"], res["roff"])
    assert len(gall) == cap // 2
    # event ordering: compare the records of the events fully inside cap // 2
    seen = 0
    for e in range(batch.n_events):
        a, b = int(roff[e]), int(roff[e + 1])
        if b > cap // 2:
            break
        ev = batch.event(e)
        _, opk, orz = oracle.run_event(tab, ev.layer, ev.phi, ev.z)
        np.testing.assert_array_equal(gall[a:b], orz[:b - a].astype(H.RZ_DTYPE))
        seen += 1
    assert seen >= 1


@pytest.mark.parametrize("tuning,kw", [
    (dict(rz_counter_bits=4), {}),
    (dict(rz_counter_bits=4, rz_waves_per_cu=16), dict(n_phi=4, n_qpt=8, n_cot=70)),  # > 192 members: slow path
    (dict(rz_counter_bits=8), {}),
    (dict(rz_counter_bits=16), {}),
    # up to about 3000 members per cell: within the 8-bit form's 4096-member
    # list (counts past 255 are caught as overflows and redone exactly)
    (dict(rz_counter_bits=8), dict(n_phi=4, n_qpt=8, n_cot=70)),
    # up to about 6000 members per cell: past every member list, so the exact
    # path with the members in LDS
    (dict(rz_counter_bits=16), dict(n_phi=2, n_qpt=4, n_cot=9)),
    # shorter member lists than the cells need: the exact path for many
    # candidates
    (dict(rz_counter_bits=8, rz_member_cap=256), dict(n_phi=16, n_qpt=8, n_cot=40)),
    (None, dict(z0_lo_um=-2147483000, z0_hi_um=2147483000, n_z0=64)),  # general kernel
    (None, dict(cot_lo=1.2, cot_hi=-1.2)),          # Z decreasing in the cot bin
    (None, dict(n_cot=100)),                        # a last pass of 36 cot bins
])
def test_rz_kernel_variants(H, tuning, kw):
    spec = small_spec(**kw)
    batch = ragged_batch()
    res = run_gpu(H, spec, batch, tuning=tuning)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e, rz=True)


def test_rz_marked_records_past_the_list_are_found_by_the_scan(H):
    """More candidates left to the exact path than the list of them holds
    (a 4-entry list): the exact-path kernel scans every record instead, and
    the records equal the oracle's and the list path's."""
    spec = small_spec(n_phi=16, n_qpt=8, n_cot=40)
    batch = ragged_batch()
    base = dict(rz_counter_bits=8, rz_member_cap=256)
    res_list = run_gpu(H, spec, batch, tuning=base)
    res_scan = run_gpu(H, spec, batch, tuning=dict(base, rz_redo_list=4))
    tab = oracle.Tables(spec)
    marked = 0
    for e in range(batch.n_events):
        check_event(H, tab, res_scan, batch, e, rz=True)
        a = H.rz_numpy(res_list["rz"], res_list["roff"], e)
        b = H.rz_numpy(res_scan["rz"], res_scan["roff"], e)
        assert np.array_equal(a, b)
        marked += int((b["n_members"] > 256).sum())
    assert marked > 4


def test_rz_exact_path_past_the_lds_member_list(H):
    """A cell with more members than the exact path's LDS list (8192): the
    global-histogram path, against the oracle."""
    spec = small_spec(n_phi=2, n_qpt=4, n_cot=7, n_z0=32)
    rng = np.random.default_rng(77)
    n = 20000
    batch = synth.concat_events([(rng.integers(0, 10, n).astype(np.uint8),
                                  rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                                  rng.integers(-1_200_000, 1_200_000, n).astype(np.int32))])
    res = run_gpu(H, spec, batch, tuning=dict(rz_counter_bits=16))
    tab = oracle.Tables(spec)
    check_event(H, tab, res, batch, 0, rz=True)
    assert H.rz_numpy(res["rz"], res["roff"], 0)["n_members"].max() > 8192


@pytest.mark.parametrize("bits,copies", [(4, 3), (8, 3), (16, 3), (8, 26)])
def test_rz_counter_overflow_goes_to_exact_path(H, bits, copies):
    # identical bin-centre tracks put 10 members per copy into one (cot, z0)
    # bin of their cell: 3 copies pass a 4-bit counter, 26 copies an 8-bit
    # one, which must detect it and take the exact path; wider counters
    # hold the count directly
    spec = small_spec()
    K, N = spec["n_qpt"], spec["n_phi"]
    kap = spec["qpt_lo"] + (np.arange(K) + 0.5) * (spec["qpt_hi"] - spec["qpt_lo"]) / K
    layer, phi, z = synth.track_hits(kap[20], (77 + 0.5) / N * 2 * math.pi,
        cot=-1.2 + 160.5 * 2.4 / 256, z0=-200.0 + 140.5 * 400.0 / 256)
    rng = np.random.default_rng(9)
    nl, nphi, nz = (rng.integers(0, 10, 400).astype(np.uint8),
                    rng.integers(0, 1 << 32, 400, dtype=np.uint64).astype(np.uint32),
                    rng.integers(-1_200_000, 1_200_000, 400).astype(np.int32))
    batch = synth.concat_events([(np.concatenate([layer] * copies + [nl]),
                                  np.concatenate([phi] * copies + [nphi]),
                                  np.concatenate([z] * copies + [nz]))])
    res = run_gpu(H, spec, batch, tuning=dict(rz_counter_bits=bits))
    tab = oracle.Tables(spec)
    check_event(H, tab, res, batch, 0, rz=True)
    grz = H.rz_numpy(res["rz"], res["roff"], 0)
    assert grz["count"].max() >= 10 * copies


@pytest.mark.parametrize("tuning", [None, dict(vote_algo=4), dict(vote_algo=5, vote_items=2)])
def test_many_small_events_take_the_per_event_kernels(H, tuning):
    """A batch of more than two events per compute unit: the layer sort,
    the bucket bounds (direct form and the rank form's tile mode) and the
    candidate selection run one workgroup per event (smaller batches split
    each event over several workgroups); every event equals the oracle, rz
    records with a candidate cap included."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    spec = small_spec(n_qpt=16, n_phi=256, rz_max_candidates=3)
    evs = []
    for e in range(2 * n_cu + 7):
        rng = np.random.default_rng(5000 + e)
        n = int(rng.integers(0, 60))
        evs.append((rng.integers(0, 10, n).astype(np.uint8),
                    rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                    rng.integers(-1_200_000, 1_200_000, n).astype(np.int32)))
    batch = synth.concat_events(evs)
    res = run_gpu(H, spec, batch, tuning=tuning)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e, rz=True)


def test_rz_offsets_of_a_batch_past_the_one_workgroup_scan(H):
    """More events (8,300) than the fused one-workgroup candidate-offset
    kernel takes: the count, scan and counter-reset launches; every event's
    rz records equal the oracle's."""
    spec = small_spec(n_qpt=4, n_phi=8, n_cot=16, n_z0=16, rz_max_candidates=2)
    evs = []
    rng = np.random.default_rng(31)
    for e in range(8300):
        n = int(rng.integers(0, 4))
        evs.append((rng.integers(0, 10, n).astype(np.uint8),
                    rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                    rng.integers(-1_200_000, 1_200_000, n).astype(np.int32)))
    batch = synth.concat_events(evs)
    res = run_gpu(H, spec, batch)
    tab = oracle.Tables(spec)
    roff = H.offsets_numpy(res["roff"]).astype(np.int64)
    want = [0]
    for e in range(batch.n_events):
        ev = batch.event(e)
        _, opk, orz = oracle.run_event(tab, ev.layer, ev.phi, ev.z)
        want.append(want[-1] + len(orz))
        if e % 97 == 0:
            np.testing.assert_array_equal(H.rz_numpy(res["rz"], res["roff"], e), orz.astype(H.RZ_DTYPE),
                                          err_msg=f"rz of event {e}")
    np.testing.assert_array_equal(roff, np.array(want, np.int64))


def test_rz_candidate_cap_selection(H):
    spec = small_spec(rz_max_candidates=37)
    batch = ragged_batch()
    res = run_gpu(H, spec, batch)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e, rz=True)


def test_bin_centre_tracks_full_layer_peaks(H):
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    K, N = spec["n_qpt"], spec["n_phi"]
    kap = spec["qpt_lo"] + (np.arange(K) + 0.5) * (spec["qpt_hi"] - spec["qpt_lo"]) / K
    cot = spec["cot_lo"] + (np.arange(256) + 0.5) * (spec["cot_hi"] - spec["cot_lo"]) / 256
    cells = [(3, 1000, 17, 40), (700, 5, 200, 128), (1023, 511, 255, 0)]
    evs = []
    for k, p, j, b in cells:
        z0 = (-200000 + (b + 0.5) * 400000 / 256) / 1000.0
        evs.append(synth.track_hits(kap[k], (p + 0.5) / N * 2 * math.pi, cot=cot[j], z0=z0))
    batch = synth.concat_events(evs)
    res = run_gpu(H, spec, batch)
    for e, (k, p, j, b) in enumerate(cells):
        acc = H.acc_numpy(res["acc"][e:e + 1])[0]
        assert acc[0, k, p] == 0x3FF
        gpk = H.peaks_numpy(res["pk"], res["poff"], e)
        i = int(np.nonzero(gpk["cell"] == k * N + p)[0][0])
        grz = H.rz_numpy(res["rz"], res["roff"], e)
        rec = grz[grz["peak"] == i][0]
        assert (rec["cot_bin"], rec["z0_bin"], rec["count"], rec["n_members"]) == (j, b, 10, 10)


def test_hit_permutation_and_repeat_determinism(H):
    spec = small_spec()
    batch = ragged_batch()
    a = run_gpu(H, spec, batch)
    b = run_gpu(H, spec, batch)
    perm_evs = []
    for e in range(batch.n_events):
        ev = batch.event(e)
        p = np.random.default_rng(e).permutation(ev.n_hits)
        perm_evs.append((ev.layer[p], ev.phi[p], ev.z[p]))
    c = run_gpu(H, spec, synth.concat_events(perm_evs))
    for x in (b, c):
        np.testing.assert_array_equal(H.acc_numpy(a["acc"]), H.acc_numpy(x["acc"]))
        np.testing.assert_array_equal(H.peaks_numpy(a["pk"], a["poff"]), H.peaks_numpy(x["pk"], x["poff"]))
        np.testing.assert_array_equal(H.rz_numpy(a["rz"], a["roff"]), H.rz_numpy(x["rz"], x["roff"]))


def test_graph_replays_match_oracle_and_eager(H):
    import torch
    spec = small_spec(rz_max_candidates=50)
    batch = ragged_batch()
    eager = run_gpu(H, spec, batch)
    tab = oracle.Tables(spec)
    want = [oracle.run_event(tab, *(lambda ev: (ev.layer, ev.phi, ev.z))(batch.event(e)))
            for e in range(batch.n_events)]
    ctx = H.HoughContext(spec, max_events=batch.n_events, max_hits=batch.n_hits)
    hits = H.DeviceHits.from_batch(batch)
    acc = ctx.new_acc(batch.n_events)
    cap = batch.n_events * ctx.cells
    pk, poff = ctx.new_peaks(cap), ctx.new_offsets(batch.n_events)
    rz, roff = ctx.new_rz(cap), ctx.new_offsets(batch.n_events)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = ctx.graph_capture(hits, acc, pk, cap, poff, rz, cap, roff, stream=stream)
    for rep in range(3):
        acc.fill_(-1)
        pk.fill_(-1)
        rz.fill_(-1)
        torch.cuda.synchronize()
        g.launch(stream)
        stream.synchronize()
        np.testing.assert_array_equal(H.acc_numpy(acc), H.acc_numpy(eager["acc"]), err_msg=f"replay {rep}")
        np.testing.assert_array_equal(H.peaks_numpy(pk, poff), H.peaks_numpy(eager["pk"], eager["poff"]))
        np.testing.assert_array_equal(H.rz_numpy(rz, roff), H.rz_numpy(eager["rz"], eager["roff"]))
        for e, (A, opk, orz) in enumerate(want):
            np.testing.assert_array_equal(H.acc_numpy(acc[e:e + 1])[0], A, err_msg=f"replay {rep}, event {e}")
            np.testing.assert_array_equal(H.peaks_numpy(pk, poff, e), opk.astype(H.PEAK_DTYPE))
            np.testing.assert_array_equal(H.rz_numpy(rz, roff, e), orz.astype(H.RZ_DTYPE))
        # eager work on the same context between replays
        run_gpu(H, spec, batch)
    g.close()


def test_limits_and_bad_arguments_raise(H):
    spec = small_spec()
    batch = ragged_batch()
    ctx = H.HoughContext(spec, max_events=2, max_hits=100)
    hits = H.DeviceHits.from_batch(batch)
    with pytest.raises(H.HoughError):
        ctx.vote(hits)
    with pytest.raises(H.HoughError):
        ctx.set_tuning(vote_rows=3)
    with pytest.raises(H.HoughError):
        ctx.set_tuning(vote_algo=5)
    with pytest.raises(H.HoughError):
        H.HoughContext(dict(spec, n_phi=48))


@pytest.mark.parametrize("name", list(synth.CONFIGS))
def test_device_tables_match_oracle(H, name):
    """The tables a context uploaded, read back from the device, equal the
    oracle's independently built ones; the rz kernel's (Z + z0_lo) copy
    equals Z + z0_lo."""
    spec = synth.grid_spec(name)
    ctx = H.HoughContext(spec, max_events=1, max_hits=16)
    tab = oracle.Tables(spec)
    if spec["n_z0"]:
        O, V, Z, Zl = ctx.get_tables(zl=True)
        np.testing.assert_array_equal(Zl.astype(np.int64), tab.Z.astype(np.int64) + spec["z0_lo_um"])
    else:
        O, V, Z = ctx.get_tables()
        with pytest.raises(H.HoughError):
            ctx.get_tables(zl=True)
    np.testing.assert_array_equal(O, tab.O)
    np.testing.assert_array_equal(V, tab.V)
    np.testing.assert_array_equal(Z, tab.Z)


def test_cluster_fit_without_bucket_index_is_refused(H):
    """A context made without an rz grid and without max_peaks keeps no
    (layer, azimuth bucket) index: the fit refuses before launching."""
    spec = synth.grid_spec("c1_single_100trk")
    batch = synth.gen_config("c1_single_100trk")
    ctx = H.HoughContext(spec, max_events=1, max_hits=batch.n_hits)
    hits = H.DeviceHits.from_batch(batch)
    pk, poff = ctx.new_peaks(16), ctx.new_offsets(1)
    cl, coff = ctx.new_clusters(16), ctx.new_offsets(1)
    with pytest.raises(H.HoughError, match="invalid argument"):
        ctx.cluster_fit(hits, pk, poff, cl, coff, peak_capacity=16, capacity=16)


@pytest.mark.parametrize("n_layers", [7, 13, 16])
@pytest.mark.parametrize("tuning", [None, dict(vote_algo=5, vote_items=1), dict(vote_algo=5, vote_items=2),
                                    dict(vote_algo=4), dict(peak_algo=1), dict(rz_counter_bits=8)])
def test_other_layer_counts(H, n_layers, tuning):
    """Detectors of 7, 13 and 16 layers (the kernels' general layer-count
    instances; every other test uses ten): accumulators, peaks and rz
    records of ragged events against the oracle, under the vote forms (rank
    form with whole events and with single tiles, direct form), both peak
    forms and 8-bit rz counters."""
    radii = [40.0 + (800.0 - 40.0) * i / (n_layers - 1) for i in range(n_layers)]
    spec = small_spec(n_layers=n_layers, layer_r_mm=radii, threshold=min(8, n_layers - 2), n_phi=256)
    evs = []
    for e, n in enumerate([0, 5, 300, 1200, 4000, 1]):
        rng = np.random.default_rng(700 + e)
        layer = rng.integers(0, n_layers, n).astype(np.uint8)
        layer[::53] = n_layers + 2                   # out-of-range layers are ignored
        evs.append((layer, rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32),
                    rng.integers(-1_200_000, 1_200_000, n).astype(np.int32)))
    batch = synth.concat_events(evs)
    res = run_gpu(H, spec, batch, tuning=tuning)
    tab = oracle.Tables(spec)
    for e in range(batch.n_events):
        check_event(H, tab, res, batch, e, rz=True)
