"""Plateau clusters (candidate confirmation) on the GPU against the CPU
oracle, bit for bit: per-peak cluster indices, cluster records and event
offsets.  Peak lists come from the GPU path on the workloads (checked equal
to the oracle's first) or are built directly: random peak images with phi0
wrap, two phi0 bins, a d0 axis, one grid-filling component; truncated peak
lists and cluster-capacity overflow; repeat determinism."""
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


FIELDS = ("first", "popcount", "mask_or", "n_peaks", "sum_dk", "sum_dp", "sum_dd")


def expected(tab, pk, off, peak_cap):
    """Oracle labels, records and cluster offsets of the stored peaks."""
    labels, recs, coff = [], [], [0]
    for e in range(len(off) - 1):
        lo, hi = min(int(off[e]), peak_cap), min(int(off[e + 1]), peak_cap)
        lab, cl = oracle.clusters(tab, pk[lo:hi])
        labels.append(lab)
        recs.append(cl)
        coff.append(coff[-1] + len(cl))
    return np.concatenate(labels), np.concatenate(recs), np.array(coff, np.uint64)


def compare(H, got, want, peak_off, peak_cap, cl_cap, what=""):
    labels, cl, coff = got
    wl, wc, wo = want
    np.testing.assert_array_equal(H.offsets_numpy(coff), wo, err_msg=f"cluster offsets {what}")
    np.testing.assert_array_equal(H.labels_numpy(labels, peak_off, peak_cap), wl, err_msg=f"labels {what}")
    gc = cl[:min(len(wc), cl_cap)].cpu().numpy().view(H.CLUSTER_DTYPE).reshape(-1)
    for f in FIELDS:
        np.testing.assert_array_equal(gc[f], wc[f][:cl_cap], err_msg=f"{f} {what}")


def run_workload(H, name, batch, events=None):
    import torch
    spec = synth.grid_spec(name)
    tab = oracle.Tables(spec)
    E = batch.n_events
    cap = E * tab.cells
    ctx = H.HoughContext(spec, max_events=E, max_hits=max(batch.n_hits, 1), max_peaks=cap)
    hits = H.DeviceHits.from_batch(batch)
    acc = ctx.vote(hits)
    pk, poff = ctx.peaks(acc, E, capacity=cap)
    labels, cl, coff = ctx.peak_clusters(pk, poff, E, capacity=min(cap, 1 << 26))
    torch.cuda.synchronize()
    off = H.offsets_numpy(poff)
    gco = H.offsets_numpy(coff)
    for e in (range(E) if events is None else events):
        ev = batch.event(e)
        opk = oracle.peaks(tab, oracle.vote_mask(tab, ev.layer, ev.phi))
        np.testing.assert_array_equal(H.peaks_numpy(pk, poff, e), opk.astype(H.PEAK_DTYPE),
                                      err_msg=f"peaks of event {e}")
        wl, wc = oracle.clusters(tab, opk)
        np.testing.assert_array_equal(H.labels_numpy(labels, poff, event=e), wl, err_msg=f"labels of event {e}")
        assert int(gco[e + 1] - gco[e]) == len(wc)
        gc = H.clusters_numpy(cl, coff, e)
        for f in FIELDS:
            np.testing.assert_array_equal(gc[f], wc[f], err_msg=f"{f} of event {e}")
    return ctx, off, gco


def test_c1_full(H):
    name = "c1_single_100trk"
    run_workload(H, name, synth.gen_config(name))


def test_c2_full(H):
    name = "c2_single_1ktrk_rz"
    _, off, gco = run_workload(H, name, synth.gen_config(name))
    assert 0 < gco[-1] < off[-1]            # plateaus merge


def test_c3_full_displaced_3d(H):
    name = "c3_pileup_displaced_3d"
    run_workload(H, name, synth.gen_config(name))


def test_c4_full_batch_sampled_events(H):
    name = "c4_batch_4096"
    batch = synth.gen_config(name)
    sizes = np.diff(batch.offsets.astype(np.int64))
    sample = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 0, 1, 2047, 4095})
    _, off, gco = run_workload(H, name, batch, events=sample)
    assert gco[0] == 0 and np.all(np.diff(gco.astype(np.int64)) >= 0)


# --------------------------------------------------------------------------
# peak lists built directly
# --------------------------------------------------------------------------

def upload(H, pk, off):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(pk).view(np.int32).reshape(-1, 2).copy()).cuda()
    o = torch.from_numpy(np.asarray(off, np.uint64).view(np.int64).copy()).cuda()
    return t, o


def image_peaks(rng, shape, density, all_cells=False):
    img = np.ones(shape, bool) if all_cells else rng.random(shape) < density
    cells = np.flatnonzero(img.ravel())
    pk = np.zeros(len(cells), oracle.PEAK_DTYPE)
    pk["cell"] = cells
    pc = rng.integers(1, 11, len(cells))
    pk["popcount"] = pc
    pk["mask"] = (1 << pc) - 1 << rng.integers(0, 7, len(cells))
    pk["mask"] &= 0xFFFF
    return pk


def run_lists(H, spec, events, peak_cap=None, cl_cap=None, reps=1):
    import torch
    tab = oracle.Tables(spec)
    pk = np.concatenate(events) if events else np.zeros(0, oracle.PEAK_DTYPE)
    off = np.concatenate([[0], np.cumsum([len(x) for x in events])]).astype(np.uint64)
    n = int(off[-1])
    peak_cap = n if peak_cap is None else peak_cap
    want = expected(tab, pk, off, peak_cap)
    cl_cap = len(want[1]) if cl_cap is None else cl_cap
    ctx = H.HoughContext(spec, max_events=len(events), max_hits=1, max_peaks=max(peak_cap, 1))
    tpk, toff = upload(H, pk[:peak_cap], off)
    outs = []
    for _ in range(reps):
        outs.append(ctx.peak_clusters(tpk, toff, len(events), peak_capacity=peak_cap, capacity=cl_cap))
        torch.cuda.synchronize()
    for i, got in enumerate(outs):
        compare(H, got, want, toff, peak_cap, cl_cap, what=f"rep {i}")
    return want


@pytest.mark.parametrize("n_d0,n_qpt,n_phi,density,seed", [
    (1, 40, 64, 0.3, 0), (1, 40, 64, 0.55, 1), (1, 33, 2, 0.5, 2), (4, 24, 32, 0.2, 3),
    (1, 64, 8, 0.7, 4), (3, 16, 16, 0.35, 5)])
def test_random_peak_images(H, n_d0, n_qpt, n_phi, density, seed):
    spec = synth.grid_spec("c1_single_100trk")
    spec.update(n_qpt=n_qpt, n_phi=n_phi, n_d0=n_d0, d0_lo_mm=-50.0, d0_hi_mm=50.0, threshold=1)
    rng = np.random.default_rng(seed)
    events = [image_peaks(rng, (n_d0, n_qpt, n_phi), density) for _ in range(5)]
    events.insert(2, events[0][:0])                       # an empty event
    want = run_lists(H, spec, events, reps=2)
    assert len(want[1]) > 0


def test_grid_filling_component_and_wrap_rows(H):
    # every cell a peak: one cluster per event, long union chains
    spec = synth.grid_spec("c4_batch_4096")
    rng = np.random.default_rng(7)
    full = image_peaks(rng, (1, 512, 512), 1.0, all_cells=True)
    # single-cell-wide rows touching across the phi0 wrap only
    cells = np.array([k * 512 + p for k in range(0, 512, 2) for p in (0, 511)])
    rows = np.zeros(len(cells), oracle.PEAK_DTYPE)
    rows["cell"] = np.sort(cells)
    rows["popcount"], rows["mask"] = 10, 0x3FF
    want = run_lists(H, spec, [full, rows])
    assert want[2].tolist() == [0, 1, 1 + 256]


def test_truncated_peak_list_and_cluster_overflow(H):
    spec = synth.grid_spec("c1_single_100trk")
    spec.update(n_qpt=32, n_phi=64, threshold=1)
    rng = np.random.default_rng(11)
    events = [image_peaks(rng, (1, 32, 64), 0.3) for _ in range(4)]
    n = sum(len(x) for x in events)
    # peaks past peak_cap are not seen; event 2 is cut in the middle
    cut = len(events[0]) + len(events[1]) + len(events[2]) // 2
    want = run_lists(H, spec, events, peak_cap=cut)
    assert len(want[0]) == cut < n
    # clusters past capacity are dropped, offsets keep the true counts
    total = len(expected(oracle.Tables(spec), np.concatenate(events),
                         np.concatenate([[0], np.cumsum([len(x) for x in events])]), n)[1])
    run_lists(H, spec, events, cl_cap=total // 3)
    run_lists(H, spec, events, cl_cap=0)


def test_workload_peaks_repeat_determinism(H):
    import torch
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    batch = synth.gen_config(name)
    cells = oracle.Tables(spec).cells
    ctx = H.HoughContext(spec, max_events=1, max_hits=batch.n_hits, max_peaks=cells)
    hits = H.DeviceHits.from_batch(batch)
    pk, poff = ctx.peaks(ctx.vote(hits), 1, capacity=cells)
    a = ctx.peak_clusters(pk, poff, 1)
    torch.cuda.synchronize()
    ref = [x.clone() for x in a]
    for _ in range(3):
        ctx.peak_clusters(pk, poff, 1, labels=a[0], out=a[1], offsets=a[2])
        torch.cuda.synchronize()
        n = int(H.offsets_numpy(a[2])[-1])
        assert torch.equal(a[0][:int(H.offsets_numpy(poff)[-1])], ref[0][:int(H.offsets_numpy(poff)[-1])])
        assert torch.equal(a[1][:n], ref[1][:n]) and torch.equal(a[2], ref[2])


def test_cluster_limits_and_bad_arguments(H):
    import torch
    spec = synth.grid_spec("c1_single_100trk")
    ctx = H.HoughContext(spec, max_events=2, max_hits=16, max_peaks=100)
    pk = ctx.new_peaks(200)
    off = torch.zeros(3, dtype=torch.int64, device="cuda")
    with pytest.raises(H.HoughError):
        ctx.peak_clusters(pk, off, 2, peak_capacity=101)            # beyond max_peaks
    with pytest.raises(H.HoughError):
        ctx.peak_clusters(pk, off, 3, peak_capacity=10)             # beyond max_events
    lab = ctx.new_labels(100)
    cl = ctx.new_clusters(10)
    with pytest.raises(H.HoughError):                                # clusters not 8-byte aligned
        ctx.peak_clusters(pk, off, 2, peak_capacity=10, labels=lab,
                          out=cl.view(torch.int32).reshape(-1)[1:].view(torch.int32))
    # no peaks at all: every offset 0
    labels, cl, coff = ctx.peak_clusters(pk, off, 2, peak_capacity=10)
    torch.cuda.synchronize()
    assert H.offsets_numpy(coff).tolist() == [0, 0, 0]
    with pytest.raises(H.HoughError):
        H.HoughContext(spec, max_events=1, max_hits=16, max_peaks=1 << 32)


# --------------------------------------------------------------------------
# track fit of each cluster
# --------------------------------------------------------------------------

# fp64 throughout; the device sums members in another order and uses its own
# sin/cos (within 2 ulp).  With at most a few hundred members and normal
# equations whose condition number stays below ~1e5 on these workloads, the
# differences are below 1e-10 in q/pT (1/GeV), phi0 (rad) and rms (mm); the
# bar leaves a factor 100 of margin.
FIT_TOL = 1e-8
WORST = {}


def check_fit(H, got, want, what=""):
    np.testing.assert_array_equal(got["n_hits"], want["n_hits"], err_msg=f"n_hits {what}")
    np.testing.assert_array_equal(got["status"], want["status"], err_msg=f"status {what}")
    np.testing.assert_array_equal(got["status_z"], want["status_z"], err_msg=f"status_z {what}")
    for f in ("qpt", "phi0", "qpt_c", "phi0_c", "rms_mm", "cot", "z0_mm", "rms_z_mm"):
        d = np.abs(got[f] - want[f])
        if f.startswith("phi0"):
            d = np.minimum(d, 2 * np.pi - d)            # the same angle across the wrap
        scale = np.maximum(1.0, np.abs(want[f]))
        assert np.all(d <= FIT_TOL * scale), (f, what, float(d.max()))
        WORST[f] = max(WORST.get(f, 0.0), float(d.max()) if len(d) else 0.0)


def run_fit(H, name, batch, events=None, cl_cap=None):
    import torch
    spec = synth.grid_spec(name)
    tab = oracle.Tables(spec)
    E = batch.n_events
    cap = E * tab.cells
    ctx = H.HoughContext(spec, max_events=E, max_hits=max(batch.n_hits, 1), max_peaks=cap)
    hits = H.DeviceHits.from_batch(batch)
    pk, poff = ctx.peaks(ctx.vote(hits), E, capacity=cap)
    cl_cap = min(cap, 1 << 26) if cl_cap is None else cl_cap
    labels, cl, coff = ctx.peak_clusters(pk, poff, E, capacity=cl_cap)
    fits = ctx.cluster_fit(hits, pk, poff, cl, coff, peak_capacity=cap, capacity=cl_cap)
    torch.cuda.synchronize()
    gco = H.offsets_numpy(coff)
    for e in (range(E) if events is None else events):
        ev = batch.event(e)
        opk = oracle.peaks(tab, oracle.vote_mask(tab, ev.layer, ev.phi))
        _, ocl = oracle.clusters(tab, opk)
        want = oracle.fit(tab, ev.layer, ev.phi, opk, ocl, ev.z if spec["n_z0"] else None)
        lo, hi = min(int(gco[e]), cl_cap), min(int(gco[e + 1]), cl_cap)
        got = fits[lo:hi].cpu().numpy().view(H.FIT_DTYPE).reshape(-1)
        check_fit(H, got, want[:hi - lo], what=f"event {e}")
    return fits, coff


def test_fit_c1_full(H):
    run_fit(H, "c1_single_100trk", synth.gen_config("c1_single_100trk"))


def test_fit_c2_full(H):
    name = "c2_single_1ktrk_rz"
    fits, coff = run_fit(H, name, synth.gen_config(name))
    f = H.fits_numpy(fits, coff)
    assert np.count_nonzero(f["status"]) > len(f) // 2
    assert np.count_nonzero(f["status_z"]) > len(f) // 2          # the rz grid fits the helix


def test_fit_c4_sampled_events_and_cluster_capacity(H):
    name = "c4_batch_4096"
    batch = synth.gen_batch(name, 64)
    run_fit(H, name, batch, events=[0, 1, 31, 63])
    # only the stored clusters are fitted: events past the capacity get none
    run_fit(H, name, batch, events=[0, 1], cl_cap=1000)


def test_fit_generator_tracks_recover_truth(H):
    # noiseless helices off the bin centres: the device fit lands on the
    # generator's parameters (cot 0.4, z0 12.5 mm), as the oracle's does
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    truth = [(0.3131, 1.234), (-0.8765, 4.5678), (0.0217, 0.0004), (-0.5, 2 * np.pi - 0.0007)]
    from synth.events import concat_events
    batch = concat_events([synth.track_hits(q, p, cot=0.4, z0=12.5) for q, p in truth])
    fits, coff = run_fit(H, name, batch)
    for e, (q, p) in enumerate(truth):
        f = H.fits_numpy(fits, coff, e)
        good = f[f["status"] == 1]
        assert len(good) and np.all(np.abs(good["qpt"] - q) < 2e-6)
        assert np.all(np.abs(np.angle(np.exp(1j * (good["phi0"] - p)))) < 1e-7)
        assert np.all(good["status_z"] == 1)
        assert np.all(np.abs(good["cot"] - 0.4) < 5e-6) and np.all(np.abs(good["z0_mm"] - 12.5) < 1e-3)


def test_fit_rejects_d0_grid_and_reports_worst_difference(H):
    spec = synth.grid_spec("c3_pileup_displaced_3d")
    ctx = H.HoughContext(spec, max_events=1, max_hits=16, max_peaks=16)
    hits = H.DeviceHits(np.zeros(1, np.uint8), np.zeros(1, np.uint32), None, np.array([0, 1], np.uint64))
    pk, off = ctx.new_peaks(16), ctx.new_offsets(1)
    with pytest.raises(H.HoughError):
        ctx.cluster_fit(hits, pk, off, ctx.new_clusters(4), off, peak_capacity=16, capacity=4)
    print("largest fit differences from the oracle:", WORST)
