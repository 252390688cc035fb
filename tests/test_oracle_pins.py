"""Pins of the CPU oracle against things other than itself.

Each test fixes part of the oracle against the mathematics or the paper:
continuous-angle brute force through an independent trajectory construction,
closed forms, the vote-count invariant, bin-centre tracks, missing-hit
tolerance (Section 4: the transform tolerates missing hits), exact rotation
covariance, hit-order independence, a library maximum filter, and a dense
argmax of the rz grid.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from synth.events import _helix_hits, C_LIGHT

TURN = 4294967296.0


def tiny_spec(n_qpt=16, n_phi=32, n_d0=1, d0=(0.0, 0.0), threshold=8, rz=False,
              rz_max_candidates=0, qpt=(-1.0, 1.0)):
    s = synth.grid_spec("c1_single_100trk")
    s.update(n_qpt=n_qpt, n_phi=n_phi, n_d0=n_d0, d0_lo_mm=d0[0], d0_hi_mm=d0[1],
             threshold=threshold, qpt_lo=qpt[0], qpt_hi=qpt[1],
             rz_max_candidates=rz_max_candidates)
    if rz:
        s.update(n_z0=256, z0_lo_um=-200000, z0_hi_um=200000, n_cot=256, cot_lo=-1.2, cot_hi=1.2)
    return s


def centres(lo, hi, n):
    return lo + (np.arange(n) + 0.5) * ((hi - lo) / n)


def random_hits(rng, n, n_layers=10):
    layer = rng.integers(0, n_layers, n).astype(np.uint8)
    phi = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    z = rng.integers(-1_200_000, 1_200_000, n).astype(np.int32)
    return layer, phi, z


def geometric_offsets(spec):
    """Azimuth of the crossing point of each bin-centre track with phi0 = 0,
    from the generator's chord construction (not the oracle's formula).
    Returns angles [L, D, K] in turns and a reachability mask."""
    K, D, L = spec["n_qpt"], spec["n_d0"], spec["n_layers"]
    kap = centres(spec["qpt_lo"], spec["qpt_hi"], K)
    d0s = np.zeros(1) if D == 1 else centres(spec["d0_lo_mm"], spec["d0_hi_mm"], D)
    kk, dd = np.meshgrid(kap, d0s)                        # [D, K]
    phi, _, ok = _helix_hits(kk.ravel(), np.zeros(kk.size), dd.ravel(), np.zeros(kk.size),
                             np.zeros(kk.size), spec["layer_r_mm"][:L], spec["b_tesla"])
    ang = (phi / (2 * math.pi)).T.reshape(L, D, K)
    return ang, ok.T.reshape(L, D, K)


def continuous_accumulator(spec, layer, phi):
    """Layer-mask accumulator from continuous FP64 angles; also returns how
    many votes fell within 2**-30 turns of a bin edge (ambiguous in FP)."""
    ang, ok = geometric_offsets(spec)
    D, K, N = spec["n_d0"], spec["n_qpt"], spec["n_phi"]
    A = np.zeros((D, K, N), np.uint16)
    near = 0
    for h in range(len(layer)):
        l = int(layer[h])
        t = np.mod(float(phi[h]) / TURN - ang[l], 1.0)   # [D, K] turn fraction of phi0
        x = t * N
        p = np.floor(x).astype(np.int64) % N
        frac = x - np.floor(x)
        near += int(np.sum(ok[l] & ((frac < 2.0 ** -30 * N) | (1 - frac < 2.0 ** -30 * N))))
        d_idx, k_idx = np.nonzero(ok[l])
        A[d_idx, k_idx, p[d_idx, k_idx]] |= np.uint16(1 << l)
    return A, near


# --------------------------------------------------------------------------
# P1: brute force on tiny events, continuous angles, independent geometry
# --------------------------------------------------------------------------

@pytest.mark.parametrize("case", [
    dict(n_qpt=16, n_phi=32),
    dict(n_qpt=8, n_phi=16, n_d0=4, d0=(-120.0, 120.0)),
    dict(n_qpt=32, n_phi=8),
])
def test_p1_vote_matches_continuous_geometry(case):
    spec = tiny_spec(**case)
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(11)
    layer, phi, _ = random_hits(rng, 50)
    A = oracle.vote_mask(tab, layer, phi)
    Ac, near = continuous_accumulator(spec, layer, phi)
    assert near == 0
    np.testing.assert_array_equal(A, Ac)


def test_p1_validity_matches_reachability():
    spec = tiny_spec(n_qpt=8, n_phi=16, n_d0=4, d0=(-120.0, 120.0))
    tab = oracle.Tables(spec)
    _, ok = geometric_offsets(spec)
    np.testing.assert_array_equal(tab.V.astype(bool), ok)
    # |d0| = 90 mm cannot reach the 40 and 70 mm layers; |d0| = 30 mm reaches all
    assert not tab.V[0, 0].any() and not tab.V[1, 0].any() and tab.V[2, 0].all()
    assert tab.V[:, 1].all() and tab.V[:, 2].all()


def test_offset_closed_form_special_angle():
    # choose B so that rho * r / 2 = 1/2 at r = 800 mm for the single bin
    # centre kappa = 1: the prompt offset is then -asin(1/2) = -pi/6 = -1/12 turn
    spec = tiny_spec(n_qpt=1, qpt=(0.5, 1.5))
    spec["b_tesla"] = (1.0 / 800.0) / C_LIGHT
    tab = oracle.Tables(spec)
    got = int(tab.O[9, 0, 0])
    want = (TURN - TURN / 12.0) % TURN
    assert abs(got - want) <= 2
    # a straight track (kappa -> 0) has no azimuth offset at any radius
    spec = tiny_spec(n_qpt=2, qpt=(-1e-12, 1e-12))
    tab = oracle.Tables(spec)
    o = tab.O.astype(np.int64)
    o = np.where(o >= 2 ** 31, o - 2 ** 32, o)
    assert np.abs(o).max() <= 1


def test_zshift_closed_form_straight_track():
    # kappa -> 0: arc length equals radius; cot = 1 exactly -> Z = r in micrometres
    spec = tiny_spec(n_qpt=2, qpt=(-1e-9, 1e-9), rz=True)
    spec.update(n_cot=1, cot_lo=0.5, cot_hi=1.5)
    tab = oracle.Tables(spec)
    for l, r in enumerate(spec["layer_r_mm"]):
        assert tab.Z[0, l, 0] == int(round(r * 1000))
        assert tab.Z[1, l, 0] == int(round(r * 1000))


def test_zshift_matches_generator_arc_length():
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    spec.update(n_qpt=64)
    tab = oracle.Tables(spec)
    kap = centres(-1, 1, 64)
    cotj = centres(-1.2, 1.2, 256)
    # the generator's z for a prompt track with z0 = 0 is cot * s
    for k in (0, 17, 63):
        for j in (0, 100, 255):
            _, z_mm, _ = _helix_hits([kap[k]], [0.3], [0.0], [cotj[j]], [0.0],
                                     spec["layer_r_mm"], spec["b_tesla"])
            np.testing.assert_allclose(tab.Z[k, :, j], z_mm[0] * 1000.0, atol=1.0)


# --------------------------------------------------------------------------
# P2 / P3: invariants of the counting and mask forms
# --------------------------------------------------------------------------

def test_p2_total_votes_is_hits_times_rows():
    spec = synth.grid_spec("c1_single_100trk")
    tab = oracle.Tables(spec)
    ev = synth.gen_config("c1_single_100trk")
    C = oracle.vote_count(tab, ev.layer, ev.phi)
    assert int(C.sum()) == ev.n_hits * spec["n_qpt"]
    # every row of a prompt grid receives exactly one vote per hit
    assert np.all(C.sum(axis=2) == ev.n_hits)


def test_p2_displaced_total_is_valid_rows():
    spec = tiny_spec(n_qpt=8, n_phi=16, n_d0=4, d0=(-120.0, 120.0))
    tab = oracle.Tables(spec)
    layer, phi, _ = random_hits(np.random.default_rng(5), 300)
    C = oracle.vote_count(tab, layer, phi)
    valid_rows = tab.V.reshape(10, -1).sum(axis=1)
    assert int(C.sum()) == int(valid_rows[layer].sum())


def test_p3_mask_popcount_bounded_by_counts():
    spec = synth.grid_spec("c1_single_100trk")
    tab = oracle.Tables(spec)
    ev = synth.gen_config("c1_single_100trk")
    A = oracle.vote_mask(tab, ev.layer, ev.phi)
    C = oracle.vote_count(tab, ev.layer, ev.phi)
    pop = np.unpackbits(A.view(np.uint8)).reshape(A.shape + (16,)).sum(-1)
    assert np.all(pop <= C)
    assert np.all((A == 0) == (C == 0))
    assert pop.sum() < C.sum()            # 2000 hits on 256 bins share cells


def test_p3_single_track_sets_ten_bits_per_row():
    spec = synth.grid_spec("c1_single_100trk")
    tab = oracle.Tables(spec)
    layer, phi, _ = synth.track_hits(0.37, 1.1)
    A = oracle.vote_mask(tab, layer, phi)
    pop = np.unpackbits(A.view(np.uint8)).sum()
    assert pop == 10 * spec["n_qpt"]
    C = oracle.vote_count(tab, layer, phi)
    assert C.sum() == 10 * spec["n_qpt"]


# --------------------------------------------------------------------------
# P4 / P5: bin-centre tracks and missing-hit tolerance
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name,cells", [
    ("c1_single_100trk", [(0, 0), (255, 255), (128, 17), (3, 250)]),
    ("c2_single_1ktrk_rz", [(0, 1023), (511, 0), (1023, 512)]),
])
def test_p4_bin_centre_track_full_layer_peak(name, cells):
    spec = synth.grid_spec(name)
    tab = oracle.Tables(spec)
    K, N = spec["n_qpt"], spec["n_phi"]
    kap = centres(spec["qpt_lo"], spec["qpt_hi"], K)
    for k, p in cells:
        phi0 = (p + 0.5) / N * 2 * math.pi
        layer, phi, _ = synth.track_hits(kap[k], phi0)
        A = oracle.vote_mask(tab, layer, phi)
        assert A[0, k, p] == 0x3FF
        pk = oracle.peaks(tab, A)
        assert (k * N + p) in set(pk["cell"].tolist())


def test_p4_bin_centre_track_in_noise():
    spec = synth.grid_spec("c1_single_100trk")
    tab = oracle.Tables(spec)
    ev = synth.gen_config("c1_single_100trk")
    kap = centres(-1, 1, 256)
    k, p = 77, 201
    layer, phi, _ = synth.track_hits(kap[k], (p + 0.5) / 256 * 2 * math.pi)
    A = oracle.vote_mask(tab, np.concatenate([ev.layer, layer]), np.concatenate([ev.phi, phi]))
    assert A[0, k, p] == 0x3FF
    pk = oracle.peaks(tab, A)
    row = pk[pk["cell"] == k * 256 + p]
    assert len(row) == 1 and row["popcount"][0] == 10 and row["mask"][0] == 0x3FF


def test_p4_displaced_bin_centre_tracks():
    spec = synth.grid_spec("c3_pileup_displaced_3d")
    spec.update(n_qpt=64, n_phi=128)
    tab = oracle.Tables(spec)
    kap = centres(-1, 1, 64)
    d0c = centres(-100, 100, 64)
    r = np.array(spec["layer_r_mm"])
    for d, k, p in [(0, 5, 7), (31, 40, 127), (63, 63, 0), (20, 0, 64)]:
        layer, phi, _ = synth.track_hits(kap[k], (p + 0.5) / 128 * 2 * math.pi, d0=d0c[d])
        A = oracle.vote_mask(tab, layer, phi)
        expect = int(np.sum(r > abs(d0c[d])))
        assert len(layer) == expect
        assert bin(int(A[d, k, p])).count("1") == expect
        pk = oracle.peaks(tab, A) if expect >= spec["threshold"] else None
        if pk is not None:
            assert ((d * 64 + k) * 128 + p) in set(pk["cell"].tolist())


def test_p5_missing_hits_still_peak():
    spec = synth.grid_spec("c1_single_100trk")
    tab = oracle.Tables(spec)
    kap = centres(-1, 1, 256)
    k, p = 200, 33
    layer, phi, _ = synth.track_hits(kap[k], (p + 0.5) / 256 * 2 * math.pi, drop_layers=(2, 7))
    A = oracle.vote_mask(tab, layer, phi)
    assert A[0, k, p] == 0x3FF & ~((1 << 2) | (1 << 7))
    pk = oracle.peaks(tab, A)
    row = pk[pk["cell"] == k * 256 + p]
    assert len(row) == 1 and row["popcount"][0] == 8
    # one more missing hit drops it under the threshold of 8 layers
    layer, phi, _ = synth.track_hits(kap[k], (p + 0.5) / 256 * 2 * math.pi, drop_layers=(2, 7, 9))
    pk = oracle.peaks(tab, oracle.vote_mask(tab, layer, phi))
    assert (k * 256 + p) not in set(pk["cell"].tolist())


# --------------------------------------------------------------------------
# P7 / P8: exact symmetries
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c1_single_100trk", "c3_small"])
def test_p7_rotation_covariance(name):
    if name == "c3_small":
        spec = tiny_spec(n_qpt=32, n_phi=64, n_d0=8, d0=(-100.0, 100.0), threshold=7)
        layer, phi, _ = random_hits(np.random.default_rng(3), 400)
    else:
        spec = synth.grid_spec(name)
        ev = synth.gen_config(name)
        layer, phi = ev.layer, ev.phi
    tab = oracle.Tables(spec)
    N = spec["n_phi"]
    W = (1 << 32) // N
    A = oracle.vote_mask(tab, layer, phi)
    pk = oracle.peaks(tab, A)
    for m in (1, 5, N - 1):
        phi2 = (phi.astype(np.uint64) + m * W) % (1 << 32)
        A2 = oracle.vote_mask(tab, layer, phi2.astype(np.uint32))
        np.testing.assert_array_equal(A2, np.roll(A, m, axis=2))
        pk2 = oracle.peaks(tab, A2)
        cells = pk["cell"].astype(np.int64)
        rot = (cells // N) * N + (cells % N + m) % N
        assert sorted(rot.tolist()) == pk2["cell"].tolist()


def test_p8_hit_order_independence():
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    spec.update(n_qpt=256, n_phi=256)
    tab = oracle.Tables(spec)
    ev = synth.gen_config(name)
    layer, phi, z = ev.layer[:4000], ev.phi[:4000], ev.z[:4000]
    A, pk, _ = oracle.run_event(tab, layer, phi, z, with_rz=False)
    sel = pk[::97]
    r = oracle.rz(tab, layer, phi, z, sel)
    perm = np.random.default_rng(9).permutation(len(layer))
    A2, pk2, _ = oracle.run_event(tab, layer[perm], phi[perm], z[perm], with_rz=False)
    np.testing.assert_array_equal(A, A2)
    np.testing.assert_array_equal(pk, pk2)
    r2 = oracle.rz(tab, layer[perm], phi[perm], z[perm], sel)
    np.testing.assert_array_equal(r, r2)


# --------------------------------------------------------------------------
# Local maxima: a library maximum filter and hand-worked cases
# --------------------------------------------------------------------------

def popcount16(A):
    return np.unpackbits(A.view(np.uint8)).reshape(A.shape + (16,)).sum(-1)


def filter_peaks(spec, A):
    pop = popcount16(A).astype(np.int32)
    if spec["n_d0"] == 1:
        mx = ndimage.maximum_filter(pop[0], size=3, mode=["constant", "wrap"], cval=-1)[None]
    else:
        mx = ndimage.maximum_filter(pop, size=3, mode=["constant", "constant", "wrap"], cval=-1)
    ok = (pop >= spec["threshold"]) & (pop == mx)
    return np.flatnonzero(ok.ravel())


@pytest.mark.parametrize("n_d0,fill", [(1, 0.5), (1, 0.8), (4, 0.7), (1, 0.95)])
def test_peaks_match_maximum_filter(n_d0, fill):
    spec = tiny_spec(n_qpt=24, n_phi=32, n_d0=n_d0, d0=(-50.0, 50.0), threshold=5)
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(int(fill * 100) + n_d0)
    bits = rng.random((n_d0, 24, 32, 10)) < fill
    A = (bits * (1 << np.arange(10))).sum(-1).astype(np.uint16)
    pk = oracle.peaks(tab, A)
    np.testing.assert_array_equal(pk["cell"], filter_peaks(spec, A))
    np.testing.assert_array_equal(pk["mask"], A.ravel()[pk["cell"]])
    np.testing.assert_array_equal(pk["popcount"], popcount16(A).ravel()[pk["cell"]])


def _mask(n):
    return (1 << n) - 1


def test_peaks_hand_cases_2d():
    spec = tiny_spec(n_qpt=4, n_phi=8, threshold=8)
    tab = oracle.Tables(spec)
    A = np.zeros((1, 4, 8), np.uint16)
    A[0, 0, 3] = _mask(9)              # isolated 9: a peak
    A[0, 2, 4] = _mask(9)              # plateau of two 9s: both peaks (non-strict)
    A[0, 2, 5] = _mask(9)
    A[0, 0, 0] = _mask(8)              # p = 0 with a 10 at p = 7 in the row below: wrap kills it
    A[0, 1, 7] = _mask(10)             # the 10 itself is a peak
    A[0, 0, 1] = _mask(10)             # a 10 in row 0 ...
    A[0, 3, 0] = _mask(9)              # ... is no neighbour of row 3: kappa does not wrap
    A[0, 3, 2] = _mask(7)              # under threshold
    pk = oracle.peaks(tab, A)
    want = [0 * 8 + 1, 0 * 8 + 3, 1 * 8 + 7, 2 * 8 + 4, 2 * 8 + 5, 3 * 8 + 0]
    assert pk["cell"].tolist() == want


def test_peaks_hand_cases_3d():
    spec = tiny_spec(n_qpt=3, n_phi=4, n_d0=3, d0=(-30.0, 30.0), threshold=7)
    tab = oracle.Tables(spec)
    A = np.zeros((3, 3, 4), np.uint16)
    A[1, 1, 0] = _mask(8)
    A[2, 2, 3] = _mask(9)              # diagonal neighbour (d+1, k+1, p-1 wrapped): kills (1,1,0)
    A[0, 0, 2] = _mask(7)              # isolated at threshold: a peak
    pk = oracle.peaks(tab, A)
    assert pk["cell"].tolist() == sorted([(2 * 3 + 2) * 4 + 3, (0 * 3 + 0) * 4 + 2])


# --------------------------------------------------------------------------
# rz refinement: dense argmax, bin-centre track, hand cases
# --------------------------------------------------------------------------

def dense_rz(tab, layer, phi, z, cell):
    """R[j][b] materialised in full, argmax by numpy (first = smallest j, b)."""
    s = tab.spec
    N, K = s["n_phi"], s["n_qpt"]
    sh = 32 - int(math.log2(N))
    k, p = (cell // N) % K, cell % N
    mem = [h for h in range(len(layer))
           if ((int(phi[h]) - int(tab.O[layer[h], 0, k])) % (1 << 32)) >> sh == p]
    R = np.zeros((s["n_cot"], s["n_z0"]), np.int64)
    span = s["z0_hi_um"] - s["z0_lo_um"]
    for h in mem:
        z0 = int(z[h]) - tab.Z[k, layer[h], :].astype(np.int64)
        b = np.floor_divide((z0 - s["z0_lo_um"]) * s["n_z0"], span)
        ok = (b >= 0) & (b < s["n_z0"])
        np.add.at(R, (np.nonzero(ok)[0], b[ok]), 1)
    i = int(np.argmax(R))
    return i // s["n_z0"], i % s["n_z0"], int(R.max()), len(mem)


def test_rz_matches_dense_argmax():
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    spec.update(n_qpt=128, n_phi=128)
    tab = oracle.Tables(spec)
    ev = synth.gen_config(name)
    layer, phi, z = ev.layer[:3000], ev.phi[:3000], ev.z[:3000]
    A, pk, _ = oracle.run_event(tab, layer, phi, z, with_rz=False)
    sel = pk[::max(1, len(pk) // 25)]
    r = oracle.rz(tab, layer, phi, z, sel)
    for i, rec in enumerate(r):
        j, b, cnt, nm = dense_rz(tab, layer, phi, z, int(sel["cell"][rec["peak"]]))
        assert (rec["cot_bin"], rec["z0_bin"], rec["count"], rec["n_members"]) == (j, b, cnt, nm)


def test_p6_rz_bin_centre_track():
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    tab = oracle.Tables(spec)
    kap = centres(-1, 1, 1024)
    cotc = centres(-1.2, 1.2, 256)
    for k, p, j, b in [(100, 7, 31, 128), (900, 1000, 200, 3), (512, 512, 128, 250)]:
        z0_mm = (-200000 + (b + 0.5) * 400000 / 256) / 1000.0
        layer, phi, z = synth.track_hits(kap[k], (p + 0.5) / 1024 * 2 * math.pi,
                                         cot=cotc[j], z0=z0_mm)
        A, pk, r = oracle.run_event(tab, layer, phi, z)
        i = int(np.nonzero(pk["cell"] == k * 1024 + p)[0][0])
        rec = r[r["peak"] == i][0]
        assert (rec["cot_bin"], rec["z0_bin"], rec["count"], rec["n_members"]) == (j, b, 10, 10)


def test_rz_binning_edges_and_ties():
    # one cot bin centred on 0 -> Z = 0 and z0 = z: bins are floor((z - lo) * n / span)
    spec = tiny_spec(n_qpt=2, n_phi=4, threshold=0)
    spec.update(n_z0=4, z0_lo_um=-100, z0_hi_um=100, n_cot=1, cot_lo=-0.5, cot_hi=0.5)
    tab = oracle.Tables(spec)
    assert not tab.Z.any()

    def rec_for(zs):
        zs = np.array(zs, np.int32)
        n = len(zs)
        layer = np.arange(n, dtype=np.uint8) % 10
        # every hit in the same cell of row 0: phi = O[l][0][0] + half a bin
        phi = (tab.O[layer, 0, 0].astype(np.uint64) + (1 << 29)) % (1 << 32)
        pk = np.zeros(1, oracle.PEAK_DTYPE)
        pk["cell"] = 0
        pk["popcount"] = n
        return oracle.rz(tab, layer, phi.astype(np.uint32), zs, pk)[0]

    r = rec_for([-100, -51, 99, 100, -101])     # bins 0, 0, 3, out, out
    assert (r["z0_bin"], r["count"], r["n_members"]) == (0, 2, 5)
    r = rec_for([60, -60])                       # one each in bins 3 and 0: tie -> smaller bin
    assert (r["z0_bin"], r["count"]) == (0, 1)
    r = rec_for([100, 250])                      # nothing in range -> (0, 0) with count 0
    assert (r["cot_bin"], r["z0_bin"], r["count"], r["n_members"]) == (0, 0, 0, 2)
    r = rec_for([-1, 0])                         # floor, not truncation: -1 -> bin 1, 0 -> bin 2
    assert (r["z0_bin"], r["count"]) == (1, 1)


def test_rz_candidate_order_with_cap():
    spec = tiny_spec(rz=True, rz_max_candidates=3)
    tab = oracle.Tables(spec)
    pk = np.zeros(5, oracle.PEAK_DTYPE)
    pk["popcount"] = [8, 10, 9, 10, 8]
    assert oracle.rz_candidates(tab, pk).tolist() == [1, 3, 2]
    spec["rz_max_candidates"] = 10
    assert oracle.rz_candidates(oracle.Tables(spec), pk).tolist() == [1, 3, 2, 0, 4]
    spec["rz_max_candidates"] = 0
    assert oracle.rz_candidates(oracle.Tables(spec), pk).tolist() == [0, 1, 2, 3, 4]


def test_spec_validation():
    assert oracle.check_spec(tiny_spec())
    bad = tiny_spec(); bad["n_phi"] = 48
    assert not oracle.check_spec(bad)
    bad = tiny_spec(n_d0=4, d0=(-10, 10), rz=True)
    assert not oracle.check_spec(bad)


# --------------------------------------------------------------------------
# the counting form's local maxima (the paper's A[B[i]] += 1 accumulator)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_d0,lam", [(1, 1.0), (1, 4.0), (3, 2.5)])
def test_count_peaks_match_maximum_filter(n_d0, lam):
    spec = tiny_spec(n_qpt=24, n_phi=32, n_d0=n_d0, d0=(-50.0, 50.0), threshold=3)
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(int(lam * 10) + n_d0)
    Cc = rng.poisson(lam, (n_d0, 24, 32)).astype(np.uint32)
    Cc[0, 5, 7] = 70000                                   # beyond 16 bits
    pk = oracle.peaks_count(tab, Cc)
    v = Cc.astype(np.int64)
    if n_d0 == 1:
        mx = ndimage.maximum_filter(v[0], size=3, mode=["constant", "wrap"], cval=-1)[None]
    else:
        mx = ndimage.maximum_filter(v, size=3, mode=["constant", "constant", "wrap"], cval=-1)
    want = np.flatnonzero(((v >= spec["threshold"]) & (v == mx)).ravel())
    np.testing.assert_array_equal(pk["cell"], want)
    np.testing.assert_array_equal(pk["count"], Cc.ravel()[want])
    assert Cc.ravel()[5 * 32 + 7 + 0] == 70000 and (5 * 32 + 7) in pk["cell"]


def test_count_peaks_equal_mask_peaks_when_layers_hit_once():
    # with at most one hit per layer per cell the count of a cell equals the
    # popcount of its layer mask, so both peak lists coincide
    spec = synth.grid_spec("c1_single_100trk")
    spec.update(n_qpt=64, n_phi=128, threshold=6)
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(5)
    layer, phi, _ = synth.track_hits(rng.uniform(-1, 1, 30), rng.uniform(0, 2 * np.pi, 30))
    Cc = oracle.vote_count(tab, layer, phi)
    A = oracle.vote_mask(tab, layer, phi)
    if (Cc == popcount16(A)).all():
        pc, pm = oracle.peaks_count(tab, Cc), oracle.peaks(tab, A)
        np.testing.assert_array_equal(pc["cell"], pm["cell"])
        np.testing.assert_array_equal(pc["count"], pm["popcount"])
    else:                                                  # two tracks met in a cell
        assert (Cc >= popcount16(A)).all()


def test_count_peaks_hand_cases_and_capacity():
    spec = tiny_spec(n_qpt=3, n_phi=8, threshold=2)
    tab = oracle.Tables(spec)
    Cc = np.zeros((1, 3, 8), np.uint32)
    Cc[0, 0, 0] = 5                        # row 0, p 0 ...
    Cc[0, 1, 7] = 5                        # ... ties with its wrapped diagonal neighbour: both peaks
    Cc[0, 2, 5] = 2                        # at threshold, isolated: peak
    Cc[0, 2, 4] = 1                        # below threshold
    Cc[0, 1, 2] = 3                        # loses to (0, 2) above it
    Cc[0, 0, 2] = 4                        # peak
    Cc[0, 2, 1] = 2                        # at threshold but (1, 2) = 3 is a diagonal neighbour
    pk = oracle.peaks_count(tab, Cc)
    assert pk["cell"].tolist() == [0, 2, 15, 21]
    assert pk["count"].tolist() == [5, 4, 5, 2]
    cell = np.zeros(2, np.uint32)
    cnt = np.zeros(2, np.uint32)
    import ctypes
    n = oracle._load().orc_peaks_count(ctypes.byref(tab.cs), oracle._p(Cc.reshape(-1)), oracle._p(cell),
                                       oracle._p(cnt), 2)
    assert n == 4 and cell.tolist() == [0, 2]


# --------------------------------------------------------------------------
# Candidate confirmation: plateau clusters of adjacent peaks
# --------------------------------------------------------------------------

def peak_list(A, cells):
    """Peak records for the given cells of A (any cells: the clustering
    does not re-check the local-maximum rule)."""
    cells = np.sort(np.asarray(cells, np.int64))
    pk = np.zeros(len(cells), oracle.PEAK_DTYPE)
    pk["cell"] = cells
    pk["mask"] = A.ravel()[cells]
    pk["popcount"] = popcount16(A).ravel()[cells]
    return pk


def _random_image(rng, shape, density):
    img = rng.random(shape) < density
    c0 = int(rng.integers(shape[-1]))
    img[..., c0] = False                       # an empty phi0 column
    return img, c0


@pytest.mark.parametrize("n_d0,density,seed", [(1, 0.25, 0), (1, 0.35, 1), (1, 0.6, 2),
                                                (3, 0.15, 3), (3, 0.25, 4)])
def test_clusters_match_ndimage_label(n_d0, density, seed):
    # With an empty phi0 column rolled to the array edge no adjacency crosses
    # the edge, so scipy's non-periodic labelling with full connectivity gives
    # exactly the periodic components.
    rng = np.random.default_rng(seed)
    spec = tiny_spec(n_qpt=20, n_phi=32, n_d0=n_d0, d0=(-50.0, 50.0), threshold=1)
    tab = oracle.Tables(spec)
    img, c0 = _random_image(rng, (n_d0, 20, 32), density)
    A = (rng.integers(1, 1 << 10, img.shape) * img).astype(np.uint16)
    pk = peak_list(A, np.flatnonzero(img.ravel()))
    lab, cl = oracle.clusters(tab, pk)
    rolled = np.roll(img, -c0, axis=-1)
    ref, n_ref = ndimage.label(rolled if n_d0 > 1 else rolled[0],
                               structure=np.ones((3,) * (3 if n_d0 > 1 else 2)))
    ref = np.roll(ref.reshape(img.shape), c0, axis=-1).ravel()[pk["cell"]]
    assert len(cl) == n_ref
    pairs = set(zip(lab.tolist(), ref.tolist()))
    assert len(pairs) == n_ref                  # one-to-one between the two labellings
    # numbering: by first peak, which is the smallest index carrying the label
    assert np.all(np.diff(cl["first"].astype(np.int64)) > 0)
    first_idx = np.array([np.flatnonzero(lab == c)[0] for c in range(len(cl))])
    np.testing.assert_array_equal(cl["first"], first_idx)
    np.testing.assert_array_equal(cl["n_peaks"], np.bincount(lab, minlength=len(cl)))
    # OR of masks and the first peak's popcount
    for c in range(len(cl)):
        assert cl["mask_or"][c] == np.bitwise_or.reduce(pk["mask"][lab == c])
    np.testing.assert_array_equal(cl["popcount"], pk["popcount"][cl["first"]])
    # centroids against scipy's centre of mass in the rolled frame, for
    # clusters narrower than half the phi0 period
    D, K, P = oracle.cluster_centroids(tab, pk, cl)
    rl, _ = ndimage.label(rolled, structure=np.ones((3, 3, 3)) if n_d0 > 1 else
                          np.pad(np.ones((1, 3, 3)), ((1, 1), (0, 0), (0, 0))))
    idx = np.arange(1, n_ref + 1)
    com = np.array(ndimage.center_of_mass(rolled.astype(float), rl, idx))
    ext = [s[-1].stop - s[-1].start for s in ndimage.find_objects(rl)]
    rcell = pk["cell"][cl["first"]]
    rpos = np.array(np.unravel_index(rcell, img.shape)).T
    rpos[:, 2] = (rpos[:, 2] - c0) % 32
    rlab = rl[tuple(rpos.T)]                    # scipy label of each cluster's first peak
    checked = 0
    for c in range(len(cl)):
        j = rlab[c] - 1
        if ext[j] >= 16:
            continue
        checked += 1
        assert D[c] == pytest.approx(com[j][0], abs=1e-12)
        assert K[c] == pytest.approx(com[j][1], abs=1e-12)
        assert (P[c] - c0) % 32 == pytest.approx(com[j][2], abs=1e-9)
    assert checked >= len(cl) // 2


def test_clusters_hand_cases():
    spec = tiny_spec(n_qpt=4, n_phi=8, threshold=1)
    tab = oracle.Tables(spec)
    A = np.zeros((1, 4, 8), np.uint16)
    cells = [(0, 0), (0, 7),                   # wrap neighbours in phi0: one cluster
             (1, 3),                           # diagonal of nothing: alone
             (2, 5), (3, 6),                   # diagonal pair
             (3, 0)]                           # kappa does not wrap: (0, 0) is no neighbour
    for k, p in cells:
        A[0, k, p] = 0x7
    A[0, 0, 7] = 0x38
    pk = peak_list(A, [k * 8 + p for k, p in cells])
    lab, cl = oracle.clusters(tab, pk)
    # list order: 0, 7, 11, 21, 24, 30
    assert lab.tolist() == [0, 0, 1, 2, 3, 2]
    assert cl["first"].tolist() == [0, 2, 3, 4]
    assert cl["n_peaks"].tolist() == [2, 1, 2, 1]
    assert cl["sum_dp"].tolist() == [-1, 0, 1, 0]  # (0,7) is one step below (0,0)
    assert cl["sum_dk"].tolist() == [0, 0, 1, 0]
    assert cl["mask_or"].tolist() == [0x3F, 0x7, 0x7, 0x7]
    _, _, P = oracle.cluster_centroids(tab, pk, cl)
    assert P[0] == pytest.approx(7.5)          # centroid across the wrap


def test_clusters_two_phi_bins_and_d0_axis():
    # n_phi = 2: both phi0 neighbours are the same cell
    spec = tiny_spec(n_qpt=3, n_phi=2, threshold=1)
    tab = oracle.Tables(spec)
    A = np.full((1, 3, 2), 1, np.uint16)
    lab, cl = oracle.clusters(tab, peak_list(A, [0, 1, 5]))
    assert lab.tolist() == [0, 0, 1] and cl["sum_dp"].tolist() == [-1, 0]
    # d0 axis: (d, k, p) and (d + 1, k + 1, p - 1) touch; d does not wrap
    spec = tiny_spec(n_qpt=3, n_phi=4, n_d0=3, d0=(-30.0, 30.0), threshold=1)
    tab = oracle.Tables(spec)
    A = np.full((3, 3, 4), 1, np.uint16)
    c = lambda d, k, p: (d * 3 + k) * 4 + p
    lab, cl = oracle.clusters(tab, peak_list(A, [c(0, 0, 0), c(1, 1, 3), c(2, 0, 0)]))
    assert lab.tolist() == [0, 0, 0] and cl["sum_dd"].tolist() == [3]
    lab, cl = oracle.clusters(tab, peak_list(A, [c(0, 1, 1), c(2, 1, 1)]))
    assert lab.tolist() == [0, 1]


@pytest.mark.parametrize("name,cells", [
    ("c1_single_100trk", [(128, 17), (77, 201), (40, 255)]),
    ("c2_single_1ktrk_rz", [(512, 1023), (300, 0)]),
])
def test_clusters_merge_a_bin_centre_ridge(name, cells):
    # One noiseless bin-centre track leaves a ridge of equal full-layer peaks
    # along q/pT; away from the q/pT edges the ridge is symmetric about the
    # track's bin, so it becomes one cluster whose centroid is that bin.
    spec = synth.grid_spec(name)
    tab = oracle.Tables(spec)
    K, N = spec["n_qpt"], spec["n_phi"]
    kap = centres(spec["qpt_lo"], spec["qpt_hi"], K)
    for k, p in cells:
        layer, phi, _ = synth.track_hits(kap[k], (p + 0.5) / N * 2 * math.pi)
        pk = oracle.peaks(tab, oracle.vote_mask(tab, layer, phi))
        assert len(pk) > 1
        lab, cl = oracle.clusters(tab, pk)
        assert len(cl) == 1 and cl["popcount"][0] == 10 and cl["mask_or"][0] == 0x3FF
        _, kc, pc = oracle.cluster_centroids(tab, pk, cl)
        assert kc[0] == k and pc[0] == p


def test_clusters_of_real_peaks_are_equal_valued_and_separated():
    # Adjacent local maxima are each >= the other, so a cluster's members
    # share one popcount; members of different clusters are never adjacent.
    spec = tiny_spec(n_qpt=32, n_phi=64, threshold=4)
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(5)
    layer, phi, _ = random_hits(rng, 300)
    pk = oracle.peaks(tab, oracle.vote_mask(tab, layer, phi))
    lab, cl = oracle.clusters(tab, pk)
    assert len(cl) < len(pk)
    np.testing.assert_array_equal(pk["popcount"], cl["popcount"][lab])
    k = pk["cell"] // 64
    p = pk["cell"] % 64
    dk = np.abs(k[:, None].astype(int) - k[None, :])
    dp = np.abs(p[:, None].astype(int) - p[None, :])
    adj = (dk <= 1) & (np.minimum(dp, 64 - dp) <= 1)
    same = lab[:, None] == lab[None, :]
    assert not np.any(adj & ~same)


# --------------------------------------------------------------------------
# Candidate confirmation: track fit over a cluster's first-cell members
# --------------------------------------------------------------------------

def _clusters_of(tab, layer, phi):
    pk = oracle.peaks(tab, oracle.vote_mask(tab, layer, phi))
    lab, cl = oracle.clusters(tab, pk)
    return pk, cl


@pytest.mark.parametrize("name,qpt,phi0", [
    ("c2_single_1ktrk_rz", 0.3131, 1.234), ("c2_single_1ktrk_rz", -0.8765, 4.5678),
    ("c2_single_1ktrk_rz", 0.0217, 0.0004), ("c2_single_1ktrk_rz", -0.5, 2 * math.pi - 0.0007),
    ("c1_single_100trk", 0.61, 3.0), ("c1_single_100trk", -0.05, 5.9)])
def test_fit_recovers_generator_track(name, qpt, phi0):
    # noiseless hits from the generator's own helix construction, at track
    # parameters off the bin centres: the fit lands on the true parameters
    # (to the uint32 azimuth quantisation), closer than the cluster centroid
    spec = synth.grid_spec(name)
    tab = oracle.Tables(spec)
    layer, phi, _ = synth.track_hits(qpt, phi0)
    pk, cl = _clusters_of(tab, layer, phi)
    f = oracle.fit(tab, layer, phi, pk, cl)
    good = f[f["status"] == 1]
    # side plateaus of a lower popcount can form their own clusters; every
    # member is still a hit of this track
    assert np.any((good["n_hits"] == 10) & (cl["popcount"][f["status"] == 1] == 10))
    assert np.all(np.abs(good["qpt"] - qpt) < 2e-6)
    dphi = np.angle(np.exp(1j * (good["phi0"] - phi0)))
    assert np.all(np.abs(dphi) < 1e-7)
    assert np.all(good["rms_mm"] < 1e-5)
    assert np.all((good["phi0"] >= 0) & (good["phi0"] < 2 * math.pi))
    dc = np.abs(good["qpt_c"] - qpt)
    assert np.all(np.abs(good["qpt"] - qpt) < dc + 1e-12)


def test_fit_matches_lstsq_on_noisy_members():
    # with noise hits among the members the fit is the least-squares
    # solution of the linear system y' = t x' - alpha r^2 (numpy lstsq)
    spec = synth.grid_spec("c1_single_100trk")
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(21)
    layer, phi, _ = synth.track_hits(rng.uniform(-0.9, 0.9, 40), rng.uniform(0, 2 * math.pi, 40),
                                     rng=rng)
    nl, nphi, _ = random_hits(rng, 3000)
    layer, phi = np.concatenate([layer, nl]), np.concatenate([phi, nphi])
    pk, cl = _clusters_of(tab, layer, phi)
    f = oracle.fit(tab, layer, phi, pk, cl)
    s = 32 - 8
    R = np.asarray(spec["layer_r_mm"][:spec["n_layers"]])
    checked = 0
    for c in np.flatnonzero(f["status"] == 1)[:300]:
        cell = int(pk["cell"][cl["first"][c]])
        k, p = cell // 256, cell % 256
        mem = [h for h in range(len(layer)) if tab.V[layer[h], 0, k]
               and ((int(phi[h]) - int(tab.O[layer[h], 0, k])) % (1 << 32)) >> s == p]
        assert len(mem) == f["n_hits"][c]
        ref = (p << s) + (1 << (s - 1))
        ang = ((phi[mem].astype(np.int64) - ref + (1 << 31)) % (1 << 32) - (1 << 31)) * (2 * math.pi / 2 ** 32)
        r = R[layer[mem]]
        x, y = r * np.cos(ang), r * np.sin(ang)
        sol, *_ = np.linalg.lstsq(np.stack([x, -r * r], 1), y, rcond=None)
        t, alpha = sol
        cosp = 1 / math.sqrt(1 + t * t)
        assert f["phi0"][c] == pytest.approx((ref * 2 * math.pi / 2 ** 32 + math.atan(t)) % (2 * math.pi),
                                             abs=1e-9)
        assert f["qpt"][c] == pytest.approx(2 * alpha * cosp / (0.299792458e-3 * spec["b_tesla"]),
                                            rel=1e-7, abs=1e-9)
        res = (y - t * x + alpha * r * r) * cosp
        assert f["rms_mm"][c] == pytest.approx(math.sqrt(np.mean(res ** 2)), rel=1e-6, abs=1e-9)
        checked += 1
    assert checked >= 20


def test_fit_centroid_and_degenerate_clusters():
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    tab = oracle.Tables(spec)
    K, N = spec["n_qpt"], spec["n_phi"]
    kap = centres(spec["qpt_lo"], spec["qpt_hi"], K)
    k, p = 700, 3
    layer, phi, _ = synth.track_hits(kap[k], (p + 0.5) / N * 2 * math.pi)
    pk, cl = _clusters_of(tab, layer, phi)
    f = oracle.fit(tab, layer, phi, pk, cl)
    assert len(f) == 1
    assert f["qpt_c"][0] == pytest.approx(kap[k], abs=1e-12)
    assert f["phi0_c"][0] == pytest.approx((p + 0.5) / N * 2 * math.pi, abs=1e-12)
    # a cluster whose first cell holds fewer than three hits is not fitted
    fake = np.zeros(2, oracle.PEAK_DTYPE)
    fake["cell"] = [5 * N + 100, 9 * N + 7]
    lab, fcl = oracle.clusters(tab, fake)
    two = np.zeros(2, np.uint8), np.array([0, 1 << 20], np.uint32)
    g = oracle.fit(tab, two[0], two[1], fake, fcl)
    assert g["status"].tolist() == [0, 0]
    assert np.all(g["qpt"] == 0) and np.all(g["rms_mm"] == 0)
    assert g["qpt_c"][1] == pytest.approx(kap[9], abs=1e-12)


@pytest.mark.parametrize("qpt,phi0,cot,z0", [(0.3131, 1.234, 0.7, 23.4), (-0.8765, 4.5678, -1.1, -80.0),
                                             (0.0217, 0.0004, 0.05, 1.5), (0.6, 6.0, 0.0, 0.0)])
def test_helix_fit_recovers_generator_cot_and_z0(qpt, phi0, cot, z0):
    # noiseless generator helices (z quantised to 1 um): the line through
    # (arc length, z) of the members gives back cot(theta) and z0
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    tab = oracle.Tables(spec)
    layer, phi, z = synth.track_hits(qpt, phi0, cot=cot, z0=z0)
    pk, cl = _clusters_of(tab, layer, phi)
    f = oracle.fit(tab, layer, phi, pk, cl, z)
    g = f[f["status_z"] == 1]
    assert len(g) == np.count_nonzero(f["status"]) >= 1
    assert np.all(np.abs(g["cot"] - cot) < 5e-6)
    assert np.all(np.abs(g["z0_mm"] - z0) < 1e-3)
    assert np.all(g["rms_z_mm"] < 1e-3)
    # without z only the transverse part is fitted
    h = oracle.fit(tab, layer, phi, pk, cl)
    assert np.all(h["status_z"] == 0) and np.all(h["cot"] == 0)
    np.testing.assert_array_equal(h["qpt"], f["qpt"])


def test_helix_fit_line_matches_lstsq():
    spec = synth.grid_spec("c2_single_1ktrk_rz")
    tab = oracle.Tables(spec)
    rng = np.random.default_rng(31)
    layer, phi, z = synth.track_hits(rng.uniform(-0.9, 0.9, 30), rng.uniform(0, 2 * math.pi, 30),
                                     cot=rng.uniform(-1, 1, 30), z0=rng.normal(0, 50, 30), rng=rng)
    nl, nphi, nz = random_hits(rng, 20000)
    layer, phi, z = (np.concatenate([layer, nl]), np.concatenate([phi, nphi]), np.concatenate([z, nz]))
    pk, cl = _clusters_of(tab, layer, phi)
    f = oracle.fit(tab, layer, phi, pk, cl, z)
    s = 32 - 10
    R = np.asarray(spec["layer_r_mm"][:spec["n_layers"]])
    C = 0.299792458e-3 * spec["b_tesla"]
    checked = 0
    for c in np.flatnonzero(f["status_z"] == 1)[:200]:
        cell = int(pk["cell"][cl["first"][c]])
        k, p = cell // 1024, cell % 1024
        mem = np.array([h for h in range(len(layer)) if tab.V[layer[h], 0, k]
                        and ((int(phi[h]) - int(tab.O[layer[h], 0, k])) % (1 << 32)) >> s == p])
        r = R[layer[mem]]
        x = 0.5 * f["qpt"][c] * C * r
        sa = np.where(x == 0, r, r * np.arcsin(x) / np.where(x == 0, 1, x))
        sol, *_ = np.linalg.lstsq(np.stack([np.ones_like(sa), sa], 1), z[mem] * 1e-3, rcond=None)
        assert f["z0_mm"][c] == pytest.approx(sol[0], rel=1e-7, abs=1e-7)
        assert f["cot"][c] == pytest.approx(sol[1], rel=1e-7, abs=1e-9)
        res = z[mem] * 1e-3 - sol[0] - sol[1] * sa
        assert f["rms_z_mm"][c] == pytest.approx(math.sqrt(np.mean(res ** 2)), rel=1e-6, abs=1e-9)
        checked += 1
    assert checked >= 20
