"""The five benchmark workloads: detector, track populations and grid specs.

The paper's own study uses a transverse-plane toy Monte Carlo (Section 4,
"Hough Transform Algorithm", the paragraph on the simulated detector); the
workloads below are synthetic stand-ins of the same kind with a 10-layer
barrel, a 3.8 T field and uint32 fixed-point azimuth.

A grid spec is a plain dict whose keys mirror the C struct fields of the
library header and of the oracle; each side converts it to its own struct.
"""

DETECTOR_R_MM = (40.0, 70.0, 110.0, 250.0, 340.0, 430.0, 520.0, 610.0, 700.0, 800.0)
B_TESLA = 3.8
Z_ACCEPT_MM = 1200.0


# The paper's own toy detector (Section 4): 10 evenly spaced layers out to
# 1.1 m (read as r = 11 i cm), 0.4 mm hit resolution.
PAPER_R_MM = tuple(110.0 * i for i in range(1, 11))


def _spec(n_qpt, n_phi, threshold, n_d0=1, d0=(0.0, 0.0), rz=False,
          rz_max_candidates=0, radii=DETECTOR_R_MM):
    s = dict(
        n_layers=len(radii), layer_r_mm=list(radii),
        b_tesla=B_TESLA,
        n_qpt=n_qpt, qpt_lo=-1.0, qpt_hi=1.0,
        n_phi=n_phi,
        n_d0=n_d0, d0_lo_mm=d0[0], d0_hi_mm=d0[1],
        threshold=threshold,
        n_z0=0, z0_lo_um=0, z0_hi_um=0,
        n_cot=0, cot_lo=0.0, cot_hi=0.0,
        rz_max_candidates=rz_max_candidates,
    )
    if rz:
        s.update(n_z0=256, z0_lo_um=-200000, z0_hi_um=200000,
                 n_cot=256, cot_lo=-1.2, cot_hi=1.2)
    return s


# Workload descriptions.  "noise" is either an absolute count or, when
# "noise_per_track_hit" is set, a multiple of the event's track-hit count.
CONFIGS = {
    "c1_single_100trk": dict(
        index=0, n_events=1, tracks=("fixed", 100), noise=1000,
        displaced_frac=0.0,
        spec=_spec(256, 256, 8)),
    "c2_single_1ktrk_rz": dict(
        index=1, n_events=1, tracks=("fixed", 1000), noise=10000,
        displaced_frac=0.0,
        spec=_spec(1024, 1024, 8, rz=True)),
    "c3_pileup_displaced_3d": dict(
        index=2, n_events=1, tracks=("fixed", 10000), noise=100000,
        displaced_frac=0.2, d0_range_mm=(-100.0, 100.0),
        spec=_spec(512, 512, 7, n_d0=64, d0=(-100.0, 100.0))),
    "c4_batch_4096": dict(
        index=3, n_events=4096, tracks=("lognormal", 300.0, 0.8, 10, 10000),
        noise_per_track_hit=5, displaced_frac=0.0,
        spec=_spec(512, 512, 8)),
    "c5_serving": dict(
        index=4, n_events=None, tracks=("loguniform", 100, 10000),
        noise_per_track_hit=5, displaced_frac=0.0,
        spec=_spec(512, 512, 8, rz=True, rz_max_candidates=1024)),
    # the paper's counting accumulator on its 2048 x 2048 grid and detector
    # (time vs number of tracks is swept by passing n_tracks to gen_event)
    "p6_paper_2048_count": dict(
        index=5, n_events=1, tracks=("fixed", 1000), noise=0,
        displaced_frac=0.0, sigma_rphi_mm=0.4,
        spec=_spec(2048, 2048, 8, radii=PAPER_R_MM)),
}


def grid_spec(name):
    """A fresh copy of the named workload's grid spec."""
    s = dict(CONFIGS[name]["spec"])
    s["layer_r_mm"] = list(s["layer_r_mm"])
    return s


def workload(name):
    return CONFIGS[name]
