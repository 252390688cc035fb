"""Seeded synthetic events: helix tracks crossing a barrel detector, plus noise.

Hits are produced by explicit trajectory geometry (perigee point, chord,
position vector, atan2), which is deliberately a different construction from
the tracker's own inverse formula, so a bin-centre track is an independent
check of the tracker's offset tables.

Conventions (shared with the tracker only through the physics, not code):
  * B along +z; a positive q/pT bends clockwise (azimuth decreases with r).
  * Perigee point P0 = d0 * (-sin phi0, cos phi0); direction (cos phi0, sin phi0).
  * Curvature rho = 0.299792458e-3 * B[T] * q/pT[1/GeV]  in 1/mm.
  * Azimuth stored as uint32 turn fraction (2**32 == one turn), z as int32 um.
"""
from dataclasses import dataclass, field
import numpy as np

from .configs import CONFIGS, DETECTOR_R_MM, B_TESLA, Z_ACCEPT_MM

TWO_PI = 2.0 * np.pi
C_LIGHT = 0.299792458e-3        # GeV / (T * mm)
SIGMA_RPHI_MM = 0.020
SIGMA_Z_MM = 0.050
Z_NOISE_UM = 1_200_000


@dataclass
class EventBatch:
    """Structure-of-arrays hits of one or more events, concatenated."""
    layer: np.ndarray            # uint8
    phi: np.ndarray              # uint32 turn fraction
    z: np.ndarray                # int32 micrometres
    offsets: np.ndarray          # uint64 [n_events + 1]
    n_tracks: np.ndarray = field(default=None)   # per event

    @property
    def n_events(self):
        return len(self.offsets) - 1

    @property
    def n_hits(self):
        return int(self.offsets[-1])

    def event(self, e):
        a, b = int(self.offsets[e]), int(self.offsets[e + 1])
        return EventBatch(self.layer[a:b], self.phi[a:b], self.z[a:b],
                          np.array([0, b - a], dtype=np.uint64),
                          None if self.n_tracks is None else self.n_tracks[e:e + 1])


def _quantize_phi(phi_rad):
    t = np.mod(np.asarray(phi_rad, dtype=np.float64) / TWO_PI, 1.0)
    q = np.floor(t * 4294967296.0 + 0.5)
    return np.mod(q, 4294967296.0).astype(np.uint64).astype(np.uint32)


def _quantize_z(z_mm):
    return np.floor(np.asarray(z_mm, dtype=np.float64) * 1000.0 + 0.5).astype(np.int64)


def _helix_hits(kappa, phi0, d0, cot, z0, radii, b_tesla):
    """Exact crossing points of helices with the cylinders in `radii`.

    All track arrays have shape [T]; returns (phi_rad, z_mm, ok) of shape [T, L].
    The chord c from the perigee to the crossing at radius r obeys
    c^2 = (r^2 - d0^2) / (1 - rho d0); the track turns by 2*asin(rho c / 2)
    along that chord and the chord direction is phi0 minus half the turn.
    """
    kappa = np.asarray(kappa, np.float64)[:, None]
    phi0 = np.asarray(phi0, np.float64)[:, None]
    d0 = np.asarray(d0, np.float64)[:, None]
    cot = np.asarray(cot, np.float64)[:, None]
    z0 = np.asarray(z0, np.float64)[:, None]
    r = np.asarray(radii, np.float64)[None, :]
    rho = C_LIGHT * b_tesla * kappa
    denom = 1.0 - rho * d0
    c2 = (r * r - d0 * d0) / denom
    ok = (r > np.abs(d0)) & (denom > 0) & (c2 > 0)
    c = np.sqrt(np.where(ok, c2, 0.0))
    t = rho * c * 0.5
    ok &= np.abs(t) <= 1.0
    half_turn = np.arcsin(np.clip(t, -1.0, 1.0))
    x0 = -d0 * np.sin(phi0)
    y0 = d0 * np.cos(phi0)
    x = x0 + c * np.cos(phi0 - half_turn)
    y = y0 + c * np.sin(phi0 - half_turn)
    phi = np.arctan2(y, x)
    # arc length from the perigee: s = 2*asin(t)/rho, which tends to c as rho -> 0
    safe_t = np.where(np.abs(t) > 1e-12, t, 1.0)
    s = np.where(np.abs(t) > 1e-12, c * half_turn / safe_t, c)
    z = z0 + cot * s
    return phi, z, ok


def track_hits(kappa, phi0, d0=0.0, cot=0.0, z0=0.0, radii=DETECTOR_R_MM,
               b_tesla=B_TESLA, rng=None, drop_layers=(), sigma_rphi_mm=SIGMA_RPHI_MM):
    """Hits of tracks with the given true parameters (noiseless unless rng).

    Scalars or arrays of equal length.  Returns (layer u8, phi u32, z i32).
    """
    kappa, phi0, d0, cot, z0 = (np.atleast_1d(np.asarray(v, np.float64))
                                for v in (kappa, phi0, d0, cot, z0))
    n = max(len(kappa), len(phi0), len(d0), len(cot), len(z0))
    kappa, phi0, d0, cot, z0 = (np.broadcast_to(v, (n,)) for v in (kappa, phi0, d0, cot, z0))
    phi, z, ok = _helix_hits(kappa, phi0, d0, cot, z0, radii, b_tesla)
    radii = np.asarray(radii, np.float64)
    if rng is not None:
        phi = phi + rng.normal(0.0, 1.0, phi.shape) * (sigma_rphi_mm / radii[None, :])
        z = z + rng.normal(0.0, SIGMA_Z_MM, z.shape)
    ok = ok & (np.abs(z) < Z_ACCEPT_MM)
    for l in drop_layers:
        ok[:, l] = False
    layer = np.broadcast_to(np.arange(len(radii), dtype=np.uint8)[None, :], ok.shape)
    return (layer[ok].astype(np.uint8), _quantize_phi(phi[ok]),
            _quantize_z(z[ok]).astype(np.int32))


def _n_tracks(cfg, rng):
    kind = cfg["tracks"][0]
    if kind == "fixed":
        return int(cfg["tracks"][1])
    if kind == "lognormal":
        _, median, sigma, lo, hi = cfg["tracks"]
        v = np.exp(rng.normal(np.log(median), sigma))
        return int(np.clip(np.rint(v), lo, hi))
    if kind == "loguniform":
        _, lo, hi = cfg["tracks"]
        return int(np.clip(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi)))), lo, hi))
    raise ValueError(kind)


def gen_event(cfg, rng, n_tracks=None):
    """One event of workload `cfg` (a CONFIGS entry) from generator `rng`."""
    spec = cfg["spec"]
    radii = spec["layer_r_mm"][:spec["n_layers"]]
    if n_tracks is None:
        n_tracks = _n_tracks(cfg, rng)
    kappa = rng.uniform(-1.0, 1.0, n_tracks)
    phi0 = rng.uniform(0.0, TWO_PI, n_tracks)
    eta = rng.uniform(-1.0, 1.0, n_tracks)
    cot = np.sinh(eta)
    z0 = rng.normal(0.0, 50.0, n_tracks)
    d0 = np.zeros(n_tracks)
    frac = cfg.get("displaced_frac", 0.0)
    if frac > 0:
        n_disp = int(round(frac * n_tracks))
        lo, hi = cfg["d0_range_mm"]
        d0[:n_disp] = rng.uniform(lo, hi, n_disp)
    layer, phi, z = track_hits(kappa, phi0, d0, cot, z0, radii, spec["b_tesla"], rng=rng,
                               sigma_rphi_mm=cfg.get("sigma_rphi_mm", SIGMA_RPHI_MM))
    n_track_hits = len(layer)
    if "noise_per_track_hit" in cfg:
        n_noise = int(cfg["noise_per_track_hit"] * n_track_hits)
    else:
        n_noise = int(cfg["noise"])
    nl = rng.integers(0, spec["n_layers"], n_noise).astype(np.uint8)
    nphi = rng.integers(0, 1 << 32, n_noise, dtype=np.uint64).astype(np.uint32)
    nz = rng.integers(-Z_NOISE_UM, Z_NOISE_UM, n_noise).astype(np.int32)
    layer = np.concatenate([layer, nl])
    phi = np.concatenate([phi, nphi])
    z = np.concatenate([z, nz])
    perm = rng.permutation(len(layer))
    return layer[perm], phi[perm], z[perm], n_tracks


def concat_events(events, n_tracks=None):
    """Concatenate a list of (layer, phi, z[, ...]) tuples into an EventBatch."""
    sizes = np.array([len(e[0]) for e in events], dtype=np.uint64)
    offsets = np.zeros(len(events) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    if len(events):
        layer = np.concatenate([e[0] for e in events]).astype(np.uint8)
        phi = np.concatenate([e[1] for e in events]).astype(np.uint32)
        z = np.concatenate([e[2] for e in events]).astype(np.int32)
    else:
        layer = np.zeros(0, np.uint8); phi = np.zeros(0, np.uint32); z = np.zeros(0, np.int32)
    return EventBatch(layer, phi, z, offsets,
                      None if n_tracks is None else np.asarray(n_tracks))


def event_rng(cfg_index, event_index):
    """Per-event stream: root seed 0, spawn key (config, event)."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(0, spawn_key=(cfg_index, event_index))))


def aux_rng(cfg_index, which):
    """Auxiliary streams of a config (1: event sizes, 2: arrival times)."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(0, spawn_key=(cfg_index, 1_000_000 + which))))


def gen_batch(name, n_events=None, first_event=0):
    """Events [first_event, first_event + n_events) of workload `name`."""
    cfg = CONFIGS[name]
    if n_events is None:
        n_events = cfg["n_events"] or 1
    evs, ntr = [], []
    for e in range(first_event, first_event + n_events):
        rng = event_rng(cfg["index"], e)
        layer, phi, z, nt = gen_event(cfg, rng)
        evs.append((layer, phi, z))
        ntr.append(nt)
    return concat_events(evs, ntr)


def gen_config(name):
    """The full event set of a fixed-size workload (C1-C4)."""
    return gen_batch(name)


def arrival_times(name, rate_hz, n):
    """Poisson arrival times (seconds from 0) for the serving workload."""
    cfg = CONFIGS[name]
    rng = aux_rng(cfg["index"], 2 + int(rate_hz))
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))
