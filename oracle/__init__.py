"""CPU ORACLE for the Hough-transform tracker -- TEST INFRASTRUCTURE ONLY.

A numpy-facing wrapper over oracle.c (plain C, built with gcc -O2).  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product library and its Python binding never do.

Functions follow Section 4 of the paper (voting, then local maxima) and the
Discussion section's counting form; see oracle.c for the exact definitions
and the readings of points the paper leaves open.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build

_lib = None


class OrcSpec(C.Structure):
    _fields_ = [
        ("n_layers", C.c_uint32),
        ("layer_r_mm", C.c_double * 16),
        ("b_tesla", C.c_double),
        ("n_qpt", C.c_uint32),
        ("qpt_lo", C.c_double), ("qpt_hi", C.c_double),
        ("n_phi", C.c_uint32),
        ("n_d0", C.c_uint32),
        ("d0_lo_mm", C.c_double), ("d0_hi_mm", C.c_double),
        ("threshold", C.c_uint32),
        ("n_z0", C.c_uint32),
        ("z0_lo_um", C.c_int32), ("z0_hi_um", C.c_int32),
        ("n_cot", C.c_uint32),
        ("cot_lo", C.c_double), ("cot_hi", C.c_double),
        ("rz_max_candidates", C.c_uint32),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        P = C.c_void_p
        lib.orc_check_spec.argtypes = [P]
        lib.orc_check_spec.restype = C.c_int
        lib.orc_offsets.argtypes = [P, P, P]
        lib.orc_zshift.argtypes = [P, P]
        lib.orc_vote_mask.argtypes = [P, P, P, C.c_uint64, P, P, P]
        lib.orc_vote_count.argtypes = [P, P, P, C.c_uint64, P, P, P]
        lib.orc_peaks.argtypes = [P, P, P, P, P, C.c_uint64]
        lib.orc_peaks.restype = C.c_uint64
        lib.orc_peaks_count.argtypes = [P, P, P, P, C.c_uint64]
        lib.orc_peaks_count.restype = C.c_uint64
        lib.orc_rz_candidates.argtypes = [P, C.c_uint64, P, P]
        lib.orc_rz_candidates.restype = C.c_uint64
        lib.orc_rz.argtypes = [P, P, P, P, C.c_uint64, P, P, P, C.c_uint64, P, P,
                               P, P, P, P, P]
        lib.orc_rz.restype = C.c_uint64
        lib.orc_clusters.argtypes = [P, C.c_uint64, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_clusters.restype = C.c_uint64
        lib.orc_fit.argtypes = [P, P, P, C.c_uint64, P, P, P, C.c_uint64, P, P, P, P,
                                P, P, P, P, P, P, P, P, P, P, P]
        _lib = lib
    return _lib


def make_spec(d):
    s = OrcSpec()
    for name, _ in OrcSpec._fields_:
        if name == "layer_r_mm":
            arr = (C.c_double * 16)()
            for i, v in enumerate(d["layer_r_mm"][:16]):
                arr[i] = v
            s.layer_r_mm = arr
        else:
            setattr(s, name, d[name])
    return s


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def check_spec(spec):
    s = make_spec(spec)
    return _load().orc_check_spec(C.byref(s)) == 0


class Tables:
    """The oracle's own offset (O, V) and z-shift (Z) tables."""

    def __init__(self, spec):
        lib = _load()
        self.spec = dict(spec)
        self.cs = make_spec(spec)
        if lib.orc_check_spec(C.byref(self.cs)) != 0:
            raise ValueError("invalid grid spec")
        L, D, K = spec["n_layers"], spec["n_d0"], spec["n_qpt"]
        self.O = np.zeros(L * D * K, np.uint32)
        self.V = np.zeros(L * D * K, np.uint8)
        lib.orc_offsets(C.byref(self.cs), _p(self.O), _p(self.V))
        self.O = self.O.reshape(L, D, K)
        self.V = self.V.reshape(L, D, K)
        if spec["n_z0"]:
            self.Z = np.zeros(K * L * spec["n_cot"], np.int32)
            lib.orc_zshift(C.byref(self.cs), _p(self.Z))
            self.Z = self.Z.reshape(K, L, spec["n_cot"])
        else:
            self.Z = np.zeros((K, L, 0), np.int32)

    @property
    def cells(self):
        s = self.spec
        return s["n_d0"] * s["n_qpt"] * s["n_phi"]


def _hits(layer, phi, z=None):
    layer = np.ascontiguousarray(layer, np.uint8)
    phi = np.ascontiguousarray(phi, np.uint32)
    z = None if z is None else np.ascontiguousarray(z, np.int32)
    return layer, phi, z


def vote_mask(tab, layer, phi):
    """Layer-bitmask accumulator A[d][k][p] (uint16) of one event."""
    layer, phi, _ = _hits(layer, phi)
    s = tab.spec
    A = np.zeros(tab.cells, np.uint16)
    _load().orc_vote_mask(C.byref(tab.cs), _p(tab.O), _p(tab.V), len(layer),
                          _p(layer), _p(phi), _p(A))
    return A.reshape(s["n_d0"], s["n_qpt"], s["n_phi"])


def vote_count(tab, layer, phi):
    """The counting accumulator C[d][k][p] (uint32) of one event."""
    layer, phi, _ = _hits(layer, phi)
    s = tab.spec
    Cc = np.zeros(tab.cells, np.uint32)
    _load().orc_vote_count(C.byref(tab.cs), _p(tab.O), _p(tab.V), len(layer),
                           _p(layer), _p(phi), _p(Cc))
    return Cc.reshape(s["n_d0"], s["n_qpt"], s["n_phi"])


PEAK_DTYPE = np.dtype([("cell", np.uint32), ("mask", np.uint16), ("popcount", np.uint16)])
RZ_DTYPE = np.dtype([("peak", np.uint32), ("cot_bin", np.uint16), ("z0_bin", np.uint16),
                     ("count", np.uint32), ("n_members", np.uint32)])


def peaks(tab, A):
    """Local maxima of one event's accumulator, ascending by cell."""
    A = np.ascontiguousarray(A, np.uint16).reshape(-1)
    cap = A.size
    cell = np.zeros(cap, np.uint32)
    mask = np.zeros(cap, np.uint16)
    pc = np.zeros(cap, np.uint16)
    n = _load().orc_peaks(C.byref(tab.cs), _p(A), _p(cell), _p(mask), _p(pc), cap)
    out = np.zeros(n, PEAK_DTYPE)
    out["cell"], out["mask"], out["popcount"] = cell[:n], mask[:n], pc[:n]
    return out


COUNT_PEAK_DTYPE = np.dtype([("cell", np.uint32), ("count", np.uint32)])


def peaks_count(tab, Cc):
    """Local maxima of one event's counting accumulator, ascending by cell."""
    Cc = np.ascontiguousarray(Cc, np.uint32).reshape(-1)
    cap = Cc.size
    cell = np.zeros(cap, np.uint32)
    cnt = np.zeros(cap, np.uint32)
    n = _load().orc_peaks_count(C.byref(tab.cs), _p(Cc), _p(cell), _p(cnt), cap)
    out = np.zeros(n, COUNT_PEAK_DTYPE)
    out["cell"], out["count"] = cell[:n], cnt[:n]
    return out


def rz_candidates(tab, pk):
    pc = np.ascontiguousarray(pk["popcount"], np.uint16)
    cand = np.zeros(len(pc) + 1, np.uint32)
    n = _load().orc_rz_candidates(C.byref(tab.cs), len(pc), _p(pc), _p(cand))
    return cand[:n]


def rz(tab, layer, phi, z, pk):
    """rz refinement records of one event, in candidate order."""
    layer, phi, z = _hits(layer, phi, z)
    cell = np.ascontiguousarray(pk["cell"], np.uint32)
    pc = np.ascontiguousarray(pk["popcount"], np.uint16)
    n = len(cell)
    op = np.zeros(n + 1, np.uint32); oc = np.zeros(n + 1, np.uint16)
    oz = np.zeros(n + 1, np.uint16); on = np.zeros(n + 1, np.uint32)
    om = np.zeros(n + 1, np.uint32)
    m = _load().orc_rz(C.byref(tab.cs), _p(tab.O), _p(tab.V), _p(tab.Z), len(layer),
                       _p(layer), _p(phi), _p(z), n, _p(cell), _p(pc),
                       _p(op), _p(oc), _p(oz), _p(on), _p(om))
    out = np.zeros(m, RZ_DTYPE)
    out["peak"], out["cot_bin"], out["z0_bin"] = op[:m], oc[:m], oz[:m]
    out["count"], out["n_members"] = on[:m], om[:m]
    return out


CLUSTER_DTYPE = np.dtype([("first", np.uint32), ("n_peaks", np.uint32), ("sum_dd", np.int32),
                          ("sum_dk", np.int32), ("sum_dp", np.int32), ("popcount", np.uint16),
                          ("mask_or", np.uint16)])


def clusters(tab, pk):
    """Plateau clusters of one event's peak list (connected components of
    adjacent peak cells, phi0 periodic): (label per peak, cluster records in
    the order of their first peak)."""
    cell = np.ascontiguousarray(pk["cell"], np.uint32)
    mask = np.ascontiguousarray(pk["mask"], np.uint16)
    pc = np.ascontiguousarray(pk["popcount"], np.uint16)
    n = len(cell)
    label = np.zeros(n + 1, np.uint32)
    a = [np.zeros(n + 1, t) for t in (np.uint32, np.uint32, np.int32, np.int32, np.int32,
                                      np.uint16, np.uint16)]
    m = _load().orc_clusters(C.byref(tab.cs), n, _p(cell), _p(mask), _p(pc), _p(label),
                             *[_p(x) for x in a])
    out = np.zeros(m, CLUSTER_DTYPE)
    for name, x in zip(CLUSTER_DTYPE.names, a):
        out[name] = x[:m]
    return label[:n], out


def cluster_centroids(tab, pk, cl):
    """Centroid bin coordinates (d, k, p) of each cluster, fp64, p in
    [0, n_phi): the first peak's bin plus the mean member offset."""
    s = tab.spec
    np_, nk = s["n_phi"], s["n_qpt"]
    f = pk["cell"][cl["first"]].astype(np.int64)
    n = cl["n_peaks"].astype(np.float64)
    d = f // (np_ * nk) + cl["sum_dd"] / n
    k = (f // np_) % nk + cl["sum_dk"] / n
    p = np.mod(f % np_ + cl["sum_dp"] / n, np_)
    return d, k, p


FIT_DTYPE = np.dtype([("qpt", np.float64), ("phi0", np.float64), ("qpt_c", np.float64),
                      ("phi0_c", np.float64), ("rms_mm", np.float64), ("cot", np.float64),
                      ("z0_mm", np.float64), ("rms_z_mm", np.float64), ("n_hits", np.uint32),
                      ("status", np.uint32), ("status_z", np.uint32)])


def fit(tab, layer, phi, pk, cl, z=None):
    """Helix fit of each cluster of one event over the hits that voted into
    its first peak cell (beam-line grids only): the transverse circle, and,
    when z is given, the line z = z0 + cot s; plus the centroid parameters.
    FIT_DTYPE records in cluster order."""
    if tab.spec["n_d0"] != 1:
        raise ValueError("the cluster fit needs a grid without a d0 axis")
    layer, phi, z = _hits(layer, phi, z)
    n = len(cl)
    first = np.ascontiguousarray(pk["cell"][cl["first"]], np.uint32)
    npk = np.ascontiguousarray(cl["n_peaks"], np.uint32)
    sdk = np.ascontiguousarray(cl["sum_dk"], np.int32)
    sdp = np.ascontiguousarray(cl["sum_dp"], np.int32)
    d = [np.zeros(n + 1) for _ in range(8)]
    u = [np.zeros(n + 1, np.uint32) for _ in range(3)]
    _load().orc_fit(C.byref(tab.cs), _p(tab.O), _p(tab.V), len(layer), _p(layer), _p(phi),
                    None if z is None else _p(z), n,
                    _p(first), _p(npk), _p(sdk), _p(sdp), *[_p(x) for x in d[:5]], *[_p(x) for x in d[5:]],
                    *[_p(x) for x in u])
    out = np.zeros(n, FIT_DTYPE)
    for name, x in zip(FIT_DTYPE.names, d + u):
        out[name] = x[:n]
    return out


def run_event(tab, layer, phi, z=None, with_rz=None):
    """Full oracle pass over one event: accumulator, peaks and (if the grid
    has an rz stage) rz records."""
    A = vote_mask(tab, layer, phi)
    pk = peaks(tab, A)
    if with_rz is None:
        with_rz = bool(tab.spec["n_z0"])
    r = rz(tab, layer, phi, z, pk) if with_rz else None
    return A, pk, r
