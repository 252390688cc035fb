"""Python binding of libhough.so: argument marshalling only.

Every step of the track finder runs in the library's HIP kernels; this module
allocates device buffers as torch tensors, passes their addresses and the
current HIP stream through ctypes, and converts results to numpy on request.
It never computes a vote, a peak or an rz result itself, and it raises if the
compiled library is missing: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhough.so")

HOUGH_OK, HOUGH_EINVAL, HOUGH_ENOMEM, HOUGH_EDEVICE, HOUGH_ECAPACITY, HOUGH_ELIMIT = 0, -1, -2, -3, -4, -5

EXPORTED = [
    "hough_create", "hough_destroy", "hough_vote", "hough_peaks", "hough_rz_refine",
    "hough_graph_capture", "hough_graph_launch", "hough_graph_destroy",
    "hough_check_spec", "hough_build_tables", "hough_set_tuning", "hough_get_tuning",
    "hough_set_profiling", "hough_kernel_times", "hough_kernel_times_reset",
    "hough_strerror", "hough_last_error", "hough_device_cus", "hough_gather_events",
    "hough_vote_count", "hough_peaks_count", "hough_peak_clusters",
    "hough_cluster_fit", "hough_get_tables", "hough_peaks_noalloc",
]

PEAK_DTYPE = np.dtype([("cell", np.uint32), ("mask", np.uint16), ("popcount", np.uint16)])
COUNT_PEAK_DTYPE = np.dtype([("cell", np.uint32), ("count", np.uint32)])
RZ_DTYPE = np.dtype([("peak", np.uint32), ("cot_bin", np.uint16), ("z0_bin", np.uint16),
                     ("count", np.uint32), ("n_members", np.uint32)])
CLUSTER_DTYPE = np.dtype([("first", np.uint32), ("popcount", np.uint16), ("mask_or", np.uint16),
                          ("n_peaks", np.uint32), ("sum_dk", np.int32), ("sum_dp", np.int32),
                          ("sum_dd", np.int32)])
FIT_DTYPE = np.dtype([("qpt", np.float64), ("phi0", np.float64), ("qpt_c", np.float64),
                      ("phi0_c", np.float64), ("rms_mm", np.float64), ("cot", np.float64),
                      ("z0_mm", np.float64), ("rms_z_mm", np.float64), ("n_hits", np.uint32),
                      ("status", np.uint32), ("status_z", np.uint32), ("reserved", np.uint32)])


class GridSpec(C.Structure):
    _fields_ = [
        ("n_layers", C.c_uint32), ("layer_r_mm", C.c_double * 16), ("b_tesla", C.c_double),
        ("n_qpt", C.c_uint32), ("qpt_lo", C.c_double), ("qpt_hi", C.c_double),
        ("n_phi", C.c_uint32),
        ("n_d0", C.c_uint32), ("d0_lo_mm", C.c_double), ("d0_hi_mm", C.c_double),
        ("threshold", C.c_uint32),
        ("n_z0", C.c_uint32), ("z0_lo_um", C.c_int32), ("z0_hi_um", C.c_int32),
        ("n_cot", C.c_uint32), ("cot_lo", C.c_double), ("cot_hi", C.c_double),
        ("rz_max_candidates", C.c_uint32),
    ]


class Limits(C.Structure):
    _fields_ = [("max_events", C.c_uint32), ("max_hits", C.c_uint64), ("max_peaks", C.c_uint64)]


class Hits(C.Structure):
    _fields_ = [("layer", C.c_void_p), ("phi", C.c_void_p), ("z_um", C.c_void_p),
                ("event_offsets", C.c_void_p), ("n_events", C.c_uint32), ("n_hits", C.c_uint64)]


class Tuning(C.Structure):
    _fields_ = [("vote_rows", C.c_uint32), ("vote_threads", C.c_uint32),
                ("vote_wgs_per_cu", C.c_uint32), ("peak_rows", C.c_uint32),
                ("rz_waves_per_cu", C.c_uint32), ("vote_algo", C.c_uint32),
                ("rz_slow_path", C.c_uint32), ("rz_counter_bits", C.c_uint32),
                ("vote_items", C.c_uint32), ("peak_algo", C.c_uint32), ("rz_member_cap", C.c_uint32),
                ("rz_redo_list", C.c_uint32)]


_lib = None


def load_library():
    """Load libhough.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1310_7556_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sig = {
        "hough_create": ([P, P, i32, P], i32),
        "hough_destroy": ([P], None),
        "hough_vote": ([P, P, P, P], i32),
        "hough_peaks": ([P, P, u32, P, u64, P, P], i32),
        "hough_peaks_noalloc": ([P, P, u32, P, u64, P, P], i32),
        "hough_rz_refine": ([P, P, P, u64, P, P, u64, P, P], i32),
        "hough_graph_capture": ([P, P, P, P, u64, P, P, u64, P, P, P], i32),
        "hough_graph_launch": ([P, P], i32),
        "hough_graph_destroy": ([P], None),
        "hough_check_spec": ([P], i32),
        "hough_build_tables": ([P, P, P, C.c_size_t, P, C.c_size_t], i32),
        "hough_set_tuning": ([P, P], i32),
        "hough_get_tuning": ([P, P], i32),
        "hough_set_profiling": ([P, i32], i32),
        "hough_kernel_times": ([P, P, P, P, i32], i32),
        "hough_kernel_times_reset": ([P], None),
        "hough_strerror": ([i32], C.c_char_p),
        "hough_last_error": ([P], C.c_char_p),
        "hough_device_cus": ([P], i32),
        "hough_gather_events": ([P, P, P, P, P, P, u32, P, P, P, u64, P], i32),
        "hough_get_tables": ([P, P, P, C.c_size_t, P, C.c_size_t, P, C.c_size_t], i32),
        "hough_vote_count": ([P, P, P, P], i32),
        "hough_peaks_count": ([P, P, u32, P, u64, P, P], i32),
        "hough_peak_clusters": ([P, P, u64, P, u32, P, P, u64, P, P], i32),
        "hough_cluster_fit": ([P, P, P, u64, P, P, u64, P, P, P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class HoughError(RuntimeError):
    pass


def _check(rc, ctx=None, what=""):
    if rc != HOUGH_OK:
        lib = load_library()
        msg = lib.hough_strerror(rc).decode()
        if ctx is not None:
            detail = lib.hough_last_error(ctx).decode()
            if detail:
                msg += f" ({detail})"
        raise HoughError(f"{what}: {msg} [{rc}]")


def make_spec(d):
    s = GridSpec()
    for name, _ in GridSpec._fields_:
        if name == "layer_r_mm":
            arr = (C.c_double * 16)()
            for i, v in enumerate(list(d["layer_r_mm"])[:16]):
                arr[i] = float(v)
            s.layer_r_mm = arr
        else:
            setattr(s, name, d[name])
    return s


def check_spec(spec):
    return load_library().hough_check_spec(C.byref(make_spec(spec))) == HOUGH_OK


def build_tables(spec):
    """The library's host tables (O, V as [L, D, K]; Z as [K, L, C])."""
    lib = load_library()
    s = make_spec(spec)
    L, D, K = spec["n_layers"], spec["n_d0"], spec["n_qpt"]
    O = np.zeros(L * D * K, np.uint32)
    V = np.zeros(L * D * K, np.uint8)
    nz = K * L * spec["n_cot"] if spec["n_z0"] else 0
    Z = np.zeros(max(nz, 1), np.int32)
    rc = lib.hough_build_tables(C.byref(s), O.ctypes.data, V.ctypes.data, O.size,
                                Z.ctypes.data if nz else None, nz)
    _check(rc, what="hough_build_tables")
    return O.reshape(L, D, K), V.reshape(L, D, K), Z[:nz].reshape(K, L, spec["n_cot"] if nz else 0)


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class DeviceHits:
    """Structure-of-arrays hits of one or more events on the GPU."""

    def __init__(self, layer, phi, z, offsets, device="cuda"):
        torch = _torch()

        def to_dev(a, np_dtype, view_dtype):
            if isinstance(a, torch.Tensor):
                return a.to(device=device).contiguous()
            a = np.ascontiguousarray(a, dtype=np_dtype).view(view_dtype)
            return torch.from_numpy(a).to(device)

        self.layer = to_dev(layer, np.uint8, np.uint8)
        self.phi = to_dev(phi, np.uint32, np.int32)
        self.z = None if z is None else to_dev(z, np.int32, np.int32)
        off = offsets if isinstance(offsets, torch.Tensor) else np.asarray(offsets, np.uint64)
        self.offsets = to_dev(off, np.uint64, np.int64)
        if isinstance(offsets, torch.Tensor):
            host_off = offsets.cpu().numpy()
        else:
            host_off = np.asarray(offsets, np.uint64)
        self.n_events = len(host_off) - 1
        self.n_hits = int(self.layer.numel())

    @classmethod
    def from_batch(cls, batch, device="cuda"):
        return cls(batch.layer, batch.phi, batch.z, batch.offsets, device)

    def struct(self):
        h = Hits()
        h.layer = self.layer.data_ptr() if self.n_hits else None
        h.phi = self.phi.data_ptr() if self.n_hits else None
        h.z_um = self.z.data_ptr() if (self.z is not None and self.n_hits) else None
        h.event_offsets = self.offsets.data_ptr()
        h.n_events = self.n_events
        h.n_hits = self.n_hits
        return h


class HoughGraph:
    def __init__(self, ctx, handle, keep):
        self._ctx = ctx
        self._h = handle
        self._keep = keep

    def launch(self, stream=None):
        _check(self._ctx.lib.hough_graph_launch(self._h, _stream(stream)), self._ctx._h, "hough_graph_launch")

    def close(self):
        if self._h:
            self._ctx.lib.hough_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HoughContext:
    """A library context: tables and scratch for one grid spec on one GPU."""

    def __init__(self, spec, max_events=1, max_hits=1 << 20, max_peaks=0, device=0):
        self.lib = load_library()
        self.spec = dict(spec)
        self._spec = make_spec(spec)
        self.limits = Limits(max_events, max_hits, max_peaks)
        self.device = device
        h = C.c_void_p()
        _check(self.lib.hough_create(C.byref(self._spec), C.byref(self.limits), device, C.byref(h)),
               what="hough_create")
        self._h = h
        self.cells = spec["n_d0"] * spec["n_qpt"] * spec["n_phi"]

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hough_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers -------------------------------------------------------
    def new_acc(self, n_events):
        torch = _torch()
        return torch.empty((n_events, self.spec["n_d0"], self.spec["n_qpt"], self.spec["n_phi"]),
                           dtype=torch.int16, device=f"cuda:{self.device}")

    def new_peaks(self, capacity):
        torch = _torch()
        return torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=f"cuda:{self.device}")

    def new_offsets(self, n_events):
        torch = _torch()
        return torch.empty(n_events + 1, dtype=torch.int64, device=f"cuda:{self.device}")

    def new_rz(self, capacity):
        torch = _torch()
        return torch.empty((max(capacity, 1), 4), dtype=torch.int32, device=f"cuda:{self.device}")

    # ---- hot path ------------------------------------------------------
    def vote(self, hits, acc=None, stream=None):
        if acc is None:
            acc = self.new_acc(hits.n_events)
        h = hits.struct()
        _check(self.lib.hough_vote(self._h, C.byref(h), _ptr(acc), _stream(stream)), self._h, "hough_vote")
        return acc

    def peaks(self, acc, n_events, capacity=None, peaks=None, offsets=None, stream=None):
        if capacity is None:
            capacity = n_events * self.cells
        if peaks is None:
            peaks = self.new_peaks(capacity)
        if offsets is None:
            offsets = self.new_offsets(n_events)
        _check(self.lib.hough_peaks(self._h, _ptr(acc), n_events, _ptr(peaks), capacity, _ptr(offsets),
                                    _stream(stream)), self._h, "hough_peaks")
        return peaks, offsets

    def new_counts(self, n_events):
        """Counting accumulator: int32 tensor holding uint32 counts."""
        torch = _torch()
        return torch.empty((n_events, self.spec["n_d0"], self.spec["n_qpt"], self.spec["n_phi"]),
                           dtype=torch.int32, device=f"cuda:{self.device}")

    def vote_count(self, hits, counts=None, stream=None):
        if counts is None:
            counts = self.new_counts(hits.n_events)
        h = hits.struct()
        _check(self.lib.hough_vote_count(self._h, C.byref(h), _ptr(counts), _stream(stream)), self._h,
               "hough_vote_count")
        return counts

    def peaks_count(self, counts, n_events, capacity=None, peaks=None, offsets=None, stream=None):
        if capacity is None:
            capacity = n_events * self.cells
        if peaks is None:
            peaks = self.new_peaks(capacity)
        if offsets is None:
            offsets = self.new_offsets(n_events)
        _check(self.lib.hough_peaks_count(self._h, _ptr(counts), n_events, _ptr(peaks), capacity,
                                          _ptr(offsets), _stream(stream)), self._h, "hough_peaks_count")
        return peaks, offsets

    def rz_refine(self, hits, peaks, peak_offsets, peak_capacity=None, capacity=None, out=None,
                  offsets=None, stream=None):
        if peak_capacity is None:
            peak_capacity = peaks.shape[0]
        if capacity is None:
            capacity = peak_capacity
        if out is None:
            out = self.new_rz(capacity)
        if offsets is None:
            offsets = self.new_offsets(hits.n_events)
        h = hits.struct()
        _check(self.lib.hough_rz_refine(self._h, C.byref(h), _ptr(peaks), peak_capacity, _ptr(peak_offsets),
                                        _ptr(out), capacity, _ptr(offsets), _stream(stream)),
               self._h, "hough_rz_refine")
        return out, offsets

    def new_clusters(self, capacity):
        """Cluster records: int64 tensor (8-byte aligned) of 3 words each."""
        torch = _torch()
        return torch.empty((max(capacity, 1), 3), dtype=torch.int64, device=f"cuda:{self.device}")

    def new_labels(self, capacity):
        torch = _torch()
        return torch.empty(max(capacity, 1), dtype=torch.int32, device=f"cuda:{self.device}")

    def peak_clusters(self, peaks, peak_offsets, n_events, peak_capacity=None, capacity=None, labels=None,
                      out=None, offsets=None, stream=None):
        """Plateau clusters of a peak list: (per-peak cluster index within its
        event, cluster records, event cluster offsets)."""
        if peak_capacity is None:
            peak_capacity = peaks.shape[0]
        if capacity is None:
            capacity = peak_capacity
        if labels is None:
            labels = self.new_labels(peak_capacity)
        if out is None:
            out = self.new_clusters(capacity)
        if offsets is None:
            offsets = self.new_offsets(n_events)
        _check(self.lib.hough_peak_clusters(self._h, _ptr(peaks), peak_capacity, _ptr(peak_offsets), n_events,
                                            _ptr(labels), _ptr(out), capacity, _ptr(offsets), _stream(stream)),
               self._h, "hough_peak_clusters")
        return labels, out, offsets

    def new_fits(self, capacity):
        """Fit records: float64 tensor of 10 words (80 bytes) each."""
        torch = _torch()
        return torch.empty((max(capacity, 1), 10), dtype=torch.float64, device=f"cuda:{self.device}")

    def cluster_fit(self, hits, peaks, peak_offsets, clusters, cluster_offsets, peak_capacity=None,
                    capacity=None, out=None, stream=None):
        """Helix fit of every stored cluster (grids without a d0 axis)."""
        if peak_capacity is None:
            peak_capacity = peaks.shape[0]
        if capacity is None:
            capacity = clusters.shape[0]
        if out is None:
            out = self.new_fits(capacity)
        h = hits.struct()
        _check(self.lib.hough_cluster_fit(self._h, C.byref(h), _ptr(peaks), peak_capacity, _ptr(peak_offsets),
                                          _ptr(clusters), capacity, _ptr(cluster_offsets), _ptr(out),
                                          _stream(stream)), self._h, "hough_cluster_fit")
        return out

    def graph_capture(self, hits, acc, peaks, peak_capacity, peak_offsets, rz=None, rz_capacity=0,
                      rz_offsets=None, stream=None):
        h = hits.struct()
        g = C.c_void_p()
        _check(self.lib.hough_graph_capture(self._h, C.byref(h), _ptr(acc), _ptr(peaks), peak_capacity,
                                            _ptr(peak_offsets), _ptr(rz), rz_capacity, _ptr(rz_offsets),
                                            _stream(stream), C.byref(g)), self._h, "hough_graph_capture")
        return HoughGraph(self, g, (hits, acc, peaks, peak_offsets, rz, rz_offsets))

    def get_tables(self, zl=False):
        """The tables this context uploaded, read back from the device: O, V
        as [L, D, K]; Z as [K, L, C] (empty without an rz stage); with zl,
        also Z + z0_lo as the rz kernel reads it."""
        s = self.spec
        L, D, K = s["n_layers"], s["n_d0"], s["n_qpt"]
        nz = K * L * s["n_cot"] if s["n_z0"] else 0
        O = np.zeros(L * D * K, np.uint32)
        V = np.zeros(L * D * K, np.uint8)
        Z = np.zeros(max(nz, 1), np.int32)
        Zl = np.zeros(max(nz, 1), np.int32) if zl else None
        rc = self.lib.hough_get_tables(self._h, O.ctypes.data, V.ctypes.data, O.size,
                                       Z.ctypes.data if nz else None, nz,
                                       Zl.ctypes.data if zl else None, nz if zl else 0)
        _check(rc, self._h, "hough_get_tables")
        C_ = s["n_cot"] if nz else 0
        out = (O.reshape(L, D, K), V.reshape(L, D, K), Z[:nz].reshape(K, L, C_))
        return out + (Zl[:nz].reshape(K, L, C_),) if zl else out

    # ---- tuning and timing --------------------------------------------
    def set_tuning(self, **kw):
        t = Tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(self.lib.hough_set_tuning(self._h, C.byref(t)), self._h, "hough_set_tuning")

    def get_tuning(self):
        t = Tuning()
        _check(self.lib.hough_get_tuning(self._h, C.byref(t)), self._h, "hough_get_tuning")
        return {name: getattr(t, name) for name, _ in Tuning._fields_}

    def set_profiling(self, enable=True):
        _check(self.lib.hough_set_profiling(self._h, int(enable)), self._h, "hough_set_profiling")

    def kernel_times(self):
        n = 64
        names = (C.c_char_p * n)()
        launches = (C.c_uint64 * n)()
        ms = (C.c_double * n)()
        m = self.lib.hough_kernel_times(self._h, names, launches, ms, n)
        return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(min(m, n))}

    def kernel_times_reset(self):
        self.lib.hough_kernel_times_reset(self._h)

    @property
    def n_cu(self):
        return self.lib.hough_device_cus(self._h)


def gather_events(src, src_off, lens, dst_off, n, dst_layer, dst_phi, dst_z, stream=None):
    """Assemble n events of `src` (DeviceHits) into contiguous destination
    arrays (device tensors); src_off/lens/dst_off are device int64 tensors.
    Nothing is written past the destination tensors' length."""
    lib = load_library()
    cap = int(min(dst_layer.numel(), dst_phi.numel(), dst_z.numel() if dst_z is not None else 1 << 62))
    rc = lib.hough_gather_events(_ptr(src.layer), _ptr(src.phi), _ptr(src.z) if dst_z is not None else None,
                                 _ptr(src_off), _ptr(lens), _ptr(dst_off), n, _ptr(dst_layer),
                                 _ptr(dst_phi), _ptr(dst_z), cap, _stream(stream))
    _check(rc, what="hough_gather_events")


# ---- numpy views of device results ----------------------------------------

def acc_numpy(acc):
    return acc.cpu().numpy().view(np.uint16)


def offsets_numpy(off):
    return off.cpu().numpy().view(np.uint64)


def peaks_numpy(peaks, offsets, event=None):
    """Peak records (all events, or one) as a PEAK_DTYPE array."""
    off = offsets_numpy(offsets)
    n = int(off[-1])
    cap = peaks.shape[0]
    arr = peaks[:min(n, cap)].cpu().numpy().view(PEAK_DTYPE).reshape(-1)
    if event is None:
        return arr
    return arr[int(off[event]):int(off[event + 1])]


def counts_numpy(counts):
    return counts.cpu().numpy().view(np.uint32)


def count_peaks_numpy(peaks, offsets, event=None):
    """Count-peak records (all events, or one) as a COUNT_PEAK_DTYPE array."""
    off = offsets_numpy(offsets)
    n = int(off[-1])
    arr = peaks[:min(n, peaks.shape[0])].cpu().numpy().view(COUNT_PEAK_DTYPE).reshape(-1)
    if event is None:
        return arr
    return arr[int(off[event]):int(off[event + 1])]


def rz_numpy(rz, offsets, event=None):
    off = offsets_numpy(offsets)
    n = int(off[-1])
    arr = rz[:min(n, rz.shape[0])].cpu().numpy().view(RZ_DTYPE).reshape(-1)
    if event is None:
        return arr
    return arr[int(off[event]):int(off[event + 1])]


def clusters_numpy(clusters, offsets, event=None):
    """Cluster records (all events, or one) as a CLUSTER_DTYPE array."""
    off = offsets_numpy(offsets)
    n = int(off[-1])
    arr = clusters[:min(n, clusters.shape[0])].cpu().numpy().view(CLUSTER_DTYPE).reshape(-1)
    if event is None:
        return arr
    return arr[int(off[event]):int(off[event + 1])]


def labels_numpy(labels, peak_offsets, peak_capacity=None, event=None):
    """Per-peak cluster indices (all stored peaks, or one event's)."""
    off = offsets_numpy(peak_offsets)
    cap = labels.shape[0] if peak_capacity is None else peak_capacity
    arr = labels[:min(int(off[-1]), cap)].cpu().numpy().view(np.uint32)
    if event is None:
        return arr
    return arr[min(int(off[event]), cap):min(int(off[event + 1]), cap)]


def fits_numpy(fits, cluster_offsets, event=None):
    """Fit records (all stored clusters, or one event's) as a FIT_DTYPE array."""
    off = offsets_numpy(cluster_offsets)
    n = int(off[-1])
    arr = fits[:min(n, fits.shape[0])].cpu().numpy().view(FIT_DTYPE).reshape(-1)
    if event is None:
        return arr
    return arr[int(off[event]):int(off[event + 1])]
