"""ctypes binding of libsvt.so (declared in include/svt.h).

Argument marshalling only: every step of the fit runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  Importing this module
loads the library and raises if it has not been built -- there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsvt.so")

SVT_OK, SVT_E_INVAL, SVT_E_RANGE, SVT_E_NOMEM, SVT_E_STATE, SVT_E_AGAIN, SVT_E_DEVICE = \
    0, -1, -2, -3, -4, -5, -6
SVT_MEM_PAGEABLE, SVT_MEM_PINNED, SVT_MEM_MAPPED, SVT_MEM_DEVICE = 0, 1, 2, 3

P = ctypes.c_void_p


class svt_event_batch(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("n_roads", ctypes.c_int32),
                ("n_hits", ctypes.c_int32), ("mem_kind", ctypes.c_int32),
                ("road_offsets", P), ("sector", P), ("nhits", P), ("hit_offsets", P),
                ("hits", P), ("xft", P)]


class svt_results(ctypes.Structure):
    _fields_ = [("ncomb", P), ("npass", P), ("best", P), ("chi2", P), ("params", P),
                ("hit_index", P), ("ntracks", P), ("comb_offsets", P),
                ("mem_kind", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class svt_summary(ctypes.Structure):
    _fields_ = [("total_comb", ctypes.c_int64), ("total_pass", ctypes.c_int64),
                ("total_tracks", ctypes.c_int32), ("err_road", ctypes.c_int32),
                ("err_event", ctypes.c_int32), ("status", ctypes.c_int32),
                ("device_ns", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class svt_tuning(ctypes.Structure):
    _fields_ = [("events_per_chunk", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("kernel", ctypes.c_int32)]


class svt_device_info(ctypes.Structure):
    _fields_ = [("compute_units", ctypes.c_int32), ("clock_khz", ctypes.c_int32),
                ("hbm_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64),
                ("used_bytes", ctypes.c_int64), ("arch", ctypes.c_char * 32)]


class svt_shadow_tracks(ctypes.Structure):
    _fields_ = [("n_tracks", ctypes.c_int32), ("n_sectors", ctypes.c_int32),
                ("x", P), ("tau", P), ("sector_offsets", P),
                ("w", ctypes.c_float * 3), ("pad_", ctypes.c_int32)]


class svt_pass_list(ctypes.Structure):
    _fields_ = [("offsets", P), ("k", P), ("chi2", P), ("params", P), ("capacity", ctypes.c_int64)]


class svt_unpack_out(ctypes.Structure):
    _fields_ = [("road_offsets", P), ("sector", P), ("nhits", P), ("hit_offsets", P), ("hits", P),
                ("xft", P), ("max_events", ctypes.c_int32), ("max_roads", ctypes.c_int32),
                ("max_hits", ctypes.c_int32), ("pad_", ctypes.c_int32)]


# (name, restype, argtypes) of every exported entry point
SIGNATURES = {
    "svt_create": (ctypes.c_int32, [ctypes.POINTER(P), ctypes.c_int32, ctypes.c_size_t]),
    "svt_destroy": (ctypes.c_int32, [P]),
    "svt_load_constants": (ctypes.c_int32, [P, ctypes.c_int32, P, P, ctypes.c_uint64]),
    "svt_fit_events": (ctypes.c_int32, [P, ctypes.POINTER(svt_event_batch),
                                        ctypes.POINTER(svt_results), P,
                                        ctypes.POINTER(ctypes.c_int64)]),
    "svt_result": (ctypes.c_int32, [P, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.POINTER(svt_summary)]),
    "svt_list_passing": (ctypes.c_int32, [P, ctypes.POINTER(svt_event_batch), P,
                                          ctypes.POINTER(svt_pass_list), P,
                                          ctypes.POINTER(ctypes.c_int64)]),
    "svt_list_passing_noalloc": (ctypes.c_int32, [P, ctypes.POINTER(svt_event_batch), P,
                                                  ctypes.POINTER(svt_pass_list), P,
                                                  ctypes.POINTER(ctypes.c_int64)]),
    "svt_unpack_stream": (ctypes.c_int32, [P, P, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.POINTER(svt_unpack_out), P,
                                           ctypes.POINTER(ctypes.c_int64)]),
    "svt_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "svt_last_error": (ctypes.c_char_p, []),
    "svt_set_tuning": (ctypes.c_int32, [P, ctypes.POINTER(svt_tuning)]),
    "svt_get_tuning": (ctypes.c_int32, [P, ctypes.POINTER(svt_tuning)]),
    "svt_set_timing": (ctypes.c_int32, [P, ctypes.c_int32]),
    "svt_get_device_info": (ctypes.c_int32, [P, ctypes.POINTER(svt_device_info)]),
    "svt_io_probe": (ctypes.c_int32, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_size_t,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "svt_plan_create": (ctypes.c_int32, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         P, ctypes.POINTER(P)]),
    "svt_plan_destroy": (ctypes.c_int32, [P]),
    "svt_plan_buffers": (ctypes.c_int32, [P, ctypes.POINTER(svt_event_batch),
                                          ctypes.POINTER(svt_results)]),
    "svt_plan_fit": (ctypes.c_int32, [P, ctypes.POINTER(svt_event_batch),
                                      ctypes.POINTER(svt_results), P,
                                      ctypes.POINTER(ctypes.c_int64)]),
    "svt_ring_info": (ctypes.c_int32, [P, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "svt_ring_create": (ctypes.c_int32, [P, ctypes.c_int32, ctypes.POINTER(svt_event_batch),
                                         ctypes.POINTER(svt_results), ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(P)]),
    "svt_ring_run": (ctypes.c_int32, [P, P, ctypes.POINTER(ctypes.c_int64)]),
    "svt_ring_destroy": (ctypes.c_int32, [P]),
    "svt_shadow_slices": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    "svt_shadow_forward": (ctypes.c_int32, [P, ctypes.POINTER(svt_shadow_tracks), P, P, P, P, P]),
    "svt_shadow_backward": (ctypes.c_int32, [P, ctypes.POINTER(svt_shadow_tracks), P, P, P, P, P,
                                             P, P, P]),
    "svt_shadow_penalty": (ctypes.c_int32, [P, ctypes.c_int32, P, ctypes.c_double, P, P, P, P]),
    "svt_shadow_adam": (ctypes.c_int32, [P, ctypes.c_int32, P, P, P, P, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_int32, P]),
    "svt_requantize": (ctypes.c_int32, [P, ctypes.c_int32, P, P, ctypes.c_int32, P, P, P, P, P]),
}


def _load():
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
    # first makes libsvt.so bind to that same runtime by SONAME; loading
    # libsvt.so first would bring in a second HIP/HSA runtime from /opt/rocm and
    # the two cannot share the device in one process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1311_0380_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class SVTError(RuntimeError):
    def __init__(self, status, what=""):
        msg = lib.svt_status_string(status).decode()
        if status == SVT_E_DEVICE:
            msg += " (" + lib.svt_last_error().decode() + ")"
        super().__init__(f"{what}: {msg}" if what else msg)
        self.status = status


def check(status, what=""):
    if status != SVT_OK:
        raise SVTError(status, what)
    return status


# ---------------------------------------------------------------------------
# same-name wrappers of the C ABI
# ---------------------------------------------------------------------------
def svt_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = P()
    check(lib.svt_create(ctypes.byref(h), int(device), int(hbm_budget_bytes)), "svt_create")
    return h


def svt_destroy(ctx):
    return lib.svt_destroy(ctx)


def svt_load_constants(ctx, coef: np.ndarray, offset: np.ndarray, chi2_cut: int) -> int:
    coef = np.ascontiguousarray(coef, np.int32)
    offset = np.ascontiguousarray(offset, np.int32)
    return lib.svt_load_constants(ctx, int(coef.shape[0]), coef.ctypes.data, offset.ctypes.data,
                                  ctypes.c_uint64(int(chi2_cut)))


def svt_fit_events(ctx, batch: svt_event_batch, res: svt_results, stream=None):
    t = ctypes.c_int64(0)
    st = lib.svt_fit_events(ctx, ctypes.byref(batch), ctypes.byref(res),
                            None if stream is None else P(stream), ctypes.byref(t))
    return st, t.value


def svt_result(ctx, ticket: int, wait_us: int = -1):
    s = svt_summary()
    st = lib.svt_result(ctx, int(ticket), int(wait_us), ctypes.byref(s))
    return st, s


def svt_status_string(status: int) -> str:
    return lib.svt_status_string(int(status)).decode()


def svt_set_tuning(ctx, events_per_chunk=0, blocks_per_cu=0, schedule=0, kernel=0):
    t = svt_tuning(int(events_per_chunk), int(blocks_per_cu), int(schedule), int(kernel))
    return lib.svt_set_tuning(ctx, ctypes.byref(t))


def svt_set_timing(ctx, every: int):
    return lib.svt_set_timing(ctx, int(every))


def svt_get_tuning(ctx) -> dict:
    t = svt_tuning()
    check(lib.svt_get_tuning(ctx, ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in t._fields_}


def svt_get_device_info(ctx) -> dict:
    i = svt_device_info()
    check(lib.svt_get_device_info(ctx, ctypes.byref(i)))
    d = {f: getattr(i, f) for f, _ in i._fields_}
    d["arch"] = d["arch"].decode()
    return d


def shadow_slices(n_tracks: int, n_sectors: int) -> int:
    v = ctypes.c_int32(0)
    check(lib.svt_shadow_slices(int(n_tracks), int(n_sectors), ctypes.byref(v)), "svt_shadow_slices")
    return v.value


# ---------------------------------------------------------------------------
# torch-facing helpers (device memory and streams come from torch)
# ---------------------------------------------------------------------------
BATCH_FIELDS = ("road_offsets", "sector", "nhits", "hit_offsets", "hits", "xft")
RESULT_FIELDS = ("ncomb", "npass", "best", "chi2", "params", "hit_index", "ntracks")


@dataclass
class DeviceBatch:
    """A batch resident in device memory (torch tensors on cuda)."""
    road_offsets: "torch.Tensor"
    sector: "torch.Tensor"
    nhits: "torch.Tensor"
    hit_offsets: "torch.Tensor"
    hits: "torch.Tensor"
    xft: "torch.Tensor"

    @property
    def n_events(self):
        return int(self.road_offsets.numel() - 1)

    @property
    def n_roads(self):
        return int(self.sector.numel())

    @property
    def n_hits(self):
        return int(self.hits.numel())

    def struct(self, mem_kind=SVT_MEM_DEVICE) -> svt_event_batch:
        return svt_event_batch(self.n_events, self.n_roads, self.n_hits, mem_kind,
                               *[getattr(self, f).data_ptr() for f in BATCH_FIELDS])

    def nbytes(self) -> int:
        return sum(getattr(self, f).numel() * getattr(self, f).element_size() for f in BATCH_FIELDS)


def to_device(batch, device="cuda") -> DeviceBatch:
    import torch
    return DeviceBatch(**{f: torch.from_numpy(np.ascontiguousarray(getattr(batch, f))).to(device)
                          for f in BATCH_FIELDS})


class DeviceResults:
    """Result buffers (torch tensors) for a batch of n_events / n_roads."""

    def __init__(self, n_events, n_roads, device="cuda", comb_offsets=False, pin=False):
        import torch
        kw = dict(device=device) if not pin else dict(pin_memory=True)
        self.ncomb = torch.empty(n_roads, dtype=torch.int32, **kw)
        self.npass = torch.empty(n_roads, dtype=torch.int32, **kw)
        self.best = torch.empty(n_roads, dtype=torch.int32, **kw)
        self.chi2 = torch.empty(n_roads, dtype=torch.int64, **kw)      # bit pattern of uint64
        self.params = torch.empty((n_roads, 3), dtype=torch.int32, **kw)
        self.hit_index = torch.empty((n_roads, 4), dtype=torch.uint8, **kw)
        self.ntracks = torch.empty(n_events, dtype=torch.int32, **kw)
        self.comb_offsets = torch.empty(n_roads + 1, dtype=torch.int64, **kw) if comb_offsets else None
        self.mem_kind = SVT_MEM_PINNED if pin else SVT_MEM_DEVICE

    def struct(self) -> svt_results:
        return svt_results(*[getattr(self, f).data_ptr() for f in RESULT_FIELDS],
                           self.comb_offsets.data_ptr() if self.comb_offsets is not None else None,
                           self.mem_kind, 0)

    def numpy(self) -> dict:
        out = {f: getattr(self, f).cpu().numpy() for f in RESULT_FIELDS}
        out["chi2"] = out["chi2"].view(np.uint64)
        if self.comb_offsets is not None:
            out["comb_offsets"] = self.comb_offsets.cpu().numpy()
        return out


def svt_io_probe(ctx, kind, direction, nbytes, reps=20):
    us = ctypes.c_double(0.0)
    check(lib.svt_io_probe(ctx, int(kind), int(direction), int(nbytes), int(reps),
                           ctypes.byref(us)), "svt_io_probe")
    return us.value


def svt_plan_create(ctx, max_events, max_roads, max_hits, events_per_chunk=0, blocks_per_cu=0,
                    schedule=0, kernel=0):
    h = P()
    t = svt_tuning(int(events_per_chunk), int(blocks_per_cu), int(schedule), int(kernel))
    check(lib.svt_plan_create(ctx, int(max_events), int(max_roads), int(max_hits),
                              ctypes.byref(t), ctypes.byref(h)), "svt_plan_create")
    return h


def svt_plan_destroy(plan):
    return lib.svt_plan_destroy(plan)


def svt_plan_buffers(plan):
    b, r = svt_event_batch(), svt_results()
    check(lib.svt_plan_buffers(plan, ctypes.byref(b), ctypes.byref(r)), "svt_plan_buffers")
    return b, r


def svt_ring_info(ring):
    """(n_passes, passes_per_launch, n_launches) of a ring."""
    v = [ctypes.c_int32(0) for _ in range(3)]
    check(lib.svt_ring_info(ring, *[ctypes.byref(x) for x in v]), "svt_ring_info")
    return tuple(x.value for x in v)


def svt_ring_create(ctx, batches, results, n_passes, passes_per_launch=0):
    """A ring over device batches / results (lists of svt_event_batch and
    svt_results of equal length); returns (status, ring handle or None)."""
    n = len(batches)
    ba = (svt_event_batch * n)(*batches)
    ra = (svt_results * n)(*results)
    h = P()
    st = lib.svt_ring_create(ctx, n, ba, ra, int(n_passes), int(passes_per_launch),
                             ctypes.byref(h))
    return st, (h if st == SVT_OK else None)


def svt_ring_run(ring, stream=None):
    t = ctypes.c_int64(0)
    st = lib.svt_ring_run(ring, None if stream is None else P(stream), ctypes.byref(t))
    return st, t.value


def svt_ring_destroy(ring):
    return lib.svt_ring_destroy(ring)


def svt_list_passing(ctx, batch: svt_event_batch, npass_ptr: int, lst: svt_pass_list, stream=None):
    t = ctypes.c_int64(0)
    st = lib.svt_list_passing(ctx, ctypes.byref(batch), P(npass_ptr), ctypes.byref(lst),
                              None if stream is None else P(stream), ctypes.byref(t))
    return st, t.value


def svt_list_passing_noalloc(ctx, batch: svt_event_batch, npass_ptr: int, lst: svt_pass_list,
                             stream=None):
    t = ctypes.c_int64(0)
    st = lib.svt_list_passing_noalloc(ctx, ctypes.byref(batch), P(npass_ptr), ctypes.byref(lst),
                                      None if stream is None else P(stream), ctypes.byref(t))
    return st, t.value


def svt_unpack_stream(ctx, words_ptr: int, n_words: int, mem_kind: int, out: svt_unpack_out,
                      stream=None):
    t = ctypes.c_int64(0)
    st = lib.svt_unpack_stream(ctx, None if not words_ptr else P(words_ptr), int(n_words),
                               int(mem_kind), ctypes.byref(out),
                               None if stream is None else P(stream), ctypes.byref(t))
    return st, t.value


class DeviceUnpacked:
    """Device arrays (torch tensors) an unpack fills, at given capacities."""

    def __init__(self, max_events: int, max_roads: int, max_hits: int, device="cuda"):
        import torch
        self.caps = (int(max_events), int(max_roads), int(max_hits))
        z = lambda n, dt: torch.zeros(n, dtype=dt, device=device)
        self.road_offsets = z(max_events + 1, torch.int32)
        self.sector = z(max(max_roads, 1), torch.uint8)
        self.nhits = z((max(max_roads, 1), 4), torch.uint8)
        self.hit_offsets = z(max_roads + 1, torch.int32)
        self.hits = z(max(max_hits, 1), torch.int16)
        self.xft = z((max(max_roads, 1), 2), torch.int16)

    def struct(self) -> svt_unpack_out:
        return svt_unpack_out(*[getattr(self, f).data_ptr() for f in BATCH_FIELDS], *self.caps, 0)

    def batch(self, n_events: int, n_roads: int, n_hits: int) -> "DeviceBatch":
        """The unpacked batch (views of the leading entries)."""
        return DeviceBatch(road_offsets=self.road_offsets[:n_events + 1], sector=self.sector[:n_roads],
                           nhits=self.nhits[:n_roads], hit_offsets=self.hit_offsets[:n_roads + 1],
                           hits=self.hits[:n_hits], xft=self.xft[:n_roads])


class DevicePassList:
    """Device buffers of a passing-combination list (torch tensors)."""

    def __init__(self, n_roads: int, capacity: int, device="cuda"):
        import torch
        cap = max(int(capacity), 0)
        self.capacity = cap
        self.offsets = torch.zeros(n_roads + 1, dtype=torch.int64, device=device)
        self.k = torch.zeros(max(cap, 1), dtype=torch.int32, device=device)
        self.chi2 = torch.zeros(max(cap, 1), dtype=torch.int64, device=device)
        self.params = torch.zeros((max(cap, 1), 3), dtype=torch.int32, device=device)

    def struct(self) -> svt_pass_list:
        return svt_pass_list(self.offsets.data_ptr(), self.k.data_ptr(), self.chi2.data_ptr(),
                             self.params.data_ptr(), self.capacity)

    def numpy(self, n=None) -> dict:
        off = self.offsets.cpu().numpy()
        n = min(int(off[-1]) if n is None else n, self.capacity)
        return dict(offsets=off, k=self.k.cpu().numpy()[:n],
                    chi2=self.chi2.cpu().numpy().view(np.uint64)[:n],
                    params=self.params.cpu().numpy()[:n])


def svt_plan_fit(plan, batch: svt_event_batch, res: svt_results, stream=None):
    t = ctypes.c_int64(0)
    st = lib.svt_plan_fit(plan, ctypes.byref(batch), ctypes.byref(res),
                          None if stream is None else P(stream), ctypes.byref(t))
    return st, t.value


class Context:
    """Owns an svt_ctx; thin convenience layer over the C calls."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.handle = svt_create(device, hbm_budget_bytes)

    def close(self):
        if self.handle:
            svt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_constants(self, coef, offset, chi2_cut):
        check(svt_load_constants(self.handle, coef, offset, chi2_cut), "svt_load_constants")

    def submit(self, batch_struct: svt_event_batch, res_struct: svt_results, stream=None) -> int:
        st, t = svt_fit_events(self.handle, batch_struct, res_struct, stream)
        check(st, "svt_fit_events")
        return t

    def result(self, ticket: int, wait_us: int = -1):
        return svt_result(self.handle, ticket, wait_us)

    def fit(self, dbatch: DeviceBatch, res: DeviceResults = None, stream=None):
        """Fit a device-resident batch on torch's current stream; blocks."""
        import torch
        if res is None:
            res = DeviceResults(dbatch.n_events, dbatch.n_roads, device=dbatch.sector.device)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        t = self.submit(dbatch.struct(), res.struct(), stream)
        st, summ = self.result(t, -1)
        return st, summ, res

    def list_passing(self, dbatch: DeviceBatch, res: DeviceResults, capacity=None, stream=None):
        """Every passing combination of a fitted device batch (res holds its
        fit); blocks.  capacity None sizes the list from the fit's pass
        counts.  Returns (status, summary, DevicePassList)."""
        import torch
        if capacity is None:
            capacity = int(res.npass.sum().item())
        lst = DevicePassList(dbatch.n_roads, capacity, device=dbatch.sector.device)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        st, t = svt_list_passing(self.handle, dbatch.struct(), res.npass.data_ptr(), lst.struct(),
                                 stream)
        check(st, "svt_list_passing")
        st, summ = self.result(t, -1)
        return st, summ, lst

    def unpack_stream(self, words, mem_kind=None, caps=None, stream=None):
        """Unpack a packed word stream (a torch tensor of int32/uint32 words on
        the device or in pinned host memory, or a numpy array); blocks.
        caps = (max_events, max_roads, max_hits), by default the most the
        stream could hold.  Returns (status, summary, DeviceBatch or None)."""
        import torch
        if isinstance(words, np.ndarray):
            host = torch.from_numpy(np.ascontiguousarray(words).view(np.int32))
            kind = SVT_MEM_PAGEABLE if mem_kind is None else mem_kind
            ptr, n = host.data_ptr(), host.numel()
        else:
            host = words
            kind = (SVT_MEM_DEVICE if words.is_cuda else SVT_MEM_MAPPED) if mem_kind is None else mem_kind
            ptr, n = words.data_ptr(), words.numel()
        if caps is None:
            caps = (n, n // 2, 2 * n)
        out = DeviceUnpacked(*caps)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        st, t = svt_unpack_stream(self.handle, ptr, n, kind, out.struct(), stream)
        check(st, "svt_unpack_stream")
        st, summ = self.result(t, -1)
        del host
        if st != SVT_OK:
            return st, summ, None
        return st, summ, out.batch(summ.total_tracks, int(summ.total_comb), int(summ.total_pass))

    def set_tuning(self, **kw):
        check(svt_set_tuning(self.handle, **kw), "svt_set_tuning")

    def tuning(self):
        return svt_get_tuning(self.handle)

    def set_timing(self, every: int):
        """Which later fit requests measure their device time (1 all, N every
        N-th ticket, 0 none); untimed ones report device_ns 0."""
        check(svt_set_timing(self.handle, every), "svt_set_timing")

    def device_info(self):
        return svt_get_device_info(self.handle)
