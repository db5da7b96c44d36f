"""CPU oracle for the SVT linearized track fit -- TEST INFRASTRUCTURE.

Only `tests/`, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product path (the HIP library and its binding) never imports
it, and it imports nothing from the product path: inputs come in as plain
numpy arrays.

`fit()` wraps the plain-C nested loops in svt_oracle.c (paper Sec. 2 fit
equation, Sec. 2.1 three nested loops); `list_passing()` keeps every passing
combination rather than the best per road; `unpack_stream()` parses the
packed input word stream.  The float-shadow functions live in
`oracle.shadow`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "svt_oracle.c")
LIB = os.path.join(HERE, "libsvt_oracle.so")

OK, E_INVAL, E_RANGE = 0, -1, -2


class Summary(ctypes.Structure):
    _fields_ = [("total_comb", ctypes.c_int64), ("total_pass", ctypes.c_int64),
                ("total_tracks", ctypes.c_int32), ("err_road", ctypes.c_int32),
                ("err_event", ctypes.c_int32), ("pad", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, -O2, no fast-math, OpenMP event loop)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                        "-Wall", "-Wextra", "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        L.orc_fit.restype = ctypes.c_int
        L.orc_fit.argtypes = [ctypes.c_int32] * 3 + [P] * 6 + [ctypes.c_int32, P, P,
                                                              ctypes.c_uint64] + [P] * 8 + \
            [ctypes.c_int32, ctypes.POINTER(Summary)]
        L.orc_check_constants.restype = ctypes.c_int
        L.orc_check_constants.argtypes = [ctypes.c_int32, P, P, ctypes.c_uint64]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_unpack_stream.restype = ctypes.c_int
        L.orc_unpack_stream.argtypes = [P, ctypes.c_int64] + [ctypes.c_int32] * 3 + [P] * 8
        L.orc_list_passing.restype = ctypes.c_int
        L.orc_list_passing.argtypes = [ctypes.c_int32] * 3 + [P] * 6 + [ctypes.c_int32, P, P,
                                                                       ctypes.c_uint64,
                                                                       ctypes.c_int64] + \
            [P] * 4 + [ctypes.POINTER(Summary)]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def check_constants(coef, offset, chi2_cut) -> int:
    coef = np.ascontiguousarray(coef, np.int32)
    offset = np.ascontiguousarray(offset, np.int32)
    return lib().orc_check_constants(int(coef.shape[0]), _ptr(coef), _ptr(offset),
                                     ctypes.c_uint64(int(chi2_cut)))


def fit(road_offsets, sector, nhits, hit_offsets, hits, xft, coef, offset, chi2_cut,
        n_threads: int = 1, comb_offsets: bool = True, n_roads=None, n_hits=None):
    """Run the oracle.  Returns (status, results dict, summary dict)."""
    ro = np.ascontiguousarray(road_offsets, np.int32)
    sector = np.ascontiguousarray(sector, np.uint8)
    nhits = np.ascontiguousarray(nhits, np.uint8).reshape(-1)
    ho = np.ascontiguousarray(hit_offsets, np.int32)
    hits = np.ascontiguousarray(hits, np.int16)
    xft = np.ascontiguousarray(xft, np.int16).reshape(-1)
    coef = np.ascontiguousarray(coef, np.int32)
    offset = np.ascontiguousarray(offset, np.int32)
    n_events = ro.shape[0] - 1
    nr = sector.shape[0] if n_roads is None else n_roads
    nh = hits.shape[0] if n_hits is None else n_hits
    out = dict(ncomb=np.zeros(max(nr, 0), np.int32), npass=np.zeros(max(nr, 0), np.int32),
               best=np.zeros(max(nr, 0), np.int32), chi2=np.zeros(max(nr, 0), np.uint64),
               params=np.zeros((max(nr, 0), 3), np.int32),
               hit_index=np.zeros((max(nr, 0), 4), np.uint8),
               ntracks=np.zeros(max(n_events, 0), np.int32),
               comb_offsets=np.zeros(max(nr, 0) + 1, np.int64) if comb_offsets else None)
    s = Summary()
    rc = lib().orc_fit(n_events, nr, nh, _ptr(ro), _ptr(sector), _ptr(nhits), _ptr(ho),
                       _ptr(hits), _ptr(xft), int(coef.shape[0]), _ptr(coef), _ptr(offset),
                       ctypes.c_uint64(int(chi2_cut)), _ptr(out["ncomb"]), _ptr(out["npass"]),
                       _ptr(out["best"]), _ptr(out["chi2"]), _ptr(out["params"]),
                       _ptr(out["hit_index"]), _ptr(out["ntracks"]), _ptr(out["comb_offsets"]),
                       int(n_threads), ctypes.byref(s))
    summ = dict(total_comb=s.total_comb, total_pass=s.total_pass, total_tracks=s.total_tracks,
                err_road=s.err_road, err_event=s.err_event)
    return rc, out, summ


def fit_batch(batch, consts, **kw):
    """Convenience wrapper taking objects with the batch / constants fields."""
    return fit(batch.road_offsets, batch.sector, batch.nhits, batch.hit_offsets, batch.hits,
               batch.xft, consts.coef, consts.offset, consts.chi2_cut, **kw)


def list_passing(road_offsets, sector, nhits, hit_offsets, hits, xft, coef, offset, chi2_cut,
                 capacity=None):
    """Every passing combination, road by road in combination-index order.
    Returns (status, dict(offsets, k, chi2, params), summary dict); with
    capacity None the list is sized by a first counting run."""
    ro = np.ascontiguousarray(road_offsets, np.int32)
    sector = np.ascontiguousarray(sector, np.uint8)
    nhits = np.ascontiguousarray(nhits, np.uint8).reshape(-1)
    ho = np.ascontiguousarray(hit_offsets, np.int32)
    hits = np.ascontiguousarray(hits, np.int16)
    xft = np.ascontiguousarray(xft, np.int16).reshape(-1)
    coef = np.ascontiguousarray(coef, np.int32)
    offset = np.ascontiguousarray(offset, np.int32)
    n_events, nr, nh = ro.shape[0] - 1, sector.shape[0], hits.shape[0]

    def run(cap):
        out = dict(offsets=np.zeros(nr + 1, np.int64), k=np.zeros(max(cap, 1), np.int32),
                   chi2=np.zeros(max(cap, 1), np.uint64), params=np.zeros((max(cap, 1), 3), np.int32))
        s = Summary()
        rc = lib().orc_list_passing(n_events, nr, nh, _ptr(ro), _ptr(sector), _ptr(nhits), _ptr(ho),
                                    _ptr(hits), _ptr(xft), int(coef.shape[0]), _ptr(coef),
                                    _ptr(offset), ctypes.c_uint64(int(chi2_cut)),
                                    ctypes.c_int64(int(cap)), _ptr(out["offsets"]), _ptr(out["k"]),
                                    _ptr(out["chi2"]), _ptr(out["params"]), ctypes.byref(s))
        n = min(int(out["offsets"][-1]), cap)
        for f in ("k", "chi2", "params"):
            out[f] = out[f][:n]
        summ = dict(total_comb=s.total_comb, total_pass=s.total_pass, err_road=s.err_road,
                    err_event=s.err_event)
        return rc, out, summ

    if capacity is None:
        rc, out, summ = run(0)
        if rc not in (OK, E_RANGE) or summ["err_road"] >= 0 or summ["err_event"] >= 0:
            return rc, out, summ
        capacity = summ["total_pass"]
    return run(int(capacity))


def list_passing_batch(batch, consts, **kw):
    return list_passing(batch.road_offsets, batch.sector, batch.nhits, batch.hit_offsets,
                        batch.hits, batch.xft, consts.coef, consts.offset, consts.chi2_cut, **kw)


def unpack_stream(words, max_events=None, max_roads=None, max_hits=None):
    """Sequential parse of a packed word stream.  Returns (status, arrays,
    counts (events, roads, hits), first bad word or -1).  Capacities default
    to what the stream could hold at most."""
    w = np.ascontiguousarray(words, np.uint32)
    n = int(w.shape[0])
    me = n if max_events is None else int(max_events)
    mr = n if max_roads is None else int(max_roads)
    mh = 2 * n if max_hits is None else int(max_hits)
    out = dict(road_offsets=np.zeros(me + 1, np.int32), sector=np.zeros(max(mr, 1), np.uint8),
               nhits=np.zeros((max(mr, 1), 4), np.uint8), hit_offsets=np.zeros(mr + 1, np.int32),
               hits=np.zeros(max(mh, 1), np.int16), xft=np.zeros((max(mr, 1), 2), np.int16))
    counts = np.zeros(3, np.int64)
    bad = ctypes.c_int64(0)
    rc = lib().orc_unpack_stream(_ptr(w), n, me, mr, mh, _ptr(out["road_offsets"]),
                                 _ptr(out["sector"]), _ptr(out["nhits"]), _ptr(out["hit_offsets"]),
                                 _ptr(out["hits"]), _ptr(out["xft"]), _ptr(counts),
                                 ctypes.byref(bad))
    ne, nr, nh = (int(v) for v in counts)
    if rc == OK:
        out = dict(road_offsets=out["road_offsets"][:ne + 1], sector=out["sector"][:nr],
                   nhits=out["nhits"][:nr], hit_offsets=out["hit_offsets"][:nr + 1],
                   hits=out["hits"][:nh], xft=out["xft"][:nr])
    return rc, out, (ne, nr, nh), int(bad.value)


def max_threads() -> int:
    return int(lib().orc_max_threads())
