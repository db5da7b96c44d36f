"""Helpers for GPU tests: run the library on generator batches, compare with
the oracle field by field."""
from __future__ import annotations

import numpy as np

FIELDS = ("ncomb", "npass", "best", "chi2", "params", "hit_index", "ntracks")


def lib_fit(ctx, batch, mem_kind=3, res_kind=3, comb_offsets=False, stream=None):
    """Fit a numpy batch with the library.  Inputs and results live in the
    memory kind asked for; returns (status, summary dict, results dict)."""
    import torch
    from paper_1311_0380_amd import svt

    def put(arr, kind):
        t = torch.from_numpy(np.ascontiguousarray(arr))
        if kind == svt.SVT_MEM_DEVICE:
            return t.cuda()
        if kind in (svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED):
            return t.pin_memory()
        return t.clone()

    dev = {f: put(getattr(batch, f), mem_kind) for f in svt.BATCH_FIELDS}
    b = svt.svt_event_batch(batch.n_events, batch.n_roads, batch.n_hits, mem_kind,
                            *[dev[f].data_ptr() for f in svt.BATCH_FIELDS])
    nr, ne = batch.n_roads, batch.n_events
    shapes = dict(ncomb=((nr,), torch.int32), npass=((nr,), torch.int32),
                  best=((nr,), torch.int32), chi2=((nr,), torch.int64),
                  params=((nr, 3), torch.int32), hit_index=((nr, 4), torch.uint8),
                  ntracks=((ne,), torch.int32), comb_offsets=((nr + 1,), torch.int64))
    out = {}
    for f, (shape, dt) in shapes.items():
        if f == "comb_offsets" and not comb_offsets:
            out[f] = None
            continue
        if res_kind == svt.SVT_MEM_DEVICE:
            out[f] = torch.full(shape, -7, dtype=dt, device="cuda") if dt != torch.uint8 else \
                torch.full(shape, 77, dtype=dt, device="cuda")
        elif res_kind in (svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED):
            out[f] = torch.zeros(shape, dtype=dt).pin_memory()
        else:
            out[f] = torch.zeros(shape, dtype=dt)
    r = svt.svt_results(*[out[f].data_ptr() for f in FIELDS],
                        out["comb_offsets"].data_ptr() if comb_offsets else None, res_kind, 0)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st, ticket = svt.svt_fit_events(ctx, b, r, stream)
    if st != svt.SVT_OK:
        return st, None, None
    st, summ = svt.svt_result(ctx, ticket, -1)
    torch.cuda.synchronize()
    res = {f: (v.cpu().numpy() if v is not None else None) for f, v in out.items()}
    res["chi2"] = res["chi2"].view(np.uint64)
    return st, summ.as_dict(), res


def assert_equal_results(got, want, fields=FIELDS, where=""):
    for f in fields:
        a = np.asarray(got[f])
        b = np.asarray(want[f])
        if f == "chi2":
            a, b = a.astype(np.uint64), b.astype(np.uint64)
        else:
            a, b = a.astype(np.int64), b.astype(np.int64)
        a = a.reshape(b.shape)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            i = tuple(bad[0])
            raise AssertionError(f"{where}{f}: {len(bad)} of {b.size} differ; first at {i}: "
                                 f"got {a[i]} want {b[i]}")
