"""Independent checks that pin the CPU oracle (and, through it, the GPU path).

`brute_fit` enumerates combinations with itertools.product and evaluates all
fit rows at once as an integer matrix product (numpy int64), then picks the
best passing combination with a lexicographic sort.  It shares no code or
loop structure with the oracle's scalar nested loops; it is used on tiny
inputs only.
"""
from __future__ import annotations

import itertools

import numpy as np


def brute_fit(batch, consts):
    """Per-road results for every road of the batch (dict of arrays)."""
    nr, ne = batch.n_roads, batch.n_events
    res = dict(ncomb=np.zeros(nr, np.int64), npass=np.zeros(nr, np.int64),
               best=np.full(nr, -1, np.int64), chi2=np.full(nr, np.iinfo(np.uint64).max, np.uint64),
               params=np.zeros((nr, 3), np.int64), hit_index=np.full((nr, 4), 255, np.int64),
               ntracks=np.zeros(ne, np.int64))
    cut = int(consts.chi2_cut)
    for r in range(nr):
        n = [int(v) for v in batch.nhits[r]]
        h0 = int(batch.hit_offsets[r])
        layers, pos = [], h0
        for nl in n:
            layers.append([int(v) for v in batch.hits[pos:pos + nl]])
            pos += nl
        combos = list(itertools.product(*[range(nl) for nl in n]))   # last layer fastest
        res["ncomb"][r] = len(combos)
        if not combos:
            continue
        X = np.array([[layers[0][c[0]], layers[1][c[1]], layers[2][c[2]], layers[3][c[3]],
                       int(batch.xft[r, 0]), int(batch.xft[r, 1])] for c in combos], np.int64)
        s = int(batch.sector[r])
        Y = X @ consts.coef[s].astype(np.int64).T + consts.offset[s].astype(np.int64)
        chi2 = [int(a) * int(a) + int(b) * int(b) + int(c) * int(c) for a, b, c in Y[:, 3:]]
        passing = [k for k in range(len(combos)) if chi2[k] <= cut]
        res["npass"][r] = len(passing)
        if passing:
            k = min(passing, key=lambda q: (chi2[q], q))
            res["best"][r] = k
            res["chi2"][r] = np.uint64(chi2[k])
            res["params"][r] = Y[k, :3]
            res["hit_index"][r] = combos[k]
    for e in range(ne):
        r0, r1 = int(batch.road_offsets[e]), int(batch.road_offsets[e + 1])
        res["ntracks"][e] = int((res["best"][r0:r1] >= 0).sum())
    return res


def brute_list(batch, consts):
    """Every passing combination, road by road in combination order, by the
    same itertools enumeration and matrix product as brute_fit."""
    nr = batch.n_roads
    cut = int(consts.chi2_cut)
    offsets, ks, chis, pars = [0], [], [], []
    for r in range(nr):
        n = [int(v) for v in batch.nhits[r]]
        layers, pos = [], int(batch.hit_offsets[r])
        for nl in n:
            layers.append([int(v) for v in batch.hits[pos:pos + nl]])
            pos += nl
        combos = list(itertools.product(*[range(nl) for nl in n]))
        if combos:
            X = np.array([[layers[0][c[0]], layers[1][c[1]], layers[2][c[2]], layers[3][c[3]],
                           int(batch.xft[r, 0]), int(batch.xft[r, 1])] for c in combos], np.int64)
            s = int(batch.sector[r])
            Y = X @ consts.coef[s].astype(np.int64).T + consts.offset[s].astype(np.int64)
            for k in range(len(combos)):
                c2 = sum(int(v) * int(v) for v in Y[k, 3:])
                if c2 <= cut:
                    ks.append(k)
                    chis.append(c2)
                    pars.append([int(v) for v in Y[k, :3]])
        offsets.append(len(ks))
    return dict(offsets=np.array(offsets, np.int64), k=np.array(ks, np.int64),
                chi2=np.array(chis, np.uint64), params=np.array(pars, np.int64).reshape(-1, 3))


FIELDS = ("ncomb", "npass", "best", "chi2", "params", "hit_index", "ntracks")
LIST_FIELDS = ("offsets", "k", "chi2", "params")


def assert_same(got: dict, want: dict, fields=FIELDS, where=""):
    for f in fields:
        a = np.asarray(got[f]).astype(np.int64) if f != "chi2" else np.asarray(got[f]).astype(np.uint64)
        b = np.asarray(want[f]).astype(np.int64) if f != "chi2" else np.asarray(want[f]).astype(np.uint64)
        a = a.reshape(b.shape)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            i = tuple(bad[0])
            raise AssertionError(f"{where}{f}: {len(bad)} mismatches, first at {i}: "
                                 f"got {a[i]} want {b[i]}")
