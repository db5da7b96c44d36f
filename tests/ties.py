"""Batches whose layers repeat hit words, so that combinations tie on chi2
(twins share every fit input), and the invariant the tie rule implies."""
import numpy as np

from paper_1311_0380_amd import synth


def tie_batch(seed, max_hits, n_events=300, roads_per_event=24):
    rng = np.random.default_rng(seed)
    consts = synth.lattice_constants(rng)
    rpe = np.full(n_events, roads_per_event)
    n_roads = int(rpe.sum())
    nh = rng.integers(1, max_hits + 1, (n_roads, 4))
    mask = rng.random(n_roads) < 0.6
    b = synth.make_events(rng, rpe, nh, consts.n_sectors, mask, consts)
    hits = b.hits.astype(np.int64)
    nhits = b.nhits.astype(np.int64)
    for r in range(n_roads):
        base = int(b.hit_offsets[r])
        starts = base + np.concatenate([[0], np.cumsum(nhits[r])[:3]])
        for l in range(4):
            n = int(nhits[r, l])
            if n < 2:
                continue
            seg = slice(int(starts[l]), int(starts[l]) + n)
            layer = hits[seg]
            if b.track_road[r] and rng.random() < 0.8:
                # the true word at one or two more places, before or after it
                tp = int(b.track_pos[r, l])
                for j in rng.choice(n, size=min(n, 1 + int(rng.integers(0, 2))), replace=False):
                    layer[j] = layer[tp]
            if rng.random() < 0.5:
                # a random word copied onto another place
                i, j = rng.choice(n, size=2, replace=False)
                layer[j] = layer[i]
            if rng.random() < 0.15:
                # the layer repeats a short pattern: every word has a twin
                p = int(rng.integers(1, max(2, n // 2) + 1))
                layer[:] = np.resize(layer[:p], n)
            hits[seg] = layer
    b.hits = hits.astype(np.int16)
    return b, consts


def twin_roads(batch, best_hi):
    """Roads whose best combination has a twin: some layer holds its word
    at another index too.  Returns (count, violations), where a violation
    is a best whose word occurs at a lower index of the same layer (the
    lower twin has the same chi2 and a lower k, so the tie rule picks it)."""
    count = viol = 0
    for r in range(batch.n_roads):
        hi = best_hi[r]
        if hi[0] == 0xFF:
            continue
        base = int(batch.hit_offsets[r])
        n = batch.nhits[r].astype(np.int64)
        starts = base + np.concatenate([[0], np.cumsum(n)[:3]])
        twin = False
        for l in range(4):
            layer = batch.hits[int(starts[l]):int(starts[l]) + int(n[l])]
            v = layer[hi[l]]
            eq = np.nonzero(layer == v)[0]
            twin |= eq.size > 1
            viol += int(eq[0] != hi[l])
        count += int(twin)
    return count, viol
