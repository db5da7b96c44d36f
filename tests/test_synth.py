"""Generators: determinism, shapes and the lattice-constant identities."""
import numpy as np

from paper_1311_0380_amd import synth


def _same(a, b):
    for f in ("road_offsets", "sector", "nhits", "hit_offsets", "hits", "xft"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_seeded_determinism():
    a, ca = synth.cfg1()
    b, cb = synth.cfg1()
    _same(a, b)
    assert np.array_equal(ca.coef, cb.coef) and ca.chi2_cut == cb.chi2_cut
    c, _ = synth.cfg1(seed=2)
    assert not np.array_equal(a.hits[:100], c.hits[:100])


def test_lattice_identities():
    assert np.all(synth.NULL_N @ synth.TRACK_H == 0)
    assert np.array_equal(synth.LEFT_INV5 @ synth.TRACK_H, 5 * np.eye(3, dtype=np.int64))
    consts = synth.lattice_constants(np.random.default_rng(0))
    A = consts.coef.astype(np.int64)
    assert np.all(np.einsum("skj,jc->skc", A[:, 3:], synth.TRACK_H) == 0)
    assert np.all(np.einsum("skj,jc->skc", A[:, :3], synth.TRACK_H) == 5 * np.eye(3, dtype=np.int64))
    assert np.abs(A).max() < 1024


def test_cfg_shapes():
    b, c = synth.cfg1()
    assert b.n_events == 100 and b.n_roads == 800
    assert b.nhits.min() >= 1 and b.nhits.max() <= 2
    assert c.coef.min() >= -1024 and c.coef.max() < 1024 and c.chi2_cut == 1 << 42
    b, c = synth.cfg2(n_events=50)
    assert b.n_roads == 50 * 64 and b.nhits.min() >= 1 and b.nhits.max() <= 4
    assert b.track_road.reshape(50, 64).sum(axis=1).tolist() == [32] * 50
    assert b.hits.min() >= 0 and b.hits.max() < 4096
    assert np.all(np.diff(b.hit_offsets) == b.nhits.astype(np.int64).sum(axis=1))
    b, c = synth.cfg3(n_events=400)
    rpe = np.diff(b.road_offsets)
    assert rpe.min() >= 1 and rpe.max() <= 256 and b.nhits.max() <= 8
    b, c = synth.paper_sweep(3)
    assert np.all(b.nhits == 4) and b.n_roads == 24


def test_planted_hits_on_manifold():
    b, c = synth.cfg2(n_events=20)
    tr = np.nonzero(b.track_road)[0]
    for r in tr[:50]:
        n = b.nhits[r].astype(int)
        lo = int(b.hit_offsets[r]) + np.concatenate([[0], np.cumsum(n)[:3]])
        words = [int(b.hits[lo[l] + b.track_pos[r, l]]) for l in range(4)] + list(b.xft[r])
        want = c.x0[b.sector[r]] + synth.TRACK_H @ b.track_theta[r]
        assert words == list(want)
        # noise hits of the layer differ from the planted word
        for l in range(4):
            seg = b.hits[lo[l]:lo[l] + n[l]]
            assert int((seg == words[l]).sum()) == 1


def test_select_and_concat_roundtrip():
    b, _ = synth.cfg3(n_events=30)
    parts = [b.select_events(0, 7), b.select_events(7, 19), b.select_events(19, 30)]
    _same(synth.concat(parts), b)


def test_bursts():
    rng = np.random.default_rng(5)
    s = synth.burst_sizes(rng, 20000)
    assert s.min() >= 1 and s.max() <= 3000
    assert abs(s.mean() - synth.log_uniform_mean()) / synth.log_uniform_mean() < 0.05
    t = synth.poisson_arrivals(rng, 1000, 1e5, synth.log_uniform_mean())
    assert np.all(np.diff(t) > 0)
