"""Pins for the packed-word-stream unpack of the CPU oracle: round trips
through the packer, a stream written out word by word from the format, and
malformed streams whose first bad word is known by construction."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth

FIELDS = ("road_offsets", "sector", "nhits", "hit_offsets", "hits", "xft")

EV = 3 << 30


def road(sector, n, xft):
    """Road header and XFT word of the format, written out directly."""
    return [(2 << 30) | (sector << 22) | n[0] | (n[1] << 5) | (n[2] << 10) | (n[3] << 15),
            (1 << 30) | (xft[1] << 12) | xft[0]]


def hitwords(hits):
    out = []
    for i in range(0, len(hits), 2):
        second = hits[i + 1] if i + 1 < len(hits) else 0
        out.append(hits[i] | (second << 12))
    return out


def same_batch(out, batch):
    for f in FIELDS:
        a = np.asarray(out[f]).reshape(-1).astype(np.int64)
        b = np.asarray(getattr(batch, f)).reshape(-1).astype(np.int64)
        assert np.array_equal(a, b), f


@pytest.mark.parametrize("name", ["small", "scaled", "uneven", "sweep", "deep"])
def test_round_trip(oracle_lib, name):
    rng = np.random.default_rng(5)
    batch = {"small": lambda: synth.cfg1(n_events=40)[0],
             "scaled": lambda: synth.cfg2(n_events=60)[0],
             "uneven": lambda: synth.cfg3(n_events=500)[0],
             "sweep": lambda: synth.paper_sweep(20)[0],
             "deep": lambda: synth.random_small(rng, n_events=40, max_roads=6, max_hits=16,
                                                n_sectors=72)}[name]()
    words = synth.pack_stream(batch)
    rc, out, counts, bad = oracle_lib.unpack_stream(words)
    assert rc == 0 and bad == -1
    assert counts == (batch.n_events, batch.n_roads, batch.n_hits)
    same_batch(out, batch)


def test_written_out_stream(oracle_lib):
    """Two events (the second empty) and a third with two roads, one of them
    with no hit in layer 2 and an odd hit count, built word by word."""
    w = [EV]
    w += road(7, (2, 1, 1, 1), (100, 4095)) + hitwords([1, 2, 3, 4, 5])
    w += [EV, EV]
    w += road(71, (1, 3, 0, 2), (0, 17)) + hitwords([10, 11, 12, 13, 14, 15])
    w += road(0, (1, 1, 1, 1), (5, 6)) + hitwords([4095, 0, 7, 8])
    rc, out, counts, bad = oracle_lib.unpack_stream(np.array(w, np.uint32))
    assert rc == 0 and bad == -1 and counts == (3, 3, 15)
    assert list(out["road_offsets"]) == [0, 1, 1, 3]
    assert list(out["sector"]) == [7, 71, 0]
    assert out["nhits"].tolist() == [[2, 1, 1, 1], [1, 3, 0, 2], [1, 1, 1, 1]]
    assert list(out["hit_offsets"]) == [0, 5, 11, 15]
    assert list(out["hits"]) == [1, 2, 3, 4, 5, 10, 11, 12, 13, 14, 15, 4095, 0, 7, 8]
    assert out["xft"].tolist() == [[100, 4095], [0, 17], [5, 6]]
    # packing the decoded batch gives the same words back
    b = synth.Batch(**{f: np.asarray(out[f]) for f in FIELDS})
    assert np.array_equal(synth.pack_stream(b), np.array(w, np.uint32))


def _base():
    w = [EV]
    w += road(3, (1, 2, 1, 1), (9, 10)) + hitwords([1, 2, 3, 4, 5])   # words 1..5
    w += road(4, (1, 1, 1, 1), (11, 12)) + hitwords([6, 7, 8, 9])     # words 6..9
    w += [EV]                                                          # word 10
    w += road(5, (2, 2, 2, 2), (13, 14)) + hitwords(list(range(8)))   # words 11..16
    return w


def _mutations():
    b = _base()
    n = len(b)
    m = {}
    m["first word a road header"] = (b[1:], 0)
    m["first word a hit word"] = ([5] + b, 0)
    m["hit word in place of the XFT word"] = (b[:2] + [3] + b[3:], 2)
    m["XFT word with reserved bits"] = (b[:2] + [b[2] | (1 << 25)] + b[3:], 2)
    m["one hit word missing"] = (b[:5] + b[6:], 5)            # next road header comes early
    m["one hit word too many"] = (b[:6] + [77] + b[6:], 6)
    m["odd road's last word with a second hit"] = (b[:5] + [b[5] | (9 << 12)] + b[6:], 5)
    m["layer count above 16"] = (b[:6] + [b[6] | (17 << 5)] + b[7:], 6)
    m["road header reserved bits"] = (b[:6] + [b[6] | (1 << 20)] + b[7:], 6)
    m["event header reserved bits"] = (b[:10] + [EV | 1] + b[11:], 10)
    m["XFT word out of place"] = (b[:10] + [b[2]] + b[10:], 10)
    m["hit word after an event header"] = (b[:11] + [3] + b[11:], 11)
    m["ends inside the hits"] = (b[:-1], n - 1)
    m["ends after a road header"] = (b[:12], 12)
    m["hit word with reserved bits"] = (b[:3] + [b[3] | (1 << 29)] + b[4:], 3)
    return m


MUT = _mutations()


@pytest.mark.parametrize("name", sorted(MUT))
def test_first_bad_word(oracle_lib, name):
    words, at = MUT[name]
    rc, _, _, bad = oracle_lib.unpack_stream(np.array(words, np.uint32))
    assert rc == oracle_lib.E_RANGE and bad == at


def test_capacity_and_empty(oracle_lib):
    batch, _ = synth.cfg2(n_events=5)
    words = synth.pack_stream(batch)
    for kw in (dict(max_events=4), dict(max_roads=batch.n_roads - 1), dict(max_hits=batch.n_hits - 1)):
        rc, _, counts, bad = oracle_lib.unpack_stream(words, **kw)
        assert rc == oracle_lib.E_RANGE and bad == -1, kw
        assert counts == (batch.n_events, batch.n_roads, batch.n_hits)
    rc, out, counts, bad = oracle_lib.unpack_stream(np.zeros(0, np.uint32))
    assert rc == 0 and counts == (0, 0, 0) and list(out["road_offsets"]) == [0]
    rc, out, counts, _ = oracle_lib.unpack_stream(np.array([EV, EV], np.uint32))
    assert rc == 0 and counts == (2, 0, 0) and list(out["road_offsets"]) == [0, 0, 0]
