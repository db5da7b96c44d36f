"""GPU parity of the packed-word-stream unpack: every batch array equal to
the oracle parser's (and to the batch the stream was packed from), the first
bad word of malformed streams equal to the oracle's, through the C ABI from
device, host-mapped (zero copy) and pageable memory."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth
from tests.test_stream_oracle import MUT

pytestmark = pytest.mark.gpu

FIELDS = ("road_offsets", "sector", "nhits", "hit_offsets", "hits", "xft")


@pytest.fixture(scope="module")
def ctx():
    from paper_1311_0380_amd import svt
    c = svt.Context(0)
    yield c
    c.close()


def put(words, kind):
    import torch
    from paper_1311_0380_amd import svt
    t = torch.from_numpy(np.ascontiguousarray(words, np.uint32).view(np.int32))
    if kind == svt.SVT_MEM_DEVICE:
        return t.cuda()
    if kind == svt.SVT_MEM_MAPPED:
        return t.pin_memory()
    return np.ascontiguousarray(words, np.uint32)


def same_arrays(dbatch, want, where=""):
    for f in FIELDS:
        a = getattr(dbatch, f).cpu().numpy().reshape(-1).astype(np.int64)
        b = np.asarray(want[f] if isinstance(want, dict) else getattr(want, f)).reshape(-1).astype(np.int64)
        assert np.array_equal(a, b), f"{where}{f}"


SHAPES = {
    "small plain fit": lambda rng: synth.cfg1(n_events=100)[0],
    "scaled-up fit, 400 events (several tiles)": lambda rng: synth.cfg2(n_events=400)[0],
    "uneven, 3000 events": lambda rng: synth.cfg3(n_events=3000)[0],
    "deep layers": lambda rng: synth.random_small(rng, n_events=200, max_roads=10, max_hits=16,
                                                  n_sectors=72),
}


@pytest.mark.parametrize("kind", [3, 2, 0])
@pytest.mark.parametrize("name", sorted(SHAPES))
def test_unpack_matches_oracle(ctx, oracle_lib, name, kind):
    batch = SHAPES[name](np.random.default_rng(3))
    words = synth.pack_stream(batch)
    rc, want, counts, bad = oracle_lib.unpack_stream(words)
    assert rc == 0 and counts == (batch.n_events, batch.n_roads, batch.n_hits)
    st, summ, got = ctx.unpack_stream(put(words, kind), mem_kind=kind)
    assert st == 0, summ.as_dict()
    assert (summ.total_tracks, summ.total_comb, summ.total_pass) == counts
    same_arrays(got, want, f"{name}, kind {kind}: ")
    same_arrays(got, batch, f"{name}, kind {kind} (packed batch): ")


@pytest.mark.parametrize("name", sorted(MUT))
def test_first_bad_word_small(ctx, oracle_lib, name):
    from paper_1311_0380_amd import svt
    words, at = MUT[name]
    words = np.array(words, np.uint32)
    st, summ, _ = ctx.unpack_stream(put(words, 3), mem_kind=3)
    assert st == svt.SVT_E_RANGE and summ.err_road == at


def _corrupt(words, rng, how):
    w = words.copy()
    p = int(rng.integers(1, len(w) - 1))
    if how == "retag":
        w[p] = (w[p] & np.uint32(0x3FFFFFFF)) | np.uint32(int(rng.integers(0, 4)) << 30)
        if w[p] == words[p]:
            w[p] ^= np.uint32(1 << 31)
    elif how == "drop":
        w = np.delete(w, p)
    elif how == "insert":
        w = np.insert(w, p, np.uint32(int(rng.integers(0, 1 << 32))))
    elif how == "reserved":
        w[p] |= np.uint32(1 << 28)
    elif how == "truncate":
        w = w[:p]
    return w


@pytest.mark.parametrize("how", ["retag", "drop", "insert", "reserved", "truncate"])
def test_first_bad_word_across_tiles(ctx, oracle_lib, how):
    """Corruptions anywhere in a stream of many 2048-word tiles: the lowest
    flagged word equals the sequential parser's first failure."""
    from paper_1311_0380_amd import svt
    batch, _ = synth.cfg2(n_events=300)
    words = synth.pack_stream(batch)
    rng = np.random.default_rng({"retag": 1, "drop": 2, "insert": 3, "reserved": 4, "truncate": 5}[how])
    seen = 0
    for _ in range(12):
        w = _corrupt(words, rng, how)
        rc, _, _, bad = oracle_lib.unpack_stream(w)
        st, summ, got = ctx.unpack_stream(put(w, 3), mem_kind=3)
        if rc == 0:      # some corruptions leave a valid stream (e.g. a changed hit)
            assert st == 0
            continue
        seen += 1
        assert st == svt.SVT_E_RANGE and summ.err_road == bad, (how, bad, summ.err_road)
    assert seen > 0


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_device_words(ctx, shift):
    """Words at an address that is not 16-byte aligned (4-byte loads instead
    of 16-byte ones), with a ragged tail."""
    import torch
    batch, _ = synth.cfg2(n_events=50)
    words = synth.pack_stream(batch)
    buf = torch.zeros(len(words) + 4, dtype=torch.int32, device="cuda")
    buf[shift:shift + len(words)] = torch.from_numpy(words.view(np.int32)).cuda()
    view = buf[shift:shift + len(words)]
    assert view.data_ptr() % 16 != 0
    st, summ, got = ctx.unpack_stream(view, mem_kind=3)
    assert st == 0, summ.as_dict()
    same_arrays(got, batch, f"shift {shift}: ")


def test_capacity(ctx, oracle_lib):
    from paper_1311_0380_amd import svt
    batch, _ = synth.cfg2(n_events=30)
    words = synth.pack_stream(batch)
    full = (batch.n_events, batch.n_roads, batch.n_hits)
    for caps in ((29, full[1], full[2]), (full[0], full[1] - 1, full[2]), (full[0], full[1], full[2] - 1)):
        st, summ, got = ctx.unpack_stream(put(words, 3), mem_kind=3, caps=caps)
        assert st == svt.SVT_E_RANGE and summ.err_road == -1, caps
        assert (summ.total_tracks, summ.total_comb, summ.total_pass) == full
    st, summ, got = ctx.unpack_stream(put(words, 3), mem_kind=3, caps=full)
    assert st == 0
    same_arrays(got, batch)


def test_empty_and_event_only(ctx):
    import torch
    from paper_1311_0380_amd import svt
    st, summ, got = ctx.unpack_stream(torch.zeros(0, dtype=torch.int32, device="cuda"), caps=(1, 1, 1))
    assert st == 0 and (summ.total_tracks, summ.total_comb, summ.total_pass) == (0, 0, 0)
    assert got.road_offsets.cpu().tolist() == [0]
    w = np.array([3 << 30] * 3, np.uint32)
    st, summ, got = ctx.unpack_stream(put(w, 3), mem_kind=3)
    assert st == 0 and summ.total_tracks == 3 and got.road_offsets.cpu().tolist() == [0, 0, 0, 0]


def test_unpack_then_fit(ctx, oracle_lib):
    """The unpacked batch fits to the oracle's results of the original."""
    from tests.gpu_helpers import FIELDS as RFIELDS
    batch, consts = synth.cfg2(n_events=200)
    st, summ, got = ctx.unpack_stream(put(synth.pack_stream(batch), 2), mem_kind=2)
    assert st == 0
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    st, fsum, res = ctx.fit(got)
    assert st == 0
    rc, want, wsum = oracle_lib.fit_batch(batch, consts, n_threads=8)
    out = res.numpy()
    for f in RFIELDS:
        a = out[f].astype(np.uint64 if f == "chi2" else np.int64).reshape(-1)
        b = want[f].astype(np.uint64 if f == "chi2" else np.int64).reshape(-1)
        assert np.array_equal(a, b), f


def test_invalid_calls(ctx):
    from paper_1311_0380_amd import svt
    out = svt.DeviceUnpacked(4, 4, 4)
    s = out.struct()
    for args in ((None, 5, 3), (1, -1, 3), (1, 5, 9)):
        st, _ = svt.svt_unpack_stream(ctx.handle, args[0] or 0, args[1], args[2], s)
        assert st == svt.SVT_E_INVAL, args
    bad = svt.svt_unpack_out(*[getattr(out, f).data_ptr() for f in FIELDS], -1, 4, 4, 0)
    st, _ = svt.svt_unpack_stream(ctx.handle, out.hits.data_ptr(), 0, 3, bad)
    assert st == svt.SVT_E_INVAL
    st, _ = svt.svt_unpack_stream(ctx.handle, out.hits.data_ptr(), 1 << 31, 3, s)
    assert st == svt.SVT_E_INVAL


def test_large_stream_grid_stride(ctx, oracle_lib):
    """More tiles than the last pass has blocks (4,095 at most: each block
    then loops over several tiles, carrying the sums before them): 20,000
    events of 64 roads, 9.3 M words in 2048-word tiles."""
    batch, _ = synth.cfg2(n_events=20000)
    words = synth.pack_stream(batch)
    assert len(words) > 4096 * 2048
    st, summ, got = ctx.unpack_stream(put(words, 3), mem_kind=3)
    assert st == 0 and summ.total_comb == batch.n_roads
    same_arrays(got, batch)
    # and a bad word in the last tiles
    # (a hit word: bit 29 is reserved there, while in a road header it is
    # part of the sector)
    w = words.copy()
    pos = max(i for i in range(len(w) - 200, len(w)) if (int(w[i]) >> 30) == 0)
    w[pos] |= np.uint32(1 << 29)
    rc, _, _, bad = oracle_lib.unpack_stream(w)
    st, summ, _ = ctx.unpack_stream(put(w, 3), mem_kind=3)
    assert rc != 0 and summ.err_road == bad
