"""GPU parity of the passing-combination list: the HIP library's
svt_list_passing against the oracle's list, entry by entry (combination
index, chi2, fit rows 0..2) and offset by offset, through the C ABI."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1311_0380_amd import svt
    c = svt.Context(0)
    yield c
    c.close()


def gpu_list(ctx, batch, consts, capacity=None, npass_edit=None):
    """Fit the batch on the device, then list its passing combinations.
    Returns (status, summary dict, list dict)."""
    import torch
    from paper_1311_0380_amd import svt
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    db = svt.to_device(batch)
    st, summ, res = ctx.fit(db)
    svt.check(st, "fit")
    if npass_edit is not None:
        npass_edit(res.npass)
    st, lsum, lst = ctx.list_passing(db, res, capacity=capacity)
    torch.cuda.synchronize()
    return st, lsum.as_dict(), lst.numpy()


def assert_same_list(got, want, where=""):
    assert np.array_equal(got["offsets"], want["offsets"]), f"{where}offsets"
    for f in ("k", "chi2", "params"):
        a, b = np.asarray(got[f]), np.asarray(want[f])
        assert a.shape == b.shape, f"{where}{f}: shape {a.shape} vs {b.shape}"
        if not np.array_equal(a.astype(np.int64) if f != "chi2" else a,
                              b.astype(np.int64) if f != "chi2" else b):
            i = int(np.argwhere((a != b).reshape(len(a), -1).any(axis=1))[0][0])
            raise AssertionError(f"{where}{f}: first mismatch at entry {i}: got {a[i]} want {b[i]}")


CASES = {
    "small plain fit (uniform constants)": lambda: synth.cfg1(n_events=100),
    "scaled-up fit, 40 events": lambda: synth.cfg2(n_events=40),
    "uneven batches, 2000 events": lambda: synth.cfg3(n_events=2000),
    "equal roads, 4^4 combinations": lambda: synth.paper_sweep(50),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_list_matches_oracle(ctx, oracle_lib, name):
    batch, consts = CASES[name]()
    rc, want, wsum = oracle_lib.list_passing_batch(batch, consts)
    assert rc == 0
    st, summ, got = gpu_list(ctx, batch, consts)
    assert st == 0, summ
    assert_same_list(got, want, f"{name}: ")
    assert summ["total_pass"] == wsum["total_pass"] == len(want["k"])


@pytest.mark.parametrize("cut", [1 << 32, (1 << 44) - 1, (1 << 48) - 1])
def test_list_deep_layers_and_cuts(ctx, oracle_lib, cut):
    """Up to 16 hits per layer (roads of up to 65536 combinations spread over
    many 64-lane rounds) and cuts up to the largest allowed."""
    rng = np.random.default_rng(77)
    consts = synth.lattice_constants(rng, chi2_cut=cut)
    batch = synth.random_small(rng, n_events=30, max_roads=8, max_hits=16, n_sectors=72,
                               consts=consts, track_frac=0.5)
    rc, want, _ = oracle_lib.list_passing_batch(batch, consts)
    assert rc == 0
    st, summ, got = gpu_list(ctx, batch, consts)
    assert st == 0, summ
    assert_same_list(got, want, f"cut {cut}: ")


def test_list_full_scaled_up_batch(ctx, oracle_lib):
    """The 3000-event x 64-road batch the benchmark times, every entry."""
    batch, consts = synth.cfg2()
    rc, want, _ = oracle_lib.list_passing_batch(batch, consts)
    assert rc == 0
    st, summ, got = gpu_list(ctx, batch, consts)
    assert st == 0, summ
    assert_same_list(got, want, "3000 events: ")


def test_list_grid_stride(ctx, oracle_lib):
    """More roads than the grid covers in one pass (1,056,000 roads: blocks of
    the list kernel loop over groups, the tile sums over tiles), every entry."""
    batch, consts = synth.cfg2(n_events=16500)
    assert batch.n_roads > 4096 * 256
    rc, want, _ = oracle_lib.list_passing_batch(batch, consts)
    assert rc == 0
    st, summ, got = gpu_list(ctx, batch, consts)
    assert st == 0, summ
    assert_same_list(got, want, "16500 events: ")


def test_list_road_by_road_staging(ctx, oracle_lib):
    """A malformed road whose hit range is 5000 hits longer than its hits
    (the later roads' hits shifted behind them): its group of 16 roads cannot
    stage its hit range at once and stages road by road.  The malformed road
    is reported, and every other road's entries equal the oracle's list of
    the unmodified batch."""
    import torch
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=20)
    X = 37                                   # inside the group of roads 32..47
    rc, want, _ = oracle_lib.list_passing_batch(batch, consts)
    assert rc == 0
    rc, fit, _ = oracle_lib.fit_batch(batch, consts, n_threads=8)
    assert rc == 0
    cut = int(batch.hit_offsets[X + 1])
    hits = np.concatenate([batch.hits[:cut], np.zeros(5000, np.int16), batch.hits[cut:]])
    ho = batch.hit_offsets.copy()
    ho[X + 1:] += 5000
    mod = synth.Batch(road_offsets=batch.road_offsets, sector=batch.sector, nhits=batch.nhits,
                      hit_offsets=ho, hits=hits, xft=batch.xft)
    npass = fit["npass"].astype(np.int32).copy()
    npass[X] = 0
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    db = svt.to_device(mod)
    np_dev = torch.from_numpy(npass).cuda()
    lst = svt.DevicePassList(mod.n_roads, int(npass.sum()))
    st, t = svt.svt_list_passing(ctx.handle, db.struct(), np_dev.data_ptr(), lst.struct(),
                                 torch.cuda.current_stream().cuda_stream)
    svt.check(st, "svt_list_passing")
    st, summ = ctx.result(t, -1)
    assert st == svt.SVT_E_RANGE and summ.err_road == X
    got = lst.numpy()
    go, wo = got["offsets"], want["offsets"]
    assert go[X + 1] == go[X]
    for r in range(mod.n_roads):
        if r == X:
            continue
        a, b, c, d = int(go[r]), int(go[r + 1]), int(wo[r]), int(wo[r + 1])
        assert b - a == d - c, r
        for f in ("k", "chi2", "params"):
            assert np.array_equal(np.asarray(got[f])[a:b], np.asarray(want[f])[c:d]), (r, f)


def test_list_capacity(ctx, oracle_lib):
    """A list that does not fit: SVT_E_RANGE with err_road -1, complete
    offsets, and the entries that fit equal the start of the full list."""
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=20)
    rc, want, _ = oracle_lib.list_passing_batch(batch, consts)
    n = len(want["k"])
    st, summ, got = gpu_list(ctx, batch, consts, capacity=n - 11)
    assert st == svt.SVT_E_RANGE and summ["err_road"] == -1 and summ["total_pass"] == n
    assert np.array_equal(got["offsets"], want["offsets"])
    for f in ("k", "chi2", "params"):
        assert np.array_equal(np.asarray(got[f]), np.asarray(want[f])[:n - 11]), f


def test_list_pass_count_mismatch(ctx):
    """A pass count that disagrees with the road's passing combinations
    names that road (the lowest one)."""
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=20)

    def bump(npass):
        nz = (npass > 0).nonzero().flatten()
        npass[int(nz[5])] += 1
        npass[int(nz[9])] += 2
        bump.road = int(nz[5])

    st, summ, _ = gpu_list(ctx, batch, consts, npass_edit=bump)
    assert st == svt.SVT_E_RANGE and summ["err_road"] == bump.road


def test_list_negative_npass(ctx):
    """A negative pass count is reported as a bad road (the lowest one), ahead
    of a later count mismatch."""
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=20)

    def edit(npass):
        nz = (npass > 0).nonzero().flatten()
        npass[int(nz[3])] = -1
        npass[int(nz[8])] += 1
        edit.road = int(nz[3])

    st, summ, _ = gpu_list(ctx, batch, consts, npass_edit=edit, capacity=1 << 20)
    assert st == svt.SVT_E_RANGE and summ["err_road"] == edit.road


def test_list_empty_and_no_pass(ctx, oracle_lib):
    from paper_1311_0380_amd import svt
    b0 = synth.Batch(road_offsets=np.zeros(1, np.int32), sector=np.zeros(0, np.uint8),
                     nhits=np.zeros((0, 4), np.uint8), hit_offsets=np.zeros(1, np.int32),
                     hits=np.zeros(0, np.int16), xft=np.zeros((0, 2), np.int16))
    _, consts = synth.cfg2(n_events=2)
    st, summ, got = gpu_list(ctx, b0, consts)
    assert st == 0 and summ["total_pass"] == 0 and list(got["offsets"]) == [0]
    # a cut of 0 on random hits: nothing passes, nothing is evaluated again
    batch, consts = synth.cfg1(n_events=10)
    consts.chi2_cut = 0
    rc, want, _ = oracle_lib.list_passing_batch(batch, consts)
    st, summ, got = gpu_list(ctx, batch, consts)
    assert st == 0 and summ["total_comb"] == 0
    assert_same_list(got, want)


def test_list_invalid_calls(ctx):
    from paper_1311_0380_amd import svt
    import ctypes
    batch, consts = synth.cfg2(n_events=2)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    db = svt.to_device(batch)
    st, _, res = ctx.fit(db)
    lst = svt.DevicePassList(batch.n_roads, 10)
    good = lst.struct()
    bad_cap = svt.svt_pass_list(good.offsets, good.k, good.chi2, good.params, -1)
    no_off = svt.svt_pass_list(None, good.k, good.chi2, good.params, 10)
    for s in (bad_cap, no_off):
        st, _ = svt.svt_list_passing(ctx.handle, db.struct(), res.npass.data_ptr(), s)
        assert st == svt.SVT_E_INVAL
    host = db.struct()
    host.mem_kind = svt.SVT_MEM_PINNED
    st, _ = svt.svt_list_passing(ctx.handle, host, res.npass.data_ptr(), good)
    assert st == svt.SVT_E_INVAL
    st = svt.lib.svt_list_passing(None, ctypes.byref(db.struct()), None, ctypes.byref(good), None,
                                  ctypes.byref(ctypes.c_int64()))
    assert st == svt.SVT_E_INVAL
