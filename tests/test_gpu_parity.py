"""GPU parity: the HIP library against the CPU oracle, bit-exact on every
field (indices, counts, fit words, chi2), through the C ABI."""
import json
import os

import numpy as np
import pytest

from paper_1311_0380_amd import synth
from tests.gpu_helpers import FIELDS, assert_equal_results, lib_fit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1311_0380_amd import svt
    h = svt.svt_create(0, 0)
    yield h
    svt.svt_destroy(h)


def load(ctx, consts):
    from paper_1311_0380_amd import svt
    svt.check(svt.svt_load_constants(ctx, consts.coef, consts.offset, consts.chi2_cut))


def oracle_run(oracle_lib, batch, consts, **kw):
    rc, out, summ = oracle_lib.fit_batch(batch, consts, n_threads=8, **kw)
    assert rc == 0
    return out, summ


def check_case(ctx, oracle_lib, batch, consts, where="", **kw):
    load(ctx, consts)
    want, wsum = oracle_run(oracle_lib, batch, consts)
    st, summ, got = lib_fit(ctx, batch, **kw)
    assert st == 0, (where, st, summ)
    assert_equal_results(got, want, where=where)
    assert summ["total_comb"] == wsum["total_comb"]
    assert summ["total_pass"] == wsum["total_pass"]
    assert summ["total_tracks"] == wsum["total_tracks"]
    return got, summ


def test_small_plain_fit(ctx, oracle_lib):
    batch, consts = synth.cfg1()
    check_case(ctx, oracle_lib, batch, consts, "cfg1: ")


@pytest.mark.parametrize("n_events", [1, 7, 300])
def test_lattice_fit_subsets(ctx, oracle_lib, n_events):
    batch, consts = synth.cfg2(n_events=n_events)
    check_case(ctx, oracle_lib, batch, consts, f"cfg2[{n_events}]: ")


def test_scaled_up_full_size(ctx, oracle_lib):
    """3000 events x 64 roads, in the launch shape the benchmark times."""
    batch, consts = synth.cfg2()
    got, summ = check_case(ctx, oracle_lib, batch, consts, "cfg2 full: ")
    # planted tracks come back exactly
    tr = batch.track_road
    assert np.all(got["chi2"][tr] == 0)
    assert np.array_equal(got["params"][tr].astype(np.int64),
                          synth.RECOVERY_SCALE * batch.track_theta[tr])


def test_uneven_full_size(ctx, oracle_lib):
    batch, consts = synth.cfg3()
    check_case(ctx, oracle_lib, batch, consts, "cfg3 full: ")


@pytest.mark.parametrize("n_events", [1, 100, 3000])
def test_paper_sweep_shape(ctx, oracle_lib, n_events):
    batch, consts = synth.paper_sweep(n_events)
    check_case(ctx, oracle_lib, batch, consts, f"sweep[{n_events}]: ")


@pytest.mark.parametrize("name", ["plainfit_uniform_12ev", "plainfit_lattice_6ev", "uneven_20ev"])
def test_golden(ctx, name):
    from tests.golden.make_golden import make
    with open(os.path.join(os.path.dirname(__file__), "golden", name + ".json")) as f:
        doc = json.load(f)
    batch, consts = make(doc["inputs"])
    load(ctx, consts)
    st, summ, got = lib_fit(ctx, batch, comb_offsets=True)
    assert st == 0
    want = {k: np.array(v, dtype=np.uint64 if k == "chi2" else np.int64)
            for k, v in doc["results"].items()}
    assert_equal_results(got, want, fields=FIELDS + ("comb_offsets",))
    assert summ["total_comb"] == doc["summary"]["total_comb"]


@pytest.mark.parametrize("seed", range(6))
def test_irregular_small_batches(ctx, oracle_lib, seed):
    """Empty events, empty layers, up to 16 hits per layer, random cuts."""
    rng = np.random.default_rng(500 + seed)
    consts = synth.lattice_constants(rng, n_sectors=int(rng.integers(1, 73)))
    consts.chi2_cut = int(rng.choice([0, 1 << 20, 1 << 32, 1 << 38, (1 << 48) - 1]))
    batch = synth.random_small(rng, n_events=int(rng.integers(1, 400)), max_roads=12,
                               max_hits=int(rng.choice([3, 6, 16])), n_sectors=consts.n_sectors,
                               consts=consts, track_frac=0.5)
    check_case(ctx, oracle_lib, batch, consts, f"irregular[{seed}]: ", comb_offsets=True)


def test_maximum_roads(ctx, oracle_lib):
    """Roads with 16 hits in every layer (65536 combinations, 64 hits, 256
    rows) next to tiny ones, across sub-chunk capacity limits."""
    rng = np.random.default_rng(77)
    consts = synth.lattice_constants(rng)
    consts.chi2_cut = (1 << 48) - 1
    nh = rng.integers(1, 5, (600, 4))
    nh[::37] = 16
    nh[5:9] = [[16, 16, 1, 1], [1, 1, 16, 16], [16, 1, 16, 1], [0, 16, 16, 16]]
    rpe = np.full(30, 20)
    batch = synth.make_events(rng, rpe, nh, consts.n_sectors)
    check_case(ctx, oracle_lib, batch, consts, "max roads: ")


def test_one_giant_event(ctx, oracle_lib):
    """A single event with many roads (one work item spanning many sub-chunks)."""
    rng = np.random.default_rng(78)
    consts = synth.lattice_constants(rng)
    nh = rng.integers(1, 6, (5000, 4))
    batch = synth.make_events(rng, [5000], nh, consts.n_sectors,
                              rng.random(5000) < 0.5, consts)
    check_case(ctx, oracle_lib, batch, consts, "giant event: ")


def test_empty_inputs(ctx, oracle_lib):
    from paper_1311_0380_amd import svt
    consts = synth.lattice_constants(np.random.default_rng(1))
    load(ctx, consts)
    # events but no roads
    b = synth.Batch(road_offsets=np.zeros(5, np.int32), sector=np.zeros(0, np.uint8),
                    nhits=np.zeros((0, 4), np.uint8), hit_offsets=np.zeros(1, np.int32),
                    hits=np.zeros(0, np.int16), xft=np.zeros((0, 2), np.int16))
    st, summ, got = lib_fit(ctx, b)
    assert st == 0 and list(got["ntracks"]) == [0] * 4 and summ["total_comb"] == 0
    # no events at all
    b0 = synth.Batch(road_offsets=np.zeros(1, np.int32), sector=np.zeros(0, np.uint8),
                     nhits=np.zeros((0, 4), np.uint8), hit_offsets=np.zeros(1, np.int32),
                     hits=np.zeros(0, np.int16), xft=np.zeros((0, 2), np.int16))
    st, summ, got = lib_fit(ctx, b0, comb_offsets=True)
    assert st == 0 and summ["total_comb"] == 0 and list(got["comb_offsets"]) == [0]


def restore_tuning(ctx):
    from paper_1311_0380_amd import svt
    svt.check(svt.svt_set_tuning(ctx, events_per_chunk=0, blocks_per_cu=0, schedule=1, kernel=0))


def test_only_the_block_kernel(ctx):
    from paper_1311_0380_amd import svt
    assert svt.svt_set_tuning(ctx, kernel=2) == svt.SVT_E_INVAL
    assert svt.svt_set_tuning(ctx, kernel=-1) == svt.SVT_E_INVAL
    svt.check(svt.svt_set_tuning(ctx, kernel=1))
    restore_tuning(ctx)


@pytest.mark.parametrize("tuning", [
    dict(kernel=1), dict(kernel=1, events_per_chunk=1), dict(kernel=1, events_per_chunk=7),
    dict(kernel=1, events_per_chunk=256), dict(kernel=1, blocks_per_cu=1, schedule=1),
    dict(kernel=1, blocks_per_cu=3, schedule=1), dict(kernel=1, blocks_per_cu=8, schedule=2),
    dict(kernel=1, events_per_chunk=3, schedule=2),
    # balanced by roads: each block's event range split into chunks of E
    dict(kernel=1, schedule=3), dict(kernel=1, schedule=3, events_per_chunk=1),
    dict(kernel=1, schedule=3, events_per_chunk=5, blocks_per_cu=1),
    dict(kernel=1, schedule=3, blocks_per_cu=16)])
def test_launch_shapes_same_bits(ctx, oracle_lib, tuning):
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg3(n_events=2000)
    try:
        svt.check(svt.svt_set_tuning(ctx, **tuning))
        check_case(ctx, oracle_lib, batch, consts, f"{tuning}: ")
    finally:
        restore_tuning(ctx)


@pytest.mark.parametrize("schedule", [1, 3])
@pytest.mark.parametrize("cut", [1 << 32, (1 << 44) - 1, 1 << 44, (1 << 48) - 1])
def test_cut_forms_and_deep_layers(ctx, oracle_lib, schedule, cut):
    """Up to 16 hits per layer (every inner trip count 1..16, rows of up to
    256 combinations per (i0, i1)), cuts on both sides of 2^44 (where the
    kernel switches between the fraction-encoded minimum and the general
    compare-and-select form) and at the largest allowed value."""
    from paper_1311_0380_amd import svt
    rng = np.random.default_rng(44 + schedule)
    consts = synth.lattice_constants(rng, chi2_cut=cut)
    batch = synth.random_small(rng, n_events=40, max_roads=10, max_hits=16, n_sectors=72,
                               consts=consts, track_frac=0.5)
    try:
        svt.check(svt.svt_set_tuning(ctx, schedule=schedule))
        got, summ = check_case(ctx, oracle_lib, batch, consts, f"schedule {schedule} cut {cut}: ")
        assert summ["total_pass"] > 0
    finally:
        restore_tuning(ctx)


@pytest.mark.parametrize("kinds", [(0, 0), (1, 1), (2, 2), (1, 3), (3, 1), (2, 3)])
def test_memory_kinds(ctx, oracle_lib, kinds):
    batch, consts = synth.cfg2(n_events=64)
    check_case(ctx, oracle_lib, batch, consts, f"kinds {kinds}: ", mem_kind=kinds[0],
               res_kind=kinds[1], comb_offsets=True)


def test_repeatable_bits(ctx):
    batch, consts = synth.cfg3(n_events=1500)
    load(ctx, consts)
    _, s1, a = lib_fit(ctx, batch)
    _, s2, b = lib_fit(ctx, batch)
    assert_equal_results(a, b)
    assert s1["total_pass"] == s2["total_pass"]


@pytest.mark.parametrize("kinds", [(3, 3), (1, 1)])
def test_sampled_timing(ctx, kinds):
    """svt_set_timing: untimed requests (only their completion recorded)
    report device_ns 0 and the same bits, timed ones a device time; a
    negative setting is refused."""
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=64)
    load(ctx, consts)
    _, s0, want = lib_fit(ctx, batch, *kinds)
    assert s0["device_ns"] > 0
    try:
        for every in (3, 0):
            svt.check(svt.svt_set_timing(ctx, every))
            seen = set()
            for _ in range(6):
                st, s, got = lib_fit(ctx, batch, *kinds)
                assert st == 0
                assert_equal_results(got, want)
                assert s["total_pass"] == s0["total_pass"]
                seen.add(s["device_ns"] > 0)
            assert seen == ({True, False} if every == 3 else {False})
        assert svt.svt_set_timing(ctx, -1) == svt.SVT_E_INVAL
    finally:
        svt.check(svt.svt_set_timing(ctx, 1))


# ---------------------------------------------------------------------------
# malformed data: same status and offending road / event as the oracle
# ---------------------------------------------------------------------------
def _copy(b):
    return synth.Batch(**{f: getattr(b, f).copy() for f in
                          ("road_offsets", "sector", "nhits", "hit_offsets", "hits", "xft")})


CORRUPT = {
    "sector": lambda b: b.sector.__setitem__(700, 200),
    "nhits>16": lambda b: b.nhits.__setitem__((650, 1), 40),
    "nhits_sum": lambda b: b.nhits.__setitem__((610, 0), b.nhits[610, 0] + 1),
    "hit_value": lambda b: b.hits.__setitem__(int(b.hit_offsets[820]) + 2, 5000),
    "hit_negative": lambda b: b.hits.__setitem__(int(b.hit_offsets[1500]), -3),
    "xft": lambda b: b.xft.__setitem__((900, 0), -1),
    "two_bad": lambda b: (b.sector.__setitem__(1900, 99), b.xft.__setitem__((1200, 1), 4096)),
    "first_offset": lambda b: (b.hit_offsets.__setitem__(0, 1)),
    "last_offset": lambda b: (b.hit_offsets.__setitem__(-1, b.hit_offsets[-1] - 1)),
}


@pytest.mark.parametrize("name", sorted(CORRUPT))
def test_range_errors_match_oracle(ctx, oracle_lib, name):
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=40)
    bad = _copy(batch)
    CORRUPT[name](bad)
    rc, _, wsum = oracle_lib.fit_batch(bad, consts)
    assert rc == svt.SVT_E_RANGE
    load(ctx, consts)
    st, summ, _ = lib_fit(ctx, bad)
    assert st == svt.SVT_E_RANGE
    assert summ["err_road"] == wsum["err_road"]
    assert summ["err_event"] == wsum["err_event"] == -1


@pytest.mark.parametrize("schedule", [1, 3])
def test_event_offset_errors(ctx, oracle_lib, schedule):
    """Malformed event offsets give the oracle's status and lowest bad
    event, also when the schedule partitions events by searching them."""
    from paper_1311_0380_amd import svt
    batch, consts = synth.cfg2(n_events=40)
    load(ctx, consts)
    mutations = (lambda b: b.road_offsets.__setitem__(5, b.road_offsets[6] + 3),
                 lambda b: b.road_offsets.__setitem__(-1, b.road_offsets[-1] - 2),
                 lambda b: b.road_offsets.__setitem__(0, 1),
                 lambda b: b.road_offsets.__setitem__(20, b.road_offsets[3]),
                 lambda b: b.road_offsets.__setitem__(30, 10 ** 6))
    try:
        svt.check(svt.svt_set_tuning(ctx, kernel=1, schedule=schedule, blocks_per_cu=4))
        for mutate in mutations:
            bad = _copy(batch)
            mutate(bad)
            rc, _, wsum = oracle_lib.fit_batch(bad, consts)
            assert rc == svt.SVT_E_RANGE
            st, summ, _ = lib_fit(ctx, bad)
            assert st == svt.SVT_E_RANGE
            assert summ["err_event"] == wsum["err_event"]
    finally:
        restore_tuning(ctx)


def test_invalid_calls(ctx):
    from paper_1311_0380_amd import svt
    import ctypes
    b = svt.svt_event_batch(1, 0, 5, 3, None, None, None, None, None, None)
    r = svt.svt_results()
    st, _ = svt.svt_fit_events(ctx, b, r)
    assert st == svt.SVT_E_INVAL
    b = svt.svt_event_batch(1, 1, 0, 9, 1, 1, 1, 1, 1, 1)
    st, _ = svt.svt_fit_events(ctx, b, r)
    assert st == svt.SVT_E_INVAL
    st, _ = svt.svt_result(ctx, 123456, 0)
    assert st == svt.SVT_E_INVAL
    coef = np.zeros((2, 6, 6), np.int32)
    coef[0, 0, 0] = 1 << 20
    assert svt.svt_load_constants(ctx, coef, np.zeros((2, 6), np.int32), 1) == svt.SVT_E_RANGE
    assert svt.svt_load_constants(ctx, np.zeros((2, 6, 6), np.int32), np.zeros((2, 6), np.int32),
                                  1 << 48) == svt.SVT_E_RANGE
    h = ctypes.c_void_p()
    assert svt.lib.svt_create(ctypes.byref(h), 99, 0) == svt.SVT_E_INVAL


def test_state_and_budget():
    from paper_1311_0380_amd import svt
    h = svt.svt_create(0, 0)
    try:
        batch, consts = synth.cfg1(n_events=4)
        st, _, _ = lib_fit(h, batch)
        assert st == svt.SVT_E_STATE          # no constants yet
    finally:
        svt.svt_destroy(h)
    # a budget too small for the staging buffers of a pinned request (the
    # context's own scratch takes ~8.5 MB of it)
    h = svt.svt_create(0, 12 << 20)
    try:
        batch, consts = synth.cfg2(n_events=3000)
        svt.check(svt.svt_load_constants(h, consts.coef, consts.offset, consts.chi2_cut))
        st, _, _ = lib_fit(h, batch, mem_kind=svt.SVT_MEM_PINNED, res_kind=svt.SVT_MEM_PINNED)
        assert st == svt.SVT_E_NOMEM
        small, _ = synth.cfg2(n_events=10)
        st, _, _ = lib_fit(h, small, mem_kind=svt.SVT_MEM_PINNED, res_kind=svt.SVT_MEM_PINNED)
        assert st == svt.SVT_OK
    finally:
        svt.svt_destroy(h)
