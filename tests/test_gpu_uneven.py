"""Uneven batching: the graph-captured persistent plan and the per-event
launch baseline give the oracle's results bit for bit, across replays of one
graph with batches of different sizes (checked after every replay, with eager
fits in between)."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth
from tests.gpu_helpers import FIELDS, assert_equal_results, lib_fit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1311_0380_amd import svt, uneven
    batch, consts = synth.cfg3()
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    yield dict(batch=batch, consts=consts, ctx=ctx, svt=svt, uneven=uneven, torch=torch)
    ctx.close()


def plan_fit(env, plan, batch):
    svt = env["svt"]
    db = svt.to_device(batch)
    dr = svt.DeviceResults(batch.n_events, batch.n_roads)
    st, summ = plan.fit(db.struct(), dr.struct())
    return st, summ, dr.numpy()


def test_plan_replays_match_oracle(env, oracle_lib):
    svt, uneven = env["svt"], env["uneven"]
    batch, consts = env["batch"], env["consts"]
    plan = uneven.Plan(env["ctx"], batch.n_events, batch.n_roads, batch.n_hits)
    try:
        for e0, e1 in ((0, batch.n_events), (0, 2000), (3000, 3500), (0, 1), (0, batch.n_events)):
            sub = batch.select_events(e0, e1)
            st, summ, got = plan_fit(env, plan, sub)
            assert st == 0, (e0, e1, st)
            rc, want, wsum = oracle_lib.fit_batch(sub, consts, n_threads=8)
            assert rc == 0
            assert_equal_results(got, want, where=f"replay [{e0},{e1}): ")
            assert summ.total_comb == wsum["total_comb"]
            # eager work between replays
            st2, _, eager = lib_fit(env["ctx"].handle, sub)
            assert st2 == 0
            assert_equal_results(eager, want, where="eager: ")
    finally:
        plan.close()


def test_plan_in_place_buffers(env, oracle_lib):
    svt, uneven = env["svt"], env["uneven"]
    sub = env["batch"].select_events(100, 1300)
    plan = uneven.Plan(env["ctx"], 2000, 40000, 300000)
    try:
        st, _, first = plan_fit(env, plan, sub)
        assert st == 0
        # the inputs are now in the plan's buffers: fit them in place, results in place
        inb, outb = plan.inb, plan.outb
        inb.n_events, inb.n_roads, inb.n_hits = sub.n_events, sub.n_roads, sub.n_hits
        st, summ = plan.fit(inb, outb)
        assert st == 0
        import torch
        # read the in-place results through a copy into torch buffers
        dr = svt.DeviceResults(sub.n_events, sub.n_roads)
        st, summ2 = plan.fit(inb, dr.struct())
        assert st == 0
        assert_equal_results(dr.numpy(), first)
    finally:
        plan.close()


def test_plan_untimed_replays(env, oracle_lib):
    """Plan replays that svt_set_timing leaves untimed report device_ns 0
    and the same bits; timed ones a device time."""
    uneven = env["uneven"]
    ctx = env["ctx"]
    sub = env["batch"].select_events(0, 1500)
    rc, want, _ = oracle_lib.fit_batch(sub, env["consts"], n_threads=8)
    assert rc == 0
    plan = uneven.Plan(ctx, sub.n_events, sub.n_roads, sub.n_hits)
    try:
        for every, timed in ((0, False), (1, True)):
            ctx.set_timing(every)
            for _ in range(2):
                st, summ, got = plan_fit(env, plan, sub)
                assert st == 0
                assert_equal_results(got, want, where=f"timing {every}: ")
                assert (summ.device_ns > 0) == timed
    finally:
        ctx.set_timing(1)
        plan.close()


def test_plan_errors(env):
    svt, uneven = env["svt"], env["uneven"]
    batch, consts = env["batch"], env["consts"]
    plan = uneven.Plan(env["ctx"], 10, 400, 4000)
    try:
        big = batch.select_events(0, 20)
        db = svt.to_device(big)
        dr = svt.DeviceResults(big.n_events, big.n_roads)
        st, _ = svt.svt_plan_fit(plan.handle, db.struct(), dr.struct())
        assert st == svt.SVT_E_INVAL            # above capacity
        env["ctx"].load_constants(consts.coef, consts.offset, consts.chi2_cut)
        small = batch.select_events(0, 3)
        db = svt.to_device(small)
        dr = svt.DeviceResults(small.n_events, small.n_roads)
        st, _ = svt.svt_plan_fit(plan.handle, db.struct(), dr.struct())
        assert st == svt.SVT_E_STATE            # constants changed since capture
    finally:
        plan.close()


def test_per_event_baseline_matches_batched(env, oracle_lib):
    uneven = env["uneven"]
    sub = env["batch"].select_events(0, 1500)
    per = uneven.PerEventBatches(sub)
    wall, dev_ns, done = per.run(env["ctx"])
    assert np.all(dev_ns > 0) and np.all(np.diff(done) >= -1e-9)
    rc, want, _ = oracle_lib.fit_batch(sub, env["consts"], n_threads=8)
    assert rc == 0
    assert_equal_results(per.res.numpy(), want, where="per-event: ")


def test_autotune_choice_gives_same_bits(env, oracle_lib, tmp_path, monkeypatch):
    svt, uneven = env["svt"], env["uneven"]
    monkeypatch.setattr(uneven, "CACHE_PATH", str(tmp_path / "tune.json"))
    sub = env["batch"].select_events(0, 3000)
    db = svt.to_device(sub)
    dr = svt.DeviceResults(sub.n_events, sub.n_roads)
    best, table = uneven.autotune(env["ctx"], db, dr, reps=3)
    assert len(table) >= 4 and all(t > 0 for _, t in table)
    plan = uneven.Plan(env["ctx"], sub.n_events, sub.n_roads, sub.n_hits, best)
    try:
        st, _, got = plan_fit(env, plan, sub)
        assert st == 0
        rc, want, _ = oracle_lib.fit_batch(sub, env["consts"], n_threads=8)
        assert_equal_results(got, want)
    finally:
        plan.close()
    # the cache answers the second call
    best2, _ = uneven.autotune(env["ctx"], db, dr, reps=3)
    assert best2 == best
