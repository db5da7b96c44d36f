"""Rings: resident batches fitted back to back in one captured graph.  Every
pass's results equal the oracle's for its batch, the summary sums all passes,
and the ring follows the context's state rules."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth
from tests.gpu_helpers import assert_equal_results

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_1311_0380_amd import svt
    ctx = svt.svt_create(0, 0)
    yield svt, ctx
    svt.svt_destroy(ctx)


@pytest.mark.parametrize("per_launch", [1, 3, 0, 7])
def test_ring_passes_match_the_oracle(env, oracle_lib, per_launch):
    svt, ctx = env
    import torch
    # three different batches (sizes differ, so grids differ per pass)
    batches, consts = [], None
    for i, ne in enumerate((300, 17, 1000)):
        b, c = synth.cfg2(seed=2, n_events=3000)
        b = b.select_events(ne * i, ne * i + ne)
        batches.append(b)
        consts = c
    svt.check(svt.svt_load_constants(ctx, consts.coef, consts.offset, consts.chi2_cut))
    dbs = [svt.to_device(b) for b in batches]
    drs = [svt.DeviceResults(b.n_events, b.n_roads) for b in batches]
    st, ring = svt.svt_ring_create(ctx, [d.struct() for d in dbs], [r.struct() for r in drs], 7,
                                   per_launch)
    svt.check(st, "svt_ring_create")
    try:
        n_passes, k, n_launch = svt.svt_ring_info(ring)
        assert n_passes == 7 and n_launch == (7 + k - 1) // k
        if per_launch:
            assert k == per_launch
        print(f"ring: 7 passes, {k} per launch", flush=True)
        wants, tot = [], dict(total_comb=0, total_pass=0, total_tracks=0)
        for b in batches:
            rc, w, s = oracle_lib.fit_batch(b, consts, n_threads=8)
            assert rc == 0
            wants.append(w)
        for p in range(7):
            s = oracle_lib.fit_batch(batches[p % 3], consts, n_threads=8)[2]
            for k in tot:
                tot[k] += s[k]
        for run in range(3):
            for r in drs:       # stale values must be overwritten
                for f in svt.RESULT_FIELDS:
                    getattr(r, f).fill_(-3)
            torch.cuda.synchronize()
            st, t = svt.svt_ring_run(ring, torch.cuda.current_stream().cuda_stream)
            svt.check(st, "svt_ring_run")
            st2, t2 = svt.svt_ring_run(ring, torch.cuda.current_stream().cuda_stream)
            assert st2 == svt.SVT_E_AGAIN            # one run of a ring at a time
            st, summ = svt.svt_result(ctx, t, -1)
            svt.check(st, "ring result")
            assert summ.total_comb == tot["total_comb"]
            assert summ.total_pass == tot["total_pass"]
            assert summ.total_tracks == tot["total_tracks"]
            assert summ.err_road == -1 and summ.err_event == -1
            assert summ.device_ns > 0
            for r, w in zip(drs, wants):
                assert_equal_results(r.numpy(), w, where=f"run {run}: ")
    finally:
        svt.svt_ring_destroy(ring)


def ring_case(svt, ctx, oracle_lib, batches, consts, n_passes, per_launch, runs=2):
    """Fit the batches n_passes times round-robin in one ring; every batch's
    results and the summary must equal the oracle's."""
    import torch
    svt.check(svt.svt_load_constants(ctx, consts.coef, consts.offset, consts.chi2_cut))
    dbs = [svt.to_device(b) for b in batches]
    drs = [svt.DeviceResults(b.n_events, b.n_roads) for b in batches]
    wants, sums, tot = [], [], dict(total_comb=0, total_pass=0, total_tracks=0)
    for b in batches:
        rc, w, s = oracle_lib.fit_batch(b, consts, n_threads=8)
        assert rc == 0
        wants.append(w)
        sums.append(s)
    for p in range(n_passes):
        for k in tot:
            tot[k] += sums[p % len(batches)][k]
    st, ring = svt.svt_ring_create(ctx, [d.struct() for d in dbs], [r.struct() for r in drs],
                                   n_passes, per_launch)
    svt.check(st, "svt_ring_create")
    try:
        print(f"ring: {n_passes} passes, shape {svt.svt_ring_info(ring)}", flush=True)
        for run in range(runs):
            for r in drs:
                for f in svt.RESULT_FIELDS:
                    getattr(r, f).fill_(-3)
            torch.cuda.synchronize()
            st, t = svt.svt_ring_run(ring, torch.cuda.current_stream().cuda_stream)
            svt.check(st, "svt_ring_run")
            st, summ = svt.svt_result(ctx, t, -1)
            svt.check(st, "ring result")
            assert (summ.total_comb, summ.total_pass, summ.total_tracks) == \
                (tot["total_comb"], tot["total_pass"], tot["total_tracks"])
            assert summ.err_road == -1 and summ.err_event == -1
            for i, (r, w) in enumerate(zip(drs, wants)):
                assert_equal_results(r.numpy(), w, where=f"run {run}, batch {i}: ")
    finally:
        svt.svt_ring_destroy(ring)


def shape_batches(seed=91):
    """Batches whose chunks differ in kind: runs of events without roads, one
    event of many sub-chunks, and events of ragged sizes."""
    rng = np.random.default_rng(seed)
    consts = synth.lattice_constants(rng)
    out = []
    rpe = np.zeros(600, np.int64)
    rpe[rng.choice(600, 40, replace=False)] = rng.integers(1, 30, 40)
    nr = int(rpe.sum())
    out.append(synth.make_events(rng, rpe, rng.integers(0, 5, (nr, 4)), consts.n_sectors,
                                 rng.random(nr) < 0.5, consts))
    out.append(synth.make_events(rng, [3000], rng.integers(1, 6, (3000, 4)), consts.n_sectors,
                                 rng.random(3000) < 0.5, consts))
    rpe = rng.integers(1, 80, 400)
    nr = int(rpe.sum())
    out.append(synth.make_events(rng, rpe, rng.integers(1, 5, (nr, 4)), consts.n_sectors,
                                 rng.random(nr) < 0.5, consts))
    return out, consts


@pytest.mark.parametrize("n_passes,per_launch,shape", [(128, 0, (128, 128, 1)), (130, 0, (130, 65, 2)),
                                                       (100, 128, (100, 100, 1))])
def test_ring_many_passes_per_launch(env, oracle_lib, n_passes, per_launch, shape):
    """Long launches (the automatic choice takes up to 128 passes in one):
    every batch's results and the summed totals equal the oracle's."""
    svt, ctx = env
    batches, consts = shape_batches(seed=93)
    svt.check(svt.svt_load_constants(ctx, consts.coef, consts.offset, consts.chi2_cut))
    dbs = [svt.to_device(b) for b in batches]
    drs = [svt.DeviceResults(b.n_events, b.n_roads) for b in batches]
    st, ring = svt.svt_ring_create(ctx, [d.struct() for d in dbs], [r.struct() for r in drs],
                                   n_passes, per_launch)
    svt.check(st, "svt_ring_create")
    try:
        assert svt.svt_ring_info(ring) == shape
    finally:
        svt.svt_ring_destroy(ring)
    ring_case(svt, ctx, oracle_lib, batches, consts, n_passes, per_launch, runs=1)


@pytest.mark.parametrize("n_passes,per_launch", [(3, 1), (4, 1), (5, 1), (9, 2), (8, 2)])
def test_ring_direct_and_graph_runs(env, oracle_lib, n_passes, per_launch):
    """Rings of up to four launches enqueue their kernels at each run, longer
    ones replay a captured graph: both sides of that boundary, with one-pass
    and two-pass launches, give the oracle's results and totals, run after
    run (the sequence number advances the same way in both forms)."""
    svt, ctx = env
    batches, consts = shape_batches(seed=95)
    ring_case(svt, ctx, oracle_lib, batches, consts, n_passes, per_launch, runs=3)


@pytest.mark.parametrize("n_passes", [20, 12])
def test_ring_full_batch_head_and_tail_chunks(env, oracle_lib, n_passes):
    """The 3000-event x 64-road batch and a 1000-event slice of it in one
    ring: a multi-pass launch cuts the full batch's passes into chunks of
    three times a lone pass's (the slice keeps the lone pass's) and its last
    passes (enough to fill the grid once, at most a quarter of the launch:
    four of 20, three of 12) into the lone pass's chunks, so one launch holds
    blocks of both sizes and both kinds of batch in its head and its tail.
    Every result equals the oracle's, run after run."""
    svt, ctx = env
    full, consts = synth.cfg2()
    batches = [full, full.select_events(1000, 2000)]
    print(f"full batch ring: {n_passes} passes", flush=True)
    ring_case(svt, ctx, oracle_lib, batches, consts, n_passes, 0, runs=2)


@pytest.mark.parametrize("tuning", [dict(), dict(events_per_chunk=1), dict(events_per_chunk=3, schedule=2),
                                    dict(blocks_per_cu=1), dict(events_per_chunk=256)])
@pytest.mark.parametrize("per_launch", [3, 0])
def test_ring_launch_shapes(env, oracle_lib, tuning, per_launch):
    svt, ctx = env
    batches, consts = shape_batches()
    svt.check(svt.svt_set_tuning(ctx, **tuning))
    try:
        print(f"tuning {tuning}, {per_launch} per launch", flush=True)
        ring_case(svt, ctx, oracle_lib, batches, consts, 8, per_launch)
    finally:
        svt.check(svt.svt_set_tuning(ctx, events_per_chunk=0, blocks_per_cu=0, schedule=1, kernel=0))


def test_ring_rules(env):
    svt, ctx = env
    b, c = synth.cfg1(n_events=20)
    svt.check(svt.svt_load_constants(ctx, c.coef, c.offset, c.chi2_cut))
    db, dr = svt.to_device(b), svt.DeviceResults(b.n_events, b.n_roads)
    bs, rs = db.struct(), dr.struct()
    # host buffers, comb_offsets and bad counts are refused
    hb = svt.svt_event_batch(*[getattr(bs, f) for f, _ in bs._fields_])
    hb.mem_kind = svt.SVT_MEM_PINNED
    assert svt.svt_ring_create(ctx, [hb], [rs], 2)[0] == svt.SVT_E_INVAL
    co = svt.DeviceResults(b.n_events, b.n_roads, comb_offsets=True)
    assert svt.svt_ring_create(ctx, [bs], [co.struct()], 2)[0] == svt.SVT_E_INVAL
    assert svt.svt_ring_create(ctx, [bs], [rs], 0)[0] == svt.SVT_E_INVAL
    assert svt.svt_ring_create(ctx, [bs, bs], [rs, rs], 1)[0] == svt.SVT_E_INVAL
    assert svt.svt_ring_create(ctx, [bs], [rs], 2, -1)[0] == svt.SVT_E_INVAL
    assert svt.svt_ring_create(ctx, [bs], [rs], 2, 129)[0] == svt.SVT_E_INVAL
    # the largest count is taken, and clamped to the passes there are
    st, r128 = svt.svt_ring_create(ctx, [bs], [rs], 2, 128)
    svt.check(st)
    try:
        assert svt.svt_ring_info(r128) == (2, 2, 1)
    finally:
        svt.svt_ring_destroy(r128)
    st, ring = svt.svt_ring_create(ctx, [bs], [rs], 3)
    svt.check(st)
    try:
        # constants are captured: a reload makes the ring stale
        svt.check(svt.svt_load_constants(ctx, c.coef, c.offset, c.chi2_cut))
        assert svt.svt_ring_run(ring)[0] == svt.SVT_E_STATE
    finally:
        svt.svt_ring_destroy(ring)


def test_ring_reports_malformed_roads(env, oracle_lib):
    svt, ctx = env
    b, c = synth.cfg1(n_events=30)
    b.hits[5] = 5000                      # a word out of range
    svt.check(svt.svt_load_constants(ctx, c.coef, c.offset, c.chi2_cut))
    db, dr = svt.to_device(b), svt.DeviceResults(b.n_events, b.n_roads)
    st, ring = svt.svt_ring_create(ctx, [db.struct()], [dr.struct()], 2)
    svt.check(st)
    try:
        st, t = svt.svt_ring_run(ring)
        svt.check(st)
        st, summ = svt.svt_result(ctx, t, -1)
        rc, _, ws = oracle_lib.fit_batch(b, c)
        assert st == svt.SVT_E_RANGE and rc == svt.SVT_E_RANGE
        assert summ.err_road == ws["err_road"]
    finally:
        svt.svt_ring_destroy(ring)
