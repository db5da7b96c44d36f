"""Serving loop on the GPU: each burst's results in the merged launches equal
the same burst fitted alone (bit-exact); a small device-memory budget still
serves every burst; the per-event baseline matches the oracle."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth
from tests.gpu_helpers import FIELDS, assert_equal_results, lib_fit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    from paper_1311_0380_amd import serve, svt
    batch, consts = synth.cfg2(seed=12, n_events=1500)
    yield dict(batch=batch, consts=consts, serve=serve, svt=svt)


def make_ctx(env, budget=0):
    ctx = env["svt"].Context(0, budget)
    c = env["consts"]
    ctx.load_constants(c.coef, c.offset, c.chi2_cut)
    return ctx


def test_alone_equals_in_mix(env, oracle_lib):
    """Every burst served in merged launches equals the same burst fitted
    alone by the library, and equals the oracle's results for its events
    (one oracle run over the pool, sliced: roads and events are fitted
    independently, so a burst's results are the slice of the pool's)."""
    serve = env["serve"]
    batch = env["batch"]
    rc, want_all, _ = oracle_lib.fit_batch(batch, env["consts"], n_threads=8)
    assert rc == 0
    ctx = make_ctx(env)
    try:
        pool = serve.HostPool(batch)
        dev = serve.LibraryDevice(ctx, 3)
        srv = serve.Server(dev, pool, n_slots=3, max_events=4000, keep_results=True)
        rng = np.random.default_rng(4)
        arr = serve.make_arrivals(rng, 80, 2e5, pool.batch.n_events, max_events=600)
        recs = srv.run(arr)
        assert len(recs) == 80 and all(r.done > 0 for r in recs)
        assert len(set(r.launch for r in recs)) < 80       # some bursts were merged
        for r in recs:
            alone = batch.select_events(r.e0, r.e1)
            st, _, got = lib_fit(ctx.handle, alone)
            assert st == 0
            assert_equal_results(srv.results[r.idx], got, where=f"burst {r.idx} vs alone: ")
            r0, r1 = int(batch.road_offsets[r.e0]), int(batch.road_offsets[r.e1])
            want = {f: (v[r.e0:r.e1] if f == "ntracks" else v[r0:r1]) for f, v in want_all.items()
                    if f in FIELDS}
            assert_equal_results(srv.results[r.idx], want, where=f"burst {r.idx} vs oracle: ")
    finally:
        ctx.close()


def test_small_budget_admission(env):
    serve = env["serve"]
    # room for a few launches of ~300 events next to the context's own scratch
    ctx = make_ctx(env, budget=(8 << 20) + (24 << 20))
    try:
        pool = serve.HostPool(env["batch"])
        dev = serve.LibraryDevice(ctx, 4)
        srv = serve.Server(dev, pool, n_slots=4, max_events=1200, keep_results=False)
        arr = [(0.0, 300 * (i % 4), 300 * (i % 4) + 300) for i in range(12)]
        recs = srv.run(arr)
        assert len(recs) == 12 and all(r.done > 0 for r in recs)
        assert ctx.device_info()["used_bytes"] <= (8 << 20) + (24 << 20)
    finally:
        ctx.close()


def test_plain_per_event_matches_oracle(env, oracle_lib):
    serve = env["serve"]
    ctx = make_ctx(env)
    try:
        pool = serve.HostPool(env["batch"])
        plain = serve.PlainServer(ctx, pool, window=16)
        arr = [(0.0, 0, 40), (0.0005, 100, 130)]
        recs = plain.run(arr)
        assert len(recs) == 2 and all(r.done > r.arrival for r in recs)
        sub = env["batch"].select_events(100, 130)
        rc, want, _ = oracle_lib.fit_batch(sub, env["consts"])
        r0, r1 = int(env["batch"].road_offsets[100]), int(env["batch"].road_offsets[130])
        got = {k: v.numpy()[r0:r1] for k, v in plain.res.items() if k != "ntracks"}
        got["chi2"] = got["chi2"].view(np.uint64)
        got["ntracks"] = plain.res["ntracks"].numpy()[100:130]
        assert_equal_results(got, want)
    finally:
        ctx.close()
