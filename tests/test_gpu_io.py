"""Transfer study on the GPU: the probe reports plausible times for every
memory kind and direction, and round trips through pageable, pinned and
mapped buffers return the same results as the device-resident fit."""
import numpy as np
import pytest

from tests.gpu_helpers import assert_equal_results

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1311_0380_amd import svt, synth
    assert torch.cuda.is_available()
    batch, consts = synth.cfg2(n_events=200)
    ctx = svt.Context(0)
    ctx.load_constants(consts.coef, consts.offset, consts.chi2_cut)
    yield dict(ctx=ctx, batch=batch, consts=consts, svt=svt)
    ctx.close()


def test_probe_all_kinds(env):
    svt = env["svt"]
    for kind in (svt.SVT_MEM_PAGEABLE, svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED):
        for direction in (0, 1):
            small = svt.svt_io_probe(env["ctx"].handle, kind, direction, 4096, 5)
            big = svt.svt_io_probe(env["ctx"].handle, kind, direction, 16 << 20, 5)
            assert 0 < small < 1e5
            assert big > small
            # 16 MB in under 100 ms: more than 0.16 GB/s on any path
            assert big < 1e5


def test_probe_rejects_bad_arguments(env):
    svt = env["svt"]
    h = env["ctx"].handle
    for kind, direction, n, reps in ((svt.SVT_MEM_DEVICE, 0, 4096, 3), (7, 0, 4096, 3),
                                     (svt.SVT_MEM_PINNED, 2, 4096, 3),
                                     (svt.SVT_MEM_PINNED, 0, 0, 3),
                                     (svt.SVT_MEM_PINNED, 0, 4096, 0)):
        with pytest.raises(svt.SVTError):
            svt.svt_io_probe(h, kind, direction, n, reps)


def test_round_trip_rows_and_results(env):
    from paper_1311_0380_amd import iostudy
    svt = env["svt"]
    rows = iostudy.round_trip(env["ctx"], env["batch"], event_counts=(1, 50, 200), reps=2)
    assert len(rows) == 9
    for r in rows:
        assert r["round_trip_us"] > 0 and r["fit_us"] > 0
        assert 0.0 <= r["transfer_share"] <= 1.0
    # the host-memory requests produce the device-resident answer
    batch = env["batch"]
    dr = iostudy._results(batch.n_events, batch.n_roads, svt.SVT_MEM_DEVICE)
    db = svt.to_device(batch)
    st, want = env["ctx"].result(env["ctx"].submit(db.struct(), dr.struct()), -1)
    assert st == 0
    want_np = dr.numpy()
    for kind in (svt.SVT_MEM_PAGEABLE, svt.SVT_MEM_PINNED, svt.SVT_MEM_MAPPED):
        host = iostudy._host_copy(batch, kind)
        b = svt.svt_event_batch(batch.n_events, batch.n_roads, batch.n_hits, kind,
                                *[host[f].data_ptr() for f in svt.BATCH_FIELDS])
        res = iostudy._results(batch.n_events, batch.n_roads, kind)
        st, got = env["ctx"].result(env["ctx"].submit(b, res.struct()), -1)
        assert st == 0
        assert got.total_comb == want.total_comb and got.total_pass == want.total_pass
        got_np = res.numpy()
        for k in want_np:
            np.testing.assert_array_equal(got_np[k], want_np[k], err_msg=f"{k} kind={kind}")


def test_transfer_sweep_shape(env):
    from paper_1311_0380_amd import iostudy
    rows = iostudy.transfer_sweep(env["ctx"], sizes=(4096, 1 << 20), reps=3)
    assert len(rows) == 3 * 2 * 2
    assert all(r["gbs"] > 0 for r in rows)
