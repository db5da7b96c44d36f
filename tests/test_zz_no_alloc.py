"""svt_list_passing_noalloc, the list entry point that allocates nothing,
against svt_list_passing: the same offsets and entries on two calls in a
row, the second with a smaller batch (the shared scratch keeps the first
call's contents); the context allocates nothing for it; a batch above its
scratch is refused."""
import numpy as np
import pytest

from paper_1311_0380_amd import synth

pytestmark = pytest.mark.gpu


def _lists(svt, ctx, batch, consts, fn):
    import torch
    svt.check(svt.svt_load_constants(ctx, consts.coef, consts.offset, consts.chi2_cut))
    db = svt.to_device(batch)
    res = svt.DeviceResults(batch.n_events, batch.n_roads)
    stream = torch.cuda.current_stream().cuda_stream
    st, t = svt.svt_fit_events(ctx, db.struct(), res.struct(), stream)
    svt.check(st, "fit")
    svt.check(svt.svt_result(ctx, t, -1)[0], "fit result")
    cap = int(res.npass.sum().item())
    lst = svt.DevicePassList(batch.n_roads, cap)
    lst.offsets.fill_(-9)
    lst.k.fill_(-9)
    used = svt.svt_get_device_info(ctx)["used_bytes"]
    st, t = fn(ctx, db.struct(), res.npass.data_ptr(), lst.struct(), stream)
    svt.check(st, "list submit")
    st, summ = svt.svt_result(ctx, t, -1)
    svt.check(st, "list result")
    torch.cuda.synchronize()
    return summ.total_pass, lst.numpy(), svt.svt_get_device_info(ctx)["used_bytes"] - used


def test_noalloc_list_matches_list_on_two_calls():
    from paper_1311_0380_amd import svt
    big, consts = synth.cfg2(n_events=3000)
    small = big.select_events(100, 400)
    ref = svt.svt_create(0, 0)
    ctx = svt.svt_create(0, 0)
    try:
        for i, batch in enumerate((big, small)):
            n_ref, want, grew_ref = _lists(svt, ref, batch, consts, svt.svt_list_passing)
            n_got, got, grew = _lists(svt, ctx, batch, consts, svt.svt_list_passing_noalloc)
            assert n_got == n_ref and n_ref > 0, (i, n_got, n_ref)
            for f in ("offsets", "k", "chi2", "params"):
                assert np.array_equal(got[f], want[f]), (i, f)
            # the allocating call grows its context on first use; this one never
            assert grew == 0
            if i == 0:
                assert grew_ref > 0
    finally:
        svt.svt_destroy(ctx)
        svt.svt_destroy(ref)


def test_noalloc_list_refuses_batches_above_its_scratch():
    from paper_1311_0380_amd import svt
    ctx = svt.svt_create(0, 0)
    try:
        b = svt.svt_event_batch(1, (1 << 24) + 1, 0, svt.SVT_MEM_DEVICE, 8, 8, 8, 8, 8, 8)
        lst = svt.svt_pass_list(8, 8, 8, 8, 0)
        st, _ = svt.svt_list_passing_noalloc(ctx, b, 8, lst)
        assert st == svt.SVT_E_NOMEM
        assert "2^24" in svt.lib.svt_last_error().decode()
    finally:
        svt.svt_destroy(ctx)
