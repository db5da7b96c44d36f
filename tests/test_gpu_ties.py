"""GPU tie rule: among combinations of equal chi2 the lowest combination
index k wins (the nested-loop order of Sec. 2.1, layer 0 most significant).

Random 12-bit hits almost never give two combinations the same chi2, so the
batches here repeat hit words inside a layer on purpose: in roads with a
planted track the true word is copied to other places of its layer (several
combinations then reach chi2 = 0), and in every road some words are copied
onto others (every combination through them has a twin).  Twins share every
fit input, so they tie exactly whatever the constants.  The fit runs at a
cut below 2^44 (the fraction-encoded minimum) and above it (the general
compare-and-select), with inner-layer counts up to 4, 8 and 16 and mixed
counts in a wavefront, with the default chunks and with one event per
chunk; every field is compared with the oracle."""
import pytest

from tests.gpu_helpers import assert_equal_results, lib_fit
from tests.ties import tie_batch, twin_roads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1311_0380_amd import svt
    h = svt.svt_create(0, 0)
    yield h
    svt.svt_destroy(h)


@pytest.mark.parametrize("events_per_chunk", [0, 1])
@pytest.mark.parametrize("cut", [1 << 32, (1 << 44) + 12345])
@pytest.mark.parametrize("max_hits", [4, 8, 16])
def test_lowest_index_wins_ties(ctx, oracle_lib, events_per_chunk, cut, max_hits):
    from paper_1311_0380_amd import svt
    batch, consts = tie_batch(900 + max_hits, max_hits)
    consts.chi2_cut = cut
    rc, want, wsum = oracle_lib.fit_batch(batch, consts, n_threads=8)
    assert rc == 0
    n_twin, viol = twin_roads(batch, want["hit_index"])
    # the batch exercises the rule: many bests have a twin, and the oracle
    # always takes the lowest
    assert n_twin >= batch.n_roads // 10, n_twin
    assert viol == 0
    svt.check(svt.svt_load_constants(ctx, consts.coef, consts.offset, consts.chi2_cut))
    svt.check(svt.svt_set_tuning(ctx, events_per_chunk=events_per_chunk))
    try:
        st, summ, got = lib_fit(ctx, batch)
    finally:
        svt.check(svt.svt_set_tuning(ctx, events_per_chunk=0))
    assert st == 0, (st, summ)
    assert_equal_results(got, want,
                         where=f"events per chunk {events_per_chunk} cut {cut} max_hits {max_hits}: ")
    assert summ["total_pass"] == wsum["total_pass"]
