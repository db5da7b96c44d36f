"""GPU float shadow: fp32 kernels against the FP64 oracle within the stated
tolerance, the hand-written backward against the FP64 gradient, the autograd
wrapper, requantization bit for bit, calibration to its closed-form endpoint,
and rescoring on the integer path.

The forward / backward / autograd parity runs at 120k helix tracks (one slice
per sector), at the calibration workload's full 1e6 tracks (seven slices per
sector, so the per-sector reductions across slices are compared) and on a
skewed batch whose largest sector holds 400k tracks (the slice count clamps
at 64 and sectors split unevenly, down to slices of zero or one track)."""
import numpy as np
import pytest

from oracle import shadow as osh
from paper_1311_0380_amd import synth

pytestmark = pytest.mark.gpu

W = (1.0 / 400.0, 1.0 / 1.0e4, 1.0)


class _Tracks:
    """Tracks grouped by sector, in the generator's layout."""

    def __init__(self, x, truth, sector_offsets):
        self.x, self.truth, self.sector_offsets = x, truth, sector_offsets


def _skewed(seed=46):
    """Three sectors of 400k, 7 and 300k tracks: 235,669 tracks per sector on
    average, so the slice count clamps at 64; the 7-track sector gets slices
    of zero or one track.  Words uniform in [0, 4096), truth a linear map of
    them plus noise."""
    rng = np.random.default_rng(seed)
    ns = [400000, 7, 300000]
    x = rng.uniform(0, 4096, (sum(ns), 6)).astype(np.float32)
    F = rng.normal(0, 1e-2, (3, 6))
    tau = (x.astype(np.float64) @ F.T + rng.normal(0, 1.0, (x.shape[0], 3))).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    return _Tracks(x, tau, off)


def _constants(h, seed=5):
    coef, off = synth.pilot_constants(h) if hasattr(h, "xq") else _pilot_plain(h)
    rng = np.random.default_rng(seed)
    # a point away from the optimum: residuals are large, as early in a calibration
    coef = (coef * (1 + rng.normal(0, 0.02, coef.shape))).astype(np.float32)
    off = (off + rng.normal(0, 5.0, off.shape)).astype(np.float32)
    return coef, off


def _pilot_plain(h):
    n_s = h.sector_offsets.shape[0] - 1
    rng = np.random.default_rng(3)
    coef = rng.normal(0, 0.3, (n_s, 6, 6)).astype(np.float32)
    off = rng.normal(0, 50.0, (n_s, 6)).astype(np.float32)
    return coef, off


@pytest.fixture(scope="module", params=["helix120k", "helix1e6", "skewed"])
def env(request):
    import torch
    from paper_1311_0380_amd import shadow, svt
    if request.param == "helix120k":
        h = synth.helix_tracks(120000, seed=44)
    elif request.param == "helix1e6":
        h = synth.helix_tracks(1000000, seed=44)
    else:
        h = _skewed()
    coef, off = _constants(h)
    handle = svt.svt_create(0, 0)
    tr = shadow.ShadowTracks(x=torch.tensor(h.x, dtype=torch.float32, device="cuda"),
                             tau=torch.tensor(h.truth, dtype=torch.float32, device="cuda"),
                             sector_offsets=torch.tensor(h.sector_offsets, dtype=torch.int32,
                                                         device="cuda"), w=W)
    n_s = len(h.sector_offsets) - 1
    print(f"\nshadow case {request.param}: {h.x.shape[0]} tracks, {n_s} sectors, "
          f"{svt.shadow_slices(h.x.shape[0], n_s)} slices per sector", flush=True)
    yield dict(name=request.param, h=h, coef=coef, off=off, handle=handle, tracks=tr,
               torch=torch, shadow=shadow)
    svt.svt_destroy(handle)


def dev(env, a):
    return env["torch"].tensor(a, device="cuda")


def test_slice_counts_cover_the_reduction_paths(env):
    from paper_1311_0380_amd import svt
    h = env["h"]
    n_s = len(h.sector_offsets) - 1
    want = {"helix120k": 1, "helix1e6": 7, "skewed": 64}[env["name"]]
    assert svt.shadow_slices(h.x.shape[0], n_s) == want


def test_forward_rows_and_loss(env):
    h, coef, off = env["h"], env["coef"], env["off"]
    loss, y = env["shadow"].forward(env["handle"], env["tracks"], dev(env, coef), dev(env, off),
                                    want_y=True)
    y = y.cpu().numpy().astype(np.float64)
    xs = h.x.astype(np.float32)
    want_loss, want_y = osh.data_loss(coef, off, xs, h.truth.astype(np.float32),
                                      h.sector_offsets, W)
    # |y - y*| <= 1e-6 * max(|y*|, S), S = sum_j |A_kj x_j| + |b_k|
    s = np.repeat(np.arange(len(h.sector_offsets) - 1), np.diff(h.sector_offsets))
    S = np.einsum("tkj,tj->tk", np.abs(coef.astype(np.float64))[s], np.abs(xs.astype(np.float64))) \
        + np.abs(off.astype(np.float64))[s]
    err = np.abs(y - want_y) / np.maximum(np.abs(want_y), S)
    assert err.max() <= 1e-6, err.max()
    assert abs(loss.item() - want_loss) <= 1e-6 * want_loss


def test_backward_matches_fp64_gradient(env):
    h, coef, off = env["h"], env["coef"], env["off"]
    g64, o64, g32, o32 = env["shadow"].backward(env["handle"], env["tracks"], dev(env, coef),
                                                dev(env, off))
    gA, gb = osh.data_grad(coef, off, h.x.astype(np.float32), h.truth.astype(np.float32),
                           h.sector_offsets, W)
    assert np.abs(g64.cpu().numpy() - gA).max() <= 1e-6 * np.abs(gA).max()
    assert np.abs(o64.cpu().numpy() - gb).max() <= 1e-6 * np.abs(gb).max()
    assert np.array_equal(g32.cpu().numpy(), g64.cpu().numpy().astype(np.float32))
    # bit-reproducible
    g64b, o64b, _, _ = env["shadow"].backward(env["handle"], env["tracks"], dev(env, coef),
                                              dev(env, off))
    assert env["torch"].equal(g64, g64b) and env["torch"].equal(o64, o64b)


def test_penalty(env):
    torch = env["torch"]
    coef = env["coef"]
    lam = 7.0
    g = torch.zeros((coef.shape[0], 6, 6), dtype=torch.float64, device="cuda")
    val = env["shadow"].penalty(env["handle"], dev(env, coef), lam, g)
    want_v, want_g = osh.penalty(coef, lam)
    assert abs(val.item() - want_v) <= 1e-9 * max(1.0, want_v)
    assert np.abs(g.cpu().numpy() - want_g).max() <= 1e-9 * max(1.0, np.abs(want_g).max())


def test_autograd_function_and_finite_differences(env):
    torch = env["torch"]
    h, coef, off = env["h"], env["coef"], env["off"]
    A = dev(env, coef).requires_grad_(True)
    b = dev(env, off).requires_grad_(True)
    L = env["shadow"].SVTShadowFit.apply(A, b, env["handle"], env["tracks"]) * 3.0
    L.backward()
    gA, gb = osh.data_grad(coef, off, h.x.astype(np.float32), h.truth.astype(np.float32),
                           h.sector_offsets, W)
    assert np.abs(A.grad.cpu().numpy() - 3.0 * gA).max() <= 2e-6 * np.abs(3.0 * gA).max()
    assert np.abs(b.grad.cpu().numpy() - 3.0 * gb).max() <= 2e-6 * np.abs(3.0 * gb).max()
    if env["name"] != "helix120k":
        return
    # the FP64 gradient it matches is itself checked by central differences
    for idx in [(3, 0, 0), (10, 4, 2)]:
        fd = osh.finite_difference(coef, off, h.x.astype(np.float32), h.truth.astype(np.float32),
                                   h.sector_offsets, W, 0.0, idx, h=1e-3)
        assert abs(fd - gA[idx]) <= 1e-6 * max(1.0, abs(gA[idx]))


def test_requantize_bit_exact(env):
    coef, off = env["coef"], env["off"]
    ci, oi, sh, status = env["shadow"].requantize(env["handle"], dev(env, coef), dev(env, off))
    wci, woi, wsh = osh.requantize(coef, off)
    assert status.item() == 0
    assert np.array_equal(sh.cpu().numpy(), wsh)
    assert np.array_equal(ci.cpu().numpy(), wci)
    assert np.array_equal(oi.cpu().numpy(), woi)


def test_calibration_reduces_loss_and_rescore(env, oracle_lib):
    if env["name"] != "helix120k":
        pytest.skip("one calibration and rescore run suffices (helix120k)")
    from paper_1311_0380_amd import svt
    h = env["h"]
    coef, off = synth.pilot_constants(h)
    res = env["shadow"].calibrate(env["handle"], env["tracks"], dev(env, coef), dev(env, off),
                                  steps=60, lr=2e-3, lam=10.0, record_every=20)
    losses = [l for _, l, _ in res.history]
    assert all(np.isfinite(l) and l >= 0 for l in losses)
    start, _ = osh.data_loss(coef, off, h.x.astype(np.float32), h.truth.astype(np.float32),
                             h.sector_offsets, W)
    assert losses[-1] < start
    # requantize and rescore the quantized words on the integer path: one
    # road per track with one hit per layer
    ci, oi, sh, status = env["shadow"].requantize(env["handle"], res.coef, res.offset)
    assert status.item() == 0
    ci, oi = ci.cpu().numpy(), oi.cpu().numpy()
    n = 20000
    xq = h.xq[:n].astype(np.int16)
    b = synth.Batch(road_offsets=np.arange(n + 1, dtype=np.int32),
                    sector=h.sector[:n].astype(np.uint8),
                    nhits=np.ones((n, 4), np.uint8),
                    hit_offsets=(np.arange(n + 1) * 4).astype(np.int32),
                    hits=xq[:, :4].reshape(-1).copy(), xft=xq[:, 4:6].copy())
    cut = (1 << 48) - 1
    svt.check(svt.svt_load_constants(env["handle"], ci, oi, cut))
    from tests.gpu_helpers import assert_equal_results, lib_fit
    st, summ, got = lib_fit(env["handle"], b)
    assert st == 0
    rc, want, _ = oracle_lib.fit_batch(b, synth.Constants(ci, oi, cut))
    assert rc == 0
    assert_equal_results(got, want)


def _endpoint_workload(seed=11):
    """Three sectors of 3000, 5000 and 8000 tracks with well-separated input
    variances (0.05 ... 4 along a random rotation) and truth a linear map of
    the inputs plus N(0, 0.01) noise: a calibration that Adam drives to its
    closed-form optimum in a few thousand steps."""
    rng = np.random.default_rng(seed)
    ns = [3000, 5000, 8000]
    F = rng.normal(0, 1, (3, 3, 6))
    f = rng.normal(0, 1, (3, 3))
    xs, ts = [], []
    for s in range(3):
        q, _ = np.linalg.qr(rng.normal(size=(6, 6)))
        L = q * np.sqrt([0.05, 0.1, 0.2, 1.0, 2.0, 4.0])
        x = rng.normal(0, 0.5, 6) + rng.normal(size=(ns[s], 6)) @ L.T
        xs.append(x)
        ts.append(x @ F[s].T + f[s] + rng.normal(0, 0.01, (ns[s], 3)))
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    coef0 = rng.normal(0, 0.3, (3, 6, 6)).astype(np.float32)
    off0 = rng.normal(0, 0.3, (3, 6)).astype(np.float32)
    return (np.vstack(xs).astype(np.float32), np.vstack(ts).astype(np.float32), off,
            coef0, off0)


def test_calibration_reaches_closed_form_endpoint():
    """Adam in the library's kernels (backward, penalty, Adam step) converges
    to the optimum the oracle gives in closed form: the parameter rows to the
    per-sector least-squares fit of the truth on [x, 1]
    (osh.lstsq_parameter_rows) and the constraint rows to the span of the
    three smallest-variance directions with squared norms
    1 - (N_s/N) e_i / (2 lambda) (osh.constraint_optimum).  The constraint
    rows are unique only up to a rotation inside that span, so C^T C (6x6)
    and the offsets -C mu are compared."""
    import torch
    from paper_1311_0380_amd import shadow, svt
    x, tau, off, coef0, off0 = _endpoint_workload()
    lam = 10.0
    handle = svt.svt_create(0, 0)
    try:
        tr = shadow.ShadowTracks(x=torch.tensor(x, device="cuda"), tau=torch.tensor(tau, device="cuda"),
                                 sector_offsets=torch.tensor(off, device="cuda"), w=(1.0, 1.0, 1.0))
        c, o = torch.tensor(coef0, device="cuda"), torch.tensor(off0, device="cuda")
        for lr, steps in ((1e-2, 1500), (1e-3, 1000), (1e-4, 1000)):
            res = shadow.calibrate(handle, tr, c, o, steps=steps, lr=lr, lam=lam, record_every=steps)
            c, o = res.coef, res.offset
        torch.cuda.synchronize()
    finally:
        svt.svt_destroy(handle)
    c = c.cpu().numpy().astype(np.float64)
    o = o.cpu().numpy().astype(np.float64)
    F, f = osh.lstsq_parameter_rows(x, tau, off)
    assert np.abs(c[:, :3] - F).max() <= 1e-4, np.abs(c[:, :3] - F).max()
    assert np.abs(o[:, :3] - f).max() <= 1e-4, np.abs(o[:, :3] - f).max()
    for s, (e, V, mu, frac) in enumerate(osh.constraint_optimum(x, off, lam)):
        C = c[s, 3:]
        want = (V * (1.0 - frac * e / (2.0 * lam))) @ V.T
        assert np.abs(C.T @ C - want).max() <= 1e-4, (s, np.abs(C.T @ C - want).max())
        assert np.abs(o[s, 3:] + C @ mu).max() <= 1e-4, (s, np.abs(o[s, 3:] + C @ mu).max())


def test_default_stream_ordering():
    """Library calls on torch's default stream (handle 0) are ordered with
    torch's own work on it: a copy issued right after the backward sees the
    finished gradient, at a size where the backward takes tens of µs."""
    import torch
    from paper_1311_0380_amd import shadow, svt
    h = synth.helix_tracks(1000000, seed=45)
    coef, off = synth.pilot_constants(h)
    handle = svt.svt_create(0, 0)
    try:
        tr = shadow.ShadowTracks.from_helix(h, W)
        A, b = torch.tensor(coef, device="cuda"), torch.tensor(off, device="cuda")
        assert torch.cuda.current_stream().cuda_stream == 0
        for _ in range(3):
            g64, o64, _, _ = shadow.backward(handle, tr, A, b)
            early = torch.cat([g64.reshape(-1), o64.reshape(-1)]).clone()
            loss, _ = shadow.forward(handle, tr, A, b)
            early_loss = loss.item()
            torch.cuda.synchronize()
            late = torch.cat([g64.reshape(-1), o64.reshape(-1)])
            assert torch.equal(early, late)
            assert np.isfinite(early_loss) and early_loss == loss.item() and early_loss >= 0
    finally:
        svt.svt_destroy(handle)
