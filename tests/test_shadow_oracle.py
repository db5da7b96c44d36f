"""Pins for the FP64 float-shadow oracle: finite differences, closed-form
optima (least squares for the parameter rows, eigenvectors for the
constraint rows), the zero-constant special case, and requantization worked
by hand."""
import numpy as np
import pytest

from oracle import shadow as osh
from paper_1311_0380_amd import synth


@pytest.fixture(scope="module")
def tracks():
    g = synth.HelixGeometry(n_sectors=4)
    return synth.helix_tracks(6000, seed=41, geom=g)


def random_constants(rng, n_s):
    coef = rng.normal(0, 0.05, (n_s, 6, 6))
    off = rng.normal(0, 50.0, (n_s, 6))
    return coef, off


def test_gradient_matches_central_differences(tracks):
    rng = np.random.default_rng(1)
    coef, off = random_constants(rng, 4)
    w = (1.0 / 400, 1.0 / 1e4, 1.0)
    lam = 3.0
    gA, gb = osh.data_grad(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, w)
    _, pA = osh.penalty(coef, lam)
    gA = gA + pA
    for idx in [(0, 0, 0), (1, 2, 5), (2, 3, 1), (3, 5, 4), (0, 4, 2)]:
        fd = osh.finite_difference(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, w,
                                   lam, idx, h=1e-4)
        assert abs(fd - gA[idx]) <= 1e-6 * max(1.0, abs(gA[idx])), (idx, fd, gA[idx])
    for idx in [(0, 0), (2, 4), (3, 5)]:
        fd = osh.finite_difference(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, w,
                                   lam, idx, h=1e-3, which="offset")
        assert abs(fd - gb[idx]) <= 1e-6 * max(1.0, abs(gb[idx])), (idx, fd, gb[idx])


def test_zero_constants_special_case(tracks):
    """A = 0, b = 0: y = 0, loss = mean weighted tau^2, db = -(2/N) sum w tau."""
    n_s = 4
    coef = np.zeros((n_s, 6, 6))
    off = np.zeros((n_s, 6))
    w = (0.5, 0.25, 2.0)
    loss, y = osh.data_loss(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, w)
    assert np.all(y == 0)
    want = float((np.array(w) * tracks.truth ** 2).sum() / len(tracks.x))
    assert abs(loss - want) <= 1e-12 * want
    _, gb = osh.data_grad(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, w)
    for s in range(n_s):
        a, e = tracks.sector_offsets[s], tracks.sector_offsets[s + 1]
        want_b = -2.0 * np.array(w) * tracks.truth[a:e].sum(axis=0) / len(tracks.x)
        assert np.allclose(gb[s, :3], want_b, rtol=1e-12, atol=0)
        assert np.all(gb[s, 3:] == 0)


def test_parameter_rows_optimum_is_least_squares(tracks):
    """At the per-sector least-squares solution the parameter-row gradient
    vanishes (normal equations)."""
    F, f = osh.lstsq_parameter_rows(tracks.x, tracks.truth, tracks.sector_offsets)
    coef = np.zeros((4, 6, 6))
    off = np.zeros((4, 6))
    coef[:, :3] = F
    off[:, :3] = f
    gA, gb = osh.data_grad(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, (1, 1, 1))
    scale = np.abs(tracks.x).max() * np.abs(tracks.truth).max()
    assert np.abs(gA[:, :3]).max() < 1e-8 * scale
    assert np.abs(gb[:, :3]).max() < 1e-8 * np.abs(tracks.truth).max()


def test_constraint_rows_optimum_is_eigenvectors(tracks):
    """Rows along the 3 smallest-variance directions with squared norms
    1 - (N_s/N) e/(2 lambda), centred on the mean, zero the full gradient."""
    lam = 50.0
    coef = np.zeros((4, 6, 6))
    off = np.zeros((4, 6))
    for s, (ev, V, mu, frac) in enumerate(osh.constraint_optimum(tracks.x, tracks.sector_offsets,
                                                                   lam)):
        d = np.sqrt(1.0 - frac * ev / (2 * lam))
        coef[s, 3:] = (V * d).T
        off[s, 3:] = -coef[s, 3:] @ mu
    gA, gb = osh.data_grad(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, (0, 0, 0))
    _, pA = osh.penalty(coef, lam)
    g = gA + pA
    assert np.abs(g[:, 3:]).max() < 1e-7
    assert np.abs(gb[:, 3:]).max() < 1e-7
    # and it is a minimum along a random direction
    base = osh.total_loss(coef, off, tracks.x, tracks.truth, tracks.sector_offsets, (0, 0, 0), lam)
    rng = np.random.default_rng(3)
    for _ in range(3):
        dA = np.zeros_like(coef)
        dA[:, 3:] = rng.normal(0, 1e-3, (4, 3, 6))
        moved = osh.total_loss(coef + dA, off, tracks.x, tracks.truth, tracks.sector_offsets,
                               (0, 0, 0), lam)
        assert moved >= base


def test_requantize_worked_example():
    """Sector 0: max |A| = 3.3 -> largest S with |rint(A 2^S)| < 1024 is 8
    (3.3 * 256 = 844.8 -> 845; 3.3 * 512 = 1689.6 is too big).  Ties round to
    even: 0.5 * 2^S with S = 8 is exact (128), and 2.5 / 2^8 -> 2.5 exactly
    with S = 0 in sector 1 (max |A| = 640.0 -> S = 0; 2.5 -> 2, 3.5 -> 4)."""
    coef = np.zeros((2, 6, 6), np.float32)
    off = np.zeros((2, 6), np.float32)
    coef[0, 0, 0] = 3.3
    coef[0, 1, 2] = -0.5
    off[0, 3] = 7.25
    coef[1, 2, 2] = 640.0
    coef[1, 0, 1] = 2.5
    coef[1, 0, 2] = 3.5
    off[1, 0] = -1.5
    ci, oi, sh = osh.requantize(coef, off)
    assert list(sh) == [8, 0]
    assert ci[0, 0, 0] == 845 and ci[0, 1, 2] == -128 and oi[0, 3] == 7.25 * 256
    assert ci[1, 2, 2] == 640 and ci[1, 0, 1] == 2 and ci[1, 0, 2] == 4 and oi[1, 0] == -2


def test_requantize_respects_bound():
    """Large offsets force a smaller shift than the coefficient limit alone."""
    coef = np.full((1, 6, 6), 0.9, np.float32)
    off = np.full((1, 6), 3.0e6, np.float32)
    ci, oi, sh = osh.requantize(coef, off)
    assert np.abs(ci).max() < 1024
    assert np.all(np.abs(ci[0]).sum(axis=1) * 4095 + np.abs(oi[0]) <= (1 << 31) - 1)
    # without the offsets the shift would be 10 (0.9 * 1024 = 921.6 -> 922)
    ci2, oi2, sh2 = osh.requantize(coef, np.zeros((1, 6), np.float32))
    assert sh2[0] == 10 and sh[0] < 10
