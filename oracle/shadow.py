"""FP64 oracle of the float-shadow fit and its calibration -- TEST INFRASTRUCTURE.

The float shadow evaluates the same linearized fit as the integer path
(paper Sec. 2: every fit row is a scalar product of per-sector constants with
the input words plus an offset) on unquantized words, so that the constants
can be calibrated by gradient descent before they are quantized.

Loss (a reading of the calibration objective; the paper has none):
    L = (1/N) sum_t [ sum_{k<3} w_k (y_k - tau_k)^2 + sum_{k>=3} y_k^2 ]
        + lambda sum_s || C_s C_s^T - I ||_F^2
with y = A_s x_t + b_s, tau the generator's truth for the three parameter
rows, C_s the three constraint rows of sector s.  Tracks are grouped by
sector: tracks of sector s are [off[s], off[s+1]).

Plain numpy in float64; nothing here is shared with the HIP library.
"""
from __future__ import annotations

import numpy as np


def _sector_of(off: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(off.shape[0] - 1), np.diff(off))


def fit_rows(coef, offset, x, off):
    """y[t] = A_s x_t + b_s for every track (float64)."""
    s = _sector_of(off)
    A = np.asarray(coef, np.float64)[s]          # [N,6,6]
    b = np.asarray(offset, np.float64)[s]        # [N,6]
    return np.einsum("tkj,tj->tk", A, np.asarray(x, np.float64)) + b


def data_loss(coef, offset, x, tau, off, w):
    """Data term of L (the mean weighted chi2-like sum)."""
    y = fit_rows(coef, offset, x, off)
    r = y.copy()
    r[:, :3] -= np.asarray(tau, np.float64)
    wk = np.concatenate([np.asarray(w, np.float64), np.ones(3)])
    return float((wk * r * r).sum() / x.shape[0]), y


def data_grad(coef, offset, x, tau, off, w):
    """dL_data/dA [S,6,6] and dL_data/db [S,6]: (2/N) sum_t w_k r_tk x_tj."""
    n_s = off.shape[0] - 1
    y = fit_rows(coef, offset, x, off)
    r = y.copy()
    r[:, :3] -= np.asarray(tau, np.float64)
    wk = np.concatenate([np.asarray(w, np.float64), np.ones(3)])
    r *= wk
    gA = np.zeros((n_s, 6, 6))
    gb = np.zeros((n_s, 6))
    xs = np.asarray(x, np.float64)
    for s in range(n_s):
        a, e = int(off[s]), int(off[s + 1])
        gA[s] = r[a:e].T @ xs[a:e]
        gb[s] = r[a:e].sum(axis=0)
    n = x.shape[0]
    return 2.0 * gA / n, 2.0 * gb / n


def penalty(coef, lam):
    """lambda sum_s ||C C^T - I||^2 and its gradient with respect to A."""
    C = np.asarray(coef, np.float64)[:, 3:, :]               # [S,3,6]
    G = C @ np.transpose(C, (0, 2, 1)) - np.eye(3)[None]
    val = lam * float((G * G).sum())
    g = np.zeros(np.shape(coef))
    g[:, 3:, :] = 4.0 * lam * (G @ C)
    return val, g


def total_loss(coef, offset, x, tau, off, w, lam):
    d, _ = data_loss(coef, offset, x, tau, off, w)
    p, _ = penalty(coef, lam)
    return d + p


def finite_difference(coef, offset, x, tau, off, w, lam, idx, h=1e-3, which="coef"):
    """Central difference of the FP64 loss along one constant."""
    c1 = np.array(coef, np.float64)
    o1 = np.array(offset, np.float64)
    c2, o2 = c1.copy(), o1.copy()
    if which == "coef":
        c1[idx] += h
        c2[idx] -= h
    else:
        o1[idx] += h
        o2[idx] -= h
    return (total_loss(c1, o1, x, tau, off, w, lam) - total_loss(c2, o2, x, tau, off, w, lam)) / (2 * h)


def lstsq_parameter_rows(x, tau, off):
    """Closed-form optimum of the parameter rows: per-sector least squares of
    the truth on [x, 1]."""
    n_s = off.shape[0] - 1
    F = np.zeros((n_s, 3, 6))
    f = np.zeros((n_s, 3))
    for s in range(n_s):
        a, e = int(off[s]), int(off[s + 1])
        X = np.hstack([np.asarray(x[a:e], np.float64), np.ones((e - a, 1))])
        sol, *_ = np.linalg.lstsq(X, np.asarray(tau[a:e], np.float64), rcond=None)
        F[s] = sol[:6].T
        f[s] = sol[6]
    return F, f


def constraint_optimum(x, off, lam):
    """Closed-form optimum of the constraint rows: rows along the three
    smallest-variance directions of the sector's inputs, with squared norms
    1 - (N_s/N) e_i / (2 lambda) (e_i the eigenvalues of the sector's
    population covariance; the data term averages over all N tracks), and
    offsets that centre them on the sector mean.  Returns, per sector,
    (e_i, eigenvectors, mean, N_s/N)."""
    n_s = off.shape[0] - 1
    n = int(off[-1])
    out = []
    for s in range(n_s):
        a, e = int(off[s]), int(off[s + 1])
        xs = np.asarray(x[a:e], np.float64)
        mu = xs.mean(axis=0)
        cov = (xs - mu).T @ (xs - mu) / (e - a)
        evals, evecs = np.linalg.eigh(cov)
        out.append((evals[:3], evecs[:, :3], mu, (e - a) / n))
    return out


def requantize(coef, offset, max_abs=1024, bound=(1 << 31) - 1, word_max=4095):
    """Integer constants from float ones: per sector the largest shift S
    (-30..30) such that every |rint(A 2^S)| < max_abs and every row keeps
    sum_j |A_int| word_max + |b_int| <= bound; rint is round-half-to-even."""
    coef = np.asarray(coef, np.float32)
    offset = np.asarray(offset, np.float32)
    n_s = coef.shape[0]
    ci = np.zeros((n_s, 6, 6), np.int64)
    oi = np.zeros((n_s, 6), np.int64)
    sh = np.zeros(n_s, np.int64)
    for s in range(n_s):
        for S in range(30, -31, -1):
            a = np.rint(coef[s].astype(np.float64) * 2.0 ** S)
            b = np.rint(offset[s].astype(np.float64) * 2.0 ** S)
            if np.abs(a).max() >= max_abs:
                continue
            if np.any(np.abs(a).sum(axis=1) * word_max + np.abs(b) > bound):
                continue
            ci[s], oi[s], sh[s] = a, b, S
            break
        else:
            raise ValueError(f"sector {s}: no shift fits")
    return ci.astype(np.int32), oi.astype(np.int32), sh.astype(np.int32)
