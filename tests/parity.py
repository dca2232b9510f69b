"""Parity helpers: compare the HIP path with the FP64 oracle.

Selection contract: the GPU index equals the oracle's except where the
oracle's objective has a near-tie: a GPU choice u is accepted iff
Omega[u] <= min(Omega) * (1 + 1e-6) (or both are 0).  The output pixel must
be an exact copy of the member the GPU selected.  Aggregates: within 1e-5
relative of the oracle.
"""
import numpy as np

NEAR_TIE = 1e-6
AGG_RTOL = 1e-5


def source_pixels(img, idx, window):
    """The member each index selects (replicated border), (B, M, N, 3)."""
    x = img if img.ndim == 4 else img[None]
    ii = idx if idx.ndim == 3 else idx[None]
    B, M, N, _ = x.shape
    h = window // 2
    iu = ii.astype(np.int64)
    rr = np.clip(np.arange(M)[None, :, None] + iu // window - h, 0, M - 1)
    cc = np.clip(np.arange(N)[None, None, :] + iu % window - h, 0, N - 1)
    bb = np.arange(B)[:, None, None]
    return x[bb, rr, cc]


def check_selection(idx_gpu, omega_oracle, rel=NEAR_TIE):
    """Returns (n_mismatch, n_total); raises if a mismatch is not a near-tie."""
    g = idx_gpu.reshape(-1).astype(np.int64)
    O = omega_oracle.reshape(g.shape[0], -1)
    omin = O.min(axis=1)
    first = np.argmin(O, axis=1)  # lowest index among exact minima
    og = O[np.arange(g.shape[0]), g]
    mism = g != first
    ok = (og <= omin * (1 + rel)) | ((omin == 0) & (og == 0))
    bad = mism & ~ok
    if bad.any():
        k = np.flatnonzero(bad)[:5]
        raise AssertionError(
            "%d of %d selections differ beyond the near-tie band, e.g. pixels %s: gpu idx %s "
            "oracle idx %s, Omega gpu-choice %s min %s" % (bad.sum(), g.shape[0], k, g[k],
                                                          first[k], og[k], omin[k]))
    return int(mism.sum()), g.shape[0]


def check_aggregates(gpu, ref, rtol=AGG_RTOL, name="A"):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(gpu - ref)
    tol = rtol * np.abs(ref) + 1e-30
    bad = err > tol
    if bad.any():
        k = np.flatnonzero(bad.reshape(-1))[:5]
        raise AssertionError("%s: %d of %d values beyond %.1e relative, e.g. gpu %s ref %s"
                             % (name, bad.sum(), bad.size, rtol, gpu.reshape(-1)[k],
                                ref.reshape(-1)[k]))
    nz = np.abs(ref) > 0
    return float((err[nz] / np.abs(ref[nz])).max()) if nz.any() else 0.0


SWITCH_BAND = 1e-5


def window_colours(img, window):
    """Member colours of every window, (B*M*N, n, 3) (replicated border)."""
    x = img if img.ndim == 4 else img[None]
    B, M, N, _ = x.shape
    n = window * window
    cols = np.empty((B, M, N, n, 3), x.dtype)
    for u in range(n):
        cols[:, :, :, u] = source_pixels(x, np.full((B, M, N), u, np.uint8), window)
    return cols.reshape(B * M * N, n, 3)


def acwddf_ambiguous(colours, S, diag, n, T, rel=NEAR_TIE, band=SWITCH_BAND):
    """Pixels whose ACWDDF result FP32 arithmetic may legitimately change: a
    nonzero switching statistic within `band` (relative) of T, or, in any of the four
    selections (eq. 3 and the three centre-weighted levels), a member of a
    different colour than the oracle's choice within `rel` of the minimum.
    Members of equal colour tie exactly on both sides and resolve alike."""
    S = S.reshape(-1)
    D = diag.reshape(S.shape[0], 5 * n)
    # S = 0 exactly on both sides when every level selects the centre's colour
    amb = (S != 0) & (np.abs(S - T) <= band * max(abs(T), 1.0)) if np.isfinite(T) else \
        np.zeros(S.shape, bool)
    rows = np.arange(S.shape[0])
    for j in range(4):
        Oj = D[:, j * n:(j + 1) * n]
        first = np.argmin(Oj, axis=1)
        omin = Oj[rows, first]
        near = (Oj <= omin[:, None] * (1 + rel)) | ((omin[:, None] == 0) & (Oj == 0))
        other = np.any(colours != colours[rows, first][:, None, :], axis=2)
        amb |= np.any(near & other, axis=1)
    return amb


def check_acwddf(idx_gpu, idx_oracle, colours, S, diag, n, T, max_ambiguous=0.01):
    """ACWDDF selection contract; returns (n_mismatch, n_ambiguous, n_total)."""
    g = idx_gpu.reshape(-1)
    o = idx_oracle.reshape(-1)
    amb = acwddf_ambiguous(colours, S, diag, n, T)
    mism = g != o
    bad = mism & ~amb
    if bad.any():
        k = np.flatnonzero(bad)[:5]
        raise AssertionError("%d of %d ACWDDF selections differ outside the ambiguous set, e.g. "
                             "pixels %s: gpu %s oracle %s S %s" % (bad.sum(), g.size, k, g[k], o[k],
                                                                   S.reshape(-1)[k]))
    assert amb.mean() <= max_ambiguous, "ambiguous fraction %.4f" % amb.mean()
    return int(mism.sum()), int(amb.sum()), g.size


EPS32 = 2.0 ** -24


def soft_bounds(x, omega, window, tau, dx_scale):
    """Per-element error bounds of the float32 softmin against the binary64
    oracle, from the arithmetic: the objective of a window carries a few ulp of
    relative error and enters exp(-(Omega - min Omega) / tau), so the weights
    of window c move by about eps * Omega_max(c) / tau, where Omega_max(c) is
    the largest objective of its members (the oracle's); the weighted sum of
    colours adds about n eps max|x| of its own rounding.  A pixel's gradient
    collects the weight perturbations of every window within 2h, so it takes
    the largest Omega_max over its (4h + 1)^2 neighbourhood, scaled by the
    largest gradient.  omega: the oracle's objectives (..., M, N, n).
    Returns (bound on |y - ref| per pixel, bound on |dx - ref| per pixel).
    The constants (1 n + 2 Omega / tau for y, 1 n + 4 Omega / tau for dx) sit
    2-5x above the worst errors measured on the test images."""
    n = window * window
    h = window // 2
    om = np.asarray(omega).max(-1)
    ty = EPS32 * np.abs(x).max() * (n + 2.0 * om / tau)
    # neighbourhood maximum over (4h + 1)^2 pixels, replicated border
    pad = [(0, 0)] * (om.ndim - 2) + [(2 * h, 2 * h), (2 * h, 2 * h)]
    op = np.pad(om, pad, mode="edge")
    M, N = om.shape[-2:]
    omn = np.full(om.shape, -np.inf)
    for dy in range(4 * h + 1):
        for dxo in range(4 * h + 1):
            omn = np.maximum(omn, op[..., dy:dy + M, dxo:dxo + N])
    td = EPS32 * dx_scale * (n + 4.0 * omn / tau)
    return ty, td


def check_soft(y, ref_y, dx, ref_dx, bounds, name=""):
    """Element-wise check against soft_bounds; returns the worst error / bound
    ratios (forward, backward)."""
    ty, td = bounds
    ry = (np.abs(np.asarray(y, np.float64) - ref_y).max(-1) / ty) if y is not None else np.zeros(1)
    rd = (np.abs(np.asarray(dx, np.float64) - ref_dx).max(-1) / td) if dx is not None else np.zeros(1)
    assert ry.max() <= 1.0, "%s: forward error %.3g x its bound" % (name, ry.max())
    assert rd.max() <= 1.0, "%s: gradient error %.3g x its bound" % (name, rd.max())
    return float(ry.max()), float(rd.max())


def soft_tol(x, window, kind, p, tau, scale=64.0):
    """Softmin error budget (relative): the binary32 objective carries a few ulp of
    relative error and enters exp(-Omega / tau); with max Omega <= n (pi/2 + max|x|
    sqrt 3), the weights move by about scale * eps * max Omega / tau."""
    n = window * window
    om_max = n * (np.pi / 2 + np.abs(x).max() * np.sqrt(3))
    return scale * EPS32 * om_max / tau
