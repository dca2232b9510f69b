"""Pins of the oracle's ACWDDF (Section III, Experiment 2: the switching rule
and the centre weights of eq. 9) against closed forms and properties the
definition fixes, independent of the oracle's own code path."""
import math

import numpy as np
import pytest

import oracle
from oracle import DDF, EXACT, MINIMAX, RGB


def _theta_l2(a, b):
    """Angle (acos of the normalised dot product, well conditioned at the
    angles used here) and Euclidean distance of two colours."""
    a, b = np.asarray(a, float), np.asarray(b, float)
    cos = float(a @ b) / math.sqrt(float(a @ a) * float(b @ b))
    return math.acos(cos), math.sqrt(float((a - b) @ (a - b)))


def _impulse_window(w, bg, imp):
    x = np.empty((w, w, 3), np.float64)
    x[:] = bg
    x[w // 2, w // 2] = imp
    return x


@pytest.mark.parametrize("w", [3, 5])
@pytest.mark.parametrize("bg,imp", [((100, 100, 100), (100, 100, 140)),
                                    ((30, 200, 90), (220, 10, 40)),
                                    ((12, 40, 7), (13, 40, 7))])
def test_lone_impulse_closed_form(w, bg, imp):
    """Background colour a everywhere but the centre b.  With the weights of
    eq. (9), at level k the centre member's objective is ((n-1) th)((n-1) L)
    and every background member's is (w_d th)(w_d L), w_d = n - 2k + 2; the
    eq. (3) objectives are (n-1)^2 th L and th L."""
    n = w * w
    d = (n - 1) // 2
    th, L = _theta_l2(bg, imp)
    x = _impulse_window(w, bg, imp)
    pix = [d]  # the centre pixel of the w x w image
    for lam in (1, 2, 3):
        _, _, S, dg = oracle.acwddf_at(x, pix, window=w, dist=EXACT, lam=lam, T=0.0)
        dg = dg[0]
        assert dg[d] == pytest.approx((n - 1) ** 2 * th * L, rel=1e-12)
        assert dg[0] == pytest.approx(th * L, rel=1e-12)
        for j in range(3):
            k = lam + j
            wd = n - 2 * k + 2
            cw = dg[(1 + j) * n:(2 + j) * n]
            assert cw[d] == pytest.approx((n - 1) ** 2 * th * L, rel=1e-12)
            assert cw[0] == pytest.approx(wd * wd * th * L, rel=1e-12)
        # A(x_u, x_d) L2(x_u, x_d): th L for the background, 0 for the centre
        assert dg[4 * n] == pytest.approx(th * L, rel=1e-12) and dg[4 * n + d] == 0.0
        # k = 1 keeps the impulse (w_d = n > n - 1); k >= 2 picks the background
        picks_centre = sum(1 for j in range(3) if lam + j == 1)
        assert S[0] == pytest.approx((3 - picks_centre) * th * L, rel=1e-12)


@pytest.mark.parametrize("w", [3, 5])
def test_lone_impulse_switch_threshold(w):
    """lambda = 2: S = 3 th L; the DDF output (the background member u = 0)
    when S > T, the centre (the impulse) otherwise."""
    bg, imp = (100, 100, 100), (100, 100, 140)
    th, L = _theta_l2(bg, imp)
    S_expect = 3 * th * L
    x = _impulse_window(w, bg, imp)
    d = (w * w - 1) // 2
    out, idx, S, _ = oracle.acwddf_at(x, [d], window=w, lam=2, T=0.5 * S_expect)
    assert idx[0] == 0 and tuple(out[0]) == bg and S[0] == pytest.approx(S_expect, rel=1e-12)
    out, idx, S, _ = oracle.acwddf_at(x, [d], window=w, lam=2, T=2.0 * S_expect)
    assert idx[0] == d and tuple(out[0]) == imp


@pytest.mark.parametrize("w", [3, 5])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_level_d_is_eq3(w, dist):
    """At k = d every weight of eq. (9) is 1: the third centre-weighted
    objective with lambda = d - 2 is the eq. (3) objective, bitwise."""
    n = w * w
    lam = (n + 1) // 2 - 2
    x = np.random.default_rng(5).integers(0, 256, (7, 9, 3))
    _, _, _, dg = oracle.acwddf(x, window=w, dist=dist, lam=lam, diag=True)
    assert np.array_equal(dg[..., 3 * n:4 * n], dg[..., 0:n])
    # and levels below d are not eq. (3)
    assert not np.array_equal(dg[..., n:2 * n], dg[..., 0:n])


@pytest.mark.parametrize("w", [3, 5])
@pytest.mark.parametrize("dist", [EXACT, RGB])
def test_level1_keeps_centre_colour(w, dist):
    """k = 1 puts weight n on the centre.  The angle and the chromaticity
    distance are metrics on directions and L2 is a metric, so by the triangle
    inequality the centre's weighted sums are no larger than any member's:
    CWDDF^1 returns the centre's colour (random colours, so no window is
    entirely collinear)."""
    n = w * w
    rng = np.random.default_rng(17)
    x = rng.integers(0, 256, (12, 14, 3)).astype(np.float64)
    M, N = x.shape[:2]
    _, _, _, dg = oracle.acwddf(x, window=w, dist=dist, lam=1, diag=True)
    sel = np.argmin(dg[..., n:2 * n], axis=-1)
    h = w // 2
    for r in range(M):
        for c in range(N):
            u = sel[r, c]
            src = x[min(max(r + u // w - h, 0), M - 1), min(max(c + u % w - h, 0), N - 1)]
            assert np.array_equal(src, x[r, c]), (r, c, u)


@pytest.mark.parametrize("w", [3, 5])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_switch_extremes(w, dist):
    """T below every S: the output is the eq. (3) selection (lowest index of
    the smallest product), which is also the DDF of p = 1/2 up to near-ties.
    T = +inf: the centre everywhere."""
    n = w * w
    x = np.random.default_rng(23).integers(0, 256, (10, 11, 3))
    out, idx, S, dg = oracle.acwddf(x, window=w, dist=dist, T=-1.0, diag=True)
    assert (S >= 0).all()
    assert np.array_equal(idx, np.argmin(dg[..., :n], axis=-1))
    _, ddf_idx, _, _, om = oracle.filter(x, window=w, kind=DDF, p=0.5, dist=dist, aggregates=True)
    diff = idx != ddf_idx
    # a differing pick must be a tie of the plain DDF objective
    sel_om = np.take_along_axis(om, idx[..., None].astype(np.int64), -1)[..., 0]
    assert np.all(sel_om[diff] <= om.min(-1)[diff] * (1 + 1e-12))
    _, idx_inf, _ = oracle.acwddf(x, window=w, dist=dist, T=math.inf)
    assert (idx_inf == (n - 1) // 2).all()


def test_constant_image_keeps_centre():
    x = np.full((6, 7, 3), 77.0)
    out, idx, S = oracle.acwddf(x)
    assert (S == 0).all() and (idx == 4).all() and np.array_equal(out, x)


def test_channel_permutation_invariant():
    x = np.random.default_rng(29).integers(0, 256, (9, 10, 3))
    _, i0, S0 = oracle.acwddf(x, T=10.8)
    _, i1, S1 = oracle.acwddf(x[..., [2, 0, 1]], T=10.8)
    assert np.array_equal(i0, i1) and np.array_equal(S0, S1)


def test_at_matches_full_and_rejects():
    x = np.random.default_rng(31).integers(0, 256, (2, 8, 9, 3))
    out, idx, S, dg = oracle.acwddf(x, window=5, dist=RGB, lam=3, T=5.0, diag=True)
    pix = np.array([0, 5, 71, 72, 143])
    o2, i2, S2, d2 = oracle.acwddf_at(x, pix, window=5, dist=RGB, lam=3, T=5.0)
    assert np.array_equal(o2, out.reshape(-1, 3)[pix]) and np.array_equal(i2, idx.ravel()[pix])
    assert np.array_equal(S2, S.ravel()[pix]) and np.array_equal(d2, dg.reshape(-1, 125)[pix])
    for bad in (dict(lam=0), dict(lam=4), dict(T=math.nan), dict(window=17), dict(window=10)):
        kw = dict(window=3, lam=2, T=1.0)
        kw.update(bad)
        with pytest.raises(ValueError):
            oracle.acwddf(x, **kw)


@pytest.mark.parametrize("w,lam", [(3, 1), (3, 2), (5, 4), (11, 2), (15, 100)])
def test_statistic_sums_the_three_levels(w, lam):
    """S is the sum, over the levels lambda .. lambda + 2 only (their columns
    are pinned by the closed forms above), of A(y_k, x_d) L2(y_k, x_d) at each
    level's selection; the eq. (3) selection does not enter it."""
    n = w * w
    x = np.random.default_rng(37).integers(0, 256, (9, 12, 3))
    _, _, S, dg = oracle.acwddf(x, window=w, lam=lam, diag=True)
    cen = dg[..., 4 * n:5 * n]
    expect = np.zeros(S.shape)
    for j in (1, 2, 3):
        sel = np.argmin(dg[..., j * n:(j + 1) * n], axis=-1)
        expect += np.take_along_axis(cen, sel[..., None], -1)[..., 0]
    assert np.allclose(S, expect, rtol=1e-14, atol=0)
    sel0 = np.argmin(dg[..., :n], axis=-1)
    with_ddf = expect - np.take_along_axis(cen, np.argmin(dg[..., 3 * n:4 * n], -1)[..., None],
                                           -1)[..., 0] + np.take_along_axis(cen, sel0[..., None],
                                                                             -1)[..., 0]
    assert not np.allclose(S, with_ddf, rtol=1e-14, atol=0)


@pytest.mark.parametrize("w", [11, 15])
def test_large_windows_reduce_to_the_plain_filters(w):
    """Past 9 x 9 as below: T < 0 switches every window to the eq. (3)
    selection, which is DDF with p = 1/2 (its objective the square root of the
    product); T = +inf keeps every centre."""
    x = np.random.default_rng(w).integers(0, 256, (9, 11, 3))
    n = w * w
    _, i_neg, _, dg = oracle.acwddf(x, window=w, dist=EXACT, lam=2, T=-1.0, diag=True)
    _, i_ddf, A, D, _ = oracle.filter(x, w, DDF, 0.5, EXACT, 4, aggregates=True)
    assert np.allclose(dg[..., :n], A * D, rtol=1e-12)
    assert np.array_equal(i_neg, i_ddf)
    _, i_inf, _ = oracle.acwddf(x, window=w, dist=EXACT, lam=2, T=math.inf)
    assert np.all(i_inf == (n - 1) // 2)
