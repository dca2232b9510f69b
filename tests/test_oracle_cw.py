"""Pins of the oracle's centre-weighted filters (Section III, eq. 9): CWVMF^k,
the weighted L2 sum of eq. (9), and CWDDF^k, the same weights on both sums of
eq. (3).  Checked against closed forms, the unweighted filters they reduce to
at k = d, and the triangle inequality at k = 1 -- not against the oracle's own
arithmetic."""
import math

import numpy as np
import pytest

import oracle
from oracle import BVDF, DDF, EXACT, MINIMAX, RGB
from paper_1009_0958_amd import synth


def _l2(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return math.sqrt(float((a - b) @ (a - b)))


def _angle(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return math.acos(float(a @ b) / math.sqrt(float(a @ a) * float(b @ b)))


@pytest.mark.parametrize("w", [3, 5, 11])
@pytest.mark.parametrize("vmf", [True, False])
def test_lone_impulse_closed_form(w, vmf):
    """A w x w image of colour a with colour b at one pixel: the objectives of
    the window centred on the image centre in closed form, for every level
    (11 x 11: the first two, a middle one and the last)."""
    n = w * w
    d = (n - 1) // 2
    a, b = (30, 200, 90), (220, 10, 40)
    L, th = _l2(a, b), _angle(a, b)
    for where in (d, 0):  # the impulse at the centre, then in a corner
        x = np.empty((w, w, 3))
        x[:] = a
        x[where // w, where % w] = b
        levels = range(1, (n + 1) // 2 + 1) if w <= 5 else (1, 2, 30, (n + 1) // 2)
        for k in levels:
            wd = n - 2 * k + 2
            _, idx, obj = oracle.cwfilter(x, w, vmf, EXACT, 4, k)
            o = obj[w // 2, w // 2]
            f = (lambda s_th, s_l: s_l) if vmf else (lambda s_th, s_l: s_th * s_l)
            if where == d:
                # impulse: n - 1 background members of weight 1; background
                # members: the impulse (the centre) with weight w_d
                assert o[d] == pytest.approx(f((n - 1) * th, (n - 1) * L), rel=1e-12)
                assert o[0] == pytest.approx(f(wd * th, wd * L), rel=1e-12)
                # the impulse stays only at k = 1 (w_d = n > n - 1)
                assert idx[w // 2, w // 2] == (d if k == 1 else 0)
            else:
                # impulse in the corner: the weighted centre is background
                assert o[where] == pytest.approx(f((n - 2 + wd) * th, (n - 2 + wd) * L),
                                                 rel=1e-12)
                assert o[d] == pytest.approx(f(th, L), rel=1e-12)
                assert idx[w // 2, w // 2] == (1 if where == 0 else 0)


@pytest.mark.parametrize("w", [3, 5, 11, 15])
def test_level_d_is_the_unweighted_filter(w):
    """At k = d every weight is 1: CWVMF^d is the vector median (DDF p = 1) and
    CWDDF^d the product of eq. (3) (DDF p = 1/2, whose objective is its square
    root)."""
    x = synth.image_corr(14, 17, 0.2, key=w)
    d = (w * w + 1) // 2
    for dist in (EXACT, MINIMAX, RGB):
        _, i_v, o_v = oracle.cwfilter(x, w, True, dist, 4, d)
        _, i_1, _, D1, O1 = oracle.filter(x, w, DDF, 1.0, dist, 4, aggregates=True)
        assert np.allclose(o_v, D1, rtol=1e-12)
        assert np.array_equal(i_v, i_1)
        _, i_p, o_p = oracle.cwfilter(x, w, False, dist, 4, d)
        _, i_h, A, D, Oh = oracle.filter(x, w, DDF, 0.5, dist, 4, aggregates=True)
        assert np.allclose(o_p, A * D, rtol=1e-12)
        assert np.allclose(np.sqrt(o_p), Oh, rtol=1e-12)


@pytest.mark.parametrize("w", [3, 5, 13])
@pytest.mark.parametrize("vmf", [True, False])
def test_level_1_keeps_the_centre_colour(w, vmf):
    """k = 1 weighs the centre by n: by the triangle inequality of L2 (and of
    the angle, the chromaticity distance and its eq. 10 image, for CWDDF) no
    member of another colour can beat the centre."""
    x = synth.image_uncorr(20, 23, 0.3, key=9)
    for dist in ((EXACT, RGB) if not vmf else (EXACT,)):
        out, _, _ = oracle.cwfilter(x, w, vmf, dist, 4, 1)
        assert np.array_equal(out, x.astype(float))


def test_levels_match_the_acwddf_levels():
    """CWDDF^k equals the level-k objective the ACWDDF oracle reports (k = lambda
    .. lambda + 2)."""
    x = synth.image_corr(11, 13, 0.2, key=4)
    for lam in (1, 2, 3):
        _, _, _, dg = oracle.acwddf(x, 3, EXACT, 4, lam, 10.8, diag=True)
        for j in range(3):
            _, _, o = oracle.cwfilter(x, 3, False, EXACT, 4, lam + j)
            assert np.array_equal(o, dg[..., (1 + j) * 9:(2 + j) * 9])


def test_rejects_bad_levels():
    x = np.zeros((4, 4, 3))
    for w, k in ((3, 0), (3, 6), (5, 14)):
        with pytest.raises(ValueError):
            oracle.cwfilter(x, w, True, EXACT, 4, k)
    oracle.cwfilter(x, 5, True, EXACT, 4, 13)
    assert BVDF == 0
