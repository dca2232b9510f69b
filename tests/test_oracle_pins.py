"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than the oracle:
closed-form angles, 50-digit brute force, the error values printed in Table 1,
the fitted line of eq. (10), textbook special cases and invariants.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
from oracle import BVDF, DDF, EXACT, MINIMAX, RGB

mpmath.mp.dps = 50

# Table 1 error column (Section 2.1): rows ASIN/ACOS, q = 2, 3, 4.
TABLE1_EPS = {
    ("asin", 2): 1.830987519e-03, ("asin", 3): 1.358426903e-04, ("asin", 4): 2.097813673e-05,
    ("acos", 2): 9.154936808e-04, ("acos", 3): 6.792158693e-05, ("acos", 4): 1.048948667e-05,
}


def _angle(a, b, dist=EXACT, kind=BVDF, q=4):
    th, _ = oracle.pair_terms(np.array([a], float), np.array([b], float), kind, dist, q)
    return th[0]


# ------------------------------------------------------------ exact angle (eq. 2)

def test_closed_form_angles():
    assert _angle((1, 0, 0), (0, 1, 0)) == pytest.approx(math.pi / 2, rel=1e-15)
    assert _angle((1, 1, 0), (1, 0, 0)) == pytest.approx(math.pi / 4, rel=1e-15)
    assert _angle((1, 1, 1), (1, 0, 0)) == pytest.approx(math.acos(1 / math.sqrt(3)), rel=1e-15)
    assert _angle((7, 7, 7), (3, 3, 3)) == 0.0
    # zero vector takes the achromatic direction (1,1,1)
    assert _angle((0, 0, 0), (5, 5, 5)) == 0.0
    assert _angle((0, 0, 0), (0, 0, 0)) == 0.0
    assert _angle((0, 0, 0), (9, 0, 0)) == pytest.approx(math.acos(1 / math.sqrt(3)), rel=1e-15)


def _mp_angle(a, b):
    a = [mpmath.mpf(int(v)) for v in a]
    b = [mpmath.mpf(int(v)) for v in b]
    if not any(a):
        a = [mpmath.mpf(1)] * 3
    if not any(b):
        b = [mpmath.mpf(1)] * 3
    dot = sum(x * y for x, y in zip(a, b))
    na = mpmath.sqrt(sum(x * x for x in a))
    nb = mpmath.sqrt(sum(x * x for x in b))
    z = dot / (na * nb)
    z = min(max(z, mpmath.mpf(-1)), mpmath.mpf(1))
    return mpmath.acos(z)


def test_exact_angle_vs_50_digits():
    rng = np.random.default_rng(11)
    a = rng.integers(0, 256, (300, 3))
    b = a + rng.integers(-1, 2, (300, 3))  # near-parallel pairs: the hard case for acos
    b = np.clip(b, 0, 255)
    a2 = rng.integers(0, 256, (300, 3))
    b2 = rng.integers(0, 256, (300, 3))
    A = np.concatenate([a, a2])
    Bv = np.concatenate([b, b2])
    th, _ = oracle.pair_terms(A, Bv, BVDF, EXACT)
    for i in range(A.shape[0]):
        ref = _mp_angle(A[i], Bv[i])
        if ref < 1e-20:  # parallel: 0 up to the 50-digit rounding of acos
            assert th[i] == 0.0
        else:
            assert abs(th[i] - float(ref)) <= 1e-14 * float(ref), (A[i], Bv[i])


def test_smallest_uint8_angles():
    # the smallest non-zero angle between uint8 colours is ~ 1/(sqrt(3) 255^2 ...) rad
    th = _angle((255, 255, 254), (254, 254, 253))
    ref = float(_mp_angle((255, 255, 254), (254, 254, 253)))
    assert 1e-6 < ref < 1e-5
    assert th == pytest.approx(ref, rel=1e-13)


def test_pair_terms_symmetric_bitwise():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 256, (2000, 3)).astype(float)
    b = rng.integers(0, 256, (2000, 3)).astype(float)
    a[:50] = 0
    for dist in (EXACT, MINIMAX, RGB):
        for kind in (BVDF, DDF):
            for q in (2, 3, 4):
                t1, l1 = oracle.pair_terms(a, b, kind, dist, q)
                t2, l2 = oracle.pair_terms(b, a, kind, dist, q)
                assert np.array_equal(t1, t2)
                assert np.array_equal(l1, l2)


# ------------------------------------------------------------ Method 1 (Table 1)

@pytest.mark.parametrize("q", [2, 3, 4])
def test_table1_error_reproduced(q):
    """Max error of the oracle's minimax angle on each branch matches Table 1's epsilon."""
    # ACOS branch: z uniform in [0, 1/2)
    z = np.linspace(0.0, 0.5, 1_000_001)[:-1]
    t = np.arccos(z)
    a = np.tile([1.0, 0.0, 0.0], (z.size, 1))
    b = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], 1)
    th, _ = oracle.pair_terms(a, b, BVDF, MINIMAX, q)
    # the true angle of the vectors actually passed
    ref = np.arctan2(b[:, 1], b[:, 0])
    err_acos = np.max(np.abs(th - ref))
    # ASIN branch: tau uniform in [0, 1/sqrt 2], z = 1 - tau^2 >= 1/2
    tau = np.linspace(0.0, 1 / np.sqrt(2), 1_000_001)[:-1]
    t = 2 * np.arcsin(tau / np.sqrt(2))
    b = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)], 1)
    th, _ = oracle.pair_terms(a, b, BVDF, MINIMAX, q)
    ref = np.arctan2(b[:, 1], b[:, 0])
    err_asin = np.max(np.abs(th - ref))
    assert err_acos == pytest.approx(TABLE1_EPS[("acos", q)], rel=0.02)
    assert err_asin == pytest.approx(TABLE1_EPS[("asin", q)], rel=0.02)


@pytest.mark.parametrize("q", [2, 3, 4])
def test_minimax_constant_window_and_sign(q):
    """Identical directions sit at tau = 0 of the ASIN row, whose value is a_0
    (Table 1); an angle is never negative, so the q = 3 row (a_0 < 0) is clamped
    at 0.  A constant window's aggregate is n times that value (self pair included)."""
    a0 = {2: 1.829125e-03, 3: -1.358425e-04, 4: 2.097797e-05}[q]
    img = np.full((6, 6, 3), (30, 90, 150), np.uint8)
    for w in (3, 5):
        _, _, A, _, _ = oracle.filter(img, w, BVDF, 0, MINIMAX, q, aggregates=True)
        assert np.allclose(A, w * w * max(a0, 0.0), rtol=1e-14, atol=0)
    rng = np.random.default_rng(q)
    a = rng.integers(0, 256, (20000, 3)).astype(float)
    b = np.clip(a + rng.integers(-2, 3, a.shape), 0, 255)
    th, _ = oracle.pair_terms(a, b, BVDF, MINIMAX, q)
    assert th.min() >= 0.0


def test_minimax_branch_at_sixty_degrees():
    # z = 1/2 exactly: (1,1,0).(0,1,1) = 1, |a|^2 |b|^2 = 4 -> ASIN row at tau = 1/sqrt 2
    for q in (2, 3, 4):
        th = _angle((1, 1, 0), (0, 1, 1), MINIMAX, q=q)
        assert abs(th - math.pi / 3) <= TABLE1_EPS[("asin", q)] * 1.02


# ------------------------------------------------------------ Method 2 (eq. 7, eq. 10)

def test_eq10_line_reproduced():
    """A total-least-squares line through (B, A) over uniform integer RGB pairs
    reproduces the slope and intercept printed in eq. (10)."""
    rng = np.random.default_rng(1009)
    a = rng.integers(0, 256, (1_000_000, 3)).astype(float)
    b = rng.integers(0, 256, (1_000_000, 3)).astype(float)
    keep = (a.sum(1) > 0) & (b.sum(1) > 0)
    a, b = a[keep], b[keep]
    A, _ = oracle.pair_terms(a, b, BVDF, EXACT)
    Bd, _ = oracle.pair_terms(a, b, BVDF, RGB)
    X = np.stack([Bd - Bd.mean(), A - A.mean()], 1)
    _, _, vt = np.linalg.svd(X, full_matrices=False)
    nx, ny = vt[0]
    slope = ny / nx
    intercept = A.mean() - slope * Bd.mean()
    assert slope == pytest.approx(1.436437, abs=3e-3)
    assert intercept == pytest.approx(0.027664, abs=1.5e-3)
    # DDF's rgb pair term is that line applied to B
    Bddf, _ = oracle.pair_terms(a[:1000], b[:1000], DDF, RGB)
    assert np.allclose(Bddf, 1.436437 * Bd[:1000] + 0.027664, rtol=0, atol=1e-15)


def test_chromaticity_closed_forms():
    # chromaticities (1,0,0) and (0,1,0): distance sqrt 2
    assert _angle((10, 0, 0), (0, 3, 0), RGB) == pytest.approx(math.sqrt(2), rel=1e-15)
    # scale-free: (2,4,6) and (1,2,3) have the same chromaticity
    assert _angle((2, 4, 6), (1, 2, 3), RGB) == 0.0
    # zero vector is achromatic (1/3,1/3,1/3)
    ref = math.sqrt((1 - 1 / 3) ** 2 + 2 * (1 / 3) ** 2)
    assert _angle((0, 0, 0), (5, 0, 0), RGB) == pytest.approx(ref, rel=1e-15)


def test_l2_is_euclidean():
    _, l2 = oracle.pair_terms(np.array([[3.0, 0, 0], [0, 0, 0]]), np.array([[0.0, 4, 0], [1, 2, 2]]))
    assert l2[0] == 5.0 and l2[1] == 3.0


# ------------------------------------------------------------ filters by brute force

def _tiny_image(seed, M=6, N=5):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, (M, N, 3)).astype(np.uint8)
    img[1, 1] = img[2, 3]  # a duplicated colour
    img[0, 4] = 0  # a zero vector
    img[3, 2] = img[3, 1] // 2  # a collinear pair
    return img


def _mp_chroma(a, b):
    def ch(x):
        x = [mpmath.mpf(int(v)) for v in x]
        if not any(x):
            x = [mpmath.mpf(1)] * 3
        s = sum(x)
        return [v / s for v in x]
    ca, cb = ch(a), ch(b)
    return mpmath.sqrt(sum((u - v) ** 2 for u, v in zip(ca, cb)))


def _mp_filter(img, w, kind, p, dist):
    """50-digit brute force of eqs. 1-3 over every window (replicated border).
    The two pair terms of a pair of colours are evaluated once and reused
    (windows larger than the image repeat its few colours many times)."""
    M, N, _ = img.shape
    h = w // 2
    A = np.empty((M, N, w * w))
    D = np.empty((M, N, w * w))
    memo = {}

    def terms(xu, xv):
        key = (tuple(int(v) for v in xu), tuple(int(v) for v in xv))
        if key not in memo:
            if dist == EXACT:
                a = _mp_angle(xu, xv)
            else:
                bb = _mp_chroma(xu, xv)
                a = (mpmath.mpf("1.436437") * bb + mpmath.mpf("0.027664")) if kind == DDF else bb
            d = mpmath.sqrt(sum((mpmath.mpf(int(x)) - int(y)) ** 2 for x, y in zip(xu, xv)))
            memo[key] = (a, d)
        return memo[key]

    for r in range(M):
        for c in range(N):
            mem = [img[min(max(r + dy, 0), M - 1), min(max(c + dx, 0), N - 1)]
                   for dy in range(-h, h + 1) for dx in range(-h, h + 1)]
            for u, xu in enumerate(mem):
                sa = mpmath.mpf(0)
                sd = mpmath.mpf(0)
                for xv in mem:
                    a, d = terms(xu, xv)
                    sa += a
                    sd += d
                A[r, c, u] = float(sa)
                D[r, c, u] = float(sd)
    return A, D


@pytest.mark.parametrize("w,kind,p,dist", [
    (w, kind, p, dist) for w in (3, 5) for kind, p in ((BVDF, 0.0), (DDF, 0.25), (DDF, 0.5))
    for dist in (EXACT, RGB)] + [(7, BVDF, 0.0, EXACT), (7, DDF, 0.25, EXACT),
                                 (9, BVDF, 0.0, EXACT), (9, DDF, 0.25, RGB),
                                 (11, BVDF, 0.0, EXACT), (11, DDF, 0.25, EXACT),
                                 (13, DDF, 0.5, RGB), (15, BVDF, 0.0, RGB),
                                 (15, DDF, 0.25, EXACT)])
def test_filter_vs_50_digit_bruteforce(w, kind, p, dist):
    """Every window size the filter takes, 3 x 3 to 15 x 15: at 11 x 11 and
    above on images smaller than the window, so that most members are
    replicated border pixels and many aggregates tie exactly."""
    img = _tiny_image(w * 10 + kind, {3: 6, 5: 5, 7: 4, 9: 4}.get(w, 4), 5)
    out, idx, A, D, O = oracle.filter(img, w, kind, p, dist, aggregates=True)
    mA, mD = _mp_filter(img, w, kind, p, dist)
    assert np.allclose(A, mA, rtol=1e-13, atol=1e-13)
    if kind == DDF:
        assert np.allclose(D, mD, rtol=1e-13, atol=1e-13)
        mO = mA ** (1 - p) * mD ** p
    else:
        mO = mA
    # selection: the lowest index among the 50-digit minima (exact ties kept)
    M, N, n = mO.shape
    for r in range(M):
        for c in range(N):
            o = mO[r, c]
            cand = np.flatnonzero(o <= o.min() * (1 + 1e-12) + 1e-300)
            assert idx[r, c] == cand[0] or o[idx[r, c]] <= o.min() * (1 + 1e-12)
            u = int(idx[r, c])
            h = w // 2
            sr = min(max(r + u // w - h, 0), M - 1)
            sc = min(max(c + u % w - h, 0), N - 1)
            assert np.array_equal(out[r, c], img[sr, sc].astype(float))


@pytest.mark.parametrize("q", [2, 3, 4])
@pytest.mark.parametrize("w", [3, 5, 7, 9, 11, 15])
def test_minimax_aggregates_within_table1_bound(q, w):
    img = _tiny_image(70 + q, 8, 8)
    _, _, Ae, _, _ = oracle.filter(img, w, BVDF, 0, EXACT, aggregates=True)
    _, _, Am, _, _ = oracle.filter(img, w, BVDF, 0, MINIMAX, q, aggregates=True)
    bound = w * w * max(TABLE1_EPS[("asin", q)], TABLE1_EPS[("acos", q)]) * 1.0001
    assert np.max(np.abs(Am - Ae)) <= bound


# ------------------------------------------------------------ DDF special cases

def _window_stack(img, w):
    M, N, _ = img.shape
    h = w // 2
    rr = np.clip(np.arange(M)[:, None] + np.arange(-h, h + 1)[None, :], 0, M - 1)
    cc = np.clip(np.arange(N)[:, None] + np.arange(-h, h + 1)[None, :], 0, N - 1)
    win = img[rr[:, None, :, None], cc[None, :, None, :]]  # M, N, w, w, 3
    return win.reshape(M, N, w * w, 3).astype(np.float64)


def _near_tie_ok(idx_a, idx_b, omega, rel=1e-9):
    """Selections agree except where the objective has a near-tie."""
    bad = idx_a != idx_b
    if not bad.any():
        return True
    o = np.take_along_axis(omega, idx_a[..., None].astype(np.int64), -1)[..., 0]
    ob = np.take_along_axis(omega, idx_b[..., None].astype(np.int64), -1)[..., 0]
    return bool(np.all(np.abs(o - ob)[bad] <= rel * np.abs(ob[bad]) + 1e-300))


def test_ddf_p0_equals_bvdf():
    img = _tiny_image(3, 24, 20)
    for dist in (EXACT, MINIMAX, RGB):
        _, i0 = oracle.filter(img, 3, DDF, 0.0, dist)
        _, ib = oracle.filter(img, 3, BVDF, 0.0, dist)
        if dist == RGB:  # DDF uses alpha*B + beta: an increasing map of BVDF's B
            _, _, _, _, O = oracle.filter(img, 3, BVDF, 0.0, dist, aggregates=True)
            assert _near_tie_ok(i0, ib, O)
        else:
            assert np.array_equal(i0, ib)


@pytest.mark.parametrize("w", [3, 5, 7, 9])
def test_ddf_p1_is_vector_median(w):
    """p = 1 orders by the aggregated L2 distance: the vector median filter (eq. 1)."""
    img = _tiny_image(4, 20, 18)
    _, idx = oracle.filter(img, w, DDF, 1.0, EXACT)
    win = _window_stack(img, w)
    dist = np.linalg.norm(win[:, :, :, None, :] - win[:, :, None, :, :], axis=-1).sum(-1)
    ref = np.argmin(dist, axis=-1)
    assert _near_tie_ok(idx, ref, dist)


@pytest.mark.parametrize("w", [3, 5, 7, 9])
def test_ddf_half_is_eq3_product(w):
    """p = 1/2 orders by sqrt(A D): the product form of eq. (3)."""
    img = _tiny_image(5, 20, 18)
    _, idx = oracle.filter(img, w, DDF, 0.5, EXACT)
    win = _window_stack(img, w)
    d = np.where(np.all(win == 0, -1, keepdims=True), 1.0, win)
    nrm = np.linalg.norm(d, axis=-1)
    cos = np.einsum("...uk,...vk->...uv", d, d) / (nrm[..., :, None] * nrm[..., None, :])
    A = np.arccos(np.clip(cos, -1, 1)).sum(-1)
    L = np.linalg.norm(win[:, :, :, None, :] - win[:, :, None, :, :], axis=-1).sum(-1)
    prod = A * L
    ref = np.argmin(prod, axis=-1)
    # np.arccos near 1 is only accurate to ~1e-8: compare with a looser tie band
    assert _near_tie_ok(idx, ref, prod, rel=1e-6)


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_scaling_by_two_keeps_bvdf_selection(dist):
    img = (_tiny_image(8, 16, 16) // 2).astype(np.uint8)
    _, i1 = oracle.filter(img, 3, BVDF, 0, dist)
    _, i2 = oracle.filter(img * 2, 3, BVDF, 0, dist)
    assert np.array_equal(i1, i2)


def test_scaling_keeps_ddf_selection_up_to_near_ties():
    img = (_tiny_image(9, 16, 16) // 2).astype(np.uint8)
    _, i1, _, _, O = oracle.filter(img, 5, DDF, 0.25, EXACT, aggregates=True)
    _, i2 = oracle.filter(img * 2, 5, DDF, 0.25, EXACT)
    assert _near_tie_ok(i2, i1, O, rel=1e-12)


@pytest.mark.parametrize("kind,p", [(BVDF, 0), (DDF, 0.25), (DDF, 0.5)])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_constant_image_maps_to_itself(kind, p, dist):
    img = np.full((7, 9, 3), (120, 40, 200), np.uint8)
    out, idx = oracle.filter(img, 5, kind, p, dist)
    assert np.array_equal(out, img.astype(float))
    assert np.all(idx == 0)


@pytest.mark.parametrize("kind,p", [(BVDF, 0), (DDF, 0.25), (DDF, 0.5)])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_lone_impulse_never_selected(kind, p, dist):
    img = np.full((9, 9, 3), (100, 50, 20), np.uint8)
    img[4, 4] = (20, 200, 40)
    out, idx, A, D, O = oracle.filter(img, 3, kind, p, dist, aggregates=True)
    assert np.all(out == np.array([100, 50, 20], float))
    # in the impulse's own window the impulse's aggregate is (n-1) times a
    # background member's for exact (the background pairs contribute 0)
    if dist == EXACT:
        a = A[4, 4]
        assert a[4] == pytest.approx(8 * a[0], rel=1e-14)
        assert O[4, 4, 4] == pytest.approx(8 * O[4, 4, 0], rel=1e-12)
    # 7x7: the impulse's aggregate is 48 times a background member's
    out7, _, A7, _, _ = oracle.filter(img, 7, kind, p, dist, aggregates=True)
    assert np.all(out7 == np.array([100, 50, 20], float))
    if dist == EXACT:
        assert A7[4, 4, 24] == pytest.approx(48 * A7[4, 4, 0], rel=1e-14)


def test_channel_permutation_keeps_selection():
    img = _tiny_image(12, 16, 16)
    for dist in (EXACT, RGB, MINIMAX):
        _, i1 = oracle.filter(img, 3, BVDF, 0, dist)
        _, i2 = oracle.filter(img[..., [2, 0, 1]], 3, BVDF, 0, dist)
        assert np.array_equal(i1, i2)


def test_collinear_window_selects_first_member():
    # a gray ramp: every angle is 0, so every objective is 0 (also for DDF,
    # whose objective is a product) and the lowest index wins
    ramp = np.repeat(np.arange(10, 10 + 8 * 12, 12, dtype=np.uint8)[:, None], 8, 1)
    img = np.repeat(ramp[..., None], 3, 2)
    for kind, p in ((BVDF, 0), (DDF, 0.5)):
        _, idx = oracle.filter(img, 3, kind, p, EXACT)
        assert np.all(idx == 0)


def _collinear_image(M, N, seed):
    """Mostly positive multiples of (1, 2, 3) at different brightness, with a
    few other colours and a zero pixel scattered in."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 86, (M, N))
    img = (k[..., None] * np.array([1, 2, 3])).astype(np.uint8)
    other = rng.random((M, N)) < 0.25
    img[other] = rng.integers(0, 256, (int(other.sum()), 3))
    img[0, 0] = 0
    return img


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("w", [3, 5])
def test_collinear_colours_tie_exactly(dist, w):
    """eq. (2) and eq. (7) are scale-free: members that are positive multiples
    of one colour have mathematically equal angle sums.  The oracle ties them
    bit for bit (canonical directions) and takes the lowest index among the
    members of the minimum; the 50-digit sums of those members agree."""
    img = _collinear_image(6, 7, 40 + w + dist)
    _, idx, A, _, _ = oracle.filter(img, w, BVDF, 0.0, dist, aggregates=True)
    win = _window_stack(img, w).astype(np.int64)
    M, N, n = A.shape
    ties = 0
    for r in range(M):
        for c in range(N):
            mem = win[r, c]
            for u in range(n):
                for v in range(u):
                    if np.any(mem[u]) and np.any(mem[v]) and np.all(np.cross(mem[u], mem[v]) == 0):
                        assert A[r, c, u] == A[r, c, v]
            amin = A[r, c].min()
            first = int(np.flatnonzero(A[r, c] == amin)[0])
            assert idx[r, c] == first
            if np.all(np.cross(mem[first], mem[np.argsort(A[r, c], kind="stable")[1]]) == 0) \
                    and A[r, c, np.argsort(A[r, c], kind="stable")[1]] == amin:
                ties += 1
    assert ties > M * N // 4  # the image does exercise collinear ties at the minimum
    if dist != MINIMAX:
        mA, _ = _mp_filter(img[:4, :4], w, BVDF, 0.0, dist)
        _, _, A4, _, _ = oracle.filter(img[:4, :4], w, BVDF, 0.0, dist, aggregates=True)
        assert np.allclose(A4, mA, rtol=1e-13, atol=1e-13)
        w4 = _window_stack(img[:4, :4], w).astype(np.int64)
        for r in range(4):
            for c in range(4):
                for u in range(n):
                    for v in range(u):
                        a, b = w4[r, c, u], w4[r, c, v]
                        if np.any(a) and np.any(b) and np.all(np.cross(a, b) == 0):
                            # equal to 50 digits (acos next to 1 leaves ~1e-25 of 0)
                            assert abs(mA[r, c, u] - mA[r, c, v]) <= 1e-20


def test_canonical_direction_keeps_scaled_images():
    """Any positive integer multiple of a uint8 image (here 3x, past 255, as
    float64) gives the BVDF selections of the image itself, bit for bit."""
    img = _tiny_image(17, 12, 11)
    for dist in (EXACT, MINIMAX, RGB):
        _, i1 = oracle.filter(img, 3, BVDF, 0.0, dist)
        _, i3 = oracle.filter(img.astype(np.float64) * 3, 3, BVDF, 0.0, dist)
        assert np.array_equal(i1, i3)


# ------------------------------------------------------------ hard backward

@pytest.mark.parametrize("w,kind,p,dist", [(3, DDF, 0.25, EXACT), (5, BVDF, 0.0, MINIMAX),
                                           (7, DDF, 0.5, RGB), (5, DDF, 0.3, EXACT),
                                           (13, DDF, 0.25, MINIMAX)])
def test_filter_at_matches_full_filter(w, kind, p, dist):
    """filter_at (the sampled form the full-size parity tests and the benchmark's
    mismatch counts use) returns, at each listed flat position (b*M + r)*N + c,
    exactly what the full filter computes there: the decode of b, r, c and the
    packing of out, idx, A, D and Omega, in list order (repeats and borders
    included)."""
    rng = np.random.default_rng(50 + w)
    x = rng.integers(0, 256, (3, 11, 13, 3)).astype(np.float64)
    x[rng.random((3, 11, 13)) < 0.1] = 0
    out, idx, A, D, O = oracle.filter(x, w, kind, p, dist, aggregates=True)
    B, M, N = idx.shape
    corners = [(b * M + r) * N + c for b in (0, B - 1) for r in (0, M - 1) for c in (0, N - 1)]
    pix = np.concatenate([rng.permutation(B * M * N)[:120], corners, [7, 7, B * M * N - 1]])
    o2, i2, A2, D2, O2 = oracle.filter_at(x, pix, w, kind, p, dist)
    n = w * w
    assert np.array_equal(o2, out.reshape(-1, 3)[pix])
    assert np.array_equal(i2, idx.reshape(-1)[pix])
    for got, full in ((A2, A), (D2, D), (O2, O)):
        assert np.array_equal(got, full.reshape(-1, n)[pix])
    for bad in ([-1], [B * M * N]):
        with pytest.raises(ValueError):
            oracle.filter_at(x, bad, w, kind, p, dist)


def test_backward_hard_routes_and_conserves():
    rng = np.random.default_rng(2)
    img = _tiny_image(13, 12, 10)
    for w in (3, 5, 7, 9, 11, 15):
        _, idx = oracle.filter(img, w, DDF, 0.25, EXACT)
        dy = rng.standard_normal(img.shape)
        dx = oracle.backward_hard(idx, dy, w)
        assert dx.sum() == pytest.approx(dy.sum(), rel=1e-12, abs=1e-12)
        ones = oracle.backward_hard(idx, np.ones(img.shape), w)
        # independent count of how often each pixel is selected
        M, N = idx.shape
        h = w // 2
        iu = idx.astype(np.int64)
        rr = np.clip(np.arange(M)[:, None] + iu // w - h, 0, M - 1)
        cc = np.clip(np.arange(N)[None, :] + iu % w - h, 0, N - 1)
        cnt = np.zeros((M, N))
        np.add.at(cnt, (rr, cc), 1.0)
        assert np.array_equal(ones[..., 0], cnt)
        assert np.array_equal(ones[..., 1], cnt)
        ref = np.zeros_like(dy)
        np.add.at(ref, (rr, cc), dy)
        assert np.allclose(dx, ref, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------ softmin relaxation

def _float_tiny(seed, M, N):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.05, 1.0, (M, N, 3))


@pytest.mark.parametrize("w,kind,p,tau", [(3, BVDF, 0.0, 0.1), (3, DDF, 0.25, 0.1),
                                          (5, DDF, 0.25, 0.1), (5, DDF, 0.25, 0.01),
                                          (3, DDF, 0.5, 0.01), (5, BVDF, 0.0, 0.01),
                                          (11, DDF, 0.25, 0.1)])
def test_softmin_gradient_vs_central_differences(w, kind, p, tau):
    x = _float_tiny(21 + w, 5, 6)
    rng = np.random.default_rng(3)
    dy = rng.standard_normal(x.shape)
    g = oracle.softmin_bwd(x, dy, w, kind, p, tau)
    eps = 1e-6
    num = np.empty_like(x)
    flat = x.reshape(-1)
    for i in range(flat.size):
        xp = flat.copy(); xp[i] += eps
        xm = flat.copy(); xm[i] -= eps
        fp = (oracle.softmin_fwd(xp.reshape(x.shape), w, kind, p, tau) * dy).sum()
        fm = (oracle.softmin_fwd(xm.reshape(x.shape), w, kind, p, tau) * dy).sum()
        num.reshape(-1)[i] = (fp - fm) / (2 * eps)
    assert np.allclose(g, num, rtol=1e-5, atol=1e-6 * np.abs(num).max())


def test_softmin_limits():
    x = _float_tiny(40, 9, 8)
    # tau -> 0: the hard selection (where the minimum is well separated)
    for kind, p in ((BVDF, 0.0), (DDF, 0.25)):
        out, idx, _, _, O = oracle.filter(x, 3, kind, p, EXACT, aggregates=True)
        y, pi = oracle.softmin_fwd(x, 3, kind, p, 1e-7, weights=True)
        srt = np.sort(O, -1)
        clear = (srt[..., 1] - srt[..., 0]) > 1e-4
        assert np.allclose(y[clear], out[clear], rtol=0, atol=1e-12)
        assert np.allclose(pi.sum(-1), 1.0, rtol=0, atol=1e-14)
    # tau -> infinity: the plain mean of the (replicated) window
    y = oracle.softmin_fwd(x, 3, DDF, 0.25, 1e9)
    assert np.allclose(y, _window_stack(x, 3).mean(2), rtol=0, atol=1e-8)


def test_window_range():
    """The filters, the hard backward and the softmin relaxation take every odd
    window from 3 x 3 to 15 x 15 (the member index is a byte).  Even and larger
    windows are rejected."""
    img = _tiny_image(3, 4, 5)
    for w in (1, 2, 4, 10, 17):
        with pytest.raises(ValueError):
            oracle.filter(img, w, BVDF, 0.0, EXACT)
        with pytest.raises(ValueError):
            oracle.backward_hard(np.zeros((4, 5), np.uint8), np.zeros((4, 5, 3)), w)
    x = img.astype(np.float64)
    for w in (10, 17):
        with pytest.raises(ValueError):
            oracle.softmin_fwd(x, w, DDF, 0.25, 0.1)
    for w in (10, 17):
        with pytest.raises(ValueError):
            oracle.cwfilter(img, w, True, EXACT, 4, 1)
    # a constant image: every member ties, the lowest index wins
    for w in (11, 13, 15):
        out, idx = oracle.filter(np.full((5, 6, 3), 77, np.uint8), w, DDF, 0.25, EXACT)
        assert np.all(idx == 0) and np.all(out == 77.0)
