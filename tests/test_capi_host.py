"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/odf.h declares, and rejects bad arguments before any
launch (return codes and messages)."""
import ctypes

import pytest

from paper_1009_0958_amd import odf

FAKE = ctypes.c_void_p(0x7F0000000000)  # never dereferenced: validation fails first
FAKE2 = ctypes.c_void_p(0x7F0000100000)


def test_exports_every_declared_function():
    L = odf.lib()
    names = odf.declared_functions()
    assert "odf_filter_u8" in names and "odf_last_error" in names
    for name in names:
        assert hasattr(L, name), name
    assert L.odf_version() >= 1


def _u8(img, B, M, N, w, kind, p, dist, q, out, idx=None):
    return odf.lib().odf_filter_u8(img, B, M, N, w, kind, p, dist, q, out, idx, None)


@pytest.mark.parametrize("args,code,text", [
    ((None, 1, 8, 8, 3, 0, 0.0, 0, 4, FAKE2), odf.EINVAL, "img"),
    ((FAKE, 1, 8, 8, 3, 0, 0.0, 0, 4, None), odf.EINVAL, "out"),
    ((FAKE, 0, 8, 8, 3, 0, 0.0, 0, 4, FAKE2), odf.EINVAL, "sizes"),
    ((FAKE, 1, -1, 8, 3, 0, 0.0, 0, 4, FAKE2), odf.EINVAL, "sizes"),
    ((FAKE, 1, 8, 0, 3, 0, 0.0, 0, 4, FAKE2), odf.EINVAL, "sizes"),
    ((FAKE, 4096, 4096, 4096, 3, 0, 0.0, 0, 4, FAKE2), odf.EINVAL, "2^31"),
    ((FAKE, 1, 8, 8, 17, 0, 0.0, 0, 4, FAKE2), odf.EUNSUPPORTED, "window"),
    ((FAKE, 1, 8, 8, 4, 0, 0.0, 0, 4, FAKE2), odf.EUNSUPPORTED, "window"),
    ((FAKE, 1, 8, 8, 12, 0, 0.0, 0, 4, FAKE2), odf.EUNSUPPORTED, "window"),
    ((FAKE, 1, 8, 8, 1, 0, 0.0, 0, 4, FAKE2), odf.EUNSUPPORTED, "window"),
    ((FAKE, 1, 8, 8, 13, 2, 0.0, 0, 4, FAKE2), odf.EINVAL, "kind"),  # 13x13: checked as 3x3
    ((FAKE, 1, 8, 8, 3, 2, 0.0, 0, 4, FAKE2), odf.EINVAL, "kind"),
    ((FAKE, 1, 8, 8, 3, 0, 0.0, 3, 4, FAKE2), odf.EINVAL, "dist"),
    ((FAKE, 1, 8, 8, 3, 0, 0.0, 1, 5, FAKE2), odf.EINVAL, "q"),
    ((FAKE, 1, 8, 8, 3, 0, 0.0, 1, 1, FAKE2), odf.EINVAL, "q"),
    ((FAKE, 1, 8, 8, 3, 1, 1.5, 0, 4, FAKE2), odf.EINVAL, "p"),
    ((FAKE, 1, 8, 8, 3, 1, -0.1, 0, 4, FAKE2), odf.EINVAL, "p"),
    ((FAKE, 1, 8, 8, 3, 1, float("nan"), 0, 4, FAKE2), odf.EINVAL, "p"),
    ((FAKE, 1, 8, 8, 3, 0, 0.0, 0, 4, FAKE), odf.EINVAL, "overlaps"),
    ((FAKE, 1, 8, 8, 3, 0, 0.0, 0, 4, ctypes.c_void_p(0x7F0000000000 + 100)), odf.EINVAL,
     "overlaps"),
])
def test_filter_rejects(args, code, text):
    rc = _u8(*args)
    assert rc == code
    assert text in odf.last_error()


def test_idx_aliasing_rejected():
    rc = _u8(FAKE, 1, 8, 8, 3, 0, 0.0, 0, 4, FAKE2, ctypes.c_void_p(0x7F0000100000 + 10))
    assert rc == odf.EINVAL and "idx" in odf.last_error()


def test_f32_and_aggregates_reject():
    L = odf.lib()
    assert L.odf_filter_f32(None, 1, 4, 4, 3, 0, 0.0, 0, 4, FAKE2, None, None) == odf.EINVAL
    assert L.odf_aggregates_f32(FAKE, 1, 1, 4, 4, 3, 0, 0.0, 0, 4, None, None, None, None) == odf.EINVAL
    assert "A" in odf.last_error()
    assert L.odf_aggregates_f32(FAKE, 1, 1, 4, 4, 3, 0, 0.0, 0, 4, FAKE2, FAKE2, None, None) == odf.EINVAL
    assert "overlap" in odf.last_error()
    # windows past 9x9 run the direct form, which exports no aggregates
    assert L.odf_aggregates_f32(FAKE, 1, 1, 4, 4, 11, 0, 0.0, 0, 4, FAKE2, None, None,
                                None) == odf.EUNSUPPORTED
    assert "aggregates" in odf.last_error()


def test_general_windows_validated_like_the_others():
    """11x11 to 15x15: the hard backward and the tuning table reject what they
    do not offer; ACWDDF, the centre-weighted filters and the softmin validate
    their own arguments at these sizes (nothing is launched here)."""
    L = odf.lib()
    B = odf._batch_lib()
    bwd = lambda w, dx=FAKE2: L.odf_backward_hard_f32(  # noqa: E731
        FAKE, ctypes.c_void_p(0x7F0000200000), 1, 8, 8, w, dx, None)
    for w in (2, 16, 17):
        assert bwd(w) == odf.EUNSUPPORTED and "window" in odf.last_error()
    assert bwd(15, dx=ctypes.c_void_p(0x7F0000200000 + 12)) == odf.EINVAL  # dx overlaps dy
    for w in (11, 13, 15):
        n = w * w
        # lambda <= (n + 1) / 2 - 2 and level <= (n + 1) / 2 at every size
        assert L.odf_acwddf_u8(FAKE, 1, 8, 8, w, 0, 4, (n + 1) // 2 - 1, 10.8, FAKE2, None,
                               None) == odf.EINVAL and "lambda" in odf.last_error()
        assert L.odf_cw_filter_u8(FAKE, 1, 8, 8, w, odf.CWVMF, 0, 4, (n + 1) // 2 + 1, FAKE2,
                                  None, None) == odf.EINVAL and "level" in odf.last_error()
        assert L.odf_acwddf_u8(FAKE, 1, 8, 8, w, 0, 4, 2, 10.8, FAKE, None, None) == odf.EINVAL
        assert L.odf_softmin_fwd_f32(FAKE, 1, 8, 8, w, 1, 0.25, 0.0, FAKE2, None) \
            == odf.EINVAL and "tau" in odf.last_error()
    for w in (10, 17):
        assert L.odf_acwddf_u8(FAKE, 1, 8, 8, w, 0, 4, 2, 10.8, FAKE2, None, None) \
            == odf.EUNSUPPORTED
        assert L.odf_cw_filter_u8(FAKE, 1, 8, 8, w, odf.CWVMF, 0, 4, 1, FAKE2, None, None) \
            == odf.EUNSUPPORTED
        assert B.odf_tune_get(w, odf.DDF, 0, 1) == odf.EINVAL


def test_declared_names_match_binding():
    # every declared function has a binding attribute configured or a plain C symbol
    for name in odf.declared_functions():
        assert callable(getattr(odf.lib(), name))


class _Job(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("idx", ctypes.c_void_p),
                ("M", ctypes.c_int), ("N", ctypes.c_int), ("window", ctypes.c_int),
                ("kind", ctypes.c_int), ("dist", ctypes.c_int), ("q", ctypes.c_int),
                ("p", ctypes.c_float)]


@pytest.mark.parametrize("fields,code,text", [
    (dict(img=None), odf.EINVAL, "img"),
    (dict(M=0), odf.EINVAL, "size"),
    (dict(window=11), odf.EUNSUPPORTED, "window"),
    (dict(kind=3), odf.EINVAL, "kind"),
    (dict(dist=5), odf.EINVAL, "dist"),
    (dict(dist=1, q=9), odf.EINVAL, "q"),
    (dict(kind=1, p=2.0), odf.EINVAL, "p"),
    (dict(out=0x7F0000000000 + 10), odf.EINVAL, "overlap"),
])
def test_batch_plan_rejects(fields, code, text):
    L = odf._batch_lib()
    base = dict(img=0x7F0000000000, out=0x7F0000100000, idx=None, M=8, N=8, window=3, kind=0,
                dist=0, q=4, p=0.5)
    base.update(fields)
    jobs = (_Job * 2)(_Job(**dict(base, img=0x7F0000200000, out=0x7F0000300000)), _Job(**base))
    plan = ctypes.c_void_p()
    rc = L.odf_batch_plan(ctypes.cast(jobs, ctypes.c_void_p), 2, ctypes.byref(plan), None)
    assert rc == code and not plan.value
    assert text in odf.last_error()


def test_batch_and_tune_argument_errors():
    L = odf._batch_lib()
    plan = ctypes.c_void_p()
    assert L.odf_batch_plan(None, 1, ctypes.byref(plan), None) == odf.EINVAL
    assert L.odf_batch_launch(None, None) == odf.EINVAL
    assert L.odf_plan_destroy(None) == odf.EINVAL
    assert L.odf_tune_set(3, 0, 0, 1, 9) == odf.EINVAL
    assert L.odf_tune_set(3, 0, 0, 1, -1) == odf.EINVAL
    assert L.odf_tune_get(4, 0, 0, 1) == odf.EINVAL
    assert odf.tile_config(0) == (32, 32) and odf.tile_config(3) == (64, 8)
    # configs 4, 5: the strip form (32 x 16 bands): BVDF and DDF at 3x3 to 7x7, BVDF 9x9 on
    # uint8, the centre-weighted kinds at 3x3 to 7x7
    assert odf.tile_config(odf.STRIP) == (32, 16) and odf.tile_config(odf.SHORT_STRIP) == (32, 16)
    assert L.odf_tile_config(odf.NUM_TILE_CONFIGS, ctypes.byref(ctypes.c_int()),
                             ctypes.byref(ctypes.c_int())) == odf.EINVAL
    for w, kind, u8 in ((3, odf.BVDF, 1), (3, odf.DDF, 0), (5, odf.BVDF, 1), (5, odf.DDF, 1),
                        (7, odf.BVDF, 0), (7, odf.DDF, 1), (9, odf.BVDF, 1)):
        saved = odf.tune_get(w, kind, odf.EXACT, u8)
        assert L.odf_tune_set(w, kind, odf.EXACT, u8, odf.STRIP) == odf.OK
        assert odf.tune_get(w, kind, odf.EXACT, u8) == odf.STRIP
        assert L.odf_tune_set(w, kind, odf.EXACT, u8, odf.SHORT_STRIP) == odf.OK
        odf.tune_set(w, kind, odf.EXACT, u8, saved)
    for w, kind, u8 in ((3, odf.ACWDDF, 1), (5, odf.CWVMF, 0), (5, odf.CWDDF, 1)):
        saved = odf.tune_get(w, kind, odf.EXACT, u8)
        assert L.odf_tune_set(w, kind, odf.EXACT, u8, odf.SHORT_STRIP) == odf.OK
        odf.tune_set(w, kind, odf.EXACT, u8, saved)
    for w, kind, u8 in ((9, odf.DDF, 1), (9, odf.BVDF, 0)):
        assert L.odf_tune_set(w, kind, odf.EXACT, u8, odf.STRIP) == odf.EINVAL
        assert L.odf_tune_set(w, kind, odf.EXACT, u8, odf.SHORT_STRIP) == odf.EINVAL
    assert L.odf_tune_set(3, 0, 0, 1, odf.NUM_TILE_CONFIGS) == odf.EINVAL
    assert L.odf_autotune(3, 0, 0, 1, 0, 10, 1, None, None, None) == odf.EINVAL
    # batch tuning table: defaults, range checks, and the retired persistent form
    assert L.odf_batch_tune_get(3, odf.DDF) == 0 and L.odf_batch_tune_get(5, odf.BVDF) == 2
    assert L.odf_batch_tune_get(7, odf.DDF) == 2 and L.odf_batch_tune_get(9, odf.DDF) == 2
    assert L.odf_batch_tune_get(11, odf.DDF) == odf.EINVAL
    # 9x9 groups: shape 2, and the strips for BVDF (uint8)
    assert L.odf_batch_tune_set(9, odf.DDF, odf.STRIP) == odf.EINVAL
    assert L.odf_batch_tune_set(9, odf.DDF, 3) == odf.EINVAL
    assert L.odf_batch_tune_set(9, odf.BVDF, odf.SHORT_STRIP) == odf.OK
    assert L.odf_batch_tune_set(9, odf.BVDF, 2) == odf.OK
    # 7x7 groups: the 512-thread shapes and the strips, as the per-image table
    assert L.odf_batch_tune_set(7, odf.DDF, 0) == odf.EINVAL
    assert L.odf_batch_tune_set(7, odf.BVDF, 1) == odf.EINVAL
    assert L.odf_batch_tune_set(7, odf.DDF, odf.STRIP) == odf.OK
    assert L.odf_batch_tune_get(7, odf.DDF) == odf.STRIP
    assert L.odf_batch_tune_set(7, odf.DDF, 2) == odf.OK
    assert L.odf_batch_tune_get(3, odf.ACWDDF) == odf.EINVAL
    assert L.odf_batch_tune_set(3, odf.BVDF, odf.NUM_TILE_CONFIGS) == odf.EINVAL
    assert L.odf_batch_tune_set(3, odf.BVDF, odf.STRIP) == odf.OK  # the strip form
    assert L.odf_batch_tune_get(3, odf.BVDF) == odf.STRIP
    assert L.odf_batch_tune_set(3, odf.BVDF, 2) == odf.OK
    assert L.odf_batch_tune_set(5, odf.DDF, -1) == odf.EINVAL
    assert L.odf_batch_tune_set(5, odf.DDF, 1) == odf.OK and L.odf_batch_tune_get(5, odf.DDF) == 1
    assert L.odf_batch_tune_set(5, odf.DDF, 2) == odf.OK
    assert L.odf_autotune_batch(11, 0, 1, None, None, None) == odf.EINVAL
    assert L.odf_autotune_batch(3, 0, 0, None, None, None) == odf.EINVAL
    jobs = (odf._Job * 1)()
    assert L.odf_autotune_batch_jobs(None, 1, 2, None, None, None) == odf.EINVAL
    assert L.odf_autotune_batch_jobs(ctypes.cast(jobs, ctypes.c_void_p), 1, 0, None, None,
                                     None) == odf.EINVAL
    assert L.odf_plan_configs(None, None) == odf.EINVAL
    assert L.odf_batch_plan_ex(ctypes.cast(jobs, ctypes.c_void_p), 1, 0, ctypes.byref(plan),
                               None) == odf.EUNSUPPORTED
    assert "retired" in odf.last_error() and not plan.value
    assert L.odf_batch_plan_ex(ctypes.cast(jobs, ctypes.c_void_p), 1, 7, ctypes.byref(plan),
                               None) == odf.EINVAL


@pytest.mark.parametrize("args,code,text", [
    ((None, 1, 8, 8, 3, 0, 4, 2, 10.8, FAKE2), odf.EINVAL, "img"),
    ((FAKE, 1, 8, 8, 3, 0, 4, 2, 10.8, None), odf.EINVAL, "out"),
    ((FAKE, 1, 8, 8, 17, 0, 4, 2, 10.8, FAKE2), odf.EUNSUPPORTED, "window"),
    ((FAKE, 1, 8, 8, 3, 3, 4, 2, 10.8, FAKE2), odf.EINVAL, "dist"),
    ((FAKE, 1, 8, 8, 3, 1, 7, 2, 10.8, FAKE2), odf.EINVAL, "q"),
    ((FAKE, 1, 8, 8, 3, 0, 4, 0, 10.8, FAKE2), odf.EINVAL, "lambda"),
    ((FAKE, 1, 8, 8, 3, 0, 4, 4, 10.8, FAKE2), odf.EINVAL, "lambda"),
    ((FAKE, 1, 8, 8, 5, 0, 4, 12, 10.8, FAKE2), odf.EINVAL, "lambda"),
    ((FAKE, 1, 8, 8, 7, 0, 4, 24, 10.8, FAKE2), odf.EINVAL, "lambda"),  # 7x7: lambda <= 23
    ((FAKE, 1, 8, 8, 3, 0, 4, 2, float("nan"), FAKE2), odf.EINVAL, "NaN"),
    ((FAKE, 1, 8, 8, 3, 0, 4, 2, 10.8, FAKE), odf.EINVAL, "overlaps"),
])
def test_acwddf_rejects(args, code, text):
    L = odf.lib()
    assert L.odf_acwddf_u8(*args, None, None) == code
    assert text in odf.last_error()
    assert L.odf_acwddf_f32(*args, None, None) == code


def test_acwddf_tuning_table():
    L = odf._batch_lib()
    assert L.odf_tune_get(3, odf.ACWDDF, 0, 1) == 2  # default: 32 x 16 everywhere
    assert L.odf_tune_get(5, odf.ACWDDF, 0, 1) == 2
    assert L.odf_tune_set(5, odf.ACWDDF, 0, 1, 0) == odf.EINVAL  # 1024-thread shape not offered
    assert L.odf_tune_set(5, odf.ACWDDF, 0, 1, 3) == odf.OK
    assert L.odf_tune_set(5, odf.ACWDDF, 0, 1, 2) == odf.OK
    assert L.odf_tune_get(3, 5, 0, 1) == odf.EINVAL  # kinds end at ODF_CWDDF
    assert L.odf_tune_get(7, odf.ACWDDF, 0, 1) == 2
    assert L.odf_tune_set(7, odf.ACWDDF, 0, 1, 1) == odf.EINVAL  # 512-thread shapes only
    assert L.odf_tune_set(7, odf.ACWDDF, 0, 1, 4) == odf.OK  # the strip form
    assert L.odf_tune_set(7, odf.ACWDDF, 0, 1, 2) == odf.OK
    assert L.odf_tune_get(9, odf.ACWDDF, 0, 1) == odf.EINVAL  # no 9x9 ACWDDF
    assert L.odf_tune_get(7, odf.DDF, 0, 1) == 2
    assert L.odf_tune_set(7, odf.DDF, 0, 1, 1) == odf.EINVAL  # 512-thread shapes only


def test_noise_and_quality_reject():
    L = odf.lib()
    ok = (FAKE, FAKE2, 1, 8, 8, 0.1, 0.25, 0.25, 0.25, 1, None)
    for i, bad, text in ((0, None, "NULL"), (2, 0, "sizes"), (5, 1.5, "phi"), (5, -0.1, "phi"),
                         (6, -0.25, "phi"), (8, 0.6, "sum")):
        args = list(ok)
        args[i] = bad
        assert L.odf_noise_eq8_u8(*args) == odf.EINVAL, (i, bad)
        assert text in odf.last_error()
    assert L.odf_noise_eq8_u8(FAKE, ctypes.c_void_p(0x7F0000000000 + 7), 1, 8, 8, 0.1, 0.25, 0.25,
                              0.25, 1, None) == odf.EINVAL
    assert "overlaps" in odf.last_error()
    assert L.odf_quality_workspace(3) == 48 and L.odf_quality_workspace(0) == 0
    W = ctypes.c_void_p(0x7F0000200000)
    assert L.odf_quality_u8(FAKE, FAKE2, 2, 4, 4, W, W, W, 16, None) == odf.EINVAL
    assert "workspace" in odf.last_error()
    assert L.odf_quality_u8(FAKE, FAKE2, 2, 4, 4, W, W, ctypes.c_void_p(0x7F0000200004), 64,
                            None) == odf.EINVAL
    assert L.odf_quality_u8(FAKE, FAKE2, 70000, 1, 1, W, W, W, 1 << 20, None) == odf.EINVAL
    assert L.odf_quality_u8(None, FAKE2, 1, 4, 4, W, W, W, 64, None) == odf.EINVAL


def test_softmin_window_limits():
    """The softmin takes every odd window from 3 to 15; its 7x7 backward
    workspace holds one 32 x 16 extended tile (26 x 10 windows) of float32
    triples per tile, from 11x11 (the direct form) n triples per pixel."""
    L = odf.lib()
    assert L.odf_softmin_fwd_f32(FAKE, 1, 8, 8, 17, 1, 0.25, 0.1, FAKE2, None) == odf.EUNSUPPORTED
    assert "window" in odf.last_error()
    assert L.odf_softmin_bwd_workspace(1, 8, 8, 17, 1) == 0
    assert L.odf_softmin_bwd_workspace(1, 8, 8, 12, 1) == 0
    assert L.odf_softmin_bwd_workspace(2, 8, 9, 13, 1) == 2 * 8 * 9 * 169 * 3 * 4
    assert L.odf_softmin_bwd_workspace(1, 8, 8, 9, 1) == 1 * 1 * 512 * 3 * 4  # 24 x 8 windows
    tiles = 2 * -(-100 // 26) * -(-45 // 10)
    assert L.odf_softmin_bwd_workspace(2, 45, 100, 7, 1) == tiles * 512 * 3 * 4


def test_softmin_f64_rejects():
    L = odf.lib()
    D = ctypes.c_double
    fwd = lambda *a: L.odf_softmin_fwd_f64(*a[:6], D(a[6]), D(a[7]), a[8], None)  # noqa: E731
    assert fwd(None, 1, 4, 4, 3, 1, 0.25, 0.1, FAKE2) == odf.EINVAL and "x" in odf.last_error()
    assert fwd(FAKE, 1, 4, 4, 3, 1, 0.25, 0.1, None) == odf.EINVAL and "y" in odf.last_error()
    assert fwd(FAKE, 1, 4, 4, 11, 1, 0.25, 0.1, FAKE2) == odf.EUNSUPPORTED
    assert fwd(FAKE, 1, 4, 4, 3, 1, 1.5, 0.1, FAKE2) == odf.EINVAL and "p" in odf.last_error()
    assert fwd(FAKE, 1, 4, 4, 3, 1, 0.25, 0.0, FAKE2) == odf.EINVAL and "tau" in odf.last_error()
    assert fwd(FAKE, 1, 4, 4, 3, 1, 0.25, float("inf"), FAKE2) == odf.EINVAL
    assert fwd(FAKE, 1, 4, 4, 3, 3, 0.25, 0.1, FAKE2) == odf.EINVAL and "kind" in odf.last_error()
    assert fwd(FAKE, 1, 4, 4, 3, 1, 0.25, 0.1, ctypes.c_void_p(0x7F0000000000 + 64)) == odf.EINVAL
    assert "overlaps" in odf.last_error()
    need = L.odf_softmin_bwd_f64_workspace(1, 4, 4, 5)
    assert need == 4 * 4 * 25 * 3 * 8
    assert L.odf_softmin_bwd_f64_workspace(1, 4, 4, 7) == 4 * 4 * 49 * 3 * 8
    assert L.odf_softmin_bwd_f64_workspace(1, 4, 4, 9) == 4 * 4 * 81 * 3 * 8
    assert L.odf_softmin_bwd_f64_workspace(1, 4, 4, 11) == 0
    F3 = ctypes.c_void_p(0x7F0000200000)
    WS = ctypes.c_void_p(0x7F0000300000)
    bwd = lambda ws, nbytes, w=5: L.odf_softmin_bwd_f64(  # noqa: E731
        FAKE, FAKE2, 1, 4, 4, w, 1, D(0.25), D(0.1), F3, ws, nbytes, None)
    assert bwd(WS, need - 1) == odf.EINVAL and "workspace" in odf.last_error()
    assert bwd(ctypes.c_void_p(0x7F0000300004), need) == odf.EINVAL
    assert "aligned" in odf.last_error()
    assert bwd(None, need) == odf.EINVAL
    assert bwd(ctypes.c_void_p(0x7F0000200000 + 64), need) == odf.EINVAL
    assert "overlap" in odf.last_error()


def test_cw_filter_rejects():
    L = odf.lib()
    f = lambda w, kind, level, dist=0, out=FAKE2: L.odf_cw_filter_u8(  # noqa: E731
        FAKE, 1, 8, 8, w, kind, dist, 4, level, out, None, None)
    assert f(3, odf.CWVMF, 0) == odf.EINVAL and "level" in odf.last_error()
    assert f(3, odf.CWVMF, 6) == odf.EINVAL and "level" in odf.last_error()
    assert f(5, odf.CWDDF, 14) == odf.EINVAL
    assert f(3, odf.DDF, 1) == odf.EINVAL and "kind" in odf.last_error()
    assert f(3, odf.ACWDDF, 1) == odf.EINVAL
    assert f(17, odf.CWVMF, 1) == odf.EUNSUPPORTED
    assert f(7, odf.CWDDF, 26) == odf.EINVAL and "level" in odf.last_error()  # 7x7: k <= 25
    assert f(3, odf.CWDDF, 1, dist=3) == odf.EINVAL and "dist" in odf.last_error()
    assert f(3, odf.CWVMF, 1, out=None) == odf.EINVAL and "out" in odf.last_error()
    assert f(3, odf.CWVMF, 1, out=FAKE) == odf.EINVAL and "overlaps" in odf.last_error()


def test_binding_checks_caller_outputs():
    """Caller-supplied out / idx are checked before their pointers reach the
    kernel (which writes B*M*N*3 elements of out and B*M*N bytes of idx)."""
    import torch
    img = torch.zeros((2, 5, 7, 3), dtype=torch.uint8)
    ok_out = torch.empty_like(img)
    ok_idx = torch.empty((2, 5, 7), dtype=torch.uint8)
    odf.check_outputs(img, ok_out, ok_idx)
    odf.check_outputs(img, None, ok_idx.reshape(-1))  # any shape with B*M*N elements
    odf.check_outputs(img[0], torch.empty((5, 7, 3), dtype=torch.uint8), None)
    odf.check_outputs(img[0], torch.empty((1, 5, 7, 3), dtype=torch.uint8), None)
    bad = [
        (torch.empty((2, 5, 6, 3), dtype=torch.uint8), None, "shape"),
        (torch.empty((5, 7, 3), dtype=torch.uint8), None, "shape"),  # 3-D out for a batch
        (torch.empty((2, 5, 7, 3), dtype=torch.float32), None, "tensor like img"),
        (torch.empty((2, 7, 5, 3), dtype=torch.uint8).transpose(1, 2), None, "contiguous"),
        (None, torch.empty((2, 5, 6), dtype=torch.uint8), "elements"),
        (None, torch.empty((2, 5, 7), dtype=torch.int64), "uint8"),
        (None, torch.empty((2, 7, 5), dtype=torch.uint8).transpose(1, 2), "contiguous"),
    ]
    for out, idx, text in bad:
        with pytest.raises(ValueError, match=text):
            odf.check_outputs(img, out, idx)
    fimg = torch.zeros((5, 7, 3), dtype=torch.float32)
    with pytest.raises(ValueError, match="tensor like img"):
        odf.check_outputs(fimg, torch.empty((5, 7, 3), dtype=torch.uint8), None)
    if torch.cuda.is_available():  # device mismatch needs a second device type
        with pytest.raises(ValueError, match="device"):
            odf.check_outputs(img.cuda(), ok_out, None)


def test_allocation_failure_reports_enomem(monkeypatch):
    """ODF_TEST_FAIL_ALLOC makes the allocating calls take their allocation-failure
    path: ODF_ENOMEM with a message, nothing allocated, no device touched."""
    import ctypes as ct
    L = odf._batch_lib()
    jobs = (_Job * 2)()
    jobs[0] = _Job(0x7F0000000000, 0x7F0000100000, 0, 40, 50, 3, 1, 0, 4, 0.25)
    jobs[1] = _Job(0x7F0000200000, 0x7F0000300000, 0, 20, 30, 5, 0, 2, 4, 0.0)
    monkeypatch.setenv("ODF_TEST_FAIL_ALLOC", "1")
    plan = ct.c_void_p()
    rc = L.odf_batch_plan(ct.cast(jobs, ct.c_void_p), 2, ct.byref(plan), None)
    assert rc == odf.ENOMEM and "allocation" in odf.last_error() and not plan.value
    times = (ct.c_float * 16)()
    for w, kind, dist, u8 in ((3, odf.DDF, odf.EXACT, 1), (5, odf.CWVMF, odf.EXACT, 0),
                              (7, odf.BVDF, odf.RGB, 1)):
        rc = L.odf_autotune(w, kind, dist, u8, 64, 64, 2, None, ct.cast(times, ct.c_void_p), None)
        assert rc == odf.ENOMEM and "allocation" in odf.last_error()
    rc = L.odf_autotune_batch(5, odf.DDF, 2, None, ct.cast(times, ct.c_void_p), None)
    assert rc == odf.ENOMEM and "allocation" in odf.last_error()
    rc = L.odf_autotune_batch_jobs(ct.cast(jobs, ct.c_void_p), 2, 2, None, None, None)
    assert rc == odf.ENOMEM and "allocation" in odf.last_error()
    # validation still comes first
    rc = L.odf_autotune(11, odf.DDF, odf.EXACT, 1, 64, 64, 2, None, None, None)
    assert rc == odf.EINVAL
    assert L.odf_autotune_batch(11, odf.DDF, 2, None, None, None) == odf.EINVAL
    monkeypatch.setenv("ODF_TEST_FAIL_ALLOC", "0")
    bad = (_Job * 1)()
    bad[0] = _Job(0, 0x7F0000100000, 0, 40, 50, 3, 1, 0, 4, 0.25)
    assert L.odf_batch_plan(ct.cast(bad, ct.c_void_p), 1, ct.byref(plan), None) == odf.EINVAL


def test_tuning_table_has_centre_weighted_entries():
    """CWVMF^k and CWDDF^k have tile table entries of their own (5x5: the
    512-thread shapes only, as at 7x7; no 9x9); CWVMF, which has no angular
    term, keeps one entry for every dist."""
    L = odf._batch_lib()
    for kind in (odf.CWVMF, odf.CWDDF):
        assert odf.tune_get(3, kind, odf.EXACT) == 2
        assert L.odf_tune_get(7, kind, odf.EXACT, 1) == 2
        assert L.odf_tune_set(7, kind, odf.EXACT, 1, 0) == odf.EINVAL
        assert L.odf_tune_get(9, kind, odf.EXACT, 1) == odf.EINVAL
        assert L.odf_tune_set(5, kind, odf.EXACT, 1, 0) == odf.EINVAL  # 1024 threads
    odf.tune_set(3, odf.CWDDF, odf.RGB, True, 1)
    assert odf.tune_get(3, odf.CWDDF, odf.RGB) == 1
    assert odf.tune_get(3, odf.ACWDDF, odf.RGB) == 2  # a slot of its own
    odf.tune_set(5, odf.CWVMF, odf.MINIMAX, True, 3)
    assert odf.tune_get(5, odf.CWVMF, odf.EXACT) == 3
    odf.tune_set(3, odf.CWDDF, odf.RGB, True, 2)
    odf.tune_set(5, odf.CWVMF, odf.RGB, True, 2)


def test_noalloc_softmin_rejects_before_launch():
    L = odf.lib()
    f = L.odf_softmin_bwd_f32_noalloc
    # 1 x 4096 x 4096 at 5x5 needs ~300 MiB of workspace, beyond the 128 MiB static scratch
    assert f(FAKE, FAKE2, 1, 4096, 4096, 5, odf.DDF, 0.25, 0.1,
             ctypes.c_void_p(0x7F0010000000), None) == odf.EINVAL
    assert "static scratch" in odf.last_error()
    assert f(FAKE, None, 1, 8, 8, 5, odf.DDF, 0.25, 0.1, FAKE2, None) == odf.EINVAL
    assert f(FAKE, FAKE2, 1, 8, 8, 5, odf.DDF, 0.25, 0.0, FAKE2, None) == odf.EINVAL  # tau
    assert f(FAKE, FAKE2, 1, 8, 8, 17, odf.DDF, 0.25, 0.1, FAKE2, None) == odf.EUNSUPPORTED
    assert f(FAKE, FAKE2, 1, 8, 8, 5, odf.DDF, 0.25, 0.1, FAKE, None) == odf.EINVAL  # dx = x
    assert "overlaps" in odf.last_error()


def test_header_config_constants_match_binding():
    """The binding's config constants are the header's."""
    import re
    text = open(odf.HEADER).read()
    defs = dict(re.findall(r"#define (ODF_\w+) (\d+)", text))
    assert int(defs["ODF_NUM_TILE_CONFIGS"]) == odf.NUM_TILE_CONFIGS
    assert int(defs["ODF_STRIP_CONFIG"]) == odf.STRIP
    assert int(defs["ODF_SHORT_STRIP_CONFIG"]) == odf.SHORT_STRIP
