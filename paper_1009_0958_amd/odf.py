"""Python binding of libodf (ctypes).  Argument marshalling only: every step
of the filter runs in the HIP kernels of ``libodf.so``; torch provides device
memory and the current stream.

Images are torch tensors of shape (B, M, N, 3) or (M, N, 3), uint8 or
float32, contiguous, on a ROCm device.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# ODF_LIB names another build of the same library (the host-sanitized build the
# sanitizer tests load); by default the in-tree libodf.so
LIB_PATH = os.environ.get("ODF_LIB") or os.path.join(HERE, "libodf.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "odf.h")

BVDF, DDF, ACWDDF, CWVMF, CWDDF = 0, 1, 2, 3, 4
EXACT, MINIMAX, RGB = 0, 1, 2
OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM = 0, -1, -2, -3, -4
NUM_TILE_CONFIGS = 6  # ODF_NUM_TILE_CONFIGS: four tile shapes and two strip heights
STRIP = 4             # ODF_STRIP_CONFIG: strips of 8 bands
SHORT_STRIP = 5       # ODF_SHORT_STRIP_CONFIG: strips of 3 bands

_KIND = {"bvdf": BVDF, "ddf": DDF, "acwddf": ACWDDF, "cwvmf": CWVMF, "cwddf": CWDDF}
_DIST = {"exact": EXACT, "minimax": MINIMAX, "rgb": RGB}

_lib = None


class ODFError(RuntimeError):
    """A libodf call returned a non-zero status."""

    def __init__(self, code, msg):
        super().__init__("libodf error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load ``libodf.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libodf.so is not built (%s); run python -m paper_1009_0958_amd.build"
                               % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I, F = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.odf_version.restype = I
        L.odf_last_error.restype = ctypes.c_char_p
        L.odf_filter_u8.argtypes = [P, I, I, I, I, I, F, I, I, P, P, P]
        L.odf_filter_f32.argtypes = [P, I, I, I, I, I, F, I, I, P, P, P]
        L.odf_acwddf_u8.argtypes = [P, I, I, I, I, I, I, I, F, P, P, P]
        L.odf_acwddf_f32.argtypes = [P, I, I, I, I, I, I, I, F, P, P, P]
        L.odf_cw_filter_u8.argtypes = [P, I, I, I, I, I, I, I, I, P, P, P]
        L.odf_cw_filter_f32.argtypes = [P, I, I, I, I, I, I, I, I, P, P, P]
        L.odf_aggregates_f32.argtypes = [P, I, I, I, I, I, I, F, I, I, P, P, P, P]
        Dbl = ctypes.c_double
        L.odf_noise_eq8_u8.argtypes = [P, P, I, I, I, Dbl, Dbl, Dbl, Dbl, ctypes.c_uint64, P]
        L.odf_quality_workspace.argtypes = [I]
        L.odf_quality_workspace.restype = ctypes.c_size_t
        L.odf_quality_u8.argtypes = [P, P, I, I, I, P, P, P, ctypes.c_size_t, P]
        L.odf_backward_hard_f32.argtypes = [P, P, I, I, I, I, P, P]
        L.odf_softmin_fwd_f32.argtypes = [P, I, I, I, I, I, F, F, P, P]
        L.odf_softmin_bwd_workspace.argtypes = [I, I, I, I, I]
        L.odf_softmin_bwd_workspace.restype = ctypes.c_size_t
        L.odf_softmin_bwd_f32.argtypes = [P, P, I, I, I, I, I, F, F, P, P, ctypes.c_size_t, P]
        L.odf_softmin_bwd_f32_noalloc.argtypes = [P, P, I, I, I, I, I, F, F, P, P]
        L.odf_softmin_fwd_f64.argtypes = [P, I, I, I, I, I, Dbl, Dbl, P, P]
        L.odf_softmin_bwd_f64_workspace.argtypes = [I, I, I, I]
        L.odf_softmin_bwd_f64_workspace.restype = ctypes.c_size_t
        L.odf_softmin_bwd_f64.argtypes = [P, P, I, I, I, I, I, Dbl, Dbl, P, P, ctypes.c_size_t, P]
        for name in ("odf_filter_u8", "odf_filter_f32", "odf_aggregates_f32",
                     "odf_backward_hard_f32", "odf_softmin_fwd_f32", "odf_softmin_bwd_f32",
                     "odf_softmin_bwd_f32_noalloc",
                     "odf_softmin_fwd_f64", "odf_softmin_bwd_f64"):
            getattr(L, name).restype = I
        _lib = L
    return _lib


def declared_functions():
    """Names of the functions declared in include/odf.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(odf_\w+)\s*\(", src, flags=re.M)))


def last_error() -> str:
    return lib().odf_last_error().decode()


def _check(rc):
    if rc != OK:
        raise ODFError(rc, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    if not torch.cuda.is_available():
        return None
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _kind(kind):
    return _KIND[kind.lower()] if isinstance(kind, str) else int(kind)


def _dist(dist):
    return _DIST[dist.lower()] if isinstance(dist, str) else int(dist)


def _as_batch(img):
    if img.dim() == 3:
        return img.unsqueeze(0), True
    if img.dim() != 4 or img.shape[-1] != 3:
        raise ValueError("image must be (M, N, 3) or (B, M, N, 3)")
    return img, False


def _check_tensor(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def check_outputs(img, out, idx):
    """Check caller-supplied outputs of a forward call on ``img`` ((M, N, 3) or
    (B, M, N, 3)) before their pointers go to the kernel, which writes B*M*N*3
    elements of out and B*M*N bytes of idx: out must have img's dtype, device
    and shape (or the batched shape), idx must be uint8 on img's device with
    B*M*N elements; both contiguous.  Raises ValueError."""
    x, _ = _as_batch(img)
    B, M, N, _ = x.shape
    if out is not None:
        if not isinstance(out, torch.Tensor) or out.dtype != x.dtype:
            raise ValueError("out must be a %s tensor like img" % x.dtype)
        if out.device != x.device:
            raise ValueError("out must be on the device of img (%s)" % x.device)
        if tuple(out.shape) not in (tuple(img.shape), tuple(x.shape)):
            raise ValueError("out must have the shape of img %s, not %s"
                             % (tuple(img.shape), tuple(out.shape)))
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
    if idx is not None:
        if not isinstance(idx, torch.Tensor) or idx.dtype != torch.uint8:
            raise ValueError("idx must be a uint8 tensor")
        if idx.device != x.device:
            raise ValueError("idx must be on the device of img (%s)" % x.device)
        if idx.numel() != B * M * N:
            raise ValueError("idx must have B*M*N = %d elements, not %d" % (B * M * N, idx.numel()))
        if not idx.is_contiguous():
            raise ValueError("idx must be contiguous")


def _forward_outputs(img, x, squeeze, out, idx, return_idx):
    """(out, idx) to hand to the kernel (batched views) and (out, idx) to return:
    the caller's own tensors when given, else new ones (unbatched when img is)."""
    check_outputs(img, out, idx)
    B, M, N, _ = x.shape
    if out is None:
        out_k = torch.empty_like(x)
        out_r = out_k[0] if squeeze else out_k
    else:
        out_k, out_r = out, out
    if idx is None and return_idx:
        idx_k = torch.empty((B, M, N), dtype=torch.uint8, device=x.device)
        idx_r = idx_k[0] if squeeze else idx_k
    else:
        idx_k, idx_r = idx, idx
    return out_k, idx_k, out_r, idx_r


def filter(img, window=3, kind=BVDF, p=0.5, dist=EXACT, q=4, out=None, idx=None,
           return_idx=True):
    """Forward filter.  Returns (out, idx) (idx None unless ``return_idx``)."""
    x, squeeze = _as_batch(img)
    _check_tensor(x, "img")
    B, M, N, _ = x.shape
    if x.dtype not in (torch.uint8, torch.float32):
        raise ValueError("img must be uint8 or float32")
    out_k, idx_k, out, idx = _forward_outputs(img, x, squeeze, out, idx, return_idx)
    fn = lib().odf_filter_u8 if x.dtype == torch.uint8 else lib().odf_filter_f32
    _check(fn(_ptr(x), B, M, N, window, _kind(kind), float(p), _dist(dist), q, _ptr(out_k),
              _ptr(idx_k), _stream(x.device)))
    return out, idx


def acwddf(img, window=3, dist=EXACT, q=4, lam=2, T=10.8, out=None, idx=None,
           return_idx=True):
    """Adaptive centre-weighted DDF (Section III, Experiment 2).  Returns
    (out, idx): idx is the DDF selection where the switching statistic exceeds
    T and the centre (n - 1) / 2 elsewhere."""
    x, squeeze = _as_batch(img)
    _check_tensor(x, "img")
    B, M, N, _ = x.shape
    if x.dtype not in (torch.uint8, torch.float32):
        raise ValueError("img must be uint8 or float32")
    out_k, idx_k, out, idx = _forward_outputs(img, x, squeeze, out, idx, return_idx)
    fn = lib().odf_acwddf_u8 if x.dtype == torch.uint8 else lib().odf_acwddf_f32
    _check(fn(_ptr(x), B, M, N, window, _dist(dist), q, int(lam), float(T), _ptr(out_k),
              _ptr(idx_k), _stream(x.device)))
    return out, idx


def cw_filter(img, window=3, kind=CWVMF, level=1, dist=EXACT, q=4, out=None, idx=None,
              return_idx=True):
    """Centre-weighted filter at smoothing level k = ``level`` (Section III,
    eq. 9): CWVMF^k (the weighted L2 sum) or CWDDF^k (the weights on both sums
    of eq. 3).  Returns (out, idx)."""
    x, squeeze = _as_batch(img)
    _check_tensor(x, "img")
    B, M, N, _ = x.shape
    if x.dtype not in (torch.uint8, torch.float32):
        raise ValueError("img must be uint8 or float32")
    out_k, idx_k, out, idx = _forward_outputs(img, x, squeeze, out, idx, return_idx)
    fn = lib().odf_cw_filter_u8 if x.dtype == torch.uint8 else lib().odf_cw_filter_f32
    _check(fn(_ptr(x), B, M, N, window, _kind(kind), _dist(dist), q, int(level), _ptr(out_k),
              _ptr(idx_k), _stream(x.device)))
    return out, idx


def noise_eq8(img, phi, phi_rgb=(0.25, 0.25, 0.25), seed=0, out=None):
    """eq. (8) impulsive noise on uint8 images (Philox4x32-10 draws keyed by
    ``seed``, counter = flat pixel index).  ``out`` may be ``img`` itself."""
    x, squeeze = _as_batch(img)
    _check_tensor(x, "img")
    if x.dtype != torch.uint8:
        raise ValueError("img must be uint8")
    B, M, N, _ = x.shape
    if out is None:
        out = torch.empty_like(img)
    o = out if out.dim() == 4 else out[None]
    _check_tensor(o, "out")
    if o.shape != x.shape or o.dtype != torch.uint8:
        raise ValueError("out must be a uint8 image of the shape of img")
    _check(lib().odf_noise_eq8_u8(_ptr(x), _ptr(o), B, M, N, float(phi), float(phi_rgb[0]),
                                  float(phi_rgb[1]), float(phi_rgb[2]), int(seed),
                                  _stream(x.device)))
    return out


def quality(y, ref, workspace=None):
    """MAE and PSNR of uint8 images y against ref: two float64 tensors (B,)."""
    a, _ = _as_batch(y)
    b, _ = _as_batch(ref)
    _check_tensor(a, "y")
    _check_tensor(b, "ref")
    if a.shape != b.shape or a.dtype != torch.uint8 or b.dtype != torch.uint8:
        raise ValueError("y and ref must be uint8 images of one shape")
    B, M, N, _ = a.shape
    mae = torch.empty(B, dtype=torch.float64, device=a.device)
    psnr = torch.empty_like(mae)
    nbytes = lib().odf_quality_workspace(B)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=a.device)
    _check(lib().odf_quality_u8(_ptr(a), _ptr(b), B, M, N, _ptr(mae), _ptr(psnr), _ptr(workspace),
                                workspace.numel() * workspace.element_size(), _stream(a.device)))
    return mae, psnr


def aggregates(img, window=3, kind=BVDF, p=0.5, dist=EXACT, q=4):
    """Per-window aggregates (A, D, Omega), each (..., n) float32 (test hook)."""
    x, squeeze = _as_batch(img)
    _check_tensor(x, "img")
    B, M, N, _ = x.shape
    n = window * window
    A = torch.empty((B, M, N, n), dtype=torch.float32, device=x.device)
    D = torch.empty_like(A)
    O = torch.empty_like(A)
    _check(lib().odf_aggregates_f32(_ptr(x), int(x.dtype == torch.uint8), B, M, N, window,
                                _kind(kind), float(p), _dist(dist), q, _ptr(A), _ptr(D), _ptr(O),
                                _stream(x.device)))
    if squeeze:
        A, D, O = A[0], D[0], O[0]
    return A, D, O


# ------------------------------------------------------------------ gradients

def backward_hard(idx, dy, window):
    """Gradient of the hard filter: dy routed to the selected pixels (float32)."""
    g, squeeze = _as_batch(dy)
    _check_tensor(g, "dy")
    _check_tensor(idx, "idx")
    if g.dtype != torch.float32 or idx.dtype != torch.uint8:
        raise ValueError("dy must be float32 and idx uint8")
    B, M, N, _ = g.shape
    if idx.numel() != B * M * N:
        raise ValueError("idx must have B*M*N elements")
    dx = torch.empty_like(g)
    _check(lib().odf_backward_hard_f32(_ptr(idx), _ptr(g), B, M, N, window, _ptr(dx),
                                       _stream(g.device)))
    return dx[0] if squeeze else dx


def softmin_forward(x, window=5, kind=DDF, p=0.25, tau=0.1):
    """Softmin relaxation y = sum_u pi_u x_u (exact angle): float32 on the fast
    path, float64 on the binary64 twin (for gradient checks)."""
    xb, squeeze = _as_batch(x)
    _check_tensor(xb, "x")
    if xb.dtype not in (torch.float32, torch.float64):
        raise ValueError("x must be float32 or float64")
    B, M, N, _ = xb.shape
    y = torch.empty_like(xb)
    if xb.dtype == torch.float32:
        _check(lib().odf_softmin_fwd_f32(_ptr(xb), B, M, N, window, _kind(kind), float(p),
                                         float(tau), _ptr(y), _stream(xb.device)))
    else:
        _check(lib().odf_softmin_fwd_f64(_ptr(xb), B, M, N, window, _kind(kind), float(p),
                                         float(tau), _ptr(y), _stream(xb.device)))
    return y[0] if squeeze else y


def softmin_backward(x, dy, window=5, kind=DDF, p=0.25, tau=0.1, workspace=None):
    """Gradient of sum(dy * softmin_forward(x)) with respect to x (float32, or
    float64 on the binary64 twin)."""
    xb, squeeze = _as_batch(x)
    g, _ = _as_batch(dy)
    _check_tensor(xb, "x")
    _check_tensor(g, "dy")
    if xb.dtype not in (torch.float32, torch.float64) or g.dtype != xb.dtype or \
            g.shape != xb.shape:
        raise ValueError("x and dy must be float32 (or both float64) of the same shape")
    B, M, N, _ = xb.shape
    f64 = xb.dtype == torch.float64
    L = lib()
    need = (L.odf_softmin_bwd_f64_workspace(B, M, N, window) if f64
            else L.odf_softmin_bwd_workspace(B, M, N, window, _kind(kind)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=xb.device)
    dx = torch.empty_like(xb)
    fn = L.odf_softmin_bwd_f64 if f64 else L.odf_softmin_bwd_f32
    _check(fn(_ptr(xb), _ptr(g), B, M, N, window, _kind(kind), float(p), float(tau), _ptr(dx),
              _ptr(workspace), workspace.numel(), _stream(xb.device)))
    return dx[0] if squeeze else dx


def softmin_backward_noalloc(x, dy, window=5, kind=DDF, p=0.25, tau=0.1, dx=None):
    """softmin_backward (float32) on the library's static device scratch instead of a
    workspace: for callers that cannot allocate (e.g. under graph capture, with
    ``dx`` given).  Shapes needing more than 128 MiB of workspace are rejected."""
    xb, squeeze = _as_batch(x)
    g, _ = _as_batch(dy)
    _check_tensor(xb, "x")
    _check_tensor(g, "dy")
    if xb.dtype != torch.float32 or g.dtype != torch.float32 or g.shape != xb.shape:
        raise ValueError("x and dy must be float32 of the same shape")
    B, M, N, _ = xb.shape
    if dx is None:
        dx = torch.empty_like(x)
    dxb = dx if dx.dim() == 4 else dx[None]
    _check_tensor(dxb, "dx")
    if dxb.shape != xb.shape or dxb.dtype != torch.float32 or dxb.device != xb.device:
        raise ValueError("dx must be a float32 tensor of the shape of x on its device")
    _check(lib().odf_softmin_bwd_f32_noalloc(_ptr(xb), _ptr(g), B, M, N, window, _kind(kind),
                                             float(p), float(tau), _ptr(dxb), _stream(xb.device)))
    return dx


class HardFilter(torch.autograd.Function):
    """y = filter(x) with the one-hot backward of the selection."""

    @staticmethod
    def forward(ctx, x, window, kind, p, dist, q):
        out, idx = filter(x.contiguous(), window, kind, p, dist, q)
        ctx.save_for_backward(idx)
        ctx.window = window
        ctx.mark_non_differentiable(idx)
        return out, idx

    @staticmethod
    def backward(ctx, gy, gidx):
        (idx,) = ctx.saved_tensors
        return backward_hard(idx, gy.contiguous(), ctx.window), None, None, None, None, None


class SoftminFilter(torch.autograd.Function):
    """y = softmin relaxation of the filter, differentiable through A and D."""

    @staticmethod
    def forward(ctx, x, window, kind, p, tau):
        x = x.contiguous()
        ctx.save_for_backward(x)
        ctx.args = (window, kind, p, tau)
        return softmin_forward(x, window, kind, p, tau)

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        window, kind, p, tau = ctx.args
        return softmin_backward(x, gy.contiguous(), window, kind, p, tau), None, None, None, None


def hard_filter(x, window=5, kind=DDF, p=0.25, dist=EXACT, q=4):
    """Differentiable hard filter on float32 images: returns (y, idx)."""
    return HardFilter.apply(x, window, _kind(kind), float(p), _dist(dist), q)


def softmin_filter(x, window=5, kind=DDF, p=0.25, tau=0.1):
    """Differentiable softmin relaxation on float32 images (float64: the binary64
    twin, e.g. for torch.autograd.gradcheck)."""
    return SoftminFilter.apply(x, window, _kind(kind), float(p), float(tau))


# ------------------------------------------------------------------ batches

class _Job(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p), ("idx", ctypes.c_void_p),
                ("M", ctypes.c_int), ("N", ctypes.c_int), ("window", ctypes.c_int),
                ("kind", ctypes.c_int), ("dist", ctypes.c_int), ("q", ctypes.c_int),
                ("p", ctypes.c_float)]


def _batch_lib():
    L = lib()
    if not hasattr(L, "_batch_ready"):
        P, I = ctypes.c_void_p, ctypes.c_int
        L.odf_batch_plan.argtypes = [P, I, ctypes.POINTER(ctypes.c_void_p), P]
        L.odf_batch_plan_ex.argtypes = [P, I, I, ctypes.POINTER(ctypes.c_void_p), P]
        L.odf_batch_launch.argtypes = [P, P]
        L.odf_plan_info.argtypes = [P, P, P, P, P]
        L.odf_plan_destroy.argtypes = [P]
        L.odf_tile_config.argtypes = [I, P, P]
        L.odf_tune_get.argtypes = [I, I, I, I]
        L.odf_tune_set.argtypes = [I, I, I, I, I]
        L.odf_autotune.argtypes = [I, I, I, I, I, I, I, ctypes.c_char_p, P, P]
        L.odf_tune_load.argtypes = [ctypes.c_char_p]
        L.odf_plan_configs.argtypes = [P, P]
        L.odf_batch_tune_get.argtypes = [I, I]
        L.odf_batch_tune_set.argtypes = [I, I, I]
        L.odf_autotune_batch.argtypes = [I, I, I, ctypes.c_char_p, P, P]
        L.odf_autotune_batch_jobs.argtypes = [P, I, I, ctypes.c_char_p, P, P]
        for name in ("odf_batch_plan", "odf_batch_plan_ex", "odf_batch_launch", "odf_plan_info",
                     "odf_plan_destroy", "odf_plan_configs", "odf_tile_config", "odf_tune_get",
                     "odf_tune_set", "odf_autotune", "odf_tune_load", "odf_batch_tune_get",
                     "odf_batch_tune_set", "odf_autotune_batch", "odf_autotune_batch_jobs"):
            getattr(L, name).restype = I
        L._batch_ready = True
    return L


NUM_BATCH_GROUPS = 8  # ((window - 3) / 2) * 2 + kind, windows 3, 5, 7, 9
NUM_CLASSES = 3 * NUM_BATCH_GROUPS  # group * 3 + dist


def _job_array(jobs):
    """The C job array of a list of job dicts (checked), and the tensors it
    points into (kept alive by the caller)."""
    keep = []
    arr = (_Job * len(jobs))()
    for i, j in enumerate(jobs):
        img, out, idx = j["img"], j["out"], j.get("idx")
        for t, name in ((img, "img"), (out, "out")):
            _check_tensor(t, name)
            if t.dtype != torch.uint8 or t.dim() != 3 or t.shape[-1] != 3:
                raise ValueError("batch %s must be an (M, N, 3) uint8 tensor" % name)
        if out.shape != img.shape:
            raise ValueError("out must have the shape of img")
        if idx is not None:
            _check_tensor(idx, "idx")
            if idx.dtype != torch.uint8 or idx.numel() != img.shape[0] * img.shape[1]:
                raise ValueError("idx must be uint8 with M*N elements")
        keep.extend([img, out, idx])
        M, N, _ = img.shape
        arr[i] = _Job(img.data_ptr(), out.data_ptr(), 0 if idx is None else idx.data_ptr(),
                      M, N, int(j.get("window", 3)), _kind(j.get("kind", BVDF)),
                      _dist(j.get("dist", EXACT)), int(j.get("q", 4)), float(j.get("p", 0.5)))
    return arr, keep


class BatchPlan:
    """A planned batch of uint8 jobs; ``launch()`` enqueues it on the current
    stream (graph-capturable), ``capture()`` records it in a CUDA/HIP graph.

    jobs: iterable of dicts with keys img, out, idx (tensors; idx may be None),
    window, kind, p, dist, q.  One workgroup per tile, on each group's shape
    from the batch tuning table (``batch_tune_get``, ``autotune_batch``).
    """

    def __init__(self, jobs):
        arr, self._keep = _job_array(jobs)
        self._jobs = arr
        self._plan = ctypes.c_void_p()
        L = _batch_lib()
        _check(L.odf_batch_plan(ctypes.cast(arr, ctypes.c_void_p), len(jobs),
                                ctypes.byref(self._plan), _stream(torch.cuda.current_device())))

    def launch(self):
        _check(_batch_lib().odf_batch_launch(self._plan, _stream(torch.cuda.current_device())))

    def capture(self):
        """Record one launch in a graph (replay with ``graph.replay()``)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch()
        return g

    def info(self):
        nj = ctypes.c_int()
        npix = ctypes.c_longlong()
        tiles = (ctypes.c_int * NUM_CLASSES)()
        grids = (ctypes.c_int * NUM_CLASSES)()
        _check(_batch_lib().odf_plan_info(self._plan, ctypes.byref(nj), ctypes.byref(npix),
                                          ctypes.cast(tiles, ctypes.c_void_p),
                                          ctypes.cast(grids, ctypes.c_void_p)))
        cfg = (ctypes.c_int * NUM_BATCH_GROUPS)()
        _check(_batch_lib().odf_plan_configs(self._plan, ctypes.cast(cfg, ctypes.c_void_p)))
        return {"jobs": nj.value, "pixels": npix.value, "tiles": list(tiles), "grids": list(grids),
                "configs": list(cfg),
                "ext_tiles": {"w%d_%s" % (3 + 2 * (g // 2), ("bvdf", "ddf")[g % 2]):
                              tile_config(cfg[g]) for g in range(NUM_BATCH_GROUPS)}}

    def close(self):
        if self._plan:
            _batch_lib().odf_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ tuning

def tile_config(config):
    w, h = ctypes.c_int(), ctypes.c_int()
    _check(_batch_lib().odf_tile_config(config, ctypes.byref(w), ctypes.byref(h)))
    return w.value, h.value


def tune_get(window, kind, dist, is_u8=True):
    return _batch_lib().odf_tune_get(window, _kind(kind), _dist(dist), int(is_u8))


def tune_set(window, kind, dist, is_u8, config):
    _check(_batch_lib().odf_tune_set(window, _kind(kind), _dist(dist), int(is_u8), config))


def autotune(window, kind, dist, is_u8=True, M=1024, N=1024, reps=10, cache_path=None):
    """Time every forward config (the four tile shapes and the two strip
    heights), keep the fastest; returns (best, [ms per config], -1 where not
    offered)."""
    times = (ctypes.c_float * NUM_TILE_CONFIGS)()
    path = None if cache_path is None else cache_path.encode()
    _check(_batch_lib().odf_autotune(window, _kind(kind), _dist(dist), int(is_u8), M, N, reps,
                                     path, ctypes.cast(times, ctypes.c_void_p),
                                     _stream(torch.cuda.current_device())))
    return tune_get(window, kind, dist, is_u8), list(times)


def batch_tune_get(window, kind):
    rc = _batch_lib().odf_batch_tune_get(window, _kind(kind))
    if rc < 0:
        raise ODFError(rc, "no batch group for window %d kind %s" % (window, kind))
    return rc


def batch_tune_set(window, kind, config):
    _check(_batch_lib().odf_batch_tune_set(window, _kind(kind), config))


def autotune_batch(window, kind, reps=3, cache_path=None):
    """Time the batch group's configs (four tile shapes, two strip heights) on a
    mixed work list, keep the fastest; returns (best, [ms per config])."""
    times = (ctypes.c_float * NUM_TILE_CONFIGS)()
    path = None if cache_path is None else cache_path.encode()
    _check(_batch_lib().odf_autotune_batch(window, _kind(kind), reps, path,
                                           ctypes.cast(times, ctypes.c_void_p),
                                           _stream(torch.cuda.current_device())))
    return batch_tune_get(window, kind), list(times)


def autotune_batch_jobs(jobs, reps=2, cache_path=None):
    """Time every batch group's configs on these jobs (their outputs are
    written), keep the fastest per group; returns {group name: (best,
    [ms per config])} for the groups that hold jobs."""
    arr, keep = _job_array(jobs)
    C = NUM_TILE_CONFIGS
    times = (ctypes.c_float * (NUM_BATCH_GROUPS * C))()
    path = None if cache_path is None else cache_path.encode()
    _check(_batch_lib().odf_autotune_batch_jobs(ctypes.cast(arr, ctypes.c_void_p), len(jobs), reps,
                                                path, ctypes.cast(times, ctypes.c_void_p),
                                                _stream(torch.cuda.current_device())))
    res = {}
    for g in range(NUM_BATCH_GROUPS):
        ms = list(times[C * g:C * g + C])
        if any(m >= 0 for m in ms):
            w, k = 3 + 2 * (g // 2), g % 2
            res["w%d_%s" % (w, ("bvdf", "ddf")[k])] = (batch_tune_get(w, k), ms)
    del keep
    return res


def tune_load(cache_path):
    """Apply a tuning cache; returns the number of entries applied."""
    rc = _batch_lib().odf_tune_load(cache_path.encode())
    if rc < 0:
        raise ODFError(rc, "cannot read tuning cache %s" % cache_path)
    return rc
