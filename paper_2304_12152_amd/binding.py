"""ctypes binding of libhalftone with the names of the C entry points.

Argument marshalling only: every step runs in the HIP library. torch supplies
device memory (outputs and workspaces) and the current stream. If the
library is not built, or the device is not a gfx950, calls fail loudly.
"""
import ctypes
import os

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhalftone.so")

HS_OK, HS_EINVAL, HS_ESHAPE, HS_EUNSUPPORTED, HS_EWORKSPACE, HS_EHIP = 0, -1, -2, -3, -4, -5
HS_ENONFINITE = -6
HS_CHECK_FINITE = 0x100
HS_FP32, HS_BF16, HS_FP16, HS_FP8 = 0, 1, 2, 3
HS_NOISE_GAUSS, HS_NOISE_UNIFORM = 0, 1
HS_WRT_PROB, HS_WRT_LOGIT = 0, 1
HS_EST_LE, HS_EST_COMA = 0, 1
HS_PARAM_COUNT = 37889
HS_MAX_LEVELS = 8


class HsLossParams(ctypes.Structure):
    _fields_ = [("w_s", ctypes.c_float), ("w_a", ctypes.c_float), ("hvs_sigma", ctypes.c_float),
                ("hvs_radius", ctypes.c_int), ("ssim_sigma", ctypes.c_float),
                ("ssim_radius", ctypes.c_int), ("k", ctypes.c_float), ("c1", ctypes.c_float),
                ("c2", ctypes.c_float), ("as_patch", ctypes.c_int), ("estimator", ctypes.c_int),
                ("levels", ctypes.c_int), ("flags", ctypes.c_int)]


class HsTrainParams(ctypes.Structure):
    _fields_ = [("loss", HsLossParams), ("lr_max", ctypes.c_float), ("lr_min", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("noise_kind", ctypes.c_int), ("recompute", ctypes.c_int)]


class HsPolicy(ctypes.Structure):
    _fields_ = [("mem", ctypes.c_void_p), ("bytes", ctypes.c_size_t), ("packed", ctypes.c_int),
                ("fp8", ctypes.c_int)]


class HalftoneError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libhalftone error %d: %s" % (code, msg))
        self.code = code


_lib = None
P = ctypes.c_void_p
I = ctypes.c_int
SZ = ctypes.c_size_t
F = ctypes.c_float

_SIGS = {
    "halftone_default_loss_params": (None, [ctypes.POINTER(HsLossParams)]),
    "halftone_default_train_params": (None, [ctypes.POINTER(HsTrainParams)]),
    "halftone_version": (I, []),
    "halftone_last_error": (ctypes.c_char_p, []),
    "halftone_param_count": (ctypes.c_int64, []),
    "halftone_infer_workspace_size": (SZ, [I, I, I, I]),
    "halftone_infer": (I, [P, P, P, I, I, I, I, I, F, P, P, P, P, SZ, P]),
    "halftone_infer_noalloc": (I, [P, P, P, I, I, I, I, I, F, P, P, P, P]),
    "halftone_infer_pages_workspace_size": (SZ, [I, P, I]),
    "halftone_infer_pages": (I, [P, P, P, I, P, I, I, F, P, P, P, P, SZ, P]),
    "halftone_infer_levels": (I, [P, P, P, I, P, I, I, I, F, P, P, P, P, SZ, P]),
    "halftone_policy_bytes": (SZ, []),
    "halftone_policy_pack": (I, [ctypes.POINTER(HsPolicy), P, P, SZ, I, P]),
    "halftone_policy_infer": (I, [ctypes.POINTER(HsPolicy), P, P, I, P, I, I, I, F, F, F, P, P, P,
                                  P, SZ, P]),
    "halftone_layer_max": (I, [P, P, P, I, I, I, I, P, P, SZ, P]),
    "halftone_policy_set_fp8": (I, [ctypes.POINTER(HsPolicy), P, P]),
    "halftone_policy_workspace_size": (SZ, [I, I, I, I]),
    "halftone_policy_forward": (I, [P, P, P, I, I, I, I, ctypes.c_uint32, I, P, P, SZ, P]),
    "halftone_policy_backward": (I, [P, P, P, I, I, I, I, P, P, SZ, P]),
    "halftone_loss_workspace_size": (SZ, [I, I, I, I, I, I, ctypes.POINTER(HsLossParams)]),
    "halftone_loss": (I, [P, P, I, I, I, P, I, I, I, ctypes.POINTER(HsLossParams), P, P, SZ, P]),
    "halftone_loss_backward": (I, [P, P, P, I, I, I, P, I, I, I, ctypes.POINTER(HsLossParams), I,
                                   P, P, P, SZ, P]),
    "halftone_train_workspace_size": (SZ, [I, I, I, I, I, I, I]),
    "halftone_train_workspace_size_params": (SZ, [I, I, I, I, I, I, I,
                                                  ctypes.POINTER(HsTrainParams)]),
    "policy_train_step": (I, [P, P, P, P, P, I, I, I, P, P, I, I, I, ctypes.c_int64,
                              ctypes.c_int64, ctypes.POINTER(HsTrainParams), I, P, P, P, P, SZ,
                              P]),
    "halftone_error_diffusion_host": (I, [P, I, I, I, P]),
    "halftone_error_diffusion_levels_host": (I, [P, I, I, I, I, P]),
    "halftone_spectrum_rings": (I, [I]),
    "halftone_spectrum_workspace_size": (SZ, [I, I, I, I]),
    "halftone_spectrum": (I, [P, I, I, I, I, P, P, P, SZ, P]),
    "halftone_profile_start": (I, []),
    "halftone_profile_stop": (I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
}


def lib():
    """Load libhalftone.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhalftone.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != HS_OK:
        raise HalftoneError(rc, lib().halftone_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
    return t


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def default_loss_params(**kw):
    p = HsLossParams()
    lib().halftone_default_loss_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def default_train_params(**kw):
    p = HsTrainParams()
    lib().halftone_default_train_params(ctypes.byref(p))
    loss_kw = {k: v for k, v in kw.items() if k in dict(HsLossParams._fields_)}
    for k, v in loss_kw.items():
        setattr(p.loss, k, v)
    for k, v in kw.items():
        if k not in loss_kw:
            setattr(p, k, v)
    return p


# recheck band per precision: about 1.3 times the largest logit error of the
# fused pass measured on the C2 batch (BF16 0.042, FP16 0.0056)
RECHECK_TAU = {HS_FP32: 0.0, HS_BF16: 0.055, HS_FP16: 0.0075}


def _tau(precision, recheck_tau):
    return RECHECK_TAU.get(precision, 0.0) if recheck_tau is None else recheck_tau


def halftone_infer(weights, contone, seeds, noise_kind=HS_NOISE_GAUSS, precision=HS_BF16,
                   recheck_tau=None, logits=False, stats=False, workspace=None):
    """bits [B,H,W] uint8 (and optionally logits, and stats =
    (rechecked, flipped, recomputed in FP32, FP16 overflow re-run,
    recomputed by the split stage, 0, 0, 0)).
    recheck_tau None: the band of RECHECK_TAU for the precision."""
    recheck_tau = _tau(precision, recheck_tau)
    B, H, W = contone.shape
    dev = contone.device
    _dev(weights, torch.float32), _dev(contone, torch.float32), _dev(seeds, torch.int64)
    bits = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
    lg = torch.empty((B, H, W), dtype=torch.float32, device=dev) if logits else None
    st = torch.zeros(8, dtype=torch.int32, device=dev) if stats else None
    need = lib().halftone_infer_workspace_size(B, H, W, precision)
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    _check(lib().halftone_infer(_ptr(weights), _ptr(contone), _ptr(seeds), B, H, W, noise_kind,
                                precision, recheck_tau, _ptr(bits), _ptr(lg), _ptr(st), _ptr(ws),
                                ws.numel(), _stream()))
    out = [bits]
    if logits:
        out.append(lg)
    if stats:
        out.append(st)
    return out[0] if len(out) == 1 else tuple(out)


def halftone_infer_noalloc(weights, contone, seeds, noise_kind=HS_NOISE_GAUSS, precision=HS_BF16,
                           recheck_tau=None, logits=False, stats=False):
    """halftone_infer without a workspace (the library's static scratch):
    bits [B,H,W] uint8, and optionally logits and stats."""
    recheck_tau = _tau(precision, recheck_tau)
    B, H, W = contone.shape
    dev = contone.device
    _dev(weights, torch.float32), _dev(contone, torch.float32), _dev(seeds, torch.int64)
    bits = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
    lg = torch.empty((B, H, W), dtype=torch.float32, device=dev) if logits else None
    st = torch.zeros(8, dtype=torch.int32, device=dev) if stats else None
    _check(lib().halftone_infer_noalloc(_ptr(weights), _ptr(contone), _ptr(seeds), B, H, W,
                                        noise_kind, precision, recheck_tau, _ptr(bits), _ptr(lg),
                                        _ptr(st), _stream()))
    out = [bits]
    if logits:
        out.append(lg)
    if stats:
        out.append(st)
    return out[0] if len(out) == 1 else tuple(out)


def page_shapes_array(shapes):
    """int32 [npages][2] host array of (H, W) pairs."""
    return np.ascontiguousarray(np.asarray(shapes, dtype=np.int32).reshape(-1, 2))


def halftone_infer_pages(weights, contone, seeds, shapes, noise_kind=HS_NOISE_GAUSS,
                         precision=HS_BF16, recheck_tau=None, logits=False, stats=False,
                         workspace=None, levels=None):
    """Pages of different sizes in one call. contone: flat FP32 device tensor
    of the pages concatenated (page p at offset sum of the earlier H*W);
    shapes: (H, W) per page; returns flat bits (and logits, stats). With
    `levels` (2..HS_MAX_LEVELS) the multitone call halftone_infer_levels:
    level indices instead of bits."""
    recheck_tau = _tau(precision, recheck_tau)
    sh = page_shapes_array(shapes)
    n = sh.shape[0]
    N = int((sh[:, 0].astype("int64") * sh[:, 1]).sum())
    dev = contone.device
    _dev(weights, torch.float32), _dev(contone, torch.float32), _dev(seeds, torch.int64)
    assert contone.numel() == N and seeds.numel() == n, (contone.numel(), N, seeds.numel(), n)
    bits = torch.empty(N, dtype=torch.uint8, device=dev)
    lg = torch.empty(N, dtype=torch.float32, device=dev) if logits else None
    st = torch.zeros(8, dtype=torch.int32, device=dev) if stats else None
    shp = sh.ctypes.data_as(ctypes.c_void_p)
    need = lib().halftone_infer_pages_workspace_size(n, shp, precision)
    if need == 0:
        raise HalftoneError(HS_ESHAPE, "bad page shapes")
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    if levels is None:
        _check(lib().halftone_infer_pages(_ptr(weights), _ptr(contone), _ptr(seeds), n, shp,
                                          noise_kind, precision, recheck_tau, _ptr(bits),
                                          _ptr(lg), _ptr(st), _ptr(ws), ws.numel(), _stream()))
    else:
        _check(lib().halftone_infer_levels(_ptr(weights), _ptr(contone), _ptr(seeds), n, shp,
                                           int(levels), noise_kind, precision, recheck_tau,
                                           _ptr(bits), _ptr(lg), _ptr(st), _ptr(ws), ws.numel(),
                                           _stream()))
    out = [bits]
    if logits:
        out.append(lg)
    if stats:
        out.append(st)
    return out[0] if len(out) == 1 else tuple(out)


class Policy:
    """A packed inference policy (halftone_policy_pack): the weights and all
    their derived copies in one device buffer owned by this object."""

    def __init__(self, weights, check_finite=False):
        _dev(weights, torch.float32)
        n = lib().halftone_policy_bytes()
        self.mem = torch.empty(n, dtype=torch.uint8, device=weights.device)
        self.handle = HsPolicy()
        _check(lib().halftone_policy_pack(ctypes.byref(self.handle), _ptr(weights), _ptr(self.mem),
                                          n, HS_CHECK_FINITE if check_finite else 0, _stream()))
        self.act_max = None

    def set_fp8(self, act_max):
        """halftone_policy_set_fp8: the FP8 copy from the calibrated maxima
        of layers 1..4's activations (4 floats, e.g. the first four of
        halftone_layer_max on calibration images)."""
        a = np.ascontiguousarray(np.asarray(act_max, dtype=np.float32)[:4])
        assert a.shape == (4,)
        _check(lib().halftone_policy_set_fp8(ctypes.byref(self.handle),
                                             a.ctypes.data_as(ctypes.c_void_p), _stream()))
        self.act_max = a.copy()
        return self


def halftone_layer_max(weights, contone, seeds, noise_kind=HS_NOISE_GAUSS, workspace=None):
    """The largest activation of layers 1..5 of the FP32 forward over the
    batch contone [B,H,W]: a float32 tensor of 5 on the device."""
    _dev(weights, torch.float32), _dev(contone, torch.float32), _dev(seeds, torch.int64)
    B, H, W = contone.shape
    out = torch.empty(5, dtype=torch.float32, device=contone.device)
    need = lib().halftone_infer_workspace_size(B, H, W, HS_FP32)
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, contone.device)
    _check(lib().halftone_layer_max(_ptr(weights), _ptr(contone), _ptr(seeds), B, H, W, noise_kind,
                                    _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def halftone_policy_infer(policy, contone, seeds, shapes=None, noise_kind=HS_NOISE_GAUSS,
                          precision=HS_BF16, recheck_tau=None, recheck_tau16=-1.0,
                          recheck_tau2=-1.0, logits=False, stats=False, workspace=None, levels=2):
    """halftone_policy_infer on a packed Policy. contone: [B,H,W] (a uniform
    batch) or the flat concatenation of pages with `shapes`; the outputs
    have the contone's shape. The cone stages' bands recheck_tau16 and
    recheck_tau2: -1 for the default rules. HS_FP8 needs policy.set_fp8 and
    an explicit recheck_tau (calibrate.bands)."""
    if precision == HS_FP8 and recheck_tau is None:
        raise ValueError("HS_FP8 has no default band: pass recheck_tau (calibrate.bands)")
    recheck_tau = _tau(precision, recheck_tau)
    if shapes is None:
        B, H, W = contone.shape
        shapes = [(H, W)] * B
    sh = page_shapes_array(shapes)
    n = sh.shape[0]
    dev = contone.device
    _dev(contone, torch.float32), _dev(seeds, torch.int64)
    assert seeds.numel() == n
    out = torch.empty(contone.shape, dtype=torch.uint8, device=dev)
    lg = torch.empty(contone.shape, dtype=torch.float32, device=dev) if logits else None
    st = torch.zeros(8, dtype=torch.int32, device=dev) if stats else None
    shp = sh.ctypes.data_as(ctypes.c_void_p)
    need = lib().halftone_infer_pages_workspace_size(n, shp, precision)
    if need == 0:
        raise HalftoneError(HS_ESHAPE, "bad page shapes")
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    _check(lib().halftone_policy_infer(ctypes.byref(policy.handle), _ptr(contone), _ptr(seeds), n,
                                       shp, int(levels), noise_kind, precision, recheck_tau,
                                       recheck_tau16, recheck_tau2, _ptr(out), _ptr(lg), _ptr(st),
                                       _ptr(ws),
                                       ws.numel(), _stream()))
    res = [out]
    if logits:
        res.append(lg)
    if stats:
        res.append(st)
    return res[0] if len(res) == 1 else tuple(res)


def halftone_policy_forward(weights, contone, seeds, step=0, noise_kind=HS_NOISE_GAUSS,
                            precision=HS_FP32, workspace=None):
    """probs [B,H,W] and the workspace holding the saved activations."""
    B, H, W = contone.shape
    dev = contone.device
    probs = torch.empty((B, H, W), dtype=torch.float32, device=dev)
    need = lib().halftone_policy_workspace_size(B, H, W, precision)
    ws = workspace if workspace is not None and workspace.numel() >= need else _ws(need, dev)
    _check(lib().halftone_policy_forward(_ptr(weights), _ptr(contone), _ptr(seeds), B, H, W,
                                         noise_kind, step, precision, _ptr(probs), _ptr(ws),
                                         ws.numel(), _stream()))
    return probs, ws


def halftone_policy_backward(weights, grad_probs, probs, workspace, precision=HS_FP32):
    B, H, W = probs.shape
    gw = torch.empty(HS_PARAM_COUNT, dtype=torch.float32, device=probs.device)
    _check(lib().halftone_policy_backward(_ptr(weights), _ptr(grad_probs.contiguous()),
                                          _ptr(probs), B, H, W, precision, _ptr(gw),
                                          _ptr(workspace), workspace.numel(), _stream()))
    return gw


def halftone_loss(actions, contone, probs_gray=None, prm=None):
    """Tensor [3B+2]: per image (MSE, CSSIM, R), then L_AS, then the total
    loss -mean(R) + w_a L_AS."""
    prm = prm or default_loss_params()
    B, H, W = contone.shape
    Bg, Hg, Wg = probs_gray.shape if probs_gray is not None else (0, 0, 0)
    out = torch.empty(3 * B + 2, dtype=torch.float32, device=contone.device)
    need = lib().halftone_loss_workspace_size(B, H, W, Bg, Hg, Wg, ctypes.byref(prm))
    ws = _ws(need, contone.device)
    _check(lib().halftone_loss(_ptr(actions), _ptr(contone), B, H, W, _ptr(probs_gray), Bg, Hg,
                               Wg, ctypes.byref(prm), _ptr(out), _ptr(ws), ws.numel(),
                               _stream()))
    return out


def halftone_loss_backward(actions, contone, probs=None, probs_gray=None, prm=None,
                           grad_space=HS_WRT_PROB, workspace=None, out=None):
    """(grad_probs, grad_probs_gray or None). out: a (grad_probs,
    grad_probs_gray) pair to write into instead of new tensors; workspace: a
    uint8 device tensor reused when large enough."""
    prm = prm or default_loss_params()
    B, H, W = contone.shape
    Bg, Hg, Wg = probs_gray.shape if probs_gray is not None else (0, 0, 0)
    if out is not None:
        gp, gg = out
        _dev(gp, torch.float32)
        assert tuple(gp.shape) == (B, H, W)
        if probs_gray is not None:
            _dev(gg, torch.float32)
            assert tuple(gg.shape) == (Bg, Hg, Wg)
    else:
        gp = torch.empty((B, H, W), dtype=torch.float32, device=contone.device)
        gg = torch.empty((Bg, Hg, Wg), dtype=torch.float32, device=contone.device) \
            if probs_gray is not None else None
    need = lib().halftone_loss_workspace_size(B, H, W, Bg, Hg, Wg, ctypes.byref(prm))
    ws = workspace if workspace is not None and workspace.numel() >= need else \
        _ws(need, contone.device)
    _check(lib().halftone_loss_backward(_ptr(actions), _ptr(contone), _ptr(probs), B, H, W,
                                        _ptr(probs_gray), Bg, Hg, Wg, ctypes.byref(prm),
                                        grad_space, _ptr(gp), _ptr(gg), _ptr(ws), ws.numel(),
                                        _stream()))
    return gp, gg


class TrainState:
    """FP32 master weights and Adam moments on the device, plus a workspace."""

    def __init__(self, weights, B, H, W, Bg=0, Hg=0, Wg=0, precision=HS_BF16, tp=None):
        dev = weights.device
        self.weights = weights.clone()
        self.m = torch.zeros_like(self.weights)
        self.v = torch.zeros_like(self.weights)
        self.precision = precision
        self.tp = tp or default_train_params()
        self.shape = (B, H, W, Bg, Hg, Wg)
        need = lib().halftone_train_workspace_size_params(B, H, W, Bg, Hg, Wg, precision,
                                                          ctypes.byref(self.tp))
        self.ws = _ws(need, dev)
        self.metrics = torch.zeros(8, dtype=torch.float32, device=dev)


def policy_train_step(state, contones, seeds, gray, gray_seeds, step, total_steps,
                      actions_out=None, grad_out=None):
    B, H, W = contones.shape
    if gray is not None:
        Bg, Hg, Wg = gray.shape
    else:
        Bg = Hg = Wg = 0
    _check(lib().policy_train_step(_ptr(state.weights), _ptr(state.m), _ptr(state.v),
                                   _ptr(contones), _ptr(seeds), B, H, W, _ptr(gray),
                                   _ptr(gray_seeds), Bg, Hg, Wg, step, total_steps,
                                   ctypes.byref(state.tp), state.precision, _ptr(state.metrics),
                                   _ptr(actions_out), _ptr(grad_out), _ptr(state.ws),
                                   state.ws.numel(), _stream()))
    return state.metrics


def halftone_spectrum(bits, P=32):
    """(RAPSD, anisotropy) per ring of the mean periodogram over the P x P
    patches of bits (uint8 [B][H][W] or [H][W] on the GPU), FP32 tensors."""
    _dev(bits, torch.uint8)
    B, H, W = bits.shape if bits.dim() == 3 else (1, *bits.shape)
    n = lib().halftone_spectrum_rings(P)
    if n <= 0:
        raise HalftoneError(HS_EUNSUPPORTED, f"halftone_spectrum: P={P}")
    r = torch.empty(n, dtype=torch.float32, device=bits.device)
    a = torch.empty(n, dtype=torch.float32, device=bits.device)
    ws = _ws(lib().halftone_spectrum_workspace_size(B, H, W, P), bits.device)
    _check(lib().halftone_spectrum(_ptr(bits), B, H, W, P, _ptr(r), _ptr(a), _ptr(ws), ws.numel(),
                                   _stream()))
    return r, a


def halftone_profile_start():
    _check(lib().halftone_profile_start())


def halftone_profile_stop():
    """(summed milliseconds of the dominant kernel, number of recorded calls)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int(0)
    _check(lib().halftone_profile_stop(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def halftone_error_diffusion_host(contone_host):
    """Floyd-Steinberg on the host: numpy/torch CPU float32 [B,H,W] -> uint8."""
    c = torch.as_tensor(contone_host, dtype=torch.float32).contiguous()
    if c.dim() == 2:
        c = c[None]
    B, H, W = c.shape
    bits = torch.empty((B, H, W), dtype=torch.uint8)
    _check(lib().halftone_error_diffusion_host(_ptr(c), B, H, W, _ptr(bits)))
    return bits


def halftone_error_diffusion_levels_host(contone_host, levels):
    """L-level Floyd-Steinberg on the host: float32 [B,H,W] -> uint8 level indices."""
    c = torch.as_tensor(contone_host, dtype=torch.float32).contiguous()
    if c.dim() == 2:
        c = c[None]
    B, H, W = c.shape
    out = torch.empty((B, H, W), dtype=torch.uint8)
    _check(lib().halftone_error_diffusion_levels_host(_ptr(c), B, H, W, int(levels), _ptr(out)))
    return out
