"""Python face of the plain CPU oracle (``halftone_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. Nothing in the product package imports
this module, and this module imports nothing from the product package.

All arithmetic lives in the C file (FP64, plain loops); this wrapper only
marshals numpy arrays. The few lines of arithmetic here (the sigmoid and the
-dR/B scaling of the Local Expectation gradient) are spelled out where used.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "halftone_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# The policy of the build: six 3x3 conv layers, 32 channels, one-channel head.
CH = (2, 32, 32, 32, 32, 32, 1)

# Loss parameters (Sec. VI-A: w_s = 0.06, w_a = 0.002; Sec. V: k = 2 and the
# 11x11 sigma = 1.5 SSIM window; the 11x11 Gaussian sigma = 2 HVS filter;
# SSIM constants from Wang et al. 2004 with K1 = 0.01, K2 = 0.03, L = 1).
# estimator: 0 = Local Expectation (Eq. le), 1 = COMA (Eq. coma).
DEFAULT_PRM = dict(w_s=0.06, w_a=0.002, hvs_sigma=2.0, hvs_r=5, ssim_sigma=1.5,
                   ssim_r=5, k=2.0, C1=1e-4, C2=9e-4, as_patch=32, estimator=0, levels=2)
PRM_ORDER = ("w_s", "w_a", "hvs_sigma", "hvs_r", "ssim_sigma", "ssim_r", "k",
             "C1", "C2", "as_patch", "estimator", "levels")
# Optimiser (Sec. VI-A: Adam, cosine 3e-4 -> 1e-5; textbook Adam constants).
DEFAULT_TRAIN = dict(lr_max=3e-4, lr_min=1e-5, beta1=0.9, beta2=0.999, eps=1e-8)


def build(force=False):
    """Compile the oracle with plain gcc -O2 (no fast-math, no intrinsics)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread", "-o", tmp,
                               SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        D = ctypes.POINTER(ctypes.c_double)
        U8 = ctypes.POINTER(ctypes.c_uint8)
        U32 = ctypes.POINTER(ctypes.c_uint32)
        U64 = ctypes.POINTER(ctypes.c_uint64)
        I = ctypes.POINTER(ctypes.c_int)
        c_int, c_long, c_double, c_u32, c_u64 = (ctypes.c_int, ctypes.c_long, ctypes.c_double,
                                                  ctypes.c_uint32, ctypes.c_uint64)
        sig = {
            "or_set_threads": (None, [c_int]),
            "or_get_threads": (c_int, []),
            "or_philox4x32_10": (None, [U32, U32, U32]),
            "or_uniform": (c_double, [c_u64, c_u64, c_u32, c_u32]),
            "or_normal": (c_double, [c_u64, c_u64, c_u32, c_u32]),
            "or_noise_map": (None, [U64, c_int, c_int, c_int, c_int, c_u32, c_u32, D]),
            "or_bernoulli": (None, [D, U64, c_int, c_int, c_int, c_u32, U8]),
            "or_param_count": (c_long, [I, c_int]),
            "or_policy_forward": (None, [D, I, c_int, D, D, c_int, c_int, c_int, D]),
            "or_policy_forward_window": (None, [D, I, c_int, D, D, c_int, c_int, c_int, c_int,
                                                c_int, c_int, D]),
            "or_threshold": (None, [D, c_long, U8]),
            "or_policy_backward": (None, [D, I, c_int, D, D, c_int, c_int, c_int, D, D, D]),
            "or_gauss_window": (None, [c_double, c_int, D]),
            "or_filter_valid": (None, [D, c_int, c_int, D, c_int, D]),
            "or_reward": (None, [D, D, c_int, c_int, c_int, D, D]),
            "or_le_delta_brute": (None, [D, D, c_int, c_int, c_int, D, D]),
            "or_le_delta_local": (None, [D, D, c_int, c_int, c_int, D, D]),
            "or_coma_grad_logit": (None, [D, D, D, c_int, c_int, c_int, D, D]),
            "or_multitone_actions": (None, [D, U64, c_int, c_int, c_int, c_int, c_u32, U8]),
            "or_multitone_levels": (None, [D, c_long, c_int, U8]),
            "or_multitone_delta_brute": (None, [D, D, D, c_int, c_int, c_int, c_int, D, D]),
            "or_multitone_delta_local": (None, [D, D, D, c_int, c_int, c_int, c_int, D, D]),
            "or_ring_index": (c_int, [c_int, c_int, c_int]),
            "or_as_loss": (c_double, [D, c_int, c_int, c_int, c_int, D]),
            "or_anisotropy": (None, [D, c_int, D, D]),
            "or_spectrum": (c_int, [D, c_int, c_int, c_int, c_int, D, D]),
            "or_lr_cosine": (c_double, [c_long, c_long, c_double, c_double]),
            "or_adam_step": (None, [D, D, D, D, c_long, c_long, c_double, c_double, c_double,
                                    c_double]),
            "or_train_step": (None, [D, D, D, I, c_int, D, U64, c_int, c_int, c_int, D, U64,
                                     c_int, c_int, c_int, c_long, c_long, D, D, c_int, U8, U8, D,
                                     D]),
            "or_floyd_steinberg": (None, [D, c_int, c_int, c_int, U8]),
            "or_floyd_steinberg_levels": (None, [D, c_int, c_int, c_int, c_int, U8]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def set_threads(n):
    """Threads for the conv stack's channel loops (results are bit-identical
    for any count); returns the previous count."""
    prev = lib().or_get_threads()
    lib().or_set_threads(int(n))
    return prev


class threads:
    """Context manager: run the oracle on n threads inside the block."""

    def __init__(self, n):
        self.n = n

    def __enter__(self):
        self.prev = set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _ch(ch):
    a = np.ascontiguousarray(ch, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _prm(prm):
    p = dict(DEFAULT_PRM)
    if prm:
        p.update(prm)
    return _d(np.array([p[k] for k in PRM_ORDER], dtype=np.float64))


def _bhw(x):
    x = np.asarray(x)
    if x.ndim == 2:
        return 1, x.shape[0], x.shape[1]
    return x.shape[0], x.shape[1], x.shape[2]


# ---------------------------------------------------------------- random ----
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    P = ctypes.POINTER(ctypes.c_uint32)
    lib().or_philox4x32_10(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def uniform(seed, a, stream, step):
    return lib().or_uniform(seed, a, stream, step)


def normal(seed, a, stream, step):
    return lib().or_normal(seed, a, stream, step)


def noise_map(seeds, H, W, kind=0, stream=1, step=0):
    """[len(seeds)][H][W] noise: kind 0 Gaussian, kind 1 uniform."""
    s, sp = _u64(seeds)
    B = s.size
    z, zp = _d(np.zeros((B, H, W)))
    lib().or_noise_map(sp, B, H, W, kind, stream, step, zp)
    return z


def bernoulli(p, seeds, step=0):
    B, H, W = _bhw(p)
    p, pp = _d(p)
    s, sp = _u64(seeds)
    h, hp = _u8(np.zeros((B, H, W)))
    lib().or_bernoulli(pp, sp, B, H, W, step, hp)
    return h


# ---------------------------------------------------------------- policy ----
def param_count(ch=CH):
    a, ap = _ch(ch)
    return lib().or_param_count(ap, len(ch) - 1)


def policy_forward(w, c, z, ch=CH):
    B, H, W = _bhw(c)
    w, wp = _d(w)
    a, ap = _ch(ch)
    c, cp = _d(np.reshape(c, (B, H, W)))
    z, zp = _d(np.reshape(z, (B, H, W)))
    x, xp = _d(np.zeros((B, H, W)))
    lib().or_policy_forward(wp, ap, len(ch) - 1, cp, zp, B, H, W, xp)
    return x


def policy_forward_window(w, c, z, y0, y1, x0, x1, ch=CH):
    """Logits of one image (c, z: H x W) over the window [y0,y1) x [x0,x1)."""
    H, W = c.shape
    w, wp = _d(w)
    a, ap = _ch(ch)
    c, cp = _d(c)
    z, zp = _d(z)
    x, xp = _d(np.zeros((y1 - y0, x1 - x0)))
    lib().or_policy_forward_window(wp, ap, len(ch) - 1, cp, zp, H, W, y0, y1, x0, x1, xp)
    return x


def threshold(logits):
    x, xp = _d(logits)
    b, bp = _u8(np.zeros(x.shape))
    lib().or_threshold(xp, x.size, bp)
    return b


def policy_backward(w, c, z, g_logit, ch=CH):
    """Returns (dLoss/dtheta, dLoss/d(c,z)) for dLoss/dlogit = g_logit."""
    B, H, W = _bhw(c)
    w, wp = _d(w)
    a, ap = _ch(ch)
    c, cp = _d(np.reshape(c, (B, H, W)))
    z, zp = _d(np.reshape(z, (B, H, W)))
    g, gp = _d(np.reshape(g_logit, (B, H, W)))
    gw, gwp = _d(np.zeros(w.shape))
    gi, gip = _d(np.zeros((B, 2, H, W)))
    lib().or_policy_backward(wp, ap, len(ch) - 1, cp, zp, B, H, W, gp, gwp, gip)
    return gw, gi


# ---------------------------------------------------------------- metrics ---
def gauss_window(sigma, r):
    g, gp = _d(np.zeros((2 * r + 1, 2 * r + 1)))
    lib().or_gauss_window(sigma, r, gp)
    return g


def filter_valid(img, g, r):
    H, W = img.shape
    img, ip = _d(img)
    g, gp = _d(g)
    out, op = _d(np.zeros((H - 2 * r, W - 2 * r)))
    lib().or_filter_valid(ip, H, W, gp, r, op)
    return out


def reward(h, c, prm=None):
    """(B, 3) array of per-image (MSE, CSSIM, R)."""
    B, H, W = _bhw(c)
    h, hp = _d(np.reshape(h, (B, H, W)))
    c, cp = _d(np.reshape(c, (B, H, W)))
    p, pp = _prm(prm)
    out, op = _d(np.zeros((B, 3)))
    lib().or_reward(hp, cp, B, H, W, pp, op)
    return out


def le_delta(h, c, prm=None, brute=False):
    """dR_a = R(h_a=1, h_-a) - R(h_a=0, h_-a) for every pixel."""
    B, H, W = _bhw(c)
    h, hp = _d(np.reshape(h, (B, H, W)))
    c, cp = _d(np.reshape(c, (B, H, W)))
    p, pp = _prm(prm)
    d, dp = _d(np.zeros((B, H, W)))
    (lib().or_le_delta_brute if brute else lib().or_le_delta_local)(hp, cp, B, H, W, pp, dp)
    return d


def le_grad_probs(h, c, prm=None):
    """dL_MARL/dp_a = -dR_a / B (Eq. marl, mini-batch mean)."""
    d = le_delta(h, c, prm)
    return -d / d.shape[0]


def multitone_actions(v, seeds, L, step=0):
    """Level indices k_a in {k_f, k_f + 1} around v_a (Sec. VI-E, its unnumbered rounding equation)."""
    B, H, W = _bhw(v)
    v, vp = _d(np.reshape(v, (B, H, W)))
    s, sp = _u64(seeds)
    k, kp = _u8(np.zeros((B, H, W)))
    lib().or_multitone_actions(vp, sp, B, H, W, L, step, kp)
    return k


def multitone_levels(logits, L):
    """Test phase: index of the level nearest to sigmoid(x), ties up."""
    x, xp = _d(logits)
    k, kp = _u8(np.zeros(x.shape))
    lib().or_multitone_levels(xp, x.size, L, kp)
    return k


def multitone_delta(h, c, v, L, prm=None, brute=False):
    """dR_a = R(h_a = l_{k_f+1}) - R(h_a = l_{k_f}); h holds image values."""
    B, H, W = _bhw(c)
    h, hp = _d(np.reshape(h, (B, H, W)))
    c, cp = _d(np.reshape(c, (B, H, W)))
    v, vp = _d(np.reshape(v, (B, H, W)))
    p, pp = _prm(prm)
    d, dp = _d(np.zeros((B, H, W)))
    fn = lib().or_multitone_delta_brute if brute else lib().or_multitone_delta_local
    fn(hp, cp, vp, B, H, W, L, pp, dp)
    return d


def coma_grad_logits(h, c, p, prm=None):
    """dL/dx_a of the COMA estimator (Eqs. baseline, coma), batch mean."""
    B, H, W = _bhw(c)
    h, hp = _d(np.reshape(h, (B, H, W)))
    c, cp = _d(np.reshape(c, (B, H, W)))
    p, pxp = _d(np.reshape(p, (B, H, W)))
    q, qp = _prm(prm)
    g, gp = _d(np.zeros((B, H, W)))
    lib().or_coma_grad_logit(hp, cp, pxp, B, H, W, qp, gp)
    return g


def ring_index(u, v, P=32):
    return lib().or_ring_index(u, v, P)


def as_loss(x, P=32, grad=True):
    """(L_AS, dL_AS/dx or None) over the P x P patches of x ([Bg][Hg][Wg])."""
    B, H, W = _bhw(x)
    x, xp = _d(np.reshape(x, (B, H, W)))
    if grad:
        g, gp = _d(np.zeros((B, H, W)))
    else:
        g, gp = None, None
    L = lib().or_as_loss(xp, B, H, W, P, gp)
    return L, g


def anisotropy(patch):
    P = patch.shape[0]
    patch, pp = _d(patch)
    n = ring_index(P // 2, P // 2, P) + 1
    r, rp = _d(np.zeros(n))
    a, ap = _d(np.zeros(n))
    lib().or_anisotropy(pp, P, rp, ap)
    return r, a


def spectrum(img, P=32):
    """(RAPSD, anisotropy) per ring of the mean periodogram over the P x P
    patches of img ([B][H][W] or [H][W])."""
    B, H, W = _bhw(img)
    x, xp = _d(np.reshape(img, (B, H, W)))
    n = ring_index(P // 2, P // 2, P) + 1
    r, rp = _d(np.zeros(n))
    a, ap = _d(np.zeros(n))
    lib().or_spectrum(xp, B, H, W, P, rp, ap)
    return r, a


def lr_cosine(t, T, lr_max=3e-4, lr_min=1e-5):
    return lib().or_lr_cosine(t, T, lr_max, lr_min)


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays theta, m, v."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g, gp = _d(g)
    P = ctypes.POINTER(ctypes.c_double)
    lib().or_adam_step(theta.ctypes.data_as(P), m.ctypes.data_as(P), v.ctypes.data_as(P), gp,
                       theta.size, t, lr, b1, b2, eps)


def train_step(w, m, v, c, seeds, cg, gseeds, step, total, prm=None, tprm=None, noise_kind=0,
               actions=None, ch=CH):
    """One TRAIN iteration of Algorithm 1, in place on float64 w, m, v.

    Returns dict(actions, grad, metrics)."""
    B, H, W = _bhw(c)
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    c, cp = _d(np.reshape(c, (B, H, W)))
    s, sp = _u64(seeds)
    if cg is None or len(cg) == 0:
        Bg, Hg, Wg = 0, 0, 0
        cg, cgp = _d(np.zeros(1))
        gs, gsp = _u64(np.zeros(1))
    else:
        Bg, Hg, Wg = _bhw(cg)
        cg, cgp = _d(np.reshape(cg, (Bg, Hg, Wg)))
        gs, gsp = _u64(gseeds)
    p, pp = _prm(prm)
    t = dict(DEFAULT_TRAIN)
    if tprm:
        t.update(tprm)
    tp, tpp = _d(np.array([t["lr_max"], t["lr_min"], t["beta1"], t["beta2"], t["eps"]]))
    chn, chp = _ch(ch)
    if actions is not None:
        ain, ainp = _u8(np.reshape(actions, (B, H, W)))
    else:
        ain, ainp = None, None
    aout, aoutp = _u8(np.zeros((B, H, W)))
    grad, gp = _d(np.zeros(w.shape))
    met, mp = _d(np.zeros(7))
    P = ctypes.POINTER(ctypes.c_double)
    lib().or_train_step(w.ctypes.data_as(P), m.ctypes.data_as(P), v.ctypes.data_as(P), chp,
                        len(ch) - 1, cp, sp, B, H, W, cgp, gsp, Bg, Hg, Wg, step, total, pp, tpp,
                        noise_kind, ainp, aoutp, gp, mp)
    names = ("mse", "cssim", "reward", "l_as", "lr", "grad_norm", "fill")
    return dict(actions=aout, grad=grad, metrics=dict(zip(names, met.tolist())))


def floyd_steinberg(c):
    B, H, W = _bhw(c)
    c, cp = _d(np.reshape(c, (B, H, W)))
    h, hp = _u8(np.zeros((B, H, W)))
    lib().or_floyd_steinberg(cp, B, H, W, hp)
    return h


def floyd_steinberg_levels(c, L):
    """Level indices of L-level Floyd-Steinberg error diffusion."""
    B, H, W = _bhw(c)
    c, cp = _d(np.reshape(c, (B, H, W)))
    k, kp = _u8(np.zeros((B, H, W)))
    lib().or_floyd_steinberg_levels(cp, B, H, W, L, kp)
    return k


def sigmoid(x):
    """pi_a(h = 1) = 1 / (1 + exp(-x_a)) (Sec. VI-A: pixel-wise sigmoid)."""
    return 1.0 / (1.0 + np.exp(-np.asarray(x, dtype=np.float64)))
