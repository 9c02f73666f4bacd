"""Seeded synthetic inputs shared by the oracle checks and the HIP path.

This module holds none of the halftoning method's arithmetic: it only makes
input data (contone images, initial weights, constant-gray batches, page
sizes) from seeds, with numpy's own counter-based generator. The method's
own random draws (noise map, actions) are not made here.

Contone recipe (a stand-in for the paper's grayscale photographs, which are
not available): base level plus two linear ramps, eight random step edges,
and Gaussian-blurred uniform noise for texture, clamped to [0, 1] so that
saturated flats occur (the case the contrast-weighted SSIM is designed for).
"""
import numpy as np

CH = (2, 32, 32, 32, 32, 32, 1)


def _rng(seed, tag):
    return np.random.Generator(np.random.Philox(key=(int(seed) & ((1 << 64) - 1)) | (int(tag) << 64)))


def _blur_kernel(sigma=3.0, r=9):
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-t * t / (2.0 * sigma * sigma))
    return g / g.sum()


def _blur_clamp(n, sigma=3.0, r=9):
    """Separable normalised Gaussian blur with clamp-to-edge borders."""
    g = _blur_kernel(sigma, r)
    H, W = n.shape
    p = np.pad(n, ((r, r), (0, 0)), mode="edge")
    v = np.zeros((H, W))
    for i in range(2 * r + 1):
        v += g[i] * p[i:i + H, :]
    p = np.pad(v, ((0, 0), (r, r)), mode="edge")
    out = np.zeros((H, W))
    for i in range(2 * r + 1):
        out += g[i] * p[:, i:i + W]
    return out


def contone(seed, H, W):
    """One H x W float32 contone in [0, 1] (1 = white)."""
    prm = _rng(seed, 3)
    a0 = prm.uniform(0.25, 0.75)
    a1, a2 = prm.uniform(-0.25, 0.25, size=2)
    y = np.arange(H, dtype=np.float64)[:, None]
    x = np.arange(W, dtype=np.float64)[None, :]
    img = a0 + a1 * x / max(W - 1, 1) + a2 * y / max(H - 1, 1)
    s = prm.uniform(-0.15, 0.15, size=8)
    phi = prm.uniform(0.0, 2.0 * np.pi, size=8)
    px = prm.uniform(0.0, W, size=8)
    py = prm.uniform(0.0, H, size=8)
    for k in range(8):
        img = img + s[k] * (((x - px[k]) * np.cos(phi[k]) + (y - py[k]) * np.sin(phi[k])) >= 0)
    n = _rng(seed, 2).uniform(-0.5, 0.5, size=(H, W))
    img = img + 4.0 * _blur_clamp(n)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def contone_torch(seed, H, W, device):
    """The contone recipe of `contone` on a torch device, for page-sized
    inputs: the same ramp and edge parameters (numpy's generator), the
    texture noise drawn from torch's generator seeded with `seed` instead of
    numpy's, so the texture realisation differs from `contone`'s."""
    import torch
    prm = _rng(seed, 3)
    a0 = prm.uniform(0.25, 0.75)
    a1, a2 = prm.uniform(-0.25, 0.25, size=2)
    s = prm.uniform(-0.15, 0.15, size=8)
    phi = prm.uniform(0.0, 2.0 * np.pi, size=8)
    px = prm.uniform(0.0, W, size=8)
    py = prm.uniform(0.0, H, size=8)
    f64 = torch.float64
    y = torch.arange(H, dtype=f64, device=device)[:, None]
    x = torch.arange(W, dtype=f64, device=device)[None, :]
    img = a0 + a1 * x / max(W - 1, 1) + a2 * y / max(H - 1, 1)
    for k in range(8):
        img = img + s[k] * (((x - px[k]) * np.cos(phi[k]) + (y - py[k]) * np.sin(phi[k])) >= 0)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) & ((1 << 63) - 1))
    n = torch.rand((H, W), generator=gen, dtype=torch.float32, device=device).to(f64) - 0.5
    g = torch.tensor(_blur_kernel(), dtype=f64, device=device)
    r = (g.numel() - 1) // 2
    p = torch.nn.functional.pad(n[None, None], (0, 0, r, r), mode="replicate")
    n = torch.nn.functional.conv2d(p, g.view(1, 1, -1, 1))
    p = torch.nn.functional.pad(n, (r, r, 0, 0), mode="replicate")
    n = torch.nn.functional.conv2d(p, g.view(1, 1, 1, -1))[0, 0]
    img = img + 4.0 * n
    return img.clamp(0.0, 1.0).to(torch.float32)


def contone_batch(seeds, H, W):
    return np.stack([contone(s, H, W) for s in seeds]).astype(np.float32)


def he_weights(seed, ch=CH, head_std=None):
    """Flat float32 weights, layer by layer W[cout][cin][3][3] then bias[cout].

    He initialisation N(0, 2 / (9 cin)) with zero bias; if head_std is given
    the last layer uses N(0, head_std^2) instead (the paper initialises every
    layer with N(0, 0.01^2) so that the first actions are near p = 0.5)."""
    rng = _rng(seed, 6)
    parts = []
    L = len(ch) - 1
    for l in range(L):
        ci, co = ch[l], ch[l + 1]
        std = np.sqrt(2.0 / (9.0 * ci))
        if head_std is not None and l == L - 1:
            std = head_std
        parts.append(rng.normal(0.0, std, size=co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def gray_batch(n_levels=64, H=64, W=64):
    """Constant-gray images at the midpoints (k + 1/2) / n_levels."""
    lv = (np.arange(n_levels, dtype=np.float64) + 0.5) / n_levels
    return np.broadcast_to(lv[:, None, None], (n_levels, H, W)).astype(np.float32).copy()


def flat_contones(seed, n, H, W):
    """n constant images with gray levels drawn uniformly from [0, 1]."""
    lv = _rng(seed, 8).uniform(0.0, 1.0, size=n)
    return np.broadcast_to(lv[:, None, None], (n, H, W)).astype(np.float32).copy()


def seeds_array(seeds):
    return np.asarray(list(seeds), dtype=np.uint64)


def page_sizes(seed, n=48, wmin=600, wmax=4960, hmin=800, hmax=7016):
    """(H, W) of n pages, each side uniform over its range."""
    rng = _rng(seed, 7)
    W = rng.integers(wmin, wmax + 1, size=n)
    H = rng.integers(hmin, hmax + 1, size=n)
    return [(int(h), int(w)) for h, w in zip(H, W)]
