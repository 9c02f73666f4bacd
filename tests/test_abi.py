"""CPU-side checks of the C ABI: the library loads and exports every function
declared in include/halftone.h, defaults match the documented values, and
argument errors are reported before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2304_12152_amd import binding as hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "halftone.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hb.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return hb.lib()


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("halftone_infer", "halftone_loss", "halftone_loss_backward", "policy_train_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol(lib):
    for name in declared_functions():
        assert name in hb._SIGS, name


def test_defaults(lib):
    p = hb.default_loss_params()
    assert (p.w_s, p.w_a, p.hvs_radius, p.ssim_radius, p.as_patch) == (
        pytest.approx(0.06), pytest.approx(0.002), 5, 5, 32)
    assert (p.hvs_sigma, p.ssim_sigma, p.k) == (2.0, 1.5, 2.0)
    assert p.c1 == pytest.approx(1e-4) and p.c2 == pytest.approx(9e-4)
    t = hb.default_train_params()
    assert t.lr_max == pytest.approx(3e-4) and t.lr_min == pytest.approx(1e-5)
    assert t.beta1 == pytest.approx(0.9) and t.beta2 == pytest.approx(0.999)
    assert lib.halftone_param_count() == 37889


def test_workspace_sizes_positive_and_monotone(lib):
    a = lib.halftone_infer_workspace_size(1, 64, 64, hb.HS_BF16)
    b = lib.halftone_infer_workspace_size(2, 64, 64, hb.HS_BF16)
    assert 0 < a < b
    assert lib.halftone_infer_workspace_size(0, 64, 64, hb.HS_BF16) == 0
    prm = hb.default_loss_params()
    assert lib.halftone_loss_workspace_size(2, 64, 64, 0, 0, 0, ctypes.byref(prm)) > 0
    assert lib.halftone_train_workspace_size(4, 64, 64, 4, 64, 64, hb.HS_BF16) > \
        lib.halftone_train_workspace_size(4, 64, 64, 0, 0, 0, hb.HS_BF16)


def test_bf16_infer_workspace_holds_all_buffers(lib):
    # fused-kernel fragments (4800 x 16 B), the split hi and lo copies of the
    # four 32->32 layers (2 x 36864 BF16) and their FP32 transposes (4 x 9216
    # floats), plus per pixel: a segmented-list entry and an FP32-stage list
    # entry (4 B each), plus the segment counts and counters
    weights = 4800 * 16 + 2 * 36864 * 2 + 4 * 9216 * 4
    for shape in [(1, 1, 1), (1, 37, 45), (2, 64, 64), (8, 1024, 1024)]:
        n = shape[0] * shape[1] * shape[2]
        assert lib.halftone_infer_workspace_size(*shape, hb.HS_BF16) >= \
            weights + 2 * 4 * n + 2 * 256 * 4 + 64


def _fake(n=64):
    # host buffers stand in for device pointers: every call below must fail
    # validation before it would touch them
    return ctypes.c_void_p(ctypes.addressof(ctypes.create_string_buffer(n)))


def test_fp16_inference_takes_the_bf16_workspace(lib):
    """HS_FP16 runs the same stages as HS_BF16 (plus a BF16 re-run that
    exits at once unless the FP16 pass overflowed), in the same workspace."""
    for B, H, W in [(1, 8, 8), (8, 1024, 1024)]:
        assert lib.halftone_infer_workspace_size(B, H, W, hb.HS_FP16) == \
            lib.halftone_infer_workspace_size(B, H, W, hb.HS_BF16)
    assert hb.RECHECK_TAU[hb.HS_FP16] < hb.RECHECK_TAU[hb.HS_BF16] / 4


def test_infer_argument_errors(lib):
    p = _fake()
    ws = lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_FP32)
    args = [p, p, p, 1, 8, 8, 0, hb.HS_FP32, 0.05, p, None, None, p, ws, None]
    a = list(args); a[0] = None
    assert lib.halftone_infer(*a) == hb.HS_EINVAL
    assert b"null" in lib.halftone_last_error()
    a = list(args); a[3] = 0
    assert lib.halftone_infer(*a) == hb.HS_ESHAPE
    a = list(args); a[4] = -3
    assert lib.halftone_infer(*a) == hb.HS_ESHAPE
    a = list(args); a[7] = 7
    assert lib.halftone_infer(*a) == hb.HS_EUNSUPPORTED
    a = list(args); a[6] = 5
    assert lib.halftone_infer(*a) == hb.HS_EINVAL
    a = list(args); a[8] = -1.0
    assert lib.halftone_infer(*a) == hb.HS_EINVAL
    a = list(args); a[13] = ws - 1
    assert lib.halftone_infer(*a) == hb.HS_EWORKSPACE


def test_pages_argument_errors(lib):
    import numpy as np
    p = _fake()
    sh = hb.page_shapes_array([(8, 8), (3, 20)])
    shp = sh.ctypes.data_as(ctypes.c_void_p)
    ws = lib.halftone_infer_pages_workspace_size(2, shp, hb.HS_BF16)
    assert ws > lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_BF16) > 0
    assert lib.halftone_infer_pages_workspace_size(0, shp, hb.HS_BF16) == 0
    bad = hb.page_shapes_array([(8, 8), (0, 20)])
    assert lib.halftone_infer_pages_workspace_size(2, bad.ctypes.data_as(ctypes.c_void_p),
                                                   hb.HS_BF16) == 0
    huge = hb.page_shapes_array([(65536, 32768)])  # 2^31 pixels
    assert lib.halftone_infer_pages_workspace_size(1, huge.ctypes.data_as(ctypes.c_void_p),
                                                   hb.HS_BF16) == 0
    args = [p, p, p, 2, shp, 0, hb.HS_BF16, 0.05, p, None, None, p, ws, None]
    a = list(args); a[1] = None
    assert lib.halftone_infer_pages(*a) == hb.HS_EINVAL
    a = list(args); a[4] = bad.ctypes.data_as(ctypes.c_void_p)
    assert lib.halftone_infer_pages(*a) == hb.HS_ESHAPE
    a = list(args); a[3] = 0
    assert lib.halftone_infer_pages(*a) == hb.HS_ESHAPE
    a = list(args); a[6] = 9
    assert lib.halftone_infer_pages(*a) == hb.HS_EUNSUPPORTED
    a = list(args); a[12] = ws - 1
    assert lib.halftone_infer_pages(*a) == hb.HS_EWORKSPACE
    # the FP32 path runs page by page in the workspace of the largest page
    ws32 = lib.halftone_infer_pages_workspace_size(2, shp, hb.HS_FP32)
    assert ws32 == lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_FP32)


def test_loss_argument_errors(lib):
    p = _fake()
    prm = hb.default_loss_params()
    ws = 1 << 20
    base = [p, p, 1, 32, 32, None, 0, 0, 0, ctypes.byref(prm), p, p, ws, None]
    a = list(base); a[3] = 10  # smaller than the 11 x 11 window
    assert lib.halftone_loss(*a) == hb.HS_ESHAPE
    bad = hb.default_loss_params(hvs_radius=9)
    a = list(base); a[9] = ctypes.byref(bad)
    assert lib.halftone_loss(*a) == hb.HS_EINVAL
    bad = hb.default_loss_params(as_patch=16)
    a = list(base); a[9] = ctypes.byref(bad)
    assert lib.halftone_loss(*a) == hb.HS_EUNSUPPORTED
    a = list(base); a[6] = 3  # Bg > 0 with no gray batch
    assert lib.halftone_loss(*a) == hb.HS_EINVAL
    a = list(base); a[12] = 16
    assert lib.halftone_loss(*a) == hb.HS_EWORKSPACE
    # backward: logit space needs probs
    b = [p, p, None, 1, 32, 32, None, 0, 0, 0, ctypes.byref(prm), hb.HS_WRT_LOGIT, p, None, p,
         ws, None]
    assert lib.halftone_loss_backward(*b) == hb.HS_EINVAL
    b[11] = 7
    assert lib.halftone_loss_backward(*b) == hb.HS_EINVAL


def test_train_argument_errors(lib):
    p = _fake()
    tp = hb.default_train_params()
    ws = lib.halftone_train_workspace_size(1, 16, 16, 0, 0, 0, hb.HS_FP32)
    base = [p, p, p, p, p, 1, 16, 16, None, None, 0, 0, 0, 0, 10, ctypes.byref(tp), hb.HS_FP32,
            p, None, None, p, ws, None]
    a = list(base); a[0] = None
    assert lib.policy_train_step(*a) == hb.HS_EINVAL
    a = list(base); a[16] = 9
    assert lib.policy_train_step(*a) == hb.HS_EUNSUPPORTED
    a = list(base); a[16] = hb.HS_FP16  # inference only
    assert lib.policy_train_step(*a) == hb.HS_EUNSUPPORTED
    a = list(base); a[13] = -1
    assert lib.policy_train_step(*a) == hb.HS_EINVAL
    a = list(base); a[6] = 8
    assert lib.policy_train_step(*a) == hb.HS_ESHAPE
    a = list(base); a[21] = ws - 256
    assert lib.policy_train_step(*a) == hb.HS_EWORKSPACE
    a = list(base); a[8] = p  # gray batch without seeds
    assert lib.policy_train_step(*a) == hb.HS_EINVAL


def test_host_error_diffusion_matches_oracle(orc, lib):
    from paper_2304_12152_amd import synth
    c = synth.contone_batch([3, 4, 5], 37, 53)
    got = hb.halftone_error_diffusion_host(c).numpy()
    want = orc.floyd_steinberg(c.astype(np.float64))
    assert np.array_equal(got, want)
    assert np.array_equal(hb.halftone_error_diffusion_host(np.full((6, 6), 0.5, np.float32))[0].numpy(),
                          orc.floyd_steinberg(np.full((1, 6, 6), 0.5))[0])


def test_spectrum_argument_errors(lib):
    p = _fake()
    assert lib.halftone_spectrum_rings(32) == 24
    assert lib.halftone_spectrum_rings(64) == 46
    assert lib.halftone_spectrum_rings(48) == 0
    ws = lib.halftone_spectrum_workspace_size(2, 70, 90, 32)
    assert ws >= (2 * 2 * 2 * 32 * 32 + 32 * 32) * 4
    assert lib.halftone_spectrum_workspace_size(2, 31, 90, 32) == 0
    assert lib.halftone_spectrum_workspace_size(2, 70, 90, 16) == 0
    args = [p, 2, 70, 90, 32, p, p, p, ws, None]
    a = list(args); a[4] = 48
    assert lib.halftone_spectrum(*a) == hb.HS_EUNSUPPORTED
    a = list(args); a[3] = 31
    assert lib.halftone_spectrum(*a) == hb.HS_ESHAPE
    a = list(args); a[1] = 0
    assert lib.halftone_spectrum(*a) == hb.HS_ESHAPE
    a = list(args); a[0] = None
    assert lib.halftone_spectrum(*a) == hb.HS_EINVAL
    a = list(args); a[8] = ws - 1
    assert lib.halftone_spectrum(*a) == hb.HS_EWORKSPACE


def test_levels_argument_errors(lib):
    p = _fake()
    ws = 1 << 20
    for bad, code in ((1, hb.HS_EINVAL), (hb.HS_MAX_LEVELS + 1, hb.HS_EINVAL)):
        prm = hb.default_loss_params(levels=bad)
        assert lib.halftone_loss(p, p, 1, 32, 32, None, 0, 0, 0, ctypes.byref(prm), p, p, ws,
                                 None) == code
    prm = hb.default_loss_params(levels=4, estimator=hb.HS_EST_COMA)
    assert lib.halftone_loss(p, p, 1, 32, 32, None, 0, 0, 0, ctypes.byref(prm), p, p, ws,
                             None) == hb.HS_EUNSUPPORTED
    # multitone gradients need the probabilities (the pair of levels)
    prm = hb.default_loss_params(levels=4)
    b = [p, p, None, 1, 32, 32, None, 0, 0, 0, ctypes.byref(prm), hb.HS_WRT_PROB, p, None, p,
         ws, None]
    assert lib.halftone_loss_backward(*b) == hb.HS_EINVAL
    sh = hb.page_shapes_array([(8, 8)])
    shp = sh.ctypes.data_as(ctypes.c_void_p)
    need = lib.halftone_infer_pages_workspace_size(1, shp, hb.HS_BF16)
    args = [p, p, p, 1, shp, 4, 0, hb.HS_BF16, 0.05, p, None, None, p, need, None]
    for bad in (0, 1, hb.HS_MAX_LEVELS + 1):
        a = list(args); a[5] = bad
        assert lib.halftone_infer_levels(*a) == hb.HS_EINVAL
    a = list(args); a[13] = need - 1
    assert lib.halftone_infer_levels(*a) == hb.HS_EWORKSPACE


def test_recompute_workspace_and_errors(lib):
    full = hb.default_train_params()
    rec = hb.default_train_params(recompute=1)
    for prec, px in ((hb.HS_BF16, 64), (hb.HS_FP32, 128)):
        n0 = lib.halftone_train_workspace_size_params(32, 256, 256, 64, 64, 64, prec,
                                                      ctypes.byref(full))
        n1 = lib.halftone_train_workspace_size_params(32, 256, 256, 64, 64, 64, prec,
                                                      ctypes.byref(rec))
        assert n0 == lib.halftone_train_workspace_size(32, 256, 256, 64, 64, 64, prec)
        # three NHWC activation maps of the larger batch fewer
        assert n0 - n1 >= 3 * 32 * 256 * 256 * px
    bad = hb.default_train_params(recompute=2)
    p = _fake()
    n = 1 << 30
    assert lib.policy_train_step(p, p, p, p, p, 1, 32, 32, None, None, 0, 0, 0, 0, 10,
                                 ctypes.byref(bad), hb.HS_BF16, p, None, None, p, n,
                                 None) == hb.HS_EINVAL


@pytest.mark.parametrize("L", [2, 3, 4, 8])
def test_host_error_diffusion_levels_matches_oracle(orc, lib, L):
    from paper_2304_12152_amd import synth
    c = synth.contone_batch([6, 7], 41, 50)
    got = hb.halftone_error_diffusion_levels_host(c, L).numpy()
    assert np.array_equal(got, orc.floyd_steinberg_levels(c.astype(np.float64), L))
    if L == 2:
        assert np.array_equal(got, hb.halftone_error_diffusion_host(c).numpy())
    with pytest.raises(hb.HalftoneError):
        hb.halftone_error_diffusion_levels_host(c, 9)


def test_policy_handle_argument_errors(lib):
    p = _fake()
    n = lib.halftone_policy_bytes()
    # the FP32 weight copy, the BF16 and FP16 fragments, the split and FP32
    # recheck copies and the FP32 per-layer fragments
    assert n >= 37889 * 4 + 2 * 4800 * 16 + 2 * 36864 * 2 + 4 * 9216 * 4 + 4 * 9216 * 4
    pol = hb.HsPolicy()
    # before any device work: null pointers, bad flags, misaligned or short memory
    assert lib.halftone_policy_pack(None, p, p, n, 0, None) == hb.HS_EINVAL
    assert lib.halftone_policy_pack(ctypes.byref(pol), None, p, n, 0, None) == hb.HS_EINVAL
    assert lib.halftone_policy_pack(ctypes.byref(pol), p, p, n, 0x2, None) == hb.HS_EINVAL
    assert lib.halftone_policy_pack(ctypes.byref(pol), p, ctypes.c_void_p(4096 + 8), n, 0,
                                    None) == hb.HS_EINVAL
    assert lib.halftone_policy_pack(ctypes.byref(pol), p, ctypes.c_void_p(4096), n - 1, 0,
                                    None) == hb.HS_EWORKSPACE
    assert pol.packed == 0
    sh = hb.page_shapes_array([(8, 8)])
    shp = sh.ctypes.data_as(ctypes.c_void_p)
    ws = lib.halftone_infer_pages_workspace_size(1, shp, hb.HS_BF16)
    args = [ctypes.byref(pol), p, p, 1, shp, 2, 0, hb.HS_BF16, 0.05, -1.0, -1.0, p, None, None, p,
            ws, None]
    assert lib.halftone_policy_infer(*args) == hb.HS_EINVAL  # not packed
    assert b"not packed" in lib.halftone_last_error()
    a = list(args); a[0] = None
    assert lib.halftone_policy_infer(*a) == hb.HS_EINVAL
    pol.packed, pol.mem, pol.bytes = 1, 4096, n  # a packed-looking handle: argument checks only
    a = list(args); a[9] = -0.5
    assert lib.halftone_policy_infer(*a) == hb.HS_EINVAL
    a = list(args); a[10] = float("nan")
    assert lib.halftone_policy_infer(*a) == hb.HS_EINVAL
    a = list(args); a[5] = 9
    assert lib.halftone_policy_infer(*a) == hb.HS_EINVAL
    a = list(args); a[15] = ws - 1
    assert lib.halftone_policy_infer(*a) == hb.HS_EWORKSPACE
    a = list(args); a[1] = None
    assert lib.halftone_policy_infer(*a) == hb.HS_EINVAL


def test_finite_check_flag_is_validated(lib):
    p = _fake()
    ws = lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_FP32)
    args = [p, p, p, 1, 8, 8, 0, hb.HS_FP32, 0.05, p, None, None, p, ws, None]
    a = list(args); a[6] = hb.HS_CHECK_FINITE | 0x2  # unknown noise kind under the flag
    assert lib.halftone_infer(*a) == hb.HS_EINVAL
    prm = hb.default_loss_params(flags=0x4)  # unknown loss flag
    lws = lib.halftone_loss_workspace_size(1, 16, 16, 0, 0, 0, ctypes.byref(prm))
    assert lib.halftone_loss(p, p, 1, 16, 16, None, 0, 0, 0, ctypes.byref(prm), p, p, lws,
                             None) == hb.HS_EINVAL
    assert hb.default_loss_params().flags == 0


def test_fp8_argument_errors(lib):
    """HS_FP8: refused without a packed policy's FP8 copy; set_fp8 and
    layer_max reject bad arguments before any device work."""
    p = _fake()
    n = lib.halftone_policy_bytes()
    ws = lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_FP8)
    assert ws == lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_BF16)
    args = [p, p, p, 1, 8, 8, 0, hb.HS_FP8, 0.5, p, None, None, p, ws, None]
    assert lib.halftone_infer(*args) == hb.HS_EUNSUPPORTED
    assert b"halftone_policy_set_fp8" in lib.halftone_last_error()
    pol = hb.HsPolicy()
    amax = np.ones(4, dtype=np.float32)
    ap = amax.ctypes.data_as(ctypes.c_void_p)
    assert lib.halftone_policy_set_fp8(None, ap, None) == hb.HS_EINVAL
    assert lib.halftone_policy_set_fp8(ctypes.byref(pol), ap, None) == hb.HS_EINVAL  # not packed
    pol.packed, pol.mem, pol.bytes = 1, 4096, n
    assert lib.halftone_policy_set_fp8(ctypes.byref(pol), None, None) == hb.HS_EINVAL
    for bad in (-1.0, float("inf"), float("nan")):
        a = amax.copy(); a[2] = bad
        assert lib.halftone_policy_set_fp8(ctypes.byref(pol), a.ctypes.data_as(ctypes.c_void_p),
                                           None) == hb.HS_EINVAL
    assert pol.fp8 == 0
    sh = hb.page_shapes_array([(8, 8)])
    shp = sh.ctypes.data_as(ctypes.c_void_p)
    pws = lib.halftone_infer_pages_workspace_size(1, shp, hb.HS_FP8)
    pargs = [ctypes.byref(pol), p, p, 1, shp, 2, 0, hb.HS_FP8, 0.5, -1.0, -1.0, p, None, None, p,
             pws, None]
    assert lib.halftone_policy_infer(*pargs) == hb.HS_EUNSUPPORTED  # no FP8 copy
    fws = lib.halftone_infer_workspace_size(1, 8, 8, hb.HS_FP32)
    largs = [p, p, p, 1, 8, 8, 0, p, p, fws, None]
    for i in (0, 1, 2, 7, 8):
        a = list(largs); a[i] = None
        assert lib.halftone_layer_max(*a) == hb.HS_EINVAL
    a = list(largs); a[6] = 5
    assert lib.halftone_layer_max(*a) == hb.HS_EINVAL
    a = list(largs); a[4] = 0
    assert lib.halftone_layer_max(*a) == hb.HS_ESHAPE
    a = list(largs); a[9] = fws - 1
    assert lib.halftone_layer_max(*a) == hb.HS_EWORKSPACE
