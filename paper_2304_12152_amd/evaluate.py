"""Blue-noise evaluation of a policy: the spectral analysis of constant-gray
halftones (Sec. IV, Eqs. psd, rapsd, anis; the paper's spectral figure
shows the grays 15, 80, 100 and 127 of 255).

For every gray g a batch of B constant pages of H x W is halftoned by the
policy (Alg. 1 TEST, a packed policy's `halftone_policy_infer`, in the
cheapest exact-bit precision that `calibrate.plan` finds for the weights,
with the recheck bands measured per gray) and by Floyd-Steinberg error
diffusion; `halftone_spectrum` estimates the power spectrum as the mean
periodogram of all P x P patches of the batch and reduces it to the radially
averaged power and the anisotropy per ring. Reported per method and gray:
  fill        the fraction of ones (against g);
  hvs_mse     the HVS-filtered MSE of `halftone_loss`;
  rapsd_db    10 log10(RAPSD / (g (1 - g))) for rings 1 .. P/2, the power
              relative to the white-noise level of the same gray;
  anis_db     10 log10(anisotropy) for rings 1 .. P/2 (rings with zero
              power report -inf);
  anis_mean_db the mean of anis_db over those rings;
  low_power   the share of the AC power in rings below the principal
              frequency sqrt(min(g, 1 - g)) (in cycles per pixel, times P);
  policy only: bands, the recheck bands measured for the weights on two
              of the gray's pages (`calibrate.bands`); logit_hist,
              the fraction of pixels whose logit magnitude
              |x| falls in the decades [0, 1e-4), [1e-4, 1e-3), ...,
              [10, inf) -- a bimodal policy keeps almost all of them in the
              top decades -- and recheck / split / fp32, the fractions the
              16-bit path listed, recomputed with split-BF16 and in FP32;
              with levels > 2
              also near_level, the share of v (L - 1) within 0.1 of an
              integer.
With K periodograms averaged, an isotropic spectrum has anisotropy about
1 / K, so -10 log10(K) dB is the floor the figures are read against.
With --levels L > 2 the policy is the multitoning variant (Sec. VI-E): its
output is the level index k, the image k / (L - 1) is scored, and its
power is taken in units of that image (the level indices' spectrum divided
by (L - 1)^2); the reference is Floyd-Steinberg with the same L levels.

Command line:
    python -m paper_2304_12152_amd.evaluate --weights weights.npy
"""
import argparse
import json
import math
import sys

import numpy as np

from . import calibrate
from . import synth

GRAYS = (15, 80, 100, 127)
LOGIT_DECADES = (1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0)


def _summary(bits, c, g, P, hb, levels=2):
    B = c.shape[0]
    loss = hb.halftone_loss(bits, c, prm=hb.default_loss_params(levels=levels))
    loss = loss[:3 * B].view(B, 3).double()
    r, a = hb.halftone_spectrum(bits, P)
    r = r.double().cpu().numpy() / float((levels - 1) ** 2)
    a = a.double().cpu().numpy()
    var = g * (1.0 - g)
    rings = np.arange(1, P // 2 + 1)
    with np.errstate(divide="ignore"):
        rdb = 10.0 * np.log10(r[rings] / var)
        adb = 10.0 * np.log10(a[rings])
    ac = r[1:]
    counts = _ring_counts(P)[1:]
    fp = math.sqrt(min(g, 1.0 - g)) * P
    low = float((ac * counts)[np.arange(1, len(r)) < fp].sum() / max((ac * counts).sum(), 1e-30))
    return {
        "fill": float(bits.double().mean()) / (levels - 1),
        "hvs_mse": float(loss[:, 0].mean()),
        "rapsd_db": [round(float(v), 3) for v in rdb],
        "anis_db": [round(float(v), 3) for v in adb],
        "anis_mean_db": float(np.mean(adb[np.isfinite(adb)])) if np.isfinite(adb).any() else None,
        "low_power": low,
    }


def _ring_counts(P):
    """Number of frequencies per ring (the folded radius rounded half up)."""
    u = np.arange(P)
    ub = np.minimum(u, P - u)
    q4 = 4 * (ub[:, None] ** 2 + ub[None, :] ** 2)
    rho = np.floor((np.sqrt(q4) + 1.0) / 2.0).astype(int)
    # exact integer correction of the float estimate
    rho = np.where((2 * rho + 1) ** 2 <= q4, rho + 1, rho)
    rho = np.where((rho > 0) & ((2 * rho - 1) ** 2 > q4), rho - 1, rho)
    return np.bincount(rho.ravel())


def bluenoise(weights, grays=GRAYS, B=8, H=512, W=512, P=64, precision=None, with_fs=True,
              seed=1000, levels=2):
    """Spectral summary per gray level (dict keyed by the gray out of 255)."""
    import torch
    from . import binding as hb
    dev = torch.device("cuda", torch.cuda.current_device())
    w = torch.as_tensor(np.asarray(weights, dtype=np.float32)).to(dev)
    # default: the cheapest exact-bit precision for these weights
    prec = calibrate.plan(w, levels=levels)["precision"] if precision is None else precision
    pol = hb.Policy(w)
    out = {"P": P, "periodograms": B * (H // P) * (W // P), "pages": [B, H, W],
           "precision": {hb.HS_FP32: "fp32", hb.HS_BF16: "bf16", hb.HS_FP16: "fp16"}[prec]}
    out["floor_db"] = -10.0 * math.log10(out["periodograms"])
    for gi in grays:
        g = gi / 255.0
        c = torch.full((B, H, W), g, dtype=torch.float32, device=dev)
        s = torch.arange(seed + B * gi, seed + B * gi + B, dtype=torch.int64, device=dev)
        # the recheck bands for these weights, measured on two of the pages
        if prec != hb.HS_FP32:
            b = calibrate.bands(w, prec, c[:2], s[:2].tolist(), levels=levels)
        else:
            b = {"tau": 0.0, "tau16": -1.0, "tau2": -1.0}
        bits, x, st = hb.halftone_policy_infer(pol, c, s, precision=prec, recheck_tau=b["tau"],
                                               recheck_tau16=b["tau16"], recheck_tau2=b["tau2"],
                                               logits=True, stats=True, levels=levels)
        rec = {"policy": _summary(bits, c, g, P, hb, levels)}
        n = float(B * H * W)
        edges = torch.tensor(LOGIT_DECADES, dtype=torch.float32, device=dev)
        cnt = torch.bucketize(x.abs().flatten(), edges, right=True).bincount(
            minlength=len(LOGIT_DECADES) + 1)
        rec["policy"]["logit_hist"] = [round(float(v) / n, 6) for v in cnt.cpu()]
        if levels > 2:
            # the paper's multitone histogram: outputs gather at the levels
            t = torch.sigmoid(x.double()) * (levels - 1)
            rec["policy"]["near_level"] = float(((t - t.round()).abs() < 0.1).double().mean())
        st = st.cpu().numpy()
        rec["policy"]["bands"] = {k: v for k, v in b.items() if k != "errors"}
        rec["policy"]["recheck"] = float(st[0]) / n
        rec["policy"]["split"] = float(st[4]) / n
        rec["policy"]["fp32"] = float(st[2]) / n
        if with_fs:
            flat = np.full((B, H, W), g, dtype=np.float32)
            fs = (hb.halftone_error_diffusion_levels_host(flat, levels) if levels > 2
                  else hb.halftone_error_diffusion_host(flat))
            rec["fs"] = _summary(fs.to(dev), c, g, P, hb, levels)
        out[str(gi)] = rec
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--weights", help=".npy of the flat FP32 weights (default: He init)")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--P", type=int, default=64, choices=(32, 64))
    ap.add_argument("--no-fs", action="store_true")
    ap.add_argument("--levels", type=int, default=2, help="2 = halftone, 3..8 = multitone")
    ap.add_argument("--out", help="write the JSON here as well")
    a = ap.parse_args(argv)
    w = np.load(a.weights) if a.weights else synth.he_weights(42)
    res = bluenoise(w, B=a.batch, H=a.size, W=a.size, P=a.P, with_fs=not a.no_fs,
                    levels=a.levels)
    for gi in GRAYS:
        for m, r in res[str(gi)].items():
            am = r["anis_mean_db"]
            print(f"g={gi:3d}/255 {m:6s} fill={r['fill']:.4f} hvs_mse={r['hvs_mse']:.3e} "
                  f"anis_mean={am if am is None else round(am, 2)} dB "
                  f"low_power={r['low_power']:.3f}", flush=True)
    line = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")
    print(line)
    return 0


if __name__ == "__main__":
    sys.exit(main())
