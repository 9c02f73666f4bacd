"""Training of the policy (Algorithm 1, TRAIN) and the held-out judge.

Every training iteration is one `policy_train_step` call: forward of the
batch and of the constant-gray side batch, Bernoulli actions, the Local
Expectation gradient of the reward (Sec. III-B/C), the anisotropy gradient
(Eq. as), backward through the conv stack and Adam with the cosine schedule
(Sec. VI-A) -- all in the library's kernels. This module only feeds it
batches and seeds.

Training data: a pool of synthetic contones (the seeded generator of
`synth.contone`, standing in for the paper's photograph crops), a share of
which (--flat-frac, default 1/4) are constant grays drawn uniformly from
[0, 1] -- photographs hold flat areas at every gray, the textured generator
only at its clamps, and a policy that never sees a mid-gray flat under the
reward is free to render it black, which also zeroes the anisotropy loss of
the side batch -- and the 64 constant grays (k + 1/2) / 64 of the side
batch. The judge halftones
held-out contones with the policy (bits = [p >= 0.5], Alg. 1 TEST) and with
Floyd-Steinberg error diffusion, and scores both by the HVS-filtered MSE of
`halftone_loss` (Gaussian sigma = 2, 11 x 11, valid region); a second judge
does the same on 16 constant grays (k + 1/2) / 16.

Command line (prints a progress line every few seconds and one JSON line
at the end):
    python -m paper_2304_12152_amd.train --steps 50000 --out weights.npy
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import synth

TRAIN_SEED0 = 1_000_000   # training contones: seeds TRAIN_SEED0 + i
JUDGE_SEED0 = 2_000_000   # held-out contones: seeds JUDGE_SEED0 + i
MASK64 = (1 << 64) - 1


def _contone_chunk(args):
    seeds, H, W = args
    return synth.contone_batch(seeds, H, W)


def contone_pool(seeds, H, W, workers=None):
    """float32 [N, H, W] numpy array of synthetic contones.

    Uses forked host workers; call it before anything initialises the GPU."""
    seeds = list(seeds)
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(seeds) < 64:
        return synth.contone_batch(seeds, H, W)
    chunk = (len(seeds) + 4 * workers - 1) // (4 * workers)
    jobs = [(seeds[i:i + chunk], H, W) for i in range(0, len(seeds), chunk)]
    import multiprocessing as mp
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        parts = list(ex.map(_contone_chunk, jobs))
    return np.concatenate(parts).astype(np.float32)


def step_seeds(run_seed, step, n, salt=0):
    """Per-image Philox keys of one step: distinct over (run, step, image)."""
    base = (int(run_seed) * 0x9E3779B97F4A7C15 + (int(step) * 4 + salt) * 0xD1B54A32D192ED03) & MASK64
    return np.array([(base + i) & MASK64 for i in range(n)], dtype=np.uint64)


class Trainer:
    """Holds the device pool, the side batch and the training state."""

    def __init__(self, pool, total_steps, batch=32, gray_levels=64, gray_size=64,
                 run_seed=0, weight_seed=42, head_std=0.01, precision=None, tp=None,
                 weights=None):
        import torch
        from . import binding as hb
        self.torch, self.hb = torch, hb
        dev = torch.device("cuda", torch.cuda.current_device())
        self.dev = dev
        self.pool = torch.as_tensor(pool).to(dev)
        self.N, self.H, self.W = self.pool.shape
        self.batch = batch
        self.total = int(total_steps)
        self.run_seed = run_seed
        if weights is None:
            weights = synth.he_weights(weight_seed, head_std=head_std)
        w = torch.as_tensor(np.asarray(weights, dtype=np.float32)).to(dev)
        self.gray = None
        self.Bg = 0
        if gray_levels:
            self.gray = torch.as_tensor(synth.gray_batch(gray_levels, gray_size, gray_size)).to(dev)
            self.Bg = gray_levels
        prec = hb.HS_BF16 if precision is None else precision
        self.state = hb.TrainState(w, batch, self.H, self.W, self.Bg,
                                   gray_size if gray_levels else 0,
                                   gray_size if gray_levels else 0, prec, tp)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(int(run_seed) * 7919 + 17)
        self.step_no = 0

    def step(self):
        torch, hb = self.torch, self.hb
        idx = torch.randint(0, self.N, (self.batch,), generator=self.gen, device=self.dev)
        contones = self.pool.index_select(0, idx).contiguous()
        seeds = torch.as_tensor(step_seeds(self.run_seed, self.step_no, self.batch).view(np.int64)).to(self.dev)
        gseeds = None
        if self.gray is not None:
            gseeds = torch.as_tensor(step_seeds(self.run_seed, self.step_no, self.Bg, salt=1).view(np.int64)).to(self.dev)
        m = hb.policy_train_step(self.state, contones, seeds, self.gray, gseeds,
                                 self.step_no, self.total)
        self.step_no += 1
        return m

    @property
    def weights(self):
        return self.state.weights


def judge(weights, contones, seeds, precision=None, with_fs=True, levels=2):
    """Mean HVS-MSE of the policy's halftones (and of Floyd-Steinberg's).

    contones: float32 [N, H, W] (host); seeds: uint64 [N] noise keys. With
    levels > 2 the policy's output is its multitone (nearest-level) image
    and the reference is Floyd-Steinberg with the same levels."""
    import torch
    from . import binding as hb
    dev = torch.device("cuda", torch.cuda.current_device())
    c = torch.as_tensor(contones).to(dev)
    s = torch.as_tensor(np.asarray(seeds, dtype=np.uint64).view(np.int64)).to(dev)
    w = torch.as_tensor(np.asarray(weights, dtype=np.float32)).to(dev) \
        if not torch.is_tensor(weights) else weights.to(dev)
    prec = hb.HS_FP32 if precision is None else precision
    out = {}
    N = c.shape[0]
    if levels > 2:
        H, W = c.shape[1:]
        k = hb.halftone_infer_pages(w, c.reshape(-1), s, [(H, W)] * N, precision=prec,
                                    levels=levels).view(N, H, W)
        loss = hb.halftone_loss(k, c, prm=hb.default_loss_params(levels=levels))
        fill = k.double().mean() / (levels - 1)
    else:
        bits = hb.halftone_infer(w, c, s, precision=prec)
        loss = hb.halftone_loss(bits, c)
        fill = bits.double().mean()
    loss = loss[:3 * N].view(N, 3).double()
    out["policy_hvs_mse"] = float(loss[:, 0].mean())
    out["policy_cssim"] = float(loss[:, 1].mean())
    out["policy_fill"] = float(fill)
    if with_fs:
        if levels > 2:
            fs = hb.halftone_error_diffusion_levels_host(np.asarray(contones), levels).to(dev)
            lf = hb.halftone_loss(fs, c, prm=hb.default_loss_params(levels=levels))
        else:
            fs = hb.halftone_error_diffusion_host(np.asarray(contones)).to(dev)
            lf = hb.halftone_loss(fs, c)
        lf = lf[:3 * N].view(N, 3).double()
        out["fs_hvs_mse"] = float(lf[:, 0].mean())
        out["fs_cssim"] = float(lf[:, 1].mean())
    out["contone_mean"] = float(c.double().mean())
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--pool", type=int, default=20000, help="training contones")
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--judge", type=int, default=256, help="held-out contones")
    ap.add_argument("--flat-frac", type=float, default=0.25,
                    help="share of the pool made of constant grays drawn from U(0, 1)")
    ap.add_argument("--run-seed", type=int, default=0)
    ap.add_argument("--weight-seed", type=int, default=42)
    ap.add_argument("--log-every", type=float, default=10.0, help="seconds between progress lines")
    ap.add_argument("--fp32", action="store_true", help="FP32 instead of BF16 activations")
    ap.add_argument("--ws", type=float, default=None,
                    help="CSSIM weight w_s of the reward (default 0.06; 0 = HVS-MSE only)")
    ap.add_argument("--wa", type=float, default=None, help="anisotropy weight w_a (default 0.002)")
    ap.add_argument("--wa-from", type=int, default=0,
                    help="first step with the anisotropy loss (w_a = 0 before it)")
    ap.add_argument("--estimator", choices=["le", "coma"], default="le",
                    help="policy-gradient estimator: Local Expectation (Eq. le) or COMA (Eq. coma)")
    ap.add_argument("--levels", type=int, default=2,
                    help="output levels: 2 = binary halftoning, 3..8 = multitoning (Sec. VI-E)")
    ap.add_argument("--judge-every", type=int, default=0,
                    help="steps between held-out evaluations of the policy during training")
    ap.add_argument("--out", default=None, help="write the trained weights (.npy)")
    ap.add_argument("--init", default=None,
                    help="start from these weights (.npy); with --steps 0 this only judges them")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.perf_counter()
    nflat = int(round(args.flat_frac * args.pool))
    pool = contone_pool(range(TRAIN_SEED0, TRAIN_SEED0 + args.pool - nflat), args.size, args.size)
    if nflat:
        pool = np.concatenate([pool, synth.flat_contones(TRAIN_SEED0, nflat, args.size, args.size)])
    held = contone_pool(range(JUDGE_SEED0, JUDGE_SEED0 + args.judge), args.size, args.size)
    hseeds = np.arange(JUDGE_SEED0, JUDGE_SEED0 + args.judge, dtype=np.uint64)
    gheld = synth.gray_batch(16, args.size, args.size)
    gseeds = np.arange(JUDGE_SEED0 + args.judge, JUDGE_SEED0 + args.judge + 16, dtype=np.uint64)
    log("pool: %d + %d contones %dx%d in %.1f s" % (args.pool, args.judge, args.size, args.size,
                                                  time.perf_counter() - t0))

    import torch
    from . import binding as hb
    prec = hb.HS_FP32 if args.fp32 else hb.HS_BF16
    kw = {}
    if args.ws is not None:
        kw["w_s"] = args.ws
    if args.wa is not None:
        kw["w_a"] = args.wa
    kw["estimator"] = hb.HS_EST_COMA if args.estimator == "coma" else hb.HS_EST_LE
    kw["levels"] = args.levels
    tp = hb.default_train_params(**kw)
    init = np.load(args.init).astype(np.float32) if args.init else None
    tr = Trainer(pool, args.steps, batch=args.batch, run_seed=args.run_seed,
                 weight_seed=args.weight_seed, precision=prec, tp=tp, weights=init)
    w0 = tr.weights.clone()
    before = judge(w0, held, hseeds, levels=args.levels)
    log("untrained: " + json.dumps(before))
    gbefore = judge(w0, gheld, gseeds, levels=args.levels)
    log("untrained, constant grays: " + json.dumps(gbefore))
    t1 = time.perf_counter()
    last = t1
    hist = []
    curve = []
    wa_full = tp.loss.w_a
    if args.wa_from > 0:
        tr.state.tp.loss.w_a = 0.0
    for i in range(args.steps):
        if args.wa_from > 0 and i == args.wa_from:
            tr.state.tp.loss.w_a = wa_full
            log("step %d: anisotropy loss on (w_a = %g)" % (i, wa_full))
        m = tr.step()
        now = time.perf_counter()
        if now - last >= args.log_every or i == args.steps - 1:
            mv = m.cpu().tolist()
            hist.append([i + 1] + mv[:7])
            log("step %d/%d  %.1f steps/s  mse %.5f cssim %.4f R %.5f L_AS %.4g lr %.2e |g| %.3g fill %.3f"
                % (i + 1, args.steps, (i + 1) / (now - t1), mv[0], mv[1], mv[2], mv[3], mv[4],
                   mv[5], mv[6]))
            last = now
        if args.judge_every and (i + 1) % args.judge_every == 0 and i + 1 < args.steps:
            j = judge(tr.weights, held, hseeds, with_fs=False, levels=args.levels)
            curve.append([i + 1, j["policy_hvs_mse"], j["policy_fill"]])
            log("judge at step %d: policy HVS-MSE %.6g (FS %.6g) fill %.4f"
                % (i + 1, j["policy_hvs_mse"], before["fs_hvs_mse"], j["policy_fill"]))
    torch.cuda.synchronize()
    train_s = max(time.perf_counter() - t1, 1e-9)
    after = judge(tr.weights, held, hseeds, levels=args.levels)
    log("trained: " + json.dumps(after))
    gafter = judge(tr.weights, gheld, gseeds, levels=args.levels)
    log("trained, constant grays: " + json.dumps(gafter))
    if args.out:
        np.save(args.out, tr.weights.cpu().numpy())
    res = {"steps": args.steps, "batch": args.batch, "pool": args.pool, "size": args.size,
           "w_s": tp.loss.w_s, "w_a": tp.loss.w_a, "estimator": args.estimator,
           "precision": "fp32" if args.fp32 else "bf16", "train_seconds": round(train_s, 2),
           "steps_per_s": round(args.steps / train_s, 2), "judge_images": args.judge,
           "flat_frac": args.flat_frac, "levels": args.levels, "wa_from": args.wa_from,
           "untrained": before, "trained": after, "judge_curve": curve,
           "untrained_gray": gbefore, "trained_gray": gafter,
           "trained_beats_fs": after["policy_hvs_mse"] < after["fs_hvs_mse"]}
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
