"""Train the learned surrogate on the GPU with the library's own kernels.

Data: seeded 256 x 256 RGB crops (Voronoi cells + Gaussian detail, 10-40
cells, sigma 0.05; lambda ~ U[0.5, 2], p ~ U[0.5, 1]), labelled by plain
GPU ILS with N = 4 (batched, one launch per pass).  Training: mean squared
error, Adam with a linear warm-up and cosine decay of the learning rate,
shuffled mini-batches; after every epoch the network is scored on held-out
validation crops (PSNR against plain ILS) and the best epoch's parameters
are the ones saved.  --grad-log N prints per-layer gradient norms and Adam
step sizes every N steps (diagnostics for the learning rate).  The gate
threshold tau is the 99th percentile of the fixed-point residual of plain
ILS N = 4 itself on held-out calibration crops.  Checkpoints hold the
parameters, Adam moments, step, epoch and the shuffling RNG state.

    python -m paper_2003_07504_amd.train_surrogate --crops 20000 --epochs 60 \
        --out paper_2003_07504_amd/weights/surrogate.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _say(msg):
    print(f"[train] {msg}", flush=True)


def _gen(spec):
    return spec.image()


def make_crops(n, first_seed, workers):
    from synth import train_crop_specs
    specs = train_crop_specs(n, first_seed=first_seed)
    imgs = np.empty((n, 3, 256, 256), dtype=np.float32)
    with Pool(workers) as pool:
        for i, im in enumerate(pool.imap(_gen, specs, chunksize=32)):
            imgs[i] = im
    lam = np.array([s.lam for s in specs], dtype=np.float32)
    p = np.array([s.p for s in specs], dtype=np.float32)
    return imgs, lam, p


def label_with_ils(plan, f_dev, lam, p, chunk=64):
    """Plain GPU ILS N = 4 for every crop (batched calls)."""
    import torch
    out = torch.empty_like(f_dev)
    for s in range(0, f_dev.shape[0], chunk):
        e = min(s + chunk, f_dev.shape[0])
        frames = [(f_dev[i], float(lam[i]), float(p[i]), 1e-4, 4) for i in range(s, e)]
        plan.smooth_batch(frames, outs=[out[i] for i in range(s, e)])
    torch.cuda.synchronize()
    return out


def residuals(plan, f_dev, u_dev, lam, p):
    """rms(T(u) - u) per image, T = one ILS iteration from u with data term f."""
    import torch
    tv = torch.empty_like(u_dev)
    for i in range(f_dev.shape[0]):
        plan.iterate_from(f_dev[i], u_dev[i], float(lam[i]), float(p[i]), 1e-4, 1, out=tv[i])
    out = []
    for s in range(0, tv.shape[0], 512):  # at most 512 images per reduction call
        e = min(s + 512, tv.shape[0])
        out.append(plan.rms_diff([tv[i] for i in range(s, e)], [u_dev[i] for i in range(s, e)]))
    torch.cuda.synchronize()
    return torch.cat(out).cpu().numpy()


def psnr(a, b):
    mse = float(((a - b) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--crops", type=int, default=20000)
    ap.add_argument("--calib", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=4e-4)
    ap.add_argument("--lr-min", type=float, default=1e-5)
    ap.add_argument("--warmup", type=int, default=1500, help="steps of linear learning-rate warm-up")
    ap.add_argument("--val", type=int, default=256, help="validation crops scored after every epoch")
    ap.add_argument("--grad-log", type=int, default=0, help="log per-layer gradient norms every N steps")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2003_07504_amd", "weights", "surrogate.npz"))
    ap.add_argument("--resume", default=None)
    ap.add_argument("--max-seconds", type=float, default=1e9, help="stop (checkpointed) after this much training")
    args = ap.parse_args()

    import torch

    from paper_2003_07504_amd import ils, surrogate

    t0 = time.time()
    _say(f"generating {args.crops} training crops and {args.calib} calibration crops")
    f_np, lam, p = make_crops(args.crops, 100000, args.workers)
    fc_np, lamc, pc = make_crops(args.calib, 200000, args.workers)
    _say(f"  done in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    f = torch.from_numpy(f_np).to(dev)
    fc = torch.from_numpy(fc_np).to(dev)
    del f_np, fc_np
    plan = ils.Plan(256, 256, 3, max_frames=64)
    t1 = time.time()
    tgt = label_with_ils(plan, f, lam, p)
    tgtc = label_with_ils(plan, fc, lamc, pc)
    _say(f"labelled {args.crops + args.calib} crops with plain ILS N=4 in {time.time() - t1:.2f}s")
    rc = residuals(plan, fc, tgtc, lamc, pc)
    tau = float(np.quantile(rc, 0.99))
    _say(f"calibration: residual of plain ILS N=4 median {np.median(rc):.3e}, 99th pct (tau) {tau:.3e}")

    net = surrogate.Net(args.batch, 256, 256, device=dev, seed=args.seed)
    rng = np.random.default_rng(args.seed)
    epoch0 = 0
    if args.resume:
        meta = net.load(args.resume)
        epoch0 = int(meta.get("epoch", 0))
        if "rng_state" in meta:
            rng.bit_generator.state = json.loads(str(meta["rng_state"]))
        _say(f"resumed from {args.resume} at epoch {epoch0}, step {net.get_state()[3]}")
    steps_per_epoch = args.crops // args.batch
    total = steps_per_epoch * args.epochs
    lam_d = torch.from_numpy(lam).to(dev)
    p_d = torch.from_numpy(p).to(dev)
    t_train = time.time()
    stopped = False
    nval = min(args.val, fc.shape[0])

    def val_psnr():
        v = torch.empty_like(fc[:nval])
        for s0 in range(0, nval, args.batch):
            e0 = min(s0 + args.batch, nval)
            net.forward(fc[s0:e0].contiguous(), torch.from_numpy(lamc[s0:e0]).to(dev),
                        torch.from_numpy(pc[s0:e0]).to(dev), out=v[s0:e0])
        mse = ((v - tgtc[:nval]) ** 2).mean(dim=(1, 2, 3)).double().cpu().numpy()
        return float(np.mean(10.0 * np.log10(1.0 / np.maximum(mse, 1e-30))))

    sizes = surrogate.layer_param_sizes()
    best = (-1.0, None, 0)  # (validation PSNR, state, epoch)
    for ep in range(epoch0, args.epochs):
        perm = rng.permutation(args.crops)
        losses = []
        te = time.time()
        for s in range(steps_per_epoch):
            step = ep * steps_per_epoch + s
            if step < args.warmup:
                lr = args.lr * (step + 1) / args.warmup
            else:
                t = (step - args.warmup) / max(1, total - args.warmup)
                lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1 + np.cos(np.pi * t))
            idx = torch.from_numpy(perm[s * args.batch:(s + 1) * args.batch]).to(dev)
            fb = f.index_select(0, idx).contiguous()
            tb = tgt.index_select(0, idx).contiguous()
            lb, pb = lam_d.index_select(0, idx), p_d.index_select(0, idx)
            if args.grad_log and step % args.grad_log == 0:
                g = net.gradients(fb, lb, pb, tb)[0].cpu().numpy()
                p0 = net.get_state()[0]
                loss = net.train_step(fb, lb, pb, tb, lr)
                dp = net.get_state()[0] - p0
                norms, steps_, o = [], [], 0
                for n in sizes:
                    norms.append(float(np.linalg.norm(g[o:o + n])))
                    steps_.append(float(np.linalg.norm(dp[o:o + n]) / max(np.linalg.norm(p0[o:o + n]), 1e-30)))
                    o += n
                _say(f"step {step}: lr {lr:.2e} loss {float(loss.cpu()):.3e} grad norms "
                     + " ".join(f"{x:.2e}" for x in norms) + " | relative Adam steps "
                     + " ".join(f"{x:.1e}" for x in steps_))
            else:
                loss = net.train_step(fb, lb, pb, tb, lr)
            if s % 100 == 0:
                losses.append(float(loss.cpu()))
        torch.cuda.synchronize()
        vp = val_psnr()
        if vp > best[0]:
            best = (vp, net.get_state(), ep + 1)
        ckpt_rng = json.dumps(rng.bit_generator.state)
        os.makedirs(os.path.dirname(args.out), exist_ok=True)
        net.save(args.out + ".ckpt.npz", epoch=np.int64(ep + 1), rng_state=np.array(ckpt_rng), tau=np.float32(tau))
        _say(f"epoch {ep + 1}/{args.epochs}: loss {np.mean(losses):.3e} (last {losses[-1]:.3e}), "
             f"validation {vp:.2f} dB (best {best[0]:.2f} at epoch {best[2]}), {time.time() - te:.1f}s, lr {lr:.2e}")
        if time.time() - t_train > args.max_seconds:
            _say("time budget reached; checkpoint written")
            stopped = True
            break
    if best[1] is not None:
        net.set_state(*best[1])
        _say(f"keeping the parameters of epoch {best[2]} (validation {best[0]:.2f} dB)")

    # validation on the calibration crops: PSNR vs plain ILS, residuals, gate
    vs = torch.empty_like(fc)
    for s in range(0, fc.shape[0], args.batch):
        e = min(s + args.batch, fc.shape[0])
        net.forward(fc[s:e].contiguous(), torch.from_numpy(lamc[s:e]).to(dev), torch.from_numpy(pc[s:e]).to(dev),
                    out=vs[s:e])
    torch.cuda.synchronize()
    rv = residuals(plan, fc, vs, lamc, pc)
    ps = [psnr(vs[i].cpu().numpy(), tgtc[i].cpu().numpy()) for i in range(fc.shape[0])]
    _say(f"validation: PSNR vs plain ILS mean {np.mean(ps):.2f} dB (min {np.min(ps):.2f}), "
         f"gate pass rate {np.mean(rv <= tau):.3f}")
    p_, m_, v_, st = net.get_state()
    np.savez(args.out, params=p_, m=m_, v=v_, step=np.int64(st), tau=np.float32(tau),
             epoch=np.int64(best[2] if best[1] is not None else (args.epochs if not stopped else ep + 1)),
             val_psnr_mean=np.float32(np.mean(ps)), val_pass_rate=np.float32(np.mean(rv <= tau)),
             crops=np.int64(args.crops), batch=np.int64(args.batch))
    _say(f"saved {args.out} ({time.time() - t0:.1f}s total)")
    net.close()
    plan.close()


if __name__ == "__main__":
    main()
