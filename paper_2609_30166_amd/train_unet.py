"""Train the correction network on generated phantoms and compare the learned
pipeline with plain SIRT.

    python -m paper_2609_30166_amd.train_unet --phantoms 512 --test 32 \
        --out weights.npz --summary summary.json

Training follows the stage-wise scheme of ``learned.train`` on the
learned-correction configuration (256^3 volumes, 180 projections of 384^2
pixels, Poisson noise at 1e4 incident photons); the summary holds the loss
history and the held-out comparison (PSNR, ||A x - b||, wall time).
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from synth import configs

from . import learned
from .unet import UNet


def save(path, nets, meta, optimizer_state=True):
    """The stage networks' parameters (and, optionally, their Adam moments
    and steps) as one .npz; keys are prefixed ``s<k>.``."""
    nets = nets if isinstance(nets, (list, tuple)) else [nets]
    arrays = dict(n_nets=np.int64(len(nets)), meta=json.dumps(meta))
    for k, net in enumerate(nets):
        pre = "s%d." % k
        arrays[pre + "scale"] = np.float64(net.scale)
        arrays.update({pre + "p." + n: v for n, v in net.params().items()})
        if optimizer_state:
            st = net.state_dict()
            arrays.update({pre + "step": np.int64(st["step"]), pre + "theta": st["theta"],
                           pre + "m": st["m"], pre + "v": st["v"]})
    np.savez(path, **arrays)


def load(path, device=None):
    """The list of stage UNets stored by ``save`` (with their Adam state
    when present)."""
    z = np.load(path, allow_pickle=False)
    nets = []
    for k in range(int(z["n_nets"])):
        pre = "s%d." % k
        params = {n[len(pre) + 2:]: z[n] for n in z.files if n.startswith(pre + "p.")}
        net = UNet(device, params=params, scale=float(z[pre + "scale"]))
        if pre + "theta" in z.files:
            net.load_state_dict(dict(theta=z[pre + "theta"], m=z[pre + "m"], v=z[pre + "v"],
                                     step=int(z[pre + "step"])))
        nets.append(net)
    return nets


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--phantoms", type=int, default=512)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--stages", type=int, default=4)
    ap.add_argument("--iters-per-stage", type=int, default=1)
    ap.add_argument("--sirt-iters", type=int, default=50)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--crop", type=int, default=128,
                    help="edge of the random training blocks (0 = whole volume)")
    ap.add_argument("--crop-steps", type=int, default=8, help="Adam steps per stage sample")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--scale", type=float, default=None,
                    help="network input scale (default: the volume width, since the "
                         "configuration stores attenuation per volume width)")
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--subsets", type=int, default=0,
                    help="physics steps: OS-SIRT epochs over this many interleaved "
                         "projection subsets (0 or 1: plain SIRT iterations)")
    ap.add_argument("--shared", action="store_true",
                    help="one network for all stages (default: one per stage)")
    ap.add_argument("--eval-only", action="store_true",
                    help="skip training: evaluate the network of --resume")
    ap.add_argument("--weights-only", default=None,
                    help="also write the parameters alone (no optimizer state) here")
    ap.add_argument("--resume", default=None, help="weights file to continue from")
    ap.add_argument("--out", default="unet_weights.npz")
    ap.add_argument("--summary", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    cfg, geom = learned.learned_geometry()
    scale = a.scale if a.scale else float(min(cfg.shape[1:]))
    if a.resume:
        net = load(a.resume, geom.device)
    else:
        n_nets = 1 if a.shared else a.stages
        net = [UNet(geom.device, seed=a.seed + k, scale=scale) for k in range(n_nets)]
    seeds = list(configs.TRAIN_SEEDS)[:a.phantoms]
    t0 = time.time()
    summary = {}
    if not a.eval_only:
        hists = []
        for ep in range(a.epochs):
            log("epoch %d" % (ep + 1))
            hists.append(learned.train(geom, net, cfg, seeds, lr=a.lr, lr_final=a.lr_final,
                                       n_stages=a.stages, iters_per_stage=a.iters_per_stage,
                                       crop=a.crop or None, crop_steps=a.crop_steps, log=log,
                                       seed=a.seed + ep, subsets=a.subsets or None))
        hist = np.concatenate(hists)
        t_train = time.time() - t0
        meta = dict(config="learned", phantoms=a.phantoms, epochs=a.epochs, stages=a.stages,
                    iters_per_stage=a.iters_per_stage, lr=a.lr, lr_final=a.lr_final,
                    crop=a.crop, crop_steps=a.crop_steps, seed=a.seed, scale=net[0].scale,
                    train_s=t_train, networks=len(net), adam_steps=[n.step for n in net],
                    fov_mask=True, subsets=a.subsets)
        save(a.out, net, meta)
        if a.weights_only:
            save(a.weights_only, net, meta, optimizer_state=False)
        log("trained on %d phantoms in %.1f s -> %s" % (len(seeds), t_train, a.out))
        summary = dict(meta=meta, mse_first=hist[:8].mean(0).tolist(),
                       mse_last_ellipsoids=hist[-8::2].mean(0).tolist(),
                       mse_last_foam=hist[-7::2].mean(0).tolist())
    if a.test > 0:
        fov = True
        if a.eval_only and a.resume:
            m = json.loads(str(np.load(a.resume, allow_pickle=False)["meta"]))
            fov = bool(m.get("fov_mask", False))
            a.stages, a.iters_per_stage = int(m["stages"]), int(m["iters_per_stage"])
            a.subsets = int(m.get("subsets", 0))
        res = learned.compare(geom, net, cfg, list(configs.TEST_SEEDS)[:a.test],
                              sirt_iters=a.sirt_iters, n_stages=a.stages,
                              iters_per_stage=a.iters_per_stage, log=log, fov=fov,
                              subsets=a.subsets or None)
        summary["compare"] = res
        m = res["mean"]
        log("mean PSNR: SIRT-%d %.2f dB, physics alone (%s, %d steps) %.2f dB, learned %.2f dB; "
            "time %.3f s vs %.3f s (ratio %.3f); learned >= SIRT-%d PSNR on every phantom: %s" % (
                a.sirt_iters, m["psnr_sirt"], res["physics"], a.stages * a.iters_per_stage,
                m["psnr_sirt_same_budget"], m["psnr_learned"], m["t_learned"], m["t_sirt"],
                res["time_ratio"], a.sirt_iters, res["learned_reaches_sirt_psnr"]))
    if a.summary:
        with open(a.summary, "w") as f:
            json.dump(summary, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
