"""Unrolled SIRT with a learned correction between iterations.

The paper names learned correction terms between physics-based operator
applications as the extension of its operator framework (Sec. 5).  Here the
correction is the 3D U-Net of ``unet.UNet`` applied after each of a few
unrolled SIRT iterations of Eq. (1), with the data residual as the arbiter:

* stage k: ``iters_per_stage`` SIRT updates x <- x + alpha C A^T R (b - A x)
  (libctrex ``ctrex_sirt_iterate``) — or, with ``subsets``, that many epochs
  of ordered-subset SIRT (Sec. 2.3.2: Eq. (1) once per subset of
  projections, each with its own R and C) — then x~ = x + m U_k(x) with the
  stage's own network (or one network shared by all stages), m the scanned
  field of view (the inscribed cylinder about the rotation axis);
* the correction is kept only if ||A x~ - b|| <= ||A x - b||
  (``ctrex_residual_norm``); otherwise it is discarded and the remaining
  stages run plain SIRT (the fallback);
* training is stage-wise: MSE of x + U_k(x) to the true volume, Adam, batch
  1, the SIRT inputs of each stage taken from the pipeline as it stands (no
  gradient through the projector).

Every operator, network layer, loss and optimizer step runs in libctrex's
kernels; this module sequences them.  Phantom and noise synthesis for
training come from ``synth`` (input generation), and the reporting metric
(PSNR) is a torch reduction on the device.
"""

from __future__ import annotations

import time

import numpy as np
import torch

from synth import configs, noise

from .projector import Geometry, ordered_subsets
from .unet import UNet


def learned_geometry(device=None, n_proj=None):
    """The projector for the learned-correction configuration (256^3 volume,
    180 projections of 384^2 pixels on a circular cone-beam orbit)."""
    cfg = configs.make_config("learned", n_proj=n_proj)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=device)
    return cfg, g


def noise_generator(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(1_000_003 * int(seed) + 17)
    return g


def make_sample(cfg, geom, seed, I0=None):
    """(x_true, b): a phantom and its noisy sinogram -ln(Poisson(I0 e^{-A x}) / I0)."""
    x_true = configs.make_learned_phantom(cfg, seed, geom.device, dtype=torch.float32).contiguous()
    y = geom.forward(x_true)
    I0 = I0 if I0 is not None else cfg.extra.get("I0", 1e4)
    b = noise.poisson_log_transform_torch(y, I0, noise_generator(seed, geom.device)).contiguous()
    return x_true, b


def fov_mask(shape, device):
    """Inscribed cylinder about the z axis (radius (min(nx, ny) - 1) / 2)."""
    nz, ny, nx = shape
    y = torch.arange(ny, device=device, dtype=torch.float64) - 0.5 * (ny - 1)
    x = torch.arange(nx, device=device, dtype=torch.float64) - 0.5 * (nx - 1)
    r = 0.5 * (min(nx, ny) - 1)
    disc = (x[None, :] ** 2 + y[:, None] ** 2) <= r * r
    return disc.expand(nz, ny, nx)


def fov_weight(shape, device):
    """The field-of-view mask as float32 weights (1 inside, 0 outside)."""
    return fov_mask(shape, device).to(torch.float32).contiguous()


def psnr(x, x_true, mask):
    """10 log10(range^2 / MSE) with range = max - min of x_true, MSE in mask."""
    t = x_true.double()
    rng = float(t.max() - t.min())
    d = (x.double() - t)[mask]
    mse = float((d * d).mean())
    return float("inf") if mse == 0 else 10.0 * np.log10(rng * rng / mse)


def _subsets(geom, subsets):
    """None (plain SIRT), a subset count (interleaved subsets) or explicit lists."""
    if subsets is None or isinstance(subsets, (list, tuple)):
        return subsets
    return ordered_subsets(geom.n_proj, int(subsets)) if int(subsets) > 1 else None


def physics(geom, x, b, iters, subsets=None, alpha=1.0):
    """``iters`` SIRT iterations of Eq. (1), or ``iters`` OS-SIRT epochs over
    ``subsets`` (lists of projections); in place, no host wait."""
    if subsets is None:
        geom.sirt(x, b, iters, alpha=alpha, norms=False)
    else:
        geom.os_sirt(x, b, subsets, iters, alpha=alpha)


def _stage_nets(net, n_stages):
    nets = list(net) if isinstance(net, (list, tuple)) else [net]
    if len(nets) not in (1, n_stages):
        raise ValueError("give one network or one per stage (%d)" % n_stages)
    return nets if len(nets) == n_stages else nets * n_stages


class LearnedSirt:
    """``n_stages`` x (SIRT update(s) + U-Net correction) with the residual
    acceptance rule and plain-SIRT fallback.  ``net``: one UNet for all
    stages or a list with one per stage."""

    def __init__(self, geom, net, n_stages=4, iters_per_stage=1, alpha=1.0, mask="fov",
                 subsets=None):
        self.geom = geom
        self.subsets = _subsets(geom, subsets)
        self.n_stages, self.iters = int(n_stages), int(iters_per_stage)
        self.nets = _stage_nets(net, self.n_stages)
        self.alpha = float(alpha)
        self.mask = fov_weight(geom.shape, geom.device) if isinstance(mask, str) else mask

    def __call__(self, b, x=None):
        """Reconstruct from sinogram ``b``; returns (x, per-stage records)."""
        g = self.geom
        if x is None:
            x = torch.zeros(g.shape, dtype=torch.float32, device=g.device)
        stages = []
        fallback = False
        for k in range(self.n_stages):
            physics(g, x, b, self.iters, self.subsets, self.alpha)
            if fallback:
                stages.append(dict(stage=k, corrected=False, fallback=True))
                continue
            rho = g.residual_norm(x, b)
            xt = self.nets[k].forward(x, mask=self.mask)
            rho_t = g.residual_norm(xt, b)
            ok = bool(rho_t <= rho)
            if ok:
                x = xt
            else:
                fallback = True
            stages.append(dict(stage=k, corrected=ok, fallback=not ok, rho_sirt=rho,
                               rho_corrected=rho_t))
        return x, stages


def train(geom, net, cfg, seeds, lr=1e-3, lr_final=None, n_stages=4, iters_per_stage=1,
          crop=None, crop_steps=1, log=None, log_every=8, seed=0, subsets=None):
    """Stage-wise training over the phantoms of ``seeds``.

    Each stage runs the SIRT update(s) on the full volume, then takes
    ``crop_steps`` Adam steps on random ``crop``^3 blocks of (iterate, truth)
    (the whole volume when ``crop`` is None), then corrects the full volume
    with the updated network to form the next stage's input.  The learning
    rate falls linearly from ``lr`` to ``lr_final`` over the run.  The
    correction is confined to the field of view, so the loss sees only the
    errors there (outside it the output is the iterate itself).  Returns
    per phantom and stage [loss of the SIRT iterate, loss after correction]
    on the full volume (MSE to the truth, measured before the stage's steps
    and after them)."""
    rng = np.random.default_rng([seed, 23])
    nets = _stage_nets(net, n_stages)
    subsets = _subsets(geom, subsets)
    lr_final = lr if lr_final is None else lr_final
    mask = fov_weight(geom.shape, geom.device)
    total = len(seeds) * n_stages * crop_steps
    k_step = 0
    hist = []
    t0 = time.time()
    nz, ny, nx = geom.shape
    for i, pseed in enumerate(seeds):
        x_true, b = make_sample(cfg, geom, pseed)
        x = torch.zeros(geom.shape, dtype=torch.float32, device=geom.device)
        rows = []
        for k in range(n_stages):
            net = nets[k]
            physics(geom, x, b, iters_per_stage, subsets)
            before = net.mse(x, x_true)
            for _ in range(crop_steps):
                rate = lr + (lr_final - lr) * k_step / max(total - 1, 1)
                k_step += 1
                if crop:
                    z0, y0, x0 = (int(rng.integers(0, n - crop + 1)) for n in (nz, ny, nx))
                    sl = (slice(z0, z0 + crop), slice(y0, y0 + crop), slice(x0, x0 + crop))
                    net.train_step(x[sl].contiguous(), x_true[sl].contiguous(), lr=rate,
                                   mask=mask[sl].contiguous())
                else:
                    net.train_step(x, x_true, lr=rate, mask=mask)
            x = net.forward(x, mask=mask)
            rows.append((before, net.mse(x, x_true)))
        hist.append(rows)
        if log and (i % log_every == 0 or i + 1 == len(seeds)):
            log("phantom %4d/%d seed %d (%s) stage MSE sirt->corrected %s  lr %.2e  %.1f s" % (
                i + 1, len(seeds), pseed, "ellipsoids" if pseed % 2 == 0 else "foam",
                " ".join("%.2e->%.2e" % r for r in rows), rate, time.time() - t0))
    return np.asarray(hist)


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def compare(geom, net, cfg, seeds, sirt_iters=50, n_stages=4, iters_per_stage=1, log=None,
            fov=True, subsets=None):
    """Learned pipeline versus plain SIRT on held-out phantoms: PSNR, data
    residual ||A x - b|| and wall time of each; returns a summary dict.
    ``fov``: confine the corrections to the field of view (as in training).
    ``subsets``: the pipeline's physics steps are OS-SIRT epochs; the
    same-budget baseline (``psnr_sirt_same_budget``) is always the pipeline's
    own physics steps without corrections, so it isolates the networks."""
    mask = fov_mask(geom.shape, geom.device)
    subsets = _subsets(geom, subsets)
    pipe = LearnedSirt(geom, net, n_stages, iters_per_stage, mask="fov" if fov else None,
                       subsets=subsets)
    budget = n_stages * iters_per_stage
    rows = []
    for seed in seeds:
        x_true, b = make_sample(cfg, geom, seed)
        z = lambda: torch.zeros(geom.shape, dtype=torch.float32, device=geom.device)
        # warm caches (SIRT weights, view lists, network buffers) outside the timings
        if not rows:
            geom.sirt(z(), b, 1, norms=False)
            physics(geom, z(), b, 1, subsets)
            pipe(b)
        xs = z()
        _, t_sirt = _timed(lambda: geom.sirt(xs, b, sirt_iters, norms=False))
        xb = z()
        _, t_budget = _timed(lambda: physics(geom, xb, b, budget, subsets))
        (xl, st), t_learned = _timed(lambda: pipe(b))
        row = dict(seed=int(seed),
                   psnr_sirt=psnr(xs, x_true, mask), psnr_sirt_same_budget=psnr(xb, x_true, mask),
                   psnr_learned=psnr(xl, x_true, mask),
                   resid_sirt=geom.residual_norm(xs, b), resid_learned=geom.residual_norm(xl, b),
                   resid_true=geom.residual_norm(x_true, b),
                   t_sirt=t_sirt, t_learned=t_learned, t_same_budget=t_budget,
                   accepted=sum(1 for s in st if s.get("corrected")))
        rows.append(row)
        if log:
            log("seed %d: PSNR SIRT-%d %.2f dB (SIRT-%d %.2f), learned %.2f dB; "
                "|Ax-b| %.4g vs %.4g; %.3f s vs %.3f s; %d/%d corrections kept" % (
                    seed, sirt_iters, row["psnr_sirt"], budget, row["psnr_sirt_same_budget"],
                    row["psnr_learned"], row["resid_sirt"], row["resid_learned"], t_sirt,
                    t_learned, row["accepted"], n_stages))
    keys = [k for k in rows[0] if k != "seed"]
    mean = {k: float(np.mean([r[k] for r in rows])) for k in keys}
    reached = all(r["psnr_learned"] >= r["psnr_sirt"] for r in rows)
    return dict(rows=rows, mean=mean, sirt_iters=sirt_iters, n_stages=n_stages,
                physics="SIRT" if subsets is None else "OS-SIRT, %d subsets" % len(subsets),
                learned_reaches_sirt_psnr=bool(reached),
                time_ratio=mean["t_learned"] / mean["t_sirt"])
