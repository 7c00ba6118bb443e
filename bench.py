"""Benchmark of the projector hot path on one MI355X.

Workload: 512^3 FP32 volume of 200 seeded random ellipsoids plus a uniform
cylinder; circular cone beam, 720 projections of a 768 x 768 detector
(pitch 1.5, SOD 1600, SDD 3200), ray-march step 0.5 voxel.  One step is one
SIRT iteration of Eq. (1) over all 720 projections: forward projection with
the fused correction R (b - A x), exact-transpose backprojection, update.
The SIRT weights R and C are built once per geometry (during warm-up).

Metric: FP+BP Gsamples/s = 2 N_s / (time per step) with N_s the exact
number of trilinear samples of one forward projection.  Kernel times come
from HIP events the library records on its launch stream inside the timed
steps.  The CPU baseline is the FP64 oracle on a bounded view subset.

The JSON line also carries, when the trained correction networks are
present, the time-to-PSNR comparison of the learned pipeline (4 stages of an
ordered-subset SIRT epoch + U-Net) against 50 plain SIRT iterations on one
held-out phantom of the learned-correction configuration (256^3, 180 x 384^2,
Poisson noise).

HBM traffic: ``roofline.traffic`` is read from the committed counter summary
(two rocprofv3 --pmc passes, FETCH_SIZE then WRITE_SIZE, scaled by the
same counters of a plain copy kernel of known size, ``--copy-calibrate``);
it is null when the dominant kernel's sources changed since.

The ``voxel_bp`` object repeats the SIRT run with the paper's voxel-driven
backprojector in place of the exact transpose (speed, and residual and PSNR
after the same number of iterations); the ``cylinder`` object runs SIRT on the
aligned cylindrical domain (a polar grid inscribed in the same box) with the
same scan.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f32|bf16]
                       [--copy-calibrate] [--no-learned] [--no-voxel-bp] [--no-cylinder]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP+BP Gsamples/s @512³×720 proj; time-to-PSNR learned vs plain SIRT"
HBM_PEAK_GBS = 8000.0
GATHER_BYTES = {"f32": 32, "bf16": 16}   # 8 voxel reads per sample
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_sirt_512cube_720x768sq.md")
WEIGHTS_FILE = os.path.join(ROOT, "paper_2609_30166_amd", "weights", "unet_learned_256.npz")
KERNEL_SOURCES = {
    "bp_brick_kernel": ["backproject.hip", "ray_common.h", "ctrex_internal.h"],
    "fp_kernel": ["projector.hip", "ray_common.h", "ctrex_internal.h"],
    "vbp_kernel": ["voxel_bp.hip", "ray_common.h", "ctrex_internal.h"],
}


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, x, n_views):
    """FP64 oracle on the first ``n_views`` projections: FP + BP samples/s."""
    import numpy as np

    import oracle

    views = list(range(0, cfg.n_proj, cfg.n_proj // n_views))[:n_views]
    xd = x.astype(np.float64)
    t0 = time.perf_counter()
    y, cnt = oracle.forward(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, xd, cfg.step, views=views,
                            return_count=True)
    t1 = time.perf_counter()
    oracle.back(cfg.P, cfg.shape, cfg.n_u, cfg.n_v, y, cfg.step, views=views)
    t2 = time.perf_counter()
    rate = 2.0 * cnt / (t2 - t0) / 1e9
    return {"value": rate, "unit": "Gsamples/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle FP+BP over %d of 720 views of the same 512^3 phantom "
                      "(%d samples each way; FP %.1f s, BP %.1f s)" % (n_views, cnt, t1 - t0,
                                                                        t2 - t1)}


def source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2609_30166_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, dtype):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None if absent or taken on other sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1)).get("%s/%s" % (kernel, dtype))
    if not rec or rec.get("source_hash") != source_hash(kernel):
        return None
    return rec["hbm_bytes_per_launch"]


def copy_calibration(dev):
    """A plain copy of 2^27 floats (512 MiB read + 512 MiB written) through the
    library's conversion kernel, for scaling the FETCH/WRITE counters."""
    import torch
    from paper_2609_30166_amd import _lib

    n = 1 << 27
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    import ctypes
    ctx = ctypes.c_void_p()
    L = _lib.lib()
    _lib.check(None, L.ctrex_create(ctypes.byref(ctx), dev.index))
    for _ in range(3):
        _lib.check(ctx, L.ctrex_convert(ctx, ctypes.c_void_p(src.data_ptr()), _lib.F32,
                                        ctypes.c_void_p(dst.data_ptr()), _lib.F32, n, None))
    torch.cuda.synchronize()
    L.ctrex_destroy(ctx)
    _log("copy calibration: 3 copies of %d bytes" % (4 * n))


def time_to_psnr(dev):
    """Learned 4-stage pipeline vs 50 plain SIRT iterations on one held-out
    phantom; None when the trained weights are not present."""
    if not os.path.exists(WEIGHTS_FILE):
        return None
    import numpy as np

    from paper_2609_30166_amd import learned
    from paper_2609_30166_amd.train_unet import load
    from synth import configs

    cfg, geom = learned.learned_geometry(device=dev)
    net = load(WEIGHTS_FILE, dev)
    seed = list(configs.TEST_SEEDS)[0]
    meta = json.loads(str(np.load(WEIGHTS_FILE, allow_pickle=False)["meta"]))
    stages, per = int(meta.get("stages", 4)), int(meta.get("iters_per_stage", 1))
    subsets = int(meta.get("subsets", 0)) or None
    res = learned.compare(geom, net, cfg, [seed], sirt_iters=50, n_stages=stages,
                          iters_per_stage=per, log=lambda s: _log("learned: " + s),
                          fov=bool(meta.get("fov_mask", False)), subsets=subsets)
    r = res["rows"][0]
    return {"sirt_iters": 50, "stages": stages, "iters_per_stage": per, "phantom_seed": seed,
            "physics_steps": res["physics"],
            "psnr_sirt_db": r["psnr_sirt"], "psnr_learned_db": r["psnr_learned"],
            "psnr_physics_alone_same_steps_db": r["psnr_sirt_same_budget"],
            "t_physics_alone_s": r["t_same_budget"],
            "resid_sirt": r["resid_sirt"], "resid_learned": r["resid_learned"],
            "t_sirt_s": r["t_sirt"], "t_learned_s": r["t_learned"],
            "time_ratio": r["t_learned"] / r["t_sirt"],
            "reaches_sirt_psnr": bool(r["psnr_learned"] >= r["psnr_sirt"]),
            "workload": "256^3, 180 projections of 384x384, Poisson I0=1e4, seeded held-out "
                        "phantom; inference only"}


def voxel_bp_comparison(g, b, sdt, xt, vol_exact, norms_exact, args, bp_ms_exact, ms_exact):
    """The same SIRT run (warm-up + timed steps + one more) with the paper's
    voxel-driven backprojector B and C = 1 / (B 1) in place of the exact
    transpose: per-step and per-kernel times, and the residual norm and PSNR
    reached after the same number of iterations as the exact-transpose run."""
    import numpy as np
    import torch

    from paper_2609_30166_amd.learned import fov_mask, psnr

    vol = torch.zeros_like(vol_exact)
    ws = g.workspace(gather_dtype=sdt)
    for _ in range(args.warmup):
        g.sirt(vol, b, 1, gather_dtype=sdt, workspace=ws, norms=False, voxel_bp=True)
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.sirt(vol, b, 1, gather_dtype=sdt, workspace=ws, norms=False, voxel_bp=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    norms = g.sirt(vol, b, 1, gather_dtype=sdt, workspace=ws, voxel_bp=True)
    mask = fov_mask(g.shape, g.device)
    bp_ms = prof["back"][0] / max(prof["back"][1], 1)
    n_vv = float(np.prod(g.shape)) * g.n_proj
    res = {
        "iterations": args.warmup + args.steps + 1,
        "ms_per_step": 1e3 * (t1 - t0) / args.steps,
        "fp_ms": prof["forward"][0] / max(prof["forward"][1], 1),
        "bp_ms": bp_ms,
        "update_ms": prof["update"][0] / max(prof["update"][1], 1),
        "bp_voxel_views_per_s": n_vv / (bp_ms * 1e-3),
        "bp_speedup_vs_exact": bp_ms_exact / bp_ms,
        "step_speedup_vs_exact": ms_exact / (1e3 * (t1 - t0) / args.steps),
        "residual_norm_after": float(norms[0]),
        "residual_norm_after_exact": float(norms_exact[0]),
        "psnr_db": psnr(vol, xt, mask),
        "psnr_db_exact": psnr(vol_exact, xt, mask),
    }
    del ws, vol
    return res


def cylinder_sirt(dev, cfg, args):
    """SIRT on the aligned cylindrical domain with the same scan (720 x 768^2):
    a polar grid of 256 rings x 1608 angles x 512 slices (dr = dz = 1; the
    cylinder inscribed in the 512^3 box, ~1 voxel arc spacing at the rim)
    holding a seeded vial phantom; forward projection clipped to the
    cylinder, voxel-driven backprojection over the polar voxels.  Reports
    per-step and per-kernel times, samples of one forward projection and the
    residual norms of the iterates."""
    import numpy as np
    import torch

    from paper_2609_30166_amd import CylinderGeometry
    from synth.phantoms import vial_polar

    n_r, n_phi, n_z = 256, 1608, 512
    g = CylinderGeometry(cfg.P, cfg.n_u, cfg.n_v, n_r, n_phi, n_z, 1.0, 1.0, cfg.step,
                         device=dev)
    x = torch.from_numpy(vial_polar(n_r, n_phi, n_z, 1.0, 1.0, np.random.default_rng(17))).to(dev)
    b = g.forward(x)
    n_s = g.sample_count()
    vol = torch.zeros_like(x)
    ws = g.workspace()
    for _ in range(args.warmup):
        g.sirt(vol, b, 1, workspace=ws, norms=False)
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.sirt(vol, b, 1, workspace=ws, norms=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    norms = g.sirt(vol, b, 1, workspace=ws)
    fp_ms = prof["forward"][0] / max(prof["forward"][1], 1)
    bp_ms = prof["back"][0] / max(prof["back"][1], 1)
    res = {
        "workload": "SIRT iteration on a 256 x 1608 x 512 polar grid (dr = dz = 1), 720 "
                    "circular cone-beam projections of 768x768, step 0.5",
        "iterations": args.warmup + args.steps + 1,
        "ms_per_step": 1e3 * (t1 - t0) / args.steps,
        "fp_ms": fp_ms,
        "bp_ms": bp_ms,
        "update_ms": prof["update"][0] / max(prof["update"][1], 1),
        "samples_per_fp": n_s,
        "fp_gsamples_per_s": n_s / (fp_ms * 1e-3) / 1e9,
        "bp_voxel_views_per_s": float(n_r * n_phi * n_z) * g.n_proj / (bp_ms * 1e-3),
        "residual_norm_data": float(torch.linalg.vector_norm(b.double())),
        "residual_norm_after": float(norms[0]),
    }
    del x, b, vol, ws
    g.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--cpu-views", type=int, default=2,
                    help="views of the CPU-oracle baseline sample (0 = skip)")
    ap.add_argument("--n-proj", type=int, default=720, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="also run a plain copy kernel of known size (counter calibration)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-SIRT time-to-PSNR comparison")
    ap.add_argument("--no-voxel-bp", action="store_true",
                    help="skip the SIRT run with the voxel-driven backprojector")
    ap.add_argument("--no-cylinder", action="store_true",
                    help="skip the SIRT run on the aligned cylindrical domain")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2609_30166_amd import Geometry
    from synth.configs import make_config, make_phantom

    dev = torch.device("cuda", 0)
    cfg = make_config("full", n_proj=args.n_proj)
    _log("phantom 512^3 ...")
    x, _ = make_phantom(cfg, seed=0)
    g = Geometry(cfg.P, cfg.n_u, cfg.n_v, cfg.shape, cfg.step, device=dev)
    n_s = g.sample_count()
    _log("samples per forward projection: %d" % n_s)
    xt = torch.from_numpy(x).to(dev)
    sdt = torch.float32 if args.dtype == "f32" else torch.bfloat16
    b = g.forward(xt if sdt == torch.float32 else xt.to(sdt), out_dtype=sdt)
    vol = torch.zeros(cfg.shape, dtype=torch.float32, device=dev)
    ws = g.workspace(gather_dtype=sdt)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        g.sirt(vol, b, 1, gather_dtype=sdt, workspace=ws, norms=False)
        torch.cuda.synchronize()
        _log("warmup %d done" % i)

    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        g.sirt(vol, b, 1, gather_dtype=sdt, workspace=ws, norms=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    _log("timed %d steps in %.3f s" % (args.steps, t1 - t0))
    norms = g.sirt(vol, b, 1, gather_dtype=sdt, workspace=ws)

    ms_step = 1e3 * (t1 - t0) / args.steps
    value = 2.0 * n_s * args.steps / (t1 - t0) / 1e9
    fp_ms = prof["forward"][0] / max(prof["forward"][1], 1)
    bp_ms = prof["back"][0] / max(prof["back"][1], 1)
    up_ms = prof["update"][0] / max(prof["update"][1], 1)
    dom, dom_ms = ("bp_brick_kernel", bp_ms) if bp_ms >= fp_ms else ("fp_kernel", fp_ms)
    achieved = GATHER_BYTES[args.dtype] * n_s / (dom_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded 512^3 ellipsoid+cylinder phantom, noise-free)",
        "config": {
            "workload": "SIRT iteration, 512^3 volume, 720 circular cone-beam projections of "
                        "768x768, step 0.5 voxel (FP with fused correction + exact-transpose BP "
                        "+ update)",
            "samples_per_fp": n_s,
            "fp_ms": fp_ms, "bp_ms": bp_ms, "update_ms": up_ms,
            "residual_norm_after": float(norms[0]),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom, args.dtype),
            "basis": "gather-equivalent bytes: %d B per sample (8 voxel reads) x %d samples "
                     "per launch / mean launch time" % (GATHER_BYTES[args.dtype], n_s),
        },
    }
    if not args.no_voxel_bp:
        _log("SIRT with the voxel-driven backprojector ...")
        out["voxel_bp"] = voxel_bp_comparison(g, b, sdt, xt, vol, norms, args, bp_ms, ms_step)
    if args.copy_calibrate:
        copy_calibration(dev)
    del b, vol, ws, xt
    g.close()
    torch.cuda.empty_cache()
    if not args.no_cylinder:
        _log("SIRT on the aligned cylindrical domain ...")
        out["cylinder"] = cylinder_sirt(dev, cfg, args)
        torch.cuda.empty_cache()
    if not args.no_learned:
        _log("learned pipeline vs SIRT-50 ...")
        out["time_to_psnr"] = time_to_psnr(dev)
    if args.cpu_views > 0:
        _log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(cfg, x, args.cpu_views)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
