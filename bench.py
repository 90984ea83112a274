#!/usr/bin/env python3
"""Throughput of the right-hand side + low-storage RK stage on one MI355X.

One step = one hrx_rk_stage call: primitive/thermochemistry pass (Newton energy
inversion, mixture transport, finite-rate chemistry), flux pass (stencil gradients,
convective + viscous + diffusive fluxes), divergence + source + sponge + RK update,
wall-row update.  Inputs are the seeded synthetic 5-species-air flat-plate field
(512 x 256, M = 10, FP64), resident in HBM before timing starts.

Prints one JSON line with the metric, the dominant kernel's roofline position
(per-kernel HIP-event durations inside the timed region) and the CPU oracle timed
on a bounded sample of the same workload.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the flat-plate stage kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE scaled by a 256 MiB copy kernel (fetch x2.0, write x1.0), for the kernels
# as they stand (profiles/stage_air5_flatplate_512x256.md)
PRIM_TRAFFIC_BYTES = (9460 + 20480) * 1024
TRAFFIC_BYTES = {"flux": (25566 + 16384) * 1024, "div": (43205 + 16392) * 1024}
FP64_VECTOR_PEAK_TFLOPS = 78.6

# Algorithmic HBM bytes per grid point of each kernel (FP64 planes read once + written
# once; stencil neighbours counted once), for a 2-D 5-species-air stage without AD:
#   prim : read Q (8 planes) + T of the previous stage; write Wd (u, v, T: 3) and
#          Wp (mu, kappa, D_1..5, wdot_1..5, h_1..5: 17)
#   flux : read Wd (3) + Wp (mu, kappa, D_s, h_s: 12) + Q (8: the partial densities give
#          the tile's mole fractions and the pressure); write F (2 x 8)
#   div  : read F (16) + wdot (5) + Q (8) + dQ (8); write Q, dQ (16)  (+ Q_ref in sponges)
BYTES_PER_POINT_AIR5_2D = {"prim": 8 * (9 + 20), "flux": 8 * (23 + 16),
                           "div": 8 * (37 + 16)}
# FP64 floating-point operations per grid point of the pointwise thermochemistry
# (energy inversion from the previous stage's temperature, transport, kinetics,
# enthalpies): SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes / points, read with rocprofv3 on
# this workload (profiles/stage_air5_flatplate_512x256.md).  MI355X has no FP64
# transcendental unit, so this includes the instruction sequences of exp/log/sqrt/div.
FLOPS_PER_POINT_PRIM_AIR5_2D = 2766.0


def sponge_fraction(cfg):
    import numpy as np
    from paper_2210_05547_amd import fields
    nx, ny = cfg.nx, cfg.ny
    m = np.zeros((ny, nx), bool)
    if cfg.sponge_in:
        m[:, :cfg.sponge_in] = True
    if cfg.sponge_out:
        m[:, nx - cfg.sponge_out:] = True
    if cfg.sponge_top:
        m[ny - cfg.sponge_top:, :] = True
    return float(m.mean())


def cpu_baseline(cfg, Q, Qr, info, budget_s):
    """Oracle stages on the same field until about budget_s seconds of CPU work."""
    import numpy as np
    from oracle import rhs as orhs
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], info["hold"])
    Qo, dQo = Q.copy(), np.zeros_like(Q)
    t0 = time.perf_counter()
    n = 0
    while True:
        orhs.rk_stage(Qo, dQo, Qr, case, n, info["dt"])
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=cfg.npts * n / dt / 1e6, unit="Mpts/s", cores=1, kind="oracle",
                sample=f"{n} RK stages of the same {cfg.nx}x{cfg.ny} field, numpy FP64, "
                       f"single thread, {dt:.1f} s")


def time_form(cfg, Q, Qr, info, steps, warmup, precision, setup=None):
    """Mpts/s of the same stage loop in another form (graph replay on); setup(ctx) may
    prepare the context first (the surrogate form trains its network there)."""
    import torch
    from paper_2210_05547_amd import hrx
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"], precision=precision)
    if setup is not None:
        setup(ctx)
    ctx.counters(reset=True)
    Qd = torch.from_numpy(Q).to("cuda:0")
    Qrd = torch.from_numpy(Qr).to("cuda:0")
    dQd = torch.zeros_like(Qd)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for k in range(warmup):
            hrx.rk_stage(ctx, k, info["dt"], Qd, dQd, Qrd)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(warmup, warmup + steps):
            hrx.rk_stage(ctx, k, info["dt"], Qd, dQd, Qrd)
        b.record()
        torch.cuda.synchronize()
    time_form.fallbacks = ctx.counters()["surrogate_fallbacks"]
    ctx.close()
    return cfg.npts * steps / (a.elapsed_time(b) * 1e-3) / 1e6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--grid", type=int, nargs="+", default=None, metavar="N",
                    help="run the configuration's workload on another grid (nx ny [nz])")
    ap.add_argument("--stefan-maxwell", action="store_true",
                    help="Stefan-Maxwell diffusion (Eq. 17) instead of Eq. (18)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip timing the mixed FP32/FP64 form on the same workload")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip training the surrogate and timing its form")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 10 times (counter scaling)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "reps": 10}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path's multi-GPU sharding is described in DESIGN.md, not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2210_05547_amd import fields, hrx

    cfg = fields.get_config(args.config)
    if args.grid:
        cfg = cfg.scaled(*args.grid)
    if args.stefan_maxwell:
        cfg = dataclasses.replace(cfg, diffusion=1)
    Q, Qr, info = fields.initial_field(cfg)
    dev = torch.device("cuda:0")
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"])
    Qd = torch.from_numpy(Q).to(dev)
    Qrd = torch.from_numpy(Qr).to(dev)
    dQd = torch.zeros_like(Qd)
    # a non-null stream lets the library replay each stage as a captured HIP graph
    stream = torch.cuda.Stream()
    stage = 0
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            hrx.rk_stage(ctx, stage, info["dt"], Qd, dQd, Qrd)
            stage += 1
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            hrx.rk_stage(ctx, stage, info["dt"], Qd, dQd, Qrd)
            stage += 1
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        # per-kernel HIP-event durations: the same stages again with direct launches
        # bracketed by events on this stream (graph replay is off while timing)
        hrx.timing_enable(ctx, True)
        for _ in range(args.steps):
            hrx.rk_stage(ctx, stage, info["dt"], Qd, dQd, Qrd)
            stage += 1
        torch.cuda.synchronize()
        kt = hrx.timing_read(ctx)
        hrx.timing_enable(ctx, False)
    cnt = ctx.counters()
    finite = bool(torch.isfinite(Qd).all())
    value = cfg.npts * args.steps / (ms * 1e-3) / 1e6

    kernels = {}
    for name, (tms, nl) in kt.items():
        if nl:
            kernels[name] = dict(avg_us=round(1e3 * tms / nl, 3), launches=nl)
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    model = cfg.gas == 1 and cfg.ndim == 2 and not cfg.ad
    # the counter-based traffic figures were taken on the flat plate's own grid
    counted = cfg.name == fields.get_config("c2").name and cfg.npts == 512 * 256
    roofs = {}
    if model:
        bpp = dict(BYTES_PER_POINT_AIR5_2D)
        bpp["div"] = bpp["div"] + 8 * 8 * sponge_fraction(cfg)
        for name, kd in kernels.items():
            if name not in bpp:
                continue
            sec = kd["avg_us"] * 1e-6
            gbs = bpp[name] * cfg.npts / sec / 1e9
            kd["GBps"] = round(gbs, 1)
            if name == "prim":
                tf = FLOPS_PER_POINT_PRIM_AIR5_2D * cfg.npts / sec / 1e12
                kd["TFLOPs_fp64"] = round(tf, 2)
                roofs[name] = dict(kernel=name, bound="alu", achieved=round(tf, 2),
                                   peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                                   frac=round(tf / FP64_VECTOR_PEAK_TFLOPS, 4),
                                   traffic=PRIM_TRAFFIC_BYTES if counted else None)
            else:
                roofs[name] = dict(kernel=name, bound="hbm", achieved=round(gbs, 1),
                                   peak=HBM_PEAK_GBS, unit="GB/s",
                                   frac=round(gbs / HBM_PEAK_GBS, 4),
                                   traffic=TRAFFIC_BYTES.get(name) if counted else None)
    roof = roofs.get(dom)
    out = {
        "metric": "grid-point RHS+RK-stage evals/s (Mpts/s), FP64",
        "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded flat-plate boundary-layer field)",
        "config": {"workload": cfg.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "points": cfg.npts,
                   "gas": {0: "cpg", 1: "air5", 2: "tpg"}[cfg.gas], "rk": "2N-RK3",
                   "fd_order": cfg.fd_order, "artificial_diffusivity": bool(cfg.ad),
                   "diffusion": "stefan-maxwell" if cfg.diffusion else "ramshaw"},
        "roofline": roof,
        "kernels": kernels,
        "kernel_rooflines": roofs,
        "state_finite": finite,
        "newton_failures": cnt["newton_nonconverged"] + cnt["energy_below_min"],
    }
    if not args.no_mixed:
        out["forms"] = {"fp64": out["value"],
                        "mixed": round(time_form(cfg, Q, Qr, info, args.steps, args.warmup,
                                                 hrx.PREC_MIXED), 2)}
    if not args.no_surrogate and cfg.gas == 1 and not cfg.diffusion:
        from paper_2210_05547_amd import surrogate
        summary = {}

        def setup(ctx):
            t0 = time.perf_counter()
            summary.update(surrogate.train(ctx))
            torch.cuda.synchronize()
            summary["train_seconds"] = round(time.perf_counter() - t0, 1)
            hrx.set_thermo_mode(ctx, hrx.THERMO_SURROGATE)
        rate = time_form(cfg, Q, Qr, info, args.steps, args.warmup, hrx.PREC_FP64, setup)
        out.setdefault("forms", {"fp64": out["value"]})["surrogate"] = round(rate, 2)
        summary["fallback_fraction"] = round(
            time_form.fallbacks / (cfg.npts * (args.steps + args.warmup)), 5)
        out["surrogate"] = summary
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, Q, Qr, info, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
