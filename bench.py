#!/usr/bin/env python3
"""Throughput of the right-hand side + explicit RK stage on one MI355X.

One step = one hrx_rk_stage call on the whole grid: pointwise thermochemistry (Newton
energy inversion, mixture transport, finite-rate chemistry), artificial diffusivity,
first derivatives and fluxes, divergence + sources + sponge + RK update, wall row.
Default workload: the 3-D jet-in-crossflow-shaped box of 5-species air,
512 x 256 x 128 points, FP64, artificial diffusivity on (the largest workload of the
metric that fits one GPU); the mixed FP32/FP64 form and the learned-surrogate form are
timed on the same field.  Inputs are seeded synthetic fields resident in HBM before
timing starts.

Prints one JSON line: the metric, the dominant kernel's position against the HBM
roofline (algorithmic bytes per launch over its HIP-event duration inside the timed
region), every kernel's figures, the failure counters, and the CPU oracle timed on a
bounded sample of the same workload at one core and at all cores (before the GPU is
touched).
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import re
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point RHS+RK-stage evals/s (Mpts/s), FP64 vs mixed/surrogate, % HBM peak"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
RK_NAMES = {0: "2N-RK3 (Williamson)", 1: "2N-RK4(3)5 (Carpenter-Kennedy)",
            2: "three-register TVD RK3 (Shu-Osher)"}

# HBM traffic per launch from rocprofv3 --pmc (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB per
# dispatch; the factors come from a plain 256 MiB copy), keyed by workload and kernel,
# valid only for the kernel source whose SHA-256 prefix is given (profiles/ holds the
# summaries and the commands).  Any other source reports traffic null.
TRAFFIC = {
    ('jisc_air5_m8_512x256x128', 16777216, 'explicit', 'flux'): 10418798643,
    ('jisc_air5_m8_512x256x128', 16777216, 'explicit', 'div'): 10832650961,
    ('jisc_air5_m8_512x256x128', 16777216, 'explicit', 'prim'): 5226785684,
    ('jisc_air5_m8_512x256x128', 16777216, 'explicit', 'ad_d4'): 2488781520,
    ('jisc_air5_m8_512x256x128', 16777216, 'explicit', 'ad_src'): 1004862212,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'flux'): 11273500530,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'prim'): 5226632943,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'fin'): 6866683414,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'ad_d4'): 2464529902,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'ad_filter_z'): 2281594325,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'ad_src'): 1476263483,
    ('jisc_air5_m8_512x256x128', 16777216, 'compact', 'cderiv'): 2818649685,
    ('sbli_air5_m5.92_2048x512', 1048576, 'explicit', 'div'): 510500769,
    ('sbli_air5_m5.92_2048x512', 1048576, 'explicit', 'prim'): 260053849,
    ('sbli_air5_m5.92_2048x512', 1048576, 'explicit', 'flux'): 413994935,
    ('sbli_air5_m5.92_2048x512', 1048576, 'explicit', 'ad_d4'): 171196927,
    ('sbli_air5_m5.92_2048x512', 1048576, 'explicit', 'ad_src'): 35601651,
    ('flatplate_air5_m10_512x256', 131072, 'explicit', 'prim'): 25479495,
    ('flatplate_air5_m10_512x256', 131072, 'explicit', 'div'): 61078061,
    ('flatplate_air5_m10_512x256', 131072, 'explicit', 'flux'): 37727903,
    ('flatplate_air5_sm_m10_512x256', 131072, 'explicit', 'prim'): 35965369,
    ('flatplate_air5_sm_m10_512x256', 131072, 'explicit', 'flux'): 43011044,
    ('flatplate_air5_sm_m10_512x256', 131072, 'explicit', 'div'): 61037132,
    ('flatplate_tpg_m6_512x256', 131072, 'explicit', 'div'): 27156759,
    ('flatplate_tpg_m6_512x256', 131072, 'explicit', 'prim'): 11534425,
    ('flatplate_tpg_m6_512x256', 131072, 'explicit', 'flux'): 19698747,
}
TRAFFIC_SOURCE_SHA = "9f613edb3f76c77a"


def source_sha():
    p = os.path.join(ROOT, "paper_2210_05547_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(p)):
        with open(os.path.join(p, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sponge_fraction(cfg):
    import numpy as np
    m = np.zeros((cfg.ny, cfg.nx), bool)
    if cfg.sponge_in:
        m[:, :cfg.sponge_in] = True
    if cfg.sponge_out:
        m[:, cfg.nx - cfg.sponge_out:] = True
    if cfg.sponge_top:
        m[cfg.ny - cfg.sponge_top:, :] = True
    return float(m.mean())


def algorithmic_bytes(cfg, rt, surrogate=False):
    """Algorithmic HBM bytes per grid point of each kernel of one stage (every plane a
    kernel needs read once, every plane it produces written once; stencil neighbours
    count once), as {kernel: (bytes per point, launches per stage)}.  rt: bytes of the
    transport/AD planes (8 FP64, 4 mixed)."""
    air, ad = cfg.gas == 1, cfg.ad
    sm = air and cfg.diffusion == 1
    nd = cfg.ndim
    ns = 5 if air else 1
    nv = ns + nd + 1
    comp = getattr(cfg, "fd_scheme", 0) == 1
    xp = air and (nd == 3 or comp)                 # X_s and p stored as planes
    wd_out = nd + 1 + (5 + 1 if xp else (0 if air else 1))
    if air:
        # mu, kappa, D_s, wdot_s (+ 1/D_sr, + c); the flux forms h_s from T itself
        wp = 12 + (10 if sm else 0) + (1 if ad else 0)
        flux_wp = 2 + (0 if sm else 5) + (10 if sm else 0) + (1 if ad else 0)
    else:
        wp = (1 if cfg.gas == 0 else 2) + (1 if ad else 0)
        flux_wp = wp
    nad = 3 + (5 if air else 0)
    warm = 8 if cfg.gas in (1, 2) else 0
    prim = 8 * nv + warm + 8 * wd_out + rt * wp + (rt * (1 + (5 if air else 0)) if ad else 0)
    if surrogate:
        prim += 8 * nv + 2 * 32                    # network pass: Q in, 8 floats out and back
    out = {"prim": (prim, 1)}
    if ad:
        out["ad_src"] = ((2 * rt + (0 if comp else 8 * nd)) + (8 * nd * nd if comp else 0), 1)
        out["ad_d4"] = (2 * nad * rt, 1)
        if nd == 3 and comp:
            # (the explicit 3-D flux applies the z filter to the planes it reads)
            out["ad_filter_z"] = (2 * nad * rt, 1)
    nsrc = nd + 1 + (5 if air else 0)
    flux_in = 8 * (nd + 1 + (5 if (air and nd == 3) else 0) + (1 if (not air or nd == 3) else 0))
    if comp:
        # u, T, p at the point (X_s too for Stefan-Maxwell) and the gradient planes
        flux_in = 8 * (nd + 1 + 1 + (5 if sm else 0)) + 8 * nd * nsrc
    flux_in += 8 * nv + rt * flux_wp + (rt * nad if ad else 0)
    out["flux"] = (flux_in + 8 * nd * nv, 1)
    sponge = 8 * nv * sponge_fraction(cfg)
    if comp:
        # gradients: nsrc planes read and written per direction; divergence: F read, R
        # written (x) or read and written (y, z)
        grad = nd * nsrc * 16
        div = nv * (16 + (nd - 1) * 24)
        out["cderiv"] = ((grad + div) / (2 * nd), 2 * nd)
        out["fin"] = (8 * nv + (rt * 5 if air else 0) + 32 * nv + sponge, 1)
    else:
        out["div"] = (8 * nd * nv + (rt * 5 if air else 0) + 32 * nv + sponge, 1)
    return out


def compulsory_bytes(cfg):
    """Read Q and dQ, write Q and dQ (plus Q_ref in the sponges): 32 nvar B per point."""
    return 32 * cfg.nvar + 8 * cfg.nvar * sponge_fraction(cfg)


# ------------------------------------------------------------------ CPU oracle baseline
def _oracle_block(job):
    """One worker of the all-cores baseline: oracle stages on an x block (with halo) of
    the sample field for about `seconds`; returns (interior points x stages, seconds)."""
    import numpy as np
    from oracle import rhs as orhs
    cfg, Q, Qr, x, y, z, dt, interior, seconds = job
    case = orhs.Case(cfg, x, y, z, None)
    Qo, dQo = Q.copy(), np.zeros_like(Q)
    t0 = time.perf_counter()
    n = 0
    while True:
        orhs.rk_stage(Qo, dQo, Qr, case, n, dt)
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    return interior * n, time.perf_counter() - t0


def cpu_baseline(cfg, seconds, cores):
    """The oracle's RK stage on a bounded sample of the workload: the full grid in 2-D,
    an 8-plane periodic-z slab in 3-D; one process for the one-core figure, then the
    sample split along x into `cores` blocks with a halo of 12 points (the dependency
    reach of the AD chain), one process each; rates count interior points only."""
    import multiprocessing as mp
    import numpy as np
    from paper_2210_05547_amd import fields
    sc = dataclasses.replace(cfg, nz=8) if cfg.ndim == 3 else cfg
    Q, Qr, info = fields.initial_field(sc)
    x, y, z = info["x"], info["y"], info["z"]
    one = _oracle_block((sc, Q, Qr, x, y, z, info["dt"], sc.npts, seconds))
    single = one[0] / one[1] / 1e6
    H = 12
    edges = np.linspace(0, sc.nx, cores + 1).astype(int)
    jobs = []
    for b in range(cores):
        i0, i1 = edges[b], edges[b + 1]
        a, e = max(0, i0 - H), min(sc.nx, i1 + H)
        cb = dataclasses.replace(sc, nx=e - a, sponge_in=0, sponge_out=0, sponge_top=0)
        jobs.append((cb, np.ascontiguousarray(Q[..., a:e]), np.ascontiguousarray(Qr[..., a:e]),
                     x[a:e], y, z, info["dt"], (i1 - i0) * sc.ny * sc.nz, seconds))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_block, jobs)
    wall = time.perf_counter() - t0
    allc = sum(r[0] for r in res) / wall / 1e6
    what = (f"{sc.nx}x{sc.ny}x{sc.nz} periodic-z slab of the workload" if cfg.ndim == 3
            else f"the full {sc.nx}x{sc.ny} grid")
    return dict(value=round(allc, 4), unit="Mpts/s", cores=cores, kind="oracle",
                sample=f"oracle RK stages (numpy FP64) on {what}, about {seconds:.0f} s per "
                       f"run; all cores: {cores} processes on x blocks with a 12-point halo, "
                       f"interior points counted, wall {wall:.1f} s incl. start-up",
                single_core=dict(value=round(single, 4), cores=1,
                                 sample=f"{int(round(one[0] / sc.npts))} stages in {one[1]:.1f} s"))


# ------------------------------------------------------------------ GPU timing
def time_form(cfg, Q, Qr, info, steps, warmup, precision, setup=None):
    """Mpts/s of the stage loop in another form (graph replay on); setup(ctx) may prepare
    the context first (the surrogate form trains its network there)."""
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
    c = ctx.counters()
    time_form.counters = c
    time_form.finite = bool(torch.isfinite(Qd).all())
    ctx.close()
    del Qd, Qrd, dQd
    return cfg.npts * steps / (a.elapsed_time(b) * 1e-3) / 1e6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--grid", type=int, nargs="+", default=None, metavar="N",
                    help="run the configuration's workload on another grid (nx ny [nz])")
    ap.add_argument("--stefan-maxwell", action="store_true",
                    help="Stefan-Maxwell diffusion (Eq. 17) instead of Eq. (18)")
    ap.add_argument("--scheme", choices=("explicit", "compact"), default="explicit")
    ap.add_argument("--rk", type=int, default=None, help="0 2N-RK3, 1 2N-RK4(3)5, 2 TVD RK3")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="processes of the all-cores baseline (0: min(16, available))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip timing the mixed FP32/FP64 form on the same workload")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip training the surrogate and timing its form")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 10 times (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (sharding "
              "the grid over several GPUs is not built)",
              file=sys.stderr)
        sys.exit(2)
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

    from paper_2210_05547_amd import fields
    cfg = fields.get_config(args.config)
    if args.grid:
        cfg = cfg.scaled(*args.grid)
        dims = [cfg.nx, cfg.ny] + ([cfg.nz] if cfg.ndim == 3 else [])
        cfg = dataclasses.replace(cfg, name=re.sub(r"_\d+x\d+(x\d+)?$", "_" + "x".join(map(str, dims)),
                                                    cfg.name))
    if args.stefan_maxwell:
        cfg = dataclasses.replace(cfg, diffusion=1, name=cfg.name.replace("air5_", "air5_sm_", 1))
    if args.scheme == "compact":
        cfg = dataclasses.replace(cfg, fd_scheme=1)
    if args.rk is not None:
        cfg = dataclasses.replace(cfg, rk=args.rk)

    # the CPU baseline runs first, in processes forked before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        cores = args.cpu_cores or min(16, len(os.sched_getaffinity(0)))
        print(f"[bench] CPU oracle baseline ({cores} cores)...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, args.cpu_seconds, cores)

    import numpy as np  # noqa: F401
    import torch
    from paper_2210_05547_amd import hrx
    print(f"[bench] field {cfg.name} {cfg.nx}x{cfg.ny}x{cfg.nz}...", file=sys.stderr, flush=True)
    Q, Qr, info = fields.initial_field(cfg)
    dev = torch.device("cuda:0")
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"])
    Qd = torch.from_numpy(Q).to(dev)
    Qrd = torch.from_numpy(Qr).to(dev)
    dQd = torch.zeros_like(Qd)
    # a non-null stream lets the library replay each stage as a captured HIP graph
    stream = torch.cuda.Stream()
    stage = 0
    print("[bench] FP64 stages...", file=sys.stderr, flush=True)
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
        # per-kernel HIP-event durations on this stream: the same stages again with direct
        # launches, each kernel bracketed by events (graph replay is off while timing)
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
    ctx.close()
    del Qd, Qrd, dQd

    sha = source_sha()
    model = algorithmic_bytes(cfg, 8)
    kernels = {}
    for name, (tms, nl) in kt.items():
        if not nl:
            continue
        avg = 1e3 * tms / nl
        kd = dict(avg_us=round(avg, 3), launches=nl, share=0.0)
        if name in model:
            bpp, per_stage = model[name]
            gbs = bpp * cfg.npts / (avg * 1e-6) / 1e9
            kd.update(bytes_per_point=round(bpp, 1), GBps=round(gbs, 1),
                      hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
        kernels[name] = kd
    tot = sum(k["avg_us"] * k["launches"] for k in kernels.values())
    for k in kernels.values():
        k["share"] = round(k["avg_us"] * k["launches"] / tot, 4)
    dom = max((k for k in kernels if k in model), key=lambda k: kernels[k]["share"])
    kd = kernels[dom]
    tr = TRAFFIC.get((cfg.name, cfg.npts, args.scheme, dom)) if sha == TRAFFIC_SOURCE_SHA else None
    roof = dict(kernel=dom, bound="hbm", achieved=kd["GBps"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=kd["hbm_frac"], traffic=tr,
                traffic_note=("HBM bytes per launch, rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE "
                              "(profiles/stage_*.md of this workload)") if tr else
                ("no counter run of this kernel source and workload" if sha != TRAFFIC_SOURCE_SHA
                 else "no counter run of this workload"),
                algorithmic_bytes_per_launch=int(round(model[dom][0] * cfg.npts)),
                avg_launch_us=kd["avg_us"])
    eff = compulsory_bytes(cfg) * value * 1e6 / 1e9
    fails = {k: cnt[k] for k in ("newton_nonconverged", "energy_below_min", "nonfinite")}
    out = {
        "metric": METRIC,
        "value": round(value, 2), "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded field of the workload's shape; inputs resident in HBM)",
        "config": {"workload": cfg.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "points": cfg.npts,
                   "gas": {0: "cpg", 1: "air5", 2: "tpg"}[cfg.gas], "rk": RK_NAMES[cfg.rk],
                   "fd_order": cfg.fd_order, "fd_scheme": args.scheme,
                   "artificial_diffusivity": bool(cfg.ad),
                   "diffusion": "stefan-maxwell" if cfg.diffusion else "ramshaw"},
        "roofline": roof,
        "effective_hbm": dict(compulsory_bytes_per_point=round(compulsory_bytes(cfg), 1),
                              GBps=round(eff, 1), frac=round(eff / HBM_PEAK_GBS, 4)),
        "kernels": kernels,
        "kernel_source_sha": sha,
        "state_finite": finite,
        "failures": fails,
        "valid": finite and cnt["status"] == hrx.HRX_OK,
    }
    if not out["valid"]:
        print(f"[bench] WARNING: the timed state is not clean: finite={finite} {fails}",
              file=sys.stderr, flush=True)
    forms = {"fp64": out["value"]}
    if not args.no_mixed:
        print("[bench] mixed form...", file=sys.stderr, flush=True)
        forms["mixed"] = round(time_form(cfg, Q, Qr, info, args.steps, args.warmup,
                                         hrx.PREC_MIXED), 2)
    if not args.no_surrogate and cfg.gas == 1 and not cfg.diffusion:
        from paper_2210_05547_amd import surrogate
        print("[bench] surrogate form (training first)...", file=sys.stderr, flush=True)
        summary = {}

        def setup(c):
            t0 = time.perf_counter()
            summary.update(surrogate.train(c))
            torch.cuda.synchronize()
            summary["train_seconds"] = round(time.perf_counter() - t0, 1)
            hrx.set_thermo_mode(c, hrx.THERMO_SURROGATE)
        forms["surrogate"] = round(time_form(cfg, Q, Qr, info, args.steps, args.warmup,
                                             hrx.PREC_FP64, setup), 2)
        summary["fallback_fraction"] = round(
            time_form.counters["surrogate_fallbacks"] / (cfg.npts * (args.steps + args.warmup)), 5)
        summary["design"] = surrogate.DESIGN_NOTE
        out["surrogate"] = summary
    out["forms"] = forms
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
