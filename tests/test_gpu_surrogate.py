"""Learned thermochemistry surrogate: training on the GPU with the library's own
kernels, accuracy against the plain evaluation, hull fallback, the right-hand side
with the surrogate, and what the network gains over the plain evaluation.

Data: 10^6 oracle states (T ~ U(200, 8000) K, rho ~ 10^U(-4, 0) kg/m^3, air
compositions at every dissociation degree; recipe in surrogate_util); 90 % train,
10 % held out.  Bars: the FP64 energy inversion keeps T at 1e-12; the RHS with
surrogate transport within 1e-3 normwise per field of the plain FP64 RHS (the
surrogate's parity bar); held-out transport per point: RMS relative error <= 1e-3,
99.9th percentile <= 5e-3, max <= 1e-2; out-of-hull points reproduce the plain
evaluation to 1e-12.
"""
import math
import os
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_05547_amd import fields, hrx  # noqa: E402
from oracle import mlp as omlp  # noqa: E402
from oracle import rhs as orhs  # noqa: E402
from oracle import thermo as oth  # noqa: E402
from oracle import transport as otr  # noqa: E402
from gpu_util import field_errors, normwise, tie_free_rows, write_report  # noqa: E402
from surrogate_util import (LOGRHO_RANGE, T_RANGE, XI_N_RANGE, element_N_fraction,  # noqa: E402
                            features, fit_norm, network_targets, raw_dataset, set_norm, states)

DEV = "cuda:0"
NTOT = 1_000_000
BATCH = 4096
EPOCHS = int(os.environ.get("HRX_SURROGATE_EPOCHS", "200"))
REPORT = {}


def report(k, v):
    REPORT[k] = v
    print(" ", k, v, flush=True)
    write_report("surrogate_report.json", REPORT)


def air_ctx(cfg=None, hold=None):
    cfg = cfg or fields.get_config("c2").scaled(16, 16)
    x, y, z = fields.grid(cfg)
    return hrx.Context(cfg, x, y, z, hold)


@pytest.fixture(scope="module")
def trained():
    t0 = time.time()
    X, Yt, raw = raw_dataset(NTOT, seed=20221011 + 5)
    ntr = int(0.9 * NTOT)
    nm = fit_norm(X[:ntr], Yt[:ntr])
    Xs = ((X - nm["xm"]) / nm["xs"]).astype(np.float32)
    Ys = network_targets(X, Yt, nm).astype(np.float32)
    report("oracle_dataset_seconds", round(time.time() - t0, 1))
    ctx = air_ctx()
    hrx.mlp_init(ctx, BATCH)
    theta0 = omlp.init_params(11).astype(np.float32)
    hrx.mlp_set_params(ctx, torch.from_numpy(theta0).to(DEV))
    Xd = torch.from_numpy(Xs).to(DEV)
    Yd = torch.from_numpy(Ys).to(DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    rng = np.random.default_rng(0)
    steps_per_epoch = ntr // BATCH
    total = EPOCHS * steps_per_epoch
    lr0, t = 2e-3, 0
    hist = []
    torch.cuda.synchronize()
    t1 = time.time()
    for ep in range(EPOCHS):
        perm = torch.from_numpy(rng.permutation(ntr).astype(np.int32)).to(DEV)
        loss.zero_()
        for b in range(steps_per_epoch):
            t += 1
            lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * t / total)) + 1e-6
            hrx.mlp_train_step(ctx, BATCH, perm[b * BATCH:(b + 1) * BATCH], Xd, Yd, lr, t, loss)
        hist.append(float(loss.item()) / steps_per_epoch)
    torch.cuda.synchronize()
    report("train_seconds_gpu", round(time.time() - t1, 2))
    report("train_loss_first_last", [hist[0], hist[-1]])
    set_norm(hrx, ctx, nm)
    theta = torch.empty(hrx.MLP_NPARAM, dtype=torch.float32, device=DEV)
    hrx.mlp_get_params(ctx, theta)
    held = slice(ntr, NTOT)
    return dict(ctx=ctx, theta=theta, norm=nm, hist=hist, Xs=Xs, Ys=Ys, raw=raw,
                held=held, ntr=ntr)


def with_surrogate(ctx, tr):
    hrx.mlp_init(ctx, 16)
    hrx.mlp_set_params(ctx, tr["theta"])
    set_norm(hrx, ctx, tr["norm"])
    hrx.set_thermo_mode(ctx, hrx.THERMO_SURROGATE)
    return ctx


def test_features_match_oracle_side():
    """The library's raw features (log10 rho, ln T_c, Y) equal the ones the training set
    is built with here, to FP32 precision."""
    n = 5000
    rho, T, Y = states(n, seed=77)
    e = oth.mixture_e(T, Y)
    ctx = air_ctx()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    f = torch.empty((n, 7), dtype=torch.float32, device=DEV)
    hrx.mlp_features(ctx, n, d(rho), d(e), d(Y), f)
    ref = features(rho, e, Y)
    assert np.max(np.abs(f.cpu().numpy() - ref)) <= 2e-5


def test_dataset_and_fit_on_device():
    """hrx_mlp_dataset's targets equal the oracle's (1e-12: the plain FP64 evaluation;
    the features to rounding), and hrx_mlp_fit's statistics and standardised rows equal
    a NumPy fit of the same rows (statistics 1e-10; rows to FP32 rounding)."""
    n = 20000
    X_o, Y_o, raw = raw_dataset(n, seed=31)
    ctx = air_ctx()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    F = torch.empty((n, 7), dtype=torch.float64, device=DEV)
    Tt = torch.empty((n, 8), dtype=torch.float64, device=DEV)
    st = torch.empty(n, dtype=torch.int32, device=DEV)
    hrx.mlp_dataset(ctx, n, d(raw["rho"]), d(raw["e"]), d(raw["Y"]), F, Tt, status=st)
    Fh, Th = F.cpu().numpy(), Tt.cpu().numpy()
    assert int((st != 0).sum()) == 0
    for o in range(8):
        assert normwise(Th[:, o], Y_o[:, o]) <= 1e-12, o
    assert np.max(np.abs(Fh - X_o)) <= 1e-13 * np.max(np.abs(X_o))
    hrx.mlp_init(ctx, 16)
    Xs = torch.empty((n, 7), dtype=torch.float32, device=DEV)
    Ys = torch.empty((n, 8), dtype=torch.float32, device=DEV)
    stg = hrx.mlp_fit(ctx, n, F, Tt, Xs, Ys, LOGRHO_RANGE, T_RANGE, XI_N_RANGE)
    nm = fit_norm(Fh, Th)
    for k in ("xm", "xs", "ym", "ys", "L"):
        assert np.max(np.abs(stg[k] - nm[k])) <= 1e-10 * max(1.0, np.max(np.abs(nm[k]))), k
    Xr = (Fh - nm["xm"]) / nm["xs"]
    Yr = network_targets(Fh, Th, nm)
    assert np.max(np.abs(Xs.cpu().numpy() - Xr)) <= 1e-6 * np.max(np.abs(Xr))
    assert np.max(np.abs(Ys.cpu().numpy() - Yr)) <= 1e-5 * np.max(np.abs(Yr))


def test_training_reduces_loss(trained):
    h = trained["hist"]
    assert h[-1] < 0.05 * h[0]
    # where the remaining error sits: the trained weights in FP64 without BF16 rounding
    th = trained["theta"].cpu().numpy().astype(np.float64)
    Xh, Yh = trained["Xs"][trained["held"]][:50000], trained["Ys"][trained["held"]][:50000]
    for bf in (False, True):
        out, _ = omlp.forward(th, Xh.astype(np.float64), bf16=bf)
        report("held_out_rms_standardised_bf16_%s" % bf,
               [float(v) for v in np.sqrt(np.mean((out - Yh) ** 2, axis=0))])


def test_network_matches_oracle_network(trained):
    """The trained parameters give the same outputs through the matrix cores as
    through the oracle's network (BF16 operands) on held-out inputs."""
    Xh = trained["Xs"][trained["held"]][:20000]
    Yd = torch.empty((len(Xh), 8), dtype=torch.float32, device=DEV)
    hrx.mlp_forward(trained["ctx"], len(Xh), torch.from_numpy(Xh).to(DEV), Yd)
    ref, acts = omlp.forward(trained["theta"].cpu().numpy().astype(np.float64),
                             Xh.astype(np.float64), bf16=True)
    Yg = Yd.cpu().numpy()
    assert normwise(Yg, ref) <= 2e-3
    ok = tie_free_rows(acts)          # no BF16 rounding decision near a tie
    report("network_tie_free_rows_fraction", float(ok.mean()))
    assert ok.mean() > 0.2 and normwise(Yg[ok], ref[ok]) <= 1e-4


def _thermo(ctx, raw, sel):
    n = len(raw["rho"][sel])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    T = torch.zeros(n, dtype=torch.float64, device=DEV)   # no temperature guess: cold start
    mu, ka = torch.empty_like(T), torch.empty_like(T)
    D = torch.empty((5, n), dtype=torch.float64, device=DEV)
    st = torch.empty(n, dtype=torch.int32, device=DEV)
    hrx.thermo_eval(ctx, n, d(raw["rho"][sel]), d(raw["e"][sel]), d(raw["Y"][:, sel]), T,
                    mu=mu, kappa=ka, D=D, status=st)
    torch.cuda.synchronize()
    return T.cpu().numpy(), mu.cpu().numpy(), ka.cpu().numpy(), D.cpu().numpy(), st.cpu().numpy()


def test_surrogate_thermo_accuracy_held_out(trained):
    raw = trained["raw"]
    sel = np.arange(trained["ntr"], NTOT)
    ctx = trained["ctx"]
    hrx.set_thermo_mode(ctx, hrx.THERMO_SURROGATE)
    ctx.counters(reset=True)
    T, mu, ka, D, st = _thermo(ctx, raw, sel)
    c = ctx.counters(reset=True)
    hrx.set_thermo_mode(ctx, hrx.THERMO_PLAIN)
    rel = lambda a, b: np.abs(a / b - 1.0)  # noqa: E731
    e_mu, e_ka = rel(mu, raw["mu"][sel]), rel(ka, raw["kappa"][sel])
    e_D = rel(D, raw["D"][:, sel])
    report("held_out_T_normwise", normwise(T, raw["T"][sel]))
    report("held_out_rel_err_max", dict(mu=float(e_mu.max()), kappa=float(e_ka.max()),
                                        D=float(e_D.max())))
    report("held_out_rel_err_rms", dict(mu=float(np.sqrt(np.mean(e_mu ** 2))),
                                        kappa=float(np.sqrt(np.mean(e_ka ** 2))),
                                        D=float(np.sqrt(np.mean(e_D ** 2)))))
    e_all = np.concatenate([e_mu[None], e_ka[None], e_D])
    report("held_out_rel_err_p999", [float(v) for v in np.quantile(e_all, 0.999, axis=1)])
    report("held_out_fallbacks", int(c["surrogate_fallbacks"]))
    assert np.all(st == 0)
    assert c["surrogate_fallbacks"] == 0
    assert normwise(T, raw["T"][sel]) <= 1e-12
    assert np.sqrt(np.mean(e_all ** 2, axis=1)).max() <= 1e-3
    assert np.quantile(e_all, 0.999, axis=1).max() <= 5e-3
    assert e_all.max() <= 1e-2


def test_out_of_hull_falls_back_to_plain(trained):
    ctx = trained["ctx"]
    n = 1000
    rho, T0, Y, _ = fields.thermo_states(n, seed=99, T_range=(9000.0, 12000.0))
    rho = rho * 3.0          # part of them also above the density range
    e = oth.mixture_e(T0, Y)
    raw = dict(rho=rho, e=e, Y=Y)
    hrx.set_thermo_mode(ctx, hrx.THERMO_SURROGATE)
    ctx.counters(reset=True)
    T, mu, ka, D, st = _thermo(ctx, raw, slice(0, n))
    c = ctx.counters(reset=True)
    hrx.set_thermo_mode(ctx, hrx.THERMO_PLAIN)
    assert c["surrogate_fallbacks"] == n
    Tr, _, _ = oth.temperature_from_energy(e, Y)
    p, mur, kr, Dr = otr.air5_properties(rho, Tr, Y)
    assert normwise(T, Tr) <= 1e-12 and normwise(mu, mur) <= 1e-12 and normwise(ka, kr) <= 1e-12
    for s in range(5):
        assert normwise(D[s], Dr[s]) <= 1e-12


def test_composition_outside_hull_falls_back(trained):
    """Compositions whose element-N fraction lies outside the training range fall back
    (and only those); states inside take the network."""
    ctx = trained["ctx"]
    n = 4000
    rho, T0, Y, _ = fields.thermo_states(n, seed=98, T_range=(1000.0, 6000.0),
                                         logrho_range=(-3.0, -1.0))
    e = oth.mixture_e(T0, Y)
    xi = element_N_fraction(Y)
    outside = (xi < XI_N_RANGE[0]) | (xi > XI_N_RANGE[1])
    assert 0 < outside.sum() < n
    hrx.set_thermo_mode(ctx, hrx.THERMO_SURROGATE)
    ctx.counters(reset=True)
    T, mu, ka, D, st = _thermo(ctx, dict(rho=rho, e=e, Y=Y), slice(0, n))
    c = ctx.counters(reset=True)
    hrx.set_thermo_mode(ctx, hrx.THERMO_PLAIN)
    assert c["surrogate_fallbacks"] == int(outside.sum())
    Tr, _, _ = oth.temperature_from_energy(e, Y)
    p, mur, kr, Dr = otr.air5_properties(rho, Tr, Y)
    assert normwise(T, Tr) <= 1e-12
    assert normwise(mu[outside], mur[outside]) <= 1e-12


def test_rhs_with_surrogate_on_sbli_field(trained):
    cfg = fields.get_config("c3").scaled(512, 128)
    Q, Qr, info = fields.initial_field(cfg)
    ctx = with_surrogate(air_ctx(cfg, info["hold"]), trained)
    Qd = torch.from_numpy(Q).to(DEV)
    Rd = torch.empty_like(Qd)
    ctx.counters(reset=True)
    hrx.rhs_eval(ctx, Qd, torch.from_numpy(Qr).to(DEV), Rd)
    c = ctx.counters(reset=True)
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], info["hold"])
    R = orhs.rhs(Q, Qr, case)
    errs = field_errors(Rd.cpu().numpy(), R)
    report("sbli_512x128_rhs_errors_surrogate", [float(e) for e in errs])
    report("sbli_512x128_in_hull_fraction", 1.0 - c["surrogate_fallbacks"] / cfg.npts)
    assert max(errs) <= 1e-3


def test_rhs_with_surrogate_on_full_sbli_field(trained):
    """The surrogate form on the whole 2048 x 512 SBLI-shaped field (the surrogate's
    workload; the large-grid launch shapes): RHS within 1e-3 per field of the plain FP64
    oracle, which also judges its error."""
    cfg = fields.get_config("c3")
    Q, Qr, info = fields.initial_field(cfg)
    ctx = with_surrogate(air_ctx(cfg, info["hold"]), trained)
    Qd = torch.from_numpy(Q).to(DEV)
    Rd = torch.empty_like(Qd)
    ctx.counters(reset=True)
    hrx.rhs_eval(ctx, Qd, torch.from_numpy(Qr).to(DEV), Rd)
    c = ctx.counters(reset=True)
    Rg = Rd.cpu().numpy()
    ctx.close()
    del Qd, Rd
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], info["hold"])
    R = orhs.rhs(Q, Qr, case)
    errs = field_errors(Rg, R)
    report("sbli_2048x512_rhs_errors_surrogate", [float(e) for e in errs])
    report("sbli_2048x512_in_hull_fraction", 1.0 - c["surrogate_fallbacks"] / cfg.npts)
    assert max(errs) <= 1e-3
    assert c["surrogate_fallbacks"] < 0.01 * cfg.npts


# The surrogate's measured gains over the plain evaluation, as DESIGN records them
# (below 1: on MI355X the plain FP64 path is the faster one).  The guard fails if the
# surrogate form falls more than 15 % behind them.
DOCUMENTED_GAIN = dict(thermo_eval=0.86, sbli_stage=0.96)


def _stage_rate(ctx, cfg, Q, Qr, dt, stages=40):
    Qd = torch.from_numpy(Q).to(DEV)
    Qrd = torch.from_numpy(Qr).to(DEV)
    dQ = torch.zeros_like(Qd)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for k in range(6):
            hrx.rk_stage(ctx, k % 3, dt, Qd, dQ, Qrd)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(stages):
            hrx.rk_stage(ctx, k % 3, dt, Qd, dQ, Qrd)
        b.record()
        torch.cuda.synchronize()
    assert bool(torch.isfinite(Qd).all())
    return cfg.npts * stages / (a.elapsed_time(b) * 1e-3) / 1e6


def test_surrogate_gain_measured(trained):
    """What the trained network gains over the method without it, measured at the
    accuracy the tests above establish, in two settings:
    * the pointwise SI call on 2^21 held-out-like states, where the network also gives
      the energy inversion its start (the plain call starts cold);
    * RK stages of the SBLI-shaped field, where the inversion starts warm from the
      previous stage and the network replaces the transport only.
    Both ratios are reported (surrogate_report.json); the assertions check that the
    surrogate form ran on the network (no fallbacks), kept the state finite, and kept
    within 15 % of the gains recorded in DOCUMENTED_GAIN (the sign is not asserted: the
    recorded gains are below 1)."""
    n = 1 << 21
    rho, T0, Y = states(n, seed=123)
    e = oth.mixture_e(T0, Y)
    ctx = trained["ctx"]
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    rd, ed, Yd = d(rho), d(e), d(Y)
    T = torch.zeros(n, dtype=torch.float64, device=DEV)   # no temperature guess: cold start
    p, mu, ka = torch.empty_like(T), torch.empty_like(T), torch.empty_like(T)
    h = torch.empty((5, n), dtype=torch.float64, device=DEV)
    D = torch.empty((5, n), dtype=torch.float64, device=DEV)
    res = {}
    for mode in (hrx.THERMO_PLAIN, hrx.THERMO_SURROGATE):
        hrx.set_thermo_mode(ctx, mode)
        for _ in range(2):
            T.zero_()
            hrx.thermo_eval(ctx, n, rd, ed, Yd, T, p, h, mu, ka, D)
        ctx.counters(reset=True)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            T.zero_()                          # every call starts its inversion cold
            hrx.thermo_eval(ctx, n, rd, ed, Yd, T, p, h, mu, ka, D)
        b.record()
        torch.cuda.synchronize()
        res[mode] = a.elapsed_time(b) / 10
        assert ctx.counters(reset=True)["surrogate_fallbacks"] == 0
    hrx.set_thermo_mode(ctx, hrx.THERMO_PLAIN)
    report("thermo_eval_Mpts_per_s", dict(plain=n / res[0] / 1e3, surrogate=n / res[1] / 1e3))
    report("thermo_eval_gain", res[hrx.THERMO_PLAIN] / res[hrx.THERMO_SURROGATE])
    # RK stages on the SBLI-shaped field
    cfg = fields.get_config("c3").scaled(512, 128)
    Q, Qr, info = fields.initial_field(cfg)
    rate = {}
    for mode in (hrx.THERMO_PLAIN, hrx.THERMO_SURROGATE):
        c = air_ctx(cfg, info["hold"])
        if mode == hrx.THERMO_SURROGATE:
            with_surrogate(c, trained)
        rate[mode] = _stage_rate(c, cfg, Q, Qr, info["dt"])
        if mode == hrx.THERMO_SURROGATE:
            assert c.counters(reset=True)["surrogate_fallbacks"] < 0.01 * cfg.npts * 46
        c.close()
    report("sbli_512x128_stage_Mpts_per_s", dict(plain=rate[0], surrogate=rate[1]))
    report("sbli_512x128_stage_gain", rate[1] / rate[0])
    assert res[0] > 0 and res[1] > 0
    assert res[hrx.THERMO_PLAIN] / res[hrx.THERMO_SURROGATE] >= 0.85 * DOCUMENTED_GAIN["thermo_eval"]
    assert rate[1] / rate[0] >= 0.85 * DOCUMENTED_GAIN["sbli_stage"]
