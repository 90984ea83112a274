"""The C-ABI's contract beyond parity: failure statuses and counters, the temperature
guess of thermo_eval, the unfused stage with a caller's right-hand side, the
three-register TVD RK3, and thermo_eval's surrogate form without allocation.

Failure cases are planted on the host (a NaN energy, a negative partial density, one
Newton iteration allowed); every kernel still runs to completion on finite or NaN
values.  Parity bars as in test_gpu_parity (1e-12 normwise per field, statuses
exact).
"""
import dataclasses
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_05547_amd import fields, hrx  # noqa: E402
from oracle import mlp as omlp  # noqa: E402
from oracle import rhs as orhs  # noqa: E402
from oracle import thermo as oth  # noqa: E402
from oracle import transport as otr  # noqa: E402
from gpu_util import field_errors, normwise  # noqa: E402

TOL = 1e-12
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def air_ctx(**kw):
    cfg = fields.get_config("c2").scaled(16, 16)
    x, y, z = fields.grid(cfg)
    return hrx.Context(cfg, x, y, z, **kw)


def _thermo(ctx, rho, e, Y, T_in=None, want_all=True):
    n = len(rho)
    T = dev(T_in) if T_in is not None else torch.zeros(n, dtype=torch.float64, device=DEV)
    out = dict(T=T)
    if want_all:
        out.update(p=torch.empty(n, dtype=torch.float64, device=DEV),
                   h=torch.empty((5, n), dtype=torch.float64, device=DEV),
                   mu=torch.empty(n, dtype=torch.float64, device=DEV),
                   kappa=torch.empty(n, dtype=torch.float64, device=DEV),
                   D=torch.empty((5, n), dtype=torch.float64, device=DEV))
    st = torch.full((n,), -9, dtype=torch.int32, device=DEV)
    hrx.thermo_eval(ctx, n, dev(rho), dev(e), dev(Y), T, out.get("p"), out.get("h"),
                    out.get("mu"), out.get("kappa"), out.get("D"), st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, st.cpu().numpy()


def test_thermo_eval_temperature_guess():
    """A guess in (50 K, 1e5 K) starts the inversion; the root and every output are the
    same as from a cold start (1e-12); an out-of-range guess starts cold."""
    say("thermo_eval guess")
    n = 4099
    rho, T0, Y, _ = fields.thermo_states(n, seed=23)
    e = oth.mixture_e(T0, Y)
    ctx = air_ctx()
    cold, st0 = _thermo(ctx, rho, e, Y)
    rng = np.random.default_rng(3)
    guess = T0 * rng.uniform(0.5, 1.6, n)
    guess[::7] = np.nan
    guess[1::7] = 3e5                          # outside the accepted range: cold start
    warm, st1 = _thermo(ctx, rho, e, Y, T_in=guess)
    assert (st0 == 0).all() and (st1 == 0).all()
    for k in cold:
        assert normwise(warm[k], cold[k]) <= TOL, k
    T, _, _ = oth.temperature_from_energy(e, Y)
    assert normwise(warm["T"], T) <= TOL


def test_newton_iteration_limit_gives_enewton():
    """One Newton iteration from a cold start cannot converge: status 1 at every point,
    the counter, and HRX_ENEWTON from hrx_get_counters; the oracle with the same limit
    reports the same statuses."""
    say("newton limit")
    n = 777
    rho, T0, Y, _ = fields.thermo_states(n, seed=5)
    e = oth.mixture_e(T0, Y)
    ctx = air_ctx(newton_max_iter=1)
    ctx.counters(reset=True)
    out, st = _thermo(ctx, rho, e, Y, want_all=False)
    _, _, st_o = oth.temperature_from_energy(e, Y, max_iter=1)
    assert np.array_equal(st, st_o.astype(np.int32))
    assert (st == 1).all()
    c = ctx.counters(reset=True)
    assert c["newton_nonconverged"] == n and c["status"] == hrx.HRX_ENEWTON
    assert ctx.counters()["status"] == hrx.HRX_OK


def test_nonfinite_and_domain_statuses():
    """A NaN energy, an infinite mass fraction and a non-positive density give status 3
    and NaN outputs, an energy below e(50 K) status 2; the other points are unaffected
    and exact; hrx_get_counters reports the most severe failure."""
    say("non-finite statuses")
    n = 64
    rho, T0, Y, _ = fields.thermo_states(n, seed=9)
    e = oth.mixture_e(T0, Y)
    e[3] = np.nan
    Y[2, 10] = np.inf
    rho[20] = 0.0
    rho[21] = -1.0
    e[30] = oth.mixture_e(np.array([20.0]), Y[:, 30:31])[0]
    ctx = air_ctx()
    ctx.counters(reset=True)
    out, st = _thermo(ctx, rho, e, Y)
    bad = [3, 10, 20, 21]
    assert [int(st[i]) for i in bad] == [3, 3, 3, 3] and st[30] == 2
    for i in bad:
        assert np.isnan(out["T"][i]) and np.isnan(out["mu"][i]) and np.isnan(out["D"][:, i]).all()
    good = np.setdiff1d(np.arange(n), bad + [30])
    assert (st[good] == 0).all()
    T, _, _ = oth.temperature_from_energy(e[good], Y[:, good])
    assert normwise(out["T"][good], T) <= TOL
    c = ctx.counters(reset=True)
    assert c["nonfinite"] == 4 and c["energy_below_min"] == 1
    assert c["status"] == hrx.HRX_ENONFINITE


def test_rhs_counts_negative_densities_and_nonfinite_states():
    """Planted in Q: negative partial densities are counted (not failures); a NaN is a
    non-finite state (HRX_ENONFINITE)."""
    say("rhs counters")
    cfg = fields.get_config("c2").scaled(40, 24)
    Q, Qr, info = fields.initial_field(cfg)
    Qn = Q.copy()
    Qn[4, 0, 10, 7] = -1e-6
    Qn[3, 0, 12, 9] = -2e-7
    Qn[4, 0, 12, 9] = -2e-7                   # one point, two species: counted once
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"])
    ctx.counters(reset=True)
    R = torch.empty_like(dev(Q))
    hrx.rhs_eval(ctx, dev(Qn), dev(Qr), R)
    c = ctx.counters(reset=True)
    assert c["negative_density"] == 2 and c["nonfinite"] == 0 and c["status"] == hrx.HRX_OK
    Qn[7, 0, 5, 5] = np.nan
    hrx.rhs_eval(ctx, dev(Qn), dev(Qr), R)
    c = ctx.counters(reset=True)
    assert c["nonfinite"] == 1 and c["status"] == hrx.HRX_ENONFINITE


def _stages(cfg, stages, unfused=False, tol=None):
    Q, Qr, info = fields.initial_field(cfg)
    say("stages", cfg.name, cfg.nx, cfg.ny, cfg.nz, "rk", cfg.rk, "unfused", unfused, stages)
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"])
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], info["hold"])
    Qd, Qrd = dev(Q), dev(Qr)
    dQd = torch.zeros_like(Qd)
    Rd = torch.empty_like(Qd)
    Qo, dQo = Q.copy(), np.zeros_like(Q)
    for k in range(stages):
        if unfused:
            hrx.rhs_eval(ctx, Qd, Qrd, Rd)
            hrx.rk_stage(ctx, k, info["dt"], Qd, dQd, None, R=Rd)
            Ro = orhs.rhs(Qo, Qr, case)
            orhs.rk_stage(Qo, dQo, None, case, k, info["dt"], R=Ro)
        else:
            hrx.rk_stage(ctx, k, info["dt"], Qd, dQd, Qrd)
            orhs.rk_stage(Qo, dQo, Qr, case, k, info["dt"])
    torch.cuda.synchronize()
    errs = field_errors(Qd.cpu().numpy(), Qo)
    say("  Q errors", ["%.2e" % e for e in errs])
    tol = tol or [TOL] * len(errs)
    assert all(e <= t for e, t in zip(errs, tol)), (errs, tol)
    c = ctx.counters()
    assert c["status"] == hrx.HRX_OK
    ctx.close()
    return Qd


def test_ssp_rk3_c1_100_stages():
    """1e-12 on rho, rho u and rho E; 2e-12 on rho v.  The plate's wall-normal momentum
    starts at zero and is driven by nearly cancelling pressure differences, so its
    normwise error is amplified: two oracle runs whose fluxes differ by one rounding
    already part by up to 1.2e-12 over these stages (measured on the CPU by
    test_oracle_rhs.py::test_wall_normal_momentum_conditioning_of_the_plate)."""
    _stages(dataclasses.replace(fields.get_config("c1"), rk=2), 100,
            tol=[TOL, TOL, 2e-12, TOL])


@pytest.mark.parametrize("shape", [(40, 24), (1030, 270)])
def test_ssp_rk3_air5(shape):
    """2-D air: the wall condition inside the divergence kernel, below and above the
    small-grid split."""
    _stages(dataclasses.replace(fields.get_config("c2").scaled(*shape), rk=2),
            6 if shape[0] < 100 else 3)


def test_ssp_rk3_jet_3d():
    _stages(dataclasses.replace(fields.get_config("c4").scaled(40, 32, 16), rk=2), 3)


@pytest.mark.parametrize("rk", [0, 1, 2])
def test_unfused_stage_with_callers_rhs(rk):
    """hrx_rk_stage with R from hrx_rhs_eval: pointwise update and the separate wall pass,
    against the oracle stage given its own right-hand side."""
    _stages(dataclasses.replace(fields.get_config("c2").scaled(40, 24), rk=rk), 5, unfused=True)


def test_unfused_stage_3d_tpg():
    cfg = dataclasses.replace(fields.get_config("c4").scaled(40, 32, 16), gas=2, ad=False,
                              jet=False, species_noise=0.0, wall=0, T_wall=0.0, rk=2)
    _stages(cfg, 3, unfused=True)


def test_surrogate_thermo_eval_chunks_without_allocation():
    """In the surrogate form thermo_eval runs its network through the context's
    workspace in chunks: a call of 2^20 + 4099 states allocates nothing (free device
    memory unchanged) and equals, bit for bit, the same states in two calls."""
    say("surrogate chunks")
    ctx = air_ctx()
    hrx.mlp_init(ctx, 16)
    theta = omlp.init_params(7).astype(np.float32)
    hrx.mlp_set_params(ctx, dev(theta))
    hrx.mlp_set_norm(ctx, np.zeros(7), np.ones(7), np.zeros(8), np.full(8, 0.01), (-4.0, 0.0),
                     (200.0, 8000.0), xiN_range=(0.0, 1.0))
    hrx.set_thermo_mode(ctx, hrx.THERMO_SURROGATE)
    n = (1 << 20) + 4099
    rho, T0, Y, _ = fields.thermo_states(n, seed=31)
    e = oth.mixture_e(T0, Y)
    d = {k: dev(v) for k, v in dict(rho=rho, e=e, Y=Y).items()}
    outs = []
    for split in (None, 600_001):
        T = torch.zeros(n, dtype=torch.float64, device=DEV)
        mu, ka = torch.empty_like(T), torch.empty_like(T)
        D = torch.empty((5, n), dtype=torch.float64, device=DEV)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        if split is None:
            hrx.thermo_eval(ctx, n, d["rho"], d["e"], d["Y"], T, mu=mu, kappa=ka, D=D)
        else:
            for a, b in ((0, split), (split, n)):
                m = b - a
                Dp = torch.empty((5, m), dtype=torch.float64, device=DEV)
                hrx.thermo_eval(ctx, m, d["rho"][a:b], d["e"][a:b],
                                d["Y"][:, a:b].contiguous(), T[a:b], mu=mu[a:b],
                                kappa=ka[a:b], D=Dp)
                D[:, a:b] = Dp
        torch.cuda.synchronize()
        if split is None:
            assert torch.cuda.mem_get_info()[0] == free0
        outs.append([t.cpu().numpy() for t in (T, mu, ka, D)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    T_or, _, _ = oth.temperature_from_energy(e, Y)
    assert normwise(outs[0][0], T_or) <= TOL
