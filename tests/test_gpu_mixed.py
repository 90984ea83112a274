"""Mixed-precision form through the C-ABI against the FP64 oracle.

The mixed form keeps planes, stencils, fluxes, transport and rate products in FP32 and
the energy inversion, the Arrhenius exponentials at T >= 2000 K, the conserved state
and the RK update in FP64.  Bar: 1e-5 relative, normwise per field, on every
component of R, on the change of Q over the stages, and on mu, kappa, D_s, wdot_s of
the pointwise calls.  Per-field errors are printed (and written to
mixed_errors.json in the folder HRX_REPORT_DIR names, if set).
"""
import dataclasses
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_05547_amd import fields, hrx  # noqa: E402
from oracle import chemistry as och  # noqa: E402
from oracle import rhs as orhs  # noqa: E402
from oracle import thermo as oth  # noqa: E402
from oracle import transport as otr  # noqa: E402
from gpu_util import JET_WINDOW, field_errors, normwise, oracle_window, write_report  # noqa: E402

TOL = 1e-5
DEV = "cuda:0"
REPORT = {}


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _record(name, errs):
    REPORT[name] = [float(e) for e in errs]
    write_report("mixed_errors.json", REPORT)


def _mixed_case(cfg, stages, name):
    Q, Qr, info = fields.initial_field(cfg)
    say("mixed case", name, cfg.nx, cfg.ny, cfg.nz)
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"], precision=hrx.PREC_MIXED)
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], info["hold"])
    Qd, Qrd = dev(Q), dev(Qr)
    Rd = torch.empty_like(Qd)
    hrx.rhs_eval(ctx, Qd, Qrd, Rd)
    torch.cuda.synchronize()
    R = orhs.rhs(Q, Qr, case)
    errs = field_errors(Rd.cpu().numpy(), R)
    say("  R errors", ["%.2e" % e for e in errs])
    _record(name + ":R", errs)
    assert max(errs) <= TOL
    if stages:
        dQd = torch.zeros_like(Qd)
        Qo, dQo = Q.copy(), np.zeros_like(Q)
        for k in range(stages):
            hrx.rk_stage(ctx, k, info["dt"], Qd, dQd, Qrd)
            orhs.rk_stage(Qo, dQo, Qr, case, k, info["dt"])
        torch.cuda.synchronize()
        errs = field_errors(Qd.cpu().numpy() - Q, Qo - Q)
        say("  dQ-over-stages errors", ["%.2e" % e for e in errs])
        _record(name + ":Q_change", errs)
        assert max(errs) <= TOL
    ctx.close()


def test_mixed_c1_cpg():
    _mixed_case(fields.get_config("c1"), 10, "c1")


def test_mixed_c1t_tpg():
    _mixed_case(fields.get_config("c1t"), 10, "c1t")


def test_mixed_c2_stefan_maxwell():
    cfg = dataclasses.replace(fields.get_config("c2").scaled(67, 41), diffusion=1)
    _mixed_case(cfg, 3, "c2_sm_67x41")


def test_mixed_stefan_maxwell_3d_and_with_ad():
    """The Stefan-Maxwell flux in the mixed form on the 3-D jet and on the SBLI with
    artificial diffusivity."""
    cfg = dataclasses.replace(fields.get_config("c4").scaled(40, 32, 16), diffusion=1)
    _mixed_case(cfg, 2, "c4_sm_40x32x16")
    cfg = dataclasses.replace(fields.get_config("c3").scaled(96, 48), diffusion=1)
    _mixed_case(cfg, 2, "c3_sm_96x48")


def test_mixed_c4_ragged_3d():
    _mixed_case(fields.get_config("c4").scaled(37, 29, 13), 2, "c4_37x29x13")


def test_mixed_c2_full():
    _mixed_case(fields.get_config("c2"), 3, "c2")


def test_mixed_c3_sbli_ad():
    _mixed_case(fields.get_config("c3").scaled(256, 96), 3, "c3_256x96")


def test_mixed_c4_jisc():
    _mixed_case(fields.get_config("c4").scaled(48, 32, 16), 2, "c4_48x32x16")


def test_mixed_c3_full():
    _mixed_case(fields.get_config("c3"), 1, "c3_full")


def test_mixed_c4_full_size_window():
    """The full 3-D jet grid in the mixed form: R and the change of Q over one stage on
    an x-y window, against the oracle on that window (see the FP64 window test)."""
    cfg = fields.get_config("c4")
    Q, Qr, info = fields.initial_field(cfg)
    ia, ib, jb, M = (JET_WINDOW[k] for k in ("ia", "ib", "jb", "margin"))
    say("mixed case c4 full size; window x", ia, ib, "y 0", jb)
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"], precision=hrx.PREC_MIXED)
    Qd, Qrd = dev(Q), dev(Qr)
    Rd = torch.empty_like(Qd)
    hrx.rhs_eval(ctx, Qd, Qrd, Rd)
    dQd = torch.zeros_like(Qd)
    hrx.rk_stage(ctx, 0, info["dt"], Qd, dQd, Qrd)
    torch.cuda.synchronize()
    Rg = Rd[..., :jb, ia:ib].cpu().numpy()
    Qg = Qd[..., :jb, ia:ib].cpu().numpy()
    ctx.close()
    del Rd, Qd, dQd, Qrd
    case, Qw, Qrw = oracle_window(cfg, info, Q, Qr, ia, ib, jb)
    del Q, Qr
    sl = (slice(None), slice(None), slice(0, jb - M), slice(M, ib - ia - M))
    R = orhs.rhs(Qw, Qrw, case)
    errs = field_errors(Rg[sl], R[sl])
    say("  R errors", ["%.2e" % e for e in errs])
    _record("c4_full_window:R", errs)
    assert max(errs) <= TOL
    Qo, dQo = Qw.copy(), np.zeros_like(Qw)
    orhs.rk_stage(Qo, dQo, Qrw, case, 0, info["dt"])
    errs = field_errors(Qg[sl] - Qw[sl], Qo[sl] - Qw[sl])
    say("  dQ-over-stages errors", ["%.2e" % e for e in errs])
    _record("c4_full_window:Q_change", errs)
    assert max(errs) <= TOL


def test_mixed_pointwise():
    cfg = fields.get_config("c2").scaled(16, 16)
    x, y, z = fields.grid(cfg)
    ctx = hrx.Context(cfg, x, y, z, precision=hrx.PREC_MIXED)
    n = 30000
    rho, T0, Y, _ = fields.thermo_states(n, seed=21)
    e = oth.mixture_e(T0, Y)
    T = torch.zeros(n, dtype=torch.float64, device=DEV)   # no temperature guess: cold start
    mu = torch.empty_like(T)
    kap = torch.empty_like(T)
    D = torch.empty((5, n), dtype=torch.float64, device=DEV)
    hrx.thermo_eval(ctx, n, dev(rho), dev(e), dev(Y), T, mu=mu, kappa=kap, D=D)
    Tr, _, _ = oth.temperature_from_energy(e, Y)
    p, mur, kr, Dr = otr.air5_properties(rho, Tr, Y)
    errs = [normwise(T.cpu().numpy(), Tr), normwise(mu.cpu().numpy(), mur),
            normwise(kap.cpu().numpy(), kr)] + [normwise(D.cpu().numpy()[s], Dr[s]) for s in range(5)]
    rhos = rho[None] * Y
    w = torch.empty((5, n), dtype=torch.float64, device=DEV)
    hrx.chem_source(ctx, n, dev(rhos), dev(Tr), w)
    torch.cuda.synchronize()
    wr = och.production_rates(rhos, Tr)
    errs += [normwise(w.cpu().numpy()[s], wr[s]) for s in range(5)]
    say("  pointwise errors T, mu, kappa, D1-5, wdot1-5", ["%.2e" % v for v in errs])
    _record("pointwise:T,mu,kappa,D1..5,wdot1..5", errs)
    assert errs[0] <= 1e-12            # the energy inversion stays FP64
    assert max(errs) <= TOL
