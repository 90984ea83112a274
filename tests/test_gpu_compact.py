"""GPU parity of the compact (Pade) first derivatives (Sec. 3.1 reading; hrx_config
fd_scheme = HRX_FD_COMPACT) against the oracle (oracle/compact.py in oracle/rhs.py).

The line solves of the gradients and of the divergence (x: one wavefront per line with
an affine scan, up to 8 lines per wavefront in turn; y, z: 16 lines per block held on chip, 16 chunks per line joined by an
affine scan, z cyclic; lines over 512 points: one thread per line) feed the same physics
as the explicit path.  Bars as in test_gpu_parity: 1e-12 normwise per field for the FP64 path
(RHS and Q after the stages), 1e-5 for the mixed form.
"""
import dataclasses
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2210_05547_amd import fields, hrx  # noqa: E402
from oracle import rhs as orhs  # noqa: E402
from gpu_util import field_errors  # noqa: E402

TOL = 1e-12
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def compact(cfg, **kw):
    return dataclasses.replace(cfg, fd_scheme=1, **kw)


def _run(cfg, stages, rhs=True, precision=hrx.PREC_FP64, tol=TOL, noalloc=False):
    Q, Qr, info = fields.initial_field(cfg)
    say("compact case", cfg.name, cfg.nx, cfg.ny, cfg.nz, "order", cfg.fd_order, "rk", cfg.rk,
        "stages", stages, "mixed" if precision else "fp64")
    ctx = hrx.Context(cfg, info["x"], info["y"], info["z"], info["hold"], precision=precision)
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], info["hold"])
    Qd, Qrd = dev(Q), dev(Qr)
    if rhs:
        Rd = torch.empty_like(Qd)
        (hrx.rhs_eval_noalloc if noalloc else hrx.rhs_eval)(ctx, Qd, Qrd, Rd)
        torch.cuda.synchronize()
        R = orhs.rhs(Q, Qr, case)
        errs = field_errors(Rd.cpu().numpy(), R)
        say("  rhs errors", ["%.2e" % e for e in errs])
        assert max(errs) <= tol
    if stages:
        dQd = torch.zeros_like(Qd)
        Qo, dQo = Q.copy(), np.zeros_like(Q)
        for k in range(stages):
            hrx.rk_stage(ctx, k, info["dt"], Qd, dQd, Qrd)
            orhs.rk_stage(Qo, dQo, Qr, case, k, info["dt"])
        torch.cuda.synchronize()
        errs = field_errors(Qd.cpu().numpy(), Qo)
        say("  Q errors after", stages, ["%.2e" % e for e in errs])
        assert max(errs) <= tol
    c = ctx.counters()
    assert c["status"] == hrx.HRX_OK
    ctx.close()


def test_compact_c1_cpg_rhs_and_stages():
    _run(compact(fields.get_config("c1")), 30)


def test_compact_c1_fourth_order_rk4_isothermal():
    _run(compact(fields.get_config("c1"), fd_order=4, rk=1, wall=1, T_wall=600.0), 10)


def test_compact_c1_ssp_rk3():
    _run(compact(fields.get_config("c1").scaled(64, 40), rk=2), 9)


# x lines of 40, 67, 200 and 700 points: the x solve's chunks of 1, 2, 4 and 16 points
@pytest.mark.parametrize("shape", [(40, 24), (67, 41), (200, 40), (700, 24)])
def test_compact_c2_air5_reduced(shape):
    _run(compact(fields.get_config("c2").scaled(*shape)), 4)


def test_compact_c2_full_size():
    """The bench's flat plate, 512 x 256, with compact derivatives: RHS and two stages."""
    _run(compact(fields.get_config("c2")), 2)


def test_compact_c2_above_split_ragged():
    _run(compact(fields.get_config("c2").scaled(1030, 270)), 1)


def test_compact_c3_sbli_ad_reduced():
    _run(compact(fields.get_config("c3").scaled(96, 48)), 3)


def test_compact_c4_jet_3d_reduced():
    """3-D: y lines and cyclic z lines, the jet inlet held, artificial diffusivity."""
    _run(compact(fields.get_config("c4").scaled(40, 32, 16)), 2)


def test_compact_c4_jet_3d_fourth_order():
    _run(compact(fields.get_config("c4").scaled(36, 24, 16), fd_order=4), 1)


@pytest.mark.parametrize("shape", [(37, 45, 21), (21, 17, 9), (18, 70, 33)])
def test_compact_c4_ragged_3d(shape):
    """Line counts off the 16-line groups and line lengths off the 16-chunk split (empty
    and partial chunks, y and cyclic z)."""
    _run(compact(fields.get_config("c4").scaled(*shape)), 1)


@pytest.mark.parametrize("shape", [(16, 127, 67), (100, 90, 25), (72, 61, 61)])
def test_compact_x_lines_several_per_wavefront(shape):
    """Grids with enough x lines that each wavefront of the x solve takes 8, 2 and 4 lines
    in turn (line counts not a multiple of the lines per block)."""
    _run(compact(fields.get_config("c4").scaled(*shape)), 1)


def test_compact_x_lines_longest_chunks_several_per_wavefront():
    """x lines of 520 points (chunks of 16 per lane) with two lines per wavefront."""
    _run(compact(fields.get_config("c4").scaled(520, 20, 110)), 0)


@pytest.mark.parametrize("base,shape", [("c2", (20, 300)), ("c4", (12, 300, 10)),
                                        ("c4", (12, 16, 270))])
def test_compact_long_on_chip_lines(base, shape):
    """y and cyclic z lines of 257..512 points: the on-chip solve's longest chunks (32)."""
    _run(compact(fields.get_config(base).scaled(*shape)), 1)


def test_compact_tall_lines_fallback():
    """y lines over 512 points take the thread-per-line solve."""
    _run(compact(fields.get_config("c2").scaled(20, 530)), 1)


def test_compact_stefan_maxwell_and_tpg():
    _run(compact(fields.get_config("c2").scaled(40, 24), diffusion=1), 2)
    _run(compact(fields.get_config("c1t")), 6)


def test_compact_mixed_form():
    _run(compact(fields.get_config("c3").scaled(96, 48)), 2, precision=hrx.PREC_MIXED,
         tol=1e-5)


def test_compact_noalloc_entry():
    _run(compact(fields.get_config("c3").scaled(96, 48)), 0, noalloc=True)
