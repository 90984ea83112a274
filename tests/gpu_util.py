"""Helpers shared by the GPU parity tests (error norms, oracle windows of a full grid)."""
import dataclasses
import json
import os

import numpy as np

# x-y window of the full 3-D jet grid checked against the oracle (every z plane; wall
# row and jet inlet inside), and the margin kept from its cut edges: the RHS at a point
# depends on points up to 12 away through the artificial-diffusivity chain (source
# derivative 3, fourth difference 2, filter 4, flux derivative 3) plus the metric's
# reach; at 12 or more the window oracle equals the whole-domain oracle exactly.
JET_WINDOW = dict(ia=196, ib=260, jb=48, margin=16)


def normwise(a, b):
    """||a - b||_inf / ||b||_inf (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if b.size else 0.0
    if den == 0.0:
        return num
    return num / den


def field_errors(A, B):
    return [normwise(A[k], B[k]) for k in range(A.shape[0])]


def oracle_window(cfg, info, Q, Qr, ia, ib, jb):
    """Oracle case and fields of the window x in [ia, ib), y in [0, jb), all z, of a
    full grid: the window's own coordinates (metrics), no sponge (the window lies outside
    the sponges) and the held inlet points inside it."""
    from oracle import rhs as orhs
    nw = ib - ia
    hw = None
    if info["hold"] is not None:
        hold = np.asarray(info["hold"], dtype=np.int64)
        k, rem = np.divmod(hold, cfg.nx * cfg.ny)
        j, i = np.divmod(rem, cfg.nx)
        inw = (i >= ia) & (i < ib) & (j < jb)
        hw = (k[inw] * jb + j[inw]) * nw + (i[inw] - ia)
    cw = dataclasses.replace(cfg, nx=nw, ny=jb, sponge_in=0, sponge_out=0, sponge_top=0)
    case = orhs.Case(cw, info["x"][ia:ib], info["y"][:jb], info["z"], hw)
    Qw = np.ascontiguousarray(Q[..., :jb, ia:ib])
    Qrw = np.ascontiguousarray(Qr[..., :jb, ia:ib])
    return case, Qw, Qrw


def tie_free_rows(acts, margin=1e-5):
    """Rows of the oracle's forward pass whose hidden activations (the inputs of layers
    2..4, rounded to BF16 there) all lie farther than margin (relative) from a BF16
    rounding midpoint, or are exactly zero (inactive units)."""
    ok = np.ones(acts[0].shape[0], dtype=bool)
    for a in acts[1:4]:
        f = np.abs(a).astype(np.float32)
        u = f.view(np.uint32)
        lo = (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
        hi = ((u & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
        mid = 0.5 * (lo + hi)
        d = np.abs(f.astype(np.float64) - mid) / np.maximum(f.astype(np.float64), 1e-300)
        ok &= np.all((f == 0.0) | (d > margin), axis=1)
    return ok


def write_report(name, data):
    """Writes a test's per-field figures as JSON into the folder that HRX_REPORT_DIR names,
    when it names one (nothing is written otherwise)."""
    out = os.environ.get("HRX_REPORT_DIR")
    if out and os.path.isdir(out):
        with open(os.path.join(out, name), "w") as f:
            json.dump(data, f, indent=1)
