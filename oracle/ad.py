"""Artificial-diffusivity coefficients (oracle; test infrastructure only).

Sec. 3.3 states only that shocks are captured with artificial bulk and shear
viscosity (and, by the works it cites, artificial conductivity and species
diffusivity), without formulas.  Reading taken here, in index space with local
spacings Delta_l = dx_l/dxi_l and their geometric mean Delta_bar:

  mu*   = C_mu    rho        G[ | sum_l D4_l(|S|)   Delta_l^2 | ]
  beta* = C_beta  rho f_sw   G[ | sum_l D4_l(theta) Delta_l^2 | ]
  kap*  = C_kappa rho c / T  G[ | sum_l D4_l(e)     Delta_l   | ]
  D*_s  = c G[ C_D | sum_l D4_l(Y_s) Delta_l | + C_Y (|Y_s| - 1 + |1 - Y_s|)/2 Delta_bar ]

with |S| = sqrt(S_ij S_ij), theta = div u, the switch
f_sw = H(-theta) theta^2 / (theta^2 + |omega|^2 + 1e-32) (H(0) = 0), D4 the fourth
difference (1,-4,6,-4,1) along direction l, and G the 9-point truncated Gaussian
filter applied along x, then y, then z.  rho, c (frozen sound speed), T and e are
nondimensional.
"""
import numpy as np

from . import stencils as st

TINY = 1e-32


def switch(G, nd):
    theta = sum(G[i][i] for i in range(nd))
    if nd == 2:
        w2 = (G[1][0] - G[0][1]) ** 2
    else:
        w2 = ((G[2][1] - G[1][2]) ** 2 + (G[0][2] - G[2][0]) ** 2 + (G[1][0] - G[0][1]) ** 2)
    fsw = np.where(theta < 0.0, theta * theta / (theta * theta + w2 + TINY), 0.0)
    return theta, fsw


def strain_magnitude(G, nd):
    s2 = 0.0
    for i in range(nd):
        for j in range(nd):
            sij = 0.5 * (G[i][j] + G[j][i])
            s2 = s2 + sij * sij
    return np.sqrt(s2)


def filt(f, case):
    out = f
    for d in range(case.ndim):
        out = st.gaussian_filter(out, case.axis(d), periodic=(d == 2))
    return out


def d4sum(f, case, power):
    acc = 0.0
    for d in range(case.ndim):
        ax = case.axis(d)
        delta = st.spacing([case.x, case.y, case.z][d], periodic=(d == 2))
        sh = [1, 1, 1]
        sh[ax] = len(delta)
        acc = acc + st.fourth_difference(f, ax, periodic=(d == 2)) * (delta ** power).reshape(sh)
    return np.abs(acc)


def mean_spacing(case):
    ds = [st.spacing([case.x, case.y, case.z][d], periodic=(d == 2)) for d in range(case.ndim)]
    g = ds[0][None, None, :] * ds[1][None, :, None]
    if case.ndim == 3:
        g = g * ds[2][:, None, None]
    return g ** (1.0 / case.ndim)


def coefficients(P, G, case):
    """mu*, beta*, kappa*, D*_s (nondimensional) from the primitive state and velocity gradients."""
    Cmu, Cbeta, Ckap, CD, CY = case.cfg.ad_coef
    nd = case.ndim
    rho, c, T, e = P["rho"], P["c"], P["T"], P["e"]
    theta, fsw = switch(G, nd)
    S = strain_magnitude(G, nd)
    mu = Cmu * rho * filt(d4sum(S, case, 2), case)
    beta = Cbeta * rho * fsw * filt(d4sum(theta, case, 2), case)
    kap = Ckap * rho * c / T * filt(d4sum(e, case, 1), case)
    out = dict(mu=mu, beta=beta, kappa=kap)
    if case.air5:
        dbar = mean_spacing(case)
        D = []
        for s in range(case.ns):
            Ys = P["Y"][s]
            over = 0.5 * (np.abs(Ys) - 1.0 + np.abs(1.0 - Ys))
            D.append(c * filt(CD * d4sum(Ys, case, 1) + CY * over * dbar, case))
        out["D"] = np.array(D)
    return out
