"""Right-hand side F(Q) and Runge-Kutta stages (oracle; test infrastructure only).

Follows Sec. 2.1: Eq. (5)-(6) dQ/dt = -div F_C + div F_D + S with
  F_C = (rho_s u, rho u (x) u + p I, rho H u),  F_D = (-rho_s V_s, tau, tau.u - q),
  S = (omega_s, 0, 0);
the stress of Eq. (9), the heat flux of Eq. (10) (diffusive-enthalpy term only with
finite-rate chemistry), Ramshaw's diffusion flux Eq. (18) with the averaged
coefficient of Eq. (19), the nondimensionalisation of Eq. (7)-(8), the sponge term of
Eq. (26) (Sec. 3.2) and the explicit low-storage Runge-Kutta stages of Sec. 3.1.

State vector: Q = [rho, rho u, rho v, (rho w), rho E] for the calorically perfect gas;
for 5-species air all species equations are solved and global continuity is dropped
(the alternative offered in Sec. 2.1): Q = [rho_1..rho_5, rho u.., rho E].  Layout
[nvar][nz][ny][nx], x fastest.

Readings (where the paper is silent or garbled):
* Eq. (9) prints no 2/3 on the divergence term; Stokes' hypothesis -2/3 is used.
* Eq. (18) prints grad Y_s with the molar prefactor c M_s; it is read as grad X_s,
  consistent with the driving force of Eq. (16).  Both readings give sum J_s = 0.
* CPG conductivity: kappa = mu nondimensionally (Sec. 2.2.2).
* Thermally perfect gas (Sec. 2.2.2): the state of module tpg, with the calorically
  perfect gas's state vector and equation of state.
* Boundaries (Sec. 3.2): inflow column held (R = 0); no-slip wall with zero momentum
  RHS; after each stage the wall row gets extrapolated mass fractions (zero normal
  gradient, non-catalytic), the evolved density, zero momentum and the energy of the
  wall temperature (isothermal) or of the extrapolated temperature (adiabatic);
  optional held points (jet patch) have R = 0.  Sponge sigma = sigma_max s^3 with s
  the normalised depth into each sponge (a cubic, Sec. 3.2); overlapping sponges
  take the maximum.
"""
import numpy as np

from . import compact as cp
from . import species as sp
from . import stencils as st
from . import thermo
from . import transport
from . import chemistry
from . import refstate as rs
from . import tpg

# Low-storage (2N) Runge-Kutta coefficients: Williamson's third-order scheme and the
# Carpenter-Kennedy five-stage fourth-order scheme.
RK3_A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK3_B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
RK4_A = (0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
         -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0)
RK4_B = (1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
         1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
         2277821191437.0 / 14882151754819.0)
RK_SCHEMES = {0: (RK3_A, RK3_B), 1: (RK4_A, RK4_B)}
# The three-register TVD (strong-stability-preserving) RK3 of Shu and Osher, the third
# scheme Sec. 3.1 names: with Q0 the step's initial state, stage k sets
# Q <- a_k Q0 + b_k (Q + dt R(Q)).
SSP_RK3 = ((0.0, 1.0), (3.0 / 4.0, 1.0 / 4.0), (1.0 / 3.0, 2.0 / 3.0))
SSPRK3 = 2

# wall extrapolation with zero normal derivative (point-0 closure set to zero)
WALL_EXTRAP = (48.0 / 25.0, -36.0 / 25.0, 16.0 / 25.0, -3.0 / 25.0)


class Case:
    """Geometry, reference state, metrics and sponge of one workload."""

    def __init__(self, cfg, x, y, z, hold=None):
        self.cfg = cfg
        self.ref = rs.reference_from_config(cfg)
        self.air5 = cfg.gas == 1
        self.gas = cfg.gas
        self.ns = 5 if self.air5 else 1
        self.ndim = cfg.ndim
        self.nvar = self.ns + self.ndim + 1
        self.x, self.y, self.z = np.asarray(x), np.asarray(y), np.asarray(z)
        o = cfg.fd_order
        # first derivatives: explicit stencils (module stencils) or compact (module compact)
        self.compact = getattr(cfg, "fd_scheme", 0) == 1
        met = cp.metric if self.compact else st.metric
        self.m = [met(self.x, o), met(self.y, o)]
        if self.ndim == 3:
            self.m.append(st.metric_periodic(self.z))
        self.sigma = self._sponge()
        self.hold = None if hold is None else np.asarray(hold, dtype=np.int64)

    def _sponge(self):
        c = self.cfg
        nx, ny = c.nx, c.ny
        sx = np.zeros(nx)
        sy = np.zeros(ny)
        if c.sponge_in > 0:
            i1 = c.sponge_in
            s = (self.x[i1] - self.x[:i1]) / (self.x[i1] - self.x[0])
            sx[:i1] = np.maximum(sx[:i1], c.sigma_max * s ** 3)
        if c.sponge_out > 0:
            i0 = nx - 1 - c.sponge_out
            s = (self.x[i0 + 1:] - self.x[i0]) / (self.x[-1] - self.x[i0])
            sx[i0 + 1:] = np.maximum(sx[i0 + 1:], c.sigma_max * s ** 3)
        if c.sponge_top > 0:
            j0 = ny - 1 - c.sponge_top
            s = (self.y[j0 + 1:] - self.y[j0]) / (self.y[-1] - self.y[j0])
            sy[j0 + 1:] = np.maximum(sy[j0 + 1:], c.sigma_max * s ** 3)
        return np.maximum(sx[None, None, :], sy[None, :, None])

    # axis of each direction in a [nz][ny][nx] field
    @staticmethod
    def axis(d):
        return (2, 1, 0)[d]

    def deriv(self, f, d):
        """Physical first derivative along direction d (0: x, 1: y, 2: z)."""
        ax = self.axis(d)
        op = cp.first_derivative if self.compact else st.first_derivative
        Df = op(f, ax, self.cfg.fd_order, periodic=(d == 2))
        sh = [1, 1, 1]
        sh[ax] = len(self.m[d])
        return Df * self.m[d].reshape(sh)


def primitives(Q, case):
    """Pointwise state from Q: rho, Y, u, e, T (nondim and K), p, transport, h_s, omega."""
    ref = case.ref
    ns, nd = case.ns, case.ndim
    P = {}
    if case.air5:
        rhos = Q[:ns]
        rho = np.sum(rhos, axis=0)
        Y = rhos / rho
    else:
        rho = Q[0]
        Y = None
    vel = [Q[ns + i] / rho for i in range(nd)]
    E = Q[ns + nd] / rho
    e = E - 0.5 * sum(u * u for u in vel)
    P.update(rho=rho, Y=Y, vel=vel, e=e)
    if case.gas == 2:
        # thermally perfect gas (module tpg): Newton for T, Eq. (22) for p, Eqs. (24-25)
        g = ref["gamma"]
        T, _, ok = tpg.temperature(e, ref["k0"], ref["th"], g)
        p = thermo.cpg_pressure(rho, T, g)
        Tk = T * ref["T_ref"]
        mu = transport.sutherland(Tk) / ref["mu_inf"]
        kap = tpg.keyes(Tk) / ref["kappa_inf"]
        # equilibrium sound speed: gamma(T) = c_p / c_v = 1 + ((g - 1)/g) / c_v(T)
        gT = 1.0 + ((g - 1.0) / g) / tpg.cv(T, ref["k0"], ref["th"], g)
        P.update(T=T, p=p, mu=mu, kappa=kap, c=np.sqrt(gT * p / rho),
                 status=np.where(ok, 0, 1))
        return P
    if not case.air5:
        g = ref["gamma"]
        T = thermo.cpg_temperature(e, g)
        p = thermo.cpg_pressure(rho, T, g)
        Tk = T * ref["T_ref"]
        mu = transport.sutherland(Tk) / ref["mu_inf"]
        P.update(T=T, p=p, mu=mu, kappa=mu, c=np.sqrt(g * p / rho), status=np.zeros(T.shape, int))
        return P
    c2 = ref["c_inf"] ** 2
    Tk, _, status = thermo.temperature_from_energy(e * c2, Y)
    T = Tk / ref["T_ref"]
    Rmix = thermo.mixture_R(Y)
    g = ref["gamma"]
    p = rho * T * (g - 1.0) / g * Rmix / ref["R_inf"]
    rho_d = rho * ref["rho_inf"]
    p_d = p * ref["rho_inf"] * c2
    mu, kap = transport.mixture_viscosity_conductivity(Tk, Y)
    D = transport.averaged_diffusion(Tk, p_d, Y)
    h = thermo.h_species(Tk) / c2
    X = transport.mole_fractions(Y)
    Mbar = 1.0 / np.sum(Y / sp.M.reshape(5, 1, 1, 1), axis=0)
    wdot = chemistry.production_rates(rhos * ref["rho_inf"], Tk) * ref["L_ref"] / (
        ref["rho_inf"] * ref["c_inf"])
    gam_f = thermo.frozen_gamma(Tk, Y)
    c = np.sqrt(gam_f * Rmix * Tk) / ref["c_inf"]
    P.update(T=T, Tk=Tk, p=p, mu=mu / ref["mu_inf"], kappa=kap / ref["kappa_inf"],
             D=D / (ref["c_inf"] * ref["L_ref"]), h=h, X=X, Mbar=Mbar, wdot=wdot, c=c,
             status=status, rho_d=rho_d)
    if getattr(case.cfg, "diffusion", 0) == 1:
        P["Dsr"] = transport.binary_diffusion(Tk, p_d) / (ref["c_inf"] * ref["L_ref"])
    return P


def velocity_gradients(P, case):
    nd = case.ndim
    return [[case.deriv(P["vel"][i], j) for j in range(nd)] for i in range(nd)]


def fluxes(Q, P, case, G, ad=None):
    """Total flux F_j = F_C,j - F_D,j for each direction j: list of [nvar] arrays."""
    ref = case.ref
    ns, nd = case.ns, case.ndim
    Re = ref["Re"]
    Pr = ref["Pr"]
    rho, vel, p = P["rho"], P["vel"], P["p"]
    theta = sum(G[i][i] for i in range(nd))
    mu_eff = P["mu"] / Re
    kap_eff = P["kappa"] / (Re * Pr)
    beta = 0.0
    if ad is not None:
        mu_eff = mu_eff + ad["mu"]
        kap_eff = kap_eff + ad["kappa"]
        beta = ad["beta"]
    dT = [case.deriv(P["T"], j) for j in range(nd)]
    if case.air5:
        Dtot = P["D"] if ad is None else P["D"] + ad["D"]
        dX = [[case.deriv(P["X"][s], j) for j in range(nd)] for s in range(ns)]
        # J_s,j = -rho (M_s/Mbar) D_s dX_s/dx_j + Y_s sum_i rho (M_i/Mbar) D_i dX_i/dx_j
        a = [rho * (sp.M[s] / P["Mbar"]) * Dtot[s] for s in range(ns)]
    out = []
    rhoE = Q[ns + nd]
    for j in range(nd):
        F = [None] * case.nvar
        # species (or density) rows
        if case.air5:
            if "Dsr" in P:
                # Stefan-Maxwell system, Eq. (17) (transport.stefan_maxwell_fluxes); the
                # artificial diffusivities, if any, add a flux of the form of Eq. (18)
                gX = np.stack([dX[s][j] for s in range(ns)])[:, None]
                Jsm = transport.stefan_maxwell_fluxes(rho, P["Y"], gX, P["Dsr"])
                J = [Jsm[s, 0] for s in range(ns)]
                if ad is not None:
                    aa = [rho * (sp.M[s] / P["Mbar"]) * ad["D"][s] for s in range(ns)]
                    ca = sum(aa[i] * dX[i][j] for i in range(ns))
                    J = [J[s] - aa[s] * dX[s][j] + P["Y"][s] * ca for s in range(ns)]
            else:
                corr = sum(a[i] * dX[i][j] for i in range(ns))
                J = [-a[s] * dX[s][j] + P["Y"][s] * corr for s in range(ns)]
            for s in range(ns):
                F[s] = Q[s] * vel[j] + J[s]
        else:
            F[0] = Q[0] * vel[j]
        # momentum rows
        tau = []
        for i in range(nd):
            t = mu_eff * (G[i][j] + G[j][i])
            if i == j:
                t = t - mu_eff * (2.0 / 3.0) * theta + beta * theta
            tau.append(t)
            conv = Q[ns + i] * vel[j] + (p if i == j else 0.0)
            F[ns + i] = conv - t
        # energy row
        q = -kap_eff * dT[j]
        if case.air5:
            q = q + sum(P["h"][s] * J[s] for s in range(ns))
        work = sum(tau[i] * vel[i] for i in range(nd))
        F[ns + nd] = (rhoE + p) * vel[j] - (work - q)
        out.append(F)
    return out


def rhs(Q, Q_ref, case, return_parts=False):
    """R = -sum_j d/dx_j F_j + S - sigma (Q - Q_ref) with the boundary rows of the module doc."""
    Q = np.asarray(Q, dtype=np.float64)
    nd, ns = case.ndim, case.ns
    P = primitives(Q, case)
    G = velocity_gradients(P, case)
    ad = None
    if case.cfg.ad:
        from . import ad as adm
        ad = adm.coefficients(P, G, case)
    F = fluxes(Q, P, case, G, ad)
    R = np.zeros_like(Q)
    for k in range(case.nvar):
        acc = 0.0
        for j in range(nd):
            acc = acc + case.deriv(F[j][k], j)
        R[k] = -acc
    if case.air5:
        R[:ns] = R[:ns] + P["wdot"]
    if Q_ref is not None:
        R = R - case.sigma[None] * (Q - Q_ref)
    apply_rhs_boundaries(R, case)
    if return_parts:
        return R, P, ad
    return R


def apply_rhs_boundaries(R, case):
    nd, ns = case.ndim, case.ns
    R[:, :, :, 0] = 0.0                      # inflow column held
    for i in range(nd):                      # no-slip wall: momentum held at zero
        R[ns + i][:, 0, :] = 0.0
    if case.hold is not None and len(case.hold):
        R.reshape(R.shape[0], -1)[:, case.hold] = 0.0


def wall_energy(rho, T, Y, case):
    """rho E at the wall from T (nondim) and Y with zero velocity."""
    ref = case.ref
    if case.gas == 2:
        return rho * tpg.energy(T, ref["k0"], ref["th"], ref["gamma"])
    if not case.air5:
        return rho * T / ref["gamma"]
    Tk = T * ref["T_ref"]
    e = thermo.mixture_e(Tk, Y) / ref["c_inf"] ** 2
    return rho * e


def apply_bc(Q, case):
    """Post-stage wall row update (module doc); points of the wall row that are held keep Q."""
    cfg = case.cfg
    nd, ns = case.ndim, case.ns
    ref = case.ref
    Qw = Q[:, :, 0, 1:]                      # [nvar][nz][nx-1], i >= 1
    rows = [Q[:, :, j, 1:] for j in range(1, 5)]
    if case.air5:
        rho_w = np.sum(Qw[:ns], axis=0)
        Yr = [r[:ns] / np.sum(r[:ns], axis=0) for r in rows]
        Yw = sum(c * y for c, y in zip(WALL_EXTRAP, Yr))
    else:
        rho_w = Qw[0].copy()
        Yw = None
    if cfg.wall == 1:
        Tw = np.full(rho_w.shape, cfg.T_wall / ref["T_ref"])
    else:
        Ts = []
        for r in rows:
            P = primitives(r[:, :, None, :], case)
            Ts.append(P["T"][:, 0, :])
        Tw = sum(c * t for c, t in zip(WALL_EXTRAP, Ts))
    new = np.empty_like(Qw)
    if case.air5:
        new[:ns] = rho_w[None] * Yw
    else:
        new[0] = rho_w
    new[ns:ns + nd] = 0.0
    new[ns + nd] = wall_energy(rho_w, Tw, Yw if case.air5 else None, case)
    if case.hold is not None and len(case.hold):
        nx, ny = cfg.nx, cfg.ny
        held = np.zeros((cfg.nz, nx), dtype=bool)
        k, rem = np.divmod(case.hold, nx * ny)
        j, i = np.divmod(rem, nx)
        held[k[j == 0], i[j == 0]] = True
        keep = held[:, 1:]
        new = np.where(keep[None], Qw, new)
    Q[:, :, 0, 1:] = new
    return Q


def rk_stage(Q, dQ, Q_ref, case, stage, dt, R=None):
    """One stage k of the configured scheme, then the wall update.

    Low-storage (2N) schemes: dQ <- A_k dQ + dt R(Q); Q <- Q + B_k dQ.
    Three-register TVD RK3: at k = 0 dQ <- Q (the step's initial state Q0); then
    Q <- a_k Q0 + b_k (Q + dt R(Q)).
    R, when given, is used instead of evaluating R(Q).
    """
    if R is None:
        R = rhs(Q, Q_ref, case)
    if case.cfg.rk == SSPRK3:
        k = stage % len(SSP_RK3)
        a, b = SSP_RK3[k]
        if k == 0:
            dQ[...] = Q
        Q[...] = a * dQ + b * (Q + dt * R)
    else:
        A, B = RK_SCHEMES[case.cfg.rk]
        k = stage % len(A)
        dQ[...] = A[k] * dQ + dt * R
        Q[...] = Q + B[k] * dQ
    apply_bc(Q, case)
    return Q, dQ
