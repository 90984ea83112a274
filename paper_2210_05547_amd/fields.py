"""Seeded synthetic inputs: workload configurations, grids and initial fields.

This module is the only code that both the library's callers (tests, benchmark)
and the CPU checker use.  It holds no arithmetic of the method itself: it builds
coordinates, a conserved-variable field Q of the right shape and value ranges, the
unperturbed reference field Q_ref, a time step and random thermochemical states.
The internal energy it puts into Q comes from a deliberately crude energy model of
its own (frozen translational + rotational heat capacity, no vibration, plus 0 K
formation enthalpies); the temperature that the thermodynamic model later recovers
from that energy is therefore close to, not equal to, the nominal profile below.

Workloads follow the paper's cases (Sec. 4.1 flat plates, Table 1/2; Sec. 4.2 SBLI
at M = 5.92, Table 3; Sec. 4.3 jet in crossflow, Tables 4/5), adapted in grid size,
dimension and Mach number.  Grid stretching in y is the paper's cubic-plus-linear
mapping of Eq. (27) or a tanh clustering.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

# --- crude energy model of the generator (not the thermodynamic model of the method)
_RU = 8.314462618
_M = np.array([28.0134e-3, 31.9988e-3, 30.0061e-3, 14.0067e-3, 15.9994e-3])
_HF = np.array([0.0, 0.0, 89.775e3, 470.82e3, 246.79e3]) / _M
_CV_RT = np.array([2.5, 2.5, 2.5, 1.5, 1.5])
Y_AIR = np.array([0.767082, 0.232918, 0.0, 0.0, 0.0])
Y_DISS = np.array([0.733743, 0.02, 0.05, 0.01, 0.186257])
SPECIES = ("N2", "O2", "NO", "N", "O")

GAS_CPG = 0
GAS_AIR5 = 1
GAS_TPG = 2      # thermally perfect single-species air
WALL_ADIABATIC = 0
WALL_ISOTHERMAL = 1


@dataclass
class FlowConfig:
    """One workload: geometry, free stream, wall, numerics and input recipe."""
    name: str
    gas: int
    nx: int
    ny: int
    nz: int = 1
    x0: float = 14.0
    x1: float = 86.0
    y0: float = 0.0
    y1: float = 1.6
    z0: float = 0.0
    z1: float = 5.0
    stretch: str = "cubic"        # 'cubic' (Eq. 27) or 'tanh'
    kappa_y: float = 0.15
    beta: float = 3.0
    mach: float = 6.0
    T_inf: float = 220.0          # K
    p_inf: float = 3596.0         # Pa (air5)
    gamma: float = 1.4            # CPG and TPG
    Pr: float = 0.72              # CPG only
    Re: float = 1.0e5
    L_ref: float = 0.0            # m; > 0 overrides Re for air5
    wall: int = WALL_ADIABATIC
    T_wall: float = 0.0           # K (isothermal)
    Y_inf: tuple = tuple(Y_AIR)
    sponge_in: int = 0            # points
    sponge_out: int = 0
    sponge_top: int = 0
    sigma_max: float = 2.0
    ad: bool = False
    diffusion: int = 0            # 0: Ramshaw (Eq. 18), 1: Stefan-Maxwell (Eq. 17)
    ad_coef: tuple = (0.002, 1.75, 0.01, 0.01, 100.0)   # C_mu, C_beta, C_kappa, C_D, C_Y
    fd_order: int = 6
    fd_scheme: int = 0            # 0: explicit central differences, 1: compact (Pade)
    rk: int = 0                   # 0: 2N-RK3, 1: 2N-RK4(3)5, 2: three-register TVD RK3
    cfl: float = 0.5
    noise: float = 1e-4
    species_noise: float = 0.0
    delta0: float = 0.15          # boundary-layer thickness at x0 (nondim)
    shock_deflection_deg: float = 0.0
    shock_x_imp: float = 0.0
    jet: bool = False
    jet_x: float = 52.5
    jet_z: float = 2.5
    jet_radius_cells: float = 8.0
    inflow_noise: float = 0.0     # u' / U_inf (3-D)
    stages: int = 100
    seed: int = 20221011

    @property
    def ns(self):
        return 5 if self.gas == GAS_AIR5 else 1

    @property
    def ndim(self):
        return 3 if self.nz > 1 else 2

    @property
    def nvar(self):
        base = 5 if self.gas == GAS_AIR5 else 1
        return base + self.ndim + 1

    @property
    def npts(self):
        return self.nx * self.ny * self.nz

    def scaled(self, nx, ny, nz=None, **kw):
        """Same workload on a smaller grid (sponge extents scaled with it)."""
        nz = self.nz if nz is None else nz
        fx, fy = nx / self.nx, ny / self.ny
        return dataclasses.replace(
            self, nx=nx, ny=ny, nz=nz,
            sponge_in=max(0, int(round(self.sponge_in * fx))) if self.sponge_in else 0,
            sponge_out=max(0, int(round(self.sponge_out * fx))) if self.sponge_out else 0,
            sponge_top=max(0, int(round(self.sponge_top * fy))) if self.sponge_top else 0,
            jet_radius_cells=max(3.0, self.jet_radius_cells * fx),
            **kw)


def _cfg_c1():
    return FlowConfig(name="flatplate_cpg_m6_128x64", gas=GAS_CPG, nx=128, ny=64,
                      x0=14.0, x1=86.0, y0=0.0, y1=1.6, stretch="tanh", beta=3.0,
                      mach=6.0, T_inf=220.0, gamma=1.4, Pr=0.72, Re=1.0e5,
                      wall=WALL_ADIABATIC, sponge_out=13, sponge_top=6, stages=100,
                      seed=20221011 + 1)


def _cfg_c2():
    return FlowConfig(name="flatplate_air5_m10_512x256", gas=GAS_AIR5, nx=512, ny=256,
                      x0=14.0, x1=86.0, y0=0.0, y1=1.6, stretch="cubic", kappa_y=0.15,
                      mach=10.0, T_inf=350.0, p_inf=3596.0, Re=1.0e5,
                      wall=WALL_ISOTHERMAL, T_wall=1500.0, sponge_in=36, sponge_out=107,
                      sponge_top=32, species_noise=1e-3, seed=20221011 + 2)


def _cfg_c3():
    return FlowConfig(name="sbli_air5_m5.92_2048x512", gas=GAS_AIR5, nx=2048, ny=512,
                      x0=19.0, x1=254.0, y0=0.0, y1=36.0, stretch="cubic", kappa_y=0.15,
                      mach=5.92, T_inf=1110.5, p_inf=60967.0, Re=1631.8,
                      wall=WALL_ADIABATIC, sponge_in=40, sponge_out=80, sponge_top=48,
                      ad=True, delta0=1.0, shock_deflection_deg=12.0, shock_x_imp=119.05,
                      species_noise=1e-3, cfl=0.25, seed=20221011 + 3,
                      # a weaker sponge (2 or 10) lets a mode at the corner of the held
                      # inflow column and the top boundary grow until the energy there
                      # drops below e(50 K) after about 300 stages
                      sigma_max=50.0)


def _cfg_c4():
    return FlowConfig(name="jisc_air5_m8_512x256x128", gas=GAS_AIR5, nx=512, ny=256, nz=128,
                      x0=38.5, x1=71.0, y0=0.0, y1=10.0, z0=0.0, z1=5.0, stretch="cubic",
                      kappa_y=0.15, mach=8.0, T_inf=947.0, p_inf=49800.0, Re=25291.0,
                      wall=WALL_ISOTHERMAL, T_wall=4000.0, sponge_in=16, sponge_out=32,
                      sponge_top=10, ad=True, delta0=0.8, jet=True, jet_x=52.5, jet_z=2.5,
                      jet_radius_cells=8.0, inflow_noise=0.05, species_noise=1e-3, cfl=0.1,
                      seed=20221011 + 4)


def _cfg_c1t():
    """The c1 flat plate as a thermally perfect gas (Sec. 2.2.2): its adiabatic wall
    reaches about 1600 K, where the vibrational specific heat matters."""
    return dataclasses.replace(_cfg_c1(), name="flatplate_tpg_m6_128x64", gas=GAS_TPG,
                               seed=20221011 + 5)


def _cfg_c3t():
    """The SBLI as a thermally perfect gas (Sec. 4.2 runs both gas models on it)."""
    return dataclasses.replace(_cfg_c3(), name="sbli_tpg_m5.92_2048x512", gas=GAS_TPG,
                               species_noise=0.0, cfl=0.1, seed=20221011 + 6)


CONFIGS = {"c1": _cfg_c1, "c2": _cfg_c2, "c3": _cfg_c3, "c4": _cfg_c4, "c1t": _cfg_c1t,
           "c3t": _cfg_c3t}


def get_config(key: str) -> FlowConfig:
    return CONFIGS[key]()


# --------------------------------------------------------------------------- grids
def grid(cfg: FlowConfig):
    """Separable coordinates (x[nx], y[ny], z[nz]); z is periodic and uniform."""
    x = np.linspace(cfg.x0, cfg.x1, cfg.nx)
    eta = np.linspace(0.0, 1.0, cfg.ny)
    if cfg.stretch == "tanh":
        y = cfg.y0 + (cfg.y1 - cfg.y0) * (1.0 - np.tanh(cfg.beta * (1.0 - eta)) / math.tanh(cfg.beta))
    else:  # Eq. (27): cubic plus linear mapping of the index
        y = cfg.y0 + (cfg.y1 - cfg.y0) * ((1.0 - cfg.kappa_y) * eta ** 3 + cfg.kappa_y * eta)
    if cfg.nz > 1:
        z = cfg.z0 + (cfg.z1 - cfg.z0) * np.arange(cfg.nz) / cfg.nz
    else:
        z = np.zeros(1)
    return x, y, z


# --------------------------------------------------------------------------- fields
def _crude_energy(T, Y):
    """Generator energy model [J/kg]: sum_s Y_s (c_s R_s T + h_f,s), no vibration."""
    Rs = _RU / _M
    sh = (5,) + (1,) * (np.ndim(T))
    return np.sum(Y * (_CV_RT.reshape(sh) * Rs.reshape(sh) * T + _HF.reshape(sh)), axis=0)


def _smooth121(a, axis, periodic):
    if periodic:
        return 0.25 * np.roll(a, 1, axis) + 0.5 * a + 0.25 * np.roll(a, -1, axis)
    b = a.copy()
    sl = [slice(None)] * a.ndim
    def s(i0, i1):
        t = list(sl); t[axis] = slice(i0, i1); return tuple(t)
    b[s(1, -1)] = 0.25 * a[s(0, -2)] + 0.5 * a[s(1, -1)] + 0.25 * a[s(2, None)]
    return b


def initial_field(cfg: FlowConfig):
    """Return (Q, Q_ref, info): nondimensional conserved variables, layout [nvar][nz][ny][nx].

    Q = [rho (CPG) | rho_1..rho_5 (air5), rho u, rho v, (rho w), rho E].  Q_ref is the
    unperturbed field.  info holds the nominal primitive fields and the time step.
    """
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    x, y, z = grid(cfg)
    Z3, Y3, X3 = np.meshgrid(z, y, x, indexing="ij")          # [nz][ny][nx]
    g = cfg.gamma if cfg.gas != GAS_AIR5 else 1.4
    Pr = cfg.Pr if cfg.gas != GAS_AIR5 else 0.72
    M = cfg.mach
    Tinf = cfg.T_inf
    # boundary-layer velocity and Crocco-Busemann temperature (nominal, K)
    delta = cfg.delta0 * np.sqrt(X3 / cfg.x0)
    uh = np.tanh(3.0 * (Y3 - cfg.y0) / delta)
    Taw = Tinf * (1.0 + math.sqrt(Pr) * 0.5 * (g - 1.0) * M * M)
    Tw = Taw if cfg.wall == WALL_ADIABATIC else cfg.T_wall
    T = Tw + (Taw - Tw) * uh - (Taw - Tinf) * uh * uh
    p = np.ones_like(T)                      # p / p_inf
    u = M * uh                               # u / c_inf (nominal c_inf)
    v = np.zeros_like(T)
    w = np.zeros_like(T)
    rho_fac = np.ones_like(T)                # density factor on top of p/T
    # oblique shock impinging at x_imp (SBLI-shaped field)
    if cfg.shock_deflection_deg > 0.0:
        th = math.radians(cfg.shock_deflection_deg)
        b = _shock_angle(M, th, g)
        Mn = M * math.sin(b)
        p21 = 1.0 + 2.0 * g / (g + 1.0) * (Mn * Mn - 1.0)
        r21 = (g + 1.0) * Mn * Mn / ((g - 1.0) * Mn * Mn + 2.0)
        xs = cfg.shock_x_imp - (Y3 - cfg.y0) / math.tan(b)
        dx = (cfg.x1 - cfg.x0) / (cfg.nx - 1)
        s = 0.5 * (1.0 + np.tanh((X3 - xs) / (2.0 * dx)))
        p = p * (1.0 + (p21 - 1.0) * s)
        rho_fac = rho_fac * (1.0 + (r21 - 1.0) * s) / (1.0 + (p21 - 1.0) * s)
        # velocity turned towards the wall behind the shock, speed reduced (nominal)
        Vt = 1.0 - (1.0 - math.cos(th) * (1.0 - (1.0 - 1.0 / r21) * math.sin(b) ** 2)) * s
        vdir = -math.tan(th) * s * (1.0 - np.exp(-((Y3 - cfg.y0) / delta) ** 2))
        v = u * Vt * vdir
        u = u * Vt
    if cfg.gas == GAS_AIR5:
        Yinf = np.asarray(cfg.Y_inf)
        phi = np.clip((T - 2000.0) / 4000.0, 0.0, 1.0)
        Ys = (1.0 - phi)[None] * Yinf.reshape(5, 1, 1, 1) + phi[None] * Y_DISS.reshape(5, 1, 1, 1)
    else:
        Ys = np.ones((1,) + T.shape)
    # jet patch (pure N2, sonic, p_j = 10 p_inf, T_j = T_inf) on the first 3 wall rows
    hold = None
    if cfg.jet:
        hx = (cfg.x1 - cfg.x0) / (cfg.nx - 1)
        dxi = (X3 - cfg.jet_x) / hx
        dzi = (Z3 - cfg.jet_z) / hx          # distances in units of the x spacing
        r2 = (dxi ** 2 + dzi ** 2) / cfg.jet_radius_cells ** 2
        wxz = np.exp(-r2)
        wxz[wxz < 1e-3] = 0.0
        # full jet state on the first 3 wall rows (held), decaying smoothly above them
        jidx = np.arange(cfg.ny).reshape(1, -1, 1)
        yj = (Y3 - Y3[:, 2:3, :])[:1]          # height above the last held row
        gy = np.where(jidx < 3, 1.0, np.exp(-(yj / 0.3) ** 2))
        wj = wxz * gy
        jrow = np.zeros_like(T)
        jrow[:, :3, :] = 1.0
        Yj = np.array([1.0, 0, 0, 0, 0]).reshape(5, 1, 1, 1)
        Ys = (1.0 - wj)[None] * Ys + wj[None] * Yj
        T = (1.0 - wj) * T + wj * Tinf
        p = (1.0 - wj) * p + wj * 10.0
        cj = math.sqrt(1.4 * (_RU / _M[0]) * Tinf)
        cinf = math.sqrt(g * (_RU / _molar_mass(np.asarray(cfg.Y_inf))) * Tinf)
        v = (1.0 - wj) * v + wj * (cj / cinf)
        u = (1.0 - wj) * u
        hold = np.flatnonzero((wxz * jrow).reshape(-1) > 0.0).astype(np.int64)
    # assemble nondimensional conserved variables (one species: the generator's energy
    # model is the calorically perfect one for the thermally perfect gas too)
    if cfg.gas != GAS_AIR5:
        rho = p / (T / Tinf) * rho_fac
        e = (T / Tinf) / (g * (g - 1.0))            # nominal e / c_inf^2
        rhos = rho[None]
    else:
        Yinf = np.asarray(cfg.Y_inf)
        Minf = _molar_mass(Yinf)
        Mmix = _molar_mass(Ys)
        rho = p * (Tinf / T) * (Mmix / Minf) * rho_fac
        cinf2 = g * (_RU / Minf) * Tinf
        e = _crude_energy(T, Ys) / cinf2
        rhos = rho[None] * Ys
    vel = [u, v] + ([w] if cfg.ndim == 3 else [])
    E = e + 0.5 * sum(c * c for c in vel)
    Qref = np.concatenate([rhos] + [(rho * c)[None] for c in vel] + [(rho * E)[None]], axis=0)
    Qref = np.ascontiguousarray(Qref, dtype=np.float64)
    # perturbations
    Q = Qref.copy()
    nsp = rhos.shape[0]
    if cfg.species_noise > 0.0 and cfg.gas == GAS_AIR5:
        Yp = Ys + rng.uniform(-cfg.species_noise, cfg.species_noise, Ys.shape)
        Yp = np.maximum(Yp, 0.0)
        Yp = Yp / np.sum(Yp, axis=0)
        Q[:nsp] = rho[None] * Yp
    if cfg.inflow_noise > 0.0 and cfg.ndim == 3:
        # wall-normal envelope, and a ramp that keeps the inflow column and its closures
        # free of perturbations
        fac = (1.0 - np.exp(-(Y3 - cfg.y0) / delta)) * (1.0 - np.exp(-((X3 - cfg.x0) / 1.5) ** 2))
        for k in range(3):
            n = rng.standard_normal(T.shape)
            for _ in range(4):
                n = _smooth121(n, 2, False)
                n = _smooth121(n, 1, False)
                n = _smooth121(n, 0, True)
            n = n / np.std(n)
            du = cfg.inflow_noise * M * n * fac
            uk = Q[nsp + k] / rho
            # keep the internal energy: add the kinetic-energy change to rho E
            Q[-1] = Q[-1] + rho * (uk * du + 0.5 * du * du)
            Q[nsp + k] = Q[nsp + k] + rho * du
    if cfg.noise > 0.0:
        Q = Q * (1.0 + cfg.noise * rng.standard_normal(Q.shape))
    # no-slip wall: zero momentum at j = 0 (both fields), except on the jet inlet
    wall = np.ones(T.shape, dtype=bool)
    wall[:, 1:, :] = False
    if hold is not None:
        wall.reshape(-1)[hold] = False
    for k in range(cfg.ndim):
        Q[nsp + k][wall] = 0.0
        Qref[nsp + k][wall] = 0.0
    if hold is not None:
        Q.reshape(Q.shape[0], -1)[:, hold] = Qref.reshape(Q.shape[0], -1)[:, hold]
    # time step: acoustic CFL on the nominal field (c ~ sqrt(T/T_inf) in units of c_inf)
    dx = np.min(np.diff(x))
    dy = np.min(np.diff(y))
    dmin = min(dx, dy) if cfg.ndim == 2 else min(dx, dy, (cfg.z1 - cfg.z0) / cfg.nz)
    smax = float(np.max(np.sqrt(sum(c * c for c in vel)) + np.sqrt(T / Tinf)))
    dt = cfg.cfl * dmin / smax
    info = dict(x=x, y=y, z=z, T_nominal=T, dt=dt, hold=hold)
    return np.ascontiguousarray(Q), Qref, info


def _molar_mass(Y):
    Y = np.asarray(Y)
    sh = (5,) + (1,) * (Y.ndim - 1)
    return 1.0 / np.sum(Y / _M.reshape(sh), axis=0)


def _shock_angle(M, theta, g):
    """Weak oblique-shock angle for deflection theta (theta-beta-M relation, bisection)."""
    lo, hi = math.asin(1.0 / M) + 1e-9, math.pi / 2 * 0.9
    def f(b):
        return math.atan(2.0 / math.tan(b) * (M * M * math.sin(b) ** 2 - 1.0)
                         / (M * M * (g + math.cos(2 * b)) + 2.0)) - theta
    # find the maximum-deflection angle region: the weak root is below it
    bs = np.linspace(lo, hi, 2000)
    fs = np.array([f(b) for b in bs])
    i = int(np.argmax(fs > 0))
    a, c = bs[i - 1], bs[i]
    for _ in range(100):
        m = 0.5 * (a + c)
        if f(m) > 0:
            c = m
        else:
            a = m
    return 0.5 * (a + c)


# --------------------------------------------------------------- pointwise states
def thermo_states(n, seed=7, T_range=(200.0, 8000.0), logrho_range=(-4.0, 0.0)):
    """Random SI states for the pointwise calls.

    Returns (rho [kg/m3], T [K], Y [5][n], e [J/kg]) with T ~ U(T_range),
    rho ~ 10^U(logrho_range), Y ~ Dirichlet(1,1,1,1,1); e is the generator's crude
    energy at (T, Y), so the temperature a thermodynamic model recovers from it lies
    near, not at, T.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(T_range[0], T_range[1], n)
    rho = 10.0 ** rng.uniform(logrho_range[0], logrho_range[1], n)
    Y = np.ascontiguousarray(rng.dirichlet(np.ones(5), n).T)
    return rho, T, Y, _crude_energy(T, Y)


def air_compositions(n, rng, xi_range=(0.70, 0.83)):
    """Air mass fractions [5][n] at every dissociation degree (surrogate training set).

    The mass fraction of the element N is xi_N ~ U(xi_range) (air: 0.767); a share of
    the elements is bound in NO (up to half of what the scarcer element allows, density
    rising towards zero); the rest of each element splits between its molecule and its
    atom with an atomic share ~ U(0, 1).
    """
    xiN = rng.uniform(xi_range[0], xi_range[1], n)
    xiO = 1.0 - xiN
    fN, fO = _M[3] / _M[2], _M[4] / _M[2]     # element mass shares of NO
    no_max = np.minimum(xiN / fN, xiO / fO)
    yNO = rng.uniform(0.0, 1.0, n) ** 2 * 0.5 * no_max
    remN, remO = xiN - fN * yNO, xiO - fO * yNO
    aN, aO = rng.uniform(0.0, 1.0, n), rng.uniform(0.0, 1.0, n)
    Y = np.stack([remN * (1.0 - aN), remO * (1.0 - aO), yNO, remN * aN, remO * aO])
    return np.ascontiguousarray(Y / Y.sum(0))


def air_states(n, seed, T_range=(200.0, 8000.0), logrho_range=(-4.0, 0.0)):
    """Random SI air states (rho [kg/m3], T [K], Y [5][n], e [J/kg]): T ~ U(T_range),
    rho ~ 10^U(logrho_range), Y from air_compositions; e is the generator's crude energy
    at (T, Y) (a thermodynamic model recovers a temperature near, not at, T)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(T_range[0], T_range[1], n)
    rho = 10.0 ** rng.uniform(logrho_range[0], logrho_range[1], n)
    Y = air_compositions(n, rng)
    return rho, T, Y, _crude_energy(T, Y)
