"""Plain FP64 CPU oracle for the reacting-flow right-hand side and Runge-Kutta stage.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` do.  It shares no code, tables or constants
with the HIP library: every constant below is typed here independently.  Its only
shared dependency is the seeded input generator ``paper_2210_05547_amd.fields``,
which holds none of the method's arithmetic.

Module map (each function cites the passage of the paper it follows):

* ``species``     species and mechanism data (5-species air), physical constants
* ``thermo``      RRHO species thermodynamics, mixture sums (Eq. 12), CPG (Eq. 22),
                  Newton energy -> temperature inversion (Sec. 3.4)
* ``transport``   Sutherland (Eq. 24), Chapman-Enskog/Wilke/Eucken mixture transport,
                  averaged diffusion coefficient (Eq. 19)
* ``chemistry``   Arrhenius rates and net production (Eqs. 13-15)
* ``refstate``    reference state and nondimensional numbers (Eqs. 7, 11)
* ``stencils``    explicit central first-derivative operators (Sec. 3.1 reading),
                  fourth difference and Gaussian filter (Sec. 3.3 reading)
* ``ad``          artificial-diffusivity coefficients (Sec. 3.3 reading)
* ``rhs``         F(Q) of Eqs. (5)-(6) with the sponge of Eq. (26), boundary rows and
                  the low-storage Runge-Kutta stages (Sec. 3.1)
* ``mlp``         FP64 reference of the surrogate network, its gradient and Adam
* ``equilibrium`` law-of-mass-action equilibrium (mpmath), used only as a pin

Pins (tests/test_oracle_*.py) tie each module to something other than itself:
printed constants, closed-form flows, exact rational stencil identities, 50-digit
bisection, Gibbs-Helmholtz, detailed balance at an independently solved
equilibrium, RK stability polynomials and convergence order, finite-difference
gradients, closed forms of the artificial-diffusivity coefficients on a uniform grid
(their formulas are a reading of Sec. 3.3, which prints none).  Parity unpinned
(checked only through properties, not values): the absolute values of the
Chapman-Enskog transport model beyond its pure-species/binary limits and a handbook
plausibility check (Sec. 2.2.1 names the library that computes them but prints no
model).
"""
