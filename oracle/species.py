"""Species and mechanism data for 5-species air (oracle copy; test infrastructure only).

The paper computes species properties "using kinetic theory and statistical
mechanics" through its thermochemical library (Sec. 2.2.1) and names the mixture
N2, O2, N, O, NO (Sec. 4.1) but prints no species data or rate constants.  The
values below are the reading this oracle takes:

* rigid-rotor / harmonic-oscillator constants (theta_v, theta_r, symmetry number)
  from spectroscopic omega_e and B_e; ground electronic multiplet lumped into a
  degeneracy g_el; 0 K formation enthalpies of the JANAF tables;
* Lennard-Jones 12-6 parameters of Svehla (NASA TR R-132);
* Park's 5-species air mechanism (three dissociations with third-body partners and
  two Zeldovich exchanges), written in the third-body form of Eq. (14).
"""
import numpy as np

# SI 2019 exact constants.
K_B = 1.380649e-23          # J/K
H_PLANCK = 6.62607015e-34   # J s
N_A = 6.02214076e23         # 1/mol
R_U = K_B * N_A             # J/(mol K)
P_STD = 1.0e5               # Pa, standard-state pressure of the Gibbs energies

NAMES = ("N2", "O2", "NO", "N", "O")
NS = 5

M = np.array([28.0134e-3, 31.9988e-3, 30.0061e-3, 14.0067e-3, 15.9994e-3])   # kg/mol
THETA_V = np.array([3393.5, 2273.6, 2739.7, 0.0, 0.0])     # K, vibrational temperature
THETA_R = np.array([2.875, 2.080, 2.406, 0.0, 0.0])        # K, rotational temperature
SIGMA_SYM = np.array([2.0, 2.0, 1.0, 1.0, 1.0])            # rotational symmetry number
G_EL = np.array([1.0, 3.0, 4.0, 4.0, 9.0])                 # lumped electronic degeneracy
HF0 = np.array([0.0, 0.0, 89.775e3, 470.82e3, 246.79e3])   # J/mol, formation enthalpy at 0 K
DIATOMIC = np.array([1.0, 1.0, 1.0, 0.0, 0.0])             # 1: one rotational + one vibrational mode

LJ_SIGMA = np.array([3.798, 3.467, 3.492, 3.298, 3.050]) * 1e-10   # m
LJ_EPS = np.array([71.4, 106.7, 116.7, 71.4, 106.7])               # K (epsilon / k_B)

# Element composition (rows: species, columns: N, O), used by conservation pins.
ELEMENTS = np.array([[2, 0], [0, 2], [1, 1], [1, 0], [0, 1]], dtype=float)

# Mechanism in the form of Eq. (13)-(14): nu' (reactants), nu'' (products),
# Arrhenius C [cm^3 mol^-1 s^-1], n, theta_a [K], and third-body efficiencies Z
# (None where the reaction has no third body, i.e. the sum factor of Eq. (14) is 1).
#                 N2 O2 NO  N  O
REACTIONS = [
    dict(name="N2+M=2N+M", nu_f=[1, 0, 0, 0, 0], nu_b=[0, 0, 0, 2, 0],
         C=7.0e21, n=-1.6, theta=113200.0, Z=[1.0, 1.0, 1.0, 30.0 / 7.0, 30.0 / 7.0]),
    dict(name="O2+M=2O+M", nu_f=[0, 1, 0, 0, 0], nu_b=[0, 0, 0, 0, 2],
         C=2.0e21, n=-1.5, theta=59500.0, Z=[1.0, 1.0, 1.0, 5.0, 5.0]),
    dict(name="NO+M=N+O+M", nu_f=[0, 0, 1, 0, 0], nu_b=[0, 0, 0, 1, 1],
         C=5.0e15, n=0.0, theta=75500.0, Z=[1.0, 1.0, 22.0, 22.0, 22.0]),
    dict(name="N2+O=NO+N", nu_f=[1, 0, 0, 0, 1], nu_b=[0, 0, 1, 1, 0],
         C=6.4e17, n=-1.0, theta=38400.0, Z=None),
    dict(name="NO+O=O2+N", nu_f=[0, 0, 1, 0, 1], nu_b=[0, 1, 0, 1, 0],
         C=8.4e12, n=0.0, theta=19450.0, Z=None),
]

# The same mechanism with every collision partner written out (17 reactions):
# (reactant stoichiometry, product stoichiometry, C, n, theta).  Used only to pin
# the third-body form above against an independent partner-explicit sum.
EXPLICIT_17 = []
for _s, _C in zip(range(5), [7.0e21, 7.0e21, 7.0e21, 3.0e22, 3.0e22]):
    nf = [1, 0, 0, 0, 0]; nb = [0, 0, 0, 2, 0]
    nf[_s] += 1; nb[_s] += 1
    EXPLICIT_17.append((nf, nb, _C, -1.6, 113200.0))
for _s, _C in zip(range(5), [2.0e21, 2.0e21, 2.0e21, 1.0e22, 1.0e22]):
    nf = [0, 1, 0, 0, 0]; nb = [0, 0, 0, 0, 2]
    nf[_s] += 1; nb[_s] += 1
    EXPLICIT_17.append((nf, nb, _C, -1.5, 59500.0))
for _s, _C in zip(range(5), [5.0e15, 5.0e15, 1.1e17, 1.1e17, 1.1e17]):
    nf = [0, 0, 1, 0, 0]; nb = [0, 0, 0, 1, 1]
    nf[_s] += 1; nb[_s] += 1
    EXPLICIT_17.append((nf, nb, _C, 0.0, 75500.0))
EXPLICIT_17.append(([1, 0, 0, 0, 1], [0, 0, 1, 1, 0], 6.4e17, -1.0, 38400.0))
EXPLICIT_17.append(([0, 0, 1, 0, 1], [0, 1, 0, 1, 0], 8.4e12, 0.0, 19450.0))

# Calorically perfect gas (Sec. 2.2.2): Sutherland constants of Eq. (24).
SUTH_C1 = 1.458e-6      # kg m^-1 s^-1 K^-1/2
SUTH_TS = 110.4         # K
