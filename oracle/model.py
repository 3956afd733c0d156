"""Constants, parameters, stoichiometry and initial state (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Sources in arXiv 2511.05233:
  * physical constants: Sec. 2.2 (after Eq. 01);
  * solid/cathode parameters: Tab. 5 (solid phase); liquid parameters:
    Tab. 5 (liquid phase);
  * cathode composition (volume fractions 0.168 and 0.0956): Tab. 2;
  * reaction scheme: Tab. 3;
  * analytical equilibrium initial state: Tab. InitialState (Eq. 55);
  * 3D localisation of the structure-related quantities: Eq. 57;
  * theoretical capacity, sulfur loading and current density: App. C.

Readings taken where the paper is silent or inconsistent:
  * T = 298.15 K.  The text says 298 K, but the equilibrium values printed
    in Tab. 5 are reproduced (to one unit in the last digit) only with
    298.15 K; U0_5 and U0_6 are recomputed from Tab. InitialState instead of
    taking their rounded printed values.
  * The solid is equipotential at V (the gauge of Sec. 2.10); Phi_S is not a
    field.  The separator face x = L_x receives the Li+ flux j_el/F and the
    ionic current j_el; all other faces are no-flux.
  * Voxel phases: pore voxels carry no solid, no carbon-binder and no
    reactions; structure voxels follow Eq. 57 with eps_struct = 1 - (pore
    fraction of the mask).
  * Synthetic workloads override the diffusivities D0 and the
    electrochemical rate constants k_E = i0 / F; all else is Tab. 5.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction as Fr

import numpy as np

# --- physical constants (Sec. 2.2) -----------------------------------------
F = 96485.332          # C/mol
R_GAS = 8.3145         # J/(mol K)
T_K = 298.15           # K (reading: see module docstring)
C_REF = 1000.0         # mol/m^3 (Sec. 2.4 and Sec. 2.5)
ETA_K = 7.76e-4        # m^3/mol, exponent of the viscosity law (Eq. 02)

# Species of the liquid phase, in state order, plus the eliminated anion.
LIQUID = ("Li+", "S8(L)", "S8^2-", "S6^2-", "S4^2-", "S^2-")
Z = np.array([1.0, 0.0, -2.0, -2.0, -2.0, -2.0])   # charge numbers
Z_ANION = -1.0

# --- Tab. 5, liquid phase: infinite-dilution diffusivities [m^2/s] ---------
# order (Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-, anion)
D0_PAPER = np.array([9.3e-10, 10.0e-10, 5.3e-10, 5.3e-10, 7.6e-10, 0.6e-10, 9.3e-10])
C_LI_0 = 1500.0        # initial Li+ concentration [mol/m^3]

# --- Tab. 5, solid phase ---------------------------------------------------
K_SP = np.array([0.006, 8e-15])                   # C1, C2 solubility products
K_C = np.array([120.0, 3e-3])                     # mol/(s m^3)
U0_PRINTED = np.array([2.41, 2.32, 2.31, 1.985])  # U0_1..U0_4 [V]
K_E_PAPER = np.array([2.53e-6, 3.54e-8, 1.49e-10, 2.05e-7, 9.11e-10, 1.37e-15])  # mol/(s m^2)
A_V0 = 94.908e6        # 1/m
RHO = np.array([2070.4, 1659.0])                  # S8(S), Li2S(S) [kg/m^3]
MOLAR = np.array([0.2565, 0.0459])                # S8(S), Li2S(S) [kg/mol]
EPS_S8_0 = 0.095
EPS_LI2S_0 = 2.77e-6
A_PASS = 0.1392
B_PASS_H = 3.310       # h
K_E_ANODE = 5e-3       # mol/(s m^2)
X_CATHODE = 0.168      # Tab. 2: cathode solids volume fraction
X_SULFUR = 0.0956      # Tab. 2: sulfur volume fraction
CUTOFF_V = 1.9         # V

# --- Tab. 3: Tradeoff Chemistry ---------------------------------------------
# Rows: Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-, S8(S), Li2S(S), e-(S).
# Columns: C1, C2, E1..E6.  Reactants negative, products positive.
SPECIES_ALL = LIQUID + ("S8(S)", "Li2S(S)", "e-")
REACTIONS = ("C1", "C2", "E1", "E2", "E3", "E4", "E5", "E6")
NU_EXACT = [[Fr(0)] * 8 for _ in range(9)]


def _set(col, **kw):
    names = {"Li": 0, "S8L": 1, "S8m": 2, "S6m": 3, "S4m": 4, "S2m": 5,
             "S8s": 6, "Li2S": 7, "e": 8}
    for k, v in kw.items():
        NU_EXACT[names[k]][col] = Fr(v)


_set(0, S8s=-1, S8L=1)                                  # S8(S) <-> S8(L)
_set(1, Li2S=-1, Li=2, S2m=1)                           # Li2S(S) <-> 2Li+ + S^2-
_set(2, S8L="-1/2", e=-1, S8m="1/2")                    # 1/2 S8 + e <-> 1/2 S8^2-
_set(3, S8m="-3/2", e=-1, S6m=2)                        # 3/2 S8^2- + e <-> 2 S6^2-
_set(4, S6m=-1, e=-1, S4m="3/2")                        # S6^2- + e <-> 3/2 S4^2-
_set(5, S4m="-1/6", e=-1, S2m="2/3")                    # 1/6 S4^2- + e <-> 2/3 S^2-
_set(6, S8m="-1/2", e=-1, S4m=1)                        # 1/2 S8^2- + e <-> S4^2-
_set(7, S4m="-1/6", Li="-4/3", e=-1, Li2S="2/3")        # 1/6 S4^2- + 4/3 Li+ + e <-> 2/3 Li2S
NU = np.array([[float(x) for x in row] for row in NU_EXACT])  # (9, 8)


def rt_over_f(T=T_K):
    return R_GAS * T / F


def equilibrium_state(T=T_K, c_li=C_LI_0):
    """Tab. InitialState evaluated top to bottom (thermodynamic equilibrium).

    Returns a dict with the six intrinsic concentrations, the anion, the
    equilibrium solid-liquid potential difference dPhi0 and the derived
    standard potentials U0_5, U0_6, plus the full U0 vector (6,).
    """
    rtf = R_GAS * T / F
    U1, U2, U3, U4 = U0_PRINTED
    c_s8 = K_SP[0] * C_REF
    c_s2 = K_SP[1] * C_REF ** 3 / c_li ** 2
    dphi0 = ((1.0 / 6.0) * (0.75 * U1 + 0.25 * U2) + U3 / 12.0 + 0.75 * U4
             + rtf * np.log((c_s8 / C_REF) ** (1.0 / 16.0) / (c_s2 / C_REF) ** 0.5))
    c_s8m = c_s8 * np.exp(-2.0 * (dphi0 - U1) / rtf)
    c_s6m = C_REF * (c_s8 / C_REF) ** 0.75 * np.exp(-2.0 * (dphi0 - (0.75 * U1 + 0.25 * U2)) / rtf)
    c_s4m = C_REF * (c_s2 / C_REF) ** 4 * np.exp(6.0 * (dphi0 - U4) / rtf)
    U5 = dphi0 - rtf * np.log((c_s8m / C_REF) ** 0.5 / (c_s4m / C_REF))
    U6 = dphi0 - rtf * np.log((c_s4m / C_REF) ** (1.0 / 6.0) * (c_li / C_REF) ** (4.0 / 3.0))
    conc = np.array([c_li, c_s8, c_s8m, c_s6m, c_s4m, c_s2])
    # anion from local electroneutrality (Sec. 2.7, item (i))
    c_anion = -np.dot(Z, conc) / Z_ANION
    return {
        "c": conc, "c_anion": c_anion, "dphi0": dphi0,
        "U5": U5, "U6": U6, "U0": np.array([U1, U2, U3, U4, U5, U6]),
    }


def theoretical_capacity():
    """c_theo = n_e F / M_S8 with n_e = 16 (App. C), in C/kg."""
    return 16.0 * F / MOLAR[0]


def smooth_step(t):
    """T_H(t) = (1 + tanh(6 (t - 1)))/2 with t in seconds (Eq. 56)."""
    return 0.5 * (1.0 + np.tanh(6.0 * (t - 1.0)))


@dataclasses.dataclass
class Problem:
    """A voxel cathode, its parameters and the DG order (oracle side)."""
    nx: int
    ny: int
    nz: int
    h: float
    k: int
    phase: np.ndarray                  # uint8, shape (nz, ny, nx); 1 = structure
    D0: np.ndarray = dataclasses.field(default_factory=lambda: D0_PAPER.copy())
    kE: np.ndarray = dataclasses.field(default_factory=lambda: K_E_PAPER.copy())
    f_C: float = 0.1                   # 1/h
    T: float = T_K
    sigma: float | None = None         # penalty factor; None -> default by order
    c_min: float = 1e-20               # activity clamp [mol/m^3]
    epsL_min: float = 1e-6
    use_TH: bool = True
    j_el: float | None = None          # override of the App. C current [A/m^2]
    eps_struct: float | None = None    # override of 1 - pore fraction

    def __post_init__(self):
        self.phase = np.asarray(self.phase, dtype=np.uint8).reshape(self.nz, self.ny, self.nx)
        eq = equilibrium_state(self.T)
        self.eq = eq
        self.U0 = eq["U0"]
        self.V = eq["dphi0"]            # solid potential gauge (Sec. 2.10)
        if self.sigma is None:
            self.sigma = 1.0 if self.k == 0 else float((self.k + 1) ** 2)
        ph = self.phase.reshape(-1).astype(np.float64)
        pore_frac = 1.0 - ph.mean()
        es = (1.0 - pore_frac) if self.eps_struct is None else self.eps_struct
        self.eps_struct_used = es
        struct = ph > 0
        # Eq. 57 localisation, applied to structure voxels only
        inv = 1.0 / es if es > 0 else 0.0
        self.epsCBD_e = np.where(struct, (X_CATHODE - X_SULFUR) * inv, 0.0)
        self.epsS8_0_e = np.where(struct, EPS_S8_0 * inv, 0.0)
        self.epsLi2S_0_e = np.where(struct, EPS_LI2S_0 * inv, 0.0)
        self.aV0_e = np.where(struct, A_V0 * inv, 0.0)
        self.pass_e = np.where(struct, A_PASS * np.exp(-B_PASS_H * self.f_C) * inv, 0.0)
        self.react_e = struct.astype(np.float64)   # reactions only in the structure
        # App. C: j_el = f_C c_theo m_A, m_A = rho_S8 * (sulfur volume per separator area)
        if self.j_el is None:
            vol_s8 = self.epsS8_0_e.sum() * self.h ** 3
            area = self.ny * self.nz * self.h ** 2
            m_A = RHO[0] * vol_s8 / area
            self.j_el = self.f_C / 3600.0 * theoretical_capacity() * m_A

    @property
    def n_elem(self):
        return self.nx * self.ny * self.nz

    @property
    def n_nodes(self):
        return (self.k + 1) ** 3

    def initial_concentrations(self):
        """Uniform intrinsic concentrations of Tab. InitialState."""
        return self.eq["c"].copy()
