// Model constants, parameter derivation and the device parameter block.
//
// Sources (arXiv 2511.05233): physical constants Sec. 2.2; parameters Tab. 5
// (solid and liquid phase) and Tab. 2 (cathode volume fractions); reaction
// scheme Tab. 3; equilibrium initial state Tab. InitialState; localisation
// Eq. 57; applied current App. C.  T = 298.15 K reproduces the printed
// equilibrium column of Tab. 5 (the text's 298 K does not).
#pragma once

#include <cmath>
#include <cstdint>

namespace lsbdg {

constexpr double kFaraday = 96485.332;   // C/mol
constexpr double kGas = 8.3145;          // J/(mol K)
constexpr double kCref = 1000.0;         // mol/m^3
constexpr double kEta = 7.76e-4;         // m^3/mol, viscosity exponent (Eq. 02)

// charge numbers of the six dissolved species and the eliminated anion
constexpr double kZ[6] = {1.0, 0.0, -2.0, -2.0, -2.0, -2.0};
constexpr double kZA = -1.0;

// Tab. 5, solid phase
constexpr double kKsp[2] = {0.006, 8e-15};
constexpr double kKC[2] = {120.0, 3e-3};
constexpr double kU0first[4] = {2.41, 2.32, 2.31, 1.985};
constexpr double kKEpaper[6] = {2.53e-6, 3.54e-8, 1.49e-10, 2.05e-7, 9.11e-10, 1.37e-15};
constexpr double kAV0 = 94.908e6;
constexpr double kRho[2] = {2070.4, 1659.0};
constexpr double kMolar[2] = {0.2565, 0.0459};
constexpr double kEpsS8init = 0.095;
constexpr double kEpsLi2Sinit = 2.77e-6;
constexpr double kPassA = 0.1392;
constexpr double kPassBh = 3.310;        // h
constexpr double kKEanode = 5e-3;
// Tab. 5, liquid phase (order Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-, anion)
constexpr double kD0paper[7] = {9.3e-10, 10.0e-10, 5.3e-10, 5.3e-10, 7.6e-10, 0.6e-10, 9.3e-10};
constexpr double kCLi0 = 1500.0;
// Tab. 2
constexpr double kXcathode = 0.168;
constexpr double kXsulfur = 0.0956;

// Equilibrium of Tab. InitialState, evaluated in its printed order.
struct Equilibrium {
  double c[6];     // Li+, S8(L), S8^2-, S6^2-, S4^2-, S^2-
  double dphi0;    // Phi_S - Phi_L
  double U0[6];    // U0_1..U0_4 as printed, U0_5 and U0_6 recomputed
};

inline Equilibrium equilibrium(double T) {
  Equilibrium q{};
  const double rtf = kGas * T / kFaraday;
  const double U1 = kU0first[0], U2 = kU0first[1], U3 = kU0first[2], U4 = kU0first[3];
  const double cLi = kCLi0;
  const double cS8 = kKsp[0] * kCref;
  const double cS = kKsp[1] * kCref * kCref * kCref / (cLi * cLi);
  const double dphi = U1 / 8.0 + U2 / 24.0 + U3 / 12.0 + 0.75 * U4 +
                      rtf * (std::log(cS8 / kCref) / 16.0 - 0.5 * std::log(cS / kCref));
  const double c8 = cS8 * std::exp(-2.0 * (dphi - U1) / rtf);
  const double c6 = kCref * std::pow(cS8 / kCref, 0.75) *
                    std::exp(-2.0 * (dphi - (0.75 * U1 + 0.25 * U2)) / rtf);
  const double c4 = kCref * std::pow(cS / kCref, 4.0) * std::exp(6.0 * (dphi - U4) / rtf);
  const double U5 = dphi - rtf * (0.5 * std::log(c8 / kCref) - std::log(c4 / kCref));
  const double U6 = dphi - rtf * (std::log(c4 / kCref) / 6.0 + 4.0 / 3.0 * std::log(cLi / kCref));
  q.c[0] = cLi; q.c[1] = cS8; q.c[2] = c8; q.c[3] = c6; q.c[4] = c4; q.c[5] = cS;
  q.dphi0 = dphi;
  q.U0[0] = U1; q.U0[1] = U2; q.U0[2] = U3; q.U0[3] = U4; q.U0[4] = U5; q.U0[5] = U6;
  return q;
}

// Per-voxel-phase quantities after the Eq. 57 localisation (index 0 = pore,
// 1 = structure).  Pore voxels hold no solid and carry no reactions.
struct PhaseTable {
  double epsCBD[2];
  double aV0[2];
  double s8ref[2];     // 1.2 * eps_S8,0 (localised)
  double pass[2];      // a exp(-b f_C) (localised)
  double react[2];     // 1 where reactions act
  double epsS8init[2];
  double epsLi2Sinit[2];
};

constexpr int32_t kAllFields = 0xff;

struct Conc6 {
  double c[6];
};
constexpr int32_t kSolidsBit = 0x80;

// Parameter block handed to every kernel by value.  All arithmetic that
// depends only on parameters is folded here on the host in double.
struct DevParams {
  double D0[7];
  double zDA[6];       // z_j (D0_j - D0_A): charge diffusion weights
  double wL[6];        // z_j (z_j D0_j - z_A D0_A): conductivity weights
  double kE[6];
  double kC[2];
  double sqrtK[2];
  double U0[6];
  double F, frt, frt2; // F, F/(RT), F/(2RT)
  double V;
  double inv_cref, c_min, epsL_min;
  double rhoM[2];
  double sig_h;        // sigma / h
  double sq3_h;        // sqrt(3)/h: Q1 line derivative
  double W3, W2;       // Q1 nodal volume weight (h/2)^3 and face weight (h/2)^2
  double jel;          // A/m^2
  double TH;           // regularisation factor at the evaluation time
  double inv_dt;
  double epsCBD[2], aV0[2], s8ref[2], pass[2], react[2];
  int32_t nx, ny, nz;
  // Unknowns taking part in a solve: bit f (f < 7) for the transported
  // fields, bit 7 for the solid fractions.  Inactive rows of a tangent are
  // zero and inactive solid fractions stay frozen (kAllFields: all active).
  int32_t active;
  int32_t np;          // nodes per voxel, (k + 1)^3
  double two_h;        // 2/h: d xi / dx
  int64_t Ne;
};

}  // namespace lsbdg
