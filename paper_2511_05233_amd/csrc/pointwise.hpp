// Pointwise constitutive laws and reaction sources on the device.
//
// Transport (Eq. 02-03 with Bruggeman, Sec. 2.3): every effective
// diffusivity is D_i = D0_i * f with the common factor
//     f = eps_L^(3/2) exp(-7.76e-4 c_S),   c_S = c_S^2- + 4c_S4 + 6c_S6 + 8c_S8^2- + 8c_S8,
// so the migration, charge-diffusion and conductivity coefficients of
// Tab. 4 are f times per-species constants (zDA, wL) and the concentrations.
// Reactions (Eq. 05-06, 18-24, Tab. 3) in exponential form:
//     chemical       r = sqrt(K) a_reac - a_prod / sqrt(K)
//     electrochem.   r = a_reac e^{-A} - a_prod e^{A},  A = F(V - Phi_L - U0)/(2RT)
// with ln a = ln(max(c, c_min)/c_ref) for dissolved species, 1 for solids.
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"

namespace lsbdg {

template <typename T>
__device__ __forceinline__ T clamp_lo(T x, T lo) { return x > lo ? x : lo; }

// Liquid fraction eps_L = 1 - eps_CBD - eps_S8 - eps_Li2S (Sec. 2.7 (ii)), floored.
template <typename T>
__device__ __forceinline__ T liquid_fraction(T epsCBD, T eS8, T eLi2S, T floor_) {
  return clamp_lo(T(1) - epsCBD - eS8 - eLi2S, floor_);
}

template <typename T>
__device__ __forceinline__ T sulfur_sum(const T* c) {
  return c[5] + T(4) * c[4] + T(6) * c[3] + T(8) * c[2] + T(8) * c[1];
}

// Bruggeman-viscosity factor f of the effective diffusivities.
template <typename T>
__device__ __forceinline__ T transport_factor(const T* c, T eL) {
  return eL * sqrt(eL) * exp(-T(kEta) * sulfur_sum(c));
}

// Harmonic mean of Eq. 45 with the guard a b > 0.
template <typename T>
__device__ __forceinline__ T harm(T a, T b) {
  return (a * b > T(0)) ? T(2) * a * b / (a + b) : T(0);
}

// Volumetric sources at a node of a reactive voxel.
//   S[0..5]: dissolved species, S[6]: charge (S_Phi), S[7..8]: solids.
template <typename T>
__device__ __forceinline__ void node_sources(const DevParams& P, int ph, const T* u, T* S) {
  const T inv_cref = T(P.inv_cref), cmin = T(P.c_min);
  T la[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) la[m] = log(clamp_lo(u[m], cmin) * inv_cref);
  const T TH = T(P.TH);
  const T r0 = T(P.sqrtK[0]) - exp(la[1]) / T(P.sqrtK[0]);
  const T r1 = (T(P.sqrtK[1]) - exp(T(2) * la[0] + la[5]) / T(P.sqrtK[1])) * TH;
  // ln activities of reactants / products of E1..E6 (Tab. 3)
  const T lr[6] = {T(0.5) * la[1], T(1.5) * la[2], la[3], la[4] / T(6), T(0.5) * la[2],
                   la[4] / T(6) + T(4) / T(3) * la[0]};
  const T lp[6] = {T(0.5) * la[2], T(2) * la[3], T(1.5) * la[4], T(2) / T(3) * la[5], la[4], T(0)};
  const T base = T(P.frt2) * (T(P.V) - u[6]);
  T sE[6];
  // specific surface, Eq. 18 with Eq. 57 localisation
  const T x1 = clamp_lo(u[7], T(0)) / T(P.s8ref[ph]);
  const T x2 = clamp_lo(u[8], T(0)) / T(P.pass[ph]);
  const T aV = T(P.aV0[ph]) * clamp_lo(T(1) - x1 * sqrt(x1) - x2 * sqrt(x2), T(0));
  T sumE = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T A = base - T(P.frt2) * T(P.U0[k]);
    T r = exp(lr[k] - A) - exp(lp[k] + A);
    if (k == 3) r *= TH;
    sE[k] = aV * T(P.kE[k]) * r;
    sumE += sE[k];
  }
  const T vC0 = u[7] * T(P.kC[0]) * r0;
  const T vC1 = u[8] * T(P.kC[1]) * r1;
  const T t6 = T(1) / T(6), t3 = T(1) / T(3);
  S[0] = T(2) * vC1 - T(4) * t3 * sE[5];
  S[1] = vC0 - T(0.5) * sE[0];
  S[2] = T(0.5) * sE[0] - T(1.5) * sE[1] - T(0.5) * sE[4];
  S[3] = T(2) * sE[1] - sE[2];
  S[4] = T(1.5) * sE[2] - t6 * sE[3] + sE[4] - t6 * sE[5];
  S[5] = vC1 + T(2) * t3 * sE[3];
  S[6] = -T(P.F) * sumE;
  S[7] = -vC0;
  S[8] = -vC1 + T(2) * t3 * sE[5];
}

}  // namespace lsbdg
