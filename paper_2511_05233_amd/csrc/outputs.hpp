// Battery outputs and conservation sums of a Q1 state (FP64).
//
// One grid-stride pass over the nodes accumulates, per node with nodal
// weight W = (h/2)^3 (Q1 Gauss-Legendre weights are 1):
//   0..8   the nine unknowns (volume means: Q1 weights are equal),
//   9      dissolved sulfur c_S = c_S^2- + 4 c_S4 + 6 c_S6 + 8 c_S8^2- + 8 c_S8,
//   10     sulfur atoms   W (eps_L (8 c_S8 + 8 c_S8^2- + 6 c_S6 + 4 c_S4 + c_S^2-)
//                            + 8 (rho/M)_S8 eps_S8 + (rho/M)_Li2S eps_Li2S),
//   11     lithium atoms  W (eps_L c_Li + 2 (rho/M)_Li2S eps_Li2S),
//   12     stored charge  W (2 eps_L sum of the polysulfide anions + 2 (rho/M)_Li2S eps_Li2S),
//   13     reaction current -W S_Phi,
//   14     the local cell voltage at the separator-face points.
// Cell voltage (App. A with the anode law Eq. 27): the lithium anode carries
// j_el by Butler-Volmer kinetics, which inverts in closed form to
// e^A = y = (q + sqrt(q^2 + 4 a_Li))/2 with q = j_el/(F k_E,Ano), so the
// local voltage is V - Phi_L - (2RT/F) ln y at each face point, averaged.
#pragma once

#include <hip/hip_runtime.h>

#include "krylov.hpp"
#include "model.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"

namespace lsbdg {

constexpr int kNumSums = 15;

__global__ void __launch_bounds__(256)
outputs_kernel(const double* __restrict__ U, const uint8_t* __restrict__ phase, DevParams P, double q_anode,
               double rtf2, double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc[kNumSums];
#pragma unroll
  for (int j = 0; j < kNumSums; ++j) acc[j] = 0.0;
  const int64_t FS = P.Ne * 8;
  const double W = P.W3;
  const double rm0 = P.rhoM[0], rm1 = P.rhoM[1];
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256) {
    const int64_t e = k >> 3;
    const int n = int(k & 7);
    const int ph = phase[e];
    double us[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      us[f] = U[f * FS + k];
      acc[f] += us[f];
    }
    acc[9] += us[5] + 4.0 * us[4] + 6.0 * us[3] + 8.0 * us[2] + 8.0 * us[1];
    const double eL = liquid_fraction(P.epsCBD[ph], us[7], us[8], P.epsL_min);
    acc[10] += W * (eL * (8.0 * us[1] + 8.0 * us[2] + 6.0 * us[3] + 4.0 * us[4] + us[5]) +
                    8.0 * rm0 * us[7] + rm1 * us[8]);
    acc[11] += W * (eL * us[0] + 2.0 * rm1 * us[8]);
    acc[12] += W * (2.0 * eL * (us[2] + us[3] + us[4] + us[5]) + 2.0 * rm1 * us[8]);
    if (P.react[ph] != 0.0) {
      double Sx[9];
      node_sources(P, ph, us, Sx);
      acc[13] -= W * Sx[6];
    }
    if ((n & 1) && int(e % P.nx) == P.nx - 1) {
      // face point x = L_x on this node's x-line: near node = this one
      const int64_t kp = k ^ 1;
      const double phi = kLam1 * us[6] + kLam0 * U[6 * FS + kp];
      const double cli = kLam1 * us[0] + kLam0 * U[kp];
      const double a = (cli > P.c_min ? cli : P.c_min) * P.inv_cref;
      const double y = 0.5 * (q_anode + sqrt(q_anode * q_anode + 4.0 * a));
      acc[14] += P.V - phi - rtf2 * log(y);
    }
  }
#pragma unroll
  for (int j = 0; j < kNumSums; ++j) {
    const double t = block_sum(acc[j], sh);
    if (threadIdx.x == 0) partial[j * int64_t(gridDim.x) + blockIdx.x] = t;
  }
}

// Sum of the block partials of outputs_kernel, one thread per sum, in block
// order (the order, and so the rounding, of the host sum of dg_outputs).
__global__ void __launch_bounds__(64)
outputs_finish_kernel(const double* __restrict__ partial, int nb, double* __restrict__ sums) {
  const int j = threadIdx.x;
  if (j >= kNumSums) return;
  double a = 0.0;
  for (int b = 0; b < nb; ++b) a += partial[int64_t(j) * nb + b];
  sums[j] = a;
}

// Relative difference sums for the H211b error: partial[0] = sum (a - b)^2,
// partial[gridDim] = sum a^2.
__global__ void __launch_bounds__(256)
diff_norm_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                 double* __restrict__ partial) {
  __shared__ double sh[4];
  double d2 = 0.0, a2 = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256) {
    const double d = a[k] - b[k];
    d2 += d * d;
    a2 += a[k] * a[k];
  }
  const double t0 = block_sum(d2, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t0;
  const double t1 = block_sum(a2, sh);
  if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = t1;
}

// Richardson extrapolation of the H211b step: out = 2 zF - zC.
__global__ void __launch_bounds__(256)
richardson_kernel(const double* __restrict__ zF, const double* __restrict__ zC, double* __restrict__ out,
                  int64_t n) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256)
    out[k] = 2.0 * zF[k] - zC[k];
}

}  // namespace lsbdg
