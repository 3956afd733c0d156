// Vertex-based slope limiter of the Q1 scheme (Kuzmin's definition, as the
// paper's DG1 runs use it in App. B; the positivity-preserving p = 1 scheme
// its outlook asks for), on the conserved densities m_i = eps_L c_i of the
// six dissolved species:
//
//   * each voxel's mean of m_i (its eight nodal values, equal quadrature
//     weights) is kept;
//   * every mesh vertex is bounded by the largest and smallest voxel mean
//     around it;
//   * the voxel's deviation from its mean is scaled by the largest factor
//     alpha in [0, 1] that keeps the trilinear polynomial's eight corner
//     values within their vertices' bounds.
//
// A trilinear function lies between its corner values, so the limited
// nodal values lie within the means around the voxel: non-negative means
// give a non-negative state.  Phi_L and the solid fractions are untouched.
//
// Two passes, one thread per voxel: the means (limit_means_kernel), then
// the factors and the limited state (limit_apply_kernel), which reads the
// 3 x 3 x 3 means around its voxel and writes only its own nodes, so the
// state is limited in place.
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"
#include "pointwise.hpp"

namespace lsbdg {

// Values at the voxel's ends xi = +-1 of the two Gauss-node Lagrange
// functions: the node on the same side ((1 + sqrt 3) / 2) and the other
// one ((1 - sqrt 3) / 2).
constexpr double kEndNear = 1.3660254037844386;
constexpr double kEndFar = -0.3660254037844386;

// Liquid fraction of node k (phase ph), as the time term takes it.
__device__ __forceinline__ double limiter_eL(const double* __restrict__ U, int64_t FS, int64_t k, double epsCBD,
                                             double floor_) {
  return liquid_fraction(epsCBD, U[7 * FS + k], U[8 * FS + k], floor_);
}

// Mean of m_i over the eight nodes, summed in pairs ((0+1)+(2+3))+((4+5)+(6+7)).
__device__ __forceinline__ double mean8(const double* m) {
  return (((m[0] + m[1]) + (m[2] + m[3])) + ((m[4] + m[5]) + (m[6] + m[7]))) * 0.125;
}

__global__ void __launch_bounds__(256)
limit_means_kernel(const double* __restrict__ U, const uint8_t* __restrict__ phase, DevParams P,
                   double* __restrict__ mbar) {
  const int64_t Ne = P.Ne, FS = Ne * 8;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < Ne; e += int64_t(gridDim.x) * 256) {
    const double eC = P.epsCBD[phase[e]];
    double eL[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) eL[a] = limiter_eL(U, FS, e * 8 + a, eC, P.epsL_min);
#pragma unroll 1
    for (int i = 0; i < 6; ++i) {
      double m[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) m[a] = eL[a] * U[i * FS + e * 8 + a];
      mbar[i * Ne + e] = mean8(m);
    }
  }
}

// Corner values of the trilinear polynomial through m (node a = x + 2y + 4z
// bits; corner c likewise, bit 0 = the low end of the axis).
__device__ __forceinline__ void corner_values(const double* m, double* w) {
  double tx[8], ty[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {          // along x: corner bit 0 from nodes x = 0, 1
    const int cx = c & 1, r = c & 6;
    tx[c] = (cx ? kEndFar : kEndNear) * m[r] + (cx ? kEndNear : kEndFar) * m[r | 1];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {          // along y
    const int cy = (c >> 1) & 1, r = c & 5;
    ty[c] = (cy ? kEndFar : kEndNear) * tx[r] + (cy ? kEndNear : kEndFar) * tx[r | 2];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {          // along z
    const int cz = (c >> 2) & 1, r = c & 3;
    w[c] = (cz ? kEndFar : kEndNear) * ty[r] + (cz ? kEndNear : kEndFar) * ty[r | 4];
  }
}

__global__ void __launch_bounds__(256)
limit_apply_kernel(double* __restrict__ U, const uint8_t* __restrict__ phase, DevParams P,
                   const double* __restrict__ mbar, double* __restrict__ alpha_out) {
  const int64_t Ne = P.Ne, FS = Ne * 8;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < Ne; e += int64_t(gridDim.x) * 256) {
    const int ix = int(e % nx), iy = int((e / nx) % ny), iz = int(e / (int64_t(nx) * ny));
    const double eC = P.epsCBD[phase[e]];
    double eL[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) eL[a] = limiter_eL(U, FS, e * 8 + a, eC, P.epsL_min);
#pragma unroll 1
    for (int i = 0; i < 6; ++i) {
      // means of the 3 x 3 x 3 voxels around e (absent outside the mesh)
      double nb[27];
      bool in[27];
#pragma unroll
      for (int q = 0; q < 27; ++q) {
        const int jx = ix - 1 + q % 3, jy = iy - 1 + (q / 3) % 3, jz = iz - 1 + q / 9;
        in[q] = jx >= 0 && jx < nx && jy >= 0 && jy < ny && jz >= 0 && jz < nz;
        nb[q] = in[q] ? mbar[i * Ne + jx + int64_t(nx) * (jy + int64_t(ny) * jz)] : 0.0;
      }
      const double mb = nb[13];
      double m[8], w[8];
#pragma unroll
      for (int a = 0; a < 8; ++a) m[a] = eL[a] * U[i * FS + e * 8 + a];
      corner_values(m, w);
      double al = 1.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        double hi = mb, lo = mb;            // the voxel itself shares every corner
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int q = (cx + (s & 1)) + 3 * (cy + ((s >> 1) & 1)) + 9 * (cz + (s >> 2));
          if (in[q]) {
            hi = nb[q] > hi ? nb[q] : hi;
            lo = nb[q] < lo ? nb[q] : lo;
          }
        }
        const double d = w[c] - mb;
        const double r = d > 0.0 ? (hi - mb) / d : d < 0.0 ? (lo - mb) / d : 1.0;
        al = r < al ? r : al;
      }
#pragma unroll
      for (int a = 0; a < 8; ++a) U[i * FS + e * 8 + a] = (mb + al * (m[a] - mb)) / eL[a];
      if (alpha_out) alpha_out[i * Ne + e] = al;
    }
  }
}

}  // namespace lsbdg
