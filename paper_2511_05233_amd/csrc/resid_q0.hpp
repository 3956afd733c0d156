// The k = 0 scheme (piecewise-constant DG, the paper's production
// discretisation): one lane per voxel.
//
// With one node per voxel the traces on a face are the two cell values and
// every gradient inside a cell vanishes, so the volume term and the
// consistency part of the face flux drop out and Eq. 43-47 reduce to the
// seven-point finite-volume scheme of Eq. 48: the flux through a face is
// the interior penalty alone, sigma/h times the harmonic means of the
// coefficients times the jumps, with sigma = 1.  Quadrature: the nodal
// weight of a voxel is h^3, of a face h^2.  The face flux is face_flux of
// resid_q1.hpp with zero normal derivatives, in the same canonical
// orientation (lower voxel first).
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"
#include "dual.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"

namespace lsbdg {

// Rows of voxel e (residual: N = S; tangents: N = Dual<S>), written to Out.
template <typename S, typename N, int Mode>
__device__ __forceinline__ void q0_voxel(const S* __restrict__ U, const S* __restrict__ V,
                                         const S* __restrict__ M, S* __restrict__ Out,
                                         const uint8_t* __restrict__ phase, const DevParams& P, int64_t e) {
  using T = N;
  const int64_t FS = P.Ne;
  const int ix = int(e % P.nx), iy = int((e / P.nx) % P.ny), iz = int(e / (int64_t(P.nx) * P.ny));
  const int ph = phase[e];
  T u[9], r[9];
  load_node<S, N, Mode>(U, V, M, FS, e, u);
  // time rows W (eps_L c_i - m_i)/dt and the solid rows (the nodal index of
  // q1_mass_rows is the voxel itself: one node per voxel)
  {
    const T eL = liquid_fraction(T(P.epsCBD[ph]), u[7], u[8], T(P.epsL_min));
    const T W3 = T(P.W3), idt = T(P.inv_dt);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const T mi = (Mode == kResidual) ? T(M[i * FS + e]) : T(0);
      r[i] = W3 * (eL * u[i] - mi) * idt;
    }
    r[6] = T(0);
    const T m6 = (Mode == kResidual) ? T(M[6 * FS + e]) : T(0);
    const T m7 = (Mode == kResidual) ? T(M[7 * FS + e]) : T(0);
    r[7] = W3 * T(P.rhoM[0]) * (u[7] - m6) * idt;
    r[8] = W3 * T(P.rhoM[1]) * (u[8] - m7) * idt;
  }
  const T W2 = T(P.W2);
  T zero[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) zero[f] = T(0);
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    const int coord = d == 0 ? ix : d == 1 ? iy : iz;
    const int ncell = d == 0 ? P.nx : d == 1 ? P.ny : P.nz;
    const int64_t stride = d == 0 ? 1 : d == 1 ? int64_t(P.nx) : int64_t(P.nx) * P.ny;
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {                // s = 1: the voxel's high face along d
      const int cn = coord + (s ? 1 : -1);
      T q[7];
      if (cn >= 0 && cn < ncell) {
        const int64_t e2 = e + (s ? stride : -stride);
        T un[9];
        load_node<S, N, Mode, true>(U, V, M, FS, e2, un);
        const int ph2 = phase[e2];
        T flux[7];
        if (s)
          face_flux(P, ph, ph2, u, un, zero, zero, flux);
        else
          face_flux(P, ph2, ph, un, u, zero, zero, flux);
        const T side = s ? T(1) : T(-1);
#pragma unroll
        for (int f = 0; f < 7; ++f) q[f] = side * flux[f];
      } else {
#pragma unroll
        for (int f = 0; f < 7; ++f) q[f] = T(0);
        if (d == 0 && s == 1) {                  // separator face x = L_x
          q[0] = -T(P.jel) / T(P.F);
          q[6] = -T(P.jel);
        }
      }
#pragma unroll
      for (int f = 0; f < 7; ++f) r[f] += W2 * q[f];
    }
  }
  if (P.react[ph] != 0.0) {
    T Sx[9];
    node_sources(P, ph, u, Sx);
    const T W3 = T(P.W3);
#pragma unroll
    for (int f = 0; f < 9; ++f) r[f] -= W3 * Sx[f];
  }
  if constexpr (Mode == kResidual) {
#pragma unroll
    for (int f = 0; f < 9; ++f) Out[f * FS + e] = r[f];
  } else {
    constexpr int nout = (Mode == kJvpFull) ? 9 : 7;
#pragma unroll
    for (int f = 0; f < nout; ++f) {
      const bool on = (P.active >> (f < 7 ? f : 7)) & 1;
      Out[f * FS + e] = on ? deriv_of(r[f]) : S(0);
    }
  }
}

template <typename S, typename N, int Mode>
__global__ void __launch_bounds__(256)
q0_kernel(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ M, S* __restrict__ Out,
          const uint8_t* __restrict__ phase, DevParams P) {
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < P.Ne; e += int64_t(gridDim.x) * 256)
    q0_voxel<S, N, Mode>(U, V, M, Out, phase, P, e);
}

}  // namespace lsbdg
