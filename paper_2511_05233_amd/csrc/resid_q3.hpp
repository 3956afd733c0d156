// The k = 3 scheme (tricubic, 4 x 4 x 4 Gauss-Legendre nodes per voxel):
// residual and tangents of Eq. 43-47 and 50 with one wavefront per voxel,
// one lane per node n = a0 + 4 a1 + 16 a2 (x fastest).
//
// Sum factorisation on the collocated nodes.  Along axis d the nodes of a
// line are the four lanes that differ in the two bits of a_d (lane stride
// 1, 4, 16), so a line is gathered with four cross-lane reads:
//   * gradient at node a:   (2/h) sum_j D[a_d][j] psi_j      (D[i][j] = l_j'(xi_i))
//   * volume term of row a: (h/2)^3 w_b w_c (2/h) sum_q w_q D[q][a_d] F_d(q)
//     (b, c the other two indices of a), the transposed contraction of the
//     fluxes F_d gathered from the same four lanes;
//   * the face point of a line at side s (a_d = 0: xi = -1, a_d = 3: xi = +1)
//     is evaluated by the line's end lane: traces sum_j l_j(s) psi_j and
//     normal derivatives (2/h) sum_j l_j'(s) psi_j from the gathered values
//     on its own side and from the neighbour voxel's four line nodes in
//     memory on the other; its flux reaches the four lanes of the line with
//     weights (h/2)^2 w_b w_c l_{a_d}(s).
// The face flux is face_flux of resid_q1.hpp in the same canonical
// orientation (lower voxel first, the same operation sequence on both
// sides), so the two contributions of a face cancel in any sum over voxels.
// Penalty sigma/h with sigma = (k+1)^2 = 16 (DevParams::sig_h).
//
// The basis tables are computed at compile time from the Gauss-Legendre
// nodes by the Lagrange formulas.
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"
#include "dual.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"

namespace lsbdg {

struct Q3Basis {
  double w[4];          // Gauss-Legendre weights
  double D[4][4];       // D[i][j] = l_j'(xi_i)
  double E[2][4];       // E[s][j] = l_j(-1 or +1)
  double G[2][4];       // G[s][j] = l_j'(-1 or +1)
};

constexpr double kQ3x[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                            0.86113631159405257522};
constexpr double kQ3w[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                            0.34785484513745385737};

constexpr double q3_lag(int j, double x) {
  double p = 1.0;
  for (int m = 0; m < 4; ++m)
    if (m != j) p *= (x - kQ3x[m]) / (kQ3x[j] - kQ3x[m]);
  return p;
}

constexpr double q3_dlag(int j, double x) {
  double s = 0.0;
  for (int k = 0; k < 4; ++k) {
    if (k == j) continue;
    double p = 1.0 / (kQ3x[j] - kQ3x[k]);
    for (int m = 0; m < 4; ++m)
      if (m != j && m != k) p *= (x - kQ3x[m]) / (kQ3x[j] - kQ3x[m]);
    s += p;
  }
  return s;
}

constexpr Q3Basis make_q3_basis() {
  Q3Basis b{};
  for (int i = 0; i < 4; ++i) {
    b.w[i] = kQ3w[i];
    for (int j = 0; j < 4; ++j) b.D[i][j] = q3_dlag(j, kQ3x[i]);
  }
  for (int j = 0; j < 4; ++j) {
    b.E[0][j] = q3_lag(j, -1.0);
    b.E[1][j] = q3_lag(j, 1.0);
    b.G[0][j] = q3_dlag(j, -1.0);
    b.G[1][j] = q3_dlag(j, 1.0);
  }
  return b;
}

__constant__ Q3Basis kQ3 = make_q3_basis();

// sum_j c[j] v[j] with one fixed operation sequence (both sides of a face
// form a trace with it, so their copies agree bit for bit).
template <typename T>
__device__ __forceinline__ T dot4(double c0, double c1, double c2, double c3, const T* v) {
  return ((T(c0) * v[0] + T(c1) * v[1]) + T(c2) * v[2]) + T(c3) * v[3];
}

__device__ __forceinline__ float lane_read(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double lane_read(double v, int src) { return __shfl(v, src, 64); }
template <typename S>
__device__ __forceinline__ Dual<S> lane_read(Dual<S> v, int src) {
  return {__shfl(v.v, src, 64), __shfl(v.d, src, 64)};
}

// Rows of node n (lane) of voxel e; u: its nine unknowns.
template <typename S, typename N, int Mode>
__device__ __forceinline__ void q3_rows(const S* __restrict__ U, const S* __restrict__ V,
                                        const S* __restrict__ M, const uint8_t* __restrict__ phase,
                                        const DevParams& P, int64_t e, int n, int64_t FS, const N* u, N* r) {
  using T = N;
  const int ix = int(e % P.nx), iy = int((e / P.nx) % P.ny), iz = int(e / (int64_t(P.nx) * P.ny));
  const int ph = phase[e];
  const int a[3] = {n & 3, (n >> 2) & 3, n >> 4};
  const double h2 = P.two_h;
  const double wn = kQ3.w[a[0]] * kQ3.w[a[1]] * kQ3.w[a[2]];
  const T W3n = T(P.W3 * wn);
  // time rows W (eps_L c_i - m_i)/dt and the solid rows
  {
    const T eL = liquid_fraction(T(P.epsCBD[ph]), u[7], u[8], T(P.epsL_min));
    const T idt = T(P.inv_dt);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const T mi = (Mode == kResidual) ? T(M[i * FS + e * 64 + n]) : T(0);
      r[i] = W3n * (eL * u[i] - mi) * idt;
    }
    r[6] = T(0);
    const T m6 = (Mode == kResidual) ? T(M[6 * FS + e * 64 + n]) : T(0);
    const T m7 = (Mode == kResidual) ? T(M[7 * FS + e * 64 + n]) : T(0);
    r[7] = W3n * T(P.rhoM[0]) * (u[7] - m6) * idt;
    r[8] = W3n * T(P.rhoM[1]) * (u[8] - m7) * idt;
  }
  const T eLn = liquid_fraction(T(P.epsCBD[ph]), u[7], u[8], T(P.epsL_min));
  const T fN = transport_factor(u, eLn);
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    const int ad = a[d];
    const int st = d == 0 ? 1 : d == 1 ? 4 : 16;              // lane stride of a d-line
    const int base = n - ad * st;                               // lane of the line's first node
    const int b1 = a[d == 0 ? 1 : 0], b2 = a[d == 2 ? 1 : 2];   // the two other indices
    const double wt = kQ3.w[b1] * kQ3.w[b2];
    const bool end = (ad == 0 || ad == 3);
    const int s = ad == 3 ? 1 : 0;                              // side of this lane's face point
    // gradient along d at the node; traces and normal derivatives at the
    // line's end (used by the end lanes)
    T g[7], tr[9], nd[7];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      T l[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) l[j] = lane_read(u[f], base + j * st);
      tr[f] = dot4(kQ3.E[s][0], kQ3.E[s][1], kQ3.E[s][2], kQ3.E[s][3], l);
      if (f < 7) {
        g[f] = T(h2) * dot4(kQ3.D[ad][0], kQ3.D[ad][1], kQ3.D[ad][2], kQ3.D[ad][3], l);
        nd[f] = T(h2) * dot4(kQ3.G[s][0], kQ3.G[s][1], kQ3.G[s][2], kQ3.G[s][3], l);
      }
    }
    // volume term: the transposed line contraction of the fluxes
    {
      T Fd[7];
      axis_flux(P, fN, u, g, Fd);
      const T c = T(P.W3 * wt * h2);
#pragma unroll
      for (int f = 0; f < 7; ++f) {
        T acc = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += T(kQ3.w[q] * kQ3.D[q][ad]) * lane_read(Fd[f], base + q * st);
        r[f] += c * acc;
      }
    }
    // face points: the end lanes of the line evaluate theirs
    T q[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) q[f] = T(0);
    const int coord = d == 0 ? ix : d == 1 ? iy : iz;
    const int ncell = d == 0 ? P.nx : d == 1 ? P.ny : P.nz;
    const int64_t stride = d == 0 ? 1 : d == 1 ? int64_t(P.nx) : int64_t(P.nx) * P.ny;
    if (end) {
      const bool hi = s == 1;
      const int cn = coord + (hi ? 1 : -1);
      if (cn >= 0 && cn < ncell) {
        const int64_t e2 = e + (hi ? stride : -stride);
        const int ph2 = phase[e2];
        // the neighbour's line: same tangential indices, its trace at the
        // opposite side
        T tn[9], gn[7];
        {
          T l[4][9];
#pragma unroll
          for (int j = 0; j < 4; ++j)
            load_node<S, N, Mode, true>(U, V, M, FS, e2 * 64 + (base + j * st), l[j]);
          const int so = 1 - s;
#pragma unroll
          for (int f = 0; f < 9; ++f) {
            const T lf[4] = {l[0][f], l[1][f], l[2][f], l[3][f]};
            tn[f] = dot4(kQ3.E[so][0], kQ3.E[so][1], kQ3.E[so][2], kQ3.E[so][3], lf);
            if (f < 7) gn[f] = T(h2) * dot4(kQ3.G[so][0], kQ3.G[so][1], kQ3.G[so][2], kQ3.G[so][3], lf);
          }
        }
        T ta[9], tb[9], ga[7], gb[7];
#pragma unroll
        for (int f = 0; f < 9; ++f) {
          ta[f] = hi ? tr[f] : tn[f];
          tb[f] = hi ? tn[f] : tr[f];
          if (f < 7) {
            ga[f] = hi ? nd[f] : gn[f];
            gb[f] = hi ? gn[f] : nd[f];
          }
        }
        const int phA = hi ? ph : ph2, phB = hi ? ph2 : ph;
        T flux[7];
        face_flux(P, phA, phB, ta, tb, ga, gb, flux);
        const T side = hi ? T(1) : T(-1);
#pragma unroll
        for (int f = 0; f < 7; ++f) q[f] = side * flux[f];
      } else if (d == 0 && hi) {
        // separator face x = L_x: inward Li+ flux j_el/F and ionic current j_el
        q[0] = -T(P.jel) / T(P.F);
        q[6] = -T(P.jel);
      }
    }
    // distribution along the line: both end lanes' fluxes, weighted by this
    // node's basis function at the two ends
    const T c0 = T(P.W2 * wt * kQ3.E[0][ad]), c1 = T(P.W2 * wt * kQ3.E[1][ad]);
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      const T qlo = lane_read(q[f], base);
      const T qhi = lane_read(q[f], base + 3 * st);
      r[f] += c0 * qlo + c1 * qhi;
    }
  }
  if (P.react[ph] != 0.0) {
    T Sx[9];
    node_sources(P, ph, u, Sx);
#pragma unroll
    for (int f = 0; f < 9; ++f) r[f] -= W3n * Sx[f];
  }
}

// One wavefront per voxel, four voxels per workgroup (grid-stride over
// voxels; every lane of a wavefront shares its voxel, so the cross-lane
// reads always see the whole line).
template <typename S, typename N, int Mode>
__global__ void __launch_bounds__(256)
q3_kernel(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ M, S* __restrict__ Out,
          const uint8_t* __restrict__ phase, DevParams P) {
  const int n = threadIdx.x & 63;
  const int64_t FS = P.Ne * 64;
  for (int64_t e = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); e < P.Ne; e += int64_t(gridDim.x) * 4) {
    N u[9], r[9];
    load_node<S, N, Mode>(U, V, M, FS, e * 64 + n, u);
    q3_rows<S, N, Mode>(U, V, M, phase, P, e, n, FS, u, r);
    if constexpr (Mode == kResidual) {
#pragma unroll
      for (int f = 0; f < 9; ++f) Out[f * FS + e * 64 + n] = r[f];
    } else {
      constexpr int nout = (Mode == kJvpFull) ? 9 : 7;
#pragma unroll
      for (int f = 0; f < nout; ++f) {
        const bool on = (P.active >> (f < 7 ? f : 7)) & 1;
        Out[f * FS + e * 64 + n] = on ? deriv_of(r[f]) : S(0);
      }
    }
  }
}

}  // namespace lsbdg
