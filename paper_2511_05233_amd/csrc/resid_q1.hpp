// Q1 (trilinear, 2x2x2 Gauss-Legendre nodes) DG residual on gfx950.
//
// Work decomposition: one lane per DG node, eight consecutive lanes per
// voxel (lane & 7 = node index n = a0 + 2 a1 + 4 a2).  Along axis d the two
// nodes of a line differ in bit d of n, so every line partner is the lane
// n ^ (1 << d) of the same 8-lane group and line gradients, traces and the
// two-node face distribution are single cross-lane swizzles.
//
// Q1 facts used (nodes at xi = -+1/sqrt(3), weights 1):
//   line derivative  d/dx = sqrt(3)/h (u_1 - u_0) at both nodes of the line;
//   trace at the near face = lam1 u_near + lam0 u_far,
//   lam1 = (1 + sqrt(3))/2, lam0 = (1 - sqrt(3))/2;
//   grad phi_a . e_d at either node of a's d-line = sqrt(3)/h sgn(a_d).
// Each lane evaluates the single face point on its own normal line at its
// own side of the voxel, so the 8 lanes cover the 6 faces x 4 points.
//
// Residual rows (Eq. 43-47, 50): see include/lsbdg.h.  Face flux seen from
// the element with outward normal n = s e_d:
//   q = -1/2 s (F^- + F^+)_d + sigma/h [ {D}_H (c^- - c^+) + {M}_H (Phi^- - Phi^+) ]
// with every coefficient taken from the traced state on its own side.
// Because D_i = D0_i f, M_i = z_i F/RT D0_i f c_i, K_j = z_j F (D0_j - D0_A) f
// and kappa = F^2/RT f sum_j wL_j c_j, the harmonic means factor as
// D0_i H(f^-, f^+), z_i F/RT D0_i H(f^- c^-, f^+ c^+), etc.
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"
#include "dual.hpp"
#include "pointwise.hpp"

namespace lsbdg {

constexpr double kSqrt3 = 1.7320508075688772;
constexpr double kLam1 = 0.5 * (1.0 + kSqrt3);
constexpr double kLam0 = 0.5 * (1.0 - kSqrt3);

// XCD-aware block order: the grid is a multiple of 8 blocks; hardware
// dispatches block b to XCD b % 8, so each XCD receives a contiguous range
// of voxels and their face neighbours hit that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t nblocks_padded) {
  const int64_t b = blockIdx.x;
  const int64_t per = nblocks_padded / 8;
  return (b % 8) * per + b / 8;
}

template <typename T>
__device__ __forceinline__ T xlane(T v, int mask) { return __shfl_xor(v, mask); }

// Trace at the near face of a Q1 line, lam1 u_near + lam0 u_far, with one
// explicitly fused rounding: both elements of a face form every trace with
// the same operation sequence, so their copies agree bit for bit.
__device__ __forceinline__ double face_trace(double near, double far) {
  return __builtin_fma(kLam1, near, kLam0 * far);
}
__device__ __forceinline__ float face_trace(float near, float far) {
  return __builtin_fmaf(float(kLam1), near, float(kLam0) * far);
}
template <typename S>
__device__ __forceinline__ Dual<S> face_trace(Dual<S> near, Dual<S> far) {
  return {face_trace(near.v, far.v), face_trace(near.d, far.d)};
}
template <typename S>
__device__ __forceinline__ Dual<S> xlane(Dual<S> v, int mask) {
  return {__shfl_xor(v.v, mask), __shfl_xor(v.d, mask)};
}

// Volume flux components (species 0..5 and charge) along one axis at a node
// with transport factor f, nodal state u and line gradients g[0..6].
template <typename T>
__device__ __forceinline__ void axis_flux(const DevParams& P, T f, const T* u, const T* g, T* out) {
  const T frt = T(P.frt);
  T lam = T(0), sdiff = T(0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    out[j] = T(P.D0[j]) * f * (g[j] + T(kZ[j]) * frt * u[j] * g[6]);
    lam += T(P.wL[j]) * u[j];
    sdiff += T(P.zDA[j]) * g[j];
  }
  out[6] = f * T(P.F) * (sdiff + frt * lam * g[6]);
}

// Operator modes of the Q1 kernel.
// kJvpCondensed reads the solid-fraction tangent coefficients C of every
// node it touches from the linearisation array (see solid_tangent_kernel).
enum Q1Mode { kResidual = 0, kJvpFull = 1, kJvpCondensed = 2 };

// Node-local elimination of the solid fractions for a direction v on the
// transported fields: the solid rows W ((rho/M)(eps - m)/dt - S_eps) have
// tangent zero when  A w = dS_eps/du v,  A = diag(rho/M)/dt - dS_eps/deps.
// Returns w (the solid-fraction tangents).  Non-reactive voxels give w = 0.
template <typename S>
__device__ __forceinline__ void condense_solids(const DevParams& P, int ph, const S* us, const S* v7,
                                                S& w0, S& w1) {
  w0 = S(0);
  w1 = S(0);
  if (P.react[ph] == 0.0 || !(P.active & kSolidsBit)) return;
  using D = Dual<S>;
  D x[9], Sx[9];
#pragma unroll
  for (int f = 0; f < 7; ++f) x[f] = D(us[f], v7[f]);
  x[7] = D(us[7], S(0));
  x[8] = D(us[8], S(0));
  node_sources(P, ph, x, Sx);
  const S t7 = Sx[7].d, t8 = Sx[8].d;
#pragma unroll
  for (int f = 0; f < 7; ++f) x[f].d = S(0);
  x[7].d = S(1);
  node_sources(P, ph, x, Sx);
  const S c70 = Sx[7].d, c80 = Sx[8].d;
  x[7].d = S(0);
  x[8].d = S(1);
  node_sources(P, ph, x, Sx);
  const S c71 = Sx[7].d, c81 = Sx[8].d;
  const S idt = S(P.inv_dt);
  const S a00 = S(P.rhoM[0]) * idt - c70, a01 = -c71;
  const S a10 = -c80, a11 = S(P.rhoM[1]) * idt - c81;
  const S det = a00 * a11 - a01 * a10;
  w0 = (a11 * t7 - a01 * t8) / det;
  w1 = (a00 * t8 - a10 * t7) / det;
}

// Solid-fraction tangent of one node for the transported-field direction v,
// w = C v with the node's 2 x 7 coefficients C.  Stored as 14 field-major
// arrays: Cw[j] = C[0][j] and Cw[7 + j] = C[0][j] + C[1][j] (j < 7), so that
// the tangent of eps_S8 + eps_Li2S -- all a face neighbour's solid fractions
// enter through, via the liquid fraction -- costs seven loads.
template <typename S>
__device__ __forceinline__ S solid_tangent_row(const S* __restrict__ Cw, int row, int64_t FS, int64_t idx,
                                               const S* v7) {
  S a = S(0);
#pragma unroll
  for (int j = 0; j < 7; ++j) a += Cw[(row * 7 + j) * FS + idx] * v7[j];
  return a;
}

// Per-node coefficients C of the condensation (condense_solids applied to
// the seven unit directions); nodes without reactions, or with frozen solid
// fractions, get C = 0.  Once per linearisation point; every condensed
// tangent at that point then costs at most two 7-term products per node.
template <typename S>
__device__ __forceinline__ void solid_tangent_node(const S* __restrict__ U, S* __restrict__ Cw, int ph,
                                                   const DevParams& P, int64_t k, int64_t FS) {
  if (P.react[ph] == 0.0 || !(P.active & kSolidsBit)) {
#pragma unroll
    for (int j = 0; j < 14; ++j) Cw[j * FS + k] = S(0);
    return;
  }
  using D = Dual<S>;
  D x[9], Sx[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) x[f] = D(U[f * FS + k], S(0));
  x[7].d = S(1);
  node_sources(P, ph, x, Sx);
  const S c70 = Sx[7].d, c80 = Sx[8].d;
  x[7].d = S(0);
  x[8].d = S(1);
  node_sources(P, ph, x, Sx);
  const S c71 = Sx[7].d, c81 = Sx[8].d;
  x[8].d = S(0);
  const S idt = S(P.inv_dt);
  const S a00 = S(P.rhoM[0]) * idt - c70, a01 = -c71;
  const S a10 = -c80, a11 = S(P.rhoM[1]) * idt - c81;
  const S det = a00 * a11 - a01 * a10;
#pragma unroll 1
  for (int j = 0; j < 7; ++j) {
    x[j].d = S(1);
    node_sources(P, ph, x, Sx);
    x[j].d = S(0);
    const S t7 = Sx[7].d, t8 = Sx[8].d;
    const S w0 = (a11 * t7 - a01 * t8) / det;
    const S w1 = (a00 * t8 - a10 * t7) / det;
    Cw[j * FS + k] = w0;
    Cw[(7 + j) * FS + k] = w0 + w1;
  }
}

template <typename S>
__global__ void __launch_bounds__(256)
solid_tangent_kernel(const S* __restrict__ U, S* __restrict__ Cw, const uint8_t* __restrict__ phase,
                     DevParams P) {
  const int64_t FS = P.Ne * P.np;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256)
    solid_tangent_node(U, Cw, int(phase[k / P.np]), P, k, FS);
}

// Load the nine unknowns of one node as operator numbers (Cw: the
// linearisation coefficients, read in kJvpCondensed only).  kFace: a face
// neighbour, whose solid fractions enter through their sum only (the
// tangent of eps_S8 carries that sum, eps_Li2S none).
template <typename S, typename N, int Mode, bool kFace = false>
__device__ __forceinline__ void load_node(const S* __restrict__ U, const S* __restrict__ V,
                                          const S* __restrict__ Cw, int64_t FS, int64_t idx, N* x) {
  if constexpr (Mode == kResidual) {
#pragma unroll
    for (int f = 0; f < 9; ++f) x[f] = U[f * FS + idx];
  } else if constexpr (Mode == kJvpFull) {
#pragma unroll
    for (int f = 0; f < 9; ++f) x[f] = N(U[f * FS + idx], V[f * FS + idx]);
  } else {
    S vs[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) vs[f] = V[f * FS + idx];
    const S ws = solid_tangent_row(Cw, 1, FS, idx, vs);
    S w0 = ws, w1 = S(0);
    if constexpr (!kFace) {
      w0 = solid_tangent_row(Cw, 0, FS, idx, vs);
      w1 = ws - w0;
    }
#pragma unroll
    for (int f = 0; f < 7; ++f) x[f] = N(U[f * FS + idx], vs[f]);
    x[7] = N(U[7 * FS + idx], w0);
    x[8] = N(U[8 * FS + idx], w1);
  }
}

// Face flux from the lower element A to the upper element B at one face
// point (outward normal +e_d of A), Eq. 45-47: traces ta, tb (9 fields) and
// normal derivatives ga, gb (7 fields) of both sides; every coefficient is
// taken from the traced state of its own side and averaged harmonically.
template <typename T>
__device__ __forceinline__ void face_flux(const DevParams& P, int phA, int phB, const T* ta, const T* tb,
                                          const T* ga, const T* gb, T* flux) {
  const T sigh = T(P.sig_h);
  const T fa = transport_factor(ta, liquid_fraction(T(P.epsCBD[phA]), ta[7], ta[8], T(P.epsL_min)));
  const T fb = transport_factor(tb, liquid_fraction(T(P.epsCBD[phB]), tb[7], tb[8], T(P.epsL_min)));
  const T Hf = harm(fa, fb);
  const T frt = T(P.frt);
  const T dphi = ta[6] - tb[6];
  T lama = T(0), lamb = T(0), sda = T(0), sdb = T(0), pen6 = T(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T D0 = T(P.D0[i]);
    const T z = T(kZ[i]);
    const T Fa = fa * (ga[i] + z * frt * ta[i] * ga[6]);
    const T Fb = fb * (gb[i] + z * frt * tb[i] * gb[6]);
    flux[i] = -T(0.5) * D0 * (Fa + Fb) +
              sigh * D0 * (Hf * (ta[i] - tb[i]) + z * frt * harm(fa * ta[i], fb * tb[i]) * dphi);
    lama += T(P.wL[i]) * ta[i];
    lamb += T(P.wL[i]) * tb[i];
    sda += T(P.zDA[i]) * ga[i];
    sdb += T(P.zDA[i]) * gb[i];
    pen6 += T(P.zDA[i]) * (ta[i] - tb[i]);
  }
  const T Fq = T(P.F);
  const T Ga = fa * Fq * (sda + frt * lama * ga[6]);
  const T Gb = fb * Fq * (sdb + frt * lamb * gb[6]);
  flux[6] = -T(0.5) * (Ga + Gb) + sigh * Fq * (Hf * pen6 + frt * harm(fa * lama, fb * lamb) * dphi);
}

// Time (mass) rows of node n: W (eps_L c_i - m_i)/dt, W (rho/M)_s (eps_s -
// m_{6+s})/dt (the old mass m enters the residual only), charge row 0.
template <typename S, typename N, int Mode>
__device__ __forceinline__ void q1_mass_rows(const S* __restrict__ M, const DevParams& P, int64_t e, int n,
                                             int ph, int64_t FS, const N* u, N* r) {
  using T = N;
  const T eL = liquid_fraction(T(P.epsCBD[ph]), u[7], u[8], T(P.epsL_min));
  const T W3 = T(P.W3);
  const T idt = T(P.inv_dt);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T mi = (Mode == kResidual) ? T(M[i * FS + e * 8 + n]) : T(0);
    r[i] = W3 * (eL * u[i] - mi) * idt;
  }
  r[6] = T(0);
  const T m6 = (Mode == kResidual) ? T(M[6 * FS + e * 8 + n]) : T(0);
  const T m7 = (Mode == kResidual) ? T(M[7 * FS + e * 8 + n]) : T(0);
  r[7] = W3 * T(P.rhoM[0]) * (u[7] - m6) * idt;
  r[8] = W3 * T(P.rhoM[1]) * (u[8] - m7) * idt;
}

// Volume and face terms along axis d of node n's rows (fields 0..6), added
// to r; fN is the transport factor at the node.  Neighbour nodes are read
// from U (and from V in the JVP modes); with kNbrZero their direction is
// zero (element-diagonal Jacobian blocks).
template <typename S, typename N, int Mode, bool kNbrZero>
__device__ __forceinline__ void q1_axis(const S* __restrict__ U, const S* __restrict__ V,
                                        const S* __restrict__ M, const uint8_t* __restrict__ phase,
                                        const DevParams& P, int64_t e, int n, int ph, int ix, int iy, int iz,
                                        int64_t FS, const N* u, const N& fN, int d, N* r) {
  using T = N;
  const T W3 = T(P.W3), W2 = T(P.W2), sq3h = T(P.sq3_h);
  const T lam1 = T(kLam1), lam0 = T(kLam0);
  const int coord = d == 0 ? ix : d == 1 ? iy : iz;
  const int ncell = d == 0 ? P.nx : d == 1 ? P.ny : P.nz;
  const int64_t stride = d == 0 ? 1 : d == 1 ? int64_t(P.nx) : int64_t(P.nx) * P.ny;

  const int mask = 1 << d;
  const bool hi = (n & mask) != 0;
  const T sgn = hi ? T(1) : T(-1);
  T up[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) up[f] = xlane(u[f], mask);
  T g[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) g[f] = sq3h * (hi ? u[f] - up[f] : up[f] - u[f]);

  // the face neighbour's two nodes on this lane's line, loaded before the
  // volume term so the loads overlap it (at a boundary the lane's own
  // voxel stands in: loaded, never used)
  const int cn = coord + (hi ? 1 : -1);
  const bool inside = cn >= 0 && cn < ncell;
  const int64_t e2 = inside ? e + (hi ? stride : -stride) : e;
  T vn[9], vf[9];
  {
    const int64_t in_ = e2 * 8 + (n ^ mask), if_ = e2 * 8 + n;   // nearest the face, far side
    if constexpr (kNbrZero) {
#pragma unroll
      for (int f = 0; f < 9; ++f) {
        vn[f] = T(U[f * FS + in_]);
        vf[f] = T(U[f * FS + if_]);
      }
    } else {
      load_node<S, N, Mode, true>(U, V, M, FS, in_, vn);
      load_node<S, N, Mode, true>(U, V, M, FS, if_, vf);
    }
  }
  const int ph2 = phase[e2];

  // volume term along d: sqrt(3)/h sgn(a_d) W3 (F_d(a) + F_d(a'))
  {
    T Fd[7];
    axis_flux(P, fN, u, g, Fd);
#pragma unroll
    for (int f = 0; f < 7; ++f) r[f] += sq3h * sgn * W3 * (Fd[f] + xlane(Fd[f], mask));
  }

  // face point on this lane's line at its own side s = sgn
  T q[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) q[f] = T(0);
  if (inside) {
    // Canonical orientation: A = the lower element of the face (outward
    // normal +e_d), B = the upper one.  Both elements evaluate the flux
    // from A to B with the same operation sequence on the same operands
    // and take +-1 times it, so a face's two contributions cancel exactly
    // in any sum over elements (discrete conservation to the last bit).
    T ta[9], tb[9], ga[7], gb[7];
    {
#pragma unroll
      for (int f = 0; f < 9; ++f) {
        const T tm = face_trace(u[f], up[f]);
        const T tp = face_trace(vn[f], vf[f]);
        ta[f] = hi ? tm : tp;
        tb[f] = hi ? tp : tm;
        if (f < 7) {
          const T gp = sq3h * (hi ? vf[f] - vn[f] : vn[f] - vf[f]);
          ga[f] = hi ? g[f] : gp;
          gb[f] = hi ? gp : g[f];
        }
      }
    }
    const int phA = hi ? ph : ph2, phB = hi ? ph2 : ph;
    const T side = hi ? T(1) : T(-1);          // +flux for A, -flux for B
    T flux[7];
    face_flux(P, phA, phB, ta, tb, ga, gb, flux);
#pragma unroll
    for (int f = 0; f < 7; ++f) q[f] = side * flux[f];
  } else if (d == 0 && hi) {
    // separator face x = L_x: inward Li+ flux j_el/F and ionic current j_el
    q[0] = -T(P.jel) / T(P.F);
    q[6] = -T(P.jel);
  }
#pragma unroll
  for (int f = 0; f < 7; ++f) r[f] += W2 * (lam1 * q[f] + lam0 * xlane(q[f], mask));
}

// Rows of the Q1 operator at one node (lane): residual rows (N = S) or their
// tangents (N = Dual<S>).  u holds the lane's own nine unknowns as N.
template <typename S, typename N, int Mode, bool kNbrZero, bool kSources = true>
__device__ __forceinline__ void q1_rows(const S* __restrict__ U, const S* __restrict__ V,
                                        const S* __restrict__ M, const uint8_t* __restrict__ phase,
                                        const DevParams& P, int64_t e, int n, int ph, int ix, int iy,
                                        int iz, int64_t FS, const N* u, N* r) {
  using T = N;
  const T W3 = T(P.W3);
  q1_mass_rows<S, N, Mode>(M, P, e, n, ph, FS, u, r);
  const T eL = liquid_fraction(T(P.epsCBD[ph]), u[7], u[8], T(P.epsL_min));
  const T fN = transport_factor(u, eL);
#pragma unroll 1
  for (int d = 0; d < 3; ++d) q1_axis<S, N, Mode, kNbrZero>(U, V, M, phase, P, e, n, ph, ix, iy, iz, FS, u, fN, d, r);

  if constexpr (kSources) {
    if (P.react[ph] != 0.0) {
      T Sx[9];
      node_sources(P, ph, u, Sx);
#pragma unroll
      for (int f = 0; f < 9; ++f) r[f] -= W3 * Sx[f];
    }
  }
}

// Q1 operator: residual (Mode 0, N = S) or Jacobian-vector product (Modes 1
// and 2, N = Dual<S>, output = derivative part).  M: the old mass
// (residual) or the linearisation coefficients of solid_tangent_kernel
// (condensed tangent); unused otherwise.
// Rows of node n of voxel e (e < P.Ne) with field stride FS; the arrays and
// the phase map start at the structure's first voxel.
template <typename S, typename N, int Mode>
__device__ __forceinline__ void q1_node(const S* __restrict__ U, const S* __restrict__ V,
                                        const S* __restrict__ M, S* __restrict__ Out,
                                        const uint8_t* __restrict__ phase, const DevParams& P,
                                        int64_t e, int n, int64_t FS) {
  const int ix = int(e % P.nx);
  const int iy = int((e / P.nx) % P.ny);
  const int iz = int(e / (int64_t(P.nx) * P.ny));
  const int ph = phase[e];
  N u[9], r[9];
  load_node<S, N, Mode>(U, V, M, FS, e * 8 + n, u);
  q1_rows<S, N, Mode, false>(U, V, M, phase, P, e, n, ph, ix, iy, iz, FS, u, r);
  if constexpr (Mode == kResidual) {
#pragma unroll
    for (int f = 0; f < 9; ++f) Out[f * FS + e * 8 + n] = r[f];
  } else {
    constexpr int nout = (Mode == kJvpFull) ? 9 : 7;
#pragma unroll
    for (int f = 0; f < nout; ++f) {
      const bool on = (P.active >> (f < 7 ? f : 7)) & 1;
      Out[f * FS + e * 8 + n] = on ? deriv_of(r[f]) : S(0);
    }
  }
}

// kLanes lanes per workgroup (kLanes / 8 voxels).
template <typename S, typename N, int Mode, int kLanes>
__device__ __forceinline__ void q1_body(const S* __restrict__ U, const S* __restrict__ V,
                                        const S* __restrict__ M, S* __restrict__ Out,
                                        const uint8_t* __restrict__ phase, const DevParams& P,
                                        int64_t nblocks_padded) {
  const int64_t blk = xcd_block(nblocks_padded);
  const int64_t gid = blk * kLanes + threadIdx.x;
  const int64_t e = gid >> 3;
  if (e >= P.Ne) return;                     // whole 8-lane groups leave together
  q1_node<S, N, Mode>(U, V, M, Out, phase, P, e, int(gid & 7), P.Ne * 8);
}

template <typename S, typename N, int Mode, int kLanes = 256>
__global__ void __launch_bounds__(kLanes)
q1_kernel(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ M,
          S* __restrict__ Out, const uint8_t* __restrict__ phase, DevParams P,
          int64_t nblocks_padded) {
  q1_body<S, N, Mode, kLanes>(U, V, M, Out, phase, P, nblocks_padded);
}

// The same operator held to 256 registers per lane (two waves per SIMD):
// the FP32 tangent otherwise takes a few accumulation registers beyond 256
// and drops to one wave per SIMD.
template <typename S, typename N, int Mode, int kLanes = 256>
__global__ void __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(2)))
q1_kernel_w2(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ M,
             S* __restrict__ Out, const uint8_t* __restrict__ phase, DevParams P,
             int64_t nblocks_padded) {
  q1_body<S, N, Mode, kLanes>(U, V, M, Out, phase, P, nblocks_padded);
}

// Old mass: m[i] = eps_L c_i (i < 6), m[6 + s] = eps_s.
template <typename T>
__global__ void __launch_bounds__(256)
mass_kernel(const T* __restrict__ U, T* __restrict__ M, const uint8_t* __restrict__ phase,
            DevParams P, int np) {
  const int64_t FS = P.Ne * np;
  for (int64_t gid = int64_t(blockIdx.x) * 256 + threadIdx.x; gid < FS; gid += int64_t(gridDim.x) * 256) {
    const int ph = phase[gid / np];
    const T e7 = U[7 * FS + gid], e8 = U[8 * FS + gid];
    const T eL = liquid_fraction(T(P.epsCBD[ph]), e7, e8, T(P.epsL_min));
#pragma unroll
    for (int i = 0; i < 6; ++i) M[i * FS + gid] = eL * U[i * FS + gid];
    M[6 * FS + gid] = e7;
    M[7 * FS + gid] = e8;
  }
}

}  // namespace lsbdg
