// Krylov operator of the Q1 scheme: the condensed tangent at a linearisation
// point, with every face inside a brick of voxels evaluated once and every
// tangent written out by hand.
//
// The rows are those of q1_node in resid_q1.hpp (Eq. 43-47 and 50: time,
// volume, interior-penalty face and source terms), differentiated in the
// direction v of the seven transported fields with the solid fractions
// condensed node by node (w = A^-1 dS_eps/du v, A = diag(rho/M)/dt -
// dS_eps/deps).  Only the tangent is formed: no flux or source value that
// no derivative needs is computed, and no dual-number arithmetic runs.
//
// Work decomposition:
//   * A workgroup owns a brick of 4 x 4 x 4 voxels, one lane per DG node
//     (512 lanes; node n = lane & 7 as everywhere, so the line partners of
//     a node are the lanes n ^ 1, n ^ 2, n ^ 4).
//   * Node phase: every lane loads u and v of its node, condenses its solid
//     fractions from its own source Jacobian, adds its time, volume and
//     source rows, and leaves in LDS what a face needs from a node:
//     c_0..c_5, Phi_L, eps_S8 + eps_Li2S and their tangents.
//   * Face phase: the faces touching the brick lie in 15 planes of 16 faces
//     (5 per axis: 3 inside the brick, 2 on its surface), 64 face points per
//     plane, one wavefront per plane and round: the 9 inner planes (each
//     face evaluated once, both voxels' records from LDS) come first, the 6
//     surface planes last (the outer voxel's two line nodes from memory,
//     their solid tangent from the row sums of the stored linearisation).
//     Each point leaves its flux tangent, seen from the lower voxel (outward
//     normal +e_d), in LDS.  A wavefront without a plane in the second
//     round leaves the loop.
//   * Gather: every node takes the fluxes of the two face points on its
//     normal lines, lam1 times the near one and lam0 times the far one,
//     with the sign of its side.
//
// Face points on the mesh boundary carry no tangent (the separator current
// and the no-flux condition are constants).  Bricks reaching past the mesh
// leave the missing voxels idle.
#pragma once

#include <hip/hip_runtime.h>

#include "model.hpp"
#include "dual.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"

namespace lsbdg {

constexpr int kBE = 4;                             // brick edge in voxels
constexpr int kBrickVox = kBE * kBE * kBE;         // 64
constexpr int kBrickLanes = 8 * kBrickVox;         // 512
constexpr int kRec = 16;                           // LDS record: 8 values, 8 tangents
constexpr int kPlanes = 3 * (kBE + 1);             // 15 face planes of 16 faces
constexpr int kFacePts = kPlanes * 64;             // 960 face points

// Parameters of the tangent in the kernel's precision (folded on the host).
template <typename S>
struct KP {
  S D0[6], zf[6], wL[6], zDA[6];       // diffusivities; z F/RT; conductivity and diffusion-potential weights
  S F, frt, frt2, eta, sigh, sq3h, W2, W3, W3idt;
  S epsCBD[2], epsL_min;
  S V, AU0[6], kE[6], kC[2], sqrtK[2], isqrtK[2], inv_cref, cmin, TH;   // AU0 = F U0/(2RT)
  S aV0[2], is8ref[2], ipass[2], rhoMidt[2];
  int react[2];
  int active;
  int nx, ny, nz;
  int64_t Ne;
};

template <typename S>
KP<S> make_kp(const DevParams& P) {
  KP<S> K{};
  for (int i = 0; i < 6; ++i) {
    K.D0[i] = S(P.D0[i]);
    K.zf[i] = S(kZ[i] * P.frt);
    K.wL[i] = S(P.wL[i]);
    K.zDA[i] = S(P.zDA[i]);
    K.AU0[i] = S(P.frt2 * P.U0[i]);
    K.kE[i] = S(P.kE[i]);
  }
  K.F = S(P.F);
  K.frt = S(P.frt);
  K.frt2 = S(P.frt2);
  K.eta = S(kEta);
  K.sigh = S(P.sig_h);
  K.sq3h = S(P.sq3_h);
  K.W2 = S(P.W2);
  K.W3 = S(P.W3);
  K.W3idt = S(P.W3 * P.inv_dt);
  K.epsL_min = S(P.epsL_min);
  K.V = S(P.V);
  K.inv_cref = S(P.inv_cref);
  K.cmin = S(P.c_min);
  K.TH = S(P.TH);
  for (int s = 0; s < 2; ++s) {
    K.epsCBD[s] = S(P.epsCBD[s]);
    K.kC[s] = S(P.kC[s]);
    K.sqrtK[s] = S(P.sqrtK[s]);
    K.isqrtK[s] = S(1.0 / P.sqrtK[s]);
    K.aV0[s] = S(P.aV0[s]);
    K.is8ref[s] = P.s8ref[s] > 0 ? S(1.0 / P.s8ref[s]) : S(0);
    K.ipass[s] = P.pass[s] > 0 ? S(1.0 / P.pass[s]) : S(0);
    K.rhoMidt[s] = S(P.rhoM[s] * P.inv_dt);
    K.react[s] = P.react[s] != 0.0;
  }
  K.active = P.active;
  K.nx = P.nx;
  K.ny = P.ny;
  K.nz = P.nz;
  K.Ne = P.Ne;
  return K;
}

// Node index of the point on the line with tangential position p (bits of
// the two other axes, lower axis first) at side s (bit d) of a voxel.
__device__ __forceinline__ int line_node(int d, int s, int p) {
  const int lo = p & 1, hi = p >> 1;
  return d == 0 ? (s | (lo << 1) | (hi << 2)) : d == 1 ? (lo | (s << 1) | (hi << 2)) : (lo | (hi << 1) | (s << 2));
}

// Tangential position of node n on a face normal to axis d.
__device__ __forceinline__ int line_pos(int d, int n) {
  return d == 0 ? (n >> 1) : d == 1 ? ((n & 1) | ((n >> 2) << 1)) : (n & 3);
}

// Face planes in evaluation order: the inner planes j = 1..3 of each axis,
// then the surface planes j = 0 and j = 4 (plane j of axis d separates the
// brick's voxels j - 1 and j along d).  Slot of plane (d, j) in that order.
__device__ __forceinline__ int plane_slot(int d, int j) {
  return (j >= 1 && j < kBE) ? 3 * d + (j - 1) : 3 * kBE - 3 + 2 * d + (j == kBE);
}
__device__ __forceinline__ void plane_of_slot(int q, int& d, int& j) {
  if (q < 3 * (kBE - 1)) {
    d = q / (kBE - 1);
    j = 1 + q % (kBE - 1);
  } else {
    const int r = q - 3 * (kBE - 1);
    d = r >> 1;
    j = (r & 1) ? kBE : 0;
  }
}

// LDS slots.  Node records: one pad word after every 32, so that the two
// voxels of a face, 32 words apart, fall on different banks.  Face points:
// 65 words per plane, so that the gather's reads of one voxel row from
// several planes fall on different banks.
__device__ __forceinline__ int rec_slot(int l) { return l + (l >> 5); }
__device__ __forceinline__ int q_slot(int k) { return k + (k >> 6); }
constexpr int kRecRow = kBrickLanes + kBrickLanes / 32;
constexpr int kQRow = kFacePts + kPlanes;

template <typename S>
struct BrickLds {
  S rec[kRec][kRecRow];              // node records, field-major
  S q[7][kQRow];                     // flux tangents of the face points
  int ph[kBrickVox];                 // voxel phases
};

// Division, exponential and logarithm of the tangent: hardware reciprocal,
// exp2 and log2 in FP32 (the operator of the inner FP32 solve, whose root
// is fixed by the FP64 residual), IEEE division and the device library in
// FP64 -- as the dual numbers of dual.hpp.
template <typename S>
__device__ __forceinline__ S tdiv(S a, S b) { return dual_div(a, b); }
template <typename S>
__device__ __forceinline__ S texp(S a) { return dual_exp(a); }
template <typename S>
__device__ __forceinline__ S tlog(S a) { return dual_log(a); }
__device__ __forceinline__ float tsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double tsqrt(double a) { return ::sqrt(a); }

// Harmonic mean 2ab/(a+b) (0 unless ab > 0, Eq. 45) and its tangent.
template <typename S>
__device__ __forceinline__ S harm_t(S a, S da, S b, S db, S& dh) {
  const S p = a * b;
  const bool ok = p > S(0);
  const S r = tdiv(S(1), ok ? a + b : S(1));
  const S r2 = S(2) * r;
  dh = ok ? r2 * r * (b * b * da + a * a * db) : S(0);
  return ok ? r2 * p : S(0);
}

// Transport factor f = eps_L^(3/2) exp(-eta c_S) of a traced state (t:
// c_0..c_5, Phi, eps_S8 + eps_Li2S) and its tangent df; eps_L floored
// (zero tangent when the floor is active).
template <typename S>
__device__ __forceinline__ S transport_t(const KP<S>& K, S epsCBD, const S* t, const S* dt, S& df) {
  S eL = S(1) - epsCBD - t[7];
  S deL = -dt[7];
  if (!(eL > K.epsL_min)) {
    eL = K.epsL_min;
    deL = S(0);
  }
  const S cS = t[5] + S(4) * t[4] + S(6) * t[3] + S(8) * t[2] + S(8) * t[1];
  const S dcS = dt[5] + S(4) * dt[4] + S(6) * dt[3] + S(8) * dt[2] + S(8) * dt[1];
  const S f = eL * tsqrt(eL) * texp(-K.eta * cS);
  df = f * (S(1.5) * tdiv(deL, eL) - K.eta * dcS);
  return f;
}

// Flux tangent at one face point (outward normal +e_d of the lower voxel
// A), Eq. 45-47: traces t and normal derivatives g of both sides with
// their tangents dt, dg; every coefficient from its own side's trace,
// averaged harmonically.  dq[0..6]: species and charge rows.
template <typename S>
__device__ __forceinline__ void face_tangent(const KP<S>& K, S eCa, S eCb, const S* ta, const S* dta,
                                             const S* ga, const S* dga, const S* tb, const S* dtb, const S* gb,
                                             const S* dgb, S* dq) {
  S dfa, dfb;
  const S fa = transport_t(K, eCa, ta, dta, dfa);
  const S fb = transport_t(K, eCb, tb, dtb, dfb);
  S dHf;
  const S Hf = harm_t(fa, dfa, fb, dfb, dHf);
  const S dphi = ta[6] - tb[6], ddphi = dta[6] - dtb[6];
  S lama = S(0), dlama = S(0), lamb = S(0), dlamb = S(0);
  S sda = S(0), dsda = S(0), sdb = S(0), dsdb = S(0), pen = S(0), dpen = S(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const S Dl = ta[i] - tb[i], dDl = dta[i] - dtb[i];
    S Ga = ga[i], dGa = dga[i], Gb = gb[i], dGb = dgb[i], mig = S(0);
    if (kZ[i] != 0.0) {
      const S z = K.zf[i];
      Ga += z * ta[i] * ga[6];
      dGa += z * (dta[i] * ga[6] + ta[i] * dga[6]);
      Gb += z * tb[i] * gb[6];
      dGb += z * (dtb[i] * gb[6] + tb[i] * dgb[6]);
      S dHm;
      const S Hm = harm_t(fa * ta[i], dfa * ta[i] + fa * dta[i], fb * tb[i], dfb * tb[i] + fb * dtb[i], dHm);
      mig = z * (dHm * dphi + Hm * ddphi);
    }
    const S dFa = dfa * Ga + fa * dGa, dFb = dfb * Gb + fb * dGb;
    dq[i] = K.D0[i] * (S(-0.5) * (dFa + dFb) + K.sigh * (dHf * Dl + Hf * dDl + mig));
    lama += K.wL[i] * ta[i];
    dlama += K.wL[i] * dta[i];
    lamb += K.wL[i] * tb[i];
    dlamb += K.wL[i] * dtb[i];
    sda += K.zDA[i] * ga[i];
    dsda += K.zDA[i] * dga[i];
    sdb += K.zDA[i] * gb[i];
    dsdb += K.zDA[i] * dgb[i];
    pen += K.zDA[i] * Dl;
    dpen += K.zDA[i] * dDl;
  }
  const S Ga6 = K.F * (sda + K.frt * lama * ga[6]);
  const S dGa6 = K.F * (dsda + K.frt * (dlama * ga[6] + lama * dga[6]));
  const S Gb6 = K.F * (sdb + K.frt * lamb * gb[6]);
  const S dGb6 = K.F * (dsdb + K.frt * (dlamb * gb[6] + lamb * dgb[6]));
  S dHl;
  const S Hl = harm_t(fa * lama, dfa * lama + fa * dlama, fb * lamb, dfb * lamb + fb * dlamb, dHl);
  dq[6] = S(-0.5) * (dfa * Ga6 + fa * dGa6 + dfb * Gb6 + fb * dGb6) +
          K.sigh * K.F * (dHf * pen + Hf * dpen + K.frt * (dHl * dphi + Hl * ddphi));
}

// Traces and normal derivatives (with tangents) of one side of a face from
// the records of its near and far line nodes; sgn = +1 for the lower voxel
// (near node at the higher coordinate), -1 for the upper one.
template <typename S>
__device__ __forceinline__ void side_traces(const KP<S>& K, const S* nv, const S* nd, const S* fv, const S* fd,
                                            S sgn, S* t, S* dt, S* g, S* dg) {
  const S l1 = S(kLam1), l0 = S(kLam0), s = sgn * K.sq3h;
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    t[f] = face_trace(nv[f], fv[f]);
    dt[f] = face_trace(nd[f], fd[f]);
  }
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    g[f] = s * (nv[f] - fv[f]);
    dg[f] = s * (nd[f] - fd[f]);
  }
  (void)l1;
  (void)l0;
}

template <typename S>
__device__ __forceinline__ void rec_lds(const BrickLds<S>& L, int node, S* v, S* d) {
  const int l = rec_slot(node);
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    v[f] = L.rec[f][l];
    d[f] = L.rec[8 + f][l];
  }
}

// Record of global node idx: u, v and the solid tangent sum from the row
// sums of the stored linearisation (zero without reactions).
template <typename S>
__device__ __forceinline__ void rec_global(const S* __restrict__ U, const S* __restrict__ V,
                                           const S* __restrict__ Cw, int64_t FS, int64_t idx, bool react, S* v,
                                           S* d) {
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    v[f] = U[f * FS + idx];
    d[f] = V[f * FS + idx];
  }
  v[7] = U[7 * FS + idx] + U[8 * FS + idx];
  S ws = S(0);
  if (react) {
#pragma unroll
    for (int j = 0; j < 7; ++j) ws += Cw[(7 + j) * FS + idx] * d[j];
  }
  d[7] = ws;
}

// Face point between lower voxel A (near record na, far fa) and upper voxel
// B (near nb, far fb).
template <typename S>
__device__ __forceinline__ void face_point(const KP<S>& K, int phA, int phB, const S* nav, const S* nad,
                                           const S* fav, const S* fad, const S* nbv, const S* nbd, const S* fbv,
                                           const S* fbd, S* dq) {
  S ta[8], dta[8], ga[7], dga[7], tb[8], dtb[8], gb[7], dgb[7];
  side_traces(K, nav, nad, fav, fad, S(1), ta, dta, ga, dga);
  side_traces(K, nbv, nbd, fbv, fbd, S(-1), tb, dtb, gb, dgb);
  face_tangent(K, K.epsCBD[phA], K.epsCBD[phB], ta, dta, ga, dga, tb, dtb, gb, dgb, dq);
}

// Source tangent of a reactive node and the condensation of its solid
// fractions: given the node's state u[9] and direction v[7], returns the
// solid tangents w0, w1 and the source rows' tangent dS[0..6] (Eq. 05-06,
// 18-24 in exponential form; T_H on C2 and E4).
template <typename S>
__device__ __forceinline__ void source_tangent(const KP<S>& K, int ph, const S* u, const S* v, bool solids,
                                               S& w0, S& w1, S* dS) {
  S la[6], dla[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const bool up = u[m] > K.cmin;
    const S c = up ? u[m] : K.cmin;
    la[m] = tlog(c * K.inv_cref);
    dla[m] = up ? tdiv(v[m], u[m]) : S(0);
  }
  // electrochemical reactions E1..E6 (Tab. 3), rates per unit a_V k_E
  const S lr[6] = {S(0.5) * la[1], S(1.5) * la[2], la[3], la[4] / S(6), S(0.5) * la[2],
                   la[4] / S(6) + S(4) / S(3) * la[0]};
  const S lp[6] = {S(0.5) * la[2], S(2) * la[3], S(1.5) * la[4], S(2) / S(3) * la[5], la[4], S(0)};
  const S dlr[6] = {S(0.5) * dla[1], S(1.5) * dla[2], dla[3], dla[4] / S(6), S(0.5) * dla[2],
                    dla[4] / S(6) + S(4) / S(3) * dla[0]};
  const S dlp[6] = {S(0.5) * dla[2], S(2) * dla[3], S(1.5) * dla[4], S(2) / S(3) * dla[5], dla[4], S(0)};
  const S base = K.frt2 * (K.V - u[6]);
  const S dA = -K.frt2 * v[6];
  S q[6], dq[6];                          // k_E r_k and its tangent at fixed a_V
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const S A = base - K.AU0[k];
    const S ef = texp(lr[k] - A), eb = texp(lp[k] + A);
    const S th = k == 3 ? K.TH : S(1);
    q[k] = K.kE[k] * th * (ef - eb);
    dq[k] = K.kE[k] * th * (ef * (dlr[k] - dA) - eb * (dlp[k] + dA));
  }
  // specific surface (Eq. 18 with Eq. 57) and its derivatives in eps
  const bool p7 = u[7] > S(0), p8 = u[8] > S(0);
  const S x1 = (p7 ? u[7] : S(0)) * K.is8ref[ph], x2 = (p8 ? u[8] : S(0)) * K.ipass[ph];
  const S s1 = tsqrt(x1), s2 = tsqrt(x2);
  const S inner = S(1) - x1 * s1 - x2 * s2;
  const bool open = inner > S(0);
  const S aV = open ? K.aV0[ph] * inner : S(0);
  const S aV7 = (open && p7) ? -S(1.5) * K.aV0[ph] * s1 * K.is8ref[ph] : S(0);
  const S aV8 = (open && p8) ? -S(1.5) * K.aV0[ph] * s2 * K.ipass[ph] : S(0);
  // chemical reactions C1 (S8 dissolution), C2 (Li2S dissolution)
  const S e1 = texp(la[1]), e2 = texp(S(2) * la[0] + la[5]);
  const S r0 = K.sqrtK[0] - e1 * K.isqrtK[0];
  const S dr0 = -e1 * K.isqrtK[0] * dla[1];
  const S r1 = (K.sqrtK[1] - e2 * K.isqrtK[1]) * K.TH;
  const S dr1 = -e2 * K.isqrtK[1] * (S(2) * dla[0] + dla[5]) * K.TH;
  // direction without solid change, then the condensation of the solid rows
  //   S7 = -vC0,  S8 = -vC1 + 2/3 sE5,  vC0 = eps7 kC0 r0,  vC1 = eps8 kC1 r1
  S dvC0 = u[7] * K.kC[0] * dr0, dvC1 = u[8] * K.kC[1] * dr1;
  S dsE[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) dsE[k] = aV * dq[k];
  w0 = S(0);
  w1 = S(0);
  if (solids) {
    const S t7 = -dvC0, t8 = -dvC1 + S(2) / S(3) * dsE[5];
    const S c70 = -K.kC[0] * r0;
    const S c80 = S(2) / S(3) * aV7 * q[5], c81 = -K.kC[1] * r1 + S(2) / S(3) * aV8 * q[5];
    const S a00 = K.rhoMidt[0] - c70, a10 = -c80, a11 = K.rhoMidt[1] - c81;   // a01 = 0
    const S idet = tdiv(S(1), a00 * a11);
    w0 = a11 * t7 * idet;
    w1 = (a00 * t8 - a10 * t7) * idet;
    const S daV = aV7 * w0 + aV8 * w1;
#pragma unroll
    for (int k = 0; k < 6; ++k) dsE[k] += daV * q[k];
    dvC0 += w0 * K.kC[0] * r0;
    dvC1 += w1 * K.kC[1] * r1;
  }
  const S t6 = S(1) / S(6), t3 = S(1) / S(3);
  dS[0] = S(2) * dvC1 - S(4) * t3 * dsE[5];
  dS[1] = dvC0 - S(0.5) * dsE[0];
  dS[2] = S(0.5) * dsE[0] - S(1.5) * dsE[1] - S(0.5) * dsE[4];
  dS[3] = S(2) * dsE[1] - dsE[2];
  dS[4] = S(1.5) * dsE[2] - t6 * dsE[3] + dsE[4] - t6 * dsE[5];
  dS[5] = dvC1 + S(2) * t3 * dsE[3];
  dS[6] = -K.F * (dsE[0] + dsE[1] + dsE[2] + dsE[3] + dsE[4] + dsE[5]);
}

// The operator on one brick (index `brick` of the structure's nbx x nby x
// nbz bricks, x fastest; an index past the last brick does nothing) of a
// structure whose arrays start at U, V, Cw, Out and phase, with field
// stride FS (the structure's own node count, or a batch's).
template <typename S>
__device__ __forceinline__ void brick_jvp(const S* __restrict__ U, const S* __restrict__ V,
                                          const S* __restrict__ Cw, S* __restrict__ Out,
                                          const uint8_t* __restrict__ phase, const KP<S>& K, int nbx, int nby,
                                          int64_t brick, int64_t FS, BrickLds<S>& L,
                                          const S* __restrict__ Rsub = nullptr) {
  const int lane = threadIdx.x;
  const int n = lane & 7, vb = lane >> 3;
  const int bx = vb & 3, by = (vb >> 2) & 3, bz = vb >> 4;
  const int64_t bi = brick % nbx, bj = (brick / nbx) % nby, bk = brick / (int64_t(nbx) * nby);
  const bool brick_ok = bk < (K.nz + kBE - 1) / kBE;
  const int ox0 = int(bi) * kBE, oy0 = int(bj) * kBE, oz0 = int(bk) * kBE;   // brick origin
  const int ix = ox0 + bx, iy = oy0 + by, iz = oz0 + bz;
  const bool valid = brick_ok && ix < K.nx && iy < K.ny && iz < K.nz;
  const int64_t e = valid ? ix + int64_t(K.nx) * (iy + int64_t(K.ny) * iz) : 0;
  const int ph = valid ? int(phase[e]) : 0;
  const bool solids = K.react[ph] && (K.active & kSolidsBit);

  // ---- node phase ----
  S acc[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) acc[f] = S(0);
  if (valid) {
    const int64_t idx = e * 8 + n;
    S u[9], v[7];
#pragma unroll
    for (int f = 0; f < 9; ++f) u[f] = U[f * FS + idx];
#pragma unroll
    for (int f = 0; f < 7; ++f) v[f] = V[f * FS + idx];
    S w0 = S(0), w1 = S(0);
    if (K.react[ph]) {
      S dS[7];
      source_tangent(K, ph, u, v, solids, w0, w1, dS);
#pragma unroll
      for (int f = 0; f < 7; ++f) acc[f] = -K.W3 * dS[f];
    }
    // time rows: W (eps_L c_i)'/dt
    S eL = S(1) - K.epsCBD[ph] - u[7] - u[8];
    S deL = -(w0 + w1);
    if (!(eL > K.epsL_min)) {
      eL = K.epsL_min;
      deL = S(0);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] += K.W3idt * (eL * v[i] + u[i] * deL);
    // volume rows along each axis: sqrt(3)/h sgn(a_d) W (F_d(a) + F_d(a'))
    const S cS = u[5] + S(4) * u[4] + S(6) * u[3] + S(8) * u[2] + S(8) * u[1];
    const S dcS = v[5] + S(4) * v[4] + S(6) * v[3] + S(8) * v[2] + S(8) * v[1];
    const S fN = eL * tsqrt(eL) * texp(-K.eta * cS);
    const S dfN = fN * (S(1.5) * tdiv(deL, eL) - K.eta * dcS);
    S lam = S(0), dlam = S(0);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      lam += K.wL[i] * u[i];
      dlam += K.wL[i] * v[i];
    }
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
      const int mask = 1 << d;
      const bool hi = (n & mask) != 0;
      const S s = hi ? K.sq3h : -K.sq3h;
      S g[7], dg[7];
#pragma unroll
      for (int f = 0; f < 7; ++f) {
        g[f] = s * (u[f] - xlane(u[f], mask));
        dg[f] = s * (v[f] - xlane(v[f], mask));
      }
      S dF[7], sd = S(0), dsd = S(0);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        S G = g[i], dG = dg[i];
        if (kZ[i] != 0.0) {
          G += K.zf[i] * u[i] * g[6];
          dG += K.zf[i] * (v[i] * g[6] + u[i] * dg[6]);
        }
        dF[i] = K.D0[i] * (dfN * G + fN * dG);
        sd += K.zDA[i] * g[i];
        dsd += K.zDA[i] * dg[i];
      }
      const S G6 = K.F * (sd + K.frt * lam * g[6]);
      const S dG6 = K.F * (dsd + K.frt * (dlam * g[6] + lam * dg[6]));
      dF[6] = dfN * G6 + fN * dG6;
      const S c = s * K.W3;
#pragma unroll
      for (int f = 0; f < 7; ++f) acc[f] += c * (dF[f] + xlane(dF[f], mask));
    }
    const int sl = rec_slot(lane);
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      L.rec[f][sl] = u[f];
      L.rec[8 + f][sl] = v[f];
    }
    L.rec[7][sl] = u[7] + u[8];
    L.rec[15][sl] = w0 + w1;
  } else {
#pragma unroll
    for (int f = 0; f < kRec; ++f) L.rec[f][rec_slot(lane)] = S(0);
  }
  if (n == 0) L.ph[vb] = ph;
  __syncthreads();

  // ---- face phase: one face point per lane and round, a plane per
  // wavefront (inner planes first) ----
  for (int k = lane; k < kFacePts; k += kBrickLanes) {
    int d, j;
    plane_of_slot(k >> 6, d, j);
    const int f16 = (k >> 2) & 15, p = k & 3;
    const int t1 = f16 & 3, t2 = f16 >> 2;             // voxel coordinates on the two other axes
    // brick-local coordinates of the lower voxel A (j - 1 along d) and the upper B (j)
    int ax, ay, az;
    if (d == 0) { ax = j - 1; ay = t1; az = t2; }
    else if (d == 1) { ax = t1; ay = j - 1; az = t2; }
    else { ax = t1; ay = t2; az = j - 1; }
    const int bxu = ax + (d == 0), byu = ay + (d == 1), bzu = az + (d == 2);
    const int gax = ox0 + ax, gay = oy0 + ay, gaz = oz0 + az;
    const int gbx = ox0 + bxu, gby = oy0 + byu, gbz = oz0 + bzu;
    const bool ok = brick_ok && gax >= 0 && gay >= 0 && gaz >= 0 && gbx < K.nx && gby < K.ny && gbz < K.nz;
    S q[7];
    if (ok) {
      S nav[8], nad[8], fav[8], fad[8], nbv[8], nbd[8], fbv[8], fbd[8];
      int phA, phB;
      const int nA = line_node(d, 1, p), fA = line_node(d, 0, p);   // near / far node of A
      if (j >= 1) {
        const int va = ax + kBE * (ay + kBE * az);
        rec_lds(L, 8 * va + nA, nav, nad);
        rec_lds(L, 8 * va + fA, fav, fad);
        phA = L.ph[va];
      } else {
        const int64_t ea = gax + int64_t(K.nx) * (gay + int64_t(K.ny) * gaz);
        phA = int(phase[ea]);
        const bool react = K.react[phA] && (K.active & kSolidsBit);
        rec_global(U, V, Cw, FS, ea * 8 + nA, react, nav, nad);
        rec_global(U, V, Cw, FS, ea * 8 + fA, react, fav, fad);
      }
      if (j < kBE) {
        const int vu = bxu + kBE * (byu + kBE * bzu);
        rec_lds(L, 8 * vu + fA, nbv, nbd);        // B's near node is its bit-d-clear node
        rec_lds(L, 8 * vu + nA, fbv, fbd);
        phB = L.ph[vu];
      } else {
        const int64_t eb = gbx + int64_t(K.nx) * (gby + int64_t(K.ny) * gbz);
        phB = int(phase[eb]);
        const bool react = K.react[phB] && (K.active & kSolidsBit);
        rec_global(U, V, Cw, FS, eb * 8 + fA, react, nbv, nbd);
        rec_global(U, V, Cw, FS, eb * 8 + nA, react, fbv, fbd);
      }
      face_point(K, phA, phB, nav, nad, fav, fad, nbv, nbd, fbv, fbd, q);
    } else {
#pragma unroll
      for (int f = 0; f < 7; ++f) q[f] = S(0);
    }
#pragma unroll
    for (int f = 0; f < 7; ++f) L.q[f][q_slot(k)] = q[f];
  }
  __syncthreads();
  if (!valid) return;

  // ---- gather: lam1 x the face point at the node's own side of each
  // normal line, lam0 x the one at the other side; +flux on the lower
  // voxel of a face, -flux on the upper ----
  const S lam1 = S(kLam1), lam0 = S(kLam0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int p = line_pos(d, n);
    const int c = d == 0 ? bx : d == 1 ? by : bz;
    const int t1 = d == 0 ? by : bx, t2 = d == 2 ? by : bz;
    const int s_own = (n >> d) & 1;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int s = side == 0 ? s_own : 1 - s_own;       // 1: the voxel's high face
      const S w = K.W2 * (side == 0 ? lam1 : lam0) * (s ? S(1) : S(-1));
      const int k = q_slot(plane_slot(d, c + s) * 64 + (t1 + 4 * t2) * 4 + p);
#pragma unroll
      for (int f = 0; f < 7; ++f) acc[f] += w * L.q[f][k];
    }
  }
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    const bool on = (K.active >> f) & 1;
    const int64_t idx = f * FS + e * 8 + n;
    const S jv = on ? acc[f] : S(0);
    Out[idx] = Rsub ? Rsub[idx] - jv : jv;
  }
}

// One structure: one workgroup per brick, XCD-aware order.  Rsub
// (optional): Out = Rsub - J v instead (the residual the multiplicative
// preconditioner leaves to the element blocks).
template <typename S>
__global__ void __launch_bounds__(kBrickLanes)
q1_brick_jvp_kernel(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ Cw,
                    S* __restrict__ Out, const uint8_t* __restrict__ phase, KP<S> K, int nbx, int nby,
                    int64_t nbricks_padded, const S* __restrict__ Rsub = nullptr) {
  __shared__ BrickLds<S> L;
  brick_jvp(U, V, Cw, Out, phase, K, nbx, nby, xcd_block(nbricks_padded), K.Ne * 8, L, Rsub);
}

}  // namespace lsbdg
