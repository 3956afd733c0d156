// Element block-Jacobi preconditioner for the Q1 operator on gfx950.
//
// Assembly: the element-diagonal block J_EE of the (condensed) Jacobian is
// the tangent of the element's own rows with respect to its own unknowns,
// every neighbour held fixed.  Column j is the dual-number evaluation of
// the Q1 operator body seeded with the unit direction e_j on this element
// and zero on its neighbours.  Block index = field * 8 + node; storage is
// column-major per element, B[e][col][row].
//
// Inversion: one wavefront per element, lane i holds row i in registers.
// In-place Gauss-Jordan with partial pivoting and no physical row swaps:
// at step k the unused row p with the largest |a_ik| becomes the pivot of
// column k, its row is broadcast with readlane, every other row is
// eliminated and the pivot row scaled (one multiply-add per entry on every
// lane), and column k is replaced by the corresponding column of the
// partial inverse.  Rotating each row left by one after every step keeps
// the active column at register 0, so no register is indexed dynamically.
// With pivot rows p_0..p_{n-1} the result B satisfies
//     A^{-1}[k][p_m] = B[p_k][m],
// which the write-out applies.
//
// Storage of the inverse: column quads per row, element block e at
// e * NB * NB, entry (row, col) at ((col / 4) * NB + row) * 4 + col % 4, so
// that lane r of the apply reads four columns of its row with one 16-byte
// (FP32) load and a wavefront's load covers a contiguous 56 x 16 bytes.
//
// Apply: y_e = B_e^{-1} x_e, one wavefront per element, lane r = row r;
// optionally (y + a) / d entrywise in the same pass.
#pragma once

#include <hip/hip_runtime.h>

#include "dual.hpp"
#include "resid_q1.hpp"

namespace lsbdg {

__device__ __forceinline__ float bcast(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double bcast(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Element-diagonal blocks.  Mode kJvpFull (9 fields, nb = 72) or
// kJvpCondensed (7 fields, nb = 56).  One lane per node, as q1_kernel.
// Cw: linearisation coefficients at U (kJvpCondensed).
// Node n's rows of voxel e's block (e < P.Ne; field stride FS; the arrays,
// the phase map and Bout start at the structure's first voxel).
template <typename S, int Mode>
__device__ __forceinline__ void q1_block_node(const S* __restrict__ U, const S* __restrict__ Cw,
                                              S* __restrict__ Bout, const uint8_t* __restrict__ phase,
                                              const DevParams& P, int64_t e, int n, int64_t FS) {
  using N = Dual<S>;
  constexpr int NF = (Mode == kJvpFull) ? 9 : 7;
  constexpr int NB = NF * 8;
  const int ix = int(e % P.nx);
  const int iy = int((e / P.nx) % P.ny);
  const int iz = int(e / (int64_t(P.nx) * P.ny));
  const int ph = phase[e];
  S us[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) us[f] = U[f * FS + e * 8 + n];
  S* Be = Bout + e * int64_t(NB) * NB;
  const S W3 = S(P.W3);

  // Columns in the order (field fj, node nj).  Along axis d a node's rows
  // depend only on the two nodes of its own d-line (volume term: the line
  // gradient and the node's own state; face term: the traces of that line
  // at the voxel side, the neighbour's direction being zero), so a node's
  // rows see only itself and its three line partners n ^ 1, n ^ 2, n ^ 4.
  // For each field fj and axis d two passes seed the nodes with bit d = 0,
  // then those with bit d = 1 -- one node of every d-line -- and each lane
  // reads off its rows' derivative with respect to its own node (seeded) or
  // its d-partner (not seeded).  The own column accumulates the time term,
  // the three axes in order and the node-local sources, as the operator
  // itself does; the partner columns take their single axis.  The sources
  // are node-local, through the tangent ks of the lane's own unknown fj
  // (with the condensed solid-fraction tangent), formed once per field.
#pragma unroll 1
  for (int fj = 0; fj < NF; ++fj) {
    if (!((P.active >> (fj < 7 ? fj : 7)) & 1)) {   // inactive unknown: identity columns
#pragma unroll 1
      for (int nj = 0; nj < 8; ++nj) {
        const int col = fj * 8 + nj;
#pragma unroll
        for (int f = 0; f < NF; ++f) Be[col * NB + f * 8 + n] = (f == fj && n == nj) ? S(1) : S(0);
      }
      continue;
    }
    S vo[9];                                     // direction at the seeded node
#pragma unroll
    for (int f = 0; f < 9; ++f) vo[f] = (f == fj) ? S(1) : S(0);
    if constexpr (Mode == kJvpCondensed) {
      const S c0 = Cw[fj * FS + e * 8 + n];
      const S cs = Cw[(7 + fj) * FS + e * 8 + n];
      vo[7] = c0;
      vo[8] = cs - c0;
    }
    S ks[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) ks[f] = S(0);
    if (P.react[ph] != 0.0) {
      N x[9], Sx[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) x[f] = N(us[f], vo[f]);
      node_sources(P, ph, x, Sx);
#pragma unroll
      for (int f = 0; f < NF; ++f) ks[f] = Sx[f].d;
    }
    S own[NF], nb0[NF], nb1[NF], nb2[NF];
    {
      N x[9], r[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) x[f] = N(us[f], vo[f]);
      q1_mass_rows<S, N, kJvpFull>(static_cast<const S*>(nullptr), P, e, n, ph, FS, x, r);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        own[f] = r[f].d;
        nb0[f] = nb1[f] = nb2[f] = S(0);
      }
    }
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
#pragma unroll 1
      for (int s = 0; s < 2; ++s) {
        const bool seeded = ((n >> d) & 1) == s;
        N u[9], r[9];
#pragma unroll
        for (int f = 0; f < 9; ++f) u[f] = N(us[f], seeded ? vo[f] : S(0));
        const N eL = liquid_fraction(N(P.epsCBD[ph]), u[7], u[8], N(P.epsL_min));
        const N fN = transport_factor(u, eL);
#pragma unroll
        for (int f = 0; f < 7; ++f) {
          const S acc = seeded ? own[f] : (d == 0 ? nb0[f] : d == 1 ? nb1[f] : nb2[f]);
          r[f] = N(S(0), acc);
        }
        q1_axis<S, N, kJvpFull, true>(U, nullptr, nullptr, phase, P, e, n, ph, ix, iy, iz, FS, u, fN, d, r);
#pragma unroll
        for (int f = 0; f < 7; ++f) {
          const S v = r[f].d;
          own[f] = seeded ? v : own[f];
          nb0[f] = (!seeded && d == 0) ? v : nb0[f];
          nb1[f] = (!seeded && d == 1) ? v : nb1[f];
          nb2[f] = (!seeded && d == 2) ? v : nb2[f];
        }
      }
    }
#pragma unroll 1
    for (int nj = 0; nj < 8; ++nj) {
      const int col = fj * 8 + nj;
      const int x = nj ^ n;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const S val = x == 0 ? own[f] - W3 * ks[f]
                             : x == 1 ? nb0[f] : x == 2 ? nb1[f] : x == 4 ? nb2[f] : S(0);
        Be[col * NB + f * 8 + n] = ((P.active >> (f < 7 ? f : 7)) & 1) ? val : S(0);
      }
    }
  }
}

template <typename S, int Mode>
__global__ void __launch_bounds__(256)
q1_block_kernel(const S* __restrict__ U, const S* __restrict__ Cw, S* __restrict__ Bout,
                const uint8_t* __restrict__ phase, DevParams P, int64_t nblocks_padded) {
  const int64_t blk = xcd_block(nblocks_padded);
  const int64_t gid = blk * 256 + threadIdx.x;
  const int64_t e = gid >> 3;
  if (e >= P.Ne) return;
  q1_block_node<S, Mode>(U, Cw, Bout, phase, P, e, int(gid & 7), P.Ne * 8);
}

// Entry (row, col) of a block in the column-quad storage.
template <int NB>
__host__ __device__ __forceinline__ int quad_index(int row, int col) {
  return ((col >> 2) * NB + row) * 4 + (col & 3);
}

// Wave-wide argmax of a non-negative key (-1 = excluded); returns the lane.
// The key keeps the block's precision: entries of trace-species rows lie
// far below the FP32 range, where FP32 keys would all tie.
template <typename S>
__device__ __forceinline__ int wave_argmax(S key, int lane) {
  S k = key;
  int l = lane;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const S ok = __shfl_xor(k, off);
    const int ol = __shfl_xor(l, off);
    if (ok > k || (ok == k && ol < l)) {
      k = ok;
      l = ol;
    }
  }
  return l;
}

// bfloat16 copy of FP32 inverses for the apply (half the bytes; only the
// preconditioner changes, not the solution): entry (row, col) at
// ((col / 8) * NB + row) * 8 + col % 8, rounded to nearest even.
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t((u >> 16) | ((u & 0x007fffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// In-place inversion of every element block (see header comment).  A block
// whose best available pivot is zero or not finite sets *status = 1.  With
// kToBf16 (S = float) the inverse goes to H in the bfloat16 layout of
// blocks_to_bf16_kernel instead, and B keeps the assembled blocks.
template <typename S, int NB, bool kToBf16 = false>
__global__ void __launch_bounds__(256)
invert_blocks_kernel(S* __restrict__ B, int64_t Ne, int* __restrict__ status,
                     uint16_t* __restrict__ H = nullptr) {
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t e = int64_t(blockIdx.x) * 4 + w;
  if (e >= Ne) return;                       // whole wavefronts leave together
  const bool act = lane < NB;
  S* Be = B + e * int64_t(NB) * NB;
  S r[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) r[j] = act ? Be[j * NB + lane] : S(0);
  bool used = !act;
  int kk = 0;        // step at which this lane's row was the pivot
  int mypiv = 0;     // lane m keeps the pivot row of step m
  bool bad = false;
#pragma unroll 1
  for (int k = 0; k < NB; ++k) {
    const S key = used ? S(-1) : S(fabs(r[0]));
    const int p = wave_argmax(key, lane);
    const S pv = bcast(r[0], p);
    if (!(fabs(pv) > S(0)) || !isfinite(pv)) bad = true;
    if (lane == k) mypiv = p;
    if (lane == p) {
      used = true;
      kk = k;
    }
    const S inv = S(1) / pv;
    // one multiply-add per entry on every lane: the other rows take
    // r_j - f inv p_j, the pivot row (whose broadcast entry is its own)
    // r_j + (inv - 1) r_j = inv r_j
    const S c = (lane == p) ? inv - S(1) : -r[0] * inv;
#pragma unroll
    for (int j = 1; j < NB; ++j) r[j - 1] = fma(c, bcast(r[j], p), r[j]);
    r[NB - 1] = (lane == p) ? inv : c;
  }
  if (bad && lane == 0) atomicOr(status, 1);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    const int pm = __builtin_amdgcn_readlane(mypiv, m);
    if constexpr (kToBf16) {
      if (act) H[e * int64_t(NB) * NB + ((pm >> 3) * NB + kk) * 8 + (pm & 7)] = to_bf16(float(r[m]));
    } else {
      if (act) Be[quad_index<NB>(kk, pm)] = r[m];
    }
  }
}

// Column-major copy of the stored inverses: out[e][col][row].
template <typename S, int NB>
__global__ void __launch_bounds__(256)
export_blocks_kernel(const S* __restrict__ B, S* __restrict__ out, int64_t Ne) {
  const int64_t total = Ne * NB * NB;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int64_t e = k / (NB * NB);
    const int w = int(k - e * NB * NB);
    const int col = w / NB, row = w - col * NB;
    out[k] = B[e * NB * NB + quad_index<NB>(row, col)];
  }
}

// y_e = B_e x_e for vectors in the field-major layout [f][e][n] (NF fields).
template <typename S, int NF>
__global__ void __launch_bounds__(256)
apply_blocks_kernel(const S* __restrict__ B, const S* __restrict__ X, S* __restrict__ Y, int64_t Ne,
                    const S* __restrict__ A = nullptr, const S* __restrict__ D = nullptr) {
  constexpr int NB = NF * 8;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t e = int64_t(blockIdx.x) * 4 + w;
  if (e >= Ne) return;
  const int64_t FS = Ne * 8;
  const bool act = lane < NB;
  const int fl = lane >> 3, nl = lane & 7;
  const S xl = act ? X[fl * FS + e * 8 + nl] : S(0);
  const S* Be = B + e * int64_t(NB) * NB;
  struct alignas(4 * sizeof(S)) Quad { S a, b, c, d; };
  S acc = S(0);
#pragma unroll
  for (int c4 = 0; c4 < NB / 4; ++c4) {
    Quad q{S(0), S(0), S(0), S(0)};
    if (act) q = *reinterpret_cast<const Quad*>(Be + (c4 * NB + lane) * 4);
    acc += q.a * bcast(xl, 4 * c4);
    acc += q.b * bcast(xl, 4 * c4 + 1);
    acc += q.c * bcast(xl, 4 * c4 + 2);
    acc += q.d * bcast(xl, 4 * c4 + 3);
  }
  if (act) {
    // optional epilogue of the two-level preconditioner: (B x + A) / D
    const int64_t idx = fl * FS + e * 8 + nl;
    if (A) acc = A[idx] + acc;
    if (D) acc = acc / D[idx];
    Y[idx] = acc;
  }
}

template <int NB>
__global__ void __launch_bounds__(256)
blocks_to_bf16_kernel(const float* __restrict__ B, uint16_t* __restrict__ H, int64_t Ne) {
  const int64_t total = Ne * NB * NB;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int64_t e = k / (NB * NB);
    const int w = int(k - e * NB * NB);
    const int i = w & 7, row = (w >> 3) % NB, c8 = (w >> 3) / NB;
    H[k] = to_bf16(B[e * NB * NB + quad_index<NB>(row, 8 * c8 + i)]);
  }
}

template <int NF>
__global__ void __launch_bounds__(256)
apply_blocks_bf16_kernel(const uint16_t* __restrict__ H, const float* __restrict__ X, float* __restrict__ Y,
                         int64_t Ne, const float* __restrict__ A = nullptr, const float* __restrict__ D = nullptr) {
  constexpr int NB = NF * 8;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t e = int64_t(blockIdx.x) * 4 + w;
  if (e >= Ne) return;
  const int64_t FS = Ne * 8;
  const bool act = lane < NB;
  const int fl = lane >> 3, nl = lane & 7;
  const float xl = act ? X[fl * FS + e * 8 + nl] : 0.0f;
  const uint16_t* He = H + e * int64_t(NB) * NB;
  float acc = 0.0f;
#pragma unroll
  for (int c8 = 0; c8 < NB / 8; ++c8) {
    uint4 q = make_uint4(0u, 0u, 0u, 0u);
    if (act) q = *reinterpret_cast<const uint4*>(He + (c8 * NB + lane) * 8);
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc += __uint_as_float(wd[t] << 16) * bcast(xl, 8 * c8 + 2 * t);
      acc += __uint_as_float(wd[t] & 0xffff0000u) * bcast(xl, 8 * c8 + 2 * t + 1);
    }
  }
  if (act) {
    // optional epilogue of the two-level preconditioner: (B x + A) / D
    const int64_t idx = fl * FS + e * 8 + nl;
    if (A) acc = A[idx] + acc;
    if (D) acc = acc / D[idx];
    Y[idx] = acc;
  }
}

}  // namespace lsbdg
