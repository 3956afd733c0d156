// Element block-Jacobi preconditioner for the k = 3 operator on gfx950:
// 448 x 448 blocks (7 fields x 64 Gauss nodes) of the condensed Jacobian.
//
// Assembly: exact, by probing the Krylov operator (the condensed tangent at
// the stored linearisation).  The unit direction e_j seeded on every voxel
// of one checkerboard colour reaches a voxel's own rows only from the voxel
// itself, since its face neighbours have the other colour; so the operator
// applied to it holds column j of every such voxel's block.  Two colours x
// 448 columns; seed_q3_kernel builds the direction, scatter_q3_kernel files
// the column.  Block index = field * 64 + node, storage column-major per
// element: B[e][col][row].
//
// Inversion (invert_q3_kernel): blocked in-place Gauss-Jordan with partial
// pivoting over all unused rows, one 512-lane workgroup per element (lane i
// owns row i), in panels of W columns (64 in FP32, 32 in FP64).  For a
// panel C:
//   1. each lane holds its row's W panel entries in registers and W
//      unblocked Gauss-Jordan steps run on them alone, each choosing as
//      pivot the unused row with the largest magnitude in its column (ties:
//      the lowest row).  The registers rotate by one per step, so the
//      active column is always register 0 and no register is indexed at
//      run time; the argmax of the next column is taken in the same pass,
//      and the pivot row reaches the other lanes through LDS: two barriers
//      per step.  With pivot rows R this leaves, in the panel columns, E's
//      columns at R, where E is the row transformation of the W steps (E = I
//      except in columns R; rows R of E are the inverse of A[R, C]);
//   2. every other column is updated at once with that transformation:
//      A[i, X] = [i not in R] A[i, X] + sum_s E[i, R_s] A[R_s, X], a
//      448 x W by W x 448 product on the matrix cores (16 x 16 x 4 MFMA
//      tiles).  The panel goes to LDS as the left operand; each wavefront
//      owns whole 16-column tiles, so it reads the pivot rows' entries of a
//      tile into registers before it writes any of them.
// Apply (apply_q3_kernel): y = A^-1 x as z = B x', x'_m = x[p_m], then
// y_k = z[p_k]; one workgroup per element, lane r = row r, each wavefront
// reading 64 consecutive rows of a column (256 bytes in FP32).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace lsbdg {

constexpr int kQ3NB = 448;

template <typename S>
struct Q3Panel;
template <>
struct Q3Panel<float> {
  static constexpr int W = 64;
};
template <>
struct Q3Panel<double> {
  static constexpr int W = 32;
};

typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef double v4f64 __attribute__((ext_vector_type(4)));

template <typename S>
struct Acc4;
template <>
struct Acc4<float> {
  using T = v4f32;
};
template <>
struct Acc4<double> {
  using T = v4f64;
};

// acc += A_tile(16 x 4) B_tile(4 x 16): lane l gives A[l % 16][l / 16] and
// B[l / 16][l % 16].  acc[v] of lane l is entry (mfma_row<S>(l, v), l % 16):
// row 4 (l / 16) + v in FP32, row l / 16 + 4 v in FP64 (checked on the
// device for both builtins).
__device__ __forceinline__ void mfma_16x16x4(float a, float b, v4f32& acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma_16x16x4(double a, double b, v4f64& acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}
template <typename S>
__device__ __forceinline__ int mfma_row(int lane, int v) {
  return std::is_same<S, double>::value ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

__device__ __forceinline__ int q3_colour(int64_t e, int nx, int ny) {
  const int64_t ix = e % nx, iy = (e / nx) % ny, iz = e / (int64_t(nx) * ny);
  return int((ix + iy + iz) & 1);
}

// v[f][e][n] = 1 where f * 64 + n == j on voxels of colour c, else 0.
template <typename S>
__global__ void __launch_bounds__(256)
seed_q3_kernel(S* __restrict__ v, int64_t Ne, int nx, int ny, int c, int j) {
  const int64_t FS = Ne * 64, total = 7 * FS;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int f = int(k / FS);
    const int64_t r = k - f * FS;
    const int64_t e = r >> 6;
    const int n = int(r & 63);
    v[k] = (f * 64 + n == j && q3_colour(e, nx, ny) == c) ? S(1) : S(0);
  }
}

// B[e][j][row] = w[row / 64][e][row % 64] on voxels of colour c.
template <typename S>
__global__ void __launch_bounds__(256)
scatter_q3_kernel(const S* __restrict__ w, S* __restrict__ B, int64_t Ne, int nx, int ny, int c, int j) {
  const int64_t FS = Ne * 64, total = Ne * kQ3NB;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int64_t e = k / kQ3NB;
    const int row = int(k - e * kQ3NB);
    if (q3_colour(e, nx, ny) != c) continue;
    B[(e * kQ3NB + j) * kQ3NB + row] = w[(row >> 6) * FS + e * 64 + (row & 63)];
  }
}

// Largest key over the workgroup's 8 wavefronts (ties: the lowest row):
// the wavefront's winner goes to red_v / red_i[wave].
template <typename S>
__device__ __forceinline__ void q3_pivot_partial(S key, int row, int lane, int wv, S* red_v, int* red_i) {
  S best = key;
  int bi = row;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const S ov = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    red_v[wv] = best;
    red_i[wv] = bi;
  }
}

// Pivot key of a row: |a| (a NaN counts as 0), compared in S (entries of
// trace-species rows lie far below the FP32 range); -1 for rows already
// used and lanes without a row.
template <typename S>
__device__ __forceinline__ S q3_key(S a, bool avail) {
  const S m = fabs(a);
  return avail ? (m == m ? m : S(0)) : S(-1);
}

// In-place inversion of every element block (see the header comment); one
// workgroup per element.  A pivot that is zero or not finite sets *status.
template <typename S>
__global__ void __launch_bounds__(512)
invert_q3_kernel(S* __restrict__ B, int16_t* __restrict__ piv, int* __restrict__ status) {
  constexpr int NB = kQ3NB, W = Q3Panel<S>::W, NT = NB / 16, NW = 8;
  static_assert(NB % W == 0 && W % 16 == 0, "panel width");
  __shared__ S pan[W][NB];      // the eliminated panel: left operand of the update
  __shared__ S prow[W];         // the pivot row of the current step (rotated as the registers)
  __shared__ S red_v[NW];
  __shared__ int red_i[NW];
  __shared__ int pivl[W];
  __shared__ uint8_t inpan[NB]; // row is a pivot of the current panel
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool has_row = tid < NB;
  const int64_t e = blockIdx.x;
  S* __restrict__ Be = B + e * int64_t(NB) * NB;
  bool used = false, bad = false;
  if (has_row) inpan[tid] = 0;
  S r[W];
#pragma unroll 1
  for (int c0 = 0; c0 < NB; c0 += W) {
#pragma unroll
    for (int j = 0; j < W; ++j) r[j] = has_row ? Be[int64_t(c0 + j) * NB + tid] : S(0);
    q3_pivot_partial(q3_key(r[0], has_row && !used), tid, lane, wv, red_v, red_i);
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < W; ++t) {
      S bv = red_v[0];
      int p = red_i[0];
#pragma unroll
      for (int w = 1; w < NW; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < p)) {
          bv = red_v[w];
          p = red_i[w];
        }
      const bool me = tid == p;
      if (me) {
#pragma unroll
        for (int j = 0; j < W; ++j) prow[j] = r[j];
        inpan[p] = 1;
        used = true;
      }
      if (tid == 0) {
        pivl[t] = p;
        piv[e * NB + c0 + t] = int16_t(p);
      }
      __syncthreads();
      const S pv = prow[0];
      if (!(fabs(pv) > S(0)) || !isfinite(pv)) bad = true;
      const S inv = S(1) / pv;
      const S f = r[0];
#pragma unroll
      for (int j = 1; j < W; ++j) {
        const S pr = prow[j] * inv;
        r[j - 1] = me ? pr : r[j] - f * pr;
      }
      r[W - 1] = me ? inv : -f * inv;
      if (t + 1 < W) q3_pivot_partial(q3_key(r[0], has_row && !used), tid, lane, wv, red_v, red_i);
      __syncthreads();
    }
    // W rotations: register j holds panel column j again
    if (has_row) {
#pragma unroll
      for (int j = 0; j < W; ++j) {
        pan[j][tid] = r[j];
        Be[int64_t(c0 + j) * NB + tid] = r[j];
      }
    }
    __syncthreads();
    for (int jt = wv; jt < NT; jt += NW) {
      const int j0 = jt * 16;
      if (j0 >= c0 && j0 < c0 + W) continue;
      const int j = j0 + (lane & 15);
      S* __restrict__ colj = Be + int64_t(j) * NB;
      S g[W / 4];
#pragma unroll
      for (int kk = 0; kk < W / 4; ++kk) g[kk] = colj[pivl[4 * kk + (lane >> 4)]];
#pragma unroll 1
      for (int it = 0; it < NT; ++it) {
        const int i0 = it * 16;
        typename Acc4<S>::T acc = {S(0), S(0), S(0), S(0)};
#pragma unroll
        for (int kk = 0; kk < W / 4; ++kk) mfma_16x16x4(pan[4 * kk + (lane >> 4)][i0 + (lane & 15)], g[kk], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + mfma_row<S>(lane, v);
          colj[i] = (inpan[i] ? S(0) : colj[i]) + acc[v];
        }
      }
    }
    __syncthreads();
    if (has_row) inpan[tid] = 0;
  }
  if (bad && tid == 0) atomicOr(status, 1);
}

// y_e = A_e^-1 x_e for 7-field vectors [f][e][n] (n < 64); one workgroup of
// 512 lanes per element (448 active).
template <typename S>
__global__ void __launch_bounds__(512)
apply_q3_kernel(const S* __restrict__ B, const int16_t* __restrict__ piv, const S* __restrict__ X,
                S* __restrict__ Y, int64_t Ne) {
  constexpr int NB = kQ3NB;
  __shared__ S xs[NB];
  __shared__ S zs[NB];
  __shared__ int ps[NB];
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t FS = Ne * 64;
  if (tid < NB) {
    const int p = piv[e * NB + tid];
    ps[tid] = p;
    xs[tid] = X[(p >> 6) * FS + e * 64 + (p & 63)];
  }
  __syncthreads();
  if (tid < NB) {
    const S* __restrict__ col = B + e * int64_t(NB) * NB + tid;
    S acc = S(0);
#pragma unroll 8
    for (int m = 0; m < NB; ++m) acc += col[int64_t(m) * NB] * xs[m];
    zs[tid] = acc;
  }
  __syncthreads();
  if (tid < NB) Y[(tid >> 6) * FS + e * 64 + (tid & 63)] = zs[ps[tid]];
}

// out[e][col][row] = A_e^-1[row][col]: with ip the inverse pivot list,
// A^-1[k][j] = B[p_k][ip[j]].
template <typename S>
__global__ void __launch_bounds__(512)
export_q3_kernel(const S* __restrict__ B, const int16_t* __restrict__ piv, S* __restrict__ out) {
  constexpr int NB = kQ3NB;
  __shared__ int ps[NB];
  __shared__ int ip[NB];
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < NB) {
    const int p = piv[e * NB + tid];
    ps[tid] = p;
    ip[p] = tid;
  }
  __syncthreads();
  const S* __restrict__ Be = B + e * int64_t(NB) * NB;
  S* __restrict__ Oe = out + e * int64_t(NB) * NB;
  for (int k = tid; k < NB * NB; k += 512) {
    const int j = k / NB, row = k - j * NB;
    Oe[k] = Be[int64_t(ip[j]) * NB + ps[row]];
  }
}

}  // namespace lsbdg
