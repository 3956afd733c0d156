// Vector kernels of the Newton-Krylov solver (gfx950).
//
// All vectors use the field-major layout [f][e][n]; a Krylov vector holds
// the 7 transported fields (length 7 * Ne * np).  Reductions accumulate in
// the vector precision S inside a thread, then in a block tree, then over
// block partials; FP32 vectors therefore use FP32 accumulation throughout.
#pragma once

#include <hip/hip_runtime.h>

#include "dual.hpp"
#include "model.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"

namespace lsbdg {

constexpr int kRedBlocks = 4096;   // partial sums per reduction
constexpr int kMaxDots = 32;       // vectors per multi-dot (restart + 2)

template <typename A, typename B>
__global__ void __launch_bounds__(256) cast_kernel(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    y[i] = B(x[i]);
}

// y = B(scale * x), the product taken in double (scale: a power of two)
template <typename A, typename B>
__global__ void __launch_bounds__(256) scaled_cast_kernel(const A* __restrict__ x, double scale,
                                                          B* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    y[i] = B(scale * double(x[i]));
}

// y = a * x (elementwise) or y = x / a
template <typename S, bool kDiv>
__global__ void __launch_bounds__(256) emul_kernel(const S* __restrict__ a, const S* __restrict__ x,
                                                   S* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    y[i] = kDiv ? x[i] / a[i] : a[i] * x[i];
}

// y = alpha x + beta y
template <typename S>
__global__ void __launch_bounds__(256) axpby_kernel(S alpha, const S* __restrict__ x, S beta,
                                                    S* __restrict__ y, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    y[i] = (alpha == S(0) ? S(0) : alpha * x[i]) + (beta == S(0) ? S(0) : beta * y[i]);
}

template <typename S>
__device__ __forceinline__ S block_sum(S v, S* sh) {
  // 256 threads: wave reduction then across the 4 waves
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// Block sums of acc[0..nv) over 256 threads into partial[i * gridDim + b]:
// for each sum the tree of block_sum (wave shuffle tree, then the four wave
// sums added in order), so the values are those of nv block_sum calls, but
// with one barrier for all of them instead of two per sum.
template <typename S>
__device__ __forceinline__ void store_block_sums(S (&acc)[kMaxDots], int nv, S (*sh)[kMaxDots],
                                                 S* __restrict__ partial) {
#pragma unroll
  for (int i = 0; i < kMaxDots; ++i)
    if (i < nv) {
      S v = acc[i];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      acc[i] = v;
    }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nv) sh[w][i] = acc[i];
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < nv) partial[i * gridDim.x + blockIdx.x] = sh[0][i] + sh[1][i] + sh[2][i] + sh[3][i];
}

// out[i] = sum_b partial[i * nb + b]; one block per i
template <typename S>
__global__ void __launch_bounds__(256) finish_sum_kernel(const S* __restrict__ partial, int nb,
                                                         S* __restrict__ out) {
  __shared__ S sh[4];
  S v = S(0);
  for (int b = threadIdx.x; b < nb; b += 256) v += partial[blockIdx.x * nb + b];
  v = block_sum(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// w -= sum_i h[i] V_i   (h in device memory)
template <typename S>
__global__ void __launch_bounds__(256)
multi_axpy_kernel(const S* __restrict__ V, int64_t ldv, int nv, const S* __restrict__ h, S sign,
                  S* __restrict__ w, int64_t n) {
  struct alignas(4 * sizeof(S)) Q { S a, b, c, d; };
  const int64_t n4 = n >> 2;                 // n, ldv: multiples of 4
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n4; k += int64_t(gridDim.x) * 256) {
    Q acc{S(0), S(0), S(0), S(0)};
    for (int i = 0; i < nv; ++i) {
      const S hi = h[i];
      const Q v = reinterpret_cast<const Q*>(V + i * ldv)[k];
      acc.a += hi * v.a;
      acc.b += hi * v.b;
      acc.c += hi * v.c;
      acc.d += hi * v.d;
    }
    Q wk = reinterpret_cast<Q*>(w)[k];
    wk.a += sign * acc.a;
    wk.b += sign * acc.b;
    wk.c += sign * acc.c;
    wk.d += sign * acc.d;
    reinterpret_cast<Q*>(w)[k] = wk;
  }
}

// partial sums per field f < 7 of a_f * b_f (field stride FS)
template <typename S>
__global__ void __launch_bounds__(256)
field_dot_kernel(const S* __restrict__ a, const S* __restrict__ b, int64_t FS, S* __restrict__ partial) {
  __shared__ S sh[4];
  S acc[7];
#pragma unroll
  for (int f = 0; f < 7; ++f) acc[f] = S(0);
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256) {
#pragma unroll
    for (int f = 0; f < 7; ++f) acc[f] += a[f * FS + k] * b[f * FS + k];
  }
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    const S s = block_sum(acc[f], sh);
    if (threadIdx.x == 0) partial[f * gridDim.x + blockIdx.x] = s;
  }
}

// Coarse correction coefficients yc = Ainv zr with zr = sums of partials.
template <typename S>
__global__ void __launch_bounds__(256)
coarse_solve_kernel(const S* __restrict__ partial, int nb, const double* __restrict__ Ainv,
                    S* __restrict__ yc) {
  __shared__ S sh[4];
  __shared__ double zr[7];
  for (int f = 0; f < 7; ++f) {
    S v = S(0);
    for (int b = threadIdx.x; b < nb; b += 256) v += partial[f * nb + b];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) zr[f] = double(v);
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    double s = 0.0;
    for (int g = 0; g < 7; ++g) s += Ainv[threadIdx.x * 7 + g] * zr[g];
    yc[threadIdx.x] = S(s);
  }
}

// out_f += sc_f * yc_f
template <typename S>
__global__ void __launch_bounds__(256)
coarse_add_kernel(const S* __restrict__ sc, const S* __restrict__ yc, S* __restrict__ out, int64_t FS) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 7 * FS; k += int64_t(gridDim.x) * 256)
    out[k] += sc[k] * yc[k / FS];
}

// t = sc on field f, zero elsewhere (coarse basis vector)
template <typename S>
__global__ void __launch_bounds__(256)
field_select_kernel(const S* __restrict__ sc, int f, S* __restrict__ t, int64_t FS) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 7 * FS; k += int64_t(gridDim.x) * 256)
    t[k] = (k / FS == f) ? sc[k] : S(0);
}

// rhs = -(R_u - y_u) on the 7 transported fields (R in FP64)
template <typename S>
__global__ void __launch_bounds__(256)
condensed_rhs_kernel(const double* __restrict__ R, double scale, const S* __restrict__ y9, S* __restrict__ rhs,
                     int64_t FS, int active) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 7 * FS; k += int64_t(gridDim.x) * 256)
    rhs[k] = ((active >> int(k / FS)) & 1) ? -(S(scale * R[k]) - y9[k]) : S(0);
}

// Zero the inactive fields of a 7-field vector.
template <typename S>
__global__ void __launch_bounds__(256)
mask_fields_kernel(S* __restrict__ a, int64_t FS, int active) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 7 * FS; k += int64_t(gridDim.x) * 256)
    if (!((active >> int(k / FS)) & 1)) a[k] = S(0);
}

// Tab. InitialState concentrations everywhere, Phi_L = 0, solid fractions
// of the voxel's phase.
__global__ void __launch_bounds__(256)
uniform_state_kernel(double* __restrict__ U, const uint8_t* __restrict__ phase, int64_t FS, int np,
                     Conc6 c0, double epsS8_pore, double epsS8_struct, double epsLi2S_pore,
                     double epsLi2S_struct) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256) {
    const int ph = phase[k / np];
#pragma unroll
    for (int f = 0; f < 6; ++f) U[f * FS + k] = c0.c[f];
    U[6 * FS + k] = 0.0;
    U[7 * FS + k] = ph ? epsS8_struct : epsS8_pore;
    U[8 * FS + k] = ph ? epsLi2S_struct : epsLi2S_pore;
  }
}

// v9 = scale (0 on the 7 transported fields, w_R on the solid fractions)
template <typename S>
__global__ void __launch_bounds__(256)
solid_direction_kernel(const double* __restrict__ wR, double scale, S* __restrict__ v9, int64_t FS) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 9 * FS; k += int64_t(gridDim.x) * 256)
    v9[k] = (k < 7 * FS) ? S(0) : S(scale * wR[k - 7 * FS]);
}

// Unknown scales of the 7 transported fields: max(|u_f|, floor_f).
template <typename S>
__global__ void __launch_bounds__(256)
scales_kernel(const double* __restrict__ u, S* __restrict__ sc, int64_t FS, double phi_floor) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 7 * FS; k += int64_t(gridDim.x) * 256) {
    const double x = fabs(u[k]);
    const double fl = (k / FS == 6) ? phi_floor : 1e-20;
    sc[k] = S(x > fl ? x : fl);
  }
}

// w_R at one node (see solid_rhs_kernel).
__device__ __forceinline__ void solid_rhs_node(const double* __restrict__ U, const double* __restrict__ R,
                                               double* __restrict__ wR, const uint8_t* __restrict__ phase,
                                               const DevParams& P, int np, int64_t FS, int64_t k) {
  if (!(P.active & kSolidsBit)) {             // frozen solid fractions
    wR[k] = 0.0;
    wR[FS + k] = 0.0;
    return;
  }
  const int ph = phase[k / np];
  double us[9];
#pragma unroll
  for (int f = 0; f < 9; ++f) us[f] = U[f * FS + k];
  const double W3 = P.W3, idt = P.inv_dt;
  double a00 = P.rhoM[0] * idt, a01 = 0.0, a10 = 0.0, a11 = P.rhoM[1] * idt;
  if (P.react[ph] != 0.0) {
    using D = Dual<double>;
    D x[9], Sx[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) x[f] = D(us[f], f == 7 ? 1.0 : 0.0);
    node_sources(P, ph, x, Sx);
    a00 -= Sx[7].d;
    a10 -= Sx[8].d;
    x[7].d = 0.0;
    x[8].d = 1.0;
    node_sources(P, ph, x, Sx);
    a01 -= Sx[7].d;
    a11 -= Sx[8].d;
  }
  const double r0 = R[7 * FS + k] / W3, r1 = R[8 * FS + k] / W3;
  const double det = a00 * a11 - a01 * a10;
  wR[k] = (a11 * r0 - a01 * r1) / det;
  wR[FS + k] = (a00 * r1 - a10 * r0) / det;
}

// w_R = J_ee^-1 R_eps per node (node-local 2x2, see condense_solids).
__global__ void __launch_bounds__(256)
solid_rhs_kernel(const double* __restrict__ U, const double* __restrict__ R, double* __restrict__ wR,
                 const uint8_t* __restrict__ phase, DevParams P, int np) {
  const int64_t FS = P.Ne * np;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256)
    solid_rhs_node(U, R, wR, phase, P, np, FS, k);
}

// Solid-fraction part of the Newton direction: d_eps = -w_R + w(du).
__global__ void __launch_bounds__(256)
solid_delta_kernel(const double* __restrict__ U, const double* __restrict__ du7,
                   const double* __restrict__ wR, double* __restrict__ deps,
                   const uint8_t* __restrict__ phase, DevParams P, int np) {
  const int64_t FS = P.Ne * np;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256) {
    const int ph = phase[k / np];
    double us[9], vs[7];
#pragma unroll
    for (int f = 0; f < 9; ++f) us[f] = U[f * FS + k];
#pragma unroll
    for (int f = 0; f < 7; ++f) vs[f] = du7[f * FS + k];
    double w0, w1;
    condense_solids(P, ph, us, vs, w0, w1);
    deps[k] = -wR[k] + w0;
    deps[FS + k] = -wR[FS + k] + w1;
  }
}

// u_out = u (+) lam du: positive unknowns multiplicatively, x exp(lam du/x)
// with the exponent clamped to [-ln 10, ln 10] (at most a factor 10 per
// iteration either way, so no unknown collapses to zero or to the scale
// floor in one step); Phi_L and non-positive entries additively.  With
// cross = 1 (steps whose root is limited afterwards) the exponent is
// clamped from above only: an unknown may then fall to zero in one
// iteration (exp underflows) and continue additively, so that the
// iteration can reach a root with negative nodal values.  Also returns
// per-block maxima of |du|/scale (full step).
__global__ void __launch_bounds__(256)
newton_update_kernel(const double* __restrict__ U, const double* __restrict__ dU, double lam,
                     double* __restrict__ Uout, int64_t FS, double phi_floor, double* __restrict__ partial,
                     int cross) {
  __shared__ double sh[4];
  double mx = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 9 * FS; k += int64_t(gridDim.x) * 256) {
    const int f = int(k / FS);
    const double x = U[k], d = dU[k];
    const double fl = (f == 6) ? phi_floor : (f < 6 ? 1e-20 : 1e-12);
    const double s = fabs(x) > fl ? fabs(x) : fl;
    const double rel = fabs(d) / s;
    mx = rel > mx ? rel : mx;
    double y;
    if (f == 6 || !(x > 0.0)) {
      y = x + lam * d;
    } else {
      double ex = lam * d / x;
      ex = ex < 2.302585092994046 ? ex : 2.302585092994046;
      if (!cross) ex = ex > -2.302585092994046 ? ex : -2.302585092994046;
      y = x * exp(ex);
    }
    Uout[k] = y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sh[0];
    for (int i = 1; i < 4; ++i) m = sh[i] > m ? sh[i] : m;
    partial[blockIdx.x] = m;
  }
}

// Merit contributions: sum of squares of x (n entries) into block partials.
template <typename S>
__global__ void __launch_bounds__(256)
sumsq_kernel(const S* __restrict__ x, int64_t n, double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc = 0.0;                          // FP64: no overflow of FP32 squares
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256) {
    const double v = double(x[k]);
    acc += v * v;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Solid rows scaled by their time-term diagonal and the unknown scale.
__global__ void __launch_bounds__(256)
solid_merit_kernel(const double* __restrict__ R, const double* __restrict__ U, int64_t FS, DevParams P,
                   double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 2 * FS; k += int64_t(gridDim.x) * 256) {
    const int s = int(k / FS);
    const double x = fabs(U[(7 + s) * FS + (k % FS)]);
    const double sc = x > 1e-12 ? x : 1e-12;
    const double v = R[7 * FS + k] / (P.W3 * P.rhoM[s] * P.inv_dt * sc);
    if (P.active & kSolidsBit) acc += v * v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// ---- GMRES(m) control on the device ----
//
// The Hessenberg matrix, the Givens rotations, the rotated right side and the
// stopping test of one restart cycle live in device memory and are updated
// by single-workgroup kernels between the vector kernels of an iteration, so
// an iteration needs no read-back: the host learns of convergence from a
// flag it reads one iteration later, and the kernels of an iteration issued
// past convergence change nothing (they test the flag).
struct GmresState {
  double H[kMaxDots * kMaxDots];   // H[i * kMaxDots + j], (m + 1) x m upper Hessenberg
  double cs[kMaxDots], sn[kMaxDots], g[kMaxDots + 1];
  double y[kMaxDots];              // solution of the cycle's least-squares problem
  double beta0;                    // norm of the first residual of the solve
  double rtol;                     // stopping test: |g_{j+1}| <= rtol beta0
  double rel;                      // |g_{j+1}| / beta0 after the last column
  double scale;                    // 1 / norm of the newest basis vector
  int32_t done;                    // cycle finished (converged or breakdown)
  int32_t converged;               // the stopping test held
  int32_t cols;                    // columns of the cycle (j + 1 at the end)
  int32_t its;                     // iterations of the whole solve
  // delayed reorthogonalisation (dcgs_* kernels): the unrotated Hessenberg
  // matrix, the second-pass coefficients c and the norm ratio gam of the
  // newest basis vector (stored once orthogonalised, unit norm), this
  // iteration's first-pass coefficients h1 and the factor alpha
  double Hu[kMaxDots * kMaxDots];
  double c[kMaxDots];
  double h1[kMaxDots];
  double gam, alpha;
};

// Start of a cycle: beta = |r0| from block partials of its square; g = beta
// e_1; the first basis vector is r0 / beta.  first: beta0 = beta.
__global__ void __launch_bounds__(256)
gmres_start_kernel(GmresState* __restrict__ st, const double* __restrict__ partial, int nb, int first,
                   double rtol) {
  __shared__ double sh[4];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) v += partial[b];
  v = block_sum(v, sh);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(v);
  if (first) {
    st->beta0 = beta;
    st->its = 0;
  }
  st->rtol = rtol;
  for (int i = 0; i <= kMaxDots; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->cols = 0;
  st->rel = st->beta0 > 0.0 ? beta / st->beta0 : 0.0;
  const bool ok = beta > 0.0 && isfinite(beta);
  st->done = ok ? 0 : 1;
  st->converged = ok ? 0 : 1;
  st->scale = ok ? 1.0 / beta : 0.0;
  st->gam = 1.0;                   // the first basis vector is exact
}

// ---- Classical Gram-Schmidt applied twice, the second pass delayed ----
//
// The second projection of iteration j is not applied at once: the basis
// vector is stored once orthogonalised, vt_{j+1} = w1 / |w1| (unit norm),
// with its second-pass coefficients c = h2 / |w1| and gam = |w2| / |w1|
// (|w2|^2 = |w1|^2 - |h2|^2 for orthonormal V).  The next iteration applies
// the operator to vt_{j+1}, z = A vt_{j+1}, and in one sweep over the basis
// both corrects the vector, v_{j+1} = (vt_{j+1} - V c) / gam, and forms the
// projections V^T z and vt^T z.  Since A v = (z - A V c) / gam and, by the
// Arnoldi relation of the earlier columns (unrotated Hessenberg Hu),
// A V c = V (Hu c), the first-pass coefficients of A v_{j+1} follow from those
// dots without another sweep, and one further sweep forms w1 and its
// second-pass projections.  Two sweeps over the basis per iteration instead
// of three; in exact arithmetic the iterates are those of the undelayed
// method.

// Sweep 1 of iteration j: V_j <- (V_j - sum_{i<j} c_i V_i) / gam (skipped
// once the cycle is done), with partial sums of V_i . z (i < j) and of the
// uncorrected V_j . z (slot j).
template <typename S>
__global__ void __launch_bounds__(256)
dcgs_sweep1_kernel(const GmresState* __restrict__ st, S* __restrict__ V, int64_t ldv, int j,
                   const S* __restrict__ z, int64_t n, S* __restrict__ partial) {
  struct alignas(4 * sizeof(S)) Q { S a, b, c, d; };
  __shared__ S sh[4][kMaxDots];
  const bool write = !st->done;
  S cs[kMaxDots];
#pragma unroll
  for (int i = 0; i < kMaxDots; ++i) cs[i] = i < j ? S(st->c[i]) : S(0);
  const S ig = S(1.0 / st->gam);
  S acc[kMaxDots];
#pragma unroll
  for (int i = 0; i < kMaxDots; ++i) acc[i] = S(0);
  const int64_t n4 = n >> 2;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n4; k += int64_t(gridDim.x) * 256) {
    const Q zk = reinterpret_cast<const Q*>(z)[k];
    const Q vt = reinterpret_cast<const Q*>(V + j * ldv)[k];
    Q s{S(0), S(0), S(0), S(0)};
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < j) {
        const Q v = reinterpret_cast<const Q*>(V + i * ldv)[k];
        acc[i] += v.a * zk.a + v.b * zk.b + v.c * zk.c + v.d * zk.d;
        s.a += cs[i] * v.a;
        s.b += cs[i] * v.b;
        s.c += cs[i] * v.c;
        s.d += cs[i] * v.d;
      }
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i == j) acc[i] += vt.a * zk.a + vt.b * zk.b + vt.c * zk.c + vt.d * zk.d;
    if (write && j > 0) {
      Q o;
      o.a = (vt.a - s.a) * ig;
      o.b = (vt.b - s.b) * ig;
      o.c = (vt.c - s.c) * ig;
      o.d = (vt.d - s.d) * ig;
      reinterpret_cast<Q*>(V + j * ldv)[k] = o;
    }
  }
  store_block_sums(acc, j + 1, sh, partial);
}

// Coefficients of iteration j from sweep 1's sums d (d_i = V_i . z, i < j;
// d_j = vt_j . z): g = Hu[0..j, 0..j-1] c, V^T z with (V^T z)_j =
// (d_j - c . d) / gam, h1 = (V^T z - g) / gam (kept in the state), and
// sweep 2's w1 = alpha z - V beta with alpha = 1 / gam, beta = g / gam + h1.
// One thread; no-op once the cycle is done.
template <typename S>
__global__ void __launch_bounds__(64)
dcgs_coef_kernel(GmresState* __restrict__ st, const S* __restrict__ d, int j, S* __restrict__ beta) {
  if (threadIdx.x != 0 || st->done) return;
  const double gam = st->gam;
  double cd = 0.0;
  for (int i = 0; i < j; ++i) cd += st->c[i] * double(d[i]);
  for (int k = 0; k <= j; ++k) {
    double g = 0.0;
    for (int i = 0; i < j; ++i) g += st->Hu[k * kMaxDots + i] * st->c[i];
    const double vz = k < j ? double(d[k]) : (double(d[j]) - cd) / gam;
    const double h1 = (vz - g) / gam;
    st->h1[k] = h1;
    beta[k] = S(g / gam + h1);
  }
  st->alpha = 1.0 / gam;
}

// Sweep 2 of iteration j: w <- alpha w - sum_{i<nv} beta_i V_i (w holds z on
// entry), with partial sums of V_i . w (the second-pass projections) and
// FP64 partial sums of |w|^2.
template <typename S>
__global__ void __launch_bounds__(256)
dcgs_sweep2_kernel(const GmresState* __restrict__ st, const S* __restrict__ V, int64_t ldv, int nv,
                   const S* __restrict__ beta, S* __restrict__ w, int64_t n, S* __restrict__ partial,
                   double* __restrict__ partial64) {
  struct alignas(4 * sizeof(S)) Q { S a, b, c, d; };
  __shared__ S sh[4][kMaxDots];
  __shared__ double sh64[4];
  const S al = S(st->alpha);
  S acc[kMaxDots];
#pragma unroll
  for (int i = 0; i < kMaxDots; ++i) acc[i] = S(0);
  double nrm = 0.0;
  const int64_t n4 = n >> 2;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n4; k += int64_t(gridDim.x) * 256) {
    Q vq[kMaxDots];
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nv) vq[i] = reinterpret_cast<const Q*>(V + i * ldv)[k];
    Q s{S(0), S(0), S(0), S(0)};
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nv) {
        const S bi = beta[i];
        s.a += bi * vq[i].a;
        s.b += bi * vq[i].b;
        s.c += bi * vq[i].c;
        s.d += bi * vq[i].d;
      }
    Q wk = reinterpret_cast<Q*>(w)[k];
    wk.a = al * wk.a - s.a;
    wk.b = al * wk.b - s.b;
    wk.c = al * wk.c - s.c;
    wk.d = al * wk.d - s.d;
    reinterpret_cast<Q*>(w)[k] = wk;
#pragma unroll
    for (int i = 0; i < kMaxDots; ++i)
      if (i < nv) acc[i] += vq[i].a * wk.a + vq[i].b * wk.b + vq[i].c * wk.c + vq[i].d * wk.d;
    const double a = double(wk.a), b = double(wk.b), c = double(wk.c), d = double(wk.d);
    nrm += a * a;
    nrm += b * b;
    nrm += c * c;
    nrm += d * d;
  }
  store_block_sums(acc, nv, sh, partial);
  const double t = block_sum(nrm, sh64);
  if (threadIdx.x == 0) partial64[blockIdx.x] = t;
}

// Column j from sweep 2's sums gs = [|w1|^2 (FP64)][.. (kMaxDots x S)][h2
// (kMaxDots x S)]: Hu[:, j] = h1 + h2, Hu[j+1, j] = |w2| = sqrt(|w1|^2 -
// |h2|^2); the rotations, the rotated right side and the stopping test as
// gmres_column_kernel; then c = h2 / |w1|, gam = |w2| / |w1| and the scale
// 1 / |w1| of the next (once orthogonalised) basis vector.  One thread;
// no-op once the cycle is done.
template <typename S>
__global__ void __launch_bounds__(64)
dcgs_column_kernel(GmresState* __restrict__ st, const double* __restrict__ gs, int j, int m) {
  if (threadIdx.x != 0 || st->done) return;
  const S* h2 = reinterpret_cast<const S*>(gs + 1) + kMaxDots;
  double* H = st->H;
  const double nw1 = sqrt(gs[0]);
  double h2sq = 0.0;
  for (int i = 0; i <= j; ++i) {
    const double h = double(h2[i]);
    h2sq += h * h;
    st->Hu[i * kMaxDots + j] = st->h1[i] + h;
    H[i * kMaxDots + j] = st->h1[i] + h;
  }
  const double w2sq = gs[0] - h2sq;
  const double hn = w2sq > 0.0 ? sqrt(w2sq) : 0.0;
  st->Hu[(j + 1) * kMaxDots + j] = hn;
  for (int i = j + 2; i < kMaxDots; ++i) st->Hu[i * kMaxDots + j] = 0.0;   // Hessenberg: below is zero
  H[(j + 1) * kMaxDots + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = H[i * kMaxDots + j], c = H[(i + 1) * kMaxDots + j];
    H[i * kMaxDots + j] = st->cs[i] * a + st->sn[i] * c;
    H[(i + 1) * kMaxDots + j] = -st->sn[i] * a + st->cs[i] * c;
  }
  const double a = H[j * kMaxDots + j], c = H[(j + 1) * kMaxDots + j];
  const double rr = hypot(a, c);
  st->cs[j] = rr > 0.0 ? a / rr : 1.0;
  st->sn[j] = rr > 0.0 ? c / rr : 0.0;
  H[j * kMaxDots + j] = rr;
  H[(j + 1) * kMaxDots + j] = 0.0;
  st->g[j + 1] = -st->sn[j] * st->g[j];
  st->g[j] = st->cs[j] * st->g[j];
  st->rel = fabs(st->g[j + 1]) / st->beta0;
  st->cols = j + 1;
  st->its += 1;
  const bool conv = st->rel <= st->rtol;
  if (conv || !(hn > 0.0) || !(nw1 > 0.0) || j + 1 == m) {
    st->done = 1;
    st->converged = conv ? 1 : 0;
  } else {
    for (int i = 0; i <= j; ++i) st->c[i] = double(h2[i]) / nw1;
    st->gam = hn / nw1;
    st->scale = 1.0 / nw1;
  }
}

// y = scale * x with the scale of the state (next basis vector); no-op once
// the cycle is done (and in place for the first vector).
template <typename S>
__global__ void __launch_bounds__(256)
gmres_scale_kernel(const GmresState* __restrict__ st, const S* __restrict__ x, S* __restrict__ y, int64_t n) {
  if (st->done && x != y) return;
  const S a = S(st->scale);
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    y[i] = a * x[i];
}

// Back substitution H y = g on the cycle's cols x cols upper triangle; y in
// the state (FP64) and as S for the update x += V y.
template <typename S>
__global__ void __launch_bounds__(64)
gmres_solve_kernel(GmresState* __restrict__ st, S* __restrict__ ys) {
  if (threadIdx.x != 0) return;
  const int k = st->cols;
  for (int i = k - 1; i >= 0; --i) {
    double s = st->g[i];
    for (int c = i + 1; c < k; ++c) s -= st->H[i * kMaxDots + c] * st->y[c];
    st->y[i] = s / st->H[i * kMaxDots + i];
  }
  for (int i = 0; i < k; ++i) ys[i] = S(st->y[i]);
}

}  // namespace lsbdg
