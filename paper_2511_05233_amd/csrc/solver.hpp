// Newton-Krylov solve of one backward-Euler step (host orchestration).
//
// Outer loop in FP64 (residual, condensed right side, update, line search,
// convergence test); inner GMRES(m) in the precision S with classical
// Gram-Schmidt applied twice.  The Krylov operator is the condensed 7-field
// Jacobian, scaled by the unknown magnitudes sc (so every Krylov vector is
// O(1), far from the FP32 range limits although raw residual entries are
// ~1e-20), deflated by a global per-field coarse space and left-
// preconditioned by the element blocks B.
//
// Deflation: with Z_f = sc on field f, E = Z^T J Z (7 x 7) and
// P = I - J Z E^-1 Z^T, GMRES solves  sc^-1 B^-1 P J sc y = sc^-1 B^-1 P rhs
// and the correction is
//     du = xhat + Z E^-1 Z^T (rhs - J xhat),  xhat = sc y,
// so its coarse component (a near-null mode: the level of Phi_L with the
// species in quasi-equilibrium, which only the reaction current resists) is
// solved exactly instead of to the GMRES tolerance, and the coarse part of
// J du - rhs vanishes.
//
// Condensed right side: with w_R = J_ee^-1 R_eps (node-local),
//     rhs = -(R_u - J_ue w_R),   and afterwards  d_eps = -w_R + w(du),
// which is Newton's direction of the full 9-field system.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "krylov.hpp"

namespace lsbdg {

// A caller-owned device workspace: buffers are carved from it in order,
// 256-byte aligned, and never freed or moved (a carved buffer cannot grow).
struct Arena {
  unsigned char* base = nullptr;
  size_t size = 0, used = 0;
  size_t short_by = 0;              // bytes missing at the last failed request
  static size_t aligned(size_t n) { return (n + 255) & ~size_t(255); }
};

// Device buffer: hipMalloc'd by the library, or carved from an Arena.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* arena = nullptr;
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
  hipError_t ensure(size_t n) {
    if (bytes >= n) return hipSuccess;
    if (arena) {
      if (p) {                      // sized once; a different size means another use than planned
        arena->short_by = n - bytes;
        return hipErrorOutOfMemory;
      }
      const size_t off = Arena::aligned(arena->used);
      if (off + n > arena->size) {
        arena->short_by = off + n - arena->size;
        return hipErrorOutOfMemory;
      }
      p = arena->base + off;
      arena->used = off + n;
      bytes = n;
      return hipSuccess;
    }
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  void release() {
    if (p && !arena) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct SolverWork {
  DevBuf m_old, R, Rtry, u_try, du, wR;            // FP64
  DevBuf uS, sc, V, w, t, pJ, rhs, b, x, y9, v9, JZ;   // precision S
  DevBuf partial, partial64, dots, yc, Ainv, hbuf;
  DevBuf gsum;                                     // one Gram-Schmidt step's sums: [|w|^2][h1][h2]
  DevBuf z0, zC, zF, out_partial;                  // time controller, outputs (FP64)
  DevBuf pc, pc2, scc;                             // two-level preconditioner temporaries, scales (S)
  DevBuf gstate;                                   // GMRES cycle state on the device (GmresState)
  DevBuf lmean;                                    // limiter: voxel means of eps_L c_i (FP64, 6 x Ne)
  int m = 0;
  template <typename F>
  void for_each(F f) {
    for (DevBuf* d : {&m_old, &R, &Rtry, &u_try, &du, &wR, &uS, &sc, &V, &w, &t, &pJ, &rhs, &b, &x,
                      &y9, &v9, &JZ, &partial, &partial64, &dots, &yc, &Ainv, &hbuf, &z0, &zC, &zF,
                      &out_partial, &pc, &pc2, &scc, &gsum, &gstate, &lmean})
      f(*d);
  }
  void release_all() {
    for (DevBuf* d : {&m_old, &R, &Rtry, &u_try, &du, &wR, &uS, &sc, &V, &w, &t, &pJ, &rhs, &b, &x,
                      &y9, &v9, &JZ, &partial, &partial64, &dots, &yc, &Ainv, &hbuf, &z0, &zC, &zF,
                      &out_partial, &pc, &pc2, &scc, &gsum, &gstate, &lmean})
      d->release();
  }
};

inline dim3 grid1(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return dim3{unsigned(b), 1, 1};
}

// Small dense solve with partial pivoting (host, double).  Returns false if
// singular.
inline bool dense_solve(int n, std::vector<double> A, std::vector<double>& x) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (!(std::fabs(A[p * n + k]) > 0.0)) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(x[k], x[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      x[i] -= f * x[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * x[j];
    x[i] = s / A[i * n + i];
  }
  return true;
}

}  // namespace lsbdg
