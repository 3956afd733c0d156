// Multilevel aggregation coarse correction of the Krylov preconditioner:
// the GPU stand-in for the algebraic multigrid with which the paper
// preconditions its linear solves (Sec. 2.9).
//
// Hierarchy.  Level 1 is the aggregation coarse space of coarse.hpp:
// aggregates of A x A x A voxels, basis Z_{f,a} = the unknown scales of
// field f on the nodes of aggregate a.  Level l + 1 groups the level-l
// aggregates 2 x 2 x 2 by their integer coordinates (parent = a / 2 per
// axis), with the 0/1 prolongation P_l that copies a parent's value to its
// children.  The operators are Galerkin products, E_1 = Z^T J Z and
// E_{l+1} = P_l^T E_l P_l.  J couples a voxel to its six face neighbours
// only, so every E_l couples an aggregate to itself and its six face
// neighbours: it is stored as a stencil of seven 7 x 7 blocks per
// aggregate, E[s][g][f][a] (slot s = self, -x, +x, -y, +y, -z, +z; row
// field g, column field f; aggregate fastest, so a thread per aggregate
// reads each entry coalesced).  Coarse vectors are field-major, x[f][a].
//
// Cycle.  On every level but the last: nu damped block-Jacobi sweeps
// x <- x + omega D^-1 (b - E x) from x = 0 (D: the self blocks), the next
// level's cycle on the restricted residual P^T (b - E x), its prolongation
// added to x, nu more sweeps.  The last level is solved exactly with the
// explicit inverse of its equilibrated dense operator (coarse.hpp).
//
// All level arithmetic is FP64, whatever the Krylov precision: the
// levels are small next to the fine vectors, and their operators span the
// magnitudes of the whole system.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "coarse.hpp"

namespace lsbdg {

constexpr int kMgMaxLevels = 8;

struct MgGrid {
  int32_t ax, ay, az, pad;
  int64_t na;
};

__host__ __device__ inline MgGrid mg_coarser(const MgGrid& g) {
  MgGrid c{};
  c.ax = (g.ax + 1) / 2;
  c.ay = (g.ay + 1) / 2;
  c.az = (g.az + 1) / 2;
  c.na = int64_t(c.ax) * c.ay * c.az;
  return c;
}

// Neighbour of aggregate (x, y, z) in stencil slot s (0: itself), or -1.
__device__ __forceinline__ int64_t mg_neighbour(const MgGrid& g, int x, int y, int z, int s) {
  if (s == 1) --x;
  else if (s == 2) ++x;
  else if (s == 3) --y;
  else if (s == 4) ++y;
  else if (s == 5) --z;
  else if (s == 6) ++z;
  if (x < 0 || y < 0 || z < 0 || x >= g.ax || y >= g.ay || z >= g.az) return -1;
  return int64_t(x) + int64_t(g.ax) * (y + int64_t(g.ay) * z);
}

// One thread per item (the level kernels below have no grid-stride loop).
inline dim3 mg_grid(int64_t n) { return dim3{unsigned((n + 255) / 256), 1, 1}; }

__device__ __forceinline__ int64_t mg_entry(int s, int g, int f, int64_t a, int64_t na) {
  return (int64_t((s * 7 + g) * 7 + f)) * na + a;
}

// x[k] = v for k < n (grid-stride).  Used instead of a memset so that the
// clears stay kernels.
template <typename T>
__global__ void __launch_bounds__(256) mg_fill_kernel(T* __restrict__ x, int64_t n, T v) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256) x[k] = v;
}

// Level-1 stencil entries from the probe product Jv of colour c, field f:
// for aggregate b (one workgroup each), the unique aggregate a* of colour c
// in b's stencil, at slot s*, gives E_1[s*][g][f][b] = sum over b's nodes
// of sc_g (J v)_g.  Every entry is written by exactly one (f, c) probe; the
// slots that no neighbour fills stay as cleared.
template <typename S>
__global__ void __launch_bounds__(256)
mg_probe_stencil_kernel(const S* __restrict__ sc, const S* __restrict__ Jv, int f, int c, AggGrid G, int64_t FS,
                        double* __restrict__ E1) {
  __shared__ double sh[7][4];
  const int64_t b = blockIdx.x;
  const int bx = int(b % G.nax), by = int((b / G.nax) % G.nay), bz = int(b / (int64_t(G.nax) * G.nay));
  int sstar = -1;
  {
    const int d[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    for (int s = 0; s < 7; ++s) {
      const int ax = bx + d[s][0], ay = by + d[s][1], az = bz + d[s][2];
      if (ax < 0 || ay < 0 || az < 0 || ax >= G.nax || ay >= G.nay || az >= G.naz) continue;
      if (agg_colour(ax, ay, az) == c) sstar = s;
    }
  }
  if (sstar < 0) return;                      // whole block: nothing of colour c reaches b
  double acc[7];
  agg_sums(sc, Jv, G, FS, bx, by, bz, acc);
  block_sum7(acc, sh);
  if (threadIdx.x < 7) E1[mg_entry(sstar, threadIdx.x, f, b, G.na)] = acc[threadIdx.x];
}

// Galerkin product E_c = P^T E_f P, one thread per coarse aggregate and
// block entry (g, f): the children's blocks are summed into the self slot
// when the neighbour they couple to has the same parent, into slot s
// otherwise (that neighbour's parent is then the coarse neighbour in
// direction s).
__global__ void __launch_bounds__(256)
mg_galerkin_kernel(const double* __restrict__ Ef, MgGrid gf, double* __restrict__ Ec, MgGrid gc) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= 49 * gc.na) return;
  const int gfp = int(k / gc.na);             // g * 7 + f
  const int64_t A = k - int64_t(gfp) * gc.na;
  const int g = gfp / 7, f = gfp % 7;
  const int X = int(A % gc.ax), Y = int((A / gc.ax) % gc.ay), Z = int(A / (int64_t(gc.ax) * gc.ay));
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int cz = 2 * Z; cz < min(2 * Z + 2, gf.az); ++cz)
    for (int cy = 2 * Y; cy < min(2 * Y + 2, gf.ay); ++cy)
      for (int cx = 2 * X; cx < min(2 * X + 2, gf.ax); ++cx) {
        const int64_t a = int64_t(cx) + int64_t(gf.ax) * (cy + int64_t(gf.ay) * cz);
#pragma unroll
        for (int s = 0; s < 7; ++s) {
          int nx = cx, ny = cy, nz = cz;
          if (s == 1) --nx;
          else if (s == 2) ++nx;
          else if (s == 3) --ny;
          else if (s == 4) ++ny;
          else if (s == 5) --nz;
          else if (s == 6) ++nz;
          if (nx < 0 || ny < 0 || nz < 0 || nx >= gf.ax || ny >= gf.ay || nz >= gf.az) continue;
          const bool inside = (nx >> 1) == X && (ny >> 1) == Y && (nz >> 1) == Z;
          const double v = Ef[mg_entry(s, g, f, a, gf.na)];
          if (inside) acc[0] += v;
          else acc[s] += v;
        }
      }
#pragma unroll
  for (int s = 0; s < 7; ++s) Ec[mg_entry(s, g, f, A, gc.na)] = acc[s];
}

// Inverses of the self blocks, Dinv[g][f][a], one thread per aggregate:
// Gauss-Jordan with partial pivoting on [E_aa | I] held in registers (row
// exchanges by selects over fixed indices, so nothing is indexed at run
// time).  A column without a nonzero pivot (a field with no equation on
// this aggregate: an inactive field) takes pivot 1, so that its unknown is
// left to its right side.
__global__ void __launch_bounds__(256)
mg_block_inverse_kernel(const double* __restrict__ E, int64_t na, double* __restrict__ Dinv) {
  const int64_t a = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (a >= na) return;
  double M[7][14];
#pragma unroll
  for (int g = 0; g < 7; ++g)
#pragma unroll
    for (int f = 0; f < 14; ++f) M[g][f] = f < 7 ? E[mg_entry(0, g, f, a, na)] : (f - 7 == g ? 1.0 : 0.0);
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    int p = k;
    double best = fabs(M[k][k]);
#pragma unroll
    for (int i = k + 1; i < 7; ++i)
      if (fabs(M[i][k]) > best) {
        best = fabs(M[i][k]);
        p = i;
      }
#pragma unroll
    for (int i = k + 1; i < 7; ++i) {
      if (i == p) {
#pragma unroll
        for (int j = 0; j < 14; ++j) {
          const double t = M[k][j];
          M[k][j] = M[i][j];
          M[i][j] = t;
        }
      }
    }
    if (!(best > 0.0) || !isfinite(best)) M[k][k] = 1.0;
    const double ip = 1.0 / M[k][k];
#pragma unroll
    for (int j = 0; j < 14; ++j) M[k][j] *= ip;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      if (i == k) continue;
      const double m = M[i][k];
#pragma unroll
      for (int j = 0; j < 14; ++j) M[i][j] -= m * M[k][j];
    }
  }
#pragma unroll
  for (int g = 0; g < 7; ++g)
#pragma unroll
    for (int f = 0; f < 7; ++f) Dinv[(int64_t(g) * 7 + f) * na + a] = M[g][7 + f];
}

// r = b - E x on one aggregate (x == nullptr: x = 0).
__device__ __forceinline__ void mg_row_residual(const double* __restrict__ E, const MgGrid& gr,
                                                const double* __restrict__ b, const double* __restrict__ x,
                                                int64_t a, double* r) {
#pragma unroll
  for (int g = 0; g < 7; ++g) r[g] = b[int64_t(g) * gr.na + a];
  if (!x) return;
  const int X = int(a % gr.ax), Y = int((a / gr.ax) % gr.ay), Z = int(a / (int64_t(gr.ax) * gr.ay));
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int64_t nb = mg_neighbour(gr, X, Y, Z, s);
    if (nb < 0) continue;
    double xv[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) xv[f] = x[int64_t(f) * gr.na + nb];
#pragma unroll
    for (int g = 0; g < 7; ++g) {
      double acc = 0.0;
#pragma unroll
      for (int f = 0; f < 7; ++f) acc += E[mg_entry(s, g, f, a, gr.na)] * xv[f];
      r[g] -= acc;
    }
  }
}

// One damped block-Jacobi sweep: xo = x + omega Dinv (b - E x), one thread
// per aggregate (x == nullptr: from x = 0).
__global__ void __launch_bounds__(256)
mg_smooth_kernel(const double* __restrict__ E, const double* __restrict__ Dinv, MgGrid gr,
                 const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ xo,
                 double omega) {
  const int64_t a = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (a >= gr.na) return;
  double r[7];
  mg_row_residual(E, gr, b, x, a, r);
#pragma unroll
  for (int g = 0; g < 7; ++g) {
    double acc = 0.0;
#pragma unroll
    for (int f = 0; f < 7; ++f) acc += Dinv[(int64_t(g) * 7 + f) * gr.na + a] * r[f];
    xo[int64_t(g) * gr.na + a] = (x ? x[int64_t(g) * gr.na + a] : 0.0) + omega * acc;
  }
}

// Restricted residual bc = P^T (b - E x), one thread per coarse aggregate:
// the residuals of its (up to eight) children, summed.
__global__ void __launch_bounds__(256)
mg_residual_restrict_kernel(const double* __restrict__ E, MgGrid gf, const double* __restrict__ b,
                            const double* __restrict__ x, MgGrid gc, double* __restrict__ bc) {
  const int64_t A = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (A >= gc.na) return;
  const int X = int(A % gc.ax), Y = int((A / gc.ax) % gc.ay), Z = int(A / (int64_t(gc.ax) * gc.ay));
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int cz = 2 * Z; cz < min(2 * Z + 2, gf.az); ++cz)
    for (int cy = 2 * Y; cy < min(2 * Y + 2, gf.ay); ++cy)
      for (int cx = 2 * X; cx < min(2 * X + 2, gf.ax); ++cx) {
        const int64_t a = int64_t(cx) + int64_t(gf.ax) * (cy + int64_t(gf.ay) * cz);
        double r[7];
        mg_row_residual(E, gf, b, x, a, r);
#pragma unroll
        for (int g = 0; g < 7; ++g) acc[g] += r[g];
      }
#pragma unroll
  for (int g = 0; g < 7; ++g) bc[int64_t(g) * gc.na + A] = acc[g];
}

// x[g][a] += xc[g][parent(a)], one thread per aggregate of the finer level.
__global__ void __launch_bounds__(256)
mg_prolong_add_kernel(const double* __restrict__ xc, MgGrid gc, MgGrid gf, double* __restrict__ x) {
  const int64_t a = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (a >= gf.na) return;
  const int X = int(a % gf.ax), Y = int((a / gf.ax) % gf.ay), Z = int(a / (int64_t(gf.ax) * gf.ay));
  const int64_t A = int64_t(X >> 1) + int64_t(gc.ax) * ((Y >> 1) + int64_t(gc.ay) * (Z >> 1));
#pragma unroll
  for (int g = 0; g < 7; ++g) x[int64_t(g) * gf.na + a] += xc[int64_t(g) * gc.na + A];
}

// Dense column-major form of a level's stencil operator, D[(g na + a) +
// nc (f na + nb(a, s))] = E[s][g][f][a] (D cleared beforehand), one thread
// per stencil entry.
__global__ void __launch_bounds__(256)
mg_dense_kernel(const double* __restrict__ E, MgGrid gr, double* __restrict__ D) {
  const int64_t total = 343 * gr.na;
  const int64_t nc = 7 * gr.na;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int sgf = int(k / gr.na);
    const int64_t a = k - int64_t(sgf) * gr.na;
    const int s = sgf / 49, g = (sgf / 7) % 7, f = sgf % 7;
    const int X = int(a % gr.ax), Y = int((a / gr.ax) % gr.ay), Z = int(a / (int64_t(gr.ax) * gr.ay));
    const int64_t nb = mg_neighbour(gr, X, Y, Z, s);
    if (nb < 0) continue;
    D[(int64_t(g) * gr.na + a) + nc * (int64_t(f) * gr.na + nb)] = E[k];
  }
}

}  // namespace lsbdg
