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
// aggregate (slot s = self, -x, +x, -y, +y, -z, +z; row field g, column
// field f).  Every level kernel runs eight lanes per aggregate, lane g
// owning row g (lane 7 carries a zero pad), so the layouts put the row
// index innermost: E[s][f][a][8], Dinv[f][a][8] and level vectors x[a][8]
// (pad entries zero).  A lane loads one entry of its neighbour's vector
// and the group shares the seven by cross-lane reads.
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

// Entry (row g, column f) of slot s of aggregate a in E[s][f][a][8].
__device__ __forceinline__ int64_t mg_entry(int s, int g, int f, int64_t a, int64_t na) {
  return ((int64_t(s * 7 + f)) * na + a) * 8 + g;
}

// x[k] = v for k < n (grid-stride).  Used instead of a memset so that the
// clears stay kernels.
template <typename T>
__global__ void __launch_bounds__(256) mg_fill_kernel(T* __restrict__ x, int64_t n, T v) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256) x[k] = v;
}

// Fine-to-level-1 restriction b[a][g] = sum over aggregate a's nodes of
// sc_g r_g (Z^T r), one workgroup per aggregate; the pad entry set to zero.
template <typename S>
__global__ void __launch_bounds__(256)
mg_restrict_fine_kernel(const S* __restrict__ sc, const S* __restrict__ r, AggGrid G, int64_t FS,
                        double* __restrict__ b) {
  __shared__ double sh[7][4];
  const int64_t a = blockIdx.x;
  const int ax = int(a % G.nax), ay = int((a / G.nax) % G.nay), az = int(a / (int64_t(G.nax) * G.nay));
  double acc[7];
  agg_sums(sc, r, G, FS, ax, ay, az, acc);
  block_sum7(acc, sh);
  if (threadIdx.x < 8) b[a * 8 + threadIdx.x] = threadIdx.x < 7 ? acc[threadIdx.x] : 0.0;
}

// Level-1-to-fine prolongation out += Z y (y[a][8]), or out = Z y when
// set, one thread per node; div (optional): the result divided entrywise
// by div in the same pass.
template <typename S>
__global__ void __launch_bounds__(256)
mg_prolong_fine_kernel(const S* __restrict__ sc, const double* __restrict__ y, AggGrid G, int64_t FS,
                       S* __restrict__ out, const S* __restrict__ div, bool set = false) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256) {
    const int64_t a = agg_of_voxel(G, k >> 3);
#pragma unroll
    for (int g = 0; g < 7; ++g) {
      const S v = (set ? S(0) : out[g * FS + k]) + sc[g * FS + k] * S(y[a * 8 + g]);
      out[g * FS + k] = div ? v / div[g * FS + k] : v;
    }
  }
}

// Level-1 stencil entries from the probe product Jv of colour c, field f:
// for aggregate b (one workgroup each), the unique aggregate a* of colour c
// in b's stencil, at slot s*, gives column f of slot s* of b's rows,
// sum over b's nodes of sc_g (J v)_g.  Every entry is written by exactly
// one (f, c) probe; the slots that no neighbour fills stay as cleared.
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

// Galerkin product E_c = P^T E_f P, one thread per (column field f, coarse
// aggregate A, row g; pad rows written zero): the children's entries are
// summed into the self slot when the neighbour they couple to has the same
// parent, into slot s otherwise (that neighbour's parent is then the
// coarse neighbour in direction s).
__global__ void __launch_bounds__(256)
mg_galerkin_kernel(const double* __restrict__ Ef, MgGrid gf, double* __restrict__ Ec, MgGrid gc) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= 56 * gc.na) return;
  const int g = int(t & 7);
  const int64_t q = t >> 3;
  const int f = int(q / gc.na);
  const int64_t A = q - int64_t(f) * gc.na;
  const int X = int(A % gc.ax), Y = int((A / gc.ax) % gc.ay), Z = int(A / (int64_t(gc.ax) * gc.ay));
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if (g < 7) {
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
  }
#pragma unroll
  for (int s = 0; s < 7; ++s) Ec[mg_entry(s, g, f, A, gc.na)] = acc[s];
}

// Inverses of the self blocks, Dinv[f][a][8] (row g innermost, pad zero),
// one thread per aggregate: Gauss-Jordan with partial pivoting on
// [E_aa | I] held in registers (row exchanges by selects over fixed
// indices, so nothing is indexed at run time).  A column without a nonzero
// pivot (a field with no equation on this aggregate: an inactive field)
// takes pivot 1, so that its unknown is left to its right side.
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
  for (int f = 0; f < 7; ++f) {
#pragma unroll
    for (int g = 0; g < 7; ++g) Dinv[(int64_t(f) * na + a) * 8 + g] = M[g][7 + f];
    Dinv[(int64_t(f) * na + a) * 8 + 7] = 0.0;
  }
}

// Row g of b - E x on aggregate a (x == nullptr: x = 0), for lane g of the
// aggregate's group of eight: each lane loads entry g of a neighbour's
// iterate and the group exchanges them (slots without a neighbour hold
// zero entries, so every lane takes every step).
__device__ __forceinline__ double mg_row_residual(const double* __restrict__ E, const MgGrid& gr,
                                                  const double* __restrict__ b, const double* __restrict__ x,
                                                  int64_t a, int g) {
  double r = b[a * 8 + g];
  if (!x) return r;
  const int X = int(a % gr.ax), Y = int((a / gr.ax) % gr.ay), Z = int(a / (int64_t(gr.ax) * gr.ay));
#pragma unroll
  for (int s = 0; s < 7; ++s) {
    const int64_t nb = mg_neighbour(gr, X, Y, Z, s);
    const double xg = nb >= 0 ? x[nb * 8 + g] : 0.0;
#pragma unroll
    for (int f = 0; f < 7; ++f) r -= E[mg_entry(s, g, f, a, gr.na)] * __shfl(xg, f, 8);
  }
  return r;
}

// One damped block-Jacobi sweep xo = x + omega Dinv (b - E x), eight lanes
// per aggregate (x == nullptr: from x = 0).
__global__ void __launch_bounds__(256)
mg_smooth_kernel(const double* __restrict__ E, const double* __restrict__ Dinv, MgGrid gr,
                 const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ xo,
                 double omega) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= 8 * gr.na) return;                 // whole groups of eight leave together
  const int64_t a = t >> 3;
  const int g = int(t & 7);
  const double r = mg_row_residual(E, gr, b, x, a, g);
  double acc = 0.0;
#pragma unroll
  for (int f = 0; f < 7; ++f) acc += Dinv[(int64_t(f) * gr.na + a) * 8 + g] * __shfl(r, f, 8);
  xo[t] = (x ? x[t] : 0.0) + omega * acc;
}

// Residual r = b - E x of a level, eight lanes per aggregate.
__global__ void __launch_bounds__(256)
mg_residual_kernel(const double* __restrict__ E, MgGrid gr, const double* __restrict__ b,
                   const double* __restrict__ x, double* __restrict__ r) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= 8 * gr.na) return;
  r[t] = mg_row_residual(E, gr, b, x, t >> 3, int(t & 7));
}

// Restriction bc = P^T r: entry g of coarse aggregate A sums its (up to
// eight) children's, one thread per (A, g).
__global__ void __launch_bounds__(256)
mg_restrict_kernel(const double* __restrict__ r, MgGrid gf, MgGrid gc, double* __restrict__ bc) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= 8 * gc.na) return;
  const int64_t A = t >> 3;
  const int g = int(t & 7);
  const int X = int(A % gc.ax), Y = int((A / gc.ax) % gc.ay), Z = int(A / (int64_t(gc.ax) * gc.ay));
  double acc = 0.0;
  for (int cz = 2 * Z; cz < min(2 * Z + 2, gf.az); ++cz)
    for (int cy = 2 * Y; cy < min(2 * Y + 2, gf.ay); ++cy)
      for (int cx = 2 * X; cx < min(2 * X + 2, gf.ax); ++cx)
        acc += r[(int64_t(cx) + int64_t(gf.ax) * (cy + int64_t(gf.ay) * cz)) * 8 + g];
  bc[t] = acc;
}

// x[a][g] += xc[parent(a)][g], one thread per entry of the finer level.
__global__ void __launch_bounds__(256)
mg_prolong_add_kernel(const double* __restrict__ xc, MgGrid gc, MgGrid gf, double* __restrict__ x) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= 8 * gf.na) return;
  const int64_t a = t >> 3;
  const int X = int(a % gf.ax), Y = int((a / gf.ax) % gf.ay), Z = int(a / (int64_t(gf.ax) * gf.ay));
  const int64_t A = int64_t(X >> 1) + int64_t(gc.ax) * ((Y >> 1) + int64_t(gc.ay) * (Z >> 1));
  x[t] += xc[A * 8 + (t & 7)];
}

// Dense column-major form of a level's stencil operator in the padded
// ordering (unknown a * 8 + g, nc = 8 na): D[(a 8 + g) + nc (nb 8 + f)] =
// entry (g, f) of slot s of a (D cleared beforehand; the pad rows and
// columns stay zero), one thread per stencil entry.
__global__ void __launch_bounds__(256)
mg_dense_kernel(const double* __restrict__ E, MgGrid gr, double* __restrict__ D) {
  const int64_t total = 392 * gr.na;
  const int64_t nc = 8 * gr.na;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int g = int(k & 7);
    const int64_t q = k >> 3;                 // (s 7 + f) na + a
    const int sf = int(q / gr.na);
    const int64_t a = q - int64_t(sf) * gr.na;
    const int s = sf / 7, f = sf % 7;
    if (g == 7) continue;
    const int X = int(a % gr.ax), Y = int((a / gr.ax) % gr.ay), Z = int(a / (int64_t(gr.ax) * gr.ay));
    const int64_t nb = mg_neighbour(gr, X, Y, Z, s);
    if (nb < 0) continue;
    D[(a * 8 + g) + nc * (nb * 8 + f)] = E[k];
  }
}

// A level operator in the exported layout out[((s 7 + g) 7 + f) na + a].
__global__ void __launch_bounds__(256)
mg_export_kernel(const double* __restrict__ E, MgGrid gr, double* __restrict__ out) {
  const int64_t total = 343 * gr.na;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int sgf = int(k / gr.na);
    const int64_t a = k - int64_t(sgf) * gr.na;
    const int s = sgf / 49, g = (sgf / 7) % 7, f = sgf % 7;
    out[k] = E[mg_entry(s, g, f, a, gr.na)];
  }
}

}  // namespace lsbdg
