// Aggregation coarse space for the Krylov preconditioner.
//
// The voxels are grouped into A x A x A aggregates (the last ones along an
// axis may be thinner).  Coarse basis vector Z_{f,a} is the unknown scale sc
// of field f on the nodes of aggregate a, zero elsewhere; a coarse vector y
// has entries y[f * na + a].  The coarse operator E = Z^T J Z couples each
// aggregate to itself and its six face neighbours only (the operator's
// stencil is one voxel wide), so it is assembled exactly from 7 x 7
// probes: with colour(a) = (ax + 2 ay + 3 az) mod 7 the seven aggregates of
// any such stencil have distinct colours, and the product J v with v the sum
// of Z_{f,a} over one colour class, restricted to aggregate b, is the
// column (f, a*) of E for the unique aggregate a* of that colour in b's
// stencil.  One workgroup per aggregate forms each sum, so every entry is
// written exactly once, without atomics.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lsbdg {

struct AggGrid {
  int32_t nx, ny, nz, A;
  int32_t nax, nay, naz, pad;
  int64_t na;
};

__device__ __forceinline__ int agg_colour(int ax, int ay, int az) { return (ax + 2 * ay + 3 * az) % 7; }

__device__ __forceinline__ int64_t agg_of_voxel(const AggGrid& G, int64_t e) {
  const int ix = int(e % G.nx);
  const int iy = int((e / G.nx) % G.ny);
  const int iz = int(e / (int64_t(G.nx) * G.ny));
  return int64_t(ix / G.A) + int64_t(G.nax) * (iy / G.A + int64_t(G.nay) * (iz / G.A));
}

__device__ __forceinline__ int agg_colour_of_voxel(const AggGrid& G, int64_t e) {
  const int ix = int(e % G.nx);
  const int iy = int((e / G.nx) % G.ny);
  const int iz = int(e / (int64_t(G.nx) * G.ny));
  return agg_colour(ix / G.A, iy / G.A, iz / G.A);
}

// v = sum of Z_{f,a} over the aggregates a of colour c (7 fields, 8 nodes/voxel).
template <typename S>
__global__ void __launch_bounds__(256)
agg_probe_kernel(const S* __restrict__ sc, int f, int c, AggGrid G, int64_t FS, S* __restrict__ v) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < 7 * FS; k += int64_t(gridDim.x) * 256) {
    const int g = int(k / FS);
    const int64_t node = k - int64_t(g) * FS;
    v[k] = (g == f && agg_colour_of_voxel(G, node >> 3) == c) ? sc[k] : S(0);
  }
}

// Block-wide sums of 7 values (256 threads).
__device__ __forceinline__ void block_sum7(double* acc, double (*sh)[4]) {
#pragma unroll
  for (int g = 0; g < 7; ++g) {
    double v = acc[g];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) sh[g][threadIdx.x >> 6] = v;
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < 7; ++g) acc[g] = sh[g][0] + sh[g][1] + sh[g][2] + sh[g][3];
}

// acc[g] = sum over the nodes of aggregate b of w_g x_g (w, x: 7 fields).
template <typename S>
__device__ __forceinline__ void agg_sums(const S* __restrict__ w, const S* __restrict__ x, const AggGrid& G,
                                         int64_t FS, int bx, int by, int bz, double* acc) {
  const int x0 = bx * G.A, y0 = by * G.A, z0 = bz * G.A;
  const int lx = min(G.A, G.nx - x0), ly = min(G.A, G.ny - y0), lz = min(G.A, G.nz - z0);
  const int64_t nn = int64_t(lx) * ly * lz * 8;
#pragma unroll
  for (int g = 0; g < 7; ++g) acc[g] = 0.0;
  for (int64_t t = threadIdx.x; t < nn; t += 256) {
    const int n = int(t & 7);
    const int64_t vox = t >> 3;
    const int ix = x0 + int(vox % lx);
    const int iy = y0 + int((vox / lx) % ly);
    const int iz = z0 + int(vox / (int64_t(lx) * ly));
    const int64_t node = (int64_t(ix) + int64_t(G.nx) * (iy + int64_t(G.ny) * iz)) * 8 + n;
#pragma unroll
    for (int g = 0; g < 7; ++g) acc[g] += double(w[g * FS + node]) * double(x[g * FS + node]);
  }
}

// Column (f, a*) rows (g, b) of E from the probe product Jv of colour c; one
// workgroup per aggregate b.  E is column-major with leading dimension ld.
template <typename S>
__global__ void __launch_bounds__(256)
agg_probe_reduce_kernel(const S* __restrict__ sc, const S* __restrict__ Jv, int f, int c, AggGrid G, int64_t FS,
                        double* __restrict__ E, int64_t ld) {
  __shared__ double sh[7][4];
  const int64_t b = blockIdx.x;
  const int bx = int(b % G.nax), by = int((b / G.nax) % G.nay), bz = int(b / (int64_t(G.nax) * G.nay));
  // the aggregate of colour c in b's seven-point stencil (uniform per block)
  int64_t astar = -1;
  {
    const int d[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int s = 0; s < 7; ++s) {
      const int ax = bx + d[s][0], ay = by + d[s][1], az = bz + d[s][2];
      if (ax < 0 || ay < 0 || az < 0 || ax >= G.nax || ay >= G.nay || az >= G.naz) continue;
      if (agg_colour(ax, ay, az) == c) astar = ax + int64_t(G.nax) * (ay + int64_t(G.nay) * az);
    }
  }
  if (astar < 0) return;                      // whole block: nothing of colour c reaches b
  double acc[7];
  agg_sums(sc, Jv, G, FS, bx, by, bz, acc);
  block_sum7(acc, sh);
  if (threadIdx.x < 7) {
    const int g = threadIdx.x;
    E[(int64_t(g) * G.na + b) + ld * (int64_t(f) * G.na + astar)] = acc[g];
  }
}

// Restriction rc[g * na + b] = sum over aggregate b of sc_g r_g (FP64).
template <typename S>
__global__ void __launch_bounds__(256)
agg_restrict_kernel(const S* __restrict__ sc, const S* __restrict__ r, AggGrid G, int64_t FS,
                    double* __restrict__ rc) {
  __shared__ double sh[7][4];
  const int64_t b = blockIdx.x;
  const int bx = int(b % G.nax), by = int((b / G.nax) % G.nay), bz = int(b / (int64_t(G.nax) * G.nay));
  double acc[7];
  agg_sums(sc, r, G, FS, bx, by, bz, acc);
  block_sum7(acc, sh);
  if (threadIdx.x < 7) rc[int64_t(threadIdx.x) * G.na + b] = acc[threadIdx.x];
}

// Prolongation out += Z y: out[g][node] += sc[g][node] y[g * na + agg(node)];
// one thread per node finds its aggregate once for the seven fields.
// div (optional): the sum is then divided entrywise by div (the unknown
// scales of the Krylov system), in the same pass.
template <typename S>
__global__ void __launch_bounds__(256)
agg_prolong_add_kernel(const S* __restrict__ sc, const double* __restrict__ y, AggGrid G, int64_t FS,
                       S* __restrict__ out, const S* __restrict__ div) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < FS; k += int64_t(gridDim.x) * 256) {
    const int64_t a = agg_of_voxel(G, k >> 3);
#pragma unroll
    for (int g = 0; g < 7; ++g) {
      const S v = out[g * FS + k] + sc[g * FS + k] * S(y[int64_t(g) * G.na + a]);
      out[g * FS + k] = div ? v / div[g * FS + k] : v;
    }
  }
}

// Coarse correction y = d .* (A (d .* x)) with the explicit inverse A of the
// equilibrated coarse operator (column-major, nc x nc, FP64).  Split over
// column chunks so that the launch fills the chip: pass 1 writes
// part[chunk][i] = sum over the chunk's columns j of A[i][j] d[j] x[j]
// (grid: row tiles of 256 x kCoarseChunks), pass 2 sums the chunks.
constexpr int kCoarseChunks = 32;

// X = identity (n x n, column-major), grid-stride.
__global__ void __launch_bounds__(256) identity_kernel(double* __restrict__ X, int64_t n) {
  const int64_t nn = n * n;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < nn; k += int64_t(gridDim.x) * 256)
    X[k] = (k % n == k / n) ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(256)
coarse_gemv_partial_kernel(const double* __restrict__ A, int64_t nc, const double* __restrict__ x,
                           const double* __restrict__ d, int64_t chunk, double* __restrict__ part) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t j0 = int64_t(blockIdx.y) * chunk;
  const int64_t j1 = j0 + chunk < nc ? j0 + chunk : nc;
  if (i >= nc) return;
  double acc = 0.0;
  for (int64_t j = j0; j < j1; ++j) acc += A[i + j * nc] * (d[j] * x[j]);
  part[int64_t(blockIdx.y) * nc + i] = acc;
}

__global__ void __launch_bounds__(256)
coarse_gemv_finish_kernel(const double* __restrict__ part, int64_t nc, const double* __restrict__ d,
                          double* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nc; i += int64_t(gridDim.x) * 256) {
    double s = 0.0;
#pragma unroll 4
    for (int k = 0; k < kCoarseChunks; ++k) s += part[int64_t(k) * nc + i];
    y[i] = d[i] * s;
  }
}

// Symmetric equilibration of the coarse matrix: d_i = |E_ii|^-1/2 (1 where
// E_ii = 0 or not finite); inactive coarse unknowns (zero rows and columns)
// get E_ii = 1.
__global__ void __launch_bounds__(256)
coarse_diag_kernel(double* __restrict__ E, int64_t nc, int64_t ld, double* __restrict__ d) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nc; i += int64_t(gridDim.x) * 256) {
    const double a = fabs(E[i + ld * i]);
    if (!(a > 0.0) || !isfinite(a)) {
      E[i + ld * i] = 1.0;
      d[i] = 1.0;
    } else {
      d[i] = 1.0 / sqrt(a);
    }
  }
}

__global__ void __launch_bounds__(256)
coarse_scale_kernel(double* __restrict__ E, int64_t nc, int64_t ld, const double* __restrict__ d) {
  const int64_t total = nc * nc;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += int64_t(gridDim.x) * 256) {
    const int64_t j = k / nc, i = k - j * nc;
    E[i + ld * j] *= d[i] * d[j];
  }
}

}  // namespace lsbdg
