// Batched operators: many voxel structures of uneven size in one launch.
//
// The structures are concatenated voxel by voxel in the field-major layout
// a[f][E][n] (E = total voxels; structure s owns voxels [base_s, base_s +
// Ne_s)).  The work items are tiles of 32 consecutive voxels of one
// structure -- 256 lanes, one per node, as in the single-structure kernels
// -- so a workgroup never straddles two structures.  Each lane offsets the
// array bases by its structure's first voxel and runs the same node code as
// the single-structure kernels with the batch's field stride; the results
// therefore equal those of one launch per structure.  Per-structure
// parameters (time step, regularisation time, applied current, phase
// table) are read from a device array indexed by the tile's structure.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "model.hpp"
#include "resid_q1.hpp"
#include "brick_q1.hpp"
#include "blockjacobi.hpp"

namespace lsbdg {

struct BatchTile {
  int32_t s;       // structure
  int32_t v0;      // first voxel of the tile within the structure
  int64_t base;    // first voxel of the structure in the concatenation
};

constexpr int kTileVoxels = 32;   // 256 lanes / 8 nodes: the default work item

// Work-item sizes the batched residual and tangents can be launched with
// (8 lanes per voxel: 64, 128 or 256 lanes).  The batch keeps one tile list
// per size; the size and whether the grid is persistent are chosen per
// operator and precision (the library's autotuner times them all).
constexpr int kTileChoices[3] = {8, 16, 32};

// Position `i` of a padded grid in XCD-aware order (as xcd_block).  A
// persistent grid strides by a multiple of 8 workgroups, so every pass of a
// workgroup stays within the voxel range of the XCD it was dispatched to.
__device__ __forceinline__ int64_t xcd_order(int64_t i, int64_t nblocks_padded) {
  const int64_t per = nblocks_padded / 8;
  return (i % 8) * per + i / 8;
}

// The tile of this workgroup (XCD-aware order) and the lane's voxel within
// its structure; false for lanes past the structure's last voxel and for
// the padding workgroups of the grid.
__device__ __forceinline__ bool batch_lane(const BatchTile* __restrict__ tiles, int64_t ntiles,
                                           int64_t nblocks_padded, const DevParams* __restrict__ Ps,
                                           BatchTile& t, const DevParams*& P, int64_t& e) {
  const int64_t blk = xcd_block(nblocks_padded);
  if (blk >= ntiles) return false;
  t = tiles[blk];
  P = Ps + t.s;
  e = int64_t(t.v0) + (threadIdx.x >> 3);
  return e < P->Ne;
}

template <typename S>
__device__ __forceinline__ const S* shift(const S* p, int64_t o) { return p ? p + o : p; }

// Residual or tangent of the work items of this workgroup.  One-shot grid
// (a workgroup per item, gridDim.x = nblocks_padded): one item.  Persistent
// grid (gridDim.x a smaller multiple of 8): items blockIdx.x, blockIdx.x +
// gridDim.x, ... -- bounds fixed at launch, so every workgroup exits.  The
// two forms are separate kernels: the loop's own registers would push the
// FP64 residual past 256 and halve its occupancy in the one-shot form.
template <typename S, typename N, int Mode>
__device__ __forceinline__ void q1_batch_item(const S* __restrict__ U, const S* __restrict__ V,
                                              const S* __restrict__ M, S* __restrict__ Out,
                                              const uint8_t* __restrict__ phase,
                                              const DevParams* __restrict__ Ps,
                                              const BatchTile* __restrict__ tiles, int64_t ntiles, int64_t FS,
                                              int64_t nblocks_padded, int64_t i) {
  const int64_t blk = xcd_order(i, nblocks_padded);
  if (blk >= ntiles) return;
  const BatchTile t = tiles[blk];
  const DevParams* P = Ps + t.s;
  const int64_t e = int64_t(t.v0) + (threadIdx.x >> 3);
  if (e >= P->Ne) return;                    // whole 8-lane groups leave together
  const int64_t o = t.base * 8;
  q1_node<S, N, Mode>(U + o, shift(V, o), shift(M, o), Out + o, phase + t.base, *P, e, int(threadIdx.x & 7), FS);
}

template <typename S, typename N, int Mode, bool kPersistent>
__device__ __forceinline__ void q1_batch_body(const S* __restrict__ U, const S* __restrict__ V,
                                              const S* __restrict__ M, S* __restrict__ Out,
                                              const uint8_t* __restrict__ phase,
                                              const DevParams* __restrict__ Ps,
                                              const BatchTile* __restrict__ tiles, int64_t ntiles, int64_t FS,
                                              int64_t nblocks_padded) {
  if constexpr (kPersistent) {
    for (int64_t i = blockIdx.x; i < nblocks_padded; i += gridDim.x)
      q1_batch_item<S, N, Mode>(U, V, M, Out, phase, Ps, tiles, ntiles, FS, nblocks_padded, i);
  } else {
    q1_batch_item<S, N, Mode>(U, V, M, Out, phase, Ps, tiles, ntiles, FS, nblocks_padded, blockIdx.x);
  }
}

template <typename S, typename N, int Mode, int kLanes, bool kPersistent>
__global__ void __launch_bounds__(kLanes)
q1_batch_kernel(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ M, S* __restrict__ Out,
                const uint8_t* __restrict__ phase, const DevParams* __restrict__ Ps,
                const BatchTile* __restrict__ tiles, int64_t ntiles, int64_t FS, int64_t nblocks_padded) {
  q1_batch_body<S, N, Mode, kPersistent>(U, V, M, Out, phase, Ps, tiles, ntiles, FS, nblocks_padded);
}

// As q1_kernel_w2: the FP32 tangent held to two waves per SIMD.
template <typename S, typename N, int Mode, int kLanes, bool kPersistent>
__global__ void __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(2)))
q1_batch_kernel_w2(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ M,
                   S* __restrict__ Out, const uint8_t* __restrict__ phase, const DevParams* __restrict__ Ps,
                   const BatchTile* __restrict__ tiles, int64_t ntiles, int64_t FS, int64_t nblocks_padded) {
  q1_batch_body<S, N, Mode, kPersistent>(U, V, M, Out, phase, Ps, tiles, ntiles, FS, nblocks_padded);
}

// Element blocks of every structure (Bout: E blocks of nb x nb).
template <typename S, int Mode>
__global__ void __launch_bounds__(256)
q1_block_batch_kernel(const S* __restrict__ U, const S* __restrict__ Cw, S* __restrict__ Bout,
                      const uint8_t* __restrict__ phase, const DevParams* __restrict__ Ps,
                      const BatchTile* __restrict__ tiles, int64_t ntiles, int64_t FS, int64_t nblocks_padded) {
  constexpr int NB = (Mode == kJvpFull) ? 72 : 56;
  BatchTile t;
  const DevParams* P;
  int64_t e;
  if (!batch_lane(tiles, ntiles, nblocks_padded, Ps, t, P, e)) return;
  const int64_t o = t.base * 8;
  q1_block_node<S, Mode>(U + o, Cw + o, Bout + t.base * int64_t(NB) * NB, phase + t.base, *P, e,
                         int(threadIdx.x & 7), FS);
}

// Krylov operator of a batch on bricks of 4 x 4 x 4 voxels: one workgroup
// per work item (structure s, brick v0 of its own brick grid, first voxel
// base of the structure in the concatenation), with the structure's folded
// parameters and the batch's field stride FS.  Each structure's values are
// those of q1_brick_jvp_kernel on it (the same body, array bases offset).
template <typename S>
__global__ void __launch_bounds__(kBrickLanes)
q1_brick_jvp_batch_kernel(const S* __restrict__ U, const S* __restrict__ V, const S* __restrict__ Cw,
                          S* __restrict__ Out, const uint8_t* __restrict__ phase, const KP<S>* __restrict__ Ks,
                          const BatchTile* __restrict__ items, int64_t nitems, int64_t FS,
                          int64_t nitems_padded) {
  __shared__ BrickLds<S> L;
  const int64_t blk = xcd_block(nitems_padded);
  if (blk >= nitems) return;                     // a padding workgroup leaves as a whole
  const BatchTile t = items[blk];
  const int s = __builtin_amdgcn_readfirstlane(t.s);
  const KP<S>& K = Ks[s];                        // read in place: a copy would go to scratch
  const int nbx = (K.nx + kBE - 1) / kBE, nby = (K.ny + kBE - 1) / kBE;
  const int64_t o = t.base;
  brick_jvp(U + o * 8, V + o * 8, Cw + o * 8, Out + o * 8, phase + o, K, nbx, nby, int64_t(t.v0), FS, L);
}

// Linearisation coefficients of the condensed tangent (14 x E x 8).
template <typename S>
__global__ void __launch_bounds__(256)
solid_tangent_batch_kernel(const S* __restrict__ U, S* __restrict__ Cw, const uint8_t* __restrict__ phase,
                           const DevParams* __restrict__ Ps, const BatchTile* __restrict__ tiles,
                           int64_t ntiles, int64_t FS, int64_t nblocks_padded) {
  BatchTile t;
  const DevParams* P;
  int64_t e;
  if (!batch_lane(tiles, ntiles, nblocks_padded, Ps, t, P, e)) return;
  const int64_t o = t.base * 8;
  solid_tangent_node(U + o, Cw + o, int(phase[t.base + e]), *P, e * 8 + (threadIdx.x & 7), FS);
}

// Old mass of every structure: m[i] = eps_L c_i (i < 6), m[6 + s] = eps_s.
template <typename T>
__global__ void __launch_bounds__(256)
mass_batch_kernel(const T* __restrict__ U, T* __restrict__ M, const uint8_t* __restrict__ phase,
                  const DevParams* __restrict__ Ps, const BatchTile* __restrict__ tiles, int64_t ntiles,
                  int64_t FS, int64_t nblocks_padded) {
  BatchTile t;
  const DevParams* P;
  int64_t e;
  if (!batch_lane(tiles, ntiles, nblocks_padded, Ps, t, P, e)) return;
  const int64_t g = (t.base + e) * 8 + (threadIdx.x & 7);
  const int ph = phase[t.base + e];
  const T e7 = U[7 * FS + g], e8 = U[8 * FS + g];
  const T eL = liquid_fraction(T(P->epsCBD[ph]), e7, e8, T(P->epsL_min));
#pragma unroll
  for (int i = 0; i < 6; ++i) M[i * FS + g] = eL * U[i * FS + g];
  M[6 * FS + g] = e7;
  M[7 * FS + g] = e8;
}

}  // namespace lsbdg
