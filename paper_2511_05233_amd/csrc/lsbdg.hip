// C-ABI of the lsbdg library (declared in include/lsbdg.h).
//
// Host side: argument checks, parameter derivation (Tab. InitialState,
// Eq. 57, App. C), device tables and kernel launches.  No exception leaves
// an extern "C" function; every failure returns a dg_status and records a
// message for dg_last_error().
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/lsbdg.h"
#include "model.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"
#include "resid_q0.hpp"
#include "resid_q3.hpp"
#include "brick_q1.hpp"
#include "blockjacobi.hpp"
#include "blocks_q3.hpp"
#include "solver.hpp"
#include "outputs.hpp"
#include "limiter.hpp"
#include "coarse.hpp"
#include "multigrid.hpp"
#include "batch.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

using namespace lsbdg;

struct dg_ctx {
  dg_mesh mesh{};
  dg_params params{};
  Equilibrium eq{};
  PhaseTable phase_tab{};
  double j_el = 0.0;
  double eps_struct = 1.0;
  double sigma = 1.0;
  int64_t Ne = 0;
  int np = 1;
  uint8_t* d_phase = nullptr;
  DevBuf phase;                     // device phase map (d_phase points into it)
  // element block-Jacobi storage (condensed inverses, 56 x 56 at k = 1 and
  // 448 x 448 at k = 3, column-major); at k = 3 also the pivot lists and two
  // 7-field vectors for the probes of the assembly
  DevBuf blocks, qpiv, probe;
  int blocks_prec = -1;
  // linearisation coefficients of the condensed tangent (14 x nodes)
  DevBuf lin;
  // aggregation coarse space: LU of the equilibrated coarse operator,
  // equilibration, pivots, a coarse vector, LAPACK status
  DevBuf cE, cd, crc, crc2, cipiv, cinfo, cpart;
  DevBuf cX;                        // E^-1 (solve of the LU factors against the identity)
  // bfloat16 copy of FP32 block inverses (block_bf16), current while bh_valid
  DevBuf bh;
  bool bh_valid = false;
  rocblas_handle blas = nullptr;
  DevBuf blasws;                    // rocBLAS/rocSOLVER scratch (workspace contexts)
  int lin_prec = -1;
  DevBuf status;                    // singular-block flag of the block setup
  SolverWork work;
  // multilevel coarse correction (multigrid.hpp): level grids, stencil
  // operators, inverses of their self blocks, right sides and two iterates
  // per level; unit scales and two probe vectors of dg_mg_setup
  struct Multigrid {
    int levels = 0, nu = 2;
    double omega = 0.7;
    AggGrid G{};                      // level-1 aggregates on the voxels
    MgGrid g[kMgMaxLevels]{};
    DevBuf E[kMgMaxLevels], Dinv[kMgMaxLevels], b[kMgMaxLevels], xa[kMgMaxLevels], xb[kMgMaxLevels];
    DevBuf r[kMgMaxLevels];
    DevBuf ones, pv, pjv;
    int prec = -1;                    // precision of a dg_mg_setup hierarchy (-1: none current)
  } mg;
  // caller-owned workspace (dg_setup_ws): every DevBuf above is carved from it
  Arena arena;
  bool owns_memory = true;
  template <typename F>
  void for_each_buf(F f) {
    for (DevBuf* d : {&phase, &blocks, &qpiv, &probe, &lin, &cE, &cX, &cd, &crc, &crc2, &cipiv, &cinfo, &cpart, &bh, &blasws, &status})
      f(*d);
    for (int l = 0; l < kMgMaxLevels; ++l)
      for (DevBuf* d : {&mg.E[l], &mg.Dinv[l], &mg.b[l], &mg.xa[l], &mg.xb[l], &mg.r[l]}) f(*d);
    for (DevBuf* d : {&mg.ones, &mg.pv, &mg.pjv}) f(*d);
    work.for_each(f);
  }
  // GMRES cycle: pinned done flags of the last two iterations and their events
  int32_t* gm_flags = nullptr;
  hipEvent_t gm_ev[2] = {nullptr, nullptr};
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Device memory for `what` (need bytes) was not available: from the
// caller's workspace of a dg_setup_ws context (the message says how much
// it lacks), or from hipMalloc.
int fail_mem(const dg_ctx* ctx, const std::string& what, size_t need) {
  if (!ctx->owns_memory)
    return fail(DG_ENOMEM, what + ": the caller's workspace lacks " + std::to_string(ctx->arena.short_by) +
                               " bytes (size it with dg_workspace_bytes for this use)");
  return fail(DG_ENOMEM, what + ": device allocation of " + std::to_string(need) + " bytes failed");
}

#define DG_HIP(call)                                                              \
  do {                                                                            \
    hipError_t err_ = (call);                                                     \
    if (err_ != hipSuccess)                                                       \
      return fail(DG_EHIP, std::string(#call) + ": " + hipGetErrorString(err_)); \
  } while (0)

DevParams make_params(const dg_ctx* c, double t_eval, double dt) {
  DevParams P{};
  const dg_params& p = c->params;
  const double RT = kGas * p.T;
  for (int i = 0; i < 7; ++i) P.D0[i] = p.D0[i];
  for (int j = 0; j < 6; ++j) {
    P.zDA[j] = kZ[j] * (p.D0[j] - p.D0[6]);
    P.wL[j] = kZ[j] * (kZ[j] * p.D0[j] - kZA * p.D0[6]);
    P.kE[j] = p.kE[j];
    P.U0[j] = c->eq.U0[j];
  }
  for (int s = 0; s < 2; ++s) {
    P.kC[s] = kKC[s];
    P.sqrtK[s] = std::sqrt(kKsp[s]);
    P.rhoM[s] = kRho[s] / kMolar[s];
  }
  P.F = kFaraday;
  P.frt = kFaraday / RT;
  P.frt2 = 0.5 * kFaraday / RT;
  P.V = c->eq.dphi0;
  P.inv_cref = 1.0 / kCref;
  P.c_min = p.c_min;
  P.epsL_min = p.epsL_min;
  const double h = c->mesh.h;
  P.sig_h = c->sigma / h;
  P.sq3_h = std::sqrt(3.0) / h;
  // nodal weights: (h/2)^3 w_a w_b w_c with the Gauss-Legendre weights of
  // the order (1 for the two-point rule of Q1, 2 for the one-point rule of
  // k = 0), and (h/2)^2 w w on faces
  const double wgl = c->mesh.order == 0 ? 2.0 : 1.0;
  P.W3 = (h / 2) * (h / 2) * (h / 2) * wgl * wgl * wgl;
  P.W2 = (h / 2) * (h / 2) * wgl * wgl;
  P.jel = c->j_el;
  P.TH = p.use_TH ? 0.5 * (1.0 + std::tanh(6.0 * (t_eval - 1.0))) : 1.0;
  P.inv_dt = dt > 0 ? 1.0 / dt : 0.0;
  for (int q = 0; q < 2; ++q) {
    P.epsCBD[q] = c->phase_tab.epsCBD[q];
    P.aV0[q] = c->phase_tab.aV0[q];
    P.s8ref[q] = c->phase_tab.s8ref[q];
    P.pass[q] = c->phase_tab.pass[q];
    P.react[q] = c->phase_tab.react[q];
  }
  P.nx = c->mesh.nx;
  P.ny = c->mesh.ny;
  P.nz = c->mesh.nz;
  P.Ne = c->Ne;
  P.np = c->np;
  P.two_h = 2.0 / h;
  P.active = kAllFields;
  return P;
}

int check_ctx(const dg_ctx* c) {
  if (!c) return fail(DG_EINVAL, "null context");
  return DG_OK;
}

// Entry points built for Q1 only: at k = 0 the library provides the
// operators (mass, residual, tangents, linearisation).
int check_q1(const dg_ctx* c, const char* fn) {
  if (c->mesh.order != 1)
    return fail(DG_EUNSUPPORTED, std::string(fn) + ": order " + std::to_string(c->mesh.order) +
                                     " provides the operators only (mass, residual, tangents, linearisation)");
  return DG_OK;
}

// Entry points of the element block-Jacobi preconditioner: k = 1 and 3.
int check_blocks_order(const dg_ctx* c, const char* fn) {
  if (c->mesh.order != 1 && c->mesh.order != 3)
    return fail(DG_EUNSUPPORTED, std::string(fn) + ": order " + std::to_string(c->mesh.order) +
                                     " provides the operators only (mass, residual, tangents, linearisation)");
  return DG_OK;
}

// Condensed block size: 7 fields x the element's nodes.
int condensed_block_size(const dg_ctx* c) { return 7 * c->np; }

}  // namespace

// Device scratch of dg_outputs_noalloc: the block partials of the outputs
// kernel (kNumSums x kOutBlocks) and the finished sums (kNumSums), 123 KB
// per device, held by every GPU the library runs on until the process
// ends.  Host code never uses this name as an address: each device's own
// copy is looked up once with hipGetSymbolAddress and used from then on.
constexpr int kOutBlocks = 1024;
constexpr size_t kScratchDoubles = size_t(kNumSums) * kOutBlocks + kNumSums;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Address of the current device's scratch (looked up on the first call on
// that device, with that device current).
int device_scratch(double** out) {
  int dev = -1;
  DG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return DG_OK;
}

}  // namespace

namespace {

template <typename S, typename N, int Mode>
void launch_q1(const dg_ctx* ctx, const DevParams& P, const void* u, const void* v, const void* m,
               void* out, hipStream_t st) {
  if (ctx->np == 1) {                          // k = 0: one lane per voxel
    const int64_t nb = std::min<int64_t>((ctx->Ne + 255) / 256, 16384);
    hipLaunchKernelGGL((q0_kernel<S, N, Mode>), dim3(unsigned(nb)), dim3(256), 0, st, static_cast<const S*>(u),
                       static_cast<const S*>(v), static_cast<const S*>(m), static_cast<S*>(out), ctx->d_phase, P);
    return;
  }
  if (ctx->np == 64) {                         // k = 3: one wavefront per voxel, four per workgroup
    const int64_t nb = std::min<int64_t>((ctx->Ne + 3) / 4, 65536);
    hipLaunchKernelGGL((q3_kernel<S, N, Mode>), dim3(unsigned(nb)), dim3(256), 0, st, static_cast<const S*>(u),
                       static_cast<const S*>(v), static_cast<const S*>(m), static_cast<S*>(out), ctx->d_phase, P);
    return;
  }
  const int64_t threads = ctx->Ne * 8;
  if constexpr (std::is_same<S, float>::value && Mode != kResidual) {
    // the FP32 tangent (two waves per SIMD) in workgroups of one wave, the
    // shape the batch autotuner picks for the batched form of this kernel
    constexpr int kLanes = 64;
    const int64_t nb = ((threads + kLanes - 1) / kLanes + 7) / 8 * 8;
    hipLaunchKernelGGL((q1_kernel_w2<S, N, Mode, kLanes>), dim3(unsigned(nb)), dim3(kLanes), 0, st,
                       static_cast<const S*>(u), static_cast<const S*>(v), static_cast<const S*>(m),
                       static_cast<S*>(out), ctx->d_phase, P, nb);
    return;
  }
  int64_t nb = (threads + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  hipLaunchKernelGGL((q1_kernel<S, N, Mode>), grid, block, 0, st, static_cast<const S*>(u),
                     static_cast<const S*>(v), static_cast<const S*>(m), static_cast<S*>(out), ctx->d_phase, P,
                     nb);
}

// Krylov operator: condensed tangent at the stored linearisation, one
// workgroup per brick of 4 x 4 x 4 voxels (inner faces evaluated once).
template <typename S>
void launch_brick_jvp(const dg_ctx* ctx, const DevParams& P, const void* u, const void* v, const void* lin,
                      void* out, hipStream_t st, const void* rsub = nullptr) {
  const int nbx = (ctx->mesh.nx + kBE - 1) / kBE, nby = (ctx->mesh.ny + kBE - 1) / kBE;
  const int64_t nbz = (ctx->mesh.nz + kBE - 1) / kBE;
  const int64_t nb = (int64_t(nbx) * nby * nbz + 7) / 8 * 8;
  hipLaunchKernelGGL(q1_brick_jvp_kernel<S>, dim3(unsigned(nb)), dim3(kBrickLanes), 0, st,
                     static_cast<const S*>(u), static_cast<const S*>(v), static_cast<const S*>(lin),
                     static_cast<S*>(out), ctx->d_phase, make_kp<S>(P), nbx, nby, nb, static_cast<const S*>(rsub));
}

// Linearisation coefficients of the condensed tangent at u (precision S).
template <typename S>
int linearize(dg_ctx* ctx, const DevParams& P, const S* u, hipStream_t st) {
  const int64_t FS = ctx->Ne * ctx->np;
  const size_t lin_bytes = size_t(14) * FS * sizeof(S);
  if (ctx->lin.ensure(lin_bytes) != hipSuccess) return fail_mem(ctx, "linearisation storage", lin_bytes);
  int64_t nb = (FS + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(solid_tangent_kernel<S>, dim3(unsigned(nb)), dim3(256), 0, st, u, ctx->lin.as<S>(),
                     ctx->d_phase, P);
  DG_HIP(hipGetLastError());
  ctx->lin_prec = std::is_same<S, double>::value ? DG_F64 : DG_F32;
  return DG_OK;
}

}  // namespace


namespace {

// Build and invert the condensed element blocks of precision S at uS
// (needs the linearisation at uS).
// bf16_only (S = float): the inverses go straight to the bfloat16 copy, and
// the FP32 storage keeps the assembled blocks (not usable as inverses).
template <typename S>
int blocks_setup(dg_ctx* ctx, const DevParams& P, const S* uS, hipStream_t st, bool bf16_only = false) {
  const size_t need = size_t(ctx->Ne) * 56 * 56 * sizeof(S);
  if (ctx->blocks.ensure(need) != hipSuccess) return fail_mem(ctx, "block storage", need);
  if (ctx->status.ensure(sizeof(int)) != hipSuccess) return fail_mem(ctx, "status flag", sizeof(int));
  int* d_status = ctx->status.as<int>();
  DG_HIP(hipMemsetAsync(d_status, 0, sizeof(int), st));
  int64_t nb = (ctx->Ne * 8 + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  const dim3 grid_w{unsigned((ctx->Ne + 3) / 4), 1, 1};
  hipLaunchKernelGGL((q1_block_kernel<S, kJvpCondensed>), grid, block, 0, st, uS, ctx->lin.as<S>(),
                     ctx->blocks.as<S>(), ctx->d_phase, P, nb);
  ctx->bh_valid = false;
  if constexpr (std::is_same<S, float>::value) {
    if (bf16_only) {
      if (ctx->bh.ensure(size_t(ctx->Ne) * 56 * 56 * 2) != hipSuccess)
        return fail_mem(ctx, "bf16 blocks", size_t(ctx->Ne) * 56 * 56 * 2);
      hipLaunchKernelGGL((invert_blocks_kernel<float, 56, true>), grid_w, block, 0, st,
                         ctx->blocks.as<float>(), ctx->Ne, ctx->status.as<int>(), ctx->bh.as<uint16_t>());
    }
  }
  if (!bf16_only)
    hipLaunchKernelGGL((invert_blocks_kernel<S, 56>), grid_w, block, 0, st, ctx->blocks.as<S>(),
                       ctx->Ne, ctx->status.as<int>(), nullptr);
  DG_HIP(hipGetLastError());
  int h_status = 0;
  DG_HIP(hipMemcpyAsync(&h_status, ctx->status.as<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
  DG_HIP(hipStreamSynchronize(st));
  if (bf16_only) {
    ctx->blocks_prec = -1;                     // FP32 storage holds no inverses
    ctx->bh_valid = true;
  } else {
    ctx->blocks_prec = std::is_same<S, double>::value ? DG_F64 : DG_F32;
  }
  if (h_status) return fail(DG_ENAN, "singular or non-finite element block");
  return DG_OK;
}

// The k = 3 blocks at uS: the linearisation, then two colours x 448
// probes of the Krylov operator filed column by column, then the blocked
// Gauss-Jordan inversion on the matrix cores.
template <typename S>
int blocks_setup_q3(dg_ctx* ctx, const DevParams& P, const S* uS, hipStream_t st) {
  const int64_t Ne = ctx->Ne, FS = Ne * 64;
  const size_t need = size_t(Ne) * kQ3NB * kQ3NB * sizeof(S);
  if (ctx->blocks.ensure(need) != hipSuccess) return fail_mem(ctx, "dg_blockjacobi_setup: block storage", need);
  if (ctx->qpiv.ensure(size_t(Ne) * kQ3NB * sizeof(int16_t)) != hipSuccess)
    return fail_mem(ctx, "dg_blockjacobi_setup: pivot lists", size_t(Ne) * kQ3NB * sizeof(int16_t));
  if (ctx->probe.ensure(size_t(14) * FS * sizeof(S)) != hipSuccess)
    return fail_mem(ctx, "dg_blockjacobi_setup: probe vectors", size_t(14) * FS * sizeof(S));
  if (ctx->status.ensure(sizeof(int)) != hipSuccess) return fail_mem(ctx, "dg_blockjacobi_setup: status flag", 4);
  if (int s = linearize<S>(ctx, P, uS, st)) return s;
  S* v = ctx->probe.as<S>();
  S* w = v + 7 * FS;
  S* B = ctx->blocks.as<S>();
  const int nx = ctx->mesh.nx, ny = ctx->mesh.ny;
  const unsigned g_seed = unsigned(std::min<int64_t>((7 * FS + 255) / 256, 8192));
  const unsigned g_scat = unsigned(std::min<int64_t>((Ne * kQ3NB + 255) / 256, 8192));
  for (int c = 0; c < 2; ++c)
    for (int j = 0; j < kQ3NB; ++j) {
      hipLaunchKernelGGL(seed_q3_kernel<S>, dim3(g_seed), dim3(256), 0, st, v, Ne, nx, ny, c, j);
      launch_q1<S, Dual<S>, kJvpCondensed>(ctx, P, uS, v, ctx->lin.p, w, st);
      hipLaunchKernelGGL(scatter_q3_kernel<S>, dim3(g_scat), dim3(256), 0, st, w, B, Ne, nx, ny, c, j);
    }
  DG_HIP(hipGetLastError());
  DG_HIP(hipMemsetAsync(ctx->status.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(invert_q3_kernel<S>, dim3(unsigned(Ne)), dim3(512), 0, st, B, ctx->qpiv.as<int16_t>(),
                     ctx->status.as<int>());
  DG_HIP(hipGetLastError());
  int h_status = 0;
  DG_HIP(hipMemcpyAsync(&h_status, ctx->status.as<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
  DG_HIP(hipStreamSynchronize(st));
  ctx->blocks_prec = std::is_same<S, double>::value ? DG_F64 : DG_F32;
  ctx->bh_valid = false;
  if (h_status) return fail(DG_ENAN, "dg_blockjacobi_setup: singular or non-finite element block");
  return DG_OK;
}

// Pinned done flags and events of the GMRES cycle (made once per context).
int gmres_host_state(dg_ctx* ctx) {
  if (ctx->gm_flags) return DG_OK;
  DG_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->gm_flags), 2 * sizeof(int32_t)));
  for (hipEvent_t& ev : ctx->gm_ev) DG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  return DG_OK;
}

// Device buffers of the Newton-GMRES step solve with inner precision of
// sS bytes, with their sizes (the solve ensures exactly these).
std::vector<std::pair<DevBuf*, size_t>> solver_buffers(dg_ctx* ctx, const dg_solver_opts& o, size_t sS) {
  const int64_t FS = ctx->Ne * ctx->np, n7 = 7 * FS, n9 = 9 * FS;
  const int m = o.gmres_restart;
  SolverWork& W = ctx->work;
  const bool global_coarse = o.coarse == 1 || o.coarse == 2;
  return {std::make_pair(&W.m_old, size_t(8 * FS) * 8), std::make_pair(&W.R, size_t(n9) * 8),
          std::make_pair(&W.Rtry, size_t(n9) * 8), std::make_pair(&W.u_try, size_t(n9) * 8),
          std::make_pair(&W.du, size_t(n9) * 8), std::make_pair(&W.wR, size_t(2 * FS) * 8),
          std::make_pair(&W.uS, size_t(n9) * sS), std::make_pair(&W.sc, size_t(n7) * sS),
          std::make_pair(&W.V, size_t(m + 1) * n7 * sS), std::make_pair(&W.w, size_t(n7) * sS),
          std::make_pair(&W.t, size_t(n7) * sS), std::make_pair(&W.pJ, size_t(n7) * sS),
          std::make_pair(&W.rhs, size_t(n7) * sS), std::make_pair(&W.b, size_t(n7) * sS),
          std::make_pair(&W.x, size_t(n7) * sS), std::make_pair(&W.y9, size_t(n9) * sS),
          std::make_pair(&W.v9, size_t(n9) * sS),
          std::make_pair(&W.JZ, global_coarse ? size_t(7) * n7 * sS : size_t(0)),
          std::make_pair(&W.partial, size_t(kMaxDots) * kRedBlocks * sS),
          std::make_pair(&W.partial64, size_t(kRedBlocks) * 8),
          std::make_pair(&W.dots, size_t(kMaxDots) * 8), std::make_pair(&W.yc, size_t(8) * 8),
          std::make_pair(&W.Ainv, size_t(49) * 8), std::make_pair(&W.hbuf, size_t(kMaxDots) * 8),
          std::make_pair(&W.pc, size_t(n7) * sS), std::make_pair(&W.pc2, size_t(n7) * sS),
          std::make_pair(&W.scc, size_t(n7) * sS),
          std::make_pair(&W.gsum, size_t(8) + 2 * size_t(kMaxDots) * sS),
          std::make_pair(&W.gstate, sizeof(GmresState))};
}

// Internal value of dg_solver_opts.coarse between normalize_opts and
// resolve_opts: the library default, which depends on the mesh.
constexpr int kCoarseDefault = 100;

// Levels of the multilevel coarse correction for options o on this mesh:
// o.mg_levels when set (0: none), else (-1) automatic.  The exact two-level
// solve is kept while it can use aggregates of at most 8 voxels per edge
// (coarse_agg if set) within 8192 coarse unknowns; beyond that its
// aggregates grow coarse and the cycle does better: level-1 aggregates of
// coarse_agg (0: 4) voxels per edge, and as many 2 x 2 x 2 coarsenings as
// bring the last level to at most 4096 unknowns.
int mg_levels_for(const dg_mesh& mesh, const dg_solver_opts& o) {
  if (o.mg_levels >= 0) return o.mg_levels;
  if (o.coarse != 3 && o.coarse != 4) return 0;
  auto naggs = [&](int a) {
    return int64_t((mesh.nx + a - 1) / a) * ((mesh.ny + a - 1) / a) * ((mesh.nz + a - 1) / a);
  };
  if (7 * naggs(o.coarse_agg > 0 ? o.coarse_agg : 8) <= 8192) return 0;
  const int A = o.coarse_agg > 0 ? o.coarse_agg : 4;
  MgGrid g{(mesh.nx + A - 1) / A, (mesh.ny + A - 1) / A, (mesh.nz + A - 1) / A, 0, 0};
  g.na = int64_t(g.ax) * g.ay * g.az;
  int L = 1;
  while (8 * g.na > 4096 && L < kMgMaxLevels) {
    g = mg_coarser(g);
    ++L;
  }
  return L;
}

// The default coarse space for this mesh: additive aggregation (3), or
// multiplicative (4) where the multilevel cycle is used (on the slab it
// saved a quarter of the GMRES iterations and 4% of the step time: the
// extra Krylov operator per iteration costs less than the iterations).
dg_solver_opts resolve_opts(const dg_mesh& mesh, const dg_solver_opts& in) {
  dg_solver_opts o = in;
  if (o.coarse == kCoarseDefault) {
    o.coarse = 3;
    if (mg_levels_for(mesh, o) >= 2) o.coarse = 4;
  }
  return o;
}

// Aggregates of the two-level coarse space: opts.coarse_agg voxels per
// edge, or the smallest edge >= 4 with at most 8192 coarse unknowns (4
// under the multilevel correction).
AggGrid coarse_grid(const dg_mesh& mesh, const dg_solver_opts& o) {
  AggGrid G{};
  const int nx = mesh.nx, ny = mesh.ny, nz = mesh.nz;
  auto naggs = [&](int a) { return int64_t((nx + a - 1) / a) * ((ny + a - 1) / a) * ((nz + a - 1) / a); };
  int A = o.coarse_agg;
  if (A <= 0) {
    A = 4;
    if (mg_levels_for(mesh, o) < 2)
      while (7 * naggs(A) > 8192) ++A;
  }
  G.nx = nx; G.ny = ny; G.nz = nz; G.A = A;
  G.nax = (nx + A - 1) / A; G.nay = (ny + A - 1) / A; G.naz = (nz + A - 1) / A;
  G.na = naggs(A);
  return G;
}

// Level grids of the multilevel coarse correction: the level-1 aggregates
// of G, then 2 x 2 x 2 groups of the level above.
void mg_grids(const AggGrid& G, int levels, MgGrid* g) {
  g[0] = MgGrid{G.nax, G.nay, G.naz, 0, G.na};
  for (int l = 1; l < levels; ++l) g[l] = mg_coarser(g[l - 1]);
}

// Unknowns of the dense coarse solve: the aggregation coarse space itself,
// or the last level of the multilevel correction.
int64_t coarse_dense_size(const dg_mesh& mesh, const dg_solver_opts& o) {
  const AggGrid G = coarse_grid(mesh, o);
  const int L = mg_levels_for(mesh, o);
  if (L < 2) return 7 * G.na;
  MgGrid g[kMgMaxLevels];
  mg_grids(G, L, g);
  return 8 * g[L - 1].na;                      // the padded ordering of the last level
}

// Device buffers of the multilevel levels (FP64): stencil operators on
// every level, inverses of the self blocks on all but the last, a right
// side and two iterates per level.
std::vector<std::pair<DevBuf*, size_t>> mg_buffers(dg_ctx* ctx, int levels, const MgGrid* g) {
  std::vector<std::pair<DevBuf*, size_t>> out;
  auto& M = ctx->mg;
  for (int l = 0; l < levels; ++l) {
    const size_t na = size_t(g[l].na);
    out.push_back(std::make_pair(&M.E[l], 392 * na * 8));
    if (l + 1 < levels) out.push_back(std::make_pair(&M.Dinv[l], 56 * na * 8));
    out.push_back(std::make_pair(&M.b[l], 8 * na * 8));
    out.push_back(std::make_pair(&M.xa[l], 8 * na * 8));
    out.push_back(std::make_pair(&M.xb[l], 8 * na * 8));
    if (l + 1 < levels) out.push_back(std::make_pair(&M.r[l], 8 * na * 8));
  }
  return out;
}

std::vector<std::pair<DevBuf*, size_t>> coarse_buffers(dg_ctx* ctx, int64_t nc) {
  return {std::make_pair(&ctx->cE, size_t(nc) * nc * 8), std::make_pair(&ctx->cX, size_t(nc) * nc * 8),
          std::make_pair(&ctx->cd, size_t(nc) * 8),
          std::make_pair(&ctx->crc, size_t(nc) * 8), std::make_pair(&ctx->crc2, size_t(nc) * 8),
          std::make_pair(&ctx->cpart, size_t(kCoarseChunks) * nc * 8),
          std::make_pair(&ctx->cipiv, size_t(nc) * 4), std::make_pair(&ctx->cinfo, size_t(4))};
}

// Device scratch rocSOLVER needs for the LU and the inverse of an nc x nc
// FP64 matrix (a size query: nothing runs).  false if the query failed.
bool rocsolver_scratch_bytes(rocblas_handle h, int64_t nc, size_t& bytes) {
  double dummy_d = 0.0;
  rocblas_int dummy_i = 0;
  double* A = &dummy_d;                 // not dereferenced in a size query
  rocblas_int* ip = &dummy_i;
  bytes = 0;
  if (rocblas_start_device_memory_size_query(h) != rocblas_status_success) return false;
  (void)rocsolver_dgetrf(h, rocblas_int(nc), rocblas_int(nc), A, rocblas_int(nc), ip, ip);
  (void)rocsolver_dgetrs(h, rocblas_operation_none, rocblas_int(nc), rocblas_int(nc), A, rocblas_int(nc), ip, A,
                         rocblas_int(nc));
  return rocblas_stop_device_memory_size_query(h, &bytes) == rocblas_status_success;
}

// Hands the handle a scratch of `bytes` from buffer b (carved from the
// context's workspace): rocBLAS then allocates nothing itself.
int give_blas_scratch(dg_ctx* ctx, size_t bytes) {
  if (ctx->blasws.ensure(bytes > 0 ? bytes : 1) != hipSuccess) return fail_mem(ctx, "rocSOLVER scratch", bytes);
  if (rocblas_set_workspace(ctx->blas, ctx->blasws.p, bytes) != rocblas_status_success)
    return fail(DG_EHIP, "rocblas_set_workspace failed");
  return DG_OK;
}

// Every device buffer a context needs for the uses in `features` (a
// DG_WS_* mask) with solver options o, in carve order.  *rocsolver: the
// LU scratch in bytes (0 without the aggregation coarse space).
std::vector<std::pair<DevBuf*, size_t>> plan_workspace(dg_ctx* ctx, const dg_solver_opts& o_in, int features,
                                                       bool& need_rocsolver, int64_t& nc) {
  const dg_solver_opts o = resolve_opts(ctx->mesh, o_in);
  const int64_t FS = ctx->Ne * ctx->np;
  const size_t sS = o.inner_prec == DG_F32 ? 4 : 8;
  std::vector<std::pair<DevBuf*, size_t>> out = {
      std::make_pair(&ctx->phase, size_t(ctx->Ne)), std::make_pair(&ctx->status, sizeof(int)),
      std::make_pair(&ctx->lin, size_t(14) * FS * 8),
      std::make_pair(&ctx->work.out_partial, size_t(kNumSums) * kOutBlocks * 8)};
  const bool step = features & (DG_WS_STEP | DG_WS_NAIVE | DG_WS_H211B);
  if (step || (features & DG_WS_BLOCKS)) {
    const size_t nb = size_t(7) * ctx->np;
    out.push_back(std::make_pair(&ctx->blocks, size_t(ctx->Ne) * nb * nb * sS));
    if (ctx->np == 64) {
      out.push_back(std::make_pair(&ctx->qpiv, size_t(ctx->Ne) * nb * sizeof(int16_t)));
      out.push_back(std::make_pair(&ctx->probe, size_t(14) * FS * sS));
    } else if (sS == 4 && o.block_bf16) {
      out.push_back(std::make_pair(&ctx->bh, size_t(ctx->Ne) * 56 * 56 * 2));
    }
  }
  need_rocsolver = false;
  nc = 0;
  if (step) {
    for (const auto& pr : solver_buffers(ctx, o, sS)) out.push_back(pr);
    if (o.coarse == 3 || o.coarse == 4) {
      nc = coarse_dense_size(ctx->mesh, o);
      for (const auto& pr : coarse_buffers(ctx, nc)) out.push_back(pr);
      need_rocsolver = true;
    }
  }
  const int mgL = mg_levels_for(ctx->mesh, o);
  if ((features & DG_WS_MG) || (step && (o.coarse == 3 || o.coarse == 4) && mgL >= 2)) {
    MgGrid g[kMgMaxLevels];
    mg_grids(coarse_grid(ctx->mesh, o), mgL, g);
    for (const auto& pr : mg_buffers(ctx, mgL, g)) out.push_back(pr);
  }
  if (features & DG_WS_MG) {
    // dg_mg_setup / dg_mg_apply: unit scales, two probe vectors, the dense
    // last level (shared with the solver's when both are planned)
    for (DevBuf* d : {&ctx->mg.ones, &ctx->mg.pv, &ctx->mg.pjv}) out.push_back(std::make_pair(d, size_t(7) * FS * sS));
    if (!need_rocsolver) {
      nc = coarse_dense_size(ctx->mesh, o);
      for (const auto& pr : coarse_buffers(ctx, nc)) out.push_back(pr);
      need_rocsolver = true;
    }
  }
  if ((features & DG_WS_LIMITER) || (step && o.limiter))
    out.push_back(std::make_pair(&ctx->work.lmean, size_t(6) * ctx->Ne * 8));
  if (features & (DG_WS_NAIVE | DG_WS_H211B)) out.push_back(std::make_pair(&ctx->work.z0, size_t(9) * FS * 8));
  if (features & DG_WS_H211B) {
    out.push_back(std::make_pair(&ctx->work.zC, size_t(9) * FS * 8));
    out.push_back(std::make_pair(&ctx->work.zF, size_t(9) * FS * 8));
  }
  return out;
}

// Explicit inverse of the equilibrated coarse operator: cE holds the
// dense nc x nc operator (column-major); afterwards cd holds the
// equilibration d and cX the inverse of D cE D (rocSOLVER LU, then the
// solve of its factors against the identity: level-3 triangular solves,
// where an in-place inverse runs on latency-bound panels).
int coarse_dense_inverse(dg_ctx* ctx, int64_t nc, hipStream_t st) {
  const dim3 blk{256, 1, 1};
  double* cE = ctx->cE.as<double>();
  double* cX = ctx->cX.as<double>();
  double* cd = ctx->cd.as<double>();
  rocblas_int* cipiv = ctx->cipiv.as<rocblas_int>();
  rocblas_int* cinfo = ctx->cinfo.as<rocblas_int>();
  hipLaunchKernelGGL(coarse_diag_kernel, grid1(nc), blk, 0, st, cE, nc, nc, cd);
  hipLaunchKernelGGL(coarse_scale_kernel, dim3(8192), blk, 0, st, cE, nc, nc, cd);
  DG_HIP(hipGetLastError());
  if (rocsolver_dgetrf(ctx->blas, rocblas_int(nc), rocblas_int(nc), cE, rocblas_int(nc), cipiv, cinfo) !=
      rocblas_status_success)
    return fail(DG_EHIP, "rocsolver_dgetrf failed");
  rocblas_int hinfo = 0;
  DG_HIP(hipMemcpyAsync(&hinfo, cinfo, sizeof(hinfo), hipMemcpyDeviceToHost, st));
  DG_HIP(hipStreamSynchronize(st));
  if (hinfo != 0) return fail(DG_ENAN, "singular aggregation coarse operator");
  hipLaunchKernelGGL(identity_kernel, dim3(8192), blk, 0, st, cX, nc);
  if (rocsolver_dgetrs(ctx->blas, rocblas_operation_none, rocblas_int(nc), rocblas_int(nc), cE, rocblas_int(nc),
                       cipiv, cX, rocblas_int(nc)) != rocblas_status_success)
    return fail(DG_EHIP, "rocsolver_dgetrs failed");
  return DG_OK;
}

// Multilevel hierarchy at the stored linearisation (precision S; the
// context's mg levels, grids, sweeps and damping set): level 1 from 7 x 7
// coloured probes of the Krylov operator with basis scales `scales`
// (fields outside `active` keep zero rows and columns), the Galerkin
// products, the inverses of the self blocks and the explicit inverse of
// the last level.  v, Jv: two 7-field vectors of scratch.
template <typename S>
int mg_build(dg_ctx* ctx, const DevParams& P, const S* uS, const S* scales, S* v, S* Jv, int active,
             hipStream_t st) {
  auto& M = ctx->mg;
  const int L = M.levels;
  const int64_t FS = ctx->Ne * ctx->np;
  const dim3 blk{256, 1, 1};
  hipLaunchKernelGGL(mg_fill_kernel<double>, grid1(392 * M.g[0].na), blk, 0, st, M.E[0].as<double>(), 392 * M.g[0].na, 0.0);
  for (int f = 0; f < 7; ++f) {
    if (!((active >> f) & 1)) continue;
    for (int c = 0; c < 7; ++c) {
      hipLaunchKernelGGL(agg_probe_kernel<S>, grid1(7 * FS), blk, 0, st, scales, f, c, M.G, FS, v);
      launch_brick_jvp<S>(ctx, P, uS, v, ctx->lin.p, Jv, st);
      hipLaunchKernelGGL(mg_probe_stencil_kernel<S>, dim3(unsigned(M.G.na)), blk, 0, st, scales, Jv, f, c, M.G, FS,
                         M.E[0].as<double>());
    }
  }
  for (int l = 1; l < L; ++l)
    hipLaunchKernelGGL(mg_galerkin_kernel, mg_grid(56 * M.g[l].na), blk, 0, st, M.E[l - 1].as<const double>(),
                       M.g[l - 1], M.E[l].as<double>(), M.g[l]);
  for (int l = 0; l + 1 < L; ++l)
    hipLaunchKernelGGL(mg_block_inverse_kernel, mg_grid(M.g[l].na), blk, 0, st, M.E[l].as<const double>(), M.g[l].na,
                       M.Dinv[l].as<double>());
  const int64_t nc = 8 * M.g[L - 1].na;
  hipLaunchKernelGGL(mg_fill_kernel<double>, dim3(8192), blk, 0, st, ctx->cE.as<double>(), nc * nc, 0.0);
  hipLaunchKernelGGL(mg_dense_kernel, grid1(392 * M.g[L - 1].na), blk, 0, st, M.E[L - 1].as<const double>(),
                     M.g[L - 1], ctx->cE.as<double>());
  DG_HIP(hipGetLastError());
  return coarse_dense_inverse(ctx, nc, st);
}

// One V-cycle of the multilevel correction on the right side in mg.b[0];
// returns the level-1 result (one of the level's two iterates).
const double* mg_vcycle(dg_ctx* ctx, hipStream_t st) {
  auto& M = ctx->mg;
  const int L = M.levels;
  const dim3 blk{256, 1, 1};
  double* cur[kMgMaxLevels] = {};
  auto sweep = [&](int l, double*& x) {
    double* out = (x == M.xa[l].as<double>()) ? M.xb[l].as<double>() : M.xa[l].as<double>();
    hipLaunchKernelGGL(mg_smooth_kernel, mg_grid(8 * M.g[l].na), blk, 0, st, M.E[l].as<const double>(),
                       M.Dinv[l].as<const double>(), M.g[l], M.b[l].as<const double>(),
                       static_cast<const double*>(x), out, M.omega);
    x = out;
  };
  for (int l = 0; l + 1 < L; ++l) {
    double* x = nullptr;                      // zero
    for (int k = 0; k < M.nu; ++k) sweep(l, x);
    hipLaunchKernelGGL(mg_residual_kernel, mg_grid(8 * M.g[l].na), blk, 0, st, M.E[l].as<const double>(), M.g[l],
                       M.b[l].as<const double>(), static_cast<const double*>(x), M.r[l].as<double>());
    hipLaunchKernelGGL(mg_restrict_kernel, mg_grid(8 * M.g[l + 1].na), blk, 0, st, M.r[l].as<const double>(),
                       M.g[l], M.g[l + 1], M.b[l + 1].as<double>());
    cur[l] = x;
  }
  const int64_t nc = 8 * M.g[L - 1].na;
  const int64_t chunk = (nc + kCoarseChunks - 1) / kCoarseChunks;
  hipLaunchKernelGGL(coarse_gemv_partial_kernel, dim3(unsigned((nc + 255) / 256), kCoarseChunks, 1), blk, 0, st,
                     ctx->cX.as<const double>(), nc, M.b[L - 1].as<const double>(), ctx->cd.as<const double>(), chunk,
                     ctx->cpart.as<double>());
  hipLaunchKernelGGL(coarse_gemv_finish_kernel, grid1(nc), blk, 0, st, ctx->cpart.as<const double>(), nc,
                     ctx->cd.as<const double>(), M.xa[L - 1].as<double>());
  cur[L - 1] = M.xa[L - 1].as<double>();
  for (int l = L - 2; l >= 0; --l) {
    double* x = cur[l];
    if (!x) {
      x = M.xa[l].as<double>();
      hipLaunchKernelGGL(mg_fill_kernel<double>, grid1(8 * M.g[l].na), blk, 0, st, x, 8 * M.g[l].na, 0.0);
    }
    hipLaunchKernelGGL(mg_prolong_add_kernel, mg_grid(8 * M.g[l].na), blk, 0, st,
                       static_cast<const double*>(cur[l + 1]), M.g[l + 1], M.g[l], x);
    for (int k = 0; k < M.nu; ++k) sweep(l, x);
    cur[l] = x;
  }
  return cur[0];
}

template <typename S>
int newton_solve(dg_ctx* ctx, double t_n, double dt, double* u, const dg_solver_opts& o_in,
                 dg_step_report* rep, hipStream_t st, int active = kAllFields) {
  const dg_solver_opts o = resolve_opts(ctx->mesh, o_in);
  const int64_t FS = ctx->Ne * ctx->np, n7 = 7 * FS, n9 = 9 * FS;
  const int m = o.gmres_restart;
  SolverWork& W = ctx->work;
  const size_t sS = sizeof(S);
  for (const auto& pr : solver_buffers(ctx, o, sS))
    if (pr.first->ensure(pr.second) != hipSuccess) return fail_mem(ctx, "dg_step workspace", pr.second);
  if (int s = gmres_host_state(ctx)) return s;
  DevParams P = make_params(ctx, t_n + dt, dt);
  P.active = active;
  const double phi_floor = kGas * ctx->params.T / kFaraday;
  // The linear system of the inner solve is J du = rhs multiplied by rs (a
  // power of two): raw residual rows span ~1e-42 (trace species near the
  // root) to ~1e-10, below the FP32 normal range at the small end, and the
  // scaled ones sit well inside it.  The correction is divided by rs in FP64.
  const double rs = std::is_same<S, float>::value ? 0x1p40 : 1.0;
  double* m_old = W.m_old.as<double>();
  double* R = W.R.as<double>();
  double* Rtry = W.Rtry.as<double>();
  double* u_try = W.u_try.as<double>();
  double* du = W.du.as<double>();
  double* wR = W.wR.as<double>();
  S *uS = W.uS.as<S>(), *sc = W.sc.as<S>(), *V = W.V.as<S>(), *w = W.w.as<S>(), *t = W.t.as<S>();
  S *pJ = W.pJ.as<S>(), *rhs = W.rhs.as<S>(), *b = W.b.as<S>(), *x = W.x.as<S>();
  S *y9 = W.y9.as<S>(), *v9 = W.v9.as<S>(), *partial = W.partial.as<S>(), *dots = W.dots.as<S>();
  S *yc = W.yc.as<S>(), *hbuf = W.hbuf.as<S>(), *JZ = W.JZ.as<S>();
  S *pc = W.pc.as<S>(), *pc2 = W.pc2.as<S>(), *scc = W.scc.as<S>();
  double* partial64 = W.partial64.as<double>();
  double* Ainv = W.Ainv.as<double>();
  double* gs = W.gsum.as<double>();             // [|w|^2 (FP64)][h1 (kMaxDots x S)][h2 (kMaxDots x S)]
  S* gs_h1 = reinterpret_cast<S*>(gs + 1);
  S* gs_h2 = gs_h1 + kMaxDots;
  const dim3 blk{256, 1, 1};
  // Reductions run on kRedBlocks workgroups, or on fewer for small meshes:
  // no more workgroups than a Krylov vector has quads of 4 entries per 256
  // lanes (the extra ones would only add empty block sums and partials).
  // The consumers of the partials read exactly nred of them.
  const int nred = int(std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (n7 / 4 + 255) / 256)));
  const dim3 gred{unsigned(nred), 1, 1};
  const dim3 gw{unsigned((ctx->Ne + 3) / 4), 1, 1};
  const dim3 g1{1, 1, 1}, g7{7, 1, 1};

  // aggregation coarse space (coarse = 3)
  AggGrid G{};
  int64_t nc = 0;
  const bool agg = (o.coarse == 3 || o.coarse == 4);
  const int mgL = mg_levels_for(ctx->mesh, o);
  const bool mgm = agg && mgL >= 2;            // the coarse solve by a multilevel V-cycle
  auto& MG = ctx->mg;
  if (agg) {
    G = coarse_grid(ctx->mesh, o);
    nc = coarse_dense_size(ctx->mesh, o);
    if (nc > (int64_t(1) << 20)) return fail(DG_EINVAL, "dg_step: coarse space too large (raise coarse_agg)");
    if (mgm) {
      if (nc > 8192) return fail(DG_EINVAL, "dg_step: the last multigrid level has more than 8192 unknowns (add levels)");
      MG.prec = -1;                              // the hierarchy becomes the solver's
      MG.levels = mgL;
      MG.nu = o.mg_sweeps;
      MG.omega = o.mg_omega;
      MG.G = G;
      mg_grids(G, MG.levels, MG.g);
      for (const auto& pr : mg_buffers(ctx, MG.levels, MG.g))
        if (pr.first->ensure(pr.second) != hipSuccess) return fail_mem(ctx, "multigrid levels", pr.second);
    }
    for (const auto& pr : coarse_buffers(ctx, nc))
      if (pr.first->ensure(pr.second) != hipSuccess) return fail_mem(ctx, "coarse space", pr.second);
    if (!ctx->blas && rocblas_create_handle(&ctx->blas) != rocblas_status_success)
      return fail(DG_EHIP, "rocblas_create_handle failed");
    if (rocblas_set_stream(ctx->blas, st) != rocblas_status_success) return fail(DG_EHIP, "rocblas_set_stream failed");
    if (!ctx->owns_memory && ctx->blasws.bytes == 0) {
      // the LU's scratch from the caller's workspace too
      size_t need = 0;
      if (!rocsolver_scratch_bytes(ctx->blas, nc, need))
        return fail(DG_EHIP, "dg_step: rocSOLVER scratch size query failed");
      if (int s = give_blas_scratch(ctx, need)) return s;
    }
  }
  double* cE = ctx->cE.as<double>();
  double* cX = ctx->cX.as<double>();
  double* cd = ctx->cd.as<double>();
  double* crc = ctx->crc.as<double>();
  double* crc2 = ctx->crc2.as<double>();
  double* cgemv = ctx->cpart.as<double>();     // partial sums of the coarse GEMV
  rocblas_int* cipiv = ctx->cipiv.as<rocblas_int>();
  rocblas_int* cinfo = ctx->cinfo.as<rocblas_int>();
  const dim3 gagg{unsigned(G.na > 0 ? G.na : 1), 1, 1};

  auto resid64 = [&](const double* uu, double* out) {
    launch_q1<double, double, kResidual>(ctx, P, uu, nullptr, m_old, out, st);
  };
  auto jvp_cond = [&](const S* v7, S* out) { launch_brick_jvp<S>(ctx, P, uS, v7, ctx->lin.p, out, st); };
  // coarse coefficients yc = E^-1 Z^T r (E = Z^T J Z, Z_f = sc on field f)
  auto coarse_coeffs = [&](const S* r) {
    hipLaunchKernelGGL(field_dot_kernel<S>, gred, blk, 0, st, sc, r, FS, partial);
    hipLaunchKernelGGL(coarse_solve_kernel<S>, g1, blk, 0, st, partial, nred, Ainv, yc);
  };
  // deflation r <- P r = r - J Z E^-1 Z^T r (leaves yc = E^-1 Z^T r)
  auto deflate = [&](S* r) {
    if (o.coarse != 2) return;
    coarse_coeffs(r);
    hipLaunchKernelGGL(multi_axpy_kernel<S>, grid1(n7), blk, 0, st, JZ, n7, 7, yc, S(-1), r, n7);
  };
  // preconditioner: out = B^-1 r (+ Z E^-1 Z^T r for the additive coarse
  // space; the deflated variant has already removed that part from r)
  // out = Z E^-1 Z^T r (aggregation coarse space): E^-1 = D Einv D with the
  // explicit inverse Einv of the equilibrated operator, applied as one dense
  // GEMV (triangular solves with the LU factors run far below HBM speed)
  auto coarse_solve_into = [&](const S* r, S* out, bool add, const S* div = nullptr) {
    if (mgm) {
      hipLaunchKernelGGL(mg_restrict_fine_kernel<S>, gagg, blk, 0, st, scc, r, G, FS, MG.b[0].as<double>());
      const double* y = mg_vcycle(ctx, st);
      hipLaunchKernelGGL(mg_prolong_fine_kernel<S>, grid1(FS), blk, 0, st, scc, y, G, FS, out, div, !add);
      return;
    }
    hipLaunchKernelGGL(agg_restrict_kernel<S>, gagg, blk, 0, st, scc, r, G, FS, crc);
    const int64_t chunk = (nc + kCoarseChunks - 1) / kCoarseChunks;
    hipLaunchKernelGGL(coarse_gemv_partial_kernel, dim3(unsigned((nc + 255) / 256), kCoarseChunks, 1), blk, 0, st,
                       cX, nc, crc, cd, chunk, cgemv);
    hipLaunchKernelGGL(coarse_gemv_finish_kernel, grid1(nc), blk, 0, st, cgemv, nc, cd, crc2);
    if (!add) hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(0), out, S(0), out, n7);
    hipLaunchKernelGGL(agg_prolong_add_kernel<S>, grid1(FS), blk, 0, st, scc, crc2, G, FS, out, div);
  };
  // out = M^-1 r, divided entrywise by the unknown scales sc (fused into the
  // coarse prolongation when the coarse space is additive on aggregates)
  auto precond = [&](S* r, S* out) {
    auto unscale = [&]() { hipLaunchKernelGGL((emul_kernel<S, true>), grid1(n7), blk, 0, st, sc, out, out, n7); };
    if (o.coarse == 4) {
      // multiplicative two-level: coarse solve, then the element blocks on
      // the remaining residual: out = (c + B^-1 (r - J c)) / sc with
      // c = Z E^-1 Z^T r; the Krylov operator forms r - J c and the block
      // apply adds c and divides by the scales in their own passes
      coarse_solve_into(r, pc, false);
      launch_brick_jvp<S>(ctx, P, uS, pc, ctx->lin.p, pc2, st, r);
      if constexpr (std::is_same<S, float>::value) {
        if (o.block_bf16)
          hipLaunchKernelGGL((apply_blocks_bf16_kernel<7>), gw, blk, 0, st, ctx->bh.as<const uint16_t>(), pc2,
                             out, ctx->Ne, pc, sc);
        else
          hipLaunchKernelGGL((apply_blocks_kernel<S, 7>), gw, blk, 0, st, ctx->blocks.as<const S>(),
                             pc2, out, ctx->Ne, pc, sc);
      } else {
        hipLaunchKernelGGL((apply_blocks_kernel<S, 7>), gw, blk, 0, st, ctx->blocks.as<const S>(), pc2,
                           out, ctx->Ne, pc, sc);
      }
      return;
    }
    deflate(r);
    if constexpr (std::is_same<S, float>::value) {
      if (o.block_bf16)
        hipLaunchKernelGGL((apply_blocks_bf16_kernel<7>), gw, blk, 0, st, ctx->bh.as<const uint16_t>(), r, out,
                           ctx->Ne);
      else
        hipLaunchKernelGGL((apply_blocks_kernel<S, 7>), gw, blk, 0, st, ctx->blocks.as<const S>(), r,
                           out, ctx->Ne);
    } else {
      hipLaunchKernelGGL((apply_blocks_kernel<S, 7>), gw, blk, 0, st, ctx->blocks.as<const S>(), r,
                         out, ctx->Ne);
    }
    if (o.coarse == 1) {
      coarse_coeffs(r);
      hipLaunchKernelGGL(coarse_add_kernel<S>, grid1(n7), blk, 0, st, sc, yc, out, FS);
      unscale();
    } else if (o.coarse == 3) {
      coarse_solve_into(r, out, true, sc);  // additive: out += Z E^-1 Z^T r, then / sc
    } else {
      unscale();
    }
  };
  auto opA = [&](const S* v, S* out) {           // out = sc^-1 M^-1 J (sc v)
    hipLaunchKernelGGL((emul_kernel<S, false>), grid1(n7), blk, 0, st, sc, v, t, n7);
    jvp_cond(t, pJ);
    precond(pJ, out);
  };
  // out <- the sum of the FP64 block partials in partial64
  auto finish_sumsq = [&](double& out) -> int {
    hipLaunchKernelGGL(finish_sum_kernel<double>, g1, blk, 0, st, partial64, nred,
                       reinterpret_cast<double*>(hbuf));
    double hs = 0;
    DG_HIP(hipMemcpyAsync(&hs, hbuf, sizeof(double), hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    out = hs;
    return DG_OK;
  };
  auto sumsq = [&](const S* a, int64_t n, double& out) -> int {
    hipLaunchKernelGGL(sumsq_kernel<S>, gred, blk, 0, st, a, n, partial64);
    double hs = 0;
    if (int s = finish_sumsq(hs)) return s;
    out = hs;
    return DG_OK;
  };
  // merit(Rv)^2 = ||sc^-1 M^-1 R_u||^2 (+ ||E^-1 Z^T R_u||^2 when deflated)
  //              + ||R_eps / (W (rho/M)/dt sc_eps)||^2,
  // with the operators, scales and iterate of this Newton iteration: the
  // norm in which GMRES reduced the linearised residual (the deflated coarse
  // part of it vanishes exactly), so the Newton direction descends it.
  auto merit = [&](const double* Rv, double& out) -> int {
    hipLaunchKernelGGL((scaled_cast_kernel<double, S>), grid1(n7), blk, 0, st, Rv, rs, t, n7);
    if (active != kAllFields) hipLaunchKernelGGL(mask_fields_kernel<S>, grid1(n7), blk, 0, st, t, FS, active);
    double cpart = 0.0;
    precond(t, pJ);
    if (o.coarse == 2) {
      S hy[7];
      DG_HIP(hipMemcpyAsync(hy, yc, 7 * sizeof(S), hipMemcpyDeviceToHost, st));
      DG_HIP(hipStreamSynchronize(st));
      for (int f = 0; f < 7; ++f) cpart += double(hy[f]) * double(hy[f]);
    }
    double a = 0.0;
    if (int s = sumsq(pJ, n7, a)) return s;
    hipLaunchKernelGGL(solid_merit_kernel, gred, blk, 0, st, Rv, u, FS, P, partial64);
    hipLaunchKernelGGL(finish_sum_kernel<double>, g1, blk, 0, st, partial64, nred,
                       reinterpret_cast<double*>(hbuf));
    double bsum = 0.0;
    DG_HIP(hipMemcpyAsync(&bsum, hbuf, sizeof(double), hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    out = (a + cpart) / (rs * rs) + bsum;
    return DG_OK;
  };

  // old mass of the step and first residual
  hipLaunchKernelGGL(mass_kernel<double>, grid1(n9), blk, 0, st, u, m_old, ctx->d_phase, P, ctx->np);
  resid64(u, R);
  DG_HIP(hipGetLastError());
  dg_step_report r{};
  r.mg_levels = mgm ? mgL : 0;
  int status = DG_ENOCONV;
  // Near the root the linear-solve tolerance is tightened, and the iteration
  // stops once a full step no longer shrinks the update: the attainable
  // accuracy of an iterative solve is then reached (the report says so).
  double gm_rtol = o.gmres_rtol;
  double best_upd = 1e300;
  int stall = 0, prev_its = 0;
  // Operator and preconditioner are rebuilt at every Newton iterate: a
  // preconditioner kept from an earlier iterate cost more GMRES iterations
  // than its rebuild on the 16^3 cube.
  int coarse_built = 0;                       // iterate of the last coarse rebuild
  for (int it = 1; it <= o.newton_maxit; ++it) {
    r.newton_its = it;
    hipLaunchKernelGGL((cast_kernel<double, S>), grid1(n9), blk, 0, st, u, uS, n9);
    if (int s = linearize<S>(ctx, P, uS, st)) return s;
    // FP32 inner solves with block_bf16 use only the bfloat16 inverses
    // the element blocks are rebuilt at every iterate, or (block_reuse > 0)
    // only at the first and after an update whose largest relative change
    // exceeded block_reuse: near the root the Jacobian moves by the size of
    // the update, and blocks of an earlier iterate precondition as well
    if (it == 1 || !(o.block_reuse > 0.0) || r.last_update > o.block_reuse) {
      if (int s = blocks_setup<S>(ctx, P, uS, st, std::is_same<S, float>::value && o.block_bf16 != 0)) return s;
      ++r.block_builds;
    }
    hipLaunchKernelGGL(scales_kernel<S>, grid1(n7), blk, 0, st, u, sc, FS, phi_floor);
    // the aggregation coarse operator is rebuilt at the first iterate, after
    // an update whose largest relative change of an unknown exceeded 2 (E
    // moves with the iterate) and every coarse_every iterates; in between,
    // E^-1 of the last rebuild stays a good coarse correction (the element
    // blocks are rebuilt at every iterate)
    if (agg && (it == 1 || r.last_update > 2.0 || it - coarse_built >= o.coarse_every)) {
      // aggregation coarse operator E = Z^T J Z by coloured probes, then LU;
      // Z keeps the unknown scales of this rebuild (scc)
      coarse_built = it;
      hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(1), sc, S(0), scc, n7);
      if (mgm) {
        if (int s = mg_build<S>(ctx, P, uS, scc, t, pJ, active, st))
          return fail(s, std::string("dg_step: ") + g_last_error);
      } else {
        DG_HIP(hipMemsetAsync(cE, 0, size_t(nc) * nc * 8, st));
        for (int f = 0; f < 7; ++f) {
          if (!((active >> f) & 1)) continue;
          for (int c = 0; c < 7; ++c) {
            hipLaunchKernelGGL(agg_probe_kernel<S>, grid1(n7), blk, 0, st, scc, f, c, G, FS, t);
            jvp_cond(t, pJ);
            hipLaunchKernelGGL(agg_probe_reduce_kernel<S>, gagg, blk, 0, st, scc, pJ, f, c, G, FS, cE, nc);
          }
        }
        if (int s = coarse_dense_inverse(ctx, nc, st)) return fail(s, std::string("dg_step: ") + g_last_error);
      }
    }
    // coarse operator Ac[g][f] = sum_g sc_g (J Z_f)_g
    if (o.coarse == 1 || o.coarse == 2) {
      std::vector<double> Ac(49), col(7);
      for (int f = 0; f < 7; ++f) {
        S* JZf = JZ + int64_t(f) * n7;
        if (!((active >> f) & 1)) {            // inactive field: identity row and column
          hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(0), JZf, S(0), JZf, n7);
          for (int g = 0; g < 7; ++g) Ac[g * 7 + f] = (g == f) ? 1.0 : 0.0;
          continue;
        }
        hipLaunchKernelGGL(field_select_kernel<S>, grid1(n7), blk, 0, st, sc, f, t, FS);
        jvp_cond(t, JZf);
        hipLaunchKernelGGL(field_dot_kernel<S>, gred, blk, 0, st, sc, JZf, FS, partial);
        hipLaunchKernelGGL(finish_sum_kernel<S>, g7, blk, 0, st, partial, nred, dots);
        std::vector<S> hs(7);
        DG_HIP(hipMemcpyAsync(hs.data(), dots, 7 * sizeof(S), hipMemcpyDeviceToHost, st));
        DG_HIP(hipStreamSynchronize(st));
        for (int g = 0; g < 7; ++g) Ac[g * 7 + f] = ((active >> g) & 1) ? double(hs[g]) : 0.0;
      }
      // symmetric equilibration D Ac D, D = |diag|^-1/2, before inverting:
      // the entries of Ac span many orders of magnitude
      std::vector<double> dsc(7), As(49), inv(49);
      for (int g = 0; g < 7; ++g) {
        const double a = std::fabs(Ac[g * 7 + g]);
        dsc[g] = (a > 0 && std::isfinite(a)) ? 1.0 / std::sqrt(a) : 1.0;
      }
      for (int g = 0; g < 7; ++g)
        for (int f = 0; f < 7; ++f) As[g * 7 + f] = dsc[g] * Ac[g * 7 + f] * dsc[f];
      for (int c = 0; c < 7; ++c) {
        std::vector<double> e(7, 0.0);
        e[c] = 1.0;
        if (!dense_solve(7, As, e)) return fail(DG_ENAN, "dg_step: singular coarse operator");
        for (int g = 0; g < 7; ++g) inv[g * 7 + c] = dsc[g] * e[g] * dsc[c];
      }
      DG_HIP(hipMemcpyAsync(Ainv, inv.data(), 49 * sizeof(double), hipMemcpyHostToDevice, st));
    }
    // condensed right side
    hipLaunchKernelGGL(solid_rhs_kernel, grid1(FS), blk, 0, st, u, R, wR, ctx->d_phase, P, ctx->np);
    hipLaunchKernelGGL(solid_direction_kernel<S>, grid1(n9), blk, 0, st, wR, rs, v9, FS);
    launch_q1<S, Dual<S>, kJvpFull>(ctx, P, uS, v9, nullptr, y9, st);
    hipLaunchKernelGGL(condensed_rhs_kernel<S>, grid1(n7), blk, 0, st, R, rs, y9, rhs, FS, active);
    hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(1), rhs, S(0), w, n7);
    precond(w, b);
    double merit0 = 0.0;
    if (int s = merit(R, merit0)) return s;
    if (!std::isfinite(merit0)) return fail(DG_ENAN, "dg_step: non-finite residual");
    if (it == 1) r.merit0 = std::sqrt(merit0);

    // GMRES(m) on sc^-1 M^-1 J sc y = b, x0 = 0, with the cycle's Hessenberg
    // matrix, rotations and stopping test on the device (GmresState): an
    // iteration issues its kernels without waiting for the previous one;
    // the host reads the cycle's done flag one iteration late (pinned copy
    // and event), so at most one iteration past convergence is issued, and
    // its kernels change nothing.
    hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(0), b, S(0), x, n7);
    double beta0 = 0.0;
    if (int s = sumsq(b, n7, beta0)) return s;
    beta0 = std::sqrt(beta0);
    if (!std::isfinite(beta0)) return fail(DG_ENAN, "dg_step: non-finite preconditioned right side");
    int its = 0;
    // near the root an FP32 Krylov solve may stagnate above its tolerance:
    // bound its cost by the previous solve instead of running to gmres_maxit
    const bool near_root = best_upd < 1e-7;
    const int maxit = near_root ? std::min(o.gmres_maxit, std::max(200, 4 * prev_its)) : o.gmres_maxit;
    double rel = 0.0;
    if (beta0 > 0.0) {
      GmresState* gst = W.gstate.as<GmresState>();
      int32_t* hflag = ctx->gm_flags;
      bool first = true;
      while (its < maxit) {
        S* V0 = V;
        if (first) {
          hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(1), b, S(0), V0, n7);
        } else {
          opA(x, w);
          hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(1), b, S(-1), w, n7);
          hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(1), w, S(0), V0, n7);
        }
        hipLaunchKernelGGL(sumsq_kernel<S>, gred, blk, 0, st, V0, n7, partial64);
        hipLaunchKernelGGL(gmres_start_kernel, g1, blk, 0, st, gst, partial64, nred, first ? 1 : 0, gm_rtol);
        hipLaunchKernelGGL(gmres_scale_kernel<S>, grid1(n7), blk, 0, st, gst, V0, V0, n7);
        first = false;
        DG_HIP(hipMemcpyAsync(&hflag[0], &gst->done, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        DG_HIP(hipStreamSynchronize(st));
        if (hflag[0]) break;                       // zero residual: nothing to do
        for (int jj = 0; jj < m && its + jj < maxit; ++jj) {
          opA(V + int64_t(jj) * n7, w);
          // classical Gram-Schmidt applied twice (with FP32 basis vectors a
          // single pass, even with a reorthogonalisation test, loses enough
          // orthogonality to slow the preconditioned iteration), its second
          // pass delayed to the next iteration (krylov.hpp): two sweeps over
          // the basis, sweep 1 correcting the previous vector and projecting
          // the operator's output, sweep 2 forming w1 with its second-pass
          // projections and |w1|^2
          const dim3 gj{unsigned(jj + 1), 1, 1};
          hipLaunchKernelGGL(dcgs_sweep1_kernel<S>, gred, blk, 0, st, gst, V, n7, jj, w, n7, partial);
          hipLaunchKernelGGL(finish_sum_kernel<S>, gj, blk, 0, st, partial, nred, gs_h1);
          hipLaunchKernelGGL(dcgs_coef_kernel<S>, g1, dim3(64), 0, st, gst, gs_h1, jj, hbuf);
          hipLaunchKernelGGL(dcgs_sweep2_kernel<S>, gred, blk, 0, st, gst, V, n7, jj + 1, hbuf, w, n7, partial,
                             partial64);
          hipLaunchKernelGGL(finish_sum_kernel<S>, gj, blk, 0, st, partial, nred, gs_h2);
          hipLaunchKernelGGL(finish_sum_kernel<double>, g1, blk, 0, st, partial64, nred, gs);
          hipLaunchKernelGGL(dcgs_column_kernel<S>, g1, dim3(64), 0, st, gst, gs, jj, m);
          hipLaunchKernelGGL(gmres_scale_kernel<S>, grid1(n7), blk, 0, st, gst, w, V + int64_t(jj + 1) * n7, n7);
          DG_HIP(hipMemcpyAsync(&hflag[jj & 1], &gst->done, sizeof(int32_t), hipMemcpyDeviceToHost, st));
          DG_HIP(hipEventRecord(ctx->gm_ev[jj & 1], st));
          if (jj >= 1) {
            DG_HIP(hipEventSynchronize(ctx->gm_ev[(jj - 1) & 1]));
            if (hflag[(jj - 1) & 1]) break;
          }
        }
        DG_HIP(hipGetLastError());
        // x += V y with the cycle's least-squares solution
        GmresState hs;
        hipLaunchKernelGGL(gmres_solve_kernel<S>, g1, dim3(64), 0, st, gst, hbuf);
        DG_HIP(hipMemcpyAsync(&hs.rel, &gst->rel, sizeof(double) + 4 * sizeof(int32_t) + sizeof(double),
                              hipMemcpyDeviceToHost, st));
        DG_HIP(hipStreamSynchronize(st));
        if (hs.cols > 0)
          hipLaunchKernelGGL(multi_axpy_kernel<S>, grid1(n7), blk, 0, st, V, n7, hs.cols, hbuf, S(1), x, n7);
        its = hs.its;
        rel = hs.rel;
        if (hs.converged || hs.cols == 0) break;
      }
    }
    r.gmres_its += its;
    r.gmres_last_rel = rel;
    prev_its = its;
    const bool gmres_short = rel > gm_rtol;
    // Newton direction: xhat = sc x, then the exact coarse component
    //   du_u = xhat + Z E^-1 Z^T (rhs - J xhat),
    // solids from the condensation.
    hipLaunchKernelGGL((emul_kernel<S, false>), grid1(n7), blk, 0, st, sc, x, t, n7);
    if (o.coarse == 2) {
      jvp_cond(t, pJ);
      hipLaunchKernelGGL(axpby_kernel<S>, grid1(n7), blk, 0, st, S(1), rhs, S(-1), pJ, n7);
      coarse_coeffs(pJ);
      hipLaunchKernelGGL(coarse_add_kernel<S>, grid1(n7), blk, 0, st, sc, yc, t, FS);
    }
    hipLaunchKernelGGL((scaled_cast_kernel<S, double>), grid1(n7), blk, 0, st, t, 1.0 / rs, du, n7);
    hipLaunchKernelGGL(solid_delta_kernel, grid1(FS), blk, 0, st, u, du, wR, du + n7, ctx->d_phase, P,
                       ctx->np);
    if (o.verbose >= 2) {
      std::vector<double> hu(n9), hd(n9);
      DG_HIP(hipMemcpyAsync(hu.data(), u, n9 * 8, hipMemcpyDeviceToHost, st));
      DG_HIP(hipMemcpyAsync(hd.data(), du, n9 * 8, hipMemcpyDeviceToHost, st));
      DG_HIP(hipStreamSynchronize(st));
      std::fprintf(stderr, "[dg_step]   field: min u | max |du|/max(|u|,floor)\n");
      for (int f = 0; f < 9; ++f) {
        double mn = 1e300, mx = 0;
        const double fl = f == 6 ? phi_floor : (f < 6 ? 1e-20 : 1e-12);
        int64_t at = 0;
        for (int64_t k = 0; k < FS; ++k) {
          const double x = hu[f * FS + k];
          mn = std::min(mn, x);
          const double r = std::fabs(hd[f * FS + k]) / std::max(std::fabs(x), fl);
          if (r > mx) { mx = r; at = k; }
        }
        std::fprintf(stderr, "[dg_step]   %d: %.3e | %.3e at node %lld (u %.3e du %.3e)\n", f, mn, mx,
                     (long long)at, hu[f * FS + at], hd[f * FS + at]);
      }
    }
    // backtracking line search on the merit (weights of this iterate)
    double lam = 1.0, upd = 0.0, mt = 0.0;
    bool found = false;
    for (int ls = 0; ls <= (near_root ? 3 : 40); ++ls) {
      hipLaunchKernelGGL(newton_update_kernel, gred, blk, 0, st, u, du, lam, u_try, FS, phi_floor, partial64,
                         o.limiter);
      std::vector<double> pm(nred);
      DG_HIP(hipMemcpyAsync(pm.data(), partial64, nred * sizeof(double), hipMemcpyDeviceToHost, st));
      resid64(u_try, Rtry);
      if (int s = merit(Rtry, mt)) return s;
      upd = *std::max_element(pm.begin(), pm.end());
      // near the root the merit (preconditioned in the inner precision)
      // cannot rank steps any more: full steps are then taken as iterative
      // refinement and the update-based stall test ends the iteration
      if (std::isfinite(mt) && (mt < merit0 || (lam == 1.0 && (upd < 1e-8 || near_root)))) {
        found = true;
        break;
      }
      lam *= 0.5;
      ++r.line_search_cuts;
    }
    if (!found) {
      // no decrease along this direction: near the root the linear solve has
      // reached its attainable accuracy (keep the iterate); elsewhere fail
      if (o.verbose)
        std::fprintf(stderr, "[dg_step] newton %d: line search found no decrease (update %.3e)\n", it, upd);
      if (std::min(best_upd, upd) < 1e-7) {
        status = DG_OK;
        r.stalled = 1;
      }
      break;
    }
    DG_HIP(hipMemcpyAsync(u, u_try, n9 * sizeof(double), hipMemcpyDeviceToDevice, st));
    DG_HIP(hipMemcpyAsync(R, Rtry, n9 * sizeof(double), hipMemcpyDeviceToDevice, st));
    r.merit_final = std::sqrt(mt);
    r.last_update = upd;
    if (o.verbose)
      std::fprintf(stderr, "[dg_step] newton %d gmres %d (rel %.2e) update %.3e lambda %.3g merit %.3e -> %.3e\n",
                   it, its, rel, upd, lam, std::sqrt(merit0), std::sqrt(mt));
    if (!std::isfinite(mt)) {
      status = DG_ENAN;
      break;
    }
    if (lam == 1.0 && upd < o.newton_tol) {
      status = DG_OK;
      break;
    }
    if (near_root && gmres_short) {
      // the linear solve stagnated at its attainable accuracy: stop here
      status = DG_OK;
      r.stalled = 1;
      break;
    }
    if (lam == 1.0 && upd < 1e-7) {
      // FP32 Krylov vectors cannot resolve much below their unit roundoff
      const double floor_rtol = std::is_same<S, float>::value ? 1e-5 : 0.0;
      gm_rtol = std::max(std::min(gm_rtol, o.gmres_rtol_final), floor_rtol);
      if (upd < 0.5 * best_upd) {
        stall = 0;
      } else if (++stall >= (std::is_same<S, float>::value ? 6 : 3)) {
        status = DG_OK;
        r.stalled = 1;
        break;
      }
    }
    best_upd = std::min(best_upd, upd);
  }
  DG_HIP(hipStreamSynchronize(st));
  r.status = status;
  if (rep) *rep = r;
  if (status == DG_ENOCONV) return fail(DG_ENOCONV, "dg_step: Newton did not converge");
  if (status == DG_ENAN) return fail(DG_ENAN, "dg_step: non-finite residual");
  return DG_OK;
}

// Checked copy of the solver options with the precision-dependent default
// coarse space filled in.
int normalize_opts(const dg_solver_opts* in, dg_solver_opts& o, const char* fn) {
  if (in) o = *in; else dg_solver_opts_default(&o);
  if (o.gmres_restart < 1 || o.gmres_restart > kMaxDots - 2)
    return fail(DG_EINVAL, std::string(fn) + ": gmres_restart must be in 1..30");
  if (o.newton_maxit < 1 || o.gmres_maxit < 1) return fail(DG_EINVAL, std::string(fn) + ": iteration limits");
  if (o.inner_prec != DG_F32 && o.inner_prec != DG_F64)
    return fail(DG_EINVAL, std::string(fn) + ": bad inner precision");
  if (o.coarse > 4) return fail(DG_EINVAL, std::string(fn) + ": coarse must be -1..4");
  if (o.coarse == 0) o.coarse = kCoarseDefault;  // 3 or 4, once the mesh is known (resolve_opts)
  if (o.coarse < 0) o.coarse = 0;
  if (o.coarse_every == 0) o.coarse_every = 3;
  if (o.coarse_every < 0) return fail(DG_EINVAL, std::string(fn) + ": coarse_every must be >= 0");
  if (o.limiter != 0 && o.limiter != 1) return fail(DG_EINVAL, std::string(fn) + ": limiter must be 0 or 1");
  if (o.mg_levels != 0) {
    if (o.mg_levels != -1 && (o.mg_levels < 2 || o.mg_levels > kMgMaxLevels))
      return fail(DG_EINVAL, std::string(fn) + ": mg_levels must be -1, 0 or 2..8");
    if (o.mg_sweeps < 0 || o.mg_sweeps > 8) return fail(DG_EINVAL, std::string(fn) + ": mg_sweeps must be in 0..8");
    if (!(o.mg_omega > 0.0 && o.mg_omega <= 1.0))
      return fail(DG_EINVAL, std::string(fn) + ": mg_omega must be in (0, 1]");
  }
  if (o.coarse_agg < 0) return fail(DG_EINVAL, std::string(fn) + ": coarse_agg must be >= 0");
  if (!(o.block_reuse >= 0.0)) return fail(DG_EINVAL, std::string(fn) + ": block_reuse must be >= 0");
  return DG_OK;
}

// Vertex-based limiter of the Q1 state u in place (limiter.hpp); alpha:
// optional device array of the factors (6 x Ne).  Order 0 has nothing to
// limit.
int limit_state(dg_ctx* ctx, double* u, double* alpha, hipStream_t st) {
  if (ctx->np == 1) return DG_OK;
  if (ctx->np != 8) return fail(DG_EUNSUPPORTED, "dg_limit: the vertex-based limiter is for orders 0 and 1");
  const size_t need = size_t(6) * ctx->Ne * sizeof(double);
  if (ctx->work.lmean.ensure(need) != hipSuccess) return fail_mem(ctx, "limiter workspace", need);
  const DevParams P = make_params(ctx, 0.0, 1.0);
  double* mb = ctx->work.lmean.as<double>();
  hipLaunchKernelGGL(limit_means_kernel, grid1(ctx->Ne), dim3(256), 0, st, u, ctx->d_phase, P, mb);
  hipLaunchKernelGGL(limit_apply_kernel, grid1(ctx->Ne), dim3(256), 0, st, u, ctx->d_phase, P,
                     static_cast<const double*>(mb), alpha);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int solve_once(dg_ctx* ctx, double t_n, double dt, double* u, const dg_solver_opts& o, dg_step_report* rep,
               hipStream_t st, int active = kAllFields) {
  const int s = o.inner_prec == DG_F32 ? newton_solve<float>(ctx, t_n, dt, u, o, rep, st, active)
                                       : newton_solve<double>(ctx, t_n, dt, u, o, rep, st, active);
  if (s != DG_OK || !o.limiter || active != kAllFields) return s;
  if (int e = limit_state(ctx, u, nullptr, st)) return e;
  DG_HIP(hipStreamSynchronize(st));
  return DG_OK;
}

}  // namespace

// A batch of independent structures: one context per structure for its
// derived parameters, plus the concatenated device tables of the batch.
struct dg_batch {
  std::vector<dg_ctx*> subs;
  std::vector<int64_t> off;            // voxel offsets, n + 1 values
  int64_t E = 0;                       // total voxels
  int64_t ntiles = 0;
  uint8_t* d_phase = nullptr;
  BatchTile* d_tiles = nullptr;        // 32-voxel work items (= d_tiles_by[2])
  BatchTile* d_tiles_by[3] = {};       // work items of kTileChoices[i] voxels
  int64_t ntiles_by[3] = {};
  dg_batch_shape shape[2][3];          // launch shape by precision and operator (dg_batch_op)
  int n_cu = 0;                        // compute units of the device
  DevParams* d_params = nullptr;
  DevParams* h_params = nullptr;       // pinned staging of d_params
  BatchTile* d_bricks = nullptr;       // bricks of 4 x 4 x 4 voxels (v0 = brick index in its structure)
  int64_t nbricks = 0;
  KP<float>* d_kpf = nullptr;          // folded parameters of the brick operator, by precision
  KP<double>* d_kpd = nullptr;
  KP<float>* h_kpf = nullptr;          // pinned staging of d_kpf, d_kpd
  KP<double>* h_kpd = nullptr;
  hipEvent_t staged = nullptr;         // recorded after each upload of h_params
  DevBuf lin, blocks, status;
  int lin_prec = -1, blocks_prec = -1;
  std::vector<DevBuf> wstate;          // per-worker contiguous states (batched solves)
};

namespace {

// Per-structure parameter blocks at (t_new[s], dt[s]) (mass: at t = 0,
// without a step) to the device, on the stream of the call that reads them.
// With kp, also the brick operator's folded parameters in both precisions.
int batch_params(dg_batch* b, const double* t_new, const double* dt, bool step, hipStream_t st,
                 const char* fn, bool kp = false) {
  const int n = int(b->subs.size());
  if (step) {
    if (!t_new || !dt) return fail(DG_EINVAL, std::string(fn) + ": null t_new or dt");
    for (int s = 0; s < n; ++s)
      if (!(dt[s] > 0)) return fail(DG_EINVAL, std::string(fn) + ": dt[" + std::to_string(s) + "] must be positive");
  }
  DG_HIP(hipEventSynchronize(b->staged));   // the previous upload has left the staging buffers
  for (int s = 0; s < n; ++s) {
    b->h_params[s] = make_params(b->subs[s], step ? t_new[s] : 0.0, step ? dt[s] : 0.0);
    if (kp) {
      b->h_kpf[s] = make_kp<float>(b->h_params[s]);
      b->h_kpd[s] = make_kp<double>(b->h_params[s]);
    }
  }
  DG_HIP(hipMemcpyAsync(b->d_params, b->h_params, size_t(n) * sizeof(DevParams), hipMemcpyHostToDevice, st));
  if (kp) {
    DG_HIP(hipMemcpyAsync(b->d_kpf, b->h_kpf, size_t(n) * sizeof(KP<float>), hipMemcpyHostToDevice, st));
    DG_HIP(hipMemcpyAsync(b->d_kpd, b->h_kpd, size_t(n) * sizeof(KP<double>), hipMemcpyHostToDevice, st));
  }
  DG_HIP(hipEventRecord(b->staged, st));
  return DG_OK;
}

int64_t batch_grid(const dg_batch* b) { return (b->ntiles + 7) / 8 * 8; }

// Launch shapes chosen by dg_batch_autotune, kept for the process by
// precision, operator and size class (the bit length of the voxel count);
// batches set up later in the same class start from them.
std::mutex g_shape_mu;
std::map<std::tuple<int, int, int>, dg_batch_shape> g_shape_cache;

int size_class(int64_t E) {
  int c = 0;
  while (E >>= 1) ++c;
  return c;
}

constexpr dg_batch_shape kDefaultShape{kTileVoxels, 0};
// The brick shape of the condensed tangent: work items of 4 x 4 x 4 voxels
// (inner faces evaluated once), the default of that operator.
constexpr dg_batch_shape kBrickShape{kBrickVox, 0};

constexpr dg_batch_shape default_shape(int op) { return op == DG_BOP_JVP_CONDENSED7 ? kBrickShape : kDefaultShape; }

template <typename S>
constexpr int prec_index() { return std::is_same<S, double>::value ? DG_F64 : DG_F32; }

template <int Mode>
constexpr int op_index() {
  return Mode == kResidual ? DG_BOP_RESIDUAL : Mode == kJvpFull ? DG_BOP_JVP_FULL9 : DG_BOP_JVP_CONDENSED7;
}

template <typename S, typename N, int Mode, int kLanes, bool kPersistent>
const void* q1_batch_symbol() {
  if constexpr (std::is_same<S, float>::value && Mode != kResidual)
    return reinterpret_cast<const void*>(&q1_batch_kernel_w2<S, N, Mode, kLanes, kPersistent>);
  else
    return reinterpret_cast<const void*>(&q1_batch_kernel<S, N, Mode, kLanes, kPersistent>);
}

// One launch of a batched residual or tangent in tiles of kLanes / 8
// voxels.  persistent > 0: that many workgroups per compute unit (at least
// 8 and at most one per work item, a multiple of 8), each striding over the
// work items; 0: one workgroup per work item.
template <typename S, typename N, int Mode, int kLanes>
void launch_q1_batch_lanes(const dg_batch* b, int persistent, const void* u, const void* v, const void* m,
                           void* out, hipStream_t st) {
  constexpr int ti = kLanes == 64 ? 0 : kLanes == 128 ? 1 : 2;
  static_assert(kTileChoices[ti] * 8 == kLanes, "tile size and workgroup size disagree");
  const int64_t nt = b->ntiles_by[ti];
  const int64_t nb = (nt + 7) / 8 * 8;
  int64_t grid = nb;
  if (persistent > 0) grid = std::min(nb, std::max<int64_t>(8, int64_t(persistent) * b->n_cu / 8 * 8));
  const dim3 g{unsigned(grid), 1, 1}, blk{unsigned(kLanes), 1, 1};
  const int64_t FS = b->E * 8;
  using K = void (*)(const S*, const S*, const S*, S*, const uint8_t*, const DevParams*, const BatchTile*, int64_t,
                     int64_t, int64_t);
  const K kern = reinterpret_cast<K>(const_cast<void*>(
      persistent > 0 ? q1_batch_symbol<S, N, Mode, kLanes, true>() : q1_batch_symbol<S, N, Mode, kLanes, false>()));
  hipLaunchKernelGGL(kern, g, blk, 0, st, static_cast<const S*>(u), static_cast<const S*>(v),
                     static_cast<const S*>(m), static_cast<S*>(out), b->d_phase, b->d_params, b->d_tiles_by[ti], nt,
                     FS, nb);
}

template <typename S, typename N, int Mode>
void launch_q1_batch_shape(const dg_batch* b, dg_batch_shape sh, const void* u, const void* v, const void* m,
                           void* out, hipStream_t st) {
  switch (sh.tile_voxels) {
    case 8: launch_q1_batch_lanes<S, N, Mode, 64>(b, sh.persistent, u, v, m, out, st); break;
    case 16: launch_q1_batch_lanes<S, N, Mode, 128>(b, sh.persistent, u, v, m, out, st); break;
    default: launch_q1_batch_lanes<S, N, Mode, 256>(b, sh.persistent, u, v, m, out, st); break;
  }
}

// Workgroups of tile_voxels * 8 lanes of the persistent kernel that one
// compute unit holds at once (0 if the runtime cannot tell).
template <typename S, typename N, int Mode>
int q1_batch_resident(int tile_voxels) {
  int n = 0;
  hipError_t e;
  switch (tile_voxels) {
    case 8:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, q1_batch_symbol<S, N, Mode, 64, true>(), 64, 0);
      break;
    case 16:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, q1_batch_symbol<S, N, Mode, 128, true>(), 128, 0);
      break;
    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, q1_batch_symbol<S, N, Mode, 256, true>(), 256, 0);
      break;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return n;
}

// Condensed tangent at the batch linearisation on bricks of 4 x 4 x 4
// voxels: one workgroup per brick of every structure, XCD-aware order.
// Needs the folded parameters of batch_params(..., kp = true).
template <typename S>
void launch_brick_batch(const dg_batch* b, const void* u, const void* v, void* out, hipStream_t st) {
  const int64_t nb = (b->nbricks + 7) / 8 * 8;
  const KP<S>* Ks;
  if constexpr (std::is_same<S, double>::value)
    Ks = b->d_kpd;
  else
    Ks = b->d_kpf;
  hipLaunchKernelGGL(q1_brick_jvp_batch_kernel<S>, dim3(unsigned(nb)), dim3(kBrickLanes), 0, st,
                     static_cast<const S*>(u), static_cast<const S*>(v), b->lin.as<const S>(), static_cast<S*>(out),
                     b->d_phase, Ks, b->d_bricks, b->nbricks, b->E * 8, nb);
}

template <typename S, typename N, int Mode>
void launch_q1_batch(const dg_batch* b, const void* u, const void* v, const void* m, void* out, hipStream_t st) {
  const dg_batch_shape sh = b->shape[prec_index<S>()][op_index<Mode>()];
  if (Mode == kJvpCondensed && sh.tile_voxels == kBrickShape.tile_voxels)
    launch_brick_batch<S>(b, u, v, out, st);
  else
    launch_q1_batch_shape<S, N, Mode>(b, sh, u, v, m, out, st);
}

template <typename S>
int batch_linearize(dg_batch* b, const S* u, hipStream_t st) {
  const int64_t FS = b->E * 8;
  hipError_t e = b->lin.ensure(size_t(14) * FS * sizeof(S));
  if (e != hipSuccess) return fail(DG_ENOMEM, std::string("batch linearisation storage: ") + hipGetErrorString(e));
  const int64_t nb = batch_grid(b);
  hipLaunchKernelGGL(solid_tangent_batch_kernel<S>, dim3(unsigned(nb)), dim3(256), 0, st, u, b->lin.as<S>(),
                     b->d_phase, b->d_params, b->d_tiles, b->ntiles, FS, nb);
  DG_HIP(hipGetLastError());
  b->lin_prec = std::is_same<S, double>::value ? DG_F64 : DG_F32;
  return DG_OK;
}

template <typename S>
int batch_blocks(dg_batch* b, const S* u, hipStream_t st) {
  if (int s = batch_linearize<S>(b, u, st)) return s;
  const size_t need = size_t(b->E) * 56 * 56 * sizeof(S);
  hipError_t e = b->blocks.ensure(need);
  if (e != hipSuccess) return fail(DG_ENOMEM, std::string("batch block storage: ") + hipGetErrorString(e));
  e = b->status.ensure(sizeof(int));
  if (e != hipSuccess) return fail(DG_ENOMEM, "batch status allocation");
  DG_HIP(hipMemsetAsync(b->status.p, 0, sizeof(int), st));
  const int64_t nb = batch_grid(b);
  hipLaunchKernelGGL((q1_block_batch_kernel<S, kJvpCondensed>), dim3(unsigned(nb)), dim3(256), 0, st, u,
                     b->lin.as<S>(), b->blocks.as<S>(), b->d_phase, b->d_params, b->d_tiles, b->ntiles,
                     b->E * 8, nb);
  hipLaunchKernelGGL((invert_blocks_kernel<S, 56>), dim3(unsigned((b->E + 3) / 4)), dim3(256), 0, st,
                     b->blocks.as<S>(), b->E, b->status.as<int>());
  DG_HIP(hipGetLastError());
  int h_status = 0;
  DG_HIP(hipMemcpyAsync(&h_status, b->status.p, sizeof(int), hipMemcpyDeviceToHost, st));
  DG_HIP(hipStreamSynchronize(st));
  b->blocks_prec = std::is_same<S, double>::value ? DG_F64 : DG_F32;
  if (h_status) return fail(DG_ENAN, "dg_batch_blockjacobi_setup: singular or non-finite element block");
  return DG_OK;
}

}  // namespace

namespace {

// Means, sums and cell voltage from the kNumSums node sums of outputs_kernel.
void outputs_from_sums(const dg_ctx* ctx, const double* acc, double* U_cell, double* means, double* sums) {
  const double nodes = double(ctx->Ne) * ctx->np;
  if (means)
    for (int f = 0; f < 10; ++f) means[f] = acc[f] / nodes;
  if (sums)
    for (int j = 0; j < 4; ++j) sums[j] = acc[10 + j];
  if (U_cell) *U_cell = acc[14] / (double(ctx->mesh.ny) * ctx->mesh.nz * 4.0);
}

}  // namespace

// STREAM triad out = a + s b over n2 pairs of doubles (16-byte accesses,
// grid-stride, two pairs per lane per pass so that each wave keeps four
// loads in flight).
__global__ void __launch_bounds__(256)
triad_kernel(double2* __restrict__ out, const double2* __restrict__ a, const double2* __restrict__ b, double s,
             int64_t n2) {
  const int64_t stride = int64_t(gridDim.x) * 256;
  int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  for (; i + stride < n2; i += 2 * stride) {
    const double2 a0 = a[i], b0 = b[i], a1 = a[i + stride], b1 = b[i + stride];
    out[i] = make_double2(a0.x + s * b0.x, a0.y + s * b0.y);
    out[i + stride] = make_double2(a1.x + s * b1.x, a1.y + s * b1.y);
  }
  if (i < n2) {
    const double2 a0 = a[i], b0 = b[i];
    out[i] = make_double2(a0.x + s * b0.x, a0.y + s * b0.y);
  }
}

extern "C" {

void dg_params_default(dg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->T = 298.15;
  for (int i = 0; i < 7; ++i) p->D0[i] = kD0paper[i];
  for (int k = 0; k < 6; ++k) p->kE[k] = kKEpaper[k];
  p->f_C = 0.1;
  p->j_el = -1.0;
  p->eps_struct = -1.0;
  p->sigma = -1.0;
  p->c_min = 1e-20;
  p->epsL_min = 1e-6;
  p->use_TH = 1;
}

}  // extern "C"

namespace {

// Checked host side of a context: mesh, phase map and parameters, and what
// derives from them (Tab. InitialState, Eq. 57 localisation, App. C
// current).  No device work.
int make_context(const dg_mesh* mesh, const uint8_t* phase, const dg_params* params, const char* fn,
                 dg_ctx** out) {
  if (!mesh || !phase || !params || !out) return fail(DG_EINVAL, std::string(fn) + ": null argument");
  *out = nullptr;
  if (mesh->nx <= 0 || mesh->ny <= 0 || mesh->nz <= 0 || !(mesh->h > 0))
    return fail(DG_EINVAL, std::string(fn) + ": mesh sizes and h must be positive");
  if (mesh->order != 0 && mesh->order != 1 && mesh->order != 3)
    return fail(DG_EINVAL, std::string(fn) + ": order " + std::to_string(mesh->order) + " is not one of 0, 1, 3");
  if (!(params->T > 0)) return fail(DG_EINVAL, std::string(fn) + ": temperature must be positive");
  const int64_t Ne = int64_t(mesh->nx) * mesh->ny * mesh->nz;
  int64_t n_struct = 0;
  for (int64_t e = 0; e < Ne; ++e) {
    if (phase[e] > 1) return fail(DG_EINVAL, std::string(fn) + ": phase values must be 0 or 1");
    n_struct += phase[e];
  }
  dg_ctx* c = new dg_ctx;
  c->mesh = *mesh;
  c->params = *params;
  c->Ne = Ne;
  const int K = mesh->order + 1;
  c->np = K * K * K;
  c->eq = equilibrium(params->T);
  const double pore_frac = 1.0 - double(n_struct) / double(Ne);
  c->eps_struct = params->eps_struct > 0 ? params->eps_struct : 1.0 - pore_frac;
  c->sigma = params->sigma > 0 ? params->sigma : (mesh->order == 0 ? 1.0 : double(K * K));
  const double inv = c->eps_struct > 0 ? 1.0 / c->eps_struct : 0.0;
  PhaseTable& t = c->phase_tab;
  std::memset(&t, 0, sizeof(t));
  t.epsCBD[1] = (kXcathode - kXsulfur) * inv;
  t.aV0[1] = kAV0 * inv;
  t.epsS8init[1] = kEpsS8init * inv;
  t.epsLi2Sinit[1] = kEpsLi2Sinit * inv;
  t.s8ref[1] = 1.2 * t.epsS8init[1];
  t.pass[1] = kPassA * std::exp(-kPassBh * params->f_C) * inv;
  t.react[1] = 1.0;
  if (params->j_el >= 0) {
    c->j_el = params->j_el;
  } else {
    // App. C: j_el = f_C c_theo m_A, c_theo = 16 F / M_S8, m_A = rho_S8 *
    // (initial S8 volume) / (separator area)
    const double h = mesh->h;
    const double vol = double(n_struct) * t.epsS8init[1] * h * h * h;
    const double area = double(mesh->ny) * mesh->nz * h * h;
    const double c_theo = 16.0 * kFaraday / kMolar[0];
    c->j_el = params->f_C / 3600.0 * c_theo * kRho[0] * vol / area;
  }
  *out = c;
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_setup(const dg_mesh* mesh, const uint8_t* phase, const dg_params* params, dg_ctx** out) {
  try {
    dg_ctx* c = nullptr;
    if (int s = make_context(mesh, phase, params, "dg_setup", &c)) return s;
    double* scr = nullptr;
    if (int s = device_scratch(&scr)) {
      delete c;
      return s;
    }
    hipError_t err = c->phase.ensure(size_t(c->Ne));
    if (err != hipSuccess) {
      delete c;
      return fail(DG_ENOMEM, std::string("dg_setup: hipMalloc: ") + hipGetErrorString(err));
    }
    c->d_phase = c->phase.as<uint8_t>();
    err = hipMemcpy(c->d_phase, phase, size_t(c->Ne), hipMemcpyHostToDevice);
    if (err != hipSuccess) {
      c->phase.release();
      delete c;
      return fail(DG_EHIP, std::string("dg_setup: hipMemcpy: ") + hipGetErrorString(err));
    }
    *out = c;
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_setup: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_setup: unexpected exception");
  }
}

int dg_workspace_bytes(const dg_mesh* mesh, const dg_params* params, const dg_solver_opts* opts, int32_t features,
                       size_t* bytes) {
  try {
    if (!mesh || !params || !bytes) return fail(DG_EINVAL, "dg_workspace_bytes: null argument");
    if (features & ~int32_t(DG_WS_ALL)) return fail(DG_EINVAL, "dg_workspace_bytes: unknown feature bits");
    *bytes = 0;
    dg_solver_opts o;
    if (int s = normalize_opts(opts, o, "dg_workspace_bytes")) return s;
    if ((features & DG_WS_MG) && o.mg_levels < 2)
      return fail(DG_EINVAL, "dg_workspace_bytes: DG_WS_MG needs opts->mg_levels >= 2");
    // a host-only context of the mesh (an all-structure map: the sizes do
    // not depend on the phases)
    const int64_t Ne = int64_t(mesh->nx) * mesh->ny * mesh->nz;
    if (mesh->nx <= 0 || mesh->ny <= 0 || mesh->nz <= 0) return fail(DG_EINVAL, "dg_workspace_bytes: mesh sizes");
    std::vector<uint8_t> ones(size_t(Ne), 1);
    dg_ctx* c = nullptr;
    if (int s = make_context(mesh, ones.data(), params, "dg_workspace_bytes", &c)) return s;
    const int32_t allowed = c->mesh.order == 1   ? int32_t(DG_WS_ALL)
                            : c->mesh.order == 3 ? int32_t(DG_WS_OPERATORS | DG_WS_BLOCKS)
                                                 : int32_t(DG_WS_OPERATORS);
    if (features & ~allowed) {
      delete c;
      return fail(DG_EUNSUPPORTED, "dg_workspace_bytes: order 0 provides the operators only (DG_WS_OPERATORS), order 3 "
                                   "the operators and blocks (DG_WS_BLOCKS)");
    }
    bool need_rs = false;
    int64_t nc = 0;
    size_t total = 0;
    for (const auto& pr : plan_workspace(c, o, features, need_rs, nc)) total = Arena::aligned(total) + pr.second;
    delete c;
    if (need_rs) {
      rocblas_handle h = nullptr;
      if (rocblas_create_handle(&h) != rocblas_status_success)
        return fail(DG_EHIP, "dg_workspace_bytes: rocblas_create_handle failed");
      size_t rs = 0;
      const bool ok = rocsolver_scratch_bytes(h, nc, rs);
      (void)rocblas_destroy_handle(h);
      if (!ok) return fail(DG_EHIP, "dg_workspace_bytes: rocSOLVER scratch size query failed");
      total = Arena::aligned(total) + (rs > 0 ? rs : 1);
    }
    *bytes = Arena::aligned(total);
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_workspace_bytes: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_workspace_bytes: unexpected exception");
  }
}

int dg_setup_ws(const dg_mesh* mesh, const uint8_t* phase, const dg_params* params, const dg_solver_opts* opts,
                int32_t features, void* workspace, size_t ws_bytes, dg_stream stream, dg_ctx** out) {
  try {
    if (!workspace) return fail(DG_EINVAL, "dg_setup_ws: null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(DG_EINVAL, "dg_setup_ws: the workspace must be 256-byte aligned");
    if (features & ~int32_t(DG_WS_ALL)) return fail(DG_EINVAL, "dg_setup_ws: unknown feature bits");
    dg_solver_opts o;
    if (int s = normalize_opts(opts, o, "dg_setup_ws")) return s;
    if ((features & DG_WS_MG) && o.mg_levels < 2)
      return fail(DG_EINVAL, "dg_setup_ws: DG_WS_MG needs opts->mg_levels >= 2");
    dg_ctx* c = nullptr;
    if (int s = make_context(mesh, phase, params, "dg_setup_ws", &c)) return s;
    const int32_t allowed = c->mesh.order == 1   ? int32_t(DG_WS_ALL)
                            : c->mesh.order == 3 ? int32_t(DG_WS_OPERATORS | DG_WS_BLOCKS)
                                                 : int32_t(DG_WS_OPERATORS);
    if (features & ~allowed) {
      delete c;
      return fail(DG_EUNSUPPORTED, "dg_setup_ws: order 0 provides the operators only (DG_WS_OPERATORS), order 3 "
                                   "the operators and blocks (DG_WS_BLOCKS)");
    }
    double* scr = nullptr;
    if (int s = device_scratch(&scr)) {
      delete c;
      return s;
    }
    c->owns_memory = false;
    c->arena.base = static_cast<unsigned char*>(workspace);
    c->arena.size = ws_bytes;
    c->for_each_buf([c](DevBuf& b) { b.arena = &c->arena; });
    bool need_rs = false;
    int64_t nc = 0;
    for (const auto& pr : plan_workspace(c, o, features, need_rs, nc)) {
      if (pr.first->ensure(pr.second) != hipSuccess) {
        const int s = fail_mem(c, "dg_setup_ws", pr.second);
        delete c;
        return s;
      }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (need_rs) {
      if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        delete c;
        return fail(DG_EHIP, "dg_setup_ws: rocblas_create_handle failed");
      }
      size_t rs = 0;
      int s = rocsolver_scratch_bytes(c->blas, nc, rs) ? give_blas_scratch(c, rs)
                                                       : fail(DG_EHIP, "dg_setup_ws: rocSOLVER scratch size query failed");
      if (s) {
        (void)rocblas_destroy_handle(c->blas);
        delete c;
        return s;
      }
    }
    if (features & (DG_WS_STEP | DG_WS_NAIVE | DG_WS_H211B)) {
      if (int s = gmres_host_state(c)) {
        if (c->blas) (void)rocblas_destroy_handle(c->blas);
        delete c;
        return s;
      }
    }
    c->d_phase = c->phase.as<uint8_t>();
    hipError_t err = hipMemcpyAsync(c->d_phase, phase, size_t(c->Ne), hipMemcpyHostToDevice, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);    // the host phase map may go after return
    if (err != hipSuccess) {
      if (c->blas) (void)rocblas_destroy_handle(c->blas);
      delete c;
      return fail(DG_EHIP, std::string("dg_setup_ws: hipMemcpyAsync: ") + hipGetErrorString(err));
    }
    *out = c;
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_setup_ws: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_setup_ws: unexpected exception");
  }
}

int dg_destroy(dg_ctx* ctx) {
  if (!ctx) return DG_OK;
  // buffers carved from a caller's workspace are the caller's: release()
  // only forgets them
  ctx->for_each_buf([](DevBuf& b) { b.release(); });
  if (ctx->blas) (void)rocblas_destroy_handle(ctx->blas);
  for (hipEvent_t ev : ctx->gm_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->gm_flags) (void)hipHostFree(ctx->gm_flags);
  delete ctx;
  return DG_OK;
}

int dg_info(const dg_ctx* ctx, double* V, double* c0, double* U0, double* j_el, double* eps_struct) {
  if (int s = check_ctx(ctx)) return s;
  if (V) *V = ctx->eq.dphi0;
  if (c0)
    for (int i = 0; i < 6; ++i) c0[i] = ctx->eq.c[i];
  if (U0)
    for (int i = 0; i < 6; ++i) U0[i] = ctx->eq.U0[i];
  if (j_el) *j_el = ctx->j_el;
  if (eps_struct) *eps_struct = ctx->eps_struct;
  return DG_OK;
}

int dg_mass(dg_ctx* ctx, dg_prec prec, const void* u, void* m, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!u || !m) return fail(DG_EINVAL, "dg_mass: null array");
  const DevParams P = make_params(ctx, 0.0, 0.0);
  const int64_t n = ctx->Ne * ctx->np;
  const dim3 grid{unsigned((n + 255) / 256), 1, 1}, block{256, 1, 1};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prec == DG_F64)
    hipLaunchKernelGGL(mass_kernel<double>, grid, block, 0, st, static_cast<const double*>(u),
                       static_cast<double*>(m), ctx->d_phase, P, ctx->np);
  else if (prec == DG_F32)
    hipLaunchKernelGGL(mass_kernel<float>, grid, block, 0, st, static_cast<const float*>(u),
                       static_cast<float*>(m), ctx->d_phase, P, ctx->np);
  else
    return fail(DG_EINVAL, "dg_mass: bad precision");
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_residual(dg_ctx* ctx, dg_prec prec, const void* u, const void* m_old, double t_new,
                double dt, void* r, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!u || !m_old || !r) return fail(DG_EINVAL, "dg_residual: null array");
  if (!(dt > 0)) return fail(DG_EINVAL, "dg_residual: dt must be positive");
  const DevParams P = make_params(ctx, t_new, dt);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prec == DG_F64)
    launch_q1<double, double, kResidual>(ctx, P, u, nullptr, m_old, r, st);
  else if (prec == DG_F32)
    launch_q1<float, float, kResidual>(ctx, P, u, nullptr, m_old, r, st);
  else
    return fail(DG_EINVAL, "dg_residual: bad precision");
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_jvp(dg_ctx* ctx, dg_prec prec, dg_jvp_mode mode, const void* u, const void* v,
           double t_new, double dt, void* jv, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!u || !v || !jv) return fail(DG_EINVAL, "dg_jvp: null array");
  if (!(dt > 0)) return fail(DG_EINVAL, "dg_jvp: dt must be positive");
  const DevParams P = make_params(ctx, t_new, dt);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (mode == DG_JVP_FULL9) {
    if (prec == DG_F64)
      launch_q1<double, Dual<double>, kJvpFull>(ctx, P, u, v, nullptr, jv, st);
    else if (prec == DG_F32)
      launch_q1<float, Dual<float>, kJvpFull>(ctx, P, u, v, nullptr, jv, st);
    else
      return fail(DG_EINVAL, "dg_jvp: bad precision");
  } else if (mode == DG_JVP_CONDENSED7 || mode == DG_JVP_LINEARIZED7) {
    if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_jvp: bad precision");
    if (mode == DG_JVP_CONDENSED7) {
      const int s = prec == DG_F64 ? linearize<double>(ctx, P, static_cast<const double*>(u), st)
                                   : linearize<float>(ctx, P, static_cast<const float*>(u), st);
      if (s) return s;
    } else if (ctx->lin_prec != int(prec)) {
      return fail(DG_ESTATE, "dg_jvp: no linearisation of this precision (dg_linearize)");
    }
    if (ctx->np != 8) {
      if (prec == DG_F64)
        launch_q1<double, Dual<double>, kJvpCondensed>(ctx, P, u, v, ctx->lin.p, jv, st);
      else
        launch_q1<float, Dual<float>, kJvpCondensed>(ctx, P, u, v, ctx->lin.p, jv, st);
    } else if (prec == DG_F64) {
      launch_brick_jvp<double>(ctx, P, u, v, ctx->lin.p, jv, st);
    } else {
      launch_brick_jvp<float>(ctx, P, u, v, ctx->lin.p, jv, st);
    }
  } else {
    return fail(DG_EINVAL, "dg_jvp: bad mode");
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}


int dg_linearize(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!u) return fail(DG_EINVAL, "dg_linearize: null array");
  if (!(dt > 0)) return fail(DG_EINVAL, "dg_linearize: dt must be positive");
  const DevParams P = make_params(ctx, t_new, dt);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prec == DG_F64) return linearize<double>(ctx, P, static_cast<const double*>(u), st);
  if (prec == DG_F32) return linearize<float>(ctx, P, static_cast<const float*>(u), st);
  return fail(DG_EINVAL, "dg_linearize: bad precision");
}

constexpr int kNB = 56;   // condensed Q1 block size: 7 fields x 8 nodes

int dg_blockjacobi_setup(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt,
                         dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (int s = check_blocks_order(ctx, "dg_blockjacobi_setup")) return s;
  if (!u) return fail(DG_EINVAL, "dg_blockjacobi_setup: null array");
  if (!(dt > 0)) return fail(DG_EINVAL, "dg_blockjacobi_setup: dt must be positive");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_blockjacobi_setup: bad precision");
  if (ctx->np == 64) {
    const DevParams P = make_params(ctx, t_new, dt);
    hipStream_t st = static_cast<hipStream_t>(stream);
    ctx->blocks_prec = -1;
    return prec == DG_F64 ? blocks_setup_q3<double>(ctx, P, static_cast<const double*>(u), st)
                          : blocks_setup_q3<float>(ctx, P, static_cast<const float*>(u), st);
  }
  const size_t esz = prec == DG_F64 ? sizeof(double) : sizeof(float);
  const size_t need = size_t(ctx->Ne) * kNB * kNB * esz;
  if (ctx->blocks.ensure(need) != hipSuccess) return fail_mem(ctx, "dg_blockjacobi_setup: block storage", need);
  if (ctx->status.ensure(sizeof(int)) != hipSuccess) return fail_mem(ctx, "dg_blockjacobi_setup: status flag", 4);
  hipStream_t st = static_cast<hipStream_t>(stream);
  DG_HIP(hipMemsetAsync(ctx->status.p, 0, sizeof(int), st));
  const DevParams P = make_params(ctx, t_new, dt);
  int64_t nb = (ctx->Ne * 8 + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  const dim3 grid_w{unsigned((ctx->Ne + 3) / 4), 1, 1};
  if (int s = prec == DG_F64 ? linearize<double>(ctx, P, static_cast<const double*>(u), st)
                             : linearize<float>(ctx, P, static_cast<const float*>(u), st))
    return s;
  if (prec == DG_F64) {
    hipLaunchKernelGGL((q1_block_kernel<double, kJvpCondensed>), grid, block, 0, st,
                       static_cast<const double*>(u), ctx->lin.as<double>(), ctx->blocks.as<double>(),
                       ctx->d_phase, P, nb);
    hipLaunchKernelGGL((invert_blocks_kernel<double, kNB>), grid_w, block, 0, st,
                       ctx->blocks.as<double>(), ctx->Ne, ctx->status.as<int>());
  } else {
    hipLaunchKernelGGL((q1_block_kernel<float, kJvpCondensed>), grid, block, 0, st,
                       static_cast<const float*>(u), ctx->lin.as<float>(), ctx->blocks.as<float>(),
                       ctx->d_phase, P, nb);
    hipLaunchKernelGGL((invert_blocks_kernel<float, kNB>), grid_w, block, 0, st,
                       ctx->blocks.as<float>(), ctx->Ne, ctx->status.as<int>());
  }
  DG_HIP(hipGetLastError());
  int h_status = 0;
  DG_HIP(hipMemcpyAsync(&h_status, ctx->status.as<int>(), sizeof(int), hipMemcpyDeviceToHost, st));
  DG_HIP(hipStreamSynchronize(st));
  ctx->blocks_prec = int(prec);
  ctx->bh_valid = false;
  if (h_status) return fail(DG_ENAN, "dg_blockjacobi_setup: singular or non-finite element block");
  return DG_OK;
}

int dg_blockjacobi_apply(dg_ctx* ctx, dg_prec prec, const void* x, void* y, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (int s = check_blocks_order(ctx, "dg_blockjacobi_apply")) return s;
  if (!x || !y) return fail(DG_EINVAL, "dg_blockjacobi_apply: null array");
  if (ctx->blocks_prec < 0) return fail(DG_ESTATE, "dg_blockjacobi_apply: no setup yet");
  if (int(prec) != ctx->blocks_prec)
    return fail(DG_EINVAL, "dg_blockjacobi_apply: precision differs from the setup");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->np == 64) {
    const dim3 g{unsigned(ctx->Ne), 1, 1}, b{512, 1, 1};
    if (prec == DG_F64)
      hipLaunchKernelGGL(apply_q3_kernel<double>, g, b, 0, st, ctx->blocks.as<const double>(),
                         ctx->qpiv.as<const int16_t>(), static_cast<const double*>(x), static_cast<double*>(y),
                         ctx->Ne);
    else
      hipLaunchKernelGGL(apply_q3_kernel<float>, g, b, 0, st, ctx->blocks.as<const float>(),
                         ctx->qpiv.as<const int16_t>(), static_cast<const float*>(x), static_cast<float*>(y),
                         ctx->Ne);
    DG_HIP(hipGetLastError());
    return DG_OK;
  }
  const dim3 grid{unsigned((ctx->Ne + 3) / 4), 1, 1}, block{256, 1, 1};
  if (prec == DG_F64)
    hipLaunchKernelGGL((apply_blocks_kernel<double, 7>), grid, block, 0, st,
                       ctx->blocks.as<const double>(), static_cast<const double*>(x),
                       static_cast<double*>(y), ctx->Ne);
  else
    hipLaunchKernelGGL((apply_blocks_kernel<float, 7>), grid, block, 0, st,
                       ctx->blocks.as<const float>(), static_cast<const float*>(x),
                       static_cast<float*>(y), ctx->Ne);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_blockjacobi_apply_bf16(dg_ctx* ctx, const void* x, void* y, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (int s = check_q1(ctx, "dg_blockjacobi_apply_bf16")) return s;
  if (!x || !y) return fail(DG_EINVAL, "dg_blockjacobi_apply_bf16: null array");
  if (!ctx->bh_valid && ctx->blocks_prec != DG_F32)
    return fail(DG_ESTATE, "dg_blockjacobi_apply_bf16: no FP32 setup");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!ctx->bh_valid) {
    if (ctx->bh.ensure(size_t(ctx->Ne) * kNB * kNB * 2) != hipSuccess)
      return fail_mem(ctx, "dg_blockjacobi_apply_bf16", size_t(ctx->Ne) * kNB * kNB * 2);
    hipLaunchKernelGGL((blocks_to_bf16_kernel<kNB>), dim3(8192), dim3(256), 0, st,
                       ctx->blocks.as<const float>(), ctx->bh.as<uint16_t>(), ctx->Ne);
    DG_HIP(hipGetLastError());
    ctx->bh_valid = true;
  }
  const dim3 grid{unsigned((ctx->Ne + 3) / 4), 1, 1}, block{256, 1, 1};
  hipLaunchKernelGGL((apply_blocks_bf16_kernel<7>), grid, block, 0, st, ctx->bh.as<const uint16_t>(),
                     static_cast<const float*>(x), static_cast<float*>(y), ctx->Ne);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_blockjacobi_info(const dg_ctx* ctx, int32_t* prec, int32_t* block_size) {
  if (int s = check_ctx(ctx)) return s;
  if (!prec || !block_size) return fail(DG_EINVAL, "dg_blockjacobi_info: null argument");
  if (ctx->blocks_prec < 0) return fail(DG_ESTATE, "dg_blockjacobi_info: no inverses stored");
  *prec = ctx->blocks_prec;
  *block_size = condensed_block_size(ctx);
  return DG_OK;
}

int dg_blockjacobi_export(dg_ctx* ctx, void* out, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!out) return fail(DG_EINVAL, "dg_blockjacobi_export: null array");
  if (ctx->blocks_prec < 0) return fail(DG_ESTATE, "dg_blockjacobi_export: no setup yet");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->np == 64) {
    if (ctx->blocks_prec == DG_F64)
      hipLaunchKernelGGL(export_q3_kernel<double>, dim3(unsigned(ctx->Ne)), dim3(512), 0, st,
                         ctx->blocks.as<const double>(), ctx->qpiv.as<const int16_t>(), static_cast<double*>(out));
    else
      hipLaunchKernelGGL(export_q3_kernel<float>, dim3(unsigned(ctx->Ne)), dim3(512), 0, st,
                         ctx->blocks.as<const float>(), ctx->qpiv.as<const int16_t>(), static_cast<float*>(out));
    DG_HIP(hipGetLastError());
    return DG_OK;
  }
  if (ctx->blocks_prec == DG_F64)
    hipLaunchKernelGGL((export_blocks_kernel<double, kNB>), dim3(4096), dim3(256), 0, st,
                       ctx->blocks.as<const double>(), static_cast<double*>(out), ctx->Ne);
  else
    hipLaunchKernelGGL((export_blocks_kernel<float, kNB>), dim3(4096), dim3(256), 0, st,
                       ctx->blocks.as<const float>(), static_cast<float*>(out), ctx->Ne);
  DG_HIP(hipGetLastError());
  return DG_OK;
}


// Multilevel coarse correction through the C ABI (multigrid.hpp), with
// unit basis scales: dg_mg_setup linearises at u and builds the hierarchy,
// dg_mg_apply returns Z V(Z^T r).
int dg_mg_setup(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt, const dg_solver_opts* opts,
                dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (int s = check_q1(ctx, "dg_mg_setup")) return s;
    if (!u) return fail(DG_EINVAL, "dg_mg_setup: null array");
    if (!(dt > 0)) return fail(DG_EINVAL, "dg_mg_setup: dt must be positive");
    if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_mg_setup: bad precision");
    dg_solver_opts o;
    if (int s = normalize_opts(opts, o, "dg_mg_setup")) return s;
    o = resolve_opts(ctx->mesh, o);
    if (o.mg_levels < 2) return fail(DG_EINVAL, "dg_mg_setup: mg_levels must be in 2..8");
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto& M = ctx->mg;
    M.prec = -1;
    const AggGrid G = coarse_grid(ctx->mesh, o);
    MgGrid g[kMgMaxLevels];
    mg_grids(G, o.mg_levels, g);
    const int64_t nc = 8 * g[o.mg_levels - 1].na;
    if (nc > 8192) return fail(DG_EINVAL, "dg_mg_setup: the last level has more than 8192 unknowns (add levels)");
    const int64_t FS = ctx->Ne * ctx->np;
    const size_t sS = prec == DG_F64 ? 8 : 4;
    for (const auto& pr : mg_buffers(ctx, o.mg_levels, g))
      if (pr.first->ensure(pr.second) != hipSuccess) return fail_mem(ctx, "dg_mg_setup: levels", pr.second);
    for (const auto& pr : coarse_buffers(ctx, nc))
      if (pr.first->ensure(pr.second) != hipSuccess) return fail_mem(ctx, "dg_mg_setup: last level", pr.second);
    for (DevBuf* d : {&M.ones, &M.pv, &M.pjv})
      if (d->ensure(size_t(7) * FS * sS) != hipSuccess) return fail_mem(ctx, "dg_mg_setup: probe vectors", 7 * FS * sS);
    if (!ctx->blas && rocblas_create_handle(&ctx->blas) != rocblas_status_success)
      return fail(DG_EHIP, "rocblas_create_handle failed");
    if (rocblas_set_stream(ctx->blas, st) != rocblas_status_success) return fail(DG_EHIP, "rocblas_set_stream failed");
    if (!ctx->owns_memory && ctx->blasws.bytes == 0) {
      size_t need = 0;
      if (!rocsolver_scratch_bytes(ctx->blas, nc, need))
        return fail(DG_EHIP, "dg_mg_setup: rocSOLVER scratch size query failed");
      if (int s = give_blas_scratch(ctx, need)) return s;
    }
    M.levels = o.mg_levels;
    M.nu = o.mg_sweeps;
    M.omega = o.mg_omega;
    M.G = G;
    for (int l = 0; l < M.levels; ++l) M.g[l] = g[l];
    const DevParams P = make_params(ctx, t_new, dt);
    const dim3 blk{256, 1, 1};
    int s = DG_OK;
    if (prec == DG_F64) {
      hipLaunchKernelGGL(mg_fill_kernel<double>, grid1(7 * FS), blk, 0, st, M.ones.as<double>(), 7 * FS, 1.0);
      s = linearize<double>(ctx, P, static_cast<const double*>(u), st);
      if (!s)
        s = mg_build<double>(ctx, P, static_cast<const double*>(u), M.ones.as<const double>(), M.pv.as<double>(),
                             M.pjv.as<double>(), kAllFields, st);
    } else {
      hipLaunchKernelGGL(mg_fill_kernel<float>, grid1(7 * FS), blk, 0, st, M.ones.as<float>(), 7 * FS, 1.0f);
      s = linearize<float>(ctx, P, static_cast<const float*>(u), st);
      if (!s)
        s = mg_build<float>(ctx, P, static_cast<const float*>(u), M.ones.as<const float>(), M.pv.as<float>(),
                            M.pjv.as<float>(), kAllFields, st);
    }
    if (s) return fail(s, std::string("dg_mg_setup: ") + g_last_error);
    DG_HIP(hipStreamSynchronize(st));
    M.prec = int(prec);
    return DG_OK;
  } catch (...) {
    return fail(DG_EINVAL, "dg_mg_setup: unexpected exception");
  }
}

int dg_mg_export(dg_ctx* ctx, int32_t level, double* out, int64_t n, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!out) return fail(DG_EINVAL, "dg_mg_export: null array");
  if (ctx->mg.prec < 0) return fail(DG_ESTATE, "dg_mg_export: no dg_mg_setup hierarchy is current");
  if (level < 1 || level > ctx->mg.levels) return fail(DG_EINVAL, "dg_mg_export: no such level");
  const int64_t need = 343 * ctx->mg.g[level - 1].na;
  if (n < need) return fail(DG_EINVAL, "dg_mg_export: out holds fewer than 343 x (aggregates of the level) entries");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(mg_export_kernel, grid1(need), dim3(256), 0, st, ctx->mg.E[level - 1].as<const double>(),
                     ctx->mg.g[level - 1], out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_mg_apply(dg_ctx* ctx, dg_prec prec, const void* r, void* out, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!r || !out) return fail(DG_EINVAL, "dg_mg_apply: null array");
  if (ctx->mg.prec < 0) return fail(DG_ESTATE, "dg_mg_apply: no dg_mg_setup hierarchy is current");
  if (int(prec) != ctx->mg.prec) return fail(DG_EINVAL, "dg_mg_apply: precision differs from the setup");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto& M = ctx->mg;
  const int64_t FS = ctx->Ne * ctx->np, n7 = 7 * FS;
  const dim3 blk{256, 1, 1}, gagg{unsigned(M.G.na), 1, 1};
  if (prec == DG_F64) {
    hipLaunchKernelGGL(mg_restrict_fine_kernel<double>, gagg, blk, 0, st, M.ones.as<const double>(),
                       static_cast<const double*>(r), M.G, FS, M.b[0].as<double>());
    const double* y = mg_vcycle(ctx, st);
    hipLaunchKernelGGL(mg_fill_kernel<double>, grid1(n7), blk, 0, st, static_cast<double*>(out), n7, 0.0);
    hipLaunchKernelGGL(mg_prolong_fine_kernel<double>, grid1(FS), blk, 0, st, M.ones.as<const double>(), y, M.G, FS,
                       static_cast<double*>(out), static_cast<const double*>(nullptr));
  } else {
    hipLaunchKernelGGL(mg_restrict_fine_kernel<float>, gagg, blk, 0, st, M.ones.as<const float>(),
                       static_cast<const float*>(r), M.G, FS, M.b[0].as<double>());
    const double* y = mg_vcycle(ctx, st);
    hipLaunchKernelGGL(mg_fill_kernel<float>, grid1(n7), blk, 0, st, static_cast<float*>(out), n7, 0.0f);
    hipLaunchKernelGGL(mg_prolong_fine_kernel<float>, grid1(FS), blk, 0, st, M.ones.as<const float>(), y, M.G, FS,
                       static_cast<float*>(out), static_cast<const float*>(nullptr));
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

void dg_solver_opts_default(dg_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->inner_prec = DG_F32;
  o->gmres_restart = 30;
  o->gmres_maxit = 1500;
  o->newton_maxit = 60;
  o->gmres_rtol = 1e-4;
  o->gmres_rtol_final = 1e-11;
  o->newton_tol = 1e-11;
  o->coarse = 0;           // 0: the aggregation coarse space (3)
  o->block_bf16 = 1;       // FP32 inner solves stream bfloat16 block inverses
  o->verbose = 0;
  o->coarse_every = 3;     // aggregation coarse operator rebuilt every third iterate
  o->mg_levels = -1;       // multilevel cycle where the exact two-level space would need coarse aggregates
  o->mg_sweeps = 3;
  o->mg_omega = 0.7;
  o->block_reuse = 1.0;    // element blocks kept while updates change no unknown by more than 100%
}

int dg_step(dg_ctx* ctx, double t_n, double dt, void* u, const dg_solver_opts* opts,
            dg_step_report* report, dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (!u) return fail(DG_EINVAL, "dg_step: null state");
    if (int s = check_q1(ctx, "dg_step")) return s;
    if (!(dt > 0)) return fail(DG_EINVAL, "dg_step: dt must be positive");
    dg_solver_opts o;
    if (int s = normalize_opts(opts, o, "dg_step")) return s;
    if (report) std::memset(report, 0, sizeof(*report));
    return solve_once(ctx, t_n, dt, static_cast<double*>(u), o, report, static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_step: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_step: unexpected exception");
  }
}

int dg_initial_state(dg_ctx* ctx, double t0, void* u, const dg_solver_opts* opts,
                     dg_step_report* report, dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (!u) return fail(DG_EINVAL, "dg_initial_state: null state");
    if (int s = check_q1(ctx, "dg_initial_state")) return s;
    dg_solver_opts o;
    if (int s = normalize_opts(opts, o, "dg_initial_state")) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (report) std::memset(report, 0, sizeof(*report));
    const int64_t FS = ctx->Ne * ctx->np;
    Conc6 c0{};
    for (int f = 0; f < 6; ++f) c0.c[f] = ctx->eq.c[f];
    const PhaseTable& pt = ctx->phase_tab;
    hipLaunchKernelGGL(uniform_state_kernel, grid1(FS), dim3(256), 0, st, static_cast<double*>(u),
                       ctx->d_phase, FS, ctx->np, c0, pt.epsS8init[0], pt.epsS8init[1], pt.epsLi2Sinit[0],
                       pt.epsLi2Sinit[1]);
    DG_HIP(hipGetLastError());
    // charge rows only, at t0 with unit dt (the time terms of the frozen
    // unknowns do not enter)
    constexpr int kPhiOnly = 1 << 6;
    return solve_once(ctx, t0 - 1.0, 1.0, static_cast<double*>(u), o, report, st, kPhiOnly);
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_initial_state: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_initial_state: unexpected exception");
  }
}

int dg_outputs(dg_ctx* ctx, const void* u, double t, double* U_cell, double* means, double* sums,
               dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (!u) return fail(DG_EINVAL, "dg_outputs: null state");
    if (int s = check_q1(ctx, "dg_outputs")) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    constexpr int nb = kOutBlocks;
    SolverWork& W = ctx->work;
    if (W.out_partial.ensure(size_t(kNumSums) * nb * sizeof(double)) != hipSuccess)
      return fail_mem(ctx, "dg_outputs workspace", size_t(kNumSums) * nb * sizeof(double));
    const DevParams P = make_params(ctx, t, 1.0);
    const double RT = kGas * ctx->params.T;
    const double q = ctx->j_el / (kFaraday * kKEanode);
    hipLaunchKernelGGL(outputs_kernel, dim3(nb), dim3(256), 0, st, static_cast<const double*>(u), ctx->d_phase,
                       P, q, 2.0 * RT / kFaraday, W.out_partial.as<double>());
    DG_HIP(hipGetLastError());
    std::vector<double> part(size_t(kNumSums) * nb);
    DG_HIP(hipMemcpyAsync(part.data(), W.out_partial.p, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    double acc[kNumSums];
    for (int j = 0; j < kNumSums; ++j) {
      double a = 0.0;
      for (int b = 0; b < nb; ++b) a += part[size_t(j) * nb + b];
      acc[j] = a;
    }
    outputs_from_sums(ctx, acc, U_cell, means, sums);
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_outputs: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_outputs: unexpected exception");
  }
}

int dg_outputs_noalloc(dg_ctx* ctx, const void* u, double t, double* U_cell, double* means, double* sums,
                       dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (!u) return fail(DG_EINVAL, "dg_outputs_noalloc: null state");
    if (int s = check_q1(ctx, "dg_outputs_noalloc")) return s;
    double* scr = nullptr;
    if (int s = device_scratch(&scr)) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* partial = scr;                                  // kNumSums x kOutBlocks
    double* total = scr + size_t(kNumSums) * kOutBlocks;    // kNumSums
    const DevParams P = make_params(ctx, t, 1.0);
    const double RT = kGas * ctx->params.T;
    const double q = ctx->j_el / (kFaraday * kKEanode);
    // every partial and every sum is overwritten before it is read: nothing
    // to clear between calls
    hipLaunchKernelGGL(outputs_kernel, dim3(kOutBlocks), dim3(256), 0, st, static_cast<const double*>(u),
                       ctx->d_phase, P, q, 2.0 * RT / kFaraday, partial);
    hipLaunchKernelGGL(outputs_finish_kernel, dim3(1), dim3(64), 0, st, partial, kOutBlocks, total);
    DG_HIP(hipGetLastError());
    double acc[kNumSums];
    DG_HIP(hipMemcpyAsync(acc, total, sizeof(acc), hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    outputs_from_sums(ctx, acc, U_cell, means, sums);
    return DG_OK;
  } catch (...) {
    return fail(DG_EINVAL, "dg_outputs_noalloc: unexpected exception");
  }
}

void dg_controller_init(dg_controller* c, int32_t kind, double dt0, double tol) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->kind = kind;
  c->max_halvings = 30;
  c->successes = 3;
  c->sct = 0;
  c->dt = dt0;
  c->dt_max = 100.0;
  c->grow = 1.2;
  c->tol = tol;
  c->err_prev = tol;
  c->dt_prev = dt0;
}

}  // extern "C"

namespace {
// H211b trials rejected by their error in one dg_advance call before DG_ENOCONV.
constexpr int kMaxH211bRejections = 100;
}  // namespace

extern "C" {

int dg_advance(dg_ctx* ctx, dg_controller* c, double* t, void* u_, const dg_solver_opts* opts,
               dg_advance_report* report, dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (!c || !t || !u_) return fail(DG_EINVAL, "dg_advance: null argument");
    if (int s = check_q1(ctx, "dg_advance")) return s;
    if (!(c->dt > 0) || !(c->dt_max > 0)) return fail(DG_EINVAL, "dg_advance: step sizes must be positive");
    if (c->kind != DG_CTRL_NAIVE && c->kind != DG_CTRL_H211B) return fail(DG_EINVAL, "dg_advance: controller kind");
    if (c->kind == DG_CTRL_H211B && !(c->tol > 0)) return fail(DG_EINVAL, "dg_advance: H211b needs tol > 0");
    dg_solver_opts o;
    if (int s = normalize_opts(opts, o, "dg_advance")) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* u = static_cast<double*>(u_);
    const int64_t n9 = 9 * ctx->Ne * ctx->np;
    const size_t bytes = size_t(n9) * sizeof(double);
    SolverWork& W = ctx->work;
    for (DevBuf* b : {&W.z0, &W.zC, &W.zF}) {
      if (b != &W.z0 && c->kind != DG_CTRL_H211B) continue;
      if (b->ensure(bytes) != hipSuccess) return fail_mem(ctx, "dg_advance workspace", bytes);
    }
    double* z0 = W.z0.as<double>();
    DG_HIP(hipMemcpyAsync(z0, u, bytes, hipMemcpyDeviceToDevice, st));
    dg_advance_report r{};
    auto solve = [&](double* z, double tn, double dt) -> int {
      dg_step_report sr{};
      const int s = solve_once(ctx, tn, dt, z, o, &sr, st);
      r.newton_its += sr.newton_its;
      r.gmres_its += sr.gmres_its;
      return s;
    };
    auto failed_solve = [](int s) { return s == DG_ENOCONV || s == DG_ENAN; };
    auto restore = [&]() -> int {
      DG_HIP(hipMemcpyAsync(u, z0, bytes, hipMemcpyDeviceToDevice, st));
      DG_HIP(hipStreamSynchronize(st));
      return DG_OK;
    };
    int halvings = 0;
    if (c->kind == DG_CTRL_NAIVE) {
      for (;;) {
        const double dt = c->dt;
        ++r.trials;
        const int s = solve(u, *t, dt);
        if (s == DG_OK) {
          if (++c->sct >= c->successes) {
            c->dt = std::min(dt * c->grow, c->dt_max);
            c->sct = 0;
          }
          *t += dt;
          r.dt = dt;
          break;
        }
        if (int e = restore()) return e;
        if (!failed_solve(s)) return s;
        ++halvings;
        ++r.halvings;
        c->sct = 0;
        if (halvings > c->max_halvings) {
          if (report) *report = r;
          return fail(DG_ENOCONV, "dg_advance: more than max_halvings consecutive halvings");
        }
        c->dt = dt / 2;
      }
    } else {
      double* zC = W.zC.as<double>();
      double* zF = W.zF.as<double>();
      double lim = 0.0, err = HUGE_VAL, dt = c->dt;
      int rejections = 0;
      constexpr int nb = 1024;
      if (W.out_partial.ensure(size_t(kNumSums) * nb * sizeof(double)) != hipSuccess)
        return fail_mem(ctx, "dg_advance workspace", size_t(kNumSums) * nb * sizeof(double));
      while (lim < 0.9 || err > 1.02 * c->tol) {
        dt = c->dt;
        ++r.trials;
        DG_HIP(hipMemcpyAsync(zC, z0, bytes, hipMemcpyDeviceToDevice, st));
        int s = solve(zC, *t, dt);
        if (s == DG_OK) {
          DG_HIP(hipMemcpyAsync(zF, z0, bytes, hipMemcpyDeviceToDevice, st));
          s = solve(zF, *t, dt / 2);
          if (s == DG_OK) s = solve(zF, *t + dt / 2, dt / 2);
        }
        if (s != DG_OK) {
          if (!failed_solve(s)) {
            (void)restore();
            return s;
          }
          ++halvings;
          ++r.halvings;
          if (halvings > c->max_halvings) {
            if (report) *report = r;
            return fail(DG_ENOCONV, "dg_advance: more than max_halvings consecutive halvings");
          }
          c->dt = dt / 2;
          lim = 0.0;
          err = HUGE_VAL;
          continue;
        }
        hipLaunchKernelGGL(diff_norm_kernel, dim3(nb), dim3(256), 0, st, zF, zC, n9, W.out_partial.as<double>());
        DG_HIP(hipGetLastError());
        std::vector<double> part(2 * nb);
        DG_HIP(hipMemcpyAsync(part.data(), W.out_partial.p, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        DG_HIP(hipStreamSynchronize(st));
        double d2 = 0.0, f2 = 0.0;
        for (int b = 0; b < nb; ++b) {
          d2 += part[b];
          f2 += part[nb + b];
        }
        err = std::max(std::sqrt(d2) / std::sqrt(f2), 1e-300);
        const double rho = std::pow(c->tol / err, 0.25) * std::pow(c->tol / c->err_prev, 0.25) *
                           std::pow(dt / c->dt_prev, -0.25);
        lim = 1.0 + std::atan(rho - 1.0);
        if (lim < 0.9 || err > 1.02 * c->tol) {
          c->dt = std::min(lim, 0.9) * dt;
          // an error estimate with a floor above the tolerance (the inner
          // solve's attainable accuracy) would otherwise shrink dt forever
          if (++rejections > kMaxH211bRejections) {
            if (report) *report = r;
            return fail(DG_ENOCONV, "dg_advance: H211b rejected more than " +
                                        std::to_string(kMaxH211bRejections) + " trials by their error");
          }
        }
      }
      hipLaunchKernelGGL(richardson_kernel, grid1(n9), dim3(256), 0, st, zF, zC, u, n9);
      DG_HIP(hipGetLastError());
      if (o.limiter)                  // the extrapolated state is limited as each step's root is
        if (int s = limit_state(ctx, u, nullptr, st)) return s;
      DG_HIP(hipStreamSynchronize(st));
      c->err_prev = err;
      c->dt_prev = dt;
      c->dt = std::min(lim * dt, c->dt_max);
      *t += dt;
      r.dt = dt;
      r.err = err;
    }
    if (report) *report = r;
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_advance: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_advance: unexpected exception");
  }
}

int dg_batch_destroy(dg_batch* b) {
  if (!b) return DG_OK;
  for (dg_ctx* c : b->subs) dg_destroy(c);
  if (b->d_phase) (void)hipFree(b->d_phase);
  for (BatchTile* t : b->d_tiles_by)
    if (t) (void)hipFree(t);
  if (b->d_params) (void)hipFree(b->d_params);
  if (b->d_bricks) (void)hipFree(b->d_bricks);
  if (b->d_kpf) (void)hipFree(b->d_kpf);
  if (b->d_kpd) (void)hipFree(b->d_kpd);
  if (b->staged) {
    (void)hipEventSynchronize(b->staged);
    (void)hipEventDestroy(b->staged);
  }
  if (b->h_params) (void)hipHostFree(b->h_params);
  if (b->h_kpf) (void)hipHostFree(b->h_kpf);
  if (b->h_kpd) (void)hipHostFree(b->h_kpd);
  b->lin.release();
  b->blocks.release();
  b->status.release();
  for (DevBuf& w : b->wstate) w.release();
  delete b;
  return DG_OK;
}

int dg_batch_setup(int32_t n, const dg_mesh* meshes, const uint8_t* const* phases, const dg_params* params,
                   dg_batch** out) {
  try {
    if (!out) return fail(DG_EINVAL, "dg_batch_setup: null argument");
    *out = nullptr;
    if (n < 1 || !meshes || !phases || !params)
      return fail(DG_EINVAL, "dg_batch_setup: null argument or fewer than one structure");
    dg_batch* b = new dg_batch;
    auto abandon = [&](int code) {
      dg_batch_destroy(b);
      return code;
    };
    b->off.push_back(0);
    for (int s = 0; s < n; ++s) {
      if (!phases[s])
        return abandon(fail(DG_EINVAL, "dg_batch_setup: null phase map of structure " + std::to_string(s)));
      if (meshes[s].order != 1)
        return abandon(fail(DG_EUNSUPPORTED, "dg_batch_setup: structure " + std::to_string(s) +
                                                 ": batches are built for order 1"));
      dg_ctx* c = nullptr;
      if (int code = dg_setup(&meshes[s], phases[s], &params[s], &c)) {
        const std::string why = g_last_error;
        return abandon(fail(code, "dg_batch_setup: structure " + std::to_string(s) + ": " + why));
      }
      b->subs.push_back(c);
      if (c->Ne > int64_t(INT32_MAX))
        return abandon(fail(DG_EINVAL, "dg_batch_setup: structure " + std::to_string(s) + " has more than 2^31 voxels"));
      b->off.push_back(b->off.back() + c->Ne);
    }
    b->E = b->off.back();
    std::vector<BatchTile> tiles[3];
    for (int ti = 0; ti < 3; ++ti)
      for (int s = 0; s < n; ++s)
        for (int64_t v0 = 0; v0 < b->subs[s]->Ne; v0 += kTileChoices[ti])
          tiles[ti].push_back(BatchTile{int32_t(s), int32_t(v0), b->off[s]});
    std::vector<BatchTile> bricks;
    for (int s = 0; s < n; ++s) {
      const dg_mesh& m = b->subs[s]->mesh;
      const int64_t nbr = int64_t((m.nx + kBE - 1) / kBE) * ((m.ny + kBE - 1) / kBE) * ((m.nz + kBE - 1) / kBE);
      for (int64_t k = 0; k < nbr; ++k) bricks.push_back(BatchTile{int32_t(s), int32_t(k), b->off[s]});
    }
    b->nbricks = int64_t(bricks.size());
    hipError_t e = hipMalloc(&b->d_phase, size_t(b->E));
    for (int ti = 0; ti < 3 && e == hipSuccess; ++ti) {
      b->ntiles_by[ti] = int64_t(tiles[ti].size());
      e = hipMalloc(&b->d_tiles_by[ti], tiles[ti].size() * sizeof(BatchTile));
    }
    b->d_tiles = b->d_tiles_by[2];
    b->ntiles = b->ntiles_by[2];
    if (e == hipSuccess) e = hipMalloc(&b->d_params, size_t(n) * sizeof(DevParams));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_params, size_t(n) * sizeof(DevParams));
    if (e == hipSuccess) e = hipMalloc(&b->d_bricks, bricks.size() * sizeof(BatchTile));
    if (e == hipSuccess) e = hipMalloc(&b->d_kpf, size_t(n) * sizeof(KP<float>));
    if (e == hipSuccess) e = hipMalloc(&b->d_kpd, size_t(n) * sizeof(KP<double>));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_kpf, size_t(n) * sizeof(KP<float>));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_kpd, size_t(n) * sizeof(KP<double>));
    if (e != hipSuccess) return abandon(fail(DG_ENOMEM, std::string("dg_batch_setup: ") + hipGetErrorString(e)));
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
    for (int s = 0; s < n && e == hipSuccess; ++s)
      e = hipMemcpy(b->d_phase + b->off[s], phases[s], size_t(b->subs[s]->Ne), hipMemcpyHostToDevice);
    for (int ti = 0; ti < 3 && e == hipSuccess; ++ti)
      e = hipMemcpy(b->d_tiles_by[ti], tiles[ti].data(), tiles[ti].size() * sizeof(BatchTile),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(b->d_bricks, bricks.data(), bricks.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
    if (e != hipSuccess) return abandon(fail(DG_EHIP, std::string("dg_batch_setup: ") + hipGetErrorString(e)));
    {
      std::lock_guard<std::mutex> lk(g_shape_mu);
      for (int p = 0; p < 2; ++p)
        for (int op = 0; op < 3; ++op) {
          auto it = g_shape_cache.find({p, op, size_class(b->E)});
          b->shape[p][op] = it == g_shape_cache.end() ? default_shape(op) : it->second;
        }
    }
    *out = b;
    return DG_OK;
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_batch_setup: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_batch_setup: unexpected exception");
  }
}

int dg_batch_layout(const dg_batch* b, int64_t* offsets, int64_t* n_tiles) {
  if (!b) return fail(DG_EINVAL, "dg_batch_layout: null batch");
  if (offsets)
    for (size_t i = 0; i < b->off.size(); ++i) offsets[i] = b->off[i];
  if (n_tiles) *n_tiles = b->ntiles;
  return DG_OK;
}

int dg_batch_mass(dg_batch* b, dg_prec prec, const void* u, void* m, dg_stream stream) {
  if (!b) return fail(DG_EINVAL, "dg_batch_mass: null batch");
  if (!u || !m) return fail(DG_EINVAL, "dg_batch_mass: null array");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_mass: bad precision");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int s = batch_params(b, nullptr, nullptr, false, st, "dg_batch_mass")) return s;
  const int64_t nb = batch_grid(b);
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  if (prec == DG_F64)
    hipLaunchKernelGGL(mass_batch_kernel<double>, grid, block, 0, st, static_cast<const double*>(u),
                       static_cast<double*>(m), b->d_phase, b->d_params, b->d_tiles, b->ntiles, b->E * 8, nb);
  else
    hipLaunchKernelGGL(mass_batch_kernel<float>, grid, block, 0, st, static_cast<const float*>(u),
                       static_cast<float*>(m), b->d_phase, b->d_params, b->d_tiles, b->ntiles, b->E * 8, nb);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_batch_residual(dg_batch* b, dg_prec prec, const void* u, const void* m_old, const double* t_new,
                      const double* dt, void* r, dg_stream stream) {
  if (!b) return fail(DG_EINVAL, "dg_batch_residual: null batch");
  if (!u || !m_old || !r) return fail(DG_EINVAL, "dg_batch_residual: null array");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_residual: bad precision");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int s = batch_params(b, t_new, dt, true, st, "dg_batch_residual")) return s;
  if (prec == DG_F64)
    launch_q1_batch<double, double, kResidual>(b, u, nullptr, m_old, r, st);
  else
    launch_q1_batch<float, float, kResidual>(b, u, nullptr, m_old, r, st);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_batch_linearize(dg_batch* b, dg_prec prec, const void* u, const double* t_new, const double* dt,
                       dg_stream stream) {
  if (!b) return fail(DG_EINVAL, "dg_batch_linearize: null batch");
  if (!u) return fail(DG_EINVAL, "dg_batch_linearize: null array");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_linearize: bad precision");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int s = batch_params(b, t_new, dt, true, st, "dg_batch_linearize")) return s;
  return prec == DG_F64 ? batch_linearize<double>(b, static_cast<const double*>(u), st)
                        : batch_linearize<float>(b, static_cast<const float*>(u), st);
}

int dg_batch_jvp(dg_batch* b, dg_prec prec, dg_jvp_mode mode, const void* u, const void* v,
                 const double* t_new, const double* dt, void* jv, dg_stream stream) {
  if (!b) return fail(DG_EINVAL, "dg_batch_jvp: null batch");
  if (!u || !v || !jv) return fail(DG_EINVAL, "dg_batch_jvp: null array");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_jvp: bad precision");
  if (mode != DG_JVP_FULL9 && mode != DG_JVP_CONDENSED7 && mode != DG_JVP_LINEARIZED7)
    return fail(DG_EINVAL, "dg_batch_jvp: bad mode");
  if (mode == DG_JVP_LINEARIZED7 && b->lin_prec != int(prec))
    return fail(DG_ESTATE, "dg_batch_jvp: no batch linearisation of this precision (dg_batch_linearize)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int s = batch_params(b, t_new, dt, true, st, "dg_batch_jvp", mode != DG_JVP_FULL9)) return s;
  if (mode == DG_JVP_FULL9) {
    if (prec == DG_F64)
      launch_q1_batch<double, Dual<double>, kJvpFull>(b, u, v, nullptr, jv, st);
    else
      launch_q1_batch<float, Dual<float>, kJvpFull>(b, u, v, nullptr, jv, st);
  } else {
    if (mode == DG_JVP_CONDENSED7) {
      const int s = prec == DG_F64 ? batch_linearize<double>(b, static_cast<const double*>(u), st)
                                   : batch_linearize<float>(b, static_cast<const float*>(u), st);
      if (s) return s;
    }
    if (prec == DG_F64)
      launch_q1_batch<double, Dual<double>, kJvpCondensed>(b, u, v, b->lin.p, jv, st);
    else
      launch_q1_batch<float, Dual<float>, kJvpCondensed>(b, u, v, b->lin.p, jv, st);
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_batch_blockjacobi_setup(dg_batch* b, dg_prec prec, const void* u, const double* t_new,
                               const double* dt, dg_stream stream) {
  if (!b) return fail(DG_EINVAL, "dg_batch_blockjacobi_setup: null batch");
  if (!u) return fail(DG_EINVAL, "dg_batch_blockjacobi_setup: null array");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_blockjacobi_setup: bad precision");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int s = batch_params(b, t_new, dt, true, st, "dg_batch_blockjacobi_setup")) return s;
  return prec == DG_F64 ? batch_blocks<double>(b, static_cast<const double*>(u), st)
                        : batch_blocks<float>(b, static_cast<const float*>(u), st);
}

int dg_batch_blockjacobi_apply(dg_batch* b, dg_prec prec, const void* x, void* y, dg_stream stream) {
  if (!b) return fail(DG_EINVAL, "dg_batch_blockjacobi_apply: null batch");
  if (!x || !y) return fail(DG_EINVAL, "dg_batch_blockjacobi_apply: null array");
  if (b->blocks_prec < 0) return fail(DG_ESTATE, "dg_batch_blockjacobi_apply: no setup yet");
  if (int(prec) != b->blocks_prec)
    return fail(DG_EINVAL, "dg_batch_blockjacobi_apply: precision differs from the setup");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid{unsigned((b->E + 3) / 4), 1, 1}, block{256, 1, 1};
  if (prec == DG_F64)
    hipLaunchKernelGGL((apply_blocks_kernel<double, 7>), grid, block, 0, st, b->blocks.as<const double>(),
                       static_cast<const double*>(x), static_cast<double*>(y), b->E);
  else
    hipLaunchKernelGGL((apply_blocks_kernel<float, 7>), grid, block, 0, st, b->blocks.as<const float>(),
                       static_cast<const float*>(x), static_cast<float*>(y), b->E);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // extern "C"

namespace {

// Run job(s, worker, stream) for every structure of the batch on `workers`
// host threads, each with a HIP stream of its own and default priority:
// the structures' Newton solves are independent, and their host-driven
// control flow (convergence tests, line searches, restarts) diverges, so
// they proceed side by side rather than in lock step.  Structures are
// taken largest first.  Every job runs; the first failing structure (in
// structure order) gives the return status and message.
template <typename Job>
int batch_run(dg_batch* b, int workers, const char* fn, Job job) {
  const int n = int(b->subs.size());
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->subs[x]->Ne > b->subs[y]->Ne; });
  int dev = 0;
  DG_HIP(hipGetDevice(&dev));
  std::vector<hipStream_t> streams(workers, nullptr);
  for (int w = 0; w < workers; ++w) {
    hipError_t e = hipStreamCreate(&streams[w]);
    if (e != hipSuccess) {
      for (int v = 0; v < w; ++v) (void)hipStreamDestroy(streams[v]);
      return fail(DG_EHIP, std::string(fn) + ": hipStreamCreate: " + hipGetErrorString(e));
    }
  }
  std::vector<int> status(n, DG_OK);
  std::vector<std::string> msg(n);
  std::atomic<int> next{0};
  auto work = [&](int w) {
    (void)hipSetDevice(dev);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const int s = order[k];
      try {
        status[s] = job(s, w, streams[w]);
      } catch (...) {
        status[s] = fail(DG_EINVAL, "unexpected exception");
      }
      if (status[s]) msg[s] = g_last_error;   // this worker's thread-local message
    }
    (void)hipStreamSynchronize(streams[w]);
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < workers; ++w) {
    try {
      pool.emplace_back(work, w);
    } catch (...) {
      break;   // fewer threads: the shared counter hands their structures to the others
    }
  }
  work(0);
  for (auto& t : pool) t.join();
  for (hipStream_t st : streams) (void)hipStreamDestroy(st);
  for (int s = 0; s < n; ++s)
    if (status[s]) return fail(status[s], std::string(fn) + ": structure " + std::to_string(s) + ": " + msg[s]);
  return DG_OK;
}

// Per-worker contiguous state of the largest structure (9 fields, FP64).
int batch_state_buffers(dg_batch* b, int workers, const char* fn) {
  int64_t max_ne = 0;
  for (dg_ctx* c : b->subs) max_ne = std::max(max_ne, c->Ne);
  if (int(b->wstate.size()) < workers) b->wstate.resize(workers);
  for (int w = 0; w < workers; ++w) {
    hipError_t e = b->wstate[w].ensure(size_t(9) * max_ne * 8 * sizeof(double));
    if (e != hipSuccess) return fail(DG_ENOMEM, std::string(fn) + ": state buffers: " + hipGetErrorString(e));
  }
  return DG_OK;
}

// Structure s's slice of a batch state (field stride E * 8) to or from a
// contiguous 9 x Ne_s x 8 state.
hipError_t batch_copy(const dg_batch* b, int s, double* batch_u, double* own, bool to_own, hipStream_t st) {
  const size_t row = size_t(b->subs[s]->Ne) * 8 * sizeof(double);
  const size_t pitch = size_t(b->E) * 8 * sizeof(double);
  double* slice = batch_u + b->off[s] * 8;
  return to_own ? hipMemcpy2DAsync(own, row, slice, pitch, row, 9, hipMemcpyDeviceToDevice, st)
                : hipMemcpy2DAsync(slice, pitch, own, row, row, 9, hipMemcpyDeviceToDevice, st);
}

int batch_workers(const dg_batch* b, int32_t workers) {
  const int n = int(b->subs.size());
  int w = workers > 0 ? workers : 4;
  return std::max(1, std::min(w, n));
}

// Times one batched operator in every launch shape (three tile sizes, each
// with one workgroup per work item and as a persistent grid at the
// occupancy the compiled kernel allows), keeps the fastest for the batch
// and the process cache, and reports it with the default shape's time.
template <typename S, typename N, int Mode>
int tune_op(dg_batch* b, const void* u, const void* v, const void* m, void* work, int reps, hipEvent_t t0,
            hipEvent_t t1, dg_batch_tuning* rep, hipStream_t st) {
  constexpr int op = op_index<Mode>();
  constexpr dg_batch_shape def = default_shape(op);
  dg_batch_shape best = def;
  double best_ms = INFINITY, def_ms = NAN;
  int tried = 0;
  auto time_shape = [&](dg_batch_shape sh, bool brick) -> int {
    auto launch = [&] {
      if (brick)
        launch_brick_batch<S>(b, u, v, work, st);
      else
        launch_q1_batch_shape<S, N, Mode>(b, sh, u, v, m, work, st);
    };
    launch();   // warm-up
    DG_HIP(hipEventRecord(t0, st));
    for (int r = 0; r < reps; ++r) launch();
    DG_HIP(hipGetLastError());
    DG_HIP(hipEventRecord(t1, st));
    DG_HIP(hipEventSynchronize(t1));
    float ms = 0.f;
    DG_HIP(hipEventElapsedTime(&ms, t0, t1));
    const double per = double(ms) / reps;
    if (sh.tile_voxels == def.tile_voxels && sh.persistent == def.persistent) def_ms = per;
    if (per < best_ms) {
      best_ms = per;
      best = sh;
    }
    return DG_OK;
  };
  for (int tv : kTileChoices) {
    const int occ = q1_batch_resident<S, N, Mode>(tv);
    const int forms = occ > 0 ? 2 : 1;             // occupancy unknown: no persistent form
    for (int f = 0; f < forms; ++f) {
      if (int s = time_shape(dg_batch_shape{tv, f == 0 ? 0 : occ}, false)) return s;
      tried += 1;
    }
  }
  if (Mode == kJvpCondensed)
    if (int s = time_shape(kBrickShape, true)) return s;
  b->shape[prec_index<S>()][op] = best;
  {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shape_cache[{prec_index<S>(), op, size_class(b->E)}] = best;
  }
  rep->shape[op] = best;
  rep->ms[op] = best_ms;
  rep->ms_default[op] = def_ms;
  rep->candidates = tried;
  return DG_OK;
}

template <typename S>
int batch_autotune(dg_batch* b, const S* u, const S* v, const S* m_old, S* work, int reps, dg_batch_tuning* rep,
                   hipStream_t st) {
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  int status = e == hipSuccess ? DG_OK : fail(DG_EHIP, std::string("dg_batch_autotune: ") + hipGetErrorString(e));
  if (!status) status = tune_op<S, S, kResidual>(b, u, nullptr, m_old, work, reps, t0, t1, rep, st);
  if (!status) status = tune_op<S, Dual<S>, kJvpFull>(b, u, v, nullptr, work, reps, t0, t1, rep, st);
  if (!status) status = batch_linearize<S>(b, u, st);
  if (!status) status = tune_op<S, Dual<S>, kJvpCondensed>(b, u, v, b->lin.p, work, reps, t0, t1, rep, st);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  return status;
}

}  // namespace

extern "C" {

int dg_batch_set_shape(dg_batch* b, dg_prec prec, int32_t op, const dg_batch_shape* shape) {
  if (!b || !shape) return fail(DG_EINVAL, "dg_batch_set_shape: null argument");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_set_shape: bad precision");
  if (op < 0 || op > 2) return fail(DG_EINVAL, "dg_batch_set_shape: bad operator");
  const int tv = shape->tile_voxels;
  if (tv == kBrickShape.tile_voxels) {
    if (op != DG_BOP_JVP_CONDENSED7)
      return fail(DG_EINVAL, "dg_batch_set_shape: the brick shape (64) is for the condensed tangent only");
    if (shape->persistent != 0) return fail(DG_EINVAL, "dg_batch_set_shape: the brick shape takes persistent = 0");
  } else if (std::find(std::begin(kTileChoices), std::end(kTileChoices), tv) == std::end(kTileChoices)) {
    return fail(DG_EINVAL, "dg_batch_set_shape: tile_voxels must be 8, 16, 32 or (condensed tangent) 64");
  }
  if (shape->persistent < 0 || shape->persistent > 64)
    return fail(DG_EINVAL, "dg_batch_set_shape: persistent must be in [0, 64]");
  b->shape[prec][op] = *shape;
  return DG_OK;
}

int dg_batch_get_shape(const dg_batch* b, dg_prec prec, int32_t op, dg_batch_shape* shape) {
  if (!b || !shape) return fail(DG_EINVAL, "dg_batch_get_shape: null argument");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_get_shape: bad precision");
  if (op < 0 || op > 2) return fail(DG_EINVAL, "dg_batch_get_shape: bad operator");
  *shape = b->shape[prec][op];
  return DG_OK;
}

int dg_batch_autotune(dg_batch* b, dg_prec prec, const void* u, const void* v, const void* m_old,
                      const double* t_new, const double* dt, void* work, int32_t reps, dg_batch_tuning* report,
                      dg_stream stream) {
  if (!b || !report) return fail(DG_EINVAL, "dg_batch_autotune: null argument");
  if (!u || !v || !m_old || !work) return fail(DG_EINVAL, "dg_batch_autotune: null array");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_batch_autotune: bad precision");
  if (reps > 1000) return fail(DG_EINVAL, "dg_batch_autotune: reps above 1000");
  const int r = reps > 0 ? reps : 5;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::memset(report, 0, sizeof(*report));
  if (int s = batch_params(b, t_new, dt, true, st, "dg_batch_autotune", true)) return s;
  return prec == DG_F64
             ? batch_autotune<double>(b, static_cast<const double*>(u), static_cast<const double*>(v),
                                      static_cast<const double*>(m_old), static_cast<double*>(work), r, report, st)
             : batch_autotune<float>(b, static_cast<const float*>(u), static_cast<const float*>(v),
                                     static_cast<const float*>(m_old), static_cast<float*>(work), r, report, st);
}

int dg_batch_initial_state(dg_batch* b, const double* t0, void* u, const dg_solver_opts* opts,
                           dg_step_report* reports, int32_t workers, dg_stream stream) {
  try {
    if (!b) return fail(DG_EINVAL, "dg_batch_initial_state: null batch");
    if (!t0 || !u) return fail(DG_EINVAL, "dg_batch_initial_state: null t0 or state");
    const int nw = batch_workers(b, workers);
    if (int s = batch_state_buffers(b, nw, "dg_batch_initial_state")) return s;
    DG_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    double* bu = static_cast<double*>(u);
    return batch_run(b, nw, "dg_batch_initial_state", [&](int s, int w, hipStream_t st) -> int {
      double* own = b->wstate[w].as<double>();
      dg_step_report rep{};
      const int code = dg_initial_state(b->subs[s], t0[s], own, opts, &rep, st);
      if (reports) reports[s] = rep;
      if (code) return code;
      DG_HIP(batch_copy(b, s, bu, own, false, st));
      DG_HIP(hipStreamSynchronize(st));
      return DG_OK;
    });
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_batch_initial_state: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_batch_initial_state: unexpected exception");
  }
}

int dg_batch_step(dg_batch* b, const double* t_n, const double* dt, void* u, const dg_solver_opts* opts,
                  dg_step_report* reports, int32_t workers, dg_stream stream) {
  try {
    if (!b) return fail(DG_EINVAL, "dg_batch_step: null batch");
    if (!t_n || !dt || !u) return fail(DG_EINVAL, "dg_batch_step: null t_n, dt or state");
    for (size_t s = 0; s < b->subs.size(); ++s)
      if (!(dt[s] > 0)) return fail(DG_EINVAL, "dg_batch_step: dt[" + std::to_string(s) + "] must be positive");
    const int nw = batch_workers(b, workers);
    if (int s = batch_state_buffers(b, nw, "dg_batch_step")) return s;
    DG_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    double* bu = static_cast<double*>(u);
    return batch_run(b, nw, "dg_batch_step", [&](int s, int w, hipStream_t st) -> int {
      double* own = b->wstate[w].as<double>();
      DG_HIP(batch_copy(b, s, bu, own, true, st));
      dg_step_report rep{};
      const int code = dg_step(b->subs[s], t_n[s], dt[s], own, opts, &rep, st);
      if (reports) reports[s] = rep;
      // the last iterate goes back on failure too, as dg_step leaves it in u
      DG_HIP(batch_copy(b, s, bu, own, false, st));
      DG_HIP(hipStreamSynchronize(st));
      return code;
    });
  } catch (const std::bad_alloc&) {
    return fail(DG_ENOMEM, "dg_batch_step: host allocation failed");
  } catch (...) {
    return fail(DG_EINVAL, "dg_batch_step: unexpected exception");
  }
}

int dg_limit(dg_ctx* ctx, void* u, void* alpha, dg_stream stream) {
  try {
    if (int s = check_ctx(ctx)) return s;
    if (!u) return fail(DG_EINVAL, "dg_limit: null state");
    return limit_state(ctx, static_cast<double*>(u), static_cast<double*>(alpha), static_cast<hipStream_t>(stream));
  } catch (...) {
    return fail(DG_EINVAL, "dg_limit: unexpected exception");
  }
}

int dg_triad(double* out, const double* a, const double* b, double s, int64_t n, dg_stream stream) {
  try {
    if (n < 0) return fail(DG_EINVAL, "dg_triad: negative length");
    if (n == 0) return DG_OK;
    if (!out || !a || !b) return fail(DG_EINVAL, "dg_triad: null array");
    if ((n & 1) || ((reinterpret_cast<uintptr_t>(out) | reinterpret_cast<uintptr_t>(a) |
                     reinterpret_cast<uintptr_t>(b)) & 15))
      return fail(DG_EINVAL, "dg_triad: arrays must be 16-byte aligned and of even length");
    const int64_t n2 = n / 2;
    // one pass of the grid where possible: each lane two 16-byte pairs
    const int64_t want = (n2 + 511) / 512;
    const unsigned nb = unsigned(want < (int64_t(1) << 20) ? want : (int64_t(1) << 20));
    hipLaunchKernelGGL(triad_kernel, dim3(nb), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<double2*>(out), reinterpret_cast<const double2*>(a),
                       reinterpret_cast<const double2*>(b), s, n2);
    DG_HIP(hipGetLastError());
    return DG_OK;
  } catch (...) {
    return fail(DG_EINVAL, "dg_triad: unexpected exception");
  }
}

const char* dg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
