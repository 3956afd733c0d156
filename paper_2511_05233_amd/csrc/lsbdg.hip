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
#include <new>
#include <string>
#include <vector>

#include "../../include/lsbdg.h"
#include "model.hpp"
#include "pointwise.hpp"
#include "resid_q1.hpp"
#include "blockjacobi.hpp"

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
  // element block-Jacobi storage (condensed 56 x 56 inverses, column-major)
  void* d_blocks = nullptr;
  size_t blocks_bytes = 0;
  int blocks_prec = -1;
  int* d_status = nullptr;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
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
  P.W3 = (h / 2) * (h / 2) * (h / 2);
  P.W2 = (h / 2) * (h / 2);
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
  return P;
}

int check_ctx(const dg_ctx* c) {
  if (!c) return fail(DG_EINVAL, "null context");
  return DG_OK;
}

}  // namespace

namespace {

template <typename S, typename N, int Mode>
void launch_q1(const dg_ctx* ctx, const DevParams& P, const void* u, const void* v, const void* m,
               void* out, hipStream_t st) {
  const int64_t threads = ctx->Ne * 8;
  int64_t nb = (threads + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  hipLaunchKernelGGL((q1_kernel<S, N, Mode>), grid, block, 0, st, static_cast<const S*>(u),
                     static_cast<const S*>(v), static_cast<const S*>(m), static_cast<S*>(out),
                     ctx->d_phase, P, nb);
}

}  // namespace

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

int dg_setup(const dg_mesh* mesh, const uint8_t* phase, const dg_params* params, dg_ctx** out) {
  try {
    if (!mesh || !phase || !params || !out) return fail(DG_EINVAL, "dg_setup: null argument");
    *out = nullptr;
    if (mesh->nx <= 0 || mesh->ny <= 0 || mesh->nz <= 0 || !(mesh->h > 0))
      return fail(DG_EINVAL, "dg_setup: mesh sizes and h must be positive");
    if (mesh->order != 1)
      return fail(DG_EUNSUPPORTED, "dg_setup: order " + std::to_string(mesh->order) +
                                       " not implemented (supported: 1)");
    if (!(params->T > 0)) return fail(DG_EINVAL, "dg_setup: temperature must be positive");
    const int64_t Ne = int64_t(mesh->nx) * mesh->ny * mesh->nz;
    int64_t n_struct = 0;
    for (int64_t e = 0; e < Ne; ++e) {
      if (phase[e] > 1) return fail(DG_EINVAL, "dg_setup: phase values must be 0 or 1");
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
    hipError_t err = hipMalloc(&c->d_phase, size_t(Ne));
    if (err != hipSuccess) {
      delete c;
      return fail(DG_ENOMEM, std::string("dg_setup: hipMalloc: ") + hipGetErrorString(err));
    }
    err = hipMemcpy(c->d_phase, phase, size_t(Ne), hipMemcpyHostToDevice);
    if (err != hipSuccess) {
      (void)hipFree(c->d_phase);
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

int dg_destroy(dg_ctx* ctx) {
  if (!ctx) return DG_OK;
  if (ctx->d_phase) (void)hipFree(ctx->d_phase);
  if (ctx->d_blocks) (void)hipFree(ctx->d_blocks);
  if (ctx->d_status) (void)hipFree(ctx->d_status);
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
  } else if (mode == DG_JVP_CONDENSED7) {
    if (prec == DG_F64)
      launch_q1<double, Dual<double>, kJvpCondensed>(ctx, P, u, v, nullptr, jv, st);
    else if (prec == DG_F32)
      launch_q1<float, Dual<float>, kJvpCondensed>(ctx, P, u, v, nullptr, jv, st);
    else
      return fail(DG_EINVAL, "dg_jvp: bad precision");
  } else {
    return fail(DG_EINVAL, "dg_jvp: bad mode");
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}


constexpr int kNB = 56;   // condensed Q1 block size: 7 fields x 8 nodes

int dg_blockjacobi_setup(dg_ctx* ctx, dg_prec prec, const void* u, double t_new, double dt,
                         dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!u) return fail(DG_EINVAL, "dg_blockjacobi_setup: null array");
  if (!(dt > 0)) return fail(DG_EINVAL, "dg_blockjacobi_setup: dt must be positive");
  if (prec != DG_F64 && prec != DG_F32) return fail(DG_EINVAL, "dg_blockjacobi_setup: bad precision");
  const size_t esz = prec == DG_F64 ? sizeof(double) : sizeof(float);
  const size_t need = size_t(ctx->Ne) * kNB * kNB * esz;
  if (ctx->blocks_bytes < need) {
    if (ctx->d_blocks) (void)hipFree(ctx->d_blocks);
    ctx->d_blocks = nullptr;
    ctx->blocks_bytes = 0;
    hipError_t err = hipMalloc(&ctx->d_blocks, need);
    if (err != hipSuccess)
      return fail(DG_ENOMEM, std::string("dg_blockjacobi_setup: hipMalloc of ") +
                                 std::to_string(need) + " bytes: " + hipGetErrorString(err));
    ctx->blocks_bytes = need;
  }
  if (!ctx->d_status) {
    hipError_t err = hipMalloc(&ctx->d_status, sizeof(int));
    if (err != hipSuccess) return fail(DG_ENOMEM, "dg_blockjacobi_setup: status allocation");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  DG_HIP(hipMemsetAsync(ctx->d_status, 0, sizeof(int), st));
  const DevParams P = make_params(ctx, t_new, dt);
  int64_t nb = (ctx->Ne * 8 + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  const dim3 grid_w{unsigned((ctx->Ne + 3) / 4), 1, 1};
  if (prec == DG_F64) {
    hipLaunchKernelGGL((q1_block_kernel<double, kJvpCondensed>), grid, block, 0, st,
                       static_cast<const double*>(u), static_cast<double*>(ctx->d_blocks),
                       ctx->d_phase, P, nb);
    hipLaunchKernelGGL((invert_blocks_kernel<double, kNB>), grid_w, block, 0, st,
                       static_cast<double*>(ctx->d_blocks), ctx->Ne, ctx->d_status);
  } else {
    hipLaunchKernelGGL((q1_block_kernel<float, kJvpCondensed>), grid, block, 0, st,
                       static_cast<const float*>(u), static_cast<float*>(ctx->d_blocks),
                       ctx->d_phase, P, nb);
    hipLaunchKernelGGL((invert_blocks_kernel<float, kNB>), grid_w, block, 0, st,
                       static_cast<float*>(ctx->d_blocks), ctx->Ne, ctx->d_status);
  }
  DG_HIP(hipGetLastError());
  int h_status = 0;
  DG_HIP(hipMemcpyAsync(&h_status, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, st));
  DG_HIP(hipStreamSynchronize(st));
  ctx->blocks_prec = int(prec);
  if (h_status) return fail(DG_ENAN, "dg_blockjacobi_setup: singular or non-finite element block");
  return DG_OK;
}

int dg_blockjacobi_apply(dg_ctx* ctx, dg_prec prec, const void* x, void* y, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!x || !y) return fail(DG_EINVAL, "dg_blockjacobi_apply: null array");
  if (ctx->blocks_prec < 0) return fail(DG_ESTATE, "dg_blockjacobi_apply: no setup yet");
  if (int(prec) != ctx->blocks_prec)
    return fail(DG_EINVAL, "dg_blockjacobi_apply: precision differs from the setup");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const dim3 grid{unsigned((ctx->Ne + 3) / 4), 1, 1}, block{256, 1, 1};
  if (prec == DG_F64)
    hipLaunchKernelGGL((apply_blocks_kernel<double, 7>), grid, block, 0, st,
                       static_cast<const double*>(ctx->d_blocks), static_cast<const double*>(x),
                       static_cast<double*>(y), ctx->Ne);
  else
    hipLaunchKernelGGL((apply_blocks_kernel<float, 7>), grid, block, 0, st,
                       static_cast<const float*>(ctx->d_blocks), static_cast<const float*>(x),
                       static_cast<float*>(y), ctx->Ne);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int dg_blockjacobi_export(dg_ctx* ctx, void* out, dg_stream stream) {
  if (int s = check_ctx(ctx)) return s;
  if (!out) return fail(DG_EINVAL, "dg_blockjacobi_export: null array");
  if (ctx->blocks_prec < 0) return fail(DG_ESTATE, "dg_blockjacobi_export: no setup yet");
  const size_t esz = ctx->blocks_prec == DG_F64 ? sizeof(double) : sizeof(float);
  DG_HIP(hipMemcpyAsync(out, ctx->d_blocks, size_t(ctx->Ne) * kNB * kNB * esz,
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return DG_OK;
}

const char* dg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
