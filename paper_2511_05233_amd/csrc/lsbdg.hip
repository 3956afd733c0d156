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
  const int64_t threads = ctx->Ne * 8;
  int64_t nb = (threads + 255) / 256;
  nb = (nb + 7) / 8 * 8;
  const dim3 grid{unsigned(nb), 1, 1}, block{256, 1, 1};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (prec == DG_F64)
    hipLaunchKernelGGL(resid_q1_kernel<double>, grid, block, 0, st,
                       static_cast<const double*>(u), static_cast<const double*>(m_old),
                       static_cast<double*>(r), ctx->d_phase, P, nb);
  else if (prec == DG_F32)
    hipLaunchKernelGGL(resid_q1_kernel<float>, grid, block, 0, st,
                       static_cast<const float*>(u), static_cast<const float*>(m_old),
                       static_cast<float*>(r), ctx->d_phase, P, nb);
  else
    return fail(DG_EINVAL, "dg_residual: bad precision");
  DG_HIP(hipGetLastError());
  return DG_OK;
}

const char* dg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
