// C ABI of the filtered LB-MHD engine (lbmhd.h, lbmhd_learned.h): parameter
// validation, rates, buffer binding, time/parity bookkeeping and error
// reporting.  The per-cell arithmetic and all device work live in
// lbmhd_kernels.hip and lbmhd_learned.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "lbmhd.h"
#include "lbmhd_internal.h"
#include "lbmhd_learned.h"

struct lbm_ctx {
  lbm_params p;
  lbm::Launch L;
  int64_t t = 0;
  bool initialized = false;
  bool mlp_set = false;  // learned closure: a network has been installed
  bool cus_known = false;  // compute-unit count queried
  bool lag_ready = false;  // lagged schedule: moment set t & 1 holds step t - 1
  int32_t corr_every = 1;  // learned closure: correction evaluated every corr_every steps
  bool corr_ready = false;  // learned closure: the correction planes hold a held correction
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(LBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validate and derive rates.  Returns LBM_OK or LBM_EINVAL with a message.
int check_params(const lbm_params* p, lbm::Launch* L) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->dtype != LBM_FP64 && p->dtype != LBM_FP32 && p->dtype != LBM_FP16 && p->dtype != LBM_BF16)
    return fail(LBM_EINVAL, "dtype must be LBM_FP64, LBM_FP32, LBM_FP16 or LBM_BF16");
  if (p->nx < 4 || p->ny < 4 || p->nx > 32768 || p->ny > 32768)
    return fail(LBM_EINVAL, "nx and ny must lie in [4, 32768]");
  if (!finite_pos(p->nu) || !finite_pos(p->eta)) return fail(LBM_EINVAL, "nu and eta must be finite and > 0");
  const double ghost[4] = {p->s5, p->s6, p->s7, p->s8};
  for (double g : ghost) {
    if (!std::isfinite(g)) return fail(LBM_EINVAL, "ghost rates must be finite");
    if (g > 0.0 && g >= 2.0) return fail(LBM_EINVAL, "ghost rates must lie in (0, 2) (or <= 0 for s3)");
  }
  if (!std::isfinite(p->delta) || p->delta < 0.0) return fail(LBM_EINVAL, "delta must be finite and >= 0");
  if (!std::isfinite(p->closure_scale)) return fail(LBM_EINVAL, "closure_scale must be finite");
  if (p->grad_stencil < LBM_STENCIL_ISO9 || p->grad_stencil > LBM_STENCIL_LOCAL_CENTRAL5)
    return fail(LBM_EINVAL, "grad_stencil must be one of LBM_STENCIL_*");
  if (p->grad_stencil >= LBM_STENCIL_LOCAL_ISO9 && p->schedule == LBM_SCHED_AA_LAGGED)
    return fail(LBM_EINVAL, "local gradients need the current populations: not with LBM_SCHED_AA_LAGGED");
  if (p->schedule != LBM_SCHED_FUSED && p->schedule != LBM_SCHED_AA && p->schedule != LBM_SCHED_AA_LAGGED)
    return fail(LBM_EINVAL, "schedule must be LBM_SCHED_FUSED, LBM_SCHED_AA or LBM_SCHED_AA_LAGGED");
  if (p->closure != LBM_CLOSURE_ANALYTIC && p->closure != LBM_CLOSURE_LEARNED && p->closure != LBM_CLOSURE_FULL)
    return fail(LBM_EINVAL, "closure must be one of LBM_CLOSURE_*");
  if (p->closure == LBM_CLOSURE_FULL &&
      (p->schedule != LBM_SCHED_FUSED || p->grad_stencil >= LBM_STENCIL_LOCAL_ISO9))
    return fail(LBM_EINVAL, "the density-gradient closure runs with LBM_SCHED_FUSED and a stencil gradient only");
  if (p->closure == LBM_CLOSURE_LEARNED && p->schedule != LBM_SCHED_FUSED)
    return fail(LBM_EINVAL, "the learned closure runs with LBM_SCHED_FUSED only");
  if (p->mag_lattice != LBM_MAG_D2Q5 && p->mag_lattice != LBM_MAG_D2Q9)
    return fail(LBM_EINVAL, "mag_lattice must be LBM_MAG_D2Q5 or LBM_MAG_D2Q9");
  if (p->reserved != 0) return fail(LBM_EINVAL, "reserved must be 0");
  if (p->mag_lattice == LBM_MAG_D2Q9 &&
      (p->schedule != LBM_SCHED_FUSED || p->closure == LBM_CLOSURE_LEARNED ||
       p->grad_stencil >= LBM_STENCIL_LOCAL_ISO9 || (p->dtype != LBM_FP64 && p->dtype != LBM_FP32)))
    return fail(LBM_EINVAL, "the D2Q9 vector distribution runs with LBM_SCHED_FUSED, a stencil gradient, "
                            "the analytic or density-gradient closure and FP64 or FP32 storage");
  if (!finite_pos(p->rho0)) return fail(LBM_EINVAL, "rho0 must be finite and > 0");
  if (!std::isfinite(p->bref_x) || !std::isfinite(p->bref_y)) return fail(LBM_EINVAL, "bref must be finite");
  if (L) {
    // nu = 1/(3 s) - 1/6, eta = 1/(3 s_m) - 1/6 (Sec. 2); nu, eta > 0 put s in (0, 2).
    const double s = 2.0 / (6.0 * p->nu + 1.0);
    L->nx = p->nx;
    L->ny = p->ny;
    L->pitch = lbm::row_pitch(p->nx);
    L->dtype = p->dtype;
    L->schedule = p->schedule;
    L->stencil = p->grad_stencil;
    L->qg = p->mag_lattice == LBM_MAG_D2Q9 ? 9 : 5;
    L->learned = p->closure == LBM_CLOSURE_LEARNED;
    L->full = p->closure == LBM_CLOSURE_FULL;
    for (double& r : L->rate) r = 0.0;
    L->rate[3] = s;
    L->rate[4] = s;
    for (int k = 0; k < 4; ++k) L->rate[5 + k] = ghost[k] > 0.0 ? ghost[k] : s;
    L->sm = 2.0 / (6.0 * p->eta + 1.0);
    L->k2 = p->closure_scale * p->delta * p->delta / 12.0;
    // FP32 stores f_i - w_i rho0 and g_i - w'_i B_ref (the small dynamic part
    // keeps its digits); FP64 stores the populations themselves, so
    // natural-layout state IO round-trips exactly.
    L->rho0 = p->dtype == LBM_FP64 ? 0.0 : p->rho0;
    L->bref[0] = p->dtype == LBM_FP64 ? 0.0 : p->bref_x;
    L->bref[1] = p->dtype == LBM_FP64 ? 0.0 : p->bref_y;
  }
  return LBM_OK;
}

bool aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 255u) == 0; }

int check_ctx(const lbm_ctx* ctx, bool need_state) {
  if (!ctx) return fail(LBM_EINVAL, "context is NULL");
  if (need_state && !ctx->initialized)
    return fail(LBM_ESTATE, "state not initialised: call lbm_init_kh_jet or lbm_set_state first");
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_state_bytes(const lbm_params* p) {
  if (check_params(p, nullptr) != LBM_OK) return 0;
  return lbm::state_bytes(p->nx, p->ny, p->dtype, p->schedule, p->mag_lattice == LBM_MAG_D2Q9 ? 9 : 5);
}

size_t lbm_work_bytes(const lbm_params* p) {
  lbm::Launch L;
  if (check_params(p, &L) != LBM_OK) return 0;
  return lbm::work_layout(L);
}

int lbm_create(lbm_ctx** out, const lbm_params* p, void* state_dev, void* work_dev, void* hip_stream) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm::Launch L;
  int rc = check_params(p, &L);
  if (rc != LBM_OK) return rc;
  if (!state_dev || !work_dev) return fail(LBM_EINVAL, "state and work buffers must not be NULL");
  if (!aligned(state_dev) || !aligned(work_dev)) return fail(LBM_EINVAL, "device buffers must be 256-byte aligned");
  lbm::work_layout(L);
  L.state = state_dev;
  L.work = work_dev;
  L.stream = static_cast<hipStream_t>(hip_stream);
  lbm_ctx* ctx = new (std::nothrow) lbm_ctx;
  if (!ctx) return fail(LBM_EINVAL, "out of host memory");
  ctx->p = *p;
  ctx->L = L;
  *out = ctx;
  return LBM_OK;
}

int lbm_init_kh_jet(lbm_ctx* ctx, const lbm_kh_params* kh) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!kh) return fail(LBM_EINVAL, "kh params are NULL");
  const double vals[6] = {kh->U0, kh->delta_over_L, kh->B0, kh->rho0, kh->pert_amp_over_U0, kh->noise_amp};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(LBM_EINVAL, "kh params must be finite");
  if (!(kh->delta_over_L > 0.0) || !(kh->rho0 > 0.0))
    return fail(LBM_EINVAL, "delta_over_L and rho0 must be > 0");
  hipError_t e = lbm::launch_init_kh(ctx->L, *kh);
  if (e != hipSuccess) return hip_fail(e, "lbm_init_kh_jet");
  ctx->t = 0;
  ctx->initialized = true;
  ctx->lag_ready = false;
  ctx->corr_ready = false;
  return LBM_OK;
}

int lbm_init_sech2_jet(lbm_ctx* ctx, const lbm_sech2_params* jet) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!jet) return fail(LBM_EINVAL, "jet params are NULL");
  const double vals[4] = {jet->U0, jet->B0, jet->pert, jet->rho0};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(LBM_EINVAL, "jet params must be finite");
  if (!(jet->rho0 > 0.0) || jet->k < 1 || jet->reserved != 0)
    return fail(LBM_EINVAL, "rho0 must be > 0, k >= 1 and reserved 0");
  hipError_t e = lbm::launch_init_sech2(ctx->L, *jet);
  if (e != hipSuccess) return hip_fail(e, "lbm_init_sech2_jet");
  ctx->t = 0;
  ctx->initialized = true;
  ctx->lag_ready = false;
  ctx->corr_ready = false;
  return LBM_OK;
}

int lbm_init_from_moments(lbm_ctx* ctx, const double* mom_dev, int64_t t) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!mom_dev || !aligned(mom_dev)) return fail(LBM_EINVAL, "mom_dev must be a non-NULL 256-byte aligned pointer");
  if (t < 0) return fail(LBM_EINVAL, "t must be >= 0");
  hipError_t e = lbm::launch_init_moments(ctx->L, t, mom_dev);
  if (e != hipSuccess) return hip_fail(e, "lbm_init_from_moments");
  ctx->t = t;
  ctx->initialized = true;
  ctx->lag_ready = false;
  ctx->corr_ready = false;
  return LBM_OK;
}

int lbm_step(lbm_ctx* ctx, int64_t n) {
  int rc = check_ctx(ctx, true);
  if (rc != LBM_OK) return rc;
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (ctx->L.learned && !ctx->mlp_set)
    return fail(LBM_ESTATE, "learned closure: install a network with lbm_set_closure_mlp first");
  if (n > 0 && !ctx->cus_known) {
    // launch shapes depend on the compute-unit count of the current device
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      ctx->L.cus = cus;
    ctx->cus_known = true;
  }
  if (n > 0 && ctx->L.schedule == LBM_SCHED_AA_LAGGED && ctx->L.k2 != 0.0 && !ctx->lag_ready) {
    hipError_t e = lbm::launch_lag_prime(ctx->L, ctx->t);
    if (e != hipSuccess) return hip_fail(e, "lbm_step");
    ctx->lag_ready = true;
  }
  for (int64_t k = 0; k < n; ++k) {
    const bool refresh = !ctx->corr_ready || ctx->t % ctx->corr_every == 0;
    hipError_t e = lbm::launch_step(ctx->L, ctx->t, refresh);
    if (e != hipSuccess) return hip_fail(e, "lbm_step");
    ctx->corr_ready = ctx->L.learned;
    ++ctx->t;
  }
  return LBM_OK;
}

int lbm_get_time(const lbm_ctx* ctx, int64_t* t_out) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!t_out) return fail(LBM_EINVAL, "t_out is NULL");
  *t_out = ctx->t;
  return LBM_OK;
}

int lbm_moments(lbm_ctx* ctx, double* out_dev) {
  int rc = check_ctx(ctx, true);
  if (rc != LBM_OK) return rc;
  if (!out_dev || !aligned(out_dev)) return fail(LBM_EINVAL, "out_dev must be a non-NULL 256-byte aligned pointer");
  hipError_t e = lbm::launch_moments(ctx->L, ctx->t, out_dev, false);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments");
}

int lbm_get_state(lbm_ctx* ctx, double* out_dev) {
  int rc = check_ctx(ctx, true);
  if (rc != LBM_OK) return rc;
  if (!out_dev || !aligned(out_dev)) return fail(LBM_EINVAL, "out_dev must be a non-NULL 256-byte aligned pointer");
  hipError_t e = lbm::launch_get_state(ctx->L, ctx->t, out_dev);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_get_state");
}

int lbm_set_state(lbm_ctx* ctx, const double* in_dev, int64_t t) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!in_dev || !aligned(in_dev)) return fail(LBM_EINVAL, "in_dev must be a non-NULL 256-byte aligned pointer");
  if (t < 0) return fail(LBM_EINVAL, "t must be >= 0");
  hipError_t e = lbm::launch_set_state(ctx->L, t, in_dev);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_state");
  ctx->t = t;
  ctx->initialized = true;
  ctx->lag_ready = false;
  ctx->corr_ready = false;
  return LBM_OK;
}

int lbm_diagnostics(lbm_ctx* ctx, lbm_diag* out_host) {
  int rc = check_ctx(ctx, true);
  if (rc != LBM_OK) return rc;
  if (!out_host) return fail(LBM_EINVAL, "out_host is NULL");
  double v[lbm::kDiagVals];
  hipError_t e = lbm::launch_diagnostics(ctx->L, ctx->t, v);
  if (e != hipSuccess) return hip_fail(e, "lbm_diagnostics");
  const double n = double(ctx->L.nx) * double(ctx->L.ny);
  out_host->t = ctx->t;
  out_host->mass = v[0];
  out_host->mom_x = v[1];
  out_host->mom_y = v[2];
  out_host->bsum_x = v[3];
  out_host->bsum_y = v[4];
  out_host->e_kin = v[5] / n;
  out_host->e_mag = v[6] / n;
  out_host->enstrophy = v[7] / n;
  out_host->j2 = v[8] / n;
  out_host->divb_rms = std::sqrt(v[9] / n);
  out_host->divb_max = v[10];
  out_host->nonfinite = (int64_t)v[11];
  if (out_host->nonfinite > 0) return fail(LBM_ENONFINITE, "state holds non-finite populations");
  return LBM_OK;
}

int lbm_set_closure_mlp(lbm_ctx* ctx, const void* packed_dev) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!ctx->L.learned) return fail(LBM_ESTATE, "context was not created with closure = LBM_CLOSURE_LEARNED");
  if (!packed_dev || !aligned(packed_dev))
    return fail(LBM_EINVAL, "packed_dev must be a non-NULL 256-byte aligned pointer");
  hipError_t e = hipMemcpyAsync(static_cast<char*>(ctx->L.work) + ctx->L.off_mlp, packed_dev, LBM_MLP_PACKED_BYTES,
                                hipMemcpyDeviceToDevice, ctx->L.stream);
  if (e != hipSuccess) return hip_fail(e, "lbm_set_closure_mlp");
  ctx->mlp_set = true;
  ctx->corr_ready = false;
  return LBM_OK;
}

int lbm_set_correction_interval(lbm_ctx* ctx, int32_t every) {
  int rc = check_ctx(ctx, false);
  if (rc != LBM_OK) return rc;
  if (!ctx->L.learned) return fail(LBM_ESTATE, "context was not created with closure = LBM_CLOSURE_LEARNED");
  if (every < 1) return fail(LBM_EINVAL, "every must be >= 1");
  ctx->corr_every = every;
  ctx->corr_ready = false;
  return LBM_OK;
}

int lbm_closure_correction(lbm_ctx* ctx, float* out_dev) {
  int rc = check_ctx(ctx, true);
  if (rc != LBM_OK) return rc;
  if (!ctx->L.learned || !ctx->mlp_set)
    return fail(LBM_ESTATE, "needs closure = LBM_CLOSURE_LEARNED and an installed network");
  if (!out_dev || !aligned(out_dev)) return fail(LBM_EINVAL, "out_dev must be a non-NULL 256-byte aligned pointer");
  hipError_t e = lbm::launch_correction(ctx->L, ctx->t, out_dev);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_closure_correction");
}

// ---------------------------------------------------------------------------
// Learned closure, filtered DNS and spectra (lbmhd_learned.h)
// ---------------------------------------------------------------------------

int lbm_mlp_pack(const float* params_dev, const lbm_mlp_norm* norm_dev, void* packed_dev, void* hip_stream) {
  if (!params_dev || !norm_dev || !packed_dev || !aligned(params_dev) || !aligned(norm_dev) || !aligned(packed_dev))
    return fail(LBM_EINVAL, "params, norm and packed must be non-NULL 256-byte aligned device pointers");
  hipError_t e = lbm::launch_mlp_pack(params_dev, norm_dev, packed_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_pack");
}

int lbm_mlp_forward(const void* packed_dev, const float* x_dev, int64_t n, float* y_dev, int32_t* ood_dev,
                    void* hip_stream) {
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  if (!packed_dev || !x_dev || !y_dev || !aligned(packed_dev) || !aligned(x_dev) || !aligned(y_dev) ||
      (ood_dev && !aligned(ood_dev)))
    return fail(LBM_EINVAL, "packed, x, y (and ood if given) must be non-NULL 256-byte aligned device pointers");
  hipError_t e = lbm::launch_mlp_forward(packed_dev, x_dev, n, y_dev, ood_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_forward");
}

size_t lbm_mlp_stats_work_bytes(int64_t n) { return n >= 2 ? lbm::mlp_stats_work_bytes() : 0; }

int lbm_mlp_feature_stats(const float* x_dev, const float* t_dev, int64_t n, lbm_mlp_norm* norm_dev, void* work_dev,
                          size_t work_bytes, void* hip_stream) {
  if (n < 2) return fail(LBM_EINVAL, "n must be >= 2");
  if (!x_dev || !t_dev || !norm_dev || !work_dev || !aligned(x_dev) || !aligned(t_dev) || !aligned(norm_dev) ||
      !aligned(work_dev))
    return fail(LBM_EINVAL, "x, t, norm and work must be non-NULL 256-byte aligned device pointers");
  if (work_bytes < lbm::mlp_stats_work_bytes()) return fail(LBM_EINVAL, "work buffer too small");
  hipError_t e = lbm::launch_mlp_stats(x_dev, t_dev, n, norm_dev, work_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_feature_stats");
}

size_t lbm_mlp_train_work_bytes(int32_t batch) {
  return (batch >= 1 && batch <= (1 << 20)) ? lbm::mlp_train_work_bytes(batch) : 0;
}

int lbm_mlp_gradient(const float* params_dev, const lbm_mlp_norm* norm_dev, const float* x_dev, const float* t_dev,
                     const int32_t* idx_dev, int32_t batch, void* work_dev, size_t work_bytes, float* grad_dev,
                     float* loss_dev, void* hip_stream) {
  if (batch < 1 || batch > (1 << 20)) return fail(LBM_EINVAL, "batch must lie in [1, 2^20]");
  const void* ptrs[] = {params_dev, norm_dev, x_dev, t_dev, idx_dev, work_dev, grad_dev};
  for (const void* q : ptrs)
    if (!q || !aligned(q)) return fail(LBM_EINVAL, "device pointers must be non-NULL and 256-byte aligned");
  if (work_bytes < lbm::mlp_train_work_bytes(batch)) return fail(LBM_EINVAL, "work buffer too small");
  hipError_t e = lbm::launch_mlp_gradient(params_dev, norm_dev, x_dev, t_dev, idx_dev, batch, work_dev, grad_dev,
                                          loss_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_gradient");
}

int lbm_mlp_adam(float* params_dev, float* adam_m_dev, float* adam_v_dev, const float* grad_dev, int64_t step,
                 double lr, void* hip_stream) {
  if (step < 1) return fail(LBM_EINVAL, "step must be >= 1");
  if (!std::isfinite(lr) || lr <= 0.0) return fail(LBM_EINVAL, "lr must be finite and > 0");
  const void* ptrs[] = {params_dev, adam_m_dev, adam_v_dev, grad_dev};
  for (const void* q : ptrs)
    if (!q || !aligned(q)) return fail(LBM_EINVAL, "device pointers must be non-NULL and 256-byte aligned");
  hipError_t e = lbm::launch_mlp_adam(params_dev, adam_m_dev, adam_v_dev, grad_dev, step, lr,
                                      static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_adam");
}

int lbm_mlp_train_step(float* params_dev, float* adam_m_dev, float* adam_v_dev, int64_t step, double lr,
                       const lbm_mlp_norm* norm_dev, const float* x_dev, const float* t_dev, const int32_t* idx_dev,
                       int32_t batch, void* work_dev, size_t work_bytes, float* loss_dev, void* hip_stream) {
  if (batch < 1 || batch > (1 << 20)) return fail(LBM_EINVAL, "batch must lie in [1, 2^20]");
  if (step < 1) return fail(LBM_EINVAL, "step must be >= 1");
  if (!std::isfinite(lr) || lr <= 0.0) return fail(LBM_EINVAL, "lr must be finite and > 0");
  const void* ptrs[] = {params_dev, adam_m_dev, adam_v_dev, norm_dev, x_dev, t_dev, idx_dev, work_dev};
  for (const void* q : ptrs)
    if (!q || !aligned(q)) return fail(LBM_EINVAL, "device pointers must be non-NULL and 256-byte aligned");
  if (work_bytes < lbm::mlp_train_work_bytes(batch)) return fail(LBM_EINVAL, "work buffer too small");
  hipError_t e = lbm::launch_mlp_train(params_dev, adam_m_dev, adam_v_dev, step, lr, norm_dev, x_dev, t_dev, idx_dev,
                                       batch, work_dev, loss_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_train_step");
}

int lbm_mlp_train_step_noalloc(float* params_dev, float* adam_m_dev, float* adam_v_dev, int64_t step, double lr,
                               const lbm_mlp_norm* norm_dev, const float* x_dev, const float* t_dev,
                               const int32_t* idx_dev, int32_t batch, float* loss_dev, void* hip_stream) {
  if (batch < 1 || batch > LBM_MLP_TRAIN_NOALLOC_BATCH || !lbm::mlp_train_noalloc_limit_ok(batch))
    return fail(LBM_EINVAL, "batch must lie in [1, LBM_MLP_TRAIN_NOALLOC_BATCH = 16384] without a work buffer");
  if (step < 1) return fail(LBM_EINVAL, "step must be >= 1");
  if (!std::isfinite(lr) || lr <= 0.0) return fail(LBM_EINVAL, "lr must be finite and > 0");
  const void* ptrs[] = {params_dev, adam_m_dev, adam_v_dev, norm_dev, x_dev, t_dev, idx_dev};
  for (const void* q : ptrs)
    if (!q || !aligned(q)) return fail(LBM_EINVAL, "device pointers must be non-NULL and 256-byte aligned");
  hipError_t e = lbm::launch_mlp_train_noalloc(params_dev, adam_m_dev, adam_v_dev, step, lr, norm_dev, x_dev, t_dev,
                                               idx_dev, batch, loss_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_mlp_train_step_noalloc");
}

namespace {
int check_filter(int32_t nx, int32_t ny, int32_t factor, double delta) {
  if (nx < 4 || ny < 4 || nx > 32768 || ny > 32768) return fail(LBM_EINVAL, "nx and ny must lie in [4, 32768]");
  if (factor != 1 && factor != 2 && factor != 4 && factor != 8 && factor != 16)
    return fail(LBM_EINVAL, "factor must be 1, 2, 4, 8 or 16");
  if (nx % factor || ny % factor) return fail(LBM_EINVAL, "factor must divide nx and ny");
  if (!std::isfinite(delta) || delta <= 0.0) return fail(LBM_EINVAL, "delta must be finite and > 0");
  const int R = lbm::filter_radius(delta);
  if (R > 127 || R >= nx || R >= ny) return fail(LBM_EINVAL, "filter radius ceil(5 delta / sqrt(12)) too large");
  return LBM_OK;
}
}  // namespace

size_t lbm_filter_work_bytes(int32_t nx, int32_t ny, int32_t factor, double delta) {
  if (check_filter(nx, ny, factor, delta) != LBM_OK) return 0;
  return lbm::filter_work_bytes(nx, ny, factor);
}

int lbm_filter_subsample(const double* mom_dev, int32_t nx, int32_t ny, int32_t factor, double delta,
                         double* out_dev, void* work_dev, size_t work_bytes, void* hip_stream) {
  int rc = check_filter(nx, ny, factor, delta);
  if (rc != LBM_OK) return rc;
  if (!mom_dev || !out_dev || !work_dev || !aligned(mom_dev) || !aligned(out_dev) || !aligned(work_dev))
    return fail(LBM_EINVAL, "mom, out and work must be non-NULL 256-byte aligned device pointers");
  if (work_bytes < lbm::filter_work_bytes(nx, ny, factor)) return fail(LBM_EINVAL, "work buffer too small");
  hipError_t e =
      lbm::launch_filter(mom_dev, nx, ny, factor, delta, out_dev, work_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_filter_subsample");
}

int lbm_closure_samples(const double* coarse_dev, int32_t nx, int32_t ny, double delta, int32_t grad_stencil,
                        float* x_dev, float* t_dev, void* hip_stream) {
  if (nx < 4 || ny < 4 || nx > 32768 || ny > 32768) return fail(LBM_EINVAL, "nx and ny must lie in [4, 32768]");
  if (!std::isfinite(delta) || delta < 0.0) return fail(LBM_EINVAL, "delta must be finite and >= 0");
  if (grad_stencil != LBM_STENCIL_ISO9 && grad_stencil != LBM_STENCIL_CENTRAL5)
    return fail(LBM_EINVAL, "grad_stencil must be LBM_STENCIL_ISO9 or LBM_STENCIL_CENTRAL5");
  if (!coarse_dev || !x_dev || !t_dev || !aligned(coarse_dev) || !aligned(x_dev) || !aligned(t_dev))
    return fail(LBM_EINVAL, "coarse, x and t must be non-NULL 256-byte aligned device pointers");
  hipError_t e = lbm::launch_closure_samples(coarse_dev, nx, ny, delta, grad_stencil, x_dev, t_dev,
                                             static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_closure_samples");
}

namespace {
bool spectra_n_ok(int32_t n) { return n >= 8 && n <= 16384 && (n & (n - 1)) == 0; }
}  // namespace

int32_t lbm_spectra_bins(int32_t n) { return spectra_n_ok(n) ? lbm::spectra_bins(n) : 0; }

size_t lbm_spectra_work_bytes(int32_t n) { return spectra_n_ok(n) ? lbm::spectra_work_bytes(n) : 0; }

int lbm_spectra(const double* mom_dev, int32_t n, double* ek_dev, double* em_dev, double* ekx_dev, void* work_dev,
                size_t work_bytes, void* hip_stream) {
  if (!spectra_n_ok(n)) return fail(LBM_EINVAL, "n must be a power of two in [8, 16384]");
  if (!mom_dev || !ek_dev || !em_dev || !work_dev || !aligned(mom_dev) || !aligned(ek_dev) || !aligned(em_dev) ||
      !aligned(work_dev) || (ekx_dev && !aligned(ekx_dev)))
    return fail(LBM_EINVAL, "mom, ek, em, work (and ekx if given) must be non-NULL 256-byte aligned device pointers");
  if (work_bytes < lbm::spectra_work_bytes(n)) return fail(LBM_EINVAL, "work buffer too small");
  hipError_t e =
      lbm::launch_spectra(mom_dev, n, ek_dev, em_dev, ekx_dev, work_dev, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_spectra");
}

int lbm_destroy(lbm_ctx* ctx) {
  delete ctx;
  return LBM_OK;
}

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "success";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ESTATE: return "invalid call order";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite state";
    default: return "unknown error";
  }
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
