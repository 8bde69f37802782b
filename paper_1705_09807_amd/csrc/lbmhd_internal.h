// Internal interface between the C ABI (lbmhd_api.cpp) and the kernel
// launchers (lbmhd_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbmhd.h"
#include "lbmhd_learned.h"

namespace lbm {

constexpr int kQ = 19;            // 9 (f) + 5 (g_x) + 5 (g_y) populations per cell (D2Q5 g;
                                  // 9 + 9 + 9 with the D2Q9 vector distribution)
constexpr int kDiagVals = 12;     // accumulators of the diagnostics reduction
constexpr int kDiagBlocksMax = 2048;

// Everything a launcher needs; filled once by lbm_create.
struct Launch {
  int nx = 0, ny = 0;
  int64_t pitch = 0;              // elements from one population row to the next within a
                                  // lattice row (>= nx; a lattice row holds 9 + 2 qg of them)
  int dtype = LBM_FP64;
  int schedule = LBM_SCHED_FUSED;
  int stencil = LBM_STENCIL_ISO9;
  int qg = 5;                     // velocities of the vector distribution: 5 (D2Q5) or 9 (D2Q9)
  int cus = 256;                  // compute units of the device (queried at the first step)
  double rate[9] = {0};           // MRT rates s0..s8 (s0..s2 = 0)
  double sm = 0;                  // magnetic SRT rate
  double k2 = 0;                  // closure_scale * Delta^2 / 12
  double rho0 = 1;                // rest density subtracted from stored f (0 for FP64)
  double bref[2] = {0, 0};        // reference field subtracted from stored g (0 for FP64)
  void* state = nullptr;          // caller-owned population storage
  void* work = nullptr;           // caller-owned work buffer
  size_t off_mb = 0;              // moment planes for the in-place closure sweep
                                  // (two sets for the lagged schedule, set t & 1
                                  // holding the moments of step t - 1)
  size_t off_diag = 0;            // 5 FP64 moment planes for the diagnostics
  size_t off_part = 0;            // per-block reduction partials
  size_t off_final = 0;           // final reduction values
  int diag_blocks = 0;
  bool learned = false;           // analytic closure plus the network's correction
  bool full = false;              // closure with the filtered-density gradient terms
  size_t off_cellin = 0;          // network input vectors (16 bytes per cell)
  size_t off_corr = 0;            // 4 FP32 correction planes
  size_t off_mlp = 0;             // packed network
  hipStream_t stream = nullptr;
};

// Layout helpers (host).
size_t storage_bytes(int dtype);
int64_t row_pitch(int nx);
// Elements of one population buffer: ny lattice rows of (9 + 2 qg) population
// rows each, element (q, x, y) at (y * (9 + 2 qg) + q) * pitch + x.
int64_t buffer_elems(int nx, int ny, int qg);
// Byte offset of the second population buffer of the fused schedule.
size_t buffer_offset_bytes(int nx, int ny, int dtype, int qg);
size_t state_bytes(int nx, int ny, int dtype, int schedule, int qg);
// Work layout for the given geometry; returns total bytes and fills offsets.
size_t work_layout(Launch& L);

// Launchers: enqueue on L.stream, return the first HIP error.
hipError_t launch_init_kh(const Launch& L, const lbm_kh_params& kh);
hipError_t launch_init_sech2(const Launch& L, const lbm_sech2_params& jet);
hipError_t launch_init_moments(const Launch& L, int64_t t, const double* mom);
// State at time t -> t + 1; with the learned closure, corr_refresh = false
// reuses the correction planes of an earlier step instead of evaluating the
// network on this state.
hipError_t launch_step(const Launch& L, int64_t t, bool corr_refresh = true);
// Lagged schedule: moments of the state at time t into moment set t & 1.
hipError_t launch_lag_prime(const Launch& L, int64_t t);
hipError_t launch_get_state(const Launch& L, int64_t t, double* out);
hipError_t launch_set_state(const Launch& L, int64_t t, const double* in);
hipError_t launch_moments(const Launch& L, int64_t t, double* out, bool mark_nonfinite);
// Diagnostics: enqueue, copy kDiagVals doubles to host, synchronise the stream.
hipError_t launch_diagnostics(const Launch& L, int64_t t, double* vals_host);
// Learned correction of the state at time t into 4 FP32 planes.
hipError_t launch_correction(const Launch& L, int64_t t, float* out);

// Learned closure, filtered DNS and spectra (lbmhd_learned.hip).
hipError_t launch_mlp_pack(const float* params, const lbm_mlp_norm* norm, void* packed, hipStream_t st);
hipError_t launch_mlp_forward(const void* packed, const float* x, int64_t n, float* y, int32_t* ood, hipStream_t st);
size_t mlp_train_work_bytes(int batch);
hipError_t launch_mlp_gradient(const float* params, const lbm_mlp_norm* norm, const float* x, const float* t,
                               const int32_t* idx, int batch, void* work, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, double lr,
                           hipStream_t st);
hipError_t launch_mlp_train(float* params, float* m, float* v, int64_t step, double lr, const lbm_mlp_norm* norm,
                            const float* x, const float* t, const int32_t* idx, int batch, void* work, float* loss,
                            hipStream_t st);
// The same step with its work in the library's fixed per-device array
// (batch <= LBM_MLP_TRAIN_NOALLOC_BATCH; hipErrorInvalidValue beyond).
bool mlp_train_noalloc_limit_ok(int batch);
hipError_t launch_mlp_train_noalloc(float* params, float* m, float* v, int64_t step, double lr,
                                    const lbm_mlp_norm* norm, const float* x, const float* t, const int32_t* idx,
                                    int batch, float* loss, hipStream_t st);
size_t mlp_stats_work_bytes();
hipError_t launch_mlp_stats(const float* x, const float* t, int64_t n, lbm_mlp_norm* norm, void* work,
                            hipStream_t st);
int filter_radius(double delta);
size_t filter_work_bytes(int nx, int ny, int factor);
hipError_t launch_filter(const double* mom, int nx, int ny, int factor, double delta, double* out, void* work,
                         hipStream_t st);
hipError_t launch_closure_samples(const double* c12, int nx, int ny, double delta, int stencil, float* x, float* t,
                                  hipStream_t st);
// The network on per-cell input vectors (16 bytes per cell, written by the
// first stage of launch_correction).
hipError_t launch_mlp_correct(const void* cell_in, const void* packed, float* corr, int nx, int ny, hipStream_t st);
int spectra_bins(int n);
size_t spectra_work_bytes(int n);
hipError_t launch_spectra(const double* mom, int n, double* ek, double* em, double* ekx, void* work,
                          hipStream_t st);

}  // namespace lbm
