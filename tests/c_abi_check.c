/* The ABI as a C caller sees it: the headers compile as C99 and the host-only
 * calls (sizes, parameter validation, context life cycle with placeholder
 * device pointers, error strings) behave as documented.  No device work is
 * enqueued.  Exit status 0 on success; prints the first failed check. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lbmhd.h"
#include "lbmhd_learned.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      printf("check failed at line %d: %s\n", __LINE__, #c);       \
      return 1;                                                    \
    }                                                              \
  } while (0)

static lbm_params params(void) {
  lbm_params p;
  memset(&p, 0, sizeof p);
  p.nx = 64;
  p.ny = 48;
  p.nu = 1e-3;
  p.eta = 2e-3;
  p.delta = 2.0;
  p.closure_scale = 1.0;
  p.grad_stencil = LBM_STENCIL_ISO9;
  p.dtype = LBM_FP32;
  p.schedule = LBM_SCHED_FUSED;
  p.closure = LBM_CLOSURE_ANALYTIC;
  p.mag_lattice = LBM_MAG_D2Q5;
  p.rho0 = 1.0;
  p.bref_x = 0.01;
  return p;
}

int main(void) {
  lbm_params p = params();
  /* one buffer: 48 lattice rows of 19 (27) population rows of 64 elements;
     the second starts 4 KB past the 64 KB boundary after the first */
  CHECK(lbm_state_bytes(&p) == 4 * 65536 + 4096 + (size_t)(48 * 19 * 64) * 4);
  p.mag_lattice = LBM_MAG_D2Q9;
  CHECK(lbm_state_bytes(&p) == 6 * 65536 + 4096 + (size_t)(48 * 27 * 64) * 4);
  p.schedule = LBM_SCHED_AA;
  CHECK(lbm_state_bytes(&p) == 0);  /* D2Q9 g runs with the fused schedule only */
  CHECK(strlen(lbm_last_error()) > 0);
  p = params();
  CHECK(lbm_work_bytes(&p) > 0);
  p.nu = -1.0;
  CHECK(lbm_state_bytes(&p) == 0);
  p = params();

  lbm_ctx* ctx = NULL;
  CHECK(lbm_create(&ctx, &p, (void*)(uintptr_t)(1u << 20), (void*)(uintptr_t)(1u << 21), NULL) == LBM_OK);
  CHECK(ctx != NULL);
  int64_t t = -1;
  CHECK(lbm_get_time(ctx, &t) == LBM_OK && t == 0);
  CHECK(lbm_step(ctx, 1) == LBM_ESTATE);  /* no initial state yet */
  CHECK(lbm_init_kh_jet(ctx, NULL) == LBM_EINVAL);
  CHECK(lbm_init_sech2_jet(ctx, NULL) == LBM_EINVAL);
  CHECK(lbm_destroy(ctx) == LBM_OK);
  CHECK(lbm_create(&ctx, &p, (void*)(uintptr_t)((1u << 20) + 8), (void*)(uintptr_t)(1u << 21), NULL) == LBM_EINVAL);

  CHECK(lbm_spectra_bins(64) > 0 && lbm_spectra_bins(63) == 0);
  CHECK(lbm_mlp_train_work_bytes(0) == 0 && lbm_mlp_train_work_bytes(4096) > 0);
  CHECK(strcmp(lbm_strerror(LBM_OK), lbm_strerror(LBM_EINVAL)) != 0);
  CHECK(sizeof(lbm_params) == 2 * 4 + 8 * 8 + 6 * 4 + 3 * 8);
  printf("c abi ok\n");
  return 0;
}
