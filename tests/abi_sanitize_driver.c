/* Host-side paths of libwave that need no GPU, run under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitize.py): parameter
 * validation, workspace planning, create-time argument checks, variant
 * queries and null handles.  Exit status 0 when every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "wave.h"

#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);      \
      return 1;                                                             \
    }                                                                       \
  } while (0)

static void base(wave_params *p) {
  wave_params_init(p);
  p->nx = 16;
  p->ny = 12;
  p->nz = 10;
  p->dx = p->dy = p->dz = 10.0;
  p->dt = 1e-4;
}

int main(void) {
  wave_params p;
  size_t b0 = 0, b = 0;
  base(&p);
  CHECK(wave_workspace_bytes(&p, &b0) == WAVE_OK && b0 > 0 && b0 % 256 == 0);

  /* every invalid field is rejected before anything else happens */
  for (int k = 0; k < 14; ++k) {
    base(&p);
    switch (k) {
      case 0: p.nx = 0; break;
      case 1: p.dt = 0.0; break;
      case 2: p.storage = 7; break;
      case 3: p.sponge_width = -1; break;
      case 4: p.src[0] = 16; p.src[1] = 0; p.src[2] = 0; break;
      case 5: p.variant = 999; break;
      case 6: p.zchunk = -1; break;
      case 7: p.tune = 3; break;
      case 8: p.cpml_width = 6; break;           /* 2 W > nz */
      case 9: p.cpml_width = 2; p.sponge_width = 2; break;
      case 10: p.adjoint = 1; p.nt_max = 0; break;
      case 11: p.nx = 4097; p.ny = 4096; break;  /* plane above 2^24 nodes */
      case 12: p.nrec = 1; p.rec = NULL; break;
      case 13: p.cpml_width = 2; p.cpml_reflection = 2.0; break;
    }
    CHECK(wave_workspace_bytes(&p, &b) == WAVE_EINVAL);
  }

  /* receivers outside the grid */
  int32_t rec[6] = {1, 2, 3, 16, 0, 0};
  base(&p);
  p.nrec = 2;
  p.rec = rec;
  CHECK(wave_workspace_bytes(&p, &b) == WAVE_EINVAL);
  rec[3] = 15;
  CHECK(wave_workspace_bytes(&p, &b) == WAVE_OK && b >= b0);

  /* adjoint, 16-bit and CPML layouts grow or shrink the workspace as planned */
  base(&p);
  p.adjoint = 1;
  p.nt_max = 100;
  CHECK(wave_workspace_bytes(&p, &b) == WAVE_OK && b > b0);
  base(&p);
  p.storage = WAVE_F16;
  CHECK(wave_workspace_bytes(&p, &b) == WAVE_OK && b < b0);
  base(&p);
  p.cpml_width = 3;
  CHECK(wave_workspace_bytes(&p, &b) == WAVE_OK && b > b0);

  /* create: null, misaligned and short workspaces fail before any GPU call */
  wave_t w = NULL;
  static char fake[1 << 16];
  base(&p);
  CHECK(wave_create(&p, NULL, fake, sizeof(fake), NULL, &w) == WAVE_EINVAL && w == NULL);
  CHECK(wave_create(&p, (const float *)fake, fake + 1, sizeof(fake), NULL, &w) == WAVE_EINVAL);
  CHECK(wave_create(&p, (const float *)fake, (void *)(((uintptr_t)fake + 255) & ~(uintptr_t)255), 256, NULL, &w) ==
        WAVE_ENOSPC);
  p.nx = 0;
  CHECK(wave_create(&p, (const float *)fake, fake, sizeof(fake), NULL, &w) == WAVE_EINVAL);

  /* variants, status strings and null handles */
  const int nv = wave_variant_count();
  CHECK(nv >= 1);
  for (int v = 0; v < nv; ++v) {
    int32_t info[5];
    memset(info, 0xff, sizeof(info));
    CHECK(wave_variant_info(v, info) == WAVE_OK && info[1] >= 1 && info[4] >= 1);
  }
  int32_t info[5];
  CHECK(wave_variant_info(nv, info) == WAVE_EINVAL && wave_variant_info(0, NULL) == WAVE_EINVAL);
  for (int s = -6; s <= 0; ++s) CHECK(wave_status_string(s) != NULL && strlen(wave_status_string(s)) > 0);
  size_t sb;
  int32_t n;
  uint32_t f;
  CHECK(wave_destroy(NULL) == WAVE_EINVAL && wave_reset(NULL) == WAVE_EINVAL);
  CHECK(wave_state_bytes(NULL, &sb) == WAVE_EINVAL && wave_save_state(NULL, fake) == WAVE_EINVAL);
  CHECK(wave_load_state(NULL, fake) == WAVE_EINVAL && wave_time_index(NULL, &n) == WAVE_EINVAL);
  CHECK(wave_sync_status(NULL, &f) == WAVE_EINVAL && wave_step(NULL, 1, NULL, NULL) == WAVE_EINVAL);
  CHECK(wave_run(NULL, 1, NULL, NULL) == WAVE_EINVAL && wave_adjoint(NULL, 1, NULL, NULL, NULL) == WAVE_EINVAL);
  CHECK(wave_read_field(NULL, 0, NULL) == WAVE_EINVAL && wave_workspace_bytes(NULL, &b) == WAVE_EINVAL);
  CHECK(wave_write_field(NULL, 0, NULL) == WAVE_EINVAL);
  {
    wave_params q;
    double dtmax = 0.0;
    wave_params_init(&q);
    q.dx = q.dy = q.dz = 10.0;
    CHECK(wave_stable_dt(&q, 4500.0, &dtmax) == WAVE_OK && dtmax > 0.0);
    CHECK(wave_stable_dt(&q, -1.0, &dtmax) == WAVE_EINVAL && wave_stable_dt(NULL, 1.0, &dtmax) == WAVE_EINVAL);
  }
  int32_t tiling[3];
  CHECK(wave_tiling(NULL, tiling) == WAVE_EINVAL);
  wave_params_init(NULL);
  printf("sanitized host paths: ok\n");
  return 0;
}
