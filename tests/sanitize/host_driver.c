/* The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (its device
 * kernels are linked unsanitized and never launched: no device is needed).  Drives every entry
 * point whose work is host-side (operation tables, workspace sizes, argument checks, the
 * selector's cost model, features and choice, batched plans and the tuning controls) over
 * ragged, empty and large shapes, and checks a few invariants.  Exit status 0 when every check
 * holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/strassen.h"

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      fprintf(stderr, "FAIL line %d: %s\n", __LINE__, #c);          \
      ++failures;                                                   \
    }                                                               \
  } while (0)

int main(void) {
  EXPECT(strassen_version() && strlen(strassen_version()) > 0);

  /* operation tables */
  const int products[4] = {1, 7, 49, 343};
  for (int lv = 0; lv <= 3; ++lv) {
    EXPECT(strassen_table_size(lv) == products[lv]);
    for (int r = 0; r < products[lv]; ++r) {
      int na = 0, nb = 0, nc = 0, a[8], b[8], c[8];
      EXPECT(strassen_table_get(lv, r, &na, a, &nb, b, &nc, c) == 0);
      EXPECT(na >= 1 && na <= 8 && nb >= 1 && nb <= 8 && nc >= 1 && nc <= 8);
      const int blocks = 1 << (2 * lv);
      for (int i = 0; i < na; ++i) EXPECT(a[i] != 0 && abs(a[i]) <= blocks);
      for (int i = 0; i < nb; ++i) EXPECT(b[i] != 0 && abs(b[i]) <= blocks);
      for (int i = 0; i < nc; ++i) EXPECT(c[i] != 0 && abs(c[i]) <= blocks);
    }
  }
  {
    int na, nb, nc, t[8];
    EXPECT(strassen_table_size(4) == -1 && strassen_table_size(-1) == -1);
    EXPECT(strassen_table_get(1, 7, &na, t, &nb, t, &nc, t) == -2);
    EXPECT(strassen_table_get(5, 0, &na, t, &nb, t, &nc, t) == -1);
  }

  /* workspace sizes, the cost model, the selector's features and choice */
  const int64_t s[] = {0, 1, 2, 3, 7, 8, 63, 64, 65, 127, 128, 129, 1000, 4097, 16383, 20000, 65537};
  const int ns = (int)(sizeof s / sizeof s[0]);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j)
      for (int l = 0; l < ns; ++l) {
        const int64_t m = s[i], n = s[j], k = s[l];
        for (int lv = 0; lv <= 3; ++lv)
          for (int v = 0; v < 3; ++v) {
            size_t bytes = 1;
            const int rc = strassen_workspace_size(m, n, k, lv, v, &bytes);
            EXPECT(rc == 0 || (lv == 3 && v != STRASSEN_ABC && rc == -5));
            if (rc == 0 && v == STRASSEN_ABC && lv <= 2) {
              size_t w = 0;
              if (lv >= 1) EXPECT(strassen_workspace_size_winograd(m, n, k, lv, &w) == 0);
            }
          }
        for (int lv = 0; lv <= 2; ++lv)
          for (int cp = 0; cp <= 2; ++cp) {
            size_t bytes = 1;
            EXPECT(strassen_workspace_size_ex(m, n, k, lv, cp, &bytes) == 0);
            if (cp == 0) EXPECT(bytes == 0);
          }
        for (int d = 0; d <= 1; ++d) {
          double sec[7];
          float x[11];
          int lv = -1, var = -1;
          EXPECT(strassen_cost_model(m, n, k, d, sec) == 0);
          EXPECT(strassen_selector_features(m, n, k, d, x) == 0);
          EXPECT(strassen_select(m, n, k, d, &lv, &var) == 0);
          EXPECT(lv >= 0 && lv <= 2 && var >= 0 && var <= 2 && (d == 0 || var == STRASSEN_ABC));
          for (int c = 0; c < 7; ++c) EXPECT(x[4 + c] >= 0.0f && x[4 + c] <= 1.0f);
        }
      }
  EXPECT(strassen_workspace_size(-1, 1, 1, 1, 0, NULL) < 0);
  EXPECT(strassen_cost_model(1, 1, 1, 2, NULL) < 0);
  {
    size_t b;
    EXPECT(strassen_mlp_work_size(100, &b) == 0 && b > 0);
    EXPECT(strassen_mlp_work_size(-1, &b) == -1);
  }

  /* argument checks: rejected on the host, before any device call */
  double dummy[64];
  memset(dummy, 0, sizeof dummy);
  EXPECT(strassen_dgemm(-1, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 1, 0, NULL) == -1);
  EXPECT(strassen_dgemm(4, 4, 4, 1.0, dummy, 3, dummy, 4, 1.0, dummy, 4, 1, 0, NULL) == -6);
  EXPECT(strassen_dgemm(4, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 9, 0, NULL) == -12);
  EXPECT(strassen_dgemm(4, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 1, 7, NULL) == -13);
  EXPECT(strlen(strassen_last_error()) > 0);
  EXPECT(strassen_dgemm(0, 4, 4, 1.0, dummy, 1, dummy, 4, 1.0, dummy, 1, 1, 0, NULL) == 0);
  EXPECT(strassen_gemm('X', 'N', 4, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 1, 0, NULL) < 0);
  EXPECT(strassen_dgemm_winograd(4, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 3, NULL) < 0);
  EXPECT(strassen_dgemm_noalloc(-2, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 1, 0, NULL) == -1);
  EXPECT(strassen_gemm_ex(4, 4, 4, 1.0, dummy, 4, dummy, 4, 1.0, dummy, 4, 1, 0, 9, 0, 0, NULL) < 0);
  EXPECT(strassen_dgetrf_nopiv(8, dummy, 8, 48, 0, NULL) == -4);
  EXPECT(strassen_dgetrf_nopiv(8, dummy, 4, 64, 0, NULL) == -3);

  /* batched plans: the default rule over many shapes */
  {
    enum { N = 300 };
    int64_t m[N], n[N], k[N];
    for (int i = 0; i < N; ++i) {
      m[i] = 64 * (1 + (i * 7) % 64);
      n[i] = 64 * (1 + (i * 13) % 64);
      k[i] = (i % 5 == 0) ? 0 : 64 * (1 + (i * 29) % 64);
    }
    void *plan = NULL;
    EXPECT(strassen_batched_plan(N, m, n, k, NULL, NULL, &plan) == 0 && plan != NULL);
    for (int i = 0; i < N; ++i) {
      int lv = -1, cfg = -1;
      EXPECT(strassen_batched_choice(plan, i, &lv, &cfg) == 0);
      EXPECT(lv >= 0 && lv <= 2);
    }
    EXPECT(strassen_batched_choice(plan, N, NULL, NULL) < 0);
    EXPECT(strassen_batched_destroy(plan) == 0);
    EXPECT(strassen_batched_plan(-1, m, n, k, NULL, NULL, &plan) == -1);
  }

  /* tuning controls */
  for (int cfg = -1; cfg <= 6; ++cfg) EXPECT(strassen_set_tile_config(cfg) == 0);
  EXPECT(strassen_set_tile_config(7) == -1);
  EXPECT(strassen_set_tile_config(-1) == 0);
  EXPECT(strassen_set_workspace_limit((size_t)1 << 20) == 0);
  EXPECT(strassen_set_workspace_limit(0) == 0);
  EXPECT(strassen_set_workspace(NULL, 0) == 0);
  EXPECT(strassen_set_workspace(dummy + 1, 64) == -1);
  {
    float bad[5383];
    for (int i = 0; i < 5383; ++i) bad[i] = 0.0f;
    bad[17] = 1.0f / 0.0f;
    EXPECT(strassen_selector_load(bad) == -1);
    EXPECT(strassen_selector_load(NULL) == 0);
  }
  if (failures) return 1;
  printf("host checks passed\n");
  return 0;
}
