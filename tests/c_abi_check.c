/* Plain C99 client of the C ABI: plans, validation codes and status strings,
 * no device memory and no kernel launch (runs without a GPU). Built and run by
 * tests/test_abi.py; exits 0 when every check holds. */
#include <stdio.h>
#include <string.h>

#include "traknn.h"

static int failures = 0;
#define CHECK(cond)                                             \
  do {                                                          \
    if (!(cond)) {                                              \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                               \
    }                                                           \
  } while (0)

int main(void) {
  traknn_config c;
  memset(&c, 0, sizeof c);
  c.T = 27394;
  c.D = 8192;
  c.L_min = 5;
  c.L_max = 5;
  c.k = 10;
  c.precision = TRAKNN_BF16X3;
  c.row_batch = 0;
  traknn_plan_t p = NULL;
  size_t ws = 0;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_OK);
  CHECK(p != NULL);
  /* the whole distance matrix dominates the workspace */
  CHECK(ws >= (size_t)27394 * 27456 * 4);
  CHECK(traknn_plan_destroy(p) == TRAKNN_OK);

  /* band mode holds a band of the matrix */
  size_t ws_band = 0;
  c.row_batch = 4088;
  CHECK(traknn_plan(&c, &p, &ws_band) == TRAKNN_OK);
  CHECK(ws_band < ws / 2);
  CHECK(traknn_plan_destroy(p) == TRAKNN_OK);

  /* rejected configurations, with the documented codes */
  c.row_batch = 12;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_ERR_INVALID_ARG && p == NULL);
  c.row_batch = 0;
  c.k = 0;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_ERR_INVALID_ARG);
  c.k = 10;
  c.L_min = 2;
  c.L_max = 4;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_ERR_UNSUPPORTED);
  c.L_min = 5;
  c.precision = 7;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_ERR_INVALID_ARG);
  /* FP64 only in fused mode; the fused mode holds no distance matrix */
  c.L_max = 5;
  c.precision = TRAKNN_FP64;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_ERR_UNSUPPORTED);
  c.mode = TRAKNN_MODE_FUSED;
  size_t ws_fused = 0;
  CHECK(traknn_plan(&c, &p, &ws_fused) == TRAKNN_OK);
  CHECK(ws_fused < (size_t)27394 * 27456 * 4 / 3);
  CHECK(traknn_plan_destroy(p) == TRAKNN_OK);
  c.mode = 5;
  CHECK(traknn_plan(&c, &p, &ws) == TRAKNN_ERR_INVALID_ARG);
  c.mode = TRAKNN_MODE_MATRIX;
  c.precision = TRAKNN_BF16X3;
  CHECK(traknn_plan(NULL, &p, &ws) == TRAKNN_ERR_INVALID_ARG);

  /* calls on a NULL plan enqueue nothing */
  CHECK(traknn_knn(NULL, NULL, 0, NULL, 0, NULL, NULL, NULL) == TRAKNN_ERR_INVALID_ARG);
  CHECK(traknn_score(NULL, NULL, NULL, NULL) == TRAKNN_ERR_INVALID_ARG);
  CHECK(traknn_score_prefix(NULL, NULL, NULL, NULL) == TRAKNN_ERR_INVALID_ARG);
  CHECK(traknn_local_dim(NULL, NULL, NULL, NULL) == TRAKNN_ERR_INVALID_ARG);
  CHECK(traknn_score_backward(NULL, NULL, 0, NULL, NULL, NULL, 0, NULL, 0, NULL) ==
        TRAKNN_ERR_INVALID_ARG);
  CHECK(traknn_plan_destroy(NULL) == TRAKNN_ERR_INVALID_ARG);

  CHECK(strcmp(traknn_status_string(TRAKNN_OK), "ok") == 0);
  CHECK(traknn_status_string(-99) != NULL);

  if (failures) return 1;
  printf("c abi ok\n");
  return 0;
}
