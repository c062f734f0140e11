/* Host-side driver for the sanitizer build of the library: exercises the C
 * ABI paths that need no GPU (parameter validation, index creation and
 * destruction, file parsing of missing, bad and truncated index files, calls
 * on an unbuilt index, the bucket table), so that AddressSanitizer and
 * UndefinedBehaviorSanitizer see the host code. Exit status 0 on success. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/rabitq.h"

#define CHECK(cond)                                             \
  do {                                                          \
    if (!(cond)) {                                              \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      return 1;                                                 \
    }                                                           \
  } while (0)

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : "/tmp";
  rbq_params p;
  CHECK(rbq_params_default(&p, 128, 16) == RBQ_OK);
  CHECK(p.bq == 4 && p.code_bits == 0);
  rbq_index* idx = NULL;
  CHECK(rbq_index_create(&p, &idx) == RBQ_OK && idx);
  rbq_index_info info;
  CHECK(rbq_index_info_get(idx, &info) == RBQ_OK && info.code_bits == 128 && info.n == 0);
  /* calls on an unbuilt index */
  rbq_search_opts o;
  memset(&o, 0, sizeof(o));
  o.k = 10;
  o.nprobe = 1;
  CHECK(rbq_search(idx, NULL, 1, &o, NULL, NULL, NULL, NULL) == RBQ_ESTATE);
  int64_t sizes[16];
  CHECK(rbq_index_list_sizes(idx, sizes) == RBQ_ESTATE);
  char path[512];
  snprintf(path, sizeof(path), "%s/never.rbq", dir);
  CHECK(rbq_index_save(idx, path) == RBQ_ESTATE);
  CHECK(rbq_index_set_eps0(idx, -1.f) == RBQ_EINVAL);
  CHECK(rbq_index_set_eps0(idx, 2.5f) == RBQ_OK);
  CHECK(rbq_index_destroy(idx) == RBQ_OK);
  CHECK(rbq_index_destroy(NULL) == RBQ_EINVAL);
  /* invalid parameters */
  const int bad_bq[] = {0, 9};
  for (int i = 0; i < 2; ++i) {
    rbq_params q = p;
    q.bq = bad_bq[i];
    rbq_index* x = NULL;
    CHECK(rbq_index_create(&q, &x) == RBQ_EINVAL);
    CHECK(strlen(rbq_last_error()) > 0);
  }
  for (int bq = 1; bq <= 8; ++bq) {
    rbq_params q = p;
    q.bq = bq;
    rbq_index* x = NULL;
    CHECK(rbq_index_create(&q, &x) == RBQ_OK);
    CHECK(rbq_index_destroy(x) == RBQ_OK);
  }
  /* files: missing, bad header, truncated payload */
  rbq_index* ld = NULL;
  snprintf(path, sizeof(path), "%s/none.rbq", dir);
  CHECK(rbq_index_load(path, &ld) == RBQ_EINVAL);
  snprintf(path, sizeof(path), "%s/bad.rbq", dir);
  FILE* f = fopen(path, "wb");
  CHECK(f);
  const char junk[72] = "NOTANIDX";
  fwrite(junk, 1, sizeof(junk), f);
  fclose(f);
  CHECK(rbq_index_load(path, &ld) == RBQ_EFORMAT);
  snprintf(path, sizeof(path), "%s/trunc.rbq", dir);
  f = fopen(path, "wb");
  CHECK(f);
  struct {
    char magic[8];
    unsigned int version;
    int dim, dp, nlist, bq, rot;
    float eps0;
    unsigned int pad;
    unsigned long long seed;
    long long n;
  } h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "RBQIDX01", 8);
  h.version = 1;
  h.dim = 64;
  h.dp = 64;
  h.nlist = 2;
  h.bq = 4;
  h.eps0 = 1.9f;
  h.n = 10;
  fwrite(&h, sizeof(h), 1, f);
  char zeros[100] = {0};
  fwrite(zeros, 1, sizeof(zeros), f);
  fclose(f);
  CHECK(rbq_index_load(path, &ld) == RBQ_EFORMAT);
  int32_t table[32];
  CHECK(rbq_nprobe_bucket_table(table) == RBQ_OK && table[0] == 4 && table[31] == 512);
  CHECK(rbq_nprobe_bucket_table(NULL) == RBQ_EINVAL);
  printf("sanitized host checks passed\n");
  return 0;
}
