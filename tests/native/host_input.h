/* Input reader and exact printout helpers for the sanitizer drivers of the host tests.
 *
 * Input file (little-endian, written by tests/test_host_sanitized.py):
 *   int32 kind: 0 score, 1 weighted score, 2 compare
 *   kind 0, 1: int32 n, int32 L, int64 nnz, int32 row_ptr[n + 1], int32 col_idx[nnz],
 *              (kind 1) float32 w[nnz], int32 labels[n]
 *   kind 2:    int32 N, int32 La, int32 Lb, int32 la[N], int32 lb[N]
 * Every array is read into a buffer of exactly its length, so a read past it is caught.
 * Output: one "name value" line per result; integers in decimal, binary64 values as the
 * hex of their bits, arrays as the FNV-1a 64 hash of their bytes. */
#ifndef HOST_INPUT_H
#define HOST_INPUT_H

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t kind, n, L, La, Lb;
  int64_t nnz;
  int32_t *rp, *ci, *lab, *la, *lb;
  float* w;
} host_input;

static inline void* rd_exact(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
    fprintf(stderr, "short input\n");
    exit(3);
  }
  return p;
}

static inline void rd_val(FILE* f, void* dst, size_t bytes) {
  if (fread(dst, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(3);
  }
}

static inline void read_input(const char* path, host_input* in) {
  FILE* f = fopen(path, "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    exit(3);
  }
  memset(in, 0, sizeof(*in));
  rd_val(f, &in->kind, 4);
  if (in->kind == 0 || in->kind == 1) {
    rd_val(f, &in->n, 4);
    rd_val(f, &in->L, 4);
    rd_val(f, &in->nnz, 8);
    in->rp = rd_exact(f, 4 * ((size_t)in->n + 1));
    in->ci = rd_exact(f, 4 * (size_t)in->nnz);
    if (in->kind == 1) in->w = rd_exact(f, 4 * (size_t)in->nnz);
    in->lab = rd_exact(f, 4 * (size_t)in->n);
  } else {
    rd_val(f, &in->n, 4);
    rd_val(f, &in->La, 4);
    rd_val(f, &in->Lb, 4);
    in->la = rd_exact(f, 4 * (size_t)in->n);
    in->lb = rd_exact(f, 4 * (size_t)in->n);
  }
  fclose(f);
}

static inline void free_input(host_input* in) {
  free(in->rp);
  free(in->ci);
  free(in->w);
  free(in->lab);
  free(in->la);
  free(in->lb);
}

static inline uint64_t fnv1a(const void* p, size_t bytes) {
  const unsigned char* b = (const unsigned char*)p;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < bytes; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

static inline void put_i(const char* k, int64_t x) { printf("%s %lld\n", k, (long long)x); }
static inline void put_d(const char* k, double x) {
  uint64_t u;
  memcpy(&u, &x, 8);
  printf("%s %016llx\n", k, (unsigned long long)u);
}
static inline void put_h(const char* k, const void* p, size_t bytes) {
  printf("%s %016llx\n", k, (unsigned long long)fnv1a(p, bytes));
}

#endif
