/* Drives every oracle entry point on small sketches, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Exit status 0 when every call
 * returned what it should; the sanitizers abort on the first memory or UB error. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  uint32_t q, r, delta, eta, qp, rp, etap, deltap, theta, anet_side;
  uint64_t seed;
} or_params;
typedef struct {
  uint32_t host, live, flags, pad;
  double estimate;
} or_result;
typedef struct or_sketch or_sketch;

or_sketch *or_create(const or_params *p);
void or_destroy(or_sketch *s);
int or_ingest(or_sketch *s, const uint32_t *pkts, uint64_t n, uint32_t slice);
int or_ingest_threads(or_sketch *s, const uint32_t *pkts, uint64_t n, uint32_t slice,
                      uint32_t nthreads);
int or_set_slice(or_sketch *s, uint32_t slice);
int or_merge(or_sketch *dst, or_sketch *const *srcs, uint32_t nsrc);
int or_rebase(or_sketch *s, uint32_t offset);
void or_row_live(const or_sketch *s, uint32_t k, uint64_t *out);
void or_hot(or_sketch *s, uint32_t k, uint8_t *out);
int64_t or_join_tuples(const or_sketch *s, const uint8_t *hot, uint32_t *out, uint64_t cap,
                       uint64_t tuple_cap, uint64_t *level_sizes);
int or_features(const or_sketch *s, uint32_t k, const uint32_t *hosts, uint64_t n, uint32_t *x);
int64_t or_estimate_filter(const or_sketch *s, uint32_t k, double threshold,
                           const uint32_t *cands, uint64_t ncand, or_result *out, uint64_t cap);
uint16_t *or_sre_ptr(or_sketch *s);
uint64_t or_sre_cells(const or_sketch *s);

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                               \
    }                                                         \
  } while (0)

static uint64_t st = 0x5EED;
static uint32_t next32(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return (uint32_t)(st >> 16);
}

int main(void) {
  or_params p = {12, 6, 5, 8, 8, 5, 256, 64, 64, 0, 0x1234};
  or_params bad = p;
  uint32_t n = 60000, s, i;
  uint32_t *pk = malloc((size_t)n * 2 * sizeof(uint32_t));
  uint8_t *hot = malloc((size_t)p.r << p.q);
  uint32_t cands[1 << 14], x[8 * 4];
  uint64_t live[8], levels[8];
  or_result res[1 << 12];
  or_sketch *a = or_create(&p), *b = or_create(&p), *c = or_create(&p);
  CHECK(pk && hot && a && b && c);
  bad.delta = 1; /* coverage (r-2)*delta + q < 32 */
  CHECK(or_create(&bad) == NULL);
  for (s = 1; s <= 6; s++) {
    for (i = 0; i < n; i++) {
      pk[2 * i] = next32();
      pk[2 * i + 1] = (next32() % 97) * 2654435761u;
    }
    CHECK(or_ingest(a, pk, n / 2, s) == 0);
    CHECK(or_ingest_threads(b, pk + n, n / 2, s, 3) == 0);
  }
  CHECK(or_ingest(a, pk, 1, 2) != 0); /* slice below the current one */
  CHECK(or_set_slice(c, 6) == 0);
  {
    or_sketch *srcs[2] = {a, b};
    CHECK(or_merge(c, srcs, 2) == 0);
  }
  or_row_live(c, 3, live);
  or_hot(c, 3, hot);
  {
    int64_t nc = or_join_tuples(c, hot, cands, 1 << 14, 1 << 20, levels);
    int64_t kept;
    CHECK(nc >= 0 && nc <= (1 << 14));
    kept = or_estimate_filter(c, 3, 50.0, cands, (uint64_t)nc, res, 1 << 12);
    CHECK(kept >= 0);
    CHECK(or_features(c, 4, cands, nc < 8 ? (uint64_t)nc : 8, x) == 0);
  }
  CHECK(or_rebase(c, 7) != 0); /* beyond the current slice */
  CHECK(or_rebase(c, 2) == 0);
  or_row_live(c, 3, live);
  CHECK(or_sre_ptr(c) != NULL && or_sre_cells(c) == ((uint64_t)p.r << p.q) * p.eta);
  or_destroy(a);
  or_destroy(b);
  or_destroy(c);
  or_destroy(NULL);
  free(pk);
  free(hot);
  printf("oracle sanitizer run ok\n");
  return 0;
}
