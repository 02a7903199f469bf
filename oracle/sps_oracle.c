/*
 * sps_oracle.c -- CPU oracle for the sliding super point sketch (SRE array + SLE array).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no source with the HIP path: hashes, seed expansion, derived constants and
 * every step of the method are written out again here, from the paper and from the hash
 * specification in the design notes.
 *
 * Plain, slow, obviously correct code: fp64 for every floating-point step, loops in the
 * order the paper states them, no blocking or fusion.
 *
 * Paper: "Memory efficient distributed sliding super point cardinality estimation by GPU"
 * (arXiv 1805.09246).  Citations name the section, equation or algorithm.
 *
 * State is kept as u16 *stamps* (slice number of the last write, 0 = never written) instead
 * of the paper's u16 *distances* (Sec. 3.2: initialised to 65535, set to 0 on a write and
 * incremented once per slice).  The two are equivalent: distance d = cur - stamp, and a cell
 * counts toward the k-weight |SRE|^k / |SLE|^k (d < k) exactly when stamp >= cur - k + 1.
 * Merging "takes the biggest" recorder in the paper's Alg. 2 / Alg. 7; the union of two
 * routers' observations is the smallest distance, i.e. the largest stamp.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ESLICE (-2)
#define OR_EMISMATCH (-3)
#define OR_ENOMEM (-4)
#define OR_ECAPACITY (-5)

#define OR_MAX_ROWS 32
#define OR_MAX_SLICE 65534u

/* flag bits on an estimate */
#define OR_F_SATURATED 1u  /* corrected weight clamped to eta'-1 */
#define OR_F_CLAMPLOW 16u  /* corrected weight clamped to 0 */
#define OR_F_NEAR 8u       /* |estimate - threshold| <= 1e-9 * threshold */

typedef struct {
  uint32_t q, r, delta, eta;     /* SRE array: 2^q columns, r rows, RHFG shift step, cells per SRE */
  uint32_t qp, rp, etap, deltap; /* SLE array: 2^q' SLEs per row, r' rows, cells per SLE, offset */
  uint32_t theta;                /* create-time threshold, fixes tau (Eq. 1) */
  uint32_t anet_side;            /* 0: aip = dst, bip = src; 1: aip = src, bip = dst */
  uint64_t seed;
} or_params;

typedef struct {
  or_params p;
  uint32_t tau;     /* Eq. 1 */
  uint32_t hot_cut; /* smallest integer weight >= rho * eta (Sec. 3.2) */
  uint64_t row_len; /* L' = 2^q' * delta' + eta' - delta' (Sec. 4) */
  uint32_t s_h1, s_h2, s_h3, s_rhfg0, s_lh[OR_MAX_ROWS];
  uint16_t *sre;  /* [r][2^q][eta] */
  uint16_t *slea; /* [r'][L'] */
  uint32_t cur;   /* last slice written (0 before any) */
} or_sketch;

/* ------------------------------------------------------------------------------------- */
/* Hash specification (restated from the published definitions).                        */
/* ------------------------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea, Flood 2014): state += golden gamma, then a 64-bit mix. */
static uint64_t or_splitmix64(uint64_t *state) {
  uint64_t z;
  *state = *state + 0x9E3779B97F4A7C15ull;
  z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* MurmurHash3 32-bit finalizer (Appleby, public domain); a bijection on 32 bits. */
static uint32_t or_fmix32(uint32_t h) {
  h = h ^ (h >> 16);
  h = h * 0x85EBCA6Bu;
  h = h ^ (h >> 13);
  h = h * 0xC2B2AE35u;
  h = h ^ (h >> 16);
  return h;
}

/* Seed j (j = 0, 1, 2, ...) is the low 32 bits of the (j+1)-th SplitMix64 output.
 * j = 0: H1, 1: H2, 2: H3, 3: RHFG[0], 4 + i: LH_i. */
static void or_expand_seeds(or_sketch *s) {
  uint64_t st = s->p.seed;
  uint32_t i;
  s->s_h1 = (uint32_t)or_splitmix64(&st);
  s->s_h2 = (uint32_t)or_splitmix64(&st);
  s->s_h3 = (uint32_t)or_splitmix64(&st);
  s->s_rhfg0 = (uint32_t)or_splitmix64(&st);
  for (i = 0; i < OR_MAX_ROWS; i++) s->s_lh[i] = (uint32_t)or_splitmix64(&st);
}

/* Def. 3: LSB(i) is the index of the lowest set bit; LSB(0) is taken to be 32. */
uint32_t or_lsb(uint32_t v) {
  uint32_t n = 0;
  if (v == 0) return 32;
  while ((v & 1u) == 0) {
    v >>= 1;
    n++;
  }
  return n;
}

/* H1: 32-bit hash of the opposite host; its LSB decides sampling (Sec. 3.2). */
static uint32_t or_H1(const or_sketch *s, uint32_t bip) { return or_fmix32(bip ^ s->s_h1); }
/* H2: cell of an SRE, in [0, eta) (Sec. 3.2). */
static uint32_t or_H2(const or_sketch *s, uint32_t bip) {
  return or_fmix32(bip ^ s->s_h2) % s->p.eta;
}
/* H3: cell of an SLE, in [0, eta') (Sec. 4). */
static uint32_t or_H3(const or_sketch *s, uint32_t bip) {
  return or_fmix32(bip ^ s->s_h3) % s->p.etap;
}
/* RHFG[i] (Eq. 6): RHFG[0] is a random hash into [0, 2^q); row i >= 1 xors RHFG[0] with the
 * q address bits starting at (i-1)*delta.  (The printed shift is i*delta; with that shift
 * bits [0, delta) would never be recovered, while the stated coverage condition
 * (r-2)*delta + q >= 32 is exactly the condition for the (i-1)*delta shift.) */
static uint32_t or_RHFG(const or_sketch *s, uint32_t i, uint32_t aip) {
  uint32_t qmask = (uint32_t)((1ull << s->p.q) - 1ull);
  uint32_t c0 = or_fmix32(aip ^ s->s_rhfg0) & qmask;
  if (i == 0) return c0;
  return ((aip >> ((i - 1) * s->p.delta)) ^ c0) & qmask;
}
/* LH_i: SLE index of row i, in [0, 2^q') (Sec. 4, Alg. 6). */
static uint32_t or_LH(const or_sketch *s, uint32_t i, uint32_t aip) {
  return or_fmix32(aip ^ s->s_lh[i]) % (uint32_t)(1ull << s->p.qp);
}

/* exported for the pin tests */
uint32_t or_hash(const or_sketch *s, uint32_t which, uint32_t row, uint32_t x) {
  switch (which) {
    case 0: return or_H1(s, x);
    case 1: return or_H2(s, x);
    case 2: return or_H3(s, x);
    case 3: return or_RHFG(s, row, x);
    case 4: return or_LH(s, row, x);
    default: return 0;
  }
}
uint32_t or_fmix32_export(uint32_t h) { return or_fmix32(h); }
uint64_t or_splitmix64_export(uint64_t state) { return or_splitmix64(&state); }

/* ------------------------------------------------------------------------------------- */
/* Derived constants                                                                     */
/* ------------------------------------------------------------------------------------- */

static int or_is_pow2(uint64_t v) { return v != 0 && (v & (v - 1)) == 0; }

/* Eq. 1, tau = ceil(log2(theta / eta)), in integer form: the smallest t >= 0 with
 * eta * 2^t >= theta. */
uint32_t or_tau(uint32_t theta, uint32_t eta) {
  uint32_t t = 0;
  while ((uint64_t)eta << t < (uint64_t)theta) t++;
  return t;
}

/* Sec. 3.2: an SRE is hot when its weight is no smaller than rho * eta with
 * rho = 0.99 * (1 - e^(-1/3)); for an integer weight that is weight >= ceil(rho * eta). */
uint32_t or_hot_cut(uint32_t eta) {
  double rho = 0.99 * (1.0 - exp(-1.0 / 3.0));
  return (uint32_t)ceil(rho * (double)eta);
}

/* Sec. 4: a row of the SLE array holds 2^q' * delta' + eta' - delta' cells. */
uint64_t or_row_len(uint32_t qp, uint32_t etap, uint32_t deltap) {
  return (1ull << qp) * deltap + etap - deltap;
}

/* Eq. 10: memory reduction rate of sharing cells between adjacent SLEs. */
double or_mrr(uint32_t qp, uint32_t etap, uint32_t deltap) {
  return 1.0 - (double)or_row_len(qp, etap, deltap) / ((double)etap * (double)(1ull << qp));
}

int or_check_params(const or_params *p) {
  if (!p) return OR_EINVAL;
  if (p->q < 1 || p->q > 24 || p->r < 2 || p->r > OR_MAX_ROWS) return OR_EINVAL;
  if (p->delta < 1 || p->delta >= p->q) return OR_EINVAL;
  if ((uint64_t)(p->r - 2) * p->delta + p->q < 32) return OR_EINVAL; /* coverage, Eq. 6 */
  if ((uint64_t)(p->r - 2) * p->delta > 31) return OR_EINVAL;
  if (!or_is_pow2(p->eta) || p->eta > 64) return OR_EINVAL;
  if (p->qp < 1 || p->qp > 24 || p->rp < 1 || p->rp > OR_MAX_ROWS) return OR_EINVAL;
  if (!or_is_pow2(p->etap) || p->etap > 65536) return OR_EINVAL;
  if (p->deltap < 1 || p->deltap > p->etap) return OR_EINVAL;
  if (p->theta < 1 || p->anet_side > 1) return OR_EINVAL;
  return OR_OK;
}

/* ------------------------------------------------------------------------------------- */
/* Sketch object                                                                         */
/* ------------------------------------------------------------------------------------- */

or_sketch *or_create(const or_params *p) {
  or_sketch *s;
  if (or_check_params(p) != OR_OK) return NULL;
  s = (or_sketch *)calloc(1, sizeof(or_sketch));
  if (!s) return NULL;
  s->p = *p;
  s->tau = or_tau(p->theta, p->eta);
  s->hot_cut = or_hot_cut(p->eta);
  s->row_len = or_row_len(p->qp, p->etap, p->deltap);
  or_expand_seeds(s);
  s->sre = (uint16_t *)calloc((size_t)p->r << p->q, (size_t)p->eta * sizeof(uint16_t));
  s->slea = (uint16_t *)calloc((size_t)p->rp * s->row_len, sizeof(uint16_t));
  if (!s->sre || !s->slea) {
    free(s->sre);
    free(s->slea);
    free(s);
    return NULL;
  }
  s->cur = 0;
  return s;
}

void or_destroy(or_sketch *s) {
  if (!s) return;
  free(s->sre);
  free(s->slea);
  free(s);
}

uint32_t or_get_tau(const or_sketch *s) { return s->tau; }
uint32_t or_get_hot_cut(const or_sketch *s) { return s->hot_cut; }
uint64_t or_get_row_len(const or_sketch *s) { return s->row_len; }
uint32_t or_get_cur(const or_sketch *s) { return s->cur; }
uint16_t *or_sre_ptr(or_sketch *s) { return s->sre; }
uint16_t *or_slea_ptr(or_sketch *s) { return s->slea; }
uint64_t or_sre_cells(const or_sketch *s) { return ((uint64_t)s->p.r << s->p.q) * s->p.eta; }
uint64_t or_slea_cells(const or_sketch *s) { return (uint64_t)s->p.rp * s->row_len; }

static uint16_t *or_sre_cell(or_sketch *s, uint32_t row, uint32_t col, uint32_t e) {
  return &s->sre[(((uint64_t)row << s->p.q) + col) * s->p.eta + e];
}
static uint16_t *or_slea_cell(or_sketch *s, uint32_t row, uint64_t j) {
  return &s->slea[(uint64_t)row * s->row_len + j];
}

/* ------------------------------------------------------------------------------------- */
/* Ingest: Alg. 3 (update the SRE array for one IP pair) and Alg. 6 (update the SLE array) */
/* ------------------------------------------------------------------------------------- */

int or_set_slice(or_sketch *s, uint32_t slice) {
  if (slice < 1 || slice > OR_MAX_SLICE || slice < s->cur) return OR_ESLICE;
  s->cur = slice;
  return OR_OK;
}

/* pkts: n pairs (src, dst) of u32; slice: the stamp written ("distance 0" in the paper). */
int or_ingest(or_sketch *s, const uint32_t *pkts, uint64_t n, uint32_t slice) {
  uint64_t k;
  uint32_t i;
  int rc = or_set_slice(s, slice);
  if (rc != OR_OK) return rc;
  for (k = 0; k < n; k++) {
    uint32_t src = pkts[2 * k], dst = pkts[2 * k + 1];
    uint32_t aip = s->p.anet_side == 0 ? dst : src;
    uint32_t bip = s->p.anet_side == 0 ? src : dst;
    /* Alg. 3: sample bip by the LSB of H1; if sampled, set cell H2(bip) of SRE RHFG[i](aip)
     * in every row i. */
    uint32_t lsb = or_lsb(or_H1(s, bip));
    if (lsb >= s->tau) {
      uint32_t e = or_H2(s, bip);
      for (i = 0; i < s->p.r; i++) *or_sre_cell(s, i, or_RHFG(s, i, aip), e) = (uint16_t)slice;
    }
    /* Alg. 6: cell H3(bip) of SLE LH_i(aip) in every row i; SLE j starts at cell j*delta'. */
    {
      uint32_t z = or_H3(s, bip);
      for (i = 0; i < s->p.rp; i++)
        *or_slea_cell(s, i, (uint64_t)or_LH(s, i, aip) * s->p.deltap + z) = (uint16_t)slice;
    }
  }
  return OR_OK;
}

/* The same update on several threads: the work is cut by row -- the r SRE rows (Alg. 3)
 * and the r' SLE rows (Alg. 6) are separate tasks, handed to the threads round robin --
 * and every thread walks all packets writing only its rows' cells.  No cell belongs to two
 * tasks, so the state equals or_ingest's for any thread count. */
typedef struct {
  or_sketch *s;
  const uint32_t *pkts;
  uint64_t n;
  uint32_t slice, first, step;
} or_ingest_job;

static void *or_ingest_worker(void *arg) {
  or_ingest_job *j = (or_ingest_job *)arg;
  or_sketch *s = j->s;
  uint32_t task;
  for (task = j->first; task < s->p.r + s->p.rp; task += j->step) {
    uint64_t k;
    for (k = 0; k < j->n; k++) {
      uint32_t src = j->pkts[2 * k], dst = j->pkts[2 * k + 1];
      uint32_t aip = s->p.anet_side == 0 ? dst : src;
      uint32_t bip = s->p.anet_side == 0 ? src : dst;
      if (task < s->p.r) {
        if (or_lsb(or_H1(s, bip)) >= s->tau)
          *or_sre_cell(s, task, or_RHFG(s, task, aip), or_H2(s, bip)) = (uint16_t)j->slice;
      } else {
        uint32_t i = task - s->p.r;
        *or_slea_cell(s, i, (uint64_t)or_LH(s, i, aip) * s->p.deltap + or_H3(s, bip)) =
            (uint16_t)j->slice;
      }
    }
  }
  return NULL;
}

int or_ingest_threads(or_sketch *s, const uint32_t *pkts, uint64_t n, uint32_t slice,
                      uint32_t nthreads) {
  pthread_t th[64];
  or_ingest_job jobs[64];
  uint32_t t;
  int rc = or_set_slice(s, slice);
  if (rc != OR_OK) return rc;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  if (nthreads > s->p.r + s->p.rp) nthreads = s->p.r + s->p.rp;
  for (t = 0; t < nthreads; t++) {
    jobs[t].s = s;
    jobs[t].pkts = pkts;
    jobs[t].n = n;
    jobs[t].slice = slice;
    jobs[t].first = t;
    jobs[t].step = nthreads;
    pthread_create(&th[t], NULL, or_ingest_worker, &jobs[t]);
  }
  for (t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  return OR_OK;
}

/* ------------------------------------------------------------------------------------- */
/* Merge: Alg. 2 and Alg. 7, cell-wise, keeping the most recent observation (max stamp).  */
/* dst <- max(dst, src_0, ..., src_{n-1}).                                               */
/* ------------------------------------------------------------------------------------- */

static int or_same_params(const or_params *a, const or_params *b) {
  return a->q == b->q && a->r == b->r && a->delta == b->delta && a->eta == b->eta &&
         a->qp == b->qp && a->rp == b->rp && a->etap == b->etap && a->deltap == b->deltap &&
         a->theta == b->theta && a->anet_side == b->anet_side && a->seed == b->seed;
}

int or_merge(or_sketch *dst, or_sketch *const *srcs, uint32_t nsrc) {
  uint32_t z;
  uint64_t j, n_sre = or_sre_cells(dst), n_slea = or_slea_cells(dst);
  for (z = 0; z < nsrc; z++)
    if (!or_same_params(&dst->p, &srcs[z]->p)) return OR_EMISMATCH;
  for (j = 0; j < n_sre; j++) {
    uint16_t v = dst->sre[j];
    for (z = 0; z < nsrc; z++)
      if (v < srcs[z]->sre[j]) v = srcs[z]->sre[j];
    dst->sre[j] = v;
  }
  for (j = 0; j < n_slea; j++) {
    uint16_t v = dst->slea[j];
    for (z = 0; z < nsrc; z++)
      if (v < srcs[z]->slea[j]) v = srcs[z]->slea[j];
    dst->slea[j] = v;
  }
  for (z = 0; z < nsrc; z++)
    if (srcs[z]->cur > dst->cur) dst->cur = srcs[z]->cur;
  return OR_OK;
}

/* ------------------------------------------------------------------------------------- */
/* Rebase of the time base.  The paper's distance recorders (Sec. 3.2) saturate at 65535;  */
/* u16 stamps run out at slice 65534 instead.  Shifting every stamp down by `offset`      */
/* (stamps at or below it become 0, never written) and the current slice with them keeps  */
/* every window of at most cur - offset slices unchanged: a recorder within such a window */
/* has a stamp above offset before the shift and a positive stamp after it.              */
/* ------------------------------------------------------------------------------------- */

int or_rebase(or_sketch *s, uint32_t offset) {
  uint64_t j, n_sre = or_sre_cells(s), n_slea = or_slea_cells(s);
  if (offset > s->cur) return OR_ESLICE;
  for (j = 0; j < n_sre; j++) s->sre[j] = s->sre[j] > offset ? (uint16_t)(s->sre[j] - offset) : 0;
  for (j = 0; j < n_slea; j++)
    s->slea[j] = s->slea[j] > offset ? (uint16_t)(s->slea[j] - offset) : 0;
  s->cur -= offset;
  return OR_OK;
}

/* ------------------------------------------------------------------------------------- */
/* Scan, part 1: k-weights.                                                              */
/* ------------------------------------------------------------------------------------- */

/* first live stamp of the window of k slices ending at the current slice */
static uint32_t or_window_lo(uint32_t cur, uint32_t k) {
  return cur >= k ? cur - k + 1 : 1;
}

/* Def. 4 numerators: for every SLE-array row, the number of cells whose distance is < k. */
void or_row_live(const or_sketch *s, uint32_t k, uint64_t *out) {
  uint32_t lo = or_window_lo(s->cur, k), i;
  uint64_t j;
  for (i = 0; i < s->p.rp; i++) {
    uint64_t n = 0;
    for (j = 0; j < s->row_len; j++)
      if (s->slea[(uint64_t)i * s->row_len + j] >= lo) n++;
    out[i] = n;
  }
}

/* Hot SREs (Sec. 3.3): out[i * 2^q + col] = 1 when SRE (i, col) has k-weight >= hot cut. */
void or_hot(or_sketch *s, uint32_t k, uint8_t *out) {
  uint32_t lo = or_window_lo(s->cur, k), i, col, e;
  for (i = 0; i < s->p.r; i++)
    for (col = 0; col < (1u << s->p.q); col++) {
      uint32_t w = 0;
      for (e = 0; e < s->p.eta; e++)
        if (*or_sre_cell(s, i, col, e) >= lo) w++;
      out[((uint64_t)i << s->p.q) + col] = w >= s->hot_cut ? 1 : 0;
    }
}

/* ------------------------------------------------------------------------------------- */
/* Scan, part 2: candidate recovery.                                                     */
/* ------------------------------------------------------------------------------------- */

/* Plain definition of the recovered set: every 32-bit address whose SRE is hot in every row.
 * Exhaustive over [0, 2^32), split over threads. */
typedef struct {
  const or_sketch *s;
  const uint8_t *hot;
  uint64_t lo, hi;
  uint32_t *out;
  uint64_t cap, n;
} or_brute_job;

static void *or_brute_worker(void *arg) {
  or_brute_job *jb = (or_brute_job *)arg;
  uint64_t x;
  uint32_t i;
  jb->n = 0;
  for (x = jb->lo; x < jb->hi; x++) {
    int all = 1;
    for (i = 0; i < jb->s->p.r && all; i++)
      if (!jb->hot[((uint64_t)i << jb->s->p.q) + or_RHFG(jb->s, i, (uint32_t)x)]) all = 0;
    if (all) {
      if (jb->n < jb->cap) jb->out[jb->n] = (uint32_t)x;
      jb->n++;
    }
  }
  return NULL;
}

/* returns the number of addresses found (may exceed cap; only cap are written) */
int64_t or_join_brute(const or_sketch *s, const uint8_t *hot, uint32_t *out, uint64_t cap,
                      uint32_t nthreads) {
  pthread_t th[256];
  or_brute_job jobs[256];
  uint64_t total = 0, written = 0, t;
  uint32_t *bufs[256];
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  for (t = 0; t < nthreads; t++) {
    bufs[t] = (uint32_t *)malloc((cap + 1) * sizeof(uint32_t));
    if (!bufs[t]) return OR_ENOMEM;
    jobs[t].s = s;
    jobs[t].hot = hot;
    jobs[t].lo = (1ull << 32) * t / nthreads;
    jobs[t].hi = (1ull << 32) * (t + 1) / nthreads;
    jobs[t].out = bufs[t];
    jobs[t].cap = cap;
    pthread_create(&th[t], NULL, or_brute_worker, &jobs[t]);
  }
  for (t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
  /* thread ranges are ascending, so concatenation is ascending */
  for (t = 0; t < nthreads; t++) {
    uint64_t m;
    for (m = 0; m < jobs[t].n && m < cap; m++)
      if (written < cap) out[written++] = bufs[t][m];
    total += jobs[t].n;
    free(bufs[t]);
  }
  return (int64_t)total;
}

/* The paper's tuple-growing procedure (Sec. 3.3, Alg. 4 and Alg. 5), breadth first with
 * two candidate-tuple buffers.  B(i) = he_0 xor he_i recovers the q address bits at shift
 * (i-1)*delta (Eq. 7).  A tuple grown by row i survives when the high q-delta bits of B(i-1)
 * equal the low q-delta bits of B(i).  Bits that would lie at or above bit 32 must be zero.
 * After the last row the address is assembled and checked against RHFG[0].
 * hot lists: lists[i] has counts[i] ascending columns.  Returns the count of recovered
 * addresses (ascending after a final sort in the caller), or an error.  level_sizes (r
 * entries, or NULL) receives the number of tuples grown through each row i >= 1: entry 1
 * counts the pairs (he0, he1) whose B(1) fits 32 bits, entry i the tuples (he0 .. he_i). */
static int or_cmp_u32(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int or_bits_fit(const or_sketch *s, uint32_t i, uint32_t b) {
  /* row i (>= 1) holds address bits [(i-1)delta, (i-1)delta + q); bits beyond 31 are zero */
  uint32_t shift = (i - 1) * s->p.delta;
  if (shift + s->p.q <= 32) return 1;
  return (b >> (32 - shift)) == 0;
}

int64_t or_join_tuples(const or_sketch *s, const uint8_t *hot, uint32_t *out, uint64_t cap,
                       uint64_t tuple_cap, uint64_t *level_sizes) {
  uint32_t r = s->p.r, q = s->p.q, d = s->p.delta, i;
  uint32_t ncols = 1u << q;
  uint32_t low_mask = (1u << (q - d)) - 1u;
  uint32_t *lists[OR_MAX_ROWS], counts[OR_MAX_ROWS];
  uint32_t *rctb, *sctb, *tmp;
  uint64_t nr = 0, ns, a, b, c, m, found = 0;
  /* HSE(i): ascending lists of hot columns */
  for (i = 0; i < r; i++) {
    uint32_t col;
    lists[i] = (uint32_t *)malloc(((size_t)ncols + 1) * sizeof(uint32_t));
    counts[i] = 0;
    for (col = 0; col < ncols; col++)
      if (hot[((uint64_t)i << q) + col]) lists[i][counts[i]++] = col;
  }
  rctb = (uint32_t *)malloc((size_t)(tuple_cap + 1) * r * sizeof(uint32_t));
  sctb = (uint32_t *)malloc((size_t)(tuple_cap + 1) * r * sizeof(uint32_t));
  if (!rctb || !sctb) {
    for (i = 0; i < r; i++) free(lists[i]);
    free(rctb);
    free(sctb);
    return OR_ENOMEM;
  }
  if (level_sizes)
    for (i = 0; i < r; i++) level_sizes[i] = 0;
  /* Alg. 4: tuples (he0, he1, he2) from rows 0..2, checking B(1) against B(2) */
  for (a = 0; a < counts[0]; a++)
    for (b = 0; b < counts[1]; b++) {
      uint32_t he0 = lists[0][a], he1 = lists[1][b];
      uint32_t B1 = he0 ^ he1;
      if (!or_bits_fit(s, 1, B1)) continue;
      if (level_sizes) level_sizes[1]++;
      for (c = 0; c < counts[2]; c++) {
        uint32_t he2 = lists[2][c];
        uint32_t B2 = he0 ^ he2;
        if ((B1 >> d) != (B2 & low_mask)) continue;
        if (!or_bits_fit(s, 2, B2)) continue;
        if (nr >= tuple_cap) goto overflow;
        rctb[nr * r + 0] = he0;
        rctb[nr * r + 1] = he1;
        rctb[nr * r + 2] = he2;
        nr++;
      }
    }
  if (level_sizes && r > 2) level_sizes[2] = nr;
  /* Alg. 5: rows 3..r-1, extending every tuple of the reading buffer by one hot SRE */
  for (i = 3; i < r; i++) {
    ns = 0;
    for (m = 0; m < nr; m++) {
      uint32_t he0 = rctb[m * r + 0];
      uint32_t Bprev = he0 ^ rctb[m * r + (i - 1)];
      for (c = 0; c < counts[i]; c++) {
        uint32_t hei = lists[i][c];
        uint32_t Bi = he0 ^ hei;
        if ((Bprev >> d) != (Bi & low_mask)) continue;
        if (!or_bits_fit(s, i, Bi)) continue;
        if (ns >= tuple_cap) goto overflow;
        memcpy(&sctb[ns * r], &rctb[m * r], (size_t)i * sizeof(uint32_t));
        sctb[ns * r + i] = hei;
        ns++;
      }
    }
    tmp = rctb;
    rctb = sctb;
    sctb = tmp;
    nr = ns;
    if (level_sizes) level_sizes[i] = nr;
  }
  /* reconstruct aip from B(1..r-1) and keep it when RHFG[0](aip) is he0 */
  for (m = 0; m < nr; m++) {
    uint32_t he0 = rctb[m * r + 0];
    uint64_t x = 0;
    for (i = 1; i < r; i++) x |= (uint64_t)(he0 ^ rctb[m * r + i]) << ((i - 1) * d);
    if (x >> 32) continue;
    if (or_RHFG(s, 0, (uint32_t)x) != he0) continue;
    if (found < cap) out[found] = (uint32_t)x;
    found++;
  }
  for (i = 0; i < r; i++) free(lists[i]);
  free(rctb);
  free(sctb);
  if (found <= cap) qsort(out, (size_t)found, sizeof(uint32_t), or_cmp_u32);
  return (int64_t)found;
overflow:
  for (i = 0; i < r; i++) free(lists[i]);
  free(rctb);
  free(sctb);
  return OR_ECAPACITY;
}

/* ------------------------------------------------------------------------------------- */
/* Scan, part 3: Alg. 8, the cardinality estimate of one candidate, and the final filter. */
/* ------------------------------------------------------------------------------------- */

/* USLE of aip (Alg. 8): cell z of the union SLE combines cell z of aip's SLE in every row.
 * The paper keeps the largest distance, so a union cell is within the window only when it
 * is within the window in every row (the intersection Eq. 11 assumes); in stamps that is
 * the smallest stamp.  (The printed loop reads row 0 for every i; row i is meant.) */
static void or_usle(const or_sketch *s, uint32_t aip, uint16_t *m) {
  uint32_t z, i;
  for (z = 0; z < s->p.etap; z++) m[z] = 0xFFFF;
  for (i = 0; i < s->p.rp; i++) {
    uint64_t j0 = (uint64_t)or_LH(s, i, aip) * s->p.deltap;
    for (z = 0; z < s->p.etap; z++) {
      uint16_t v = s->slea[(uint64_t)i * s->row_len + j0 + z];
      if (v < m[z]) m[z] = v;
    }
  }
}

/* Per-age cumulative live counts of aip's USLE: x[a] = number of union cells last written
 * within the newest a+1 slices (a < k).  x[k-1] is |USLE|^k. */
int or_features(const or_sketch *s, uint32_t k, const uint32_t *hosts, uint64_t n, uint32_t *x) {
  uint16_t *m;
  uint64_t h;
  uint32_t a, z;
  if (k < 1) return OR_EINVAL;
  m = (uint16_t *)malloc((size_t)s->p.etap * sizeof(uint16_t));
  if (!m) return OR_ENOMEM;
  for (h = 0; h < n; h++) {
    or_usle(s, hosts[h], m);
    for (a = 0; a < k; a++) {
      uint32_t lo_a = s->cur >= a + 1 ? s->cur - a : 1, cnt = 0;
      if (lo_a < 1) lo_a = 1;
      for (z = 0; z < s->p.etap; z++)
        if (m[z] >= lo_a) cnt++;
      x[h * k + a] = cnt;
    }
  }
  free(m);
  return OR_OK;
}

/* Eq. 12 then Eq. 9.  row_live: Def. 4 numerators of every SLE-array row. */
double or_estimate_one(const or_sketch *s, uint32_t U, const uint64_t *row_live, double threshold,
                       uint32_t *flags) {
  double etap = (double)s->p.etap, P = 1.0, w;
  uint32_t i, f = 0;
  /* product of the row setting factors SF(i, k) (Def. 4), rows in order */
  for (i = 0; i < s->p.rp; i++) P = P * ((double)row_live[i] / (double)s->row_len);
  /* Eq. 12: expected share of union cells set by other hosts removed */
  if (P >= 1.0)
    w = (double)U;
  else
    w = ((double)U - etap * P) / (1.0 - P);
  if (w < 0.0) {
    w = 0.0;
    f |= OR_F_CLAMPLOW;
  }
  if (w > etap - 1.0) {
    w = etap - 1.0;
    f |= OR_F_SATURATED;
  }
  /* Eq. 9 (linear counting): n = -eta' ln((eta' - w) / eta') = -eta' log1p(-w / eta') */
  {
    double est = -etap * log1p(-w / etap);
    if (fabs(est - threshold) <= 1e-9 * threshold) f |= OR_F_NEAR;
    *flags = f;
    return est;
  }
}

typedef struct {
  uint32_t host;
  uint32_t live;  /* |USLE|^k */
  uint32_t flags;
  uint32_t pad;
  double estimate;
} or_result;

/* Estimate every host of a candidate list (ascending) and keep those whose estimate reaches
 * the threshold (final filter, end of Sec. 4).  Output ascending by host.
 * Returns the number kept (may exceed cap; then only cap are written). */
int64_t or_estimate_filter(const or_sketch *s, uint32_t k, double threshold,
                           const uint32_t *cands, uint64_t ncand, or_result *out, uint64_t cap) {
  uint64_t row_live[OR_MAX_ROWS], h, kept = 0;
  uint32_t *x;
  if (k < 1) return OR_EINVAL;
  or_row_live(s, k, row_live);
  x = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
  if (!x) return OR_ENOMEM;
  for (h = 0; h < ncand; h++) {
    uint32_t flags, U;
    double est;
    or_features(s, k, &cands[h], 1, x);
    U = x[k - 1];
    est = or_estimate_one(s, U, row_live, threshold, &flags);
    if (est >= threshold) {
      if (kept < cap) {
        out[kept].host = cands[h];
        out[kept].live = U;
        out[kept].flags = flags;
        out[kept].pad = 0;
        out[kept].estimate = est;
      }
      kept++;
    }
  }
  free(x);
  return (int64_t)kept;
}

/* Whole scan at the current slice: hot SREs, recovery by the plain definition, estimate and
 * filter.  cand_out (optional, cand_cap entries) receives the recovered candidates. */
int64_t or_scan(or_sketch *s, uint32_t k, double threshold, or_result *out, uint64_t cap,
                uint32_t *cand_out, uint64_t cand_cap, uint64_t *n_cand, uint32_t nthreads) {
  uint8_t *hot;
  uint32_t *cands;
  int64_t nc, kept;
  uint64_t ccap = 1u << 22;
  if (k < 1) return OR_EINVAL;
  hot = (uint8_t *)malloc((size_t)s->p.r << s->p.q);
  cands = (uint32_t *)malloc((size_t)ccap * sizeof(uint32_t));
  if (!hot || !cands) {
    free(hot);
    free(cands);
    return OR_ENOMEM;
  }
  or_hot(s, k, hot);
  nc = or_join_brute(s, hot, cands, ccap, nthreads);
  free(hot);
  if (nc < 0 || (uint64_t)nc > ccap) {
    free(cands);
    return nc < 0 ? nc : OR_ECAPACITY;
  }
  if (n_cand) *n_cand = (uint64_t)nc;
  if (cand_out) memcpy(cand_out, cands, (size_t)((uint64_t)nc < cand_cap ? (uint64_t)nc : cand_cap) * 4);
  kept = or_estimate_filter(s, k, threshold, cands, (uint64_t)nc, out, cap);
  free(cands);
  return kept;
}
