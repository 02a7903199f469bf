/*
 * sps.h -- C ABI of the sliding super point sketch library (MI355X / gfx950).
 *
 * Implements the per-slice pipeline of "Memory efficient distributed sliding super point
 * cardinality estimation by GPU" (arXiv 1805.09246): the reversible sliding rough estimator
 * array (SRE array, Sec. 3.2-3.3) that finds candidate super points, and the sliding linear
 * estimator array (SLE array, Sec. 4) that estimates their cardinalities, both updated per
 * packet, merged across routers, and scanned at the end of each time slice.
 *
 * State representation: every recorder is a u16 *stamp* -- the number of the last slice that
 * wrote it, 0 = never.  The paper's distance recorder (Sec. 3.2) is cur - stamp; a recorder
 * is within a window of k slices ending at the current slice cur exactly when
 * stamp >= max(1, cur - k + 1).  Slices are numbered 1..65534; sps_rebase shifts the time
 * base so a long-running sketch can go on past that.
 *
 * Conventions for every function:
 *   - Returns SPS_OK (0) or a negative SPS_E* code; no exception or abort crosses the ABI.
 *   - Pointers named d_* are device pointers (HIP device memory on the sketch's device);
 *     pointers named h_* are host pointers.  `stream` is a hipStream_t (NULL = default stream).
 *   - All device work is stream-ordered on `stream`.  Errors of asynchronous kernels surface
 *     at the next synchronizing call (sps_scan, sps_export, sps_sync).
 *   - A sketch is not thread-safe; calls on one sketch must be serialized by the caller.
 *   - Buffers owned by the caller must stay valid until the stream has passed the call.
 */
#ifndef SPS_H
#define SPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------------------------ */
#define SPS_OK 0
#define SPS_EINVAL (-1)     /* null pointer, unsupported size, coverage (r-2)*delta+q < 32 */
#define SPS_ESLICE (-2)     /* slice 0, slice below the current slice, or slice > 65534 */
#define SPS_EMISMATCH (-3)  /* merge of sketches with different parameters or seeds */
#define SPS_ENOMEM (-4)     /* device allocation failed or caller block too small */
#define SPS_ECAPACITY (-5)  /* result or candidate buffer too small (required count reported) */
#define SPS_EHIP (-6)       /* HIP runtime error; sps_strerror(SPS_EHIP) gives the last detail */
#define SPS_EBUDGET (-7)    /* admission refused: device-memory budget exhausted */

/* ---- flags of a result ------------------------------------------------------------------- */
#define SPS_F_SATURATED 1u   /* corrected weight clamped to eta'-1: linear counting saturated */
#define SPS_F_LC_FALLBACK 2u /* a learned estimator was attached but linear counting was used */
#define SPS_F_MLP 4u         /* estimate comes from the learned estimator */
#define SPS_F_NEAR 8u        /* |estimate - threshold| <= 1e-9 * threshold */
#define SPS_F_CLAMPLOW 16u   /* corrected weight clamped to 0 */

/* ---- scan info words (sps_scan_async's d_info, 8 x u32) ---------------------------------- */
#define SPS_INFO_KEPT 0      /* hosts kept by the final filter */
#define SPS_INFO_CAND 1      /* candidates recovered from the SRE array (may exceed capacity) */
#define SPS_INFO_FLAGS 2     /* bit 0: candidate buffer overflow; bit 1: result buffer overflow;
                                bit 2 (with bit 0): candidate search not run or not completed --
                                its expected size from the rows' hot rates passed 2^36 nodes (SRE
                                array saturated), or its waves timed out waiting for each other
                                (about a second; not expected) */
#define SPS_INFO_HSE0 3      /* hot SREs in row 0 */
#define SPS_INFO_HSE1 4      /* hot SREs in row 1 */
#define SPS_INFO_NODES_LO 5  /* candidate-search nodes expanded (low 32 bits; Alg. 4-5 tuples */
#define SPS_INFO_NODES_HI 6  /*   grown by one row, (he0, he1) pairs included); high 32 bits */
#define SPS_INFO_WORDS 8

/* One IP pair as the 8-byte record the paper buffers per packet (Sec. 3.3): (src, dst). */
typedef struct sps_pkt {
  uint32_t src;
  uint32_t dst;
} sps_pkt;

/* Sketch shape.  Notation of the paper:
 *   SRE array (Sec. 3.3): r rows x 2^q SREs, eta u16 cells per SRE, RHFG shift step delta.
 *     Requires 3 <= r <= 32, 6 <= q <= 24, 1 <= delta <= 5, delta < q, (r-2)*delta + q >= 32
 *     (every address bit is recovered, Eq. 6-7), (r-2)*delta <= 31, eta in {8, 16, 32, 64}.
 *   SLE array (Sec. 4): r' rows x 2^q' SLEs, eta' cells per SLE, adjacent SLEs offset by
 *     delta' cells (a row holds 2^q' * delta' + eta' - delta' cells).  Requires
 *     1 <= q' <= 26, 1 <= r' <= 8, eta' a power of two in [16, 65536], delta' a power of
 *     two in [1, eta'].
 *   theta: create-time super point threshold; fixes the sampling depth tau (Eq. 1).
 *   anet_side: 0 -> aip = dst, bip = src;  1 -> aip = src, bip = dst (Def. 1).
 *   seed: expands to the hash seeds (H1, H2, H3, RHFG[0], LH_i).
 *   cand_cap: capacity of the candidate list of one scan (0 -> 262144).
 *   mode: SPS_MODE_SLIDING (u16 stamps, any window) or SPS_MODE_DISCRETE: one bit per
 *     recorder -- the rough estimator RE (Sec. 3.2) and linear estimator LE (Sec. 4) of a
 *     discrete time window, 16 times smaller.  A discrete sketch holds every pair since its
 *     last sps_reset; its scans take window 1 (k = 1), its merge is a bitwise or, and
 *     sps_features is not available.  Recorders are set with 32-bit atomic or.
 *   row_counts: 1 -> the sketch keeps per-row stamp histograms (sliding mode only; see
 *     sps_ingest): scans skip the sweep of the SLE array, ingests cost one 32-bit
 *     compare-and-swap per SLE cell they change.  0 -> plain stores, scans sweep. */
#define SPS_MODE_SLIDING 0u
#define SPS_MODE_DISCRETE 1u
typedef struct sps_params {
  uint32_t q, r, delta, eta;
  uint32_t qp, rp, etap, deltap;
  uint32_t theta;
  uint32_t anet_side;
  uint64_t seed;
  uint32_t cand_cap;
  uint32_t mode;
  uint32_t row_counts;
} sps_params;

/* One reported host (Alg. 8 and the final filter at the end of Sec. 4). */
typedef struct sps_result {
  uint32_t host;    /* aip */
  uint32_t live;    /* |USLE|^k: union-SLE cells within the window */
  uint32_t flags;   /* SPS_F_* */
  uint32_t pad;     /* 0 */
  double estimate;  /* cardinality estimate (Eq. 12 then Eq. 9, or the learned estimator) */
} sps_result;

typedef struct sps_sketch sps_sketch;

/* Bytes of device memory a sketch with these parameters needs (state + scan workspace).
 * Returns SPS_EINVAL for unsupported parameters. */
int sps_sketch_bytes(const sps_params* p, size_t* bytes);

/* Create a sketch on the current HIP device, all recorders 0, current slice 0.
 * d_mem: NULL -> the library allocates (and frees in sps_destroy); otherwise a caller-owned
 * device block of at least sps_sketch_bytes() bytes, 256-byte aligned, that must outlive
 * the sketch.  Synchronous. */
int sps_create(const sps_params* p, void* d_mem, size_t bytes, sps_sketch** out);

/* Destroy a sketch; frees library-owned memory.  Synchronizes the device first. */
int sps_destroy(sps_sketch* s);

/* Set every recorder to 0 and the current slice to 0, and clear the scan counters
 * (stream-ordered fill kernels). */
int sps_reset(sps_sketch* s, void* stream);

/* Per-packet update of a time slice: Alg. 3 (SRE array) and Alg. 6 (SLE array) for each of
 * the n pairs d_pkts[0..n).  Every written recorder receives `slice`.  Requires
 * 1 <= slice <= 65534 and slice >= the current slice (else SPS_ESLICE, nothing written);
 * sets the current slice.  n may be 0.  Because every write carries a stamp no smaller than
 * any stored one, a write equals a max and the result is independent of packet order
 * (Sec. 3.3: recorders need no synchronization).
 * Row counts (params.row_counts = 1): the sketch also keeps, per SLE-array row, how many
 * cells hold each stamp value; the ingest sets SLE cells by 32-bit compare-and-swap and moves
 * one count per cell whose stamp it changes, so scans read the row live counts of Def. 4
 * from these histograms instead of sweeping the SLE array.  Merging other sketches into a
 * sketch, importing a dump or replaying a probe into it stops the counting for that sketch
 * (its scans then sweep the array; results are the same) until its next sps_reset. */
int sps_ingest(sps_sketch* s, const sps_pkt* d_pkts, size_t n, uint32_t slice, void* stream);

/* The same for m sketches (routers) at once, in one launch per 64 routers: sketch h_s[j]
 * ingests the h_n[j] pairs at h_pkts[j].  h_s, h_pkts, h_n are host arrays of m entries; the
 * pair buffers are device memory.  As the paper requires of distributed nodes (Sec. 3.3),
 * all sketches share parameters and seed (else SPS_EMISMATCH) and live on the current
 * device; the slice rules of sps_ingest apply to each (checked for all before anything is
 * written).  Work is cut into tiles of a tuned size so uneven batches share one launch. */
int sps_ingest_batched(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                       uint32_t m, uint32_t slice, void* stream);

/* Launch shape of the ingest kernels: blocks per compute unit for sps_ingest and
 * sps_ingest_batched, the tile (pairs per work item) of sps_ingest_batched, and the number
 * of host classes the pairs are partitioned into (1, 2, 4 or 8): every block reads all pairs
 * and writes those of its class, and blocks of one class run on 8 / host_classes of the 8
 * XCDs, so the recorders of one host are written through as few L2 caches as that allows.
 * Chosen by sps_autotune_ingest or set directly (0 keeps the current value).  Defaults:
 * 16 blocks per CU, tiles of 4096 pairs, 8 host classes.  scan_overlap (not tuned): 1 (the
 * default) runs a scan's sweep of the SLE array for the row live counts in waves of its own
 * inside the candidate search's launch, beside the search; 2 runs the sweep as a kernel of
 * its own after the search.  Either way a scan is one stream of kernels on the caller's
 * stream. */
typedef struct sps_tuning {
  uint32_t blocks_per_cu;
  uint32_t batch_tile;
  uint32_t host_classes;
  uint32_t scan_overlap;
} sps_tuning;
int sps_get_tuning(const sps_sketch* s, sps_tuning* out);
int sps_set_tuning(sps_sketch* s, const sps_tuning* t);

/* Autotuner: ingests the given batch (exactly like sps_ingest_batched; for m == 1 like
 * sps_ingest) once per candidate launch shape, timing each with HIP events, and keeps the
 * fastest shape in every sketch of h_s.  Candidates: blocks per CU in {2, 4, 8, 16, 32, 64}
 * x host classes in {1, 8}, and for m > 1 also tiles in {512, 2048, 8192, 32768}, in that
 * nesting order (blocks outermost).  Re-ingesting the same pairs at the same slice is
 * idempotent, so the resulting state equals a single ingest.  Synchronous.  *best (may be
 * NULL) receives the chosen shape; h_ms (may be NULL, h_ms_cap entries) the time of each
 * candidate in the order tried.  The choice is also recorded in the process's tuning cache
 * under (device architecture, sketch shape, m > 1). */
int sps_autotune_ingest(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                        uint32_t m, uint32_t slice, void* stream, sps_tuning* best,
                        float* h_ms, uint32_t h_ms_cap);

/* Tuning cache: launch shapes chosen by sps_autotune_ingest, keyed by the device
 * architecture name (e.g. "gfx950"), the sketch shape (q, r, delta, eta, q', r', eta',
 * delta', mode) and whether the batched ingest (m > 1) was tuned.  sps_tuning_lookup sets
 * *found to 1 and *out to the entry for `arch` (NULL: the current device's architecture),
 * p and batched, else *found = 0.  sps_tuning_cache_save writes every entry to a JSON file
 * ({"sps_tuning_cache": 1, "entries": [...]}, one entry object per line);
 * sps_tuning_cache_load adds the entries of such a file (replacing equal keys) and returns
 * SPS_EINVAL for a file it cannot read or parse (nothing added); sps_tuning_cache_clear
 * empties the cache.  Thread-safe; host only. */
int sps_tuning_lookup(const char* arch, const sps_params* p, uint32_t batched, sps_tuning* out,
                      int* found);
int sps_tuning_cache_save(const char* path);
int sps_tuning_cache_load(const char* path);
int sps_tuning_cache_clear(void);

/* ---- stream capture ------------------------------------------------------------------------
 * Every library call that only launches kernels (ingest, batched ingest, reset, merge,
 * scan_async, features, estimate_hosts, mlp_*) may be captured.  sps_graph_begin starts
 * capturing `stream`; sps_graph_end ends it and instantiates the graph; sps_graph_launch
 * replays it on a stream.  Host-side state (the current slice) is updated when the call is
 * captured, so a captured slice is meant to be launched once (replays of an ingest are
 * idempotent). */
typedef struct sps_graph sps_graph;
int sps_graph_begin(void* stream);
int sps_graph_end(void* stream, sps_graph** out);
/* End capturing `stream` and make g run the newly captured work: when the new capture has
 * the same topology as g's graph (same kernels in the same order; only arguments differ),
 * g's executable graph is updated in place (hipGraphExecUpdate, no instantiation) and
 * *updated (may be NULL) is set to 1; otherwise g is re-instantiated from the new capture
 * and *updated is 0.  g must not be executing (wait for its last launch first). */
int sps_graph_end_update(void* stream, sps_graph* g, int* updated);
int sps_graph_launch(sps_graph* g, void* stream);
int sps_graph_destroy(sps_graph* g);

/* Time passes with no packets: set the current slice (same rules as sps_ingest). */
int sps_advance(sps_sketch* s, uint32_t slice);

/* Rebase of the time base (Sec. 3.2: the paper's u16 distance recorders saturate; u16
 * stamps run out at slice 65534 instead).  Every stamp v of the SRE and SLE arrays becomes
 * max(v - offset, 0) -- recorders last written at or before slice `offset` read as never
 * written -- and the current slice becomes cur - offset; later ingests number their slices
 * in the new base.  Every scan, feature and estimate with a window of at most cur - offset
 * slices is unchanged; longer windows lose the slices shifted out.  Requires
 * offset <= cur (else SPS_ESLICE, nothing changed).  Sketches that will be merged must be
 * rebased by the same offset.  Discrete-mode sketches hold no stamps: only the current
 * slice moves.  Stream-ordered, one fill-type kernel, capturable. */
int sps_rebase(sps_sketch* s, uint32_t offset, void* stream);

/* Distributed merge (Alg. 2 and Alg. 7): cell-wise, dst <- max(dst, src[0..nsrc)) over the
 * SRE and SLE arrays (the most recent observation of any router wins), and the current
 * slice becomes the largest of all.  h_src is a host array of nsrc sketches with parameters
 * and seed equal to dst's (else SPS_EMISMATCH).  dst may appear in h_src. */
int sps_merge(sps_sketch* dst, const sps_sketch* const* h_src, uint32_t nsrc, void* stream);

/* End-of-slice scan with a window of `window` slices ending at the current slice:
 * k-weights of every SRE and row setting factors SF(i,k) (Sec. 3.3, Def. 4); hot SREs; the
 * candidate hosts whose SRE is hot in every row, recovered through the RHFG (Alg. 4-5,
 * Eq. 6-7); per candidate the union SLE, the noise-corrected weight (Eq. 12) and the linear
 * counting estimate (Eq. 9); the hosts whose estimate is >= threshold, ascending by host.
 * Synchronous: h_out is host memory of `cap` results; *n_out receives the number of kept
 * hosts.  If that exceeds cap, returns SPS_ECAPACITY with *n_out = the required count and
 * nothing written; if the candidate list overflows cand_cap, returns SPS_ECAPACITY with
 * *n_out = 0.  1 <= window <= 65534. */
int sps_scan(sps_sketch* s, uint32_t window, double threshold, sps_result* h_out, size_t cap,
             size_t* n_out, void* stream);

/* Asynchronous scan: the same pipeline with results in device memory d_out (cap entries,
 * ascending by host; entries beyond cap are dropped and flagged) and SPS_INFO_WORDS u32
 * counters in device memory d_info.  Launches a fixed sequence of kernels with no host
 * synchronization or allocation (suitable for stream capture). */
int sps_scan_async(sps_sketch* s, uint32_t window, double threshold, sps_result* d_out,
                   size_t cap, uint32_t* d_info, void* stream);

/* Per-age features of given hosts for the learned estimator: d_x[h * window + a] = number
 * of union-SLE cells of host d_hosts[h] last written within the newest a+1 slices
 * (a < window; d_x[h*window + window-1] = |USLE|^k).  1 <= window <= 32. */
int sps_features(const sps_sketch* s, const uint32_t* d_hosts, size_t n, uint32_t window,
                 uint32_t* d_x, void* stream);

/* Estimates of given hosts (no recovery, no filter): for each d_hosts[h] the union SLE,
 * Eq. 12 and Eq. 9 (or the attached learned estimator) over a window of `window` slices
 * ending at the current slice, written to d_out[h] in input order.  1 <= window <= 65534. */
int sps_estimate_hosts(sps_sketch* s, const uint32_t* d_hosts, size_t n, uint32_t window,
                       sps_result* d_out, void* stream);

/* ---- learned cardinality estimator (an addition to the paper's method) --------------------
 * A 3-layer perceptron maps the per-age union-SLE live counts x_0..x_9 of a host (window 10,
 * each divided by eta') through 64 and 64 ReLU units to the natural log of its cardinality.
 * Parameters: SPS_MLP_PARAMS float32 in the order W1 (64 x 10, row-major), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (1 x 64), b3 (1). */
#define SPS_MLP_IN 10
#define SPS_MLP_HIDDEN 64
#define SPS_MLP_PARAMS (SPS_MLP_HIDDEN * SPS_MLP_IN + SPS_MLP_HIDDEN + SPS_MLP_HIDDEN * SPS_MLP_HIDDEN + SPS_MLP_HIDDEN + SPS_MLP_HIDDEN + 1)

/* Attach a trained network to the sketch's scans and host estimates (d_weights NULL
 * detaches).  d_weights: caller-owned device buffer, read by every later scan.  The network
 * replaces linear counting for a host only when its window is 10 slices, |USLE|^k >=
 * min_live, every feature x_a / eta' lies in [h_feat_lo[a], h_feat_hi[a]] (host arrays of
 * 10 floats, copied), x_0 < eta' - 1 (some age is unsaturated), and the output lies in
 * [0, log(max_card)]; otherwise linear counting is kept and SPS_F_LC_FALLBACK is set.  When
 * linear counting is saturated (SPS_F_SATURATED) the network can only raise its estimate.
 * Inference rounds weights and activations to bfloat16 and accumulates in float32. */
int sps_attach_mlp(sps_sketch* s, const float* d_weights, const float* h_feat_lo,
                   const float* h_feat_hi, uint32_t min_live, double max_card);

/* Bytes of the workspace sps_mlp_grad needs for a batch of n samples. */
int sps_mlp_work_bytes(size_t n, size_t* bytes);

/* Gradient of the mean squared error of log-cardinality predictions over a batch:
 * samples d_idx[0..n) (or 0..n when d_idx is NULL) of the feature matrix d_feat (u32,
 * n_rows x 10 counts, divided by eta' inside) with targets d_target (float, log of the true
 * cardinality).  Writes SPS_MLP_PARAMS floats to d_grad and the batch loss to d_loss
 * (may be NULL).  d_work: sps_mlp_work_bytes(n) bytes of device memory.  Deterministic:
 * partial gradients are summed in a fixed order. */
int sps_mlp_grad(const float* d_w, const uint32_t* d_feat, const float* d_target,
                 const uint32_t* d_idx, size_t n, uint32_t etap, void* d_work, float* d_grad,
                 float* d_loss, void* stream);

/* Allocation-free variant of sps_mlp_grad, for callers that cannot allocate device memory
 * or pass a workspace (code under stream capture, tight training or serving loops): the
 * same kernels and the same result, bit for bit, with the per-wave partial gradients kept in
 * a static device array of the library (about 5 MiB per device, held until the process
 * exits) instead of d_work.  n <= SPS_MLP_NOALLOC_MAX_N (else SPS_ECAPACITY, nothing
 * launched).  Calls no allocator.  All calls on one device share that array: calls that
 * overlap in time on one device (different streams or threads) race and must be serialized
 * by the caller.  The first call on a device looks up the array's address (synchronous). */
#define SPS_MLP_NOALLOC_MAX_N 4096
int sps_mlp_grad_noalloc(const float* d_w, const uint32_t* d_feat, const float* d_target,
                         const uint32_t* d_idx, size_t n, uint32_t etap, float* d_grad,
                         float* d_loss, void* stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected; step counts from 1) on d_w with moment
 * buffers d_m, d_v (SPS_MLP_PARAMS floats each). */
int sps_mlp_adam(float* d_w, float* d_m, float* d_v, const float* d_grad, uint32_t step,
                 float lr, double beta1, double beta2, float eps, void* stream);

/* Batched inference: d_y[s] = predicted log cardinality of feature row s (n rows of 10 u32
 * counts).  bf16 != 0 uses the scan's precision (bfloat16 weights and activations, float32
 * accumulation); 0 uses float32 throughout. */
int sps_mlp_forward(const float* d_w, const uint32_t* d_feat, size_t n, uint32_t etap, int bf16,
                    float* d_y, void* stream);

/* Bytes of a state dump (header + SRE array + SLE array, dense). */
int sps_state_bytes(const sps_sketch* s, size_t* bytes);

/* Bit-exact state dump into host memory h_buf (checkpoint).  Layout: 64-byte header
 * (magic "SPS1", params, current slice), then the SRE array, then the SLE array.  Sliding
 * mode: u16 SRE[r][2^q][eta], then u16 SLE[r'][L'].  Discrete mode: the SRE bits (bit
 * ((i << q) + col) * eta + e, little-endian u32 words), then for every SLE row
 * ceil(L' / 32) u32 words of bits (bit j = cell j).  Synchronous. */
int sps_export(const sps_sketch* s, void* h_buf, size_t bytes, void* stream);

/* Restore a dump written by sps_export of a sketch with identical parameters and seed
 * (else SPS_EMISMATCH).  Synchronous. */
int sps_import(sps_sketch* s, const void* h_buf, size_t bytes, void* stream);

/* Current slice of the sketch (0 before any ingest). */
int sps_current_slice(const sps_sketch* s, uint32_t* slice);

/* Derived constants: tau (Eq. 1), hot cut ceil(rho*eta) (Sec. 3.2), SLE row length L'. */
int sps_derived(const sps_sketch* s, uint32_t* tau, uint32_t* hot_cut, uint64_t* row_len);

/* Internal scan buffers of the last scan, for inspection: which = 0 hot bitmap
 * (r x 2^q bits as u32 words, bit j of word w = SRE 32w + j in row-major order), 1 candidate
 * list (u32, unordered, at most cand_cap), 2 SLE row live counts (r' x u32), 3 the per-row
 * stamp histograms (r' x 65536 u32: entry [i][v] = cells of SLE-array row i with stamp v,
 * v >= 1; size 0 when the sketch does not keep them, see sps_ingest).  Copies
 * min(bytes, size) bytes to host memory h_buf (may be NULL to query); *size gets the full
 * size.  Synchronous. */
int sps_debug_copy(const sps_sketch* s, int which, void* h_buf, size_t bytes, size_t* size,
                   void* stream);

/* ---- measurement ------------------------------------------------------------------------ */
/* Stage timing with HIP events on the stream each kernel is launched on.  While enabled
 * (process-wide), every library kernel launch of a stage whose bit is set in `stage_mask`
 * (bit SPS_STAGE_x; 0 disables, ~0 records all) is bracketed by a pair of events, and
 * SPS_STAGE_SCAN brackets a whole scan.  Reading synchronizes on the recorded events and
 * returns, per stage, the summed milliseconds and the number of launches since the last
 * read, then clears.  Launches on a capturing stream are not recorded.  h_ms / h_launches:
 * host arrays of nstages entries (stages beyond SPS_NSTAGES are zeroed). */
#define SPS_STAGE_INGEST 0
#define SPS_STAGE_INGEST_BATCHED 1
#define SPS_STAGE_MERGE 2
#define SPS_STAGE_FILL 3
#define SPS_STAGE_SCAN_RESET 4
#define SPS_STAGE_SCAN_STATS 5
#define SPS_STAGE_JOIN 6
#define SPS_STAGE_ESTIMATE 7
#define SPS_STAGE_SORT 8
#define SPS_STAGE_FEATURES 9
#define SPS_STAGE_PROBE 10
#define SPS_STAGE_MLP 11
#define SPS_STAGE_SCAN 12
#define SPS_STAGE_REBASE 13
#define SPS_STAGE_SCAN_ROWS 14  /* a scan's row-count sweep when it is a kernel of its own */
#define SPS_NSTAGES 15
int sps_profile_enable(uint32_t stage_mask);
int sps_profile_read(double* h_ms, uint32_t* h_launches, int nstages);

/* Roofline probes (measurement only, not part of the method).
 * sps_probe_scatter: n_stores u16 stores of `value` at uniformly random cells of a device
 *   array of `cells` u16 (addresses from a counter hash of the store index and seed), one
 *   store per lane -- the access pattern of the ingest with no hashing of packets.
 * sps_probe_stream: reads `bytes` (multiple of 16) of device memory with 16-byte lane loads
 *   and writes one u32 checksum to d_sum -- the access pattern of the scan's first stage. */
/* Replay probe of the ingest (measurement only).  sps_probe_replay_record writes to d_cells
 * (device, cap u32 entries) every state cell that sps_ingest(s, d_pkts, n) would write, as an
 * index in u16 units into the SRE array followed by the SLE array (the SLE array starts at
 * its offset in the sketch's block), grouped into 8 regions by the ingest's host class;
 * h_class_off (host, 9 entries) receives the region offsets and, in h_class_off[8], the
 * total.  Returns SPS_ECAPACITY (offsets filled, nothing recorded) when the total exceeds
 * cap.  Synchronous; allocates 64 bytes of device memory for its counters.  sps_probe_replay
 * stores `value` into every recorded cell of s's state, region c from the blocks the ingest
 * gives host class c (the same XCD), with the ingest's launch shape: the ingest's stores
 * without reading or hashing pairs.  Sliding mode only. */
int sps_probe_replay_record(const sps_sketch* s, const sps_pkt* d_pkts, size_t n,
                            uint32_t* d_cells, size_t cap, uint64_t* h_class_off, void* stream);
int sps_probe_replay(sps_sketch* s, const uint32_t* d_cells, const uint64_t* h_class_off,
                     uint16_t value, void* stream);
int sps_probe_scatter(uint16_t* d_cells, uint64_t cells, uint64_t n_stores, uint32_t seed,
                      uint16_t value, void* stream);
int sps_probe_stream(const void* d_buf, uint64_t bytes, uint32_t* d_sum, void* stream);

/* Completion time of stream work: when `stream` reaches this point (everything queued
 * before it has finished), the host's CLOCK_MONOTONIC time in seconds is stored to *h_time
 * (host memory that must stay valid until then).  A host function on the stream; the stream
 * waits for it.  Not for use under stream capture. */
int sps_stream_host_time(double* h_time, void* stream);

/* Wait for all work the library queued on `stream`; reports asynchronous HIP errors. */
int sps_sync(void* stream);

/* Human-readable text of an error code. */
const char* sps_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SPS_H */
