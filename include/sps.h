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
 * stamp >= max(1, cur - k + 1).  Slices are numbered 1..65534.
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
#define SPS_INFO_FLAGS 2     /* bit 0: candidate buffer overflow; bit 1: result buffer overflow */
#define SPS_INFO_HSE0 3      /* hot SREs in row 0 */
#define SPS_INFO_HSE1 4      /* hot SREs in row 1 */
#define SPS_INFO_WORDS 8

/* One IP pair as the 8-byte record the paper buffers per packet (Sec. 3.3): (src, dst). */
typedef struct sps_pkt {
  uint32_t src;
  uint32_t dst;
} sps_pkt;

/* Sketch shape.  Notation of the paper:
 *   SRE array (Sec. 3.3): r rows x 2^q SREs, eta u16 cells per SRE, RHFG shift step delta.
 *     Requires 3 <= r <= 32, 1 <= delta < q <= 24, (r-2)*delta + q >= 32 (every address bit
 *     is recovered, Eq. 6-7), (r-2)*delta <= 31, eta in {8, 16, 32, 64}.
 *   SLE array (Sec. 4): r' rows x 2^q' SLEs, eta' cells per SLE, adjacent SLEs offset by
 *     delta' cells (a row holds 2^q' * delta' + eta' - delta' cells).  Requires
 *     1 <= q' <= 26, 1 <= r' <= 8, eta' a power of two in [16, 65536], delta' a power of
 *     two in [1, eta'].
 *   theta: create-time super point threshold; fixes the sampling depth tau (Eq. 1).
 *   anet_side: 0 -> aip = dst, bip = src;  1 -> aip = src, bip = dst (Def. 1).
 *   seed: expands to the hash seeds (H1, H2, H3, RHFG[0], LH_i).
 *   cand_cap: capacity of the candidate list of one scan (0 -> 262144). */
typedef struct sps_params {
  uint32_t q, r, delta, eta;
  uint32_t qp, rp, etap, deltap;
  uint32_t theta;
  uint32_t anet_side;
  uint64_t seed;
  uint32_t cand_cap;
  uint32_t reserved;
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

/* Set every recorder to 0 and the current slice to 0 (stream-ordered fill kernel). */
int sps_reset(sps_sketch* s, void* stream);

/* Per-packet update of a time slice: Alg. 3 (SRE array) and Alg. 6 (SLE array) for each of
 * the n pairs d_pkts[0..n).  Every written recorder receives `slice`.  Requires
 * 1 <= slice <= 65534 and slice >= the current slice (else SPS_ESLICE, nothing written);
 * sets the current slice.  n may be 0.  Because every write carries a stamp no smaller than
 * any stored one, plain stores equal a max and the result is independent of packet order
 * (Sec. 3.3: recorders need no synchronization). */
int sps_ingest(sps_sketch* s, const sps_pkt* d_pkts, size_t n, uint32_t slice, void* stream);

/* The same for m sketches (routers) at once, in one persistent launch: sketch s[j] ingests
 * the n[j] pairs at d_pkts[j].  h_s, h_pkts, h_n are host arrays of m entries; the
 * pair buffers are device memory.  All sketches must be on the current device; the slice
 * rules of sps_ingest apply to each (checked for all before anything is written). */
int sps_ingest_batched(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                       uint32_t m, uint32_t slice, void* stream);

/* Time passes with no packets: set the current slice (same rules as sps_ingest). */
int sps_advance(sps_sketch* s, uint32_t slice);

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

/* Attach a learned estimator to the sketch's scans (NULL detaches).  d_weights: device
 * buffer of SPS_MLP_PARAMS floats in the order W1(64x10), b1, W2(64x64), b2, W3(1x64), b3,
 * caller-owned, read by every later scan.  feat_lo/feat_hi: per-feature bounds of the
 * training range (host arrays of 10 floats, copied); outside them, or when every feature is
 * saturated, or when the output leaves [0, log(max_card)], linear counting is used.
 * Only scans with window 10 use it. */
#define SPS_MLP_IN 10
#define SPS_MLP_HIDDEN 64
#define SPS_MLP_PARAMS (SPS_MLP_HIDDEN * SPS_MLP_IN + SPS_MLP_HIDDEN + SPS_MLP_HIDDEN * SPS_MLP_HIDDEN + SPS_MLP_HIDDEN + SPS_MLP_HIDDEN + 1)
int sps_attach_mlp(sps_sketch* s, const float* d_weights, const float* h_feat_lo,
                   const float* h_feat_hi, double max_card);

/* Bytes of a state dump (header + SRE array + SLE array, dense). */
int sps_state_bytes(const sps_sketch* s, size_t* bytes);

/* Bit-exact state dump into host memory h_buf (checkpoint).  Layout: 64-byte header
 * (magic "SPS1", params, current slice), then u16 SRE[r][2^q][eta], then u16 SLE[r'][L'].
 * Synchronous. */
int sps_export(const sps_sketch* s, void* h_buf, size_t bytes, void* stream);

/* Restore a dump written by sps_export of a sketch with identical parameters and seed
 * (else SPS_EMISMATCH).  Synchronous. */
int sps_import(sps_sketch* s, const void* h_buf, size_t bytes, void* stream);

/* Current slice of the sketch (0 before any ingest). */
int sps_current_slice(const sps_sketch* s, uint32_t* slice);

/* Derived constants: tau (Eq. 1), hot cut ceil(rho*eta) (Sec. 3.2), SLE row length L'. */
int sps_derived(const sps_sketch* s, uint32_t* tau, uint32_t* hot_cut, uint64_t* row_len);

/* Internal scan buffers of the last scan, for inspection: which = 0 hot bitmap
 * (r x 2^q bits as u32 words), 1 candidate list (u32, unordered), 2 SLE row live counts
 * (r' x u64 ... stored as u32).  Copies min(bytes, size) bytes to host memory; *size gets
 * the full size.  Synchronous. */
int sps_debug_copy(const sps_sketch* s, int which, void* h_buf, size_t bytes, size_t* size,
                   void* stream);

/* Wait for all work the library queued on `stream`; reports asynchronous HIP errors. */
int sps_sync(void* stream);

/* Human-readable text of an error code. */
const char* sps_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SPS_H */
