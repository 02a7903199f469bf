// sps_internal.h -- device-side view of a sketch, shared by the kernels and the runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include "sps.h"

namespace sps {

constexpr int kMaxRP = 8;      // SLE-array rows supported
constexpr int kMaxR = 32;      // SRE-array rows supported
constexpr int kMaxBatch = 64;  // routers per batched launch
constexpr int kMaxMerge = 32;  // sources per merge launch (more are chained)
constexpr uint32_t kHistBins = 65536;  // one bin per u16 stamp value
// partial row counts of a scan's sweep per row: one per block of the candidate search, or one
// per wave of k_scan_rows (4 per CU), at most
constexpr uint32_t kRowsPartWaves = 4096;
// waves of a scan's estimate launch; wave w handles candidates w, w + kEstWaves, ... and
// keeps its hosts in a region of its own of the kept list
constexpr uint32_t kEstWaves = 2048;
// entries of one estimate wave's region of the kept list: room for every candidate it can get
inline __host__ __device__ uint32_t kept_region(uint32_t cand_cap) {
  return (cand_cap + kEstWaves - 1) / kEstWaves;
}

// Per-scan counters kept in device memory (one 256-byte block per sketch).  Every scan
// leaves the working fields zero when it ends (its last kernel clears them), so a scan
// needs no reset launch and replays of a captured scan start clean.
struct Ctrl {
  uint32_t row_live[kMaxRP];  // live cells of every SLE-array row (Def. 4 numerators)
  uint32_t hse_count[2];      // hot SREs found in rows 0 and 1
  uint32_t n_cand;            // candidates recovered (counts past the capacity)
  uint32_t n_kept;            // hosts kept by the final filter (set by the ordering kernel)
  unsigned long long join_nodes;  // nodes the candidate search expanded
  uint32_t sort_done;     // blocks of the ordering kernel done with their tiles
  uint32_t pad0;
  uint32_t join_skipped;  // the candidate search was not run: its expected size was too large
  uint32_t pad1;
  uint32_t hot_rows[kMaxR];  // hot SREs of every row
  // copies of the last scan's counters, for inspection (not cleared)
  uint32_t last_row_live[kMaxRP];
  uint32_t last_n_cand;
  uint32_t last_hse[2];
  uint32_t pad[64 - 2 * kMaxRP - 4 - 2 - 2 - 2 - kMaxR - 3];
};
constexpr uint32_t kCtrlWorkingWords = kMaxRP + 4 + 2 + 2 + 2 + kMaxR;  // cleared after a scan
static_assert(sizeof(Ctrl) == 256, "Ctrl is one 256-byte block");

// Learned-estimator attachment (weights in device memory, bounds by value).
struct MlpRef {
  const float* w;         // SPS_MLP_PARAMS floats, or null
  float lo[SPS_MLP_IN];   // training range of every feature
  float hi[SPS_MLP_IN];
  float log_max;          // outputs above log(max cardinality) fall back
  uint32_t min_live;      // the network is used only when |USLE|^k >= min_live
};

// Everything a kernel needs to know about one sketch; passed by value.
struct Dev {
  uint16_t* sre;          // [r][2^q][eta] stamps (discrete mode: bits, as u32 words)
  uint16_t* slea;         // [r'][row_stride] cells >= row_len are padding (always 0)
  uint32_t* hot;          // [r][2^q / 32] hot-SRE bitmap
  uint32_t* hot_t;        // [r][2^q / 32] the same bits transposed for the join: bit
                          // (low << delta) + top of row i is hot_i[low | top << (q - delta)]
  uint32_t* hse;          // [2][2^q] hot-SRE column lists of rows 0 and 1
  uint32_t* cand;         // [cand_cap] recovered candidates
  sps_result* kept;       // [kEstWaves][kept_region(cand_cap)] kept hosts: estimate wave w
                          // leaves its wave_kept[w] hosts at the start of region w
  uint32_t* wave_kept;    // [kEstWaves] hosts each estimate wave kept in the last scan
  uint64_t* skeys;        // [cand_cap] (host << 32 | index into kept), sorted per 4096-tile
  Ctrl* ctrl;
  uint32_t* rows_part;    // [kMaxRP][kRowsPartWaves] partial row live counts of a scan's
                          // sweep, per block or per wave (summed by the estimate)
  uint32_t* hist;         // [r'][kHistBins] per-row stamp histograms: hist[i][v] = cells of
                          // SLE-array row i whose stamp is v (v >= 1; bin 0 unused)
  uint64_t row_len;       // L' = 2^q' delta' + eta' - delta'
  uint64_t row_stride;    // cells between SLE-array rows (row_len rounded up to 64)
  uint32_t q, r, delta, eta;
  uint32_t qp, rp, etap, deltap;
  uint32_t tau_mask;      // low tau bits; a pair is sampled when H1 has them all clear
  uint32_t hot_cut;
  uint32_t anet_side;
  uint32_t cand_cap;
  uint32_t mode;          // SPS_MODE_SLIDING: u16 stamps; SPS_MODE_DISCRETE: one bit per cell
  uint32_t seed_h1, seed_h2, seed_h3, seed_rhfg0;
  uint32_t seed_lh[kMaxRP];
};

// ---- hashes (the project's specification: fmix32 of the key xor a per-function seed) ----
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// Input encoding of the learned estimator: the count x of live union-SLE cells at one age is
// turned into the log of that age's own linear-counting estimate, scaled to about [0, 1]:
// phi = log1p(-eta' log1p(-x / (eta' + 1))) / 8  (x <= eta', so the argument never reaches 1).
__device__ __forceinline__ float mlp_encode(uint32_t x, uint32_t etap) {
  const float u = (float)x / (float)(etap + 1u);
  return log1pf(-(float)etap * log1pf(-u)) * 0.125f;
}

// Stage timing (sps_api.hip), while profiling is on and the stream is not being captured.
// A marker scope brackets whatever it encloses with two recorded events.  A kernel scope
// records nothing itself: its two events go to the one launch it encloses (launch_k), which
// sets them from the kernel's own start and end, so timing adds no packets to the stream.
class ProfScope {
 public:
  enum Kind { kMarkers, kKernel };
  ProfScope(int stage, hipStream_t st, Kind kind = kMarkers);
  ~ProfScope();
  bool kernel_timed() const { return kind_ == kKernel && ev0_ != nullptr; }
  hipEvent_t start() const { return static_cast<hipEvent_t>(ev0_); }
  hipEvent_t stop() const { return static_cast<hipEvent_t>(ev1_); }

 private:
  int stage_;
  hipStream_t st_;
  Kind kind_;
  void* ev0_;
  void* ev1_;
};

// One launch, timed by its own dispatch when `ps` is a timed kernel scope.
template <typename F, typename... Args>
inline void launch_k(const ProfScope& ps, F kernel, dim3 grid, dim3 block, uint32_t lds,
                     hipStream_t st, Args... args) {
  if (ps.kernel_timed())
    hipExtLaunchKernelGGL(kernel, grid, block, lds, st, ps.start(), ps.stop(), 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

// Launchers (sps_kernels.hip).
// track: keep d.hist exact (SLE cells set by compare-and-swap, each stamp change counted)
hipError_t launch_ingest(const Dev& d, const sps_pkt* pkts, uint64_t n, uint16_t stamp,
                         int blocks, int threads, uint32_t host_classes, bool track,
                         hipStream_t st);

struct BatchItem {
  uint16_t* sre;
  uint16_t* slea;
  uint32_t* hist;  // the sketch's stamp histograms, or null when they are not kept
  const sps_pkt* pkts;
  uint64_t n;
};
struct BatchTable {
  BatchItem item[kMaxBatch];
  uint64_t tile_start[kMaxBatch + 1];  // prefix sums of tiles per router
};
hipError_t launch_ingest_batched(const Dev& shape, const BatchTable& t, uint32_t m,
                                 uint32_t tile, uint16_t stamp, int blocks, int threads,
                                 uint32_t host_classes, hipStream_t st);
hipError_t launch_fill_zero(void* p, uint64_t bytes, hipStream_t st);
hipError_t launch_scan_reset(const Dev& d, bool with_table, hipStream_t st);
hipError_t launch_rebase(uint16_t* p, uint64_t bytes, uint32_t offset, hipStream_t st);
hipError_t launch_hist_rebase(uint32_t* hist, uint32_t rows, uint32_t offset, hipStream_t st);
hipError_t launch_merge(uint16_t* dst, const uint16_t* const* srcs, uint32_t nsrc,
                        uint64_t bytes, bool bits, hipStream_t st);
hipError_t prepare_join();  // allows the join its LDS (call before the first scan)
// Where a scan's row-count sweep runs: in waves of its own inside the candidate search's
// launch, or as a kernel of its own after the search.
enum ScanMode : uint32_t { kScanFused = 1, kScanSerial = 2 };
// use_hist: row live counts from d.hist instead of a sweep of the SLE array
hipError_t launch_scan(const Dev& d, uint32_t cur, uint32_t window, double threshold,
                       sps_result* out, uint32_t cap, uint32_t* info, const MlpRef& mlp,
                       bool use_hist, uint32_t mode, int n_cu, hipStream_t st);
// Region offsets of the replay probe's cell list, one region per host class (XCD).
struct ClassOffsets {
  uint64_t off[9];
};
hipError_t launch_probe_record(const Dev& d, const sps_pkt* pkts, uint64_t n, uint32_t sle_off,
                               uint32_t* cells, unsigned long long* pos, bool fill,
                               hipStream_t st);
hipError_t launch_probe_replay(uint16_t* state, const uint32_t* cells, const ClassOffsets& co,
                               uint16_t value, int blocks, hipStream_t st);
hipError_t launch_probe_scatter(uint16_t* cells, uint64_t n_cells, uint64_t n_stores,
                                uint32_t seed, uint16_t value, int n_cu, hipStream_t st);
hipError_t launch_probe_stream(const void* buf, uint64_t bytes, uint32_t* sum, int n_cu,
                               hipStream_t st);
hipError_t launch_features(const Dev& d, uint32_t cur, uint32_t window, const uint32_t* hosts,
                           uint64_t n, uint32_t* x, int n_cu, hipStream_t st);
hipError_t launch_estimate_hosts(const Dev& d, uint32_t cur, uint32_t window,
                                 const uint32_t* hosts, uint32_t n, sps_result* out,
                                 const MlpRef& mlp, bool use_hist, int n_cu, hipStream_t st);

// Learned estimator (sps_mlp.hip).
uint32_t mlp_grad_waves(uint32_t n);
// Largest batch of the allocation-free gradient call (its workspace is a static device array).
constexpr uint32_t kMlpNoAllocMaxN = SPS_MLP_NOALLOC_MAX_N;
hipError_t mlp_scratch(float** out, uint64_t* floats);
hipError_t launch_mlp_grad(const float* w, const uint32_t* feat, const float* target,
                           const uint32_t* idx, uint32_t n, uint32_t etap, float* partial,
                           float* partial_loss, float* grad, float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* w, float* m, float* v, const float* grad, uint32_t step,
                           float lr, double b1, double b2, float eps, hipStream_t st);
hipError_t launch_mlp_forward(const float* w, const uint32_t* feat, uint32_t n, uint32_t etap,
                              int bf16, float* y, int n_cu, hipStream_t st);

}  // namespace sps
