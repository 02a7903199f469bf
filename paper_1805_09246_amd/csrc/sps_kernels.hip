// sps_kernels.hip -- gfx950 kernels of the sliding super point sketch (wave64).
//
// Ingest (Alg. 3 + Alg. 6), merge (Alg. 2 + Alg. 7), end-of-slice scan (k-weights and hot
// SREs of Sec. 3.3 / Def. 4, candidate recovery of Alg. 4-5 through Eq. 6-7, union SLE and
// estimate of Alg. 8 with Eq. 12 and Eq. 9, final filter), and the per-age features.
// Recorders are u16 stamps (slice of the last write, 0 = never); see include/sps.h.
#include <hip/hip_runtime.h>

#include "sps_internal.h"

namespace sps {

constexpr int kWave = 64;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Inclusive prefix sum over the 64 lanes with DPP moves: shifts of 1, 2, 4 and 8 lanes within
// each 16-lane row, then the last lane of row 0 (and of row 2) added to row 1 (and 3), then
// the last lane of row 1 added to rows 2 and 3.  Lanes whose source is outside the row keep
// the `old` operand, 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// ---------------------------------------------------------------------------------------
// Ingest.  One lane per IP pair: H3(bip) picks the SLE cell, LH_i(aip) the SLE of row i
// (Alg. 6); when LSB(H1(bip)) >= tau (low tau bits of H1 clear), H2(bip) picks the SRE
// cell and RHFG[i](aip) the SRE of row i (Alg. 3, Eq. 6 with shift (i-1)*delta).  Every
// store writes the same stamp, so plain u16 stores are race-free maxima.
// ---------------------------------------------------------------------------------------
// Cells a pair writes: emit(cell, false, i) for its SLE cell in each row i < r' (index into
// the SLE array), then, when it is sampled, emit(cell, true, i) for its SRE cell in each row
// i < r (index into the SRE array).  Rows come in the same order on every lane.
template <class Emit>
__device__ __forceinline__ void pair_cells(const Dev& d, uint32_t src, uint32_t dst, Emit&& emit) {
  const uint32_t aip = d.anet_side ? src : dst;
  const uint32_t bip = d.anet_side ? dst : src;
  const uint32_t z = fmix32(bip ^ d.seed_h3) & (d.etap - 1u);
  const uint32_t qpmask = (1u << d.qp) - 1u;
#pragma unroll
  for (int i = 0; i < kMaxRP; ++i) {
    if (i < (int)d.rp) {
      const uint32_t j = fmix32(aip ^ d.seed_lh[i]) & qpmask;
      emit((uint64_t)i * d.row_stride + (uint64_t)j * d.deltap + z, false, (uint32_t)i);
    }
  }
  const uint32_t h1 = fmix32(bip ^ d.seed_h1);
  if ((h1 & d.tau_mask) == 0u) {
    const uint32_t e = fmix32(bip ^ d.seed_h2) & (d.eta - 1u);
    const uint32_t qmask = (1u << d.q) - 1u;
    const uint32_t c0 = fmix32(aip ^ d.seed_rhfg0) & qmask;
    for (uint32_t i = 0; i < d.r; ++i) {
      const uint32_t col = i == 0 ? c0 : ((aip >> ((i - 1u) * d.delta)) ^ c0) & qmask;
      emit(((((uint64_t)i << d.q) + col) << __builtin_ctz(d.eta)) + e, true, i);
    }
  }
}

// Per-row stamp histograms kept by the ingest (sliding mode).  hist[i][v] counts the cells
// of SLE-array row i whose stamp is v, so the live count of row i in a window [lo, cur]
// (Def. 4) is the sum of bins lo..cur and a scan need not sweep the array.  An ingest at
// stamp s changes a cell only from an older stamp `old` to s, once per cell and launch, so
// each change moves one count from bin old to bin s.  The change is made with a 32-bit
// compare-and-swap on the word holding the u16 cell: the lane whose swap succeeds is the one
// that changed the cell, and every other lane sees s already (or a failed swap returns the
// word, which changes at most twice per launch: once per cell).  Counts are gathered per
// block in LDS -- additions to bin s per row, removals by age s - old for ages below
// kHistNear -- and added to the histograms once per block; older removals go straight to
// their bins.
constexpr uint32_t kHistNear = 128;
struct HistAgg {
  uint32_t inc[kMaxRP];
  uint32_t dec[kMaxRP][kHistNear];
};

__device__ __forceinline__ void hist_agg_clear(HistAgg* a) {
  for (uint32_t j = threadIdx.x; j < (uint32_t)kMaxRP * (kHistNear + 1u); j += blockDim.x) {
    if (j < (uint32_t)kMaxRP) a->inc[j] = 0u;
    else a->dec[(j - kMaxRP) / kHistNear][(j - kMaxRP) % kHistNear] = 0u;
  }
}

// The block's gathered counts into hist (called by every thread of the block, after a
// barrier that follows the block's last change); the LDS counts are left zero.
__device__ __forceinline__ void hist_agg_flush(HistAgg* a, uint32_t* hist, uint32_t rp,
                                               uint32_t stamp) {
  for (uint32_t j = threadIdx.x; j < rp * (kHistNear + 1u); j += blockDim.x) {
    if (j < rp) {
      const uint32_t c = a->inc[j];
      if (c) atomicAdd(&hist[(uint64_t)j * kHistBins + stamp], c);
      a->inc[j] = 0u;
    } else {
      const uint32_t row = (j - rp) / kHistNear, age = (j - rp) % kHistNear;
      const uint32_t c = a->dec[row][age];
      if (c) atomicSub(&hist[(uint64_t)row * kHistBins + stamp - age], c);  // age < stamp
      a->dec[row][age] = 0u;
    }
  }
}

// Stamp `stamp` into SLE cell `cell` of row `row`, counting the change.
__device__ __forceinline__ void tracked_sle_store(uint16_t* __restrict__ slea, uint32_t* hist,
                                                  HistAgg* agg, uint64_t cell, uint32_t row,
                                                  uint32_t stamp) {
  uint32_t* const w = reinterpret_cast<uint32_t*>(slea) + (cell >> 1);  // rows hold even cells
  const uint32_t sh = (uint32_t)(cell & 1u) * 16u;
  uint32_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t ov = 0u;
  bool changed = false;
  for (uint32_t tries = 0;; ++tries) {
    ov = (old >> sh) & 0xFFFFu;
    if (ov >= stamp) break;
    const uint32_t nw = (old & ~(0xFFFFu << sh)) | (stamp << sh);
    if (tries == 8u) {  // not reached: the word changes at most twice per launch
      slea[cell] = (uint16_t)stamp;
      break;
    }
    const uint32_t got = atomicCAS(w, old, nw);
    if (got == old) {
      changed = true;
      break;
    }
    old = got;
  }
  const uint64_t m = __ballot(changed);
  if (m && lane_id() == (uint32_t)__builtin_ctzll(m)) atomicAdd(&agg->inc[row], (uint32_t)__popcll(m));
  if (changed && ov != 0u) {
    const uint32_t age = stamp - ov;
    if (age < kHistNear) atomicAdd(&agg->dec[row][age], 1u);
    else atomicSub(&hist[(uint64_t)row * kHistBins + ov], 1u);
  }
}

// kBits: the discrete variant (one bit per recorder, set by atomic or); else u16 stamps.
template <bool kTrack, bool kBits>
__device__ __forceinline__ void ingest_pair(const Dev& d, uint16_t* __restrict__ sre,
                                            uint16_t* __restrict__ slea, uint32_t* hist,
                                            HistAgg* agg, uint32_t src, uint32_t dst,
                                            uint16_t stamp) {
  pair_cells(d, src, dst, [&](uint64_t cell, bool in_sre, uint32_t row) {
    uint16_t* const a = in_sre ? sre : slea;
    if (kBits)
      atomicOr(&reinterpret_cast<uint32_t*>(a)[cell >> 5], 1u << (cell & 31u));
    else if (kTrack && !in_sre)
      tracked_sle_store(slea, hist, agg, cell, row, stamp);
    else
      a[cell] = stamp;
  });
}

// XCD-aware ingest.  A host's recorders are written from one XCD only, so the repeated
// writes of a heavy host merge in that XCD's L2 instead of being spread over eight L2s that
// each write the same lines back.  Consecutive workgroups go to consecutive XCDs, so the grid
// is cut into groups of n_cls consecutive blocks; every block of a group reads the same
// packets and keeps those whose host class (top bits of a multiplicative hash of aip) is its
// position in the group.  The stores are the same plain stamp stores in any order.
constexpr uint32_t kXcds = 8;
static_assert(sizeof(ClassOffsets) == (kXcds + 1) * 8, "one region per host class");

__device__ __forceinline__ uint32_t host_class(uint32_t aip) { return (aip * 0x9E3779B1u) >> 29; }

template <bool kTrack, bool kBits>
__global__ void __launch_bounds__(256) k_ingest(Dev d, const u32x2* __restrict__ pkts,
                                                uint64_t n, uint16_t stamp, uint32_t n_cls) {
  __shared__ HistAgg agg;
  if (kTrack) {
    hist_agg_clear(&agg);
    __syncthreads();
  }
  const uint32_t cls = blockIdx.x % n_cls, cls_mask = n_cls - 1u;
  const uint64_t stride = (uint64_t)(gridDim.x / n_cls) * blockDim.x;
  for (uint64_t i = (uint64_t)(blockIdx.x / n_cls) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const u32x2 pk = pkts[i];
    const uint32_t aip = d.anet_side ? pk.x : pk.y;
    if ((host_class(aip) & cls_mask) == cls)
      ingest_pair<kTrack, kBits>(d, d.sre, d.slea, d.hist, &agg, pk.x, pk.y, stamp);
  }
  if (kTrack) {
    __syncthreads();
    hist_agg_flush(&agg, d.hist, d.rp, stamp);
  }
}

// The same ingest for the stamp sketch without histograms, with the pairs of the block's
// class compacted per wave: a wave reads 64 pairs per step and appends those of its class
// to a queue in LDS (ballot and mbcnt), and hashes and stores only when the queue holds 64
// of them.  With n_cls classes a pair is the block's one time in n_cls, so without the queue
// most lanes of every hashing and store instruction would sit idle.
__global__ void __launch_bounds__(256) k_ingest_compact(Dev d, const u32x2* __restrict__ pkts,
                                                        uint64_t n, uint16_t stamp,
                                                        uint32_t n_cls) {
  __shared__ u32x2 queue[256 / kWave][2 * kWave];
  const uint32_t lane = lane_id();
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  u32x2* const q = queue[wv];
  const uint32_t cls = blockIdx.x % n_cls, cls_mask = n_cls - 1u;
  const uint64_t stride = (uint64_t)(gridDim.x / n_cls) * blockDim.x;
  uint32_t len = 0;  // pairs in this wave's queue (wave-uniform)
  for (uint64_t b0 = (uint64_t)(blockIdx.x / n_cls) * blockDim.x + wv * kWave; b0 < n;
       b0 += stride) {
    const uint64_t i = b0 + lane;
    u32x2 pk = {0u, 0u};
    if (i < n) pk = pkts[i];
    const uint32_t aip = d.anet_side ? pk.x : pk.y;
    const bool mine = i < n && (host_class(aip) & cls_mask) == cls;
    const uint64_t m = __ballot(mine);
    if (mine)
      q[len + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = pk;
    len += (uint32_t)__popcll(m);
    if (len >= kWave) {  // a full wave of the class's pairs
      const u32x2 p = q[lane];
      ingest_pair<false, false>(d, d.sre, d.slea, nullptr, nullptr, p.x, p.y, stamp);
      len -= kWave;  // the rest (at most 63) moves to the front
      const u32x2 t = q[kWave + lane];
      if (lane < len) q[lane] = t;
    }
  }
  if (lane < len) {
    const u32x2 p = q[lane];
    ingest_pair<false, false>(d, d.sre, d.slea, nullptr, nullptr, p.x, p.y, stamp);
  }
}

// Host classes: 1, 2, 4 or 8 (blocks b and b + n_cls share a class; with 8 a class is one
// XCD, with fewer a class spans 8 / n_cls XCDs), fewer when the grid is smaller than that.
uint32_t ingest_classes(int blocks, uint32_t host_classes) {
  uint32_t c = host_classes >= 1u && host_classes <= kXcds ? host_classes : kXcds;
  while (c > 1u && blocks < (int)c) c >>= 1;
  return c;
}

hipError_t launch_ingest(const Dev& d, const sps_pkt* pkts, uint64_t n, uint16_t stamp,
                         int blocks, int threads, uint32_t host_classes, bool track,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t need = (n + threads - 1) / threads;
  const uint32_t n_cls = ingest_classes(blocks, host_classes);
  uint64_t b = (uint64_t)blocks / n_cls * n_cls;
  if (b > need * n_cls) b = need * n_cls;
  if (b < n_cls) b = n_cls;
  ProfScope ps(SPS_STAGE_INGEST, st, ProfScope::kKernel);
  const u32x2* p2 = reinterpret_cast<const u32x2*>(pkts);
  if (d.mode == SPS_MODE_DISCRETE)
    launch_k(ps, (k_ingest<false, true>), dim3((uint32_t)b), dim3(threads), 0, st, d, p2,
             n, stamp, n_cls);
  else if (track)
    launch_k(ps, (k_ingest<true, false>), dim3((uint32_t)b), dim3(threads), 0, st, d, p2,
             n, stamp, n_cls);
  else if (n_cls > 1u && threads == 256)
    launch_k(ps, k_ingest_compact, dim3((uint32_t)b), dim3(threads), 0, st, d, p2, n, stamp,
             n_cls);
  else
    launch_k(ps, (k_ingest<false, false>), dim3((uint32_t)b), dim3(threads), 0, st, d, p2, n,
             stamp, n_cls);
  return hipGetLastError();
}

// Batched ingest: the packets of m routers (same shape and hashes, separate arrays) are cut
// into tiles; work items are tiles, so one launch covers uneven batches.  Block group g takes
// tiles g, g + groups, ...; the router of a tile is found by binary search of the tile
// prefix sums held in the kernel arguments.
template <bool kTrack, bool kBits>
__global__ void __launch_bounds__(256) k_ingest_batched(Dev d, BatchTable t, uint32_t m,
                                                        uint32_t tile, uint16_t stamp,
                                                        uint32_t n_cls) {
  __shared__ HistAgg agg;
  if (kTrack) {
    hist_agg_clear(&agg);
    __syncthreads();
  }
  // tiles go to groups of n_cls consecutive blocks, one host class per block (see k_ingest)
  const uint32_t cls = blockIdx.x % n_cls, cls_mask = n_cls - 1u;
  __shared__ u32x2 queue[256 / kWave][2 * kWave];
  const uint32_t lane = lane_id();
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint64_t total = t.tile_start[m];
  for (uint64_t w = blockIdx.x / n_cls; w < total; w += gridDim.x / n_cls) {
    uint32_t lo = 0, hi = m;  // find j with tile_start[j] <= w < tile_start[j+1]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (t.tile_start[mid] <= w) lo = mid; else hi = mid;
    }
    const BatchItem it = t.item[lo];
    const uint64_t first = (w - t.tile_start[lo]) * tile;
    uint64_t last = first + tile;
    if (last > it.n) last = it.n;
    const u32x2* pk2 = reinterpret_cast<const u32x2*>(it.pkts);
    const bool track = kTrack && it.hist != nullptr;  // uniform
    if (!kTrack && !kBits && n_cls > 1u) {
      // the class's pairs of this tile compacted per wave, as in k_ingest_compact
      u32x2* const q = queue[wv];
      uint32_t len = 0;
      for (uint64_t b0 = first + wv * kWave; b0 < last; b0 += blockDim.x) {
        const uint64_t i = b0 + lane;
        u32x2 pk = {0u, 0u};
        if (i < last) pk = pk2[i];
        const uint32_t aip = d.anet_side ? pk.x : pk.y;
        const bool mine = i < last && (host_class(aip) & cls_mask) == cls;
        const uint64_t m = __ballot(mine);
        if (mine)
          q[len + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = pk;
        len += (uint32_t)__popcll(m);
        if (len >= kWave) {
          const u32x2 p = q[lane];
          ingest_pair<false, false>(d, it.sre, it.slea, nullptr, nullptr, p.x, p.y, stamp);
          len -= kWave;
          const u32x2 t = q[kWave + lane];
          if (lane < len) q[lane] = t;
        }
      }
      if (lane < len) {
        const u32x2 p = q[lane];
        ingest_pair<false, false>(d, it.sre, it.slea, nullptr, nullptr, p.x, p.y, stamp);
      }
      continue;
    }
    for (uint64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
      const u32x2 pk = pk2[i];
      const uint32_t aip = d.anet_side ? pk.x : pk.y;
      if ((host_class(aip) & cls_mask) == cls) {
        if (track)
          ingest_pair<kTrack, kBits>(d, it.sre, it.slea, it.hist, &agg, pk.x, pk.y, stamp);
        else
          ingest_pair<false, kBits>(d, it.sre, it.slea, nullptr, nullptr, pk.x, pk.y, stamp);
      }
    }
    if (track) {  // this tile's counts go to its router's histograms
      __syncthreads();
      hist_agg_flush(&agg, it.hist, d.rp, stamp);
      __syncthreads();
    }
  }
}

hipError_t launch_ingest_batched(const Dev& shape, const BatchTable& t, uint32_t m,
                                 uint32_t tile, uint16_t stamp, int blocks, int threads,
                                 uint32_t host_classes, hipStream_t st) {
  const uint64_t total = t.tile_start[m];
  if (total == 0) return hipSuccess;
  bool track = false;
  for (uint32_t j = 0; j < m; ++j) track = track || t.item[j].hist != nullptr;
  const uint32_t n_cls = ingest_classes(blocks, host_classes);
  uint64_t b = (uint64_t)blocks / n_cls * n_cls;
  if (b > total * n_cls) b = total * n_cls;
  if (b < n_cls) b = n_cls;
  ProfScope ps(SPS_STAGE_INGEST_BATCHED, st, ProfScope::kKernel);
  if (shape.mode == SPS_MODE_DISCRETE)
    launch_k(ps, (k_ingest_batched<false, true>), dim3((uint32_t)b), dim3(threads), 0, st,
             shape, t, m, tile, stamp, n_cls);
  else if (track)
    launch_k(ps, (k_ingest_batched<true, false>), dim3((uint32_t)b), dim3(threads), 0, st,
             shape, t, m, tile, stamp, n_cls);
  else
    launch_k(ps, (k_ingest_batched<false, false>), dim3((uint32_t)b), dim3(threads), 0, st,
             shape, t, m, tile, stamp, n_cls);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Fill with zeros (reset); a kernel rather than a memset so it can sit inside a graph.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fill_zero(u32x4* __restrict__ p, uint64_t nvec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
    p[i] = z;
}

hipError_t launch_fill_zero(void* p, uint64_t bytes, hipStream_t st) {
  const uint64_t nvec = bytes / 16;
  if (nvec == 0) return hipSuccess;
  uint64_t blocks = (nvec + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  ProfScope ps(SPS_STAGE_FILL, st, ProfScope::kKernel);
  launch_k(ps, k_fill_zero, dim3((uint32_t)blocks), dim3(256), 0, st,
           reinterpret_cast<u32x4*>(p), nvec);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Merge (Alg. 2, Alg. 7): dst <- cell-wise max(dst, src_0, ...), 8 stamps per 16-byte lane
// access; the u16 maxima compile to packed v_pk_max_u16.
// ---------------------------------------------------------------------------------------
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

struct MergeSrcs {
  const u16x8* p[kMaxMerge];
};

__global__ void __launch_bounds__(256) k_merge_max(u16x8* __restrict__ dst, MergeSrcs s,
                                                   uint32_t nsrc, uint64_t nvec, int bits) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) {
    u16x8 v = dst[i];
    if (bits) {  // discrete mode: the union of recorder bits
      for (uint32_t j = 0; j < nsrc; ++j) v = v | s.p[j][i];
    } else {
      for (uint32_t j = 0; j < nsrc; ++j) v = __builtin_elementwise_max(v, s.p[j][i]);
    }
    dst[i] = v;
  }
}

hipError_t launch_merge(uint16_t* dst, const uint16_t* const* srcs, uint32_t nsrc,
                        uint64_t bytes, bool bits, hipStream_t st) {
  const uint64_t nvec = bytes / 16;
  uint64_t blocks = (nvec + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  for (uint32_t b = 0; b < nsrc; b += kMaxMerge) {
    MergeSrcs s{};
    const uint32_t k = nsrc - b < (uint32_t)kMaxMerge ? nsrc - b : (uint32_t)kMaxMerge;
    for (uint32_t j = 0; j < k; ++j) s.p[j] = reinterpret_cast<const u16x8*>(srcs[b + j]);
    ProfScope ps(SPS_STAGE_MERGE, st, ProfScope::kKernel);
    launch_k(ps, k_merge_max, dim3((uint32_t)blocks), dim3(256), 0, st,
             reinterpret_cast<u16x8*>(dst), s, k, nvec, bits ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// Rebase of the time base: every stamp v becomes max(v - offset, 0), 8 stamps per 16-byte
// lane access with packed saturating subtracts (padding cells are 0 and stay 0).
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rebase(u16x8* __restrict__ p, uint64_t nvec,
                                                uint32_t offset) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const u16x8 off = (unsigned short)offset;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
    p[i] = __builtin_elementwise_sub_sat(p[i], off);
}

hipError_t launch_rebase(uint16_t* p, uint64_t bytes, uint32_t offset, hipStream_t st) {
  const uint64_t nvec = bytes / 16;
  if (nvec == 0 || offset == 0) return hipSuccess;
  uint64_t blocks = (nvec + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  ProfScope ps(SPS_STAGE_REBASE, st, ProfScope::kKernel);
  launch_k(ps, k_rebase, dim3((uint32_t)blocks), dim3(256), 0, st,
           reinterpret_cast<u16x8*>(p), nvec, offset);
  return hipGetLastError();
}

// Rebase of the stamp histograms: bin v takes bin v + offset (stamps at or below `offset`
// became 0 and drop out).  One block per row; each round reads its bins before any thread
// writes, and later rounds only read bins above every bin written so far.
__global__ void __launch_bounds__(256) k_hist_rebase(uint32_t* __restrict__ hist,
                                                     uint32_t offset) {
  uint32_t* const h = hist + (uint64_t)blockIdx.x * kHistBins;
  for (uint32_t base = 1; base < kHistBins; base += blockDim.x) {
    const uint32_t v = base + threadIdx.x;
    const uint32_t src = v + offset;
    const uint32_t val = v < kHistBins && src < kHistBins ? h[src] : 0u;
    __syncthreads();
    if (v < kHistBins) h[v] = val;
    __syncthreads();
  }
}

hipError_t launch_hist_rebase(uint32_t* hist, uint32_t rows, uint32_t offset, hipStream_t st) {
  if (offset == 0 || rows == 0) return hipSuccess;
  ProfScope ps(SPS_STAGE_REBASE, st, ProfScope::kKernel);
  launch_k(ps, k_hist_rebase, dim3(rows), dim3(256), 0, st, hist, offset);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Scan.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scan_reset(Ctrl* c, uint32_t* hot_t, uint32_t words) {
  if (blockIdx.x == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(c);
    for (uint32_t i = threadIdx.x; i < kCtrlWorkingWords; i += blockDim.x) w[i] = 0;
  }
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
    hot_t[i] = 0;
}

hipError_t launch_scan_reset(const Dev& d, bool with_table, hipStream_t st) {
  const uint32_t words = with_table ? (uint32_t)(((uint64_t)d.r << d.q) >> 5) : 0u;
  uint32_t blocks = (words + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  ProfScope ps(SPS_STAGE_SCAN_RESET, st, ProfScope::kKernel);
  launch_k(ps, k_scan_reset, dim3(blocks), dim3(256), 0, st, d.ctrl, d.hot_t, words);
  return hipGetLastError();
}

// number of the 8 u16 stamps in v that are >= lo
__device__ __forceinline__ uint32_t live8(u32x4 v, uint32_t lo) {
  uint32_t n = 0;
  n += (v.x & 0xFFFFu) >= lo;
  n += (v.x >> 16) >= lo;
  n += (v.y & 0xFFFFu) >= lo;
  n += (v.y >> 16) >= lo;
  n += (v.z & 0xFFFFu) >= lo;
  n += (v.z >> 16) >= lo;
  n += (v.w & 0xFFFFu) >= lo;
  n += (v.w >> 16) >= lo;
  return n;
}

// Live stamps of 8 cells, two per 32-bit word with packed 16-bit integer operations: the
// saturating difference stamp - (lo - 1) is nonzero exactly when stamp >= lo, and its
// minimum with 1 is the 0/1 count of that half.  The result holds the count of the low
// halves in bits 0-15 and of the high halves in bits 16-31 (each at most 4).
__device__ __forceinline__ uint32_t live_pairs(uint32_t w, uint32_t lom1, uint32_t ones) {
  uint32_t d, m;
  asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(d) : "v"(w), "v"(lom1));
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(m) : "v"(d), "v"(ones));
  return m;
}

__device__ __forceinline__ uint32_t live8_pairs(u32x4 v, uint32_t lom1, uint32_t ones) {
  return live_pairs(v.x, lom1, ones) + live_pairs(v.y, lom1, ones) +
         live_pairs(v.z, lom1, ones) + live_pairs(v.w, lom1, ones);
}

// k-weight of one SRE (Sec. 3.3): its live cells, or its set bits in the discrete variant.
__device__ __forceinline__ uint32_t sre_weight(const Dev& d, uint32_t lo, uint64_t sre_idx) {
  uint32_t w = 0;
  if (d.mode == SPS_MODE_DISCRETE) {  // eta bits per SRE: eta / 8 bytes
    const uint8_t* by = reinterpret_cast<const uint8_t*>(d.sre) + (sre_idx * d.eta >> 3);
    for (uint32_t b = 0; b < d.eta / 8; ++b) w += __popc((uint32_t)by[b]);
  } else {
    const u32x4* cell = reinterpret_cast<const u32x4*>(d.sre + (sre_idx << __builtin_ctz(d.eta)));
    for (uint32_t v = 0; v < d.eta / 8; ++v) w += live8(cell[v], lo);
  }
  return w;
}

// One SRE per lane (64 consecutive SREs per wave): k-weight >= hot cut marks it hot.
__device__ __forceinline__ void sre_group(const Dev& d, uint32_t lo, uint64_t sre_idx) {
  const bool hot = sre_weight(d, lo, sre_idx) >= d.hot_cut;
  const uint64_t mask = __ballot(hot);
  const uint32_t row = (uint32_t)(sre_idx >> d.q);
  const uint32_t col = (uint32_t)(sre_idx & ((1u << d.q) - 1u));
  if (lane_id() == 0) {
    uint32_t* hw = d.hot + (sre_idx >> 5);
    hw[0] = (uint32_t)mask;
    hw[1] = (uint32_t)(mask >> 32);
    if (mask) atomicAdd(&d.ctrl->hot_rows[row], (uint32_t)__popcll(mask));
  }
  if (hot) {  // the join's layout: all 2^delta extensions of a node in one entry
    const uint32_t low = col & ((1u << (d.q - d.delta)) - 1u);
    const uint32_t top = col >> (d.q - d.delta);
    const uint32_t pos = (row << d.q) + (low << d.delta) + top;
    atomicOr(&d.hot_t[pos >> 5], 1u << (pos & 31u));
  }
  if (row < 2 && mask != 0) {
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(&d.ctrl->hse_count[row], (uint32_t)__popcll(mask));
    base = __shfl(base, 0, kWave);
    if (hot) {
      const uint32_t below = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
      d.hse[((uint64_t)row << d.q) + base + below] = col;
    }
  }
}

// Stage 1: the row live counts (Def. 4 numerators) and the hot SREs (Sec. 3.3).
//
// Row live counts come from one of three places: the stamp histograms (a few hundred bins per
// row), a sweep of the SLE array run inside the candidate search's launch, or a sweep run as a
// kernel of its own.  A sweep streams the rows as one flat range (grid-stride with eight
// 16-byte non-temporal loads in flight per lane and the next eight issued before the current
// ones are counted), so all lanes carry equal work.
//
// Hot SREs: a wave takes 64 SREs, one per lane; k-weight >= hot cut marks it hot.  The 64
// verdicts become two words of the hot bitmap, rows 0 and 1 append their hot columns to the
// HSE lists, and every hot SRE sets its bit of the join's table.
constexpr uint32_t kStatsSre = 1u;   // the SREs (hot bitmap, lists, join table, row counts)
constexpr uint32_t kStatsHist = 2u;  // row live counts from the stamp histograms
constexpr uint32_t kStatsRows = 4u;  // row live counts (histograms, else a sweep)
constexpr uint32_t kStatsPartials = 8u;  // the sweep leaves per-wave counts in d.rows_part

// Row b's live cells from its histogram: the bins lo..hi (one block; added to row_live).
__device__ __forceinline__ void hist_row_live(const Dev& d, uint32_t b, uint32_t lo,
                                              uint32_t hi) {
  __shared__ uint32_t red[1024 / kWave];
  const uint32_t* h = d.hist + (uint64_t)b * kHistBins;
  uint32_t c = 0;
  for (uint32_t v = lo + threadIdx.x; v <= hi; v += blockDim.x) c += h[v];
  c = wave_sum(c);
  if (lane_id() == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) t += red[w];
    atomicAdd(&d.ctrl->row_live[b], t);
  }
}

// 16-byte loads a sweep lane keeps in one batch (two batches in flight).
constexpr int kSweepBatch = 8;

// One lane's share of a sweep of `step` lanes (this one is lane `first`): its live cells of
// every row, added to cnt[row].
__device__ __forceinline__ void sweep_lane(const Dev& d, uint32_t lo, uint64_t first,
                                           uint64_t step, uint32_t (&cnt)[kMaxRP]) {
  auto add_to = [&cnt](uint32_t row, uint32_t c) {
#pragma unroll
    for (int j = 0; j < kMaxRP; ++j)
      if ((uint32_t)j == row) cnt[j] += c;
  };
  if (d.mode == SPS_MODE_DISCRETE) {  // one bit per cell: a row is row_stride / 128 vectors
    for (uint32_t row = 0; row < d.rp; ++row) {
      const u32x4* rowb = reinterpret_cast<const u32x4*>(
          reinterpret_cast<const uint32_t*>(d.slea) + (uint64_t)row * (d.row_stride >> 5));
      const uint64_t nvb = d.row_stride >> 7;
      uint32_t c = 0;
      for (uint64_t v = first; v < nvb; v += step) {
        const u32x4 a = __builtin_nontemporal_load(&rowb[v]);
        c += __popc(a.x) + __popc(a.y) + __popc(a.z) + __popc(a.w);
      }
      add_to(row, c);
    }
    return;
  }
  // the rows are one flat range: the sweep runs across row ends without draining, and a
  // lane's counts move to the next row when its index passes a row boundary
  const u32x4* vec = reinterpret_cast<const u32x4*>(d.slea);
  const uint64_t nvec = d.row_stride / 8, total = (uint64_t)d.rp * nvec;
  uint32_t row = (uint32_t)(first / nvec);
  uint64_t next_b = (uint64_t)(row + 1u) * nvec;  // first vector of the next row
  uint32_t acc = 0;
  auto account = [&](uint64_t idx, uint32_t c) {
    while (idx >= next_b) {
      add_to(row, acc);
      acc = 0;
      ++row;
      next_b += nvec;
    }
    acc += c;
  };
  const uint32_t lom1 = (lo - 1u) * 0x10001u, ones = 0x10001u;
  // two batches of kSweepBatch loads, the next issued before the current one is counted; load
  // indices are clamped into the array so the batches are unconditional
  constexpr int N = kSweepBatch;
  auto load_batch = [&](u32x4* a, uint64_t v0) {
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const uint64_t j = v0 + u * step;
      a[u] = __builtin_nontemporal_load(&vec[j < total ? j : total - 1]);
    }
  };
  auto count_batch = [&](const u32x4* a, uint64_t v0) {
    if (v0 + (N - 1) * step < next_b) {  // all of the batch in the current row
      uint32_t pr = 0;  // packed counts, at most 4 N per half
#pragma unroll
      for (int u = 0; u < N; ++u) pr += live8_pairs(a[u], lom1, ones);
      acc += (pr & 0xFFFFu) + (pr >> 16);
    } else {
#pragma unroll
      for (int u = 0; u < N; ++u) account(v0 + u * step, live8(a[u], lo));
    }
  };
  uint64_t v = first;
  u32x4 A[N], B[N];
  load_batch(A, v);
  for (;;) {
    if (v + (N - 1) * step >= total) break;
    load_batch(B, v + N * step);
    count_batch(A, v);
    v += N * step;
    if (v + (N - 1) * step >= total) break;
    load_batch(A, v + N * step);
    count_batch(B, v);
    v += N * step;
  }
  for (; v < total; v += step) account(v, live8(__builtin_nontemporal_load(&vec[v]), lo));
  add_to(row, acc);
}

// A wave's sweep counts as one plain store per row into the partials (wave gw of the sweep),
// summed by the estimate: no LDS and no same-address atomics at the end of the sweep.
__device__ __forceinline__ void sweep_partials(const Dev& d, const uint32_t (&cnt)[kMaxRP],
                                               uint32_t gw) {
  for (uint32_t j = 0; j < d.rp; ++j) {
    uint32_t c = 0;
#pragma unroll
    for (int jj = 0; jj < kMaxRP; ++jj)
      if ((uint32_t)jj == j) c = cnt[jj];
    c = wave_sum(c);
    if (lane_id() == 0) d.rows_part[(uint64_t)j * kRowsPartWaves + gw] = c;
  }
}

__device__ __forceinline__ void scan_stats_body(const Dev& d, uint32_t lo, uint32_t hi,
                                                uint32_t flags) {
  __shared__ uint32_t red[kMaxRP][256 / kWave];
  const uint32_t b = blockIdx.x;
  const bool with_sre = (flags & kStatsSre) != 0u;
  if ((flags & kStatsRows) && (flags & kStatsHist)) {
    if (b < d.rp) hist_row_live(d, b, lo, hi);
  } else if (flags & kStatsRows) {
    uint32_t cnt[kMaxRP];
#pragma unroll
    for (int j = 0; j < kMaxRP; ++j) cnt[j] = 0;
    sweep_lane(d, lo, (uint64_t)b * blockDim.x + threadIdx.x, (uint64_t)gridDim.x * blockDim.x,
               cnt);
    if (flags & kStatsPartials) {
      sweep_partials(d, cnt, b * (blockDim.x / kWave) + threadIdx.x / kWave);
    } else {
      for (uint32_t j = 0; j < d.rp; ++j) {
        uint32_t c = 0;
#pragma unroll
        for (int jj = 0; jj < kMaxRP; ++jj)
          if ((uint32_t)jj == j) c = cnt[jj];
        c = wave_sum(c);
        if (lane_id() == 0) red[j][threadIdx.x / kWave] = c;
      }
      __syncthreads();
      if (threadIdx.x < d.rp) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < blockDim.x / kWave; ++w) t += red[threadIdx.x][w];
        atomicAdd(&d.ctrl->row_live[threadIdx.x], t);
      }
    }
  }
  if (!with_sre) return;
  // then the SREs, 64 per wave at a time (r 2^q is a multiple of 64: q >= 6)
  const uint64_t n_groups = ((uint64_t)d.r << d.q) / kWave;
  const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint64_t n_waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  for (uint64_t g = (uint64_t)b * (blockDim.x / kWave) + wib; g < n_groups; g += n_waves)
    sre_group(d, lo, g * kWave + lane_id());
}

// The row live counts and/or the hot SREs one SRE per lane, the join table by atomic ORs.
__global__ void __launch_bounds__(256) k_scan_stats(Dev d, uint32_t lo, uint32_t hi,
                                                    uint32_t flags) {
  scan_stats_body(d, lo, hi, flags);
}

// The hot SREs by tiles (for q - delta >= 6).  A tile is one row's 64 consecutive low parts
// (the column's q - delta low bits) with all 2^delta top parts: 2^(delta+6) SREs whose bits
// of the join's table (position (low << delta) + top within the row) fill 2^(delta+1) whole
// words.  A block owns its tiles' words of the hot bitmap and of the table, so both take
// plain stores, and a tile's hot count and (rows 0 and 1) its place in the HSE list take one
// atomic each.  With `hist` the first r' blocks first take the row live counts from the
// histograms.
__global__ void __launch_bounds__(256) k_scan_sre(Dev d, uint32_t lo, uint32_t hi,
                                                  uint32_t hist) {
  __shared__ unsigned long long gm[1u << 5];  // hot masks of the tile's groups (delta <= 5)
  __shared__ uint32_t pre[(1u << 5) + 1u];    // hot SREs of the groups before each one
  __shared__ uint32_t base_sh;
  if (hist && blockIdx.x < d.rp) {
    hist_row_live(d, blockIdx.x, lo, hi);
    __syncthreads();
  }
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t lane = lane_id(), nw = blockDim.x / kWave;
  const uint32_t lowbits = d.q - d.delta, groups = 1u << d.delta;
  const uint32_t tiles_row = 1u << (lowbits - 6u);
  const uint32_t n_tiles = d.r << (lowbits - 6u);
  for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const uint32_t row = tile >> (lowbits - 6u);
    const uint32_t l0 = (tile & (tiles_row - 1u)) << 6;
    const uint64_t row0 = (uint64_t)row << d.q;
    for (uint32_t t = wave; t < groups; t += nw) {
      const uint64_t first = row0 + l0 + (t << lowbits);  // a multiple of 64
      const bool hot = sre_weight(d, lo, first + lane) >= d.hot_cut;
      const uint64_t mask = __ballot(hot);
      if (lane < 2u) d.hot[(first >> 5) + lane] = (uint32_t)(mask >> (32u * lane));
      if (lane == 0u) gm[t] = mask;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t s = 0;
      for (uint32_t t = 0; t < groups; ++t) {
        pre[t] = s;
        s += (uint32_t)__popcll(gm[t]);
      }
      if (s) atomicAdd(&d.ctrl->hot_rows[row], s);
      base_sh = (row < 2u && s) ? atomicAdd(&d.ctrl->hse_count[row], s) : 0u;
    }
    // bit b of the tile's table word j is position p = 32 j + b = (low offset << delta) + top
    if (threadIdx.x < (2u << d.delta)) {
      uint32_t v = 0;
      for (uint32_t b = 0; b < 32u; ++b) {
        const uint32_t p = threadIdx.x * 32u + b;
        v |= (uint32_t)((gm[p & (groups - 1u)] >> (p >> d.delta)) & 1ull) << b;
      }
      d.hot_t[((row0 + ((uint64_t)l0 << d.delta)) >> 5) + threadIdx.x] = v;
    }
    __syncthreads();
    if (row < 2u) {
      for (uint32_t t = wave; t < groups; t += nw) {
        const uint64_t m = gm[t];
        if ((m >> lane) & 1ull) {
          const uint32_t below = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          d.hse[row0 + base_sh + pre[t] + below] = l0 + lane + (t << lowbits);
        }
      }
    }
    __syncthreads();  // gm, pre and base_sh are rewritten by the next tile
  }
}

// The row live counts alone, as per-wave partial counts, in a launch of its own.
template <bool kBits>  // a separate symbol for the discrete variant's sweep of bits
__global__ void __launch_bounds__(256) k_scan_rows(Dev d, uint32_t lo, uint32_t hi) {
  scan_stats_body(d, lo, hi, kStatsRows | kStatsPartials);
}

// Hot extensions of a node (Alg. 4-5 check, in bulk).  Row i's SRE for the extension t is
// he0 ^ B(i): its low q-delta bits are `low` (B(i)'s low bits xor he0's, from bits already
// fixed) and its top delta bits are u = t ^ top0 (top0: he0's top bits).  The transposed
// table keeps, for each (row, low), the 2^delta hot bits over u in one entry; the result is
// that entry, indexed by u (the caller maps u back to t = u ^ top0).
__device__ __forceinline__ uint32_t hot_tops(const uint32_t* __restrict__ tb, uint32_t q,
                                             uint32_t dl, uint32_t wmask, uint32_t row,
                                             uint32_t low) {
  const uint32_t pos = (row << q) + (low << dl);
  return (tb[pos >> 5] >> (pos & 31u)) & wmask;
}

// The extensions allowed by bit 32 as a mask over u = t ^ top0.  Row i's new bits start at
// sx = (i-2) delta + q; only the f = min(32 - sx, delta) low ones can be set (f = 0 when
// sx >= 32), so t < 2^f: a block of 2^f consecutive u values starting at top0 with its low
// f bits cleared.
__device__ __forceinline__ uint32_t fit_tops(uint32_t sx, uint32_t dl, uint32_t wmask,
                                             uint32_t top0) {
  const uint32_t f = sx >= 32u ? 0u : (32u - sx < dl ? 32u - sx : dl);
  if (f == dl) return wmask;
  const uint32_t blk = 1u << f;  // <= 16 here
  return ((1u << blk) - 1u) << (top0 & ~(blk - 1u));
}

// Stage 2, candidate recovery (Alg. 4-5 through Eq. 6-7).  A pair (he0, he1) of hot SREs of
// rows 0 and 1 fixes B(1) = he0 ^ he1, the address bits [0, q).  Row i >= 2 adds the delta
// bits [(i-2)delta + q, (i-1)delta + q); the overlap of B(i) with B(i-1) holds by
// construction, so an extension survives when SRE he0 ^ B(i) of row i is hot and no bit at
// or above 32 is set.  Each node's surviving extensions come from one load of the
// transposed hot table.  A full tuple is kept when RHFG[0] of the address is he0.
//
// Work: every wave runs its own search with a stack of nodes in LDS.  A node is
// (x, he0, i): the address bits fixed so far, the row-0 SRE and the next row to extend.
// Each iteration the wave takes up to 64 nodes from the top of its stack, tops the batch
// up with fresh (he0, he1) pairs when the stack holds fewer than 64, expands all of them at
// once (one node per lane) and pushes the children; nodes at the last row check their
// extensions in place.  Children of lanes nearer the top are pushed above the others, so
// the stack stays ordered by row from bottom to top and stays small: a batch that reaches
// into the nodes of row i takes every node above row i with it, so no row holds more than
// 64 times the extensions of one node.  That bound (64 * sum_i |extensions of row i|, 2048
// entries at q = 14, delta = 2) would cost so much LDS that few waves fit on a compute unit,
// so the stack is smaller (join_stack_entries); when a batch's children do not fit, each
// lane instead searches its own node's subtree depth first in registers (join_lane_dfs)
// and nothing is pushed.  Either way every node is expanded exactly once.
//
// Pairs are numbered a * n1 + b and cut into groups of 64; block b owns groups b, b + B,
// b + 2B, ... and its waves take them one at a time from a counter in LDS.  A wave keeps the
// (a, b) of the first pair of its current and of its next group; a lane's pair follows from
// them with at most one wrap to the next row (n1 >= 128) or from a corrected
// double-precision quotient.  The hot table, the stacks and (when they fit) the two hot
// lists live in LDS, so the loop touches no global memory except to record a candidate.
constexpr uint32_t kLdsBytes = 160u << 10;  // LDS of one gfx950 compute unit
constexpr uint32_t kJoinWaves = 16;        // waves per block at most

__host__ __device__ __forceinline__ uint32_t popc32(uint32_t v) {
#ifdef __HIP_DEVICE_COMPILE__
  return __popc(v);
#else
  return (uint32_t)__builtin_popcount(v);
#endif
}

// Recovered addresses go to a per-block buffer in LDS first and reach the global list with
// one counter update per block at the end (same-address atomics from every finding lane
// would otherwise serialise); when the buffer is full they go straight to the global list.
constexpr uint32_t kCandBuf = 1024;  // entries of the block's candidate buffer

struct CandSink {
  uint32_t* cnt;  // LDS: addresses offered to the buffer (may pass kCandBuf)
  uint32_t* buf;  // LDS: kCandBuf entries
};

__device__ __forceinline__ void put_cand(const Dev& d, const CandSink& cs, uint32_t addr) {
  const uint32_t k = atomicAdd(cs.cnt, 1u);
  if (k < kCandBuf) {
    cs.buf[k] = addr;
  } else {
    const uint32_t pos = atomicAdd(&d.ctrl->n_cand, 1u);
    if (pos < d.cand_cap) d.cand[pos] = addr;
  }
}

// Stack entries per wave: room for a full batch of children (64 nodes x 2^delta) on top of
// what the stack usually holds.
uint32_t join_stack_entries(uint32_t dl) {
  const uint32_t need = 64u * (1u << dl) + 64u;
  return need > 768u ? need : 768u;
}

// Hot lists as read by the join: u16 entries in LDS when q <= 16, else u32 (global).
template <typename T>
struct HotLists {
  const T* l0;
  const T* l1;
  __device__ __forceinline__ uint32_t he0(uint32_t a) const { return l0[a]; }
  __device__ __forceinline__ uint32_t he1(uint32_t b) const { return l1[b]; }
};

// a = p / n1, b = p % n1 from a double-precision estimate corrected by one step (the
// estimate is off by less than one: p < 2^48 and rcp = 1/n1 to 53 bits).
template <bool kSmall>
__device__ __forceinline__ void pair_coords(uint64_t p, uint32_t n1, double rcp, uint32_t& a,
                                            uint32_t& b) {
  if (kSmall) {  // p < 2^32, n0 and n1 < 2^24: the quotient and n1 fit 24-bit factors
    const uint32_t p32 = (uint32_t)p;
    const uint32_t q0 = (uint32_t)((double)p32 * rcp);
    const int32_t rem = (int32_t)(p32 - __umul24(q0, n1));
    const bool neg = rem < 0, over = rem >= (int32_t)n1;
    a = neg ? q0 - 1u : (over ? q0 + 1u : q0);
    b = (uint32_t)(neg ? rem + (int32_t)n1 : (over ? rem - (int32_t)n1 : rem));
  } else {
    uint64_t q0 = (uint64_t)((double)p * rcp);
    int64_t rem = (int64_t)(p - q0 * n1);
    if (rem < 0) {
      --q0;
      rem += n1;
    } else if ((uint64_t)rem >= n1) {
      ++q0;
      rem -= n1;
    }
    a = (uint32_t)q0;
    b = (uint32_t)rem;
  }
}

// Subtree search of one lane, with the partial address as its only state: used when a
// wave's stack has no room for a batch's children.  (x, he0, i) is a node whose row-i
// extensions (over u = t ^ top0) are R; every descendant is visited once, depth first:
// backing up from row i to row i-1 clears row i-1's extension bits from x and recomputes
// row i-1's extensions above the one just finished.
__device__ __forceinline__ uint32_t join_lane_dfs(const Dev& d, const CandSink& cs,
                                               const uint32_t* __restrict__ tb, uint32_t wmask, uint32_t lowmask, uint32_t qmask,
                                               uint32_t x, uint32_t he0, uint32_t i, uint32_t R) {
  const uint32_t q = d.q, dl = d.delta, r = d.r;
  const uint32_t top0 = he0 >> (q - dl), dmask = (1u << dl) - 1u;
  const uint32_t i0 = i;
  uint32_t expanded = 0;  // nodes expanded below (x, he0, i)
  for (;;) {
    if (R == 0u) {
      if (i == i0) return expanded;
      --i;  // back up: the extension taken at row i
      const uint32_t sx = (i - 2u) * dl + q;
      const uint32_t t = sx < 32u ? (x >> sx) & dmask : 0u;
      if (sx < 32u) x &= (1u << sx) - 1u;
      const uint32_t u = t ^ top0;
      const uint32_t low = ((x >> ((i - 1u) * dl)) ^ he0) & lowmask;
      const uint32_t above = u >= 31u ? 0u : ~((2u << u) - 1u);
      R = hot_tops(tb, q, dl, wmask, i, low) & fit_tops(sx, dl, wmask, top0) & above;
      continue;
    }
    const uint32_t t = (uint32_t)__builtin_ctz(R) ^ top0;
    R &= R - 1u;
    const uint32_t sx = (i - 2u) * dl + q;
    const uint32_t xi = sx < 32u ? x | (t << sx) : x;
    if (i + 1u == r) {
      if ((fmix32(xi ^ d.seed_rhfg0) & qmask) == he0) put_cand(d, cs, xi);
    } else {
      x = xi;
      ++i;
      ++expanded;
      const uint32_t sxn = (i - 2u) * dl + q;
      const uint32_t low = ((x >> ((i - 1u) * dl)) ^ he0) & lowmask;
      R = hot_tops(tb, q, dl, wmask, i, low) & fit_tops(sxn, dl, wmask, top0);
    }
  }
}

// kFullFit: every row's extensions stay below bit 32 ((r-2) delta + q <= 32), so the
// bit-32 limit never removes an extension and extension bits always shift in range.
template <bool kSmall, bool kFullFit, typename L>
__device__ __forceinline__ uint32_t join_wave(const Dev& d, const CandSink& cs,
                                              const uint32_t* __restrict__ tb,
                                              u32x2* __restrict__ stk, uint32_t cap, L lists,
                                              uint32_t n0, uint32_t n1, uint32_t* next) {
  const uint32_t q = d.q, dl = d.delta, r = d.r;
  const uint64_t pairs = (uint64_t)n0 * n1;
  const uint32_t lane = lane_id();
  const uint32_t qmask = (1u << q) - 1u, lowmask = (1u << (q - dl)) - 1u;
  const uint32_t wmask = dl == 5u ? 0xFFFFFFFFu : ((1u << (1u << dl)) - 1u);
  const double rcp = 1.0 / (double)n1;

  // Block b owns the groups b, b + B, b + 2B, ... of 64 pairs; its waves take them one at a
  // time from a counter in LDS (waves of a block do not progress at equal speed).
  auto take = [&]() -> uint64_t {
    uint32_t k = 0;
    if (lane == 0) k = atomicAdd(next, 1u);
    const uint64_t g = blockIdx.x + (uint64_t)__builtin_amdgcn_readfirstlane(k) * gridDim.x;
    return g * 64ull;  // its first pair
  };
  auto group_n = [pairs](uint64_t first) -> uint32_t {
    return first < pairs ? (pairs - first < 64ull ? (uint32_t)(pairs - first) : 64u) : 0u;
  };
  uint64_t p_cur = take(), p_nxt = take();  // first pairs of the current and the next group
  uint32_t cur_n = group_n(p_cur), nxt_n = group_n(p_nxt);
  // (a, b) of the first pair of the current and of the next group (uniform); with n1 >= 128 a
  // lane's pair is at most 126 further on, one step past the end of row a at most
  const bool near = n1 >= 128u;
  uint32_t ca, cb, na, nb;
  pair_coords<false>(p_cur, n1, rcp, ca, cb);
  pair_coords<false>(p_nxt, n1, rcp, na, nb);
  uint32_t used = 0;  // pairs of the current group already taken (uniform)
  uint32_t size = 0;  // nodes on this wave's stack (uniform)
  uint32_t nodes = 0;  // nodes this wave expanded (uniform; at most a few times 10^5)
  for (;;) {
    const uint32_t popped = size < 64u ? size : 64u;
    const uint32_t need = 64u - popped;
    const uint32_t t1 = cur_n - used < need ? cur_n - used : need;  // from the current group
    const uint32_t t2 = nxt_n < need - t1 ? nxt_n : need - t1;      // then from the next
    if (popped + t1 + t2 == 0u) break;  // stack empty and no pairs left
    nodes += popped + t1 + t2;
    const uint32_t k = lane - popped;   // this lane's rank among the fresh pairs
    // Every lane reads both a stack entry and a pair and keeps the one its role asks for:
    // the reads are issued once per wave either way, and no exec-mask branches are needed.
    const bool pop = lane < popped;
    const bool fresh = !pop && k < t1 + t2;
    const u32x2 nd = stk[pop ? size - 1u - lane : 0u];
    uint32_t a, b;
    if (near) {  // uniform
      a = k < t1 ? ca : na;
      b = k < t1 ? cb + used + k : nb + (k - t1);
      const bool wrap = b >= n1;
      a = wrap ? a + 1u : a;
      b = wrap ? b - n1 : b;
    } else {
      pair_coords<kSmall>(k < t1 ? p_cur + used + k : p_nxt + (k - t1), n1, rcp, a, b);
    }
    const uint32_t phe0 = lists.he0(fresh ? a : 0u), phe1 = lists.he1(fresh ? b : 0u);
    const uint32_t x = pop ? nd.x : (fresh ? phe0 ^ phe1 : 0u);
    const uint32_t he0 = pop ? nd.y & 0xFFFFFFu : (fresh ? phe0 : 0u);
    const uint32_t i = pop ? nd.y >> 24 : 2u;
    const uint32_t top0 = he0 >> (q - dl);
    const uint32_t sx = __umul24(i - 2u, dl) + q;  // first bit of the extension
    const uint32_t low = ((x >> __umul24(i - 1u, dl)) ^ he0) & lowmask;  // (i-1)delta <= 31
    uint32_t R = hot_tops(tb, q, dl, wmask, i, low);
    if (!kFullFit) R &= fit_tops(sx, dl, wmask, top0);
    R = pop || fresh ? R : 0u;
    used += t1;
    if (used == cur_n && nxt_n != 0u) {  // move on to the next group
      p_cur = p_nxt;
      cur_n = nxt_n;
      used = t2;
      ca = na;
      cb = nb;
      p_nxt = take();
      nxt_n = group_n(p_nxt);
      pair_coords<false>(p_nxt, n1, rcp, na, nb);
    }
    const bool last = i + 1u == r;
    if (last) {
      while (R) {
        const uint32_t t = (uint32_t)__builtin_ctz(R) ^ top0;
        R &= R - 1u;
        const uint32_t addr = kFullFit || sx < 32u ? x | (t << sx) : x;
        if ((fmix32(addr ^ d.seed_rhfg0) & qmask) == he0) put_cand(d, cs, addr);
      }
    }
    const uint32_t c = popc32(R);  // children to push (0 at the last row)
    const uint32_t incl = wave_incl_scan(c);
    const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
    const uint32_t below = incl - c;
    const uint32_t base = size - popped;
    if (base + total <= cap) {  // uniform: the children fit on the stack
      uint32_t pos = base + total - below;  // this lane's children end here
      const uint32_t meta = he0 | ((i + 1u) << 24);
      while (R) {
        const uint32_t t = (uint32_t)__builtin_ctz(R) ^ top0;
        R &= R - 1u;
        const u32x2 child = {kFullFit || sx < 32u ? x | (t << sx) : x, meta};
        if (--pos < cap) stk[pos] = child;  // always true; keeps every store inside the stack
      }
      size = base + total;
    } else {  // no room: every lane searches its own node's subtree depth first instead
      const uint32_t e = join_lane_dfs(d, cs, tb, wmask, lowmask, qmask, x, he0, i, R);
      nodes += __builtin_amdgcn_readfirstlane(wave_sum(e));
      size = base;
    }
  }
  return nodes;
}

// The same search with rows 1-3 taken in bulk (delta = 2, dense rows).  For a row-0 SRE he0
// and v, the low q - 2 bits of B(4), the prefixes x = j | v << 6 (j: the low 6 address bits)
// whose windows B(1), B(2), B(3) land on hot SREs he0 ^ B(i) of rows 1-3 form a 64-bit mask
// over j: B(1) = j | (v << 6 mod 2^q) spans 64 consecutive columns of row 1, B(2) 16
// columns of row 2 and B(3) 4 of row 3, all XOR-shifted by he0's low bits.  Indexing the
// mask by j' = j ^ (he0 mod 64), stored with its 2-bit digits reversed (bit p(j') with
// p = (j' mod 4) * 16 + (j' / 4 mod 4) * 4 + j' / 16), makes row 1's part a plain 64-bit
// word of a reordered copy of its bitmap, row 2's part a 16-bit pattern repeated 4 times and
// row 3's a 4-bit pattern repeated 16 times; both patterns only need a XOR permutation of
// bit positions that is the same for the whole wave (he0 is uniform).  Rows 1 and 2 only
// see w = v mod 2^(q-4), so a lane takes one w and its four v = w + k 2^(q-4): one row-1
// and one row-2 chunk serve all four, and reordered copies of rows 3 and 4 hold the four
// row-3 patterns and the four row-4 extension sets in one 16-bit entry each.  The mask's
// prefixes are exactly the search's row-3 tuples; those whose row-4 entry is not empty go
// on the stack as nodes of row 4 for the ordinary search (one store each: expanding their
// extensions here, lane by lane, measured slower).  Every v is visited (2^(q-2) per he0),
// so this pays off only when rows are dense; the caller decides.  The row-2 and row-3
// tuples the masks resolve are counted, so the node count is the same as the ordinary
// search's.
__device__ __forceinline__ uint32_t xor_perm16(uint32_t x, uint32_t c) {  // bit y <- bit y ^ c
  if (c & 1u) x = ((x >> 1) & 0x5555u) | ((x & 0x5555u) << 1);
  if (c & 2u) x = ((x >> 2) & 0x3333u) | ((x & 0x3333u) << 2);
  if (c & 4u) x = ((x >> 4) & 0x0F0Fu) | ((x & 0x0F0Fu) << 4);
  if (c & 8u) x = ((x >> 8) & 0x00FFu) | ((x & 0x00FFu) << 8);
  return x;
}

// digit-reversed bit position of j' in the 64-bit mask (an involution)
__host__ __device__ __forceinline__ uint32_t fold_pos(uint32_t j) {
  return ((j & 3u) << 4) | (j & 12u) | (j >> 4);
}

// Reordered bitmaps of rows 1-4; for rows 3 and 4, L is the low q - 4 bits of the column
// index (row 3: of the column / 4; row 4: of the column's low q - 2 bits) and T the two bits
// above them, so that the four values of T sit in one 16-bit entry.
struct FoldTables {
  const u32x2* f1;     // row 1: 2^(q-6) chunks of 64 columns, bit fold_pos(c mod 64)
  const uint16_t* f2;  // row 2: 2^(q-4) chunks of 16 columns, bit (c mod 4) * 4 + (c / 4 mod 4)
  const uint16_t* f3;  // row 3: entry L, bit 4T + b = column 4 (L + T 2^(q-4)) + b
  const uint16_t* f4;  // row 4: entry L, bit 4T + u = column L + T 2^(q-4) + u 2^(q-2)
  const uint16_t* l0;  // hot columns of row 0
  uint32_t* next;      // LDS: groups of this block handed out so far
};

template <bool kFullFit>
__device__ __forceinline__ uint32_t join_wave_fold(const Dev& d, const CandSink& cs,
                                                   const uint32_t* __restrict__ tb,
                                               FoldTables ft, u32x2* __restrict__ stk,
                                               uint32_t cap, uint32_t n0) {
  const uint32_t q = d.q, r = d.r;
  constexpr uint32_t dl = 2u, wmask = 0xFu;
  const uint32_t lane = lane_id();
  const uint32_t qmask = (1u << q) - 1u, lowmask = (1u << (q - dl)) - 1u;
  const uint32_t gsh = q - 10u;  // 2^(q-10) groups of 64 w values per he0
  // Block b owns groups b, b + B, b + 2B, ... (interleaved, so every block sees the same mix
  // of row-0 SREs); its waves take them one at a time from a counter in LDS, so waves that get
  // fewer issue slots simply take fewer groups and all waves of the block run out of work
  // together.
  const uint32_t g_end = n0 << gsh;
  auto take = [&]() -> uint32_t {
    uint32_t k = 0;
    if (lane == 0) k = atomicAdd(ft.next, 1u);
    return blockIdx.x + __builtin_amdgcn_readfirstlane(k) * gridDim.x;
  };
  uint32_t g = take();
  uint32_t size = 0;       // nodes on this wave's stack (uniform)
  uint32_t nodes = 0;      // stack nodes expanded (uniform)
  uint32_t resolved = 0;   // row-2 and row-3 tuples resolved by the masks (per lane)
  uint32_t he0_next = ft.l0[g < g_end ? g >> gsh : 0u];  // row-0 SRE of the next group
  for (;;) {
    if (size >= 64u || (g >= g_end && size != 0u)) {  // a batch from the top of the stack
      const uint32_t popped = size < 64u ? size : 64u;
      nodes += popped;
      const bool pop = lane < popped;
      const u32x2 nd = stk[pop ? size - 1u - lane : 0u];
      const uint32_t x = pop ? nd.x : 0u;
      const uint32_t he0 = pop ? nd.y & 0xFFFFFFu : 0u;
      const uint32_t i = pop ? nd.y >> 24 : 2u;
      const uint32_t top0 = he0 >> (q - dl);
      const uint32_t sx = (i - 2u) * dl + q;
      const uint32_t low = ((x >> ((i - 1u) * dl)) ^ he0) & lowmask;
      uint32_t R = hot_tops(tb, q, dl, wmask, i, low);
      if (!kFullFit) R &= fit_tops(sx, dl, wmask, top0);
      R = pop ? R : 0u;
      if (i + 1u == r) {
        while (R) {
          const uint32_t t = (uint32_t)__builtin_ctz(R) ^ top0;
          R &= R - 1u;
          const uint32_t addr = kFullFit || sx < 32u ? x | (t << sx) : x;
          if ((fmix32(addr ^ d.seed_rhfg0) & qmask) == he0) put_cand(d, cs, addr);
        }
      }
      const uint32_t c = popc32(R);
      const uint32_t incl = wave_incl_scan(c);
      const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
      const uint32_t base = size - popped;
      if (base + total <= cap) {
        uint32_t pos = base + total - (incl - c);
        const uint32_t meta = he0 | ((i + 1u) << 24);
        while (R) {
          const uint32_t t = (uint32_t)__builtin_ctz(R) ^ top0;
          R &= R - 1u;
          const u32x2 child = {kFullFit || sx < 32u ? x | (t << sx) : x, meta};
          if (--pos < cap) stk[pos] = child;
        }
        size = base + total;
      } else {
        const uint32_t e = join_lane_dfs(d, cs, tb, wmask, lowmask, qmask, x, he0, i, R);
        nodes += __builtin_amdgcn_readfirstlane(wave_sum(e));
        size = base;
      }
    } else if (g < g_end) {  // 64 values of w for one he0, each with its 4 values of v
      const uint32_t he0 = __builtin_amdgcn_readfirstlane(he0_next);
      const uint32_t w = ((g & ((1u << gsh) - 1u)) << 6) | lane;  // w < 2^(q-4)
      g = take();
      he0_next = ft.l0[g < g_end ? g >> gsh : 0u];
      const uint32_t e = he0 & 63u, top0 = he0 >> (q - dl);
      const uint32_t c2 = (he0 ^ (he0 >> 2)) & 15u;  // row 2: column offset j'/4 ^ c2
      const uint32_t c3 = (he0 ^ (he0 >> 4)) & 3u;   // row 3: column offset j'/16 ^ c3
      const uint32_t wm = (1u << (q - 4u)) - 1u;
      const u32x2 m1 = ft.f1[((he0 >> 6) ^ w) & (qmask >> 6)];
      const uint32_t p2 = xor_perm16(ft.f2[((he0 >> 4) ^ w) & wm], ((c2 & 3u) << 2) | (c2 >> 2));
      // row 3 and row 4 for v = w + k 2^(q-4), k = 0..3: nibble k of each, after the shuffle
      const uint32_t n3s = xor_perm16(ft.f3[((he0 >> 2) ^ w) & wm], c3 | (top0 << 2));
      const uint32_t m4s = xor_perm16(ft.f4[(he0 ^ w) & wm], ((he0 >> (q - 4u)) & 3u) << 2);
      const uint32_t r2 = p2 | (p2 << 16);
      const uint32_t ax = m1.x & r2, ay = m1.y & r2;  // row-2 tuples of (he0, w)
      resolved += popc32(ax) + popc32(ay);
      // Row-3 tuples with at least one row-4 extension go on the stack as nodes of row 4 (they
      // are counted when expanded); the others are counted here.
      uint64_t M0, M1, M2, M3;
      uint32_t c = 0;
      auto row3 = [&](uint32_t k, uint64_t& Mk) {
        const uint32_t n3 = (n3s >> (4u * k)) & 15u;
        uint32_t r3 = n3 | (n3 << 4);
        r3 |= r3 << 8;
        r3 |= r3 << 16;
        const uint32_t mx = ax & r3, my = ay & r3;
        const uint32_t n_j = popc32(mx) + popc32(my);  // row-3 tuples of (he0, v)
        const bool ext = ((m4s >> (4u * k)) & 15u) != 0u;
        resolved += ext ? 0u : n_j;
        c += ext ? n_j : 0u;
        Mk = ext ? ((uint64_t)my << 32) | mx : 0ull;
      };
      row3(0u, M0);
      row3(1u, M1);
      row3(2u, M2);
      row3(3u, M3);
      const uint32_t incl = wave_incl_scan(c);
      const uint32_t total = __builtin_amdgcn_readlane(incl, 63);
      if (size + total <= cap) {  // uniform
        uint32_t pos = size + total - (incl - c);  // this lane's nodes end here
        const uint32_t meta = he0 | (4u << 24);
        while ((M0 | M1) | (M2 | M3)) {  // lowest k first, one prefix per pass
          const bool z0 = M0 != 0ull, z1 = M1 != 0ull, z2 = M2 != 0ull;
          const uint32_t k = z0 ? 0u : (z1 ? 1u : (z2 ? 2u : 3u));
          const uint64_t Mk = z0 ? M0 : (z1 ? M1 : (z2 ? M2 : M3));
          const uint32_t p = (uint32_t)__builtin_ctzll(Mk);
          const uint64_t rest = Mk & (Mk - 1ull);
          M0 = k == 0u ? rest : M0;
          M1 = k == 1u ? rest : M1;
          M2 = k == 2u ? rest : M2;
          M3 = k == 3u ? rest : M3;
          const u32x2 node = {((w | (k << (q - 4u))) << 6) | (fold_pos(p) ^ e), meta};
          stk[--pos] = node;  // positions stay in [size, size + total)
        }
        size += total;
      } else {  // no room: each lane searches its nodes' subtrees itself
        uint32_t e_sub = 0;
        uint64_t Ms[4] = {M0, M1, M2, M3};
        for (uint32_t k = 0; k < 4u; ++k) {
          const uint32_t m4 = (m4s >> (4u * k)) & 15u;
          const uint32_t xv = (w | (k << (q - 4u))) << 6;
          uint64_t Mk = Ms[k];
          while (Mk) {
            const uint32_t x4 = xv | (fold_pos((uint32_t)__builtin_ctzll(Mk)) ^ e);
            Mk &= Mk - 1ull;
            e_sub += 1u + join_lane_dfs(d, cs, tb, wmask, lowmask, qmask, x4, he0, 4u, m4);
          }
        }
        nodes += __builtin_amdgcn_readfirstlane(wave_sum(e_sub));
      }
    } else {
      break;
    }
  }
  return nodes + __builtin_amdgcn_readfirstlane(wave_sum(resolved));
}

// Block-wide copy from global memory into LDS with eight loads per thread in flight before
// the first store (a plain strided loop waits out each load's latency in turn).
// n elements copied by the block's first nt threads (nt = blockDim.x: the whole block)
template <typename D, typename S>
__device__ __forceinline__ void copy_to_lds(D* __restrict__ dst, const S* __restrict__ src,
                                            uint32_t n, uint32_t nt) {
  for (uint32_t base = 0; base < n; base += 8u * nt) {
    S v[8];
#pragma unroll
    for (uint32_t u = 0; u < 8u; ++u) {
      const uint32_t i = base + u * nt + threadIdx.x;
      v[u] = i < n ? src[i] : S(0);
    }
#pragma unroll
    for (uint32_t u = 0; u < 8u; ++u) {
      const uint32_t i = base + u * nt + threadIdx.x;
      if (i < n) dst[i] = (D)v[u];
    }
  }
}
template <typename D, typename S>
__device__ __forceinline__ void copy_to_lds(D* __restrict__ dst, const S* __restrict__ src,
                                            uint32_t n) {
  copy_to_lds(dst, src, n, blockDim.x);
}

// Barrier of the search waves alone, for a launch whose other waves sweep meanwhile and must
// not wait: each wave adds one to an LDS counter (zeroed before the waves split) and waits,
// sleeping, until all `jw` search waves have arrived for this generation.  Every search wave
// calls it the same number of times (the prologue's branches are block-uniform); the wait is
// still bounded (about 2^26 sleeps, over a second): past it the wave goes on and the result
// is false, which the caller reports as a failed search instead of hanging.
__device__ __forceinline__ bool search_sync(uint32_t* ctr, uint32_t jw, uint32_t& gen) {
  ++gen;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (lane_id() == 0u)
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  bool ok = true;
  for (uint32_t spins = 0;
       __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < jw * gen;
       ++spins) {
    if (spins == (1u << 26)) {
      ok = false;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return ok;
}

// LDS: [hot table (kTbLds)] [stacks: waves x cap entries] [hot lists, list_words words]
// [count, base, next group, -, candidate buffer of kCandBuf entries].
// Expected number of nodes of the candidate search when row i is hot at the rate
// hot_rows[i] / 2^q independently: n0 n1 pairs, then each row multiplies by its surviving
// extensions (2^delta values, fewer where bit 32 cuts them off) times its hot rate.
__device__ double join_expected_nodes(const Dev& d) {
  const Ctrl* c = d.ctrl;
  double level = (double)c->hse_count[0] * (double)c->hse_count[1], total = level;
  for (uint32_t i = 2; i < d.r; ++i) {
    const uint32_t sx = (i - 2u) * d.delta + d.q;
    const uint32_t bits = sx >= 32u ? 0u : (32u - sx < d.delta ? 32u - sx : d.delta);
    level *= (double)(1u << bits) * ((double)c->hot_rows[i] / (double)(1u << d.q));
    total += level;
  }
  return total;
}

// Above this many expected nodes (2^36, about 2000 times the search of the scale workload,
// a few tenths of a second) the SRE array is taken as saturated for the window: the search is
// not run and the scan reports a candidate overflow instead of running for minutes.
constexpr double kJoinNodeBudget = 68719476736.0;

// The block's first `jw` waves search; with kSweep the others sweep the SLE array for the row
// live counts meanwhile (one lane of the sweep each, partial counts per wave), so the
// HBM-bound sweep runs beside the ALU-bound search in the same launch.  Sweep waves take part
// in the block's barriers and leave the stacks, lists and candidate buffer alone.
// kSweep: 0 no sweep; 1 the stamp array; 2 the discrete variant's bit array (a symbol of its
// own, so that profiles keep the two apart).
constexpr int kSweepNone = 0, kSweepStamps = 1, kSweepBits = 2;
template <bool kTbLds, int kSweep>
__global__ void __launch_bounds__(kJoinWaves * 64) k_join(Dev d, uint32_t cap,
                                                          uint32_t list_words, uint32_t jw,
                                                          uint32_t lo) {
  extern __shared__ uint32_t sh[];
  const uint32_t q = d.q, r = d.r;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const bool sweeper = kSweep != kSweepNone && wave >= jw;
  const uint32_t off = kTbLds ? (r << q) >> 5 : 0u;  // words of the table in LDS (even)
  // stacks for the search waves only (a sweep wave's pointer is never used)
  u32x2* const stk = reinterpret_cast<u32x2*>(sh + off) + (uint64_t)wave * cap;
  uint32_t* const lw = sh + off + 2u * cap * jw;
  // [count, base, next group, -, kCandBuf entries, sweep counts (kMaxRP per sweep wave)]
  uint32_t* const sink = lw + list_words;
  uint32_t* const swc = sink + 4u + kCandBuf;
  uint32_t* const sctr = swc + (blockDim.x / kWave - jw) * kMaxRP;  // search_sync's counter
  // threads of the search: with sweep waves the search's loops and barriers leave them out, so
  // they start sweeping at once
  const uint32_t nt = kSweep != kSweepNone ? jw * kWave : blockDim.x;
  uint32_t gen = 0;
  auto sync = [&]() {
    if constexpr (kSweep != kSweepNone) {
      if (!search_sync(sctr, jw, gen) && lane_id() == 0u) d.ctrl->join_skipped = 1u;
    } else {
      __syncthreads();
    }
  };
  // a sweep wave's share of the sweep: its per-row counts into the LDS
  auto sweep = [&]() {
    __builtin_amdgcn_s_setprio(2);  // ahead of the search's waves for issue
    const uint32_t sw = blockDim.x / kWave - jw;
    const uint32_t gw = blockIdx.x * sw + (wave - jw);
    uint32_t cnt[kMaxRP];
#pragma unroll
    for (int j = 0; j < kMaxRP; ++j) cnt[j] = 0;
    sweep_lane(d, lo, (uint64_t)gw * kWave + lane_id(), (uint64_t)gridDim.x * sw * kWave, cnt);
#pragma unroll
    for (int j = 0; j < kMaxRP; ++j) {
      const uint32_t c = wave_sum(cnt[j]);
      if (lane_id() == 0) swc[(wave - jw) * kMaxRP + j] = c;
    }
  };
  // after a barrier: the block's counts, one partial per block and row
  auto sweep_store = [&]() {
    if (kSweep != kSweepNone && threadIdx.x < d.rp) {
      uint32_t t = 0;
      for (uint32_t w = 0; w < blockDim.x / kWave - jw; ++w) t += swc[w * kMaxRP + threadIdx.x];
      d.rows_part[(uint64_t)threadIdx.x * kRowsPartWaves + blockIdx.x] = t;
    }
  };
  if (kSweep != kSweepNone) {
    if (threadIdx.x == 0) *sctr = 0u;
    __syncthreads();  // the counter is zero before the waves split
  }
  const uint32_t n0 = d.ctrl->hse_count[0], n1 = d.ctrl->hse_count[1];
  if (n0 == 0u || n1 == 0u || join_expected_nodes(d) > kJoinNodeBudget) {
    // the same verdict in every block: no search; the sweep still runs
    if (n0 != 0u && n1 != 0u && blockIdx.x == 0 && threadIdx.x == 0) d.ctrl->join_skipped = 1u;
    if (kSweep != kSweepNone) {
      if (sweeper) sweep();
      __syncthreads();
      sweep_store();
    }
    return;
  }
  const CandSink cs{sink, sink + 4};
  uint32_t nodes = 0;             // nodes this wave expanded
  unsigned long long extra = 0;   // nodes counted once per grid
  if (sweeper) {
    sweep();
  } else {
  const uint32_t* __restrict__ tb = d.hot_t;
  if (kTbLds) {
    copy_to_lds(sh, d.hot_t, off, nt);
    tb = sh;
  }
  if (threadIdx.x == 0) sink[0] = sink[2] = 0u;  // visible after the first barrier below
  const uint32_t* g0 = d.hse;
  const uint32_t* g1 = d.hse + (1u << q);
  // 32-bit pair arithmetic (24-bit products): pair count and both list sizes small enough
  const bool small = (uint64_t)n0 * n1 <= 0xFFFFFFFFull && n0 < (1u << 24) && n1 < (1u << 24);
  const bool full = (r - 2u) * d.delta + q <= 32u;
  // rows 1-3 in bulk: delta = 2, rows at least 1/8 hot (row 1 stands for all), the tables
  // (3 bitmaps of 2^q bits and the row-0 list) fit in the LDS left after the stacks
  const uint32_t fw = 4u << (q - 5u);  // words of the four reordered bitmaps
  if (kTbLds && d.delta == 2u && r >= 6u && q >= 10u && q <= 16u && (n1 << 3) >= (1u << q) &&
      fw + (n0 + 1u) / 2u <= list_words && fw <= 2u * cap * jw) {
    const uint32_t rw = 1u << (q - 5u);  // words of one bitmap row
    u32x2* const f1 = reinterpret_cast<u32x2*>(lw);
    uint16_t* const f2 = reinterpret_cast<uint16_t*>(lw + rw);
    uint16_t* const f3 = reinterpret_cast<uint16_t*>(lw + 2u * rw);
    uint16_t* const f4 = reinterpret_cast<uint16_t*>(lw + 3u * rw);
    uint16_t* const l0 = reinterpret_cast<uint16_t*>(lw + fw);
    // rows 1-4 of the plain bitmap, staged where the stacks will be
    uint32_t* const h = reinterpret_cast<uint32_t*>(sh + off);
    copy_to_lds(h, d.hot + rw, fw, nt);
    copy_to_lds(l0, g0, n0, nt);
    sync();
    auto hot_bit = [&](uint32_t row, uint32_t col) {  // row >= 1
      return (h[(row - 1u) * rw + (col >> 5)] >> (col & 31u)) & 1u;
    };
    for (uint32_t c = threadIdx.x; c < (1u << (q - 6u)); c += nt) {
      u32x2 o = {0u, 0u};
      for (uint32_t j = 0; j < 64u; ++j) {
        const uint32_t bit = hot_bit(1u, 64u * c + j), p = fold_pos(j);
        if (p < 32u) o.x |= bit << p; else o.y |= bit << (p - 32u);
      }
      f1[c] = o;
    }
    const uint32_t wn = 1u << (q - 4u);
    for (uint32_t c = threadIdx.x; c < wn; c += nt) {
      uint32_t o2 = 0, o3 = 0, o4 = 0;
      for (uint32_t j = 0; j < 16u; ++j) {
        const uint32_t t = j >> 2, b = j & 3u;  // slot t, bit b
        o2 |= hot_bit(2u, 16u * c + j) << ((b << 2) | t);
        o3 |= hot_bit(3u, 4u * (c | (t << (q - 4u))) + b) << j;
        o4 |= hot_bit(4u, (c | (t << (q - 4u))) | (b << (q - 2u))) << j;
      }
      f2[c] = (uint16_t)o2;
      f3[c] = (uint16_t)o3;
      f4[c] = (uint16_t)o4;
    }
    if (blockIdx.x == 0)  // row-1 tuples: every pair (he0, he1)
      extra = (unsigned long long)n0 * n1;
    sync();
    const FoldTables ft{f1, f2, f3, f4, l0, sink + 2};
    nodes = full ? join_wave_fold<true>(d, cs, tb, ft, stk, cap, n0)
                 : join_wave_fold<false>(d, cs, tb, ft, stk, cap, n0);
  } else {
    auto run = [&](auto lists) -> uint32_t {
      if (small && full) return join_wave<true, true>(d, cs, tb, stk, cap, lists, n0, n1, sink + 2);
      if (small) return join_wave<true, false>(d, cs, tb, stk, cap, lists, n0, n1, sink + 2);
      if (full) return join_wave<false, true>(d, cs, tb, stk, cap, lists, n0, n1, sink + 2);
      return join_wave<false, false>(d, cs, tb, stk, cap, lists, n0, n1, sink + 2);
    };
    if (q <= 16u && (n0 + n1 + 1u) / 2u <= list_words) {  // u16 lists in LDS
      uint16_t* const h = reinterpret_cast<uint16_t*>(lw);
      copy_to_lds(h, g0, n0, nt);
      copy_to_lds(h + n0, g1, n1, nt);
      sync();
      nodes = run(HotLists<uint16_t>{h, h + n0});
    } else {
      sync();
      nodes = run(HotLists<uint32_t>{g0, g1});
    }
  }
  }  // the search
  // One counter update per block (thousands of same-address atomics from every wave would
  // queue behind each other at the end of the kernel): each wave leaves its count in its
  // own stack, which is empty by now.
  if (!sweeper && (threadIdx.x & 63u) == 0u) stk[0] = u32x2{nodes, 0u};
  __syncthreads();
  sweep_store();
  const uint32_t nb = sink[0] < kCandBuf ? sink[0] : kCandBuf;  // buffered candidates
  if (threadIdx.x == 0) {
    const u32x2* const stacks = reinterpret_cast<const u32x2*>(sh + off);
    for (uint32_t w = 0; w < jw; ++w) extra += stacks[(uint64_t)w * cap].x;
    atomicAdd(&d.ctrl->join_nodes, extra);
    sink[1] = nb != 0u ? atomicAdd(&d.ctrl->n_cand, nb) : 0u;
  }
  __syncthreads();
  const uint32_t base = sink[1];
  for (uint32_t j = threadIdx.x; j < nb; j += blockDim.x)
    if (base + j < d.cand_cap) d.cand[base + j] = cs.buf[j];
}

// Launch shape of the join: one block per compute unit with as many search waves (up to 16,
// less the sweep waves) as the LDS holds after the hot table (when it is small) and a reserve
// for the hot lists; the lists take whatever LDS is left.  (Two blocks of 10 waves per CU,
// with smaller stacks, measured 7 % slower at the config-2 shape than one block of 16.)
// Sweep waves in each block of the search when the sweep runs inside its launch.  They run at
// a raised wave priority, so that their loads issue as soon as they can: measured at the
// config-2 shape, two such waves beside 14 search waves take 125 us per scan, against 131 us
// with 3 or 4 and 156 us with 1 (137 us with 4 at the default priority).
constexpr uint32_t kJoinSweepWaves = 2;

struct JoinShape {
  bool tb_lds;
  uint32_t cap, waves, sweep_waves, lds, blocks, list_words;
};

JoinShape join_shape(const Dev& d, int n_cu, uint32_t sweep_waves) {
  JoinShape s{};
  s.cap = join_stack_entries(d.delta);
  const uint32_t stack = s.cap * 8u;  // at most 16.5 KiB
  const uint32_t tb = (uint32_t)((((uint64_t)d.r << d.q) >> 5) * 4);
  const uint32_t reserve = 16u << 10;  // 8 Ki u16 list entries at least, when they fit
  s.tb_lds = tb <= (32u << 10) && tb + stack + reserve <= kLdsBytes;
  const uint32_t fixed = s.tb_lds ? tb : 0u;
  s.waves = kLdsBytes >= fixed + stack + reserve ? (kLdsBytes - fixed - reserve) / stack : 1u;
  if (s.waves > kJoinWaves - sweep_waves) s.waves = kJoinWaves - sweep_waves;
  if (s.waves < 1u) s.waves = 1u;
  s.sweep_waves = sweep_waves;
  s.lds = kLdsBytes;
  s.blocks = (uint32_t)n_cu;
  s.list_words = (s.lds - fixed - s.waves * stack - (kCandBuf + 4u) * 4u -
                  (sweep_waves ? (sweep_waves * kMaxRP + 1u) * 4u : 0u)) / 4u;
  return s;
}

hipError_t prepare_join() {
  const void* fns[6] = {reinterpret_cast<const void*>(&k_join<true, kSweepNone>),
                        reinterpret_cast<const void*>(&k_join<false, kSweepNone>),
                        reinterpret_cast<const void*>(&k_join<true, kSweepStamps>),
                        reinterpret_cast<const void*>(&k_join<false, kSweepStamps>),
                        reinterpret_cast<const void*>(&k_join<true, kSweepBits>),
                        reinterpret_cast<const void*>(&k_join<false, kSweepBits>)};
  for (const void* f : fns) {
    hipError_t e =
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Union SLE of host x (Alg. 8): cell z keeps the smallest stamp over the r' rows, i.e. the
// largest distance, so it is live only when live in every row.  When SLEs start on 8-cell
// boundaries each lane takes 8 consecutive cells per pass (one 16-byte load per row, all
// rows' loads in flight together); otherwise one cell per lane.  Per-lane counts are summed
// over the wave once at the end; lane a ends up holding x_a (cells with stamp >=
// max(1, cur - a)) for a < nfeat, and every lane holds |USLE|^k in `live`.
__device__ __forceinline__ void usle_counts(const Dev& d, uint32_t x, uint32_t cur, uint32_t lo,
                                            uint32_t nfeat, uint32_t& live, uint32_t& feat) {
  uint64_t base[kMaxRP];
  const uint32_t qpmask = (1u << d.qp) - 1u;
#pragma unroll
  for (int i = 0; i < kMaxRP; ++i)
    base[i] = (uint64_t)i * d.row_stride + (uint64_t)(fmix32(x ^ d.seed_lh[i]) & qpmask) * d.deltap;
  const uint32_t lane = lane_id();
  uint32_t c_live = 0, c_age[32];
  for (uint32_t a = 0; a < 32; ++a) c_age[a] = 0;
  const bool vec = ((d.deltap & 7u) == 0) && ((d.etap & 7u) == 0);  // uniform
  if (d.mode == SPS_MODE_DISCRETE) {
    // bits: lane takes 32 consecutive cells per pass; a cell of the union is set only when
    // set in every row (the window of 32 bits may straddle two words)
    const uint32_t* w = reinterpret_cast<const uint32_t*>(d.slea);
    for (uint32_t z0 = 0; z0 < d.etap; z0 += 32 * kWave) {
      const uint32_t z = z0 + lane * 32;
      if (z < d.etap) {
        uint32_t m = d.etap - z >= 32u ? 0xFFFFFFFFu : ((1u << (d.etap - z)) - 1u);
#pragma unroll
        for (int i = 0; i < kMaxRP; ++i)
          if (i < (int)d.rp) {
            const uint64_t b = base[i] + z;
            const uint32_t sh = (uint32_t)(b & 31u);
            const uint32_t w0 = w[b >> 5];
            const uint32_t v = sh ? (w0 >> sh) | (w[(b >> 5) + 1] << (32u - sh)) : w0;
            m &= v;
          }
        c_live += __popc(m);
      }
    }
  } else if (vec) {
    // two passes of 8 cells per lane at a time: all rows' loads of both passes in flight
    auto count8 = [&](const u32x4* v) {
      uint32_t m[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) m[k] = 0xFFFFu;
#pragma unroll
      for (int i = 0; i < kMaxRP; ++i) {
        if (i < (int)d.rp) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t w = k < 2 ? v[i].x : (k < 4 ? v[i].y : (k < 6 ? v[i].z : v[i].w));
            const uint32_t c = (k & 1) ? w >> 16 : w & 0xFFFFu;
            m[k] = c < m[k] ? c : m[k];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        c_live += m[k] >= lo;  // lo >= 1, so never-written cells are not live
        for (uint32_t a = 0; a < nfeat; ++a) {
          const uint32_t lo_a = cur > a + 1u ? cur - a : 1u;
          c_age[a] += m[k] >= lo_a;
        }
      }
    };
    for (uint32_t z0 = 0; z0 < d.etap; z0 += 16 * kWave) {
      const uint32_t za = z0 + lane * 8, zb = za + 8 * kWave;
      const bool ina = za < d.etap, inb = zb < d.etap;
      u32x4 va[kMaxRP], vb[kMaxRP];
#pragma unroll
      for (int i = 0; i < kMaxRP; ++i) {
        if (i < (int)d.rp) {
          if (ina) va[i] = *reinterpret_cast<const u32x4*>(d.slea + base[i] + za);
          if (inb) vb[i] = *reinterpret_cast<const u32x4*>(d.slea + base[i] + zb);
        }
      }
      if (ina) count8(va);
      if (inb) count8(vb);
    }
  } else {
    for (uint32_t z0 = 0; z0 < d.etap; z0 += kWave) {
      const uint32_t z = z0 + lane;
      if (z < d.etap) {
        uint32_t m = 0xFFFFu;
#pragma unroll
        for (int i = 0; i < kMaxRP; ++i)
          if (i < (int)d.rp) {
            const uint32_t v = d.slea[base[i] + z];
            m = v < m ? v : m;
          }
        c_live += m >= lo;
        for (uint32_t a = 0; a < nfeat; ++a) {
          const uint32_t lo_a = cur > a + 1u ? cur - a : 1u;
          c_age[a] += m >= lo_a;
        }
      }
    }
  }
  live = wave_sum(c_live);
  feat = 0;
  for (uint32_t a = 0; a < nfeat; ++a) {
    const uint32_t t = wave_sum(c_age[a]);
    if (lane == a) feat = t;
  }
}

// Learned estimator (3-layer perceptron 10 -> 64 -> 64 -> 1 with ReLU): features in lanes
// 0..9 of the wave, hidden unit j in lane j.  Weights are read as float and rounded to
// bfloat16 (round to nearest even), activations likewise; products accumulate in float.
__device__ __forceinline__ float to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ float mlp_forward_wave(const float* __restrict__ w, float in_lane) {
  // in_lane: encoded feature of lane k (k < 10)
  const uint32_t lane = lane_id();
  const float* W1 = w;
  const float* b1 = W1 + SPS_MLP_HIDDEN * SPS_MLP_IN;
  const float* W2 = b1 + SPS_MLP_HIDDEN;
  const float* b2 = W2 + SPS_MLP_HIDDEN * SPS_MLP_HIDDEN;
  const float* W3 = b2 + SPS_MLP_HIDDEN;
  const float* b3 = W3 + SPS_MLP_HIDDEN;
  const float xin = to_bf16(in_lane);
  float acc = 0.f;
  for (int k = 0; k < SPS_MLP_IN; ++k)
    acc += to_bf16(W1[lane * SPS_MLP_IN + k]) * __shfl(xin, k, kWave);
  float h1 = to_bf16(fmaxf(acc + b1[lane], 0.f));
  acc = 0.f;
  for (int k = 0; k < SPS_MLP_HIDDEN; ++k)
    acc += to_bf16(W2[lane * SPS_MLP_HIDDEN + k]) * __shfl(h1, k, kWave);
  const float h2 = to_bf16(fmaxf(acc + b2[lane], 0.f));
  float y = to_bf16(W3[lane]) * h2;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) y += __shfl_xor(y, o, kWave);
  return y + b3[0];
}

// Stage 4: order the kept hosts ascending (hosts are distinct; keys are host << 32 | index
// into the kept list, padded with keys above every host).  Every block first turns the
// estimate waves' kept counts into the ordinal of each wave's first host (a prefix sum).
//   n <= 1024: block 0 alone, one key per thread, a bitonic network in registers with
//              cross-lane moves (DPP, permutes) for partners closer than 64 and LDS beyond.
//   n <= 4096: block 0 alone, the same network with two or four keys per thread (partners
//              1024 or more keys apart in the same thread).
//   n >  4096: every block sorts 4096-key tiles with that network and writes them to
//              skeys; the last block to finish (a counter) then places every key at its
//              rank: its position in its own tile plus, for every other tile, the number of
//              smaller keys there (a binary search).
// The block that ends the kernel writes the info words and the inspection copies and clears
// the working counters for the next scan (kernel boundaries make the earlier kernels'
// results visible; within this kernel the tiles pass through a release / acquire pair).
constexpr int kSortThreads = 1024;
constexpr int kSortTile = 4096;
constexpr uint32_t kSortMaxBlocks = 16;  // blocks of the sort (tiles taken round robin)

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t n, uint32_t lo) {
  uint32_t P = lo;
  while (P < n) P <<= 1;
  return P;
}

// The end of a scan: info words, inspection copies, working counters cleared.
__device__ void scan_finish(const Dev& d, uint32_t cap, uint32_t* __restrict__ info) {
  Ctrl* c = d.ctrl;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (info) {
      info[SPS_INFO_KEPT] = c->n_kept;
      info[SPS_INFO_CAND] = c->n_cand;
      info[SPS_INFO_FLAGS] = (c->n_cand > d.cand_cap || c->join_skipped ? 1u : 0u) |
                             (c->n_kept > cap ? 2u : 0u) | (c->join_skipped ? 4u : 0u);
      info[SPS_INFO_HSE0] = c->hse_count[0];
      info[SPS_INFO_HSE1] = c->hse_count[1];
      info[SPS_INFO_NODES_LO] = (uint32_t)c->join_nodes;
      info[SPS_INFO_NODES_HI] = (uint32_t)(c->join_nodes >> 32);
      info[7] = 0;
    }
    for (uint32_t i = 0; i < (uint32_t)kMaxRP; ++i) c->last_row_live[i] = c->row_live[i];
    c->last_n_cand = c->n_cand;
    c->last_hse[0] = c->hse_count[0];
    c->last_hse[1] = c->hse_count[1];
  }
  __syncthreads();
  uint32_t* w = reinterpret_cast<uint32_t*>(c);
  for (uint32_t i = threadIdx.x; i < kCtrlWorkingWords; i += blockDim.x) w[i] = 0;
}

// Offsets of the kept hosts.  Estimate wave w left wave_kept[w] hosts at the start of region
// w of the kept list; pre[w] receives the number of kept hosts in the waves before w (the
// ordinal of its first one).  Two waves' counts per thread (a, b); returns the total.
__device__ __forceinline__ uint32_t kept_offsets(const Dev& d, uint32_t* pre, uint32_t& a,
                                                 uint32_t& b) {
  static_assert(kEstWaves == 2u * kSortThreads, "two estimate waves per thread of the sort");
  __shared__ uint32_t wave_tot[kSortThreads / kWave];
  const uint32_t t = threadIdx.x;
  const uint32_t region = kept_region(d.cand_cap);  // no wave keeps more
  a = min(d.wave_kept[2 * t], region);
  b = min(d.wave_kept[2 * t + 1], region);
  const uint32_t inc = wave_incl_scan(a + b);
  if (lane_id() == kWave - 1) wave_tot[t / kWave] = inc;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (uint32_t w = 0; w < kSortThreads / kWave; ++w) {
    const uint32_t v = wave_tot[w];
    before += w < t / kWave ? v : 0u;
    total += v;
  }
  pre[2 * t] = before + inc - a - b;
  pre[2 * t + 1] = before + inc - b;
  __syncthreads();
  return min(total, d.cand_cap);  // at most one kept host per candidate
}

// Index into the kept list of kept host number i (i < total): it belongs to the last wave
// whose offset is at most i.
__device__ __forceinline__ uint32_t kept_slot(const uint32_t* pre, uint32_t region, uint32_t i) {
  uint32_t lo = 0, hi = kEstWaves;  // pre[lo] <= i, and i < the offset past wave hi - 1
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= i) lo = mid; else hi = mid;
  }
  return lo * region + (i - pre[lo]);
}

// The value of lane (this lane ^ J), J < 64: DPP within a quad (J = 1, 2) or a 16-lane row
// (J = 4, 8; row_ror:n reads lane (l - n) mod 16), a cross-lane permute for 16 and 32.
template <uint32_t J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // 1,0,3,2
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // 2,3,0,1
  } else if constexpr (J == 4) {
    const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false);
    const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x12C, 0xF, 0xF, false);
    return (lane_id() & 4u) ? dn : up;
  } else if constexpr (J == 8) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
  } else {
    return (uint32_t)__shfl_xor((int)v, (int)J, kWave);
  }
}

// Stages J, J/2, ..., 1 of bitonic merge step k on one key per lane, in registers (the
// partner distance is a compile-time constant, so every stage is one fixed exchange).
template <uint32_t J>
__device__ __forceinline__ void bitonic_lanes(uint64_t& v, uint32_t i, uint32_t k) {
  const uint32_t lo = lane_xor<J>((uint32_t)v), hi = lane_xor<J>((uint32_t)(v >> 32));
  const uint64_t w = ((uint64_t)hi << 32) | lo;
  const bool up = (i & k) == 0u, lower = (i & J) == 0u;
  v = (lower == up) ? (v < w ? v : w) : (v < w ? w : v);
  if constexpr (J > 1) bitonic_lanes<J / 2>(v, i, k);
}

// Ascending / descending compare-exchange of two keys held by one thread.
__device__ __forceinline__ void key_cmpx(uint64_t& a, uint64_t& b, bool up) {
  const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = up ? lo : hi;
  b = up ? hi : lo;
}

// Bitonic sort of the first n (1024 < n <= S * 1024) keys of key[] by one block of 1024
// threads: thread t holds keys s * 1024 + t (slot s < S) in registers.  Partners 1024 or more
// keys apart are in the same thread, partners 64 ... 512 apart are exchanged through LDS,
// closer ones within the wave.  Keys past n are padding above every key.
template <uint32_t S>
__device__ __forceinline__ void bitonic_slots(uint64_t* key, uint32_t n, uint64_t (&v)[S]) {
  const uint32_t t = threadIdx.x;
#pragma unroll
  for (uint32_t s = 0; s < S; ++s) v[s] = s * 1024u + t < n ? key[s * 1024u + t] : ~0ull;
#pragma unroll
  for (uint32_t s = 0; s < S; ++s) {
    const uint32_t x = s * 1024u + t;
    bitonic_lanes<1>(v[s], x, 2);
    bitonic_lanes<2>(v[s], x, 4);
    bitonic_lanes<4>(v[s], x, 8);
    bitonic_lanes<8>(v[s], x, 16);
    bitonic_lanes<16>(v[s], x, 32);
    bitonic_lanes<32>(v[s], x, 64);
  }
  for (uint32_t k = 128; k <= S * 1024u; k <<= 1) {
    // slot pairs (s, s + j / 1024); the pair sorts ascending when key s * 1024 + t has bit k
    // clear (t < 1024 < k here)
    for (uint32_t j = k >> 1; j >= 1024u; j >>= 1) {
      if (j == 2048u) {
        if constexpr (S == 4) {
          key_cmpx(v[0], v[2], true);
          key_cmpx(v[1], v[3], (1024u & k) == 0u);
        }
      } else {
        key_cmpx(v[0], v[1], true);
        if constexpr (S == 4) key_cmpx(v[2], v[3], (2048u & k) == 0u);
      }
    }
    for (uint32_t j = (k >> 1) < 512u ? (k >> 1) : 512u; j >= 64u; j >>= 1) {
      __syncthreads();  // the previous stage's readers are done
#pragma unroll
      for (uint32_t s = 0; s < S; ++s) key[s * 1024u + t] = v[s];
      __syncthreads();
#pragma unroll
      for (uint32_t s = 0; s < S; ++s) {
        const uint32_t x = s * 1024u + t;
        const uint64_t w = key[x ^ j];
        const bool asc = (x & k) == 0u, lower = (x & j) == 0u;
        v[s] = (lower == asc) ? (v[s] < w ? v[s] : w) : (v[s] < w ? w : v[s]);
      }
    }
#pragma unroll
    for (uint32_t s = 0; s < S; ++s) bitonic_lanes<32>(v[s], s * 1024u + t, k);
  }
}

__global__ void __launch_bounds__(kSortThreads) k_rank_sort(Dev d, sps_result* __restrict__ out,
                                                            uint32_t cap,
                                                            uint32_t* __restrict__ info) {
  __shared__ uint64_t key[kSortTile];
  __shared__ uint32_t pre[kEstWaves];
  __shared__ uint32_t last;
  Ctrl* c = d.ctrl;
  uint32_t cnt_a, cnt_b;
  // the same in every lane; said so, the loops below stay scalar
  const uint32_t n = __builtin_amdgcn_readfirstlane(kept_offsets(d, pre, cnt_a, cnt_b));
  const uint32_t region = kept_region(d.cand_cap);
  const bool tiled = out && n > (uint32_t)kSortTile;
  if (!tiled && blockIdx.x != 0) return;  // block 0 orders short lists alone
  if (out && !tiled) {
    // key[i] = host << 32 | index into the kept list, for kept host number i
    for (uint32_t h = 0; h < 2u; ++h) {
      const uint32_t w = 2 * threadIdx.x + h, cnt = h ? cnt_b : cnt_a;
      for (uint32_t l = 0; l < cnt && pre[w] + l < n; ++l) {
        const uint32_t slot = w * region + l;
        key[pre[w] + l] = ((uint64_t)d.kept[slot].host << 32) | slot;
      }
    }
    __syncthreads();
  }
  if (out && n <= (uint32_t)kSortThreads) {
    const uint32_t P = pow2_at_least(n, 64u);
    const uint32_t i = threadIdx.x;
    uint64_t v = i < n ? key[i] : ~0ull;
    // merge steps k = 2 ... 64 within the wave, then k = 128 ... P: the stages with partners
    // 64 or more lanes away through LDS, the rest within the wave
    bitonic_lanes<1>(v, i, 2);
    bitonic_lanes<2>(v, i, 4);
    bitonic_lanes<4>(v, i, 8);
    bitonic_lanes<8>(v, i, 16);
    bitonic_lanes<16>(v, i, 32);
    bitonic_lanes<32>(v, i, 64);
    for (uint32_t k = 128; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j >= 64u; j >>= 1) {
        __syncthreads();  // the previous stage's readers are done
        key[i] = v;
        __syncthreads();
        const uint64_t w = key[i ^ j];
        const bool up = (i & k) == 0u, lower = (i & j) == 0u;
        v = (lower == up) ? (v < w ? v : w) : (v < w ? w : v);
      }
      bitonic_lanes<32>(v, i, k);
    }
    const uint32_t m = n < cap ? n : cap;
    if (i < m) out[i] = d.kept[(uint32_t)v];
  } else if (out && !tiled) {
    const uint32_t m = n < cap ? n : cap;
    if (n <= 2048u) {
      uint64_t v[2];
      bitonic_slots<2>(key, n, v);
#pragma unroll
      for (uint32_t s = 0; s < 2u; ++s)
        if (s * 1024u + threadIdx.x < m) out[s * 1024u + threadIdx.x] = d.kept[(uint32_t)v[s]];
    } else {
      uint64_t v[4];
      bitonic_slots<4>(key, n, v);
#pragma unroll
      for (uint32_t s = 0; s < 4u; ++s)
        if (s * 1024u + threadIdx.x < m) out[s * 1024u + threadIdx.x] = d.kept[(uint32_t)v[s]];
    }
  } else if (tiled) {
    const uint32_t n_tiles = (n + kSortTile - 1) / kSortTile;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
      const uint32_t t0 = t * kSortTile;
      const uint32_t len = n - t0 < (uint32_t)kSortTile ? n - t0 : (uint32_t)kSortTile;
      for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        const uint32_t slot = kept_slot(pre, region, t0 + i);
        key[i] = ((uint64_t)d.kept[slot].host << 32) | slot;
      }
      __syncthreads();
      uint64_t v[4];
      bitonic_slots<4>(key, len, v);
#pragma unroll
      for (uint32_t s = 0; s < 4u; ++s)
        if (s * 1024u + threadIdx.x < len) d.skeys[t0 + s * 1024u + threadIdx.x] = v[s];
      __syncthreads();  // key[] is rewritten by the next tile
    }
    // release this block's tiles, then count it; the last block goes on alone
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(&c->sort_done, 1u) == gridDim.x - 1u ? 1u : 0u;
    __syncthreads();
    if (!last) return;
    __threadfence();  // acquire: every block's tiles are visible from here on
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint64_t k = d.skeys[i];
      const uint32_t own = i / kSortTile;
      uint32_t rank = i - own * kSortTile;
      for (uint32_t t = 0; t < n_tiles; ++t) {
        if (t == own) continue;
        const uint64_t* tk = d.skeys + (uint64_t)t * kSortTile;
        uint32_t lo = 0, hi = n - t * kSortTile < (uint32_t)kSortTile ? n - t * kSortTile
                                                                    : (uint32_t)kSortTile;
        while (lo < hi) {  // number of keys of tile t below k
          const uint32_t mid = (lo + hi) >> 1;
          if (tk[mid] < k) lo = mid + 1u; else hi = mid;
        }
        rank += lo;
      }
      if (rank < cap) out[rank] = d.kept[(uint32_t)k];
    }
  }
  if (threadIdx.x == 0) c->n_kept = n;  // read by scan_finish in this same thread
  scan_finish(d, cap, info);
}

// Stage 3 (Alg. 8, Eq. 12, Eq. 9, final filter).  One wave per candidate.  With a host
// list (`hosts` non-null) every host is estimated and written to direct[c] unfiltered.
// In a scan the blocks also clear the join's table (the join has finished) for the next
// scan.
__global__ void __launch_bounds__(256) k_estimate(Dev d, uint32_t cur, uint32_t lo, uint32_t k,
                                                  double threshold, MlpRef mlp,
                                                  const uint32_t* __restrict__ hosts,
                                                  uint32_t n_hosts,
                                                  sps_result* __restrict__ direct,
                                                  uint32_t rows_waves) {
  __shared__ uint32_t rl[kMaxRP];
  if (rows_waves) {
    // the row live counts from the sweep's per-wave partials (each block adds them up; block
    // 0 also leaves them in the control words)
    __shared__ uint32_t red[kMaxRP][256 / kWave];
    uint32_t v[kMaxRP];  // every row's loads issued before any is summed
#pragma unroll
    for (int j = 0; j < kMaxRP; ++j) {
      uint32_t c = 0;
      if ((uint32_t)j < d.rp)
        for (uint32_t w = threadIdx.x; w < rows_waves; w += blockDim.x)
          c += d.rows_part[(uint64_t)j * kRowsPartWaves + w];
      v[j] = c;
    }
#pragma unroll
    for (int j = 0; j < kMaxRP; ++j) {
      const uint32_t c = wave_sum(v[j]);
      if (lane_id() == 0 && (uint32_t)j < d.rp) red[j][threadIdx.x / kWave] = c;
    }
    __syncthreads();
    if (threadIdx.x < d.rp) {
      uint32_t t = 0;
      for (uint32_t w = 0; w < blockDim.x / kWave; ++w) t += red[threadIdx.x][w];
      rl[threadIdx.x] = t;
      if (blockIdx.x == 0) d.ctrl->row_live[threadIdx.x] = t;
    }
  } else if (threadIdx.x < d.rp) {
    rl[threadIdx.x] = d.ctrl->row_live[threadIdx.x];
  }
  __syncthreads();
  const uint32_t n = hosts ? n_hosts : min(d.ctrl->n_cand, d.cand_cap);
  const uint32_t* __restrict__ src = hosts ? hosts : d.cand;
  if (!hosts) {
    const uint32_t words = (d.r << d.q) >> 5;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < words; w += gridDim.x * blockDim.x)
      d.hot_t[w] = 0;
  }
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  const uint32_t lane = lane_id();
  const bool use_mlp = mlp.w != nullptr && k == SPS_MLP_IN;
  const uint32_t nfeat = use_mlp ? SPS_MLP_IN : 0u;
  double P = 1.0;  // product of the row setting factors SF(i, k), rows in order
  for (uint32_t i = 0; i < d.rp; ++i)
    P = P * ((double)rl[i] / (double)d.row_len);
  const uint32_t c0 = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  // the first host is read before the count is known (in bounds: c0 < the list's capacity)
  const uint32_t x0 = c0 < (hosts ? n_hosts : d.cand_cap) ? src[c0] : 0u;
  // in a scan (kEstWaves waves) wave c0 keeps its hosts in region c0 of the kept list, which
  // holds every candidate it can get, and leaves their number in wave_kept[c0]: no counter
  // shared between waves
  const uint32_t region = kept_region(d.cand_cap);
  uint32_t n_keep = 0;
  for (uint32_t c = c0; c < n; c += waves) {
    const uint32_t x = __builtin_amdgcn_readfirstlane(c == c0 ? x0 : src[c]);
    uint32_t U, feat;
    usle_counts(d, x, cur, lo, nfeat, U, feat);
    const double etap = (double)d.etap;
    double w;
    uint32_t flags = 0;
    if (P >= 1.0)
      w = (double)U;
    else
      w = ((double)U - etap * P) / (1.0 - P);
    if (w < 0.0) {
      w = 0.0;
      flags |= SPS_F_CLAMPLOW;
    }
    if (w > etap - 1.0) {
      w = etap - 1.0;
      flags |= SPS_F_SATURATED;
    }
    double est = -etap * log1p(-w / etap);
    if (use_mlp) {
      // the network replaces linear counting only inside its validated domain
      const float f = lane < SPS_MLP_IN ? (float)feat / (float)d.etap : 0.f;
      const bool in_range = lane >= SPS_MLP_IN || (f >= mlp.lo[lane] && f <= mlp.hi[lane]);
      const bool all_in = __ballot(!in_range) == 0;
      const bool informative = __shfl(feat, 0, kWave) < d.etap - 1u;
      const float y = mlp_forward_wave(mlp.w, lane < SPS_MLP_IN ? mlp_encode(feat, d.etap) : 0.f);
      if (U >= mlp.min_live && all_in && informative && y >= 0.f && y <= mlp.log_max) {
        // a saturated linear count is the largest value it can express, so the network
        // may only raise it
        const double e_net = (double)expf(y);
        est = (flags & SPS_F_SATURATED) && e_net < est ? est : e_net;
        flags |= SPS_F_MLP;
      } else {
        flags |= SPS_F_LC_FALLBACK;
      }
    }
    if (fabs(est - threshold) <= 1e-9 * threshold) flags |= SPS_F_NEAR;
    // lane 0's decision (every lane computes the same estimate)
    const bool keep = !direct && __builtin_amdgcn_readfirstlane(est >= threshold ? 1 : 0);
    if (lane == 0) {
      sps_result res;
      res.host = x;
      res.live = U;
      res.flags = flags;
      res.pad = 0;
      res.estimate = est;
      if (direct)
        direct[c] = res;
      else if (keep)
        d.kept[(uint64_t)c0 * region + n_keep] = res;
    }
    n_keep += keep ? 1u : 0u;
  }
  if (!direct && lane == 0) d.wave_kept[c0] = n_keep;
}

hipError_t launch_scan(const Dev& d, uint32_t cur, uint32_t window, double threshold,
                       sps_result* out, uint32_t cap, uint32_t* info, const MlpRef& mlp,
                       bool use_hist, uint32_t mode, int n_cu, hipStream_t st) {
  const uint32_t lo = cur >= window ? cur - window + 1 : 1u;
  ProfScope whole(SPS_STAGE_SCAN, st);
  // The row live counts are needed only by the estimate, and the sweep that makes them
  // (HBM-bound) shares nothing with the candidate search (ALU-bound, in LDS): by default the
  // sweep runs in the search's own launch, in waves of their own beside the search's, with
  // no cross-stream synchronization.  With histograms the counts are a few hundred bins,
  // taken with the SRE pass.  Partial counts: one per block of the search, or one per wave
  // of k_scan_rows (n_cu blocks of 4 waves).
  const bool fits = (uint32_t)n_cu * 4u <= kRowsPartWaves;
  const bool fused = !use_hist && fits && mode != kScanSerial;
  const bool serial = !use_hist && fits && mode == kScanSerial;
  uint32_t rows_waves = 0;  // partial counts of the sweep for the estimate to add up
  {
    // the hot SREs (and, with histograms or when no partials fit, the row live counts)
    ProfScope ps(SPS_STAGE_SCAN_STATS, st, ProfScope::kKernel);
    const bool sweep_here = !use_hist && !fits;
    if (d.q - d.delta >= 6u && !sweep_here) {
      const uint32_t tiles = d.r << (d.q - d.delta - 6u);
      const uint32_t blocks = tiles < (uint32_t)n_cu * 8u ? tiles : (uint32_t)n_cu * 8u;
      launch_k(ps, k_scan_sre, dim3(blocks > d.rp ? blocks : d.rp), dim3(256), 0, st, d, lo,
               cur, use_hist ? 1u : 0u);
    } else {
      const uint32_t rows = use_hist ? (kStatsRows | kStatsHist) : sweep_here ? kStatsRows : 0u;
      launch_k(ps, k_scan_stats, dim3((uint32_t)n_cu), dim3(256), 0, st, d, lo, cur,
               kStatsSre | rows);
    }
  }
  {
    ProfScope ps(SPS_STAGE_JOIN, st, ProfScope::kKernel);
    const JoinShape js = join_shape(d, n_cu, fused ? kJoinSweepWaves : 0u);
    const dim3 grid(js.blocks), block((js.waves + js.sweep_waves) * kWave);
    if (fused) rows_waves = js.blocks;  // one partial per block
    const bool bits = d.mode == SPS_MODE_DISCRETE;
    if (fused && bits) {
      if (js.tb_lds)
        launch_k(ps, k_join<true, kSweepBits>, grid, block, js.lds, st, d, js.cap,
                 js.list_words, js.waves, lo);
      else
        launch_k(ps, k_join<false, kSweepBits>, grid, block, js.lds, st, d, js.cap,
                 js.list_words, js.waves, lo);
    } else if (fused) {
      if (js.tb_lds)
        launch_k(ps, k_join<true, kSweepStamps>, grid, block, js.lds, st, d, js.cap,
                 js.list_words, js.waves, lo);
      else
        launch_k(ps, k_join<false, kSweepStamps>, grid, block, js.lds, st, d, js.cap,
                 js.list_words, js.waves, lo);
    } else {
      if (js.tb_lds)
        launch_k(ps, k_join<true, kSweepNone>, grid, block, js.lds, st, d, js.cap,
                 js.list_words, js.waves, lo);
      else
        launch_k(ps, k_join<false, kSweepNone>, grid, block, js.lds, st, d, js.cap,
                 js.list_words, js.waves, lo);
    }
  }
  if (serial) {  // the sweep as a kernel of its own after the search
    ProfScope ps(SPS_STAGE_SCAN_ROWS, st, ProfScope::kKernel);
    if (d.mode == SPS_MODE_DISCRETE)
      launch_k(ps, k_scan_rows<true>, dim3((uint32_t)n_cu), dim3(256), 0, st, d, lo, cur);
    else
      launch_k(ps, k_scan_rows<false>, dim3((uint32_t)n_cu), dim3(256), 0, st, d, lo, cur);
    rows_waves = (uint32_t)n_cu * 4u;
  }
  {
    ProfScope ps(SPS_STAGE_ESTIMATE, st, ProfScope::kKernel);
    launch_k(ps, k_estimate, dim3(kEstWaves / (256 / kWave)), dim3(256), 0, st, d, cur, lo,
             window, threshold, mlp, (const uint32_t*)nullptr, 0u, (sps_result*)nullptr,
             rows_waves);
  }
  {
    ProfScope ps(SPS_STAGE_SORT, st, ProfScope::kKernel);
    // few blocks: the kept count is known only on the device, and most scans keep fewer than
    // kSortTile hosts, which block 0 orders alone while the others only start and exit
    const uint32_t tiles = (d.cand_cap + kSortTile - 1) / kSortTile;
    const uint32_t blocks = tiles < kSortMaxBlocks ? tiles : kSortMaxBlocks;
    launch_k(ps, k_rank_sort, dim3(blocks), dim3(kSortThreads), 0, st, d, out, cap, info);
  }
  return hipGetLastError();
}

// Estimates of given hosts: SLE row live counts, then the estimate of every host, then the
// counters cleared.
hipError_t launch_estimate_hosts(const Dev& d, uint32_t cur, uint32_t window,
                                 const uint32_t* hosts, uint32_t n, sps_result* out,
                                 const MlpRef& mlp, bool use_hist, int n_cu, hipStream_t st) {
  const uint32_t lo = cur >= window ? cur - window + 1 : 1u;
  {
    // row live counts only (no SREs)
    ProfScope ps(SPS_STAGE_SCAN_STATS, st, ProfScope::kKernel);
    launch_k(ps, k_scan_stats, dim3((uint32_t)n_cu), dim3(256), 0, st, d, lo, cur,
             kStatsRows | (use_hist ? kStatsHist : 0u));
  }
  if (n) {
    uint32_t blocks = (n + 3) / 4;
    if (blocks > (uint32_t)n_cu * 8) blocks = (uint32_t)n_cu * 8;
    ProfScope ps(SPS_STAGE_ESTIMATE, st, ProfScope::kKernel);
    launch_k(ps, k_estimate, dim3(blocks), dim3(256), 0, st, d, cur, lo, window, 0.0, mlp,
             hosts, n, out, 0u);
  }
  return launch_scan_reset(d, false, st);  // the counters are clear again
}

// Features only: per-age cumulative union-SLE live counts of given hosts.
__global__ void __launch_bounds__(256) k_features(Dev d, uint32_t cur, uint32_t k,
                                                  const uint32_t* __restrict__ hosts,
                                                  uint64_t n, uint32_t* __restrict__ x) {
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / kWave);
  const uint32_t lo = cur >= k ? cur - k + 1 : 1u;
  for (uint64_t c = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; c < n; c += waves) {
    const uint32_t h = __builtin_amdgcn_readfirstlane(hosts[c]);
    uint32_t U, feat;
    usle_counts(d, h, cur, lo, k, U, feat);
    if (lane_id() < k) x[c * k + lane_id()] = feat;
  }
}

hipError_t launch_features(const Dev& d, uint32_t cur, uint32_t window, const uint32_t* hosts,
                           uint64_t n, uint32_t* x, int n_cu, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 3) / 4;
  if (blocks > (uint64_t)n_cu * 8) blocks = (uint64_t)n_cu * 8;
  ProfScope ps(SPS_STAGE_FEATURES, st, ProfScope::kKernel);
  launch_k(ps, k_features, dim3((uint32_t)blocks), dim3(256), 0, st, d, cur, window,
           hosts, n, x);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Roofline probes: the ingest's store pattern and the scan's read pattern, without the
// method's hashing.
// ---------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_probe_scatter(uint16_t* __restrict__ cells,
                                                       uint64_t n_cells, uint64_t n,
                                                       uint32_t seed, uint16_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t h1 = fmix32((uint32_t)i ^ seed);
    const uint32_t h2 = fmix32((uint32_t)(i >> 32) ^ h1 ^ 0x9E3779B9u);
    const uint64_t r = ((uint64_t)h1 << 32) | h2;
    cells[__umul64hi(r, n_cells)] = v;
  }
}

__global__ void __launch_bounds__(256) k_probe_stream(const u32x4* __restrict__ buf,
                                                      uint64_t nvec, uint32_t* sum) {
  // the scan's SLE access shape: grid-stride, eight 16-byte non-temporal loads per lane
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 7 * stride < nvec; i += 8 * stride) {
    u32x4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(&buf[i + u * stride]);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < nvec; i += stride) {
    const u32x4 v = __builtin_nontemporal_load(&buf[i]);
    acc += v.x ^ v.y ^ v.z ^ v.w;
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) atomicAdd(sum, acc);
}

// Replay probe: exactly the stores of an ingest -- the same cells and stamp, issued from the
// XCD the ingest's host-class partition sends them to -- taken from a recorded list of cell
// indices instead of hashed pairs.  k_probe_record (one pair per lane) counts the cells of
// each host class (fill = 0; pos[c] accumulates) or, with pos[c] preset to the classes'
// region offsets, writes each pair's cells as u32 indices into the SRE-then-SLE state
// (u16 units) into its class's region (fill = 1).
__global__ void __launch_bounds__(256) k_probe_record(Dev d, const u32x2* __restrict__ pkts,
                                                      uint64_t n, uint32_t sle_off,
                                                      uint32_t* __restrict__ cells,
                                                      unsigned long long* __restrict__ pos,
                                                      uint32_t fill) {
  __shared__ uint32_t cnt[kXcds];
  __shared__ unsigned long long base[kXcds];
  if (threadIdx.x < kXcds) cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t cls = 0, mine = 0;
  u32x2 pk = {0u, 0u};
  if (i < n) {
    pk = pkts[i];
    cls = host_class(d.anet_side ? pk.x : pk.y) & (kXcds - 1u);
    uint32_t m = 0;
    pair_cells(d, pk.x, pk.y, [&](uint64_t, bool, uint32_t) { ++m; });
    mine = atomicAdd(&cnt[cls], m);
  }
  __syncthreads();
  if (threadIdx.x < kXcds)
    base[threadIdx.x] = atomicAdd(&pos[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
  __syncthreads();
  if (fill && i < n) {
    uint64_t o = base[cls] + mine;
    pair_cells(d, pk.x, pk.y, [&](uint64_t cell, bool in_sre, uint32_t) {
      cells[o++] = (uint32_t)(in_sre ? cell : sle_off + cell);
    });
  }
}

__global__ void __launch_bounds__(256) k_probe_replay(uint16_t* __restrict__ state,
                                                      const uint32_t* __restrict__ cells,
                                                      ClassOffsets co, uint16_t v) {
  const uint32_t cls = blockIdx.x % kXcds;
  const uint64_t stride = (uint64_t)(gridDim.x / kXcds) * blockDim.x;
  const uint64_t end = co.off[cls + 1];
  for (uint64_t i = co.off[cls] + (uint64_t)(blockIdx.x / kXcds) * blockDim.x + threadIdx.x;
       i < end; i += stride)
    state[cells[i]] = v;
}

hipError_t launch_probe_record(const Dev& d, const sps_pkt* pkts, uint64_t n, uint32_t sle_off,
                               uint32_t* cells, unsigned long long* pos, bool fill,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  ProfScope ps(SPS_STAGE_PROBE, st, ProfScope::kKernel);
  launch_k(ps, k_probe_record, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, d,
           reinterpret_cast<const u32x2*>(pkts), n, sle_off, cells, pos,
           fill ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_probe_replay(uint16_t* state, const uint32_t* cells, const ClassOffsets& co,
                               uint16_t value, int blocks, hipStream_t st) {
  uint32_t b = (uint32_t)blocks / kXcds * kXcds;
  if (b < kXcds) b = kXcds;
  ProfScope ps(SPS_STAGE_PROBE, st, ProfScope::kKernel);
  launch_k(ps, k_probe_replay, dim3(b), dim3(256), 0, st, state, cells, co, value);
  return hipGetLastError();
}

hipError_t launch_probe_scatter(uint16_t* cells, uint64_t n_cells, uint64_t n_stores,
                                uint32_t seed, uint16_t value, int n_cu, hipStream_t st) {
  if (n_stores == 0) return hipSuccess;
  ProfScope ps(SPS_STAGE_PROBE, st, ProfScope::kKernel);
  launch_k(ps, k_probe_scatter, dim3(n_cu * 16), dim3(256), 0, st, cells, n_cells,
           n_stores, seed, value);
  return hipGetLastError();
}

hipError_t launch_probe_stream(const void* buf, uint64_t bytes, uint32_t* sum, int n_cu,
                               hipStream_t st) {
  ProfScope ps(SPS_STAGE_PROBE, st, ProfScope::kKernel);
  launch_k(ps, k_probe_stream, dim3(n_cu), dim3(256), 0, st,
           reinterpret_cast<const u32x4*>(buf), bytes / 16, sum);
  return hipGetLastError();
}

}  // namespace sps
