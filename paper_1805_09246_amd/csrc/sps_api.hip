// sps_api.hip -- host runtime behind the C ABI of include/sps.h.
//
// A sketch is one device block: [scan counters | info words | SRE array | SLE array |
// hot bitmap | HSE lists | candidates | kept hosts | ordered results | sort keys].  The SRE and SLE
// arrays are contiguous, so reset and merge treat them as one flat u16 range.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <stddef.h>
#include <string.h>
#include <time.h>

#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "sps_internal.h"

using sps::Ctrl;
using sps::Dev;

struct sps_sketch {
  sps_params p;
  Dev dev;
  sps::MlpRef mlp;
  void* base;
  bool owns;
  size_t bytes;
  uint16_t* state;        // == dev.sre; SRE then SLE array, contiguous
  uint64_t state_bytes;   // bytes of SRE + SLE arrays (incl. padding)
  uint64_t sre_bytes;     // bytes of the SRE array (dense)
  uint64_t row_bytes;     // bytes of one dense SLE row in a dump
  uint32_t* d_info;       // SPS_INFO_WORDS u32
  sps_result* d_sorted;   // cand_cap results (synchronous scan target)
  uint32_t* h_info;       // pinned SPS_INFO_WORDS u32
  uint32_t cur;
  int device;
  int n_cu;
  sps_tuning tune;
  bool hist_valid;        // dev.hist matches the SLE array (sliding mode; see k_ingest)
};

namespace {

thread_local char g_hip_detail[256] = "";

int hip_fail(hipError_t e, const char* where) {
  snprintf(g_hip_detail, sizeof(g_hip_detail), "%s: %s", where, hipGetErrorString(e));
  return SPS_EHIP;
}

#define SPS_HIP(call)                              \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

bool is_pow2(uint64_t v) { return v != 0 && (v & (v - 1)) == 0; }
uint32_t log2u(uint64_t v) {
  uint32_t n = 0;
  while ((1ull << n) < v) ++n;
  return n;
}
uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

uint32_t effective_cand_cap(const sps_params* p) { return p->cand_cap ? p->cand_cap : (1u << 18); }

int validate(const sps_params* p) {
  if (!p) return SPS_EINVAL;
  if (p->q < 6 || p->q > 24 || p->r < 3 || p->r > (uint32_t)sps::kMaxR) return SPS_EINVAL;
  if (p->delta < 1 || p->delta > 5 || p->delta >= p->q) return SPS_EINVAL;
  if ((uint64_t)(p->r - 2) * p->delta + p->q < 32) return SPS_EINVAL;  // every bit recovered
  if ((uint64_t)(p->r - 2) * p->delta > 31) return SPS_EINVAL;
  if (!(p->eta == 8 || p->eta == 16 || p->eta == 32 || p->eta == 64)) return SPS_EINVAL;
  if (p->qp < 1 || p->qp > 26 || p->rp < 1 || p->rp > (uint32_t)sps::kMaxRP) return SPS_EINVAL;
  if (!is_pow2(p->etap) || p->etap < 16 || p->etap > 65536) return SPS_EINVAL;
  if (!is_pow2(p->deltap) || p->deltap > p->etap) return SPS_EINVAL;
  if (p->qp + log2u(p->deltap) > 31) return SPS_EINVAL;  // row live counts fit u32
  if (p->theta < 1 || p->anet_side > 1) return SPS_EINVAL;
  if (effective_cand_cap(p) > (1u << 26)) return SPS_EINVAL;
  if (p->mode > SPS_MODE_DISCRETE) return SPS_EINVAL;
  if (p->row_counts > 1 || (p->row_counts && p->mode != SPS_MODE_SLIDING)) return SPS_EINVAL;
  return SPS_OK;
}

// Sampling depth, Eq. 1 in integer form: smallest t with eta * 2^t >= theta.
uint32_t sampling_depth(uint32_t theta, uint32_t eta) {
  uint32_t t = 0;
  while (((uint64_t)eta << t) < theta) ++t;
  return t;
}

// Hot cut of Sec. 3.2: weight >= rho * eta with rho = 0.99 (1 - e^(-1/3)).
uint32_t hot_cut_of(uint32_t eta) {
  const double rho = 0.99 * (1.0 - exp(-1.0 / 3.0));
  return (uint32_t)ceil(rho * (double)eta);
}

// SplitMix64 step; seed j of the sketch is the low word of output j.
uint64_t splitmix64_next(uint64_t& st) {
  st += 0x9E3779B97F4A7C15ull;
  uint64_t z = st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Layout {
  uint64_t ctrl, info, sre, slea, hot, hot_t, hse, cand, kept, wkept, sorted, skeys, part,
      hist, total;
  uint64_t row_len, row_stride, sre_bytes, slea_bytes;
};

Layout layout_of(const sps_params* p) {
  Layout L{};
  const uint64_t cap = effective_cand_cap(p);
  L.row_len = ((uint64_t)1 << p->qp) * p->deltap + p->etap - p->deltap;
  const uint64_t sre_cells = ((uint64_t)p->r << p->q) * p->eta;
  if (p->mode == SPS_MODE_DISCRETE) {
    // bits; a row ends with at least one spare word so 32-bit windows never cross it
    L.row_stride = round_up(L.row_len + 32, 1024);
    L.sre_bytes = sre_cells / 8;
    L.slea_bytes = (uint64_t)p->rp * L.row_stride / 8;
  } else {
    L.row_stride = round_up(L.row_len, 128);  // 256-byte rows, whole u16x8 vectors
    L.sre_bytes = sre_cells * 2;
    L.slea_bytes = (uint64_t)p->rp * L.row_stride * 2;
  }
  uint64_t o = 0;
  L.ctrl = o;   o += sizeof(Ctrl);
  L.info = o;   o += 256;
  L.sre = o;    o += round_up(L.sre_bytes, 256);
  L.slea = o;   o += round_up(L.slea_bytes, 256);
  L.hot = o;    o += round_up(((uint64_t)p->r << p->q) / 8, 256);
  L.hot_t = o;  o += round_up(((uint64_t)p->r << p->q) / 8, 256);
  L.hse = o;    o += round_up(((uint64_t)2 << p->q) * 4, 256);
  L.cand = o;   o += round_up(cap * 4, 256);
  L.kept = o;   o += round_up((uint64_t)sps::kEstWaves * sps::kept_region((uint32_t)cap) *
                                sizeof(sps_result), 256);
  L.wkept = o;  o += sps::kEstWaves * 4;
  L.sorted = o; o += round_up(cap * sizeof(sps_result), 256);
  L.skeys = o;  o += round_up(cap * 8, 256);
  L.part = o;   o += (uint64_t)sps::kMaxRP * sps::kRowsPartWaves * 4;
  L.hist = o;   o += p->row_counts ? (uint64_t)p->rp * sps::kHistBins * 4 : 0;
  L.total = o;
  return L;
}

bool same_shape(const sps_params& a, const sps_params& b) {
  return a.q == b.q && a.r == b.r && a.delta == b.delta && a.eta == b.eta && a.qp == b.qp &&
         a.rp == b.rp && a.etap == b.etap && a.deltap == b.deltap && a.theta == b.theta &&
         a.anet_side == b.anet_side && a.seed == b.seed && a.mode == b.mode;
}

int check_slice(const sps_sketch* s, uint32_t slice) {
  if (slice < 1 || slice > 65534u || slice < s->cur) return SPS_ESLICE;
  return SPS_OK;
}

// 64-byte dump header: the parameter fields up to and including `mode` (the sketch's
// shape; row_counts is a property of the live sketch, not of its state)
constexpr size_t kHeaderParams = offsetof(sps_params, mode) + sizeof(uint32_t);
struct Header {
  char magic[4];
  uint32_t cur;
  uint8_t params[kHeaderParams];
};
static_assert(sizeof(Header) == 64, "dump header is 64 bytes");

// ---- stage timing ----------------------------------------------------------------------
std::atomic<uint32_t> g_prof_mask{0};
std::mutex g_prof_mu;
struct ProfRec {
  int stage;
  hipEvent_t a, b;
};
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_free;

hipEvent_t prof_event() {
  hipEvent_t e = nullptr;
  if (!g_prof_free.empty()) {
    e = g_prof_free.back();
    g_prof_free.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

int device_cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

// ---- tuning cache ----------------------------------------------------------------------
// Key: architecture name and (q, r, delta, eta, q', r', eta', delta', mode, batched).
struct TuneEntry {
  char arch[64];
  uint32_t k[10];
  sps_tuning t;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;
constexpr const char* kTuneLineFmt =
    "{\"arch\": \"%s\", \"q\": %u, \"r\": %u, \"delta\": %u, \"eta\": %u, \"qp\": %u, "
    "\"rp\": %u, \"etap\": %u, \"deltap\": %u, \"mode\": %u, \"batched\": %u, "
    "\"blocks_per_cu\": %u, \"batch_tile\": %u, \"host_classes\": %u}";
constexpr const char* kTuneLineScan =
    "{\"arch\": \"%63[^\"]\", \"q\": %u, \"r\": %u, \"delta\": %u, \"eta\": %u, "
    "\"qp\": %u, \"rp\": %u, \"etap\": %u, \"deltap\": %u, \"mode\": %u, \"batched\": %u, "
    "\"blocks_per_cu\": %u, \"batch_tile\": %u, \"host_classes\": %u}%n";

void tune_key(const sps_params& p, bool batched, uint32_t* k) {
  const uint32_t v[10] = {p.q, p.r, p.delta, p.eta, p.qp, p.rp, p.etap, p.deltap, p.mode,
                          batched ? 1u : 0u};
  memcpy(k, v, sizeof(v));
}

bool tune_key_equal(const TuneEntry& e, const char* arch, const sps_params& p, bool batched) {
  uint32_t k[10];
  tune_key(p, batched, k);
  return strcmp(e.arch, arch) == 0 && memcmp(e.k, k, sizeof(k)) == 0;
}

void tune_cache_put(const char* arch, const sps_params& p, bool batched, const sps_tuning& t) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (TuneEntry& e : g_tune) {
    if (tune_key_equal(e, arch, p, batched)) {
      e.t = t;
      return;
    }
  }
  TuneEntry e{};
  snprintf(e.arch, sizeof(e.arch), "%s", arch);
  tune_key(p, batched, e.k);
  e.t = t;
  g_tune.push_back(e);
}

// Architecture name of a device without feature suffixes ("gfx950").
int device_arch(int dev, char* out) {
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  size_t n = 0;
  while (n < 63 && prop.gcnArchName[n] && prop.gcnArchName[n] != ':') {
    out[n] = prop.gcnArchName[n];
    ++n;
  }
  out[n] = 0;
  return SPS_OK;
}

}  // namespace

namespace sps {
ProfScope::ProfScope(int stage, hipStream_t st, Kind kind)
    : stage_(stage), st_(st), kind_(kind), ev0_(nullptr), ev1_(nullptr) {
  if (!((g_prof_mask.load(std::memory_order_relaxed) >> stage) & 1u)) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t a = prof_event();
  if (!a) return;
  if (kind == kKernel) {
    hipEvent_t b = prof_event();
    if (!b) {
      g_prof_free.push_back(a);
      return;
    }
    ev0_ = a;
    ev1_ = b;
  } else if (hipEventRecord(a, st) == hipSuccess) {
    ev0_ = a;
  } else {
    g_prof_free.push_back(a);
  }
}
ProfScope::~ProfScope() {
  if (!ev0_) return;
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t a = static_cast<hipEvent_t>(ev0_);
  hipEvent_t b = static_cast<hipEvent_t>(ev1_);
  if (kind_ == kMarkers) {
    b = prof_event();
    if (!b || hipEventRecord(b, st_) != hipSuccess) {
      if (b) g_prof_free.push_back(b);
      g_prof_free.push_back(a);
      return;
    }
  }
  g_prof_recs.push_back({stage_, a, b});
}
}  // namespace sps

extern "C" {

int sps_profile_enable(uint32_t stage_mask) {
  g_prof_mask.store(stage_mask);
  return SPS_OK;
}

int sps_profile_read(double* h_ms, uint32_t* h_launches, int nstages) {
  if (!h_ms || !h_launches || nstages < 0) return SPS_EINVAL;
  for (int i = 0; i < nstages; ++i) {
    h_ms[i] = 0.0;
    h_launches[i] = 0;
  }
  std::lock_guard<std::mutex> g(g_prof_mu);
  int rc = SPS_OK;
  for (const ProfRec& r : g_prof_recs) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) rc = hip_fail(e, "sps_profile_read");
    if (r.stage < nstages) {
      h_ms[r.stage] += t;
      h_launches[r.stage] += 1;
    }
    g_prof_free.push_back(r.a);
    g_prof_free.push_back(r.b);
  }
  g_prof_recs.clear();
  return rc;
}

int sps_probe_scatter(uint16_t* d_cells, uint64_t cells, uint64_t n_stores, uint32_t seed,
                      uint16_t value, void* stream) {
  if (!d_cells || cells == 0) return SPS_EINVAL;
  SPS_HIP(sps::launch_probe_scatter(d_cells, cells, n_stores, seed, value, device_cu_count(),
                                    (hipStream_t)stream));
  return SPS_OK;
}

int sps_probe_stream(const void* d_buf, uint64_t bytes, uint32_t* d_sum, void* stream) {
  if (!d_buf || !d_sum || (bytes & 15u)) return SPS_EINVAL;
  SPS_HIP(sps::launch_probe_stream(d_buf, bytes, d_sum, device_cu_count(), (hipStream_t)stream));
  return SPS_OK;
}

int sps_probe_replay_record(const sps_sketch* s, const sps_pkt* d_pkts, size_t n,
                            uint32_t* d_cells, size_t cap, uint64_t* h_class_off, void* stream) {
  if (!s || !h_class_off || (n && !d_pkts) || (cap && !d_cells)) return SPS_EINVAL;
  if (s->p.mode != SPS_MODE_SLIDING) return SPS_EINVAL;
  const uint64_t sle_off = (uint64_t)(s->dev.slea - s->dev.sre);
  if (sle_off + (uint64_t)s->dev.rp * s->dev.row_stride > 0xFFFFFFFFull) return SPS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* d_pos = nullptr;
  SPS_HIP(hipMalloc((void**)&d_pos, 8 * sizeof(unsigned long long)));
  unsigned long long pos[8] = {};
  int rc = SPS_OK;
  hipError_t e = hipMemcpyAsync(d_pos, pos, sizeof(pos), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = sps::launch_probe_record(s->dev, d_pkts, n, (uint32_t)sle_off, nullptr, d_pos, false, st);
  if (e == hipSuccess) e = hipMemcpyAsync(pos, d_pos, sizeof(pos), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    uint64_t acc = 0;
    for (int c = 0; c < 8; ++c) {
      h_class_off[c] = acc;
      acc += pos[c];
      pos[c] = h_class_off[c];
    }
    h_class_off[8] = acc;
    if (acc > cap) {
      rc = SPS_ECAPACITY;
    } else {
      e = hipMemcpyAsync(d_pos, pos, sizeof(pos), hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = sps::launch_probe_record(s->dev, d_pkts, n, (uint32_t)sle_off, d_cells, d_pos, true,
                                     st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
  }
  if (e != hipSuccess) rc = hip_fail(e, "sps_probe_replay_record");
  (void)hipFree(d_pos);
  return rc;
}

int sps_probe_replay(sps_sketch* s, const uint32_t* d_cells, const uint64_t* h_class_off,
                     uint16_t value, void* stream) {
  if (!s || !h_class_off || s->p.mode != SPS_MODE_SLIDING) return SPS_EINVAL;
  sps::ClassOffsets co{};
  for (int c = 0; c < 9; ++c) {
    co.off[c] = h_class_off[c];
    if (c && co.off[c] < co.off[c - 1]) return SPS_EINVAL;
  }
  if (co.off[8] && !d_cells) return SPS_EINVAL;
  SPS_HIP(sps::launch_probe_replay(s->state, d_cells, co, value,
                                   s->n_cu * (int)s->tune.blocks_per_cu, (hipStream_t)stream));
  s->hist_valid = false;  // plain stores: the histograms no longer follow the cells
  return SPS_OK;
}

const char* sps_strerror(int code) {
  switch (code) {
    case SPS_OK: return "ok";
    case SPS_EINVAL: return "invalid argument or unsupported sketch parameters";
    case SPS_ESLICE: return "slice out of order or out of range (1..65534, >= current slice)";
    case SPS_EMISMATCH: return "sketch parameters or seeds differ";
    case SPS_ENOMEM: return "out of device memory or caller block too small";
    case SPS_ECAPACITY: return "result or candidate buffer too small";
    case SPS_EHIP: return g_hip_detail[0] ? g_hip_detail : "HIP runtime error";
    case SPS_EBUDGET: return "device-memory budget exhausted";
    default: return "unknown error";
  }
}

int sps_sketch_bytes(const sps_params* p, size_t* bytes) {
  if (!bytes) return SPS_EINVAL;
  int rc = validate(p);
  if (rc) return rc;
  *bytes = (size_t)layout_of(p).total;
  return SPS_OK;
}

int sps_create(const sps_params* p, void* d_mem, size_t bytes, sps_sketch** out) {
  if (!out) return SPS_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  const Layout L = layout_of(p);
  if (d_mem && (bytes < L.total || ((uintptr_t)d_mem & 255u))) return SPS_ENOMEM;
  int device = 0, n_cu = 0;
  SPS_HIP(hipGetDevice(&device));
  SPS_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
  SPS_HIP(sps::prepare_join());
  sps_sketch* s = new (std::nothrow) sps_sketch();
  if (!s) return SPS_ENOMEM;
  s->p = *p;
  s->p.cand_cap = effective_cand_cap(p);
  s->device = device;
  s->n_cu = n_cu;
  if (d_mem) {
    s->base = d_mem;
    s->owns = false;
  } else {
    if (hipMalloc(&s->base, L.total) != hipSuccess) {
      delete s;
      return SPS_ENOMEM;
    }
    s->owns = true;
  }
  if (hipHostMalloc((void**)&s->h_info, 256, hipHostMallocDefault) != hipSuccess) {
    if (s->owns) (void)hipFree(s->base);
    delete s;
    return SPS_ENOMEM;
  }

  s->bytes = L.total;
  uint8_t* b = static_cast<uint8_t*>(s->base);
  Dev& d = s->dev;
  d.ctrl = reinterpret_cast<Ctrl*>(b + L.ctrl);
  d.sre = reinterpret_cast<uint16_t*>(b + L.sre);
  d.slea = reinterpret_cast<uint16_t*>(b + L.slea);
  d.hot = reinterpret_cast<uint32_t*>(b + L.hot);
  d.hot_t = reinterpret_cast<uint32_t*>(b + L.hot_t);
  d.hse = reinterpret_cast<uint32_t*>(b + L.hse);
  d.cand = reinterpret_cast<uint32_t*>(b + L.cand);
  d.kept = reinterpret_cast<sps_result*>(b + L.kept);
  d.wave_kept = reinterpret_cast<uint32_t*>(b + L.wkept);
  d.skeys = reinterpret_cast<uint64_t*>(b + L.skeys);
  d.rows_part = reinterpret_cast<uint32_t*>(b + L.part);
  d.hist = p->row_counts ? reinterpret_cast<uint32_t*>(b + L.hist) : nullptr;
  s->d_info = reinterpret_cast<uint32_t*>(b + L.info);
  s->d_sorted = reinterpret_cast<sps_result*>(b + L.sorted);
  d.row_len = L.row_len;
  d.row_stride = L.row_stride;
  d.q = p->q;
  d.r = p->r;
  d.delta = p->delta;
  d.eta = p->eta;
  d.qp = p->qp;
  d.rp = p->rp;
  d.etap = p->etap;
  d.deltap = p->deltap;
  const uint32_t tau = sampling_depth(p->theta, p->eta);
  d.tau_mask = tau >= 32 ? 0xFFFFFFFFu : ((1u << tau) - 1u);
  d.hot_cut = hot_cut_of(p->eta);
  d.anet_side = p->anet_side;
  d.cand_cap = s->p.cand_cap;
  d.mode = p->mode;
  uint64_t st = p->seed;
  d.seed_h1 = (uint32_t)splitmix64_next(st);
  d.seed_h2 = (uint32_t)splitmix64_next(st);
  d.seed_h3 = (uint32_t)splitmix64_next(st);
  d.seed_rhfg0 = (uint32_t)splitmix64_next(st);
  for (int i = 0; i < sps::kMaxRP; ++i) d.seed_lh[i] = (uint32_t)splitmix64_next(st);
  s->state = d.sre;
  s->sre_bytes = L.sre_bytes;
  s->state_bytes = (L.slea - L.sre) + L.slea_bytes;
  s->row_bytes = p->mode == SPS_MODE_DISCRETE ? (L.row_len + 31) / 32 * 4 : L.row_len * 2;
  s->cur = 0;
  s->mlp.w = nullptr;
  s->tune.blocks_per_cu = 16;
  s->tune.batch_tile = 4096;
  s->tune.host_classes = 8;
  s->tune.scan_overlap = 1;
  s->hist_valid = p->row_counts != 0;  // all zero, like the state
  // zero state and workspace once, synchronously
  hipError_t e = hipMemset(s->base, 0, L.total);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)sps_destroy(s);
    return hip_fail(e, "sps_create");
  }
  *out = s;
  return SPS_OK;
}

int sps_destroy(sps_sketch* s) {
  if (!s) return SPS_EINVAL;
  (void)hipDeviceSynchronize();
  if (s->owns) (void)hipFree(s->base);
  (void)hipHostFree(s->h_info);

  delete s;
  return SPS_OK;
}

namespace {
uint64_t hist_bytes(const sps_sketch* s) { return (uint64_t)s->dev.rp * sps::kHistBins * 4; }
}  // namespace

int sps_reset(sps_sketch* s, void* stream) {
  if (!s) return SPS_EINVAL;
  SPS_HIP(sps::launch_fill_zero(s->state, s->state_bytes, (hipStream_t)stream));
  if (s->p.row_counts) {
    SPS_HIP(sps::launch_fill_zero(s->dev.hist, hist_bytes(s), (hipStream_t)stream));
    s->hist_valid = true;
  }
  SPS_HIP(sps::launch_scan_reset(s->dev, true, (hipStream_t)stream));
  s->cur = 0;
  return SPS_OK;
}

int sps_ingest(sps_sketch* s, const sps_pkt* d_pkts, size_t n, uint32_t slice, void* stream) {
  if (!s || (n && !d_pkts)) return SPS_EINVAL;
  int rc = check_slice(s, slice);
  if (rc) return rc;
  SPS_HIP(sps::launch_ingest(s->dev, d_pkts, n, (uint16_t)slice,
                             s->n_cu * (int)s->tune.blocks_per_cu, 256, s->tune.host_classes,
                             s->hist_valid, (hipStream_t)stream));
  s->cur = slice;
  return SPS_OK;
}

namespace {
// Validate a batch and launch it with the given shape (64 routers per launch).
int ingest_batched_with(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                        uint32_t m, uint32_t slice, hipStream_t st, const sps_tuning& t) {
  const uint32_t tile = t.batch_tile;
  for (uint32_t b = 0; b < m; b += sps::kMaxBatch) {
    const uint32_t k = m - b < (uint32_t)sps::kMaxBatch ? m - b : (uint32_t)sps::kMaxBatch;
    sps::BatchTable tb{};
    uint64_t acc = 0;
    for (uint32_t j = 0; j < k; ++j) {
      tb.item[j].sre = h_s[b + j]->dev.sre;
      tb.item[j].slea = h_s[b + j]->dev.slea;
      tb.item[j].hist = h_s[b + j]->hist_valid ? h_s[b + j]->dev.hist : nullptr;
      tb.item[j].pkts = h_pkts[b + j];
      tb.item[j].n = h_n[b + j];
      tb.tile_start[j] = acc;
      acc += (h_n[b + j] + tile - 1) / tile;
    }
    tb.tile_start[k] = acc;
    SPS_HIP(sps::launch_ingest_batched(h_s[0]->dev, tb, k, tile, (uint16_t)slice,
                                       h_s[0]->n_cu * (int)t.blocks_per_cu, 256, t.host_classes,
                                       st));
  }
  return SPS_OK;
}

int check_batch(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                uint32_t m, uint32_t slice) {
  if (!h_s || !h_pkts || !h_n || m == 0) return SPS_EINVAL;
  for (uint32_t j = 0; j < m; ++j) {
    if (!h_s[j] || (h_n[j] && !h_pkts[j])) return SPS_EINVAL;
    if (!same_shape(h_s[j]->p, h_s[0]->p)) return SPS_EMISMATCH;
    int rc = check_slice(h_s[j], slice);
    if (rc) return rc;
  }
  return SPS_OK;
}
}  // namespace

int sps_ingest_batched(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                       uint32_t m, uint32_t slice, void* stream) {
  int rc = check_batch(h_s, h_pkts, h_n, m, slice);
  if (rc) return rc;
  rc = ingest_batched_with(h_s, h_pkts, h_n, m, slice, (hipStream_t)stream, h_s[0]->tune);
  if (rc) return rc;
  for (uint32_t j = 0; j < m; ++j) h_s[j]->cur = slice;
  return SPS_OK;
}

int sps_get_tuning(const sps_sketch* s, sps_tuning* out) {
  if (!s || !out) return SPS_EINVAL;
  *out = s->tune;
  return SPS_OK;
}

int sps_set_tuning(sps_sketch* s, const sps_tuning* t) {
  if (!s || !t) return SPS_EINVAL;
  if (t->blocks_per_cu > 256 || (t->batch_tile && (t->batch_tile < 64 || t->batch_tile > (1u << 24))))
    return SPS_EINVAL;
  if (t->host_classes > 8 || (t->host_classes & (t->host_classes - 1u))) return SPS_EINVAL;
  if (t->scan_overlap > 2) return SPS_EINVAL;
  if (t->scan_overlap) s->tune.scan_overlap = t->scan_overlap;
  if (t->blocks_per_cu) s->tune.blocks_per_cu = t->blocks_per_cu;
  if (t->batch_tile) s->tune.batch_tile = t->batch_tile;
  if (t->host_classes) s->tune.host_classes = t->host_classes;
  return SPS_OK;
}

int sps_autotune_ingest(sps_sketch* const* h_s, const sps_pkt* const* h_pkts, const size_t* h_n,
                        uint32_t m, uint32_t slice, void* stream, sps_tuning* best,
                        float* h_ms, uint32_t h_ms_cap) {
  int rc = check_batch(h_s, h_pkts, h_n, m, slice);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  static const uint32_t kBlocks[] = {2, 4, 8, 16, 32, 64};
  static const uint32_t kTiles[] = {512, 2048, 8192, 32768};
  static const uint32_t kClasses[] = {1, 8};
  std::vector<sps_tuning> cands;
  for (uint32_t b : kBlocks) {
    for (uint32_t c : kClasses) {
      if (m == 1) {
        cands.push_back({b, h_s[0]->tune.batch_tile, c, h_s[0]->tune.scan_overlap});
      } else {
        for (uint32_t t : kTiles) cands.push_back({b, t, c, h_s[0]->tune.scan_overlap});
      }
    }
  }
  hipEvent_t e0, e1;
  SPS_HIP(hipEventCreate(&e0));
  SPS_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  sps_tuning pick = h_s[0]->tune;
  uint32_t idx = 0;
  for (int rep = 0; rep < 2; ++rep) {  // first pass warms caches, second pass is timed
    for (const sps_tuning& c : cands) {
      SPS_HIP(hipEventRecord(e0, st));
      if (m == 1) {
        SPS_HIP(sps::launch_ingest(h_s[0]->dev, h_pkts[0], h_n[0], (uint16_t)slice,
                                   h_s[0]->n_cu * (int)c.blocks_per_cu, 256, c.host_classes,
                                   h_s[0]->hist_valid, st));
      } else {
        rc = ingest_batched_with(h_s, h_pkts, h_n, m, slice, st, c);
        if (rc) return rc;
      }
      SPS_HIP(hipEventRecord(e1, st));
      SPS_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SPS_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1) {
        if (h_ms && idx < h_ms_cap) h_ms[idx] = ms;
        ++idx;
        if (ms < best_ms) {
          best_ms = ms;
          pick = c;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (uint32_t j = 0; j < m; ++j) {
    h_s[j]->tune = pick;
    h_s[j]->cur = slice;
  }
  if (best) *best = pick;
  char arch[64];
  if (device_arch(h_s[0]->device, arch) == SPS_OK) tune_cache_put(arch, h_s[0]->p, m > 1, pick);
  return SPS_OK;
}

int sps_tuning_lookup(const char* arch, const sps_params* p, uint32_t batched, sps_tuning* out,
                      int* found) {
  if (!p || !out || !found) return SPS_EINVAL;
  *found = 0;
  char cur[64];
  if (!arch) {
    int dev = 0;
    SPS_HIP(hipGetDevice(&dev));
    int rc = device_arch(dev, cur);
    if (rc) return rc;
    arch = cur;
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const TuneEntry& e : g_tune) {
    if (tune_key_equal(e, arch, *p, batched != 0)) {
      *out = e.t;
      *found = 1;
      break;
    }
  }
  return SPS_OK;
}

int sps_tuning_cache_save(const char* path) {
  if (!path) return SPS_EINVAL;
  FILE* f = fopen(path, "w");
  if (!f) return SPS_EINVAL;
  std::lock_guard<std::mutex> g(g_tune_mu);
  fprintf(f, "{\"sps_tuning_cache\": 1, \"entries\": [\n");
  for (size_t i = 0; i < g_tune.size(); ++i) {
    const TuneEntry& e = g_tune[i];
    fprintf(f, kTuneLineFmt, e.arch, e.k[0], e.k[1], e.k[2], e.k[3], e.k[4], e.k[5], e.k[6],
            e.k[7], e.k[8], e.k[9], e.t.blocks_per_cu, e.t.batch_tile, e.t.host_classes);
    fprintf(f, "%s\n", i + 1 < g_tune.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  const bool ok = fclose(f) == 0;
  return ok ? SPS_OK : SPS_EINVAL;
}

int sps_tuning_cache_load(const char* path) {
  if (!path) return SPS_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return SPS_EINVAL;
  std::vector<TuneEntry> got;
  char line[512];
  bool header = false, bad = false;
  while (fgets(line, sizeof(line), f)) {
    if (strstr(line, "\"sps_tuning_cache\": 1")) {
      header = true;
      continue;
    }
    const char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p != '{') continue;  // closing bracket and blank lines
    TuneEntry e{};
    int used = 0;
    const int n = sscanf(p, kTuneLineScan, e.arch, &e.k[0], &e.k[1], &e.k[2], &e.k[3], &e.k[4],
                         &e.k[5], &e.k[6], &e.k[7], &e.k[8], &e.k[9], &e.t.blocks_per_cu,
                         &e.t.batch_tile, &e.t.host_classes, &used);
    if (n != 14 || used == 0 || e.t.blocks_per_cu == 0 || e.t.blocks_per_cu > 256 ||
        e.t.batch_tile < 64 || e.t.host_classes == 0 || e.t.host_classes > 8 ||
        (e.t.host_classes & (e.t.host_classes - 1u)) || e.k[9] > 1) {
      bad = true;
      break;
    }
    got.push_back(e);
  }
  fclose(f);
  if (!header || bad) return SPS_EINVAL;
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const TuneEntry& e : got) {
    bool replaced = false;
    for (TuneEntry& x : g_tune) {
      if (strcmp(x.arch, e.arch) == 0 && memcmp(x.k, e.k, sizeof(e.k)) == 0) {
        x.t = e.t;
        replaced = true;
      }
    }
    if (!replaced) g_tune.push_back(e);
  }
  return SPS_OK;
}

int sps_tuning_cache_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  return SPS_OK;
}

struct sps_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int sps_graph_begin(void* stream) {
  SPS_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  return SPS_OK;
}

int sps_graph_end(void* stream, sps_graph** out) {
  if (!out) return SPS_EINVAL;
  *out = nullptr;
  hipGraph_t g = nullptr;
  SPS_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
  hipGraphExec_t e = nullptr;
  hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(err, "hipGraphInstantiate");
  }
  sps_graph* r = new (std::nothrow) sps_graph{g, e};
  if (!r) {
    (void)hipGraphExecDestroy(e);
    (void)hipGraphDestroy(g);
    return SPS_ENOMEM;
  }
  *out = r;
  return SPS_OK;
}

int sps_graph_end_update(void* stream, sps_graph* g, int* updated) {
  if (!g) return SPS_EINVAL;
  if (updated) *updated = 0;
  hipGraph_t ng = nullptr;
  SPS_HIP(hipStreamEndCapture((hipStream_t)stream, &ng));
  hipGraphExecUpdateResult res = hipGraphExecUpdateError;
  hipGraphNode_t bad = nullptr;
  hipError_t err = hipGraphExecUpdate(g->exec, ng, &bad, &res);
  if (err == hipSuccess && res == hipGraphExecUpdateSuccess) {
    (void)hipGraphDestroy(g->graph);
    g->graph = ng;
    if (updated) *updated = 1;
    return SPS_OK;
  }
  (void)hipGetLastError();  // a refused update leaves an error behind; the graph is rebuilt
  hipGraphExec_t e = nullptr;
  err = hipGraphInstantiate(&e, ng, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    (void)hipGraphDestroy(ng);
    return hip_fail(err, "hipGraphInstantiate");
  }
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  g->graph = ng;
  g->exec = e;
  return SPS_OK;
}

namespace {
// Host function run by the stream: stores the host's CLOCK_MONOTONIC time in seconds.
void store_host_time(void* p) {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  *static_cast<volatile double*>(p) = (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}
}  // namespace

int sps_stream_host_time(double* h_time, void* stream) {
  if (!h_time) return SPS_EINVAL;
  SPS_HIP(hipLaunchHostFunc((hipStream_t)stream, store_host_time, h_time));
  return SPS_OK;
}

int sps_graph_launch(sps_graph* g, void* stream) {
  if (!g) return SPS_EINVAL;
  SPS_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return SPS_OK;
}

int sps_graph_destroy(sps_graph* g) {
  if (!g) return SPS_EINVAL;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return SPS_OK;
}

int sps_advance(sps_sketch* s, uint32_t slice) {
  if (!s) return SPS_EINVAL;
  int rc = check_slice(s, slice);
  if (rc) return rc;
  s->cur = slice;
  return SPS_OK;
}

int sps_rebase(sps_sketch* s, uint32_t offset, void* stream) {
  if (!s) return SPS_EINVAL;
  if (offset > s->cur) return SPS_ESLICE;
  if (s->p.mode == SPS_MODE_SLIDING) {
    SPS_HIP(sps::launch_rebase(s->state, s->state_bytes, offset, (hipStream_t)stream));
    if (s->hist_valid)
      SPS_HIP(sps::launch_hist_rebase(s->dev.hist, s->dev.rp, offset, (hipStream_t)stream));
  }
  s->cur -= offset;
  return SPS_OK;
}

int sps_merge(sps_sketch* dst, const sps_sketch* const* h_src, uint32_t nsrc, void* stream) {
  if (!dst || (nsrc && !h_src)) return SPS_EINVAL;
  const uint16_t* srcs[256];
  if (nsrc > 256) return SPS_EINVAL;
  uint32_t cur = dst->cur;
  for (uint32_t j = 0; j < nsrc; ++j) {
    if (!h_src[j]) return SPS_EINVAL;
    if (!same_shape(dst->p, h_src[j]->p)) return SPS_EMISMATCH;
    srcs[j] = h_src[j]->state;
    if (h_src[j]->cur > cur) cur = h_src[j]->cur;
  }
  bool other = false;
  for (uint32_t j = 0; j < nsrc; ++j) other = other || h_src[j] != dst;
  if (nsrc)
    SPS_HIP(sps::launch_merge(dst->state, srcs, nsrc, dst->state_bytes,
                              dst->p.mode == SPS_MODE_DISCRETE, (hipStream_t)stream));
  if (other) dst->hist_valid = false;  // merged cells are not counted; scans sweep instead
  dst->cur = cur;
  return SPS_OK;
}

int sps_scan_async(sps_sketch* s, uint32_t window, double threshold, sps_result* d_out,
                   size_t cap, uint32_t* d_info, void* stream) {
  if (!s || !d_info || (cap && !d_out)) return SPS_EINVAL;
  if (window < 1 || window > 65534u) return SPS_EINVAL;
  if (s->p.mode == SPS_MODE_DISCRETE && window != 1) return SPS_EINVAL;
  if (cap > 0xFFFFFFFFull) cap = 0xFFFFFFFFull;
  SPS_HIP(sps::launch_scan(s->dev, s->cur, window, threshold, d_out, (uint32_t)cap, d_info,
                           s->mlp, s->hist_valid, s->tune.scan_overlap, s->n_cu,
                           (hipStream_t)stream));
  return SPS_OK;
}

int sps_scan(sps_sketch* s, uint32_t window, double threshold, sps_result* h_out, size_t cap,
             size_t* n_out, void* stream) {
  if (!s || !n_out || (cap && !h_out)) return SPS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = sps_scan_async(s, window, threshold, s->d_sorted, s->p.cand_cap, s->d_info, stream);
  if (rc) return rc;
  SPS_HIP(hipMemcpyAsync(s->h_info, s->d_info, SPS_INFO_WORDS * 4, hipMemcpyDeviceToHost, st));
  SPS_HIP(hipStreamSynchronize(st));
  const uint32_t kept = s->h_info[SPS_INFO_KEPT];
  if (s->h_info[SPS_INFO_FLAGS] & 1u) {
    *n_out = 0;
    return SPS_ECAPACITY;
  }
  *n_out = kept;
  if (kept > cap) return SPS_ECAPACITY;
  if (kept) {
    SPS_HIP(hipMemcpyAsync(h_out, s->d_sorted, (size_t)kept * sizeof(sps_result),
                           hipMemcpyDeviceToHost, st));
    SPS_HIP(hipStreamSynchronize(st));
  }
  return SPS_OK;
}

int sps_features(const sps_sketch* s, const uint32_t* d_hosts, size_t n, uint32_t window,
                 uint32_t* d_x, void* stream) {
  if (!s || (n && (!d_hosts || !d_x))) return SPS_EINVAL;
  if (window < 1 || window > 32 || s->p.mode == SPS_MODE_DISCRETE) return SPS_EINVAL;
  SPS_HIP(sps::launch_features(s->dev, s->cur, window, d_hosts, n, d_x, s->n_cu,
                               (hipStream_t)stream));
  return SPS_OK;
}

int sps_estimate_hosts(sps_sketch* s, const uint32_t* d_hosts, size_t n, uint32_t window,
                       sps_result* d_out, void* stream) {
  if (!s || (n && (!d_hosts || !d_out))) return SPS_EINVAL;
  if (window < 1 || window > 65534u || n > 0xFFFFFFFFull) return SPS_EINVAL;
  if (s->p.mode == SPS_MODE_DISCRETE && window != 1) return SPS_EINVAL;
  SPS_HIP(sps::launch_estimate_hosts(s->dev, s->cur, window, d_hosts, (uint32_t)n, d_out, s->mlp,
                                     s->hist_valid, s->n_cu, (hipStream_t)stream));
  return SPS_OK;
}

int sps_attach_mlp(sps_sketch* s, const float* d_weights, const float* h_feat_lo,
                   const float* h_feat_hi, uint32_t min_live, double max_card) {
  if (!s) return SPS_EINVAL;
  if (!d_weights) {
    s->mlp.w = nullptr;
    return SPS_OK;
  }
  if (!h_feat_lo || !h_feat_hi || !(max_card > 1.0)) return SPS_EINVAL;
  s->mlp.w = d_weights;
  for (int i = 0; i < SPS_MLP_IN; ++i) {
    s->mlp.lo[i] = h_feat_lo[i];
    s->mlp.hi[i] = h_feat_hi[i];
  }
  s->mlp.log_max = (float)log(max_card);
  s->mlp.min_live = min_live;
  return SPS_OK;
}

int sps_mlp_work_bytes(size_t n, size_t* bytes) {
  if (!bytes || n == 0 || n > 0xFFFFFFFFull) return SPS_EINVAL;
  const uint64_t w = sps::mlp_grad_waves((uint32_t)n);
  *bytes = (size_t)(w * SPS_MLP_PARAMS * 4 + w * 4);
  return SPS_OK;
}

int sps_mlp_grad(const float* d_w, const uint32_t* d_feat, const float* d_target,
                 const uint32_t* d_idx, size_t n, uint32_t etap, void* d_work, float* d_grad,
                 float* d_loss, void* stream) {
  if (!d_w || !d_feat || !d_target || !d_work || !d_grad || n == 0 || n > 0xFFFFFFFFull ||
      etap == 0)
    return SPS_EINVAL;
  const uint64_t w = sps::mlp_grad_waves((uint32_t)n);
  float* partial = static_cast<float*>(d_work);
  float* partial_loss = partial + w * SPS_MLP_PARAMS;
  SPS_HIP(sps::launch_mlp_grad(d_w, d_feat, d_target, d_idx, (uint32_t)n, etap, partial,
                               partial_loss, d_grad, d_loss, (hipStream_t)stream));
  return SPS_OK;
}

int sps_mlp_grad_noalloc(const float* d_w, const uint32_t* d_feat, const float* d_target,
                         const uint32_t* d_idx, size_t n, uint32_t etap, float* d_grad,
                         float* d_loss, void* stream) {
  if (!d_w || !d_feat || !d_target || !d_grad || n == 0 || etap == 0) return SPS_EINVAL;
  if (n > SPS_MLP_NOALLOC_MAX_N) return SPS_ECAPACITY;
  float* scratch = nullptr;
  uint64_t floats = 0;
  SPS_HIP(sps::mlp_scratch(&scratch, &floats));
  const uint64_t w = sps::mlp_grad_waves((uint32_t)n);
  if (w * (SPS_MLP_PARAMS + 1) > floats) return SPS_ECAPACITY;
  SPS_HIP(sps::launch_mlp_grad(d_w, d_feat, d_target, d_idx, (uint32_t)n, etap, scratch,
                               scratch + w * SPS_MLP_PARAMS, d_grad, d_loss,
                               (hipStream_t)stream));
  return SPS_OK;
}

int sps_mlp_adam(float* d_w, float* d_m, float* d_v, const float* d_grad, uint32_t step,
                 float lr, double beta1, double beta2, float eps, void* stream) {
  if (!d_w || !d_m || !d_v || !d_grad || step == 0) return SPS_EINVAL;
  SPS_HIP(sps::launch_mlp_adam(d_w, d_m, d_v, d_grad, step, lr, beta1, beta2, eps,
                               (hipStream_t)stream));
  return SPS_OK;
}

int sps_mlp_forward(const float* d_w, const uint32_t* d_feat, size_t n, uint32_t etap, int bf16,
                    float* d_y, void* stream) {
  if (!d_w || (n && (!d_feat || !d_y)) || n > 0xFFFFFFFFull || etap == 0) return SPS_EINVAL;
  SPS_HIP(sps::launch_mlp_forward(d_w, d_feat, (uint32_t)n, etap, bf16, d_y,
                                  device_cu_count(), (hipStream_t)stream));
  return SPS_OK;
}

int sps_state_bytes(const sps_sketch* s, size_t* bytes) {
  if (!s || !bytes) return SPS_EINVAL;
  const Dev& d = s->dev;
  *bytes = sizeof(Header) + (size_t)s->sre_bytes + (size_t)d.rp * s->row_bytes;
  return SPS_OK;
}

int sps_export(const sps_sketch* s, void* h_buf, size_t bytes, void* stream) {
  size_t need = 0;
  if (!h_buf) return SPS_EINVAL;
  int rc = sps_state_bytes(s, &need);
  if (rc) return rc;
  if (bytes < need) return SPS_ECAPACITY;
  hipStream_t st = (hipStream_t)stream;
  Header h{};
  memcpy(h.magic, "SPS1", 4);
  h.cur = s->cur;
  memcpy(h.params, &s->p, kHeaderParams);
  memcpy(h_buf, &h, sizeof(h));
  uint8_t* o = static_cast<uint8_t*>(h_buf) + sizeof(Header);
  const Dev& d = s->dev;
  SPS_HIP(hipStreamSynchronize(st));
  const size_t pitch = d.mode == SPS_MODE_DISCRETE ? (size_t)d.row_stride / 8
                                                   : (size_t)d.row_stride * 2;
  SPS_HIP(hipMemcpy(o, d.sre, (size_t)s->sre_bytes, hipMemcpyDeviceToHost));
  o += (size_t)s->sre_bytes;
  SPS_HIP(hipMemcpy2D(o, (size_t)s->row_bytes, d.slea, pitch, (size_t)s->row_bytes, d.rp,
                      hipMemcpyDeviceToHost));
  return SPS_OK;
}

int sps_import(sps_sketch* s, const void* h_buf, size_t bytes, void* stream) {
  size_t need = 0;
  if (!h_buf) return SPS_EINVAL;
  int rc = sps_state_bytes(s, &need);
  if (rc) return rc;
  if (bytes < need) return SPS_ECAPACITY;
  Header h;
  memcpy(&h, h_buf, sizeof(h));
  sps_params want = s->p;
  if (memcmp(h.magic, "SPS1", 4) != 0) return SPS_EINVAL;
  sps_params hp = want;
  memcpy(&hp, h.params, kHeaderParams);
  hp.cand_cap = want.cand_cap;
  if (!same_shape(hp, want) || h.cur > 65534u) return SPS_EMISMATCH;
  hipStream_t st = (hipStream_t)stream;
  const Dev& d = s->dev;
  const uint8_t* o = static_cast<const uint8_t*>(h_buf) + sizeof(Header);
  SPS_HIP(hipStreamSynchronize(st));
  const size_t pitch = d.mode == SPS_MODE_DISCRETE ? (size_t)d.row_stride / 8
                                                   : (size_t)d.row_stride * 2;
  SPS_HIP(hipMemcpy(d.sre, o, (size_t)s->sre_bytes, hipMemcpyHostToDevice));
  o += (size_t)s->sre_bytes;
  SPS_HIP(hipMemcpy2D(d.slea, pitch, o, (size_t)s->row_bytes, (size_t)s->row_bytes, d.rp,
                      hipMemcpyHostToDevice));
  s->cur = h.cur;
  s->hist_valid = false;  // imported cells are not counted; scans sweep instead
  return SPS_OK;
}

int sps_current_slice(const sps_sketch* s, uint32_t* slice) {
  if (!s || !slice) return SPS_EINVAL;
  *slice = s->cur;
  return SPS_OK;
}

int sps_derived(const sps_sketch* s, uint32_t* tau, uint32_t* hot_cut, uint64_t* row_len) {
  if (!s) return SPS_EINVAL;
  if (tau) *tau = (uint32_t)__builtin_popcount(s->dev.tau_mask);
  if (hot_cut) *hot_cut = s->dev.hot_cut;
  if (row_len) *row_len = s->dev.row_len;
  return SPS_OK;
}

int sps_debug_copy(const sps_sketch* s, int which, void* h_buf, size_t bytes, size_t* size,
                   void* stream) {
  if (!s || !size) return SPS_EINVAL;
  const Dev& d = s->dev;
  const void* src = nullptr;
  size_t full = 0;
  switch (which) {
    case 0: src = d.hot; full = ((size_t)d.r << d.q) / 8; break;
    case 1: {
      Ctrl c;
      SPS_HIP(hipStreamSynchronize((hipStream_t)stream));
      SPS_HIP(hipMemcpy(&c, d.ctrl, sizeof(c), hipMemcpyDeviceToHost));
      const uint32_t n = c.last_n_cand < d.cand_cap ? c.last_n_cand : d.cand_cap;
      src = d.cand;
      full = (size_t)n * 4;
      break;
    }
    case 2:
      src = reinterpret_cast<const uint8_t*>(d.ctrl) + offsetof(Ctrl, last_row_live);
      full = (size_t)d.rp * 4;
      break;
    case 3:  // stamp histograms, only while the ingest keeps them
      src = d.hist;
      full = s->hist_valid ? (size_t)hist_bytes(s) : 0;
      break;
    default: return SPS_EINVAL;
  }
  *size = full;
  if (h_buf && bytes) {
    SPS_HIP(hipStreamSynchronize((hipStream_t)stream));
    SPS_HIP(hipMemcpy(h_buf, src, bytes < full ? bytes : full, hipMemcpyDeviceToHost));
  }
  return SPS_OK;
}

int sps_sync(void* stream) {
  SPS_HIP(hipStreamSynchronize((hipStream_t)stream));
  SPS_HIP(hipGetLastError());
  return SPS_OK;
}

}  // extern "C"
