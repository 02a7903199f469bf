// synth_gen.hip -- GPU generator of planted hosts for the learned-estimator workload.
//
// Input generation only (no arithmetic of the sketch method).  Host j of a stream has
// card[j] distinct peers; peer i of host j is addr_mix(i + peer_salt[j]) (a bijection of i,
// so peers of one host are distinct).  Arrival law 0: every peer first appears in a slice f
// drawn uniformly from 1..window and appears again in each later slice with probability
// 0.3.  Law 1 (the scale workload's planted hosts): the peers are fresh in every slice and
// spread evenly, peer i appearing only in slice 1 + (i mod window).  Only its last
// appearance matters to a max-of-stamps sketch, so one packet (peer, host) is written per
// peer, into the bucket of its last slice.
//
// Randomness: rng(key, ctr) = SplitMix64 output number ctr + 1 from seed `key`
// (Steele, Lea, Flood 2014), i.e. mix64(key + (ctr + 1) * 0x9E3779B97F4A7C15).
// Peer g of the stream (g = prefix[j] + i) uses ctr = g * 16 for its first slice and
// ctr = g * 16 + s for slice s; integer comparisons only, so a CPU twin reproduces it bit
// for bit.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t rng(uint64_t key, uint64_t ctr) {
  return mix64(key + (ctr + 1) * 0x9E3779B97F4A7C15ull);
}

__device__ __forceinline__ uint32_t addr_mix(uint32_t v, uint32_t salt) {
  v ^= salt;
  v *= 0x2C1B3C6Du;
  v ^= v >> 12;
  v *= 0x297A2D39u;
  v ^= v >> 15;
  return v;
}

constexpr uint32_t kRepeat = 1288490189u;  // round(0.3 * 2^32)

__global__ void __launch_bounds__(256) k_gen_planted(
    const uint32_t* __restrict__ host, const uint64_t* __restrict__ prefix,
    const uint32_t* __restrict__ peer_salt, uint32_t m, uint64_t key, uint32_t window,
    uint32_t peer_domain_salt, uint32_t law, uint32_t* __restrict__ out, uint64_t cap,
    unsigned long long* __restrict__ counts) {
  const uint64_t total = prefix[m];
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t iters = (total + stride - 1) / stride;  // uniform trip count per wave
  for (uint64_t it = 0; it < iters; ++it) {
    const uint64_t g = start + it * stride;
    const bool active = g < total;
    uint32_t bucket = 0xFFFFFFFFu, src = 0, dst = 0;
    if (active) {
      uint32_t lo = 0, hi = m;  // prefix[lo] <= g < prefix[lo + 1]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid;
      }
      const uint32_t i = (uint32_t)(g - prefix[lo]);
      src = addr_mix(i + peer_salt[lo], peer_domain_salt);
      dst = host[lo];
      if (law == 1) {
        bucket = i % window;
      } else {
        const uint32_t u = (uint32_t)(rng(key, g * 16) >> 32);
        const uint32_t f = 1u + (uint32_t)(((uint64_t)u * window) >> 32);
        uint32_t last = f;
        for (uint32_t s = f + 1; s <= window; ++s)
          if ((uint32_t)(rng(key, g * 16 + s) >> 32) < kRepeat) last = s;
        bucket = last - 1;
      }
    }
    for (uint32_t b = 0; b < window; ++b) {
      const uint64_t mask = __ballot(bucket == b);
      if (mask == 0) continue;
      const uint32_t leader = (uint32_t)__ffsll((long long)mask) - 1;
      unsigned long long base = 0;
      if (__lane_id() == leader) base = atomicAdd(&counts[b], (unsigned long long)__popcll(mask));
      base = __shfl(base, (int)leader, 64);
      if (bucket == b) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const uint64_t pos = base + below;
        if (pos < cap) {
          out[(b * cap + pos) * 2] = src;
          out[(b * cap + pos) * 2 + 1] = dst;
        }
      }
    }
  }
}

}  // namespace

extern "C" int synth_gen_planted(const uint32_t* d_host, const uint64_t* d_prefix,
                                 const uint32_t* d_peer_salt, uint32_t m, uint64_t key,
                                 uint32_t window, uint32_t peer_domain_salt, uint32_t law,
                                 uint32_t* d_out, uint64_t cap, unsigned long long* d_counts,
                                 void* stream) {
  if (window < 1 || window > 15 || m == 0 || law > 1) return -1;
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -6;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -6;
  hipLaunchKernelGGL(k_gen_planted, dim3(n_cu * 8), dim3(256), 0, (hipStream_t)stream, d_host,
                     d_prefix, d_peer_salt, m, key, window, peer_domain_salt, law, d_out, cap,
                     d_counts);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}
