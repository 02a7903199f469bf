// Drives the host-only paths of the C ABI (argument validation, error texts, the tuning
// cache and its file format) for a build of the host code with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  No call here reaches the GPU.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sps.h"

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                      \
    }                                                                \
  } while (0)

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : "/tmp";
  sps_params p;
  memset(&p, 0, sizeof(p));
  p.q = 14; p.r = 11; p.delta = 2; p.eta = 8;
  p.qp = 16; p.rp = 5; p.etap = 1024; p.deltap = 1024;
  p.theta = 1024; p.seed = 7;
  size_t bytes = 0;
  CHECK(sps_sketch_bytes(&p, &bytes) == SPS_OK && bytes > (size_t)640 << 20);
  sps_params bad = p;
  bad.delta = 1;  // coverage (r-2)*delta + q < 32
  CHECK(sps_sketch_bytes(&bad, &bytes) == SPS_EINVAL);
  bad = p;
  bad.etap = 1000;  // not a power of two
  CHECK(sps_sketch_bytes(&bad, &bytes) == SPS_EINVAL);
  CHECK(sps_sketch_bytes(nullptr, &bytes) == SPS_EINVAL);
  sps_sketch* s = nullptr;
  CHECK(sps_create(&bad, nullptr, 0, &s) == SPS_EINVAL && s == nullptr);
  CHECK(sps_create(&p, nullptr, 0, nullptr) == SPS_EINVAL);
  for (int c = 1; c >= -8; --c) CHECK(sps_strerror(c) != nullptr && sps_strerror(c)[0]);
  CHECK(sps_destroy(nullptr) == SPS_EINVAL);
  CHECK(sps_reset(nullptr, nullptr) == SPS_EINVAL);
  CHECK(sps_ingest(nullptr, nullptr, 0, 1, nullptr) == SPS_EINVAL);
  CHECK(sps_merge(nullptr, nullptr, 0, nullptr) == SPS_EINVAL);
  size_t n_out = 0;
  CHECK(sps_scan(nullptr, 10, 1.0, nullptr, 0, &n_out, nullptr) == SPS_EINVAL);
  CHECK(sps_rebase(nullptr, 1, nullptr) == SPS_EINVAL);
  CHECK(sps_graph_end_update(nullptr, nullptr, nullptr) == SPS_EINVAL);
  CHECK(sps_stream_host_time(nullptr, nullptr) == SPS_EINVAL);
  CHECK(sps_probe_replay(nullptr, nullptr, nullptr, 1, nullptr) == SPS_EINVAL);
  size_t wb = 0;
  CHECK(sps_mlp_work_bytes(100, &wb) == SPS_OK && wb > 0);
  CHECK(sps_mlp_work_bytes(0, &wb) == SPS_EINVAL);
  float dummy[4];
  uint32_t udummy[4];
  CHECK(sps_mlp_grad_noalloc(dummy, udummy, dummy, nullptr, SPS_MLP_NOALLOC_MAX_N + 1, 1024,
                             dummy, nullptr, nullptr) == SPS_ECAPACITY);
  double ms[SPS_NSTAGES];
  uint32_t launches[SPS_NSTAGES];
  CHECK(sps_profile_enable(0) == SPS_OK);
  CHECK(sps_profile_read(ms, launches, SPS_NSTAGES) == SPS_OK);
  // tuning cache: write, read back, look up, reject a malformed file whole
  char path[512], badpath[512];
  snprintf(path, sizeof(path), "%s/tune.json", dir);
  snprintf(badpath, sizeof(badpath), "%s/bad.json", dir);
  FILE* f = fopen(path, "w");
  CHECK(f != nullptr);
  fprintf(f, "{\"sps_tuning_cache\": 1, \"entries\": [\n");
  fprintf(f, "{\"arch\": \"gfx950\", \"q\": 14, \"r\": 11, \"delta\": 2, \"eta\": 8, \"qp\": 16, "
             "\"rp\": 5, \"etap\": 1024, \"deltap\": 1024, \"mode\": 0, \"batched\": 1, "
             "\"blocks_per_cu\": 8, \"batch_tile\": 2048, \"host_classes\": 1}\n]}\n");
  fclose(f);
  CHECK(sps_tuning_cache_clear() == SPS_OK);
  CHECK(sps_tuning_cache_load(path) == SPS_OK);
  sps_tuning t;
  int found = 0;
  CHECK(sps_tuning_lookup("gfx950", &p, 1, &t, &found) == SPS_OK && found == 1);
  CHECK(t.blocks_per_cu == 8 && t.batch_tile == 2048 && t.host_classes == 1);
  CHECK(sps_tuning_lookup("gfx950", &p, 0, &t, &found) == SPS_OK && found == 0);
  CHECK(sps_tuning_cache_save(path) == SPS_OK);
  CHECK(sps_tuning_cache_load(path) == SPS_OK);
  f = fopen(badpath, "w");
  CHECK(f != nullptr);
  fprintf(f, "{\"sps_tuning_cache\": 1, \"entries\": [\n{\"arch\": \"gfx950\", \"q\": 14}\n]}\n");
  fclose(f);
  CHECK(sps_tuning_cache_load(badpath) == SPS_EINVAL);
  CHECK(sps_tuning_cache_load("/nonexistent/dir/x.json") == SPS_EINVAL);
  CHECK(sps_tuning_cache_clear() == SPS_OK);
  printf("host ABI sanitizer run ok\n");
  return 0;
}
