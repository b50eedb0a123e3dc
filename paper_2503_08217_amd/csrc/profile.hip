// Opt-in per-kernel timing with HIP events recorded on the launching stream
// around every kernel the library enqueues (off by default; never used while
// a stream is being captured into a graph).
#include <vector>

#include "internal.hpp"

namespace s3r {

static const char* kNames[K_COUNT] = {
    "compose", "plain_transform", "project", "block_offsets", "records", "scan", "emit_pairs",
    "radix", "tile_ranges", "tile_order", "tile_sort", "tile_sort_merge",
    "tile_bin", "raster_fwd", "l1_loss", "zero_g2d", "raster_bwd", "pair_reduce",
    "project_bwd", "pose_bwd", "pose6", "plain_transform_bwd", "visibility", "zero"};

namespace {
struct Pending {
  int id;
  int e0, e1;
};
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  int used = 0;
  double total_ms[K_COUNT] = {};
  long long count[K_COUNT] = {};
  int open_id = -1;
  int open_ev = -1;
  int only = -1;  // >= 0: bracket this kernel only
};
Prof g_prof;
constexpr int kPool = 8192;

void drain() {
  if (g_prof.pending.empty()) {
    g_prof.used = 0;
    return;
  }
  (void)hipEventSynchronize(g_prof.pool[g_prof.pending.back().e1]);
  for (const Pending& p : g_prof.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_prof.pool[p.e0], g_prof.pool[p.e1]) == hipSuccess) {
      g_prof.total_ms[p.id] += ms;
      g_prof.count[p.id] += 1;
    }
  }
  g_prof.pending.clear();
  g_prof.used = 0;
}
}  // namespace

void prof_begin(int id, hipStream_t st) {
  if (!g_prof.on || (g_prof.only >= 0 && id != g_prof.only)) return;
  if (g_prof.used + 2 > (int)g_prof.pool.size()) drain();
  g_prof.open_id = id;
  g_prof.open_ev = g_prof.used++;
  (void)hipEventRecord(g_prof.pool[g_prof.open_ev], st);
}

void prof_end(int id, hipStream_t st) {
  if (!g_prof.on || g_prof.open_id != id) return;
  const int e1 = g_prof.used++;
  (void)hipEventRecord(g_prof.pool[e1], st);
  g_prof.pending.push_back({id, g_prof.open_ev, e1});
  g_prof.open_id = -1;
}

}  // namespace s3r

using namespace s3r;

extern "C" {

int s3r_profile_enable(int on) {
  if (on && g_prof.pool.empty()) {
    g_prof.pool.resize(kPool);
    for (auto& e : g_prof.pool)
      if (hipEventCreate(&e) != hipSuccess) return S3R_E_HIP;
  }
  if (!on) drain();
  g_prof.on = on != 0;
  return S3R_OK;
}

int s3r_profile_only(int32_t id) {
  if (id >= K_COUNT) return S3R_E_ARG;
  g_prof.only = id < 0 ? -1 : id;
  return S3R_OK;
}

int s3r_profile_reset(void) {
  drain();
  for (int i = 0; i < K_COUNT; ++i) {
    g_prof.total_ms[i] = 0.0;
    g_prof.count[i] = 0;
  }
  return S3R_OK;
}

int s3r_profile_read(int32_t id, double* total_ms, int64_t* count) {
  if (id < 0 || id >= K_COUNT) return S3R_E_ARG;
  if (!total_ms || !count) return S3R_E_NULL;
  drain();
  *total_ms = g_prof.total_ms[id];
  *count = g_prof.count[id];
  return S3R_OK;
}

const char* s3r_profile_name(int32_t id) { return (id >= 0 && id < K_COUNT) ? kNames[id] : ""; }

int s3r_profile_kernels(void) { return K_COUNT; }

}  // extern "C"
