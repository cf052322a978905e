// Host runtime of the TABI packer: argument checks, work-space carving from
// the device's stream-ordered memory pool, launch sequence.  Implements the C
// ABI declared in include/tabi.h.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>
#include <string.h>
#include <vector>

#include "../../include/tabi.h"
#include "tabi_internal.h"

using namespace tabi;

namespace {

thread_local char g_last_hip[256] = "";

int hip_fail(hipError_t e) {
  strncpy(g_last_hip, hipGetErrorString(e), sizeof(g_last_hip) - 1);
  return TABI_EHIP;
}

int slices_for_quality(int q) { return q == 0 ? 2 : (q == 1 ? 5 : 10); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Per-device set-up, once: the LDS a workgroup may use, and a release
// threshold on the default stream-ordered pool so that work space freed at
// the end of one call is reused by the next instead of returned to the OS.
int lds_budget() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  std::lock_guard<std::mutex> lk(mu);
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    cache[dev] = v;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
  }
  return cache[dev];
}

// ---- opt-in per-stage timing with HIP events on the call's stream ----------
enum Stage { ST_PREP = 0, ST_SORT, ST_SETUP, ST_PAIRS, ST_PACK, ST_SELECT, ST_COUNT };
struct Timing {
  std::mutex mu;
  bool on = false;
  struct Mark { int stage; hipEvent_t a, b; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  double ms[ST_COUNT] = {0};
  int launches[ST_COUNT] = {0};
} g_timing;

hipEvent_t pool_event() {
  if (!g_timing.pool.empty()) {
    hipEvent_t e = g_timing.pool.back();
    g_timing.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct StageScope {  // brackets one stage's launches with a pair of events
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageScope(int s_, hipStream_t st_) : stage(s_), st(st_) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (!g_timing.on) return;
    a = pool_event();
    if (a) (void)hipEventRecord(a, st);
  }
  ~StageScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    hipEvent_t b = pool_event();
    if (!b) return;
    (void)hipEventRecord(b, st);
    g_timing.marks.push_back({stage, a, b});
  }
};

// static shared memory of k_pack (s_cnt, s_red, s_red64, s_lrn, s_lrover, s_lr)
constexpr int kPackStaticLds = 4 * 4 + 8 * 6 * 4 + 8 * 8 + 8 + 256 * 3 * 4 + 64;

struct Job {
  Params P{};
  Work W{};
  void* base = nullptr;
  PackLds L{};
};

// Carve the work space for N charts over `count` atlases with B scale slots.
int make_job(Job& j, int count, int N, int q, int p, int B, int fixed_k, int nmax, int Wdmax,
             hipStream_t st) {
  j.P.count = count;
  j.P.N = N;
  j.P.K = slices_for_quality(q);
  j.P.q = q;
  j.P.p = p;
  j.P.B = B;
  j.P.stride = kchart_stride(j.P.K);
  j.P.fixed_k = fixed_k;
  const size_t n1 = (size_t)(N > 0 ? N : 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_recs = take(n1 * sizeof(Chart));
  const size_t o_srecs = take(n1 * sizeof(Chart));
  const size_t o_keys = take(n1 * 8);
  const size_t o_perm = take(n1 * 4);
  const size_t o_ca = take(n1 * 4);
  const size_t o_desc = take((size_t)count * sizeof(AtlasDesc));
  const size_t o_kc = take((size_t)B * n1 * j.P.stride);
  const size_t o_cd = take((size_t)B * n1 * 4);
  const size_t o_fl = take((size_t)B * n1);
  const size_t o_xs = take((size_t)B * n1 * 4);
  const size_t o_ys = take((size_t)B * n1 * 4);
  const size_t o_mir = take((size_t)B * n1);
  const size_t o_feas = take((size_t)count * B * 4);
  const size_t o_rows = take((size_t)count * B * 4);
  const int budget = lds_budget();
  hipError_t e = hipMallocAsync(&j.base, off, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? TABI_ENOMEM : hip_fail(e);
  }
  unsigned char* b = static_cast<unsigned char*>(j.base);
  j.W.recs = reinterpret_cast<Chart*>(b + o_recs);
  j.W.srecs = reinterpret_cast<Chart*>(b + o_srecs);
  j.W.keys = reinterpret_cast<uint64_t*>(b + o_keys);
  j.W.perm = reinterpret_cast<int32_t*>(b + o_perm);
  j.W.chart_atlas = reinterpret_cast<int32_t*>(b + o_ca);
  j.W.desc = reinterpret_cast<AtlasDesc*>(b + o_desc);
  j.W.kc = b + o_kc;
  j.W.cd = reinterpret_cast<int32_t*>(b + o_cd);
  j.W.fl = b + o_fl;
  j.W.xs = reinterpret_cast<int32_t*>(b + o_xs);
  j.W.ys = reinterpret_cast<int32_t*>(b + o_ys);
  j.W.mir = b + o_mir;
  j.W.feas = reinterpret_cast<int32_t*>(b + o_feas);
  j.W.rows = reinterpret_cast<int32_t*>(b + o_rows);
  j.L = pack_lds_plan(nmax, Wdmax, budget - kPackStaticLds);
  return TABI_OK;
}

void free_job(Job& j, hipStream_t st) {
  if (j.base) (void)hipFreeAsync(j.base, st);
  j.base = nullptr;
}

bool bad_atlas(int32_t w, int32_t h, int32_t p) {
  return w < 1 || h < 1 || (int64_t)w + p > 16384 || (int64_t)h + p > 16384;
}

int check_common(int32_t n, int32_t padding, int32_t quality) {
  if (n < 0 || n > TABI_MAX_CHARTS || padding < 0 || quality < 0 || quality > 2) return TABI_EINVAL;
  return TABI_OK;
}

// front half shared by the single-atlas entry points: descriptors, proxies, order, bound
int front(Job& j, const tabi_charts* ch, int32_t n, int32_t aw, int32_t ah, hipStream_t st) {
  hipError_t e;
  {
    StageScope t(ST_PREP, st);
    e = launch_prep(j.P, j.W, ch->xy, ch->offsets, nullptr, nullptr, aw, ah, st);
  }
  if (e == hipSuccess) {
    StageScope t(ST_SORT, st);
    e = launch_sort(j.P, j.W, st);
  }
  return e == hipSuccess ? TABI_OK : hip_fail(e);
}

}  // namespace

extern "C" {

int tabi_pack(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
              int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
              float* out_scale, tabi_stream_t stream) {
  if (check_common(n, padding, quality) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !out_scale || (n > 0 && (!charts->xy || !charts->offsets || !out_xy || !out_orient)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  // every candidate scale at once: one workgroup per scale, no host round trip
  int rc = make_job(j, 1, n, quality, padding, 64, 0, n, atlas_w + padding, st);
  if (rc) return rc;
  rc = front(j, charts, n, atlas_w, atlas_h, st);
  hipError_t e = hipSuccess;
  if (!rc) { StageScope t(ST_SETUP, st); e = launch_setup(j.P, j.W, 0, st); }
  if (!rc && e == hipSuccess) { StageScope t(ST_PAIRS, st); e = launch_pairs(j.P, j.W, 0, st); }
  if (!rc && e == hipSuccess) {
    StageScope t(ST_PACK, st);
    e = launch_pack(j.P, j.W, 0, j.L.bytes, j.L.RC, j.L.SC, st);
  }
  if (!rc && e == hipSuccess) {
    StageScope t(ST_SELECT, st);
    e = launch_select(j.P, j.W, 0, 1, out_xy, out_orient, out_scale, st);
  }
  if (!rc && e != hipSuccess) rc = hip_fail(e);
  free_job(j, st);
  return rc;
}

int tabi_pack_many(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                   int32_t count, const int32_t* atlas_wh, int32_t padding, int32_t quality,
                   int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                   tabi_stream_t stream) {
  (void)xy; (void)vert_offsets; (void)atlas_offsets; (void)count; (void)atlas_wh;
  (void)padding; (void)quality; (void)out_xy; (void)out_orient; (void)out_scale; (void)stream;
  return TABI_EINVAL;
}

int tabi_debug_order(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, int32_t quality, int32_t* perm, int32_t* khi,
                     tabi_stream_t stream) {
  if (check_common(n, padding, quality) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !khi || (n > 0 && (!charts->xy || !charts->offsets || !perm)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  int rc = make_job(j, 1, n, quality, padding, 1, 0, n, atlas_w + padding, st);
  if (rc) return rc;
  rc = front(j, charts, n, atlas_w, atlas_h, st);
  if (!rc) {
    hipError_t e = hipSuccess;
    if (n > 0) e = hipMemcpyAsync(perm, j.W.perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(khi, &j.W.desc[0].ktop, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  free_job(j, st);
  return rc;
}

int tabi_debug_pairs(const tabi_charts* charts, int32_t n, int32_t padding, int32_t quality,
                     int32_t k, int32_t* cd, uint8_t* flags, tabi_stream_t stream) {
  if (check_common(n, padding, quality) || k < 1 || k > 64 || !charts ||
      (n > 0 && (!charts->xy || !charts->offsets || !cd || !flags)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  int rc = make_job(j, 1, n, quality, padding, 1, k, n, 1 + padding, st);
  if (rc) return rc;
  rc = front(j, charts, n, 16384 - padding, 16384 - padding, st);
  hipError_t e = hipSuccess;
  if (!rc) e = launch_setup(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess) e = launch_pairs(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess && n > 0)
    e = hipMemcpyAsync(cd, j.W.cd, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
  if (!rc && e == hipSuccess && n > 0)
    e = hipMemcpyAsync(flags, j.W.fl, n, hipMemcpyDeviceToDevice, st);
  if (!rc && e != hipSuccess) rc = hip_fail(e);
  free_job(j, st);
  return rc;
}

int tabi_debug_feasible(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                        int32_t padding, int32_t quality, int32_t k, int32_t* out_xy,
                        uint8_t* out_orient, int32_t* feasible, int32_t* rows,
                        tabi_stream_t stream) {
  if (check_common(n, padding, quality) || bad_atlas(atlas_w, atlas_h, padding) || k < 1 ||
      k > 64 || !charts || !feasible || !rows ||
      (n > 0 && (!charts->xy || !charts->offsets || !out_xy || !out_orient)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  int rc = make_job(j, 1, n, quality, padding, 1, k, n, atlas_w + padding, st);
  if (rc) return rc;
  rc = front(j, charts, n, atlas_w, atlas_h, st);
  hipError_t e = hipSuccess;
  if (!rc) e = launch_setup(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess) e = launch_pairs(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess) e = launch_pack(j.P, j.W, 0, j.L.bytes, j.L.RC, j.L.SC, st);
  if (!rc && e == hipSuccess) e = launch_scatter(j.P, j.W, out_xy, out_orient, feasible, rows, st);
  if (!rc && e != hipSuccess) rc = hip_fail(e);
  free_job(j, st);
  return rc;
}

const char* tabi_strerror(int code) {
  switch (code) {
    case TABI_OK: return "ok";
    case TABI_EINVAL: return "invalid argument";
    case TABI_ENOMEM: return "out of device memory";
    case TABI_EHIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

const char* tabi_last_hip_error(void) { return g_last_hip; }

int tabi_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  g_timing.on = on != 0;
  return TABI_OK;
}

int tabi_timing_read(double* ms, int32_t* launches, int32_t nstages) {
  std::vector<Timing::Mark> marks;
  {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    marks.swap(g_timing.marks);
  }
  int rc = TABI_OK;
  for (auto& m : marks) {
    float t = 0.f;
    hipError_t e = hipEventSynchronize(m.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, m.a, m.b);
    if (e != hipSuccess) rc = hip_fail(e);
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.ms[m.stage] += t;
    g_timing.launches[m.stage] += 1;
    g_timing.pool.push_back(m.a);
    g_timing.pool.push_back(m.b);
  }
  std::lock_guard<std::mutex> lk(g_timing.mu);
  for (int i = 0; i < nstages && i < ST_COUNT; ++i) {
    if (ms) ms[i] = g_timing.ms[i];
    if (launches) launches[i] = g_timing.launches[i];
  }
  return rc;
}

void tabi_timing_reset(void) {
  int32_t dummy[ST_COUNT];
  tabi_timing_read(nullptr, dummy, 0);
  std::lock_guard<std::mutex> lk(g_timing.mu);
  for (int i = 0; i < ST_COUNT; ++i) { g_timing.ms[i] = 0; g_timing.launches[i] = 0; }
}

int64_t tabi_pack_lds_bytes(int32_t n, int32_t atlas_w, int32_t padding) {
  PackLds L = pack_lds_plan(n, atlas_w + padding, lds_budget() - kPackStaticLds);
  return (int64_t)L.bytes + kPackStaticLds;
}

}  // extern "C"
