// Host runtime of the TABI packer: argument checks, work-space layout, the
// launch sequence.  Implements the C ABI declared in include/tabi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// A method code names the method's knobs (Sec. 5 ablations): the quality
// presets 0, 1, 2, or a packed custom setting (bit 24 set) of the local-AABB
// count (bits 4-7), t_opt + 1 (bits 8-15) and variant (bits 16-19).
constexpr int32_t kCustom = 1 << 24;
struct Method {
  int K, topt, variant;  // topt < 0: the paper's setting, per atlas
  int cls;               // 0..2: the preset whose tuned batched shapes it uses
};
bool code_ok(int32_t code) {
  if (code >= 0 && code <= 2) return true;
  if ((code >> 24) != 1) return false;
  const int K = (code >> 4) & 0xf, topt = ((code >> 8) & 0xff) - 1, v = (code >> 16) & 0xf;
  return (K == 1 || K == 2 || K == 5 || K == 10) && topt >= -1 && topt <= 100 && v <= 2;
}
Method decode_method(int32_t code) {
  if (code >= 0 && code <= 2)
    return {code == 0 ? 2 : (code == 1 ? 5 : 10), code == 0 ? 5 : (code == 1 ? 2 : -1),
            TABI_FULL, code};
  const int K = (code >> 4) & 0xf, topt = ((code >> 8) & 0xff) - 1, v = (code >> 16) & 0xf;
  const int Kr = v == TABI_BALANCED_ONLY ? 1 : K;  // balanced-only packs the boxes
  return {Kr, topt, v, Kr >= 10 ? 2 : (Kr >= 5 ? 1 : 0)};
}
int32_t encode_method(const tabi_method& m) {
  return kCustom | ((m.slices & 0xf) << 4) | (((m.topt_percent + 1) & 0xff) << 8) |
         ((m.variant & 0xf) << 16);
}
bool method_ok(const tabi_method* m) {
  return m && (m->slices == 1 || m->slices == 2 || m->slices == 5 || m->slices == 10) &&
         m->topt_percent >= -1 && m->topt_percent <= 100 && m->variant >= TABI_FULL &&
         m->variant <= TABI_BALANCED_ONLY;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// static shared memory of k_pack, read from the compiled kernel once
int kPackStaticLds = 32 * 1024;
// test knobs: upper bound on the row staging area (texel columns) and on the
// profile arena (32-bit words); < 0 = default
int g_stage_cap = -1;
int g_pack_lds = -1;
int64_t g_profile_cap = -1;

// Per-device set-up, once: the LDS a workgroup may use (the packing kernel is
// allowed all of it), and a release threshold on the default stream-ordered
// pool so that work space freed by one call is reused by the next.
int lds_budget() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  std::lock_guard<std::mutex> lk(mu);
  if (!cache[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
      v = 64 * 1024;
    cache[dev] = v;
    kPackStaticLds = pack_static_lds() + 256;
    (void)pack_set_max_lds(v - kPackStaticLds);
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
enum Stage { ST_PREP = 0, ST_SORT, ST_SETUP, ST_PROFILE, ST_PACK, ST_SELECT, ST_COUNT };
struct Timing {
  std::mutex mu;
  bool on = false;
  uint32_t mask = (1u << ST_COUNT) - 1;  // the stages bracketed while on
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
    if (!g_timing.on || !((g_timing.mask >> s_) & 1u)) return;
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

// ---- work space -------------------------------------------------------------
struct Layout {
  size_t o_recs, o_srecs, o_keys, o_pl, o_skey, o_satl, o_rank, o_perm, o_ca, o_desc, o_kc, o_cd, o_fl, o_xs, o_ys, o_mir,
      o_feas, o_rows, o_wdv, o_hdv, o_kslot, o_pcol, o_prow, o_lrpre, o_Hs, o_segneed, o_segbase, o_cnt, o_gq, o_gq_cnt, o_live, o_aord,
      o_tailF, o_tail_t0, o_tail_kt, o_tail_obj, o_arena,
      total;
};

// Profile arena words for B scale slots over N charts in `count` atlases of
// grown width up to Wdmax.  A chart of grown extents w x h takes w + 2h words
// at a scale (its columns, then its rows once per proxy); per slot and chart
// `per` words are set aside (the single pack spreads its 64 slots over scales
// 1..k_top, so it needs fewer on average: about 8,400 words per chart over
// all 64 scales for the 2,000-chart 2048^2 workload; a batch of mixed
// atlases about 1,100 over its top 8 scales), plus four atlas widths per
// (atlas, slot).  Segments are placed in descending-scale order and those
// that do not fit are evaluated directly, so the figure only trades memory
// for speed.
int64_t arena_words(const Params& P) {
  if (g_profile_cap >= 0) return g_profile_cap;
  const int64_t per = P.B >= 64 ? 150 : 180;
  int64_t v = (int64_t)P.B * P.N * per + (int64_t)P.B * P.count * 4 * P.Wdmax;
  const int64_t lim = 0x7fffffffLL;  // word indices are int32
  return v > lim ? lim : v;
}

Layout layout(const Params& P) {
  Layout L{};
  const size_t n1 = (size_t)(P.N > 0 ? P.N : 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  L.o_recs = take(n1 * sizeof(Chart));
  L.o_srecs = take(n1 * sizeof(Chart));
  L.o_keys = take(n1 * 8);
  L.o_pl = take(n1 * 16);
  const size_t nt = (n1 + 255) / 256 * 256;  // whole key tiles
  L.o_skey = take(nt * 8);
  L.o_satl = take(nt * 4);
  L.o_rank = take(n1 * 4);
  L.o_perm = take(n1 * 4);
  L.o_ca = take(n1 * 4);
  L.o_desc = take((size_t)P.count * sizeof(AtlasDesc));
  L.o_kc = take((size_t)P.B * n1 * P.stride);
  L.o_cd = take((size_t)P.B * n1 * 4);
  L.o_fl = take((size_t)P.B * n1);
  L.o_xs = take((size_t)P.B * n1 * 4);
  L.o_ys = take((size_t)P.B * n1 * 4);
  L.o_mir = take((size_t)P.B * n1);
  L.o_feas = take((size_t)P.count * P.B * 4);
  L.o_rows = take((size_t)P.count * P.B * 4);
  L.o_wdv = take((size_t)P.B * n1 * 4);
  L.o_hdv = take((size_t)P.B * n1 * 4);
  L.o_kslot = take((size_t)P.B * n1 * 4);
  L.o_pcol = take((size_t)P.B * n1 * 4);
  L.o_prow = take((size_t)P.B * n1 * 4);
  L.o_lrpre = take((size_t)P.B * n1 * 4);
  L.o_Hs = take(n1 * 4);
  L.o_segneed = take((size_t)P.count * P.B * 8);
  L.o_segbase = take((size_t)P.count * P.B * 4);
  L.o_cnt = take((size_t)P.count * 4);
  L.o_gq = take((size_t)P.B * ((n1 + PROF_CH - 1) / PROF_CH) * 4);
  L.o_gq_cnt = take(4);
  L.o_live = take((MAX_ROUNDS + 1) * 4);
  L.o_aord = take((size_t)P.count * 4);
  const size_t hb = P.hybrid ? (size_t)P.B : 0;
  L.o_tailF = take(hb * (size_t)P.Wdmax * 4);
  L.o_tail_t0 = take(hb * 4);
  L.o_tail_kt = take(hb * 4);
  L.o_tail_obj = take(P.hybrid ? (hb + 1) * 16 : 0);
  L.o_arena = take((size_t)P.arena_cap * 4);
  L.total = off;
  return L;
}

Work carve(void* base, const Layout& L) {
  unsigned char* b = static_cast<unsigned char*>(base);
  Work W;
  W.recs = reinterpret_cast<Chart*>(b + L.o_recs);
  W.srecs = reinterpret_cast<Chart*>(b + L.o_srecs);
  W.keys = reinterpret_cast<uint64_t*>(b + L.o_keys);
  W.pl = reinterpret_cast<int4*>(b + L.o_pl);
  W.skey = reinterpret_cast<uint64_t*>(b + L.o_skey);
  W.satl = reinterpret_cast<int32_t*>(b + L.o_satl);
  W.rank = reinterpret_cast<int32_t*>(b + L.o_rank);
  W.perm = reinterpret_cast<int32_t*>(b + L.o_perm);
  W.chart_atlas = reinterpret_cast<int32_t*>(b + L.o_ca);
  W.desc = reinterpret_cast<AtlasDesc*>(b + L.o_desc);
  W.kc = b + L.o_kc;
  W.cd = reinterpret_cast<int32_t*>(b + L.o_cd);
  W.fl = b + L.o_fl;
  W.xs = reinterpret_cast<int32_t*>(b + L.o_xs);
  W.ys = reinterpret_cast<int32_t*>(b + L.o_ys);
  W.mir = b + L.o_mir;
  W.feas = reinterpret_cast<int32_t*>(b + L.o_feas);
  W.rows = reinterpret_cast<int32_t*>(b + L.o_rows);
  W.wdv = reinterpret_cast<int32_t*>(b + L.o_wdv);
  W.hdv = reinterpret_cast<int32_t*>(b + L.o_hdv);
  W.kslot = reinterpret_cast<int32_t*>(b + L.o_kslot);
  W.pcol = reinterpret_cast<int32_t*>(b + L.o_pcol);
  W.prow = reinterpret_cast<int32_t*>(b + L.o_prow);
  W.lrpre = reinterpret_cast<int32_t*>(b + L.o_lrpre);
  W.Hs = reinterpret_cast<int32_t*>(b + L.o_Hs);
  W.segneed = reinterpret_cast<int64_t*>(b + L.o_segneed);
  W.segbase = reinterpret_cast<int32_t*>(b + L.o_segbase);
  W.cnt = reinterpret_cast<int32_t*>(b + L.o_cnt);
  W.gq = reinterpret_cast<int32_t*>(b + L.o_gq);
  W.gq_cnt = reinterpret_cast<int32_t*>(b + L.o_gq_cnt);
  W.live = reinterpret_cast<int32_t*>(b + L.o_live);
  W.aord = reinterpret_cast<int32_t*>(b + L.o_aord);
  W.tailF = reinterpret_cast<int32_t*>(b + L.o_tailF);
  W.tail_t0 = reinterpret_cast<int32_t*>(b + L.o_tail_t0);
  W.tail_kt = reinterpret_cast<int32_t*>(b + L.o_tail_kt);
  W.tail_obj = reinterpret_cast<uint64_t*>(b + L.o_tail_obj);
  W.arena = reinterpret_cast<uint32_t*>(b + L.o_arena);
  return W;
}

struct Job {
  Params P{};
  Work W{};
  void* base = nullptr;  // owned (stream-ordered pool) when set
  PackLds L{};
  int stage_cap = 0x7fffffff;
};

Params make_params(int count, int N, int q, int p, int B, int fixed_k, int nmax, int Wdmax) {
  const Method m = decode_method(q);
  Params P{};
  P.count = count;
  P.N = N;
  P.K = m.K;
  P.q = m.cls;
  P.topt = m.topt;
  P.variant = m.variant;
  P.p = p;
  P.B = B;
  P.Br = B;
  P.koff = 0;
  P.stride = kchart_stride(P.K);
  P.fixed_k = fixed_k;
  P.nmax = nmax;
  P.Wdmax = Wdmax;
  P.arena_cap = 0;
  P.pack_nt = 0;
  P.arena_cap = arena_words(P);
  return P;
}

// lds_cap: upper bound on the packing kernel's shared memory (0: device limit)
int make_job(Job& j, const Params& P, hipStream_t st, void* ws = nullptr, size_t ws_bytes = 0,
             int lds_cap = 0) {
  j.P = P;
  const int budget = lds_budget();
  int b = budget - kPackStaticLds;
  // a preferred cap (two workgroups per CU) yields to what the widest atlas
  // needs: the offsets of every configuration plus a staged row of twice the
  // atlas width (compaction lets a row's boxes overlap)
  if (lds_cap > 0 && lds_cap < b) {
    const PackLds c = pack_lds_plan(P.nmax, P.Wdmax, lds_cap);
    if (c.bytes <= lds_cap && c.PW >= 4 * c.RC + 3 * P.Wdmax) b = lds_cap;
  }
  if (g_pack_lds >= 0)  // test knob: at most this much, at least the smallest plan
    b = std::min(b, std::max(g_pack_lds, pack_lds_plan(P.nmax, P.Wdmax, 0).bytes));
  j.L = pack_lds_plan(P.nmax, P.Wdmax, b);
  if (j.L.bytes > b) return TABI_EINVAL;  // rows of this atlas cannot fit in LDS
  j.stage_cap = g_stage_cap >= 0 ? g_stage_cap : 0x7fffffff;
  const Layout L = layout(P);
  if (ws) {
    if (ws_bytes < L.total) return TABI_EINVAL;
    j.base = nullptr;
    j.W = carve(ws, L);
  } else {
    void* base = nullptr;
    hipError_t e = hipMallocAsync(&base, L.total, st);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e == hipErrorOutOfMemory ? TABI_ENOMEM : hip_fail(e);
    }
    j.base = base;
    j.W = carve(base, L);
  }
  return TABI_OK;
}

void free_job(Job& j, hipStream_t st) {
  if (j.base) (void)hipFreeAsync(j.base, st);
  j.base = nullptr;
}

bool bad_atlas(int32_t w, int32_t h, int32_t p) {
  return w < 1 || h < 1 || (int64_t)w + p > 16384 || (int64_t)h + p > 16384;
}

// code: a method code (pack_single); the public entry points that take a
// quality preset use check_common, which admits only the presets
int check_common_code(int32_t n, int32_t padding, int32_t code) {
  if (n < 0 || n > TABI_MAX_CHARTS || padding < 0 || padding > TABI_MAX_PADDING ||
      !code_ok(code))
    return TABI_EINVAL;
  return TABI_OK;
}
int check_common(int32_t n, int32_t padding, int32_t quality) {
  if (quality < 0 || quality > 2) return TABI_EINVAL;
  return check_common_code(n, padding, quality);
}

hipError_t run_front(Job& j, const int32_t* xy, const int32_t* voff, const int32_t* aoff,
                     const int32_t* awh, int32_t aw, int32_t ah, hipStream_t st,
                     const int32_t* cloop = nullptr) {
  hipError_t e;
  {
    StageScope t(ST_PREP, st);
    e = launch_prep(j.P, j.W, xy, voff, aoff, awh, aw, ah, st, cloop);
  }
  if (e == hipSuccess) {
    StageScope t(ST_SORT, st);
    e = launch_sort(j.P, j.W, st);
  }
  return e;
}

// rounds of descending scales per atlas until each atlas has its answer:
// round r evaluates slots[r] scales below those of the earlier rounds
hipError_t run_search(Job& j, const int* slots, int rounds, int32_t* out_xy, uint8_t* out_orient,
                      float* out_scale, hipStream_t st) {
  hipError_t e = hipSuccess;
  const Params P0 = j.P;
  int koff = 0;
  for (int r = 0; r < rounds && e == hipSuccess; ++r) {
    j.P = P0;
    j.P.Br = slots[r];
    j.P.koff = koff;
    koff += slots[r];
    {
      StageScope t(ST_SETUP, st);
      e = launch_setup(j.P, j.W, r, st);
    }
    if (e == hipSuccess) {
      StageScope t(ST_PROFILE, st);
      e = launch_profiles(j.P, j.W, r, st);
    }
    if (e == hipSuccess) {  // with the scale selection of a single atlas
      StageScope t(ST_PACK, st);
      e = launch_pack(j.P, j.W, r, j.L.bytes, j.L.RC, j.L.PW, j.stage_cap, r == rounds - 1, out_xy,
                      out_orient, out_scale, st);
    }
    if (e == hipSuccess && j.P.count > 1) {
      StageScope t(ST_SELECT, st);
      e = launch_select(j.P, j.W, r, r == rounds - 1, out_xy, out_orient, out_scale, st);
    }
  }
  j.P = P0;
  return e;
}

// Batched shape: the round schedule (b0 scale slots per round for the first
// `flat` rounds, then doubling up to bmax, until the 64 candidate scales are
// covered: rounds far from an atlas's area bound cost fewer round trips),
// the fold-and-push workgroup size, and the shared-memory cap of that
// workgroup (78 KB lets two 512-thread workgroups share a CU; 0 = the device
// limit).  Chosen per device, quality and batch size class by
// tabi_tune_many; the first entry is the default.
struct ManyShape {
  int b0, flat, bmax, nt, cap;
};
const ManyShape kManyShapes[] = {
    {8, 64, 8, 512, 78 * 1024}, {4, 64, 4, 512, 78 * 1024}, {16, 64, 16, 512, 78 * 1024},
    {8, 64, 8, 1024, 0},        {16, 64, 16, 1024, 0},      {4, 2, 32, 512, 78 * 1024},
    {4, 3, 16, 512, 78 * 1024}, {4, 64, 4, 1024, 0}};
constexpr int kNumManyShapes = (int)(sizeof(kManyShapes) / sizeof(kManyShapes[0]));

// slots per round of a schedule; returns the number of rounds (<= 64)
int schedule(const ManyShape& sh, int* slots) {
  int r = 0, covered = 0;
  while (covered < 64) {
    const int b = r < sh.flat ? sh.b0 : std::min(sh.bmax, sh.b0 << std::min(r - sh.flat + 1, 6));
    slots[r++] = b;
    covered += b;
  }
  return r;
}
int schedule_max(const ManyShape& sh) {
  int slots[64];
  const int n = schedule(sh, slots);
  int m = 1;
  for (int i = 0; i < n; ++i) m = std::max(m, slots[i]);
  return m;
}
// batch size classes: up to 8 atlases, up to 64, more
constexpr int kShapeClasses = 3;
int shape_class(int count) { return count <= 8 ? 0 : (count <= 64 ? 1 : 2); }
std::mutex g_shape_mu;
// [device][quality][class]: index + 1 into kManyShapes, 0 = default
int g_shape[64][3][kShapeClasses] = {};

ManyShape many_shape(int code, int count) {
  int dev = 0;
  if (!code_ok(code) || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return kManyShapes[0];
  const int quality = decode_method(code).cls;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  const int i = g_shape[dev][quality][shape_class(count)];
  return i > 0 ? kManyShapes[i - 1] : kManyShapes[0];
}
// cls < 0: every size class
void set_many_shape(int code, int cls, int index) {
  int dev = 0;
  if (!code_ok(code) || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  const int quality = decode_method(code).cls;
  std::lock_guard<std::mutex> lk(g_shape_mu);
  for (int c = 0; c < kShapeClasses; ++c)
    if (cls < 0 || c == cls) g_shape[dev][quality][c] = index + 1;
}

int many_check(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
               int32_t count, const int32_t* atlas_wh, int32_t total_charts, int32_t max_charts,
               int32_t max_side, int32_t padding, int32_t quality, int32_t* out_xy,
               uint8_t* out_orient, float* out_scale) {
  if (count < 0 || total_charts < 0 || max_charts < 0 || max_charts > TABI_MAX_CHARTS ||
      max_side < 1 || (int64_t)max_side + padding > 16384 || padding < 0 ||
      padding > TABI_MAX_PADDING || !code_ok(quality))
    return TABI_EINVAL;
  if (count > 0 && (!atlas_offsets || !atlas_wh || !out_scale)) return TABI_EINVAL;
  if (total_charts > 0 && (!xy || !vert_offsets || !out_xy || !out_orient)) return TABI_EINVAL;
  return TABI_OK;
}

Params many_params(int32_t count, int32_t total_charts, int32_t max_charts, int32_t max_side,
                   int32_t padding, int32_t quality) {
  const ManyShape sh = many_shape(quality, count);
  Params P = make_params(count, total_charts, quality, padding, schedule_max(sh), 0,
                         max_charts > 0 ? max_charts : 1, max_side + padding);
  P.pack_nt = sh.nt;
  return P;
}

int pack_many_impl(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                   int32_t count, const int32_t* atlas_wh, int32_t total_charts,
                   int32_t max_charts, int32_t max_side, int32_t padding, int32_t quality,
                   int32_t* out_xy, uint8_t* out_orient, float* out_scale, void* ws,
                   size_t ws_bytes, tabi_stream_t stream, const void* records = nullptr) {
  int rc = many_check(records ? (const int32_t*)records : xy,
                      records ? atlas_offsets : vert_offsets, atlas_offsets, count, atlas_wh,
                      total_charts, max_charts, max_side, padding, quality, out_xy, out_orient,
                      out_scale);
  if (rc) return rc;
  if (count == 0) return TABI_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  const ManyShape sh = many_shape(quality, count);
  rc = make_job(j, many_params(count, total_charts, max_charts, max_side, padding, quality), st,
                ws, ws_bytes, sh.cap);
  if (rc) {
    free_job(j, st);
    return rc;
  }
  hipError_t e;
  if (records) {
    {
      StageScope t(ST_PREP, st);
      e = launch_from_records(j.P, j.W, static_cast<const Chart*>(records), atlas_offsets,
                              atlas_wh, st);
    }
    if (e == hipSuccess) {
      StageScope t(ST_SORT, st);
      e = launch_sort(j.P, j.W, st);
    }
  } else {
    e = run_front(j, xy, vert_offsets, atlas_offsets, atlas_wh, 0, 0, st);
  }
  int slots[64];
  const int rounds = schedule(sh, slots);
  if (e == hipSuccess) e = run_search(j, slots, rounds, out_xy, out_orient, out_scale, st);
  if (e != hipSuccess) rc = hip_fail(e);
  free_job(j, st);
  return rc;
}

int single_front(Job& j, const tabi_charts* ch, int32_t aw, int32_t ah, hipStream_t st,
                 const int32_t* cloop = nullptr) {
  hipError_t e = run_front(j, ch->xy, ch->offsets, nullptr, nullptr, aw, ah, st, cloop);
  return e == hipSuccess ? TABI_OK : hip_fail(e);
}

// A single pack with method code `code`: every candidate scale at once, one
// workgroup per scale, no host round trip.
int pack_single(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                int32_t padding, int32_t code, int32_t* out_xy, uint8_t* out_orient,
                float* out_scale, tabi_stream_t stream, const int32_t* cloop = nullptr) {
  if (check_common_code(n, padding, code) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !out_scale || (n > 0 && (!charts->xy || !charts->offsets || !out_xy || !out_orient)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  Params P = make_params(1, n, code, padding, 64, 0, n > 0 ? n : 1, atlas_w + padding);
  P.loops = cloop != nullptr;
  int rc = make_job(j, P, st);
  if (!rc) rc = single_front(j, charts, atlas_w, atlas_h, st, cloop);
  if (!rc) {
    const int all[1] = {64};
    hipError_t e = run_search(j, all, 1, out_xy, out_orient, out_scale, st);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  free_job(j, st);
  return rc;
}

// Work space of tabi_pack_noalloc: a static device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses
// the array's name as an address: its device address is looked up once per
// device (scratch_ptr) and that pointer is what the kernels receive.
constexpr size_t kScratchBytes = (size_t)TABI_NOALLOC_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// Device address of `scratch` on the current device; nullptr (and the HIP
// error recorded) if the lookup fails.
void* scratch_ptr() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= 64) {
    if (e != hipSuccess) hip_fail(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

namespace tabi {

int64_t host_many_workspace_bytes(int count, int N, int nmax, int max_side, int p, int q) {
  return (int64_t)layout(many_params(count, N, nmax, max_side, p, q)).total;
}

int host_pack_many_records_ws(const Chart* recs, const int32_t* aoff, int count,
                              const int32_t* awh, int N, int nmax, int max_side, int p, int q,
                              int32_t* out_xy, uint8_t* out_orient, float* out_scale, void* ws,
                              size_t ws_bytes, hipStream_t st) {
  if (!ws) return TABI_EINVAL;
  return pack_many_impl(nullptr, nullptr, aoff, count, awh, N, nmax, max_side, p, q, out_xy,
                        out_orient, out_scale, ws, ws_bytes, reinterpret_cast<tabi_stream_t>(st),
                        recs ? static_cast<const void*>(recs) : static_cast<const void*>(aoff));
}

size_t host_prep_scratch_bytes(int M) {
  return align_up((size_t)(M > 0 ? M : 1) * 8, 256) + align_up((size_t)(M > 0 ? M : 1) * 4, 256);
}

int host_prep_records(const int32_t* xy, const int32_t* voff, const int32_t* goff, int groups,
                      int M, int q, Chart* recs, void* scratch, hipStream_t st) {
  if (M <= 0) return TABI_OK;
  Params P = make_params(groups, M, q, 0, 1, 0, 1, 1);
  Work W{};
  W.recs = recs;
  W.keys = static_cast<uint64_t*>(scratch);
  W.chart_atlas = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(scratch) +
                                             align_up((size_t)M * 8, 256));
  W.desc = nullptr;  // no atlas descriptors, no ranks
  const hipError_t e = launch_prep(P, W, xy, voff, goff, nullptr, 0, 0, st);
  return e == hipSuccess ? TABI_OK : hip_fail(e);
}

int host_hip_fail(hipError_t e) { return hip_fail(e); }

}  // namespace tabi

extern "C" {

int tabi_pack(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
              int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
              float* out_scale, tabi_stream_t stream) {
  if (quality < 0 || quality > 2) return TABI_EINVAL;
  return pack_single(charts, n, atlas_w, atlas_h, padding, quality, out_xy, out_orient, out_scale,
                     stream);
}

int tabi_pack_loops(const tabi_charts_loops* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                    int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
                    float* out_scale, tabi_stream_t stream) {
  if (quality < 0 || quality > 2 || !charts || charts->total_loops < 0 ||
      (n > 0 && (!charts->xy || !charts->loop_offsets || !charts->chart_loops)))
    return TABI_EINVAL;
  // the loops' vertex offsets stand where the charts' would, and the chart
  // -> loops table tells the proxy kernel which loops make a chart
  const tabi_charts as_charts{charts->xy, charts->loop_offsets, 0};
  return pack_single(&as_charts, n, atlas_w, atlas_h, padding, quality, out_xy, out_orient,
                     out_scale, stream, charts->chart_loops);
}

int tabi_pack_method(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, const tabi_method* method, int32_t* out_xy,
                     uint8_t* out_orient, float* out_scale, tabi_stream_t stream) {
  if (!method_ok(method)) return TABI_EINVAL;
  return pack_single(charts, n, atlas_w, atlas_h, padding, encode_method(*method), out_xy,
                     out_orient, out_scale, stream);
}

int tabi_pack_hybrid(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, const tabi_method* method, int32_t* out_xy,
                     uint8_t* out_orient, float* out_chart_scale, float* out_scale,
                     tabi_stream_t stream) {
  if (!method_ok(method) || method->variant != TABI_FULL) return TABI_EINVAL;
  const int32_t code = encode_method(*method);
  if (check_common_code(n, padding, code) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !out_scale ||
      (n > 0 && (!charts->xy || !charts->offsets || !out_xy || !out_orient || !out_chart_scale)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Params P = make_params(1, n, code, padding, 64, 0, n > 0 ? n : 1, atlas_w + padding);
  P.hybrid = 1;
  Job j;
  int rc = make_job(j, P, st);
  if (!rc) rc = single_front(j, charts, atlas_w, atlas_h, st);
  if (!rc) {
    // every scale in one round: per-scale set-up, profiles and pairs, the
    // rows before the t_opt switch, the tails, then the choice
    hipError_t e;
    {
      StageScope t(ST_SETUP, st);
      e = launch_setup(j.P, j.W, 0, st);
    }
    if (e == hipSuccess) {
      StageScope t(ST_PROFILE, st);
      e = launch_profiles(j.P, j.W, 0, st);
    }
    if (e == hipSuccess) {
      StageScope t(ST_PACK, st);
      e = launch_pack(j.P, j.W, 0, j.L.bytes, j.L.RC, j.L.PW, j.stage_cap, 1, out_xy, out_orient,
                      out_scale, st);
      if (e == hipSuccess) e = launch_tail(j.P, j.W, j.L.bytes, j.L.RC, j.L.PW, st);
    }
    if (e == hipSuccess) {
      StageScope t(ST_SELECT, st);
      e = launch_select_hybrid(j.P, j.W, out_xy, out_orient, out_chart_scale, out_scale, st);
    }
    if (e != hipSuccess) rc = hip_fail(e);
  }
  free_job(j, st);
  return rc;
}

int tabi_pack_prerotate(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                        int32_t padding, int32_t quality, int32_t* out_rxy, uint8_t* out_dir,
                        int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                        tabi_stream_t stream) {
  if (check_common(n, padding, quality) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !out_scale ||
      (n > 0 && (!charts->xy || !charts->offsets || !out_rxy || !out_dir || !out_xy ||
                 !out_orient)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = launch_prerotate(charts->xy, charts->offsets, n, out_rxy, out_dir, st);
  if (e != hipSuccess) return hip_fail(e);
  // the turned charts are packed like any other input
  const tabi_charts turned{out_rxy, charts->offsets, charts->total_verts};
  return pack_single(&turned, n, atlas_w, atlas_h, padding, quality, out_xy, out_orient,
                     out_scale, stream);
}

int tabi_pack_noalloc(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                      int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
                      float* out_scale, tabi_stream_t stream) {
  if (check_common(n, padding, quality) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !out_scale || (n > 0 && (!charts->xy || !charts->offsets || !out_xy || !out_orient)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the same plan as tabi_pack; the profile arena takes what the fixed
  // arrays leave of the static work space (segments beyond it are evaluated
  // from the proxy records, with the same results)
  Params P = make_params(1, n, quality, padding, 64, 0, n > 0 ? n : 1, atlas_w + padding);
  const int64_t want = P.arena_cap;
  P.arena_cap = 0;
  const size_t fixed = layout(P).total;
  if (fixed > kScratchBytes) return TABI_ETOOBIG;
  P.arena_cap = std::min<int64_t>(want, (int64_t)((kScratchBytes - fixed) / 4));
  if (layout(P).total > kScratchBytes) P.arena_cap = 0;  // alignment slack
  void* ws = scratch_ptr();
  if (!ws) return TABI_EHIP;
  Job j;
  int rc = make_job(j, P, st, ws, kScratchBytes);
  if (!rc) rc = single_front(j, charts, atlas_w, atlas_h, st);
  if (!rc) {
    const int all[1] = {64};
    hipError_t e = run_search(j, all, 1, out_xy, out_orient, out_scale, st);
    if (e != hipSuccess) rc = hip_fail(e);
  }
  return rc;  // nothing to release: the work space is the static array
}

int tabi_pack_many(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                   int32_t count, const int32_t* atlas_wh, int32_t total_charts,
                   int32_t max_charts, int32_t max_side, int32_t padding, int32_t quality,
                   int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                   tabi_stream_t stream) {
  if (quality < 0 || quality > 2) return TABI_EINVAL;
  return pack_many_impl(xy, vert_offsets, atlas_offsets, count, atlas_wh, total_charts, max_charts,
                        max_side, padding, quality, out_xy, out_orient, out_scale, nullptr, 0,
                        stream);
}

int tabi_pack_many_method(const int32_t* xy, const int32_t* vert_offsets,
                          const int32_t* atlas_offsets, int32_t count, const int32_t* atlas_wh,
                          int32_t total_charts, int32_t max_charts, int32_t max_side,
                          int32_t padding, const tabi_method* method, int32_t* out_xy,
                          uint8_t* out_orient, float* out_scale, tabi_stream_t stream) {
  if (!method_ok(method)) return TABI_EINVAL;
  return pack_many_impl(xy, vert_offsets, atlas_offsets, count, atlas_wh, total_charts, max_charts,
                        max_side, padding, encode_method(*method), out_xy, out_orient, out_scale,
                        nullptr, 0, stream);
}

int tabi_tune_many(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                   int32_t count, const int32_t* atlas_wh, int32_t total_charts,
                   int32_t max_charts, int32_t max_side, int32_t padding, int32_t quality,
                   int32_t* out_xy, uint8_t* out_orient, float* out_scale, int32_t reps,
                   int32_t* shape, float* ms_per_shape, tabi_stream_t stream) {
  if (quality < 0 || quality > 2) return TABI_EINVAL;
  int rc = many_check(xy, vert_offsets, atlas_offsets, count, atlas_wh, total_charts, max_charts,
                      max_side, padding, quality, out_xy, out_orient, out_scale);
  if (rc) return rc;
  if (count == 0 || reps < 1) return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e);
  int best = -1;
  float best_ms = 0.f;
  for (int i = 0; i < kNumManyShapes && rc == TABI_OK; ++i) {
    set_many_shape(quality, shape_class(count), i);
    // one untimed call (pool growth, first launches), then reps timed ones
    rc = pack_many_impl(xy, vert_offsets, atlas_offsets, count, atlas_wh, total_charts, max_charts,
                        max_side, padding, quality, out_xy, out_orient, out_scale, nullptr, 0,
                        stream);
    if (rc == TABI_EINVAL) {  // this shape cannot hold the batch's rows; skip it
      rc = TABI_OK;
      if (ms_per_shape) ms_per_shape[i] = -1.f;
      continue;
    }
    if (rc) break;
    e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && rc == TABI_OK && e == hipSuccess; ++r)
      rc = pack_many_impl(xy, vert_offsets, atlas_offsets, count, atlas_wh, total_charts,
                          max_charts, max_side, padding, quality, out_xy, out_orient, out_scale,
                          nullptr, 0, stream);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { rc = hip_fail(e); break; }
    ms /= (float)reps;
    if (ms_per_shape) ms_per_shape[i] = ms;
    if (best < 0 || ms < best_ms) { best = i; best_ms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_many_shape(quality, shape_class(count), best >= 0 ? best : 0);
  if (rc == TABI_OK && best < 0) rc = TABI_EINVAL;
  if (rc == TABI_OK && shape) {
    const ManyShape& b = kManyShapes[best];
    shape[0] = b.b0; shape[1] = b.flat; shape[2] = b.bmax; shape[3] = b.nt; shape[4] = b.cap;
  }
  return rc;
}

int tabi_many_shape(int32_t quality, int32_t count, int32_t* shape) {
  if (!shape || quality < 0 || quality > 2 || count < 0) return TABI_EINVAL;
  const ManyShape sh = many_shape(quality, count);
  shape[0] = sh.b0; shape[1] = sh.flat; shape[2] = sh.bmax; shape[3] = sh.nt; shape[4] = sh.cap;
  return TABI_OK;
}

int32_t tabi_many_shape_count(void) { return kNumManyShapes; }

int tabi_debug_set_many_shape(int32_t quality, int32_t index) {
  if (quality < 0 || quality > 2 || index >= kNumManyShapes) return TABI_EINVAL;
  set_many_shape(quality, -1, index < 0 ? 0 : index);
  return TABI_OK;
}

int64_t tabi_pack_many_workspace_bytes(int32_t count, int32_t total_charts, int32_t max_charts,
                                       int32_t max_side, int32_t padding, int32_t quality) {
  if (count < 0 || total_charts < 0 || max_side < 1 || quality < 0 || quality > 2 || padding < 0 ||
      padding > TABI_MAX_PADDING)
    return -1;
  return (int64_t)layout(many_params(count, total_charts, max_charts, max_side, padding, quality))
      .total;
}

int tabi_pack_many_ws(const int32_t* xy, const int32_t* vert_offsets,
                      const int32_t* atlas_offsets, int32_t count, const int32_t* atlas_wh,
                      int32_t total_charts, int32_t max_charts, int32_t max_side,
                      int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
                      float* out_scale, void* workspace, int64_t workspace_bytes,
                      tabi_stream_t stream) {
  if (quality < 0 || quality > 2) return TABI_EINVAL;
  if (!workspace || workspace_bytes <= 0) return TABI_EINVAL;
  return pack_many_impl(xy, vert_offsets, atlas_offsets, count, atlas_wh, total_charts, max_charts,
                        max_side, padding, quality, out_xy, out_orient, out_scale, workspace,
                        (size_t)workspace_bytes, stream);
}

int64_t tabi_record_bytes(void) { return (int64_t)sizeof(Chart); }

int tabi_prep_records(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                      int32_t count, int32_t total_charts, int32_t quality, void* records,
                      tabi_stream_t stream) {
  if (count < 1 || total_charts < 0 || quality < 0 || quality > 2 || !atlas_offsets ||
      (total_charts > 0 && (!xy || !vert_offsets || !records)))
    return TABI_EINVAL;
  if (total_charts == 0) return TABI_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  void* scratch = nullptr;
  hipError_t e = hipMallocAsync(&scratch, host_prep_scratch_bytes(total_charts), st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? TABI_ENOMEM : hip_fail(e);
  }
  const int rc = host_prep_records(xy, vert_offsets, atlas_offsets, count, total_charts, quality,
                                   static_cast<Chart*>(records), scratch, st);
  (void)hipFreeAsync(scratch, st);
  return rc;
}

int tabi_splice_records(void* records, const int32_t* index, int32_t m, const void* new_records,
                        tabi_stream_t stream) {
  if (m < 0 || (m > 0 && (!records || !index || !new_records))) return TABI_EINVAL;
  hipError_t e = launch_splice(static_cast<Chart*>(records), index, m,
                               static_cast<const Chart*>(new_records),
                               reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? TABI_OK : hip_fail(e);
}

int tabi_pack_many_records(const void* records, const int32_t* atlas_offsets, int32_t count,
                           const int32_t* atlas_wh, int32_t total_charts, int32_t max_charts,
                           int32_t max_side, int32_t padding, int32_t quality, int32_t* out_xy,
                           uint8_t* out_orient, float* out_scale, tabi_stream_t stream) {
  if (quality < 0 || quality > 2) return TABI_EINVAL;
  if (total_charts > 0 && !records) return TABI_EINVAL;
  return pack_many_impl(nullptr, nullptr, atlas_offsets, count, atlas_wh, total_charts, max_charts,
                        max_side, padding, quality, out_xy, out_orient, out_scale, nullptr, 0,
                        stream, records ? records : atlas_offsets);
}

int tabi_debug_order(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, int32_t quality, int32_t* perm, int32_t* khi,
                     tabi_stream_t stream) {
  if (check_common(n, padding, quality) || bad_atlas(atlas_w, atlas_h, padding) || !charts ||
      !khi || (n > 0 && (!charts->xy || !charts->offsets || !perm)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  int rc = make_job(j, make_params(1, n, quality, padding, 1, 0, n > 0 ? n : 1, atlas_w + padding),
                    st);
  if (!rc) rc = single_front(j, charts, atlas_w, atlas_h, st);
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
  if (check_common(n, padding, quality) || k < 1 || k > 64 || !charts || padding >= 16384 ||
      (n > 0 && (!charts->xy || !charts->offsets || !cd || !flags)))
    return TABI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Job j;
  int rc = make_job(j, make_params(1, n, quality, padding, 1, k, n > 0 ? n : 1, 1 + padding), st);
  if (!rc) rc = single_front(j, charts, 16384 - padding, 16384 - padding, st);
  hipError_t e = hipSuccess;
  if (!rc) e = launch_setup(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess) e = launch_profiles(j.P, j.W, 0, st);
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
  int rc = make_job(j, make_params(1, n, quality, padding, 1, k, n > 0 ? n : 1, atlas_w + padding),
                    st);
  if (!rc) rc = single_front(j, charts, atlas_w, atlas_h, st);
  hipError_t e = hipSuccess;
  if (!rc) e = launch_setup(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess) e = launch_profiles(j.P, j.W, 0, st);
  if (!rc && e == hipSuccess)
    e = launch_pack(j.P, j.W, 0, j.L.bytes, j.L.RC, j.L.PW, j.stage_cap, 1, nullptr, nullptr,
                    nullptr, st);
  if (!rc && e == hipSuccess) e = launch_scatter(j.P, j.W, out_xy, out_orient, feasible, rows, st);
  if (!rc && e != hipSuccess) rc = hip_fail(e);
  free_job(j, st);
  return rc;
}

int tabi_shutdown(void) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  hipMemPool_t pool;
  if (e == hipSuccess) e = hipDeviceGetDefaultMemPool(&pool, dev);
  if (e == hipSuccess) e = hipMemPoolTrimTo(pool, 0);
  return e == hipSuccess ? TABI_OK : hip_fail(e);
}

const char* tabi_strerror(int code) {
  switch (code) {
    case TABI_OK: return "ok";
    case TABI_EINVAL: return "invalid argument";
    case TABI_ENOMEM: return "out of device memory";
    case TABI_EHIP: return "HIP runtime error";
    case TABI_ETOOBIG:
      return "input needs more work space than tabi_pack_noalloc's static array holds";
    default: return "unknown error";
  }
}

const char* tabi_last_hip_error(void) { return g_last_hip; }

int tabi_debug_phase_clock(int64_t* out, int32_t slots) {
  if (!out || slots < 1) return TABI_EINVAL;
  const int r = read_phase_clock(out, slots);
  if (r == -2) return TABI_EINVAL;
  return r < 0 ? hip_fail(hipGetLastError()) : r;
}

int tabi_debug_set_pack_lds(int32_t bytes) {
  g_pack_lds = bytes < 0 ? -1 : bytes;
  return TABI_OK;
}

int tabi_debug_set_stage_cap(int32_t entries) {
  g_stage_cap = entries;
  return TABI_OK;
}

int tabi_debug_set_profile_cap(int64_t words) {
  g_profile_cap = words < 0 ? -1 : (words > 0x7fffffffLL ? 0x7fffffffLL : words);
  return TABI_OK;
}

int tabi_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  g_timing.on = on != 0;
  return TABI_OK;
}

int tabi_timing_stages(uint32_t mask) {
  if (mask == 0 || (mask >> ST_COUNT) != 0) return TABI_EINVAL;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  g_timing.mask = mask;
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
  tabi_timing_read(nullptr, nullptr, 0);
  std::lock_guard<std::mutex> lk(g_timing.mu);
  for (int i = 0; i < ST_COUNT; ++i) {
    g_timing.ms[i] = 0;
    g_timing.launches[i] = 0;
  }
}

int64_t tabi_pack_lds_bytes(int32_t n, int32_t atlas_w, int32_t padding) {
  const int budget = lds_budget();  // also reads the kernel's static size
  PackLds L = pack_lds_plan(n, atlas_w + padding, budget - kPackStaticLds);
  return (int64_t)L.bytes + kPackStaticLds;
}

}  // extern "C"
