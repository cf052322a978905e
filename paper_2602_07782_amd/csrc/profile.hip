// Per-texel profiles of every chart at every candidate scale of a round.
//
// The pushing step compares, texel column by texel column, a chart's grown
// TopEdge against the frontline and scores its grown BottomEdge; the
// interlock test and the compacting distance compare grown left / right
// bounds row by row (App. A, "Parallel Pushing", "Detecting Interlocking
// Charts"; Sec. 4.1.2).  These bounds depend only on the chart and the scale,
// so they are evaluated once here, at full occupancy, instead of inside the
// sequential row loop:
//
//   k_layout   one workgroup per (atlas, scale slot): prefix sums of the
//              grown widths and heights, one allocation in the arena
//   k_profile  one wavefront per (scale slot, chart): every grown column
//              (top, bottom) and every grown row (left, right)
//
// Within a (atlas, slot) segment the charts' columns are stored back to back
// in sorted order, so the candidates of a row are one contiguous range and a
// row's texel e is word pcol[first chart] + e.  A segment that does not fit
// the arena gets no profiles (pcol = prow = -1) and its consumers evaluate
// the proxies directly; results are the same either way.
#include "tabi_internal.h"

namespace tabi {

constexpr int LAY_NT = 256;
constexpr int PROF_WAVES = 4;

__global__ __launch_bounds__(LAY_NT) void k_layout(Params P, Work w, int round) {
  __shared__ int64_t s_tot[LAY_NT / WAVE][2];
  __shared__ int64_t s_base;
  const int a = blockIdx.x, s = blockIdx.y;
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  const AtlasDesc d = w.desc[a];
  const bool run = P.fixed_k > 0 ? !d.bad : (!d.done && d.ktop >= 1);
  if (!run || d.n <= 0) return;
  const int k = slot_k(P, d, round, s);
  if (k < 1) return;
  const size_t slot = (size_t)s * P.N + d.c0;
  const int n = d.n, per = (n + LAY_NT - 1) / LAY_NT;
  const int t0 = min(n, tid * per), t1 = min(n, t0 + per);
  int64_t sw = 0, sh = 0;
  for (int t = t0; t < t1; ++t) {
    sw += w.wdv[slot + t];
    sh += w.hdv[slot + t];
  }
  // block-wide exclusive scans of both sums
  int64_t iw = sw, ih = sh;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t uw = __shfl_up((long long)iw, o), uh = __shfl_up((long long)ih, o);
    if (lane >= o) { iw += uw; ih += uh; }
  }
  if (lane == WAVE - 1) { s_tot[wv][0] = iw; s_tot[wv][1] = ih; }
  __syncthreads();
  int64_t pw = 0, ph = 0, tw = 0, th = 0;
#pragma unroll
  for (int q = 0; q < LAY_NT / WAVE; ++q) {
    if (q < wv) { pw += s_tot[q][0]; ph += s_tot[q][1]; }
    tw += s_tot[q][0];
    th += s_tot[q][1];
  }
  if (tid == 0) {
    // claim [base, base + need) only if it fits: the counter never passes
    // the capacity, so a large segment that fails leaves room for others
    const unsigned long long need = (unsigned long long)(tw + th);
    const unsigned long long cap = (unsigned long long)P.arena_cap;
    long long base = -1;
    unsigned long long cur = atomicAdd(w.atop, 0ull);
    while (need <= cap && cur <= cap - need) {
      const unsigned long long old = atomicCAS(w.atop, cur, cur + need);
      if (old == cur) { base = (long long)cur; break; }
      cur = old;
    }
    s_base = base;
  }
  __syncthreads();
  const int64_t base = s_base;
  int64_t col = base + pw + iw - sw, row = base + tw + ph + ih - sh;
  for (int t = t0; t < t1; ++t) {
    w.pcol[slot + t] = base < 0 ? -1 : (int32_t)col;
    w.prow[slot + t] = base < 0 ? -1 : (int32_t)row;
    col += w.wdv[slot + t];
    row += w.hdv[slot + t];
  }
}

// Grown bounds of one chart, one wavefront.  Lane l of a chunk evaluates
// undilated column (row) u = j0 - p + l; the gutter growth over [u-p, u]
// comes from p shuffles, so a chunk advances 64 - p entries (p <= 32).
__global__ __launch_bounds__(PROF_WAVES * WAVE) void k_profile(Params P, Work w, int round) {
  const int wv = threadIdx.x / WAVE, lane = lane_id();
  const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * PROF_WAVES + wv);
  const int s = blockIdx.y;
  if (c >= P.N) return;
  const AtlasDesc d = w.desc[w.chart_atlas[c]];
  const bool run = P.fixed_k > 0 ? !d.bad : (!d.done && d.ktop >= 1);
  if (!run) return;
  const int k = slot_k(P, d, round, s);
  if (k < 1) return;
  const size_t sc = (size_t)s * P.N + c;
  const int32_t pc = w.pcol[sc], pr = w.prow[sc];
  if (pc < 0) return;
  const KView kv = kview(w.kc + sc * P.stride, P.K);
  const Chart& ch = w.srecs[c];
  const int K = P.K, p = P.p, wt = kv.hd->w, ht = kv.hd->h;
  const int step = WAVE - p;
  uint32_t* out = w.arena + pc;
  for (int j0 = 0; j0 < wt + p; j0 += step) {
    const int u = j0 - p + lane;
    int32_t tp = BIG, bt = -BIG;
    if (u >= 0 && u < wt) column_bounds(kv, ch, K, k, u, tp, bt);
    int32_t T = tp, Bo = bt;
    for (int q = 1; q <= p; ++q) {
      T = min(T, __shfl_up(tp, q));
      Bo = max(Bo, __shfl_up(bt, q));
    }
    if (lane >= p && u < wt + p) out[u] = pack16(T, Bo + p);
  }
  out = w.arena + pr;
  for (int j0 = 0; j0 < ht + p; j0 += step) {
    const int u = j0 - p + lane;
    int32_t l = BIG, r = -BIG;
    if (u >= 0 && u < ht) row_bounds(kv, ch, K, k, u, l, r);
    int32_t L = l, R = r;
    for (int q = 1; q <= p; ++q) {
      L = min(L, __shfl_up(l, q));
      R = max(R, __shfl_up(r, q));
    }
    if (lane >= p && u < ht + p) out[u] = pack16(L, R + p);
  }
}

hipError_t launch_profiles(const Params& P, const Work& w, int round, hipStream_t st) {
  if (P.N <= 0) return hipSuccess;
  // with no arena the layout still runs: it marks every segment unprofiled
  hipLaunchKernelGGL(k_layout, dim3(P.count, P.B), dim3(LAY_NT), 0, st, P, w, round);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || P.arena_cap <= 0) return e;
  hipLaunchKernelGGL(k_profile, dim3((P.N + PROF_WAVES - 1) / PROF_WAVES, P.B),
                     dim3(PROF_WAVES * WAVE), 0, st, P, w, round);
  return hipGetLastError();
}

}  // namespace tabi
