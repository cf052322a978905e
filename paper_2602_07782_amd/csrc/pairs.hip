// Horizontal compacting distance and interlock flags of sorted neighbours
// (Sec. 4.1.2 "Compacting Horizontal Gaps", App. A "Detecting Interlocking
// Charts"), one wavefront per (scale slot, pair).  Lanes walk the rows of the
// two charts' grown row profiles: the compacting distance is a min-reduction,
// the interlock tests are prefix max / prefix min scans.
#include "tabi_internal.h"
#include "pairs_dev.h"

namespace tabi {

constexpr int PAIR_WAVES = 4;

__global__ __launch_bounds__(256) void k_pairs(Params P, Work w, int round) {
  const int wv = threadIdx.x / WAVE, lane = lane_id();
  const int c = blockIdx.x * PAIR_WAVES + wv;
  const int s = blockIdx.y;
  if (c >= P.N) return;
  const AtlasDesc d = w.desc[w.chart_atlas[c]];
  const size_t slot = (size_t)s * P.N;
  const bool run = P.fixed_k > 0 ? !d.bad : (!d.done && d.ktop >= 1);
  if (!run) return;
  const int k = slot_k(P, d, round, s);
  if (k < 1) return;
  if (c == d.c0) {
    if (lane == 0) { w.cd[slot + c] = 0; w.fl[slot + c] = 0; }
    return;
  }
  const int K = P.K, p = P.p;
  const KView A = kview(w.kc + (slot + c - 1) * P.stride, K);
  const KView B = kview(w.kc + (slot + c) * P.stride, K);
  const Chart& cA = w.srecs[c - 1];
  const Chart& cB = w.srecs[c];
  const int hdA = A.hd->h + p, hdB = B.hd->h + p, wdA = A.hd->w + p;
  const int rows = min(hdA, hdB);
  // compacting distance: min over shared rows of (w'A - RightA(j) + LeftB(j))
  int32_t cdv = BIG;
  for (int j0 = 0; j0 < rows; j0 += WAVE) {
    const int j = j0 + lane;
    if (j < rows) {
      int32_t la, ra, lb, rb;
      row_bounds_grown(A, cA, K, k, p, j, la, ra);
      row_bounds_grown(B, cB, K, k, p, j, lb, rb);
      cdv = min(cdv, wdA - ra + lb);
    }
  }
  cdv = wave_min(cdv);
  const int32_t fl = pair_flags(A, cA, B, cB, K, k, p, wdA - cdv);
  if (lane == 0) {
    w.cd[slot + c] = cdv;
    w.fl[slot + c] = (uint8_t)fl;
  }
}

hipError_t launch_pairs(const Params& P, const Work& w, int round, hipStream_t st) {
  if (P.N > 0)
    hipLaunchKernelGGL(k_pairs, dim3((P.N + PAIR_WAVES - 1) / PAIR_WAVES, P.B), dim3(256), 0, st,
                       P, w, round);
  return hipGetLastError();
}

}  // namespace tabi
