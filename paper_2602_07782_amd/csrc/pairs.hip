// Horizontal compacting distance and interlock flags of sorted neighbours
// (Sec. 4.1.2 "Compacting Horizontal Gaps", App. A "Detecting Interlocking
// Charts"), one wavefront per (scale slot, pair).  One sweep over the rows
// gives the compacting distance (a min-reduction) and both interlock
// thresholds (prefix max / prefix min scans), reading the stored grown rows
// of both charts; without stored profiles the two charts' proxy records are
// copied to LDS and the rows evaluated directly.
#include "tabi_internal.h"
#include "pairs_dev.h"

namespace tabi {

constexpr int PAIR_WAVES = 4;

struct alignas(16) PairCache {
  Chart ch[2];
  unsigned char kc[2][KREC_MAX];
};

__global__ __launch_bounds__(256) void k_pairs(Params P, Work w, int round) {
  __shared__ PairCache cache[PAIR_WAVES];  // used when the rows are not stored
  const int wv = threadIdx.x / WAVE, lane = lane_id();
  const int c = blockIdx.x * PAIR_WAVES + wv;
  const int s = blockIdx.y;
  if (c >= P.N) return;  // whole wavefront leaves; no block barrier below
  const int a = w.chart_atlas[c];
  const AtlasDesc d = w.desc[a];
  const size_t slot = (size_t)s * P.N;
  const bool run = P.fixed_k > 0 ? !d.bad : (!d.done && d.ktop >= 1);
  if (!run) return;
  const int k = slot_k(P, d, round, s);
  if (k < 1) return;
  if (c == d.c0) {
    if (lane == 0) { w.cd[slot + c] = 0; w.fl[slot + c] = 0; }
    return;
  }
  const int32_t base = w.segbase[(size_t)a * P.B + s];
  if (base >= 0) {  // stored grown rows
    const int32_t prA = base + w.prow[slot + c - 1], prB = base + w.prow[slot + c];
    const int wdA = w.wdv[slot + c - 1];
    const PairSweep r = pair_sweep_rows(w.arena + prA, w.hdv[slot + c - 1], w.arena + prB,
                                        w.hdv[slot + c], wdA);
    if (lane == 0) {
      w.cd[slot + c] = r.cd;
      w.fl[slot + c] = (uint8_t)pair_flags_at(r, wdA, wdA - r.cd);
    }
    return;
  }
  const int K = P.K, p = P.p, stride = P.stride;
  // stage both charts (records of chart c-1 and c) in LDS
  {
    const int nch = (int)(sizeof(Chart) / 16), nkc = stride / 16;
    const int4* srcA = reinterpret_cast<const int4*>(&w.srecs[c - 1]);
    const int4* srcB = reinterpret_cast<const int4*>(&w.srecs[c]);
    const int4* kcA = reinterpret_cast<const int4*>(w.kc + (slot + c - 1) * stride);
    const int4* kcB = reinterpret_cast<const int4*>(w.kc + (slot + c) * stride);
    int4* dch = reinterpret_cast<int4*>(cache[wv].ch);
    int4* dk0 = reinterpret_cast<int4*>(cache[wv].kc[0]);
    int4* dk1 = reinterpret_cast<int4*>(cache[wv].kc[1]);
    for (int i = lane; i < 2 * nch + 2 * nkc; i += WAVE) {
      if (i < nch) dch[i] = srcA[i];
      else if (i < 2 * nch) dch[i] = srcB[i - nch];
      else if (i < 2 * nch + nkc) dk0[i - 2 * nch] = kcA[i - 2 * nch];
      else dk1[i - 2 * nch - nkc] = kcB[i - 2 * nch - nkc];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const KView A = kview(cache[wv].kc[0], K);
  const KView B = kview(cache[wv].kc[1], K);
  const PairSweep r = pair_sweep(A, cache[wv].ch[0], B, cache[wv].ch[1], K, k, p);
  const int wdA = A.hd->w + p;
  if (lane == 0) {
    w.cd[slot + c] = r.cd;
    w.fl[slot + c] = (uint8_t)pair_flags_at(r, wdA, wdA - r.cd);
  }
}

hipError_t launch_pairs(const Params& P, const Work& w, int round, hipStream_t st) {
  if (P.N > 0)
    hipLaunchKernelGGL(k_pairs, dim3((P.N + PAIR_WAVES - 1) / PAIR_WAVES, P.B), dim3(256), 0, st,
                       P, w, round);
  return hipGetLastError();
}

}  // namespace tabi
