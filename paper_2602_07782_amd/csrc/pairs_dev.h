// Compacting distance and interlock thresholds of two charts of a row, in
// wavefront-cooperative sweeps over the rows.
//
// A chart's grown rows are stored per proxy (profile arena): its local-AABB
// rows, then its OBB rows, hd words each, a word holding the grown left
// bound L' (low half) and the grown right bound R' (high half, gutter
// included).  Sorted neighbours are compacted by the larger of the two
// proxies' distances and take their interlock flags from the proxy that gave
// it (Sec. 4.1.2; App. A, "Detecting Interlocking Charts"); other pairs of a
// row that share columns are tested on the rows both proxies allow (per
// grown row, the intersection of the two proxies' spans).
#pragma once

#include "tabi_device.h"

namespace tabi {

struct PairSweep {
  int32_t cd;  // horizontal compacting distance
  int32_t D1;  // B may not move above A exactly when its box offset d < D1
  int32_t D2;  // A may not move above B exactly when d < D2
};

// With R'A / L'B the grown right / left row bounds of one proxy of A and of
// B (B, later in sorted order, is at most as tall):
//   cd = min over shared rows j of (w'A - R'A(j) + L'B(j));
//   B rising by 1..j texels brings row j of B beside rows above j of A, so
//   B may not rise iff some j >= 1 has d + L'B(j) < max_{j'<j} R'A(j'),
//   i.e. iff d < D1 = max_j (max_{j'<j} R'A(j') - L'B(j));
//   symmetrically A may not rise iff d < D2 = max_j (R'A(j) - min_{j'<j} L'B(j')).
// SweepState is the running state of one such sweep in chunks of rows.
struct SweepState {
  int32_t cd, D1, D2, cmax, cmin;
};
__device__ inline SweepState sweep_start() { return {BIG, -BIG, -BIG, -BIG, BIG}; }

// Lane moves within 16-lane rows (four independent sweeps per wavefront).
constexpr int DPP_ROW_ROR1 = 0x121, DPP_ROW_ROR2 = 0x122, DPP_ROW_ROR4 = 0x124,
              DPP_ROW_ROR8 = 0x128;
__device__ inline int32_t row_last(int32_t v) {  // lane 15 of the caller's row
  const int g = lane_id() >> 4;
  const int32_t a = __builtin_amdgcn_readlane(v, 15), b = __builtin_amdgcn_readlane(v, 31);
  const int32_t c = __builtin_amdgcn_readlane(v, 47), d = __builtin_amdgcn_readlane(v, 63);
  return g == 0 ? a : (g == 1 ? b : (g == 2 ? c : d));
}
__device__ inline int32_t row_all_max(int32_t v) {
  v = max(v, dpp_move<DPP_ROW_ROR8>(v, -BIG));
  v = max(v, dpp_move<DPP_ROW_ROR4>(v, -BIG));
  v = max(v, dpp_move<DPP_ROW_ROR2>(v, -BIG));
  return max(v, dpp_move<DPP_ROW_ROR1>(v, -BIG));
}
__device__ inline int32_t row_all_min(int32_t v) {
  v = min(v, dpp_move<DPP_ROW_ROR8>(v, BIG));
  v = min(v, dpp_move<DPP_ROW_ROR4>(v, BIG));
  v = min(v, dpp_move<DPP_ROW_ROR2>(v, BIG));
  return min(v, dpp_move<DPP_ROW_ROR1>(v, BIG));
}

// One chunk: each lane holds grown row j of A (Ra, when act) and of B (Lb,
// when shr: j < both heights).  ROW16: the chunk is 16 rows per 16-lane row
// of the wavefront, four sweeps side by side; otherwise 64 consecutive rows
// of one sweep.  Every lane of the wavefront must call it.
template <bool ROW16>
__device__ inline void sweep_chunk(SweepState& s, int32_t Ra, int32_t Lb, bool act, bool shr,
                                   int j, int wdA) {
  Ra = act ? Ra : -BIG;
  Lb = shr ? Lb : BIG;
  if (shr) s.cd = min(s.cd, wdA - Ra + Lb);
  int32_t emax, emin;
  if constexpr (ROW16) {
    int32_t imax = Ra, imin = Lb;
    imax = max(imax, dpp_move<DPP_ROW_SHR1>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR1>(imin, BIG));
    imax = max(imax, dpp_move<DPP_ROW_SHR2>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR2>(imin, BIG));
    imax = max(imax, dpp_move<DPP_ROW_SHR4>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR4>(imin, BIG));
    imax = max(imax, dpp_move<DPP_ROW_SHR8>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR8>(imin, BIG));
    emax = max(dpp_move<DPP_ROW_SHR1>(imax, -BIG), s.cmax);
    emin = min(dpp_move<DPP_ROW_SHR1>(imin, BIG), s.cmin);
    s.cmax = max(s.cmax, row_last(imax));
    s.cmin = min(s.cmin, row_last(imin));
  } else {
    const int32_t imax = wave_incl_max(Ra), imin = wave_incl_min(Lb);
    emax = max(wave_shr1(imax, -BIG), s.cmax);
    emin = min(wave_shr1(imin, BIG), s.cmin);
    s.cmax = max(s.cmax, lane63(imax));
    s.cmin = min(s.cmin, lane63(imin));
  }
  if (shr && j >= 1) s.D1 = max(s.D1, emax - Lb);
  if (act && j >= 1) s.D2 = max(s.D2, Ra - emin);
}
template <bool ROW16>
__device__ inline PairSweep sweep_end(const SweepState& s) {
  PairSweep r;
  if constexpr (ROW16) {
    r.cd = row_all_min(s.cd);
    r.D1 = row_all_max(s.D1);
    r.D2 = row_all_max(s.D2);
  } else {
    r.cd = wave_min(s.cd);
    r.D1 = wave_max(s.D1);
    r.D2 = wave_max(s.D2);
  }
  return r;
}

// Interlock flags for box offset d (bit0: B may not move above A, bit1: A may
// not move above B); none without a shared column.
__device__ inline int32_t pair_flags_at(const PairSweep& s, int wdA, int d) {
  if (d >= wdA) return 0;
  return (d < s.D1 ? 1 : 0) | (d < s.D2 ? 2 : 0);
}

// A neighbour pair from its two proxies' sweeps: the larger distance (the
// local AABBs' on a tie) and the flags of the proxy that gave it.
struct PairResult {
  int32_t cd, flags;
};
__device__ inline PairResult pair_pick(const PairSweep& sa, const PairSweep& so, int wdA) {
  const bool obb = so.cd > sa.cd;
  PairResult r;
  r.cd = obb ? so.cd : sa.cd;
  r.flags = pair_flags_at(obb ? so : sa, wdA, wdA - r.cd);
  return r;
}

// A neighbour pair (A, B) over stored grown rows: ra, rb point at the
// charts' local-AABB rows (their OBB rows follow after hd words).  ROW16:
// four pairs per wavefront, one per 16-lane row; a row without a pair passes
// hdA = 0; results hold in every lane of the row.  Otherwise one pair over
// the whole wavefront.
template <bool ROW16>
__device__ inline PairResult pair_rows_both(const uint32_t* ra, int hdA, const uint32_t* rb,
                                            int hdB, int wdA) {
  constexpr int STEP = ROW16 ? 16 : WAVE;
  const int gl = ROW16 ? (lane_id() & 15) : lane_id();
  SweepState sa = sweep_start(), so = sweep_start();
  const int steps = ROW16 ? wave_max((hdA + 15) >> 4) : (hdA + WAVE - 1) / WAVE;
  for (int q = 0; q < steps; ++q) {
    const int j = q * STEP + gl;
    const bool act = j < hdA, shr = act && j < hdB;
    uint32_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    if (act) { a0 = ra[j]; a1 = ra[hdA + j]; }
    if (shr) { b0 = rb[j]; b1 = rb[hdB + j]; }
    sweep_chunk<ROW16>(sa, hi16(a0), lo16(b0), act, shr, j, wdA);
    sweep_chunk<ROW16>(so, hi16(a1), lo16(b1), act, shr, j, wdA);
  }
  return pair_pick(sweep_end<ROW16>(sa), sweep_end<ROW16>(so), wdA);
}

// A pair that is not a neighbour pair, over stored grown rows (one
// wavefront): the intersection of the two proxies' rows.
__device__ inline PairSweep pair_rows_meet(const uint32_t* ra, int hdA, const uint32_t* rb,
                                           int hdB, int wdA) {
  const int lane = lane_id();
  SweepState s = sweep_start();
  for (int j0 = 0; j0 < hdA; j0 += WAVE) {
    const int j = j0 + lane;
    const bool act = j < hdA, shr = act && j < hdB;
    int32_t Ra = -BIG, Lb = BIG;
    if (act) Ra = min(hi16(ra[j]), hi16(ra[hdA + j]));
    if (shr) Lb = max(lo16(rb[j]), lo16(rb[hdB + j]));
    sweep_chunk<false>(s, Ra, Lb, act, shr, j, wdA);
  }
  return sweep_end<false>(s);
}

// The same sweeps from the proxy records, when the rows are not stored (one
// wavefront; every lane must call with the same arguments).  Each lane
// evaluates one undilated row of each chart; the gutter growth over rows
// [j-p, j] comes from p lane moves, so a chunk advances 64 - p rows.
// ROWS: 0 the local-AABB rows, 1 the OBB rows, 2 their intersection.
template <int ROWS>
__device__ inline PairSweep pair_records_sweep(const KView& A, const Chart& cA, const KView& B,
                                               const Chart& cB, int K, int k, int p) {
  const int lane = lane_id();
  const int hA = A.hd->h, hB = B.hd->h, wdA = A.hd->w + p;
  const int hdA = hA + p, hdB = hB + p;
  SweepState st = sweep_start();
  const int step = WAVE - p;
  for (int j0 = 0; j0 < hdA; j0 += step) {
    const int u = j0 - p + lane;  // undilated row held by this lane
    int32_t raa = -BIG, rao = -BIG, lba = BIG, lbo = BIG;
    if (u >= 0 && u < hA) {
      int32_t l1, l2;
      row_proxies(A, cA, K, k, u, l1, raa, l2, rao);
    }
    if (u >= 0 && u < hB) {
      int32_t r1, r2;
      row_proxies(B, cB, K, k, u, lba, r1, lbo, r2);
    }
    // each proxy's rows grow on their own (lanes >= p see rows [u-p, u] of
    // this chunk); the intersection is taken of the grown rows
    int32_t ra = ROWS == 1 ? rao : raa, lb = ROWS == 1 ? lbo : lba;
    int32_t Ra = ra, Lb = lb, Ro = rao, Lo = lbo;
    for (int s = 1; s <= p; ++s) {
      ra = wave_shr1(ra, -BIG);
      lb = wave_shr1(lb, BIG);
      Ra = max(Ra, ra);
      Lb = min(Lb, lb);
      if constexpr (ROWS == 2) {
        rao = wave_shr1(rao, -BIG);
        lbo = wave_shr1(lbo, BIG);
        Ro = max(Ro, rao);
        Lo = min(Lo, lbo);
      }
    }
    if constexpr (ROWS == 2) {
      Ra = min(Ra, Ro);
      Lb = max(Lb, Lo);
    }
    const int j = u;  // grown row j = lanes [j-p, j] of this chunk
    const bool act = lane >= p && j < hdA, shr = act && j < hdB;
    sweep_chunk<false>(st, Ra + p, Lb, act, shr, j, wdA);
  }
  return sweep_end<false>(st);
}

// A neighbour pair from the proxy records: both proxies' sweeps in one pass
// over the rows (each row of each chart evaluated once), the larger distance.
__device__ inline PairResult pair_records_both(const KView& A, const Chart& cA, const KView& B,
                                               const Chart& cB, int K, int k, int p) {
  const int lane = lane_id();
  const int hA = A.hd->h, hB = B.hd->h, wdA = A.hd->w + p;
  const int hdA = hA + p, hdB = hB + p;
  SweepState sa = sweep_start(), so = sweep_start();
  const int step = WAVE - p;
  for (int j0 = 0; j0 < hdA; j0 += step) {
    const int u = j0 - p + lane;  // undilated row held by this lane
    int32_t raa = -BIG, rao = -BIG, lba = BIG, lbo = BIG;
    if (u >= 0 && u < hA) {
      int32_t l1, l2;
      row_proxies(A, cA, K, k, u, l1, raa, l2, rao);
    }
    if (u >= 0 && u < hB) {
      int32_t r1, r2;
      row_proxies(B, cB, K, k, u, lba, r1, lbo, r2);
    }
    int32_t Ra = raa, La = lba, Ro = rao, Lo = lbo;
    for (int s = 1; s <= p; ++s) {
      raa = wave_shr1(raa, -BIG);
      lba = wave_shr1(lba, BIG);
      rao = wave_shr1(rao, -BIG);
      lbo = wave_shr1(lbo, BIG);
      Ra = max(Ra, raa);
      La = min(La, lba);
      Ro = max(Ro, rao);
      Lo = min(Lo, lbo);
    }
    const int j = u;  // grown row j = lanes [j-p, j] of this chunk
    const bool act = lane >= p && j < hdA, shr = act && j < hdB;
    sweep_chunk<false>(sa, Ra + p, La, act, shr, j, wdA);
    sweep_chunk<false>(so, Ro + p, Lo, act, shr, j, wdA);
  }
  return pair_pick(sweep_end<false>(sa), sweep_end<false>(so), wdA);
}

}  // namespace tabi
