// Compacting distance and interlock thresholds of two charts of a row, in
// one wavefront-cooperative sweep over the rows.
#pragma once

#include "tabi_device.h"

namespace tabi {

struct PairSweep {
  int32_t cd;  // horizontal compacting distance (Sec. 4.1.2)
  int32_t D1;  // B may not move above A exactly when its box offset d < D1
  int32_t D2;  // A may not move above B exactly when d < D2
};

// One pass over the grown rows of A (B, later in sorted order, is at most as
// tall).  With R'A / L'B the grown right / left row bounds:
//   cd = min over shared rows j of (w'A - R'A(j) + L'B(j));
//   B rising by 1..j texels brings row j of B beside rows above j of A, so
//   B may not rise iff some j >= 1 has d + L'B(j) < max_{j'<j} R'A(j'),
//   i.e. iff d < D1 = max_j (max_{j'<j} R'A(j') - L'B(j));
//   symmetrically A may not rise iff d < D2 = max_j (R'A(j) - min_{j'<j} L'B(j'))
// (App. A, "Detecting Interlocking Charts").  Each lane evaluates one
// undilated row of each chart; the gutter growth over rows [j-p, j] comes
// from p shuffles, so a chunk advances 64 - p rows.  All lanes of the
// wavefront must call this with the same arguments.
__device__ inline PairSweep pair_sweep(const KView& A, const Chart& cA, const KView& B,
                                       const Chart& cB, int K, int k, int p) {
  const int lane = lane_id();
  const int hA = A.hd->h, hB = B.hd->h, wdA = A.hd->w + p;
  const int hdA = hA + p, hdB = hB + p;
  int32_t cd = BIG, D1 = -BIG, D2 = -BIG;
  int32_t carry_max = -BIG, carry_min = BIG;
  const int step = WAVE - p;
  for (int j0 = 0; j0 < hdA; j0 += step) {
    const int u = j0 - p + lane;  // undilated row held by this lane
    int32_t ra = -BIG, lb = BIG;
    if (u >= 0 && u < hA) {
      int32_t l, r;
      row_bounds(A, cA, K, k, u, l, r);
      ra = r;
    }
    if (u >= 0 && u < hB) {
      int32_t l, r;
      row_bounds(B, cB, K, k, u, l, r);
      lb = l;
    }
    int32_t Ra = ra, Lb = lb, sa = ra, sb = lb;
    for (int s = 1; s <= p; ++s) {  // lanes >= p see rows [u-p, u] of this chunk
      sa = wave_shr1(sa, -BIG);
      sb = wave_shr1(sb, BIG);
      Ra = max(Ra, sa);
      Lb = min(Lb, sb);
    }
    const int j = u;  // grown row j = lanes [j-p, j] of this chunk
    const bool act = lane >= p && j < hdA;
    Ra = act ? Ra + p : -BIG;
    Lb = (act && j < hdB) ? Lb : BIG;
    if (act && j < hdB) cd = min(cd, wdA - Ra + Lb);
    const int32_t imax = wave_incl_max(Ra), imin = wave_incl_min(Lb);
    const int32_t emax = max(wave_shr1(imax, -BIG), carry_max);
    const int32_t emin = min(wave_shr1(imin, BIG), carry_min);
    if (act && j >= 1 && j < hdB) D1 = max(D1, emax - Lb);
    if (act && j >= 1) D2 = max(D2, Ra - emin);
    carry_max = max(carry_max, lane63(imax));
    carry_min = min(carry_min, lane63(imin));
  }
  PairSweep r;
  r.cd = wave_min(cd);
  r.D1 = wave_max(D1);
  r.D2 = wave_max(D2);
  return r;
}

// The same sweep over stored grown rows: ra / rb hold, per grown row j, the
// grown left bound L' (low half) and grown right bound R' (high half, gutter
// included) of A and B.  Grown rows need no shuffles, so each chunk advances
// a full wavefront.
__device__ inline PairSweep pair_sweep_rows(const uint32_t* ra, int hdA, const uint32_t* rb,
                                            int hdB, int wdA) {
  const int lane = lane_id();
  int32_t cd = BIG, D1 = -BIG, D2 = -BIG;
  int32_t carry_max = -BIG, carry_min = BIG;
  for (int j0 = 0; j0 < hdA; j0 += WAVE) {
    const int j = j0 + lane;
    const bool act = j < hdA, shr = act && j < hdB;
    const int32_t Ra = act ? hi16(ra[j]) : -BIG;
    const int32_t Lb = shr ? lo16(rb[j]) : BIG;
    if (shr) cd = min(cd, wdA - Ra + Lb);
    const int32_t imax = wave_incl_max(Ra), imin = wave_incl_min(Lb);
    const int32_t emax = max(wave_shr1(imax, -BIG), carry_max);
    const int32_t emin = min(wave_shr1(imin, BIG), carry_min);
    if (shr && j >= 1) D1 = max(D1, emax - Lb);
    if (act && j >= 1) D2 = max(D2, Ra - emin);
    carry_max = max(carry_max, lane63(imax));
    carry_min = min(carry_min, lane63(imin));
  }
  PairSweep r;
  r.cd = wave_min(cd);
  r.D1 = wave_max(D1);
  r.D2 = wave_max(D2);
  return r;
}

// The same sweep for four pairs at once, one per 16-lane row of the
// wavefront: each step covers 16 grown rows and every scan stays inside the
// row (DPP row shifts), the row's last lane carries its running extremes to
// the next step, and the results are reduced within the row (rotations).
// Every lane of the wavefront must call it; a row without a pair passes
// hdA = 0.  The results hold in every lane of the row.
__device__ inline int32_t row_last(int32_t v) {  // lane 15 of the caller's row
  const int g = lane_id() >> 4;
  const int32_t a = __builtin_amdgcn_readlane(v, 15), b = __builtin_amdgcn_readlane(v, 31);
  const int32_t c = __builtin_amdgcn_readlane(v, 47), d = __builtin_amdgcn_readlane(v, 63);
  return g == 0 ? a : (g == 1 ? b : (g == 2 ? c : d));
}
constexpr int DPP_ROW_ROR1 = 0x121, DPP_ROW_ROR2 = 0x122, DPP_ROW_ROR4 = 0x124,
              DPP_ROW_ROR8 = 0x128;
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
__device__ inline PairSweep pair_sweep_rows16(const uint32_t* ra, int hdA, const uint32_t* rb,
                                              int hdB, int wdA) {
  const int gl = lane_id() & 15;
  int32_t cd = BIG, D1 = -BIG, D2 = -BIG;
  int32_t carry_max = -BIG, carry_min = BIG;
  const int steps = wave_max((hdA + 15) >> 4);  // the longest of the four pairs
  for (int q = 0; q < steps; ++q) {
    const int j = q * 16 + gl;
    const bool act = j < hdA, shr = act && j < hdB;
    const int32_t Ra = act ? hi16(ra[j]) : -BIG;
    const int32_t Lb = shr ? lo16(rb[j]) : BIG;
    if (shr) cd = min(cd, wdA - Ra + Lb);
    int32_t imax = Ra, imin = Lb;
    imax = max(imax, dpp_move<DPP_ROW_SHR1>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR1>(imin, BIG));
    imax = max(imax, dpp_move<DPP_ROW_SHR2>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR2>(imin, BIG));
    imax = max(imax, dpp_move<DPP_ROW_SHR4>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR4>(imin, BIG));
    imax = max(imax, dpp_move<DPP_ROW_SHR8>(imax, -BIG));
    imin = min(imin, dpp_move<DPP_ROW_SHR8>(imin, BIG));
    const int32_t emax = max(dpp_move<DPP_ROW_SHR1>(imax, -BIG), carry_max);
    const int32_t emin = min(dpp_move<DPP_ROW_SHR1>(imin, BIG), carry_min);
    if (shr && j >= 1) D1 = max(D1, emax - Lb);
    if (act && j >= 1) D2 = max(D2, Ra - emin);
    carry_max = max(carry_max, row_last(imax));
    carry_min = min(carry_min, row_last(imin));
  }
  PairSweep r;
  r.cd = row_all_min(cd);
  r.D1 = row_all_max(D1);
  r.D2 = row_all_max(D2);
  return r;
}

// Interlock flags for box offset d (bit0: B may not move above A, bit1: A may
// not move above B); none without a shared column.
__device__ inline int32_t pair_flags_at(const PairSweep& s, int wdA, int d) {
  if (d >= wdA) return 0;
  return (d < s.D1 ? 1 : 0) | (d < s.D2 ? 2 : 0);
}

}  // namespace tabi
