// Interlock test of two charts of one compacted row, wavefront-cooperative.
#pragma once

#include "tabi_device.h"

namespace tabi {

// Flags for chart A and a later chart B whose grown box starts d texels right
// of A's (App. A, "Detecting Interlocking Charts").  bit0: B may not move
// above A, set when some row j >= 1 of B starts left of where A ends in a row
// above j; bit1: A may not move above B, set when some row j >= 1 of A ends
// right of where B starts in a row above j.  Raising one chart by 1..j texels
// brings exactly those rows side by side, so a clear flag means no upward
// shift can make the proxies meet.  No shared column, no flag.  All lanes of
// the wavefront must call this with the same arguments.
__device__ inline int32_t pair_flags(const KView& A, const Chart& cA, const KView& B,
                                     const Chart& cB, int K, int k, int p, int d) {
  const int lane = lane_id();
  const int hdA = A.hd->h + p, hdB = B.hd->h + p, wdA = A.hd->w + p;
  if (d >= wdA) return 0;
  int32_t carry_max = -BIG;  // max of A's right ends over the rows before this chunk
  int32_t carry_min = BIG;   // min of B's left ends over the rows before this chunk
  int flags = 0;
  for (int j0 = 0; j0 < hdA && flags != 3; j0 += WAVE) {
    const int j = j0 + lane;
    int32_t ra = -BIG, lb = BIG;
    if (j < hdA) {
      int32_t l, r;
      row_bounds_grown(A, cA, K, k, p, j, l, r);
      ra = r;
    }
    if (j < hdB) {
      int32_t l, r;
      row_bounds_grown(B, cB, K, k, p, j, l, r);
      lb = l;
    }
    const int32_t imax = wave_incl_max(ra), imin = wave_incl_min(lb);
    int32_t emax = __shfl_up(imax, 1), emin = __shfl_up(imin, 1);
    if (lane == 0) { emax = -BIG; emin = BIG; }
    emax = max(emax, carry_max);
    emin = min(emin, carry_min);
    const bool b_up = j >= 1 && j < hdB && d + lb < emax;
    const bool a_up = j >= 1 && j < hdA && ra > d + emin;
    if (ballot64(b_up)) flags |= 1;
    if (ballot64(a_up)) flags |= 2;
    carry_max = max(carry_max, __shfl(imax, WAVE - 1));
    carry_min = min(carry_min, __shfl(imin, WAVE - 1));
  }
  return flags;
}

}  // namespace tabi
