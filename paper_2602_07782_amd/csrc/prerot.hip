// Pre-rotation of UV charts to their tight boxes before packing (Sec. 5,
// experimental setup: UV charts are turned so that their tight bounding boxes
// line up with the axes; texture-space-shading charts are packed as given).
//
//   k_prerotate  one wavefront per chart, lane m evaluating direction
//                m pi / 128 (m = 0..63) over every vertex of the chart: the
//                vertices are loaded 64 at a time, one per lane, and read back
//                as wave-uniform values (v_readlane), so each vertex is
//                fetched once and the 64 directions cost no cross-lane
//                traffic until a single exact arg-min of the box areas.
//
// The tight box is sought over 64 directions, the OBB proxy's 8 among them
// (every 8th), as integer vectors 2^14 (cos, sin) rounded.  The area of the
// box at direction m is (b - a)(f - e) / (C^2 + S^2) with [a, b] x [e, f] the
// vertex extents along (C, S) and (-S, C); it is compared exactly (128-bit
// cross products), ties going to the smaller m.  The chart is turned about its
// box corner, (dx, dy) -> (C dx + S dy, -S dx + C dy) / 2^14 rounded to the
// nearest Q8 unit (halves up), and moved so that the turned box starts at the
// origin.  Charts the pack rejects (fewer than 3 vertices, a coordinate
// outside (-2^22, 2^22)) are copied as they are, with direction 0.
#include "tabi_internal.h"

namespace tabi {

// round(2^14 cos(m pi / 128)), round(2^14 sin(m pi / 128)), m = 0..63
__constant__ static const int32_t kTurnC[64] = {
    16384, 16379, 16364, 16340, 16305, 16261, 16207, 16143, 16069, 15986, 15893, 15791, 15679,
    15557, 15426, 15286, 15137, 14978, 14811, 14635, 14449, 14256, 14053, 13842, 13623, 13395,
    13160, 12916, 12665, 12406, 12140, 11866, 11585, 11297, 11003, 10702, 10394, 10080, 9760,
    9434,  9102,  8765,  8423,  8076,  7723,  7366,  7005,  6639,  6270,  5897,  5520,  5139,
    4756,  4370,  3981,  3590,  3196,  2801,  2404,  2006,  1606,  1205,  804,   402};
__constant__ static const int32_t kTurnS[64] = {
    0,     402,   804,   1205,  1606,  2006,  2404,  2801,  3196,  3590,  3981,  4370,  4756,
    5139,  5520,  5897,  6270,  6639,  7005,  7366,  7723,  8076,  8423,  8765,  9102,  9434,
    9760,  10080, 10394, 10702, 11003, 11297, 11585, 11866, 12140, 12406, 12665, 12916, 13160,
    13395, 13623, 13842, 14053, 14256, 14449, 14635, 14811, 14978, 15137, 15286, 15426, 15557,
    15679, 15791, 15893, 15986, 16069, 16143, 16207, 16261, 16305, 16340, 16364, 16379};

__device__ inline int wave_min_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}

constexpr int PREROT_WAVES = 4;  // charts per 256-thread block

// xy and out may be the same array (each wave reads its chart whole before
// it writes, and then writes only the vertices its lanes have just read).
__global__ __launch_bounds__(256) void k_prerotate(const int32_t* xy,
                                                   const int32_t* __restrict__ voff, int n,
                                                   int32_t* out, uint8_t* __restrict__ dir) {
  const int lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * PREROT_WAVES + (threadIdx.x >> 6));
  if (c >= n) return;  // whole wavefront
  const int v0 = __builtin_amdgcn_readfirstlane(voff[c]);
  const int nv = __builtin_amdgcn_readfirstlane(voff[c + 1]) - v0;
  const int2* V = reinterpret_cast<const int2*>(xy) + v0;
  int2* O = reinterpret_cast<int2*>(out) + v0;

  int bad = nv < 3, xmn = INT32_MAX, ymn = INT32_MAX;
  for (int i = lane; i < nv; i += 64) {
    const int2 p = V[i];
    bad |= p.x <= -(1 << 22) || p.x >= (1 << 22) || p.y <= -(1 << 22) || p.y >= (1 << 22);
    xmn = min(xmn, p.x);
    ymn = min(ymn, p.y);
  }
  if (__builtin_amdgcn_readfirstlane(__any(bad))) {
    for (int i = lane; i < nv; i += 64) O[i] = V[i];
    if (lane == 0) dir[c] = 0;
    return;
  }
  xmn = wave_min_i32(xmn);
  ymn = wave_min_i32(ymn);

  // extents of the chart along direction m = lane; offsets from the box
  // corner are below 2^23 and the table below 2^15, so products fit 2^38
  const int64_t C = kTurnC[lane], S = kTurnS[lane];
  int64_t a = INT64_MAX, b = INT64_MIN, e = INT64_MAX, f = INT64_MIN;
  for (int i0 = 0; i0 < nv; i0 += 64) {
    int dx = 0, dy = 0;
    if (i0 + lane < nv) {
      const int2 p = V[i0 + lane];
      dx = p.x - xmn;
      dy = p.y - ymn;
    }
    const int cnt = min(64, nv - i0);
    for (int j = 0; j < cnt; ++j) {
      const int64_t x = __builtin_amdgcn_readlane(dx, j), y = __builtin_amdgcn_readlane(dy, j);
      const int64_t p = C * x + S * y, q = C * y - S * x;
      a = min(a, p); b = max(b, p);
      e = min(e, q); f = max(f, q);
    }
  }

  // exact arg-min of (b - a)(f - e) / N over the lanes: the other lane wins
  // when ext' N < ext N' (products below 2^107), or on a tie with smaller m
  using u128 = unsigned __int128;
  u128 ext = (u128)(uint64_t)(b - a) * (uint64_t)(f - e);
  uint32_t N = (uint32_t)(C * C + S * S);
  int best = lane;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint64_t ohi = __shfl_xor((unsigned long long)(uint64_t)(ext >> 64), off);
    const uint64_t olo = __shfl_xor((unsigned long long)(uint64_t)ext, off);
    const uint32_t oN = __shfl_xor(N, off);
    const int ob = __shfl_xor(best, off);
    const u128 oext = ((u128)ohi << 64) | olo;
    const u128 l = oext * N, r = ext * oN;
    if (l < r || (l == r && ob < best)) { ext = oext; N = oN; best = ob; }
  }
  best = __builtin_amdgcn_readfirstlane(best);

  // turn about the box corner; the rounding is monotone, so the smallest
  // rounded coordinate is the rounded smallest extent of direction best
  const int64_t ab = __shfl(a, best), eb = __shfl(e, best);
  const int64_t tx = (ab + 8192) >> 14, ty = (eb + 8192) >> 14;
  const int64_t Cb = kTurnC[best], Sb = kTurnS[best];
  for (int i = lane; i < nv; i += 64) {
    const int2 p = V[i];
    const int64_t x = p.x - xmn, y = p.y - ymn;
    int2 r;
    r.x = (int32_t)(((Cb * x + Sb * y + 8192) >> 14) - tx);
    r.y = (int32_t)(((Cb * y - Sb * x + 8192) >> 14) - ty);
    O[i] = r;
  }
  if (lane == 0) dir[c] = (uint8_t)best;
}

hipError_t launch_prerotate(const int32_t* xy, const int32_t* voff, int n, int32_t* out,
                            uint8_t* dir, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + PREROT_WAVES - 1) / PREROT_WAVES;
  hipLaunchKernelGGL(k_prerotate, dim3(blocks), dim3(256), 0, st, xy, voff, n, out, dir);
  return hipGetLastError();
}

}  // namespace tabi
