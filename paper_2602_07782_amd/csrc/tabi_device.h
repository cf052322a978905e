// Device-side data layout and helpers of the MI355X TABI packer (gfx950).
//
// Every quantity on the packing path is an integer; the per-texel proxy
// bounds are exact rationals rounded outward with floor / ceil.  Wavefronts
// are 64 lanes wide.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tabi {

constexpr int KMAX = 10;     // local AABB slices per axis, largest quality
constexpr int64_t QS = 16384; // Q8 units per texel (256) times 64 scale steps
constexpr int WAVE = 64;
constexpr int32_t BIG = 0x3fffffff;

// Chart proxies in the chart's final local frame (after the quarter turn and
// reflections), Q8 units.  Sec. 4.1.1: local AABBs along x and y, and an
// approximate OBB from 8 directions.
struct alignas(16) Chart {
  int32_t W, H;      // extents, H >= W
  int32_t bits;      // bit0 quarter turn, bit1 mirror x, bit2 mirror y
  int32_t m;         // OBB direction index (0: axis aligned, adds nothing)
  int64_t a, b, e, f;  // OBB: a <= C u + S v <= b, e <= -S u + C v <= f
  int32_t ylo[KMAX], yhi[KMAX];  // x-slices: v-range inside u in [jW/K, (j+1)W/K]
  int32_t xlo[KMAX], xhi[KMAX];  // y-slices: u-range inside v in [jH/K, (j+1)H/K]
  int64_t area2;     // twice the polygon area, Q8^2
  int32_t src;       // input index (within its atlas)
  int32_t valid;
};

// OBB direction m*pi/16 as 2^14 (cos, sin), rounded to integers.
__constant__ static const int32_t kDirC[8] = {16384, 16069, 15137, 13623, 11585, 9102, 6270, 3196};
__constant__ static const int32_t kDirS[8] = {0, 3196, 6270, 9102, 11585, 13623, 15137, 16069};

// Per (scale, chart) rasterisation set-up.  At scale k the local-AABB proxy
// becomes 2K integer texel rectangles (x-slices then y-slices); the OBB
// boundary on each of the four sides is evaluated per texel from one line,
// chosen by which side of the box corner the texel lies (see side_value).
struct alignas(16) KHead {
  int32_t w, h;      // texel extents at this scale (undilated)
  int32_t obb;       // OBB present
  int32_t pad;
};
struct alignas(16) KSide {
  int32_t sa;        // texels t with t+1 <= sa use line A at t+1
  int32_t sb;        // texels t >= sb use line B at t (otherwise: corner)
  int32_t corner;    // rounded corner coordinate
  int32_t last;      // full value for the last texel (extent may end mid-texel)
};
struct alignas(8) KRect {
  int16_t c0, c1, r0, r1;  // columns [c0,c1) x rows [r0,r1)
};

// Bytes of one per-(scale, chart) record for K slices.
__host__ __device__ inline int kchart_stride(int K) {
  return (int)(sizeof(KHead) + 4 * sizeof(KSide) + 2 * K * sizeof(KRect));
}

constexpr int KREC_MAX = 16 + 4 * 16 + 2 * KMAX * 8;  // kchart_stride(KMAX)

// A chart and its per-scale record, staged in LDS by one wavefront.
struct alignas(16) ChartCache {
  Chart ch;
  unsigned char kc[KREC_MAX];
};

struct KView {
  const KHead* hd;
  const KSide* sd;   // [0] top, [1] bottom, [2] left, [3] right
  const KRect* rc;   // 2K rectangles
};
// Last-workgroup pattern: the calling workgroup (all its threads) makes its
// global writes visible device-wide and counts itself in *counter; returns
// true, uniformly, in the workgroup that counts last of `total`, after it has
// acquired the others' writes.  Every wavefront waits for its own stores to
// reach the L2, then one thread releases them all with its increment (a
// single write-back of the XCD's L2, where a fence in every thread would
// write back and invalidate once per wavefront); only the last workgroup
// acquires.  flag: one int of shared memory.
__device__ inline bool last_to_finish(int32_t* counter, int total, int32_t* flag) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool last =
        __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == total - 1;
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = last;
  }
  __syncthreads();
  return *flag != 0;
}

__device__ inline KView kview(const unsigned char* base, int K) {
  KView v;
  v.hd = reinterpret_cast<const KHead*>(base);
  v.sd = reinterpret_cast<const KSide*>(base + sizeof(KHead));
  v.rc = reinterpret_cast<const KRect*>(base + sizeof(KHead) + 4 * sizeof(KSide));
  return v;
}

// ---------------------------------------------------------------------------
// exact integer division
// ---------------------------------------------------------------------------
// floor(n / d) for 0 < d < 2^31 and |n| < 2^53: the double quotient is within
// one unit of the true one, so one integer correction makes it exact.
__device__ inline int64_t fdiv53(int64_t n, int64_t d) {
  int64_t q = (int64_t)floor((double)n / (double)d);
  int64_t r = n - q * d;
  if (r < 0) q -= 1;
  else if (r >= d) q += 1;
  return q;
}
__device__ inline int64_t cdiv53(int64_t n, int64_t d) { return -fdiv53(-n, d); }

// floor(n / d) for 0 < d < 2^31 and |n| < 2^53, cheaper when the quotient is
// small: the single-precision estimate (conversions of n and d, an
// approximate reciprocal within one ulp, the product: relative error below
// 2^-21) is within 1/2 of n / d whenever |n / d| < 2^20, so its floor is off
// by at most one and one integer correction makes it exact.  Larger
// quotients take fdiv53.
__device__ inline int64_t fdiv_q(int64_t n, int64_t d) {
  const float qf = floorf((float)n * __builtin_amdgcn_rcpf((float)d));
  if (fabsf(qf) < 1048576.0f) {
    int64_t q = (int64_t)(int32_t)qf;
    const int64_t r = n - q * d;
    if (r < 0) q -= 1;
    else if (r >= d) q += 1;
    return q;
  }
  return fdiv53(n, d);
}

// floor / ceil for any int64 with d > 0
__host__ __device__ inline int64_t fdiv64(int64_t n, int64_t d) {
  int64_t q = n / d;
  if ((n % d) != 0 && n < 0) q -= 1;
  return q;
}
__host__ __device__ inline int64_t cdiv64(int64_t n, int64_t d) { return -fdiv64(-n, d); }

// floor / ceil for any int64 n and d > 0, fast when the quotient is small:
// the single-precision estimate (n and d rounded, an approximate reciprocal,
// the product: relative error below 2^-21) is within 1/2 of n / d when
// |n / d| < 2^20, so one correction makes its floor exact (n - q d cannot
// overflow: |q d| <= |n| + d).  Other quotients take the 64-bit division.
__device__ inline int64_t fdiv_i64(int64_t n, int64_t d) {
  const float qf = floorf((float)n * __builtin_amdgcn_rcpf((float)d));
  if (fabsf(qf) < 1048576.0f) {
    int64_t q = (int64_t)(int32_t)qf;
    const int64_t r = n - q * d;
    if (r < 0) q -= 1;
    else if (r >= d) q += 1;
    return q;
  }
  return fdiv64(n, d);
}
__device__ inline int64_t cdiv_i64(int64_t n, int64_t d) { return -fdiv_i64(-n, d); }

__device__ inline int32_t clamp32(int64_t v) {
  return (int32_t)(v < -(1 << 30) ? -(1 << 30) : (v > (1 << 30) ? (1 << 30) : v));
}

// ---------------------------------------------------------------------------
// per-texel proxy evaluation
// ---------------------------------------------------------------------------
// Whole-record loads: every field of a rectangle / side / head in one memory
// operation, so that the K rectangles of a proxy are fetched together rather
// than field by field behind the comparisons.
__device__ inline void krect_load(const KRect* p, int32_t& c0, int32_t& c1, int32_t& r0,
                                  int32_t& r1) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  c0 = (int32_t)(int16_t)(uint16_t)(v.x & 0xffffu);
  c1 = (int32_t)v.x >> 16;
  r0 = (int32_t)(int16_t)(uint16_t)(v.y & 0xffffu);
  r1 = (int32_t)v.y >> 16;
}
__device__ inline KSide kside_load(const KSide* p) {
  const int4 v = *reinterpret_cast<const int4*>(p);
  KSide s;
  s.sa = v.x; s.sb = v.y; s.corner = v.z; s.last = v.w;
  return s;
}
__device__ inline KHead khead_load(const KHead* p) {
  const int4 v = *reinterpret_cast<const int4*>(p);
  KHead h;
  h.w = v.x; h.h = v.y; h.obb = v.z; h.pad = v.w;
  return h;
}

// OBB side value at texel t (column for top/bottom, row for left/right) of an
// extent with n texels.  Line A applies left of (above) the corner, line B
// right of (below) it; each line is (n0 + n1 * x) / d rounded down (lo sides)
// or up (hi sides).
// floor(P / d) in 32-bit arithmetic for |P| < 2^30 and 3196 <= d <= 2^14
// (the OBB directions' rounded 2^14 cos / sin): |P / d| < 2^19, and the
// single-precision estimate (P rounded, d exact, an approximate reciprocal
// within one ulp, the product rounded: relative error below 2^-21) is
// within 1/4 of P / d, so its floor is off by at most one and one
// correction makes it exact.
__device__ inline int32_t fdiv_i32(int32_t P, int32_t d) {
  int32_t q = (int32_t)floorf((float)P * __builtin_amdgcn_rcpf((float)d));
  const int32_t r = P - q * d;
  q += r < 0 ? -1 : (r >= d ? 1 : 0);
  return q;
}

// Branch-free: every lane selects its line first, so a wavefront whose
// lanes straddle the corner still performs one division.  Every line has
// n1 and d multiples of 2^14 (= QS), so with n0 = 2^14 M + L, 0 <= L < 2^14,
//   floor((n0 + n1 x) / d) = floor((M + (n1 / 2^14) x) / (d / 2^14)),
// because L < 2^14 cannot lift the numerator past the next multiple of d:
// the whole evaluation fits 32 bits (|M| < 2^30, |n1 / 2^14| <= 2^14 and
// |x| <= 2^15 + 64 bound the numerator by 2^30 + 2^29; larger values take
// the 64-bit route).
template <bool CEIL>
__device__ inline int32_t side_value(const KSide& s, int32_t t, int32_t n, int64_t n0a, int64_t n1a,
                                     int64_t da, int64_t n0b, int64_t n1b, int64_t db) {
  const bool useA = t + 1 <= s.sa, useB = t >= s.sb;
  const int64_t n0 = useA ? n0a : n0b, n1 = useA ? n1a : n1b, d = useA ? da : db;
  const int64_t x = useA ? (int64_t)t + 1 : (int64_t)t;
  // ceil(v / d) = -floor(-v / d)
  const int64_t N0 = CEIL ? -n0 : n0, N1 = CEIL ? -n1 : n1;
  const int64_t P = (N0 >> 14) + (N1 >> 14) * x;
  int32_t q;
  if (P > -(1ll << 30) && P < (1ll << 30)) q = fdiv_i32((int32_t)P, (int32_t)(d >> 14));
  else q = (int32_t)fdiv_q(N0 + N1 * x, d);
  if (CEIL) q = -q;
  return t == n - 1 ? s.last : ((useA || useB) ? q : s.corner);
}

// Top / bottom of column i over the local-AABB slices: the x-slices and the
// y-slices covering the column each give a range; the proxy keeps their
// intersection.  KT > 0 fixes the slice count at compile time (K == KT).
template <int KT = 0>
__device__ inline void column_rects(const KView& kv, int K, int i, int32_t& top, int32_t& bot) {
  if (KT) K = KT;
  int32_t tx = BIG, bx = -BIG, ty = BIG, by = -BIG;
#pragma unroll
  for (int j = 0; j < (KT ? KT : KMAX); ++j) {
    if (KT || j < K) {
      int32_t c0, c1, r0, r1;
      krect_load(kv.rc + j, c0, c1, r0, r1);
      const bool in = c0 <= i && i < c1;
      tx = in ? min(tx, r0) : tx;
      bx = in ? max(bx, r1) : bx;
      krect_load(kv.rc + K + j, c0, c1, r0, r1);
      const bool iny = c0 <= i && i < c1;
      ty = iny ? min(ty, r0) : ty;
      by = iny ? max(by, r1) : by;
    }
  }
  top = max(tx, ty);
  bot = min(bx, by);
}

// Undilated TopEdge / BottomEdge of column i (App. A, "Parallel Pushing"):
// the tightest of the two proxies, rounded outward.
template <int KT = 0>
__device__ inline void column_bounds(const KView& kv, const Chart& ch, int K, int k, int i,
                                     int32_t& top, int32_t& bot) {
  int32_t t, b;
  column_rects<KT>(kv, K, i, t, b);
  const KHead hd = khead_load(kv.hd);
  if (hd.obb) {
    const int64_t C = kDirC[ch.m], S = kDirS[ch.m];
    const int64_t kk = k;
    const KSide s0 = kside_load(kv.sd + 0), s1 = kside_load(kv.sd + 1);
    // top = max(A: (k a - 16384 C x)/(16384 S), B: (k e + 16384 S x)/(16384 C))
    int32_t to = side_value<false>(s0, i, hd.w, kk * ch.a, -QS * C, QS * S, kk * ch.e, QS * S, QS * C);
    // bottom = min(A: (k f + 16384 S x)/(16384 C), B: (k b - 16384 C x)/(16384 S))
    int32_t bo = side_value<true>(s1, i, hd.w, kk * ch.f, QS * S, QS * C, kk * ch.b, -QS * C, QS * S);
    t = max(t, to);
    b = min(b, bo);
  }
  top = t;
  bot = b;
}

// Left / right of row j over the local-AABB slices.
template <int KT = 0>
__device__ inline void row_rects(const KView& kv, int K, int j, int32_t& left, int32_t& right) {
  if (KT) K = KT;
  int32_t ly = BIG, ry = -BIG, lx = BIG, rx = -BIG;
#pragma unroll
  for (int q = 0; q < (KT ? KT : KMAX); ++q) {
    if (KT || q < K) {
      int32_t c0, c1, r0, r1;
      krect_load(kv.rc + K + q, c0, c1, r0, r1);
      const bool iny = r0 <= j && j < r1;
      ly = iny ? min(ly, c0) : ly;
      ry = iny ? max(ry, c1) : ry;
      krect_load(kv.rc + q, c0, c1, r0, r1);
      const bool inx = r0 <= j && j < r1;
      lx = inx ? min(lx, c0) : lx;
      rx = inx ? max(rx, c1) : rx;
    }
  }
  left = max(ly, lx);
  right = min(ry, rx);
}

// The two lines of an OBB side in 32-bit form: line value at x is
// floor((M + n x) / d) (negated for a rounded-up side), from side_value's
// (n0, n1, d) by the same exact reduction (M = n0 >> 14, n = n1 / 2^14,
// d / 2^14).  ok is false when an M is too large for 32-bit evaluation
// (|M| >= 2^29: a chart far larger than any atlas), then side_value is used.
struct SideLines {
  int32_t MA, nA, dA, MB, nB, dB;
  bool ok;
};
template <bool CEIL>
__device__ inline SideLines side_lines(int64_t n0a, int64_t n1a, int64_t da, int64_t n0b,
                                       int64_t n1b, int64_t db) {
  const int64_t MA = (CEIL ? -n0a : n0a) >> 14, MB = (CEIL ? -n0b : n0b) >> 14;
  SideLines L;
  L.ok = MA > -(1ll << 29) && MA < (1ll << 29) && MB > -(1ll << 29) && MB < (1ll << 29);
  L.MA = (int32_t)MA;
  L.MB = (int32_t)MB;
  L.nA = (int32_t)((CEIL ? -n1a : n1a) >> 14);
  L.nB = (int32_t)((CEIL ? -n1b : n1b) >> 14);
  L.dA = (int32_t)(da >> 14);
  L.dB = (int32_t)(db >> 14);
  return L;
}
// side value at texel t (|t| <= 2^15 + 64, so |M + n x| < 2^31)
template <bool CEIL>
__device__ inline int32_t side_eval(const KSide& s, int32_t t, int32_t n, const SideLines& L) {
  const bool useA = t + 1 <= s.sa, useB = t >= s.sb;
  const int32_t M = useA ? L.MA : L.MB, nn = useA ? L.nA : L.nB, d = useA ? L.dA : L.dB;
  const int32_t x = useA ? t + 1 : t;
  int32_t q = fdiv_i32(M + nn * x, d);
  if (CEIL) q = -q;
  return t == n - 1 ? s.last : ((useA || useB) ? q : s.corner);
}

// Column i and row j of the same chart at once (the profile sweep needs
// both): every slice rectangle is loaded once and tested against both, and
// the four OBB side values are independent of each other.  The column's
// top / bottom are the tightest of both proxies; the row's bounds are given
// per proxy: la, ra from the local AABBs, lo, ro from the OBB kept inside
// the chart's texel box [0, w] (that box when the chart has no OBB), so that
// the compacting distance can be measured on each proxy (Sec. 4.1.2).
template <int KT>
__device__ inline void column_row_bounds(const KView& kv, const Chart& ch, int k, int i, int j,
                                         int32_t& top, int32_t& bot, int32_t& la, int32_t& ra,
                                         int32_t& lo, int32_t& ro) {
  constexpr int K = KT;
  int32_t tx = BIG, bx = -BIG, ty = BIG, by = -BIG;
  int32_t ly = BIG, ry = -BIG, lx = BIG, rx = -BIG;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    int32_t c0, c1, r0, r1;
    krect_load(kv.rc + q, c0, c1, r0, r1);  // x-slice
    const bool ci = c0 <= i && i < c1, rj = r0 <= j && j < r1;
    tx = ci ? min(tx, r0) : tx;
    bx = ci ? max(bx, r1) : bx;
    lx = rj ? min(lx, c0) : lx;
    rx = rj ? max(rx, c1) : rx;
    krect_load(kv.rc + K + q, c0, c1, r0, r1);  // y-slice
    const bool ci2 = c0 <= i && i < c1, rj2 = r0 <= j && j < r1;
    ty = ci2 ? min(ty, r0) : ty;
    by = ci2 ? max(by, r1) : by;
    ly = rj2 ? min(ly, c0) : ly;
    ry = rj2 ? max(ry, c1) : ry;
  }
  int32_t t = max(tx, ty), b = min(bx, by);
  la = max(ly, lx);
  ra = min(ry, rx);
  const KHead hd = khead_load(kv.hd);
  int32_t l = 0, rr = hd.w;
  if (hd.obb) {
    const int64_t C = kDirC[ch.m], S = kDirS[ch.m];
    const int64_t kk = k;
    const KSide s0 = kside_load(kv.sd + 0), s1 = kside_load(kv.sd + 1);
    const KSide s2 = kside_load(kv.sd + 2), s3 = kside_load(kv.sd + 3);
    // the same lines as column_bounds / row_proxies
    const SideLines L0 = side_lines<false>(kk * ch.a, -QS * C, QS * S, kk * ch.e, QS * S, QS * C);
    const SideLines L1 = side_lines<true>(kk * ch.f, QS * S, QS * C, kk * ch.b, -QS * C, QS * S);
    const SideLines L2 = side_lines<false>(kk * ch.a, -QS * S, QS * C, -kk * ch.f, QS * C, QS * S);
    const SideLines L3 = side_lines<true>(-kk * ch.e, QS * C, QS * S, kk * ch.b, -QS * S, QS * C);
    if (L0.ok && L1.ok && L2.ok && L3.ok) {
      t = max(t, side_eval<false>(s0, i, hd.w, L0));
      b = min(b, side_eval<true>(s1, i, hd.w, L1));
      l = max(l, side_eval<false>(s2, j, hd.h, L2));
      rr = min(rr, side_eval<true>(s3, j, hd.h, L3));
    } else {
      t = max(t, side_value<false>(s0, i, hd.w, kk * ch.a, -QS * C, QS * S, kk * ch.e, QS * S, QS * C));
      b = min(b, side_value<true>(s1, i, hd.w, kk * ch.f, QS * S, QS * C, kk * ch.b, -QS * C, QS * S));
      l = max(l, side_value<false>(s2, j, hd.h, kk * ch.a, -QS * S, QS * C, -kk * ch.f, QS * C, QS * S));
      rr = min(rr, side_value<true>(s3, j, hd.h, -kk * ch.e, QS * C, QS * S, kk * ch.b, -QS * S, QS * C));
    }
  }
  top = t;
  bot = b;
  lo = l;
  ro = rr;
}

// Undilated left / right bounds of row j under each proxy separately, as
// column_row_bounds gives them.
template <int KT = 0>
__device__ inline void row_proxies(const KView& kv, const Chart& ch, int K, int k, int j,
                                   int32_t& la, int32_t& ra, int32_t& lo, int32_t& ro) {
  row_rects<KT>(kv, K, j, la, ra);
  const KHead hd = khead_load(kv.hd);
  int32_t l = 0, rr = hd.w;
  if (hd.obb) {
    const int64_t C = kDirC[ch.m], S = kDirS[ch.m];
    const int64_t kk = k;
    const KSide s2 = kside_load(kv.sd + 2), s3 = kside_load(kv.sd + 3);
    // left = max(A: (k a - 16384 S y)/(16384 C), B: (16384 C y - k f)/(16384 S))
    l = max(l, side_value<false>(s2, j, hd.h, kk * ch.a, -QS * S, QS * C, -kk * ch.f, QS * C, QS * S));
    // right = min(A: (16384 C y - k e)/(16384 S), B: (k b - 16384 S y)/(16384 C))
    rr = min(rr, side_value<true>(s3, j, hd.h, -kk * ch.e, QS * C, QS * S, kk * ch.b, -QS * S, QS * C));
  }
  lo = l;
  ro = rr;
}

// The per-(scale, chart) set-up record of chart ch at scale k/64, written to
// `base` (KHead, four KSide, 2K KRect): the chart's texel extents, its
// local-AABB slices as texel rectangles, and the OBB sides' split points and
// corners at this scale.  wt, ht: the texel extents.
template <int KT>
__device__ inline void build_krec(const Chart& ch, int k, unsigned char* base, int32_t& wt,
                                  int32_t& ht) {
  constexpr int K = KT;
  KHead* hd = reinterpret_cast<KHead*>(base);
  KSide* sd = reinterpret_cast<KSide*>(base + sizeof(KHead));
  KRect* rc = reinterpret_cast<KRect*>(base + sizeof(KHead) + 4 * sizeof(KSide));
  const int64_t kk = k, W = ch.W, H = ch.H;
  wt = (int32_t)cdiv_i64(kk * W, QS);
  ht = (int32_t)cdiv_i64(kk * H, QS);
  KHead h;
  h.w = wt;
  h.h = ht;
  h.obb = ch.m != 0;
  h.pad = 0;
  *hd = h;
  // local-AABB slices as texel rectangles at this scale
  // (values are clamped to int16; only a chart larger than any atlas reaches
  // the clamp, and such a scale fails on that chart's width or height anyway)
  auto i16 = [](int64_t v) { return (int16_t)(v > 32767 ? 32767 : v); };
  // slice boundaries: j W k / 2^14 < 11 * 2^23 * 64 / 2^14 < 2^19, so the
  // quotient by K is a 32-bit division by a constant
  auto slab = [](int64_t num) { return (int32_t)(uint32_t)((uint64_t)num >> 14) / K; };
#pragma unroll
  for (int j = 0; j < K; ++j) {
    KRect r;
    r.c0 = i16(slab((int64_t)j * W * kk));
    r.c1 = i16(slab((int64_t)(j + 1) * W * kk + QS * K - 1));
    r.r0 = i16(((int64_t)ch.ylo[j] * kk) >> 14);
    r.r1 = i16(((int64_t)ch.yhi[j] * kk + QS - 1) >> 14);
    rc[j] = r;
    KRect y;
    y.c0 = i16(((int64_t)ch.xlo[j] * kk) >> 14);
    y.c1 = i16(((int64_t)ch.xhi[j] * kk + QS - 1) >> 14);
    y.r0 = i16(slab((int64_t)j * H * kk));
    y.r1 = i16(slab((int64_t)(j + 1) * H * kk + QS * K - 1));
    rc[K + j] = y;
  }
  if (!h.obb) return;
  const int64_t C = kDirC[ch.m], S = kDirS[ch.m], N = C * C + S * S, D = QS * N;
  const int64_t a = ch.a, b = ch.b, e = ch.e, f = ch.f;
  auto split = [&](int64_t num, KSide& sdv) {  // corner position num/D (texels)
    sdv.sa = clamp32(fdiv_i64(num, D));
    sdv.sb = clamp32(cdiv_i64(num, D));
  };
  KSide st, sb, sL, sR;
  // top: corner (p=a, q=e); A: (k a - 16384 C x)/(16384 S); B: (k e + 16384 S x)/(16384 C)
  split(kk * (C * a - S * e), st);
  st.corner = clamp32(fdiv_i64(kk * (S * a + C * e), D));
  // bottom: corner (p=b, q=f); A: (k f + 16384 S x)/(16384 C); B: (k b - 16384 C x)/(16384 S)
  split(kk * (C * b - S * f), sb);
  sb.corner = clamp32(cdiv_i64(kk * (S * b + C * f), D));
  // left: corner (p=a, q=f) at row k(Sa+Cf)/D; A: (k a - 16384 S y)/(16384 C); B: (16384 C y - k f)/(16384 S)
  split(kk * (S * a + C * f), sL);
  sL.corner = clamp32(fdiv_i64(kk * (C * a - S * f), D));
  // right: corner (p=b, q=e) at row k(Sb+Ce)/D; A: (16384 C y - k e)/(16384 S); B: (k b - 16384 S y)/(16384 C)
  split(kk * (S * b + C * e), sR);
  sR.corner = clamp32(cdiv_i64(kk * (C * b - S * e), D));
  // last column / row: the extent may end inside the texel
  const int64_t tw = wt - 1, th = ht - 1;
  const bool wfrac = (kk * W) % QS != 0, hfrac = (kk * H) % QS != 0;
  // top
  if (!wfrac ? (tw + 1 <= st.sa) : (W * N <= C * a - S * e))
    st.last = clamp32(!wfrac ? fdiv_i64(kk * a - QS * C * (tw + 1), QS * S) : fdiv_i64(kk * (a - C * W), QS * S));
  else if (tw >= st.sb) st.last = clamp32(fdiv_i64(kk * e + QS * S * tw, QS * C));
  else st.last = st.corner;
  // bottom
  if (!wfrac ? (tw + 1 <= sb.sa) : (W * N <= C * b - S * f))
    sb.last = clamp32(!wfrac ? cdiv_i64(kk * f + QS * S * (tw + 1), QS * C) : cdiv_i64(kk * (f + S * W), QS * C));
  else if (tw >= sb.sb) sb.last = clamp32(cdiv_i64(kk * b - QS * C * tw, QS * S));
  else sb.last = sb.corner;
  // left
  if (!hfrac ? (th + 1 <= sL.sa) : (H * N <= S * a + C * f))
    sL.last = clamp32(!hfrac ? fdiv_i64(kk * a - QS * S * (th + 1), QS * C) : fdiv_i64(kk * (a - S * H), QS * C));
  else if (th >= sL.sb) sL.last = clamp32(fdiv_i64(QS * C * th - kk * f, QS * S));
  else sL.last = sL.corner;
  // right
  if (!hfrac ? (th + 1 <= sR.sa) : (H * N <= S * b + C * e))
    sR.last = clamp32(!hfrac ? cdiv_i64(QS * C * (th + 1) - kk * e, QS * S) : cdiv_i64(kk * (C * H - e), QS * S));
  else if (th >= sR.sb) sR.last = clamp32(cdiv_i64(kk * b - QS * S * th, QS * C));
  else sR.last = sR.corner;
  sd[0] = st;
  sd[1] = sb;
  sd[2] = sL;
  sd[3] = sR;
}

// Gutter growth: a footprint grows by [0,p]^2 toward +x, +y, so a grown
// column i takes the min top / max bottom over undilated columns [i-p, i].
__device__ inline void column_bounds_grown(const KView& kv, const Chart& ch, int K, int k, int p,
                                           int i, int32_t& top, int32_t& bot) {
  const int w = kv.hd->w;
  int lo = max(0, i - p), hi = min(w - 1, i);
  int32_t t = BIG, b = -BIG;
  for (int c = lo; c <= hi; ++c) {
    int32_t tt, bb;
    column_bounds(kv, ch, K, k, c, tt, bb);
    t = min(t, tt);
    b = max(b, bb);
  }
  top = t;
  bot = b + p;
}
// ---------------------------------------------------------------------------
// stored per-texel profiles: two int16 bounds in one 32-bit word
// ---------------------------------------------------------------------------
// Bounds stay within a chart's own texel extent (plus the gutter); only a
// chart larger than any atlas would reach the clamp, and such a chart fails
// its scale on width or height whichever value is stored.
__device__ inline uint32_t pack16(int32_t lo, int32_t hi) {
  const int32_t a = lo < -32768 ? -32768 : (lo > 32767 ? 32767 : lo);
  const int32_t b = hi < -32768 ? -32768 : (hi > 32767 ? 32767 : hi);
  return (uint32_t)(uint16_t)(int16_t)a | ((uint32_t)(uint16_t)(int16_t)b << 16);
}
__device__ inline int32_t lo16(uint32_t v) { return (int32_t)(int16_t)(uint16_t)(v & 0xffffu); }
__device__ inline int32_t hi16(uint32_t v) { return (int32_t)v >> 16; }

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

// Lane moves by DPP (data-parallel primitives of the VALU; a 64-lane
// wavefront is four rows of 16): row_shr:n takes lane l-n of the same row,
// row_bcast:15 / :31 feed lane 15 of a row (31 of the wavefront) to the rows
// selected by the row mask, wave_shr:1 / wave_shl:1 take lane l-1 / l+1.
// Lanes without a source keep `fill`.  Every lane of the wavefront must be
// active: a disabled source lane supplies whatever its register holds.
template <int CTRL, int ROWS = 0xf>
__device__ inline int32_t dpp_move(int32_t v, int32_t fill) {
  return __builtin_amdgcn_update_dpp(fill, v, CTRL, ROWS, 0xf, false);
}
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114,
              DPP_ROW_SHR8 = 0x118, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143,
              DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

// value of lane l-1 (lane 0: fill) / lane l+1 (lane 63: fill)
__device__ inline int32_t wave_shr1(int32_t v, int32_t fill) {
  return dpp_move<DPP_WAVE_SHR1>(v, fill);
}
__device__ inline int32_t wave_shl1(int32_t v, int32_t fill) {
  return dpp_move<DPP_WAVE_SHL1>(v, fill);
}
__device__ inline int32_t lane63(int32_t v) { return __builtin_amdgcn_readlane(v, 63); }

// inclusive prefix over lanes 0..l: Hillis-Steele within each row, then the
// row totals carried by the two broadcasts
#define TABI_WAVE_SCAN(OP, ID)                                  \
  v = OP(v, dpp_move<DPP_ROW_SHR1>(v, ID));                     \
  v = OP(v, dpp_move<DPP_ROW_SHR2>(v, ID));                     \
  v = OP(v, dpp_move<DPP_ROW_SHR4>(v, ID));                     \
  v = OP(v, dpp_move<DPP_ROW_SHR8>(v, ID));                     \
  v = OP(v, dpp_move<DPP_ROW_BCAST15, 0xa>(v, ID));             \
  v = OP(v, dpp_move<DPP_ROW_BCAST31, 0xc>(v, ID));
__device__ inline int32_t add32(int32_t a, int32_t b) { return a + b; }
__device__ inline int32_t max32(int32_t a, int32_t b) { return max(a, b); }
__device__ inline int32_t min32(int32_t a, int32_t b) { return min(a, b); }
__device__ inline int32_t wave_incl_sum(int32_t v) {
  TABI_WAVE_SCAN(add32, 0)
  return v;
}
__device__ inline int32_t wave_incl_max(int32_t v) {
  TABI_WAVE_SCAN(max32, -BIG)
  return v;
}
__device__ inline int32_t wave_incl_min(int32_t v) {
  TABI_WAVE_SCAN(min32, BIG)
  return v;
}
#undef TABI_WAVE_SCAN
__device__ inline int32_t wave_max(int32_t v) { return lane63(wave_incl_max(v)); }
__device__ inline int32_t wave_min(int32_t v) { return lane63(wave_incl_min(v)); }

// Segmented inclusive max over runs of equal keys, for keys that do not
// decrease across the valid lanes (lanes after them may hold any smaller
// key).  The keys of every step's source lane are computed once (SegKeys) and
// shared by the scans of several value arrays over the same segments.  A
// guarded step only combines lanes with equal keys; since keys are
// non-decreasing, a lane whose step source has another key has no earlier
// lane of its segment either, so the guarded scan is exact.
struct SegKeys {
  int32_t k1, k2, k4, k8, k15, k31;
};
__device__ inline SegKeys seg_keys(int32_t key) {
  constexpr int32_t NONE = -0x40000000;  // never a key
  SegKeys s;
  s.k1 = dpp_move<DPP_ROW_SHR1>(key, NONE);
  s.k2 = dpp_move<DPP_ROW_SHR2>(key, NONE);
  s.k4 = dpp_move<DPP_ROW_SHR4>(key, NONE);
  s.k8 = dpp_move<DPP_ROW_SHR8>(key, NONE);
  s.k15 = dpp_move<DPP_ROW_BCAST15, 0xa>(key, NONE);
  s.k31 = dpp_move<DPP_ROW_BCAST31, 0xc>(key, NONE);
  return s;
}
__device__ inline int32_t seg_scan_max(int32_t v, int32_t key, const SegKeys& s) {
  int32_t u;
  u = dpp_move<DPP_ROW_SHR1>(v, -BIG);
  v = s.k1 == key ? max(v, u) : v;
  u = dpp_move<DPP_ROW_SHR2>(v, -BIG);
  v = s.k2 == key ? max(v, u) : v;
  u = dpp_move<DPP_ROW_SHR4>(v, -BIG);
  v = s.k4 == key ? max(v, u) : v;
  u = dpp_move<DPP_ROW_SHR8>(v, -BIG);
  v = s.k8 == key ? max(v, u) : v;
  u = dpp_move<DPP_ROW_BCAST15, 0xa>(v, -BIG);
  v = s.k15 == key ? max(v, u) : v;
  u = dpp_move<DPP_ROW_BCAST31, 0xc>(v, -BIG);
  v = s.k31 == key ? max(v, u) : v;
  return v;
}

__device__ inline int64_t wave_max64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    int64_t u = __shfl_xor((long long)v, o);
    v = u > v ? u : v;
  }
  return v;
}
__device__ inline int64_t wave_min64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    int64_t u = __shfl_xor((long long)v, o);
    v = u < v ? u : v;
  }
  return v;
}
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
  return v;
}
__device__ inline uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }

}  // namespace tabi
