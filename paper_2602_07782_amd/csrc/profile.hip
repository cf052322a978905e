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
//              grown widths and heights (offsets within the segment)
//   k_alloc    one workgroup: segment bases in descending-scale priority
//   k_profile  per (scale slot, 16 charts): every grown column (top,
//              bottom) and every grown row (left, right) of each proxy, in
//              chunks spread over the wavefronts, then the neighbour pairs'
//              compacting distances and interlock flags
//
// Within a (atlas, slot) segment the charts' columns are stored back to back
// in sorted order, so the candidates of a row are one contiguous range and a
// row's texel e is word segbase + pcol[first chart] + e.  A segment that does
// not fit the arena is not stored (segbase = -1) and its consumers evaluate
// the proxies directly; results are the same either way.
#include "tabi_internal.h"
#include "pairs_dev.h"

namespace tabi {


constexpr int ALLOC_NT = 1024;
constexpr int PROF_NT = 256;
constexpr int PROF_GEN_BLOCKS = 1024;  // grid of the queued-block launch

// ---- a chart's per-scale record in the form the profile sweep evaluates ----
// Each slice rectangle (columns [c0, c1) x rows [r0, r1)) as pairs of 16-bit
// values, so that one set of two-lane integer operations tests an entry's
// column i and row j against it together:
//   lo = (c0, r0), span = (c1 - 1 - c0, r1 - 1 - r0): i lies in [c0, c1) iff
//   (i - c0) mod 2^16 <= c1 - 1 - c0, i.e. iff the saturating difference
//   x = (i - c0) -sat span is 0 (the same for j and the rows; an empty range
//   is lo = 2^15, span = 0, which no entry reaches);
//   vmin = (r0, c0), offset by 2^15 so that unsigned 16-bit min orders them
//   as the signed values, and vmaxc = (r1, c1) offset the same way and
//   complemented (2^16 - 1 - v), so that the max of the bottoms and rights
//   is also taken as a min: what the rectangle gives the column's top and
//   the row's left, the column's bottom and the row's right.
// x * (2^16 - 1) + v, saturated, is v inside and 2^16 - 1 (the min's
// identity) outside: one packed multiply-add with clamp per value.
// A chart of at most 16384 texels per side at the scale keeps every value
// and difference within 16 bits (entries lie in [-32, 16416)); larger charts,
// and OBB lines that need 64 bits, take the general evaluation.
struct alignas(16) SweepRect {
  uint32_t lo, span, vmin, vmaxc;
};
// An OBB side: split points, corner and last values, both lines in 32-bit
// form, and the single-precision reciprocals of their divisors (those the
// division takes, computed once).
struct alignas(16) SweepSide {
  int32_t sa, sb, corner, last;
  int32_t MA, nA, dA, MB, nB, dB;
  float rA, rB;
};
enum { SWEEP_AABB = 0, SWEEP_OBB = 1, SWEEP_GENERAL = 2 };
struct alignas(16) SweepRec {
  SweepRect rc[2 * KMAX];  // x-slices, then y-slices
  SweepSide sd[4];         // top, bottom, left, right
  int32_t mode, w, h, pad;
};

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pair16(int32_t a, int32_t b) {
  return (uint32_t)(uint16_t)a | ((uint32_t)(uint16_t)b << 16);
}
// per 16-bit half: min(a * b + c, 2^16 - 1), from the full-width product
__device__ inline uint32_t pk_mad_sat_u16(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_pk_mad_u16 %0, %1, %2, %3 clamp" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// Slice rectangle q of the chart (x-slices q < K, y-slices K + q) in sweep form.
__device__ inline SweepRect sweep_rect_of(const KView& kv, int q) {
  int32_t c0, c1, r0, r1;
  krect_load(kv.rc + q, c0, c1, r0, r1);
  const bool ce = c1 - 1 < c0, re = r1 - 1 < r0;  // empty ranges
  SweepRect r;
  r.lo = pair16(ce ? 0x8000 : c0, re ? 0x8000 : r0);
  r.span = pair16(ce ? 0 : c1 - 1 - c0, re ? 0 : r1 - 1 - r0);
  r.vmin = pair16(r0 ^ 0x8000, c0 ^ 0x8000);
  r.vmaxc = ~pair16(r1 ^ 0x8000, c1 ^ 0x8000);
  return r;
}

// OBB side sd of the chart (0 top, 1 bottom, 2 left, 3 right): its lines as
// column_row_bounds forms them; false when they need 64-bit evaluation.
__device__ inline bool sweep_side_of(const KView& kv, const Chart& ch, int k, int sd,
                                     SweepSide& o) {
  const int64_t C = kDirC[ch.m], S = kDirS[ch.m], kk = k;
  SideLines L;
  if (sd == 0) L = side_lines<false>(kk * ch.a, -QS * C, QS * S, kk * ch.e, QS * S, QS * C);
  else if (sd == 1) L = side_lines<true>(kk * ch.f, QS * S, QS * C, kk * ch.b, -QS * C, QS * S);
  else if (sd == 2) L = side_lines<false>(kk * ch.a, -QS * S, QS * C, -kk * ch.f, QS * C, QS * S);
  else L = side_lines<true>(-kk * ch.e, QS * C, QS * S, kk * ch.b, -QS * S, QS * C);
  const KSide ks = kside_load(kv.sd + sd);
  o.sa = ks.sa;
  o.sb = ks.sb;
  o.corner = ks.corner;
  o.last = ks.last;
  o.MA = L.MA; o.nA = L.nA; o.dA = L.dA;
  o.MB = L.MB; o.nB = L.nB; o.dB = L.dB;
  o.rA = __builtin_amdgcn_rcpf((float)L.dA);
  o.rB = __builtin_amdgcn_rcpf((float)L.dB);
  return L.ok;
}

// side_eval with the line data and reciprocal read from the sweep record.
// The whole record is loaded at once and every case is computed and then
// selected, so a side costs one shared-memory round trip and no branch.  The
// products run on the 24-bit multiplier: |n|, d <= 2^14 (a direction's
// cosine or sine in 2^14 units), |t| < 2^15 and |q| < 2^23 (|P| < 2^31,
// d >= 3196 for an OBB direction), and q * d is only needed modulo 2^32.
template <bool CEIL>
__device__ inline int32_t sweep_side(const SweepSide& s, int32_t t, int32_t n) {
  const int4 h0 = *reinterpret_cast<const int4*>(&s.sa);  // sa, sb, corner, last
  const int4 h1 = *reinterpret_cast<const int4*>(&s.MA);  // MA, nA, dA, MB
  const int4 h2 = *reinterpret_cast<const int4*>(&s.nB);  // nB, dB, rA, rB
  const bool useA = t + 1 <= h0.x, useB = t >= h0.y;
  const int32_t M = useA ? h1.x : h1.w, nn = useA ? h1.y : h2.x, d = useA ? h1.z : h2.y;
  const float rc = __int_as_float(useA ? h2.z : h2.w);
  const int32_t P = M + __mul24(nn, useA ? t + 1 : t);
  int32_t q = (int32_t)floorf((float)P * rc);
  const int32_t r = P - __mul24(q, d);
  q += r < 0 ? -1 : (r >= d ? 1 : 0);
  if (CEIL) q = -q;
  return t == n - 1 ? h0.w : ((useA || useB) ? q : h0.z);
}

// Top / bottom of column u and the per-proxy left / right of row u, as
// column_row_bounds computes them, from the sweep record (mode SWEEP_AABB or
// SWEEP_OBB).
template <int KT>
__device__ inline void sweep_bounds(const SweepRec& R, int32_t u, int32_t& top, int32_t& bot,
                                    int32_t& la, int32_t& ra, int32_t& lo, int32_t& ro) {
  const u16x2 ij = {(unsigned short)u, (unsigned short)u};
  const uint32_t ones = 0xffffffffu;
  // (top, left) minima and complemented (bottom, right) maxima of the x- and
  // y-slices; 0xffff means no rectangle contains the column (row)
  u16x2 mnx = {0xffff, 0xffff}, mcx = {0xffff, 0xffff}, mny = {0xffff, 0xffff},
        mcy = {0xffff, 0xffff};
#pragma unroll
  for (int q = 0; q < 2 * KT; ++q) {
    const uint4 v = *reinterpret_cast<const uint4*>(&R.rc[q]);
    // 0 inside, > 0 outside
    const u16x2 x = __builtin_elementwise_sub_sat(ij - __builtin_bit_cast(u16x2, v.x),
                                                  __builtin_bit_cast(u16x2, v.y));
    const uint32_t xb = __builtin_bit_cast(uint32_t, x);
    const u16x2 cmin = __builtin_bit_cast(u16x2, pk_mad_sat_u16(xb, ones, v.z));
    const u16x2 cmaxc = __builtin_bit_cast(u16x2, pk_mad_sat_u16(xb, ones, v.w));
    if (q < KT) {
      mnx = __builtin_elementwise_min(mnx, cmin);
      mcx = __builtin_elementwise_min(mcx, cmaxc);
    } else {
      mny = __builtin_elementwise_min(mny, cmin);
      mcy = __builtin_elementwise_min(mcy, cmaxc);
    }
  }
  // top = max(x, y tops), left = max(y, x lefts); bottom / right = min
  const u16x2 tl = __builtin_elementwise_max(mnx, mny);
  const u16x2 br = ~__builtin_elementwise_max(mcx, mcy);
  int32_t t = tl.x == 0xffff ? BIG : (int32_t)tl.x - 0x8000;
  int32_t l = tl.y == 0xffff ? BIG : (int32_t)tl.y - 0x8000;
  int32_t b = br.x == 0 ? -BIG : (int32_t)br.x - 0x8000;
  int32_t r = br.y == 0 ? -BIG : (int32_t)br.y - 0x8000;
  // the OBB's rows kept inside the chart's texel box [0, w]
  int32_t ol = 0, orr = R.w;
  if (R.mode == SWEEP_OBB) {
    t = max(t, sweep_side<false>(R.sd[0], u, R.w));
    b = min(b, sweep_side<true>(R.sd[1], u, R.w));
    ol = max(ol, sweep_side<false>(R.sd[2], u, R.h));
    orr = min(orr, sweep_side<true>(R.sd[3], u, R.h));
  }
  top = t;
  bot = b;
  la = l;
  ra = r;
  lo = ol;
  ro = orr;
}

// Segment placement in priority order: slot-major (every atlas's largest
// candidate scale first), so that when the arena runs out the segments left
// unstored are those of the smallest scales.  A segment is stored when it ends
// within the arena counting every segment before it.  One workgroup of NT
// threads; s_tot: NT / 64 entries of shared memory.
template <int NT>
__device__ void alloc_segments(const Params& P, const Work& w, int64_t* s_tot) {
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  const int64_t total = (int64_t)P.count * P.Br;  // this round's segments
  int64_t run = 0;
  for (int64_t q0 = 0; q0 < total; q0 += NT) {
    const int64_t q = q0 + tid;
    int64_t a = 0, s = 0, need = 0;
    if (q < total) {
      s = q / P.count;
      a = q - s * P.count;
      need = w.segneed[a * P.B + s];
    }
    int64_t inc = need;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int64_t u = __shfl_up((long long)inc, o);
      if (lane >= o) inc += u;
    }
    if (lane == WAVE - 1) s_tot[wv] = inc;
    __syncthreads();
    int64_t pre = 0, chunk = 0;
    for (int i = 0; i < NT / WAVE; ++i) {
      if (i < wv) pre += s_tot[i];
      chunk += s_tot[i];
    }
    if (q < total) {
      const int64_t end = run + pre + inc;
      w.segbase[a * P.B + s] = (need > 0 && end <= P.arena_cap) ? (int32_t)(end - need) : -1;
    }
    run += chunk;
    __syncthreads();
  }
}
__global__ __launch_bounds__(ALLOC_NT) void k_alloc(Params P, Work w, int round) {
  __shared__ int64_t s_tot[ALLOC_NT / WAVE];
  if (round_idle(w, round)) return;
  alloc_segments<ALLOC_NT>(P, w, s_tot);
}

// Offsets of every chart's grown columns and rows within its (atlas, slot)
// segment, and the segment's size in words (0 when the slot does not run).
// A chart's rows take two words each: its local-AABB rows, then its OBB rows.
template <int LAY_NT>
__global__ __launch_bounds__(LAY_NT) void k_layout(Params P, Work w, int round) {
  __shared__ int64_t s_tot[LAY_NT / WAVE][2];
  __shared__ int32_t s_last;
  if (round_idle(w, round)) return;
  const int a = w.aord[blockIdx.x], s = blockIdx.y;  // atlases with more charts first
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  const AtlasDesc d = w.desc[a];
  const bool run = P.fixed_k > 0 ? !d.bad : (!d.done && d.ktop >= 1);
  const int k = slot_k(P, d, round, s);
  if (!run || d.n <= 0 || k < 1) {
    if (tid == 0) w.segneed[(size_t)a * P.B + s] = 0;
  } else {
  const size_t slot = (size_t)s * P.N + d.c0;
  const int n = d.n, per = (n + LAY_NT - 1) / LAY_NT;
  const int t0 = min(n, tid * per), t1 = min(n, t0 + per);
  int64_t sw = 0, sh = 0;
  for (int t = t0; t < t1; ++t) {
    sw += w.wdv[slot + t];
    sh += 2 * w.hdv[slot + t];
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
  if (tid == 0) w.segneed[(size_t)a * P.B + s] = tw + th;
  // a segment larger than the arena is never stored, so offsets beyond the
  // int32 range are never used
  int64_t col = pw + iw - sw, row = tw + ph + ih - sh;
  for (int t = t0; t < t1; ++t) {
    w.pcol[slot + t] = (int32_t)min<int64_t>(col, 0x7fffffff);
    w.prow[slot + t] = (int32_t)min<int64_t>(row, 0x7fffffff);
    col += w.wdv[slot + t];
    row += 2 * w.hdv[slot + t];
  }
  }
  // Single atlas: the last of its workgroups to finish places the segments
  // (no separate launch); the counter is zeroed again for the packing
  // kernel, which counts with it next.  Batches launch the placement.
  if (P.count != 1) return;
  if (!last_to_finish(&w.cnt[0], P.Br, &s_last)) return;
  if (tid == 0) w.cnt[0] = 0;
  alloc_segments<LAY_NT>(P, w, &s_tot[0][0]);
}

// Stores the grown columns and rows of the workgroup's charts (KT slices per
// axis).  The work is split into items: chunk m of a chart covers grown
// columns and grown rows [m (G - p), (m + 1) (G - p)), both evaluated in the
// same pass by a group of G lanes (G = 16, 32 or 64, chosen per workgroup so
// that small charts do not leave most of a wavefront idle); the wavefronts
// take 64 / G items at a time, so a tall chart's chunks also run side by
// side.  s_ni is the exclusive prefix of the charts' item counts.  The gutter
// growth shifts values by one lane across the whole wavefront: a group's first
// p lanes only feed the others and are never stored, so no value crosses from
// one group into another's stored lanes.
template <int KT, bool GEN>
__device__ void profile_charts(const Work& w, const ChartCache* cache, const SweepRec* sw,
                               const int32_t* s_pc, const int32_t* s_pr, const int32_t* s_k,
                               const int32_t* s_ni, const int32_t* s_cols, int p, int G) {
  constexpr int NJ = PROF_CH + 1;
  const int wv = threadIdx.x / WAVE, lane = lane_id();
  const int per = WAVE / G, gi = lane / G, gl = lane - gi * G, step = G - p;
  const int total = s_ni[NJ];
  int j = 0;  // chart of the lane's item; items only move forward
  for (int it0 = wv * per; it0 < total; it0 += (PROF_NT / WAVE) * per) {
    const int it = it0 + gi;
    const bool live = it < total;
    // lanes past the last item evaluate the last item again (never stored),
    // so every lane reads a record that was copied
    const int itc = live ? it : total - 1;
    while (s_ni[j + 1] <= itc) ++j;
    const int m = itc - s_ni[j];
    const SweepRec& rec = sw[j];
    const int wt = rec.w, ht = rec.h;
    const int u = m * step - p + gl;  // undilated column and row of this lane
    int32_t tp = BIG, bt = -BIG, la = BIG, ra = -BIG, lo = BIG, ro = -BIG;
    {
      int32_t t1, b1, la1, ra1, lo1, ro1;
      if (!GEN || rec.mode != SWEEP_GENERAL)
        sweep_bounds<KT>(rec, u, t1, b1, la1, ra1, lo1, ro1);
      else
        column_row_bounds<KT>(kview(cache[j].kc, KT), cache[j].ch, s_k[j], u, u, t1, b1, la1,
                              ra1, lo1, ro1);
      if (u >= 0 && u < wt) { tp = t1; bt = b1; }
      if (u >= 0 && u < ht) { la = la1; ra = ra1; lo = lo1; ro = ro1; }
    }
    // gutter growth: after step q the lane holds the extremes over entries
    // [u - q, u] (the window of the lane before it, one entry longer); the
    // fill is each extreme's identity, so the move and the min / max fold
    // into one instruction.  Each proxy's rows grow on their own.
    int32_t T = tp, Bo = bt, LA = la, RA = ra, LO = lo, RO = ro;
    for (int q = 0; q < p; ++q) {
      T = min(T, wave_shr1(T, INT32_MAX));
      Bo = max(Bo, wave_shr1(Bo, INT32_MIN));
      LA = min(LA, wave_shr1(LA, INT32_MAX));
      RA = max(RA, wave_shr1(RA, INT32_MIN));
      LO = min(LO, wave_shr1(LO, INT32_MAX));
      RO = max(RO, wave_shr1(RO, INT32_MIN));
    }
    if (live && gl >= p) {
      if (s_cols[j] && u < wt + p) w.arena[s_pc[j] + u] = pack16(T, Bo + p);
      if (u < ht + p) {
        w.arena[s_pr[j] + u] = pack16(LA, RA + p);
        w.arena[s_pr[j] + ht + p + u] = pack16(LO, RO + p);
      }
    }
  }
}

// Grown bounds of PROF_CH charts of one scale slot per workgroup, then the
// compacting distance and interlock flags of their pairs with the preceding
// chart (Sec. 4.1.2; App. A "Detecting Interlocking Charts").  The charts'
// records, and the record of the chart before the first, are copied to LDS
// in one burst and their segment offsets loaded in parallel; the wavefronts
// evaluate chunks of them from LDS (charts are sorted by height, so few
// charts per workgroup keep the tallest ones from forming one long
// workgroup).  Lane l of a chunk evaluates undilated column
// (row) u = j0 - p + l; the gutter growth over [u-p, u] comes from p
// one-lane moves, so a chunk advances 64 - p entries (p <= 32).  After a barrier
// the pairs read the rows just stored; pairs in segments without stored
// profiles evaluate the rows from the LDS records.
// GEN: the block may hold charts without a sweep form or pairs without
// stored rows, evaluated from the proxy records (64-bit line arithmetic).
// Without it (the lean form, which needs far fewer registers and so runs at
// full occupancy) such a block is queued for profile_general instead and
// leaves; returns false then.
template <int KT, bool GEN>
__device__ bool profile_block(const Params& P, const Work& w, int bx, int s) {
  constexpr int NJ = PROF_CH + 1;  // entry 0: the chart before the block's first
  constexpr int K = KT;
  // 16-byte words of a chart record copied (the lean form reads only the
  // leading ones: extents, bits, OBB direction and bounds) and of its set-up
  // record (P.stride)
  constexpr int nch = GEN ? (int)(sizeof(Chart) / 16) : (int)((offsetof(Chart, ylo) + 15) / 16);
  constexpr int nkc = (int)((sizeof(KHead) + 4 * sizeof(KSide) + 2 * KT * sizeof(KRect)) / 16);
  __shared__ ChartCache cache[NJ];
  __shared__ SweepRec sw[NJ];
  __shared__ int32_t s_pc[NJ], s_pr[NJ], s_k[NJ], s_a[NJ], s_run[NJ], s_nc[NJ], s_ni[NJ + 1], s_G;
  __shared__ int32_t s_ok[NJ * 4];
  __shared__ int32_t s_gen;
  const int tid = threadIdx.x, wv = tid / WAVE, lane = lane_id();
  const int cb = bx * PROF_CH;
  // the charts' atlases, scales at this slot and offsets within their
  // segments: independent loads, issued together
  if (tid < NJ) {
    const int c = cb - 1 + tid;
    int32_t a = -1, kk = 0, oc = 0, orw = 0;
    if (c >= 0 && c < P.N) {
      const size_t sc = (size_t)s * P.N + c;
      a = w.chart_atlas[c];
      kk = w.kslot[sc];
      oc = w.pcol[sc];
      orw = w.prow[sc];
    }
    s_a[tid] = a;
    s_k[tid] = kk;
    s_pc[tid] = oc;
    s_pr[tid] = orw;
  }
  __syncthreads();
  // run bit 1: the chart runs at this slot; bit 2: it is the first chart of
  // its atlas (no pair before it); charts of an atlas are contiguous
  if (tid < NJ) s_run[tid] = (s_k[tid] > 0) | (tid > 0 && s_a[tid - 1] != s_a[tid] ? 2 : 0);
  // nothing to do when none of the block's charts runs at this slot (their
  // atlas is finished or its scale is out of range): leave before any copy
  const int active = tid >= 1 && tid < NJ && s_k[tid] > 0;
  if (!__syncthreads_or(active)) return true;
  // segment bases (they depend on the atlas) and the records of the running
  // charts are loaded together
  if (tid < NJ && s_k[tid] > 0) {
    const int32_t base = w.segbase[(size_t)s_a[tid] * P.B + s];
    s_pc[tid] = base >= 0 ? base + s_pc[tid] : -1;
    s_pr[tid] = base >= 0 ? base + s_pr[tid] : -1;
  } else if (tid < NJ) {
    s_pc[tid] = -1;
    s_pr[tid] = -1;
  }
  {
    constexpr int per = nch + nkc;
    const int j0 = cb > 0 ? 0 : 1, j1 = min(NJ, P.N - cb + 1);
    for (int i = tid; i < (j1 - j0) * per; i += PROF_NT) {
      const int j = j0 + i / per, r = i % per, c = cb - 1 + j;
      if (s_k[j] <= 0) continue;  // record not needed
      if (r < nch) {
        reinterpret_cast<int4*>(&cache[j].ch)[r] = reinterpret_cast<const int4*>(&w.srecs[c])[r];
      } else {
        reinterpret_cast<int4*>(cache[j].kc)[r - nch] =
            reinterpret_cast<const int4*>(w.kc + ((size_t)s * P.N + c) * P.stride)[r - nch];
      }
    }
  }
  __syncthreads();
  const int p = P.p;
  // the sweep form of every copied record: rectangles, and one thread per
  // (chart, OBB side) for the lines
  for (int i = tid; i < NJ * 2 * K; i += PROF_NT) {
    const int j = i / (2 * K), q = i - j * (2 * K);
    if (s_run[j] & 1) sw[j].rc[q] = sweep_rect_of(kview(cache[j].kc, K), q);
  }
  if (tid < NJ * 4 && (s_run[tid >> 2] & 1)) {
    const int j = tid >> 2;
    s_ok[tid] = sweep_side_of(kview(cache[j].kc, K), cache[j].ch, s_k[j], tid & 3, sw[j].sd[tid & 3]);
  }
  __syncthreads();
  if (wv == 0) {  // evaluation mode; lane group size, work items per chart and their prefix
    if (lane < NJ && (s_run[lane] & 1)) {
      const KHead hd = khead_load(kview(cache[lane].kc, K).hd);
      const bool lines = s_ok[4 * lane] && s_ok[4 * lane + 1] && s_ok[4 * lane + 2] &&
                         s_ok[4 * lane + 3];
      const bool fits = hd.w <= 16384 && hd.h <= 16384 && (!hd.obb || lines);
      sw[lane].mode = !fits ? SWEEP_GENERAL : (hd.obb ? SWEEP_OBB : SWEEP_AABB);
      sw[lane].w = hd.w;
      sw[lane].h = hd.h;
    }
    int e = 0;  // grown entries to evaluate (rows cover columns: h >= w)
    // the chart before the block is only needed for its rows, and only when
    // it belongs to the same atlas as the block's first chart (its columns
    // are stored by its own workgroup)
    if (lane < NJ && s_pc[lane] >= 0 && !(lane == 0 && (s_a[0] != s_a[1] || (s_run[1] & 2)))) {
      const KHead hd = khead_load(kview(cache[lane].kc, K).hd);
      e = max(hd.h, lane > 0 ? hd.w : 0) + p;
    }
    // lanes spent per group size: sum of chunks x G; a group needs p <= G / 2
    int G = WAVE;
    int best = lane63(wave_incl_sum((e + WAVE - p - 1) / (WAVE - p))) * WAVE;
    for (int g = 32; g >= 16; g >>= 1) {
      if (2 * p > g) break;
      const int cost = lane63(wave_incl_sum((e + g - p - 1) / (g - p))) * g;
      if (cost < best) { best = cost; G = g; }
    }
    const int ni = (e + G - p - 1) / (G - p);
    const int incl = wave_incl_sum(ni);
    if (lane < NJ) { s_nc[lane] = lane > 0; s_ni[lane + 1] = incl; }
    if (lane == 0) { s_ni[0] = 0; s_G = G; }
    // general evaluation needed: a chart with entries and no sweep form, or
    // a pair (with the chart before, same atlas) whose rows are not stored
    const bool gen_item = lane < NJ && e > 0 && sw[lane].mode == SWEEP_GENERAL;
    const bool gen_pair = lane >= 1 && lane < NJ && s_run[lane] == 1 && s_pr[lane] < 0;
    if (lane == 0) s_gen = 0;
    if (ballot64(gen_item || gen_pair) != 0 && lane == 0) s_gen = 1;
  }
  __syncthreads();
  if (!GEN && s_gen) return false;
  const int G = s_G;
  profile_charts<KT, GEN>(w, cache, sw, s_pc, s_pr, s_k, s_ni, s_nc, p, G);
  __syncthreads();  // the block's stored rows are visible to all its wavefronts
  // wavefront wv takes the pairs ending at charts 1 + 4 wv .. 4 + 4 wv: side
  // by side in its four 16-lane rows when all of them read stored rows, else
  // one at a time over the whole wavefront (rows evaluated from the records
  // where none are stored)
  const int jg = 1 + 4 * wv + (lane >> 4);
  const bool pg = (s_run[jg] & 1) && !(s_run[jg] & 2);  // a pair with the chart before
  if (!GEN || ballot64(pg && s_pr[jg] < 0) == 0) {
    int hdA = 0, hdB = 0, wdA = 0;
    const uint32_t* ra = w.arena;
    const uint32_t* rb = w.arena;
    if (pg) {
      const KHead ha = khead_load(kview(cache[jg - 1].kc, K).hd);
      hdA = ha.h + p;
      wdA = ha.w + p;
      hdB = khead_load(kview(cache[jg].kc, K).hd).h + p;
      ra = w.arena + s_pr[jg - 1];
      rb = w.arena + s_pr[jg];
    }
    const PairResult r = pair_rows_both<true>(ra, hdA, rb, hdB, wdA);
    if ((lane & 15) == 0 && (s_run[jg] & 1)) {
      const size_t sc = (size_t)s * P.N + (cb - 1 + jg);
      w.cd[sc] = pg ? r.cd : 0;
      w.fl[sc] = pg ? (uint8_t)r.flags : 0;
    }
  } else if constexpr (GEN) {
    for (int j = 1 + 4 * wv; j < 5 + 4 * wv; ++j) {
      const int run = s_run[j];
      if (!(run & 1)) continue;
      const size_t sc = (size_t)s * P.N + (cb - 1 + j);
      if (run & 2) {
        if (lane == 0) { w.cd[sc] = 0; w.fl[sc] = 0; }
        continue;
      }
      const KView A = kview(cache[j - 1].kc, K), B = kview(cache[j].kc, K);
      PairResult r;
      if (s_pr[j] >= 0) {
        r = pair_rows_both<false>(w.arena + s_pr[j - 1], khead_load(A.hd).h + p,
                                  w.arena + s_pr[j], khead_load(B.hd).h + p,
                                  khead_load(A.hd).w + p);
      } else {
        r = pair_records_both(A, cache[j - 1].ch, B, cache[j].ch, K, s_k[j], p);
      }
      if (lane == 0) {
        w.cd[sc] = r.cd;
        w.fl[sc] = (uint8_t)r.flags;
      }
    }
  }
  return true;
}

// Grown bounds and pairs of PROF_CH charts of one scale slot per workgroup
// (Sec. 4.1.2; App. A).  GEN false: the lean form, which queues the blocks
// that need the general evaluation (w.gq, counted in w.gq_cnt).
template <int KT, bool GEN>
__global__ __launch_bounds__(PROF_NT) void k_profile(Params P, Work w, int round) {
  if (round_idle(w, round)) return;
  if (!profile_block<KT, GEN>(P, w, blockIdx.x, blockIdx.y) && threadIdx.x == 0)
    w.gq[atomicAdd(w.gq_cnt, 1)] = (int32_t)(blockIdx.y * gridDim.x + blockIdx.x);
}

// The queued blocks, in full form, spread over a fixed grid.  The lean
// launch has finished, so these blocks' outputs are all written here.
template <int KT>
__global__ __launch_bounds__(PROF_NT) void k_profile_general(Params P, Work w, int round, int nbx) {
  if (round_idle(w, round)) return;
  const int nq = *w.gq_cnt;
  for (int i = blockIdx.x; i < nq; i += gridDim.x) {
    __syncthreads();  // the previous block's shared data is no longer read
    const int q = w.gq[i];
    profile_block<KT, true>(P, w, q % nbx, q / nbx);
  }
}

hipError_t launch_profiles(const Params& P, const Work& w, int round, hipStream_t st) {
  if (P.N <= 0) return hipSuccess;
  // with no arena the placement still runs: it marks every segment unstored
  // 256 threads per (atlas, slot) for a single atlas of up to 4,096 charts;
  // 1024 for larger ones and for batches, whose largest atlases hold thousands
  if (P.count == 1 && P.nmax <= 4096)
    hipLaunchKernelGGL(k_layout<256>, dim3(P.count, P.Br), dim3(256), 0, st, P, w, round);
  else
    hipLaunchKernelGGL(k_layout<1024>, dim3(P.count, P.Br), dim3(1024), 0, st, P, w, round);
  if (P.count != 1)  // a single atlas is placed by the last k_layout workgroup
    hipLaunchKernelGGL(k_alloc, dim3(1), dim3(ALLOC_NT), 0, st, P, w, round);
  const int nbx = (P.N + PROF_CH - 1) / PROF_CH;
  const dim3 grid(nbx, P.Br);
  // the lean form at full occupancy, then the queued blocks in full form
  // (the queue counter was cleared by the set-up kernel of this round); a
  // single atlas without stored profiles takes the full form at once
  if (P.count == 1 && P.arena_cap == 0) {
    if (P.K == 10) hipLaunchKernelGGL((k_profile<10, true>), grid, dim3(PROF_NT), 0, st, P, w, round);
    else if (P.K == 5) hipLaunchKernelGGL((k_profile<5, true>), grid, dim3(PROF_NT), 0, st, P, w, round);
    else if (P.K == 2) hipLaunchKernelGGL((k_profile<2, true>), grid, dim3(PROF_NT), 0, st, P, w, round);
    else hipLaunchKernelGGL((k_profile<1, true>), grid, dim3(PROF_NT), 0, st, P, w, round);
    return hipGetLastError();
  }
  // (a single atlas's queue is usually empty: a smaller grid leaves sooner)
  const dim3 ggrid(P.count == 1 ? PROF_GEN_BLOCKS / 4 : PROF_GEN_BLOCKS);
  if (P.K == 10) {
    hipLaunchKernelGGL((k_profile<10, false>), grid, dim3(PROF_NT), 0, st, P, w, round);
    hipLaunchKernelGGL(k_profile_general<10>, ggrid, dim3(PROF_NT), 0, st, P, w, round, nbx);
  } else if (P.K == 5) {
    hipLaunchKernelGGL((k_profile<5, false>), grid, dim3(PROF_NT), 0, st, P, w, round);
    hipLaunchKernelGGL(k_profile_general<5>, ggrid, dim3(PROF_NT), 0, st, P, w, round, nbx);
  } else if (P.K == 2) {
    hipLaunchKernelGGL((k_profile<2, false>), grid, dim3(PROF_NT), 0, st, P, w, round);
    hipLaunchKernelGGL(k_profile_general<2>, ggrid, dim3(PROF_NT), 0, st, P, w, round, nbx);
  } else {
    hipLaunchKernelGGL((k_profile<1, false>), grid, dim3(PROF_NT), 0, st, P, w, round);
    hipLaunchKernelGGL(k_profile_general<1>, ggrid, dim3(PROF_NT), 0, st, P, w, round, nbx);
  }
  return hipGetLastError();
}

}  // namespace tabi
