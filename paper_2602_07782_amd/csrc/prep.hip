// Per-chart proxy construction, sorting, the candidate-scale bound and the
// per-(scale, chart) rasterisation set-up.
//
//   k_init   atlas descriptors
//   k_prep   one wavefront per chart: AABB, quarter turn, area, local-AABB
//            slices (LDS atomics per edge), orientation, 8-direction OBB
//            (Sec. 4.1.1; App. A "Computing Local AABBs / OBBs / Orientations")
//   k_rank,  height-descending order within each atlas (Sec. 3.1, 4.3):
//   k_place  tiled rank counting, then a scatter
//   k_plan   largest candidate scale per atlas (area and largest chart fit)
//   k_setup  per (scale slot, chart): texel rectangles of the slices and the
//            OBB side split points used by per-texel evaluation, grown
//            extents
#include "tabi_internal.h"

namespace tabi {

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Descriptor of atlas a (the scale bound and the degenerate-chart flag come
// later, from k_plan).  Called by the first threads of the proxy (or
// records) kernel, or by k_init when there are no charts.
__device__ inline void init_desc(const Params& P, const Work& w, const int32_t* atlas_off,
                                 const int32_t* atlas_wh, int single_w, int single_h, int a) {
  AtlasDesc d;
  if (atlas_off) {
    d.c0 = atlas_off[a];
    d.n = atlas_off[a + 1] - atlas_off[a];
    d.Wa = atlas_wh[2 * a];
    d.Ha = atlas_wh[2 * a + 1];
  } else {
    d.c0 = 0;
    d.n = P.N;
    d.Wa = single_w;
    d.Ha = single_h;
  }
  d.ktop = 0;
  d.bad = 0;
  d.done = 0;
  d.kstar = 0;
  w.desc[a] = d;
  if (w.cnt) w.cnt[a] = 0;
  if (a == 0 && w.live)
    for (int r = 0; r <= MAX_ROUNDS; ++r) w.live[r] = 0;
}
__global__ void k_init(Params P, Work w, const int32_t* atlas_off, const int32_t* atlas_wh,
                       int single_w, int single_h) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < P.count) init_desc(P, w, atlas_off, atlas_wh, single_w, single_h, a);
}

// k_prep: one group of PREP_G lanes (a DPP row) per chart, PREP_CH charts
// per 256-thread block; charts have a few dozen vertices, so a whole
// wavefront per chart would leave most lanes idle and pay six-step 64-bit
// reductions over 64 lanes
constexpr int PREP_G = 16;
constexpr int PREP_CH = 256 / PREP_G;

// Reductions over the 16-lane row of the calling lane by row rotations
// (every lane of the row receives the result).
template <int R>
__device__ inline int32_t row_ror(int32_t v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + R, 0xf, 0xf, false);
}
template <int R>
__device__ inline int64_t row_ror64(int64_t v) {
  const uint32_t lo = (uint32_t)row_ror<R>((int32_t)(uint32_t)(uint64_t)v);
  const uint32_t hi = (uint32_t)row_ror<R>((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline int32_t row_min(int32_t v) {
  v = min(v, row_ror<8>(v)); v = min(v, row_ror<4>(v));
  v = min(v, row_ror<2>(v)); return min(v, row_ror<1>(v));
}
__device__ inline int32_t row_max(int32_t v) {
  v = max(v, row_ror<8>(v)); v = max(v, row_ror<4>(v));
  v = max(v, row_ror<2>(v)); return max(v, row_ror<1>(v));
}
__device__ inline int64_t row_min64(int64_t v) {
  int64_t u = row_ror64<8>(v); v = u < v ? u : v;
  u = row_ror64<4>(v); v = u < v ? u : v;
  u = row_ror64<2>(v); v = u < v ? u : v;
  u = row_ror64<1>(v); return u < v ? u : v;
}
__device__ inline int64_t row_max64(int64_t v) {
  int64_t u = row_ror64<8>(v); v = u > v ? u : v;
  u = row_ror64<4>(v); v = u > v ? u : v;
  u = row_ror64<2>(v); v = u > v ? u : v;
  u = row_ror64<1>(v); return u > v ? u : v;
}
__device__ inline uint64_t row_sum_u64(uint64_t v) {
  v += (uint64_t)row_ror64<8>((int64_t)v); v += (uint64_t)row_ror64<4>((int64_t)v);
  v += (uint64_t)row_ror64<2>((int64_t)v); return v + (uint64_t)row_ror64<1>((int64_t)v);
}

__device__ inline void slab_contrib(int32_t* lo, int32_t* hi, int K, int64_t E, int64_t a1,
                                    int64_t b1, int64_t a2, int64_t b2) {
  // a = slab axis coordinate, b = value; slabs are K*a in [jE, (j+1)E].
  // The local coordinates lie in [0, E] with 0 < E < 2^23, so K*a < 2^27 and
  // the slab indices come from 32-bit divisions (same quotients as 64-bit).
  const int64_t A1 = (int64_t)K * a1, A2 = (int64_t)K * a2;
  const int32_t e32 = (int32_t)E, a1s = (int32_t)A1, a2s = (int32_t)A2;
  // endpoint (a1, b1): the slab containing it, or both slabs at a slab line
  const int32_t q = a1s / e32, r = a1s - q * e32;
  int jh = min(q, K - 1);
  int jl = (r == 0) ? max(q - 1, 0) : jh;
  for (int j = jl; j <= jh; ++j) {
    atomicMin(&lo[j], (int32_t)b1);
    atomicMax(&hi[j], (int32_t)b1);
  }
  // crossings with interior slab lines strictly between the endpoints
  const int32_t mn = min(a1s, a2s), mx = max(a1s, a2s);
  int32_t m0 = mn / e32 + 1, m1 = (mx - 1) / e32;  // mx - 1 >= -1 truncates to 0
  if (m0 < 1) m0 = 1;
  if (m1 > K - 1) m1 = K - 1;
  for (int64_t m = m0; m <= m1; ++m) {
    int64_t num = b1 * (A2 - A1) + (b2 - b1) * (m * E - A1);
    int64_t den = A2 - A1;
    if (den < 0) { num = -num; den = -den; }
    int32_t f = (int32_t)fdiv53(num, den), c = (int32_t)cdiv53(num, den);
    atomicMin(&lo[m - 1], f); atomicMin(&lo[m], f);
    atomicMax(&hi[m - 1], c); atomicMax(&hi[m], c);
  }
}

__global__ __launch_bounds__(256) void k_prep(Params P, Work w, const int32_t* __restrict__ xy,
                                              const int32_t* __restrict__ voff,
                                              const int32_t* __restrict__ atlas_off,
                                              const int32_t* __restrict__ atlas_wh, int single_w,
                                              int single_h, const int32_t* __restrict__ cloop) {
  __shared__ int32_t sl[PREP_CH][4][KMAX];
  {  // atlas descriptors: thread i of the grid initialises atlas i
    const int ai = blockIdx.x * blockDim.x + threadIdx.x;
    if (w.desc && ai < P.count) init_desc(P, w, atlas_off, atlas_wh, single_w, single_h, ai);
  }
  const int g = threadIdx.x / PREP_G, lane = threadIdx.x % PREP_G;  // lane within the group
  const int base = lane_id() - lane;  // wavefront lane of the group's first lane
  const int c = blockIdx.x * PREP_CH + g;
  if (c >= P.N) return;  // whole group leaves; no block barrier below
  const int K = P.K;
  int a = 0;
  if (atlas_off) {  // atlas of this chart: last a with atlas_off[a] <= c
    int lo = 0, hi = P.count - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (atlas_off[mid] <= c) lo = mid; else hi = mid - 1;
    }
    a = lo;
  }
  const int local = c - (atlas_off ? atlas_off[a] : 0);
  if (lane == 0) w.chart_atlas[c] = a;
  // vertices of the chart: one loop (voff: chart vertex offsets), or its
  // loops [cloop[c], cloop[c+1]) when cloop is given (voff: loop vertex
  // offsets); each vertex's edge runs to the next vertex of its own loop
  const int l0 = cloop ? cloop[c] : 0, l1 = cloop ? cloop[c + 1] : 0;
  const int v0 = cloop ? voff[l0] : voff[c], nv = (cloop ? voff[l1] : voff[c + 1]) - v0;
  auto next_of = [&](int i) {
    if (!cloop) return (i + 1 == nv) ? 0 : i + 1;
    int l = l0;
    while (l + 1 < l1 && voff[l + 1] <= v0 + i) ++l;
    return (v0 + i + 1 == voff[l + 1]) ? voff[l] - v0 : i + 1;
  };
  int short_loop = 0;  // a loop of fewer than 3 vertices
  if (cloop)
    for (int l = l0 + lane; l < l1; l += PREP_G) short_loop |= voff[l + 1] - voff[l] < 3;
  const int2* V = reinterpret_cast<const int2*>(xy) + v0;

  int32_t xmn = BIG, xmx = -BIG, ymn = BIG, ymx = -BIG;
  int range_bad = 0;
  for (int i = lane; i < nv; i += PREP_G) {
    int2 p = V[i];
    if (p.x <= -(1 << 22) || p.x >= (1 << 22) || p.y <= -(1 << 22) || p.y >= (1 << 22)) range_bad = 1;
    xmn = min(xmn, p.x); xmx = max(xmx, p.x);
    ymn = min(ymn, p.y); ymx = max(ymx, p.y);
  }
  xmn = row_min(xmn); xmx = row_max(xmx);
  ymn = row_min(ymn); ymx = row_max(ymx);
  range_bad = row_max(range_bad | short_loop);
  const int32_t W0 = xmx - xmn, H0 = ymx - ymn;
  Chart* out = &w.recs[c];
  if (nv < 3 || range_bad || W0 <= 0 || H0 <= 0) {
    if (lane == 0) {
      out->valid = 0;
      out->src = local;
      w.keys[c] = ((uint64_t)0x7fffff << 41) | ((uint64_t)0x7fffff << 18) | (uint64_t)local;
      if (w.rank) w.rank[c] = 0;
      if (w.pl) w.pl[c] = make_int4(0, 0, 0, -1);
    }
    return;
  }
  // quarter turn so the box is at least as tall as wide: (u,v) -> (H0 - v, u)
  const bool rot = W0 > H0;
  const int32_t W = rot ? H0 : W0, H = rot ? W0 : H0;
  auto local_uv = [&](int i, int64_t& u, int64_t& v) {
    int2 p = V[i];
    int64_t u0 = p.x - xmn, vv = p.y - ymn;
    if (rot) { u = H0 - vv; v = u0; } else { u = u0; v = vv; }
  };

  int32_t* ylo = sl[g][0];
  int32_t* yhi = sl[g][1];
  int32_t* xlo = sl[g][2];
  int32_t* xhi = sl[g][3];
  if (lane < K) { ylo[lane] = BIG; yhi[lane] = -BIG; xlo[lane] = BIG; xhi[lane] = -BIG; }
  wave_sync();

  uint64_t area = 0;
  for (int i = lane; i < nv; i += PREP_G) {
    const int i2 = next_of(i);
    int64_t u1, v1, u2, v2;
    local_uv(i, u1, v1);
    local_uv(i2, u2, v2);
    area += (uint64_t)(u1 * v2) - (uint64_t)(u2 * v1);
    slab_contrib(ylo, yhi, K, W, u1, v1, u2, v2);  // x-slices: slab axis u
    slab_contrib(xlo, xhi, K, H, v1, u1, v2, u2);  // y-slices: slab axis v
  }
  area = row_sum_u64(area);
  int64_t area2 = (int64_t)area;
  if (area2 < 0) area2 = -area2;
  if (cloop && l1 - l0 > 1) {
    // several loops: the largest loop's area less every other loop's (exact
    // for an outer loop with holes, a lower bound otherwise, which keeps the
    // area bound on the scale rigorous)
    int64_t amax = 0, arest = 0;
    for (int l = l0; l < l1; ++l) {
      uint64_t al = 0;
      for (int i = voff[l] - v0 + lane; i < voff[l + 1] - v0; i += PREP_G) {
        const int i2 = (v0 + i + 1 == voff[l + 1]) ? voff[l] - v0 : i + 1;
        int64_t u1, v1, u2, v2;
        local_uv(i, u1, v1);
        local_uv(i2, u2, v2);
        al += (uint64_t)(u1 * v2) - (uint64_t)(u2 * v1);
      }
      int64_t a = (int64_t)row_sum_u64(al);
      if (a < 0) a = -a;
      if (a > amax) { arest += amax; amax = a; }
      else arest += a;
    }
    area2 = amax > arest ? amax - arest : 0;
  }
  wave_sync();

  // orientation: lanes j < K hold slice j.  A slice that meets no loop
  // (only between islands of one chart: a connected loop meets every slice)
  // takes the slice's whole box, a conservative local AABB.
  int32_t sylo = 0, syhi = 0, sxlo = 0, sxhi = 0;
  if (lane < K) { sylo = ylo[lane]; syhi = yhi[lane]; sxlo = xlo[lane]; sxhi = xhi[lane]; }
  if (sylo > syhi) { sylo = 0; syhi = H; }
  if (sxlo > sxhi) { sxlo = 0; sxhi = W; }
  const bool in = lane < K;
  // empty area above the top boundary vs below the bottom boundary
  int64_t top_area = (int64_t)row_sum_u64(in ? (uint64_t)(int64_t)sylo : 0);
  int64_t bot_area = (int64_t)row_sum_u64(in ? (uint64_t)(int64_t)(H - syhi) : 0);
  const bool flipy = top_area > bot_area;
  if (flipy) {
    int32_t l2 = H - syhi, h2 = H - sylo;
    sylo = l2; syhi = h2;
    const int src = base + (in ? K - 1 - lane : 0);
    int32_t a1 = __shfl(sxlo, src), a2 = __shfl(sxhi, src);
    if (in) { sxlo = a1; sxhi = a2; }
  }
  int64_t Ls = (int64_t)row_sum_u64(in ? (uint64_t)(int64_t)sxlo : 0);
  int64_t Rs = (int64_t)row_sum_u64(in ? (uint64_t)(int64_t)(W - sxhi) : 0);
  const int half = K / 2;
  int64_t BL = (int64_t)row_sum_u64((lane < half) ? (uint64_t)(int64_t)(H - syhi) : 0);
  int64_t BR = (int64_t)row_sum_u64((lane >= K - half && in) ? (uint64_t)(int64_t)(H - syhi) : 0);
  int64_t diff = Ls - Rs;
  bool flipx;
  if (10 * diff > (int64_t)K * W) flipx = true;
  else if (10 * (diff < 0 ? -diff : diff) <= (int64_t)K * W) flipx = BL > BR;
  else flipx = false;
  if (flipx) {
    const int src = base + (in ? K - 1 - lane : 0);
    int32_t a1 = __shfl(sylo, src), a2 = __shfl(syhi, src);
    if (in) { sylo = a1; syhi = a2; }
    int32_t l2 = W - sxhi, h2 = W - sxlo;
    sxlo = l2; sxhi = h2;
  }

  // approximate OBB of the chart as packed (after the reflections)
  int64_t pmin[8], pmax[8], qmin[8], qmax[8];
#pragma unroll
  for (int m = 1; m < 8; ++m) { pmin[m] = INT64_MAX; pmax[m] = INT64_MIN; qmin[m] = INT64_MAX; qmax[m] = INT64_MIN; }
  for (int i = lane; i < nv; i += PREP_G) {
    int64_t u, v;
    local_uv(i, u, v);
    if (flipx) u = W - u;
    if (flipy) v = H - v;
#pragma unroll
    for (int m = 1; m < 8; ++m) {
      const int64_t C = kDirC[m], S = kDirS[m];
      int64_t pp = C * u + S * v, qq = C * v - S * u;
      pmin[m] = min(pmin[m], pp); pmax[m] = max(pmax[m], pp);
      qmin[m] = min(qmin[m], qq); qmax[m] = max(qmax[m], qq);
    }
  }
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    pmin[m] = row_min64(pmin[m]); pmax[m] = row_max64(pmax[m]);
    qmin[m] = row_min64(qmin[m]); qmax[m] = row_max64(qmax[m]);
  }
  // smallest area (b-a)(f-e)/(C^2+S^2), exact; ties keep the smaller m
  int best = 0;
  unsigned __int128 bext = (unsigned __int128)((uint64_t)QS * W) * (uint64_t)(QS * H);
  unsigned __int128 bN = (unsigned __int128)(QS * QS);
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    const uint64_t C = kDirC[m], S = kDirS[m];
    unsigned __int128 ext = (unsigned __int128)(uint64_t)(pmax[m] - pmin[m]) * (uint64_t)(qmax[m] - qmin[m]);
    unsigned __int128 N = (unsigned __int128)(C * C + S * S);
    if (ext * bN < bext * N) { best = m; bext = ext; bN = N; }
  }
  if (P.variant == 2) best = 0;  // balanced-only: the chart's box alone
  int64_t ba = 0, bb = 0, be = 0, bf = 0;
#pragma unroll
  for (int m = 1; m < 8; ++m)
    if (m == best) { ba = pmin[m]; bb = pmax[m]; be = qmin[m]; bf = qmax[m]; }

  if (in) {
    out->ylo[lane] = sylo; out->yhi[lane] = syhi;
    out->xlo[lane] = sxlo; out->xhi[lane] = sxhi;
  }
  if (lane == 0) {
    out->W = W;
    out->H = H;
    out->bits = (rot ? 1 : 0) | (flipx ? 2 : 0) | (flipy ? 4 : 0);
    out->m = best;
    out->a = ba; out->b = bb; out->e = be; out->f = bf;
    out->area2 = area2;
    out->src = local;
    out->valid = 1;
    // ascending key = height descending, width descending, input index
    w.keys[c] = ((uint64_t)(0x7fffff - H) << 41) | ((uint64_t)(0x7fffff - W) << 18) | (uint64_t)local;
    if (w.rank) w.rank[c] = 0;
    if (w.pl) w.pl[c] = make_int4((int32_t)(uint32_t)area2, (int32_t)((uint64_t)area2 >> 32), W, H);
  }
}

// Rank of each chart's key inside its atlas (keys are unique), then scatter
// to the sorted position.  Workgroup (x, y) holds the 256 charts of tile x
// and streams key tiles y, y + gridDim.y, ... of the union of the atlases
// those charts belong to through LDS; every thread counts the smaller keys
// of its own atlas and adds the count to its rank (integer atomics: the sum
// does not depend on the order).  Ranks start at zero (written with the keys).
// Atlases of up to RANK_DIRECT charts compare every key of a tile; larger
// ones first sort each aligned key tile by (atlas, key) (k_tile_sort) and
// then count with two binary searches per tile.
constexpr int RANK_DIRECT = 256;
constexpr int RANK_SCATTER = 256;

// Bitonic sort of key tile blockIdx.x, ascending by (atlas, key), into
// skey / satl; entries past N are the largest.
// A single atlas's scale plan does not depend on the sort: it runs as the
// extra workgroup plan_block (-1: none) of the sort's first launch.
template <int PLAN_NT>
__device__ void plan_atlas(const Params& P, const Work& w, int a);

__global__ __launch_bounds__(256) void k_tile_sort(Params P, Work w, int plan_block) {
  __shared__ uint64_t sk[256];
  __shared__ int32_t sa[256];
  if ((int)blockIdx.x == plan_block) {
    plan_atlas<256>(P, w, 0);
    return;
  }
  const int t = threadIdx.x, i = blockIdx.x * 256 + t;
  sk[t] = i < P.N ? w.keys[i] : ~0ull;
  sa[t] = i < P.N ? w.chart_atlas[i] : INT32_MAX;
  __syncthreads();
  for (int k = 2; k <= 256; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int u = t ^ j;
      if (u > t) {
        const int32_t a0 = sa[t], a1 = sa[u];
        const uint64_t k0 = sk[t], k1 = sk[u];
        const bool gt = a0 > a1 || (a0 == a1 && k0 > k1);
        if (gt == ((t & k) == 0)) {  // ascending where bit k of t is clear
          sa[t] = a1; sa[u] = a0;
          sk[t] = k1; sk[u] = k0;
        }
      }
      __syncthreads();
    }
  }
  w.skey[i] = sk[t];
  w.satl[i] = sa[t];
}

// entries of a sorted tile before (a, k)
__device__ inline int tile_lower_bound(const int32_t* ta, const uint64_t* tk, int32_t a,
                                       uint64_t k) {
  int pos = 0;
#pragma unroll
  for (int step = 256; step > 0; step >>= 1) {
    const int x = pos + step - 1;
    if (x < 256 && (ta[x] < a || (ta[x] == a && tk[x] < k))) pos += step;
  }
  return pos;
}

// SCATTER: one workgroup per chart tile walks every key tile of its atlases,
// so each rank is complete in its thread, which writes the chart to its
// sorted position (no k_place launch); otherwise ranks accumulate by atomics
// over the grid's y dimension and k_place scatters.
template <bool SORTED, bool SCATTER>
__global__ __launch_bounds__(256) void k_rank(Params P, Work w, int plan_block) {
  __shared__ uint64_t tile[256];
  __shared__ int32_t tatl[256];
  __shared__ int s_lo, s_hi;
  if ((int)blockIdx.x == plan_block) {  // the extra column: one workgroup plans
    if (blockIdx.y == 0) plan_atlas<256>(P, w, 0);
    return;
  }
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = c < P.N;
  int lo = 0, hi = 0, a = 0;
  uint64_t key = 0;
  if (act) {
    a = w.chart_atlas[c];
    const AtlasDesc d = w.desc[a];
    lo = d.c0;
    hi = d.c0 + d.n;
    key = w.keys[c];
  }
  if (threadIdx.x == 0) s_lo = lo;
  const int last = min(P.N, (int)(blockIdx.x + 1) * (int)blockDim.x) - 1;
  if (c == last) s_hi = hi;
  __syncthreads();
  const int blo = s_lo, bhi = s_hi;
  int rank = 0;
  if (SORTED) {
    // the aligned sorted tiles that overlap the block's atlases
    for (int t = blo / 256 + (int)blockIdx.y; t * 256 < bhi; t += (int)gridDim.y) {
      tile[threadIdx.x] = w.skey[t * 256 + threadIdx.x];
      tatl[threadIdx.x] = w.satl[t * 256 + threadIdx.x];
      __syncthreads();
      if (act) rank += tile_lower_bound(tatl, tile, a, key) - tile_lower_bound(tatl, tile, a, 0);
      __syncthreads();
    }
  } else {
    for (int base = blo + (int)blockIdx.y * 256; base < bhi; base += (int)gridDim.y * 256) {
      const int i = base + threadIdx.x;
      tile[threadIdx.x] = i < bhi ? w.keys[i] : ~0ull;
      __syncthreads();
      if (act) {
        const int j0 = max(lo - base, 0), j1 = min(hi - base, 256);
        if (j0 == 0 && j1 == 256) {  // a whole tile of this atlas: reads kept in flight
          int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
#pragma unroll 8
          for (int j = 0; j < 256; j += 4) {
            r0 += tile[j] < key;
            r1 += tile[j + 1] < key;
            r2 += tile[j + 2] < key;
            r3 += tile[j + 3] < key;
          }
          rank += r0 + r1 + r2 + r3;
        } else {
          for (int j = j0; j < j1; ++j) rank += tile[j] < key;
        }
      }
      __syncthreads();
    }
  }
  if (SCATTER) {
    if (act) {
      const int pos = lo + rank;
      w.srecs[pos] = w.recs[c];
      w.perm[pos] = c - lo;
    }
  } else if (act && rank) {
    atomicAdd(&w.rank[c], rank);
  }
}

__global__ __launch_bounds__(256) void k_place(Params P, Work w) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.N) return;
  const int lo = w.desc[w.chart_atlas[c]].c0;
  const int pos = lo + w.rank[c];
  w.srecs[pos] = w.recs[c];
  w.perm[pos] = c - lo;
}

// candidate scales: the charts' total area and the largest chart must fit,
// and so must the charts' grown footprints.  At scale s = k/64 the texels a
// chart is packed as (its proxies' per-texel bounds) cover the chart, so at
// least a s^2 of them (a its area), and reach every column and row of its
// w x h texel box; the gutter growth adds at least p texels to every row of
// them (past the rightmost) and then p to every column of the result (w + p
// columns), so the grown footprint covers at least a s^2 + p (w + h) + p^2
// texels.  A packing's grown footprints are disjoint inside the
// (W+p) x (H+p) grown atlas, hence, with w, h >= s W, s H (W, H the box in
// Q8) and everything times 2^29:
//   sum(area2) k^2 + 2^15 p k sum(W + H) + 2^29 n p^2 <= 2^29 (W+p)(H+p).
// (For charts of several loops only the area and p^2 terms are used.)  Both
// bounds are exact prunes: they never remove a scale whose packing succeeds.
// Per-thread sums stay below 2^57 (area2 < 2^47, at most 1,024 charts per
// thread) and a wavefront's below 2^63; the block total is taken in 128 bits.
// Lane k - 1 of wavefront 0 tests scale k; k_top is the largest passing one.
constexpr int ORDER_MAX = 4096;  // largest batch whose atlases are reordered for packing
// PLAN_NT threads per atlas: 256 up to 1,024 charts, 1024 above
template <int PLAN_NT>
__device__ void plan_atlas(const Params& P, const Work& w, int a) {
  constexpr int PW = PLAN_NT / WAVE;
  __shared__ uint64_t s_sum[PW], s_before[PW], s_wh[PW];
  __shared__ int32_t s_maxw[PW], s_maxh[PW], s_bad[PW];
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const AtlasDesc d = w.desc[a];
  uint64_t sum = 0, wh = 0;  // wh: sum of W + H (Q8), below 2^42
  int32_t mw = 0, mh = 0, bad = 0;  // bad: a degenerate chart
#pragma unroll 4
  for (int t = threadIdx.x; t < d.n; t += blockDim.x) {
    const int4 q = w.pl[d.c0 + t];  // the atlas's charts in input order (the sums do not care)
    if (q.w < 0) {
      bad = 1;
    } else {
      sum += ((uint64_t)(uint32_t)q.y << 32) | (uint32_t)q.x;
      wh += (uint64_t)q.z + (uint64_t)q.w;
      mw = max(mw, q.z);
      mh = max(mh, q.w);
    }
  }
  // the packing kernel takes the atlases with more charts first (their
  // searches take longest, so they should not start last), ties by index;
  // a batch of more than ORDER_MAX atlases keeps its own order
  uint64_t before = 0;
  if (P.count <= ORDER_MAX)
    for (int b = threadIdx.x; b < P.count; b += blockDim.x) {
      const int nb = w.desc[b].n;
      before += (nb > d.n || (nb == d.n && b < a)) ? 1 : 0;
    }
  sum = wave_sum_u64(sum);
  wh = wave_sum_u64(wh);
  before = wave_sum_u64(before);
  mw = wave_max(mw);
  mh = wave_max(mh);
  bad = wave_max(bad);
  if (lane == 0) {
    s_sum[wv] = sum;
    s_wh[wv] = wh;
    s_maxw[wv] = mw;
    s_maxh[wv] = mh;
    s_bad[wv] = bad;
    s_before[wv] = before;
  }
  __syncthreads();
  if (wv != 0) return;
  if (lane == 0) {
    uint64_t pos = 0;
    for (int q = 0; q < PW; ++q) pos += s_before[q];
    w.aord[P.count <= ORDER_MAX ? (int)pos : a] = a;
  }
  unsigned __int128 S = 0;
  uint64_t SWH = 0;
  int32_t MW = 0, MH = 0;
  bad = 0;
  for (int q = 0; q < PW; ++q) {
    S += s_sum[q];
    SWH += s_wh[q];
    MW = max(MW, s_maxw[q]);
    MH = max(MH, s_maxh[q]);
    bad |= s_bad[q];
  }
  int ktop = 0;
  if (bad) {
    ktop = -1;
  } else if (d.n == 0) {
    ktop = 64;
  } else {
    const unsigned __int128 cap = ((unsigned __int128)1 << 29) * (unsigned)d.Wa * (unsigned)d.Ha;
    const int k = lane + 1;
    const bool area_ok = S * (unsigned)(k * k) <= cap;
    const bool fit = cdiv64((int64_t)k * MW, QS) <= d.Wa && cdiv64((int64_t)k * MH, QS) <= d.Ha;
    const uint64_t pp = (uint64_t)P.p;
    const unsigned __int128 grown =
        S * (unsigned)(k * k) +
        (P.loops ? 0 : ((unsigned __int128)(pp * (uint64_t)k) * SWH << 15)) +
        ((unsigned __int128)((uint64_t)d.n * pp * pp) << 29);
    const unsigned __int128 gcap =
        ((unsigned __int128)((uint64_t)(d.Wa + P.p) * (uint64_t)(d.Ha + P.p))) << 29;
    const uint64_t pass = ballot64(area_ok && fit && grown <= gcap);
    ktop = pass ? 64 - __builtin_clzll(pass) : 0;
    // the hybrid tail packs its charts at a smaller scale, so neither bound
    // holds for the scale of the rows before it: every scale is a candidate
    if (P.hybrid) ktop = 64;
  }
  if (lane == 0) {
    w.desc[a].ktop = ktop;
    w.desc[a].bad = bad;
    if (P.hybrid) {  // the total area, for the choice among the hybrid packs
      w.tail_obj[2 * P.B] = (uint64_t)S;
      w.tail_obj[2 * P.B + 1] = (uint64_t)(S >> 64);
    }
  }
}
template <int PLAN_NT>
__global__ __launch_bounds__(PLAN_NT) void k_plan(Params P, Work w) {
  plan_atlas<PLAN_NT>(P, w, blockIdx.x);
}

// one thread per (slot, chart)
// The record of chart c at slot s, written to `base` (LDS); returns the
// slot's scale k, 0 when the chart does not run at this slot.
template <int KT>
__device__ int32_t setup_record(const Params& P, const Work& w, int round, int c, int s,
                             unsigned char* base) {
  const AtlasDesc d = w.desc[w.chart_atlas[c]];
  const bool run = P.fixed_k > 0 ? !d.bad : (!d.done && d.ktop >= 1);
  if (!run) return 0;
  const int k = slot_k(P, d, round, s);
  if (k < 1) return 0;
  const Chart& ch = w.srecs[c];
  int32_t wt, ht;
  build_krec<KT>(ch, k, base, wt, ht);
  const size_t sc = (size_t)s * P.N + c;
  w.wdv[sc] = wt + P.p;
  w.hdv[sc] = ht + P.p;
  if (s == 0) w.Hs[c] = ch.H;
  return k;
}

// Records are built in LDS by their threads and written out together with
// coalesced 16-byte stores (one thread writing its own 16 + 64 + 16K bytes
// field by field would cost a memory transaction per field).
constexpr int SETUP_NT = 128;
template <int KT>
__global__ __launch_bounds__(SETUP_NT) void k_setup(Params P, Work w, int round) {
  __shared__ __align__(16) unsigned char s_rec[SETUP_NT * KREC_MAX];
  if (round_idle(w, round)) return;
  // the round's slots of one chart range run on one XCD (blocks are dealt
  // to the XCDs in turn), one after another, so the chart records they all
  // read come from that XCD's L2 after the first; the grid is padded to a
  // multiple of XCDS chart ranges
  const int xcd = blockIdx.x % XCDS, j = blockIdx.x / XCDS;
  const int s = j % P.Br, cblk = (j / P.Br) * XCDS + xcd;
  if (cblk * SETUP_NT >= P.N) return;
  const int c = cblk * blockDim.x + threadIdx.x;
  const int32_t k = c < P.N ? setup_record<KT>(P, w, round, c, s, s_rec + threadIdx.x * P.stride) : 0;
  if (c < P.N) w.kslot[(size_t)s * P.N + c] = k;  // read by the profile kernel
  if (c == 0 && s == 0) *w.gq_cnt = 0;  // the profile kernel's queue of this round
  const bool active = k > 0;
  if (!__syncthreads_or(active)) return;  // no chart of the block runs at this slot
  const int c0 = cblk * blockDim.x, nc = min(SETUP_NT, P.N - c0);
  const int n16 = nc * (P.stride / 16);
  const int4* src = reinterpret_cast<const int4*>(s_rec);
  int4* dst = reinterpret_cast<int4*>(w.kc + ((size_t)s * P.N + c0) * P.stride);
  for (int i = threadIdx.x; i < n16; i += SETUP_NT) dst[i] = src[i];
}

// Start of the packing path from resident proxy records: copy, keys, atlas
// of each chart, degenerate flags.
__global__ __launch_bounds__(256) void k_from_records(Params P, Work w, const Chart* __restrict__ in,
                                                      const int32_t* __restrict__ atlas_off,
                                                      const int32_t* __restrict__ atlas_wh) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P.count) init_desc(P, w, atlas_off, atlas_wh, 0, 0, c);
  if (c >= P.N) return;
  int lo = 0, hi = P.count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (atlas_off[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int a = lo;
  const Chart ch = in[c];
  w.recs[c] = ch;
  w.chart_atlas[c] = a;
  const uint64_t local = (uint64_t)ch.src;
  w.rank[c] = 0;
  if (ch.valid) {
    w.keys[c] = ((uint64_t)(0x7fffff - ch.H) << 41) | ((uint64_t)(0x7fffff - ch.W) << 18) | local;
    w.pl[c] = make_int4((int32_t)(uint32_t)ch.area2, (int32_t)((uint64_t)ch.area2 >> 32), ch.W, ch.H);
  } else {
    w.keys[c] = ((uint64_t)0x7fffff << 41) | ((uint64_t)0x7fffff << 18) | local;
    w.pl[c] = make_int4(0, 0, 0, -1);
  }
}

// dst[idx[i]] = src[i], keeping the replaced chart's input index
__global__ __launch_bounds__(256) void k_splice(Chart* __restrict__ dst, const int32_t* __restrict__ idx,
                                                int m, const Chart* __restrict__ src) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int j = idx[i];
  Chart c = src[i];
  c.src = dst[j].src;
  dst[j] = c;
}

// Records of a serving batch: request r owns charts [aoff[r], aoff[r+1]) of
// the batch.  A re-pack (src_res[r] != 0) starts from its atlas's resident
// records, a new atlas from its freshly prepared records at poff[r]; every
// record is also written to the request's new resident block dst_res[r].
__global__ __launch_bounds__(256) void k_assemble(int N, int count, const int32_t* __restrict__ aoff,
                                                  const int32_t* __restrict__ poff,
                                                  const uint64_t* __restrict__ src_res,
                                                  const uint64_t* __restrict__ dst_res,
                                                  const Chart* __restrict__ prep, Chart* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  int lo = 0, hi = count - 1;  // last r with aoff[r] <= c
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (aoff[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int t = c - aoff[lo];
  const Chart* src = reinterpret_cast<const Chart*>(src_res[lo]);
  const Chart ch = src ? src[t] : prep[poff[lo] + t];
  out[c] = ch;
  reinterpret_cast<Chart*>(dst_res[lo])[t] = ch;
}

// The replaced charts of the re-packs: prepared record i of request r
// (i in [poff[r], poff[r+1])) replaces chart idx[i] of the request, which
// keeps its input index.
__global__ __launch_bounds__(256) void k_assemble_splice(int M, int count,
                                                         const int32_t* __restrict__ aoff,
                                                         const int32_t* __restrict__ poff,
                                                         const uint64_t* __restrict__ src_res,
                                                         const uint64_t* __restrict__ dst_res,
                                                         const int32_t* __restrict__ idx,
                                                         const Chart* __restrict__ prep,
                                                         Chart* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  int lo = 0, hi = count - 1;  // last r with poff[r] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (poff[mid] <= i) lo = mid; else hi = mid - 1;
  }
  if (!src_res[lo]) return;  // a new atlas: already in place
  const int j = idx[i];
  Chart ch = prep[i];
  ch.src = j;
  out[aoff[lo] + j] = ch;
  reinterpret_cast<Chart*>(dst_res[lo])[j] = ch;
}

hipError_t launch_assemble(int N, int M, int count, const int32_t* aoff, const int32_t* poff,
                           const uint64_t* src_res, const uint64_t* dst_res, const int32_t* idx,
                           const Chart* prep, Chart* out, hipStream_t st) {
  if (N > 0)
    hipLaunchKernelGGL(k_assemble, dim3((N + 255) / 256), dim3(256), 0, st, N, count, aoff, poff,
                       src_res, dst_res, prep, out);
  if (M > 0)
    hipLaunchKernelGGL(k_assemble_splice, dim3((M + 255) / 256), dim3(256), 0, st, M, count, aoff,
                       poff, src_res, dst_res, idx, prep, out);
  return hipGetLastError();
}

hipError_t launch_from_records(const Params& P, const Work& w, const Chart* in,
                               const int32_t* atlas_off, const int32_t* atlas_wh, hipStream_t st) {
  // the records kernel also writes the atlas descriptors
  if (P.N > 0)
    hipLaunchKernelGGL(k_from_records, dim3((max(P.N, P.count) + 255) / 256), dim3(256), 0, st, P,
                       w, in, atlas_off, atlas_wh);
  else
    hipLaunchKernelGGL(k_init, dim3((P.count + 255) / 256), dim3(256), 0, st, P, w, atlas_off,
                       atlas_wh, 0, 0);
  return hipGetLastError();
}

hipError_t launch_splice(Chart* dst, const int32_t* idx, int m, const Chart* src, hipStream_t st) {
  if (m > 0) hipLaunchKernelGGL(k_splice, dim3((m + 255) / 256), dim3(256), 0, st, dst, idx, m, src);
  return hipGetLastError();
}

hipError_t launch_prep(const Params& P, const Work& w, const int32_t* xy, const int32_t* voff,
                       const int32_t* atlas_off, const int32_t* atlas_wh, int single_w,
                       int single_h, hipStream_t st, const int32_t* cloop) {
  // the proxy kernel also writes the atlas descriptors (enough blocks for
  // both)
  if (P.N > 0) {
    const int blocks = max((P.N + PREP_CH - 1) / PREP_CH, w.desc ? (P.count + 255) / 256 : 0);
    hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, st, P, w, xy, voff, atlas_off, atlas_wh,
                       single_w, single_h, cloop);
  } else if (w.desc) {
    hipLaunchKernelGGL(k_init, dim3((P.count + 255) / 256), dim3(256), 0, st, P, w, atlas_off,
                       atlas_wh, single_w, single_h);
  }
  return hipGetLastError();
}

hipError_t launch_sort(const Params& P, const Work& w, hipStream_t st) {
  if (P.N > 0) {
    // key tiles per chart tile: a tile's atlases span at most 2 nmax + 256
    // charts when every atlas holds at most nmax (longer spans are still
    // covered, by the loop inside k_rank)
    const int tiles = (P.N + 255) / 256;
    int ny = (2 * P.nmax + 255) / 256 + 2;
    if (ny > tiles) ny = tiles;
    // a single atlas of up to 4,096 charts plans in an extra workgroup of the
    // first sort launch (larger ones plan with 1024 threads afterwards)
    const int pb = P.count == 1 && P.nmax <= 4096 ? tiles : -1;
    // atlases of up to RANK_SCATTER charts (one key tile) rank with one
    // workgroup per chart tile, which also scatters; for larger ones a
    // workgroup walking every key tile of its atlases costs more than the
    // separate scatter launch
    const bool sc = P.nmax <= RANK_SCATTER;
    if (P.nmax > RANK_DIRECT) {
      hipLaunchKernelGGL(k_tile_sort, dim3(tiles + (pb >= 0)), dim3(256), 0, st, P, w, pb);
      if (sc) hipLaunchKernelGGL((k_rank<true, true>), dim3(tiles), dim3(256), 0, st, P, w, -1);
      else hipLaunchKernelGGL((k_rank<true, false>), dim3(tiles, ny), dim3(256), 0, st, P, w, -1);
    } else {
      if (sc) hipLaunchKernelGGL((k_rank<false, true>), dim3(tiles + (pb >= 0)), dim3(256), 0, st, P, w, pb);
      else hipLaunchKernelGGL((k_rank<false, false>), dim3(tiles + (pb >= 0), ny), dim3(256), 0, st, P, w, pb);
    }
    if (!sc) hipLaunchKernelGGL(k_place, dim3(tiles), dim3(256), 0, st, P, w);
    if (pb >= 0) return hipGetLastError();
  }
  if (P.nmax <= 1024)
    hipLaunchKernelGGL(k_plan<256>, dim3(P.count), dim3(256), 0, st, P, w);
  else
    hipLaunchKernelGGL(k_plan<1024>, dim3(P.count), dim3(1024), 0, st, P, w);
  return hipGetLastError();
}

hipError_t launch_setup(const Params& P, const Work& w, int round, hipStream_t st) {
  if (P.N > 0)
  {
    const int nblk = (P.N + SETUP_NT - 1) / SETUP_NT;
    const dim3 grid(((nblk + XCDS - 1) / XCDS) * XCDS * P.Br);
    if (P.K == 10) hipLaunchKernelGGL(k_setup<10>, grid, dim3(SETUP_NT), 0, st, P, w, round);
    else if (P.K == 5) hipLaunchKernelGGL(k_setup<5>, grid, dim3(SETUP_NT), 0, st, P, w, round);
    else if (P.K == 2) hipLaunchKernelGGL(k_setup<2>, grid, dim3(SETUP_NT), 0, st, P, w, round);
    else hipLaunchKernelGGL(k_setup<1>, grid, dim3(SETUP_NT), 0, st, P, w, round);
  }
  return hipGetLastError();
}

}  // namespace tabi
