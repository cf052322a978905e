/*
 * TABI oracle: a plain CPU implementation of the packing method of
 * "TABI: Tight and Balanced Interactive Atlas Packing" (Gu, Vining, Sheffer,
 * Eurographics 2026).
 *
 * TEST INFRASTRUCTURE ONLY.  The GPU library never links, loads or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * The method is a heuristic, so this file is the algorithm itself, written
 * step by step in the paper's order:
 *   chart AABB and 90-degree turn ............ Sec. 3.1, Sec. 4.3
 *   local-AABB slices ......................... Sec. 4.1.1, App. A (local AABBs)
 *   chart orientation (reflections) .......... Sec. 4.1.1, App. A (orientations)
 *   approximate OBB over 8 directions ......... Sec. 4.1.1, App. A (OBBs)
 *   sort by height ............................ Sec. 3.1, Sec. 4.3
 *   per-texel TopEdge/BottomEdge (and the row-wise Left/Right analogue)
 *                                              App. A (Parallel Pushing), Fig. pushing
 *   horizontal compacting distance ............ Sec. 4.1.2, Alg. 2
 *   interlock flags (CannotMoveAbove) ........ Sec. 4.1.3, App. A (Interlocking)
 *   fold, push, correct, update, score ....... Alg. 2, Alg. 1, Alg. 3
 *   knees: detection and location update ..... Sec. 4.2, App. A, Alg. 4
 *   t_opt tail rows ........................... Sec. 4.4
 *   scale search over k/64 .................... Sec. 3.1, Sec. 4.3, Sec. 5
 *
 * Where the paper leaves a choice open (rounding direction, ties, the exact
 * tail rule, gutters, pairs beyond neighbours) the reading used is stated at
 * the point of use.
 */
#include "tabi_oracle.h"

#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

#define QS 16384  /* Q8 (1/256 texel) times the 64 scale steps: texel = k*u/16384 */

/* floor(a/b) and ceil(a/b) for b != 0 */
static int64_t fdiv64(int64_t a, int64_t b) {
  int64_t q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) q--;
  return q;
}
static int64_t cdiv64(int64_t a, int64_t b) { return -fdiv64(-a, b); }
static i128 fdiv128(i128 a, i128 b) {
  i128 q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) q--;
  return q;
}
static i128 cdiv128(i128 a, i128 b) { return -fdiv128(-a, b); }
static int64_t mini64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t maxi64(int64_t a, int64_t b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Quality presets: number of local AABBs and t_opt (Sec. 5 ablations:
 * K in {2,5,10}, t_opt in {5,2,1,0}%; the paper's default is K=10 with
 * t_opt = 0% up to 10,000 charts and 1% above).                             */
void orc_quality(int32_t quality, int32_t n, int32_t* K, int32_t* topt) {
  if (quality == 0) { *K = 2; *topt = 5; }
  else if (quality == 1) { *K = 5; *topt = 2; }
  else { *K = 10; *topt = (n > 10000) ? 1 : 0; }
}

/* The method's knobs (Sec. 5 ablations; App. D, local-AABB count and t_opt
 * tables): K local AABBs per axis, t_opt in percent of the atlas height
 * (negative: the paper's setting, 0 up to 10,000 charts and 1 above), and
 * the variant:
 *   ORC_FULL           tightness and balance (the method);
 *   ORC_TIGHT_ONLY     tightness without balanced folding: every row is
 *                      folded at the full atlas width with compaction, in the
 *                      fixed alternation of one left-to-right row to two
 *                      right-to-left rows, with no knees and no per-row
 *                      choice of direction or compaction;
 *   ORC_BALANCED_ONLY  balanced folding without tightening: the charts'
 *                      boxes stand in for the proxies (one slice per axis, no
 *                      OBB), so nothing compacts and no chart is reflected. */
static int method_resolve(int K, int topt, int variant, int n, int* Kout, int* topt_out,
                          int* use_obb) {
  if (variant < ORC_FULL || variant > ORC_BALANCED_ONLY) return -1;
  if (variant == ORC_BALANCED_ONLY) K = 1;
  if (K < 1 || K > ORC_KMAX || topt > 100) return -1;
  *Kout = K;
  *topt_out = topt < 0 ? ((n > 10000) ? 1 : 0) : topt;
  *use_obb = variant != ORC_BALANCED_ONLY;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The 8 box directions m*pi/16, m = 0..7 (App. A: eight evenly spaced
 * rotations in [0, 7pi/16]), as integer vectors 2^14 (cos, sin) rounded.   */
static void direction(int m, int64_t* C, int64_t* S) {
  *C = llround(16384.0 * cos((double)m * M_PI / 16.0));
  *S = llround(16384.0 * sin((double)m * M_PI / 16.0));
}

/* Range [lo, hi] of the value axis b over the part of the closed polygon
 * whose slab axis a lies in the slab K*a in [j*E, (j+1)*E].  The extreme
 * values over polygon-inside-slab lie on the boundary clipped to the slab:
 * edge endpoints inside it, and crossings of edges with the two slab lines.
 * Rounded outward to whole Q8 units.                                        */
static void slice_range(const int64_t* A, const int64_t* B, const int* nxt, int nv, int64_t E,
                        int K, int j, int64_t* lo, int64_t* hi) {
  int64_t L = (int64_t)j * E, R = (int64_t)(j + 1) * E;
  int64_t l = INT64_MAX, h = INT64_MIN;
  for (int i = 0; i < nv; ++i) {
    int i2 = nxt[i];  /* the edge to the next vertex of the same loop */
    int64_t a1 = (int64_t)K * A[i], a2 = (int64_t)K * A[i2];
    int64_t b1 = B[i], b2 = B[i2];
    if (L <= a1 && a1 <= R) { l = mini64(l, b1); h = maxi64(h, b1); }
    for (int s = 0; s < 2; ++s) {
      int64_t line = s ? R : L;
      if ((a1 < line && line < a2) || (a2 < line && line < a1)) {
        /* b at the crossing = b1 + (b2-b1)*(line-a1)/(a2-a1) */
        int64_t num = b1 * (a2 - a1) + (b2 - b1) * (line - a1);
        int64_t den = a2 - a1;
        l = mini64(l, fdiv64(num, den));
        h = maxi64(h, cdiv64(num, den));
      }
    }
  }
  *lo = l;
  *hi = h;
}

/* A chart of nl boundary loops: loop l holds vertices [lofs[l], lofs[l+1])
 * of xy (lofs[0] = 0).  One loop is the common case; a mesh chart with holes
 * has an outer loop and hole loops, and a chart may also hold several
 * islands.  The proxies bound every loop's edges and vertices. */
static int prep_loops(const int32_t* xy, const int32_t* lofs, int nl, int32_t K, int32_t use_obb,
                      orc_chart* ch) {
  memset(ch, 0, sizeof(*ch));
  ch->K = K;
  if (nl < 1) return 0;
  for (int l = 0; l < nl; ++l)
    if (lofs[l + 1] - lofs[l] < 3) return 0;
  const int nv = lofs[nl];
  int64_t xmin = INT64_MAX, ymin = INT64_MAX, xmax = INT64_MIN, ymax = INT64_MIN;
  for (int i = 0; i < nv; ++i) {
    int64_t x = xy[2 * i], y = xy[2 * i + 1];
    if (x <= -(1 << 22) || x >= (1 << 22) || y <= -(1 << 22) || y >= (1 << 22)) return 0;
    xmin = mini64(xmin, x); xmax = maxi64(xmax, x);
    ymin = mini64(ymin, y); ymax = maxi64(ymax, y);
  }
  int64_t w0 = xmax - xmin, h0 = ymax - ymin;
  if (w0 == 0 || h0 == 0) return 0;
  ch->xmin = xmin;
  ch->ymin = ymin;

  /* 90-degree turn so that the box is at least as tall as wide (Sec. 3.1).
   * Clockwise in y-down coordinates: (u, v) -> (h0 - v, u).  No turn when
   * the box is square. */
  int64_t* u = (int64_t*)malloc(sizeof(int64_t) * nv);
  int64_t* v = (int64_t*)malloc(sizeof(int64_t) * nv);
  ch->rot = w0 > h0;
  for (int i = 0; i < nv; ++i) {
    int64_t u0 = xy[2 * i] - xmin, v0 = xy[2 * i + 1] - ymin;
    if (ch->rot) { u[i] = h0 - v0; v[i] = u0; }
    else { u[i] = u0; v[i] = v0; }
  }
  int64_t W = ch->rot ? h0 : w0, H = ch->rot ? w0 : h0;
  ch->W = W;
  ch->H = H;
  int* nxt = (int*)malloc(sizeof(int) * nv);
  for (int l = 0; l < nl; ++l)
    for (int i = lofs[l]; i < lofs[l + 1]; ++i) nxt[i] = i + 1 < lofs[l + 1] ? i + 1 : lofs[l];

  /* twice the area (shoelace), per loop; the chart's area is taken as the
   * largest loop's less every other loop's: exact for an outer loop with
   * holes, and a lower bound otherwise, which keeps the area bound on the
   * scale rigorous (it may only start the search higher) */
  i128 amax = 0, arest = 0;
  for (int l = 0; l < nl; ++l) {
    i128 s = 0;
    for (int i = lofs[l]; i < lofs[l + 1]; ++i)
      s += (i128)u[i] * v[nxt[i]] - (i128)u[nxt[i]] * v[i];
    if (s < 0) s = -s;
    if (s > amax) { arest += amax; amax = s; }
    else arest += s;
  }
  ch->area2 = (int64_t)(amax > arest ? amax - arest : 0);

  /* local AABBs: K equal slices along x (giving top/bottom bounds) and along
   * y (giving left/right bounds) (Sec. 4.1.1, App. A) */
  for (int j = 0; j < K; ++j) slice_range(u, v, nxt, nv, W, K, j, &ch->ylo[j], &ch->yhi[j]);
  for (int j = 0; j < K; ++j) slice_range(v, u, nxt, nv, H, K, j, &ch->xlo[j], &ch->xhi[j]);
  free(nxt);
  /* A slice that meets no loop (only possible between islands of one
   * chart: a connected loop meets every slice) takes the slice's whole box,
   * a conservative local AABB. */
  for (int j = 0; j < K; ++j) {
    if (ch->ylo[j] > ch->yhi[j]) { ch->ylo[j] = 0; ch->yhi[j] = H; }
    if (ch->xlo[j] > ch->xhi[j]) { ch->xlo[j] = 0; ch->xhi[j] = W; }
  }

  /* orientation (App. A, "Computing Chart Orientations").  Empty area above
   * the top boundary vs below the bottom boundary: reflect vertically when
   * the top one is larger. */
  int64_t top_area = 0, bot_area = 0;
  for (int j = 0; j < K; ++j) { top_area += ch->ylo[j]; bot_area += H - ch->yhi[j]; }
  if (top_area > bot_area) {
    ch->flipy = 1;
    for (int j = 0; j < K; ++j) {
      int64_t lo = H - ch->yhi[j], hi = H - ch->ylo[j];
      ch->ylo[j] = lo; ch->yhi[j] = hi;
    }
    for (int j = 0; j < K / 2; ++j) {
      int64_t t;
      t = ch->xlo[j]; ch->xlo[j] = ch->xlo[K - 1 - j]; ch->xlo[K - 1 - j] = t;
      t = ch->xhi[j]; ch->xhi[j] = ch->xhi[K - 1 - j]; ch->xhi[K - 1 - j] = t;
    }
  }
  /* Left vs right empty area; reflect horizontally when left exceeds right by
   * more than 10% of the AABB area (areas in units of H/K: 10*(L-R) > K*W).
   * When they differ by at most that much, compare the bottom empty area left
   * of the midline with the part right of it (a middle slice, for odd K, is
   * shared equally and cancels). */
  int64_t L = 0, R = 0;
  for (int j = 0; j < K; ++j) { L += ch->xlo[j]; R += W - ch->xhi[j]; }
  int64_t diff = L - R;
  if (10 * diff > (int64_t)K * W) {
    ch->flipx = 1;
  } else if (10 * (diff < 0 ? -diff : diff) <= (int64_t)K * W) {
    int half = K / 2;
    int64_t bl = 0, br = 0;
    for (int j = 0; j < half; ++j) bl += H - ch->yhi[j];
    for (int j = K - half; j < K; ++j) br += H - ch->yhi[j];
    if (bl > br) ch->flipx = 1;
  }
  if (ch->flipx) {
    for (int j = 0; j < K / 2; ++j) {
      int64_t t;
      t = ch->ylo[j]; ch->ylo[j] = ch->ylo[K - 1 - j]; ch->ylo[K - 1 - j] = t;
      t = ch->yhi[j]; ch->yhi[j] = ch->yhi[K - 1 - j]; ch->yhi[K - 1 - j] = t;
    }
    for (int j = 0; j < K; ++j) {
      int64_t lo = W - ch->xhi[j], hi = W - ch->xlo[j];
      ch->xlo[j] = lo; ch->xhi[j] = hi;
    }
  }

  /* approximate OBB of the chart as it will be packed: the minimum-area box
   * over the 8 directions (App. A), areas compared exactly; ties keep the
   * smaller m.  An axis-aligned winner adds nothing to the AABB. */
  for (int i = 0; i < nv; ++i) {
    if (ch->flipx) u[i] = W - u[i];
    if (ch->flipy) v[i] = H - v[i];
  }
  int best = -1;
  i128 best_ext = 0, best_N = 1;
  int64_t bC = 0, bS = 0, ba = 0, bb = 0, be = 0, bf = 0;
  for (int m = 0; m < 8; ++m) {
    int64_t C, S;
    direction(m, &C, &S);
    int64_t a = INT64_MAX, b = INT64_MIN, e = INT64_MAX, f = INT64_MIN;
    for (int i = 0; i < nv; ++i) {
      int64_t p = C * u[i] + S * v[i], q = -S * u[i] + C * v[i];
      a = mini64(a, p); b = maxi64(b, p);
      e = mini64(e, q); f = maxi64(f, q);
    }
    i128 ext = (i128)(b - a) * (i128)(f - e);
    i128 N = (i128)C * C + (i128)S * S;
    if (best < 0 || ext * best_N < best_ext * N) {
      best = m; best_ext = ext; best_N = N;
      bC = C; bS = S; ba = a; bb = b; be = e; bf = f;
    }
  }
  if (!use_obb) {  /* the chart's box alone: the axis-aligned direction */
    best = 0;
    direction(0, &bC, &bS);
    ba = 0; bb = bC * W; be = 0; bf = bC * H;
  }
  ch->obb_m = best;
  ch->obb = best != 0;
  ch->C = bC; ch->S = bS; ch->a = ba; ch->b = bb; ch->e = be; ch->f = bf;
  free(u);
  free(v);
  ch->valid = 1;
  return 1;
}

int orc_prep_chart_loops(const int32_t* xy, const int32_t* lofs, int32_t nl, int32_t K,
                         orc_chart* ch) {
  return prep_loops(xy, lofs, nl, K, 1, ch);
}

int orc_prep_chart_ex(const int32_t* xy, int32_t nv, int32_t K, int32_t use_obb, orc_chart* ch) {
  const int32_t lofs[2] = {0, nv};
  return prep_loops(xy, lofs, 1, K, use_obb, ch);
}

int orc_prep_chart(const int32_t* xy, int32_t nv, int32_t K, orc_chart* ch) {
  return orc_prep_chart_ex(xy, nv, K, 1, ch);
}

/* ------------------------------------------------------------------------ */
/* Per-texel profiles at scale k/64 (App. A, "Parallel Pushing Algorithm").
 *
 * Texel coverage: a chart covers texel (i, j) when the open unit square
 * (i, i+1) x (j, j+1) meets the polygon interior; a chart then spans
 * w = ceil(k W / 16384) columns and h = ceil(k H / 16384) rows.
 *
 * TopEdge(i) is the tightest of three lower bounds on the chart's v inside
 * the open column (i, i+1): the x-slices overlapping it, the y-slices whose
 * u-range reaches into it, and the OBB's top boundary over the column.  The
 * paper takes the largest per texel; rounding is outward (floor for a top,
 * ceil for a bottom) so that separation is never violated.  Left/Right per
 * row are the same construction with the axes exchanged.                    */

/* OBB boundary evaluations.  The box is a <= p <= b, e <= q <= f with
 * p = C u + S v and q = -S u + C v (C, S > 0).  In scaled coordinates
 * U = k u / 16384, V = k v / 16384 its top boundary is
 *   top(U) = max( (k a - 16384 C U) / (16384 S), (k e + 16384 S U) / (16384 C) ),
 * the max of a decreasing and an increasing line, so its minimum over a column
 * is at one of the column's ends or at the box's top corner (p = a, q = e) if
 * that lies inside.  Bottom, left and right boundaries are analogous. */

/* value of a line (n0 + n1 * U) / den at U = num_u / den_u, floored or ceiled */
static i128 line_at(i128 n0, i128 n1, i128 den, i128 num_u, i128 den_u, int ceil_) {
  i128 num = n0 * den_u + n1 * num_u;
  i128 d = den * den_u;
  return ceil_ ? cdiv128(num, d) : fdiv128(num, d);
}

static void obb_column(const orc_chart* ch, int64_t k, int64_t i, int64_t* To, int64_t* Bo) {
  i128 C = ch->C, S = ch->S, N = C * C + S * S, K = k;
  /* column [i, ub], ub = min(i+1, kW/16384) as a rational num/den */
  i128 ub_n, ub_d;
  if ((i128)QS * (i + 1) <= K * ch->W) { ub_n = i + 1; ub_d = 1; }
  else { ub_n = K * ch->W; ub_d = QS; }
  /* top(U) = max( (k a - 16384 C U) / (16384 S), (k e + 16384 S U) / (16384 C) ) */
  i128 t_i = line_at(K * ch->a, -(i128)QS * C, (i128)QS * S, i, 1, 0);
  i128 t2 = line_at(K * ch->e, (i128)QS * S, (i128)QS * C, i, 1, 0);
  if (t2 > t_i) t_i = t2;
  i128 t_u = line_at(K * ch->a, -(i128)QS * C, (i128)QS * S, ub_n, ub_d, 0);
  t2 = line_at(K * ch->e, (i128)QS * S, (i128)QS * C, ub_n, ub_d, 0);
  if (t2 > t_u) t_u = t2;
  i128 top = t_i < t_u ? t_i : t_u;
  /* top corner (p = a, q = e): U = k (C a - S e) / (16384 N) */
  i128 cu = K * (C * ch->a - S * ch->e);
  if (cu * ub_d >= (i128)QS * N * i * ub_d && cu * ub_d <= (i128)QS * N * ub_n) {
    i128 cv = fdiv128(K * (S * ch->a + C * ch->e), (i128)QS * N);
    if (cv < top) top = cv;
  }
  /* bottom(U) = min( (k b - 16384 C U) / (16384 S), (k f + 16384 S U) / (16384 C) ) */
  i128 b_i = line_at(K * ch->b, -(i128)QS * C, (i128)QS * S, i, 1, 1);
  i128 b2 = line_at(K * ch->f, (i128)QS * S, (i128)QS * C, i, 1, 1);
  if (b2 < b_i) b_i = b2;
  i128 b_u = line_at(K * ch->b, -(i128)QS * C, (i128)QS * S, ub_n, ub_d, 1);
  b2 = line_at(K * ch->f, (i128)QS * S, (i128)QS * C, ub_n, ub_d, 1);
  if (b2 < b_u) b_u = b2;
  i128 bot = b_i > b_u ? b_i : b_u;
  /* bottom corner (p = b, q = f) */
  cu = K * (C * ch->b - S * ch->f);
  if (cu * ub_d >= (i128)QS * N * i * ub_d && cu * ub_d <= (i128)QS * N * ub_n) {
    i128 cv = cdiv128(K * (S * ch->b + C * ch->f), (i128)QS * N);
    if (cv > bot) bot = cv;
  }
  *To = (int64_t)top;
  *Bo = (int64_t)bot;
}

static void obb_row(const orc_chart* ch, int64_t k, int64_t j, int64_t* Lo, int64_t* Ro) {
  i128 C = ch->C, S = ch->S, N = C * C + S * S, K = k;
  i128 vb_n, vb_d;
  if ((i128)QS * (j + 1) <= K * ch->H) { vb_n = j + 1; vb_d = 1; }
  else { vb_n = K * ch->H; vb_d = QS; }
  /* left(V) = max( (k a - 16384 S V) / (16384 C), (16384 C V - k f) / (16384 S) ) */
  i128 l_j = line_at(K * ch->a, -(i128)QS * S, (i128)QS * C, j, 1, 0);
  i128 l2 = line_at(-K * ch->f, (i128)QS * C, (i128)QS * S, j, 1, 0);
  if (l2 > l_j) l_j = l2;
  i128 l_v = line_at(K * ch->a, -(i128)QS * S, (i128)QS * C, vb_n, vb_d, 0);
  l2 = line_at(-K * ch->f, (i128)QS * C, (i128)QS * S, vb_n, vb_d, 0);
  if (l2 > l_v) l_v = l2;
  i128 left = l_j < l_v ? l_j : l_v;
  /* left corner (p = a, q = f): V = k (S a + C f) / (16384 N), U = k (C a - S f) / (16384 N) */
  i128 cv = K * (S * ch->a + C * ch->f);
  if (cv * vb_d >= (i128)QS * N * j * vb_d && cv * vb_d <= (i128)QS * N * vb_n) {
    i128 cu = fdiv128(K * (C * ch->a - S * ch->f), (i128)QS * N);
    if (cu < left) left = cu;
  }
  /* right(V) = min( (k b - 16384 S V) / (16384 C), (16384 C V - k e) / (16384 S) ) */
  i128 r_j = line_at(K * ch->b, -(i128)QS * S, (i128)QS * C, j, 1, 1);
  i128 r2 = line_at(-K * ch->e, (i128)QS * C, (i128)QS * S, j, 1, 1);
  if (r2 < r_j) r_j = r2;
  i128 r_v = line_at(K * ch->b, -(i128)QS * S, (i128)QS * C, vb_n, vb_d, 1);
  r2 = line_at(-K * ch->e, (i128)QS * C, (i128)QS * S, vb_n, vb_d, 1);
  if (r2 < r_v) r_v = r2;
  i128 right = r_j > r_v ? r_j : r_v;
  /* right corner (p = b, q = e) */
  cv = K * (S * ch->b + C * ch->e);
  if (cv * vb_d >= (i128)QS * N * j * vb_d && cv * vb_d <= (i128)QS * N * vb_n) {
    i128 cu = cdiv128(K * (C * ch->b - S * ch->e), (i128)QS * N);
    if (cu > right) right = cu;
  }
  *Lo = (int64_t)left;
  *Ro = (int64_t)right;
}

/* Left / right of texel row j under each proxy separately (Sec. 4.1.1):
 * la, ra from the local AABBs (the y-slices overlapping the open row, merged
 * with the x-slices whose v-range reaches into it: the two sets of local
 * AABBs refine each other); lo, ro from the OBB alone, over the row band,
 * kept inside the chart's own texel box [0, w] (when the best of the 8
 * boxes is the axis-aligned one, the OBB is that box).  Outward rounding
 * throughout.                                                              */
static void row_proxies(const orc_chart* ch, int64_t kk, int64_t j, int64_t* la, int64_t* ra,
                        int64_t* lo, int64_t* ro) {
  const int64_t W = ch->W, H = ch->H, K = ch->K;
  const int64_t w = cdiv64(kk * W, QS);
  int64_t ly = INT64_MAX, ry = INT64_MIN;
  for (int64_t s = 0; s < K; ++s) {
    if (s * H * kk < QS * K * (j + 1) && (s + 1) * H * kk > QS * K * j) {
      ly = mini64(ly, fdiv64(ch->xlo[s] * kk, QS));
      ry = maxi64(ry, cdiv64(ch->xhi[s] * kk, QS));
    }
  }
  int64_t lx = INT64_MAX, rx = INT64_MIN;
  for (int64_t s = 0; s < K; ++s) {
    if (ch->ylo[s] * kk < QS * (j + 1) && ch->yhi[s] * kk > QS * j) {
      lx = mini64(lx, fdiv64(s * W * kk, QS * K));
      rx = maxi64(rx, cdiv64((s + 1) * W * kk, QS * K));
    }
  }
  *la = maxi64(ly, lx);
  *ra = mini64(ry, rx);
  int64_t ol = 0, orr = w;
  if (ch->obb) {
    obb_row(ch, kk, j, &ol, &orr);
    ol = maxi64(ol, 0);
    orr = mini64(orr, w);
  }
  *lo = ol;
  *ro = orr;
}

void orc_profiles(const orc_chart* ch, int32_t k, int32_t* w_out, int32_t* h_out,
                  int32_t* top, int32_t* bot, int32_t* left, int32_t* right) {
  const int64_t W = ch->W, H = ch->H, K = ch->K, kk = k;
  int64_t w = cdiv64(kk * W, QS), h = cdiv64(kk * H, QS);
  *w_out = (int32_t)w;
  *h_out = (int32_t)h;
  for (int64_t i = 0; i < w; ++i) {
    int64_t T = INT64_MIN, B = INT64_MAX;
    /* x-slices whose scaled closed range meets the open column (i, i+1) */
    int64_t tx = INT64_MAX, bx = INT64_MIN;
    for (int64_t j = 0; j < K; ++j) {
      if (j * W * kk < QS * K * (i + 1) && (j + 1) * W * kk > QS * K * i) {
        tx = mini64(tx, fdiv64(ch->ylo[j] * kk, QS));
        bx = maxi64(bx, cdiv64(ch->yhi[j] * kk, QS));
      }
    }
    /* y-slices whose u-range reaches into the open column */
    int64_t ty = INT64_MAX, by = INT64_MIN;
    for (int64_t j = 0; j < K; ++j) {
      if (ch->xlo[j] * kk < QS * (i + 1) && ch->xhi[j] * kk > QS * i) {
        ty = mini64(ty, fdiv64(j * H * kk, QS * K));
        by = maxi64(by, cdiv64((j + 1) * H * kk, QS * K));
      }
    }
    T = maxi64(tx, ty);
    B = mini64(bx, by);
    if (ch->obb) {
      int64_t to, bo;
      obb_column(ch, kk, i, &to, &bo);
      T = maxi64(T, to);
      B = mini64(B, bo);
    }
    top[i] = (int32_t)T;
    bot[i] = (int32_t)B;
  }
  for (int64_t j = 0; j < h; ++j) {
    int64_t la, ra, lo, ro;
    row_proxies(ch, kk, j, &la, &ra, &lo, &ro);
    left[j] = (int32_t)maxi64(la, lo);
    right[j] = (int32_t)mini64(ra, ro);
  }
}

void orc_row_proxies(const orc_chart* ch, int32_t k, int32_t* h_out, int32_t* la, int32_t* ra,
                     int32_t* lo, int32_t* ro) {
  int64_t h = cdiv64((int64_t)k * ch->H, QS);
  *h_out = (int32_t)h;
  for (int64_t j = 0; j < h; ++j) {
    int64_t a, b, c, d;
    row_proxies(ch, k, j, &a, &b, &c, &d);
    la[j] = (int32_t)a; ra[j] = (int32_t)b; lo[j] = (int32_t)c; ro[j] = (int32_t)d;
  }
}

/* ------------------------------------------------------------------------ */
/* Sorting (Sec. 3.1): height descending; ties by width descending, then by
 * input index.                                                              */
static _Thread_local const orc_chart* g_sort_charts;  /* per thread: packs may run side by side */
static int cmp_order(const void* pa, const void* pb) {
  int ia = *(const int*)pa, ib = *(const int*)pb;
  const orc_chart *a = &g_sort_charts[ia], *b = &g_sort_charts[ib];
  if (a->H != b->H) return a->H > b->H ? -1 : 1;
  if (a->W != b->W) return a->W > b->W ? -1 : 1;
  return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

/* Largest k in 1..64 whose scaled charts' total area fits the atlas:
 * sum(area2) * k^2 <= 2^29 * W * H  (area2 in Q8^2; a pack is overlap free,
 * so no larger k can succeed). 0 if even k = 1 is too big.                  */
static int area_bound(const orc_chart* ch, int n, int Wa, int Ha) {
  i128 s = 0;
  for (int c = 0; c < n; ++c) s += ch[c].area2;
  int khi = 0;
  for (int k = 1; k <= 64; ++k)
    if (s * k * k <= ((i128)1 << 29) * Wa * Ha) khi = k;
  return khi;
}

/* ------------------------------------------------------------------------ */
/* Per-scale data: dilated profiles, compacting distances.                   */
typedef struct {
  int n, Wd, Hd, Wa, Ha, p, topt;
  int static_rows;                   /* tight-only: every row folded like a tail row */
  int k;                             /* the scale, k/64 */
  int hybrid;                        /* tail rows folded by prefix sums (Sec. 4.4) */
  const orc_chart* ch;               /* charts and their order, for tails at */
  const int* perm;                   /* other scales */
  int32_t *wd, *hd, *h;
  int64_t* Hq;                       /* unscaled Q8 heights, for knees */
  int32_t **topd, **botd;
  /* grown row bounds of each proxy: local AABBs (la, ra) and OBB (lo, ro) */
  int32_t **lad, **rad, **lod, **rod;
  int32_t* cd;
  uint8_t* nfl;                      /* interlock flags of (c-1, c) */
} kdata;

static void free_kdata(kdata* D) {
  for (int c = 0; c < D->n; ++c) {
    free(D->topd[c]); free(D->botd[c]);
    free(D->lad[c]); free(D->rad[c]); free(D->lod[c]); free(D->rod[c]);
  }
  free(D->topd); free(D->botd); free(D->lad); free(D->rad); free(D->lod); free(D->rod);
  free(D->wd); free(D->hd); free(D->h); free(D->Hq); free(D->cd); free(D->nfl);
}

/* Gutters: a chart's footprint is grown by [0,p] x [0,p] toward +x,+y and
 * footprints may not share a texel.  Two grown footprints are disjoint exactly
 * when at least p empty texels separate the charts; the grown atlas is
 * (W+p) x (H+p), so charts may touch the atlas edges (Sec. 5: gutters between
 * charts, none along the 4 atlas edges).                                     */
static void build_kdata(kdata* D, const orc_chart* ch, const int* perm, int n, int k,
                        int Wa, int Ha, int p, int topt) {
  D->n = n; D->Wa = Wa; D->Ha = Ha; D->p = p; D->topt = topt; D->static_rows = 0;
  D->k = k; D->hybrid = 0; D->ch = ch; D->perm = perm;
  D->Wd = Wa + p; D->Hd = Ha + p;
  D->wd = calloc(n + 1, sizeof(int32_t)); D->hd = calloc(n + 1, sizeof(int32_t));
  D->h = calloc(n + 1, sizeof(int32_t)); D->Hq = calloc(n + 1, sizeof(int64_t));
  D->cd = calloc(n + 1, sizeof(int32_t));
  D->nfl = calloc(n + 1, 1);
  D->topd = calloc(n + 1, sizeof(int32_t*)); D->botd = calloc(n + 1, sizeof(int32_t*));
  D->lad = calloc(n + 1, sizeof(int32_t*)); D->rad = calloc(n + 1, sizeof(int32_t*));
  D->lod = calloc(n + 1, sizeof(int32_t*)); D->rod = calloc(n + 1, sizeof(int32_t*));
  for (int c = 0; c < n; ++c) {
    const orc_chart* q = &ch[perm[c]];
    int64_t w = cdiv64((int64_t)k * q->W, QS), h = cdiv64((int64_t)k * q->H, QS);
    int32_t* top = malloc(sizeof(int32_t) * w);
    int32_t* bot = malloc(sizeof(int32_t) * w);
    int32_t* lft = malloc(sizeof(int32_t) * h);
    int32_t* rgt = malloc(sizeof(int32_t) * h);
    int32_t* pr[4];
    for (int e = 0; e < 4; ++e) pr[e] = malloc(sizeof(int32_t) * h);
    int32_t ww, hh;
    orc_profiles(q, k, &ww, &hh, top, bot, lft, rgt);
    orc_row_proxies(q, k, &hh, pr[0], pr[1], pr[2], pr[3]);
    int wd = ww + p, hd = hh + p;
    D->wd[c] = wd; D->hd[c] = hd; D->h[c] = hh; D->Hq[c] = q->H;
    D->topd[c] = malloc(sizeof(int32_t) * wd); D->botd[c] = malloc(sizeof(int32_t) * wd);
    for (int i = 0; i < wd; ++i) {
      int lo = i - p < 0 ? 0 : i - p, hi = i < ww - 1 ? i : ww - 1;
      int32_t t = INT32_MAX, b = INT32_MIN;
      for (int s = lo; s <= hi; ++s) { if (top[s] < t) t = top[s]; if (bot[s] > b) b = bot[s]; }
      D->topd[c][i] = t;
      D->botd[c][i] = b + p;
    }
    int32_t** dst[4] = {&D->lad[c], &D->rad[c], &D->lod[c], &D->rod[c]};
    for (int e = 0; e < 4; e += 2) {  /* each proxy's rows, grown */
      int32_t* L = malloc(sizeof(int32_t) * hd);
      int32_t* R = malloc(sizeof(int32_t) * hd);
      for (int j = 0; j < hd; ++j) {
        int lo = j - p < 0 ? 0 : j - p, hi = j < hh - 1 ? j : hh - 1;
        int32_t l = INT32_MAX, r = INT32_MIN;
        for (int s = lo; s <= hi; ++s) {
          if (pr[e][s] < l) l = pr[e][s];
          if (pr[e + 1][s] > r) r = pr[e + 1][s];
        }
        L[j] = l;
        R[j] = r + p;
      }
      *dst[e] = L;
      *dst[e + 1] = R;
    }
    free(top); free(bot); free(lft); free(rgt);
    for (int e = 0; e < 4; ++e) free(pr[e]);
  }
  /* Horizontal compacting distance between sorted neighbours (Sec. 4.1.2):
   * with both charts top-aligned, each proxy gives the largest leftward
   * slide of the second chart that keeps the proxies apart in every shared
   * texel row; the pair is compacted by the larger of the two.  The
   * interlock flags come from the proxy that gave that distance (App. A,
   * "Detecting Interlocking Charts"; the local AABBs on a tie), and a zero
   * distance restricts neither chart. */
  D->cd[0] = 0;
  for (int c = 1; c < n; ++c) {
    int rows = D->hd[c - 1] < D->hd[c] ? D->hd[c - 1] : D->hd[c];
    int32_t ga = INT32_MAX, go = INT32_MAX;
    for (int j = 0; j < rows; ++j) {
      int32_t g = D->wd[c - 1] - D->rad[c - 1][j] + D->lad[c][j];
      if (g < ga) ga = g;
      g = D->wd[c - 1] - D->rod[c - 1][j] + D->lod[c][j];
      if (g < go) go = g;
    }
    int obb_wins = go > ga;
    D->cd[c] = obb_wins ? go : ga;
    D->nfl[c] = (uint8_t)orc_interlock(obb_wins ? D->rod[c - 1] : D->rad[c - 1], D->hd[c - 1],
                                       D->wd[c - 1], obb_wins ? D->lod[c] : D->lad[c], D->hd[c],
                                       D->wd[c - 1] - D->cd[c]);
  }
}

/* Interlock flags (Sec. 4.1.3, App. A "Detecting Interlocking Charts"),
 * for A and a later chart B whose grown box starts d texels to the right of
 * A's.  B "cannot move above A" when some row j >= 1 of B starts left of where
 * A ends in some row above j (then raising B by 1..j texels may make them
 * meet); symmetrically for A.  Flags are conservative: any upward shift that
 * could bring the two proxies together sets the flag.  No shared column, no
 * flag. */
int orc_interlock(const int32_t* rightA, int32_t hdA, int32_t wdA,
                  const int32_t* leftB, int32_t hdB, int32_t d) {
  if (d >= wdA) return 0;
  int flags = 0;
  int32_t pm = rightA[0];
  for (int j = 1; j < hdB; ++j) {
    if (d + leftB[j] < pm) { flags |= 1; break; }
    if (j < hdA && rightA[j] > pm) pm = rightA[j];
  }
  int32_t pn = leftB[0];
  for (int j = 1; j < hdA; ++j) {
    if (rightA[j] > d + pn) { flags |= 2; break; }
    if (j < hdB && leftB[j] < pn) pn = leftB[j];
  }
  return flags;
}

/* CorrectYOffsets (Alg. 1): for each constrained pair (A, B, flags), while
 * some chart sits above a chart it may not move above, move it down to that
 * chart's offset (offsets grow downward).  Offsets only increase, so the loop
 * ends at the least solution above the pushed offsets. */
void orc_correct(int32_t m, const int32_t* pa, int32_t* y) {
  int violation;
  do {
    violation = 0;
    for (int q = 0; q < m; ++q) {
      int A = pa[3 * q], B = pa[3 * q + 1], fl = pa[3 * q + 2];
      if ((fl & 1) && y[B] < y[A]) { y[B] = y[A]; violation = 1; }
      if ((fl & 2) && y[A] < y[B]) { y[A] = y[B]; violation = 1; }
    }
  } while (violation);
}

/* ------------------------------------------------------------------------ */
/* Row folding (Alg. 2): from the row's first chart, lay charts left to right;
 * a chart is included while its grown box ends inside the folding width;
 * the first that does not fit ends the row.  With horizontal compacting the
 * next chart starts compactingDistance earlier.                             */
static int fold_row(const kdata* D, int rs, int width, int hc, int32_t* X) {
  int64_t x = 0;
  int cnt = 0;
  for (int c = rs; c < D->n; ++c) {
    if (x + D->wd[c] > width) break;
    X[cnt++] = (int32_t)x;
    x = x + D->wd[c] - ((hc && c + 1 < D->n) ? D->cd[c + 1] : 0);
  }
  return cnt;
}

enum { LR = 0, RL = 1 };

typedef struct {
  int R0, R1, dir, hc, cnt, knee;
  int32_t *X, *xa, *y, *Fp;
  int64_t whole, region;
} config;

/* Push, correct, update and score one row configuration (Alg. 3 inner loop).
 * Right-to-left rows place each chart mirrored inside its own box (so its
 * profiles read backwards) at R1 - X - w'. */
static void evaluate(const kdata* D, const int32_t* F, int rs, config* g) {
  int cnt = g->cnt;
  for (int t = 0; t < cnt; ++t) {
    int c = rs + t;
    g->xa[t] = g->dir == LR ? g->R0 + g->X[t] : g->R1 - g->X[t] - D->wd[c];
  }
  /* push: each chart rises until it touches the frontline */
  for (int t = 0; t < cnt; ++t) {
    int c = rs + t, wd = D->wd[c];
    int32_t y = INT32_MIN;
    for (int i = 0; i < wd; ++i) {
      int32_t tp = g->dir == LR ? D->topd[c][i] : D->topd[c][wd - 1 - i];
      int32_t v = F[g->xa[t] + i] - tp;
      if (v > y) y = v;
    }
    g->y[t] = y;
  }
  /* correct (Alg. 1): charts that may not move above a compacted neighbour
   * are moved down to it until no such pair is out of order.  Neighbours
   * carry the flags of their compacting distance.  Every other pair whose
   * grown boxes share columns is checked too: a narrow chart between two
   * others can let the outer two share columns.  Such a pair has no
   * distance of its own; its flags are tested on the rows both proxies
   * allow (per grown row, the intersection of the two proxies' spans). */
  if (g->hc) {
    int cap = 16, m = 0;
    int32_t* pa = malloc(sizeof(int32_t) * cap * 3);
    for (int A = 0; A < cnt; ++A) {
      for (int Bt = A + 1; Bt < cnt; ++Bt) {
        int d = g->X[Bt] - g->X[A];
        if (d >= D->wd[rs + A]) break;
        int fl;
        if (Bt == A + 1) {
          fl = D->nfl[rs + Bt];
        } else {
          int ca = rs + A, cb = rs + Bt;
          int32_t* rA = malloc(sizeof(int32_t) * D->hd[ca]);
          int32_t* lB = malloc(sizeof(int32_t) * D->hd[cb]);
          for (int j = 0; j < D->hd[ca]; ++j) rA[j] = mini64(D->rad[ca][j], D->rod[ca][j]);
          for (int j = 0; j < D->hd[cb]; ++j) lB[j] = maxi64(D->lad[cb][j], D->lod[cb][j]);
          fl = orc_interlock(rA, D->hd[ca], D->wd[ca], lB, D->hd[cb], d);
          free(rA);
          free(lB);
        }
        if (!fl) continue;
        if (m == cap) { cap *= 2; pa = realloc(pa, sizeof(int32_t) * cap * 3); }
        pa[3 * m] = A; pa[3 * m + 1] = Bt; pa[3 * m + 2] = fl; ++m;
      }
    }
    orc_correct(m, pa, g->y);
    free(pa);
  }
  /* update a private copy of the frontline with the charts' bottoms */
  memcpy(g->Fp, F, sizeof(int32_t) * D->Wd);
  for (int t = 0; t < cnt; ++t) {
    int c = rs + t, wd = D->wd[c];
    for (int i = 0; i < wd; ++i) {
      int32_t bt = g->dir == LR ? D->botd[c][i] : D->botd[c][wd - 1 - i];
      int32_t v = g->y[t] + bt;
      if (v > g->Fp[g->xa[t] + i]) g->Fp[g->xa[t] + i] = v;
    }
  }
  /* scores: deepest frontline texel overall, and inside the folding region */
  int64_t s = INT64_MIN, r = INT64_MIN;
  for (int x = 0; x < D->Wd; ++x) {
    if (g->Fp[x] > s) s = g->Fp[x];
    if (x >= g->R0 && x < g->R1 && g->Fp[x] > r) r = g->Fp[x];
  }
  g->whole = s;
  g->region = r;
}

typedef struct { int active, dir, left, right; } knee_t;

/* Knee update (Alg. 4): the concavity wall moves to the nearest texel of the
 * knee chart whose frontline is at least as deep as the frontline just past
 * the wall.  A wall probe outside the atlas ends the knee.                  */
static void update_knee(knee_t* kn, const int32_t* F, int Wd) {
  if (kn->dir == LR) {
    int probe = kn->right;
    if (probe < 0 || probe >= Wd) { kn->active = 0; return; }
    int32_t h0 = F[probe];
    int nl = kn->left - 1;
    for (int x = kn->left; x < kn->right; ++x)
      if (F[x] >= h0 && x > nl) nl = x;
    kn->right = nl + 1;
  } else {
    int probe = kn->left - 1;
    if (probe < 0 || probe >= Wd) { kn->active = 0; return; }
    int32_t h0 = F[probe];
    int nl = kn->right;
    for (int x = kn->left; x < kn->right; ++x)
      if (F[x] >= h0 && x < nl) nl = x;
    kn->left = nl;
  }
}

int orc_knee_update(const int32_t* F, int32_t Wd, int32_t dir, int32_t* left, int32_t* right) {
  knee_t kn = {1, dir, *left, *right};
  update_knee(&kn, F, Wd);
  *left = kn.left;
  *right = kn.right;
  return kn.active;
}

/* Knee detection (Sec. 4.2, App. A): the largest drop in unscaled height
 * between consecutive charts of the row that is at least 10% of the atlas
 * height and at least 20% of the taller chart; ties go to the first pair.
 * The knee is the taller chart's grown span in the atlas.                   */
static knee_t find_knee(const kdata* D, int rs, const config* g) {
  knee_t kn = {0, 0, 0, 0};
  int64_t best = -1;
  for (int t = 0; t + 1 < g->cnt; ++t) {
    int c = rs + t;
    int64_t dl = D->Hq[c] - D->Hq[c + 1];
    if (10 * dl >= 256 * (int64_t)D->Ha && 5 * dl >= D->Hq[c] && dl > best) {
      best = dl;
      kn.active = 1;
      kn.dir = g->dir;
      kn.left = g->xa[t];
      kn.right = g->xa[t] + D->wd[c];
    }
  }
  return kn;
}

static void config_alloc(config* g, int n, int Wd) {
  g->X = malloc(sizeof(int32_t) * (n + 1));
  g->xa = malloc(sizeof(int32_t) * (n + 1));
  g->y = malloc(sizeof(int32_t) * (n + 1));
  g->Fp = malloc(sizeof(int32_t) * Wd);
}
static void config_free(config* g) { free(g->X); free(g->xa); free(g->y); free(g->Fp); }

/* Hybrid tail (Sec. 4.4, "Performance Optimization"): the charts from t0 on
 * are folded all at once.  Each gets an offset, its grown width at the head
 * scale less its compacting distance to the next chart; the prefix sums of
 * the offsets, divided by the grown atlas width, give every chart its row
 * (prefix-sum folding, as in FastAtlas, with the compaction added).  Rows so
 * formed may run past the atlas's right edge, so the tail is downscaled: its
 * scale kt is the largest k' <= k at which every row, laid out left to right
 * with compaction at k', fits the width.  The rows are then placed in the
 * fixed one left-to-right : two right-to-left alternation and pushed up
 * against the frontline like any other row, at kt.  Returns 1 on success
 * (positions of the tail charts written, *kt_out set), 0 when some row does
 * not fit at any scale or the frontline passes the atlas height.            */
static int hybrid_tail(const kdata* D, int32_t* F, int t0, int32_t* xs, int32_t* ys,
                       uint8_t* mir, int* kt_out) {
  const int n = D->n, m = n - t0, Wd = D->Wd;
  int64_t* row = malloc(sizeof(int64_t) * (m + 1));
  int32_t* X = malloc(sizeof(int32_t) * (m + 1));
  int64_t P = 0;
  for (int j = 0; j < m; ++j) {
    const int c = t0 + j;
    row[j] = P / Wd;
    P += D->wd[c] - (c + 1 < n ? D->cd[c + 1] : 0);
  }
  kdata T;
  int kt, fits = 0;
  for (kt = D->k; kt >= 1 && !fits; --kt) {
    build_kdata(&T, D->ch, D->perm + t0, m, kt, D->Wa, D->Ha, D->p, D->topt);
    fits = 1;
    int64_t x = 0;
    for (int j = 0; j < m && fits; ++j) {
      if (j > 0) x = row[j] != row[j - 1] ? 0 : x + T.wd[j - 1] - T.cd[j];
      X[j] = (int32_t)x;
      if (x + T.wd[j] > Wd) fits = 0;
    }
    if (!fits) free_kdata(&T);
  }
  int ok = fits;
  if (fits) {
    ++kt;  /* the loop stepped past the scale that fit */
    config g;
    config_alloc(&g, m, Wd);
    int trow = 0;
    for (int j0 = 0; j0 < m && ok;) {
      int j1 = j0 + 1;
      while (j1 < m && row[j1] == row[j0]) ++j1;
      g.R0 = 0; g.R1 = Wd; g.hc = 1; g.knee = 0;
      g.dir = (trow % 3 == 0) ? LR : RL;
      ++trow;
      g.cnt = j1 - j0;
      memcpy(g.X, X + j0, sizeof(int32_t) * g.cnt);
      evaluate(&T, F, j0, &g);
      memcpy(F, g.Fp, sizeof(int32_t) * Wd);
      for (int t = 0; t < g.cnt; ++t) {
        xs[t0 + j0 + t] = g.xa[t];
        ys[t0 + j0 + t] = g.y[t];
        mir[t0 + j0 + t] = (uint8_t)(g.dir == RL);
      }
      if (g.whole > D->Hd) ok = 0;
      j0 = j1;
    }
    config_free(&g);
    free_kdata(&T);
    *kt_out = kt;
  }
  free(row);
  free(X);
  return ok;
}

/* Full packing at one scale (Alg. 3).  Positions (sorted order) into xs, ys,
 * mirror flags into mir.  Returns 1 when every chart is placed without the
 * frontline passing the (grown) atlas height.                               */
static int pack_scale_ex(const kdata* D, int32_t* xs, int32_t* ys, uint8_t* mir, int* rows_out,
                         int* t0_out, int* kt_out);
static int pack_scale(const kdata* D, int32_t* xs, int32_t* ys, uint8_t* mir, int* rows_out) {
  return pack_scale_ex(D, xs, ys, mir, rows_out, NULL, NULL);
}

/* t0_out: the first chart of the hybrid tail (n without one); kt_out: the
 * tail's scale (k without a tail). */
static int pack_scale_ex(const kdata* D, int32_t* xs, int32_t* ys, uint8_t* mir, int* rows_out,
                         int* t0_out, int* kt_out) {
  int n = D->n, Wd = D->Wd, Hd = D->Hd;
  int32_t* F = calloc(Wd, sizeof(int32_t));
  int32_t* Xoff = malloc(sizeof(int32_t) * (n + 1));
  int32_t* Xon = malloc(sizeof(int32_t) * (n + 1));
  config full[2], kc[2];
  for (int d = 0; d < 2; ++d) { config_alloc(&full[d], n, Wd); config_alloc(&kc[d], n, Wd); }
  knee_t kn = {0, 0, 0, 0};
  int tail = D->static_rows, trow = 0, rs = 0, rows = 0, ok = 1;
  if (t0_out) *t0_out = n;
  if (kt_out) *kt_out = D->k;
  while (rs < n) {
    if (kn.active) update_knee(&kn, F, Wd);
    /* t_opt (Sec. 4.4): once no knee is pending and the row's tallest chart
     * is shorter than t_opt of the atlas height, the remaining rows are full
     * width, compacted, in the fixed 1 left-to-right : 2 right-to-left
     * alternation, without per-row configuration search. */
    if (!tail && !kn.active && 100 * (int64_t)D->h[rs] < (int64_t)D->topt * D->Ha) {
      tail = 1;
      if (D->hybrid) {
        int kt = 0;
        ok = hybrid_tail(D, F, rs, xs, ys, mir, &kt);
        if (t0_out) *t0_out = rs;
        if (kt_out) *kt_out = kt;
        break;
      }
    }
    config* ch;
    int knee_used = 0;
    if (tail) {
      ch = &full[0];
      ch->R0 = 0; ch->R1 = Wd; ch->hc = 1; ch->knee = 0;
      ch->dir = (trow % 3 == 0) ? LR : RL;
      ++trow;
      ch->cnt = fold_row(D, rs, Wd, 1, ch->X);
      if (ch->cnt == 0) { ok = 0; break; }
      evaluate(D, F, rs, ch);
    } else {
      int coff = fold_row(D, rs, Wd, 0, Xoff);
      int con = fold_row(D, rs, Wd, 1, Xon);
      if (con == 0) { ok = 0; break; }   /* first chart wider than the atlas */
      /* compaction is used when it fits more charts in the row */
      int hc = con > coff;
      for (int d = 0; d < 2; ++d) {
        config* g = &full[d];
        g->R0 = 0; g->R1 = Wd; g->dir = d; g->hc = hc; g->knee = 0;
        g->cnt = hc ? con : coff;
        memcpy(g->X, hc ? Xon : Xoff, sizeof(int32_t) * g->cnt);
        evaluate(D, F, rs, g);
      }
      /* direction: smaller maximal frontline height, ties left-to-right */
      ch = full[RL].whole < full[LR].whole ? &full[RL] : &full[LR];
      if (kn.active) {
        int R0 = kn.dir == LR ? kn.right : 0;
        int R1 = kn.dir == LR ? Wd : kn.left;
        int koff = fold_row(D, rs, R1 - R0, 0, Xoff);
        int kon = fold_row(D, rs, R1 - R0, 1, Xon);
        if (kon > 0) {
          int khc = kon > koff;
          for (int d = 0; d < 2; ++d) {
            config* g = &kc[d];
            g->R0 = R0; g->R1 = R1; g->dir = d; g->hc = khc; g->knee = 1;
            g->cnt = khc ? kon : koff;
            memcpy(g->X, khc ? Xon : Xoff, sizeof(int32_t) * g->cnt);
            evaluate(D, F, rs, g);
          }
          /* inside the knee region the direction is judged on the region */
          config* kb = kc[RL].region < kc[LR].region ? &kc[RL] : &kc[LR];
          /* the knee fold wins only if it is strictly lower overall */
          if (kb->whole < ch->whole) { ch = kb; knee_used = 1; }
        }
      }
    }
    /* commit */
    memcpy(F, ch->Fp, sizeof(int32_t) * Wd);
    for (int t = 0; t < ch->cnt; ++t) {
      xs[rs + t] = ch->xa[t];
      ys[rs + t] = ch->y[t];
      mir[rs + t] = (uint8_t)(ch->dir == RL);
    }
    ++rows;
    if (!tail && !knee_used) kn = find_knee(D, rs, ch);
    if (ch->whole > Hd) { ok = 0; break; }
    rs += ch->cnt;
  }
  for (int d = 0; d < 2; ++d) { config_free(&full[d]); config_free(&kc[d]); }
  free(F); free(Xoff); free(Xon);
  if (rows_out) *rows_out = rows;
  return ok;
}

/* ------------------------------------------------------------------------ */
static int check_args(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                      int32_t Ha, int32_t p, int32_t q) {
  if (n < 0 || (n > 0 && (!xy || !offsets))) return -1;
  if (Wa <= 0 || Ha <= 0 || p < 0 || Wa + p > 16384 || Ha + p > 16384) return -1;
  if (q < 0 || q > 2) return -1;
  if (n > 0 && offsets[0] != 0) return -1;
  for (int c = 0; c < n; ++c)
    if (offsets[c + 1] < offsets[c]) return -1;
  return 0;
}

static int prep_all(const int32_t* xy, const int32_t* offsets, int n, int K, int use_obb,
                    orc_chart* ch) {
  int ok = 1;
  for (int c = 0; c < n; ++c) {
    int nv = offsets[c + 1] - offsets[c];
    if (!orc_prep_chart_ex(xy + 2 * (int64_t)offsets[c], nv, K, use_obb, &ch[c])) ok = 0;
  }
  return ok;
}

static void sort_charts(const orc_chart* ch, int n, int* perm) {
  for (int c = 0; c < n; ++c) perm[c] = c;
  g_sort_charts = ch;
  qsort(perm, n, sizeof(int), cmp_order);
}

/* Whole pack with the given knobs (K slices, t_opt percent, OBB used,
 * static rows). */
/* Whole pack of prepared charts (ok: every chart valid). */
static int pack_charts(orc_chart* ch, int ok, int32_t n, int32_t Wa, int32_t Ha, int32_t p, int topt,
                       int static_rows, int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                       int32_t* out_k);

static int pack_with(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa, int32_t Ha,
                     int32_t p, int K, int topt, int use_obb, int static_rows, int32_t* out_xy,
                     uint8_t* out_orient, float* out_scale, int32_t* out_k) {
  if (n == 0) { *out_scale = 1.0f; if (out_k) *out_k = 64; return 0; }
  orc_chart* ch = calloc(n, sizeof(orc_chart));
  const int ok = prep_all(xy, offsets, n, K, use_obb, ch);
  return pack_charts(ch, ok, n, Wa, Ha, p, topt, static_rows, out_xy, out_orient, out_scale,
                     out_k);
}

static int pack_charts(orc_chart* ch, int ok, int32_t n, int32_t Wa, int32_t Ha, int32_t p, int topt,
                       int static_rows, int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                       int32_t* out_k) {
  for (int c = 0; c < n; ++c) { out_xy[2 * c] = -1; out_xy[2 * c + 1] = -1; out_orient[c] = 0; }
  if (!ok) {
    free(ch);
    *out_scale = -1.0f;
    if (out_k) *out_k = -1;
    return 0;
  }
  int* perm = malloc(sizeof(int) * n);
  sort_charts(ch, n, perm);
  int khi = area_bound(ch, n, Wa, Ha);
  int32_t* xs = malloc(sizeof(int32_t) * n);
  int32_t* ys = malloc(sizeof(int32_t) * n);
  uint8_t* mir = malloc(n);
  int kstar = 0;
  /* Scale search (Sec. 3.1, 4.3): the largest k/64 whose packing succeeds. */
  for (int k = khi; k >= 1; --k) {
    kdata D;
    build_kdata(&D, ch, perm, n, k, Wa, Ha, p, topt);
    D.static_rows = static_rows;
    int ok = pack_scale(&D, xs, ys, mir, NULL);
    free_kdata(&D);
    if (ok) { kstar = k; break; }
  }
  if (kstar > 0) {
    for (int t = 0; t < n; ++t) {
      int c = perm[t];
      out_xy[2 * c] = xs[t];
      out_xy[2 * c + 1] = ys[t];
      out_orient[c] = (uint8_t)(ch[c].rot | (ch[c].flipx << 1) | (ch[c].flipy << 2) | (mir[t] << 3));
    }
  }
  *out_scale = (float)kstar / 64.0f;
  if (out_k) *out_k = kstar;
  free(xs); free(ys); free(mir); free(perm); free(ch);
  return 0;
}

/* Whole pack with the hybrid tail (Sec. 4.4): with the tail at its own
 * scale the final scale differs between the charts placed row by row (k/64)
 * and the tail (kt/64), so the chosen candidate k maximises the charts'
 * final scales weighted by their areas, sum over charts of area * scale,
 * among the k whose packing succeeds; ties keep the larger k.  The scale
 * bound from the total area no longer holds (the tail is smaller), so every
 * k from 64 down is a candidate; the search stops once k times the total
 * area, which no packing at k or below can exceed, is no more than the best
 * found.  out_k: k of the head; out_ks[c]: each chart's own k.             */
int tabi_oracle_pack_hybrid(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                            int32_t Ha, int32_t p, int32_t K, int32_t topt, int32_t* out_xy,
                            uint8_t* out_orient, int32_t* out_ks, int32_t* out_k) {
  if (check_args(xy, offsets, n, Wa, Ha, p, 0)) return -1;
  if (!(K == 1 || K == 2 || K == 5 || K == 10) || topt < -1 || topt > 100) return -1;
  if (topt < 0) topt = n > 10000 ? 1 : 0;
  for (int c = 0; c < n; ++c) {
    out_xy[2 * c] = -1; out_xy[2 * c + 1] = -1; out_orient[c] = 0; out_ks[c] = 0;
  }
  if (n <= 0) { *out_k = 64; return 0; }
  orc_chart* ch = calloc(n, sizeof(orc_chart));
  if (!prep_all(xy, offsets, n, K, 1, ch)) {
    free(ch);
    *out_k = -1;
    return 0;
  }
  int* perm = malloc(sizeof(int) * n);
  sort_charts(ch, n, perm);
  i128 total = 0;
  for (int c = 0; c < n; ++c) total += ch[c].area2;
  int32_t* xs = malloc(sizeof(int32_t) * n);
  int32_t* ys = malloc(sizeof(int32_t) * n);
  uint8_t* mir = malloc(n);
  int32_t* bx = malloc(sizeof(int32_t) * n);
  int32_t* by = malloc(sizeof(int32_t) * n);
  uint8_t* bm = malloc(n);
  int best = 0, bt0 = n, bkt = 0;
  i128 bobj = 0;
  for (int k = 64; k >= 1; --k) {
    if (best > 0 && (i128)k * total <= bobj) break;
    kdata D;
    build_kdata(&D, ch, perm, n, k, Wa, Ha, p, topt);
    D.hybrid = 1;
    int t0 = n, kt = k;
    const int ok = pack_scale_ex(&D, xs, ys, mir, NULL, &t0, &kt);
    free_kdata(&D);
    if (!ok) continue;
    i128 head = 0, tail = 0;
    for (int t = 0; t < n; ++t) {
      if (t < t0) head += ch[perm[t]].area2;
      else tail += ch[perm[t]].area2;
    }
    const i128 obj = (i128)k * head + (i128)kt * tail;
    if (best == 0 || obj > bobj) {
      best = k; bobj = obj; bt0 = t0; bkt = kt;
      memcpy(bx, xs, sizeof(int32_t) * n);
      memcpy(by, ys, sizeof(int32_t) * n);
      memcpy(bm, mir, n);
    }
  }
  if (best > 0) {
    for (int t = 0; t < n; ++t) {
      const int c = perm[t];
      out_xy[2 * c] = bx[t];
      out_xy[2 * c + 1] = by[t];
      out_orient[c] = (uint8_t)(ch[c].rot | (ch[c].flipx << 1) | (ch[c].flipy << 2) | (bm[t] << 3));
      out_ks[c] = t < bt0 ? best : bkt;
    }
  }
  *out_k = best;
  free(xs); free(ys); free(mir); free(bx); free(by); free(bm); free(perm); free(ch);
  return 0;
}

/* One candidate scale of the hybrid pack: feasibility, positions in sorted
 * order, the tail's first chart t0 and scale kt. */
int tabi_oracle_feasible_hybrid(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                                int32_t Ha, int32_t p, int32_t K, int32_t topt, int32_t k,
                                int32_t* out_xs, int32_t* out_ys, uint8_t* out_mir,
                                int32_t* out_t0, int32_t* out_kt) {
  if (check_args(xy, offsets, n, Wa, Ha, p, 0) || n < 0 || k < 1 || k > 64) return -1;
  if (!(K == 1 || K == 2 || K == 5 || K == 10) || topt < 0 || topt > 100) return -1;
  orc_chart* ch = calloc(n > 0 ? n : 1, sizeof(orc_chart));
  if (!prep_all(xy, offsets, n, K, 1, ch)) { free(ch); return -2; }
  int* perm = malloc(sizeof(int) * (n > 0 ? n : 1));
  sort_charts(ch, n, perm);
  kdata D;
  build_kdata(&D, ch, perm, n, k, Wa, Ha, p, topt);
  D.hybrid = 1;
  const int ok = pack_scale_ex(&D, out_xs, out_ys, out_mir, NULL, out_t0, out_kt);
  free_kdata(&D);
  free(perm); free(ch);
  return ok;
}

int tabi_oracle_pack(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                     int32_t Ha, int32_t p, int32_t q, int32_t* out_xy, uint8_t* out_orient,
                     float* out_scale, int32_t* out_k) {
  if (check_args(xy, offsets, n, Wa, Ha, p, q)) return -1;
  int K, topt;
  orc_quality(q, n, &K, &topt);
  return pack_with(xy, offsets, n, Wa, Ha, p, K, topt, 1, 0, out_xy, out_orient, out_scale, out_k);
}

/* ------------------------------------------------------------------------ */
/* Pre-rotation of a chart to its tight box (Sec. 5, "Experimental Setup":
 * UV charts are rotated so that their tight bounding boxes align with the
 * axes before packing).  The box is sought, as for the OBB proxy, over a
 * fixed set of directions, here 64 (m pi / 128, m = 0..63, which include
 * the OBB's 8), as integer vectors 2^14 (cos, sin) rounded; the box of least
 * area wins (exact comparison; ties keep the smaller m).  The chart is then
 * turned about its box corner, (dx, dy) -> (C dx + S dy, -S dx + C dy) / 2^14
 * rounded to the nearest Q8 unit (halves up), and moved so that its new box
 * starts at (0, 0).  A chart the pack rejects anyway (fewer than 3 vertices,
 * a coordinate outside (-2^22, 2^22)) is copied unchanged with m = 0.       */
static void predir(int m, int64_t* C, int64_t* S) {
  *C = llround(16384.0 * cos((double)m * M_PI / 128.0));
  *S = llround(16384.0 * sin((double)m * M_PI / 128.0));
}

int orc_prerotate(const int32_t* xy, int32_t nv, int32_t* out, int32_t* m_out) {
  int bad = nv < 3;
  for (int i = 0; i < 2 * nv; ++i)
    if (xy[i] <= -(1 << 22) || xy[i] >= (1 << 22)) bad = 1;
  if (bad) {
    for (int i = 0; i < 2 * nv; ++i) out[i] = xy[i];
    *m_out = 0;
    return 0;
  }
  int64_t xmin = INT64_MAX, ymin = INT64_MAX;
  for (int i = 0; i < nv; ++i) {
    xmin = mini64(xmin, xy[2 * i]);
    ymin = mini64(ymin, xy[2 * i + 1]);
  }
  int best = 0;
  i128 bext = 0, bN = 1;
  for (int m = 0; m < 64; ++m) {
    int64_t C, S;
    predir(m, &C, &S);
    int64_t a = INT64_MAX, b = INT64_MIN, e = INT64_MAX, f = INT64_MIN;
    for (int i = 0; i < nv; ++i) {
      int64_t dx = xy[2 * i] - xmin, dy = xy[2 * i + 1] - ymin;
      int64_t p = C * dx + S * dy, q = -S * dx + C * dy;
      a = mini64(a, p); b = maxi64(b, p);
      e = mini64(e, q); f = maxi64(f, q);
    }
    i128 ext = (i128)(b - a) * (i128)(f - e), N = (i128)C * C + (i128)S * S;
    if (m == 0 || ext * bN < bext * N) { best = m; bext = ext; bN = N; }
  }
  int64_t C, S, tx = INT64_MAX, ty = INT64_MAX;
  predir(best, &C, &S);
  for (int i = 0; i < nv; ++i) {
    int64_t dx = xy[2 * i] - xmin, dy = xy[2 * i + 1] - ymin;
    out[2 * i] = (int32_t)fdiv64(C * dx + S * dy + 8192, 16384);
    out[2 * i + 1] = (int32_t)fdiv64(-S * dx + C * dy + 8192, 16384);
    tx = mini64(tx, out[2 * i]);
    ty = mini64(ty, out[2 * i + 1]);
  }
  for (int i = 0; i < nv; ++i) {
    out[2 * i] -= (int32_t)tx;
    out[2 * i + 1] -= (int32_t)ty;
  }
  *m_out = best;
  return best;
}

int tabi_oracle_pack_prerotate(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                               int32_t Ha, int32_t p, int32_t q, int32_t* out_xy,
                               uint8_t* out_orient, uint8_t* out_dir, float* out_scale,
                               int32_t* out_k) {
  if (check_args(xy, offsets, n, Wa, Ha, p, q)) return -1;
  const int64_t V = n > 0 ? offsets[n] : 0;
  int32_t* rxy = malloc(sizeof(int32_t) * (2 * V + 2));
  for (int c = 0; c < n; ++c) {
    int32_t m = 0;
    orc_prerotate(xy + 2 * (int64_t)offsets[c], offsets[c + 1] - offsets[c],
                  rxy + 2 * (int64_t)offsets[c], &m);
    out_dir[c] = (uint8_t)m;
  }
  const int rc = tabi_oracle_pack(rxy, offsets, n, Wa, Ha, p, q, out_xy, out_orient, out_scale,
                                  out_k);
  free(rxy);
  return rc;
}

int tabi_oracle_pack_loops(const int32_t* xy, const int32_t* loop_offsets,
                           const int32_t* chart_loops, int32_t n, int32_t Wa, int32_t Ha,
                           int32_t p, int32_t q, int32_t* out_xy, uint8_t* out_orient,
                           float* out_scale, int32_t* out_k) {
  if (n < 0 || (n > 0 && (!xy || !loop_offsets || !chart_loops)) || Wa <= 0 || Ha <= 0 || p < 0 ||
      Wa + p > 16384 || Ha + p > 16384 || q < 0 || q > 2)
    return -1;
  if (n > 0 && (chart_loops[0] != 0 || loop_offsets[0] != 0)) return -1;
  for (int c = 0; c < n; ++c)
    if (chart_loops[c + 1] <= chart_loops[c]) return -1;  /* at least one loop per chart */
  for (int l = 0; n > 0 && l < chart_loops[n]; ++l)
    if (loop_offsets[l + 1] < loop_offsets[l]) return -1;
  int K, topt;
  orc_quality(q, n, &K, &topt);
  if (n == 0) { *out_scale = 1.0f; if (out_k) *out_k = 64; return 0; }
  orc_chart* ch = calloc(n, sizeof(orc_chart));
  int ok = 1;
  for (int c = 0; c < n; ++c) {
    const int l0 = chart_loops[c], nl = chart_loops[c + 1] - l0, v0 = loop_offsets[l0];
    int32_t* lofs = malloc(sizeof(int32_t) * (nl + 1));
    for (int l = 0; l <= nl; ++l) lofs[l] = loop_offsets[l0 + l] - v0;
    if (!prep_loops(xy + 2 * (int64_t)v0, lofs, nl, K, 1, &ch[c])) ok = 0;
    free(lofs);
  }
  return pack_charts(ch, ok, n, Wa, Ha, p, topt, 0, out_xy, out_orient, out_scale, out_k);
}

int tabi_oracle_pack_method(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                            int32_t Ha, int32_t p, int32_t K, int32_t topt, int32_t variant,
                            int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                            int32_t* out_k) {
  int Kr, tr, use_obb;
  if (check_args(xy, offsets, n, Wa, Ha, p, 0) || method_resolve(K, topt, variant, n, &Kr, &tr,
                                                                 &use_obb))
    return -1;
  return pack_with(xy, offsets, n, Wa, Ha, p, Kr, tr, use_obb, variant == ORC_TIGHT_ONLY, out_xy,
                   out_orient, out_scale, out_k);
}

int tabi_oracle_feasible(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                         int32_t Ha, int32_t p, int32_t q, int32_t k, int32_t* out_xy,
                         uint8_t* out_orient, int32_t* rows_out) {
  if (check_args(xy, offsets, n, Wa, Ha, p, q) || k < 1 || k > 64) return -1;
  int K, topt;
  orc_quality(q, n, &K, &topt);
  if (n == 0) return 1;
  orc_chart* ch = calloc(n, sizeof(orc_chart));
  if (!prep_all(xy, offsets, n, K, 1, ch)) { free(ch); return -1; }
  int* perm = malloc(sizeof(int) * n);
  sort_charts(ch, n, perm);
  int32_t* xs = malloc(sizeof(int32_t) * n);
  int32_t* ys = malloc(sizeof(int32_t) * n);
  uint8_t* mir = calloc(n, 1);
  for (int t = 0; t < n; ++t) { xs[t] = -1; ys[t] = -1; }
  kdata D;
  build_kdata(&D, ch, perm, n, k, Wa, Ha, p, topt);
  int ok = pack_scale(&D, xs, ys, mir, rows_out);
  free_kdata(&D);
  for (int t = 0; t < n; ++t) {
    int c = perm[t];
    out_xy[2 * c] = xs[t];
    out_xy[2 * c + 1] = ys[t];
    /* charts not reached before the scan stopped: no transform reported */
    out_orient[c] = xs[t] < 0 ? 0 : (uint8_t)(ch[c].rot | (ch[c].flipx << 1) | (ch[c].flipy << 2) | (mir[t] << 3));
  }
  free(xs); free(ys); free(mir); free(perm); free(ch);
  return ok;
}

int tabi_oracle_order(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                      int32_t Ha, int32_t q, int32_t* perm_out, int32_t* k_hi) {
  if (check_args(xy, offsets, n, Wa, Ha, 0, q)) return -1;
  int K, topt;
  orc_quality(q, n, &K, &topt);
  orc_chart* ch = calloc(n > 0 ? n : 1, sizeof(orc_chart));
  if (!prep_all(xy, offsets, n, K, 1, ch)) { free(ch); return -1; }
  int* perm = malloc(sizeof(int) * (n > 0 ? n : 1));
  sort_charts(ch, n, perm);
  for (int t = 0; t < n; ++t) perm_out[t] = perm[t];
  *k_hi = n ? area_bound(ch, n, Wa, Ha) : 64;
  free(perm); free(ch);
  return 0;
}

int tabi_oracle_pairs(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t p,
                      int32_t q, int32_t k, int32_t* cd, uint8_t* flags) {
  if (check_args(xy, offsets, n, 1, 1, p, q) || k < 1 || k > 64) return -1;
  int K, topt;
  orc_quality(q, n, &K, &topt);
  if (n == 0) return 0;
  orc_chart* ch = calloc(n, sizeof(orc_chart));
  if (!prep_all(xy, offsets, n, K, 1, ch)) { free(ch); return -1; }
  int* perm = malloc(sizeof(int) * n);
  sort_charts(ch, n, perm);
  kdata D;
  build_kdata(&D, ch, perm, n, k, 1, 1, p, topt);
  cd[0] = 0;
  flags[0] = 0;
  for (int c = 1; c < n; ++c) {
    cd[c] = D.cd[c];
    flags[c] = D.nfl[c];
  }
  free_kdata(&D);
  free(perm); free(ch);
  return 0;
}
