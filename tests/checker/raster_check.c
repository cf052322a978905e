/*
 * Brute-force layout checker for atlas packings (test infrastructure).
 *
 * Written independently of the oracle and of the GPU library: it shares no
 * code with either.  From the input polygons and a packer's output (box
 * positions, orientation bits, scale k/64) it rebuilds every chart's atlas
 * polygon exactly in Q14 (1/16384 texel), rasterises it with the rule
 * "texel (i,j) is covered when the open square (i,i+1)x(j,j+1) meets the
 * polygon interior", grows each footprint by [0,p]^2 and checks that
 *   - no two grown footprints share a texel (overlap / gutter violation),
 *   - every covered texel lies inside the atlas.
 *
 * Orientation bits: bit0 quarter turn (u,v) -> (h0 - v, u), bit1 mirror in x
 * inside the box, bit2 mirror in y inside the box, bit3 mirror in x inside the
 * scaled texel box.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
#define T 16384

/* does segment P->Q meet the open box (x0,x1)x(y0,y1)? exact */
static int seg_hits_open_box(int64_t px, int64_t py, int64_t qx, int64_t qy,
                             int64_t x0, int64_t x1, int64_t y0, int64_t y1) {
  /* parameter interval (lo, hi) of t in [0,1], as rationals n/d with d > 0;
   * lo_closed / hi_closed mark whether the bound itself is admissible */
  i128 lo_n = 0, lo_d = 1, hi_n = 1, hi_d = 1;
  int lo_closed = 1, hi_closed = 1;
  int64_t P[2] = {px, py}, D[2] = {qx - px, qy - py};
  int64_t A[2] = {x0, y0}, B[2] = {x1, y1};
  for (int ax = 0; ax < 2; ++ax) {
    if (D[ax] == 0) {
      if (!(A[ax] < P[ax] && P[ax] < B[ax])) return 0;
      continue;
    }
    /* A < P + t D < B  (open) */
    i128 n1 = A[ax] - P[ax], n2 = B[ax] - P[ax], d = D[ax];
    if (d < 0) { i128 t = n1; n1 = -n2; n2 = -t; d = -d; }
    /* t > n1/d and t < n2/d */
    /* raise lower bound */
    if (n1 * lo_d > lo_n * d || (n1 * lo_d == lo_n * d && lo_closed)) {
      lo_n = n1; lo_d = d; lo_closed = 0;
    }
    if (n2 * hi_d < hi_n * d || (n2 * hi_d == hi_n * d && hi_closed)) {
      hi_n = n2; hi_d = d; hi_closed = 0;
    }
  }
  i128 l = lo_n * hi_d, h = hi_n * lo_d;
  if (l < h) return 1;
  if (l == h && lo_closed && hi_closed) return 1;
  return 0;
}

/* even-odd test of a point that is known not to lie on the boundary */
static int point_inside(const int64_t* X, const int64_t* Y, int m, int64_t cx, int64_t cy) {
  int in = 0;
  for (int i = 0; i < m; ++i) {
    int j = (i + 1) % m;
    int64_t yi = Y[i], yj = Y[j];
    if ((yi > cy) != (yj > cy)) {
      /* x of the crossing = X[i] + (cy - yi) (X[j]-X[i]) / (yj - yi); test cx < it */
      i128 num = (i128)(cy - yi) * (X[j] - X[i]);
      i128 den = yj - yi;
      i128 lhs = (i128)(cx - X[i]) * den;
      if (den > 0 ? lhs < num : lhs > num) in = !in;
    }
  }
  return in;
}

static int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) q--;
  return q;
}

/* Rasterise a polygon with Q14 integer vertices into mask[bh][bw] whose
 * texel (0,0) is atlas texel (bx, by).  Returns the number of covered texels.
 * Texels outside the mask window are counted in *outside. */
long tabi_check_raster(const int64_t* X, const int64_t* Y, int32_t m, int64_t bx, int64_t by,
                       int64_t bw, int64_t bh, uint8_t* mask, long* outside) {
  memset(mask, 0, (size_t)(bw * bh));
  long out = 0;
  int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
  for (int i = 1; i < m; ++i) {
    if (X[i] < xmin) xmin = X[i];
    if (X[i] > xmax) xmax = X[i];
    if (Y[i] < ymin) ymin = Y[i];
    if (Y[i] > ymax) ymax = Y[i];
  }
  int64_t i0 = fdiv(xmin, T), i1 = fdiv(xmax - 1, T) + 1;
  int64_t j0 = fdiv(ymin, T), j1 = fdiv(ymax - 1, T) + 1;
  /* texels touched by an edge */
  uint8_t* edge_hit = calloc((size_t)((i1 - i0) * (j1 - j0)), 1);
  for (int e = 0; e < m; ++e) {
    int f = (e + 1) % m;
    int64_t ex0 = X[e] < X[f] ? X[e] : X[f], ex1 = X[e] < X[f] ? X[f] : X[e];
    int64_t ey0 = Y[e] < Y[f] ? Y[e] : Y[f], ey1 = Y[e] < Y[f] ? Y[f] : Y[e];
    int64_t a0 = fdiv(ey0, T), a1 = fdiv(ey1, T);
    for (int64_t j = a0; j <= a1; ++j) {
      if (j < j0 || j >= j1) continue;
      int64_t b0 = fdiv(ex0, T), b1 = fdiv(ex1, T);
      /* narrow the column range to the part of the edge inside the strip */
      if (Y[e] != Y[f]) {
        int64_t ylo = j * T > ey0 ? j * T : ey0, yhi = (j + 1) * T < ey1 ? (j + 1) * T : ey1;
        /* x at ylo and yhi */
        i128 dx = X[f] - X[e], dy = Y[f] - Y[e];
        i128 xa = (i128)X[e] * dy + dx * (ylo - Y[e]);
        i128 xb = (i128)X[e] * dy + dx * (yhi - Y[e]);
        if (dy < 0) { xa = -xa; xb = -xb; dy = -dy; }
        i128 lo = xa < xb ? xa : xb, hi = xa < xb ? xb : xa;
        int64_t c0 = (int64_t)(lo / dy) / T - 1, c1 = (int64_t)(hi / dy) / T + 1;
        if (c0 > b0) b0 = c0;
        if (c1 < b1) b1 = c1;
      }
      for (int64_t i = b0; i <= b1; ++i) {
        if (i < i0 || i >= i1) continue;
        if (seg_hits_open_box(X[e], Y[e], X[f], Y[f], i * T, (i + 1) * T, j * T, (j + 1) * T))
          edge_hit[(j - j0) * (i1 - i0) + (i - i0)] = 1;
      }
    }
  }
  long cnt = 0;
  for (int64_t j = j0; j < j1; ++j) {
    for (int64_t i = i0; i < i1; ++i) {
      int cov = edge_hit[(j - j0) * (i1 - i0) + (i - i0)];
      if (!cov) cov = point_inside(X, Y, m, i * T + T / 2, j * T + T / 2);
      if (!cov) continue;
      ++cnt;
      int64_t li = i - bx, lj = j - by;
      if (li < 0 || lj < 0 || li >= bw || lj >= bh) { ++out; continue; }
      mask[lj * bw + li] = 1;
    }
  }
  free(edge_hit);
  if (outside) *outside = out;
  return cnt;
}

/* Atlas-space Q14 polygon of chart c from the packer's output. */
static void place_chart(const int32_t* xy, int m, int32_t ox, int32_t oy, int orient, int64_t k,
                        int64_t* X, int64_t* Y) {
  int64_t xmin = xy[0], xmax = xy[0], ymin = xy[1], ymax = xy[1];
  for (int i = 1; i < m; ++i) {
    if (xy[2 * i] < xmin) xmin = xy[2 * i];
    if (xy[2 * i] > xmax) xmax = xy[2 * i];
    if (xy[2 * i + 1] < ymin) ymin = xy[2 * i + 1];
    if (xy[2 * i + 1] > ymax) ymax = xy[2 * i + 1];
  }
  int64_t w0 = xmax - xmin, h0 = ymax - ymin;
  int64_t W = (orient & 1) ? h0 : w0, H = (orient & 1) ? w0 : h0;
  int64_t wt = (k * W + T - 1) / T;
  for (int i = 0; i < m; ++i) {
    int64_t u = xy[2 * i] - xmin, v = xy[2 * i + 1] - ymin;
    if (orient & 1) { int64_t t = u; u = h0 - v; v = t; }
    if (orient & 2) u = W - u;
    if (orient & 4) v = H - v;
    int64_t U = k * u, V = k * v;
    if (orient & 8) U = T * wt - U;
    X[i] = (int64_t)ox * T + U;
    Y[i] = (int64_t)oy * T + V;
  }
}

/* Check a whole layout.  stats[0] = texels covered by two or more grown
 * footprints, stats[1] = covered texels outside the atlas, stats[2] = covered
 * texels in total, stats[3] = charts with fewer than one covered texel.
 * Returns stats[0] + stats[1]. */
long tabi_check_layout_ks(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                          int32_t Ha, int32_t p, const int32_t* out_xy, const uint8_t* out_orient,
                          const int32_t* ks, int64_t* stats);

long tabi_check_layout(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                       int32_t Ha, int32_t p, const int32_t* out_xy, const uint8_t* out_orient,
                       int32_t k, int64_t* stats) {
  int32_t* ks = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
  for (int c = 0; c < n; ++c) ks[c] = k;
  long r = tabi_check_layout_ks(xy, offsets, n, Wa, Ha, p, out_xy, out_orient, ks, stats);
  free(ks);
  return r;
}

/* The same with a scale ks[c]/64 of its own for every chart. */
long tabi_check_layout_ks(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                          int32_t Ha, int32_t p, const int32_t* out_xy, const uint8_t* out_orient,
                          const int32_t* ks, int64_t* stats) {
  int64_t Wd = (int64_t)Wa + p, Hd = (int64_t)Ha + p;
  uint8_t* grid = calloc((size_t)(Wd * Hd), 1);
  int64_t overlap = 0, outside = 0, total = 0, empty = 0;
  for (int c = 0; c < n; ++c) {
    int m = offsets[c + 1] - offsets[c];
    const int32_t* v = xy + 2 * (int64_t)offsets[c];
    int64_t* X = malloc(sizeof(int64_t) * m);
    int64_t* Y = malloc(sizeof(int64_t) * m);
    place_chart(v, m, out_xy[2 * c], out_xy[2 * c + 1], out_orient[c], ks[c], X, Y);
    int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
    for (int i = 1; i < m; ++i) {
      if (X[i] < xmin) xmin = X[i];
      if (X[i] > xmax) xmax = X[i];
      if (Y[i] < ymin) ymin = Y[i];
      if (Y[i] > ymax) ymax = Y[i];
    }
    int64_t bx = fdiv(xmin, T), by = fdiv(ymin, T);
    int64_t bw = fdiv(xmax - 1, T) + 1 - bx, bh = fdiv(ymax - 1, T) + 1 - by;
    uint8_t* mask = malloc((size_t)(bw * bh));
    long outs = 0;
    long cnt = tabi_check_raster(X, Y, m, bx, by, bw, bh, mask, &outs);
    total += cnt;
    if (cnt == 0) ++empty;
    /* grow by [0,p]^2 and stamp into the grown atlas grid */
    int64_t gw = bw + p, gh = bh + p;
    uint8_t* grown = calloc((size_t)(gw * gh), 1);
    for (int64_t j = 0; j < bh; ++j)
      for (int64_t i = 0; i < bw; ++i) {
        if (!mask[j * bw + i]) continue;
        int64_t ai = bx + i, aj = by + j;
        if (ai < 0 || aj < 0 || ai >= Wa || aj >= Ha) ++outside;
        for (int64_t dj = 0; dj <= p; ++dj)
          for (int64_t di = 0; di <= p; ++di) grown[(j + dj) * gw + (i + di)] = 1;
      }
    for (int64_t j = 0; j < gh; ++j)
      for (int64_t i = 0; i < gw; ++i) {
        if (!grown[j * gw + i]) continue;
        int64_t ai = bx + i, aj = by + j;
        if (ai < 0 || aj < 0 || ai >= Wd || aj >= Hd) continue; /* counted as outside above */
        uint8_t* g = &grid[aj * Wd + ai];
        if (*g) ++overlap;
        else *g = 1;
      }
    free(grown);
    free(mask);
    free(X);
    free(Y);
  }
  free(grid);
  stats[0] = overlap;
  stats[1] = outside;
  stats[2] = total;
  stats[3] = empty;
  return (long)(overlap + outside);
}
