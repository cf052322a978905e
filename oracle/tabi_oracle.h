/*
 * Reference (oracle) implementation of TABI atlas packing, host only.
 *
 * TEST INFRASTRUCTURE: this library exists to check the GPU library.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Plain, slow, single-threaded C.  Every quantity is an integer (or an exact
 * rational evaluated with floor / ceil); the only float is the returned scale
 * k/64, which is exact.
 *
 * Coordinates: input vertices are int32 in Q8 (1/256 texel), y grows downward.
 */
#ifndef TABI_ORACLE_H
#define TABI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_KMAX 10   /* largest number of local-AABB slices per axis */

/* Per-chart proxy record, in the chart's final local frame (after the
 * 90-degree turn and the reflections).  Units: Q8. */
typedef struct {
  int32_t valid;          /* 0: degenerate chart (fewer than 3 vertices, zero extent, huge coords) */
  int32_t rot, flipx, flipy;
  int64_t xmin, ymin;     /* input AABB origin */
  int64_t W, H;           /* final-frame extents, H >= W */
  int32_t K;              /* slices per axis */
  int64_t ylo[ORC_KMAX], yhi[ORC_KMAX];  /* x-slices: v-range of chart within u in [jW/K,(j+1)W/K] */
  int64_t xlo[ORC_KMAX], xhi[ORC_KMAX];  /* y-slices: u-range of chart within v in [jH/K,(j+1)H/K] */
  int32_t obb;            /* 1 when the chosen box is not axis aligned */
  int32_t obb_m;          /* index of the chosen direction, 0..7 */
  int64_t C, S;           /* box axes: p = C u + S v, q = -S u + C v (C, S > 0 when obb) */
  int64_t a, b, e, f;     /* box: a <= p <= b, e <= q <= f */
  int64_t area2;          /* twice the polygon area, Q8^2 */
} orc_chart;

/* Proxy construction for one chart (Sec. 4.1.1, App. A). */
int orc_prep_chart(const int32_t* xy, int32_t nverts, int32_t K, orc_chart* out);

/* Undilated per-texel profiles at scale k/64 (App. A, "Parallel Pushing").
 * top/bot: w entries; left/right: h entries.  Returns w and h. */
void orc_profiles(const orc_chart* ch, int32_t k, int32_t* w, int32_t* h,
                  int32_t* top, int32_t* bot, int32_t* left, int32_t* right);

/* Per-proxy left / right of each texel row at scale k/64 (Sec. 4.1.1):
 * la, ra from the local AABBs, lo, ro from the OBB kept inside the chart's
 * texel box.  h entries each; returns h. */
void orc_row_proxies(const orc_chart* ch, int32_t k, int32_t* h, int32_t* la, int32_t* ra,
                     int32_t* lo, int32_t* ro);

/* Proxy construction with K slices (1..10); use_obb 0 keeps the chart's
 * axis-aligned box as its second proxy. */
int orc_prep_chart_ex(const int32_t* xy, int32_t nverts, int32_t K, int32_t use_obb,
                      orc_chart* out);

/* Proxy construction for a chart of nl loops: loop l is vertices
 * [lofs[l], lofs[l+1]) of xy (lofs[0] = 0). */
int orc_prep_chart_loops(const int32_t* xy, const int32_t* lofs, int32_t nl, int32_t K,
                         orc_chart* out);

/* Quality preset -> slices K and t_opt percent for a set of n charts. */
void orc_quality(int32_t quality, int32_t n, int32_t* K, int32_t* topt);

/* Whole pack of charts given as one or more boundary loops each: loop l is
 * vertices [loop_offsets[l], loop_offsets[l+1]) of xy, chart c is loops
 * [chart_loops[c], chart_loops[c+1]) (at least one).  Outputs as
 * tabi_oracle_pack. */
int tabi_oracle_pack_loops(const int32_t* xy, const int32_t* loop_offsets,
                           const int32_t* chart_loops, int32_t n, int32_t Wa, int32_t Ha,
                           int32_t p, int32_t q, int32_t* out_xy, uint8_t* out_orient,
                           float* out_scale, int32_t* out_k);

/* Whole pack with the hybrid tail of Sec. 4.4 (prefix-sum folding of the
 * charts after the t_opt switch, downscaled to fit, and the candidate scale
 * chosen by the area-weighted final scale).  K slices, t_opt percent (-1:
 * the paper's setting).  out_ks[c]: chart c's own k (0 when nothing fits);
 * out_k: the head's k (0 no fit, -1 degenerate chart). */
int tabi_oracle_pack_hybrid(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                            int32_t Ha, int32_t p, int32_t K, int32_t topt, int32_t* out_xy,
                            uint8_t* out_orient, int32_t* out_ks, int32_t* out_k);
/* One candidate k of it: returns 1 feasible, 0 not, -1 bad arguments, -2 a
 * degenerate chart; positions in sorted order, the tail's first chart t0 (n:
 * no tail) and its k. */
int tabi_oracle_feasible_hybrid(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                                int32_t Ha, int32_t p, int32_t K, int32_t topt, int32_t k,
                                int32_t* out_xs, int32_t* out_ys, uint8_t* out_mir,
                                int32_t* out_t0, int32_t* out_kt);

/* Pre-rotation of one chart to its tight box over 64 directions m pi/128
 * (Sec. 5 "Experimental Setup"): turned vertices (Q8, new box corner at the
 * origin) into out[2 nv]; returns and stores the direction m (0, vertices
 * copied, for a chart the pack rejects). */
int orc_prerotate(const int32_t* xy, int32_t nv, int32_t* out, int32_t* m_out);

/* Whole pack after pre-rotating every chart; out_dir[n] = its direction. */
int tabi_oracle_pack_prerotate(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                               int32_t Ha, int32_t p, int32_t q, int32_t* out_xy,
                               uint8_t* out_orient, uint8_t* out_dir, float* out_scale,
                               int32_t* out_k);

/* Variants of the method (Sec. 5 ablations). */
enum { ORC_FULL = 0, ORC_TIGHT_ONLY = 1, ORC_BALANCED_ONLY = 2 };

/* Whole pack with the method's knobs: K local AABBs per axis (1..10; the
 * balanced-only variant uses 1), t_opt percent (< 0: the paper's setting,
 * 0 up to 10,000 charts, 1 above), variant ORC_*.  Outputs as
 * tabi_oracle_pack; -1 on invalid arguments. */
int tabi_oracle_pack_method(const int32_t* xy, const int32_t* offsets, int32_t n, int32_t Wa,
                            int32_t Ha, int32_t p, int32_t K, int32_t topt, int32_t variant,
                            int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                            int32_t* out_k);

/* Whole pack.  Returns 0 on success, -1 on invalid arguments.
 * out_xy[2n]: texel (X,Y) of each chart's box top-left, out_orient[n]: bit0 turn,
 * bit1 flipX, bit2 flipY, bit3 row mirror.  *out_scale = k* / 64, 0 if no k
 * fits, -1 if some chart is degenerate.  *out_k = k* (0 / -1 likewise). */
int tabi_oracle_pack(const int32_t* xy, const int32_t* offsets, int32_t n,
                     int32_t atlas_w, int32_t atlas_h, int32_t padding, int32_t quality,
                     int32_t* out_xy, uint8_t* out_orient, float* out_scale, int32_t* out_k);

/* Diagnostics ------------------------------------------------------------ */

/* Fold-and-push at one scale (Alg. 3).  Returns 1 if every chart is placed
 * without overflow, 0 otherwise, -1 on bad arguments.  Positions / orientation
 * of the charts placed so far are written in input order (others -1 and 0);
 * rows_out (optional) receives the number of committed rows. */
int tabi_oracle_feasible(const int32_t* xy, const int32_t* offsets, int32_t n,
                         int32_t atlas_w, int32_t atlas_h, int32_t padding, int32_t quality,
                         int32_t k, int32_t* out_xy, uint8_t* out_orient, int32_t* rows_out);

/* Sorted order (position -> input index) and the area bound k_hi. */
int tabi_oracle_order(const int32_t* xy, const int32_t* offsets, int32_t n,
                      int32_t atlas_w, int32_t atlas_h, int32_t quality,
                      int32_t* perm, int32_t* k_hi);

/* Horizontal compacting distance and interlock flags of every adjacent sorted
 * pair at scale k: cd[c], flags[c] (bit0: c may not move above c-1,
 * bit1: c-1 may not move above c) for c >= 1; cd[0] = flags[0] = 0.
 * cd is the larger of the local-AABB and the OBB distance (Sec. 4.1.2);
 * the flags come from the proxy that gave it (App. A). */
int tabi_oracle_pairs(const int32_t* xy, const int32_t* offsets, int32_t n,
                      int32_t padding, int32_t quality, int32_t k,
                      int32_t* cd, uint8_t* flags);

/* Interlock flags of two dilated row profiles at horizontal offset d
 * (B starts d texels right of A).  Returns bit0 = B may not move above A,
 * bit1 = A may not move above B.  Zero when d >= wdA (no shared columns). */
int orc_interlock(const int32_t* rightA, int32_t hdA, int32_t wdA,
                  const int32_t* leftB, int32_t hdB, int32_t d);

/* UpdateKneeLocation (Alg. 4) on a committed frontline F[Wd] for a knee of
 * direction dir (0 left-to-right, 1 right-to-left) spanning [left, right);
 * updates the span and returns 0 when the knee ends (its probe texel lies
 * outside the frontline), 1 otherwise. */
int orc_knee_update(const int32_t* F, int32_t Wd, int32_t dir, int32_t* left, int32_t* right);

/* CorrectYOffsets over m constrained pairs pa[3q..3q+2] = (A, B, flags):
 * flags bit0 -> y[B] >= y[A], bit1 -> y[A] >= y[B]; y updated in place. */
void orc_correct(int32_t m, const int32_t* pa, int32_t* y);

#ifdef __cplusplus
}
#endif
#endif
