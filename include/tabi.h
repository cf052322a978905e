/*
 * tabi.h - C ABI of the MI355X TABI atlas packer.
 *
 * Packs 2D polygon charts into a fixed-size texture atlas following
 * "TABI: Tight and Balanced Interactive Atlas Packing" (Gu, Vining, Sheffer,
 * Eurographics 2026).  The problem (Sec. 4, "Method", first paragraph): charts
 * are polygons in texel units, the atlas has fixed dimensions; the output is
 * one scale for all charts plus, per chart, a rigid transform (quarter turn,
 * reflections, translation) such that no two charts nor their gutters overlap.
 * The scale is the largest of the 64 factors k/64 whose packing succeeds
 * (Sec. 5, "Experimental Setup"; Sec. 4.3).
 *
 * Conventions shared by every entry point
 *  - Vertex coordinates are int32 fixed point with 8 fractional bits ("Q8",
 *    1/256 texel); y grows downward.  Chart c is one simple polygon loop given
 *    by vertices [offsets[c], offsets[c+1]) of the interleaved array xy.
 *  - All arrays passed to tabi_pack / tabi_pack_many are DEVICE pointers owned
 *    by the caller.  The library never frees or retains them.
 *  - The functions are asynchronous and ordered on `stream` (0 = the null
 *    stream).  Work space is taken from, and returned to, the device's
 *    stream-ordered memory pool on the same stream; calls on different streams
 *    are independent.
 *  - The return value reports only errors the host can see.  Conditions found
 *    on the device are written into out_scale (see tabi_pack).
 *  - Gutters: `padding` is the minimum number of empty texels between two
 *    charts (the paper's 1-pixel gutters around charts correspond to
 *    padding = 2), 0 <= padding <= TABI_MAX_PADDING.  Charts may touch the
 *    atlas edges.
 *  - quality selects the paper's quality/speed knob (Sec. 5 ablations):
 *      0: 2 local AABBs per axis, t_opt = 5 %
 *      1: 5 local AABBs per axis, t_opt = 2 %
 *      2: 10 local AABBs per axis, t_opt = 0 % up to 10,000 charts, 1 % above
 *         (the paper's default).
 */
#ifndef TABI_H
#define TABI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* tabi_stream_t; /* a hipStream_t */

enum {
  TABI_OK = 0,
  TABI_EINVAL = -1, /* bad argument: null pointer, n < 0 or n > TABI_MAX_CHARTS,
                       atlas side < 1, side + padding > 16384, padding < 0 or
                       padding > TABI_MAX_PADDING,
                       quality not in {0,1,2}, count < 0, work space too small,
                       or a wide atlas with more charts than the packing
                       kernel's shared memory holds (see tabi_pack_lds_bytes) */
  TABI_ENOMEM = -2, /* the device memory pool could not supply the work space */
  TABI_EHIP = -3,   /* a HIP runtime call failed (launch, memory); see tabi_last_hip_error */
  TABI_ETOOBIG = -4, /* tabi_pack_noalloc: the input needs more work space than its
                       static array of TABI_NOALLOC_BYTES holds; a served request
                       larger than the serving context's memory or staging */
  TABI_ENOTRESIDENT = -5 /* a served re-pack of an atlas whose records are no longer
                            resident (evicted under the memory budget) */
};

#define TABI_MAX_CHARTS 262144 /* charts per atlas */
#define TABI_MAX_PADDING 32    /* gutter texels; the gutter growth of a texel profile is
                                  taken within one 64-lane wavefront */

typedef struct {
  const int32_t* xy;      /* device int32[2*total_verts]: x0,y0,x1,y1,... in Q8 */
  const int32_t* offsets; /* device int32[n+1]: CSR vertex offsets, offsets[0] = 0 */
  int32_t total_verts;    /* V = offsets[n] */
} tabi_charts;

/* Pack n charts into an atlas_w x atlas_h texel atlas (Alg. 3 for every
 * candidate scale, largest success returned; Sec. 4.3).
 *
 * Outputs (device memory, written before the stream reaches the end of the call):
 *   out_xy[2c], out_xy[2c+1]: texel column X and row Y of the top-left corner
 *       of chart c's box in the atlas.
 *   out_orient[c]: bit0 quarter turn applied first, (u,v) -> (h0 - v, u) in
 *       the chart's box (h0 its input height); bit1 mirror in x inside the box;
 *       bit2 mirror in y inside the box; bit3 mirror in x inside the scaled
 *       texel box (rows placed right to left).  With s = k/64 the atlas
 *       position of a chart point, in texels, is (X + s*u', Y + s*v') where
 *       (u', v') is the point after bits 0-2, and bit3 then maps
 *       s*u' -> ceil(s*W') - s*u' (W' the box width after bit0).
 *   out_scale[0]: k/64 for the chosen k >= 1 (exact);
 *        0.0f if no scale fits (out_xy filled with -1);
 *       -1.0f if some chart is degenerate: fewer than 3 vertices, zero width
 *             or height, or a coordinate with |x| >= 2^22 (out_xy filled with -1).
 * Errors: TABI_EINVAL, TABI_ENOMEM, TABI_EHIP (nothing is written then). */
int tabi_pack(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
              int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
              float* out_scale, tabi_stream_t stream);

/* Charts of one or more boundary loops each (a mesh chart's outer boundary
 * and holes, or several islands packed as one chart; all device arrays):
 * loop l is vertices [loop_offsets[l], loop_offsets[l+1]) of xy (Q8,
 * loop_offsets[0] = 0), chart c is loops [chart_loops[c], chart_loops[c+1])
 * (chart_loops[0] = 0, at least one loop per chart, total_loops of them). */
typedef struct {
  const int32_t* xy;
  const int32_t* loop_offsets;
  const int32_t* chart_loops;
  int32_t total_loops;
} tabi_charts_loops;

/* tabi_pack for charts of several loops: the proxies (Sec. 4.1.1) bound the
 * edges and vertices of every loop, and the area that bounds the scale from
 * above is the largest loop's less all others' (exact for an outer loop with
 * holes, a lower bound for islands, so no feasible scale is skipped).  A
 * chart with a loop of fewer than 3 vertices is degenerate (out_scale -1).
 * Outputs and errors as tabi_pack. */
int tabi_pack_loops(const tabi_charts_loops* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                    int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
                    float* out_scale, tabi_stream_t stream);

/* tabi_pack after turning every chart to its tight box (Sec. 5,
 * experimental setup: UV charts are pre-rotated so that their tight bounding
 * boxes are axis-aligned; texture-space-shading charts are not).  The box is
 * the least-area one over 64 directions m*pi/128, m = 0..63 (the OBB proxy's
 * 8 directions are m = 0, 8, ..., 56), with C = round(2^14 cos(m*pi/128)),
 * S = round(2^14 sin(m*pi/128)); areas are compared exactly and ties go to
 * the smaller m.  Vertex (x, y) of chart c, with (x0, y0) the corner of the
 * chart's input box, becomes
 *     x' = floor((C (x - x0) + S (y - y0) + 2^13) / 2^14) - tx
 *     y' = floor((C (y - y0) - S (x - x0) + 2^13) / 2^14) - ty
 * (a turn by -m*pi/128, rounded to the nearest Q8 unit) with (tx, ty) the
 * smallest such values, so that the turned box starts at (0, 0).
 *   out_rxy: device int32[2*total_verts], the turned vertices (CSR offsets as
 *            charts->offsets); it may be charts->xy itself (turned in place).
 *   out_dir: device uint8[n], the direction m of each chart.
 * A chart the pack rejects as degenerate (fewer than 3 vertices, a
 * coordinate with |x| >= 2^22) is copied unchanged with m = 0.
 * out_xy, out_orient, out_scale: as tabi_pack, for the turned charts.
 * Errors: TABI_EINVAL (nothing written); TABI_ENOMEM or TABI_EHIP after the
 * pre-rotation has been enqueued (out_rxy and out_dir may be written). */
int tabi_pack_prerotate(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                        int32_t padding, int32_t quality, int32_t* out_rxy, uint8_t* out_dir,
                        int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                        tabi_stream_t stream);

/* The method's knobs (Sec. 5 "Ablations"; App. D, local-AABB count and t_opt
 * tables), for the ablation variants and sweeps.  The quality presets are
 * {2, 5, FULL}, {5, 2, FULL} and {10, -1, FULL}.
 *   slices:        local AABBs per axis: 1, 2, 5 or 10 (Sec. 4.1.1)
 *   topt_percent:  t_opt of Sec. 4.4 in percent of the atlas height, 0..100;
 *                  -1: the paper's setting, 0 up to 10,000 charts and 1 above
 *   variant:       TABI_FULL: the method;
 *                  TABI_TIGHT_ONLY: tightness without balanced folding (every
 *                  row folded at the atlas width with compaction, one
 *                  left-to-right row to two right-to-left rows, no knees, no
 *                  per-row choices);
 *                  TABI_BALANCED_ONLY: balanced folding without tightening
 *                  (the charts' boxes as proxies: one slice per axis whatever
 *                  `slices` says, no OBB, so no compaction and no reflection). */
enum { TABI_FULL = 0, TABI_TIGHT_ONLY = 1, TABI_BALANCED_ONLY = 2 };
typedef struct {
  int32_t slices, topt_percent, variant;
} tabi_method;

/* tabi_pack with the method's knobs instead of a quality preset.
 * TABI_EINVAL for knobs outside the ranges above. */
int tabi_pack_method(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, const tabi_method* method, int32_t* out_xy,
                     uint8_t* out_orient, float* out_scale, tabi_stream_t stream);

/* tabi_pack_method with the hybrid tail of Sec. 4.4 ("Performance
 * Optimization"), for the full method (method->variant = TABI_FULL).  Rows
 * are folded and pushed one by one until the t_opt switch (no knee pending
 * and the row's first chart shorter than t_opt of the atlas height); the
 * remaining charts, in sorted order, are then folded all at once: each
 * chart's offset is its grown width less its compacting distance to the next
 * chart, and the prefix sum of the offsets divided by the grown atlas width
 * W + padding gives its row.  The tail is downscaled to the largest k' <= k
 * at which every such row, laid out with compaction at k', fits the width;
 * its rows are placed in the fixed one left-to-right : two right-to-left
 * alternation and pushed up at k'.  Head and tail scales differ, so the
 * candidate k is the one whose packing succeeds with the largest sum over
 * charts of area * final scale (ties to the larger k), searched over all 64.
 * Outputs as tabi_pack, except:
 *   out_scale[0]:       k/64 of the rows before the switch (or 0 / -1 as
 *                       tabi_pack);
 *   out_chart_scale[c]: device float[n], chart c's own scale (k/64 before
 *                       the switch, k'/64 in the tail; 0 when nothing fits),
 *                       which takes the place of s in tabi_pack's transform.
 * With t_opt 0 there is no tail and the result is tabi_pack_method's.
 * Errors: TABI_EINVAL (also for a variant other than TABI_FULL), TABI_ENOMEM,
 * TABI_EHIP. */
int tabi_pack_hybrid(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, const tabi_method* method, int32_t* out_xy,
                     uint8_t* out_orient, float* out_chart_scale, float* out_scale,
                     tabi_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tabi_pack
 * with the same arguments, outputs and device-detected conditions, whose work
 * space is a static device array of TABI_NOALLOC_BYTES held by every GPU the
 * library runs on until the process ends.  It calls no allocation routine
 * and no memset (its kernels initialise what they read).  The per-scale
 * profile arena takes what the fixed arrays leave of the array; segments
 * beyond it are evaluated from the proxy records, so results equal
 * tabi_pack's bit for bit (larger inputs run slower, not differently).
 * About 2,000 charts of a 2048^2 atlas at quality 2 fit with their profiles
 * stored, about 7,000 charts at all.
 * Every call on one GPU uses that GPU's one array: calls that overlap on the
 * same GPU (different streams, or host threads) race and give wrong results;
 * order them on one stream.
 * Errors: as tabi_pack, and TABI_ETOOBIG when the input's fixed work space
 * (per-chart records and per-(scale, chart) set-up) exceeds the array. */
#define TABI_NOALLOC_BYTES (128ll << 20)
int tabi_pack_noalloc(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                      int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
                      float* out_scale, tabi_stream_t stream);

/* Pack `count` independent atlases in one set of launches (batched path).
 * Charts of all atlases form one CSR (xy, vert_offsets over all charts, device
 * int32); atlas a owns charts [atlas_offsets[a], atlas_offsets[a+1]) and is
 * atlas_wh[2a] x atlas_wh[2a+1] texels (device int32 arrays).  The host
 * arguments total_charts (= atlas_offsets[count]), max_charts (most charts in
 * one atlas) and max_side (largest atlas side) size the work space and shared
 * memory without reading device memory; an atlas exceeding them gets
 * out_scale = -2.  out_xy / out_orient are indexed by global chart index,
 * out_scale by atlas.  Per atlas the result equals tabi_pack on that atlas
 * alone: every atlas evaluates its candidate scales from the largest down in
 * rounds (a few scales per atlas per round, the number set by the batched
 * shape, see tabi_tune_many) and stops at the first round with a success.
 * padding and quality are shared.  Errors as tabi_pack. */
int tabi_pack_many(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                   int32_t count, const int32_t* atlas_wh, int32_t total_charts,
                   int32_t max_charts, int32_t max_side, int32_t padding, int32_t quality,
                   int32_t* out_xy, uint8_t* out_orient, float* out_scale,
                   tabi_stream_t stream);

/* tabi_pack_many with the method's knobs (shared by the batch) instead of a
 * quality preset; batched shapes are those tuned for the preset with the
 * nearest slice count. */
int tabi_pack_many_method(const int32_t* xy, const int32_t* vert_offsets,
                          const int32_t* atlas_offsets, int32_t count, const int32_t* atlas_wh,
                          int32_t total_charts, int32_t max_charts, int32_t max_side,
                          int32_t padding, const tabi_method* method, int32_t* out_xy,
                          uint8_t* out_orient, float* out_scale, tabi_stream_t stream);

/* Bytes of device work space tabi_pack_many_ws needs for this batch shape
 * (host only; -1 for a bad shape). */
int64_t tabi_pack_many_workspace_bytes(int32_t count, int32_t total_charts, int32_t max_charts,
                                       int32_t max_side, int32_t padding, int32_t quality);

/* tabi_pack_many on a caller-provided device work space of workspace_bytes
 * (at least tabi_pack_many_workspace_bytes).  Launches kernels only (no
 * allocation, no memset), so a caller may capture it in a HIP graph and
 * replay it; calls sharing one work space must not overlap. */
int tabi_pack_many_ws(const int32_t* xy, const int32_t* vert_offsets,
                      const int32_t* atlas_offsets, int32_t count, const int32_t* atlas_wh,
                      int32_t total_charts, int32_t max_charts, int32_t max_side,
                      int32_t padding, int32_t quality, int32_t* out_xy, uint8_t* out_orient,
                      float* out_scale, void* workspace, int64_t workspace_bytes,
                      tabi_stream_t stream);

/* ---- batched shape autotuning ---------------------------------------------
 * tabi_pack_many evaluates every atlas's candidate scales in rounds of B
 * descending scales (one fold-and-push workgroup per (atlas, scale)); B, the
 * workgroup size (512 or 1024 threads) and its shared-memory cap (two
 * 512-thread workgroups per CU, or one with the whole LDS) form its shape.
 * Results never depend on the shape, only the speed does.
 *
 * tabi_tune_many packs the given batch (arguments as tabi_pack_many) once
 * untimed and `reps` times timed with HIP events on `stream` for each of the
 * tabi_many_shape_count() candidate shapes, keeps the fastest as the shape of
 * later tabi_pack_many / _ws / _records calls with this quality and a batch
 * of the same size class (up to 8 atlases, up to 64, more) on the current
 * device, and writes it to shape[5] = {b0, flat, bmax, threads, LDS cap bytes
 * (0: device limit)}: the search runs rounds of b0 scale slots for the first
 * `flat` rounds, then doubles the slots per round up to bmax until the 64
 * candidate scales are covered, with fold-and-push workgroups of `threads`
 * threads; ms_per_shape (may be NULL) receives the mean milliseconds
 * per call of each candidate (-1 for a shape the batch's rows do not fit).
 * Synchronizes `stream`.  A workspace sized with
 * tabi_pack_many_workspace_bytes before tuning must be sized again after it
 * (the round size changes the work space).  Outputs hold the last call's
 * results. */
int tabi_tune_many(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                   int32_t count, const int32_t* atlas_wh, int32_t total_charts,
                   int32_t max_charts, int32_t max_side, int32_t padding, int32_t quality,
                   int32_t* out_xy, uint8_t* out_orient, float* out_scale, int32_t reps,
                   int32_t* shape, float* ms_per_shape, tabi_stream_t stream);

/* Current batched shape for `quality` and a batch of `count` atlases on the
 * current device (shape[5] as above); the number of candidate shapes the
 * tuner tries. */
int tabi_many_shape(int32_t quality, int32_t count, int32_t* shape);
int32_t tabi_many_shape_count(void);

/* Test knob: make candidate shape `index` (0 .. tabi_many_shape_count()-1;
 * negative: the default, index 0) the batched shape for `quality` and every
 * batch size on the current device. */
int tabi_debug_set_many_shape(int32_t quality, int32_t index);

/* ---- resident proxies (incremental re-packs) ----------------------------
 * The per-chart proxies of Sec. 4.1.1 (box, turn, reflections, local AABBs,
 * OBB; everything that does not depend on the scale) as opaque device
 * records of tabi_record_bytes() bytes each.  A server keeps them resident;
 * a re-pack that replaces some charts recomputes only those records. */
int64_t tabi_record_bytes(void);

/* Records of total_charts charts grouped into `count` atlases
 * (atlas_offsets over the charts, device int32[count+1]); a record keeps its
 * chart's index within its atlas.  quality fixes the number of slices and
 * must match the later pack.  records: device buffer of
 * total_charts * tabi_record_bytes() bytes. */
int tabi_prep_records(const int32_t* xy, const int32_t* vert_offsets, const int32_t* atlas_offsets,
                      int32_t count, int32_t total_charts, int32_t quality, void* records,
                      tabi_stream_t stream);

/* records[index[i]] = new_records[i] for i < m (device arrays), keeping the
 * replaced chart's index within its atlas. */
int tabi_splice_records(void* records, const int32_t* index, int32_t m, const void* new_records,
                        tabi_stream_t stream);

/* tabi_pack_many starting from resident records instead of polygons; the
 * result equals tabi_pack_many on the polygons the records came from. */
int tabi_pack_many_records(const void* records, const int32_t* atlas_offsets, int32_t count,
                           const int32_t* atlas_wh, int32_t total_charts, int32_t max_charts,
                           int32_t max_side, int32_t padding, int32_t quality, int32_t* out_xy,
                           uint8_t* out_orient, float* out_scale, tabi_stream_t stream);

/* ---- serving (continuous batching with resident proxies) ----------------
 * A serving context admits pack requests as they arrive and runs them in
 * batches, one batch per launch slot (a HIP stream of its own), so batches on
 * different slots overlap on the GPU and requests that arrive while others
 * run join the next batch as slots and memory free up.  Each atlas's chart
 * proxy records (Sec. 4.1.1) stay resident on the device, so a re-pack with
 * some charts replaced recomputes only those charts' records.  A request's
 * result equals tabi_pack of its chart set alone, bit for bit.
 *
 * Memory: the context allocates, once at creation, device_bytes of device
 * memory (batches in flight and resident records, admitted by footprint;
 * least recently used atlases are evicted when a batch needs room) and two
 * pinned host staging buffers of staging_bytes per slot.  Nothing else is
 * allocated afterwards.  Unlike tabi_pack, chart data and outputs are HOST
 * arrays: inputs are copied before tabi_submit / tabi_repack return; the
 * output arrays must stay valid until tabi_poll reports the ticket done.
 * A context is used from one host thread at a time. */
typedef struct tabi_ctx tabi_ctx;
typedef struct {
  int32_t quality, padding; /* as tabi_pack, shared by every request */
  int32_t streams;          /* launch slots, 1..16 */
  int32_t max_batch;        /* requests per batch, 1..1024 */
  int64_t device_bytes;     /* device memory budget (>= 1 MiB) */
  int64_t staging_bytes;    /* pinned staging per slot and direction (>= 64 KiB) */
} tabi_ctx_config;
typedef struct {
  int64_t ticket;
  int32_t atlas_id;
  int32_t status;      /* TABI_OK, TABI_ETOOBIG, TABI_ENOTRESIDENT or a launch error */
  int32_t batch;       /* batch it ran in (0: it did not run) */
  int32_t pad;
  double latency_ms;   /* submission to completion of its batch on the GPU */
  double submit_ms;    /* submission time since the context was created */
  double done_ms;      /* completion time since the context was created */
} tabi_done;

/* Errors: TABI_EINVAL for a bad configuration; TABI_ENOMEM / TABI_EHIP if
 * the memory, streams or events cannot be created (*ctx stays NULL). */
int tabi_ctx_create(const tabi_ctx_config* cfg, tabi_ctx** ctx);
/* Waits for the batches in flight, then releases everything. */
int tabi_ctx_destroy(tabi_ctx* ctx);
/* A pack of a new atlas: n >= 1 charts (host CSR: xy int32[2*offsets[n]]
 * in Q8, offsets int32[n+1]) into atlas_w x atlas_h.  Returns the atlas id
 * its records stay resident under and a ticket.  Outputs as tabi_pack
 * (host arrays): out_xy int32[2n], out_orient uint8[n], out_scale float[1]. */
int tabi_submit(tabi_ctx* ctx, const int32_t* xy, const int32_t* offsets, int32_t n,
                int32_t atlas_w, int32_t atlas_h, int32_t* out_xy, uint8_t* out_orient,
                float* out_scale, int32_t* atlas_id, int64_t* ticket);
/* tabi_submit with the request's own padding and quality preset instead of
 * the context's: requests are batched only with consecutive requests of the
 * same settings (tabi_pack_many shares them across a batch).  Re-packs keep
 * the settings of their atlas. */
int tabi_submit_with(tabi_ctx* ctx, const int32_t* xy, const int32_t* offsets, int32_t n,
                     int32_t atlas_w, int32_t atlas_h, int32_t padding, int32_t quality,
                     int32_t* out_xy, uint8_t* out_orient, float* out_scale, int32_t* atlas_id,
                     int64_t* ticket);
/* A re-pack of a resident atlas whose charts replaced_idx[0..m) (strictly
 * increasing indices of its current chart set) are replaced by the m charts
 * of the host CSR (xy, offsets); every other chart keeps its records and its
 * index.  The atlas's chart set becomes the new one (later re-packs build on
 * it, in submission order).  Outputs as tabi_submit, for the whole atlas. */
int tabi_repack(tabi_ctx* ctx, int32_t atlas_id, const int32_t* replaced_idx, int32_t m,
                const int32_t* xy, const int32_t* offsets, int32_t* out_xy,
                uint8_t* out_orient, float* out_scale, int64_t* ticket);
/* Retire completed batches (their outputs are written to the callers'
 * arrays), admit queued requests into free slots, and report up to max_done
 * finished tickets in done[0..*n_done).  wait != 0: block until at least one
 * batch completes when none is reported yet and some are in flight. */
int tabi_poll(tabi_ctx* ctx, int32_t wait, tabi_done* done, int32_t max_done, int32_t* n_done);
/* stats[0..nstats): batches launched, requests finished, requests failed,
 * atlases evicted, atlases resident, device bytes in use, peak device bytes,
 * requests queued, batches in flight, cross-slot waits, most batches in
 * flight at once. */
int tabi_ctx_stats(tabi_ctx* ctx, int64_t* stats, int32_t nstats);

/* ---- diagnostics (same conventions; device pointers) ------------------- */

/* Sorted chart order (Sec. 3.1: height descending, then width descending,
 * then input index) and the largest candidate scale k_top (total chart area
 * and the largest chart must fit the atlas at k_top / 64).
 * perm[t] = input index of the t-th chart; khi[0] = k_top, or -1 if a chart
 * is degenerate. */
int tabi_debug_order(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                     int32_t padding, int32_t quality, int32_t* perm, int32_t* khi,
                     tabi_stream_t stream);

/* Horizontal compacting distance and interlock flags of each sorted neighbour
 * pair (c-1, c) at scale k/64 (Sec. 4.1.2, App. A): cd[c] in texels and
 * flags[c] (bit0: c may not move above c-1; bit1: c-1 may not move above c);
 * cd[0] = flags[0] = 0.  Indexed by sorted position. */
int tabi_debug_pairs(const tabi_charts* charts, int32_t n, int32_t padding, int32_t quality,
                     int32_t k, int32_t* cd, uint8_t* flags, tabi_stream_t stream);

/* Fold-and-push at the single scale k/64 (Alg. 3).  feasible[0] = 1 if every
 * chart was placed within the atlas height, 0 if a row overflowed or a chart
 * is wider than the atlas; out_xy / out_orient as in tabi_pack for the charts
 * placed before the scan stopped, -1 / 0 for the rest; rows[0] = number of
 * rows committed. */
int tabi_debug_feasible(const tabi_charts* charts, int32_t n, int32_t atlas_w, int32_t atlas_h,
                        int32_t padding, int32_t quality, int32_t k, int32_t* out_xy,
                        uint8_t* out_orient, int32_t* feasible, int32_t* rows,
                        tabi_stream_t stream);

/* Diagnostic: with the library built with TABI_PHASE_CLOCK defined
 * (`python -m paper_2602_07782_amd.build --phase-clock`, a separate
 * libtabi_hip_phase.so), the fold-and-push kernel of a single pack sums per
 * scale slot the device's constant 100 MHz clock between the phases of its
 * rows as wavefront 0 sees them.  Writes 11 values per slot for `slots`
 * slots (at most 64) to host memory `out`: [0] the previous row's commit and
 * the loop head, [1] knee update, [2] fold, [3] configurations and staging,
 * [4] push, [5] correction and score, [6] selection and knee detection,
 * [7] rows whose pairs that share columns without being neighbours overflow
 * the shared list, times 2^32, plus the number of such pairs (the list's
 * count, capped at its overflow), [8] rows, [9] the slot's scale k, [10] its
 * outcome (1 feasible, 0 not), from the last pack.  Returns the number of slots written;
 * TABI_EINVAL when the library was built without the clock. */
int tabi_debug_phase_clock(int64_t* out, int32_t slots);

/* Test knob: cap the per-row LDS staging of texel bounds at `entries`
 * (texel columns; -1 restores the default).  Rows that do not fit read the
 * stored bounds from device memory; results are identical either way. */
int tabi_debug_set_stage_cap(int32_t entries);

/* Test knob: cap the packing kernel's shared memory for its rows at `bytes`,
 * but never below the smallest plan (the frontline, one set of fold offsets
 * and four configurations' offsets of a full row; -1 restores the default,
 * the device's limit).  A smaller row pool stages fewer rows and folds fewer
 * rows while the row before them commits (only rows that fit the second set
 * of offsets at the pool's top are).  Results are identical either way. */
int tabi_debug_set_pack_lds(int32_t bytes);

/* Test knob: size of the per-call arena of stored per-texel profiles, in
 * 32-bit words (one per grown texel column or row of a chart at a scale;
 * -1 restores the default, 0 stores none).  Charts whose profiles do not fit
 * are evaluated from their proxy records inside the pairing and packing
 * kernels; results are identical either way.  Affects later calls of this
 * process, including tabi_pack_many_workspace_bytes. */
int tabi_debug_set_profile_cap(int64_t words);

/* Returns to the device the memory that earlier calls left in the current
 * device's stream-ordered pool (work spaces are taken from that pool and kept
 * there between calls so that later calls reuse them).  Waits for all work on
 * the device first, so no call may be in flight on another thread.  The
 * library stays usable; the next call takes fresh memory.  TABI_EHIP if the
 * device or its pool is unavailable. */
int tabi_shutdown(void);

/* Text for a return code; last HIP error string seen by the library. */
const char* tabi_strerror(int code);
const char* tabi_last_hip_error(void);

/* Stage timing (host side).  When enabled, the calling process brackets each
 * stage of later tabi_pack / tabi_pack_many calls with a pair of HIP events on
 * the call's stream.  Stages, in order: 0 chart proxies (prep), 1 sort and
 * scale bound, 2 per-scale set-up, 3 per-texel profiles and neighbour pairs,
 * 4 fold-and-push, 5 scale selection.  tabi_timing_read waits for the recorded events and writes the
 * summed milliseconds and the number of bracketed launches per stage since
 * the last reset (arrays of nstages entries, either may be NULL).
 * tabi_timing_stages selects the stages bracketed while timing is enabled
 * (bit s for stage s; all six by default): each pair of events adds a few
 * microseconds to the call, so a caller that times whole calls brackets only
 * the stages it needs.  TABI_EINVAL for an empty mask or bits past stage 5. */
int tabi_timing_enable(int on);
int tabi_timing_stages(uint32_t mask);
int tabi_timing_read(double* ms, int32_t* launches, int32_t nstages);
void tabi_timing_reset(void);

/* Device shared memory (bytes) the packing kernel will use for an atlas of
 * width atlas_w + padding and n charts (host only; no device work).  The
 * row state of one scale lives in the packing kernel's shared memory: the
 * frontline (4 (W + p) bytes) and the offsets of a row's charts
 * (24 min(n, W + p) + 8 bytes at least).  A call whose atlas needs more than
 * the device's shared memory per workgroup less the kernel's own use (about
 * 148 KB on MI355X) returns TABI_EINVAL: this limits atlases of width 8192
 * to about 4,800 charts and of width 16384 to about 3,400; atlases up to
 * 4096 wide take any chart count up to TABI_MAX_CHARTS. */
int64_t tabi_pack_lds_bytes(int32_t n, int32_t atlas_w, int32_t padding);

#ifdef __cplusplus
}
#endif
#endif /* TABI_H */
