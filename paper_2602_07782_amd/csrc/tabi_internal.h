// Internal interface between the host runtime and the kernels of the TABI
// packer.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tabi_device.h"

namespace tabi {

// One atlas of a batch.
struct AtlasDesc {
  int32_t c0, n;       // charts [c0, c0+n) of the flattened chart arrays
  int32_t Wa, Ha;      // atlas size in texels
  int32_t ktop;        // largest candidate scale (plan); -1 degenerate chart; 0 none
  int32_t bad;         // set when a chart is degenerate
  int32_t done;        // a feasible scale has been found (or the search ended)
  int32_t kstar;       // chosen scale
};

struct Params {
  int32_t count;       // atlases
  int32_t N;           // charts over all atlases
  int32_t K;           // local AABB slices per axis
  int32_t q;           // quality preset
  int32_t p;           // padding
  int32_t B;           // scale slots of the largest round (stride of the per-slot arrays)
  int32_t Br;          // scale slots of the current round (<= B)
  int32_t koff;        // candidate scales the earlier rounds covered
  int32_t stride;      // bytes of one per-(scale, chart) record
  int32_t fixed_k;     // > 0: evaluate exactly this scale in slot 0 (diagnostics)
  int32_t nmax;        // largest chart count of one atlas the work space was sized for
  int32_t Wdmax;       // largest grown atlas width the shared memory was sized for
  int64_t arena_cap;   // 32-bit words of the profile arena (0: no stored profiles)
  int32_t pack_nt;     // fold-and-push workgroup size: 512, 1024, or 0 (by atlas count)
  int32_t topt;        // t_opt in percent; < 0: 0 up to 10,000 charts in the atlas, 1 above
  int32_t variant;     // 0 full, 1 tight-only (static rows), 2 balanced-only (boxes)
  int32_t hybrid;      // 1: after the t_opt switch the charts are folded by prefix sums at a
                       // scale of their own (Sec. 4.4); single atlas, every scale a slot
  int32_t loops;       // 1: charts of several boundary loops (not necessarily connected)
};

// Work-space views (device pointers).
constexpr int XCDS = 8;  // workgroups are dealt to the 8 XCDs in turn; each has its own L2
constexpr int MAX_ROUNDS = 64;  // a round covers at least one of the 64 scales
constexpr int PROF_CH = 16;  // charts per profile workgroup

struct Work {
  Chart* recs;          // [N] by input position
  Chart* srecs;         // [N] by sorted position (per atlas)
  uint64_t* keys;       // [N]
  int4* pl;             // [N] by input position, read by the scale plan: twice the area
                        // (low, high word), W, H; H = -1 marks a degenerate chart
  uint64_t* skey;       // [ceil(N / 256) * 256] key tiles of 256, each sorted by (atlas, key)
  int32_t* satl;        //   and the atlas of each entry (padding: largest atlas and key)
  int32_t* rank;        // [N] position of the chart within its atlas's sorted order
  int32_t* perm;        // [N] sorted position -> local input index
  int32_t* chart_atlas; // [N]
  AtlasDesc* desc;      // [count]
  unsigned char* kc;    // [B][N] per-(scale, chart) set-up records
  int32_t* cd;          // [B][N] compacting distance of (c-1, c)
  uint8_t* fl;          // [B][N] interlock flags of (c-1, c)
  int32_t* xs;          // [B][N] placed box column
  int32_t* ys;          // [B][N] placed box row
  uint8_t* mir;         // [B][N] row mirror bit
  int32_t* feas;        // [count][B] 1 feasible, 0 not, -1 not evaluated
  int32_t* rows;        // [count][B]
  int32_t* wdv;         // [B][N] grown width w + p at the slot's scale
  int32_t* hdv;         // [B][N] grown height h + p
  int32_t* kslot;       // [B][N] the chart's scale k at the slot, 0 when it does not run
  int32_t* pcol;        // [B][N] first grown column of the chart within its segment
  int32_t* prow;        // [B][N] first grown row of the chart within its segment
  int32_t* Hs;          // [N] unscaled height (Q8) by sorted position
  int32_t* lrpre;       // [B][N] rows with many non-neighbour pairs: prefix of their counts
  int64_t* segneed;     // [count][B] arena words of the (atlas, slot) segment
  int32_t* segbase;     // [count][B] arena word where the segment starts, -1: not stored
  int32_t* cnt;         // [count] fold-and-push workgroups of the atlas done this round
  int32_t* gq;          // [B][ceil(N / PROF_CH)] profile blocks queued for the general evaluation
  int32_t* gq_cnt;      // [1] queued blocks this round (cleared by the set-up kernel)
  int32_t* aord;        // [count] dispatch order of the packing kernel's atlases
  int32_t* live;        // [MAX_ROUNDS + 1] live[r] != 0: some atlas still searches in round
                        // r >= 1 (set by round r - 1's selection, cleared at the start)
  int32_t* tailF;       // [B][Wdmax] hybrid: the frontline at the t_opt switch
  int32_t* tail_t0;     // [B] hybrid: first chart of the tail (sorted), n when there is none
  int32_t* tail_kt;     // [B] hybrid: the tail's scale
  uint64_t* tail_obj;   // [B + 1][2] hybrid: sum over charts of area2 * scale (low, high
                        // word) per slot, then the charts' total area2 (from the plan)
  uint32_t* arena;      // profiles: per grown column (top, bottom), per grown row
                        // (left, right) of the local AABBs, then of the OBB, int16
                        // pairs (pack16)
};

// scale of slot s of the current round for an atlas (< 1: the slot does not
// run); round r covers scales k_top - koff - s, s < Br
__host__ __device__ inline int32_t slot_k(const Params& P, const AtlasDesc& d, int r, int s) {
  (void)r;
  if (P.fixed_k > 0) return s == 0 ? P.fixed_k : 0;
  return s < P.Br ? d.ktop - P.koff - s : 0;
}

// Round r >= 1 of a search in which every atlas finished in an earlier
// round: its kernels leave at once.
__device__ inline bool round_idle(const Work& w, int round) {
  return round > 0 && w.live[round] == 0;
}

// Launchers (one per kernel), all enqueue on `st`.
// cloop: charts of several boundary loops (chart c: loops [cloop[c],
// cloop[c+1]), voff then holds the loops' vertex offsets); nullptr: one loop
// per chart (voff: the charts' vertex offsets)
hipError_t launch_prep(const Params& P, const Work& w, const int32_t* xy, const int32_t* voff,
                       const int32_t* atlas_off, const int32_t* atlas_wh, int single_w,
                       int single_h, hipStream_t st, const int32_t* cloop = nullptr);
hipError_t launch_from_records(const Params& P, const Work& w, const Chart* in,
                               const int32_t* atlas_off, const int32_t* atlas_wh, hipStream_t st);
hipError_t launch_splice(Chart* dst, const int32_t* idx, int m, const Chart* src, hipStream_t st);
hipError_t launch_sort(const Params& P, const Work& w, hipStream_t st);
hipError_t launch_setup(const Params& P, const Work& w, int round, hipStream_t st);
// records of a serving batch (N charts of `count` requests, M of them freshly
// prepared): resident or prepared records into `out` and each request's new
// resident block, then the re-packs' replaced charts
hipError_t launch_assemble(int N, int M, int count, const int32_t* aoff, const int32_t* poff,
                           const uint64_t* src_res, const uint64_t* dst_res, const int32_t* idx,
                           const Chart* prep, Chart* out, hipStream_t st);
// pre-rotation of n single-loop charts to their tight boxes (64 directions):
// turned vertices into out (may be xy itself), each chart's direction into dir
hipError_t launch_prerotate(const int32_t* xy, const int32_t* voff, int n, int32_t* out,
                            uint8_t* dir, hipStream_t st);
// per-texel profiles and neighbour pairs (compacting distance, interlock flags)
hipError_t launch_profiles(const Params& P, const Work& w, int round, hipStream_t st);
// fold-and-push of the round's scales; for a single atlas its last workgroup
// also selects the scale and writes the outputs (not for a fixed diagnostic
// scale), batches select in launch_select (a no-op for a single atlas)
hipError_t launch_pack(const Params& P, const Work& w, int round, int lds_bytes, int RC, int PW,
                       int stage_cap, int last_round, int32_t* out_xy, uint8_t* out_orient,
                       float* out_scale, hipStream_t st);
hipError_t launch_select(const Params& P, const Work& w, int round, int last_round,
                         int32_t* out_xy, uint8_t* out_orient, float* out_scale, hipStream_t st);
// hybrid tail of every slot that reached the t_opt switch (single atlas,
// after launch_pack), then the choice of the scale by the area-weighted
// final scale and the outputs, with each chart's own scale in out_ks
hipError_t launch_tail(const Params& P, const Work& w, int lds_bytes, int RC, int PW,
                       hipStream_t st);
hipError_t launch_select_hybrid(const Params& P, const Work& w, int32_t* out_xy,
                                uint8_t* out_orient, float* out_ks, float* out_scale,
                                hipStream_t st);

hipError_t launch_scatter(const Params& P, const Work& w, int32_t* out_xy, uint8_t* out_orient,
                          int32_t* feasible, int32_t* rows, hipStream_t st);

// the diagnostic build's per-slot phase clock of the last single pack
// (slots x 11 values); -2 when the library was built without it
int read_phase_clock(int64_t* out, int slots);

hipError_t pack_set_max_lds(int bytes);
int pack_static_lds();

// shared-memory plan of the packing kernel: RC charts per row at most, a
// per-row pool of PW 32-bit words (offsets of every configuration, then the
// staged texel bounds and the texel -> chart map when they fit; its top also
// holds the second set of fold offsets, into which the next row is folded
// while the current one commits, for rows of at most (PW - 2) / 6 charts)
struct PackLds {
  int RC, PW, bytes;
};
PackLds pack_lds_plan(int nmax, int Wd, int budget);

// Host runtime shared by the C ABI entry points (api.cpp) and the serving
// context (serve.cpp).  Return TABI_* codes.
// bytes of work space a batched call of this shape takes
int64_t host_many_workspace_bytes(int count, int N, int nmax, int max_side, int p, int q);
// the batched pack from proxy records, on a caller work space
int host_pack_many_records_ws(const Chart* recs, const int32_t* aoff, int count,
                              const int32_t* awh, int N, int nmax, int max_side, int p, int q,
                              int32_t* out_xy, uint8_t* out_orient, float* out_scale, void* ws,
                              size_t ws_bytes, hipStream_t st);
// proxy records of M charts in `groups` groups (group g: charts
// [goff[g], goff[g+1]); a record's input index is its position in its group)
// with caller scratch of host_prep_scratch_bytes(M)
size_t host_prep_scratch_bytes(int M);
int host_prep_records(const int32_t* xy, const int32_t* voff, const int32_t* goff, int groups,
                      int M, int q, Chart* recs, void* scratch, hipStream_t st);
// record the HIP error text of a failed call; returns TABI_EHIP
int host_hip_fail(hipError_t e);

}  // namespace tabi
