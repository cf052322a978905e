// Fold-and-push at one candidate scale per workgroup (Alg. 3), and the scale
// selection.
//
// One workgroup (16 or 8 wavefronts) owns one (atlas, scale) pair and walks
// its rows in order.  The committed frontline lives in LDS.  Per row:
//   1. knee update (Alg. 4)            block max/min over the knee span
//   2. folding (Alg. 2)                wavefront prefix sums of chart advances,
//                                      first overflow by ballot; folds with
//                                      and without compaction and at full and
//                                      knee width come from the same two scans
//   3. staging                         the candidates' stored grown
//                                      TopEdge/BottomEdge (one contiguous range
//                                      of the profile arena) into LDS with a
//                                      texel -> chart map; rows that do not fit
//                                      read the arena directly, and charts
//                                      without stored profiles are evaluated
//                                      from their proxy records
//   4. push                            every texel of every configuration:
//                                      frontline - TopEdge, segmented max per
//                                      chart across the wavefront (DPP lane
//                                      moves), one LDS atomic per chart run
//   5. correction (Alg. 1)             per configuration one wavefront: forward
//                                      and backward segmented max scans over the
//                                      interlock chain, plus the rare pairs that
//                                      share columns without being neighbours
//   6. scores                          max over texels of offset + BottomEdge;
//                                      no private frontline copy is needed since
//                                      max(F, updates) = max(max F, max updates)
//   7. selection (Sec. 4.2 "Placing Rows") and commit, knee detection.
// All threads keep the per-row scalars in registers and compute them
// identically from LDS, so only data arrays and reductions cross threads.
#include "tabi_internal.h"
#include "pairs_dev.h"

namespace tabi {

// pairs per row that share columns without being neighbours, held in shared
// memory at once; a row with more walks them in chunks of this size
constexpr int LRCAP = 256;
constexpr int FWIN = 1024;  // charts per row whose fold data is staged in LDS
// single-configuration rows of at least this many charts are corrected by the
// whole workgroup
constexpr int LONG_ROW = 192;

// Diagnostic build (TABI_PHASE_CLOCK): the fold-and-push kernel of a single
// pack sums, per scale slot, the constant 100 MHz clock between the phases
// of its rows as wavefront 0 sees them (loop head, knee update, fold,
// configurations and staging, push, correction and score, selection,
// commit), with the slot's rows, scale and outcome; read back by
// tabi_debug_phase_clock.  The product build has none of it.
#ifdef TABI_PHASE_CLOCK
__device__ long long g_phase_clock[64][11];
#define PHASE_CLOCK_DECL long long ph_acc[8] = {0, 0, 0, 0, 0, 0, 0, 0}, ph_t = wall_clock64();
#define PHASE_CLOCK(q)                       \
  do {                                       \
    const long long ph_n = wall_clock64();   \
    ph_acc[q] += ph_n - ph_t;                \
    ph_t = ph_n;                             \
  } while (0)
// rows whose non-neighbour pairs overflow the shared list (x 2^32) + pairs
#define PHASE_PAIRS(over, pairs) (ph_acc[7] += ((long long)(over) << 32) + (long long)(pairs))
#else
#define PHASE_PAIRS(over, pairs) ((void)0)
#define PHASE_CLOCK_DECL
#define PHASE_CLOCK(q) \
  do {                 \
  } while (0)
#endif
enum { DIR_LR = 0, DIR_RL = 1 };

// A value every thread of the workgroup holds alike (read from shared
// memory after a barrier): kept in a scalar register.
__device__ inline int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// largest t in [0, cand) with Xoff[t] <= e
__device__ inline int find_chart(const int32_t* Xoff, int cand, int e) {
  int lo = 0, hi = cand - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (Xoff[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Segmented prefix max over the runs of a wavefront that start at `head`
// lanes, continuing `carry` into the lanes before the first head: the run
// start (a max-scan of head lanes) is a non-decreasing key for seg_scan_max.
__device__ inline int32_t run_scan_max(int32_t v, bool head, int32_t carry) {
  const int32_t key = wave_incl_max(head ? lane_id() : -1);
  v = seg_scan_max(v, key, seg_keys(key));
  return key < 0 ? max(v, carry) : v;
}

// CorrectYOffsets (Alg. 1) for one configuration, one wavefront.  Chain links
// come from the neighbour flags; fl[t] holds the flags of (t-1, t).
// chain_scans closes the chain constraints (a forward and a backward
// segmented max scan); apply_pairs applies those of non-neighbour pairs
// lr[0..lrn) once and reports whether any offset moved.
__device__ void chain_scans(int32_t* y, int cnt, const uint8_t* fl) {
  const int lane = lane_id();
  int32_t carry = -BIG;
  for (int t0 = 0; t0 < cnt; t0 += WAVE) {  // y[t] >= y[t-1] where bit0 of fl[t]
    const int t = t0 + lane;
    int32_t v = t < cnt ? y[t] : -BIG;
    const bool head = !(t >= 1 && t < cnt && (fl[t] & 1));
    v = run_scan_max(v, head, carry);
    if (t < cnt) y[t] = v;
    carry = lane63(v);
  }
  wsync();
  carry = -BIG;
  for (int r0 = 0; r0 < cnt; r0 += WAVE) {  // y[t] >= y[t+1] where bit1 of fl[t+1]
    const int r = r0 + lane, t = cnt - 1 - r;
    int32_t v = r < cnt ? y[t] : -BIG;
    const bool head = !(r >= 1 && r < cnt && (fl[t + 1] & 2));
    v = run_scan_max(v, head, carry);
    if (r < cnt) y[t] = v;
    carry = lane63(v);
  }
  wsync();
}
__device__ bool apply_pairs(int32_t* y, int cnt, const int32_t (*lr)[3], int lrn) {
  const int lane = lane_id();
  int changed = 0;
  for (int q0 = 0; q0 < lrn; q0 += WAVE) {
    const int q = q0 + lane;
    if (q < lrn) {
      const int A = lr[q][0], C = lr[q][1], f = lr[q][2];
      if (C < cnt) {
        const int32_t ya = y[A], yc = y[C];
        if ((f & 1) && yc < ya) { atomicMax(&y[C], ya); changed = 1; }
        if ((f & 2) && ya < yc) { atomicMax(&y[A], yc); changed = 1; }
      }
    }
  }
  const bool any = ballot64(changed) != 0;
  wsync();
  return any;
}
__device__ void correct_offsets(int32_t* y, int cnt, const uint8_t* fl, const int32_t (*lr)[3],
                                int lrn) {
  do {
    chain_scans(y, cnt, fl);
  } while (apply_pairs(y, cnt, lr, lrn));
}

// chain_scans by the whole workgroup, for a long row of a single
// configuration: 64 charts per wavefront, each wavefront's segmented scan
// continued by the carry of the wavefronts before it (a wavefront that holds
// a chain head passes on its last value, one without passes on the larger of
// the carry and its last value), the same results as one wavefront walking
// the chunks in order.  red: 2 * PACK_NT / WAVE ints.
template <int PACK_NT>
__device__ void chain_scans_block(int32_t* y, int cnt, const uint8_t* fl, int32_t* red) {
  constexpr int WAVES = PACK_NT / WAVE;
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {  // forward: y[t] >= y[t-1] where bit0 of fl[t];
    int32_t carry = -BIG;             // backward: y[t] >= y[t+1] where bit1 of fl[t+1]
    for (int b0 = 0; b0 < cnt; b0 += PACK_NT) {
      const int r = b0 + (int)threadIdx.x, t = dir == 0 ? r : cnt - 1 - r;
      int32_t v = r < cnt ? y[t] : -BIG;
      const bool head = !(r >= 1 && r < cnt && (dir == 0 ? (fl[t] & 1) : (fl[t + 1] & 2)));
      const int32_t key = wave_incl_max(head ? lane : -1);
      v = seg_scan_max(v, key, seg_keys(key));
      const bool hh = ballot64(head) != 0;
      const int32_t last = lane63(v);
      if (lane == 0) {
        red[2 * wv] = hh;
        red[2 * wv + 1] = last;
      }
      __syncthreads();
      int32_t c = carry, cn = carry;
      for (int q = 0; q < WAVES; ++q) {
        const int32_t h = red[2 * q], l = red[2 * q + 1];
        if (q == wv) c = cn;
        cn = h ? l : max(cn, l);
      }
      if (key < 0) v = max(v, c);
      if (r < cnt) y[t] = v;
      carry = cn;
      __syncthreads();  // red is written again by the next chunk or pass
    }
  }
}
// correct_offsets by the whole workgroup (same results): the block's chain
// scans, wavefront 0 applying the non-neighbour pairs, until no offset moves
template <int PACK_NT>
__device__ __attribute__((noinline)) void correct_offsets_block(int32_t* y, int cnt, const uint8_t* fl,
                                      const int32_t (*lr)[3], int lrn, int32_t* red) {
  for (;;) {
    chain_scans_block<PACK_NT>(y, cnt, fl, red);
    int moved = 0;
    if (threadIdx.x < WAVE) moved = apply_pairs(y, cnt, lr, lrn);
    if (!__syncthreads_or(moved)) break;
  }
}

// Non-neighbour partners of each candidate A of a compacted row: the charts
// C >= A + 2 whose offset lies within A's grown width (offsets increase, so
// they are consecutive).  Writes the exclusive prefix of their counts to
// pre[0..cand) and returns the total (whole workgroup; red: PACK_WAVES ints).
template <int PACK_NT>
__device__ int pair_prefix(const int32_t* Xon, const int32_t* Xoff, int cand, int32_t* pre,
                           int32_t* red) {
  constexpr int PACK_WAVES = PACK_NT / WAVE;
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  auto count = [&](int A) {
    const int lim = Xon[A] + (Xoff[A + 1] - Xoff[A]);
    int lo = A + 2, hi = cand;  // first C >= A + 2 with Xon[C] >= lim
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Xon[mid] < lim) lo = mid + 1; else hi = mid;
    }
    return max(0, lo - (A + 2));
  };
  const int per = (cand + PACK_NT - 1) / PACK_NT;
  const int a0 = min(cand, tid * per), a1 = min(cand, a0 + per);
  int sum = 0;
  for (int A = a0; A < a1; ++A) sum += count(A);
  const int incl = wave_incl_sum(sum);
  __syncthreads();
  if (lane == WAVE - 1) red[wv] = incl;
  __syncthreads();
  int base = 0, total = 0;
  for (int i = 0; i < PACK_WAVES; ++i) {
    if (i < wv) base += red[i];
    total += red[i];
  }
  int run = base + incl - sum;
  for (int A = a0; A < a1; ++A) {
    pre[A] = run;
    run += count(A);
  }
  __syncthreads();  // pre[] written by every thread before it is searched
  return total;
}

// The correction of a row whose pairs that share columns without being
// neighbours outnumber the shared-memory list (rare; every thread of the
// workgroup calls it).  Their flags depend only on the compacted offsets,
// the same in every configuration; each pass recomputes them chunk by chunk
// and applies them, until a whole pass moves no offset.  Kept out of line so
// that its registers do not add to those of the row loop.  lrpre, flv,
// prowv, hdv: the slot's per-chart arrays of the atlas; seg: the profile
// segment (stored rows) when prof.
template <int PACK_NT>
__device__ __attribute__((noinline)) void correct_many_pairs(
    const int32_t* Xon, const int32_t* Xoff, int cand, int rs, int32_t* lrpre, int32_t* red,
    int32_t (*lr)[3], int32_t* my_y, int my_cnt, int my_hc, const uint8_t* flv, bool prof,
    const uint32_t* seg, const int32_t* prowv, const int32_t* hdv, const unsigned char* kcb,
    int stride, const Chart* ch, int K, int k, int p) {
  constexpr int PACK_WAVES = PACK_NT / WAVE;
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  auto KV = [&](int c) { return kview(kcb + (size_t)c * stride, K); };
  const int total = pair_prefix<PACK_NT>(Xon, Xoff, cand, lrpre + rs, red);
  for (;;) {
    if (my_hc) chain_scans(my_y, my_cnt, flv + rs);
    int moved = 0;
    for (int q0 = 0; q0 < total; q0 += LRCAP) {
      const int m = min(LRCAP, total - q0);
      __syncthreads();  // the previous chunk is no longer read
      for (int t = tid; t < m; t += PACK_NT) {
        const int q = q0 + t;
        int lo = 0, hi = cand - 1;  // last A with pre[A] <= q
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (lrpre[rs + mid] <= q) lo = mid; else hi = mid - 1;
        }
        lr[t][0] = lo;
        lr[t][1] = lo + 2 + (q - lrpre[rs + lo]);
      }
      __syncthreads();
      for (int q = wv; q < m; q += PACK_WAVES) {
        const int A = lr[q][0], C = lr[q][1];
        const int wdA = Xoff[A + 1] - Xoff[A];
        const int dd = Xon[C] - Xon[A];
        int f;
        if (prof) {
          f = pair_flags_at(pair_rows_meet(seg + prowv[rs + A], hdv[rs + A], seg + prowv[rs + C],
                                           hdv[rs + C], wdA),
                            wdA, dd);
        } else {
          f = pair_flags_at(pair_records_sweep<2>(KV(rs + A), ch[rs + A], KV(rs + C), ch[rs + C],
                                                  K, k, p),
                            wdA, dd);
        }
        if (lane == 0) lr[q][2] = f;
      }
      __syncthreads();
      if (my_hc && apply_pairs(my_y, my_cnt, lr, m)) moved = 1;
    }
    if (!__syncthreads_or(moved)) break;
  }
}

// The hybrid tail's hand-over: the frontline and the tail's first chart
// (kept out of line, off the row loop's registers).
template <int PACK_NT>
__device__ __attribute__((noinline)) void save_tail(const int32_t* F, int Wd, int32_t* dst,
                                                    int32_t* t0, int rs) {
  for (int x = threadIdx.x; x < Wd; x += PACK_NT) dst[x] = F[x];
  if (threadIdx.x == 0) *t0 = rs;
}

template <int PACK_WAVES>
__device__ inline int32_t block_reduce_max(int32_t v, int32_t* red) {
  v = wave_max(v);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  int32_t r = red[0];
#pragma unroll
  for (int i = 1; i < PACK_WAVES; ++i) r = max(r, red[i]);
  return uni(r);
}
template <int PACK_WAVES>
__device__ inline int32_t block_reduce_min(int32_t v, int32_t* red) {
  v = wave_min(v);
  __syncthreads();
  if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  int32_t r = red[0];
#pragma unroll
  for (int i = 1; i < PACK_WAVES; ++i) r = min(r, red[i]);
  return uni(r);
}

// Largest feasible scale of this round for atlas a (one workgroup, any size
// of at least one wavefront); outputs in input order.  sh: 3 ints of shared
// memory.
__device__ void select_atlas(const Params& P, const Work& w, int round, int last_round, int a,
                             int32_t* out_xy, uint8_t* out_orient, float* out_scale, int32_t* sh) {
  const AtlasDesc d = w.desc[a];
  if (d.done) return;
  if (threadIdx.x < WAVE) {  // lane s reads slot s (at most 64 slots)
    const bool live = !d.bad && d.n > 0 && d.ktop >= 1;
    const int s = threadIdx.x;
    const int f = live && s < P.Br ? w.feas[a * P.B + s] : 0;
    const uint64_t ok = ballot64(f == 1);
    const int best = ok ? __builtin_ctzll(ok) : -1;
    const int limit = ballot64(f == -2) != 0;
    if (threadIdx.x == 0) {
      sh[0] = best;
      sh[1] = limit;
      // more candidate scales remain for a later round
      sh[2] = live && best < 0 && !limit && !last_round && slot_k(P, d, round, P.Br - 1) > 1;
    }
  }
  __syncthreads();
  const int best = sh[0], limit = sh[1];
  if (sh[2]) {  // the atlas searches on: the next round runs
    if (threadIdx.x == 0 && round < MAX_ROUNDS) w.live[round + 1] = 1;
    return;
  }
  float scale;
  int kstar = 0;
  if (d.bad) scale = -1.0f;
  else if (d.n == 0) { scale = 1.0f; kstar = 64; }
  else if (limit) scale = -2.0f;
  else if (best >= 0) { kstar = slot_k(P, d, round, best); scale = (float)kstar / 64.0f; }
  else scale = 0.0f;
  const size_t slot = (size_t)(best >= 0 ? best : 0) * P.N;
  const bool placed = kstar > 0 && best >= 0;
  // four charts per thread at a time: all their loads are issued before any
  // of their stores (a store may alias a later load as far as the compiler
  // knows, so a chart at a time would wait for its loads once per chart)
  constexpr int U = 4;
  for (int t0 = threadIdx.x; t0 < d.n; t0 += U * (int)blockDim.x) {
    int dst[U];
    int32_t x[U], y[U];
    uint8_t o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      dst[u] = -1;
      x[u] = -1;
      y[u] = -1;
      o[u] = 0;
      if (t < d.n) {
        const int c = d.c0 + t;
        dst[u] = d.c0 + w.perm[c];
        if (placed) {
          x[u] = w.xs[slot + c];
          y[u] = w.ys[slot + c];
          o[u] = (uint8_t)(w.srecs[c].bits | (w.mir[slot + c] << 3));
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (dst[u] < 0) continue;
      out_xy[2 * (size_t)dst[u]] = x[u];
      out_xy[2 * (size_t)dst[u] + 1] = y[u];
      out_orient[dst[u]] = o[u];
    }
  }
  if (threadIdx.x == 0) {
    out_scale[a] = scale;
    w.desc[a].done = 1;
    w.desc[a].kstar = kstar;
  }
}

// PACK_NT threads per workgroup: 1024 for a single pack (every per-texel
// phase of a row spread over 16 wavefronts), 512 for batches (two workgroups
// per CU when their shared memory allows it).  At most 128 VGPRs either way.
// HYB: the hybrid tail's variant (a single atlas), which hands the rows
// after the t_opt switch over to k_tail.
template <int PACK_NT, bool HYB = false>
__global__ __launch_bounds__(PACK_NT) __attribute__((amdgpu_waves_per_eu(4))) void k_pack(
    Params P, Work w, int round, int RC, int PW, int stage_cap, int last_round, int32_t* out_xy,
    uint8_t* out_orient, float* out_scale) {
  constexpr int PACK_WAVES = PACK_NT / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_cnt[4];
  __shared__ int32_t s_red[PACK_WAVES * 6];
  __shared__ int32_t s_knee[4];  // knee found by the last row's detection: on, direction, span
  __shared__ uint32_t s_touch;   // keeps the next row's cache warm-up loads (never read)
  __shared__ int32_t s_lrn, s_lrover;
  __shared__ int32_t s_lr[LRCAP][3];
  // window of chart data read by the fold, the knee test and the chain
  // scans, charts [wb, wb + nwin): grown width, compacting distance to the
  // next chart, unscaled height, interlock flags with the previous chart; it
  // slides when fewer than FWIN / 2 charts remain ahead
  __shared__ int32_t s_wd[FWIN], s_cdn[FWIN], s_H[FWIN];
  __shared__ uint8_t s_fl[FWIN];  // interlock flags of (c-1, c), read by the chain scans

  if (round_idle(w, round)) return;
  const int s = blockIdx.x, a = w.aord[blockIdx.y];
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
  const AtlasDesc d = w.desc[a];
  const int k = slot_k(P, d, round, s);
  const bool run = P.fixed_k > 0 ? (k >= 1 && !d.bad) : (!d.done && d.ktop >= 1 && k >= 1);
  // outcome of this (atlas, scale): 1 feasible, 0 not, -1 not run, -2 the
  // atlas exceeds the shape the call was sized for; rows placed
  int feasible = -1, rows = 0;
  do {  // every workgroup reaches the epilogue below
  if (!run) break;
  const int n = d.n, Wd = d.Wa + P.p, Hd = d.Ha + P.p, Ha = d.Ha, p = P.p, K = P.K;
  if (n > P.nmax || Wd > P.Wdmax) {  // batch larger than the caller's declared shape
    feasible = -2;
    break;
  }
  // t_opt (Sec. 4.4): the call's setting, or the paper's per atlas
  const int topt = P.topt >= 0 ? P.topt : (n > 10000 ? 1 : 0);
  const size_t slot = (size_t)s * P.N + d.c0;
  // dynamic LDS: frontline F[Wd], fold offsets without / with compaction
  // Xoff, Xon[RC+1], then a per-row pool of PW words.  A second pair of
  // offset arrays for rows of up to RA charts sits at the top of the pool,
  // RA the most for which the rest of the pool still holds four
  // configurations' offsets: the next row is folded into the other pair
  // while this row commits (rows of more charts are folded again, into the
  // first pair, after the opening barrier)
  int32_t* const F = reinterpret_cast<int32_t*>(smem);
  int32_t* const X0 = F + Wd;
  int32_t* const pool = X0 + 2 * (RC + 1);
  const int RA = min(RC, (PW - 2) / 6);
  const int PWr = PW - 2 * (RA + 1);  // the pool below the second pair
  int32_t* const X1 = pool + PWr;
  int32_t* Xoff = X0;  // this row's offsets: (X0, X0 + RC + 1) or (X1, X1 + RA + 1)
  int32_t* Xon = X0 + (RC + 1);
  const unsigned char* kcb = w.kc + slot * P.stride;
  const Chart* ch = w.srecs + d.c0;
  const int32_t* cdv = w.cd + slot;
  const uint8_t* flv = w.fl + slot;
  const int32_t* wdv = w.wdv + slot;
  const int32_t* hdv = w.hdv + slot;
  const int32_t* prowv = w.prow + slot;
  int32_t* lrpre = w.lrpre + slot;
  const int32_t sbase = w.segbase[(size_t)a * P.B + s];  // -1: profiles not stored
  const int32_t* Hs = w.Hs + d.c0;
  int32_t* xs = w.xs + slot;
  int32_t* ys = w.ys + slot;
  uint8_t* mir = w.mir + slot;
  auto KV = [&](int c) { return kview(kcb + (size_t)c * P.stride, K); };

  for (int x = tid; x < Wd; x += PACK_NT) F[x] = 0;
  for (int t = tid; t < n; t += PACK_NT) { xs[t] = -1; ys[t] = -1; mir[t] = 0; }

  // per-row state, identical in every thread; the tight-only variant folds
  // every row like a tail row (Sec. 5 ablations)
  int rs = 0, tail = P.variant == 1, trow = 0;
  feasible = 1;
  int kn = 0, kdir = 0, kl = 0, kr = 0;
  if (tid == 0) s_knee[0] = -1;
  int32_t fmax = 0;
  int wb = -FWIN, nwin = 0;
  // arena word of the row's first grown column (-1: no stored profiles); the
  // charts of a segment are stored back to back, so it advances by the
  // committed grown width
  int32_t pc0 = n > 0 ? sbase : -1;
  // end of the segment's column area (its rows follow): the cache warm-up
  // loads for the next row never read past it
  const int32_t colend = pc0 >= 0 ? sbase + prowv[0] : 0;

  // ---- folding (Alg. 2), by one wavefront: the row from chart rs_f (window
  // index r0_f), offsets without / with compaction into xo_b / xn_b; the
  // counts that fit the full width and, for a knee fold, width kw_f go to
  // s_cnt, and the row's pair list is cleared
  auto fold = [&](int rs_f, int r0_f, int32_t* xo_b, int32_t* xn_b, int cap, int kw_f) {
    int cfo = -1, cfn = -1, cko = -1, ckn = -1;
    int xo = 0, xn = 0;
    for (int t0 = 0; cfn < 0; t0 += WAVE) {
      const int t = t0 + lane, c = rs_f + t;
      int wd = Wd + 1, cdn = 0;
      if (r0_f + t < nwin) {
        wd = s_wd[r0_f + t];
        cdn = s_cdn[r0_f + t];
      } else if (c < n) {
        wd = wdv[c];
        if (c + 1 < n) cdn = cdv[c + 1];
      }
      const int ao = wd, an = wd - cdn;
      const int io = wave_incl_sum(ao), in = wave_incl_sum(an);
      const int Xo = xo + io - ao, Xn = xn + in - an;
      if (t <= cap) { xo_b[t] = Xo; xn_b[t] = Xn; }
      const uint64_t bfo = ballot64(Xo + wd > Wd), bfn = ballot64(Xn + wd > Wd);
      const uint64_t bko = ballot64(Xo + wd > kw_f), bkn = ballot64(Xn + wd > kw_f);
      if (cfo < 0 && bfo) cfo = t0 + __builtin_ctzll(bfo);
      if (cfn < 0 && bfn) cfn = t0 + __builtin_ctzll(bfn);
      if (cko < 0 && bko) cko = t0 + __builtin_ctzll(bko);
      if (ckn < 0 && bkn) ckn = t0 + __builtin_ctzll(bkn);
      xo += lane63(io);
      xn += lane63(in);
    }
    if (lane == 0) {
      s_cnt[0] = cfo; s_cnt[1] = cfn; s_cnt[2] = cko; s_cnt[3] = ckn;
      s_lrn = 0; s_lrover = 0;
    }
  };
  // the knee counts of a row folded ahead, from its offsets: chart t's grown
  // width is Xoff[t + 1] - Xoff[t] (stored up to the full-width count cfn),
  // and a knee count never exceeds the full-width one
  auto knee_counts = [&](int kw_f) {
    const int cfo = uni(s_cnt[0]), cfn = uni(s_cnt[1]);
    int cko = -1, ckn = -1;
    if (cfn >= 1 && cfn <= RC) {
      for (int t0 = 0; ckn < 0; t0 += WAVE) {
        const int t = t0 + lane;
        bool po = t >= cfo, pn = t >= cfn;
        if (t < cfn) {
          const int x0 = Xoff[t], wd = Xoff[t + 1] - x0;
          po = po || x0 + wd > kw_f;
          pn = Xon[t] + wd > kw_f;
        }
        const uint64_t bo = ballot64(po), bn = ballot64(pn);
        if (cko < 0 && bo) cko = t0 + __builtin_ctzll(bo);
        if (ckn < 0 && bn) ckn = t0 + __builtin_ctzll(bn);
      }
    }
    if (lane == 0) { s_cnt[2] = cko; s_cnt[3] = ckn; }
  };
  // 1: the next row is being folded while this row commits; then, after the
  // opening barrier, 1 if it fitted the other pair
  int ahead = 0, pre = 0;

  PHASE_CLOCK_DECL
  for (;;) {
    __syncthreads();
    {  // the previous row's knee detection (-1: none ran)
      const int kf = uni(s_knee[0]);
      if (kf >= 0) kn = kf;
      if (kf > 0) { kdir = uni(s_knee[1]); kl = uni(s_knee[2]); kr = uni(s_knee[3]); }
    }
    if (rs >= n) break;
    pre = 0;
    if (ahead) {  // the row folded ahead: into the other pair if it fitted
      pre = uni(s_cnt[1]) <= RA;
      if (pre && Xoff == X0) { Xoff = X1; Xon = X1 + (RA + 1); }
      else { Xoff = X0; Xon = X0 + (RC + 1); }
    }
    if (rs - wb > FWIN / 2) {
      wb = rs;
      nwin = min(FWIN, n - wb);
      for (int t = tid; t < nwin; t += PACK_NT) {
        const int c = wb + t;
        s_wd[t] = wdv[c];
        s_cdn[t] = c + 1 < n ? cdv[c + 1] : 0;
        s_H[t] = Hs[c];
        s_fl[t] = flv[c];
      }
      __syncthreads();
    }
    const int r0 = rs - wb;  // window index of the row's first chart
    PHASE_CLOCK(0);
    // ---- 1. knee location update (Alg. 4)
    if (kn) {
      const int probe = kdir == DIR_LR ? kr : kl - 1;
      if (probe < 0 || probe >= Wd) {
        kn = 0;
      } else {
        const int32_t h0 = F[probe];
        if (kdir == DIR_LR) {
          int32_t best = kl - 1;
          for (int x = kl + tid; x < kr; x += PACK_NT) if (F[x] >= h0) best = max(best, x);
          best = block_reduce_max<PACK_WAVES>(best, s_red);
          kr = best + 1;
        } else {
          int32_t best = kr;
          for (int x = kl + tid; x < kr; x += PACK_NT) if (F[x] >= h0) best = min(best, x);
          best = block_reduce_min<PACK_WAVES>(best, s_red);
          kl = best;
        }
      }
    }
    PHASE_CLOCK(1);
    // ---- t_opt switch (Sec. 4.4), on the first chart's texel height
    const int64_t h0 = cdiv64((int64_t)k * uni(s_H[r0]), QS);
    if (!tail && !kn && 100 * h0 < (int64_t)topt * Ha) {
      tail = 1;
      if (HYB) {  // the rest is folded by prefix sums (k_tail)
        save_tail<PACK_NT>(F, Wd, w.tailF + (size_t)s * P.Wdmax, w.tail_t0 + s, rs);
        feasible = 2;
        break;
      }
    }
    // ---- 2. folding (Alg. 2), wavefront 0
    const bool prof = pc0 >= 0;  // stored profiles: texel e of the row is word pc0 + e
    const uint32_t* gprof = w.arena + (prof ? pc0 : 0);
    uint32_t* st = reinterpret_cast<uint32_t*>(pool);
    const int kw = kn ? (kdir == DIR_LR ? Wd - kr : kl) : 0;
    if (!pre) {
      if (wv == 0) fold(rs, r0, Xoff, Xon, RC, kw);
      __syncthreads();
    } else if (kn) {
      if (wv == 0) knee_counts(kw);
      __syncthreads();
    }
    PHASE_CLOCK(2);
    const int cfo = uni(s_cnt[0]), cfn = uni(s_cnt[1]), cko = uni(s_cnt[2]), ckn = uni(s_cnt[3]);
    if (cfn == 0) { feasible = 0; break; }  // a chart wider than the atlas
    if (cfn > RC) { feasible = -2; break; }   // cannot happen: advances are >= 1
    // ---- configurations: direction x compaction x (full | knee) (Sec. 4.2)
    int ncfg, c_cnt[4], c_hc[4], c_dir[4], c_R0[4], c_R1[4];
    if (tail) {
      ncfg = 1;
      c_cnt[0] = cfn; c_hc[0] = 1; c_dir[0] = (trow % 3 == 0) ? DIR_LR : DIR_RL;
      c_R0[0] = 0; c_R1[0] = Wd;
      ++trow;
    } else {
      const int hc = cfn > cfo, cnt = hc ? cfn : cfo;
      ncfg = 2;
      c_cnt[0] = c_cnt[1] = cnt; c_hc[0] = c_hc[1] = hc;
      c_dir[0] = DIR_LR; c_dir[1] = DIR_RL;
      c_R0[0] = c_R0[1] = 0; c_R1[0] = c_R1[1] = Wd;
      if (kn && ckn > 0) {
        const int khc = ckn > cko, kc = khc ? ckn : cko;
        ncfg = 4;
        c_cnt[2] = c_cnt[3] = kc; c_hc[2] = c_hc[3] = khc;
        c_dir[2] = DIR_LR; c_dir[3] = DIR_RL;
        c_R0[2] = c_R0[3] = kdir == DIR_LR ? kr : 0;
        c_R1[2] = c_R1[3] = kdir == DIR_LR ? Wd : kl;
      }
    }
    for (int j = ncfg; j < 4; ++j) { c_cnt[j] = 0; c_hc[j] = 0; c_dir[j] = 0; c_R0[j] = 0; c_R1[j] = 0; }
    // every configuration takes a prefix of the cfn candidates
    const int cand = cfn;
    int anyhc = 0, yofs[4], ysum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) { anyhc |= c_hc[j]; yofs[j] = ysum; ysum += c_cnt[j]; }
    const int E = uni(Xoff[cand]);  // grown texel columns of the candidates
    // pool: (when staged) packed (top, bottom) of texel e at st[e] and its
    // chart at emap[e]; offsets Y of configuration j at the top of the pool
    // (the pool's top holds the other pair while the next row is folded,
    // which happens for rows of at most RA charts)
    ahead = cand <= RA;
    int32_t* Yb = pool + (ahead ? PWr : PW) - ysum;
    int16_t* emap = reinterpret_cast<int16_t*>(pool + E);
    const bool staged = prof && E <= stage_cap && ysum + E + (E + 1) / 2 <= (ahead ? PWr : PW);
    // grown top (tp) / bottom (bt) of texel e and its chart t in the row
    auto texel = [&](int e, int& t, int32_t& tp, int32_t& bt) {
      if (staged) {
        t = emap[e];
        const uint32_t v = st[e];
        tp = lo16(v);
        bt = hi16(v);
      } else {
        t = find_chart(Xoff, cand, e);
        if (prof) {
          const uint32_t v = gprof[e];
          tp = lo16(v);
          bt = hi16(v);
        } else {
          column_bounds_grown(KV(rs + t), ch[rs + t], K, k, p, e - Xoff[t], tp, bt);
        }
      }
    };
    // ---- 3. staging, offset init, non-neighbour pairs that share columns
    if (staged) {
      for (int e = tid; e < E; e += PACK_NT) st[e] = gprof[e];
      // texel -> chart map, filled chart by chart: a thread per chart when
      // charts are narrow, a wavefront per chart when they are wide
      if (E < 16 * cand) {
        for (int t = tid; t < cand; t += PACK_NT)
          for (int e = Xoff[t]; e < Xoff[t + 1]; ++e) emap[e] = (int16_t)t;
      } else {
        for (int t = wv; t < cand; t += PACK_WAVES)
          for (int e = Xoff[t] + lane; e < Xoff[t + 1]; e += WAVE) emap[e] = (int16_t)t;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      for (int t = tid; t < c_cnt[j]; t += PACK_NT) Yb[yofs[j] + t] = -BIG;
    if (anyhc) {
      for (int A = tid; A + 2 < cand; A += PACK_NT) {
        const int wdA = Xoff[A + 1] - Xoff[A];
        for (int C = A + 2; C < cand && Xon[C] - Xon[A] < wdA; ++C) {
          const int q = atomicAdd(&s_lrn, 1);
          if (q < LRCAP) { s_lr[q][0] = A; s_lr[q][1] = C; s_lr[q][2] = 0; }
          else s_lrover = 1;
        }
      }
    }
    __syncthreads();
    // more pairs than the shared list holds, or pairs whose rows are not
    // stored: none is swept with the push, the correction walks them out of
    // line (both rare)
    PHASE_CLOCK(3);
    const bool lrover = uni(s_lrover) != 0 || (!prof && uni(s_lrn) > 0);
    const int lrn = lrover ? 0 : uni(s_lrn);
    PHASE_PAIRS(lrover, uni(s_lrn));
    // ---- 4. push every configuration against the committed frontline; the
    // last wavefronts (at most a quarter) sweep the non-neighbour pairs at
    // the same time
    const int nlr = min(lrn, PACK_WAVES / 4), npush = PACK_WAVES - nlr;
    // bring the words after this row's range (where the next row's range
    // ends) into the caches while the push runs, so that the next row's
    // staging copy hits them; the sum is consumed only after the push
    uint32_t t0 = 0, t1 = 0, t2 = 0, t3 = 0;
    if (staged) {
      const int L = min(Wd + Wd / 2, colend - (pc0 + E));
      const uint32_t* g = gprof + E;
      if (tid < L) t0 = g[tid];
      if (tid + PACK_NT < L) t1 = g[tid + PACK_NT];
      if (tid + 2 * PACK_NT < L) t2 = g[tid + 2 * PACK_NT];
      if (tid + 3 * PACK_NT < L) t3 = g[tid + 3 * PACK_NT];
    }
    for (int e0 = wv * WAVE; wv < npush && e0 < E; e0 += npush * WAVE) {
      const int e = e0 + lane;
      const bool valid = e < E;
      int t = -1;
      int32_t tp = 0, bt = 0;
      if (valid) texel(e, t, tp, bt);
      const int i = valid ? e - Xoff[t] : 0;
      // chart t's texels are a run of lanes (t does not decrease along e):
      // a segmented prefix max leaves the chart's maximum in its last lane
      const SegKeys sk = seg_keys(t);
      const bool tail = valid && wave_shl1(t, -2) != t;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j >= ncfg) break;
        int32_t v = -BIG;
        if (valid && t < c_cnt[j]) {
          const int X = c_hc[j] ? Xon[t] : Xoff[t];
          const int col = c_dir[j] == DIR_LR ? c_R0[j] + X + i : c_R1[j] - 1 - X - i;
          v = F[col] - tp;
        }
        v = seg_scan_max(v, t, sk);
        if (tail && v > -BIG) atomicMax(&Yb[yofs[j] + t], v);
      }
    }
    if ((t0 ^ t1 ^ t2 ^ t3) == 0x9e3779b9u) s_touch = t0;
    // interlock flags of the non-neighbour pairs, read only by the correction
    for (int q = wv - npush; wv >= npush && q < lrn; q += nlr) {
      const int A = s_lr[q][0], C = s_lr[q][1];
      const int wdA = Xoff[A + 1] - Xoff[A];
      const int dd = Xon[C] - Xon[A];  // rows stored (prof): the others go out of line
      const int f = pair_flags_at(pair_rows_meet(w.arena + sbase + prowv[rs + A], hdv[rs + A],
                                                 w.arena + sbase + prowv[rs + C], hdv[rs + C],
                                                 wdA),
                                  wdA, dd);
      if (lane == 0) s_lr[q][2] = f;
    }
    __syncthreads();
    PHASE_CLOCK(4);
    // ---- 5. correction and score, one wavefront per configuration.  The
    // score is the largest offset + grown bottom over the configuration's
    // texels.  A chart's largest bottom is its height h: every proxy bounds
    // the chart from outside, so at a column holding the chart's lowest
    // point all of them reach h, and the local AABBs never pass it; grown,
    // the largest is h + p.  So a configuration scores max over its charts
    // of offset + h + p, one term per chart, taken by the wavefront that
    // corrected it; the other wavefronts take the frontline's maximum over
    // the knee region meanwhile.
    const int my_cnt = wv == 0 ? c_cnt[0] : wv == 1 ? c_cnt[1] : wv == 2 ? c_cnt[2] : c_cnt[3];
    const int my_hc = wv < ncfg && (wv == 0 ? c_hc[0] : wv == 1 ? c_hc[1] : wv == 2 ? c_hc[2] : c_hc[3]);
    int32_t* my_y = Yb + (wv == 0 ? yofs[0] : wv == 1 ? yofs[1] : wv == 2 ? yofs[2] : yofs[3]);
    if (lrover)
      correct_many_pairs<PACK_NT>(Xon, Xoff, cand, rs, lrpre, s_red, s_lr, my_y, my_cnt, my_hc,
                                  flv, prof, w.arena + (prof ? sbase : 0), prowv, hdv, kcb,
                                  P.stride, ch, K, k, p);
    // the chain's flags from the window when the row lies inside it (a long
    // row's scans then wait on no global load)
    const uint8_t* chain_fl = r0 + c_cnt[0] <= nwin ? s_fl + r0 : flv + rs;
    int32_t M[4] = {-BIG, -BIG, -BIG, -BIG}, fr = -BIG;
    if (ncfg == 1 && c_cnt[0] >= LONG_ROW) {
      // a long single-configuration row: the whole workgroup corrects and
      // scores it
      if (!lrover && c_hc[0]) correct_offsets_block<PACK_NT>(Yb, c_cnt[0], chain_fl, s_lr, lrn, s_red);
      int32_t m = -BIG;
      for (int t = tid; t < c_cnt[0]; t += PACK_NT) {
        const int64_t Hq = r0 + t < nwin ? s_H[r0 + t] : Hs[rs + t];
        m = max(m, Yb[t] + (int32_t)((k * Hq + QS - 1) >> 14) + p);
      }
      m = wave_max(m);
      if (lane == 0) s_red[2 * PACK_WAVES + wv] = m;
      __syncthreads();
      for (int q = 0; q < PACK_WAVES; ++q) M[0] = max(M[0], uni(s_red[2 * PACK_WAVES + q]));
      PHASE_CLOCK(5);
    } else {
      if (wv < 4) {
        if (!lrover && my_hc)
          correct_offsets(my_y, my_cnt, r0 + my_cnt <= nwin ? s_fl + r0 : flv + rs, s_lr, lrn);
        int32_t m = -BIG;
        if (wv < ncfg)
          for (int t = lane; t < my_cnt; t += WAVE) {
            const int64_t Hq = r0 + t < nwin ? s_H[r0 + t] : Hs[rs + t];
            m = max(m, my_y[t] + (int32_t)((k * Hq + QS - 1) >> 14) + p);
          }
        m = wave_max(m);
        if (lane == 0) s_red[wv] = m;
      } else if (ncfg == 4) {
        int32_t f = -BIG;
        for (int x = c_R0[2] + tid - 4 * WAVE; x < c_R1[2]; x += PACK_NT - 4 * WAVE) f = max(f, F[x]);
        f = wave_max(f);
        if (lane == 0) s_red[wv] = f;
      }
      __syncthreads();
      PHASE_CLOCK(5);
#pragma unroll
      for (int j = 0; j < 4; ++j) M[j] = uni(s_red[j]);
      if (ncfg == 4)
        for (int q = 4; q < PACK_WAVES; ++q) fr = max(fr, uni(s_red[q]));
    }
    // ---- 7. selection: lower maximal height wins, ties left to right; the
    // knee fold only if strictly lower over the whole frontline
    int win = 0, knee_used = 0;
    int32_t whole[4], region[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) { whole[j] = max(fmax, M[j]); region[j] = max(fr, M[j]); }
    if (!tail) {
      win = whole[1] < whole[0] ? 1 : 0;
      if (ncfg == 4) {
        const int kb = region[3] < region[2] ? 3 : 2;
        if (whole[kb] < whole[win]) { win = kb; knee_used = 1; }
      }
    }
    const int w_cnt = win == 0 ? c_cnt[0] : win == 1 ? c_cnt[1] : win == 2 ? c_cnt[2] : c_cnt[3];
    const int w_hc = win == 0 ? c_hc[0] : win == 1 ? c_hc[1] : win == 2 ? c_hc[2] : c_hc[3];
    const int w_dir = win == 0 ? c_dir[0] : win == 1 ? c_dir[1] : win == 2 ? c_dir[2] : c_dir[3];
    const int w_R0 = win == 0 ? c_R0[0] : win == 1 ? c_R0[1] : win == 2 ? c_R0[2] : c_R0[3];
    const int w_R1 = win == 0 ? c_R1[0] : win == 1 ? c_R1[1] : win == 2 ? c_R1[2] : c_R1[3];
    const int32_t w_score = win == 0 ? whole[0] : win == 1 ? whole[1] : win == 2 ? whole[2] : whole[3];
    const int32_t* Yw = Yb + (win == 0 ? yofs[0] : win == 1 ? yofs[1] : win == 2 ? yofs[2] : yofs[3]);
    // ---- commit: frontline update, placements.  No barrier before it: every
    // read of the frontline in this row (push, knee region maximum) happened
    // before the barrier of the score reduction, and the reduction slots and
    // offsets read since are next written after the loop's opening barrier.
    // (wavefronts 1.. commit while wavefront 0 runs the knee detection below;
    // with the second offset pair, wavefront 1 folds the next row into it
    // instead: its counts and pair list are read only after the next opening
    // barrier)
    const int cw = ahead ? 2 : 1;  // the first wavefront that commits
    if (ahead && wv == 1) {
      if (Xoff == X0) fold(rs + w_cnt, rs + w_cnt - wb, X1, X1 + (RA + 1), RA, 0);
      else fold(rs + w_cnt, rs + w_cnt - wb, X0, X0 + (RC + 1), RA, 0);
    }
    const int Ew = Xoff[w_cnt];
    for (int e = tid - cw * WAVE; wv >= cw && e < Ew; e += PACK_NT - cw * WAVE) {
      int t;
      int32_t tp, bt;
      texel(e, t, tp, bt);
      const int i = e - Xoff[t];
      const int X = w_hc ? Xon[t] : Xoff[t];
      const int col = w_dir == DIR_LR ? w_R0 + X + i : w_R1 - 1 - X - i;
      atomicMax(&F[col], Yw[t] + bt);
    }
    for (int t = tid - cw * WAVE; wv >= cw && t < w_cnt; t += PACK_NT - cw * WAVE) {
      const int X = w_hc ? Xon[t] : Xoff[t];
      const int wd = Xoff[t + 1] - Xoff[t];
      xs[rs + t] = w_dir == DIR_LR ? w_R0 + X : w_R1 - X - wd;
      ys[rs + t] = Yw[t];
      mir[rs + t] = (uint8_t)(w_dir == DIR_RL);
    }
    // knee detection on a row folded at full width (Sec. 4.2; App. A): the
    // largest drop in unscaled height between consecutive charts that is at
    // least 10% of the atlas height and 20% of the taller chart; first wins
    // (wavefront 0 alone; the others take the result from LDS after the
    // next row's opening barrier)
    if (wv == 0 && (tail || knee_used)) {
      if (lane == 0) s_knee[0] = -1;  // no detection: the knee state stays
    } else if (wv == 0) {
      int64_t best = -1;
      for (int t = lane; t + 1 < w_cnt; t += WAVE) {
        const int64_t h1 = r0 + t < nwin ? s_H[r0 + t] : Hs[rs + t];
        const int64_t h2 = r0 + t + 1 < nwin ? s_H[r0 + t + 1] : Hs[rs + t + 1], dl = h1 - h2;
        if (10 * dl >= 256 * (int64_t)Ha && 5 * dl >= h1) {
          const int64_t key = (dl << 20) | (int64_t)((1 << 20) - 1 - t);
          best = key > best ? key : best;
        }
      }
      const int64_t b = wave_max64(best);
      if (lane == 0) {
        if (b >= 0) {
          const int t = (1 << 20) - 1 - (int)(b & ((1 << 20) - 1));
          const int X = w_hc ? Xon[t] : Xoff[t];
          const int wd = Xoff[t + 1] - Xoff[t];
          const int l = w_dir == DIR_LR ? w_R0 + X : w_R1 - X - wd;
          s_knee[0] = 1;
          s_knee[1] = w_dir;
          s_knee[2] = l;
          s_knee[3] = l + wd;
        } else {
          s_knee[0] = 0;
        }
      }
    }
    PHASE_CLOCK(6);
    fmax = max(fmax, w_score);
    ++rows;
    if (w_score > Hd) { feasible = 0; break; }
    rs += w_cnt;
    if (pc0 >= 0) pc0 += Ew;
  }
#ifdef TABI_PHASE_CLOCK
    if (!HYB && tid == 0 && P.count == 1 && s < 64) {
      for (int q = 0; q < 8; ++q) g_phase_clock[s][q] = ph_acc[q];
      g_phase_clock[s][8] = rows;
      g_phase_clock[s][9] = k;
      g_phase_clock[s][10] = feasible;
    }
#endif
  } while (false);
  if (tid == 0) {
    w.feas[a * P.B + s] = feasible;
    w.rows[a * P.B + s] = rows;
    if (HYB && feasible != 2) w.tail_t0[s] = d.n;
  }
  // Single atlas: the last of its workgroups to finish selects the scale and
  // writes the outputs (no separate launch).  Every workgroup publishes its
  // results, then counts itself; the counter is zeroed again by the last
  // one.  Batches launch the selection instead: a device-wide fence in each
  // of their many workgroups costs more than the launch it saves.
  if (P.fixed_k > 0 || P.count != 1 || HYB) return;
  if (!last_to_finish(&w.cnt[a], P.Br, s_cnt)) return;
  if (tid == 0) w.cnt[a] = 0;
  select_atlas(P, w, round, last_round, a, out_xy, out_orient, out_scale, s_red);
}

// Scale selection of every atlas of a batch, one workgroup per atlas.
__global__ __launch_bounds__(256) void k_select(Params P, Work w, int round, int last_round,
                                                int32_t* out_xy, uint8_t* out_orient,
                                                float* out_scale) {
  __shared__ int32_t sh[3];
  if (round_idle(w, round)) return;
  select_atlas(P, w, round, last_round, blockIdx.x, out_xy, out_orient, out_scale, sh);
}

// Placements of the single diagnostic scale (slot 0, atlas 0) in input order.
__global__ __launch_bounds__(256) void k_scatter(Params P, Work w, int32_t* out_xy,
                                                 uint8_t* out_orient, int32_t* feasible,
                                                 int32_t* rows) {
  const AtlasDesc d = w.desc[0];
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    feasible[0] = d.bad ? -1 : w.feas[0];
    rows[0] = d.bad ? 0 : w.rows[0];
  }
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < d.n; t += gridDim.x * blockDim.x) {
    const int dst = w.perm[t];
    const int32_t x = d.bad ? -1 : w.xs[t];
    out_xy[2 * (size_t)dst] = x >= 0 ? x : -1;
    out_xy[2 * (size_t)dst + 1] = x >= 0 ? w.ys[t] : -1;
    out_orient[dst] = x >= 0 ? (uint8_t)(w.srecs[t].bits | (w.mir[t] << 3)) : 0;
  }
}

hipError_t launch_scatter(const Params& P, const Work& w, int32_t* out_xy, uint8_t* out_orient,
                          int32_t* feasible, int32_t* rows, hipStream_t st) {
  int blocks = (P.N + 255) / 256;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(256), 0, st, P, w, out_xy, out_orient, feasible,
                     rows);
  return hipGetLastError();
}

PackLds pack_lds_plan(int nmax, int Wd, int budget) {
  PackLds L;
  L.RC = nmax < Wd ? nmax : Wd;
  if (L.RC < 1) L.RC = 1;
  const int fixed = 4 * Wd + 8 * (L.RC + 1);
  int pw = (budget - fixed) / 4;
  if (pw < 4 * L.RC) pw = 4 * L.RC;  // the offsets of four configurations must fit
  if (pw > (1 << 20)) pw = 1 << 20;
  L.PW = pw;
  L.bytes = fixed + 4 * L.PW;
  return L;
}

int pack_static_lds() {
  int r = 0;
  for (const void* f : {(const void*)k_pack<512>, (const void*)k_pack<1024>}) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, f) != hipSuccess) return 32 * 1024;
    r = (int)a.sharedSizeBytes > r ? (int)a.sharedSizeBytes : r;
  }
  return r;
}

hipError_t pack_set_max_lds(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_pack<512>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pack<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             bytes);
}

hipError_t launch_select(const Params& P, const Work& w, int round, int last_round,
                         int32_t* out_xy, uint8_t* out_orient, float* out_scale, hipStream_t st) {
  if (P.count == 1 || P.fixed_k > 0) return hipSuccess;  // done inside k_pack / not wanted
  hipLaunchKernelGGL(k_select, dim3(P.count), dim3(256), 0, st, P, w, round, last_round, out_xy,
                     out_orient, out_scale);
  return hipGetLastError();
}

hipError_t launch_pack(const Params& P, const Work& w, int round, int lds_bytes, int RC, int PW,
                       int stage_cap, int last_round, int32_t* out_xy, uint8_t* out_orient,
                       float* out_scale, hipStream_t st) {
  // one atlas: latency matters, use the wider workgroup (batches: as tuned)
  if (P.hybrid) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_pack<1024, true>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pack<1024, true>), dim3(P.Br, P.count), dim3(1024), lds_bytes, st, P, w,
                       round, RC, PW, stage_cap, last_round, out_xy, out_orient, out_scale);
  } else if (P.pack_nt == 1024 || (P.pack_nt == 0 && P.count == 1))
    hipLaunchKernelGGL(k_pack<1024>, dim3(P.Br, P.count), dim3(1024), lds_bytes, st, P, w, round,
                       RC, PW, stage_cap, last_round, out_xy, out_orient, out_scale);
  else
    hipLaunchKernelGGL(k_pack<512>, dim3(P.Br, P.count), dim3(512), lds_bytes, st, P, w, round, RC,
                       PW, stage_cap, last_round, out_xy, out_orient, out_scale);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Hybrid tail (Sec. 4.4, "Performance Optimization"), single atlas.
//
// The fold-and-push workgroup of a scale slot that reaches the t_opt switch
// leaves its frontline and the tail's first chart t0 in the work space
// (feasible = 2).  k_tail then takes that slot, one workgroup:
//   1. rows by prefix-sum folding at the head scale k: chart j's offset is
//      its grown width less the compacting distance to chart j + 1, and the
//      prefix sum of the offsets divided by the grown atlas width is its row;
//   2. the tail's scale kt, from k down, accepted when every row laid out
//      with compaction at kt fits the width;
//   3. the rows in order, in the one left-to-right : two right-to-left
//      alternation: push, correction (Alg. 1), frontline update and the
//      overflow test.
//   4. the slot's sum over charts of area * scale.
// A hybrid pack evaluates every scale 1..64 in a slot of its own, so all
// the tail needs at kt (grown extents, set-up records, compacting distances
// and flags of sorted neighbours, stored profiles) is read, unchanged, from
// the slot of scale kt.
// k_select_hybrid then keeps the slot with the largest sum (ties to the
// larger k) and writes the outputs with each chart's own scale.
// ---------------------------------------------------------------------------
constexpr int TAIL_NT = 1024;

// inclusive block scan of int32 values whose block total fits 31 bits;
// `total` gets the block total (every thread); red: TAIL_NT / WAVE ints
template <int WAVES>
__device__ inline int32_t block_incl_sum(int32_t v, int32_t* red, int32_t& total) {
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const int32_t incl = wave_incl_sum(v);
  __syncthreads();
  if (lane == WAVE - 1) red[wv] = incl;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    const int32_t r = red[i];
    base += i < wv ? r : 0;
    tot += r;
  }
  total = uni(tot);
  return base + incl;
}

// inclusive block max scan (same contract)
template <int WAVES>
__device__ inline int32_t block_incl_max(int32_t v, int32_t* red, int32_t& total) {
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const int32_t incl = wave_incl_max(v);
  __syncthreads();
  if (lane == WAVE - 1) red[wv] = incl;
  __syncthreads();
  int32_t base = -BIG, tot = -BIG;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    const int32_t r = red[i];
    base = i < wv ? max(base, r) : base;
    tot = max(tot, r);
  }
  total = uni(tot);
  return max(base, incl);
}

__global__ __launch_bounds__(TAIL_NT) void k_tail(Params P, Work w, int RC, int PW) {
  constexpr int WAVES = TAIL_NT / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_red[WAVES * 6];
  __shared__ int32_t s_lr[LRCAP][3];
  __shared__ int32_t s_lrn, s_lrover;
  __shared__ int32_t s_seg[TAIL_NT];
  __shared__ uint64_t s_area[2 * WAVES];
  const int s = blockIdx.x;
  if (w.feas[s] != 2) return;  // no tail at this slot (uniform)
  const AtlasDesc d = w.desc[0];
  const int k = slot_k(P, d, 0, s);
  const int n = d.n, Wd = d.Wa + P.p, Hd = d.Ha + P.p, p = P.p, K = P.K;
  const int tid = threadIdx.x, wv = tid / WAVE, lane = lane_id();
  // dynamic LDS (the fold-and-push plan): frontline, row offsets without /
  // with compaction, then a pool of PW words: the row's offsets Y (RC) and
  // its texel bounds
  int32_t* F = reinterpret_cast<int32_t*>(smem);
  int32_t* Xoff = F + Wd;
  int32_t* Xon = Xoff + (RC + 1);
  int32_t* Y = Xon + (RC + 1);
  const Chart* ch = w.srecs;
  const size_t slot = (size_t)s * P.N;
  int32_t* xs = w.xs + slot;   // first: each tail chart's row start
  int32_t* ys = w.ys + slot;   // first: each tail chart's row (low 32 bits)
  uint8_t* mir = w.mir + slot;
  int32_t* lrpre = w.lrpre + slot;
  const int t0 = w.tail_t0[s];

  int32_t fm = 0;
  for (int x = tid; x < Wd; x += TAIL_NT) {
    const int32_t v = w.tailF[(size_t)s * P.Wdmax + x];
    F[x] = v;
    fm = max(fm, v);
  }
  int32_t fmax = block_reduce_max<WAVES>(fm, s_red);

  // ---- 1. rows by prefix sums of the offsets at the head scale
  {
    const int32_t* wdk = w.wdv + slot;
    const int32_t* cdk = w.cd + slot;
    int64_t carry = 0;
    for (int b0 = t0; b0 < n; b0 += TAIL_NT) {
      const int j = b0 + tid;
      const int32_t a = j < n ? wdk[j] - (j + 1 < n ? cdk[j + 1] : 0) : 0;
      int32_t tot;
      const int32_t incl = block_incl_sum<WAVES>(a, s_red, tot);
      if (j < n) ys[j] = (int32_t)(uint32_t)((uint64_t)(carry + incl - a) / (uint64_t)Wd);
      carry += tot;
    }
    __syncthreads();
    // row start of every tail chart: a running max of the row heads
    int32_t run = t0;
    for (int b0 = t0; b0 < n; b0 += TAIL_NT) {
      const int j = b0 + tid;
      const bool head = j < n && (j == t0 || ys[j] != ys[j - 1]);
      int32_t tot;
      const int32_t st = max(run, block_incl_max<WAVES>(head ? j : -BIG, s_red, tot));
      if (j < n) xs[j] = st;
      run = max(run, tot);
    }
  }

  // ---- 2. the tail's scale: the largest kt <= k at which every row fits.
  // A chunk of charts at a time (offsets within the rows, a segmented sum);
  // a candidate is dropped at the first chunk with a chart past the right
  // edge (rows folded by prefix sums mostly end in such a chart).
  int kt = k, feasible = 0;
  for (; kt >= 1 && !feasible; --kt) {
    const size_t sl = (size_t)(d.ktop - P.koff - kt) * P.N;  // the slot of scale kt
    const int32_t* wdt = w.wdv + sl;
    const int32_t* cdt = w.cd + sl;
    int over = 0;
    int32_t xc = 0;  // offset of the chart after the previous chunk, within its row
    for (int b0 = t0; b0 < n && !over; b0 += TAIL_NT) {
      const int j = b0 + tid, b1 = min(n, b0 + TAIL_NT);
      const bool in = j < b1;
      // X_j = X_{j-1} + w'_{j-1} - cd_j, 0 at a row's first chart
      const bool head = in && xs[j] == j;
      const int32_t inc = (in && !head) ? wdt[j - 1] - cdt[j] : 0;
      int32_t tot;
      const int32_t S = block_incl_sum<WAVES>(inc, s_red, tot);
      s_seg[tid] = S;
      __syncthreads();
      int32_t X = 0;
      if (in) {
        const int st = xs[j];
        X = st < b0 ? xc + S : S - s_seg[st - b0];
        over = X + wdt[j] > Wd;
      }
      if (j == b1 - 1) s_red[WAVES * 6 - 1] = X;
      over = __syncthreads_or(over);
      xc = uni(s_red[WAVES * 6 - 1]);
    }
    if (!over) feasible = 1;
  }
  ++kt;  // the loop stepped past the scale that fit

  // ---- 3. the rows, pushed up in the fixed direction alternation, with
  // the data of the slot of scale kt
  if (feasible) {
    const size_t sl = (size_t)(d.ktop - P.koff - kt) * P.N;
    const int32_t* wdt = w.wdv + sl;
    const int32_t* hdt = w.hdv + sl;
    const int32_t* cdt = w.cd + sl;
    const uint8_t* flt = w.fl + sl;
    const int32_t* pcol = w.pcol + sl;
    const int32_t* prow = w.prow + sl;
    const unsigned char* kct = w.kc + sl * P.stride;
    const int32_t sbase = w.segbase[d.ktop - P.koff - kt];  // -1: profiles not stored
    const bool prof = sbase >= 0;
    const uint32_t* seg = w.arena + (prof ? sbase : 0);
    auto KV = [&](int c) { return kview(kct + (size_t)c * P.stride, K); };
    int rs = t0, trow = 0;
    while (rs < n) {
      int re = n;  // the row ends at the first chart of another row
      for (int b0 = rs + 1; b0 < n; b0 += TAIL_NT) {
        const int j = b0 + tid;
        const int e = block_reduce_min<WAVES>(j < n && xs[j] != rs ? j : n, s_red);
        if (e < n) { re = e; break; }
      }
      const int cnt = re - rs;
      if (cnt > RC) { feasible = -2; break; }  // cannot happen: advances are >= 1
      int32_t co = 0, cn = 0;
      for (int b0 = 0; b0 < cnt; b0 += TAIL_NT) {
        const int t = b0 + tid, c = rs + t;
        const int32_t wd = t < cnt ? wdt[c] : 0;
        const int32_t adv = t < cnt ? wd - (t + 1 < cnt ? cdt[c + 1] : 0) : 0;
        int32_t to, tn;
        const int32_t io = block_incl_sum<WAVES>(wd, s_red, to);
        const int32_t in = block_incl_sum<WAVES>(adv, s_red, tn);
        if (t < cnt) {
          Xoff[t] = co + io - wd;
          Xon[t] = cn + in - adv;
          Y[t] = -BIG;
        }
        co += to;
        cn += tn;
      }
      if (tid == 0) {
        Xoff[cnt] = co;
        Xon[cnt] = cn;
        s_lrn = 0;
        s_lrover = 0;
      }
      __syncthreads();
      const int dir = (trow % 3 == 0) ? DIR_LR : DIR_RL;
      ++trow;
      const int E = co;  // grown columns of the row's charts
      // texel bounds: stored (the row's charts are consecutive in the
      // segment, so texel e is word pcol[rs] + e), else from the records and
      // kept in shared memory for the update when they fit
      uint32_t* stg = reinterpret_cast<uint32_t*>(Y + RC);
      const bool staged = !prof && RC + E <= PW;
      const uint32_t* gprof = seg + (prof ? pcol[rs] : 0);
      for (int e = tid; e < E; e += TAIL_NT) {
        const int t = find_chart(Xoff, cnt, e), i = e - Xoff[t];
        int32_t tp, bt;
        if (prof) {
          tp = lo16(gprof[e]);
        } else {
          column_bounds_grown(KV(rs + t), ch[rs + t], K, kt, p, i, tp, bt);
          if (staged) stg[e] = pack16(tp, bt);
        }
        const int col = dir == DIR_LR ? Xon[t] + i : Wd - 1 - Xon[t] - i;
        atomicMax(&Y[t], F[col] - tp);
      }
      // pairs that share columns without being neighbours
      for (int A = tid; A + 2 < cnt; A += TAIL_NT) {
        const int wdA = Xoff[A + 1] - Xoff[A];
        for (int C = A + 2; C < cnt && Xon[C] - Xon[A] < wdA; ++C) {
          const int q = atomicAdd(&s_lrn, 1);
          if (q < LRCAP) { s_lr[q][0] = A; s_lr[q][1] = C; s_lr[q][2] = 0; }
          else s_lrover = 1;
        }
      }
      __syncthreads();
      if (uni(s_lrover)) {  // more than the shared list holds: out of line
        correct_many_pairs<TAIL_NT>(Xon, Xoff, cnt, rs, lrpre, s_red, s_lr, Y, cnt, wv == 0, flt,
                                    prof, seg, prow, hdt, kct, P.stride, ch, K, kt, p);
      } else {
        const int lrn = uni(s_lrn);
        for (int q = wv; q < lrn; q += WAVES) {
          const int A = s_lr[q][0], C = s_lr[q][1];
          const int wdA = Xoff[A + 1] - Xoff[A];
          const PairSweep sw =
              prof ? pair_rows_meet(seg + prow[rs + A], hdt[rs + A], seg + prow[rs + C],
                                    hdt[rs + C], wdA)
                   : pair_records_sweep<2>(KV(rs + A), ch[rs + A], KV(rs + C), ch[rs + C], K,
                                           kt, p);
          const int f = pair_flags_at(sw, wdA, Xon[C] - Xon[A]);
          if (lane == 0) s_lr[q][2] = f;
        }
        __syncthreads();
        if (wv == 0) correct_offsets(Y, cnt, flt + rs, s_lr, lrn);
      }
      __syncthreads();
      for (int e = tid; e < E; e += TAIL_NT) {
        const int t = find_chart(Xoff, cnt, e), i = e - Xoff[t];
        int32_t tp, bt;
        if (prof) bt = hi16(gprof[e]);
        else if (staged) bt = hi16(stg[e]);
        else column_bounds_grown(KV(rs + t), ch[rs + t], K, kt, p, i, tp, bt);
        const int col = dir == DIR_LR ? Xon[t] + i : Wd - 1 - Xon[t] - i;
        atomicMax(&F[col], Y[t] + bt);
      }
      // the row's score: a chart's largest grown bottom is h + p
      int32_t M = -BIG;
      for (int t = tid; t < cnt; t += TAIL_NT) {
        const int c = rs + t;
        M = max(M, Y[t] + hdt[c]);
        const int wd = Xoff[t + 1] - Xoff[t];
        xs[c] = dir == DIR_LR ? Xon[t] : Wd - Xon[t] - wd;
        ys[c] = Y[t];
        mir[c] = (uint8_t)(dir == DIR_RL);
      }
      fmax = max(fmax, block_reduce_max<WAVES>(M, s_red));
      if (fmax > Hd) { feasible = 0; break; }
      rs = re;
    }
  }

  // ---- 4. sum over charts of area2 * scale: head at k, tail at kt
  uint64_t ah = 0, at = 0;  // per thread below 2^56 (area2 < 2^47, n <= 2^18)
  for (int c = tid; c < n; c += TAIL_NT) {
    if (c < t0) ah += (uint64_t)ch[c].area2;
    else at += (uint64_t)ch[c].area2;
  }
  ah = wave_sum_u64(ah);  // per wavefront below 2^62
  at = wave_sum_u64(at);
  __syncthreads();
  if (lane == 0) { s_area[wv] = ah; s_area[WAVES + wv] = at; }
  __syncthreads();
  if (tid == 0) {
    unsigned __int128 H = 0, T = 0;
    for (int i = 0; i < WAVES; ++i) { H += s_area[i]; T += s_area[WAVES + i]; }
    const unsigned __int128 obj = H * (unsigned)k + T * (unsigned)(feasible == 1 ? kt : 0);
    w.tail_obj[2 * s] = (uint64_t)obj;
    w.tail_obj[2 * s + 1] = (uint64_t)(obj >> 64);
    w.tail_kt[s] = feasible == 1 ? kt : 0;
    w.feas[s] = feasible;
  }
}

// The scale of a hybrid pack: among the feasible slots, the largest sum
// over charts of area2 * scale (slots without a tail: k times the total
// area), ties to the larger k; then the outputs with each chart's scale.
// Every workgroup finds the same slot and writes its share of the charts.
__global__ __launch_bounds__(256) void k_select_hybrid(Params P, Work w, int32_t* out_xy,
                                                       uint8_t* out_orient, float* out_ks,
                                                       float* out_scale) {
  __shared__ int32_t s_best;
  const AtlasDesc d = w.desc[0];
  const int tid = threadIdx.x, lane = lane_id();
  if (tid < WAVE) {
    const unsigned __int128 total =
        ((unsigned __int128)w.tail_obj[2 * P.B + 1] << 64) | w.tail_obj[2 * P.B];
    const int sl = lane;
    const bool live = !d.bad && d.n > 0 && sl < P.Br;
    const int f = live ? w.feas[sl] : 0;
    const int k = live ? slot_k(P, d, 0, sl) : 0;
    const bool ok = f == 1 && k >= 1;
    unsigned __int128 obj = 0;
    if (ok) {
      if (w.tail_t0[sl] < d.n)
        obj = ((unsigned __int128)w.tail_obj[2 * sl + 1] << 64) | w.tail_obj[2 * sl];
      else
        obj = total * (unsigned)k;
    }
    int kk = ok ? k : 0, best = ok ? sl : -1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const uint64_t ohi = __shfl_xor((unsigned long long)(uint64_t)(obj >> 64), o);
      const uint64_t olo = __shfl_xor((unsigned long long)(uint64_t)obj, o);
      const int okk = __shfl_xor(kk, o), ob = __shfl_xor(best, o);
      const unsigned __int128 oo = ((unsigned __int128)ohi << 64) | olo;
      if (ob >= 0 && (best < 0 || oo > obj || (oo == obj && okk > kk))) {
        obj = oo;
        kk = okk;
        best = ob;
      }
    }
    if (lane == 0) s_best = best;
  }
  __syncthreads();
  const int best = s_best;
  const int k = best >= 0 ? slot_k(P, d, 0, best) : 0;
  const int t0 = best >= 0 ? w.tail_t0[best] : 0;
  const int kt = best >= 0 && t0 < d.n ? w.tail_kt[best] : k;
  const size_t slot = (size_t)(best >= 0 ? best : 0) * P.N;
  for (int t = blockIdx.x * blockDim.x + tid; t < d.n; t += gridDim.x * blockDim.x) {
    const int dst = w.perm[t];
    if (!d.bad && best >= 0) {
      out_xy[2 * (size_t)dst] = w.xs[slot + t];
      out_xy[2 * (size_t)dst + 1] = w.ys[slot + t];
      out_orient[dst] = (uint8_t)(w.srecs[t].bits | (w.mir[slot + t] << 3));
      out_ks[dst] = (float)(t < t0 ? k : kt) / 64.0f;
    } else {
      out_xy[2 * (size_t)dst] = -1;
      out_xy[2 * (size_t)dst + 1] = -1;
      out_orient[dst] = 0;
      out_ks[dst] = 0.0f;
    }
  }
  if (blockIdx.x == 0 && tid == 0)
    out_scale[0] = d.bad ? -1.0f : (d.n == 0 ? 1.0f : (best >= 0 ? (float)k / 64.0f : 0.0f));
}

int read_phase_clock(int64_t* out, int slots) {
#ifdef TABI_PHASE_CLOCK
  static long long buf[64][11];
  if (hipMemcpyFromSymbol(buf, HIP_SYMBOL(g_phase_clock), sizeof(buf)) != hipSuccess) return -1;
  const int m = slots < 64 ? slots : 64;
  for (int i = 0; i < m; ++i)
    for (int q = 0; q < 11; ++q) out[i * 11 + q] = buf[i][q];
  return m;
#else
  (void)out;
  (void)slots;
  return -2;
#endif
}

hipError_t launch_tail(const Params& P, const Work& w, int lds_bytes, int RC, int PW,
                       hipStream_t st) {
  const hipError_t e = hipFuncSetAttribute((const void*)k_tail,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tail, dim3(P.Br), dim3(TAIL_NT), lds_bytes, st, P, w, RC, PW);
  return hipGetLastError();
}

hipError_t launch_select_hybrid(const Params& P, const Work& w, int32_t* out_xy,
                                uint8_t* out_orient, float* out_ks, float* out_scale,
                                hipStream_t st) {
  int blocks = (P.N + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_select_hybrid, dim3(blocks), dim3(256), 0, st, P, w, out_xy, out_orient,
                     out_ks, out_scale);
  return hipGetLastError();
}


}  // namespace tabi
