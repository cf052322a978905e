// Serving context: continuous batching of pack requests over several HIP
// streams, with the charts' proxy records resident on the device so that a
// re-pack recomputes only the replaced charts.  Implements tabi_ctx_* /
// tabi_submit / tabi_repack / tabi_poll of include/tabi.h.
//
// Memory: one device allocation of the configured budget, carved by a
// first-fit allocator into (a) one region per batch in flight (its uploaded
// tables and chart data, prepared and assembled records, outputs and the
// batched work space), freed when the batch completes, and (b) one block of
// records per resident atlas version.  Each stream (launch slot) owns two
// pinned host staging buffers, one per direction, so every copy is
// asynchronous from memory the context owns and keeps until the batch's
// event.  Nothing is allocated after creation.
//
// Versions: a re-pack writes a new records block (copy on write); the old
// block is released once no batch in flight reads it.  A batch holds at most
// one request per atlas, and a re-pack whose atlas version is written by a
// batch still in flight on another stream waits for that batch's event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <stdint.h>
#include <string.h>
#include <unordered_map>
#include <vector>

#include "../../include/tabi.h"
#include "tabi_internal.h"

using namespace tabi;

namespace {

constexpr size_t ALIGN = 256;
size_t rup(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// First-fit allocator over [0, cap) in ALIGN units.
class Arena {
 public:
  void init(size_t cap) {
    cap_ = cap / ALIGN * ALIGN;
    free_.clear();
    if (cap_) free_[0] = cap_;
    used_ = peak_ = 0;
  }
  static constexpr size_t NONE = ~(size_t)0;
  size_t alloc(size_t bytes) {
    bytes = rup(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return off;
    }
    return NONE;
  }
  void release(size_t off, size_t bytes) {
    bytes = rup(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t cap() const { return cap_; }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Block {       // one version of an atlas's records
  size_t off = 0, bytes = 0;
  int refs = 0;      // the atlas table and every batch in flight that reads or writes it
  int64_t writer = -1;  // batch writing it (-1: written)
};

struct Atlas {
  int32_t n = 0, W = 0, H = 0, padding = 0, quality = 0;
  int64_t block = -1;   // current version (-1: not resident)
  int64_t last_use = 0;
};

struct Req {
  int64_t ticket = 0;
  int32_t atlas = 0, n = 0, W = 0, H = 0, padding = 0, quality = 0;
  bool repack = false;
  std::vector<int32_t> xy, off, idx;  // prepared charts (all of a new atlas, or the replaced)
  int32_t* oxy = nullptr;
  uint8_t* oor = nullptr;
  float* osc = nullptr;
  double t_submit = 0;
};

struct Plan {  // byte offsets of one batch's device region
  int count = 0, N = 0, M = 0, nmax = 0, side = 0, padding = 0, quality = 0;
  int64_t V = 0;
  size_t aoff, poff, awh, src, dst, voff, idx, xy, up_end;  // uploaded part
  size_t scratch, prep, recs;
  size_t oxy, oor, osc, down_end;  // downloaded part, from oxy
  size_t ws, ws_bytes, total;
};

struct Batch {
  int64_t seq = 0;
  int slot = 0;
  int status = 0;  // TABI_OK, or the error of an enqueue that failed midway
  std::vector<Req> reqs;
  Plan pl;
  size_t off = 0;  // region in the arena
  std::vector<int64_t> blocks;  // block refs held until completion
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  unsigned char* up = nullptr;
  unsigned char* down = nullptr;
  int64_t batch = -1;  // in flight, or -1
};

}  // namespace

struct tabi_ctx {
  std::mutex mu;
  tabi_ctx_config cfg{};
  int dev = 0;
  unsigned char* base = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  std::deque<Req> queue;
  std::map<int64_t, Batch> inflight;
  std::unordered_map<int64_t, Block> blocks;
  std::map<int32_t, Atlas> atlases;
  std::vector<tabi_done> done;
  int64_t next_ticket = 1, next_batch = 1, next_block = 1, use_clock = 0;
  int32_t next_atlas = 0;
  hipEvent_t t0ev = nullptr;
  std::chrono::steady_clock::time_point t0;
  int64_t n_launches = 0, n_done = 0, n_evicted = 0, n_failed = 0, n_waits = 0, peak_inflight = 0;
  int broken = 0;  // a batch's completion event could not be recorded: unusable
};

namespace {

double now_s(const tabi_ctx* c) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - c->t0).count();
}

Plan plan_batch(const tabi_ctx* c, const std::vector<const Req*>& rs) {
  Plan p;
  p.count = (int)rs.size();
  if (!rs.empty()) {  // the requests of a batch share padding and quality
    p.padding = rs[0]->padding;
    p.quality = rs[0]->quality;
  }
  for (const Req* r : rs) {
    p.N += r->n;
    p.M += (int)(r->off.size() - 1);
    p.V += (int64_t)r->xy.size() / 2;
    p.nmax = std::max(p.nmax, r->n);
    p.side = std::max(p.side, std::max(r->W, r->H));
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = rup(o + bytes);
    return at;
  };
  p.aoff = take(4 * (size_t)(p.count + 1));
  p.poff = take(4 * (size_t)(p.count + 1));
  p.awh = take(8 * (size_t)p.count);
  p.src = take(8 * (size_t)p.count);
  p.dst = take(8 * (size_t)p.count);
  p.voff = take(4 * (size_t)(p.M + 1));
  p.idx = take(4 * (size_t)std::max(p.M, 1));
  p.xy = take(8 * (size_t)std::max<int64_t>(p.V, 1));
  p.up_end = o;
  p.scratch = take(host_prep_scratch_bytes(p.M));
  p.prep = take(sizeof(Chart) * (size_t)std::max(p.M, 1));
  p.recs = take(sizeof(Chart) * (size_t)std::max(p.N, 1));
  p.oxy = take(8 * (size_t)std::max(p.N, 1));
  p.oor = take((size_t)std::max(p.N, 1));
  p.osc = take(4 * (size_t)p.count);
  p.down_end = o;
  p.ws_bytes = (size_t)host_many_workspace_bytes(p.count, p.N, p.nmax, p.side, p.padding,
                                                 p.quality);
  p.ws = take(p.ws_bytes);
  p.total = o;
  return p;
}

void block_unref(tabi_ctx* c, int64_t id) {
  auto it = c->blocks.find(id);
  if (it == c->blocks.end()) return;
  if (--it->second.refs == 0) {
    c->arena.release(it->second.off, it->second.bytes);
    c->blocks.erase(it);
  }
}

void finish(tabi_ctx* c, const Req& r, int status, int batch, double t_done) {
  tabi_done d;
  d.ticket = r.ticket;
  d.atlas_id = r.atlas;
  d.status = status;
  d.batch = batch;
  d.latency_ms = status == TABI_OK ? (t_done - r.t_submit) * 1000.0 : 0.0;
  d.submit_ms = r.t_submit * 1000.0;
  d.done_ms = t_done * 1000.0;
  c->done.push_back(d);
  if (status != TABI_OK) ++c->n_failed;
}

// Evict the least recently used resident atlas not needed by `keep`;
// false when none can go (every other block is read by a batch in flight).
bool evict_one(tabi_ctx* c, const std::vector<int32_t>& keep) {
  int32_t victim = -1;
  int64_t oldest = 0;
  for (auto& kv : c->atlases) {
    const Atlas& a = kv.second;
    if (a.block < 0 || std::find(keep.begin(), keep.end(), kv.first) != keep.end()) continue;
    const Block& b = c->blocks[a.block];
    if (b.refs != 1) continue;  // a batch in flight still holds it
    if (victim < 0 || a.last_use < oldest) { victim = kv.first; oldest = a.last_use; }
  }
  if (victim < 0) return false;
  Atlas& a = c->atlases[victim];
  block_unref(c, a.block);
  a.block = -1;
  ++c->n_evicted;
  return true;
}

// Allocate a batch's region and one new records block per request; on
// failure nothing stays allocated.
bool alloc_batch(tabi_ctx* c, const Plan& pl, const std::vector<const Req*>& rs, size_t* region,
                 std::vector<size_t>* offs) {
  *region = c->arena.alloc(pl.total);
  if (*region == Arena::NONE) return false;
  offs->clear();
  for (const Req* r : rs) {
    const size_t o = c->arena.alloc(sizeof(Chart) * (size_t)r->n);
    if (o == Arena::NONE) {
      for (size_t k = 0; k < offs->size(); ++k)
        c->arena.release((*offs)[k], sizeof(Chart) * (size_t)rs[k]->n);
      c->arena.release(*region, pl.total);
      return false;
    }
    offs->push_back(o);
  }
  return true;
}

int launch(tabi_ctx* c, int si, std::vector<Req>& reqs, const Plan& pl, size_t region,
           const std::vector<size_t>& newoffs) {
  Slot& s = c->slots[si];
  unsigned char* d = c->base + region;
  unsigned char* up = s.up;
  int32_t* aoff = reinterpret_cast<int32_t*>(up + pl.aoff);
  int32_t* poff = reinterpret_cast<int32_t*>(up + pl.poff);
  int32_t* awh = reinterpret_cast<int32_t*>(up + pl.awh);
  uint64_t* src = reinterpret_cast<uint64_t*>(up + pl.src);
  uint64_t* dst = reinterpret_cast<uint64_t*>(up + pl.dst);
  int32_t* voff = reinterpret_cast<int32_t*>(up + pl.voff);
  int32_t* idx = reinterpret_cast<int32_t*>(up + pl.idx);
  int32_t* xy = reinterpret_cast<int32_t*>(up + pl.xy);
  Batch b;
  b.seq = c->next_batch++;
  b.slot = si;
  b.pl = pl;
  b.off = region;
  aoff[0] = 0;
  poff[0] = 0;
  voff[0] = 0;
  int64_t v = 0;
  int m = 0;
  std::vector<hipEvent_t> waits;
  for (size_t q = 0; q < reqs.size(); ++q) {
    Req& r = reqs[q];
    Atlas& a = c->atlases[r.atlas];
    aoff[q + 1] = aoff[q] + r.n;
    const int mq = (int)r.off.size() - 1;
    poff[q + 1] = poff[q] + mq;
    awh[2 * q] = r.W;
    awh[2 * q + 1] = r.H;
    for (int i = 0; i < mq; ++i) {
      voff[m + i + 1] = (int32_t)(v + r.off[i + 1]);
      if (r.repack) idx[m + i] = r.idx[i];
    }
    memcpy(xy + 2 * v, r.xy.data(), r.xy.size() * 4);
    v += (int64_t)r.xy.size() / 2;
    m += mq;
    src[q] = 0;
    if (r.repack) {  // read the current version
      Block& ob = c->blocks[a.block];
      src[q] = reinterpret_cast<uint64_t>(c->base + ob.off);
      ++ob.refs;
      b.blocks.push_back(a.block);
      if (ob.writer >= 0) {
        auto w = c->inflight.find(ob.writer);
        if (w != c->inflight.end() && w->second.slot != si) {
          waits.push_back(c->slots[w->second.slot].ev);
          ++c->n_waits;
        }
      }
    }
    // the new version
    const int64_t id = c->next_block++;
    Block nb;
    nb.off = newoffs[q];
    nb.bytes = sizeof(Chart) * (size_t)r.n;
    nb.refs = 2;  // the atlas table and this batch
    nb.writer = b.seq;
    c->blocks[id] = nb;
    b.blocks.push_back(id);
    dst[q] = reinterpret_cast<uint64_t>(c->base + nb.off);
    if (a.block >= 0) block_unref(c, a.block);  // the table's hold on the old version
    a.block = id;
    a.last_use = ++c->use_clock;
  }
  hipError_t e = hipMemcpyAsync(d, up, pl.up_end, hipMemcpyHostToDevice, s.st);
  for (hipEvent_t w : waits)
    if (e == hipSuccess) e = hipStreamWaitEvent(s.st, w, 0);
  int rc = e == hipSuccess ? TABI_OK : host_hip_fail(e);
  const int32_t* daoff = reinterpret_cast<const int32_t*>(d + pl.aoff);
  const int32_t* dpoff = reinterpret_cast<const int32_t*>(d + pl.poff);
  Chart* prep = reinterpret_cast<Chart*>(d + pl.prep);
  Chart* recs = reinterpret_cast<Chart*>(d + pl.recs);
  if (!rc)
    rc = host_prep_records(reinterpret_cast<const int32_t*>(d + pl.xy),
                           reinterpret_cast<const int32_t*>(d + pl.voff), dpoff, pl.count, pl.M,
                           pl.quality, prep, d + pl.scratch, s.st);
  if (!rc) {
    e = launch_assemble(pl.N, pl.M, pl.count, daoff, dpoff,
                        reinterpret_cast<const uint64_t*>(d + pl.src),
                        reinterpret_cast<const uint64_t*>(d + pl.dst),
                        reinterpret_cast<const int32_t*>(d + pl.idx), prep, recs, s.st);
    if (e != hipSuccess) rc = host_hip_fail(e);
  }
  if (!rc)
    rc = host_pack_many_records_ws(recs, daoff, pl.count,
                                   reinterpret_cast<const int32_t*>(d + pl.awh), pl.N, pl.nmax,
                                   pl.side, pl.padding, pl.quality,
                                   reinterpret_cast<int32_t*>(d + pl.oxy), d + pl.oor,
                                   reinterpret_cast<float*>(d + pl.osc), d + pl.ws, pl.ws_bytes,
                                   s.st);
  if (!rc) {
    e = hipMemcpyAsync(s.down, d + pl.oxy, pl.down_end - pl.oxy, hipMemcpyDeviceToHost, s.st);
    if (e != hipSuccess) rc = host_hip_fail(e);
  }
  // a batch whose enqueue failed midway still completes in order (its event
  // follows whatever was enqueued); its requests then report the error
  b.status = rc;
  e = hipEventRecord(s.ev, s.st);
  b.reqs = std::move(reqs);
  s.batch = b.seq;
  c->inflight[b.seq] = std::move(b);
  ++c->n_launches;
  c->peak_inflight = std::max<int64_t>(c->peak_inflight, (int64_t)c->inflight.size());
  if (e != hipSuccess) {
    c->broken = host_hip_fail(e);
    return c->broken;
  }
  return TABI_OK;
}

// Admit queued requests into free slots as batches, in arrival order.
int pump(tabi_ctx* c) {
  for (;;) {
    if (c->queue.empty()) return TABI_OK;
    int si = -1;
    for (size_t k = 0; k < c->slots.size(); ++k)
      if (c->slots[k].batch < 0) { si = (int)k; break; }
    if (si < 0) return TABI_OK;
    // requests that cannot run at all leave the queue now
    {
      Req& r = c->queue.front();
      const Atlas& a = c->atlases[r.atlas];
      if (r.repack && a.block < 0) {  // evicted, or its first pack failed
        finish(c, r, TABI_ENOTRESIDENT, 0, now_s(c));
        c->queue.pop_front();
        continue;
      }
    }
    std::vector<const Req*> rs;
    std::vector<int32_t> ids;
    Plan pl;
    for (size_t q = 0; q < c->queue.size() && (int)rs.size() < c->cfg.max_batch; ++q) {
      const Req& r = c->queue[q];
      if (std::find(ids.begin(), ids.end(), r.atlas) != ids.end()) break;  // one per atlas
      if (!rs.empty() && (r.padding != rs[0]->padding || r.quality != rs[0]->quality))
        break;  // a batch shares padding and quality
      if (r.repack && c->atlases[r.atlas].block < 0) break;
      rs.push_back(&r);
      const Plan t = plan_batch(c, rs);
      if (t.up_end > (size_t)c->cfg.staging_bytes ||
          t.down_end - t.oxy > (size_t)c->cfg.staging_bytes) {
        rs.pop_back();
        break;
      }
      pl = t;
      ids.push_back(r.atlas);
    }
    if (rs.empty()) {  // the first request alone exceeds the staging buffers
      finish(c, c->queue.front(), TABI_ETOOBIG, 0, now_s(c));
      c->queue.pop_front();
      continue;
    }
    size_t region = 0;
    std::vector<size_t> newoffs;
    for (;;) {
      if (alloc_batch(c, pl, rs, &region, &newoffs)) break;
      if (evict_one(c, ids)) continue;
      if (rs.size() > 1) {  // a smaller batch
        rs.pop_back();
        ids.pop_back();
        pl = plan_batch(c, rs);
        continue;
      }
      rs.clear();
      break;
    }
    if (rs.empty()) {
      if (!c->inflight.empty()) return TABI_OK;  // memory frees up as batches complete
      finish(c, c->queue.front(), TABI_ETOOBIG, 0, now_s(c));  // can never fit
      c->queue.pop_front();
      continue;
    }
    std::vector<Req> take;
    for (size_t k = 0; k < rs.size(); ++k) {
      take.push_back(std::move(c->queue.front()));
      c->queue.pop_front();
    }
    const int rc = launch(c, si, take, pl, region, newoffs);
    if (rc) return rc;  // the context is unusable
  }
}

// Completed batches: results to the callers' buffers, memory released.
int retire(tabi_ctx* c, bool wait_one) {
  bool waited = false;
  for (auto it = c->inflight.begin(); it != c->inflight.end();) {
    Batch& b = it->second;
    Slot& s = c->slots[b.slot];
    hipError_t e = hipEventQuery(s.ev);
    if (e == hipErrorNotReady && wait_one && !waited) {
      e = hipEventSynchronize(s.ev);
      waited = true;
    }
    if (e == hipErrorNotReady) {
      (void)hipGetLastError();
      ++it;
      continue;
    }
    if (e != hipSuccess) return host_hip_fail(e);
    waited = true;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, c->t0ev, s.ev);
    if (e != hipSuccess) return host_hip_fail(e);
    const double t_done = ms / 1000.0;
    const Plan& pl = b.pl;
    const unsigned char* dn = s.down;
    const int32_t* oxy = reinterpret_cast<const int32_t*>(dn);
    const uint8_t* oor = dn + (pl.oor - pl.oxy);
    const float* osc = reinterpret_cast<const float*>(dn + (pl.osc - pl.oxy));
    int64_t a0 = 0;
    for (size_t q = 0; q < b.reqs.size(); ++q) {
      const Req& r = b.reqs[q];
      if (b.status == TABI_OK) {
        memcpy(r.oxy, oxy + 2 * a0, 8 * (size_t)r.n);
        memcpy(r.oor, oor + a0, (size_t)r.n);
        *r.osc = osc[q];
      }
      a0 += r.n;
      finish(c, r, b.status, (int)b.seq, t_done);
      ++c->n_done;
    }
    if (b.status != TABI_OK) {  // versions this batch was to write are not valid
      for (const Req& r : b.reqs) {
        Atlas& a = c->atlases[r.atlas];
        auto bl = a.block >= 0 ? c->blocks.find(a.block) : c->blocks.end();
        if (bl != c->blocks.end() && bl->second.writer == b.seq) {
          block_unref(c, a.block);
          a.block = -1;
        }
      }
    }
    for (int64_t id : b.blocks) {
      auto bl = c->blocks.find(id);
      if (bl != c->blocks.end() && bl->second.writer == b.seq) bl->second.writer = -1;
      block_unref(c, id);
    }
    c->arena.release(b.off, pl.total);
    s.batch = -1;
    it = c->inflight.erase(it);
  }
  return TABI_OK;
}

bool check_csr(const int32_t* xy, const int32_t* off, int32_t n) {
  if (!off || off[0] != 0) return false;
  for (int32_t i = 0; i < n; ++i)
    if (off[i + 1] < off[i]) return false;
  return n == 0 || xy != nullptr || off[n] == 0;
}

}  // namespace

extern "C" {

int tabi_ctx_create(const tabi_ctx_config* cfg, tabi_ctx** out) {
  if (!cfg || !out || cfg->quality < 0 || cfg->quality > 2 || cfg->padding < 0 ||
      cfg->padding > TABI_MAX_PADDING || cfg->streams < 1 || cfg->streams > 16 ||
      cfg->max_batch < 1 || cfg->max_batch > 1024 || cfg->device_bytes < (1 << 20) ||
      cfg->staging_bytes < (1 << 16))
    return TABI_EINVAL;
  *out = nullptr;
  tabi_ctx* c = new tabi_ctx();
  c->cfg = *cfg;
  hipError_t e = hipGetDevice(&c->dev);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->base), (size_t)cfg->device_bytes);
  if (e == hipSuccess) c->arena.init((size_t)cfg->device_bytes);
  c->slots.resize(cfg->streams);
  for (Slot& s : c->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s.ev);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s.up), (size_t)cfg->staging_bytes);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&s.down), (size_t)cfg->staging_bytes);
  }
  if (e == hipSuccess) e = hipEventCreate(&c->t0ev);
  if (e == hipSuccess) e = hipEventRecord(c->t0ev, c->slots[0].st);
  if (e == hipSuccess) e = hipEventSynchronize(c->t0ev);
  c->t0 = std::chrono::steady_clock::now();
  if (e != hipSuccess) {
    const int rc = e == hipErrorOutOfMemory ? TABI_ENOMEM : host_hip_fail(e);
    (void)hipGetLastError();
    tabi_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return TABI_OK;
}

int tabi_ctx_destroy(tabi_ctx* c) {
  if (!c) return TABI_EINVAL;
  hipError_t first = hipSuccess;
  auto keep = [&](hipError_t e) { if (first == hipSuccess && e != hipSuccess) first = e; };
  for (Slot& s : c->slots)
    if (s.st) keep(hipStreamSynchronize(s.st));
  for (Slot& s : c->slots) {
    if (s.up) keep(hipHostFree(s.up));
    if (s.down) keep(hipHostFree(s.down));
    if (s.ev) keep(hipEventDestroy(s.ev));
    if (s.st) keep(hipStreamDestroy(s.st));
  }
  if (c->t0ev) keep(hipEventDestroy(c->t0ev));
  if (c->base) keep(hipFree(c->base));
  delete c;
  return first == hipSuccess ? TABI_OK : host_hip_fail(first);
}

int tabi_submit_with(tabi_ctx* c, const int32_t* xy, const int32_t* offsets, int32_t n,
                     int32_t atlas_w, int32_t atlas_h, int32_t padding, int32_t quality,
                     int32_t* out_xy, uint8_t* out_orient, float* out_scale, int32_t* atlas_id,
                     int64_t* ticket) {
  if (!c || n < 1 || n > TABI_MAX_CHARTS || atlas_w < 1 || atlas_h < 1 || padding < 0 ||
      padding > TABI_MAX_PADDING || quality < 0 || quality > 2 ||
      (int64_t)atlas_w + padding > 16384 || (int64_t)atlas_h + padding > 16384 ||
      !out_xy || !out_orient || !out_scale || !check_csr(xy, offsets, n))
    return TABI_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->broken) return c->broken;
  Req r;
  r.ticket = c->next_ticket++;
  r.atlas = c->next_atlas++;
  r.n = n;
  r.W = atlas_w;
  r.H = atlas_h;
  r.padding = padding;
  r.quality = quality;
  r.xy.assign(xy, xy + 2 * (size_t)offsets[n]);
  r.off.assign(offsets, offsets + n + 1);
  r.oxy = out_xy;
  r.oor = out_orient;
  r.osc = out_scale;
  r.t_submit = now_s(c);
  Atlas& a = c->atlases[r.atlas];
  a.n = n;
  a.W = atlas_w;
  a.H = atlas_h;
  a.padding = padding;
  a.quality = quality;
  if (atlas_id) *atlas_id = r.atlas;
  if (ticket) *ticket = r.ticket;
  c->queue.push_back(std::move(r));
  return pump(c);
}

int tabi_submit(tabi_ctx* c, const int32_t* xy, const int32_t* offsets, int32_t n,
                int32_t atlas_w, int32_t atlas_h, int32_t* out_xy, uint8_t* out_orient,
                float* out_scale, int32_t* atlas_id, int64_t* ticket) {
  if (!c) return TABI_EINVAL;
  return tabi_submit_with(c, xy, offsets, n, atlas_w, atlas_h, c->cfg.padding, c->cfg.quality,
                          out_xy, out_orient, out_scale, atlas_id, ticket);
}

int tabi_repack(tabi_ctx* c, int32_t atlas_id, const int32_t* replaced_idx, int32_t m,
                const int32_t* xy, const int32_t* offsets, int32_t* out_xy,
                uint8_t* out_orient, float* out_scale, int64_t* ticket) {
  if (!c || m < 1 || !replaced_idx || !out_xy || !out_orient || !out_scale ||
      !check_csr(xy, offsets, m))
    return TABI_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->broken) return c->broken;
  auto it = c->atlases.find(atlas_id);
  if (it == c->atlases.end() || m > it->second.n) return TABI_EINVAL;
  const int32_t n = it->second.n;
  std::vector<int32_t> idx(replaced_idx, replaced_idx + m);
  for (int32_t i = 0; i < m; ++i)  // strictly increasing chart indices of the atlas
    if (idx[i] < 0 || idx[i] >= n || (i > 0 && idx[i] <= idx[i - 1])) return TABI_EINVAL;
  Req r;
  r.ticket = c->next_ticket++;
  r.atlas = atlas_id;
  r.n = n;
  r.W = it->second.W;
  r.H = it->second.H;
  r.repack = true;
  r.padding = it->second.padding;  // a re-pack keeps its atlas's settings
  r.quality = it->second.quality;
  r.idx = std::move(idx);
  r.xy.assign(xy, xy + 2 * (size_t)offsets[m]);
  r.off.assign(offsets, offsets + m + 1);
  r.oxy = out_xy;
  r.oor = out_orient;
  r.osc = out_scale;
  r.t_submit = now_s(c);
  if (ticket) *ticket = r.ticket;
  c->queue.push_back(std::move(r));
  return pump(c);
}

int tabi_poll(tabi_ctx* c, int32_t wait, tabi_done* done, int32_t max_done, int32_t* n_done) {
  if (!c || max_done < 0 || (max_done > 0 && !done) || !n_done) return TABI_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  *n_done = 0;
  if (c->broken) return c->broken;
  int rc = retire(c, false);
  if (!rc) rc = pump(c);
  if (!rc && wait && c->done.empty() && !c->inflight.empty()) {
    rc = retire(c, true);
    if (!rc) rc = pump(c);
  }
  const int32_t k = std::min<int32_t>(max_done, (int32_t)c->done.size());
  for (int32_t i = 0; i < k; ++i) done[i] = c->done[i];
  c->done.erase(c->done.begin(), c->done.begin() + k);
  *n_done = k;
  return rc;
}

int tabi_ctx_stats(tabi_ctx* c, int64_t* stats, int32_t nstats) {
  if (!c || nstats < 0 || (nstats > 0 && !stats)) return TABI_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  int64_t resident = 0;
  for (auto& kv : c->atlases) resident += kv.second.block >= 0;
  const int64_t v[] = {c->n_launches, c->n_done, c->n_failed, c->n_evicted, resident,
                       (int64_t)c->arena.used(), (int64_t)c->arena.peak(),
                       (int64_t)c->queue.size(), (int64_t)c->inflight.size(), c->n_waits,
                       c->peak_inflight};
  for (int32_t i = 0; i < nstats && i < (int32_t)(sizeof(v) / sizeof(v[0])); ++i) stats[i] = v[i];
  return TABI_OK;
}

}  // extern "C"
