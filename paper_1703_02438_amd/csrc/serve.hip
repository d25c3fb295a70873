// serve.hip -- the serving loop: continuous batching of compression and range
// decompression requests under a device memory budget (numarck_server_* in
// include/numarck.h).
//
// One scheduler thread per server.  Each pass it retires finished batches
// (HIP events), then builds a batch from the queued requests that are
// eligible (no earlier request of the same variable unfinished) and whose
// record and workspace fit in the arena, and launches it on a free slot's
// stream: the compressions as one plan (numarck_plan_*), the range
// decompressions after it on the same stream.  Record headers and decode
// flags come back through pinned host memory copied on that stream.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "arena.h"
#include "../../include/numarck.h"

namespace {

using nk::Arena;
constexpr uint32_t kMaxSlots = 8;
constexpr uint32_t kMaxRangePerBatch = 64;

uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }
uint64_t elem_bytes(numarck_dtype d) { return d == NUMARCK_F32 ? 4 : 8; }

// Offsets of a record's buffers inside its arena block.
struct RecordLayout {
  uint64_t packed, centers, incomp, blocks, hdr, total;
};

RecordLayout record_layout(uint64_t n, numarck_dtype dt, uint32_t B, uint64_t bb) {
  const uint64_t L = elem_bytes(dt);
  const uint64_t nb = numarck_block_count(n, B, bb);
  RecordLayout r{};
  uint64_t o = 0;
  r.packed = o;
  o += a256(numarck_packed_bytes(n, B) + 4);
  r.centers = o;
  o += a256(numarck_centers_bytes(B, dt));
  r.incomp = o;
  o += a256((n ? n : 1) * L);
  r.blocks = o;
  o += a256((nb ? nb : 1) * 8);
  r.hdr = o;
  o += a256(sizeof(numarck_header));
  r.total = o;
  return r;
}

struct Record {
  uint64_t off = Arena::kFail;  // arena block
  numarck_out out{};
  numarck_header hdr{};         // host copy, taken when the compression completed
  const void* ref = nullptr;    // the snapshot it was compressed against
  bool valid() const { return off != Arena::kFail; }
};

// Views of the record buffers in the block at `base`.
numarck_out record_view(char* base, const RecordLayout& rl) {
  numarck_out o{};
  o.packed = reinterpret_cast<uint32_t*>(base + rl.packed);
  o.centers = base + rl.centers;
  o.incomp = base + rl.incomp;
  o.block_inc_off = reinterpret_cast<int64_t*>(base + rl.blocks);
  o.recon = nullptr;
  o.bin_ids = nullptr;
  o.hdr = reinterpret_cast<numarck_header*>(base + rl.hdr);
  return o;
}

uint64_t range_ws_bytes(uint64_t len) { return a256(numarck_decompress_workspace_bytes(len)) + 256; }

struct Variable {
  uint64_t n;
  numarck_dtype dtype;
  double E;
  uint32_t B;
  uint64_t bb;
  const void* ref;  // resident previous snapshot
  Record rec;       // latest record (a view of rec_off[cur])
  uint64_t rec_off[2] = {Arena::kFail, Arena::kFail};  // its two record blocks
  int cur = -1;     // block of the latest record, -1 before the first
  bool busy = false;
  uint64_t queued = 0;  // requests waiting
  RecordLayout rl;
  uint64_t tail_small;  // tail capacity of a first attempt (a bounded workspace)
  uint64_t need;        // largest transient block one request of it can take
};

struct Pending {
  numarck_request r;
  double submit_us;
  bool full_tail;  // a retry with the tail capacity that cannot overflow
};

struct Item {
  uint64_t ticket;
  uint32_t var, kind;
  const void* curr = nullptr;     // COMPRESS: the new snapshot
  bool full_tail = false;         // COMPRESS: workspace with full tail capacity
  Record rec;                     // COMPRESS: the new record
  uint64_t ws_off = Arena::kFail;  // RANGE: workspace + flags block
  uint64_t bytes;
  double submit_us;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  numarck_header* pin_hdr = nullptr;  // pinned, one per compression of a batch
  uint32_t* pin_flags = nullptr;      // pinned, one per range request of a batch
  bool busy = false;
  // the batch in flight
  uint64_t serial = 0;
  double start_us = 0.0;
  numarck_plan* plan = nullptr;
  uint64_t ws_off = Arena::kFail;
  std::vector<Item> comp, range;
};

}  // namespace

struct numarck_server {
  numarck_server_config cfg{};
  void* base = nullptr;  // the arena
  Arena arena;
  std::vector<Slot> slots;
  std::vector<Variable> vars;
  std::map<uint64_t, Pending> pending;  // by ticket (submission order)
  std::deque<numarck_completion> done;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread thr;
  bool stop = false;
  uint64_t next_ticket = 1, submitted = 0, completed = 0, batches = 0, max_batch_seen = 0;
  uint64_t resident = 0, waits = 0, tail_retries = 0;
  uint64_t permanent = 0;  // arena bytes held by record blocks
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
        .count();
  }
  char* at(uint64_t off) const { return static_cast<char*>(base) + off; }

  void loop();
  bool retire();
  bool launch();
  void complete(const Item& it, int32_t status, uint32_t flags, uint64_t serial, double start,
                double end);
};

void numarck_server::complete(const Item& it, int32_t status, uint32_t flags, uint64_t serial,
                              double start, double end) {
  numarck_completion c{};
  c.ticket = it.ticket;
  c.var = it.var;
  c.kind = it.kind;
  c.status = status;
  c.flags = flags;
  c.bytes = it.bytes;
  c.batch = serial;
  c.submit_us = it.submit_us;
  c.start_us = start;
  c.done_us = end;
  done.push_back(c);
  ++completed;
}

// Finish the batches whose events have completed.  Caller holds mu.
bool numarck_server::retire() {
  bool any = false;
  for (Slot& s : slots) {
    if (!s.busy) continue;
    const hipError_t q = hipEventQuery(s.done);
    if (q == hipErrorNotReady) continue;
    const double t = now_us();
    const int32_t st = q == hipSuccess ? NUMARCK_OK : NUMARCK_EHIP;
    for (size_t i = 0; i < s.comp.size(); ++i) {
      Item& it = s.comp[i];
      Variable& v = vars[it.var];
      if (st == NUMARCK_OK && (s.pin_hdr[i].flags & NUMARCK_FLAG_TAIL_OVERFLOW) && !it.full_tail) {
        // the bounded tail did not hold this snapshot's out-of-window points:
        // run it again, first in its variable's queue, with full capacity
        numarck_request r{};
        r.kind = NUMARCK_REQ_COMPRESS;
        r.var = it.var;
        r.curr = it.curr;
        pending[it.ticket] = Pending{r, it.submit_us, true};
        ++v.queued;
        v.busy = false;
        ++tail_retries;
        continue;
      }
      if (st == NUMARCK_OK) {  // the new record becomes the latest
        it.rec.hdr = s.pin_hdr[i];
        v.rec = it.rec;
        v.cur = v.rec_off[0] == it.rec.off ? 0 : 1;
        v.ref = it.curr;
      }
      v.busy = false;
      complete(it, st, st == NUMARCK_OK ? s.pin_hdr[i].flags : 0u, s.serial, s.start_us, t);
    }
    for (size_t i = 0; i < s.range.size(); ++i) {
      Item& it = s.range[i];
      arena.release(it.ws_off);
      vars[it.var].busy = false;
      complete(it, st, st == NUMARCK_OK ? s.pin_flags[i] : 0u, s.serial, s.start_us, t);
    }
    if (s.plan) numarck_plan_destroy(s.plan);
    s.plan = nullptr;
    if (s.ws_off != Arena::kFail) arena.release(s.ws_off);
    s.ws_off = Arena::kFail;
    s.comp.clear();
    s.range.clear();
    s.busy = false;
    any = true;
  }
  if (any) cv_done.notify_all();
  return any;
}

// Build and launch one batch on a free slot.  Caller holds mu.
bool numarck_server::launch() {
  Slot* slot = nullptr;
  for (Slot& s : slots)
    if (!s.busy) {
      slot = &s;
      break;
    }
  if (!slot || pending.empty()) return false;

  // Spread the runnable compressions over the free slots: a batch takes at
  // most ceil(runnable / free slots) of them (and max_batch), so several
  // batches run at once.  One batch of every variable leaves nothing to
  // overlap with its slowest job or with the host's work between batches,
  // and measured slower than a few smaller ones on concurrent streams.
  uint32_t free_slots = 0;
  for (const Slot& s : slots) free_slots += s.busy ? 0u : 1u;
  uint64_t runnable = 0;
  {
    // the head request of every variable not busy (a variable's requests run
    // in order); stop once every variable has been seen
    std::vector<char> seen(vars.size(), 0);
    size_t nseen = 0;
    for (auto it = pending.begin(); it != pending.end() && nseen < vars.size(); ++it) {
      const numarck_request& r = it->second.r;
      if (seen[r.var]) continue;
      seen[r.var] = 1;
      ++nseen;
      if (!vars[r.var].busy && r.kind == NUMARCK_REQ_COMPRESS) ++runnable;
    }
  }
  const uint64_t share = (runnable + free_slots - 1) / free_slots;
  const uint64_t cap = share < cfg.max_batch ? (share > 0 ? share : 1) : cfg.max_batch;

  std::vector<Item> comp, range;
  // variables given a request in this batch, or held back behind one
  std::vector<char> taken(vars.size(), 0);
  size_t ntaken = 0;
  auto take = [&](uint32_t var) {
    ntaken += taken[var] ? 0u : 1u;
    taken[var] = 1;
  };
  bool starved = false;
  for (auto it = pending.begin(); it != pending.end() && ntaken < vars.size();) {
    if (comp.size() >= cap && range.size() >= kMaxRangePerBatch) break;
    const numarck_request& r = it->second.r;
    Variable& v = vars[r.var];
    if (v.busy || taken[r.var]) {  // an earlier request of this variable is unfinished
      take(r.var);
      ++it;
      continue;
    }
    Item item{};
    item.ticket = it->first;
    item.var = r.var;
    item.kind = r.kind;
    item.submit_us = it->second.submit_us;
    item.full_tail = it->second.full_tail;
    if (r.kind == NUMARCK_REQ_COMPRESS) {
      if (comp.size() >= cap) {
        take(r.var);  // keep its later requests behind it
        ++it;
        continue;
      }
      // the variable's record block not holding its latest record
      const uint64_t off = v.rec_off[v.cur == 0 ? 1 : 0];
      item.curr = r.curr;
      item.bytes = v.n * elem_bytes(v.dtype);
      item.rec.off = off;
      item.rec.ref = v.ref;
      item.rec.out = record_view(at(off), v.rl);
      comp.push_back(item);
    } else {
      if (range.size() >= kMaxRangePerBatch) {
        take(r.var);
        ++it;
        continue;
      }
      item.bytes = r.len * elem_bytes(v.dtype);
      if (!v.rec.valid()) {  // nothing compressed yet: fails at once
        complete(item, NUMARCK_EINVAL, 0u, 0, now_us(), now_us());
        --v.queued;
        it = pending.erase(it);
        cv_done.notify_all();
        continue;
      }
      const uint64_t off = arena.alloc(range_ws_bytes(r.len));
      if (off == Arena::kFail) {
        starved = true;
        take(r.var);
        ++it;
        continue;
      }
      item.ws_off = off;
      range.push_back(item);
    }
    take(r.var);
    ++it;
  }

  // one workspace block for the compressions; shed the newest until it fits
  uint64_t ws_off = Arena::kFail;
  std::vector<numarck_job> jobs;
  while (!comp.empty()) {
    jobs.clear();
    for (const Item& c : comp) {
      const Variable& v = vars[c.var];
      numarck_job j{};
      j.prev = v.ref;
      j.curr = c.curr;
      j.n = v.n;
      j.dtype = v.dtype;
      j.E = v.E;
      j.B = v.B;
      j.block_bytes = v.bb;
      j.out = c.rec.out;
      j.tail_cap = c.full_tail ? 0 : v.tail_small;
      jobs.push_back(j);
    }
    ws_off = arena.alloc(numarck_batch_workspace_bytes(jobs.data(), (uint32_t)jobs.size()));
    if (ws_off != Arena::kFail) break;
    starved = true;
    comp.pop_back();
  }
  if (starved) ++waits;
  if (comp.empty() && range.empty()) return false;

  // dequeue what runs (and collect the events its inputs wait for)
  std::vector<hipEvent_t> ready;
  for (const Item& c : comp) {
    if (pending[c.ticket].r.ready) ready.push_back(static_cast<hipEvent_t>(pending[c.ticket].r.ready));
    pending.erase(c.ticket);
    vars[c.var].busy = true;
    --vars[c.var].queued;
  }
  for (const Item& r : range) {
    vars[r.var].busy = true;
    --vars[r.var].queued;
  }
  std::vector<numarck_request> rreq;
  for (const Item& r : range) {
    if (pending[r.ticket].r.ready) ready.push_back(static_cast<hipEvent_t>(pending[r.ticket].r.ready));
    rreq.push_back(pending[r.ticket].r);
    pending.erase(r.ticket);
  }

  Slot& s = *slot;
  s.busy = true;
  s.serial = ++batches;
  s.start_us = now_us();
  s.ws_off = ws_off;
  s.comp = comp;
  s.range = range;
  if (comp.size() + range.size() > max_batch_seen) max_batch_seen = comp.size() + range.size();
  numarck_status st = NUMARCK_OK;
  for (const hipEvent_t ev : ready)
    if (st == NUMARCK_OK && hipStreamWaitEvent(s.stream, ev, 0) != hipSuccess) st = NUMARCK_EHIP;
  if (!comp.empty() && st == NUMARCK_OK) {
    st = numarck_plan_create(jobs.data(), (uint32_t)jobs.size(), nullptr, at(ws_off),
                             numarck_batch_workspace_bytes(jobs.data(), (uint32_t)jobs.size()),
                             s.stream, &s.plan);
    if (st == NUMARCK_OK) st = numarck_plan_run(s.plan, s.stream);
    for (size_t i = 0; i < comp.size() && st == NUMARCK_OK; ++i)
      if (hipMemcpyAsync(&s.pin_hdr[i], comp[i].rec.out.hdr, sizeof(numarck_header),
                         hipMemcpyDeviceToHost, s.stream) != hipSuccess)
        st = NUMARCK_EHIP;
  }
  for (size_t i = 0; i < range.size() && st == NUMARCK_OK; ++i) {
    const Item& it = range[i];
    const Variable& v = vars[it.var];
    const numarck_request& r = rreq[i];
    char* w = at(it.ws_off);
    uint32_t* fl = reinterpret_cast<uint32_t*>(w);
    const size_t wsb = numarck_decompress_workspace_bytes(r.len);
    if (hipMemsetAsync(fl, 0, 4, s.stream) != hipSuccess) st = NUMARCK_EHIP;
    if (st == NUMARCK_OK)
      st = numarck_decompress_range(&v.rec.hdr, v.rec.ref, v.rec.out.packed, v.rec.out.centers,
                                    v.rec.out.incomp, v.rec.out.block_inc_off, r.start, r.len,
                                    r.out, fl, w + 256, wsb, s.stream);
    if (st == NUMARCK_OK && hipMemcpyAsync(&s.pin_flags[i], fl, 4, hipMemcpyDeviceToHost,
                                           s.stream) != hipSuccess)
      st = NUMARCK_EHIP;
  }
  if (st == NUMARCK_OK && hipEventRecord(s.done, s.stream) != hipSuccess) st = NUMARCK_EHIP;
  if (st != NUMARCK_OK) {
    // nothing usable was produced: wait for what was queued, then fail the batch
    (void)hipStreamSynchronize(s.stream);
    const double t = now_us();
    for (Item& c : s.comp) {
      vars[c.var].busy = false;
      complete(c, st, 0u, s.serial, s.start_us, t);
    }
    for (Item& r : s.range) {
      arena.release(r.ws_off);
      vars[r.var].busy = false;
      complete(r, st, 0u, s.serial, s.start_us, t);
    }
    if (s.plan) numarck_plan_destroy(s.plan);
    s.plan = nullptr;
    if (s.ws_off != Arena::kFail) arena.release(s.ws_off);
    s.ws_off = Arena::kFail;
    s.comp.clear();
    s.range.clear();
    s.busy = false;
    cv_done.notify_all();
  }
  return true;
}

void numarck_server::loop() {
  (void)hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool inflight = false;
    for (const Slot& s : slots) inflight |= s.busy;
    if (stop && !inflight && pending.empty()) break;
    bool progressed = retire();
    progressed |= launch();
    if (progressed) continue;
    inflight = false;
    for (const Slot& s : slots) inflight |= s.busy;
    if (!inflight && !pending.empty()) {
      // Nothing runs and nothing could be admitted: the oldest request can
      // never fit (the arena is whole again).  Fail it rather than wait.
      auto it = pending.begin();
      Item item{};
      item.ticket = it->first;
      item.var = it->second.r.var;
      item.kind = it->second.r.kind;
      item.submit_us = it->second.submit_us;
      --vars[item.var].queued;
      pending.erase(it);
      complete(item, NUMARCK_ECAPACITY, 0u, 0, now_us(), now_us());
      cv_done.notify_all();
      continue;
    }
    if (inflight) {  // poll the events again shortly
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      cv_work.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

extern "C" {

numarck_status numarck_server_create(const numarck_server_config* cfg, numarck_server** out) {
  if (!cfg || !out) return NUMARCK_EINVAL;
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > kMaxSlots || cfg->max_batch < 1 ||
      cfg->max_batch > NUMARCK_MAX_JOBS || cfg->arena_bytes < 4096)
    return NUMARCK_EINVAL;
  if (cfg->arena_bytes > cfg->budget_bytes) return NUMARCK_ECAPACITY;
  numarck_server* s = new numarck_server();
  s->cfg = *cfg;
  hipError_t e = hipSetDevice(cfg->device);
  if (e == hipSuccess) e = hipMalloc(&s->base, cfg->arena_bytes);
  if (e == hipSuccess) s->arena.reset(cfg->arena_bytes);
  s->slots.resize(cfg->slots);
  for (Slot& sl : s->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.pin_hdr),
                        sizeof(numarck_header) * cfg->max_batch, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.pin_flags), 4 * kMaxRangePerBatch,
                        hipHostMallocDefault);
  }
  if (e != hipSuccess) {
    for (Slot& sl : s->slots) {
      if (sl.pin_hdr) (void)hipHostFree(sl.pin_hdr);
      if (sl.pin_flags) (void)hipHostFree(sl.pin_flags);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->base) (void)hipFree(s->base);
    delete s;
    return NUMARCK_EHIP;
  }
  s->thr = std::thread([s] { s->loop(); });
  *out = s;
  return NUMARCK_OK;
}

numarck_status numarck_server_add_variable(numarck_server* s, uint64_t n, numarck_dtype dtype,
                                           double E, uint32_t B, uint64_t block_bytes,
                                           const void* initial, uint32_t* var_id) {
  if (!s || !var_id) return NUMARCK_EINVAL;
  if (dtype != NUMARCK_F32 && dtype != NUMARCK_F64) return NUMARCK_EDTYPE;
  if (B < 1 || B > 16) return NUMARCK_EBITS;
  if (!(E > 0.0 && E <= 1.0)) return NUMARCK_EBOUND;
  if (n >= ((uint64_t)1 << 32) || (n > 0 && !initial)) return NUMARCK_EINVAL;
  if (((uintptr_t)initial & 15u) != 0) return NUMARCK_EALIGN;
  if (block_bytes == 0) block_bytes = (uint64_t)1 << 20;
  if (8 * block_bytes < B) return NUMARCK_EINVAL;
  Variable v{};
  v.n = n;
  v.dtype = dtype;
  v.E = E;
  v.B = B;
  v.bb = block_bytes;
  v.ref = initial;
  v.rl = record_layout(n, dtype, B, block_bytes);
  // first attempts use a bounded tail; a retry needs the full capacity
  const uint64_t small = n / 16 > ((uint64_t)1 << 20) ? n / 16 : ((uint64_t)1 << 20);
  v.tail_small = small < n ? small : n;
  numarck_job j{};
  j.n = n;
  j.dtype = dtype;
  j.B = B;
  const uint64_t slice = numarck_batch_workspace_bytes(&j, 1);  // tail_cap 0: full
  const uint64_t rws = range_ws_bytes(n);
  v.need = slice > rws ? slice : rws;
  std::lock_guard<std::mutex> lk(s->mu);
  // two caller snapshots of the variable stay in device memory: the latest
  // record's reference and the next compression's previous snapshot
  const uint64_t res = 2 * n * elem_bytes(dtype);
  if (s->resident + res + s->cfg.arena_bytes > s->cfg.budget_bytes) return NUMARCK_ECAPACITY;
  // two record blocks for good (latest + next), from the top of the arena;
  // what stays below must still take any one request's workspace
  uint64_t need = v.need;
  for (const Variable& o : s->vars) need = o.need > need ? o.need : need;
  const uint64_t r0 = s->arena.alloc_top(v.rl.total);
  const uint64_t r1 = r0 == Arena::kFail ? Arena::kFail : s->arena.alloc_top(v.rl.total);
  if (r1 == Arena::kFail || s->arena.capacity() - s->permanent - 2 * a256(v.rl.total) < need) {
    if (r0 != Arena::kFail) s->arena.release(r0);
    if (r1 != Arena::kFail) s->arena.release(r1);
    return NUMARCK_ECAPACITY;
  }
  v.rec_off[0] = r0;
  v.rec_off[1] = r1;
  s->permanent += 2 * a256(v.rl.total);
  s->resident += res;
  *var_id = (uint32_t)s->vars.size();
  s->vars.push_back(v);
  return NUMARCK_OK;
}

numarck_status numarck_server_submit(numarck_server* s, const numarck_request* r,
                                     uint64_t* ticket) {
  if (!s || !r) return NUMARCK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return NUMARCK_EINVAL;
  if (r->var >= s->vars.size()) return NUMARCK_EINVAL;
  const Variable& v = s->vars[r->var];
  if (r->kind == NUMARCK_REQ_COMPRESS) {
    if (v.n > 0 && !r->curr) return NUMARCK_EINVAL;
    if (((uintptr_t)r->curr & 15u) != 0) return NUMARCK_EALIGN;
  } else if (r->kind == NUMARCK_REQ_RANGE) {
    if (r->start > v.n || r->len > v.n - r->start) return NUMARCK_ERANGE;
    if (r->len > 0 && !r->out) return NUMARCK_EINVAL;
    if (((uintptr_t)r->out & 15u) != 0) return NUMARCK_EALIGN;
  } else {
    return NUMARCK_EINVAL;
  }
  const uint64_t t = s->next_ticket++;
  s->pending[t] = Pending{*r, s->now_us(), false};
  ++s->vars[r->var].queued;
  ++s->submitted;
  if (ticket) *ticket = t;
  s->cv_work.notify_one();
  return NUMARCK_OK;
}

uint32_t numarck_server_poll(numarck_server* s, numarck_completion* out, uint32_t cap) {
  if (!s || !out) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  uint32_t k = 0;
  while (k < cap && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  return k;
}

numarck_status numarck_server_drain(numarck_server* s) {
  if (!s) return NUMARCK_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [s] { return s->completed == s->submitted; });
  return NUMARCK_OK;
}

numarck_status numarck_server_fetch(numarck_server* s, uint32_t var, const numarck_out* dst,
                                    void* stream) {
  if (!s || !dst) return NUMARCK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (var >= s->vars.size()) return NUMARCK_EINVAL;
  const Variable& v = s->vars[var];
  if (!v.rec.valid() || v.busy || v.queued) return NUMARCK_EINVAL;
  if (!dst->hdr || !dst->centers || (v.n > 0 && (!dst->packed || !dst->incomp ||
                                                 !dst->block_inc_off)))
    return NUMARCK_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const numarck_header& h = v.rec.hdr;
  const uint64_t L = elem_bytes(v.dtype);
  hipError_t e = hipMemcpyAsync(dst->hdr, v.rec.out.hdr, sizeof(numarck_header),
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && h.packed_bytes)
    e = hipMemcpyAsync(dst->packed, v.rec.out.packed, h.packed_bytes, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst->centers, v.rec.out.centers, numarck_centers_bytes(v.B, v.dtype),
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && h.n_inc)
    e = hipMemcpyAsync(dst->incomp, v.rec.out.incomp, h.n_inc * L, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && h.n_blocks)
    e = hipMemcpyAsync(dst->block_inc_off, v.rec.out.block_inc_off, h.n_blocks * 8,
                       hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? NUMARCK_OK : NUMARCK_EHIP;
}

numarck_status numarck_server_get_stats(numarck_server* s, numarck_server_stats* st) {
  if (!s || !st) return NUMARCK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->batches = s->batches;
  st->max_batch_seen = s->max_batch_seen;
  st->arena_capacity = s->arena.capacity();
  st->arena_peak = s->arena.peak();
  st->resident_bytes = s->resident;
  st->waits_for_memory = s->waits;
  st->tail_retries = s->tail_retries;
  return NUMARCK_OK;
}

void numarck_server_destroy(numarck_server* s) {
  if (!s) return;
  (void)numarck_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_one();
  if (s->thr.joinable()) s->thr.join();
  for (Slot& sl : s->slots) {
    (void)hipStreamSynchronize(sl.stream);
    if (sl.pin_hdr) (void)hipHostFree(sl.pin_hdr);
    if (sl.pin_flags) (void)hipHostFree(sl.pin_flags);
    (void)hipEventDestroy(sl.done);
    (void)hipStreamDestroy(sl.stream);
  }
  (void)hipFree(s->base);
  delete s;
}

}  // extern "C"
