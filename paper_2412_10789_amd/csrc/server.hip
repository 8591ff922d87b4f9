// Query server: resident recurrence state for many queries, advanced by
// one batched Chebyshev step per launch (iteration-level batching).
//
// Slot s of the server owns column (s % bw) of tile (s / bw) in three
// tile-major matrices [n][bw] (two recurrence buffers and the estimate, the
// same layout as cp_power_batch).  The two recurrence buffers swap roles
// after every launch for all slots at once; a query admitted at a step
// boundary is initialised straight into the current roles (r~_0 into the
// buffer about to be overwritten, r~_1 into the one about to be gathered),
// so slots at different k share every launch.  A finished slot is
// finalised (y = D yacc into the caller's buffer) and its columns zeroed in
// one pass, ready for the next query.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace {

using Clock = std::chrono::steady_clock;

// An idle server with q waiting queries can run them one by one on the
// single-source path, the last one done after about q K t_s, or admit them
// all to one batched tile, all done after about K t_b (t_s, t_b: the time
// of a single-source step and of a one-tile batched step; a few queries
// sit in the first slots, whose narrow launch costs 1.3 ms on a 4M-node
// graph against 1.75 ms for a whole 32-wide tile and 0.4 ms for a
// single-source step).  One by one wins while q <= t_b / t_s: the worker
// keeps running means of both times and applies that limit.  Until both
// are measured, the limit is kDirectQueue.
constexpr size_t kDirectQueue = 3;
constexpr size_t kDirectQueueMax = 16;
constexpr double kMeanWeight = 0.125;  // weight of a new sample in the running means

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

enum TicketState { kQueued = 0, kRunning = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

struct Ticket {
  int state = kQueued;
  bool cancel_requested = false;
  cp_query q{};
  void* y = nullptr;
  cp::QueryPlan plan;  // source, coefficients, steps (top), step factor
  int32_t slot = -1;
  Clock::time_point t_submit, t_admit, t_done;
};

}  // namespace

struct cp_server {
  const cp_graph* g = nullptr;
  int32_t prec = CP_F32, bw = 32, nslots = 0, ntiles = 0;
  size_t max_queue = 0;
  hipStream_t st = nullptr;
  char* dev = nullptr;
  size_t dev_bytes = 0;
  // device layout
  size_t o_rA = 0, o_rB = 0, o_y = 0, o_hcount = 0, o_hpart = 0, o_coef = 0, o_src = 0, o_c01 = 0,
         o_rec = 0, o_fslots = 0, o_fouts = 0, o_part = 0, o_ws1 = 0;
  size_t ws1_bytes = 0;       // workspace of the single-source path (idle-server queries)
  uint64_t direct_ticket = 0; // query running on the single-source path, 0 if none
  int64_t direct = 0;         // queries run on the single-source path
  size_t direct_limit = kDirectQueue;  // longest queue an idle server runs one by one
  double mean_step_ms = 0;    // single-source path, per Chebyshev step (worker thread)
  double mean_tick_ms = 0;    // one-tile batched step launch (worker thread)
  std::vector<double> sp;  // host image of the slot parameters [kSlotParams][slots]

  std::mutex mu;
  std::condition_variable cv;       // wakes the worker
  std::condition_variable done_cv;  // wakes waiters
  bool stop = false;
  int32_t waiters = 0;  // threads inside cp_server_wait (destroy waits for them to leave)
  int32_t failed_hip = 0;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::deque<uint64_t> queue;
  std::vector<uint64_t> slot_ticket;  // 0 = free
  std::vector<int32_t> slot_k;        // current k of the slot's query
  uint64_t next_ticket = 1;
  int parity = 0;
  int64_t completed = 0, cancelled = 0, ticks = 0, narrow_ticks = 0;
  std::thread worker;

  void run();
  static void note_time(double& mean, double ms) { mean = mean > 0 ? mean + kMeanWeight * (ms - mean) : ms; }
  void update_direct_limit() {  // with mu held
    if (mean_step_ms > 0 && mean_tick_ms > 0)
      direct_limit = std::min(kDirectQueueMax, std::max<size_t>(1, (size_t)(mean_tick_ms / mean_step_ms)));
  }
};

namespace {

size_t storage_bytes(int32_t prec) { return prec == CP_F64 ? 8 : prec == CP_BF16 ? 2 : 4; }
size_t acc_bytes(int32_t prec) { return prec == CP_F64 || prec == CP_F32 ? 8 : 4; }

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

void fill_info(const Ticket& t, cp_info* info) {
  if (!info) return;
  info->K = t.plan.K;
  info->steps = t.plan.top - 1;
  info->tail = t.plan.tail;
  info->tail_bound_l1 = t.plan.tail * t.plan.L;
  info->mass = NAN;
  info->elapsed_ms = NAN;
  info->step_ms = NAN;
  info->latency_ms = t.state == kDone ? ms_between(t.t_submit, t.t_done) : NAN;
  info->wait_ms = t.state >= kRunning ? ms_between(t.t_submit, t.t_admit) : NAN;
  info->pushes = 0;
  info->arcs = 0;
  info->walks = 0;
  info->walk_steps = 0;
}

}  // namespace

void cp_server::run() {
  using namespace cp;
  const size_t nslot = (size_t)nslots;
  std::vector<double> coef_row(nslot), c01(2 * nslot);
  std::vector<int64_t> src(nslot);
  std::vector<int32_t> fin_slots;
  std::vector<void*> fin_outs;
  cp_query direct_q{};
  void* direct_y = nullptr;
  for (;;) {
    std::vector<int32_t> admitted, stepping, finishing, clearing;
    std::vector<uint64_t> fin_tickets;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        if (stop) return true;
        if (failed_hip) return false;
        if (!queue.empty() && std::find(slot_ticket.begin(), slot_ticket.end(), 0) != slot_ticket.end())
          return true;
        for (uint64_t t : slot_ticket)
          if (t) return true;
        return false;
      });
      if (stop) break;
      // an idle server with a short queue runs its oldest query on the
      // single-source path: a few queries in a batched launch would pay a
      // whole tile's gathers for a few sources
      if (!queue.empty() && queue.size() <= direct_limit &&
          std::all_of(slot_ticket.begin(), slot_ticket.end(), [](uint64_t t) { return !t; })) {
        direct_ticket = queue.front();
        queue.pop_front();
        Ticket& tk = tickets[direct_ticket];
        tk.state = kRunning;
        tk.t_admit = Clock::now();
        direct_q = tk.q;
        direct_q.flags &= CP_Q_PWMETHOD;
        direct_y = tk.y;
      }
    }
    if (direct_ticket) {
      const Clock::time_point t0 = Clock::now();
      const cp_status rc = cp_power(g, &direct_q, prec, direct_y, dev + o_ws1, ws1_bytes, st, nullptr);
      hipError_t e = rc == CP_OK ? hipStreamSynchronize(st) : (hipError_t)cp_last_hip_error();
      if (rc != CP_OK && e == hipSuccess) e = hipErrorUnknown;
      {
        std::lock_guard<std::mutex> lk(mu);
        Ticket& tk = tickets[direct_ticket];
        direct_ticket = 0;
        if (e == hipSuccess) {
          note_time(mean_step_ms, ms_between(t0, Clock::now()) / std::max(1, tk.plan.K));
          update_direct_limit();
        }
        if (e != hipSuccess) {
          failed_hip = (int32_t)e;
          for (auto& kv : tickets)
            if (kv.second.state == kQueued || kv.second.state == kRunning) kv.second.state = kFailed;
          queue.clear();
        } else {
          tk.state = tk.cancel_requested ? kCancelled : kDone;
          tk.t_done = Clock::now();
          if (tk.state == kDone) ++completed; else ++cancelled;
          ++direct;
        }
      }
      done_cv.notify_all();
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      // running queries whose cancellation was requested: clear their slots
      for (int32_t s = 0; s < nslots; ++s) {
        const uint64_t t = slot_ticket[s];
        if (t && tickets[t].cancel_requested) {
          clearing.push_back(s);
          Ticket& tk = tickets[t];
          tk.state = kCancelled;
          tk.slot = -1;
          slot_ticket[s] = 0;
          ++cancelled;
        }
      }
      // admit waiting queries into the lowest free slots
      for (int32_t s = 0; s < nslots && !queue.empty(); ++s) {
        if (slot_ticket[s]) continue;
        if (std::find(clearing.begin(), clearing.end(), s) != clearing.end()) continue;
        const uint64_t t = queue.front();
        queue.pop_front();
        Ticket& tk = tickets[t];
        tk.state = kRunning;
        tk.slot = s;
        tk.t_admit = Clock::now();
        slot_ticket[s] = t;
        slot_k[s] = 1;
        admitted.push_back(s);
      }
      std::fill(coef_row.begin(), coef_row.end(), 0.0);
      for (int32_t s = 0; s < nslots; ++s) {
        const uint64_t t = slot_ticket[s];
        if (!t) continue;
        const Ticket& tk = tickets[t];
        if (slot_k[s] < tk.plan.top) {
          stepping.push_back(s);
          coef_row[s] = tk.plan.c[slot_k[s] + 1];
        }
      }
      std::fill(src.begin(), src.end(), -1);
      for (int32_t s : admitted) {
        const Ticket& tk = tickets[slot_ticket[s]];
        src[s] = tk.plan.s_int;
        c01[s] = tk.plan.c[0];
        c01[nslot + s] = tk.plan.c[1];
        sp[s] = tk.plan.rec;
        sp[nslot + s] = tk.plan.oexp;
        sp[2 * nslot + s] = tk.plan.oscale;
      }
      // queries that finish with this launch (or right after init when K == 1)
      for (int32_t s = 0; s < nslots; ++s) {
        const uint64_t t = slot_ticket[s];
        if (!t) continue;
        const Ticket& tk = tickets[t];
        const int32_t k_after = slot_k[s] < tk.plan.top ? slot_k[s] + 1 : slot_k[s];
        if (k_after >= tk.plan.top) {
          finishing.push_back(s);
          fin_tickets.push_back(t);
        }
      }
      fin_slots.clear();
      fin_outs.clear();
      for (size_t i = 0; i < finishing.size(); ++i) {
        fin_slots.push_back(finishing[i]);
        fin_outs.push_back(tickets[fin_tickets[i]].y);
      }
      for (int32_t s : clearing) {
        fin_slots.push_back(s);
        fin_outs.push_back(nullptr);
      }
    }

    // ---- GPU work for this step boundary (no lock held)
    const Clock::time_point t0 = Clock::now();
    int32_t step_tiles = 0, lanes = 0;
    bool narrow = false;
    hipError_t e = hipSuccess;
    char* w = dev;
    void* xbuf = w + (parity ? o_rA : o_rB);  // gathered this launch (holds r~_k)
    void* zbuf = w + (parity ? o_rB : o_rA);  // r~_{k-1}, overwritten with r~_{k+1}
    auto chk = [&](hipError_t x) {
      if (e == hipSuccess && x != hipSuccess) e = x;
    };
    if (!admitted.empty()) {
      chk(launch_upload(w + o_src, src.data(), nslot * sizeof(int64_t), st));
      chk(launch_upload(w + o_c01, c01.data(), 2 * nslot * sizeof(double), st));
      chk(launch_upload(w + o_rec, sp.data(), 3 * nslot * sizeof(double), st));
      BatchInitArgs ia{g->row_ptr, g->col_idx, reinterpret_cast<const int64_t*>(w + o_src), g->n, bw, nslots,
                       zbuf, xbuf, w + o_y, reinterpret_cast<const double*>(w + o_c01)};
      chk(launch_batch_init(prec, ia, nslots, st));
    }
    if (!stepping.empty()) {
      int32_t tiles = 0;
      for (int32_t s : stepping) tiles = std::max(tiles, s / bw + 1);
      step_tiles = tiles;
      // only the first 8 or 16 slots step (admission takes the lowest free
      // slots, so a lightly loaded server keeps its queries there): a narrow
      // launch gathers that many values of each row instead of bw
      const int32_t top_slot = *std::max_element(stepping.begin(), stepping.end());
      for (int32_t l : kNarrowLanes)
        if (!lanes && l < bw && top_slot < l) lanes = l;
      narrow = lanes != 0;
      chk(launch_upload(w + o_coef, coef_row.data(), nslot * sizeof(double), st));
      BatchStepArgs sa{};
      set_batch_plan(g, sa, w + o_part);
      sa.n = g->n;
      sa.bw = bw;
      sa.ntiles = tiles;
      sa.nq_pad = nslots;
      sa.x = xbuf;
      sa.z = zbuf;
      sa.yacc = w + o_y;
      sa.coef_row = reinterpret_cast<const double*>(w + o_coef);
      sa.rec = reinterpret_cast<const double*>(w + o_rec);
      sa.hub_partial = w + o_hpart;
      sa.hub_count = reinterpret_cast<int32_t*>(w + o_hcount);
      sa.ntiles_total = ntiles;
      sa.lanes = lanes;
      chk(launch_batch_step(prec, sa, st));
    }
    if (!fin_slots.empty()) {
      chk(launch_upload(w + o_fslots, fin_slots.data(), fin_slots.size() * sizeof(int32_t), st));
      chk(launch_upload(w + o_fouts, fin_outs.data(), fin_outs.size() * sizeof(void*), st));
      const double* dsp = reinterpret_cast<const double*>(w + o_rec);
      SlotFinishArgs fa{g->row_ptr, g->perm, g->n, bw, reinterpret_cast<const int32_t*>(w + o_fslots),
                        reinterpret_cast<void* const*>(w + o_fouts), w + o_rA, w + o_rB, w + o_y,
                        dsp + nslot, dsp + 2 * nslot};
      chk(launch_slot_finish(prec, fa, (int32_t)fin_slots.size(), st));
    }
    chk(hipStreamSynchronize(st));

    {
      std::lock_guard<std::mutex> lk(mu);
      if (e != hipSuccess) {
        failed_hip = (int32_t)e;
        for (auto& kv : tickets)
          if (kv.second.state == kQueued || kv.second.state == kRunning) kv.second.state = kFailed;
        queue.clear();
        std::fill(slot_ticket.begin(), slot_ticket.end(), 0);
        done_cv.notify_all();
        continue;
      }
      if (!stepping.empty()) {
        parity ^= 1;
        ++ticks;
        narrow_ticks += narrow ? 1 : 0;
        for (int32_t s : stepping) ++slot_k[s];
      }
      if (step_tiles == 1 && admitted.empty() && fin_slots.empty()) {  // a plain one-tile step
        note_time(mean_tick_ms, ms_between(t0, Clock::now()));
        update_direct_limit();
      }
      const Clock::time_point now = Clock::now();
      for (size_t i = 0; i < finishing.size(); ++i) {
        Ticket& tk = tickets[fin_tickets[i]];
        tk.state = tk.cancel_requested ? kCancelled : kDone;
        tk.t_done = now;
        tk.slot = -1;
        slot_ticket[finishing[i]] = 0;
        if (tk.state == kDone) ++completed; else ++cancelled;
      }
    }
    done_cv.notify_all();
  }
}

using namespace cp;

extern "C" {

cp_status cp_server_create(const cp_graph* g, size_t hbm_budget_bytes, int32_t max_slots, int32_t max_queue,
                           int32_t prec, cp_server** out) {
  if (!g || !out || max_queue < 0 || max_slots < 0 || !(prec == CP_F64 || prec == CP_F32 || prec == CP_F32F || prec == CP_BF16))
    return CP_EINVAL;
  *out = nullptr;
  cp_server* s = nullptr;
  try {
    s = new cp_server();
  } catch (const std::bad_alloc&) {
    return CP_ENOMEM;
  }
  s->g = g;
  s->prec = prec;
  // one tile row is one 128-byte line per gathered node
  s->bw = prec == CP_F64 ? 16 : prec == CP_BF16 ? 64 : 32;
  const size_t per_tile = a256((size_t)g->n * s->bw * storage_bytes(prec)) * 2 +
                          a256((size_t)g->n * s->bw * acc_bytes(prec)) * (g->hot_split ? 2 : 1);
  int64_t tiles = (int64_t)(hbm_budget_bytes / per_tile);
  const int32_t cap = max_slots > 0 ? std::min(max_slots, 1024) : 1024;
  tiles = std::min<int64_t>(tiles, (cap + s->bw - 1) / s->bw);
  if (tiles < 1) {
    delete s;
    return CP_ENOMEM;
  }
  s->ntiles = (int32_t)tiles;
  s->nslots = s->ntiles * s->bw;
  s->max_queue = (size_t)max_queue;
  const size_t ns = (size_t)s->nslots;
  size_t off = 0;
  s->o_rA = off; off += a256((size_t)g->n * ns * storage_bytes(prec));
  s->o_rB = off; off += a256((size_t)g->n * ns * storage_bytes(prec));
  s->o_y = off; off += a256((size_t)g->n * ns * acc_bytes(prec));
  s->o_hcount = off; off += a256((size_t)batch_hub_rows(g) * s->ntiles * 4);
  s->o_hpart = off; off += a256((size_t)batch_hub_segments(g) * ns * 8);
  s->o_coef = off; off += a256(ns * 8);
  s->o_src = off; off += a256(ns * 8);
  s->o_c01 = off; off += a256(2 * ns * 8);
  s->o_rec = off; off += a256(kSlotParams * ns * 8);
  s->o_fslots = off; off += a256(ns * 4);
  s->o_fouts = off; off += a256(ns * 8);
  s->o_part = off;
  if (g->hot_split) off += a256((size_t)g->n * ns * acc_bytes(prec));  // partial row sums of the hot pass
  s->o_ws1 = off;
  s->ws1_bytes = single_ws_bytes(g, prec);
  off += a256(s->ws1_bytes);
  s->dev_bytes = off;
  hipError_t e = hipStreamCreate(&s->st);
  if (e != hipSuccess) { set_hip_error(e); delete s; return CP_EHIP; }
  e = hipMalloc(&s->dev, off);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(s->st);
    delete s;
    if (e == hipErrorOutOfMemory) return CP_ENOMEM;
    set_hip_error(e);
    return CP_EHIP;
  }
  e = launch_zero(s->dev, s->o_hpart, s->st);  // state buffers and hub counters start at zero
  s->sp = slot_params(s->nslots);
  if (e == hipSuccess) e = launch_upload(s->dev + s->o_rec, s->sp.data(), s->sp.size() * sizeof(double), s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) {
    set_hip_error(e);
    (void)hipFree(s->dev);
    (void)hipStreamDestroy(s->st);
    delete s;
    return CP_EHIP;
  }
  s->slot_ticket.assign(ns, 0);
  s->slot_k.assign(ns, 0);
  try {
    s->worker = std::thread([s] { s->run(); });
  } catch (...) {
    (void)hipFree(s->dev);
    (void)hipStreamDestroy(s->st);
    delete s;
    return CP_ENOMEM;
  }
  *out = s;
  return CP_OK;
}

cp_status cp_server_submit(cp_server* s, const cp_query* q, void* y_out, uint64_t* ticket) {
  if (!s || !q || !y_out || !ticket) return CP_EINVAL;
  Ticket tk;
  cp_status rc = plan_query(s->g, q, kBatchKCap, &tk.plan);
  if (rc != CP_OK) return rc;
  tk.q = *q;
  tk.y = y_out;
  tk.t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed_hip) { set_hip_error((hipError_t)s->failed_hip); return CP_EHIP; }
    // the queue holds max_queue waiting queries beyond those about to take a free slot
    // (a query on the single-source path holds one of them)
    const size_t free_slots = (size_t)std::count(s->slot_ticket.begin(), s->slot_ticket.end(), (uint64_t)0) -
                              (s->direct_ticket ? 1 : 0);
    if (s->queue.size() >= s->max_queue + free_slots) return CP_EBUSY;
    const uint64_t id = s->next_ticket++;
    s->tickets.emplace(id, std::move(tk));
    s->queue.push_back(id);
    *ticket = id;
  }
  s->cv.notify_one();
  return CP_OK;
}

static cp_status poll_locked(cp_server* s, uint64_t ticket, cp_info* info) {
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return CP_ENOTFOUND;
  const Ticket& tk = it->second;
  switch (tk.state) {
    case kDone:
      fill_info(tk, info);
      s->tickets.erase(it);
      return CP_OK;
    case kCancelled:
      s->tickets.erase(it);
      return CP_ECANCELLED;
    case kFailed:
      s->tickets.erase(it);
      set_hip_error((hipError_t)s->failed_hip);
      return CP_EHIP;
    default:
      return CP_EPENDING;
  }
}

cp_status cp_server_poll(cp_server* s, uint64_t ticket, cp_info* info) {
  if (!s) return CP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  return poll_locked(s, ticket, info);
}

cp_status cp_server_wait(cp_server* s, uint64_t ticket, int64_t timeout_ms, cp_info* info) {
  if (!s) return CP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] {
    auto it = s->tickets.find(ticket);
    return it == s->tickets.end() || it->second.state >= kDone;
  };
  ++s->waiters;
  if (timeout_ms < 0) s->done_cv.wait(lk, ready);
  else s->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  const cp_status rc = poll_locked(s, ticket, info);
  if (--s->waiters == 0 && s->stop) s->done_cv.notify_all();
  return rc;
}

cp_status cp_server_cancel(cp_server* s, uint64_t ticket) {
  if (!s) return CP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end() || it->second.state >= kDone) return CP_ENOTFOUND;
    Ticket& tk = it->second;
    if (tk.state == kQueued) {
      s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
      tk.state = kCancelled;
      ++s->cancelled;
    } else {
      tk.cancel_requested = true;
    }
  }
  s->cv.notify_one();
  s->done_cv.notify_all();
  return CP_OK;
}

cp_status cp_server_get_stats(cp_server* s, cp_server_stats* out) {
  if (!s || !out) return CP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->slots = s->nslots;
  out->active = (int64_t)std::count_if(s->slot_ticket.begin(), s->slot_ticket.end(), [](uint64_t t) { return t; }) +
                (s->direct_ticket ? 1 : 0);
  out->direct = s->direct;
  out->direct_limit = (int32_t)s->direct_limit;
  out->narrow_ticks = s->narrow_ticks;
  out->queued = (int64_t)s->queue.size();
  out->completed = s->completed;
  out->cancelled = s->cancelled;
  out->ticks = s->ticks;
  out->device_bytes = (int64_t)s->dev_bytes;
  out->tile_width = s->bw;
  out->prec = s->prec;
  out->waiters = s->waiters;
  return CP_OK;
}

cp_status cp_server_destroy(cp_server* s) {
  if (!s) return CP_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  hipError_t e = hipStreamSynchronize(s->st);
  hipError_t e2 = hipFree(s->dev);
  hipError_t e3 = hipStreamDestroy(s->st);
  {
    // cancel what is left, wake the waiters and let them leave before the
    // server is freed
    std::unique_lock<std::mutex> lk(s->mu);
    for (auto& kv : s->tickets)
      if (kv.second.state < kDone) kv.second.state = kCancelled;
    s->done_cv.notify_all();
    s->done_cv.wait(lk, [&] { return s->waiters == 0; });
  }
  delete s;
  if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    set_hip_error(e != hipSuccess ? e : e2 != hipSuccess ? e2 : e3);
    return CP_EHIP;
  }
  return CP_OK;
}

}  // extern "C"
