// Serving: continuous batching of filter requests over prepared handles.
//
// Each registered handle gets a worker thread, its own HIP stream and its
// own tile of R slots of the batched CG engine, so solves on different
// meshes run concurrently on the device. A request (one field, several
// scales) becomes one column per scale. Columns enter the tile between CG
// iterations as slots free up, and leave it as they converge; a request is
// admitted when its device footprint fits the server's memory budget. A
// column's arithmetic does not depend on its tile neighbours, its slot or
// its start time, so a result is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "internal.h"

using namespace ifl;
using Clock = std::chrono::steady_clock;

struct ifl_ticket {
  std::mutex mu;
  std::condition_variable cv;
  bool done = false;
  ifl_status status = IFL_OK;
  std::string error;
  int32_t mesh_id = 0;
  int32_t n_scales = 0;
  std::vector<double> k;
  const double* field = nullptr;  // caller's host field (borrowed until ifl_wait)
  double* out = nullptr;          // caller's host buffer, n_scales x L (NULL: energies only)
  std::vector<ifl_solve_stats> stats;
  int remaining = 0;
  size_t footprint = 0;
  double* dev_field = nullptr;
  Clock::time_point t_submit, t_done;
};

namespace {

struct Column {
  ifl_ticket* t;
  int scale;
};

struct Worker {
  ifl_server* srv = nullptr;
  Handle* h = nullptr;
  int id = 0;
  int R = 0;
  hipStream_t stream = nullptr;
  BatchWork w;
  BatchMatrix bm;
  double* col_out = nullptr;  // R x L device staging of finished columns
  double* stage = nullptr;    // L doubles: a request's field on its way to row order
  int64_t L = 0;
  std::deque<ifl_ticket*> queue;  // submitted, not yet admitted (guarded by srv->mu)
  std::deque<Column> pending;     // admitted columns waiting for a slot (worker only)
  std::vector<Column> slot;       // column in each slot
  std::vector<Clock::time_point> t_in;
  std::vector<double*> field_pool;  // device field buffers (row order, n_pad) for reuse (worker only)
  std::thread th;
  // set (under srv->mu) when the worker stopped on an error: submits to its
  // mesh then fail with this status instead of queueing to nobody
  bool dead = false;
  ifl_status exit_status = IFL_OK;
  std::string exit_msg;
  // set by ifl_server_cancel: the worker fails its admitted columns that
  // have not entered a slot at the top of its next loop
  std::atomic<bool> cancel{false};
  // the handle solves with IFL_SOLVER_SHIFTED (order >= 2): columns one at a
  // time through the shifted first-order solves, no tile
  bool shifted = false;
  // order 2 with IFL_SOLVER_SHIFTED in a complex tile (2 real slots per
  // column: real and imaginary parts) over the first-order operator
  bool cx = false;
  double* zero_rows = nullptr;  // n_pad zeros: the imaginary part of a field
};

}  // namespace

struct ifl_server {
  size_t budget = 0;
  size_t tiles = 0;  // work space of the registered tiles (guarded by mu)
  size_t used = 0;   // device memory of admitted requests (guarded by mu)
  // counters for ifl_server_query (guarded by mu)
  size_t peak_used = 0;
  int64_t in_flight = 0, peak_in_flight = 0;
  int64_t submitted = 0, admitted = 0, completed = 0;
  int slots = 32;
  int device = 0;
  std::vector<std::unique_ptr<Worker>> workers;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
};

namespace {

void finish_ticket(ifl_ticket* t, ifl_status st, const std::string& msg) {
  std::lock_guard<std::mutex> lk(t->mu);
  if (st != IFL_OK && t->status == IFL_OK) {
    t->status = st;
    t->error = msg;
  }
  t->done = true;
  t->t_done = Clock::now();
  t->cv.notify_all();
}

// Admit queued requests of this worker whose footprint fits the budget
// (oldest first; a request that does not fit blocks the ones behind it so
// that large requests are not starved), while fewer than 2 R of the
// worker's admitted columns wait for a slot: a mesh whose columns run slowly
// does not take the whole budget for requests it cannot start yet.
void admit(Worker* wk, std::vector<ifl_ticket*>* admitted) {
  ifl_server* s = wk->srv;
  std::lock_guard<std::mutex> lk(s->mu);
  size_t waiting = wk->pending.size();
  while (!wk->queue.empty() && waiting < 2 * (size_t)wk->R) {
    ifl_ticket* t = wk->queue.front();
    // one request is always admitted when none is in flight, so a request
    // larger than the budget still runs (alone)
    if (s->tiles + s->used + t->footprint > s->budget && s->used > 0) break;
    s->used += t->footprint;
    s->peak_used = std::max(s->peak_used, s->used);
    s->admitted += 1;
    s->in_flight += 1;
    s->peak_in_flight = std::max(s->peak_in_flight, s->in_flight);
    wk->queue.pop_front();
    admitted->push_back(t);
    waiting += (size_t)t->n_scales;
  }
}

// Device field buffers are pooled per worker: hipFree would synchronise the
// whole device and stall the other meshes' streams.
void release_ticket(Worker* wk, ifl_ticket* t) {
  if (t->dev_field) wk->field_pool.push_back(t->dev_field);
  t->dev_field = nullptr;
  {
    std::lock_guard<std::mutex> lk(wk->srv->mu);
    wk->srv->used -= t->footprint;
    wk->srv->in_flight -= 1;
    wk->srv->completed += 1;
  }
  wk->srv->cv.notify_all();
}

// After ifl_server_cancel: the admitted columns that wait for a slot end
// with IFL_ECANCELED (their requests finish once no column is left running).
void cancel_pending(Worker* wk) {
  if (!wk->cancel.exchange(false)) return;
  for (const Column& c : wk->pending) {
    ifl_ticket* t = c.t;
    t->stats[c.scale].status = IFL_ECANCELED;
    if (--t->remaining == 0) {
      release_ticket(wk, t);
      finish_ticket(t, IFL_ECANCELED, "request cancelled by ifl_server_cancel");
    } else {
      std::lock_guard<std::mutex> lk(t->mu);
      if (t->status == IFL_OK) {
        t->status = IFL_ECANCELED;
        t->error = "request cancelled by ifl_server_cancel";
      }
    }
  }
  wk->pending.clear();
}

// Admit queued requests that fit the budget, stage each field on the device
// in row order (checked for NaN / Inf there), and queue its columns.
void stage_admitted(Worker* wk) {
  std::vector<ifl_ticket*> adm;
  admit(wk, &adm);
  for (ifl_ticket* t : adm) {
    if (!wk->field_pool.empty()) {
      t->dev_field = wk->field_pool.back();
      wk->field_pool.pop_back();
    } else if (hipMalloc((void**)&t->dev_field, sizeof(double) * wk->bm.n_pad) != hipSuccess) {
      t->dev_field = nullptr;
    }
    // the field goes through the staging buffer into row order (stream order
    // keeps the staging buffer's reuse safe); the permutation raises the
    // device flag on a NaN or Inf at a wet entry
    bool bad = false;
    if (!t->dev_field || batch_clear_flag(wk->w, wk->stream) != IFL_OK ||
        hipMemcpyAsync(wk->stage, t->field, sizeof(double) * wk->L, hipMemcpyHostToDevice, wk->stream) !=
            hipSuccess ||
        batch_permute_fields(wk->bm, wk->stage, wk->L, 1, t->dev_field, wk->w.flag, wk->stream) != IFL_OK ||
        batch_check_flag(wk->w, wk->stream, &bad) != IFL_OK) {
      (void)hipGetLastError();
      release_ticket(wk, t);
      finish_ticket(t, IFL_ENOMEM, "device allocation or copy for the request failed");
      continue;
    }
    if (bad) {
      release_ticket(wk, t);
      finish_ticket(t, IFL_EINVAL, "field has a NaN or Inf at a wet entry");
      continue;
    }
    for (int j = 0; j < t->n_scales; ++j) wk->pending.push_back({t, j});
  }
}

// Complete a request whose last column is done.
void complete_ticket(Worker* wk, ifl_ticket* t) {
  bool all_ok = true, cancelled = false;
  for (const auto& x : t->stats) {
    all_ok &= x.status == IFL_OK;
    cancelled |= x.status == IFL_ECANCELED;
  }
  release_ticket(wk, t);
  if (cancelled) finish_ticket(t, IFL_ECANCELED, "request cancelled by ifl_server_cancel");
  else finish_ticket(t, all_ok ? IFL_OK : IFL_ENOTCONV, all_ok ? "" : "a column did not converge");
}

ifl_status run_worker(Worker* wk) {
  Handle* h = wk->h;
  const int R = wk->R;
  const double rtol = h->opt.rtol;
  BatchParams prm;
  prm.max_iter = h->opt.max_iter;
  prm.graphs = h->opt.graphs != 0;
  const int chunk = wk->w.chunk;
  int active = 0;
  for (;;) {
    // 0. cancellation: admitted columns still waiting for a slot end here
    cancel_pending(wk);
    // 1. admit and stage new requests
    stage_admitted(wk);
    // 2. fill free slots
    uint64_t mask = 0;
    SlotScales cs{};
    const double* src[64] = {};
    // a column takes one slot, or in a complex tile the pair (j, j + 1)
    const int step = wk->cx ? 2 : 1;
    for (int j = 0; j < R && !wk->pending.empty(); j += step) {
      if (wk->slot[j].t) continue;
      const Column col = wk->pending.front();
      wk->pending.pop_front();
      src[j] = col.t->dev_field;
      if (wk->cx) {
        src[j + 1] = wk->zero_rows;
        cx_shift(h, col.t->k[col.scale], &cs.c[j], &cs.c[j + 1]);
        mask |= 3ull << j;
      } else {
        cs.c[j] = h->opt.gamma / std::pow(col.t->k[col.scale], 2.0 * h->op.order);
        mask |= 1ull << j;
      }
      wk->slot[j] = col;
      wk->t_in[j] = Clock::now();
      ++active;
    }
    if (mask) {
      ifl_status st = batch_load_columns(wk->bm, wk->w, mask, src, true, wk->stream);
      if (st == IFL_OK) st = batch_init(wk->bm, wk->w, mask, cs, rtol, wk->stream);
      if (st != IFL_OK) return st;
    }
    if (active == 0) {
      // nothing to run: wait for a submit, a release of memory elsewhere or
      // a cancel (a queued request that does not fit yet must not spin)
      std::unique_lock<std::mutex> lk(wk->srv->mu);
      if (wk->srv->stop && wk->queue.empty()) return IFL_OK;
      wk->srv->cv.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    // 3. iterate
    ifl_status st = batch_iterate(wk->bm, wk->w, chunk, prm, wk->stream);
    if (st != IFL_OK) return st;
    if ((st = batch_read_slots(wk->w, wk->stream)) != IFL_OK) return st;
    // 4. retire finished columns
    uint64_t fin = 0;
    std::vector<double*> dst(R, nullptr);
    for (int j = 0; j < R; j += step) {
      if (!wk->slot[j].t || wk->w.slots_host[j].done == 0) continue;
      fin |= (wk->cx ? 3ull : 1ull) << j;
      if (wk->slot[j].t->out) dst[j] = wk->col_out + (int64_t)j * wk->L;
    }
    if (!fin) continue;
    if ((st = batch_finish(wk->bm, wk->w, fin, dst.data(), wk->stream)) != IFL_OK) return st;
    if ((st = batch_read_slots(wk->w, wk->stream)) != IFL_OK) return st;
    const auto now = Clock::now();
    for (int j = 0; j < R; j += step) {
      if (!((fin >> j) & 1ull)) continue;
      const Column col = wk->slot[j];
      ifl_ticket* t = col.t;
      const BSlot& sl = wk->w.slots_host[j];
      if (t->out && (hipMemcpyAsync(t->out + (int64_t)col.scale * wk->L, dst[j], sizeof(double) * wk->L,
                                    hipMemcpyDeviceToHost, wk->stream) != hipSuccess ||
                     hipStreamSynchronize(wk->stream) != hipSuccess))
        return fail(IFL_EDEVICE, "copy of a finished column failed");
      ifl_solve_stats& so = t->stats[col.scale];
      so.iterations = sl.iters;
      so.refinements = sl.updates;
      so.status = sl.done == 1 ? IFL_OK : IFL_ENOTCONV;
      so.reserved = 0;
      so.rel_residual = sl.bb > 0 ? std::sqrt(sl.res2 / sl.bb) : std::sqrt(sl.res2);
      so.seconds = std::chrono::duration<double>(now - wk->t_in[j]).count();
      so.energy = 0.5 * sl.energy2 / handle_mass_sum(h);
      wk->slot[j] = Column{nullptr, 0};
      --active;
      if (--t->remaining == 0) complete_ticket(wk, t);
    }
    if ((st = batch_release(wk->w, fin, wk->stream)) != IFL_OK) return st;
  }
}

// A handle of order n >= 2 with IFL_SOLVER_SHIFTED: its requests' columns
// are solved one at a time by the shifted first-order solves (one kernel
// per COCG iteration) on the handle's stream, under the handle's lock; the
// other meshes' workers run concurrently on their own streams.
ifl_status run_worker_shifted(Worker* wk) {
  Handle* h = wk->h;
  for (;;) {
    cancel_pending(wk);
    stage_admitted(wk);
    if (wk->pending.empty()) {
      std::unique_lock<std::mutex> lk(wk->srv->mu);
      if (wk->srv->stop && wk->queue.empty()) return IFL_OK;
      wk->srv->cv.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    const Column col = wk->pending.front();
    wk->pending.pop_front();
    ifl_ticket* t = col.t;
    double* dst = t->out ? wk->col_out : nullptr;
    ifl_solve_stats so{};
    ifl_status st;
    {
      std::lock_guard<std::mutex> lk(h->mu);
      st = device_solve_shifted_rows(h, t->dev_field, t->k[col.scale], dst, &so);
    }
    if (st != IFL_OK && st != IFL_ENOTCONV) {
      wk->pending.push_front(col);
      return st;
    }
    if (t->out && (hipMemcpyAsync(t->out + (int64_t)col.scale * wk->L, dst, sizeof(double) * wk->L,
                                  hipMemcpyDeviceToHost, wk->stream) != hipSuccess ||
                   hipStreamSynchronize(wk->stream) != hipSuccess)) {
      wk->pending.push_front(col);
      return fail(IFL_EDEVICE, "copy of a finished column failed");
    }
    t->stats[col.scale] = so;
    if (--t->remaining == 0) complete_ticket(wk, t);
  }
}

void worker_main(Worker* wk) {
  (void)hipSetDevice(wk->srv->device);
  ifl_status st = wk->shifted ? run_worker_shifted(wk) : run_worker(wk);
  if (st != IFL_OK) {
    // fail everything this worker still holds, so no waiter blocks forever;
    // admitted requests (in a slot or waiting for one) give their memory
    // back first, so that other meshes' requests are not held up by it
    const std::string msg = std::string("serving worker failed: ") + ifl_last_error();
    std::vector<ifl_ticket*> held;
    for (int j = 0; j < wk->R; ++j)
      if (wk->slot[j].t) held.push_back(wk->slot[j].t);
    for (const Column& c : wk->pending) held.push_back(c.t);
    std::sort(held.begin(), held.end());
    held.erase(std::unique(held.begin(), held.end()), held.end());
    for (ifl_ticket* t : held) release_ticket(wk, t);
    for (int j = 0; j < wk->R; ++j)
      if (wk->slot[j].t) {
        ifl_ticket* t = wk->slot[j].t;
        wk->slot[j] = Column{nullptr, 0};
        if (--t->remaining == 0) finish_ticket(t, st, msg);
      }
    for (const Column& c : wk->pending)
      if (--c.t->remaining == 0) finish_ticket(c.t, st, msg);
    wk->pending.clear();
    std::lock_guard<std::mutex> lk(wk->srv->mu);
    for (ifl_ticket* t : wk->queue) finish_ticket(t, st, msg);
    wk->queue.clear();
    wk->exit_status = st;
    wk->exit_msg = msg;
    wk->dead = true;
  }
}

}  // namespace

extern "C" {

ifl_status ifl_server_create(size_t hbm_budget_bytes, int32_t slots, ifl_server** out) {
  if (!out) return fail(IFL_EINVAL, "out is NULL");
  *out = nullptr;
  if (slots < 1 || slots > 64) return fail(IFL_EINVAL, "slots must be in 1..64");
  if (hbm_budget_bytes == 0) return fail(IFL_EINVAL, "memory budget must be > 0");
  ifl_server* s = new ifl_server();
  s->budget = hbm_budget_bytes;
  int R = 1;
  while (R * 2 <= slots) R *= 2;
  s->slots = R;
  *out = s;
  return IFL_OK;
}

ifl_status ifl_server_add(ifl_server* s, ifl_handle* hh, int32_t* mesh_id) {
  if (!s || !hh || !mesh_id) return fail(IFL_EINVAL, "server / handle / mesh_id is NULL");
  Handle* h = static_cast<Handle*>(hh);
  if (!h->dev) return fail(IFL_EDEVICE, "host-only handle (device = -1)");
  std::unique_ptr<Worker> wk(new Worker());
  wk->srv = s;
  wk->h = h;
  wk->R = s->slots;
  wk->L = h->op.field_len;
  s->device = h->opt.device;
  if (hipSetDevice(h->opt.device) != hipSuccess) return fail(IFL_EDEVICE, "hipSetDevice failed");
  wk->cx = handle_cx_tiles(h);
  wk->shifted = h->opt.solver == IFL_SOLVER_SHIFTED && h->op.order >= 2 && !wk->cx;
  if (wk->cx) {
    if (s->slots > 32) return fail(IFL_EINVAL, "complex tiles of order-2 shifted handles hold at most 32 slots");
    wk->R = 2 * s->slots;
    wk->bm = handle_batch_matrix_k1(h, wk->R, h->opt.precision == IFL_MIXED);
  } else {
    wk->bm = handle_batch_matrix(h, wk->R, h->opt.precision == IFL_MIXED);
  }
  const int n_out = wk->shifted ? 1 : wk->R;  // output staging columns
  size_t work = 0;
  if (wk->shifted) {
    std::lock_guard<std::mutex> lk(h->mu);
    if (ifl_status st = device_shift_work(h, &work)) return st;
  } else {
    work = batch_bytes(wk->bm.n_pad, wk->R, h->opt.precision == IFL_MIXED, wk->bm.chunk);
    if (wk->cx) work += sizeof(double) * (size_t)wk->bm.n_pad;  // zero imaginary parts
  }
  const size_t tile = work + sizeof(double) * (size_t)(n_out + 1) * wk->L;  // + output and field staging
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->tiles + s->used + tile > s->budget)
      return fail(IFL_ENOMEM, "tile work space exceeds the server's memory budget");
    s->tiles += tile;
  }
  ifl_status st = IFL_OK;
  if (!wk->shifted) st = batch_alloc(&wk->w, wk->bm, wk->R, h->opt.precision == IFL_MIXED, wk->cx);
  else if (hipMalloc((void**)&wk->w.flag, sizeof(int)) != hipSuccess)  // only the field check's flag
    st = fail(IFL_ENOMEM, "hipMalloc of the field check flag failed");
  if (st == IFL_OK && wk->cx) {
    wk->w.cx_g = handle_cx_gnorm(h);
    if (hipMalloc((void**)&wk->zero_rows, sizeof(double) * (size_t)wk->bm.n_pad) != hipSuccess ||
        hipMemset(wk->zero_rows, 0, sizeof(double) * (size_t)wk->bm.n_pad) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
      st = fail(IFL_ENOMEM, "allocation of the zero imaginary parts failed");
  }
  if (st == IFL_OK && hipMalloc((void**)&wk->stage, sizeof(double) * (size_t)wk->L) != hipSuccess)
    st = fail(IFL_ENOMEM, "hipMalloc of the field staging failed");
  if (st == IFL_OK && hipMalloc((void**)&wk->col_out, sizeof(double) * (size_t)n_out * wk->L) != hipSuccess)
    st = fail(IFL_ENOMEM, "hipMalloc of the output staging failed");
  if (st == IFL_OK && hipStreamCreateWithFlags(&wk->stream, hipStreamNonBlocking) != hipSuccess)
    st = fail(IFL_EDEVICE, "hipStreamCreate failed");
  if (st != IFL_OK) {
    batch_free(&wk->w);
    if (wk->col_out) (void)hipFree(wk->col_out);
    if (wk->stage) (void)hipFree(wk->stage);
    if (wk->zero_rows) (void)hipFree(wk->zero_rows);
    std::lock_guard<std::mutex> lk(s->mu);
    s->tiles -= tile;
    return st;
  }
  wk->slot.assign(wk->R, Column{nullptr, 0});
  wk->t_in.resize(wk->R);
  std::lock_guard<std::mutex> lk(s->mu);
  wk->id = (int)s->workers.size();
  *mesh_id = wk->id;
  Worker* raw = wk.get();
  s->workers.push_back(std::move(wk));
  raw->th = std::thread(worker_main, raw);
  return IFL_OK;
}

ifl_status ifl_submit(ifl_server* s, int32_t mesh_id, const double* field, int32_t n_scales, const double* k,
                      double* out, ifl_ticket** ticket) {
  if (!s || !field || !k || !ticket) return fail(IFL_EINVAL, "NULL argument");
  *ticket = nullptr;
  Worker* wk = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (mesh_id < 0 || mesh_id >= (int)s->workers.size()) return fail(IFL_EINVAL, "unknown mesh id");
    wk = s->workers[mesh_id].get();
    if (s->stop) return fail(IFL_EINVAL, "server is shutting down");
  }
  if (n_scales < 1) return fail(IFL_EINVAL, "n_scales must be >= 1");
  for (int32_t j = 0; j < n_scales; ++j)
    if (!(k[j] > 0) || !std::isfinite(k[j])) return fail(IFL_EINVAL, "wavenumbers must be finite and > 0");
  const HostOperator& op = wk->h->op;
  ifl_ticket* t = new ifl_ticket();
  t->mesh_id = mesh_id;
  t->n_scales = n_scales;
  t->k.assign(k, k + n_scales);
  t->field = field;
  t->out = out;
  t->stats.assign(n_scales, ifl_solve_stats{});
  t->remaining = n_scales;
  // the request's device field, in row order (padded to whole slices)
  t->footprint = sizeof(double) * (size_t)((op.n + 63) / 64 * 64);
  t->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (wk->dead) {
      delete t;
      return fail(wk->exit_status, wk->exit_msg);
    }
    wk->queue.push_back(t);
    s->submitted += 1;
  }
  s->cv.notify_all();
  *ticket = t;
  return IFL_OK;
}

ifl_status ifl_server_cancel(ifl_server* s) {
  if (!s) return fail(IFL_EINVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& wk : s->workers) {
      for (ifl_ticket* t : wk->queue) finish_ticket(t, IFL_ECANCELED, "request cancelled by ifl_server_cancel");
      s->completed += (int64_t)wk->queue.size();
      wk->queue.clear();
      wk->cancel.store(true);
    }
  }
  s->cv.notify_all();
  return IFL_OK;
}

ifl_status ifl_server_query(ifl_server* s, ifl_server_info* info) {
  if (!s || !info) return fail(IFL_EINVAL, "server / info is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  info->budget = s->budget;
  info->tiles = s->tiles;
  info->used = s->used;
  info->peak_used = s->peak_used;
  info->submitted = s->submitted;
  info->admitted = s->admitted;
  info->completed = s->completed;
  info->in_flight = s->in_flight;
  info->peak_in_flight = s->peak_in_flight;
  int64_t queued = 0;
  for (const auto& wk : s->workers) queued += (int64_t)wk->queue.size();
  info->queued = queued;
  return IFL_OK;
}

int32_t ifl_poll(const ifl_ticket* t) {
  if (!t) return 0;
  std::lock_guard<std::mutex> lk(const_cast<ifl_ticket*>(t)->mu);
  return t->done ? 1 : 0;
}

double ifl_ticket_latency(const ifl_ticket* t) {
  if (!t) return 0.0;
  std::lock_guard<std::mutex> lk(const_cast<ifl_ticket*>(t)->mu);
  if (!t->done) return std::chrono::duration<double>(Clock::now() - t->t_submit).count();
  return std::chrono::duration<double>(t->t_done - t->t_submit).count();
}

ifl_status ifl_wait(ifl_ticket* t, ifl_solve_stats* stats) {
  if (!t) return fail(IFL_EINVAL, "ticket is NULL");
  ifl_status st;
  std::string msg;
  {
    std::unique_lock<std::mutex> lk(t->mu);
    t->cv.wait(lk, [&] { return t->done; });
    if (stats)
      for (int32_t j = 0; j < t->n_scales; ++j) stats[j] = t->stats[j];
    st = t->status;
    msg = t->error;
  }
  delete t;
  if (st != IFL_OK) return fail(st, msg);
  return IFL_OK;
}

void ifl_server_destroy(ifl_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& wk : s->workers) {
    if (wk->th.joinable()) wk->th.join();
    (void)hipSetDevice(s->device);
    if (wk->stream) (void)hipStreamSynchronize(wk->stream);
    batch_free(&wk->w);
    if (wk->col_out) (void)hipFree(wk->col_out);
    if (wk->stage) (void)hipFree(wk->stage);
    if (wk->zero_rows) (void)hipFree(wk->zero_rows);
    for (double* f : wk->field_pool) (void)hipFree(f);
    if (wk->stream) (void)hipStreamDestroy(wk->stream);
  }
  delete s;
}

}  // extern "C"
