// Request loop: continuous batching of coupled solves on one GPU.
//
// Requests are queued by sd_submit (all host inputs copied).  A scheduler
// thread admits them in arrival order when a slot is free and their device
// footprint fits the HBM budget; a preparation thread then assembles the
// system, builds the AMG hierarchies and uploads everything (matrices,
// hierarchies and Krylov state stay resident until the request retires).
// The scheduler advances every active solve through its resumable FGMRES
// state machine on the request's own stream: each step enqueues one
// hipGraph-captured Arnoldi column (or a restart) without blocking, so the
// kernels of concurrent requests overlap on the device.  Requests join and
// leave at iteration boundaries; a finished request's solution is copied to
// the host and its device memory released at once.  Every request runs its
// own deterministic kernels, so its result is bit-identical alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>

#include "sd.h"
#include "solver.h"

namespace {

enum { R_PENDING = SD_REQ_PENDING, R_RUNNING = SD_REQ_RUNNING, R_DONE = SD_REQ_DONE,
       R_FAILED = SD_REQ_FAILED };

struct Request {
  uint64_t id = 0;
  // owned copies of the host inputs
  sd_grid grid{};
  sd_physics phys{};
  sd_bcs bcs{};
  sd_forcing forcing{};
  sd_solver_opts opts{};
  std::vector<double> K, bc[9], f[3];
  // lifecycle
  int state = R_PENDING;
  int status = SD_OK;
  std::string err;
  std::atomic<bool> cancel{false};
  size_t est_bytes = 0, bytes = 0;
  std::unique_ptr<sd::HostProblem> hp;
  std::unique_ptr<sd::Solver> solver;
  double* d_x = nullptr;
  sd::SolveRun run;
  std::vector<double> x;
  int64_t N = 0;
  sd_stats stats{};
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

int64_t unknowns(const sd_grid& g, int ff_right) {
  const int64_t nux = ff_right == SD_BC_TRACTION ? g.nx : g.nx - 1;
  return nux * g.ny + 2LL * g.nx * g.ny + (int64_t)g.nx * g.ny_pm;
}

// Conservative device footprint before assembly (bytes).
size_t estimate_bytes(const sd_grid& g, int ff_right, const sd_solver_opts& o) {
  const double N = (double)unknowns(g, ff_right);
  const double nnz = 8.0 * N;
  const double tb = o.precision != SD_PRECISION_FP64 ? 4.0 : 8.0;
  double b = nnz * 12.0 * 1.2;                                  // FP64 A (SELL)
  if (o.precision == SD_PRECISION_MIXED32) b += nnz * 8.0 * 1.2;  // FP32 copy
  b += 2.5 * nnz * (4.0 + tb) * 1.2;                            // hierarchies, P, R
  b += 12.0 * N * tb;                                           // level work vectors
  if (o.schur == SD_SCHUR_CC) b += 0.25 * 2.5 * nnz * (4.0 + tb) * 1.2;  // L_p hierarchy
  const double nc = std::min(N, (double)o.coarse_max);
  b += (o.schur == SD_SCHUR_CC ? 3.0 : 2.0) * nc * nc * 8.0;    // coarse inverses
  b += (o.restart + 2.0) * N * 8.0 + o.restart * N * tb;        // basis, Z, W
  b += 4.0 * N * 8.0 + (4 << 20);                               // b, x, misc
  return (size_t)b;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct sd_server {
  sd_server_opts opts{};
  sd_allocator alloc{};            // device memory of the requests (alloc.alloc NULL: pool)
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_prep, cv_done, cv_sched;
  std::deque<Request*> pending;    // waiting for admission
  std::deque<Request*> to_prep;    // admitted: host assembly, setup, upload
  std::vector<Request*> ready;     // uploaded, not yet started
  std::vector<Request*> active;    // iterating (scheduler thread only)
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  size_t used = 0;
  int slots = 0;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread sched;
  std::vector<std::thread> prep;
  std::vector<hipStream_t> prep_streams;
  double t0 = 0.0;

  void prep_loop(hipStream_t stream);
  void sched_loop();
  void retire(Request* r, int status, const std::string& err);
};

void sd_server::retire(Request* r, int status, const std::string& err) {
  // called by the scheduler thread without the lock held
  if (r->solver) {
    if (status == SD_OK || status == SD_E_NOCONV) {
      r->x.resize((size_t)r->N);
      (void)hipMemcpyAsync(r->x.data(), r->d_x, (size_t)r->N * sizeof(double),
                           hipMemcpyDeviceToHost, r->solver->stream);
    }
    (void)hipStreamSynchronize(r->solver->stream);
  }
  r->solver.reset();
  r->d_x = nullptr;
  r->hp.reset();
  std::lock_guard<std::mutex> lk(mu);
  r->status = status;
  r->err = err;
  r->state = (status == SD_OK || status == SD_E_NOCONV) ? R_DONE : R_FAILED;
  r->t_done = now_s() - t0;
  used -= std::min(used, r->bytes);
  slots -= 1;
  cv_done.notify_all();
  cv_sched.notify_all();
}

void sd_server::prep_loop(hipStream_t prep_stream) {
  (void)hipSetDevice(opts.device);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_prep.wait(lk, [&] { return stop || !to_prep.empty(); });
      if (stop) return;
      r = to_prep.front();
      to_prep.pop_front();
    }
    int code = SD_OK;
    std::string msg;
    try {
      if (r->cancel) throw sd::Error(SD_E_INVALID, "cancelled");
      r->hp.reset(new sd::HostProblem());
      sd::assemble_host(&r->grid, &r->phys, &r->bcs, r->K.data(), &r->forcing, *r->hp);
      r->N = r->hp->L.N;
      r->solver.reset(new sd::Solver());
      r->solver->setup_host(r->hp.get(), &r->opts);
      r->solver->upload(alloc.alloc ? &alloc : nullptr, prep_stream);
      r->d_x = r->solver->mem->array<double>((size_t)r->N);
    } catch (const sd::Error& e) {
      code = e.code;
      msg = e.what();
    } catch (const std::exception& e) {
      code = SD_E_INVALID;
      msg = e.what();
    }
    std::lock_guard<std::mutex> lk(mu);
    if (code != SD_OK) {
      r->solver.reset();
      r->d_x = nullptr;
      r->hp.reset();
      r->status = code;
      r->err = msg;
      r->state = R_FAILED;
      r->t_done = now_s() - t0;
      used -= std::min(used, r->est_bytes);
      slots -= 1;
      cv_done.notify_all();
    } else {
      r->bytes = r->solver->device_bytes() + (size_t)r->N * sizeof(double);
      used = used - std::min(used, r->est_bytes) + r->bytes;
      ready.push_back(r);
    }
    cv_sched.notify_all();
  }
}

void sd_server::sched_loop() {
  (void)hipSetDevice(opts.device);
  for (;;) {
    std::vector<Request*> started;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (active.empty())
        cv_sched.wait_for(lk, std::chrono::milliseconds(50), [&] {
          return stop || !pending.empty() || !ready.empty();
        });
      if (stop) return;
      // admission in arrival order: a free slot and room in the HBM budget
      while (!pending.empty() && slots < opts.max_slots) {
        Request* r = pending.front();
        if (r->cancel) {
          pending.pop_front();
          r->state = R_FAILED;
          r->status = SD_E_INVALID;
          r->err = "cancelled";
          r->t_done = now_s() - t0;
          cv_done.notify_all();
          continue;
        }
        if (used + r->est_bytes > budget) break;
        pending.pop_front();
        used += r->est_bytes;
        slots += 1;
        to_prep.push_back(r);
        cv_prep.notify_one();
      }
      started.swap(ready);
    }
    for (Request* r : started) {
      if (r->cancel) {
        retire(r, SD_E_INVALID, "cancelled");
        continue;
      }
      r->run = sd::SolveRun();
      r->run.b = r->solver->b_dev;
      r->run.x = r->d_x;
      r->run.use_x0 = 0;
      try {
        r->solver->prec->start(*r->solver, r->run);
      } catch (const sd::Error& e) {
        retire(r, e.code, e.what());
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        r->state = R_RUNNING;
        r->t_admit = now_s() - t0;
      }
      active.push_back(r);
    }
    bool progressed = false;
    for (size_t i = 0; i < active.size();) {
      Request* r = active[i];
      int code = SD_OK;
      std::string msg;
      bool finished = false;
      try {
        if (r->cancel) {
          code = SD_E_INVALID;
          msg = "cancelled";
          finished = true;
        } else {
          progressed |= r->solver->prec->step(*r->solver, r->run, false);
          if (r->run.phase == sd::SolveRun::DONE) {
            finished = true;
            code = r->run.status;
            r->stats = r->run.out;
            if (code == SD_E_NOCONV) msg = "maximum number of iterations reached";
            if (code == SD_E_BREAKDOWN) msg = "non-finite value or zero pivot";
          }
        }
      } catch (const sd::Error& e) {
        finished = true;
        code = e.code;
        msg = e.what();
      }
      if (finished) {
        retire(r, code, msg);
        active.erase(active.begin() + (long)i);
        progressed = true;
      } else {
        ++i;
      }
    }
    if (!progressed && !active.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

extern "C" {

int sd_server_create(const sd_server_opts* opts, const sd_allocator* allocator,
                     sd_server** out) {
  if (!out) return SD_E_INVALID;
  *out = nullptr;
  if (allocator && (!allocator->alloc) != (!allocator->free)) return SD_E_INVALID;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return SD_E_DEVICE;
  }
  std::unique_ptr<sd_server> s(new sd_server());
  s->opts.hbm_budget = opts ? opts->hbm_budget : 0;
  s->opts.max_slots = (opts && opts->max_slots > 0) ? opts->max_slots : 8;
  s->opts.device = opts ? opts->device : 0;
  if (allocator && allocator->alloc) s->alloc = *allocator;
  if (s->opts.device < 0 || s->opts.device >= n) return SD_E_INVALID;
  if (hipSetDevice(s->opts.device) != hipSuccess) return SD_E_DEVICE;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return SD_E_DEVICE;
  s->budget = s->opts.hbm_budget ? s->opts.hbm_budget : (size_t)(0.8 * (double)free_b);
  // host preparation (assembly, AMG setup, upload) of several admitted
  // requests runs in parallel
  const int hw = (int)std::max(2u, std::thread::hardware_concurrency());
  const int n_prep = std::max(1, std::min({8, s->opts.max_slots, hw / 2}));
  for (int k = 0; k < n_prep; ++k) {
    hipStream_t ps = nullptr;
    if (hipStreamCreateWithFlags(&ps, hipStreamNonBlocking) != hipSuccess) return SD_E_DEVICE;
    s->prep_streams.push_back(ps);
  }
  s->t0 = now_s();
  sd_server* raw = s.get();
  for (hipStream_t ps : s->prep_streams) s->prep.emplace_back([raw, ps] { raw->prep_loop(ps); });
  s->sched = std::thread([raw] { raw->sched_loop(); });
  *out = s.release();
  return SD_OK;
}

int sd_submit(sd_server* sv, const sd_request* req, uint64_t* ticket) {
  if (!sv || !req || !ticket || !req->K) return SD_E_INVALID;
  const sd_grid& g = req->grid;
  if (g.nx < 2 || g.ny < 2 || g.ny_pm < 1) return SD_E_INVALID;
  if (g.nz != 0) return SD_E_INVALID;   // the request loop serves 2-D problems
  if (req->opts.krylov == SD_KRYLOV_BICGSTAB) return SD_E_INVALID;  // resumable driver
  std::unique_ptr<Request> r(new Request());
  r->grid = g;
  r->phys = req->phys;
  r->opts = req->opts;
  r->bcs = req->bcs;
  r->bcs.ff_left_tz = r->bcs.ff_right_tz = r->bcs.ff_top_tz = nullptr;   // 3-D only
  r->bcs.ff_back_u = r->bcs.ff_back_v = r->bcs.ff_back_n = nullptr;
  r->bcs.ff_front_u = r->bcs.ff_front_v = r->bcs.ff_front_n = nullptr;
  r->bcs.pm_back_p = r->bcs.pm_front_p = nullptr;
  const int64_t nx = g.nx, ny = g.ny, nyp = g.ny_pm;
  const int64_t npm = g.nx_pm > 0 ? g.nx_pm : nx;
  if (g.nx_pm < 0 || g.pm_i0 < 0 || g.pm_i0 + npm > nx) return SD_E_INVALID;
  r->K.assign(req->K, req->K + npm * nyp);
  const double* src[9] = {req->bcs.ff_left_n, req->bcs.ff_left_t, req->bcs.ff_right_n,
                          req->bcs.ff_right_t, req->bcs.ff_top_t, req->bcs.ff_top_n,
                          req->bcs.pm_left_p, req->bcs.pm_right_p, req->bcs.pm_bottom_p};
  const int64_t len[9] = {ny, ny + 1, ny, ny + 1, nx + 1, nx, nyp, nyp, npm};
  const double** dst[9] = {&r->bcs.ff_left_n, &r->bcs.ff_left_t, &r->bcs.ff_right_n,
                           &r->bcs.ff_right_t, &r->bcs.ff_top_t, &r->bcs.ff_top_n,
                           &r->bcs.pm_left_p, &r->bcs.pm_right_p, &r->bcs.pm_bottom_p};
  for (int k = 0; k < 9; ++k) {
    if (src[k]) {
      r->bc[k].assign(src[k], src[k] + len[k]);
      *dst[k] = r->bc[k].data();
    } else {
      *dst[k] = nullptr;
    }
  }
  r->forcing.f_w = nullptr;
  const double* fs[3] = {req->forcing.f_u, req->forcing.f_v, req->forcing.q_pm};
  const int64_t fl[3] = {ny * (nx + 1), (ny + 1) * nx, nyp * npm};
  const double** fd[3] = {&r->forcing.f_u, &r->forcing.f_v, &r->forcing.q_pm};
  for (int k = 0; k < 3; ++k) {
    if (fs[k]) {
      r->f[k].assign(fs[k], fs[k] + fl[k]);
      *fd[k] = r->f[k].data();
    } else {
      *fd[k] = nullptr;
    }
  }
  r->est_bytes = estimate_bytes(g, req->bcs.ff_right, req->opts);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (r->est_bytes > sv->budget) return SD_E_NOMEM;
  r->id = sv->next_id++;
  r->t_submit = now_s() - sv->t0;
  *ticket = r->id;
  sv->pending.push_back(r.get());
  sv->reqs[r->id] = std::move(r);
  sv->cv_sched.notify_all();
  return SD_OK;
}

static void fill_result(const Request& r, sd_result* out) {
  out->state = r.state;
  out->status = r.status;
  out->x_host = (r.state == R_DONE && !r.x.empty()) ? r.x.data() : nullptr;
  out->N = r.N;
  out->stats = r.stats;
  out->t_submit = r.t_submit;
  out->t_admit = r.t_admit;
  out->t_done = r.t_done;
}

int sd_poll(sd_server* sv, uint64_t ticket, sd_result* out) {
  if (!sv || !out) return SD_E_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return SD_E_NOTFOUND;
  fill_result(*it->second, out);
  return SD_OK;
}

int sd_wait(sd_server* sv, uint64_t ticket, double timeout_s, sd_result* out) {
  if (!sv) return SD_E_INVALID;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return SD_E_NOTFOUND;
  Request* r = it->second.get();
  const bool ok = sv->cv_done.wait_for(
      lk, std::chrono::duration<double>(timeout_s > 0 ? timeout_s : 0.0),
      [&] { return r->state == R_DONE || r->state == R_FAILED; });
  if (out) fill_result(*r, out);
  return ok ? SD_OK : SD_E_BUSY;
}

int sd_result_release(sd_server* sv, uint64_t ticket) {
  if (!sv) return SD_E_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return SD_E_NOTFOUND;
  if (it->second->state != R_DONE && it->second->state != R_FAILED) return SD_E_BUSY;
  sv->reqs.erase(it);
  return SD_OK;
}

int sd_cancel(sd_server* sv, uint64_t ticket) {
  if (!sv) return SD_E_INVALID;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return SD_E_NOTFOUND;
  it->second->cancel = true;
  sv->cv_sched.notify_all();
  return SD_OK;
}

void sd_server_destroy(sd_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_prep.notify_all();
  sv->cv_sched.notify_all();
  for (auto& t : sv->prep)
    if (t.joinable()) t.join();
  if (sv->sched.joinable()) sv->sched.join();
  (void)hipSetDevice(sv->opts.device);
  for (Request* r : sv->active) {
    if (r->solver) (void)hipStreamSynchronize(r->solver->stream);
    r->solver.reset();
    r->d_x = nullptr;
  }
  for (Request* r : sv->ready) {
    r->solver.reset();
    r->d_x = nullptr;
  }
  for (hipStream_t ps : sv->prep_streams) (void)hipStreamDestroy(ps);
  delete sv;
}

}  // extern "C"
