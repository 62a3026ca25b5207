// Request loop: continuous batching of coupled solves on one GPU.
//
// Requests are queued by sd_submit (all host inputs copied).  A scheduler
// thread admits them in arrival order when a slot is free and their device
// footprint fits the HBM budget; a preparation thread then assembles the
// system, builds the AMG hierarchies and uploads everything (matrices,
// hierarchies and Krylov state stay resident until the request retires).
// The scheduler advances every active solve through its resumable FGMRES
// state machine on the request's own stream (restart residuals, the
// least-squares update at the end of a cycle), without blocking.
//
// The Arnoldi columns of concurrent solves run in shared launches: every
// request records one column of its iteration once (copy-in of u_j, the
// preconditioner's V-cycles and block sweep on fixed buffers, copy-out into
// Z[j], the Gram-Schmidt step; the step j is read on the device), and
// requests whose recorded columns have the same kernel sequence form a group.
// A group keeps a device table with one region per slot (each member's
// kernel arguments and workgroup counts) and one hipGraph with ONE batched
// launch per kernel of the column, covering every slot; each replay advances
// every member by one column, whatever column each is at.  Requests join a
// group after their restart residual and leave it at the end of their cycle
// (their table region's workgroup counts zeroed, their stream ordered after
// the group's last replay).  A member computes exactly what its own kernels
// would (same arithmetic per row and the same reduction order), so every
// result is bit-identical alone, in a mix and to a direct sd_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
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
  // shared-launch state: the recorded column, its table region, the group
  std::vector<sd::RecordedOp> rec;
  std::vector<char> region;
  struct Group* grp = nullptr;
  int slot = -1;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

// Requests whose recorded columns have the same kernel sequence (launch
// shapes aside) share a group; see the top of this file.
constexpr int kGroupAhead = 2;        // replays enqueued beyond the completed ones

struct GroupOp {
  const void* fn = nullptr;
  int threads = 0;
  size_t lds = 0, args_size = 0;
  int args_off = 0;                   // in a slot region
  int cap = 0;                        // workgroups per slot in the graph
};

struct Member {
  Request* r = nullptr;
  uint64_t join_step = 0;             // the replay that runs its column 0
  bool active = false;                // still in the table's workgroup counts
};

struct Group {
  std::string key;
  std::vector<GroupOp> ops;
  int slots = 0;
  int stride = 0, nb_off = 0;         // slot region bytes; workgroup counts at nb_off
  char* table = nullptr;              // device, slots * stride bytes
  std::vector<Member> mem;            // per slot
  hipStream_t stream = nullptr;
  hipGraphExec_t graph = nullptr;
  bool dirty = true;                  // capture before the next replay
  uint64_t enq = 0, done = 0;         // replays enqueued / completed
  std::vector<hipEvent_t> ev;         // ring, one per replay in flight
  int members() const {
    int n = 0;
    for (const Member& m : mem) n += m.r != nullptr;
    return n;
  }
};

// The group key of a recorded column: each kernel with its block size,
// dynamic LDS and argument size.
std::string group_key(const std::vector<sd::RecordedOp>& ops) {
  std::string k;
  for (const sd::RecordedOp& o : ops) {
    const uintptr_t f = (uintptr_t)o.fn;
    const uint64_t v[4] = {(uint64_t)f, (uint64_t)o.threads, (uint64_t)o.lds,
                           (uint64_t)o.args.size()};
    k.append(reinterpret_cast<const char*>(v), sizeof(v));
  }
  return k;
}

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
  b += N * (8.0 + tb);                                          // replayed-column buffers
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
  int prep_threads = 0;   // host threads per preparation (set_host_threads)
  std::vector<hipStream_t> prep_streams;
  double t0 = 0.0;
  // groups of the shared launches (scheduler thread only)
  std::map<std::string, std::unique_ptr<Group>> groups;
  std::atomic<int64_t> n_groups{0}, n_replays{0}, n_member_columns{0};
  std::atomic<int> max_members{0};

  void prep_loop(hipStream_t stream);
  void sched_loop();
  void retire(Request* r, int status, const std::string& err);
  // shared launches (scheduler thread)
  void join_group(Request* r);
  void leave_group(Request* r, bool end_cycle, bool full);
  bool step_group(Group& g);
  void capture(Group& g);
  void destroy_groups();
};

void sd_server::capture(Group& g) {
  if (g.graph) {
    SD_HIP(hipStreamSynchronize(g.stream));
    SD_HIP(hipGraphExecDestroy(g.graph));
    g.graph = nullptr;
  }
  hipGraph_t graph = nullptr;
  SD_HIP(hipStreamBeginCapture(g.stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  for (size_t k = 0; k < g.ops.size() && err == hipSuccess; ++k) {
    const GroupOp& o = g.ops[k];
    const char* base = g.table;
    int stride = g.stride, aoff = o.args_off, noff = g.nb_off + 4 * (int)k, cap = o.cap;
    void* args[] = {&base, &stride, &aoff, &noff, &cap};
    err = hipLaunchKernel(o.fn, dim3((unsigned)(g.slots * o.cap)), dim3((unsigned)o.threads), args,
                          o.lds, g.stream);
  }
  const hipError_t e2 = hipStreamEndCapture(g.stream, &graph);
  if (err != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    throw sd::Error(SD_E_DEVICE, std::string("capturing the shared column graph: ") +
                                     hipGetErrorString(err != hipSuccess ? err : e2));
  }
  SD_HIP(hipGraphInstantiate(&g.graph, graph, nullptr, nullptr, 0));
  SD_HIP(hipGraphDestroy(graph));
  g.dirty = false;
}

void sd_server::join_group(Request* r) {
  sd::Solver& S = *r->solver;
  if (r->rec.empty()) {
    S.prec->record_column(S, r->rec);
    if (r->rec.empty()) throw sd::Error(SD_E_INVALID, "empty recorded column");
  }
  const std::string key = group_key(r->rec);
  auto it = groups.find(key);
  Group* g = nullptr;
  if (it != groups.end() && it->second->members() < it->second->slots) {
    g = it->second.get();
  } else if (it == groups.end()) {
    std::unique_ptr<Group> ng(new Group());
    ng->key = key;
    ng->slots = opts.max_slots;
    int off = 0;
    for (const sd::RecordedOp& o : r->rec) {
      GroupOp go;
      go.fn = o.fn;
      go.threads = o.threads;
      go.lds = o.lds;
      go.args_size = o.args.size();
      go.args_off = off;
      go.cap = 0;
      off += (int)((o.args.size() + 15) / 16 * 16);
      ng->ops.push_back(go);
    }
    ng->nb_off = off;
    ng->stride = (int)((off + 4 * (int)r->rec.size() + 255) / 256 * 256);
    ng->mem.resize((size_t)ng->slots);
    SD_HIP(hipStreamCreateWithFlags(&ng->stream, hipStreamNonBlocking));
    // the table (a few KiB per slot) comes from the stream-ordered pool
    void* t = nullptr;
    SD_HIP(hipMallocAsync(&t, (size_t)ng->slots * ng->stride, ng->stream));
    ng->table = static_cast<char*>(t);
    ng->ev.resize(kGroupAhead + 2);
    for (auto& e : ng->ev) SD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // empty slots: zero workgroup counts
    SD_HIP(hipMemsetAsync(ng->table, 0, (size_t)ng->slots * ng->stride, ng->stream));
    g = ng.get();
    groups[key] = std::move(ng);
    n_groups.fetch_add(1);
  } else {
    return;   // the group is full: this request joins once a slot frees
  }
  int slot = -1;
  for (int k = 0; k < g->slots; ++k)
    if (!g->mem[(size_t)k].r) {
      slot = k;
      break;
    }
  // the slot's region: each kernel's arguments, then the workgroup counts
  r->region.assign((size_t)g->stride, 0);
  for (size_t k = 0; k < g->ops.size(); ++k) {
    const sd::RecordedOp& o = r->rec[k];
    std::memcpy(r->region.data() + g->ops[k].args_off, o.args.data(), o.args.size());
    const int nb = o.nblocks;
    std::memcpy(r->region.data() + g->nb_off + 4 * k, &nb, sizeof(int));
    if (nb > g->ops[k].cap) {
      g->ops[k].cap = nb + nb / 8;   // room for members with a few more rows
      g->dirty = true;
    }
  }
  if (!r->ev_in) SD_HIP(hipEventCreateWithFlags(&r->ev_in, hipEventDisableTiming));
  if (!r->ev_out) SD_HIP(hipEventCreateWithFlags(&r->ev_out, hipEventDisableTiming));
  // the replays start after the request's restart work
  SD_HIP(hipEventRecord(r->ev_in, S.stream));
  SD_HIP(hipStreamWaitEvent(g->stream, r->ev_in, 0));
  SD_HIP(hipMemcpyAsync(g->table + (size_t)slot * g->stride, r->region.data(), (size_t)g->stride,
                        hipMemcpyHostToDevice, g->stream));
  g->mem[(size_t)slot] = Member{r, g->enq, true};
  r->grp = g;
  r->slot = slot;
  r->run.batched = true;
  r->run.j_enq = 0;
  r->run.completed = -1;
}

void sd_server::leave_group(Request* r, bool end_cycle, bool full) {
  Group* g = r->grp;
  Member& m = g->mem[(size_t)r->slot];
  if (m.active)
    SD_HIP(hipMemsetAsync(g->table + (size_t)r->slot * g->stride + g->nb_off, 0,
                          4 * g->ops.size(), g->stream));
  // the request's stream continues after every replay that included it
  SD_HIP(hipEventRecord(r->ev_out, g->stream));
  SD_HIP(hipStreamWaitEvent(r->solver->stream, r->ev_out, 0));
  m = Member{};
  r->grp = nullptr;
  r->slot = -1;
  if (end_cycle) r->solver->prec->end_cycle(*r->solver, r->run, full, r->solver->stream);
  r->run.batched = false;
}

// One scheduling round of a group: capture if needed, enqueue a replay while
// fewer than kGroupAhead + 1 are in flight, retire completed replays, and let
// members whose cycle has ended leave.  Returns whether anything happened.
bool sd_server::step_group(Group& g) {
  bool progress = false;
  // completed replays
  while (g.done < g.enq) {
    const hipError_t q = hipEventQuery(g.ev[(size_t)(g.done % g.ev.size())]);
    if (q == hipErrorNotReady) break;
    SD_HIP(q);
    ++g.done;
    progress = true;
  }
  // members whose cycle ended: a completed column's flag, or every column
  // of the cycle enqueued
  for (Member& m : g.mem) {
    if (!m.r) continue;
    Request* r = m.r;
    sd::SolveRun& R = r->run;
    const int64_t c = std::min<int64_t>((int64_t)(g.done - std::min(g.done, m.join_step)),
                                        R.j_enq);
    bool done = false;
    for (int q = 0; q < c && !done; ++q) done = r->solver->hf->cycle_done[q] != 0;
    if (done || R.j_enq >= R.m_cycle) {
      leave_group(r, true, !done);
      progress = true;
    }
  }
  bool any = false;
  for (const Member& m : g.mem) any = any || (m.r && m.active);
  if (!any || g.enq - g.done > (uint64_t)kGroupAhead) return progress;
  if (g.dirty) capture(g);
  SD_HIP(hipGraphLaunch(g.graph, g.stream));
  SD_HIP(hipEventRecord(g.ev[(size_t)(g.enq % g.ev.size())], g.stream));
  ++g.enq;
  int n_in = 0;
  for (const Member& m : g.mem) n_in += m.r && m.active;
  n_replays.fetch_add(1);
  n_member_columns.fetch_add(n_in);
  if (n_in > max_members.load()) max_members.store(n_in);
  for (Member& m : g.mem) {
    if (!m.r || !m.active) continue;
    if (++m.r->run.j_enq >= m.r->run.m_cycle) {
      // every column of its cycle is enqueued: no further replay includes it
      SD_HIP(hipMemsetAsync(g.table + (size_t)m.r->slot * g.stride + g.nb_off, 0,
                            4 * g.ops.size(), g.stream));
      m.active = false;
    }
  }
  return true;
}

void sd_server::destroy_groups() {
  for (auto& kv : groups) {
    Group& g = *kv.second;
    if (g.stream) (void)hipStreamSynchronize(g.stream);
    if (g.graph) (void)hipGraphExecDestroy(g.graph);
    for (auto e : g.ev) (void)hipEventDestroy(e);
    if (g.table) (void)hipFreeAsync(g.table, g.stream);
    if (g.stream) {
      (void)hipStreamSynchronize(g.stream);
      (void)hipStreamDestroy(g.stream);
    }
  }
  groups.clear();
}

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
  for (hipEvent_t* e : {&r->ev_in, &r->ev_out})
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  r->rec.clear();
  r->region.clear();
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
  sd::set_host_threads(prep_threads);
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
      sd::TraceRange trace("sd: request preparation");
      if (r->cancel) throw sd::Error(SD_E_INVALID, "cancelled");
      r->hp.reset(new sd::HostProblem());
      sd::assemble_host(&r->grid, &r->phys, &r->bcs, r->K.data(), &r->forcing, *r->hp);
      r->N = r->hp->L.N;
      r->solver.reset(new sd::Solver());
      r->solver->setup_host(r->hp.get(), &r->opts);
      r->solver->upload(alloc.alloc ? &alloc : nullptr, prep_stream);
      r->d_x = r->solver->mem->array<double>((size_t)r->N);
      r->solver->enable_column_replay();
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
          if (r->grp) leave_group(r, false, false);
          code = SD_E_INVALID;
          msg = "cancelled";
          finished = true;
        } else {
          progressed |= r->solver->prec->step(*r->solver, r->run, false);
          // a cycle about to start joins the shared launches of its group
          if (r->run.phase == sd::SolveRun::ITER && !r->run.batched && !r->grp) {
            join_group(r);
            progressed = true;
          }
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
        // a member that fails leaves its group first: no later replay may
        // read its buffers once retire frees them
        if (r->grp) {
          try {
            leave_group(r, false, false);
          } catch (const sd::Error&) {
            // the device failed: at least no host step touches r again
            r->grp->mem[(size_t)r->slot] = Member{};
            r->grp = nullptr;
            r->slot = -1;
          }
        }
        retire(r, code, msg);
        active.erase(active.begin() + (long)i);
        progressed = true;
      } else {
        ++i;
      }
    }
    for (auto& kv : groups) {
      try {
        progressed |= step_group(*kv.second);
      } catch (const sd::Error& e) {
        // a failed replay fails every member of the group
        Group& g = *kv.second;
        for (Member& m : g.mem) {
          if (!m.r) continue;
          Request* r = m.r;
          m = Member{};
          r->grp = nullptr;
          r->slot = -1;
          r->cancel = true;
        }
        (void)e;
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
  // each preparation's set-up steps take a share of the (at most 16) host
  // threads: eight set-ups on 16 threads each would spend a fifth of their
  // CPU time starting and joining threads
  s->prep_threads = std::max(1, std::min(16, hw) / n_prep);
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

int sd_server_batch_stats(sd_server* sv, sd_batch_stats* out) {
  if (!sv || !out) return SD_E_INVALID;
  out->groups = sv->n_groups.load();
  out->replays = sv->n_replays.load();
  out->member_columns = sv->n_member_columns.load();
  out->max_members = sv->max_members.load();
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
  // no replay may still read a request's memory when it is freed
  sv->destroy_groups();
  for (Request* r : sv->active) {
    if (r->solver) (void)hipStreamSynchronize(r->solver->stream);
    r->solver.reset();
    r->d_x = nullptr;
  }
  for (Request* r : sv->ready) {
    r->solver.reset();
    r->d_x = nullptr;
  }
  for (auto& kv : sv->reqs)
    for (hipEvent_t e : {kv.second->ev_in, kv.second->ev_out})
      if (e) (void)hipEventDestroy(e);
  for (hipStream_t ps : sv->prep_streams) (void)hipStreamDestroy(ps);
  delete sv;
}

}  // extern "C"
