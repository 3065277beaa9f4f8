// Continuous-batching engine for many steady sensitivity solves on one GPU.
//
// Requests (problem descriptor, mask, design field) queue in arrival order.
// Each lbm_batch_step admits queued requests, first come first served, while
// a slot is free and the request's workspace and fields fit in the caller's
// arena (the HBM budget).  Every admitted request is a slot and stays
// resident until collected.  Work is issued in quanta on lanes: a lane is a
// HIP stream with its own slot and tile tables; a quantum on a lane is
// `quantum` launches of the ragged-batch kernel, each advancing every slot of
// the lane's run set by one lattice step, whatever its grid size and whether
// it is in the forward or the adjoint sweep, followed by the per-slot
// residual sums.  When a lane's quantum has completed its slots are checked:
// a slot moves from the forward sweep to the adjoint sweep to the
// sensitivity when its residual criterion (or step cap) is met, exactly as a
// single solve would, and its memory returns to the arena when the caller
// has collected the result.  No arithmetic of one slot depends on another,
// nor on when or on which lane it runs, so each result is bit for bit the
// result of the same request solved alone.
//
// Policies (which slots a lane's next quantum advances):
//   ALL      one lane; every resident slot (processor sharing by steps: a
//            small request moves at the pace of the largest one beside it).
//   SRW      one lane; shortest remaining work first, filled: slots ordered
//            by an upper bound of their remaining node updates (nodes x steps
//            left to the step caps), taken greedily while the run set stays
//            within `fill` tiles of 256 nodes; the first is always taken.
//   OVERLAP  two lanes whose quanta run concurrently (default).  The latency
//            lane takes small slots (at most `fill` tiles each) in arrival
//            order, greedily up to `fill` tiles: below a few hundred tiles a
//            launch costs its fixed latency rather than its bytes, so these
//            share launches for free.  The bandwidth lane takes the oldest
//            remaining slot and, if that one is small, fills up with further
//            small ones.  A large request thus streams at nearly full HBM
//            bandwidth in arrival order while small ones progress beside it in
//            the bandwidth it leaves idle, instead of waiting behind it.
//   OVERLAP_FIFO  the lanes of OVERLAP, but the latency lane only takes small
//            slots that arrived before the oldest running slot too large for
//            it.  Every request is then slowed only by requests that arrived
//            before it (which plain arrival order would have run before it
//            in full), so the latency tail is no worse than arrival order,
//            while small requests still run beside a large one instead of
//            after it.
// A slot not in any run set keeps its state and its step count.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "lbm_internal.h"
#include "lbmadj.h"

using namespace lbmadj;

namespace {

enum SlotPhase { PH_IDLE = 0, PH_FORWARD = 1, PH_ADJOINT = 2, PH_DONE = 3, PH_FAILED = 4 };

constexpr int kLanes = 2;
// Run sets of at least this many tiles are issued as plain stream launches:
// a graph replay adds a few microseconds of dispatch per kernel, which only
// pays for itself on kernels too short to hide a launch from the host.
constexpr int kDirectTiles = 1024;
// A lone request on the OVERLAP bandwidth lane that is too large for the
// latency lane keeps the lane until it finishes (the lane takes the oldest
// request), so its quanta run up to its next residual check, at most this
// many quanta: every return to the host between quanta leaves the lane's
// stream idle for the host's turnaround, which on a 10-30 us step costs
// several per cent of a 250-step quantum.
constexpr int kSoloQuanta = 4;

struct Request {
  int64_t ticket;
  lbm_desc_t desc;
  std::vector<uint8_t> mask;
  std::vector<float> gamma;
};

struct Slot {
  bool used = false;
  int64_t ticket = -1;
  std::unique_ptr<lbm_problem> p;
  size_t off = 0, bytes = 0;
  float *gamma = nullptr, *drho = nullptr, *u = nullptr, *T = nullptr, *dJ = nullptr;
  int phase = PH_IDLE;
  int steps = 0;  // steps taken in the current phase
  int lane = -1;  // lane whose in-flight quantum holds the slot, or -1
  int fwd_steps = 0, adj_steps = 0;
  int status = LBM_OK;
  double prev[2] = {0, 0}, res[2] = {0, 0}, mon[2] = {0, 0};
  bool have_prev = false;
  int fwd_status = LBM_NOT_CONVERGED, adj_status = LBM_NOT_CONVERGED;
  double J = 0.0;
  std::string error;
};

// Host thread that issues a lane's launches.  The runtime lets only a few
// hundred launches wait on a stream and blocks the issuing thread beyond
// that, so a quantum is issued from the lane's own thread: a lane that
// blocks while its quantum drains does not hold up the other lane's
// completions and launches.
struct Worker {
  std::thread th;
  std::mutex m;
  std::condition_variable cv;
  std::function<hipError_t()> job;
  bool pending = false, quit = false;
  std::atomic<bool> posted{true};  // the last job has been issued
  std::atomic<int> err{0};
};

void worker_main(Worker* w, int dev) {
  (void)hipSetDevice(dev);
  std::unique_lock<std::mutex> lk(w->m);
  for (;;) {
    w->cv.wait(lk, [&] { return w->pending || w->quit; });
    if (w->quit) return;
    std::function<hipError_t()> job = std::move(w->job);
    w->pending = false;
    lk.unlock();
    const hipError_t e = job();
    if (e != hipSuccess) w->err.store((int)e);
    w->posted.store(true, std::memory_order_release);
    lk.lock();
  }
}

void post(Worker* w, std::function<hipError_t()> job) {
  w->posted.store(false, std::memory_order_relaxed);
  {
    std::lock_guard<std::mutex> lk(w->m);
    w->job = std::move(job);
    w->pending = true;
  }
  w->cv.notify_one();
}

// One stream with its own device tables.  The kernel's step index of a slot
// is (lane launch counter - SlotDev.start); start is set when the tables are
// uploaded, from the slot's step count and the counter at that time.  The
// counter lives on the device (d_base, advanced by the quantum itself) and is
// mirrored in `launch`.  A quantum is replayed from a HIP graph captured once
// per tile count: its launches read the tables and the counter from device
// memory, so one graph serves every quantum of that size.
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  SlotDev* d_slots = nullptr;
  Tile* d_tiles = nullptr;
  double* d_sums = nullptr;
  int* d_base = nullptr;
  unsigned* d_bar = nullptr;  // grid-barrier arrivals of a persistent quantum
  int* d_abort = nullptr;     // raised when a persistent quantum's barrier wait gives up
  double* h_sums = nullptr;  // pinned
  int* h_abort = nullptr;    // pinned copy of *d_abort after each persistent quantum
  bool persistent = false;   // the quantum in flight is a persistent launch
  std::map<int, hipGraphExec_t> graphs;  // quantum graph per tile count
  // quanta of a lone slot: the single-problem kernels, arguments by value,
  // keyed by (ticket, phase, parity of the first step, residual step at end)
  std::map<std::tuple<int64_t, int, int, int>, hipGraphExec_t> solo;
  std::unique_ptr<Worker> worker;
  std::vector<SlotDev> h_slots;
  std::vector<Tile> h_tiles;
  SlotDev* pin_slots = nullptr;  // pinned staging of the uploads
  Tile* pin_tiles = nullptr;
  std::vector<char> run;         // run set of the lane's current / next quantum
  std::vector<int64_t> up_ticket;  // ticket whose entry the device slot table holds
  bool busy = false;             // a quantum is in flight
  int qsteps = 0;                // steps of the quantum in flight
  int launch = 0;
  long long nodes = 0;    // nodes advanced per launch
};

// First-fit allocator over [0, size) of the arena, in 256-byte units.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t o = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

}  // namespace

struct lbm_batch {
  int thermal = 0, objective = 0, max_slots = 0, quantum = 0;
  int policy = LBM_BATCH_POLICY_OVERLAP;
  int fill_tiles = 512;
  int persist_tiles = 0;     // run sets of at most this many tiles run as one persistent launch
  int persist_grid = 0;      // resident blocks of the persistent kernel on the device
  int spin_limit = 1 << 21;  // polls of a grid-barrier wait before it gives up
  int dev = -1;
  char* base = nullptr;  // request arena start (aligned)
  Arena arena;
  int max_tiles = 0;     // per lane
  Lane lanes[kLanes];
  char* stage = nullptr;  // pinned staging of request uploads and results
  size_t stage_bytes = 0;
  std::vector<Slot> slots;
  std::deque<Request> queue;
  std::map<int64_t, int> slot_of;  // ticket -> slot
  int64_t next_ticket = 1;
  long long node_updates = 0;
  long long launches = 0;
};

namespace {

size_t fields_bytes(const lbm_problem* p) {
  // gamma, drho, u (3), T, dJ, each N floats, 256-byte aligned
  return 7 * align256((size_t)p->N * sizeof(float));
}

// Device table bytes of one lane.
size_t lane_table_bytes(int max_slots, int max_tiles) {
  return align256((size_t)max_slots * sizeof(SlotDev)) + align256((size_t)max_tiles * sizeof(Tile)) +
         align256((size_t)max_slots * 4 * sizeof(double)) + 256;
}

size_t request_bytes(const lbm_problem* p) { return layout_of(p).total + fields_bytes(p); }

bool two_lanes(int policy) {
  return policy == LBM_BATCH_POLICY_OVERLAP || policy == LBM_BATCH_POLICY_OVERLAP_FIFO;
}
int lanes_used(const lbm_batch* b) { return two_lanes(b->policy) ? kLanes : 1; }

bool running(const Slot& s) { return s.used && (s.phase == PH_FORWARD || s.phase == PH_ADJOINT); }

// Pinned staging of at least `bytes` (grown by doubling; the engine's
// streams are idle for the stage whenever this is called).
int ensure_stage(lbm_batch* b, size_t bytes) {
  if (bytes <= b->stage_bytes) return LBM_OK;
  size_t nb = std::max<size_t>(b->stage_bytes * 2, size_t(16) << 20);
  while (nb < bytes) nb *= 2;
  if (b->stage) HIPCHK(hipHostFree(b->stage));
  b->stage = nullptr;
  b->stage_bytes = 0;
  HIPCHK(hipHostMalloc((void**)&b->stage, nb, hipHostMallocDefault));
  b->stage_bytes = nb;
  return LBM_OK;
}

// Point the problem at its arena region and upload its node data and design.
int bind_slot(lbm_batch* b, Slot& s, const Request& r, hipStream_t st) {
  lbm_problem* p = s.p.get();
  char* base = b->base + s.off;
  const Layout L = layout_of(p);
  const bool th = thermal_of(p);
  p->ws = base;
  p->ws_bytes = L.total;
  p->dev = b->dev;
  for (int k = 0; k < 2; ++k) {
    p->f[k] = (float*)(base + L.f[k]);
    p->a[k] = (float*)(base + L.a[k]);
    p->g[k] = th ? (float*)(base + L.g[k]) : nullptr;
    p->b[k] = th ? (float*)(base + L.b[k]) : nullptr;
    p->R[k] = th ? (float*)(base + L.R[k]) : nullptr;
  }
  p->rcur = 0;
  p->gneq = th ? (float*)(base + L.gneq) : nullptr;
  p->G = (p->d.objective == LBM_OBJ_DISSIPATION) ? (float*)(base + L.G) : nullptr;
  p->uin = (float*)(base + L.uin);
  p->flags = (uint8_t*)(base + L.flags);
  p->partials = (double*)(base + L.partials);
  p->sums = (double*)(base + L.sums);
  char* fb = base + L.total;
  const size_t fs = align256((size_t)p->N * sizeof(float));
  s.gamma = (float*)(fb);
  s.drho = (float*)(fb + fs);
  s.u = (float*)(fb + 2 * fs);
  s.T = th ? (float*)(fb + 5 * fs) : nullptr;
  s.dJ = (float*)(fb + 6 * fs);
  const size_t ub = align256((size_t)p->Np * sizeof(float));
  const size_t gb = align256((size_t)p->N * sizeof(float));
  int rc = ensure_stage(b, ub + gb + (size_t)p->Np);
  if (rc) return rc;
  float* uin = (float*)b->stage;
  float* gam = (float*)(b->stage + ub);
  uint8_t* fl = (uint8_t*)(b->stage + ub + gb);
  std::fill(uin, uin + p->Np, 0.0f);
  std::copy(p->uin_host.begin(), p->uin_host.end(), uin);
  std::copy(r.gamma.begin(), r.gamma.end(), gam);
  std::fill(fl, fl + p->Np, (uint8_t)K_WALL);
  std::copy(p->flags_host.begin(), p->flags_host.end(), fl);
  HIPCHK(hipMemcpyAsync(p->uin, uin, p->Np * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->flags, fl, p->Np, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s.gamma, gam, (size_t)p->N * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(launch_fill(p->f[0], (size_t)qf_of(p) * p->Np, st));
  if (th) {
    HIPCHK(launch_fill(p->g[0], (size_t)qg_of(p) * p->Np, st));
    HIPCHK(launch_ref_init(p->R[0], p->flags, p->kp, st));
    HIPCHK(launch_heat_init(p->g[0], s.gamma, p->flags, p->kp, st));
  }
  HIPCHK(hipStreamSynchronize(st));  // the staging is reused
  return LBM_OK;
}

void release_slot(lbm_batch* b, int i) {
  Slot& s = b->slots[i];
  if (s.bytes) b->arena.release(s.off, s.bytes);
  b->slot_of.erase(s.ticket);
  s = Slot();
}

int admit(lbm_batch* b, hipStream_t st) {
  while (!b->queue.empty()) {
    int free_slot = -1;
    for (int i = 0; i < b->max_slots; ++i)
      if (!b->slots[i].used) {
        free_slot = i;
        break;
      }
    if (free_slot < 0) return LBM_OK;
    Request& r = b->queue.front();
    auto p = std::make_unique<lbm_problem>();
    int rc = validate_and_setup(p.get(), r.desc, r.mask.data());
    if (rc) return rc;  // validated at submit; cannot fail here
    size_t off = 0;
    const size_t bytes = request_bytes(p.get());
    if (!b->arena.alloc(bytes, &off)) return LBM_OK;  // wait for memory (first come, first served)
    Slot& s = b->slots[free_slot];
    s = Slot();
    s.used = true;
    s.ticket = r.ticket;
    s.p = std::move(p);
    s.off = off;
    s.bytes = bytes;
    rc = bind_slot(b, s, r, st);
    if (rc) return rc;
    s.phase = PH_FORWARD;
    s.steps = 0;
    b->slot_of[r.ticket] = free_slot;
    b->queue.pop_front();
  }
  return LBM_OK;
}

// True if the lane's device tables do not describe its run set at the
// lane's current launch counter.
bool needs_upload(const lbm_batch* b, const Lane& ln) {
  for (int i = 0; i < b->max_slots; ++i) {
    const Slot& s = b->slots[i];
    const SlotDev& d = ln.h_slots[i];
    const bool want = ln.run[i] && running(s);
    if (want != (d.phase != 0)) return true;
    if (want && (ln.up_ticket[i] != s.ticket || d.phase != s.phase ||
                 d.start != ln.launch - s.steps))
      return true;
  }
  return false;
}

// Device slot table and tile table of a lane from its run set.
int upload_tables(lbm_batch* b, Lane& ln) {
  ln.h_tiles.clear();
  ln.nodes = 0;
  for (int i = 0; i < b->max_slots; ++i) {
    Slot& s = b->slots[i];
    SlotDev& d = ln.h_slots[i];
    std::memset((void*)&d, 0, sizeof(SlotDev));
    ln.up_ticket[i] = -1;
    if (!ln.run[i] || !running(s)) continue;
    ln.up_ticket[i] = s.ticket;
    lbm_problem* p = s.p.get();
    d.phase = s.phase;
    d.start = ln.launch - s.steps;
    d.max_steps = p->d.max_steps;
    d.check = p->d.check_every;
    p->fcur = 0;
    p->acur = 0;
    p->rcur = 0;
    d.fa = fwd_args(p, s.gamma, s.drho, s.u, s.T);
    d.aa = adj_args(p, s.gamma, s.u, s.T);
    d.R1 = p->R[1];
    for (int t = 0; t < p->nblk; ++t) ln.h_tiles.push_back(Tile{i, t});
    ln.nodes += p->N;
  }
  if ((int)ln.h_tiles.size() > b->max_tiles) return fail(LBM_ENOMEM, "tile table full");
  // copies from pinned memory only: a pageable source can make the copy wait
  // for work queued on other streams
  std::memcpy((void*)ln.pin_slots, ln.h_slots.data(), b->max_slots * sizeof(SlotDev));
  std::memcpy((void*)ln.pin_tiles, ln.h_tiles.data(), ln.h_tiles.size() * sizeof(Tile));
  HIPCHK(hipMemcpyAsync(ln.d_slots, ln.pin_slots, b->max_slots * sizeof(SlotDev),
                        hipMemcpyHostToDevice, ln.stream));
  if (!ln.h_tiles.empty())
    HIPCHK(hipMemcpyAsync(ln.d_tiles, ln.pin_tiles, ln.h_tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice, ln.stream));
  HIPCHK(hipStreamSynchronize(ln.stream));  // the staging is rewritten later
  return LBM_OK;
}

// Phase bookkeeping of one slot after a quantum of its lane completed.
int after_quantum(lbm_batch* b, int i, Lane& ln) {
  Slot& s = b->slots[i];
  lbm_problem* p = s.p.get();
  hipStream_t st = ln.stream;
  const int done = s.steps;
  const int check = p->d.check_every;
  const bool at_check = check > 0 && done > 0 && done % check == 0;
  const bool at_end = done >= p->d.max_steps;
  if (!at_check && !at_end) return LBM_OK;
  const bool th = thermal_of(p);
  const double* sums = ln.h_sums + (size_t)i * 4;
  s.mon[0] = sums[0] / p->n_nonwall;
  s.mon[1] = sums[1] / p->n_nonwall;
  if (!std::isfinite(s.mon[0]) || !std::isfinite(s.mon[1])) {
    s.error = std::string(s.phase == PH_FORWARD ? "forward" : "adjoint") + " sweep diverged";
    if (s.phase == PH_FORWARD) s.fwd_steps = done;
    else s.adj_steps = done;  // adj_steps > 0 tells a failed adjoint from a failed forward
    s.phase = PH_FAILED;
    s.status = LBM_EDIVERGED;
    return LBM_OK;
  }
  bool converged = false;
  if (at_check) {
    if (s.have_prev) {
      s.res[0] = std::fabs(s.mon[0] - s.prev[0]) / std::max(std::fabs(s.mon[0]), 1e-300);
      s.res[1] = std::fabs(s.mon[1] - s.prev[1]) / std::max(std::fabs(s.mon[1]), 1e-300);
      converged = rel_converged(s.mon[0], s.prev[0], p->d.tol) &&
                  (!th || rel_converged(s.mon[1], s.prev[1], p->d.tol));
    }
    s.prev[0] = s.mon[0];
    s.prev[1] = s.mon[1];
    s.have_prev = true;
  }
  if (!converged && !at_end) return LBM_OK;
  if (s.phase == PH_FORWARD) {
    s.fwd_steps = done;
    s.fwd_status = converged ? LBM_OK : LBM_NOT_CONVERGED;
    double J = 0.0;
    if (p->d.objective == LBM_OBJ_DISSIPATION) {
      HIPCHK(launch_dissipation_objective(s.u, s.gamma, p->flags, p->partials, p->kp, st));
      HIPCHK(launch_finalize(p->partials, p->nblk, kRedDiss, p->sums, st));
      HIPCHK(hipMemcpyAsync(ln.h_sums + (size_t)i * 4, p->sums, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      J = ln.h_sums[(size_t)i * 4];
      HIPCHK(launch_dissipation_source(s.u, s.gamma, p->flags, p->G, p->kp, st));
    } else if (p->d.objective == LBM_OBJ_HEATGEN) {
      J = -sums[3];
    } else {
      if (p->n_inlet > 0) J += p->d.w_dp * (sums[2] / p->n_inlet) / 3.0;
      if (p->d.objective == LBM_OBJ_HEATSINK) J += sums[3] / p->n_layer;
    }
    s.J = J;
    HIPCHK(launch_fill(p->a[0], (size_t)qf_of(p) * p->Np, st));
    if (th) HIPCHK(launch_fill(p->b[0], (size_t)qg_of(p) * p->Np, st));
    s.phase = PH_ADJOINT;
    s.steps = 0;
    s.have_prev = false;
    s.res[0] = s.res[1] = 0.0;
  } else {
    s.adj_steps = done;
    s.adj_status = converged ? LBM_OK : LBM_NOT_CONVERGED;
    // final adjoint state is buffer (done & 1)
    p->acur = done & 1;
    SensArgs A{};
    A.ain = p->a[sens_buffer(p)];
    A.bin = p->b[p->acur];
    A.flags = p->flags;
    A.gamma = s.gamma;
    A.u = s.u;
    A.T = s.T;
    A.gneq = p->gneq;
    A.dJ = s.dJ;
    A.partials = p->partials;
    A.objective = p->d.objective;
    A.P = p->kp;
    HIPCHK(launch_sensitivity(A, th, st));
    s.phase = PH_DONE;
    s.status = (s.fwd_status == LBM_OK && s.adj_status == LBM_OK) ? LBM_OK : LBM_NOT_CONVERGED;
  }
  return LBM_OK;
}

// Run set of lane L's next quantum under the engine's policy, from the
// running slots that no in-flight quantum holds.
void choose_run_set(lbm_batch* b, int L) {
  Lane& ln = b->lanes[L];
  std::fill(ln.run.begin(), ln.run.end(), 0);
  std::vector<int> cand;
  for (int i = 0; i < b->max_slots; ++i)
    if (running(b->slots[i]) && b->slots[i].lane < 0) cand.push_back(i);
  if (cand.empty()) return;
  const int F = b->fill_tiles;
  auto nblk = [&](int i) { return b->slots[i].p->nblk; };
  auto by_ticket = [&](int x, int y) { return b->slots[x].ticket < b->slots[y].ticket; };
  // greedy fill in the given order; the first is always taken when `first`
  auto fill = [&](const std::vector<int>& order, bool first, long long tiles) {
    for (size_t k = 0; k < order.size(); ++k) {
      const int i = order[k];
      if (!(first && k == 0) && tiles + nblk(i) > F) continue;
      ln.run[i] = 1;
      tiles += nblk(i);
    }
  };
  if (b->policy == LBM_BATCH_POLICY_ALL) {
    for (int i : cand) ln.run[i] = 1;
  } else if (b->policy == LBM_BATCH_POLICY_SRW) {
    std::vector<std::pair<double, int>> w;
    for (int i : cand) {
      const Slot& s = b->slots[i];
      const int cap = s.p->d.max_steps;
      const double left = s.phase == PH_FORWARD ? double(cap - s.steps) + cap : double(cap - s.steps);
      w.push_back({left * s.p->N, i});
    }
    std::sort(w.begin(), w.end(), [&](const auto& x, const auto& y) {
      return x.first != y.first ? x.first < y.first : by_ticket(x.second, y.second);
    });
    std::vector<int> order;
    for (auto& e : w) order.push_back(e.second);
    fill(order, true, 0);
  } else if (L == 0) {  // OVERLAP, latency lane: small slots in arrival order
    // OVERLAP_FIFO: only those older than every running slot too large for
    // this lane (held by a quantum in flight or not)
    int64_t before = INT64_MAX;
    if (b->policy == LBM_BATCH_POLICY_OVERLAP_FIFO)
      for (int i = 0; i < b->max_slots; ++i)
        if (running(b->slots[i]) && nblk(i) > F) before = std::min(before, b->slots[i].ticket);
    std::vector<int> small;
    for (int i : cand)
      if (nblk(i) <= F && b->slots[i].ticket < before) small.push_back(i);
    std::sort(small.begin(), small.end(), by_ticket);
    fill(small, true, 0);
  } else {  // OVERLAP, bandwidth lane: the oldest slot, then small ones if it is small
    std::sort(cand.begin(), cand.end(), by_ticket);
    const int head = cand[0];
    ln.run[head] = 1;
    if (nblk(head) <= F) {
      std::vector<int> small;
      for (size_t k = 1; k < cand.size(); ++k)
        if (nblk(cand[k]) <= F) small.push_back(cand[k]);
      fill(small, false, nblk(head));
    }
  }
}

// Capture the stream's work issued by `issue` into an executable graph.
template <class F>
int capture(hipStream_t st, F&& issue, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const hipError_t e = issue();
  const hipError_t e2 = hipStreamEndCapture(st, &g);
  HIPCHK(e);
  HIPCHK(e2);
  const hipError_t e3 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e3);
  return LBM_OK;
}

// Quantum of lane L whose run set is the one slot i: the single-problem
// forward or adjoint kernel per step, with the buffer parity and the
// residual step exactly where a single solve has them (a residual check can
// only fall on the last step of a quantum, the check period and the step cap
// being multiples of the quantum), so a lone slot costs what a single solve
// costs per step.
int launch_solo(lbm_batch* b, int L, int i) {
  Lane& ln = b->lanes[L];
  Slot& s = b->slots[i];
  lbm_problem* p = s.p.get();
  const bool th = thermal_of(p);
  const int s0 = s.steps, cap = p->d.max_steps, chk = p->d.check_every;
  int n = std::min(b->quantum, cap - s0);
  if (two_lanes(b->policy) && L == 1 && p->nblk > b->fill_tiles &&
      p->nblk >= kDirectTiles) {
    // up to the next residual check (the check period and the step cap are
    // multiples of the quantum, so this is a whole number of quanta)
    const int to_check = chk > 0 ? chk - s0 % chk : cap - s0;
    n = std::min({to_check, cap - s0, kSoloQuanta * b->quantum});
  }
  const int last = s0 + n;
  const bool diag = (chk > 0 && last % chk == 0) || last == cap;
  // reference buffer of the thermal state during this quantum: it flips at
  // every re-base, which follows a diagnostic step, and those only end quanta
  const int rpar = chk > 0 ? (s0 / chk) & 1 : 0;
  const bool rebase = th && diag && s.phase == PH_FORWARD;
  if (p->nblk >= kDirectTiles) {
    // argument sets for even and odd steps, built here, issued by the worker
    const int phase = s.phase, obj = p->d.objective;
    FwdArgs fa[2];
    AdjArgs aa[2];
    p->rcur = rpar;
    for (int par = 0; par < 2; ++par) {
      p->fcur = par;
      p->acur = par;
      fa[par] = fwd_args(p, s.gamma, s.drho, s.u, s.T);
      aa[par] = adj_args(p, s.gamma, s.u, s.T);
    }
    p->fcur = last & 1;  // the state after the quantum's last step
    const RebaseArgs ra = rebase_args(p, s.T);
    const double* part = p->partials;
    const int nblk = p->nblk;
    hipStream_t st = ln.stream;
    hipEvent_t ev = ln.done;
    double* hs = ln.h_sums + (size_t)i * 4;
    double* ds = ln.d_sums + (size_t)i * 4;
    int* base = ln.d_base;
    post(ln.worker.get(), [=]() -> hipError_t {
      hipError_t e = hipSuccess;
      for (int q = 0; q < n && e == hipSuccess; ++q) {
        const bool dq = diag && q == n - 1;
        const int par = (s0 + q) & 1;
        e = phase == PH_FORWARD ? launch_forward(fa[par], th, dq, st)
                                : launch_adjoint(aa[par], th, obj, dq, st);
      }
      if (e == hipSuccess && rebase) e = launch_rebase(ra, st);
      if (e == hipSuccess && diag)
        e = launch_finalize(part, nblk, phase == PH_FORWARD ? kRedFwd : kRedAdj, ds, st);
      if (e == hipSuccess) e = launch_advance(base, n, st);
      if (e == hipSuccess && diag)
        e = hipMemcpyAsync(hs, ds, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipEventRecord(ev, st);
      return e;
    });
    s.lane = L;
    ln.qsteps = n;
    ln.launch += n;
    b->launches += n;
    b->node_updates += (long long)p->N * n;
    ln.busy = true;
    return LBM_OK;
  }
  const auto key = std::make_tuple(s.ticket, s.phase, s0 & 1, int(diag) | (rpar << 1));
  auto it = ln.solo.find(key);
  if (it == ln.solo.end()) {
    if (ln.solo.size() >= 8) {
      for (auto& g : ln.solo) (void)hipGraphExecDestroy(g.second);
      ln.solo.clear();
    }
    const int phase = s.phase;
    auto issue = [&]() -> hipError_t {
      hipError_t e = hipSuccess;
      for (int q = 0; q < n && e == hipSuccess; ++q) {
        const bool dq = diag && q == n - 1;
        if (phase == PH_FORWARD) {
          p->fcur = (s0 + q) & 1;
          p->rcur = rpar;
          e = launch_forward(fwd_args(p, s.gamma, s.drho, s.u, s.T), th, dq, ln.stream);
        } else {
          p->acur = (s0 + q) & 1;
          e = launch_adjoint(adj_args(p, s.gamma, s.u, s.T), th, p->d.objective, dq, ln.stream);
        }
      }
      if (e == hipSuccess && rebase) {
        p->fcur = last & 1;
        p->rcur = rpar;
        e = launch_rebase(rebase_args(p, s.T), ln.stream);
      }
      if (e == hipSuccess && diag)
        e = launch_finalize(p->partials, p->nblk, phase == PH_FORWARD ? kRedFwd : kRedAdj,
                            ln.d_sums + (size_t)i * 4, ln.stream);
      if (e == hipSuccess) e = launch_advance(ln.d_base, b->quantum, ln.stream);
      return e;
    };
    hipGraphExec_t x = nullptr;
    int rc = capture(ln.stream, issue, &x);
    if (rc) return rc;
    it = ln.solo.emplace(key, x).first;
  }
  hipGraphExec_t x = it->second;
  hipStream_t st = ln.stream;
  hipEvent_t ev = ln.done;
  double* hs = ln.h_sums + (size_t)i * 4;
  const double* ds = ln.d_sums + (size_t)i * 4;
  post(ln.worker.get(), [=]() -> hipError_t {
    hipError_t e = hipGraphLaunch(x, st);
    if (e == hipSuccess && diag)
      e = hipMemcpyAsync(hs, ds, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    return e;
  });
  s.lane = L;
  ln.qsteps = b->quantum;
  ln.launch += b->quantum;
  b->launches += n;
  b->node_updates += (long long)p->N * n;
  ln.busy = true;
  return LBM_OK;
}

// One quantum of lane L as a single persistent launch (its tables are
// uploaded): barrier counters cleared, the quantum's steps and the re-base in
// one cooperative launch, the per-slot residual sums, the launch counter, the
// copies to the host and the completion event.
int launch_persistent(lbm_batch* b, int L, int ntiles) {
  Lane& ln = b->lanes[L];
  const Tile* tiles = ln.d_tiles;
  const SlotDev* sl = ln.d_slots;
  int* base = ln.d_base;
  unsigned* bar = ln.d_bar;
  int* abort = ln.d_abort;
  int* habort = ln.h_abort;
  double* ds = ln.d_sums;
  double* hs = ln.h_sums;
  hipStream_t st = ln.stream;
  hipEvent_t ev = ln.done;
  const int Q = b->quantum, ns = b->max_slots, obj = b->objective, grid = b->persist_grid;
  const int spin = b->spin_limit;
  const bool th = b->thermal != 0;
  post(ln.worker.get(), [=]() -> hipError_t {
    // bar and abort are single words: 0.0f fills them with zero bits
    hipError_t e = launch_fill((float*)bar, 1, st);
    if (e == hipSuccess) e = launch_fill((float*)abort, 1, st);
    if (e == hipSuccess)
      e = launch_batch_persistent(tiles, ntiles, sl, base, Q, th, obj, bar, abort, spin, grid, st);
    if (e == hipSuccess) e = launch_finalize_slots(sl, ns, ds, st);
    if (e == hipSuccess) e = launch_advance(base, Q, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hs, ds, ns * 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(habort, abort, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    return e;
  });
  ln.qsteps = b->quantum;
  ln.launch += b->quantum;
  b->launches += 1;
  for (int i = 0; i < b->max_slots; ++i)
    if (ln.run[i] && running(b->slots[i])) b->slots[i].lane = L;
  b->node_updates += ln.nodes * b->quantum;  // slots that finish early idle their tiles
  ln.persistent = true;
  ln.busy = true;
  return LBM_OK;
}

// Issue one quantum of lane L (tables, `quantum` batch launches, residual
// sums to the host, completion event).  No-op for an empty run set.
int launch_quantum(lbm_batch* b, int L) {
  Lane& ln = b->lanes[L];
  int nrun = 0, only = -1;
  for (int i = 0; i < b->max_slots; ++i)
    if (ln.run[i] && running(b->slots[i])) {
      ++nrun;
      only = i;
    }
  if (nrun == 0) return LBM_OK;
  const bool persist_ok = b->persist_grid > 0 && b->persist_tiles > 0;
  if (nrun == 1 && !(persist_ok && b->slots[only].p->nblk <= b->persist_tiles))
    return launch_solo(b, L, only);
  if (needs_upload(b, ln)) {
    int rc = upload_tables(b, ln);
    if (rc) return rc;
  }
  const int ntiles = (int)ln.h_tiles.size();
  if (ntiles == 0) return LBM_OK;
  if (persist_ok && ntiles <= b->persist_tiles) return launch_persistent(b, L, ntiles);
  hipGraphExec_t x = nullptr;
  if (ntiles < kDirectTiles) {
    auto it = ln.graphs.find(ntiles);
    if (it == ln.graphs.end()) {
      if (ln.graphs.size() >= 32) {  // bound the cache
        for (auto& g : ln.graphs) (void)hipGraphExecDestroy(g.second);
        ln.graphs.clear();
      }
      auto issue = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int q = 0; q < b->quantum && e == hipSuccess; ++q)
          e = launch_batch(ln.d_tiles, ntiles, ln.d_slots, ln.d_base, q, b->thermal != 0,
                           b->objective, ln.stream);
        // diagnostic steps end quanta: re-base the thermal states they left
        if (e == hipSuccess && b->thermal)
          e = launch_batch_rebase(ln.d_tiles, ntiles, ln.d_slots, ln.d_base, b->quantum - 1,
                                  ln.stream);
        if (e == hipSuccess) e = launch_finalize_slots(ln.d_slots, b->max_slots, ln.d_sums, ln.stream);
        if (e == hipSuccess) e = launch_advance(ln.d_base, b->quantum, ln.stream);
        return e;
      };
      int rc = capture(ln.stream, issue, &x);
      if (rc) return rc;
      it = ln.graphs.emplace(ntiles, x).first;
    }
    x = it->second;
  }
  const Tile* tiles = ln.d_tiles;
  const SlotDev* sl = ln.d_slots;
  int* base = ln.d_base;
  double* ds = ln.d_sums;
  double* hs = ln.h_sums;
  hipStream_t st = ln.stream;
  hipEvent_t ev = ln.done;
  const int Q = b->quantum, ns = b->max_slots, obj = b->objective;
  const bool th = b->thermal != 0;
  post(ln.worker.get(), [=]() -> hipError_t {
    hipError_t e = hipSuccess;
    if (x) {
      e = hipGraphLaunch(x, st);
    } else {
      for (int q = 0; q < Q && e == hipSuccess; ++q)
        e = launch_batch(tiles, ntiles, sl, base, q, th, obj, st);
      if (e == hipSuccess && th) e = launch_batch_rebase(tiles, ntiles, sl, base, Q - 1, st);
      if (e == hipSuccess) e = launch_finalize_slots(sl, ns, ds, st);
      if (e == hipSuccess) e = launch_advance(base, Q, st);
    }
    // the copy to host memory stays out of graphs (as a node it is slower)
    if (e == hipSuccess) e = hipMemcpyAsync(hs, ds, ns * 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    return e;
  });
  ln.qsteps = b->quantum;
  ln.launch += b->quantum;
  b->launches += b->quantum;
  for (int i = 0; i < b->max_slots; ++i)
    if (ln.run[i] && running(b->slots[i])) b->slots[i].lane = L;
  b->node_updates += ln.nodes * b->quantum;  // slots that finish early idle their tiles
  ln.busy = true;
  return LBM_OK;
}

// Bookkeeping once lane L's quantum has completed.
int complete_quantum(lbm_batch* b, int L) {
  Lane& ln = b->lanes[L];
  const bool gave_up = ln.persistent && *ln.h_abort != 0;
  ln.persistent = false;
  for (int i = 0; i < b->max_slots; ++i) {
    Slot& s = b->slots[i];
    if (!running(s) || s.lane != L) continue;
    s.lane = -1;
    if (gave_up) {
      // the quantum stopped part-way: its slots' states are not steps of their solves
      s.error = "persistent batch launch: a grid barrier wait gave up";
      s.phase = PH_FAILED;
      s.status = LBM_EDEVICE;
      continue;
    }
    s.steps = std::min(s.steps + ln.qsteps, s.p->d.max_steps);
    int rc = after_quantum(b, i, ln);
    if (rc) return rc;
  }
  HIPCHK(hipStreamSynchronize(ln.stream));  // post-quantum kernels
  ln.busy = false;
  return LBM_OK;
}

void drop_graphs(Lane& ln) {
  for (auto& g : ln.graphs) (void)hipGraphExecDestroy(g.second);
  ln.graphs.clear();
  for (auto& g : ln.solo) (void)hipGraphExecDestroy(g.second);
  ln.solo.clear();
}

void stop_worker(Lane& ln) {
  if (!ln.worker) return;
  {
    std::lock_guard<std::mutex> lk(ln.worker->m);
    ln.worker->quit = true;
  }
  ln.worker->cv.notify_one();
  if (ln.worker->th.joinable()) ln.worker->th.join();
  ln.worker.reset();
}

void free_lanes(lbm_batch* b) {
  for (Lane& ln : b->lanes) {
    stop_worker(ln);
    if (ln.stream) {
      (void)hipStreamSynchronize(ln.stream);
      drop_graphs(ln);
      (void)hipStreamDestroy(ln.stream);
    }
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.h_sums) (void)hipHostFree(ln.h_sums);
    if (ln.h_abort) (void)hipHostFree(ln.h_abort);
    ln.h_abort = nullptr;
    if (ln.pin_slots) (void)hipHostFree(ln.pin_slots);
    if (ln.pin_tiles) (void)hipHostFree(ln.pin_tiles);
    ln.stream = nullptr;
    ln.done = nullptr;
    ln.h_sums = nullptr;
    ln.pin_slots = nullptr;
    ln.pin_tiles = nullptr;
    ln.busy = false;
  }
}

}  // namespace

extern "C" {

int lbm_batch_create(int32_t thermal, int32_t objective, int32_t max_slots, int32_t quantum,
                     lbm_batch_t** out) {
  last_error().clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if ((thermal != 0 && thermal != 1) || objective < 0 || objective > 3 || max_slots < 1 ||
      max_slots > 4096 || quantum < 1)
    return fail(LBM_EINVAL, "bad batch parameters");
  lbm_batch* b = new lbm_batch();
  b->thermal = thermal;
  b->objective = objective;
  b->max_slots = max_slots;
  b->quantum = quantum;
  b->slots.resize(max_slots);
  for (Lane& ln : b->lanes) {
    ln.h_slots.assign(max_slots, SlotDev{});
    ln.run.assign(max_slots, 0);
    ln.up_ticket.assign(max_slots, -1);
  }
  *out = b;
  return LBM_OK;
}

size_t lbm_batch_table_bytes(const lbm_batch_t* b, size_t arena_bytes) {
  if (!b) return 0;
  // one tile per 256 nodes; every node needs at least 4 x 9 floats of
  // workspace (two forward and two adjoint D2Q9 buffers)
  const size_t max_tiles = arena_bytes / (4 * 9 * 4 * kBlock) + b->max_slots;
  return kLanes * lane_table_bytes(b->max_slots, (int)max_tiles) + 256;
}

int lbm_batch_bind_arena(lbm_batch_t* b, void* device_ptr, size_t bytes) {
  last_error().clear();
  if (!b || !device_ptr) return fail(LBM_EINVAL, "batch or arena is NULL");
  for (const Slot& s : b->slots)
    if (s.used) return fail(LBM_ESTATE, "cannot rebind while requests are resident");
  const size_t max_tiles = bytes / (4 * 9 * 4 * kBlock) + b->max_slots;
  if (max_tiles > (size_t)INT32_MAX) return fail(LBM_EINVAL, "arena too large");
  const size_t tb = lbm_batch_table_bytes(b, bytes);
  if (bytes <= tb + 256) return fail(LBM_EINVAL, "arena too small");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (b->dev >= 0 && dev != b->dev) free_lanes(b);
  b->dev = dev;
  char* base = (char*)(((uintptr_t)device_ptr + 255) & ~uintptr_t(255));
  const size_t usable = bytes - (size_t)(base - (char*)device_ptr);
  b->max_tiles = (int)max_tiles;
  char* t = base;
  for (Lane& ln : b->lanes) {
    ln.d_slots = (SlotDev*)t;
    ln.d_tiles = (Tile*)(t + align256(b->max_slots * sizeof(SlotDev)));
    ln.d_sums = (double*)((char*)ln.d_tiles + align256((size_t)b->max_tiles * sizeof(Tile)));
    ln.d_base = (int*)((char*)ln.d_sums + align256((size_t)b->max_slots * 4 * sizeof(double)));
    ln.d_bar = (unsigned*)((char*)ln.d_base + 64);
    ln.d_abort = (int*)((char*)ln.d_base + 128);
    t += lane_table_bytes(b->max_slots, b->max_tiles);
    if (!ln.stream) HIPCHK(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking));
    if (!ln.done) HIPCHK(hipEventCreateWithFlags(&ln.done, hipEventDisableTiming));
    if (!ln.h_sums)
      HIPCHK(hipHostMalloc((void**)&ln.h_sums, b->max_slots * 4 * sizeof(double), hipHostMallocDefault));
    if (!ln.h_abort) HIPCHK(hipHostMalloc((void**)&ln.h_abort, 4 * sizeof(int), hipHostMallocDefault));
    *ln.h_abort = 0;
    if (!ln.pin_slots)
      HIPCHK(hipHostMalloc((void**)&ln.pin_slots, b->max_slots * sizeof(SlotDev), hipHostMallocDefault));
    if (ln.pin_tiles) HIPCHK(hipHostFree(ln.pin_tiles));
    ln.pin_tiles = nullptr;
    HIPCHK(hipHostMalloc((void**)&ln.pin_tiles, (size_t)b->max_tiles * sizeof(Tile), hipHostMallocDefault));
    // empty slot tables on both sides
    std::fill(ln.h_slots.begin(), ln.h_slots.end(), SlotDev{});
    std::fill(ln.up_ticket.begin(), ln.up_ticket.end(), -1);
    HIPCHK(hipMemsetAsync(ln.d_slots, 0, b->max_slots * sizeof(SlotDev), ln.stream));
    HIPCHK(hipMemsetAsync(ln.d_base, 0, sizeof(int), ln.stream));
    HIPCHK(hipStreamSynchronize(ln.stream));
    drop_graphs(ln);  // captured with the previous arena's addresses
    ln.launch = 0;
    if (!ln.worker) {
      ln.worker = std::make_unique<Worker>();
      ln.worker->th = std::thread(worker_main, ln.worker.get(), dev);
    }
  }
  b->base = base + tb;
  b->arena.reset((usable - tb) & ~size_t(255));
  b->persist_grid = persistent_grid_limit(b->thermal != 0, b->objective);
  return LBM_OK;
}

int lbm_batch_set_policy(lbm_batch_t* b, int32_t policy, int32_t fill_tiles) {
  last_error().clear();
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if ((policy != LBM_BATCH_POLICY_ALL && policy != LBM_BATCH_POLICY_SRW &&
       policy != LBM_BATCH_POLICY_OVERLAP && policy != LBM_BATCH_POLICY_OVERLAP_FIFO) ||
      fill_tiles < 1)
    return fail(LBM_EINVAL, "bad policy or fill");
  for (const Lane& ln : b->lanes)
    if (ln.busy) return fail(LBM_ESTATE, "cannot change the policy while a quantum is in flight");
  b->policy = policy;
  b->fill_tiles = fill_tiles;
  return LBM_OK;
}

int lbm_batch_set_persistent(lbm_batch_t* b, int32_t max_tiles) {
  last_error().clear();
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (max_tiles < 0) return fail(LBM_EINVAL, "max_tiles must be >= 0");
  for (const Lane& ln : b->lanes)
    if (ln.busy) return fail(LBM_ESTATE, "cannot change the launch form while a quantum is in flight");
  b->persist_tiles = max_tiles;
  return LBM_OK;
}

int lbm_batch_submit(lbm_batch_t* b, const lbm_desc_t* desc, const uint8_t* mask,
                     const float* gamma_host, int64_t* ticket) {
  last_error().clear();
  if (!b || !desc || !mask || !gamma_host || !ticket) return fail(LBM_EINVAL, "null argument");
  if (!b->base) return fail(LBM_ESTATE, "no arena bound");
  if (desc->thermal != b->thermal || desc->objective != b->objective)
    return fail(LBM_EINVAL, "request lattice/objective differ from the batch's");
  if (desc->max_steps % b->quantum != 0 || (desc->check_every > 0 && desc->check_every % b->quantum != 0))
    return fail(LBM_EINVAL, "max_steps and check_every must be multiples of the quantum");
  lbm_problem probe;
  int rc = validate_and_setup(&probe, *desc, mask);
  if (rc) return rc;
  if (request_bytes(&probe) > b->arena.size()) return fail(LBM_ENOMEM, "request larger than the arena");
  if (probe.nblk > b->max_tiles) return fail(LBM_ENOMEM, "request larger than the tile table");
  Request r;
  r.ticket = b->next_ticket++;
  r.desc = *desc;
  r.mask.assign(mask, mask + probe.N);
  r.gamma.assign(gamma_host, gamma_host + probe.N);
  b->queue.push_back(std::move(r));
  *ticket = b->queue.back().ticket;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch_t* b, void* stream, int32_t* active, int32_t* queued) {
  last_error().clear();
  if (!b || !b->base) return fail(LBM_ESTATE, "no arena bound");
  DeviceGuard guard(b->dev);
  hipStream_t st = (hipStream_t)stream;
  int rc = admit(b, st);
  if (rc) return rc;
  const int nl = lanes_used(b);
  for (int L = 0; L < nl; ++L) {
    if (b->lanes[L].busy) continue;
    choose_run_set(b, L);
    rc = launch_quantum(b, L);
    if (rc) return rc;
  }
  bool any = false;
  for (int L = 0; L < nl; ++L) any = any || b->lanes[L].busy;
  while (any) {
    bool got = false;
    for (int L = 0; L < nl; ++L) {
      Lane& ln = b->lanes[L];
      if (!ln.busy) continue;
      if (!ln.worker->posted.load(std::memory_order_acquire)) continue;
      const int we = ln.worker->err.exchange(0);
      if (we) {
        ln.busy = false;
        for (Slot& sl : b->slots)
          if (sl.lane == L) sl.lane = -1;
        return fail(LBM_EDEVICE, std::string("lane launch failed: ") + hipGetErrorString((hipError_t)we));
      }
      const hipError_t e = hipEventQuery(ln.done);
      if (e == hipErrorNotReady) continue;
      HIPCHK(e);
      rc = complete_quantum(b, L);
      if (rc) return rc;
      // the lane's next quantum goes out now, not at the caller's next call:
      // its stream would otherwise idle through the caller's own bookkeeping
      choose_run_set(b, L);
      rc = launch_quantum(b, L);
      if (rc) return rc;
      got = true;
    }
    if (got) break;
    std::this_thread::yield();
  }
  int na = 0;
  for (const Slot& s : b->slots)
    if (running(s)) ++na;
  if (active) *active = na;
  if (queued) *queued = (int32_t)b->queue.size();
  return LBM_OK;
}

int lbm_batch_poll(lbm_batch_t* b, int64_t ticket, lbm_batch_result_t* res, float* dJ_host,
                   void* stream) {
  last_error().clear();
  if (!b || !res) return fail(LBM_EINVAL, "null argument");
  std::memset(res, 0, sizeof(*res));
  res->ticket = ticket;
  for (const Request& r : b->queue)
    if (r.ticket == ticket) {
      res->state = LBM_BATCH_QUEUED;
      return LBM_OK;
    }
  auto it = b->slot_of.find(ticket);
  if (it == b->slot_of.end()) return fail(LBM_EINVAL, "unknown or already collected ticket");
  const int i = it->second;
  Slot& s = b->slots[i];
  res->nodes = s.p->N;
  res->fwd_steps = s.phase == PH_FORWARD ? s.steps : s.fwd_steps;
  res->adj_steps = s.phase == PH_ADJOINT ? s.steps : s.adj_steps;
  if (running(s)) {
    res->state = LBM_BATCH_RUNNING;
    return LBM_OK;
  }
  DeviceGuard guard(b->dev);
  res->J = s.J;
  res->status = s.status;
  res->state = s.phase == PH_DONE ? LBM_BATCH_DONE : LBM_BATCH_FAILED;
  if (s.phase == PH_DONE && dJ_host) {
    const size_t nb = (size_t)s.p->N * sizeof(float);
    int rc = ensure_stage(b, nb);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(b->stage, s.dJ, nb, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    std::memcpy(dJ_host, b->stage, nb);
  }
  release_slot(b, i);
  return LBM_OK;
}

int lbm_batch_stats(const lbm_batch_t* b, lbm_batch_stats_t* out) {
  last_error().clear();
  if (!b || !out) return fail(LBM_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->arena_bytes = b->arena.size();
  out->bytes_in_use = b->arena.used();
  for (const Slot& s : b->slots) {
    if (!s.used) continue;
    if (running(s)) ++out->running;
    else ++out->finished;
  }
  out->queued = (int32_t)b->queue.size();
  out->launches = b->launches;
  out->node_updates = b->node_updates;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch_t* b) {
  if (!b) return;
  if (b->dev >= 0) {
    DeviceGuard guard(b->dev);
    free_lanes(b);
  }
  if (b->stage) (void)hipHostFree(b->stage);
  delete b;
}

}  // extern "C"
