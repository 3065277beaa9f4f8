// Continuous-batching engine for many steady sensitivity solves on one GPU.
//
// Requests (problem descriptor, mask, design field) queue in arrival order.
// At every quantum boundary the engine admits queued requests, first come
// first served, while a slot is free and the request's workspace and fields
// fit in the caller's arena (the HBM budget).  Every admitted request is a
// slot; one ragged-batch kernel launch advances all slots by one lattice step
// each, whatever their grid size and whether they are in the forward or the
// adjoint sweep.  At quantum boundaries the per-slot residual sums are read
// back; a slot moves from the forward sweep to the adjoint sweep to the
// sensitivity when its residual criterion (or step cap) is met, exactly as a
// single solve would, and its memory returns to the arena when the caller has
// collected the result.  No arithmetic of one slot depends on another, so
// each result is bit for bit the result of the same request solved alone.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "lbm_internal.h"
#include "lbmadj.h"

using namespace lbmadj;

namespace {

enum SlotPhase { PH_IDLE = 0, PH_FORWARD = 1, PH_ADJOINT = 2, PH_DONE = 3, PH_FAILED = 4 };

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
  int start = 0;
  int fwd_steps = 0, adj_steps = 0;
  int status = LBM_OK;
  double prev[2] = {0, 0}, res[2] = {0, 0}, mon[2] = {0, 0};
  bool have_prev = false;
  int fwd_status = LBM_NOT_CONVERGED, adj_status = LBM_NOT_CONVERGED;
  double J = 0.0;
  std::string error;
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
  int dev = -1;
  char* base = nullptr;  // arena start (aligned)
  Arena arena;
  // fixed tables carved at the start of the caller's memory
  SlotDev* d_slots = nullptr;
  Tile* d_tiles = nullptr;
  double* d_sums = nullptr;
  double* h_sums = nullptr;  // pinned
  int max_tiles = 0;
  std::vector<SlotDev> h_slots;
  std::vector<Tile> h_tiles;
  bool tables_dirty = true;
  std::vector<Slot> slots;
  std::deque<Request> queue;
  std::map<int64_t, int> slot_of;  // ticket -> slot
  int64_t next_ticket = 1;
  int launch = 0;
  long long node_updates = 0;
  long long launches = 0;
};

namespace {

size_t fields_bytes(const lbm_problem* p) {
  // gamma, drho, u (3), T, dJ, each N floats, 256-byte aligned
  return 7 * align256((size_t)p->N * sizeof(float));
}

size_t request_bytes(const lbm_problem* p) { return layout_of(p).total + fields_bytes(p); }

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
  }
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
  std::vector<float> uin(p->Np, 0.0f);
  std::copy(p->uin_host.begin(), p->uin_host.end(), uin.begin());
  std::vector<uint8_t> fl(p->Np, (uint8_t)K_WALL);
  std::copy(p->flags_host.begin(), p->flags_host.end(), fl.begin());
  HIPCHK(hipMemcpyAsync(p->uin, uin.data(), p->Np * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p->flags, fl.data(), p->Np, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s.gamma, r.gamma.data(), (size_t)p->N * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(launch_fill(p->f[0], (size_t)19 * p->Np, st));
  if (th) HIPCHK(launch_fill(p->g[0], (size_t)7 * p->Np, st));
  HIPCHK(hipStreamSynchronize(st));  // the host vectors above go out of scope
  return LBM_OK;
}

void release_slot(lbm_batch* b, int i) {
  Slot& s = b->slots[i];
  if (s.bytes) b->arena.release(s.off, s.bytes);
  b->slot_of.erase(s.ticket);
  s = Slot();
  b->tables_dirty = true;
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
    s.start = b->launch;
    b->slot_of[r.ticket] = free_slot;
    b->queue.pop_front();
    b->tables_dirty = true;
  }
  return LBM_OK;
}

// Device slot table and tile table from the host state.
int upload_tables(lbm_batch* b, hipStream_t st) {
  b->h_tiles.clear();
  for (int i = 0; i < b->max_slots; ++i) {
    Slot& s = b->slots[i];
    SlotDev& d = b->h_slots[i];
    std::memset((void*)&d, 0, sizeof(SlotDev));
    if (!s.used || (s.phase != PH_FORWARD && s.phase != PH_ADJOINT)) continue;
    lbm_problem* p = s.p.get();
    d.phase = s.phase;
    d.start = s.start;
    d.max_steps = p->d.max_steps;
    d.check = p->d.check_every;
    p->fcur = 0;
    p->acur = 0;
    d.fa = fwd_args(p, s.gamma, s.drho, s.u, s.T);
    d.aa = adj_args(p, s.gamma, s.u, s.T);
    for (int t = 0; t < p->nblk; ++t) b->h_tiles.push_back(Tile{i, t});
  }
  if ((int)b->h_tiles.size() > b->max_tiles) return fail(LBM_ENOMEM, "tile table full");
  HIPCHK(hipMemcpyAsync(b->d_slots, b->h_slots.data(), b->max_slots * sizeof(SlotDev),
                        hipMemcpyHostToDevice, st));
  if (!b->h_tiles.empty())
    HIPCHK(hipMemcpyAsync(b->d_tiles, b->h_tiles.data(), b->h_tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  b->tables_dirty = false;
  return LBM_OK;
}

// Phase bookkeeping of one slot after the quantum that ended at b->launch.
int after_quantum(lbm_batch* b, int i, hipStream_t st) {
  Slot& s = b->slots[i];
  lbm_problem* p = s.p.get();
  const int done = std::min(b->launch - s.start, p->d.max_steps);
  const int check = p->d.check_every;
  const bool at_check = check > 0 && done > 0 && done % check == 0;
  const bool at_end = done >= p->d.max_steps;
  if (!at_check && !at_end) return LBM_OK;
  const bool th = thermal_of(p);
  const double* sums = b->h_sums + (size_t)i * 4;
  s.mon[0] = sums[0] / p->n_nonwall;
  s.mon[1] = sums[1] / p->n_nonwall;
  if (!std::isfinite(s.mon[0]) || !std::isfinite(s.mon[1])) {
    s.error = std::string(s.phase == PH_FORWARD ? "forward" : "adjoint") + " sweep diverged";
    s.phase = PH_FAILED;
    s.status = LBM_EDIVERGED;
    b->tables_dirty = true;
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
      double v = 0.0;
      HIPCHK(hipMemcpyAsync(b->h_sums + (size_t)i * 4, p->sums, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      v = b->h_sums[(size_t)i * 4];
      J = v;
      HIPCHK(launch_dissipation_source(s.u, s.gamma, p->flags, p->G, p->kp, st));
    } else {
      if (p->n_inlet > 0) J += p->d.w_dp * (sums[2] / p->n_inlet) / 3.0;
      if (p->d.objective == LBM_OBJ_HEATSINK) J += sums[3] / p->n_layer;
    }
    s.J = J;
    HIPCHK(launch_fill(p->a[0], (size_t)19 * p->Np, st));
    if (th) HIPCHK(launch_fill(p->b[0], (size_t)7 * p->Np, st));
    s.phase = PH_ADJOINT;
    s.start = b->launch;
    s.have_prev = false;
    s.res[0] = s.res[1] = 0.0;
  } else {
    s.adj_steps = done;
    s.adj_status = converged ? LBM_OK : LBM_NOT_CONVERGED;
    // final adjoint state is buffer (done & 1)
    p->acur = done & 1;
    SensArgs A{};
    A.ain = p->a[p->acur];
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
  b->tables_dirty = true;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_create(int32_t thermal, int32_t objective, int32_t max_slots, int32_t quantum,
                     lbm_batch_t** out) {
  last_error().clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if ((thermal != 0 && thermal != 1) || objective < 0 || objective > 2 || max_slots < 1 ||
      max_slots > 4096 || quantum < 1)
    return fail(LBM_EINVAL, "bad batch parameters");
  lbm_batch* b = new lbm_batch();
  b->thermal = thermal;
  b->objective = objective;
  b->max_slots = max_slots;
  b->quantum = quantum;
  b->slots.resize(max_slots);
  b->h_slots.resize(max_slots);
  *out = b;
  return LBM_OK;
}

size_t lbm_batch_table_bytes(const lbm_batch_t* b, size_t arena_bytes) {
  if (!b) return 0;
  // one tile per 256 nodes; every node needs at least 4 x 19 floats of workspace
  const size_t max_tiles = arena_bytes / (4 * 19 * 4 * kBlock) + b->max_slots;
  return align256(b->max_slots * sizeof(SlotDev)) + align256(max_tiles * sizeof(Tile)) +
         align256(b->max_slots * 4 * sizeof(double)) + 256;
}

int lbm_batch_bind_arena(lbm_batch_t* b, void* device_ptr, size_t bytes) {
  last_error().clear();
  if (!b || !device_ptr) return fail(LBM_EINVAL, "batch or arena is NULL");
  for (const Slot& s : b->slots)
    if (s.used) return fail(LBM_ESTATE, "cannot rebind while requests are resident");
  const size_t tb = lbm_batch_table_bytes(b, bytes);
  if (bytes <= tb + 256) return fail(LBM_EINVAL, "arena too small");
  HIPCHK(hipGetDevice(&b->dev));
  char* base = (char*)(((uintptr_t)device_ptr + 255) & ~uintptr_t(255));
  const size_t usable = bytes - (size_t)(base - (char*)device_ptr);
  b->max_tiles = (int)((tb - align256(b->max_slots * sizeof(SlotDev)) -
                        align256(b->max_slots * 4 * sizeof(double)) - 256) / sizeof(Tile));
  b->d_slots = (SlotDev*)base;
  b->d_tiles = (Tile*)(base + align256(b->max_slots * sizeof(SlotDev)));
  b->d_sums = (double*)((char*)b->d_tiles + align256((size_t)b->max_tiles * sizeof(Tile)));
  b->base = base + tb;
  b->arena.reset((usable - tb) & ~size_t(255));
  if (!b->h_sums) HIPCHK(hipHostMalloc((void**)&b->h_sums, b->max_slots * 4 * sizeof(double), hipHostMallocDefault));
  b->tables_dirty = true;
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
  if (b->tables_dirty) {
    rc = upload_tables(b, st);
    if (rc) return rc;
  }
  const int ntiles = (int)b->h_tiles.size();
  if (ntiles > 0) {
    long long nodes_per_launch = 0;
    for (const Slot& s : b->slots)
      if (s.used && (s.phase == PH_FORWARD || s.phase == PH_ADJOINT)) nodes_per_launch += s.p->N;
    for (int q = 0; q < b->quantum; ++q) {
      HIPCHK(launch_batch(b->d_tiles, ntiles, b->d_slots, b->launch, b->thermal != 0, b->objective, st));
      ++b->launch;
      ++b->launches;
    }
    b->node_updates += nodes_per_launch * b->quantum;  // slots that finish early idle their tiles
    HIPCHK(launch_finalize_slots(b->d_slots, b->max_slots, b->d_sums, st));
    HIPCHK(hipMemcpyAsync(b->h_sums, b->d_sums, b->max_slots * 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < b->max_slots; ++i) {
      Slot& s = b->slots[i];
      if (!s.used || (s.phase != PH_FORWARD && s.phase != PH_ADJOINT)) continue;
      rc = after_quantum(b, i, st);
      if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(st));
  }
  int na = 0;
  for (const Slot& s : b->slots)
    if (s.used && (s.phase == PH_FORWARD || s.phase == PH_ADJOINT)) ++na;
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
  res->fwd_steps = s.phase == PH_FORWARD ? b->launch - s.start : s.fwd_steps;
  res->adj_steps = s.phase == PH_ADJOINT ? b->launch - s.start : s.adj_steps;
  if (s.phase == PH_FORWARD || s.phase == PH_ADJOINT) {
    res->state = LBM_BATCH_RUNNING;
    return LBM_OK;
  }
  DeviceGuard guard(b->dev);
  res->J = s.J;
  res->status = s.status;
  res->state = s.phase == PH_DONE ? LBM_BATCH_DONE : LBM_BATCH_FAILED;
  if (s.phase == PH_DONE && dJ_host) {
    HIPCHK(hipMemcpyAsync(dJ_host, s.dJ, (size_t)s.p->N * sizeof(float), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
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
    if (s.phase == PH_FORWARD || s.phase == PH_ADJOINT) ++out->running;
    else ++out->finished;
  }
  out->queued = (int32_t)b->queue.size();
  out->launches = b->launches;
  out->node_updates = b->node_updates;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch_t* b) {
  if (!b) return;
  if (b->h_sums) (void)hipHostFree(b->h_sums);
  delete b;
}

}  // extern "C"
