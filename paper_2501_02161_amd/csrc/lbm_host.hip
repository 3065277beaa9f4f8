// Host side of the C ABI declared in include/lbmadj.h: descriptor and mask
// validation, node set-up (flags, inlet profile, objective layer), the
// workspace layout, and the forward / adjoint solve loops with the residual
// criterion of Sec. 3.1 of arXiv 2501.02161.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_internal.h"
#include "lbmadj.h"

using namespace lbmadj;

namespace lbmadj {

std::string& last_error() {
  thread_local std::string err;
  return err;
}

}  // namespace lbmadj

namespace lbmadj {

bool thermal_of(const lbm_problem* p) { return p->d.thermal != 0; }
int qf_of(const lbm_problem* p) { return p->d.nz == 1 ? 9 : 19; }
int qg_of(const lbm_problem* p) { return p->d.nz == 1 ? 5 : 7; }

Layout layout_of(const lbm_problem* p) {
  Layout L{};
  size_t off = 0;
  const size_t pf = (size_t)qf_of(p) * p->Np * sizeof(float), pg = (size_t)qg_of(p) * p->Np * sizeof(float);
  const bool th = thermal_of(p);
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  for (int k = 0; k < 2; ++k) L.f[k] = take(pf);
  for (int k = 0; k < 2; ++k) L.g[k] = th ? take(pg) : 0;
  for (int k = 0; k < 2; ++k) L.a[k] = take(pf);
  for (int k = 0; k < 2; ++k) L.b[k] = th ? take(pg) : 0;
  for (int k = 0; k < 2; ++k) L.R[k] = th ? take((size_t)p->Np * sizeof(float)) : 0;
  L.gneq = th ? take(pg) : 0;
  L.G = (p->d.objective == LBM_OBJ_DISSIPATION) ? take((size_t)3 * p->Np * sizeof(float)) : 0;
  L.uin = take((size_t)p->Np * sizeof(float));
  L.flags = take((size_t)p->Np);
  L.partials = take((size_t)p->nblk * 4 * sizeof(double));
  L.sums = take(16 * sizeof(double));
  L.total = off + 256;  // slack for aligning the caller's pointer
  return L;
}

int validate_and_setup(lbm_problem* p, const lbm_desc_t& d, const uint8_t* mask) {
  if (d.nx < 3 || d.ny < 3 || (d.nz < 3 && d.nz != 1))
    return fail(LBM_EINVAL, "nx, ny must be >= 3 and nz >= 3 (D3Q19) or nz == 1 (D2Q9)");
  const bool two_d = d.nz == 1;
  if (two_d && d.symmetric[2])
    return fail(LBM_EINVAL, "the 2D lattice (nz == 1) has no z axis to be symmetric");
  const long long N = (long long)d.nx * d.ny * d.nz;
  if (N > (1LL << 31) / 32) return fail(LBM_EINVAL, "grid too large for 32-bit indexing");
  if (!(d.tau > 0.5)) return fail(LBM_EINVAL, "tau must be > 1/2");
  if (!(d.rho0 > 0.0)) return fail(LBM_EINVAL, "rho0 must be > 0");
  if (d.thermal != 0 && d.thermal != 1) return fail(LBM_EINVAL, "thermal must be 0 or 1");
  for (int a = 0; a < 3; ++a)
    if (d.periodic[a] != 0 && d.periodic[a] != 1) return fail(LBM_EINVAL, "periodic must be 0 or 1");
  if (d.objective < 0 || d.objective > 3) return fail(LBM_EINVAL, "unknown objective");
  if (d.max_steps < 1) return fail(LBM_EINVAL, "max_steps must be >= 1");
  if (d.check_every < 0) return fail(LBM_EINVAL, "check_every must be >= 0");
  if (!(d.tol >= 0.0)) return fail(LBM_EINVAL, "tol must be >= 0");
  if (d.adjoint_kind != LBM_ADJOINT_DISCRETE && d.adjoint_kind != LBM_ADJOINT_CONTINUOUS)
    return fail(LBM_EINVAL, "unknown adjoint kind");
  if (d.adjoint_kind == LBM_ADJOINT_CONTINUOUS && d.thermal)
    return fail(LBM_EINVAL, "the continuous adjoint is for the flow lattice only");
  for (int a = 0; a < 3; ++a) {
    if (d.symmetric[a] != 0 && d.symmetric[a] != 1) return fail(LBM_EINVAL, "symmetric must be 0 or 1");
    if (d.symmetric[a] && d.periodic[a]) return fail(LBM_EINVAL, "an axis cannot be periodic and symmetric");
  }
  if (d.symmetric[0] && d.nx < 4) return fail(LBM_EINVAL, "a symmetric axis needs at least 4 layers");
  if (d.symmetric[1] && d.ny < 4) return fail(LBM_EINVAL, "a symmetric axis needs at least 4 layers");
  if (d.symmetric[2] && d.nz < 4) return fail(LBM_EINVAL, "a symmetric axis needs at least 4 layers");
  if (!(d.inlet_rho >= 0.0)) return fail(LBM_EINVAL, "inlet_rho must be >= 0");
  if (!(d.beta_max >= 0.0) || (d.beta_max > 0.0 && !d.thermal))
    return fail(LBM_EINVAL, "beta_max must be >= 0 and needs the thermal lattice");
  if (d.objective == LBM_OBJ_HEATGEN && (!d.thermal || !(d.beta_max > 0.0)))
    return fail(LBM_EINVAL, "the heat-generation objective needs the thermal lattice and beta_max > 0");
  if (!(d.alpha_max >= 0.0) || !(d.q_brink > 0.0)) return fail(LBM_EINVAL, "need alpha_max >= 0, q > 0");
  if (!(d.tau * d.alpha_max < 1.0)) return fail(LBM_EINVAL, "tau * alpha_max must be < 1 (chi > 0)");
  if (d.thermal) {
    if (!(d.Pr > 0.0) || !(d.k_ratio > 0.0) || !(d.q_ramp >= 0.0))
      return fail(LBM_EINVAL, "need Pr > 0, k_ratio > 0, q_ramp >= 0");
  }
  if (d.objective == LBM_OBJ_HEATSINK && !d.thermal)
    return fail(LBM_EINVAL, "the heat-sink objective needs the thermal lattice");
  if (!mask) return fail(LBM_EINVAL, "mask is NULL");

  p->d = d;
  p->N = (int)N;
  p->Np = (int)((N + 63) / 64 * 64);
  p->nblk = (int)((N + kBlock - 1) / kBlock);
  p->flags_host.assign(mask, mask + N);
  p->uin_host.assign(N, 0.0f);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int lim[3] = {nx, ny, nz};
  auto coords = [&](long long n, int* c) {
    c[0] = (int)(n % nx);
    c[1] = (int)((n / nx) % ny);
    c[2] = (int)(n / ((long long)nx * ny));
  };
  for (long long n = 0; n < N; ++n) {
    const unsigned m = mask[n];
    const int kind = m & 7, nc = (m >> 3) & 7;
    if ((m >> 6) != 0 || kind > K_SYM) return fail(LBM_EINVAL, "bad mask byte at node " + std::to_string(n));
    int c[3];
    coords(n, c);
    bool on_sym = false;
    for (int a = 0; a < 3; ++a) on_sym = on_sym || (d.symmetric[a] && c[a] == lim[a] - 1);
    if (on_sym != (kind == K_SYM))
      return fail(LBM_EINVAL, "SYM nodes must fill exactly the last layer of each symmetric axis (node " +
                                  std::to_string(n) + ")");
    bool on_face[3];
    for (int a = 0; a < 3; ++a) on_face[a] = !d.periodic[a] && (c[a] == 0 || c[a] == lim[a] - 1);
    if (two_d) on_face[2] = false;  // the single layer of a 2D lattice has no z faces
    const bool boundary_kind = kind >= K_INLET;
    if ((on_face[0] || on_face[1] || on_face[2]) && !boundary_kind)
      return fail(LBM_EINVAL, "interior node on a non-periodic face at node " + std::to_string(n));
    if (kind == K_INLET || kind == K_OUTLET || kind == K_HEATED) {
      if (nc > (two_d ? 3 : 5)) return fail(LBM_EINVAL, "bad normal code at node " + std::to_string(n));
    } else {
      p->flags_host[n] = (uint8_t)kind;  // normal bits are meaningless here
    }
    if (kind == K_INLET || kind == K_OUTLET) {
      const int ax = nc / 2;
      const int face = (nc % 2 == 0) ? 0 : lim[ax] - 1;
      if (d.periodic[ax] || c[ax] != face)
        return fail(LBM_EINVAL, "port normal is not the inward normal of its face at node " + std::to_string(n));
      for (int b2 = 0; b2 < 3; ++b2)
        if (b2 != ax && on_face[b2])
          return fail(LBM_EINVAL, "port on an edge of two faces at node " + std::to_string(n));
    }
    if (kind == K_HEATED) {
      for (int a = 0; a < 3; ++a) {
        const int cc = c[a] + NVEC_HOST[nc][a];
        if (cc < 0 || cc >= lim[a]) return fail(LBM_EINVAL, "heated wall normal points out of the box");
      }
    }
  }
  // counts, objective layer
  p->n_inlet = p->n_layer = p->n_nonwall = p->n_design = 0;
  for (long long n = 0; n < N; ++n) {
    const int kind = p->flags_host[n] & 7;
    if (kind == K_INLET) ++p->n_inlet;
    if (kind == K_DESIGN) ++p->n_design;
    if (kind < K_WALL) ++p->n_nonwall;
    if (kind == K_HEATED) {
      const int nc = (p->flags_host[n] >> 3) & 7;
      int c[3];
      coords(n, c);
      const long long m = (c[0] + NVEC_HOST[nc][0]) + (long long)nx * ((c[1] + NVEC_HOST[nc][1]) + (long long)ny * (c[2] + NVEC_HOST[nc][2]));
      if ((mask[m] & 7) < K_WALL) p->flags_host[m] |= (uint8_t)kLayerBit;
    }
  }
  for (long long n = 0; n < N; ++n)
    if (p->flags_host[n] & kLayerBit) ++p->n_layer;
  if (p->n_nonwall == 0) return fail(LBM_EINVAL, "no non-wall nodes");
  if ((d.objective == LBM_OBJ_PRESSURE_DROP || d.objective == LBM_OBJ_HEATSINK) && d.w_dp != 0.0 &&
      p->n_inlet == 0)
    return fail(LBM_EINVAL, "the pressure-drop term needs inlet nodes");
  if (d.objective == LBM_OBJ_HEATSINK && p->n_layer == 0)
    return fail(LBM_EINVAL, "the heat-sink objective needs HEATED walls next to non-wall nodes");
  const double nu = (d.tau - 0.5) / 3.0;
  const bool pin = d.inlet_rho > 0.0;  // pressure inlets
  if (p->n_inlet > 0 && !pin && !(d.L_ref > 0.0)) return fail(LBM_EINVAL, "L_ref must be > 0 with inlets");
  const double U = (p->n_inlet > 0 && !pin) ? d.Re * nu / d.L_ref : 0.0;
  // inlet profile: product of parabolas over the inlet set of each normal
  for (int code = 0; code < 6; ++code) {
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    bool any = false;
    for (long long n = 0; n < N; ++n) {
      if ((p->flags_host[n] & 7) != K_INLET || ((p->flags_host[n] >> 3) & 7) != code) continue;
      any = true;
      int c[3];
      coords(n, c);
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], c[a]);
        hi[a] = std::max(hi[a], c[a]);
      }
    }
    if (!any) continue;
    for (long long n = 0; n < N; ++n) {
      if ((p->flags_host[n] & 7) != K_INLET || ((p->flags_host[n] >> 3) & 7) != code) continue;
      int c[3];
      coords(n, c);
      double prof = 1.0;
      for (int a = 0; a < 3; ++a) {
        if (NVEC_HOST[code][a] != 0) continue;
        if (lo[a] == 0 && hi[a] == lim[a] - 1) continue;
        // an inlet set reaching a mirror plane continues in its image
        const int h = (d.symmetric[a] && hi[a] == lim[a] - 2) ? 2 * lim[a] - 3 - lo[a] : hi[a];
        const double s = (c[a] - lo[a] + 0.5) / double(h - lo[a] + 1);
        prof *= 4.0 * s * (1.0 - s);
      }
      p->uin_host[n] = (float)(U * prof);
    }
  }
  // kernel constants
  KParams& k = p->kp;
  k.nx = nx;
  k.ny = ny;
  k.nz = nz;
  k.N = p->N;
  k.Np = p->Np;
  k.plane = nx * ny;
  k.px = d.periodic[0];
  k.py = d.periodic[1];
  k.pz = d.periodic[2];
  k.nblk = p->nblk;
  k.xcd_per = p->nblk / 8;
  k.xcd_rem = p->nblk % 8;
  k.omega = (float)(1.0 / d.tau);
  k.rho0 = (float)d.rho0;
  k.tab = (float)(d.tau * d.alpha_max * d.q_brink);
  k.amq = (float)(d.alpha_max * d.q_brink);
  k.qb = (float)d.q_brink;
  k.dfc = d.thermal ? (float)(4.0 * nu / d.Pr) : 0.0f;
  k.kr = (float)d.k_ratio;
  k.qr = (float)d.q_ramp;
  k.q_w = (float)d.q_w;
  k.T_in = (float)d.T_in;
  k.c_in = p->n_inlet > 0 ? (float)(d.w_dp / (3.0 * p->n_inlet)) : 0.0f;
  k.c_layer = p->n_layer > 0 ? (float)(1.0 / p->n_layer) : 0.0f;
  k.two_nu = (float)(2.0 * nu);
  k.nu = (float)nu;
  k.cont = d.adjoint_kind == LBM_ADJOINT_CONTINUOUS ? 1 : 0;
  k.sx = d.symmetric[0];
  k.sy = d.symmetric[1];
  k.sz = d.symmetric[2];
  k.pin = pin ? 1 : 0;
  k.drho_in = pin ? (float)(d.inlet_rho - d.rho0) : 0.0f;
  k.beta = (float)d.beta_max;
  k.heatgen = d.objective == LBM_OBJ_HEATGEN ? 1 : 0;
  k.q = d.nz == 1 ? 9 : 19;
  return LBM_OK;
}

// Sweep timing: events before the first and after the last step kernel of a
// sweep; the caller has synchronised the stream when sweep_end runs.
int sweep_begin(lbm_problem* p, hipStream_t s) {
  if (!p->timing) return LBM_OK;
  HIPCHK(hipEventRecord(p->sweep_ev[0], s));
  return LBM_OK;
}

int sweep_end(lbm_problem* p, int kind, int launches, hipStream_t s) {
  if (!p->timing) return LBM_OK;
  HIPCHK(hipEventRecord(p->sweep_ev[1], s));
  HIPCHK(hipEventSynchronize(p->sweep_ev[1]));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, p->sweep_ev[0], p->sweep_ev[1]));
  p->t_ms[kind] += ms;
  p->t_n[kind] += launches;
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free binding: a static workspace per device, for callers that
// cannot allocate device memory.  `scratch` is one array per GPU (each device
// holds its own copy at its own address); host code uses only the address
// hipGetSymbolAddress gives on each device, taken once per device.  One
// problem at a time owns a device's array: binding another one takes it over
// (the previous owner's later calls return LBM_ESTATE).
// ---------------------------------------------------------------------------
constexpr size_t kStaticBytes = size_t(32) << 20;
constexpr int kStaticDevices = 64;
__device__ __align__(256) char scratch[kStaticBytes];

struct StaticWorkspace {
  std::mutex mu;
  void* ptr[kStaticDevices] = {};
  const lbm_problem* owner[kStaticDevices] = {};
};
StaticWorkspace& static_ws() {
  static StaticWorkspace s;
  return s;
}

bool static_owned(const lbm_problem* p) {
  if (!p->static_ws || p->dev < 0 || p->dev >= kStaticDevices) return false;
  StaticWorkspace& sw = static_ws();
  std::lock_guard<std::mutex> lk(sw.mu);
  return sw.owner[p->dev] == p;
}

void static_release(const lbm_problem* p) {
  if (!p->static_ws || p->dev < 0 || p->dev >= kStaticDevices) return;
  StaticWorkspace& sw = static_ws();
  std::lock_guard<std::mutex> lk(sw.mu);
  if (sw.owner[p->dev] == p) sw.owner[p->dev] = nullptr;
}

// Workspace pointers of p at base (256-byte aligned) of `bytes` bytes.
void set_workspace(lbm_problem* p, char* base, size_t bytes) {
  const Layout L = layout_of(p);
  const bool th = thermal_of(p);
  p->ws = base;
  p->ws_bytes = bytes;
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
}

bool rel_converged(double now, double before, double tol) {
  if (!(tol > 0.0)) return false;
  return std::fabs(now - before) <= tol * std::fabs(now);
}

int read_sums(lbm_problem* p, int nvals, hipStream_t s) {
  HIPCHK(launch_finalize(p->partials, p->nblk, nvals, p->sums, s));
  HIPCHK(hipMemcpyAsync(p->pinned, p->sums, nvals * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return LBM_OK;
}

FwdArgs fwd_args(lbm_problem* p, const float* gamma, float* drho, float* u, float* T) {
  FwdArgs A{};
  A.fin = p->f[p->fcur];
  A.fout = p->f[1 - p->fcur];
  A.gin = p->g[p->fcur];
  A.gout = p->g[1 - p->fcur];
  A.Rin = p->R[p->rcur];
  A.flags = p->flags;
  A.gamma = gamma;
  A.uin = p->uin;
  A.drho = drho;
  A.u = u;
  A.T = T;
  A.gneq = p->gneq;
  A.partials = p->partials;
  A.P = p->kp;
  return A;
}

int objective_value(lbm_problem* p, const float* gamma, const float* u, hipStream_t s, double* J) {
  const lbm_desc_t& d = p->d;
  if (d.objective == LBM_OBJ_DISSIPATION) {
    HIPCHK(launch_dissipation_objective(u, gamma, p->flags, p->partials, p->kp, s));
    int rc = read_sums(p, kRedDiss, s);
    if (rc) return rc;
    *J = p->pinned[0];
    return LBM_OK;
  }
  // p->pinned holds the forward partial sums of the last diagnostic step
  double v = 0.0;
  if (d.objective == LBM_OBJ_HEATGEN) {
    *J = -p->pinned[3];  // J = -sum_j Q(x_j)
    return LBM_OK;
  }
  if (p->n_inlet > 0) v += d.w_dp * (p->pinned[2] / p->n_inlet) / 3.0;
  if (d.objective == LBM_OBJ_HEATSINK) v += p->pinned[3] / p->n_layer;
  *J = v;
  return LBM_OK;
}

// Forward iterations k = 1..nsteps from the current state.  With check > 0 the
// residual criterion is evaluated every `check` steps; the last step always
// writes the fields.
int run_forward(lbm_problem* p, const float* gamma, float* drho, float* u, float* T, int nsteps,
                int check, double tol, hipStream_t s, lbm_info_t* info) {
  const bool th = thermal_of(p);
  double prev[2] = {0, 0}, res[2] = {0, 0}, mon[2] = {0, 0};
  bool have_prev = false;
  int status = LBM_NOT_CONVERGED, k = 0;
  int rc0 = sweep_begin(p, s);
  if (rc0) return rc0;
  for (k = 1; k <= nsteps; ++k) {
    const bool at_check = check > 0 && k % check == 0;
    const bool diag = at_check || k == nsteps;
    HIPCHK(launch_forward(fwd_args(p, gamma, drho, u, T), th, diag, s));
    p->fcur = 1 - p->fcur;
    if (!diag) continue;
    if (th) {
      // move the thermal state's reference onto this step's temperature
      HIPCHK(launch_rebase(rebase_args(p, T), s));
      p->rcur = 1 - p->rcur;
    }
    int rc = read_sums(p, kRedFwd, s);
    if (rc) return rc;
    mon[0] = p->pinned[0] / p->n_nonwall;
    mon[1] = p->pinned[1] / p->n_nonwall;
    if (!std::isfinite(mon[0]) || !std::isfinite(mon[1])) {
      p->fwd_done = false;
      p->have_gneq = false;
      return fail(LBM_EDIVERGED, "forward solve diverged at step " + std::to_string(k));
    }
    if (at_check) {
      if (have_prev) {
        res[0] = std::fabs(mon[0] - prev[0]) / std::max(std::fabs(mon[0]), 1e-300);
        res[1] = std::fabs(mon[1] - prev[1]) / std::max(std::fabs(mon[1]), 1e-300);
        if (rel_converged(mon[0], prev[0], tol) && (!th || rel_converged(mon[1], prev[1], tol))) {
          status = LBM_OK;
          if (k != nsteps) {
            // fields of this step are already written (diag)
          }
          break;
        }
      }
      prev[0] = mon[0];
      prev[1] = mon[1];
      have_prev = true;
    }
  }
  int rc = sweep_end(p, 0, std::min(k, nsteps), s);
  if (rc) return rc;
  double J = 0.0;
  rc = objective_value(p, gamma, u, s, &J);
  if (rc) return rc;
  p->J = J;
  p->fwd_done = true;
  p->have_gneq = true;
  p->adj_done = false;
  if (info) {
    info->steps = std::min(k, nsteps);
    info->status = status;
    info->residual[0] = res[0];
    info->residual[1] = res[1];
    info->monitor[0] = mon[0];
    info->monitor[1] = mon[1];
    info->J = J;
  }
  return status;
}

RebaseArgs rebase_args(lbm_problem* p, const float* T) {
  RebaseArgs A{};
  A.g = p->g[p->fcur];
  A.Rin = p->R[p->rcur];
  A.Rout = p->R[1 - p->rcur];
  A.T = T;
  A.flags = p->flags;
  A.P = p->kp;
  return A;
}

AdjArgs adj_args(lbm_problem* p, const float* gamma, const float* u, const float* T) {
  AdjArgs A{};
  A.ain = p->a[p->acur];
  A.aout = p->a[1 - p->acur];
  A.bin = p->b[p->acur];
  A.bout = p->b[1 - p->acur];
  A.flags = p->flags;
  A.gamma = gamma;
  A.u = u;
  A.T = T;
  A.G = p->G;
  A.partials = p->partials;
  A.P = p->kp;
  return A;
}

int run_adjoint(lbm_problem* p, const float* gamma, const float* u, const float* T, int nsteps,
                int check, double tol, hipStream_t s, lbm_info_t* info) {
  const bool th = thermal_of(p);
  double prev[2] = {0, 0}, res[2] = {0, 0}, mon[2] = {0, 0};
  bool have_prev = false;
  int status = LBM_NOT_CONVERGED, k = 0;
  int rc0 = sweep_begin(p, s);
  if (rc0) return rc0;
  for (k = 1; k <= nsteps; ++k) {
    const bool at_check = check > 0 && k % check == 0;
    const bool diag = at_check || k == nsteps;
    HIPCHK(launch_adjoint(adj_args(p, gamma, u, T), th, p->d.objective, diag, s));
    p->acur = 1 - p->acur;
    if (!diag) continue;
    int rc = read_sums(p, kRedAdj, s);
    if (rc) return rc;
    mon[0] = p->pinned[0] / p->n_nonwall;
    mon[1] = p->pinned[1] / p->n_nonwall;
    if (!std::isfinite(mon[0]) || !std::isfinite(mon[1])) {
      p->adj_done = p->adj_state = false;
      return fail(LBM_EDIVERGED, "adjoint solve diverged at step " + std::to_string(k));
    }
    if (at_check) {
      if (have_prev) {
        res[0] = std::fabs(mon[0] - prev[0]) / std::max(std::fabs(mon[0]), 1e-300);
        res[1] = std::fabs(mon[1] - prev[1]) / std::max(std::fabs(mon[1]), 1e-300);
        if (rel_converged(mon[0], prev[0], tol) && (!th || rel_converged(mon[1], prev[1], tol))) {
          status = LBM_OK;
          break;
        }
      }
      prev[0] = mon[0];
      prev[1] = mon[1];
      have_prev = true;
    }
  }
  int rc = sweep_end(p, 1, std::min(k, nsteps), s);
  if (rc) return rc;
  p->adj_done = p->adj_state = true;
  if (info) {
    info->steps = std::min(k, nsteps);
    info->status = status;
    info->residual[0] = res[0];
    info->residual[1] = res[1];
    info->monitor[0] = mon[0];
    info->monitor[1] = mon[1];
    info->J = p->J;
  }
  return status;
}

// Thermal lattice alone with the velocity frozen, from g_eq(T, u), until the
// mean-T residual criterion or nsteps.
int run_thermal(lbm_problem* p, const float* gamma, const float* u, const float* T, int nsteps,
                int check, double tol, hipStream_t s, lbm_info_t* info) {
  ThermArgs A{};
  A.flags = p->flags;
  A.gamma = gamma;
  A.u = u;
  A.T = T;
  A.gneq = p->gneq;
  A.partials = p->partials;
  A.P = p->kp;
  A.gout = p->g[0];
  A.R = p->R[0];  // the given temperature is the reference throughout the re-solve
  HIPCHK(launch_thermal_init(A, s));
  p->fcur = 0;
  p->rcur = 0;
  double prev = 0, res = 0, mon = 0;
  bool have_prev = false;
  int status = LBM_NOT_CONVERGED, k = 0;
  for (k = 1; k <= nsteps; ++k) {
    const bool at_check = check > 0 && k % check == 0;
    const bool diag = at_check || k == nsteps;
    A.gin = p->g[p->fcur];
    A.gout = p->g[1 - p->fcur];
    HIPCHK(launch_thermal(A, diag, s));
    p->fcur = 1 - p->fcur;
    if (!diag) continue;
    int rc = read_sums(p, kRedFwd, s);
    if (rc) return rc;
    mon = p->pinned[1] / p->n_nonwall;
    if (!std::isfinite(mon)) {
      p->have_gneq = false;
      return fail(LBM_EDIVERGED, "thermal re-solve diverged at step " + std::to_string(k));
    }
    if (at_check) {
      if (have_prev) {
        res = std::fabs(mon - prev) / std::max(std::fabs(mon), 1e-300);
        if (rel_converged(mon, prev, tol)) {
          status = LBM_OK;
          break;
        }
      }
      prev = mon;
      have_prev = true;
    }
  }
  p->have_gneq = true;
  p->fwd_done = false;  // the flow populations are not a forward state any more
  p->adj_done = false;
  p->J = std::nan("");
  if (info) {
    info->steps = std::min(k, nsteps);
    info->status = status;
    info->residual[0] = 0.0;
    info->residual[1] = res;
    info->monitor[0] = 0.0;
    info->monitor[1] = mon;
    info->J = p->J;
  }
  return status;
}

int check_bound(const lbm_problem* p) {
  if (!p) return fail(LBM_EINVAL, "problem is NULL");
  if (!p->ws) return fail(LBM_ESTATE, "no workspace bound");
  if (p->static_ws && !static_owned(p))
    return fail(LBM_ESTATE, "the device's static workspace has been bound to another problem since");
  return LBM_OK;
}

// Adjoint buffer the sensitivity contracts.  The step kernels store the
// post-collision state y_k of step k; the contraction pulls it (S^T).  For the
// discrete adjoint that is the state Eq. (66) takes.  The continuous variant
// steps collision -> streaming -> boundary, so its complete state after step
// k is the post-boundary f*_k, which on design nodes (never ports) equals the
// pulled state of step k - 1: the other buffer.
int sens_buffer(const lbm_problem* p) {
  return p->d.adjoint_kind == LBM_ADJOINT_CONTINUOUS ? 1 - p->acur : p->acur;
}

}  // namespace lbmadj

extern "C" {

const char* lbm_last_error(void) { return last_error().c_str(); }

int lbm_problem_create(const lbm_desc_t* desc, const uint8_t* mask, lbm_problem_t** out) {
  last_error().clear();
  if (!desc || !out) return fail(LBM_EINVAL, "desc or out is NULL");
  *out = nullptr;
  lbm_problem* p = nullptr;
  try {
    p = new lbm_problem();
  } catch (...) {
    return fail(LBM_ENOMEM, "host allocation failed");
  }
  int rc;
  try {
    rc = validate_and_setup(p, *desc, mask);
  } catch (...) {
    rc = fail(LBM_ENOMEM, "host allocation failed");
  }
  if (rc != LBM_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_problem_t* p) {
  if (!p) return 0;
  return layout_of(p).total;
}

int lbm_bind_workspace(lbm_problem_t* p, void* device_ptr, size_t bytes) {
  last_error().clear();
  if (!p || !device_ptr) return fail(LBM_EINVAL, "problem or workspace is NULL");
  const Layout L = layout_of(p);
  if (bytes < L.total) return fail(LBM_EINVAL, "workspace too small");
  static_release(p);
  p->static_ws = false;
  HIPCHK(hipGetDevice(&p->dev));
  char* base = (char*)(((uintptr_t)device_ptr + 255) & ~uintptr_t(255));
  set_workspace(p, base, bytes);
  if (!p->pinned_owned) {
    p->pinned = nullptr;
    HIPCHK(hipHostMalloc((void**)&p->pinned, 16 * sizeof(double), hipHostMallocDefault));
    p->pinned_owned = true;
  }
  std::vector<float> uin(p->Np, 0.0f);
  std::copy(p->uin_host.begin(), p->uin_host.end(), uin.begin());
  std::vector<uint8_t> fl(p->Np, (uint8_t)K_WALL);
  std::copy(p->flags_host.begin(), p->flags_host.end(), fl.begin());
  HIPCHK(hipMemcpy(p->uin, uin.data(), p->Np * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->flags, fl.data(), p->Np, hipMemcpyHostToDevice));
  p->fwd_done = p->adj_done = p->adj_state = false;
  return LBM_OK;
}

int lbm_bind_static_workspace(lbm_problem_t* p) {
  last_error().clear();
  if (!p) return fail(LBM_EINVAL, "problem is NULL");
  const Layout L = layout_of(p);
  if (L.total > kStaticBytes)
    return fail(LBM_EINVAL, "the problem needs " + std::to_string(L.total) +
                                " bytes of workspace; the static workspace holds " +
                                std::to_string(kStaticBytes));
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kStaticDevices) return fail(LBM_EINVAL, "device index out of range");
  void* base = nullptr;
  {
    StaticWorkspace& sw = static_ws();
    std::lock_guard<std::mutex> lk(sw.mu);
    if (!sw.ptr[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      sw.ptr[dev] = ptr;
    }
    base = sw.ptr[dev];
    if (p->static_ws && p->dev >= 0 && p->dev < kStaticDevices && sw.owner[p->dev] == p)
      sw.owner[p->dev] = nullptr;
    sw.owner[dev] = p;
  }
  p->static_ws = true;
  p->dev = dev;
  set_workspace(p, (char*)base, kStaticBytes);
  if (!p->pinned_owned) p->pinned = p->pinned_local;
  // node flags and inlet profile; the padding beyond N is a wall with no inflow
  const size_t pad = (size_t)(p->Np - p->N);
  HIPCHK(hipMemcpy(p->uin, p->uin_host.data(), (size_t)p->N * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->flags, p->flags_host.data(), (size_t)p->N, hipMemcpyHostToDevice));
  HIPCHK(launch_fill(p->uin + p->N, pad, nullptr));
  HIPCHK(launch_fill_u8(p->flags + p->N, pad, (uint8_t)K_WALL, nullptr));
  HIPCHK(hipStreamSynchronize(nullptr));
  p->fwd_done = p->adj_done = p->adj_state = p->have_gneq = false;
  return LBM_OK;
}

int lbm_forward_solve(lbm_problem_t* p, const float* gamma, float* drho, float* u, float* T,
                      lbm_info_t* info, void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!gamma || !drho || !u || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  p->fwd_done = p->adj_done = p->have_gneq = false;
  p->fcur = 0;
  p->rcur = 0;
  HIPCHK(launch_fill(p->f[0], (size_t)qf_of(p) * p->Np, s));
  if (thermal_of(p)) {
    HIPCHK(launch_fill(p->g[0], (size_t)qg_of(p) * p->Np, s));
    HIPCHK(launch_ref_init(p->R[0], p->flags, p->kp, s));
    HIPCHK(launch_heat_init(p->g[0], gamma, p->flags, p->kp, s));
  }
  return run_forward(p, gamma, drho, u, T, p->d.max_steps, p->d.check_every, p->d.tol, s, info);
}

int lbm_forward_continue(lbm_problem_t* p, const float* gamma, int32_t nsteps, float* drho,
                         float* u, float* T, lbm_info_t* info, void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!p->fwd_done) return fail(LBM_ESTATE, "no forward state to continue");
  if (nsteps < 1) return fail(LBM_EINVAL, "nsteps must be >= 1");
  if (!gamma || !drho || !u || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  return run_forward(p, gamma, drho, u, T, nsteps, 0, 0.0, (hipStream_t)stream, info);
}

int lbm_adjoint_solve(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                      const float* T, lbm_info_t* info, void* stream) {
  (void)drho;
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (thermal_of(p) && !p->have_gneq)
    return fail(LBM_ESTATE, "adjoint solve needs lbm_forward_solve or lbm_thermal_resolve first");
  if (!gamma || !u || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  p->adj_done = p->adj_state = false;
  p->acur = 0;
  if (p->d.objective == LBM_OBJ_DISSIPATION)
    HIPCHK(launch_dissipation_source(u, gamma, p->flags, p->G, p->kp, s));
  HIPCHK(launch_fill(p->a[0], (size_t)qf_of(p) * p->Np, s));
  if (thermal_of(p)) HIPCHK(launch_fill(p->b[0], (size_t)qg_of(p) * p->Np, s));
  return run_adjoint(p, gamma, u, T, p->d.max_steps, p->d.check_every, p->d.tol, s, info);
}

int lbm_thermal_resolve(lbm_problem_t* p, const float* gamma, const float* u, const float* T,
                        lbm_info_t* info, void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!thermal_of(p)) return fail(LBM_EINVAL, "the problem has no thermal lattice");
  if (!gamma || !u || !T) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  return run_thermal(p, gamma, u, T, p->d.max_steps, p->d.check_every, p->d.tol, (hipStream_t)stream,
                     info);
}

int lbm_forward_resume(lbm_problem_t* p, const float* gamma, float* drho, float* u, float* T,
                       lbm_info_t* info, void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!p->fwd_done) return fail(LBM_ESTATE, "no forward state to resume");
  if (!gamma || !drho || !u || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  return run_forward(p, gamma, drho, u, T, p->d.max_steps, p->d.check_every, p->d.tol,
                     (hipStream_t)stream, info);
}

int lbm_adjoint_resume(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                       const float* T, lbm_info_t* info, void* stream) {
  (void)drho;
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!p->adj_state) return fail(LBM_ESTATE, "no adjoint state to resume");
  if (thermal_of(p) && !p->have_gneq)
    return fail(LBM_ESTATE, "adjoint resume needs the thermal state of a forward solve");
  if (!gamma || !u || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  if (p->d.objective == LBM_OBJ_DISSIPATION)
    HIPCHK(launch_dissipation_source(u, gamma, p->flags, p->G, p->kp, s));
  return run_adjoint(p, gamma, u, T, p->d.max_steps, p->d.check_every, p->d.tol, s, info);
}

int lbm_levelset_update(lbm_problem_t* p, const float* phi, float* phi_out, const float* dJ,
                        float* gamma, double K, const double* sigma, double vmax,
                        lbm_levelset_info_t* info, void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!phi || !phi_out || !dJ || !gamma || !sigma) return fail(LBM_EINVAL, "null pointer");
  if (phi == phi_out) return fail(LBM_EINVAL, "phi and phi_out must differ (stencil)");
  if (!(K > 0.0) || !(sigma[0] >= 0.0) || !(sigma[1] >= 0.0) || !(sigma[2] >= 0.0) ||
      !(vmax > 0.0 && vmax <= 1.0))
    return fail(LBM_EINVAL, "need K > 0, sigma >= 0, 0 < vmax <= 1");
  if (p->n_design == 0) return fail(LBM_EINVAL, "the problem has no design nodes");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  const float sg[3] = {(float)sigma[0], (float)sigma[1], (float)sigma[2]};
  HIPCHK(launch_levelset_stats(phi, dJ, p->flags, p->partials, p->kp, s));
  rc = read_sums(p, 2, s);
  if (rc) return rc;
  const double scale = p->pinned[0] / p->n_design;  // mean |J'| over the design domain
  const double volume = p->pinned[1] / p->n_design; // fluid fraction (phi >= 0, Eq. 15)
  const double G = volume - vmax;                     // volume constraint of Eq. (10)
  const float inv_scale = scale > 0.0 ? (float)(1.0 / scale) : 0.0f;
  HIPCHK(launch_levelset_lambda(phi, dJ, p->flags, inv_scale, sg, p->partials, p->kp, s));
  rc = read_sums(p, 1, s);
  if (rc) return rc;
  const double lambda = std::exp(G) * p->pinned[0] / p->n_design;  // Eq. (67)
  // Semi-implicit step (I - K lap_sigma) phi_new = phi - K (J'/scale + lambda),
  // solved by red-black Gauss-Seidel.  The Jacobi iteration of this diagonally
  // dominant system contracts by rho = b / (1 + b) per sweep, b = 2 K (sigma_x +
  // sigma_y + sigma_z) bounding K times any row's neighbour weight; red-black
  // ordering squares that, so the sweep count brings the error below 1e-8 of
  // the starting guess's.
  const double b = 2.0 * K * (sigma[0] + sigma[1] + sigma[2]);
  int sweeps = 0;
  if (b > 0.0) {
    const double rho = b / (1.0 + b);
    const double n_sw = std::ceil(std::log(1e-8) / (2.0 * std::log(rho))) + 8.0;
    if (!(n_sw <= 100000.0)) return fail(LBM_EINVAL, "K * sigma too large for the level-set solve");
    sweeps = (int)n_sw;
  }
  HIPCHK(launch_levelset_update(phi, phi_out, dJ, p->flags, gamma, inv_scale, (float)K, (float)lambda,
                                sg, sweeps, p->kp, s));
  if (info) {
    info->lambda = lambda;
    info->volume = volume;
    info->G = G;
    info->scale = scale;
  }
  return LBM_OK;
}

int lbm_adjoint_continue(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                         const float* T, int32_t nsteps, lbm_info_t* info, void* stream) {
  (void)drho;
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!p->adj_done) return fail(LBM_ESTATE, "no adjoint state to continue");
  if (nsteps < 1) return fail(LBM_EINVAL, "nsteps must be >= 1");
  if (!gamma || !u || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  if (p->d.objective == LBM_OBJ_DISSIPATION)
    HIPCHK(launch_dissipation_source(u, gamma, p->flags, p->G, p->kp, s));
  return run_adjoint(p, gamma, u, T, nsteps, 0, 0.0, s, info);
}

int lbm_sensitivity(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                    const float* T, float* dJdgamma, double* J, void* stream) {
  (void)drho;
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!p->adj_done) return fail(LBM_ESTATE, "sensitivity needs an adjoint solve first");
  if (!gamma || !u || !dJdgamma || (thermal_of(p) && !T)) return fail(LBM_EINVAL, "null field pointer");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  SensArgs A{};
  A.ain = p->a[sens_buffer(p)];
  A.bin = p->b[p->acur];
  A.flags = p->flags;
  A.gamma = gamma;
  A.u = u;
  A.T = T;
  A.gneq = p->gneq;
  A.dJ = dJdgamma;
  A.partials = p->partials;
  A.objective = p->d.objective;
  A.P = p->kp;
  HIPCHK(launch_sensitivity(A, thermal_of(p), s));
  rc = read_sums(p, kRedSens, s);
  if (rc) return rc;
  if (J) *J = p->J;
  return LBM_OK;
}

int lbm_copy_state(const lbm_problem_t* p, int32_t which, float* dst, void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!dst) return fail(LBM_EINVAL, "dst is NULL");
  const float* src = nullptr;
  int q = 0;
  switch (which) {
    case 0: src = p->f[p->fcur]; q = qf_of(p); break;
    case 1: src = p->g[p->fcur]; q = qg_of(p); break;
    case 2: src = p->a[p->acur]; q = qf_of(p); break;
    case 3: src = p->b[p->acur]; q = qg_of(p); break;
    case 4: src = p->gneq; q = qg_of(p); break;
    default: return fail(LBM_EINVAL, "which must be 0..4");
  }
  if (!src) return fail(LBM_EINVAL, "no such state for this problem");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < q; ++i)
    HIPCHK(hipMemcpyAsync(dst + (size_t)i * p->N, src + (size_t)i * p->Np, (size_t)p->N * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
  // the forward thermal state is kept relative to a per-node reference;
  // export it in the shift of T_in
  if (which == 1) HIPCHK(launch_export_thermal(src, p->R[p->rcur], p->flags, dst, p->kp, s));
  return LBM_OK;
}

int lbm_set_kernel_timing(lbm_problem_t* p, int32_t enable) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  DeviceGuard guard(p->dev);
  if (enable && !p->sweep_ev[0]) {
    HIPCHK(hipEventCreate(&p->sweep_ev[0]));
    HIPCHK(hipEventCreate(&p->sweep_ev[1]));
  }
  p->timing = enable != 0;
  return LBM_OK;
}

int lbm_kernel_timing(lbm_problem_t* p, double* ms, int64_t* launches, int32_t reset) {
  last_error().clear();
  if (!p || !ms || !launches) return fail(LBM_EINVAL, "null argument");
  for (int k = 0; k < 2; ++k) {
    ms[k] = p->t_ms[k];
    launches[k] = p->t_n[k];
    if (reset) {
      p->t_ms[k] = 0.0;
      p->t_n[k] = 0;
    }
  }
  return LBM_OK;
}

int lbm_copy_probe(const void* src, void* dst, uint64_t bytes, int32_t launches,
                   double* us_per_launch, void* stream) {
  last_error().clear();
  if (!src || !dst || !us_per_launch) return fail(LBM_EINVAL, "null argument");
  if (((uintptr_t)src | (uintptr_t)dst) & 15u) return fail(LBM_EINVAL, "buffers must be 16-byte aligned");
  if (bytes == 0 || (bytes & 15u)) return fail(LBM_EINVAL, "bytes must be a positive multiple of 16");
  if (launches < 1 || launches > 1000000) return fail(LBM_EINVAL, "launches must be in [1, 1000000]");
  const char* s0 = (const char*)src;
  const char* d0 = (const char*)dst;
  if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(LBM_EINVAL, "buffers overlap");
  hipStream_t s = (hipStream_t)stream;
  const size_t n16 = (size_t)(bytes / 16);
  for (int i = 0; i < 3; ++i) HIPCHK(launch_copy16(src, dst, n16, s));
  hipEvent_t ev[2];
  HIPCHK(hipEventCreate(&ev[0]));
  hipError_t e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(LBM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  e = hipEventRecord(ev[0], s);
  for (int i = 0; i < launches && e == hipSuccess; ++i) e = launch_copy16(src, dst, n16, s);
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("copy probe: ") + hipGetErrorString(e));
  *us_per_launch = (double)ms * 1e3 / launches;
  return LBM_OK;
}

int lbm_stream_probe(lbm_problem_t* p, const float* gamma, int32_t launches, double* us_per_launch,
                     void* stream) {
  last_error().clear();
  int rc = check_bound(p);
  if (rc) return rc;
  if (!gamma || !us_per_launch) return fail(LBM_EINVAL, "null argument");
  if (launches < 1 || launches > 1000000) return fail(LBM_EINVAL, "launches must be in [1, 1000000]");
  DeviceGuard guard(p->dev);
  hipStream_t s = (hipStream_t)stream;
  // the probe overwrites both forward buffers: no state survives it
  p->fwd_done = p->adj_done = p->adj_state = p->have_gneq = false;
  p->fcur = 0;
  FwdArgs a = fwd_args(p, gamma, nullptr, nullptr, nullptr);
  int cur = 0;
  auto swap_ab = [&]() {
    cur = 1 - cur;
    a.fin = p->f[cur];
    a.fout = p->f[1 - cur];
    a.gin = p->g[cur];
    a.gout = p->g[1 - cur];
  };
  for (int i = 0; i < 10; ++i) {
    HIPCHK(launch_stream_probe(a, thermal_of(p), s));
    swap_ab();
  }
  hipEvent_t ev[2];
  HIPCHK(hipEventCreate(&ev[0]));
  hipError_t e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(LBM_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
  }
  e = hipEventRecord(ev[0], s);
  for (int i = 0; i < launches && e == hipSuccess; ++i) {
    e = launch_stream_probe(a, thermal_of(p), s);
    swap_ab();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("stream probe: ") + hipGetErrorString(e));
  *us_per_launch = 1e3 * (double)ms / launches;
  return LBM_OK;
}

int lbm_lattice(int32_t which, int32_t* e, double* w) {
  if (!e || !w || which < 0 || which > 3) return fail(LBM_EINVAL, "bad arguments");
  lattice_table(which, e, w);
  return LBM_OK;
}

void lbm_problem_destroy(lbm_problem_t* p) {
  if (!p) return;
  if (p->dev >= 0 && p->sweep_ev[0]) {
    DeviceGuard guard(p->dev);
    (void)hipEventDestroy(p->sweep_ev[0]);
    (void)hipEventDestroy(p->sweep_ev[1]);
  }
  static_release(p);
  if (p->pinned && p->pinned_owned) (void)hipHostFree(p->pinned);
  delete p;
}

}  // extern "C"
