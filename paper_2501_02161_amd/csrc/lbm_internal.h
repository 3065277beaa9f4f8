// Internal interface between the C-ABI host code (lbm_host.hip) and the
// gfx950 kernels (lbm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lbmadj.h"

namespace lbmadj {

constexpr int kBlock = 256;      // threads per block: 4 wave64s
constexpr int kRedFwd = 4;       // forward partial sums: |u|, T, inlet drho, layer T
constexpr int kRedAdj = 2;       // adjoint partial sums: |sum e a|, |sum b|
constexpr int kRedSens = 2;      // sensitivity partial sums: dJ, dJ^2
constexpr int kRedDiss = 1;      // dissipation objective

// Node flag byte on the device: bits 0-2 kind, 3-5 inward-normal code (as in
// the mask), bit 6 = node of the heat-sink objective layer.
enum : int { K_DESIGN = 0, K_FLUID = 1, K_INLET = 2, K_OUTLET = 3, K_WALL = 4, K_HEATED = 5, K_SYM = 6 };
constexpr unsigned kLayerBit = 0x40u;

enum : int { OBJ_PRESSURE_DROP = 0, OBJ_DISSIPATION = 1, OBJ_HEATSINK = 2, OBJ_HEATGEN = 3 };

// Per-problem constants handed to every kernel by value.
struct KParams {
  int nx, ny, nz, N, Np, plane;  // grid, node count, population stride, nx*ny
  int px, py, pz;                // periodic axes
  int nblk, xcd_per, xcd_rem;    // block count and its split over the 8 XCDs
  float omega;                   // 1/tau
  float rho0;
  float tab;                     // tau * alpha_max * q   (chi = 1 - tab (1-g)/(q+g))
  float amq;                     // alpha_max * q         (a_B = amq (1-g)/(q+g))
  float qb;                      // q of the Brinkman interpolation
  float dfc;                     // (nu/Pr)/cs2 of D3Q7: tau_g = 1/2 + dfc k(g)
  float kr, qr;                  // conductivity ratio and RAMP parameter
  float q_w;                     // heat flux per heated wall node and step
  float T_in;                    // inlet (Dirichlet) temperature
  float c_in;                    // w_dp / (3 N_inlet): dJ/df_i at inlet nodes
  float c_layer;                 // 1 / N_layer: dJ/dg_i at objective-layer nodes
  float two_nu;                  // 2 nu (dissipation source)
  float nu;
  int cont;                      // adjoint: 1 = continuous variant (flow lattice only)
  int sx, sy, sz;                // mirror plane before the last layer of the axis
  int pin;                       // 1: inlets are pressure inlets at rho0 + drho_in
  float drho_in;
  float beta;                    // heat generation beta_max (0: none)
  int heatgen;                   // objective J = -sum beta (1 - T): forward partial 3
  int q;                         // flow lattice: 19 (D3Q19) or 9 (D2Q9, nz = 1)
};

// Thermal populations are stored relative to a per-node reference
// temperature R: the slot of population i at node x holds g_i - w_i R(x), and
// a pull from node y adds w_i (R(y) - R(x)).  Wall nodes hold R = +inf and
// carry the values they bounce back in the shift of the node that reads them
// (no term is added across a wall).  R is re-based onto the current
// temperature at every residual check of a forward sweep (k_rebase), which
// keeps the stored values at the size of their deviations from the local
// temperature, so their FP32 rounding does not stall the slow approach to the
// steady state.
struct FwdArgs {
  const float* fin;
  float* fout;
  const float* gin;
  float* gout;
  const float* Rin;     // reference temperature per node (thermal), read only in a step
  const uint8_t* flags;
  const float* gamma;
  const float* uin;     // prescribed normal inlet speed per node
  float* drho;          // outputs (diagnostic step only)
  float* u;
  float* T;
  float* gneq;
  double* partials;
  KParams P;
};

struct AdjArgs {
  const float* ain;     // adjoint flow state (after the adjoint BC), 19 (2D: 9) x Np
  float* aout;
  const float* bin;     // adjoint thermal state, 7 (2D: 5) x Np
  float* bout;
  const uint8_t* flags;
  const float* gamma;
  const float* u;       // [3][N] forward velocity
  const float* T;       // [N] forward temperature
  const float* G;       // [3][Np] dissipation source (dJ/du / rho0)
  double* partials;
  KParams P;
};

struct SensArgs {
  const float* ain;
  const float* bin;
  const uint8_t* flags;
  const float* gamma;
  const float* u;
  const float* T;
  const float* gneq;    // 7 (2D: 5) x Np
  float* dJ;
  double* partials;
  int objective;
  KParams P;
};

// Thermal lattice alone, advected by a frozen velocity field.
struct ThermArgs {
  const float* gin;
  float* gout;
  float* R;             // reference temperature per node (the given T; +inf at walls)
  const uint8_t* flags;
  const float* gamma;
  const float* u;       // [3][N] frozen velocity
  const float* T;       // [N] initial temperature (init kernel only)
  float* gneq;          // 7 (2D: 5) x Np (diagnostic step)
  double* partials;
  KParams P;
};

// Re-base of a forward thermal state (in place on g) from the reference Rin
// onto the temperature field T, writing the new reference to Rout.
struct RebaseArgs {
  float* g;
  const float* Rin;
  float* Rout;
  const float* T;
  const uint8_t* flags;
  KParams P;
};

// Ragged batch: one slot per resident problem, one tile per 256-node block of
// a slot.  A batch launch advances every slot in the forward or adjoint phase
// by one step; the slot's step in its phase is (launch - start), where the
// launch index is *base + q (a per-lane device counter plus the launch's place
// in its quantum); the A/B buffers alternate with the step's parity (even
// steps read buffer 0).
struct SlotDev {
  int phase;        // 0 idle, 1 forward, 2 adjoint
  int start;        // launch index of the phase's first step
  int max_steps;
  int check;        // residual check period (0: only the last step)
  FwdArgs fa;       // fin/gin = buffer 0, fout/gout = buffer 1, Rin = reference buffer 0
  AdjArgs aa;       // ain/bin = buffer 0, aout/bout = buffer 1
  float* R1;        // reference buffer 1 (the forward re-bases at every diagnostic step)
};
struct Tile {
  int slot;
  int blk;
};

// Launchers (return the hipError_t of the launch).
hipError_t launch_fill(float* p, size_t count, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, size_t count, uint8_t value, hipStream_t s);
// Copy of n16 16-byte words (dwordx4 loads and stores); both pointers 16-byte aligned.
hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t s);
// Level-set design update (per-block FP64 partials: stats 2 values, lambda 1).
hipError_t launch_levelset_stats(const float* phi, const float* dJ, const uint8_t* flags,
                                 double* partials, const KParams& P, hipStream_t s);
hipError_t launch_levelset_lambda(const float* phi, const float* dJ, const uint8_t* flags,
                                  float inv_scale, const float* sigma, double* partials,
                                  const KParams& P, hipStream_t s);
// Semi-implicit step: r = phi - K (J'/scale + lambda) into phi_out, `sweeps`
// red-black Gauss-Seidel sweeps of (I - K lap_sigma) x = r in place
// (sigma[3]: per-axis coefficients, host array), then the clamp and
// gamma = (phi_out >= 0).
hipError_t launch_levelset_update(const float* phi, float* phi_out, const float* dJ,
                                  const uint8_t* flags, float* gamma, float inv_scale, float K,
                                  float lambda, const float* sigma, int sweeps, const KParams& P,
                                  hipStream_t s);
// Adds the first collision's heat source to a zero-filled thermal state
// (no-op without heat generation).
hipError_t launch_heat_init(float* g, const float* gamma, const uint8_t* flags, const KParams& P,
                            hipStream_t s);
// Reference temperature of a forward start: T_in at non-wall nodes, +inf at walls.
hipError_t launch_ref_init(float* R, const uint8_t* flags, const KParams& P, hipStream_t s);
// Re-base of a forward thermal state (see RebaseArgs).
hipError_t launch_rebase(const RebaseArgs& a, hipStream_t s);
// Thermal state in the shift of T_in (g_i - w_i T_in, node-major planes of N
// floats) from the stored per-node-reference form (src planes of Np floats).
hipError_t launch_export_thermal(const float* src, const float* R, const uint8_t* flags, float* dst,
                                 const KParams& P, hipStream_t s);
// Batch form of the re-base: every slot whose step `*base + q - start` was a
// diagnostic forward step re-bases its tiles.
hipError_t launch_batch_rebase(const Tile* tiles, int ntiles, const SlotDev* slots, const int* base,
                               int q, hipStream_t s);
// Step kernels; with non-null events the launch records them at the start and
// end of the kernel itself (hipExtLaunchKernelGGL), for per-launch timing.
hipError_t launch_forward(const FwdArgs& a, bool thermal, bool diag, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_adjoint(const AdjArgs& a, bool thermal, int objective, bool diag, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_sensitivity(const SensArgs& a, bool thermal, hipStream_t s);
hipError_t launch_thermal(const ThermArgs& a, bool diag, hipStream_t s);
// The forward step's pulls and stores with no arithmetic (fin -> fout, gin -> gout).
hipError_t launch_stream_probe(const FwdArgs& a, bool thermal, hipStream_t s);
hipError_t launch_thermal_init(const ThermArgs& a, hipStream_t s);
hipError_t launch_dissipation_source(const float* u, const float* gamma, const uint8_t* flags,
                                     float* G, const KParams& P, hipStream_t s);
hipError_t launch_dissipation_objective(const float* u, const float* gamma, const uint8_t* flags,
                                        double* partials, const KParams& P, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nblk, int nvals, double* out,
                           hipStream_t s);
hipError_t launch_batch(const Tile* tiles, int ntiles, const SlotDev* slots, const int* base,
                        int q, bool thermal, int objective, hipStream_t s);
// Persistent form of a quantum: one cooperative launch of `grid` resident
// blocks (at most persistent_grid_limit(), capped at ntiles) that steps every
// slot Q times with a grid barrier between steps and re-bases the thermal
// states of diagnostic steps at the end.  *bar must be 0 at launch; *abort is
// raised (and the launch leaves early) if a barrier wait exceeds spin_limit
// polls.
hipError_t launch_batch_persistent(const Tile* tiles, int ntiles, const SlotDev* slots,
                                   const int* base, int Q, bool thermal, int objective,
                                   unsigned* bar, int* abort, int spin_limit, int grid,
                                   hipStream_t s);
// Blocks of the persistent kernel that fit on the device at once (0 if unknown).
int persistent_grid_limit(bool thermal, int objective);
// *base += q on the device (end of a quantum of q launches).
hipError_t launch_advance(int* base, int q, hipStream_t s);
// Per-slot residual sums of the slots' last diagnostic step: out[slot * 4 + v].
hipError_t launch_finalize_slots(const SlotDev* slots, int nslots, double* out, hipStream_t s);

// Host-side copies of the direction tables (for lbm_lattice).
void lattice_table(int which, int32_t* e, double* w);

// ---------------------------------------------------------------------------
// Host-side helpers shared by the single-problem ABI and the batch engine.
// ---------------------------------------------------------------------------
std::string& last_error();
inline int fail(int code, const std::string& msg) {
  last_error() = msg;
  return code;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::lbmadj::fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int NVEC_HOST[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace lbmadj

// One lattice problem: validated description, host-side node data and the
// pointers into its bound workspace.
struct lbm_problem {
  lbm_desc_t d{};
  int N = 0, Np = 0, nblk = 0;
  std::vector<uint8_t> flags_host;
  std::vector<float> uin_host;
  int n_inlet = 0, n_layer = 0, n_nonwall = 0, n_design = 0;
  lbmadj::KParams kp{};
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int dev = -1;
  float* f[2] = {nullptr, nullptr};
  float* g[2] = {nullptr, nullptr};
  float* a[2] = {nullptr, nullptr};
  float* b[2] = {nullptr, nullptr};
  float* R[2] = {nullptr, nullptr};  // reference temperature of the thermal state (rcur current)
  int rcur = 0;
  float* gneq = nullptr;
  float* G = nullptr;
  float* uin = nullptr;
  uint8_t* flags = nullptr;
  double* partials = nullptr;
  double* sums = nullptr;
  double* pinned = nullptr;        // host copy of the reduction sums
  bool pinned_owned = false;       // pinned was allocated by lbm_bind_workspace
  double pinned_local[16] = {};    // pageable stand-in of the allocation-free binding
  bool static_ws = false;          // bound to the device's static workspace
  int fcur = 0, acur = 0;
  bool fwd_done = false, adj_done = false;
  bool adj_state = false;  // the adjoint populations hold a finished adjoint solve (resumable)
  bool have_gneq = false;  // thermal non-equilibrium of a converged state in the workspace
  double J = 0.0;
  // sweep timing: one event pair around each forward / adjoint sweep
  bool timing = false;
  hipEvent_t sweep_ev[2] = {nullptr, nullptr};
  double t_ms[2] = {0.0, 0.0};
  long long t_n[2] = {0, 0};
};

namespace lbmadj {

// Workspace regions of a problem (byte offsets, 256-byte aligned).
struct Layout {
  size_t f[2], g[2], a[2], b[2], R[2], gneq, G, uin, flags, partials, sums, total;
};
Layout layout_of(const lbm_problem* p);
bool thermal_of(const lbm_problem* p);
int qf_of(const lbm_problem* p);  // flow directions: 19, or 9 for a 2D lattice
int qg_of(const lbm_problem* p);  // thermal directions: 7, or 5 for a 2D lattice
int sens_buffer(const lbm_problem* p);  // adjoint buffer the sensitivity contracts
int validate_and_setup(lbm_problem* p, const lbm_desc_t& d, const uint8_t* mask);
FwdArgs fwd_args(lbm_problem* p, const float* gamma, float* drho, float* u, float* T);
AdjArgs adj_args(lbm_problem* p, const float* gamma, const float* u, const float* T);
RebaseArgs rebase_args(lbm_problem* p, const float* T);  // re-base of g[fcur] from R[rcur]
bool rel_converged(double now, double before, double tol);

}  // namespace lbmadj
