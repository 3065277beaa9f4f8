// Internal interface between the C-ABI host code (lbm_host.hip) and the
// gfx950 kernels (lbm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmadj {

constexpr int kBlock = 256;      // threads per block: 4 wave64s
constexpr int kRedFwd = 4;       // forward partial sums: |u|, T, inlet drho, layer T
constexpr int kRedAdj = 2;       // adjoint partial sums: |sum e a|, |sum b|
constexpr int kRedSens = 2;      // sensitivity partial sums: dJ, dJ^2
constexpr int kRedDiss = 1;      // dissipation objective

// Node flag byte on the device: bits 0-2 kind, 3-5 inward-normal code (as in
// the mask), bit 6 = node of the heat-sink objective layer.
enum : int { K_DESIGN = 0, K_FLUID = 1, K_INLET = 2, K_OUTLET = 3, K_WALL = 4, K_HEATED = 5 };
constexpr unsigned kLayerBit = 0x40u;

enum : int { OBJ_PRESSURE_DROP = 0, OBJ_DISSIPATION = 1, OBJ_HEATSINK = 2 };

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
  float T_ref;                   // thermal shift (= T_in)
  float dT_in;                   // T_in - T_ref
  float c_in;                    // w_dp / (3 N_inlet): dJ/df_i at inlet nodes
  float c_layer;                 // 1 / N_layer: dJ/dg_i at objective-layer nodes
  float two_nu;                  // 2 nu (dissipation source)
  float nu;
};

struct FwdArgs {
  const float* fin;
  float* fout;
  const float* gin;
  float* gout;
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
  const float* ain;     // adjoint flow state (after the adjoint BC), 19 x Np
  float* aout;
  const float* bin;     // adjoint thermal state, 7 x Np
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
  const float* gneq;    // 7 x Np
  float* dJ;
  double* partials;
  int objective;
  KParams P;
};

// Launchers (return the hipError_t of the launch).
hipError_t launch_fill(float* p, size_t count, hipStream_t s);
// Step kernels; with non-null events the launch records them at the start and
// end of the kernel itself (hipExtLaunchKernelGGL), for per-launch timing.
hipError_t launch_forward(const FwdArgs& a, bool thermal, bool diag, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_adjoint(const AdjArgs& a, bool thermal, int objective, bool diag, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_sensitivity(const SensArgs& a, bool thermal, hipStream_t s);
hipError_t launch_dissipation_source(const float* u, const float* gamma, const uint8_t* flags,
                                     float* G, const KParams& P, hipStream_t s);
hipError_t launch_dissipation_objective(const float* u, const float* gamma, const uint8_t* flags,
                                        double* partials, const KParams& P, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nblk, int nvals, double* out,
                           hipStream_t s);

// Host-side copies of the direction tables (for lbm_lattice).
void lattice_table(int which, int32_t* e, double* w);

}  // namespace lbmadj
