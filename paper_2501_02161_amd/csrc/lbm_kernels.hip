// gfx950 kernels of the steady discrete adjoint lattice Boltzmann method
// (arXiv 2501.02161): the fused forward step (streaming, boundary conditions,
// collision of Eq. 35 for D3Q19 and the coupled D3Q7 lattice), the fused
// adjoint step (Eqs. 54-56 in reverse: reversed pull of Eq. 61, adjoint
// collision of Eq. 65, local adjoint boundary condition), the sensitivity of
// Eq. (66) and FP64 wave-shuffle reductions.
//
// Data layout: populations are structure-of-arrays, plane q at q*Np, node
// n = x + nx*(y + ny*z), so the 64 lanes of a wave touch 64 consecutive
// floats of each population plane.  Every kernel is a pull: each stored value
// is read by exactly one thread per step (there is no reuse to stage in LDS);
// the only cross-lane sharing is the +-1 misalignment of the x-neighbour
// loads, which the L2 absorbs because consecutive blocks are mapped to the
// same XCD.  Forward populations are stored shifted, f_i - w_i rho0 and
// g_i - w_i T_ref, to keep FP32 resolution on the small deviations.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbm_internal.h"

namespace lbmadj {
namespace {

// ----------------------------------------------------------------------------
// Velocity sets.  D3Q19 weights of Eq. (5); order: rest, the six axis
// directions (+x,-x,+y,-y,+z,-z), then the twelve edge diagonals in opposite
// pairs.  D3Q7 for temperature: rest 1/4, axes 1/8 (cs2 = 1/4).  In both sets
// the axis direction with normal code c (+x 0, -x 1, ... -z 5) is index c + 1.
// ----------------------------------------------------------------------------
struct Q19 {
  static constexpr int Q = 19;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr float w[19] = {1.f / 3.f,  1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                                  1.f / 18.f, 1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                  1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                  1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};
// D2Q9 (the 2D flow lattice, nz = 1): rest 4/9, axes 1/9, diagonals 1/36, in
// the same axis-first order with ez = 0.
struct Q9 {
  static constexpr int Q = 9;
  static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
  static constexpr float w[9] = {4.f / 9.f,  1.f / 9.f,  1.f / 9.f,  1.f / 9.f, 1.f / 9.f,
                                 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
};
struct Q7 {
  static constexpr int Q = 7;
  static constexpr int ex[7] = {0, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[7] = {0, 0, 0, 1, -1, 0, 0};
  static constexpr int ez[7] = {0, 0, 0, 0, 0, 1, -1};
  static constexpr int opp[7] = {0, 2, 1, 4, 3, 6, 5};
  static constexpr float w[7] = {0.25f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f, 0.125f};
};
// D2Q5, the thermal lattice of a 2D problem: rest 1/2, axes 1/8, so that
// cs2 = 1/4 as on D3Q7 (same equilibrium and relaxation time).
struct Q5 {
  static constexpr int Q = 5;
  static constexpr int ex[5] = {0, 1, -1, 0, 0};
  static constexpr int ey[5] = {0, 0, 0, 1, -1};
  static constexpr int ez[5] = {0, 0, 0, 0, 0};
  static constexpr int opp[5] = {0, 2, 1, 4, 3};
  static constexpr float w[5] = {0.5f, 0.125f, 0.125f, 0.125f, 0.125f};
};
// Thermal lattice paired with a flow lattice.
template <class L>
struct ThermalOf {
  using type = Q7;
};
template <>
struct ThermalOf<Q9> {
  using type = Q5;
};

template <int V>
using ic = std::integral_constant<int, V>;

// Compile-time loop: f(ic<0>), ..., f(ic<N-1>), so that every population
// index is a constant and the arrays stay in registers.
template <int I, int N, class F>
__device__ __forceinline__ void sfor_impl(F& f) {
  if constexpr (I < N) {
    f(ic<I>{});
    sfor_impl<I + 1, N>(f);
  }
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl<0, N>(f);
}

// Block index -> logical tile: blocks are dealt round-robin to the 8 XCDs,
// so give each XCD a contiguous run of tiles (its L2 then sees the x/y
// neighbour lines of adjacent tiles).
__device__ __forceinline__ int remap_block(int b, const KParams& P) {
  const int xcd = b & 7, idx = b >> 3;
  return xcd < P.xcd_rem ? xcd * (P.xcd_per + 1) + idx
                         : P.xcd_rem * (P.xcd_per + 1) + (xcd - P.xcd_rem) * P.xcd_per + idx;
}

// Neighbour coordinates of one node for offsets -1, 0, +1 along each axis,
// wrapped on periodic axes and flagged invalid beyond a non-periodic face
// (reads there return 0: only wall populations that point out of the box and
// port unknowns, which the boundary rule overwrites, come from outside).
struct Nbr {
  int X[3], Yo[3], Zo[3];
  bool vx[3], vy[3], vz[3];
};

__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, const KParams& P) {
  Nbr b;
  b.X[1] = x;
  b.vx[1] = true;
  b.X[0] = x - 1;
  b.vx[0] = true;
  b.X[2] = x + 1;
  b.vx[2] = true;
  if (x == 0) {
    if (P.px) b.X[0] = P.nx - 1; else b.vx[0] = false;
  }
  if (x == P.nx - 1) {
    if (P.px) b.X[2] = 0; else b.vx[2] = false;
  }
  int Y[3] = {y - 1, y, y + 1};
  b.vy[0] = b.vy[1] = b.vy[2] = true;
  if (y == 0) {
    if (P.py) Y[0] = P.ny - 1; else b.vy[0] = false;
  }
  if (y == P.ny - 1) {
    if (P.py) Y[2] = 0; else b.vy[2] = false;
  }
  int Z[3] = {z - 1, z, z + 1};
  b.vz[0] = b.vz[1] = b.vz[2] = true;
  if (z == 0) {
    if (P.pz) Z[0] = P.nz - 1; else b.vz[0] = false;
  }
  if (z == P.nz - 1) {
    if (P.pz) Z[2] = 0; else b.vz[2] = false;
  }
  for (int k = 0; k < 3; ++k) {
    b.Yo[k] = Y[k] * P.nx;
    b.Zo[k] = Z[k] * P.plane;
  }
  return b;
}

// Value of plane `base` at node + (DX, DY, DZ), 0 outside the box.
template <int DX, int DY, int DZ>
__device__ __forceinline__ float load_nbr(const float* __restrict__ base, const Nbr& b, int n) {
  const bool v = b.vx[DX + 1] && b.vy[DY + 1] && b.vz[DZ + 1];
  const int s = v ? b.X[DX + 1] + b.Yo[DY + 1] + b.Zo[DZ + 1] : n;
  const float r = base[s];
  return v ? r : 0.0f;
}

// Direction index of lattice L with velocity (ex, ey, ez), and of direction I
// reflected in the axes of mask M (bit 0 x, 1 y, 2 z).
template <class L>
constexpr int find_dir(int ex, int ey, int ez) {
  for (int i = 0; i < L::Q; ++i)
    if (L::ex[i] == ex && L::ey[i] == ey && L::ez[i] == ez) return i;
  return -1;
}
template <class L, int I, int M>
constexpr int mirror_dir() {
  return find_dir<L>((M & 1) ? -L::ex[I] : L::ex[I], (M & 2) ? -L::ey[I] : L::ey[I],
                     (M & 4) ? -L::ez[I] : L::ez[I]);
}

// Whether the + neighbour along each axis is the layer beyond a mirror plane.
struct Mirror {
  bool x, y, z;
};
// Problems without mirror planes are compiled with MIR = false, which makes
// every Mirror constant false and folds the reflection selects away.
__device__ __forceinline__ bool has_mirror(const KParams& P) { return (P.sx | P.sy | P.sz) != 0; }
__device__ __forceinline__ Mirror mirror_of(int x, int y, int z, const KParams& P) {
  Mirror m;
  m.x = P.sx && x == P.nx - 2;
  m.y = P.sy && y == P.ny - 2;
  m.z = P.sz && z == P.nz - 2;
  return m;
}

// Population I pulled from the neighbour n + (DX, DY, DZ) (zero beyond a
// non-periodic face).  Where that neighbour lies beyond a mirror plane (only
// possible on the + side of an axis), the mirror image is read instead: the
// node's own layer along that axis and direction I reflected in it (specular
// reflection at the plane midway between the two layers; the quarter-domain
// heat sink).  Forward pulls use (-e_I), adjoint pulls (+e_I); in both the
// reflected slot is the transpose of the other's.
// Where population I of node n is pulled from: the neighbour n + (DX, DY, DZ)
// and slot I, or for a neighbour beyond a mirror plane the node's own layer
// along that axis and the reflected slot; `valid` is false beyond a
// non-periodic face (then node = n, and the pulled value is 0).
struct Src {
  int slot;
  int node;
  bool valid;
};
template <class L, int I, int DX, int DY, int DZ>
__device__ __forceinline__ Src pull_src(const Nbr& b, int n, const Mirror& m) {
  if constexpr (DX != 1 && DY != 1 && DZ != 1) {
    const bool v = b.vx[DX + 1] && b.vy[DY + 1] && b.vz[DZ + 1];
    return Src{I, v ? b.X[DX + 1] + b.Yo[DY + 1] + b.Zo[DZ + 1] : n, v};
  } else {
    const bool rx = (DX == 1) && m.x, ry = (DY == 1) && m.y, rz = (DZ == 1) && m.z;
    constexpr int I1 = mirror_dir<L, I, 1>(), I2 = mirror_dir<L, I, 2>(), I3 = mirror_dir<L, I, 3>();
    constexpr int I4 = mirror_dir<L, I, 4>(), I5 = mirror_dir<L, I, 5>(), I6 = mirror_dir<L, I, 6>();
    constexpr int I7 = mirror_dir<L, I, 7>();
    const int p = rz ? (ry ? (rx ? I7 : I6) : (rx ? I5 : I4)) : (ry ? (rx ? I3 : I2) : (rx ? I1 : I));
    const int X = rx ? b.X[1] : b.X[DX + 1];
    const int Yo = ry ? b.Yo[1] : b.Yo[DY + 1];
    const int Zo = rz ? b.Zo[1] : b.Zo[DZ + 1];
    const bool v = (rx || b.vx[DX + 1]) && (ry || b.vy[DY + 1]) && (rz || b.vz[DZ + 1]);
    return Src{p, v ? X + Yo + Zo : n, v};
  }
}

template <class L, int I, int DX, int DY, int DZ>
__device__ __forceinline__ float load_pull(const float* __restrict__ base, size_t Np, const Nbr& b,
                                           int n, const Mirror& m) {
  const Src sr = pull_src<L, I, DX, DY, DZ>(b, n, m);
  const float r = base[(size_t)sr.slot * Np + sr.node];
  return sr.valid ? r : 0.0f;
}

// A reference temperature of +inf marks a wall node.
__device__ __forceinline__ bool ref_is_node(float R) { return R <= 3.0e38f; }

// Forward thermal pull in the per-node reference form: the value of slot I
// pulled from its source node, moved into node n's shift by
// w_I (R(source) - R(n)) unless the source or node n is a wall (walls hold
// their values in the shift of the node that reads them).  Split in two so
// that a caller issues the loads of every direction before it uses any
// (one memory round trip for the whole pull): RefPull holds what one
// direction read, ref_pull_value moves it into node n's shift.
struct RefPull {
  float r, Rs;
  bool valid;
};
template <class G, int I, int DX, int DY, int DZ>
__device__ __forceinline__ RefPull load_ref_pull(const float* __restrict__ base,
                                                 const float* __restrict__ R, size_t Np,
                                                 const Nbr& b, int n, const Mirror& m) {
  if constexpr (DX == 0 && DY == 0 && DZ == 0) {
    return RefPull{base[(size_t)I * Np + n], 0.0f, true};
  } else {
    const Src sr = pull_src<G, I, DX, DY, DZ>(b, n, m);
    return RefPull{base[(size_t)sr.slot * Np + sr.node], R[sr.node], sr.valid};
  }
}
template <class G, int I>
__device__ __forceinline__ float ref_pull_value(const RefPull& p, float Rn, bool wall_here) {
  if constexpr (G::ex[I] == 0 && G::ey[I] == 0 && G::ez[I] == 0) {
    return p.r;
  } else {
    const bool shift = p.valid && !wall_here && ref_is_node(p.Rs);
    return p.valid ? (shift ? p.r + G::w[I] * (p.Rs - Rn) : p.r) : 0.0f;
  }
}
// All Q thermal pulls of node n in that form: loads first, then the shifts.
// Direction own_dir (an outlet's inward normal, else -1) keeps the raw value
// read: its source lies outside the box (a port's normal is the inward
// normal of a non-periodic face), so the read fell back to node n's own
// slot, which is what the zero-gradient outflow rule takes.
template <class G>
__device__ __forceinline__ void load_pull_ref_all(float (&k)[G::Q], const float* __restrict__ base,
                                                  const float* __restrict__ R, size_t Np,
                                                  const Nbr& b, int n, const Mirror& m, float Rn,
                                                  bool wall_here, int own_dir) {
  RefPull pr[G::Q];
  sfor<G::Q>([&](auto I) {
    constexpr int i = I;
    pr[i] = load_ref_pull<G, i, -G::ex[i], -G::ey[i], -G::ez[i]>(base, R, Np, b, n, m);
  });
  sfor<G::Q>([&](auto I) {
    constexpr int i = I;
    k[i] = (i == own_dir) ? pr[i].r : ref_pull_value<G, i>(pr[i], Rn, wall_here);
  });
}

// ---------------------------------------------------------------------------
// Design parametrisation (see the header): chi, a_B, thermal tau and their
// derivatives with respect to gamma.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float chi_of(float g, const KParams& P) {
  return 1.0f - P.tab * (1.0f - g) / (P.qb + g);
}
__device__ __forceinline__ float khat_of(float g, const KParams& P) {
  return P.kr + (1.0f - P.kr) * g / (1.0f + P.qr * (1.0f - g));
}

// Inward normal (nx, ny, nz) of normal code c (+x 0, -x 1, +y 2, -y 3, +z 4, -z 5).
struct Normal {
  int x, y, z;
};

// Calls f(n) with the inward normal of code nc as a compile-time constant in
// each case, so that the direction tests of the port rules below fold away
// (a runtime normal costs every wave that holds a port node the generic
// select chains).  2D lattices have no z normals.
template <class L, class F>
__device__ __forceinline__ void with_normal(int nc, F&& f) {
  switch (nc) {
    case 0: f(Normal{1, 0, 0}); break;
    case 1: f(Normal{-1, 0, 0}); break;
    case 2: f(Normal{0, 1, 0}); break;
    case 3: f(Normal{0, -1, 0}); break;
    default:
      if constexpr (L::Q != 9) {
        if (nc == 4) f(Normal{0, 0, 1});
        else f(Normal{0, 0, -1});
      }
      break;
  }
}

// ---------------------------------------------------------------------------
// Zou-He rule at a port with inward normal n (Eqs. 7, 8 generalised), on
// shifted populations h = f - w rho0.  For unknown i (e_i.n > 0):
//   h_i = h_ibar + 6 w_i j_n - 1/2 e_i.N,  N = sum_{e_j.n = 0} e_j h_j
// (N has no normal component, so e_i.N is the sum over the tangential axes);
// j_n = rho0 u_n at a velocity inlet, and at a pressure outlet rho = rho0
// gives j_n = -sum_{e.n=0} h - 2 sum_{e.n<0} h.  Written generically in the
// normal with selects, so the populations stay in registers; the step kernels
// call it through with_normal, where the normal is a constant and the
// selects fold.
// ---------------------------------------------------------------------------
// Generic Zou-He rule on shifted populations (f - w rho0).  Velocity inlet:
// prescribed rho0 u_n = jn_in.  Pressure outlet / pressure inlet:
// rho0 u_n = rho_b - sum_T f - 2 sum_O f, i.e. drho_b - (sum_T h + 2 sum_O h).
template <class L>
__device__ __forceinline__ void zou_he(float (&h)[L::Q], Normal nv, bool inlet, float jn_in,
                                       float drho_b = 0.0f) {
  float sT = 0.f, sO = 0.f, Nx = 0.f, Ny = 0.f, Nz = 0.f;
  sfor<L::Q>([&](auto I) {
    constexpr int i = I;
    const int c = L::ex[i] * nv.x + L::ey[i] * nv.y + L::ez[i] * nv.z;
    const float t = (c == 0) ? h[i] : 0.f;
    sT += t;
    sO += (c < 0) ? h[i] : 0.f;
    if constexpr (L::ex[i] != 0) Nx += float(L::ex[i]) * t;
    if constexpr (L::ey[i] != 0) Ny += float(L::ey[i]) * t;
    if constexpr (L::ez[i] != 0) Nz += float(L::ez[i]) * t;
  });
  const float jn = inlet ? jn_in : drho_b - (sT + 2.0f * sO);
  float o[L::Q];
  sfor<L::Q>([&](auto I) {
    constexpr int i = I;
    const int c = L::ex[i] * nv.x + L::ey[i] * nv.y + L::ez[i] * nv.z;
    float v = h[L::opp[i]] + (6.0f * L::w[i]) * jn;
    if constexpr (L::ex[i] != 0) v -= 0.5f * float(L::ex[i]) * Nx;
    if constexpr (L::ey[i] != 0) v -= 0.5f * float(L::ey[i]) * Ny;
    if constexpr (L::ez[i] != 0) v -= 0.5f * float(L::ez[i]) * Nz;
    o[i] = (c > 0) ? v : h[i];
  });
  sfor<L::Q>([&](auto I) { h[I] = o[I]; });
}

// Transpose of the rule above (Eq. 54 at a port; Eqs. 59, 60 in 2D), in place
// on c = f*_C -> f*:  f*_i = 0 for unknown i; for tangential j
//   f*_j = c_j - 1/2 e_j.P - [outlet] S6,
// for outgoing j:  f*_j = c_j + c_jbar - [outlet] 2 S6,
// with P = sum_{unknown i} e_i c_i and S6 = sum_{unknown i} 6 w_i c_i.
// Boundary step of the continuous adjoint (Sec. 2.3, Eqs. 25-29 generalised to
// any axis normal): on the streamed values of a port node, every direction
// leaving the domain (e_j . n < 0) takes
//   f*_j = f*_jbar - 12 sum_{e_k.n > 0} w_k f*_k   (pressure outlet)
//   f*_j = f*_jbar - src                         (velocity inlet; src = twice
//                                                  the objective's weight)
// which zeroes the coefficient of delta f_j in the boundary integral of
// Eq. (21); the other directions keep their values.
template <class L>
__device__ __forceinline__ void zou_he_continuous(float (&a)[L::Q], Normal nv, bool outlet, float src) {
  float S12 = 0.f;
  sfor<L::Q>([&](auto I) {
    constexpr int i = I;
    const int cl = L::ex[i] * nv.x + L::ey[i] * nv.y + L::ez[i] * nv.z;
    S12 += (cl > 0) ? (12.0f * L::w[i]) * a[i] : 0.f;
  });
  const float sub = outlet ? S12 : src;
  float o[L::Q];
  sfor<L::Q>([&](auto I) {
    constexpr int j = I;
    const int cl = L::ex[j] * nv.x + L::ey[j] * nv.y + L::ez[j] * nv.z;
    o[j] = (cl < 0) ? a[L::opp[j]] - sub : a[j];
  });
  sfor<L::Q>([&](auto I) { a[I] = o[I]; });
}

template <class L>
__device__ __forceinline__ void zou_he_transpose(float (&c)[L::Q], Normal nv, bool outlet) {
  float S6 = 0.f, Px = 0.f, Py = 0.f, Pz = 0.f;
  sfor<L::Q>([&](auto I) {
    constexpr int i = I;
    const int cl = L::ex[i] * nv.x + L::ey[i] * nv.y + L::ez[i] * nv.z;
    const float t = (cl > 0) ? c[i] : 0.f;
    S6 += (6.0f * L::w[i]) * t;
    if constexpr (L::ex[i] != 0) Px += float(L::ex[i]) * t;
    if constexpr (L::ey[i] != 0) Py += float(L::ey[i]) * t;
    if constexpr (L::ez[i] != 0) Pz += float(L::ez[i]) * t;
  });
  const float s6 = outlet ? S6 : 0.0f;
  float o[L::Q];
  sfor<L::Q>([&](auto I) {
    constexpr int j = I;
    const int cl = L::ex[j] * nv.x + L::ey[j] * nv.y + L::ez[j] * nv.z;
    float tv = c[j] - s6;
    if constexpr (L::ex[j] != 0) tv -= 0.5f * float(L::ex[j]) * Px;
    if constexpr (L::ey[j] != 0) tv -= 0.5f * float(L::ey[j]) * Py;
    if constexpr (L::ez[j] != 0) tv -= 0.5f * float(L::ez[j]) * Pz;
    const float ov = c[j] + c[L::opp[j]] - 2.0f * s6;
    o[j] = (cl == 0) ? tv : ((cl < 0) ? ov : 0.0f);
  });
  sfor<L::Q>([&](auto I) { c[I] = o[I]; });
}

// ---------------------------------------------------------------------------
// FP64 block reduction: wave64 shuffle tree, then the 4 wave partials in a
// fixed order (deterministic), written to out[0..NV).
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* __restrict__ out) {
  __shared__ double red[kBlock / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double s = acc[v];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) red[wave][v] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) s += red[k][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Forward step: pull (Eq. 37), boundary (Eqs. 7-9), collision (Eq. 36 with the
// equilibrium of Eq. 12), plus the coupled D3Q7 step advected by the same
// node's velocity.  DIAG additionally writes the macroscopic fields, the
// thermal non-equilibrium populations and the residual partial sums.
// ---------------------------------------------------------------------------
// EARLY: the node's own inputs are read together with the populations (one
// dependent memory round trip per step instead of two); pays off on lattices
// too small to keep several waves per SIMD in flight, and costs the large
// in-cache ones, so the launch chooses it by block count.
template <class L, bool MIR, bool THERMAL, bool DIAG, bool EARLY = false>
__device__ __forceinline__ void forward_tile(const FwdArgs& A, int blk) {
  using G = typename ThermalOf<L>::type;  // thermal lattice
  const KParams& P = A.P;
  const int n = blk * kBlock + threadIdx.x;
  double acc[kRedFwd] = {0.0, 0.0, 0.0, 0.0};
  if (n < P.N) {
    const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
    const Nbr nb = make_nbr(x, y, z, P);
    const Mirror mr = MIR ? mirror_of(x, y, z, P) : Mirror{false, false, false};
    const unsigned fl = A.flags[n];
    const int kind = fl & 7, nc = (fl >> 3) & 7;
    float gam_n = 1.0f, uin_n = 0.0f;
    if constexpr (EARLY) {
      gam_n = A.gamma[n];
      uin_n = A.uin[n];
    }
    float h[L::Q];
    sfor<L::Q>([&](auto I) {
      constexpr int i = I;
      h[i] = load_pull<L, i, -L::ex[i], -L::ey[i], -L::ez[i]>(A.fin, P.Np, nb, n, mr);
    });
    float k[G::Q];
    float Rn = 0.0f;  // the node's reference temperature (thermal shift)
    if constexpr (THERMAL) {
      Rn = A.Rin[n];
      // zero-gradient outflow: the population along the inward normal takes
      // the node's own post-collision value
      load_pull_ref_all<G>(k, A.gin, A.Rin, P.Np, nb, n, mr, Rn, kind >= K_WALL,
                           kind == K_OUTLET ? nc + 1 : -1);
    }
    // the early per-node values are consumed here, ahead of the branches on
    // the node kind, so that the compiler cannot sink their loads into those
    // branches (a second memory round trip); the empty asm only needs them in
    // registers
    if constexpr (EARLY) asm volatile("" ::"v"(gam_n), "v"(uin_n));
    // post-step populations, stored once after both branches: a wave that
    // holds wall and fluid nodes then writes each cache line with one store
    // instead of two partial ones
    float fo[L::Q];
    float go[G::Q];
    if (kind >= K_WALL) {
      // full-way bounce-back, no collision (the heated wall adds q_w)
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        fo[i] = h[L::opp[i]];
      });
      if constexpr (THERMAL) {
        float ko[G::Q];
        sfor<G::Q>([&](auto I) {
          constexpr int i = I;
          ko[i] = k[G::opp[i]];
        });
        if (kind == K_HEATED) {
          const int d = nc + 1;
          sfor<G::Q>([&](auto I) { ko[I] += (I == d) ? P.q_w : 0.0f; });
        }
        sfor<G::Q>([&](auto I) { go[I] = ko[I]; });
      }
      if constexpr (DIAG) {
        A.drho[n] = 0.f;
        A.u[n] = 0.f;
        A.u[P.N + n] = 0.f;
        A.u[2 * P.N + n] = 0.f;
        if constexpr (THERMAL) {
          A.T[n] = 0.f;
          sfor<G::Q>([&](auto I) { A.gneq[(size_t)I * P.Np + n] = 0.f; });
        }
      }
    } else {
      if (kind == K_INLET || kind == K_OUTLET) {
        const bool vin = kind == K_INLET && !P.pin;   // velocity inlet
        const float jn = vin ? (EARLY ? uin_n : A.uin[n]) * P.rho0 : 0.f;
        const float drho_b = (kind == K_INLET) ? P.drho_in : 0.0f;
        with_normal<L>(nc, [&](Normal nv) { zou_he<L>(h, nv, vin, jn, drho_b); });
      }
      if constexpr (THERMAL) {
        if (kind == K_INLET) {
          // Dirichlet T = T_in by the sum rule on the inward-normal population
          const int d = nc + 1;
          float s = 0.f;
          sfor<G::Q>([&](auto J) { s += (J == d) ? 0.0f : k[J]; });
          sfor<G::Q>([&](auto J) { k[J] = (J == d) ? (P.T_in - Rn) - s : k[J]; });
        }
      }
      // moments of the post-boundary state (Eq. 6)
      float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        drho += h[i];
        if constexpr (L::ex[i] != 0) jx += float(L::ex[i]) * h[i];
        if constexpr (L::ey[i] != 0) jy += float(L::ey[i]) * h[i];
        if constexpr (L::ez[i] != 0) jz += float(L::ez[i]) * h[i];
      });
      const float inv_rho0 = 1.0f / P.rho0;
      const float ux = jx * inv_rho0, uy = jy * inv_rho0, uz = jz * inv_rho0;
      float gam = 1.0f;
      if constexpr (EARLY) gam = (kind == K_DESIGN) ? gam_n : 1.0f;
      else if (kind == K_DESIGN) gam = A.gamma[n];
      const float chi = (kind == K_DESIGN) ? chi_of(gam, P) : 1.0f;
      const float vx = chi * ux, vy = chi * uy, vz = chi * uz;
      const float vv = vx * vx + vy * vy + vz * vz;
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        const float eu = float(L::ex[i]) * vx + float(L::ey[i]) * vy + float(L::ez[i]) * vz;
        const float heq = L::w[i] * (drho + P.rho0 * (3.0f * eu + 4.5f * eu * eu - 1.5f * vv));
        fo[i] = h[i] + P.omega * (heq - h[i]);
      });
      float Tabs = 0.f;
      if constexpr (THERMAL) {
        float dT = 0.f;
        sfor<G::Q>([&](auto I) { dT += k[I]; });
        Tabs = Rn + dT;
        const float tg = 0.5f + P.dfc * ((kind == K_DESIGN) ? khat_of(gam, P) : 1.0f);
        const float og = 1.0f / tg;
        // heat generation Q = beta_max (1 - gamma) (1 - T) in the design domain
        const float Qh = (kind == K_DESIGN) ? P.beta * (1.0f - gam) * (1.0f - Tabs) : 0.0f;
        sfor<G::Q>([&](auto I) {
          constexpr int i = I;
          const float eu = float(G::ex[i]) * ux + float(G::ey[i]) * uy + float(G::ez[i]) * uz;
          const float keq = G::w[i] * (dT + 4.0f * Tabs * eu);
          go[i] = k[i] + og * (keq - k[i]) + G::w[i] * Qh;
          if constexpr (DIAG) A.gneq[(size_t)i * P.Np + n] = k[i] - keq;
        });
        if constexpr (DIAG) {
          if (P.heatgen) acc[3] = (double)Qh;
        }
      }
      if constexpr (DIAG) {
        A.drho[n] = drho;
        A.u[n] = ux;
        A.u[P.N + n] = uy;
        A.u[2 * P.N + n] = uz;
        if constexpr (THERMAL) A.T[n] = Tabs;
        acc[0] = sqrt((double)ux * ux + (double)uy * uy + (double)uz * uz);
        acc[1] = (double)Tabs;
        if (kind == K_INLET) acc[2] = (double)drho;
        // slot 3 holds the objective's own sum: the heat generated (J = -sum Q)
        // or the temperature of the layer next to the heated walls
        if (!P.heatgen && (fl & kLayerBit)) acc[3] = (double)Tabs;
      }
    }
    sfor<L::Q>([&](auto I) { A.fout[(size_t)I * P.Np + n] = fo[I]; });
    if constexpr (THERMAL) sfor<G::Q>([&](auto I) { A.gout[(size_t)I * P.Np + n] = go[I]; });
  }
  if constexpr (DIAG) block_reduce_store<kRedFwd>(acc, A.partials + (size_t)blk * kRedFwd);
}

template <class L, bool MIR, bool THERMAL, bool DIAG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_forward(FwdArgs A) {
  forward_tile<L, MIR, THERMAL, DIAG, false>(A, remap_block(blockIdx.x, A.P));
}

// The coupled step on lattices too small to fill the device (the early
// per-node loads): no occupancy target, so the compiler keeps every load of
// the step in flight at once instead of trading registers for waves such a
// lattice does not have.
template <class L, bool MIR>
__global__ __launch_bounds__(kBlock) void k_forward_early(FwdArgs A) {
  forward_tile<L, MIR, true, false, true>(A, remap_block(blockIdx.x, A.P));
}

// ---------------------------------------------------------------------------
// Adjoint step (the paper's order reversed onto a pull kernel): reversed pull
// a_i(x) = f*_i(x + e_i) (Eq. 61), adjoint collision minus the objective
// source (Eq. 65), then the node's own adjoint boundary condition (Eq. 54),
// so the stored state is f* = B^T f*_C.  The collision transpose is applied
// matrix-free through moments: for the equilibrium of Eq. (12),
//   sum_m a_m d feq_m / d f_i = M0 + e_i.V,  V = chi (3 M1 + 9 K - 3 M0 chi u),
//   M0 = sum w a, M1 = sum w a e, K = sum w a (e.chi u) e;
// the coupling from the thermal lattice adds e_i.W, W = 4 T/(tau_g rho0) sum w b e,
// and the thermal transpose is (1 - 1/tau_g) b_i + (1/tau_g) sum w b (1 + 4 e.u).
// ---------------------------------------------------------------------------
template <class L, bool MIR, bool THERMAL, int OBJ, bool DIAG, bool CONT = false, bool EARLY = false>
__device__ __forceinline__ void adjoint_tile(const AdjArgs& A, int blk) {
  using G = typename ThermalOf<L>::type;  // thermal lattice
  static_assert(!(CONT && THERMAL), "the continuous variant is for the flow lattice");
  const KParams& P = A.P;
  const int n = blk * kBlock + threadIdx.x;
  double acc[kRedAdj] = {0.0, 0.0};
  if (n < P.N) {
    const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
    const Nbr nb = make_nbr(x, y, z, P);
    const Mirror mr = MIR ? mirror_of(x, y, z, P) : Mirror{false, false, false};
    const unsigned fl = A.flags[n];
    const int kind = fl & 7, nc = (fl >> 3) & 7;
    float gam_n = 1.0f, ux_n = 0.f, uy_n = 0.f, uz_n = 0.f, T_n = 0.f;
    if constexpr (EARLY) {
      gam_n = A.gamma[n];
      ux_n = A.u[n];
      uy_n = A.u[P.N + n];
      if constexpr (L::Q != 9) uz_n = A.u[2 * P.N + n];
      if constexpr (THERMAL) T_n = A.T[n];
    }
    float a[L::Q];
    sfor<L::Q>([&](auto I) {
      constexpr int i = I;
      a[i] = load_pull<L, i, L::ex[i], L::ey[i], L::ez[i]>(A.ain, P.Np, nb, n, mr);
    });
    float b[G::Q];
    if constexpr (THERMAL) {
      sfor<G::Q>([&](auto I) {
        constexpr int i = I;
        b[i] = load_pull<G, i, G::ex[i], G::ey[i], G::ez[i]>(A.bin, P.Np, nb, n, mr);
      });
      // transpose of the outflow self-copy
      if (kind == K_OUTLET) {
        const int d = nc + 1;
        const float own = A.bin[(size_t)d * P.Np + n];
        sfor<G::Q>([&](auto I) { b[I] += (I == d) ? own : 0.0f; });
      }
    }
    if constexpr (DIAG) {
      if (kind < K_WALL) {
        float mx = 0.f, my = 0.f, mz = 0.f;
        sfor<L::Q>([&](auto I) {
          constexpr int i = I;
          if constexpr (L::ex[i] != 0) mx += float(L::ex[i]) * a[i];
          if constexpr (L::ey[i] != 0) my += float(L::ey[i]) * a[i];
          if constexpr (L::ez[i] != 0) mz += float(L::ez[i]) * a[i];
        });
        acc[0] = sqrt((double)mx * mx + (double)my * my + (double)mz * mz);
        if constexpr (THERMAL) {
          float sb = 0.f;
          sfor<G::Q>([&](auto I) { sb += b[I]; });
          acc[1] = fabs((double)sb);
        }
      }
    }
    if constexpr (CONT) {
      // continuous variant: boundary step on the streamed values, before the
      // collision (order collision -> streaming -> boundary of Eq. 30); the
      // inlet-pressure objective enters here and not as a collision source
      if (kind == K_INLET || kind == K_OUTLET) {
        // a pressure inlet follows the outlet rule; the inlet pressure it fixes
        // gives the objective no boundary term there
        const bool prs = kind == K_OUTLET || P.pin;
        const float src = (OBJ == OBJ_PRESSURE_DROP && !prs) ? 2.0f * P.c_in : 0.0f;
        with_normal<L>(nc, [&](Normal nv) { zou_he_continuous<L>(a, nv, prs, src); });
      }
    }
    // the new state, stored once after both branches (one full store per
    // cache line in waves that hold wall and fluid nodes)
    float c[L::Q];
    float cg[G::Q];
    if (kind >= K_WALL) {
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        c[i] = a[L::opp[i]];
      });
      if constexpr (THERMAL) {
        sfor<G::Q>([&](auto I) {
          constexpr int i = I;
          cg[i] = b[G::opp[i]];
        });
      }
    } else {
      float ux, uy, uz, gam = 1.0f;
      if constexpr (EARLY) {
        ux = ux_n;
        uy = uy_n;
        uz = uz_n;
        gam = (kind == K_DESIGN) ? gam_n : 1.0f;
      } else {
        ux = A.u[n];
        uy = A.u[P.N + n];
        uz = (L::Q == 9) ? 0.0f : A.u[2 * P.N + n];  // 2D: no z component
        if (kind == K_DESIGN) gam = A.gamma[n];
      }
      const float chi = (kind == K_DESIGN) ? chi_of(gam, P) : 1.0f;
      const float vx = chi * ux, vy = chi * uy, vz = chi * uz;
      float M0 = 0.f, M1x = 0.f, M1y = 0.f, M1z = 0.f, Kx = 0.f, Ky = 0.f, Kz = 0.f;
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        const float wa = L::w[i] * a[i];
        M0 += wa;
        const float ev = float(L::ex[i]) * vx + float(L::ey[i]) * vy + float(L::ez[i]) * vz;
        const float wae = wa * ev;
        if constexpr (L::ex[i] != 0) { M1x += float(L::ex[i]) * wa; Kx += float(L::ex[i]) * wae; }
        if constexpr (L::ey[i] != 0) { M1y += float(L::ey[i]) * wa; Ky += float(L::ey[i]) * wae; }
        if constexpr (L::ez[i] != 0) { M1z += float(L::ez[i]) * wa; Kz += float(L::ez[i]) * wae; }
      });
      const float Vx = chi * (3.0f * M1x + 9.0f * Kx - 3.0f * M0 * vx);
      const float Vy = chi * (3.0f * M1y + 9.0f * Ky - 3.0f * M0 * vy);
      const float Vz = chi * (3.0f * M1z + 9.0f * Kz - 3.0f * M0 * vz);
      float Wx = 0.f, Wy = 0.f, Wz = 0.f;
      float Bg = 0.f, og = 0.f, Sbw = 0.f;
      if constexpr (THERMAL) {
        const float Tn = EARLY ? T_n : A.T[n];
        const float tg = 0.5f + P.dfc * ((kind == K_DESIGN) ? khat_of(gam, P) : 1.0f);
        og = 1.0f / tg;
        float Sb = 0.f, Mbx = 0.f, Mby = 0.f, Mbz = 0.f;
        sfor<G::Q>([&](auto I) {
          constexpr int i = I;
          const float wb = G::w[i] * b[i];
          Sb += wb;
          if constexpr (G::ex[i] != 0) Mbx += float(G::ex[i]) * wb;
          if constexpr (G::ey[i] != 0) Mby += float(G::ey[i]) * wb;
          if constexpr (G::ez[i] != 0) Mbz += float(G::ez[i]) * wb;
        });
        Bg = Sb + 4.0f * (ux * Mbx + uy * Mby + uz * Mbz);
        Sbw = Sb;
        const float cW = 4.0f * og * Tn / P.rho0;
        Wx = cW * Mbx;
        Wy = cW * Mby;
        Wz = cW * Mbz;
      }
      // objective sources dJ/df_i = c + e_i.G and dJ/dg_i = d
      float csrc = 0.f, dsrc = 0.f, Gx = 0.f, Gy = 0.f, Gz = 0.f;
      if constexpr ((OBJ == OBJ_PRESSURE_DROP || OBJ == OBJ_HEATSINK) && !CONT) {
        if (kind == K_INLET) csrc = P.c_in;
      }
      if constexpr (OBJ == OBJ_HEATSINK) {
        if (fl & kLayerBit) dsrc = P.c_layer;
      }
      // heat generation beta (1 - T): its d/dg_j in the collision, and
      // dJ/dg_j = beta for J = -sum beta (1 - T)
      const float bq = (THERMAL && kind == K_DESIGN) ? P.beta * (1.0f - gam) : 0.0f;
      if constexpr (OBJ == OBJ_HEATGEN) dsrc = bq;
      if constexpr (OBJ == OBJ_DISSIPATION) {
        Gx = A.G[n];
        Gy = A.G[(size_t)P.Np + n];
        Gz = A.G[2 * (size_t)P.Np + n];
      }
      const float Sx = P.omega * Vx + Wx - Gx, Sy = P.omega * Vy + Wy - Gy,
                  Sz = P.omega * Vz + Wz - Gz;
      const float base = P.omega * M0 - csrc;
      const float keep = 1.0f - P.omega;
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        float v = keep * a[i] + base;
        if constexpr (L::ex[i] != 0) v += float(L::ex[i]) * Sx;
        if constexpr (L::ey[i] != 0) v += float(L::ey[i]) * Sy;
        if constexpr (L::ez[i] != 0) v += float(L::ez[i]) * Sz;
        c[i] = v;
      });
      if constexpr (!CONT) {
        if (kind == K_INLET || kind == K_OUTLET) {
          const bool outlet = kind == K_OUTLET || P.pin;
          with_normal<L>(nc, [&](Normal nv) { zou_he_transpose<L>(c, nv, outlet); });
        }
      }
      if constexpr (THERMAL) {
        const float bb = og * Bg - dsrc - bq * Sbw;
        sfor<G::Q>([&](auto I) {
          constexpr int i = I;
          cg[i] = (1.0f - og) * b[i] + bb;
        });
        if (kind == K_INLET) {
          // transpose of the Dirichlet sum rule
          const int d = nc + 1;
          float cd = 0.f;
          sfor<G::Q>([&](auto J) { cd += (J == d) ? cg[J] : 0.0f; });
          sfor<G::Q>([&](auto J) { cg[J] = (J == d) ? 0.0f : cg[J] - cd; });
        }
      }
    }
    sfor<L::Q>([&](auto I) { A.aout[(size_t)I * P.Np + n] = c[I]; });
    if constexpr (THERMAL) sfor<G::Q>([&](auto I) { A.bout[(size_t)I * P.Np + n] = cg[I]; });
  }
  if constexpr (DIAG) block_reduce_store<kRedAdj>(acc, A.partials + (size_t)blk * kRedAdj);
}

template <class L, bool MIR, bool THERMAL, int OBJ, bool DIAG, bool CONT = false, bool EARLY = false>
__global__ __launch_bounds__(kBlock) void k_adjoint(AdjArgs A) {
  adjoint_tile<L, MIR, THERMAL, OBJ, DIAG, CONT, EARLY>(A, remap_block(blockIdx.x, A.P));
}

// ---------------------------------------------------------------------------
// Sensitivity, Eq. (66) with the exact derivative of the collision:
// dJ/dgamma = explicit - (1/tau) chi' rho0 sum_i w_i a_i [3 e.u + 9 chi (e.u)^2
// - 3 chi |u|^2] - (tau_g'/tau_g^2) sum_i b_i (g_i - geq_i), a, b the reversed
// pulls of the final adjoint state; with heat generation also
// + beta_max (1 - T) sum_i w_i b_i (and + beta_max (1 - T) for J = -sum Q).
// Non-design nodes get 0.
// ---------------------------------------------------------------------------
template <class L, bool MIR, bool THERMAL>
__global__ __launch_bounds__(kBlock) void k_sensitivity(SensArgs A) {
  using G = typename ThermalOf<L>::type;  // thermal lattice
  const KParams& P = A.P;
  const int blk = remap_block(blockIdx.x, P);
  const int n = blk * kBlock + threadIdx.x;
  double acc[kRedSens] = {0.0, 0.0};
  if (n < P.N) {
    const unsigned fl = A.flags[n];
    const int kind = fl & 7;
    float out = 0.0f;
    if (kind == K_DESIGN) {
      const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
      const Nbr nb = make_nbr(x, y, z, P);
      const Mirror mr = MIR ? mirror_of(x, y, z, P) : Mirror{false, false, false};
      const float ux = A.u[n], uy = A.u[P.N + n], uz = (L::Q == 9) ? 0.0f : A.u[2 * P.N + n];  // 2D: no z component
      const float gam = A.gamma[n];
      const float chi = chi_of(gam, P);
      const float qg = P.qb + gam;
      const float dchi = P.tab * (1.0f + P.qb) / (qg * qg);
      const float uu = ux * ux + uy * uy + uz * uz;
      float s = 0.f;
      sfor<L::Q>([&](auto I) {
        constexpr int i = I;
        const float a = load_pull<L, i, L::ex[i], L::ey[i], L::ez[i]>(A.ain, P.Np, nb, n, mr);
        const float eu = float(L::ex[i]) * ux + float(L::ey[i]) * uy + float(L::ez[i]) * uz;
        s += L::w[i] * a * (3.0f * eu + 9.0f * chi * eu * eu - 3.0f * chi * uu);
      });
      out = -P.omega * P.rho0 * dchi * s;
      if constexpr (THERMAL) {
        const float den = 1.0f + P.qr * (1.0f - gam);
        const float kh = P.kr + (1.0f - P.kr) * gam / den;
        const float dkh = (1.0f - P.kr) * (1.0f + P.qr) / (den * den);
        const float tg = 0.5f + P.dfc * kh;
        const float dtg = P.dfc * dkh;
        float sg = 0.f, swb = 0.f;
        sfor<G::Q>([&](auto I) {
          constexpr int i = I;
          const float b = load_pull<G, i, G::ex[i], G::ey[i], G::ez[i]>(A.bin, P.Np, nb, n, mr);
          sg += b * A.gneq[(size_t)i * P.Np + n];
          swb += G::w[i] * b;
        });
        out -= dtg / (tg * tg) * sg;
        // heat generation: d(w_i beta (1 - T))/dgamma = -w_i beta_max (1 - T),
        // and the explicit dJ/dgamma = beta_max (1 - T) of J = -sum Q
        if (P.beta > 0.0f) {
          const float q = P.beta * (1.0f - A.T[n]);
          out += q * swb;
          if (A.objective == OBJ_HEATGEN) out += q;
        }
      }
      if (A.objective == OBJ_DISSIPATION) {
        const float dab = -P.amq * (1.0f + P.qb) / (qg * qg);
        out += dab * P.rho0 * uu;
      }
    }
    A.dJ[n] = out;
    acc[0] = (double)out;
    acc[1] = (double)out * out;
  }
  block_reduce_store<kRedSens>(acc, A.partials + (size_t)blk * kRedSens);
}

// ---------------------------------------------------------------------------
// Dissipation objective: source G = dJ/du / rho0 per node and the value of J.
// Edges join axis neighbours inside the box (no wrap) that are both non-wall.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_dissipation_source(const float* __restrict__ u,
                                                               const float* __restrict__ gamma,
                                                               const uint8_t* __restrict__ flags,
                                                               float* __restrict__ G, KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N) return;
  const int kind = flags[n] & 7;
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (kind < K_WALL) {
    const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
    const float ux = u[n], uy = u[P.N + n], uz = u[2 * P.N + n];
    const int c[3] = {x, y, z}, lim[3] = {P.nx, P.ny, P.nz}, off[3] = {1, P.nx, P.plane};
    for (int a = 0; a < 3; ++a) {
      for (int s = -1; s <= 1; s += 2) {
        const int cc = c[a] + s;
        if (cc < 0 || cc >= lim[a]) continue;
        const int m = n + s * off[a];
        if ((flags[m] & 7) >= K_WALL) continue;
        gx += P.two_nu * (ux - u[m]);
        gy += P.two_nu * (uy - u[P.N + m]);
        gz += P.two_nu * (uz - u[2 * P.N + m]);
      }
    }
    if (kind == K_DESIGN) {
      const float g = gamma[n];
      const float ab = P.amq * (1.0f - g) / (P.qb + g);
      gx += 2.0f * ab * ux;
      gy += 2.0f * ab * uy;
      gz += 2.0f * ab * uz;
    }
  }
  G[n] = gx;
  G[(size_t)P.Np + n] = gy;
  G[2 * (size_t)P.Np + n] = gz;
}

__global__ __launch_bounds__(kBlock) void k_dissipation_objective(const float* __restrict__ u,
                                                                  const float* __restrict__ gamma,
                                                                  const uint8_t* __restrict__ flags,
                                                                  double* __restrict__ partials,
                                                                  KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  double acc[kRedDiss] = {0.0};
  if (n < P.N) {
    const int kind = flags[n] & 7;
    if (kind < K_WALL) {
      const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
      const double ux = u[n], uy = u[P.N + n], uz = u[2 * P.N + n];
      const int c[3] = {x, y, z}, lim[3] = {P.nx, P.ny, P.nz}, off[3] = {1, P.nx, P.plane};
      double s = 0.0;
      for (int a = 0; a < 3; ++a) {
        if (c[a] + 1 >= lim[a]) continue;
        const int m = n + off[a];
        if ((flags[m] & 7) >= K_WALL) continue;
        const double dx = u[m] - ux, dy = u[P.N + m] - uy, dz = u[2 * P.N + m] - uz;
        s += (double)P.rho0 * (double)P.nu * (dx * dx + dy * dy + dz * dz);
      }
      if (kind == K_DESIGN) {
        const double g = gamma[n];
        const double ab = (double)P.amq * (1.0 - g) / ((double)P.qb + g);
        s += ab * (double)P.rho0 * (ux * ux + uy * uy + uz * uz);
      }
      acc[0] = s;
    }
  }
  block_reduce_store<kRedDiss>(acc, partials + (size_t)blockIdx.x * kRedDiss);
}

// Deterministic final sum of block partials (one block, fixed order).
__device__ __forceinline__ void finalize_block(const double* __restrict__ partials, int nblk, int nvals,
                                               double* __restrict__ out) {
  __shared__ double sh[kBlock];
  for (int v = 0; v < nvals; ++v) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kBlock) s += partials[(size_t)i * nvals + v];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = sh[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict__ partials, int nblk,
                                                     int nvals, double* __restrict__ out) {
  finalize_block(partials, nblk, nvals, out);
}

// One block per slot; the forward phase reduces 4 sums, the adjoint phase 2.
__global__ __launch_bounds__(kBlock) void k_finalize_slots(const SlotDev* __restrict__ slots,
                                                           double* __restrict__ out) {
  const SlotDev& S = slots[blockIdx.x];
  if (S.phase == 0) return;
  const int nvals = S.phase == 1 ? kRedFwd : kRedAdj;
  finalize_block(S.fa.partials, S.fa.P.nblk, nvals, out + (size_t)blockIdx.x * 4);
}

// Ragged-batch step: block -> tile (XCD-contiguous runs of tiles) -> slot ->
// the slot's forward or adjoint step on that tile, with the same tile code as
// the single-problem kernels, so a slot computes bit for bit what it would
// alone.
template <class L, bool MIR, bool THERMAL, int OBJ>
__device__ __forceinline__ void batch_tile(const SlotDev& S, int blk, int k, bool diag) {
  const bool odd = (k & 1) != 0;
  if (S.phase == 1) {
    FwdArgs A = S.fa;
    if (odd) {
      A.fin = S.fa.fout;
      A.fout = const_cast<float*>(S.fa.fin);
      A.gin = S.fa.gout;
      A.gout = const_cast<float*>(S.fa.gin);
    }
    // the reference buffers alternate at every re-base (after each
    // diagnostic step of the sweep)
    if (THERMAL && S.check > 0 && ((k / S.check) & 1)) A.Rin = S.R1;
    if (diag) forward_tile<L, MIR, THERMAL, true>(A, blk);
    else forward_tile<L, MIR, THERMAL, false>(A, blk);
  } else {
    AdjArgs A = S.aa;
    if (odd) {
      A.ain = S.aa.aout;
      A.aout = const_cast<float*>(S.aa.ain);
      A.bin = S.aa.bout;
      A.bout = const_cast<float*>(S.aa.bin);
    }
    if constexpr (!THERMAL) {
      if (A.P.cont) {
        if (diag) adjoint_tile<L, MIR, THERMAL, OBJ, true, true>(A, blk);
        else adjoint_tile<L, MIR, THERMAL, OBJ, false, true>(A, blk);
        return;
      }
    }
    if (diag) adjoint_tile<L, MIR, THERMAL, OBJ, true>(A, blk);
    else adjoint_tile<L, MIR, THERMAL, OBJ, false>(A, blk);
  }
}

// One tile of a ragged-batch launch: the tile's slot takes its forward or
// adjoint step number `launch - start` (nothing if the slot is idle there).
template <bool THERMAL, int OBJ>
__device__ __forceinline__ void batch_step_tile(const Tile* __restrict__ tiles,
                                                const SlotDev* __restrict__ slots, int t,
                                                int launch) {
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  const int k = launch - S.start;
  if (S.phase == 0 || k < 0 || k >= S.max_steps) return;  // uniform over the block
  const bool diag = (S.check > 0 && (k + 1) % S.check == 0) || (k + 1 == S.max_steps);
  const bool mir = has_mirror(S.fa.P);
  if (S.fa.P.q == 9) {
    if (mir) batch_tile<Q9, true, THERMAL, OBJ>(S, tl.blk, k, diag);
    else batch_tile<Q9, false, THERMAL, OBJ>(S, tl.blk, k, diag);
    return;
  }
  if (mir) batch_tile<Q19, true, THERMAL, OBJ>(S, tl.blk, k, diag);
  else batch_tile<Q19, false, THERMAL, OBJ>(S, tl.blk, k, diag);
}

// Ragged-batch step: block -> tile (XCD-contiguous runs of tiles) -> slot ->
// the slot's forward or adjoint step on that tile, with the same tile code as
// the single-problem kernels, so a slot computes bit for bit what it would
// alone.  An engine takes 3D and 2D requests side by side (the lattice is
// uniform over a block: a tile belongs to one slot).
template <bool THERMAL, int OBJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_batch(const Tile* __restrict__ tiles,
                                                  const SlotDev* __restrict__ slots,
                                                  const int* __restrict__ base, int q, int xper,
                                                  int xrem) {
  const int b = blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int t = xcd < xrem ? xcd * (xper + 1) + idx : xrem * (xper + 1) + (xcd - xrem) * xper + idx;
  batch_step_tile<THERMAL, OBJ>(tiles, slots, t, *base + q);
}

__global__ void k_advance(int* base, int q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base += q;
}

// ---------------------------------------------------------------------------
// Thermal lattice alone with the velocity frozen (a saved field): the D3Q7 part
// of the forward step, used to recover the converged thermal non-equilibrium
// populations from (u, T) only.  Same pull, boundary rules and collision as
// the coupled kernel; DIAG writes g - g_eq and the mean-T partial sums.
// ---------------------------------------------------------------------------
template <class G, bool DIAG, bool MIR>
__global__ __launch_bounds__(kBlock) void k_thermal(ThermArgs A) {
  const KParams& P = A.P;
  const int blk = remap_block(blockIdx.x, P);
  const int n = blk * kBlock + threadIdx.x;
  double acc[kRedFwd] = {0.0, 0.0, 0.0, 0.0};
  if (n < P.N) {
    const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
    const Nbr nb = make_nbr(x, y, z, P);
    const Mirror mr = MIR ? mirror_of(x, y, z, P) : Mirror{false, false, false};
    const unsigned fl = A.flags[n];
    const int kind = fl & 7, nc = (fl >> 3) & 7;
    float k[G::Q];
    const float Rn = A.R[n];
    const int d = nc + 1;
    load_pull_ref_all<G>(k, A.gin, A.R, P.Np, nb, n, mr, Rn, kind >= K_WALL,
                         kind == K_OUTLET ? d : -1);
    float ko[G::Q];  // stored once after both branches
    if (kind >= K_WALL) {
      sfor<G::Q>([&](auto I) { ko[I] = k[G::opp[I]]; });
      if (kind == K_HEATED) sfor<G::Q>([&](auto I) { ko[I] += (I == d) ? P.q_w : 0.0f; });
      if constexpr (DIAG) sfor<G::Q>([&](auto I) { A.gneq[(size_t)I * P.Np + n] = 0.f; });
    } else {
      if (kind == K_INLET) {
        float s = 0.f;
        sfor<G::Q>([&](auto J) { s += (J == d) ? 0.0f : k[J]; });
        sfor<G::Q>([&](auto J) { k[J] = (J == d) ? (P.T_in - Rn) - s : k[J]; });
      }
      const float ux = A.u[n], uy = A.u[P.N + n], uz = A.u[2 * P.N + n];
      float dT = 0.f;
      sfor<G::Q>([&](auto I) { dT += k[I]; });
      const float Tabs = Rn + dT;
      const float gm = (kind == K_DESIGN) ? A.gamma[n] : 1.0f;
      const float tg = 0.5f + P.dfc * ((kind == K_DESIGN) ? khat_of(gm, P) : 1.0f);
      const float og = 1.0f / tg;
      const float Qh = (kind == K_DESIGN) ? P.beta * (1.0f - gm) * (1.0f - Tabs) : 0.0f;
      sfor<G::Q>([&](auto I) {
        constexpr int i = I;
        const float eu = float(G::ex[i]) * ux + float(G::ey[i]) * uy + float(G::ez[i]) * uz;
        const float keq = G::w[i] * (dT + 4.0f * Tabs * eu);
        ko[i] = k[i] + og * (keq - k[i]) + G::w[i] * Qh;
        if constexpr (DIAG) A.gneq[(size_t)i * P.Np + n] = k[i] - keq;
      });
      if constexpr (DIAG) {
        acc[1] = (double)Tabs;
        if (!P.heatgen && (fl & kLayerBit)) acc[3] = (double)Tabs;
      }
    }
    sfor<G::Q>([&](auto I) { A.gout[(size_t)I * P.Np + n] = ko[I]; });
  }
  if constexpr (DIAG) block_reduce_store<kRedFwd>(acc, A.partials + (size_t)blk * kRedFwd);
}

// Initial thermal state g = g_eq(T, u) at non-wall nodes, stored relative
// to the reference R = T (so only the advective part 4 w T e.u remains), and
// 0 at walls (whose reference is +inf).
template <class G>
__global__ __launch_bounds__(kBlock) void k_thermal_init(ThermArgs A) {
  const KParams& P = A.P;
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N) return;
  const int kind = A.flags[n] & 7;
  const float ux = A.u[n], uy = A.u[P.N + n], uz = A.u[2 * P.N + n];
  const float Tabs = A.T[n];
  A.R[n] = (kind >= K_WALL) ? INFINITY : Tabs;
  sfor<G::Q>([&](auto I) {
    constexpr int i = I;
    const float eu = float(G::ex[i]) * ux + float(G::ey[i]) * uy + float(G::ez[i]) * uz;
    const float keq = G::w[i] * (4.0f * Tabs * eu);
    A.gout[(size_t)i * P.Np + n] = (kind >= K_WALL) ? 0.0f : keq;
  });
}

// Reference of a forward start: T_in at non-wall nodes, +inf at walls (and in
// the padding beyond N).
__global__ __launch_bounds__(kBlock) void k_ref_init(float* __restrict__ R,
                                                     const uint8_t* __restrict__ flags, KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.Np) return;
  R[n] = (n < P.N && (flags[n] & 7) < K_WALL) ? P.T_in : INFINITY;
}

// Re-base of the forward thermal state onto the temperature field T: every
// non-wall node n moves its own slots by w_i (Rin(n) - T(n)) and, for each
// direction whose pull source is a wall, the wall slot it reads (walls hold
// values in their reader's shift; each slot has one reader, so the writes do
// not collide); Rout = T at non-wall nodes, +inf at walls.  Exact up to one
// FP32 rounding per slot.
template <class G, bool MIR>
__device__ __forceinline__ void rebase_tile(const RebaseArgs& A, int blk) {
  const KParams& P = A.P;
  const int n = blk * kBlock + threadIdx.x;
  if (n >= P.N) return;
  const int kind = A.flags[n] & 7;
  if (kind >= K_WALL) {
    A.Rout[n] = INFINITY;
    return;
  }
  const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
  const Nbr nb = make_nbr(x, y, z, P);
  const Mirror mr = MIR ? mirror_of(x, y, z, P) : Mirror{false, false, false};
  const float Tn = A.T[n];
  const float dR = A.Rin[n] - Tn;
  A.Rout[n] = Tn;
  sfor<G::Q>([&](auto I) {
    constexpr int i = I;
    float* own = A.g + (size_t)i * P.Np + n;
    *own = *own + G::w[i] * dR;
    if constexpr (i != 0) {
      const Src sr = pull_src<G, i, -G::ex[i], -G::ey[i], -G::ez[i]>(nb, n, mr);
      if (sr.valid && (A.flags[sr.node] & 7) >= K_WALL) {
        float* ws = A.g + (size_t)sr.slot * P.Np + sr.node;
        *ws = *ws + G::w[i] * dR;
      }
    }
  });
}

template <class G, bool MIR>
__global__ __launch_bounds__(kBlock) void k_rebase(RebaseArgs A) {
  rebase_tile<G, MIR>(A, blockIdx.x);
}

// Re-base after the step `launch` of the tile's slot, if that was a
// diagnostic forward step (thermal engines only).
__device__ __forceinline__ void batch_rebase_tile(const Tile* __restrict__ tiles,
                                                  const SlotDev* __restrict__ slots, int t,
                                                  int launch) {
  const Tile tl = tiles[t];
  const SlotDev& S = slots[tl.slot];
  const int k = launch - S.start;
  if (S.phase != 1 || k < 0 || k >= S.max_steps) return;  // uniform over the block
  const bool diag = (S.check > 0 && (k + 1) % S.check == 0) || (k + 1 == S.max_steps);
  if (!diag) return;
  const bool r1 = S.check > 0 && ((k / S.check) & 1);
  RebaseArgs A;
  A.g = ((k + 1) & 1) ? S.fa.gout : const_cast<float*>(S.fa.gin);  // state after step k
  A.Rin = r1 ? S.R1 : S.fa.Rin;
  A.Rout = r1 ? const_cast<float*>(S.fa.Rin) : S.R1;
  A.T = S.fa.T;
  A.flags = S.fa.flags;
  A.P = S.fa.P;
  const bool mir = has_mirror(A.P);
  if (A.P.q == 9) {
    if (mir) rebase_tile<Q5, true>(A, tl.blk);
    else rebase_tile<Q5, false>(A, tl.blk);
  } else {
    if (mir) rebase_tile<Q7, true>(A, tl.blk);
    else rebase_tile<Q7, false>(A, tl.blk);
  }
}

// Re-base after launch q of a quantum: each slot whose step in that launch
// was a diagnostic forward step re-bases its tiles (thermal engines only).
__global__ __launch_bounds__(kBlock) void k_batch_rebase(const Tile* __restrict__ tiles,
                                                         const SlotDev* __restrict__ slots,
                                                         const int* __restrict__ base, int q,
                                                         int xper, int xrem) {
  const int b = blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int t = xcd < xrem ? xcd * (xper + 1) + idx : xrem * (xper + 1) + (xcd - xrem) * xper + idx;
  batch_rebase_tile(tiles, slots, t, *base + q);
}

// Grid-wide barrier of a persistent launch whose blocks are all resident:
// every block's writes are made visible at device scope, block 0's thread 0
// of each block counts in, and waits until `target` arrivals are counted.
// The wait is bounded: after `spin_limit` polls, or once another block has
// given up, the block raises `abort` and returns false, so every block
// leaves its loop (the host then reports the quantum as failed).
__device__ __forceinline__ bool grid_barrier(unsigned* bar, int* abort, unsigned target,
                                             int spin_limit) {
  __shared__ int ok;
  // every wave's stores have reached the L2 before the block counts in (a
  // workgroup barrier alone does not wait for them); thread 0's release then
  // writes the L2 back for the other XCDs, and one acquire after the wait
  // drops stale lines (the polls themselves are relaxed: an acquire per poll
  // would invalidate the L2 under the blocks still computing)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1, spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > spin_limit) {
        __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Persistent ragged-batch quantum: one launch whose blocks (all resident)
// loop over the quantum's Q lattice steps.  Each block owns a contiguous run
// of tiles (blocks of one XCD own neighbouring runs), advances them by one
// step of their slots, then waits at a grid barrier for the whole step; after
// the last step the thermal states of diagnostic steps are re-based.  The
// arithmetic of every tile is the per-launch kernel's, so the results are
// bit for bit those of Q launches of k_batch.  `bar` counts barrier
// arrivals and must be 0 at launch.
template <bool THERMAL, int OBJ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_persistent(
    const Tile* __restrict__ tiles, int ntiles, const SlotDev* __restrict__ slots,
    const int* __restrict__ base, int Q, unsigned* bar, int* abort, int spin_limit) {
  const int G = gridDim.x;
  const int b = blockIdx.x, xcd = b & 7, idx = b >> 3;
  const int xper = G / 8, xrem = G % 8;
  const int lb = xcd < xrem ? xcd * (xper + 1) + idx : xrem * (xper + 1) + (xcd - xrem) * xper + idx;
  const int t0 = (int)((long long)lb * ntiles / G), t1 = (int)((long long)(lb + 1) * ntiles / G);
  const int launch0 = *base;
  for (int q = 0; q < Q; ++q) {
    for (int t = t0; t < t1; ++t) {
      batch_step_tile<THERMAL, OBJ>(tiles, slots, t, launch0 + q);
      __syncthreads();  // the block reduction's shared memory is reused by the next tile
    }
    if (!grid_barrier(bar, abort, (unsigned)(q + 1) * (unsigned)G, spin_limit)) return;
  }
  if constexpr (THERMAL)
    for (int t = t0; t < t1; ++t) batch_rebase_tile(tiles, slots, t, launch0 + Q - 1);
}

// The stored thermal state in the shift of T_in: own slots of non-wall nodes
// and the wall slots they read move by w_i (R(n) - T_in); every other slot was
// copied beforehand unchanged.
template <class G, bool MIR>
__global__ __launch_bounds__(kBlock) void k_export_thermal(const float* __restrict__ src,
                                                           const float* __restrict__ R,
                                                           const uint8_t* __restrict__ flags,
                                                           float* __restrict__ dst, KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N || (flags[n] & 7) >= K_WALL) return;
  const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
  const Nbr nb = make_nbr(x, y, z, P);
  const Mirror mr = MIR ? mirror_of(x, y, z, P) : Mirror{false, false, false};
  const float dR = R[n] - P.T_in;
  sfor<G::Q>([&](auto I) {
    constexpr int i = I;
    dst[(size_t)i * P.N + n] = src[(size_t)i * P.Np + n] + G::w[i] * dR;
    if constexpr (i != 0) {
      const Src sr = pull_src<G, i, -G::ex[i], -G::ey[i], -G::ez[i]>(nb, n, mr);
      if (sr.valid && (flags[sr.node] & 7) >= K_WALL)
        dst[(size_t)sr.slot * P.N + sr.node] = src[(size_t)sr.slot * P.Np + sr.node] + G::w[i] * dR;
    }
  });
}

// Device copy in 16-byte words (dwordx4 loads and stores): one word per
// thread, consecutive lanes on consecutive words.  Measured on MI355X, one
// word per thread over many blocks streams faster (6.2-6.3 TB/s read + write
// on 1 GiB) than two, four or eight words per thread (5.9, 5.8, 4.4 TB/s).
// The measured device ceiling that the step kernels' bytes are set against.
constexpr int kCopyUnroll = 1;
__global__ __launch_bounds__(kBlock) void k_copy16(const float4* __restrict__ src,
                                                   float4* __restrict__ dst, size_t n16) {
  const size_t base = (size_t)blockIdx.x * (kBlock * kCopyUnroll) + threadIdx.x;
  float4 v[kCopyUnroll];
#pragma unroll
  for (int k = 0; k < kCopyUnroll; ++k) {
    const size_t i = base + (size_t)k * kBlock;
    if (i < n16) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < kCopyUnroll; ++k) {
    const size_t i = base + (size_t)k * kBlock;
    if (i < n16) dst[i] = v[k];
  }
}

__global__ void k_fill(float* __restrict__ p, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0f;
}

__global__ void k_fill_u8(uint8_t* __restrict__ p, size_t count, uint8_t value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Level-set update of the design (Eqs. 14, 15, 67) on the design nodes.
// Laplacian: 7-point stencil (5-point in 2D) in lattice units over design
// nodes; a neighbour that is not a design node (or lies outside the box)
// counts as the node itself (no flux out of the design domain).
// ---------------------------------------------------------------------------
// sigma-weighted sum of the design neighbours' values and of their weights
// (sigma_x for the x neighbours, ...; the anisotropic regularisation of
// Sec. 3.3.4, all equal for the isotropic one).
struct LsNbr {
  float s;
  float w;
};
__device__ __forceinline__ LsNbr levelset_neighbours(const float* __restrict__ phi,
                                                     const uint8_t* __restrict__ flags, int n,
                                                     float sx, float sy, float sz,
                                                     const KParams& P) {
  const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
  LsNbr r{0.f, 0.f};
  auto add = [&](bool inside, int m, float sg) {
    if (!inside || (flags[m] & 7) != K_DESIGN) return;
    r.s += sg * phi[m];
    r.w += sg;
  };
  add(x > 0, n - 1, sx);
  add(x < P.nx - 1, n + 1, sx);
  add(y > 0, n - P.nx, sy);
  add(y < P.ny - 1, n + P.nx, sy);
  add(z > 0, n - P.plane, sz);
  add(z < P.nz - 1, n + P.plane, sz);
  return r;
}

// sum_a sigma_a d_aa phi at a design node
__device__ __forceinline__ float levelset_laplacian(const float* __restrict__ phi,
                                                    const uint8_t* __restrict__ flags, int n,
                                                    float sx, float sy, float sz,
                                                    const KParams& P) {
  const LsNbr r = levelset_neighbours(phi, flags, n, sx, sy, sz, P);
  return r.s - r.w * phi[n];
}

// Pass 1: sum |J'| and the fluid count (phi >= 0) over design nodes.
__global__ __launch_bounds__(kBlock) void k_levelset_stats(const float* __restrict__ phi,
                                                           const float* __restrict__ dJ,
                                                           const uint8_t* __restrict__ flags,
                                                           double* __restrict__ partials,
                                                           KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (n < P.N && (flags[n] & 7) == K_DESIGN) {
    acc[0] = fabs((double)dJ[n]);
    acc[1] = phi[n] >= 0.0f ? 1.0 : 0.0;
  }
  block_reduce_store<2>(acc, partials + (size_t)blockIdx.x * 2);
}

// Pass 2: sum |J'/scale - sigma lap(phi)| over design nodes (for lambda).
__global__ __launch_bounds__(kBlock) void k_levelset_lambda(const float* __restrict__ phi,
                                                            const float* __restrict__ dJ,
                                                            const uint8_t* __restrict__ flags,
                                                            float inv_scale, float sx, float sy,
                                                            float sz, double* __restrict__ partials,
                                                            KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  double acc[1] = {0.0};
  if (n < P.N && (flags[n] & 7) == K_DESIGN)
    acc[0] = fabs((double)(dJ[n] * inv_scale - levelset_laplacian(phi, flags, n, sx, sy, sz, P)));
  block_reduce_store<1>(acc, partials + blockIdx.x);
}

// Right-hand side of the semi-implicit step, r = phi - K (J'/scale + lambda),
// written to phi_out as the starting guess (non-design nodes copy phi).
__global__ __launch_bounds__(kBlock) void k_levelset_rhs(const float* __restrict__ phi,
                                                         float* __restrict__ phi_out,
                                                         const float* __restrict__ dJ,
                                                         const uint8_t* __restrict__ flags,
                                                         float inv_scale, float K, float lambda,
                                                         KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N) return;
  const bool d = (flags[n] & 7) == K_DESIGN;
  phi_out[n] = d ? phi[n] - K * (dJ[n] * inv_scale + lambda) : phi[n];
}

// One half-sweep of red-black Gauss-Seidel on (1 + K w) x - K s = r (the
// step (I - K sigma lap) phi_new = r with the sigma-weighted neighbour sum s
// and weight w), in place on x over the design nodes of parity `color`
// ((x + y + z) mod 2).
__global__ __launch_bounds__(kBlock) void k_levelset_sweep(const float* __restrict__ phi,
                                                           float* __restrict__ xs,
                                                           const float* __restrict__ dJ,
                                                           const uint8_t* __restrict__ flags,
                                                           float inv_scale, float K, float lambda,
                                                           float sx, float sy, float sz, int color,
                                                           KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N || (flags[n] & 7) != K_DESIGN) return;
  const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
  if (((x + y + z) & 1) != color) return;
  const LsNbr r = levelset_neighbours(xs, flags, n, sx, sy, sz, P);
  const float rhs = phi[n] - K * (dJ[n] * inv_scale + lambda);
  xs[n] = (rhs + K * r.s) / (1.0f + K * r.w);
}

// Last pass: clamp to [-1, 1] (Eq. 13) and gamma = 1 where phi >= 0, else 0
// (Eq. 15).
__global__ __launch_bounds__(kBlock) void k_levelset_finish(float* __restrict__ phi_out,
                                                            const uint8_t* __restrict__ flags,
                                                            float* __restrict__ gamma, KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N || (flags[n] & 7) != K_DESIGN) return;
  const float v = fminf(1.0f, fmaxf(-1.0f, phi_out[n]));
  phi_out[n] = v;
  gamma[n] = v >= 0.0f ? 1.0f : 0.0f;
}

hipError_t launch_levelset_stats(const float* phi, const float* dJ, const uint8_t* flags,
                                 double* partials, const KParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_levelset_stats, dim3(P.nblk), dim3(kBlock), 0, s, phi, dJ, flags, partials, P);
  return hipGetLastError();
}
hipError_t launch_levelset_lambda(const float* phi, const float* dJ, const uint8_t* flags,
                                  float inv_scale, const float* sigma, double* partials,
                                  const KParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_levelset_lambda, dim3(P.nblk), dim3(kBlock), 0, s, phi, dJ, flags, inv_scale,
                     sigma[0], sigma[1], sigma[2], partials, P);
  return hipGetLastError();
}
hipError_t launch_levelset_update(const float* phi, float* phi_out, const float* dJ,
                                  const uint8_t* flags, float* gamma, float inv_scale, float K,
                                  float lambda, const float* sigma, int sweeps, const KParams& P,
                                  hipStream_t s) {
  const dim3 g(P.nblk), b(kBlock);
  hipLaunchKernelGGL(k_levelset_rhs, g, b, 0, s, phi, phi_out, dJ, flags, inv_scale, K, lambda, P);
  for (int it = 0; it < sweeps; ++it)
    for (int color = 0; color < 2; ++color)
      hipLaunchKernelGGL(k_levelset_sweep, g, b, 0, s, phi, phi_out, dJ, flags, inv_scale, K,
                         lambda, sigma[0], sigma[1], sigma[2], color, P);
  hipLaunchKernelGGL(k_levelset_finish, g, b, 0, s, phi_out, flags, gamma, P);
  return hipGetLastError();
}

// Initial thermal state with heat generation: the rest state (zero in shifted
// variables) after its first collision, which adds w_i Q with
// Q = beta_max (1 - gamma) (1 - T_in) on design nodes.  The step kernels
// store post-collision populations, so this makes the stored start the image
// of the rest state under the collision, as the forward map C -> S -> B from
// the rest state has it (without a source that collision is the identity).
template <class G>
__global__ __launch_bounds__(kBlock) void k_heat_init(float* __restrict__ g,
                                                      const float* __restrict__ gamma,
                                                      const uint8_t* __restrict__ flags,
                                                      KParams P) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n >= P.N) return;
  if ((flags[n] & 7) != K_DESIGN) return;
  const float Q = P.beta * (1.0f - gamma[n]) * (1.0f - P.T_in);
  sfor<G::Q>([&](auto I) { g[(size_t)I * P.Np + n] = G::w[I] * Q; });
}

hipError_t launch_heat_init(float* g, const float* gamma, const uint8_t* flags, const KParams& P,
                            hipStream_t s) {
  if (!(P.beta > 0.0f)) return hipSuccess;
  const dim3 grid((P.N + kBlock - 1) / kBlock), block(kBlock);
  if (P.q == 9) hipLaunchKernelGGL((k_heat_init<Q5>), grid, block, 0, s, g, gamma, flags, P);
  else hipLaunchKernelGGL((k_heat_init<Q7>), grid, block, 0, s, g, gamma, flags, P);
  return hipGetLastError();
}

hipError_t launch_ref_init(float* R, const uint8_t* flags, const KParams& P, hipStream_t s) {
  const dim3 grid((P.Np + kBlock - 1) / kBlock), block(kBlock);
  hipLaunchKernelGGL(k_ref_init, grid, block, 0, s, R, flags, P);
  return hipGetLastError();
}

hipError_t launch_rebase(const RebaseArgs& a, hipStream_t s) {
  const dim3 grid(a.P.nblk), block(kBlock);
  const bool mir = (a.P.sx | a.P.sy | a.P.sz) != 0;
  if (a.P.q == 9) {
    if (mir) hipLaunchKernelGGL((k_rebase<Q5, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_rebase<Q5, false>), grid, block, 0, s, a);
  } else {
    if (mir) hipLaunchKernelGGL((k_rebase<Q7, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_rebase<Q7, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_export_thermal(const float* src, const float* R, const uint8_t* flags, float* dst,
                                 const KParams& P, hipStream_t s) {
  const dim3 grid(P.nblk), block(kBlock);
  const bool mir = (P.sx | P.sy | P.sz) != 0;
  if (P.q == 9) {
    if (mir) hipLaunchKernelGGL((k_export_thermal<Q5, true>), grid, block, 0, s, src, R, flags, dst, P);
    else hipLaunchKernelGGL((k_export_thermal<Q5, false>), grid, block, 0, s, src, R, flags, dst, P);
  } else {
    if (mir) hipLaunchKernelGGL((k_export_thermal<Q7, true>), grid, block, 0, s, src, R, flags, dst, P);
    else hipLaunchKernelGGL((k_export_thermal<Q7, false>), grid, block, 0, s, src, R, flags, dst, P);
  }
  return hipGetLastError();
}

template <bool TH, int OBJ>
static hipError_t persistent_launch(const Tile* tiles, int ntiles, const SlotDev* slots,
                                    const int* base, int Q, unsigned* bar, int* abort,
                                    int spin_limit, int grid, hipStream_t s) {
  void* args[] = {(void*)&tiles, (void*)&ntiles, (void*)&slots, (void*)&base, (void*)&Q,
                  (void*)&bar,   (void*)&abort,  (void*)&spin_limit};
  return hipLaunchCooperativeKernel((const void*)k_batch_persistent<TH, OBJ>, dim3(grid), dim3(kBlock),
                                    args, 0, s);
}

int persistent_grid_limit(bool thermal, int objective) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* k = nullptr;
  if (thermal) {
    switch (objective) {
      case OBJ_PRESSURE_DROP: k = (const void*)k_batch_persistent<true, OBJ_PRESSURE_DROP>; break;
      case OBJ_DISSIPATION: k = (const void*)k_batch_persistent<true, OBJ_DISSIPATION>; break;
      case OBJ_HEATGEN: k = (const void*)k_batch_persistent<true, OBJ_HEATGEN>; break;
      default: k = (const void*)k_batch_persistent<true, OBJ_HEATSINK>; break;
    }
  } else {
    k = objective == OBJ_PRESSURE_DROP ? (const void*)k_batch_persistent<false, OBJ_PRESSURE_DROP>
                                       : (const void*)k_batch_persistent<false, OBJ_DISSIPATION>;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kBlock, 0) != hipSuccess) return 0;
  return per * cus;
}

hipError_t launch_batch_persistent(const Tile* tiles, int ntiles, const SlotDev* slots,
                                   const int* base, int Q, bool thermal, int objective,
                                   unsigned* bar, int* abort, int spin_limit, int grid,
                                   hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  grid = std::min(grid, ntiles);
  if (thermal) {
    switch (objective) {
      case OBJ_PRESSURE_DROP:
        return persistent_launch<true, OBJ_PRESSURE_DROP>(tiles, ntiles, slots, base, Q, bar, abort, spin_limit, grid, s);
      case OBJ_DISSIPATION:
        return persistent_launch<true, OBJ_DISSIPATION>(tiles, ntiles, slots, base, Q, bar, abort, spin_limit, grid, s);
      case OBJ_HEATGEN:
        return persistent_launch<true, OBJ_HEATGEN>(tiles, ntiles, slots, base, Q, bar, abort, spin_limit, grid, s);
      default:
        return persistent_launch<true, OBJ_HEATSINK>(tiles, ntiles, slots, base, Q, bar, abort, spin_limit, grid, s);
    }
  }
  if (objective == OBJ_PRESSURE_DROP)
    return persistent_launch<false, OBJ_PRESSURE_DROP>(tiles, ntiles, slots, base, Q, bar, abort, spin_limit, grid, s);
  return persistent_launch<false, OBJ_DISSIPATION>(tiles, ntiles, slots, base, Q, bar, abort, spin_limit, grid, s);
}

hipError_t launch_batch_rebase(const Tile* tiles, int ntiles, const SlotDev* slots, const int* base,
                               int q, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int xper = ntiles / 8, xrem = ntiles % 8;
  hipLaunchKernelGGL(k_batch_rebase, dim3(ntiles), dim3(kBlock), 0, s, tiles, slots, base, q,
                     xper, xrem);
  return hipGetLastError();
}

hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t s) {
  if (n16 == 0) return hipSuccess;
  const size_t per = (size_t)kBlock * kCopyUnroll;
  const unsigned blocks = (unsigned)((n16 + per - 1) / per);
  hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(kBlock), 0, s, (const float4*)src, (float4*)dst,
                     n16);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, size_t count, uint8_t value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(kBlock), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, s, p, count);
  return hipGetLastError();
}

// Launch `kern` plainly, or with start/stop events stamped by the dispatch.
// Below this many blocks (4 waves per SIMD on 256 CUs) a lattice cannot keep
// enough waves in flight to hide memory latency: the step kernels then read
// the node's own inputs early (EARLY above).
constexpr int kEarlyBlocks = 1024;

template <class K, class A>
static void launch_step(K kern, int nblk, const A& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(kern, dim3(nblk), dim3(kBlock), 0, s, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(kBlock), 0, s, a);
}

// ---------------------------------------------------------------------------
// Streaming probe: the forward step's memory traffic without its arithmetic.
// Every population is pulled exactly as k_forward pulls it (same neighbour
// offsets, zero beyond non-periodic faces), gamma and the flag byte are read,
// and the pulled values are stored unchanged.  Its time per launch is the
// ceiling the pull pattern itself leaves the step kernel on the device.
// ---------------------------------------------------------------------------
template <class L, bool THERMAL>
__global__ __launch_bounds__(kBlock) void k_stream_probe(FwdArgs A) {
  using G = typename ThermalOf<L>::type;
  const KParams& P = A.P;
  const int n = remap_block(blockIdx.x, P) * kBlock + threadIdx.x;
  if (n >= P.N) return;
  const int x = n % P.nx, t = n / P.nx, y = t % P.ny, z = t / P.ny;
  const Nbr nb = make_nbr(x, y, z, P);
  const Mirror mr{false, false, false};
  // bit 7 of a flag byte is always clear: the select keeps the pulled value
  // while gamma and the flags are still read as the step reads them
  const bool never = (A.flags[n] & 0x80u) != 0;
  const float gv = A.gamma[n];
  float h[L::Q];
  sfor<L::Q>([&](auto I) {
    constexpr int i = I;
    h[i] = load_pull<L, i, -L::ex[i], -L::ey[i], -L::ez[i]>(A.fin, P.Np, nb, n, mr);
  });
  float k[G::Q];
  if constexpr (THERMAL) {
    // the reference temperatures are read where the step reads them
    const float Rn = A.Rin[n];
    load_pull_ref_all<G>(k, A.gin, A.Rin, P.Np, nb, n, mr, Rn, never, -1);
  }
  sfor<L::Q>([&](auto I) { A.fout[(size_t)I * P.Np + n] = never ? gv : h[I]; });
  if constexpr (THERMAL) sfor<G::Q>([&](auto I) { A.gout[(size_t)I * P.Np + n] = never ? gv : k[I]; });
}

template <class L, bool TH>
static void fwd_dispatch(const FwdArgs& a, bool diag, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const bool early = TH && a.P.nblk < kEarlyBlocks;
  if ((a.P.sx | a.P.sy | a.P.sz) != 0) {
    if (diag) launch_step(k_forward<L, true, TH, true>, a.P.nblk, a, s, ev0, ev1);
    else if constexpr (TH) {
      if (early) launch_step(k_forward_early<L, true>, a.P.nblk, a, s, ev0, ev1);
      else launch_step(k_forward<L, true, TH, false>, a.P.nblk, a, s, ev0, ev1);
    } else launch_step(k_forward<L, true, TH, false>, a.P.nblk, a, s, ev0, ev1);
  } else {
    if (diag) launch_step(k_forward<L, false, TH, true>, a.P.nblk, a, s, ev0, ev1);
    else if constexpr (TH) {
      if (early) launch_step(k_forward_early<L, false>, a.P.nblk, a, s, ev0, ev1);
      else launch_step(k_forward<L, false, TH, false>, a.P.nblk, a, s, ev0, ev1);
    } else launch_step(k_forward<L, false, TH, false>, a.P.nblk, a, s, ev0, ev1);
  }
}

hipError_t launch_forward(const FwdArgs& a, bool thermal, bool diag, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1) {
  if (thermal && a.P.q == 9) fwd_dispatch<Q9, true>(a, diag, s, ev0, ev1);
  else if (thermal) fwd_dispatch<Q19, true>(a, diag, s, ev0, ev1);
  else if (a.P.q == 9) fwd_dispatch<Q9, false>(a, diag, s, ev0, ev1);
  else fwd_dispatch<Q19, false>(a, diag, s, ev0, ev1);
  return hipGetLastError();
}

hipError_t launch_stream_probe(const FwdArgs& a, bool thermal, hipStream_t s) {
  if (thermal && a.P.q == 9) launch_step(k_stream_probe<Q9, true>, a.P.nblk, a, s, nullptr, nullptr);
  else if (thermal) launch_step(k_stream_probe<Q19, true>, a.P.nblk, a, s, nullptr, nullptr);
  else if (a.P.q == 9) launch_step(k_stream_probe<Q9, false>, a.P.nblk, a, s, nullptr, nullptr);
  else launch_step(k_stream_probe<Q19, false>, a.P.nblk, a, s, nullptr, nullptr);
  return hipGetLastError();
}

template <class L, bool MIR, bool TH, int OBJ>
static void adj_launch(const AdjArgs& a, bool diag, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if constexpr (!TH) {
    if (a.P.cont) {
      if (diag) launch_step(k_adjoint<L, MIR, TH, OBJ, true, true>, a.P.nblk, a, s, ev0, ev1);
      else launch_step(k_adjoint<L, MIR, TH, OBJ, false, true>, a.P.nblk, a, s, ev0, ev1);
      return;
    }
  }
  if (diag) launch_step(k_adjoint<L, MIR, TH, OBJ, true>, a.P.nblk, a, s, ev0, ev1);
  else if (TH && a.P.nblk < kEarlyBlocks) launch_step(k_adjoint<L, MIR, TH, OBJ, false, false, TH>, a.P.nblk, a, s, ev0, ev1);
  else launch_step(k_adjoint<L, MIR, TH, OBJ, false>, a.P.nblk, a, s, ev0, ev1);
}

template <class L, bool TH, int OBJ>
static void adj_dispatch(const AdjArgs& a, bool diag, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if ((a.P.sx | a.P.sy | a.P.sz) != 0) adj_launch<L, true, TH, OBJ>(a, diag, s, ev0, ev1);
  else adj_launch<L, false, TH, OBJ>(a, diag, s, ev0, ev1);
}

template <class L>
static void adj_dispatch_flow(const AdjArgs& a, int objective, bool diag, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1) {
  if (objective == OBJ_PRESSURE_DROP) adj_dispatch<L, false, OBJ_PRESSURE_DROP>(a, diag, s, ev0, ev1);
  else adj_dispatch<L, false, OBJ_DISSIPATION>(a, diag, s, ev0, ev1);
}

template <class L>
static void adj_dispatch_thermal(const AdjArgs& a, int objective, bool diag, hipStream_t s,
                                 hipEvent_t ev0, hipEvent_t ev1) {
  switch (objective) {
    case OBJ_PRESSURE_DROP: adj_dispatch<L, true, OBJ_PRESSURE_DROP>(a, diag, s, ev0, ev1); break;
    case OBJ_DISSIPATION: adj_dispatch<L, true, OBJ_DISSIPATION>(a, diag, s, ev0, ev1); break;
    case OBJ_HEATGEN: adj_dispatch<L, true, OBJ_HEATGEN>(a, diag, s, ev0, ev1); break;
    default: adj_dispatch<L, true, OBJ_HEATSINK>(a, diag, s, ev0, ev1); break;
  }
}

hipError_t launch_adjoint(const AdjArgs& a, bool thermal, int objective, bool diag, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1) {
  if (thermal && a.P.q == 9) {
    adj_dispatch_thermal<Q9>(a, objective, diag, s, ev0, ev1);
  } else if (thermal) {
    adj_dispatch_thermal<Q19>(a, objective, diag, s, ev0, ev1);
  } else if (a.P.q == 9) {
    adj_dispatch_flow<Q9>(a, objective, diag, s, ev0, ev1);
  } else {
    adj_dispatch_flow<Q19>(a, objective, diag, s, ev0, ev1);
  }
  return hipGetLastError();
}

template <bool MIR>
static void sens_launch(const SensArgs& a, bool thermal, hipStream_t s) {
  const dim3 grid(a.P.nblk), block(kBlock);
  if (thermal && a.P.q == 9) hipLaunchKernelGGL((k_sensitivity<Q9, MIR, true>), grid, block, 0, s, a);
  else if (thermal) hipLaunchKernelGGL((k_sensitivity<Q19, MIR, true>), grid, block, 0, s, a);
  else if (a.P.q == 9) hipLaunchKernelGGL((k_sensitivity<Q9, MIR, false>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((k_sensitivity<Q19, MIR, false>), grid, block, 0, s, a);
}

hipError_t launch_sensitivity(const SensArgs& a, bool thermal, hipStream_t s) {
  if ((a.P.sx | a.P.sy | a.P.sz) != 0) sens_launch<true>(a, thermal, s);
  else sens_launch<false>(a, thermal, s);
  return hipGetLastError();
}

template <class G>
static void thermal_launch(const ThermArgs& a, bool diag, hipStream_t s) {
  const dim3 grid(a.P.nblk), block(kBlock);
  if ((a.P.sx | a.P.sy | a.P.sz) != 0) {
    if (diag) hipLaunchKernelGGL((k_thermal<G, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_thermal<G, false, true>), grid, block, 0, s, a);
  } else {
    if (diag) hipLaunchKernelGGL((k_thermal<G, true, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_thermal<G, false, false>), grid, block, 0, s, a);
  }
}

hipError_t launch_thermal(const ThermArgs& a, bool diag, hipStream_t s) {
  if (a.P.q == 9) thermal_launch<Q5>(a, diag, s);
  else thermal_launch<Q7>(a, diag, s);
  return hipGetLastError();
}

hipError_t launch_thermal_init(const ThermArgs& a, hipStream_t s) {
  if (a.P.q == 9) hipLaunchKernelGGL((k_thermal_init<Q5>), dim3(a.P.nblk), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_thermal_init<Q7>), dim3(a.P.nblk), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_dissipation_source(const float* u, const float* gamma, const uint8_t* flags,
                                     float* G, const KParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_dissipation_source, dim3(P.nblk), dim3(kBlock), 0, s, u, gamma, flags, G, P);
  return hipGetLastError();
}

hipError_t launch_dissipation_objective(const float* u, const float* gamma, const uint8_t* flags,
                                        double* partials, const KParams& P, hipStream_t s) {
  hipLaunchKernelGGL(k_dissipation_objective, dim3(P.nblk), dim3(kBlock), 0, s, u, gamma, flags,
                     partials, P);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblk, int nvals, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, partials, nblk, nvals, out);
  return hipGetLastError();
}

hipError_t launch_batch(const Tile* tiles, int ntiles, const SlotDev* slots, const int* base,
                        int q, bool thermal, int objective, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int xper = ntiles / 8, xrem = ntiles % 8;
  const dim3 grid(ntiles), block(kBlock);
  if (thermal) {
    switch (objective) {
      case OBJ_PRESSURE_DROP:
        hipLaunchKernelGGL((k_batch<true, OBJ_PRESSURE_DROP>), grid, block, 0, s, tiles, slots, base, q, xper, xrem);
        break;
      case OBJ_DISSIPATION:
        hipLaunchKernelGGL((k_batch<true, OBJ_DISSIPATION>), grid, block, 0, s, tiles, slots, base, q, xper, xrem);
        break;
      case OBJ_HEATGEN:
        hipLaunchKernelGGL((k_batch<true, OBJ_HEATGEN>), grid, block, 0, s, tiles, slots, base, q, xper, xrem);
        break;
      default:
        hipLaunchKernelGGL((k_batch<true, OBJ_HEATSINK>), grid, block, 0, s, tiles, slots, base, q, xper, xrem);
        break;
    }
  } else {
    switch (objective) {
      case OBJ_PRESSURE_DROP:
        hipLaunchKernelGGL((k_batch<false, OBJ_PRESSURE_DROP>), grid, block, 0, s, tiles, slots, base, q, xper, xrem);
        break;
      default:
        hipLaunchKernelGGL((k_batch<false, OBJ_DISSIPATION>), grid, block, 0, s, tiles, slots, base, q, xper, xrem);
        break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_advance(int* base, int q, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, base, q);
  return hipGetLastError();
}

hipError_t launch_finalize_slots(const SlotDev* slots, int nslots, double* out, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_slots, dim3(nslots), dim3(kBlock), 0, s, slots, out);
  return hipGetLastError();
}

// Direction table of lattice `which` (0 D3Q19, 1 D3Q7, 2 D2Q9, 3 D2Q5).
template <class L>
static void table_of(int32_t* e, double* w, const double* wd) {
  for (int i = 0; i < L::Q; ++i) {
    e[3 * i] = L::ex[i];
    e[3 * i + 1] = L::ey[i];
    e[3 * i + 2] = L::ez[i];
    w[i] = wd[i];
  }
}

void lattice_table(int which, int32_t* e, double* w) {
  if (which == 0) {
    double wd[19];
    for (int i = 0; i < 19; ++i) wd[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    table_of<Q19>(e, w, wd);
  } else if (which == 1) {
    double wd[7];
    for (int i = 0; i < 7; ++i) wd[i] = (i == 0) ? 0.25 : 0.125;
    table_of<Q7>(e, w, wd);
  } else if (which == 2) {
    double wd[9];
    for (int i = 0; i < 9; ++i) wd[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    table_of<Q9>(e, w, wd);
  } else {
    double wd[5];
    for (int i = 0; i < 5; ++i) wd[i] = (i == 0) ? 0.5 : 0.125;
    table_of<Q5>(e, w, wd);
  }
}

}  // namespace lbmadj
