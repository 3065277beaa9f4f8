// FP64 CPU oracle for the discrete adjoint lattice Boltzmann method of
// J.-W. Luo, L. Chen, K. Yaji, W.-Q. Tao, "Improved adjoint lattice Boltzmann
// method for topology optimization of laminar convective heat transfer"
// (arXiv 2501.02161).
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously-correct
// reference used by the test suite, by the smoke check and by the CPU
// baseline timing of the benchmark.  The GPU library never links, loads or
// calls it, and it shares no code, header or table with the GPU library.
//
// Everything is written node by node in the order the paper states it:
//   forward step   f -> C (collision, Eq. 36 with the design-extended
//                  equilibrium of Eq. 12) -> S (streaming, periodic so that S
//                  is a permutation, Eq. 37) -> B (boundary conditions, Eqs. 7-9)
//   adjoint step   f*_C -> B^T (Eq. 54) -> S^T (Eqs. 55, 61) -> C^T minus dJ/df
//                  (Eqs. 56, 65), starting from f*_C = 0 (Eq. 53)
//   sensitivity    dJ/dgamma = explicit part - f*_S^T dC/dgamma (Eq. 66, first
//                  equality, with the exact derivative of Eq. 12)
// Arrays are node-major (the Q populations of one node are adjacent, as the
// paper lays out the global vector in Sec. 2.4); node index n = x + nx*(y + ny*z).
//
// Readings of the paper that this file adopts where the text is silent
// (3D boundary rules, thermal model, design parametrisation, objectives) are
// stated at the functions that implement them.  Every operator is templated
// on the scalar type so that complex-step differentiation can check the
// adjoint against the forward map.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double v) { return v; }
inline double re(const cplx& v) { return v.real(); }

// Node kinds and normal codes of the mask byte (input format).
enum Kind { K_DESIGN = 0, K_FLUID = 1, K_INLET = 2, K_OUTLET = 3, K_WALL = 4, K_HEATED = 5, K_SYM = 6 };
enum Objective { OBJ_PRESSURE_DROP = 0, OBJ_DISSIPATION = 1, OBJ_HEATSINK = 2, OBJ_HEATGEN = 3 };
const int NORMAL_VEC[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

// ---------------------------------------------------------------------------
// Lattices.  Weights follow Eq. (5).  The D2Q9 ordering is the one that makes
// Eqs. (7), (8), (58)-(60) read as printed: 0 rest, 1 (+1,0), 2 (0,+1),
// 3 (-1,0), 4 (0,-1), 5 (+1,+1), 6 (-1,+1), 7 (-1,-1), 8 (+1,-1).
// D3Q19: 0 rest, 1-6 the axis directions, 7-18 the twelve edge diagonals.
// D3Q7 (thermal): 0 rest, 1-6 the axis directions, weights 1/4 and 1/8, so that
// the lattice sound speed squared of the thermal lattice is 1/4.
// ---------------------------------------------------------------------------
struct Lattice {
  int Q = 0;
  int e[19][3] = {};
  double w[19] = {};
  int opp[19] = {};
  double cs2 = 1.0 / 3.0;
};

void finish_lattice(Lattice& L) {
  for (int i = 0; i < L.Q; ++i)
    for (int j = 0; j < L.Q; ++j)
      if (L.e[j][0] == -L.e[i][0] && L.e[j][1] == -L.e[i][1] && L.e[j][2] == -L.e[i][2])
        L.opp[i] = j;
}

Lattice make_d2q9() {
  Lattice L;
  L.Q = 9;
  const int e[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
  for (int i = 0; i < 9; ++i) {
    L.e[i][0] = e[i][0];
    L.e[i][1] = e[i][1];
    L.e[i][2] = 0;
    L.w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
  finish_lattice(L);
  return L;
}

Lattice make_d3q19() {
  Lattice L;
  L.Q = 19;
  const int e[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                        {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                        {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                        {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  for (int i = 0; i < 19; ++i) {
    for (int a = 0; a < 3; ++a) L.e[i][a] = e[i][a];
    L.w[i] = (i == 0) ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  finish_lattice(L);
  return L;
}

// D2Q5 (thermal lattice of a 2D problem): rest and the four axis directions,
// weights 1/2 and 1/8, so that the lattice sound speed squared is 1/4 as on
// D3Q7: the same equilibrium w T (1 + 4 e.u) and the same tau_g(D).
Lattice make_d2q5() {
  Lattice L;
  L.Q = 5;
  const int e[5][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}};
  for (int i = 0; i < 5; ++i) {
    for (int a = 0; a < 3; ++a) L.e[i][a] = e[i][a];
    L.w[i] = (i == 0) ? 0.5 : 0.125;
  }
  L.cs2 = 0.25;
  finish_lattice(L);
  return L;
}

Lattice make_d3q7() {
  Lattice L;
  L.Q = 7;
  const int e[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  for (int i = 0; i < 7; ++i) {
    for (int a = 0; a < 3; ++a) L.e[i][a] = e[i][a];
    L.w[i] = (i == 0) ? 0.25 : 0.125;
  }
  L.cs2 = 0.25;
  finish_lattice(L);
  return L;
}

}  // namespace

// Configuration handed over from Python (plain C layout).
struct OrcConfig {
  int32_t nx, ny, nz, dim, thermal, objective;
  double tau, rho0, Re, L_ref, alpha_max, q_brink, Pr, k_ratio, q_ramp, q_w, T_in, w_dp;
  // symmetric[a] = 1: mirror plane between layers n_a - 2 and n_a - 1 of axis a
  // (layer n_a - 1 holds SYM nodes); inlet_rho > 0: pressure inlets at that
  // density; beta_max > 0: volumetric heat generation beta(gamma) (1 - T)
  int32_t symmetric[3], pad;
  double inlet_rho, beta_max;
};

namespace {

struct Problem {
  OrcConfig c{};
  int nx = 0, ny = 0, nz = 0, N = 0;
  Lattice F, G;  // flow lattice, thermal lattice
  bool thermal = false;
  double nu = 0, U_peak = 0, Df = 0;
  std::vector<int> kind, ncode;   // per node
  // streaming as a gather: slot (n, i) of the streamed state takes slot
  // src[n*Q + i] of the post-collision state (flow F, thermal G)
  std::vector<int64_t> srcF, srcG;
  std::vector<double> u_in;       // prescribed normal inlet speed
  std::vector<char> layer;        // objective layer (first layer on a heated wall)
  int n_inlet = 0, n_layer = 0, n_nonwall = 0;

  int idx(int x, int y, int z) const { return x + nx * (y + ny * z); }
  void coords(int n, int& x, int& y, int& z) const {
    x = n % nx;
    y = (n / nx) % ny;
    z = n / (nx * ny);
  }
  // node n + s*e with periodic wrap (the paper makes S a permutation this way, Sec. 2.4 (2))
  int shift(int n, const int* e, int s) const {
    int x, y, z;
    coords(n, x, y, z);
    x = ((x + s * e[0]) % nx + nx) % nx;
    y = ((y + s * e[1]) % ny + ny) % ny;
    z = ((z + s * e[2]) % nz + nz) % nz;
    return idx(x, y, z);
  }
  // nodes that do not collide and are not part of the fluid: walls, heated
  // walls and the layers beyond a symmetry plane (never read)
  bool is_wall(int n) const { return kind[n] == K_WALL || kind[n] == K_HEATED || kind[n] == K_SYM; }
  bool collides(int n) const { return !is_wall(n); }
  bool is_design(int n) const { return kind[n] == K_DESIGN; }
  // index of the lattice direction equal to the node's inward normal
  int normal_dir(const Lattice& L, int n) const {
    const int* v = NORMAL_VEC[ncode[n]];
    for (int i = 0; i < L.Q; ++i)
      if (L.e[i][0] == v[0] && L.e[i][1] == v[1] && L.e[i][2] == v[2]) return i;
    return -1;
  }
};

// ---------------------------------------------------------------------------
// Design parametrisation.  The paper relaxes the fluid indicator alpha of
// Eq. (11) and enters it through u <- alpha u in the equilibrium (Eq. 12).
// Here the design field gamma in [0,1] sets a Brinkman inverse permeability
// a_B(gamma) = alpha_max q (1-gamma)/(q+gamma) and the velocity scale of Eq. (12)
// is chi = 1 - tau a_B(gamma), which removes exactly a_B rho0 u of momentum per
// step.  Non-design nodes use chi = 1.
// ---------------------------------------------------------------------------
template <class S>
S brinkman(const Problem& P, const S& g) {
  return P.c.alpha_max * P.c.q_brink * (1.0 - g) / (P.c.q_brink + g);
}
template <class S>
S brinkman_d(const Problem& P, const S& g) {
  return -P.c.alpha_max * P.c.q_brink * (1.0 + P.c.q_brink) / ((P.c.q_brink + g) * (P.c.q_brink + g));
}
template <class S>
S chi_of(const Problem& P, int n, const S& g) {
  if (!P.is_design(n)) return S(1.0);
  return 1.0 - P.c.tau * brinkman(P, g);
}
template <class S>
S chi_d(const Problem& P, int n, const S& g) {
  if (!P.is_design(n)) return S(0.0);
  return -P.c.tau * brinkman_d(P, g);
}
// Thermal relaxation time: tau_g = 1/2 + D k(gamma)/cs2, D = nu/Pr the fluid
// diffusivity, k the RAMP interpolation between solid (ratio r) and fluid (1).
template <class S>
S khat(const Problem& P, const S& g) {
  const double r = P.c.k_ratio, q = P.c.q_ramp;
  return r + (1.0 - r) * g / (1.0 + q * (1.0 - g));
}
template <class S>
S khat_d(const Problem& P, const S& g) {
  const double r = P.c.k_ratio, q = P.c.q_ramp;
  const S den = 1.0 + q * (1.0 - g);
  return (1.0 - r) * (1.0 + q) / (den * den);
}
template <class S>
S tau_g(const Problem& P, int n, const S& g) {
  if (!P.is_design(n)) return S(0.5 + P.Df / P.G.cs2);
  return 0.5 + P.Df * khat(P, g) / P.G.cs2;
}
template <class S>
S tau_g_d(const Problem& P, int n, const S& g) {
  if (!P.is_design(n)) return S(0.0);
  return P.Df * khat_d(P, g) / P.G.cs2;
}

// Volumetric heat generation of the paper's heat sink (Eqs. 68, 69, 71):
// Q = beta(gamma) (1 - T) with beta(gamma) = beta_max (1 - gamma) on design
// nodes (gamma = 1 fluid, 0 solid: heat is generated in the solid), 0 elsewhere.
template <class S>
S beta_of(const Problem& P, int n, const S& g) {
  if (!P.is_design(n) || P.c.beta_max <= 0.0) return S(0.0);
  return P.c.beta_max * (1.0 - g);
}
double beta_d(const Problem& P, int n) { return (P.is_design(n) && P.c.beta_max > 0.0) ? -P.c.beta_max : 0.0; }

// Macroscopic moments of Eq. (6) at one node.
template <class S>
void moments(const Problem& P, const S* f, S& rho, S u[3]) {
  rho = 0.0;
  u[0] = u[1] = u[2] = 0.0;
  for (int i = 0; i < P.F.Q; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) u[a] += double(P.F.e[i][a]) * f[i];
  }
  for (int a = 0; a < 3; ++a) u[a] /= P.c.rho0;
}

// ---------------------------------------------------------------------------
// Collision, Eq. (36), with the equilibrium of Eq. (12) (incompressible model of
// Eq. (4) with u replaced by chi u).  Thermal populations relax with tau_g to
// g_eq = w T (1 + e.u/cs2), advected by the node's velocity u (the thermal model
// of the paper's Ref. [14] is not given; this linear-equilibrium D3Q7 BGK is the
// reading).  Wall nodes do not collide.
// ---------------------------------------------------------------------------
template <class S>
void collide(const Problem& P, const S* gamma, S* f, S* g) {
  const int Q = P.F.Q, Qg = P.G.Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    if (!P.collides(n)) continue;
    S* fn = f + (size_t)n * Q;
    S rho, u[3];
    moments(P, fn, rho, u);
    const S chi = chi_of(P, n, gamma[n]);
    const S ux = chi * u[0], uy = chi * u[1], uz = chi * u[2];
    const S uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < Q; ++i) {
      const S eu = double(P.F.e[i][0]) * ux + double(P.F.e[i][1]) * uy + double(P.F.e[i][2]) * uz;
      const S feq = P.F.w[i] * (rho + P.c.rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
      fn[i] = fn[i] - (fn[i] - feq) / P.c.tau;
    }
    if (P.thermal) {
      S* gn = g + (size_t)n * Qg;
      S T = 0.0;
      for (int i = 0; i < Qg; ++i) T += gn[i];
      const S tg = tau_g(P, n, gamma[n]);
      const S Qh = beta_of(P, n, gamma[n]) * (1.0 - T);  // heat source of Eq. (71)
      for (int i = 0; i < Qg; ++i) {
        const S eu = double(P.G.e[i][0]) * u[0] + double(P.G.e[i][1]) * u[1] + double(P.G.e[i][2]) * u[2];
        const S geq = P.G.w[i] * T * (1.0 + eu / P.G.cs2);
        gn[i] = gn[i] - (gn[i] - geq) / tg + P.G.w[i] * Qh;
      }
    }
  }
}

// Source slot of streaming for slot (n, i) of lattice L.  Streaming pulls
// from n - e_i (periodic wrap, so S is a permutation as in Sec. 2.4 (2)).  A
// source on the layer beyond a symmetry plane is replaced by its mirror image:
// the node one layer back, with the direction's normal component reversed
// (specular reflection at a plane midway between the two layers; the paper's
// quarter-domain heat sink, Sec. 3.3).  To keep S a permutation, the nodes of
// that layer keep their own slots and a source that would wrap around the
// other end of a symmetric axis reverses direction at the node itself; both
// only ever touch slots that no fluid node reads.  The thermal outflow is the
// other exception: at an OUTLET node the population along the inward normal
// would come from outside and takes the node's own post-collision value
// instead (zero-gradient outflow, a reading: the paper's Ref. [14] is not
// given).
int64_t stream_source(const Problem& P, const Lattice& L, bool thermal, int n, int i) {
  if (P.kind[n] == K_SYM) return (int64_t)n * L.Q + i;
  if (thermal && P.kind[n] == K_OUTLET && i == P.normal_dir(L, n)) return (int64_t)n * L.Q + i;
  const int lim[3] = {P.nx, P.ny, P.nz};
  int x[3], e[3] = {L.e[i][0], L.e[i][1], L.e[i][2]};
  P.coords(n, x[0], x[1], x[2]);
  int c[3];
  for (int a = 0; a < 3; ++a) {
    c[a] = x[a] - e[a];
    if (P.c.symmetric[a] && c[a] == lim[a] - 1) {
      c[a] = lim[a] - 2;
      e[a] = -e[a];
    } else if (P.c.symmetric[a] && c[a] < 0) {
      c[a] = x[a];
      e[a] = -e[a];
    }
    c[a] = (c[a] % lim[a] + lim[a]) % lim[a];
  }
  int d = -1;
  for (int j = 0; j < L.Q; ++j)
    if (L.e[j][0] == e[0] && L.e[j][1] == e[1] && L.e[j][2] == e[2]) d = j;
  return (int64_t)P.idx(c[0], c[1], c[2]) * L.Q + d;
}

// ---------------------------------------------------------------------------
// Streaming, Eq. (37), as the gather S: f_S(slot) = f_C(src(slot)).
// ---------------------------------------------------------------------------
template <class S>
void stream(const Problem& P, const S* fC, const S* gC, S* fS, S* gS) {
  const int Q = P.F.Q, Qg = P.G.Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    for (int i = 0; i < Q; ++i) fS[(size_t)n * Q + i] = fC[P.srcF[(size_t)n * Q + i]];
    if (P.thermal)
      for (int i = 0; i < Qg; ++i) gS[(size_t)n * Qg + i] = gC[P.srcG[(size_t)n * Qg + i]];
  }
}

// Direction classes at a port with inward normal nv: unknown (e.nv > 0),
// outgoing (e.nv < 0), tangential (e.nv == 0).
int dir_class(const Lattice& L, int i, const int* nv) {
  const int d = L.e[i][0] * nv[0] + L.e[i][1] * nv[1] + L.e[i][2] * nv[2];
  return d > 0 ? 1 : (d < 0 ? -1 : 0);
}
// Tangential axes of a port (the axes of the lattice other than the normal axis).
int tangential_axes(const Problem& P, const int* nv, int* t) {
  int m = 0;
  const int dim = P.c.dim;
  for (int a = 0; a < dim; ++a)
    if (nv[a] == 0) t[m++] = a;
  return m;
}

// ---------------------------------------------------------------------------
// Zou-He open boundary, generalising Eqs. (7) and (8) to any axis normal and to
// D3Q19 (the paper's 3D version is in a supplement that is not available).
// For unknown i:   f_i = f_ibar + 6 w_i rho0 u_n - 1/2 sum_t (e_i.t) N_t,
//                  N_t = sum over tangential j of (e_j.t) f_j.
// Velocity inlet: u_n is the prescribed normal speed (tangential speed 0, as in
// Eq. 7).  Pressure outlet (rho = rho0, Eq. 8):
//                  rho0 u_n = rho0 - sum_tangential f - 2 sum_outgoing f,
// and a pressure inlet (the paper's heat sink is driven by a fixed inlet
// pressure, Sec. 3.3) by the same rule with rho_in in place of rho0.
// For D2Q9 at the left inlet and the bottom outlet this is Eq. (7) and Eq. (8)
// term by term.
// ---------------------------------------------------------------------------
template <class S>
void zou_he(const Problem& P, int n, S* f) {
  const Lattice& L = P.F;
  const int* nv = NORMAL_VEC[P.ncode[n]];
  int t[3];
  const int nt = tangential_axes(P, nv, t);
  S Nt[3] = {0.0, 0.0, 0.0};
  S sumT0 = 0.0, sumO = 0.0;
  for (int j = 0; j < L.Q; ++j) {
    const int c = dir_class(L, j, nv);
    if (c == 0) {
      sumT0 += f[j];
      for (int k = 0; k < nt; ++k) Nt[k] += double(L.e[j][t[k]]) * f[j];
    } else if (c < 0) {
      sumO += f[j];
    }
  }
  S jn;  // rho0 * u_n
  if (P.kind[n] == K_INLET && P.c.inlet_rho <= 0.0)
    jn = P.c.rho0 * P.u_in[n];
  else  // pressure outlet (rho0), or pressure inlet (inlet_rho) by the same rule
    jn = (P.kind[n] == K_INLET ? P.c.inlet_rho : P.c.rho0) - sumT0 - 2.0 * sumO;
  for (int i = 0; i < L.Q; ++i) {
    if (dir_class(L, i, nv) != 1) continue;
    S v = f[L.opp[i]] + 6.0 * L.w[i] * jn;
    for (int k = 0; k < nt; ++k) v -= 0.5 * double(L.e[i][t[k]]) * Nt[k];
    f[i] = v;
  }
}

// ---------------------------------------------------------------------------
// Boundary step B (Eqs. 7-9).  Walls: full bounce-back, every pair i <-> ibar
// is swapped and the wall node does not collide, so the local block is a
// symmetric permutation (the paper's statement on walls in Sec. 2.4).
// Thermal: inlet Dirichlet T = T_in by the sum rule on the population along the
// inward normal; heated wall: swap, then the heat flux q_w is added to the
// population along the inward normal; outlet: handled in streaming.
// ---------------------------------------------------------------------------
template <class S>
void boundary(const Problem& P, S* f, S* g) {
  const int Q = P.F.Q, Qg = P.G.Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    S* fn = f + (size_t)n * Q;
    const int k = P.kind[n];
    if (k == K_WALL || k == K_HEATED) {
      S tmp[19];
      for (int i = 0; i < Q; ++i) tmp[i] = fn[P.F.opp[i]];
      for (int i = 0; i < Q; ++i) fn[i] = tmp[i];
    } else if (k == K_INLET || k == K_OUTLET) {
      zou_he(P, n, fn);
    }
    if (!P.thermal) continue;
    S* gn = g + (size_t)n * Qg;
    if (k == K_WALL || k == K_HEATED) {
      S tmp[7];
      for (int i = 0; i < Qg; ++i) tmp[i] = gn[P.G.opp[i]];
      for (int i = 0; i < Qg; ++i) gn[i] = tmp[i];
      if (k == K_HEATED) gn[P.normal_dir(P.G, n)] += P.c.q_w;
    } else if (k == K_INLET) {
      const int in = P.normal_dir(P.G, n);
      S s = 0.0;
      for (int j = 0; j < Qg; ++j)
        if (j != in) s += gn[j];
      gn[in] = P.c.T_in - s;
    }
  }
}

// Equilibrium at rest, the initial state f(0).
template <class S>
void init_state(const Problem& P, S* f, S* g) {
  for (int n = 0; n < P.N; ++n) {
    for (int i = 0; i < P.F.Q; ++i) f[(size_t)n * P.F.Q + i] = P.F.w[i] * P.c.rho0;
    if (P.thermal)
      for (int i = 0; i < P.G.Q; ++i) g[(size_t)n * P.G.Q + i] = P.G.w[i] * P.c.T_in;
  }
}

// Convergence quantity of the paper's residual |I(t) - I(t - 1000 dt)| / |I(t)|
// (Sec. 3.1), with I = mean |u| (and mean T) over the non-wall nodes.
template <class S>
void forward_monitor(const Problem& P, const S* f, const S* g, double& Iu, double& IT) {
  double su = 0.0, sT = 0.0;
  for (int n = 0; n < P.N; ++n) {
    if (P.is_wall(n)) continue;
    S rho, u[3];
    moments(P, f + (size_t)n * P.F.Q, rho, u);
    su += std::sqrt(re(u[0]) * re(u[0]) + re(u[1]) * re(u[1]) + re(u[2]) * re(u[2]));
    if (P.thermal) {
      S T = 0.0;
      for (int i = 0; i < P.G.Q; ++i) T += g[(size_t)n * P.G.Q + i];
      sT += re(T);
    }
  }
  Iu = su / P.n_nonwall;
  IT = sT / P.n_nonwall;
}

bool rel_converged(double now, double before, double tol) {
  if (!(tol > 0.0)) return false;
  return std::fabs(now - before) <= tol * std::fabs(now);
}

// Forward solve: f(0) at rest (or the given state when warm), then repeat
// C, S, B (Eq. 35) until the residual criterion or max_steps.  Returns 0 when
// converged, 1 when max_steps was reached, -1 on a non-finite monitor.
template <class S>
int forward(const Problem& P, const S* gamma, S* f, S* g, int max_steps, double tol, int check_every,
            int warm, int* steps_out, double* res_out) {
  if (!warm) init_state(P, f, g);
  std::vector<S> fS((size_t)P.N * P.F.Q), gS(P.thermal ? (size_t)P.N * P.G.Q : 1);
  double prevU = 0, prevT = 0, resU = 0, resT = 0;
  bool have_prev = false;
  int status = 1, k = 0;
  for (k = 1; k <= max_steps; ++k) {
    collide(P, gamma, f, g);
    stream(P, f, g, fS.data(), gS.data());
    std::copy(fS.begin(), fS.end(), f);
    if (P.thermal) std::copy(gS.begin(), gS.end(), g);
    boundary(P, f, g);
    if (check_every > 0 && k % check_every == 0) {
      double Iu, IT;
      forward_monitor(P, f, g, Iu, IT);
      if (!std::isfinite(Iu) || !std::isfinite(IT)) {
        status = -1;
        break;
      }
      if (have_prev) {
        resU = std::fabs(Iu - prevU) / std::max(std::fabs(Iu), 1e-300);
        resT = std::fabs(IT - prevT) / std::max(std::fabs(IT), 1e-300);
        if (rel_converged(Iu, prevU, tol) && (!P.thermal || rel_converged(IT, prevT, tol))) {
          status = 0;
          break;
        }
      }
      prevU = Iu;
      prevT = IT;
      have_prev = true;
    }
  }
  if (steps_out) *steps_out = std::min(k, max_steps);
  if (res_out) {
    res_out[0] = resU;
    res_out[1] = resT;
  }
  return status;
}

// ---------------------------------------------------------------------------
// Objectives, evaluated on the post-boundary state f (and g).
//  PRESSURE_DROP (the paper's J = p_in of Eq. 34, minus the constant outlet
//    pressure): J = w_dp (mean over inlet nodes of rho/3 - rho0/3).
//  DISSIPATION: J = sum over axis edges between in-box non-wall nodes of
//    rho0 nu |u(x+e) - u(x)|^2 + sum over design nodes of a_B(gamma) rho0 |u|^2.
//  HEATSINK: J = mean T over the layer of nodes on the heated walls
//    + w_dp (mean inlet rho/3 - rho0/3).
// ---------------------------------------------------------------------------
template <class S>
S objective(const Problem& P, const S* gamma, const S* f, const S* g) {
  S J = 0.0;
  const int obj = P.c.objective;
  if (obj == OBJ_PRESSURE_DROP || obj == OBJ_HEATSINK) {
    S s = 0.0;
    for (int n = 0; n < P.N; ++n) {
      if (P.kind[n] != K_INLET) continue;
      for (int i = 0; i < P.F.Q; ++i) s += f[(size_t)n * P.F.Q + i];
    }
    J += P.c.w_dp * (s / double(P.n_inlet) / 3.0 - P.c.rho0 / 3.0);
  }
  if (obj == OBJ_HEATSINK) {
    S s = 0.0;
    for (int n = 0; n < P.N; ++n) {
      if (!P.layer[n]) continue;
      for (int i = 0; i < P.G.Q; ++i) s += g[(size_t)n * P.G.Q + i];
    }
    J += s / double(P.n_layer);
  }
  if (obj == OBJ_HEATGEN) {
    // J = - sum_j Q(x_j) = - sum_j beta(gamma_j) (1 - T_j)   (Eq. 72)
    for (int n = 0; n < P.N; ++n) {
      if (!P.is_design(n)) continue;
      S T = 0.0;
      for (int i = 0; i < P.G.Q; ++i) T += g[(size_t)n * P.G.Q + i];
      J -= beta_of(P, n, gamma[n]) * (1.0 - T);
    }
  }
  if (obj == OBJ_DISSIPATION) {
    std::vector<S> u((size_t)P.N * 3);
    for (int n = 0; n < P.N; ++n) {
      S rho;
      moments(P, f + (size_t)n * P.F.Q, rho, &u[(size_t)n * 3]);
    }
    for (int n = 0; n < P.N; ++n) {
      if (P.is_wall(n)) continue;
      int x, y, z;
      P.coords(n, x, y, z);
      const int c[3] = {x, y, z}, lim[3] = {P.nx, P.ny, P.nz};
      for (int a = 0; a < 3; ++a) {
        if (c[a] + 1 >= lim[a]) continue;
        const int m = n + (a == 0 ? 1 : (a == 1 ? P.nx : P.nx * P.ny));
        if (P.is_wall(m)) continue;
        for (int b = 0; b < 3; ++b) {
          const S d = u[(size_t)m * 3 + b] - u[(size_t)n * 3 + b];
          J += P.c.rho0 * P.nu * d * d;
        }
      }
      if (P.is_design(n)) {
        const S ab = brinkman(P, gamma[n]);
        for (int b = 0; b < 3; ++b) J += ab * P.c.rho0 * u[(size_t)n * 3 + b] * u[(size_t)n * 3 + b];
      }
    }
  }
  return J;
}

// Partial derivatives of J: dJ/df (Q per node), dJ/dg (Qg per node), and the
// explicit dJ/dgamma (per node).  Written out from the objectives above.
void objective_grad(const Problem& P, const double* gamma, const double* f, const double* g, double* jf,
                    double* jg, double* jgam) {
  const int Q = P.F.Q, Qg = P.G.Q;
  std::fill(jf, jf + (size_t)P.N * Q, 0.0);
  if (P.thermal) std::fill(jg, jg + (size_t)P.N * Qg, 0.0);
  std::fill(jgam, jgam + P.N, 0.0);
  const int obj = P.c.objective;
  if (obj == OBJ_PRESSURE_DROP || obj == OBJ_HEATSINK) {
    const double c = P.c.w_dp / (3.0 * P.n_inlet);
    for (int n = 0; n < P.N; ++n)
      if (P.kind[n] == K_INLET)
        for (int i = 0; i < Q; ++i) jf[(size_t)n * Q + i] += c;
  }
  if (obj == OBJ_HEATSINK) {
    const double c = 1.0 / P.n_layer;
    for (int n = 0; n < P.N; ++n)
      if (P.layer[n])
        for (int i = 0; i < Qg; ++i) jg[(size_t)n * Qg + i] += c;
  }
  if (obj == OBJ_HEATGEN) {
    // dJ/dg_i = beta(gamma) (T = sum g), explicit dJ/dgamma = -beta'(gamma) (1 - T)
    for (int n = 0; n < P.N; ++n) {
      if (!P.is_design(n)) continue;
      double T = 0.0;
      for (int i = 0; i < Qg; ++i) T += g[(size_t)n * Qg + i];
      const double b = beta_of(P, n, gamma[n]);
      for (int i = 0; i < Qg; ++i) jg[(size_t)n * Qg + i] += b;
      jgam[n] += -beta_d(P, n) * (1.0 - T);
    }
  }
  if (obj == OBJ_DISSIPATION) {
    std::vector<double> u((size_t)P.N * 3), dJdu((size_t)P.N * 3, 0.0);
    for (int n = 0; n < P.N; ++n) {
      double rho;
      moments(P, f + (size_t)n * Q, rho, &u[(size_t)n * 3]);
    }
    for (int n = 0; n < P.N; ++n) {
      if (P.is_wall(n)) continue;
      int x, y, z;
      P.coords(n, x, y, z);
      const int c[3] = {x, y, z}, lim[3] = {P.nx, P.ny, P.nz};
      for (int a = 0; a < 3; ++a) {
        if (c[a] + 1 >= lim[a]) continue;
        const int m = n + (a == 0 ? 1 : (a == 1 ? P.nx : P.nx * P.ny));
        if (P.is_wall(m)) continue;
        for (int b = 0; b < 3; ++b) {
          const double d = u[(size_t)m * 3 + b] - u[(size_t)n * 3 + b];
          dJdu[(size_t)m * 3 + b] += 2.0 * P.c.rho0 * P.nu * d;
          dJdu[(size_t)n * 3 + b] -= 2.0 * P.c.rho0 * P.nu * d;
        }
      }
      if (P.is_design(n)) {
        const double ab = brinkman(P, gamma[n]);
        double uu = 0.0;
        for (int b = 0; b < 3; ++b) {
          dJdu[(size_t)n * 3 + b] += 2.0 * ab * P.c.rho0 * u[(size_t)n * 3 + b];
          uu += u[(size_t)n * 3 + b] * u[(size_t)n * 3 + b];
        }
        jgam[n] += brinkman_d(P, gamma[n]) * P.c.rho0 * uu;
      }
    }
    // u = sum_i e_i f_i / rho0 (Eq. 6), so dJ/df_i = e_i . dJ/du / rho0
    for (int n = 0; n < P.N; ++n)
      for (int i = 0; i < Q; ++i) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += double(P.F.e[i][b]) * dJdu[(size_t)n * 3 + b];
        jf[(size_t)n * Q + i] += s / P.c.rho0;
      }
  }
}

// ---------------------------------------------------------------------------
// Local boundary Jacobian B_j = d f / d f_S at a port node (Eq. 57), written
// out from the Zou-He rule above: identity rows for the known populations, and
// for unknown i
//   B_ij = [j == ibar] - 1/2 [j tangential] sum_t (e_i.t)(e_j.t) - 6 w_i c_j,
// with c_j = 0 at a velocity inlet, and at an outlet or a pressure inlet
// c_j = 1 for tangential j and 2 for outgoing j (from rho0 u_n = rho_b -
// sum_T f - 2 sum_O f).  For the D2Q9 inlet this is the matrix printed as
// Eq. (58).
// ---------------------------------------------------------------------------
void bc_matrix(const Problem& P, int n, double* B) {
  const Lattice& L = P.F;
  const int Q = L.Q;
  for (int i = 0; i < Q * Q; ++i) B[i] = 0.0;
  const int k = P.kind[n];
  if (k == K_WALL || k == K_HEATED) {
    for (int i = 0; i < Q; ++i) B[i * Q + L.opp[i]] = 1.0;
    return;
  }
  if (k != K_INLET && k != K_OUTLET) {
    for (int i = 0; i < Q; ++i) B[i * Q + i] = 1.0;
    return;
  }
  const int* nv = NORMAL_VEC[P.ncode[n]];
  int t[3];
  const int nt = tangential_axes(P, nv, t);
  for (int i = 0; i < Q; ++i) {
    if (dir_class(L, i, nv) != 1) {
      B[i * Q + i] = 1.0;
      continue;
    }
    for (int j = 0; j < Q; ++j) {
      const int cj = dir_class(L, j, nv);
      double v = (j == L.opp[i]) ? 1.0 : 0.0;
      if (cj == 0)
        for (int kk = 0; kk < nt; ++kk) v -= 0.5 * L.e[i][t[kk]] * L.e[j][t[kk]];
      if (k == K_OUTLET || P.c.inlet_rho > 0.0) v -= 6.0 * L.w[i] * (cj == 0 ? 1.0 : (cj < 0 ? 2.0 : 0.0));
      B[i * Q + j] = v;
    }
  }
}
// Thermal boundary Jacobian (7x7) at a node: swap at walls (the heat flux is a
// constant), sum rule at the inlet, identity elsewhere.
void bc_matrix_thermal(const Problem& P, int n, double* B) {
  const Lattice& L = P.G;
  const int Q = L.Q;
  for (int i = 0; i < Q * Q; ++i) B[i] = 0.0;
  const int k = P.kind[n];
  if (k == K_WALL || k == K_HEATED) {
    for (int i = 0; i < Q; ++i) B[i * Q + L.opp[i]] = 1.0;
    return;
  }
  for (int i = 0; i < Q; ++i) B[i * Q + i] = 1.0;
  if (k == K_INLET) {
    const int in = P.normal_dir(L, n);
    for (int j = 0; j < Q; ++j) B[in * Q + j] = (j == in) ? 0.0 : -1.0;
  }
}

// Adjoint boundary condition, Eq. (54): f* = B^T f*_C, node by node with the
// matrices above (Eqs. 59 and 60 for the D2Q9 inlet and outlet).
void adjoint_bc(const Problem& P, const double* fsC, const double* gsC, double* fs, double* gs) {
  const int Q = P.F.Q, Qg = P.G.Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    double B[19 * 19];
    bc_matrix(P, n, B);
    for (int j = 0; j < Q; ++j) {
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s += B[i * Q + j] * fsC[(size_t)n * Q + i];
      fs[(size_t)n * Q + j] = s;
    }
    if (!P.thermal) continue;
    double Bg[7 * 7];
    bc_matrix_thermal(P, n, Bg);
    for (int j = 0; j < Qg; ++j) {
      double s = 0.0;
      for (int i = 0; i < Qg; ++i) s += Bg[i * Qg + j] * gsC[(size_t)n * Qg + i];
      gs[(size_t)n * Qg + j] = s;
    }
  }
}

// Adjoint streaming, Eqs. (55) and (61): the transpose of the gather S,
// f*_S(src) = sum over the slots d with src(d) = src of f*(d).  Without
// symmetry planes and outflow this is f*_S,i(x) = f*_i(x + e_i), the reverse
// of the periodic permutation; the thermal outflow copy and the mirror
// images make some sources feed two slots or none.
void adjoint_stream(const Problem& P, const double* fs, const double* gs, double* fsS, double* gsS) {
  const size_t MF = (size_t)P.N * P.F.Q, MG = (size_t)P.N * P.G.Q;
  std::fill(fsS, fsS + MF, 0.0);
  for (size_t d = 0; d < MF; ++d) fsS[P.srcF[d]] += fs[d];
  if (!P.thermal) return;
  std::fill(gsS, gsS + MG, 0.0);
  for (size_t d = 0; d < MG; ++d) gsS[P.srcG[d]] += gs[d];
}

// ---------------------------------------------------------------------------
// Adjoint collision, Eqs. (56), (63)-(65):
//   f*_C,i = f*_S,i - (1/tau)[f*_S,i - sum_m (d feq_m / d f_i) f*_S,m]
//            + sum_m (d C^g_m / d f_i) g*_S,m - dJ/df_i
//   g*_C,i = g*_S,i - (1/tau_g)[g*_S,i - sum_m (d geq_m / d g_i) g*_S,m]
//            - beta(gamma) sum_m w^g_m g*_S,m - dJ/dg_i
// with, from Eq. (12) and rho = sum f, rho0 u = sum e f (Eq. 6),
//   d feq_m / d f_i = w_m [1 + 3 chi e_m.e_i + 9 chi^2 (e_m.u)(e_m.e_i) - 3 chi^2 u.e_i],
//   d C^g_m / d f_i = (1/tau_g) w^g_m T (e^g_m.e_i) / (cs2 rho0),
//   d geq_m / d g_i = w^g_m (1 + e^g_m.u / cs2).
// The double sums are evaluated literally.  Wall nodes: C = I.
// ---------------------------------------------------------------------------
void adjoint_collide(const Problem& P, const double* gamma, const double* f, const double* g,
                     const double* fsS, const double* gsS, const double* jf, const double* jg, double* fsC,
                     double* gsC) {
  const int Q = P.F.Q, Qg = P.G.Q;
  const Lattice &F = P.F, &G = P.G;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    const double* a = fsS + (size_t)n * Q;
    const double* b = P.thermal ? gsS + (size_t)n * Qg : nullptr;
    if (!P.collides(n)) {
      for (int i = 0; i < Q; ++i) fsC[(size_t)n * Q + i] = a[i] - jf[(size_t)n * Q + i];
      if (P.thermal)
        for (int i = 0; i < Qg; ++i) gsC[(size_t)n * Qg + i] = b[i] - jg[(size_t)n * Qg + i];
      continue;
    }
    double rho, u[3];
    moments(P, f + (size_t)n * Q, rho, u);
    const double chi = chi_of(P, n, gamma[n]);
    double T = 0.0, tg = 1.0;
    if (P.thermal) {
      for (int i = 0; i < Qg; ++i) T += g[(size_t)n * Qg + i];
      tg = tau_g(P, n, gamma[n]);
    }
    for (int i = 0; i < Q; ++i) {
      double s = 0.0;
      for (int m = 0; m < Q; ++m) {
        const double emei = F.e[m][0] * F.e[i][0] + F.e[m][1] * F.e[i][1] + F.e[m][2] * F.e[i][2];
        const double emu = F.e[m][0] * u[0] + F.e[m][1] * u[1] + F.e[m][2] * u[2];
        const double uei = u[0] * F.e[i][0] + u[1] * F.e[i][1] + u[2] * F.e[i][2];
        const double d = F.w[m] * (1.0 + 3.0 * chi * emei + 9.0 * chi * chi * emu * emei - 3.0 * chi * chi * uei);
        s += d * a[m];
      }
      double v = a[i] - (a[i] - s) / P.c.tau;
      if (P.thermal) {
        double c = 0.0;
        for (int m = 0; m < Qg; ++m) {
          const double egei = G.e[m][0] * F.e[i][0] + G.e[m][1] * F.e[i][1] + G.e[m][2] * F.e[i][2];
          c += (1.0 / tg) * G.w[m] * T * egei / (G.cs2 * P.c.rho0) * b[m];
        }
        v += c;
      }
      fsC[(size_t)n * Q + i] = v - jf[(size_t)n * Q + i];
    }
    if (P.thermal) {
      // heat source w_m beta (1 - T) of Eq. (71): d/dg_i = -w_m beta
      const double bq = beta_of(P, n, gamma[n]);
      double wb = 0.0;
      for (int m = 0; m < Qg; ++m) wb += G.w[m] * b[m];
      for (int i = 0; i < Qg; ++i) {
        double s = 0.0;
        for (int m = 0; m < Qg; ++m) {
          const double emu = G.e[m][0] * u[0] + G.e[m][1] * u[1] + G.e[m][2] * u[2];
          s += G.w[m] * (1.0 + emu / G.cs2) * b[m];
        }
        gsC[(size_t)n * Qg + i] = b[i] - (b[i] - s) / tg - bq * wb - jg[(size_t)n * Qg + i];
      }
    }
  }
}

// One adjoint step in the paper's order (Sec. 2.4, steps (2)-(4)).
void adjoint_step(const Problem& P, const double* gamma, const double* f, const double* g, const double* jf,
                  const double* jg, double* fsC, double* gsC, double* fsS, double* gsS, double* fs,
                  double* gs) {
  adjoint_bc(P, fsC, gsC, fs, gs);
  adjoint_stream(P, fs, gs, fsS, gsS);
  adjoint_collide(P, gamma, f, g, fsS, gsS, jf, jg, fsC, gsC);
}

// Residual quantity of the adjoint: mean over non-wall nodes of
// |sum_i e_i f*_S,i| (and of |sum_i g*_S,i|).
void adjoint_monitor(const Problem& P, const double* fsS, const double* gsS, double& If, double& Ig) {
  double sf = 0.0, sg = 0.0;
  for (int n = 0; n < P.N; ++n) {
    if (P.is_wall(n)) continue;
    double m[3] = {0, 0, 0};
    for (int i = 0; i < P.F.Q; ++i)
      for (int a = 0; a < 3; ++a) m[a] += P.F.e[i][a] * fsS[(size_t)n * P.F.Q + i];
    sf += std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    if (P.thermal) {
      double s = 0.0;
      for (int i = 0; i < P.G.Q; ++i) s += gsS[(size_t)n * P.G.Q + i];
      sg += std::fabs(s);
    }
  }
  If = sf / P.n_nonwall;
  Ig = sg / P.n_nonwall;
}

// Adjoint solve: f*_C = 0 (Eq. 53) or the given state when warm, then repeat
// B^T, S^T, C^T - dJ/df until the residual criterion or max_steps.
int adjoint(const Problem& P, const double* gamma, const double* f, const double* g, double* fsC, double* gsC,
            int max_steps, double tol, int check_every, int warm, int* steps_out, double* res_out) {
  const int Q = P.F.Q, Qg = P.G.Q;
  std::vector<double> jf((size_t)P.N * Q), jg(P.thermal ? (size_t)P.N * Qg : 1), jgam(P.N);
  objective_grad(P, gamma, f, g, jf.data(), jg.data(), jgam.data());
  if (!warm) {
    std::fill(fsC, fsC + (size_t)P.N * Q, 0.0);
    if (P.thermal) std::fill(gsC, gsC + (size_t)P.N * Qg, 0.0);
  }
  std::vector<double> fsS((size_t)P.N * Q), gsS(P.thermal ? (size_t)P.N * Qg : 1);
  std::vector<double> fs((size_t)P.N * Q), gs(P.thermal ? (size_t)P.N * Qg : 1);
  double prevF = 0, prevG = 0, resF = 0, resG = 0;
  bool have_prev = false;
  int status = 1, k = 0;
  for (k = 1; k <= max_steps; ++k) {
    adjoint_step(P, gamma, f, g, jf.data(), jg.data(), fsC, gsC, fsS.data(), gsS.data(), fs.data(), gs.data());
    if (check_every > 0 && k % check_every == 0) {
      double If, Ig;
      adjoint_monitor(P, fsS.data(), gsS.data(), If, Ig);
      if (!std::isfinite(If) || !std::isfinite(Ig)) {
        status = -1;
        break;
      }
      if (have_prev) {
        resF = std::fabs(If - prevF) / std::max(std::fabs(If), 1e-300);
        resG = std::fabs(Ig - prevG) / std::max(std::fabs(Ig), 1e-300);
        if (rel_converged(If, prevF, tol) && (!P.thermal || rel_converged(Ig, prevG, tol))) {
          status = 0;
          break;
        }
      }
      prevF = If;
      prevG = Ig;
      have_prev = true;
    }
  }
  if (steps_out) *steps_out = std::min(k, max_steps);
  if (res_out) {
    res_out[0] = resF;
    res_out[1] = resG;
  }
  return status;
}

// ---------------------------------------------------------------------------
// Continuous adjoint variant (Sec. 2.3): the adjoint equation discretised as in
// Eq. (30), stepped in the order adjoint collision -> adjoint streaming ->
// adjoint boundary condition, starting from f* = 0 (Eq. 24).  Collision and
// streaming are the operators of the discrete adjoint above; the boundary
// step is the one obtained from the boundary integral of Eq. (21):
//   walls: bounce back (the adjoint of bounce back);
//   ports: for every direction j leaving the domain through the port
//          (e_j . n < 0, n the inward normal) the coefficient of delta f_j in
//          sum_i (e_i . n_out) f*_i delta f_i + dJ, with the unknown
//          delta f_k (e_k . n > 0) expressed through the boundary scheme,
//          delta f_k = sum_j B_kj delta f_j, must vanish (Eqs. 25-26, 28):
//            f*_j = sum_{k unknown} B_kj f*_k - sum_i B_ij dJ/df_i ,
//          the other directions keep their streamed values.  The coefficients
//          of the other delta f_j cannot be made zero as well; that is the
//          inconsistency Sec. 2.3 points out.  For the D2Q9 outlet on the
//          bottom wall and inlet on the left wall this is Eqs. (27) and (29).
// The objective enters here only through its boundary part (the inlet
// pressure of the pressure-drop objective, Eq. 22); a volume objective
// (dissipation) stays a source in the collision.  Flow lattice only.
// ---------------------------------------------------------------------------
void cont_adjoint_bc(const Problem& P, const double* jfb, const double* fsS, double* fsB) {
  const Lattice& L = P.F;
  const int Q = L.Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    const double* a = fsS + (size_t)n * Q;
    double* out = fsB + (size_t)n * Q;
    const int k = P.kind[n];
    if (k == K_WALL || k == K_HEATED) {
      for (int i = 0; i < Q; ++i) out[i] = a[L.opp[i]];
      continue;
    }
    for (int i = 0; i < Q; ++i) out[i] = a[i];
    if (k != K_INLET && k != K_OUTLET) continue;
    double B[19 * 19];
    bc_matrix(P, n, B);
    const int* nv = NORMAL_VEC[P.ncode[n]];
    for (int j = 0; j < Q; ++j) {
      if (dir_class(L, j, nv) != -1) continue;
      double v = 0.0;
      for (int kk = 0; kk < Q; ++kk)
        if (dir_class(L, kk, nv) == 1) v += B[kk * Q + j] * a[kk];
      for (int i = 0; i < Q; ++i) v -= B[i * Q + j] * jfb[(size_t)n * Q + i];
      out[j] = v;
    }
  }
}

// Split dJ/df into its boundary part (handled by the boundary step of the
// continuous adjoint) and its volume part (a collision source).
void cont_split_objective(const Problem& P, const double* jf, double* jfb, double* jfv) {
  const size_t M = (size_t)P.N * P.F.Q;
  const bool boundary = P.c.objective == OBJ_PRESSURE_DROP;
  for (size_t i = 0; i < M; ++i) {
    jfb[i] = boundary ? jf[i] : 0.0;
    jfv[i] = boundary ? 0.0 : jf[i];
  }
}

// One continuous adjoint step: y = C^T f*_B - (volume source), then
// f*_S = S^T y (returned for the residual), f*_B = boundary step of f*_S.
void cont_adjoint_step(const Problem& P, const double* gamma, const double* f, const double* jfb,
                       const double* jfv, double* fsB, double* y, double* fsS) {
  adjoint_collide(P, gamma, f, nullptr, fsB, nullptr, jfv, nullptr, y, nullptr);
  adjoint_stream(P, y, nullptr, fsS, nullptr);
  cont_adjoint_bc(P, jfb, fsS, fsB);
}

// Continuous adjoint solve from f*_B = 0 (or the given state when warm), with
// the residual of the discrete solve taken on the streamed values.
int cont_adjoint(const Problem& P, const double* gamma, const double* f, double* fsB, int max_steps,
                 double tol, int check_every, int warm, int* steps_out, double* res_out) {
  const int Q = P.F.Q;
  const size_t M = (size_t)P.N * Q;
  std::vector<double> jf(M), jg(1), jgam(P.N), jfb(M), jfv(M), y(M), fsS(M);
  objective_grad(P, gamma, f, nullptr, jf.data(), jg.data(), jgam.data());
  cont_split_objective(P, jf.data(), jfb.data(), jfv.data());
  if (!warm) std::fill(fsB, fsB + M, 0.0);
  double prev = 0, res = 0;
  bool have_prev = false;
  int status = 1, k = 0;
  for (k = 1; k <= max_steps; ++k) {
    cont_adjoint_step(P, gamma, f, jfb.data(), jfv.data(), fsB, y.data(), fsS.data());
    if (check_every > 0 && k % check_every == 0) {
      double If, Ig;
      adjoint_monitor(P, fsS.data(), nullptr, If, Ig);
      if (!std::isfinite(If)) {
        status = -1;
        break;
      }
      if (have_prev) {
        res = std::fabs(If - prev) / std::max(std::fabs(If), 1e-300);
        if (rel_converged(If, prev, tol)) {
          status = 0;
          break;
        }
      }
      prev = If;
      have_prev = true;
    }
  }
  if (steps_out) *steps_out = std::min(k, max_steps);
  if (res_out) {
    res_out[0] = res;
    res_out[1] = 0.0;
  }
  return status;
}

// ---------------------------------------------------------------------------
// Sensitivity contraction of Eq. (66) (first equality), with the exact
// derivative of the collision with respect to the design variable:
//   sum_i f*_S,i dC_i/dgamma + sum_i g*_S,i dC^g_i/dgamma, where
//   dC_i/dgamma   = (1/tau) w_i rho0 [3 e_i.u + 9 chi (e_i.u)^2 - 3 chi |u|^2] chi'(gamma)
//   dC^g_i/dgamma = (g_i - geq_i) tau_g'(gamma) / tau_g^2 + w^g_i beta'(gamma) (1 - T)
// (the bracket printed in Eq. (66) is the secant feq(u) - feq(0); the exact
// derivative is used so that the result is the gradient of the discrete J).
// Non-design nodes give 0.
// ---------------------------------------------------------------------------
void sens_contract(const Problem& P, const double* gamma, const double* f, const double* g, const double* fsS,
                   const double* gsS, double* out) {
  const int Q = P.F.Q, Qg = P.G.Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < P.N; ++n) {
    out[n] = 0.0;
    if (!P.is_design(n)) continue;
    double rho, u[3];
    moments(P, f + (size_t)n * Q, rho, u);
    const double chi = chi_of(P, n, gamma[n]);
    const double dchi = chi_d(P, n, gamma[n]);
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double s = 0.0;
    for (int i = 0; i < Q; ++i) {
      const double eu = P.F.e[i][0] * u[0] + P.F.e[i][1] * u[1] + P.F.e[i][2] * u[2];
      const double dC = (1.0 / P.c.tau) * P.F.w[i] * P.c.rho0 * (3.0 * eu + 9.0 * chi * eu * eu - 3.0 * chi * uu) * dchi;
      s += fsS[(size_t)n * Q + i] * dC;
    }
    if (P.thermal) {
      double T = 0.0;
      for (int i = 0; i < Qg; ++i) T += g[(size_t)n * Qg + i];
      const double tg = tau_g(P, n, gamma[n]);
      const double dtg = tau_g_d(P, n, gamma[n]);
      const double db = beta_d(P, n);
      for (int i = 0; i < Qg; ++i) {
        const double eu = P.G.e[i][0] * u[0] + P.G.e[i][1] * u[1] + P.G.e[i][2] * u[2];
        const double geq = P.G.w[i] * T * (1.0 + eu / P.G.cs2);
        const double dC = (g[(size_t)n * Qg + i] - geq) * dtg / (tg * tg) + P.G.w[i] * db * (1.0 - T);
        s += gsS[(size_t)n * Qg + i] * dC;
      }
    }
    out[n] = s;
  }
}

// ---------------------------------------------------------------------------
// Geometry set-up from the mask: node kinds, port normals, inlet profile and
// the objective layer.  The inlet profile is the product of parabolas
// 4 s (1 - s) over the tangential axes of the inlet set, s measured from the
// midway wall just outside the set; an axis the inlet set spans entirely is
// uniform.  The peak speed follows from Re = U L / nu with nu from Eq. (3).
// ---------------------------------------------------------------------------
bool build_problem(const OrcConfig& c, const uint8_t* mask, Problem& P, std::string& err) {
  P.c = c;
  P.nx = c.nx;
  P.ny = c.ny;
  P.nz = c.nz;
  P.N = c.nx * c.ny * c.nz;
  if (c.dim == 2) {
    if (c.nz != 1) {
      err = "2D problems need nz == 1";
      return false;
    }
    P.F = make_d2q9();
  } else if (c.dim == 3) {
    P.F = make_d3q19();
  } else {
    err = "dim must be 2 or 3";
    return false;
  }
  P.thermal = c.thermal != 0;
  P.G = (c.dim == 2) ? make_d2q5() : make_d3q7();
  P.nu = (c.tau - 0.5) / 3.0;
  P.U_peak = (c.L_ref > 0) ? c.Re * P.nu / c.L_ref : 0.0;
  P.Df = (c.Pr > 0) ? P.nu / c.Pr : 0.0;
  P.kind.assign(P.N, 0);
  P.ncode.assign(P.N, 0);
  P.u_in.assign(P.N, 0.0);
  P.layer.assign(P.N, 0);
  for (int n = 0; n < P.N; ++n) {
    const int k = mask[n] & 7, nc = (mask[n] >> 3) & 7;
    if (k > K_SYM || (mask[n] >> 6) != 0) {
      err = "bad mask byte";
      return false;
    }
    P.kind[n] = k;
    P.ncode[n] = (k == K_INLET || k == K_OUTLET || k == K_HEATED) ? nc : 0;
    if (P.ncode[n] > 5 || (c.dim == 2 && P.ncode[n] > 3)) {
      err = "bad normal code";
      return false;
    }
  }
  // symmetry planes: layer n_a - 1 of a symmetric axis holds SYM nodes only,
  // and SYM nodes appear nowhere else
  const int lim[3] = {P.nx, P.ny, P.nz};
  for (int a = 0; a < 3; ++a) {
    if (c.symmetric[a] != 0 && c.symmetric[a] != 1) {
      err = "symmetric must be 0 or 1";
      return false;
    }
    if (c.symmetric[a] && (lim[a] < 4 || (c.dim == 2 && a == 2))) {
      err = "a symmetric axis needs at least 4 layers";
      return false;
    }
  }
  for (int n = 0; n < P.N; ++n) {
    int x[3];
    P.coords(n, x[0], x[1], x[2]);
    bool on = false;
    for (int a = 0; a < 3; ++a) on = on || (c.symmetric[a] && x[a] == lim[a] - 1);
    if (on != (P.kind[n] == K_SYM)) {
      err = "SYM nodes must fill exactly the last layer of each symmetric axis";
      return false;
    }
    // a port sits on the face its inward normal points away from; a heated
    // wall's inward neighbour lies inside the box
    const int k = P.kind[n], nc = P.ncode[n], ax = nc / 2, sgn = (nc % 2 == 0) ? 1 : -1;
    if ((k == K_INLET || k == K_OUTLET) && x[ax] != (sgn > 0 ? 0 : lim[ax] - 1)) {
      err = "port normal is not the inward normal of its face";
      return false;
    }
    if (k == K_HEATED && (x[ax] + sgn < 0 || x[ax] + sgn >= lim[ax])) {
      err = "heated wall normal points out of the box";
      return false;
    }
  }
  if (c.beta_max < 0.0 || (c.beta_max > 0.0 && !c.thermal)) {
    err = "beta_max must be >= 0 and needs the thermal lattice";
    return false;
  }
  if (c.objective == OBJ_HEATGEN && (!c.thermal || c.beta_max <= 0.0)) {
    err = "heat-generation objective needs the thermal lattice and beta_max > 0";
    return false;
  }
  if (c.inlet_rho < 0.0) {
    err = "inlet_rho must be >= 0";
    return false;
  }
  // inlet profile, per normal code
  for (int code = 0; code < 6; ++code) {
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    bool any = false;
    for (int n = 0; n < P.N; ++n) {
      if (P.kind[n] != K_INLET || P.ncode[n] != code) continue;
      any = true;
      int x[3];
      P.coords(n, x[0], x[1], x[2]);
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], x[a]);
        hi[a] = std::max(hi[a], x[a]);
      }
    }
    if (!any) continue;
    const int* nv = NORMAL_VEC[code];
    for (int n = 0; n < P.N; ++n) {
      if (P.kind[n] != K_INLET || P.ncode[n] != code) continue;
      int x[3];
      P.coords(n, x[0], x[1], x[2]);
      double prof = 1.0;
      for (int a = 0; a < c.dim; ++a) {
        if (nv[a] != 0) continue;
        if (lo[a] == 0 && hi[a] == lim[a] - 1) continue;
        // an inlet set reaching a symmetry plane continues in its mirror image
        const int h = (c.symmetric[a] && hi[a] == lim[a] - 2) ? 2 * lim[a] - 3 - lo[a] : hi[a];
        const double s = (x[a] - lo[a] + 0.5) / double(h - lo[a] + 1);
        prof *= 4.0 * s * (1.0 - s);
      }
      P.u_in[n] = P.U_peak * prof;
    }
  }
  for (int n = 0; n < P.N; ++n) {
    if (P.kind[n] == K_INLET) ++P.n_inlet;
    if (!P.is_wall(n)) ++P.n_nonwall;
    if (P.kind[n] == K_HEATED) {
      int x[3];
      P.coords(n, x[0], x[1], x[2]);
      const int* nv = NORMAL_VEC[P.ncode[n]];
      int y[3];
      bool inside = true;
      for (int a = 0; a < 3; ++a) {
        y[a] = x[a] + nv[a];
        if (y[a] < 0 || y[a] >= lim[a]) inside = false;
      }
      if (inside) {
        const int m = P.idx(y[0], y[1], y[2]);
        if (!P.is_wall(m)) P.layer[m] = 1;
      }
    }
  }
  for (int n = 0; n < P.N; ++n) P.n_layer += P.layer[n];
  // streaming gather maps
  P.srcF.resize((size_t)P.N * P.F.Q);
  for (int n = 0; n < P.N; ++n)
    for (int i = 0; i < P.F.Q; ++i) P.srcF[(size_t)n * P.F.Q + i] = stream_source(P, P.F, false, n, i);
  if (P.thermal) {
    P.srcG.resize((size_t)P.N * P.G.Q);
    for (int n = 0; n < P.N; ++n)
      for (int i = 0; i < P.G.Q; ++i) P.srcG[(size_t)n * P.G.Q + i] = stream_source(P, P.G, true, n, i);
  }
  if ((c.objective == OBJ_PRESSURE_DROP || c.objective == OBJ_HEATSINK) && c.w_dp != 0.0 && P.n_inlet == 0) {
    err = "pressure-drop term needs inlet nodes";
    return false;
  }
  if (c.objective == OBJ_HEATSINK && (!P.thermal || P.n_layer == 0)) {
    err = "heat-sink objective needs the thermal lattice and heated walls";
    return false;
  }
  if (P.n_nonwall == 0) {
    err = "no non-wall nodes";
    return false;
  }
  return true;
}

thread_local std::string g_err;

}  // namespace

// ===========================================================================
// C interface for the Python test harness.  Suffix _d: double, _z: complex
// (interleaved re/im pairs).  All arrays are node-major.
// ===========================================================================
extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

// Threads of the OpenMP loops started from the calling thread (the harness
// runs independent small solves in parallel host threads with 1 each).
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void* orc_create(const OrcConfig* c, const uint8_t* mask) {
  Problem* P = new Problem();
  if (!build_problem(*c, mask, *P, g_err)) {
    delete P;
    return nullptr;
  }
  return P;
}

void orc_destroy(void* h) { delete static_cast<Problem*>(h); }

// out: N, Q, Qg, n_inlet, n_layer, n_nonwall
void orc_sizes(void* h, int32_t* out) {
  const Problem& P = *static_cast<Problem*>(h);
  out[0] = P.N;
  out[1] = P.F.Q;
  out[2] = P.thermal ? P.G.Q : 0;
  out[3] = P.n_inlet;
  out[4] = P.n_layer;
  out[5] = P.n_nonwall;
}

// which 0: flow lattice, 1: thermal lattice.  e: Q*3 ints, w: Q doubles.
void orc_lattice(void* h, int which, int32_t* e, double* w) {
  const Problem& P = *static_cast<Problem*>(h);
  const Lattice& L = which ? P.G : P.F;
  for (int i = 0; i < L.Q; ++i) {
    for (int a = 0; a < 3; ++a) e[i * 3 + a] = L.e[i][a];
    w[i] = L.w[i];
  }
}

void orc_geometry(void* h, double* u_in, uint8_t* layer) {
  const Problem& P = *static_cast<Problem*>(h);
  for (int n = 0; n < P.N; ++n) {
    u_in[n] = P.u_in[n];
    layer[n] = (uint8_t)P.layer[n];
  }
}

void orc_init_d(void* h, double* f, double* g) { init_state(*static_cast<Problem*>(h), f, g); }
void orc_init_z(void* h, cplx* f, cplx* g) { init_state(*static_cast<Problem*>(h), f, g); }

void orc_collide_d(void* h, const double* gam, double* f, double* g) { collide(*static_cast<Problem*>(h), gam, f, g); }
void orc_collide_z(void* h, const cplx* gam, cplx* f, cplx* g) { collide(*static_cast<Problem*>(h), gam, f, g); }

void orc_stream_d(void* h, const double* fC, const double* gC, double* fS, double* gS) {
  stream(*static_cast<Problem*>(h), fC, gC, fS, gS);
}
void orc_stream_z(void* h, const cplx* fC, const cplx* gC, cplx* fS, cplx* gS) {
  stream(*static_cast<Problem*>(h), fC, gC, fS, gS);
}

void orc_boundary_d(void* h, double* f, double* g) { boundary(*static_cast<Problem*>(h), f, g); }
void orc_boundary_z(void* h, cplx* f, cplx* g) { boundary(*static_cast<Problem*>(h), f, g); }

int orc_forward_d(void* h, const double* gam, double* f, double* g, int max_steps, double tol, int check_every,
                  int warm, int32_t* steps, double* res) {
  return forward(*static_cast<Problem*>(h), gam, f, g, max_steps, tol, check_every, warm, steps, res);
}
int orc_forward_z(void* h, const cplx* gam, cplx* f, cplx* g, int max_steps, double tol, int check_every, int warm,
                  int32_t* steps, double* res) {
  return forward(*static_cast<Problem*>(h), gam, f, g, max_steps, tol, check_every, warm, steps, res);
}

// rho[N], u[3N] (node-major xyz), T[N]
void orc_macro_d(void* h, const double* f, const double* g, double* rho, double* u, double* T) {
  const Problem& P = *static_cast<Problem*>(h);
  for (int n = 0; n < P.N; ++n) {
    moments(P, f + (size_t)n * P.F.Q, rho[n], u + (size_t)n * 3);
    if (P.thermal && T) {
      double s = 0.0;
      for (int i = 0; i < P.G.Q; ++i) s += g[(size_t)n * P.G.Q + i];
      T[n] = s;
    }
  }
}

void orc_objective_d(void* h, const double* gam, const double* f, const double* g, double* J) {
  *J = objective(*static_cast<Problem*>(h), gam, f, g);
}
void orc_objective_z(void* h, const cplx* gam, const cplx* f, const cplx* g, cplx* J) {
  *J = objective(*static_cast<Problem*>(h), gam, f, g);
}

void orc_objective_grad_d(void* h, const double* gam, const double* f, const double* g, double* jf, double* jg,
                          double* jgam) {
  objective_grad(*static_cast<Problem*>(h), gam, f, g, jf, jg, jgam);
}

void orc_bc_matrix(void* h, int node, double* B) { bc_matrix(*static_cast<Problem*>(h), node, B); }
void orc_bc_matrix_thermal(void* h, int node, double* B) { bc_matrix_thermal(*static_cast<Problem*>(h), node, B); }

void orc_adjoint_bc_d(void* h, const double* fsC, const double* gsC, double* fs, double* gs) {
  adjoint_bc(*static_cast<Problem*>(h), fsC, gsC, fs, gs);
}
void orc_adjoint_stream_d(void* h, const double* fs, const double* gs, double* fsS, double* gsS) {
  adjoint_stream(*static_cast<Problem*>(h), fs, gs, fsS, gsS);
}
void orc_adjoint_collide_d(void* h, const double* gam, const double* f, const double* g, const double* fsS,
                           const double* gsS, const double* jf, const double* jg, double* fsC, double* gsC) {
  adjoint_collide(*static_cast<Problem*>(h), gam, f, g, fsS, gsS, jf, jg, fsC, gsC);
}

int orc_adjoint_d(void* h, const double* gam, const double* f, const double* g, double* fsC, double* gsC,
                  int max_steps, double tol, int check_every, int warm, int32_t* steps, double* res) {
  return adjoint(*static_cast<Problem*>(h), gam, f, g, fsC, gsC, max_steps, tol, check_every, warm, steps, res);
}

void orc_adjoint_monitor_d(void* h, const double* fsS, const double* gsS, double* out) {
  adjoint_monitor(*static_cast<Problem*>(h), fsS, gsS, out[0], out[1]);
}
void orc_forward_monitor_d(void* h, const double* f, const double* g, double* out) {
  forward_monitor(*static_cast<Problem*>(h), f, g, out[0], out[1]);
}

void orc_sens_contract_d(void* h, const double* gam, const double* f, const double* g, const double* fsS,
                         const double* gsS, double* out) {
  sens_contract(*static_cast<Problem*>(h), gam, f, g, fsS, gsS, out);
}

// dJ/dgamma = explicit dJ/dgamma - sum_i f*_S,i dC_i/dgamma (Eq. 66), from the
// adjoint state f*_C, with f*_S = S^T B^T f*_C.
void orc_sensitivity_d(void* h, const double* gam, const double* f, const double* g, const double* fsC,
                       const double* gsC, double* dJ) {
  const Problem& P = *static_cast<Problem*>(h);
  const int Q = P.F.Q, Qg = P.G.Q;
  std::vector<double> fs((size_t)P.N * Q), gs(P.thermal ? (size_t)P.N * Qg : 1);
  std::vector<double> fsS((size_t)P.N * Q), gsS(P.thermal ? (size_t)P.N * Qg : 1);
  adjoint_bc(P, fsC, gsC, fs.data(), gs.data());
  adjoint_stream(P, fs.data(), gs.data(), fsS.data(), gsS.data());
  std::vector<double> jf((size_t)P.N * Q), jg(P.thermal ? (size_t)P.N * Qg : 1), jgam(P.N), c(P.N);
  objective_grad(P, gam, f, g, jf.data(), jg.data(), jgam.data());
  sens_contract(P, gam, f, g, fsS.data(), gsS.data(), c.data());
  for (int n = 0; n < P.N; ++n) dJ[n] = P.is_design(n) ? jgam[n] - c[n] : 0.0;
}

void orc_cont_adjoint_bc_d(void* h, const double* jfb, const double* fsS, double* fsB) {
  cont_adjoint_bc(*static_cast<Problem*>(h), jfb, fsS, fsB);
}

int orc_cont_adjoint_d(void* h, const double* gam, const double* f, double* fsB, int max_steps, double tol,
                       int check_every, int warm, int32_t* steps, double* res) {
  const Problem& P = *static_cast<Problem*>(h);
  if (P.thermal) {
    g_err = "continuous adjoint: flow lattice only";
    return -2;
  }
  return cont_adjoint(P, gam, f, fsB, max_steps, tol, check_every, warm, steps, res);
}

// Continuous sensitivity, Eq. (32) with the exact derivative of Eq. (12) (as
// in Eq. 66): explicit dJ/dgamma - sum_i f*_i dC_i/dgamma with f* the adjoint
// state after the boundary step (equal to the streamed values at the design
// nodes, which are interior).
void orc_cont_sensitivity_d(void* h, const double* gam, const double* f, const double* fsB, double* dJ) {
  const Problem& P = *static_cast<Problem*>(h);
  const int Q = P.F.Q;
  std::vector<double> jf((size_t)P.N * Q), jg(1), jgam(P.N), c(P.N);
  objective_grad(P, gam, f, nullptr, jf.data(), jg.data(), jgam.data());
  sens_contract(P, gam, f, nullptr, fsB, nullptr, c.data());
  for (int n = 0; n < P.N; ++n) dJ[n] = P.is_design(n) ? jgam[n] - c[n] : 0.0;
}

}  // extern "C"
