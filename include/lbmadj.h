/*
 * lbmadj.h -- C ABI of the MI355X (gfx950) library for the steady discrete
 * adjoint lattice Boltzmann method of Luo, Chen, Yaji and Tao, "Improved
 * adjoint lattice Boltzmann method for topology optimization of laminar
 * convective heat transfer" (arXiv 2501.02161).
 *
 * One problem = one lattice: a D3Q19 BGK flow lattice with the incompressible
 * equilibrium of Eq. (4), extended by the design field as in Eq. (12), and
 * optionally a coupled D3Q7 BGK advection-diffusion lattice for temperature
 * (Eq. 71, with the volumetric source of Eq. 69 when beta_max > 0).  A grid
 * with nz == 1 is a 2D problem on the D2Q9 lattice of Eq. (5), for which
 * Eqs. (7), (8) and (58)-(60) are the printed special cases of the generic
 * port rules, with a D2Q5 thermal lattice (rest 1/2, axes 1/8, cs2 = 1/4 as
 * on D3Q7) when thermal.  Three calls make the hot path:
 *
 *   lbm_forward_solve   the steady forward sweep: collision (Eq. 36),
 *                       streaming (Eq. 37), boundary conditions (Eqs. 7-9)
 *                       repeated until the residual criterion of Sec. 3.1;
 *   lbm_adjoint_solve   the steady discrete adjoint sweep (Sec. 2.4, Eqs.
 *                       53-56): adjoint boundary condition (Eqs. 54, 59, 60),
 *                       reversed streaming (Eq. 61), adjoint collision minus
 *                       the objective derivative (Eq. 65);
 *   lbm_sensitivity     dJ/dgamma per node (Eq. 66, first equality, with the
 *                       exact derivative of the collision).
 *
 * Units and conventions
 *   Lattice units (dx = dt = 1).  Node n = x + nx*(y + ny*z); every field is
 *   a contiguous FP32 array [z][y][x] (x fastest) of N = nx*ny*nz entries;
 *   vector fields are [3][z][y][x] (component-major).
 *   Design field gamma in [0,1] (1 fluid, 0 solid): Brinkman inverse
 *   permeability a_B = alpha_max q (1-gamma)/(q+gamma); the equilibrium of
 *   Eq. (12) uses chi u with chi = 1 - tau a_B (a velocity-shift forcing that
 *   removes a_B rho0 u of momentum per step).  Thermal relaxation time
 *   tau_g = 1/2 + 4 (nu/Pr) k(gamma), k = r + (1-r) gamma/(1 + q_r (1-gamma))
 *   (RAMP, r = k_ratio).  Non-design nodes use chi = 1 and k = 1.
 *   The peak inlet speed is U = Re nu / L_ref, nu = (tau - 1/2)/3 (Eq. 3); the
 *   inlet profile is a product of parabolas over the inlet set's extent in
 *   each tangential axis (uniform along an axis the set spans entirely).
 *
 * Memory and ownership
 *   Device pointers are caller-owned (e.g. torch tensors) and must stay valid
 *   for the call; the library never frees them.  Its only device memory is the
 *   workspace the caller binds (lbm_workspace_bytes / lbm_bind_workspace),
 *   which holds the A/B population buffers, node flags and reduction scratch.
 *   Host pointers (desc, mask, info, J) are read/written during the call only.
 *   All device work is enqueued on the HIP stream `stream` (NULL = default
 *   stream); calls that return host values (info, J) synchronise that stream.
 *   One problem handle must be used by one host thread at a time.
 *
 * Errors
 *   0 LBM_OK; +1 LBM_NOT_CONVERGED (max_steps reached: the outputs are still
 *   written).  Negative values are errors, with a message from
 *   lbm_last_error() (thread-local): LBM_EINVAL (null pointer, bad size or
 *   parameter, bad mask), LBM_ESTATE (no workspace bound, adjoint before a
 *   forward solve, sensitivity before an adjoint solve), LBM_EDEVICE (a HIP
 *   call failed), LBM_EDIVERGED (the residual monitor became non-finite).
 *   No C++ exception crosses this interface.
 */
#ifndef LBMADJ_H
#define LBMADJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_NOT_CONVERGED 1
#define LBM_EINVAL (-1)
#define LBM_ESTATE (-2)
#define LBM_ENOMEM (-3)
#define LBM_EDEVICE (-4)
#define LBM_EDIVERGED (-5)

/* Mask byte, one per node (host array of N bytes, [z][y][x]).
 * bits 0-2: node kind; bits 3-5: inward normal for INLET, OUTLET and HEATED
 * nodes (the direction pointing into the domain); bits 6-7: zero.
 *   DESIGN  interior node whose chi and k follow gamma
 *   FLUID   interior node with chi = 1, k = 1 (not designable)
 *   INLET   Zou-He velocity inlet (Eq. 7 generalised to any axis normal and
 *           to D3Q19), or a pressure inlet at desc.inlet_rho (the outlet
 *           rule at that density); thermal Dirichlet T = T_in
 *   OUTLET  Zou-He pressure outlet rho = rho0 (Eq. 8 generalised); thermal
 *           zero-gradient outflow
 *   WALL    full-way bounce-back (Eq. 9): every pair is swapped, no
 *           collision; adiabatic for the thermal lattice
 *   HEATED  a WALL that adds the heat flux q_w per step to the thermal
 *           population along its inward normal
 *   SYM     the layer beyond a mirror plane (desc.symmetric): never read;
 *           a pull that would reach it reads the mirror image instead (the
 *           node's own layer along that axis, the direction reflected in it)
 * On every non-periodic axis the two outer layers must be WALL, HEATED,
 * INLET, OUTLET or SYM nodes; SYM nodes fill exactly the last layer of each
 * symmetric axis; a port's normal must be the inward normal of its face and
 * ports may not sit on an edge of two non-periodic faces. */
#define LBM_NODE_DESIGN 0
#define LBM_NODE_FLUID 1
#define LBM_NODE_INLET 2
#define LBM_NODE_OUTLET 3
#define LBM_NODE_WALL 4
#define LBM_NODE_HEATED 5
#define LBM_NODE_SYM 6
#define LBM_NORMAL_PX 0
#define LBM_NORMAL_MX 1
#define LBM_NORMAL_PY 2
#define LBM_NORMAL_MY 3
#define LBM_NORMAL_PZ 4
#define LBM_NORMAL_MZ 5

/* Objectives, evaluated on the post-boundary state (the moments of Eq. 6).
 *   PRESSURE_DROP  J = w_dp (mean over inlet nodes of rho/3 - rho0/3): the
 *                  paper's J = p_in of Eq. (34) minus the fixed outlet pressure.
 *   DISSIPATION    J = sum over axis edges between non-wall nodes (no
 *                  wrap-around) of rho0 nu |u(x+e) - u(x)|^2
 *                  + sum over design nodes of a_B(gamma) rho0 |u|^2.
 *   HEATSINK       J = mean T over the node layer next to the HEATED walls
 *                  (x + normal of each HEATED node) + w_dp (mean inlet rho/3
 *                  - rho0/3); needs the thermal lattice. */
#define LBM_OBJ_PRESSURE_DROP 0
#define LBM_OBJ_DISSIPATION 1
#define LBM_OBJ_HEATSINK 2
/*   HEATGEN        J = - sum over design nodes of beta(gamma) (1 - T), the
 *                  heat generated in the solid (Eq. 72 with Eqs. 69, 71);
 *                  needs the thermal lattice and beta_max > 0. */
#define LBM_OBJ_HEATGEN 3

/* Adjoint kinds (lbm_desc_t.adjoint_kind).
 *   DISCRETE    the fully consistent discrete adjoint of Sec. 2.4 (Eqs. 53-65).
 *   CONTINUOUS  the continuous adjoint of Sec. 2.3 discretised as Eq. (30):
 *               same collision and streaming, stepped collision -> streaming
 *               -> boundary, with the boundary step of Eqs. (25)-(29)
 *               generalised to any axis normal (every direction leaving the
 *               domain at a port: f*_j = f*_jbar - 12 sum_{e_k.n>0} w_k f*_k
 *               at an outlet, f*_j = f*_jbar - 2 dJ/drho at an inlet); the
 *               inlet-pressure objective enters through that step.  Kept for
 *               comparison: its boundary step cannot satisfy all of Eq. (25),
 *               its dJ/dgamma is not the gradient and it loses stability at
 *               lower Re.  Flow lattice only (LBM_EINVAL with thermal). */
#define LBM_ADJOINT_DISCRETE 0
#define LBM_ADJOINT_CONTINUOUS 1

typedef struct lbm_desc {
  int32_t nx, ny, nz;      /* grid: nx, ny >= 3; nz >= 3 (D3Q19) or nz == 1   */
                           /* (2D: D2Q9 + D2Q5, z not symmetric and its      */
                           /* periodic flag ignored, normals in x or y)      */
  int32_t thermal;         /* 0: flow only; 1: coupled D3Q7 temperature       */
  int32_t periodic[3];     /* 1: periodic streaming along x / y / z           */
  int32_t objective;       /* LBM_OBJ_*                                       */
  double tau;              /* flow relaxation time, > 1/2                     */
  double rho0;             /* reference density of the incompressible model  */
  double Re;               /* Reynolds number U L_ref / nu (sets inlet speed) */
  double L_ref;            /* length of Re, > 0 when there are inlets         */
  double alpha_max, q_brink; /* Brinkman interpolation a_B(gamma)             */
  double Pr;               /* Prandtl number: fluid diffusivity nu/Pr         */
  double k_ratio, q_ramp;  /* solid/fluid conductivity ratio, RAMP parameter  */
  double q_w;              /* heat flux per HEATED node and step              */
  double T_in;             /* inlet temperature                               */
  double w_dp;             /* weight of the pressure-drop term                */
  int32_t max_steps;       /* step cap of each solve, >= 1                    */
  int32_t check_every;     /* steps between residual checks (0: never)        */
  double tol;              /* residual tolerance (0: run max_steps)           */
  int32_t adjoint_kind;    /* LBM_ADJOINT_DISCRETE or LBM_ADJOINT_CONTINUOUS  */
  int32_t symmetric[3];    /* 1: mirror plane between layers n-2 and n-1 of  */
                           /* the axis; layer n-1 holds LBM_NODE_SYM nodes    */
  double inlet_rho;        /* > 0: every inlet is a pressure inlet at this    */
                           /* density (Re, L_ref then unused); 0: velocity    */
  double beta_max;         /* heat generation beta(gamma) (1 - T) per step,   */
                           /* beta = beta_max (1 - gamma) on design nodes     */
} lbm_desc_t;

/* Result of a solve.  Residuals follow Sec. 3.1: |I(t) - I(t - c)| / |I(t)|
 * with c = check_every; forward I = (mean |u|, mean T) over non-wall nodes,
 * adjoint I = (mean |sum_i e_i f*_S,i|, mean |sum_i g*_S,i|).  The solve has
 * converged when both are <= tol at a check (never when tol == 0). */
typedef struct lbm_info {
  int32_t steps;           /* steps taken                                     */
  int32_t status;          /* LBM_OK or LBM_NOT_CONVERGED                     */
  double residual[2];      /* last residuals (flow, thermal)                  */
  double monitor[2];       /* last monitored quantities I                     */
  double J;                /* forward: objective; adjoint/sensitivity: copy   */
} lbm_info_t;

typedef struct lbm_problem lbm_problem_t;

/* Validate desc and the host mask (N bytes) and create a handle.  Nothing is
 * allocated on the device.  Returns LBM_EINVAL on a bad descriptor/mask. */
int lbm_problem_create(const lbm_desc_t* desc, const uint8_t* mask, lbm_problem_t** out);

/* Device bytes the workspace must have (including 256-byte alignment slack). */
size_t lbm_workspace_bytes(const lbm_problem_t* p);

/* Bind caller-owned device memory of at least lbm_workspace_bytes() bytes on
 * the current device and upload the node flags and inlet profile
 * (synchronous).  The workspace must outlive every later call. */
int lbm_bind_workspace(lbm_problem_t* p, void* device_ptr, size_t bytes);

/* Allocation-free binding, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Binds the library's static workspace of the current device
 * (a 32 MiB device array the library holds on every GPU it runs on until the
 * process ends) in place of caller memory, and uploads the node flags and
 * inlet profile (synchronous, on the default stream).  Neither this call nor
 * the later calls on p allocate device or pinned host memory (the residual
 * sums come back through pageable host memory, which can make those copies
 * wait for other streams).  Every problem bound this way on one device
 * shares that device's array, which keeps the last call's contents: binding
 * another problem takes the array over, after which the previous owner's
 * calls return LBM_ESTATE until it is bound again; calls on problems that
 * share a device's array must not overlap in time (they race).  The solves
 * clear every buffer they need zeroed themselves.  LBM_EINVAL if
 * lbm_workspace_bytes(p) exceeds 32 MiB (about 60,000 nodes of the coupled
 * D3Q19 + D3Q7 lattices); LBM_EDEVICE if the array's address cannot be
 * taken. */
int lbm_bind_static_workspace(lbm_problem_t* p);

/* Steady forward solve from rest (f = f_eq(rho0, 0), T = T_in).
 * gamma: device [N] design field (read).  drho: device [N], written with the
 * density deviation rho - rho0 (pressure deviation drho/3); u: device [3][N]
 * velocity; T: device [N] temperature (may be NULL without the thermal
 * lattice).  All fields are the moments of the final post-boundary state;
 * wall nodes get 0.  info (host, may be NULL) receives steps, residuals and J.
 * Returns LBM_OK, LBM_NOT_CONVERGED or an error. */
int lbm_forward_solve(lbm_problem_t* p, const float* gamma, float* drho, float* u, float* T,
                      lbm_info_t* info, void* stream);

/* Run exactly nsteps more forward steps from the current forward state (no
 * reset, no residual check) and write drho, u, T as lbm_forward_solve does.
 * Needs a previous lbm_forward_solve. */
int lbm_forward_continue(lbm_problem_t* p, const float* gamma, int32_t nsteps, float* drho,
                         float* u, float* T, lbm_info_t* info, void* stream);

/* Steady adjoint solve (Sec. 2.4) about the state (u, T) of the last forward
 * solve, starting from f*_C = 0 (Eq. 53).  gamma, u (device [3][N]) and T
 * (device [N], NULL without thermal) must be the ones that forward solve used
 * and returned; drho may be NULL (the incompressible equilibrium's Jacobian
 * does not depend on rho).  With the thermal lattice, the sensitivity also
 * needs the converged thermal non-equilibrium populations, which the last
 * lbm_forward_solve or lbm_thermal_resolve left in the workspace; without
 * one of them the call returns LBM_ESTATE.  A flow-only adjoint needs
 * nothing but (gamma, u).  info may be NULL.  Returns LBM_OK,
 * LBM_NOT_CONVERGED or an error. */
int lbm_adjoint_solve(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                      const float* T, lbm_info_t* info, void* stream);

/* Recover the converged thermal non-equilibrium populations from saved fields
 * only (for callers that keep gamma, u, T and not the populations, such as a
 * differentiable wrapper): the D3Q7 lattice is solved alone with u frozen,
 * from g = g_eq(T, u), to the residual criterion on mean T (desc tol,
 * check_every, max_steps).  At a converged forward state this is the same
 * linear fixed point.  Afterwards lbm_adjoint_solve may run; the forward flow
 * state is no longer available (lbm_forward_continue returns LBM_ESTATE) and
 * the J reported by later calls is NaN.  LBM_EINVAL without the thermal
 * lattice. */
int lbm_thermal_resolve(lbm_problem_t* p, const float* gamma, const float* u, const float* T,
                        lbm_info_t* info, void* stream);

/* Warm restarts for an optimisation loop: continue the forward (adjoint)
 * solve from its current state, with a possibly changed gamma, under the
 * descriptor's residual criterion (max_steps, tol, check_every), writing the
 * same outputs as lbm_forward_solve (lbm_adjoint_solve).  LBM_ESTATE without
 * a previous solve of that kind (and, with the thermal lattice, for the
 * adjoint without the thermal state of a forward solve). */
int lbm_forward_resume(lbm_problem_t* p, const float* gamma, float* drho, float* u, float* T,
                       lbm_info_t* info, void* stream);
int lbm_adjoint_resume(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                       const float* T, lbm_info_t* info, void* stream);

/* Level-set design update of the topology-optimisation loop (Sec. 2.2,
 * Eqs. 13-15 and 67), on the design nodes of the problem:
 *   s      = mean |J'| over the design nodes (J' = dJ, the sensitivity)
 *   lambda = exp(G) mean |J'/s - sigma lap(phi)|,  G = V - vmax   (Eq. 67)
 *   phi'   solves (I - K sigma lap) phi' = phi - K (J'/s + lambda), the
 *          step of Eq. (14) with the diffusion term taken at the new level
 *          set, then phi' = clamp(phi', -1, 1) (Eq. 13)
 *   gamma  = 1 where phi' >= 0, else 0 (Eq. 15)
 * V is the fluid fraction (phi >= 0) of the design domain before the step.
 * sigma lap is the 7-point stencil (5-point in 2D) in lattice units over
 * the design nodes, sum_a sigma[a] (phi(x + e_a) + phi(x - e_a) - 2 phi(x))
 * with sigma (host, 3 doubles) the coefficient per axis x, y, z (the
 * anisotropic regularisation of Sec. 3.3.4; equal for the isotropic one); a
 * neighbour that is not a design node (or lies outside the box) counts as
 * the node itself (no flux).  A dimensionless coefficient on a length L is
 * sigma L^2 here.  The implicit system is solved by red-black Gauss-Seidel
 * sweeps, as many as take the error below 1e-8 of the starting guess's.  phi, phi_out, dJ,
 * gamma: device [N] float; phi_out must not alias phi; non-design entries
 * of phi_out copy phi, of gamma are left unchanged.  Synchronises the
 * stream (two small reductions).  LBM_EINVAL for K <= 0, a sigma < 0, vmax
 * outside (0, 1], K sigma too large for 100000 sweeps, or no design nodes. */
typedef struct lbm_levelset_info {
  double lambda;           /* Eq. (67)                                        */
  double volume;           /* fluid fraction of the design domain (before)    */
  double G;                /* volume - vmax                                   */
  double scale;            /* mean |J'| over the design domain                */
} lbm_levelset_info_t;
int lbm_levelset_update(lbm_problem_t* p, const float* phi, float* phi_out, const float* dJ,
                        float* gamma, double K, const double* sigma, double vmax,
                        lbm_levelset_info_t* info, void* stream);

/* Run exactly nsteps more adjoint steps from the current adjoint state. */
int lbm_adjoint_continue(lbm_problem_t* p, const float* gamma, const float* drho,
                         const float* u, const float* T, int32_t nsteps, lbm_info_t* info,
                         void* stream);

/* dJ/dgamma (device [N], written; 0 on non-design nodes) from the last
 * adjoint state, Eq. (66): explicit dJ/dgamma - sum_i f*_S,i dC_i/dgamma
 * - sum_i g*_S,i dC^g_i/dgamma.  J (host, may be NULL) receives the objective
 * of the last forward solve.  Needs a previous lbm_adjoint_solve. */
int lbm_sensitivity(lbm_problem_t* p, const float* gamma, const float* drho, const float* u,
                    const float* T, float* dJdgamma, double* J, void* stream);

/* Copy a workspace state to device memory dst: which 0 = forward flow
 * populations (Q x N, Q = 19, or 9 on a 2D lattice), 1 = forward thermal
 * (Qg x N, Qg = 7, or 5 on a 2D lattice), 2 = adjoint flow (Q x N),
 * 3 = adjoint thermal (Qg x N), 4 = thermal non-equilibrium populations of
 * the last forward state (Qg x N).  Populations are
 * population-major [q][z][y][x] and stored shifted: f_i - w_i rho0 (forward
 * flow), g_i - w_i T_in (forward thermal); the forward state is the
 * post-collision one, the adjoint state the one after the adjoint boundary
 * condition.  Direction order is given by lbm_lattice. */
int lbm_copy_state(const lbm_problem_t* p, int32_t which, float* dst, void* stream);

/* Timing of the step kernels, for roofline reporting.  When enabled, each
 * forward and each adjoint sweep (a solve or a continuation) is bracketed by
 * a pair of HIP events on the call's stream; the step kernels of a sweep run
 * back to back, so sweep time over its step-kernel launches is their average
 * launch duration (the few residual reductions and host checks inside a
 * sweep are included, well under 1 % of it).  lbm_kernel_timing returns the
 * totals (ms[0], launches[0]: forward sweeps; ms[1], launches[1]: adjoint
 * sweeps) and, if reset != 0, clears them.  Enabling creates two events on
 * the bound device (needs a bound workspace). */
int lbm_set_kernel_timing(lbm_problem_t* p, int32_t enable);
int lbm_kernel_timing(lbm_problem_t* p, double* ms, int64_t* launches, int32_t reset);

/* Streaming ceiling of the forward step on the bound device: `launches`
 * back-to-back launches (after 10 untimed ones) of a kernel that moves
 * exactly the forward step's bytes in its pattern (every population pulled
 * from the same neighbour as in the step, gamma and the node flags read,
 * the pulled values stored unchanged) but does none of its arithmetic; the
 * average time per launch (HIP events on `stream`, synchronised) goes to
 * us_per_launch.  The step kernel's time over this one is how close the
 * step runs to what its access pattern allows.  gamma: device [N].  The
 * probe overwrites the workspace's forward populations, so afterwards no
 * forward or adjoint state remains (continue, resume and sensitivity calls
 * return LBM_ESTATE until the next solve).  LBM_EINVAL for launches outside
 * [1, 1000000]. */
int lbm_stream_probe(lbm_problem_t* p, const float* gamma, int32_t launches, double* us_per_launch,
                     void* stream);

/* Device-copy ceiling: `launches` back-to-back launches (after 3 untimed
 * ones) of the library's streaming copy kernel (16-byte loads and stores,
 * coalesced) from src to dst, `bytes` each; the average time per launch (HIP
 * events on `stream`, synchronised) goes to us_per_launch.  2 * bytes over
 * that time is the read + write bandwidth the device gives a plain stream;
 * buffers larger than the 256 MB Infinity Cache measure HBM.  src, dst:
 * caller-owned device buffers, 16-byte aligned, not overlapping; dst is
 * overwritten.  LBM_EINVAL for null or misaligned pointers, overlap, bytes
 * not a positive multiple of 16, or launches outside [1, 1000000]. */
int lbm_copy_probe(const void* src, void* dst, uint64_t bytes, int32_t launches,
                   double* us_per_launch, void* stream);

/* Direction table of the library: which 0 = D3Q19 (19 entries), 1 = D3Q7
 * (7 entries), 2 = D2Q9 (9 entries, e_z = 0), 3 = D2Q5 (5 entries); e
 * receives 3 ints per direction, w the weight. */
int lbm_lattice(int32_t which, int32_t* e, double* w);

/* ---------------------------------------------------------------------------
 * Continuous batching of many sensitivity solves (serving).
 *
 * A batch engine holds requests of one kind (thermal flag and objective) on
 * one GPU; a flow-only engine takes 2D (D2Q9) and 3D requests side by side,
 * with or without mirror planes, and either adjoint kind.  lbm_batch_submit queues a request (descriptor, host mask, host
 * design field; all copied).  Each lbm_batch_step call first admits queued
 * requests in arrival order while a slot is free and the request's workspace
 * and fields fit in the arena the caller bound (the HBM budget).  Work is
 * issued in quanta on lanes (HIP streams the engine owns): a quantum is
 * `quantum` ragged-batch kernel launches, each advancing every request of
 * the lane's run set (chosen by the policy, lbm_batch_set_policy) by one
 * step of its forward or adjoint sweep.  When a lane's quantum completes,
 * the residuals of its requests are checked and requests move from the
 * forward sweep to the adjoint sweep to dJ/dgamma exactly as
 * lbm_forward_solve / lbm_adjoint_solve / lbm_sensitivity would, so each
 * result is bit for bit the result of the same request solved alone.  A
 * request's max_steps and check_every must be multiples of the quantum.
 * lbm_batch_poll reports a ticket's state; once DONE or FAILED it returns
 * the result (copying dJ/dgamma to dJ_host, N floats, if non-NULL) and
 * releases the request's memory.  A request whose sweep diverges is FAILED
 * with status LBM_EDIVERGED and does not affect the others.  The arena is
 * caller-owned device memory; it must outlive the engine.  One host thread
 * at a time per engine.
 * ------------------------------------------------------------------------- */
#define LBM_BATCH_QUEUED 0
#define LBM_BATCH_RUNNING 1
#define LBM_BATCH_DONE 2
#define LBM_BATCH_FAILED 3

/* Scheduling policies: which resident requests a quantum advances. */
#define LBM_BATCH_POLICY_ALL 0     /* one lane: every resident request            */
#define LBM_BATCH_POLICY_SRW 1     /* one lane: shortest remaining work, filled    */
#define LBM_BATCH_POLICY_OVERLAP 2 /* two concurrent lanes (default)               */
#define LBM_BATCH_POLICY_OVERLAP_FIFO 3 /* two lanes, no request slowed by a later one */

typedef struct lbm_batch lbm_batch_t;

typedef struct lbm_batch_result {
  int64_t ticket;
  int32_t state;           /* LBM_BATCH_*                                      */
  int32_t status;          /* LBM_OK, LBM_NOT_CONVERGED or LBM_EDIVERGED        */
  int32_t nodes;           /* N of the request                                  */
  int32_t fwd_steps;       /* steps taken (so far, or until it failed) by the   */
                           /* forward sweep                                     */
  int32_t adj_steps;       /* same for the adjoint sweep (0: never started)     */
  int32_t reserved;
  double J;                /* objective (DONE only)                             */
} lbm_batch_result_t;

typedef struct lbm_batch_stats {
  uint64_t arena_bytes;    /* usable arena (budget)                             */
  uint64_t bytes_in_use;   /* held by resident requests                         */
  int32_t running, finished, queued, reserved;
  int64_t launches;        /* ragged-batch kernel launches so far               */
  int64_t node_updates;    /* node-steps advanced so far                        */
} lbm_batch_stats_t;

/* Engine for requests with this thermal flag and objective; at most
 * max_slots resident requests; quantum = steps a lane advances its run set
 * between visits of the host (admission, residual checks).  Under OVERLAP a
 * lone request too large for the latency lane runs on the bandwidth lane up
 * to its next residual check, at most 4 quanta, per visit.  LBM_EINVAL on bad
 * parameters. */
int lbm_batch_create(int32_t thermal, int32_t objective, int32_t max_slots, int32_t quantum,
                     lbm_batch_t** out);
/* Bytes of the arena taken by the engine's own tables for an arena of
 * arena_bytes (the rest is the budget for requests). */
size_t lbm_batch_table_bytes(const lbm_batch_t* b, size_t arena_bytes);
/* Bind caller-owned device memory as the arena (current device). */
int lbm_batch_bind_arena(lbm_batch_t* b, void* device_ptr, size_t bytes);
/* Scheduling policy.  ALL (one lane): every resident request advances every
 * quantum.  SRW (one lane): requests ordered by an upper bound of their
 * remaining node updates (nodes x steps left to the step caps of both
 * sweeps), taken greedily while the run set stays within fill_tiles tiles of
 * 256 nodes (the first is always taken).  OVERLAP (two lanes whose quanta
 * run concurrently): the latency lane takes requests of at most fill_tiles
 * tiles in arrival order, greedily up to fill_tiles; the bandwidth lane takes
 * the oldest remaining request and, if it is that small too, further small
 * ones up to fill_tiles.  OVERLAP_FIFO: the lanes of OVERLAP, but the
 * latency lane only takes requests that arrived before the oldest resident
 * request too large for it, so no request is slowed by one that arrived
 * after it (no worse than arrival order at the tail, small requests still
 * running beside large ones).  Requests in no run set stay resident and
 * paused.
 * The policy changes latency and throughput only, never a result.  Default
 * OVERLAP, fill 512.  LBM_EINVAL on an unknown policy or fill_tiles < 1,
 * LBM_ESTATE while a quantum is in flight. */
int lbm_batch_set_policy(lbm_batch_t* b, int32_t policy, int32_t fill_tiles);
/* Persistent quanta: a lane whose run set spans at most max_tiles tiles of
 * 256 nodes (a lone request included) runs its whole quantum as one
 * cooperative launch of the ragged-batch kernel, sized to the blocks the
 * device holds at once; its blocks loop over the quantum's steps with a
 * device-wide barrier between steps (a bounded wait: a barrier that waits
 * too long makes the launch give up and the lane's requests FAILED with
 * LBM_EDEVICE).  Larger run sets take one launch per step.  The arithmetic,
 * and so every result, is the same either way.  max_tiles = 0 turns the
 * persistent form off.  Default 0: on MI355X a device-wide barrier (a
 * device-scope atomic per block plus the L2 write-back every XCD needs) costs
 * more than the kernel boundary it replaces, so one launch per step is
 * faster at every run-set size measured.  LBM_EINVAL for max_tiles < 0,
 * LBM_ESTATE while a quantum is in flight. */
int lbm_batch_set_persistent(lbm_batch_t* b, int32_t max_tiles);
/* Queue a request; validates it (LBM_EINVAL, or LBM_ENOMEM if it can never
 * fit the arena) and returns its ticket. */
int lbm_batch_submit(lbm_batch_t* b, const lbm_desc_t* desc, const uint8_t* mask,
                     const float* gamma_host, int64_t* ticket);
/* Admit (uploads on `stream`, synchronised), start a quantum on every idle
 * lane, then wait until at least one lane's quantum has completed, do its
 * residual checks and phase moves and start that lane's next quantum.
 * Quanta may still be in flight on return.  active/queued (may be NULL)
 * receive the resident running requests and the queue length. */
int lbm_batch_step(lbm_batch_t* b, void* stream, int32_t* active, int32_t* queued);
/* State of a ticket; DONE/FAILED results are returned once and released. */
int lbm_batch_poll(lbm_batch_t* b, int64_t ticket, lbm_batch_result_t* res, float* dJ_host,
                   void* stream);
int lbm_batch_stats(const lbm_batch_t* b, lbm_batch_stats_t* out);
void lbm_batch_destroy(lbm_batch_t* b);

/* Release the handle (not the caller's workspace). */
void lbm_problem_destroy(lbm_problem_t* p);

/* Message of the last error on this thread ("" when none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMADJ_H */
