/*
 * sld.h -- C ABI of the MI355X (gfx950) pressure Schur-complement library for the
 * staggered semi-Lagrangian IMEX DG scheme of Tavelli & Boscheri (main triangles
 * carry pressure, edge-based dual quads split into two sub-triangles carry velocity).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns sld_status (SLD_OK = 0); none throws, aborts or exits.
 *   On failure sld_last_error() returns a thread-local message valid until the next
 *   call on the same thread.
 * - Degree p is 1..4.  N_phi = (p+1)(p+2)/2 main DOFs per triangle (Section 3.2),
 *   N_psi = (p+1)^2 dual DOFs per edge (Section 3.2).
 * - Main (pressure) vectors: float64 [ne][N_phi], row-major, triangle-major.  DOF k of
 *   a triangle is the Lagrange node (a/p, b/p) of the reference triangle, numbered with
 *   b outer and a inner, mapped by the affine map of eq. linmap (vertex 0 -> (0,0),
 *   vertex 1 -> (1,0), vertex 2 -> (0,1)).
 * - Dual (velocity) vectors: float64 [nd][2][N_psi]: edge-major, then component x/y,
 *   then dual node (a/p, b/p) of the reference square numbered k = b*(p+1) + a
 *   (Section 3.2).  Nodes with a+b <= p lie in the left sub-triangle (b_l, A, B) with
 *   (1,0) -> A, (0,1) -> B; nodes with a+b > p lie in the right sub-triangle through
 *   x = b_r + (1-b/p)(A-b_r) + (1-a/p)(B-b_r) (eq. mapDual).
 * - Edge numbering (Section 3.1 leaves l and r arbitrary): edges are numbered in order of
 *   first appearance scanning triangles i = 0.. and local edges alpha = 0,1,2, i.e. the
 *   vertex pairs (v0,v1), (v1,v2), (v2,v0).  l(j) is the first triangle that references
 *   edge j, A -> B follow l's counter-clockwise order, the unit normal n_j points from l
 *   to r.  A boundary (wall) edge has r(j) = -1.
 * - Device pointers are caller-owned (e.g. torch tensors' data_ptr()) and must hold the
 *   stated number of float64 values on the handle's device.  The library keeps no caller
 *   pointer after a call returns.  All device work is ordered on `stream` (a hipStream_t,
 *   NULL = the default stream); functions return without waiting unless stated.
 * - Handles are not thread-safe: calls on one handle must not overlap.
 */
#ifndef SLD_H
#define SLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLD_OK = 0,
    SLD_E_INVALID = 1,   /* bad argument: null pointer, degree out of range, bad size */
    SLD_E_MESH = 2,      /* invalid mesh: non-positive area, non-manifold edge, ... */
    SLD_E_NOMEM = 3,     /* device or host allocation failed */
    SLD_E_HIP = 4,       /* a HIP runtime call failed */
    SLD_E_NOCONV = 5,    /* CG stopped before rtol (maxit, or the FP64 rounding floor of the
                            recomputed residual); the last iterate and report are written */
    SLD_E_BREAKDOWN = 6, /* CG breakdown: d.Ad <= 0 or a non-finite scalar */
    SLD_E_BUDGET = 7     /* a size or memory budget is exceeded */
} sld_status;

typedef struct sld_mesh_s* sld_mesh;
typedef struct sld_disc_s* sld_disc;

/* Thread-local message describing the last failure on this thread. */
const char* sld_last_error(void);
/* ABI version of this header (bumped on incompatible changes). */
int32_t sld_abi_version(void);

/* ------------------------------------------------------------------ mesh (Section 3.1)
 * sld_mesh_create: build the staggered mesh from host arrays.
 *   xy     host float64 [nv][2] vertex coordinates
 *   tri    host int32 [ne][3] vertex ids, counter-clockwise (positive Jacobian, Section 3.4.1)
 *   period host float64 [2] periodic box lengths, or NULL for a bounded domain.  For a
 *          periodic box every triangle is unwrapped to the image of each vertex nearest
 *          to its vertex 0, so triangles must be smaller than half a period.
 *   device HIP device ordinal that will hold the geometry, or -1 for a host-only handle
 *          (edge table and node queries only; device entry points then return
 *          SLD_E_INVALID).
 * Validation: ids in range, positive area, each vertex pair shared by at most two
 * triangles with opposite orientation, no edge joining a triangle to itself
 * (SLD_E_MESH otherwise).  Stores per triangle only its two edge vectors and its
 * neighbour table on the device (the paper's point that only geometric quantities are
 * stored per element, Section 3.4.1). */
sld_status sld_mesh_create(const double* xy, int64_t nv, const int32_t* tri, int64_t ne,
                           const double* period, int32_t device, sld_mesh* out);
sld_status sld_mesh_counts(sld_mesh mesh, int64_t* ne, int64_t* nd, int64_t* nv);
/* Host copies of the edge table: left/right triangle, and the local edge index (0..2) of
 * the edge in each; right = alpha_right = -1 on boundary edges.  Each array is [nd];
 * any pointer may be NULL. */
sld_status sld_mesh_edges(sld_mesh mesh, int32_t* left, int32_t* right,
                          int32_t* alpha_left, int32_t* alpha_right);
/* Drops the caller's handle; the mesh lives on while discs built on it exist. */
void sld_mesh_destroy(sld_mesh mesh);

/* ------------------------------------------------------------------ discretisation
 * sld_disc_create: reference operators of degree p (Section 3.4: mass matrices and the
 * reference divergence/gradient operators, here in the equivalent form of reference
 * stiffness, edge-node derivative and sub-triangle correction matrices), computed on the
 * host in float64 by exact Gauss quadrature, plus the solver workspace on the device.
 * The disc holds a reference to its mesh: sld_mesh_destroy may come before sld_disc_destroy,
 * and the mesh is freed when its handle and every disc built on it are destroyed.
 * flags: reserved, pass 0. */
sld_status sld_disc_create(sld_mesh mesh, int32_t p, uint32_t flags, sld_disc* out);
sld_status sld_disc_info(sld_disc disc, int32_t* p, int32_t* nphi, int32_t* npsi);
/* Host float64 [ne][N_phi][2] physical positions of the main DOF nodes (each triangle in
 * its own unwrapped frame). */
sld_status sld_main_nodes(sld_disc disc, double* xy_out);
/* Host float64 [nd][N_psi][2] physical positions of the dual DOF nodes (in the frame of
 * the edge's left triangle). */
sld_status sld_dual_nodes(sld_disc disc, double* xy_out);
/* Host float64 [ne][N_phi]: int_{T_i} phi_k dx (weights of the pressure gauge). */
sld_status sld_main_weights(sld_disc disc, double* w_out);
/* sld_ref_operator: host copy of one reference operator of the disc (Section 3.4; the
 * semi-Lagrangian rule of Section 3.5), float64, row-major, for inspection and tests.
 *   which  0: S    [3][N_phi][N_phi]  int_{T_ref} grad phi_k grad phi_l by derivative pair
 *                                     (xi xi, xi eta + eta xi, eta eta)
 *          1: Sh   [3][N_phi][N_phi]  the same over the sub-triangle of local edge alpha
 *          2: E    [2][p+1][N_phi]    d_xi / d_eta of phi_l at the nodes of edge alpha
 *          3: Pt   [2][N_phi][p+1]    sub-triangle correction of edge alpha (device form of
 *                                     the condensed dual mass inverse)
 *          4: C    [p+1][p+1]         S0^{-1} M1 (edge condensation)
 *          5: M1   [p+1][p+1]         1D mass matrix of the edge nodes
 *          6: w    [N_phi]            int_{T_ref} phi_k
 *          7: SL points  [(p+1)^2][2] Gauss points of the semi-Lagrangian projection
 *          8: SL proj    [N_phi][(p+1)^2] M_ref^{-1} Phi^T diag(w)
 *          9: Mref [N_phi][N_phi]     int_{T_ref} phi_k phi_l (Mbar_i = 2|T_i| Mref)
 *         10: Ldm  [N_phi][N_phi]     dual -> main projection of the half of the dual cell of
 *                                     edge alpha: Mref^{-1} int_{T^alpha} phi_k phi_n(zeta),
 *                                     n the sub-triangle's nodes (eq. d2m)
 *   alpha  local edge 0..2 (which = 1, 2, 3, 10), ignored otherwise
 *   host_out may be NULL (size query); *count receives the number of doubles; cap is the
 *   capacity of host_out in doubles (SLD_E_INVALID if too small). */
sld_status sld_ref_operator(sld_disc disc, int32_t which, int32_t alpha, double* host_out,
                            int64_t cap, int64_t* count);
void sld_disc_destroy(sld_disc disc);

/* ------------------------------------------------------------------ operators (device)
 * sld_schur_apply: Kp = K p with K of eq. pressure_final,
 *   (K p)_i = sum_{j in S_i} D_ij Mhat_j^{-1} (Q_{l(j),j} p_l + Q_{r(j),j} p_r),
 * in the paper's sign (K is symmetric negative semi-definite; K 1 = 0).  Wall edges do
 * not couple (K sums over interior edges).  p, Kp: device [ne][N_phi]; must not alias. */
sld_status sld_schur_apply(sld_disc disc, const double* p, double* Kp, void* stream);
/* sld_schur_apply_mx: the same K p (eq. pressure_final) with its reference contractions on the
 * matrix cores (Section 3.4.1: every triangle's blocks are the same reference matrices times its
 * geometry, so a tile of triangles contracts as two matrix products, MFMA).  Meshes without wall
 * edges (periodic boxes) only: SLD_E_INVALID otherwise.
 *   engine 0 (SLD_MX_F64): p, Kp device float64 [ne][N_phi], FP64 MFMA (v_mfma_f64_16x16x4);
 *   engine 1 (SLD_MX_BF16X3): p, Kp device float32 [ne][N_phi], the FP32 operator of the
 *     mixed-precision solve: BF16 MFMA (v_mfma_f32_16x16x32_bf16) on three-term bfloat16
 *     splits of both operands (24 bits, the six products above 2^-24 kept) accumulated in
 *     FP32, FP32 pointwise work on FP64-formed geometry.
 * Uses the disc's CG workspace as staging: must not overlap a solve on the same disc.  p and
 * Kp must not alias. */
enum { SLD_MX_F64 = 0, SLD_MX_BF16X3 = 1 };
sld_status sld_schur_apply_mx(sld_disc disc, const void* p, void* Kp, int32_t engine, void* stream);
/* sld_gradient: ghat_j = Mhat_j^{-1} (Q_{l(j),j} p_l + Q_{r(j),j} p_r) (eq. ad4.2, lambda = 1).
 * p device [ne][N_phi] -> g device [nd][2][N_psi]; zero on wall edges. */
sld_status sld_gradient(sld_disc disc, const double* p, double* g, void* stream);
/* sld_divergence: (D v)_i = sum_{j in S_i} D_ij v_j (eq. D), interior edges only.
 * v device [nd][2][N_psi] -> out device [ne][N_phi]. */
sld_status sld_divergence(sld_disc disc, const double* v, double* out, void* stream);
/* sld_pressure_rhs: b = scale * D v_star (right-hand side of eq. pressure_IMEX without the
 * gravity and buoyancy sources; scale = 1/(a_ss dt)). */
sld_status sld_pressure_rhs(sld_disc disc, const double* v_star, double scale, double* b,
                            void* stream);
/* sld_velocity_correct: v = v_star - coef * Mhat^{-1}(Q_l p_l + Q_r p_r) (eq. nc.2 solved for
 * the new velocity after the pressure solve; coef = a_ss dt).  v may alias v_star. */
sld_status sld_velocity_correct(sld_disc disc, const double* v_star, const double* p,
                                double coef, double* v, void* stream);

/* ------------------------------------------------------------------ semi-Lagrangian stage
 * sld_sl_advect: advection of main-grid DG fields over one step dt (Section 3.5; the Gauss-point
 * projection of the SL-IMEX stages, eq. intstage).  For every triangle and every point of the
 * collapsed Gauss-Legendre rule with p + 1 points per direction, the backward characteristic
 * is followed cell by cell with straight (explicit Euler) segments, the velocity of each
 * segment being the current cell's DG velocity at the segment's start; crossing an interior
 * edge continues in the neighbour (periodic boxes included), a wall edge or a cell whose
 * velocity points straight back out ends the walk.  The fields are evaluated at the foot in
 * the cell reached and projected onto the main basis:
 *   q_out_i = M_ref^{-1} sum_g w_g phi(xi_g) q(foot_g).
 *   vbar   device float64 [ne][2][N_phi]: nodal DG velocity on the main grid
 *   q      device float64 [ne][nc][N_phi]: the nc fields to advect (1 <= nc <= 8)
 *   dt     the time step (the trace goes back by dt)
 *   q_out  device float64 [ne][nc][N_phi]; must not alias q or vbar
 * Asynchronous on `stream`.  SLD_E_INVALID for bad arguments. */
sld_status sld_sl_advect(sld_disc disc, const double* vbar, const double* q, int32_t nc, double dt,
                         double* q_out, void* stream);

/* ------------------------------------------------------------------ CG (Section 3.3)
 * sld_cg_solve: matrix-free conjugate gradients for K p = b (run on -K, which is SPSD).
 *   b device [ne][N_phi]; it is projected onto the complement of the constant vector
 *   (the kernel of K on a periodic or all-wall mesh) before the solve.
 *   p device [ne][N_phi]; in: initial guess if params->warm_start, out: the solution with
 *   int_Omega p dx = 0.
 * Stopping rule: ||b - K p||_2 <= rtol ||b||_2 on coefficient vectors, with the residual
 * recomputed in FP64.  FP64: the iteration accumulates the correction to p since the last
 * residual replacement; the recursive CG residual is replaced by the recomputed one (p absorbs
 * the correction) whenever its norm has dropped by 1e-3 since the last replacement and whenever
 * it meets its target (d and the CG scalars are kept, or the iteration restarts from the new
 * residual when the two residuals differ by more than 30%).  When the recomputed residual
 * misses rtol, the recursive target is lowered fourfold -- unless the difference between the
 * two residuals, the rounding error of evaluating b - K p in FP64 (about
 * eps || |K| |p| || / ||b||: 3e-12 on a 128x128x2, p = 3 mesh, 4e-11 on 512x512x2), is at least
 * rtol / 2: rtol is then below what FP64 can confirm, and the solve returns SLD_E_NOCONV with
 * converged = 0 and the recomputed residual in rel_res_true.
 * Iterations run as a captured HIP graph of graph_block iterations
 * (scalars stay on the device); the calling thread blocks until the solve ends and reads the
 * scalars copied after each graph to test convergence.  From the second FP64 solve of a kind
 * (pressure or viscous) on a disc, the next graph is queued on `stream` before the current
 * one's scalars are read, while the disc's recent solves predict two more graphs; a graph
 * queued after convergence runs only launches that exit at entry.  Results are deterministic
 * (fixed-order reductions, no atomics) and do not depend on that queueing.  On SLD_E_NOCONV p
 * holds the last iterate and the report is filled. */
typedef struct {
    double rtol;          /* relative residual tolerance, e.g. 1e-12 (FP64) / 1e-11 (mixed) */
    double inner_rtol;    /* mixed only: reduction of the FP32 residual between two FP64
                             reliable updates (refreshes of x and of the true residual), e.g. 0.5 */
    int32_t maxit;        /* iteration cap (mixed: per inner solve) */
    int32_t warm_start;   /* nonzero: p holds the initial guess */
    int32_t graph_block;  /* iterations per convergence check (even, 2..4096; the mixed form's
                             FP32 blocks take at most 128, its bound between reliable updates) */
    int32_t profile;      /* nonzero: HIP events on `stream` around each captured block of
                             graph_block iterations; the report gives the mean time per
                             iteration over the blocks whose launches all iterated (FP64 only) */
    int32_t precision;    /* 0: FP64 CG.  1: mixed: one CG process in FP32 (FP32 vectors and
                             operator arithmetic; FP64 geometry and dot products) refreshed by
                             FP64 reliable updates (x accumulated in FP64, residual b - K x
                             recomputed in FP64, whenever the FP32 residual has dropped by
                             inner_rtol and at least every 128 FP32 iterations; the FP32
                             operator subtracts one DOF value from the inputs of each piece of
                             K, exact since each piece maps constants to zero, which keeps its
                             rounding relative to the local variation; the search direction
                             is kept while the recursive FP32 residual is within 0.3 of the
                             recomputed one, else the FP32 process restarts).  Stops at rtol on the FP64 residual,
                             or when it no longer improves (rounding floor) */
    int32_t max_outer;    /* mixed only: cap on reliable updates */
    int32_t engine;       /* reference contractions of the pressure iterations: 1 = the vector
                             units; 2 = the matrix cores (FP64 MFMA for FP64 iterations, BF16x3
                             MFMA for the FP32 inner iterations; see sld_schur_apply_mx) on
                             meshes without wall edges, the vector units otherwise; 0 = the
                             library's choice per precision (the faster form measured on the
                             512x512x2, p = 3 mesh).  Viscous solves use the vector units. */
    int32_t pipelined;    /* FP64 pressure iterations: 1 = CG as in Section 3.3; 2 = pipelined
                             CG (Ghysels and Vanroose: the same iterates in exact arithmetic,
                             the operator applied to a vector the previous iteration completed,
                             so it overlaps the global dot-product sums; residual replacement
                             as for CG), only where the CG grid holds one tile of 64 triangles
                             per block (cache-resident meshes, e.g. 128x128x2) and with the
                             vector units, SLD_E_INVALID otherwise; 0 = the library's choice. */
} sld_cg_params;

typedef struct {
    int32_t iters;        /* CG iterations performed (mixed: inner iterations, summed) */
    int32_t converged;    /* 1 if the recomputed residual met rtol */
    double rel_res;       /* ||r|| / ||b|| at exit: the residual last recomputed in FP64 */
    double rel_res_true;  /* ||b - K p|| / ||b|| recomputed at exit */
    double seconds;       /* wall time of the solve on the host */
    double step_us;       /* profile only: mean time per CG iteration inside captured blocks */
    int32_t timed_iters;  /* profile only: iterations the mean is taken over */
    int32_t outer_iters;  /* FP64: residual replacements; mixed: reliable updates */
} sld_cg_report;

sld_status sld_cg_solve(sld_disc disc, const double* b, double* p, const sld_cg_params* params,
                        sld_cg_report* report, void* stream);

/* sld_cg_solve_static: sld_cg_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same FP64
 * iteration, residual replacement and stopping rule, with the CG workspace (vectors, dot
 * partials, scalars) in a static device array of the library instead of the disc's workspace,
 * and plain kernel launches instead of captured graphs (a synchronisation after every
 * graph_block iterations); it calls no hipMalloc, hipFree or other allocating routine.
 *   Limit: the array holds 2^23 doubles (64 MiB) per device, enough for about 9.3e5 DOFs
 *   (ne * N_phi: e.g. a 215x215x2 mesh at p = 3); a larger disc returns SLD_E_BUDGET.  The
 *   array is set aside on each device the library runs on until the process ends.
 *   params: precision must be 0 (FP64) and profile 0 (SLD_E_INVALID otherwise).
 *   Every call on a device shares that device's array and the disc's pinned scalar mirror:
 *   calls that overlap on one device race (results undefined); calls in turn are independent
 *   (each call's setup rewrites every workspace word it reads).
 * Blocks like sld_cg_solve; results equal sld_cg_solve's up to rounding (the same kernels in
 * the same order). */
sld_status sld_cg_solve_static(sld_disc disc, const double* b, double* p,
                               const sld_cg_params* params, sld_cg_report* report, void* stream);

/* ------------------------------------------------------------------ IMEX time step (Section 4)
 * Grid transfers (eqs. d2m and m2d), the L2 projections between the main and the dual space
 * through the operator U of eq. u (U_ij[k][l] = int over T_ij of psi_k^(j) phi_l^(i)):
 *   sld_dual_to_main: out_i = Mbar_i^{-1} sum_{j in S_i} U_ij^T v_j
 *     v   device float64 [nd][nc][N_psi], out device float64 [ne][nc][N_phi]
 *   sld_main_to_dual: out_j = Mhat_j^{-1} (U_lj v_l + U_rj v_r)
 *     v   device float64 [ne][nc][N_phi], out device float64 [nd][nc][N_psi]; a wall edge's
 *     dual cell is its left half alone: the DOFs of the absent right half are set to 0
 * 1 <= nc <= 8; out must not alias v.  Asynchronous on `stream`.  SLD_E_INVALID for bad
 * arguments. */
sld_status sld_dual_to_main(sld_disc disc, const double* v, int32_t nc, double* out, void* stream);
sld_status sld_main_to_dual(sld_disc disc, const double* v, int32_t nc, double* out, void* stream);

/* Viscous / thermal (implicit diffusion) solve of the IMEX stages, the advection-diffusion
 * scheme of eq. ad5 with the main-grid Laplacian built from the staggered gradient and
 * divergence (eq. pressure_final) plus wall cells:
 *   (Mbar - c K_W) x = Mbar f + c G_b,   c = a_ss dt (viscosity or diffusivity) >= 0
 * (c = 0: x = f).  On a wall edge the dual cell is the left half alone.  Edges flagged in
 * wall_dirichlet (device uint8 [nd], caller's edge numbering; NULL: none) are Dirichlet: the
 * cell's gradient takes the jump to the data wall_values (device float64 [nd][p+1], the values
 * at the edge's p+1 nodes counted from its first vertex A; NULL: zero data), which enter G_b.
 * The other wall edges have zero flux (the cell keeps its sub-triangle stiffness, no jump).
 * f, x device float64 [ne][N_phi] (may alias).  Conjugate gradients on the positive definite
 * (1/c) Mbar - K_W, warm-started from f, with the iteration kernel of sld_cg_solve; params as
 * there (precision must be 0: FP64; warm_start is ignored); the stopping rule is relative to
 * ||(1/c) Mbar f + G_b||.  Blocks like sld_cg_solve.  SLD_E_NOCONV / SLD_E_BREAKDOWN as there. */
sld_status sld_viscous_solve(sld_disc disc, const double* f, double c,
                             const uint8_t* wall_dirichlet, const double* wall_values, double* x,
                             const sld_cg_params* params, sld_cg_report* report, void* stream);

/* sld_state: the device workspace of sld_imex_step on one disc (velocity on the main grid,
 * its semi-Lagrangian projection, the viscous solution, the dual intermediate velocity and a
 * right-hand side: 7 ne N_phi + 2 nd N_psi doubles).  Destroy it before its disc.  Steps on
 * one state (and any solve on its disc) must not overlap. */
typedef struct sld_state_s* sld_state;
sld_status sld_state_create(sld_disc disc, sld_state* out);
void sld_state_destroy(sld_state state);

typedef struct {
    double nu;                /* kinematic viscosity, >= 0 (0: no viscous solve) */
    int32_t R;                /* IMEX member (appendix tableaux): 0 = one stage, first order;
                                 only R = 0 is built */
    sld_cg_params pressure;   /* the pressure solve (FP64 or mixed) */
    sld_cg_params viscous;    /* the two viscous solves (FP64) */
} sld_imex_params;

typedef struct {
    sld_cg_report pressure;
    sld_cg_report viscous[2]; /* one per velocity component */
    double seconds;           /* wall time of the step on the host */
} sld_imex_report;

/* One step of the semi-Lagrangian IMEX scheme for incompressible Navier-Stokes (Section 4),
 * R = 0 (a_ss = 1), on a periodic mesh, without gravity or buoyancy sources:
 *   1. vbar = L_dm(v)                                      (eq. d2m)
 *   2. vbar_F = sld_sl_advect of vbar by itself over dt     (Section 3.5, eq. intstage)
 *   3. (Mbar - a_ss dt nu K) vbar* = Mbar vbar_F per component  (eq. ad5)
 *   4. v* = L_md(vbar*)                                     (eq. m2d)
 *   5. K p = (1 / (a_ss dt)) D v*, int p = 0                (eq. pressure_IMEX)
 *   6. v = v* - a_ss dt Mhat^{-1} (Q_l p_l + Q_r p_r)       (eq. nc.2)
 * v  device float64 [nd][2][N_psi]: in the velocity at t, out at t + dt.
 * p  device float64 [ne][N_phi]: out the pressure of the step (in: the initial guess when
 *    params->pressure.warm_start).  v and p must not alias.
 * Blocks until the step ends (synchronises `stream`).  SLD_E_INVALID for bad
 * arguments, R != 0 or a mesh with walls; a solver status (SLD_E_NOCONV, ...) stops the step
 * where it failed and is returned with the report filled so far. */
sld_status sld_imex_step(sld_state state, const sld_imex_params* params, double dt, double* v,
                         double* p, sld_imex_report* report, void* stream);

/* One R = 0 step of the Boussinesq natural-convection model (eqs. nc.1-nc.3 with the sources
 * of eq. pressure_IMEX) in a closed box, nondimensional with g beta = Delta T = L = 1 (so
 * nu = sqrt(Pr/Ra), kappa = 1/sqrt(Ra Pr) for the differentially heated cavity):
 *   1. vbar = L_dm(v); v and T advected to the feet of vbar over dt (sld_sl_advect)
 *   2. T: (Mbar - dt kappa K_W) T = Mbar T_F + dt kappa G_b with Dirichlet data temp_values
 *      on the walls flagged in temp_dirichlet and zero flux on the others (sld_viscous_solve)
 *   3. vbar*: (Mbar - dt nu K_W) vbar* = Mbar vbar_F per component, no-slip: Dirichlet zero on
 *      every wall
 *   4. v* = L_md(vbar*) + dt g beta (0, L_md(T)) on interior cells, zero on the wall cells
 *      (prescribed no-slip velocity; the constant gravity is absorbed into the pressure)
 *   5. K p = (1/dt) D v*, int p = 0; v = v* - dt Mhat^{-1} Q p
 * temp_dirichlet device uint8 [nd] (NULL: all walls adiabatic), temp_values device float64
 * [nd][p+1] at the edges' nodes from their first vertex (NULL: zero data).
 * v device [nd][2][N_psi], T device [ne][N_phi]: in at t, out at t + dt.  p device
 * [ne][N_phi] out (in: initial guess if params->pressure.warm_start).  No aliasing.
 * SLD_E_INVALID for bad arguments, R != 0 or a mesh without walls.  Blocks until done. */
typedef struct {
    double nu, kappa, gbeta;  /* viscosity, thermal diffusivity, g beta (>= 0, >= 0, any) */
    int32_t R;                /* 0 only */
    sld_cg_params pressure;   /* the pressure solve (FP64 or mixed) */
    sld_cg_params viscous;    /* the diffusion solves (FP64) */
} sld_boussinesq_params;

typedef struct {
    sld_cg_report pressure;
    sld_cg_report viscous[2];
    sld_cg_report temperature;
    double seconds;
} sld_boussinesq_report;

sld_status sld_boussinesq_step(sld_state state, const sld_boussinesq_params* params, double dt,
                               const uint8_t* temp_dirichlet, const double* temp_values,
                               double* v, double* T, double* p, sld_boussinesq_report* report,
                               void* stream);

/* ------------------------------------------------------------------ serving
 * Continuous batching of independent pressure solves (the paper's pressure stage of
 * eq. pressure_final, one per request) and IMEX steps (sld_server_submit_imex).  Requests are queued as they arrive; a worker thread
 * admits the first queued request whose disc is idle and whose footprint fits the remaining
 * memory budget (one request is always admitted when none runs), and runs sld_cg_solve on its
 * own HIP stream, so requests overlap on the device.  Requests on the same disc run in turn
 * (the disc owns the CG workspace).  Results are bitwise independent of the mix.
 *
 * sld_disc_footprint: device bytes a solve on `disc` uses (geometry, tables, workspace). */
typedef struct sld_server_s* sld_server;
sld_status sld_disc_footprint(sld_disc disc, uint64_t* bytes);
/* hbm_budget_bytes: cap on the summed footprint (plus b and p) of running requests;
 * nworkers: concurrent solves (1..64), each with its own default-priority HIP stream. */
sld_status sld_server_create(int32_t device, uint64_t hbm_budget_bytes, int32_t nworkers,
                             sld_server* out);
/* Queue a solve of K p = b on `disc`.  b, p: device [ne][N_phi] buffers that must stay valid
 * until the ticket completes.  The solve waits for work already queued on `stream` (the
 * submitter's stream, NULL = default stream) before reading b.  SLD_E_BUDGET if the request
 * alone exceeds the budget. */
sld_status sld_server_submit(sld_server server, sld_disc disc, const double* b, double* p,
                             const sld_cg_params* params, void* stream, uint64_t* ticket);
/* Queue one IMEX step (sld_imex_step) on `state`.  v, p: device buffers as for sld_imex_step
 * that must stay valid until the ticket completes; the step waits for work already queued on
 * `stream` before it starts.  The ticket's report is the step's pressure-solve report.  An
 * IMEX request holds its state's disc while it runs, like a solve on that disc.
 * SLD_E_BUDGET if the request alone exceeds the budget. */
sld_status sld_server_submit_imex(sld_server server, sld_state state, const sld_imex_params* params,
                                  double dt, double* v, double* p, void* stream, uint64_t* ticket);
/* Completion of a ticket: *done = 1 when p holds the result (then *status is the solve's
 * sld_status and *report its report, and the ticket is retired).  wait != 0 blocks until done. */
sld_status sld_server_poll(sld_server server, uint64_t ticket, int32_t wait, int32_t* done,
                           int32_t* status, sld_cg_report* report);
sld_status sld_server_stats(sld_server server, int32_t* queued, int32_t* running,
                            uint64_t* in_flight_bytes, uint64_t* completed);
/* Finishes every queued request, then joins the workers. */
void sld_server_destroy(sld_server server);

#ifdef __cplusplus
}
#endif

#endif /* SLD_H */
