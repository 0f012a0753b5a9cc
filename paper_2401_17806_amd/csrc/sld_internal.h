// Internal state of the library: mesh and discretisation handles, error helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sld.h"
#include "refops.h"

// Thread-local error message (sld_last_error).
void sld_set_error(const std::string& msg);

#define SLD_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            sld_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));            \
            return SLD_E_HIP;                                                            \
        }                                                                                \
    } while (0)

// Triangles per tile: one thread block of the apply kernels owns a tile of consecutive
// triangles; the host builds each tile's halo (its neighbours outside the tile).
constexpr int kTriPerBlock = 64;
constexpr int kSlotWall = 1023;  // tile-local slot of a wall neighbour

// Neighbour entry packing: (triangle << 2) | local edge in that triangle; -1 = wall.
inline int32_t pack_nbr(int32_t tri, int32_t alpha) { return tri < 0 ? -1 : (tri << 2) | alpha; }

struct sld_mesh_s {
    std::atomic<int> refs{1};  // the caller's handle + one per disc built on the mesh
    int device = 0;
    int64_t ne = 0, nd = 0, nv = 0;
    bool periodic = false;
    // host copies
    std::vector<double> P;         // [ne][3][2] unwrapped vertex coordinates
    std::vector<int32_t> left, right, alpha_l, alpha_r;  // [nd]
    std::vector<int32_t> tedge;    // [ne][3] edge id of local edge alpha
    std::vector<double> shift;     // [nd][2] r's frame minus l's frame
    // device
    double4* geo = nullptr;        // [ne] (e1x, e1y, e2x, e2y): e1 = P1-P0, e2 = P2-P0
    int4* nbr = nullptr;           // [ne] packed neighbour across local edges 0,1,2; w unused
    // Internal triangle order of the CG (a Morton curve over centroids, so that tiles of
    // consecutive triangles are compact patches with small halos):
    int* perm = nullptr;           // [ne] internal index -> caller's triangle index
    double4* geo_i = nullptr;      // [ne] geo in internal order
    double4* geo_nb = nullptr;     // [ne][3] internal order: geo_i of the neighbour across local
                                   // edge alpha (zeros on a wall)
    int4* nbr_i = nullptr;         // [ne] internal neighbour ids (packed as nbr); w = the three
                                   // tile-local slots (10 bits each): 0..63 own tile, 64+h halo
    int* halo_pad = nullptr;       // [ntiles][max(hmax, 1)] halo triangles (internal ids) of
                                   // every tile, sorted, -1 padded
    int hmax = 0;                  // largest halo
    int64_t halo_total = 0;        // sum of halo sizes (diagnostics)
    int4* edges = nullptr;         // [nd] (l, r, alpha_l, alpha_r)
    int4* tedges = nullptr;        // [ne] (2*j + beta) per local edge; beta = 1 if i = r(j)
    double area_total = 0;         // |Omega|
};

// Workspace of the CG solver (allocated with the disc).
constexpr int kCgMaxGrid = 4096;     // blocks of the three-lane CG kernel (grid-stride beyond)
struct CgWork {
    double* x = nullptr;
    double* e = nullptr;           // FP64 CG: the correction to x since the last residual
                                   // replacement (the iteration kernel accumulates into e)
    double* r[2] = {nullptr, nullptr};  // ping-pong by iteration parity
    double* q[2] = {nullptr, nullptr};
    double* d[2] = {nullptr, nullptr};
    double* b = nullptr;           // projected right-hand side
    double* part = nullptr;        // [2][4][grid] partials of rr, dq, rq, qq (by parity)
    double* part_s = nullptr;      // [2][grid] partials of setup / finish reductions
    double* scal = nullptr;        // device scalars (CgScalars)
    double* host_scal = nullptr;   // pinned mirror of scal, then two block copy slots
    int grid = 0;                  // blocks of every CG kernel (FP64)
    int grid32 = 0;                // blocks of the FP32 vector-unit iteration and its reliable
                                   // updates (>= grid: that kernel holds fewer registers)
    bool front = false;            // iteration kernel variant: one tile per block, four roles
    int stream_x = -1;             // x with non-temporal accesses: -1 by working-set size, 0/1
    unsigned char* wall_i = nullptr;  // [ne] internal order: Dirichlet wall edges (bit per local
                                      // edge) of the current diffusion solve
    std::vector<hipEvent_t> events;  // block profiling and copy events (created on first solve)
    // graph blocks the last three FP64 solves of each kind (pressure, viscous) ran, newest
    // first, at graph size last_gb: how far the host may queue blocks ahead of its reads
    int last_blocks[2][3] = {{0, 0, 0}, {0, 0, 0}};
    int last_gb[2] = {0, 0};
    // mixed precision: FP32 inner CG state (e32 = the correction), its partials and scalars
    float* r32[2] = {nullptr, nullptr};
    float* q32[2] = {nullptr, nullptr};
    float* d32[2] = {nullptr, nullptr};
    float* e32 = nullptr;
    double* part32 = nullptr;      // [2][4][grid]
    double* scal_in = nullptr;     // inner-solve scalars (CgScalars)
    double* host_scal_in = nullptr;
    hipGraphExec_t graph32 = nullptr;
    int graph32_block = 0;
    hipStream_t capture = nullptr;   // private stream used to capture the iteration graph
    hipGraphExec_t graph = nullptr;  // captured block of iterations
    int graph_block = 0;             // iterations in `graph`
    hipGraphExec_t graph_shift = nullptr;  // the same for the viscous (mass-shifted) system
    int graph_shift_block = 0;
    // MFMA operator (kernels_mx.hip): available on meshes without wall edges (mx_ok); used by the
    // pressure and FP32 inner iterations of the current solve when use_mx; the graphs above were
    // captured with graph_mx[fp64, shift, fp32]
    bool mx_ok = false;
    bool use_mx = false;
    bool graph_mx[3] = {false, false, false};
    // pipelined CG (launch_pcg_*): FP64 pressure iterations of the current solve on a mesh of
    // one tile per block; the FP64 graph was captured with graph_pcg
    bool use_pcg = false;
    bool graph_pcg = false;
};

struct sld_disc_s {
    sld_mesh mesh = nullptr;
    int p = 0, nphi = 0, npsi = 0;
    void* ops_dev = nullptr;       // RefOps<p> on the device
    void* ops_host = nullptr;      // RefOps<p> on the host
    void* ops32_dev = nullptr;     // RefOps32<p> on the device (mixed precision)
    void* sl_dev = nullptr;        // SlOps<p> on the device (semi-Lagrangian projection)
    void* mx_dev = nullptr;        // MxTab<p> on the device (MFMA operands of the operator)
    size_t ops_bytes = 0;
    CgWork cg;
};

uint64_t sld_disc_bytes(const sld_disc_s* d);

// Kernel launchers (kernels_ops.hip, kernels_cg.hip).  All return hipError_t of the launch.
hipError_t launch_schur_apply(const sld_disc_s* d, const double* p, double* out, double scale,
                              hipStream_t s);
hipError_t launch_gradient(const sld_disc_s* d, const double* p, const double* vstar, double coef,
                           double* out, hipStream_t s);
hipError_t launch_divergence(const sld_disc_s* d, const double* v, double scale, double* out,
                             hipStream_t s);

// CG building blocks (kernels_cg.hip)
struct CgScalars {
    // layout of CgWork::scal (doubles)
    enum { RR = 0, BB = 1, TOL2 = 2, ITER = 3, DONE = 4, MAXIT = 5, MEAN = 6, ZERO = 7,
           RTRUE = 8, INTX = 9, ITER0 = 10, ITER1 = 11, IRS = 12, RRNOW = 13, GAP = 14, SIGMA = 15,
           RTH = 16, TOLU = 17, PA0 = 18, PA1 = 19, PG0 = 20, PG1 = 21, PLR = 22, NSCAL = 23 };
    // DONE codes written by the iteration kernel
    enum { kConverged = 1, kMaxit = 2, kBreakdown = 3, kRefresh = 4 };
};
// FP64 CG: the recursive residual is replaced by the recomputed one whenever its norm has dropped
// by this factor since the last replacement (and whenever it meets rtol)
constexpr double kReplaceFactor = 1e-3;
constexpr double kGapRestart = 0.3;
int cg_grid_for(const sld_disc_s* d, bool* front);
int cg_grid32_for(const sld_disc_s* d, int grid, bool front);
// engine 0 of sld_cg_solve (the library's choice): whether the pressure iterations of each
// precision run on the matrix cores, by the measured time per iteration on the 512x512x2, p = 3
// mesh (the vector-unit kernels are faster there in both precisions)
constexpr bool kAutoMx64 = false;
constexpr bool kAutoMx32 = false;
// sigma > 0: the viscous system (sigma Mbar - K) x = -b instead of -K x = -b (no 1^perp
// projection, no gauge)
hipError_t launch_cg_setup(const sld_disc_s* d, const double* b, const double* p0, bool warm,
                           double rtol, int maxit, double sigma, hipStream_t s);
hipError_t launch_cg_step(const sld_disc_s* d, int parity, bool shift, hipStream_t s);
hipError_t launch_cg_finish(const sld_disc_s* d, double* p_out, double sigma, hipStream_t s);
// FP64 residual replacement on the state the iteration kernel stopped on (buffers of parity src):
// x += e, e = 0; r = K x - b_int recomputed in FP64, d and q kept (moved to buffers 0), the four
// dots summed directly; scal: RR = |r|^2, GAP = |r - r_recursive|^2, DONE cleared,
// RTH = kReplaceFactor^2 RR; after a stop at rtol whose recomputed residual misses the target
// TOLU, the recursive target TOL2 is lowered fourfold; ITER0 = ITER + 1 -- or, when
// GAP > kGapRestart^2 RR (the kept
// direction is no longer conjugate to the new residual), a restart: ITER0 = 0 (the next launch
// takes d = r) and MAXIT reduced by the iterations done
hipError_t launch_cg_replace(const sld_disc_s* d, int src, double sigma, hipStream_t s);
// x += e, e = 0 (FP64 CG, before the solution is read)
hipError_t launch_cg_fold(const sld_disc_s* d, hipStream_t s);
// Pipelined CG (kernels_cg.hip): possible when the disc's CG grid has one tile per block; the
// iteration (replaces launch_cg_step when use_pcg), its setup after launch_cg_setup, and its
// residual replacement (in place of launch_cg_replace)
bool pcg_possible(const sld_disc_s* d);
hipError_t launch_pcg_step(const sld_disc_s* d, int parity, hipStream_t s);
hipError_t launch_pcg_init(const sld_disc_s* d, hipStream_t s);
hipError_t launch_pcg_replace(const sld_disc_s* d, hipStream_t s);
// engine 0 / pipelined 0 of sld_cg_solve: whether FP64 pressure solves on such meshes pipeline
constexpr bool kAutoPcg = false;
// Pipelined CG: replacement once the recursive residual has dropped by this factor.  Its
// recurrences for w, z and s carry rounding errors further than CG's, and the iteration count
// grows with the distance between replacements: on a walled 24x24x2, p = 3 mesh (rtol 1e-12;
// CG 2025 iterations) 2953 / 2628 / 2281 iterations at factors 1e-3 / 1e-2 / 1e-1.
constexpr double kPcgReplaceFactor = 0.1;
// ... and at least every kPcgSpan iterations (the residual norm can stay high for thousands of
// iterations while the recurrences drift)
constexpr int kPcgSpan = 1024;
// Static CG workspace of sld_cg_solve_static: kStaticCgDoubles doubles (64 MiB) per device, its
// device address looked up once per device (the device must be current).
constexpr size_t kStaticCgDoubles = size_t(8) << 20;
constexpr int kMaxDevices = 64;
hipError_t cg_static_scratch(int device, double** out);
// Dirichlet wall flags of the next diffusion solve from a per-edge mask (device [nd], NULL none)
hipError_t launch_wall_mask(const sld_disc_s* d, const unsigned char* edge_mask, hipStream_t s);
hipError_t launch_cg_step32(const sld_disc_s* d, int parity, hipStream_t s);
hipError_t launch_rel_init(const sld_disc_s* d, double rtol, int maxit, hipStream_t s);
hipError_t launch_rel_update(const sld_disc_s* d, hipStream_t s);
hipError_t launch_rel_restart(const sld_disc_s* d, hipStream_t s);
hipError_t launch_sl_advect(const sld_disc_s* d, const double* vbar, const double* q, int nc,
                            double dt, double* out, hipStream_t s);
hipError_t launch_rel_peek(const sld_disc_s* d, int resume, hipStream_t s);
// MFMA operator (kernels_mx.hip): table size and construction from RefOps<p> (host), LDS bytes
// of its kernels, standalone apply in caller order (f32: float in/out with the BF16x3 engine,
// else FP64), one CG iteration (the pressure or FP32 inner iteration of k_cg_step), resident
// blocks per CU of its CG kernel
size_t mx_tab_bytes(int p);
int build_mx_tables(int p, const void* refops, void* out);
size_t mx_lds_bytes(int p, int hmax, size_t word);
hipError_t launch_apply_mx(const sld_disc_s* d, const void* p, void* out, bool f32, hipStream_t s);
hipError_t launch_cg_step_mx(const sld_disc_s* d, int parity, bool f32, bool stream_x, hipStream_t s);
int mx_blocks_per_cu(const sld_disc_s* d, bool f32);
// grid transfers and the viscous right-hand side (kernels_imex.hip); strides in doubles
hipError_t launch_dual_to_main(const sld_disc_s* d, const double* vd, int nc, double* out,
                               int64_t o_is, int64_t o_cs, hipStream_t s);
hipError_t launch_main_to_dual(const sld_disc_s* d, const double* vm, int nc, int64_t v_is,
                               int64_t v_cs, double* out, hipStream_t s);
// b = scale A_i Mref f_c + gcoef gb (gb [ne][N] or NULL); x0 = f_c (or NULL)
hipError_t launch_mass_rhs(const sld_disc_s* d, const double* f, int64_t f_is, int64_t f_cs, int c,
                           double scale, const double* gb, double gcoef, double* b, double* x0,
                           hipStream_t s);
// G_b [ne][N] of Dirichlet data on the flagged wall edges (mask and values [nd][p+1] device)
hipError_t launch_dirichlet_rhs(const sld_disc_s* d, const unsigned char* edge_mask,
                                const double* values, double* out, hipStream_t s);
// v*[j][1] += coef t[j] on interior dual cells, v*[j] = 0 on wall cells (t [nd][Npsi])
hipError_t launch_buoyancy(const sld_disc_s* d, const double* t, double coef, double* vs,
                           hipStream_t s);
