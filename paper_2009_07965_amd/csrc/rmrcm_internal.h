// Internal declarations shared by the host runtime (api.cpp) and the HIP
// kernel files.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rmrcm.h"

namespace rmrcm {

// Geometry of the finest decomposition, passed by value to kernels.
struct Geo {
    int nx, ny;        // fine cells
    int bx, by;        // subdomain size (cells)
    int sg;            // segment length (cells)
    int mx, my;        // subdomains per direction
    int nsx, nsy;      // segments per S/N side and per W/E side of a subdomain
    int lines_v;       // segments along one vertical interface line (= ny / sg)
    int lines_h;       // segments along one horizontal interface line (= nx / sg)
    int nv;            // number of vertical segments
    int nseg;          // total segments
    double hx, hy;
    double alpha;
    // 3D (three_d = 1): nz cell layers of height hz; in 2D nz = 1 and
    // hz = 1 (unit depth: a face area is its 2D length)
    int nz = 1, three_d = 0;
    double hz = 1.0;
    // Neumann mode (the downscaling solves): faces on Robin slots carry no
    // conductance, and a subdomain whose pin entry is nonzero (no Dirichlet
    // face) gets the full half-cell conductance on the W face of its cell
    // (0, 0) with no datum, which fixes the constant of its Neumann problem
    int neumann = 0;
    const int* pin = nullptr;
    // general interface spaces: pieces (segments above) per U-segment and
    // per P-segment (1 and 1: the MuMM spaces)
    int mu = 1, mp = 1;
};

// Cells, boundary faces and one-sided flux blocks of a problem.
__host__ __device__ inline size_t geo_ncell(const Geo& g) { return (size_t)g.nx * g.ny * g.nz; }
__host__ __device__ inline size_t geo_nbf(const Geo& g) {
    return g.three_d ? 2 * ((size_t)g.ny * g.nz + (size_t)g.nx * g.nz + (size_t)g.nx * g.ny)
                     : 2 * (size_t)g.nx + 2 * (size_t)g.ny;
}
__host__ __device__ inline int geo_nflux(const Geo& g) { return g.three_d ? 6 : 4; }

// Slot -> segment code: (segment id << 1) | low_side, or -1 if the slot lies
// on the outer boundary.  low_side = 1 when the node is on the low (left or
// bottom) side of the segment, i.e. the slot is on its E or N side.
__host__ __device__ inline int slot_code(int seg, int low) { return (seg << 1) | low; }

// One level of the nested binary hierarchy (depth 0 = whole domain,
// depth D = finest subdomains).  Nodes at one depth all have the same
// shape; their slots (boundary segments, listed W, E, S, N) are padded to
// the full perimeter, inactive slots carry zero trace rows and columns.
struct Level {
    int depth = 0;
    int nodes_x = 0, nodes_y = 0, nnodes = 0;
    int sx = 0, sy = 0;        // node size in subdomains
    int nslot = 0;             // slots per node
    int ld = 0;                // nslot + 1 (trace columns: slots + particular)
    double* T = nullptr;       // [nnodes][nslot][ld] traces (depth >= 1)
    int* slotseg = nullptr;    // [nnodes][nslot] slot codes
    // merge of this level's nodes from their two children (depth < D)
    int cut = 0;               // 0: cut in x (children side by side), 1: cut in y
    int g = 0;                 // segments on gamma
    int xi = 0;                // 2 g interface unknowns (one Robin datum per side)
    int* pmap = nullptr;       // [nslot] (child << 24) | child slot
    int* gmap = nullptr;       // [2][g] gamma -> child-1 slot, child-2 slot
    int* gseg = nullptr;       // [nnodes][g] global segment of every gamma segment
    double* M = nullptr;       // [nnodes][4 g^2]: D^{-1}, E, S^{-1}, B of the merge
    double* X = nullptr;       // [nnodes][xi][ld] coefficients of every column
    double* work = nullptr;    // scratch of the merges (merge_work_doubles)
    unsigned char* tflag = nullptr;   // [nnodes][(nslot + 64) / 64] 64-slot tiles with an active
                                      // slot (or the particular column)
    std::vector<int> h_pmap, h_gmap, h_slotseg, h_gseg;
    std::vector<unsigned char> h_tflag;
};

}  // namespace rmrcm

struct rmrcm_ctx {
    rmrcm_params prm{};
    rmrcm::Geo geo{};
    int D = 0;                               // finest depth
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    bool any_dirichlet = false;
    bool solved = false;
    bool check_pending = false;   // device-detected errors of an asynchronous refactor
    bool setup_recorded = false;
    bool solve_recorded = false;
    bool capturing = false;       // enqueueing into a graph capture: no events, no host sync
    bool step_graph = true;       // rmrcm_step replays a captured graph (FP64, device arrays)
    hipGraphExec_t gstep = nullptr;            // rmrcm_step graph (FP64 contexts)
    const void* gstep_key[5] = {};             // the pointers it was captured with
    int ct_tune[32] = {};         // per depth: column tile of the merge apply (0 = default)
    // downward pass of the deepest short-interface depths in one launch
    // (built by build_down_sub; down_ds == D: none)
    int down_ds = 0;
    bool root_down_fused = false; // the root's downward step done by the top's particular column
    int* down_tab = nullptr;      // [subtrees][entries] source of every data-vector entry
    std::vector<int> h_down_tab;  // its host copy (built by build_down_sub)
    int down_entries = 0, down_results = 0;
    int down_toff[8] = {}, down_roff[8] = {};
    // device arrays
    double* K = nullptr;                     // [ny][nx]
    int8_t* bct = nullptr;                   // [2ny + 2nx]
    double* beta = nullptr;                  // [nseg]
    double* seglen = nullptr;                // [nseg]
    double* Pstore = nullptr;                // [nsub][by][bx][bx]  S_j^{-1} of every block row
    float* P32 = nullptr;                    // mixed mode: the same in FP32
    float* Wsc = nullptr;                    // mixed mode: sweep scratch [nsub][nslot][bx*by]
    double* resid = nullptr;                 // mixed mode: relative residual per subdomain
    int* fb = nullptr;                       // mixed mode: 1 = subdomain redone in FP64
    int* pfb = nullptr;                      // mixed mode: 1 = particular solution of the
                                             // last solve redone in FP64
    double* dscal = nullptr;                 // device scalar
    int* irst = nullptr;                     // mixed mode: {converged, passes} of setup, solve
    double* irhist = nullptr;                // mixed mode: [2][kIrHist] residual per pass
    double* Psi = nullptr;                   // [nsub][nslot][bx*by] basis pressures
    double* pbar = nullptr;                  // [nsub][bx*by] particular pressures
    double* glo = nullptr;                   // [nseg] Robin datum on the low side
    double* ghi = nullptr;                   // [nseg] Robin datum on the high side
    double* q = nullptr;                     // staging for host inputs / outputs
    double* bcv = nullptr;
    double* pout = nullptr;
    double* fout = nullptr;
    double* Uout = nullptr;
    double* Pout = nullptr;
    int* flags = nullptr;                    // [kNumFlags] device error flags
    double* gauge = nullptr;                 // partial sums of the zero-mean gauge
    std::vector<rmrcm::Level> levels;        // index = depth
    size_t device_bytes = 0;
    // Device arrays carved from a caller-provided region instead of
    // hipMalloc (the allocation-free entry point): base, capacity, bytes used.
    // Null: every array has its own allocation.
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    // Memory plan only: dalloc counts the bytes of every array and
    // allocates nothing (rmrcm_plan_bytes).
    bool counting = false;
    // timing
    hipEvent_t ev[17] = {};
    // FP64 overlap of the particular chain with the setup merges: an
    // auxiliary stream, one event per merge level of the setup, the end of
    // the local setup, the inputs of a solve and the end of the aux work
    hipStream_t aux = nullptr;
    hipEvent_t lev[32] = {};
    hipEvent_t ev_ls = nullptr, ev_done = nullptr, ev_aux = nullptr;
    bool lev_recorded = false, done_recorded = false;
    bool solve_overlapped = false;  // the last solve ran the particular chain on aux
    double t_setup_ms[8] = {};
    double t_solve_ms[8] = {};
    double iface_resid = 0.0;                // last interface residual / pressure scale
    int iface_refined = 0;                   // 1 when the last solve ran the refinement step
    double iface_resid_after = 0.0;          // residual / scale after the first step (when it ran)
    int n_pfallback = 0;                     // particular solutions redone in FP64 (last solve)
    int64_t n_local_solves = 0;
    int ir_iters_setup = 0, ir_iters_solve = 0, n_fallback = 0;
    // learned mode: surrogate network, its inputs / outputs, accepted count
    struct rmrcm_cnn* net = nullptr;
    float* lx = nullptr;                     // [nsub][2][S][S] features
    float* ly = nullptr;                     // [nsub][R][S][S] predicted basis
    int* lint = nullptr;                     // [nsub] interior mask
    double* gres = nullptr;                  // [nsub] gate residual of the prediction
    // downscaling (allocated by its first call): the Neumann factor store,
    // the cell source of the Neumann problems, their solution (per-subdomain
    // layout), the gauge flag per subdomain, staging of host inputs/outputs
    double* ds_P = nullptr;
    double* ds_q = nullptr;
    double* ds_pb = nullptr;
    int* ds_pin = nullptr;
    double* ds_stage = nullptr;              // [10][ny][nx]: p in, F in, p out, F out
    // interface refinement: the segment residuals (r13, r14), the saved
    // Robin data, the device flag that runs the refinement's chain, and
    // the flag the kernels of a chain check (null outside that chain)
    double* iref_res = nullptr;              // [2][nseg] + 4: largest residual, pressure scale
                                             // before the step and after it
    double* iref_save = nullptr;             // [2][nseg]
    int* iref_flag = nullptr;
    const int* run_ptr = nullptr;
    int n_accepted = 0;
    double ir_resid_setup = 0.0, ir_resid_solve = 0.0;
};

namespace rmrcm {

// Kernel launchers (return hipError_t of the launch).
// The permeability check and the segment Robin parameters in one launch;
// copy non-null: the permeability is also copied there in the same pass.
hipError_t launch_check_beta(rmrcm_ctx* c, double* copy);
// part = 1: the particular problem solved beside the basis (FP64, subdomains
// 16 or 32 cells wide: local_setup_solves_particular), its solution to
// pbar and its traces to the last column of the finest T.
hipError_t launch_local_setup(rmrcm_ctx* c, bool fp32, const int* mask, int want, int do_traces,
                              int basis = 1, int part = 0);
bool local_setup_solves_particular(const rmrcm_ctx* c, bool fp32);
hipError_t launch_local_particular(rmrcm_ctx* c, bool fp32, const int* mask, int want,
                                   int do_traces);
hipError_t launch_local_refine(rmrcm_ctx* c, int part, int apply);
hipError_t launch_local_traces(rmrcm_ctx* c, int part, const int* mask, int want);
// First-order correction of the finest traces for the rounding of the local
// solves (basis: columns 0..R-1; part: the particular column), from the
// FP64 residuals of the stored solutions.
hipError_t launch_trace_correct(rmrcm_ctx* c, int basis, int part);
// The device side of the mixed-precision refinement: irst[2 part] is set
// once a pass measured every residual within ir_tol (later passes return at
// once), irst[2 part + 1] counts the passes, irhist keeps their residuals;
// the fallback marking runs only when the setup refinement did not converge.
hipError_t launch_mark_fallback(rmrcm_ctx* c, double tol);
hipError_t launch_max_resid(rmrcm_ctx* c, int part);
hipError_t launch_mark_part_fallback(rmrcm_ctx* c);
// part: the particular column is eliminated with the basis columns (their
// traces already hold it), as launch_merge_particular would below the top.
hipError_t launch_merge_setup(rmrcm_ctx* c, int depth, bool part = false);
// Scratch doubles of a level's merges, all nodes (nonzero for g >= 128,
// and for every level with general interface spaces).
size_t merge_work_doubles(const rmrcm_ctx* c, const Level& L);
hipError_t launch_merge_particular(rmrcm_ctx* c, int depth);
hipError_t launch_down(rmrcm_ctx* c, int depth);
// The downward pass of every depth (the deep, short-interface depths in one launch).
hipError_t launch_down_all(rmrcm_ctx* c);
// Chooses the depths of that launch and builds its source table on the
// host (c->h_down_tab); RMRCM_* code.
int build_down_sub(rmrcm_ctx* c);
hipError_t launch_reconstruct(rmrcm_ctx* c);
hipError_t launch_iface_resid(rmrcm_ctx* c, double tol, double* mx, int* flag, const int* run);
// 3D columns: factor store, basis and particular solution (factor = 1), or
// the particular solution with the stored factor (factor = 0); the
// reconstruction
hipError_t launch_local3d(rmrcm_ctx* c, int factor, int basis, int part);
hipError_t launch_reconstruct3d(rmrcm_ctx* c);
hipError_t launch_iface_inject(rmrcm_ctx* c);
hipError_t launch_iface_apply(rmrcm_ctx* c);
hipError_t launch_ds_source(rmrcm_ctx* c, const double* F, const double* q, double* qo);
hipError_t launch_ds_compat(rmrcm_ctx* c, const int* pin, double* qo);
hipError_t launch_ds_finish(rmrcm_ctx* c, const double* pb, const double* p_in, const double* F_in,
                            const int* pin, double* p_out, double* f_out);
hipError_t launch_interface_values(rmrcm_ctx* c);
hipError_t launch_gauge(rmrcm_ctx* c);
hipError_t launch_fill_i32(rmrcm_ctx* c, int* p, size_t n, int v);
hipError_t launch_fill_f64(rmrcm_ctx* c, double* p, size_t n, double v);
hipError_t launch_compat_check(rmrcm_ctx* c);
hipError_t launch_features(rmrcm_ctx* c, float* x, int* interior);
hipError_t launch_gate(rmrcm_ctx* c, const float* Y, const int* interior, double tau);
// Merge apply of the basis columns of one depth with column tile ct (the
// autotuner times it; ct in {4, 8, 16}).
hipError_t launch_merge_apply(rmrcm_ctx* c, int depth, int ct);
bool merge_apply_tunable(rmrcm_ctx* c, int depth);

// Device error flag slots.
enum { FLAG_LOCAL_SINGULAR = 0, FLAG_MERGE_SINGULAR = 1, FLAG_BAD_PERM = 2, FLAG_FALLBACK = 3,
       FLAG_BAD_DATA = 4, FLAG_ACCEPTED = 5, FLAG_NOTCONV = 6, FLAG_PFALLBACK = 7, kNumFlags = 8 };

// Residual history entries per refinement (setup, solve) kept on the device.
constexpr int kIrHist = 16;

}  // namespace rmrcm
