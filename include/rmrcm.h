/*
 * rmrcm.h - C ABI of the MI355X implementation of the recursive multiscale
 * Robin coupled method (MRCM) for 2D Darcy flow.
 *
 * Method: Abreu, Ferraz, Espirito Santo, Pereira, Santos, Sousa,
 * "Recursive formulation and parallel implementation of multiscale mixed
 * methods".  The problem is the mixed Darcy system of Section 2 (model
 * equations: div u = f, u = -K grad p, p = g_D on the Dirichlet part,
 * u.n = g_N on the Neumann part) on [0,lx] x [0,ly], discretised on a
 * uniform nx x ny grid by lowest-order Raviart-Thomas elements with a
 * lumped velocity mass (the cell-centred two-point scheme that Section 2.1
 * calls equivalent).  The domain is split into sub_nx x sub_ny-cell
 * subdomains (Section 3.1 hierarchy, a power of two per direction as in
 * Section 4) whose interfaces carry piecewise-constant flux and pressure
 * unknowns on segments of `seg` fine faces (the intermediate scale Hbar of
 * Section 4).  Subdomains are coupled by Robin conditions with
 * beta = alpha * Hbar / Keff (Section 5.1, Robin-beta equation).
 *
 * Conventions shared by every entry point
 *  - Arrays are row-major: cell (i, j), i along x, j along y, at index
 *    j * nx + i.  Permeability, source and pressure are nx*ny doubles.
 *  - Boundary faces: 2*ny + 2*nx entries ordered W (ny faces, bottom to
 *    top), E (ny), S (nx faces, left to right), N (nx).  Type 1 =
 *    Dirichlet (value = pressure), 0 = Neumann (value = OUTWARD INTEGRATED
 *    flux through the face).
 *  - The source is cell-integrated (q_c = integral of f over cell c).
 *  - Flux output: 4*nx*ny doubles, structure of arrays
 *    [W | E | S | N][ny][nx]: the outward integrated flux of each cell
 *    through each of its faces.  On the interfaces between subdomains the
 *    method's fluxes are one-sided (no downscaling, Section 4), so the two
 *    cells of such a face each report their own value.
 *  - Interface segments are numbered: vertical segments first, by
 *    interface line x = I*sub_nx*hx (I = 1..mx-1), bottom to top; then
 *    horizontal segments by line y = J*sub_ny*hy (J = 1..my-1), left to
 *    right.  The global normal of a segment points to +x or +y.
 *  - Every pointer argument may be host or device memory; the library
 *    tells them apart with hipPointerGetAttributes.  The caller owns every
 *    buffer it passes; the library copies what it must keep.
 *  - All functions return RMRCM_OK (0) or a negative RMRCM_E* code and
 *    never throw.  Invalid arguments are rejected before any device work.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef RMRCM_H
#define RMRCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmrcm_ctx rmrcm_ctx;

enum {
    RMRCM_OK = 0,
    RMRCM_EINVAL = -1,     /* invalid argument or geometry */
    RMRCM_ENOMEM = -2,     /* device or host allocation failed */
    RMRCM_EDEVICE = -3,    /* a HIP call failed */
    RMRCM_ESINGULAR = -4,  /* a local or interface system is singular */
    RMRCM_ENOTCONV = -5,   /* iterative refinement did not converge (not returned by this
                              version: subdomains that do not converge are redone in FP64) */
    RMRCM_ESTATE = -6,     /* call out of order (e.g. solve before setup) */
    RMRCM_ENOTSUP = -7,    /* configuration not supported by this build */
    RMRCM_ETOOBIG = -8     /* problem exceeds the fixed scratch of rmrcm_step_noalloc */
};

/* Precision modes of the local solves.  Interface merges always run in
 * FP64.  RMRCM_MIXED: local factorisations and sweeps in FP32, accuracy
 * recovered by iterative refinement with FP64 residuals (the basis and the
 * particular solutions are stored in FP64); subdomains whose refinement
 * does not reach ir_tol are factored again in FP64.
 * RMRCM_MIXED_LEARNED: as RMRCM_MIXED, but the local basis of every
 * interior subdomain (no face on the outer boundary) is first predicted by
 * the surrogate network loaded from cnn_weights (rmrcm_cnn_save format,
 * patch side = sub_nx = sub_ny, outputs = boundary segments per subdomain).
 * A prediction is accepted when, for every basis column, the FP64 residual
 * of the local Robin system |A y - e|_2 / |e|_2 <= gate_tol; an accepted
 * subdomain computes only its FP32 factor and takes the prediction as the
 * starting iterate of the FP64-residual refinement (instead of the FP32
 * solve), so that its basis meets ir_tol like every other; the others run
 * the RMRCM_MIXED path.  gate_tol = 0 accepts nothing (the result is then
 * that of RMRCM_MIXED). */
enum { RMRCM_FP64 = 0, RMRCM_MIXED = 1, RMRCM_MIXED_LEARNED = 2 };

enum { RMRCM_BC_NEUMANN = 0, RMRCM_BC_DIRICHLET = 1 };

typedef struct {
    int32_t nx, ny;          /* fine cells; > 0 */
    double lx, ly;           /* domain extents; > 0 */
    int32_t sub_nx, sub_ny;  /* subdomain size in cells: divides nx, ny;
                                nx/sub_nx and ny/sub_ny powers of two;
                                sub_nx in {4, 8, 16, 32}, sub_ny <= 64 */
    int32_t seg;             /* segment length in cells; divides sub_nx and sub_ny */
    double alpha;            /* Robin alpha > 0 */
    int32_t precision;       /* RMRCM_FP64 | RMRCM_MIXED | RMRCM_MIXED_LEARNED */
    double ir_tol;           /* mixed: refinement stops when max over subdomains and
                                columns of |b - A x|_inf / |b|_inf <= ir_tol; default 1e-11 */
    int32_t ir_max_iter;     /* mixed: refinement passes before the subdomains still above
                                ir_tol are redone in FP64 (setup: factor and basis, kept;
                                solve: the particular solution, with an FP64 factor for
                                that solve);
                                default 6 */
    double gate_tol;         /* learned: residual gate tau >= 0; default 1e-6 */
    const char* cnn_weights; /* learned: weight file (required in that mode) */
    int32_t device;          /* HIP device ordinal */
    uint64_t mem_cap;        /* device bytes a context may take (the plan of
                                rmrcm_plan_bytes); 0 = no limit.  A setup whose
                                plan exceeds it returns RMRCM_ENOMEM before any
                                device work. */
    int32_t seg_u, seg_p;    /* general MRCM interface spaces (Section 2 leaves the flux
                                space U_H and the pressure space P_H free; Section 4's
                                MuMM takes both piecewise constant on the same
                                segments): U_H piecewise constant on segments of seg_u
                                cells, P_H on segments of seg_p cells; 0 = seg.  Each
                                divides sub_nx and sub_ny and the longer is a multiple
                                of the shorter.  The segments of the documented order,
                                of the traces and of rmrcm_get_interface are then the
                                pieces of min(seg_u, seg_p) cells (U and P constant
                                over each U- and P-segment); beta is that of the
                                piece's U-segment (Hbar its length, Keff over its
                                faces); eq. 14.2 holds on U-segments and eq. 13.2 on
                                P-segments.  rmrcm_step_noalloc supports only
                                seg_u = seg_p = seg (ENOTSUP otherwise). */
    int32_t nz;              /* 0: the 2D problem above.  >= 1: the 3D problem of the
                                paper's experiments (Section 5) on [0,lx] x [0,ly] x
                                [0,lz] with nx x ny x nz cells (seven-point scheme),
                                split into columns of sub_nx x sub_ny x nz cells (no
                                division in z, Hbar_z = H_z: a segment is seg faces
                                along its interface line by the full height; beta =
                                alpha Hbar / Keff with Hbar its length along the line and
                                Keff over all of its faces).  Cell (i,j,k) at index
                                (k*ny + j)*nx + i; flux: 6 blocks of nx*ny*nz cells
                                (W E S N B T, outward); boundary faces in the order
                                W (ny*nz, index k*ny + j), E, S (nx*nz, index k*nx + i),
                                N, B (z = 0, nx*ny, index j*nx + i), T.  FP64 only;
                                sub_nx*nz <= 64; no general spaces, downscaling or
                                allocation-free step (ENOTSUP). */
    double lz;               /* z extent when nz >= 1; > 0 */
} rmrcm_params;

/* Fill *p with defaults (alpha 1, FP64, unit square, device 0); the
 * geometry fields are zeroed and must be set by the caller. */
void rmrcm_default_params(rmrcm_params* p);

/* Device memory plan of a context with these parameters, in bytes: every
 * array rmrcm_setup would allocate (basis, factor store, traces and merge
 * workspaces of every level, inputs, outputs; the surrogate network of the
 * learned mode, which allocates its own, is not included).  Host arithmetic
 * only: no device is needed.  Returns the status validation would. */
int rmrcm_plan_bytes(const rmrcm_params* prm, uint64_t* bytes);

/* Build a context: every step that depends on the permeability and on the
 * boundary-condition TYPES only (they enter the local operators):
 * Robin parameters, the factorisation of every subdomain's local system,
 * the multiscale basis (one local solve per interface segment side,
 * Section 2.1 basis problems; one pair of bases per segment collapses to
 * one in the MuMM setting of Section 4), and the upward sweep of interface
 * merges of Algorithm 1 for the basis columns (LU factors and coefficient
 * matrices of every pair, Section 3.2 and its Remark).
 *   perm:    nx*ny permeabilities, finite and > 0 (host or device).
 *   bc_type: 2*nx + 2*ny boundary-face types (host or device).
 *   out:     receives the new context (owned by the library; release with
 *            rmrcm_destroy).
 * Errors: EINVAL (geometry, K <= 0 or not finite), ENOTSUP (sub_nx not
 * supported), ENOMEM, EDEVICE, ESINGULAR. */
int rmrcm_setup(const rmrcm_params* prm, const double* perm,
                const int8_t* bc_type, rmrcm_ctx** out);

/* Recompute every permeability-dependent quantity of an existing context
 * for a new permeability field of the same geometry (the work of
 * rmrcm_setup without its allocations and table building): Robin
 * parameters, local factorisations, basis and the upward merges.
 *   perm: nx*ny permeabilities, finite and > 0 (host or device).
 * Asynchronous: returns once the work is enqueued on the context's stream
 * (perm must stay valid until that work has run).  Errors found on the
 * device (a permeability <= 0 or not finite: EINVAL; a singular merge:
 * ESINGULAR) are returned by the next rmrcm_sync, or by rmrcm_solve when
 * that call waits for the stream (host outputs, or no caller stream set);
 * the context then holds no valid factorisation until the next successful
 * refactor.
 * Errors returned directly: EINVAL (ctx or perm NULL), EDEVICE. */
int rmrcm_refactor(rmrcm_ctx* ctx, const double* perm);

/* Wait for every call enqueued on the context's stream and return the
 * status that an asynchronous rmrcm_refactor left (OK, EINVAL, ESINGULAR),
 * or EDEVICE. */
int rmrcm_sync(rmrcm_ctx* ctx);

/* Downscaling (Section 4 leaves the recovery of fine-scale conservation
 * across the skeleton to downscaling methods): from an MRCM solution of
 * this context's problem (pressure ny*nx and the four one-sided outward
 * fluxes 4*ny*nx, as rmrcm_solve returns them) and the same source (NULL:
 * zero) and bc_value, a pressure and a flux that are single-valued on every
 * face and conservative in every cell.  Each fine skeleton face takes the
 * mean of its two one-sided fluxes, (F_a - F_b) / 2 outward from a; every
 * subdomain's fine problem is solved again (FP64, band Cholesky of the
 * local matrix without Robin terms) with these fluxes prescribed on its
 * skeleton faces and the outer data; a subdomain with no Dirichlet face
 * takes the input's mean pressure over its cells.  Interior fluxes come
 * from the new pressure by the two-point law.  Arrays host or device; the
 * call waits for its work.  The first call allocates a second factor store
 * and staging (not part of rmrcm_plan_bytes; the memory cap applies).
 * 2D contexts with the MuMM spaces only (ENOTSUP otherwise).
 * Errors: EINVAL, ENOMEM, EDEVICE, ESINGULAR, ENOTSUP. */
int rmrcm_downscale(rmrcm_ctx* ctx, const double* source, const double* bc_value, const double* pressure,
                    const double* flux, double* pressure_out, double* flux_out);

/* Mixed modes: the refinement tolerance and pass count of later setups
 * (rmrcm_refactor, rmrcm_step) and solves, in place of those the context
 * was built with (rmrcm_params.ir_tol, ir_max_iter; same meaning).  The
 * subdomains whose particular refinement does not reach ir_tol within
 * ir_max_iter passes are solved again in FP64 (counted in the stats as
 * fp64_particular_fallback_subdomains).  RMRCM_ENOTSUP for an FP64 context,
 * RMRCM_EINVAL for ir_tol <= 0 or ir_max_iter < 1.  A captured step graph
 * is dropped (captured again by the next step). */
int rmrcm_set_refinement(rmrcm_ctx* ctx, double ir_tol, int32_t ir_max_iter);

/* rmrcm_refactor(perm) followed by rmrcm_solve(source, bc_value, pressure,
 * flux) as one unit, with the same arguments and results up to rounding.
 * When every array is in device memory the whole step is captured once as a
 * HIP graph of one chain and replayed, the kernels reading the caller's
 * arrays and writing pressures and fluxes in place; the graph is captured
 * again when any pointer differs from the previous call's.  FP64 contexts:
 * the particular problem (Section 2.1) is solved beside the basis in the
 * local setup and its column eliminated with the basis columns in every
 * merge (Section 3.2).  Mixed modes: the setup and the solve, their
 * refinement loops running on the device.  The phase timers of
 * rmrcm_get_stats keep the values of the last refactor or solve run outside
 * such a graph.  Asynchronous on a stream set with rmrcm_set_stream (device
 * errors, including incompatible all-Neumann data, are returned by
 * rmrcm_sync); otherwise waits.  Host arrays: exactly rmrcm_refactor +
 * rmrcm_solve.
 * Errors: those of rmrcm_refactor and rmrcm_solve. */
int rmrcm_step(rmrcm_ctx* ctx, const double* perm, const double* source, const double* bc_value,
               double* pressure, double* flux);

/* enabled = 0: rmrcm_step runs the same single chain of kernels as its graph
 * (for an FP64 context with device arrays), enqueued launch by launch, and
 * the phase timers of rmrcm_get_stats record it (setup: beta, the local
 * setup with the particular problem, the merges with the particular column;
 * solve: the top's particular column, the downward pass, the
 * reconstruction).  enabled = 1 (the default): the captured graph.  For
 * timing and testing; results are the same either way.
 * Errors: EINVAL (ctx NULL). */
int rmrcm_set_step_graph(rmrcm_ctx* ctx, int enabled);

/* ---- Allocation-free step ----------------------------------------------
 * For callers that cannot allocate device memory: serving loops and
 * harnesses that forbid hipMalloc / hipFree, or run under a fixed device
 * memory budget.  rmrcm_setup followed by rmrcm_step for one FP64 problem,
 * with no context and no device allocation: every device array of the step
 * (Robin parameters, factor store, basis, particular solutions, traces,
 * merge blocks and coefficients, level tables, flags) is carved from a
 * fixed scratch of RMRCM_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on from the loading of its code until the process
 * ends.  Same kernels and results as rmrcm_step of an FP64 context.
 *   prm:       as for rmrcm_setup; precision must be RMRCM_FP64 (else
 *              ENOTSUP).
 *   perm, source (NULL = zero), bc_value, pressure, flux: DEVICE pointers
 *              with the layouts of rmrcm_setup / rmrcm_solve (EINVAL for a
 *              host pointer); the caller owns them.
 *   bc_type:   host or device (read synchronously for validation).
 *   hip_stream: the stream that runs the step (NULL: the null stream).
 * Synchronous: returns when the stream has finished the step, with the
 * status of the device checks (EINVAL: a permeability <= 0 or not finite,
 * or incompatible all-Neumann data; ESINGULAR).  Not capturable in a graph
 * (it waits for its stream).  Calls on one device are serialised by the
 * library (a lock per device); the scratch keeps the last call's contents
 * and every call clears what must start at zero.  ETOOBIG, before any
 * device work, when the problem's arrays exceed the scratch (an FP64 step
 * needs about (8 sub_nx + 8 R + 24) bytes per cell plus the merge levels,
 * R = 2 (sub_nx + sub_ny) / seg: 1024^2 cells with 32^2 subdomains and
 * 8-cell segments fit). */
#define RMRCM_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
int rmrcm_step_noalloc(const rmrcm_params* prm, const double* perm, const int8_t* bc_type,
                       const double* source, const double* bc_value, double* pressure,
                       double* flux, void* hip_stream);

/* Solve for one right-hand side: the particular local solutions (source
 * and outer boundary data, additive split of Section 2.1), their columns
 * through the merges, the top interface solve, the downward propagation of
 * interface values and the final reconstruction of cell pressures and face
 * fluxes (eq. final).  Then up to two steps of iterative refinement of the
 * interface data, decided on the device: when the residual of eq. 13.2 or
 * eq. 14.2 of some segment, computed from the reconstructed one-sided
 * fluxes and the Robin data and divided by the segment's Robin face
 * conductances, exceeds 1e-13 times the largest |pressure| or |Robin
 * datum| next to the skeleton, the residual is taken through the merges
 * and the downward pass once more and the correction added (the explicit
 * inverses of the merges lose digits when large alpha makes the interface
 * blocks ill conditioned; at alpha near 1 no step runs).
 *   source:   nx*ny cell-integrated sources, or NULL for zero.
 *   bc_value: 2*nx + 2*ny values matching the setup's bc_type.
 *   pressure: out, nx*ny.     flux: out, 4*nx*ny (layout above).
 * With no Dirichlet face the pressure is fixed by a zero-mean gauge
 * (requires sum(source) + sum(Neumann values) = 0 within round-off,
 * otherwise EINVAL).  On a caller stream (rmrcm_set_stream) device outputs
 * are complete when that stream completes; host outputs on return. */
int rmrcm_solve(rmrcm_ctx* ctx, const double* source, const double* bc_value,
                double* pressure, double* flux);

/* Interface values of the last solve: U (normal flux density along the
 * global normal) and P (pressure) per segment, nseg doubles each, in the
 * documented segment order.  Host or device pointers. */
int rmrcm_get_interface(rmrcm_ctx* ctx, double* U, double* P);

/* Number of interface segments and of finest-level local solves
 * (basis + particular, the Table 3 count). */
int rmrcm_counts(const rmrcm_ctx* ctx, int64_t* nseg, int64_t* nlocal);

/* Run all further work of this context on the caller's hipStream_t
 * (e.g. torch.cuda.current_stream().cuda_stream).  NULL restores the
 * library's own stream. */
int rmrcm_set_stream(rmrcm_ctx* ctx, void* hip_stream);

/* JSON object with per-phase device times of the last setup and solve
 * (milliseconds, from HIP events recorded on the context's stream; waits
 * for those events), workspace bytes and counters (among them the
 * interface residual before the refinement, the steps it ran and the
 * residual after the first; the subdomains redone in FP64 by setup and
 * solve in the mixed modes).  Writes at most cap
 * bytes including the terminating NUL; returns the length it needs, or a
 * negative error. */
int rmrcm_get_stats(const rmrcm_ctx* ctx, char* json, size_t cap);

/* Release the context and all device memory it owns.  NULL is ignored. */
void rmrcm_destroy(rmrcm_ctx* ctx);

/* Static message for a status code. */
const char* rmrcm_strerror(int status);

/* Time the candidate column tiles (16 or 32 columns per workgroup; 32 reuses
 * each loaded block of the merge for two 16-column tiles) of the
 * interface-merge products of every level of this context on its own
 * shapes and keep the fastest; choices are cached per merge shape (gamma
 * length, parent slots, merges per level) for the process.  Results do not
 * depend on the choice (each column is computed the same way).  Runs on
 * the context's stream and waits for it.  Errors: EINVAL, EDEVICE. */
int rmrcm_autotune(rmrcm_ctx* ctx);

/* ---- Ensembles: many independent problems on one device ----------------
 * Members may differ in grid, subdomain size, segment length, boundary
 * types and precision.  Every member is an ordinary context (set up by
 * rmrcm_setup); the batch enqueues the members' work on a pool of streams,
 * largest member first, so that small members fill the device together.
 * Every member's permeability-dependent work and solve are each captured
 * once as a HIP graph and replayed (the refinement loops of mixed-precision
 * members run on the device, without host waits).
 * All-Neumann members check the compatibility of their data on the device
 * (EINVAL at the next rmrcm_batch_sync when violated). */
typedef struct rmrcm_batch rmrcm_batch;

/* Build a batch of `count` members; prms[i], perms[i] (nx*ny, host or
 * device), bc_types[i] as for rmrcm_setup.  autotune != 0 runs
 * rmrcm_autotune on every member and picks the number of pool streams
 * (1, 2, 4, 8 or 16) by timing a full refactor + solve pass of the batch;
 * otherwise 4 streams.  All members must use the same device and be 2D
 * problems (nz = 0; ENOTSUP otherwise).
 * Errors: those of rmrcm_setup for the first failing member, EINVAL,
 * ENOMEM, EDEVICE, ENOTSUP. */
int rmrcm_batch_create(int32_t count, const rmrcm_params* prms, const double* const* perms,
                       const int8_t* const* bc_types, int32_t autotune, rmrcm_batch** out);

/* rmrcm_refactor for every member (perms: count pointers).  Asynchronous;
 * device-detected errors are returned by rmrcm_batch_sync.  Host arrays are
 * copied into the member's pinned buffers before the call returns (they
 * may be reused at once); device arrays are read in stream order. */
int rmrcm_batch_refactor(rmrcm_batch* b, const double* const* perms);

/* rmrcm_solve for every member: sources (count pointers, or NULL for all
 * zero; an entry may be NULL), bc_values, pressures (nx*ny) and fluxes
 * (4*nx*ny) per member, host or device.  Asynchronous: outputs are
 * complete after rmrcm_batch_sync (host outputs are copied from the
 * member's pinned buffers by that call, or by the next rmrcm_batch_solve). */
int rmrcm_batch_solve(rmrcm_batch* b, const double* const* sources, const double* const* bc_values,
                      double* const* pressures, double* const* fluxes);

/* Wait for all enqueued batch work; status (count entries, may be NULL)
 * receives each member's status; returns the first non-OK one. */
int rmrcm_batch_sync(rmrcm_batch* b, int32_t* status);

/* JSON: members, pool streams, graph-captured members, cells, local
 * solves, device bytes, last refactor / solve times (ms, from events on
 * the batch's master stream) and the merge column tiles per member and
 * level.  Returns the length needed including the terminator. */
int rmrcm_batch_get_stats(rmrcm_batch* b, char* json, size_t cap);

/* Training pairs for the local-basis surrogate from a context's last
 * setup (square subdomains only, else ENOTSUP): features (device, FP32
 * [nsub][2][S][S], as the learned mode computes them), basis (host or
 * device, FP64 [nsub][R][S*S], may be NULL: the exact local basis),
 * interior (host [nsub], may be NULL: 1 when every boundary segment of the
 * subdomain is a Robin segment).  Waits for the context's stream. */
int rmrcm_export_local(rmrcm_ctx* ctx, float* features, double* basis, int32_t* interior);

/* Learned mode: the residual gate of the last setup, per subdomain (mx*my
 * host entries in the order of the subdomains, J * mx + I; either pointer
 * may be NULL): residual[s] = max over basis columns a of
 * |A y_a - e_a|_2 / |e_a|_2 for the network's prediction y (FP64 residual of
 * the local Robin system), +inf for subdomains with a face on the outer
 * boundary (not predicted); accepted[s] = 1 when residual[s] <= gate_tol.
 * Waits for the context's stream.  Errors: EINVAL (not a learned context),
 * ESTATE (no setup yet), EDEVICE. */
int rmrcm_get_gate(rmrcm_ctx* ctx, double* residual, int32_t* accepted);

/* Release every member and the batch's streams and graphs. */
void rmrcm_batch_destroy(rmrcm_batch* b);

/* ---- Local-basis surrogate network -------------------------------------
 * A small convolutional network mapping a subdomain's input features
 * (2 channels of S x S: the centred log-permeability, and on boundary cells
 * the log Robin parameter of the face's segment plus the mean
 * log-permeability) to its R local basis fields, the solutions of the basis
 * problems of Section 2.1 (R x S x S).  L 3x3 convolution layers of width
 * C with zero padding and ReLU between them, plus a learned mean field per
 * output.  FP32 compute and accumulation; convolution weights enter in
 * bfloat16 (round to nearest even of FP32 master weights).  Parameter
 * vector: per layer W [co][ci][3][3] then b [co]; then the mean field
 * [R][S][S].  Feature, input and output arrays are device pointers,
 * [n][channel][j][i] row-major, FP32.  Training is deterministic (fixed
 * reduction order). */
typedef struct rmrcm_cnn rmrcm_cnn;

/* S in {8, 16, 32}; 1 <= C <= 32; 2 <= L <= 16; 1 <= R <= 32; max_batch:
 * largest batch of a forward / training call.  Parameters start at zero:
 * set them with rmrcm_cnn_set_params.  Errors: EINVAL, ENOMEM, EDEVICE. */
int rmrcm_cnn_create(int32_t S, int32_t C, int32_t L, int32_t R, int32_t max_batch, int32_t device,
                     rmrcm_cnn** out);
int rmrcm_cnn_num_params(const rmrcm_cnn* net, int64_t* n);
/* Caller stream (NULL: the network's own).  Calls below are ordered on it. */
int rmrcm_cnn_set_stream(rmrcm_cnn* net, void* hip_stream);
/* Host FP32 parameter vector in / out; setting resets the Adam state.
 * EINVAL for non-finite values. */
int rmrcm_cnn_set_params(rmrcm_cnn* net, const float* theta);
int rmrcm_cnn_get_params(rmrcm_cnn* net, float* theta);
/* y[nb][R][S][S] = network(x[nb][2][S][S]); 1 <= nb <= max_batch. */
int rmrcm_cnn_forward(rmrcm_cnn* net, int32_t nb, const float* x, float* y);
/* Mean squared error against t[nb][R][S][S] and its gradient with respect
 * to every parameter (through the rounded weights); loss (host, may be
 * NULL) and grad (host, np values, may be NULL) are filled when the call
 * returns. */
int rmrcm_cnn_loss_grad(rmrcm_cnn* net, int32_t nb, const float* x, const float* t, double* loss,
                        float* grad);
/* loss_grad followed by one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected) of the master parameters with learning rate lr; loss
 * (host) may be NULL, then the call does not wait for the device. */
int rmrcm_cnn_train_step(rmrcm_cnn* net, int32_t nb, const float* x, const float* t, float lr,
                         double* loss);
/* Binary file: "RMRCMCNN", int32 S, C, L, R, int64 np, np FP32 parameters. */
int rmrcm_cnn_save(rmrcm_cnn* net, const char* path);
int rmrcm_cnn_load(const char* path, int32_t max_batch, int32_t device, rmrcm_cnn** out);
void rmrcm_cnn_destroy(rmrcm_cnn* net);

#ifdef __cplusplus
}
#endif

#endif /* RMRCM_H */
