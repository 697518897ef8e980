/*
 * ovfem.h -- C ABI of libovfem, an MI355X (gfx950) explicit elastic-wave stepper on
 * the low-ordered orthogonal voxel finite element (OVFEM) of arXiv 2404.13683.
 *
 * What the library computes (all citations are to that paper):
 *   - the element-by-element stiffness product f = K u over cubic voxel elements,
 *     K_e = h (lam_e K_lam + mu_e K_mu), where K_lam, K_mu are the fixed reference
 *     matrices of the OVFEM element (Sec. 2, Eq. (5) with the Heaviside displacement
 *     basis of Eq. (7) and the stress basis of Eq. (8)); 256 K_lam and 128 K_mu are
 *     integer matrices with entries inside the INT8 range;
 *   - fused with the central-difference update with the exactly diagonal OVFEM mass
 *     (Sec. 2, Eqs. (3) and (6)):
 *         u^{n+1} = 2 u^n - u^{n-1} + dt^2 M^{-1} (F^n - K u^n),
 *     fixed DOFs held at zero;
 *   - in two precisions: OVFEM_FP64 evaluates the element products in FP64; the INT8
 *     forms split u into M = 8 INT8 digit slices of a 62-bit fixed-point value under a
 *     per-tile power-of-two exponent, run the digit products on the matrix cores and
 *     recombine them into FP64 (Sec. 2, Eqs. (10)-(17), hierarchical FP64-INT64-INT8
 *     form); everything outside the digit products is FP64 (Sec. 3).  Two matrix-core
 *     forms give bitwise-identical results: OVFEM_INT8 runs int8 matrix cores with
 *     INT32 accumulation; OVFEM_INT8_BF16 accumulates two digits per FP32 accumulator
 *     on bf16 matrix cores (every operand and partial sum is an integer that bf16 and
 *     FP32 represent exactly).
 *   - OVFEM_FP64_SF evaluates the same element products in FP64 without the dense
 *     24 x 24 matrices: the octant basis makes every psi-weighted displacement gradient
 *     of Eq. (5) a scaled Walsh coefficient of the 8 corner values, so K_e u_e is two
 *     8-point butterflies around a small stress evaluation (~250 instead of 2304 flops
 *     per element).  A stronger FP64 baseline than the dense "as is" form of Sec. 3.
 *     The trilinear element (ovfem_set_element) has the same factorisation with other
 *     weights of the strain moments, so OVFEM_FP64_SF runs it as well.
 *
 * Grid layout (shared by every array argument):
 *   elements e = i + nx (j + ny k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz;
 *   nodes    n = i + (nx+1) (j + (ny+1) k), 0 <= i <= nx, ...;  z points up;
 *   element e spans nodes i..i+1, j..j+1, k..k+1; voxel edge h.
 *   Nodal vectors are [node][3] float64 (x, y, z components interleaved).
 *
 * Pointers: arguments documented as HOST are ordinary CPU memory; arguments
 * documented as DEVICE are GPU memory on the solver's device (for example the
 * data_ptr() of a torch tensor).  Uploads copy: the caller keeps ownership of every
 * buffer it passes and may free it when the call returns.  The solver owns all of its
 * device state.  All GPU work is enqueued on the stream given at creation; calls that
 * return data to the host, and ovfem_synchronize, wait for that stream.  Calls that
 * allocate, copy or launch return OVFEM_ESTATE when the current HIP device is not the
 * one the solver was created on (the library never switches devices itself).
 *
 * Errors: every call returns an ovfem_status (0 = success, negative = failure) and
 * never throws.  On failure the call has no effect on the solver, and
 * ovfem_last_error() returns a message for the calling thread.
 */
#ifndef OVFEM_H
#define OVFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ovfem_status;
#define OVFEM_OK 0
#define OVFEM_EINVAL (-1)  /* invalid argument: size, index, range, null pointer */
#define OVFEM_ENOMEM (-2)  /* device or host allocation failed */
#define OVFEM_EDEVICE (-3) /* HIP runtime or kernel launch error */
#define OVFEM_ESTATE (-4)  /* call not valid in the solver's current state */

/* element type (ovfem_set_element) */
#define OVFEM_ELEMENT_OVFEM 0     /* the orthogonal voxel element of Sec. 2 (default) */
#define OVFEM_ELEMENT_TRILINEAR 1 /* the conventional lumped trilinear voxel element ("VFEM") */

/* precision of the element products */
#define OVFEM_FP64 0
#define OVFEM_INT8 1      /* INT8 digit slices, int8 matrix cores, INT32 accumulation */
#define OVFEM_INT8_BF16 2 /* INT8 digit slices, bf16 matrix cores, exact FP32 digit-pair sums */
#define OVFEM_FP64_SF 3   /* FP64, the element product sum-factorised */

/* limits */
#define OVFEM_MAX_SHOTS 4096 /* shots per solver */
#define OVFEM_MAX_BATCH 4096 /* solvers per batch */
#define OVFEM_NOALLOC_SCRATCH_BYTES (1 << 20) /* fixed device array of ovfem_batch_step_noalloc */

typedef struct ovfem_solver ovfem_solver;
typedef struct ovfem_batch ovfem_batch;

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t ovfem_version(void);

/* Message describing the last failed call on this thread ("" if none).  The string
 * stays valid until the next library call on the same thread. */
const char* ovfem_last_error(void);

/* Create a solver for an nx x ny x nz voxel grid of edge h (> 0) on the current HIP
 * device, stepping n_shots (1..OVFEM_MAX_SHOTS) independent wavefields of the same
 * model at once (one per shot; every step of every shot runs in one kernel launch).
 * stream is a hipStream_t (NULL = the legacy default stream); all work is enqueued on
 * it.  precision is OVFEM_FP64, OVFEM_INT8, OVFEM_INT8_BF16 or OVFEM_FP64_SF.
 * Device memory: 2 n_shots nodal vectors + 16 bytes per element + 8 per node.
 * EINVAL for non-positive sizes, h <= 0, unknown precision, n_shots out of range,
 * 2^31 or more nodes, or 2^32 / 24 or more nodes in one z plane (the kernels use 32-bit
 * node ids and in-plane byte offsets); ENOMEM if the device buffers do not fit. */
ovfem_status ovfem_create(ovfem_solver** out, int64_t nx, int64_t ny, int64_t nz, double h,
                          int32_t n_shots, int32_t precision, void* stream);

/* Free every device buffer of the solver (waits for its stream).  NULL is accepted. */
ovfem_status ovfem_destroy(ovfem_solver* s);

/* Switch the precision of the element products (OVFEM_FP64 / OVFEM_INT8 / OVFEM_INT8_BF16 /
 * OVFEM_FP64_SF).  EINVAL for OVFEM_INT8_BF16 while the stage count (ovfem_set_stages)
 * is not 8. */
ovfem_status ovfem_set_precision(ovfem_solver* s, int32_t precision);

/* Per-element material, HOST arrays of nx*ny*nz float64: Lame lam, shear modulus mu,
 * density rho; solid (nullable, uint8, 0 = removed voxel) marks voxels that are
 * absent.  The nodal mass is the sum of rho h^3 / 8 over the solid voxels touching a
 * node (Sec. 2, Eq. (6): the OVFEM mass is diagonal without approximation); nodes with
 * no mass do not move.  EINVAL if mu <= 0, lam + 2 mu / 3 <= 0, rho <= 0 or a value is
 * not finite in a solid voxel.  Resets the wavefield and traces. */
ovfem_status ovfem_set_model(ovfem_solver* s, const double* lam, const double* mu, const double* rho,
                             const uint8_t* solid);

/* Fixed nodes, HOST array of (nx+1)(ny+1)(nz+1) uint8 (nullable = none fixed); a
 * nonzero entry holds all three DOFs of that node at zero. */
ovfem_status ovfem_set_fixed_nodes(ovfem_solver* s, const uint8_t* fixed);

/* Time step dt (> 0).  EINVAL if dt exceeds the element-wise stability bound
 * 2 / sqrt(max eigenvalue of K_e / (rho_e h^3 / 8)) over solid voxels, which bounds
 * the central-difference limit of the assembled system from below (with Rayleigh
 * damping, the bound of ovfem_set_damping). */
ovfem_status ovfem_set_dt(ovfem_solver* s, double dt);

/* Point forces, HOST arrays: n sources at nodes node[i] (flat node id), component
 * comp[i] in {0, 1, 2}, shot[i] (nullable = all 0; must be < n_shots), with force
 * wavelet[i * nt + t] applied at step t (time t dt); no force after step nt - 1.
 * n = 0 removes all sources.  EINVAL for out-of-range indices. */
ovfem_status ovfem_set_sources(ovfem_solver* s, int32_t n, const int64_t* node, const int32_t* comp,
                               const int32_t* shot, const double* wavelet, int64_t nt);

/* Receivers, HOST array of n flat node ids (the same for every shot).  After step t
 * (t < nt_max) the three components of u^{t+1} at each receiver are recorded.  Clears
 * the recorded traces.  EINVAL for out-of-range ids or nt_max < 0. */
ovfem_status ovfem_set_receivers(ovfem_solver* s, int32_t n, const int64_t* node, int64_t nt_max);

/* u^0 = u^{-1} = 0, step counter 0, traces cleared. */
ovfem_status ovfem_reset(ovfem_solver* s);

/* Enqueue n >= 0 time steps on the solver's stream (asynchronous).  Requires the
 * model and dt.  Step t uses the force at step t and records receivers into slot t
 * while t < nt_max. */
ovfem_status ovfem_step(ovfem_solver* s, int64_t n);

/* f = K u for one nodal vector with the solver's current precision and model, no
 * boundary conditions applied (rows of fixed nodes are included).  u and Ku are
 * DEVICE arrays of (nx+1)(ny+1)(nz+1)*3 float64; they must not overlap.  The
 * wavefield state of the solver is not touched.  Asynchronous on the stream. */
ovfem_status ovfem_matvec(ovfem_solver* s, const double* u, double* Ku);

/* Copy u^n (which = 0) or u^{n-1} (which = 1) of every shot into the DEVICE array out
 * (n_shots (nx+1)(ny+1)(nz+1)*3 float64, [shot][node][3]).  Waits for the stream. */
ovfem_status ovfem_get_wavefield(ovfem_solver* s, int32_t which, double* out);

/* Replace the state by (u^n = un, u^{n-1} = unm1) at step counter `step` (>= 0).
 * DEVICE arrays as in ovfem_get_wavefield (all shots).  Resumes a run from a saved
 * state. */
ovfem_status ovfem_set_wavefield(ovfem_solver* s, const double* un, const double* unm1, int64_t step);

/* Recorded traces into the DEVICE array out, float64 laid out
 * [shot][receiver][component][t] with t < nt_max; slots of steps not yet run are 0.
 * Waits for the stream. */
ovfem_status ovfem_get_traces(ovfem_solver* s, double* out);

/* Current step counter (number of steps taken since reset / set_wavefield). */
ovfem_status ovfem_get_step(ovfem_solver* s, int64_t* step);

/* Checkpointing of forward runs for ovfem_adjoint: allocates room for max_steps steps
 * and, from now on, stores (u^s, u^{s-1}) of every shot on the device at every step s
 * that is a multiple of `every` (counted from reset).  every = 0 disables it.  Resets the
 * wavefield (as ovfem_reset).  Device memory: 2 (max_steps / every + 1) nodal vectors
 * per shot; with every = 1, max_steps + 2 per shot: the forward run then writes each new
 * state straight into its slot of one tape u^{-1}, u^0, ..., and the adjoint recomputes
 * nothing.  ENOMEM if it does not fit (the solver keeps its state and its earlier
 * checkpointing). */
ovfem_status ovfem_set_checkpointing(ovfem_solver* s, int64_t every, int64_t max_steps);

/* Gradient of a receiver misfit with respect to the per-element lam and mu, by the
 * discrete adjoint of the central-difference recursion (Sec. 2, Eq. (3)).  With
 * A = dt^2 M^{-1} (zero on fixed DOFs), R the receiver restriction and r^n = dJ/d(traces
 * at step n), the adjoint states obey
 *     w^{N+1} = w^{N+2} = 0,   w^m = 2 w^{m+1} - w^{m+2} + A (R^T r^{m-1} - K w^{m+1}),
 * which is the forward step with the residual injected at the receivers, and
 *     g_lam[e] = - sum_m h (w_e^m)^T K_lam u_e^{m-1}   (g_mu likewise with K_mu).
 * With Rayleigh damping (ovfem_set_damping) the adjoint of the damped recursion takes
 * the same form as the damped forward step (w = A lambda with A = dt^2 M^{-1} / (1 +
 * alpha dt/2)) and u^{m-1} in the gradient becomes the staged (1+b) u^{m-1} - b u^{m-2},
 * b = beta / dt.
 * Requires a forward run of N >= 1 steps from reset with checkpointing enabled, the same
 * precision, model and dt, and receivers recording every step (N <= nt_max).
 * residual: DEVICE float64 [shot][receiver][component][nt_max] (the layout of the traces;
 * entries t >= N are ignored), e.g. traces - observed for J = 1/2 |traces - observed|^2.
 * g_lam, g_mu: DEVICE float64 arrays of nx*ny*nz, overwritten (0 for removed voxels):
 * the gradient of a misfit summed over the shots, i.e. the shots' gradients summed (each
 * element's terms added step by step, shot by shot within a step).  The adjoint states of
 * all shots advance in one launch per step, as the forward steps do.
 * Each checkpoint segment is recomputed forward (bitwise identical: the kernels are
 * deterministic; every - 1 steps per segment, none with every = 1, which trades two
 * stored nodal vectors per step for the recompute) and then stepped backward; the
 * adjoint steps use the solver's precision for K.  The wavefield state and traces of the forward run are unchanged.
 * Synchronises the stream.  ESTATE if the preconditions do not hold. */
ovfem_status ovfem_adjoint(ovfem_solver* s, const double* residual, double* g_lam, double* g_mu);

/* Element type: OVFEM_ELEMENT_OVFEM (default) or OVFEM_ELEMENT_TRILINEAR, the
 * conventional voxel element the paper compares against (Sec. 2: trilinear basis,
 * integrated exactly by 2x2x2 Gauss points; the same lumped mass rho h^3 / 8 per node
 * and element).  Its matrices scaled by 72 are integer matrices in -32..32, so every
 * precision runs it (FP64 with the matrices as constants, the INT8 forms with them as
 * A operands, material scaled by h lam / 72, h mu / 72; OVFEM_FP64_SF in its
 * sum-factorised form).  Clears the model and dt (set
 * them again) and resets the wavefield.  EINVAL for an unknown element. */
ovfem_status ovfem_set_element(ovfem_solver* s, int32_t element);

/* Rayleigh damping C = alpha M + beta K (alpha, beta >= 0; both 0 = undamped, the
 * default).  The paper's experiment (Sec. 3) uses Rayleigh damping without printing its
 * time discretization; the step taken here centres the mass-proportional velocity and
 * takes the stiffness-proportional one backward, so it stays explicit with one K
 * product:
 *     (1 + alpha dt/2) u^{n+1} = 2 u^n - (1 - alpha dt/2) u^{n-1}
 *                               + dt^2 M^{-1} (F^n - K (u^n + (beta/dt)(u^n - u^{n-1}))).
 * Its stability bound on dt shrinks to w_max^2 dt (dt + 2 beta) <= 4 (checked against
 * the element bound of w_max, as ovfem_set_dt does).  A damped solver keeps a third
 * nodal vector per shot and does not replay captured graphs; damped and undamped
 * solvers cannot share a batch.  ovfem_adjoint differentiates the damped recursion.  Resets the wavefield.  EINVAL for
 * negative or non-finite values, or a dt already set that the new beta makes unstable. */
ovfem_status ovfem_set_damping(ovfem_solver* s, double alpha, double beta);

/* Digit stages M (4..8, default 8) of OVFEM_INT8: u is split under the staging exponent S
 * of its element layer into q = rint(u 2^(8M-2-S)), |q| <= 2^(8M-2), written as M balanced
 * base-256 digits (Sec. 2, Eqs. (16)-(17); the paper's Table 3 compares stage counts).
 * Fewer stages mean fewer matrix-core products and recombination steps at lower accuracy:
 * about 8M - 2 bits relative to the largest of the 17 x 17 x 2 nodes a work-group stages
 * for that layer (M = 4 is about FP32, M = 8 at least FP64).  OVFEM_INT8_BF16 runs M = 8 only (EINVAL otherwise);
 * OVFEM_FP64 ignores the setting. */
ovfem_status ovfem_set_stages(ovfem_solver* s, int32_t stages);

/* Current digit stage count (HOST out-pointer). */
ovfem_status ovfem_get_stages(ovfem_solver* s, int32_t* stages);

/* Launch configuration.  chunk_planes (1..4096): depth, in node planes, of the z-chunk a
 * work-group marches through (the tiling is 15 x 15 node columns by about chunk_planes
 * planes; default 16).  persistent_groups (>= 0): for n_shots > 1, cap on the launch
 * grid, rounded down to a multiple of 8 (0 = one work-group per tile and shot).
 * graph_steps (even, 0..4096; default 0 = never): ovfem_step calls of at least that many
 * steps replay a captured HIP graph of graph_steps steps instead of launching each step
 * (graphs are not used while checkpointing for the adjoint).  Every path gives
 * bitwise-identical results under every setting here (the INT8 staging exponent depends
 * only on the nodes staged for one element layer, not on the chunk depth); only the tile
 * height of ovfem_set_tile_rows changes which nodes a work-group stages together, and with
 * it the last bits of the INT8 forms (their accuracy bound does not change).  Keeps the wavefield state; a changed tiling
 * invalidates a checkpointed forward run.  EINVAL for out-of-range values. */
ovfem_status ovfem_set_tuning(ovfem_solver* s, int32_t chunk_planes, int32_t persistent_groups,
                              int32_t graph_steps);

/* Current launch configuration (HOST out-pointers). */
ovfem_status ovfem_get_tuning(ovfem_solver* s, int32_t* chunk_planes, int32_t* persistent_groups,
                              int32_t* graph_steps);

/* Tile height of the stepper kernels: rows = 16 (16 x 16 elements per work-group of 256
 * threads, 15 x 15 owned node columns; the default) or 32 (16 x 32 elements, 512 threads,
 * 15 x 31 owned node columns: a smaller halo, fewer tiles on grids whose node count per
 * row is just above a multiple of 15).  FP64 results are bitwise the same for both; INT8
 * results depend on the staged blocks (the staging exponent's extent) within the accuracy
 * bound of the staging exponent.  Rebuilds the tile tables (waits for the stream); a
 * checkpointed forward run is invalidated.  EINVAL for other values. */
ovfem_status ovfem_set_tile_rows(ovfem_solver* s, int32_t rows);
ovfem_status ovfem_get_tile_rows(ovfem_solver* s, int32_t* rows);

/* Autotuner: times `steps` (2..100000) plain-launch steps of the solver's own model,
 * sources and precision for each tile height (16 and 32 element rows) and candidate chunk
 * depth (8, 12, 16, 24, 32, 48, 64, 96 planes, each evened out over the chunks it gives)
 * and, for n_shots > 1, grid caps of
 * 0, 2 and 4 work-groups per compute unit, in two passes over all candidates, and keeps
 * the candidate with the fastest of its two times (the first pass also raises the clocks,
 * which would otherwise favour the candidates timed last); it then times graph_steps 0
 * and 64 at that setting and keeps the faster.  The wavefield pair, traces and step counter are
 * restored afterwards; a checkpointed forward run is invalidated.  best_ms_per_step
 * (HOST, nullable) receives the best time per step in milliseconds.  Synchronises the
 * stream.  ESTATE without model and dt. */
ovfem_status ovfem_autotune(ovfem_solver* s, int32_t steps, double* best_ms_per_step);

/* A batch of solvers of uneven grid sizes (and shot counts) stepped together: each
 * ovfem_batch_step step is one kernel launch over the tiles of every shot of every
 * member.  members: HOST array of n (1..OVFEM_MAX_BATCH) distinct solvers created on
 * the same device with the same stream; they must outlive the batch.  The batch holds
 * no wavefield state of its own: members keep theirs and may still be stepped alone. */
ovfem_status ovfem_batch_create(ovfem_batch** out, ovfem_solver* const* members, int32_t n);

/* Free the batch (waits for its stream; the members are untouched).  NULL is accepted. */
ovfem_status ovfem_batch_destroy(ovfem_batch* b);

/* Grid cap of the batched launch, as persistent_groups of ovfem_set_tuning (0 = none). */
ovfem_status ovfem_batch_set_tuning(ovfem_batch* b, int32_t persistent_groups);

/* Replay whole blocks of graph_steps batch steps from a captured HIP graph (a multiple of
 * 6 in 0..4096; 0, the default, launches every step from the host).  A block starts at a
 * batch step that is a multiple of 6 (steps before it, and the remainder, are launched
 * plainly); the graph reads the step base from device memory and is captured again when
 * the batch's argument tables move or its launch shape changes.  Damped batches are not
 * captured.  Results are bitwise those of plain launches.  Waits for the stream. */
ovfem_status ovfem_batch_set_graph(ovfem_batch* b, int32_t graph_steps);

/* Enqueue n >= 0 steps of every member (asynchronous).  Each member advances exactly as
 * ovfem_step(member, n) would (bitwise: the same kernels on the same tiles), from its
 * own step counter.  Members must share one precision (and stage count) and have model and dt set
 * (ESTATE otherwise).  Invalidates the members' checkpointed forward runs. */
ovfem_status ovfem_batch_step(ovfem_batch* b, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ovfem_batch_step with the batch's
 * argument tables in a fixed array of OVFEM_NOALLOC_SCRATCH_BYTES bytes of device memory
 * that the library holds on every device it runs on until the process ends, instead of
 * device buffers it allocates.  It calls no hipMalloc or hipFree.  Results are those of
 * ovfem_batch_step (bitwise: the same kernels on the same tables); asynchronous likewise.
 * The tables take 6 * 248 + 4 bytes per unit (a unit is one shot of one member) plus 4:
 * EINVAL beyond OVFEM_NOALLOC_SCRATCH_BYTES (702 units).  ESTATE unless every member has
 * model and dt set and has stepped since its model, fixed nodes, dt or damping last
 * changed (ovfem_step(member, 0) suffices: it builds the member's dt^2/m table).
 * Every call on one device writes the same array: calls on one stream are ordered, calls
 * on different streams of one device that overlap in time race. */
ovfem_status ovfem_batch_step_noalloc(ovfem_batch* b, int64_t n);

/* Blow-up check: *finite = 1 if every value of the current wavefield pair (u^n, u^{n-1})
 * of every shot is finite, 0 if any is NaN or infinite.  With dt inside the bound that
 * ovfem_set_dt enforces the scheme is stable, so non-finite values come from non-finite
 * inputs (wavefields passed to ovfem_set_wavefield, source wavelets).  finite is HOST
 * memory.  Waits for the stream.  EINVAL for NULL arguments. */
ovfem_status ovfem_check_finite(ovfem_solver* s, int32_t* finite);

/* Wait for all work enqueued by the solver. */
ovfem_status ovfem_synchronize(ovfem_solver* s);

#ifdef __cplusplus
}
#endif

#endif /* OVFEM_H */
