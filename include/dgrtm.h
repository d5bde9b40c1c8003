/*
 * dgrtm: nodal discontinuous-Galerkin reverse-time migration on one AMD Instinct MI355X (gfx950).
 *
 * The C ABI of libdgrtm.so.  It computes what Modave, St-Cyr, Mulder and Warburton,
 * "Nodal Discontinuous Galerkin Simulations for Reverse-Time Migration on GPU Clusters"
 * (arXiv 1506.00907), define:
 *   - the first-order acoustic pressure-velocity system with piecewise-constant rho and c,
 *     a point source f(t) delta(x - x0) in the pressure equation, and free-surface,
 *     transparent (p - rho c n.v = 0) or rigid boundaries (model section, eqs. waveSyst1/2, ABC);
 *   - its nodal DG discretisation on tetrahedra with penalty fluxes (nodal-DG section,
 *     eqs. weakFormP/V, dgLocalSchemeP/U, the appendix);
 *   - multi-rate Adams-Bashforth time stepping on levels Delta t_l = 2^(L-l) Delta t_local
 *     (time-stepping section, eqs. updateAB, updateABcoarse; Alg. 1);
 *   - the RTM procedure: forward source wavefield, backward receiver wavefield with the
 *     recorded data re-injected, and the imaging condition accumulated step by step from the
 *     AB3 dense-output polynomials of both fields (model section, eqs. imageP and imageQ;
 *     imaging section, eq. updateABcorr).
 *
 * Conventions (every entry point):
 *   - Return value: DGRTM_OK (0) or a negative error code; dgrtm_last_error() returns a
 *     thread-local message describing the last failure.
 *   - Host arrays passed in are copied during the call; the caller keeps ownership.
 *   - Device memory is never allocated by the library: every handle that owns device state
 *     works inside a caller-provided device workspace of the size the matching *_bytes query
 *     returns.  The caller keeps that workspace alive until the handle is destroyed.
 *   - Work is enqueued asynchronously on the HIP stream given at dgrtm_mesh_bind.  The time
 *     loop never waits on the host: dgrtm_forward, dgrtm_adjoint, dgrtm_shot_begin,
 *     dgrtm_step_shots, dgrtm_shot_traces and dgrtm_image return once their work is queued.
 *     Calls that copy host arrays to the device (dgrtm_mesh_bind, dgrtm_shot_create), return
 *     host values computed on the device (dgrtm_residual, dgrtm_profile_read) or are test
 *     hooks synchronise that stream.  Handles are not thread-safe.
 *   - Element numbering in every array is the caller's ("user order"); the library reorders
 *     elements internally (finest time level first).
 *   - Units are any consistent set (the tests use km, s, km/s, g/cm^3).
 */
#ifndef DGRTM_H
#define DGRTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dgrtm_status;
#define DGRTM_OK 0
#define DGRTM_ERR_ARG (-1)       /* invalid argument or call order */
#define DGRTM_ERR_WORKSPACE (-2) /* workspace too small (query the *_bytes call) */
#define DGRTM_ERR_MESH (-3)      /* invalid mesh: degenerate element, non-manifold face, bad index */
#define DGRTM_ERR_OUTSIDE (-4)   /* a source or receiver point lies outside the mesh */
#define DGRTM_ERR_HIP (-5)       /* a HIP runtime call failed */

/* boundary types of a boundary face (model section: free surface p = 0, transparent
 * p - rho c n.v = 0; rigid wall n.v = 0) */
#define DGRTM_BC_RIGID 1
#define DGRTM_BC_TRANSPARENT 2
#define DGRTM_BC_FREE 3

/* imaging conditions: classical p_S p_R (eq. imageP) or characteristic q-_S q+_R with
 * q+- = p +- rho c up.v (eqs. imageQ, charact) */
#define DGRTM_IMAGE_PRESSURE 0
#define DGRTM_IMAGE_CHARACTERISTIC 1
/* or'ed into the condition: each own step's contribution by the trapezoid rule dt/2 (S R at both
 * ends of the step; eq. trapRule, its sign read as "+") instead of the exact integral of the two
 * fields' AB3 dense outputs (eq. updateABcorr) */
#define DGRTM_IMAGE_TRAPEZOID 0x100

/* how the source wavefield is made available to the backward run (dgrtm_shot_args.storage):
 *   DGRTM_STORE_CHECKPOINTS  the AB3 state every ckpt_interval global steps, the source field
 *                            recomputed forward segment by segment (memory ~ sqrt(steps))
 *   DGRTM_STORE_BOUNDARY     the paper's strategy (RTM procedure of the model section; section on
 *                            memory transfers): p and n.v at the boundary face nodes after every
 *                            own step, and the final state; the source field is re-simulated
 *                            backward in time (penalties of opposite sign) with these traces as the
 *                            exterior state of every boundary face, beside the receiver field
 *                            (memory ~ steps x boundary faces) */
#define DGRTM_STORE_CHECKPOINTS 0
#define DGRTM_STORE_BOUNDARY 1

/* arithmetic of the element operator products: FP32 MFMA, or split-BF16 MFMA (A x evaluated as
 * A_hi x_hi + A_hi x_lo + A_lo x_hi with A = A_hi + A_lo, x = x_hi + x_lo in bf16, FP32 accumulation).
 * State, update and traces are FP32 in both; the image is accumulated in FP64 in both. */
#define DGRTM_FP32 0
#define DGRTM_SPLIT_BF16 1

/* which wavefield of a shot a test hook addresses */
#define DGRTM_SOURCE_FIELD 0
#define DGRTM_RECEIVER_FIELD 1

typedef struct dgrtm_mesh_s *dgrtm_mesh;
typedef struct dgrtm_shot_s *dgrtm_shot;

/* Message of the last failed call on this thread ("" if none). */
const char *dgrtm_last_error(void);

/*
 * Build the order-N reference element (warp-and-blend nodes, D_r, D_s, D_t, LIFT; nodal-DG
 * section and appendix), the face connectivity and the geometric factors of a tetrahedral mesh.
 *   N          polynomial order, 1..6
 *   vert_xyz   host, n_vert x 3 doubles
 *   elem_vert  host, n_elem x 4 vertex indices; elements with negative volume are re-oriented
 *   face_bc    host, n_elem x 4 boundary types (DGRTM_BC_*) read on boundary faces only, or
 *              NULL to use bc_default everywhere.  Face f of element k is numbered on the
 *              re-oriented element (vertices 2 and 3 swapped where the volume was negative):
 *              faces 0..3 are its local vertex triples (0,1,2), (0,1,3), (1,2,3), (0,2,3)
 * Host work only.  Errors: DGRTM_ERR_ARG, DGRTM_ERR_MESH.
 */
dgrtm_status dgrtm_mesh_create(int N, int64_t n_vert, const double *vert_xyz, int64_t n_elem,
                               const int64_t *elem_vert, const int8_t *face_bc, int bc_default,
                               dgrtm_mesh *out);

/*
 * Set per-element density and velocity and assign multi-rate levels (time-stepping section):
 * dt_k = cfl * l_k / ((N+1)^2 c_k) with l_k the smallest face-to-opposite-vertex distance
 * (validation section), dt_local = min_k dt_k, level l_k the coarsest l in 1..n_levels_max
 * with 2^(L-l) dt_local <= dt_k, levels then raised until face neighbours differ by at most
 * one, and empty coarse levels removed.  n_levels_max = 1 gives single-rate AB3.
 *   rho, c        host, n_elem doubles, > 0
 *   dt_local_out  receives dt_local; n_levels_out receives the number of levels L (NULL ok)
 * Host work only; must precede dgrtm_mesh_bind.  Errors: DGRTM_ERR_ARG.
 */
dgrtm_status dgrtm_set_model(dgrtm_mesh mesh, const double *rho, const double *c, int n_levels_max,
                             double cfl, double *dt_local_out, int *n_levels_out);

/* Device bytes dgrtm_mesh_bind needs: the reference operators (nodal-DG section, appendix),
 * the geometric factors and face connectivity of every element (the per-element and per-face
 * data structures of the implementation section's table), padded per multi-rate level.
 * Host only.  Errors: DGRTM_ERR_ARG (null mesh, or no dgrtm_set_model yet). */
dgrtm_status dgrtm_mesh_bytes(dgrtm_mesh mesh, size_t *bytes);

/*
 * Upload the mesh (the data counted by dgrtm_mesh_bytes: implementation section, data-structure
 * table) into the device workspace dev_ws (>= dgrtm_mesh_bytes, 256-byte aligned)
 * and bind the handle to hip_stream (a hipStream_t; NULL = default stream).
 * Errors: DGRTM_ERR_ARG, DGRTM_ERR_WORKSPACE, DGRTM_ERR_HIP.
 */
dgrtm_status dgrtm_mesh_bind(dgrtm_mesh mesh, void *dev_ws, size_t ws_bytes, void *hip_stream);

/*
 * Export the integer set-up for checking (host arrays, user element order, any may be NULL): the
 * face connectivity and node maps of the nodal-DG section (vmapM/vmapP of the appendix) and the
 * levels of the time-stepping section.
 *   EToE, EToF  n_elem x 4 neighbour element and face (self on a boundary face)
 *   vmapP       n_elem x 4 x Nfp global node id k*Np+n of the matching node on the other side
 *   level       n_elem multi-rate level (1 = coarsest)
 *   sorted_pos  n_elem position of each element in the device order
 */
dgrtm_status dgrtm_export_setup(dgrtm_mesh mesh, int32_t *EToE, int8_t *EToF, int32_t *vmapP,
                                int8_t *level, int64_t *sorted_pos);

/*
 * Element holding each point (host work only): the lowest-numbered element, in user order, whose
 * barycentric coordinates of the point are all >= -1e-12, or -1 for a point outside the mesh.
 * This is the rule dgrtm_shot_create applies to the source and the receivers; the paper leaves
 * open which element takes a point on a face or vertex shared by several (point source of the
 * nodal-DG section, eq. sourceTerm; receivers of the validation section).
 *   xyz   host, n x 3 doubles;  elem  host, n int64 (user element order)
 * Errors: DGRTM_ERR_ARG.
 */
dgrtm_status dgrtm_locate(dgrtm_mesh mesh, int64_t n, const double *xyz, int64_t *elem);

/* Reference operators in FP64 (host, row-major): the differentiation matrices Dr, Ds, Dt
 * (Np x Np) and the lift matrix LIFT (Np x 4 Nfp) of the appendix, and the warp-and-blend node
 * coordinates rst (Np x 3) of the nodal-DG section.  Any pointer may be NULL.
 * Host only.  Errors: DGRTM_ERR_ARG (null mesh). */
dgrtm_status dgrtm_export_operators(dgrtm_mesh mesh, double *Dr, double *Ds, double *Dt, double *LIFT,
                                    double *rst);

/* Sizes of the discretisation: order N, nodes per element Np = (N+1)(N+2)(N+3)/6 and per face
 * Nfp = (N+1)(N+2)/2 (nodal-DG section), elements, number of multi-rate levels L and the finest
 * step dt_local (time-stepping section).  Any pointer may be NULL.  Host only.
 * Errors: DGRTM_ERR_ARG (null mesh). */
dgrtm_status dgrtm_mesh_info(dgrtm_mesh mesh, int *N, int *Np, int *Nfp, int64_t *n_elem, int *n_levels,
                             double *dt_local);

/* Release the host handle (the caller frees the device workspace afterwards).  NULL is ignored. */
void dgrtm_mesh_destroy(dgrtm_mesh mesh);

/* One RTM shot (versioned plain struct: set struct_size = sizeof(dgrtm_shot_args)): the point
 * source and the receiver positions of the RTM procedure (model section), the Ricker wavelet of
 * the validation and RTM sections, the final time and the storage and precision choices. */
typedef struct dgrtm_shot_args {
  int32_t struct_size;
  int32_t has_source;      /* 0: no source term (test runs) */
  double src_xyz[3];
  double f_peak, t_peak, amp; /* Ricker source f(t) = amp (1 - 2 a) exp(-a), a = (pi f_peak (t - t_peak))^2 */
  const float *wavelet;    /* host, optional: f sampled at every local step j*dt_local, j = 0..n_steps;
                              overrides the Ricker when not NULL (length from dgrtm_shot_steps) */
  int64_t n_rec;           /* receivers: pressure recorded at every global step, re-injected backward */
  const double *rec_xyz;   /* host, n_rec x 3 */
  double t_final;          /* rounded up to a whole number of global steps */
  int64_t ckpt_interval;   /* global steps between source checkpoints; 0 = chosen to minimise memory */
  int32_t precision;       /* DGRTM_FP32 or DGRTM_SPLIT_BF16 */
  int32_t storage;         /* DGRTM_STORE_CHECKPOINTS (ckpt_interval applies) or DGRTM_STORE_BOUNDARY */
} dgrtm_shot_args;

/* Number of global steps of a shot (t_final / dt_global rounded up) and local steps per global
 * step, 2^(L-1) (time-stepping section, Alg. 1).  Host only.  Errors: DGRTM_ERR_ARG. */
dgrtm_status dgrtm_shot_steps(dgrtm_mesh mesh, const dgrtm_shot_args *args, int64_t *n_global,
                              int32_t *n_local);

/* Device bytes of a shot: the source and receiver wavefields with their AB3 history (eq.
 * updateAB) and trace copies (eq. updateABcoarse), the FP64 image (eqs. imageP, imageQ), the
 * receiver traces, and by storage: the source checkpoints and segment records, or the boundary
 * traces of every own step, two saved states and one global step of segment records (RTM
 * procedure, model section).  This is the footprint that admission uses.  Host only.
 * Errors: DGRTM_ERR_ARG. */
dgrtm_status dgrtm_shot_bytes(dgrtm_mesh mesh, const dgrtm_shot_args *args, size_t *bytes);

/*
 * Create a shot inside dev_ws (>= dgrtm_shot_bytes): locates the source and receivers (the
 * lowest-numbered element whose barycentric coordinates are all >= -1e-12) and projects the
 * point delta on the element's polynomial space, w = M_k^{-1} l(x0) (eq. sourceTerm).
 * Errors: DGRTM_ERR_ARG, DGRTM_ERR_WORKSPACE, DGRTM_ERR_OUTSIDE, DGRTM_ERR_HIP.
 */
dgrtm_status dgrtm_shot_create(dgrtm_mesh mesh, const dgrtm_shot_args *args, void *dev_ws, size_t ws_bytes,
                               dgrtm_shot *out);

/*
 * Forward source run from rest over [0, t_final] with multi-rate AB3 (time-stepping section,
 * eqs. updateAB and updateABcoarse, Alg. 1; first stage of the RTM procedure in the model
 * section), saving the AB3 state every ckpt_interval global steps in the workspace.  traces_out (device, may be NULL)
 * receives the recorded pressure, n_rec x (n_global + 1) floats, sample g at t = g dt_global.
 */
dgrtm_status dgrtm_forward(dgrtm_shot shot, float *traces_out);

/*
 * Second stage of the RTM procedure (model section): the receiver wavefield runs backward in
 * time from rest at t_final, with the recorded data re-injected at the receivers and the
 * penalty parameter of opposite sign (backward-in-time paragraph of the time-stepping
 * section), and the imaging condition (eq. imageP or imageQ) is accumulated in FP64 from the
 * exact time integral of the product of both fields' AB3 dense outputs over each element's own
 * steps (imaging section, eq. updateABcorr with the weights read as ebar_s and, since the
 * source field is recomputed forward here, the mixed-direction matrix Cmix).
 *   data        device, n_rec x (n_global + 1) floats (linear in time between samples, 0 after t_final)
 *   condition   DGRTM_IMAGE_PRESSURE or DGRTM_IMAGE_CHARACTERISTIC, optionally | DGRTM_IMAGE_TRAPEZOID
 *   up          host, 3 doubles: the "up" unit vector of the characteristic split
 *   g_image_start  image only over [g_image_start dt_global, t_final]; the backward run stops there
 * With DGRTM_STORE_CHECKPOINTS the source wavefield is recomputed forward segment by segment
 * from the checkpoints and paired with the receiver field step by step (the weights Cmix of an
 * integral of one forward and one backward dense output).  With DGRTM_STORE_BOUNDARY it is
 * re-simulated backward from its final state with the recorded boundary traces, in lockstep with
 * the receiver field, and the image takes the both-backward form of eq. updateABcorr (ebar_s,
 * and C as printed); the AB3 history of that backward run at t_final, on which the paper is
 * silent, is extrapolated (third order) from its reversed-time rhs at the global times t_final,
 * t_final - dt_global and t_final - 2 dt_global.  Requires a completed dgrtm_forward.  The image
 * is reset at the start of the call.
 */
dgrtm_status dgrtm_adjoint(dgrtm_shot shot, const float *data, int condition, const double *up,
                           int64_t g_image_start);

/* ---- continuous batching: several shots of one mesh advanced together ---- */

/* phases of a shot's pipeline (dgrtm_shot_state) */
#define DGRTM_PHASE_IDLE 0
#define DGRTM_PHASE_FORWARD 1
#define DGRTM_PHASE_RECOMPUTE 2
#define DGRTM_PHASE_BACKWARD 3
#define DGRTM_PHASE_DONE 4

/*
 * Reset a shot to run its whole RTM pipeline (model section: forward run, backward run with
 * imaging; the paper sums the images of independent shots) through dgrtm_step_shots: the forward run, then the
 * adjoint (segment recompute and backward run with imaging) with the given parameters (as for
 * dgrtm_adjoint).  data = NULL uses the shot's own recorded traces as the data.  Enqueues the
 * state reset only.
 */
dgrtm_status dgrtm_shot_begin(dgrtm_shot shot, const float *data, int condition, const double *up,
                              int64_t g_image_start);

/*
 * Advance each of n shots (all on one mesh and bound to one stream) by n_global global steps of
 * its pipeline (each step as in dgrtm_forward / dgrtm_adjoint: Alg. 1 with eqs. updateAB,
 * updateABcoarse and updateABcorr); shots that are idle or done are skipped.  Shots that are at the same step mode
 * (forward, recompute or backward-with-image) and precision share one kernel launch per local
 * step (up to 8 per launch), each with its own time index, sources and buffers.  Asynchronous.
 */
dgrtm_status dgrtm_step_shots(dgrtm_shot *shots, int n, int64_t n_global);

/* Copy the shot's recorded pressure at the receivers (RTM procedure, model section; the
 * validation section's receiver traces), n_rec x (n_global + 1) floats, into out (device).
 * Asynchronous.  Errors: DGRTM_ERR_ARG, DGRTM_ERR_HIP. */
dgrtm_status dgrtm_shot_traces(dgrtm_shot shot, float *out);

/* Host-side pipeline state of the RTM procedure (model section): phase (DGRTM_PHASE_*), global
 * steps done and in total.  Host only.  Errors: DGRTM_ERR_ARG. */
dgrtm_status dgrtm_shot_state(dgrtm_shot shot, int *phase, int64_t *steps_done, int64_t *steps_total);

/* The image I(x) of eq. imageP or eq. imageQ (model section) as accumulated by the backward
 * run: copy (accumulate = 0) or add (accumulate = 1, the stack over shots of the model section)
 * the FP64 nodal image into image_out (device, n_elem x Np, user element order).  Asynchronous on
 * the bound stream.  Errors: DGRTM_ERR_ARG, DGRTM_ERR_HIP. */
dgrtm_status dgrtm_image(dgrtm_shot shot, double *image_out, int accumulate);

/* Misfit of two receiver trace sets (the relative trace error of the validation section is
 * its square root over the reference's norm): sum over all samples of (a - b)^2 in FP64, a and b
 * device float arrays of n values; the result is written to the host double *out, so the call
 * synchronises the stream.  Errors: DGRTM_ERR_ARG, DGRTM_ERR_HIP. */
dgrtm_status dgrtm_residual(dgrtm_shot shot, const float *a, const float *b, int64_t n, double *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): dgrtm_residual without a shot.  It computes the same
 * FP64 sum over all samples of (a - b)^2, allocates nothing, and keeps its partial sums in a
 * static device array of the library (512 KiB per device, held until the process ends).
 *   a, b        device float arrays of n values, 0 <= n <= 2^30 (larger n: DGRTM_ERR_ARG, nothing
 *               launched)
 *   out         device, one double: receives the sum (0 for n = 0)
 *   hip_stream  the hipStream_t the two kernels are queued on (NULL = the current device's
 *               default stream); the call returns without waiting for them
 * The sum is taken in a fixed order (chunks of 16384 values, then their sums), so equal inputs
 * give equal results bit for bit.  All calls on one device share its static array: calls whose
 * kernels overlap on one device (on different streams, or from different threads) race and
 * must be serialised by the caller.
 * Errors: DGRTM_ERR_ARG, DGRTM_ERR_HIP.
 */
dgrtm_status dgrtm_residual_noalloc(const float *a, const float *b, int64_t n, double *out, void *hip_stream);

/* ---- test hooks (device arrays in user order: n_elem x 4 fields (p, vx, vy, vz) x Np) ---- */

/* Cap on the work-groups of the mesh's step launches (max_groups > 0), or the default grid
 * (max_groups = 0: about one work-group per compute unit).  A cap well above the number of compute
 * units gives every wavefront fixed tiles at a fixed stride, which turns off the counter hand-out
 * and the staggered starts of large launches: results are the same bit for bit, which is what
 * the tests check.
 * Host only; applies to later launches.  Errors: DGRTM_ERR_ARG (null mesh, negative cap). */
dgrtm_status dgrtm_mesh_set_launch_cap(dgrtm_mesh mesh, int64_t max_groups);

/* Right-hand side of the semi-discrete system (eqs. dgLocalSchemeP/U, the appendix) for the
 * given state (no source), forward time
 * (reversed = 0) or reversed time -L(q; -tau) (reversed = 1).  Uses the shot's source-field buffers. */
dgrtm_status dgrtm_apply_rhs(dgrtm_shot shot, const float *q, float *rhs, int reversed);

/* Set a wavefield's state at time 0 and its AB3 history r(-dt), r(-2 dt) (either may be NULL = 0):
 * the initialisation step of Alg. 1. */
dgrtm_status dgrtm_set_state(dgrtm_shot shot, int which, const float *q, const float *hist1, const float *hist2);

/* Read a wavefield's current nodal state (p, v of eqs. waveSyst1/2). */
dgrtm_status dgrtm_get_state(dgrtm_shot shot, int which, float *q);

/* Advance a wavefield by n_global global steps of Alg. 1 (forward; reversed = 1 uses -L(q; -tau),
 * the backward-in-time paragraph of the time-stepping section),
 * with the shot's source when with_source != 0 and the wavefield is the source field. */
dgrtm_status dgrtm_run(dgrtm_shot shot, int which, int64_t n_global, int reversed, int with_source);

/* ---- measurement ---- */

/* Measurement, not part of the method: time every sample_every-th launch of the fused step kernel with a pair of HIP events on the
 * bound stream (0 = off); clears earlier samples.  The events are created on the host by the
 * library and released by dgrtm_shot_destroy. */
dgrtm_status dgrtm_profile_start(dgrtm_shot shot, int sample_every);

/* Sum over the sampled launches of step-kernel mode `mode` (0 plain forward step, 1 source
 * recompute with segment recording, 2 backward step with imaging, 3 rhs only): total kernel
 * time in milliseconds, number of sampled launches, and real elements updated by them.
 * Synchronises the stream. */
dgrtm_status dgrtm_profile_read(dgrtm_shot shot, int mode, double *kernel_ms, int64_t *launches,
                                int64_t *element_steps);

/* Release the host handle and its timing events (the caller frees the workspace). NULL is ignored. */
void dgrtm_shot_destroy(dgrtm_shot shot);

#ifdef __cplusplus
}
#endif
#endif /* DGRTM_H */
