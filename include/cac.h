/*
 * cac.h -- C ABI of libcac, the MI355X (gfx950) implementation of one coupled
 * time step of the conservative Allen-Cahn lattice Boltzmann method with
 * geometric ghost-node wetting and global phase-field volume correction
 * (Bello, Mander, Lauricella, Guglielmo, La Rocca, Montessori, "Accurate
 * wetting dynamics via a conservative Allen-Cahn based lattice Boltzmann
 * approach for multiphase flows", Sec. II).
 *
 * Problem statement the calls follow (Sec. II B, II C): a voxel mask splits
 * the lattice into fluid nodes and solid nodes; every solid node with a fluid
 * neighbour (a "wall node") carries a prescribed contact angle theta; the
 * conserved observable is the phase-field volume M = sum over fluid nodes of
 * phi (Eq. (48)).
 *
 * Conventions
 *  - Lattice nx * ny * nz, node index n = x + nx * (y + ny * z), periodic
 *    index wrap in x, y and z (walls are solid voxels in the mask).
 *  - Vector and population fields are structure of arrays: u[d * N + n],
 *    f[i * N + n] with the D3Q27 velocities in the order
 *      0 (0,0,0); 1,2 (+-1,0,0); 3,4 (0,+-1,0); 5,6 (0,0,+-1);
 *      7,8 +-(1,1,0); 9,10 +-(1,-1,0); 11,12 +-(1,0,1); 13,14 +-(1,0,-1);
 *      15,16 +-(0,1,1); 17,18 +-(0,1,-1); 19,20 +-(1,1,1); 21,22 +-(1,1,-1);
 *      23,24 +-(1,-1,1); 25,26 +-(-1,1,1).
 *  - Pointers named d_* are device pointers (HIP global memory on the device
 *    the handle was created on); all others are host pointers.
 *  - Calls on a handle are stream-ordered on the stream given to cac_init and
 *    asynchronous unless stated; a handle is used by one host thread at a time.
 *  - The library never frees caller buffers.  Device memory of the handle is
 *    obtained through the allocation callback (or hipMalloc when it is NULL)
 *    and released by cac_destroy (callback memory: the caller's to release).
 *  - Every call returns a cac_status; on failure a message is kept for
 *    cac_last_error.  Device-side non-finite detection is reported by the next
 *    synchronising call (cac_volume, cac_sync).
 */
#ifndef CAC_H
#define CAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CAC_OK = 0,
    CAC_ERR_ARG = 1,       /* invalid argument (null pointer, size, range) */
    CAC_ERR_GEOMETRY = 2,  /* unusable mask (no fluid node, wrong size) */
    CAC_ERR_HIP = 3,       /* a HIP runtime call failed */
    CAC_ERR_NONFINITE = 4, /* a NaN/Inf appeared in phi or u (watchdog flag) */
    CAC_ERR_STATE = 5,     /* call out of order (e.g. step before set_state) */
    CAC_ERR_ALLOC = 6      /* the allocation callback or hipMalloc failed */
} cac_status;

typedef struct cac_handle cac_handle;

/* Allocation callback: returns `bytes` of device memory (256-byte aligned) that
 * stays valid until cac_destroy, or NULL on failure. */
typedef void *(*cac_alloc_fn)(size_t bytes, void *user);

/* Physical and numerical parameters, lattice units (dx = dt = 1). */
typedef struct {
    double rho_l, rho_g;     /* liquid (phi = 1) and gas (phi = 0) densities, Eq. (8) */
    double nu_l, nu_g;       /* kinematic viscosities; mu = rho nu interpolated linearly, Eqs. (9)-(10) */
    double sigma, delta;     /* surface tension and interface width: beta = 12 sigma/delta,
                                kappa_phi = 3 sigma delta / 2 (definitions after Eq. (19)) */
    double D;                /* CAC interface diffusivity, Eq. (24); kappa = 4 D / delta, Eq. (26) */
    double g[3];             /* body acceleration; F_ext = (rho(phi) - rho_g) g */
    double eps_phi;          /* interface band of the volume correction, Eq. (51) (default 1e-3) */
    double eps_n;            /* interface normal is zero where |grad phi| <= eps_n (default 1e-12) */
    double sin_tol, cot_max; /* cot(theta_c) -> sign(cos) cot_max where |sin| < sin_tol (text after Eq. (45)) */
    int volume_correction;   /* 1: apply the correction of Eq. (53) every step */
    int wall_compression;    /* compressive flux phi(1-phi)n on wall nodes: 0 -> zero,
                                1 -> g (1 - g) times the unit corrected gradient of Eq. (45) */
    int collision;           /* non-equilibrium moment A2 of the regularised populations, Eq. (14):
                                0 -> the local second moment of the pre-collision populations;
                                1 -> the gradient form of Eq. (15), -(c_s^2/omega)(grad u + grad u^T),
                                     from the isotropic stencil of Eq. (22), a solid neighbour
                                     holding the node's mirror image -u (zero at the half-link)
                                     (the thread-safe formulation of Sec. II A: no populations are
                                     stored between steps).  With 1, cac_get_populations and the
                                     adjoint (cac_tape_*, cac_adjoint) are refused with
                                     CAC_ERR_STATE; a batch takes it when all its domains do. */
    int ghost_localization;  /* factor lambda_s of the ghost extrapolation, Eq. (46):
                                1 -> sqrt(4 phi_f (1 - phi_f)) of Eq. (47) (the paper's; default);
                                0 -> 1 (a diagnostic reading for the contact-angle study: the
                                     ghost is the plain first-order extrapolation).  The adjoint
                                     (cac_tape_*, cac_adjoint) is refused with CAC_ERR_STATE for 0. */
} cac_params;

/* Fill p with the defaults (rho = 1, nu = 0.04, sigma = 0.02, delta = 4,
 * D = 0.1, g = 0, eps_phi = 1e-3, eps_n = 1e-12, sin_tol = 1e-6,
 * cot_max = 1e6, volume_correction = 1, wall_compression = 1, collision = 0,
 * ghost_localization = 1). */
cac_status cac_default_params(cac_params *p);

/* Create a handle for an nx * ny * nz lattice on the current HIP device.
 * hip_stream: hipStream_t to order all work on (NULL: the null stream).
 * alloc/alloc_user: allocation callback (NULL: hipMalloc, freed by cac_destroy).
 * Errors: CAC_ERR_ARG if a size is < 2 or 27 * N does not fit in 32 bits, or
 * a parameter is out of range (densities or viscosities <= 0, delta <= 0, D < 0). */
cac_status cac_init(cac_handle **h, int nx, int ny, int nz, const cac_params *p, cac_alloc_fn alloc,
                    void *alloc_user, void *hip_stream);

/* Set the geometry.  solid: host, N bytes, 1 = solid, 0 = fluid.
 * theta_rad: host, N floats, prescribed contact angle in radians measured
 * through the liquid (phi = 1), read only at wall nodes; NULL = pi/2.
 * Builds, on the host, the wall-node list in ascending node index: the
 * unnormalised wall normal of Eq. (36) (weights of Eq. (37)), its unit vector
 * (Eq. (38)) and the donor link of Eqs. (39)-(41), chosen among all fluid links
 * by exact integer comparison of the alignment scores, ties to the lowest link
 * index.  Wall nodes whose normal sums to zero are kept in the list but skipped
 * by the update (their ghost stays at its initial value); their count is in the
 * cac_last_error text.  Invalidates the state (call cac_set_state next).
 * Errors: CAC_ERR_ARG (null solid), CAC_ERR_GEOMETRY (no fluid node). */
cac_status cac_set_geometry(cac_handle *h, const uint8_t *solid, const float *theta_rad);

/* Number of wall nodes n_b (skipped ones included). */
cac_status cac_num_wall_nodes(cac_handle *h, int *n_b);

/* Wall-node tables (host outputs, any may be NULL): linear_index[n_b],
 * normal6[3 n_b] (six times the unnormalised wall normal, exact integers),
 * donor[n_b] (donor link index 1..26, or -1 when skipped). */
cac_status cac_wall_nodes(cac_handle *h, int32_t *linear_index, int32_t *normal6, int32_t *donor);

/* Handle-free host version of the wall-node tables (no GPU use): for the
 * mask solid (host, N bytes) writes n_b and, when cap >= n_b, the tables of
 * cac_wall_nodes.  Errors: CAC_ERR_ARG (bad size or null pointer). */
cac_status cac_wall_tables(int nx, int ny, int nz, const uint8_t *solid, int *n_b, int32_t *linear_index,
                           int32_t *normal6, int32_t *donor, int cap);

/* Replace the contact angles: d_theta_compact, device, n_b floats (radians),
 * in wall-node order.  Takes effect at the next step. */
cac_status cac_set_contact_angles(cac_handle *h, const float *d_theta_compact);

/* Initial state.  d_phi: device, N floats, phi on all nodes (the values on
 * wall nodes are the initial ghosts).  d_u (3N) and d_pstar (N): initial
 * velocity and reduced pressure p* (Eq. (5)), or NULL for zero.  Populations
 * start at the equilibrium of Eq. (11); the target volume M_target is the sum
 * of d_phi over fluid nodes (FP64).  Errors: CAC_ERR_STATE before
 * cac_set_geometry, CAC_ERR_ARG for a null d_phi. */
cac_status cac_set_state(cac_handle *h, const float *d_phi, const float *d_u, const float *d_pstar);

/* Advance nsteps coupled steps (ghost update W, hydrodynamic collide-stream H,
 * CAC update P, volume correction V; Sec. II).  Asynchronous.
 * Errors: CAC_ERR_STATE without a state, CAC_ERR_ARG for nsteps < 0,
 * CAC_ERR_HIP on a launch failure. */
cac_status cac_step(cac_handle *h, int nsteps);

/* Phase-field volume M = sum over fluid nodes of phi (Eq. (48)), accumulated
 * in FP64 in a fixed order.  Synchronises the stream; returns
 * CAC_ERR_NONFINITE if the watchdog flag is set. */
cac_status cac_volume(cac_handle *h, double *out_host);

/* Copy out the current fields (device outputs, any may be NULL): d_phi (N) =
 * phi on fluid nodes and the latest ghosts on wall nodes; d_u (3N) and
 * d_pstar (N) = velocity (Eq. (7)) and p* (Eq. (6)) of the last step (the
 * initial ones before any step).  Asynchronous. */
cac_status cac_get_fields(cac_handle *h, float *d_phi, float *d_u, float *d_pstar);

/* Copy out the post-collision populations of the last step (device, 27 N),
 * defined on fluid nodes.  CAC_ERR_STATE with collision = 1 (no populations
 * are stored). */
cac_status cac_get_populations(cac_handle *h, float *d_f);

/* Wait for the handle's stream and report the watchdog flag
 * (CAC_ERR_NONFINITE) and any deferred HIP error. */
cac_status cac_sync(cac_handle *h);

/* Launch shape.  Hydrodynamic kernel: tile of bx * by * bz nodes per workgroup
 * (powers of two, bx >= 16, product 128, 256 or 512).  phase_tile: column tile
 * of the phase-field kernel, 0 = automatic, 1..6 = 64x8, 64x4, 32x8, 32x16,
 * 16x16, 128x4.  use_graph: 1 = replay steps from captured HIP graphs.
 * Errors: CAC_ERR_ARG for an unsupported shape. */
cac_status cac_set_launch(cac_handle *h, int bx, int by, int bz, int phase_tile, int use_graph);

/* Advance nsteps steps like cac_step, with HIP events recorded on the
 * handle's stream around every kernel; adds the elapsed milliseconds of each
 * substep kernel to ms[0..3] (W ghosts, H hydrodynamics, P phase field,
 * V volume correction).  Synchronises.  For measurement only. */
cac_status cac_profile_step(cac_handle *h, int nsteps, double *ms);

/* Debug modes (flags, OR-ed; 0 = off), checks of the race-freedom and of the
 * data the step never reads (results must stay bitwise the same):
 *   CAC_DEBUG_POISON: every cac_set_state / cac_load_state afterwards fills
 *     with quiet NaNs the populations and velocity on solid nodes and phi and
 *     the compressive flux on solid nodes without a fluid neighbour (values the
 *     step must never use);
 *   CAC_DEBUG_REVERSE_ORDER: the ghost, hydrodynamic and phase kernels take
 *     their workgroups in reverse order from the next step on.
 * Errors: CAC_ERR_ARG for an unknown flag. */
enum { CAC_DEBUG_POISON = 1, CAC_DEBUG_REVERSE_ORDER = 2 };
cac_status cac_set_debug(cac_handle *h, int flags);

/* Bandwidth ceiling of the hydrodynamic kernel's access pattern: reps
 * launches of a kernel that pulls the 27 population planes from the upstream
 * neighbours (periodic wrap) and stores them, with the tiling and load hints
 * of the collide-stream kernel and none of its arithmetic (216 bytes moved per
 * node).  *ms = average milliseconds per launch (HIP events on the handle's
 * stream).  Overwrites both population buffers: the handle has no state
 * afterwards (cac_step returns CAC_ERR_STATE until cac_set_state or
 * cac_load_state).  Synchronises.  For measurement only. */
cac_status cac_pull_copy_probe(cac_handle *h, int reps, double *ms);

/* Size in bytes of a saved state (cac_save_state): a 64-byte header plus
 * 33 N floats (populations, phi with the current and the previous ghosts,
 * velocity, initial p*).  With collision = 1 the population planes hold the
 * record of the last collision (p*, a, omega) instead. */
cac_status cac_state_bytes(cac_handle *h, size_t *bytes);

/* Checkpoint: copy the complete state (populations, phi and ghosts, velocity,
 * target volume, step count) into d_buf (device, at least cac_state_bytes).
 * Synchronises the stream before writing the header.  Errors: CAC_ERR_ARG
 * (buffer too small), CAC_ERR_STATE (no state, or inside a debug step). */
cac_status cac_save_state(cac_handle *h, void *d_buf, size_t bytes);

/* Resume from a buffer written by cac_save_state on a handle with the same
 * lattice size; the geometry and angles are those set on this handle.  Stepping
 * after a load reproduces the saved run bit for bit.  Discards an adjoint
 * recording.  Errors: CAC_ERR_ARG (size or header mismatch, or a state saved
 * with another collision setting), CAC_ERR_STATE (no geometry). */
cac_status cac_load_state(cac_handle *h, const void *d_buf, size_t bytes);

/* Test hook: run one substep of the next step, in order 0 = W ghost update
 * (Sec. II B), 1 = H collide-stream (Sec. II A), 2 = P CAC update (Sec. II A 1),
 * 3 = V volume correction (Sec. II C; completes the step).  cac_step is refused
 * while a step is partly done.  Errors: CAC_ERR_STATE (out of order). */
cac_status cac_debug_substep(cac_handle *h, int which);

/* Test hook: copy an internal buffer to d_out (device): 0 = phi of the current
 * parity (fluid values; after W the new ghosts), 1 = phi of the other parity
 * (previous ghosts; after P the phase field before the correction), 2 = u (3N),
 * 3 = populations of the current parity (27N), 4 = populations of the other
 * parity (after H the post-collision populations, 27N), 5 = compressive flux
 * on wall nodes (3N).  With collision = 1: 3 = the post-collision populations
 * rebuilt by the last H substep, 4 = the record planes (p*, a, omega, then
 * unused planes), 27N each.  Errors: CAC_ERR_ARG (unknown buffer). */
cac_status cac_debug_buffer(cac_handle *h, int which, float *d_out);

/* Release the handle and the device memory it allocated itself. */
cac_status cac_destroy(cac_handle *h);

/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of the step.  The paper defines no adjoint; this is
 * the exact transpose of the Jacobian of the discrete step W -> H -> P -> V
 * (Sec. II), used to differentiate a loss of the final phase field with
 * respect to the per-wall-node contact angles (Sec. II B, Eqs. (43)-(46)) and
 * the initial phase field.  At non-smooth points (minmod, upwind side, the
 * band of Eq. (51), the normal guard, lambda_s of Eq. (47), |grad_par|, the
 * regularised cotangent) the branch taken by the forward step is
 * differentiated.  All reverse kernels are deterministic; dL/dtheta is
 * accumulated over the steps in FP64.
 * ------------------------------------------------------------------------ */

/* Advance nsteps steps from the current state, exactly as cac_step, and record
 * the sweep for cac_tape_backward: the state (populations, phi, previous
 * ghosts) is copied every K steps (checkpoints, ceil(nsteps/K) x 29 N floats)
 * together with the contact angles in use.  The last segment (the steps after
 * the last checkpoint) runs through the reverse sweep's rings, which are
 * allocated here (about 32 N floats per step of a segment), so that segment is
 * never replayed; the live state afterwards is the one cac_step would leave,
 * bit for bit.  With K >= nsteps the whole rollout is kept (about 128 bytes
 * per node and step) and nothing is replayed.  cac_set_state and
 * cac_set_geometry discard the recording.  Asynchronous.
 * Errors: CAC_ERR_ARG (nsteps or K < 1), CAC_ERR_STATE (no state, inside a
 * debug step, collision = 1 or ghost_localization = 0), CAC_ERR_ALLOC. */
cac_status cac_tape_forward(cac_handle *h, int nsteps, int K);

/* Reverse sweep of the recorded sweep.  d_phibar (device, N floats): cotangent
 * dL/dphi of the phase field after the last recorded step, on all nodes (wall
 * nodes: the ghost values that cac_get_fields reports).  Outputs:
 * d_dtheta (device, n_b doubles, wall-node order) = dL/dtheta in radians^-1
 * (zero for skipped wall nodes); d_phibar0 (device, N floats, or NULL) =
 * dL/dphi of the phase field passed to cac_set_state (fluid values and initial
 * ghosts).  Each segment of K steps is replayed from its checkpoint into rings
 * of about (33 K + 70) N floats, then reversed step by step; the last segment
 * is already in the rings after cac_tape_forward (and stays there for a
 * repeated call when it is the only segment).  With room for a second set of
 * rings, the replay of the next segment runs on a second stream while the
 * current one is reversed.  The live state is not changed.  Asynchronous.
 * Errors: CAC_ERR_ARG (null pointer), CAC_ERR_STATE (nothing recorded, or the
 * geometry changed since), CAC_ERR_ALLOC. */
cac_status cac_tape_backward(cac_handle *h, const float *d_phibar, double *d_dtheta, float *d_phibar0);

/* Loss L = 1/2 sum over fluid nodes of (phi - phi_target)^2 of the current
 * state, accumulated in FP64.  d_seed (device, N floats, or NULL): receives
 * dL/dphi = phi - phi_target on fluid nodes and 0 on solid nodes.  loss_host
 * (or NULL): the loss; when given, the call synchronises.
 * Errors: CAC_ERR_ARG, CAC_ERR_STATE (no state). */
cac_status cac_loss(cac_handle *h, const float *d_phi_target, float *d_seed, double *loss_host);

/* cac_tape_forward(nsteps, K), then cac_loss against d_phi_target (device, N
 * floats), then the reverse sweep seeded with dL/dphi: loss_host (or NULL)
 * receives L and d_dL_dtheta (device, n_b doubles) the gradient.  Leaves the
 * state after step nsteps.  Synchronises; errors as the three calls, and
 * CAC_ERR_NONFINITE from the watchdog. */
cac_status cac_adjoint(cac_handle *h, int nsteps, int K, const float *d_phi_target, double *loss_host,
                       double *d_dL_dtheta);

/* ------------------------------------------------------------------------
 * Batched step: many independent lattices ("domains") of uneven size, contact
 * angle and parameters advanced together, one launch per substep, by
 * persistent workgroups that walk a list of (domain, tile) work items.  The
 * step of every domain is the single-lattice step above (Sec. II); the batch
 * is an execution arrangement, not a change of the method.  Domain k's fields
 * keep the single-lattice layout in its own slice of shared device arrays.
 * ------------------------------------------------------------------------ */
typedef struct cac_batch cac_batch;

typedef struct {
    int nx, ny, nz;          /* each >= 2 */
    cac_params params;
    const uint8_t *solid;    /* host, N bytes, 1 = solid */
    const float *theta_rad;  /* host, N floats read at wall nodes, or NULL (pi/2) */
    const float *d_phi0;     /* device, N floats: initial phi (values on wall nodes = initial ghosts) */
} cac_domain_desc;

/* Create a batch of ndom (1..65535) domains on the current device, geometry
 * and initial state included (populations at rest equilibrium, M_target per
 * domain in FP64).  The total 27 * sum(N) must fit in 31 bits.  All domains
 * share one params.collision setting.  Errors: CAC_ERR_ARG (sizes, parameters,
 * null pointers, mixed collision settings), CAC_ERR_ALLOC, CAC_ERR_HIP. */
cac_status cac_batch_init(cac_batch **b, int ndom, const cac_domain_desc *d, cac_alloc_fn alloc, void *alloc_user,
                          void *hip_stream);

/* Block schedule: hydrodynamic tile bx * by * bz (as in cac_set_launch; bx = 0
 * fits a tile of `by` nodes to every domain, its x extent the largest power of
 * two dividing nx), phase
 * column tile code 1..6, persistent grid = grid_mult x resident workgroups per
 * CU x CUs (0: one workgroup per item), order 0 = domains in input order,
 * 1 = largest first; use_graph replays steps from captured HIP graphs. */
cac_status cac_batch_set_schedule(cac_batch *b, int bx, int by, int bz, int phase_tile, int grid_mult, int order,
                                  int use_graph);
/* Current schedule as 7 ints in the order of cac_batch_set_schedule. */
cac_status cac_batch_get_schedule(cac_batch *b, int *out7);

/* Choose the schedule by timing trial_steps steps per candidate (two passes
 * of a coordinate search over the tile, the phase tile, the grid multiplier
 * and the order).
 * The state is saved before and restored after.  cache_path (or NULL): JSON
 * file of schedules keyed by device and the histogram of domain shapes; a
 * matching entry is applied without timing (*best_ms = -1).  Synchronises. */
cac_status cac_batch_autotune(cac_batch *b, const char *cache_path, int trial_steps, double *best_ms);

/* Advance every domain nsteps steps.  Asynchronous. */
cac_status cac_batch_step(cac_batch *b, int nsteps);

/* Wait; CAC_ERR_NONFINITE if any domain produced a non-finite value. */
cac_status cac_batch_sync(cac_batch *b);

/* Phase-field volume of every domain (host out[ndom], FP64).  Synchronises. */
cac_status cac_batch_volume(cac_batch *b, double *out);

/* Fields of domain k, as cac_get_fields (device outputs, any may be NULL). */
cac_status cac_batch_get_fields(cac_batch *b, int k, float *d_phi, float *d_u, float *d_pstar);

/* Number of domains and total / fluid node counts (any output may be NULL). */
cac_status cac_batch_info(cac_batch *b, int *ndom, long long *total_nodes, long long *fluid_nodes);

/* As cac_profile_step for the batch: adds per-substep milliseconds (W, H, P, V). */
cac_status cac_batch_profile(cac_batch *b, int nsteps, double *ms);

cac_status cac_batch_destroy(cac_batch *b);
cac_status cac_batch_last_error(cac_batch *b, char *buf, size_t n);

/* ------------------------------------------------------------------------
 * Allocation-free volume, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Handle-free variant of cac_volume: the phase-field volume
 * M = sum over fluid nodes of phi (Eq. (48)), accumulated in FP64 by the same
 * kernels and in the same order as cac_volume (equal inputs give bitwise
 * equal results).
 *   d_solid: device, N bytes, 1 = solid (only fluid nodes are summed);
 *   d_phi:   device, N floats;
 *   d_out:   device, 1 double, written stream-ordered (no synchronisation);
 *   hip_stream: hipStream_t to launch on (NULL: the null stream).
 * N = nx * ny * nz must not exceed 134217728 (= 2^27, e.g. 512^3): the block
 * partials live in a static device array of 2^19 16-byte entries (8 MiB),
 * which every GPU the library runs on holds until the process ends.  No
 * memory is allocated or freed and no memset is issued; every partial is
 * written before it is read.  All calls on one device share that device's
 * array: calls that overlap in time on one device (two streams, two host
 * threads) race and must be serialised by the caller.
 * Errors: CAC_ERR_ARG (empty axis, N above the limit, null pointer; the text
 * is kept for cac_last_error(NULL, ...)), CAC_ERR_HIP (launch failure). */
cac_status cac_volume_noalloc(int nx, int ny, int nz, const uint8_t *d_solid, const float *d_phi, double *d_out,
                              void *hip_stream);

const char *cac_status_string(cac_status s);

/* Copy the message of the last failed call on h into buf (n bytes); with
 * h = NULL, the message of the last failed handle-free call of the calling
 * thread (cac_volume_noalloc). */
cac_status cac_last_error(cac_handle *h, char *buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* CAC_H */
