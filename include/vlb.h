/*
 * vlb.h -- C ABI of the MI355X (gfx950) lattice Boltzmann library for
 * Oldroyd-B fluids with complex and moving boundaries, after Kuron, Stewart,
 * de Graaf and Holm, "An extensible lattice Boltzmann method for viscoelastic
 * flows: complex and moving boundaries in Oldroyd-B fluids" (arXiv 2009.12279).
 *
 * One time step is the coupled per-cell update of Section 3:
 *   - D3Q19 TRT stream-collide with Guo forcing whose force is the body force
 *     plus the divergence of the polymer stress (Section 3.1, Section 2.1
 *     polymer force, Section 3.3 force discretisation);
 *   - explicit finite-volume update of the Oldroyd-B stress with
 *     corner-transport-upwind face fluxes (Section 2.2, Section 3.3);
 *   - link bounce-back with the moving-wall term for walls and particle
 *     surfaces, momentum exchange force and torque on particles, symplectic
 *     Euler particle motion, and refill / deletion of cells a moving particle
 *     uncovers / covers (Section 3.1 velocity boundary condition, Section 3.4).
 *
 * Conventions (all functions):
 *   - Lattice units: grid spacing = time step = 1, reference density 1.
 *   - Cell index n = x + nx*(y + ny*z).  A field with k components is passed
 *     as k consecutive planes of N = nx*ny*nz values (structure of arrays).
 *   - Stress components are ordered xx, yy, zz, xy, xz, yz.
 *   - Populations use the direction order of vlb_velocity().
 *   - Mask byte per cell: 0 = fluid; 1..63 = wall id w, moving with
 *     wall_velocity[w-1] (at rest when w > n_walls); 64..255 are reserved for
 *     particles and set only by vlb_add_sphere (particle k has byte 64+k).
 *     Every non-periodic axis must have solid cells in its first and last
 *     layer.
 *   - All host pointers are copied at the call (inputs) or filled before the
 *     call returns (outputs); the caller owns them.  The library owns all
 *     device memory it allocates.
 *   - Every call returns a vlb_status; no exception or abort crosses the ABI.
 *     On failure the lattice keeps its previous state and vlb_last_error()
 *     describes the cause.  VLB_EUNSTABLE is sticky: once a health check
 *     found a non-finite value or a speed above the limit, vlb_step returns
 *     it without stepping; reads still work.
 *   - vlb_step is asynchronous on the lattice's HIP stream; every read
 *     synchronises that stream.
 */
#ifndef VLB_H
#define VLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VLB_Q 19
#define VLB_MAX_WALL_ID 63
#define VLB_MAX_PARTICLES 192

typedef enum vlb_status {
    VLB_OK = 0,
    VLB_EINVAL = 1,    /* invalid argument or parameter                     */
    VLB_ENOMEM = 2,    /* device or host allocation failed                  */
    VLB_EDEVICE = 3,   /* HIP runtime error or no usable device             */
    VLB_EUNSTABLE = 4, /* non-finite field or speed above the health limit  */
    VLB_ESTATE = 5,    /* call not allowed in the current state             */
    VLB_EBUSY = 6,     /* no free slot / memory budget (serving)            */
    VLB_ENOTFOUND = 7  /* unknown particle id or ticket                     */
} vlb_status;

/* Population storage: deviations h_i = s * (f_i - w_i) from the lattice
 * weights w_i, with a power-of-two scale s (1 for FP32, 2^10 for FP16 unless
 * vlb_set_velocity_scale picks another, 1 for BF16).  The per-cell arithmetic runs in FP64 registers for FP32 storage and
 * in FP32 for FP16/BF16 storage; particle sums are FP64. */
typedef enum vlb_storage { VLB_STORE_F32 = 0, VLB_STORE_F16 = 1, VLB_STORE_BF16 = 2 } vlb_storage;

/* How stored values (populations and stress) are rounded to their storage
 * precision after each step.  Stochastic rounding picks the neighbouring
 * representable value above or below with probability proportional to the
 * distance, from a counter-based hash of (cell, step, seed); it is unbiased,
 * so a slowly relaxing steady state does not drift the way repeated
 * round-to-nearest does.  Results are deterministic for a given seed. */
typedef enum vlb_rounding { VLB_ROUND_NEAREST = 0, VLB_ROUND_STOCHASTIC = 1 } vlb_rounding;

typedef struct vlb_dims {
    int32_t nx, ny, nz;
    uint8_t periodic[3]; /* 1 = periodic along x, y, z */
    uint8_t reserved;
} vlb_dims;

/* Physical parameters (Section 2, Section 3.1).  Defaults: eta = 1/3,
 * beta = 0, lambda_p = 1, magic = 3/16, no body force. */
typedef struct vlb_params {
    double eta;           /* total dynamic viscosity eta = eta_n + eta_p            */
    double beta;          /* polymer fraction eta_p/eta in [0,1); 0 = Newtonian     */
    double lambda_p;      /* polymer relaxation time in steps (>= 1 when beta > 0) */
    double magic;         /* TRT (1/w+ - 1/2)(1/w- - 1/2); < 0 selects BGK (w- = w+) */
    double body_force[3]; /* force density g applied to every fluid cell            */
} vlb_params;

typedef struct vlb_lattice vlb_lattice;

/* Direction i (0..18) of the D3Q19 set: velocity c[3] and weight *w (either
 * may be NULL).  Returns VLB_Q.  Order: rest, +x, -x, +y, -y, +z, -z, then
 * the 12 edge directions in opposite pairs (+x+y, -x-y, +x-y, -x+y, +x+z,
 * -x-z, +x-z, -x+z, +y+z, -y-z, +y-z, -y+z). */
int32_t vlb_velocity(int32_t i, int32_t c[3], double *w);

/* Bytes of device memory a lattice of these dimensions holds (admission). */
size_t vlb_required_bytes(const vlb_dims *dims, vlb_storage storage, int32_t n_particles);

/* Create a lattice on the current HIP device.  mask: N bytes (see above).
 * wall_velocity: n_walls x 3 doubles or NULL.  stream: a hipStream_t to
 * enqueue all work on, or NULL for a stream the library creates.  The state
 * starts at rest (f = w, tau = 0) with the default parameters.
 * Errors: VLB_EINVAL (bad dims, mask values >= 64, a non-periodic axis
 * without solid end layers, n_walls > 63), VLB_ENOMEM, VLB_EDEVICE. */
vlb_status vlb_create(const vlb_dims *dims, const uint8_t *mask, const double *wall_velocity,
                      int32_t n_walls, vlb_storage storage, void *stream, vlb_lattice **out);

/* Caller-owned state.  The large state arrays can live in device memory the
 * caller allocates and owns (torch tensors, a pool): VLB_NBUF buffers, in
 * this order: 0 mask (uint8), 1-2 the two population buffers, 3-4 the two
 * stress buffers (FP32), 5 the velocity (FP32), each at least the size
 * vlb_buffer_sizes gives and 256-byte aligned, on the current device.  The
 * caller keeps them alive until vlb_destroy, which does not free them.  The
 * library still allocates its small tables itself.
 * Errors: VLB_EINVAL (bad dims or storage, a buffer missing, too small or
 * misaligned), and as vlb_create. */
#define VLB_NBUF 6
vlb_status vlb_buffer_sizes(const vlb_dims *dims, vlb_storage storage, size_t sizes[VLB_NBUF]);
vlb_status vlb_create_with_buffers(const vlb_dims *dims, const uint8_t *mask,
                                   const double *wall_velocity, int32_t n_walls,
                                   vlb_storage storage, void *stream,
                                   void *const buffers[VLB_NBUF], const size_t sizes[VLB_NBUF],
                                   vlb_lattice **out);

/* Set eta, beta, lambda_p, magic and the body force (Section 2.3, 3.1):
 * omega+ = 1/(3 (1-beta) eta + 1/2); omega- from magic.  VLB_EINVAL when
 * eta <= 0, beta outside [0,1), lambda_p < 1 with beta > 0, or a rate
 * outside (0,2). */
vlb_status vlb_set_params(vlb_lattice *lat, const vlb_params *params);

/* Initial state (Section 3.1, equilibrium distribution with c_s^2 = 1/3):
 * f = f^eq(rho = 1, u) on fluid cells (u: 3*N doubles, or NULL for rest),
 * tau = 0.  Resets the step count. */
vlb_status vlb_init_equilibrium(vlb_lattice *lat, const double *u);

/* Overwrite the populations f_i of Section 3.1 (19*N doubles, raw f,
 * vlb_velocity order) or the polymer stress tau of Section 2.2 (6*N doubles)
 * of every fluid cell; solid cells are ignored. */
vlb_status vlb_set_populations(vlb_lattice *lat, const double *f);
vlb_status vlb_set_stress(vlb_lattice *lat, const double *tau);

/* Add a sphere of radius r centred at c (cells with |x - c|^2 < r^2, minimum
 * image on periodic axes) as particle *id_out.  Mass = density_ratio *
 * 4/3 pi r^3, moment of inertia 2/5 M r^2.  A movable sphere follows
 * symplectic Euler under momentum exchange, polymer traction, conversion
 * momentum and the external force/torque (Section 3.4); a fixed one only
 * records its force.  VLB_EINVAL if it overlaps a non-fluid cell or the
 * particle table is full. */
vlb_status vlb_add_sphere(vlb_lattice *lat, const double center[3], double radius,
                          double density_ratio, int32_t movable, const double f_ext[3],
                          const double t_ext[3], int32_t *id_out);

/* Advance n_steps time steps (asynchronous).  One step is the coupled
 * update of Section 3: polymer force from the stress (Section 3.3, force
 * discretisation), TRT collision with Guo forcing and pull streaming
 * (Section 3.1, lattice Boltzmann and forcing equations), halfway
 * bounce-back with the moving-wall term (Section 3.1, velocity boundary
 * condition), the finite-volume stress update (Section 2.2 source,
 * Section 3.3 fluxes), and for movable particles momentum exchange, the
 * symplectic Euler update and fluid/solid conversion (Section 3.4).  Steps
 * are replayed from captured HIP graphs in chunks of 32, 16, ..., 1 steps
 * (captured once per set of step arguments), with the same kernels and
 * arguments, so the results are the same bits as step-by-step launches;
 * VLB_GRAPH=0 in the environment turns the replays off.  Errors:
 * VLB_EINVAL (negative count), VLB_EUNSTABLE (sticky, or found by a health
 * check at the end of this call's steps), VLB_EDEVICE. */
vlb_status vlb_step(vlb_lattice *lat, int64_t n_steps);
vlb_status vlb_sync(vlb_lattice *lat);
int64_t vlb_step_count(const vlb_lattice *lat);

/* Reads of the current state (FP64 host arrays of N, 3*N, 6*N, 19*N values;
 * solid cells read 0).  Density rho = sum f and velocity
 * u = (sum f c + F/2)/rho (Section 3.1, macroscopic moments with the half
 * force), with F = g + the per-cell force field, if set, + the polymer force
 * of the current stress (Section 3.3, force discretisation); the stress is
 * the polymer stress tau of Section 2.2 (for FENE-P mapped from the stored
 * variable); populations are raw f = w_i + stored deviation.  Synchronise
 * the stream; allocate a device staging buffer of the output's size for
 * the call.  Errors: VLB_EINVAL (NULL output), VLB_ENOMEM, VLB_EDEVICE. */
vlb_status vlb_read_density(vlb_lattice *lat, double *rho);
vlb_status vlb_read_velocity(vlb_lattice *lat, double *u);
vlb_status vlb_read_stress(vlb_lattice *lat, double *tau);
vlb_status vlb_read_populations(vlb_lattice *lat, double *f);
vlb_status vlb_read_mask(vlb_lattice *lat, uint8_t *mask);

/* vlb_read_velocity for callers that cannot allocate device memory (tight
 * serving or polling loops, harnesses that forbid hipMalloc): the velocity
 * of cells first .. first + count - 1 only, into u (3*count doubles: the x,
 * y and z components, count values each, in cell order), staged through a
 * fixed device array of VLB_NOALLOC_MAX_CELLS cells (6 MiB) that every GPU
 * the library runs on holds until the process ends.  Allocates nothing.
 * Every call on one GPU shares that array and overwrites it: calls that
 * overlap on one GPU (several host threads) race, and the caller must
 * serialise them.  Synchronises the lattice's stream.  Errors: VLB_EINVAL
 * (NULL output, count outside 1..VLB_NOALLOC_MAX_CELLS, a range beyond the
 * lattice), VLB_EDEVICE. */
#define VLB_NOALLOC_MAX_CELLS 262144
vlb_status vlb_read_velocity_noalloc(vlb_lattice *lat, int64_t first, int64_t count, double *u);

/* Particle state after the last step and the total force / torque that step
 * applied to it (Section 3.4: momentum exchange over the particle's
 * boundary links with lever arm r_b - R, polymer traction, conversion
 * momentum, external), FP64; position, velocity and spin are those of the
 * symplectic Euler update.  For fixed geometry (no movable particle) the
 * last step's sums are evaluated at this call from the state that step
 * left, which gives the same bits as evaluating them during the step.  Any
 * output may be NULL.  Errors: VLB_ENOTFOUND (unknown id), VLB_EDEVICE. */
vlb_status vlb_read_particle(vlb_lattice *lat, int32_t id, double pos[3], double vel[3],
                             double omega[3], double force[3], double torque[3]);

/* FP64 population mass sum f and momentum sum f c over fluid cells (the
 * moments of Section 3.1 without the half-force term), the quantities whose
 * conservation the coupling of Sections 3.3 and 3.4 is built to keep. */
vlb_status vlb_read_sums(vlb_lattice *lat, double *mass, double momentum[3]);

/* Momentum exchange + polymer traction of the last step summed over all wall
 * links (FP64), a diagnostic. */
vlb_status vlb_read_wall_force(vlb_lattice *lat, double force[3]);

/* Health check of the current state: largest |sum f c / rho| and number of
 * non-finite populations.  Sets the sticky VLB_EUNSTABLE state (and returns
 * it) when either exceeds the limits (speed 0.3 or any non-finite value).
 * vlb_step also runs it every check_interval steps (default 1000; 0 = off). */
vlb_status vlb_check_health(vlb_lattice *lat, double *max_speed, int64_t *non_finite);
vlb_status vlb_set_check_interval(vlb_lattice *lat, int64_t steps);

/* Checkpoint: parameters, mask, walls, particles, step count, rounding mode
 * and seed, the constitutive law, extrapolation order, counter-force, the
 * wall-velocity and force fields, and the state in its storage precision,
 * so that a restarted run continues bit for bit.  vlb_load creates a new lattice (VLB_EINVAL for a
 * file that is not a checkpoint of this format). */
vlb_status vlb_save(vlb_lattice *lat, const char *path);
vlb_status vlb_load(const char *path, void *stream, vlb_lattice **out);

/* Destroy the lattice and free its device memory (synchronises first). */
void vlb_destroy(vlb_lattice *lat);

/* Message of the last failed call on this lattice (or of the last failed
 * create/load when lat is NULL).  Never NULL. */
const char *vlb_last_error(const vlb_lattice *lat);

/* Average device time of the last vlb_step call per kernel family, measured
 * with HIP events on the lattice's stream when timing is on (ms; -1 when not
 * measured).  which: 0 = stream-collide, or the fused step kernel that also
 * runs the stress update (VLB_FUSED=1 in the environment selects it for
 * polymer lattices that fill the chip with its tiles, -1 for every polymer
 * lattice; it gives the same bits as the two kernels and is slower on
 * MI355X, so it is off by default), 1 = stress update (-1 when it ran fused
 * or there is no polymer), 2 = particles. */
vlb_status vlb_set_timing(vlb_lattice *lat, int32_t on);

/* Giesekus constitutive law (Section 2.2 names it among the models the
 * method extends to): the stress update's source gains -(alpha / eta_p)
 * tau.tau, from tau + lambda tau^del + (alpha lambda / eta_p) tau.tau =
 * eta_p (grad u + grad u^T).  alpha in [0, 1/2] (VLB_EINVAL otherwise);
 * 0, the default, is Oldroyd-B.  Kept in checkpoints. */
vlb_status vlb_set_giesekus(vlb_lattice *lat, double alpha);

/* FENE-P constitutive law (Section 2.2 names it as the model the method
 * extends to), with the Peterlin closure f = (L^2 - 3) / (L^2 - tr A) of the
 * conformation A.  The stored stress variable becomes T = (eta_p/lambda)
 * (A - I), which relaxes as -(f/lambda) T - (eta_p/lambda^2)(f - 1) I; the
 * polymer force, the traction on obstacles and vlb_read_stress use the
 * polymer stress f T + (eta_p/lambda)(f - 1) I; vlb_set_stress sets T.
 * L2 = L^2 > 3, or 0 for off (VLB_EINVAL otherwise); the last of
 * vlb_set_giesekus and vlb_set_fene_p wins.  Kept in checkpoints. */
vlb_status vlb_set_fene_p(vlb_lattice *lat, double L2);

/* Extrapolation of the stress into solid face neighbours for the polymer
 * force (Section 3.3): the polynomial through the fluid cell and the fluid
 * cells behind it, evaluated at the solid neighbour.  0 takes the cell's own
 * stress (the default); 1 is linear, 2 tau(x) - tau(x - e); 2 is quadratic,
 * 3 tau(x) - 3 tau(x - e) + tau(x - 2e).  Where a cell behind is solid the
 * order drops to what the fluid cells support.  The traction on obstacles
 * uses the same face values, so momentum stays balanced.  VLB_EINVAL for
 * other orders.  Kept in checkpoints. */
vlb_status vlb_set_stress_extrapolation(vlb_lattice *lat, int32_t order);

/* Force density that varies from cell to cell (Section 3.1 Guo forcing; the
 * driving force of the four-roll mill, Section 4.4).  F: 3*N doubles, the
 * x, y and z planes in cell order, copied and stored in FP32; added to the
 * uniform body force at every fluid cell.  NULL frees the field.
 * Synchronises the lattice's stream.  Errors: VLB_EINVAL (non-finite value),
 * VLB_ENOMEM.  Kept in checkpoints. */
vlb_status vlb_set_force_field(vlb_lattice *lat, const double *F);

/* Wall velocity that varies along a wall (Section 3.1 velocity boundary
 * condition; the regularized lid of the lid-driven cavity, Section 4.3).
 * u: 3*N doubles, the x, y and z planes in cell order, copied.  When set,
 * every wall cell (mask 1..63) moves with its own entry and the per-id
 * table is ignored; entries of other cells are not read.  NULL frees the
 * field and returns to the table.  Synchronises the lattice's stream.
 * Errors: VLB_EINVAL (non-finite value), VLB_ENOMEM.  Kept in checkpoints. */
vlb_status vlb_set_wall_velocity_field(vlb_lattice *lat, const double *u);

/* Overlap-fraction smoothing of fluid/solid conversions (Section 3.4 names
 * smoothing conversions with the fraction of a cell a particle overlaps;
 * the rule here is this library's reading).  samples = n: each cell's
 * overlap phi with a movable particle is the share of n^3 evenly spaced
 * points in the cell that lie inside the sphere.  Each step, a cell that is
 * fluid and stays fluid while the particle's move raised its overlap from
 * phi_old to phi_new hands the share (phi_new - phi_old) / (1 - phi_old) of
 * its stress, in equal parts, to its D3Q19 neighbours that stay fluid;
 * what a cell still holds when it is covered follows the binary rule.  The
 * total stress of the fluid is unchanged and the populations are not
 * touched.  0 (the default) is the binary conversion; 1 samples the cell
 * centre only and gives the binary conversion's bits through the smoothing
 * path.  VLB_EINVAL for samples outside 0..8.  Kept in checkpoints. */
vlb_status vlb_set_conversion_smoothing(vlb_lattice *lat, int32_t samples);

/* Counter-force for periodic systems with free particles (Section 4.5):
 * when on, every step subtracts the summed external force of the movable
 * particles from the body force, spread evenly over the cells that are
 * fluid when the step starts, so that fluid plus particle momentum stays
 * constant.  Off by default; kept in checkpoints. */
vlb_status vlb_set_counter_force(vlb_lattice *lat, int32_t on);

/* Rounding of stored values (default VLB_ROUND_STOCHASTIC, seed 0x2009). */
vlb_status vlb_set_rounding(vlb_lattice *lat, vlb_rounding mode, uint32_t seed);

/* Storage scale of FP16 populations from the largest flow speed expected
 * (a storage choice of this library; the method itself is precision
 * agnostic).  FP16 storage takes s = 2^k, the largest power of two up to
 * 2^24 with s * max(u_max, 1e-4) <= 64: the deviations of a flow at that
 * speed, at most about u_max, then sit three decades below FP16's largest
 * value, and deviations as small as 2^-14 / s (2e-9 for u_max = 1e-3) are
 * still normal FP16 numbers.  The state already stored is rescaled in place by the
 * power-of-two ratio (exact for every value that stays a normal FP16 number
 * at both scales).  FP32 and BF16 storage keep s = 1, since their exponent
 * range needs no scale; for them the call only checks u_max.  VLB_EINVAL for
 * a non-finite or non-positive u_max.  The scale is kept in checkpoints. */
vlb_status vlb_set_velocity_scale(vlb_lattice *lat, double u_max);

/* The storage scale s in use (1 for FP32 and BF16; 2^10 for FP16 unless
 * vlb_set_velocity_scale chose another); 0 for a NULL lattice. */
double vlb_storage_scale(const vlb_lattice *lat);

/* Control experiment for the storage layout (not part of the method): when
 * on, every step rounds each stored population f_i = w_i + h_i to the nearest
 * FP32 number right after stream-collide, which is what storing the raw
 * populations in FP32 would keep of them, so the deviations carry rounding
 * errors of the size of w_i's last place instead of their own.  FP32 storage
 * only (VLB_EINVAL otherwise); off by default and not kept in checkpoints. */
vlb_status vlb_set_raw_f32_control(vlb_lattice *lat, int32_t on);
double vlb_kernel_time_ms(const vlb_lattice *lat, int32_t which);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent solves (FP32 storage).
 *
 * A server owns a FIFO queue of requests, a set of slots and an arena: one
 * device allocation of the whole HBM budget, made at creation, from which
 * admitted solves take their buffers.  vlb_server_pump retires finished
 * solves (their velocity and stress are copied to the host), admits queued
 * requests in order while a slot is free and the request's footprint fits
 * in the budget and in a free range of the arena, and issues replays of
 * steps_per_launch batched steps that advance every admitted solve together
 * (a replayed hipGraph), keeping up to two replays in flight so that the
 * host's retire/admit work overlaps the GPU's.  Results are read into a
 * device buffer outside the budget (72 bytes per cell of the solves that
 * finish in one round, grown in stream order, never shrunk) and copied to
 * host memory after that round's replays are issued.  Requests submitted while
 * others run join at the next pump.  Each solve computes exactly what a lone
 * vlb_lattice with the same mask, parameters and rounding seed computes:
 * results do not depend on what else is in the batch.  Served solves are
 * Oldroyd-B or Giesekus (FENE-P is not served); walls in a request mask move
 * with the request's wall velocities (at rest by default); fixed spheres are
 * solid cells at rest; moving particles are not served.
 */
typedef enum vlb_request_state {
    VLB_REQ_QUEUED = 0,
    VLB_REQ_RUNNING = 1,
    VLB_REQ_DONE = 2,
    VLB_REQ_CANCELLED = 3,
    VLB_REQ_FAILED = 4
} vlb_request_state;

typedef struct vlb_request {
    vlb_dims dims;
    const uint8_t *mask;    /* N bytes: 0 fluid, 1..63 solid (wall id); copied      */
    vlb_params params;
    int32_t n_spheres;
    const double *spheres;  /* n_spheres x {cx, cy, cz, r}: fixed spheres, copied     */
    int64_t n_steps;
    uint32_t seed;          /* stochastic-rounding seed (vlb_set_rounding)           */
    double giesekus_alpha;  /* Giesekus mobility in [0, 1/2] (vlb_set_giesekus);
                               0 for Oldroyd-B                                       */
    int32_t n_walls;        /* 0..63: walls with ids 1..n_walls move; copied          */
    const double *wall_velocity; /* n_walls x 3: their velocities, as in vlb_create    */
} vlb_request;

typedef struct vlb_server_stats {
    int64_t submitted, completed, queued, running, launches, graph_captures, graph_updates;
    uint64_t bytes_in_use, cell_steps_launched;
} vlb_server_stats;

typedef struct vlb_server vlb_server;

/* hbm_budget_bytes bounds the summed footprint of admitted solves and is
 * allocated at once (VLB_ENOMEM if the device cannot hold it); max_slots
 * bounds their number (<= 4096); steps_per_launch is the number of batched
 * steps per replay (1..4096).  stream as for vlb_create (the server adds two
 * streams of its own for uploads, result reads and graph capture). */
vlb_status vlb_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t steps_per_launch,
                             void *stream, vlb_server **out);
/* Device bytes a request of these dimensions holds while admitted. */
size_t vlb_server_request_bytes(const vlb_dims *dims);
/* Rounding of stored values for every solve (only while idle). */
vlb_status vlb_server_set_rounding(vlb_server *srv, vlb_rounding mode);
/* Admission order of queued requests.  VLB_POLICY_FIFO (the default): in
 * submission order, no overtaking.  VLB_POLICY_SHORTEST_FIRST: the queued
 * request with the fewest cell-steps (cells x steps; ties in submission
 * order) first, which shortens the typical wait when requests queue up, at
 * the price of longer waits for the largest ones.  Either way a request is
 * admitted only when a slot and its memory are free, and its results do not
 * depend on the order.  May be changed at any time; VLB_EINVAL for an
 * unknown policy. */
typedef enum vlb_policy { VLB_POLICY_FIFO = 0, VLB_POLICY_SHORTEST_FIRST = 1 } vlb_policy;
vlb_status vlb_server_set_policy(vlb_server *srv, vlb_policy policy);
/* Queue a request (inputs copied).  VLB_EBUSY if it can never fit the budget,
 * VLB_EINVAL for invalid dimensions, mask or parameters. */
vlb_status vlb_server_submit(vlb_server *srv, const vlb_request *req, uint64_t *ticket);
/* One scheduling round: retire, admit, and top up to two replays in flight.
 * wait = 0 returns at once when two replays are in flight; wait = 1 first
 * waits for the oldest replay unless one has completed since the last call. */
vlb_status vlb_server_pump(vlb_server *srv, int32_t wait);
vlb_status vlb_server_poll(vlb_server *srv, uint64_t ticket, int32_t *state);
/* Copy the result of a finished request (u: 3*N, tau: 6*N doubles, either
 * may be NULL) and its latency from submission to completion, then forget
 * the request.  VLB_ESTATE if it has not finished. */
vlb_status vlb_server_result(vlb_server *srv, uint64_t ticket, double *u, double *tau,
                             double *latency_ms);
vlb_status vlb_server_cancel(vlb_server *srv, uint64_t ticket);
vlb_status vlb_server_stats_get(vlb_server *srv, vlb_server_stats *out);
const char *vlb_server_last_error(const vlb_server *srv);
void vlb_server_destroy(vlb_server *srv);

#ifdef __cplusplus
}
#endif
#endif
