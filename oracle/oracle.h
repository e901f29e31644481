/*
 * Plain FP64 CPU oracle for the lattice Boltzmann + Oldroyd-B method of
 * Kuron, Stewart, de Graaf and Holm (arXiv 2009.12279).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Layout of every field: cell index n = x + nx*(y + ny*z); a field with k
 * components is k consecutive planes of N = nx*ny*nz doubles.
 * Stress components are ordered xx, yy, zz, xy, xz, yz.
 * Populations use the oracle's own direction order, exposed by
 * or_velocity(); callers that exchange populations with another program
 * match directions by their velocity vectors.
 *
 * Mask byte per cell: 0 fluid; 1..63 wall id w (velocity wall_vel[w-1],
 * zero if w > n_walls); 64+k particle k (set only by or_add_sphere).
 */
#ifndef VLB_ORACLE_H
#define VLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_lattice or_lattice;

/* D3Q19 direction i of the oracle's order: velocity c[3], weight *w. Returns 19. */
int or_velocity(int i, int c[3], double *w);

/* Section 3.1, equilibrium with c_s^2 = 1/3: f_i^eq(rho, u), 19 values. */
void or_equilibrium(double rho, const double u[3], double feq[19]);

/* One cell of the collision (Section 3.1, TRT with Guo forcing):
 * f: 19 pre-collision populations, F: force density.  Outputs the
 * post-collision populations and the moments rho, u (u includes F/2). */
void or_collide_cell(const double f[19], const double F[3], double omega_plus,
                     double omega_minus, double fout[19], double *rho, double u[3]);

/* Relaxation rates from the total viscosity eta, polymer fraction beta and
 * the TRT parameter magic (magic < 0 selects BGK, omega- = omega+). */
void or_rates(double eta, double beta, double magic, double *omega_plus, double *omega_minus);

/* One explicit finite-volume update of the stress (Section 3.3) with a
 * prescribed velocity field u (3*N; at solid cells it is the boundary
 * velocity).  tau_out = tau_in + fluxes + source on fluid cells; solid cells
 * copy tau_in.  alpha > 0 adds the Giesekus term -(alpha/eta_p) tau.tau to
 * the source; L2 > 0 makes it FENE-P in the stored variable
 * T = (eta_p/lambda)(A - I) (relaxation -(f/lambda) T - (eta_p/lambda^2)(f-1) I,
 * f = (L2 - 3) / (L2 - tr A)). */
void or_fv_apply(int nx, int ny, int nz, const unsigned char *mask, const double *tau_in,
                 const double *u, double eta_p, double lambda_p, double alpha, double L2,
                 double *tau_out);

/* The discrete polymer force of Section 3.3 for a stress field (fluid cells). */
void or_polymer_force(int nx, int ny, int nz, const unsigned char *mask, const double *tau,
                      double *fp_out);
/* Same with the extrapolation into solid face neighbours of order 0
 * (constant, as above), 1 (linear through the cell behind, constant when
 * that cell is solid) or 2 (quadratic through the two cells behind, linear
 * when only the first of them is fluid). */
void or_polymer_force_ext(int nx, int ny, int nz, const unsigned char *mask, const double *tau,
                          int order, double *fp);

or_lattice *or_create(int nx, int ny, int nz, const int periodic[3], const unsigned char *mask,
                      const double *wall_vel, int n_walls);
void or_destroy(or_lattice *L);
/* Returns 0 on success, -1 for invalid parameters. */
int or_set_params(or_lattice *L, double eta, double beta, double lambda_p, double magic,
                  const double g[3]);
/* f = f^eq(1, u) on fluid cells (u = NULL: rest), tau = 0. */
/* Counter-force (Section 4.5): when on, the summed external force of the
 * movable particles is subtracted from the body force, spread evenly over
 * the cells that are fluid at the start of each step. */
void or_set_counter_force(or_lattice *L, int on);
/* Giesekus model with mobility alpha in [0, 1/2] (0 = Oldroyd-B, the
 * default); -1 for alpha out of range. */
int or_set_giesekus(or_lattice *L, double alpha);
/* FENE-P with extensibility L2 = L^2 > 3 (0 = off; the last of Giesekus and
 * FENE-P set wins).  The stored stress variable becomes
 * T = (eta_p/lambda)(A - I); or_set_stress sets T, or_read_stress returns
 * the polymer stress tau = f T + (eta_p/lambda)(f - 1) I. */
int or_set_fene_p(or_lattice *L, double L2);
/* Force density per cell (Section 3.1 Guo forcing with a force that varies
 * in space, as the four-roll mill of Section 4.4 needs): F holds 3*N values,
 * the x, y and z planes, added to the uniform body force at every fluid
 * cell.  NULL removes it. */
void or_set_force_field(or_lattice *L, const double *F);
/* Wall velocity per cell (Section 3.1 velocity boundary condition with a
 * wall velocity that varies along the wall): u holds 3*N values, the x, y
 * and z planes; when set, every wall cell (mask 1..63) moves with its own
 * entry instead of the per-id table.  NULL returns to the table. */
void or_set_wall_velocity_field(or_lattice *L, const double *u);
/* Stress extrapolation into solid face neighbours (Section 3.3): 0 constant
 * (default), 1 linear, 2 quadratic through the fluid cells behind (lower
 * where fewer of them are fluid); the traction on obstacles uses the same
 * face values.  -1 for other orders. */
int or_set_extrapolation(or_lattice *L, int order);
void or_init_equilibrium(or_lattice *L, const double *u);
void or_set_populations(or_lattice *L, const double *f);
void or_set_stress(or_lattice *L, const double *tau);
/* Returns the particle id, or -1 when the sphere overlaps a non-fluid cell. */
int or_add_sphere(or_lattice *L, const double center[3], double radius, double density_ratio,
                  int movable, const double f_ext[3], const double t_ext[3]);
void or_step(or_lattice *L, long n_steps);

void or_read_populations(const or_lattice *L, double *f);
void or_read_stress(const or_lattice *L, double *tau);
void or_read_mask(const or_lattice *L, unsigned char *mask);
/* Moments of the current state: rho = sum f, u = (sum f c + F/2)/rho with
 * F = g + F^p(tau).  Solid cells read 0. */
void or_read_density(const or_lattice *L, double *rho);
void or_read_velocity(const or_lattice *L, double *u);
void or_read_particle(const or_lattice *L, int id, double pos[3], double vel[3], double omega[3],
                      double force[3], double torque[3]);
/* Breakdown of the last step's particle force: momentum exchange, polymer
 * traction, conversion bookkeeping applied in that step. */
void or_read_particle_parts(const or_lattice *L, int id, double f_mex[3], double f_tau[3],
                            double f_conv[3]);
/* Population mass and momentum summed over fluid cells of the current state. */
void or_read_sums(const or_lattice *L, double *mass, double momentum[3]);
/* Last step's momentum exchange + polymer traction summed over wall links. */
void or_read_wall_force(const or_lattice *L, double force[3]);
/* Momentum still owed to particles by the last conversion (applied next step). */
void or_read_pending_conversion(const or_lattice *L, double momentum[3]);
/* Stress dropped because a covered cell had no fluid neighbour (6 values). */
void or_read_dropped_stress(const or_lattice *L, double tau[6]);
long or_step_count(const or_lattice *L);
/* Last conversion: counts[0] cells covered, counts[1] uncovered; the stress
 * summed over fluid cells just before and just after it. */
void or_read_conversion_stats(const or_lattice *L, int counts[2], double tau_before[6],
                              double tau_after[6]);
/* Overlap-fraction smoothing of conversions (Section 3.4): ns sub-samples
 * per axis of each cell's overlap with a moving particle, 1..8, or 0 for
 * the binary conversion (the default).  While a particle overlaps more of
 * a cell that stays fluid, the cell hands that share of its stress to its
 * neighbours that stay fluid.  -1 for ns outside 0..8. */
int or_set_conversion_smoothing(or_lattice *L, int ns);
/* Overlap fraction of cell (x, y, z) with particle id at its current
 * position, ns^3 sub-samples (-1 for an unknown id or ns < 1). */
double or_overlap_fraction(const or_lattice *L, int id, int x, int y, int z, int ns);
/* Number of threads the oracle's loops may use (OpenMP); 0 = runtime default. */
void or_set_threads(int n);
int or_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
