// Internal declarations shared by the host runtime and the gfx950 kernels of
// libvlb.  Not part of the public ABI (include/vlb.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace vlb {

constexpr int Q = 19;
constexpr int PART0 = 64;          // mask byte of particle 0
constexpr int MAX_PARTICLES = 192;
constexpr int BLOCK = 256;         // threads per block of the per-cell kernels

// D3Q19 in the public order: rest, 6 faces, 12 edges, opposite directions
// adjacent (i odd, i+1 is its opposite).
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
constexpr float WF[Q] = {1.f / 3.f,   1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                         1.f / 18.f,  1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                         1.f / 36.f,  1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                         1.f / 36.f,  1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
constexpr double WD[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                          1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Stress components xx, yy, zz, xy, xz, yz.  TROW[k][j] is the component index
// of tau_kj.
constexpr int TROW[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};

enum Storage : int { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

// Particle record, device resident, FP64 (Section 3.4).
struct Particle {
    double R[3], v[3], w[3];
    double radius, mass, inertia;
    int32_t movable, pad;
    double fext[3], text[3];
    double fconv[3], tconv[3];  // momentum owed by the last conversion
    double fmex[3], tmex[3];    // last step: momentum exchange
    double ftau[3], ttau[3];    // last step: polymer traction
    double ftot[3], ttot[3];    // last step: total applied
    double Rprev[3];            // position before the last update
};

// Geometry common to every kernel.
struct Geom {
    int32_t nx, ny, nz;
    int32_t per[3];
    uint32_t N;        // cells
    uint64_t plane;    // elements between consecutive planes of a field
    // division of a cell index by nx and by ny (set_divisors): multiplier and
    // the two shifts (low and second byte)
    uint32_t mx = 0, my = 0, shx = 0, shy = 0;
};

// Constants of the unsigned division by an invariant divisor d, 1 <= d < 2^31
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d), m = floor(2^32 (2^l - d) / d)
// + 1, s1 = min(l, 1), s2 = max(l - 1, 0), every 32-bit n has
// n / d = (t + ((n - t) >> s1)) >> s2, t = (m n) >> 32.
inline void divisor_constants(uint32_t d, uint32_t &m, uint32_t &sh)
{
    int l = 0;
    while ((uint64_t(1) << l) < d)
        ++l;
    m = static_cast<uint32_t>(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    const int s1 = l < 1 ? l : 1, s2 = l > 1 ? l - 1 : 0;
    sh = static_cast<uint32_t>(s1) | (static_cast<uint32_t>(s2) << 8);
}

inline void set_divisors(Geom &g)
{
    divisor_constants(static_cast<uint32_t>(g.nx), g.mx, g.shx);
    divisor_constants(static_cast<uint32_t>(g.ny), g.my, g.shy);
}

struct Bound {
    const double *wall_vel;  // [n_walls][3]
    int32_t n_walls;
    // per-cell wall velocity, planes [3][N]; when set it replaces wall_vel
    // for every wall cell
    const double *wall_field = nullptr;
    const Particle *parts;
    int32_t n_parts;
    int32_t moving;          // any moving wall or movable particle
    int32_t walls_move = 0;  // some wall moves (a nonzero table entry or a per-cell field)
    // overlap-fraction smoothing of conversions: sub-samples per axis of a
    // cell's overlap with a moving particle (0: binary conversion)
    int32_t smooth_ns = 0;
    // conversion in one block, particle after particle, even where the
    // particles' cells are far apart (VLB_CONV_SERIAL=1; the same bits)
    int32_t conv_serial = 0;
    // raw-FP32 storage control: after stream-collide, every population is
    // rounded to the FP32 grid of f rather than of f - w (FP32 storage only)
    int32_t raw_f32 = 0;
};

// Map from the stored stress variable to the polymer stress.  Identity for
// Oldroyd-B and Giesekus (l2m3 = 0).  FENE-P stores T = (eta_p/lambda)(A - I)
// of the conformation A; with g1 = f - 1 = c tr T / (l2m3 - c tr T),
// c = lambda/eta_p, l2m3 = L^2 - 3, the stress is T + g1 T + epl g1 I,
// epl = eta_p/lambda.
struct StressMap {
    float c = 0.f, l2m3 = 0.f, epl = 0.f;
    // extrapolation into a solid face neighbour: 0 this cell's stress, 1 linear
    // through the cell behind, 2 quadratic through the two cells behind (the
    // order drops where a cell behind is solid)
    int32_t extrap = 0;
};

struct StepArgs {
    Geom g;
    Bound b;
    const uint8_t *mask;
    const void *fin;
    void *fout;
    const float *tin;
    float *tout;
    float *u;                // 3 planes, u^n for the stress update
    // The same fields as one base pointer per plane (kernel arguments the
    // compiler keeps in scalar registers, so every access is scalar base +
    // 32-bit vector offset).
    const void *fin_p[Q];
    void *fout_p[Q];
    const float *tin_p[6];
    float *tout_p[6];
    float *u_p[3];
    double wp, wm;           // omega+, omega-
    double g3[3];            // body force density
    const double *g3_dev;    // body force read on the device instead (counter-force), or null
    // per-cell force density added to the body force: 3 planes laid out like
    // u, or null
    const float *gf_p[3] = {nullptr, nullptr, nullptr};
    double eta_p_lam, inv_lam;
    float scale, inv_scale;  // storage scale s and 1/s
    float gk;                // Giesekus alpha / eta_p (0: Oldroyd-B)
    StressMap sm;            // stored variable -> polymer stress (FENE-P)
    int32_t polymer;
    int32_t remap;           // XCD-aware block order (0 off, 1 ranges, 2 y-slabs)
    int32_t lb_remap;        // the same for stream-collide alone
    uint32_t slab_blocks;    // remap 2: blocks per XCD per z-plane
    int32_t stochastic;      // stochastic rounding of stored values
    uint32_t step;           // step index (random stream of the rounding); with
                             // step_dev, the offset added to *step_dev
    const uint32_t *step_dev = nullptr;  // base step read on the device (graph replays)
    // bytes from the input to the output population and stress buffers: the
    // fused step reaches its output planes as input plane + offset, so that
    // it keeps half as many plane pointers in scalar registers
    int64_t fdelta = 0, tdelta = 0;
    uint32_t seed;
};

// One solve of the batched (serving) step: step arguments for both buffer
// parities (index = step & 1), its block range and its step target.
struct BatchSolve {
    StepArgs args[2];
    uint32_t first_block;
    uint32_t nblocks;
    uint32_t target;
    // stress update: its block range, and 64 x 4 tiles marching through
    // chunks of fv_zc planes (fv_tiled) or one cell per thread
    uint32_t fv_tiled;
    uint32_t fv_first_block;
    uint32_t fv_nblocks;
    uint32_t fv_zc;
    uint32_t pad;
};

struct BatchTable {
    uint32_t n_solves;
    uint32_t total_blocks;
    const BatchSolve *solves;     // [n_solves]
    const uint32_t *block_solve;  // [total_blocks]
    uint32_t *steps;              // [n_solves], advanced on the device
    uint32_t fv_total_blocks;
    const uint32_t *fv_block_solve;  // [fv_total_blocks], stress-update blocks
};

// Stress-update blocks of a served solve: tiles (64 x 4, chunks of *zc
// planes) when it is at least 32 cells wide and 4 rows high, else one cell
// per thread.
uint32_t batch_fv_blocks(const Geom &g, bool *tiled, uint32_t *zc);

// Host-side launchers (vlb_kernels.hip).
// Counter-force: count the cells that are fluid now into *count, then
// g_out = g - (sum of the movable particles' F_ext) / count (g when none is
// movable), resetting *count.
hipError_t launch_body_force(const Geom &g, const uint8_t *mask, const Particle *parts,
                             int n_parts, const double body_force[3], uint32_t *count,
                             double *g_out, hipStream_t s);
hipError_t launch_lb_step(int storage, const StepArgs &a, hipStream_t s);
// Round the FP32 deviations at f (Q planes) so that w_i + h_i is an FP32 number.
hipError_t launch_raw_f32_control(const Geom &g, void *f, hipStream_t s);
// n_steps batched steps (stream-collide, stress update, counter advance per
// step) over every solve of the table: stream-collide on max_blocks blocks
// of BLOCK threads, the stress update on fv_blocks blocks of 64 x 4.
// Base step of graph replays: *step = value, or *step += value (add != 0).
hipError_t launch_set_step(uint32_t *step, uint32_t value, int add, hipStream_t s);
hipError_t launch_batch_step(const BatchTable *t, uint32_t max_blocks, uint32_t fv_blocks,
                             int stochastic, int n_steps, hipStream_t s);
// tile_rows 4 or 8 selects the tiled kernel (64 x tile_rows tiles marching
// through z_chunk planes, 0 = 16) where the lattice is large enough for it,
// -4 or -8 the tiled kernel for any lattice; anything else the per-cell
// kernel.
hipError_t launch_fv_step(int storage, const StepArgs &a, hipStream_t s, int tile_rows,
                          uint32_t z_chunk);
// Fused stream-collide + stress update of one step (64 x 4 tiles marching
// through chunks of z_chunk planes, 0 = 32, shortened to fill the chip) for a
// polymer lattice large enough to fill the chip with such tiles, or any
// polymer lattice when forced; hipErrorNotSupported, with nothing launched,
// otherwise.  step_fused_fits tells which without launching.  It gives the
// bits of the two-kernel step; on MI355X it is slower (the ring of
// neighbour velocities it recomputes costs more than the velocity round
// trip it saves), so the step runs it only when asked.
bool step_fused_fits(const Geom &g, uint32_t z_chunk, bool force, uint32_t *zc_out);
hipError_t launch_step_fused(int storage, const StepArgs &a, hipStream_t s, uint32_t z_chunk,
                             bool force);
hipError_t launch_init_equilibrium(int storage, const Geom &g, const uint8_t *mask,
                                   const double *u, void *f, float scale, hipStream_t s);
// Multiply `count` FP16 values at f by the power of two `factor`.
hipError_t launch_rescale_f16(void *f, uint64_t count, float factor, hipStream_t s);
hipError_t launch_set_populations(int storage, const Geom &g, const uint8_t *mask,
                                  const double *f_in, void *f, float scale, hipStream_t s);
hipError_t launch_set_stress(const Geom &g, const uint8_t *mask, const double *tau_in,
                             float *tau, hipStream_t s);
// gfield: per-cell force density planes (stride g.plane) added to gvec, or
// null.  Cells first .. first + count - 1 (count 0: every cell from 0) go to
// rho_out[k] and u_out[a * count + k], k = n - first.
hipError_t launch_read_moments(int storage, const Geom &g, const Bound &b, const uint8_t *mask,
                               const void *f, const float *tau, int polymer, const float gvec[3],
                               const float *gfield, float inv_scale, double *rho_out,
                               double *u_out, hipStream_t s, const StressMap &sm = StressMap{},
                               uint32_t first = 0, uint32_t count = 0);
hipError_t launch_read_populations(int storage, const Geom &g, const uint8_t *mask, const void *f,
                                   float inv_scale, double *out, hipStream_t s);
hipError_t launch_read_stress(const Geom &g, const uint8_t *mask, const float *tau, double *out,
                              hipStream_t s, const StressMap &sm = StressMap{});
// FP64 population mass/momentum + health (max speed, non-finite count):
// partial sums per block into `partials` (nblocks x 6), then a final pass
// into out[6] = {mass_dev, px, py, pz, max_speed, non_finite}.
int sums_blocks(const Geom &g);
hipError_t launch_sums(int storage, const Geom &g, const uint8_t *mask, const void *f,
                       float inv_scale, double *partials, double *out, hipStream_t s);
// Per-particle momentum exchange + polymer traction over each particle's
// bounding box (PF_BLOCKS blocks per particle, block sums into `partials`,
// MAX_PARTICLES x PF_BLOCKS x 12 doubles), then per particle the fixed-order
// FP64 sum, the totals and the symplectic Euler update of movable particles.
constexpr int PF_BLOCKS = 32;
hipError_t launch_particle_forces(int storage, const Geom &g, const uint8_t *mask, const void *f,
                                  const float *tau_n, int polymer, float inv_scale,
                                  Particle *parts, int n_parts, double *partials, hipStream_t s,
                                  const StressMap &sm = StressMap{});
// Same over wall links of the whole lattice into out[3] (two-stage).
hipError_t launch_wall_force(int storage, const Geom &g, const uint8_t *mask, const void *f,
                             const float *tau_n, int polymer, float inv_scale, double *partials,
                             double *out, hipStream_t s, const StressMap &sm = StressMap{});
// Fluid/solid conversion around every movable particle.  scratch: 3 float
// planes (stride g.plane) the smoothing may overwrite (the step's velocity
// planes, dead by then); owner: g.N bytes for the new owner of the cells
// near the particles.
hipError_t launch_conversion(int storage, const Geom &g, const Bound &b, uint8_t *mask, void *f,
                             float *tau, float scale, float inv_scale, int32_t *counters,
                             float *scratch, uint8_t *owner, hipStream_t s);

}  // namespace vlb
