// gfx950 kernels of libvlb: the per-cell lattice Boltzmann + Oldroyd-B step
// and its boundary, particle, diagnostic and readout kernels.
//
// Population layout ("pull" addressing): the pre-collision population f_i of
// fluid cell x lives in plane i at cell x - c_i, stored as a deviation from
// the lattice weight, h = s * (f_i - w_i).  The stream-collide kernel for cell
// x therefore gathers f_i from (x - c_i, i) and writes its post-collision
// populations to its own cell.  When x + c_j is solid, the population leaving
// along c_j is reflected (Section 3.1, velocity boundary condition) and
// written straight into the slot (x + c_j, opposite j), which is exactly
// where the pull of the next step looks for it; solid cells own no data of
// their own, so every slot has a single writer and the pull needs no branch.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <type_traits>

#include "vlb_internal.h"

namespace vlb {
namespace {

// ---------------------------------------------------------------------------
// Random bits for stochastic rounding: a 32-bit integer hash of (cell, step,
// seed) seeds a per-thread xorshift32 sequence; every call yields two signed
// 16-bit uniforms.

__device__ __forceinline__ uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

struct Rng {
    uint32_t s;
    __device__ __forceinline__ Rng(uint32_t cell, uint32_t step, uint32_t seed)
        : s(hash32(cell * 0x9e3779b1u ^ hash32(step * 0x85ebca77u + seed)) | 1u)
    {
    }
    // next state of the hardware pseudo-random sequence (one instruction)
    __device__ __forceinline__ uint32_t next32()
    {
        s = __builtin_amdgcn_prng_b32(s);
        return s;
    }
};

// the two signed 16-bit halves of a 32-bit random word, each in [-2^15, 2^15)
__device__ __forceinline__ int32_t rhi(uint32_t r) { return static_cast<int32_t>(r) >> 16; }
__device__ __forceinline__ int32_t rlo(uint32_t r) { return static_cast<int32_t>(r << 16) >> 16; }

// Stochastic rounding as dither-then-round-to-nearest: adding a uniform
// offset in [-1/2, 1/2) of the target format's spacing at x and rounding to
// nearest selects the upper neighbour with probability equal to the distance
// from the lower one.
__device__ __forceinline__ float sr_f32(double x, int32_t r16)
{
    // One FP32 spacing is 2^29 units in the last place of an FP64 value of
    // the same binade, so adding r16 * 2^13 to the bit pattern dithers x by
    // [-1/2, 1/2) of an FP32 spacing; the conversion then rounds to nearest.
    // |x| below 1e-300 (only ever exact zeros here) is passed through.
    const int64_t dither = static_cast<int64_t>(r16) * (int64_t(1) << 13);
    const double xd = __longlong_as_double(__double_as_longlong(x) + dither);
    return fabs(x) < 1e-300 ? static_cast<float>(x) : static_cast<float>(xd);
}

__device__ __forceinline__ float sr_f16_dither(float x, int32_t r16)
{
    uint32_t e = (__float_as_uint(x) >> 23) & 0xffu;
    e = e < 113u ? 113u : e;  // below 2^-14 the FP16 spacing is 2^-24
    const float scale = __uint_as_float((e - 26u) << 23);  // spacing * 2^-16
    return fmaf(static_cast<float>(r16), scale, x);
}

// Streaming store: every population is written once per step and read once
// in the next step, long after it would have left the caches.
template <class T>
__device__ __forceinline__ void st_stream(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------------------
// storage codecs: deviation h = s * (f - w) in FP32, FP16 or BF16.
// st() rounds to nearest; st_sr() rounds stochastically with the 16-bit
// uniform r16, which removes the systematic bias round-to-nearest leaves in
// a slowly relaxing steady state.  The scale s is 1 for FP32 and BF16 (the
// library never sets another), so their codecs skip the multiplications; FP16
// takes a power of two chosen per lattice.

template <int S>
struct Store;

template <>
struct Store<ST_F32> {
    using T = float;
#ifdef VLB_F32_REGS
    using R = float;  // measurement build: FP32 registers for FP32 storage
#else
    using R = double;  // register type of the per-cell arithmetic
#endif
    static __device__ __forceinline__ float ld(const T *p, uint64_t i, float)
    {
        return p[i];
    }
    template <class V>
    static __device__ __forceinline__ void st(T *p, uint64_t i, V v, float)
    {
        st_stream(p + i, static_cast<float>(v));
    }
    template <class V>
    static __device__ __forceinline__ void st_sr(T *p, uint64_t i, V v, float, int32_t r16)
    {
        if constexpr (sizeof(V) == 8)
            st_stream(p + i, sr_f32(v, r16));
        else
            st_stream(p + i, static_cast<float>(v));
    }
};

template <>
struct Store<ST_F16> {
    using T = __half;
    using R = float;
    static __device__ __forceinline__ float ld(const T *p, uint64_t i, float inv)
    {
        return __half2float(p[i]) * inv;
    }
    template <class V>
    static __device__ __forceinline__ void st(T *p, uint64_t i, V v, float s)
    {
        p[i] = __float2half_rn(static_cast<float>(v) * s);
    }
    template <class V>
    static __device__ __forceinline__ void st_sr(T *p, uint64_t i, V v, float s, int32_t r16)
    {
        p[i] = __float2half_rn(sr_f16_dither(static_cast<float>(v) * s, r16));
    }
};

template <>
struct Store<ST_BF16> {
    using T = uint16_t;
    using R = float;
    static __device__ __forceinline__ float ld(const T *p, uint64_t i, float)
    {
        return __uint_as_float(static_cast<uint32_t>(p[i]) << 16);
    }
    template <class V>
    static __device__ __forceinline__ void st(T *p, uint64_t i, V v, float)
    {
        // round to nearest even on the upper 16 bits
        uint32_t b = __float_as_uint(static_cast<float>(v));
        b += 0x7fffu + ((b >> 16) & 1u);
        p[i] = static_cast<uint16_t>(b >> 16);
    }
    template <class V>
    static __device__ __forceinline__ void st_sr(T *p, uint64_t i, V v, float, int32_t r16)
    {
        // uniform bits added below the kept 16 bits, then truncation
        const uint32_t b = __float_as_uint(static_cast<float>(v)) +
                           static_cast<uint32_t>(r16 + 32768);
        p[i] = static_cast<uint16_t>(b >> 16);
    }
};

template <int S, bool SR, class V>
__device__ __forceinline__ void store(typename Store<S>::T *p, uint64_t i, V v, float s, int32_t r16)
{
    if constexpr (SR)
        Store<S>::st_sr(p, i, v, s, r16);
    else
        Store<S>::st(p, i, v, s);
}

// Element `idx` of one plane addressed as (uniform plane base) + (32-bit byte
// offset), which maps to the scalar-base / vector-offset addressing form and
// keeps one VGPR per access instead of a 64-bit address.  The host
// guarantees every field plane is below 4 GiB.
template <class T>
__device__ __forceinline__ const T *elem(const T *plane, uint32_t idx)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(plane) +
                                       idx * static_cast<uint32_t>(sizeof(T)));
}
template <class T>
__device__ __forceinline__ T *elem(T *plane, uint32_t idx)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(plane) +
                                 idx * static_cast<uint32_t>(sizeof(T)));
}

// plane-addressed loads/stores of populations (deviation h = s (f - w))
template <int S>
__device__ __forceinline__ float ldp(const typename Store<S>::T *plane, uint32_t idx, float inv)
{
    return Store<S>::ld(elem(plane, idx), 0, inv);
}
template <int S, bool SR, class V>
__device__ __forceinline__ void stp(typename Store<S>::T *plane, uint32_t idx, V v, float s,
                                   int32_t r16)
{
    store<S, SR>(elem(plane, idx), 0, v, s, r16);
}

// ---------------------------------------------------------------------------
// indexing

// Block order.  The hardware hands block b to XCD b % 8, each XCD with its
// own L2.  remap 1: each XCD takes one contiguous range of blocks.  remap 2
// (used when a z-plane splits into 8 equal runs of whole blocks): XCD k
// takes the k-th y-slab of every plane and sweeps it plane by plane, so the
// three planes a stencil touches (z-1, z, z+1) of one slab stay in that
// XCD's L2 while they are reused.
__device__ __forceinline__ uint32_t block_id(int remap, uint32_t slab_blocks)
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    if (remap == 2) {
        const uint32_t k = b & 7u, q = b >> 3;
        const uint32_t z = q / slab_blocks, j = q - z * slab_blocks;
        return z * (8u * slab_blocks) + k * slab_blocks + j;
    }
    if (remap != 1)
        return b;
    const uint32_t per = G >> 3;
    if (b >= per * 8u)
        return b;
    return (b & 7u) * per + (b >> 3);
}

// Wrapped neighbour coordinates of one cell: C[0] = coordinate - 1,
// C[1] = coordinate, C[2] = coordinate + 1, and the matching index offsets.
struct Nbr {
    int xc[3], yc[3], zc[3];
    uint32_t xo[3], yo[3], zo[3];
    __device__ __forceinline__ Nbr(const Geom &g, int x, int y, int z)
    {
        xc[0] = x == 0 ? g.nx - 1 : x - 1;
        xc[1] = x;
        xc[2] = x == g.nx - 1 ? 0 : x + 1;
        yc[0] = y == 0 ? g.ny - 1 : y - 1;
        yc[1] = y;
        yc[2] = y == g.ny - 1 ? 0 : y + 1;
        zc[0] = z == 0 ? g.nz - 1 : z - 1;
        zc[1] = z;
        zc[2] = z == g.nz - 1 ? 0 : z + 1;
        const uint32_t nxy = static_cast<uint32_t>(g.nx) * g.ny;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xo[k] = xc[k];
            yo[k] = yc[k] * static_cast<uint32_t>(g.nx);
            zo[k] = zc[k] * nxy;
        }
    }
    __device__ __forceinline__ uint32_t at(int cx, int cy, int cz) const
    {
        return xo[cx + 1] + yo[cy + 1] + zo[cz + 1];
    }
};

// n / d from the constants of divisor_constants
__device__ __forceinline__ uint32_t div_by(uint32_t n, uint32_t m, uint32_t sh)
{
    const uint32_t t = __umulhi(m, n);
    return (t + ((n - t) >> (sh & 0xffu))) >> (sh >> 8);
}

__device__ __forceinline__ void coords(const Geom &g, uint32_t n, int &x, int &y, int &z)
{
    const uint32_t t = div_by(n, g.mx, g.shx);
    x = static_cast<int>(n - t * static_cast<uint32_t>(g.nx));
    const uint32_t q = div_by(t, g.my, g.shy);
    y = static_cast<int>(t - q * static_cast<uint32_t>(g.ny));
    z = static_cast<int>(q);
}

// displacement from the particle centre to a cell, minimum image on periodic axes
__device__ __forceinline__ void lever(const Geom &g, const Particle &P, int x, int y, int z,
                                      double r[3])
{
#pragma clang fp contract(off)
    const double pos[3] = {static_cast<double>(x), static_cast<double>(y), static_cast<double>(z)};
    const int len[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double d = pos[k] - P.R[k];
        if (g.per[k]) {
            const double L = static_cast<double>(len[k]);
            d -= L * floor(d / L + 0.5);
        }
        r[k] = d;
    }
}

// Section 3.4: velocity of a solid node, v + omega x (r_b - R) for a movable
// particle; for a wall cell its entry of the per-cell field when one is set,
// else the velocity of its wall id; zero otherwise.
__device__ void boundary_velocity_d(const Geom &g, const Bound &b, uint8_t m, int x, int y, int z,
                                    double ub[3])
{
    ub[0] = ub[1] = ub[2] = 0.0;
    if (m < PART0) {
        if (m >= 1 && b.wall_field) {
            const uint32_t n = static_cast<uint32_t>(x) +
                               static_cast<uint32_t>(g.nx) *
                                   (static_cast<uint32_t>(y) + static_cast<uint32_t>(g.ny) * z);
            ub[0] = b.wall_field[n];
            ub[1] = b.wall_field[g.N + n];
            ub[2] = b.wall_field[2ull * g.N + n];
        } else if (m >= 1 && m <= b.n_walls) {
            ub[0] = b.wall_vel[3 * (m - 1) + 0];
            ub[1] = b.wall_vel[3 * (m - 1) + 1];
            ub[2] = b.wall_vel[3 * (m - 1) + 2];
        }
        return;
    }
    const Particle &P = b.parts[m - PART0];
    if (!P.movable)
        return;
    double r[3];
    lever(g, P, x, y, z, r);
    ub[0] = P.v[0] + P.w[1] * r[2] - P.w[2] * r[1];
    ub[1] = P.v[1] + P.w[2] * r[0] - P.w[0] * r[2];
    ub[2] = P.v[2] + P.w[0] * r[1] - P.w[1] * r[0];
}

// deterministic block sum (fixed shuffle tree, then fixed order over waves);
// the result is valid in thread 0
template <int NT>
__device__ double block_sum(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k)
            r += sh[k];
    return r;
}

// The same for K values at once with a single barrier: each value takes the
// shuffle tree and the fixed wave order of block_sum, so the sums are the
// same bits.  sh holds K * NT / 64 doubles; the results are valid in
// thread 0.
template <int NT, int K>
__device__ void block_sums(double (&v)[K], double *sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            v[k] += __shfl_down(v[k], off, 64);
        if (lane == 0)
            sh[k * (NT / 64) + wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double r = 0.0;
            for (int w = 0; w < NT / 64; ++w)
                r += sh[k * (NT / 64) + w];
            v[k] = r;
        }
}

template <int NT>
__device__ double block_max(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = fmax(v, __shfl_down(v, off, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k)
            r = fmax(r, sh[k]);
    return r;
}

// ---------------------------------------------------------------------------
// Stream-collide (Section 3.1) with the polymer force of Section 3.3.
// Arithmetic in R (FP64 for FP32 storage, FP32 for half storage); the pulled
// populations stay in FP32 registers (exact) to keep occupancy up.

// Index deltas to the six face neighbours with periodic wrap, so that the
// neighbour along (cx, cy, cz) is n + dx[cx+1] + dy[cy+1] + dz[cz+1].
struct Delta {
    int32_t dx[3], dy[3], dz[3];
    __device__ __forceinline__ Delta(const Geom &g, int x, int y, int z)
    {
        const int32_t nx = g.nx, nxy = g.nx * g.ny, nxyz = nxy * g.nz;
        dx[0] = x == 0 ? nx - 1 : -1;
        dx[1] = 0;
        dx[2] = x == g.nx - 1 ? 1 - nx : 1;
        dy[0] = y == 0 ? nxy - nx : -nx;
        dy[1] = 0;
        dy[2] = y == g.ny - 1 ? nx - nxy : nx;
        dz[0] = z == 0 ? nxyz - nxy : -nxy;
        dz[1] = 0;
        dz[2] = z == g.nz - 1 ? nxy - nxyz : nxy;
    }
    __device__ __forceinline__ uint32_t at(uint32_t n, int cx, int cy, int cz) const
    {
        return static_cast<uint32_t>(static_cast<int32_t>(n) + dx[cx + 1] + dy[cy + 1] + dz[cz + 1]);
    }
    // same for offsets only known at run time (selects, no indexed arrays)
    __device__ __forceinline__ uint32_t at_rt(uint32_t n, int cx, int cy, int cz) const
    {
        const int32_t ox = cx < 0 ? dx[0] : (cx > 0 ? dx[2] : 0);
        const int32_t oy = cy < 0 ? dy[0] : (cy > 0 ? dy[2] : 0);
        const int32_t oz = cz < 0 ? dz[0] : (cz > 0 ? dz[2] : 0);
        return static_cast<uint32_t>(static_cast<int32_t>(n) + ox + oy + oz);
    }
};

// Runtime-indexed copies of the velocity set for the rare boundary path.
__constant__ int8_t kCX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__constant__ int8_t kCY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__constant__ int8_t kCZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

// Polymer stress component `comp` of cell m from the stored variable, in
// FP64 (readouts, obstacle forces): the identity, or for FENE-P
// T (1 + g1) + epl g1 I with g1 = f - 1 = c tr T / (l2m3 - c tr T).
__device__ __forceinline__ double mapped_stress(const StressMap &sm, const float *tau,
                                                uint64_t plane, uint32_t m, int comp)
{
    const double t = tau[comp * plane + m];
    if (!(sm.l2m3 > 0.f))
        return t;
    const double c = sm.c;
    const double tr = static_cast<double>(tau[m]) + static_cast<double>(tau[plane + m]) +
                      static_cast<double>(tau[2 * plane + m]);
    const double g1 = c * tr / (static_cast<double>(sm.l2m3) - c * tr);
    return t * (1.0 + g1) + (comp < 3 ? static_cast<double>(sm.epl) * g1 : 0.0);
}

// Stress that fluid cell nb.at(0, 0, 0) extrapolates into its solid face
// neighbour along c = (cx, cy, cz) (Section 3.3): the polynomial through the
// cell and the fluid cells behind it, evaluated one cell ahead, of degree
// sm.extrap at most (0 the cell's own stress, 1 linear, 2 quadratic) and
// lower where a cell behind is solid.
__device__ double extrap_stress(const Geom &g, const uint8_t *mask, const float *tau,
                                const StressMap &sm, const Nbr &nb, int cx, int cy, int cz,
                                int comp)
{
    const double own = mapped_stress(sm, tau, g.plane, nb.at(0, 0, 0), comp);
    if (!sm.extrap)
        return own;
    const uint32_t b1 = nb.at(-cx, -cy, -cz);
    if (mask[b1] != 0)
        return own;
    const double t1 = mapped_stress(sm, tau, g.plane, b1, comp);
    if (sm.extrap >= 2) {
        const Nbr nb1(g, nb.xc[1 - cx], nb.yc[1 - cy], nb.zc[1 - cz]);
        const uint32_t b2 = nb1.at(-cx, -cy, -cz);
        if (mask[b2] == 0)
            return 3.0 * own - 3.0 * t1 + mapped_stress(sm, tau, g.plane, b2, comp);
    }
    return 2.0 * own - t1;
}

// Field-wise copies of the geometry and boundary descriptors, for argument
// blocks that live in the constant address space (the implicit copy
// constructor cannot bind to those).
template <class G>
__device__ __forceinline__ Geom geom_copy(const G &g)
{
    Geom r;
    r.nx = g.nx;
    r.ny = g.ny;
    r.nz = g.nz;
    r.per[0] = g.per[0];
    r.per[1] = g.per[1];
    r.per[2] = g.per[2];
    r.N = g.N;
    r.plane = g.plane;
    r.mx = g.mx;
    r.my = g.my;
    r.shx = g.shx;
    r.shy = g.shy;
    return r;
}
template <class B>
__device__ __forceinline__ Bound bound_copy(const B &b)
{
    Bound r;
    r.wall_vel = b.wall_vel;
    r.n_walls = b.n_walls;
    r.wall_field = b.wall_field;
    r.parts = b.parts;
    r.n_parts = b.n_parts;
    r.moving = b.moving;
    r.walls_move = b.walls_move;
    r.smooth_ns = b.smooth_ns;
    return r;
}

// Bounce-back for every link of cell n into a solid cell (Section 3.1
// velocity boundary condition): the post-collision population just stored
// for direction j is reflected, with the moving-wall term, into the slot of
// the solid cell that the next pull of this cell reads.  `links` has bit j
// set for each solid neighbour along c_j.
template <int S, bool SR, class R, class A>
__device__ void reflect_links(const A &a, typename Store<S>::T *fout, uint32_t n,
                              const Delta &d, uint32_t links, R rho, Rng &rng)
{
    const Geom g = geom_copy(a.g);
    const Bound bnd = bound_copy(a.b);
    const uint64_t P = g.plane;
    while (links) {
        const int j = __builtin_ctz(links);
        links &= links - 1;
        const int cx = kCX[j], cy = kCY[j], cz = kCZ[j];
        const uint32_t m = d.at_rt(n, cx, cy, cz);
        R val = static_cast<R>(ldp<S>(fout + j * P, n, a.inv_scale));
        if (bnd.moving) {
            int x, y, z;
            coords(g, m, x, y, z);
            double ub[3];
            boundary_velocity_d(g, bnd, a.mask[m], x, y, z, ub);
            const double w = (cx * cx + cy * cy + cz * cz == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
            val -= R(6) * static_cast<R>(w) * rho * static_cast<R>(cx * ub[0] + cy * ub[1] + cz * ub[2]);
        }
        const int o = (j & 1) ? j + 1 : j - 1;  // opposite direction (pairs are adjacent)
        stp<S, SR>(fout + o * P, m, val, a.scale, rhi(rng.next32()));
    }
}

// Occupancy targets of the step kernels (waves per SIMD), overridable at
// build time for measurements.
#ifdef VLB_LB_WAVES
#define LB_OCCUPANCY(S) __attribute__((amdgpu_waves_per_eu(VLB_LB_WAVES)))
#else
// At least 5 waves per SIMD (at most 96 VGPRs) for 16-bit storage and 4
// (at most 128 VGPRs, a 20-byte spill) for FP32 storage with FP64
// arithmetic: both measured faster than the compiler's own choice (4 and 3
// waves)
#define LB_OCCUPANCY(S) __attribute__((amdgpu_waves_per_eu((S) == ST_F32 ? 4 : 5)))
#endif
#ifdef VLB_FV_WAVES
#define FV_OCCUPANCY __attribute__((amdgpu_waves_per_eu(VLB_FV_WAVES)))
#else
#define FV_OCCUPANCY
#endif

// Plane addresses of the step kernels.  ArgPlanes: the argument block's own
// plane pointers.  BasePlanes (fused step): every plane from one base
// pointer per buffer and the plane stride, output planes at a fixed offset
// from the input ones; the fused kernel hides the base from the optimiser
// once per plane, so that the plane addresses are formed where they are
// used instead of being held in scalar registers across the whole loop.
template <class A>
struct ArgPlanes {
    const A &a;
    __device__ __forceinline__ const void *fin(int i) const { return a.fin_p[i]; }
    __device__ __forceinline__ void *fout(int i) const { return a.fout_p[i]; }
    __device__ __forceinline__ const float *tin(int c) const { return a.tin_p[c]; }
    __device__ __forceinline__ float *tout(int c) const { return a.tout_p[c]; }
};

struct BasePlanes {
    const char *f;   // input population buffer
    uint64_t fpb;    // bytes per population plane
    int64_t fdelta;  // output population buffer - input
    const char *t;   // input stress buffer
    uint64_t tpb;    // bytes per stress plane
    int64_t tdelta;  // output stress buffer - input
    __device__ __forceinline__ const void *fin(int i) const { return f + i * fpb; }
    __device__ __forceinline__ void *fout(int i) const
    {
        return const_cast<char *>(f) + i * fpb + fdelta;
    }
    __device__ __forceinline__ const float *tin(int c) const
    {
        return reinterpret_cast<const float *>(t + c * tpb);
    }
    __device__ __forceinline__ float *tout(int c) const
    {
        return reinterpret_cast<float *>(const_cast<char *>(t) + c * tpb + tdelta);
    }
};

// Inputs of one cell's stream-collide, all loaded before any is used: the
// 19 pulled populations, which neighbours are solid (and which of those are
// particles), and the stored stress of the cell and of its face neighbours.
template <bool FENE>
struct LbIn {
    float f[Q];
    uint32_t links, plinks;  // bit j: the neighbour along c_j is solid / a particle
    float town[6];           // the cell's stored stress variable
    float tn[3][2][3];       // row k of the stored stress of the neighbours along +/- e_k
    float tdg[3][2][2];      // FENE-P: those neighbours' other two diagonal entries
};

// Issue every load of cell n's stream-collide (all addresses are in bounds,
// also for solid cells, so a wave has all its memory requests in flight at
// once).  ALL_LINKS: the solid flag of all 18 neighbours (bounce-back);
// otherwise only of the six face neighbours (enough for the polymer force).
template <int S, bool FENE, bool ALL_LINKS, class A, class PL>
__device__ __forceinline__ void lb_load(const A &a, const PL &pl, uint32_t n, const Delta &d,
                                        LbIn<FENE> &in)
{
    using T = typename Store<S>::T;
    const uint8_t *__restrict__ mask = a.mask;
    // pull: f_i(x) sits in plane i at x - c_i
#pragma unroll
    for (int i = 0; i < Q; ++i)
        in.f[i] = ldp<S>(static_cast<const T *>(pl.fin(i)), d.at(n, -CX[i], -CY[i], -CZ[i]),
                         a.inv_scale);
    in.links = 0;
    in.plinks = 0;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        if (!ALL_LINKS && j > 6)
            continue;
        const uint8_t mj = mask[d.at(n, CX[j], CY[j], CZ[j])];
        in.links |= (mj != 0 ? 1u : 0u) << j;
        in.plinks |= (mj >= PART0 ? 1u : 0u) << j;
    }
    if (a.polymer) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            in.town[c] = *elem(pl.tin(c), n);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int sg = side == 0 ? 1 : -1;
                const uint32_t m = d.at(n, sg * (k == 0), sg * (k == 1), sg * (k == 2));
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    in.tn[k][side][j] = *elem(pl.tin(TROW[k][j]), m);
                if (FENE) {
                    in.tdg[k][side][0] = *elem(pl.tin((k + 1) % 3), m);
                    in.tdg[k][side][1] = *elem(pl.tin((k + 2) % 3), m);
                }
            }
    }
}

// Force density on fluid cell n: body force (the device value under the
// counter-force), per-cell force field, and the polymer force (Section 3.3):
// the sum over faces of the face-averaged stress times the outward normal, a
// solid face neighbour taking the extrapolated stress of this cell, formed in
// FP32 (a difference of stresses, small next to the populations).  With
// FENE-P the stored variables in `in` are mapped to the polymer stress in
// place.
template <class R, bool FENE, class A>
__device__ __forceinline__ void lb_force(const A &a, uint32_t n, const Delta &d, LbIn<FENE> &in,
                                         R F[3])
{
    // contraction within an expression only (same bits wherever inlined)
#pragma clang fp contract(on)
    const Geom g = geom_copy(a.g);
    const uint8_t *__restrict__ mask = a.mask;
    const uint32_t links = in.links;
    float Fp[3] = {0.f, 0.f, 0.f};
    if (a.polymer) {
        if (FENE) {
            // polymer stress from the stored variable: T (1 + g1) + epl g1 I,
            // g1 = c tr T / (l2m3 - c tr T), at this cell and its neighbours
            const float c = a.sm.c, l2m3 = a.sm.l2m3, epl = a.sm.epl;
            const float tr0 = in.town[0] + in.town[1] + in.town[2];
            const float g0 = c * tr0 / (l2m3 - c * tr0);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const float tr = in.tn[k][side][k] + in.tdg[k][side][0] + in.tdg[k][side][1];
                    const float g1 = c * tr / (l2m3 - c * tr);
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        in.tn[k][side][j] = fmaf(in.tn[k][side][j], g1, in.tn[k][side][j]) +
                                            (j == k ? epl * g1 : 0.f);
                }
#pragma unroll
            for (int q = 0; q < 6; ++q)
                in.town[q] = fmaf(in.town[q], g0, in.town[q]) + (q < 3 ? epl * g0 : 0.f);
        }
        // face bits of `links`: +x 1, -x 2, +y 3, -y 4, +z 5, -z 6
        if (a.sm.extrap && ((links >> 1) & 63u)) {
            // linear or quadratic extrapolation into solid face neighbours
            // through the fluid cells behind (rare path)
            StressMap smc;
            smc.c = a.sm.c;
            smc.l2m3 = a.sm.l2m3;
            smc.epl = a.sm.epl;
            smc.extrap = a.sm.extrap;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const bool sp = (links >> (2 * k + 1)) & 1u, sm = (links >> (2 * k + 2)) & 1u;
                // quadratic: the cell two behind the solid face, if fluid
                float t2[3] = {0.f, 0.f, 0.f};
                bool quad = false;
                if (smc.extrap >= 2 && sp != sm) {
                    const int sg = sp ? -1 : 1;  // from the cell toward the fluid behind it
                    const int cx = sg * (k == 0), cy = sg * (k == 1), cz = sg * (k == 2);
                    const uint32_t m1 = d.at_rt(n, cx, cy, cz);
                    int x1, y1, z1;
                    coords(g, m1, x1, y1, z1);
                    const Delta d1(g, x1, y1, z1);
                    const uint32_t m2 = d1.at_rt(m1, cx, cy, cz);
                    if (mask[m2] == 0) {
                        quad = true;
                        for (int j = 0; j < 3; ++j)
                            t2[j] = static_cast<float>(
                                mapped_stress(smc, a.tin, g.plane, m2, TROW[k][j]));
                    }
                }
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float own = in.town[TROW[k][j]];
                    const float ep = quad ? fmaf(3.f, own - in.tn[k][1][j], t2[j])
                                          : 2.f * own - in.tn[k][1][j];
                    const float em = quad ? fmaf(3.f, own - in.tn[k][0][j], t2[j])
                                          : 2.f * own - in.tn[k][0][j];
                    const float vp = sp ? (sm ? own : ep) : in.tn[k][0][j];
                    const float vm = sm ? (sp ? own : em) : in.tn[k][1][j];
                    Fp[j] += 0.5f * (vp - vm);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const bool sp = (links >> (2 * k + 1)) & 1u, sm = (links >> (2 * k + 2)) & 1u;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float own = in.town[TROW[k][j]];
                    Fp[j] += 0.5f * ((sp ? own : in.tn[k][0][j]) - (sm ? own : in.tn[k][1][j]));
                }
            }
        }
    }
    // body force: the device value under the counter-force (uniform branch)
    double g3[3];
    if (a.g3_dev) {
        g3[0] = a.g3_dev[0];
        g3[1] = a.g3_dev[1];
        g3[2] = a.g3_dev[2];
    } else {
        g3[0] = a.g3[0];
        g3[1] = a.g3[1];
        g3[2] = a.g3[2];
    }
    if (a.gf_p[0]) {
        // per-cell force density (uniform branch)
        g3[0] += static_cast<double>(*elem(a.gf_p[0], n));
        g3[1] += static_cast<double>(*elem(a.gf_p[1], n));
        g3[2] += static_cast<double>(*elem(a.gf_p[2], n));
    }
    F[0] = static_cast<R>(g3[0]) + static_cast<R>(Fp[0]);
    F[1] = static_cast<R>(g3[1]) + static_cast<R>(Fp[1]);
    F[2] = static_cast<R>(g3[2]) + static_cast<R>(Fp[2]);
}

// Moments in deviation form from opposite-pair sums and differences
// (Section 3.1 with the half force): rho = 1 + h_0 + sum (h_i + h_o),
// rho u = sum c_i (h_i - h_o) + F/2.
template <class R>
struct Moments {
    R drho, rho, ux, uy, uz;
};

template <class R>
__device__ __forceinline__ Moments<R> lb_moments(const float f[Q], const R F[3])
{
    // contraction within an expression only, so that the stream-collide of a
    // cell and the moments of the same cell computed elsewhere (the ring of
    // a fused step) give the same bits
#pragma clang fp contract(on)
    R drho = static_cast<R>(f[0]), jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int k = 0; k < Q / 2; ++k) {
        const int i = 2 * k + 1;
        const R a_ = static_cast<R>(f[i]), b_ = static_cast<R>(f[i + 1]);
        drho += a_ + b_;
        const R df = a_ - b_;
        if (CX[i])
            jx += CX[i] * df;
        if (CY[i])
            jy += CY[i] * df;
        if (CZ[i])
            jz += CZ[i] * df;
    }
    Moments<R> m;
    m.drho = drho;
    m.rho = R(1) + drho;
    const R inv_rho = R(1) / m.rho;
    m.ux = (jx + R(0.5) * F[0]) * inv_rho;
    m.uy = (jy + R(0.5) * F[1]) * inv_rho;
    m.uz = (jz + R(0.5) * F[2]) * inv_rho;
    return m;
}

// Velocity u^n of cell n at (x, y, z) alone (the moments of its
// stream-collide, no stores): into uo, and the cell's stored stress
// variable into to (zero without polymer).  Returns false for a solid cell
// (uo zero).
template <int S, bool FENE, class A, class PL>
__device__ __forceinline__ bool lb_velocity(const A &a, const PL &pl, uint32_t n, int x, int y,
                                            int z, float uo[3], float to[6])
{
    using R = typename Store<S>::R;
    const Geom g = geom_copy(a.g);
    const Delta d(g, x, y, z);
    LbIn<FENE> in;
    lb_load<S, FENE, false>(a, pl, n, d, in);
#pragma unroll
    for (int c = 0; c < 6; ++c)
        to[c] = a.polymer ? in.town[c] : 0.f;
    if (a.mask[n] != 0) {
        uo[0] = uo[1] = uo[2] = 0.f;
        return false;
    }
    R F[3];
    lb_force<R, FENE>(a, n, d, in, F);
    const Moments<R> mo = lb_moments<R>(in.f, F);
    uo[0] = static_cast<float>(mo.ux);
    uo[1] = static_cast<float>(mo.uy);
    uo[2] = static_cast<float>(mo.uz);
    return true;
}

// Stream-collide of cell n at (x, y, z) of the lattice described by `a`, at
// step `step` (the step only seeds the rounding stream).  Arithmetic in R
// (FP64 for FP32 storage, FP32 for half storage); the pulled populations
// stay in FP32 registers (exact) to keep occupancy up.  FUSED: the velocity
// and the cell's stored stress go to uo / to (for a fused stress update)
// instead of the velocity planes, and the output planes are reached from
// the input planes.  Returns false for a solid cell.
template <int S, bool SR, bool FENE, bool FUSED, class A, class PL>
__device__ __forceinline__ bool lb_cell(const A &a, const PL &pl, uint32_t n, int x, int y, int z,
                                        uint32_t step, float uo[3], float to[6])
{
    const Geom g = geom_copy(a.g);
    using St = Store<S>;
    using T = typename St::T;
    using R = typename St::R;
    const Delta d(g, x, y, z);
    auto out_plane = [&](int i) -> T * { return static_cast<T *>(pl.fout(i)); };
    LbIn<FENE> in;
    lb_load<S, FENE, true>(a, pl, n, d, in);
    if (FUSED) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            to[c] = a.polymer ? in.town[c] : 0.f;
    }
    if (a.mask[n] != 0) {
        if (FUSED)
            uo[0] = uo[1] = uo[2] = 0.f;
        return false;
    }
    R F[3];
    lb_force<R, FENE>(a, n, d, in, F);
    const R Fx = F[0], Fy = F[1], Fz = F[2];
    const Moments<R> mo = lb_moments<R>(in.f, F);
    const R drho = mo.drho, rho = mo.rho, ux = mo.ux, uy = mo.uy, uz = mo.uz;
    auto pop = [&](int i) -> float { return in.f[i]; };
    const uint32_t links = in.links, plinks = in.plinks;
    const R uu = ux * ux + uy * uy + uz * uz;
    const R uF = ux * Fx + uy * Fy + uz * Fz;
    const R wp = static_cast<R>(a.wp), wm = static_cast<R>(a.wm);
    const R cp = R(1) - R(0.5) * wp, cm = R(1) - R(0.5) * wm;

    // TRT with Guo forcing, written per opposite pair (i, o) with s = h_i + h_o
    // and d = h_i - h_o as
    //   f*+ = (1-w+) s/2 + w+ f^eq+ + (1-w+/2) S+,  f*- = (1-w-) d/2 + w- f^eq- + (1-w-/2) S-
    // with f^eq+ = w (drho + rho (9/2 (c.u)^2 - 3/2 u.u)),  f^eq- = 3 w rho c.u,
    //      S+ = w (9 (c.u)(c.F) - 3 u.F),                    S- = 3 w c.F,
    // i.e. f*+ = a1 s + w (P1 + c.u (Q1 c.u + C9 c.F)),  f*- = b1 d + w (M3 c.u + C3 c.F).
    const R a1 = R(0.5) * (R(1) - wp), b1 = R(0.5) * (R(1) - wm);
    const R P1 = wp * (drho - R(1.5) * rho * uu) - R(3) * cp * uF;
    const R Q1 = R(4.5) * wp * rho, C9 = R(9) * cp;
    const R M3 = R(3) * wm * rho, C3 = R(3) * cm;
    // Bounce-back (Section 3.1 velocity boundary condition): a link into a
    // solid cell sends the post-collision population of its direction into
    // the slot of the opposite direction at the solid cell, which the next
    // pull of this cell reads.  Links into walls at rest are written from
    // registers right after the population; links that need the moving-wall
    // term (into moving walls, or into particles when some particle moves)
    // go through reflect_links afterwards.  With 16-bit storage every link
    // takes the reload path: the extra live registers of the register path
    // push the kernel past the register budget of five waves per SIMD, and
    // the spills cost more than the reloads save.
    const uint32_t slow = S != ST_F32 ? links
                                      : (a.b.moving ? (a.b.walls_move ? links : plinks) : 0u);
    const uint32_t fast = links & ~slow;
    Rng rng(n, step, a.seed);
    stp<S, SR>(out_plane(0), n,
               R(2) * a1 * static_cast<R>(pop(0)) + static_cast<R>(WD[0]) * P1, a.scale,
               rhi(rng.next32()));
    // one 32-bit random word per opposite pair, a 16-bit half each
#pragma unroll
    for (int k = 0; k < Q / 2; ++k) {
        const int i = 2 * k + 1, o = i + 1;
        const R w = static_cast<R>(WD[i]);
        const R a_ = static_cast<R>(pop(i)), b_ = static_cast<R>(pop(o));
        const R cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const R cF = CX[i] * Fx + CY[i] * Fy + CZ[i] * Fz;
        const R np = a1 * (a_ + b_) + w * (P1 + cu * (Q1 * cu + C9 * cF));
        const R nm = b1 * (a_ - b_) + w * (M3 * cu + C3 * cF);
        T *pi = out_plane(i);
        T *po = out_plane(o);
        const uint32_t r = rng.next32();
        stp<S, SR>(pi, n, np + nm, a.scale, rhi(r));
        stp<S, SR>(po, n, np - nm, a.scale, rlo(r));
        if (fast & ((1u << i) | (1u << o))) {
            if ((fast >> i) & 1u)
                stp<S, SR>(po, d.at(n, CX[i], CY[i], CZ[i]), np + nm, a.scale, rhi(rng.next32()));
            if ((fast >> o) & 1u)
                stp<S, SR>(pi, d.at(n, CX[o], CY[o], CZ[o]), np - nm, a.scale, rhi(rng.next32()));
        }
    }

    if (slow)
        reflect_links<S, SR>(a, static_cast<T *>(a.fout), n, d, slow, rho, rng);

    if (FUSED) {
        uo[0] = static_cast<float>(ux);
        uo[1] = static_cast<float>(uy);
        uo[2] = static_cast<float>(uz);
    } else if (a.polymer) {
        *elem(a.u_p[0], n) = static_cast<float>(ux);
        *elem(a.u_p[1], n) = static_cast<float>(uy);
        *elem(a.u_p[2], n) = static_cast<float>(uz);
    }
    return true;
}

template <int S, bool SR, bool FENE>
__global__ __launch_bounds__(BLOCK) LB_OCCUPANCY(S) void lb_step_kernel(StepArgs a)
{
    const uint32_t n = block_id(a.lb_remap, a.slab_blocks) * BLOCK + threadIdx.x;
    if (n >= a.g.N)
        return;
    int x, y, z;
    coords(a.g, n, x, y, z);
    lb_cell<S, SR, FENE, false>(a, ArgPlanes<StepArgs>{a}, n, x, y, z,
                                a.step_dev ? *a.step_dev + a.step : a.step, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// Finite-volume Oldroyd-B stress update (Section 2.2 source, Section 3.3).
// The increment (fluxes + source, products of small quantities) is formed in
// FP32; it is added to the stored stress in FP64 and rounded once.

// Stress update of fluid cell n at (x, y, z) from its own velocity and stress
// (u0, t0) and those of its six face neighbours (un, tn: [axis k][side], side 0
// along +e_k, side 1 along -e_k), `solid` holding bit 2k+side for each solid
// face neighbour.  Shared by the per-cell and the tiled kernels, so both give
// the same bits.  LAW selects the constitutive law at compile time: 0
// Oldroyd-B, 1 Giesekus, 2 FENE-P.
constexpr int LAW_OB = 0, LAW_GIESEKUS = 1, LAW_FENE = 2;
template <bool SR, int LAW, class A, class PL>
__device__ __forceinline__ void fv_compute(const PL &pl, const A &a, const Geom &g, uint32_t n, int x, int y, int z,
                                           uint32_t step, const float u0[3], const float t0[6],
                                           float un[3][2][3], const float tn[3][2][6],
                                           uint32_t solid)
{
    // Contraction only within an expression (and spelled out with fmaf where
    // it matters), so that every kernel this is inlined into computes the
    // same bits.
#pragma clang fp contract(on)
    // Face fluxes: the fraction of a cell moving with velocity v that crosses
    // its face along +/- e_k in one step is max(+/- v_k, 0) times the
    // product of (1 - |v_a|) over the two transverse axes a.  fo: out of this
    // cell through face (k, side); fi: into it from the neighbour there.
    float fo[3][2], fi[3][2];
    const float om[3] = {1.f - fabsf(u0[0]), 1.f - fabsf(u0[1]), 1.f - fabsf(u0[2])};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a1 = k == 0 ? 1 : 0, a2 = k == 2 ? 1 : 2;
        const float p0 = om[a1] * om[a2];
        fo[k][0] = fmaxf(u0[k], 0.f) * p0;
        fo[k][1] = fmaxf(-u0[k], 0.f) * p0;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const float *v = un[k][side];
            const float pn = (1.f - fabsf(v[a1])) * (1.f - fabsf(v[a2]));
            fi[k][side] = fmaxf(side == 0 ? -v[k] : v[k], 0.f) * pn;
        }
    }
    if (solid) {
        // no flux through a solid face; its velocity (zero for walls at
        // rest) enters the gradient below
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int side = 0; side < 2; ++side)
                if ((solid >> (2 * k + side)) & 1u) {
                    fo[k][side] = 0.f;
                    fi[k][side] = 0.f;
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        un[k][side][j] = 0.f;
                }
    }
    float G[3][3];
    float in_sum[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float out_tot = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            out_tot += fo[k][side];
#pragma unroll
            for (int c = 0; c < 6; ++c)
                in_sum[c] = fmaf(fi[k][side], tn[k][side][c], in_sum[c]);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            G[k][j] = 0.5f * (un[k][0][j] - un[k][1][j]);
    }
    if (solid && a.b.moving) {
        const Bound bnd = bound_copy(a.b);
        const Delta d(g, x, y, z);
        // velocity gradient with the boundary velocity at solid face neighbours
        while (solid) {
            const int b = __builtin_ctz(solid);
            solid &= solid - 1;
            const int k = b >> 1, s = (b & 1) ? -1 : 1;
            const uint32_t m = d.at_rt(n, s * (k == 0), s * (k == 1), s * (k == 2));
            int mx, my, mz;
            coords(g, m, mx, my, mz);
            double ub[3];
            boundary_velocity_d(g, bnd, a.mask[m], mx, my, mz, ub);
            const float hs = 0.5f * s;
            for (int j = 0; j < 3; ++j) {
                const float gj = hs * static_cast<float>(ub[j]);
                if (k == 0)
                    G[0][j] += gj;
                else if (k == 1)
                    G[1][j] += gj;
                else
                    G[2][j] += gj;
            }
        }
    }
    // source: sum_k tau_ik G_kj + sum_k tau_kj G_ki + eta_p/lam (G_ij + G_ji) - tau_ij/lam
    const float T3[3][3] = {{t0[0], t0[3], t0[4]}, {t0[3], t0[1], t0[5]}, {t0[4], t0[5], t0[2]}};
    const int PI[6] = {0, 1, 2, 0, 0, 1};
    const int PJ[6] = {0, 1, 2, 1, 2, 2};
    const float epl = static_cast<float>(a.eta_p_lam), il = static_cast<float>(a.inv_lam);
    const float gk = a.gk;
    // FENE-P: relaxation -(1 + g0) T / lambda - epl g0 / lambda I of the stored
    // variable, g0 = f - 1 from this cell's trace
    float g0 = 0.f;
    if constexpr (LAW == LAW_FENE) {
        const float fl2m3 = a.sm.l2m3, fc = a.sm.c, tr = t0[0] + t0[1] + t0[2];
        g0 = fc * tr / (fl2m3 - fc * tr);
    }
    Rng rng(n, step, a.seed ^ 0x5bd1e995u);
    uint32_t r = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int i = PI[c], j = PJ[c];
        float sdot = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            sdot = fmaf(T3[k][j], G[k][i], fmaf(T3[i][k], G[k][j], sdot));
        float inc = fmaf(-out_tot, t0[c], in_sum[c]) + sdot;
        inc = fmaf(epl, G[i][j] + G[j][i], inc);
        inc = fmaf(-t0[c], il, inc);
        if constexpr (LAW == LAW_FENE) {
            inc = fmaf(-t0[c] * g0, il, inc);
            if (c < 3)
                inc = fmaf(-epl * g0, il, inc);
        }
        if constexpr (LAW == LAW_GIESEKUS) {
            // Giesekus: -(alpha / eta_p) (tau . tau)_ij
            float tt = 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                tt = fmaf(T3[i][k], T3[k][j], tt);
            inc = fmaf(-gk, tt, inc);
        }
        const double v = static_cast<double>(t0[c]) + static_cast<double>(inc);
        if (!(c & 1))
            r = rng.next32();
        stp<ST_F32, SR>(pl.tout(c), n, v, 1.f, (c & 1) ? rlo(r) : rhi(r));
    }
}

// Per-cell stress update: every neighbour value is loaded from memory.
template <bool SR, int LAW, class A>
__device__ __forceinline__ void fv_cell(const A &a, uint32_t n, uint32_t step)
{
    const Geom g = geom_copy(a.g);
    const uint8_t *__restrict__ mask = a.mask;
    int x, y, z;
    coords(g, n, x, y, z);
    const Delta d(g, x, y, z);
    // all loads first (in bounds for every cell), selection afterwards
    const float u0[3] = {*elem(a.u_p[0], n), *elem(a.u_p[1], n), *elem(a.u_p[2], n)};
    float t0[6];
#pragma unroll
    for (int c = 0; c < 6; ++c)
        t0[c] = *elem(a.tin_p[c], n);
    float un[3][2][3], tn[3][2][6];
    uint32_t solid = 0;  // bit 2k+side: face neighbour along +/- e_k is solid
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int s = side == 0 ? 1 : -1;
            const uint32_t m = d.at(n, s * (k == 0), s * (k == 1), s * (k == 2));
            solid |= (mask[m] != 0 ? 1u : 0u) << (2 * k + side);
#pragma unroll
            for (int j = 0; j < 3; ++j)
                un[k][side][j] = *elem(a.u_p[j], m);
#pragma unroll
            for (int c = 0; c < 6; ++c)
                tn[k][side][c] = *elem(a.tin_p[c], m);
        }
    if (mask[n] != 0)
        return;
    fv_compute<SR, LAW>(ArgPlanes<A>{a}, a, g, n, x, y, z, step, u0, t0, un, tn, solid);
}

template <bool SR, int LAW>
__global__ __launch_bounds__(BLOCK) FV_OCCUPANCY void fv_step_kernel(StepArgs a)
{
    const uint32_t n = block_id(a.remap, a.slab_blocks) * BLOCK + threadIdx.x;
    if (n >= a.g.N)
        return;
    fv_cell<SR, LAW>(a, n, a.step_dev ? *a.step_dev + a.step : a.step);
}

// ---------------------------------------------------------------------------
// Counter-force for periodic systems with free particles (Section 4.5): the
// fluid cells are counted at the start of the step, then the movable
// particles' external forces are spread evenly over them.

__global__ __launch_bounds__(BLOCK) void fluid_count_kernel(Geom g, const uint8_t *mask,
                                                            uint32_t *count)
{
    // 16 mask bytes per load (the mask allocation is 256-byte aligned); the
    // last N % 16 bytes by the first thread
    const uint32_t nvec = g.N / 16u;
    const uint4 *m4 = reinterpret_cast<const uint4 *>(mask);
    uint32_t c = 0;
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < nvec; k += gridDim.x * BLOCK) {
        const uint4 v = m4[k];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                c += ((w[q] >> (8 * b)) & 0xffu) == 0u ? 1u : 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (uint32_t n = nvec * 16u; n < g.N; ++n)
            c += mask[n] == 0 ? 1u : 0u;
    // integer sums: the result does not depend on the order.  One atomic
    // per block: per-wave atomics on the one counter serialise in L2.
    __shared__ uint32_t ws[BLOCK / 64];
    for (int off = 32; off > 0; off >>= 1)
        c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0)
        ws[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < BLOCK / 64; ++w)
            t += ws[w];
        if (t)
            atomicAdd(count, t);
    }
}

__global__ void body_force_kernel(const Particle *parts, int n_parts, double g0, double g1,
                                  double g2, uint32_t *count, double *g_out)
{
    double F[3] = {0.0, 0.0, 0.0};
    bool any = false;
    for (int p = 0; p < n_parts; ++p) {
        if (!parts[p].movable)
            continue;
        any = true;
        for (int a = 0; a < 3; ++a)
            F[a] += parts[p].fext[a];
    }
    const uint32_t nf = *count;
    const double g[3] = {g0, g1, g2};
    for (int a = 0; a < 3; ++a)
        g_out[a] = (any && nf) ? g[a] - F[a] / static_cast<double>(nf) : g[a];
    *count = 0;
}

// ---------------------------------------------------------------------------
// Tiled stress update.  A block owns an FV_TX x TY tile of the x-y plane and
// marches through a chunk of z-planes.  The velocity, stress and solid flag
// of the thread's own column ride along in registers for planes z-1, z and
// z+1 (the z neighbours); plane z of the tile plus a one-cell ring is staged
// in LDS for the x and y neighbours.  Every slot holds the cell at the
// periodically wrapped coordinates, as the per-cell kernel's index deltas do.
// Per cell a thread issues its own 10 loads, plus one ring cell for about
// half of the threads, instead of the per-cell kernel's 70.

constexpr int FV_TX = 64;
constexpr int FV_NV = 10;  // u (3), tau (6), solid flag

__device__ __forceinline__ int wrap_coord(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

template <class A>
__device__ __forceinline__ void fv_load(const A &a, uint32_t idx, float v[FV_NV])
{
#pragma unroll
    for (int j = 0; j < 3; ++j)
        v[j] = *elem(a.u_p[j], idx);
#pragma unroll
    for (int c = 0; c < 6; ++c)
        v[3 + c] = *elem(a.tin_p[c], idx);
    v[9] = a.mask[idx] != 0 ? 1.f : 0.f;
}

// LDS of one tiled stress-update block: two planes of the tile plus its ring.
template <int TY>
using FvTileLds = float[2][FV_NV][(FV_TX + 2) * (TY + 2)];

// Tile b (x tile, y tile, z chunk of zc planes) of the stress update of the
// lattice described by `a`, by the FV_TX x TY threads of a block (thread
// tid); every thread of the block calls it.  `remap`: XCD-aware order of the
// tiles (each XCD a slab of y tiles of every chunk) when the y tiles split
// into 8 equal slabs.
template <bool SR, int LAW, int TY, class A>
__device__ __forceinline__ void fv_tile_block(const A &a, uint32_t b, uint32_t zc, uint32_t step,
                                              bool remap, int tid, FvTileLds<TY> &lds)
{
    static_assert(FV_TX * TY >= 2 * FV_TX + 2 * TY, "ring larger than the block");
    constexpr int W = FV_TX + 2;
    const Geom g = geom_copy(a.g);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t nxy = static_cast<uint32_t>(nx) * ny;
    const uint32_t tiles_x = (nx + FV_TX - 1) / FV_TX, tiles_y = (ny + TY - 1) / TY;
    uint32_t tx, ty, cz;
    if (remap && (tiles_y & 7u) == 0) {
        const uint32_t y8 = tiles_y >> 3, k = b & 7u, q = b >> 3, per = tiles_x * y8;
        cz = q / per;
        const uint32_t r = q - cz * per;
        ty = k * y8 + r / tiles_x;
        tx = r % tiles_x;
    } else {
        tx = b % tiles_x;
        const uint32_t t = b / tiles_x;
        ty = t % tiles_y;
        cz = t / tiles_y;
    }
    const int lx = tid % FV_TX, ly = tid / FV_TX;
    const int x = static_cast<int>(tx) * FV_TX + lx, y = static_cast<int>(ty) * TY + ly;
    const bool in_tile = x < nx && y < ny;
    const uint32_t own_xy = wrap_coord(x, nx) + static_cast<uint32_t>(nx) * wrap_coord(y, ny);
    const int own_slot = (ly + 1) * W + lx + 1;
    // ring cell loaded by this thread, if any
    int hslot = -1;
    uint32_t halo_xy = 0;
    if (tid < 2 * FV_TX) {
        const int top = tid >= FV_TX, hx = static_cast<int>(tx) * FV_TX + (tid % FV_TX);
        const int hy = top ? static_cast<int>(ty) * TY + TY : static_cast<int>(ty) * TY - 1;
        hslot = (top ? TY + 1 : 0) * W + (tid % FV_TX) + 1;
        halo_xy = wrap_coord(hx, nx) + static_cast<uint32_t>(nx) * wrap_coord(hy, ny);
    } else if (tid < 2 * FV_TX + 2 * TY) {
        const int j = tid - 2 * FV_TX, right = j >= TY, r = j % TY;
        const int hx = right ? static_cast<int>(tx) * FV_TX + FV_TX : static_cast<int>(tx) * FV_TX - 1;
        const int hy = static_cast<int>(ty) * TY + r;
        hslot = (r + 1) * W + (right ? W - 1 : 0);
        halo_xy = wrap_coord(hx, nx) + static_cast<uint32_t>(nx) * wrap_coord(hy, ny);
    }
    const int z0 = static_cast<int>(cz * zc);
    const int z1 = min(z0 + static_cast<int>(zc), nz);
    // own column at z-1, z, z+1 and the ring cell at z
    float P[FV_NV], C[FV_NV], N[FV_NV], HV[FV_NV];
    fv_load(a, own_xy + wrap_coord(z0 - 1, nz) * nxy, P);
    fv_load(a, own_xy + static_cast<uint32_t>(z0) * nxy, C);
    fv_load(a, own_xy + wrap_coord(z0 + 1, nz) * nxy, N);
    if (hslot >= 0)
        fv_load(a, halo_xy + static_cast<uint32_t>(z0) * nxy, HV);
    for (int z = z0; z < z1; ++z) {
        const int buf = (z - z0) & 1;
#pragma unroll
        for (int v = 0; v < FV_NV; ++v)
            lds[buf][v][own_slot] = C[v];
        if (hslot >= 0) {
#pragma unroll
            for (int v = 0; v < FV_NV; ++v)
                lds[buf][v][hslot] = HV[v];
        }
        // the column at z+2 is in flight while this plane is computed
        const bool more = z + 1 < z1;
        float NN[FV_NV];
        if (more)
            fv_load(a, own_xy + static_cast<uint32_t>(z + 2 < nz ? z + 2 : z + 2 - nz) * nxy, NN);
        __syncthreads();
        if (in_tile && C[9] == 0.f) {
            const float u0[3] = {C[0], C[1], C[2]};
            const float t0[6] = {C[3], C[4], C[5], C[6], C[7], C[8]};
            float un[3][2][3], tn[3][2][6];
            uint32_t solid = 0;
            const int sl[2][2] = {{own_slot + 1, own_slot - 1}, {own_slot + W, own_slot - W}};
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int q = sl[k][side];
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        un[k][side][j] = lds[buf][j][q];
#pragma unroll
                    for (int c = 0; c < 6; ++c)
                        tn[k][side][c] = lds[buf][3 + c][q];
                    solid |= (lds[buf][9][q] != 0.f ? 1u : 0u) << (2 * k + side);
                }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                un[2][0][j] = N[j];
                un[2][1][j] = P[j];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                tn[2][0][c] = N[3 + c];
                tn[2][1][c] = P[3 + c];
            }
            solid |= (N[9] != 0.f ? 1u : 0u) << 4;
            solid |= (P[9] != 0.f ? 1u : 0u) << 5;
            const uint32_t n = own_xy + static_cast<uint32_t>(z) * nxy;
            fv_compute<SR, LAW>(ArgPlanes<A>{a}, a, g, n, x, y, z, step, u0, t0, un, tn, solid);
        }
        if (more) {
#pragma unroll
            for (int v = 0; v < FV_NV; ++v) {
                P[v] = C[v];
                C[v] = N[v];
                N[v] = NN[v];
            }
            // the ring cell of the next plane (LDS buffer buf^1 is free: every
            // thread has passed this plane's barrier)
            if (hslot >= 0)
                fv_load(a, halo_xy + static_cast<uint32_t>(z + 1) * nxy, HV);
        }
    }
}

template <bool SR, int LAW, int TY>
__global__ __launch_bounds__(FV_TX * TY) FV_OCCUPANCY void fv_tile_kernel(StepArgs a, uint32_t zc)
{
    __shared__ FvTileLds<TY> lds;
    const uint32_t step = a.step_dev ? *a.step_dev + a.step : a.step;
    fv_tile_block<SR, LAW, TY>(a, blockIdx.x, zc, step, a.remap != 0, static_cast<int>(threadIdx.x),
                               lds);
}

// ---------------------------------------------------------------------------
// Fused step: stream-collide and stress update in one pass.  The stress
// update of a cell needs the velocity u^n of its six face neighbours, which
// the same step computes; instead of a round trip through HBM the block
// computes what it needs itself.  A block owns a 64 x TY tile of the x-y
// plane and marches through a chunk of z-planes.  For plane z it runs the
// stream-collide of its tile cells, computes only the moments (u^n) of the
// one-cell ring of x-y face neighbours around the tile from their pulled
// populations (the same code the owner runs, so the same bits), and stages
// velocity, stored stress and solid flag of tile and ring in LDS.  The stress
// update of plane z - 1 follows, from the staged planes z - 2, z - 1 and z.
// The tile's columns at the planes just outside the chunk get moments only.
// Per cell HBM sees the populations read and written once, the stress read
// once and written once and the mask: the algorithmic bytes; the ring's
// pulls are L2 hits on data the neighbouring tiles read.
//
// LDS holds three planes: the write of plane z + 1 can then overlap the
// stress update of plane z - 1 in other waves, so one barrier per plane
// suffices (a thread reads other threads' slots only in plane z - 1, and
// its own slot in planes z - 2 and z).


#ifdef VLB_STEP_WAVES
#define STEP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(VLB_STEP_WAVES)))
#else
// Three waves per SIMD, the most the three LDS planes of a 256-thread block
// allow (at most 168 VGPRs; the compiler's own choice is two)
#define STEP_OCCUPANCY __attribute__((amdgpu_waves_per_eu(3)))
#endif

template <int S, bool SR, int LAW, int TX, int TY>
__global__ __launch_bounds__(TX * TY) STEP_OCCUPANCY void step_tile_kernel(StepArgs a, uint32_t zc)
{
    constexpr bool FENE = LAW == LAW_FENE;
    constexpr int W = TX + 2, SL = W * (TY + 2);
    constexpr int NRING = 2 * TX + 2 * TY;
    static_assert(NRING <= TX * TY, "ring larger than the block");
    __shared__ float lds[3][FV_NV][SL];
    const Geom g = a.g;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t nxy = static_cast<uint32_t>(nx) * ny;
    const uint32_t tiles_x = (nx + TX - 1) / TX, tiles_y = (ny + TY - 1) / TY;
    // block -> (x tile, y tile, z chunk); with the XCD-aware order each of the
    // 8 XCDs takes a slab of y tiles of every chunk, so the ring rows pulled
    // from neighbouring tiles are read through its own L2
    uint32_t tx, ty, cz;
    const uint32_t b = blockIdx.x;
    if (a.remap && (tiles_y & 7u) == 0) {
        const uint32_t y8 = tiles_y >> 3, k = b & 7u, q = b >> 3, per = tiles_x * y8;
        cz = q / per;
        const uint32_t r = q - cz * per;
        ty = k * y8 + r / tiles_x;
        tx = r % tiles_x;
    } else {
        tx = b % tiles_x;
        const uint32_t t = b / tiles_x;
        ty = t % tiles_y;
        cz = t / tiles_y;
    }
    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const int x = static_cast<int>(tx) * TX + lx, y = static_cast<int>(ty) * TY + ly;
    const bool in_tile = x < nx && y < ny;
    // slots of lanes past the lattice's edge hold the periodically wrapped
    // cell, as the neighbour deltas of the per-cell kernels do
    const int wx = wrap_coord(x, nx), wy = wrap_coord(y, ny);
    const uint32_t own_xy = wx + static_cast<uint32_t>(nx) * wy;
    const int own_slot = (ly + 1) * W + lx + 1;
    // ring cell of this thread, if any: thread r takes ring cell r, so the
    // ring's moments occupy as few waves as possible (a wave issues the same
    // instructions however many of its lanes are active)
    int rslot = -1, rx = 0, ry = 0;
    uint32_t ring_xy = 0;
    {
        const int r = tid;
        if (r < NRING) {
            const int x0 = static_cast<int>(tx) * TX, y0 = static_cast<int>(ty) * TY;
            int hx, hy;
            if (r < 2 * TX) {
                const int top = r >= TX, c = r % TX;
                hx = x0 + c;
                hy = top ? y0 + TY : y0 - 1;
                rslot = (top ? TY + 1 : 0) * W + c + 1;
            } else {
                const int j = r - 2 * TX, right = j >= TY, row = j % TY;
                hx = right ? x0 + TX : x0 - 1;
                hy = y0 + row;
                rslot = (row + 1) * W + (right ? W - 1 : 0);
            }
            rx = wrap_coord(hx, nx);
            ry = wrap_coord(hy, ny);
            ring_xy = rx + static_cast<uint32_t>(nx) * ry;
        }
    }
    const int z0 = static_cast<int>(cz * zc);
    const int z1 = min(z0 + static_cast<int>(zc), nz);
    const uint32_t step = a.step_dev ? *a.step_dev + a.step : a.step;
    auto put = [&](int buf, int slot, const float u[3], const float t[6], bool fluid) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            lds[buf][j][slot] = u[j];
#pragma unroll
        for (int c = 0; c < 6; ++c)
            lds[buf][3 + c][slot] = t[c];
        lds[buf][9][slot] = fluid ? 0.f : 1.f;
    };
    // plane strides in bytes (every plane is below 4 GiB)
    const uint32_t fpb = static_cast<uint32_t>(g.plane * sizeof(typename Store<S>::T));
    const uint32_t tpb = static_cast<uint32_t>(g.plane * sizeof(float));
    for (int z = z0 - 1; z <= z1; ++z) {
        const int zz = wrap_coord(z, nz);
        const int buf = (z - z0 + 1) % 3;
        const bool body = z >= z0 && z < z1;
        // plane addresses of this plane, formed where they are used
        const char *fb = static_cast<const char *>(a.fin);
        const char *tb = reinterpret_cast<const char *>(a.tin);
        uint32_t fs = fpb, ts = tpb;
        asm volatile("" : "+s"(fb), "+s"(tb), "+s"(fs), "+s"(ts));
        const BasePlanes pl{fb, fs, a.fdelta, tb, ts, a.tdelta};
        {
            float uo[3], to[6];
            const uint32_t n = own_xy + static_cast<uint32_t>(zz) * nxy;
            const bool fl = (body && in_tile)
                                ? lb_cell<S, SR, FENE, true>(a, pl, n, x, y, zz, step, uo, to)
                                : lb_velocity<S, FENE>(a, pl, n, wx, wy, zz, uo, to);
            put(buf, own_slot, uo, to, fl);
        }
        if (body && rslot >= 0) {
            float uo[3], to[6];
            const bool fl = lb_velocity<S, FENE>(a, pl, ring_xy + static_cast<uint32_t>(zz) * nxy,
                                                 rx, ry, zz, uo, to);
            put(buf, rslot, uo, to, fl);
        }
        __syncthreads();
        // stress update of plane z - 1
        const int zf = z - 1;
        if (zf < z0 || zf >= z1 || !in_tile)
            continue;
        const int bc = (zf - z0 + 1) % 3, bm = (zf - z0 + 3) % 3, bp = (zf - z0 + 2) % 3;
        if (lds[bc][9][own_slot] != 0.f)
            continue;
        const float u0[3] = {lds[bc][0][own_slot], lds[bc][1][own_slot], lds[bc][2][own_slot]};
        float t0[6];
#pragma unroll
        for (int c = 0; c < 6; ++c)
            t0[c] = lds[bc][3 + c][own_slot];
        float un[3][2][3], tn[3][2][6];
        uint32_t solid = 0;
        const int sl[2][2] = {{own_slot + 1, own_slot - 1}, {own_slot + W, own_slot - W}};
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int q = sl[k][side];
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    un[k][side][j] = lds[bc][j][q];
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    tn[k][side][c] = lds[bc][3 + c][q];
                solid |= (lds[bc][9][q] != 0.f ? 1u : 0u) << (2 * k + side);
            }
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int bz = side == 0 ? bp : bm;
#pragma unroll
            for (int j = 0; j < 3; ++j)
                un[2][side][j] = lds[bz][j][own_slot];
#pragma unroll
            for (int c = 0; c < 6; ++c)
                tn[2][side][c] = lds[bz][3 + c][own_slot];
            solid |= (lds[bz][9][own_slot] != 0.f ? 1u : 0u) << (4 + side);
        }
        const int zfw = wrap_coord(zf, nz);
        const uint32_t n = own_xy + static_cast<uint32_t>(zfw) * nxy;
        fv_compute<SR, LAW>(pl, a, g, n, x, y, zfw, step, u0, t0, un, tn, solid);
    }
}

// ---------------------------------------------------------------------------
// Batched step over many independent lattices (serving).  Block b belongs to
// solve block_solve[b]; each solve holds the step arguments for both
// population/stress buffer parities and its own step counter, so the same
// launch advances every active solve by one step and the launches can be
// captured once and replayed.

// The tables are read through the constant address space: the block's solve
// index is wave-uniform, so every table read is a scalar load and the plane
// pointers of the solve land in SGPRs, as the kernel arguments of the
// single-lattice kernels do (vector loads would put them in VGPRs and cost
// the scalar-base addressing of every population access).
#define VLB_CONST_AS __attribute__((address_space(4)))
template <class X>
__device__ __forceinline__ const VLB_CONST_AS X *uniform_ptr(const X *p)
{
    return (const VLB_CONST_AS X *)(uintptr_t)p;
}

template <bool SR>
__global__ __launch_bounds__(BLOCK) LB_OCCUPANCY(ST_F32) void lb_batch_kernel(const BatchTable *__restrict__ t)
{
    const VLB_CONST_AS BatchTable &tb = *uniform_ptr(t);
    const uint32_t b = blockIdx.x;  // hardware order, as for a single lattice
    if (b >= tb.total_blocks)
        return;
    const uint32_t s = uniform_ptr(tb.block_solve)[b];
    const VLB_CONST_AS BatchSolve &bs = uniform_ptr(tb.solves)[s];
    const uint32_t step = uniform_ptr(tb.steps)[s];
    if (step >= bs.target)
        return;
    const VLB_CONST_AS StepArgs &a = bs.args[step & 1u];
    const uint32_t n = (b - bs.first_block) * BLOCK + threadIdx.x;
    if (n >= a.g.N)
        return;
    int x, y, z;
    coords(geom_copy(a.g), n, x, y, z);
    lb_cell<ST_F32, SR, false, false>(a, ArgPlanes<VLB_CONST_AS StepArgs>{a}, n, x, y, z, step,
                                      nullptr, nullptr);
}

// Stress update of the batch: blocks of 64 x 4 threads, each a tile of a
// solve at least 32 cells wide (the tiled stress update) or 256 cells of a
// narrower one.  Which one is uniform per block.
template <bool SR>
__global__ __launch_bounds__(FV_TX * 4) void fv_batch_kernel(const BatchTable *__restrict__ t)
{
    __shared__ FvTileLds<4> lds;
    const VLB_CONST_AS BatchTable &tb = *uniform_ptr(t);
    const uint32_t b = block_id(1, 0);
    if (b >= tb.fv_total_blocks)
        return;
    const uint32_t s = uniform_ptr(tb.fv_block_solve)[b];
    const VLB_CONST_AS BatchSolve &bs = uniform_ptr(tb.solves)[s];
    const uint32_t step = uniform_ptr(tb.steps)[s];
    if (step >= bs.target || !bs.args[0].polymer)
        return;
    const VLB_CONST_AS StepArgs &a = bs.args[step & 1u];
    const int tid = static_cast<int>(threadIdx.x + FV_TX * threadIdx.y);
    const uint32_t lb = b - bs.fv_first_block;
    // served solves are Oldroyd-B or Giesekus (the law is uniform per block)
    const bool gk = a.gk != 0.f;
    if (bs.fv_tiled) {
        if (gk)
            fv_tile_block<SR, LAW_GIESEKUS, 4>(a, lb, bs.fv_zc, step, false, tid, lds);
        else
            fv_tile_block<SR, LAW_OB, 4>(a, lb, bs.fv_zc, step, false, tid, lds);
        return;
    }
    const uint32_t n = lb * (FV_TX * 4) + static_cast<uint32_t>(tid);
    if (n >= a.g.N)
        return;
    if (gk)
        fv_cell<SR, LAW_GIESEKUS>(a, n, step);
    else
        fv_cell<SR, LAW_OB>(a, n, step);
}

__global__ void set_step_kernel(uint32_t *step, uint32_t value, int add)
{
    *step = add ? *step + value : value;
}

__global__ void batch_advance_kernel(BatchTable *t)
{
    for (uint32_t s = threadIdx.x; s < t->n_solves; s += blockDim.x)
        if (t->steps[s] < t->solves[s].target)
            t->steps[s] += 1u;
}

// ---------------------------------------------------------------------------
// state setup and readout

template <int S>
__global__ __launch_bounds__(BLOCK) void init_eq_kernel(Geom g, const uint8_t *mask,
                                                        const double *u, void *fv, float scale)
{
    using St = Store<S>;
    using T = typename St::T;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N || mask[n] != 0)
        return;
    int x, y, z;
    coords(g, n, x, y, z);
    const Nbr nb(g, x, y, z);
    T *f = static_cast<T *>(fv);
    double ux = 0.0, uy = 0.0, uz = 0.0;
    if (u) {
        ux = u[n];
        uy = u[g.N + n];
        uz = u[2ull * g.N + n];
    }
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const double dev = WD[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        St::st(f, i * g.plane + nb.at(-CX[i], -CY[i], -CZ[i]), static_cast<float>(dev), scale);
    }
}

template <int S>
__global__ __launch_bounds__(BLOCK) void set_pops_kernel(Geom g, const uint8_t *mask,
                                                         const double *fin, void *fv, float scale)
{
    using St = Store<S>;
    using T = typename St::T;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N || mask[n] != 0)
        return;
    int x, y, z;
    coords(g, n, x, y, z);
    const Nbr nb(g, x, y, z);
    T *f = static_cast<T *>(fv);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double dev = fin[static_cast<uint64_t>(i) * g.N + n] - WD[i];
        St::st(f, i * g.plane + nb.at(-CX[i], -CY[i], -CZ[i]), static_cast<float>(dev), scale);
    }
}

__global__ __launch_bounds__(BLOCK) void set_tau_kernel(Geom g, const uint8_t *mask,
                                                        const double *tin, float *tau)
{
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N)
        return;
    const bool fl = mask[n] == 0;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        tau[c * g.plane + n] = fl ? static_cast<float>(tin[static_cast<uint64_t>(c) * g.N + n]) : 0.f;
}

// Moments of cells first .. first + count - 1 into rho_out[k] and
// u_out[a * count + k], k = n - first.
template <int S>
__global__ __launch_bounds__(BLOCK) void read_moments_kernel(Geom g, Bound b, const uint8_t *mask,
                                                             const void *fv, const float *tau,
                                                             int polymer, float gx, float gy,
                                                             float gz, const float *gfield,
                                                             float inv_scale, double *rho_out,
                                                             double *u_out, StressMap sm,
                                                             uint32_t first, uint32_t count)
{
    using St = Store<S>;
    using T = typename St::T;
    const uint32_t k = blockIdx.x * BLOCK + threadIdx.x;
    if (k >= count)
        return;
    const uint32_t n = first + k;
    if (mask[n] != 0) {
        if (rho_out)
            rho_out[k] = 0.0;
        if (u_out)
            for (int a = 0; a < 3; ++a)
                u_out[static_cast<uint64_t>(a) * count + k] = 0.0;
        return;
    }
    int x, y, z;
    coords(g, n, x, y, z);
    const Nbr nb(g, x, y, z);
    const T *f = static_cast<const T *>(fv);
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double h = St::ld(f, i * g.plane + nb.at(-CX[i], -CY[i], -CZ[i]), inv_scale);
        drho += h;
        j[0] += CX[i] * h;
        j[1] += CY[i] * h;
        j[2] += CZ[i] * h;
    }
    double F[3] = {gx, gy, gz};
    if (gfield)
        for (int a = 0; a < 3; ++a)
            F[a] += static_cast<double>(gfield[a * g.plane + n]);
    if (polymer) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t ip = nb.at(k == 0, k == 1, k == 2);
            const uint32_t im = nb.at(-(k == 0), -(k == 1), -(k == 2));
            const bool solp = mask[ip] != 0, solm = mask[im] != 0;
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                const int c = TROW[k][jj];
                const double vp = solp ? extrap_stress(g, mask, tau, sm, nb, k == 0, k == 1, k == 2, c)
                                       : mapped_stress(sm, tau, g.plane, ip, c);
                const double vm = solm ? extrap_stress(g, mask, tau, sm, nb, -(k == 0), -(k == 1),
                                                       -(k == 2), c)
                                       : mapped_stress(sm, tau, g.plane, im, c);
                F[jj] += 0.5 * (vp - vm);
            }
        }
    }
    const double rho = 1.0 + drho;
    if (rho_out)
        rho_out[k] = rho;
    if (u_out)
        for (int a = 0; a < 3; ++a)
            u_out[static_cast<uint64_t>(a) * count + k] = (j[a] + 0.5 * F[a]) / rho;
}

template <int S>
__global__ __launch_bounds__(BLOCK) void read_pops_kernel(Geom g, const uint8_t *mask,
                                                          const void *fv, float inv_scale,
                                                          double *out)
{
    using St = Store<S>;
    using T = typename St::T;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N)
        return;
    const T *f = static_cast<const T *>(fv);
    if (mask[n] != 0) {
        for (int i = 0; i < Q; ++i)
            out[static_cast<uint64_t>(i) * g.N + n] = 0.0;
        return;
    }
    int x, y, z;
    coords(g, n, x, y, z);
    const Nbr nb(g, x, y, z);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        out[static_cast<uint64_t>(i) * g.N + n] =
            WD[i] + static_cast<double>(St::ld(f, i * g.plane + nb.at(-CX[i], -CY[i], -CZ[i]), inv_scale));
}

__global__ __launch_bounds__(BLOCK) void read_tau_kernel(Geom g, const uint8_t *mask,
                                                         const float *tau, double *out,
                                                         StressMap sm)
{
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N)
        return;
    const bool fl = mask[n] == 0;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        out[static_cast<uint64_t>(c) * g.N + n] = fl ? mapped_stress(sm, tau, g.plane, n, c) : 0.0;
}

// ---------------------------------------------------------------------------
// FP64 sums and health (two-stage, deterministic)

constexpr int SUM_BLOCKS_MAX = 2048;
constexpr int NSUM = 8;  // mass deviation, p[3], max speed, non-finite, fluid cells, spare

template <int S>
__global__ __launch_bounds__(BLOCK) void sums_kernel(Geom g, const uint8_t *mask, const void *fv,
                                                     float inv_scale, double *partials)
{
    using St = Store<S>;
    using T = typename St::T;
    __shared__ double sh[BLOCK / 64];
    const T *f = static_cast<const T *>(fv);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double vmax = 0.0, bad = 0.0, fluid = 0.0;
    for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < g.N; n += gridDim.x * BLOCK) {
        if (mask[n] != 0)
            continue;
        int x, y, z;
        coords(g, n, x, y, z);
        const Nbr nb(g, x, y, z);
        double d = 0.0, j[3] = {0.0, 0.0, 0.0};
        bool finite = true;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float h = St::ld(f, i * g.plane + nb.at(-CX[i], -CY[i], -CZ[i]), inv_scale);
            finite = finite && isfinite(h);
            d += h;
            j[0] += CX[i] * static_cast<double>(h);
            j[1] += CY[i] * static_cast<double>(h);
            j[2] += CZ[i] * static_cast<double>(h);
        }
        fluid += 1.0;
        if (!finite) {
            bad += 1.0;
            continue;
        }
        acc[0] += d;
        acc[1] += j[0];
        acc[2] += j[1];
        acc[3] += j[2];
        const double sp = sqrt(j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / (1.0 + d);
        vmax = fmax(vmax, sp);
    }
    double r[NSUM];
    for (int k = 0; k < 4; ++k)
        r[k] = block_sum<BLOCK>(acc[k], sh);
    r[4] = block_max<BLOCK>(vmax, sh);
    r[5] = block_sum<BLOCK>(bad, sh);
    r[6] = block_sum<BLOCK>(fluid, sh);
    r[7] = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NSUM; ++k)
            partials[blockIdx.x * NSUM + k] = r[k];
}

__global__ __launch_bounds__(BLOCK) void sums_final_kernel(const double *partials, int nblocks,
                                                           int nvals, double *out)
{
    __shared__ double sh[BLOCK / 64];
    for (int k = 0; k < nvals; ++k) {
        double v = 0.0;
        const bool is_max = (nvals == NSUM && k == 4);
        // fixed assignment of partials to threads, fixed reduction tree
        for (int b = threadIdx.x; b < nblocks; b += BLOCK)
            v = is_max ? fmax(v, partials[b * nvals + k]) : v + partials[b * nvals + k];
        const double r = is_max ? block_max<BLOCK>(v, sh) : block_sum<BLOCK>(v, sh);
        if (threadIdx.x == 0)
            out[k] = r;
    }
}

// ---------------------------------------------------------------------------
// Momentum exchange and polymer traction (Section 3.4; the traction balances
// the boundary terms of the discrete polymer force).

struct Box {
    int lo[3], ext[3];
};

__device__ Box particle_box(const Geom &g, const Particle &P, int margin)
{
    Box bx;
    const int len[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        int lo = static_cast<int>(floor(P.R[k] - P.radius)) - margin;
        int hi = static_cast<int>(ceil(P.R[k] + P.radius)) + margin;
        if (g.per[k]) {
            int e = hi - lo + 1;
            if (e > len[k]) {
                lo = 0;
                e = len[k];
            }
            bx.lo[k] = lo;
            bx.ext[k] = e;
        } else {
            lo = lo < 0 ? 0 : lo;
            hi = hi > len[k] - 1 ? len[k] - 1 : hi;
            bx.lo[k] = lo;
            bx.ext[k] = hi >= lo ? hi - lo + 1 : 0;
        }
    }
    return bx;
}

__device__ __forceinline__ void box_cell(const Geom &g, const Box &bx, uint32_t k, int &x, int &y,
                                         int &z)
{
    const uint32_t ex = bx.ext[0], ey = bx.ext[1];
    const int i = k % ex, j = (k / ex) % ey, l = k / (ex * ey);
    x = bx.lo[0] + i;
    y = bx.lo[1] + j;
    z = bx.lo[2] + l;
    x = ((x % g.nx) + g.nx) % g.nx;
    y = ((y % g.ny) + g.ny) % g.ny;
    z = ((z % g.nz) + g.nz) % g.nz;
}

// Contributions of fluid cell (x,y,z) to the force on the obstacle(s) whose
// mask byte satisfies `owner_match`: acc[0..2] momentum exchange force,
// acc[3..5] its torque about the particle centre (when P is given),
// acc[6..8] traction force, acc[9..11] traction torque.
template <int S, class Match>
__device__ void link_forces(const Geom &g, const uint8_t *mask, const void *fv, const float *tau,
                            int polymer, float inv_scale, int x, int y, int z, const Particle *P,
                            Match owner_match, double acc[12], const StressMap &sm)
{
    using St = Store<S>;
    using T = typename St::T;
    const T *f = static_cast<const T *>(fv);
    const Nbr nb(g, x, y, z);
    const uint32_t n = nb.at(0, 0, 0);
    // Every load first (all in bounds), the arithmetic on the matching links
    // afterwards: a wave then waits for memory once, not once per link.
    uint8_t mk[Q];
    float hd[Q], ho[Q];
#pragma unroll
    for (int d = 1; d < Q; ++d) {
        const uint32_t m = nb.at(CX[d], CY[d], CZ[d]);
        mk[d] = mask[m];
        // f*_d(x) in its own slot, the reflected population in the solid slot
        hd[d] = St::ld(f, d * g.plane + n, inv_scale);
        ho[d] = St::ld(f, OPP[d] * g.plane + m, inv_scale);
    }
    double town[6];  // this cell's polymer stress, for the traction
    if (polymer)
#pragma unroll
        for (int c = 0; c < 6; ++c)
            town[c] = mapped_stress(sm, tau, g.plane, n, c);
#pragma unroll
    for (int d = 1; d < Q; ++d) {
        if (!owner_match(mk[d]))
            continue;
        const double s = 2.0 * WD[d] + static_cast<double>(hd[d]) + static_cast<double>(ho[d]);
        const double dF[3] = {CX[d] * s, CY[d] * s, CZ[d] * s};
        acc[0] += dF[0];
        acc[1] += dF[1];
        acc[2] += dF[2];
        if (P) {
            double r[3];
            lever(g, *P, nb.xc[CX[d] + 1], nb.yc[CY[d] + 1], nb.zc[CZ[d] + 1], r);
            acc[3] += r[1] * dF[2] - r[2] * dF[1];
            acc[4] += r[2] * dF[0] - r[0] * dF[2];
            acc[5] += r[0] * dF[1] - r[1] * dF[0];
        }
    }
    if (!polymer)
        return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int s = side == 0 ? 1 : -1;
            const int cx = s * (k == 0), cy = s * (k == 1), cz = s * (k == 2);
            // face directions are 1..6 in the order +x, -x, +y, -y, +z, -z
            if (!owner_match(mk[2 * k + 1 + side]))
                continue;
            // the face value the polymer force used: the mean of this cell's
            // stress and the one extrapolated into the solid neighbour
            double dF[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double own = town[TROW[k][j]];
                const double face =
                    sm.extrap ? 0.5 * (own + extrap_stress(g, mask, tau, sm, nb, cx, cy, cz,
                                                           TROW[k][j]))
                              : own;
                dF[j] = -s * face;
            }
            acc[6] += dF[0];
            acc[7] += dF[1];
            acc[8] += dF[2];
            if (P) {
                double r[3];
                lever(g, *P, nb.xc[cx + 1], nb.yc[cy + 1], nb.zc[cz + 1], r);
                acc[9] += r[1] * dF[2] - r[2] * dF[1];
                acc[10] += r[2] * dF[0] - r[0] * dF[2];
                acc[11] += r[0] * dF[1] - r[1] * dF[0];
            }
        }
}

// Obstacle forces: PF_BLOCKS blocks per particle (blockIdx.y) share the
// particle's bounding box; each writes its block sum of the 12 components,
// and particle_reduce_update_kernel adds the blocks in a fixed order.
template <int S>
__global__ __launch_bounds__(BLOCK) void particle_forces_kernel(Geom g, const uint8_t *mask,
                                                                const void *fv, const float *tau,
                                                                int polymer, float inv_scale,
                                                                const Particle *parts,
                                                                double *partials, StressMap sm)
{
    __shared__ double sh[12 * (BLOCK / 64)];
    const int p = blockIdx.y;
    const Particle &P = parts[p];
    const uint8_t me = static_cast<uint8_t>(PART0 + p);
    const Box bx = particle_box(g, P, 2);
    const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
    double acc[12] = {0};
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < vol; k += PF_BLOCKS * BLOCK) {
        int x, y, z;
        box_cell(g, bx, k, x, y, z);
        const uint32_t n = x + static_cast<uint32_t>(g.nx) * (y + static_cast<uint32_t>(g.ny) * z);
        if (mask[n] != 0)
            continue;
        link_forces<S>(g, mask, fv, tau, polymer, inv_scale, x, y, z, &P,
                       [me](uint8_t m) { return m == me; }, acc, sm);
    }
    block_sums<BLOCK, 12>(acc, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 12; ++k)
            partials[(static_cast<size_t>(p) * PF_BLOCKS + blockIdx.x) * 12 + k] = acc[k];
}

// Per particle (one 64-thread block each): the fixed-order sum of its
// PF_BLOCKS block sums, one component per thread with every load in flight
// at once, then the totals and, for a movable particle, the symplectic Euler
// update (Section 3.4) by thread 0.
__global__ __launch_bounds__(64) void particle_reduce_update_kernel(Geom g, Particle *parts,
                                                                    const double *partials)
{
    __shared__ double rs[12];
    const int p = blockIdx.x, t = threadIdx.x;
    if (t < 12) {
        double v[PF_BLOCKS];
#pragma unroll
        for (int b = 0; b < PF_BLOCKS; ++b)
            v[b] = partials[(static_cast<size_t>(p) * PF_BLOCKS + b) * 12 + t];
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < PF_BLOCKS; ++b)
            acc += v[b];
        rs[t] = acc;
    }
    __syncthreads();
    if (t != 0)
        return;
    double r[12];
    for (int k = 0; k < 12; ++k)
        r[k] = rs[k];
    Particle &P = parts[p];
    for (int a = 0; a < 3; ++a) {
        P.fmex[a] = r[a];
        P.tmex[a] = r[3 + a];
        P.ftau[a] = r[6 + a];
        P.ttau[a] = r[9 + a];
    }
    for (int a = 0; a < 3; ++a) {
        P.ftot[a] = P.fmex[a] + P.ftau[a] + P.fconv[a] + P.fext[a];
        P.ttot[a] = P.tmex[a] + P.ttau[a] + P.tconv[a] + P.text[a];
        P.fconv[a] = 0.0;
        P.tconv[a] = 0.0;
    }
    if (!P.movable)
        return;
    const int len[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        P.Rprev[a] = P.R[a];
        P.v[a] += P.ftot[a] / P.mass;
        P.w[a] += P.ttot[a] / P.inertia;
    }
    for (int a = 0; a < 3; ++a) {
        P.R[a] += P.v[a];
        if (g.per[a]) {
            const double L = static_cast<double>(len[a]);
            P.R[a] -= L * floor(P.R[a] / L);
        }
    }
}

template <int S>
__global__ __launch_bounds__(BLOCK) void wall_force_kernel(Geom g, const uint8_t *mask,
                                                           const void *fv, const float *tau,
                                                           int polymer, float inv_scale,
                                                           double *partials, StressMap sm)
{
    __shared__ double sh[BLOCK / 64];
    double acc[12] = {0};
    for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < g.N; n += gridDim.x * BLOCK) {
        if (mask[n] != 0)
            continue;
        int x, y, z;
        coords(g, n, x, y, z);
        link_forces<S>(g, mask, fv, tau, polymer, inv_scale, x, y, z, nullptr,
                       [](uint8_t m) { return m != 0 && m < PART0; }, acc, sm);
    }
    for (int a = 0; a < 3; ++a) {
        const double r = block_sum<BLOCK>(acc[a] + acc[6 + a], sh);
        if (threadIdx.x == 0)
            partials[blockIdx.x * 3 + a] = r;
    }
}

// Section 3.4: totals and symplectic Euler (velocity first, then position
// with the new velocity).
// ---------------------------------------------------------------------------
// Fluid/solid conversion around movable particles (Section 3.4).  The new
// owner of a cell is a pure function of its old mask byte and the updated
// particle positions, so every phase is a gather and needs no atomics; phases
// are separated by barriers.  One block per movable particle when no
// particle's cells come near another's (each block then runs every phase for
// its particle alone, which gives the bits of the one-block order), else one
// block for all of them, particle after particle within each phase.

constexpr int CONV_THREADS = 1024;
constexpr int CONV_CHECK_BLOCKS = 16;  // blocks per particle of the change check

struct ConvCtx {
    Geom g;
    const Particle *parts;
    int n_parts;
    const uint8_t *mask;
    const int *moving;  // indices of movable particles (LDS)
    int n_moving;
    const uint8_t *owner = nullptr;  // new owner of every cell the phases look at
};

__device__ bool inside_sphere(const Geom &g, const Particle &P, int x, int y, int z)
{
#pragma clang fp contract(off)
    double r[3];
    lever(g, P, x, y, z, r);
    const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    return d2 < P.radius * P.radius;
}

// The owner of cell n after this step's moves: its particle while the
// particle still covers it, the first movable particle that covers a fluid
// cell, else the old mask byte.
__device__ uint8_t compute_owner(const ConvCtx &c, uint32_t n, int x, int y, int z)
{
    const uint8_t m = c.mask[n];
    if (m >= PART0) {
        const Particle &P = c.parts[m - PART0];
        if (P.movable && !inside_sphere(c.g, P, x, y, z))
            return 0;
        return m;
    }
    if (m == 0) {
        for (int q = 0; q < c.n_moving; ++q) {
            const int k = c.moving[q];
            if (inside_sphere(c.g, c.parts[k], x, y, z))
                return static_cast<uint8_t>(PART0 + k);
        }
    }
    return m;
}

// The same from the owner map the conversion kernel fills first (one
// coverage test per cell instead of one per look).
__device__ __forceinline__ uint8_t new_owner(const ConvCtx &c, uint32_t n, int, int, int)
{
    return c.owner[n];
}

__device__ __forceinline__ bool stays_fluid(const ConvCtx &c, uint32_t n, int x, int y, int z)
{
    return c.mask[n] == 0 && new_owner(c, n, x, y, z) == 0;
}

__device__ int fluid_neighbours(const ConvCtx &c, const Nbr &nb)
{
    int nf = 0;
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const uint32_t m = nb.at(CX[j], CY[j], CZ[j]);
        if (stays_fluid(c, m, nb.xc[CX[j] + 1], nb.yc[CY[j] + 1], nb.zc[CZ[j] + 1]))
            ++nf;
    }
    return nf;
}

// Does any cell change owner this step?  Many blocks per moving particle p
// scan its bounding box and raise flag[p]; the conversion kernel does nothing
// for p unless it is raised (and clears it).
__global__ __launch_bounds__(BLOCK) void conversion_check_kernel(Geom g, const Particle *parts,
                                                                 const uint8_t *mask,
                                                                 int32_t *flag)
{
    const int p = blockIdx.y;
    const Particle &P = parts[p];
    bool change = false;
    if (P.movable) {
        const uint8_t me = static_cast<uint8_t>(PART0 + p);
        const Box bx = particle_box(g, P, 2);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < vol; k += gridDim.x * BLOCK) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint8_t m =
                mask[x + static_cast<uint32_t>(g.nx) * (y + static_cast<uint32_t>(g.ny) * z)];
            if (m == 0)
                change = change || inside_sphere(g, P, x, y, z);
            else if (m == me)
                change = change || !inside_sphere(g, P, x, y, z);
        }
    }
    if (__syncthreads_or(change) && threadIdx.x == 0)
        atomicOr(flag + p, 1);
}

// Fraction of the unit cell around (x, y, z) that a sphere of radius r at
// Rc overlaps, sub-sampled at ns^3 evenly spaced points (ns = 1: the cell
// centre, the coverage test itself).  Minimum image on periodic axes.
__device__ double overlap_fraction(const Geom &g, const double Rc[3], double r, int x, int y, int z,
                                   int ns)
{
#pragma clang fp contract(off)
    const int len[3] = {g.nx, g.ny, g.nz};
    const int c[3] = {x, y, z};
    int in = 0;
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j)
            for (int k = 0; k < ns; ++k) {
                const int o[3] = {i, j, k};
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double pt =
                        static_cast<double>(c[a]) + (static_cast<double>(o[a]) + 0.5) / ns - 0.5;
                    double d = pt - Rc[a];
                    if (g.per[a]) {
                        const double L = static_cast<double>(len[a]);
                        d -= L * floor(d / L + 0.5);
                    }
                    d2 = a == 0 ? d * d : d2 + d * d;
                }
                in += d2 < r * r ? 1 : 0;
            }
    return static_cast<double>(in) / static_cast<double>(ns * ns * ns);
}

// Do two (possibly wrapped) boxes share a cell?
__device__ bool boxes_meet(const Geom &g, const Box &a, const Box &b)
{
    const int len[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        if (a.ext[k] <= 0 || b.ext[k] <= 0)
            return false;
        bool meet;
        if (g.per[k]) {
            int ab = (b.lo[k] - a.lo[k]) % len[k], ba = (a.lo[k] - b.lo[k]) % len[k];
            ab = ab < 0 ? ab + len[k] : ab;
            ba = ba < 0 ? ba + len[k] : ba;
            meet = ab < a.ext[k] || ba < b.ext[k];
        } else {
            meet = a.lo[k] < b.lo[k] + b.ext[k] && b.lo[k] < a.lo[k] + a.ext[k];
        }
        if (!meet)
            return false;
    }
    return true;
}

// Is (x, y, z) inside the (possibly wrapped) box?
__device__ __forceinline__ bool in_box(const Geom &g, const Box &bx, int x, int y, int z)
{
    const int c[3] = {x, y, z}, len[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
        int off = (c[a] - bx.lo[a]) % len[a];
        off = off < 0 ? off + len[a] : off;
        if (off >= bx.ext[a])
            return false;
    }
    return true;
}

template <int S>
__global__ __launch_bounds__(CONV_THREADS) void conversion_kernel(Geom g, Bound b, uint8_t *mask,
                                                                  void *fv, float *tau, float scale,
                                                                  float inv_scale, int32_t *counters,
                                                                  float *scratch, uint8_t *owner)
{
    using St = Store<S>;
    using T = typename St::T;
    __shared__ int moving[MAX_PARTICLES];
    __shared__ int n_moving;
    __shared__ double sh[CONV_THREADS / 64];
    Particle *parts = const_cast<Particle *>(b.parts);
    T *f = static_cast<T *>(fv);
    __shared__ int go;
    if (threadIdx.x == 0) {
        int k = 0;
        for (int p = 0; p < b.n_parts; ++p)
            if (parts[p].movable)
                moving[k++] = p;
        n_moving = k;
    }
    __syncthreads();
    // A particle writes cells up to one beyond its margin-2 box (populations
    // of uncovered cells' neighbours) and reads up to two beyond it, so blocks
    // of different particles share no cell when no particle's box widened by
    // 3 meets another's box.  Otherwise block 0 takes every particle in turn.
    const int nm = n_moving;
    bool clash = false;
    // (the owner map below covers two cells beyond each box, which the
    // widening by 3 keeps apart as well)
    for (int k = threadIdx.x; k < nm * nm; k += CONV_THREADS) {
        const int i = k / nm, j = k - (k / nm) * nm;
        if (i != j && boxes_meet(g, particle_box(g, parts[moving[i]], 5),
                                 particle_box(g, parts[moving[j]], 2)))
            clash = true;
    }
    const bool serial = __syncthreads_or(clash ? 1 : 0) != 0 || b.conv_serial != 0;
    if (serial ? blockIdx.x != 0 : static_cast<int>(blockIdx.x) >= nm)
        return;
    const int q0 = serial ? 0 : static_cast<int>(blockIdx.x);
    const int q1 = serial ? nm : q0 + 1;
    if (threadIdx.x == 0) {
        int any = 0;
        for (int q = q0; q < q1; ++q) {
            any |= counters[4 + moving[q]];
            counters[4 + moving[q]] = 0;
        }
        go = any;
    }
    __syncthreads();
    if (!go && b.smooth_ns <= 0)
        return;
    // With one block per particle no other movable sphere reaches the cells
    // this block reads (each sphere lies inside its margin-2 box, and the
    // boxes stay three cells apart), so the coverage tests need only this
    // block's particle.
    ConvCtx c{g, parts, b.n_parts, mask, moving + q0, q1 - q0};
    const uint64_t PL = g.plane;
    auto cell = [&](int x, int y, int z) {
        return static_cast<uint32_t>(x) + static_cast<uint32_t>(g.nx) * (y + static_cast<uint32_t>(g.ny) * z);
    };
    // The owner map over every cell the phases look at: up to two cells
    // beyond each particle's margin-2 box.  Boxes of this block's particles
    // may overlap; their cells then get the same value twice.
    for (int q = q0; q < q1; ++q) {
        const Box bx = particle_box(g, parts[moving[q]], 4);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint32_t n = cell(x, y, z);
            owner[n] = compute_owner(c, n, x, y, z);
        }
    }
    __syncthreads();
    c.owner = owner;

    // Phase 0 (overlap-fraction smoothing, particle by particle): a cell
    // that is fluid, stays fluid and is overlapped more by the particle than
    // before its last move hands the share (phi_new - phi_old) /
    // (1 - phi_old) of its stress, in equal parts, to its neighbours that
    // stay fluid.  Per box cell the share per neighbour and the kept
    // fraction go to scratch planes 0 and 1; then, one stress component at a
    // time, every receiver gathers into plane 2 and every cell applies.
    if (b.smooth_ns > 0)
        for (int q = q0; q < q1; ++q) {
            const Particle P = parts[moving[q]];
            const Box bx = particle_box(g, P, 2);
            const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
            for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
                int x, y, z;
                box_cell(g, bx, k, x, y, z);
                const uint32_t n = cell(x, y, z);
                float share = 0.f, keep = 1.f;
                if (stays_fluid(c, n, x, y, z)) {
                    const double fo = overlap_fraction(g, P.Rprev, P.radius, x, y, z, b.smooth_ns);
                    const double fn = overlap_fraction(g, P.R, P.radius, x, y, z, b.smooth_ns);
                    if (fn > fo && fo < 1.0) {
                        const double qf = (fn - fo) / (1.0 - fo);
                        const int nf = fluid_neighbours(c, Nbr(g, x, y, z));
                        if (nf > 0) {
                            share = static_cast<float>(qf / nf);
                            keep = static_cast<float>(1.0 - qf);
                        }
                    }
                }
                scratch[n] = share;
                scratch[PL + n] = keep;
            }
            __syncthreads();
            for (int cc = 0; cc < 6; ++cc) {
                for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
                    int x, y, z;
                    box_cell(g, bx, k, x, y, z);
                    const uint32_t n = cell(x, y, z);
                    if (!stays_fluid(c, n, x, y, z))
                        continue;
                    const Nbr nb(g, x, y, z);
                    float recv = 0.f;
                    for (int j = 1; j < Q; ++j) {
                        const int mx = nb.xc[CX[j] + 1], my = nb.yc[CY[j] + 1],
                                  mz = nb.zc[CZ[j] + 1];
                        if (!in_box(g, bx, mx, my, mz))
                            continue;
                        const uint32_t m = nb.at(CX[j], CY[j], CZ[j]);
                        recv += scratch[m] * tau[cc * PL + m];
                    }
                    scratch[2 * PL + n] = recv;
                }
                __syncthreads();
                for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
                    int x, y, z;
                    box_cell(g, bx, k, x, y, z);
                    const uint32_t n = cell(x, y, z);
                    if (stays_fluid(c, n, x, y, z))
                        tau[cc * PL + n] = scratch[PL + n] * tau[cc * PL + n] + scratch[2 * PL + n];
                }
                __syncthreads();
            }
        }
    // Phase 1: covers.  The populations' momentum goes to the particle; the
    // stress is shared among the D3Q19 neighbours that stay fluid (gathered
    // by each receiver).
    int covers = 0, dropped = 0;
    for (int q = q0; q < q1; ++q) {
        const int p = moving[q];
        const Particle P = parts[p];
        const uint8_t me = static_cast<uint8_t>(PART0 + p);
        const Box bx = particle_box(g, P, 2);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        double mom[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint32_t n = cell(x, y, z);
            const Nbr nb(g, x, y, z);
            if (mask[n] == 0 && new_owner(c, n, x, y, z) == me) {
                double m3[3] = {0, 0, 0};
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const double h = St::ld(f, i * PL + nb.at(-CX[i], -CY[i], -CZ[i]), inv_scale);
                    m3[0] += CX[i] * h;
                    m3[1] += CY[i] * h;
                    m3[2] += CZ[i] * h;
                }
                double r[3];
                lever(g, P, x, y, z, r);
                mom[0] += m3[0];
                mom[1] += m3[1];
                mom[2] += m3[2];
                mom[3] += r[1] * m3[2] - r[2] * m3[1];
                mom[4] += r[2] * m3[0] - r[0] * m3[2];
                mom[5] += r[0] * m3[1] - r[1] * m3[0];
                ++covers;
                if (fluid_neighbours(c, nb) == 0)
                    ++dropped;
            } else if (stays_fluid(c, n, x, y, z)) {
                float add[6] = {0, 0, 0, 0, 0, 0};
                bool any = false;
                for (int j = 1; j < Q; ++j) {
                    const uint32_t m = nb.at(CX[j], CY[j], CZ[j]);
                    const int mx = nb.xc[CX[j] + 1], my = nb.yc[CY[j] + 1], mz = nb.zc[CZ[j] + 1];
                    if (mask[m] != 0 || new_owner(c, m, mx, my, mz) != me)
                        continue;
                    const Nbr nb2(g, mx, my, mz);
                    const int nf = fluid_neighbours(c, nb2);
                    for (int cc = 0; cc < 6; ++cc)
                        add[cc] += tau[cc * PL + m] / static_cast<float>(nf);
                    any = true;
                }
                if (any)
                    for (int cc = 0; cc < 6; ++cc)
                        tau[cc * PL + n] += add[cc];
            }
        }
        double r[6];
        for (int a = 0; a < 6; ++a)
            r[a] = block_sum<CONV_THREADS>(mom[a], sh);
        if (threadIdx.x == 0)
            for (int a = 0; a < 3; ++a) {
                parts[p].fconv[a] += r[a];
                parts[p].tconv[a] += r[3 + a];
            }
        __syncthreads();
    }
    // Phase 2: covered cells hold no stress.
    for (int q = q0; q < q1; ++q) {
        const int p = moving[q];
        const Particle P = parts[p];
        const uint8_t me = static_cast<uint8_t>(PART0 + p);
        const Box bx = particle_box(g, P, 2);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint32_t n = cell(x, y, z);
            if (mask[n] == 0 && new_owner(c, n, x, y, z) == me)
                for (int cc = 0; cc < 6; ++cc)
                    tau[cc * PL + n] = 0.f;
        }
        __syncthreads();
    }
    // Phase 3: uncovers.  Equilibrium populations at the mean density of the
    // neighbours that stay fluid and the surface velocity; the particle pays
    // the created momentum; the stress is the neighbours' sum / (N_f + 1).
    int uncovers = 0;
    for (int q = q0; q < q1; ++q) {
        const int p = moving[q];
        const Particle P = parts[p];
        const uint8_t me = static_cast<uint8_t>(PART0 + p);
        const Box bx = particle_box(g, P, 2);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        double mom[6] = {0, 0, 0, 0, 0, 0};
        for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint32_t n = cell(x, y, z);
            if (!(mask[n] == me && new_owner(c, n, x, y, z) == 0))
                continue;
            const Nbr nb(g, x, y, z);
            int nf = 0;
            double rsum = 0.0;
            float ts[6] = {0, 0, 0, 0, 0, 0};
            for (int j = 1; j < Q; ++j) {
                const uint32_t m = nb.at(CX[j], CY[j], CZ[j]);
                const int mx = nb.xc[CX[j] + 1], my = nb.yc[CY[j] + 1], mz = nb.zc[CZ[j] + 1];
                if (!stays_fluid(c, m, mx, my, mz))
                    continue;
                ++nf;
                const Nbr nb2(g, mx, my, mz);
                double rho = 1.0;
                for (int i = 0; i < Q; ++i)
                    rho += St::ld(f, i * PL + nb2.at(-CX[i], -CY[i], -CZ[i]), inv_scale);
                rsum += rho;
                for (int cc = 0; cc < 6; ++cc)
                    ts[cc] += tau[cc * PL + m];
            }
            const double rho = nf > 0 ? rsum / nf : 1.0;
            double ub[3];
            boundary_velocity_d(g, b, me, x, y, z, ub);
            const double uu = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
            for (int i = 0; i < Q; ++i) {
                const double cu = CX[i] * ub[0] + CY[i] * ub[1] + CZ[i] * ub[2];
                const double dev = WD[i] * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
                St::st(f, i * PL + nb.at(-CX[i], -CY[i], -CZ[i]), static_cast<float>(dev), scale);
            }
            const double m3[3] = {rho * ub[0], rho * ub[1], rho * ub[2]};
            double r[3];
            lever(g, P, x, y, z, r);
            mom[0] -= m3[0];
            mom[1] -= m3[1];
            mom[2] -= m3[2];
            mom[3] -= r[1] * m3[2] - r[2] * m3[1];
            mom[4] -= r[2] * m3[0] - r[0] * m3[2];
            mom[5] -= r[0] * m3[1] - r[1] * m3[0];
            for (int cc = 0; cc < 6; ++cc)
                tau[cc * PL + n] = ts[cc] / static_cast<float>(nf + 1);
            ++uncovers;
        }
        double r[6];
        for (int a = 0; a < 6; ++a)
            r[a] = block_sum<CONV_THREADS>(mom[a], sh);
        if (threadIdx.x == 0)
            for (int a = 0; a < 3; ++a) {
                parts[p].fconv[a] += r[a];
                parts[p].tconv[a] += r[3 + a];
            }
        __syncthreads();
    }
    // Phase 4: the neighbours give up what the uncovered cells took.
    for (int q = q0; q < q1; ++q) {
        const int p = moving[q];
        const Particle P = parts[p];
        const uint8_t me = static_cast<uint8_t>(PART0 + p);
        const Box bx = particle_box(g, P, 2);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint32_t n = cell(x, y, z);
            if (!stays_fluid(c, n, x, y, z))
                continue;
            const Nbr nb(g, x, y, z);
            float sub[6] = {0, 0, 0, 0, 0, 0};
            bool any = false;
            for (int j = 1; j < Q; ++j) {
                const uint32_t m = nb.at(CX[j], CY[j], CZ[j]);
                const int mx = nb.xc[CX[j] + 1], my = nb.yc[CY[j] + 1], mz = nb.zc[CZ[j] + 1];
                if (!(mask[m] == me && new_owner(c, m, mx, my, mz) == 0))
                    continue;
                const Nbr nb2(g, mx, my, mz);
                const int nf = fluid_neighbours(c, nb2);
                for (int cc = 0; cc < 6; ++cc)
                    sub[cc] += tau[cc * PL + m] / static_cast<float>(nf);
                any = true;
            }
            if (any)
                for (int cc = 0; cc < 6; ++cc)
                    tau[cc * PL + n] -= sub[cc];
        }
        __syncthreads();
    }
    // Phase 5: the new mask.
    for (int q = q0; q < q1; ++q) {
        const int p = moving[q];
        const Particle P = parts[p];
        const uint8_t me = static_cast<uint8_t>(PART0 + p);
        const Box bx = particle_box(g, P, 2);
        const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
        for (uint32_t k = threadIdx.x; k < vol; k += CONV_THREADS) {
            int x, y, z;
            box_cell(g, bx, k, x, y, z);
            const uint32_t n = cell(x, y, z);
            const uint8_t m = mask[n];
            if (m == 0 || m == me) {
                const uint8_t nw = new_owner(c, n, x, y, z);
                if (m == 0 && nw == me)
                    mask[n] = me;
                else if (m == me && nw == 0)
                    mask[n] = 0;
            }
        }
        __syncthreads();
    }
    if (covers)
        atomicAdd(&counters[0], covers);
    if (uncovers)
        atomicAdd(&counters[1], uncovers);
    if (dropped)
        atomicAdd(&counters[2], dropped);
}

inline uint32_t blocks_for(uint32_t n) { return (n + BLOCK - 1) / BLOCK; }

template <class Fn>
hipError_t dispatch(int storage, Fn fn)
{
    switch (storage) {
    case ST_F32:
        return fn(std::integral_constant<int, ST_F32>{});
    case ST_F16:
        return fn(std::integral_constant<int, ST_F16>{});
    case ST_BF16:
        return fn(std::integral_constant<int, ST_BF16>{});
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

// Control experiment for the storage layout: the populations f_i = w_i + h_i
// that FP32 deviation storage holds, rounded to the nearest FP32 number, as
// storing raw populations in FP32 would keep them (the deviations then carry
// the rounding error of numbers near w_i instead of their own).
__global__ __launch_bounds__(BLOCK) void raw_f32_control_kernel(float *f, uint64_t plane, uint32_t N)
{
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    const int i = static_cast<int>(blockIdx.y);
    if (n >= N)
        return;
    const double w = i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
    float *p = f + i * plane + n;
    const float raw = static_cast<float>(w + static_cast<double>(*p));
    *p = static_cast<float>(static_cast<double>(raw) - w);
}

hipError_t launch_raw_f32_control(const Geom &g, void *f, hipStream_t s)
{
    hipLaunchKernelGGL(raw_f32_control_kernel, dim3(blocks_for(g.N), Q), dim3(BLOCK), 0, s,
                       static_cast<float *>(f), g.plane, g.N);
    return hipGetLastError();
}

hipError_t launch_lb_step(int storage, const StepArgs &a, hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        constexpr int S = decltype(st)::value;
        const dim3 grid(blocks_for(a.g.N)), block(BLOCK);
        const bool fene = a.polymer && a.sm.l2m3 > 0.f;
        if (fene) {
            if (a.stochastic)
                hipLaunchKernelGGL((lb_step_kernel<S, true, true>), grid, block, 0, s, a);
            else
                hipLaunchKernelGGL((lb_step_kernel<S, false, true>), grid, block, 0, s, a);
        } else {
            if (a.stochastic)
                hipLaunchKernelGGL((lb_step_kernel<S, true, false>), grid, block, 0, s, a);
            else
                hipLaunchKernelGGL((lb_step_kernel<S, false, false>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    });
}

hipError_t launch_fv_step(int storage, const StepArgs &a, hipStream_t s, int tile_rows,
                          uint32_t z_chunk)
{
    (void)storage;
    // The tiled kernel needs x rows that fill its 64-wide tiles and enough
    // blocks to fill the chip (chunks are shortened down to 8 planes for
    // that: with 4-plane chunks the column and ring loads at each chunk's
    // start cost more than tiling saves); small lattices take the per-cell
    // kernel unless the tiled one is forced (negative tile_rows).
    const bool force = tile_rows < 0;
    if (force)
        tile_rows = -tile_rows;
    const uint32_t rows = tile_rows > 0 ? static_cast<uint32_t>(tile_rows) : 1u;
    const uint32_t tiles_xy = ((a.g.nx + FV_TX - 1) / FV_TX) * ((a.g.ny + rows - 1) / rows);
    uint32_t zc = z_chunk ? z_chunk : 16u;
    while (!force && zc > 8 && tiles_xy * ((a.g.nz + zc - 1) / zc) < 2048)
        zc /= 2;
    // at most an eighth of the tile lanes beyond the end of the rows
    const uint32_t lanes_x = ((a.g.nx + FV_TX - 1) / FV_TX) * FV_TX;
    const bool rows_fill = 8u * (lanes_x - a.g.nx) <= lanes_x;
    const bool tiled = (tile_rows == 4 || tile_rows == 8) &&
                       (force || (rows_fill && tiles_xy * ((a.g.nz + zc - 1) / zc) >= 1024));
    const uint32_t tiles = tiles_xy * ((a.g.nz + zc - 1) / zc);
    const int law = a.sm.l2m3 > 0.f ? LAW_FENE : (a.gk != 0.f ? LAW_GIESEKUS : LAW_OB);
    auto go = [&](auto sr, auto lw) {
        constexpr bool SR = decltype(sr)::value;
        constexpr int LAW = decltype(lw)::value;
        if (tiled && tile_rows == 4)
            hipLaunchKernelGGL((fv_tile_kernel<SR, LAW, 4>), dim3(tiles), dim3(FV_TX * 4), 0, s, a, zc);
        else if (tiled)
            hipLaunchKernelGGL((fv_tile_kernel<SR, LAW, 8>), dim3(tiles), dim3(FV_TX * 8), 0, s, a, zc);
        else
            hipLaunchKernelGGL((fv_step_kernel<SR, LAW>), dim3(blocks_for(a.g.N)), dim3(BLOCK), 0, s, a);
    };
    auto with_law = [&](auto sr) {
        if (law == LAW_FENE)
            go(sr, std::integral_constant<int, LAW_FENE>{});
        else if (law == LAW_GIESEKUS)
            go(sr, std::integral_constant<int, LAW_GIESEKUS>{});
        else
            go(sr, std::integral_constant<int, LAW_OB>{});
    };
    if (a.stochastic)
        with_law(std::true_type{});
    else
        with_law(std::false_type{});
    return hipGetLastError();
}

// Tile of the fused step: 64 x 4 cells (measured faster than 16 x 4, 32 x 4,
// 64 x 6, 64 x 8 and 64 x 12).
constexpr int STEP_TX = 64, STEP_TY = 4;

bool step_fused_fits(const Geom &g, uint32_t z_chunk, bool force, uint32_t *zc_out)
{
    const int TX = STEP_TX, TY = STEP_TY;
    // rows that fill the tiles, and enough blocks to fill the chip (chunks
    // shortened down to 8 planes for that: each chunk computes the moments
    // of the two planes around it once more)
    const uint32_t tiles_xy = ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY);
    const uint32_t want = 2048u * (256u / (TX * TY));
    uint32_t zc = z_chunk ? z_chunk : 32u;
    while (!force && zc > 8 && tiles_xy * ((g.nz + zc - 1) / zc) < want)
        zc /= 2;
    const uint32_t lanes_x = ((g.nx + TX - 1) / TX) * TX;
    const bool rows_fill = 8u * (lanes_x - g.nx) <= lanes_x;
    if (zc_out)
        *zc_out = zc;
    return force || (rows_fill && tiles_xy * ((g.nz + zc - 1) / zc) >= want / 2);
}

hipError_t launch_step_fused(int storage, const StepArgs &a, hipStream_t s, uint32_t z_chunk,
                             bool force)
{
    uint32_t zc = 0;
    if (!a.polymer || !step_fused_fits(a.g, z_chunk, force, &zc))
        return hipErrorNotSupported;
    const int TX = STEP_TX, TY = STEP_TY;
    const uint32_t tiles =
        ((a.g.nx + TX - 1) / TX) * ((a.g.ny + TY - 1) / TY) * ((a.g.nz + zc - 1) / zc);
    const int law = a.sm.l2m3 > 0.f ? LAW_FENE : (a.gk != 0.f ? LAW_GIESEKUS : LAW_OB);
    return dispatch(storage, [&](auto st) {
        constexpr int S = decltype(st)::value;
        auto go = [&](auto sr, auto lw) {
            constexpr bool SR = decltype(sr)::value;
            constexpr int LAW = decltype(lw)::value;
            hipLaunchKernelGGL((step_tile_kernel<S, SR, LAW, STEP_TX, STEP_TY>), dim3(tiles),
                               dim3(STEP_TX * STEP_TY), 0, s, a, zc);
        };
        auto with_law = [&](auto sr) {
            if (law == LAW_FENE)
                go(sr, std::integral_constant<int, LAW_FENE>{});
            else if (law == LAW_GIESEKUS)
                go(sr, std::integral_constant<int, LAW_GIESEKUS>{});
            else
                go(sr, std::integral_constant<int, LAW_OB>{});
        };
        if (a.stochastic)
            with_law(std::true_type{});
        else
            with_law(std::false_type{});
        return hipGetLastError();
    });
}

hipError_t launch_set_step(uint32_t *step, uint32_t value, int add, hipStream_t s)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(1), 0, s, step, value, add);
    return hipGetLastError();
}

uint32_t batch_fv_blocks(const Geom &g, bool *tiled, uint32_t *zc)
{
    // Tiles for every solve at least half a tile wide and one tile row high,
    // in 8-plane chunks; narrower solves per cell.  Measured on a mix of
    // 32..128 edges, tiling every such solve beats per-cell for all (by 8 %),
    // and both beat tiling only the solves whose rows fill the tiles.
    const bool fill = g.nx >= FV_TX / 2 && g.ny >= 4;
    *tiled = fill;
    if (!fill) {
        *zc = 0;
        return (g.N + FV_TX * 4 - 1) / (FV_TX * 4);
    }
    *zc = static_cast<uint32_t>(g.nz < 8 ? g.nz : 8);
    return ((g.nx + FV_TX - 1) / FV_TX) * ((g.ny + 3) / 4) * ((g.nz + *zc - 1) / *zc);
}

hipError_t launch_batch_step(const BatchTable *t, uint32_t max_blocks, uint32_t fv_blocks,
                             int stochastic, int n_steps, hipStream_t s)
{
    // the stress update runs with 64 x 4 blocks, which also tells its graph
    // nodes from stream-collide's
    const dim3 fv_block(FV_TX, 4);
    for (int k = 0; k < n_steps; ++k) {
        if (stochastic) {
            hipLaunchKernelGGL(lb_batch_kernel<true>, dim3(max_blocks), dim3(BLOCK), 0, s, t);
            hipLaunchKernelGGL(fv_batch_kernel<true>, dim3(fv_blocks), fv_block, 0, s, t);
        } else {
            hipLaunchKernelGGL(lb_batch_kernel<false>, dim3(max_blocks), dim3(BLOCK), 0, s, t);
            hipLaunchKernelGGL(fv_batch_kernel<false>, dim3(fv_blocks), fv_block, 0, s, t);
        }
        // block size differs from BLOCK so graph users can tell this node apart
        hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(64), 0, s,
                           const_cast<BatchTable *>(t));
    }
    return hipGetLastError();
}

hipError_t launch_init_equilibrium(int storage, const Geom &g, const uint8_t *mask, const double *u,
                                   void *f, float scale, hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(init_eq_kernel<decltype(st)::value>, dim3(blocks_for(g.N)), dim3(BLOCK),
                           0, s, g, mask, u, f, scale);
        return hipGetLastError();
    });
}

// FP16 deviations times a power of two (a change of storage scale): exact
// wherever the value stays a normal FP16 number, rounded to nearest where it
// enters or leaves the subnormal range.
__global__ __launch_bounds__(BLOCK) void rescale_f16_kernel(__half *h, uint64_t count, float factor)
{
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * BLOCK;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x; i < count;
         i += stride)
        h[i] = __float2half_rn(__half2float(h[i]) * factor);
}

hipError_t launch_rescale_f16(void *f, uint64_t count, float factor, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    const uint64_t need = (count + BLOCK - 1) / BLOCK;
    const uint32_t blocks = static_cast<uint32_t>(need < 8192 ? need : 8192);
    hipLaunchKernelGGL(rescale_f16_kernel, dim3(blocks), dim3(BLOCK), 0, s,
                       static_cast<__half *>(f), count, factor);
    return hipGetLastError();
}

hipError_t launch_set_populations(int storage, const Geom &g, const uint8_t *mask,
                                  const double *f_in, void *f, float scale, hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(set_pops_kernel<decltype(st)::value>, dim3(blocks_for(g.N)), dim3(BLOCK),
                           0, s, g, mask, f_in, f, scale);
        return hipGetLastError();
    });
}

hipError_t launch_set_stress(const Geom &g, const uint8_t *mask, const double *tau_in, float *tau,
                             hipStream_t s)
{
    hipLaunchKernelGGL(set_tau_kernel, dim3(blocks_for(g.N)), dim3(BLOCK), 0, s, g, mask, tau_in,
                       tau);
    return hipGetLastError();
}

hipError_t launch_read_moments(int storage, const Geom &g, const Bound &b, const uint8_t *mask,
                               const void *f, const float *tau, int polymer, const float gvec[3],
                               const float *gfield, float inv_scale, double *rho_out,
                               double *u_out, hipStream_t s, const StressMap &sm, uint32_t first,
                               uint32_t count)
{
    if (count == 0)
        count = g.N;
    if (count == 0 || first >= g.N || count > g.N - first)
        return hipErrorInvalidValue;
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(read_moments_kernel<decltype(st)::value>, dim3(blocks_for(count)),
                           dim3(BLOCK), 0, s, g, b, mask, f, tau, polymer, gvec[0], gvec[1],
                           gvec[2], gfield, inv_scale, rho_out, u_out, sm, first, count);
        return hipGetLastError();
    });
}

hipError_t launch_read_populations(int storage, const Geom &g, const uint8_t *mask, const void *f,
                                   float inv_scale, double *out, hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(read_pops_kernel<decltype(st)::value>, dim3(blocks_for(g.N)),
                           dim3(BLOCK), 0, s, g, mask, f, inv_scale, out);
        return hipGetLastError();
    });
}

hipError_t launch_read_stress(const Geom &g, const uint8_t *mask, const float *tau, double *out,
                              hipStream_t s, const StressMap &sm)
{
    hipLaunchKernelGGL(read_tau_kernel, dim3(blocks_for(g.N)), dim3(BLOCK), 0, s, g, mask, tau,
                       out, sm);
    return hipGetLastError();
}

int sums_blocks(const Geom &g)
{
    uint32_t b = blocks_for(g.N);
    return static_cast<int>(b < SUM_BLOCKS_MAX ? b : SUM_BLOCKS_MAX);
}

hipError_t launch_sums(int storage, const Geom &g, const uint8_t *mask, const void *f,
                       float inv_scale, double *partials, double *out, hipStream_t s)
{
    const int nb = sums_blocks(g);
    hipError_t e = dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(sums_kernel<decltype(st)::value>, dim3(nb), dim3(BLOCK), 0, s, g, mask,
                           f, inv_scale, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(BLOCK), 0, s, partials, nb, NSUM, out);
    return hipGetLastError();
}

hipError_t launch_particle_forces(int storage, const Geom &g, const uint8_t *mask, const void *f,
                                  const float *tau_n, int polymer, float inv_scale,
                                  Particle *parts, int n_parts, double *partials, hipStream_t s,
                                  const StressMap &sm)
{
    if (n_parts <= 0)
        return hipSuccess;
    hipError_t e = dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(particle_forces_kernel<decltype(st)::value>, dim3(PF_BLOCKS, n_parts),
                           dim3(BLOCK), 0, s, g, mask, f, tau_n, polymer, inv_scale, parts,
                           partials, sm);
        return hipGetLastError();
    });
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(particle_reduce_update_kernel, dim3(n_parts), dim3(64), 0, s, g, parts,
                       partials);
    return hipGetLastError();
}

hipError_t launch_wall_force(int storage, const Geom &g, const uint8_t *mask, const void *f,
                             const float *tau_n, int polymer, float inv_scale, double *partials,
                             double *out, hipStream_t s, const StressMap &sm)
{
    const int nb = sums_blocks(g);
    hipError_t e = dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(wall_force_kernel<decltype(st)::value>, dim3(nb), dim3(BLOCK), 0, s, g,
                           mask, f, tau_n, polymer, inv_scale, partials, sm);
        return hipGetLastError();
    });
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(BLOCK), 0, s, partials, nb, 3, out);
    return hipGetLastError();
}

hipError_t launch_body_force(const Geom &g, const uint8_t *mask, const Particle *parts,
                             int n_parts, const double body_force[3], uint32_t *count,
                             double *g_out, hipStream_t s)
{
    const uint32_t vec_blocks = blocks_for(g.N / 16u + 1u);
    const uint32_t blocks = vec_blocks < 512u ? vec_blocks : 512u;
    hipLaunchKernelGGL(fluid_count_kernel, dim3(blocks), dim3(BLOCK), 0, s, g, mask, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(body_force_kernel, dim3(1), dim3(1), 0, s, parts, n_parts, body_force[0],
                       body_force[1], body_force[2], count, g_out);
    return hipGetLastError();
}

hipError_t launch_conversion(int storage, const Geom &g, const Bound &b, uint8_t *mask, void *f,
                             float *tau, float scale, float inv_scale, int32_t *counters,
                             float *scratch, uint8_t *owner, hipStream_t s)
{
    if (b.n_parts > 0) {
        hipLaunchKernelGGL(conversion_check_kernel, dim3(CONV_CHECK_BLOCKS, b.n_parts), dim3(BLOCK),
                           0, s, g, b.parts, mask, counters + 4);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return dispatch(storage, [&](auto st) {
        const uint32_t blocks = b.n_parts > 1 ? static_cast<uint32_t>(b.n_parts) : 1u;
        hipLaunchKernelGGL(conversion_kernel<decltype(st)::value>, dim3(blocks), dim3(CONV_THREADS),
                           0, s, g, b, mask, f, tau, scale, inv_scale, counters, scratch, owner);
        return hipGetLastError();
    });
}

}  // namespace vlb
