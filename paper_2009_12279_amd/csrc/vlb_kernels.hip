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

#include "vlb_internal.h"

namespace vlb {
namespace {

// ---------------------------------------------------------------------------
// counter-based random bits for stochastic rounding (a 32-bit integer hash of
// (cell, step, seed), then a linear congruential sequence per cell)

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
        : s(hash32(cell * 0x9e3779b1u ^ hash32(step * 0x85ebca77u + seed)))
    {
    }
    // 16 uniform bits
    __device__ __forceinline__ uint32_t next16()
    {
        s = s * 1664525u + 1013904223u;
        return s >> 16;
    }
};

// ---------------------------------------------------------------------------
// storage codecs: deviation h = s * (f - w) in FP32, FP16 or BF16.
// st() rounds to nearest; st_sr() rounds stochastically (up or down with
// probability proportional to the distance), which removes the systematic
// bias round-to-nearest leaves in a slowly relaxing steady state.

template <int S>
struct Store;

template <>
struct Store<ST_F32> {
    using T = float;
    using R = double;  // register type of the per-cell arithmetic
    static __device__ __forceinline__ float ld(const T *p, uint64_t i, float inv)
    {
        return p[i] * inv;
    }
    template <class V>
    static __device__ __forceinline__ void st(T *p, uint64_t i, V v, float s)
    {
        p[i] = static_cast<float>(v * s);
    }
    template <class V>
    static __device__ __forceinline__ void st_sr(T *p, uint64_t i, V v, float s, Rng &rng)
    {
        if constexpr (sizeof(V) == 8) {
            const double x = v * static_cast<double>(s);
            float f0 = __double2float_rz(x);
            const double rem = x - static_cast<double>(f0);  // exact, |rem| < one float step
            const float f1 = __uint_as_float(__float_as_uint(f0) + 1u);  // next away from zero
            const double step = fabs(static_cast<double>(f1) - static_cast<double>(f0));
            if (static_cast<double>(rng.next16()) * (1.0 / 65536.0) * step < fabs(rem))
                f0 = f1;
            p[i] = f0;
        } else {
            p[i] = v * s;
        }
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
    static __device__ __forceinline__ void st_sr(T *p, uint64_t i, V v, float s, Rng &rng)
    {
        const float x = static_cast<float>(v) * s;
        __half h0 = __float2half_rz(x);
        const float f0 = __half2float(h0);
        const float rem = x - f0;  // exact
        const __half h1 = __ushort_as_half(static_cast<unsigned short>(__half_as_ushort(h0) + 1u));
        const float step = fabsf(__half2float(h1) - f0);
        if (static_cast<float>(rng.next16()) * (1.f / 65536.f) * step < fabsf(rem))
            h0 = h1;
        p[i] = h0;
    }
};

template <>
struct Store<ST_BF16> {
    using T = uint16_t;
    using R = float;
    static __device__ __forceinline__ float ld(const T *p, uint64_t i, float inv)
    {
        return __uint_as_float(static_cast<uint32_t>(p[i]) << 16) * inv;
    }
    template <class V>
    static __device__ __forceinline__ void st(T *p, uint64_t i, V v, float s)
    {
        // round to nearest even on the upper 16 bits
        uint32_t b = __float_as_uint(static_cast<float>(v) * s);
        b += 0x7fffu + ((b >> 16) & 1u);
        p[i] = static_cast<uint16_t>(b >> 16);
    }
    template <class V>
    static __device__ __forceinline__ void st_sr(T *p, uint64_t i, V v, float s, Rng &rng)
    {
        // uniform bits added below the kept 16 bits, then truncation
        const uint32_t b = __float_as_uint(static_cast<float>(v) * s) + rng.next16();
        p[i] = static_cast<uint16_t>(b >> 16);
    }
};

template <int S, class V>
__device__ __forceinline__ void store(typename Store<S>::T *p, uint64_t i, V v, float s,
                                      bool stochastic, Rng &rng)
{
    if (stochastic)
        Store<S>::st_sr(p, i, v, s, rng);
    else
        Store<S>::st(p, i, v, s);
}

// ---------------------------------------------------------------------------
// indexing

// The hardware hands block b to XCD b % 8; give each XCD one contiguous slab
// of blocks so that the neighbour planes a block reads sit in its own L2.
__device__ __forceinline__ uint32_t block_id(int remap)
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    if (!remap)
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

__device__ __forceinline__ void coords(const Geom &g, uint32_t n, int &x, int &y, int &z)
{
    x = static_cast<int>(n % static_cast<uint32_t>(g.nx));
    const uint32_t t = n / static_cast<uint32_t>(g.nx);
    y = static_cast<int>(t % static_cast<uint32_t>(g.ny));
    z = static_cast<int>(t / static_cast<uint32_t>(g.ny));
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
// particle, the wall velocity for a wall id, zero otherwise.
__device__ void boundary_velocity_d(const Geom &g, const Bound &b, uint8_t m, int x, int y, int z,
                                    double ub[3])
{
    ub[0] = ub[1] = ub[2] = 0.0;
    if (m < PART0) {
        if (m >= 1 && m <= b.n_walls) {
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

__device__ __forceinline__ void boundary_velocity(const Geom &g, const Bound &b, uint8_t m, int x,
                                                  int y, int z, float ub[3])
{
    double d[3];
    boundary_velocity_d(g, b, m, x, y, z, d);
    ub[0] = static_cast<float>(d[0]);
    ub[1] = static_cast<float>(d[1]);
    ub[2] = static_cast<float>(d[2]);
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
// Arithmetic in R (FP64 for FP32 storage, FP32 for half storage).

template <int S>
__global__ __launch_bounds__(BLOCK) void lb_step_kernel(StepArgs a)
{
    using St = Store<S>;
    using T = typename St::T;
    using R = typename St::R;
    const uint32_t n = block_id(a.remap) * BLOCK + threadIdx.x;
    if (n >= a.g.N)
        return;
    const uint8_t *__restrict__ mask = a.mask;
    if (mask[n] != 0)
        return;
    int x, y, z;
    coords(a.g, n, x, y, z);
    const Nbr nb(a.g, x, y, z);
    const uint64_t P = a.g.plane;
    const T *__restrict__ fin = static_cast<const T *>(a.fin);
    T *__restrict__ fout = static_cast<T *>(a.fout);

    // pull: f_i(x) sits in plane i at x - c_i
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = static_cast<R>(St::ld(fin, i * P + nb.at(-CX[i], -CY[i], -CZ[i]), a.inv_scale));

    // force density: body force + polymer force, the face average of the
    // stress with a solid face neighbour taking this cell's stress
    R F[3] = {static_cast<R>(a.g3[0]), static_cast<R>(a.g3[1]), static_cast<R>(a.g3[2])};
    if (a.polymer) {
        const float *__restrict__ tin = a.tin;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t ip = nb.at(k == 0, k == 1, k == 2);
            const uint32_t im = nb.at(-(k == 0), -(k == 1), -(k == 2));
            const uint32_t sp = mask[ip] != 0 ? n : ip;
            const uint32_t sm = mask[im] != 0 ? n : im;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const uint64_t c = static_cast<uint64_t>(TROW[k][j]) * P;
                F[j] += R(0.5) * (static_cast<R>(tin[c + sp]) - static_cast<R>(tin[c + sm]));
            }
        }
    }

    // moments in deviation form: rho = 1 + sum h, rho u = sum h c + F/2
    R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += f[i];
        if (CX[i])
            jx += CX[i] * f[i];
        if (CY[i])
            jy += CY[i] * f[i];
        if (CZ[i])
            jz += CZ[i] * f[i];
    }
    const R rho = R(1) + drho;
    const R inv_rho = R(1) / rho;
    const R ux = (jx + R(0.5) * F[0]) * inv_rho;
    const R uy = (jy + R(0.5) * F[1]) * inv_rho;
    const R uz = (jz + R(0.5) * F[2]) * inv_rho;
    const R uu = ux * ux + uy * uy + uz * uz;
    const R uF = ux * F[0] + uy * F[1] + uz * F[2];
    const R wp = static_cast<R>(a.wp), wm = static_cast<R>(a.wm);
    const R cp = R(1) - R(0.5) * wp, cm = R(1) - R(0.5) * wm;

    // TRT collision on opposite pairs, Guo source split into its symmetric
    // part (second order, scaled by 1 - w+/2) and antisymmetric part (first
    // order, scaled by 1 - w-/2)
    R fo[Q];
    {
        const R eq0 = static_cast<R>(WD[0]) * (drho - R(1.5) * rho * uu);
        const R s0 = static_cast<R>(WD[0]) * (R(-3) * uF);
        fo[0] = f[0] - wp * (f[0] - eq0) + cp * s0;
    }
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const int o = i + 1;
        const R cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const R cF = CX[i] * F[0] + CY[i] * F[1] + CZ[i] * F[2];
        const R w = static_cast<R>(WD[i]);
        const R eqp = w * (drho + rho * (R(4.5) * cu * cu - R(1.5) * uu));
        const R eqm = w * rho * R(3) * cu;
        const R sp = w * (R(9) * cu * cF - R(3) * uF);
        const R sm = w * R(3) * cF;
        const R hp = R(0.5) * (f[i] + f[o]);
        const R hm = R(0.5) * (f[i] - f[o]);
        const R np = hp - wp * (hp - eqp) + cp * sp;
        const R nm = hm - wm * (hm - eqm) + cm * sm;
        fo[i] = np + nm;
        fo[o] = np - nm;
    }
    Rng rng(n, a.step, a.seed);
    const bool sr = a.stochastic != 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store<S>(fout, i * P + n, fo[i], a.scale, sr, rng);

    // links into solid cells: reflect into the solid slot the next pull reads
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        const uint32_t m = nb.at(CX[j], CY[j], CZ[j]);
        const uint8_t mb = mask[m];
        if (mb != 0) {
            R val = fo[j];
            if (a.b.moving) {
                double ub[3];
                boundary_velocity_d(a.g, a.b, mb, nb.xc[CX[j] + 1], nb.yc[CY[j] + 1],
                                    nb.zc[CZ[j] + 1], ub);
                val -= R(6) * static_cast<R>(WD[j]) * rho *
                       static_cast<R>(CX[j] * ub[0] + CY[j] * ub[1] + CZ[j] * ub[2]);
            }
            store<S>(fout, OPP[j] * P + m, val, a.scale, sr, rng);
        }
    }

    if (a.polymer) {
        a.u[n] = static_cast<float>(ux);
        a.u[P + n] = static_cast<float>(uy);
        a.u[2 * P + n] = static_cast<float>(uz);
    }
}

// ---------------------------------------------------------------------------
// Finite-volume Oldroyd-B stress update (Section 2.2 source, Section 3.3),
// arithmetic in R.

template <class R>
__device__ __forceinline__ R face_overlap(const R u[3], int k, int s)
{
    const R ue = s * u[k];
    if (ue <= R(0))
        return R(0);
    const int a1 = k == 0 ? 1 : 0, a2 = k == 2 ? 1 : 2;
    return ue * (R(1) - fabs(u[a1])) * (R(1) - fabs(u[a2]));
}

template <class R>
__global__ __launch_bounds__(BLOCK) void fv_step_kernel(StepArgs a)
{
    const uint32_t n = block_id(a.remap) * BLOCK + threadIdx.x;
    if (n >= a.g.N)
        return;
    const uint8_t *__restrict__ mask = a.mask;
    if (mask[n] != 0)
        return;
    int x, y, z;
    coords(a.g, n, x, y, z);
    const Nbr nb(a.g, x, y, z);
    const uint64_t P = a.g.plane;
    const float *__restrict__ u = a.u;
    const float *__restrict__ tin = a.tin;
    const R u0[3] = {u[n], u[P + n], u[2 * P + n]};
    R t0[6];
#pragma unroll
    for (int c = 0; c < 6; ++c)
        t0[c] = tin[c * P + n];
    R G[3][3];
    R acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R us[2][3];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int s = side == 0 ? 1 : -1;
            const int cx = s * (k == 0), cy = s * (k == 1), cz = s * (k == 2);
            const uint32_t m = nb.at(cx, cy, cz);
            const uint8_t mb = mask[m];
            if (mb == 0) {
                us[side][0] = u[m];
                us[side][1] = u[P + m];
                us[side][2] = u[2 * P + m];
                const R out = face_overlap(u0, k, s);
                const R in = face_overlap(us[side], k, -s);
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    acc[c] += in * static_cast<R>(tin[c * P + m]) - out * t0[c];
            } else {
                double ub[3];
                boundary_velocity_d(a.g, a.b, mb, nb.xc[cx + 1], nb.yc[cy + 1], nb.zc[cz + 1], ub);
                us[side][0] = static_cast<R>(ub[0]);
                us[side][1] = static_cast<R>(ub[1]);
                us[side][2] = static_cast<R>(ub[2]);
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            G[k][j] = R(0.5) * (us[0][j] - us[1][j]);
    }
    // source: sum_k tau_ik G_kj + sum_k tau_kj G_ki + eta_p/lam (G_ij + G_ji) - tau_ij/lam
    const R T3[3][3] = {{t0[0], t0[3], t0[4]}, {t0[3], t0[1], t0[5]}, {t0[4], t0[5], t0[2]}};
    const int PI[6] = {0, 1, 2, 0, 0, 1};
    const int PJ[6] = {0, 1, 2, 1, 2, 2};
    const R epl = static_cast<R>(a.eta_p_lam), il = static_cast<R>(a.inv_lam);
    float *__restrict__ tout = a.tout;
    Rng rng(n, a.step, a.seed ^ 0x5bd1e995u);
    const bool sr = a.stochastic != 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int i = PI[c], j = PJ[c];
        R s = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            s += T3[i][k] * G[k][j] + T3[k][j] * G[k][i];
        s += epl * (G[i][j] + G[j][i]) - t0[c] * il;
        store<ST_F32>(tout, c * P + n, t0[c] + (acc[c] + s), 1.f, sr, rng);
    }
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

template <int S>
__global__ __launch_bounds__(BLOCK) void read_moments_kernel(Geom g, Bound b, const uint8_t *mask,
                                                             const void *fv, const float *tau,
                                                             int polymer, float gx, float gy,
                                                             float gz, float inv_scale,
                                                             double *rho_out, double *u_out)
{
    using St = Store<S>;
    using T = typename St::T;
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N)
        return;
    if (mask[n] != 0) {
        if (rho_out)
            rho_out[n] = 0.0;
        if (u_out)
            for (int a = 0; a < 3; ++a)
                u_out[static_cast<uint64_t>(a) * g.N + n] = 0.0;
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
    if (polymer) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t ip = nb.at(k == 0, k == 1, k == 2);
            const uint32_t im = nb.at(-(k == 0), -(k == 1), -(k == 2));
            const uint32_t sp = mask[ip] != 0 ? n : ip;
            const uint32_t sm = mask[im] != 0 ? n : im;
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                const uint64_t c = static_cast<uint64_t>(TROW[k][jj]) * g.plane;
                F[jj] += 0.5 * (static_cast<double>(tau[c + sp]) - static_cast<double>(tau[c + sm]));
            }
        }
    }
    const double rho = 1.0 + drho;
    if (rho_out)
        rho_out[n] = rho;
    if (u_out)
        for (int a = 0; a < 3; ++a)
            u_out[static_cast<uint64_t>(a) * g.N + n] = (j[a] + 0.5 * F[a]) / rho;
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
                                                         const float *tau, double *out)
{
    const uint32_t n = blockIdx.x * BLOCK + threadIdx.x;
    if (n >= g.N)
        return;
    const bool fl = mask[n] == 0;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        out[static_cast<uint64_t>(c) * g.N + n] = fl ? static_cast<double>(tau[c * g.plane + n]) : 0.0;
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
                            Match owner_match, double acc[12])
{
    using St = Store<S>;
    using T = typename St::T;
    const T *f = static_cast<const T *>(fv);
    const Nbr nb(g, x, y, z);
    const uint32_t n = nb.at(0, 0, 0);
#pragma unroll
    for (int d = 1; d < Q; ++d) {
        const uint32_t m = nb.at(CX[d], CY[d], CZ[d]);
        if (!owner_match(mask[m]))
            continue;
        // f*_d(x) in its own slot, the reflected population in the solid slot
        const double s = 2.0 * WD[d] + static_cast<double>(St::ld(f, d * g.plane + n, inv_scale)) +
                         static_cast<double>(St::ld(f, OPP[d] * g.plane + m, inv_scale));
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
            const uint32_t m = nb.at(cx, cy, cz);
            if (!owner_match(mask[m]))
                continue;
            double dF[3];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dF[j] = -s * static_cast<double>(tau[TROW[k][j] * g.plane + n]);
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

template <int S>
__global__ __launch_bounds__(BLOCK) void particle_forces_kernel(Geom g, const uint8_t *mask,
                                                                const void *fv, const float *tau,
                                                                int polymer, float inv_scale,
                                                                Particle *parts)
{
    __shared__ double sh[BLOCK / 64];
    const int p = blockIdx.x;
    const Particle P = parts[p];
    const uint8_t me = static_cast<uint8_t>(PART0 + p);
    const Box bx = particle_box(g, P, 2);
    const uint32_t vol = static_cast<uint32_t>(bx.ext[0]) * bx.ext[1] * bx.ext[2];
    double acc[12] = {0};
    for (uint32_t k = threadIdx.x; k < vol; k += BLOCK) {
        int x, y, z;
        box_cell(g, bx, k, x, y, z);
        const uint32_t n = x + static_cast<uint32_t>(g.nx) * (y + static_cast<uint32_t>(g.ny) * z);
        if (mask[n] != 0)
            continue;
        link_forces<S>(g, mask, fv, tau, polymer, inv_scale, x, y, z, &P,
                       [me](uint8_t m) { return m == me; }, acc);
    }
    double r[12];
    for (int k = 0; k < 12; ++k)
        r[k] = block_sum<BLOCK>(acc[k], sh);
    if (threadIdx.x == 0) {
        Particle &Q_ = parts[p];
        for (int a = 0; a < 3; ++a) {
            Q_.fmex[a] = r[a];
            Q_.tmex[a] = r[3 + a];
            Q_.ftau[a] = r[6 + a];
            Q_.ttau[a] = r[9 + a];
        }
    }
}

template <int S>
__global__ __launch_bounds__(BLOCK) void wall_force_kernel(Geom g, const uint8_t *mask,
                                                           const void *fv, const float *tau,
                                                           int polymer, float inv_scale,
                                                           double *partials)
{
    __shared__ double sh[BLOCK / 64];
    double acc[12] = {0};
    for (uint32_t n = blockIdx.x * BLOCK + threadIdx.x; n < g.N; n += gridDim.x * BLOCK) {
        if (mask[n] != 0)
            continue;
        int x, y, z;
        coords(g, n, x, y, z);
        link_forces<S>(g, mask, fv, tau, polymer, inv_scale, x, y, z, nullptr,
                       [](uint8_t m) { return m != 0 && m < PART0; }, acc);
    }
    for (int a = 0; a < 3; ++a) {
        const double r = block_sum<BLOCK>(acc[a] + acc[6 + a], sh);
        if (threadIdx.x == 0)
            partials[blockIdx.x * 3 + a] = r;
    }
}

// Section 3.4: totals and symplectic Euler (velocity first, then position
// with the new velocity).
__global__ void particle_update_kernel(Geom g, Particle *parts, int n_parts)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_parts)
        return;
    Particle &P = parts[p];
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

// ---------------------------------------------------------------------------
// Fluid/solid conversion around movable particles (Section 3.4), one block.
// The new owner of a cell is a pure function of its old mask byte and the
// updated particle positions, so every phase is a gather and needs no
// atomics; phases are separated by barriers.

constexpr int CONV_THREADS = 1024;

struct ConvCtx {
    Geom g;
    const Particle *parts;
    int n_parts;
    const uint8_t *mask;
    const int *moving;  // indices of movable particles (LDS)
    int n_moving;
};

__device__ bool inside_sphere(const Geom &g, const Particle &P, int x, int y, int z)
{
#pragma clang fp contract(off)
    double r[3];
    lever(g, P, x, y, z, r);
    const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    return d2 < P.radius * P.radius;
}

__device__ uint8_t new_owner(const ConvCtx &c, uint32_t n, int x, int y, int z)
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

template <int S>
__global__ __launch_bounds__(CONV_THREADS) void conversion_kernel(Geom g, Bound b, uint8_t *mask,
                                                                  void *fv, float *tau, float scale,
                                                                  float inv_scale, int32_t *counters)
{
    using St = Store<S>;
    using T = typename St::T;
    __shared__ int moving[MAX_PARTICLES];
    __shared__ int n_moving;
    __shared__ double sh[CONV_THREADS / 64];
    Particle *parts = const_cast<Particle *>(b.parts);
    T *f = static_cast<T *>(fv);
    if (threadIdx.x == 0) {
        int k = 0;
        for (int p = 0; p < b.n_parts; ++p)
            if (parts[p].movable)
                moving[k++] = p;
        n_moving = k;
    }
    __syncthreads();
    ConvCtx c{g, parts, b.n_parts, mask, moving, n_moving};
    const uint64_t PL = g.plane;
    auto cell = [&](int x, int y, int z) {
        return static_cast<uint32_t>(x) + static_cast<uint32_t>(g.nx) * (y + static_cast<uint32_t>(g.ny) * z);
    };

    // Phase 1: covers.  The populations' momentum goes to the particle; the
    // stress is shared among the D3Q19 neighbours that stay fluid (gathered
    // by each receiver).
    int covers = 0, dropped = 0;
    for (int q = 0; q < n_moving; ++q) {
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
    for (int q = 0; q < n_moving; ++q) {
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
    for (int q = 0; q < n_moving; ++q) {
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
    for (int q = 0; q < n_moving; ++q) {
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
    for (int q = 0; q < n_moving; ++q) {
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

hipError_t launch_lb_step(int storage, const StepArgs &a, hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(lb_step_kernel<decltype(st)::value>, dim3(blocks_for(a.g.N)), dim3(BLOCK),
                           0, s, a);
        return hipGetLastError();
    });
}

hipError_t launch_fv_step(int storage, const StepArgs &a, hipStream_t s)
{
    if (storage == ST_F32)
        hipLaunchKernelGGL(fv_step_kernel<double>, dim3(blocks_for(a.g.N)), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(fv_step_kernel<float>, dim3(blocks_for(a.g.N)), dim3(BLOCK), 0, s, a);
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
                               float inv_scale, double *rho_out, double *u_out, hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(read_moments_kernel<decltype(st)::value>, dim3(blocks_for(g.N)),
                           dim3(BLOCK), 0, s, g, b, mask, f, tau, polymer, gvec[0], gvec[1],
                           gvec[2], inv_scale, rho_out, u_out);
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
                              hipStream_t s)
{
    hipLaunchKernelGGL(read_tau_kernel, dim3(blocks_for(g.N)), dim3(BLOCK), 0, s, g, mask, tau,
                       out);
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
                                  Particle *parts, int n_parts, hipStream_t s)
{
    if (n_parts <= 0)
        return hipSuccess;
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(particle_forces_kernel<decltype(st)::value>, dim3(n_parts), dim3(BLOCK),
                           0, s, g, mask, f, tau_n, polymer, inv_scale, parts);
        return hipGetLastError();
    });
}

hipError_t launch_wall_force(int storage, const Geom &g, const uint8_t *mask, const void *f,
                             const float *tau_n, int polymer, float inv_scale, double *partials,
                             double *out, hipStream_t s)
{
    const int nb = sums_blocks(g);
    hipError_t e = dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(wall_force_kernel<decltype(st)::value>, dim3(nb), dim3(BLOCK), 0, s, g,
                           mask, f, tau_n, polymer, inv_scale, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(sums_final_kernel, dim3(1), dim3(BLOCK), 0, s, partials, nb, 3, out);
    return hipGetLastError();
}

hipError_t launch_particle_update(const Geom &g, Particle *parts, int n_parts, hipStream_t s)
{
    if (n_parts <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(particle_update_kernel, dim3((n_parts + 63) / 64), dim3(64), 0, s, g, parts,
                       n_parts);
    return hipGetLastError();
}

hipError_t launch_conversion(int storage, const Geom &g, const Bound &b, uint8_t *mask, void *f,
                             float *tau, float scale, float inv_scale, int32_t *counters,
                             hipStream_t s)
{
    return dispatch(storage, [&](auto st) {
        hipLaunchKernelGGL(conversion_kernel<decltype(st)::value>, dim3(1), dim3(CONV_THREADS), 0,
                           s, g, b, mask, f, tau, scale, inv_scale, counters);
        return hipGetLastError();
    });
}

}  // namespace vlb
