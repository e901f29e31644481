// Host runtime of libvlb: the C ABI of include/vlb.h over the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vlb.h"
#include "vlb_internal.h"

using vlb::Particle;

namespace {

thread_local std::string g_create_error = "no error";

constexpr uint64_t kPlaneAlign = 256;  // elements; keeps every plane 512 B+ aligned

// Extra elements between consecutive planes of a field.  Planes of a
// power-of-two size would start on the same HBM channel; an odd multiple of
// the alignment staggers them.  VLB_PLANE_PAD (elements, multiple of 256)
// overrides it for tuning.
uint64_t plane_pad()
{
    static uint64_t pad = [] {
        const char *e = std::getenv("VLB_PLANE_PAD");
        if (e) {
            const long long v = std::atoll(e);
            if (v >= 0)
                return static_cast<uint64_t>(v) / kPlaneAlign * kPlaneAlign;
        }
        return static_cast<uint64_t>(9 * kPlaneAlign);
    }();
    return pad;
}

// Block order of the per-cell kernels: y-slabs per XCD when a z-plane
// splits into 8 equal runs of whole 256-cell blocks, else one contiguous
// block range per XCD.  VLB_XCD_REMAP (0, 1, 2) overrides it for tuning.
int remap_blocks(const vlb::Geom &g, uint32_t &slab_blocks)
{
    static int forced = [] {
        const char *e = std::getenv("VLB_XCD_REMAP");
        return e ? std::atoi(e) : -1;
    }();
    const uint64_t nxy = static_cast<uint64_t>(g.nx) * g.ny;
    const bool slabs_fit = nxy % (8ull * vlb::BLOCK) == 0;
    slab_blocks = slabs_fit ? static_cast<uint32_t>(nxy / (8ull * vlb::BLOCK)) : 0;
    int mode = slabs_fit ? 2 : 1;
    if (forced >= 0)
        mode = forced;
    if (mode == 2 && !slabs_fit)
        mode = 1;
    return mode;
}

// Block order of stream-collide: the hardware's (0), measured faster than
// the XCD-aware orders the stress update keeps, unless VLB_LB_REMAP (0, 1,
// 2) asks for one of those.
int lb_remap_blocks(const vlb::Geom &g)
{
    static int forced = [] {
        const char *e = std::getenv("VLB_LB_REMAP");
        return e ? std::atoi(e) : 0;
    }();
    uint32_t slab_blocks = 0;
    const int fitted = remap_blocks(g, slab_blocks);
    return forced == 2 ? fitted : (forced == 1 ? 1 : 0);
}

// Stress-update kernel: tiled (64 x 4 tiles marching through 16 planes)
// where the lattice is large enough, per-cell otherwise.  VLB_FV_TILE
// overrides it (0 = per-cell kernel, 4 or 8 = rows per tile, negative = that
// many rows whatever the lattice size) and VLB_FV_ZC sets the planes per
// chunk; both are read at every step.
int fv_tile_rows()
{
    const char *e = std::getenv("VLB_FV_TILE");
    return e ? std::atoi(e) : 4;
}

uint32_t fv_z_chunk()
{
    const char *e = std::getenv("VLB_FV_ZC");
    const long v = e ? std::atol(e) : 16;
    return static_cast<uint32_t>(v > 0 && v < 65536 ? v : 16);
}

// Fused step (stream-collide and stress update in one kernel, the same
// bits, measured slower than the two kernels): 0 (default) never, 1 where
// the lattice fills the chip with its tiles, -1 for every polymer lattice.
// VLB_FUSED selects it, VLB_STEP_ZC sets the planes per chunk (0 = the
// kernel's default); both are read at every step.
int fused_mode()
{
    const char *e = std::getenv("VLB_FUSED");
    return e ? std::atoi(e) : 0;
}

uint32_t step_z_chunk()
{
    const char *e = std::getenv("VLB_STEP_ZC");
    const long v = e ? std::atol(e) : 0;
    return static_cast<uint32_t>(v > 0 && v < 65536 ? v : 0);
}

size_t storage_bytes(int storage) { return storage == vlb::ST_F32 ? 4 : 2; }

float default_scale(int storage) { return storage == vlb::ST_F16 ? 1024.f : 1.f; }

// Conversion in one block for every particle, even where their cells are
// far apart (VLB_CONV_SERIAL=1): the reference order the per-particle blocks
// must reproduce bit for bit.  Read when the step arguments are built.
bool conv_serial()
{
    const char *e = std::getenv("VLB_CONV_SERIAL");
    return e && e[0] == '1';
}

// FP16 storage scale for a flow whose speed stays below u_max: the largest
// 2^k, k <= 24, with 2^k * max(u_max, 1e-4) <= 64.
float fp16_scale_for(double u_max)
{
    const double d = u_max > 1e-4 ? u_max : 1e-4;
    int k = 0;
    while (k < 24 && std::ldexp(d, k + 1) <= 64.0)
        ++k;
    return std::ldexp(1.f, k);
}

// A storage scale a checkpoint may carry: 1 for FP32 and BF16, a power of
// two from 1 to 2^24 for FP16.
bool valid_scale(int storage, float s)
{
    if (storage != vlb::ST_F16)
        return s == 1.f;
    int e = 0;
    return s >= 1.f && s <= 16777216.f && std::frexp(s, &e) == 0.5f;
}

}  // namespace

struct vlb_lattice {
    vlb::Geom g{};
    int storage = 0;
    float scale = 1.f, inv_scale = 1.f;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    bool external_state = false;  // state buffers owned by the caller
    uint8_t *d_mask = nullptr;
    void *d_f[2] = {nullptr, nullptr};
    float *d_tau[2] = {nullptr, nullptr};
    float *d_u = nullptr;
    double *d_wall = nullptr;
    double *d_wfield = nullptr;   // per-cell wall velocity [3][N] (null: wall table)
    std::vector<double> wfield_h; // host copy, for checkpoints
    float *d_gfield = nullptr;    // per-cell force density, 3 planes of g.plane (null: none)
    std::vector<float> gfield_h;  // host copy [3][N], for checkpoints
    // graph replays of 32, 16, 8, 4, 2 and 1 steps for each starting buffer
    // parity, with the step arguments and launch shape they were captured
    // with
    uint32_t *d_step = nullptr;   // base step the replayed kernels add their offset to
    hipGraphExec_t gexec[2][6] = {{nullptr}, {nullptr}};  // [parity][log2 length]
    bool gvalid = false;
    vlb::StepArgs gkey;
    int gshape[3] = {0, 0, 0};    // tile rows, z chunk, path flags
    bool graph_broken = false;    // capture failed once: keep launching step by step
    Particle *d_parts = nullptr;
    double *d_partials = nullptr;
    double *d_pforce = nullptr;   // block sums of the obstacle forces
    uint32_t *d_count = nullptr;  // fluid cells (counter-force)
    double *d_g3 = nullptr;       // body force under counter-force
    bool counter_force = false;
    double alpha = 0.0;           // Giesekus mobility
    double L2 = 0.0;              // FENE-P extensibility (0: off)
    int extrap = 0;               // stress extrapolation into solid neighbours
    int smooth_ns = 0;            // overlap sub-samples per axis of smoothed conversions (0: off)
    bool raw_f32 = false;         // raw-FP32 storage control (not kept in checkpoints)
    vlb::StressMap stress_map() const
    {
        vlb::StressMap m;
        m.extrap = extrap;
        if (L2 > 0.0 && polymer) {
            const double eta_p = params.beta * params.eta;
            m.c = static_cast<float>(params.lambda_p / eta_p);
            m.l2m3 = static_cast<float>(L2 - 3.0);
            m.epl = static_cast<float>(eta_p / params.lambda_p);
        }
        return m;
    }
    double *d_out = nullptr;
    int32_t *d_counters = nullptr;
    uint8_t *d_owner = nullptr;  // new owner of each cell near a converting particle
    int n_walls = 0;
    std::vector<double> wall_h;
    std::vector<Particle> parts_h;  // host copy of static particle data
    bool any_movable = false;
    bool moving_walls = false;
    std::vector<uint8_t> mask_h;
    bool mask_h_valid = true;
    vlb_params params{};
    double wp = 1.0, wm = 1.0;
    int rounding = VLB_ROUND_STOCHASTIC;
    uint32_t seed = 0x2009u;
    int polymer = 0;
    int cur = 0;
    int64_t step = 0;
    int64_t check_interval = 1000;
    bool unstable = false;
    bool timing = false;
    bool fused_last = false;  // the last step launched ran the fused kernel
    double ktime[3] = {-1.0, -1.0, -1.0};
    std::vector<hipEvent_t> events;
    std::string err = "no error";

    vlb::Bound bound() const
    {
        vlb::Bound b;
        b.wall_vel = d_wall;
        b.n_walls = n_walls;
        b.wall_field = d_wfield;
        b.parts = d_parts;
        b.n_parts = static_cast<int32_t>(parts_h.size());
        b.moving = (any_movable || moving_walls) ? 1 : 0;
        b.walls_move = moving_walls ? 1 : 0;
        b.smooth_ns = smooth_ns;
        b.conv_serial = conv_serial() ? 1 : 0;
        b.raw_f32 = raw_f32 ? 1 : 0;
        return b;
    }
};

namespace {

vlb_status fail(vlb_lattice *lat, vlb_status st, const std::string &msg)
{
    if (lat)
        lat->err = msg;
    else
        g_create_error = msg;
    return st;
}

vlb_status hip_fail(vlb_lattice *lat, hipError_t e, const char *what)
{
    return fail(lat, e == hipErrorOutOfMemory ? VLB_ENOMEM : VLB_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(lat, expr, what)                      \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess)                        \
            return hip_fail((lat), e_, (what));      \
    } while (0)

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

bool rates(const vlb_params &p, double &wp, double &wm)
{
    const double eta_n = (1.0 - p.beta) * p.eta;
    const double dwp = 1.0 / (3.0 * eta_n + 0.5);
    double dwm = dwp;
    if (p.magic >= 0.0)
        dwm = 1.0 / (0.5 + p.magic / (1.0 / dwp - 0.5));
    if (!(dwp > 0.0 && dwp < 2.0 && dwm > 0.0 && dwm < 2.0))
        return false;
    wp = dwp;
    wm = dwm;
    return true;
}

vlb_status check_dims(const vlb_dims *d)
{
    if (!d || d->nx < 1 || d->ny < 1 || d->nz < 1)
        return VLB_EINVAL;
    // kernels address every field plane with 32-bit byte offsets: a plane of
    // FP32 values must stay below 4 GiB
    const uint64_t N = static_cast<uint64_t>(d->nx) * d->ny * d->nz;
    if (N + kPlaneAlign + plane_pad() >= (1ull << 30))
        return VLB_EINVAL;
    return VLB_OK;
}

// every non-periodic axis needs solid first and last layers
bool end_layers_solid(const vlb_dims *d, const uint8_t *mask)
{
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int ax = 0; ax < 3; ++ax) {
        if (d->periodic[ax])
            continue;
        for (int z = 0; z < n[2]; ++z)
            for (int y = 0; y < n[1]; ++y)
                for (int x = 0; x < n[0]; ++x) {
                    const int c[3] = {x, y, z};
                    if (c[ax] != 0 && c[ax] != n[ax] - 1)
                        continue;
                    if (mask[x + static_cast<size_t>(n[0]) * (y + static_cast<size_t>(n[1]) * z)] == 0)
                        return false;
                }
    }
    return true;
}

vlb_status sync_mask_host(vlb_lattice *lat)
{
    if (lat->mask_h_valid)
        return VLB_OK;
    HIPCHK(lat, hipMemcpyAsync(lat->mask_h.data(), lat->d_mask, lat->g.N, hipMemcpyDeviceToHost,
                               lat->stream),
           "mask download");
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "mask download");
    lat->mask_h_valid = true;
    return VLB_OK;
}

vlb_status upload_particles(vlb_lattice *lat)
{
    if (lat->parts_h.empty())
        return VLB_OK;
    HIPCHK(lat, hipMemcpyAsync(lat->d_parts, lat->parts_h.data(),
                               sizeof(Particle) * lat->parts_h.size(), hipMemcpyHostToDevice,
                               lat->stream),
           "particle upload");
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "particle upload");
    return VLB_OK;
}

vlb_status download_particles(vlb_lattice *lat, std::vector<Particle> &out)
{
    out.resize(lat->parts_h.size());
    if (out.empty())
        return VLB_OK;
    HIPCHK(lat, hipMemcpyAsync(out.data(), lat->d_parts, sizeof(Particle) * out.size(),
                               hipMemcpyDeviceToHost, lat->stream),
           "particle download");
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "particle download");
    return VLB_OK;
}

void free_all(vlb_lattice *lat)
{
    if (lat->stream)
        (void)hipStreamSynchronize(lat->stream);
    void *state[] = {lat->d_mask, lat->d_f[0], lat->d_f[1], lat->d_tau[0], lat->d_tau[1], lat->d_u};
    if (!lat->external_state)
        for (void *p : state)
            if (p)
                (void)hipFree(p);
    for (auto &row : lat->gexec)
        for (hipGraphExec_t &x : row)
            if (x) {
                (void)hipGraphExecDestroy(x);
                x = nullptr;
            }
    void *ptrs[] = {lat->d_wall,   lat->d_parts, lat->d_partials, lat->d_out,
                    lat->d_counters, lat->d_pforce, lat->d_count, lat->d_g3,
                    lat->d_wfield, lat->d_gfield, lat->d_step, lat->d_owner};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    for (hipEvent_t e : lat->events)
        (void)hipEventDestroy(e);
    if (lat->own_stream && lat->stream)
        (void)hipStreamDestroy(lat->stream);
}

// run `fn(device_scratch)` with a temporary device buffer and copy it to host
template <class Fn>
vlb_status read_via_scratch(vlb_lattice *lat, size_t bytes, void *host, Fn fn, const char *what)
{
    void *d = nullptr;
    HIPCHK(lat, hipMalloc(&d, bytes), what);
    hipError_t e = fn(static_cast<double *>(d));
    if (e == hipSuccess)
        e = hipMemcpyAsync(host, d, bytes, hipMemcpyDeviceToHost, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    (void)hipFree(d);
    if (e != hipSuccess)
        return hip_fail(lat, e, what);
    return VLB_OK;
}

template <class Fn>
vlb_status write_via_scratch(vlb_lattice *lat, size_t bytes, const void *host, Fn fn,
                             const char *what)
{
    void *d = nullptr;
    HIPCHK(lat, hipMalloc(&d, bytes), what);
    hipError_t e = hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, lat->stream);
    if (e == hipSuccess)
        e = fn(static_cast<const double *>(d));
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    (void)hipFree(d);
    if (e != hipSuccess)
        return hip_fail(lat, e, what);
    return VLB_OK;
}

// FP64 sums of the current state into out[8]
vlb_status run_sums(vlb_lattice *lat, double out[8])
{
    HIPCHK(lat, vlb::launch_sums(lat->storage, lat->g, lat->d_mask, lat->d_f[lat->cur],
                                 lat->inv_scale, lat->d_partials, lat->d_out, lat->stream),
           "sums");
    HIPCHK(lat, hipMemcpyAsync(out, lat->d_out, 8 * sizeof(double), hipMemcpyDeviceToHost,
                               lat->stream),
           "sums");
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "sums");
    return VLB_OK;
}

constexpr double kMaxSpeed = 0.3;

// |d|^2 evaluated left to right without fused multiply-add, the same way the
// device-side coverage test does
double sq_norm(const double d[3])
{
#pragma clang fp contract(off)
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

}  // namespace

extern "C" {

int32_t vlb_velocity(int32_t i, int32_t c[3], double *w)
{
    if (i >= 0 && i < vlb::Q) {
        if (c) {
            c[0] = vlb::CX[i];
            c[1] = vlb::CY[i];
            c[2] = vlb::CZ[i];
        }
        if (w)
            *w = vlb::WD[i];
    }
    return vlb::Q;
}

size_t vlb_required_bytes(const vlb_dims *dims, vlb_storage storage, int32_t n_particles)
{
    if (check_dims(dims) != VLB_OK)
        return 0;
    const uint64_t N = static_cast<uint64_t>(dims->nx) * dims->ny * dims->nz;
    const uint64_t P = round_up(N, kPlaneAlign) + plane_pad();
    const uint64_t pops = 2ull * vlb::Q * P * storage_bytes(storage);
    const uint64_t tau = 2ull * 6 * P * sizeof(float);
    const uint64_t u = 3ull * P * sizeof(float);
    const uint64_t mask = 2 * round_up(N, 256);  // the mask and the conversion's owner map
    const uint64_t small = sizeof(Particle) * vlb::MAX_PARTICLES + 64 * 3 * sizeof(double) +
                           2048 * 8 * sizeof(double) + 4096 +
                           vlb::MAX_PARTICLES * vlb::PF_BLOCKS * 12 * sizeof(double);
    (void)n_particles;
    return static_cast<size_t>(pops + tau + u + mask + small);
}

namespace {

// sizes of the caller-providable state buffers (VLB_NBUF entries)
void state_sizes(uint64_t N, uint64_t P, size_t es, size_t sizes[VLB_NBUF])
{
    sizes[0] = static_cast<size_t>(round_up(N, 256));
    sizes[1] = sizes[2] = static_cast<size_t>(vlb::Q * P * es);
    sizes[3] = sizes[4] = static_cast<size_t>(6 * P * sizeof(float));
    sizes[5] = static_cast<size_t>(3 * P * sizeof(float));
}

vlb_status create_impl(const vlb_dims *dims, const uint8_t *mask, const double *wall_velocity,
                       int32_t n_walls, vlb_storage storage, void *stream,
                       void *const *buffers, const size_t *buffer_sizes, vlb_lattice **out)
{
    if (!out)
        return fail(nullptr, VLB_EINVAL, "vlb_create: out is NULL");
    *out = nullptr;
    if (check_dims(dims) != VLB_OK)
        return fail(nullptr, VLB_EINVAL, "vlb_create: invalid dimensions");
    if (!mask)
        return fail(nullptr, VLB_EINVAL, "vlb_create: mask is NULL");
    if (storage != VLB_STORE_F32 && storage != VLB_STORE_F16 && storage != VLB_STORE_BF16)
        return fail(nullptr, VLB_EINVAL, "vlb_create: unknown storage");
    if (n_walls < 0 || n_walls > VLB_MAX_WALL_ID || (n_walls > 0 && !wall_velocity))
        return fail(nullptr, VLB_EINVAL, "vlb_create: invalid wall table");
    for (int i = 0; i < 3 * n_walls; ++i)
        if (!std::isfinite(wall_velocity[i]))
            return fail(nullptr, VLB_EINVAL, "vlb_create: non-finite wall velocity");
    const uint64_t N = static_cast<uint64_t>(dims->nx) * dims->ny * dims->nz;
    for (uint64_t n = 0; n < N; ++n)
        if (mask[n] >= vlb::PART0)
            return fail(nullptr, VLB_EINVAL, "vlb_create: mask values >= 64 are reserved");
    if (!end_layers_solid(dims, mask))
        return fail(nullptr, VLB_EINVAL,
                    "vlb_create: a non-periodic axis needs solid first and last layers");
    if (buffers) {
        if (!buffer_sizes)
            return fail(nullptr, VLB_EINVAL, "vlb_create_with_buffers: sizes is NULL");
        size_t need[VLB_NBUF];
        state_sizes(N, round_up(N, kPlaneAlign) + plane_pad(), storage_bytes(storage), need);
        for (int k = 0; k < VLB_NBUF; ++k)
            if (!buffers[k] || buffer_sizes[k] < need[k] ||
                reinterpret_cast<uintptr_t>(buffers[k]) % 256 != 0)
                return fail(nullptr, VLB_EINVAL,
                            "vlb_create_with_buffers: buffer " + std::to_string(k) +
                                " missing, too small or not 256-byte aligned");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, VLB_EDEVICE, "vlb_create: no HIP device");

    int device = 0;
    if (hipGetDevice(&device) != hipSuccess)
        return fail(nullptr, VLB_EDEVICE, "vlb_create: no current HIP device");
    vlb_lattice *lat = new vlb_lattice();
    lat->device = device;
    lat->g.nx = dims->nx;
    lat->g.ny = dims->ny;
    lat->g.nz = dims->nz;
    for (int a = 0; a < 3; ++a)
        lat->g.per[a] = dims->periodic[a] ? 1 : 0;
    lat->g.N = static_cast<uint32_t>(N);
    lat->g.plane = round_up(N, kPlaneAlign) + plane_pad();
    vlb::set_divisors(lat->g);
    lat->storage = storage;
    lat->scale = default_scale(storage);
    lat->inv_scale = 1.f / lat->scale;
    lat->mask_h.assign(mask, mask + N);
    lat->n_walls = n_walls;
    lat->wall_h.assign(64 * 3, 0.0);
    for (int w = 0; w < n_walls; ++w)
        for (int a = 0; a < 3; ++a) {
            lat->wall_h[3 * w + a] = wall_velocity[3 * w + a];
            if (wall_velocity[3 * w + a] != 0.0)
                lat->moving_walls = true;
        }

    auto bail = [&](hipError_t e, const char *what) {
        std::string msg = std::string(what) + ": " + hipGetErrorString(e);
        free_all(lat);
        delete lat;
        return fail(nullptr, e == hipErrorOutOfMemory ? VLB_ENOMEM : VLB_EDEVICE, msg);
    };
    hipError_t e;
    if (stream) {
        lat->stream = static_cast<hipStream_t>(stream);
    } else {
        if ((e = hipStreamCreate(&lat->stream)) != hipSuccess)
            return bail(e, "stream");
        lat->own_stream = true;
    }
    const uint64_t P = lat->g.plane;
    const size_t es = storage_bytes(storage);
    if (buffers) {
        // caller-owned state (e.g. torch tensors), checked on entry
        lat->external_state = true;
        lat->d_mask = static_cast<uint8_t *>(buffers[0]);
        lat->d_f[0] = buffers[1];
        lat->d_f[1] = buffers[2];
        lat->d_tau[0] = static_cast<float *>(buffers[3]);
        lat->d_tau[1] = static_cast<float *>(buffers[4]);
        lat->d_u = static_cast<float *>(buffers[5]);
    } else {
        if ((e = hipMalloc(&lat->d_mask, round_up(N, 256))) != hipSuccess)
            return bail(e, "mask");
        for (int b = 0; b < 2; ++b) {
            if ((e = hipMalloc(&lat->d_f[b], vlb::Q * P * es)) != hipSuccess)
                return bail(e, "populations");
            if ((e = hipMalloc(&lat->d_tau[b], 6 * P * sizeof(float))) != hipSuccess)
                return bail(e, "stress");
        }
        if ((e = hipMalloc(&lat->d_u, 3 * P * sizeof(float))) != hipSuccess)
            return bail(e, "velocity");
    }
    for (int b = 0; b < 2; ++b) {
        if ((e = hipMemsetAsync(lat->d_tau[b], 0, 6 * P * sizeof(float), lat->stream)) != hipSuccess)
            return bail(e, "stress");
        if ((e = hipMemsetAsync(lat->d_f[b], 0, vlb::Q * P * es, lat->stream)) != hipSuccess)
            return bail(e, "populations");
    }
    if ((e = hipMemsetAsync(lat->d_u, 0, 3 * P * sizeof(float), lat->stream)) != hipSuccess)
        return bail(e, "velocity");
    if ((e = hipMalloc(&lat->d_wall, 64 * 3 * sizeof(double))) != hipSuccess)
        return bail(e, "walls");
    if ((e = hipMalloc(&lat->d_parts, vlb::MAX_PARTICLES * sizeof(Particle))) != hipSuccess)
        return bail(e, "particles");
    if ((e = hipMalloc(&lat->d_partials, static_cast<size_t>(vlb::sums_blocks(lat->g)) * 8 *
                                             sizeof(double))) != hipSuccess)
        return bail(e, "partials");
    if ((e = hipMalloc(&lat->d_out, 16 * sizeof(double))) != hipSuccess)
        return bail(e, "out");
    if ((e = hipMalloc(&lat->d_pforce, static_cast<size_t>(vlb::MAX_PARTICLES) * vlb::PF_BLOCKS *
                                            12 * sizeof(double))) != hipSuccess)
        return bail(e, "particle force sums");
    if ((e = hipMalloc(&lat->d_count, sizeof(uint32_t))) != hipSuccess)
        return bail(e, "fluid count");
    if ((e = hipMemsetAsync(lat->d_count, 0, sizeof(uint32_t), lat->stream)) != hipSuccess)
        return bail(e, "fluid count");
    if ((e = hipMalloc(&lat->d_g3, 3 * sizeof(double))) != hipSuccess)
        return bail(e, "body force");
    // conversion counts (covers, uncovers, dropped), one unused word, then a
    // change flag per particle
    constexpr size_t n_counters = 4 + vlb::MAX_PARTICLES;
    if ((e = hipMalloc(&lat->d_counters, n_counters * sizeof(int32_t))) != hipSuccess)
        return bail(e, "counters");
    if ((e = hipMemsetAsync(lat->d_counters, 0, n_counters * sizeof(int32_t), lat->stream)) !=
        hipSuccess)
        return bail(e, "counters");
    if ((e = hipMalloc(&lat->d_owner, round_up(N, 256))) != hipSuccess)
        return bail(e, "owner map");
    if ((e = hipMemcpyAsync(lat->d_mask, mask, N, hipMemcpyHostToDevice, lat->stream)) != hipSuccess)
        return bail(e, "mask upload");
    if ((e = hipMemcpyAsync(lat->d_wall, lat->wall_h.data(), 64 * 3 * sizeof(double),
                            hipMemcpyHostToDevice, lat->stream)) != hipSuccess)
        return bail(e, "wall upload");
    if ((e = hipStreamSynchronize(lat->stream)) != hipSuccess)
        return bail(e, "create");

    vlb_params p{};
    p.eta = 1.0 / 3.0;
    p.beta = 0.0;
    p.lambda_p = 1.0;
    p.magic = 3.0 / 16.0;
    if (vlb_set_params(lat, &p) != VLB_OK || vlb_init_equilibrium(lat, nullptr) != VLB_OK) {
        std::string msg = lat->err;
        free_all(lat);
        delete lat;
        return fail(nullptr, VLB_EDEVICE, "vlb_create: " + msg);
    }
    *out = lat;
    return VLB_OK;
}

}  // namespace

vlb_status vlb_create(const vlb_dims *dims, const uint8_t *mask, const double *wall_velocity,
                      int32_t n_walls, vlb_storage storage, void *stream, vlb_lattice **out)
{
    return create_impl(dims, mask, wall_velocity, n_walls, storage, stream, nullptr, nullptr, out);
}

vlb_status vlb_buffer_sizes(const vlb_dims *dims, vlb_storage storage, size_t sizes[VLB_NBUF])
{
    if (!sizes || check_dims(dims) != VLB_OK ||
        (storage != VLB_STORE_F32 && storage != VLB_STORE_F16 && storage != VLB_STORE_BF16))
        return VLB_EINVAL;
    const uint64_t N = static_cast<uint64_t>(dims->nx) * dims->ny * dims->nz;
    state_sizes(N, round_up(N, kPlaneAlign) + plane_pad(), storage_bytes(storage), sizes);
    return VLB_OK;
}

vlb_status vlb_create_with_buffers(const vlb_dims *dims, const uint8_t *mask,
                                   const double *wall_velocity, int32_t n_walls,
                                   vlb_storage storage, void *stream,
                                   void *const buffers[VLB_NBUF], const size_t sizes[VLB_NBUF],
                                   vlb_lattice **out)
{
    if (!buffers)
        return fail(nullptr, VLB_EINVAL, "vlb_create_with_buffers: buffers is NULL");
    return create_impl(dims, mask, wall_velocity, n_walls, storage, stream, buffers, sizes, out);
}

vlb_status vlb_set_params(vlb_lattice *lat, const vlb_params *p)
{
    if (!lat)
        return VLB_EINVAL;
    if (!p)
        return fail(lat, VLB_EINVAL, "vlb_set_params: params is NULL");
    if (!(p->eta > 0.0) || !(p->beta >= 0.0 && p->beta < 1.0))
        return fail(lat, VLB_EINVAL, "vlb_set_params: need eta > 0 and 0 <= beta < 1");
    if (p->beta > 0.0 && !(p->lambda_p >= 1.0))
        return fail(lat, VLB_EINVAL, "vlb_set_params: lambda_p must be >= 1 when beta > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->body_force[a]))
            return fail(lat, VLB_EINVAL, "vlb_set_params: non-finite body force");
    double wp, wm;
    if (!rates(*p, wp, wm))
        return fail(lat, VLB_EINVAL, "vlb_set_params: relaxation rate outside (0, 2)");
    lat->params = *p;
    lat->wp = wp;
    lat->wm = wm;
    const int was = lat->polymer;
    lat->polymer = p->beta > 0.0 ? 1 : 0;
    if (was && !lat->polymer)
        for (int b = 0; b < 2; ++b)
            HIPCHK(lat, hipMemsetAsync(lat->d_tau[b], 0, 6 * lat->g.plane * sizeof(float),
                                       lat->stream),
                   "stress reset");
    return VLB_OK;
}

vlb_status vlb_init_equilibrium(vlb_lattice *lat, const double *u)
{
    if (!lat)
        return VLB_EINVAL;
    vlb_status st = sync_mask_host(lat);
    if (st != VLB_OK)
        return st;
    const size_t N = lat->g.N;
    auto run = [&](const double *du) {
        hipError_t e = vlb::launch_init_equilibrium(lat->storage, lat->g, lat->d_mask, du,
                                                    lat->d_f[lat->cur], lat->scale, lat->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(lat->d_tau[lat->cur], 0, 6 * lat->g.plane * sizeof(float),
                               lat->stream);
        return e;
    };
    if (u) {
        st = write_via_scratch(lat, 3 * N * sizeof(double), u, run, "vlb_init_equilibrium");
    } else {
        hipError_t e = run(nullptr);
        if (e == hipSuccess)
            e = hipStreamSynchronize(lat->stream);
        if (e != hipSuccess)
            return hip_fail(lat, e, "vlb_init_equilibrium");
    }
    if (st == VLB_OK) {
        lat->step = 0;
        lat->unstable = false;
    }
    return st;
}

vlb_status vlb_set_populations(vlb_lattice *lat, const double *f)
{
    if (!lat)
        return VLB_EINVAL;
    if (!f)
        return fail(lat, VLB_EINVAL, "vlb_set_populations: f is NULL");
    return write_via_scratch(
        lat, static_cast<size_t>(vlb::Q) * lat->g.N * sizeof(double), f,
        [&](const double *d) {
            return vlb::launch_set_populations(lat->storage, lat->g, lat->d_mask, d,
                                               lat->d_f[lat->cur], lat->scale, lat->stream);
        },
        "vlb_set_populations");
}

vlb_status vlb_set_stress(vlb_lattice *lat, const double *tau)
{
    if (!lat)
        return VLB_EINVAL;
    if (!tau)
        return fail(lat, VLB_EINVAL, "vlb_set_stress: tau is NULL");
    return write_via_scratch(
        lat, 6 * static_cast<size_t>(lat->g.N) * sizeof(double), tau,
        [&](const double *d) {
            return vlb::launch_set_stress(lat->g, lat->d_mask, d, lat->d_tau[lat->cur],
                                          lat->stream);
        },
        "vlb_set_stress");
}

vlb_status vlb_add_sphere(vlb_lattice *lat, const double center[3], double radius,
                          double density_ratio, int32_t movable, const double f_ext[3],
                          const double t_ext[3], int32_t *id_out)
{
    if (!lat)
        return VLB_EINVAL;
    if (!center || !std::isfinite(center[0]) || !std::isfinite(center[1]) ||
        !std::isfinite(center[2]) || !(radius > 0.0) || !std::isfinite(radius) ||
        !(density_ratio > 0.0))
        return fail(lat, VLB_EINVAL, "vlb_add_sphere: invalid centre, radius or density");
    if (lat->parts_h.size() >= static_cast<size_t>(vlb::MAX_PARTICLES))
        return fail(lat, VLB_EINVAL, "vlb_add_sphere: particle table full");
    vlb_status st = sync_mask_host(lat);
    if (st != VLB_OK)
        return st;
    // current dynamic state of existing particles must be kept
    std::vector<Particle> cur;
    if ((st = download_particles(lat, cur)) != VLB_OK)
        return st;
    Particle P;
    std::memset(&P, 0, sizeof(P));
    for (int a = 0; a < 3; ++a) {
        P.R[a] = center[a];
        P.fext[a] = f_ext ? f_ext[a] : 0.0;
        P.text[a] = t_ext ? t_ext[a] : 0.0;
    }
    P.radius = radius;
    P.mass = density_ratio * 4.0 / 3.0 * M_PI * radius * radius * radius;
    P.inertia = 0.4 * P.mass * radius * radius;
    P.movable = movable ? 1 : 0;
    for (int a = 0; a < 3; ++a)
        P.Rprev[a] = center[a];
    const int id = static_cast<int>(cur.size());
    const int n[3] = {lat->g.nx, lat->g.ny, lat->g.nz};
    // cells with |x - R|^2 < r^2, searched over the sphere's bounding box
    // (wrapped on periodic axes; the whole axis once if the box covers it)
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = static_cast<int>(std::floor(P.R[k] - radius)) - 1;
        hi[k] = static_cast<int>(std::ceil(P.R[k] + radius)) + 1;
        if (!lat->g.per[k]) {
            lo[k] = std::max(lo[k], 0);
            hi[k] = std::min(hi[k], n[k] - 1);
        } else if (hi[k] - lo[k] + 1 >= n[k]) {
            lo[k] = 0;
            hi[k] = n[k] - 1;
        }
    }
    std::vector<uint32_t> cells;
    for (int zz = lo[2]; zz <= hi[2]; ++zz)
        for (int yy = lo[1]; yy <= hi[1]; ++yy)
            for (int xx = lo[0]; xx <= hi[0]; ++xx) {
                const int raw[3] = {xx, yy, zz};
                int c[3];
                double d[3];
                for (int k = 0; k < 3; ++k) {
                    c[k] = ((raw[k] % n[k]) + n[k]) % n[k];
                    d[k] = static_cast<double>(c[k]) - P.R[k];
                    if (lat->g.per[k]) {
                        const double L = static_cast<double>(n[k]);
                        d[k] -= L * std::floor(d[k] / L + 0.5);
                    }
                }
                if (sq_norm(d) < radius * radius) {
                    const uint32_t idx = c[0] + static_cast<uint32_t>(n[0]) *
                                                    (c[1] + static_cast<uint32_t>(n[1]) * c[2]);
                    if (lat->mask_h[idx] != 0)
                        return fail(lat, VLB_EINVAL, "vlb_add_sphere: overlaps a non-fluid cell");
                    cells.push_back(idx);
                }
            }
    for (uint32_t idx : cells)
        lat->mask_h[idx] = static_cast<uint8_t>(vlb::PART0 + id);
    cur.push_back(P);
    lat->parts_h = cur;
    if (movable)
        lat->any_movable = true;
    HIPCHK(lat, hipMemcpyAsync(lat->d_mask, lat->mask_h.data(), lat->g.N, hipMemcpyHostToDevice,
                               lat->stream),
           "mask upload");
    if ((st = upload_particles(lat)) != VLB_OK)
        return st;
    if (id_out)
        *id_out = id;
    return VLB_OK;
}

namespace {

// Graph replays hold 2^level steps, level 0..kGraphLevels-1 (1 .. 32 steps),
// so that any step count runs as a few replays.
constexpr int kGraphLevels = 6;

bool graphs_enabled()
{
    const char *e = std::getenv("VLB_GRAPH");
    return !(e && e[0] == '0');
}

// Point the plane pointers of `a` at the buffers of parity `cur`.
void set_planes(const vlb_lattice *lat, vlb::StepArgs &a, int cur)
{
    a.fin = lat->d_f[cur];
    a.fout = lat->d_f[cur ^ 1];
    a.tin = lat->d_tau[cur];
    a.tout = lat->d_tau[cur ^ 1];
    const size_t pb = lat->g.plane * storage_bytes(lat->storage);
    for (int i = 0; i < vlb::Q; ++i) {
        a.fin_p[i] = static_cast<const char *>(a.fin) + i * pb;
        a.fout_p[i] = static_cast<char *>(a.fout) + i * pb;
    }
    for (int c = 0; c < 6; ++c) {
        a.tin_p[c] = a.tin + c * lat->g.plane;
        a.tout_p[c] = a.tout + c * lat->g.plane;
    }
    for (int c = 0; c < 3; ++c)
        a.u_p[c] = a.u + c * lat->g.plane;
    a.fdelta = static_cast<const char *>(a.fout) - static_cast<const char *>(a.fin);
    a.tdelta = reinterpret_cast<const char *>(a.tout) - reinterpret_cast<const char *>(a.tin);
}

// The kernels of one step, in order: stream-collide, stress update, and for
// moving particles their forces, rigid-body update, conversion and (under
// the counter-force) the next step's body force.  `ev`, if given, receives
// events before stream-collide, before the stress update, before the
// particle path and after it.
hipError_t launch_step(vlb_lattice *lat, const vlb::StepArgs &a, bool counter, int tile_rows,
                       uint32_t z_chunk, hipEvent_t *ev, bool *fused_out = nullptr)
{
    hipStream_t st = lat->stream;
    hipError_t e = hipSuccess;
    auto rec = [&](int k) {
        if (ev && e == hipSuccess)
            e = hipEventRecord(ev[k], st);
    };
    rec(0);
    const int fm = fused_mode();
    bool fused = false;
    if (e == hipSuccess && lat->polymer && fm != 0) {
        e = vlb::launch_step_fused(lat->storage, a, st, step_z_chunk(), fm < 0);
        fused = e == hipSuccess;
        if (e == hipErrorNotSupported)
            e = hipSuccess;
    }
    if (fused_out)
        *fused_out = fused;
    if (e == hipSuccess && !fused)
        e = vlb::launch_lb_step(lat->storage, a, st);
    if (e == hipSuccess && a.b.raw_f32)
        e = vlb::launch_raw_f32_control(lat->g, a.fout, st);
    rec(1);
    if (e == hipSuccess && lat->polymer && !fused)
        e = vlb::launch_fv_step(lat->storage, a, st, tile_rows, z_chunk);
    rec(2);
    if (e == hipSuccess && lat->any_movable) {
        const int np = static_cast<int>(lat->parts_h.size());
        e = vlb::launch_particle_forces(lat->storage, lat->g, lat->d_mask, a.fout, a.tin,
                                        lat->polymer, lat->inv_scale, lat->d_parts, np,
                                        lat->d_pforce, st, lat->stress_map());
        if (e == hipSuccess)
            e = vlb::launch_conversion(lat->storage, lat->g, a.b, lat->d_mask, a.fout, a.tout,
                                       lat->scale, lat->inv_scale, lat->d_counters, lat->d_u,
                                       lat->d_owner, st);
        if (e == hipSuccess && counter)
            e = vlb::launch_body_force(lat->g, lat->d_mask, lat->d_parts, np,
                                       lat->params.body_force, lat->d_count, lat->d_g3, st);
    }
    rec(3);
    return e;
}

// Record the `len` steps that start at parity `par` into a graph
// executable; kernels take their step index as *d_step + offset.
hipError_t capture_steps(vlb_lattice *lat, const vlb::StepArgs &base, int par, int len,
                         bool counter, int tile_rows, uint32_t z_chunk, hipGraphExec_t *out)
{
    hipStream_t st = lat->stream;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return e;
    hipError_t le = hipSuccess;
    for (int k = 0; k < len && le == hipSuccess; ++k) {
        vlb::StepArgs a = base;
        set_planes(lat, a, (par + k) & 1);
        a.step = static_cast<uint32_t>(k);
        a.step_dev = lat->d_step;
        le = launch_step(lat, a, counter, tile_rows, z_chunk, nullptr);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (le == hipSuccess)
        le = e;
    if (le == hipSuccess)
        le = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    // upload now, so that the first replay of this executable does not pay
    // for it inside a caller's timed loop
    if (le == hipSuccess)
        le = hipGraphUpload(*out, st);
    if (graph)
        (void)hipGraphDestroy(graph);
    return le;
}

// One replay of 2^level steps from the lattice's current step and parity.
// Every graph (each length, both parities) is captured again at once when
// the step arguments or the launch shape differ from those they were
// captured with, so that a change costs one capture round and no later
// call of another length captures inside a caller's timed loop.
hipError_t replay_steps(vlb_lattice *lat, const vlb::StepArgs &base, bool counter, int level)
{
    const int tile_rows = fv_tile_rows();
    const uint32_t z_chunk = fv_z_chunk();
    hipError_t e = hipSuccess;
    if (!lat->d_step && (e = hipMalloc(&lat->d_step, sizeof(uint32_t))) != hipSuccess)
        return e;
    vlb::StepArgs key = base;
    set_planes(lat, key, 0);
    key.step = 0;
    key.step_dev = lat->d_step;
    const int flags = (lat->any_movable ? 1 : 0) | (counter ? 2 : 0) | ((fused_mode() + 1) << 2) |
                      static_cast<int>(step_z_chunk() << 4);
    if (!lat->gvalid || std::memcmp(&key, &lat->gkey, sizeof key) != 0 ||
        lat->gshape[0] != tile_rows || lat->gshape[1] != static_cast<int>(z_chunk) ||
        lat->gshape[2] != flags) {
        lat->gvalid = false;
        for (int par = 0; par < 2; ++par)
            for (int lv = 0; lv < kGraphLevels; ++lv) {
                hipGraphExec_t &x = lat->gexec[par][lv];
                if (x) {
                    (void)hipGraphExecDestroy(x);
                    x = nullptr;
                }
                if ((e = capture_steps(lat, base, par, 1 << lv, counter, tile_rows, z_chunk,
                                       &x)) != hipSuccess) {
                    x = nullptr;
                    return e;
                }
            }
        std::memcpy(&lat->gkey, &key, sizeof key);
        lat->gshape[0] = tile_rows;
        lat->gshape[1] = static_cast<int>(z_chunk);
        lat->gshape[2] = flags;
        lat->gvalid = true;
    }
    if ((e = vlb::launch_set_step(lat->d_step, static_cast<uint32_t>(lat->step), 0,
                                  lat->stream)) != hipSuccess)
        return e;
    return hipGraphLaunch(lat->gexec[lat->cur][level], lat->stream);
}

}  // namespace

vlb_status vlb_step(vlb_lattice *lat, int64_t n_steps)
{
    if (!lat)
        return VLB_EINVAL;
    if (n_steps < 0)
        return fail(lat, VLB_EINVAL, "vlb_step: negative step count");
    if (lat->unstable)
        return fail(lat, VLB_EUNSTABLE, "vlb_step: lattice is unstable (sticky)");
    // zeroed padding included, so that step arguments compare bytewise
    vlb::StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = lat->g;
    a.b = lat->bound();
    a.mask = lat->d_mask;
    a.u = lat->d_u;
    a.wp = lat->wp;
    a.wm = lat->wm;
    for (int k = 0; k < 3; ++k)
        a.g3[k] = lat->params.body_force[k];
    const bool counter = lat->counter_force && lat->any_movable;
    a.g3_dev = counter ? lat->d_g3 : nullptr;
    if (lat->d_gfield)
        for (int k = 0; k < 3; ++k)
            a.gf_p[k] = lat->d_gfield + k * lat->g.plane;
    const int n_parts = static_cast<int>(lat->parts_h.size());
    if (counter && n_steps > 0)
        HIPCHK(lat, vlb::launch_body_force(lat->g, lat->d_mask, lat->d_parts, n_parts,
                                           lat->params.body_force, lat->d_count, lat->d_g3,
                                           lat->stream),
               "counter-force");
    a.polymer = lat->polymer;
    if (lat->polymer) {
        a.eta_p_lam = lat->params.beta * lat->params.eta / lat->params.lambda_p;
        a.inv_lam = 1.0 / lat->params.lambda_p;
        a.gk = static_cast<float>(lat->alpha / (lat->params.beta * lat->params.eta));
        a.sm = lat->stress_map();
    }
    a.stochastic = lat->rounding == VLB_ROUND_STOCHASTIC ? 1 : 0;
    a.seed = lat->seed;
    a.scale = lat->scale;
    a.inv_scale = lat->inv_scale;
    a.remap = remap_blocks(lat->g, a.slab_blocks);
    a.lb_remap = lb_remap_blocks(lat->g);
    const int nev = lat->timing ? 6 : 0;
    if (lat->timing && lat->events.size() < static_cast<size_t>(nev * n_steps)) {
        while (lat->events.size() < static_cast<size_t>(nev * n_steps)) {
            hipEvent_t e;
            HIPCHK(lat, hipEventCreate(&e), "timing events");
            lat->events.push_back(e);
        }
    }
    // Steps replay from graphs in chunks of 32, 16, ..., 1 steps (the
    // largest that fits both the steps left and the steps to the next
    // health check); the same kernels with the same arguments run (the
    // particle path is driven from device memory alone), so the results are
    // the same bits as step-by-step launches.
    const bool graph_ok = !lat->timing && !lat->graph_broken && graphs_enabled();
    int64_t s = 0;
    while (s < n_steps) {
        const int64_t ci = lat->check_interval;
        int64_t room = n_steps - s;
        if (ci > 0)
            room = std::min<int64_t>(room, ci - lat->step % ci);
        int level = kGraphLevels - 1;
        while ((int64_t(1) << level) > room)
            --level;
        if (graph_ok) {
            const hipError_t e = replay_steps(lat, a, counter, level);
            if (e == hipSuccess) {
                const int len = 1 << level;
                lat->step += len;
                s += len;
                lat->cur ^= len & 1;
                if (lat->any_movable)
                    lat->mask_h_valid = false;
                if (ci > 0 && lat->step % ci == 0) {
                    double max_speed;
                    int64_t bad;
                    vlb_status st = vlb_check_health(lat, &max_speed, &bad);
                    if (st != VLB_OK)
                        return st;
                }
                continue;
            }
            // capture is not available on this stream: step by step from here on
            (void)hipGetLastError();
            lat->graph_broken = true;
        }
        set_planes(lat, a, lat->cur);
        a.step = static_cast<uint32_t>(lat->step);
        a.step_dev = nullptr;
        hipEvent_t *ev = lat->timing ? &lat->events[nev * s] : nullptr;
        bool fused = false;
        HIPCHK(lat, launch_step(lat, a, counter, fv_tile_rows(), fv_z_chunk(), ev, &fused),
               "step launch");
        lat->fused_last = fused;
        if (lat->any_movable)
            lat->mask_h_valid = false;
        lat->cur ^= 1;
        lat->step += 1;
        ++s;
        if (lat->check_interval > 0 && lat->step % lat->check_interval == 0) {
            double max_speed;
            int64_t bad;
            vlb_status st = vlb_check_health(lat, &max_speed, &bad);
            if (st != VLB_OK)
                return st;
        }
    }
    if (lat->timing && n_steps > 0) {
        HIPCHK(lat, hipStreamSynchronize(lat->stream), "timing");
        double acc[3] = {0, 0, 0};
        for (int64_t s = 0; s < n_steps; ++s) {
            hipEvent_t *ev = &lat->events[nev * s];
            for (int k = 0; k < 3; ++k) {
                float ms = 0.f;
                HIPCHK(lat, hipEventElapsedTime(&ms, ev[k], ev[k + 1]), "timing");
                acc[k] += ms;
            }
        }
        for (int k = 0; k < 3; ++k)
            lat->ktime[k] = acc[k] / static_cast<double>(n_steps);
        if (lat->fused_last || !lat->polymer)
            lat->ktime[1] = -1.0;  // no separate stress-update launch
    }
    return VLB_OK;
}

vlb_status vlb_sync(vlb_lattice *lat)
{
    if (!lat)
        return VLB_EINVAL;
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "vlb_sync");
    return VLB_OK;
}

int64_t vlb_step_count(const vlb_lattice *lat) { return lat ? lat->step : -1; }

// Body force seen by the next step, as floats for the moment readout: the
// counter-force takes the movable particles' external forces back from the
// cells that are fluid now.
vlb_status read_body_force(vlb_lattice *lat, float gv[3])
{
    double g[3] = {lat->params.body_force[0], lat->params.body_force[1],
                   lat->params.body_force[2]};
    if (lat->counter_force && lat->any_movable) {
        vlb_status st = sync_mask_host(lat);
        if (st != VLB_OK)
            return st;
        double F[3] = {0.0, 0.0, 0.0};
        bool any = false;
        for (const Particle &P : lat->parts_h) {
            if (!P.movable)
                continue;
            any = true;
            for (int a = 0; a < 3; ++a)
                F[a] += P.fext[a];
        }
        uint64_t nf = 0;
        for (uint8_t m : lat->mask_h)
            nf += m == 0;
        if (any && nf)
            for (int a = 0; a < 3; ++a)
                g[a] -= F[a] / static_cast<double>(nf);
    }
    for (int a = 0; a < 3; ++a)
        gv[a] = static_cast<float>(g[a]);
    return VLB_OK;
}

vlb_status vlb_read_density(vlb_lattice *lat, double *rho)
{
    if (!lat)
        return VLB_EINVAL;
    if (!rho)
        return fail(lat, VLB_EINVAL, "vlb_read_density: NULL output");
    float gv[3];
    vlb_status gst = read_body_force(lat, gv);
    if (gst != VLB_OK)
        return gst;
    return read_via_scratch(
        lat, static_cast<size_t>(lat->g.N) * sizeof(double), rho,
        [&](double *d) {
            return vlb::launch_read_moments(lat->storage, lat->g, lat->bound(), lat->d_mask,
                                            lat->d_f[lat->cur], lat->d_tau[lat->cur], lat->polymer,
                                            gv, lat->d_gfield, lat->inv_scale, d, nullptr,
                                            lat->stream,
                                            lat->stress_map());
        },
        "vlb_read_density");
}

vlb_status vlb_read_velocity(vlb_lattice *lat, double *u)
{
    if (!lat)
        return VLB_EINVAL;
    if (!u)
        return fail(lat, VLB_EINVAL, "vlb_read_velocity: NULL output");
    float gv[3];
    vlb_status gst = read_body_force(lat, gv);
    if (gst != VLB_OK)
        return gst;
    return read_via_scratch(
        lat, 3 * static_cast<size_t>(lat->g.N) * sizeof(double), u,
        [&](double *d) {
            return vlb::launch_read_moments(lat->storage, lat->g, lat->bound(), lat->d_mask,
                                            lat->d_f[lat->cur], lat->d_tau[lat->cur], lat->polymer,
                                            gv, lat->d_gfield, lat->inv_scale, nullptr, d,
                                            lat->stream,
                                            lat->stress_map());
        },
        "vlb_read_velocity");
}

namespace {

// Staging array of vlb_read_velocity_noalloc: the velocity of up to
// VLB_NOALLOC_MAX_CELLS cells, x, y and z planes of FP64.  Every device the
// library runs on holds its own copy until the process ends; host code
// reaches it only through the device address looked up below.
__device__ __align__(256) double scratch[3 * VLB_NOALLOC_MAX_CELLS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// Device address of `device`'s copy of the staging array, looked up on the
// first call for that device (which must be current) and kept.
hipError_t scratch_address(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch[device] = static_cast<double *>(p);
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace

vlb_status vlb_read_velocity_noalloc(vlb_lattice *lat, int64_t first, int64_t count, double *u)
{
    if (!lat)
        return VLB_EINVAL;
    if (!u)
        return fail(lat, VLB_EINVAL, "vlb_read_velocity_noalloc: NULL output");
    if (count < 1 || count > VLB_NOALLOC_MAX_CELLS)
        return fail(lat, VLB_EINVAL,
                    "vlb_read_velocity_noalloc: count must lie in 1.." +
                        std::to_string(VLB_NOALLOC_MAX_CELLS) + " (the staging array's size)");
    if (first < 0 || first > static_cast<int64_t>(lat->g.N) - count)
        return fail(lat, VLB_EINVAL, "vlb_read_velocity_noalloc: cell range beyond the lattice");
    float gv[3];
    vlb_status st = read_body_force(lat, gv);
    if (st != VLB_OK)
        return st;
    int prev = -1;
    HIPCHK(lat, hipGetDevice(&prev), "vlb_read_velocity_noalloc");
    if (prev != lat->device)
        HIPCHK(lat, hipSetDevice(lat->device), "vlb_read_velocity_noalloc");
    double *d = nullptr;
    hipError_t e = scratch_address(lat->device, &d);
    const uint32_t n0 = static_cast<uint32_t>(first), cnt = static_cast<uint32_t>(count);
    if (e == hipSuccess)
        e = vlb::launch_read_moments(lat->storage, lat->g, lat->bound(), lat->d_mask,
                                     lat->d_f[lat->cur], lat->d_tau[lat->cur], lat->polymer, gv,
                                     lat->d_gfield, lat->inv_scale, nullptr, d, lat->stream,
                                     lat->stress_map(), n0, cnt);
    for (int a = 0; a < 3 && e == hipSuccess; ++a)
        e = hipMemcpyAsync(u + static_cast<size_t>(a) * cnt, d + static_cast<size_t>(a) * cnt,
                           cnt * sizeof(double), hipMemcpyDeviceToHost, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    if (prev != lat->device)
        (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return hip_fail(lat, e, "vlb_read_velocity_noalloc");
    return VLB_OK;
}

vlb_status vlb_read_stress(vlb_lattice *lat, double *tau)
{
    if (!lat)
        return VLB_EINVAL;
    if (!tau)
        return fail(lat, VLB_EINVAL, "vlb_read_stress: NULL output");
    return read_via_scratch(
        lat, 6 * static_cast<size_t>(lat->g.N) * sizeof(double), tau,
        [&](double *d) {
            return vlb::launch_read_stress(lat->g, lat->d_mask, lat->d_tau[lat->cur], d,
                                           lat->stream, lat->stress_map());
        },
        "vlb_read_stress");
}

vlb_status vlb_read_populations(vlb_lattice *lat, double *f)
{
    if (!lat)
        return VLB_EINVAL;
    if (!f)
        return fail(lat, VLB_EINVAL, "vlb_read_populations: NULL output");
    return read_via_scratch(
        lat, static_cast<size_t>(vlb::Q) * lat->g.N * sizeof(double), f,
        [&](double *d) {
            return vlb::launch_read_populations(lat->storage, lat->g, lat->d_mask,
                                                lat->d_f[lat->cur], lat->inv_scale, d, lat->stream);
        },
        "vlb_read_populations");
}

vlb_status vlb_read_mask(vlb_lattice *lat, uint8_t *mask)
{
    if (!lat)
        return VLB_EINVAL;
    if (!mask)
        return fail(lat, VLB_EINVAL, "vlb_read_mask: NULL output");
    vlb_status st = sync_mask_host(lat);
    if (st != VLB_OK)
        return st;
    std::memcpy(mask, lat->mask_h.data(), lat->g.N);
    return VLB_OK;
}

vlb_status vlb_read_particle(vlb_lattice *lat, int32_t id, double pos[3], double vel[3],
                             double omega[3], double force[3], double torque[3])
{
    if (!lat)
        return VLB_EINVAL;
    if (id < 0 || id >= static_cast<int32_t>(lat->parts_h.size()))
        return fail(lat, VLB_ENOTFOUND, "vlb_read_particle: unknown particle id");
    const int np = static_cast<int>(lat->parts_h.size());
    if (!lat->any_movable && lat->step > 0) {
        // fixed geometry: the last step's exchange is recomputed from the
        // state it left (its output populations and its input stress)
        HIPCHK(lat, vlb::launch_particle_forces(lat->storage, lat->g, lat->d_mask,
                                                lat->d_f[lat->cur], lat->d_tau[lat->cur ^ 1],
                                                lat->polymer, lat->inv_scale, lat->d_parts, np,
                                                lat->d_pforce, lat->stream, lat->stress_map()),
               "particle forces");
    }
    std::vector<Particle> cur;
    vlb_status st = download_particles(lat, cur);
    if (st != VLB_OK)
        return st;
    const Particle &P = cur[id];
    for (int a = 0; a < 3; ++a) {
        if (pos)
            pos[a] = P.R[a];
        if (vel)
            vel[a] = P.v[a];
        if (omega)
            omega[a] = P.w[a];
        if (force)
            force[a] = lat->step > 0 ? P.ftot[a] : 0.0;
        if (torque)
            torque[a] = lat->step > 0 ? P.ttot[a] : 0.0;
    }
    return VLB_OK;
}

vlb_status vlb_read_sums(vlb_lattice *lat, double *mass, double momentum[3])
{
    if (!lat)
        return VLB_EINVAL;
    double out[8];
    vlb_status st = run_sums(lat, out);
    if (st != VLB_OK)
        return st;
    if (mass)
        *mass = out[6] + out[0];
    if (momentum)
        for (int a = 0; a < 3; ++a)
            momentum[a] = out[1 + a];
    return VLB_OK;
}

vlb_status vlb_read_wall_force(vlb_lattice *lat, double force[3])
{
    if (!lat)
        return VLB_EINVAL;
    if (!force)
        return fail(lat, VLB_EINVAL, "vlb_read_wall_force: NULL output");
    if (lat->step == 0) {
        force[0] = force[1] = force[2] = 0.0;
        return VLB_OK;
    }
    HIPCHK(lat, vlb::launch_wall_force(lat->storage, lat->g, lat->d_mask, lat->d_f[lat->cur],
                                       lat->d_tau[lat->cur ^ 1], lat->polymer, lat->inv_scale,
                                       lat->d_partials, lat->d_out, lat->stream, lat->stress_map()),
           "wall force");
    HIPCHK(lat, hipMemcpyAsync(force, lat->d_out, 3 * sizeof(double), hipMemcpyDeviceToHost,
                               lat->stream),
           "wall force");
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "wall force");
    return VLB_OK;
}

vlb_status vlb_check_health(vlb_lattice *lat, double *max_speed, int64_t *non_finite)
{
    if (!lat)
        return VLB_EINVAL;
    double out[8];
    vlb_status st = run_sums(lat, out);
    if (st != VLB_OK)
        return st;
    if (max_speed)
        *max_speed = out[4];
    if (non_finite)
        *non_finite = static_cast<int64_t>(out[5]);
    if (out[5] > 0.0 || !(out[4] <= kMaxSpeed)) {
        lat->unstable = true;
        char buf[160];
        std::snprintf(buf, sizeof buf, "unstable at step %lld: max speed %.3g, %lld non-finite cells",
                      static_cast<long long>(lat->step), out[4], static_cast<long long>(out[5]));
        return fail(lat, VLB_EUNSTABLE, buf);
    }
    return VLB_OK;
}

vlb_status vlb_set_check_interval(vlb_lattice *lat, int64_t steps)
{
    if (!lat)
        return VLB_EINVAL;
    if (steps < 0)
        return fail(lat, VLB_EINVAL, "vlb_set_check_interval: negative interval");
    lat->check_interval = steps;
    return VLB_OK;
}

// ---------------------------------------------------------------------------
// checkpoint

namespace {
constexpr uint64_t kMagic = 0x38304B434C424C56ull;  // "VLBLCK08"

struct FileHeader {
    uint64_t magic;
    int32_t nx, ny, nz, per[3];
    int32_t storage, n_walls, n_parts, polymer;
    int64_t step;
    vlb_params params;
    float scale;
    int32_t any_movable;
    int32_t rounding;  // vlb_rounding of stored values
    uint32_t seed;     // seed of the stochastic-rounding stream
    int32_t counter_force;
    int32_t extrap;
    double alpha;
    double L2;
    int32_t wall_field;   // 1: 3*N doubles of per-cell wall velocity follow the walls
    int32_t force_field;  // 1: 3*N floats of per-cell force density follow
    int32_t smooth_ns;    // overlap-fraction smoothing of conversions
    int32_t pad;

};
}  // namespace

vlb_status vlb_save(vlb_lattice *lat, const char *path)
{
    if (!lat)
        return VLB_EINVAL;
    if (!path)
        return fail(lat, VLB_EINVAL, "vlb_save: path is NULL");
    vlb_status st = sync_mask_host(lat);
    if (st != VLB_OK)
        return st;
    std::vector<Particle> parts;
    if ((st = download_particles(lat, parts)) != VLB_OK)
        return st;
    const uint64_t N = lat->g.N;
    const size_t es = storage_bytes(lat->storage);
    std::vector<char> f(vlb::Q * N * es);
    std::vector<float> tau(6 * N), tau_prev(6 * N);
    for (int i = 0; i < vlb::Q; ++i)
        HIPCHK(lat, hipMemcpyAsync(f.data() + i * N * es,
                                   static_cast<char *>(lat->d_f[lat->cur]) + i * lat->g.plane * es,
                                   N * es, hipMemcpyDeviceToHost, lat->stream),
               "vlb_save");
    for (int c = 0; c < 6; ++c) {
        HIPCHK(lat, hipMemcpyAsync(tau.data() + c * N, lat->d_tau[lat->cur] + c * lat->g.plane,
                                   N * sizeof(float), hipMemcpyDeviceToHost, lat->stream),
               "vlb_save");
        HIPCHK(lat, hipMemcpyAsync(tau_prev.data() + c * N,
                                   lat->d_tau[lat->cur ^ 1] + c * lat->g.plane, N * sizeof(float),
                                   hipMemcpyDeviceToHost, lat->stream),
               "vlb_save");
    }
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "vlb_save");
    FILE *fp = std::fopen(path, "wb");
    if (!fp)
        return fail(lat, VLB_EINVAL, std::string("vlb_save: cannot open ") + path);
    FileHeader h{};
    h.magic = kMagic;
    h.nx = lat->g.nx;
    h.ny = lat->g.ny;
    h.nz = lat->g.nz;
    for (int a = 0; a < 3; ++a)
        h.per[a] = lat->g.per[a];
    h.storage = lat->storage;
    h.n_walls = lat->n_walls;
    h.n_parts = static_cast<int32_t>(parts.size());
    h.polymer = lat->polymer;
    h.step = lat->step;
    h.params = lat->params;
    h.scale = lat->scale;
    h.any_movable = lat->any_movable;
    h.rounding = lat->rounding;
    h.seed = lat->seed;
    h.counter_force = lat->counter_force ? 1 : 0;
    h.alpha = lat->alpha;
    h.L2 = lat->L2;
    h.extrap = lat->extrap;
    h.wall_field = lat->d_wfield ? 1 : 0;
    h.force_field = lat->d_gfield ? 1 : 0;
    h.smooth_ns = lat->smooth_ns;
    bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1;
    ok = ok && std::fwrite(lat->wall_h.data(), sizeof(double), 64 * 3, fp) == 64 * 3;
    ok = ok && (!h.wall_field || std::fwrite(lat->wfield_h.data(), sizeof(double), 3 * N, fp) ==
                                     3 * N);
    ok = ok && (!h.force_field || std::fwrite(lat->gfield_h.data(), sizeof(float), 3 * N, fp) ==
                                      3 * N);
    ok = ok && (parts.empty() || std::fwrite(parts.data(), sizeof(Particle), parts.size(), fp) ==
                                     parts.size());
    ok = ok && std::fwrite(lat->mask_h.data(), 1, N, fp) == N;
    ok = ok && std::fwrite(f.data(), 1, f.size(), fp) == f.size();
    ok = ok && std::fwrite(tau.data(), sizeof(float), tau.size(), fp) == tau.size();
    ok = ok && std::fwrite(tau_prev.data(), sizeof(float), tau_prev.size(), fp) == tau_prev.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok)
        return fail(lat, VLB_EINVAL, std::string("vlb_save: write failed for ") + path);
    return VLB_OK;
}

vlb_status vlb_load(const char *path, void *stream, vlb_lattice **out)
{
    if (!path || !out)
        return fail(nullptr, VLB_EINVAL, "vlb_load: NULL argument");
    *out = nullptr;
    FILE *fp = std::fopen(path, "rb");
    if (!fp)
        return fail(nullptr, VLB_EINVAL, std::string("vlb_load: cannot open ") + path);
    FileHeader h{};
    if (std::fread(&h, sizeof h, 1, fp) != 1 || h.magic != kMagic || h.n_parts < 0 ||
        h.n_parts > vlb::MAX_PARTICLES || h.storage < VLB_STORE_F32 || h.storage > VLB_STORE_BF16 ||
        !valid_scale(h.storage, h.scale)) {
        std::fclose(fp);
        return fail(nullptr, VLB_EINVAL, "vlb_load: not a lattice checkpoint");
    }
    vlb_dims d{};
    d.nx = h.nx;
    d.ny = h.ny;
    d.nz = h.nz;
    for (int a = 0; a < 3; ++a)
        d.periodic[a] = static_cast<uint8_t>(h.per[a]);
    if (check_dims(&d) != VLB_OK) {
        std::fclose(fp);
        return fail(nullptr, VLB_EINVAL, "vlb_load: invalid dimensions");
    }
    const uint64_t N = static_cast<uint64_t>(h.nx) * h.ny * h.nz;
    const size_t es = storage_bytes(h.storage);
    std::vector<double> walls(64 * 3), wfield(h.wall_field == 1 ? 3 * N : 0);
    std::vector<float> gfield(h.force_field == 1 ? 3 * N : 0);
    std::vector<Particle> parts(h.n_parts);
    std::vector<uint8_t> mask(N);
    std::vector<char> f(vlb::Q * N * es);
    std::vector<float> tau(6 * N), tau_prev(6 * N);
    bool ok = std::fread(walls.data(), sizeof(double), walls.size(), fp) == walls.size();
    ok = ok && (wfield.empty() ||
                std::fread(wfield.data(), sizeof(double), wfield.size(), fp) == wfield.size());
    ok = ok && (gfield.empty() ||
                std::fread(gfield.data(), sizeof(float), gfield.size(), fp) == gfield.size());
    ok = ok && (parts.empty() || std::fread(parts.data(), sizeof(Particle), parts.size(), fp) ==
                                     parts.size());
    ok = ok && std::fread(mask.data(), 1, N, fp) == N;
    ok = ok && std::fread(f.data(), 1, f.size(), fp) == f.size();
    ok = ok && std::fread(tau.data(), sizeof(float), tau.size(), fp) == tau.size();
    ok = ok && std::fread(tau_prev.data(), sizeof(float), tau_prev.size(), fp) == tau_prev.size();
    std::fclose(fp);
    if (!ok)
        return fail(nullptr, VLB_EINVAL, "vlb_load: truncated checkpoint");
    // The restored records drive kernels that index the particle table by
    // mask byte and divide by mass and inertia: reject a mask byte naming a
    // particle beyond the table and records that are not finite, positive
    // spheres.
    for (uint64_t n = 0; n < N; ++n)
        if (mask[n] >= vlb::PART0 && mask[n] - vlb::PART0 >= h.n_parts)
            return fail(nullptr, VLB_EINVAL, "vlb_load: mask names a particle beyond the table");
    bool movable = false;
    for (const Particle &P : parts) {
        bool finite = std::isfinite(P.radius) && std::isfinite(P.mass) && std::isfinite(P.inertia);
        for (int a = 0; a < 3; ++a)
            finite = finite && std::isfinite(P.R[a]) && std::isfinite(P.v[a]) &&
                     std::isfinite(P.w[a]) && std::isfinite(P.fext[a]) &&
                     std::isfinite(P.text[a]) && std::isfinite(P.fconv[a]) &&
                     std::isfinite(P.tconv[a]);
        if (!finite || !(P.radius > 0.0) || !(P.mass > 0.0) || !(P.inertia > 0.0) ||
            (P.movable != 0 && P.movable != 1))
            return fail(nullptr, VLB_EINVAL, "vlb_load: invalid particle record");
        movable = movable || P.movable;
    }
    if ((h.any_movable != 0) != movable)
        return fail(nullptr, VLB_EINVAL, "vlb_load: movable flag disagrees with the particles");
    // create on a particle-free mask, then restore the saved mask verbatim
    std::vector<uint8_t> base(mask);
    for (auto &m : base)
        if (m >= vlb::PART0)
            m = 0;
    vlb_lattice *lat = nullptr;
    vlb_status st = vlb_create(&d, base.data(), walls.data(), h.n_walls,
                               static_cast<vlb_storage>(h.storage), stream, &lat);
    if (st != VLB_OK)
        return st;
    auto bail = [&](vlb_status s2) {
        g_create_error = lat->err;
        vlb_destroy(lat);
        return s2;
    };
    if ((st = vlb_set_params(lat, &h.params)) != VLB_OK)
        return bail(st);
    if (!wfield.empty() && (st = vlb_set_wall_velocity_field(lat, wfield.data())) != VLB_OK)
        return bail(st);
    if (!gfield.empty()) {
        // FP32 values widened exactly, so the device field is restored bit for bit
        std::vector<double> gd(gfield.begin(), gfield.end());
        if ((st = vlb_set_force_field(lat, gd.data())) != VLB_OK)
            return bail(st);
    }
    lat->mask_h = mask;
    lat->parts_h = parts;
    lat->any_movable = h.any_movable != 0;
    lat->step = h.step;
    lat->rounding = h.rounding == VLB_ROUND_NEAREST ? VLB_ROUND_NEAREST : VLB_ROUND_STOCHASTIC;
    lat->seed = h.seed;
    lat->counter_force = h.counter_force != 0;
    lat->alpha = (h.alpha >= 0.0 && h.alpha <= 0.5) ? h.alpha : 0.0;
    lat->L2 = (h.L2 > 3.0 && std::isfinite(h.L2)) ? h.L2 : 0.0;
    lat->extrap = (h.extrap >= 0 && h.extrap <= 2) ? h.extrap : 0;
    lat->smooth_ns = (h.smooth_ns >= 0 && h.smooth_ns <= 8) ? h.smooth_ns : 0;
    lat->scale = h.scale;
    lat->inv_scale = 1.f / h.scale;
    hipError_t e = hipMemcpyAsync(lat->d_mask, mask.data(), N, hipMemcpyHostToDevice, lat->stream);
    for (int i = 0; e == hipSuccess && i < vlb::Q; ++i)
        e = hipMemcpyAsync(static_cast<char *>(lat->d_f[lat->cur]) + i * lat->g.plane * es,
                           f.data() + i * N * es, N * es, hipMemcpyHostToDevice, lat->stream);
    for (int c = 0; e == hipSuccess && c < 6; ++c) {
        e = hipMemcpyAsync(lat->d_tau[lat->cur] + c * lat->g.plane, tau.data() + c * N,
                           N * sizeof(float), hipMemcpyHostToDevice, lat->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lat->d_tau[lat->cur ^ 1] + c * lat->g.plane, tau_prev.data() + c * N,
                               N * sizeof(float), hipMemcpyHostToDevice, lat->stream);
    }
    if (e == hipSuccess && !parts.empty())
        e = hipMemcpyAsync(lat->d_parts, parts.data(), sizeof(Particle) * parts.size(),
                           hipMemcpyHostToDevice, lat->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(lat->stream);
    if (e != hipSuccess) {
        hip_fail(lat, e, "vlb_load");
        return bail(VLB_EDEVICE);
    }
    *out = lat;
    return VLB_OK;
}

void vlb_destroy(vlb_lattice *lat)
{
    if (!lat)
        return;
    free_all(lat);
    delete lat;
}

const char *vlb_last_error(const vlb_lattice *lat)
{
    return lat ? lat->err.c_str() : g_create_error.c_str();
}

vlb_status vlb_set_giesekus(vlb_lattice *lat, double alpha)
{
    if (!lat)
        return VLB_EINVAL;
    if (!(alpha >= 0.0 && alpha <= 0.5))
        return fail(lat, VLB_EINVAL, "vlb_set_giesekus: alpha must lie in [0, 1/2]");
    lat->alpha = alpha;
    if (alpha > 0.0)
        lat->L2 = 0.0;
    return VLB_OK;
}

vlb_status vlb_set_stress_extrapolation(vlb_lattice *lat, int32_t order)
{
    if (!lat)
        return VLB_EINVAL;
    if (order < 0 || order > 2)
        return fail(lat, VLB_EINVAL, "vlb_set_stress_extrapolation: order must be 0, 1 or 2");
    lat->extrap = order;
    return VLB_OK;
}

vlb_status vlb_set_fene_p(vlb_lattice *lat, double L2)
{
    if (!lat)
        return VLB_EINVAL;
    if (!(L2 == 0.0 || (L2 > 3.0 && std::isfinite(L2))))
        return fail(lat, VLB_EINVAL, "vlb_set_fene_p: need L^2 > 3 (or 0 for off)");
    lat->L2 = L2;
    if (L2 > 0.0)
        lat->alpha = 0.0;
    return VLB_OK;
}

vlb_status vlb_set_force_field(vlb_lattice *lat, const double *F)
{
    if (!lat)
        return VLB_EINVAL;
    const uint64_t N = lat->g.N;
    if (F)
        for (uint64_t i = 0; i < 3 * N; ++i)
            if (!std::isfinite(F[i]))
                return fail(lat, VLB_EINVAL, "vlb_set_force_field: non-finite value");
    // work already queued may still read the old field
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "vlb_set_force_field");
    if (!F) {
        if (lat->d_gfield)
            HIPCHK(lat, hipFree(lat->d_gfield), "vlb_set_force_field");
        lat->d_gfield = nullptr;
        lat->gfield_h.clear();
        return VLB_OK;
    }
    if (!lat->d_gfield) {
        HIPCHK(lat, hipMalloc(&lat->d_gfield, 3 * lat->g.plane * sizeof(float)),
               "vlb_set_force_field");
        HIPCHK(lat, hipMemsetAsync(lat->d_gfield, 0, 3 * lat->g.plane * sizeof(float), lat->stream),
               "vlb_set_force_field");
    }
    lat->gfield_h.resize(3 * N);
    for (uint64_t i = 0; i < 3 * N; ++i)
        lat->gfield_h[i] = static_cast<float>(F[i]);
    for (int k = 0; k < 3; ++k)
        HIPCHK(lat,
               hipMemcpyAsync(lat->d_gfield + k * lat->g.plane, lat->gfield_h.data() + k * N,
                              N * sizeof(float), hipMemcpyHostToDevice, lat->stream),
               "vlb_set_force_field");
    return VLB_OK;
}

vlb_status vlb_set_wall_velocity_field(vlb_lattice *lat, const double *u)
{
    if (!lat)
        return VLB_EINVAL;
    const uint64_t N = lat->g.N;
    if (u)
        for (uint64_t i = 0; i < 3 * N; ++i)
            if (!std::isfinite(u[i]))
                return fail(lat, VLB_EINVAL, "vlb_set_wall_velocity_field: non-finite value");
    // work already queued may still read the old field
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "vlb_set_wall_velocity_field");
    bool moving = false;
    if (!u) {
        if (lat->d_wfield)
            HIPCHK(lat, hipFree(lat->d_wfield), "vlb_set_wall_velocity_field");
        lat->d_wfield = nullptr;
        lat->wfield_h.clear();
        for (int i = 0; i < 3 * lat->n_walls; ++i)
            moving = moving || lat->wall_h[i] != 0.0;
        lat->moving_walls = moving;
        return VLB_OK;
    }
    if (!lat->d_wfield)
        HIPCHK(lat, hipMalloc(&lat->d_wfield, 3 * N * sizeof(double)),
               "vlb_set_wall_velocity_field");
    lat->wfield_h.assign(u, u + 3 * N);
    HIPCHK(lat,
           hipMemcpyAsync(lat->d_wfield, lat->wfield_h.data(), 3 * N * sizeof(double),
                          hipMemcpyHostToDevice, lat->stream),
           "vlb_set_wall_velocity_field");
    // wall cells never change owner, so the host mask is current for them
    for (uint64_t n = 0; n < N && !moving; ++n) {
        const uint8_t m = lat->mask_h[n];
        if (m >= 1 && m <= VLB_MAX_WALL_ID)
            moving = u[n] != 0.0 || u[N + n] != 0.0 || u[2 * N + n] != 0.0;
    }
    lat->moving_walls = moving;
    return VLB_OK;
}

vlb_status vlb_set_conversion_smoothing(vlb_lattice *lat, int32_t samples)
{
    if (!lat)
        return VLB_EINVAL;
    if (samples < 0 || samples > 8)
        return fail(lat, VLB_EINVAL, "vlb_set_conversion_smoothing: samples must lie in 0..8");
    lat->smooth_ns = samples;
    return VLB_OK;
}

vlb_status vlb_set_counter_force(vlb_lattice *lat, int32_t on)
{
    if (!lat)
        return VLB_EINVAL;
    lat->counter_force = on != 0;
    return VLB_OK;
}

vlb_status vlb_set_rounding(vlb_lattice *lat, vlb_rounding mode, uint32_t seed)
{
    if (!lat)
        return VLB_EINVAL;
    if (mode != VLB_ROUND_NEAREST && mode != VLB_ROUND_STOCHASTIC)
        return fail(lat, VLB_EINVAL, "vlb_set_rounding: unknown mode");
    lat->rounding = mode;
    lat->seed = seed;
    return VLB_OK;
}

vlb_status vlb_set_raw_f32_control(vlb_lattice *lat, int32_t on)
{
    if (!lat)
        return VLB_EINVAL;
    if (on && lat->storage != vlb::ST_F32)
        return fail(lat, VLB_EINVAL, "vlb_set_raw_f32_control: FP32 storage only");
    lat->raw_f32 = on != 0;
    return VLB_OK;
}

vlb_status vlb_set_velocity_scale(vlb_lattice *lat, double u_max)
{
    if (!lat)
        return VLB_EINVAL;
    if (!(u_max > 0.0) || !std::isfinite(u_max))
        return fail(lat, VLB_EINVAL, "vlb_set_velocity_scale: u_max must be finite and positive");
    if (lat->storage != vlb::ST_F16)
        return VLB_OK;
    const float s = fp16_scale_for(u_max);
    if (s == lat->scale)
        return VLB_OK;
    // the stored state: the current population buffer (the other one is
    // rewritten whole by the next step before it is read)
    HIPCHK(lat, vlb::launch_rescale_f16(lat->d_f[lat->cur], vlb::Q * lat->g.plane, s / lat->scale,
                                        lat->stream),
           "vlb_set_velocity_scale");
    HIPCHK(lat, hipStreamSynchronize(lat->stream), "vlb_set_velocity_scale");
    lat->scale = s;
    lat->inv_scale = 1.f / s;
    return VLB_OK;
}

double vlb_storage_scale(const vlb_lattice *lat)
{
    return lat ? static_cast<double>(lat->scale) : 0.0;
}

vlb_status vlb_set_timing(vlb_lattice *lat, int32_t on)
{
    if (!lat)
        return VLB_EINVAL;
    lat->timing = on != 0;
    return VLB_OK;
}

double vlb_kernel_time_ms(const vlb_lattice *lat, int32_t which)
{
    if (!lat || which < 0 || which > 2)
        return -1.0;
    return lat->ktime[which];
}

}  // extern "C"
