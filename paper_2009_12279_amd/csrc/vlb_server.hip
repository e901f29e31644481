// Serving runtime of libvlb: continuous batching of independent solves.
//
// Requests wait in a FIFO queue.  A request is admitted when a slot is free
// and its device footprint fits the HBM budget; it then owns its buffers
// (populations, stress, velocity, mask) until it retires.  One batched launch
// advances every admitted solve by one step; K such steps (stream-collide,
// stress update and the per-solve step-counter advance) are captured in a
// hipGraph and replayed.  The graph only refers to fixed device tables, so
// admissions and retirements rewrite the tables between replays; the graph is
// captured again only when the total number of blocks changes.  A request's
// latency runs from vlb_server_submit to the moment its result is on the
// host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "vlb.h"
#include "vlb_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

constexpr uint64_t kAlign = 256;

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct Request {
    uint64_t ticket = 0;
    vlb_dims dims{};
    std::vector<uint8_t> mask;
    vlb_params params{};
    uint32_t steps = 0;
    uint32_t seed = 0;
    int state = VLB_REQ_QUEUED;
    clock_type::time_point submitted;
    double latency_ms = -1.0;
    std::vector<double> u, tau;  // results (host)
    std::string error;
};

struct Slot {
    uint64_t ticket = 0;
    vlb::Geom g{};
    uint64_t bytes = 0;
    uint8_t *mask = nullptr;
    float *f[2] = {nullptr, nullptr};
    float *tau[2] = {nullptr, nullptr};
    float *u = nullptr;
    vlb::StepArgs args[2]{};
    uint32_t target = 0;
    uint32_t nblocks = 0;
};

uint64_t footprint(const vlb_dims &d)
{
    const uint64_t N = static_cast<uint64_t>(d.nx) * d.ny * d.nz;
    const uint64_t P = round_up(N, kAlign);
    return 2 * vlb::Q * P * 4 + 2 * 6 * P * 4 + 3 * P * 4 + round_up(N, kAlign);
}

}  // namespace

struct vlb_server {
    uint64_t budget = 0;
    int max_slots = 0;
    int k_steps = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t next_ticket = 1;
    uint64_t used = 0;
    std::map<uint64_t, Request> requests;
    std::deque<uint64_t> queue;
    std::vector<Slot> slots;
    // device tables
    vlb::BatchTable *d_table = nullptr;
    vlb::BatchSolve *d_solves = nullptr;
    uint32_t *d_block_solve = nullptr;
    uint32_t *d_steps = nullptr;
    uint32_t table_capacity_blocks = 0;
    uint32_t total_blocks = 0;
    bool tables_dirty = true;
    // graph of k_steps batched steps for the current block count
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint32_t graph_blocks = 0;
    // kernel nodes whose grid follows the total block count
    std::vector<hipGraphNode_t> grid_nodes;
    std::vector<hipKernelNodeParams> grid_params;
    hipEvent_t done_event = nullptr;
    bool in_flight = false;
    int stochastic = 1;
    vlb_server_stats stats{};
    std::string err = "no error";
};

namespace {

vlb_status sfail(vlb_server *s, vlb_status st, const std::string &msg)
{
    if (s)
        s->err = msg;
    return st;
}

#define SCHK(srv, expr, what)                                                              \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return sfail((srv), e_ == hipErrorOutOfMemory ? VLB_ENOMEM : VLB_EDEVICE,      \
                         std::string(what) + ": " + hipGetErrorString(e_));                \
    } while (0)

void free_slot(Slot &sl)
{
    void *p[] = {sl.mask, sl.f[0], sl.f[1], sl.tau[0], sl.tau[1], sl.u};
    for (void *q : p)
        if (q)
            (void)hipFree(q);
    sl = Slot{};
}

bool params_ok(const vlb_params &p, double &wp, double &wm)
{
    if (!(p.eta > 0.0) || !(p.beta >= 0.0 && p.beta < 1.0))
        return false;
    if (p.beta > 0.0 && !(p.lambda_p >= 1.0))
        return false;
    const double eta_n = (1.0 - p.beta) * p.eta;
    wp = 1.0 / (3.0 * eta_n + 0.5);
    wm = wp;
    if (p.magic >= 0.0)
        wm = 1.0 / (0.5 + p.magic / (1.0 / wp - 0.5));
    return wp > 0.0 && wp < 2.0 && wm > 0.0 && wm < 2.0;
}

// fill the step arguments of a slot for both buffer parities
void make_args(vlb_server *srv, Slot &sl, const Request &rq)
{
    double wp, wm;
    params_ok(rq.params, wp, wm);
    for (int par = 0; par < 2; ++par) {
        vlb::StepArgs &a = sl.args[par];
        a = vlb::StepArgs{};
        a.g = sl.g;
        a.b.wall_vel = nullptr;
        a.b.n_walls = 0;
        a.b.parts = nullptr;
        a.b.n_parts = 0;
        a.b.moving = 0;
        a.mask = sl.mask;
        a.fin = sl.f[par];
        a.fout = sl.f[par ^ 1];
        a.tin = sl.tau[par];
        a.tout = sl.tau[par ^ 1];
        a.u = sl.u;
        for (int i = 0; i < vlb::Q; ++i) {
            a.fin_p[i] = sl.f[par] + i * sl.g.plane;
            a.fout_p[i] = sl.f[par ^ 1] + i * sl.g.plane;
        }
        for (int c = 0; c < 6; ++c) {
            a.tin_p[c] = sl.tau[par] + c * sl.g.plane;
            a.tout_p[c] = sl.tau[par ^ 1] + c * sl.g.plane;
        }
        for (int c = 0; c < 3; ++c)
            a.u_p[c] = sl.u + c * sl.g.plane;
        a.wp = wp;
        a.wm = wm;
        for (int k = 0; k < 3; ++k)
            a.g3[k] = rq.params.body_force[k];
        a.polymer = rq.params.beta > 0.0 ? 1 : 0;
        if (a.polymer) {
            a.eta_p_lam = rq.params.beta * rq.params.eta / rq.params.lambda_p;
            a.inv_lam = 1.0 / rq.params.lambda_p;
        }
        a.scale = 1.f;
        a.inv_scale = 1.f;
        a.remap = 0;
        a.stochastic = srv->stochastic;
        a.seed = rq.seed;
    }
}

vlb_status admit(vlb_server *srv, Request &rq)
{
    Slot sl;
    sl.ticket = rq.ticket;
    const uint64_t N = static_cast<uint64_t>(rq.dims.nx) * rq.dims.ny * rq.dims.nz;
    sl.g.nx = rq.dims.nx;
    sl.g.ny = rq.dims.ny;
    sl.g.nz = rq.dims.nz;
    for (int a = 0; a < 3; ++a)
        sl.g.per[a] = rq.dims.periodic[a] ? 1 : 0;
    sl.g.N = static_cast<uint32_t>(N);
    sl.g.plane = round_up(N, kAlign);
    sl.bytes = footprint(rq.dims);
    sl.target = rq.steps;
    sl.nblocks = static_cast<uint32_t>((N + vlb::BLOCK - 1) / vlb::BLOCK);
    const uint64_t P = sl.g.plane;
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess)
            e = hipMalloc(p, bytes);
    };
    alloc(reinterpret_cast<void **>(&sl.mask), round_up(N, kAlign));
    for (int b = 0; b < 2; ++b) {
        alloc(reinterpret_cast<void **>(&sl.f[b]), vlb::Q * P * 4);
        alloc(reinterpret_cast<void **>(&sl.tau[b]), 6 * P * 4);
    }
    alloc(reinterpret_cast<void **>(&sl.u), 3 * P * 4);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.mask, rq.mask.data(), N, hipMemcpyHostToDevice, srv->stream);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipMemsetAsync(sl.tau[b], 0, 6 * P * 4, srv->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(sl.f[b], 0, vlb::Q * P * 4, srv->stream);
    }
    if (e == hipSuccess)
        e = hipMemsetAsync(sl.u, 0, 3 * P * 4, srv->stream);
    if (e == hipSuccess)
        e = vlb::launch_init_equilibrium(vlb::ST_F32, sl.g, sl.mask, nullptr, sl.f[0], 1.f,
                                         srv->stream);
    if (e != hipSuccess) {
        free_slot(sl);
        return sfail(srv, e == hipErrorOutOfMemory ? VLB_ENOMEM : VLB_EDEVICE,
                     std::string("admission: ") + hipGetErrorString(e));
    }
    make_args(srv, sl, rq);
    srv->used += sl.bytes;
    srv->slots.push_back(sl);
    rq.state = VLB_REQ_RUNNING;
    rq.mask.clear();
    rq.mask.shrink_to_fit();
    srv->tables_dirty = true;
    return VLB_OK;
}

// device tables from the current slot list (steps of new solves start at 0;
// running solves keep theirs)
vlb_status rebuild_tables(vlb_server *srv, const std::vector<uint32_t> &steps)
{
    const uint32_t ns = static_cast<uint32_t>(srv->slots.size());
    std::vector<vlb::BatchSolve> solves(ns);
    std::vector<uint32_t> block_solve;
    uint32_t first = 0;
    for (uint32_t s = 0; s < ns; ++s) {
        const Slot &sl = srv->slots[s];
        solves[s].args[0] = sl.args[0];
        solves[s].args[1] = sl.args[1];
        solves[s].first_block = first;
        solves[s].nblocks = sl.nblocks;
        solves[s].target = sl.target;
        block_solve.insert(block_solve.end(), sl.nblocks, static_cast<uint32_t>(s));
        first += sl.nblocks;
    }
    srv->total_blocks = first;
    if (first > srv->table_capacity_blocks) {
        if (srv->d_block_solve)
            (void)hipFree(srv->d_block_solve);
        srv->d_block_solve = nullptr;
        const uint32_t cap = std::max<uint32_t>(first, 2 * srv->table_capacity_blocks);
        SCHK(srv, hipMalloc(&srv->d_block_solve, cap * sizeof(uint32_t)), "block table");
        srv->table_capacity_blocks = cap;
    }
    vlb::BatchTable t{};
    t.n_solves = ns;
    t.total_blocks = first;
    t.solves = srv->d_solves;
    t.block_solve = srv->d_block_solve;
    t.steps = srv->d_steps;
    if (ns)
        SCHK(srv, hipMemcpyAsync(srv->d_solves, solves.data(), ns * sizeof(vlb::BatchSolve),
                                 hipMemcpyHostToDevice, srv->stream),
             "solve table");
    if (first)
        SCHK(srv, hipMemcpyAsync(srv->d_block_solve, block_solve.data(), first * sizeof(uint32_t),
                                 hipMemcpyHostToDevice, srv->stream),
             "block table");
    if (ns)
        SCHK(srv, hipMemcpyAsync(srv->d_steps, steps.data(), ns * sizeof(uint32_t),
                                 hipMemcpyHostToDevice, srv->stream),
             "step table");
    SCHK(srv, hipMemcpyAsync(srv->d_table, &t, sizeof t, hipMemcpyHostToDevice, srv->stream),
         "table");
    SCHK(srv, hipStreamSynchronize(srv->stream), "tables");
    srv->tables_dirty = false;
    return VLB_OK;
}

vlb_status ensure_graph(vlb_server *srv)
{
    if (srv->graph_exec && srv->graph_blocks == srv->total_blocks)
        return VLB_OK;
    if (srv->graph_exec) {
        // same work with a different grid: update the batched kernel nodes in
        // place rather than capturing and instantiating again
        bool ok = true;
        for (size_t k = 0; k < srv->grid_nodes.size() && ok; ++k) {
            hipKernelNodeParams p = srv->grid_params[k];
            p.gridDim.x = srv->total_blocks;
            ok = hipGraphExecKernelNodeSetParams(srv->graph_exec, srv->grid_nodes[k], &p) ==
                 hipSuccess;
            if (ok)
                srv->grid_params[k] = p;
        }
        if (ok) {
            srv->graph_blocks = srv->total_blocks;
            srv->stats.graph_updates += 1;
            return VLB_OK;
        }
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(srv->graph_exec);
        (void)hipGraphDestroy(srv->graph);
        srv->graph_exec = nullptr;
        srv->graph = nullptr;
    }
    SCHK(srv, hipStreamBeginCapture(srv->stream, hipStreamCaptureModeThreadLocal), "capture");
    hipError_t e = vlb::launch_batch_step(srv->d_table, srv->total_blocks, srv->stochastic,
                                          srv->k_steps, srv->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(srv->stream, &g);
    SCHK(srv, e, "capture launch");
    SCHK(srv, e2, "end capture");
    srv->graph = g;
    SCHK(srv, hipGraphInstantiate(&srv->graph_exec, g, nullptr, nullptr, 0), "instantiate");
    // remember the per-cell kernel nodes (block size BLOCK; the counter
    // advance runs with a different block size)
    size_t count = 0;
    SCHK(srv, hipGraphGetNodes(g, nullptr, &count), "graph nodes");
    std::vector<hipGraphNode_t> nodes(count);
    SCHK(srv, hipGraphGetNodes(g, nodes.data(), &count), "graph nodes");
    srv->grid_nodes.clear();
    srv->grid_params.clear();
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        SCHK(srv, hipGraphNodeGetType(nd, &ty), "graph node type");
        if (ty != hipGraphNodeTypeKernel)
            continue;
        hipKernelNodeParams p{};
        SCHK(srv, hipGraphKernelNodeGetParams(nd, &p), "graph node params");
        if (p.blockDim.x == static_cast<unsigned>(vlb::BLOCK)) {
            srv->grid_nodes.push_back(nd);
            srv->grid_params.push_back(p);
        }
    }
    srv->graph_blocks = srv->total_blocks;
    srv->stats.graph_captures += 1;
    return VLB_OK;
}

// results of a finished slot: velocity (moments of the final state) and stress
vlb_status collect(vlb_server *srv, Slot &sl, Request &rq)
{
    const uint64_t N = sl.g.N;
    const int par = static_cast<int>(sl.target & 1u);
    double *d = nullptr;
    SCHK(srv, hipMalloc(&d, 9 * N * sizeof(double)), "result buffer");
    const float gv[3] = {static_cast<float>(rq.params.body_force[0]),
                         static_cast<float>(rq.params.body_force[1]),
                         static_cast<float>(rq.params.body_force[2])};
    vlb::Bound b{};
    hipError_t e = vlb::launch_read_moments(vlb::ST_F32, sl.g, b, sl.mask, sl.f[par], sl.tau[par],
                                            rq.params.beta > 0.0, gv, 1.f, nullptr, d, srv->stream);
    if (e == hipSuccess)
        e = vlb::launch_read_stress(sl.g, sl.mask, sl.tau[par], d + 3 * N, srv->stream);
    rq.u.resize(3 * N);
    rq.tau.resize(6 * N);
    if (e == hipSuccess)
        e = hipMemcpyAsync(rq.u.data(), d, 3 * N * sizeof(double), hipMemcpyDeviceToHost, srv->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(rq.tau.data(), d + 3 * N, 6 * N * sizeof(double), hipMemcpyDeviceToHost,
                           srv->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(srv->stream);
    (void)hipFree(d);
    SCHK(srv, e, "result readout");
    rq.latency_ms =
        std::chrono::duration<double, std::milli>(clock_type::now() - rq.submitted).count();
    rq.state = VLB_REQ_DONE;
    srv->stats.completed += 1;
    return VLB_OK;
}

}  // namespace

extern "C" {

vlb_status vlb_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t steps_per_launch,
                             void *stream, vlb_server **out)
{
    if (!out)
        return VLB_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > 4096 || steps_per_launch < 1 || steps_per_launch > 4096)
        return VLB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return VLB_EDEVICE;
    vlb_server *srv = new vlb_server();
    srv->budget = hbm_budget_bytes;
    srv->max_slots = max_slots;
    srv->k_steps = steps_per_launch;
    hipError_t e = hipSuccess;
    if (stream) {
        srv->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreate(&srv->stream);
        srv->own_stream = true;
    }
    if (e == hipSuccess)
        e = hipMalloc(&srv->d_table, sizeof(vlb::BatchTable));
    if (e == hipSuccess)
        e = hipMalloc(&srv->d_solves, max_slots * sizeof(vlb::BatchSolve));
    if (e == hipSuccess)
        e = hipMalloc(&srv->d_steps, max_slots * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&srv->done_event, hipEventDisableTiming);
    if (e != hipSuccess) {
        vlb_server_destroy(srv);
        return e == hipErrorOutOfMemory ? VLB_ENOMEM : VLB_EDEVICE;
    }
    *out = srv;
    return VLB_OK;
}

size_t vlb_server_request_bytes(const vlb_dims *dims)
{
    if (!dims || dims->nx < 1 || dims->ny < 1 || dims->nz < 1)
        return 0;
    return static_cast<size_t>(footprint(*dims));
}

vlb_status vlb_server_set_rounding(vlb_server *srv, vlb_rounding mode)
{
    if (!srv || (mode != VLB_ROUND_NEAREST && mode != VLB_ROUND_STOCHASTIC))
        return VLB_EINVAL;
    if (!srv->slots.empty() || !srv->queue.empty())
        return sfail(srv, VLB_ESTATE, "vlb_server_set_rounding: server is not idle");
    srv->stochastic = mode == VLB_ROUND_STOCHASTIC;
    return VLB_OK;
}

vlb_status vlb_server_submit(vlb_server *srv, const vlb_request *req, uint64_t *ticket)
{
    if (!srv || !req || !ticket)
        return VLB_EINVAL;
    const vlb_dims &d = req->dims;
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || !req->mask || req->n_steps < 0 ||
        req->n_steps > 0xffffffffll)
        return sfail(srv, VLB_EINVAL, "vlb_server_submit: invalid dimensions, mask or steps");
    const uint64_t N = static_cast<uint64_t>(d.nx) * d.ny * d.nz;
    if (N + kAlign >= (1ull << 30))
        return sfail(srv, VLB_EINVAL, "vlb_server_submit: lattice too large");
    double wp, wm;
    if (!params_ok(req->params, wp, wm))
        return sfail(srv, VLB_EINVAL, "vlb_server_submit: invalid parameters");
    if (footprint(d) > srv->budget)
        return sfail(srv, VLB_EBUSY, "vlb_server_submit: request exceeds the memory budget");
    Request rq;
    rq.ticket = srv->next_ticket++;
    rq.dims = d;
    rq.mask.assign(req->mask, req->mask + N);
    for (uint64_t n = 0; n < N; ++n)
        if (rq.mask[n] >= vlb::PART0)
            return sfail(srv, VLB_EINVAL, "vlb_server_submit: mask values >= 64 are reserved");
    // solid end layers on non-periodic axes
    const int n3[3] = {d.nx, d.ny, d.nz};
    for (int ax = 0; ax < 3; ++ax) {
        if (d.periodic[ax])
            continue;
        for (int z = 0; z < d.nz; ++z)
            for (int y = 0; y < d.ny; ++y)
                for (int x = 0; x < d.nx; ++x) {
                    const int c[3] = {x, y, z};
                    if ((c[ax] == 0 || c[ax] == n3[ax] - 1) &&
                        rq.mask[x + static_cast<size_t>(d.nx) * (y + static_cast<size_t>(d.ny) * z)] == 0)
                        return sfail(srv, VLB_EINVAL,
                                     "vlb_server_submit: non-periodic axis without solid end layers");
                }
    }
    // fixed spheres become solid cells at rest
    for (int k = 0; k < req->n_spheres; ++k) {
        const double *sp = req->spheres + 4 * k;
        for (int z = 0; z < d.nz; ++z)
            for (int y = 0; y < d.ny; ++y)
                for (int x = 0; x < d.nx; ++x) {
                    const int c[3] = {x, y, z};
                    double dd[3];
                    for (int a = 0; a < 3; ++a) {
                        dd[a] = static_cast<double>(c[a]) - sp[a];
                        if (d.periodic[a]) {
                            const double L = static_cast<double>(n3[a]);
                            dd[a] -= L * std::floor(dd[a] / L + 0.5);
                        }
                    }
                    double d2;
                    {
#pragma clang fp contract(off)
                        d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
                    }
                    if (d2 < sp[3] * sp[3])
                        rq.mask[x + static_cast<size_t>(d.nx) * (y + static_cast<size_t>(d.ny) * z)] = 1;
                }
    }
    rq.params = req->params;
    rq.steps = static_cast<uint32_t>(req->n_steps);
    rq.seed = req->seed;
    rq.submitted = clock_type::now();
    *ticket = rq.ticket;
    srv->queue.push_back(rq.ticket);
    srv->requests.emplace(rq.ticket, std::move(rq));
    srv->stats.submitted += 1;
    return VLB_OK;
}

vlb_status vlb_server_pump(vlb_server *srv, int32_t wait)
{
    if (!srv)
        return VLB_EINVAL;
    if (srv->in_flight) {
        if (wait) {
            SCHK(srv, hipEventSynchronize(srv->done_event), "pump wait");
        } else {
            const hipError_t q = hipEventQuery(srv->done_event);
            if (q == hipErrorNotReady)
                return VLB_OK;
            SCHK(srv, q, "pump query");
        }
        srv->in_flight = false;
    }
    // step counters of the running solves
    const uint32_t ns = static_cast<uint32_t>(srv->slots.size());
    std::vector<uint32_t> steps(ns, 0);
    if (ns) {
        SCHK(srv, hipMemcpyAsync(steps.data(), srv->d_steps, ns * sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, srv->stream),
             "step readback");
        SCHK(srv, hipStreamSynchronize(srv->stream), "step readback");
    }
    // retire finished (or cancelled) solves
    std::vector<Slot> keep;
    std::vector<uint32_t> keep_steps;
    bool changed = false;
    for (uint32_t s = 0; s < ns; ++s) {
        Slot &sl = srv->slots[s];
        Request &rq = srv->requests[sl.ticket];
        if (rq.state == VLB_REQ_CANCELLED || steps[s] >= sl.target) {
            if (rq.state != VLB_REQ_CANCELLED) {
                vlb_status st = collect(srv, sl, rq);
                if (st != VLB_OK) {
                    rq.state = VLB_REQ_FAILED;
                    rq.error = srv->err;
                }
            }
            srv->used -= sl.bytes;
            free_slot(sl);
            changed = true;
        } else {
            keep.push_back(sl);
            keep_steps.push_back(steps[s]);
        }
    }
    srv->slots.swap(keep);
    // admit from the queue while slots and memory allow (FIFO, no overtaking)
    while (!srv->queue.empty() && static_cast<int>(srv->slots.size()) < srv->max_slots) {
        Request &rq = srv->requests[srv->queue.front()];
        if (rq.state == VLB_REQ_CANCELLED) {
            srv->queue.pop_front();
            continue;
        }
        if (srv->used + footprint(rq.dims) > srv->budget)
            break;
        vlb_status st = admit(srv, rq);
        if (st != VLB_OK) {
            if (st == VLB_ENOMEM && !srv->slots.empty())
                break;  // try again once memory frees up
            rq.state = VLB_REQ_FAILED;
            rq.error = srv->err;
            srv->queue.pop_front();
            continue;
        }
        srv->queue.pop_front();
        keep_steps.push_back(0);
        changed = true;
        if (rq.steps == 0) {
            // nothing to advance: retire at the next round
        }
    }
    if (changed || srv->tables_dirty) {
        vlb_status st = rebuild_tables(srv, keep_steps);
        if (st != VLB_OK)
            return st;
    }
    srv->stats.running = static_cast<int64_t>(srv->slots.size());
    srv->stats.queued = static_cast<int64_t>(srv->queue.size());
    srv->stats.bytes_in_use = srv->used;
    if (srv->slots.empty())
        return VLB_OK;
    vlb_status st = ensure_graph(srv);
    if (st != VLB_OK)
        return st;
    SCHK(srv, hipGraphLaunch(srv->graph_exec, srv->stream), "graph launch");
    SCHK(srv, hipEventRecord(srv->done_event, srv->stream), "event");
    srv->in_flight = true;
    srv->stats.launches += 1;
    uint64_t cells = 0;
    for (size_t s = 0; s < srv->slots.size(); ++s)
        cells += srv->slots[s].g.N;
    srv->stats.cell_steps_launched += cells * static_cast<uint64_t>(srv->k_steps);
    return VLB_OK;
}

vlb_status vlb_server_poll(vlb_server *srv, uint64_t ticket, int32_t *state)
{
    if (!srv || !state)
        return VLB_EINVAL;
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end())
        return sfail(srv, VLB_ENOTFOUND, "vlb_server_poll: unknown ticket");
    *state = it->second.state;
    return VLB_OK;
}

vlb_status vlb_server_result(vlb_server *srv, uint64_t ticket, double *u, double *tau,
                             double *latency_ms)
{
    if (!srv)
        return VLB_EINVAL;
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end())
        return sfail(srv, VLB_ENOTFOUND, "vlb_server_result: unknown ticket");
    Request &rq = it->second;
    if (rq.state == VLB_REQ_FAILED)
        return sfail(srv, VLB_EDEVICE, "vlb_server_result: request failed: " + rq.error);
    if (rq.state != VLB_REQ_DONE)
        return sfail(srv, VLB_ESTATE, "vlb_server_result: request not finished");
    if (u)
        std::memcpy(u, rq.u.data(), rq.u.size() * sizeof(double));
    if (tau)
        std::memcpy(tau, rq.tau.data(), rq.tau.size() * sizeof(double));
    if (latency_ms)
        *latency_ms = rq.latency_ms;
    srv->requests.erase(it);
    return VLB_OK;
}

vlb_status vlb_server_cancel(vlb_server *srv, uint64_t ticket)
{
    if (!srv)
        return VLB_EINVAL;
    auto it = srv->requests.find(ticket);
    if (it == srv->requests.end())
        return sfail(srv, VLB_ENOTFOUND, "vlb_server_cancel: unknown ticket");
    Request &rq = it->second;
    if (rq.state == VLB_REQ_DONE || rq.state == VLB_REQ_FAILED)
        return sfail(srv, VLB_ESTATE, "vlb_server_cancel: request already finished");
    rq.state = VLB_REQ_CANCELLED;
    return VLB_OK;
}

vlb_status vlb_server_stats_get(vlb_server *srv, vlb_server_stats *out)
{
    if (!srv || !out)
        return VLB_EINVAL;
    *out = srv->stats;
    return VLB_OK;
}

const char *vlb_server_last_error(const vlb_server *srv) { return srv ? srv->err.c_str() : "no server"; }

void vlb_server_destroy(vlb_server *srv)
{
    if (!srv)
        return;
    if (srv->stream)
        (void)hipStreamSynchronize(srv->stream);
    for (Slot &sl : srv->slots)
        free_slot(sl);
    if (srv->graph_exec)
        (void)hipGraphExecDestroy(srv->graph_exec);
    if (srv->graph)
        (void)hipGraphDestroy(srv->graph);
    void *p[] = {srv->d_table, srv->d_solves, srv->d_block_solve, srv->d_steps};
    for (void *q : p)
        if (q)
            (void)hipFree(q);
    if (srv->done_event)
        (void)hipEventDestroy(srv->done_event);
    if (srv->own_stream && srv->stream)
        (void)hipStreamDestroy(srv->stream);
    delete srv;
}

}  // extern "C"
