// Serving runtime of libvlb: continuous batching of independent solves.
//
// Requests wait in a queue (FIFO, or shortest first).  A request is admitted
// when a slot is free and its device footprint fits in the server's arena, one
// device allocation of the whole HBM budget made at creation; the solve then
// owns its range of the arena (populations, stress, velocity, mask, wall table)
// until it retires.  One batched launch advances every admitted solve by one
// step; K such steps (stream-collide, stress update and the per-solve
// step-counter advance) are captured in a hipGraph and replayed.  The graph
// only refers to fixed device tables, which are rewritten in stream order
// between replays.
//
// Scheduling keeps the GPU fed: up to two replays are in flight, and the host
// retires finished solves (results read on a second stream), admits new ones
// (uploads and initialisation on that stream) and rewrites the tables while
// the earlier replay runs.  Every admitted solve advances by exactly K steps
// per replay until its target, so the host knows from the count of completed
// replays which solves have finished, without reading the device.  A retired
// solve's arena range is reused only after every replay issued while it was
// in the tables has completed.  A request's latency runs from
// vlb_server_submit to the moment its result is on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
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
    double alpha = 0.0;  // Giesekus mobility (0: Oldroyd-B)
    std::vector<double> walls;  // n_walls x 3 wall velocities
    uint32_t steps = 0;
    uint32_t seed = 0;
    int state = VLB_REQ_QUEUED;
    clock_type::time_point submitted;
    double latency_ms = -1.0;
    std::unique_ptr<double[]> result;  // host: u (3 N) then tau (6 N)
    uint64_t result_n = 0;             // N of the result
    std::string error;
};

struct Slot {
    uint64_t ticket = 0;
    uint32_t id = 0;                    // index in the device solve and step tables
    vlb::Geom g{};
    uint64_t offset = 0, bytes = 0;     // range of the arena
    uint8_t *mask = nullptr;
    float *f[2] = {nullptr, nullptr};
    float *tau[2] = {nullptr, nullptr};
    float *u = nullptr;
    double *walls = nullptr;            // 63 x 3 wall velocities (device)
    vlb::StepArgs args[2]{};
    uint32_t target = 0;
    uint32_t nblocks = 0;
    bool fv_tiled = false;              // stress update in tiles, else per cell
    uint32_t fv_nblocks = 0, fv_zc = 0;
    uint64_t last_launch = 0;           // the replay that takes it to its target
};

// arena range of a retired solve, reusable once `free_after` replays have
// completed (replays issued while it was in the tables may still touch it)
struct Quarantined {
    uint64_t offset, bytes, free_after;
};

// wall-velocity table of a solve: ids 1..63, three doubles each
constexpr uint64_t kWallBytes = 64 * 3 * sizeof(double);

uint64_t footprint(const vlb_dims &d)
{
    const uint64_t N = static_cast<uint64_t>(d.nx) * d.ny * d.nz;
    const uint64_t P = round_up(N, kAlign);
    return 2 * vlb::Q * P * 4 + 2 * 6 * P * 4 + 3 * P * 4 + round_up(N, kAlign) + kWallBytes;
}

}  // namespace

struct vlb_server {
    uint64_t budget = 0;
    int max_slots = 0;
    int k_steps = 1;
    hipStream_t stream = nullptr;   // replays and table updates
    bool own_stream = false;
    hipStream_t io = nullptr;       // admissions and result reads
    hipStream_t cap = nullptr;      // graph capture only
    uint64_t next_ticket = 1;
    uint64_t used = 0;
    std::map<uint64_t, Request> requests;
    std::deque<uint64_t> queue;
    std::vector<Slot> slots;        // admitted solves
    std::vector<uint32_t> free_ids;
    std::vector<uint32_t> new_ids;  // admitted since the last table update
    // arena: one allocation of the budget, handed out in ranges
    char *arena = nullptr;
    std::map<uint64_t, uint64_t> free_ranges;  // offset -> bytes
    std::vector<Quarantined> quarantine;
    // device tables (solves and step counters indexed by slot id) and their
    // pinned staging
    vlb::BatchTable *d_table = nullptr;
    vlb::BatchSolve *d_solves = nullptr;
    uint32_t *d_block_solve = nullptr;
    uint32_t *d_steps = nullptr;
    uint32_t table_capacity_blocks = 0;  // of the block-to-solve array (both kernels)
    vlb::BatchTable *h_table = nullptr;
    vlb::BatchSolve *h_solves = nullptr;
    uint32_t *h_block_solve = nullptr;
    uint32_t *h_zero = nullptr;
    hipEvent_t tables_copied = nullptr;
    uint32_t total_blocks = 0;
    uint32_t fv_total_blocks = 0;
    bool tables_dirty = false;
    bool admitted_since_launch = false;
    hipEvent_t io_done = nullptr;
    // device result buffer (doubles), grown in stream order on io
    double *d_result = nullptr;
    uint64_t d_result_cap = 0;
    // two graph executables, used by alternate replays, so that one can be
    // updated while the other is in flight
    struct GraphSet {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint32_t blocks = 0, fv_blocks = 0;
        // kernel nodes whose grid is the block count: stream-collide (fv
        // false) and stress update (fv true)
        std::vector<hipGraphNode_t> nodes;
        std::vector<hipKernelNodeParams> params;
        std::vector<bool> fv;
    } graphs[2];
    hipEvent_t launch_done[2] = {nullptr, nullptr};
    uint64_t n_launched = 0, n_completed = 0;
    int stochastic = 1;
    int policy = VLB_POLICY_FIFO;
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

// ---- arena ----------------------------------------------------------------

bool arena_alloc(vlb_server *srv, uint64_t bytes, uint64_t &offset)
{
    for (auto it = srv->free_ranges.begin(); it != srv->free_ranges.end(); ++it) {
        if (it->second < bytes)
            continue;
        offset = it->first;
        const uint64_t rest = it->second - bytes;
        srv->free_ranges.erase(it);
        if (rest)
            srv->free_ranges.emplace(offset + bytes, rest);
        return true;
    }
    return false;
}

void arena_release(vlb_server *srv, uint64_t offset, uint64_t bytes)
{
    auto next = srv->free_ranges.lower_bound(offset);
    if (next != srv->free_ranges.end() && offset + bytes == next->first) {
        bytes += next->second;
        next = srv->free_ranges.erase(next);
    }
    if (next != srv->free_ranges.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == offset) {
            prev->second += bytes;
            return;
        }
    }
    srv->free_ranges.emplace(offset, bytes);
}

void release_quarantine(vlb_server *srv)
{
    std::vector<Quarantined> keep;
    for (const Quarantined &q : srv->quarantine) {
        if (q.free_after <= srv->n_completed)
            arena_release(srv, q.offset, q.bytes);
        else
            keep.push_back(q);
    }
    srv->quarantine.swap(keep);
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
        bool walls_move = false;
        for (double v : rq.walls)
            walls_move = walls_move || v != 0.0;
        a.b.wall_vel = sl.walls;
        a.b.n_walls = static_cast<int32_t>(rq.walls.size() / 3);
        a.b.parts = nullptr;
        a.b.n_parts = 0;
        a.b.moving = walls_move ? 1 : 0;
        a.b.walls_move = walls_move ? 1 : 0;
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
            a.gk = static_cast<float>(rq.alpha / (rq.params.beta * rq.params.eta));
        }
        a.scale = 1.f;
        a.inv_scale = 1.f;
        a.remap = 0;
        a.lb_remap = 0;
        a.stochastic = srv->stochastic;
        a.seed = rq.seed;
    }
}

// Admit a request into an arena range: uploads and initialisation run on the
// io stream (the next replay waits for them).  `no_room` when no range is
// free yet (the request waits for retirements).
vlb_status admit(vlb_server *srv, Request &rq, bool &no_room)
{
    const uint64_t bytes = footprint(rq.dims);
    uint64_t offset = 0;
    no_room = srv->free_ids.empty() || !arena_alloc(srv, bytes, offset);
    if (no_room)
        return VLB_OK;
    Slot sl;
    sl.ticket = rq.ticket;
    sl.id = srv->free_ids.back();
    srv->free_ids.pop_back();
    const uint64_t N = static_cast<uint64_t>(rq.dims.nx) * rq.dims.ny * rq.dims.nz;
    sl.g.nx = rq.dims.nx;
    sl.g.ny = rq.dims.ny;
    sl.g.nz = rq.dims.nz;
    for (int a = 0; a < 3; ++a)
        sl.g.per[a] = rq.dims.periodic[a] ? 1 : 0;
    sl.g.N = static_cast<uint32_t>(N);
    sl.g.plane = round_up(N, kAlign);
    vlb::set_divisors(sl.g);
    sl.offset = offset;
    sl.bytes = bytes;
    sl.target = rq.steps;
    sl.nblocks = static_cast<uint32_t>((N + vlb::BLOCK - 1) / vlb::BLOCK);
    sl.fv_nblocks = vlb::batch_fv_blocks(sl.g, &sl.fv_tiled, &sl.fv_zc);
    const uint64_t P = sl.g.plane;
    char *base = srv->arena + offset;
    sl.f[0] = reinterpret_cast<float *>(base);
    sl.f[1] = sl.f[0] + vlb::Q * P;
    sl.tau[0] = sl.f[1] + vlb::Q * P;
    sl.tau[1] = sl.tau[0] + 6 * P;
    sl.u = sl.tau[1] + 6 * P;
    sl.mask = reinterpret_cast<uint8_t *>(sl.u + 3 * P);
    sl.walls = reinterpret_cast<double *>(sl.mask + round_up(N, kAlign));
    const uint64_t K = static_cast<uint64_t>(srv->k_steps);
    sl.last_launch = srv->n_launched + (sl.target + K - 1) / K - 1;  // unused for target 0
    hipError_t e = hipMemcpyAsync(sl.mask, rq.mask.data(), N, hipMemcpyHostToDevice, srv->io);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipMemsetAsync(sl.tau[b], 0, 6 * P * 4, srv->io);
        if (e == hipSuccess)
            e = hipMemsetAsync(sl.f[b], 0, vlb::Q * P * 4, srv->io);
    }
    if (e == hipSuccess)
        e = hipMemsetAsync(sl.u, 0, 3 * P * 4, srv->io);
    if (e == hipSuccess)
        e = hipMemsetAsync(sl.walls, 0, kWallBytes, srv->io);
    if (e == hipSuccess && !rq.walls.empty())
        e = hipMemcpyAsync(sl.walls, rq.walls.data(), rq.walls.size() * sizeof(double),
                           hipMemcpyHostToDevice, srv->io);
    if (e == hipSuccess)
        e = vlb::launch_init_equilibrium(vlb::ST_F32, sl.g, sl.mask, nullptr, sl.f[0], 1.f, srv->io);
    if (e != hipSuccess) {
        arena_release(srv, offset, bytes);
        srv->free_ids.push_back(sl.id);
        return sfail(srv, VLB_EDEVICE, std::string("admission: ") + hipGetErrorString(e));
    }
    make_args(srv, sl, rq);
    srv->used += sl.bytes;
    srv->new_ids.push_back(sl.id);
    srv->slots.push_back(sl);
    rq.state = VLB_REQ_RUNNING;
    srv->tables_dirty = true;
    srv->admitted_since_launch = true;
    return VLB_OK;
}

// Rewrite the device tables from the slot list, in stream order behind the
// replays already issued: solve entries by slot id (free ids get a zero
// target, so the counter advance leaves them alone), the block-to-solve map
// and zeroed step counters for newly admitted solves.
vlb_status rebuild_tables(vlb_server *srv)
{
    SCHK(srv, hipEventSynchronize(srv->tables_copied), "table staging");
    uint32_t n_ids = 0, total = 0, fv_total = 0;
    for (const Slot &sl : srv->slots) {
        n_ids = std::max(n_ids, sl.id + 1);
        total += sl.nblocks;
        fv_total += sl.fv_nblocks;
    }
    // one array: the stream-collide blocks' solves, then the stress update's
    if (total + fv_total > srv->table_capacity_blocks) {
        const uint32_t cap =
            std::max<uint32_t>(total + fv_total, 2 * srv->table_capacity_blocks);
        if (srv->d_block_solve)
            (void)hipFree(srv->d_block_solve);  // waits for the replays that use it
        if (srv->h_block_solve)
            (void)hipHostFree(srv->h_block_solve);
        srv->d_block_solve = nullptr;
        srv->h_block_solve = nullptr;
        srv->table_capacity_blocks = 0;
        SCHK(srv, hipMalloc(&srv->d_block_solve, cap * sizeof(uint32_t)), "block table");
        SCHK(srv, hipHostMalloc(&srv->h_block_solve, cap * sizeof(uint32_t)), "block table");
        srv->table_capacity_blocks = cap;
    }
    std::memset(srv->h_solves, 0, n_ids * sizeof(vlb::BatchSolve));
    uint32_t first = 0, fv_first = 0;
    for (const Slot &sl : srv->slots) {
        vlb::BatchSolve &bs = srv->h_solves[sl.id];
        bs.args[0] = sl.args[0];
        bs.args[1] = sl.args[1];
        bs.first_block = first;
        bs.nblocks = sl.nblocks;
        bs.target = sl.target;
        bs.fv_tiled = sl.fv_tiled ? 1u : 0u;
        bs.fv_first_block = fv_first;
        bs.fv_nblocks = sl.fv_nblocks;
        bs.fv_zc = sl.fv_zc;
        for (uint32_t k = 0; k < sl.nblocks; ++k)
            srv->h_block_solve[first + k] = sl.id;
        for (uint32_t k = 0; k < sl.fv_nblocks; ++k)
            srv->h_block_solve[total + fv_first + k] = sl.id;
        first += sl.nblocks;
        fv_first += sl.fv_nblocks;
    }
    srv->total_blocks = total;
    srv->fv_total_blocks = fv_total;
    vlb::BatchTable &t = *srv->h_table;
    t.n_solves = n_ids;
    t.total_blocks = total;
    t.solves = srv->d_solves;
    t.block_solve = srv->d_block_solve;
    t.steps = srv->d_steps;
    t.fv_total_blocks = fv_total;
    t.fv_block_solve = srv->d_block_solve + total;
    for (uint32_t id : srv->new_ids)
        SCHK(srv, hipMemcpyAsync(srv->d_steps + id, srv->h_zero, sizeof(uint32_t),
                                 hipMemcpyHostToDevice, srv->stream),
             "step reset");
    srv->new_ids.clear();
    if (n_ids)
        SCHK(srv, hipMemcpyAsync(srv->d_solves, srv->h_solves, n_ids * sizeof(vlb::BatchSolve),
                                 hipMemcpyHostToDevice, srv->stream),
             "solve table");
    if (total + fv_total)
        SCHK(srv, hipMemcpyAsync(srv->d_block_solve, srv->h_block_solve,
                                 (total + fv_total) * sizeof(uint32_t), hipMemcpyHostToDevice,
                                 srv->stream),
             "block table");
    SCHK(srv, hipMemcpyAsync(srv->d_table, srv->h_table, sizeof(vlb::BatchTable),
                             hipMemcpyHostToDevice, srv->stream),
         "table");
    SCHK(srv, hipEventRecord(srv->tables_copied, srv->stream), "table event");
    srv->tables_dirty = false;
    return VLB_OK;
}

void drop_graph(vlb_server::GraphSet &gs)
{
    if (gs.exec)
        (void)hipGraphExecDestroy(gs.exec);
    if (gs.graph)
        (void)hipGraphDestroy(gs.graph);
    gs = vlb_server::GraphSet{};
}

// Graph of K batched steps for the current block count.  The set is not in
// flight (its previous replay has completed), so its grid can be updated in
// place rather than captured again.
vlb_status ensure_graph(vlb_server *srv, vlb_server::GraphSet &gs)
{
    if (gs.exec && gs.blocks == srv->total_blocks && gs.fv_blocks == srv->fv_total_blocks)
        return VLB_OK;
    if (gs.exec) {
        bool ok = true;
        for (size_t k = 0; k < gs.nodes.size() && ok; ++k) {
            hipKernelNodeParams p = gs.params[k];
            p.gridDim.x = gs.fv[k] ? srv->fv_total_blocks : srv->total_blocks;
            ok = hipGraphExecKernelNodeSetParams(gs.exec, gs.nodes[k], &p) == hipSuccess;
            if (ok)
                gs.params[k] = p;
        }
        if (ok) {
            gs.blocks = srv->total_blocks;
            gs.fv_blocks = srv->fv_total_blocks;
            srv->stats.graph_updates += 1;
            return VLB_OK;
        }
        (void)hipGetLastError();
        drop_graph(gs);
    }
    SCHK(srv, hipStreamBeginCapture(srv->cap, hipStreamCaptureModeThreadLocal), "capture");
    hipError_t e = vlb::launch_batch_step(srv->d_table, srv->total_blocks, srv->fv_total_blocks,
                                          srv->stochastic, srv->k_steps, srv->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(srv->cap, &g);
    SCHK(srv, e, "capture launch");
    SCHK(srv, e2, "end capture");
    gs.graph = g;
    SCHK(srv, hipGraphInstantiate(&gs.exec, g, nullptr, nullptr, 0), "instantiate");
    // remember the nodes whose grid follows the block counts: stream-collide
    // (BLOCK x 1 threads) and the stress update (64 x 4); the counter advance
    // runs with a block of its own size
    size_t count = 0;
    SCHK(srv, hipGraphGetNodes(g, nullptr, &count), "graph nodes");
    std::vector<hipGraphNode_t> nodes(count);
    SCHK(srv, hipGraphGetNodes(g, nodes.data(), &count), "graph nodes");
    gs.nodes.clear();
    gs.params.clear();
    gs.fv.clear();
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        SCHK(srv, hipGraphNodeGetType(nd, &ty), "graph node type");
        if (ty != hipGraphNodeTypeKernel)
            continue;
        hipKernelNodeParams p{};
        SCHK(srv, hipGraphKernelNodeGetParams(nd, &p), "graph node params");
        const bool lb = p.blockDim.x == static_cast<unsigned>(vlb::BLOCK) && p.blockDim.y == 1;
        const bool fv = p.blockDim.x == 64u && p.blockDim.y == 4u;
        if (lb || fv) {
            gs.nodes.push_back(nd);
            gs.params.push_back(p);
            gs.fv.push_back(fv);
        }
    }
    gs.blocks = srv->total_blocks;
    gs.fv_blocks = srv->fv_total_blocks;
    srv->stats.graph_captures += 1;
    return VLB_OK;
}

// Results of finished solves (their last replay has completed): velocity from
// the moments of the final state and the stress.  collect_issue enqueues the
// readout kernels on the io stream and returns at once: that must happen
// before any admission can take the solves' arena ranges (a later reuse is
// stream-ordered after the readout).  collect_finish copies the results into
// each request's own host array; it runs after the next replays are issued,
// so the copies overlap GPU work.  The device result buffer grows with
// stream-ordered allocation on io: a plain free would wait for the replays
// in flight.
hipError_t collect_issue(vlb_server *srv, const std::vector<Slot> &done)
{
    uint64_t total = 0;
    for (const Slot &sl : done)
        total += 9ull * sl.g.N;
    if (total == 0)
        return hipSuccess;
    hipError_t e = hipSuccess;
    if (total > srv->d_result_cap) {
        const uint64_t cap = std::max<uint64_t>(total, 2 * srv->d_result_cap);
        if (srv->d_result)
            (void)hipFreeAsync(srv->d_result, srv->io);
        srv->d_result = nullptr;
        srv->d_result_cap = 0;
        if ((e = hipMallocAsync(reinterpret_cast<void **>(&srv->d_result), cap * sizeof(double),
                                srv->io)) != hipSuccess)
            return e;
        srv->d_result_cap = cap;
    }
    uint64_t off = 0;
    for (const Slot &sl : done) {
        const Request &rq = srv->requests[sl.ticket];
        const uint64_t N = sl.g.N;
        const int par = static_cast<int>(sl.target & 1u);
        const float gv[3] = {static_cast<float>(rq.params.body_force[0]),
                             static_cast<float>(rq.params.body_force[1]),
                             static_cast<float>(rq.params.body_force[2])};
        vlb::Bound b{};
        double *d = srv->d_result + off;
        if (e == hipSuccess)
            e = vlb::launch_read_moments(vlb::ST_F32, sl.g, b, sl.mask, sl.f[par], sl.tau[par],
                                         rq.params.beta > 0.0, gv, nullptr, 1.f, nullptr, d,
                                         srv->io);
        if (e == hipSuccess)
            e = vlb::launch_read_stress(sl.g, sl.mask, sl.tau[par], d + 3 * N, srv->io);
        off += 9 * N;
    }
    return e;
}

// e: the status of the matching collect_issue.
vlb_status collect_finish(vlb_server *srv, const std::vector<Slot> &done, hipError_t e)
{
    if (done.empty())
        return VLB_OK;
    uint64_t off = 0;
    for (const Slot &sl : done) {
        Request &rq = srv->requests[sl.ticket];
        const uint64_t N = sl.g.N;
        if (e == hipSuccess) {
            rq.result.reset(new (std::nothrow) double[9 * N]);
            if (!rq.result)
                e = hipErrorOutOfMemory;
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(rq.result.get(), srv->d_result + off, 9 * N * sizeof(double),
                               hipMemcpyDeviceToHost, srv->io);
        off += 9 * N;
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(srv->io);
    const auto now = clock_type::now();
    for (const Slot &sl : done) {
        Request &rq = srv->requests[sl.ticket];
        if (e == hipSuccess) {
            rq.result_n = sl.g.N;
            rq.latency_ms = std::chrono::duration<double, std::milli>(now - rq.submitted).count();
            rq.state = VLB_REQ_DONE;
            srv->stats.completed += 1;
        } else {
            rq.result.reset();
            rq.state = VLB_REQ_FAILED;
            rq.error = std::string("result readout: ") + hipGetErrorString(e);
        }
        rq.mask.clear();
        rq.mask.shrink_to_fit();
    }
    SCHK(srv, e, "result readout");
    return VLB_OK;
}

// Retire solves: the arena range waits in quarantine until every replay
// issued so far has completed.
void retire(vlb_server *srv, const Slot &sl)
{
    srv->quarantine.push_back(Quarantined{sl.offset, sl.bytes, srv->n_launched});
    srv->used -= sl.bytes;
    srv->free_ids.push_back(sl.id);
    srv->tables_dirty = true;
}

// Mark completed replays done; with `block`, wait for the oldest one.
vlb_status reap(vlb_server *srv, bool block)
{
    while (srv->n_completed < srv->n_launched) {
        hipEvent_t ev = srv->launch_done[srv->n_completed & 1u];
        const hipError_t q = hipEventQuery(ev);
        if (q == hipErrorNotReady) {
            if (!block)
                break;
            SCHK(srv, hipEventSynchronize(ev), "replay wait");
            block = false;
        } else {
            SCHK(srv, q, "replay query");
        }
        srv->n_completed += 1;
    }
    return VLB_OK;
}

// The queue entry admitted next: the front (FIFO), or the one with the
// fewest cell-steps (shortest first, the earliest of equal ones).  Cancelled
// entries are dropped on the way.
std::deque<uint64_t>::iterator next_in_queue(vlb_server *srv)
{
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        if (srv->requests[*it].state == VLB_REQ_CANCELLED)
            it = srv->queue.erase(it);
        else
            ++it;
    }
    if (srv->policy != VLB_POLICY_SHORTEST_FIRST || srv->queue.empty())
        return srv->queue.begin();
    auto work = [&](uint64_t t) {
        const Request &rq = srv->requests[t];
        return static_cast<uint64_t>(rq.dims.nx) * rq.dims.ny * rq.dims.nz * rq.steps;
    };
    auto best = srv->queue.begin();
    for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it)
        if (work(*it) < work(*best))
            best = it;
    return best;
}

// Admit queued requests while slots and memory allow (in the policy's order,
// no overtaking of the request next in that order) and keep up to two
// replays in flight.  Admitted requests of zero steps are moved to zero_step.
vlb_status admit_and_launch(vlb_server *srv, std::vector<Slot> &zero_step)
{
    vlb_status st = VLB_OK;
    while (static_cast<int>(srv->slots.size()) < srv->max_slots) {
        const auto next = next_in_queue(srv);
        if (next == srv->queue.end())
            break;
        Request &rq = srv->requests[*next];
        if (srv->used + footprint(rq.dims) > srv->budget)
            break;
        bool no_room = false;
        st = admit(srv, rq, no_room);
        if (no_room)
            break;  // no free range yet: wait for retirements
        srv->queue.erase(next);
        if (st != VLB_OK) {
            rq.state = VLB_REQ_FAILED;
            rq.error = srv->err;
            continue;
        }
        if (rq.steps == 0) {
            // nothing to advance: the result is the initial state
            zero_step.push_back(srv->slots.back());
            srv->slots.pop_back();
            srv->new_ids.pop_back();
        }
    }
    srv->stats.running = static_cast<int64_t>(srv->slots.size());
    srv->stats.queued = static_cast<int64_t>(srv->queue.size());
    srv->stats.bytes_in_use = srv->used;
    // keep up to two replays in flight while some solve still has steps that
    // no replay has been issued for
    while (srv->n_launched - srv->n_completed < 2) {
        uint64_t cells = 0;
        for (const Slot &sl : srv->slots)
            if (sl.last_launch >= srv->n_launched)
                cells += sl.g.N;
        if (cells == 0)
            break;
        if (srv->tables_dirty && (st = rebuild_tables(srv)) != VLB_OK)
            return st;
        if (srv->admitted_since_launch) {
            SCHK(srv, hipEventRecord(srv->io_done, srv->io), "admission event");
            SCHK(srv, hipStreamWaitEvent(srv->stream, srv->io_done, 0), "admission wait");
            srv->admitted_since_launch = false;
        }
        // this set's previous replay (two back) has completed
        const uint32_t which = static_cast<uint32_t>(srv->n_launched & 1u);
        vlb_server::GraphSet &gs = srv->graphs[which];
        if ((st = ensure_graph(srv, gs)) != VLB_OK)
            return st;
        SCHK(srv, hipGraphLaunch(gs.exec, srv->stream), "graph launch");
        SCHK(srv, hipEventRecord(srv->launch_done[which], srv->stream), "event");
        srv->n_launched += 1;
        srv->stats.launches += 1;
        srv->stats.cell_steps_launched += cells * static_cast<uint64_t>(srv->k_steps);
    }
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
    if (max_slots < 1 || max_slots > 4096 || steps_per_launch < 1 || steps_per_launch > 4096 ||
        hbm_budget_bytes < kAlign)
        return VLB_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return VLB_EDEVICE;
    vlb_server *srv = new vlb_server();
    srv->budget = hbm_budget_bytes / kAlign * kAlign;
    srv->max_slots = max_slots;
    srv->k_steps = steps_per_launch;
    for (int id = max_slots - 1; id >= 0; --id)
        srv->free_ids.push_back(static_cast<uint32_t>(id));
    hipError_t e = hipSuccess;
    if (stream) {
        srv->stream = static_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreate(&srv->stream);
        srv->own_stream = true;
    }
    if (e == hipSuccess)
        e = hipStreamCreate(&srv->io);
    if (e == hipSuccess)
        e = hipStreamCreate(&srv->cap);
    if (e == hipSuccess)
        e = hipMalloc(&srv->arena, srv->budget);
    if (e == hipSuccess)
        srv->free_ranges.emplace(0, srv->budget);
    if (e == hipSuccess)
        e = hipMalloc(&srv->d_table, sizeof(vlb::BatchTable));
    if (e == hipSuccess)
        e = hipMalloc(&srv->d_solves, max_slots * sizeof(vlb::BatchSolve));
    if (e == hipSuccess)
        e = hipMalloc(&srv->d_steps, max_slots * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipHostMalloc(&srv->h_table, sizeof(vlb::BatchTable));
    if (e == hipSuccess)
        e = hipHostMalloc(&srv->h_solves, max_slots * sizeof(vlb::BatchSolve));
    if (e == hipSuccess)
        e = hipHostMalloc(&srv->h_zero, sizeof(uint32_t));
    if (e == hipSuccess)
        *srv->h_zero = 0;
    for (hipEvent_t *ev : {&srv->launch_done[0], &srv->launch_done[1], &srv->tables_copied,
                           &srv->io_done})
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventRecord(srv->tables_copied, srv->stream);
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

vlb_status vlb_server_set_policy(vlb_server *srv, vlb_policy policy)
{
    if (!srv || (policy != VLB_POLICY_FIFO && policy != VLB_POLICY_SHORTEST_FIRST))
        return VLB_EINVAL;
    srv->policy = policy;
    return VLB_OK;
}

vlb_status vlb_server_set_rounding(vlb_server *srv, vlb_rounding mode)
{
    if (!srv || (mode != VLB_ROUND_NEAREST && mode != VLB_ROUND_STOCHASTIC))
        return VLB_EINVAL;
    if (!srv->slots.empty() || !srv->queue.empty())
        return sfail(srv, VLB_ESTATE, "vlb_server_set_rounding: server is not idle");
    const int st = mode == VLB_ROUND_STOCHASTIC;
    if (st != srv->stochastic) {
        // the rounding mode is baked into the captured kernels
        (void)hipStreamSynchronize(srv->stream);
        drop_graph(srv->graphs[0]);
        drop_graph(srv->graphs[1]);
    }
    srv->stochastic = st;
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
    if (!(req->giesekus_alpha >= 0.0 && req->giesekus_alpha <= 0.5))
        return sfail(srv, VLB_EINVAL, "vlb_server_submit: Giesekus alpha must lie in [0, 1/2]");
    if (req->n_walls < 0 || req->n_walls > 63 || (req->n_walls > 0 && !req->wall_velocity))
        return sfail(srv, VLB_EINVAL, "vlb_server_submit: n_walls must lie in 0..63 with velocities");
    for (int i = 0; i < 3 * req->n_walls; ++i)
        if (!std::isfinite(req->wall_velocity[i]))
            return sfail(srv, VLB_EINVAL, "vlb_server_submit: non-finite wall velocity");
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
    auto at = [&](int x, int y, int z) -> uint8_t & {
        return rq.mask[x + static_cast<size_t>(d.nx) * (y + static_cast<size_t>(d.ny) * z)];
    };
    for (int ax = 0; ax < 3; ++ax) {
        if (d.periodic[ax])
            continue;
        const int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
        for (int side = 0; side < 2; ++side)
            for (int j2 = 0; j2 < n3[a2]; ++j2)
                for (int j1 = 0; j1 < n3[a1]; ++j1) {
                    int c[3];
                    c[ax] = side ? n3[ax] - 1 : 0;
                    c[a1] = j1;
                    c[a2] = j2;
                    if (at(c[0], c[1], c[2]) == 0)
                        return sfail(srv, VLB_EINVAL,
                                     "vlb_server_submit: non-periodic axis without solid end layers");
                }
    }
    // fixed spheres become solid cells at rest: |x - c|^2 < r^2 over the
    // sphere's bounding box (wrapped on periodic axes, clipped otherwise)
    for (int k = 0; k < req->n_spheres; ++k) {
        const double *sp = req->spheres + 4 * k;
        if (!(sp[3] > 0.0) || !std::isfinite(sp[3]) || !std::isfinite(sp[0]) ||
            !std::isfinite(sp[1]) || !std::isfinite(sp[2]))
            return sfail(srv, VLB_EINVAL, "vlb_server_submit: invalid sphere");
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = static_cast<int>(std::floor(sp[a] - sp[3])) - 1;
            hi[a] = static_cast<int>(std::ceil(sp[a] + sp[3])) + 1;
            if (!d.periodic[a] || hi[a] - lo[a] + 1 >= n3[a]) {
                // clipped (or the box covers the whole periodic axis: scan it once)
                if (d.periodic[a]) {
                    lo[a] = 0;
                    hi[a] = n3[a] - 1;
                } else {
                    lo[a] = std::max(lo[a], 0);
                    hi[a] = std::min(hi[a], n3[a] - 1);
                }
            }
        }
        for (int zz = lo[2]; zz <= hi[2]; ++zz)
            for (int yy = lo[1]; yy <= hi[1]; ++yy)
                for (int xx = lo[0]; xx <= hi[0]; ++xx) {
                    const int raw[3] = {xx, yy, zz};
                    int c[3];
                    double dd[3];
                    for (int a = 0; a < 3; ++a) {
                        c[a] = ((raw[a] % n3[a]) + n3[a]) % n3[a];
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
                        at(c[0], c[1], c[2]) = 1;
                }
    }
    rq.params = req->params;
    rq.alpha = req->giesekus_alpha;
    if (req->n_walls > 0)
        rq.walls.assign(req->wall_velocity, req->wall_velocity + 3 * req->n_walls);
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
    const uint64_t completed_before = srv->n_completed;
    vlb_status st = reap(srv, false);
    if (st != VLB_OK)
        return st;
    if (wait && srv->n_completed == completed_before && srv->n_launched > srv->n_completed) {
        if ((st = reap(srv, true)) != VLB_OK)
            return st;
    } else if (srv->n_launched - srv->n_completed >= 2) {
        return VLB_OK;
    }
    release_quarantine(srv);
    // retire solves whose last replay has completed, and cancelled ones
    std::vector<Slot> keep, done, dropped;
    for (Slot &sl : srv->slots) {
        const Request &rq = srv->requests[sl.ticket];
        if (rq.state == VLB_REQ_CANCELLED)
            dropped.push_back(sl);
        else if (sl.last_launch < srv->n_completed)
            done.push_back(sl);
        else
            keep.push_back(sl);
    }
    srv->slots.swap(keep);
    // the readout of finished solves is issued now, before any admission can
    // take their ranges, and finished after the next replays are issued, so
    // that the host's copies overlap GPU work
    const hipError_t issued = collect_issue(srv, done);
    for (const Slot &sl : done)
        retire(srv, sl);
    for (const Slot &sl : dropped) {
        Request &rq = srv->requests[sl.ticket];
        rq.mask.clear();
        rq.mask.shrink_to_fit();
        retire(srv, sl);
    }
    if (issued != hipSuccess)
        return collect_finish(srv, done, issued);
    release_quarantine(srv);
    std::vector<Slot> zero_step;
    const vlb_status lst = admit_and_launch(srv, zero_step);
    const vlb_status cst = collect_finish(srv, done, hipSuccess);
    vlb_status zst = VLB_OK;
    if (!zero_step.empty()) {
        zst = collect_finish(srv, zero_step, collect_issue(srv, zero_step));
        for (const Slot &sl : zero_step)
            retire(srv, sl);
    }
    return lst != VLB_OK ? lst : cst != VLB_OK ? cst : zst;
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
    const uint64_t N = rq.result_n;
    if (u)
        std::memcpy(u, rq.result.get(), 3 * N * sizeof(double));
    if (tau)
        std::memcpy(tau, rq.result.get() + 3 * N, 6 * N * sizeof(double));
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
    if (srv->io) {
        if (srv->d_result)
            (void)hipFreeAsync(srv->d_result, srv->io);
        srv->d_result = nullptr;
        (void)hipStreamSynchronize(srv->io);
    }
    drop_graph(srv->graphs[0]);
    drop_graph(srv->graphs[1]);
    void *p[] = {srv->arena, srv->d_table, srv->d_solves, srv->d_block_solve, srv->d_steps};
    for (void *q : p)
        if (q)
            (void)hipFree(q);
    void *h[] = {srv->h_table, srv->h_solves, srv->h_block_solve, srv->h_zero};
    for (void *q : h)
        if (q)
            (void)hipHostFree(q);
    for (hipEvent_t ev : {srv->launch_done[0], srv->launch_done[1], srv->tables_copied,
                          srv->io_done})
        if (ev)
            (void)hipEventDestroy(ev);
    if (srv->io)
        (void)hipStreamDestroy(srv->io);
    if (srv->cap)
        (void)hipStreamDestroy(srv->cap);
    if (srv->own_stream && srv->stream)
        (void)hipStreamDestroy(srv->stream);
    delete srv;
}

}  // extern "C"
