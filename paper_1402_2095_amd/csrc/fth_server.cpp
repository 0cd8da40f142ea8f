// Serving layer: many FTH solves of different size and sparsity sharing one
// GPU, run concurrently in chunks (continuous batching).
//
// Each running request is advanced in chunks of at most steps_per_tick
// steps, issued on a stream of its own and timed with HIP events:
//   - a request that is not packed runs its context's own step schedule
//     (graphs of its step kernels, dense GEMM + epilogue, blocked kernels);
//   - sparse FP32 requests with the same ns form a packed group: one
//     persistent kernel per step walks a device list of (request, row tile |
//     pair tile) entries of all members, captured as a graph per chunk
//     length, on the group's stream.
// Chunks never cross a request's check boundary (multiples of
// steps_per_tick steps), where its estimates and block stderrs are read and
// it may retire; they are cut to a divisor of steps_per_tick when the
// previous chunk's time says they would exceed the quantum.  The tick loop
// issues a chunk to every idle request and group and then waits for the
// first chunk that ends, so admission does not wait for the slowest request.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "fth_ctx.hpp"

using namespace fth::host;

namespace {

constexpr int kPackedGrid = 2048;  // persistent workgroups (multiple of 8: one slice per XCD)
constexpr double kDefaultQuantumMs = 20.0;

struct SrvRequest {
    uint64_t id = 0;
    // deep copies of the inputs
    fth_matrix M{};
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val, dense, A, C;
    fth_gle gle{};
    double dt = 0;
    std::vector<int32_t> pairs;
    fth_options opt{};
    double target = 0;
    int64_t max_steps = 0;
    int32_t unscale_target = -1;
    bool momentum = false;            // report the <p p> block (acc_pp) instead of <q q>
    std::vector<double> kind_weight;  // 1 for a pair (i, i), else 0 (for fth_unscale)
    std::vector<int64_t> di, dj;      // output index of (i,i) and (j,j) for each pair, or -1
    // run state
    fth_ctx* ctx = nullptr;
    bool packable = false;
    int group = -1;  // ns of its packed group, or -1
    bool inflight = false;  // an unpacked chunk is on the context's stream
    bool waiting = false;   // idle at a check boundary until its packed group reaches one
    int64_t chunk_K = 0;
    double step_ms = 0.0;   // device time per step of the last chunk
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    fth_request_info info{};
    std::vector<double> est, se;
};

struct Group {
    int ns = 0;
    std::vector<SrvRequest*> members;
    fth::StepArgs<float>* d_table = nullptr;
    fth::PackedTile* d_tiles = nullptr;
    int32_t* d_counts = nullptr;  // [0]: tiles, [1]: slots (read by the graph's kernels)
    int cap_slots = 0;
    int64_t cap_tiles = 0;
    std::map<int64_t, hipGraphExec_t> graphs;  // by chunk length
    bool dirty = true;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool inflight = false;
    int64_t chunk_K = 0;
    int64_t phase = 0;      // steps of the members since their last check boundary
    double step_ms = 0.0;

    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
};

bool packable(const SrvRequest& r) {
    return r.M.format == FTH_CSR && r.opt.precision == FTH_FP32 && r.opt.replicas % 4 == 0 && r.opt.replicas >= 4 &&
           r.opt.replicas <= 256 && r.gle.ns <= fth::kNsMax;
}

}  // namespace

struct fth_server {
    fth_server_options opt{};
    std::chrono::steady_clock::time_point t0;
    int device = 0;
    uint64_t next_id = 1;
    std::map<uint64_t, std::unique_ptr<SrvRequest>> all;
    std::deque<SrvRequest*> queue;
    std::vector<SrvRequest*> running;
    size_t reserved = 0;
    std::map<int, Group> groups;
    hipEvent_t ev_ref = nullptr;  // device-clock origin (recorded at creation)

    double clock() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    ~fth_server() {
        for (auto& kv : groups)
            if (kv.second.stream) (void)hipStreamSynchronize(kv.second.stream);
        for (SrvRequest* r : running) {
            fth_destroy(r->ctx);  // waits for its stream
            if (r->ev0) (void)hipEventDestroy(r->ev0);
            if (r->ev1) (void)hipEventDestroy(r->ev1);
        }
        for (auto& kv : groups) {
            Group& g = kv.second;
            g.drop_graphs();
            (void)hipFree(g.d_table);
            (void)hipFree(g.d_tiles);
            (void)hipFree(g.d_counts);
            if (g.ev0) (void)hipEventDestroy(g.ev0);
            if (g.ev1) (void)hipEventDestroy(g.ev1);
            if (g.stream) (void)hipStreamDestroy(g.stream);
        }
        if (ev_ref) (void)hipEventDestroy(ev_ref);
    }
};

namespace {

// Chunk length: up to the next check boundary, cut to the largest divisor of
// the check interval whose predicted device time fits the quantum.  Before
// a step time is known (first chunk) a short probe chunk of at most 1/16 of
// the interval is taken.
int64_t chunk_len(const fth_server* s, int64_t phase, double step_ms) {
    const int64_t interval = s->opt.steps_per_tick;
    const int64_t rem = interval - phase;
    int64_t K = rem;
    if (s->opt.quantum_ms > 0 && (step_ms <= 0 || double(K) * step_ms > s->opt.quantum_ms)) {
        int64_t best = 1;
        for (int64_t d = 1; d <= interval; ++d) {
            if (interval % d != 0) continue;
            const bool fits = step_ms > 0 ? double(d) * step_ms <= s->opt.quantum_ms : 16 * d <= interval;
            if (fits) best = d;
        }
        K = std::min(rem, best);
    }
    return std::max<int64_t>(K, 1);
}

fth_status group_upload(fth_server* s, Group& g) {
    (void)s;
    const int nslots = int(g.members.size());
    std::vector<fth::StepArgs<float>> table(size_t(std::max(nslots, 1)));
    std::vector<fth::PackedTile> tiles;
    for (int k = 0; k < nslots; ++k) {
        fth_ctx* c = g.members[k]->ctx;
        table[k] = step_args<float>(c);
        const int per_block = c->block / (c->R / c->rpt);
        const int64_t rt = (c->n + per_block - 1) / per_block;
        for (int64_t t = 0; t < rt; ++t) tiles.push_back(fth::PackedTile{k, 0, t});
    }
    for (int k = 0; k < nslots; ++k) {  // pair tiles after all row tiles
        fth_ctx* c = g.members[k]->ctx;
        const int per_block = c->block / (c->R / c->rpt);
        const int64_t pt = (c->npairs + per_block - 1) / per_block;
        for (int64_t t = 0; t < pt; ++t) tiles.push_back(fth::PackedTile{k, 1, t});
    }
    if (int64_t(tiles.size()) > 0x7FFFFFFF) return fail(FTH_EUNSUPPORTED, "too many tiles in one packed group");
    bool realloc = false;
    if (nslots > g.cap_slots) {
        (void)hipFree(g.d_table);
        g.d_table = nullptr;
        g.cap_slots = std::max(2 * g.cap_slots, std::max(nslots, 8));
        HIP_OK(hipMalloc(&g.d_table, sizeof(fth::StepArgs<float>) * size_t(g.cap_slots)));
        realloc = true;
    }
    if (int64_t(tiles.size()) > g.cap_tiles) {
        (void)hipFree(g.d_tiles);
        g.d_tiles = nullptr;
        g.cap_tiles = std::max<int64_t>(2 * g.cap_tiles, std::max<int64_t>(int64_t(tiles.size()), 1024));
        HIP_OK(hipMalloc(&g.d_tiles, sizeof(fth::PackedTile) * size_t(g.cap_tiles)));
        realloc = true;
    }
    if (!g.d_counts) {
        HIP_OK(hipMalloc(&g.d_counts, 2 * sizeof(int32_t)));
        realloc = true;
    }
    const int32_t counts[2] = {int32_t(tiles.size()), nslots};
    HIP_OK(hipMemcpyAsync(g.d_table, table.data(), sizeof(fth::StepArgs<float>) * size_t(nslots),
                          hipMemcpyHostToDevice, g.stream));
    if (!tiles.empty())
        HIP_OK(hipMemcpyAsync(g.d_tiles, tiles.data(), sizeof(fth::PackedTile) * tiles.size(), hipMemcpyHostToDevice,
                              g.stream));
    HIP_OK(hipMemcpyAsync(g.d_counts, counts, sizeof(counts), hipMemcpyHostToDevice, g.stream));
    HIP_OK(hipStreamSynchronize(g.stream));  // the host vectors die here
    if (realloc) g.drop_graphs();            // the graphs bake the buffer addresses
    g.dirty = false;
    return FTH_OK;
}

// Graph of K packed steps plus the advance of every member's step counter.
fth_status group_graph(Group& g, int64_t K, hipGraphExec_t* out) {
    auto it = g.graphs.find(K);
    if (it != g.graphs.end()) {
        *out = it->second;
        return FTH_OK;
    }
    HIP_OK(hipStreamBeginCapture(g.stream, hipStreamCaptureModeRelaxed));
    int rc = 0;
    for (int64_t k = 0; k < K && rc == 0; ++k)
        rc = fth::launch_packed_csr(g.d_table, g.d_tiles, g.d_counts, g.ns, false, kPackedGrid, int(k), g.stream);
    if (rc == 0) rc = fth::launch_advance_all(g.d_table, g.d_counts + 1, K, g.stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g.stream, &graph);
    if (rc != 0) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(FTH_EDEVICE, "packed kernel launch failed (%d)", rc);
    }
    if (e != hipSuccess) return fail(FTH_EDEVICE, "packed graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(FTH_EDEVICE, "packed graph instantiate failed: %s", hipGetErrorString(e));
    g.graphs[K] = ex;
    *out = ex;
    return FTH_OK;
}

// The estimates a request reports: its pairs, from the <q q> block or, for a
// momentum-form request, the <p p> block that follows it.
fth_status read_reported(const SrvRequest* r, std::vector<double>& est, std::vector<double>& se, int64_t* nacc) {
    const int64_t no = fth_num_outputs(r->ctx);
    const int64_t np = r->info.n_out;
    std::vector<double> e(static_cast<size_t>(no)), v(static_cast<size_t>(no));
    fth_status st = fth_read(r->ctx, e.data(), v.data(), no, nacc);
    if (st != FTH_OK) return st;
    const int64_t off = r->momentum ? np : 0;
    if (off + np > no) return fail(FTH_ESTATE, "request has fewer outputs than it reports");
    est.assign(e.begin() + off, e.begin() + off + np);
    se.assign(v.begin() + off, v.begin() + off + np);
    return FTH_OK;
}

// Retire a request: read its results, release its context and memory.
void finish(fth_server* s, SrvRequest* r, int32_t state, fth_status st) {
    if (r->ctx) {
        r->est.assign(size_t(r->info.n_out), 0.0);
        r->se.assign(size_t(r->info.n_out), 0.0);
        if (state == FTH_REQ_DONE) (void)read_reported(r, r->est, r->se, nullptr);
        fth_destroy(r->ctx);  // waits for its stream
        r->ctx = nullptr;
        s->reserved -= r->info.footprint;
    }
    if (r->ev0) (void)hipEventDestroy(r->ev0);
    if (r->ev1) (void)hipEventDestroy(r->ev1);
    r->ev0 = r->ev1 = nullptr;
    r->inflight = false;
    if (r->group >= 0) {
        Group& g = s->groups[r->group];
        g.members.erase(std::remove(g.members.begin(), g.members.end(), r), g.members.end());
        g.dirty = true;
        r->group = -1;
    }
    s->running.erase(std::remove(s->running.begin(), s->running.end(), r), s->running.end());
    r->info.state = state;
    r->info.status = st;
    r->info.t_finish = s->clock();
}

fth_status admit(fth_server* s, SrvRequest* r) {
    fth_ctx* c = nullptr;
    fth_status st = fth_create(&r->M, &r->gle, r->dt, r->pairs.empty() ? nullptr : r->pairs.data(),
                               int64_t(r->pairs.size() / 2), &r->opt, &c);
    if (st != FTH_OK) return st;
    r->ctx = c;
    if (hipEventCreate(&r->ev0) != hipSuccess || hipEventCreate(&r->ev1) != hipSuccess) {
        fth_destroy(c);
        r->ctx = nullptr;
        return fail(FTH_EDEVICE, "event creation failed");
    }
    s->reserved += r->info.footprint;
    r->info.t_start = s->clock();
    r->info.state = FTH_REQ_RUNNING;
    // the packed kernel runs 256-thread workgroups with 4 replicas per thread
    r->packable = packable(*r) && c->rpt == 4 && c->block == 256;
    s->running.push_back(r);
    return FTH_OK;
}

// max over estimates of stderr / scale; +inf until min_blocks blocks exist
double max_rel_stderr(const SrvRequest& r, const std::vector<double>& est, const std::vector<double>& se,
                      int64_t nblocks, int min_blocks) {
    if (nblocks < min_blocks) return std::numeric_limits<double>::infinity();
    double worst = 0.0;
    for (size_t k = 0; k < est.size(); ++k) {
        double scale = std::fabs(est[k]);
        if (k < r.di.size() && r.di[k] >= 0 && r.dj[k] >= 0) {
            const double g = est[size_t(r.di[k])] * est[size_t(r.dj[k])];
            if (g > 0) scale = std::sqrt(g);
        }
        const double rel = scale > 0 ? se[k] / scale : std::numeric_limits<double>::infinity();
        worst = std::max(worst, rel);
    }
    return worst;
}

// At a check boundary: read the stderr summary and retire at the target or cap.
void check(fth_server* s, SrvRequest* r) {
    std::vector<double> est, se;
    int64_t nacc = 0;
    fth_status st = read_reported(r, est, se, &nacc);
    if (st != FTH_OK) {
        finish(s, r, FTH_REQ_FAILED, st);
        return;
    }
    r->info.nblocks = nacc / r->opt.block_len;
    r->info.max_rel_stderr = max_rel_stderr(*r, est, se, r->info.nblocks, s->opt.min_blocks);
    const bool reached = r->info.max_rel_stderr <= r->target;
    const bool capped = r->max_steps > 0 && r->info.steps >= r->max_steps;
    if (reached || capped) finish(s, r, FTH_REQ_DONE, FTH_OK);
}

double event_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? double(ms) : 0.0;
}

// Device-clock span of a finished chunk (ms since the server's origin event).
void note_span(const fth_server* s, fth_request_info& info, hipEvent_t e0, hipEvent_t e1) {
    const double a = event_ms(s->ev_ref, e0), b = event_ms(s->ev_ref, e1);
    if (info.device_first_ms < 0) info.device_first_ms = a;
    info.device_last_ms = b;
}

// Completion of an unpacked chunk whose end event has fired.
void complete_unpacked(fth_server* s, SrvRequest* r) {
    const int64_t K = r->chunk_K;
    r->inflight = false;
    const double ms = event_ms(r->ev0, r->ev1);
    fth_status st = run_complete(r->ctx, K);
    r->info.steps += K;
    r->info.chunks += 1;
    r->info.device_ms += ms;
    note_span(s, r->info, r->ev0, r->ev1);
    r->step_ms = ms / double(K);
    if (st != FTH_OK) {
        finish(s, r, FTH_REQ_FAILED, st);
        return;
    }
    if (r->info.steps % s->opt.steps_per_tick == 0) check(s, r);
}

// Completion of a packed chunk: every member advanced by K steps.
void complete_group(fth_server* s, Group& g) {
    const int64_t K = g.chunk_K;
    g.inflight = false;
    const double ms = event_ms(g.ev0, g.ev1);
    g.step_ms = ms / double(K);
    g.phase = (g.phase + K) % s->opt.steps_per_tick;
    std::vector<SrvRequest*> members(g.members);
    for (SrvRequest* r : members) {
        fth_ctx* c = r->ctx;
        c->step += K;
        r->info.steps += K;
        r->info.chunks += 1;
        r->info.device_ms += ms;
        note_span(s, r->info, g.ev0, g.ev1);
        int32_t flag = 0;
        if (hipMemcpy(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) flag = 1;
        if (flag) {
            c->poisoned = true;
            finish(s, r, FTH_REQ_FAILED,
                   fail(FTH_ENONFINITE, "non-finite state in request %llu", (unsigned long long)r->id));
            continue;
        }
        if (g.phase == 0) check(s, r);
    }
}

bool event_done(hipEvent_t e) { return hipEventQuery(e) != hipErrorNotReady; }

// Retire every finished chunk; returns how many were processed.
int complete_finished(fth_server* s) {
    int done = 0;
    for (auto& kv : s->groups) {
        Group& g = kv.second;
        if (g.inflight && event_done(g.ev1)) {
            complete_group(s, g);
            ++done;
        }
    }
    std::vector<SrvRequest*> act(s->running);
    for (SrvRequest* r : act)
        if (r->inflight && r->group < 0 && event_done(r->ev1)) {
            complete_unpacked(s, r);
            ++done;
        }
    return done;
}

Group& group_for(fth_server* s, int ns, fth_status* st) {
    Group& g = s->groups[ns];
    *st = FTH_OK;
    if (!g.stream) {
        g.ns = ns;
        if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&g.ev0) != hipSuccess || hipEventCreate(&g.ev1) != hipSuccess)
            *st = fail(FTH_EDEVICE, "packed group stream creation failed");
    }
    return g;
}

// Issue a chunk to every idle group and idle unpacked request.
void issue(fth_server* s) {
    // idle packable requests at a check boundary join their group when it is at one too
    for (SrvRequest* r : s->running) r->waiting = false;
    for (SrvRequest* r : std::vector<SrvRequest*>(s->running)) {
        if (!r->packable || r->group >= 0 || r->inflight || r->info.steps % s->opt.steps_per_tick != 0) continue;
        fth_status st;
        Group& g = group_for(s, r->gle.ns, &st);
        if (st != FTH_OK) {
            r->packable = false;
            continue;
        }
        if (g.inflight || g.phase != 0) {
            // wait for the group (issue nothing) when its chunk in flight ends at a check
            // boundary, which is at most one chunk away; else run another chunk alone
            if (g.inflight && (g.phase + g.chunk_K) % s->opt.steps_per_tick == 0) r->waiting = true;
            continue;
        }
        r->waiting = false;
        g.members.push_back(r);
        g.dirty = true;
        r->group = g.ns;
        r->info.packed = 1;
    }
    for (auto& kv : s->groups) {
        Group& g = kv.second;
        if (g.inflight || g.members.empty()) continue;
        fth_status st = g.dirty ? group_upload(s, g) : FTH_OK;
        hipGraphExec_t ex = nullptr;
        const int64_t K = chunk_len(s, g.phase, g.step_ms);
        if (st == FTH_OK) st = group_graph(g, K, &ex);
        if (st == FTH_OK && (hipEventRecord(g.ev0, g.stream) != hipSuccess || hipGraphLaunch(ex, g.stream) != hipSuccess ||
                             hipEventRecord(g.ev1, g.stream) != hipSuccess))
            st = fail(FTH_EDEVICE, "packed chunk launch failed: %s", hipGetErrorString(hipGetLastError()));
        if (st != FTH_OK) {  // the members fail; nothing of this group is in flight
            (void)hipStreamSynchronize(g.stream);
            for (SrvRequest* r : std::vector<SrvRequest*>(g.members)) finish(s, r, FTH_REQ_FAILED, st);
            continue;
        }
        g.chunk_K = K;
        g.inflight = true;
    }
    for (SrvRequest* r : std::vector<SrvRequest*>(s->running)) {
        if (r->group >= 0 || r->inflight || r->waiting) continue;
        const int64_t K = chunk_len(s, r->info.steps % s->opt.steps_per_tick, r->step_ms);
        fth_status st = FTH_OK;
        if (hipEventRecord(r->ev0, r->ctx->stream) != hipSuccess) st = fail(FTH_EDEVICE, "event record failed");
        if (st == FTH_OK) st = run_enqueue(r->ctx, K);
        if (st == FTH_OK && hipEventRecord(r->ev1, r->ctx->stream) != hipSuccess)
            st = fail(FTH_EDEVICE, "event record failed");
        if (st != FTH_OK) {
            finish(s, r, FTH_REQ_FAILED, st);  // destroys the context after its stream drains
            continue;
        }
        r->chunk_K = K;
        r->inflight = true;
    }
}

bool any_inflight(const fth_server* s) {
    for (const auto& kv : s->groups)
        if (kv.second.inflight) return true;
    for (const SrvRequest* r : s->running)
        if (r->inflight) return true;
    return false;
}

}  // namespace

extern "C" {

fth_status fth_server_create(const fth_server_options* opt, fth_server** out) {
    g_last_error.clear();
    if (!out) return fail(FTH_EINVAL, "out must not be NULL");
    *out = nullptr;
    std::unique_ptr<fth_server> s(new fth_server());
    if (opt) s->opt = *opt;
    if (s->opt.steps_per_tick <= 0) s->opt.steps_per_tick = 200;
    if (s->opt.max_active <= 0) s->opt.max_active = 64;
    if (s->opt.min_blocks <= 0) s->opt.min_blocks = 8;
    if (s->opt.quantum_ms == 0) s->opt.quantum_ms = kDefaultQuantumMs;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FTH_EDEVICE, "no HIP device available");
    HIP_OK(hipGetDevice(&s->device));
    if (s->opt.hbm_budget == 0) {
        size_t free_b = 0, total_b = 0;
        HIP_OK(hipMemGetInfo(&free_b, &total_b));
        s->opt.hbm_budget = free_b / 10 * 8;
    }
    HIP_OK(hipEventCreate(&s->ev_ref));
    HIP_OK(hipEventRecord(s->ev_ref, nullptr));
    HIP_OK(hipEventSynchronize(s->ev_ref));
    s->t0 = std::chrono::steady_clock::now();
    *out = s.release();
    return FTH_OK;
}

fth_status fth_server_submit(fth_server* s, const fth_request* q, uint64_t* id) {
    g_last_error.clear();
    if (!s || !q || !id) return fail(FTH_EINVAL, "invalid arguments");
    std::unique_ptr<SrvRequest> r(new SrvRequest());
    r->id = s->next_id;
    const fth_matrix& M = q->M;
    if (M.n < 1) return fail(FTH_EINVAL, "n must be >= 1");
    r->M = M;
    if (M.format == FTH_CSR) {
        if (!M.row_ptr || !M.col || !M.val) return fail(FTH_EINVAL, "CSR arrays must not be NULL");
        r->row_ptr.assign(M.row_ptr, M.row_ptr + M.n + 1);
        r->col.assign(M.col, M.col + M.nnz);
        r->val.resize(size_t(M.nnz));
        for (int64_t k = 0; k < M.nnz; ++k)
            r->val[k] = M.value_is_f64 ? static_cast<const double*>(M.val)[k] : static_cast<const float*>(M.val)[k];
        r->M.row_ptr = r->row_ptr.data();
        r->M.col = r->col.data();
        r->M.val = r->val.data();
        r->M.value_is_f64 = 1;
    } else if (M.format == FTH_DENSE) {
        if (!M.dense) return fail(FTH_EINVAL, "dense pointer must not be NULL");
        const size_t cnt = size_t(M.n) * size_t(M.n);
        r->dense.resize(cnt);
        for (size_t k = 0; k < cnt; ++k)
            r->dense[k] = M.value_is_f64 ? static_cast<const double*>(M.dense)[k] : static_cast<const float*>(M.dense)[k];
        r->M.dense = r->dense.data();
        r->M.value_is_f64 = 1;
    } else {
        return fail(FTH_EINVAL, "unknown matrix format");
    }
    if (!q->gle.A_p || !q->gle.C_p || q->gle.ns < 0) return fail(FTH_EINVAL, "invalid GLE");
    const size_t d = size_t(q->gle.ns + 1);
    r->A.assign(q->gle.A_p, q->gle.A_p + d * d);
    r->C.assign(q->gle.C_p, q->gle.C_p + d * d);
    r->gle.ns = q->gle.ns;
    r->gle.A_p = r->A.data();
    r->gle.C_p = r->C.data();
    r->dt = q->dt;
    if (q->npairs < 0 || (q->npairs > 0 && !q->pairs)) return fail(FTH_EINVAL, "invalid pair list");
    r->pairs.assign(q->pairs, q->pairs + 2 * q->npairs);
    fth_default_options(&r->opt);
    r->opt.seed = q->seed;
    r->opt.stream_id = q->stream_id ? q->stream_id : uint32_t(r->id);
    r->opt.precision = q->precision;
    r->opt.burn_in = q->burn_in;
    r->opt.block_len = q->block_len > 0 ? q->block_len : 100;
    r->opt.replicas = q->replicas > 0 ? q->replicas : (M.format == FTH_CSR ? 32 : 64);
    r->opt.steps_per_graph = s->opt.steps_per_tick;
    r->opt.coded_matrix = -1;  // the packed kernel reads plain CSR; keep the footprint as admitted
    r->opt.scale_r = q->scale_r;
    r->opt.scale_m = q->scale_m;
    r->opt.gle_alpha = q->gle_alpha;
    r->opt.gle_gamma = q->gle_gamma;
    if (q->unscale_target < -1 || q->unscale_target > FTH_TARGET_EXPNEG) return fail(FTH_EINVAL, "unknown unscale target");
    r->unscale_target = q->unscale_target;
    r->momentum = q->momentum_form != 0;
    r->opt.acc_pp = r->momentum ? 1 : 0;
    r->target = q->target_rel_stderr;
    r->max_steps = q->max_steps;
    // normalisation of off-diagonal estimates by the request's own diagonals
    std::map<int32_t, int64_t> diag;
    r->kind_weight.assign(size_t(q->npairs), 0.0);
    for (int64_t k = 0; k < q->npairs; ++k)
        if (r->pairs[2 * k] == r->pairs[2 * k + 1]) {
            r->kind_weight[size_t(k)] = 1.0;
            if (!diag.count(r->pairs[2 * k])) diag[r->pairs[2 * k]] = k;
        }
    r->di.assign(size_t(q->npairs), -1);
    r->dj.assign(size_t(q->npairs), -1);
    for (int64_t k = 0; k < q->npairs; ++k) {
        auto a = diag.find(r->pairs[2 * k]), b = diag.find(r->pairs[2 * k + 1]);
        if (a != diag.end()) r->di[k] = a->second;
        if (b != diag.end()) r->dj[k] = b->second;
    }
    // validation now (cheap relative to the run); device work happens at admission
    fth_status st = M.format == FTH_CSR ? check_csr(&r->M) : check_dense(&r->M);
    if (st != FTH_OK) return st;
    std::vector<double> T, S;
    st = make_propagator(&r->gle, r->dt, T, S);
    if (st != FTH_OK) return st;
    // (a momentum-form request keeps a second set of accumulators: counted as twice the pairs)
    r->info.footprint = fth_footprint_bytes(&r->M, r->gle.ns, r->opt.replicas, q->npairs * (r->momentum ? 2 : 1), 0,
                                            r->opt.precision);
    if (r->info.footprint > s->opt.hbm_budget)
        return fail(FTH_ENOMEM, "request footprint %zu exceeds the server budget %zu", r->info.footprint,
                    s->opt.hbm_budget);
    r->info.state = FTH_REQ_QUEUED;
    r->info.status = FTH_OK;
    r->info.t_submit = s->clock();
    r->info.t_start = r->info.t_finish = -1.0;
    r->info.n_out = q->npairs;
    r->info.replicas = r->opt.replicas;
    r->info.max_rel_stderr = std::numeric_limits<double>::infinity();
    r->info.device_first_ms = r->info.device_last_ms = -1.0;
    s->queue.push_back(r.get());
    *id = r->id;
    s->all[r->id] = std::move(r);
    s->next_id++;
    return FTH_OK;
}

fth_status fth_server_tick(fth_server* s) {
    g_last_error.clear();
    if (!s) return fail(FTH_EINVAL, "server must not be NULL");
    HIP_OK(hipSetDevice(s->device));
    complete_finished(s);
    // admission, in arrival order, while the footprint fits
    while (!s->queue.empty() && int(s->running.size()) < s->opt.max_active) {
        SrvRequest* r = s->queue.front();
        if (s->reserved + r->info.footprint > s->opt.hbm_budget) break;
        s->queue.pop_front();
        fth_status st = admit(s, r);
        if (st != FTH_OK) {
            r->info.state = FTH_REQ_FAILED;
            r->info.status = st;
            r->info.t_finish = s->clock();
        }
    }
    issue(s);
    // wait for the first chunk that ends
    while (any_inflight(s)) {
        if (complete_finished(s) > 0) break;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    return FTH_OK;
}

fth_status fth_server_poll(fth_server* s, uint64_t id, fth_request_info* info) {
    if (!s || !info) return fail(FTH_EINVAL, "invalid arguments");
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(FTH_EINVAL, "unknown request id %llu", (unsigned long long)id);
    *info = it->second->info;
    return FTH_OK;
}

fth_status fth_server_result(fth_server* s, uint64_t id, double* est, double* se, int64_t len) {
    if (!s) return fail(FTH_EINVAL, "invalid arguments");
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(FTH_EINVAL, "unknown request id %llu", (unsigned long long)id);
    SrvRequest* r = it->second.get();
    if (len < r->info.n_out) return fail(FTH_EINVAL, "output length too small");
    std::vector<double> e(size_t(r->info.n_out)), v(size_t(r->info.n_out));
    if (r->ctx) {  // a chunk in flight is finished and counted first, so estimates and step count agree
        if (r->group >= 0 && s->groups[r->group].inflight) {
            HIP_OK(hipEventSynchronize(s->groups[r->group].ev1));
            complete_group(s, s->groups[r->group]);
        } else if (r->group < 0 && r->inflight) {
            HIP_OK(hipEventSynchronize(r->ev1));
            complete_unpacked(s, r);
        }
    }
    if (r->ctx) {
        fth_status st = read_reported(r, e, v, nullptr);
        if (st != FTH_OK) return st;
    } else {
        if (r->info.state != FTH_REQ_DONE) return fail(FTH_ESTATE, "request has no result");
        e = r->est;
        v = r->se;
    }
    if (r->unscale_target >= 0) {
        if (r->momentum && r->opt.gle_alpha != 0.0 && r->opt.gle_alpha != 1.0) {
            // fth_unscale undoes the position prefactor gamma / alpha^2; the momentum
            // response carries gamma alone
            const double a2 = 1.0 / (r->opt.gle_alpha * r->opt.gle_alpha);
            for (size_t k = 0; k < e.size(); ++k) {
                e[k] *= a2;
                v[k] *= a2;
            }
        }
        fth_status st = fth_unscale(r->unscale_target, r->opt.scale_r == 0 ? 1.0 : r->opt.scale_r, r->opt.scale_m,
                                    r->opt.gle_alpha == 0 ? 1.0 : r->opt.gle_alpha,
                                    r->opt.gle_gamma == 0 ? 1.0 : r->opt.gle_gamma, r->info.n_out,
                                    r->kind_weight.data(), e.data(), v.data());
        if (st != FTH_OK) return st;
    }
    if (est) std::memcpy(est, e.data(), sizeof(double) * e.size());
    if (se) std::memcpy(se, v.data(), sizeof(double) * v.size());
    return FTH_OK;
}

fth_status fth_server_cancel(fth_server* s, uint64_t id) {
    if (!s) return fail(FTH_EINVAL, "invalid arguments");
    auto it = s->all.find(id);
    if (it == s->all.end()) return fail(FTH_EINVAL, "unknown request id %llu", (unsigned long long)id);
    SrvRequest* r = it->second.get();
    if (r->info.state == FTH_REQ_QUEUED) {
        s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
        r->info.state = FTH_REQ_CANCELLED;
        r->info.t_finish = s->clock();
    } else if (r->info.state == FTH_REQ_RUNNING) {
        if (r->group >= 0) {  // its group's chunk must finish before the work list changes
            Group& g = s->groups[r->group];
            if (g.inflight) {
                HIP_OK(hipEventSynchronize(g.ev1));
                complete_group(s, g);
            }
        } else if (r->inflight) {
            HIP_OK(hipEventSynchronize(r->ev1));
            r->inflight = false;
        }
        if (r->info.state == FTH_REQ_RUNNING) finish(s, r, FTH_REQ_CANCELLED, FTH_OK);
    }
    return FTH_OK;
}

double fth_server_clock(const fth_server* s) { return s ? s->clock() : 0.0; }

fth_status fth_server_stats(const fth_server* s, int64_t* queued, int64_t* running, size_t* reserved) {
    if (!s) return fail(FTH_EINVAL, "invalid arguments");
    if (queued) *queued = int64_t(s->queue.size());
    if (running) *running = int64_t(s->running.size());
    if (reserved) *reserved = s->reserved;
    return FTH_OK;
}

fth_status fth_server_destroy(fth_server* s) {
    delete s;
    return FTH_OK;
}

}  // extern "C"
