// Serving layer: many FTH solves of different size and sparsity sharing one
// GPU with continuous batching.
//
// A tick (fth_server_tick):
//   1. admission: queued requests, in arrival order, get a context (device
//      memory) while their footprint fits the remaining budget;
//   2. work: every running sparse FP32 request of a group (same ns) is
//      advanced by one persistent packed kernel per step over a device list
//      of (request, row tile | pair tile) entries -- one captured graph of
//      steps_per_tick launches plus a step-counter advance per group; the
//      other requests (dense, FP64) run their own kernels on their own
//      streams, so their work overlaps with the packed kernel on the device;
//   3. check: every running request's estimates and block stderrs are read
//      (a few KB each); requests at their target or max_steps retire and
//      release their memory for the queue.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <vector>

#include "fth_ctx.hpp"

using namespace fth::host;

namespace {

constexpr int kPackedGrid = 2048;  // persistent workgroups (multiple of 8: one slice per XCD)

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
    std::vector<int64_t> di, dj;  // output index of (i,i) and (j,j) for each pair, or -1
    // run state
    fth_ctx* ctx = nullptr;
    int group = -1;  // ns of its packed group, or -1
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
    hipGraphExec_t graph = nullptr;
    int graph_K = 0;
    bool dirty = true;
};

bool packable(const SrvRequest& r) {
    return r.M.format == FTH_CSR && r.opt.precision == FTH_FP32 && r.opt.replicas % 4 == 0 && r.opt.replicas >= 4 &&
           r.opt.replicas <= 256 && r.gle.ns <= fth::kNsMax;
}

}  // namespace

struct fth_server {
    fth_server_options opt{};
    std::chrono::steady_clock::time_point t0;
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t next_id = 1;
    std::map<uint64_t, std::unique_ptr<SrvRequest>> all;
    std::deque<SrvRequest*> queue;
    std::vector<SrvRequest*> running;
    size_t reserved = 0;
    std::map<int, Group> groups;

    double clock() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    ~fth_server() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (SrvRequest* r : running) fth_destroy(r->ctx);
        for (auto& kv : groups) {
            Group& g = kv.second;
            if (g.graph) (void)hipGraphExecDestroy(g.graph);
            (void)hipFree(g.d_table);
            (void)hipFree(g.d_tiles);
            (void)hipFree(g.d_counts);
        }
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

fth_status group_upload(fth_server* s, Group& g) {
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
    bool realloc = false;
    if (nslots > g.cap_slots) {
        (void)hipFree(g.d_table);
        g.cap_slots = std::max(2 * g.cap_slots, std::max(nslots, 8));
        HIP_OK(hipMalloc(&g.d_table, sizeof(fth::StepArgs<float>) * size_t(g.cap_slots)));
        realloc = true;
    }
    if (int64_t(tiles.size()) > g.cap_tiles) {
        (void)hipFree(g.d_tiles);
        g.cap_tiles = std::max<int64_t>(2 * g.cap_tiles, std::max<int64_t>(int64_t(tiles.size()), 1024));
        HIP_OK(hipMalloc(&g.d_tiles, sizeof(fth::PackedTile) * size_t(g.cap_tiles)));
        realloc = true;
    }
    if (!g.d_counts) {
        HIP_OK(hipMalloc(&g.d_counts, 2 * sizeof(int32_t)));
        realloc = true;
    }
    if (int64_t(tiles.size()) > 0x7FFFFFFF) return fail(FTH_EUNSUPPORTED, "too many tiles in one packed group");
    const int32_t counts[2] = {int32_t(tiles.size()), nslots};
    const int32_t nt = counts[0];
    HIP_OK(hipMemcpyAsync(g.d_table, table.data(), sizeof(fth::StepArgs<float>) * size_t(nslots),
                          hipMemcpyHostToDevice, s->stream));
    if (nt > 0)
        HIP_OK(hipMemcpyAsync(g.d_tiles, tiles.data(), sizeof(fth::PackedTile) * tiles.size(), hipMemcpyHostToDevice,
                              s->stream));
    HIP_OK(hipMemcpyAsync(g.d_counts, counts, sizeof(counts), hipMemcpyHostToDevice, s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    if (realloc && g.graph) {
        (void)hipGraphExecDestroy(g.graph);
        g.graph = nullptr;
    }
    g.dirty = false;
    return FTH_OK;
}

fth_status group_enqueue(fth_server* s, Group& g, int K) {
    const int nslots = int(g.members.size());
    if (nslots == 0) return FTH_OK;
    // The graph bakes the table pointers and the slot count of the advance.
    if (g.graph && g.graph_K != K) {
        (void)hipGraphExecDestroy(g.graph);
        g.graph = nullptr;
    }
    if (!g.graph) {
        HIP_OK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed));
        int rc = 0;
        for (int k = 0; k < K && rc == 0; ++k)
            rc = fth::launch_packed_csr(g.d_table, g.d_tiles, g.d_counts, g.ns, false, kPackedGrid, k, s->stream);
        if (rc == 0) rc = fth::launch_advance_all(g.d_table, g.d_counts + 1, K, s->stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s->stream, &graph);
        if (rc != 0) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(FTH_EDEVICE, "packed kernel launch failed (%d)", rc);
        }
        if (e != hipSuccess) return fail(FTH_EDEVICE, "packed graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&g.graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(FTH_EDEVICE, "packed graph instantiate failed: %s", hipGetErrorString(e));
        g.graph_K = K;
    }
    HIP_OK(hipGraphLaunch(g.graph, s->stream));
    return FTH_OK;
}

void finish(fth_server* s, SrvRequest* r, int32_t state, fth_status st) {
    if (r->ctx) {
        const int64_t no = fth_num_outputs(r->ctx);
        r->est.assign(size_t(no), 0.0);
        r->se.assign(size_t(no), 0.0);
        if (state == FTH_REQ_DONE) (void)fth_read(r->ctx, r->est.data(), r->se.data(), no, nullptr);
        fth_destroy(r->ctx);
        r->ctx = nullptr;
        s->reserved -= r->info.footprint;
    }
    if (r->group >= 0) {
        Group& g = s->groups[r->group];
        g.members.erase(std::remove(g.members.begin(), g.members.end(), r), g.members.end());
        g.dirty = true;
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
    s->reserved += r->info.footprint;
    r->info.t_start = s->clock();
    r->info.state = FTH_REQ_RUNNING;
    // the packed kernel runs 256-thread workgroups with 4 replicas per thread
    if (packable(*r) && c->rpt == 4 && c->block == 256) {
        r->group = r->gle.ns;
        Group& g = s->groups[r->group];
        g.ns = r->gle.ns;
        g.members.push_back(r);
        g.dirty = true;
        r->info.packed = 1;
    }
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
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FTH_EDEVICE, "no HIP device available");
    HIP_OK(hipGetDevice(&s->device));
    if (s->opt.hbm_budget == 0) {
        size_t free_b = 0, total_b = 0;
        HIP_OK(hipMemGetInfo(&free_b, &total_b));
        s->opt.hbm_budget = free_b / 10 * 8;
    }
    HIP_OK(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
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
    r->target = q->target_rel_stderr;
    r->max_steps = q->max_steps;
    // normalisation of off-diagonal estimates by the request's own diagonals
    std::map<int32_t, int64_t> diag;
    for (int64_t k = 0; k < q->npairs; ++k)
        if (r->pairs[2 * k] == r->pairs[2 * k + 1] && !diag.count(r->pairs[2 * k])) diag[r->pairs[2 * k]] = k;
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
    r->info.footprint = fth_footprint_bytes(&r->M, r->gle.ns, r->opt.replicas, q->npairs, 0, r->opt.precision);
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
    // 1. admission, in arrival order, while the footprint fits
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
    if (s->running.empty()) return FTH_OK;
    const int K = s->opt.steps_per_tick;
    // every request advances in whole ticks, so its step schedule does not depend on packing
    std::vector<SrvRequest*> active(s->running);
    std::vector<int64_t> ksteps(active.size(), K);
    // 2. work: unpacked requests on their own streams, packed groups on the server stream
    std::vector<fth_status> ust(active.size(), FTH_OK);
    for (size_t k = 0; k < active.size(); ++k) {
        SrvRequest* r = active[k];
        if (r->group >= 0 || ksteps[k] <= 0) continue;
        ust[k] = run_enqueue(r->ctx, ksteps[k]);
    }
    for (auto& kv : s->groups) {
        Group& g = kv.second;
        if (g.members.empty()) continue;
        if (g.dirty) {
            fth_status st = group_upload(s, g);
            if (st != FTH_OK) return st;
        }
        fth_status st = group_enqueue(s, g, K);
        if (st != FTH_OK) return st;
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    // 3. check and retire
    for (size_t k = 0; k < active.size(); ++k) {
        SrvRequest* r = active[k];
        fth_status st = FTH_OK;
        if (r->group >= 0) {
            fth_ctx* c = r->ctx;
            c->step += K;
            int32_t flag = 0;
            HIP_OK(hipMemcpy(&flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost));
            if (flag) {
                c->poisoned = true;
                st = fail(FTH_ENONFINITE, "non-finite state in request %llu", (unsigned long long)r->id);
            }
            r->info.steps += K;
        } else if (ksteps[k] > 0) {
            st = ust[k] == FTH_OK ? run_complete(r->ctx, ksteps[k]) : ust[k];
            r->info.steps += ksteps[k];
        }
        if (st != FTH_OK) {
            finish(s, r, FTH_REQ_FAILED, st);
            continue;
        }
        const int64_t no = fth_num_outputs(r->ctx);
        std::vector<double> est(static_cast<size_t>(no)), se(static_cast<size_t>(no));
        int64_t nacc = 0;
        st = fth_read(r->ctx, est.data(), se.data(), no, &nacc);
        if (st != FTH_OK) {
            finish(s, r, FTH_REQ_FAILED, st);
            continue;
        }
        r->info.nblocks = nacc / r->opt.block_len;
        r->info.max_rel_stderr = max_rel_stderr(*r, est, se, r->info.nblocks, s->opt.min_blocks);
        const bool reached = r->info.max_rel_stderr <= r->target;
        const bool capped = r->max_steps > 0 && r->info.steps >= r->max_steps;
        if (reached || capped) finish(s, r, FTH_REQ_DONE, FTH_OK);
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
    if (r->ctx) return fth_read(r->ctx, est, se, len, nullptr);
    if (r->info.state != FTH_REQ_DONE) return fail(FTH_ESTATE, "request has no result");
    if (est) std::memcpy(est, r->est.data(), sizeof(double) * r->est.size());
    if (se) std::memcpy(se, r->se.data(), sizeof(double) * r->se.size());
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
        HIP_OK(hipStreamSynchronize(s->stream));
        finish(s, r, FTH_REQ_CANCELLED, FTH_OK);
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
