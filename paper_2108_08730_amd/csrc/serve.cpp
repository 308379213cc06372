// Serving loop: continuous admission of solve requests on one GPU.
//
// Requests queue in arrival order.  A worker (one per slot, each with its own
// non-blocking HIP stream) takes the first queued request whose estimated
// device footprint fits in the free part of the HBM budget, so requests that
// arrive while others run start as soon as a slot and memory free up, and
// their kernels overlap on the device.  A request whose right-hand sides
// together would need more than half the budget is solved in chunks of
// right-hand sides, one after another on one operator.  Operators (with their multigrid
// hierarchies) stay resident in a cache keyed by the model and the
// discretisation; cached operators count against the budget and are evicted
// least-recently-used when an admission needs the memory.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "internal.h"

namespace h27 {

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct OpKey {
    uint64_t model;
    int nx, ny, nz;
    double h, freq;
    int npml[3];
    double R, c_ref;
    bool operator<(const OpKey& o) const {
        return std::tie(model, nx, ny, nz, h, freq, npml[0], npml[1], npml[2], R, c_ref) <
               std::tie(o.model, o.nx, o.ny, o.nz, o.h, o.freq, o.npml[0], o.npml[1], o.npml[2], o.R, o.c_ref);
    }
};

struct CachedOp {
    OpKey key;
    helm27_op* op;
    size_t bytes;
};

struct Job {
    uint64_t ticket;
    std::vector<float> vel;
    int nx, ny, nz;
    double h, freq;
    helm27_pml pml;
    std::vector<double> src;
    int nrhs;
    int chunk;                   // right-hand sides per solve (all of them unless the request is split)
    uint64_t model_key;
    void* out;
    size_t footprint;
    helm27_result res;
};

struct Server {
    helm27_ctx* ctx = nullptr;
    helm27_serve_opts opts;
    helm27_table* table = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<uint64_t, std::shared_ptr<Job>> running;
    std::map<uint64_t, helm27_result> done;
    std::list<CachedOp> cache;   // front = most recently used
    std::vector<std::thread> workers;
    size_t used = 0;             // admitted footprints + cached operators
    uint64_t next_ticket = 1;
    bool stopping = false;
};

static size_t op_estimate(int64_t N) {
    // velocity + index (6 B/pt) and the multigrid coarse grids (~1/7 more)
    return static_cast<size_t>(N) * 7 + (1u << 20);
}

static size_t job_footprint(const helm27_serve_opts& o, int64_t N, int nrhs) {
    return op_estimate(N) + solve_footprint(N, nrhs, o.solve.restart, o.solve.precision, o.solve.mg_levels);
}

// Right-hand sides per solve: all of them when the request needs at most half
// the budget, else the largest count that does (at least one), so a request
// too large to share the device is solved in chunks, one after another, on
// one operator, leaving room for other requests.
static int job_chunk(const helm27_serve_opts& o, int64_t N, int nrhs, size_t budget) {
    if (o.max_chunk_rhs > 0 && nrhs > o.max_chunk_rhs) nrhs = o.max_chunk_rhs;
    if (job_footprint(o, N, nrhs) <= budget / 2) return nrhs;
    int lo = 1, hi = nrhs;   // largest c with footprint(c) <= budget / 2 (footprint grows with c)
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (job_footprint(o, N, mid) <= budget / 2) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// statistics of a request solved in chunks: totals of the work, worst of the accuracy
static void merge_stats(helm27_solve_stats* a, const helm27_solve_stats& b, bool first) {
    if (first) {
        *a = b;
        return;
    }
    a->outer_iters = std::max(a->outer_iters, b.outer_iters);
    a->inner_iters += b.inner_iters;
    a->converged = a->converged && b.converged;
    a->max_relres = std::max(a->max_relres, b.max_relres);
    a->seconds += b.seconds;
    a->mg_levels = b.mg_levels;
    a->coarse_clamped = std::max(a->coarse_clamped, b.coarse_clamped);
    a->coarse_tables = std::max(a->coarse_tables, b.coarse_tables);
    a->inner_est = std::max(a->inner_est, b.inner_est);
}

// Evict least-recently-used cached operators until `need` bytes fit (lock held).
static void evict_for(Server* S, size_t need) {
    while (!S->cache.empty() && S->used + need > S->ctx->hbm_budget) {
        CachedOp c = S->cache.back();
        S->cache.pop_back();
        S->used -= std::min(S->used, c.bytes);
        helm27_op_destroy(c.op);
    }
}

static void worker_main(Server* S) {
    hipSetDevice(S->ctx->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    for (;;) {
        std::shared_ptr<Job> job;
        helm27_op* op = nullptr;
        OpKey key{};
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                if (S->stopping && S->queue.empty()) break;
                // first queued request that fits next to the running ones
                for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
                    std::shared_ptr<Job>& j = *it;
                    key = OpKey{j->model_key, j->nx, j->ny, j->nz, j->h, j->freq,
                                {j->pml.npml[0], j->pml.npml[1], j->pml.npml[2]}, j->pml.R, j->pml.c_ref};
                    auto hit = S->cache.end();
                    if (j->model_key != 0)
                        for (auto c = S->cache.begin(); c != S->cache.end(); ++c)
                            if (!(c->key < key) && !(key < c->key)) {
                                hit = c;
                                break;
                            }
                    const size_t need = hit != S->cache.end() ? j->footprint - std::min(j->footprint, hit->bytes)
                                                              : j->footprint;
                    if (S->used + need > S->ctx->hbm_budget) {
                        // make room from cached operators other than the one we would reuse
                        CachedOp keep{};
                        const bool have = hit != S->cache.end();
                        if (have) {
                            keep = *hit;
                            S->cache.erase(hit);
                            S->used -= std::min(S->used, keep.bytes);
                        }
                        evict_for(S, j->footprint);
                        if (have) {
                            S->cache.push_front(keep);
                            S->used += keep.bytes;
                            hit = S->cache.begin();
                        }
                    }
                    if (S->used + need <= S->ctx->hbm_budget || (S->running.empty() && it == S->queue.begin())) {
                        job = j;
                        if (hit != S->cache.end()) {
                            op = hit->op;
                            S->used -= std::min(S->used, hit->bytes);
                            S->cache.erase(hit);
                        }
                        S->used += job->footprint;
                        S->queue.erase(it);
                        break;
                    }
                }
                if (job) break;
                S->cv.wait(lk);
            }
            if (!job) break;
            job->res.t_start = now_s();
            S->running[job->ticket] = job;
        }
        int st = HELM27_OK;
        if (!op) {
            helm27_pml p = job->pml;
            st = op_create(S->ctx, S->table, job->vel.data(), job->nx, job->ny, job->nz, job->h, job->freq, &p, 0,
                           stream, &op);
        }
        helm27_solve_stats stats{};
        if (st == HELM27_OK) {
            const int64_t N = static_cast<int64_t>(job->nx) * job->ny * job->nz;
            int agg = HELM27_OK;
            for (int r0 = 0; r0 < job->nrhs; r0 += job->chunk) {
                const int nc = std::min(job->chunk, job->nrhs - r0);
                helm27_solve_stats s1{};
                void* out = static_cast<char*>(job->out) + static_cast<size_t>(r0) * N * 16;
                const int s = helm27_solve(op, job->src.data() + 5 * static_cast<size_t>(r0), out, nc, &S->opts.solve,
                                           &s1, stream);
                merge_stats(&stats, s1, r0 == 0);
                if (s == HELM27_ENOCONV) agg = HELM27_ENOCONV;   // keep solving the other chunks
                else if (s != HELM27_OK) {
                    agg = s;
                    break;
                }
            }
            st = agg;
        }
        hipStreamSynchronize(stream);
        if (op) solver_trim(op);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->used -= std::min(S->used, job->footprint);
            job->res.status = st;
            job->res.stats = stats;
            job->res.t_done = now_s();
            S->done[job->ticket] = job->res;
            S->running.erase(job->ticket);
            if (op) {
                if (job->model_key != 0 && S->opts.max_cached_ops > 0) {
                    const size_t b = op->g.bytes + op_estimate(op->g.N) / 7;
                    S->cache.push_front(CachedOp{key, op, b});
                    S->used += b;
                    while (static_cast<int>(S->cache.size()) > S->opts.max_cached_ops) {
                        CachedOp c = S->cache.back();
                        S->cache.pop_back();
                        S->used -= std::min(S->used, c.bytes);
                        helm27_op_destroy(c.op);
                    }
                } else {
                    helm27_op_destroy(op);
                }
            }
        }
        S->cv.notify_all();
    }
    if (stream) hipStreamDestroy(stream);
}

}  // namespace h27

using namespace h27;

void helm27_serve_shutdown(helm27_ctx* ctx) {
    if (ctx && ctx->serve) helm27_serve_stop(ctx);
}

extern "C" void helm27_serve_opts_default(helm27_serve_opts* o) {
    if (!o) return;
    o->max_slots = 4;
    helm27_solve_opts_default(&o->solve);
    o->table_gmin = 2.5;
    o->table_gmax = 60.0;
    o->table_dg = 0.05;
    o->table_lambda = 1e-3;
    o->max_cached_ops = 8;
    o->max_chunk_rhs = 0;
}

extern "C" int helm27_serve_start(helm27_ctx* ctx, const helm27_serve_opts* opts) {
    if (!ctx) return HELM27_EINVAL;
    std::lock_guard<std::mutex> g(ctx->mu);
    if (ctx->serve) return HELM27_EINVAL;
    helm27_serve_opts o;
    if (opts) o = *opts;
    else helm27_serve_opts_default(&o);
    if (o.max_slots < 1 || o.max_slots > 16 || o.max_cached_ops < 0 || o.max_chunk_rhs < 0) return HELM27_EINVAL;
    Server* S = new (std::nothrow) Server;
    if (!S) return HELM27_ENOMEM;
    S->ctx = ctx;
    S->opts = o;
    int st = helm27_build_table(ctx, o.table_gmin, o.table_gmax, o.table_dg, o.table_lambda, nullptr, &S->table);
    if (st) {
        delete S;
        return st;
    }
    for (int k = 0; k < o.max_slots; ++k) S->workers.emplace_back(worker_main, S);
    ctx->serve = S;
    return HELM27_OK;
}

extern "C" int helm27_serve_submit(helm27_ctx* ctx, const helm27_request* r, uint64_t* ticket) {
    if (!ctx || !r || !ticket || !ctx->serve) return HELM27_EINVAL;
    Server* S = static_cast<Server*>(ctx->serve);
    if (!r->vel || !r->src || !r->out || r->nrhs <= 0 || r->nx < 3 || r->ny < 3 || r->nz < 3 || !(r->h > 0) ||
        !(r->freq > 0))
        return HELM27_EINVAL;
    const int dims[3] = {r->nx, r->ny, r->nz};
    for (int k = 0; k < r->nrhs; ++k)
        for (int a = 0; a < 3; ++a) {
            const double v = r->src[5 * k + a];
            if (v < r->pml.npml[a] || v > dims[a] - 1 - r->pml.npml[a]) return HELM27_ERANGE;
        }
    const int64_t N = static_cast<int64_t>(r->nx) * r->ny * r->nz;
    auto job = std::make_shared<Job>();
    job->chunk = job_chunk(S->opts, N, r->nrhs, ctx->hbm_budget);
    job->footprint = job_footprint(S->opts, N, job->chunk);
    if (job->footprint > ctx->hbm_budget) return HELM27_EADMIT;
    job->vel.resize(N);
    hipPointerAttribute_t attr;
    const bool dev = hipPointerGetAttributes(&attr, r->vel) == hipSuccess && attr.type == hipMemoryTypeDevice;
    (void)hipGetLastError();
    if (dev) {
        if (hipMemcpy(job->vel.data(), r->vel, N * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
            return HELM27_EDEVICE;
    } else {
        std::memcpy(job->vel.data(), r->vel, N * sizeof(float));
    }
    job->nx = r->nx;
    job->ny = r->ny;
    job->nz = r->nz;
    job->h = r->h;
    job->freq = r->freq;
    job->pml = r->pml;
    job->src.assign(r->src, r->src + 5 * r->nrhs);
    job->nrhs = r->nrhs;
    job->model_key = r->model_key;
    job->out = r->out;
    std::memset(&job->res, 0, sizeof(job->res));
    job->res.status = HELM27_EAGAIN;
    job->res.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) return HELM27_EINVAL;
        job->ticket = S->next_ticket++;
        *ticket = job->ticket;
        S->queue.push_back(job);
    }
    S->cv.notify_all();
    return HELM27_OK;
}

extern "C" int helm27_serve_poll(helm27_ctx* ctx, uint64_t ticket, helm27_result* res) {
    if (!ctx || !ctx->serve) return HELM27_EINVAL;
    Server* S = static_cast<Server*>(ctx->serve);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->done.find(ticket);
    if (it != S->done.end()) {
        if (res) *res = it->second;
        return HELM27_OK;
    }
    if (S->running.count(ticket)) return HELM27_EAGAIN;
    for (auto& j : S->queue)
        if (j->ticket == ticket) return HELM27_EAGAIN;
    return HELM27_ENOTFOUND;
}

extern "C" int helm27_serve_wait(helm27_ctx* ctx, uint64_t ticket, helm27_result* res, double timeout_s) {
    if (!ctx || !ctx->serve) return HELM27_EINVAL;
    Server* S = static_cast<Server*>(ctx->serve);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        auto it = S->done.find(ticket);
        if (it != S->done.end()) {
            if (res) *res = it->second;
            return HELM27_OK;
        }
        bool known = S->running.count(ticket) > 0;
        for (auto& j : S->queue) known = known || j->ticket == ticket;
        if (!known) return HELM27_ENOTFOUND;
        if (S->cv.wait_until(lk, deadline) == std::cv_status::timeout) return HELM27_EAGAIN;
    }
}

extern "C" int helm27_serve_stop(helm27_ctx* ctx) {
    if (!ctx) return HELM27_EINVAL;
    Server* S = nullptr;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        S = static_cast<Server*>(ctx->serve);
        if (!S) return HELM27_EINVAL;
        ctx->serve = nullptr;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv.notify_all();
    for (auto& t : S->workers) t.join();
    for (auto& c : S->cache) helm27_op_destroy(c.op);
    S->cache.clear();
    helm27_table_destroy(S->table);
    delete S;
    return HELM27_OK;
}
