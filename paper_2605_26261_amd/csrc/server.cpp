// FTLM request server with continuous batching (ftlm_server_* in ftlm.h).
//
// A worker thread owns one HIP stream (default priority) and the caller's
// arena. The arena starts with a descriptor area (one SecWork array per
// launch group); the rest is handed out first fit, one block per request:
// its SecWork slot, bond table, sector tables and Lanczos state. Each round
// the worker admits waiting requests in arrival order while they fit, then
// issues steps_per_round Lanczos steps (H.x with fused alpha, update with
// fused beta) per group of active requests with equal N and R, reads back
// every active request's count of running chains (one synchronization per
// round), and retires the finished ones: their alpha/beta come back to the
// host, the Ritz values and the thermal reduction run there, and their memory
// returns to the arena. Chains that stop inside a round leave their sector's
// later launches of the round an early return per block.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "host.hpp"

using namespace ftlm;

namespace {

constexpr int kServerMaxActive = 256;
constexpr int kServerDefaultActive = 16;

// The arena's header: the descriptors of up to kServerMaxActive requests, then
// the work-queue counters of the persistent H.x launches (one set serves
// every launch: the worker's launches run one after the other on its stream
// and each leaves the counters at zero).
size_t server_desc_bytes() { return align256(size_t(kServerMaxActive) * sizeof(SecWork)); }
size_t server_header_bytes() { return server_desc_bytes() + kQueueBytes; }
constexpr int kServerMaxSteps = 64;
constexpr int kServerDefaultSteps = 4;

struct Request {
    uint64_t id = 0;
    // the request, copied
    int n_sites = 0, n_up = 0, R = 0, M = 0, dist = 0, nT = 0;
    uint64_t seed = 0;
    double g = 1.0;
    std::vector<int32_t> bi, bj;
    std::vector<double> J, T;
    // device residency
    ftlm_graph* graph = nullptr;
    ftlm_sector* sector = nullptr;
    size_t off = 0, bytes = 0;
    LanczosJob job;
    int32_t last_active = -1;
    // results
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = FTLM_OK;
    int steps = 0;
    std::vector<double> E, C, chi, lnZ;
    ~Request() {
        delete sector;
        ftlm_graph_destroy(graph);
    }
};

// Byte layout of one request's block.
struct ReqLayout {
    size_t secwork, bonds, table, table_bytes, total;
    SectorState st;
};

int request_layout(int n_sites, int n_up, int R, int mode, int dtype, ReqLayout& L) {
    L = ReqLayout{};
    size_t off = 0;
    L.secwork = off;
    off = align256(off + sizeof(SecWork));
    L.bonds = off;
    off = align256(off + kTablesPerGraph * sizeof(BondTable));
    if (int rc = ftlm_sector_table_bytes(n_sites, n_up, mode, &L.table_bytes)) return rc;
    L.table = off;
    off = align256(off + L.table_bytes);
    off = layout_state(binom_u64(n_sites, n_up), R, dtype, off, L.st);
    L.total = off;
    return FTLM_OK;
}

int check_request(const ftlm_request* q) {
    if (!q || !q->bi || !q->bj || !q->J || (q->nT > 0 && !q->T)) return fail(FTLM_E_INVALID, "null argument");
    if (q->n_sites < 2 || q->n_sites > kMaxSites) return fail(FTLM_E_RANGE, "n_sites %d", q->n_sites);
    if (q->n_bonds < 1 || q->n_bonds > kMaxBonds)
        return fail(FTLM_E_RANGE, "n_bonds %d not in [1, %d]", q->n_bonds, kMaxBonds);
    if (!std::isfinite(q->g)) return fail(FTLM_E_INVALID, "g is not finite");
    if (q->n_up < 0 || q->n_up > q->n_sites) return fail(FTLM_E_INVALID, "n_up %d", q->n_up);
    if (q->R < 1 || q->R > kMaxChains) return fail(FTLM_E_RANGE, "R %d not in [1, %d]", q->R, kMaxChains);
    if (q->M < 1 || q->M > kMaxSteps) return fail(FTLM_E_RANGE, "M %d", q->M);
    if (q->dist != FTLM_PM1 && q->dist != FTLM_GAUSS && q->dist != FTLM_UNIT) return fail(FTLM_E_INVALID, "dist");
    if (q->nT < 0) return fail(FTLM_E_INVALID, "nT %d", q->nT);
    for (int i = 0; i < q->nT; ++i)
        if (!(q->T[i] > 0.0)) return fail(FTLM_E_INVALID, "temperature %d not positive", i);
    return FTLM_OK;
}

// First-fit allocator over [lo, hi) of the arena.
struct Arena {
    std::map<size_t, size_t> free;  // offset -> length
    size_t used = 0, peak = 0;
    void init(size_t lo, size_t hi) {
        free.clear();
        if (hi > lo) free[lo] = hi - lo;
    }
    bool alloc(size_t n, size_t* off) {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at_ = it->first + n;
                free.erase(it);
                if (rest) free[at_] = rest;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        used -= n;
        auto it = free.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free.erase(next);
        }
        if (it != free.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free.erase(it);
            }
        }
    }
};

}  // namespace

struct ftlm_server {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    ftlm_server_opts opts{};
    std::chrono::steady_clock::time_point t0;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<std::shared_ptr<Request>> waiting;        // submitted, not admitted (arrival order)
    std::map<uint64_t, std::shared_ptr<Request>> done;   // finished, not yet polled
    std::map<uint64_t, std::shared_ptr<Request>> all;    // every unpolled request
    // worker-only state
    Arena heap;
    std::vector<std::shared_ptr<Request>> active;
    SecWork* desc_host = nullptr;          // pinned staging of the round's descriptors
    int32_t* state_host = nullptr;         // pinned [kServerMaxActive][2] readback
    std::vector<uint64_t> desc_ids;        // active requests whose descriptors are on the device
    int fatal = FTLM_OK;
    // monitoring values published by the worker
    std::atomic<uint64_t> rounds{0}, peak{0};
    std::atomic<int32_t> n_active{0};

    uint32_t* queue() const { return reinterpret_cast<uint32_t*>(arena + server_desc_bytes()); }
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void run();
    int admit(const std::shared_ptr<Request>& r);
    int round();
    void retire(const std::shared_ptr<Request>& r);
};

// Device setup of an admitted request: its graph, sector tables, descriptor
// and start vectors (on the worker's stream).
int ftlm_server::admit(const std::shared_ptr<Request>& r) {
    ReqLayout L;
    if (int rc = request_layout(r->n_sites, r->n_up, r->R, opts.mode, opts.dtype, L)) return rc;
    if (int rc = ftlm_graph_create(r->n_sites, int(r->bi.size()), r->bi.data(), r->bj.data(), r->J.data(), &r->graph))
        return rc;
    char* base = arena + r->off;
    if (int rc = ftlm_sector_create(r->n_sites, r->n_up, opts.mode, base + L.table, L.table_bytes, stream, &r->sector))
        return rc;
    job_layout(r->job, {r->sector->dev}, {L.st}, base, r->R, r->M, opts.dtype,
               reinterpret_cast<SecWork*>(base + L.secwork), {r->graph},
               {reinterpret_cast<BondTable*>(base + L.bonds)}, {0});
    r->job.queue = queue();
    if (int rc = job_start(r->job, r->seed, 0, r->dist, stream)) return rc;
    r->t_admit = now();
    return FTLM_OK;
}

// Copies a finished request's coefficients back, runs the host Ritz solves
// and the thermal reduction, and frees its arena block.
void ftlm_server::retire(const std::shared_ptr<Request>& r) {
    const int R = r->R, M = r->M;
    std::vector<double> a(size_t(R) * M), b(size_t(R) * M), th(size_t(R) * M, 0.0), w(size_t(R) * M, 0.0);
    std::vector<int32_t> steps(static_cast<size_t>(R));
    int rc = job_collect(r->job, M, a.data(), b.data(), steps.data(), stream);
    if (rc == FTLM_OK) {
        r->steps = 0;
        for (int c = 0; c < R; ++c) r->steps += steps[size_t(c)];
        // every chain solved as ftlm_ritz solves it, on host threads
        if (ftlm_ritz_batch(R, M, steps.data(), a.data(), b.data(), th.data(), w.data()) != FTLM_OK)
            rc = FTLM_E_INVALID;
    }
    if (rc == FTLM_OK && r->nT > 0) {
        ftlm_sector_result sr{};
        sr.n_up = r->n_up;
        sr.R = R;
        sr.stride = M;
        sr.dim = r->sector->dim;
        sr.mult = sector_multiplicity(r->n_sites, r->n_up);
        sr.theta = th.data();
        sr.weight = w.data();
        sr.steps = steps.data();
        r->E.assign(size_t(r->nT), 0.0);
        r->C.assign(size_t(r->nT), 0.0);
        r->chi.assign(size_t(r->nT), 0.0);
        r->lnZ.assign(size_t(r->nT), 0.0);
        rc = ftlm_thermo(r->n_sites, 1, &sr, r->nT, r->T.data(), r->g, r->E.data(), r->C.data(), r->chi.data(),
                         r->lnZ.data());
    }
    r->status = rc;
    heap.release(r->off, r->bytes);
    r->t_done = now();
}

// steps_per_round Lanczos steps for every active request: one launch pair
// per step per group of equal (N, R), or per request when batch_same_n is
// off. The groups' descriptor arrays go to the device only when the active
// set has changed since the last round.
int ftlm_server::round() {
    std::map<std::pair<int, int>, std::vector<Request*>> groups;
    std::vector<uint64_t> ids;
    for (auto& r : active) {
        const std::pair<int, int> key = opts.batch_same_n ? std::make_pair(r->n_sites, r->R)
                                                          : std::make_pair(int(r->id), -1);
        groups[key].push_back(r.get());
    }
    SecWork* desc = reinterpret_cast<SecWork*>(arena);
    std::vector<LanczosJob> jobs;
    size_t slot = 0;
    for (auto& [key, reqs] : groups) {
        // the group's descriptor array: each member's SecWork, blocks re-based
        LanczosJob g;
        g.nsec = int(reqs.size());
        g.R = reqs[0]->R;
        g.dtype = opts.dtype;
        g.mode = opts.mode;
        g.n_sites = reqs[0]->n_sites;
        uint32_t block = 0, items = 0;
        for (Request* r : reqs) {
            SecWork w = r->job.secs[0];
            w.block0 = block;
            block = (block + w.G + 7) & ~7u;
            items += w.items;
            desc_host[slot + g.secs.size()] = w;
            g.secs.push_back(w);
            g.lds = std::max(g.lds, r->job.lds);
            ids.push_back(r->id);
        }
        g.grid = int(block);
        g.items = int(items);
        // equal R and 256-byte aligned blocks give every member the same chunks
        g.chunks = reqs[0]->job.chunks;
        g.dev_secs = desc + slot;
        g.queue = queue();
        slot += reqs.size();
        jobs.push_back(std::move(g));
    }
    // the pinned staging is rewritten only after the previous round's
    // synchronization, so the copy below never races a pending one
    if (ids != desc_ids) {
        HIP_CHECK(hipMemcpyAsync(desc, desc_host, slot * sizeof(SecWork), hipMemcpyHostToDevice, stream));
        desc_ids = ids;
    }
    const int nsteps = opts.steps_per_round > 0 ? opts.steps_per_round : kServerDefaultSteps;
    for (int k = 0; k < nsteps; ++k)
        for (const LanczosJob& g : jobs)
            if (int rc = job_steps(g, stream, true, 1)) return rc;
    // read back every active request's count of running chains
    for (size_t i = 0; i < active.size(); ++i)
        HIP_CHECK(hipMemcpyAsync(&state_host[2 * i], active[i]->job.secs[0].state, 2 * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    for (size_t i = 0; i < active.size(); ++i) active[i]->last_active = state_host[2 * i + 1];
    rounds.fetch_add(1);
    peak.store(heap.peak);
    return FTLM_OK;
}

void ftlm_server::run() {
    const size_t desc_bytes = server_header_bytes();
    heap.init(desc_bytes, arena_bytes);
    const size_t max_active = size_t(opts.max_active > 0 ? std::min(opts.max_active, kServerMaxActive)
                                                         : kServerDefaultActive);
    for (;;) {
        // admission, in arrival order
        std::vector<std::shared_ptr<Request>> admit_now;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (active.empty() && waiting.empty() && !stop) cv.wait(lk, [&] { return stop || !waiting.empty(); });
            if (stop && waiting.empty() && active.empty()) return;
            while (!waiting.empty() && active.size() + admit_now.size() < max_active && fatal == FTLM_OK) {
                auto& r = waiting.front();
                size_t off = 0;
                if (!heap.alloc(r->bytes, &off)) break;
                r->off = off;
                admit_now.push_back(r);
                waiting.pop_front();
            }
        }
        for (auto& r : admit_now) {
            const int rc = admit(r);
            if (rc != FTLM_OK) {
                r->status = rc;
                heap.release(r->off, r->bytes);
                r->t_done = now();
                std::lock_guard<std::mutex> lk(mu);
                done[r->id] = r;
                if (rc == FTLM_E_DEVICE) fatal = rc;
                continue;
            }
            active.push_back(r);
        }
        if (active.empty()) {
            if (fatal != FTLM_OK) {
                std::lock_guard<std::mutex> lk(mu);
                for (auto& r : waiting) {
                    r->status = fatal;
                    done[r->id] = r;
                }
                waiting.clear();
            }
            continue;
        }
        const int rc = round();
        std::vector<std::shared_ptr<Request>> keep, finished;
        for (auto& r : active) {
            if (rc != FTLM_OK) {
                r->status = rc;
                finished.push_back(r);
            } else if (r->last_active == 0) {
                finished.push_back(r);
            } else {
                keep.push_back(r);
            }
        }
        for (auto& r : finished) {
            if (rc == FTLM_OK) retire(r);
            else {
                heap.release(r->off, r->bytes);
                r->t_done = now();
            }
        }
        active.swap(keep);
        n_active.store(int32_t(active.size()));
        if (rc != FTLM_OK) fatal = rc;
        std::lock_guard<std::mutex> lk(mu);
        for (auto& r : finished) done[r->id] = r;
    }
}

extern "C" {

int ftlm_server_request_bytes(const ftlm_request* req, int mode, int dtype, size_t* bytes) {
    if (!bytes) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_request(req)) return rc;
    if (int rc = check_dtype(dtype)) return rc;
    ReqLayout L;
    if (int rc = request_layout(req->n_sites, req->n_up, req->R, mode, dtype, L)) return rc;
    *bytes = L.total;
    return ok();
}

int ftlm_server_create(void* arena_dev, size_t arena_bytes, const ftlm_server_opts* opts, ftlm_server** out) {
    if (!arena_dev || !opts || !out) return fail(FTLM_E_INVALID, "null argument");
    *out = nullptr;
    if (opts->mode != FTLM_CLT && opts->mode != FTLM_CR && opts->mode != FTLM_FULL && opts->mode != FTLM_LIN)
        return fail(FTLM_E_INVALID, "mode %d", opts->mode);
    if (int rc = check_dtype(opts->dtype)) return rc;
    if (opts->max_active < 0 || opts->max_active > kServerMaxActive)
        return fail(FTLM_E_RANGE, "max_active %d not in [0, %d]", opts->max_active, kServerMaxActive);
    if (opts->steps_per_round < 0 || opts->steps_per_round > kServerMaxSteps)
        return fail(FTLM_E_RANGE, "steps_per_round %d not in [0, %d]", opts->steps_per_round, kServerMaxSteps);
    if (reinterpret_cast<uintptr_t>(arena_dev) % 256 != 0) return fail(FTLM_E_INVALID, "arena not 256-byte aligned");
    const size_t desc = server_header_bytes();
    if (arena_bytes <= desc) return fail(FTLM_E_NOSPACE, "arena smaller than its descriptor area (%zu bytes)", desc);
    auto* s = new ftlm_server();
    s->arena = static_cast<char*>(arena_dev);
    s->arena_bytes = arena_bytes;
    s->opts = *opts;
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->desc_host), size_t(kServerMaxActive) * sizeof(SecWork));
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&s->state_host), size_t(kServerMaxActive) * 2 * sizeof(int32_t));
    if (e != hipSuccess) {
        if (s->desc_host) (void)hipHostFree(s->desc_host);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(FTLM_E_DEVICE, "server setup: %s", hipGetErrorString(e));
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    s->worker = std::thread([s, dev] {
        (void)hipSetDevice(dev);
        s->run();
    });
    *out = s;
    return ok();
}

int ftlm_server_submit(ftlm_server* s, const ftlm_request* req, uint64_t* id) {
    if (!s || !id) return fail(FTLM_E_INVALID, "null argument");
    if (int rc = check_request(req)) return rc;
    ReqLayout L;
    if (int rc = request_layout(req->n_sites, req->n_up, req->R, s->opts.mode, s->opts.dtype, L)) return rc;
    const size_t usable = s->arena_bytes - server_header_bytes();
    if (L.total > usable)
        return fail(FTLM_E_REJECTED, "request needs %zu bytes, the arena holds %zu", L.total, usable);
    auto r = std::make_shared<Request>();
    r->n_sites = req->n_sites;
    r->n_up = req->n_up;
    r->R = req->R;
    r->M = req->M;
    r->dist = req->dist;
    r->seed = req->seed;
    r->g = req->g;
    r->nT = req->nT;
    r->bi.assign(req->bi, req->bi + req->n_bonds);
    r->bj.assign(req->bj, req->bj + req->n_bonds);
    r->J.assign(req->J, req->J + req->n_bonds);
    if (req->nT > 0) r->T.assign(req->T, req->T + req->nT);
    r->bytes = L.total;
    r->t_submit = s->now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(FTLM_E_INVALID, "server is stopping");
        r->id = s->next_id++;
        s->waiting.push_back(r);
        s->all[r->id] = r;
    }
    s->cv.notify_one();
    *id = r->id;
    return ok();
}

int ftlm_server_poll(ftlm_server* s, uint64_t id, double* E, double* C, double* chi, double* lnZ,
                     ftlm_result_info* info) {
    if (!s) return fail(FTLM_E_INVALID, "null argument");
    std::shared_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->done.find(id);
        if (it == s->done.end()) {
            if (s->all.count(id)) return FTLM_E_AGAIN;
            return fail(FTLM_E_INVALID, "unknown request id %llu", (unsigned long long)id);
        }
        r = it->second;
        s->done.erase(it);
        s->all.erase(id);
    }
    const size_t n = size_t(r->nT);
    if (r->status == FTLM_OK && n) {
        if (E) std::memcpy(E, r->E.data(), n * sizeof(double));
        if (C) std::memcpy(C, r->C.data(), n * sizeof(double));
        if (chi) std::memcpy(chi, r->chi.data(), n * sizeof(double));
        if (lnZ) std::memcpy(lnZ, r->lnZ.data(), n * sizeof(double));
    }
    if (info) {
        info->t_submit = r->t_submit;
        info->t_admit = r->t_admit;
        info->t_done = r->t_done;
        info->status = r->status;
        info->steps = r->steps;
        info->dim = binom_u64(r->n_sites, r->n_up);
        info->footprint = r->bytes;
    }
    if (r->status != FTLM_OK) return fail(r->status, "request %llu failed", (unsigned long long)id);
    return ok();
}

double ftlm_server_clock(const ftlm_server* s) { return s ? s->now() : 0.0; }

int ftlm_server_stats(const ftlm_server* s, uint64_t* peak_bytes, uint64_t* rounds, int32_t* active) {
    if (!s) return fail(FTLM_E_INVALID, "null argument");
    if (peak_bytes) *peak_bytes = s->peak.load();
    if (rounds) *rounds = s->rounds.load();
    if (active) *active = s->n_active.load();
    return ok();
}

void ftlm_server_destroy(ftlm_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->desc_host) (void)hipHostFree(s->desc_host);
    if (s->state_host) (void)hipHostFree(s->state_host);
    delete s;
}

}  // extern "C"
