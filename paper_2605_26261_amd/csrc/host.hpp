// Host-side machinery shared by the C ABI (abi.cpp) and the request server
// (server.cpp). Internal to libftlm.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ftlm.h"
#include "host_math.hpp"
#include "kernels.hpp"

struct ftlm_graph {
    int n_sites = 0;
    std::vector<int> bi, bj;   // merged bonds, caller order of first appearance
    std::vector<double> J;
    int n_input = 0;           // bonds as given (before merging)
    std::vector<int> merged_of_input;
    ftlm::BondTable table{};   // in the caller's site labels
};

struct ftlm_sector {
    int n_sites = 0, n_up = 0, mode = 0;
    int two_s = 1;          // 2s of the local spin; n_up is the digit sum A when two_s > 1
    uint64_t dim = 0;
    void* table = nullptr;
    size_t bytes = 0;
    ftlm::TableLayout layout{};
    std::vector<uint32_t> binom_host;
    ftlm::SectorDev dev{};
};

namespace ftlm {

// Thread-local error text behind ftlm_last_error; fail() records a message and
// returns its code, ok() clears it.
extern thread_local std::string g_err;
int fail(int code, const char* fmt, ...);
int ok();

#define HIP_CHECK(expr)                                                                                \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return ::ftlm::fail(FTLM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

uint64_t binom_u64(int n, int k);

// Weight of a sector in the thermal sums: the sectors +M and -M have the
// same spectrum (Sec. 2), so a sector with M != 0 stands for both.
inline double sector_multiplicity(int n_sites, int n_up) { return 2 * n_up == n_sites ? 1.0 : 2.0; }

// Two timing events destroyed on every exit path.
struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t create() {
        hipError_t e = hipEventCreate(&e0);
        return e == hipSuccess ? hipEventCreate(&e1) : e;
    }
    EventPair() = default;
    EventPair(const EventPair&) = delete;
    EventPair& operator=(const EventPair&) = delete;
    ~EventPair() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Bond tables of the row kernels (bonds.cpp).
BondTable make_bond_table(int n_sites, const std::vector<int>& lo, const std::vector<int>& hi,
                          const std::vector<double>& J, const std::vector<int>& orig, double jsum_all);
constexpr int kTablesPerGraph = 1;  // the graph's bond table
uint64_t stream_key(uint64_t seed, int n_up, uint64_t r);

// ---- stats -------------------------------------------------------------------
struct Stats {
    std::mutex mu;
    bool on = false;
    int64_t launches = 0;
    double ms = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};
extern Stats g_stats;

struct HvTimer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit HvTimer(hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> lk(g_stats.mu);
        if (!g_stats.on) return;
        if (hipEventCreate(&a) != hipSuccess) {
            a = nullptr;
            return;
        }
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, st);
    }
    ~HvTimer() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_stats.mu);
        g_stats.pending.emplace_back(a, b);
    }
};

std::vector<std::pair<int, int>> column_chunks_v(int nvec, uint64_t ld, int dtype, const std::vector<const void*>& ptrs,
                                                 int max_width = 32);
std::vector<std::pair<int, int>> column_chunks(int nvec, uint64_t ld, int dtype, std::initializer_list<const void*> ptrs,
                                               int max_width = 32);
// Widest launch of the H.x kernels of a sector: 8 columns for general spin.
inline int max_launch_width(int two_s) { return two_s > 1 ? 8 : 32; }
int check_dtype(int dtype);

// Byte offsets of one sector's Lanczos state inside a workspace or arena.
struct SectorState {
    size_t u0, u1, partials, chains, alpha, beta, ticket, keys, state;
};
size_t layout_state(uint64_t dim, int R, int dtype, size_t off, SectorState& st);

template <typename P>
P* at(void* base, size_t off) { return reinterpret_cast<P*>(static_cast<char*>(base) + off); }

// A batch of R chains in each of a list of sectors (one sector for
// ftlm_lanczos, all sectors of a plan), with the device descriptors of the
// multi-sector Lanczos kernels. Host copies stay alive until the stream work
// that reads them has been synchronized.
struct LanczosJob {
    int nsec = 0, R = 0, dtype = 0, mode = 0, n_sites = 0, grid = 0, two_s = 1;
    int items = 0;                       // work items of the persistent H.x, all sectors
    size_t lds = 0;
    std::vector<SecWork> secs;           // host copies of the descriptors
    std::vector<uint64_t> keys;          // [nsec][R] stream keys of the run
    SecWork* dev_secs = nullptr;
    std::vector<uint64_t*> key_ptrs;
    std::vector<BondTable> bonds;        // host copies, one per distinct device table
    std::vector<BondTable*> dev_bonds;   // where each copy goes
    std::vector<std::pair<int, int>> chunks;
    int max_steps = 0;                   // largest m_eff over the sectors
    uint32_t* queue = nullptr;           // work-queue counters of the persistent H.x (kQueueBytes)

    LanczosLaunch launch() const {
        LanczosLaunch a{};
        a.secs = dev_secs;
        a.nsec = nsec;
        a.grid = grid;
        a.items = items;
        for (const SecWork& w : secs) a.max_dim = std::max<uint64_t>(a.max_dim, w.S.dim);
        a.ld = uint64_t(R);
        a.dtype = dtype;
        // FP32 vectors: an exact invariant subspace leaves a residual of about
        // 1e-5 of the coefficient scale (FP32 row sums and vector updates), so
        // the threshold sits a factor 10 above it
        a.eps = dtype == FTLM_F32 ? 1e-4 : 1e-12;
        a.mode = mode;
        a.n_sites = n_sites;
        a.two_s = two_s;
        a.queue = queue;
        return a;
    }
};

// Sector i runs with graph graphs[graph_of[i]] (null: no H.x, start vectors
// only), whose kTablesPerGraph bond tables go to dev_tables[graph_of[i]].
void job_layout(LanczosJob& job, const std::vector<SectorDev>& devs, const std::vector<SectorState>& states,
                void* base, int R, int M, int dtype, SecWork* dev_secs, const std::vector<const ftlm_graph*>& graphs,
                const std::vector<BondTable*>& dev_tables, const std::vector<int>& graph_of);
int job_start(LanczosJob& job, uint64_t seed, uint64_t r0, int dist, hipStream_t st);
// The job's columns split into launches of at most max_width columns.
std::vector<std::pair<int, int>> job_chunks(const LanczosJob& job, int max_width);
int job_steps(const LanczosJob& job, hipStream_t st, bool timed = true, int nsteps = -1);
int job_collect(const LanczosJob& job, int M, double* alpha_host, double* beta_host, int32_t* steps_host,
                hipStream_t st);

}  // namespace ftlm
