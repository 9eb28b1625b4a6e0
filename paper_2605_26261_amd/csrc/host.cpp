// Host-side machinery shared by the C ABI and the request server: error
// reporting, sector/graph handles, start-vector keys, H.x timing hooks, column
// chunking and the Lanczos job (one or many sectors, one launch per kernel
// per step).
#include "host.hpp"

#include <cstdarg>
#include <cstdio>

namespace ftlm {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() {
    g_err.clear();
    return FTLM_OK;
}


uint64_t binom_u64(int n, int k) {
    if (n < 0 || k < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 c = 1;
    for (int i = 1; i <= k; ++i) c = c * unsigned(n - k + i) / unsigned(i);
    return uint64_t(c);
}

// ---- start-vector keys: SplitMix64 (Steele, Lea, Flood 2014) --------------
constexpr uint64_t kGammaHost = 0x9e3779b97f4a7c15ull;
uint64_t mix64_host(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
uint64_t first_output(uint64_t s) { return mix64_host(s + kGammaHost); }
// Key of sample r in the sector with n_up up spins.
uint64_t stream_key(uint64_t seed, int n_up, uint64_t r) {
    uint64_t k = first_output(seed);
    k = first_output(k ^ uint64_t(uint32_t(n_up)));
    return first_output(k ^ r);
}




Stats g_stats;

// ---- column chunking of a [D][ld] block --------------------------------------
// Splits columns [0, nvec) into kernel widths of at most max_width, widest
// first, keeping every vector access naturally aligned (ld, col0 and the base
// pointers).
std::vector<std::pair<int, int>> column_chunks_v(int nvec, uint64_t ld, int dtype, const std::vector<const void*>& ptrs,
                                                 int max_width) {
    const size_t es = dtype == FTLM_F32 ? 4 : 8;
    static const int w32[] = {32, 20, 16, 12, 10, 8, 4, 2, 1};
    static const int w64[] = {16, 8, 4, 2, 1};
    const int* widths = dtype == FTLM_F32 ? w32 : w64;
    const int nw = dtype == FTLM_F32 ? 9 : 5;
    std::vector<std::pair<int, int>> out;
    int col = 0;
    while (col < nvec) {
        for (int i = 0; i < nw; ++i) {
            const int vb = widths[i];
            if (vb > nvec - col || (vb > max_width && vb > 1)) continue;
            size_t vbytes = es;
            if (es == 4 && vb % 4 == 0) vbytes = 16;
            else if (vb % 2 == 0) vbytes = 2 * es;
            bool aligned = (ld * es) % vbytes == 0 && (size_t(col) * es) % vbytes == 0;
            for (const void* p : ptrs) aligned = aligned && (reinterpret_cast<uintptr_t>(p) % vbytes == 0);
            if (!aligned) continue;
            out.emplace_back(col, vb);
            col += vb;
            break;
        }
    }
    return out;
}

std::vector<std::pair<int, int>> column_chunks(int nvec, uint64_t ld, int dtype,
                                               std::initializer_list<const void*> ptrs, int max_width) {
    return column_chunks_v(nvec, ld, dtype, std::vector<const void*>(ptrs), max_width);
}

std::vector<std::pair<int, int>> job_chunks(const LanczosJob& job, int max_width) {
    std::vector<const void*> ptrs;
    for (const auto& w : job.secs) {
        ptrs.push_back(w.u[0]);
        ptrs.push_back(w.u[1]);
    }
    return column_chunks_v(job.R, uint64_t(job.R), job.dtype, ptrs, max_width);
}

int check_dtype(int dtype) {
    if (dtype != FTLM_F32 && dtype != FTLM_F64) return fail(FTLM_E_INVALID, "dtype %d is not FTLM_F32/FTLM_F64", dtype);
    return FTLM_OK;
}

// ---- Lanczos state layout -----------------------------------------------------



// Lays out the state of a sector of dimension `dim` at `off`; returns the end.
size_t layout_state(uint64_t dim, int R, int dtype, size_t off, SectorState& st) {
    const size_t es = dtype == FTLM_F32 ? 4 : 8;
    st.u0 = off; off = align256(off + size_t(dim) * size_t(R) * es);
    st.u1 = off; off = align256(off + size_t(dim) * size_t(R) * es);
    const size_t slots = std::max(stream_grid(uint32_t(dim)), sector_items(uint32_t(dim)));
    st.partials = off; off = align256(off + slots * size_t(R) * sizeof(double));
    st.chains = off; off = align256(off + size_t(R) * sizeof(Chain));
    st.alpha = off; off = align256(off + size_t(R) * kMaxSteps * sizeof(double));
    st.beta = off; off = align256(off + size_t(R) * kMaxSteps * sizeof(double));
    st.ticket = off; off = align256(off + sizeof(uint32_t));
    st.keys = off; off = align256(off + size_t(R) * sizeof(uint64_t));
    st.state = off; off = align256(off + 2 * sizeof(int32_t));
    return off;
}



// Fills job.secs for sectors whose tables are described by `devs` and whose
// state sits at `states` inside `base`. Each graph contributes its bond table
// in the caller's labels. The descriptor array goes to `dev_secs`
// (device). Blocks of the static-grid kernels: each sector gets stream_grid(D)
// blocks starting at a multiple of 8; the persistent H.x splits it into
// sector_items(D) work items.
void job_layout(LanczosJob& job, const std::vector<SectorDev>& devs, const std::vector<SectorState>& states,
                void* base, int R, int M, int dtype, SecWork* dev_secs, const std::vector<const ftlm_graph*>& graphs,
                const std::vector<BondTable*>& dev_tables, const std::vector<int>& graph_of) {
    job.nsec = int(devs.size());
    job.R = R;
    job.dtype = dtype;
    job.mode = devs[0].mode;
    job.n_sites = devs[0].n_sites;
    job.two_s = devs[0].two_s > 1 ? devs[0].two_s : 1;
    job.dev_secs = dev_secs;
    job.bonds.clear();
    job.dev_bonds.clear();
    for (size_t gi = 0; gi < graphs.size(); ++gi) {
        const ftlm_graph* g = graphs[gi];
        const BondTable zero{};
        job.bonds.push_back(g ? g->table : zero);
        for (int k = 0; k < kTablesPerGraph; ++k) job.dev_bonds.push_back(dev_tables[gi] + k);
    }
    job.secs.assign(devs.size(), SecWork{});
    job.key_ptrs.clear();
    uint32_t block = 0, items = 0;
    size_t lds = 0;
    job.max_steps = 0;
    for (size_t i = 0; i < devs.size(); ++i) {
        SecWork& w = job.secs[i];
        const SectorState& st = states[i];
        const int gi = graph_of[i];
        w.S = devs[i];
        w.bonds = dev_tables[size_t(gi)];
        w.u[0] = at<void>(base, st.u0);
        w.u[1] = at<void>(base, st.u1);
        w.chains = at<Chain>(base, st.chains);
        w.partials = at<double>(base, st.partials);
        w.ticket = at<uint32_t>(base, st.ticket);
        w.state = at<int32_t>(base, st.state);
        w.alpha = at<double>(base, st.alpha);
        w.beta = at<double>(base, st.beta);
        w.keys = at<uint64_t>(base, st.keys);
        job.key_ptrs.push_back(at<uint64_t>(base, st.keys));
        w.G = stream_grid(devs[i].dim);
        w.items = sector_items(devs[i].dim);
        items += w.items;
        w.block0 = block;
        block = (block + w.G + 7) & ~7u;
        w.m_eff = int(std::min<uint64_t>(uint64_t(M), devs[i].dim));
        job.max_steps = std::max(job.max_steps, w.m_eff);
        lds = std::max(lds, hv_lds_bytes(devs[i]));
    }
    job.grid = int(block);
    job.items = int(items);
    job.lds = lds;
    job.chunks = job_chunks(job, max_launch_width(job.two_s));
}

// Start vectors of samples r0 .. r0 + R - 1 in every sector of the job.
int job_start(LanczosJob& job, uint64_t seed, uint64_t r0, int dist, hipStream_t st) {
    job.keys.resize(size_t(job.nsec) * size_t(job.R));
    for (int s = 0; s < job.nsec; ++s) {
        job.secs[size_t(s)].r0 = r0;
        for (int c = 0; c < job.R; ++c)
            job.keys[size_t(s) * job.R + size_t(c)] = stream_key(seed, job.secs[size_t(s)].S.n_up, r0 + uint64_t(c));
    }
    HIP_CHECK(hipMemcpyAsync(job.dev_secs, job.secs.data(), job.secs.size() * sizeof(SecWork),
                             hipMemcpyHostToDevice, st));
    for (size_t i = 0; i < job.bonds.size(); ++i)
        HIP_CHECK(hipMemcpyAsync(job.dev_bonds[i], &job.bonds[i], sizeof(BondTable), hipMemcpyHostToDevice, st));
    for (int s = 0; s < job.nsec; ++s)
        HIP_CHECK(hipMemcpyAsync(job.key_ptrs[size_t(s)], job.keys.data() + size_t(s) * job.R,
                                 size_t(job.R) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    LanczosLaunch a = job.launch();
    a.dist = dist;
    HIP_CHECK(launch_chain_init(a, st));
    for (int c = 0; c < job.R; c += 4) {
        a.col0 = uint32_t(c);
        a.vb = std::min(4, job.R - c);
        HIP_CHECK(launch_start(a, st));
    }
    return FTLM_OK;
}

// Lanczos steps 1..job.max_steps for every chunk of columns (each sector's
// device step counter advances after its last chunk; sectors whose chains
// have all stopped are skipped by the kernels).
int job_steps(const LanczosJob& job, hipStream_t st, bool timed, int nsteps) {
    LanczosLaunch a = job.launch();
    const int n = nsteps < 0 ? job.max_steps : nsteps;
    for (int k = 1; k <= n; ++k) {
        for (size_t i = 0; i < job.chunks.size(); ++i) {
            a.col0 = uint32_t(job.chunks[i].first);
            a.vb = job.chunks[i].second;
            a.last_chunk = i + 1 == job.chunks.size() ? 1 : 0;
            if (timed) {
                HvTimer timer(st);
                HIP_CHECK(launch_hv_lanczos(a, job.lds, st));
            } else {
                HIP_CHECK(launch_hv_lanczos(a, job.lds, st));
            }
            HIP_CHECK(launch_update(a, st));
        }
    }
    return FTLM_OK;
}

// Copies sector s's coefficients into [R][M] host arrays (after a sync).
int job_collect(const LanczosJob& job, int M, double* alpha_host, double* beta_host, int32_t* steps_host,
                hipStream_t st) {
    const size_t R = size_t(job.R);
    std::vector<double> a(size_t(job.nsec) * R * kMaxSteps), b(a.size());
    std::vector<Chain> ch(size_t(job.nsec) * R);
    for (int s = 0; s < job.nsec; ++s) {
        const SecWork& w = job.secs[size_t(s)];
        HIP_CHECK(hipMemcpyAsync(a.data() + size_t(s) * R * kMaxSteps, w.alpha, R * kMaxSteps * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipMemcpyAsync(b.data() + size_t(s) * R * kMaxSteps, w.beta, R * kMaxSteps * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipMemcpyAsync(ch.data() + size_t(s) * R, w.chains, R * sizeof(Chain), hipMemcpyDeviceToHost, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
    int faulty = -1;
    for (int s = 0; s < job.nsec; ++s) {
        for (size_t r = 0; r < R; ++r) {
            const Chain& c = ch[size_t(s) * R + r];
            if (c.fault && faulty < 0) faulty = int(size_t(s) * R + r);
            const size_t row = size_t(s) * R + r;
            steps_host[row] = c.steps;
            for (int k = 0; k < M; ++k) {
                const bool in = k < c.steps;
                alpha_host[row * size_t(M) + size_t(k)] = in ? a[row * kMaxSteps + size_t(k)] : 0.0;
                beta_host[row * size_t(M) + size_t(k)] = in ? b[row * kMaxSteps + size_t(k)] : 0.0;
            }
        }
    }
    if (faulty >= 0)
        return fail(FTLM_E_NUMERIC, "chain %d of sector %d stopped on a non-finite alpha or beta at step %d",
                    faulty % int(R), faulty / int(R), ch[size_t(faulty)].steps);
    return FTLM_OK;
}

}  // namespace ftlm
