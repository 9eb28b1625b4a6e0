// Sector tables (basis, compressed lookup table) and the index kernels:
// rank, unrank and the neighbour-list test hook.
#include "hv_impl.hpp"

namespace ftlm {

template <typename T>
hipError_t launch_hv_typed(const SectorDev&, const BondTable&, const HvLaunch&, hipStream_t);

hipError_t launch_hv(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    if (s.two_s > 1) return launch_hv_spin(s, B, h, st);
    return h.dtype == 0 ? launch_hv_typed<float>(s, B, h, st) : launch_hv_typed<double>(s, B, h, st);
}

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(uint64_t n) {
    uint64_t b = (n + kThreads - 1) / kThreads;
    return unsigned(b > 1048576 ? 1048576 : (b == 0 ? 1 : b));
}

__device__ __forceinline__ uint64_t global_id() {
    return uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ uint64_t global_stride() { return uint64_t(gridDim.x) * blockDim.x; }

// Number of sector labels below x, for any x < 2^N: Alg. 1's sum with the
// terms of positions where the count of remaining up spins has run out
// dropped (they count labels with more up spins than the sector holds).
template <typename L>
__device__ __forceinline__ uint32_t count_below(L x, int n_sites, int n_up, Binom C) {
    uint32_t r = 0;
    int A = n_up;
    for (int p = n_sites - 1; p >= 0 && A >= 0; --p) {
        if ((x >> p) & 1) {
            r += C(p, A);
            A -= 1;
        }
    }
    return r;
}

// basis[t] = the t-th sector label (one unrank per state).
__global__ __launch_bounds__(kThreads) void build_basis_kernel(SectorDev S, uint32_t* basis) {
    extern __shared__ uint32_t lds[];
    stage_binomials(lds, S.binom, S.n_sites * S.bw);
    const Binom C{lds, S.bw};
    for (uint64_t t = global_id(); t < S.dim; t += global_stride())
        basis[t] = cr_unrank<uint32_t>(uint32_t(t), S.n_sites, S.n_up, C);
}

// One compressed-lookup-table block per thread (Eqs. 18-19): the mask bit j
// is set when label 32b + j lies in the sector (n_up up spins, below 2^N),
// and the prefix count is the number of sector labels below 32b (Eq. 18's
// running sum of block popcounts, here counted directly so every block is
// independent).
__global__ __launch_bounds__(kThreads) void build_clt_kernel(SectorDev S, CltEntry* clt, uint64_t nblocks) {
    extern __shared__ uint32_t lds[];
    stage_binomials(lds, S.binom, S.n_sites * S.bw);
    const Binom C{lds, S.bw};
    const uint64_t limit = uint64_t(1) << S.n_sites;
    for (uint64_t b = global_id(); b < nblocks; b += global_stride()) {
        uint32_t mask = 0;
        for (uint32_t j = 0; j < 32; ++j) {
            const uint64_t label = b * 32 + j;
            if (label < limit && __popcll(label) == S.n_up) mask |= 1u << j;
        }
        clt[b].mask = mask;
        clt[b].prefix = count_below<uint64_t>(b * 32, S.n_sites, S.n_up, C);
    }
}

// The full lookup table (Sec. 2): for every label of [0, 2^N) its sector
// index (the count of sector labels below it) or kNone32.
__global__ __launch_bounds__(kThreads) void build_full_kernel(SectorDev S, uint32_t* full) {
    extern __shared__ uint32_t lds[];
    stage_binomials(lds, S.binom, S.n_sites * S.bw);
    const Binom C{lds, S.bw};
    const uint64_t limit = uint64_t(1) << S.n_sites;
    for (uint64_t x = global_id(); x < limit; x += global_stride())
        full[x] = __popcll(x) == S.n_up ? count_below<uint64_t>(x, S.n_sites, S.n_up, C) : kNone32;
}

// Lin's two tables over the split label = (high part h, low part l of L
// bits): hi[h] = the number of sector labels below h * 2^L (the ones whose
// high part is smaller), lo[l] = the rank of l among the L-bit strings with
// popcount(l) up spins (Alg. 1 over the L low positions). A sector label
// (h, l) then has index hi[h] + lo[l], ascending order preserved. Low parts
// with more up spins than the sector holds never occur; they get 0.
__global__ __launch_bounds__(kThreads) void build_lin_kernel(SectorDev S, uint32_t* hi, uint32_t* lo) {
    extern __shared__ uint32_t lds[];
    stage_binomials(lds, S.binom, S.n_sites * S.bw);
    const Binom C{lds, S.bw};
    const int L = S.lin_lo_bits;
    const uint64_t nhi = uint64_t(1) << (S.n_sites - L), nlo = uint64_t(1) << L;
    for (uint64_t h = global_id(); h < nhi; h += global_stride())
        hi[h] = count_below<uint64_t>(h << L, S.n_sites, S.n_up, C);
    for (uint64_t l = global_id(); l < nlo; l += global_stride()) {
        const int k = __popcll(l);
        lo[l] = k <= S.n_up ? cr_rank<uint64_t>(l, L, k, C) : 0u;
    }
}

template <typename L>
__global__ __launch_bounds__(kThreads) void rank_kernel(SectorDev S, const uint64_t* labels, uint64_t* idx,
                                                        uint64_t n) {
    extern __shared__ uint32_t lds[];
    if (S.mode == kModeCr) stage_binomials(lds, S.binom, S.n_sites * S.bw);
    const Binom C{lds, S.bw};
    for (uint64_t i = global_id(); i < n; i += global_stride()) {
        const uint64_t x = labels[i];
        uint64_t out = ~uint64_t(0);
        const bool in_space = S.n_sites >= 64 || (x >> S.n_sites) == 0;
        if (in_space) {
            if (S.mode == kModeClt) {
                const uint32_t r = clt_lookup(S.clt, uint32_t(x));
                if (r != kNone32) out = r;
            } else if (S.mode == kModeFull) {
                const uint32_t r = S.full[x];
                if (r != kNone32) out = r;
            } else if (__popcll(x) == S.n_up) {
                if (S.mode == kModeLin) {
                    const TableMap<kModeLin> m{S.lin_hi, S.lin_lo, S.lin_lo_bits};
                    out = m.index(m.fetch(uint32_t(x)), uint32_t(x));
                } else {
                    out = cr_rank<L>(L(x), S.n_sites, S.n_up, C);
                }
            }
        }
        idx[i] = out;
    }
}

template <typename L>
__global__ __launch_bounds__(kThreads) void unrank_kernel(SectorDev S, const uint64_t* idx, uint64_t* labels,
                                                          uint64_t n) {
    extern __shared__ uint32_t lds[];
    if (S.mode == kModeCr) stage_binomials(lds, S.binom, S.n_sites * S.bw);
    const Binom C{lds, S.bw};
    for (uint64_t i = global_id(); i < n; i += global_stride()) {
        const uint64_t t = idx[i];
        uint64_t out = ~uint64_t(0);
        if (t < S.dim) {
            if (S.mode != kModeCr) out = S.basis[t];
            else out = uint64_t(cr_unrank<L>(uint32_t(t), S.n_sites, S.n_up, C));
        }
        labels[i] = out;
    }
}

// Writes the partner index of every (row, bond) in the caller's bond order,
// through the same row visitor the H.x kernels use.
struct NeighborVisitor {
    uint64_t* out;
    const BondTable& B;
    static constexpr int kGroup = 2;
    static constexpr bool kPairs = false;
    __device__ __forceinline__ void flip(int b, uint32_t idx) { out[B.orig(b)] = idx; }
    __device__ __forceinline__ void par(int b) { out[B.orig(b)] = ~uint64_t(0); }
    __device__ __forceinline__ void group(int b0, const uint32_t (&idx)[kGroup], const bool (&anti)[kGroup]) {
#pragma unroll
        for (int g = 0; g < kGroup; ++g) out[B.orig(b0 + g)] = anti[g] ? uint64_t(idx[g]) : ~uint64_t(0);
    }
};

template <typename L, int MODE>
__global__ __launch_bounds__(kBlock) void neighbors_kernel(SectorDev S, BondTable B, uint64_t t0, uint64_t count,
                                                           uint64_t* out) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t* binom_lds = reinterpret_cast<uint32_t*>(smem + hv_red_bytes());
    uint32_t* slabs = binom_lds + ((S.n_sites * S.bw + 3) & ~3);
    if constexpr (MODE == kModeCr) stage_binomials(binom_lds, S.binom, S.n_sites * S.bw);
    const Binom C{binom_lds, S.bw};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t* ylds = slabs + wave * S.n_sites * 64 + lane;
    for (uint64_t r = global_id(); r < count; r += global_stride()) {
        NeighborVisitor v{out + r * uint64_t(B.n_bonds), B};
        visit_row<L, MODE>(uint32_t(t0 + r), S.n_up, B, C, S.basis, table_map<MODE>(S), ylds, v);
    }
}

}  // namespace

hipError_t launch_build_basis(const SectorDev& s, hipStream_t st) {
    const size_t lds = size_t(s.n_sites) * s.bw * 4;
    hipLaunchKernelGGL(build_basis_kernel, dim3(blocks_for(s.dim)), dim3(kThreads), lds, st, s,
                       const_cast<uint32_t*>(s.basis));
    return hipGetLastError();
}

hipError_t launch_build_clt(const SectorDev& s, hipStream_t st) {
    const size_t lds = size_t(s.n_sites) * s.bw * 4;
    const uint64_t nb = clt_blocks(s.n_sites);
    hipLaunchKernelGGL(build_clt_kernel, dim3(blocks_for(nb)), dim3(kThreads), lds, st, s,
                       const_cast<CltEntry*>(s.clt), nb);
    return hipGetLastError();
}

hipError_t launch_build_full(const SectorDev& s, hipStream_t st) {
    const size_t lds = size_t(s.n_sites) * s.bw * 4;
    hipLaunchKernelGGL(build_full_kernel, dim3(blocks_for(uint64_t(1) << s.n_sites)), dim3(kThreads), lds, st, s,
                       const_cast<uint32_t*>(s.full));
    return hipGetLastError();
}

hipError_t launch_build_lin(const SectorDev& s, hipStream_t st) {
    const size_t lds = size_t(s.n_sites) * s.bw * 4;
    const uint64_t n = uint64_t(1) << (s.n_sites - s.lin_lo_bits > s.lin_lo_bits ? s.n_sites - s.lin_lo_bits
                                                                                  : s.lin_lo_bits);
    hipLaunchKernelGGL(build_lin_kernel, dim3(blocks_for(n)), dim3(kThreads), lds, st, s,
                       const_cast<uint32_t*>(s.lin_hi), const_cast<uint32_t*>(s.lin_lo));
    return hipGetLastError();
}

hipError_t launch_rank(const SectorDev& s, const uint64_t* labels, uint64_t* idx, uint64_t n,
                       hipStream_t st) {
    const size_t lds = size_t(s.n_sites) * s.bw * 4;
    if (s.n_sites > 32)
        hipLaunchKernelGGL(rank_kernel<uint64_t>, dim3(blocks_for(n)), dim3(kThreads), lds, st, s, labels, idx, n);
    else
        hipLaunchKernelGGL(rank_kernel<uint32_t>, dim3(blocks_for(n)), dim3(kThreads), lds, st, s, labels, idx, n);
    return hipGetLastError();
}

hipError_t launch_unrank(const SectorDev& s, const uint64_t* idx, uint64_t* labels, uint64_t n,
                         hipStream_t st) {
    const size_t lds = size_t(s.n_sites) * s.bw * 4;
    if (s.n_sites > 32)
        hipLaunchKernelGGL(unrank_kernel<uint64_t>, dim3(blocks_for(n)), dim3(kThreads), lds, st, s, idx, labels, n);
    else
        hipLaunchKernelGGL(unrank_kernel<uint32_t>, dim3(blocks_for(n)), dim3(kThreads), lds, st, s, idx, labels, n);
    return hipGetLastError();
}

hipError_t launch_neighbors(const SectorDev& s, const BondTable& B, uint64_t t0, uint64_t count,
                            uint64_t* out, hipStream_t st) {
    const size_t lds = hv_lds_bytes(s);
    const dim3 grid(blocks_for(count)), block(kBlock);
    if (s.mode == kModeClt)
        hipLaunchKernelGGL((neighbors_kernel<uint32_t, kModeClt>), grid, block, lds, st, s, B, t0, count, out);
    else if (s.mode == kModeFull)
        hipLaunchKernelGGL((neighbors_kernel<uint32_t, kModeFull>), grid, block, lds, st, s, B, t0, count, out);
    else if (s.mode == kModeLin)
        hipLaunchKernelGGL((neighbors_kernel<uint32_t, kModeLin>), grid, block, lds, st, s, B, t0, count, out);
    else if (s.n_sites > 32)
        hipLaunchKernelGGL((neighbors_kernel<uint64_t, kModeCr>), grid, block, lds, st, s, B, t0, count, out);
    else
        hipLaunchKernelGGL((neighbors_kernel<uint32_t, kModeCr>), grid, block, lds, st, s, B, t0, count, out);
    return hipGetLastError();
}

}  // namespace ftlm
