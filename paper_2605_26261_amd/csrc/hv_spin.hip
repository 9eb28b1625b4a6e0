// General-spin kernels (local spin s = two_s / 2 > 1/2; Sec. 2, Eqs. 11-17):
// the matrix-free multi-vector H.x (plain and with the Lanczos epilogue),
// the sector tables (basis, compressed lookup table over the d^N labels) and
// the index kernels (rank, unrank, neighbour lists). The spin-1/2 sectors
// keep their own kernels (hv_impl.hpp, sector.hip).
#include "hv_impl.hpp"
#include "spin.hpp"

namespace ftlm {

namespace {

// LDS of the general-spin row kernels (hv_spin_lds_bytes): FP64 scratch,
// ladder factors fu[a] = sqrt(s(s+1) - m(m+1)) (m = a - s) in FP64 and FP32,
// the cumulative dimension table (CR) or the powers d^p (CLT), and (CR) the
// two [site][lane] slabs Y_{+1}, Y_{-1} of each wave.
struct SpinLds {
    double* red;
    double* fu_d;
    float* fu_f;
    uint32_t* table;
    uint32_t* yp;
    uint32_t* ym;
};

__device__ __forceinline__ void stage_spin_table(uint32_t* dst, const SectorDev& S, int mode) {
    if (mode == kModeCr) {
        const int count = S.n_sites * S.bw * (S.two_s + 1);
        for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = *gptr(S.binom + i);
    } else if (threadIdx.x < unsigned(S.n_sites)) {
        uint32_t p = 1;
        for (unsigned k = 0; k < threadIdx.x; ++k) p *= uint32_t(S.two_s + 1);
        dst[threadIdx.x] = p;
    }
}

// Lays out and fills the LDS (visible after the caller's next barrier).
template <int MODE>
__device__ __forceinline__ SpinLds spin_lds_setup(unsigned char* smem, const SectorDev& S) {
    SpinLds l;
    l.red = reinterpret_cast<double*>(smem);
    l.fu_d = reinterpret_cast<double*>(smem + hv_red_bytes());
    l.fu_f = reinterpret_cast<float*>(smem + hv_red_bytes() + 64);
    l.table = reinterpret_cast<uint32_t*>(smem + hv_red_bytes() + 96);
    uint32_t* slabs = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(l.table) +
                                                  hv_spin_table_lds_bytes(S));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    l.yp = slabs + size_t(wave) * 2 * S.n_sites * 64 + lane;
    l.ym = l.yp + S.n_sites * 64;
    if (threadIdx.x < 8) {
        const double s = 0.5 * S.two_s, m = double(threadIdx.x) - s;
        const double v = s * (s + 1.0) - m * (m + 1.0);
        const double f = (int(threadIdx.x) <= S.two_s && v > 0.0) ? sqrt(v) : 0.0;
        l.fu_d[threadIdx.x] = f;
        l.fu_f[threadIdx.x] = float(f);
    }
    stage_spin_table(l.table, S, MODE);
    return l;
}

// Accumulates one row: the diagonal sum_b J_b m_lo m_hi and, per valid ladder
// term, (J_b / 2) * f * x[partner] (Eqs. 12-14). Partner indices are clamped
// into [0, D) like the spin-1/2 visitor's.
template <typename T, int VB, int SB = 1>
struct SpinGather {
    // column col0 of row 0 of x as bytes and the row stride in bytes, as in
    // the spin-1/2 visitor: one multiply-add per partner address
    const unsigned char* __restrict__ xb;
    uint32_t ldb;
    uint32_t last;
    const BondTable& B;
    T (&acc)[VB];
    T& dsum;
    __device__ __forceinline__ void diag(int b, T mm) { dsum += T(2) * bond_coef<T>(B, b) * mm; }
    __device__ __forceinline__ const T* row(uint32_t i) const {
        return reinterpret_cast<const T*>(xb + uint64_t(i) * ldb);
    }
    __device__ __forceinline__ void flip(int b, int, uint32_t idx, T f) {
        const T c = bond_coef<T>(B, b) * f;
        T v[VB];
        idx = idx < last ? idx : last;
        load_row<T, VB>(row(idx), v);
#pragma unroll
        for (int i = 0; i < VB; ++i) acc[i] += c * v[i];
    }
    // CR: two slots, each with the ladder terms of SB bonds, in flight
    // (spin_cr_row_pairs) at every width (SB = spin_slot_bonds). Against one
    // flip at a time, icosahedron M = 0: s = 5/2, one column 12.9 -> 8.4 ms;
    // s = 3, 8 columns 186 -> 165 ms.
    // CLT: the terms of kGroup bonds per group (spin_clt_row_groups); group
    // sizes of 1 to 4 bonds timed at s = 5/2 (one column: 9.1, 8.0, 7.4 and
    // 7.6 ms; 8 columns, Lanczos step: 30.3, 27.8, 26.3 and 26.7 ms; at 2 and
    // 4 columns two bonds were best or within 3 %).
    static constexpr bool kPairs = true;
    static constexpr int kSlotBonds = SB;
    static constexpr int kGroup = (VB == 1 || VB == 8) ? 3 : 2;
    // The two slots of kSlotBonds bonds: rows of x and their weights (J_b / 2
    // times the ladder factors for an existing term, else 0); term k is bond
    // b0 + k / 2. A missing term loads row 0.
    static constexpr int kTerms = 2 * kSlotBonds;
    T slot_a[kTerms][VB], slot_b[kTerms][VB];
    T w_a[kTerms], w_b[kTerms];
    __device__ __forceinline__ void clear_slots() {
#pragma unroll
        for (int g = 0; g < kTerms; ++g) {
            w_a[g] = w_b[g] = T(0);
#pragma unroll
            for (int i = 0; i < VB; ++i) slot_a[g][i] = slot_b[g][i] = T(0);
        }
    }
    __device__ __forceinline__ void load_slot(T (&slot)[kTerms][VB], T (&w)[kTerms], int b0,
                                              const uint32_t (&idx)[kTerms], const bool (&on)[kTerms],
                                              const T (&f)[kTerms]) {
#pragma unroll
        for (int g = 0; g < kTerms; ++g) {
            const uint32_t c = idx[g] < last ? idx[g] : last;
            load_row<T, VB>(row(on[g] ? c : 0u), slot[g]);
            const T cb = bond_coef<T>(B, b0 + g / 2);
            w[g] = on[g] ? cb * f[g] : T(0);
        }
    }
    __device__ __forceinline__ void add_slot(const T (&slot)[kTerms][VB], const T (&w)[kTerms]) {
#pragma unroll
        for (int g = 0; g < kTerms; ++g) {
#pragma unroll
            for (int i = 0; i < VB; ++i) acc[i] += w[g] * slot[g][i];
        }
    }
    __device__ __forceinline__ void load_slot_a(int b0, const uint32_t (&idx)[kTerms], const bool (&on)[kTerms],
                                                const T (&f)[kTerms]) {
        load_slot(slot_a, w_a, b0, idx, on, f);
    }
    __device__ __forceinline__ void load_slot_b(int b0, const uint32_t (&idx)[kTerms], const bool (&on)[kTerms],
                                                const T (&f)[kTerms]) {
        load_slot(slot_b, w_b, b0, idx, on, f);
    }
    __device__ __forceinline__ void add_slot_a() { add_slot(slot_a, w_a); }
    __device__ __forceinline__ void add_slot_b() { add_slot(slot_b, w_b); }
    // kGroup bonds b0, b0 + 1, ...: term k is bond b0 + k / 2, e = +1 for
    // even k; rows of the existing terms are loaded together, the others
    // stay zero under weight zero.
    __device__ __forceinline__ void group(int b0, const uint32_t (&idx)[2 * kGroup], const bool (&on)[2 * kGroup],
                                          const T (&f)[2 * kGroup]) {
        T v[2 * kGroup][VB];
#pragma unroll
        for (int k = 0; k < 2 * kGroup; ++k) {
#pragma unroll
            for (int i = 0; i < VB; ++i) v[k][i] = T(0);
            if (on[k]) load_row<T, VB>(row(idx[k] < last ? idx[k] : last), v[k]);
        }
#pragma unroll
        for (int k = 0; k < 2 * kGroup; ++k) {
            const T c = on[k] ? bond_coef<T>(B, b0 + k / 2) * f[k] : T(0);
#pragma unroll
            for (int i = 0; i < VB; ++i) acc[i] += c * v[k][i];
        }
    }
};

template <typename T>
__device__ __forceinline__ const T* ladder_factors(const SpinLds& l) {
    if constexpr (sizeof(T) == 4) return reinterpret_cast<const T*>(l.fu_f);
    else return reinterpret_cast<const T*>(l.fu_d);
}

template <int MODE, typename T, typename V>
__device__ __forceinline__ void spin_row(uint32_t t, const SectorDev& S, const BondTable& B, const SpinLds& l,
                                         V& v) {
    const T* fu = ladder_factors<T>(l);
    if constexpr (MODE == kModeCr) {
        const CumDim D{l.table, S.bw, S.two_s + 1};
        if constexpr (V::kPairs) spin_cr_row_pairs<T>(t, S.n_up, S.two_s, B, D, fu, l.yp, l.ym, v);
        else spin_cr_row<T>(t, S.n_up, S.two_s, B, D, fu, l.yp, l.ym, v);
    } else {
        const double inv_d = 1.0 / double(S.two_s + 1);
        if constexpr (V::kGroup > 0) spin_clt_row_groups<T>(t, S.two_s, B, S.basis, S.clt, l.table, fu, inv_d, v);
        else spin_clt_row<T>(t, S.two_s, B, S.basis, S.clt, l.table, fu, inv_d, v);
    }
}

// Bonds per slot of the two-slot CR pipeline (icosahedron, s = 5/2, M = 0):
// two bonds took the 8-column Lanczos step from 25.7 to 23.8 ms but the plain
// H.x at one column from 8.46 to 8.64 ms and at 8 columns from 22.9 to 23.9.
constexpr int spin_slot_bonds(int vb, int epi) { return (vb == 8 && epi == kEpiLanczos) ? 2 : 1; }

// Rows [row0, row0 + nrows) of y = H x (columns [col0, col0 + VB) of [D][ld]
// blocks) over the tiles of block `bid` of a (sub-)grid of G blocks, with the
// Lanczos epilogue of hv_body (w = hv_a H u_k - hv_b u_{k-1} and the FP64
// <u_k, w> sums per wave in wsum).
template <int MODE, typename T, int VB, int EPI>
__device__ __forceinline__ void hv_spin_body(const SectorDev& S, const BondTable& B, const SpinLds& l,
                                             const T* __restrict__ x, T* __restrict__ y, uint64_t ld, uint32_t col0,
                                             uint32_t row0, uint32_t nrows, uint32_t bid, uint32_t G, const T* ab,
                                             bool first, double* wsum) {
    const int wave = threadIdx.x >> 6;
    const uint32_t ntiles = (nrows + kBlock - 1) / kBlock;
    for_each_tile(ntiles, bid, G, [&](uint32_t tile) {
        const uint32_t r = tile * kBlock + threadIdx.x;
        const bool valid = r < nrows;
        T xt[VB], out[VB];
        if (valid) {
            const uint32_t t = row0 + r;
            T acc[VB];
#pragma unroll
            for (int c = 0; c < VB; ++c) acc[c] = T(0);
            T diag = T(0);
            SpinGather<T, VB, spin_slot_bonds(VB, EPI)> vis{reinterpret_cast<const unsigned char*>(x + col0),
                                                            uint32_t(ld * sizeof(T)), S.dim - 1, B, acc, diag};
            spin_row<MODE, T>(t, S, B, l, vis);
            load_row<T, VB>(x + uint64_t(t) * ld + col0, xt);
#pragma unroll
            for (int c = 0; c < VB; ++c) out[c] = diag * xt[c] + acc[c];
            T* yrow = y + uint64_t(r) * ld + col0;
            if constexpr (EPI == kEpiLanczos) {
                T z[VB];
                if (!first) {
                    load_row<T, VB>(yrow, z);
                } else {
#pragma unroll
                    for (int c = 0; c < VB; ++c) z[c] = T(0);
                }
#pragma unroll
                for (int c = 0; c < VB; ++c) out[c] = ab[c] * out[c] - ab[VB + c] * z[c];
            }
            store_row<T, VB>(yrow, out);
        }
        if constexpr (EPI == kEpiLanczos) {
            double p[VB];
#pragma unroll
            for (int c = 0; c < VB; ++c) p[c] = valid ? double(xt[c]) * double(out[c]) : 0.0;
            wave_fold_columns<VB>(p, wsum + wave * VB);
        }
    });
}

template <int MODE, typename T, int VB>
__global__ __launch_bounds__(kBlock) void hv_spin_kernel(SectorDev S, BondTable B, HvLaunch h) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BondTable Bs;
    stage_bonds(Bs, &B);
    const SpinLds l = spin_lds_setup<MODE>(smem, S);
    __syncthreads();
    hv_spin_body<MODE, T, VB, kEpiPlain>(S, Bs, l, static_cast<const T*>(h.x), static_cast<T*>(h.y), h.ld, h.col0,
                                         h.row0, h.nrows, blockIdx.x, gridDim.x, nullptr, false, nullptr);
}

// First half of a Lanczos step over the sectors of the launch, as
// hv_lanczos_kernel does it for spin 1/2: a persistent grid taking
// (sector, item) pairs from the per-XCD queue, partials in per-item slots,
// alpha summed by the last workgroup to leave.
template <int MODE, typename T, int VB>
__global__ __launch_bounds__(kBlock) void hv_spin_lanczos_kernel(LanczosLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int flag;
    __shared__ uint32_t next;
    __shared__ BondTable B;
    __shared__ T ab[2 * VB];
    const SecWork* secs = a.secs;
    const uint32_t xcd = blockIdx.x & 7u;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.queue + xcd, 1u);
        __syncthreads();
        uint32_t local = 0;
        const int s = queue_item(secs, a.nsec, xcd, next, &local);
        __syncthreads();  // every thread has read `next`
        if (s < 0) break;
        const SecWork& sw = secs[s];
        if (sw.state[1] == 0) continue;
        const int step = sw.state[0];
        const SectorDev S = sw.S;
        stage_bonds(B, sw.bonds);
        stage_epilogue<T, VB>(ab, sw.chains + a.col0);
        const SpinLds l = spin_lds_setup<MODE>(smem, S);
        double* wsum = l.red;
        for (int i = threadIdx.x; i < kWaves * VB; i += kBlock) wsum[i] = 0.0;
        __syncthreads();
        const T* x = static_cast<const T*>(sw.u[(step - 1) & 1]);
        T* y = static_cast<T*>(sw.u[step & 1]);
        hv_spin_body<MODE, T, VB, kEpiLanczos>(S, B, l, x, y, a.ld, a.col0, 0, S.dim, local, sw.items, ab,
                                               step == 1, wsum);
        store_partials<VB>(sw, a, wsum, local);
        __syncthreads();  // LDS (bonds, scalars, tables) is restaged by the next item
    }
    if (queue_exit(a.queue, gridDim.x, &flag)) {
        double* red = reinterpret_cast<double*>(smem);
        for (int s = 0; s < a.nsec; ++s)
            if (secs[s].state[1] != 0) finish_alpha<VB>(secs[s], a, secs[s].items, red);
    }
}

template <typename F>
hipError_t with_spin_vb(int vb, F&& f) {
    switch (vb) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        default: return hipErrorInvalidValue;
    }
}

template <typename K>
hipError_t allow_lds(K kern, size_t lds) {
    if (lds > 65536)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(lds));
    return hipSuccess;
}

// ---- sector tables and index kernels -----------------------------------------

constexpr int kThreads = 256;

inline unsigned blocks_for(uint64_t n) {
    uint64_t b = (n + kThreads - 1) / kThreads;
    return unsigned(b > 1048576 ? 1048576 : (b == 0 ? 1 : b));
}

__device__ __forceinline__ uint64_t gid() { return uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return uint64_t(gridDim.x) * blockDim.x; }

__device__ __forceinline__ uint64_t digits_to_label(uint64_t dig, int n_sites, uint64_t d) {
    uint64_t n = 0;
    for (int p = n_sites - 1; p >= 0; --p) n = n * d + uint64_t(digit_of(dig, p));
    return n;
}

// basis[t] = the t-th sector label (one unrank per state).
__global__ __launch_bounds__(kThreads) void build_basis_spin_kernel(SectorDev S, uint32_t* basis) {
    extern __shared__ uint32_t tab[];
    stage_spin_table(tab, S, kModeCr);
    __syncthreads();
    const CumDim D{tab, S.bw, S.two_s + 1};
    for (uint64_t t = gid(); t < S.dim; t += gstride()) {
        const uint64_t dig = spin_unrank_digits(uint32_t(t), S.n_sites, S.n_up, S.two_s, D);
        basis[t] = uint32_t(digits_to_label(dig, S.n_sites, uint64_t(S.two_s + 1)));
    }
}

// One compressed-lookup-table block of 32 labels per thread (Eqs. 18-19):
// mask bit j is set when label 32b + j < d^N has the sector's digit sum; the
// prefix is the number of sector labels below 32b.
__global__ __launch_bounds__(kThreads) void build_clt_spin_kernel(SectorDev S, CltEntry* clt, uint64_t nblocks) {
    extern __shared__ uint32_t tab[];
    stage_spin_table(tab, S, kModeCr);
    __syncthreads();
    const CumDim D{tab, S.bw, S.two_s + 1};
    const uint32_t d = uint32_t(S.two_s + 1);
    for (uint64_t b = gid(); b < nblocks; b += gstride()) {
        uint32_t mask = 0;
        for (uint32_t j = 0; j < 32; ++j) {
            const uint64_t label = b * 32 + j;
            if (label >= S.n_labels) break;
            int sum = 0;
            (void)label_digits64(label, S.n_sites, d, &sum);
            if (sum == S.n_up) mask |= 1u << j;
        }
        int sum = 0;
        const uint64_t dig = label_digits64(b * 32, S.n_sites, d, &sum);
        clt[b].mask = mask;
        clt[b].prefix = spin_rank_digits(dig, S.n_sites, S.n_up, D);
    }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void rank_spin_kernel(SectorDev S, const uint64_t* labels, uint64_t* idx,
                                                             uint64_t n) {
    extern __shared__ uint32_t tab[];
    if (MODE == kModeCr) stage_spin_table(tab, S, kModeCr);
    __syncthreads();
    const CumDim D{tab, S.bw, S.two_s + 1};
    for (uint64_t i = gid(); i < n; i += gstride()) {
        const uint64_t x = labels[i];
        uint64_t out = ~uint64_t(0);
        if (x < S.n_labels) {
            if (MODE == kModeClt) {
                const uint32_t r = clt_lookup(S.clt, uint32_t(x));
                if (r != kNone32) out = r;
            } else {
                int sum = 0;
                const uint64_t dig = label_digits64(x, S.n_sites, uint32_t(S.two_s + 1), &sum);
                if (sum == S.n_up) out = spin_rank_digits(dig, S.n_sites, S.n_up, D);
            }
        }
        idx[i] = out;
    }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void unrank_spin_kernel(SectorDev S, const uint64_t* idx, uint64_t* labels,
                                                               uint64_t n) {
    extern __shared__ uint32_t tab[];
    if (MODE == kModeCr) stage_spin_table(tab, S, kModeCr);
    __syncthreads();
    const CumDim D{tab, S.bw, S.two_s + 1};
    for (uint64_t i = gid(); i < n; i += gstride()) {
        const uint64_t t = idx[i];
        uint64_t out = ~uint64_t(0);
        if (t < S.dim) {
            if (MODE == kModeClt) {
                out = S.basis[t];
            } else {
                const uint64_t dig = spin_unrank_digits(uint32_t(t), S.n_sites, S.n_up, S.two_s, D);
                out = digits_to_label(dig, S.n_sites, uint64_t(S.two_s + 1));
            }
        }
        labels[i] = out;
    }
}

// Partner indices of every (row, bond, ladder term) through the same row
// functions as the H.x: entry [row][2 b] is the source with a_i + 1, a_j - 1
// and [row][2 b + 1] the one with a_i - 1, a_j + 1, for the caller's bond b
// = (i, j), i < j; FTLM_NONE where the term does not exist.
struct SpinNeighbors {
    uint64_t* out;
    const BondTable& B;
    static constexpr bool kPairs = false;
    static constexpr int kGroup = 0;  // one term at a time
    __device__ __forceinline__ void diag(int, float) {}
    __device__ __forceinline__ void flip(int b, int e, uint32_t idx, float) { out[2 * B.orig(b) + e] = idx; }
};

template <int MODE>
__global__ __launch_bounds__(kBlock) void neighbors_spin_kernel(SectorDev S, BondTable B, uint64_t t0,
                                                                uint64_t count, uint64_t* out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SpinLds l = spin_lds_setup<MODE>(smem, S);
    __syncthreads();
    for (uint64_t r = gid(); r < count; r += gstride()) {
        uint64_t* row = out + r * uint64_t(2 * B.n_bonds);
        for (int k = 0; k < 2 * B.n_bonds; ++k) row[k] = ~uint64_t(0);
        SpinNeighbors v{row, B};
        spin_row<MODE, float>(uint32_t(t0 + r), S, B, l, v);
    }
}

}  // namespace

hipError_t launch_hv_spin(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    const size_t lds = hv_spin_lds_bytes(s);
    auto go = [&](auto tt, auto mm) {
        using T = decltype(tt);
        constexpr int MODE = decltype(mm)::value;
        return with_spin_vb(h.vb, [&](auto vb) {
            auto kern = hv_spin_kernel<MODE, T, decltype(vb)::value>;
            hipError_t e = allow_lds(kern, lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(unsigned(h.grid)), dim3(kBlock), lds, st, s, B, h);
            return hipGetLastError();
        });
    };
    const auto cr = std::integral_constant<int, kModeCr>{};
    const auto clt = std::integral_constant<int, kModeClt>{};
    if (h.dtype == 0) return s.mode == kModeCr ? go(float{}, cr) : go(float{}, clt);
    return s.mode == kModeCr ? go(double{}, cr) : go(double{}, clt);
}

hipError_t launch_hv_lanczos_spin(const LanczosLaunch& a, size_t lds, hipStream_t st) {
    auto go = [&](auto tt, auto mm) {
        using T = decltype(tt);
        constexpr int MODE = decltype(mm)::value;
        return with_spin_vb(a.vb, [&](auto vb) {
            auto kern = hv_spin_lanczos_kernel<MODE, T, decltype(vb)::value>;
            if (!a.queue || a.items <= 0) return hipErrorInvalidValue;  // the queue counters are required
            hipError_t e = allow_lds(kern, lds);
            if (e != hipSuccess) return e;
            int grid = 0;
            e = persistent_grid(reinterpret_cast<const void*>(kern), lds, a.items, &grid);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(kBlock), lds, st, a);
            return hipGetLastError();
        });
    };
    const auto cr = std::integral_constant<int, kModeCr>{};
    const auto clt = std::integral_constant<int, kModeClt>{};
    if (a.dtype == 0) return a.mode == kModeCr ? go(float{}, cr) : go(float{}, clt);
    return a.mode == kModeCr ? go(double{}, cr) : go(double{}, clt);
}

static size_t spin_table_bytes(const SectorDev& s) {
    return size_t(s.n_sites) * size_t(s.bw) * size_t(s.two_s + 1) * 4;
}

hipError_t launch_build_basis_spin(const SectorDev& s, hipStream_t st) {
    hipLaunchKernelGGL(build_basis_spin_kernel, dim3(blocks_for(s.dim)), dim3(kThreads), spin_table_bytes(s), st, s,
                       const_cast<uint32_t*>(s.basis));
    return hipGetLastError();
}

hipError_t launch_build_clt_spin(const SectorDev& s, hipStream_t st) {
    const uint64_t nb = (s.n_labels + 31) / 32;
    hipLaunchKernelGGL(build_clt_spin_kernel, dim3(blocks_for(nb)), dim3(kThreads), spin_table_bytes(s), st, s,
                       const_cast<CltEntry*>(s.clt), nb);
    return hipGetLastError();
}

hipError_t launch_rank_spin(const SectorDev& s, const uint64_t* labels, uint64_t* idx, uint64_t n, hipStream_t st) {
    if (s.mode == kModeCr)
        hipLaunchKernelGGL(rank_spin_kernel<kModeCr>, dim3(blocks_for(n)), dim3(kThreads), spin_table_bytes(s), st, s,
                           labels, idx, n);
    else
        hipLaunchKernelGGL(rank_spin_kernel<kModeClt>, dim3(blocks_for(n)), dim3(kThreads), 0, st, s, labels, idx, n);
    return hipGetLastError();
}

hipError_t launch_unrank_spin(const SectorDev& s, const uint64_t* idx, uint64_t* labels, uint64_t n,
                              hipStream_t st) {
    if (s.mode == kModeCr)
        hipLaunchKernelGGL(unrank_spin_kernel<kModeCr>, dim3(blocks_for(n)), dim3(kThreads), spin_table_bytes(s), st,
                           s, idx, labels, n);
    else
        hipLaunchKernelGGL(unrank_spin_kernel<kModeClt>, dim3(blocks_for(n)), dim3(kThreads), 0, st, s, idx, labels,
                           n);
    return hipGetLastError();
}

hipError_t launch_neighbors_spin(const SectorDev& s, const BondTable& B, uint64_t t0, uint64_t count, uint64_t* out,
                                 hipStream_t st) {
    const size_t lds = hv_spin_lds_bytes(s);
    if (s.mode == kModeCr) {
        hipError_t e = allow_lds(neighbors_spin_kernel<kModeCr>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(neighbors_spin_kernel<kModeCr>, dim3(blocks_for(count)), dim3(kBlock), lds, st, s, B, t0,
                           count, out);
    } else {
        hipError_t e = allow_lds(neighbors_spin_kernel<kModeClt>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(neighbors_spin_kernel<kModeClt>, dim3(blocks_for(count)), dim3(kBlock), lds, st, s, B, t0,
                           count, out);
    }
    return hipGetLastError();
}

}  // namespace ftlm
