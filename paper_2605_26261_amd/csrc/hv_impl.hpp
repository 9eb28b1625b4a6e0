// Matrix-free multi-vector H.x kernel (paper Sec. 2, Eq. 12, row-wise gather
// form), templated on label width, indexing mode, element type, vector block
// width and epilogue. Included by hv_f32.hip and hv_f64.hip.
#pragma once

#include <type_traits>

#include "rowloop.hpp"

namespace ftlm {

// Loads/stores VB consecutive elements with the widest naturally aligned
// vector access (the host only picks a vector width whose alignment holds),
// as global-memory accesses.
template <typename T, int N>
using VecT = T __attribute__((ext_vector_type(N)));

template <typename T, int VB>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&v)[VB]) {
    if constexpr (sizeof(T) == 4 && VB % 4 == 0) {
#pragma unroll
        for (int i = 0; i < VB; i += 4) {
            const VecT<T, 4> q = *(const FTLM_GLOBAL VecT<T, 4>*)(p + i);
            v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
        }
    } else if constexpr (VB % 2 == 0) {
#pragma unroll
        for (int i = 0; i < VB; i += 2) {
            const VecT<T, 2> q = *(const FTLM_GLOBAL VecT<T, 2>*)(p + i);
            v[i] = q.x; v[i + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < VB; ++i) v[i] = *gptr(p + i);
    }
}

template <typename T, int VB>
__device__ __forceinline__ void store_row(T* __restrict__ p, const T (&v)[VB]) {
    if constexpr (sizeof(T) == 4 && VB % 4 == 0) {
#pragma unroll
        for (int i = 0; i < VB; i += 4) {
            const VecT<T, 4> q = {v[i], v[i + 1], v[i + 2], v[i + 3]};
            *(FTLM_GLOBAL VecT<T, 4>*)(p + i) = q;
        }
    } else if constexpr (VB % 2 == 0) {
#pragma unroll
        for (int i = 0; i < VB; i += 2) {
            const VecT<T, 2> q = {v[i], v[i + 1]};
            *(FTLM_GLOBAL VecT<T, 2>*)(p + i) = q;
        }
    } else {
#pragma unroll
        for (int i = 0; i < VB; ++i) *gptr(p + i) = v[i];
    }
}

template <typename T>
__device__ __forceinline__ T bond_coef(const BondTable& B, int b) {
    if constexpr (sizeof(T) == 4) return B.coef_f[b];
    else return B.coef_d[b];
}

// Accumulates the off-diagonal terms of one row: for each antiparallel bond
// the partner's row of x times J_b / 2; `anti` collects sum J_b / 2 over
// those bonds so the diagonal is sum_b J_b/4 - anti (each antiparallel bond
// turns +J_b/4 into -J_b/4).
// A partner index is in [0, D) by construction; it is clamped there anyway so
// that a defect in the index arithmetic shows up as a parity failure and
// never as an access outside x.
// Fourth word of a raw buffer resource on gfx9: data format 32 bits (a zero
// format makes every load return 0), no stride, no swizzle.
constexpr int kBufferWord3 = 0x00020000;

template <typename T, int VB, int SG = 2, bool BUF = false>
struct GatherVisitor {
    static_assert(!BUF || VB == 1, "buffer-resource gathers serve single vectors");
    // Column col0 of row 0 of x as bytes, and the row stride in bytes (at
    // most 64 columns of 8 bytes): a partner row's address is then one
    // 32 x 32 -> 64-bit multiply-add.
    const unsigned char* __restrict__ xb;
    uint32_t ldb;
    uint32_t last;  // D - 1
    // BUF: x is one contiguous vector of fewer than 2^32 bytes, read through
    // this buffer resource with 32-bit byte offsets (one shift per partner
    // instead of the clamp and the 64-bit multiply-add); the hardware's range
    // check returns 0 for an offset past the end, so a defect in the index
    // arithmetic still cannot read outside x.
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ const T* row(uint32_t i) const {
        return reinterpret_cast<const T*>(xb + uint64_t(i) * ldb);
    }
    const BondTable& B;
    T (&acc)[VB];
    T& anti;
    // row i of x into v (i is clamped into [0, D) on the pointer path)
    __device__ __forceinline__ void gather(uint32_t i, T (&v)[VB]) const {
        if constexpr (BUF) {
            if constexpr (sizeof(T) == 4)
                v[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, int(i << 2), 0, 0));
            else
                v[0] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, int(i << 3), 0, 0));
        } else {
            load_row<T, VB>(row(i < last ? i : last), v);
        }
    }
    __device__ __forceinline__ void flip(int b, uint32_t idx) {
        const T c = bond_coef<T>(B, b);
        T v[VB];
        gather(idx, v);
#pragma unroll
        for (int i = 0; i < VB; ++i) acc[i] += c * v[i];
        anti += c;
    }
    __device__ __forceinline__ void par(int) {}
    // CLT: a group of kGroup consecutive bonds: the rows of the antiparallel
    // ones are loaded together (lanes whose bond is parallel load nothing),
    // then accumulated with weight J_b / 2 or zero. Sizes measured per width
    // (Lanczos step at N = 30): 8 at one column (9.0 -> 8.3 ms against 4),
    // 6 at 8 columns, 3 at 12, 2 from 16 up, 4 elsewhere.
    static constexpr int kGroup = VB == 1 ? 8 : VB == 8 ? 6 : VB == 12 ? 3 : VB >= 16 ? 2 : 4;
    // CR: up to 8 columns, the bonds in slots of kSiteGroup = SG (site_group,
    // per width and epilogue) with two slots in flight (cr_bonds_pairs);
    // wider blocks take one bond at a time (flip /
    // par). Lanczos step at N = 30: one column 15.1 -> 9.6 ms; from 10
    // columns up the two slots were slower (12 columns 36.6 -> 41.5 ms):
    // every lane then loads a full row per bond, parallel lanes included,
    // and the kernel is bound by the traffic, not the latency, of its gathers.
    static constexpr bool kPairs = VB <= 8;
    static constexpr int kSiteGroup = SG;
    // The two slots: rows of x and their weights (J_b / 2 for a flip, else 0).
    // Every lane loads, so the loads are not under a branch and the compiler
    // can wait for exactly the older slot: a lane whose bond is parallel
    // loads row 0 (one cache line shared by all such lanes) under weight zero.
    T slot_a[kSiteGroup][VB], slot_b[kSiteGroup][VB];
    T w_a[kSiteGroup], w_b[kSiteGroup];
    __device__ __forceinline__ void clear_slots() {
#pragma unroll
        for (int g = 0; g < kSiteGroup; ++g) {
            w_a[g] = w_b[g] = T(0);
#pragma unroll
            for (int i = 0; i < VB; ++i) slot_a[g][i] = slot_b[g][i] = T(0);
        }
    }
    // A full slot of kSiteGroup bonds b0, b0 + 1, ...
    __device__ __forceinline__ void load_slot(T (&slot)[kSiteGroup][VB], T (&w)[kSiteGroup], int b0,
                                              const uint32_t (&idx)[kSiteGroup], const bool (&flips)[kSiteGroup]) {
#pragma unroll
        for (int g = 0; g < kSiteGroup; ++g) {
            gather(flips[g] ? idx[g] : 0u, slot[g]);
            const T cb = bond_coef<T>(B, b0 + g);
            w[g] = flips[g] ? cb : T(0);
        }
    }
    __device__ __forceinline__ void add_slot(const T (&slot)[kSiteGroup][VB], const T (&w)[kSiteGroup]) {
#pragma unroll
        for (int g = 0; g < kSiteGroup; ++g) {
#pragma unroll
            for (int i = 0; i < VB; ++i) acc[i] += w[g] * slot[g][i];
            anti += w[g];
        }
    }
    __device__ __forceinline__ void load_slot_a(int b0, const uint32_t (&idx)[kSiteGroup],
                                                const bool (&flips)[kSiteGroup]) {
        load_slot(slot_a, w_a, b0, idx, flips);
    }
    __device__ __forceinline__ void load_slot_b(int b0, const uint32_t (&idx)[kSiteGroup],
                                                const bool (&flips)[kSiteGroup]) {
        load_slot(slot_b, w_b, b0, idx, flips);
    }
    __device__ __forceinline__ void add_slot_a() { add_slot(slot_a, w_a); }
    __device__ __forceinline__ void add_slot_b() { add_slot(slot_b, w_b); }
    __device__ __forceinline__ void group(int b0, const uint32_t (&idx)[kGroup], const bool (&flips)[kGroup]) {
        T v[kGroup][VB];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
#pragma unroll
            for (int i = 0; i < VB; ++i) v[g][i] = T(0);
            if (flips[g]) gather(idx[g], v[g]);
        }
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            const T cb = bond_coef<T>(B, b0 + g);
            const T c = flips[g] ? cb : T(0);
#pragma unroll
            for (int i = 0; i < VB; ++i) acc[i] += c * v[g][i];
            anti += c;
        }
    }
};

// LDS layout shared by the H.x kernels: FP64 scratch (kBlock doubles), the
// binomial table (CR), then one [site][lane] slab of Y values per wave (CR).
struct HvLds {
    double* red;
    uint32_t* binom;
    uint32_t* ylds;
};

template <int MODE, bool BINOM = (MODE == kModeCr)>
__device__ __forceinline__ HvLds hv_lds_setup(unsigned char* smem, const SectorDev& S) {
    HvLds l;
    l.red = reinterpret_cast<double*>(smem);
    l.binom = reinterpret_cast<uint32_t*>(smem + hv_red_bytes());
    uint32_t* slabs = l.binom + ((S.n_sites * S.bw + 3) & ~3);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    l.ylds = slabs + wave * S.n_sites * 64 + lane;
    if constexpr (BINOM) stage_binomials(l.binom, S.binom, S.n_sites * S.bw);
    return l;
}

// The rows of one block of a (sub-)grid of G blocks: y = H x on rows
// [row0, row0 + nrows), columns [col0, col0 + VB) of [D][ld] blocks. In the
// Lanczos epilogue y holds u_{k-1} on entry (unless `first`) and receives
// w = hv_a (H u_k) - hv_b u_{k-1} per column (ab = [hv_a | hv_b], VB each); the products u_k[t] w[t] are
// folded, tile by tile, into per-wave FP64 sums wsum[wave * VB + c] (LDS).
// Bonds per slot of the two-slot CR pipeline, timed per width at N = 30 (FP32):
//   1-2 columns: three bonds (plain H.x 7.95 -> 7.78 ms at one column, 8.26 ->
//     7.97 at two; Lanczos step 9.74 -> 9.25 ms at two);
//   4 columns: three in the Lanczos step (12.16 -> 11.78 ms), two in the plain
//     H.x (9.6 against 9.7);
//   8 columns: one in the plain H.x (19.9 -> 17.7 ms), two in the Lanczos step
//     (one gave 23.6 ms against 22.0, three 22.5).
// The slot size changes no partner index and no order of accumulation.
constexpr int site_group(int vb, int epi) {
    if (vb <= 2) return 3;
    if (vb == 4) return epi == kEpiLanczos ? 3 : 2;
    if (vb == 8) return epi == kEpiPlain ? 1 : 2;
    return 2;
}

template <typename L, int MODE, typename T, int VB, int EPI, bool BUF = false>
__device__ __forceinline__ void hv_body(const SectorDev& S, const BondTable& B, const HvLds& lds,
                                        const T* __restrict__ x, T* __restrict__ y, uint64_t ld,
                                        uint32_t col0, uint32_t row0, uint32_t nrows, uint32_t bid,
                                        uint32_t G, const T* ab, bool first, double* wsum) {
    const Binom C{lds.binom, S.bw};
    const int wave = threadIdx.x >> 6;
    const T jsum4 = sizeof(T) == 4 ? T(B.jsum4_f) : T(B.jsum4_d);
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
            T anti = T(0);
            GatherVisitor<T, VB, site_group(VB, EPI), BUF> vis{
                reinterpret_cast<const unsigned char*>(x + col0), uint32_t(ld * sizeof(T)), S.dim - 1,
                __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(x), 0, BUF ? int(uint64_t(S.dim) * sizeof(T)) : 0,
                                                  kBufferWord3),
                B, acc, anti};
            visit_row<L, MODE>(t, S.n_up, B, C, S.basis, table_map<MODE>(S), lds.ylds, vis);
            load_row<T, VB>(x + uint64_t(t) * ld + col0, xt);
            const T diag = jsum4 - anti;
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
                for (int c = 0; c < VB; ++c) {
                    out[c] = ab[c] * out[c] - ab[VB + c] * z[c];
                }
            }
            store_row<T, VB>(yrow, out);
        }
        if constexpr (EPI == kEpiLanczos) {
            // every lane takes part; rows past the end add 0
            double p[VB];
#pragma unroll
            for (int c = 0; c < VB; ++c) p[c] = valid ? double(xt[c]) * double(out[c]) : 0.0;
            wave_fold_columns<VB>(p, wsum + wave * VB);
        }
    });
}

// Every H.x kernel reads its bond table from a copy in a static LDS object:
// the row loop's bond reads become broadcast LDS reads, which lets the
// compiler keep several partner rows in flight per thread (read from kernel
// arguments or through a generic pointer, the table costs scalar or flat
// loads whose waits serialise the gathers). Visible after the caller's next
// barrier.
__device__ __forceinline__ void stage_bonds(BondTable& dst, const BondTable* src) {
    uint32_t* d = reinterpret_cast<uint32_t*>(&dst);
    const uint32_t* w = reinterpret_cast<const uint32_t*>(src);
    for (int i = threadIdx.x; i < int(sizeof(BondTable) / 4); i += kBlock) d[i] = *gptr(w + i);
}

template <typename L, int MODE, typename T, int VB, bool BUF = false>
__global__ __launch_bounds__(kBlock) void hv_kernel(SectorDev S, BondTable B, HvLaunch h) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ BondTable Bs;
    stage_bonds(Bs, &B);
    const HvLds lds = hv_lds_setup<MODE>(smem, S);
    __syncthreads();
    hv_body<L, MODE, T, VB, kEpiPlain, BUF>(S, Bs, lds, static_cast<const T*>(h.x), static_cast<T*>(h.y), h.ld, h.col0,
                                        h.row0, h.nrows, blockIdx.x, gridDim.x, nullptr, false, nullptr);
}

// The epilogue scalars [hv_a | hv_b] of columns [col0, col0 + VB), in the
// vector precision, into LDS; visible after the caller's next barrier.
template <typename T, int VB>
__device__ __forceinline__ void stage_epilogue(T* ab, const Chain* chains) {
    if (threadIdx.x < VB) {
        const Chain* ch = chains + threadIdx.x;
        ab[threadIdx.x] = sizeof(T) == 4 ? T(ch->hv_a_f) : T(ch->hv_a_d);
        ab[VB + threadIdx.x] = sizeof(T) == 4 ? T(ch->hv_b_f) : T(ch->hv_b_d);
    }
}

// The block's FP64 partials of <u_k, w> for its VB columns (wsum: one row of
// VB per wave) into its slot of the sector's partials.
template <int VB>
__device__ __forceinline__ void store_partials(const SecWork& sw, const LanczosLaunch& a, const double* wsum,
                                               uint32_t slot) {
    __syncthreads();
    if (threadIdx.x < VB) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w * VB + threadIdx.x];
        sw.partials[size_t(slot) * a.ld + a.col0 + threadIdx.x] = t;
    }
}

// alpha_k of the launch's columns of one sector from its n partial slots.
template <int VB>
__device__ __forceinline__ void finish_alpha(const SecWork& sw, const LanczosLaunch& a, uint32_t n, double* red) {
    double tot[VB];
    grid_sum_cols<VB>(sw.partials, int(n), int(a.ld), int(a.col0), VB, red, tot);
    if (threadIdx.x == 0) {
        for (int c = 0; c < VB; ++c) {
            Chain* ch = &sw.chains[a.col0 + c];
            ch->alpha = ch->s_cur * tot[c];
            ch->up_d = ch->alpha * ch->s_cur;
            ch->up_f = float(ch->up_d);
        }
    }
}

// First half of Lanczos step k over every sector of the launch (one sector,
// all sectors of a plan, or a server round): w = H q_k - beta_{k-1} q_{k-1}
// and the FP64 partials of <u_k, w>, summed in slot order into alpha_k (and
// the update coefficient). A sector whose chains have all stopped is skipped.
//
// The grid is persistent, sized to the resident workgroups: each workgroup
// takes (sector, item) pairs from its XCD's counter (queue_item) and runs
// them one after the other, and each item stores its partials in its own
// slot with plain stores. The last workgroup to leave (queue_exit, the one
// device-scope fence of each workgroup) sums every sector's slots. Which
// workgroup ran an item changes nothing: the tiles of an item, its partial
// slot and the summation order depend on the sector's dimension only.
template <typename L, int MODE, typename T, int VB>
__global__ __launch_bounds__(kBlock) void hv_lanczos_kernel(LanczosLaunch a) {
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
        const HvLds lds = hv_lds_setup<MODE>(smem, S);
        double* wsum = lds.red;
        for (int i = threadIdx.x; i < kWaves * VB; i += kBlock) wsum[i] = 0.0;
        __syncthreads();
        const T* x = static_cast<const T*>(sw.u[(step - 1) & 1]);
        T* y = static_cast<T*>(sw.u[step & 1]);
        hv_body<L, MODE, T, VB, kEpiLanczos>(S, B, lds, x, y, a.ld, a.col0, 0, S.dim, local, sw.items, ab,
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

// Dynamic LDS of the plain H.x at 20 and more FP32 columns: enough that two
// workgroups fill a CU's 160 KB. Registers would allow six; with more rows in
// flight the partner rows are evicted before their reuse (at N = 30, 20
// columns: 74 -> 69 ms with CLT, 63 -> 58 ms with CR; 32 columns: 218 -> 187
// ms with CLT). Narrower blocks keep the register-limited occupancy.
template <typename T, int VB>
constexpr size_t hv_plain_lds_floor() { return (sizeof(T) == 4 && VB >= 20) ? size_t(72) * 1024 : 0; }

template <typename L, int MODE, typename T, int VB, bool BUF = false>
hipError_t launch_hv_one(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    const size_t need = hv_lds_bytes(s), floor = hv_plain_lds_floor<T, VB>();
    const size_t lds = need > floor ? need : floor;
    auto kern = hv_kernel<L, MODE, T, VB, BUF>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(h.grid)), dim3(kBlock), lds, st, s, B, h);
    return hipGetLastError();
}

// Grid of a persistent launch: the resident workgroups of the kernel at this
// LDS size (a multiple of 8, so every XCD gets the same number), capped at
// the number of work items.
hipError_t persistent_grid(const void* kern, size_t lds, int items, int* grid);

// Dynamic LDS of the Lanczos H.x that holds CR at 8 and 16 FP32 columns to
// three workgroups per CU (their registers allow four) when the vector
// block of the largest sector does not fit the 256 MB Infinity Cache: fewer
// rows in flight keep more of the partner rows cached. N = 30 Lanczos step:
// 8 columns 23.0 -> 22.2 ms, 16 columns 50.9 -> 47.0 ms; the same floor made
// 10 and 12 columns and every CLT width slower.
template <int MODE, typename T, int VB>
size_t lanczos_lds_floor(uint64_t max_dim) {
    const bool big = max_dim * uint64_t(VB) * sizeof(T) > (uint64_t(256) << 20);
    return (MODE == kModeCr && sizeof(T) == 4 && (VB == 8 || VB == 16) && big) ? size_t(48) * 1024 : 0;
}

template <typename L, int MODE, typename T, int VB>
hipError_t launch_lanczos_one(const LanczosLaunch& a, size_t lds, hipStream_t st) {
    auto kern = hv_lanczos_kernel<L, MODE, T, VB>;
    const size_t floor = lanczos_lds_floor<MODE, T, VB>(a.max_dim);
    if (lds < floor) lds = floor;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    if (!a.queue || a.items <= 0) return hipErrorInvalidValue;  // the queue counters are required
    int grid = 0;
    hipError_t e = persistent_grid(reinterpret_cast<const void*>(kern), lds, a.items, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(kBlock), lds, st, a);
    return hipGetLastError();
}

// Dispatch over the vector-block width VB (columns per launch).
template <typename T, typename F>
hipError_t with_vb(int vb, F&& f) {
    switch (vb) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 4: return f(std::integral_constant<int, 4>{});
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 10:
            if constexpr (sizeof(T) == 4) return f(std::integral_constant<int, 10>{});
            else return hipErrorInvalidValue;
        case 12:
            if constexpr (sizeof(T) == 4) return f(std::integral_constant<int, 12>{});
            else return hipErrorInvalidValue;
        case 20:
            if constexpr (sizeof(T) == 4) return f(std::integral_constant<int, 20>{});
            else return hipErrorInvalidValue;
        case 32:
            if constexpr (sizeof(T) == 4) return f(std::integral_constant<int, 32>{});
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

// Dispatch over label width and indexing mode.
template <typename F>
hipError_t with_mode(int mode, int n_sites, F&& f) {
    if (mode == kModeClt) return f(uint32_t{}, std::integral_constant<int, kModeClt>{});
    if (mode == kModeFull) return f(uint32_t{}, std::integral_constant<int, kModeFull>{});
    if (mode == kModeLin) return f(uint32_t{}, std::integral_constant<int, kModeLin>{});
    if (n_sites > 32) return f(uint64_t{}, std::integral_constant<int, kModeCr>{});
    return f(uint32_t{}, std::integral_constant<int, kModeCr>{});
}

// A single contiguous vector of fewer than 2^32 bytes takes the
// buffer-resource gathers (GatherVisitor, BUF) with CR and the compressed
// table. N = 30, one FP32 vector: CR 7.77 -> 7.37 ms, CLT 6.06 -> 5.90; FP64
// CR 8.33 -> 7.96. Lin's tables were 2 % slower and the full table
// unchanged, so they keep the pointer form; reading the compressed table
// through a buffer as well changed nothing.
template <typename T>
hipError_t launch_hv_typed(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    const bool buf = h.vb == 1 && h.ld == 1 && h.col0 == 0 && uint64_t(s.dim) * sizeof(T) < (uint64_t(1) << 32) &&
                     (s.mode == kModeCr || s.mode == kModeClt);
    return with_mode(s.mode, s.n_sites, [&](auto l, auto m) {
        using L = decltype(l);
        constexpr int MODE = decltype(m)::value;
        if constexpr (std::is_same_v<L, uint32_t> && (MODE == kModeCr || MODE == kModeClt))
            if (buf) return launch_hv_one<L, MODE, T, 1, true>(s, B, h, st);
        return with_vb<T>(h.vb, [&](auto vb) { return launch_hv_one<L, MODE, T, decltype(vb)::value>(s, B, h, st); });
    });
}

template <typename T>
hipError_t launch_lanczos_typed(int mode, int n_sites, const LanczosLaunch& a, size_t lds, hipStream_t st) {
    return with_mode(mode, n_sites, [&](auto l, auto m) {
        using L = decltype(l);
        return with_vb<T>(a.vb, [&](auto vb) {
            return launch_lanczos_one<L, decltype(m)::value, T, decltype(vb)::value>(a, lds, st);
        });
    });
}

}  // namespace ftlm
