// Matrix-free multi-vector H.x kernel (paper Sec. 2, Eq. 12, row-wise gather
// form), templated on label width, indexing mode, element type, vector block
// width and epilogue. Included by hv_f32.hip and hv_f64.hip.
#pragma once

#include <type_traits>

#include "rowloop.hpp"

namespace ftlm {

// Loads/stores VB consecutive elements with the widest naturally aligned
// vector access (the host only picks a vector width whose alignment holds).
template <typename T, int VB>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&v)[VB]) {
    if constexpr (sizeof(T) == 4 && VB % 4 == 0) {
#pragma unroll
        for (int i = 0; i < VB; i += 4) {
            const float4 q = *reinterpret_cast<const float4*>(p + i);
            v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
        }
    } else if constexpr (VB % 2 == 0) {
        using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
#pragma unroll
        for (int i = 0; i < VB; i += 2) {
            const V2 q = *reinterpret_cast<const V2*>(p + i);
            v[i] = q.x; v[i + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < VB; ++i) v[i] = p[i];
    }
}

template <typename T, int VB>
__device__ __forceinline__ void store_row(T* __restrict__ p, const T (&v)[VB]) {
    if constexpr (sizeof(T) == 4 && VB % 4 == 0) {
#pragma unroll
        for (int i = 0; i < VB; i += 4)
            *reinterpret_cast<float4*>(p + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else if constexpr (VB % 2 == 0) {
        using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
#pragma unroll
        for (int i = 0; i < VB; i += 2) {
            V2 q;
            q.x = v[i]; q.y = v[i + 1];
            *reinterpret_cast<V2*>(p + i) = q;
        }
    } else {
#pragma unroll
        for (int i = 0; i < VB; ++i) p[i] = v[i];
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
template <typename T, int VB>
struct GatherVisitor {
    const T* __restrict__ x;
    uint64_t ld;
    uint32_t col0;
    uint32_t last;  // D - 1
    const BondTable& B;
    T (&acc)[VB];
    T& anti;
    __device__ __forceinline__ void flip(int b, uint32_t idx) {
        const T c = bond_coef<T>(B, b);
        T v[VB];
        idx = idx < last ? idx : last;
        load_row<T, VB>(x + uint64_t(idx) * ld + col0, v);
#pragma unroll
        for (int i = 0; i < VB; ++i) acc[i] += c * v[i];
        anti += c;
    }
    __device__ __forceinline__ void par(int) {}
};

// LDS layout shared by the H.x kernels: FP64 scratch (kBlock doubles), the
// binomial table (CR), then one [site][lane] slab of Y values per wave (CR).
struct HvLds {
    double* red;
    uint32_t* binom;
    uint32_t* ylds;
};

template <int MODE>
__device__ __forceinline__ HvLds hv_lds_setup(unsigned char* smem, const SectorDev& S) {
    HvLds l;
    l.red = reinterpret_cast<double*>(smem);
    l.binom = reinterpret_cast<uint32_t*>(smem + hv_red_bytes());
    uint32_t* slabs = l.binom + ((S.n_sites * S.bw + 3) & ~3);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    l.ylds = slabs + wave * S.n_sites * 64 + lane;
    if constexpr (MODE == kModeCr) stage_binomials(l.binom, S.binom, S.n_sites * S.bw);
    return l;
}

// The rows of one block of a (sub-)grid of G blocks: y = H x on rows
// [row0, row0 + nrows), columns [col0, col0 + VB) of [D][ld] blocks. In the
// Lanczos epilogue y holds u_{k-1} on entry (unless `first`) and receives
// w = hv_a (H u_k) - hv_b u_{k-1} per column; the products u_k[t] w[t] are
// folded, tile by tile, into per-wave FP64 sums wsum[wave * VB + c] (LDS).
template <typename L, int MODE, typename T, int VB, int EPI>
__device__ __forceinline__ void hv_body(const SectorDev& S, const BondTable& B, const HvLds& lds,
                                        const T* __restrict__ x, T* __restrict__ y, uint64_t ld,
                                        uint32_t col0, uint32_t row0, uint32_t nrows, uint32_t bid,
                                        uint32_t G, const Chain* chains, bool first, double* wsum) {
    const Binom C{lds.binom, S.bw};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
            GatherVisitor<T, VB> vis{x, ld, col0, S.dim - 1, B, acc, anti};
            visit_row<L, MODE>(t, S.n_up, B, C, S.basis, S.clt, lds.ylds, vis);
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
                    const T a = sizeof(T) == 4 ? T(chains[c].hv_a_f) : T(chains[c].hv_a_d);
                    const T b = sizeof(T) == 4 ? T(chains[c].hv_b_f) : T(chains[c].hv_b_d);
                    out[c] = a * out[c] - b * z[c];
                }
            }
            store_row<T, VB>(yrow, out);
        }
        if constexpr (EPI == kEpiLanczos) {
            // every lane takes part in the butterfly; rows past the end add 0
#pragma unroll
            for (int c = 0; c < VB; ++c) {
                double p = valid ? double(xt[c]) * double(out[c]) : 0.0;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
                if (lane == 0) wsum[wave * VB + c] += p;
            }
        }
    });
}

template <typename L, int MODE, typename T, int VB>
__global__ __launch_bounds__(kBlock) void hv_kernel(SectorDev S, BondTable B, HvLaunch h) {
    extern __shared__ __align__(16) unsigned char smem[];
    const HvLds lds = hv_lds_setup<MODE>(smem, S);
    hv_body<L, MODE, T, VB, kEpiPlain>(S, B, lds, static_cast<const T*>(h.x), static_cast<T*>(h.y), h.ld, h.col0,
                                        h.row0, h.nrows, blockIdx.x, gridDim.x, nullptr, false, nullptr);
}

// First half of Lanczos step k over every sector of the launch (one sector,
// all sectors of a plan, or a server round): w = H q_k - beta_{k-1} q_{k-1}
// and the FP64 partials of <u_k, w>; the last block of each sector sums the
// partials in block order into alpha_k (and the update coefficient). A sector
// whose chains have all stopped is skipped.
template <typename L, int MODE, typename T, int VB>
__global__ __launch_bounds__(kBlock) void hv_lanczos_kernel(LanczosLaunch a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int flag;
    uint32_t local = 0;
    const int s = sector_of_block(a.secs, a.nsec, blockIdx.x, &local);
    if (s < 0) return;
    const SecWork& sw = a.secs[s];
    if (sw.state[1] == 0) return;
    const int step = sw.state[0];
    const SectorDev S = sw.S;
    const BondTable& B = *sw.bonds;
    const HvLds lds = hv_lds_setup<MODE>(smem, S);
    double* wsum = lds.red;
    for (int i = threadIdx.x; i < kWaves * VB; i += kBlock) wsum[i] = 0.0;
    __syncthreads();
    const T* x = static_cast<const T*>(sw.u[(step - 1) & 1]);
    T* y = static_cast<T*>(sw.u[step & 1]);
    const Chain* chains = sw.chains + a.col0;
    hv_body<L, MODE, T, VB, kEpiLanczos>(S, B, lds, x, y, a.ld, a.col0, 0, S.dim, local, sw.G, chains, step == 1,
                                          wsum);
    __syncthreads();
    if (threadIdx.x < VB) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += wsum[w * VB + threadIdx.x];
        sw.partials[size_t(local) * a.ld + a.col0 + threadIdx.x] = t;
    }
    if (last_block(sw.ticket, sw.G, &flag)) {
        for (int c = 0; c < VB; ++c) {
            const double tot = grid_sum_col(sw.partials, int(sw.G), int(a.ld), int(a.col0) + c, lds.red);
            if (threadIdx.x == 0) {
                Chain* ch = &sw.chains[a.col0 + c];
                ch->alpha = ch->s_cur * tot;
                ch->up_d = ch->alpha * ch->s_cur;
                ch->up_f = float(ch->up_d);
            }
        }
        if (threadIdx.x == 0) *sw.ticket = 0u;
    }
}

template <typename L, int MODE, typename T, int VB>
hipError_t launch_hv_one(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    const size_t lds = hv_lds_bytes(s);
    auto kern = hv_kernel<L, MODE, T, VB>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(h.grid)), dim3(kBlock), lds, st, s, B, h);
    return hipGetLastError();
}

template <typename L, int MODE, typename T, int VB>
hipError_t launch_lanczos_one(const LanczosLaunch& a, size_t lds, hipStream_t st) {
    auto kern = hv_lanczos_kernel<L, MODE, T, VB>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(a.grid)), dim3(kBlock), lds, st, a);
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
    if (n_sites > 32) return f(uint64_t{}, std::integral_constant<int, kModeCr>{});
    return f(uint32_t{}, std::integral_constant<int, kModeCr>{});
}

template <typename T>
hipError_t launch_hv_typed(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    return with_mode(s.mode, s.n_sites, [&](auto l, auto m) {
        using L = decltype(l);
        return with_vb<T>(h.vb, [&](auto vb) { return launch_hv_one<L, decltype(m)::value, T, decltype(vb)::value>(s, B, h, st); });
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
