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

__host__ __device__ constexpr size_t hv_red_bytes() { return kBlock * sizeof(double); }
inline size_t hv_binom_lds_bytes(const SectorDev& s) {
    return s.mode == kModeCr ? ((size_t(s.n_sites) * size_t(s.bw) * 4 + 15) & ~size_t(15)) : 0;
}
inline size_t hv_slab_lds_bytes(const SectorDev& s) {
    return s.mode == kModeCr ? size_t(kWaves) * size_t(s.n_sites) * 64 * 4 : 0;
}
inline size_t hv_lds_bytes(const SectorDev& s) {
    return hv_red_bytes() + hv_binom_lds_bytes(s) + hv_slab_lds_bytes(s);
}

template <typename L, int MODE, typename T, int VB, int EPI>
__global__ __launch_bounds__(kBlock) void hv_kernel(SectorDev S, BondTable B, HvLaunch h) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* red = reinterpret_cast<double*>(smem);
    uint32_t* binom_lds = reinterpret_cast<uint32_t*>(smem + hv_red_bytes());
    uint32_t* slabs = binom_lds + ((S.n_sites * S.bw + 3) & ~3);
    if constexpr (MODE == kModeCr) stage_binomials(binom_lds, S.binom, S.n_sites * S.bw);
    const Binom C{binom_lds, S.bw};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t* ylds = slabs + wave * S.n_sites * 64 + lane;

    const T* __restrict__ x = static_cast<const T*>(h.x);
    T* __restrict__ y = static_cast<T*>(h.y);
    const T jsum4 = sizeof(T) == 4 ? T(B.jsum4_f) : T(B.jsum4_d);

    // Lanczos scalars of this block's columns (wave-uniform).
    const Chain* chains = h.chains + h.col0;
    if constexpr (EPI == kEpiLanczos) {
        // per-wave running FP64 sums of <u_k, w> per column, in LDS
        for (int i = threadIdx.x; i < kWaves * VB; i += kBlock) red[i] = 0.0;
        __syncthreads();
    }

    const uint32_t ntiles = (h.nrows + kBlock - 1) / kBlock;
    for_each_tile(ntiles, [&](uint32_t tile) {
        const uint32_t r = tile * kBlock + threadIdx.x;
        const bool valid = r < h.nrows;
        T xt[VB], out[VB];
        if (valid) {
            const uint32_t t = h.row0 + r;
            T acc[VB];
#pragma unroll
            for (int c = 0; c < VB; ++c) acc[c] = T(0);
            T anti = T(0);
            GatherVisitor<T, VB> vis{x, h.ld, h.col0, S.dim - 1, B, acc, anti};
            visit_row<L, MODE>(t, S.n_up, B, C, S.basis, S.clt, ylds, vis);
            load_row<T, VB>(x + uint64_t(t) * h.ld + h.col0, xt);
            const T diag = jsum4 - anti;
#pragma unroll
            for (int c = 0; c < VB; ++c) out[c] = diag * xt[c] + acc[c];
            T* yrow = y + uint64_t(r) * h.ld + h.col0;
            if constexpr (EPI == kEpiLanczos) {
                T z[VB];
                if (!h.first) {
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
            // fold this tile's <u_k, w> terms into the wave's running sums
            // (every lane takes part in the butterfly; rows past the end add 0)
#pragma unroll
            for (int c = 0; c < VB; ++c) {
                double p = valid ? double(xt[c]) * double(out[c]) : 0.0;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) p += __shfl_xor(p, off, 64);
                if (lane == 0) red[wave * VB + c] += p;
            }
        }
    });

    if constexpr (EPI == kEpiLanczos) {
        __syncthreads();
        if (threadIdx.x < VB) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[w * VB + threadIdx.x];
            h.partials[size_t(blockIdx.x) * h.pstride + h.col0 + threadIdx.x] = s;
        }
        __shared__ int flag;
        if (last_block(h.ticket, &flag)) {
            for (int c = 0; c < VB; ++c) {
                const double tot = grid_sum_col(h.partials, int(gridDim.x), h.pstride, int(h.col0) + c, red);
                if (threadIdx.x == 0) {
                    Chain* ch = &h.chains[h.col0 + c];
                    ch->alpha = ch->s_cur * tot;
                    ch->up_d = ch->alpha * ch->s_cur;
                    ch->up_f = float(ch->up_d);
                }
            }
            if (threadIdx.x == 0) *h.ticket = 0u;
        }
    }
}

template <typename L, int MODE, typename T, int VB, int EPI>
hipError_t launch_hv_one(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    const size_t lds = hv_lds_bytes(s);
    auto kern = hv_kernel<L, MODE, T, VB, EPI>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(unsigned(h.grid)), dim3(kBlock), lds, st, s, B, h);
    return hipGetLastError();
}

template <typename L, int MODE, typename T, int EPI>
hipError_t launch_hv_vb(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    switch (h.vb) {
        case 1: return launch_hv_one<L, MODE, T, 1, EPI>(s, B, h, st);
        case 2: return launch_hv_one<L, MODE, T, 2, EPI>(s, B, h, st);
        case 4: return launch_hv_one<L, MODE, T, 4, EPI>(s, B, h, st);
        case 8: return launch_hv_one<L, MODE, T, 8, EPI>(s, B, h, st);
        case 16: return launch_hv_one<L, MODE, T, 16, EPI>(s, B, h, st);
        case 20:
            if constexpr (sizeof(T) == 4) return launch_hv_one<L, MODE, T, 20, EPI>(s, B, h, st);
            else return hipErrorInvalidValue;
        case 32:
            if constexpr (sizeof(T) == 4) return launch_hv_one<L, MODE, T, 32, EPI>(s, B, h, st);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_hv_typed(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st) {
    const bool wide = s.n_sites > 32;
    if (s.mode == kModeClt) {
        return h.epi == kEpiLanczos ? launch_hv_vb<uint32_t, kModeClt, T, kEpiLanczos>(s, B, h, st)
                                    : launch_hv_vb<uint32_t, kModeClt, T, kEpiPlain>(s, B, h, st);
    }
    if (wide) {
        return h.epi == kEpiLanczos ? launch_hv_vb<uint64_t, kModeCr, T, kEpiLanczos>(s, B, h, st)
                                    : launch_hv_vb<uint64_t, kModeCr, T, kEpiPlain>(s, B, h, st);
    }
    return h.epi == kEpiLanczos ? launch_hv_vb<uint32_t, kModeCr, T, kEpiLanczos>(s, B, h, st)
                                : launch_hv_vb<uint32_t, kModeCr, T, kEpiPlain>(s, B, h, st);
}

}  // namespace ftlm
