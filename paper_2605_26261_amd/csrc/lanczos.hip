// Lanczos kernels: start vectors and the second half of a Lanczos step
// (paper Sec. 2, the recursion after Eq. 3, without reorthogonalization).
// The first half of a step (w = H q_k - beta_{k-1} q_{k-1} and alpha_k) is the
// Lanczos epilogue of the H.x kernel.
#include <math.h>

#include "hv_impl.hpp"

namespace ftlm {

namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

// SplitMix64's output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Entry i of a start vector from the stream with key `key`: output i of the
// generator is mix64(key + (i + 1) * gamma).
__device__ __forceinline__ double start_entry(int dist, uint64_t key, uint64_t i, uint64_t sample) {
    if (dist == 0) {
        return (mix64(key + (i + 1) * kGamma) >> 63) ? -1.0 : 1.0;
    } else if (dist == 1) {
        const uint64_t u1 = mix64(key + (2 * i + 1) * kGamma);
        const uint64_t u2 = mix64(key + (2 * i + 2) * kGamma);
        const double a = double((u1 >> 11) + 1) * 0x1.0p-53;  // (0, 1]
        const double b = double(u2 >> 11) * 0x1.0p-53;        // [0, 1)
        return sqrt(-2.0 * log(a)) * cos(2.0 * 3.141592653589793 * b);
    }
    return i == sample ? 1.0 : 0.0;
}

// Writes up to four columns of start vectors and their FP64 norms; the last
// workgroup turns the norms into each chain's initial scale s_1 = 1 / |u_1|.
template <typename T, int CB>
__global__ __launch_bounds__(kBlock) void start_kernel(SectorDev S, StartLaunch a, int cbase) {
    __shared__ double red[kBlock];
    __shared__ int flag;
    T* q = static_cast<T*>(a.q);
    const int nc = min(CB, a.ncols - cbase);
    double part[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) part[c] = 0.0;
    const uint32_t ntiles = (S.dim + kBlock - 1) / kBlock;
    for_each_tile(ntiles, [&](uint32_t tile) {
        const uint32_t t = tile * kBlock + threadIdx.x;
        if (t >= S.dim) return;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            if (c < nc) {
                const T v = T(start_entry(a.dist, a.keys[cbase + c], t, a.sample[cbase + c]));
                q[uint64_t(t) * a.ld + a.col0 + cbase + c] = v;
                part[c] += double(v) * double(v);
            }
        }
    });
    block_sum<CB>(part, red);
    if (threadIdx.x < nc)
        a.partials[size_t(blockIdx.x) * a.pstride + a.col0 + cbase + threadIdx.x] = red[kWaves * CB + threadIdx.x];
    if (last_block(a.ticket, &flag)) {
        for (int c = 0; c < nc; ++c) {
            const int col = int(a.col0) + cbase + c;
            const double tot = grid_sum_col(a.partials, int(gridDim.x), a.pstride, col, red);
            if (threadIdx.x == 0) {
                Chain* ch = &a.chains[col];
                const double nrm = sqrt(tot);
                ch->norm = nrm;
                ch->s_cur = nrm > 0.0 ? 1.0 / nrm : 0.0;
                ch->s_prev = 0.0;
                ch->beta_prev = 0.0;
                ch->amax = 0.0;
                ch->alpha = 0.0;
                ch->active = nrm > 0.0 ? 1 : 0;
                ch->steps = 0;
                chain_set_hv(ch);
            }
        }
        if (threadIdx.x == 0) *a.ticket = 0u;
    }
}

// Second half of Lanczos step k for a block of VB chains:
//   w -= alpha_k q_k  (q_k = s_k u_k),  beta_k = |w|,  u_{k+1} = w,
// with |w|^2 accumulated in FP64 per workgroup and summed in fixed order by
// the last workgroup, which then records alpha_k and beta_k and applies the
// stopping rule: the chain stops after step k when k reaches min(M, D) or
// beta_k <= eps * max_{j<=k}(|alpha_j|, beta_{j-1}). A stopped chain gets
// zero scales, so its columns stay zero in every later step.
template <typename T, int VB>
__global__ __launch_bounds__(kBlock) void update_kernel(SectorDev S, UpdateLaunch a) {
    __shared__ double red[kBlock];
    __shared__ int flag;
    const T* __restrict__ u = static_cast<const T*>(a.u);
    T* __restrict__ w = static_cast<T*>(a.w);
    const Chain* chains = a.chains + a.col0;
    double part[VB];
#pragma unroll
    for (int c = 0; c < VB; ++c) part[c] = 0.0;
    const uint32_t ntiles = (S.dim + kBlock - 1) / kBlock;
    for_each_tile(ntiles, [&](uint32_t tile) {
        const uint32_t t = tile * kBlock + threadIdx.x;
        if (t >= S.dim) return;
        T uu[VB], ww[VB];
        load_row<T, VB>(u + uint64_t(t) * a.ld + a.col0, uu);
        T* wrow = w + uint64_t(t) * a.ld + a.col0;
        load_row<T, VB>(wrow, ww);
#pragma unroll
        for (int c = 0; c < VB; ++c) {
            const T coef = sizeof(T) == 4 ? T(chains[c].up_f) : T(chains[c].up_d);
            ww[c] = ww[c] - coef * uu[c];
            part[c] += double(ww[c]) * double(ww[c]);
        }
        store_row<T, VB>(wrow, ww);
    });
    block_sum<VB>(part, red);
    if (threadIdx.x < VB)
        a.partials[size_t(blockIdx.x) * a.pstride + a.col0 + threadIdx.x] = red[kWaves * VB + threadIdx.x];
    if (last_block(a.ticket, &flag)) {
        for (int c = 0; c < VB; ++c) {
            const int col = int(a.col0) + c;
            const double tot = grid_sum_col(a.partials, int(gridDim.x), a.pstride, col, red);
            if (threadIdx.x == 0) {
                Chain* ch = &a.chains[col];
                if (ch->active) {
                    const double bk = sqrt(tot);
                    const double ak = ch->alpha;
                    a.alpha[size_t(col) * a.M + (a.step - 1)] = ak;
                    a.beta[size_t(col) * a.M + (a.step - 1)] = bk;
                    const double amax = fmax(ch->amax, fmax(fabs(ak), ch->beta_prev));
                    ch->amax = amax;
                    ch->steps = a.step;
                    if (a.step >= a.m_eff || bk <= a.eps * amax) {
                        ch->active = 0;
                        ch->s_cur = 0.0;
                        ch->s_prev = 0.0;
                        ch->beta_prev = 0.0;
                    } else {
                        ch->s_prev = ch->s_cur;
                        ch->s_cur = 1.0 / bk;
                        ch->beta_prev = bk;
                    }
                    chain_set_hv(ch);
                }
            }
        }
        if (threadIdx.x == 0) *a.ticket = 0u;
    }
}

__global__ void chain_init_kernel(Chain* chains, int n, uint32_t* tickets, int nt) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        Chain c{};
        chains[i] = c;
    }
    for (int i = threadIdx.x; i < nt; i += blockDim.x) tickets[i] = 0u;
}

template <typename T>
hipError_t launch_update_t(const SectorDev& s, const UpdateLaunch& a, hipStream_t st) {
    const dim3 g(unsigned(a.grid)), b(kBlock);
    switch (a.ncols) {
        case 1: hipLaunchKernelGGL((update_kernel<T, 1>), g, b, 0, st, s, a); break;
        case 2: hipLaunchKernelGGL((update_kernel<T, 2>), g, b, 0, st, s, a); break;
        case 4: hipLaunchKernelGGL((update_kernel<T, 4>), g, b, 0, st, s, a); break;
        case 8: hipLaunchKernelGGL((update_kernel<T, 8>), g, b, 0, st, s, a); break;
        case 16: hipLaunchKernelGGL((update_kernel<T, 16>), g, b, 0, st, s, a); break;
        case 20:
            if constexpr (sizeof(T) == 4) { hipLaunchKernelGGL((update_kernel<T, 20>), g, b, 0, st, s, a); break; }
            else return hipErrorInvalidValue;
        case 32:
            if constexpr (sizeof(T) == 4) { hipLaunchKernelGGL((update_kernel<T, 32>), g, b, 0, st, s, a); break; }
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_start(const SectorDev& s, const StartLaunch& a, hipStream_t st) {
    const dim3 g(unsigned(a.grid)), b(kBlock);
    for (int cb = 0; cb < a.ncols; cb += 4) {
        if (a.dtype == 0) hipLaunchKernelGGL((start_kernel<float, 4>), g, b, 0, st, s, a, cb);
        else hipLaunchKernelGGL((start_kernel<double, 4>), g, b, 0, st, s, a, cb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_update(const SectorDev& s, const UpdateLaunch& a, hipStream_t st) {
    return a.dtype == 0 ? launch_update_t<float>(s, a, st) : launch_update_t<double>(s, a, st);
}

hipError_t launch_chain_init(Chain* chains, int n, uint32_t* tickets, int nt, hipStream_t st) {
    hipLaunchKernelGGL(chain_init_kernel, dim3(1), dim3(256), 0, st, chains, n, tickets, nt);
    return hipGetLastError();
}

}  // namespace ftlm
