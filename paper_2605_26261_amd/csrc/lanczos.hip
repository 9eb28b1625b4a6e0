// Lanczos kernels over a list of sectors: start vectors and the second half
// of a Lanczos step (paper Sec. 2, the recursion after Eq. 3, without
// reorthogonalization). The first half of a step (w = H q_k - beta_{k-1}
// q_{k-1} and alpha_k) is hv_lanczos_kernel. A launch covers one sector or
// every sector of a plan; each sector owns a contiguous range of blocks.
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "hv_impl.hpp"

namespace ftlm {

template <typename T>
hipError_t launch_lanczos_typed(int, int, const LanczosLaunch&, size_t, hipStream_t);

hipError_t persistent_grid(const void* kern, size_t lds, int items, int* grid) {
    static std::mutex mu;
    static std::map<std::pair<const void*, size_t>, int> cache;  // per kernel and LDS size
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({kern, lds});
        if (it != cache.end()) {
            per_cu = it->second;
        } else {
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds);
            if (e != hipSuccess) return e;
            cache[{kern, lds}] = per_cu;
        }
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int resident = ((std::max(1, per_cu) * cus + 7) / 8) * 8;
    const int cap = ((items + 7) / 8) * 8;
    *grid = std::max(8, std::min(resident, cap));
    return hipSuccess;
}

hipError_t launch_hv_lanczos(const LanczosLaunch& a, size_t lds, hipStream_t st) {
    if (a.two_s > 1) return launch_hv_lanczos_spin(a, lds, st);
    return a.dtype == 0 ? launch_lanczos_typed<float>(a.mode, a.n_sites, a, lds, st)
                        : launch_lanczos_typed<double>(a.mode, a.n_sites, a, lds, st);
}

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

// Writes columns [col0, col0 + vb) (vb <= CB) of every sector's start block
// u_1 and their FP64 norms; the last block of a sector turns the norms into
// each chain's initial scale s_1 = 1 / |u_1|.
template <typename T, int CB>
__global__ __launch_bounds__(kBlock) void start_kernel(LanczosLaunch a) {
    __shared__ double red[kBlock];
    __shared__ int flag;
    uint32_t local = 0;
    const int s = sector_of_block(a.secs, a.nsec, blockIdx.x, &local);
    if (s < 0) return;
    const SecWork& sw = a.secs[s];
    const uint32_t dim = sw.S.dim;
    T* q = static_cast<T*>(sw.u[0]);
    const int nc = a.vb < CB ? a.vb : CB;
    double part[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) part[c] = 0.0;
    const uint32_t ntiles = (dim + kBlock - 1) / kBlock;
    for_each_tile(ntiles, local, sw.G, [&](uint32_t tile) {
        const uint32_t t = tile * kBlock + threadIdx.x;
        if (t >= dim) return;
        const uint64_t i = t;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            if (c < nc) {
                const uint32_t col = a.col0 + c;
                const T v = T(start_entry(a.dist, sw.keys[col], i, sw.r0 + col));
                q[uint64_t(t) * a.ld + col] = v;
                part[c] += double(v) * double(v);
            }
        }
    });
    block_sum<CB>(part, red);
    if (threadIdx.x < nc) sw.partials[size_t(local) * a.ld + a.col0 + threadIdx.x] = red[kWaves * CB + threadIdx.x];
    if (last_block(sw.ticket, sw.G, &flag)) {
        double tot[CB];
        grid_sum_cols<CB>(sw.partials, int(sw.G), int(a.ld), int(a.col0), nc, red, tot);
        for (int c = 0; c < nc; ++c) {
            const int col = int(a.col0) + c;
            if (threadIdx.x == 0) {
                Chain* ch = &sw.chains[col];
                const double nrm = sqrt(tot[c]);
                sw.state[1] += nrm > 0.0 ? 1 : 0;
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
        if (threadIdx.x == 0) *sw.ticket = 0u;
    }
}

// Second half of Lanczos step k for columns [col0, col0 + VB) of every
// sector:  w -= alpha_k q_k (q_k = s_k u_k),  beta_k = |w|,  u_{k+1} = w,
// with |w|^2 accumulated in FP64 per block and summed in fixed order by the
// sector's last block, which then records alpha_k and beta_k and applies the
// stopping rule: a chain stops after step k when k reaches min(M, D) or
// beta_k <= eps * max_{j<=k}(|alpha_j|, beta_{j-1}). A stopped chain gets
// zero scales, so its columns stay zero in every later step.
// Blocks whose rows are 32 to 128 bytes (a multiple of 8) go through LDS: the
// rows of u and w staged together are contiguous, so they move with fully
// coalesced 16-byte accesses (8-byte ones for rows that are not a multiple of
// 16 bytes), while each thread still updates its own row (the same arithmetic
// and summation order as without the staging). With one thread per row, a
// vector access of rows that wide spans several cache lines per wave;
// narrower rows are already well coalesced. Rows of up to 96 bytes are staged
// a whole tile at a time, 128-byte rows half a tile at a time (two 256-row
// tiles would not fit the static LDS). A block loads its next chunk into
// registers before it stores the current one, so its reads stay in flight
// while it writes; every byte is touched once per step, so the accesses are
// non-temporal. Without the staging, 128-byte rows ran at under 1 TB/s and
// 40-byte rows at 4.0 TB/s; staged without the prefetch, 48-byte rows ran at
// 4.7 TB/s, and with it at 5.1 TB/s.
template <typename T, int VB>
__host__ __device__ constexpr bool update_staged() {
    return (VB * sizeof(T)) % 8 == 0 && VB * sizeof(T) >= 32 && VB * sizeof(T) <= 128;
}

template <typename T, int VB>
__host__ __device__ constexpr int update_stage_rows() {
    return VB * sizeof(T) <= 96 ? kBlock : kBlock / 2;
}

template <typename T, int VB>
__global__ __launch_bounds__(kBlock) void update_kernel(LanczosLaunch a) {
    __shared__ double red[kBlock];
    __shared__ int flag;
    constexpr bool kStage = update_staged<T, VB>();
    constexpr int kStageRows = update_stage_rows<T, VB>();
    __shared__ __align__(16) T stage_u[kStage ? kStageRows * VB : 1];
    __shared__ __align__(16) T stage_w[kStage ? kStageRows * VB : 1];
    uint32_t local = 0;
    const int s = sector_of_block(a.secs, a.nsec, blockIdx.x, &local);
    if (s < 0) return;
    const SecWork& sw = a.secs[s];
    if (sw.state[1] == 0) return;
    const int step = sw.state[0];
    const uint32_t dim = sw.S.dim;
    const T* __restrict__ u = static_cast<const T*>(sw.u[(step - 1) & 1]);
    T* __restrict__ w = static_cast<T*>(sw.u[step & 1]);
    // the update coefficients, read once (through a generic pointer the
    // compiler would re-read them after every store of the tile loop)
    T coef[VB];
#pragma unroll
    for (int c = 0; c < VB; ++c) {
        const Chain* ch = sw.chains + a.col0 + c;
        coef[c] = sizeof(T) == 4 ? T(ch->up_f) : T(ch->up_d);
    }
    double part[VB];
#pragma unroll
    for (int c = 0; c < VB; ++c) part[c] = 0.0;
    const uint32_t ntiles = (dim + kBlock - 1) / kBlock;
    // whole rows of [D][ld] blocks: a tile is one contiguous range
    const bool staged = kStage && a.col0 == 0 && a.ld == uint64_t(VB);
    if constexpr (kStage) {
        if (staged) {
            // copy unit: 16 bytes, or 8 for rows of an odd number of 8-byte words
            constexpr int kUnit = (VB * sizeof(T)) % 16 == 0 ? 4 : 2;
            using VU = uint32_t __attribute__((ext_vector_type(kUnit)));
            constexpr uint32_t kRowUnits = uint32_t(VB * sizeof(T)) / uint32_t(4 * kUnit);
            constexpr int kPer = int((uint32_t(kStageRows) * kRowUnits + kBlock - 1) / kBlock);
            VU* lu = reinterpret_cast<VU*>(stage_u);
            VU* lw = reinterpret_cast<VU*>(stage_w);
            // A chunk is rows [h0, h0 + hr) of one tile; the block walks its
            // tiles in tile_span's order. The next chunk's rows are loaded
            // into registers while the current chunk is stored.
            VU pu[kPer], pw[kPer];
            auto tile_rows = [&](uint32_t tile) {
                return dim - tile * kBlock < uint32_t(kBlock) ? dim - tile * kBlock : uint32_t(kBlock);
            };
            auto chunk_units = [&](uint32_t tile, uint32_t h0) {
                const uint32_t left = tile_rows(tile) - h0;
                return (left < uint32_t(kStageRows) ? left : uint32_t(kStageRows)) * kRowUnits;
            };
            auto fetch = [&](uint32_t tile, uint32_t h0) {
                const uint32_t n = chunk_units(tile, h0);
                const uint64_t r0 = uint64_t(tile) * kBlock + h0;
                const VU FTLM_GLOBAL* gu = gptr(reinterpret_cast<const VU*>(u + r0 * VB));
                const VU FTLM_GLOBAL* gw = gptr(reinterpret_cast<const VU*>(w + r0 * VB));
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const uint32_t i = threadIdx.x + uint32_t(k) * kBlock;
                    if (i < n) {
                        pu[k] = __builtin_nontemporal_load(gu + i);
                        pw[k] = __builtin_nontemporal_load(gw + i);
                    }
                }
            };
            const TileSpan sp = tile_span(ntiles, local, sw.G);
            uint32_t tile = sp.first, h0 = 0;
            if (tile < sp.end) fetch(tile, h0);
            while (tile < sp.end) {
                const uint32_t n = chunk_units(tile, h0);
                const uint32_t hr = n / kRowUnits;
#pragma unroll
                for (int k = 0; k < kPer; ++k) {
                    const uint32_t i = threadIdx.x + uint32_t(k) * kBlock;
                    if (i < n) {
                        lu[i] = pu[k];
                        lw[i] = pw[k];
                    }
                }
                __syncthreads();
                // each thread updates the row it owns (row threadIdx.x of the tile)
                if (threadIdx.x >= h0 && threadIdx.x < h0 + hr) {
                    T* wr = stage_w + (threadIdx.x - h0) * VB;
                    const T* ur = stage_u + (threadIdx.x - h0) * VB;
#pragma unroll
                    for (int c = 0; c < VB; ++c) {
                        const T v = wr[c] - coef[c] * ur[c];
                        part[c] += double(v) * double(v);
                        wr[c] = v;
                    }
                }
                __syncthreads();
                VU FTLM_GLOBAL* gw = gptr(reinterpret_cast<VU*>(w + (uint64_t(tile) * kBlock + h0) * VB));
                h0 += uint32_t(kStageRows);
                if (h0 >= tile_rows(tile)) {
                    h0 = 0;
                    tile += sp.step;
                }
                if (tile < sp.end) fetch(tile, h0);
                for (uint32_t i = threadIdx.x; i < n; i += kBlock) __builtin_nontemporal_store(lw[i], gw + i);
                __syncthreads();
            }
        }
    }
    for_each_span_tile(ntiles, local, sw.G, [&](uint32_t tile) {
        const uint32_t t = tile * kBlock + threadIdx.x;
        if constexpr (kStage) {
            if (staged) return;  // done above
        }
        if (t >= dim) return;
        T uu[VB], ww[VB];
        load_row<T, VB>(u + uint64_t(t) * a.ld + a.col0, uu);
        T* wrow = w + uint64_t(t) * a.ld + a.col0;
        load_row<T, VB>(wrow, ww);
#pragma unroll
        for (int c = 0; c < VB; ++c) {
            ww[c] = ww[c] - coef[c] * uu[c];
            part[c] += double(ww[c]) * double(ww[c]);
        }
        store_row<T, VB>(wrow, ww);
    });
    block_sum<VB>(part, red);
    if (threadIdx.x < VB) sw.partials[size_t(local) * a.ld + a.col0 + threadIdx.x] = red[kWaves * VB + threadIdx.x];
    if (last_block(sw.ticket, sw.G, &flag)) {
        double tot[VB];
        grid_sum_cols<VB>(sw.partials, int(sw.G), int(a.ld), int(a.col0), VB, red, tot);
        for (int c = 0; c < VB; ++c) {
            const int col = int(a.col0) + c;
            if (threadIdx.x == 0) {
                Chain* ch = &sw.chains[col];
                if (ch->active) {
                    const double bk = sqrt(tot[c]);
                    const double ak = ch->alpha;
                    sw.alpha[size_t(col) * kMaxSteps + (step - 1)] = ak;
                    sw.beta[size_t(col) * kMaxSteps + (step - 1)] = bk;
                    const double amax = fmax(ch->amax, fmax(fabs(ak), ch->beta_prev));
                    ch->amax = amax;
                    ch->steps = step;
                    // a non-finite coefficient ends the chain and marks it
                    // (the host reports FTLM_E_NUMERIC); the comparison below
                    // is false for NaN, so without this the chain would run on
                    const bool fault = !(isfinite(ak) && isfinite(bk));
                    if (fault) ch->fault = 1;
                    if (fault || step >= sw.m_eff || bk <= a.eps * amax) {
                        sw.state[1] -= 1;
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
        if (threadIdx.x == 0) {
            if (a.last_chunk) sw.state[0] = step + 1;
            *sw.ticket = 0u;
        }
    }
}

// Zeroes every sector's chain states and ticket and sets its step counter to
// 1 with no active chains (one block per sector).
__global__ void chain_init_kernel(LanczosLaunch a) {
    if (blockIdx.x == 0 && a.queue && threadIdx.x < unsigned(kQueueWords)) a.queue[threadIdx.x] = 0u;
    if (int(blockIdx.x) >= a.nsec) return;
    const SecWork& sw = a.secs[blockIdx.x];
    for (int i = threadIdx.x; i < int(a.ld); i += blockDim.x) {
        Chain c{};
        sw.chains[i] = c;
    }
    if (threadIdx.x == 0) {
        *sw.ticket = 0u;
        sw.state[0] = 1;
        sw.state[1] = 0;
    }
}

}  // namespace

hipError_t launch_start(const LanczosLaunch& a, hipStream_t st) {
    const dim3 g(unsigned(a.grid)), b(kBlock);
    if (a.vb < 1 || a.vb > 4) return hipErrorInvalidValue;
    if (a.dtype == 0) hipLaunchKernelGGL((start_kernel<float, 4>), g, b, 0, st, a);
    else hipLaunchKernelGGL((start_kernel<double, 4>), g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_update(const LanczosLaunch& a, hipStream_t st) {
    const dim3 g(unsigned(a.grid)), b(kBlock);
    auto go = [&](auto tt) {
        using T = decltype(tt);
        return with_vb<T>(a.vb, [&](auto vb) {
            hipLaunchKernelGGL((update_kernel<T, decltype(vb)::value>), g, b, 0, st, a);
            return hipGetLastError();
        });
    };
    return a.dtype == 0 ? go(float{}) : go(double{});
}

hipError_t launch_chain_init(const LanczosLaunch& a, hipStream_t st) {
    hipLaunchKernelGGL(chain_init_kernel, dim3(unsigned(a.nsec)), dim3(64), 0, st, a);
    return hipGetLastError();
}

}  // namespace ftlm
