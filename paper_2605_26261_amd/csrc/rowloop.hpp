// Row-tile scheduling and deterministic FP64 block reductions shared by the
// persistent row kernels.
#pragma once

#include "kernels.hpp"

namespace ftlm {

// The tiles of kBlock rows owned by block `bid` of a (sub-)grid of G blocks
// in the streaming update kernel: first, first + step, ... below end. With G
// a multiple of 8 and the sub-grid starting at a multiple of 8, block i runs
// on XCD i mod 8 (round-robin dispatch), XCD x gets the x-th contiguous
// eighth of the tiles, and inside a share the XCD's blocks stride.
struct TileSpan {
    uint32_t first, end, step;
};

__device__ __forceinline__ TileSpan tile_span(uint32_t ntiles, uint32_t bid, uint32_t G) {
    if (G >= 8 && (G & 7u) == 0) {
        const uint32_t chunk = (ntiles + 7u) >> 3;
        const uint32_t begin = (bid & 7u) * chunk;
        return {begin + (bid >> 3), begin + chunk < ntiles ? begin + chunk : ntiles, G >> 3};
    }
    return {bid, ntiles, G};
}

// Calls f(tile) for the tiles of tile_span(ntiles, bid, G), in order: the
// update kernel's unstaged widths, so that a block sums the same rows in
// the same order whether its width is staged or not.
template <typename F>
__device__ __forceinline__ void for_each_span_tile(uint32_t ntiles, uint32_t bid, uint32_t G, F&& f) {
    const TileSpan sp = tile_span(ntiles, bid, G);
    for (uint32_t tile = sp.first; tile < sp.end; tile += sp.step) f(tile);
}

// Tiles per XCD super-tile in the gather kernels' schedule (for_each_tile).
constexpr uint32_t kXcdSuperTile = 16;

// Calls f(tile) for the tiles of block `bid` (the gather kernels and the
// start vectors). With G a multiple of 8, the tiles are dealt to the XCDs
// in super-tiles of kXcdSuperTile tiles (4096 rows), round-robin: super-tile
// k belongs to XCD k mod 8, and inside its super-tiles an XCD's blocks
// stride by G / 8 tiles. All eight XCDs thus sweep one common front of the
// rows, so the partner rows that miss one XCD's L2 are fetched into the
// shared Infinity Cache once for all of them. Contiguous eighths of the rows
// per XCD were slower at every width (N = 30, CR Lanczos step at 12 columns:
// 38.0 ms against 34.5; super-tiles of 1 to 16 tiles within 1 %, 128 tiles
// 35.7 ms).
template <typename F>
__device__ __forceinline__ void for_each_tile(uint32_t ntiles, uint32_t bid, uint32_t G, F&& f) {
    if (G >= 8 && (G & 7u) == 0) {
        constexpr uint32_t S = kXcdSuperTile;
        const uint32_t xcd = bid & 7u, slot = bid >> 3, per = G >> 3;
        const uint32_t supers = (ntiles + S - 1u) / S;
        const uint32_t mine = supers > xcd ? (supers - xcd + 7u) / 8u : 0u;  // super-tiles of this XCD
        const uint32_t count = mine * S;
        for (uint32_t q = slot; q < count; q += per) {
            const uint32_t tile = (xcd + 8u * (q / S)) * S + q % S;
            if (tile < ntiles) f(tile);
        }
    } else {
        for (uint32_t tile = bid; tile < ntiles; tile += G) f(tile);
    }
}

// One level of wave_fold_columns: lanes l and l ^ off hold partial sums of
// the same columns [lo, hi) in slots [0, SK); the lane with bit `off` clear
// keeps [lo, lo + SN), the other keeps [lo + SN, hi), and each adds the
// partner's partial sum of the columns it keeps to its own (own + partner,
// the order of the xor butterfly). Slots past a lane's columns carry no
// column and are never stored.
template <int SK, int SN, int VB>
__device__ __forceinline__ void fold_level(double (&v)[VB], int off, int lane, int& lo, int& hi) {
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int j = 0; j < SN; ++j) {
        const double keep_lo = v[j];
        const double keep_hi = (SN + j < SK) ? v[SN + j] : 0.0;
        const double recv = __shfl_xor(up ? keep_lo : keep_hi, off, 64);
        v[j] = (up ? keep_hi : keep_lo) + recv;
    }
    const int mid = lo + SN;
    if (up) lo = mid;
    else hi = hi < mid ? hi : mid;
}

// Adds the sums over a wave's 64 lanes of p[0..VB) to dst[0..VB) (LDS). Each
// column's sum is the one of the xor butterfly over lane offsets 32, 16, ...,
// 1: the same pairs of partial sums are added, in the same order, at every
// level. The columns are reduced by recursive halving, though: at each level
// a lane keeps half of its columns, so VB columns take about VB + 6 exchanges
// instead of 6 VB, and column c ends in the one lane that stores it. Called by
// whole waves; VB <= 64.
template <int VB>
__device__ __forceinline__ void wave_fold_columns(const double (&p)[VB], double* dst) {
    constexpr int S1 = (VB + 1) / 2, S2 = (S1 + 1) / 2, S3 = (S2 + 1) / 2;
    constexpr int S4 = (S3 + 1) / 2, S5 = (S4 + 1) / 2, S6 = (S5 + 1) / 2;
    static_assert(S6 == 1, "at most 64 columns");
    const int lane = threadIdx.x & 63;
    double v[VB];
#pragma unroll
    for (int c = 0; c < VB; ++c) v[c] = p[c];
    int lo = 0, hi = VB;
    fold_level<VB, S1>(v, 32, lane, lo, hi);
    fold_level<S1, S2>(v, 16, lane, lo, hi);
    fold_level<S2, S3>(v, 8, lane, lo, hi);
    fold_level<S3, S4>(v, 4, lane, lo, hi);
    fold_level<S4, S5>(v, 2, lane, lo, hi);
    fold_level<S5, S6>(v, 1, lane, lo, hi);
    if (lo < hi) dst[lo] += v[0];
}

// Sums v[0..N) over the workgroup in a fixed order (butterfly inside each
// wave, then the waves in order). red must hold (kWaves + 1) * N doubles;
// after the call red[kWaves * N + c] holds the block total of column c,
// visible to all threads.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double x = v[c];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) red[wave * N + c] = x;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[w * N + threadIdx.x];
        red[kWaves * N + threadIdx.x] = s;
    }
    __syncthreads();
}

// Publishes this block's partials and reports whether it is the last of the
// G blocks sharing `ticket` to do so (then every partial is visible to it).
// The ticket is reset by that last block for the next launch on the stream.
__device__ __forceinline__ bool last_block(uint32_t* ticket, uint32_t G, int* flag_lds) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev = atomicAdd(ticket, 1u);
        *flag_lds = (prev == G - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last) __threadfence();
    return last;
}

// Fixed-order sums over the G block partials of the columns col0 .. col0 +
// nc - 1 (nc <= NC), partials[g * pstride + col]: thread i sums blocks i,
// i + kBlock, ... of every column in one pass (a block's partials of all
// columns are one contiguous load), then the block combines the threads as a
// tree, column by column, so the order depends on G only. tot[c] receives the
// totals in every thread; red holds kBlock doubles.
template <int NC>
__device__ __forceinline__ void grid_sum_cols(const double* partials, int G, int pstride, int col0, int nc,
                                              double* red, double (&tot)[NC]) {
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] = 0.0;
    for (int g = threadIdx.x; g < G; g += kBlock) {
        const double* p = partials + size_t(g) * pstride + col0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < nc) s[c] += p[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (c >= nc) break;
        red[threadIdx.x] = s[c];
        __syncthreads();
        for (int half = kBlock / 2; half >= 1; half >>= 1) {
            if (threadIdx.x < half) red[threadIdx.x] += red[threadIdx.x + half];
            __syncthreads();
        }
        tot[c] = red[0];
        __syncthreads();
    }
}

}  // namespace ftlm
