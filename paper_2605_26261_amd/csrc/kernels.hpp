// Kernel-side argument structs and the host-visible launchers of libftlm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace ftlm {

constexpr int kBlock = 256;      // threads per workgroup: four wave64s
constexpr int kWaves = kBlock / 64;
constexpr int kMaxSteps = 4096;  // row stride of the device alpha/beta arrays
constexpr int kMaxChains = 64;
constexpr int kMaxPlanSectors = 65;

// Per-chain Lanczos state, one per vector column, in device memory. The
// stored vector of step k is u_k with q_k = s_cur * u_k (the normalization
// of q_{k+1} = w / beta_k is folded into the next step's scalars instead of
// an extra pass over the vector).
struct Chain {
    double s_cur;      // scale of the current vector u_k
    double s_prev;     // scale of u_{k-1}
    double beta_prev;  // beta_{k-1}
    double amax;       // max_{j<=k}(|alpha_j|, beta_{j-1}) for the stopping rule
    double alpha;      // alpha_k of the step in flight
    double norm;       // |u_1| of the start vector
    // Scalars of the next kernels, precomputed once per step by the last
    // workgroup of the previous kernel so that every thread reads them with
    // scalar loads (no per-thread FP64 work or conversion):
    //   H.x epilogue  w = hv_a * (H u_k) - hv_b * u_{k-1}
    //   update        u_{k+1} = w - up * u_k
    double hv_a_d, hv_b_d, up_d;
    float hv_a_f, hv_b_f, up_f, pad_f;
    int32_t active;
    int32_t steps;
    int32_t fault;     // 1 once alpha_k or beta_k came out NaN or infinite
    int32_t pad_i;
};

// Sets the next-step scalars of a chain from its FP64 state.
__device__ __forceinline__ void chain_set_hv(Chain* ch) {
    ch->hv_a_d = ch->s_cur;
    ch->hv_b_d = ch->beta_prev * ch->s_prev;
    ch->hv_a_f = float(ch->hv_a_d);
    ch->hv_b_f = float(ch->hv_b_d);
}

// A sector as the kernels see it.
struct SectorDev {
    int n_sites;
    int n_up;
    int mode;
    int bw;                  // binomial table row width
    uint32_t dim;
    const uint32_t* binom;   // [N][bw]
    const uint32_t* basis;   // [D] (CLT mode)
    const CltEntry* clt;     // [2^N / 32] (CLT mode)
};

enum Epilogue { kEpiPlain = 0, kEpiLanczos = 1 };

// One plain multi-vector H.x launch over rows [row0, row0 + nrows) and the
// columns [col0, col0 + vb) of [D][ld] blocks x (input) and y (output).
struct HvLaunch {
    const void* x;
    void* y;
    uint64_t ld;
    uint32_t col0;
    uint32_t row0;
    uint32_t nrows;
    int vb;
    int dtype;
    int grid;
};

// One sector of a Lanczos launch (one sector, all sectors of a plan, or the
// active requests of a server round), in device memory. Its blocks are
// [block0, block0 + G) of the launch grid, with G = rows_grid(D) so the
// reduction order of every column depends on D only. Each sector carries its
// own bond table and step counter, so sectors of different graphs at
// different Lanczos steps can share a launch.
struct SecWork {
    SectorDev S;
    const BondTable* bonds;
    void* u[2];          // [D][ld] vector blocks; step k reads u_k from u[(k-1)&1]
    Chain* chains;       // [ld]
    double* partials;    // [G][ld]
    uint32_t* ticket;
    int32_t* state;      // [0] = current step k (1-based), [1] = chains still active
    double* alpha;       // [ld][kMaxSteps]
    double* beta;        // [ld][kMaxSteps]
    const uint64_t* keys;  // [ld] start-vector stream keys
    uint64_t r0;         // sample index of column 0
    uint32_t G;
    uint32_t block0;
    int32_t m_eff;       // min(M, D)
};

// Kernel arguments of the Lanczos kernels over a list of sectors. Columns
// [col0, col0 + vb) of every sector's [D][ld] blocks.
struct LanczosLaunch {
    const SecWork* secs;
    int nsec;
    int grid;            // total blocks (sum of the sectors' G, 8-aligned)
    uint64_t ld;
    uint32_t col0;
    int vb;
    int dtype;
    int last_chunk;      // this launch holds the last columns of a step
    double eps;          // stopping threshold
    int dist;            // start-vector distribution
    int mode;            // index mode shared by the sectors (host dispatch)
    int n_sites;         // N shared by the sectors (host dispatch)
};

hipError_t launch_hv(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st);
hipError_t launch_hv_lanczos(const LanczosLaunch& a, size_t lds, hipStream_t st);
hipError_t launch_start(const LanczosLaunch& a, hipStream_t st);
hipError_t launch_update(const LanczosLaunch& a, hipStream_t st);
hipError_t launch_chain_init(const LanczosLaunch& a, hipStream_t st);

// Sector table builders and index kernels (sector.hip).
hipError_t launch_build_basis(const SectorDev& s, hipStream_t st);
hipError_t launch_build_clt(const SectorDev& s, hipStream_t st);
hipError_t launch_rank(const SectorDev& s, const uint64_t* labels, uint64_t* idx, uint64_t n,
                       hipStream_t st);
hipError_t launch_unrank(const SectorDev& s, const uint64_t* idx, uint64_t* labels, uint64_t n,
                         hipStream_t st);
hipError_t launch_neighbors(const SectorDev& s, const BondTable& B, uint64_t t0, uint64_t count,
                            uint64_t* out, hipStream_t st);

// LDS bytes of the H.x kernels: FP64 scratch, then (CR) the binomial table
// and one [site][lane] slab of Y values per wave.
__host__ __device__ constexpr size_t hv_red_bytes() { return kBlock * sizeof(double); }
__host__ __device__ inline size_t hv_binom_lds_bytes(int n_sites, int bw, int mode) {
    return mode == kModeCr ? ((size_t(n_sites) * size_t(bw) * 4 + 15) & ~size_t(15)) : 0;
}
__host__ __device__ inline size_t hv_slab_lds_bytes(int n_sites, int mode) {
    return mode == kModeCr ? size_t(kWaves) * size_t(n_sites) * 64 * 4 : 0;
}
__host__ __device__ inline size_t hv_lds_bytes(const SectorDev& s) {
    return hv_red_bytes() + hv_binom_lds_bytes(s.n_sites, s.bw, s.mode) + hv_slab_lds_bytes(s.n_sites, s.mode);
}


// Grid of the persistent row kernels for a row count: a multiple of 8 (one
// share per XCD) capped near the number of resident workgroups, so reduction
// partials depend on the row count only.
__host__ __device__ inline uint32_t rows_grid(uint32_t nrows) {
    const uint32_t tiles = (nrows + kBlock - 1) / kBlock;
    if (tiles < 8) return tiles == 0 ? 1u : tiles;
    const uint32_t cap = 2048;
    const uint32_t g = tiles < cap ? tiles : cap;
    return (g + 7) & ~7u;
}

// The sector owning block `b` of a multi-sector launch, by a wave-uniform
// scan of the block ranges; *local receives the block's index inside the
// sector, or the function returns -1 for a padding block.
__device__ __forceinline__ int sector_of_block(const SecWork* secs, int nsec, uint32_t b,
                                               uint32_t* local) {
    for (int s = 0; s < nsec; ++s) {
        const uint32_t b0 = secs[s].block0, G = secs[s].G;
        if (b >= b0 && b < b0 + G) {
            *local = b - b0;
            return s;
        }
    }
    return -1;
}

}  // namespace ftlm
