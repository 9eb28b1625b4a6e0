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

// A sector as the kernels see it. Spin-1/2 sectors (two_s = 1) hold the
// binomial table; for a local spin s = two_s / 2 > 1/2, n_up is the sector's
// digit sum A (Eq. 17), `binom` holds the cumulative dimension table of
// Eq. (16) as [N][bw][two_s + 1] (spin.hpp), and labels are base-(two_s + 1)
// integers below n_labels (Eq. 11).
struct SectorDev {
    int n_sites;
    int n_up;
    int mode;
    int bw;                  // binomial table row width (A slots of the D_c table)
    uint32_t dim;
    const uint32_t* binom;   // [N][bw] (spin 1/2) or [N][bw][two_s + 1]
    const uint32_t* basis;   // [D] (CLT mode)
    const CltEntry* clt;     // [n_labels / 32] (CLT mode)
    int two_s;               // 2s: 1 for spin 1/2
    uint64_t n_labels;       // d^N, d = two_s + 1
    const uint32_t* full;    // [2^N] sector index per label (FULL mode)
    const uint32_t* lin_hi;  // [2^(N - lin_lo)] (LIN mode)
    const uint32_t* lin_lo;  // [2^lin_lo] (LIN mode)
    int lin_lo_bits;
};

// The stored partner-index map of a sector (CR keeps none; it gets a CLT
// map that is never read).
template <int MODE>
__device__ __forceinline__ auto table_map(const SectorDev& S) {
    if constexpr (MODE == kModeFull) return TableMap<kModeFull>{S.full};
    else if constexpr (MODE == kModeLin) return TableMap<kModeLin>{S.lin_hi, S.lin_lo, S.lin_lo_bits};
    else return TableMap<kModeClt>{S.clt};
}

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
// active requests of a server round), in device memory. In the kernels with a
// static grid (start vectors, update) its blocks are [block0, block0 + G) of
// the launch grid, with G = stream_grid(D); the persistent Lanczos H.x
// kernels (spin 1/2 and general spin) split it into `items` =
// sector_items(D) work items. Both depend on D only, and so does the reduction order of every
// column. Each sector carries its own bond table and step counter, so
// sectors of different graphs at different Lanczos steps can share a launch.
struct SecWork {
    SectorDev S;
    const BondTable* bonds;
    void* u[2];          // [D][ld] vector blocks; step k reads u_k from u[(k-1)&1]
    Chain* chains;       // [ld]
    double* partials;    // [max(G, items)][ld]
    uint32_t* ticket;
    int32_t* state;      // [0] = current step k (1-based), [1] = chains still active
    double* alpha;       // [ld][kMaxSteps]
    double* beta;        // [ld][kMaxSteps]
    const uint64_t* keys;  // [ld] start-vector stream keys
    uint64_t r0;         // sample index of column 0
    uint32_t G;
    uint32_t block0;
    uint32_t items;      // work items of the persistent H.x
    int32_t m_eff;       // min(M, D)
};

// Kernel arguments of the Lanczos kernels over a list of sectors. Columns
// [col0, col0 + vb) of every sector's [D][ld] blocks.
struct LanczosLaunch {
    const SecWork* secs;
    int nsec;
    int grid;            // total blocks (sum of the sectors' G, 8-aligned)
    int items;           // work items of the persistent H.x (sum of the sectors' items)
    uint64_t max_dim;    // the largest sector dimension (host launch tuning)
    uint64_t ld;
    uint32_t col0;
    int vb;
    int dtype;
    int last_chunk;      // this launch holds the last columns of a step
    double eps;          // stopping threshold
    int dist;            // start-vector distribution
    int mode;            // index mode shared by the sectors (host dispatch)
    int n_sites;         // N shared by the sectors (host dispatch)
    int two_s;           // local spin 2s shared by the sectors (host dispatch)
    // Work queue of the persistent H.x launch (kQueueWords counters, zero
    // between launches), or null for a grid of one block per work item.
    uint32_t* queue;
};

// The persistent Lanczos H.x takes its work items from eight counters, one
// per XCD, and counts its exiting blocks in a ninth; the last block to exit
// zeroes all nine for the next launch on the stream.
constexpr int kQueueWords = 9;
constexpr size_t kQueueBytes = 256;

hipError_t launch_hv(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st);
// General-spin sectors (two_s > 1; hv_spin.hip).
hipError_t launch_hv_spin(const SectorDev& s, const BondTable& B, const HvLaunch& h, hipStream_t st);
hipError_t launch_hv_lanczos_spin(const LanczosLaunch& a, size_t lds, hipStream_t st);
hipError_t launch_build_basis_spin(const SectorDev& s, hipStream_t st);
hipError_t launch_build_clt_spin(const SectorDev& s, hipStream_t st);
hipError_t launch_rank_spin(const SectorDev& s, const uint64_t* labels, uint64_t* idx, uint64_t n, hipStream_t st);
hipError_t launch_unrank_spin(const SectorDev& s, const uint64_t* idx, uint64_t* labels, uint64_t n,
                              hipStream_t st);
hipError_t launch_neighbors_spin(const SectorDev& s, const BondTable& B, uint64_t t0, uint64_t count,
                                 uint64_t* out, hipStream_t st);
hipError_t launch_hv_lanczos(const LanczosLaunch& a, size_t lds, hipStream_t st);
hipError_t launch_start(const LanczosLaunch& a, hipStream_t st);
hipError_t launch_update(const LanczosLaunch& a, hipStream_t st);
hipError_t launch_chain_init(const LanczosLaunch& a, hipStream_t st);

// Sector table builders and index kernels (sector.hip).
hipError_t launch_build_basis(const SectorDev& s, hipStream_t st);
hipError_t launch_build_clt(const SectorDev& s, hipStream_t st);
hipError_t launch_build_full(const SectorDev& s, hipStream_t st);
hipError_t launch_build_lin(const SectorDev& s, hipStream_t st);
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
// General spin: the FP64 scratch, the ladder factors (FP64 and FP32, eight
// each), then (every mode) the cumulative dimension table or (CLT) the powers
// d^p, and (CR) two [site][lane] slabs per wave.
__host__ __device__ inline size_t hv_spin_table_lds_bytes(const SectorDev& s) {
    const size_t t = s.mode == kModeCr ? size_t(s.n_sites) * size_t(s.bw) * size_t(s.two_s + 1) : size_t(s.n_sites);
    return (t * 4 + 15) & ~size_t(15);
}
__host__ __device__ inline size_t hv_spin_lds_bytes(const SectorDev& s) {
    return hv_red_bytes() + 8 * 8 + 8 * 4 + hv_spin_table_lds_bytes(s) + 2 * hv_slab_lds_bytes(s.n_sites, s.mode);
}
__host__ __device__ inline size_t hv_lds_bytes(const SectorDev& s) {
    if (s.two_s > 1) return hv_spin_lds_bytes(s);
    return hv_red_bytes() + hv_binom_lds_bytes(s.n_sites, s.bw, s.mode) + hv_slab_lds_bytes(s.n_sites, s.mode);
}


// Grid of a row kernel for a row count: a multiple of 8 (one share per XCD)
// and at most `cap` blocks, so reduction partials depend on the row count
// only.
__host__ __device__ inline uint32_t capped_grid(uint32_t nrows, uint32_t cap) {
    const uint32_t tiles = (nrows + kBlock - 1) / kBlock;
    if (tiles < 8) return tiles == 0 ? 1u : tiles;
    const uint32_t g = tiles < cap ? tiles : cap;
    return (g + 7) & ~7u;
}

// The plain H.x: near the number of resident workgroups (latency-bound
// gathers need every slot).
__host__ __device__ inline uint32_t rows_grid(uint32_t nrows) { return capped_grid(nrows, 2048); }

// The streaming start and update kernels: 512 blocks, two per CU. N = 30,
// 20 chains as 8 + 8 + 4 columns: 55.7 ms per Lanczos step of all three
// blocks with 2048 blocks, 55.0 with 1024 or 768, 54.3-54.7 with 512, 55.4
// with 384 and 55.9 with 256 (one column alone was 2 % slower at 512).
__host__ __device__ inline uint32_t stream_grid(uint32_t nrows) { return capped_grid(nrows, 512); }

// Work items of a sector in the persistent Lanczos H.x, each with its own
// slot of reduction partials: a multiple of 8 (an equal count per XCD), about
// four row tiles per item, at most 16384. A workgroup runs several items, so
// with many small items every workgroup ends within about one item of the
// others whatever the kernel's occupancy; the count depends on the row count
// only, so the reduction order, and every result, does not depend on the
// launch width, the index map or the other sectors.
__host__ __device__ inline uint32_t sector_items(uint32_t nrows) {
    const uint32_t tiles = (nrows + kBlock - 1) / kBlock;
    if (tiles < 8) return tiles == 0 ? 1u : tiles;
    const uint32_t cap = 16384;
    uint32_t g = (tiles + 3) / 4;
    g = g < 8 ? 8 : (g < cap ? g : cap);
    return (g + 7) & ~7u;
}

// Work item k of XCD x in a persistent launch: the sectors' items whose
// index inside the sector is x mod 8, sector by sector in launch order (an
// item index keeps its XCD, so for_each_tile still gives each XCD its own
// super-tiles). Returns the sector and *local, or -1 when the XCD's items
// are exhausted.
__device__ __forceinline__ int queue_item(const SecWork* secs, int nsec, uint32_t xcd, uint32_t k,
                                          uint32_t* local) {
    for (int s = 0; s < nsec; ++s) {
        const uint32_t G = secs[s].items;
        const uint32_t cnt = G > xcd ? (G - xcd + 7u) / 8u : 0u;
        if (k < cnt) {
            *local = xcd + 8u * k;
            return s;
        }
        k -= cnt;
    }
    return -1;
}

// Called by every block of a persistent launch after its last item. Every
// thread's writes (outputs and reduction partials) are released, then the
// block counts itself out; returns true in the last block to get here, with
// every other block's writes visible to it, after it has zeroed the counters
// for the next launch (every block has stopped taking items). These are the
// only device-scope fences of the launch: on gfx950 such a fence writes back
// and invalidates the XCD's L2, which a fence per work item would do
// thousands of times while other workgroups still gather from it.
__device__ __forceinline__ bool queue_exit(uint32_t* q, uint32_t grid, int* flag_lds) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t done = atomicAdd(q + 8, 1u);
        const bool last = done == grid - 1u;
        if (last)
            for (int i = 0; i < kQueueWords; ++i) atomicExch(q + i, 0u);
        *flag_lds = last ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last) __threadfence();
    return last;
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
