/*
 * ftlm.h - C ABI of libftlm: the data-parallel hot path of the
 * finite-temperature Lanczos method (FTLM) for spin-1/2 Heisenberg clusters
 * on one AMD Instinct MI355X (gfx950).
 *
 * Citations refer to arXiv 2605.26261, "GPU-accelerated finite-temperature
 * Lanczos method for spin Hamiltonians" (Sec. = section, Eq. = equation,
 * Alg. = algorithm).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status.   Every int-returning function returns FTLM_OK (0) or a negative
 *           FTLM_E_* code; ftlm_last_error() then returns a thread-local
 *           message. No C++ exception crosses this boundary.
 * Labels.   A basis state of N sites is the integer n whose bit k is 1 when
 *           site k is up (Eq. 11 at s = 1/2: a_k = m_k + 1/2). The sector with
 *           n_up up spins has total S^z = M = n_up - N/2 (Eq. 17) and
 *           dimension D = C(N, n_up) (Eq. 15 at s = 1/2); its basis is ordered
 *           by increasing label (the ordering behind Eq. 18).
 * Indices.  Labels and sector indices are uint64_t at this boundary. The
 *           index of a label outside the sector is FTLM_NONE (the -1 of
 *           Alg. 2). Kernels hold indices as uint32, so D must be < 2^32.
 * Memory.   Device buffers are owned by the caller (for example torch
 *           tensors on "cuda") and passed as raw device pointers; sizes come
 *           from the *_bytes() queries. These entry points never allocate
 *           device memory. Handles (ftlm_graph, ftlm_sector, ftlm_plan,
 *           ftlm_server) are host objects owned by the library, with
 *           create/destroy pairs; a handle must not outlive the device
 *           buffers it references. Handles are not thread-safe.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *           stream). Device work is enqueued in stream order and returns
 *           before it completes, unless the function returns host data, in
 *           which case it synchronizes the stream first.
 * Vectors.  A block of B vectors of a sector is stored row-major as [D][B]
 *           (row t holds component t of every vector), so one partner index
 *           serves all B vectors (Sec. 2, batched Lanczos). Element type is
 *           FTLM_F32 (float) or FTLM_F64 (double).
 */
#ifndef FTLM_H
#define FTLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FTLM_OK 0
#define FTLM_E_INVALID (-1)  /* a bad argument (null pointer, bad code, bad graph) */
#define FTLM_E_RANGE (-2)    /* a size outside what the library supports */
#define FTLM_E_NOSPACE (-3)  /* a caller buffer smaller than the size query */
#define FTLM_E_DEVICE (-4)   /* a HIP runtime error; the message names it */
#define FTLM_E_AGAIN (-5)    /* server: the result is not ready yet */
#define FTLM_E_REJECTED (-6) /* server: the request can never fit the arena */
#define FTLM_E_NUMERIC (-7)  /* a Lanczos chain met a NaN or infinite alpha or beta; it was
                                stopped at that step, the outputs are still written */

/* ---- enumerations ------------------------------------------------------ */
#define FTLM_CLT 0   /* compressed lookup table indexing (Sec. 2, Eqs. 18-21, Alg. 2) */
#define FTLM_CR 1    /* combinatorial ranking, no per-label table (Sec. 2, Eqs. 15-17, Alg. 1) */
#define FTLM_FULL 2  /* full lookup table: one uint32 index per label of [0, 2^N) (Sec. 2,
                        "State-to-index mapping"); 4 * 2^N bytes */
#define FTLM_LIN 3   /* Lin's two-dimensional search (Sec. 2, "State-to-index mapping"): the
                        label split into a high part h and a low part l of L = floor(N/2)
                        bits; index = hi[h] + lo[l], hi[h] the number of sector labels with
                        a smaller high part, lo[l] the rank of l among the L-bit strings with
                        its popcount; 4 (2^(N-L) + 2^L) bytes */

#define FTLM_F32 0
#define FTLM_F64 1

#define FTLM_PM1 0   /* i.i.d. +-1 entries */
#define FTLM_GAUSS 1 /* i.i.d. standard normal entries */
#define FTLM_UNIT 2  /* the unit vector e_r (exact trace when R = D) */

#define FTLM_NONE UINT64_MAX

typedef struct ftlm_graph ftlm_graph;
typedef struct ftlm_sector ftlm_sector;

/* Thread-local description of the last error on this thread ("" if none). */
const char* ftlm_last_error(void);

/* ABI version of this header. */
int ftlm_version(void);

/* ---- cluster graph ------------------------------------------------------
 * ftlm_graph_create: the Heisenberg model of Eq. (1) on N sites with one
 * coupling per bond, H = sum_b J_b s_i . s_j (the bond-dependent couplings
 * the outlook of Sec. 4 names). bi, bj, J are host arrays of n_bonds entries;
 * each bond needs 0 <= i, j < N and i != j; (i, j) and (j, i) are the same
 * bond, and repeated bonds are merged by summing their J. 2 <= N <= 64,
 * 1 <= n_bonds <= 128. The arrays are copied; *out receives the handle.
 * Errors: FTLM_E_INVALID for a null pointer or a bad site, FTLM_E_RANGE for
 * N or n_bonds out of range. */
int ftlm_graph_create(int n_sites, int n_bonds, const int32_t* bi, const int32_t* bj,
                      const double* J, ftlm_graph** out);
void ftlm_graph_destroy(ftlm_graph* g);
int ftlm_graph_n_sites(const ftlm_graph* g);
int ftlm_graph_n_bonds(const ftlm_graph* g);

/* ---- S^z sector -------------------------------------------------------
 * ftlm_sector_info: the sector's dimension D = C(N, n_up) (Eq. 15 at
 * s = 1/2; Eq. 17 fixes n_up = N/2 + M) and its weight in the thermal sums
 * of Eqs. 6-9: 1 for M = 0 and 2 otherwise, because the sectors +M and -M
 * have the same spectrum (Sec. 2, which restricts the runs to M >= 0). Either
 * output may be NULL. Errors: FTLM_E_RANGE for N outside [1, 64],
 * FTLM_E_INVALID for n_up outside [0, N]. */
int ftlm_sector_info(int n_sites, int n_up, uint64_t* dim, double* mult);

/* ftlm_sector_table_bytes: device bytes the sector tables need. Every mode
 * holds a binomial table C(p, k) (the cumulative dimension table D_c(p, A, 1)
 * of Eq. 16 at s = 1/2, a few KB). FTLM_CR stores nothing per label (Sec. 2,
 * CR). The stored maps add the sorted basis (uint32 per state, N <= 32) and:
 * FTLM_CLT the compressed lookup table, one {mask, prefix} pair of uint32 per
 * block of 32 labels over [0, 2^N) (Eqs. 18-21; 8 bytes per block, Eq. 21);
 * FTLM_FULL a uint32 per label of [0, 2^N); FTLM_LIN the two half tables.
 * Errors: FTLM_E_RANGE when N > 64, D >= 2^32, or N > 32 for a stored map. */
int ftlm_sector_table_bytes(int n_sites, int n_up, int mode, size_t* bytes);

/* ftlm_sector_create: builds the tables into the caller's device buffer
 * table_dev (at least ftlm_sector_table_bytes bytes, 256-byte aligned) on
 * `stream`: the binomial table, and in FTLM_CLT mode the basis (one unrank
 * per state) and the lookup table (the occupancy mask of each block and the
 * count of sector labels below it, Eq. 18). The build is asynchronous; the
 * handle may be used on the same stream at once. FTLM_E_NOSPACE if bytes is
 * too small. */
int ftlm_sector_create(int n_sites, int n_up, int mode, void* table_dev, size_t bytes,
                       void* stream, ftlm_sector** out);
uint64_t ftlm_sector_dim(const ftlm_sector* s);
int ftlm_sector_mode(const ftlm_sector* s);
void ftlm_sector_destroy(ftlm_sector* s);

/* ---- general local spin s (Sec. 2, Eqs. 11-17) --------------------------------
 * two_s = 2s in [1, 7] (d = 2s + 1 states per site), 2 <= N <= 16. A basis
 * state is the base-d integer n = sum_k a_k d^k with digit a_k = m_k + s
 * (Eq. 11); the sector is the set of labels with digit sum a_tot = N s + M
 * (Eq. 17), ordered by increasing label, of dimension D(N, a_tot) from the
 * recursion of Eq. (15). two_s = 1 is the spin-1/2 case (a_tot = n_up; these
 * calls then act as the ones above). A general-spin sector works with every
 * call that takes a sector except the plans and the server, which hold
 * spin-1/2 sectors:
 *   - ftlm_rank / ftlm_unrank take and return base-d labels (FTLM_NONE for a
 *     label outside the sector or at or above d^N);
 *   - ftlm_neighbors writes 2 * n_bonds entries per row (below);
 *   - ftlm_hv, ftlm_hv_rows, ftlm_start_vectors, ftlm_lanczos and
 *     ftlm_autotune run the same algorithms with launches of at most 8
 *     columns; start-vector streams are keyed by (seed, a_tot, r);
 *   - H = sum_b J_b (S_i^z S_j^z + (S_i^+ S_j^- + S_i^- S_j^+) / 2), the
 *     ladder terms with the coefficients of Eqs. (13)-(14).
 * Table: FTLM_CR stores the cumulative dimension table D_c of Eq. (16)
 * (N (a_tot + 3) (2s + 1) uint32); FTLM_CLT adds the basis (uint32[D]) and
 * the compressed lookup table over all d^N labels (Eqs. 18-21; needs d^N <=
 * 2^32). D must be < 2^32. Errors as for the spin-1/2 calls. */
int ftlm_sector_info_spin(int n_sites, int two_s, int a_tot, uint64_t* dim, double* mult);
int ftlm_sector_table_bytes_spin(int n_sites, int two_s, int a_tot, int mode, size_t* bytes);
int ftlm_sector_create_spin(int n_sites, int two_s, int a_tot, int mode, void* table_dev, size_t bytes,
                            void* stream, ftlm_sector** out);
int ftlm_sector_two_s(const ftlm_sector* s);

/* ftlm_rank: idx_dev[i] = sector index of labels_dev[i], FTLM_NONE when the
 * label is not in the sector. Mode FTLM_CLT looks up the table (Alg. 2);
 * mode FTLM_CR ranks digit by digit over the binomial table (Alg. 1). Both
 * arrays are device uint64[n]. */
int ftlm_rank(const ftlm_sector* s, const uint64_t* labels_dev, uint64_t* idx_dev, uint64_t n,
              void* stream);

/* ftlm_unrank: labels_dev[i] = label of sector index idx_dev[i] (FTLM_NONE
 * for an index >= D). FTLM_CLT reads the stored basis; FTLM_CR runs the
 * inverse of Alg. 1 (each digit chosen by comparing the remaining rank with
 * the cumulative counts, Sec. 2). Device uint64[n] arrays. */
int ftlm_unrank(const ftlm_sector* s, const uint64_t* idx_dev, uint64_t* labels_dev, uint64_t n,
                void* stream);

/* ftlm_clt_export: copies the lookup table's masks and prefix counts of
 * blocks [0, nblocks) to host arrays (test hook; FTLM_CLT mode only;
 * synchronizes the stream). nblocks may not exceed the table's block count
 * max(1, 2^N / 32). */
int ftlm_clt_export(const ftlm_sector* s, uint32_t* mask_host, uint32_t* prefix_host,
                    uint64_t nblocks, void* stream);

/* ftlm_neighbors: for rows t0..t0+count-1 and each bond b of the graph (the
 * merged bonds in order of first appearance, n_bonds = ftlm_graph_n_bonds),
 * idx_dev[(t - t0) * n_bonds + b] = the sector index
 * of the partner label n_t XOR (2^i + 2^j) when sites i, j of bond b are
 * antiparallel in n_t, else FTLM_NONE (Eq. 12 at s = 1/2; Eqs. 13-14 give the
 * coefficient J_b / 2). The indices come from the same code the H.x kernels
 * use. idx_dev is device uint64[count * n_bonds]. For a general-spin sector
 * each bond b = (i, j), i < j, has two entries: idx_dev[(t - t0) * 2 n_bonds
 * + 2 b] is the index of the source state with a_i + 1, a_j - 1 and entry
 * 2 b + 1 the one with a_i - 1, a_j + 1 (the two ladder terms of Eq. 12), or
 * FTLM_NONE where the digit leaves [0, 2s]; idx_dev then holds count * 2 *
 * n_bonds entries. Test hook. */
int ftlm_neighbors(const ftlm_sector* s, const ftlm_graph* g, uint64_t t0, uint64_t count,
                   uint64_t* idx_dev, void* stream);

/* ---- matrix-free H.x (Eq. 12) -------------------------------------------
 * y = H x for a block of nvec vectors in the [D][nvec] layout, in the
 * row-wise gather form of Sec. 2: each output row t is computed from its own
 * state n_t as
 *   y[t] = sum_b J_b s^z_i s^z_j x[t] + sum_{b antiparallel} (J_b / 2) x[idx(n_t ^ mask_b)]
 * with s^z_i s^z_j = +-1/4, no atomics. dtype FTLM_F32 accumulates each row in
 * FP32, FTLM_F64 in FP64. x and y must not overlap. 1 <= nvec <= 64. */
int ftlm_hv(const ftlm_sector* s, const ftlm_graph* g, const void* x_dev, void* y_dev, int nvec,
            int dtype, void* stream);

/* ftlm_hv_rows: the rows [row0, row0 + nrows) of H x only (one device's share
 * of a row-partitioned product). x_dev holds all D rows; y_dev holds nrows
 * rows (row row0 + r at position r). */
int ftlm_hv_rows(const ftlm_sector* s, const ftlm_graph* g, const void* x_dev, void* y_dev,
                 int nvec, int dtype, uint64_t row0, uint64_t nrows, void* stream);

/* ---- start vectors --------------------------------------------------------
 * ftlm_start_vectors: writes R random vectors [D][R] of the given dtype into
 * q_dev, unnormalized, and their FP64 norms into norms_host[R] (synchronizes).
 * Vector r (0 <= r < R) is sample r0 + r, drawn from the counter-based
 * SplitMix64 generator (Steele, Lea, Flood 2014) keyed by (seed, n_up,
 * r0 + r): entry i uses outputs numbered from i, so a vector never depends on
 * R. FTLM_PM1 takes the sign from the top bit of output i; FTLM_GAUSS applies
 * Box-Muller to 53-bit uniforms from outputs 2i and 2i + 1; FTLM_UNIT is
 * e_{r0+r}. The paper draws normalized random vectors (Sec. 2, FTLM) with the
 * same seeds in every precision (Sec. 3.1). work_dev/work_bytes: scratch of
 * at least ftlm_lanczos_workspace_bytes(s, R, dtype) bytes. */
int ftlm_start_vectors(const ftlm_sector* s, uint64_t seed, uint64_t r0, int R, int dist,
                       int dtype, void* q_dev, double* norms_host, void* work_dev,
                       size_t work_bytes, void* stream);

/* ---- Lanczos ----------------------------------------------------------------
 * ftlm_lanczos_workspace_bytes: device scratch for R chains of the sector. */
int ftlm_lanczos_workspace_bytes(const ftlm_sector* s, int R, int dtype, size_t* bytes);

/* ftlm_lanczos: R Lanczos chains without reorthogonalization (Sec. 2, the
 * paragraph after Eq. 3), all R advanced together by one multi-vector H.x
 * per step, started from the normalized vectors of ftlm_start_vectors. Step
 * k (Paige's ordering, FP64 reductions):
 *   w = H q_k - beta_{k-1} q_{k-1};  alpha_k = <q_k, w>;  w -= alpha_k q_k;
 *   beta_k = |w|;  q_{k+1} = w / beta_k.
 * Vectors are stored in dtype; alpha, beta and the norms are accumulated in
 * FP64 with a fixed reduction order (the result does not depend on which
 * other chains share the batch). Chain r stops after step k when k reaches
 * min(M, D) or beta_k <= eps * max_{j<=k}(|alpha_j|, beta_{j-1}), with eps =
 * 1e-4 (FP32: above the ~1e-5 round-off residual an FP32 chain leaves at an
 * exact invariant subspace) or 1e-12 (FP64). Outputs (host, synchronizes): alpha_host and
 * beta_host [R][M] (row r holds chain r; entries past steps_host[r] are 0),
 * steps_host[R]. 1 <= R <= 64, 1 <= M <= 4096. A chain whose alpha_k or
 * beta_k comes out NaN or infinite stops at that step and the call returns
 * FTLM_E_NUMERIC after writing every output. */
int ftlm_lanczos(const ftlm_sector* s, const ftlm_graph* g, uint64_t seed, uint64_t r0, int R,
                 int M, int dist, int dtype, void* work_dev, size_t work_bytes, double* alpha_host,
                 double* beta_host, int32_t* steps_host, void* stream);

/* ftlm_lanczos_noalloc: for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). It runs ftlm_lanczos, same kernels and same results bit for
 * bit, with the workspace taken from a device array of
 * FTLM_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends; it allocates no device memory. Arguments are those
 * of ftlm_lanczos without work_dev/work_bytes. The sector's tables must sit
 * on the current device (FTLM_E_INVALID otherwise). A call whose workspace
 * (ftlm_lanczos_workspace_bytes(s, R, dtype)) exceeds the array returns
 * FTLM_E_RANGE before any device work. Every call on a GPU shares that GPU's
 * array, which keeps the last call's contents (each call clears the counters
 * and chain state it needs): calls that overlap on one GPU, from two streams
 * or two threads, race and must not be made. */
#define FTLM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int ftlm_lanczos_noalloc(const ftlm_sector* s, const ftlm_graph* g, uint64_t seed, uint64_t r0,
                         int R, int M, int dist, int dtype, double* alpha_host, double* beta_host,
                         int32_t* steps_host, void* stream);

/* ---- autotuning of the batch width -------------------------------------------
 * The B chains of a Lanczos batch share each row's index work (Sec. 2,
 * batched Lanczos; the paper picks B adaptively, Sec. 3.4). ftlm_autotune
 * times one Lanczos step of B chains of the sector (the multi-vector H.x in
 * the form ftlm_lanczos would run it, and the vector update) at every launch
 * width B <= R: {1, 2, 4, 8, 10, 12, 16, 20, 32} for FP32, {1, 2, 4, 8, 16}
 * for FP64, with HIP events on `stream`, using
 * work_dev (at least ftlm_lanczos_workspace_bytes(s, R, dtype) bytes) as
 * scratch. It returns the B that minimizes the time of one Lanczos step of
 * all R chains run as floor(R / B) batches of B and one of R mod B, each
 * batch priced as the sum of its column chunks (the launch widths
 * ftlm_lanczos cuts it into). Results are cached per (N, n_up,
 * bonds, mode, dtype, R) for the life of the process; the file named by the
 * environment variable FTLM_AUTOTUNE_CACHE, when set, is read and appended
 * (one "key batch ms" line per entry). The workgroup grid is not tuned: it
 * fixes the FP64 reduction order, so results never depend on the choice. */
typedef struct ftlm_tuning {
    int32_t batch;          /* chains per ftlm_lanczos call */
    int32_t n_candidates;
    int32_t widths[12];     /* candidate B (n_candidates of them) */
    double ms[12];          /* measured step milliseconds at each B */
    double ms_per_step;     /* predicted step time of all R chains at `batch` */
    int32_t cached;         /* 1 when served from the cache */
} ftlm_tuning;
int ftlm_autotune(const ftlm_sector* s, const ftlm_graph* g, int R, int dtype, void* work_dev,
                  size_t work_bytes, void* stream, ftlm_tuning* out);

/* ---- batched all-sector plans ---------------------------------------------
 * A plan runs R Lanczos chains in each of several S^z sectors of one graph
 * (for example every sector M >= 0) with one launch per kernel per Lanczos
 * step covering all sectors: each sector owns a contiguous range of
 * workgroups sized by its dimension (sectors of dimension 1 to 10^6+ in the
 * same launch), and the M-step loop can be captured once in a HIP graph and
 * replayed. Per-chain results are bitwise the same as ftlm_lanczos on the
 * sector alone (the reduction order of a sector depends only on D).
 *
 * ftlm_plan_workspace_bytes: device bytes of the arena for the sectors
 * n_ups[0..n_sectors-1] (1 <= n_sectors <= 65): sector tables, two [D][R]
 * vector blocks per sector, reduction partials and chain states. */
typedef struct ftlm_plan ftlm_plan;
int ftlm_plan_workspace_bytes(const ftlm_graph* g, int n_sectors, const int32_t* n_ups, int mode,
                              int R, int dtype, size_t* bytes);

/* ftlm_plan_create: lays the plan out in the caller's arena (256-byte
 * aligned, at least ftlm_plan_workspace_bytes) and builds every sector's
 * tables on `stream` (synchronizes). M is the number of Lanczos steps per
 * chain (each sector stops at min(M, D_s) or on breakdown, as in
 * ftlm_lanczos). */
int ftlm_plan_create(const ftlm_graph* g, int n_sectors, const int32_t* n_ups, int mode, int R, int M,
                     int dtype, void* arena_dev, size_t arena_bytes, void* stream, ftlm_plan** out);

/* ftlm_plan_run: draws the start vectors (sample r0 + r of each sector, as
 * ftlm_start_vectors), runs the M Lanczos steps of all chains of all sectors
 * and copies the coefficients to the host (synchronizes): alpha_host and
 * beta_host are [n_sectors][R][M], steps_host [n_sectors][R]. With
 * use_graph != 0 the step loop is captured into a HIP graph on first use and
 * replayed; otherwise every kernel is launched eagerly. Work is ordered after
 * the work already enqueued on `stream`. */
int ftlm_plan_run(ftlm_plan* p, uint64_t seed, uint64_t r0, int dist, int use_graph, double* alpha_host,
                  double* beta_host, int32_t* steps_host, void* stream);

/* ftlm_plan_tune: chooses how the plan's R columns are split into kernel
 * launches (the vector-block widths of the batched Lanczos step, Sec. 3.4).
 * Candidates are the widest-first splits into launches of at most 32, 20,
 * 16, 10, 8 and 4 columns (FP64: 16, 8, 4), distinct ones only; each is timed
 * over one Lanczos step of the whole plan, after a warm-up step, with HIP
 * events on the plan's stream (ordered after the work on `stream`), twice,
 * keeping the faster time. The fastest candidate is kept for later
 * ftlm_plan_run calls; a graph captured before is dropped and captured again
 * by the next run with use_graph != 0. Chains are bitwise the same under
 * every split (the reduction order depends only on each sector's D). The
 * plan's vector blocks are overwritten. out may be NULL. Synchronizes.
 * Errors: FTLM_E_INVALID for a null plan, FTLM_E_DEVICE for a HIP error (the
 * plan then keeps its previous split). */
typedef struct ftlm_plan_tuning {
    int32_t n_candidates;
    int32_t chosen;          /* index of the kept candidate */
    int32_t max_width[8];    /* widest launch allowed in candidate i */
    int32_t n_launches[8];   /* kernel launches per Lanczos step of candidate i */
    double ms[8];            /* measured milliseconds of one Lanczos step */
} ftlm_plan_tuning;
int ftlm_plan_tune(ftlm_plan* p, void* stream, ftlm_plan_tuning* out);
void ftlm_plan_destroy(ftlm_plan* p);

/* ---- request server (continuous batching) ----------------------------------
 * A server owns a worker thread that runs FTLM requests on the device out of
 * one caller-owned arena. Requests are admitted in arrival order when their
 * HBM footprint fits the free arena (first fit) and fewer than max_active are
 * on the device; their tables, Krylov vectors and chain states stay on the
 * device until they finish. Each round advances every active request by one
 * Lanczos step, with one launch per kernel for all active requests of the
 * same N and R (sectors of different graphs and at different steps share
 * the launch). Finished requests leave at once and free their memory, so
 * waiting requests are admitted while others are still running. A request's
 * result does not depend on what else was on the device (each sector's
 * reduction order depends only on its dimension). */
typedef struct ftlm_server ftlm_server;

typedef struct ftlm_server_opts {
    int32_t mode;          /* FTLM_CLT or FTLM_CR */
    int32_t dtype;         /* FTLM_F32 or FTLM_F64 */
    int32_t max_active;    /* requests on the device at once, 1..256 (0 = 16: a small active set
                              finishes the oldest requests first at the same throughput, since
                              every round still fills the device) */
    int32_t batch_same_n;  /* 1: one launch per step for all active requests of equal N and R */
    int32_t steps_per_round;  /* Lanczos steps issued per round before finished requests are
                                 looked for, 1..64 (0 = 4); a request that finishes inside a
                                 round costs its remaining steps of the round one early return
                                 per block */
} ftlm_server_opts;

/* One FTLM job: R chains of M Lanczos steps in the sector n_up of the graph,
 * then E, C, chi (g) at the nT temperatures T. All arrays are copied at
 * submission. */
typedef struct ftlm_request {
    int32_t n_sites;
    int32_t n_bonds;
    const int32_t* bi;
    const int32_t* bj;
    const double* J;
    int32_t n_up;
    int32_t R;
    int32_t M;
    int32_t dist;
    uint64_t seed;
    int32_t nT;
    int32_t reserved;
    const double* T;
    double g;
} ftlm_request;

typedef struct ftlm_result_info {
    double t_submit;  /* seconds on the server clock (ftlm_server_clock) */
    double t_admit;
    double t_done;
    int32_t status;   /* FTLM_OK, or the error that ended the request */
    int32_t steps;    /* Lanczos steps summed over the request's chains */
    uint64_t dim;
    uint64_t footprint;
} ftlm_result_info;

/* Device bytes a request occupies in a server arena (tables + vectors + state). */
int ftlm_server_request_bytes(const ftlm_request* req, int mode, int dtype, size_t* bytes);
int ftlm_server_create(void* arena_dev, size_t arena_bytes, const ftlm_server_opts* opts, ftlm_server** out);
/* Queues a request (returns at once with its id). FTLM_E_REJECTED when its
 * footprint exceeds the whole arena; FTLM_E_INVALID for a malformed request. */
int ftlm_server_submit(ftlm_server* s, const ftlm_request* req, uint64_t* id);
/* FTLM_E_AGAIN while the request is queued or running; then copies its nT
 * values into E, C, chi, lnZ (any may be NULL), fills info and forgets it. */
int ftlm_server_poll(ftlm_server* s, uint64_t id, double* E, double* C, double* chi, double* lnZ,
                     ftlm_result_info* info);
/* Seconds since the server was created (steady clock). */
double ftlm_server_clock(const ftlm_server* s);
/* Peak arena bytes in use and rounds run so far. */
int ftlm_server_stats(const ftlm_server* s, uint64_t* peak_bytes, uint64_t* rounds, int32_t* active);
/* Stops the worker after the work already on the device and frees the handle. */
void ftlm_server_destroy(ftlm_server* s);

/* ---- Ritz values and the thermal reduction (host, FP64) --------------------
 * ftlm_ritz: eigenvalues theta[m] (ascending) of the m x m symmetric
 * tridiagonal T with diagonal alpha[0..m-1] and off-diagonal beta[0..m-2],
 * and the weights weight[k] = s_{k,1}^2, the squared first components of its
 * normalized eigenvectors (Sec. 2; they sum to 1). Implicit QL with
 * Wilkinson shifts, FP64, on the host (Sec. 2: the tridiagonal problem is
 * solved on the host in FP64). */
int ftlm_ritz(int m, const double* alpha, const double* beta, double* theta, double* weight);
/* ftlm_ritz_batch: ftlm_ritz for the n chains of one FTLM run at once, on
 * host threads (the R samples of Sec. 2 are independent). alpha, beta, theta
 * and weight are [n][stride] host arrays; chain r uses the first m[r]
 * entries of its alpha row and m[r] - 1 of its beta row (1 <= m[r] <=
 * stride) and gets theta and weight in its first m[r] entries, zeros in the
 * rest. Each chain is solved exactly as ftlm_ritz solves it, so the results
 * do not depend on the thread count. FTLM_E_INVALID for a bad argument or a
 * chain whose QL iteration does not converge (the other rows are still
 * written). */
int ftlm_ritz_batch(int n, int stride, const int32_t* m, const double* alpha, const double* beta, double* theta,
                    double* weight);

/* One sector's Lanczos samples for ftlm_thermo. theta and weight are
 * [R][stride] host arrays; sample r uses its first steps[r] entries. */
typedef struct ftlm_sector_result {
    int32_t n_up;        /* digit sum A of the sector (the up-spin count at s = 1/2) */
    int32_t R;
    int32_t stride;
    int32_t two_s;       /* 2s of the local spin; 0 or 1 for spin 1/2. M = A - N s (Eq. 17) */
    uint64_t dim;        /* D_Gamma */
    double mult;         /* 1 for M = 0, 2 for M > 0 (sectors -M mirror +M, Sec. 2) */
    const double* theta;
    const double* weight;
    const int32_t* steps;
} ftlm_sector_result;

/* ftlm_thermo: the FTLM thermal reduction over n_sectors sectors at nT
 * temperatures T[] (k_B = 1): Eqs. (6)-(8) with prefactor mult * D / R per
 * sector, every Boltzmann factor shifted by E0 = the smallest Ritz value
 * over all samples (the shift cancels in every ratio), C = beta^2 (<H^2> -
 * <H>^2), chi = g^2 beta sum_M M^2 Z_M / sum_M Z_M (Eq. 9). Writes E, C, chi
 * and lnZ = ln Z (with the shift undone) as host arrays of nT entries; any
 * output pointer may be NULL. */
int ftlm_thermo(int n_sites, int n_sectors, const ftlm_sector_result* sectors, int nT,
                const double* T, double g, double* E, double* C, double* chi, double* lnZ);

/* ---- precision diagnostics (Sec. 3.1-3.2) ------------------------------------
 * ftlm_ghosts: the Cullum-Willoughby ghost test of Eq. (25) on one chain's
 * m x m tridiagonal T (alpha[m], beta[m-1], host arrays). theta, weight:
 * the Ritz values of T in ascending order and their weights (as
 * ftlm_ritz). ell[k] = min_j |theta_k - theta1_j| over the eigenvalues
 * theta1 of T1, the matrix T without its first row and column (ell = +inf
 * when m = 1). ghost[k] = 1 when ell[k] < tau, with the tolerance the paper
 * applies to both precisions, tau = c_tau * u_FP32 * (theta_max - theta_min),
 * u_FP32 = 2^-24 (c_tau: a factor of order one). cluster[k]: the cluster of
 * theta_k, numbered in ascending order; neighbouring Ritz values within tau
 * of each other share a cluster (Fig. 5's clusters). cluster_weight[c]:
 * the total weight of cluster c for c < *n_clusters (0 beyond). All outputs
 * hold m entries. FTLM_E_INVALID for a bad argument or a QL iteration that
 * does not converge. */
int ftlm_ghosts(int m, const double* alpha, const double* beta, double c_tau, double* theta,
                double* weight, double* ell, int32_t* ghost, int32_t* cluster,
                double* cluster_weight, int32_t* n_clusters, double* tau);

/* ftlm_seed_spread: Eq. (22) over N_s independent FTLM estimates. values is
 * a [n_seeds][n] host array (row s: one run's observable at n points, for
 * example n temperatures); mean[n] and sigma[n] receive the mean over seeds
 * and sigma_emp = sqrt((1/N_s) sum_s (O_s - mean)^2). */
int ftlm_seed_spread(int n_seeds, int n, const double* values, double* mean, double* sigma);

/* ---- measurement hooks ---------------------------------------------------
 * When enabled, the library records a pair of HIP events around every H.x
 * launch on the launch's own stream and accumulates their elapsed times;
 * ftlm_stats_read synchronizes on the recorded events and reports the count
 * of H.x launches and their total milliseconds since the last reset. */
int ftlm_stats_enable(int on);
int ftlm_stats_reset(void);
int ftlm_stats_read(int64_t* hv_launches, double* hv_ms);

#ifdef __cplusplus
}
#endif

#endif /* FTLM_H */
