/*
 * mgs.h -- C ABI of libmgs, the MI355X (gfx950) hot path of the MesonGS++
 * size-aware configuration search (arXiv 2604.26799).
 *
 * Conventions for every entry point
 *   - d_* arguments are device pointers (HIP device memory of the current
 *     device), h_* arguments are host pointers.
 *   - The caller owns every buffer.  Entry points that need scratch space
 *     take a caller-provided device workspace (d_ws, ws_bytes) sized by the
 *     matching *_ws_bytes() query; nothing is allocated on these calls.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously on it; host arguments are read
 *     before the call returns, so they may be freed right after.
 *   - Every call returns an int status: MGS_OK (0) or a negative code.
 *     Argument errors are detected before anything is enqueued.  Errors that
 *     depend on data (non-finite inputs) are raised on the device into a
 *     status word kept in the workspace; mgs_status_fetch() synchronises the
 *     stream and returns it.  Launch failures return MGS_EDEVICE.
 *   - Layouts are row-major.  The attribute matrix is structure-of-arrays:
 *     attr[c * ld + i] is channel c of Gaussian i.
 */
#ifndef MGS_H
#define MGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGS_OK 0
#define MGS_EINVAL (-1)       /* bad argument (NULL, size, range, order) */
#define MGS_ENONFINITE (-2)   /* an input that must be finite was not */
#define MGS_EINFEASIBLE (-3)  /* 0-1 ILP: even the smallest allocation exceeds the budget */
#define MGS_EDEVICE (-4)      /* HIP launch or runtime failure */
#define MGS_EWORKSPACE (-5)   /* workspace missing or smaller than the query says */
#define MGS_ELIMIT (-6)       /* 0-1 ILP: exact search exceeded its state limit */

/* Largest limits of the entry points. */
#define MGS_MAX_RATIOS 64     /* reserve ratios per sweep */
#define MGS_MAX_GROUP 65535   /* group size G (histogram counts are 16-bit) */
#define MGS_MAX_BITS 16       /* candidate bit-widths are in [1, 16] */
#define MGS_MAX_VQ_DIM 64     /* vector length of VQ assignment */
#define MGS_MAX_JOBS 64       /* scenes in one multi-scene sweep launch */

/* Text for a status code (static storage). */
const char* mgs_strerror(int status);

/* Library version string (static storage). */
const char* mgs_version(void);

/*
 * Status word of a workspace: synchronises `stream`, returns MGS_ENONFINITE if
 * the last call that used d_ws met a non-finite value, MGS_OK otherwise.
 */
int mgs_status_fetch(const void* d_ws, void* stream);

/* ======================================================================
 * Reserve-ratio pruning (paper: section "Gaussians Pruning"; the reserve
 * ratio tau keeps the tau*N most important Gaussians and cuts the rest).
 *
 * For each of T keep counts h_k[t] (0 <= h_k[t] <= n), select the h_k[t]
 * Gaussians with the largest importance d_imp; equal importance is broken
 * by the smaller index (-0 and +0 compare equal).  d_kept receives, for
 * t = 0..T-1 in turn, the h_k[t] selected indices in ascending order
 * (int32, total sum_t h_k[t] entries).  Counts need not be sorted.
 * Errors: MGS_EINVAL (n < 0 or n >= 2^31, T outside [1, MGS_MAX_RATIOS], a
 * count out of range, NULL pointer with nonzero size), MGS_EWORKSPACE;
 * non-finite importance raises MGS_ENONFINITE in the status word and
 * leaves d_kept unspecified.
 * ====================================================================== */
size_t mgs_prune_select_ws_bytes(int64_t n, int32_t T);
int mgs_prune_select(const float* d_imp, int64_t n, const int64_t* h_k, int32_t T,
                     int32_t* d_kept, void* d_ws, size_t ws_bytes, void* stream);

/* ======================================================================
 * Group-wise quantization sweep (paper: section "Group-wise Attribute
 * Quantization" for the quantizer, section "Acceleration" for the loss
 * table Omega, section "Size Estimator" for the entropy size).
 *
 * For each reserve ratio t, channel c and group g -- the kept Gaussians
 * d_kept[koff_t + g*G .. min((g+1)*G, k_t)) where koff_t = sum_{s<t} k_s --
 * and each candidate bit-width b = h_bits[i]:
 *   S = (max - min) / 2^b,  Z = round(2^b - max / S)       (FP32, half-even)
 *   q = round(clamp(x / S + Z, 0, 2^b - 1)),  xhat = (q - Z) * S
 *   (a group with S == 0 has q = 0 and xhat = min)
 *   err [t][c][g][i] = sum_j w_j (xhat_j - x_j)^2   with w = d_imp   (FP64)
 *   bits[t][c][g][i] = sum_k h_k log2(n / h_k) over the code histogram h (FP64)
 *   gmin/gmax[t][c][g] = group minimum / maximum (FP32)
 * Tables hold Gmax = ceil(max_t k_t / G) group slots per (t, c); slots past
 * ceil(k_t / G) are NaN.  d_hist (optional, may be NULL) receives the code
 * histograms, uint32 [T][C][Gmax][sum_i 2^bits[i]] (2^b bins per listed b,
 * in list order); meant for small inputs.  Codes, histograms and group
 * bounds are exact.  err: each thread sums the FP32 terms of at most 32
 * elements, a wavefront sums its 64 threads in FP32, and the wavefront
 * totals are added in FP64, so for nonnegative weights it agrees with the
 * FP64 definition within 41 * 2^-24 (~2.4e-6) relative; a wavefront total
 * that overflows, or is small enough that underflowed terms could matter,
 * is recomputed with FP64 terms, as are groups that need the literal
 * division or whose step underflows.  bits: FP64 entropy,
 * within ~1e-12 relative plus G * 2^-(K+1) absolute where the entropy comes
 * from grid-rounded increments (K = 52 - ceil(log2(G log2 G + G + 1))).
 * Results are deterministic: the same inputs give bit-identical tables.
 * Workspace: mgs_quant_sweep_ws_bytes(desc) bytes, which grow with
 * sum_t ceil(k_t / G) (one int per group for the tile order); a descriptor
 * with h_k == NULL gets the bound for T ratios of N Gaussians each.
 * Limits: 1 <= G <= MGS_MAX_GROUP, 1 <= T <= MGS_MAX_RATIOS, h_bits strictly
 * increasing in [1, 16], ld >= N, 0 <= k_t <= N, kept indices in [0, N).
 * Errors: MGS_EINVAL, MGS_EWORKSPACE; non-finite attributes or weights in a
 * group, or a group range max - min that overflows, set NaN for that group
 * and MGS_ENONFINITE in the status word.
 * ====================================================================== */
typedef struct {
    int64_t N;              /* Gaussians in the scene */
    int64_t ld;             /* row stride of d_attr, in elements (>= N) */
    int32_t C;              /* attribute channels */
    int32_t T;              /* reserve ratios */
    int32_t G;              /* group size */
    int32_t nb;             /* number of candidate bit-widths */
    const int64_t* h_k;     /* host [T]: kept Gaussians per ratio */
    const uint8_t* h_bits;  /* host [nb]: candidate bit-widths */
} mgs_sweep_desc;

size_t mgs_quant_sweep_ws_bytes(const mgs_sweep_desc* desc);
int mgs_quant_sweep(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                    const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                    float* d_gmax, uint32_t* d_hist, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Allocation-free sweep, for callers that cannot allocate device memory or
 * hand over a workspace: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  mgs_quant_sweep_static computes exactly
 * what mgs_quant_sweep computes (same kernels, launch shape and results) but
 * keeps its scratch -- status word, scene descriptor, entropy tables, tile
 * order -- in a device array of MGS_STATIC_SCRATCH_BYTES inside the library,
 * one per GPU, held until the process ends.  Nothing is allocated, on the
 * device or the host.  The caller still passes inputs and outputs as for
 * mgs_quant_sweep.  Limit: the call returns MGS_EWORKSPACE (before touching
 * the device) when mgs_quant_sweep_ws_bytes(desc) exceeds
 * MGS_STATIC_SCRATCH_BYTES, i.e. for more than about 780,000 groups per
 * channel run, sum_t ceil(k_t / G), at G = 65535 (more at smaller G).
 * Every call on a GPU uses that GPU's one array and rewrites all of it
 * (status word reset, tables and tile order rebuilt), so calls that overlap
 * on one GPU -- on two streams, from two host threads, or a captured graph
 * replayed beside another call -- race; calls on one stream in order do not.
 * mgs_quant_sweep_static_status synchronises `stream` and returns the status
 * word of the current GPU's array (MGS_ENONFINITE after a call that met a
 * non-finite value, as mgs_status_fetch for a workspace).  Errors: as
 * mgs_quant_sweep; MGS_EDEVICE if the array's address cannot be taken.
 */
#define MGS_STATIC_SCRATCH_BYTES (4 << 20)
int mgs_quant_sweep_static(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                           const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                           float* d_gmax, uint32_t* d_hist, void* stream);
int mgs_quant_sweep_static_status(void* stream);

/*
 * Batched sweep: the sweeps of up to MGS_MAX_JOBS scenes (each with its own
 * N, C, reserve ratios, inputs and tables, all sharing G and the bit-width
 * list) in one launch; every table equals what mgs_quant_sweep computes for
 * that scene alone, bit for bit.  h_jobs (host, njobs entries) is read
 * during the call only.  The workspace (mgs_quant_sweep_multi_ws_bytes,
 * which depends on njobs, G and every job's group count, bounded as in
 * mgs_quant_sweep_ws_bytes for jobs whose h_k is NULL) carries one status
 * word for the whole launch.  Errors: as mgs_quant_sweep, plus MGS_EINVAL when njobs is outside
 * [1, MGS_MAX_JOBS] or the jobs differ in G or the bit-width list.
 */
typedef struct {
    mgs_sweep_desc desc;
    const float* d_attr;    /* [C][ld] */
    const float* d_imp;     /* [N] */
    const int32_t* d_kept;  /* [sum_t k_t] */
    double* d_err;          /* [T][C][Gmax][nb] */
    double* d_bits;         /* [T][C][Gmax][nb] */
    float* d_gmin;          /* [T][C][Gmax] */
    float* d_gmax;          /* [T][C][Gmax] */
    uint32_t* d_hist;       /* optional, as in mgs_quant_sweep */
} mgs_sweep_job;

size_t mgs_quant_sweep_multi_ws_bytes(const mgs_sweep_job* h_jobs, int32_t njobs);
int mgs_quant_sweep_multi(const mgs_sweep_job* h_jobs, int32_t njobs, void* d_ws, size_t ws_bytes,
                          void* stream);

/*
 * Launch shape of the sweep kernel: threads per workgroup, elements per
 * thread, LDS bytes the histogram plan may use (0 = the device maximum),
 * channels per workgroup tile (0 = all channels), and the grid: 0 = one
 * workgroup per tile, 1 = persistent (one workgroup per resident slot of the
 * device, taking tiles in order from one counter per XCD and then from the
 * other XCDs' counters; the counters live in the workspace's status block
 * and are reset by every call, so the launch stays graph-capturable).
 * mgs_sweep_autotune times every candidate shape on the given inputs (each
 * `reps` times, HIP events on `stream`, minimum kept), registers the fastest
 * for (G, nb, max bit-width) in a process-wide table used by later sweeps --
 * among shapes within 3 % of the fastest, the one with more channels per
 * tile, which fetches each tile's indices and weights fewer times -- and
 * leaves the tables computed with it.  It synchronises the stream, so it
 * must not be called during graph capture.  h_ms[i] / h_shapes[i][5]
 * (optional, mgs_sweep_shape_count() entries) receive each candidate's time
 * (-1 when it does not apply) and shape; h_best[5] (optional) the chosen one.
 * mgs_sweep_set_shape registers a shape by hand (nt == 0 clears the entry).
 * Results are identical for every shape.
 */
int mgs_sweep_shape_count(void);
int mgs_sweep_autotune(const mgs_sweep_desc* desc, const float* d_attr, const float* d_imp,
                       const int32_t* d_kept, double* d_err, double* d_bits, float* d_gmin,
                       float* d_gmax, void* d_ws, size_t ws_bytes, void* stream, int32_t reps,
                       float* h_ms, int32_t* h_shapes, int32_t* h_best);
int mgs_sweep_set_shape(int32_t G, int32_t nb, int32_t bmax, int32_t nt, int32_t ept,
                        int32_t lds_cap, int32_t cpb, int32_t persist);

/* ======================================================================
 * Final quantization at a chosen bit allocation, and its inverse (paper:
 * section "Group-wise Attribute Quantization"; the stored metadata are the
 * per-block minimum and maximum, section "Entropy Encoding").
 *
 * mgs_quantize: groups g of G consecutive entries of d_kept (k entries, the
 * last group may be shorter); ng = ceil(k / G).  For channel c the group
 * uses b = d_bw[c * ng + g] (1..16).  Writes d_codes[c * k + j] (uint16,
 * the code q of the sweep's definition) and d_gmin/d_gmax[c * ng + g].
 * mgs_dequantize: d_out[c * k + j] = xhat = (q - Z) * S, with S and Z
 * recomputed from the stored minimum, maximum and b (min when S == 0).
 * Errors: MGS_EINVAL (C < 1, k < 0, G outside [1, MGS_MAX_GROUP], NULL).
 * Bit-widths outside [1, 16] in d_bw are clamped into range on the device.
 * ====================================================================== */
int mgs_quantize(const float* d_attr, int64_t ld, int32_t C, const int32_t* d_kept, int64_t k,
                 int32_t G, const uint8_t* d_bw, uint16_t* d_codes, float* d_gmin, float* d_gmax,
                 void* stream);
int mgs_dequantize(const uint16_t* d_codes, int64_t k, int32_t C, int32_t G, const uint8_t* d_bw,
                   const float* d_gmin, const float* d_gmax, float* d_out, void* stream);

/* ======================================================================
 * Nearest-codeword assignment of the vector quantizer for the higher-degree
 * SH coefficients (paper: section "Attribute Transformation", clustering of
 * the 1+D SH coefficients with a codebook and an index table).
 *
 * d_idx[i] = argmin_j sum_d (x[i][d] - cb[j][d])^2, the distance summed in
 * FP64 over d in order; ties go to the smallest j.  d_x is [N][D] and d_cb
 * [K][D], both row-major FP32.  d_dist (optional) receives that FP64
 * distance of the winner.  d_nfallback (optional, device int64) receives
 * the number of rows that needed the exact full scan.  Exact: the result
 * equals the FP64 definition bit for bit.
 * Limits: 1 <= D <= MGS_MAX_VQ_DIM, 1 <= K <= 2^30, 0 <= N < 2^31
 * (mgs_vq_assign_ws_bytes returns 0 outside them).
 * Errors: MGS_EINVAL, MGS_EWORKSPACE; non-finite data -> MGS_ENONFINITE in
 * the status word.
 * ====================================================================== */
size_t mgs_vq_assign_ws_bytes(int64_t N, int32_t D, int32_t K);
int mgs_vq_assign(const float* d_x, int64_t N, int32_t D, const float* d_cb, int32_t K,
                  int32_t* d_idx, double* d_dist, int64_t* d_nfallback, void* d_ws,
                  size_t ws_bytes, void* stream);

/* ======================================================================
 * One mini-batch k-means iteration around the assignment above (paper:
 * section "Attribute Transformation", paragraph "Clustering 1+D SH
 * Coefficients": the codebook is refined by a batched clustering strategy,
 * Sculley's web-scale k-means, over several iterations).
 *
 * The batch is the rows d_batch[B] (int64 row indices into d_x[N][D],
 * chosen by the caller, repeats allowed).  Every batch row is assigned to its
 * nearest center of d_cb[K][D] by the rule of mgs_vq_assign (written to
 * d_assign[B] if not NULL); then every center j that received n_j > 0 rows,
 * having absorbed v_j = d_counts[j] samples before, becomes the running mean
 *   c_j <- (v_j c_j + sum of its batch rows) / (v_j + n_j)   (FP64, stored FP32)
 * and d_counts[j] += n_j.  Sculley's per-sample update (eta = 1 / v) reaches
 * the same mean.  d_cb and d_counts are updated in place (centers with no
 * rows keep their value).  The sum of a center's rows is taken in FP64 one
 * row after another in batch order (the rows are grouped by center with a
 * stable sort), then (v_j c_j + sum) / (v_j + n_j) in FP64, stored as FP32:
 * the same inputs give bit-identical centers on every run.
 * Workspace: mgs_kmeans_step_ws_bytes(B, D, K).  Errors: MGS_EINVAL
 * (N < 0, B outside [0, 2^31), D outside [1, MGS_MAX_VQ_DIM], K outside [1, 2^30], NULL
 * pointers), MGS_EWORKSPACE; non-finite rows or centers, and batch indices
 * outside [0, N) (gathered as zero rows), raise MGS_ENONFINITE in the
 * status word.
 * ====================================================================== */
size_t mgs_kmeans_step_ws_bytes(int64_t B, int32_t D, int32_t K);
int mgs_kmeans_step(const float* d_x, int64_t N, int32_t D, const int64_t* d_batch, int64_t B,
                    float* d_cb, int32_t K, int64_t* d_counts, int32_t* d_assign, void* d_ws,
                    size_t ws_bytes, void* stream);

/*
 * Budget-first retention of SH vectors (paper: same paragraph -- the budget
 * left after the essential components keeps the original vectors of the
 * top-ranked Gaussians by importance, appended to the codebook and coded
 * with it).  mgs_vq_retain_count: r = min(N, floor(remaining_bits / (32 D)))
 * vectors fit (each is stored as D FP32 values like the codebook; 0 when
 * nothing remains).  mgs_vq_retain: d_top[r] are the retained Gaussians in
 * ascending index (mgs_prune_select with the single count r); their rows of
 * d_x[N][D] are copied to rows K .. K+r-1 of d_cb_ext (whose first K rows are
 * the caller's codebook) and d_idx[d_top[e]] = K + e.  The workspace needs
 * only the status word (256 bytes); an index outside [0, N) is skipped and
 * raises MGS_ENONFINITE in it.  Errors: MGS_EINVAL (r outside [0, N], K < 0,
 * K + r >= 2^31, D outside [1, MGS_MAX_VQ_DIM], NULL pointers), MGS_EWORKSPACE.
 */
int64_t mgs_vq_retain_count(int64_t remaining_bits, int64_t N, int32_t D);
int mgs_vq_retain(const float* d_x, int64_t N, int32_t D, const int32_t* d_top, int64_t r,
                  float* d_cb_ext, int32_t K, int32_t* d_idx, void* d_ws, size_t ws_bytes, void* stream);

/* ======================================================================
 * Region-Adaptive Hierarchical Transform of attributes over voxelized
 * positions (paper: section "Attribute Transformation", paragraph "Region
 * Adaptive Hierarchical Transform": transform T_1, leaf weight 1, merged
 * weight the sum of its children's, unmatched nodes passing up, one DC and
 * N - 1 AC coefficients per channel).
 *
 * d_codes[N]: Morton codes of the occupied voxels (per level: x in bit 0,
 * y in bit 1, z in bit 2), strictly increasing, below 2^(3 depth), with
 * depth in [1, 21] bits per axis.  Step s = 0 .. 3 depth - 1 merges every
 * two live nodes whose codes agree above bit s (the one with bit s clear:
 * weight w1, value a1; the other: w2, a2):
 *   L = (sqrt(w1) a1 + sqrt(w2) a2) / sqrt(w1 + w2)   (weight w1 + w2, goes up)
 *   H = (sqrt(w1) a2 - sqrt(w2) a1) / sqrt(w1 + w2)   (AC coefficient)
 * in FP64, in that order of operations.  mgs_raht_forward reads d_attr[C][ld]
 * (attributes in the order of the codes) and writes d_coef[C][ld]: column 0
 * the DC (the root's value), columns 1 .. N-1 the AC coefficients in the
 * order they are made (step by step; within a step by Morton code), FP32.
 * mgs_raht_inverse maps such coefficients back to attributes (the merges are
 * recomputed from the codes and undone in reverse).  The transform is
 * orthonormal: sum of squared attributes = sum of squared coefficients, and
 * the DC is sqrt(N) times the mean.  Workspace: mgs_raht_ws_bytes(N, C,
 * depth).  Errors: MGS_EINVAL (N outside [1, 2048 * 4096], C < 1, ld < N,
 * depth outside [1, 21], NULL pointers), MGS_EWORKSPACE; codes that do not
 * increase or exceed 2^(3 depth) raise MGS_ENONFINITE in the status word
 * (the coefficients are then unspecified).
 * ====================================================================== */
size_t mgs_raht_ws_bytes(int64_t N, int32_t C, int32_t depth);
int mgs_raht_forward(const uint64_t* d_codes, int64_t N, int32_t C, int32_t depth, const float* d_attr,
                     int64_t ld, float* d_coef, void* d_ws, size_t ws_bytes, void* stream);
int mgs_raht_inverse(const uint64_t* d_codes, int64_t N, int32_t C, int32_t depth, const float* d_coef,
                     int64_t ld, float* d_attr, void* d_ws, size_t ws_bytes, void* stream);

/* ======================================================================
 * Replayable launch sequences (hipGraph).
 *
 * mgs_graph_begin starts capturing `stream` (which must not be the legacy
 * default stream); the mgs_* device calls that follow on it are recorded
 * instead of run (host-side argument checks still run at capture time);
 * mgs_graph_end ends the capture and returns an executable graph in
 * *h_graph, which mgs_graph_launch replays on any stream with the same
 * pointers and sizes (buffer contents may change between replays) and
 * mgs_graph_destroy frees.  Calls that synchronise (mgs_status_fetch,
 * mgs_sweep_autotune) must not be captured.  Errors: MGS_EINVAL (NULL
 * stream or handle), MGS_EDEVICE (the runtime refused the capture).
 * ====================================================================== */
int mgs_graph_begin(void* stream);
int mgs_graph_end(void* stream, void** h_graph);
int mgs_graph_launch(void* graph, void* stream);
int mgs_graph_destroy(void* graph);

/* ======================================================================
 * Host side of the search (CPU).
 *
 * mgs_ilp_solve: the 0-1 ILP of the bit allocation (paper: equation "ilp"
 * of section "Solve the MINLP"): one option per class, minimise
 * sum err[c][x_c] subject to sum size[c][x_c] <= budget.  err is FP64
 * [ncls][nopt], size int64 [ncls][nopt] (>= 0).  Exact.  Among optimal
 * solutions the smaller total size wins, then the smaller option index in
 * class order.  Writes h_choice[ncls] (option index), *h_obj and *h_used.
 * Returns MGS_EINFEASIBLE when no allocation fits, MGS_EINVAL on bad
 * arguments (nopt outside [1, 255], non-finite err, negative size),
 * MGS_ELIMIT if the exact search would need more than 2e7 DP states.
 *
 * mgs_size_table: the ILP sizes from a sweep's bits table: size =
 * ceil(bits) + 72 metadata bits per group (two FP32 bounds and one byte of
 * bit-width) when mode == 0 (entropy size); n * b + 72 when mode == 1 (the
 * linear estimator P*Q of equation "size_estim").
 *
 * mgs_search: the reserve-ratio loop of the search algorithm over one
 * sweep's tables (host copies, layout of mgs_quant_sweep; paper: Algorithm 1
 * "Hyperparameter Optimization" and the discrete sampling of tau): for each
 * ratio t build the ILP over its C * ceil(k_t / G) groups (class order:
 * channel-major, then group), skip t when twice the all-8-bit size is below
 * the budget, solve, and choose the ratio with the smallest loss (ties:
 * larger k_t).  Ratios are solved in increasing order of their LP lower
 * bound and a ratio whose bound exceeds the best optimum found is not solved
 * (it cannot win); so is a ratio whose Lagrangian bound at the multiplier of
 * the smallest ratio that passes the doubled-8-bit test exceeds the loss of
 * that ratio's greedy allocation.  flags & MGS_SEARCH_ALL solves every
 * admissible ratio.
 * Writes h_best_t, the chosen bit-widths h_best_bits[C][ceil(k_best / G)]
 * (caller sizes it for the largest k), per ratio h_obj[t] / h_used[t] (NaN / 0
 * unless solved) and, if h_status is not NULL, h_status[t] (MGS_SEARCH_*).
 * Host work runs on up to `threads` threads (0 = all cores); each of them
 * keeps, between calls, the arrays of the largest LP bound it computed
 * (about 64 bytes per class and option).  Returns MGS_EINFEASIBLE when no
 * ratio is admissible, MGS_EINVAL when a loss is not finite or (size_mode 0)
 * an entropy size is negative or not finite, in any ratio.
 * ====================================================================== */
#define MGS_SEARCH_ALL 1            /* flags: solve every admissible ratio */
#define MGS_SEARCH_SOLVED 0         /* h_status values */
#define MGS_SEARCH_SKIPPED 1        /* doubled 8-bit size below the budget (or no groups) */
#define MGS_SEARCH_INFEASIBLE 2     /* even the smallest allocation exceeds the budget */
#define MGS_SEARCH_PRUNED 3         /* a lower bound above an attained loss: not solved */
#define MGS_SEARCH_UNCONVERGED 4    /* calibrated search: max_iter allocations, none within tol */

int mgs_ilp_solve(const double* h_err, const int64_t* h_size, int64_t ncls, int32_t nopt,
                  int64_t budget, uint8_t* h_choice, double* h_obj, int64_t* h_used);

int mgs_size_table(const double* h_bits, const int64_t* h_n, int64_t ncls, int32_t nb,
                   const uint8_t* h_bitlist, int32_t mode, int64_t* h_size);

int mgs_search(const mgs_sweep_desc* desc, const double* h_err, const double* h_bits,
               int64_t budget_bits, int32_t size_mode, int32_t threads, int32_t flags,
               int32_t* h_best_t, uint8_t* h_best_bits, double* h_obj, int64_t* h_used,
               int32_t* h_status);

/* mgs_search_streamed: mgs_search while the tables are still arriving on the
 * host (the same search and results, paper: Algorithm 1), for callers that
 * copy the tables ratio by ratio so that the host solver starts on the first
 * ratio instead of waiting for the whole copy.  h_events[t] (a hipEvent_t,
 * T of them, none NULL) must be recorded after the copies of ratio t's
 * slices of h_err and h_bits (slot range [t*C*Gmax, (t+1)*C*Gmax) of each);
 * the search reads ratio t only once it has completed.  It first waits for
 * the ratios in increasing k_t until one passes the doubled-8-bit test, then
 * polls the others and bounds each as it lands, so copying the smallest
 * ratio first and then the rest by decreasing k_t (the costlier bounds
 * first) starts it soonest.  The events stay owned by the caller.  Returns
 * MGS_EDEVICE when a wait or poll fails, otherwise as mgs_search (MGS_EINVAL
 * also for a NULL event). */
int mgs_search_streamed(const mgs_sweep_desc* desc, const double* h_err, const double* h_bits,
                        int64_t budget_bits, int32_t size_mode, int32_t threads, int32_t flags,
                        int32_t* h_best_t, uint8_t* h_best_bits, double* h_obj, int64_t* h_used,
                        int32_t* h_status, void* const* h_events);

/* ======================================================================
 * mgs_ilp_hierarchical: the paper's two-step solver (section "Solve the
 * MINLP", paragraph "Hierarchical Solver") for one ILP instance whose
 * classes are C channels x ng groups, channel-major (the class order of
 * mgs_search).  Step 1 picks one option per channel, shared by all of its
 * groups (channel loss and size: the sums over its groups, in group order),
 * exactly under the whole budget.  Step 2 gives channel c the share
 * S_c = floor(budget * Q_c / sum_c Q_c), Q_c the bit-width h_bitlist[] of its
 * step-1 option, and solves each channel's group-level ILP exactly within
 * S_c.  Writes h_choice[C * ng] (option indices), *h_obj and *h_used (sums
 * over the channels) and, when not NULL, h_chan_bits[C] (Q_c) and
 * h_chan_budget[C] (S_c).  The result never exceeds the budget and its loss
 * is never below the flat optimum of mgs_ilp_solve.  Returns MGS_EINFEASIBLE
 * when step 1 finds no allocation or a channel's share cannot hold its
 * cheapest allocation; MGS_EINVAL on bad arguments (as mgs_ilp_solve, plus
 * a bit-width of 0 in h_bitlist); MGS_ELIMIT as mgs_ilp_solve.
 *
 * mgs_search_calibrated: Algorithm 1 "Hyperparameter Optimization" with the
 * paper's linear size estimator (equation "size_estim": n * b bits per group
 * plus 72 metadata bits plus the calibration term S_delta) and the entropy
 * table as the measured size (ceil(bits) + 72 per group).  Per ratio t:
 * start from all groups at 8 bits (measured size: its entropy size, or
 * n * 8 + 72 per group when 8 is not listed); skip t when twice that size is
 * below the budget; then up to max_iter times: S_delta = measured - linear
 * estimate of the current allocation, solve the exact ILP with linear sizes
 * under budget - S_delta, measure the new allocation, and stop once
 * |measured - budget| * 10^6 < tol_ppm * budget (the paper uses 5 %,
 * tol_ppm = 50000).  Writes per ratio h_obj[t] (loss of the last
 * allocation, NaN if none), h_actual[t] (its measured size, or the all-8-bit
 * size), h_iters[t] (ILP solves) and, if not NULL, h_status[t]
 * (MGS_SEARCH_SOLVED when converged, _SKIPPED, _INFEASIBLE or
 * _UNCONVERGED); h_best_t and h_best_bits[C][ceil(k_best / G)] name the
 * converged ratio with the smallest loss (ties: larger k_t).  Returns
 * MGS_EINFEASIBLE when no ratio converged.
 * ====================================================================== */
int mgs_ilp_hierarchical(const double* h_err, const int64_t* h_size, int32_t C, int64_t ng,
                         int32_t nopt, const uint8_t* h_bitlist, int64_t budget, uint8_t* h_choice,
                         double* h_obj, int64_t* h_used, uint8_t* h_chan_bits, int64_t* h_chan_budget);

int mgs_search_calibrated(const mgs_sweep_desc* desc, const double* h_err, const double* h_bits,
                          int64_t budget_bits, int32_t tol_ppm, int32_t max_iter, int32_t threads,
                          int32_t* h_best_t, uint8_t* h_best_bits, double* h_obj, int64_t* h_actual,
                          int32_t* h_iters, int32_t* h_status);

#ifdef __cplusplus
}
#endif
#endif /* MGS_H */
