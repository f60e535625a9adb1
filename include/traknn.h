/*
 * traknn.h -- C ABI of the TRAKNN hot path on AMD Instinct MI355X (gfx950).
 *
 * TRAKNN (Coulaud & Faranda, "Efficient Trajectory Aware Spatiotemporal kNN
 * for Rare Meteorological Trajectory Detection") scores every length-L
 * trajectory of a sequence of T gridded fields by the mean squared distance to
 * its k nearest non-overlapping trajectories. This library computes, exactly
 * up to floating-point rounding:
 *
 *   d(i,j)   = ||x_i||^2 + ||x_j||^2 - 2 <x_i, x_j>           (Eq. 4, on MFMA)
 *   D_L(i,j) = sum_{m<L} d(i+m, j+m)                           (Eq. 2, via Eq. 5)
 *   N_t      = the k smallest (D_L(t,j), j) over j with |t-j| >= L
 *   s_t      = (1/k) sum_{j in N_t} D_L(t,j)                    (Eq. 3)
 *
 * and the gradient of sum_t w_t s_t with respect to the fields, the neighbour
 * sets held fixed; from the same lists, the scores for every k' <= k and the
 * local intrinsic dimension of every trajectory.
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers (hipMalloc'd or equivalent) owned
 *     by the caller. The library never allocates, frees or keeps device memory;
 *     scratch space is the caller's workspace buffer.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *     is enqueued asynchronously on it; results are ready when the stream is.
 *   - Indices are 0-based. Trajectory t covers fields t .. t+L-1, so a length-L
 *     run has n'_L = T - L + 1 trajectories.
 *   - The exclusion zone is |t - j| >= L (the paper's e = L - 1).
 *   - Ties in distance are broken by the smaller neighbour index, so neighbour
 *     lists are in ascending (distance, index) order and unique.
 *   - Return value: TRAKNN_OK (0) or a negative TRAKNN_ERR_* code. Arguments are
 *     validated before anything is enqueued; on an error nothing is enqueued.
 *     No C++ exception crosses this boundary. Asynchronous device faults
 *     surface at the caller's next synchronisation.
 *   - Inputs must be finite. This is not checked on the hot path.
 *   - There is no CPU fallback: every computation runs in this library's HIP
 *     kernels on the current device.
 */
#ifndef TRAKNN_H
#define TRAKNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define TRAKNN_OK 0
#define TRAKNN_ERR_INVALID_ARG (-1) /* a size, pointer, stride or alignment is invalid */
#define TRAKNN_ERR_UNSUPPORTED (-2) /* valid request outside what this library implements */
#define TRAKNN_ERR_WORKSPACE (-3)   /* workspace pointer NULL/misaligned or too small */
#define TRAKNN_ERR_HIP (-4)         /* a HIP runtime call or kernel launch failed */
#define TRAKNN_ERR_SCRATCH_LIMIT (-5) /* plan too large for traknn_knn_noalloc's scratch */

/* Precision of the Gram contraction (Eq. 4). In every mode the fields are first
 * shifted per grid cell by an FP64 mean over at most 2048 evenly strided
 * fields (distances are translation invariant, so any shift is exact; it only
 * removes the ~1e5 Pa offset before the reduced-precision products); squared
 * norms are FP64 sums over chunks of 512 cells of the represented vectors,
 * which the FP32 Gram accumulators subtract chunk by chunk so that they carry
 * -d/2 rather than the inner product (rounding errors scale with the distance,
 * not the norms); distances are stored FP32 and trajectory sums (Eq. 2/5) are
 * FP64.
 *   TRAKNN_FP32   : centred fields rounded to FP32, FP32 MFMA (32x32x2).
 *   TRAKNN_BF16X3 : centred fields split hi = bf16(x), lo = bf16(x - hi);
 *                   G = hi.hi' + hi.lo' + lo.hi' on BF16 MFMA (32x32x16) with FP32
 *                   accumulation (the lo.lo' term is dropped).
 * In every mode the FP32 accumulator is rounded once per MFMA, n times per
 * distance (n = 3 D / 16 for BF16X3, D / 2 for FP32, D / 16 for FP16), so the
 * accumulation error grows like sqrt(n) * 2^-24 relative to the distance. For
 * BF16X3 the largest errors observed are 2e-6 at D = 8192 and 6e-6 at
 * D = 50400; by that trend 1e-5 is reached near D = 1.5e5 (near D = 6e4 for
 * FP32, which rounds 2.7x as often).
 *   TRAKNN_FP16   : centred fields rounded to FP16, one FP16 MFMA pass (32x32x16).
 *                   Requires |x - mean| < 65504 in every cell. */
#define TRAKNN_FP32 0
#define TRAKNN_BF16X3 1
#define TRAKNN_FP16 2
/*   TRAKNN_FP64   : fused mode only. Eq. 4 with FP64 operands (the FP32 fields
 *                   shifted per cell by the FP64 sample mean), FP64 products
 *                   and sums on the vector ALUs, distances then rounded to
 *                   FP32 as the other modes store them. For the small grids
 *                   of the paper's PCA comparison (13 to 33 components), where
 *                   the contraction is too shallow for MFMA to pay and a
 *                   reduced-precision Gram loses accuracy to cancellation. */
#define TRAKNN_FP64 3

/* Modes (traknn_config.mode).
 *   TRAKNN_MODE_MATRIX : the distance matrix is materialised, whole or in bands
 *                        (row_batch), and a window pass reads it.
 *   TRAKNN_MODE_FUSED  : S-free. Each tile of the upper triangle (tiles overlap
 *                        by L - 1 fields, so every trajectory pair of a tile has
 *                        its L terms inside it) forms its trajectory distances
 *                        in LDS and offers every pair to both of its rows; each
 *                        (row, tile side) keeps at most k candidates within the
 *                        row's bound in a slot of its own, so only those reach
 *                        HBM. Tiles run in rounds of growing distance from
 *                        the diagonal; after each round a refresh merges a
 *                        row's slots into its running list, whose k-th is the
 *                        row's bound in the next round, and the final k come
 *                        from a select over the running list and the last
 *                        round's slots. The MFMA precisions form
 *                        every distance as the matrix mode does, so their lists
 *                        equal its lists wherever its FP64 window recurrence is
 *                        exact (distances whose exponents span fewer than about
 *                        29 bits). Single length
 *                        only (L_min == L_max), row_batch 0; precisions FP64
 *                        (vector FP64 tiles of 128 fields) and FP32 / BF16X3 /
 *                        FP16 (the MFMA Gram of 256 fields with the tile consumer
 *                        in its epilogue). */
#define TRAKNN_MODE_MATRIX 0
#define TRAKNN_MODE_FUSED 1

#define TRAKNN_MAX_L 16
#define TRAKNN_MAX_K 64

/* Problem description (set unused fields to 0).
 *   T, D        number of fields (time steps) and cells per field, >= 1.
 *   L_min,L_max trajectory lengths, 1 <= L_min <= L_max <= TRAKNN_MAX_L. One
 *               call emits neighbour lists for every L in [L_min, L_max]
 *               (L_min == L_max for a single length). Multi-length sweeps need
 *               L_min == 1.
 *   k           neighbours per trajectory, 1 <= k <= TRAKNN_MAX_K; every length
 *               must leave each row k candidates: T - L_max + 1 >= k + 2 L_max - 1.
 *   precision   TRAKNN_FP32, TRAKNN_BF16X3 or TRAKNN_FP16; TRAKNN_FP64 in
 *               fused mode.
 *   row_batch   0: the whole T x T distance matrix is held in the workspace
 *               (about 4 T^2 bytes) and only its upper-triangular tiles are
 *               contracted. > 0, a multiple of 8: band mode (row-batched
 *               streaming, for T whose matrix does not fit; the paper names
 *               out-of-core computation as future work, Sec. 7). Pass p owns
 *               the trajectories t0 .. t1 - 1, at most row_batch of them (the
 *               plan places the pass starts on multiples of 8 so that the
 *               passes' partly idle last rounds of tiles cost least), and
 *               computes the rows t0 .. t1 + L_max - 2 of the matrix against
 *               the columns from t0 on, only the 256 x 256 tiles holding
 *               entries above the diagonal, stored as rows and transposed.
 *               Its rows' later candidates come from the rows, and every
 *               later row's candidates among its trajectories from the
 *               transposed copy (the matrix is symmetric); both are merged
 *               into running lists, final for its rows when it ends. So the
 *               Gram work is that of the whole-matrix mode plus about one
 *               diagonal tile per 256-row block-row of each pass, and the
 *               workspace holds (row_batch + L_max - 1) rows of the matrix
 *               plus T rows of row_batch + L_max - 1 entries. Each distance
 *               above the diagonal comes from the same operands in the same
 *               order as in the whole-matrix mode, so whenever the window
 *               sums are exact (FP32 distances whose exponents span fewer
 *               than about 29 bits, as for field data) the results equal the
 *               whole-matrix mode's bit for bit, for any row_batch.
 *   mode        TRAKNN_MODE_MATRIX (0) or TRAKNN_MODE_FUSED (1), above.
 *   reserved    0. */
typedef struct {
  int64_t T;
  int64_t D;
  int32_t L_min;
  int32_t L_max;
  int32_t k;
  int32_t precision;
  int64_t row_batch;
  int32_t mode;      /* TRAKNN_MODE_MATRIX or TRAKNN_MODE_FUSED */
  int32_t reserved;  /* must be 0 */
} traknn_config;

typedef struct traknn_plan_s* traknn_plan_t;

/* Validate a configuration and size the workspace (paper, Algorithm 1 inputs:
 * fields, duration, exclusion zone, k; the batch size is chosen here).
 * Pure host code: makes no HIP call, so it can be used without a GPU.
 *   cfg              [in]  problem description (copied; caller keeps ownership).
 *   out              [out] new plan handle; immutable; free with
 *                          traknn_plan_destroy. Not for concurrent use from two
 *                          threads when timing is enabled.
 *   workspace_bytes  [out] device bytes the caller must provide to traknn_knn
 *                          and traknn_score_backward (one size covers both).
 * Errors: INVALID_ARG for NULL pointers, sizes out of range or a row_batch that
 * is negative or not a multiple of 8; UNSUPPORTED for a multi-length sweep with
 * L_min != 1, or a D whose 256-field
 * Gram operand panel would reach 2 GiB (D >= 2^21 for FP32 and BF16X3,
 * D >= 2^22 for FP16). */
int traknn_plan(const traknn_config* cfg, traknn_plan_t* out,
                size_t* workspace_bytes);

/* Free a plan's host memory (and any HIP timing events it created).
 * Errors: INVALID_ARG for NULL. */
int traknn_plan_destroy(traknn_plan_t plan);

/* Exact exclusion-zone kNN over trajectories (paper, Algorithm 1 stages 1-3:
 * Eq. 4 Gram distances for the upper-triangular tile pairs -- or, in band
 * mode, for each pass's rows against the later columns -- Eq. 5 diagonal
 * recurrence, k smallest with |t - j| > e).
 *   X         [in]  T x D fields, FP32, row-major with row stride ldx floats;
 *                   16-byte aligned, ldx >= D, ldx % 4 == 0.
 *   workspace [in]  >= workspace_bytes from traknn_plan, 256-byte aligned;
 *                   contents are scratch (overwritten).
 *   nbr_idx   [out] int32 [L_max-L_min+1][T-L_min+1][k]; block for length L is
 *                   at offset (L-L_min)*(T-L_min+1)*k. Row t lists the k
 *                   neighbours of trajectory t in ascending (distance, index).
 *                   Rows t >= T-L+1 (which do not exist for that L) hold -1.
 *   nbr_dist  [out] FP64, same shape: D_L(t, nbr_idx) (squared); +inf in
 *                   non-existent rows.
 * Errors: INVALID_ARG (NULL, stride, alignment), WORKSPACE, HIP. */
int traknn_knn(traknn_plan_t plan, const float* X, int64_t ldx, void* workspace,
               size_t workspace_bytes, int32_t* nbr_idx, double* nbr_dist,
               void* stream);

/* Fixed scratch, in bytes, of traknn_knn_noalloc: a plan qualifies when its
 * workspace_bytes from traknn_plan is at most this (for example T = 2048
 * fields of D = 1024 cells, whole-matrix mode). */
#define TRAKNN_NOALLOC_MAX_BYTES (32u << 20)

/* traknn_knn without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). The scratch is a fixed TRAKNN_NOALLOC_MAX_BYTES
 * array in the library's device memory, one per GPU, created with the code
 * object and held until the process ends; its address is looked up on the
 * first call on each device. The call allocates and frees nothing. Results
 * equal traknn_knn's for the same plan and inputs bit for bit (same kernels,
 * same arithmetic). All calls on one GPU share that GPU's array, so calls
 * that overlap in time on one GPU (two streams, two threads) race and give
 * undefined results; calls on one stream are ordered and safe. The kernels
 * write every scratch byte they read, so nothing needs clearing between
 * calls.
 *   plan, X, ldx, nbr_idx, nbr_dist, stream: as for traknn_knn.
 * Errors: INVALID_ARG; SCRATCH_LIMIT if the plan's workspace_bytes exceed
 * TRAKNN_NOALLOC_MAX_BYTES (nothing enqueued); HIP (including a failed
 * scratch lookup); UNSUPPORTED for a device ordinal of 64 or more. */
int traknn_knn_noalloc(traknn_plan_t plan, const float* X, int64_t ldx, int32_t* nbr_idx,
                       double* nbr_dist, void* stream);

/* Rarity score (paper, Eq. 3): s_t = (1/k) * sum of the row of nbr_dist, summed
 * in rank order in FP64.
 *   nbr_dist [in]  as written by traknn_knn for the same plan.
 *   scores   [out] FP64 [L_max-L_min+1][T-L_min+1]; NaN in non-existent rows.
 * Errors: INVALID_ARG, HIP. */
int traknn_score(traknn_plan_t plan, const double* nbr_dist, double* scores,
                 void* stream);

/* Rarity scores for every neighbour count k' = 1..k from one search (paper,
 * Eq. 3 and the discussion of reusing one k-NN pass for several k; k' = 1 is
 * the trajectory analogue of the matrix profile). The lists of traknn_knn are
 * sorted by (distance, index), so the k' nearest are their first k' entries:
 *   scores[l][t][q] = (1/(q+1)) * sum_{r<=q} nbr_dist[l][t][r]
 * summed in rank order in FP64; scores[l][t][k-1] equals traknn_score's s.
 *   nbr_dist [in]  as written by traknn_knn for the same plan.
 *   scores   [out] FP64 [L_max-L_min+1][T-L_min+1][k]; NaN in non-existent rows.
 * Errors: INVALID_ARG, HIP. */
int traknn_score_prefix(traknn_plan_t plan, const double* nbr_dist, double* scores,
                        void* stream);

/* Local intrinsic dimension of every trajectory for every k' = 1..k from one
 * search: the maximum-likelihood kNN estimator of Levina and Bickel, which
 * the paper applies to trajectories with k in {20, 30, 40} (Sec. 5.1,
 * intrinsic dimension study). With the sorted squared distances of a list,
 *   out[l][t][q] = 2 q / sum_{j<q} ln(nbr_dist[l][t][q] / nbr_dist[l][t][j])
 * for k' = q + 1 = 2..k (the Euclidean log-ratio is half the squared one), in
 * FP64. out[l][t][0] (k' = 1, no ratio) is NaN. Degenerate lists follow IEEE
 * arithmetic: a zero distance below a positive k'-th gives 0, a zero k'-th
 * distance NaN, k' equal distances +inf. Averaging over t (and over several
 * k') gives the paper's mean local dimension; that reduction is the caller's.
 *   nbr_dist [in]  as written by traknn_knn for the same plan.
 *   out      [out] FP64 [L_max-L_min+1][T-L_min+1][k]; NaN in non-existent rows.
 * Errors: INVALID_ARG, HIP. */
int traknn_local_dim(traknn_plan_t plan, const double* nbr_dist, double* out, void* stream);

/* Gradient of F = sum_t grad_scores[t] * s_t with respect to X, the neighbour
 * sets held fixed (differentiating Eq. 2 inside Eq. 3):
 *   dF/dx_a = (2/k) sum_t w_t sum_{j in N_t} sum_{m<L}
 *             ([a = t+m] - [a = j+m]) (x_{t+m} - x_{j+m}).
 * Deterministic: every row of grad_X is gathered in a fixed order, no atomics
 * on floating-point data. No distance is needed, so none is stored or
 * recomputed beyond the field differences themselves.
 *   X           [in]  the fields passed to traknn_knn (same layout rules).
 *   nbr_idx     [in]  int32 [T-L+1][k] from traknn_knn (single length only).
 *   grad_scores [in]  FP64 [T-L+1] upstream weights w_t.
 *   grad_X      [out] FP32 T x D, row stride ldg (ldg >= D); every row written
 *                     (zeros where no term touches it).
 *   workspace   [in]  256-byte aligned scratch of at least the bytes
 *                     traknn_backward_workspace reports (the traknn_knn
 *                     workspace always suffices); overwritten.
 * Errors: INVALID_ARG, WORKSPACE, HIP; UNSUPPORTED if L_min != L_max. */
int traknn_score_backward(traknn_plan_t plan, const float* X, int64_t ldx,
                          const int32_t* nbr_idx, const double* grad_scores,
                          float* grad_X, int64_t ldg, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Device bytes traknn_score_backward needs: the layout puts its scratch at
 * the start of the workspace, so a buffer of this size (or the whole
 * traknn_knn workspace, which is never smaller) serves it. Lets a caller free
 * the forward workspace between the forward and the backward pass.
 *   bytes [out] the size, at most workspace_bytes of traknn_plan.
 * Errors: INVALID_ARG for NULL. */
int traknn_backward_workspace(traknn_plan_t plan, size_t* bytes);

/* Band mode's passes, as the plan placed them (row_batch above): the first
 * trajectory row of each pass, in increasing order, each pass at most
 * row_batch rows and the last ending at T - L_min + 1. Pure host call.
 *   starts [out] host array; the first min(*count, cap) starts are written
 *                (may be NULL when cap is 0).
 *   cap    [in]  entries starts can hold.
 *   count  [out] number of passes (0 in the whole-matrix and fused modes).
 * Errors: INVALID_ARG for a NULL plan or count, a negative cap, or NULL
 * starts with cap > 0. */
int traknn_band_passes(traknn_plan_t plan, int64_t* starts, int64_t cap, int64_t* count);

/* Static description of a status code; never NULL. */
const char* traknn_status_string(int status);

/* Per-stage timing of the most recent traknn_knn call on this plan.
 * When enabled, traknn_knn records HIP events on its stream between its
 * stages; traknn_stage_times then waits for the last event and returns the
 * elapsed milliseconds of each stage in launch order:
 *   0 centre statistics, 1 centre/convert/norms, 2 Gram + distance epilogue
 *   (in band mode: all passes, each Gram + window + merge),
 *   3 window recurrence + partial top-k, 4 top-k merge (both about 0 in band
 *   mode).
 *   enable   [in]  nonzero to record events from the next traknn_knn call on.
 *   ms       [out] host array of at least max_stages doubles.
 *   n_stages [out] number of stages written.
 * Errors: INVALID_ARG; UNSUPPORTED if timing was not enabled or no call has
 * been timed yet; HIP. */
int traknn_set_timing(traknn_plan_t plan, int enable);
int traknn_stage_times(traknn_plan_t plan, double* ms, int max_stages,
                       int* n_stages);

#ifdef __cplusplus
}
#endif

#endif /* TRAKNN_H */
