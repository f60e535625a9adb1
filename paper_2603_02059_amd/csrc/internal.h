// Internal declarations shared by the TRAKNN HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "traknn.h"

namespace traknn {

// ---------------------------------------------------------------------------
// Gram tiling (Eq. 4 stage). One workgroup owns a GRAM_TILE x GRAM_TILE block
// of the distance matrix; every K stage moves GRAM_ROW_BYTES of each of the
// 2 * GRAM_TILE operand rows through LDS.
// ---------------------------------------------------------------------------
constexpr int GRAM_TILE = 256;
constexpr int GRAM_THREADS = 512;
constexpr int GRAM_ROW_BYTES = 128;
constexpr int GRAM_STAGES = 2;
constexpr int GRAM_GROUP_ROWS = 4;  // block-rows per L2 locality group
constexpr int NUM_XCD = 8;

// K elements one stage covers: 32 FP32 values, 32 (hi, lo) BF16 pairs or 64
// FP16 values -- always 128 bytes of a centred row.
inline int stage_k(int precision) { return precision == TRAKNN_FP16 ? 64 : 32; }
inline int elem_bytes(int precision) { return precision == TRAKNN_FP16 ? 2 : 4; }

// K elements per norm chunk: the Gram accumulators subtract the two rows'
// squared norms over each chunk once it is done (distance-form accumulation),
// so the FP32 accumulators hold -d/2 of the finished chunks instead of the
// inner product, and their rounding errors scale with the distance, not with
// the norms. A multiple of every stage depth.
constexpr int GRAM_CHUNK = 512;
__host__ __device__ inline int64_t norm_chunks(int64_t Dpad) { return (Dpad + GRAM_CHUNK - 1) / GRAM_CHUNK; }

// Per-stage event slots for optional timing.
constexpr int NUM_STAGES = 5;
constexpr int COLSTAT_ROWS = 128;  // rows per partial column-sum block
// The per-cell shift is the mean of at most COLSTAT_SAMPLE evenly strided rows
// (rows 0, s, 2s, ... with s = ceil(T / COLSTAT_SAMPLE)).
constexpr int64_t COLSTAT_SAMPLE = 2048;
inline int64_t colstat_stride(int64_t T) { return (T + COLSTAT_SAMPLE - 1) / COLSTAT_SAMPLE; }
inline int colstat_chunks(int64_t T) {
  const int64_t s = colstat_stride(T);
  return (int)(((T + s - 1) / s + COLSTAT_ROWS - 1) / COLSTAT_ROWS);
}

// Fused (S-free) mode. Tiles of FUSED_F64_TILE (FP64 vector kernel) or
// GRAM_TILE (MFMA Gram) snapshot rows and columns pair B = tile - (L - 1)
// trajectories (rounded down to a multiple of 4 for the MFMA tiles) with B,
// so consecutive tiles overlap by L - 1 fields; nbt = ceil(n' / B)
// block-rows. The tiles run in rounds of offsets J - I: the first,
// [0, FUSED_FIRST_END), keeps each recipient's exact k nearest per tile
// (no bound yet); every later round, [blo, bhi), keeps only the candidates
// within each row's bound, which a refresh after each round lowers to the
// k-th of everything seen so far.
constexpr int FUSED_F64_TILE = 128;
constexpr int FUSED_ROUNDS = 4;
// The first round is offsets [0, 2). Later rounds (tile offsets 2 and up)
// hold no pair within the exclusion zone, whose width L is below the block
// stride B, and their consumer skips its test.
constexpr int FUSED_FIRST_END = 2;
static_assert(FUSED_FIRST_END >= 2, "the first round covers tile offsets 0 and 1");
// Ends of the second and third rounds: by default 8 and 32; the planner moves
// them within [6, 12] and [24, 48] to fill the launches' last waves of tiles.
constexpr int FUSED_END_DEFAULT[2] = {12, 48};
// Compute units of an MI355X: the tiles resident at once are this many times
// the workgroups of a fused tile kernel per CU (1 MFMA, 2 FP64).
constexpr int NUM_CU = 256;
constexpr int FUSED_F64_PER_CU = 2;
struct FusedGeom {
  int T, np, L, k, B, nbt;
  int blo, bhi;  // the launch's offsets J - I: [blo, bhi)
  int rend[2];   // ends of the second and third rounds
};
// Per-row slots of candidate lists: row t meets exactly nbt + 1 tile-sides
// (the column sides of tiles (I', I_t), I' <= I_t, in slots I'; the row sides
// of tiles (I_t, J), J >= I_t, in slots J + 1, with I_t its block-row), and
// each writes its list of at most k candidates, unsorted, to its own slot.
struct FusedSlots {
  int32_t* cnt;  // [n'][nslot] entries in each slot
  double* d;     // [n'][nslot][k] distances
  int32_t* i;    // [n'][nslot][k] neighbour indices
  int nslot, k;
};

struct Layout {
  // backward first: traknn_score_backward only needs the prefix up to bw_end
  size_t bw_zero, bw_ptr, bw_rev, bw_end;
  size_t mu_part, mu, ncs, xc, S, ST, part_d, part_i;  // forward
  size_t cpart_d, cpart_i;                             // band mode: column windows
  size_t f_bound, f_cnt, f_sd, f_si, f_rd, f_ri;       // fused mode
  size_t total;
};

}  // namespace traknn

struct traknn_plan_s {
  traknn_config cfg;
  int64_t T, D;
  int64_t Dpad;      // D rounded up to the Gram stage depth (zero padded)
  int64_t Tpad;      // T rounded up to GRAM_TILE, plus one tile in band mode (zero rows)
  int64_t ldS;       // row stride of the distance matrix (or band), floats
  int64_t np0;       // T - L_min + 1: rows of every output block
  int NL;            // L_max - L_min + 1
  int nb;            // ceil(T / GRAM_TILE) block-columns
  int64_t ntiles;    // nb (nb + 1) / 2 upper-triangular tile pairs
  int64_t rb;        // band mode: at most this many trajectory rows per pass (0: whole matrix)
  std::vector<int64_t> band_t0;  // band mode: the passes' first trajectory rows
  int64_t band_rows; // band mode: rows of S held, rb + L_max - 1 (at most T)
  int64_t ldST;      // band mode: row stride of the transposed band, floats
  int tchunks;       // partial column-sum blocks of the sampled rows
  int fused;         // fused (S-free) mode
  traknn::FusedGeom fg;  // fused mode: tile geometry
  int win_splits;    // column splits (waves) per window row block (W)
  int col_splits;    // band mode: the same for the column windows
  traknn::Layout lay;
  // timing
  int timing;
  int timed_calls;
  int events_ready;
  hipEvent_t ev[traknn::NUM_STAGES + 1];
};

namespace traknn {

// prep.hip
hipError_t launch_colstats(const float* X, int64_t ldx, int64_t T, int64_t D,
                           int tchunks, double* mu_part, double* mu,
                           hipStream_t s);
hipError_t launch_centre_convert(const float* X, int64_t ldx, int64_t T,
                                 int64_t D, int64_t Tpad, int64_t Dpad,
                                 int precision, const double* mu, void* xc,
                                 float* ncs, hipStream_t s);
// gram.hip
hipError_t launch_gram(const void* xc, const float* ncs, int64_t T, int64_t Tpad,
                       int64_t Dpad, int nb, int64_t ntiles, int precision,
                       float* S, int64_t ldS, hipStream_t s);
// Band mode: rows a_row0 .. a_row0 + rows_out - 1 (nbi = ceil(rows_out / 256)
// block-rows) against the columns of block-columns J0 = a_row0 / 256 .. nb -
// 1. Only the tiles J >= J0 + I, those that hold entries above the diagonal,
// are computed (ntiles = nbi nb' - nbi (nbi - 1) / 2 with nb' = nb - J0); the
// rest of both buffers is left unwritten. Field j of row a_row0 + i goes to
// S[i * ldS + j - 256 J0] and, transposed, to ST[(j - 256 J0) * ldST + i].
// a_row0 must be a multiple of 8, nbi <= nb', a_row0 + nbi * 256 <= Tpad and
// ldST >= rows_out, a multiple of 4.
hipError_t launch_gram_band(const void* xc, const float* ncs, int64_t T, int64_t Tpad,
                            int64_t Dpad, int nb, int64_t ntiles, int precision,
                            int64_t a_row0, int nbi, int64_t rows_out, int J0, float* S,
                            int64_t ldS, float* ST, int64_t ldST, hipStream_t s);
// window_topk.hip
hipError_t launch_window_topk(const float* S, int64_t ldS, int64_t T, int L_min,
                              int L_max, int k, int splits, double* part_d,
                              int32_t* part_i, hipStream_t s);
hipError_t launch_merge(const double* part_d, const int32_t* part_i, int64_t T,
                        int L_min, int L_max, int k, int splits, int32_t* idx,
                        double* dist, hipStream_t s);
// The part of the matrix a window launch sees: S holds rows s0 .. s_end - 1
// (its row 0 is row s0) and column c at column c - col0; candidates are the
// columns c_lo .. c_hi - 1 at diagonal offsets j - i in dmin .. dmax, values
// are read in the columns c_lo .. v_end - 1 and relied on only on the
// diagonals of that offset range. The whole matrix is {0, T, 0, 0, T, T, -T, T}.
struct WindowRange {
  int64_t s0, s_end, col0, c_lo, c_hi, v_end, dmin, dmax;
};
// The lists of trajectory rows t0 .. t0 + nt - 1 (counted for L_min; fewer for
// longer L) over the candidates of r go to partial lists indexed from t0:
// [split][length][row - t0][k].
hipError_t launch_window_band(const float* S, int64_t ldS, int64_t T, int L_min,
                              int L_max, int k, int splits, const WindowRange& r,
                              int64_t t0, int64_t nt, double* part_d, int32_t* part_i,
                              hipStream_t s);
// One window launch's partial lists, as the merge reads them: W splits of the
// rows t0 .. t0 + nt - 1.
constexpr int MERGE_MAX_SPLITS = 16;
struct MergeSet {
  const double* d;
  const int32_t* i;
  int W, nt;
};
// Rows t0 .. t0 + nt - 1 of idx and dist become the k smallest of the lists
// of sets a and b (both indexed from t0, each covering its first nt rows) and,
// for the rows below acc_end, of the lists already there.
hipError_t launch_merge_band(const MergeSet& a, const MergeSet& b, int64_t T, int L_min,
                             int L_max, int k, int64_t t0, int64_t nt, int64_t acc_end,
                             int32_t* idx, double* dist, hipStream_t s);
hipError_t launch_score(const double* dist, int64_t T, int L_min, int L_max,
                        int k, double* scores, hipStream_t s);
hipError_t launch_score_prefix(const double* dist, int64_t T, int L_min, int L_max,
                               int k, double* out, hipStream_t s);
hipError_t launch_local_dim(const double* dist, int64_t T, int L_min, int L_max, int k,
                            double* out, hipStream_t s);
// backward.hip
// zeroed: 2 (T - L + 1) + T int32 scratch the launch clears itself; ptr:
// T - L + 2 int32; rev: (T - L + 1) k int32.
hipError_t launch_backward(const float* X, int64_t ldx, int64_t T, int64_t D,
                           int L, int k, const int32_t* idx, const double* w,
                           float* g, int64_t ldg, int32_t* zeroed, int32_t* ptr,
                           int32_t* rev, hipStream_t s);

// Fused mode with the MFMA Gram: the tiles of offsets [g.blo, g.bhi), over
// 256-field tiles of stride g.B; establish: each recipient's exact k nearest
// per tile (no bound), else only candidates within `bound`.
hipError_t launch_gram_fused(const void* xc, const float* ncs, int64_t T, int64_t Tpad,
                             int64_t Dpad, int precision, const FusedGeom& g, bool establish,
                             const double* bound, const FusedSlots& out, hipStream_t s);
// fused.hip
int64_t fused_band_tiles(const FusedGeom& g);  // tiles of offsets [g.blo, g.bhi)
hipError_t launch_fused_f64(const float* X, int64_t ldx, int D, const double* mu,
                            const FusedGeom& g, bool establish, const double* bound,
                            const FusedSlots& out, hipStream_t s);
// After a round of offsets [hlo, hhi): each row's running list (k sorted
// entries, read only when hlo > 0) merged with the round's slots, and its
// bound set to the list's k-th (+inf while it holds fewer than k).
hipError_t launch_slots_refresh(const FusedGeom& g, const FusedSlots& out, double* bound,
                                double* run_d, int32_t* run_i, int hlo, int hhi,
                                hipStream_t s);
// The final lists: the running list (when hlo > 0) merged with the slots of
// the tiles of offsets hlo and up.
hipError_t launch_slots_final(const FusedGeom& g, const FusedSlots& out, const double* run_d,
                              const int32_t* run_i, int hlo, int32_t* idx, double* dist,
                              hipStream_t s);

// Window stage sizing shared by the planner and the launcher: LDS bytes of a
// workgroup of W waves for a pass of G lengths whose longest is L, k neighbours.
size_t window1_lds_bytes(int L, int G, int k, int W);
// Lengths a multi-length sweep handles per pass over S (1 to 5; compile-time
// tuning knob). Each pass reads S once for all of its lengths.
#ifndef TRAKNN_WIN_LENGTHS_PER_PASS
#define TRAKNN_WIN_LENGTHS_PER_PASS 2
#endif
constexpr int WINDOW_LENGTHS_PER_PASS = TRAKNN_WIN_LENGTHS_PER_PASS;
static_assert(WINDOW_LENGTHS_PER_PASS >= 1 && WINDOW_LENGTHS_PER_PASS <= 5,
              "one to five lengths per window pass");
// Rows per window block (a multiple of the 8-step group; compile-time tuning
// knob, 8 measured best on the full workload).
#ifndef TRAKNN_WINDOW1_ROWS
#define TRAKNN_WINDOW1_ROWS 8
#endif
constexpr int WINDOW1_ROWS = TRAKNN_WINDOW1_ROWS;

}  // namespace traknn
