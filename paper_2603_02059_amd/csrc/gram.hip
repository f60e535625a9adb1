// Symmetric Gram product and distance epilogue (paper, Algorithm 1 stage 1 and
// Eq. 4): for every tile pair I <= J of 256 fields,
//   d(i,j) = N_i + N_j - 2 <x_i, x_j>   (MFMA, FP32 accumulation),
// stored FP32 at (i,j) and (j,i). Only the upper triangle of tile pairs is
// computed, which halves the contraction as the paper's symmetric batching
// does.
//
// Distance-form accumulation: K runs in chunks of GRAM_CHUNK elements, and once
// a chunk's products are in the accumulators, one extra FP32 MFMA of depth 2
// adds -(N_i^c + N_j^c)/2, the chunk's squared norms (FP64 sums rounded to
// FP32, from the centring pass). The accumulators then hold -d/2 over the
// finished chunks, so they never grow much beyond the distance itself: their
// FP32 rounding errors scale with d + N/(number of chunks) instead of with the
// norms N, which for near neighbours are several times larger than d. The
// epilogue only scales by -2.
//
// Tiling for gfx950: 512 threads = 8 wave64s in a 2x4 arrangement, each wave
// owning a 128x64 block = 4x2 MFMA 32x32 blocks held in accumulation
// registers. Every K stage brings 128 bytes of each of the 512 operand rows
// into LDS (2 x 32 KB), double buffered. Rows are stored with their eight
// 16-byte chunks XOR-swizzled by the row index so that the ds_read_b128
// fragment loads of 32 consecutive rows spread over all banks.
//
// Workgroups are mapped XCD-aware: the hardware deals consecutive workgroup
// ids round-robin to the 8 XCDs, so each XCD is handed a contiguous run of a
// grouped tile order (4 block-rows x successive block-columns). The ~32 tiles
// an XCD runs at once then share 4 A panels and ~8 B panels in its L2.
//
// Band mode (row-batched streaming, for T whose T x T matrix does not fit):
// the kernel fills a band of rows a_row0 .. a_row0 + rows_out - 1 against the
// columns from block-column J0 on (the columns before it belong to earlier
// bands), every tile (I, J) of the rectangle that holds an entry above the
// diagonal computed directly. It is stored twice: as rows, into a buffer
// whose row 0 is field a_row0 and column 0 field 256 J0, and transposed, so
// that the later fields' rows of the band's columns are contiguous too.
#include <type_traits>

#include "dist_clamp.h"
#include "fused_walk.h"
#include "internal.h"

namespace traknn {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TILE = GRAM_TILE;
constexpr int RB = GRAM_ROW_BYTES;          // bytes per row per stage
constexpr int OPER_BYTES = TILE * RB;       // one operand tile in LDS (32 KB)
// Wave grid of a workgroup: WAVES_M x WAVES_N waves, each owning a
// WT_M x WT_N block of the 256 x 256 tile in 32x32 MFMA blocks.
constexpr int WAVES_M = 2;
constexpr int WAVES_N = GRAM_THREADS / 64 / WAVES_M;
constexpr int WT_M = TILE / WAVES_M, WT_N = TILE / WAVES_N;
constexpr int BM = WT_M / 32, BN = WT_N / 32;  // MFMA blocks per wave
static_assert(WT_M == 128, "the epilogue parks 32-row bands of 128-row wave tiles");
// s_waitcnt immediate waiting for vmcnt == 0 only (expcnt, lgkmcnt at max)
constexpr int VMCNT0 = 0x0F70;
// s_waitcnt immediate for vmcnt <= n (expcnt, lgkmcnt at max)
constexpr int vmcnt_le(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }
constexpr int EPI_PITCH = 36;  // floats per parked accumulator column (32 + 4)
static_assert((GRAM_THREADS / 64) * (TILE / (GRAM_THREADS / 64 / 2)) * EPI_PITCH * 4 <=
                  GRAM_STAGES * 2 * TILE * RB,
              "epilogue staging must fit in the operand LDS");
constexpr int NORM_LDS = 2 * 2 * TILE * 4;  // two chunks' norms of the I and J rows

// Physical 16-byte slot of logical chunk `chunk` in LDS row `row`. The XOR key
// (row & 7) ^ ((row >> 3) & 3) gives any 8 aligned consecutive rows 8
// distinct slots, any 16 aligned rows 16 distinct (row parity, slot) pairs and
// any 32 aligned rows 32 distinct (row mod 4, slot) pairs, so ds_read_b128 of
// 32 consecutive rows is conflict-free whether the LDS serves 8, 16 or 32
// lanes per pass. It ignores row bits 5 and up, so rows 32 apart share a key.
__device__ __forceinline__ int swz_key(int row) { return (row & 7) ^ ((row >> 3) & 3); }
__device__ __forceinline__ int swz(int row, int chunk) {
  return ((chunk ^ swz_key(row)) << 4);
}

// Tile id -> (I, J), I <= J < nb, I < nrows (<= nb), in the XCD-aware
// grouped order described above; ntiles = nrows nb - nrows (nrows - 1) / 2.
__device__ __forceinline__ bool decode_tile(int64_t wg, int nb, int nrows, int64_t ntiles,
                                            int& I, int& J) {
  const int64_t per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  const int64_t lin = (wg % NUM_XCD) * per + wg / NUM_XCD;
  if (lin >= ntiles) return false;
  int64_t u = lin;
  for (int I0 = 0; I0 < nrows; I0 += GRAM_GROUP_ROWS) {
    const int gm = nrows - I0 < GRAM_GROUP_ROWS ? nrows - I0 : GRAM_GROUP_ROWS;
    const int64_t cnt = (int64_t)gm * nb - ((int64_t)gm * I0 + (int64_t)gm * (gm - 1) / 2);
    if (u < cnt) {
      const int64_t head = (int64_t)gm * (gm - 1) / 2;
      if (u < head) {
        // head columns J = I0 + m hold m + 1 rows each
        int m = 0;
        while ((int64_t)(m + 1) * (m + 2) / 2 <= u) ++m;
        J = I0 + m;
        I = I0 + (int)(u - (int64_t)m * (m + 1) / 2);
      } else {
        const int64_t v = u - head;
        J = I0 + gm - 1 + (int)(v / gm);
        I = I0 + (int)(v % gm);
      }
      return true;
    }
    u -= cnt;
  }
  return false;
}

// Scheduling-group masks for __builtin_amdgcn_sched_group_barrier.
constexpr int SG_MFMA = 0x008;
constexpr int SG_DS_READ = 0x100;

// Operand fragments of half a K stage for one wave: two 16-byte chunks of
// each of the wave's 128 A rows and 64 B rows. Lane half h (lanes 32h ..
// 32h+31) supplies k-group h of every MFMA; A and B use the same assignment,
// so which elements a group holds does not matter. Part p of a stage:
//   BF16x3: the 16 (hi, lo) pairs of k-slice p: x0/y0 = hi (chunk 4p + 2h),
//           x1/y1 = lo (chunk 4p + 2h + 1); MFMAs hi.hi', hi.lo', lo.hi'.
//   FP16:   k-slices 2p, 2p+1 (chunks 4p + h, 4p + 2 + h), one MFMA each.
//   FP32:   chunks 4p + h, 4p + 2 + h, four depth-2 MFMAs each.
template <int PREC>
struct Part {
  using V = typename std::conditional<PREC == TRAKNN_BF16X3, bf16x8,
            typename std::conditional<PREC == TRAKNN_FP16, f16x8, f32x4>::type>::type;
  V x0[BM], x1[BM], y0[BN], y1[BN];
};
constexpr int PART_READS = 2 * (BM + BN);
template <int PREC>
constexpr int part_mfmas() {
  return PREC == TRAKNN_BF16X3 ? 3 * BM * BN : PREC == TRAKNN_FP16 ? 2 * BM * BN : 8 * BM * BN;
}

// Lane offsets of a part's two chunks in the A and B tiles of a stage buffer.
// The wave's rows wm*WT_M + q*32 + r32 (A) and wn*WT_N + q*32 + r32 (B) share
// the swizzle key of r32, so q is an immediate offset of q * 32 rows.
struct PartOffsets {
  int a0, a1, b0, b1;
};
template <int PREC>
__device__ __forceinline__ PartOffsets part_offsets(int p, int wm, int wn, int lane) {
  const int r32 = lane & 31, h = lane >> 5;
  const int key = swz_key(r32);
  const int c0 = 4 * p + (PREC == TRAKNN_BF16X3 ? 2 * h : h);
  const int c1 = c0 + (PREC == TRAKNN_BF16X3 ? 1 : 2);
  PartOffsets o;
  o.a0 = (wm * WT_M + r32) * RB + ((c0 ^ key) << 4);
  o.a1 = (wm * WT_M + r32) * RB + ((c1 ^ key) << 4);
  o.b0 = OPER_BYTES + (wn * WT_N + r32) * RB + ((c0 ^ key) << 4);
  o.b1 = OPER_BYTES + (wn * WT_N + r32) * RB + ((c1 ^ key) << 4);
  return o;
}

template <int PREC>
__device__ __forceinline__ void read_part(const char* __restrict__ buf, const PartOffsets& o,
                                          Part<PREC>& P) {
  using V = typename Part<PREC>::V;
#pragma unroll
  for (int q = 0; q < BM; ++q) {
    P.x0[q] = *(const V*)(buf + o.a0 + q * 32 * RB);
    P.x1[q] = *(const V*)(buf + o.a1 + q * 32 * RB);
  }
#pragma unroll
  for (int q = 0; q < BN; ++q) {
    P.y0[q] = *(const V*)(buf + o.b0 + q * 32 * RB);
    P.y1[q] = *(const V*)(buf + o.b1 + q * 32 * RB);
  }
}

template <int PREC>
__device__ __forceinline__ void mfma_part(const Part<PREC>& P, f32x16 (&acc)[BM][BN]) {
  if constexpr (PREC == TRAKNN_BF16X3) {
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn) {
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(P.x0[bm], P.y0[bn], acc[bm][bn], 0, 0, 0);
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(P.x0[bm], P.y1[bn], acc[bm][bn], 0, 0, 0);
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(P.x1[bm], P.y0[bn], acc[bm][bn], 0, 0, 0);
      }
  } else if constexpr (PREC == TRAKNN_FP16) {
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(P.x0[bm], P.y0[bn], acc[bm][bn], 0, 0, 0);
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(P.x1[bm], P.y1[bn], acc[bm][bn], 0, 0, 0);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn)
          acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(P.x0[bm][e], P.y0[bn][e], acc[bm][bn], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int bm = 0; bm < BM; ++bm)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn)
          acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(P.x1[bm][e], P.y1[bn][e], acc[bm][bn], 0, 0, 0);
  }
}

// Interleave a part's PART_READS reads with MF MFMAs: one MFMA, then two reads
// per MFMA, then the remaining MFMAs, so the reads are done well before the
// fragments are needed.
template <int MF, int I = 0>
__device__ __forceinline__ void interleave_reads() {
  if constexpr (I == 0) __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
  if constexpr (I < PART_READS) {
    __builtin_amdgcn_sched_group_barrier(SG_DS_READ, 2, 0);
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
    interleave_reads<MF, I + 2>();
  } else {
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, MF - 1 - PART_READS / 2, 0);
  }
}

// Fused mode (FUSE 1: the first round's launch, 2: a later round's): the tile's
// trajectory stride is fg.B = 256 - (L - 1) rounded down to a multiple of 4,
// so consecutive tiles overlap by L - 1 fields and hold every term of Eq. 2
// of their trajectory pairs. After the main loop nothing is stored: the
// distances are staged in LDS in four parts -- the rows of the first and
// second half of the tile's trajectory rows, then (transposed) the columns of
// either half of its trajectory columns, each with its L - 1 halo -- and the
// tile consumer (fused_walk.h) of each part offers every pair to its row (row
// parts) or to its column (column parts) and writes their slots. The distances are formed exactly as
// the matrix mode forms them (same operands, same order, the smaller field on
// the A side), so the two modes agree bit for bit wherever the FP64 window
// sums are exact.
constexpr int FPITCH = TILE + 1;  // floats per staged row (odd: transposed reads)
constexpr int FUSED_MAX_STAGED = (GRAM_TILE - 16) / 2 + 15;  // rows of a part, L <= 16
constexpr int FUSED_VAL_BYTES = FUSED_MAX_STAGED * FPITCH * 4;
constexpr int GRAM_LDS = GRAM_STAGES * 2 * OPER_BYTES + NORM_LDS;
// the staged part, then each wave's first-round scratch
constexpr int FUSED_EST_OFFSET = (FUSED_VAL_BYTES + 15) / 16 * 16;
constexpr int FUSED_EST_BYTES = FUSED_EST_OFFSET + (GRAM_THREADS / 64) * EST_SCRATCH_BYTES;
constexpr int FUSED_LDS = FUSED_EST_BYTES > GRAM_LDS ? FUSED_EST_BYTES : GRAM_LDS;
static_assert(FUSED_LDS <= 160 * 1024, "a fused part must fit in the LDS of a CU");

template <int PREC, bool BAND, int FUSE = 0>
__global__ __launch_bounds__(GRAM_THREADS, 1) void gram_kernel(
    const char* __restrict__ xc, int64_t pitch, int nstages,
    const float* __restrict__ ncs, int64_t T, int64_t Tpad, int nb, int64_t ntiles,
    int64_t a_row0, int nbi, int64_t rows_out, int J0, float* __restrict__ S, int64_t ldS,
    float* __restrict__ ST, int64_t ldST, FusedGeom fg, const double* __restrict__ fbound,
    FusedSlots fout) {
  __shared__ __attribute__((aligned(16))) char lds[FUSE ? FUSED_LDS : GRAM_LDS];
  float* const nrm = (float*)(lds + GRAM_STAGES * 2 * OPER_BYTES);  // [2][I 256 | J 256]
  int I, J;
  if constexpr (FUSE != 0) {
    // the round's tiles, each XCD a contiguous run of them (as decode_tile)
    const int64_t per = (ntiles + NUM_XCD - 1) / NUM_XCD;
    const int64_t lin = (int64_t)(blockIdx.x % NUM_XCD) * per + blockIdx.x / NUM_XCD;
    if (lin >= ntiles || !fused_band_tile(lin, fg, I, J)) return;
  } else if constexpr (BAND) {
    // the band's tiles that hold entries above the diagonal: J >= J0 + I,
    // the upper triangle of the columns from J0 on, cut to the band's rows
    if (!decode_tile(blockIdx.x, nb - J0, nbi, ntiles, I, J)) return;
    J += J0;
  } else {
    if (!decode_tile(blockIdx.x, nb, nb, ntiles, I, J)) return;
  }
  // first fields of the tile's A and B panels
  const int64_t arow = FUSE ? (int64_t)I * fg.B : (BAND ? a_row0 : 0) + (int64_t)I * TILE;
  const int64_t brow = FUSE ? (int64_t)J * fg.B : (int64_t)J * TILE;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int wm = w / WAVES_N, wn = w % WAVES_N;
  const char* Ag = xc + arow * pitch;
  const char* Bg = xc + brow * pitch;

  // Direct buffer -> LDS loads (buffer_load_dwordx4 ... lds): lane q of a load
  // lands at byte 16*q of the wave's 1 KB destination block, so each lane
  // fetches the logical chunk whose swizzled slot is that destination. Each
  // wave moves 8 KB of A and 8 KB of B per stage and no VGPR stages the data.
  // The buffer resources span the two 256-row panels (the planner keeps a
  // panel below 4 GiB), so a lane needs one 32-bit offset per block, shared by
  // A and B, and the stage offset travels in the scalar offset.
  constexpr int BLK_PER_WAVE = OPER_BYTES / 1024 / (GRAM_THREADS / 64);
  constexpr int RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer, gfx9 family
  const int panel_bytes = (int)(uint32_t)(TILE * pitch);
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc((void*)Ag, 0, panel_bytes, RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc((void*)Bg, 0, panel_bytes, RSRC_WORD3);
  uint32_t voff[BLK_PER_WAVE];
#pragma unroll
  for (int u = 0; u < BLK_PER_WAVE; ++u) {
    const int row = (w * BLK_PER_WAVE + u) * 8 + (lane >> 3);
    const int c = (lane & 7) ^ swz_key(row);  // inverse of swz
    voff[u] = (uint32_t)row * (uint32_t)pitch + (uint32_t)(c * 16);
  }
  auto issue = [&](int st, int buf) {
    char* A = lds + buf * 2 * OPER_BYTES;
    const uint32_t soff = (uint32_t)st * RB;
#pragma unroll
    for (int u = 0; u < BLK_PER_WAVE; ++u) {
      const int blk = w * BLK_PER_WAVE + u;  // 1 KB block
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsA, (__attribute__((address_space(3))) void*)(A + blk * 1024), 16, voff[u], soff, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsB, (__attribute__((address_space(3))) void*)(A + OPER_BYTES + blk * 1024), 16, voff[u],
          soff, 0, 0);
    }
  };

  f32x16 acc[BM][BN];
#pragma unroll
  for (int a = 0; a < BM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  // Chunk norms: wave 0 fetches the chunk's 256 N_i^c, wave 1 the 256 N_j^c
  // (one 1 KB direct load each) into the chunk's LDS slot.
  auto issue_norms = [&](int ch) {
    const float* src = ncs + (int64_t)ch * Tpad + (w == 0 ? arow : brow) + 4 * lane;
    __builtin_amdgcn_global_load_lds(src, nrm + (ch & 1) * 2 * TILE + w * TILE, 16, 0, 0);
  };
  // acc += -(N_i^c + N_j^c)/2 as a depth-2 FP32 MFMA: lanes 0-31 supply
  // k = 0 (A: N_i^c, B: -1/2), lanes 32-63 k = 1 (A: 1, B: -N_j^c/2); all
  // products are exact.
  const int r32 = lane & 31;
  const bool khi = lane >= 32;
  auto correct = [&](int ch) {
    const float* nA = nrm + (ch & 1) * 2 * TILE;
    const float* nB = nA + TILE;
    float av[BM], bv[BN];
#pragma unroll
    for (int bm = 0; bm < BM; ++bm) {
      const float x = nA[wm * WT_M + bm * 32 + r32];
      av[bm] = khi ? 1.0f : x;
    }
#pragma unroll
    for (int bn = 0; bn < BN; ++bn) {
      const float y = nB[wn * WT_N + bn * 32 + r32];
      bv[bn] = khi ? -0.5f * y : -0.5f;
    }
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
        acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[bm], bv[bn], acc[bm][bn], 0, 0, 0);
  };
  constexpr int SPC = GRAM_CHUNK / (PREC == TRAKNN_FP16 ? 64 : 32);  // stages per chunk

  // Every stage is two parts. Part 0 of stage st is read while the MFMAs of
  // part 1 of stage st - 1 run (right after the barrier that makes stage st
  // visible), part 1 of st while the MFMAs of part 0 of st run; so LDS read
  // latency hides behind MFMAs and only one part's fragments are in flight.
  const PartOffsets o0 = part_offsets<PREC>(0, wm, wn, lane);
  const PartOffsets o1 = part_offsets<PREC>(1, wm, wn, lane);
  // Stage st + 2 is issued right after the barrier in the middle of stage st
  // (its buffer, that of stage st, has then been read by every wave), so the
  // loads have the second half of st and the first half of st + 1 to land.
  // The norms of a chunk travel with the loads of the chunk's last stage.
  auto issue_stage = [&](int st) {
    issue(st, st & 1);
    if ((st + 1 == nstages || (st + 1) % SPC == 0) && w < 2) issue_norms(st / SPC);
  };
  Part<PREC> P0, P1;
  issue_stage(0);
  if (nstages > 1) {
    issue_stage(1);
    // stage 0 has landed (stage 1's loads may still be in flight)
    __builtin_amdgcn_s_waitcnt(vmcnt_le(2 * BLK_PER_WAVE));
  } else {
    __builtin_amdgcn_s_waitcnt(VMCNT0);
  }
  __syncthreads();
  read_part<PREC>(lds, o0, P0);
  for (int st = 0; st + 1 < nstages; ++st) {
    const int buf = st & 1;
    const int ch = st / SPC;
    const bool chunk_end = (st + 1) % SPC == 0;
    read_part<PREC>(lds + buf * 2 * OPER_BYTES, o1, P1);
    mfma_part<PREC>(P0, acc);
    interleave_reads<part_mfmas<PREC>()>();
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(VMCNT0);  // stage st + 1 (the only loads in flight)
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    if (st + 2 < nstages) issue_stage(st + 2);
    read_part<PREC>(lds + (buf ^ 1) * 2 * OPER_BYTES, o0, P0);
    mfma_part<PREC>(P1, acc);
    interleave_reads<part_mfmas<PREC>()>();
    __builtin_amdgcn_sched_barrier(0);
    if (chunk_end) correct(ch);
  }
  {  // last stage: nothing left to fetch
    const int st = nstages - 1;
    read_part<PREC>(lds + (st & 1) * 2 * OPER_BYTES, o1, P1);
    mfma_part<PREC>(P0, acc);
    mfma_part<PREC>(P1, acc);
    correct(st / SPC);
  }
  __syncthreads();  // every wave is done with the operand buffers

  if constexpr (FUSE != 0) {
    float* V = (float*)lds;  // [staged][FPITCH]
    const int hs = fg.B / 2;                           // recipients per part
    const int Rs = hs + fg.L - 1;                      // staged rows (columns)
    // the snapshot distances, once: d = -2 acc, clamped
#pragma unroll
    for (int bm = 0; bm < BM; ++bm)
#pragma unroll
      for (int bn = 0; bn < BN; ++bn)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[bm][bn][r] = clamp_distance(-2.f * acc[bm][bn][r]);
    // accumulator r of a 32x32 block holds row 8 (r / 4) + 4 (lane / 32) + r % 4
    // of the block, column lane % 32
    const int lrow = 4 * (lane >> 5), lcol = lane & 31;
#pragma unroll 1
    for (int part = 0; part < 4; ++part) {
      const bool cols = part >= 2;
      const int off = (part & 1) * hs;  // first staged tile row (column)
      if (!cols) {
        // rows off .. off + Rs - 1 of the tile, as staged rows
#pragma unroll
        for (int bm = 0; bm < BM; ++bm) {
          const int rb = wm * WT_M + bm * 32;
          if (rb + 32 <= off || rb >= off + Rs) continue;
          const bool whole = rb >= off && rb + 32 <= off + Rs;  // every row of the block
#pragma unroll
          for (int bn = 0; bn < BN; ++bn) {
            float* base = V + (rb - off + lrow) * FPITCH + wn * WT_N + bn * 32 + lcol;
            if (whole) {
#pragma unroll
              for (int r = 0; r < 16; ++r) base[(8 * (r >> 2) + (r & 3)) * FPITCH] = acc[bm][bn][r];
            } else {
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const int dr = 8 * (r >> 2) + (r & 3);
                const int rel = rb - off + lrow + dr;
                if (rel >= 0 && rel < Rs) base[dr * FPITCH] = acc[bm][bn][r];
              }
            }
          }
        }
      } else {
        // columns off .. off + Rs - 1 of the tile, as staged rows (transposed)
#pragma unroll
        for (int bn = 0; bn < BN; ++bn) {
          const int cb = wn * WT_N + bn * 32;
          if (cb + 32 <= off || cb >= off + Rs) continue;
          const int rel = cb + lcol - off;
          if (rel >= 0 && rel < Rs) {
#pragma unroll
            for (int bm = 0; bm < BM; ++bm) {
              float* base = V + rel * FPITCH + wm * WT_M + bm * 32 + lrow;
#pragma unroll
              for (int r = 0; r < 16; ++r) base[8 * (r >> 2) + (r & 3)] = acc[bm][bn][r];
            }
          }
        }
      }
      __syncthreads();
      // row parts: recipients are the tile's rows (slot J + 1); column parts:
      // its columns (slot I)
      const int p0 = (cols ? J : I) * fg.B + off, q0 = (cols ? I : J) * fg.B;
      char* est = lds + FUSED_EST_OFFSET + w * EST_SCRATCH_BYTES;
      const EstScratch sc{(double*)est, (int*)(est + 64 * sizeof(double))};
      side_topk_len<TILE / 64, FUSE == 1>(fg.L, V, FPITCH, 1, fg.B, hs, p0, q0, cols ? -1 : 1,
                                          cols ? I : J + 1, fg.np, w, GRAM_THREADS / 64, lane,
                                          fbound, fout, sc);
      __syncthreads();
    }
    return;
  }

  // Epilogue through LDS (the operand buffers are free now): d = -2 acc.
  // Accumulator r of
  // lane l in a 32x32 block holds row 8*(r/4) + 4*(l/32) + r%4, column l%32;
  // each 32-row band (bm) of every wave is parked column-major in LDS with
  // compile-time accumulator indices, then all threads write the band's
  // distances coalesced: rows of S for (i, j), and 128-byte runs of S rows for
  // the mirrored (j, i). The whole-matrix mode writes them non-temporally: S is
  // read back only after the Gram, far too large for the caches.
  constexpr int NWAVES = GRAM_THREADS / 64;
  float* stg = (float*)lds;  // [NWAVES][WT_N][EPI_PITCH]
  const bool diag = !BAND && I == J;
  const int64_t i_base = (int64_t)I * TILE, j_base = (int64_t)J * TILE;
  const int64_t c0 = BAND ? (int64_t)J0 * TILE : 0;  // first column held in band mode
#pragma unroll
  for (int bm = 0; bm < BM; ++bm) {
    float* mine = stg + w * WT_N * EPI_PITCH;
#pragma unroll
    for (int bn = 0; bn < BN; ++bn)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = bn * 32 + (lane & 31);
        const int row = 8 * q + 4 * (lane >> 5);
        *(f32x4*)(mine + col * EPI_PITCH + row) =
            f32x4{acc[bm][bn][4 * q + 0], acc[bm][bn][4 * q + 1],
                  acc[bm][bn][4 * q + 2], acc[bm][bn][4 * q + 3]};
      }
    __syncthreads();
    // (i, j): thread tid owns tile column jl = tid % 256 and the row halves
    // wm_ = tid / 256 (+ steps); rows wm_*128 + bm*32 + r
    {
      const int jl = tid & (TILE - 1);
      const int wn_ = jl / WT_N, c = jl % WT_N;
      const int64_t j = j_base + jl;
      if (j < T) {
        for (int wm_ = tid / TILE; wm_ < WAVES_M; wm_ += GRAM_THREADS / TILE) {
          const float* src = stg + (wm_ * WAVES_N + wn_) * WT_N * EPI_PITCH + c * EPI_PITCH;
          const int il0 = wm_ * 128 + bm * 32;
          const int64_t i0 = i_base + il0;
          // rows written: those below rows_out and, on a diagonal tile, above
          // the diagonal (il < jl); the row pointer steps by ldS
          int64_t nr = rows_out - i0;
          if (diag && jl - il0 < nr) nr = jl - il0;
          const int n = nr < 32 ? (int)nr : 32;
          float* dst = S + i0 * ldS + (j - c0);
          // band mode: a field's distance to itself is stored as 0, as the
          // mirrored pass stores it in the symmetric mode
          const int64_t dz = BAND ? j - (a_row0 + i0) : -1;
          for (int r = 0; r < n; ++r, dst += ldS) {
            const float v = clamp_distance(-2.f * src[r]);
            if constexpr (BAND)
              *dst = r == dz ? 0.f : v;
            else  // the whole matrix is read back only after the Gram: stream it
              __builtin_nontemporal_store(v, dst);
          }
        }
      }
    }
    // (j, i): 8 threads per (column, row half) write 32 consecutive i, into S
    // itself or, in band mode, into the transposed band
    {
      for (int run = tid >> 3; run < WAVES_M * TILE; run += GRAM_THREADS / 8) {
        const int jl = run / WAVES_M, wm_ = run % WAVES_M;
        const int wn_ = jl / WT_N, c = jl % WT_N;
        const int64_t j = j_base + jl;
        if (j >= T) continue;
        const int q = tid & 7;
        const int il0 = wm_ * 128 + bm * 32 + 4 * q;
        const int64_t i0 = i_base + il0;
        const f32x4 g = *(const f32x4*)(stg + (wm_ * WAVES_N + wn_) * WT_N * EPI_PITCH +
                                         c * EPI_PITCH + 4 * q);
        float f[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          f[e] = clamp_distance(-2.f * g[e]);
        }
        if constexpr (BAND) {
          // i0 is a band row: field a_row0 + i0
          float* dst = ST + (j - c0) * ldST + i0;
          const int64_t dj = j - (a_row0 + i0);  // field j's position in the run, if any
          if (i0 + 3 < rows_out && (dj < 0 || dj > 3)) {
            *(f32x4*)dst = f32x4{f[0], f[1], f[2], f[3]};
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (i0 + e < rows_out) dst[e] = dj == e ? 0.f : f[e];
          }
        } else {
          float* dst = S + j * ldS + i0;
          if (!diag && i0 + 3 < T) {
            __builtin_nontemporal_store(f32x4{f[0], f[1], f[2], f[3]}, (f32x4*)dst);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int il = il0 + e;
              if (i0 + e >= T) continue;
              if (!diag || il < jl) dst[e] = f[e];
              else if (il == jl) dst[e] = 0.f;
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_gram(const void* xc, const float* ncs, int64_t T, int64_t Tpad,
                       int64_t Dpad, int nb, int64_t ntiles, int precision,
                       float* S, int64_t ldS, hipStream_t s) {
  return launch_gram_band(xc, ncs, T, Tpad, Dpad, nb, ntiles, precision, -1, 0, 0, 0, S, ldS,
                          nullptr, 0, s);
}

hipError_t launch_gram_band(const void* xc, const float* ncs, int64_t T, int64_t Tpad,
                            int64_t Dpad, int nb, int64_t ntiles, int precision,
                            int64_t a_row0, int nbi, int64_t rows_out, int J0, float* S,
                            int64_t ldS, float* ST, int64_t ldST, hipStream_t s) {
  const int64_t pitch = Dpad * elem_bytes(precision);
  const int nstages = (int)(Dpad / stage_k(precision));
  const int64_t per = (ntiles + NUM_XCD - 1) / NUM_XCD;
  dim3 grid((unsigned)(per * NUM_XCD));
  const char* x = (const char*)xc;
  const bool band = a_row0 >= 0;
  if (!band) rows_out = T;
  const FusedGeom fg{};
  const FusedSlots fo{};
#define TRAKNN_GRAM_LAUNCH(P, B)                                                          \
  hipLaunchKernelGGL((gram_kernel<P, B>), grid, dim3(GRAM_THREADS), 0, s, x, pitch, nstages, \
                     ncs, T, Tpad, nb, ntiles, a_row0, nbi, rows_out, J0, S, ldS, ST, ldST, \
                     fg, nullptr, fo)
  switch (precision) {
    case TRAKNN_FP32:
      if (band) TRAKNN_GRAM_LAUNCH(TRAKNN_FP32, true);
      else TRAKNN_GRAM_LAUNCH(TRAKNN_FP32, false);
      break;
    case TRAKNN_BF16X3:
      if (band) TRAKNN_GRAM_LAUNCH(TRAKNN_BF16X3, true);
      else TRAKNN_GRAM_LAUNCH(TRAKNN_BF16X3, false);
      break;
    default:
      if (band) TRAKNN_GRAM_LAUNCH(TRAKNN_FP16, true);
      else TRAKNN_GRAM_LAUNCH(TRAKNN_FP16, false);
      break;
  }
#undef TRAKNN_GRAM_LAUNCH
  return hipGetLastError();
}

hipError_t launch_gram_fused(const void* xc, const float* ncs, int64_t T, int64_t Tpad,
                             int64_t Dpad, int precision, const FusedGeom& g, bool establish,
                             const double* bound, const FusedSlots& out, hipStream_t s) {
  const int64_t pitch = Dpad * elem_bytes(precision);
  const int nstages = (int)(Dpad / stage_k(precision));
  const int64_t ntiles = fused_band_tiles(g);
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)((ntiles + NUM_XCD - 1) / NUM_XCD * NUM_XCD));
  const char* x = (const char*)xc;
#define TRAKNN_GRAM_FUSED(P, F)                                                           \
  hipLaunchKernelGGL((gram_kernel<P, false, F>), grid, dim3(GRAM_THREADS), 0, s, x, pitch, \
                     nstages, ncs, T, Tpad, 0, ntiles, (int64_t)0, 0, T, 0, nullptr,        \
                     (int64_t)0, nullptr, (int64_t)0, g, bound, out)
  switch (precision) {
    case TRAKNN_FP32:
      if (establish) TRAKNN_GRAM_FUSED(TRAKNN_FP32, 1);
      else TRAKNN_GRAM_FUSED(TRAKNN_FP32, 2);
      break;
    case TRAKNN_BF16X3:
      if (establish) TRAKNN_GRAM_FUSED(TRAKNN_BF16X3, 1);
      else TRAKNN_GRAM_FUSED(TRAKNN_BF16X3, 2);
      break;
    default:
      if (establish) TRAKNN_GRAM_FUSED(TRAKNN_FP16, 1);
      else TRAKNN_GRAM_FUSED(TRAKNN_FP16, 2);
      break;
  }
#undef TRAKNN_GRAM_FUSED
  return hipGetLastError();
}

}  // namespace traknn
