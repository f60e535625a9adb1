// Fused S-free path (paper, Algorithm 1 stages 1-3 joined tile by tile, so the
// T x T distance matrix is never stored; Section 7 names out-of-core
// computation as future work) -- the FP64 tile kernel, and the bound and
// select kernels shared with the MFMA-fused Gram.
//
// FP64 precision: each tile evaluates Eq. 4, d = N_i + N_j - 2 <x_i, x_j>,
// with FP64 operands (the FP32 fields shifted per cell by the FP64 sample
// mean), FP64 products and FP64 sums on the vector ALUs. At the small grids
// of the paper's PCA comparison (13 or 33 components, Section 5.1) the
// contraction is too shallow for MFMA to matter, and FP64 removes the
// cancellation that reduced-precision Gram products suffer when a pair's
// distance is a small fraction of its norms: the rounding error is about
// 2^-53 N, far below any tolerance. The distance is then rounded once to
// FP32, as the distance matrix of the other modes stores it, and the tile
// consumer (fused_walk.h) does the rest.
#include "dist_clamp.h"
#include "fused_walk.h"
#include "internal.h"

namespace traknn {
namespace {

constexpr int F64_TILE = FUSED_F64_TILE;   // snapshot rows and columns of a tile
constexpr int F64_THREADS = 512;
constexpr int F64_ROWS = F64_TILE / (F64_THREADS / 64);  // Gram rows per wave
constexpr int F64_KC = 16;                 // cells per K chunk staged in LDS
constexpr int F64_LD = F64_TILE + 1;       // pitch of the staged distance tile (odd)
constexpr int F64_APITCH = F64_KC + 1;     // pitch of the A panel, doubles
constexpr int F64_BPITCH = F64_TILE + 2;   // pitch of the transposed B panel, doubles
constexpr int F64_PANEL_BYTES = (F64_TILE * F64_APITCH + F64_KC * F64_BPITCH) * 8;
constexpr int F64_VAL_BYTES = F64_TILE * F64_LD * 4;
constexpr int F64_UNION_BYTES = F64_PANEL_BYTES > F64_VAL_BYTES ? F64_PANEL_BYTES : F64_VAL_BYTES;
static_assert(F64_TILE == 128 && F64_ROWS == 16,
              "the Gram mapping gives each wave 16 rows and each lane 2 columns");

// Eq. 4 in FP64 from the two squared norms and the inner product: one rounding.
__device__ __forceinline__ double f64_dist(double ni, double nj, double g) {
  return __builtin_fma(-2.0, g, ni + nj);
}
// Centred cell value of field r (zero beyond the series or the grid).
__device__ __forceinline__ double centred(const float* X, int64_t ldx, int T, int D,
                                          const double* mu, int64_t r, int p) {
  return (r < T && p < D) ? (double)X[r * ldx + p] - mu[p] : 0.0;
}

template <bool ESTABLISH>
__global__ __launch_bounds__(F64_THREADS) void fused_f64_kernel(
    const float* __restrict__ X, int64_t ldx, int D, const double* __restrict__ mu,
    FusedGeom g, const double* __restrict__ bound, FusedSlots out) {
  __shared__ __attribute__((aligned(16))) char un[F64_UNION_BYTES];
  __shared__ double nrm[2][F64_TILE];  // squared norms of the A and B rows
  __shared__ double est_d[F64_THREADS / 64][64];  // each wave's first-round scratch
  __shared__ int est_i[F64_THREADS / 64][64];
  int I, J;
  if (!fused_band_tile(blockIdx.x, g, I, J)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i0 = (int64_t)I * g.B, j0 = (int64_t)J * g.B;
  double* Ap = (double*)un;                    // [F64_TILE][F64_APITCH]
  double* Bt = Ap + F64_TILE * F64_APITCH;     // [F64_KC][F64_BPITCH]

  // Gram of the tile: wave w owns the F64_ROWS rows from F64_ROWS w on (read
  // as broadcasts), each lane the columns lane and lane + 64.
  double acc[F64_ROWS][2];
#pragma unroll
  for (int r = 0; r < F64_ROWS; ++r) acc[r][0] = acc[r][1] = 0.0;
  double nacc = 0.0;  // thread t < 128: A row t, 128 <= t < 256: B row t - 128
  for (int k0 = 0; k0 < D; k0 += F64_KC) {
    __syncthreads();  // previous chunk fully read
    for (int e = tid; e < F64_TILE * F64_KC; e += F64_THREADS) {
      const int r = e / F64_KC, c = e % F64_KC;
      Ap[r * F64_APITCH + c] = centred(X, ldx, g.T, D, mu, i0 + r, k0 + c);
      Bt[c * F64_BPITCH + r] = centred(X, ldx, g.T, D, mu, j0 + r, k0 + c);
    }
    __syncthreads();
    if (tid < 2 * F64_TILE) {
      const bool a_side = tid < F64_TILE;
      const int r = a_side ? tid : tid - F64_TILE;
#pragma unroll
      for (int c = 0; c < F64_KC; ++c) {
        const double x = a_side ? Ap[r * F64_APITCH + c] : Bt[c * F64_BPITCH + r];
        nacc = __builtin_fma(x, x, nacc);
      }
    }
#pragma unroll 1
    for (int c = 0; c < F64_KC; ++c) {
      const double b0 = Bt[c * F64_BPITCH + lane];
      const double b1 = Bt[c * F64_BPITCH + lane + 64];
#pragma unroll
      for (int r = 0; r < F64_ROWS; ++r) {
        const double a = Ap[(F64_ROWS * w + r) * F64_APITCH + c];
        acc[r][0] = __builtin_fma(a, b0, acc[r][0]);
        acc[r][1] = __builtin_fma(a, b1, acc[r][1]);
      }
    }
  }
  if (tid < 2 * F64_TILE) nrm[tid >> 7][tid & (F64_TILE - 1)] = nacc;
  __syncthreads();  // panels read, norms written
  float* V = (float*)un;  // [F64_TILE][F64_LD] snapshot distances of the tile
#pragma unroll
  for (int r = 0; r < F64_ROWS; ++r) {
    const int a = F64_ROWS * w + r;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = lane + 64 * h;
      V[a * F64_LD + b] = clamp_distance((float)f64_dist(nrm[0][a], nrm[1][b], acc[r][h]));
    }
  }
  __syncthreads();
  // The row side (recipients = the tile's rows, slot J + 1) on the first half
  // of the waves, the column side (recipients = its columns, slot I) on the
  // second.
  constexpr int NW = F64_THREADS / 64;
  const int side = w / (NW / 2);
  side_topk_len<F64_TILE / 64, ESTABLISH>(g.L, V, side ? 1 : F64_LD, side ? F64_LD : 1, g.B, g.B,
                               (int)(side ? j0 : i0), (int)(side ? i0 : j0), side ? -1 : 1,
                               side ? I : J + 1, g.np, w % (NW / 2), NW / 2, lane,
                               bound, out, EstScratch{est_d[w], est_i[w]});
}

// One wave per row: the k nearest over some of the row's slots, starting
// from the row's running list when there is one (hlo > 0). The slots are
// those of the tiles whose offset J - I lies in [hlo, hhi): the column sides
// of (It - h, It), slots It - h, and the row sides of (It, It + h), slots
// It + h + 1, It the row's block-row. FINAL writes the neighbour list;
// otherwise (a refresh) the list becomes the row's running list and its k-th
// the row's bound (+inf while it holds fewer than k).
//
// Slots come 64 at a time (lane = slot): one load of their counts, a wave
// prefix sum, and the entries' positions parked in LDS (up to SEL_PARK at a
// time), so that each lane then loads one entry and a ballot filters 64
// entries against the list's k-th at once -- two memory round trips per
// batch of slots. A batch with many entries below the k-th is merged into the
// list by sorts of the list with up to 64 - k of them at a time, the others
// by insertion.
constexpr int SEL_WAVES = 4;
constexpr int SEL_PARK = 1024;
// a batch with at least this many entries to insert is merged by a sort
constexpr int SEL_SORT_MIN = 6;
template <bool FINAL>
__global__ __launch_bounds__(64 * SEL_WAVES) void select_kernel(
    FusedGeom g, FusedSlots out, double* __restrict__ bound, double* __restrict__ run_d,
    int32_t* __restrict__ run_i, int hlo, int hhi, int32_t* __restrict__ idx,
    double* __restrict__ dist) {
  __shared__ int park[SEL_WAVES][SEL_PARK];  // (slot << 6 | entry) per entry
  __shared__ double mrg_d[SEL_WAVES][64];    // a batch's entries to merge
  __shared__ int mrg_i[SEL_WAVES][64];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int t = blockIdx.x * SEL_WAVES + w;
  if (t >= g.np) return;
  const int k = out.k;
  const int It = t / g.B;
  int* mine = park[w];
  // slot ranges: column sides It - hhi + 1 .. It - hlo, row sides
  // It + hlo + 1 .. It + hhi, both cut to 0 .. nbt
  const int clo = It - hhi + 1 > 0 ? It - hhi + 1 : 0, chi = It - hlo;
  const int rlo = It + hlo + 1, rhi = It + hhi < g.nbt ? It + hhi : g.nbt;
  const int ncol = chi >= clo ? chi - clo + 1 : 0, nrow = rhi >= rlo ? rhi - rlo + 1 : 0;
  const int nsel = ncol + nrow;
  double ed = __builtin_huge_val();
  int ei = INT_MAX;
  if (hlo > 0 && lane < k) {
    ed = run_d[(int64_t)t * k + lane];
    ei = run_i[(int64_t)t * k + lane];
  }
  const int64_t row0 = (int64_t)t * out.nslot;
  for (int c0 = 0; c0 < nsel; c0 += 64) {
    const int u = c0 + lane;
    const int slot = u >= nsel ? -1 : u < ncol ? clo + u : rlo + (u - ncol);
    const int n = slot < 0 ? 0 : out.cnt[row0 + slot];
    // inclusive prefix sum of the counts over the lanes
    int incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int total = __builtin_amdgcn_readlane(incl, 63);
    for (int p0 = 0; p0 < total; p0 += SEL_PARK) {
      // entries p0 .. p0 + SEL_PARK - 1 of the batch, in lane (slot) order
      const int p1 = p0 + SEL_PARK < total ? p0 + SEL_PARK : total;
      const int qlo = p0 - (incl - n) > 0 ? p0 - (incl - n) : 0;
      const int qhi = p1 - (incl - n) < n ? p1 - (incl - n) : n;
      for (int q = qlo; q < qhi; ++q) mine[incl - n + q - p0] = (slot << 6) | q;
      __builtin_amdgcn_wave_barrier();
      for (int b0 = p0; b0 < p1; b0 += 64) {
        const int e = b0 + lane;
        double d = __builtin_huge_val();
        int c = INT_MAX;
        if (e < p1) {
          const int pk = mine[e - p0];
          const int64_t at = (row0 + (pk >> 6)) * k + (pk & 63);
          d = out.d[at];
          c = out.i[at];
        }
        const double kd = readlane_d(ed, k - 1);
        const int ki = __builtin_amdgcn_readlane(ei, k - 1);
        const bool pass = e < p1 && key_less(d, c, kd, ki);
        const uint64_t m = __ballot(pass);
        const int cnt = __builtin_popcountll(m);
        const int room = 64 - k;  // entries one sort takes beside the list
        if (cnt >= SEL_SORT_MIN && room >= SEL_SORT_MIN) {
          // the passing entries, compacted, go in with the list (lanes < k)
          // up to `room` at a time (lanes k ..), one sort each; its first k
          // lanes are the new list
          const int pos = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
          if (pass) {
            mrg_d[w][pos] = d;
            mrg_i[w][pos] = c;
          }
          __builtin_amdgcn_wave_barrier();
          for (int c0 = 0; c0 < cnt; c0 += room) {
            const int src = lane - k + c0;
            double md = lane < k ? ed : __builtin_huge_val();
            int mi = lane < k ? ei : INT_MAX - 64 + lane;
            if (lane >= k && src < cnt) {
              md = mrg_d[w][src];
              mi = mrg_i[w][src];
            }
            bitonic_sort64(md, mi, lane);
            const bool real = mi < INT_MAX - 64;
            ed = real ? md : __builtin_huge_val();
            ei = real ? mi : INT_MAX;
          }
          __builtin_amdgcn_wave_barrier();
        } else if (m) {
          insert_reg(m, d, c, k, ed, ei);
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (FINAL) {
    if (lane < k) {
      idx[(int64_t)t * k + lane] = ei == INT_MAX ? -1 : ei;
      dist[(int64_t)t * k + lane] = ed;
    }
  } else {
    if (lane < k) {
      run_d[(int64_t)t * k + lane] = ed;
      run_i[(int64_t)t * k + lane] = ei;
    }
    const double kth = readlane_d(ed, k - 1);
    if (lane == 0) bound[t] = kth;
  }
}

}  // namespace

int64_t fused_band_tiles(const FusedGeom& g) {
  const int hi = g.bhi < g.nbt ? g.bhi : g.nbt;
  int64_t n = 0;
  for (int h = g.blo; h < hi; ++h) n += g.nbt - h;
  return n;
}

hipError_t launch_fused_f64(const float* X, int64_t ldx, int D, const double* mu,
                            const FusedGeom& g, bool establish, const double* bound,
                            const FusedSlots& out, hipStream_t s) {
  const int64_t ntiles = fused_band_tiles(g);
  if (ntiles <= 0) return hipSuccess;
  if (establish)
    hipLaunchKernelGGL(fused_f64_kernel<true>, dim3((unsigned)ntiles), dim3(F64_THREADS), 0, s,
                       X, ldx, D, mu, g, bound, out);
  else
    hipLaunchKernelGGL(fused_f64_kernel<false>, dim3((unsigned)ntiles), dim3(F64_THREADS), 0, s,
                       X, ldx, D, mu, g, bound, out);
  return hipGetLastError();
}

hipError_t launch_slots_refresh(const FusedGeom& g, const FusedSlots& out, double* bound,
                                double* run_d, int32_t* run_i, int hlo, int hhi,
                                hipStream_t s) {
  const dim3 grid((unsigned)((g.np + SEL_WAVES - 1) / SEL_WAVES));
  hipLaunchKernelGGL(select_kernel<false>, grid, dim3(64 * SEL_WAVES), 0, s, g, out, bound,
                     run_d, run_i, hlo, hhi, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_slots_final(const FusedGeom& g, const FusedSlots& out, const double* run_d,
                              const int32_t* run_i, int hlo, int32_t* idx, double* dist,
                              hipStream_t s) {
  const dim3 grid((unsigned)((g.np + SEL_WAVES - 1) / SEL_WAVES));
  hipLaunchKernelGGL(select_kernel<true>, grid, dim3(64 * SEL_WAVES), 0, s, g, out, nullptr,
                     const_cast<double*>(run_d), const_cast<int32_t*>(run_i), hlo, g.nbt + 1,
                     idx, dist);
  return hipGetLastError();
}

}  // namespace traknn
