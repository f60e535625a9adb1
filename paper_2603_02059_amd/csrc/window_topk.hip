// Trajectory distances by the diagonal window recurrence and exclusion-zone
// top-k (paper, Algorithm 1 stages 2-3; Eq. 5 and Eq. 3).
//
// D_L(i,j) = sum_{m<L} d(i+m, j+m) only ever walks along a diagonal of the
// distance matrix, so the natural gfx950 mapping puts one diagonal on each lane
// of a wave64: lane q of a wave follows the diagonal delta = j - i = delta_c + q.
// At step s the 64 lanes hold the 64 consecutive columns r + delta_c .. +63 of
// row r = r0 + s, i.e. one coalesced 256-byte segment of S per step, and each
// lane advances its own window with the recurrence
//   D <- (D - d(r, r+delta)) + d(r+L, r+L+delta)             (Eq. 5)
// in FP64. Every row block restarts its windows with a direct L-term sum, so
// rounding can never drift over more than a block's rows (and for FP32 inputs
// whose exponents span less than ~29 bits the FP64 recurrence is exact).
//
// The 64 candidates of a step all belong to the same row, so the top-k filter
// is one compare per lane against that row's bound and one ballot; the rare
// insertions shift a sorted list held one entry per lane.
//
// A launch may cover part of the matrix (band mode, row-batched streaming):
// S then holds rows s0 .. s_end - 1, and column c of the matrix at column
// c - col0 of the buffer; the launch covers the trajectory rows row_lo ..
// row_cap - 1 against the candidate columns c_lo .. c_hi - 1 whose diagonal
// offset j - i lies in dmin .. dmax, reads values only in columns c_lo ..
// v_end - 1 (zero elsewhere, which leaves the windows of valid candidates
// exact), and indexes its partial lists from row_lo. Only the diagonals of
// the offset range are visited, and only their values are relied on.
//
// A multi-length request (L = L_min .. L_max) runs the kernel once per pair of
// lengths on the same distance matrix, each length with its own running sums,
// lists and exclusion zone |i - j| >= L; the merge kernel then combines, per
// length and row, the W partial lists of the row's column ranges into the
// final k in (distance, index) order. The result does not depend on the order
// in which the waves run, nor on how the lengths are grouped into passes.
#include <array>
#include <cfloat>
#include <climits>
#include <type_traits>
#include <utility>

#include "internal.h"
#include "topk_wave.h"

namespace traknn {
namespace {

// ---------------------------------------------------------------------------
// Window + top-k kernel for one trajectory length L.
//
// Each lane holds the R + L - 1 values of its diagonal for the current chunk
// (the next chunk's values are loaded meanwhile); a step is two FP64 adds, two
// readlanes of the row's bound, one compare and a ballot.
//
// The first chunk of a wave seeds each row's list with a wave-wide bitonic
// sort of its 64 candidates (the lists start empty, so every candidate would
// otherwise be inserted one by one). Later insertions shift the list one lane
// with DPP wave_shr:1, a VALU move, instead of an LDS permute.
// ---------------------------------------------------------------------------
constexpr int W1_ROWS = WINDOW1_ROWS;  // rows per block
constexpr int W1_GROUP = 8;   // steps unrolled per group
static_assert(W1_ROWS % W1_GROUP == 0 && (W1_ROWS & (W1_ROWS - 1)) == 0 && W1_ROWS <= 64,
              "rows per block: a power of two, a multiple of the group, at most a wave");
#define W1_VALS_BYTES(M) (((size_t)(M) * 64 * sizeof(float) + 15) / 16 * 16)

// One workgroup per row block: wave w scans the w-th of W contiguous ranges
// of 64-diagonal chunks and keeps its own partial lists. The waves also share
// one distance bound per row in LDS -- the smallest k-th distance any of them
// has reached -- and skip candidates above it: such a candidate already has k
// better ones elsewhere, so it cannot be among the row's k nearest
// (candidates equal to the bound still reach the exact (distance, index)
// test). Without the shared bound every wave rediscovers a tight threshold
// on its own and the insertions grow with W.
//
// The steps of a group of U rows only filter (one compare against the row's
// bound per step, ballots kept in SGPRs); the rare insertions of the group run
// afterwards, which is exact because every row of a group is a different row.
// Chunks wholly inside the row range and clear of the exclusion zone (all but
// a few per row block) skip the per-lane validity tests.
//
// G consecutive lengths L .. L + G - 1 share one pass over S (a multi-length
// sweep pairs them): each lane keeps one running sum per length, every length
// has its own lists, bounds and exclusion zone, and the values of a chunk are
// read once for all of them. Each length's sums are started and slid exactly
// as in a pass of its own, so the results do not depend on G.
template <int L, int G>
__global__ __launch_bounds__(1024) void window1_kernel(
    const float* __restrict__ S, int64_t ldS, int T, int s0, int s_end, int col0, int c_lo,
    int c_hi, int v_end, int dmin, int dmax, int row_lo, int row_cap, int k, int W,
    int64_t split_stride, int64_t len_rows, double* __restrict__ part_d,
    int32_t* __restrict__ part_i) {
  constexpr int R = W1_ROWS;
  constexpr int U = W1_GROUP;
  constexpr int LG = L + G - 1;  // longest length of the pass
  constexpr int M = R + LG - 1;  // rows of values per chunk
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int lane = threadIdx.x & 63;
  const int split = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  unsigned long long* shb = (unsigned long long*)smem;  // [G][R] bits of the shared bounds
  char* mine = smem + G * R * sizeof(unsigned long long) +
               (size_t)split * (W1_VALS_BYTES(M + U) + (size_t)G * R * k * 12);
  float* vl = (float*)mine;  // [M + U][64]: M rows of values, U rows of padding
  double* ld = (double*)(mine + W1_VALS_BYTES(M + U));  // [G][R][k]
  int* li = (int*)(ld + (size_t)G * R * k);               // [G][R][k]
  if (threadIdx.x < G * R)
    shb[threadIdx.x] = (unsigned long long)__double_as_longlong(__builtin_huge_val());
  __syncthreads();  // the only workgroup barrier: the waves' trip counts differ

  const int r0 = row_lo + (int)blockIdx.x * R;
  int chi[G];    // candidate columns of each length: c_lo .. chi - 1
  int ncand[G];  // chi - c_lo, at least 0
  int nrows[G];  // rows of this block that exist for each length
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int npl = T - (L + g) + 1;  // trajectories of length L + g
    chi[g] = c_hi < npl ? c_hi : npl;
    ncand[g] = chi[g] > c_lo ? chi[g] - c_lo : 0;
    const int hi = row_cap < npl ? row_cap : npl;
    nrows[g] = hi - r0 < R ? (hi - r0 > 0 ? hi - r0 : 0) : R;
  }
  // diagonals of the block: every candidate column of some row, within the
  // offset range
  int64_t dlo = (int64_t)c_lo - (r0 + R - 1);
  if (dlo < dmin) dlo = dmin;
  int64_t dhi = (int64_t)chi[0] - 1 - r0;
  if (dhi > dmax) dhi = dmax;
  const int64_t NC = ncand[0] > 0 && dhi >= dlo ? (dhi - dlo + 1 + 63) / 64 : 0;
  const int64_t cb = (int64_t)split * NC / W, ce = (int64_t)(split + 1) * NC / W;

  double thr_d[G];  // lane q: own k-th of row r0 + q, per length
  int thr_i[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    thr_d[g] = __builtin_huge_val();
    thr_i[g] = INT_MAX;
  }

  // Values of diagonal delta at rows r0 + m (one 256-byte segment per row
  // for the wave), zero outside the held rows and the columns c_lo ..
  // v_end - 1. The pointer walks down the rows
  // with a stride the compiler treats as opaque, so no per-row address is
  // precomputed and held across chunks; chunks wholly inside the matrix skip
  // the bounds tests, the others read a safe element and discard it.
  float nxt[M];
  auto load = [&](int64_t c) __attribute__((always_inline)) {
    const int64_t dc = dlo + 64 * c;
    int64_t stride = ldS + 1;
    asm volatile("" : "+s"(stride));
    const float* p = S + ((int64_t)(r0 - s0) * ldS + (r0 + dc + lane - col0));
    const bool inb = r0 + dc >= c_lo && r0 + M - 1 < s_end && r0 + M - 1 + dc + 63 < v_end;
    if (inb) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        nxt[m] = *p;
        p += stride;
      }
    } else {
      int rows_in = s_end - r0;  // rows r0 + m with m < rows_in are held
      int64_t vlo = c_lo, vhi = v_end;
      asm volatile("" : "+s"(rows_in), "+s"(vlo), "+s"(vhi));
      int64_t col = r0 + dc + lane;  // column of row r0 + m, stepped with m
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const bool ok = (m < rows_in) & (col >= vlo) & (col < vhi);
        const float x = *(ok ? p : S);
        nxt[m] = ok ? x : 0.f;
        p += stride;
        col += 1;
      }
    }
  };
  // after a row's own list changed: lower its shared bound to the list's k-th
  auto publish = [&](int g, int s) __attribute__((always_inline)) {
    if (lane == s && thr_d[g] != __builtin_huge_val())
      atomicMin(&shb[g * R + s], (unsigned long long)__double_as_longlong(thr_d[g]));
  };

  // First chunk of the range: the lists start empty, so each row's list is
  // seeded with a sort of its first 64 candidates.
  auto seed_chunk = [&](int64_t c) __attribute__((always_inline)) {
    const int delta = (int)(dlo + 64 * c) + lane;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int Lg = L + g;
      const bool okd = ((delta >= Lg) | (delta <= -Lg)) & (delta >= dmin) & (delta <= dmax);
      double D = 0.0;
#pragma unroll
      for (int l = 0; l < L + g; ++l) D += (double)vl[l * 64 + lane];
#pragma unroll 1
      for (int s = 0; s < nrows[g]; ++s) {
        const int col = r0 + s + delta;
        const bool valid = okd & ((unsigned)(col - c_lo) < (unsigned)ncand[g]);
        seed_row(D, col, valid, k, ld + (g * R + s) * k, li + (g * R + s) * k, lane, s,
                 thr_d[g], thr_i[g]);
        publish(g, s);
        D = (D - (double)vl[s * 64 + lane]) + (double)vl[(s + Lg) * 64 + lane];
      }
    }
  };

  // Later chunks: filter, then insert. EDGE chunks test each candidate's
  // column range, exclusion zone and row.
  auto scan_chunk = [&](int64_t c, auto edge_c) __attribute__((always_inline)) {
    constexpr bool EDGE = decltype(edge_c)::value;
    const int delta = (int)(dlo + 64 * c) + lane;
    bool okd[G];
    double D[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      okd[g] = ((delta >= L + g) | (delta <= -(L + g))) & (delta >= dmin) & (delta <= dmax);
      D[g] = 0.0;
#pragma unroll
      for (int l = 0; l < L + g; ++l) D[g] += (double)vl[l * 64 + lane];
    }
#pragma unroll 1
    for (int gr = 0; gr < R; gr += U) {
      float w[U + LG];  // rows gr .. gr+U+LG-1
#pragma unroll
      for (int j = 0; j < U + LG; ++j) w[j] = vl[(gr + j) * 64 + lane];
      // bound per row (lane q < R) and length: own k-th or the shared bound,
      // the smaller
      double bound[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const double sh = __longlong_as_double(
            (long long)__atomic_load_n(&shb[g * R + (lane & (R - 1))], __ATOMIC_RELAXED));
        bound[g] = __builtin_fmin(thr_d[g], sh);
      }
      double Dj[G][U];
      uint64_t m[G][U];
      uint64_t any = 0;
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int s = gr + j;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          Dj[g][j] = D[g];
          bool pass = D[g] <= readlane_d(bound[g], s);
          if constexpr (EDGE) {
            const int col = r0 + s + delta;
            pass = pass & okd[g] & ((unsigned)(col - c_lo) < (unsigned)ncand[g]) &
                   (s < nrows[g]);
          }
          m[g][j] = __ballot(pass);
          any |= m[g][j];
          if (j + 1 < U || gr + U < R) D[g] = (D[g] - (double)w[j]) + (double)w[j + L + g];
        }
      }
      if (any) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (m[g][j]) {
              const int s = gr + j;
              insert_seq(m[g][j], Dj[g][j], r0 + s + delta, k, ld + (g * R + s) * k,
                         li + (g * R + s) * k, lane, s, thr_d[g], thr_i[g]);
              publish(g, s);
            }
          }
        }
      }
    }
  };

  if (cb < ce) load(cb);
  // interior chunks: every row exists for every length, and the columns and
  // the exclusion zone of the longest length (the strictest) are clear
  const bool full = nrows[G - 1] == R;
  for (int64_t c = cb; c < ce; ++c) {
    // park this chunk's values in this wave's LDS rows (LDS accesses of a
    // wave execute in order), then start fetching the next chunk
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m = 0; m < M; ++m) vl[m * 64 + lane] = nxt[m];
    __builtin_amdgcn_wave_barrier();
    if (c + 1 < ce) load(c + 1);
    const int64_t dc = dlo + 64 * c;
    const bool interior = full & ((dc >= LG) | (dc + 63 <= -LG)) & (r0 + dc >= c_lo) &
                          (r0 + R - 1 + dc + 63 < chi[G - 1]) & (dc >= dmin) &
                          (dc + 63 <= dmax);
    if (c == cb)
      seed_chunk(c);
    else if (interior)
      scan_chunk(c, std::false_type{});
    else
      scan_chunk(c, std::true_type{});
  }
  // partial lists: part[(split * split_stride + g * len_rows + row - row_lo) * k
  // + q] for length L + g; a range with no chunk leaves its lists empty
#pragma unroll
  for (int g = 0; g < G; ++g) {
    for (int s = 0; s < nrows[g]; ++s) {
      const int64_t row = (int64_t)g * len_rows + (r0 - row_lo + s);
      if (lane < k) {
        const int64_t o = ((int64_t)split * split_stride + row) * k + lane;
        part_d[o] = cb < ce ? ld[(g * R + s) * k + lane] : __builtin_huge_val();
        part_i[o] = cb < ce ? li[(g * R + s) * k + lane] : INT_MAX;
      }
    }
  }
}

// Row blocks of lengths L .. L + G - 1: ceil((rows of length L) / W1_ROWS)
// workgroups of W waves.
template <int L, int G>
hipError_t launch_win1(const float* S, int64_t ldS, int T, int s0, int s_end, int col0,
                       int c_lo, int c_hi, int v_end, int dmin, int dmax, int row_lo,
                       int row_cap, int k, int W, int64_t split_stride, int64_t len_rows,
                       double* pd, int32_t* pi, hipStream_t s) {
  const size_t lds = window1_lds_bytes(L + G - 1, G, k, W);
  const int hi = row_cap < T - L + 1 ? row_cap : T - L + 1;
  const unsigned blocks = (unsigned)((hi - row_lo + W1_ROWS - 1) / W1_ROWS);
  hipLaunchKernelGGL((window1_kernel<L, G>), dim3(blocks), dim3(64 * W), lds, s, S, ldS, T,
                     s0, s_end, col0, c_lo, c_hi, v_end, dmin, dmax, row_lo, row_cap, k, W,
                     split_stride, len_rows, pd, pi);
  return hipGetLastError();
}

// One thread per (length, row): a k-step merge of the sorted partial lists
// (at most MS of them) and, for the rows below acc_end, the running list
// already in the output. Each source's current head stays in registers (the
// source loops are unrolled over MS) and only the source that advanced is
// read again; the running list is first copied to LDS, since the output that
// holds it is overwritten while it is merged.
constexpr int MERGE_THREADS = 64;
template <int MS>
__global__ __launch_bounds__(MERGE_THREADS) void merge_kernel(
    MergeSet a, MergeSet b, int T, int np0, int Lmin, int NL, int k, int t0, int nt,
    int acc_end, int32_t* __restrict__ idx, double* __restrict__ dist) {
  // rows t0 .. t0 + nt - 1 of every length. A set's partial lists are indexed
  // from t0 and cover its first rows only; empty slots of the running list
  // are index -1.
  extern __shared__ __attribute__((aligned(16))) char msm[];
  double* rd = (double*)msm + (size_t)threadIdx.x * k;                          // [64][k]
  int* ri = (int*)((double*)msm + (size_t)MERGE_THREADS * k) + (size_t)threadIdx.x * k;
  const int64_t g = (int64_t)blockIdx.x * MERGE_THREADS + threadIdx.x;
  if (g >= (int64_t)NL * nt) return;
  const int li = (int)(g / nt);
  const int tr = (int)(g % nt);
  const int t = t0 + tr;
  const int npL = T - (Lmin + li) + 1;
  int32_t* oi = idx + ((int64_t)li * np0 + t) * k;
  double* od = dist + ((int64_t)li * np0 + t) * k;
  if (t >= npL) {
    for (int q = 0; q < k; ++q) {
      oi[q] = -1;
      od[q] = __builtin_huge_val();
    }
    return;
  }
  const int nr = t < acc_end ? k : 0;
  for (int q = 0; q < nr; ++q) {
    rd[q] = od[q];
    ri[q] = oi[q] < 0 ? INT_MAX : oi[q];
  }
  const int wa = tr < a.nt ? a.W : 0, wb = tr < b.nt ? b.W : 0;
  const int ns = wa + wb;  // partial-list sources: a's splits, then b's
  // entry p of source w's list
  auto at = [&](int w, int p, double& d, int& i) __attribute__((always_inline)) {
    const bool in_a = w < wa;
    const int64_t o = (((int64_t)(in_a ? w : w - wa) * NL + li) * (in_a ? a.nt : b.nt) + tr) * k + p;
    d = in_a ? a.d[o] : b.d[o];
    i = in_a ? a.i[o] : b.i[o];
  };
  // source w's current head is (hd[w], hi[w]), entry pos[w] of its list
  int pos[MS];
  double hd[MS];
  int hi[MS];
#pragma unroll
  for (int w = 0; w < MS; ++w) {
    pos[w] = 0;
    hd[w] = __builtin_huge_val();
    hi[w] = INT_MAX;
    if (w < ns) at(w, 0, hd[w], hi[w]);
  }
  int rpos = 0;
  for (int q = 0; q < k; ++q) {
    int best = MS;  // MS: the running list
    double bd = rpos < nr ? rd[rpos] : __builtin_huge_val();
    int bi = rpos < nr ? ri[rpos] : INT_MAX;
    bool have = rpos < nr;
#pragma unroll
    for (int w = 0; w < MS; ++w) {
      if (w < ns && pos[w] < k && (!have || key_less(hd[w], hi[w], bd, bi))) {
        best = w;
        bd = hd[w];
        bi = hi[w];
        have = true;
      }
    }
    if (best == MS) {
      rpos++;
    } else {
#pragma unroll
      for (int w = 0; w < MS; ++w) {
        if (w == best) {
          pos[w]++;
          if (pos[w] < k) at(w, pos[w], hd[w], hi[w]);
        }
      }
    }
    oi[q] = bi == INT_MAX ? -1 : bi;
    od[q] = bd;
  }
}

__global__ __launch_bounds__(256) void score_kernel(
    const double* __restrict__ dist, int T, int np0, int Lmin, int NL, int k,
    double* __restrict__ scores) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)NL * np0) return;
  const int li = (int)(g / np0);
  const int t = (int)(g % np0);
  const int npL = T - (Lmin + li) + 1;
  if (t >= npL) {
    scores[g] = __builtin_nan("");
    return;
  }
  double s = 0.0;
  for (int q = 0; q < k; ++q) s += dist[g * k + q];
  scores[g] = s / (double)k;
}

// Scores for every k' <= k from one neighbour list (the lists are sorted by
// (distance, index), so the k' nearest are its first k' entries): out[q] =
// mean of dist[0..q], summed in rank order -- out[k-1] is exactly s_t.
__global__ __launch_bounds__(256) void score_prefix_kernel(
    const double* __restrict__ dist, int T, int np0, int Lmin, int NL, int k,
    double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)NL * np0) return;
  const int li = (int)(g / np0);
  const int t = (int)(g % np0);
  const int npL = T - (Lmin + li) + 1;
  double s = 0.0;
  for (int q = 0; q < k; ++q) {
    s += dist[g * k + q];
    out[g * k + q] = t < npL ? s / (double)(q + 1) : __builtin_nan("");
  }
}

// Local intrinsic dimension of every trajectory (the maximum-likelihood kNN
// estimator of Levina and Bickel that the paper applies with k in {20, 30,
// 40}, Section 5.1), for every prefix k' of its sorted list:
//   m_k' = 2 (k' - 1) / sum_{j<k'} ln(dist[k'-1] / dist[j]),
// the Euclidean log-ratio being half the log-ratio of the squared distances.
// out[0] (k' = 1, no ratio) and rows that do not exist are NaN; degenerate
// lists follow IEEE arithmetic (a zero below a positive k'-th distance gives
// 0, a zero k'-th distance NaN, k' equal distances +inf).
__global__ __launch_bounds__(256) void local_dim_kernel(
    const double* __restrict__ dist, int T, int np0, int Lmin, int NL, int k,
    double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)NL * np0) return;
  const int li = (int)(g / np0);
  const int t = (int)(g % np0);
  const bool exists = t < T - (Lmin + li) + 1;
  const double* d = dist + g * k;
  out[g * k] = __builtin_nan("");
  for (int q = 1; q < k; ++q) {
    double s = 0.0;
    for (int j = 0; j < q; ++j) s += log(d[q] / d[j]);
    out[g * k + q] = exists ? 2.0 * (double)q / s : __builtin_nan("");
  }
}

}  // namespace

// Launchers of every compiled (L, G): kWin1[L - 1] for L = 1..TRAKNN_MAX_L on
// its own, kWinG[L - 1] for the lengths L .. L + WINDOW_LENGTHS_PER_PASS - 1
// of a sweep's pass.
using WinLaunch = hipError_t (*)(const float*, int64_t, int, int, int, int, int, int, int, int,
                                 int, int, int, int, int, int64_t, int64_t, double*, int32_t*,
                                 hipStream_t);
template <int G, int... Ls>
constexpr std::array<WinLaunch, sizeof...(Ls)> win_table(std::integer_sequence<int, Ls...>) {
  return {&launch_win1<Ls + 1, G>...};
}
constexpr auto kWin1 = win_table<1>(std::make_integer_sequence<int, TRAKNN_MAX_L>{});
constexpr auto kWinG = win_table<WINDOW_LENGTHS_PER_PASS>(
    std::make_integer_sequence<int, TRAKNN_MAX_L - WINDOW_LENGTHS_PER_PASS + 1>{});

size_t window1_lds_bytes(int L, int G, int k, int W) {
  return (size_t)G * W1_ROWS * sizeof(unsigned long long) +
         (size_t)W * (W1_VALS_BYTES(W1_ROWS + L - 1 + W1_GROUP) + (size_t)G * W1_ROWS * k * 12);
}

hipError_t launch_window_topk(const float* S, int64_t ldS, int64_t T, int L_min,
                              int L_max, int k, int splits, double* part_d,
                              int32_t* part_i, hipStream_t s) {
  const WindowRange all{0, T, 0, 0, T, T, -T, T};
  return launch_window_band(S, ldS, T, L_min, L_max, k, splits, all, 0, T - L_min + 1, part_d,
                            part_i, s);
}

hipError_t launch_window_band(const float* S, int64_t ldS, int64_t T, int L_min,
                              int L_max, int k, int splits, const WindowRange& r,
                              int64_t t0, int64_t nt, double* part_d, int32_t* part_i,
                              hipStream_t s) {
  const int NL = L_max - L_min + 1;
  // partial lists: [split][length][row - t0][k]
  const int64_t split_stride = (int64_t)NL * nt;
  // a sweep runs its lengths WINDOW_LENGTHS_PER_PASS at a time (the last pass
  // takes what is left), a single length on its own
  for (int L = L_min; L <= L_max;) {
    const int G = L_max - L + 1 >= WINDOW_LENGTHS_PER_PASS ? WINDOW_LENGTHS_PER_PASS : 1;
    const int64_t off = (int64_t)(L - L_min) * nt * k;
    double* pd = part_d + off;
    int32_t* pi = part_i + off;
    // rows of length L in [t0, t0 + nt): those with t <= T - L (longer lengths
    // of the pass have fewer; none at all means the merge marks them absent)
    const int64_t hi = t0 + nt < T - L + 1 ? t0 + nt : T - L + 1;
    if (hi > t0) {
      if (L < 1 || L + G - 1 > TRAKNN_MAX_L) return hipErrorInvalidValue;
      const WinLaunch f = G > 1 ? kWinG[L - 1] : kWin1[L - 1];
      const hipError_t e =
          f(S, ldS, (int)T, (int)r.s0, (int)r.s_end, (int)r.col0, (int)r.c_lo, (int)r.c_hi,
            (int)r.v_end, (int)r.dmin, (int)r.dmax, (int)t0, (int)(t0 + nt), k, splits,
            split_stride, nt, pd, pi, s);
      if (e != hipSuccess) return e;
    }
    L += G;
  }
  return hipSuccess;
}

hipError_t launch_merge(const double* part_d, const int32_t* part_i, int64_t T,
                        int L_min, int L_max, int k, int splits, int32_t* idx,
                        double* dist, hipStream_t s) {
  const int64_t np0 = T - L_min + 1;
  const MergeSet a{part_d, part_i, splits, (int)np0}, none{nullptr, nullptr, 0, 0};
  return launch_merge_band(a, none, T, L_min, L_max, k, 0, np0, 0, idx, dist, s);
}

hipError_t launch_merge_band(const MergeSet& a, const MergeSet& b, int64_t T, int L_min,
                             int L_max, int k, int64_t t0, int64_t nt, int64_t acc_end,
                             int32_t* idx, double* dist, hipStream_t s) {
  const int np0 = (int)(T - L_min + 1);
  const int NL = L_max - L_min + 1;
  const int64_t n = (int64_t)NL * nt;
  if (n <= 0) return hipSuccess;
  if (a.W > MERGE_MAX_SPLITS || b.W > MERGE_MAX_SPLITS) return hipErrorInvalidValue;
  const int ns = a.W + b.W;
  const dim3 grid((unsigned)((n + MERGE_THREADS - 1) / MERGE_THREADS));
  const size_t lds = (size_t)MERGE_THREADS * k * (sizeof(double) + sizeof(int));
#define TRAKNN_MERGE_LAUNCH(MS)                                                              \
  hipLaunchKernelGGL(merge_kernel<MS>, grid, dim3(MERGE_THREADS), lds, s, a, b, (int)T, np0, \
                     L_min, NL, k, (int)t0, (int)nt, (int)acc_end, idx, dist)
  if (ns <= 4) TRAKNN_MERGE_LAUNCH(4);
  else if (ns <= 8) TRAKNN_MERGE_LAUNCH(8);
  else if (ns <= 16) TRAKNN_MERGE_LAUNCH(16);
  else TRAKNN_MERGE_LAUNCH(2 * MERGE_MAX_SPLITS);
#undef TRAKNN_MERGE_LAUNCH
  return hipGetLastError();
}

hipError_t launch_score(const double* dist, int64_t T, int L_min, int L_max,
                        int k, double* scores, hipStream_t s) {
  const int np0 = (int)(T - L_min + 1);
  const int NL = L_max - L_min + 1;
  const int64_t n = (int64_t)NL * np0;
  hipLaunchKernelGGL(score_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, s, dist, (int)T, np0, L_min, NL, k, scores);
  return hipGetLastError();
}

hipError_t launch_score_prefix(const double* dist, int64_t T, int L_min, int L_max,
                               int k, double* out, hipStream_t s) {
  const int np0 = (int)(T - L_min + 1);
  const int NL = L_max - L_min + 1;
  const int64_t n = (int64_t)NL * np0;
  hipLaunchKernelGGL(score_prefix_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, s, dist, (int)T, np0, L_min, NL, k, out);
  return hipGetLastError();
}

hipError_t launch_local_dim(const double* dist, int64_t T, int L_min, int L_max, int k,
                            double* out, hipStream_t s) {
  const int np0 = (int)(T - L_min + 1);
  const int NL = L_max - L_min + 1;
  const int64_t n = (int64_t)NL * np0;
  hipLaunchKernelGGL(local_dim_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     dist, (int)T, np0, L_min, NL, k, out);
  return hipGetLastError();
}

}  // namespace traknn
