// Fused S-free path (paper, Algorithm 1 stages 1-3 joined tile by tile, so the
// T x T distance matrix is never stored; Section 7 names out-of-core
// computation as future work) -- the FP64 tile kernel, the bound and select
// kernels and the exact fallback shared with the MFMA-fused Gram.
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
// walk (fused_walk.h) does the rest.
#include "dist_clamp.h"
#include "fused_walk.h"
#include "internal.h"

namespace traknn {
namespace {

constexpr int F64_TILE = FUSED_F64_TILE;   // snapshot rows and columns of a tile
constexpr int F64_THREADS = 256;
constexpr int F64_KC = 16;                 // cells per K chunk staged in LDS
constexpr int F64_LD = F64_TILE + 1;       // pitch of the staged distance tile (odd)
constexpr int F64_APITCH = F64_KC + 1;     // pitch of the A panel, doubles
constexpr int F64_BPITCH = F64_TILE + 2;   // pitch of the transposed B panel, doubles
constexpr int F64_PANEL_BYTES = (F64_TILE * F64_APITCH + F64_KC * F64_BPITCH) * 8;
constexpr int F64_VAL_BYTES = F64_TILE * F64_LD * 4;
constexpr int F64_UNION_BYTES = F64_PANEL_BYTES > F64_VAL_BYTES ? F64_PANEL_BYTES : F64_VAL_BYTES;
static_assert(F64_TILE == 128, "the Gram mapping gives each wave 32 rows and each lane 2 columns");

// Eq. 4 in FP64 from the two squared norms and the inner product: one rounding.
__device__ __forceinline__ double f64_dist(double ni, double nj, double g) {
  return __builtin_fma(-2.0, g, ni + nj);
}
// Centred cell value of field r (zero beyond the series or the grid).
__device__ __forceinline__ double centred(const float* X, int64_t ldx, int T, int D,
                                          const double* mu, int64_t r, int p) {
  return (r < T && p < D) ? (double)X[r * ldx + p] - mu[p] : 0.0;
}

// Tile (I, J) of launch tile e: ESTABLISH enumerates the tiles (I, I + h) of
// the offsets h of the geometry, I = 0 .. nbt - h - 1, offset by offset;
// FILTER the whole upper triangle row by row, and reports the tiles of the
// establishing set as skipped.
__device__ __forceinline__ bool fused_tile(int64_t e, const FusedGeom& g, bool establish,
                                           int& I, int& J) {
  if (establish) return fused_establish_tile(e, g, I, J);
  // row-major upper triangle: row I holds nbt - I tiles
  int64_t u = e;
  int i = 0;
  while (i < g.nbt && u >= g.nbt - i) {
    u -= g.nbt - i;
    ++i;
  }
  if (i >= g.nbt) return false;
  I = i;
  J = i + (int)u;
  for (int q = 0; q < g.nh; ++q)
    if (J - I == g.h[q]) return false;  // done by the establishing launch
  return true;
}

template <bool ESTABLISH>
__global__ __launch_bounds__(F64_THREADS) void fused_f64_kernel(
    const float* __restrict__ X, int64_t ldx, int D, const double* __restrict__ mu,
    FusedGeom g, const double* __restrict__ bound, FusedOut out) {
  __shared__ __attribute__((aligned(16))) char un[F64_UNION_BYTES];
  __shared__ double nrm[2][F64_TILE];  // squared norms of the A and B rows
  __shared__ double rbnd[2][F64_TILE];  // recipient bounds: rows, columns
  int I, J;
  if (!fused_tile(blockIdx.x, g, ESTABLISH, I, J)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i0 = (int64_t)I * g.B, j0 = (int64_t)J * g.B;
  double* Ap = (double*)un;                    // [F64_TILE][F64_APITCH]
  double* Bt = Ap + F64_TILE * F64_APITCH;     // [F64_KC][F64_BPITCH]

  // Gram of the tile: wave w owns rows 32w .. 32w + 31 (read as broadcasts),
  // each lane the columns lane and lane + 64.
  double acc[32][2];
#pragma unroll
  for (int r = 0; r < 32; ++r) acc[r][0] = acc[r][1] = 0.0;
  double nacc = 0.0;  // thread t < 128: A row t, t >= 128: B row t - 128
  for (int k0 = 0; k0 < D; k0 += F64_KC) {
    __syncthreads();  // previous chunk fully read
    for (int e = tid; e < F64_TILE * F64_KC; e += F64_THREADS) {
      const int r = e / F64_KC, c = e % F64_KC;
      Ap[r * F64_APITCH + c] = centred(X, ldx, g.T, D, mu, i0 + r, k0 + c);
      Bt[c * F64_BPITCH + r] = centred(X, ldx, g.T, D, mu, j0 + r, k0 + c);
    }
    __syncthreads();
    {
      const bool a_side = tid < F64_TILE;
      const int r = a_side ? tid : tid - F64_TILE;
#pragma unroll
      for (int c = 0; c < F64_KC; ++c) {
        const double x = a_side ? Ap[r * F64_APITCH + c] : Bt[c * F64_BPITCH + r];
        nacc = __builtin_fma(x, x, nacc);
      }
    }
#pragma unroll 2
    for (int c = 0; c < F64_KC; ++c) {
      const double b0 = Bt[c * F64_BPITCH + lane];
      const double b1 = Bt[c * F64_BPITCH + lane + 64];
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        const double a = Ap[(32 * w + r) * F64_APITCH + c];
        acc[r][0] = __builtin_fma(a, b0, acc[r][0]);
        acc[r][1] = __builtin_fma(a, b1, acc[r][1]);
      }
    }
  }
  nrm[tid >> 7][tid & (F64_TILE - 1)] = nacc;
  // recipient bounds of the tile's trajectory rows and columns
  if constexpr (!ESTABLISH) {
    const int side = tid >> 7, p = tid & (F64_TILE - 1);
    const int64_t t = (side ? j0 : i0) + p;
    rbnd[side][p] = (p < g.B && t < g.np) ? bound[t] : -1.0;
  }
  __syncthreads();  // panels read, norms written
  float* V = (float*)un;  // [F64_TILE][F64_LD] snapshot distances of the tile
#pragma unroll
  for (int r = 0; r < 32; ++r) {
    const int a = 32 * w + r;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = lane + 64 * h;
      V[a * F64_LD + b] = clamp_distance((float)f64_dist(nrm[0][a], nrm[1][b], acc[r][h]));
    }
  }
  __syncthreads();
  // Row walk (recipients = rows, waves 0-1) and column walk (recipients =
  // columns, waves 2-3); each group of two waves has 128 lanes >= B.
  const int grp = w >> 1, l = (w & 1) * 64 + lane;
  if constexpr (ESTABLISH) {
    if (grp == 0)
      tile_establish(V, F64_LD, 1, g.B, 0, g.B, (int)i0, (int)j0, 1, g.L, g.np, g.k, w & 1, 2,
                     lane, out);
    else
      tile_establish(V, 1, F64_LD, g.B, 0, g.B, (int)j0, (int)i0, -1, g.L, g.np, g.k, w & 1, 2,
                     lane, out);
  } else {
    if (grp == 0)
      tile_walk(V, F64_LD, 1, g.B, 0, g.B, (int)i0, (int)j0, 1, g.L, g.np, g.k, rbnd[0], l,
                lane, out);
    else
      tile_walk(V, 1, F64_LD, g.B, 0, g.B, (int)j0, (int)i0, -1, g.L, g.np, g.k, rbnd[1], l,
                lane, out);
  }
}

__global__ __launch_bounds__(256) void fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// One wave per row: the k smallest (distance, index) of the row's appended
// entries, in a lane-resident list (first chunk sorted, later chunks
// ballot-filtered against the list's k-th and inserted). FINAL writes the
// neighbour list (rows whose buffer overflowed are left to the fallback);
// otherwise the row's bound, the k-th distance (+inf with fewer than k).
template <bool FINAL>
__global__ __launch_bounds__(256) void select_kernel(FusedOut out, int np, int k,
                                                     double* __restrict__ bound,
                                                     int32_t* __restrict__ idx,
                                                     double* __restrict__ dist) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= np) return;
  const int total = out.cnt[t];
  if (FINAL && total > out.cap) return;
  const int n = total < out.cap ? total : out.cap;
  const double* bd = out.bd + t * out.cap;
  const int32_t* bi = out.bi + t * out.cap;
  double ed = __builtin_huge_val();
  int ei = INT_MAX;
  for (int c0 = 0; c0 < n; c0 += 64) {
    const bool in = c0 + lane < n;
    double d = in ? bd[c0 + lane] : __builtin_huge_val();
    int c = in ? bi[c0 + lane] : INT_MAX - 64 + lane;
    if (c0 == 0) {
      // lane r now holds the r-th smallest entry; lanes from n on the padding
      bitonic_sort64(d, c, lane);
      ed = lane < n ? d : __builtin_huge_val();
      ei = lane < n ? c : INT_MAX;
    } else {
      const double kd = readlane_d(ed, k - 1);
      const int ki = __builtin_amdgcn_readlane(ei, k - 1);
      const bool pass = in && key_less(d, c, kd, ki);
      const uint64_t m = __ballot(pass);
      if (m) insert_reg(m, d, c, k, ed, ei);
    }
  }
  if (FINAL) {
    if (lane < k) {
      idx[t * k + lane] = lane < n ? ei : -1;
      dist[t * k + lane] = lane < n ? ed : __builtin_huge_val();
    }
  } else if (lane == 0) {
    bound[t] = n >= k ? readlane_d(ed, k - 1) : __builtin_huge_val();
  }
}

// Exact recomputation of the rows whose buffer overflowed (pathological data:
// many candidates tied at a row's bound). One workgroup per row; D_L(t, j) of
// every candidate from the fields in FP64 (Eq. 4, products and sums in
// increasing cell order, exactly as the FP64 tiles form them), rounded to
// FP32 per snapshot pair as the tiles store them and summed over m in FP64.
// Each wave keeps a lane-resident list over its share of the candidates; wave
// 0 then merges the four lists.
__global__ __launch_bounds__(256) void fallback_kernel(const float* __restrict__ X, int64_t ldx,
                                                       int D, const double* __restrict__ mu,
                                                       FusedGeom g, FusedOut out,
                                                       int32_t* __restrict__ idx,
                                                       double* __restrict__ dist) {
  const int t = blockIdx.x;
  if (t >= g.np || out.cnt[t] <= out.cap) return;
  __shared__ double ld_d[4][64];
  __shared__ int ld_i[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int L = g.L, k = g.k;
  auto norm = [&](int64_t r) {
    double s = 0.0;
    for (int p = 0; p < D; ++p) {
      const double x = centred(X, ldx, g.T, D, mu, r, p);
      s = __builtin_fma(x, x, s);
    }
    return s;
  };
  double ed = __builtin_huge_val();
  int ei = INT_MAX;
  for (int j0 = w * 64; j0 < g.np; j0 += 256) {
    const int j = j0 + lane;
    const bool valid = j < g.np && (j - t >= L || t - j >= L);
    double Dl = 0.0;
    if (j < g.np) {
      for (int m = 0; m < L; ++m) {
        const int64_t a = t + m, b = j + m;
        double gab = 0.0;
        for (int p = 0; p < D; ++p)
          gab = __builtin_fma(centred(X, ldx, g.T, D, mu, a, p),
                              centred(X, ldx, g.T, D, mu, b, p), gab);
        // the pair as the tiles evaluate it: the smaller field on the A side
        const double v = a < b ? f64_dist(norm(a), norm(b), gab) : f64_dist(norm(b), norm(a), gab);
        Dl += (double)clamp_distance((float)v);
      }
    }
    const double kd = readlane_d(ed, k - 1);
    const int ki = __builtin_amdgcn_readlane(ei, k - 1);
    const bool pass = valid && key_less(Dl, j, kd, ki);
    const uint64_t m = __ballot(pass);
    if (m) insert_reg(m, Dl, j, k, ed, ei);
  }
  ld_d[w][lane] = ed;
  ld_i[w][lane] = ei;
  __syncthreads();
  if (w != 0) return;
  for (int u = 1; u < 4; ++u) {
    const double d = lane < k ? ld_d[u][lane] : __builtin_huge_val();
    const int c = lane < k ? ld_i[u][lane] : INT_MAX;
    const double kd = readlane_d(ed, k - 1);
    const int ki = __builtin_amdgcn_readlane(ei, k - 1);
    const bool pass = lane < k && c != INT_MAX && key_less(d, c, kd, ki);
    const uint64_t m = __ballot(pass);
    if (m) insert_reg(m, d, c, k, ed, ei);
  }
  if (lane < k) {
    idx[(int64_t)t * k + lane] = ei == INT_MAX ? -1 : ei;
    dist[(int64_t)t * k + lane] = ed;
  }
}

}  // namespace

int64_t fused_establish_tiles(const FusedGeom& g) {
  int64_t n = 0;
  for (int u = 0; u < g.nh; ++u) n += g.nbt - g.h[u];
  return n;
}

hipError_t launch_fused_clear(const FusedGeom& g, const FusedOut& out, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32, dim3((unsigned)((g.np + 255) / 256)), dim3(256), 0, s, out.cnt,
                     (int64_t)g.np, 0);
  return hipGetLastError();
}

hipError_t launch_fused_f64(const float* X, int64_t ldx, int D, const double* mu,
                            const FusedGeom& g, bool establish, const double* bound,
                            const FusedOut& out, hipStream_t s) {
  const int64_t ntiles = establish ? fused_establish_tiles(g)
                                   : (int64_t)g.nbt * (g.nbt + 1) / 2;
  if (ntiles <= 0) return hipSuccess;
  if (establish)
    hipLaunchKernelGGL(fused_f64_kernel<true>, dim3((unsigned)ntiles), dim3(F64_THREADS), 0, s,
                       X, ldx, D, mu, g, bound, out);
  else
    hipLaunchKernelGGL(fused_f64_kernel<false>, dim3((unsigned)ntiles), dim3(F64_THREADS), 0, s,
                       X, ldx, D, mu, g, bound, out);
  return hipGetLastError();
}

hipError_t launch_fused_bound(const FusedGeom& g, const FusedOut& out, double* bound,
                              hipStream_t s) {
  hipLaunchKernelGGL(select_kernel<false>, dim3((unsigned)((g.np + 3) / 4)), dim3(256), 0, s, out,
                     g.np, g.k, bound, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_fused_select(const float* X, int64_t ldx, int D, const double* mu,
                               const FusedGeom& g, const FusedOut& out, int32_t* idx,
                               double* dist, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel<true>, dim3((unsigned)((g.np + 3) / 4)), dim3(256), 0, s, out,
                     g.np, g.k, nullptr, idx, dist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fallback_kernel, dim3((unsigned)g.np), dim3(256), 0, s, X, ldx, D, mu, g,
                     out, idx, dist);
  return hipGetLastError();
}

}  // namespace traknn
