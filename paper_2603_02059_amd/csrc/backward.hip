// Gradient of F = sum_t w_t s_t with the neighbour sets held fixed (Eq. 3 with
// Eq. 2 inside). Writing F = sum_{a,b} W_ab ||x_a - x_b||^2 with
//   W_ab = sum_t (w_t / k) sum_{j in N_t} sum_{m<L} [a = t+m][b = j+m],
// the gradient is a graph-Laplacian product
//   g_a = 2 sum_b (W_ab + W_ba) (x_a - x_b).
// Row a's W_ab terms come straight from the neighbour lists (t = a - m); its
// W_ba terms need the reverse lists (all t with j = a - m in N_t), which are
// built as a CSR: integer counting with atomics, a scan, an atomic fill and a
// per-bucket sort by t, so the reverse lists -- and hence every floating-point
// sum -- come out in the same order on every run. Each output row is then
// gathered in FP64 (field differences of FP32 inputs are exact in FP64) and
// rounded once to FP32; rows that no term touches are written as zeros by the
// same kernel. No distance value is needed: the
// derivative of a squared distance is the field difference itself.
#include "internal.h"

namespace traknn {
namespace {

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t n,
                                                       int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// Reverse-list counts, plus the rows any term touches: a = t + m (the rows
// of a weighted trajectory) and a = j + m (those of its neighbours), m < L.
// Flags are plain stores of 1, so concurrent writers agree.
__global__ __launch_bounds__(256) void rev_count_kernel(
    const int32_t* __restrict__ idx, const double* __restrict__ w, int np,
    int k, int L, int32_t* __restrict__ cnt, int32_t* __restrict__ touch) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)np * k) return;
  const int t = (int)(g / k);
  if (w[t] == 0.0) return;
  const int j = idx[g];
  if (j < 0 || j >= np) return;
  atomicAdd(&cnt[j], 1);
  for (int m = 0; m < L; ++m) {
    touch[t + m] = 1;
    touch[j + m] = 1;
  }
}

// Exclusive scan of cnt[0..n) into ptr[0..n], one workgroup of 1024 threads.
// Each thread sums its run of counts SCAN_BATCH loads at a time, the loads of
// a batch in flight together.
constexpr int SCAN_BATCH = 16;
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ cnt,
                                                    int n, int32_t* __restrict__ ptr) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b = tid * per;
  const int e = b + per < n ? b + per : n;
  int32_t s = 0;
  for (int i0 = b; i0 < e; i0 += SCAN_BATCH) {
    int32_t v[SCAN_BATCH];
#pragma unroll
    for (int u = 0; u < SCAN_BATCH; ++u) v[u] = i0 + u < e ? cnt[i0 + u] : 0;
#pragma unroll
    for (int u = 0; u < SCAN_BATCH; ++u) s += v[u];
  }
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid > 0 ? part[tid - 1] : 0;
  for (int i0 = b; i0 < e; i0 += SCAN_BATCH) {
    int32_t v[SCAN_BATCH];
#pragma unroll
    for (int u = 0; u < SCAN_BATCH; ++u) v[u] = i0 + u < e ? cnt[i0 + u] : 0;
#pragma unroll
    for (int u = 0; u < SCAN_BATCH; ++u) {
      if (i0 + u < e) ptr[i0 + u] = run;
      run += v[u];
    }
  }
  if (tid == 1023) ptr[n] = part[1023];
}

__global__ __launch_bounds__(256) void rev_fill_kernel(
    const int32_t* __restrict__ idx, const double* __restrict__ w, int np,
    int k, const int32_t* __restrict__ ptr, int32_t* __restrict__ fill,
    int32_t* __restrict__ rev) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)np * k) return;
  const int t = (int)(g / k);
  if (w[t] == 0.0) return;
  const int j = idx[g];
  if (j < 0 || j >= np) return;
  const int pos = atomicAdd(&fill[j], 1);
  rev[ptr[j] + pos] = t;
}

// Insertion sort of each reverse bucket by t (buckets hold ~k entries).
__global__ __launch_bounds__(256) void rev_sort_kernel(const int32_t* __restrict__ ptr,
                                                       int np, int32_t* __restrict__ rev) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= np) return;
  const int b = ptr[j], e = ptr[j + 1];
  for (int i = b + 1; i < e; ++i) {
    const int32_t v = rev[i];
    int q = i - 1;
    while (q >= b && rev[q] > v) {
      rev[q + 1] = rev[q];
      --q;
    }
    rev[q + 1] = v;
  }
}

// A workgroup owns GB_COLS columns of one output row: each of its 256
// threads holds GB_VEC groups of 4 consecutive columns, loaded and stored as
// 16-byte vectors (strided rows fall back to scalar stores of the output).
// Rows that no term touches are written as zeros and nothing else; touched
// rows gather their terms in FP64, GB_BATCH terms' source vectors in flight at
// once, rounded once to FP32.
constexpr int GB_VEC = 1;
constexpr int GB_BATCH = 4;  // terms whose source vectors are loaded together
constexpr int GB_COLS = 256 * 4 * GB_VEC;

template <bool VEC_OUT>
__global__ __launch_bounds__(256) void grad_rows_kernel(
    const float* __restrict__ X, int64_t ldx, int T, int64_t D, int L, int k,
    const int32_t* __restrict__ idx, const double* __restrict__ w,
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ rev,
    const int32_t* __restrict__ touch, float* __restrict__ g, int64_t ldg) {
  const int a = blockIdx.x;
  const int np = T - L + 1;
  const int64_t cbase = (int64_t)blockIdx.y * GB_COLS + 4 * threadIdx.x;
  float* ga = g + (int64_t)a * ldg;
  auto store = [&](int64_t c, float4 v) __attribute__((always_inline)) {
    if (VEC_OUT && c + 3 < D) {
      *(float4*)(ga + c) = v;
    } else {
      if (c < D) ga[c] = v.x;
      if (c + 1 < D) ga[c + 1] = v.y;
      if (c + 2 < D) ga[c + 2] = v.z;
      if (c + 3 < D) ga[c + 3] = v.w;
    }
  };
  if (!touch[a]) {
#pragma unroll
    for (int v = 0; v < GB_VEC; ++v) store(cbase + 1024 * v, make_float4(0.f, 0.f, 0.f, 0.f));
    return;
  }
  // FP32 source vector of row r at the thread's columns (zero past D)
  auto load = [&](int64_t r, int v) __attribute__((always_inline)) {
    const int64_t c = cbase + 1024 * v;
    const float* p = X + r * ldx + c;
    if (c + 3 < D) return *(const float4*)p;
    return make_float4(c < D ? p[0] : 0.f, c + 1 < D ? p[1] : 0.f, c + 2 < D ? p[2] : 0.f,
                       c + 3 < D ? p[3] : 0.f);
  };
  double acc[GB_VEC][4];
  double xa[GB_VEC][4];
#pragma unroll
  for (int v = 0; v < GB_VEC; ++v) {
    const float4 x = load(a, v);
    xa[v][0] = x.x, xa[v][1] = x.y, xa[v][2] = x.z, xa[v][3] = x.w;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;
  }
  const double invk = 1.0 / (double)k;
  // Terms go in batches of GB_BATCH, every source vector of a batch loaded
  // before any is used, so a row with many terms waits for one memory round
  // trip per batch instead of one per term. Unused entries of a batch read the
  // row itself with weight 0 (an exact zero contribution).
  int64_t tb[GB_BATCH];
  double tc[GB_BATCH];
  int nt = 0;
  auto flush = [&]() __attribute__((always_inline)) {
    float4 xb[GB_BATCH][GB_VEC];
#pragma unroll
    for (int u = 0; u < GB_BATCH; ++u)
#pragma unroll
      for (int v = 0; v < GB_VEC; ++v) xb[u][v] = load(u < nt ? tb[u] : a, v);
#pragma unroll
    for (int u = 0; u < GB_BATCH; ++u) {
      const double c = u < nt ? tc[u] : 0.0;
#pragma unroll
      for (int v = 0; v < GB_VEC; ++v) {
        acc[v][0] += c * (xa[v][0] - (double)xb[u][v].x);
        acc[v][1] += c * (xa[v][1] - (double)xb[u][v].y);
        acc[v][2] += c * (xa[v][2] - (double)xb[u][v].z);
        acc[v][3] += c * (xa[v][3] - (double)xb[u][v].w);
      }
    }
    nt = 0;
  };
  auto term = [&](int64_t b, double c) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < GB_BATCH; ++u)
      if (u == nt) tb[u] = b, tc[u] = c;
    if (++nt == GB_BATCH) flush();
  };
  // W_ab: a = t + m, b = j + m for j in N_t
  for (int m = 0; m < L; ++m) {
    const int t = a - m;
    if (t < 0 || t >= np) continue;
    const double wt = w[t];
    if (wt == 0.0) continue;
    const double c = wt * invk;
    for (int q = 0; q < k; ++q) {
      const int j = idx[(int64_t)t * k + q];
      if (j < 0 || j >= np) continue;
      term(j + m, c);
    }
  }
  // W_ba: a = j + m with j in N_t, b = t + m
  for (int m = 0; m < L; ++m) {
    const int j = a - m;
    if (j < 0 || j >= np) continue;
    for (int r = ptr[j]; r < ptr[j + 1]; ++r) {
      const int t = rev[r];
      term(t + m, w[t] * invk);
    }
  }
  if (nt) flush();
#pragma unroll
  for (int v = 0; v < GB_VEC; ++v)
    store(cbase + 1024 * v, make_float4((float)(2.0 * acc[v][0]), (float)(2.0 * acc[v][1]),
                                        (float)(2.0 * acc[v][2]), (float)(2.0 * acc[v][3])));
}

}  // namespace

hipError_t launch_backward(const float* X, int64_t ldx, int64_t T, int64_t D,
                           int L, int k, const int32_t* idx, const double* w,
                           float* g, int64_t ldg, int32_t* zeroed, int32_t* ptr,
                           int32_t* rev, hipStream_t s) {
  // zeroed: the contiguous int32 arrays cnt [np], fill [np], touch [T]
  const int np = (int)(T - L + 1);
  int32_t* cnt = zeroed;
  int32_t* fill = zeroed + np;
  int32_t* touch = zeroed + 2 * (int64_t)np;
  const int64_t nz = 2 * (int64_t)np + T;
  const int64_t nk = (int64_t)np * k;
  const unsigned gb = (unsigned)((np + 255) / 256);
  const unsigned gk = (unsigned)((nk + 255) / 256);
  hipError_t e;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s,
                     zeroed, nz, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(rev_count_kernel, dim3(gk), dim3(256), 0, s, idx, w, np, k, L, cnt, touch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, cnt, np, ptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(rev_fill_kernel, dim3(gk), dim3(256), 0, s, idx, w, np, k, ptr,
                     fill, rev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(rev_sort_kernel, dim3(gb), dim3(256), 0, s, ptr, np, rev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 grid((unsigned)T, (unsigned)((D + GB_COLS - 1) / GB_COLS));
  const bool vec_out = ldg % 4 == 0 && ((uintptr_t)g % 16) == 0;
  if (vec_out)
    hipLaunchKernelGGL(grad_rows_kernel<true>, grid, dim3(256), 0, s, X, ldx, (int)T, D, L, k,
                       idx, w, ptr, rev, touch, g, ldg);
  else
    hipLaunchKernelGGL(grad_rows_kernel<false>, grid, dim3(256), 0, s, X, ldx, (int)T, D, L, k,
                       idx, w, ptr, rev, touch, g, ldg);
  return hipGetLastError();
}

}  // namespace traknn
