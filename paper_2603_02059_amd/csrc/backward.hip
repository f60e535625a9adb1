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

__global__ __launch_bounds__(256) void rev_count_kernel(
    const int32_t* __restrict__ idx, const double* __restrict__ w, int np,
    int k, int32_t* __restrict__ cnt) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)np * k) return;
  const int t = (int)(g / k);
  if (w[t] == 0.0) return;
  const int j = idx[g];
  if (j >= 0 && j < np) atomicAdd(&cnt[j], 1);
}

// Exclusive scan of cnt[0..n) into ptr[0..n], one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ cnt,
                                                    int n, int32_t* __restrict__ ptr) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b = tid * per;
  const int e = b + per < n ? b + per : n;
  int32_t s = 0;
  for (int i = b; i < e; ++i) s += cnt[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid > 0 ? part[tid - 1] : 0;
  for (int i = b; i < e; ++i) {
    ptr[i] = run;
    run += cnt[i];
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

// Columns per thread: a workgroup gathers one output row over 256 * GCOLS
// columns, and a second grid dimension covers the rest of the row, so a row's
// terms are gathered by several workgroups at once (the gather is latency
// bound: each term is one dependent source-row read).
constexpr int GCOLS = 4;

// Does output row a receive any term?
__device__ __forceinline__ bool row_has_terms(int a, int np, int L, const double* w,
                                              const int32_t* ptr) {
  for (int m = 0; m < L; ++m) {
    const int t = a - m;
    if (t >= 0 && t < np && (w[t] != 0.0 || ptr[t + 1] > ptr[t])) return true;
  }
  return false;
}

__global__ __launch_bounds__(256) void grad_rows_kernel(
    const float* __restrict__ X, int64_t ldx, int T, int64_t D, int L, int k,
    const int32_t* __restrict__ idx, const double* __restrict__ w,
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ rev,
    float* __restrict__ g, int64_t ldg) {
  const int a = blockIdx.x;
  const int np = T - L + 1;
  const int64_t c0 = (int64_t)blockIdx.y * 256 * GCOLS;
  float* ga = g + (int64_t)a * ldg;
  if (!row_has_terms(a, np, L, w, ptr)) {  // untouched row: zeros
#pragma unroll
    for (int e = 0; e < GCOLS; ++e) {
      const int64_t p = c0 + threadIdx.x + 256 * e;
      if (p < D) ga[p] = 0.f;
    }
    return;
  }
  const double invk = 1.0 / (double)k;
  const float* xa = X + (int64_t)a * ldx;
  {
    double acc[GCOLS];
    double xav[GCOLS];
#pragma unroll
    for (int e = 0; e < GCOLS; ++e) {
      const int64_t p = c0 + threadIdx.x + 256 * e;
      acc[e] = 0.0;
      xav[e] = p < D ? (double)xa[p] : 0.0;
    }
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
        const float* xb = X + (int64_t)(j + m) * ldx;
#pragma unroll
        for (int e = 0; e < GCOLS; ++e) {
          const int64_t p = c0 + threadIdx.x + 256 * e;
          if (p < D) acc[e] += c * (xav[e] - (double)xb[p]);
        }
      }
    }
    // W_ba: a = j + m with j in N_t, b = t + m
    for (int m = 0; m < L; ++m) {
      const int j = a - m;
      if (j < 0 || j >= np) continue;
      for (int r = ptr[j]; r < ptr[j + 1]; ++r) {
        const int t = rev[r];
        const double c = w[t] * invk;
        const float* xb = X + (int64_t)(t + m) * ldx;
#pragma unroll
        for (int e = 0; e < GCOLS; ++e) {
          const int64_t p = c0 + threadIdx.x + 256 * e;
          if (p < D) acc[e] += c * (xav[e] - (double)xb[p]);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < GCOLS; ++e) {
      const int64_t p = c0 + threadIdx.x + 256 * e;
      if (p < D) ga[p] = (float)(2.0 * acc[e]);
    }
  }
}

}  // namespace

hipError_t launch_backward(const float* X, int64_t ldx, int64_t T, int64_t D,
                           int L, int k, const int32_t* idx, const double* w,
                           float* g, int64_t ldg, int32_t* cnt, int32_t* ptr,
                           int32_t* fill, int32_t* rev, hipStream_t s) {
  const int np = (int)(T - L + 1);
  const int64_t nk = (int64_t)np * k;
  const unsigned gb = (unsigned)((np + 255) / 256);
  const unsigned gk = (unsigned)((nk + 255) / 256);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(gb), dim3(256), 0, s, cnt, (int64_t)np, 0);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(gb), dim3(256), 0, s, fill, (int64_t)np, 0);
  hipLaunchKernelGGL(rev_count_kernel, dim3(gk), dim3(256), 0, s, idx, w, np, k, cnt);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, cnt, np, ptr);
  hipLaunchKernelGGL(rev_fill_kernel, dim3(gk), dim3(256), 0, s, idx, w, np, k, ptr,
                     fill, rev);
  hipLaunchKernelGGL(rev_sort_kernel, dim3(gb), dim3(256), 0, s, ptr, np, rev);
  const unsigned col_blocks = (unsigned)((D + 256 * GCOLS - 1) / (256 * GCOLS));
  hipLaunchKernelGGL(grad_rows_kernel, dim3((unsigned)T, col_blocks), dim3(256), 0, s, X, ldx,
                     (int)T, D, L, k, idx, w, ptr, rev, g, ldg);
  return hipGetLastError();
}

}  // namespace traknn
