// Centring, precision conversion and squared norms (the precomputed norms of
// Algorithm 1, stage 1; Eq. 4).
//
// Distances are translation invariant, so the fields are shifted per grid cell
// before the Gram product: with ~1e5 Pa offsets the uncentred inner products
// would cancel against the norms and lose every bit the reduced-precision
// paths carry. Any per-cell shift gives the same distances; the shift only has
// to remove the offset. It is the FP64 mean over an evenly strided sample of
// at most COLSTAT_SAMPLE rows (every row when T is at most that), which reads
// a small fraction of X and lies within about sigma / sqrt(COLSTAT_SAMPLE) of
// the full mean. Centred values are FP64. The squared norms are taken
// per chunk of GRAM_CHUNK elements, in FP64, of exactly the vector the Gram
// stage represents (FP32, FP16 or hi + lo), so that the Gram stage's
// N_i + N_j - 2G, assembled chunk by chunk, is a distance between the same two
// vectors up to the accumulation error (and, for BF16x3, the zero-mean lo.lo
// cross term).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "internal.h"

namespace traknn {
namespace {

// Partial column sums of the sampled rows (sample r is row r * stride) over
// blocks of COLSTAT_ROWS samples: each thread sums 4 consecutive cells (one
// 16-byte load per row, 1 KB per wave and row), eight rows in flight at a
// time, in a fixed order.
__global__ __launch_bounds__(256) void colsum_partial_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t nsamp, int64_t stride, int64_t D,
    double* __restrict__ part) {
  const int64_t c = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  const int64_t r0 = (int64_t)blockIdx.y * COLSTAT_ROWS;
  if (c >= D) return;
  const int64_t r1 = r0 + COLSTAT_ROWS < nsamp ? r0 + COLSTAT_ROWS : nsamp;
  const int64_t step = stride * ldx;  // floats between sampled rows
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (c + 4 <= D) {
    const float* p = X + r0 * step + c;
    int64_t r = r0;
    for (; r + 8 <= r1; r += 8) {
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = *(const float4*)(p + u * step);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s0 += (double)v[u].x;
        s1 += (double)v[u].y;
        s2 += (double)v[u].z;
        s3 += (double)v[u].w;
      }
      p += 8 * step;
    }
    for (; r < r1; ++r, p += step) {
      const float4 v = *(const float4*)p;
      s0 += (double)v.x;
      s1 += (double)v.y;
      s2 += (double)v.z;
      s3 += (double)v.w;
    }
  } else {
    for (int64_t r = r0; r < r1; ++r) {
      const float* p = X + r * step + c;
      s0 += (double)p[0];
      if (c + 1 < D) s1 += (double)p[1];
      if (c + 2 < D) s2 += (double)p[2];
    }
  }
  double* out = part + (int64_t)blockIdx.y * D + c;
  out[0] = s0;
  if (c + 1 < D) out[1] = s1;
  if (c + 2 < D) out[2] = s2;
  if (c + 3 < D) out[3] = s3;
}

// Fixed-order reduction of the partial sums -> per-cell sample mean.
__global__ __launch_bounds__(256) void colsum_reduce_kernel(
    const double* __restrict__ part, int64_t nsamp, int64_t D, int nchunks,
    double* __restrict__ mu) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= D) return;
  double s = 0.0;
#pragma unroll 8
  for (int q = 0; q < nchunks; ++q) s += part[(int64_t)q * D + c];
  mu[c] = s / (double)nsamp;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline uint32_t bf16_bits_rne(float f) {
  // round-to-nearest-even of an FP32 value to BF16 (inputs are finite)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline double bf16_bits_to_double(uint32_t b) {
  return (double)__uint_as_float(b << 16);
}

// Wave (blockIdx.x * 4 + w) owns norm chunk ch = that index (GRAM_CHUNK
// elements; lane q the 8 consecutive elements 8q .. 8q+7) and converts it for
// CONV_ROWS consecutive rows starting at blockIdx.y * CONV_ROWS, keeping the
// chunk's means in registers: two 16-byte loads and one or two 16-byte stores
// per lane and row. Each (row, chunk) squared norm (FP64 sum, stored FP32) goes
// to ncs[chunk * Tpad + row]. PREC selects the emitted representation.
constexpr int CONV_ROWS = 16;
template <int PREC>
__global__ __launch_bounds__(256) void centre_convert_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t T, int64_t D,
    int64_t Tpad, int64_t Dpad, const double* __restrict__ mu,
    void* __restrict__ xc, float* __restrict__ ncs) {
  static_assert(GRAM_CHUNK == 64 * 8, "a wave covers one norm chunk");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t ch = (int64_t)blockIdx.x * 4 + w;
  if (ch >= norm_chunks(Dpad)) return;
  const int64_t e0 = ch * GRAM_CHUNK + 8 * lane;  // Dpad is a multiple of 8
  const bool in_pad = e0 < Dpad;
  const bool full = e0 + 8 <= D;
  double m[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) m[u] = e0 + u < D ? mu[e0 + u] : 0.0;
  for (int rr = 0; rr < CONV_ROWS; ++rr) {
    const int64_t i = (int64_t)blockIdx.y * CONV_ROWS + rr;
    if (i >= Tpad) break;
    const bool live = i < T;
    const float* xrow = X + i * ldx;
    double acc = 0.0;
    if (in_pad) {
      double v[8];
      if (live && full) {
        const float4 a = *(const float4*)(xrow + e0);
        const float4 b = *(const float4*)(xrow + e0 + 4);
        v[0] = (double)a.x - m[0];
        v[1] = (double)a.y - m[1];
        v[2] = (double)a.z - m[2];
        v[3] = (double)a.w - m[3];
        v[4] = (double)b.x - m[4];
        v[5] = (double)b.y - m[5];
        v[6] = (double)b.z - m[6];
        v[7] = (double)b.w - m[7];
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t e = e0 + u;
          v[u] = (live && e < D) ? (double)xrow[e] - m[u] : 0.0;
        }
      }
      if constexpr (PREC == TRAKNN_FP32) {
        float f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          f[u] = (float)v[u];
          acc += (double)f[u] * (double)f[u];
        }
        float4* out = (float4*)((float*)xc + i * Dpad + e0);
        out[0] = make_float4(f[0], f[1], f[2], f[3]);
        out[1] = make_float4(f[4], f[5], f[6], f[7]);
      } else if constexpr (PREC == TRAKNN_FP16) {
        uint32_t packed[4];
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          const _Float16 h0 = (_Float16)(float)v[u], h1 = (_Float16)(float)v[u + 1];
          const double d0 = (double)(float)h0, d1 = (double)(float)h1;
          acc += d0 * d0;
          acc += d1 * d1;
          packed[u / 2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) |
                          ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        }
        *(uint4*)((_Float16*)xc + i * Dpad + e0) =
            make_uint4(packed[0], packed[1], packed[2], packed[3]);
      } else {
        // BF16X3: the 16-byte chunk of 8 hi values is followed by the chunk of
        // the 8 matching lo values, so one 128-byte Gram stage row holds 32
        // (hi, lo) pairs.
        uint32_t hp[4], lp[4];
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          uint32_t hb[2], lb[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            hb[t] = bf16_bits_rne((float)v[u + t]);
            const double hd = bf16_bits_to_double(hb[t]);
            lb[t] = bf16_bits_rne((float)(v[u + t] - hd));
            // norm of the represented value hi + lo (exact in FP64). The Gram
            // stage drops only the cross term lo_i.lo_j, which has zero mean;
            // a norm made of the three kept products alone would bias every
            // distance low by sum (lo_i - lo_j)^2 ~ 2.5e-6 (N_i + N_j).
            const double xv = hd + bf16_bits_to_double(lb[t]);
            acc += xv * xv;
          }
          hp[u / 2] = hb[0] | (hb[1] << 16);
          lp[u / 2] = lb[0] | (lb[1] << 16);
        }
        uint4* out = (uint4*)((uint16_t*)xc + i * Dpad * 2 + 2 * e0);
        out[0] = make_uint4(hp[0], hp[1], hp[2], hp[3]);
        out[1] = make_uint4(lp[0], lp[1], lp[2], lp[3]);
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) ncs[ch * Tpad + i] = live ? (float)acc : 0.f;
  }
}

}  // namespace

hipError_t launch_colstats(const float* X, int64_t ldx, int64_t T, int64_t D,
                           int tchunks, double* mu_part, double* mu,
                           hipStream_t s) {
  const int64_t stride = colstat_stride(T);
  const int64_t nsamp = (T + stride - 1) / stride;
  dim3 g1((unsigned)((D + 1023) / 1024), (unsigned)tchunks);
  hipLaunchKernelGGL(colsum_partial_kernel, g1, dim3(256), 0, s, X, ldx, nsamp, stride, D,
                     mu_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((unsigned)((D + 255) / 256)),
                     dim3(256), 0, s, mu_part, nsamp, D, tchunks, mu);
  return hipGetLastError();
}

hipError_t launch_centre_convert(const float* X, int64_t ldx, int64_t T,
                                 int64_t D, int64_t Tpad, int64_t Dpad,
                                 int precision, const double* mu, void* xc,
                                 float* ncs, hipStream_t s) {
  dim3 g((unsigned)((norm_chunks(Dpad) + 3) / 4), (unsigned)((Tpad + CONV_ROWS - 1) / CONV_ROWS));
  switch (precision) {
    case TRAKNN_FP32:
      hipLaunchKernelGGL(centre_convert_kernel<TRAKNN_FP32>, g, dim3(256), 0, s,
                         X, ldx, T, D, Tpad, Dpad, mu, xc, ncs);
      break;
    case TRAKNN_BF16X3:
      hipLaunchKernelGGL(centre_convert_kernel<TRAKNN_BF16X3>, g, dim3(256), 0,
                         s, X, ldx, T, D, Tpad, Dpad, mu, xc, ncs);
      break;
    default:
      hipLaunchKernelGGL(centre_convert_kernel<TRAKNN_FP16>, g, dim3(256), 0, s,
                         X, ldx, T, D, Tpad, Dpad, mu, xc, ncs);
      break;
  }
  return hipGetLastError();
}

}  // namespace traknn
