// Centring, precision conversion and squared norms (the precomputed norms of
// Algorithm 1, stage 1; Eq. 4).
//
// Distances are translation invariant, so the fields are centred per grid cell
// before the Gram product: with ~1e5 Pa offsets the uncentred inner products
// would cancel against the norms and lose every bit the reduced-precision
// paths carry. Means and centred values are FP64. The squared norms are taken
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

// Partial column sums over blocks of COLSTAT_ROWS rows: one thread per cell,
// a wave reads 64 consecutive floats of a row.
__global__ __launch_bounds__(256) void colsum_partial_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t T, int64_t D,
    double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * COLSTAT_ROWS;
  if (c >= D) return;
  const int64_t r1 = r0 + COLSTAT_ROWS < T ? r0 + COLSTAT_ROWS : T;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += (double)X[r * ldx + c];
  part[(int64_t)blockIdx.y * D + c] = s;
}

// Fixed-order reduction of the partial sums -> per-cell mean.
__global__ __launch_bounds__(256) void colsum_reduce_kernel(
    const double* __restrict__ part, int64_t T, int64_t D, int nchunks,
    double* __restrict__ mu) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= D) return;
  double s = 0.0;
  for (int q = 0; q < nchunks; ++q) s += part[(int64_t)q * D + c];
  mu[c] = s / (double)T;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline uint16_t bf16_bits_rne(float f) {
  // round-to-nearest-even of an FP32 value to BF16 (inputs are finite)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_bits_to_double(uint16_t b) {
  return (double)__uint_as_float((uint32_t)b << 16);
}

// One workgroup of 4 waves per (padded) row; wave w converts the norm chunks
// w, w + 4, ... of GRAM_CHUNK elements and writes each chunk's squared norm
// (FP64 sum in a fixed order, stored FP32) to ncs[chunk * Tpad + row]. PREC
// selects the emitted representation.
template <int PREC>
__global__ __launch_bounds__(256) void centre_convert_kernel(
    const float* __restrict__ X, int64_t ldx, int64_t T, int64_t D,
    int64_t Tpad, int64_t Dpad, const double* __restrict__ mu,
    void* __restrict__ xc, float* __restrict__ ncs) {
  const int64_t i = blockIdx.x;
  const bool live = i < T;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nch = norm_chunks(Dpad);
  for (int64_t ch = w; ch < nch; ch += 4) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < GRAM_CHUNK / 64; ++m) {
      const int64_t c = ch * GRAM_CHUNK + m * 64 + lane;
      if (c >= Dpad) break;
      const double v = (live && c < D) ? (double)X[i * ldx + c] - mu[c] : 0.0;
      if constexpr (PREC == TRAKNN_FP32) {
        const float f = (float)v;
        const double fd = (double)f;
        acc += fd * fd;
        ((float*)xc)[i * Dpad + c] = f;
      } else if constexpr (PREC == TRAKNN_FP16) {
        const _Float16 h = (_Float16)(float)v;
        const double hd = (double)(float)h;
        acc += hd * hd;
        ((_Float16*)xc)[i * Dpad + c] = h;
      } else {
        // BF16X3: 16-byte chunks alternate 8 hi values and the 8 matching lo
        // values, so one 128-byte Gram stage row holds 32 (hi, lo) pairs.
        const uint16_t hb = bf16_bits_rne((float)v);
        const double hd = bf16_bits_to_double(hb);
        const uint16_t lb = bf16_bits_rne((float)(v - hd));
        const double ld = bf16_bits_to_double(lb);
        // norm of the represented value hi + lo (exact in FP64). The Gram
        // stage drops only the cross term lo_i.lo_j, which has zero mean; a
        // norm made of the three kept products alone would bias every
        // distance low by sum (lo_i - lo_j)^2 ~ 2.5e-6 (N_i + N_j).
        const double xv = hd + ld;
        acc += xv * xv;
        uint16_t* out = (uint16_t*)xc + i * Dpad * 2;
        const int64_t chunk = c >> 3, within = c & 7;
        out[chunk * 16 + within] = hb;
        out[chunk * 16 + 8 + within] = lb;
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
  dim3 g1((unsigned)((D + 255) / 256), (unsigned)tchunks);
  hipLaunchKernelGGL(colsum_partial_kernel, g1, dim3(256), 0, s, X, ldx, T, D,
                     mu_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((unsigned)((D + 255) / 256)),
                     dim3(256), 0, s, mu_part, T, D, tchunks, mu);
  return hipGetLastError();
}

hipError_t launch_centre_convert(const float* X, int64_t ldx, int64_t T,
                                 int64_t D, int64_t Tpad, int64_t Dpad,
                                 int precision, const double* mu, void* xc,
                                 float* ncs, hipStream_t s) {
  dim3 g((unsigned)Tpad);
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
