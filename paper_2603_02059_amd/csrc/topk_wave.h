// Wave-level (distance, index) top-k helpers shared by the window kernels and
// the fused tile kernels: a sorted list of up to 64 entries is held one entry
// per lane (lane q holds entry q), candidates arrive 64 at a time (one per
// lane), and keys compare lexicographically by (distance, index) so every
// list is unique (paper, Eq. 3 with ties broken by the smaller index).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace traknn {

__device__ __forceinline__ double readlane_d(double v, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
// (ad, ai) < (bd, bi) lexicographically; bitwise, so it compiles to three
// compares and two mask operations instead of short-circuit branches.
__device__ __forceinline__ bool key_less(double ad, int ai, double bd, int bi) {
  return (ad < bd) | ((ad == bd) & (ai < bi));
}

__device__ __forceinline__ double dpp_shr1_d(double v, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int dpp_shr1_i(int v, int old) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xF, 0xF, false);
}

// Insert the masked lanes' candidates (D, col), in lane order, into a sorted
// list held in registers (lane q < k holds entry q; lanes from k on are
// don't-care): each insertion that beats the k-th entry shifts the tail of
// the list one lane up with DPP wave_shr:1.
__device__ __forceinline__ void insert_reg(uint64_t mask, double D, int col, int k,
                                           double& ed, int& ei) {
  while (mask) {
    const int src = __builtin_ctzll(mask);
    mask &= mask - 1;
    const double cd = readlane_d(D, src);
    const int ci = __builtin_amdgcn_readlane(col, src);
    const double kd = readlane_d(ed, k - 1);
    const int ki = __builtin_amdgcn_readlane(ei, k - 1);
    if (!key_less(cd, ci, kd, ki)) continue;
    const double pd = dpp_shr1_d(ed, -__builtin_huge_val());  // lane 0: -inf
    const int pi = dpp_shr1_i(ei, INT_MIN);
    const bool lt_prev = key_less(cd, ci, pd, pi);
    const bool lt_self = key_less(cd, ci, ed, ei);
    ed = lt_prev ? pd : (lt_self ? cd : ed);
    ei = lt_prev ? pi : (lt_self ? ci : ei);
  }
}

// Insert the ballot's candidates (D, col) of row s into its sorted list in
// LDS (loaded into lanes q < k while inserting) and refresh the row threshold
// kept by lane s.
__device__ __forceinline__ void insert_seq(uint64_t mask, double D, int col, int k,
                                           double* rd, int* ri, int lane, int s,
                                           double& thr_d, int& thr_i) {
  double ed = lane < k ? rd[lane] : __builtin_huge_val();
  int ei = lane < k ? ri[lane] : INT_MAX;
  insert_reg(mask, D, col, k, ed, ei);
  if (lane < k) {
    rd[lane] = ed;
    ri[lane] = ei;
  }
  const double nd = readlane_d(ed, k - 1);
  const int ni = __builtin_amdgcn_readlane(ei, k - 1);
  if (lane == s) {
    thr_d = nd;
    thr_i = ni;
  }
}

// The value v of lane (lane ^ S), S a power of two up to 32. Strides up to
// 8 stay inside rows of 16 lanes and use DPP moves, which are plain vector
// ALU operations: quad permutes for 1 and 2; row rotations for 8 (by 8) and
// for 4 (by 12 where bit 2 of the lane is clear, giving lane + 4, else by 4,
// giving lane - 4). 16 uses a swizzle within 32 lanes and 32 a permute, both
// through the LDS crossbar. Every lane of the wave must be active.
template <int S>
__device__ __forceinline__ int lane_xor(int v, int lane) {
  static_assert(S == 1 || S == 2 || S == 4 || S == 8 || S == 16 || S == 32, "stride");
  if constexpr (S == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (S == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (S == 4) {
    const int up = __builtin_amdgcn_mov_dpp(v, 0x12C, 0xF, 0xF, false);  // row_ror:12
    const int dn = __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, false);  // row_ror:4
    return (lane & 4) ? dn : up;
  } else if constexpr (S == 8) {
    return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (S == 16) {
    return __builtin_amdgcn_ds_swizzle(v, (16 << 10) | 0x1F);  // bit mode, xor mask 16
  } else {
    return __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
  }
}

// One merge of a bitonic network over the wave: compare-exchange with the
// lane S apart, then S / 2, ... 1; blocks of SIZE lanes end ascending where
// bit SIZE of the lane is clear, descending elsewhere.
template <int SIZE, int S>
__device__ __forceinline__ void bitonic_merge64(double& d, int& c, int lane) {
  const double pd = __hiloint2double(lane_xor<S>(__double2hiint(d), lane),
                                     lane_xor<S>(__double2loint(d), lane));
  const int pc = lane_xor<S>(c, lane);
  const bool asc = (lane & SIZE) == 0;
  const bool lower = (lane & S) == 0;
  if ((lower == asc) == key_less(pd, pc, d, c)) {
    d = pd;
    c = pc;
  }
  if constexpr (S > 1) bitonic_merge64<SIZE, S / 2>(d, c, lane);
}

// Sort the wave's 64 keys (d, c) ascending by (distance, index) across the
// lanes: afterwards lane r holds the r-th smallest (bitonic network of lane
// exchanges, unrolled so that every stride is a compile-time constant). Keys
// must be distinct for a unique result; every lane must be active.
template <int SIZE = 2>
__device__ __forceinline__ void bitonic_sort64(double& d, int& c, int lane) {
  bitonic_merge64<SIZE, SIZE / 2>(d, c, lane);
  if constexpr (SIZE < 64) bitonic_sort64<SIZE * 2>(d, c, lane);
}

// The same sort as a loop over run-time strides, each exchange a permute
// through the LDS crossbar: slower per sort, but compact and light on
// registers, for kernels that sort once per wave (the window's list seeds).
// In the window kernels the unrolled network costs 4 registers, one wave per
// SIMD and, with two lengths, spills.
__device__ __forceinline__ void bitonic_sort64_compact(double& d, int& c, int lane) {
#pragma unroll 1
  for (int size = 2; size <= 64; size <<= 1)
#pragma unroll 1
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const double pd = __shfl_xor(d, stride, 64);
      const int pc = __shfl_xor(c, stride, 64);
      const bool asc = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      if ((lower == asc) == key_less(pd, pc, d, c)) {
        d = pd;
        c = pc;
      }
    }
}

// Seed row s's list with the k smallest of this step's 64 candidates: bitonic
// sort of (D, col) across the wave (invalid lanes carry +inf and a distinct
// index above every column), lanes q < k keep the q-th smallest.
__device__ __forceinline__ void seed_row(double d, int c, bool valid, int k, double* rd,
                                         int* ri, int lane, int s, double& thr_d,
                                         int& thr_i) {
  if (!valid) {
    d = __builtin_huge_val();
    c = INT_MAX - 64 + lane;
  }
  bitonic_sort64_compact(d, c, lane);
  const bool sentinel = d == __builtin_huge_val();
  if (lane < k) {
    rd[lane] = d;
    ri[lane] = sentinel ? INT_MAX : c;
  }
  const double nd = readlane_d(d, k - 1);
  const int nc = __builtin_amdgcn_readlane(c, k - 1);
  if (lane == s) {
    thr_d = nd;
    thr_i = nd == __builtin_huge_val() ? INT_MAX : nc;
  }
}

}  // namespace traknn
