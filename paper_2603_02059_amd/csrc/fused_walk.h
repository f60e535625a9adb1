// The tile consumer of the fused (S-free) path: trajectory distances and the
// row/column top-k on a tile of snapshot distances held in LDS, so the T x T
// matrix never goes to HBM (paper, Algorithm 1 stages 2-3 applied per tile of
// stage 1; Eq. 5 along the tile's diagonals; the exclusion zone and Eq. 3's
// k nearest).
//
// A tile pairs trajectory rows i = i0 + a with trajectory columns j = j0 + b,
// a, b < B, and holds the snapshot distances d(i0 + a', j0 + b') for a', b' <
// B + L - 1 (the tiles of a launch overlap by L - 1 fields, so every
// trajectory pair of the tile has all L terms of Eq. 2 inside it). Each
// unordered pair i < j is owned by exactly one tile (i's block-row, j's
// block-column, upper triangle of tiles) and is a candidate twice: for row i
// (candidate j) on the tile's ROW side and for row j (candidate i) on its
// COLUMN side. The column side is the row side of the transposed tile, so one
// routine serves both: the recipient axis p and the candidate axis q of the
// staged values are addressed as V[p * sp + q * sq].
//
// Every (recipient, tile side) writes the list of its candidates it keeps --
// at most k -- to its own slot (FusedSlots), and a select kernel takes the k
// nearest over a row's slots. Each recipient is handled by one wave (lane =
// candidate), which gathers its candidates in registers and in its own LDS
// scratch: nothing goes through global atomics and nothing can overflow.
//  * ESTABLISH (the first round, the tiles nearest the diagonal): a recipient
//    keeps its exact k nearest in the tile. A refresh then takes each row's
//    k-th over these slots: an upper bound of its true k-th distance.
//  * FILTER (every later round): a recipient keeps the k nearest of its
//    candidates within its bound. A true neighbour is never above the bound,
//    so the slots always contain the k nearest. These rounds' tiles lie two
//    or more blocks from the diagonal, so no pair is in the exclusion zone.
#pragma once

#include "internal.h"
#include "topk_wave.h"

namespace traknn {

// Tile u of a round: the tiles (I, J) with g.blo <= J - I < g.bhi, row by
// row (row I holds those of its J), so that consecutive tiles share their A
// panel and neighbouring rows most of their B panels.
__device__ __forceinline__ bool fused_band_tile(int64_t u, const FusedGeom& g, int& I, int& J) {
  const int lo = g.blo, hi = g.bhi < g.nbt ? g.bhi : g.nbt;
  const int w = hi - lo;
  if (w <= 0) return false;
  // rows I <= nbt - hi hold all w offsets; later rows nbt - I - lo of them
  const int64_t full = g.nbt - hi + 1 > 0 ? g.nbt - hi + 1 : 0;
  if (u < full * w) {
    I = (int)(u / w);
    J = I + lo + (int)(u % w);
    return true;
  }
  u -= full * w;
  for (int i = (int)full; i < g.nbt; ++i) {
    const int n = g.nbt - i - lo;
    if (n <= 0) return false;
    if (u < n) {
      I = i;
      J = i + lo + (int)u;
      return true;
    }
    u -= n;
  }
  return false;
}

// Write a recipient's list (lanes q < n hold entries) to its slot.
__device__ __forceinline__ void slot_write(const FusedSlots& o, int t, int slot, int n,
                                           double ed, int ei, int lane) {
  const int64_t s = (int64_t)t * o.nslot + slot;
  if (lane == 0) o.cnt[s] = n;
  if (lane < n) {
    o.d[s * o.k + lane] = ed;
    o.i[s * o.k + lane] = ei;
  }
}

// An FP32 bound that no FP32 sum of L <= 16 non-negative FP32 terms exceeds
// when the FP64 sum of the same terms is at most `bound`: recursive FP32
// summation errs by at most (L - 1) 2^-24 / (1 - (L - 1) 2^-24) < 2^-20 of the
// exact sum, and the FP64 sum by far less, so bound (1 + 2^-20) rounded up to
// FP32 is safe (+inf stays +inf, a negative bound stays negative).
__device__ __forceinline__ float prefilter_bound(double bound) {
  const double b = bound > 0.0 ? bound * (1.0 + 0x1p-20) : bound;
  float f = (float)b;
  // below b (only if b > 0): the next float up, by its bit pattern
  if ((double)f < b) f = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, f) + 1u);
  return f;
}

// LLVM's predicate code of an ordered <= (false on NaN), for the compare
// builtins that return the wave's lane mask directly
constexpr int FCMP_OLE = 5;

// A batch with at least this many candidates below the k-th of a sorted list
// is merged into it by sorts rather than by one insertion each.
constexpr int LIST_SORT_MIN = 6;

// Per-wave LDS scratch of a recipient's candidates: up to 64 compacted entries.
struct EstScratch {
  double* d;  // [64]
  int* i;     // [64]
};
constexpr int EST_SCRATCH_BYTES = 64 * (sizeof(double) + sizeof(int));

// Lane masks of the candidates of each batch of 64 (lane = candidate q of
// q0 + 64 b ..): q < Q and q0 + q < np and, for a recipient pg given
// (pg >= 0), outside its exclusion zone (sign (q0 + q - pg) >= L).
template <int NB>
__device__ __forceinline__ void batch_masks(int Q, int q0, int np, int pg, int sign, int L,
                                            int lane, uint64_t (&rng)[NB]) {
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int q = 64 * b + lane;
    const int qg = q0 + q;
    rng[b] = __builtin_amdgcn_ballot_w64((q < Q) & (qg < np) &
                                         (pg < 0 || sign * (qg - pg) >= L));
  }
}

// The k nearest candidates within `bound` (+inf: all) of recipient s, from
// direct L-term sums (Eq. 2) over the staged values. The candidates come 64
// at a time (lane = candidate), those of batch b in rng[b]; the NB batches of
// the recipient (Q <= 64 NB) are loaded before their ballots, as many at once as 24 staged values per
// lane allow, so a recipient costs one or two LDS round trips. With a finite
// bound (FILTER) each batch is first tested on its FP32 sums against bound32
// (prefilter_bound): a candidate whose FP64 sum is within the bound always
// passes, and only batches where some candidate passes form the FP64 sums,
// which decide. Candidates within the bound are compacted into the wave's
// scratch; while there are at most 64 of them nothing is compared, and at
// the end more than k are sorted (the k smallest kept) and at most k are
// kept as they are, unsorted. A batch that would take the scratch past 64
// entries turns it into a sorted list in registers, into which that batch
// and the later ones are merged (without a bound, by sorts when many of a
// batch are below the list's k-th; else one insertion each). Returns how many
// lanes (from 0) hold
// entries. The FP64 sums run in increasing m, as the matrix mode's windows
// start them; for FP32 snapshot distances whose exponents span less than
// about 29 bits every FP64 sum is exact, so both modes give the same D_L.
template <int L, int NB, bool FILTER>
__device__ __forceinline__ int recipient_topk(const float* V, int sp, int sq, int Q, int s,
                                              int q0, const uint64_t (&rng)[NB], int k,
                                              double bound, float bound32, int lane,
                                              const EstScratch& sc, double& ed, int& ei) {
  // batches in flight together (a divisor of NB): at most 24 staged values
  // per lane
  constexpr int NG = NB * L <= 24 ? NB : (NB % 2 == 0 && NB * L <= 48 ? NB / 2 : 1);
  const int step = sp + sq;
  ed = __builtin_huge_val();
  ei = INT_MAX;
  int total = 0;        // entries in the scratch
  bool listed = false;  // the entries are a sorted list in ed/ei instead
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += NG) {
    float w[NG][L];
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      const int q = 64 * (b0 + b) + lane;
      const float* v = V + s * sp + (q < Q ? q : 0) * sq;  // idle lanes: a valid address
#pragma unroll
      for (int m = 0; m < L; ++m) w[b][m] = v[m * step];
    }
    // the batches' candidates as wave masks (FILTER: FP32 sum within); the
    // compares give their lane masks directly, with no per-lane flag
    uint64_t cm[NG];
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      cm[b] = rng[b0 + b];
      if constexpr (FILTER) {
        float s32 = w[b][0];
#pragma unroll
        for (int m = 1; m < L; ++m) s32 += w[b][m];
        cm[b] &= __builtin_amdgcn_fcmpf(s32, bound32, FCMP_OLE);
      }
    }
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      if (!cm[b]) continue;
      const int qg = q0 + 64 * (b0 + b) + lane;
      double D = (double)w[b][0];
#pragma unroll
      for (int m = 1; m < L; ++m) D += (double)w[b][m];
      const uint64_t vm = cm[b] & __builtin_amdgcn_fcmp(D, bound, FCMP_OLE);
      if (!vm) continue;
      const bool valid = (vm >> lane) & 1;
      if (!listed) {
        const int cnt = __builtin_popcountll(vm);
        if (total + cnt <= 64) {
          const int pos = total + (int)__builtin_amdgcn_mbcnt_hi(
                                      (uint32_t)(vm >> 32),
                                      __builtin_amdgcn_mbcnt_lo((uint32_t)vm, 0));
          if (valid) {
            sc.d[pos] = D;
            sc.i[pos] = qg;
          }
          total += cnt;
          continue;
        }
        // the scratch would overflow: sort it into the list in registers
        __builtin_amdgcn_wave_barrier();
        double d = lane < total ? sc.d[lane] : __builtin_huge_val();
        int c = lane < total ? sc.i[lane] : INT_MAX - 64 + lane;
        __builtin_amdgcn_wave_barrier();
        bitonic_sort64(d, c, lane);
        const bool real = lane < (total < k ? total : k);
        ed = real ? d : __builtin_huge_val();
        ei = real ? c : INT_MAX;
        listed = true;
      }
      const double kd = readlane_d(ed, k - 1);
      const int ki = __builtin_amdgcn_readlane(ei, k - 1);
      const uint64_t m = __ballot(valid && key_less(D, qg, kd, ki));
      const int mc = __builtin_popcountll(m);
      if (!FILTER && mc >= LIST_SORT_MIN && 64 - k >= LIST_SORT_MIN) {
        // many below the k-th (the first round's unbounded case; the filter
        // rounds rarely get here and keep their code small): through the
        // (now free) scratch into sorts of the list with up to 64 - k of them
        // at a time; each sort's first k lanes are the new list
        const int pos = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        __builtin_amdgcn_wave_barrier();
        if ((m >> lane) & 1) {
          sc.d[pos] = D;
          sc.i[pos] = qg;
        }
        __builtin_amdgcn_wave_barrier();
        for (int c0 = 0; c0 < mc; c0 += 64 - k) {
          const int src = lane - k + c0;
          double md = lane < k ? ed : __builtin_huge_val();
          int mi = lane < k ? ei : INT_MAX - 64 + lane;
          if (lane >= k && src < mc) {
            md = sc.d[src];
            mi = sc.i[src];
          }
          bitonic_sort64(md, mi, lane);
          const bool real = mi < INT_MAX - 64;
          ed = real ? md : __builtin_huge_val();
          ei = real ? mi : INT_MAX;
        }
        __builtin_amdgcn_wave_barrier();
      } else if (m) {
        insert_reg(m, D, qg, k, ed, ei);
      }
    }
  }
  if (listed) return __builtin_popcountll(__ballot(lane < k && ei != INT_MAX));
  __builtin_amdgcn_wave_barrier();
  double d = lane < total ? sc.d[lane] : __builtin_huge_val();
  int c = lane < total ? sc.i[lane] : INT_MAX - 64 + lane;
  __builtin_amdgcn_wave_barrier();  // read before the next recipient writes the scratch
  if (total > k) bitonic_sort64(d, c, lane);
  const bool real = lane < (total < k ? total : k);
  ed = real ? d : __builtin_huge_val();
  ei = real ? c : INT_MAX;
  return total < k ? total : k;
}

// Bitonic network over the wave's 64 keys alone (keys are non-negative or
// +inf): one merge of strides S, S / 2, ... 1, then the next block size.
template <int SIZE, int S>
__device__ __forceinline__ float sort_keys_merge64(float key, int lane) {
  const float p = __builtin_bit_cast(float, lane_xor<S>(__builtin_bit_cast(int, key), lane));
  const bool keep_min = ((lane & S) == 0) == ((lane & SIZE) == 0);
  key = keep_min ? __builtin_fminf(key, p) : __builtin_fmaxf(key, p);
  if constexpr (S > 1) return sort_keys_merge64<SIZE, S / 2>(key, lane);
  return key;
}
template <int SIZE = 2>
__device__ __forceinline__ float sort_keys64(float key, int lane) {
  key = sort_keys_merge64<SIZE, SIZE / 2>(key, lane);
  if constexpr (SIZE < 64) return sort_keys64<SIZE * 2>(key, lane);
  return key;
}

// The k-th smallest of the wave's 64 keys.
__device__ __forceinline__ float kth_smallest64(float key, int lane, int k) {
  key = sort_keys64(key, lane);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, key), k - 1));
}

// First round (no bound yet): recipient s's exact k nearest in the tile,
// possibly unsorted. Each lane takes the smallest FP32 window sum over its
// candidates; the k-th smallest of these 64 minima, tau, belongs to k
// distinct candidates, whose FP64 sums are at most tau (1 + 2^-19) (the FP32
// sums err by less than 2^-20, the FP64 ones by far less). That value bounds
// the tile's k-th distance, so the candidates within it -- at least k -- hold
// the k nearest. They are compacted into the wave's scratch and, if there are
// more than k, sorted. Fewer than k lanes with a candidate, or more than 64
// candidates within the bound, fall back to recipient_topk with no bound.
template <int L, int NB>
__device__ __forceinline__ int recipient_establish(const float* V, int sp, int sq, int Q, int s,
                                                   int pg, int q0, int sign, int np, int k,
                                                   int lane, const EstScratch& sc, double& ed,
                                                   int& ei) {
  // batches in flight together: at most 12 staged values per lane, so that
  // the first round's kernels keep their accumulators in registers
  constexpr int NG = NB * L <= 12 ? NB : (NB % 2 == 0 && NB * L <= 24 ? NB / 2 : 1);
  const int step = sp + sq;
  const float* vrow = V + s * sp;
  auto load = [&](int b0, float (&w)[NG][L]) __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      const int q = 64 * (b0 + b) + lane;
      const float* v = vrow + (q < Q ? q : 0) * sq;  // idle lanes: a valid address
#pragma unroll
      for (int m = 0; m < L; ++m) w[b][m] = v[m * step];
    }
  };
  uint64_t rng[NB];  // the recipient's candidates, outside its exclusion zone
  batch_masks<NB>(Q, q0, np, pg, sign, L, lane, rng);
  float mn = __builtin_huge_valf();
#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += NG) {
    float w[NG][L];
    load(b0, w);
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      float s32 = w[b][0];
#pragma unroll
      for (int m = 1; m < L; ++m) s32 += w[b][m];
      if ((rng[b0 + b] >> lane) & 1) mn = __builtin_fminf(mn, s32);
    }
  }
  const float tau = kth_smallest64(mn, lane, k);
  bool fallback = tau == __builtin_huge_valf();  // fewer than k lanes hold a candidate
  const double b64 = (double)tau * (1.0 + 0x1p-19);
  const float b32 = prefilter_bound(b64);
  int total = 0;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int b0 = 0; b0 < NB && !fallback; b0 += NG) {
    float w[NG][L];
    load(b0, w);
#pragma unroll
    for (int b = 0; b < NG; ++b) {
      float s32 = w[b][0];
#pragma unroll
      for (int m = 1; m < L; ++m) s32 += w[b][m];
      const uint64_t cm = rng[b0 + b] & __builtin_amdgcn_fcmpf(s32, b32, FCMP_OLE);
      if (!cm) continue;
      double D = (double)w[b][0];
#pragma unroll
      for (int m = 1; m < L; ++m) D += (double)w[b][m];
      const uint64_t mk = cm & __builtin_amdgcn_fcmp(D, b64, FCMP_OLE);
      const bool c = (mk >> lane) & 1;
      const int pos = total + (int)__builtin_amdgcn_mbcnt_hi(
                                  (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
      if (c && pos < 64) {
        sc.d[pos] = D;
        sc.i[pos] = q0 + 64 * (b0 + b) + lane;
      }
      total += __builtin_popcountll(mk);
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (fallback || total > 64)
    return recipient_topk<L, NB, false>(V, sp, sq, Q, s, q0, rng, k, __builtin_huge_val(),
                                        __builtin_huge_valf(), lane, sc, ed, ei);
  double d = lane < total ? sc.d[lane] : __builtin_huge_val();
  int c = lane < total ? sc.i[lane] : INT_MAX - 64 + lane;
  __builtin_amdgcn_wave_barrier();  // the scratch is read before the next recipient writes it
  if (total > k) bitonic_sort64(d, c, lane);
  const bool real = lane < (total < k ? total : k);
  ed = real ? d : __builtin_huge_val();
  ei = real ? c : INT_MAX;
  return total < k ? total : k;
}

// One side of a staged part: wave w of nw keeps recipients w, w + nw, ... of
// 0 .. P - 1 and writes their slots. ESTABLISH (the first round): each
// recipient's exact k nearest in the tile (recipient_establish, using the
// wave's scratch sc). Otherwise (FILTER): its k nearest within its
// row's bound (the bounds of the wave's recipients are fetched first, one per
// lane, and read from registers). Q <= 64 NB candidates per recipient.
template <int L, int NB, bool ESTABLISH>
__device__ __forceinline__ void side_topk(const float* V, int sp, int sq, int Q, int P, int p0,
                                          int q0, int sign, int slot, int np, int wave, int nw,
                                          int lane, const double* bound, const FusedSlots& out,
                                          const EstScratch& sc) {
  if constexpr (!ESTABLISH) {
    const int pl = p0 + wave + lane * nw;  // lane u: the wave's u-th recipient
    const double mybound = (wave + lane * nw < P && pl < np) ? bound[pl] : -1.0;
    const float mybound32 = prefilter_bound(mybound);
    // the filter rounds' tiles lie past the exclusion zone: the masks hold
    // for every recipient
    uint64_t rng[NB];
    batch_masks<NB>(Q, q0, np, -1, sign, L, lane, rng);
    int u = 0;
    for (int s = wave; s < P; s += nw, ++u) {
      const int pg = p0 + s;
      if (pg >= np) continue;
      double ed;
      int ei;
      const double b = readlane_d(mybound, u);
      const float b32 = __builtin_bit_cast(
          float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mybound32), u));
      const int n = recipient_topk<L, NB, true>(V, sp, sq, Q, s, q0, rng, out.k, b, b32, lane,
                                                sc, ed, ei);
      slot_write(out, pg, slot, n, ed, ei, lane);
    }
  } else {
    for (int s = wave; s < P; s += nw) {
      const int pg = p0 + s;
      if (pg >= np) continue;
      double ed;
      int ei;
      const int n = recipient_establish<L, NB>(V, sp, sq, Q, s, pg, q0, sign, np, out.k, lane,
                                               sc, ed, ei);
      slot_write(out, pg, slot, n, ed, ei, lane);
    }
  }
}

// side_topk for the run-time length L (1 .. TRAKNN_MAX_L): each length has
// its own unrolled sums.
template <int NB, bool ESTABLISH, int LC = 1>
__device__ __forceinline__ void side_topk_len(int L, const float* V, int sp, int sq, int Q, int P,
                                              int p0, int q0, int sign, int slot, int np,
                                              int wave, int nw, int lane, const double* bound,
                                              const FusedSlots& out, const EstScratch& sc) {
  if constexpr (LC <= TRAKNN_MAX_L) {
    if (L == LC)
      side_topk<LC, NB, ESTABLISH>(V, sp, sq, Q, P, p0, q0, sign, slot, np, wave, nw, lane,
                                   bound, out, sc);
    else
      side_topk_len<NB, ESTABLISH, LC + 1>(L, V, sp, sq, Q, P, p0, q0, sign, slot, np, wave, nw,
                                           lane, bound, out, sc);
  }
}

}  // namespace traknn
