// The tile walk of the fused (S-free) path: trajectory distances and the
// row/column top-k filter on a tile of snapshot distances held in LDS, so the
// T x T matrix never goes to HBM (paper, Algorithm 1 stages 2-3 applied per
// tile of stage 1; Eq. 5 along the tile's diagonals; the exclusion zone and
// Eq. 3's k nearest).
//
// A tile pairs trajectory rows i = i0 + a with trajectory columns j = j0 + b,
// a, b < B, and holds the snapshot distances d(i0 + a', j0 + b') for a', b' <
// B + L - 1 (the tiles of a launch overlap by L - 1 fields, so every
// trajectory pair of the tile has all L terms of Eq. 2 inside it). Each
// unordered pair i < j is owned by exactly one tile (i's block-row, j's
// block-column, upper triangle of tiles) and is a candidate twice: for row i
// (candidate j) in the tile's ROW walk and for row j (candidate i) in its
// COLUMN walk. The column walk is the row walk of the transposed tile, so
// one routine serves both: the recipient axis p and the candidate axis q of
// the staged values are addressed as V[p * sp + q * sq].
//
// Lanes follow wrapped diagonals: lane l of the walk meets candidate
// q = (s + l) mod Q at step s, so at every step all lanes hold candidates of
// the same recipient p = s (one ballot per recipient and wave) and every
// lane slides its window down one diagonal, D <- D - d_old + d_new (Eq. 5),
// restarting it with a direct L-term sum where it wraps to q = 0. For FP32
// snapshot distances whose exponents span less than about 29 bits the FP64
// sums are exact, so D_L does not depend on where a window was started.
//
// Two modes:
//  * ESTABLISH (a first launch over a subset of tiles that gives every row a
//    few hundred candidates, tile_establish): each recipient's k nearest in
//    the tile are appended; a bound kernel then takes each row's k-th
//    smallest over everything appended, an upper bound of its true k-th
//    distance;
//  * FILTER (every other tile): a candidate is appended only if it is within
//    its recipient's bound. A true neighbour is never above the bound, so the
//    appended candidates always contain the k nearest, and a select kernel
//    takes them in (distance, index) order.
// Appends go to per-row buffers of `cap` entries through an atomic counter;
// the counter keeps counting past cap, which marks the row for the exact
// recomputation of the fallback kernel.
#pragma once

#include "internal.h"
#include "topk_wave.h"

namespace traknn {

// Tile (I, J) = (e, e + h) of establishing tile e: the tiles of each offset
// h of the geometry, I = 0 .. nbt - h - 1, offset after offset.
__device__ __forceinline__ bool fused_establish_tile(int64_t e, const FusedGeom& g, int& I,
                                                     int& J) {
  for (int u = 0; u < g.nh; ++u) {
    const int64_t cnt = g.nbt - g.h[u];
    if (e < cnt) {
      I = (int)e;
      J = (int)e + g.h[u];
      return true;
    }
    e -= cnt;
  }
  return false;
}

// Append the masked lanes' (D, qg) to recipient pg's buffer, one atomic per
// wave. pg is the same on every lane.
__device__ __forceinline__ void fused_append(uint64_t mask, bool mine, double D, int qg,
                                             int pg, int lane, const FusedOut& out) {
  const int n = __builtin_popcountll(mask);
  const int first = __builtin_ctzll(mask);
  int base = 0;
  if (lane == first) base = atomicAdd(out.cnt + pg, n);
  base = __builtin_amdgcn_readlane(base, first);
  if (mine) {
    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
    const int pos = base + rank;
    if (pos < out.cap) {
      out.bd[(int64_t)pg * out.cap + pos] = D;
      out.bi[(int64_t)pg * out.cap + pos] = qg;
    }
  }
}

// FILTER mode: walk recipients p_beg .. p_end - 1 of a staged tile with Q
// candidates, appending every candidate within its recipient's bound.
//   V, sp, sq  staged snapshot distances: value(p', q') = V[p' * sp + q' * sq]
//              for p' < p_end + L - 1 and q' < Q + L - 1;
//   l          this lane's index within the walk group (lanes l >= Q idle);
//   p0, q0     trajectory index of p = 0 and q = 0;
//   sign       +1: pair (p, q) is the pair (i, j) = (p0 + p, q0 + q) and
//              counts when j - i >= L; -1: (i, j) = (q0 + q, p0 + p), same rule;
//   np         trajectories of the series (indices >= np do not exist);
//   rbound     recipient bounds indexed by p (LDS or global memory).
__device__ __forceinline__ void tile_walk(const float* V, int sp, int sq, int Q, int p_beg,
                                          int p_end, int p0, int q0, int sign, int L, int np,
                                          int k, const double* rbound, int l, int lane,
                                          const FusedOut& out) {
  if (p_beg >= p_end) return;
  const bool act = l < Q;
  int q = act ? (p_beg + l) % Q : 0;
  const int step = sp + sq;  // one step down a diagonal
  double D = 0.0;
  {
    const float* v = V + p_beg * sp + q * sq;
    for (int m = 0; m < L; ++m) D += (double)v[m * step];
  }
  for (int s = p_beg; s < p_end; ++s) {
    if (s > p_beg) {
      ++q;
      if (q == Q) {  // this lane's diagonal wraps to column 0: restart it
        q = 0;
        D = 0.0;
        const float* v = V + s * sp;
        for (int m = 0; m < L; ++m) D += (double)v[m * step];
      } else {
        const float* v = V + (s - 1) * sp + (q - 1) * sq;
        D = (D - (double)v[0]) + (double)v[L * step];
      }
    }
    const int pg = p0 + s, qg = q0 + q;
    const bool valid = act & (pg < np) & (qg < np) & (sign * (qg - pg) >= L);
    const bool pass = valid && D <= rbound[s];
    const uint64_t m = __ballot(pass);
    if (m) fused_append(m, pass, D, qg, pg, lane, out);
  }
}

// ESTABLISH mode: the exact k nearest of each recipient among the tile's
// candidates. A wave owns whole recipients (p_beg + wave, + nwaves, ...): it
// takes the recipient's candidates 64 at a time, forming each D_L as a direct
// L-term sum (Eq. 2), seeds a lane-resident list with a sort of the first 64
// and ballot-filters the rest against the list's k-th, then appends the list.
// The union of these per-tile lists contains the k nearest over all the tiles
// a row meets in this launch, so their k-th is an upper bound of the row's
// true k-th distance.
__device__ __forceinline__ void tile_establish(const float* V, int sp, int sq, int Q, int p_beg,
                                               int p_end, int p0, int q0, int sign, int L,
                                               int np, int k, int wave, int nwaves, int lane,
                                               const FusedOut& out) {
  const int step = sp + sq;
  for (int s = p_beg + wave; s < p_end; s += nwaves) {
    const int pg = p0 + s;
    if (pg >= np) continue;
    double ed = __builtin_huge_val();
    int ei = INT_MAX;
    for (int c0 = 0; c0 < Q; c0 += 64) {
      const int q = c0 + lane;
      const int qg = q0 + q;
      const bool valid = (q < Q) & (qg < np) & (sign * (qg - pg) >= L);
      double D = 0.0;
      if (q < Q) {
        const float* v = V + s * sp + q * sq;
        for (int m = 0; m < L; ++m) D += (double)v[m * step];
      }
      if (c0 == 0) {
        double d = valid ? D : __builtin_huge_val();
        int c = valid ? qg : INT_MAX - 64 + lane;
        bitonic_sort64(d, c, lane);
        const bool real = c < INT_MAX - 64;  // sorted entry is a candidate
        ed = real ? d : __builtin_huge_val();
        ei = real ? c : INT_MAX;
      } else {
        const double kd = readlane_d(ed, k - 1);
        const int ki = __builtin_amdgcn_readlane(ei, k - 1);
        const bool pass = valid && key_less(D, qg, kd, ki);
        const uint64_t m = __ballot(pass);
        if (m) insert_reg(m, D, qg, k, ed, ei);
      }
    }
    const bool mine = lane < k && ei != INT_MAX;
    const uint64_t keep = __ballot(mine);
    if (keep) fused_append(keep, mine, ed, ei, pg, lane, out);
  }
}

}  // namespace traknn
