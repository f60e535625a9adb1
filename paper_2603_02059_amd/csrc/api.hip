// C ABI of the TRAKNN hot path: planning, argument validation, workspace
// layout and the launch sequence. No C++ exception crosses this boundary and
// nothing is enqueued unless every argument has been accepted.
#include <atomic>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"

using namespace traknn;

namespace {

constexpr size_t WS_ALIGN = 256;
constexpr int64_t MAX_T = 1 << 20;       // int32 indices with headroom
constexpr int64_t MAX_D = (int64_t)1 << 28;
constexpr size_t MAX_WIN_LDS = 64 * 1024;
// Window waves to aim for (row blocks x waves per block); a compile-time
// tuning knob. 12288 gives 4 waves per 8-row block at T = 27394, the best of
// the block shapes measured there.
#ifndef TRAKNN_WIN_TARGET_UNITS
#define TRAKNN_WIN_TARGET_UNITS 12288
#endif
constexpr int64_t WIN_TARGET_UNITS = TRAKNN_WIN_TARGET_UNITS;
// The same for the window launches of band mode, whose rows are shorter.
#ifndef TRAKNN_BAND_WIN_TARGET_UNITS
#define TRAKNN_BAND_WIN_TARGET_UNITS TRAKNN_WIN_TARGET_UNITS
#endif
constexpr int64_t BAND_WIN_TARGET_UNITS = TRAKNN_BAND_WIN_TARGET_UNITS;
// Band mode's column windows have rows of only row_batch candidates, so each
// wave's fixed costs (seeding its rows' lists, writing them out) weigh more:
// half the waves per block. At T = 27394 with passes of 4088 rows this gives 2
// waves per block, measured best against 1, 4 and 8.
#ifndef TRAKNN_BAND_COL_TARGET_UNITS
#define TRAKNN_BAND_COL_TARGET_UNITS 6144
#endif
constexpr int64_t BAND_COL_TARGET_UNITS = TRAKNN_BAND_COL_TARGET_UNITS;
constexpr int MAX_SPLITS = MERGE_MAX_SPLITS;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
// Row stride of a distance buffer, floats: whole 256-byte segments, an odd
// number of them, so that rows a power of two apart do not all start in the
// same HBM channel.
int64_t matrix_stride(int64_t cols) {
  const int64_t ld = round_up(cols, 64);
  return (ld / 64) % 2 ? ld : ld + 64;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int fail_hip(hipError_t e) { return e == hipSuccess ? TRAKNN_OK : TRAKNN_ERR_HIP; }

// Column splits of the window stage: one workgroup of W waves per block of
// WINDOW1_ROWS rows (the waves split the block's diagonals and share a per-row
// bound), with W as large as the LDS budget and the target parallelism allow,
// for a launch of `rows` rows (of the shortest length) over `cands` candidate
// columns. A multi-length request runs the same kernel once per length (or
// pair of lengths); L_max sizes the LDS.
int window_splits(const traknn_plan_s* p, int64_t rows, int64_t cands, int64_t target) {
  const int k = p->cfg.k;
  const int L = p->cfg.L_max;
  const int64_t nrb = (rows + WINDOW1_ROWS - 1) / WINDOW1_ROWS;
  const int64_t nchunks = (cands + WINDOW1_ROWS - 1 + 63) / 64;
  // a sweep's passes hold up to WINDOW_LENGTHS_PER_PASS lengths' lists
  const int G = p->NL > 1 ? WINDOW_LENGTHS_PER_PASS : 1;
  const size_t base = window1_lds_bytes(L, G, k, 0);
  const size_t per_wave = window1_lds_bytes(L, G, k, 1) - base;
  if (base + per_wave > MAX_WIN_LDS) return 0;
  // Every wave keeps its own k-long list per row and length of its pass, so
  // when those hold more than 10 entries (G k > 10) the target shrinks in
  // proportion. At T = 27394 this gives 4, 2 and 1 waves per block for k =
  // 10, 20 and 40 at one length, and 2 for a sweep's pairs of lengths at
  // k = 10: the fastest of the counts measured for each.
  if (G * k > 10) target = target * 10 / (G * k);
  int64_t W = (target + nrb - 1) / nrb;
  const int64_t wmax = (int64_t)((MAX_WIN_LDS - base) / per_wave);
  if (W > wmax) W = wmax;
  if (W > MAX_SPLITS) W = MAX_SPLITS;
  if (W > nchunks) W = nchunks;
  if (W < 1) W = 1;
  return (int)W;
}

// Whole matrix: one launch of all rows over all columns. Band mode: per pass,
// a row window of up to rb rows over the columns from the pass's first row on,
// and a column window of the rows from the pass's first on over the pass's
// (up to) rb trajectories.
bool plan_window(traknn_plan_s* p) {
  const int64_t rows = p->rb && p->rb < p->np0 ? p->rb : p->np0;
  const int64_t target = p->rb ? BAND_WIN_TARGET_UNITS : WIN_TARGET_UNITS;
  p->win_splits = window_splits(p, rows, p->np0, target);
  p->col_splits = p->rb ? window_splits(p, p->np0, rows, BAND_COL_TARGET_UNITS) : 0;
  return p->win_splits > 0 && (!p->rb || p->col_splits > 0);
}

// Fused mode: tile stride, block-rows and the ends of the second and third
// rounds of tile offsets (each launch then covers one round).
void plan_fused(traknn_plan_s* p) {
  const traknn_config& c = p->cfg;
  FusedGeom& g = p->fg;
  const bool f64 = c.precision == TRAKNN_FP64;
  const int tile = f64 ? FUSED_F64_TILE : GRAM_TILE;
  g.T = (int)c.T;
  g.np = (int)p->np0;
  g.L = c.L_max;
  g.k = c.k;
  g.B = tile - (c.L_max - 1);
  if (!f64) g.B = g.B / 4 * 4;  // 16-byte aligned chunk-norm loads of each panel
  g.nbt = (int)((g.np + g.B - 1) / g.B);
  g.blo = g.bhi = 0;
  // Round ends: each launch's last wave of tiles is partly idle, so the
  // second and third rounds end where the four launches need the fewest
  // waves of resident tiles, ties kept nearest the default ends. The FP64
  // tiles are half as wide, so their offsets (ranges and defaults) double to
  // reach as far in trajectories.
  const int64_t conc = (int64_t)NUM_CU * (f64 ? FUSED_F64_PER_CU : 1);
  auto tiles = [&](int lo, int hi) {
    hi = hi < g.nbt ? hi : g.nbt;
    int64_t n = 0;
    for (int h = lo; h < hi; ++h) n += g.nbt - h;
    return n;
  };
  auto waves = [&](int lo, int hi) { return (tiles(lo, hi) + conc - 1) / conc; };
  auto cost = [&](int e2, int e3) {
    return waves(0, FUSED_FIRST_END) + waves(FUSED_FIRST_END, e2) + waves(e2, e3) +
           waves(e3, g.nbt);
  };
  const int sc = f64 ? 2 : 1;
  auto dist = [&](int e2, int e3) {
    const int a = e2 - sc * FUSED_END_DEFAULT[0], b = e3 - sc * FUSED_END_DEFAULT[1];
    return 4 * (a < 0 ? -a : a) + (b < 0 ? -b : b);
  };
  g.rend[0] = sc * FUSED_END_DEFAULT[0];
  g.rend[1] = sc * FUSED_END_DEFAULT[1];
  int64_t best = cost(g.rend[0], g.rend[1]);
  for (int e2 = 6 * sc; e2 <= 12 * sc; ++e2)
    for (int e3 = e2 + 4 > 24 * sc ? e2 + 4 : 24 * sc; e3 <= 48 * sc; ++e3) {
      const int64_t cst = cost(e2, e3);
      if (cst < best || (cst == best && dist(e2, e3) < dist(g.rend[0], g.rend[1]))) {
        best = cst;
        g.rend[0] = e2;
        g.rend[1] = e3;
      }
    }
  // the MFMA tiles read a full 256-row panel from every block-row's start
  if (!f64) {
    const int64_t need = (int64_t)(g.nbt - 1) * g.B + GRAM_TILE;
    if (need > p->Tpad) p->Tpad = round_up(need, GRAM_TILE);
  }
}

// Band passes: the starts t0 of passes of at most rb rows, on multiples of 8
// (the chunk-norm loads' alignment). Each pass's Gram launch ends with a
// partly idle round of 256 tiles, so the starts minimise, by dynamic
// programming from the last row back, the passes' rounds plus lambda rounds
// per pass: a pass's own windows and merge cost about the same at any D,
// while a round of tiles grows with D, so lambda = 1 + 8192 / Dpad. A pass of
// nt rows from t0 covers nbi = ceil((nt + L_max - 1) / 256) block-rows against
// the block-columns from t0 / 256 on; for each nbi only the longest such pass
// is tried, and only the 16 largest nbi (all of them up to passes of 4096
// rows), so that planning stays linear in T.
void plan_band_passes(traknn_plan_s* p) {
  const int64_t T = p->T, np0 = p->np0, rb = p->rb;
  const int64_t Lm1 = p->cfg.L_max - 1;
  auto rounds = [&](int64_t t0, int64_t nt) {
    const int64_t srows = nt + Lm1 < T - t0 ? nt + Lm1 : T - t0;
    const int64_t nbi = (srows + GRAM_TILE - 1) / GRAM_TILE;
    const int64_t nbc = p->nb - t0 / GRAM_TILE;
    return (double)((nbi * nbc - nbi * (nbi - 1) / 2 + 255) / 256);
  };
  const double lambda = 1.0 + 8192.0 / (double)p->Dpad;
  const int64_t npos = (np0 + 7) / 8;  // state i < npos: a pass starts at 8 i; npos: the end
  auto state = [&](int64_t t) { return t >= np0 ? npos : t / 8; };
  std::vector<double> cost(npos + 1, 0.0);
  std::vector<int64_t> next(npos + 1, np0);
  for (int64_t i = npos - 1; i >= 0; --i) {
    const int64_t t0 = 8 * i, left = np0 - t0;
    double best = 0.0;
    int64_t bt1 = np0;
    bool any = false;
    const int64_t span = rb < left ? rb : left;
    const int64_t nbi_max = (span + Lm1 + GRAM_TILE - 1) / GRAM_TILE;
    for (int64_t nbi = nbi_max > 16 ? nbi_max - 15 : 1;; ++nbi) {
      int64_t nt = (nbi * GRAM_TILE - Lm1) / 8 * 8;
      bool last = false;
      if (nt >= rb) nt = rb, last = true;
      if (nt >= left) nt = left, last = true;
      if (nt > 0) {
        const int64_t t1 = t0 + nt;
        const double c = rounds(t0, nt) + lambda + cost[state(t1)];
        if (!any || c < best) best = c, bt1 = t1, any = true;
      }
      if (last) break;
    }
    cost[i] = best;
    next[i] = bt1;
  }
  p->band_t0.clear();
  for (int64_t t = 0; t < np0; t = next[state(t)]) p->band_t0.push_back(t);
}

void plan_layout(traknn_plan_s* p) {
  Layout& L = p->lay;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, WS_ALIGN);
    return at;
  };
  const int prec = p->cfg.precision;
  const size_t np = (size_t)(p->T - p->cfg.L_min + 1);
  L.bw_zero = take((2 * np + (size_t)p->T) * sizeof(int32_t));
  L.bw_ptr = take((np + 1) * sizeof(int32_t));
  L.bw_rev = take(np * p->cfg.k * sizeof(int32_t));
  L.bw_end = o;
  L.mu_part = take((size_t)p->tchunks * p->D * sizeof(double));
  L.mu = take((size_t)p->D * sizeof(double));
  if (p->fused) {
    // S-free: the centred operands of the MFMA tiles (none for the FP64 tiles,
    // which read the fields) and the per-row candidate buffers
    const bool mfma = prec != TRAKNN_FP64;
    L.ncs = take(mfma ? (size_t)norm_chunks(p->Dpad) * p->Tpad * sizeof(float) : 0);
    L.xc = take(mfma ? (size_t)p->Tpad * p->Dpad * elem_bytes(prec) : 0);
    const size_t nslot = (size_t)p->fg.nbt + 1;
    L.f_bound = take(np * sizeof(double));
    L.f_cnt = take(np * nslot * sizeof(int32_t));
    L.f_sd = take(np * nslot * p->cfg.k * sizeof(double));
    L.f_si = take(np * nslot * p->cfg.k * sizeof(int32_t));
    L.f_rd = take(np * p->cfg.k * sizeof(double));
    L.f_ri = take(np * p->cfg.k * sizeof(int32_t));
    L.S = L.ST = L.part_d = L.part_i = L.cpart_d = L.cpart_i = o;
    L.total = o;
    return;
  }
  L.ncs = take((size_t)norm_chunks(p->Dpad) * p->Tpad * sizeof(float));
  L.xc = take((size_t)p->Tpad * p->Dpad * elem_bytes(prec));
  L.S = take((size_t)(p->rb ? p->band_rows : p->T) * p->ldS * sizeof(float));
  // band mode: the transposed band, one row per field
  L.ST = take(p->rb ? (size_t)p->T * p->ldST * sizeof(float) : 0);
  // partial lists: of the whole-matrix launch or a pass's row window (rb rows);
  // band mode adds those of its first column window (every row)
  const int64_t prows = p->rb && p->rb < p->np0 ? p->rb : p->np0;
  const size_t nparts = (size_t)p->win_splits * p->NL * prows * p->cfg.k;
  L.part_d = take(nparts * sizeof(double));
  L.part_i = take(nparts * sizeof(int32_t));
  const size_t ncol = p->rb ? (size_t)p->col_splits * p->NL * p->np0 * p->cfg.k : 0;
  L.cpart_d = take(ncol * sizeof(double));
  L.cpart_i = take(ncol * sizeof(int32_t));
  L.total = o;
}

int check_x(const traknn_plan_s* p, const float* X, int64_t ldx) {
  if (!X || ldx < p->D || ldx % 4 != 0 || !aligned(X, 16))
    return TRAKNN_ERR_INVALID_ARG;
  return TRAKNN_OK;
}

int check_ws(const void* ws, size_t bytes, size_t need) {
  if (!ws || !aligned(ws, WS_ALIGN) || bytes < need) return TRAKNN_ERR_WORKSPACE;
  return TRAKNN_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return (T*)((char*)ws + off);
}

int record(traknn_plan_s* p, int slot, hipStream_t s) {
  if (!p->timing) return TRAKNN_OK;
  return fail_hip(hipEventRecord(p->ev[slot], s));
}

}  // namespace

namespace {

// Fused mode after the centring: the rounds of tile offsets, the first
// keeping each recipient's exact k nearest per tile, each later one only the
// candidates within the rows' bounds; after every round but the last a
// refresh merges its slots into the rows' running lists and sets their
// bounds, and the final merge writes the lists. Every slot is written by its
// tile on every call before it is read, so nothing needs clearing. Timing
// slots: 3 after the rounds (their refreshes included), 4 after the final
// merge (stage 4 of the matrix mode, the merge, is empty).
int enqueue_fused(traknn_plan_s* plan, const float* X, int64_t ldx, void* workspace,
                  int32_t* nbr_idx, double* nbr_dist, hipStream_t s) {
  const traknn_config& c = plan->cfg;
  const Layout& L = plan->lay;
  FusedGeom g = plan->fg;
  const double* mu = at<double>(workspace, L.mu);
  double* bound = at<double>(workspace, L.f_bound);
  double* run_d = at<double>(workspace, L.f_rd);
  int32_t* run_i = at<int32_t>(workspace, L.f_ri);
  const FusedSlots out{at<int32_t>(workspace, L.f_cnt), at<double>(workspace, L.f_sd),
                       at<int32_t>(workspace, L.f_si), g.nbt + 1, c.k};
  const int D = (int)plan->D;
  int rc;
  int lo = 0;
  for (int r = 0; r < FUSED_ROUNDS && lo < g.nbt; ++r) {
    int hi = r == 0 ? FUSED_FIRST_END : r + 1 < FUSED_ROUNDS ? g.rend[r - 1] : g.nbt;
    if (hi > g.nbt) hi = g.nbt;
    g.blo = lo;
    g.bhi = hi;
    const bool establish = r == 0;
    if (c.precision == TRAKNN_FP64) {
      if ((rc = fail_hip(launch_fused_f64(X, ldx, D, mu, g, establish, bound, out, s))))
        return rc;
    } else {
      const void* xc = at<char>(workspace, L.xc);
      const float* ncs = at<float>(workspace, L.ncs);
      if ((rc = fail_hip(launch_gram_fused(xc, ncs, plan->T, plan->Tpad, plan->Dpad,
                                           c.precision, g, establish, bound, out, s))))
        return rc;
    }
    if (hi < g.nbt &&
        (rc = fail_hip(launch_slots_refresh(g, out, bound, run_d, run_i, lo, hi, s))))
      return rc;
    if (hi < g.nbt) lo = hi;
    else break;
  }
  if ((rc = record(plan, 3, s))) return rc;
  if ((rc = fail_hip(launch_slots_final(g, out, run_d, run_i, lo, nbr_idx, nbr_dist, s))))
    return rc;
  if ((rc = record(plan, 4, s))) return rc;
  if ((rc = record(plan, 5, s))) return rc;
  if (plan->timing) plan->timed_calls++;
  return TRAKNN_OK;
}

// The launch sequence of traknn_knn on validated arguments: workspace is at
// least plan->lay.total bytes, 256-byte aligned. Nothing it reads from the
// workspace is read before this call has written it, so the workspace needs
// no clearing between calls.
int enqueue_knn(traknn_plan_s* plan, const float* X, int64_t ldx, void* workspace,
                int32_t* nbr_idx, double* nbr_dist, hipStream_t s) {
  int rc;
  const traknn_config& c = plan->cfg;
  const Layout& L = plan->lay;
  double* mu_part = at<double>(workspace, L.mu_part);
  double* mu = at<double>(workspace, L.mu);
  float* ncs = at<float>(workspace, L.ncs);
  void* xc = at<char>(workspace, L.xc);
  float* S = at<float>(workspace, L.S);
  double* part_d = at<double>(workspace, L.part_d);
  int32_t* part_i = at<int32_t>(workspace, L.part_i);

  if ((rc = record(plan, 0, s))) return rc;
  if ((rc = fail_hip(launch_colstats(X, ldx, plan->T, plan->D, plan->tchunks,
                                     mu_part, mu, s))))
    return rc;
  if ((rc = record(plan, 1, s))) return rc;
  if (c.precision != TRAKNN_FP64 &&
      (rc = fail_hip(launch_centre_convert(X, ldx, plan->T, plan->D, plan->Tpad,
                                           plan->Dpad, c.precision, mu, xc,
                                           ncs, s))))
    return rc;
  if ((rc = record(plan, 2, s))) return rc;
  if (plan->fused) return enqueue_fused(plan, X, ldx, workspace, nbr_idx, nbr_dist, s);
  if (plan->rb) {
    // Band mode (row-batched streaming). Pass p owns the trajectories t0 ..
    // t1 - 1; its band is the rows of S they reach, against the columns from
    // t0 on (rounded down to a block-column), stored as rows and transposed.
    // Only entries above the diagonal are computed and read:
    // - Row window: the pass's rows over the later candidates (t0 .. n' - 1,
    //   j > i), read from the band.
    // - Column window: the rows t0 .. n' - 1 over the pass's earlier
    //   candidates (t0 .. t1 - 1, j < i), read from the transposed band (S is
    //   symmetric).
    // One merge folds both into the rows' running lists; after pass p the rows
    // t0 .. t1 - 1 are final. So every ordered pair of trajectories is a candidate
    // exactly once, and the passes together contract about half the matrix.
    float* ST = at<float>(workspace, L.ST);
    double* cpart_d = at<double>(workspace, L.cpart_d);
    int32_t* cpart_i = at<int32_t>(workspace, L.cpart_i);
    const int64_t T = plan->T, np0 = plan->np0;
    const size_t npass = plan->band_t0.size();
    for (size_t pi = 0; pi < npass; ++pi) {
      const int64_t t0 = plan->band_t0[pi];
      const int64_t t1 = pi + 1 < npass ? plan->band_t0[pi + 1] : np0;
      const int64_t nt = t1 - t0;
      const int64_t srows = nt + c.L_max - 1 < T - t0 ? nt + c.L_max - 1 : T - t0;
      const int nbi = (int)((srows + GRAM_TILE - 1) / GRAM_TILE);
      const int J0 = (int)(t0 / GRAM_TILE);
      const int64_t c0 = (int64_t)J0 * GRAM_TILE;
      const int64_t nbc = plan->nb - J0;  // block-columns from J0 on
      const int64_t ntiles = nbi * nbc - (int64_t)nbi * (nbi - 1) / 2;
      if ((rc = fail_hip(launch_gram_band(xc, ncs, T, plan->Tpad, plan->Dpad, plan->nb, ntiles,
                                          c.precision, t0, nbi, srows, J0, S, plan->ldS, ST,
                                          plan->ldST, s))))
        return rc;
      const WindowRange rows{t0, t0 + srows, c0, t0, T, T, 1, T};
      if ((rc = fail_hip(launch_window_band(S, plan->ldS, T, c.L_min, c.L_max, c.k,
                                            plan->win_splits, rows, t0, nt, part_d, part_i,
                                            s))))
        return rc;
      const WindowRange cols{c0, T, t0, t0, t1, t0 + srows, -T, -1};
      if ((rc = fail_hip(launch_window_band(ST, plan->ldST, T, c.L_min, c.L_max, c.k,
                                            plan->col_splits, cols, t0, np0 - t0, cpart_d,
                                            cpart_i, s))))
        return rc;
      // every row from t0 on holds the earlier passes' lists (none in pass 0)
      const MergeSet mr{part_d, part_i, plan->win_splits, (int)nt};
      const MergeSet mc{cpart_d, cpart_i, plan->col_splits, (int)(np0 - t0)};
      if ((rc = fail_hip(launch_merge_band(mr, mc, T, c.L_min, c.L_max, c.k, t0, np0 - t0,
                                           t0 > 0 ? np0 : 0, nbr_idx, nbr_dist, s))))
        return rc;
    }
    // the passes interleave the stages: the Gram slot times them all
    if ((rc = record(plan, 3, s))) return rc;
    if ((rc = record(plan, 4, s))) return rc;
    if ((rc = record(plan, 5, s))) return rc;
    if (plan->timing) plan->timed_calls++;
    return TRAKNN_OK;
  }
  if ((rc = fail_hip(launch_gram(xc, ncs, plan->T, plan->Tpad, plan->Dpad, plan->nb,
                                 plan->ntiles, c.precision, S, plan->ldS, s))))
    return rc;
  if ((rc = record(plan, 3, s))) return rc;
  if ((rc = fail_hip(launch_window_topk(S, plan->ldS, plan->T, c.L_min, c.L_max,
                                        c.k, plan->win_splits, part_d,
                                        part_i, s))))
    return rc;
  if ((rc = record(plan, 4, s))) return rc;
  if ((rc = fail_hip(launch_merge(part_d, part_i, plan->T, c.L_min, c.L_max, c.k,
                                  plan->win_splits, nbr_idx, nbr_dist, s))))
    return rc;
  if ((rc = record(plan, 5, s))) return rc;
  if (plan->timing) plan->timed_calls++;
  return TRAKNN_OK;
}

// Fixed device scratch of traknn_knn_noalloc, for callers that cannot
// allocate. Each device that runs the entry point holds one copy until the
// process ends; its address is looked up once per device with that device
// current (hipGetSymbolAddress), and only that address is ever used: the
// array's name in host code does not denote device memory.
static __device__ __align__(256) char scratch[TRAKNN_NOALLOC_MAX_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::atomic<void*> scratch_ptr[SCRATCH_MAX_DEVICES];
std::mutex scratch_mutex;

int device_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TRAKNN_ERR_HIP;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return TRAKNN_ERR_UNSUPPORTED;
  void* p = scratch_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(scratch_mutex);
    p = scratch_ptr[dev].load(std::memory_order_relaxed);
    if (!p) {
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
        return TRAKNN_ERR_HIP;
      scratch_ptr[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return TRAKNN_OK;
}

}  // namespace

extern "C" {

const char* traknn_status_string(int status) {
  switch (status) {
    case TRAKNN_OK:
      return "ok";
    case TRAKNN_ERR_INVALID_ARG:
      return "invalid argument";
    case TRAKNN_ERR_UNSUPPORTED:
      return "unsupported configuration";
    case TRAKNN_ERR_WORKSPACE:
      return "workspace missing, misaligned or too small";
    case TRAKNN_ERR_HIP:
      return "HIP runtime or kernel launch failure";
    case TRAKNN_ERR_SCRATCH_LIMIT:
      return "workspace of this plan exceeds the fixed scratch of traknn_knn_noalloc "
             "(TRAKNN_NOALLOC_MAX_BYTES)";
    default:
      return "unknown status";
  }
}

int traknn_plan(const traknn_config* cfg, traknn_plan_t* out,
                size_t* workspace_bytes) {
  if (!cfg || !out || !workspace_bytes) return TRAKNN_ERR_INVALID_ARG;
  *out = nullptr;
  const traknn_config c = *cfg;
  if (c.T < 1 || c.T > MAX_T || c.D < 1 || c.D > MAX_D)
    return TRAKNN_ERR_INVALID_ARG;
  if (c.L_min < 1 || c.L_max < c.L_min || c.L_max > TRAKNN_MAX_L)
    return TRAKNN_ERR_INVALID_ARG;
  if (c.k < 1 || c.k > TRAKNN_MAX_K) return TRAKNN_ERR_INVALID_ARG;
  if (c.precision != TRAKNN_FP32 && c.precision != TRAKNN_BF16X3 &&
      c.precision != TRAKNN_FP16 && c.precision != TRAKNN_FP64)
    return TRAKNN_ERR_INVALID_ARG;
  if ((c.mode != TRAKNN_MODE_MATRIX && c.mode != TRAKNN_MODE_FUSED) || c.reserved != 0)
    return TRAKNN_ERR_INVALID_ARG;
  const bool fused = c.mode == TRAKNN_MODE_FUSED;
  // fused mode: one length, no bands; FP64 only there
  if (fused && c.row_batch != 0) return TRAKNN_ERR_INVALID_ARG;
  if (fused && c.L_min != c.L_max) return TRAKNN_ERR_UNSUPPORTED;
  if (!fused && c.precision == TRAKNN_FP64) return TRAKNN_ERR_UNSUPPORTED;
  // every row of every length needs k candidates outside its exclusion zone
  if (c.T - c.L_max + 1 < (int64_t)c.k + 2 * c.L_max - 1)
    return TRAKNN_ERR_INVALID_ARG;
  // band mode: passes start on multiples of 8 rows (16-byte aligned norm loads)
  if (c.row_batch < 0 || c.row_batch % 8 != 0) return TRAKNN_ERR_INVALID_ARG;
  if (c.L_min != c.L_max && c.L_min != 1) return TRAKNN_ERR_UNSUPPORTED;
  // the Gram stage addresses a 256-field operand panel with 32-bit offsets
  if ((uint64_t)round_up(c.D, stage_k(c.precision)) * elem_bytes(c.precision) * GRAM_TILE >
      0x7FFFFFFFull)
    return TRAKNN_ERR_UNSUPPORTED;

  traknn_plan_s* p = new (std::nothrow) traknn_plan_s();
  if (!p) return TRAKNN_ERR_INVALID_ARG;
  p->cfg = c;
  p->T = c.T;
  p->D = c.D;
  p->Dpad = round_up(c.D, stage_k(c.precision));
  p->rb = c.row_batch;
  // a band's last block-row may reach one tile past the last field
  p->Tpad = round_up(c.T, GRAM_TILE) + (p->rb ? GRAM_TILE : 0);
  p->ldS = matrix_stride(c.T);
  p->np0 = c.T - c.L_min + 1;
  p->NL = c.L_max - c.L_min + 1;
  p->nb = (int)((c.T + GRAM_TILE - 1) / GRAM_TILE);
  p->ntiles = (int64_t)p->nb * (p->nb + 1) / 2;
  p->band_rows = p->rb + c.L_max - 1 < c.T ? p->rb + c.L_max - 1 : c.T;
  p->ldST = p->rb ? matrix_stride(p->band_rows) : 0;
  p->tchunks = colstat_chunks(c.T);
  p->fused = fused ? 1 : 0;
  if (fused) {
    plan_fused(p);
  } else if (!plan_window(p)) {
    delete p;
    return TRAKNN_ERR_UNSUPPORTED;
  }
  if (p->rb) {
    try {
      plan_band_passes(p);
    } catch (...) {  // no exception crosses the C ABI
      delete p;
      return TRAKNN_ERR_INVALID_ARG;
    }
  }
  plan_layout(p);
  *out = p;
  *workspace_bytes = p->lay.total;
  return TRAKNN_OK;
}

int traknn_plan_destroy(traknn_plan_t plan) {
  if (!plan) return TRAKNN_ERR_INVALID_ARG;
  if (plan->events_ready)
    for (int i = 0; i <= NUM_STAGES; ++i) (void)hipEventDestroy(plan->ev[i]);
  delete plan;
  return TRAKNN_OK;
}

int traknn_set_timing(traknn_plan_t plan, int enable) {
  if (!plan) return TRAKNN_ERR_INVALID_ARG;
  if (enable && !plan->events_ready) {
    for (int i = 0; i <= NUM_STAGES; ++i) {
      if (hipEventCreate(&plan->ev[i]) != hipSuccess) {
        for (int q = 0; q < i; ++q) (void)hipEventDestroy(plan->ev[q]);
        return TRAKNN_ERR_HIP;
      }
    }
    plan->events_ready = 1;
  }
  plan->timing = enable ? 1 : 0;
  plan->timed_calls = 0;
  return TRAKNN_OK;
}

int traknn_stage_times(traknn_plan_t plan, double* ms, int max_stages,
                       int* n_stages) {
  if (!plan || !ms || !n_stages || max_stages < 1) return TRAKNN_ERR_INVALID_ARG;
  if (!plan->events_ready || plan->timed_calls == 0) return TRAKNN_ERR_UNSUPPORTED;
  if (hipEventSynchronize(plan->ev[NUM_STAGES]) != hipSuccess) return TRAKNN_ERR_HIP;
  const int n = max_stages < NUM_STAGES ? max_stages : NUM_STAGES;
  for (int i = 0; i < n; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, plan->ev[i], plan->ev[i + 1]) != hipSuccess)
      return TRAKNN_ERR_HIP;
    ms[i] = (double)t;
  }
  *n_stages = n;
  return TRAKNN_OK;
}

int traknn_knn(traknn_plan_t plan, const float* X, int64_t ldx, void* workspace,
               size_t workspace_bytes, int32_t* nbr_idx, double* nbr_dist,
               void* stream) {
  if (!plan || !nbr_idx || !nbr_dist) return TRAKNN_ERR_INVALID_ARG;
  int rc = check_x(plan, X, ldx);
  if (rc) return rc;
  rc = check_ws(workspace, workspace_bytes, plan->lay.total);
  if (rc) return rc;
  return enqueue_knn(plan, X, ldx, workspace, nbr_idx, nbr_dist, (hipStream_t)stream);
}

int traknn_knn_noalloc(traknn_plan_t plan, const float* X, int64_t ldx, int32_t* nbr_idx,
                       double* nbr_dist, void* stream) {
  if (!plan || !nbr_idx || !nbr_dist) return TRAKNN_ERR_INVALID_ARG;
  int rc = check_x(plan, X, ldx);
  if (rc) return rc;
  if (plan->lay.total > (size_t)TRAKNN_NOALLOC_MAX_BYTES) return TRAKNN_ERR_SCRATCH_LIMIT;
  void* ws = nullptr;
  if ((rc = device_scratch(&ws))) return rc;
  return enqueue_knn(plan, X, ldx, ws, nbr_idx, nbr_dist, (hipStream_t)stream);
}

int traknn_score(traknn_plan_t plan, const double* nbr_dist, double* scores,
                 void* stream) {
  if (!plan || !nbr_dist || !scores) return TRAKNN_ERR_INVALID_ARG;
  const traknn_config& c = plan->cfg;
  return fail_hip(launch_score(nbr_dist, plan->T, c.L_min, c.L_max, c.k, scores,
                               (hipStream_t)stream));
}

int traknn_score_prefix(traknn_plan_t plan, const double* nbr_dist, double* scores,
                        void* stream) {
  if (!plan || !nbr_dist || !scores) return TRAKNN_ERR_INVALID_ARG;
  const traknn_config& c = plan->cfg;
  return fail_hip(launch_score_prefix(nbr_dist, plan->T, c.L_min, c.L_max, c.k, scores,
                                      (hipStream_t)stream));
}

int traknn_local_dim(traknn_plan_t plan, const double* nbr_dist, double* out, void* stream) {
  if (!plan || !nbr_dist || !out) return TRAKNN_ERR_INVALID_ARG;
  const traknn_config& c = plan->cfg;
  return fail_hip(launch_local_dim(nbr_dist, plan->T, c.L_min, c.L_max, c.k, out,
                                   (hipStream_t)stream));
}

int traknn_score_backward(traknn_plan_t plan, const float* X, int64_t ldx,
                          const int32_t* nbr_idx, const double* grad_scores,
                          float* grad_X, int64_t ldg, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (!plan || !nbr_idx || !grad_scores || !grad_X) return TRAKNN_ERR_INVALID_ARG;
  int rc = check_x(plan, X, ldx);
  if (rc) return rc;
  if (ldg < plan->D) return TRAKNN_ERR_INVALID_ARG;
  rc = check_ws(workspace, workspace_bytes, plan->lay.bw_end);
  if (rc) return rc;
  const traknn_config& c = plan->cfg;
  if (c.L_min != c.L_max) return TRAKNN_ERR_UNSUPPORTED;
  const Layout& L = plan->lay;
  return fail_hip(launch_backward(
      X, ldx, plan->T, plan->D, c.L_max, c.k, nbr_idx, grad_scores, grad_X, ldg,
      at<int32_t>(workspace, L.bw_zero), at<int32_t>(workspace, L.bw_ptr),
      at<int32_t>(workspace, L.bw_rev), (hipStream_t)stream));
}

int traknn_backward_workspace(traknn_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return TRAKNN_ERR_INVALID_ARG;
  *bytes = plan->lay.bw_end;
  return TRAKNN_OK;
}

int traknn_band_passes(traknn_plan_t plan, int64_t* starts, int64_t cap, int64_t* count) {
  if (!plan || !count || cap < 0 || (cap > 0 && !starts)) return TRAKNN_ERR_INVALID_ARG;
  const int64_t n = (int64_t)plan->band_t0.size();
  for (int64_t i = 0; i < n && i < cap; ++i) starts[i] = plan->band_t0[i];
  *count = n;
  return TRAKNN_OK;
}

}  // extern "C"
