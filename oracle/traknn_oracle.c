/*
 * TRAKNN FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * call this code. It shares nothing with the HIP path: it computes the plain
 * definitions of the paper, slowly and in double precision, with every sum
 * taken in a fixed, written-out order and no reassociation (build without
 * -ffast-math and with -ffp-contract=off).
 *
 * Definitions followed (paper, Section 3.2 "Problem Definition"):
 *   trajectory of duration L starting at t:   (X_t, ..., X_{t+L-1})        (Eq. 1)
 *   squared trajectory distance:
 *       D_L(i,j) = sum_{m<L} || X_{i+m} - X_{j+m} ||_F^2                   (Eq. 2)
 *   exclusion zone: j is a candidate neighbour of t iff |t - j| > e; this
 *       library takes e = L - 1 (non-overlapping trajectories), i.e.
 *       |t - j| >= L;
 *   rarity score: s_t = (1/k) * sum over the k nearest candidates of D_L   (Eq. 3)
 *
 * Readings where the paper is silent (stated once here, used throughout):
 *   - indices are 0-based; t ranges over [0, n'), n' = T - L + 1, and every t,
 *     including the first, gets a score;
 *   - distances stay squared (no square root anywhere);
 *   - ties in distance are broken by the smaller neighbour index, i.e. the
 *     neighbours are the first k candidates in ascending (D_L, j) order;
 *   - the neighbour list is returned in that order and the score sums it in
 *     that order.
 *
 * Snapshot distances are direct differences (x_ip - x_jp)^2, NOT the Gram
 * identity of Eq. 4, and trajectory distances are direct sums over m, NOT the
 * recurrence of Eq. 5: the oracle is the definition the fast method must
 * reproduce.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

/* ||X_a - X_b||_F^2 summed over cells p = 0..D-1 in increasing order. */
static double snap_dist(const double* X, int64_t D, int64_t a, int64_t b) {
  const double* xa = X + a * D;
  const double* xb = X + b * D;
  double s = 0.0;
  for (int64_t p = 0; p < D; ++p) {
    double d = xa[p] - xb[p];
    s += d * d;
  }
  return s;
}

/* Eq. 2: sum over m = 0..L-1 (increasing) of the snapshot distances. */
static double traj_dist(const double* X, int64_t D, int L, int64_t i,
                        int64_t j) {
  double s = 0.0;
  for (int m = 0; m < L; ++m) s += snap_dist(X, D, i + m, j + m);
  return s;
}

/* Full snapshot distance matrix S[i*T + j] (T x T), computed for i <= j and
 * mirrored, so S is exactly symmetric with a zero diagonal. */
int oracle_snapshot_dist(const double* X, int64_t T, int64_t D, double* S) {
  if (!X || !S || T < 1 || D < 1) return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < T; ++i) {
    for (int64_t j = i; j < T; ++j) {
      double v = snap_dist(X, D, i, j);
      S[i * T + j] = v;
      S[j * T + i] = v;
    }
  }
  return ORACLE_OK;
}

/* Full trajectory distance matrix Dm[i*n' + j], n' = T - L + 1, as a direct
 * sum over m of an already computed snapshot matrix S (T x T). */
int oracle_traj_dist_from_snapshot(const double* S, int64_t T, int L,
                                   double* Dm) {
  if (!S || !Dm || L < 1 || L > T) return ORACLE_EINVAL;
  int64_t np_ = T - L + 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < np_; ++i) {
    for (int64_t j = 0; j < np_; ++j) {
      double s = 0.0;
      for (int m = 0; m < L; ++m) s += S[(i + m) * T + (j + m)];
      Dm[i * np_ + j] = s;
    }
  }
  return ORACLE_OK;
}

/* Rows of the trajectory distance matrix straight from X:
 * out[r*n' + j] = D_L(rows[r], j) for j in [0, n'). No S is stored, so this
 * works at any T. */
int oracle_traj_dist_rows(const double* X, int64_t T, int64_t D, int L,
                          const int64_t* rows, int64_t nrows, double* out) {
  if (!X || !rows || !out || L < 1 || L > T || D < 1) return ORACLE_EINVAL;
  int64_t np_ = T - L + 1;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= np_) return ORACLE_EINVAL;
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t t = rows[r];
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < np_; ++j) out[r * np_ + j] = traj_dist(X, D, L, t, j);
  }
  return ORACLE_OK;
}

/* Rows of every trajectory length L = 1..L_max at once, straight from X:
 *   out[((L-1)*nrows + r)*n'_1 + j] = D_L(rows[r], j)  for j in [0, T-L+1),
 * +inf for j >= T-L+1 (no such trajectory), with n'_1 = T. Each D_L is the
 * direct sum of Eq. 2 over m = 0..L-1 in increasing m, so carrying the
 * partial sum from L - 1 to L performs exactly the additions of a fresh
 * direct sum; the snapshot distances are direct differences. Every row
 * needs rows[r] + L_max <= T. */
int oracle_traj_dist_rows_multi(const double* X, int64_t T, int64_t D, int L_max,
                                const int64_t* rows, int64_t nrows, double* out) {
  if (!X || !rows || !out || L_max < 1 || L_max > T || D < 1) return ORACLE_EINVAL;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] + L_max > T) return ORACLE_EINVAL;
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t t = rows[r];
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < T; ++j) {
      double s = 0.0;
      for (int L = 1; L <= L_max; ++L) {
        double* o = out + ((int64_t)(L - 1) * nrows + r) * T + j;
        if (j + L > T) {
          *o = INFINITY;
          continue;
        }
        s += snap_dist(X, D, t + L - 1, j + L - 1);
        *o = s;
      }
    }
  }
  return ORACLE_OK;
}

/* Distances of explicit trajectory pairs (ti[q], tj[q]). */
int oracle_pair_traj_dist(const double* X, int64_t T, int64_t D, int L,
                          const int64_t* ti, const int64_t* tj, int64_t npairs,
                          double* out) {
  if (!X || !ti || !tj || !out || L < 1 || L > T || D < 1) return ORACLE_EINVAL;
  int64_t np_ = T - L + 1;
  for (int64_t q = 0; q < npairs; ++q)
    if (ti[q] < 0 || ti[q] >= np_ || tj[q] < 0 || tj[q] >= np_)
      return ORACLE_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < npairs; ++q) out[q] = traj_dist(X, D, L, ti[q], tj[q]);
  return ORACLE_OK;
}

typedef struct {
  double d;
  int64_t j;
} cand_t;

static int cand_cmp(const void* a, const void* b) {
  const cand_t* x = (const cand_t*)a;
  const cand_t* y = (const cand_t*)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  if (x->j < y->j) return -1;
  if (x->j > y->j) return 1;
  return 0;
}

/* Exclusion-zone kNN and rarity score (Eq. 3) for given rows.
 *   drows[r*n' + j] = D_L(rows[r], j)  (full rows of the trajectory matrix)
 * For each row t = rows[r]: candidates are j in [0, n') with |t - j| >= L,
 * sorted by (distance, j) ascending; the first k are the neighbours.
 * Outputs: idx[r*k + q], dist[r*k + q] in rank order, score[r] = mean of the
 * k distances summed in rank order, gap[r] = (delta_{k+1} - delta_k)/delta_k
 * (+inf if there is no (k+1)-th candidate; 0/0 is reported as 0 when both are
 * zero and +inf when only delta_k is zero).
 * Rows with fewer than k candidates are rejected (returns ORACLE_EINVAL). */
int oracle_knn_rows(const double* drows, const int64_t* rows, int64_t nrows,
                    int64_t np_, int L, int k, int32_t* idx, double* dist,
                    double* score, double* gap) {
  if (!drows || !rows || !idx || !dist || !score || !gap || k < 1 || L < 1)
    return ORACLE_EINVAL;
  cand_t* buf = (cand_t*)malloc(sizeof(cand_t) * (size_t)np_);
  if (!buf) return ORACLE_ENOMEM;
  int rc = ORACLE_OK;
  for (int64_t r = 0; r < nrows && rc == ORACLE_OK; ++r) {
    int64_t t = rows[r];
    int64_t n = 0;
    for (int64_t j = 0; j < np_; ++j) {
      int64_t gapj = t > j ? t - j : j - t;
      if (gapj >= L) {
        buf[n].d = drows[r * np_ + j];
        buf[n].j = j;
        ++n;
      }
    }
    if (n < k) {
      rc = ORACLE_EINVAL;
      break;
    }
    qsort(buf, (size_t)n, sizeof(cand_t), cand_cmp);
    double s = 0.0;
    for (int q = 0; q < k; ++q) {
      idx[r * k + q] = (int32_t)buf[q].j;
      dist[r * k + q] = buf[q].d;
      s += buf[q].d;
    }
    score[r] = s / (double)k;
    if (n > k) {
      double dk = buf[k - 1].d, dk1 = buf[k].d;
      if (dk > 0.0)
        gap[r] = (dk1 - dk) / dk;
      else
        gap[r] = dk1 > 0.0 ? INFINITY : 0.0;
    } else {
      gap[r] = INFINITY;
    }
  }
  free(buf);
  return rc;
}

/* Analytic gradient of F = sum_t w[t] * s_t with the neighbour sets idx
 * (n' x k) held fixed. Differentiating Eq. 2 inside Eq. 3:
 *   dF/dX_a = (2/k) sum_t w_t sum_{j in N_t} sum_{m<L}
 *             ([a = t+m] - [a = j+m]) (X_{t+m} - X_{j+m})
 * Accumulated term by term in (t, rank, m, p) order into g (T x D, zeroed
 * here). */
int oracle_score_grad(const double* X, int64_t T, int64_t D, int L, int k,
                      const int32_t* idx, const double* w, double* g) {
  if (!X || !idx || !w || !g || L < 1 || L > T || k < 1 || D < 1)
    return ORACLE_EINVAL;
  int64_t np_ = T - L + 1;
  memset(g, 0, sizeof(double) * (size_t)(T * D));
  for (int64_t t = 0; t < np_; ++t) {
    if (w[t] == 0.0) continue;
    double c = 2.0 * w[t] / (double)k;
    for (int q = 0; q < k; ++q) {
      int64_t j = idx[t * k + q];
      if (j < 0 || j >= np_) return ORACLE_EINVAL;
      for (int m = 0; m < L; ++m) {
        const double* xa = X + (t + m) * D;
        const double* xb = X + (j + m) * D;
        double* ga = g + (t + m) * D;
        double* gb = g + (j + m) * D;
        for (int64_t p = 0; p < D; ++p) {
          double diff = xa[p] - xb[p];
          ga[p] += c * diff;
          gb[p] -= c * diff;
        }
      }
    }
  }
  return ORACLE_OK;
}

/* Local intrinsic dimension by the maximum-likelihood kNN estimator of Levina
 * and Bickel (2004), which the paper applies to trajectories with k in
 * {20, 30, 40} (Section 5.1, "Intrinsic dimension study"):
 *   m_k(t) = [ 1/(k-1) * sum_{j=1}^{k-1} ln( T_k(t) / T_j(t) ) ]^{-1}
 * with T_j(t) the Euclidean distance from t to its j-th nearest neighbour.
 * The inputs are the sorted SQUARED distances dist[r*k + q] = T_{q+1}(t)^2
 * of each row, so ln(T_k / T_j) = ln(dist_k / dist_j) / 2, each term taken
 * as written (ratio first, then its logarithm), summed over j = 1..k'-1 in
 * increasing order.
 * Output out[r*k + q] = m_{k'}(t) for k' = q + 1 = 2..k (every prefix of the
 * list is the k'-nearest list); out[r*k] (k' = 1, no ratio) is NaN.
 * Degenerate rows follow IEEE arithmetic: a zero distance below a positive
 * T_k' makes a term +inf and the estimate 0; T_k' = 0 gives NaN; k' equal
 * distances give +inf. */
int oracle_local_dim(const double* dist, int64_t nrows, int k, double* out) {
  if (!dist || !out || nrows < 0 || k < 1) return ORACLE_EINVAL;
  for (int64_t r = 0; r < nrows; ++r) {
    const double* d = dist + r * k;
    out[r * k] = NAN;
    for (int kk = 2; kk <= k; ++kk) {
      double sum = 0.0;
      for (int j = 1; j <= kk - 1; ++j) sum += 0.5 * log(d[kk - 1] / d[j - 1]);
      out[r * k + kk - 1] = 1.0 / (sum / (double)(kk - 1));
    }
  }
  return ORACLE_OK;
}

/* OpenMP thread count actually used by the parallel loops above. */
int oracle_num_threads(void) {
  int n = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
#endif
  return n;
}
