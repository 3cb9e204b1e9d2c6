/*
 * lider_oracle.c -- plain, slow FP64 CPU reference of LIDER (Wang, Ma, Wang,
 * "LIDER: An Efficient High-dimensional Learned Index for Large-scale Dense
 * Passage Retrieval", arXiv 2205.00970): index construction and batched search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under paper_2205_00970_amd/
 * links, includes or calls this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, constant or
 * helper with the HIP path.
 *
 * Everything is computed in IEEE double, sequentially in index order, with no
 * FMA contraction (built with -ffp-contract=off), so that each step can be read
 * against the paper by eye.  Where the paper leaves a point open, the choice
 * made is marked "Reading:".
 *
 * Pins: every function here is checked by tests/test_oracle_pins.py against
 * hand-computed values, closed forms, library routines or brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ERANGE (-4)

#define OR_MAX_M 32

/* 2^53: every integer key up to this bound is exact in a double. */
static const uint64_t OR_KEY_LIMIT = (uint64_t)1 << 53;

/* ------------------------------------------------------------------------ */
/* Section 4 (ESK-LSH base hash).  Euclidean p-stable LSH digit
 *   h_i(x) = floor((a_i . x + b_i) / w),
 * the integer-valued hash whose keys the SK-LSH order of Section 4 sorts
 * (Section 4.2 notes that under Euclidean distance every hashkey element is a
 * bounded integer).  The dot product is a sequential FP64 sum in dimension order;
 * fp32*fp32 products are exact in FP64.  Floor rounds toward -infinity. */
static int or_digit(const float* a, const float* x, int32_t d, float b, double w,
                    int32_t* out) {
  double s = 0.0;
  for (int32_t l = 0; l < d; ++l) s = s + (double)a[l] * (double)x[l];
  double t = (s + (double)b) / w;
  double h = floor(t);
  if (!(h >= -2147483648.0 && h <= 2147483647.0)) return OR_ERANGE;
  *out = (int32_t)h;
  return OR_OK;
}

/* Section 4.1 (the cosine variant of ESK-LSH): random-hyperplane LSH, one
 * bit per hash function, h_i(x) = 1 if a_i . x >= 0 else 0, with the same
 * sequential FP64 dot product.  Reading: a projection of exactly zero gives 1. */
static int32_t or_bit(const float* a, const float* x, int32_t d) {
  double s = 0.0;
  for (int32_t l = 0; l < d; ++l) s = s + (double)a[l] * (double)x[l];
  return s >= 0.0 ? 1 : 0;
}

int or_digits_sign(const float* X, int64_t n, int32_t d, const float* A, int32_t nh,
                   int32_t* out) {
  if (n < 0 || d < 1 || nh < 1) return OR_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r)
    for (int32_t i = 0; i < nh; ++i) out[r * nh + i] = or_bit(A + (int64_t)i * d, X + r * d, d);
  return OR_OK;
}

/* Digits of n rows: out[r*nh + i] = h_i(X[r]).  A is [nh x d] row-major. */
int or_digits(const float* X, int64_t n, int32_t d, const float* A, const float* b,
              int32_t nh, double w, int32_t* out) {
  if (n < 0 || d < 1 || nh < 1 || !(w > 0.0)) return OR_EINVAL;
  int status = OR_OK;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < n; ++r) {
    for (int32_t i = 0; i < nh; ++i) {
      int st = or_digit(A + (int64_t)i * d, X + r * d, d, b[i], w, out + r * nh + i);
      if (st != OR_OK) {
#pragma omp atomic write
        status = st;
      }
    }
  }
  return status;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2 / 3.3.2: the corpus is partitioned by k-means.  Lloyd's
 * algorithm with squared Euclidean distance.
 * Reading: assignment = argmin_j sum_l (x_l - mu_jl)^2 in FP64, ties to the
 * smallest centroid index; centroid = FP64 mean of its members summed in
 * ascending id order, rounded once to fp32; an empty cluster keeps its
 * previous centroid. */
static double or_sqdist(const float* x, const float* mu, int32_t d) {
  double s = 0.0;
  for (int32_t l = 0; l < d; ++l) {
    double t = (double)x[l] - (double)mu[l];
    s = s + t * t;
  }
  return s;
}

int or_kmeans_assign(const float* X, int64_t n, int32_t d, const float* cent, int32_t C,
                     int32_t* assign) {
  if (n < 0 || d < 1 || C < 1) return OR_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    int32_t best = 0;
    double bd = or_sqdist(X + i * d, cent, d);
    for (int32_t j = 1; j < C; ++j) {
      double dj = or_sqdist(X + i * d, cent + (int64_t)j * d, d);
      if (dj < bd) {
        bd = dj;
        best = j;
      }
    }
    assign[i] = best;
  }
  return OR_OK;
}

int or_kmeans_update(const float* X, int64_t n, int32_t d, const int32_t* assign, int32_t C,
                     float* cent, int64_t* counts) {
  if (n < 0 || d < 1 || C < 1) return OR_EINVAL;
  double* sums = (double*)calloc((size_t)C * d, sizeof(double));
  if (!sums) return OR_ENOMEM;
  for (int32_t j = 0; j < C; ++j) counts[j] = 0;
  for (int64_t i = 0; i < n; ++i) { /* ascending id: the summation order */
    int32_t j = assign[i];
    if (j < 0 || j >= C) {
      free(sums);
      return OR_EINVAL;
    }
    counts[j] += 1;
    double* sj = sums + (int64_t)j * d;
    const float* xi = X + i * d;
    for (int32_t l = 0; l < d; ++l) sj[l] = sj[l] + (double)xi[l];
  }
  for (int32_t j = 0; j < C; ++j) {
    if (counts[j] == 0) continue; /* empty: keep previous centroid */
    for (int32_t l = 0; l < d; ++l)
      cent[(int64_t)j * d + l] = (float)(sums[(int64_t)j * d + l] / (double)counts[j]);
  }
  free(sums);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Seeded draws of the method's random inputs: the E2LSH projections
 * a_i ~ N(0, I_d) and offsets b_i ~ U[0, w) (Section 4) and the rows that seed
 * k-means (Section 3.2 only says k-means).
 * Reading: one 64-bit seed S; the draws come from SplitMix64 (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014: add
 * the golden-ratio increment to the state, then two xor-shift-multiply rounds
 * and a final xor-shift).  Stream s (0: hash parameters, 1: k-means rows)
 * starts from the state S xor (the (s+1)-th output of the generator started
 * at state 0).  A uniform is u = (x >> 11) * 2^-53 in [0, 1).  Normals come
 * in pairs from the Box-Muller transform (1958) of (u1, u2):
 * sqrt(-2 ln(1 - u1)) * (cos, sin)(2 pi u2), in that order, in FP64, then
 * rounded to fp32.  A is filled row by row ([2Hm x d], the layout of the hash
 * sets), then b_i = fp32(u * w) for each row in order (sign hashes: b = 0, no
 * draws).  k-means rows: the first `count` entries of a Fisher-Yates shuffle
 * of the ids 0..n-1 drawn from stream 1, position i swapped with
 * i + floor(x * (n - i) / 2^64) for the next output x. */
static uint64_t or_sm64(uint64_t* state) {
  *state = *state + 0x9E3779B97F4A7C15ULL;
  uint64_t z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* `count` consecutive outputs of the generator started at `state`. */
void or_splitmix64(uint64_t state, int64_t count, uint64_t* out) {
  for (int64_t i = 0; i < count; ++i) out[i] = or_sm64(&state);
}

static uint64_t or_stream(uint64_t seed, int32_t s) {
  uint64_t t = 0, v = 0;
  for (int32_t i = 0; i <= s; ++i) v = or_sm64(&t);
  return seed ^ v;
}

static double or_uniform(uint64_t* state) {
  return (double)(or_sm64(state) >> 11) * (1.0 / 9007199254740992.0);
}

int or_seeded_lsh(uint64_t seed, int32_t nh, int32_t d, double w, int32_t sign, float* A,
                  float* b) {
  if (nh < 1 || d < 1) return OR_EINVAL;
  uint64_t st = or_stream(seed, 0);
  const int64_t total = (int64_t)nh * d;
  const double two_pi = 6.283185307179586;
  for (int64_t i = 0; i < total; i += 2) {
    double u1 = or_uniform(&st);
    double u2 = or_uniform(&st);
    double rad = sqrt(-2.0 * log(1.0 - u1));
    A[i] = (float)(rad * cos(two_pi * u2));
    if (i + 1 < total) A[i + 1] = (float)(rad * sin(two_pi * u2));
  }
  for (int32_t i = 0; i < nh; ++i) b[i] = sign ? 0.0f : (float)(or_uniform(&st) * w);
  return OR_OK;
}

int or_seeded_rows(uint64_t seed, int64_t n, int32_t count, int64_t* out) {
  if (n < 1 || count < 0 || count > n) return OR_EINVAL;
  int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!ids) return OR_ENOMEM;
  for (int64_t i = 0; i < n; ++i) ids[i] = i;
  uint64_t st = or_stream(seed, 1);
  for (int32_t i = 0; i < count; ++i) {
    uint64_t x = or_sm64(&st);
    int64_t j = i + (int64_t)(((unsigned __int128)x * (uint64_t)(n - i)) >> 64);
    int64_t t = ids[i];
    ids[i] = ids[j];
    ids[j] = t;
    out[i] = ids[i];
  }
  free(ids);
  return OR_OK;
}

/* Reading: k-means initial centres by farthest-first traversal (the maximin
 * rule of Gonzalez's k-center heuristic): the first centre is a given row;
 * every next centre is the row whose squared Euclidean distance (FP64) to its
 * nearest chosen centre is largest, ties to the smallest row id. */
int or_kmeans_seed_farthest(const float* X, int64_t n, int32_t d, int32_t C, int64_t first,
                            int64_t* ids) {
  if (n < 1 || d < 1 || C < 1 || C > n || first < 0 || first >= n) return OR_EINVAL;
  double* D = (double*)malloc(sizeof(double) * (size_t)n);
  if (!D) return OR_ENOMEM;
  for (int64_t i = 0; i < n; ++i) D[i] = INFINITY;
  ids[0] = first;
  for (int32_t t = 1; t < C; ++t) {
    const float* c = X + ids[t - 1] * d;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double v = or_sqdist(X + i * d, c, d);
      if (v < D[i]) D[i] = v;
    }
    int64_t best = 0;
    for (int64_t i = 1; i < n; ++i)
      if (D[i] > D[best]) best = i;
    ids[t] = best;
  }
  free(D);
  return OR_OK;
}

/* Lloyd iterations: cent <- X[init_ids]; repeat { assign; stop if nothing
 * changed (from the second assignment on); update } at most `iters` times.
 * On return the centroids are the means of the returned assignment. */
int or_kmeans(const float* X, int64_t n, int32_t d, int32_t C, const int64_t* init_ids,
              int32_t iters, float* cent, int32_t* assign, int32_t* iters_run) {
  if (n < 1 || d < 1 || C < 1 || C > n || iters < 1) return OR_EINVAL;
  for (int32_t j = 0; j < C; ++j) {
    if (init_ids[j] < 0 || init_ids[j] >= n) return OR_EINVAL;
    memcpy(cent + (int64_t)j * d, X + init_ids[j] * d, sizeof(float) * d);
  }
  int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * n);
  int64_t* counts = (int64_t*)malloc(sizeof(int64_t) * C);
  if (!prev || !counts) {
    free(prev);
    free(counts);
    return OR_ENOMEM;
  }
  int st = OR_OK;
  int32_t it = 0;
  for (; it < iters; ++it) {
    or_kmeans_assign(X, n, d, cent, C, assign);
    if (it > 0 && memcmp(prev, assign, sizeof(int32_t) * n) == 0) {
      ++it;
      break;
    }
    st = or_kmeans_update(X, n, d, assign, C, cent, counts);
    if (st != OR_OK) break;
    memcpy(prev, assign, sizeof(int32_t) * n);
  }
  *iters_run = it;
  free(prev);
  free(counts);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Core model (Sections 3.1, 3.3.1, 5).  One sorted hashkey array and one
 * two-stage RMI. */
typedef struct {
  int64_t L;        /* number of indexed items */
  int32_t m;        /* digits per hashkey */
  int32_t m_eff;    /* leading digits that enter the numeric key */
  int32_t mins[OR_MAX_M], maxs[OR_MAX_M];
  uint64_t kmin, kmax;
  double scale;     /* (L-1)/(kmax-kmin), or 0 */
  double root[2];   /* slope, intercept */
  int32_t F;        /* second-stage width */
  double* leaf;     /* [2F] slope, intercept */
  int32_t* elo;     /* [F] min(true - predicted) over the leaf's items */
  int32_t* ehi;     /* [F] max(true - predicted) */
} or_model;

/* Section 5.1, first step of key re-scaling: the hashkey becomes one integer.
 * The paper reads a binary hashkey as a binary number; for integer digits the
 * same idea is the mixed-radix number over the model's digit box
 * [min_i, max_i], digit 1 most significant.  Numeric order then equals the
 * element-wise (lexicographic) SK-LSH order of Section 4.2.
 * Reading: if the radix product exceeds 2^53, only the longest digit prefix
 * whose product fits enters the key. */
static uint64_t or_encode_data(const int32_t* h, const or_model* M) {
  uint64_t K = 0;
  for (int32_t i = 0; i < M->m_eff; ++i) {
    uint64_t R = (uint64_t)((int64_t)M->maxs[i] - (int64_t)M->mins[i] + 1);
    K = K * R + (uint64_t)((int64_t)h[i] - (int64_t)M->mins[i]);
  }
  return K;
}

/* Reading: a query digit outside the box saturates.  Scanning from the most
 * significant digit, a digit below the box sets it and every later digit to
 * its minimum; a digit above the box sets them to their maxima and adds one.
 * The result is the number of box tuples that precede the query tuple in the
 * lexicographic order, shifted like the data keys, so its rank among the data
 * keys equals the query's rank in the sorted hashkey array. */
static uint64_t or_encode_query(const int32_t* h, const or_model* M) {
  uint64_t K = 0;
  int32_t i = 0;
  for (; i < M->m_eff; ++i) {
    uint64_t R = (uint64_t)((int64_t)M->maxs[i] - (int64_t)M->mins[i] + 1);
    if (h[i] < M->mins[i]) {
      for (; i < M->m_eff; ++i) {
        uint64_t Ri = (uint64_t)((int64_t)M->maxs[i] - (int64_t)M->mins[i] + 1);
        K = K * Ri;
      }
      return K;
    }
    if (h[i] > M->maxs[i]) {
      for (; i < M->m_eff; ++i) {
        uint64_t Ri = (uint64_t)((int64_t)M->maxs[i] - (int64_t)M->mins[i] + 1);
        K = K * Ri + (Ri - 1);
      }
      return K + 1;
    }
    K = K * R + (uint64_t)((int64_t)h[i] - (int64_t)M->mins[i]);
  }
  return K;
}

/* Section 5.1, second step, Eq. (8): min-max normalisation into [0, L-1]
 * (a = 0, b = L-1).  Reading: computed as (K - Kmin) * scale with
 * scale = (L-1)/(Kmax-Kmin), one rounding after an exact integer difference;
 * scale = 0 when all keys are equal. */
static double or_rescale(uint64_t K, const or_model* M) {
  return (double)((int64_t)K - (int64_t)M->kmin) * M->scale;
}

/* Section 5.2: the simplified RMI uses linear regressions only.
 * Reading: ordinary least squares of position y on key x over the pairs with
 * index in [lo, hi) whose leaf equals `leaf` (leaf < 0: all pairs), sums taken
 * sequentially in position order.  No variance gives slope 0 and the mean
 * position as intercept. */
static void or_ols(const double* x, int64_t lo, int64_t hi, const int32_t* leaf_of_pair,
                   int32_t leaf, double* slope, double* icpt, int64_t* count) {
  int64_t n = 0;
  double sx = 0.0, sy = 0.0;
  for (int64_t i = lo; i < hi; ++i) {
    if (leaf >= 0 && leaf_of_pair[i] != leaf) continue;
    sx = sx + x[i];
    sy = sy + (double)(i - lo);
    ++n;
  }
  *count = n;
  if (n == 0) return;
  double mx = sx / (double)n, my = sy / (double)n;
  double sxx = 0.0, sxy = 0.0;
  for (int64_t i = lo; i < hi; ++i) {
    if (leaf >= 0 && leaf_of_pair[i] != leaf) continue;
    double dx = x[i] - mx;
    double dy = (double)(i - lo) - my;
    sxx = sxx + dx * dx;
    sxy = sxy + dx * dy;
  }
  *slope = sxx > 0.0 ? sxy / sxx : 0.0;
  *icpt = my - (*slope) * mx;
}

/* Second-stage routing: the root's prediction picks the leaf that owns that
 * share of the position range (Section 5 describes each model of a layer as
 * responsible for a subspace of the locations).
 * Reading: leaf = clamp(floor(p0 * F / L), 0, F-1); NaN goes to leaf 0. */
static int32_t or_leaf_of(double root_slope, double root_icpt, int32_t F, int64_t L, double x) {
  double p0 = root_slope * x + root_icpt;
  double v = (p0 * (double)F) / (double)L;
  if (!(v >= 0.0)) return 0;
  if (v >= (double)F) return F - 1;
  return (int32_t)v;
}

/* Predicted location.  Section 7.4: predictions above L-1 are cut to L-1 and
 * negative ones to 0.  Reading: round to nearest (floor(p + 0.5)) before the
 * clamp, clamping in the double domain. */
static int64_t or_pos_of(const double* leaf, int32_t j, int64_t L, double x) {
  if (L <= 0) return 0;
  double p = leaf[2 * j] * x + leaf[2 * j + 1];
  double q = floor(p + 0.5);
  if (!(q >= 0.0)) return 0;
  if (q > (double)(L - 1)) return L - 1;
  return (int64_t)q;
}

/* Train a two-stage linear RMI on (x[i], i), i = 0..L-1 (x nondecreasing). */
int or_rmi_train(const double* x, int64_t L, int32_t F, double* root, double* leaf,
                 int32_t* elo, int32_t* ehi) {
  if (L < 0 || F < 1) return OR_EINVAL;
  root[0] = 0.0;
  root[1] = 0.0;
  for (int32_t j = 0; j < F; ++j) {
    leaf[2 * j] = 0.0;
    leaf[2 * j + 1] = 0.0;
    elo[j] = 0;
    ehi[j] = 0;
  }
  if (L == 0) return OR_OK;
  int64_t cnt;
  or_ols(x, 0, L, NULL, -1, &root[0], &root[1], &cnt);
  int32_t* lf = (int32_t*)malloc(sizeof(int32_t) * (size_t)L);
  if (!lf) return OR_ENOMEM;
  for (int64_t i = 0; i < L; ++i) lf[i] = or_leaf_of(root[0], root[1], F, L, x[i]);
  for (int32_t j = 0; j < F; ++j) {
    double s = 0.0, c = 0.0;
    or_ols(x, 0, L, lf, j, &s, &c, &cnt);
    if (cnt == 0) { /* Reading: an empty leaf copies the root */
      s = root[0];
      c = root[1];
    }
    leaf[2 * j] = s;
    leaf[2 * j + 1] = c;
  }
  int32_t* seen = (int32_t*)calloc((size_t)F, sizeof(int32_t));
  if (!seen) {
    free(lf);
    return OR_ENOMEM;
  }
  for (int64_t i = 0; i < L; ++i) {
    int32_t j = lf[i];
    int64_t e = i - or_pos_of(leaf, j, L, x[i]);
    if (!seen[j]) {
      elo[j] = (int32_t)e;
      ehi[j] = (int32_t)e;
      seen[j] = 1;
    } else {
      if (e < elo[j]) elo[j] = (int32_t)e;
      if (e > ehi[j]) ehi[j] = (int32_t)e;
    }
  }
  free(seen);
  free(lf);
  return OR_OK;
}

int64_t or_rmi_predict(const double* root, const double* leaf, int32_t F, int64_t L, double x) {
  if (L <= 0) return 0;
  return or_pos_of(leaf, or_leaf_of(root[0], root[1], F, L, x), L, x);
}

int32_t or_rmi_leaf(const double* root, int32_t F, int64_t L, double x) {
  return or_leaf_of(root[0], root[1], F, L, x);
}

/* Key of a data tuple and of a (saturated) query tuple against a box. */
static void or_model_box(or_model* M, int32_t m, const int32_t* mins, const int32_t* maxs) {
  M->m = m;
  for (int32_t i = 0; i < m; ++i) {
    M->mins[i] = mins[i];
    M->maxs[i] = maxs[i];
  }
  uint64_t prod = 1;
  int32_t me = 0;
  for (; me < m; ++me) {
    uint64_t R = (uint64_t)((int64_t)maxs[me] - (int64_t)mins[me] + 1);
    if (R > OR_KEY_LIMIT / prod) break;
    prod *= R;
  }
  M->m_eff = me;
}

uint64_t or_encode_box(const int32_t* h, int32_t m, const int32_t* mins, const int32_t* maxs,
                       int32_t query, int32_t* m_eff) {
  or_model M;
  memset(&M, 0, sizeof(M));
  or_model_box(&M, m, mins, maxs);
  *m_eff = M.m_eff;
  return query ? or_encode_query(h, &M) : or_encode_data(h, &M);
}

/* Window of the fixed-length bi-directional range search (Sections 3.3.1, 4):
 * `r` positions around the predicted one.  Reading: floor(r/2) positions to
 * the left, shifted inward at either end so min(r, L) positions are kept. */
static void or_window(int64_t pos, int64_t r, int64_t L, int64_t* start, int64_t* len) {
  int64_t lenv = r < L ? r : L;
  int64_t hi = L - r > 0 ? L - r : 0;
  int64_t s = pos - r / 2;
  if (s > hi) s = hi;
  if (s < 0) s = 0;
  *start = s;
  *len = lenv;
}

void or_window_pub(int64_t pos, int64_t r, int64_t L, int64_t* start, int64_t* len) {
  or_window(pos, r, L, start, len);
}

/* Section 4.2, extended hashkey distance of two m-bit hashkeys (bit 1 most
 * significant, as Decimal() reads them):
 *   dist_e(K1, K2) = KL(K1, K2) + KD_e(K1, K2) / C,   C = 2^B,
 * KL = the non-prefix length (m minus the length of the common prefix), KD_e =
 * |Decimal(K1[l+1 .. l+B]) - Decimal(K2[l+1 .. l+B])| over the B bits right
 * after the common prefix of length l.  Returned as the integer
 * C * dist_e = KL * 2^B + KD_e (exact).  Reading: when fewer than B bits follow
 * the prefix, the sub-sequence is the remaining bits (still divided by 2^B). */
int64_t or_dist_e(uint64_t K1, uint64_t K2, int32_t m, int32_t B) {
  int32_t l = 0;
  while (l < m && ((K1 >> (m - 1 - l)) & 1u) == ((K2 >> (m - 1 - l)) & 1u)) ++l;
  int64_t KL = m - l;
  int64_t v1 = 0, v2 = 0;
  for (int32_t t = l; t < l + B && t < m; ++t) {
    v1 = v1 * 2 + (int64_t)((K1 >> (m - 1 - t)) & 1u);
    v2 = v2 * 2 + (int64_t)((K2 >> (m - 1 - t)) & 1u);
  }
  int64_t KD = v1 > v2 ? v1 - v2 : v2 - v1;
  return KL * ((int64_t)1 << B) + KD;
}

/* Bi-directional expansion search guided by dist_e (Sections 3.3.1, 4.2):
 * starting from the predicted location, the range grows one position at a
 * time on the side whose next hashkey is closer to the query hashkey Kq in
 * dist_e, until min(r, L) positions are taken; when one side is exhausted the
 * other continues.  keys[0..L) is the sorted hashkey array.  Reading: the
 * predicted location itself is taken first and a tie goes to the left side. */
static void or_window_expand(const uint64_t* keys, int64_t L, int64_t pos, int64_t r,
                             uint64_t Kq, int32_t m, int32_t B, int64_t* start, int64_t* len) {
  int64_t take = r < L ? r : L;
  if (take <= 0) {
    *start = 0;
    *len = 0;
    return;
  }
  int64_t lo = pos - 1, hi = pos + 1, got = 1;
  while (got < take) {
    if (lo < 0) {
      ++hi;
    } else if (hi >= L) {
      --lo;
    } else if (or_dist_e(keys[lo], Kq, m, B) <= or_dist_e(keys[hi], Kq, m, B)) {
      --lo;
    } else {
      ++hi;
    }
    ++got;
  }
  *start = lo + 1;
  *len = take;
}

void or_window_expand_pub(const uint64_t* keys, int64_t L, int64_t pos, int64_t r, uint64_t Kq,
                          int32_t m, int32_t B, int64_t* start, int64_t* len) {
  or_window_expand(keys, L, pos, r, Kq, m, B, start, len);
}

/* ------------------------------------------------------------------------ */
/* Build one core model over L items whose digits (row-major, m per item) and
 * ids are given in ascending id order (Section 3.3.1): hash keys are sorted
 * (SK-LSH order, ties by id), re-scaled (Eq. (8)) and the RMI is trained on
 * (key, location).  order[p] = index (into the given items) at location p. */
static int or_core_build(or_model* M, int64_t L, int32_t m, int32_t F, const int32_t* digits,
                         int32_t binary, int64_t* order, uint64_t* keys_sorted);

typedef struct {
  uint64_t key;
  int64_t idx;
} or_kv;

static int or_kv_cmp(const void* a, const void* b) {
  const or_kv* x = (const or_kv*)a;
  const or_kv* y = (const or_kv*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

/* binary: the hashkeys are bits (Section 4.1) and the key is Decimal() of
 * the bit string (Section 5.1): the box is fixed at [0, 1] for every bit. */
static int or_core_build(or_model* M, int64_t L, int32_t m, int32_t F, const int32_t* digits,
                         int32_t binary, int64_t* order, uint64_t* keys_sorted) {
  memset(M, 0, sizeof(*M));
  M->L = L;
  M->m = m;
  M->F = F;
  M->leaf = (double*)calloc((size_t)2 * F, sizeof(double));
  M->elo = (int32_t*)calloc((size_t)F, sizeof(int32_t));
  M->ehi = (int32_t*)calloc((size_t)F, sizeof(int32_t));
  if (!M->leaf || !M->elo || !M->ehi) return OR_ENOMEM;
  if (L == 0) return OR_OK;
  int32_t mins[OR_MAX_M], maxs[OR_MAX_M];
  for (int32_t i = 0; i < m; ++i) {
    mins[i] = binary ? 0 : digits[i];
    maxs[i] = binary ? 1 : digits[i];
  }
  if (!binary)
    for (int64_t t = 1; t < L; ++t)
      for (int32_t i = 0; i < m; ++i) {
        int32_t v = digits[t * m + i];
        if (v < mins[i]) mins[i] = v;
        if (v > maxs[i]) maxs[i] = v;
      }
  or_model_box(M, m, mins, maxs);
  or_kv* kv = (or_kv*)malloc(sizeof(or_kv) * (size_t)L);
  double* x = (double*)malloc(sizeof(double) * (size_t)L);
  if (!kv || !x) {
    free(kv);
    free(x);
    return OR_ENOMEM;
  }
  for (int64_t t = 0; t < L; ++t) {
    kv[t].key = or_encode_data(digits + t * m, M);
    kv[t].idx = t;
  }
  qsort(kv, (size_t)L, sizeof(or_kv), or_kv_cmp);
  for (int64_t p = 0; p < L; ++p) {
    order[p] = kv[p].idx;
    keys_sorted[p] = kv[p].key;
  }
  M->kmin = kv[0].key;
  M->kmax = kv[L - 1].key;
  M->scale = M->kmax > M->kmin ? (double)(L - 1) / (double)(M->kmax - M->kmin) : 0.0;
  for (int64_t p = 0; p < L; ++p) x[p] = or_rescale(kv[p].key, M);
  int st = or_rmi_train(x, L, F, M->root, M->leaf, M->elo, M->ehi);
  free(kv);
  free(x);
  return st;
}

static int64_t or_model_locate(const or_model* M, const int32_t* qdigits, uint64_t* K,
                               double* xq) {
  if (M->L == 0) {
    *K = 0;
    *xq = 0.0;
    return 0;
  }
  *K = or_encode_query(qdigits, M);
  *xq = or_rescale(*K, M);
  return or_rmi_predict(M->root, M->leaf, M->F, M->L, *xq);
}

/* ------------------------------------------------------------------------ */
/* The two-layer index (Sections 3.2, 3.3.2).  Every core model keeps H
 * hashkey arrays, each with its own hash functions, sorted array and RMI
 * (Sections 3.3.1, 4.3); H = 1 is the single-array core model.  Arrays are
 * stored array-major: array h of a per-row table starts at h * n. */
typedef struct {
  int64_t n;
  int32_t d, C, m, F2, F1, H;
  double w;
  int32_t kind;        /* 0: Euclidean E2LSH digits, 1: sign bits (Section 4.1) */
  const float* X;      /* caller-owned corpus, original id order [n x d] */
  float* A;            /* [2Hm x d]: rows h*m.. layer-1 array h, H*m + h*m.. layer-2 array h */
  float* b;            /* [2Hm] */
  float* cent;         /* [C x d] */
  int32_t* assign;     /* [n] */
  int32_t iters_run;
  int64_t* off;        /* [C+1] first sorted position of each cluster */
  int64_t* perm;       /* [H x n] sorted position in array h -> original id */
  uint64_t* keys;      /* [H x n] key at each sorted position of array h */
  int32_t* digits;     /* [H x n x m] layer-2 digits of array h per original id */
  or_model* models;    /* [H x (C+1)]; model h*(C+1) + C is array h of the centroids retriever */
  int64_t* l1_order;   /* [H x C] layer-1 sorted position in array h -> cluster id */
  uint64_t* l1_keys;   /* [H x C] */
  int32_t* l1_digits;  /* [H x C x m] layer-1 digits of array h per cluster id */
} or_index;

void or_free(or_index* ix) {
  if (!ix) return;
  free(ix->A);
  free(ix->b);
  free(ix->cent);
  free(ix->assign);
  free(ix->off);
  free(ix->perm);
  free(ix->keys);
  free(ix->digits);
  if (ix->models)
    for (int64_t j = 0; j < (int64_t)ix->H * (ix->C + 1); ++j) {
      free(ix->models[j].leaf);
      free(ix->models[j].elo);
      free(ix->models[j].ehi);
    }
  free(ix->models);
  free(ix->l1_order);
  free(ix->l1_keys);
  free(ix->l1_digits);
  free(ix);
}

/* Digits of n rows under hash functions A (nh rows), either family. */
static int or_hash_rows(const or_index* ix, const float* X, int64_t n, const float* A,
                        const float* b, int32_t* out) {
  return ix->kind ? or_digits_sign(X, n, ix->d, A, ix->m, out)
                  : or_digits(X, n, ix->d, A, b, ix->m, ix->w, out);
}

/* Build: k-means (or a given assignment), then for each of the H arrays one
 * core model over the centroids (layer 1) and one per cluster over its
 * members (layer 2). */
or_index* or_build(const float* X, int64_t n, int32_t d, int32_t C, const int32_t* assign_in,
                   const int64_t* init_ids, int32_t kmeans_iters, const float* A, const float* b,
                   int32_t m, int32_t H, double w, int32_t F2, int32_t F1, int32_t kind,
                   int* status) {
  *status = OR_EINVAL;
  if (n < 1 || d < 1 || C < 1 || C > n || m < 1 || m > OR_MAX_M || H < 1 || H > 64 ||
      !(w > 0.0) || F2 < 1 || F1 < 1 || kind < 0 || kind > 1 || (kind == 1 && m > 53))
    return NULL;
  or_index* ix = (or_index*)calloc(1, sizeof(or_index));
  if (!ix) {
    *status = OR_ENOMEM;
    return NULL;
  }
  ix->n = n;
  ix->d = d;
  ix->C = C;
  ix->m = m;
  ix->H = H;
  ix->F2 = F2;
  ix->F1 = F1;
  ix->w = w;
  ix->kind = kind;
  ix->X = X;
  const size_t nh = (size_t)2 * H * m;
  ix->A = (float*)malloc(sizeof(float) * nh * d);
  ix->b = (float*)malloc(sizeof(float) * nh);
  ix->cent = (float*)malloc(sizeof(float) * (size_t)C * d);
  ix->assign = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  ix->off = (int64_t*)calloc((size_t)C + 1, sizeof(int64_t));
  ix->perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)H * n);
  ix->keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)H * n);
  ix->digits = (int32_t*)malloc(sizeof(int32_t) * (size_t)H * n * m);
  ix->models = (or_model*)calloc((size_t)H * (C + 1), sizeof(or_model));
  ix->l1_order = (int64_t*)malloc(sizeof(int64_t) * (size_t)H * C);
  ix->l1_keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)H * C);
  ix->l1_digits = (int32_t*)malloc(sizeof(int32_t) * (size_t)H * C * m);
  if (!ix->A || !ix->b || !ix->cent || !ix->assign || !ix->off || !ix->perm || !ix->keys ||
      !ix->digits || !ix->models || !ix->l1_order || !ix->l1_keys || !ix->l1_digits) {
    or_free(ix);
    *status = OR_ENOMEM;
    return NULL;
  }
  memcpy(ix->A, A, sizeof(float) * nh * d);
  if (b)
    memcpy(ix->b, b, sizeof(float) * nh);
  else
    memset(ix->b, 0, sizeof(float) * nh);
  int st;
  if (assign_in) {
    for (int64_t i = 0; i < n; ++i) {
      if (assign_in[i] < 0 || assign_in[i] >= C) {
        or_free(ix);
        *status = OR_EINVAL;
        return NULL;
      }
      ix->assign[i] = assign_in[i];
    }
    /* centroids = member means (an empty cluster has none: zero vector) */
    memset(ix->cent, 0, sizeof(float) * (size_t)C * d);
    int64_t* counts = (int64_t*)malloc(sizeof(int64_t) * C);
    if (!counts) {
      or_free(ix);
      *status = OR_ENOMEM;
      return NULL;
    }
    st = or_kmeans_update(X, n, d, ix->assign, C, ix->cent, counts);
    free(counts);
    ix->iters_run = 0;
  } else {
    st = or_kmeans(X, n, d, C, init_ids, kmeans_iters, ix->cent, ix->assign, &ix->iters_run);
  }
  if (st != OR_OK) {
    or_free(ix);
    *status = st;
    return NULL;
  }
  /* members of each cluster in ascending id order */
  for (int64_t i = 0; i < n; ++i) ix->off[ix->assign[i] + 1] += 1;
  for (int32_t j = 0; j < C; ++j) ix->off[j + 1] += ix->off[j];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)C);
  int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int32_t* mdig = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * m);
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!fill || !members || !mdig || !order) {
    free(fill);
    free(members);
    free(mdig);
    free(order);
    or_free(ix);
    *status = OR_ENOMEM;
    return NULL;
  }
  for (int32_t j = 0; j < C; ++j) fill[j] = ix->off[j];
  for (int64_t i = 0; i < n; ++i) members[fill[ix->assign[i]]++] = i;
  st = OR_OK;
  for (int32_t h = 0; h < H && st == OR_OK; ++h) {
    /* layer-2 digits of every row under array h's hash set */
    int32_t* dig = ix->digits + (size_t)h * n * m;
    const size_t row2 = (size_t)H * m + (size_t)h * m;
    st = or_hash_rows(ix, X, n, A + row2 * d, ix->b + row2, dig);
    if (st != OR_OK) break;
    for (int64_t p = 0; p < n; ++p)
      memcpy(mdig + p * m, dig + members[p] * m, sizeof(int32_t) * m);
    for (int32_t j = 0; j < C && st == OR_OK; ++j) {
      int64_t o = ix->off[j], L = ix->off[j + 1] - o;
      st = or_core_build(&ix->models[(int64_t)h * (C + 1) + j], L, m, F2, mdig + o * m, kind,
                         order + o, ix->keys + (size_t)h * n + o);
      for (int64_t p = 0; p < L; ++p) ix->perm[(size_t)h * n + o + p] = members[o + order[o + p]];
    }
    if (st != OR_OK) break;
    /* layer 1: the centroids retriever over the C centroids (array h's hash
     * set rows h*m..), ids = cluster index */
    int32_t* dg1 = ix->l1_digits + (size_t)h * C * m;
    const size_t row1 = (size_t)h * m;
    st = or_hash_rows(ix, ix->cent, C, A + row1 * d, ix->b + row1, dg1);
    if (st == OR_OK)
      st = or_core_build(&ix->models[(int64_t)h * (C + 1) + C], C, m, F1, dg1, kind,
                         ix->l1_order + (size_t)h * C, ix->l1_keys + (size_t)h * C);
  }
  free(fill);
  free(members);
  free(mdig);
  free(order);
  if (st != OR_OK) {
    or_free(ix);
    *status = st;
    return NULL;
  }
  *status = OR_OK;
  return ix;
}

/* ------------------------------------------------------------------------ */
/* Candidate verification and final top-k (Sections 3.3.1, 6.2): exact score,
 * then the k best by score, ties by smaller id (Reading), kept in a small
 * sorted array by insertion. */
typedef struct {
  double score;
  int64_t id;
} or_cand;

static int or_better(double s1, int64_t i1, double s2, int64_t i2) {
  if (s1 != s2) return s1 > s2;
  return i1 < i2;
}

/* Insert (s, id) into best[0..*cnt) kept sorted best-first, capacity k. */
static void or_topk_push(or_cand* best, int32_t* cnt, int32_t k, double s, int64_t id) {
  int32_t c = *cnt;
  if (c == k && !or_better(s, id, best[c - 1].score, best[c - 1].id)) return;
  int32_t p = c < k ? c : k - 1;
  while (p > 0 && or_better(s, id, best[p - 1].score, best[p - 1].id)) {
    best[p] = best[p - 1];
    --p;
  }
  best[p].score = s;
  best[p].id = id;
  if (c < k) *cnt = c + 1;
}

static double or_dot(const float* a, const float* x, int32_t d) {
  double s = 0.0;
  for (int32_t l = 0; l < d; ++l) s = s + (double)a[l] * (double)x[l];
  return s;
}

/* Search (Section 3.3.2): layer-1 core model routes the query to c clusters;
 * each routed cluster's core model predicts a location and scans r positions
 * around it; all candidates are scored exactly and merged into the top k.
 * With H arrays per core model (Section 3.3.1) every array predicts its own
 * location and scans its own window; a core model's candidates are the union
 * of its H windows, each item counted once.  Reading: the merge of the
 * per-array results is the top of that union (score desc, id asc), which is
 * the same as merging the per-array top lists and dropping repeats.
 * Reading: raw inner product is the score for routing and ranking.
 * Outputs: ids/scores [nq x k] (pad -1 / -inf).  Optional debug outputs:
 *   qdig [nq x 2Hm]          query digits (layer-1 sets h = 0..H-1, then layer 2)
 *   l1   [nq x H x 3]        per array: layer-1 predicted location, window start, length
 *   routed [nq x c]          routed cluster ids, score desc, id asc (-1 pad)
 *   pairs [nq x c x H x 3]   per routed cluster and array: location, start, length */
int or_search(const or_index* ix, const float* Q, int64_t nq, int32_t k, int32_t c, int32_t r,
              int32_t r1, int32_t expand_bits, int64_t* ids, double* scores, int32_t* qdig,
              int64_t* l1, int32_t* routed, int64_t* pairs) {
  if (!ix || nq < 0 || k < 1 || c < 1 || c > ix->C || r < 1 || r1 < 1) return OR_EINVAL;
  /* expand_bits = B > 0: dist_e-guided expansion (binary hashkeys only) */
  if (expand_bits < 0 || expand_bits > 16 || (expand_bits > 0 && ix->kind != 1)) return OR_EINVAL;
  const int32_t m = ix->m, d = ix->d, C = ix->C, H = ix->H;
  const int64_t n = ix->n;
  const int32_t nh = 2 * H * m;
  int status = OR_OK;
#pragma omp parallel
  {
    int32_t* dg = (int32_t*)malloc(sizeof(int32_t) * nh);
    or_cand* rb = (or_cand*)malloc(sizeof(or_cand) * (size_t)c);
    or_cand* best = (or_cand*)malloc(sizeof(or_cand) * (size_t)k);
    /* last (query, item) that took each centroid / row: repeats across the
     * arrays of one core model are skipped */
    int64_t* seen1 = (int64_t*)malloc(sizeof(int64_t) * (size_t)C);
    int64_t* seen2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!dg || !rb || !best || !seen1 || !seen2) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
      for (int32_t j = 0; j < C; ++j) seen1[j] = -1;
      for (int64_t i = 0; i < n; ++i) seen2[i] = -1;
#pragma omp for schedule(dynamic, 4)
      for (int64_t q = 0; q < nq; ++q) {
        const float* qv = Q + q * d;
        for (int32_t i = 0; i < nh; ++i) {
          if (ix->kind) {
            dg[i] = or_bit(ix->A + (int64_t)i * d, qv, d);
          } else if (or_digit(ix->A + (int64_t)i * d, qv, d, ix->b[i], ix->w, dg + i) != OR_OK) {
#pragma omp atomic write
            status = OR_ERANGE;
            dg[i] = 0;
          }
        }
        if (qdig)
          for (int32_t i = 0; i < nh; ++i) qdig[q * nh + i] = dg[i];
        /* layer 1: centroids retriever, the union of its H windows */
        uint64_t K;
        double xq;
        int32_t nr = 0;
        for (int32_t h = 0; h < H; ++h) {
          const or_model* M1 = &ix->models[(int64_t)h * (C + 1) + C];
          const int64_t* ord = ix->l1_order + (size_t)h * C;
          int64_t pos1 = or_model_locate(M1, dg + h * m, &K, &xq);
          int64_t s1, len1;
          if (expand_bits)
            or_window_expand(ix->l1_keys + (size_t)h * C, C, pos1, r1, K, m, expand_bits, &s1,
                             &len1);
          else
            or_window(pos1, r1, C, &s1, &len1);
          if (l1) {
            l1[(q * H + h) * 3 + 0] = pos1;
            l1[(q * H + h) * 3 + 1] = s1;
            l1[(q * H + h) * 3 + 2] = len1;
          }
          for (int64_t p = s1; p < s1 + len1; ++p) {
            int64_t j = ord[p];
            if (seen1[j] == q) continue;
            seen1[j] = q;
            or_topk_push(rb, &nr, c, or_dot(qv, ix->cent + j * d, d), j);
          }
        }
        if (routed)
          for (int32_t t = 0; t < c; ++t) routed[q * c + t] = t < nr ? (int32_t)rb[t].id : -1;
        /* layer 2: in-cluster retrievers, then the merge */
        int32_t nb = 0;
        for (int32_t t = 0; t < c; ++t) {
          for (int32_t h = 0; h < H; ++h) {
            int64_t pos = 0, s = 0, len = 0;
            if (t < nr) {
              int64_t j = rb[t].id;
              const or_model* Mj = &ix->models[(int64_t)h * (C + 1) + j];
              const int64_t o = ix->off[j];
              pos = or_model_locate(Mj, dg + H * m + h * m, &K, &xq);
              if (expand_bits)
                or_window_expand(ix->keys + (size_t)h * n + o, Mj->L, pos, r, K, m, expand_bits,
                                 &s, &len);
              else
                or_window(pos, r, Mj->L, &s, &len);
              for (int64_t p = s; p < s + len; ++p) {
                int64_t id = ix->perm[(size_t)h * n + o + p];
                if (seen2[id] == q * c + t) continue;
                seen2[id] = q * c + t;
                or_topk_push(best, &nb, k, or_dot(qv, ix->X + id * d, d), id);
              }
            }
            if (pairs) {
              int64_t* pp = pairs + ((q * c + t) * H + h) * 3;
              pp[0] = pos;
              pp[1] = s;
              pp[2] = len;
            }
          }
        }
        for (int32_t t = 0; t < k; ++t) {
          ids[q * k + t] = t < nb ? best[t].id : -1;
          scores[q * k + t] = t < nb ? best[t].score : -INFINITY;
        }
      }
    }
    free(dg);
    free(rb);
    free(best);
    free(seen1);
    free(seen2);
  }
  return status;
}

/* Flat exact search (the brute-force baseline of Section 7.1.2): FP64 inner
 * product against every row, top k by score desc, id asc. */
int or_bruteforce(const float* X, int64_t n, int32_t d, const float* Q, int64_t nq, int32_t k,
                  int64_t* ids, double* scores) {
  if (n < 0 || d < 1 || nq < 0 || k < 1) return OR_EINVAL;
  int status = OR_OK;
#pragma omp parallel
  {
    or_cand* best = (or_cand*)malloc(sizeof(or_cand) * (size_t)k);
    if (!best) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t q = 0; q < nq; ++q) {
        int32_t nb = 0;
        for (int64_t i = 0; i < n; ++i)
          or_topk_push(best, &nb, k, or_dot(Q + q * d, X + i * d, d), i);
        for (int32_t t = 0; t < k; ++t) {
          ids[q * k + t] = t < nb ? best[t].id : -1;
          scores[q * k + t] = t < nb ? best[t].score : -INFINITY;
        }
      }
    }
    free(best);
  }
  return status;
}

/* FP64 inner products of listed (query, row) pairs: out[t] = Q[qi[t]] . X[xi[t]]. */
void or_pair_scores(const float* X, const float* Q, int32_t d, const int64_t* qi,
                    const int64_t* xi, int64_t cnt, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < cnt; ++t) out[t] = or_dot(Q + qi[t] * d, X + xi[t] * d, d);
}

/* ------------------------------------------------------------------------ */
/* Accessors for the tests. */
int64_t or_n(const or_index* ix) { return ix->n; }
int32_t or_iters_run(const or_index* ix) { return ix->iters_run; }
void or_get_centroids(const or_index* ix, float* out) {
  memcpy(out, ix->cent, sizeof(float) * (size_t)ix->C * ix->d);
}
void or_get_assign(const or_index* ix, int32_t* out) {
  memcpy(out, ix->assign, sizeof(int32_t) * (size_t)ix->n);
}
void or_get_offsets(const or_index* ix, int64_t* out) {
  memcpy(out, ix->off, sizeof(int64_t) * ((size_t)ix->C + 1));
}
/* Per-array tables, array-major: [H x n], [H x n], [H x n x m]. */
void or_get_perm(const or_index* ix, int64_t* out) {
  memcpy(out, ix->perm, sizeof(int64_t) * (size_t)ix->H * ix->n);
}
void or_get_keys(const or_index* ix, uint64_t* out) {
  memcpy(out, ix->keys, sizeof(uint64_t) * (size_t)ix->H * ix->n);
}
void or_get_digits(const or_index* ix, int32_t* out) {
  memcpy(out, ix->digits, sizeof(int32_t) * (size_t)ix->H * ix->n * ix->m);
}
/* [H x C], [H x C], [H x C x m] */
void or_get_l1(const or_index* ix, int64_t* order, uint64_t* keys, int32_t* digits) {
  memcpy(order, ix->l1_order, sizeof(int64_t) * (size_t)ix->H * ix->C);
  memcpy(keys, ix->l1_keys, sizeof(uint64_t) * (size_t)ix->H * ix->C);
  memcpy(digits, ix->l1_digits, sizeof(int32_t) * (size_t)ix->H * ix->C * ix->m);
}
/* Model j = h * (C+1) + i of array h: i = 0..C-1 clusters, i = C layer 1.
 * ints: L, m_eff, F; mins/maxs [m];
 * keys: kmin, kmax; dbl: scale, root slope, root intercept; leaf [2F];
 * elo/ehi [F]. */
void or_get_model(const or_index* ix, int32_t j, int64_t* ints, int32_t* mins, int32_t* maxs,
                  uint64_t* kminmax, double* dbl, double* leaf, int32_t* elo, int32_t* ehi) {
  const or_model* M = &ix->models[j];
  ints[0] = M->L;
  ints[1] = M->m_eff;
  ints[2] = M->F;
  for (int32_t i = 0; i < ix->m; ++i) {
    mins[i] = M->mins[i];
    maxs[i] = M->maxs[i];
  }
  kminmax[0] = M->kmin;
  kminmax[1] = M->kmax;
  dbl[0] = M->scale;
  dbl[1] = M->root[0];
  dbl[2] = M->root[1];
  memcpy(leaf, M->leaf, sizeof(double) * 2 * (size_t)M->F);
  memcpy(elo, M->elo, sizeof(int32_t) * (size_t)M->F);
  memcpy(ehi, M->ehi, sizeof(int32_t) * (size_t)M->F);
}

/* ------------------------------------------------------------------------ */
/* One stand-alone core model for the tests: build from digits given in
 * ascending id order, export its parameters, locate query digits. */
int or_core(int64_t L, int32_t m, int32_t F, const int32_t* digits, int32_t binary,
            int64_t* order, uint64_t* keys, int32_t* meff, int32_t* mins, int32_t* maxs,
            uint64_t* kminmax, double* dbl, double* leaf, int32_t* elo, int32_t* ehi) {
  if (L < 0 || m < 1 || m > OR_MAX_M || F < 1) return OR_EINVAL;
  or_model M;
  int st = or_core_build(&M, L, m, F, digits, binary, order, keys);
  if (st == OR_OK) {
    *meff = M.m_eff;
    for (int32_t i = 0; i < m; ++i) {
      mins[i] = M.mins[i];
      maxs[i] = M.maxs[i];
    }
    kminmax[0] = M.kmin;
    kminmax[1] = M.kmax;
    dbl[0] = M.scale;
    dbl[1] = M.root[0];
    dbl[2] = M.root[1];
    memcpy(leaf, M.leaf, sizeof(double) * 2 * (size_t)F);
    memcpy(elo, M.elo, sizeof(int32_t) * (size_t)F);
    memcpy(ehi, M.ehi, sizeof(int32_t) * (size_t)F);
  }
  free(M.leaf);
  free(M.elo);
  free(M.ehi);
  return st;
}

int64_t or_core_query(int64_t L, int32_t m, int32_t F, int32_t meff, const int32_t* mins,
                      const int32_t* maxs, const uint64_t* kminmax, const double* dbl,
                      const double* leaf, const int32_t* qdig, uint64_t* K, double* x) {
  or_model M;
  memset(&M, 0, sizeof(M));
  M.L = L;
  M.m = m;
  M.m_eff = meff;
  M.F = F;
  for (int32_t i = 0; i < m; ++i) {
    M.mins[i] = mins[i];
    M.maxs[i] = maxs[i];
  }
  M.kmin = kminmax[0];
  M.kmax = kminmax[1];
  M.scale = dbl[0];
  M.root[0] = dbl[1];
  M.root[1] = dbl[2];
  M.leaf = (double*)leaf;
  return or_model_locate(&M, qdig, K, x);
}
