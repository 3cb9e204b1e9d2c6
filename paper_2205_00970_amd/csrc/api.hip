// The C ABI (include/lider.h): argument validation, index allocation and
// lifetime, build orchestration, search dispatch, exports and error state.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>

#include "lider_internal.hpp"

namespace lider {


namespace {
thread_local std::string g_err;
thread_local int32_t g_fail_next = 0;

struct Profile {
  int32_t max_calls = 0, calls = 0;
  std::vector<hipEvent_t> ev;  // (LIDER_NSTAGES + 1) per call
};
thread_local Profile g_prof;

void profile_release() {
  for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
  g_prof = Profile();
}

template <class T>
int alloc(T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(LIDER_ENOMEM, std::string("out of device memory: ") + what);
  }
  return LIDER_OK;
}

void free_device(Index& ix) {
  void* ptrs[] = {ix.X,      ix.Xb,          ix.perm,     ix.perm32,    ix.keys,
                  ix.digits, ix.assign,      ix.off,      ix.cent,      ix.cent_l1,
                  ix.cent8,  ix.cent8_scale, ix.cent_l1_b, ix.l1_order, ix.l1_order32, ix.l1_keys,
                  ix.l1_digits, ix.A,        ix.b,        ix.anorm,     ix.cent_norm_max,
                  ix.models, ix.leaves,      ix.leaf_err, ix.tiles[0],  ix.tiles[1],
                  ix.tiles[2], ix.l1_tiles,  ix.tile_base[0], ix.tile_base[1],
                  ix.tile_base[2], ix.amap,  ix.l1map,     ix.Xt,        ix.tile_blk[0],
                  ix.tile_blk[1], ix.tile_blk[2], ix.Xbt,      ix.amap16};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

// Device arrays of an index whose parameters are set (build and load).
int alloc_index(Index& ix) {
  const int64_t n = ix.n, d = ix.d, C = ix.C, m = ix.m, H = ix.H;
  const int64_t nleaf = H * (C * ix.F2 + ix.F1);
  const int64_t nh = 2 * H * m;
  int rc = LIDER_OK;
#define TRY(x)                    \
  do {                            \
    if (rc == LIDER_OK) rc = (x); \
  } while (0)
  TRY(alloc(&ix.X, size_t(n) * d, "reordered corpus"));
  TRY(alloc(&ix.perm, size_t(H) * n, "perm"));
  TRY(alloc(&ix.perm32, size_t(n), "perm32"));
  TRY(alloc(&ix.keys, size_t(H) * n, "keys"));
  TRY(alloc(&ix.digits, size_t(H) * n * m, "digits"));
  if (H > 1) {
    TRY(alloc(&ix.amap, size_t(H - 1) * n, "array position maps"));
    TRY(alloc(&ix.l1map, size_t(H - 1) * C, "layer-1 array position maps"));
  }
  TRY(alloc(&ix.assign, size_t(n), "assignment"));
  TRY(alloc(&ix.off, size_t(C) + 1, "offsets"));
  TRY(alloc(&ix.cent, size_t(C) * d, "centroids"));
  TRY(alloc(&ix.cent_l1, size_t(C) * d, "layer-1 centroids"));
  if (ix.centroid_storage == LIDER_FP8E4M3) {
    TRY(alloc(&ix.cent8, size_t(C) * d, "fp8 centroids"));
    TRY(alloc(&ix.cent8_scale, size_t(C), "fp8 scales"));
  }
  if (d % 8 == 0) TRY(alloc(&ix.cent_l1_b, size_t(C) * d, "bf16 layer-1 centroids"));
  TRY(alloc(&ix.l1_order, size_t(H) * C, "layer-1 order"));
  TRY(alloc(&ix.l1_order32, size_t(C), "layer-1 order"));
  TRY(alloc(&ix.l1_keys, size_t(H) * C, "layer-1 keys"));
  TRY(alloc(&ix.l1_digits, size_t(H) * C * m, "layer-1 digits"));
  TRY(alloc(&ix.A, size_t(nh) * d, "LSH projections"));
  TRY(alloc(&ix.b, size_t(nh), "LSH offsets"));
  TRY(alloc(&ix.anorm, size_t(nh), "LSH norms"));
  TRY(alloc(&ix.cent_norm_max, 64, "centroid norm"));
  TRY(alloc(&ix.models, size_t(H) * (C + 1), "models"));
  TRY(alloc(&ix.leaves, size_t(nleaf) * 2, "leaves"));
  TRY(alloc(&ix.leaf_err, size_t(nleaf) * 2, "leaf errors"));
#undef TRY
  return rc;
}

// Seeded draws of the method's random inputs (lider_build_params.seed,
// lider_draw_params): the E2LSH projections a_i ~ N(0, I_d) and offsets
// b_i ~ U[0, w) of Section 4, and the rows that seed k-means (Section 3.2).
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) supplies 64-bit words;
// stream s (0: hash parameters, 1: k-means rows) starts from the seed xor the
// (s+1)-th word of the generator started at state 0.  Uniforms take the top
// 53 bits; normals are Box-Muller pairs (cosine first) in FP64 rounded to
// fp32, filling A row by row; then one uniform per offset.  Seed rows are the
// prefix of a Fisher-Yates shuffle of 0..n-1 (position i takes the id at
// i + floor(x (n - i) / 2^64)).  Host code.
struct SplitMix64 {
  uint64_t state;
  uint64_t next() {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double unit() { return double(next() >> 11) * 0x1.0p-53; }
};

SplitMix64 draw_stream(uint64_t seed, int s) {
  SplitMix64 zero{0};
  uint64_t word = 0;
  for (int i = 0; i <= s; ++i) word = zero.next();
  return SplitMix64{seed ^ word};
}

void draw_hash_params(uint64_t seed, int64_t nh, int64_t d, double w, bool sign, float* A,
                      float* b) {
#pragma clang fp contract(off)
  SplitMix64 g = draw_stream(seed, 0);
  const int64_t total = nh * d;
  for (int64_t i = 0; i < total; i += 2) {
    const double u1 = g.unit();
    const double u2 = g.unit();
    const double radius = std::sqrt(-2.0 * std::log(1.0 - u1));
    const double angle = 6.283185307179586 * u2;
    A[i] = float(radius * std::cos(angle));
    if (i + 1 < total) A[i + 1] = float(radius * std::sin(angle));
  }
  for (int64_t i = 0; i < nh; ++i) b[i] = sign ? 0.f : float(g.unit() * w);
}

void draw_seed_rows(uint64_t seed, int64_t n, int64_t count, int64_t* out) {
  SplitMix64 g = draw_stream(seed, 1);
  std::unordered_map<int64_t, int64_t> moved;  // positions whose id has changed
  auto id_at = [&](int64_t p) {
    const auto it = moved.find(p);
    return it == moved.end() ? p : it->second;
  };
  for (int64_t i = 0; i < count; ++i) {
    const uint64_t x = g.next();
    const int64_t j = i + int64_t((static_cast<unsigned __int128>(x) * uint64_t(n - i)) >> 64);
    const int64_t vi = id_at(i), vj = id_at(j);
    moved[j] = vi;
    moved[i] = vj;
    out[i] = vj;
  }
}

}  // namespace

int set_error(int status, const std::string& msg) {
  g_err = msg;
  return status;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return LIDER_OK;
  return set_error(LIDER_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace lider

using namespace lider;

struct lider_index {
  Index ix;
};

extern "C" {

const char* lider_last_error(void) { return g_err.c_str(); }

void lider_debug_fail_next(int32_t status) { g_fail_next = status; }

void lider_free(lider_index* index) {
  if (!index) return;
  free_device(index->ix);
  delete index;
}

int lider_build(const float* corpus_dev, int64_t n, int32_t d, const lider_build_params* P,
                void* stream, lider_index** out) {
  g_err.clear();
  if (!out) return set_error(LIDER_EINVAL, "out is NULL");
  *out = nullptr;
  if (!corpus_dev || !P) return set_error(LIDER_EINVAL, "corpus or params is NULL");
  if (n < 1 || n > INT32_MAX) return set_error(LIDER_EINVAL, "n must be in 1..2^31-1");
  if (d < 1 || d > 65536) return set_error(LIDER_EINVAL, "d must be in 1..65536");
  if (P->n_clusters < 1 || P->n_clusters > n)
    return set_error(LIDER_EINVAL, "n_clusters must be in 1..n");
  if (P->m < 1 || P->m > LIDER_MAX_M) return set_error(LIDER_EINVAL, "m must be in 1..16");
  if (P->hash_kind != LIDER_HASH_E2LSH && P->hash_kind != LIDER_HASH_SIGN)
    return set_error(LIDER_EINVAL, "hash_kind must be LIDER_HASH_E2LSH or LIDER_HASH_SIGN");
  const bool sign = P->hash_kind == LIDER_HASH_SIGN;
  if (!sign && (!(P->w > 0.0) || !std::isfinite(P->w)))
    return set_error(LIDER_EINVAL, "w must be > 0");
  if (P->rmi_fanout < 1 || P->rmi_fanout_l1 < 0)
    return set_error(LIDER_EINVAL, "rmi_fanout must be >= 1");
  if (P->lsh_a_host && !sign && !P->lsh_b_host)
    return set_error(LIDER_EINVAL, "lsh_b_host is NULL while lsh_a_host is given");
  if (!P->assignment_dev && P->kmeans_iters < 1)
    return set_error(LIDER_EINVAL, "k-means needs kmeans_iters >= 1");
  if (P->storage != LIDER_F32 && P->storage != LIDER_BF16)
    return set_error(LIDER_EINVAL, "storage must be LIDER_F32 or LIDER_BF16");
  if (P->centroid_storage != LIDER_F32 && P->centroid_storage != LIDER_FP8E4M3)
    return set_error(LIDER_EINVAL, "centroid_storage must be LIDER_F32 or LIDER_FP8E4M3");
  if (P->kmeans_seeding != 0 && P->kmeans_seeding != 1)
    return set_error(LIDER_EINVAL, "kmeans_seeding must be 0 or 1");
  if (P->n_arrays < 0 || P->n_arrays > LIDER_MAX_H)
    return set_error(LIDER_EINVAL, "n_arrays must be in 0..16");
  if (!P->assignment_dev && P->kmeans_init_host)
    for (int32_t j = 0; j < (P->kmeans_seeding ? 1 : P->n_clusters); ++j)
      if (P->kmeans_init_host[j] < 0 || P->kmeans_init_host[j] >= n)
        return set_error(LIDER_EINVAL, "kmeans_init_host id out of range");
  hipStream_t st = static_cast<hipStream_t>(stream);
  lider_index* h = new (std::nothrow) lider_index();
  if (!h) return set_error(LIDER_ENOMEM, "out of host memory");
  Index& ix = h->ix;
  ix.n = n;
  ix.d = d;
  ix.C = P->n_clusters;
  ix.m = P->m;
  ix.F2 = P->rmi_fanout;
  ix.F1 = P->rmi_fanout_l1 > 0 ? P->rmi_fanout_l1 : P->rmi_fanout;
  ix.w = sign ? 1.0 : P->w;
  ix.hash_kind = P->hash_kind;
  ix.H = P->n_arrays > 0 ? P->n_arrays : 1;
  ix.storage = P->storage;
  ix.centroid_storage = P->centroid_storage;
  (void)hipGetDevice(&ix.device);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ix.device) == hipSuccess && prop.multiProcessorCount > 0)
      ix.n_cu = prop.multiProcessorCount;
  }
  const int64_t C = ix.C, m = ix.m, H = ix.H;
  int rc = LIDER_OK;
#define TRY(x)                 \
  do {                         \
    if (rc == LIDER_OK) rc = (x); \
  } while (0)
  TRY(alloc_index(ix));
  const int64_t nh = 2 * H * m;
  // draws from the seed where the caller gave none
  std::vector<float> seeded_a, seeded_b;
  std::vector<int64_t> seeded_rows;
  const float* a_host = P->lsh_a_host;
  const float* b_host = P->lsh_b_host;
  const int64_t* init_host = P->kmeans_init_host;
  if (rc == LIDER_OK && !a_host) {
    seeded_a.resize(size_t(nh) * d);
    seeded_b.resize(size_t(nh));
    draw_hash_params(P->seed, nh, d, ix.w, sign, seeded_a.data(), seeded_b.data());
    a_host = seeded_a.data();
    b_host = seeded_b.data();
  }
  if (rc == LIDER_OK && !P->assignment_dev && !init_host) {
    seeded_rows.resize(size_t(P->kmeans_seeding ? 1 : C));
    draw_seed_rows(P->seed, n, int64_t(seeded_rows.size()), seeded_rows.data());
    init_host = seeded_rows.data();
  }
  TRY(check_hip(hipMemcpyAsync(ix.A, a_host, size_t(nh) * d * 4, hipMemcpyHostToDevice, st),
                "copy LSH projections"));
  if (b_host)
    TRY(check_hip(hipMemcpyAsync(ix.b, b_host, size_t(nh) * 4, hipMemcpyHostToDevice,
                                 st),
                  "copy LSH offsets"));
  else
    TRY(check_hip(hipMemsetAsync(ix.b, 0, size_t(nh) * 4, st), "clear LSH offsets"));
  if (rc == LIDER_OK) launch_norm_bounds(ix.A, int32_t(nh), d, ix.anorm, st);
  if (rc == LIDER_OK) {
    if (P->assignment_dev) {
      // given clusters: copy, range-check, centroids = member means (empty: 0)
      TRY(check_hip(hipMemcpyAsync(ix.assign, P->assignment_dev, size_t(n) * 4,
                                   hipMemcpyDeviceToDevice, st),
                    "copy assignment"));
      if (rc == LIDER_OK) {
        std::vector<int32_t> h_asg(static_cast<size_t>(n));
        TRY(check_hip(hipMemcpyAsync(h_asg.data(), ix.assign, size_t(n) * 4, hipMemcpyDeviceToHost, st),
                      "read assignment"));
        TRY(check_hip(hipStreamSynchronize(st), "read assignment"));
        if (rc == LIDER_OK)
          for (int64_t i = 0; i < n; ++i)
            if (h_asg[i] < 0 || h_asg[i] >= ix.C) {
              rc = set_error(LIDER_EINVAL, "assignment value out of range");
              break;
            }
      }
      TRY(check_hip(hipMemsetAsync(ix.cent, 0, size_t(C) * d * 4, st), "zero centroids"));
      void* scr = nullptr;
      const size_t sb = centroid_means_scratch(n, ix.C);
      if (rc == LIDER_OK && hipMalloc(&scr, sb) != hipSuccess)
        rc = set_error(LIDER_ENOMEM, "out of device memory (centroid scratch)");
      TRY(run_centroid_means(corpus_dev, n, d, ix.assign, ix.C, ix.cent, scr, sb, st));
      TRY(check_hip(hipStreamSynchronize(st), "centroids"));
      if (scr) (void)hipFree(scr);
      ix.iters_run = 0;
    } else {
      TRY(run_kmeans(ix, corpus_dev, init_host, P->kmeans_iters, P->kmeans_seeding, st));
    }
  }
  TRY(build_core_models(ix, corpus_dev, st));
  TRY(check_hip(hipStreamSynchronize(st), "index build"));
#undef TRY
  if (rc != LIDER_OK) {
    lider_free(h);
    return rc;
  }
  *out = h;
  return LIDER_OK;
}

int lider_draw_params(uint64_t seed, int32_t n_arrays, int32_t m, int32_t d, double w,
                      int32_t hash_kind, float* lsh_a_host, float* lsh_b_host, int64_t n,
                      int32_t n_rows, int64_t* rows_host) {
  g_err.clear();
  const int32_t H = n_arrays > 0 ? n_arrays : 1;
  if (n_arrays < 0 || n_arrays > LIDER_MAX_H) return set_error(LIDER_EINVAL, "n_arrays must be in 0..16");
  if (m < 1 || m > LIDER_MAX_M) return set_error(LIDER_EINVAL, "m must be in 1..16");
  if (d < 1 || d > 65536) return set_error(LIDER_EINVAL, "d must be in 1..65536");
  if (hash_kind != LIDER_HASH_E2LSH && hash_kind != LIDER_HASH_SIGN)
    return set_error(LIDER_EINVAL, "hash_kind must be LIDER_HASH_E2LSH or LIDER_HASH_SIGN");
  const bool sign = hash_kind == LIDER_HASH_SIGN;
  if (lsh_a_host || lsh_b_host) {
    if (!lsh_a_host || !lsh_b_host) return set_error(LIDER_EINVAL, "give both lsh_a_host and lsh_b_host");
    if (!sign && (!(w > 0.0) || !std::isfinite(w))) return set_error(LIDER_EINVAL, "w must be > 0");
    draw_hash_params(seed, 2 * int64_t(H) * m, d, sign ? 1.0 : w, sign, lsh_a_host, lsh_b_host);
  }
  if (rows_host) {
    if (n < 1 || n > INT32_MAX || n_rows < 0 || n_rows > n)
      return set_error(LIDER_EINVAL, "need 1 <= n <= 2^31-1 and 0 <= n_rows <= n");
    draw_seed_rows(seed, n, n_rows, rows_host);
  }
  return LIDER_OK;
}

int lider_get_info(const lider_index* index, lider_info* out) {
  if (!index || !out) return set_error(LIDER_EINVAL, "NULL argument");
  const Index& ix = index->ix;
  out->n = ix.n;
  out->d = ix.d;
  out->n_clusters = ix.C;
  out->m = ix.m;
  out->rmi_fanout = ix.F2;
  out->rmi_fanout_l1 = ix.F1;
  out->kmeans_iters_run = ix.iters_run;
  out->max_cluster = ix.max_cluster;
  out->w = ix.w;
  out->storage = ix.storage;
  out->centroid_storage = ix.centroid_storage;
  out->n_arrays = ix.H;
  out->hash_kind = ix.hash_kind;
  return LIDER_OK;
}

static int validate_search(const lider_index* index, const float* Q, int64_t nq, int32_t k,
                           int32_t c, int32_t r, const lider_search_opts& o) {
  if (!index) return set_error(LIDER_EINVAL, "index is NULL");
  const Index& ix = index->ix;
  if (nq < 0 || nq > INT32_MAX) return set_error(LIDER_EINVAL, "nq must be in 0..2^31-1");
  if (k < 1 || k > LIDER_MAX_K) return set_error(LIDER_EINVAL, "k must be in 1..1024");
  if (c < 1 || c > LIDER_MAX_C || c > ix.C)
    return set_error(LIDER_EINVAL, "c must be in 1..min(128, n_clusters)");
  if (r < 1) return set_error(LIDER_EINVAL, "r must be >= 1");
  if (o.r1 < 0) return set_error(LIDER_EINVAL, "r1 must be >= 0");
  if (o.precision != LIDER_F32 && o.precision != LIDER_BF16)
    return set_error(LIDER_EINVAL, "precision must be LIDER_F32 or LIDER_BF16");
  if (o.precision == LIDER_BF16 && !ix.Xb && !ix.Xbt)
    return set_error(LIDER_EINVAL, "precision LIDER_BF16 needs an index built with storage BF16");
  if (o.precision == LIDER_BF16 && (ix.d % 8 != 0))
    return set_error(LIDER_EINVAL, "precision LIDER_BF16 needs d divisible by 8");
  if (o.shortlist_mult < 0 || (o.precision == LIDER_BF16 && int64_t(o.shortlist_mult) * k > 4096))
    return set_error(LIDER_EINVAL, "shortlist_mult * k must be at most 4096");
  if (o.tile_rows != 0 && o.tile_rows != 32 && o.tile_rows != 64 && o.tile_rows != 128)
    return set_error(LIDER_EINVAL, "tile_rows must be 0, 32, 64 or 128");
  if (o.grid_mult < 0 || o.grid_mult > 64) return set_error(LIDER_EINVAL, "grid_mult out of range");
  if (o.persistent < 0 || o.persistent > 2) return set_error(LIDER_EINVAL, "persistent must be 0, 1 or 2");
  if (o.l1_dense < -1 || o.l1_dense > 3) return set_error(LIDER_EINVAL, "l1_dense must be -1, 0, 1, 2 or 3");
  if (o.pass_pairs != 0 && o.pass_pairs != 16 && o.pass_pairs != 32 && o.pass_pairs != 64 &&
      o.pass_pairs != 128)
    return set_error(LIDER_EINVAL, "pass_pairs must be 0, 16, 32, 64 or 128");
  if (o.expand_bits < 0 || o.expand_bits > 16)
    return set_error(LIDER_EINVAL, "expand_bits must be in 0..16");
  if (o.expand_bits > 0 && index->ix.hash_kind != LIDER_HASH_SIGN)
    return set_error(LIDER_EINVAL, "expand_bits needs an index built with LIDER_HASH_SIGN");
  if (ix.H > 1 && ix.C > 65536 && std::min<int64_t>(o.r1 > 0 ? o.r1 : r, ix.C) < ix.C)
    return set_error(LIDER_EINVAL,
                     "with n_arrays > 1 and r1 < n_clusters, n_clusters must be at most 65536");
  if (nq > 0 && !Q) return set_error(LIDER_EINVAL, "queries pointer is NULL");
  return LIDER_OK;
}

size_t lider_search_workspace(const lider_index* index, int64_t nq, int32_t k, int32_t c,
                              int32_t r, const lider_search_opts* opts) {
  lider_search_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  if (validate_search(index, reinterpret_cast<const float*>(1), nq, k, c, r, o) != LIDER_OK) return 0;
  return search_workspace(index->ix, nq, k, c, r, o);
}

int lider_search_ex(const lider_index* index, const float* queries_dev, int64_t nq, int32_t k,
                    int32_t c, int32_t r, int64_t* ids_dev, float* scores_dev, void* ws_dev,
                    size_t ws_bytes, void* stream, const lider_search_opts* opts,
                    const lider_search_debug* debug) {
  g_err.clear();
  if (g_fail_next) {
    const int32_t s = g_fail_next;
    g_fail_next = 0;
    return set_error(s, "failure injected by lider_debug_fail_next");
  }
  lider_search_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  int rc = validate_search(index, queries_dev, nq, k, c, r, o);
  if (rc != LIDER_OK) return rc;
  if (nq == 0) return LIDER_OK;
  if (!ids_dev || !scores_dev || !ws_dev) return set_error(LIDER_EINVAL, "output or workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws_dev) & 255)
    return set_error(LIDER_EINVAL, "workspace must be 256-byte aligned");
  hipEvent_t* ev = nullptr;
  if (g_prof.calls < g_prof.max_calls) {
    ev = g_prof.ev.data() + size_t(g_prof.calls) * (LIDER_NSTAGES + 1);
    ++g_prof.calls;
  }
  return run_search(index->ix, queries_dev, nq, k, c, r, ids_dev, scores_dev, ws_dev, ws_bytes,
                    static_cast<hipStream_t>(stream), o, debug, ev);
}

int lider_profile_begin(int32_t max_calls) {
  g_err.clear();
  if (max_calls < 1 || max_calls > 4096) return set_error(LIDER_EINVAL, "max_calls must be in 1..4096");
  profile_release();
  g_prof.ev.resize(size_t(max_calls) * (LIDER_NSTAGES + 1));
  for (auto& e : g_prof.ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      profile_release();
      return set_error(LIDER_EDEVICE, "hipEventCreate failed");
    }
  }
  g_prof.max_calls = max_calls;
  return LIDER_OK;
}

int lider_profile_end(double* stage_ms, int32_t* calls) {
  g_err.clear();
  if (!stage_ms || !calls) return set_error(LIDER_EINVAL, "NULL argument");
  int rc = LIDER_OK;
  for (int s = 0; s < LIDER_NSTAGES; ++s) stage_ms[s] = 0.0;
  for (int32_t c = 0; c < g_prof.calls && rc == LIDER_OK; ++c) {
    hipEvent_t* ev = g_prof.ev.data() + size_t(c) * (LIDER_NSTAGES + 1);
    rc = check_hip(hipEventSynchronize(ev[LIDER_NSTAGES]), "profile event");
    for (int s = 0; s < LIDER_NSTAGES && rc == LIDER_OK; ++s) {
      float ms = 0.f;
      rc = check_hip(hipEventElapsedTime(&ms, ev[s], ev[s + 1]), "profile elapsed time");
      stage_ms[s] += ms;
    }
  }
  *calls = g_prof.calls;
  profile_release();
  return rc;
}

int lider_search(const lider_index* index, const float* queries_dev, int64_t nq, int32_t k,
                 int32_t c, int32_t r, int64_t* ids_dev, float* scores_dev, void* ws_dev,
                 size_t ws_bytes, void* stream) {
  return lider_search_ex(index, queries_dev, nq, k, c, r, ids_dev, scores_dev, ws_dev, ws_bytes,
                         stream, nullptr, nullptr);
}

// --------------------------------------------------- allocation-free search
// lider_search_noalloc's workspace: one array in the library's code object,
// which every GPU the library runs on holds until the process ends.  Host
// code reaches it only through the device address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

int scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  const int grc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (grc != LIDER_OK) return grc;
  if (dev < 0 || dev >= kMaxDevices) return set_error(LIDER_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(LIDER_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return LIDER_OK;
}
}  // namespace

size_t lider_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int lider_search_noalloc(const lider_index* index, const float* queries_dev, int64_t nq,
                         int32_t k, int32_t c, int32_t r, int64_t* ids_dev, float* scores_dev,
                         void* stream, const lider_search_opts* opts) {
  g_err.clear();
  lider_search_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts) o = *opts;
  int rc = validate_search(index, queries_dev, nq, k, c, r, o);
  if (rc != LIDER_OK) return rc;
  if (nq == 0) return LIDER_OK;
  const size_t need = lider_search_workspace(index, nq, k, c, r, &o);
  if (need > kNoAllocScratchBytes)
    return set_error(LIDER_EINVAL, "batch needs " + std::to_string(need) +
                                       " bytes of workspace, more than the " +
                                       std::to_string(kNoAllocScratchBytes) +
                                       "-byte scratch of lider_search_noalloc (use lider_search "
                                       "with a workspace, or a smaller batch)");
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc != LIDER_OK) return rc;
  return lider_search_ex(index, queries_dev, nq, k, c, r, ids_dev, scores_dev, ws,
                         kNoAllocScratchBytes, stream, &o, nullptr);
}

// ------------------------------------------------------------------ exports
namespace {
struct ExportSrc {
  const void* dev;
  size_t bytes;
  int kind;  // 0 plain device copy, 1 model ints, 2 model box, 3 model keys, 4 model doubles
};

ExportSrc export_src(const Index& ix, int32_t what) {
  const size_t n = size_t(ix.n), d = size_t(ix.d), C = size_t(ix.C), m = size_t(ix.m);
  const size_t H = size_t(ix.H);
  const size_t nleaf = H * (C * ix.F2 + ix.F1), nm = H * (C + 1);
  switch (what) {
    case LIDER_X_CENTROIDS: return {ix.cent, C * d * 4, 0};
    case LIDER_X_ASSIGN: return {ix.assign, n * 4, 0};
    case LIDER_X_OFFSETS: return {ix.off, (C + 1) * 8, 0};
    case LIDER_X_PERM: return {ix.perm, H * n * 8, 0};
    case LIDER_X_KEYS: return {ix.keys, H * n * 8, 0};
    case LIDER_X_DIGITS: return {ix.digits, H * n * m * 4, 0};
    case LIDER_X_L1_ORDER: return {ix.l1_order, H * C * 8, 0};
    case LIDER_X_L1_KEYS: return {ix.l1_keys, H * C * 8, 0};
    case LIDER_X_L1_DIGITS: return {ix.l1_digits, H * C * m * 4, 0};
    case LIDER_X_MODEL_INT: return {ix.models, nm * 3 * 8, 1};
    case LIDER_X_MODEL_BOX: return {ix.models, nm * 2 * m * 4, 2};
    case LIDER_X_MODEL_KEY: return {ix.models, nm * 2 * 8, 3};
    case LIDER_X_MODEL_DBL: return {ix.models, nm * 3 * 8, 4};
    case LIDER_X_LEAVES: return {ix.leaves, nleaf * 2 * 8, 0};
    case LIDER_X_LEAF_ERR: return {ix.leaf_err, nleaf * 2 * 4, 0};
    case LIDER_X_REORDERED: return {ix.X, n * d * 4, 0};
    default: return {nullptr, 0, 0};
  }
}
}  // namespace

size_t lider_export_bytes(const lider_index* index, int32_t what) {
  if (!index) return 0;
  return export_src(index->ix, what).bytes;
}

int lider_export(const lider_index* index, int32_t what, void* dst_host, size_t dst_bytes) {
  g_err.clear();
  if (!index || !dst_host) return set_error(LIDER_EINVAL, "NULL argument");
  const Index& ix = index->ix;
  const ExportSrc src = export_src(ix, what);
  if (!src.dev) return set_error(LIDER_EINVAL, "unknown export");
  if (dst_bytes < src.bytes) return set_error(LIDER_EINVAL, "destination too small");
  if (src.kind == 0)
    return check_hip(hipMemcpy(dst_host, src.dev, src.bytes, hipMemcpyDeviceToHost), "export");
  std::vector<Model> M(size_t(ix.H) * (size_t(ix.C) + 1));
  int rc = check_hip(hipMemcpy(M.data(), ix.models, M.size() * sizeof(Model), hipMemcpyDeviceToHost),
                     "export models");
  if (rc != LIDER_OK) return rc;
  for (size_t j = 0; j < M.size(); ++j) {
    if (src.kind == 1) {
      int64_t* o = static_cast<int64_t*>(dst_host) + 3 * j;
      o[0] = M[j].L;
      o[1] = M[j].m_eff;
      o[2] = M[j].F;
    } else if (src.kind == 2) {
      int32_t* o = static_cast<int32_t*>(dst_host) + 2 * ix.m * j;
      for (int i = 0; i < ix.m; ++i) {
        o[i] = M[j].mins[i];
        o[ix.m + i] = M[j].maxs[i];
      }
    } else if (src.kind == 3) {
      uint64_t* o = static_cast<uint64_t*>(dst_host) + 2 * j;
      o[0] = M[j].kmin;
      o[1] = M[j].kmax;
    } else {
      double* o = static_cast<double*>(dst_host) + 3 * j;
      o[0] = M[j].scale;
      o[1] = M[j].root_a;
      o[2] = M[j].root_b;
    }
  }
  return LIDER_OK;
}

// ------------------------------------------------------------ persistence
namespace {
constexpr char kMagic[8] = {'L', 'I', 'D', 'E', 'R', 'I', 'X', '1'};
constexpr uint32_t kVersion = 1;

struct FileHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int64_t n, max_cluster;
  int32_t d, C, m, F2, F1, H, iters_run, storage, centroid_storage, hash_kind, has_cent_l1_b, pad;
  double w;
};

struct Section {
  uint32_t tag;
  void* dev;
  size_t bytes;
};

// Every device array of the index in file order (absent ones have 0 bytes).
std::vector<Section> sections(const Index& ix) {
  const size_t n = size_t(ix.n), d = size_t(ix.d), C = size_t(ix.C), m = size_t(ix.m);
  const size_t H = size_t(ix.H), nh = 2 * H * m, nleaf = H * (C * ix.F2 + ix.F1);
  auto sz = [](const void* p, size_t b) { return p ? b : size_t(0); };
  return {{1, ix.X, n * d * 4},
          {2, nullptr, 0},  // bf16 copies are derived from section 1 on load
          {3, ix.perm, H * n * 8},
          {4, ix.perm32, n * 4},
          {5, ix.keys, H * n * 8},
          {6, ix.digits, H * n * m * 4},
          {7, ix.assign, n * 4},
          {8, ix.off, (C + 1) * 8},
          {9, ix.cent, C * d * 4},
          {10, ix.cent_l1, C * d * 4},
          {11, ix.cent8, sz(ix.cent8, C * d)},
          {12, ix.cent8_scale, sz(ix.cent8_scale, C * 4)},
          {13, ix.cent_l1_b, sz(ix.cent_l1_b, C * d * 2)},
          {14, ix.l1_order, H * C * 8},
          {15, ix.l1_order32, C * 4},
          {16, ix.l1_keys, H * C * 8},
          {17, ix.l1_digits, H * C * m * 4},
          {18, ix.A, nh * d * 4},
          {19, ix.b, nh * 4},
          {20, ix.anorm, nh * 4},
          {21, ix.cent_norm_max, 4},
          {22, ix.models, H * (C + 1) * sizeof(Model)},
          {23, ix.leaves, nleaf * 2 * 8},
          {24, ix.leaf_err, nleaf * 2 * 4},
          {25, ix.amap, sz(ix.amap, (H - 1) * n * 4)},
          {26, ix.l1map, sz(ix.l1map, (H - 1) * C * 4)}};
}

constexpr size_t kStage = size_t(64) << 20;  // host staging per copy

struct FileCloser {
  FILE* f;
  ~FileCloser() {
    if (f) fclose(f);
  }
};
}  // namespace

int lider_save(const lider_index* index, const char* path) {
  g_err.clear();
  if (!index || !path) return set_error(LIDER_EINVAL, "NULL argument");
  const Index& ix = index->ix;
  FileCloser fc{fopen(path, "wb")};
  if (!fc.f) return set_error(LIDER_EIO, std::string("cannot open ") + path + " for writing");
  FileHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.header_bytes = sizeof(FileHeader);
  h.n = ix.n;
  h.max_cluster = ix.max_cluster;
  h.d = ix.d;
  h.C = ix.C;
  h.m = ix.m;
  h.F2 = ix.F2;
  h.F1 = ix.F1;
  h.H = ix.H;
  h.iters_run = ix.iters_run;
  h.storage = ix.storage;
  h.centroid_storage = ix.centroid_storage;
  h.hash_kind = ix.hash_kind;
  h.has_cent_l1_b = ix.cent_l1_b != nullptr;
  h.w = ix.w;
  if (fwrite(&h, sizeof(h), 1, fc.f) != 1) return set_error(LIDER_EIO, "write failed");
  std::vector<char> stage;
  for (const Section& sec : sections(ix)) {
    const uint64_t bytes = sec.bytes;
    if (fwrite(&sec.tag, 4, 1, fc.f) != 1 || fwrite(&bytes, 8, 1, fc.f) != 1)
      return set_error(LIDER_EIO, "write failed");
    stage.resize(std::min(sec.bytes, kStage));
    for (size_t at = 0; at < sec.bytes; at += kStage) {
      const size_t nb = std::min(kStage, sec.bytes - at);
      int rc = check_hip(hipMemcpy(stage.data(), static_cast<char*>(sec.dev) + at, nb,
                                   hipMemcpyDeviceToHost),
                         "save: device to host");
      if (rc != LIDER_OK) return rc;
      if (fwrite(stage.data(), 1, nb, fc.f) != nb) return set_error(LIDER_EIO, "write failed");
    }
  }
  if (fflush(fc.f) != 0) return set_error(LIDER_EIO, "write failed");
  return LIDER_OK;
}

int lider_load(const char* path, void* stream, lider_index** out) {
  g_err.clear();
  if (!out) return set_error(LIDER_EINVAL, "out is NULL");
  *out = nullptr;
  if (!path) return set_error(LIDER_EINVAL, "path is NULL");
  FileCloser fc{fopen(path, "rb")};
  if (!fc.f) return set_error(LIDER_EIO, std::string("cannot open ") + path);
  FileHeader h;
  if (fread(&h, sizeof(h), 1, fc.f) != 1 || std::memcmp(h.magic, kMagic, 8) != 0 ||
      h.version != kVersion || h.header_bytes != sizeof(FileHeader))
    return set_error(LIDER_EIO, "not a LIDER index file of this version");
  if (h.n < 1 || h.n > INT32_MAX || h.d < 1 || h.d > 65536 || h.C < 1 || h.C > h.n || h.m < 1 ||
      h.m > LIDER_MAX_M || h.H < 1 || h.H > LIDER_MAX_H || h.F2 < 1 || h.F1 < 1 ||
      (h.storage != LIDER_F32 && h.storage != LIDER_BF16) ||
      (h.centroid_storage != LIDER_F32 && h.centroid_storage != LIDER_FP8E4M3) ||
      (h.hash_kind != LIDER_HASH_E2LSH && h.hash_kind != LIDER_HASH_SIGN) ||
      h.has_cent_l1_b != (h.d % 8 == 0))
    return set_error(LIDER_EIO, "index file parameters out of range");
  hipStream_t st = static_cast<hipStream_t>(stream);
  lider_index* li = new (std::nothrow) lider_index();
  if (!li) return set_error(LIDER_ENOMEM, "out of host memory");
  Index& ix = li->ix;
  ix.n = h.n;
  ix.d = h.d;
  ix.C = h.C;
  ix.m = h.m;
  ix.F2 = h.F2;
  ix.F1 = h.F1;
  ix.H = h.H;
  ix.w = h.w;
  ix.iters_run = h.iters_run;
  ix.storage = h.storage;
  ix.centroid_storage = h.centroid_storage;
  ix.hash_kind = h.hash_kind;
  (void)hipGetDevice(&ix.device);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ix.device) == hipSuccess && prop.multiProcessorCount > 0)
      ix.n_cu = prop.multiProcessorCount;
  }
  int rc = alloc_index(ix);
  std::vector<char> stage;
  if (rc == LIDER_OK) {
    for (const Section& sec : sections(ix)) {
      uint32_t tag = 0;
      uint64_t bytes = 0;
      if (fread(&tag, 4, 1, fc.f) != 1 || fread(&bytes, 8, 1, fc.f) != 1 || tag != sec.tag ||
          bytes != sec.bytes) {
        rc = set_error(LIDER_EIO, "index file section " + std::to_string(sec.tag) +
                                      " missing or of the wrong size");
        break;
      }
      stage.resize(std::min(sec.bytes, kStage));
      for (size_t at = 0; at < sec.bytes && rc == LIDER_OK; at += kStage) {
        const size_t nb = std::min(kStage, sec.bytes - at);
        if (fread(stage.data(), 1, nb, fc.f) != nb) {
          rc = set_error(LIDER_EIO, "index file truncated");
          break;
        }
        rc = check_hip(hipMemcpyAsync(static_cast<char*>(sec.dev) + at, stage.data(), nb,
                                      hipMemcpyHostToDevice, st),
                       "load: host to device");
        if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "load");
      }
      if (rc != LIDER_OK) break;
    }
  }
  if (rc == LIDER_OK && fgetc(fc.f) != EOF) rc = set_error(LIDER_EIO, "trailing bytes in index file");
  if (rc == LIDER_OK) rc = finish_index(ix);
  if (rc == LIDER_OK && ix.max_cluster != h.max_cluster)
    rc = set_error(LIDER_EIO, "index file offsets do not match its parameters");
  if (rc != LIDER_OK) {
    lider_free(li);
    return rc;
  }
  *out = li;
  return LIDER_OK;
}

// ------------------------------------------------------- stand-alone kernels
int lider_hash(const float* X_dev, int64_t n, int32_t d, const float* A_dev, const float* b_dev,
               int32_t nh, double w, int32_t* out_dev, void* stream) {
  g_err.clear();
  if (!X_dev || !A_dev || !b_dev || !out_dev) return set_error(LIDER_EINVAL, "NULL argument");
  if (n < 0 || d < 1 || nh < 1 || nh > 512 || !(w > 0.0))
    return set_error(LIDER_EINVAL, "bad size argument");
  if (n == 0) return LIDER_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* anorm = nullptr;
  int32_t* cs = nullptr;
  int rc = alloc(&anorm, size_t(nh), "norms");
  if (rc == LIDER_OK) rc = alloc(&cs, 64, "counters");
  if (rc == LIDER_OK) rc = check_hip(hipMemsetAsync(cs, 0, 256, st), "zero");
  if (rc == LIDER_OK) {
    launch_norm_bounds(A_dev, nh, d, anorm, st);
    rc = run_hash_ex(X_dev, n, d, A_dev, b_dev, anorm, nh, w, out_dev, cs + 1, 0, nullptr, st,
                     LIDER_HASH_E2LSH);
  }
  int32_t h_status = 0;
  if (rc == LIDER_OK)
    rc = check_hip(hipMemcpyAsync(&h_status, cs + 1, 4, hipMemcpyDeviceToHost, st), "status");
  if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "hash");
  if (rc == LIDER_OK && h_status) rc = set_error(LIDER_ERANGE, "a hash value does not fit in int32");
  if (anorm) (void)hipFree(anorm);
  if (cs) (void)hipFree(cs);
  return rc;
}

int lider_kmeans_assign(const float* X_dev, int64_t n, int32_t d, const float* cent_dev,
                        int32_t C, int32_t* assign_dev, void* stream) {
  g_err.clear();
  if (!X_dev || !cent_dev || !assign_dev) return set_error(LIDER_EINVAL, "NULL argument");
  if (n < 0 || d < 1 || C < 1) return set_error(LIDER_EINVAL, "bad size argument");
  if (n == 0) return LIDER_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  void* scr = nullptr;
  int32_t* changed = nullptr;
  int rc = LIDER_OK;
  if (hipMalloc(&scr, kmeans_assign_scratch(n, C)) != hipSuccess)
    rc = set_error(LIDER_ENOMEM, "out of device memory (k-means scratch)");
  if (rc == LIDER_OK) rc = alloc(&changed, 64, "counter");
  if (rc == LIDER_OK) rc = check_hip(hipMemsetAsync(changed, 0, 256, st), "zero");
  if (rc == LIDER_OK)
    rc = run_kmeans_assign(X_dev, n, d, cent_dev, C, assign_dev, nullptr, changed, scr, st);
  if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "k-means assignment");
  if (scr) (void)hipFree(scr);
  if (changed) (void)hipFree(changed);
  return rc;
}

}  // extern "C"
