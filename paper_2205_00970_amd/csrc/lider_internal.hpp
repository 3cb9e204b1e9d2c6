// Internal declarations of the gfx950 LIDER library: the device-resident index,
// the per-core-model parameter block, and the exact (non-contracted) FP64 key /
// RMI arithmetic shared by build and search kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lider.h"

namespace lider {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Parameters of one core model (Sections 3.1, 5): the digit box of its items,
// the re-scaling of its keys (Eq. (8)) and its two-stage linear RMI.
struct alignas(16) Model {
  int64_t L;         // items indexed
  int64_t leaf_off;  // first leaf of this model in the index's leaf arrays
  uint64_t kmin, kmax;
  double scale;      // (L-1)/(kmax-kmin), 0 if all keys are equal
  double root_a, root_b;
  int32_t m_eff;     // leading digits that enter the key (radix product <= 2^53)
  int32_t F;         // second-stage width
  int32_t mins[LIDER_MAX_M];
  int32_t maxs[LIDER_MAX_M];
};

static_assert(sizeof(Model) % 16 == 0, "models are copied in 16-byte pieces");

static constexpr uint64_t kKeyLimit = uint64_t(1) << 53;

// Dims per k-step chunk of the operand-ordered corpus copy (Xt).
static constexpr int kTileKS = 32;

// Largest cluster of a multi-array index: the union of a (query, cluster)
// pair's windows is marked in a per-wave bitmap of this many bits.
static constexpr int64_t kMaxMultiCluster = 65536;

// Mixed-radix key of a data tuple over the model's digit box (Section 5.1
// first step, generalised from binary digits to integer digits); digit 0 is
// the most significant, so numeric order is the element-wise SK-LSH order.
__host__ __device__ inline uint64_t encode_data(const int32_t* h, const Model& M) {
  uint64_t K = 0;
  for (int i = 0; i < M.m_eff; ++i) {
    uint64_t R = uint64_t(int64_t(M.maxs[i]) - int64_t(M.mins[i]) + 1);
    K = K * R + uint64_t(int64_t(h[i]) - int64_t(M.mins[i]));
  }
  return K;
}

// Key of a query tuple: digits outside the box saturate (below: this and all
// later digits at their minima; above: at their maxima, plus one), giving the
// count of box tuples lexicographically before the query.
__host__ __device__ inline uint64_t encode_query(const int32_t* h, const Model& M) {
  uint64_t K = 0;
  for (int i = 0; i < M.m_eff; ++i) {
    uint64_t R = uint64_t(int64_t(M.maxs[i]) - int64_t(M.mins[i]) + 1);
    if (h[i] < M.mins[i]) {
      for (; i < M.m_eff; ++i) K = K * uint64_t(int64_t(M.maxs[i]) - int64_t(M.mins[i]) + 1);
      return K;
    }
    if (h[i] > M.maxs[i]) {
      for (; i < M.m_eff; ++i) {
        uint64_t Ri = uint64_t(int64_t(M.maxs[i]) - int64_t(M.mins[i]) + 1);
        K = K * Ri + (Ri - 1);
      }
      return K + 1;
    }
    K = K * R + uint64_t(int64_t(h[i]) - int64_t(M.mins[i]));
  }
  return K;
}

// Eq. (8) with a = 0, b = L-1: exact integer difference, one rounding.
__host__ __device__ inline double rescale(uint64_t K, const Model& M) {
#pragma clang fp contract(off)
  return double(int64_t(K) - int64_t(M.kmin)) * M.scale;
}

// Second-stage model owning the root's predicted share of [0, L).
__host__ __device__ inline int32_t leaf_of(double ra, double rb, int32_t F, int64_t L, double x) {
#pragma clang fp contract(off)
  double p0 = ra * x + rb;
  double v = (p0 * double(F)) / double(L);
  if (!(v >= 0.0)) return 0;
  if (v >= double(F)) return F - 1;
  return int32_t(v);
}

// Predicted location: nearest integer, clamped to [0, L-1] (Section 7.4).
__host__ __device__ inline int64_t pos_of(double la, double lb, int64_t L, double x) {
#pragma clang fp contract(off)
  if (L <= 0) return 0;
  double p = la * x + lb;
  double q = floor(p + 0.5);
  if (!(q >= 0.0)) return 0;
  if (q > double(L - 1)) return L - 1;
  return int64_t(q);
}

// Fixed-length bi-directional window: floor(r/2) to the left, shifted inward at
// the ends to keep min(r, L) positions.
__host__ __device__ inline void window_of(int64_t pos, int64_t r, int64_t L, int64_t* start,
                                          int64_t* len) {
  int64_t lenv = r < L ? r : L;
  int64_t hi = L - r > 0 ? L - r : 0;
  int64_t s = pos - r / 2;
  if (s > hi) s = hi;
  if (s < 0) s = 0;
  *start = s;
  *len = lenv;
}

// encode_query with the digit loop unrolled over LIDER_MAX_M and the early
// exits turned into a saturation state (the same integer arithmetic), so that
// the model's box and the digits are read from registers.
__device__ inline uint64_t encode_query_unrolled(const int32_t (&h)[LIDER_MAX_M], const Model& M) {
  uint64_t K = 0;
  int mode = 0;  // 0: inside the box so far, 1: saturated below, 2: above
#pragma unroll
  for (int i = 0; i < LIDER_MAX_M; ++i) {
    if (i < M.m_eff) {
      const uint64_t R = uint64_t(int64_t(M.maxs[i]) - int64_t(M.mins[i]) + 1);
      if (mode == 0) mode = h[i] < M.mins[i] ? 1 : (h[i] > M.maxs[i] ? 2 : 0);
      const uint64_t dg = mode == 0 ? uint64_t(int64_t(h[i]) - int64_t(M.mins[i]))
                                    : (mode == 1 ? uint64_t(0) : R - 1);
      K = K * R + dg;
    }
  }
  return mode == 2 ? K + 1 : K;
}

// Predicted location of a query in one core model.  The model's header, its
// first m digit bounds (the key reads no others: m_eff <= m) and the query's
// m digits are loaded with all their loads in flight before the arithmetic
// starts; 16-byte loads throughout when the digits are 16-byte aligned.
__device__ inline int64_t locate(const Model* Mp, const double* leaves, const int32_t* qd, int m,
                                 uint64_t* Kout = nullptr) {
  Model M;
  {
    constexpr int kHead = int(offsetof(Model, mins) / 16), kB = LIDER_MAX_M / 4;
    static_assert(offsetof(Model, mins) % 16 == 0 && offsetof(Model, maxs) == offsetof(Model, mins) + 16 * kB,
                  "the digit bounds are whole 16-byte pieces after the header");
    const int4* src = reinterpret_cast<const int4*>(Mp);
    int4* dst = reinterpret_cast<int4*>(&M);
    const int nb = (m + 3) >> 2;
#pragma unroll
    for (int w = 0; w < kHead; ++w) dst[w] = src[w];
#pragma unroll
    for (int w = 0; w < kB; ++w) {
      dst[kHead + w] = w < nb ? src[kHead + w] : int4{0, 0, 0, 0};
      dst[kHead + kB + w] = w < nb ? src[kHead + kB + w] : int4{0, 0, 0, 0};
    }
  }
  int32_t h[LIDER_MAX_M];
  if ((m & 3) == 0 && (reinterpret_cast<uintptr_t>(qd) & 15) == 0) {
#pragma unroll
    for (int w = 0; w < LIDER_MAX_M / 4; ++w) {
      const int4 v = 4 * w < m ? reinterpret_cast<const int4*>(qd)[w] : int4{0, 0, 0, 0};
      h[4 * w] = v.x;
      h[4 * w + 1] = v.y;
      h[4 * w + 2] = v.z;
      h[4 * w + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < LIDER_MAX_M; ++i) h[i] = i < m ? qd[i] : 0;
  }
  if (M.L <= 0) return 0;
  uint64_t K = encode_query_unrolled(h, M);
  if (Kout) *Kout = K;
  double x = rescale(K, M);
  int32_t j = leaf_of(M.root_a, M.root_b, M.F, M.L, x);
  const double* lf = leaves + 2 * (M.leaf_off + j);
  return pos_of(lf[0], lf[1], M.L, x);
}

// Extended hashkey distance of two m-bit hashkeys (Section 4.2), scaled by
// C = 2^B to an exact integer: KL * 2^B + KD_e, with KL the non-prefix length
// and KD_e the absolute difference of the (at most) B bits right after the
// common prefix read as binary numbers.
__host__ __device__ inline int64_t dist_e_scaled(uint64_t a, uint64_t b, int m, int B) {
  const uint64_t x = a ^ b;
  if (x == 0) return 0;
  int p = 63;  // most significant differing bit (bit 0 = least significant)
  while (!((x >> p) & 1u)) --p;
  const int nb = B < p + 1 ? B : p + 1;
  const uint64_t mask = (uint64_t(1) << nb) - 1;
  const int64_t v1 = int64_t((a >> (p + 1 - nb)) & mask), v2 = int64_t((b >> (p + 1 - nb)) & mask);
  const int64_t kl = p + 1;  // non-prefix length: m minus the common prefix m - 1 - p
  (void)m;
  return kl * (int64_t(1) << B) + (v1 > v2 ? v1 - v2 : v2 - v1);
}

// Rigorous bound on |fl32(a.b) - a.b| for a length-d fp32 dot product summed in
// any order (plus the FP64 reference's own rounding), per unit of |a||b|.
__host__ __device__ inline double dot_err_coef(int d) {
  return double(d + 2) * (5.9604644775390625e-08 /* 2^-24 */ + 2.220446049250313e-16);
}

inline size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// ----------------------------------------------------------------- the index
struct Index {
  int device = 0;
  int64_t n = 0;
  int32_t d = 0, C = 0, m = 0, F2 = 0, F1 = 0;
  double w = 1.0;
  int32_t iters_run = 0;
  int64_t max_cluster = 0;
  int32_t storage = LIDER_F32, centroid_storage = LIDER_F32;
  int32_t hash_kind = LIDER_HASH_E2LSH;
  int32_t H = 1;               // hashkey arrays per core model
  int32_t n_cu = 256;

  // Per-array tables are array-major; array 0's sort order is the physical
  // row order (the reordered corpus, tiles, search positions).
  float* X = nullptr;          // [n x d] reordered by array 0's (cluster, key, id)
  // The same rows in the rerank's MFMA operand order (d a multiple of 32):
  // each cluster padded with zero rows to a multiple of 16; per 16-row block
  // and 32-dim k-step one 2 KB chunk of two 1 KB halves, in which lane
  // l = i + 16 s holds dims [4 s, 4 s + 4) (then [16 + 4 s, 16 + 4 s + 4)) of
  // row i -- one contiguous 1 KB wave load per half.
  float* Xt = nullptr;
  // bf16 copy in the same order (storage bf16, d a multiple of 64): 64-dim
  // k-steps, lane l holds dims [8 s, 8 s + 8) then [32 + 8 s, 32 + 8 s + 8).
  __hip_bfloat16* Xbt = nullptr;
  __hip_bfloat16* Xb = nullptr;  // [n x d] bf16 copy (precision form)
  int64_t* perm = nullptr;     // [H x n] sorted position of array h -> original id
  int32_t* perm32 = nullptr;   // [n] array 0's, int32
  uint64_t* keys = nullptr;    // [H x n]
  int32_t* digits = nullptr;   // [H x n x m] per original id
  int32_t* amap = nullptr;     // [(H-1) x n] array h's sorted position -> array 0's
  int32_t* l1map = nullptr;    // [(H-1) x C] same for the centroids retriever
  // [(H-1) x n + 8] amap as positions within the cluster (o_j + p -> the row's
  // position in cluster j): clusters hold at most 65,536 rows; 8 elements of
  // padding for whole 16-byte reads
  uint16_t* amap16 = nullptr;
  int32_t* assign = nullptr;   // [n] per original id
  int64_t* off = nullptr;      // [C+1]
  float* cent = nullptr;       // [C x d] cluster-id order
  float* cent_l1 = nullptr;    // [C x d] layer-1 order
  uint8_t* cent8 = nullptr;    // [C x d] fp8 e4m3, layer-1 order
  float* cent8_scale = nullptr;  // [C]
  __hip_bfloat16* cent_l1_b = nullptr;  // [C x d] bf16 copy of cent_l1 (routing candidates)
  int64_t* l1_order = nullptr;   // [H x C] layer-1 position of array h -> cluster id
  int32_t* l1_order32 = nullptr; // [C] array 0's
  uint64_t* l1_keys = nullptr;   // [H x C]
  int32_t* l1_digits = nullptr;  // [H x C x m]
  float* A = nullptr;          // [2Hm x d]: layer-1 sets of arrays 0..H-1, then layer 2
  float* b = nullptr;          // [2Hm]
  float* anorm = nullptr;      // [2Hm] upper bounds of |A_i|
  float* cent_norm_max = nullptr;  // [1] upper bound of max |centroid|
  // precision form (bf16 copy): upper bounds over the rows of max |x|,
  // max |x - bf16(x)| and max |bf16(x)| (host copies)
  float xb_bound[3] = {0.f, 0.f, 0.f};
  Model* models = nullptr;     // [H x (C+1)], model h*(C+1) + C = array h of layer 1
  double* leaves = nullptr;    // [H x (C*F2 + F1) x 2]
  int32_t* leaf_err = nullptr; // [H x (C*F2 + F1) x 2]
  // rerank tiles: (cluster, first row) of every tile of tile_rows rows, one
  // table per supported tile size (32, 64, 128)
  int32_t n_tiles[3] = {0, 0, 0};
  int32_t* tiles[3] = {nullptr, nullptr, nullptr};  // [n_tiles x 4]: cluster, row0, global row0, rows
  int32_t* tile_base[3] = {nullptr, nullptr, nullptr};  // [C+1] first tile of each cluster
  int32_t* tile_blk[3] = {nullptr, nullptr, nullptr};   // [n_tiles] first 16-row block in Xt
  // layer-1 scoring: the C centroids as one 64-row-tiled "cluster"
  int32_t n_l1_tiles = 0;
  int32_t* l1_tiles = nullptr;  // [n_l1_tiles x 4]: 0, row0, row0, rows
  std::vector<int64_t> h_off;  // host copy of off
};

int set_error(int status, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// ------------------------------------------------------------- build kernels
// hash.hip
// Counters a hash launch clears on the side: a [0, na), b and c [0, nb)
// (nullable each); nz is set by run_hash_ex.
struct HashZero {
  int32_t* a;
  int32_t na;
  int32_t* b;
  int32_t* c;
  int32_t nb;
  int32_t nz;
};
int run_hash_ex(const float* X, int64_t n, int32_t d, const float* A, const float* b,
                const float* anorm, int32_t nh, double w, int32_t* out, int32_t* status,
                int clamp, float* rownorm, hipStream_t st, int kind = 0,
                __hip_bfloat16* xb = nullptr, const HashZero* zero = nullptr);
void launch_norm_bounds(const float* A, int32_t rows, int32_t d, float* out, hipStream_t st);

// kmeans.hip
int run_kmeans(Index& ix, const float* X, const int64_t* init_host, int32_t iters,
               int32_t seeding, hipStream_t st);
int run_kmeans_assign(const float* X, int64_t n, int32_t d, const float* cent, int32_t C,
                      int32_t* assign, const int32_t* prev, int32_t* changed, void* scratch,
                      hipStream_t st);
size_t kmeans_assign_scratch(int64_t n, int32_t C);
int run_centroid_means(const float* X, int64_t n, int32_t d, const int32_t* assign, int32_t C,
                       float* cent, void* scratch, size_t scratch_bytes, hipStream_t st);
size_t centroid_means_scratch(int64_t n, int32_t C);

// radix_sort.hip: stable LSD radix sort of (key, value) pairs by key bits
// [0, bits), 8 bits per pass (n < 2^31; inputs and outputs distinct buffers;
// temp holds radix_sort_temp_bytes).  Asynchronous on st.
size_t radix_sort_temp_bytes(int64_t n, int key_bytes);
template <class K>
int radix_sort_pairs(const K* keys_in, const int32_t* vals_in, K* keys_out, int32_t* vals_out,
                     int64_t n, int bits, void* temp, size_t temp_bytes, hipStream_t st);

// core_build.hip
int build_core_models(Index& ix, const float* Xin, hipStream_t st);
// offsets on the host, largest cluster, rerank tile tables (after build or load)
int finish_index(Index& ix);

// search.hip
size_t search_workspace(const Index& ix, int64_t nq, int32_t k, int32_t c, int32_t r,
                        const lider_search_opts& o);
// ev: NULL or LIDER_NSTAGES + 1 events recorded at the stage boundaries
int run_search(const Index& ix, const float* Q, int64_t nq, int32_t k, int32_t c, int32_t r,
               int64_t* ids, float* scores, void* ws, size_t ws_bytes, hipStream_t st,
               const lider_search_opts& o, const lider_search_debug* dbg, hipEvent_t* ev);

}  // namespace lider
