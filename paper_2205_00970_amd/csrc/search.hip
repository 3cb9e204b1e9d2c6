// Batched LIDER search (Section 3.3.2) on gfx950.
//
//   1. E2LSH digits of every query for both layers (fp32 MFMA + FP64 edge
//      recompute, hash.hip).
//   2. Centroids retriever: key, RMI location, window of r1 centroids in its
//      sorted order (contiguous rows of the layer-1-ordered centroid copy).
//   3. Routing: inner products with the window centroids, top c clusters.  The
//      set of routed clusters is decided in FP64 (an fp32 near-tie at the c-th
//      place triggers a sequential FP64 rescoring of the window).
//   4. In-cluster retrievers: per (query, routed cluster) pair the key, RMI
//      location and window of r rows; pairs are grouped by cluster.
//   5. Rerank (where the time goes): cluster-major; one workgroup per tile of
//      consecutive rows of one cluster (rows are stored in sorted order, so a
//      window is a contiguous slab) scores the tile against every pair whose
//      window overlaps it with fp32 (or bf16) MFMA, writing each pair's window
//      scores.  Optionally persistent over the tile list.
//   6. Per query, top k over the union of its windows (score desc, id asc)
//      with a radix select + bitonic sort in LDS (Section 6.2's final merge).
#include <hip/hip_fp8.h>

#include <algorithm>
#include <type_traits>

#include "lider_internal.hpp"

namespace lider {


namespace {


struct alignas(16) Pair {
  int32_t j, s, len, pos;
};

// Counters block layout (int32): [0] unused, [1] status,
// [8..15] per-XCD tile counters of the persistent rerank, [16] active-tile
// count.
constexpr int kCtrWords = 64;

// Routing candidates kept per query for the FP64 rescoring.
constexpr int kCandCap = 256;
constexpr int kCntCopies = 8;  // copies of the per-cluster pair counters (layer 2 pairs)

constexpr int32_t kBufWord3 = 0x00020000;  // buffer resource word 3 for gfx9-family targets

struct Plan {
  size_t o_ctr, o_qdig, o_qnorm, o_l1, o_l1p, o_l1cs, o_rs, o_rs64, o_routed, o_pairs,
      o_ccount, o_cstart, o_cfill, o_wl, o_sbuf, o_qb, o_slist, o_aflag, o_alist, o_kq, o_lst,
      o_rw, o_pw, o_mask, o_rcand, o_rcnt, total;
  int32_t r1, rcap, S;
  int ti, npcm;  // rerank tile table and 16-pair blocks per pass
  bool cert;     // precision form with the certified shortlist
  size_t o_scnt;
  // l1_dense_rows: layer-1 scores of every centroid (dense product), else of
  // the r1-windows (window kernel).  Several hashkey arrays: lcap = layer-1
  // union capacity per query (list mode when r1 < C), mw = mask words per
  // (query, cluster) pair.
  bool l1_dense_rows, l1_list;
  int32_t lcap, mw;
  // block keys (the block form of the selection): nbcap per pair, 0 = none
  size_t o_bkey;
  int32_t nbcap;
};

// Rerank shape: rows per tile (index into the tile tables: 32, 64, 128) and
// 16-pair column blocks per MFMA pass.  A tile overlapped by P pairs is
// streamed ceil(P / pass) times, while a wider pass holds more accumulators.
// Unless the caller fixes them, both follow the expected overlap: the pairs
// per cluster times the share of a cluster that one pair's window (for several
// arrays, the hull of its H windows) covers, widened by the tile.  With the
// operand-ordered copy of the precision asked for and the direct schedule the
// workgroup rerank takes 128-row tiles and a pass of at least twice the
// expected overlap (the overlap varies from tile to tile; a second pass
// re-streams the tile): 16 or 32 pairs, else 128 (1M x 768: about 10 pairs per
// 128-row tile at c = 1 -> 32-pair passes; 31 at c = 8, r = 256 and 80 with
// ten arrays -> 128).  Otherwise the per-wave
// rerank: about 10 pairs per tile run fastest with 64-row tiles and 32-pair
// passes, about 26 with 32-row tiles and 64-pair passes, about 80 with 32-row
// tiles and 128-pair passes.
void rerank_shape(const Index& ix, int64_t nq, int32_t c, int32_t r, const lider_search_opts& o,
                  int* ti, int* npcm) {
  const double lbar = std::max(1.0, double(ix.n) / double(ix.C));
  const double span = std::min(lbar, double(ix.H) * std::min(double(r), lbar));
  const double per_cluster = double(nq) * c / double(ix.C);
  const bool bf16 = o.precision == LIDER_BF16;
  const bool wg_ok = o.persistent == 0 && (bf16 ? (ix.d % 64 == 0 && ix.Xbt) : (ix.d % 32 == 0 && ix.Xt));
  if (wg_ok && (o.tile_rows == 0 || o.tile_rows == 128)) {
    *ti = 2;
    if (o.pass_pairs > 0) {
      *npcm = o.pass_pairs / 16;
    } else {
      // 16 or 32 pairs keep three waves per SIMD; wider passes hold two
      // either way, so beyond 32 the widest (one pass for most tiles)
      const double est = per_cluster * std::min(1.0, (span + 128.0) / lbar);
      *npcm = 2.0 * est <= 16.0 ? 1 : 2.0 * est <= 32.0 ? 2 : 8;
    }
    return;
  }
  const double est = per_cluster * std::min(1.0, (span + 64.0) / lbar);
  const int wide = est <= 16.0 ? 0 : est <= 48.0 ? 1 : 2;
  if (o.tile_rows == 32) *ti = 0;
  else if (o.tile_rows == 64) *ti = 1;
  else if (o.tile_rows == 128) *ti = 2;
  else *ti = wide == 0 ? 1 : 0;
  *npcm = o.pass_pairs > 0 ? o.pass_pairs / 16 : (wide == 0 ? 2 : wide == 1 ? 4 : 8);
}

Plan make_plan(const Index& ix, int64_t nq, int32_t k, int32_t c, int32_t r,
               const lider_search_opts& o) {
  Plan p;
  const int32_t H = ix.H;
  const int32_t r1 = int32_t(std::min<int64_t>(o.r1 > 0 ? o.r1 : r, ix.C));
  // several arrays: a pair's candidates span up to its whole cluster.  The
  // score row stride is a multiple of 32 floats: rerank tiles start at
  // multiples of 64 rows of their cluster, so whole-cluster windows store
  // whole 128-byte lines (an odd stride splits every 16-row store segment
  // over two lines: 1.6x the score bytes reached HBM).
  const int32_t rcap = int32_t((std::max<int64_t>(
      1, H > 1 ? ix.max_cluster : std::min<int64_t>(r, ix.max_cluster)) + 31) / 32 * 32);
  // precision form: shortlist_mult 0 lists a certified shortlist (up to every
  // candidate of the query), > 0 the best shortlist_mult * k bf16 scores
  const bool cert = o.precision == LIDER_BF16 && o.shortlist_mult == 0;
  const int32_t S = o.precision == LIDER_BF16 && !cert ? std::min(4096, o.shortlist_mult * k) : 0;
  p.l1_list = H > 1 && r1 < ix.C;
  p.l1_dense_rows = H > 1 || o.l1_dense >= 0;
  p.lcap = p.l1_list ? int32_t(std::min<int64_t>(ix.C, int64_t(H) * r1)) : r1;
  p.mw = H > 1 ? int32_t((ix.max_cluster + 127) / 128 * 4) : 0;
  const int64_t np = nq * c;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += al256(bytes);
    return at;
  };
  p.o_ctr = take(kCtrWords * 4);
  p.o_qdig = take(size_t(nq) * 2 * H * ix.m * 4);
  p.o_qnorm = take(size_t(nq) * 4);
  p.o_l1 = take(size_t(nq) * H * 3 * 4);
  p.o_l1p = take(size_t(nq) * H * sizeof(Pair));
  p.o_l1cs = take(2 * 4);
  p.o_rs = take(size_t(nq) * (p.l1_dense_rows ? ix.C : r1) * 4);
  p.o_rs64 = take(size_t(nq) * p.lcap * 8);
  p.o_rcand = take(size_t(nq) * kCandCap * 4);
  p.o_rcnt = take(size_t(nq) * 4);
  p.o_lst = take(p.l1_list ? size_t(nq) * p.lcap * 4 : 0);
  p.o_rw = take(p.l1_list ? size_t(nq) * 3 * 4 : 0);
  p.o_pw = take(H > 1 ? size_t(np) * H * sizeof(Pair) : 0);
  p.o_mask = take(H > 1 ? size_t(np) * p.mw * 4 : 0);
  p.o_routed = take(size_t(nq) * c * 4);
  p.o_pairs = take(size_t(nq) * c * sizeof(Pair));
  p.o_ccount = take(size_t(kCntCopies) * ix.C * 4);
  p.o_cstart = take((size_t(ix.C) + 1) * 4);
  p.o_cfill = take(size_t(kCntCopies) * ix.C * 4);
  p.o_wl = take(size_t(nq) * c * 4);
  p.o_sbuf = take(size_t(nq) * c * rcap * 4);
  p.o_qb = take((S || cert || ix.cent8 || ix.cent_l1_b) ? size_t(nq) * ix.d * 2 : 0);
  p.cert = cert;
  p.o_slist = take(cert ? size_t(nq) * c * rcap * 4 : S ? size_t(nq) * S * 4 : 0);
  p.o_scnt = take(cert ? size_t(nq) * 4 : 0);
  // the selection's block form serves k (or the shortlist) < 16 over more
  // than 2,048 candidates per query: fewer candidates fit the per-wave
  // selection's registers, which is faster there than reading the block keys
  // first, and a larger k reads more blocks than it holds in registers (at
  // k = 64 the listing overflows and the selection falls back to its slowest
  // form); a window of at most rcap rows spans at most rcap / 32 + 1 blocks.
  // The room is taken whatever k is, so that the workspace never shrinks as
  // k grows (a workspace sized for the largest k serves every smaller one)
  const int32_t nbroom = int64_t(c) * rcap > 2048 ? rcap / 32 + 1 : 0;
  p.nbcap = (S ? S : k) < 16 ? nbroom : 0;
  p.o_bkey = take(size_t(np) * nbroom * 4);
  rerank_shape(ix, nq, c, r, o, &p.ti, &p.npcm);
  const size_t nt = o.persistent == 2 ? size_t(ix.n_tiles[p.ti]) : 0;
  p.o_aflag = take(nt * 4);
  p.o_alist = take(nt * 4);
  p.o_kq = take(o.expand_bits > 0 ? size_t(nq) * std::max<int32_t>(c, 1) * H * 8 : 0);
  p.total = off;
  p.r1 = r1;
  p.rcap = rcap;
  p.S = S;
  return p;
}

__global__ void zero_kernel(int32_t* p, int64_t cnt) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cnt;
       t += int64_t(gridDim.x) * blockDim.x)
    p[t] = 0;
}

// ------------------------------------------------------------ select helpers
// Sort key of a score: ascending key <=> descending score; -0 == +0; NaN last.
__device__ inline uint32_t score_key(float f) {
  if (f == 0.f) f = 0.f;
  uint32_t b = __float_as_uint(f);
  if (f != f) return 0xffffffffu;
  uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ~ord;
}
__device__ inline float key_score(uint32_t key) {
  uint32_t ord = ~key;
  uint32_t b = (ord & 0x80000000u) ? (ord & 0x7fffffffu) : ~ord;
  return __uint_as_float(b);
}

constexpr int kTieCap = 1024;

struct SelShared {
  uint32_t hist[256];
  uint32_t prefix, mask, kneed;
  int32_t cnt_less, cnt_tie;
  uint32_t tie_id[kTieCap];
  int32_t tie_idx[kTieCap];
  uint32_t red_id[8];
  int32_t red_idx[8];
};

// Block-wide selection of the K smallest (key, id) among n candidates (ids
// unique).  Writes (key << 32 | id) and the candidate index into srt/idx,
// sorted ascending, padded to KP (power of two >= K) with ~0.  Returns
// min(n, K).  Radix select on the 32-bit key (4 passes of 8 bits), exact tie
// handling by id, then a bitonic sort of the K winners.
template <int NT, class KeyF, class IdF>
__device__ int block_select(int n, int K, int KP, KeyF key_of, IdF id_of, uint64_t* srt,
                            int32_t* idx, SelShared& sh) {
  const int tid = threadIdx.x;
  int outn;
  if (n <= K) {
    for (int i = tid; i < n; i += NT) {
      srt[i] = (uint64_t(key_of(i)) << 32) | id_of(i);
      idx[i] = i;
    }
    outn = n;
  } else {
    if (tid == 0) {
      sh.prefix = 0;
      sh.mask = 0;
      sh.kneed = uint32_t(K);
    }
    const int lane = tid & 63;
    for (int shift = 24; shift >= 0; shift -= 8) {
      for (int b = tid; b < 256; b += NT) sh.hist[b] = 0;
      __syncthreads();
      const uint32_t pre = sh.prefix, msk = sh.mask;
      // lanes of a wave with equal digits add once, by their lowest lane
      // (the keys share their high bits: one bin takes most of them)
      for (int i0 = 0; i0 < n; i0 += NT) {
        const int i = i0 + tid;
        const uint32_t k = i < n ? key_of(i) : 0u;
        const bool act = i < n && (k & msk) == pre;
        const uint32_t dg = (k >> shift) & 255u;
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const uint64_t mb = __ballot((dg >> b) & 1u);
          peers &= ((dg >> b) & 1u) ? mb : ~mb;
        }
        if (act && int(__builtin_ctzll(peers)) == lane)
          atomicAdd(&sh.hist[dg], uint32_t(__popcll(peers)));
      }
      __syncthreads();
      if (tid < 64) {
        // the bin holding the kneed-th key: 4 bins per lane, a scan over lanes
        const uint32_t need = sh.kneed;
        uint32_t h[4], sum = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          h[b] = sh.hist[4 * lane + b];
          sum += h[b];
        }
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(incl, o);
          if (lane >= o) incl += y;
        }
        uint32_t cum = incl - sum;
        if (cum < need && need <= incl) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if (cum + h[b] >= need) {
              sh.prefix |= uint32_t(4 * lane + b) << shift;
              sh.mask |= 255u << shift;
              sh.kneed = need - cum;
              break;
            }
            cum += h[b];
          }
        }
        if (tid == 0) {
          sh.cnt_less = 0;
          sh.cnt_tie = 0;
        }
      }
      __syncthreads();
    }
    const uint32_t T = sh.prefix;
    const int kneed = int(sh.kneed);
    for (int i = tid; i < n; i += NT) {
      const uint32_t k = key_of(i);
      if (k < T) {
        const int slot = atomicAdd(&sh.cnt_less, 1);
        srt[slot] = (uint64_t(k) << 32) | id_of(i);
        idx[slot] = i;
      } else if (k == T) {
        const int slot = atomicAdd(&sh.cnt_tie, 1);
        if (slot < kTieCap) {
          sh.tie_id[slot] = id_of(i);
          sh.tie_idx[slot] = i;
        }
      }
    }
    __syncthreads();
    const int base = K - kneed;
    const int ntie = sh.cnt_tie;
    if (ntie <= kTieCap) {
      for (int t = tid; t < ntie; t += NT) {
        const uint32_t myid = sh.tie_id[t];
        int rank = 0;
        for (int u = 0; u < ntie; ++u) rank += sh.tie_id[u] < myid;
        if (rank < kneed) {
          srt[base + rank] = (uint64_t(T) << 32) | myid;
          idx[base + rank] = sh.tie_idx[t];
        }
      }
    } else {
      // many exactly equal scores: take the kneed smallest ids one at a time
      uint32_t last = 0;
      bool first = true;
      for (int rsel = 0; rsel < kneed; ++rsel) {
        uint32_t best = 0xffffffffu;
        int bidx = -1;
        for (int i = tid; i < n; i += NT) {
          if (key_of(i) != T) continue;
          const uint32_t id = id_of(i);
          if ((first || id > last) && id < best) {
            best = id;
            bidx = i;
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const uint32_t ob = __shfl_xor(best, o);
          const int oi = __shfl_xor(bidx, o);
          if (ob < best) {
            best = ob;
            bidx = oi;
          }
        }
        if ((tid & 63) == 0) {
          sh.red_id[tid >> 6] = best;
          sh.red_idx[tid >> 6] = bidx;
        }
        __syncthreads();
        if (tid == 0) {
          for (int w = 1; w < NT / 64; ++w)
            if (sh.red_id[w] < sh.red_id[0]) {
              sh.red_id[0] = sh.red_id[w];
              sh.red_idx[0] = sh.red_idx[w];
            }
          srt[base + rsel] = (uint64_t(T) << 32) | sh.red_id[0];
          idx[base + rsel] = sh.red_idx[0];
        }
        __syncthreads();
        last = sh.red_id[0];
        first = false;
        __syncthreads();
      }
    }
    outn = K;
  }
  __syncthreads();
  for (int i = outn + tid; i < KP; i += NT) {
    srt[i] = ~uint64_t(0);
    idx[i] = -1;
  }
  __syncthreads();
  for (int kk = 2; kk <= KP; kk <<= 1) {
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < KP; i += NT) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & kk) == 0;
          const uint64_t a = srt[i], b = srt[ixj];
          if ((a > b) == up) {
            srt[i] = b;
            srt[ixj] = a;
            const int32_t t = idx[i];
            idx[i] = idx[ixj];
            idx[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  return outn;
}

__host__ __device__ inline int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Precision form, certified shortlist.  The bf16 window score s~ of row x for
// query q differs from the exact inner product q.x by at most
//   E = |q - bf16(q)| |x| + |bf16(q)| |x - bf16(x)| + 2 g_d |bf16(q)| |bf16(x)|
// (q.x - bq.bx = (q - bq).x + bq.(x - bx), each term bounded by
// Cauchy-Schwarz; the products of bf16 values are exact in fp32 and g_d =
// d u / (1 - d u), u = 2^-24, bounds their fp32 accumulation in any order,
// doubled to cover the accumulator's rounding mode).  The index keeps
// Xmax >= |x|, Xres >= |x - bf16(x)| and XBmax >= |bf16(x)| over its rows, so
// E_q bounds every row of query q.  A row of the exact top k then has
// s~ >= T - 2 E_q, with T the k-th best s~ (at least k rows have
// s~ >= T, so the k-th best exact score is >= T - E_q): listing every
// candidate above that threshold and reranking the list in fp32 returns the
// fp32 top k of all candidates.
struct CertArgs {
  const float* Q = nullptr;
  const __hip_bfloat16* Qb = nullptr;
  int32_t d = 0;
  float xmax = 0.f, xres = 0.f, xbmax = 0.f;
  int32_t* scnt = nullptr;  // [nq] rows listed per query
  int64_t cap = 0;          // list entries per query (all its candidates)
};

// Wave-wide (64 active lanes): the largest key (lowest score) still listed,
// from the k-th best key T; T = 0xffffffff (fewer than k candidates) lists
// every candidate.
__device__ uint32_t cert_threshold(const CertArgs& ca, int64_t q, uint32_t T, int lane) {
  double sr = 0.0, sb = 0.0;
  const float* qv = ca.Q + q * ca.d;
  const __hip_bfloat16* qb = ca.Qb + q * ca.d;
  for (int l = lane; l < ca.d; l += 64) {
    const double b = double(__bfloat162float(qb[l]));
    const double r = double(qv[l]) - b;  // exact
    sr += r * r;
    sb += b * b;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    sb += __shfl_xor(sb, o);
  }
  if (T == 0xffffffffu) return 0xfffffffeu;
  const double up = 1.0 + 0x1p-20;  // covers the roundings of this bound's own arithmetic
  const double qres = sqrt(sr) * up, qbn = sqrt(sb) * up;
  const double du = double(ca.d) * 0x1p-24;
  const double gam = 2.0 * du / (1.0 - du);
  const double E = (qres * double(ca.xmax) + qbn * double(ca.xres) + gam * qbn * double(ca.xbmax)) * up;
  const double thr = double(key_score(T)) - 2.0 * E;
  float f = float(thr);
  if (double(f) > thr) f = nextafterf(f, -INFINITY);
  return score_key(f);
}

// ------------------------------------------------------------ layer 1
// Centroids retriever: location and window of every query; the window is also
// written as a (cluster 0, start, length) pair so the tile-scoring kernel can
// score layer 1 exactly like a cluster of C rows.
// kq (nullable) receives each query's layer-1 key for the dist_e expansion.
// One thread per (query, array) item t = q H + h: array h's model, digits and
// window.
struct L1Args {
  const Model* models;
  const double* leaves;
  const int32_t* qdig;
  int32_t m, H;
  int64_t nq;
  int32_t C, r1;
  int32_t* l1;
  Pair* l1pairs;
  int32_t* l1cs;
  uint64_t* kq;
};

__device__ inline void l1_item(const L1Args& a, int64_t t) {
  if (t == 0) {
    a.l1cs[0] = 0;
    a.l1cs[1] = int32_t(a.nq);
  }
  if (t >= a.nq * a.H) return;
  const int64_t q = t / a.H;
  const int32_t h = int32_t(t - q * a.H);
  uint64_t K = 0;
  const int64_t pos = locate(a.models + int64_t(h) * (a.C + 1) + a.C, a.leaves,
                             a.qdig + q * 2 * a.H * a.m + int64_t(h) * a.m, a.m, &K);
  int64_t s, len;
  window_of(pos, a.r1, a.C, &s, &len);  // the expansion (if any) replaces s later
  if (a.kq) a.kq[t] = K;
  a.l1[3 * t] = int32_t(pos);
  a.l1[3 * t + 1] = int32_t(s);
  a.l1[3 * t + 2] = int32_t(len);
  a.l1pairs[t] = Pair{0, int32_t(s), int32_t(len), int32_t(pos)};
}

__global__ void l1_kernel(L1Args a) { l1_item(a, int64_t(blockIdx.x) * blockDim.x + threadIdx.x); }

// Bits of the positions [a, b) that fall in word w of a bitmap (bit i of word
// w is position 32 w + i).
__device__ inline uint32_t range_bits(int32_t w, int32_t a, int32_t b) {
  const int32_t lo = max(a - 32 * w, 0), hi = min(b - 32 * w, 32);
  if (hi <= lo) return 0u;
  const uint32_t span = hi - lo == 32 ? 0xffffffffu : (1u << (hi - lo)) - 1u;
  return span << lo;
}

// Positions p (0 <= p < len) of arrays h0 .. h0 + 3's windows, mapped to array
// 0's positions by map(g, p), set in the wave's LDS bitmap: the lane's four
// positions of each of the four arrays are loaded together, then their bits
// set.  ws / wl hold array h's window start and length in lane h.
template <class Map>
__device__ inline void mark_windows4(uint32_t* bm, int32_t h0, int32_t H, int32_t ws, int32_t wl,
                                     int lane, Map map) {
  int32_t hs[4], hl[4], lmax = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    hs[g] = __shfl(ws, min(h0 + g, H - 1));
    hl[g] = h0 + g < H ? __shfl(wl, h0 + g) : 0;
    lmax = max(lmax, hl[g]);
  }
  for (int32_t p0 = 0; p0 < lmax; p0 += 256) {
    int32_t pos[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t p = p0 + lane + 64 * u;
        pos[g][u] = p < hl[g] ? map(h0 + g, hs[g], p) : -1;
      }
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (pos[g][u] >= 0) atomicOr(&bm[pos[g][u] >> 5], 1u << (pos[g][u] & 31));
  }
}

// Union of a query's H layer-1 windows, as ascending positions of array 0's
// layer-1 order: one wave per query sets the windows in an LDS bitmap of C
// bits (dynamic shared memory, 4 waves x ceil(C/32) words; array 0's window is
// a range of positions, written as whole words), then lists the set bits in
// order, 64 positions per step with one store.
// rw[q] = (0, 0, union size) is the query's window in list form.
__global__ __launch_bounds__(256) void l1_union_kernel(
    const int32_t* __restrict__ l1, int32_t H, int64_t nq, int32_t C,
    const int32_t* __restrict__ l1map, int32_t lcap, int32_t* __restrict__ lst,
    int32_t* __restrict__ rw) {
  extern __shared__ uint32_t bm_all[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t W = (C + 31) / 32;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  uint32_t* bm = bm_all + wave * W;
  for (int64_t q = int64_t(blockIdx.x) * 4 + wave; q < nq; q += int64_t(gridDim.x) * 4) {
    // the H windows, one per lane (H <= 16)
    int32_t ms = 0, ml = 0;
    if (lane < H) {
      ms = l1[3 * (q * H + lane) + 1];
      ml = l1[3 * (q * H + lane) + 2];
    }
    const int32_t s0 = __shfl(ms, 0), e0 = s0 + __shfl(ml, 0);
    for (int32_t w = lane; w < W; w += 64) bm[w] = range_bits(w, s0, e0);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    auto map = [&](int32_t h, int32_t s, int32_t p) { return l1map[int64_t(h - 1) * C + s + p]; };
    for (int32_t h0 = 1; h0 < H; h0 += 4) mark_windows4(bm, h0, H, ms, ml, lane, map);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    int32_t base = 0;
    for (int32_t p0 = 0; p0 < C; p0 += 64) {
      const int32_t p = p0 + lane;
      const bool in = p < C && ((bm[p >> 5] >> (p & 31)) & 1u);
      const uint64_t b = __ballot(in);
      if (in) lst[q * lcap + base + __popcll(b & below)] = p;
      base += __popcll(b);
    }
    if (lane == 0) {
      rw[3 * q] = 0;
      rw[3 * q + 1] = 0;
      rw[3 * q + 2] = base;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// Minimum over the 64 lanes of a wave (all lanes active), on DPP: inclusive
// prefix minima within each row of 16 (row_shr 1, 2, 4, 8; a lane whose
// source lies before its row keeps its own value), then row_bcast:15 and
// row_bcast:31 carry the row minima up to lane 63, which is read back.
__device__ inline uint32_t dpp_min_u32(uint32_t v) {
  auto step = [](uint32_t x, uint32_t y) { return x < y ? x : y; };
  v = step(v, uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), 0x111, 0xf, 0xf, false)));
  v = step(v, uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), 0x112, 0xf, 0xf, false)));
  v = step(v, uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), 0x114, 0xf, 0xf, false)));
  v = step(v, uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), 0x118, 0xf, 0xf, false)));
  v = step(v, uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), 0x142, 0xa, 0xf, false)));
  v = step(v, uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), 0x143, 0xc, 0xf, false)));
  return uint32_t(__builtin_amdgcn_readlane(int(v), 63));
}

// Sum over the 64 lanes of a wave (all lanes active), the same DPP pattern as
// dpp_min_u32 with additions (a lane whose source lies before its row adds 0).
__device__ inline int32_t dpp_sum_i32(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
  return __builtin_amdgcn_readlane(v, 63);
}

// 64-bit minimum: the minimum high word, then the minimum low word among the
// lanes holding it.
__device__ inline uint64_t wave_min_u64(uint64_t v) {
  const uint32_t hi = dpp_min_u32(uint32_t(v >> 32));
  const uint32_t lo = dpp_min_u32(uint32_t(v >> 32) == hi ? uint32_t(v) : 0xffffffffu);
  return (uint64_t(hi) << 32) | lo;
}

// Sequential FP64 inner product in dimension order (the definition).  The
// fp32 products are exact in FP64, so a fused multiply-add rounds exactly
// like the separate product and sum.  Rows of 4k floats at 16-byte aligned
// addresses are read as float4.
__device__ inline double seq_dot_f64(const float* __restrict__ q, const float* __restrict__ mu,
                                     int32_t d) {
  double acc = 0.0;
  int32_t l = 0;
  if ((d & 3) == 0 && ((reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(mu)) & 15) == 0) {
#pragma unroll 4
    for (; l < d; l += 4) {
      const float4 m = *reinterpret_cast<const float4*>(mu + l);
      const float4 x = *reinterpret_cast<const float4*>(q + l);
      acc = fma(double(x.x), double(m.x), acc);
      acc = fma(double(x.y), double(m.y), acc);
      acc = fma(double(x.z), double(m.z), acc);
      acc = fma(double(x.w), double(m.w), acc);
    }
  }
  for (; l < d; ++l) acc = fma(double(q[l]), double(mu[l]), acc);
  return acc;
}

// FP64 decision of the routed set by one wave: the sequential FP64 inner
// product of every window centroid (one lane per centroid), then c rounds of
// (score desc, cluster id asc).  Window entry p is layer-1 position lq[p]
// when a list is given, else s1 + p.
__device__ __attribute__((noinline)) void route_fp64_wave(const float* __restrict__ qv, int32_t d,
                                const float* __restrict__ cent_l1,
                                const int32_t* __restrict__ l1_order32, int32_t s1, int32_t len1,
                                const int32_t* __restrict__ lq, int32_t c,
                                double* __restrict__ r64, int32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int p = lane; p < len1; p += 64)
    r64[p] = seq_dot_f64(qv, cent_l1 + int64_t(lq ? lq[p] : s1 + p) * d, d);
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  for (int t = 0; t < c; ++t) {
    double bv = -INFINITY;
    int32_t bi = 0x7fffffff, bp = -1;
    for (int p = lane; p < len1; p += 64) {
      const double v = r64[p];
      if (v == -INFINITY) continue;  // already chosen
      const int32_t id = l1_order32[lq ? lq[p] : s1 + p];
      if (bp < 0 || v > bv || (v == bv && id < bi)) {
        bv = v;
        bi = id;
        bp = p;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o);
      const int32_t oi = __shfl_xor(bi, o), op = __shfl_xor(bp, o);
      if (op >= 0 && (bp < 0 || ov > bv || (ov == bv && oi < bi))) {
        bv = ov;
        bi = oi;
        bp = op;
      }
    }
    if (lane == 0) {
      out[t] = bp >= 0 ? bi : -1;
      if (bp >= 0) r64[bp] = -INFINITY;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// Exact routing from approximate layer-1 scores with a rigorous error bound,
// in two kernels.  Window entry p (0 <= p < len1) is layer-1 position pos(p)
// = lst[q lcap + p] with a union list, else s1 + p; its approximate score is
// rs[q rstride + pos(p)] for dense score rows (every centroid scored), else
// rs[q rstride + p].  Each approximate score is within E = ecoef |q| max|mu|
// + eadd + esub (|q| + max|mu|) (the last two for underflow) of the exact
// inner product.  Every centroid of the
// exact top c has an approximate score of at least T - 2E, T the c-th largest
// approximate score (the c best approximate scores bound the c-th best exact
// score from below by T - E), so the exact top c lies among the candidates
// above that threshold.
//
// route_filter_kernel, one wave per query: T, then the candidates.  Exactly c
// candidates: they are the routed set (written directly, rcnt = 0).  More: the
// candidates' positions go to rcand[q kCandCap ..] and rcnt[q] = their count,
// or kCandCap + 1 when they do not fit or are fewer than c (the whole window
// is then rescored).
// R: approximate scores kept in registers per lane (len1 <= 64 R), else
// re-read.

template <int R>
__global__ __launch_bounds__(256) void route_filter_kernel(
    int32_t d, int64_t nq, const int32_t* __restrict__ l1_order32,
    const int32_t* __restrict__ l1, int32_t wst, const int32_t* __restrict__ lst, int32_t lcap,
    const float* __restrict__ rs, int32_t rstride, int dense, const float* __restrict__ qnorm,
    const float* __restrict__ cent_norm_max, double ecoef, double eadd, double esub, int32_t c,
    int32_t* __restrict__ rcand, int32_t* __restrict__ rcnt, int32_t* __restrict__ routed,
    int whole) {
  __shared__ int32_t cpos[4][kCandCap];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));  // uniform
  const uint64_t below = (uint64_t(1) << lane) - 1;
  // one query per wave, no loop (per-query index arithmetic is not hoisted
  // into registers held across queries)
  const int64_t q = int64_t(blockIdx.x) * 4 + wave;
  if (q >= nq) return;
  const float* rsq = rs + q * rstride;
  // whole: every query's window is the whole dense row [0, rstride), so the
  // score loads are issued before the window is read
  float v[R > 0 ? R : 1];
  if (R > 0 && whole) {
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = rsq[uint32_t(min(lane + 64 * j, rstride - 1))];
  }
  const float qn = qnorm[q], cmax = *cent_norm_max;
  const int32_t s1 = l1[wst * q + 1], len1 = l1[wst * q + 2];
  const int32_t* lq = lst ? lst + q * lcap : nullptr;
  auto pos_of = [&](int p) { return lq ? lq[p] : s1 + p; };
  auto score_at = [&](int p) { return rsq[dense ? pos_of(p) : p]; };
  if (len1 <= c) {  // every window entry is routed
    for (int t = lane; t < c; t += 64) routed[q * c + t] = t < len1 ? l1_order32[pos_of(t)] : -1;
    if (lane == 0) rcnt[q] = 0;
    return;
  }
  if (R > 0 && !whole) {
    // all loads of a kind issued together (an index past the window re-reads
    // its last entry; those lanes are masked below)
    if (lq && dense) {
      int32_t pp[R > 0 ? R : 1];
#pragma unroll
      for (int j = 0; j < R; ++j) pp[j] = lq[min(lane + 64 * j, len1 - 1)];
#pragma unroll
      for (int j = 0; j < R; ++j) v[j] = rsq[pp[j]];
    } else {
      const int32_t o0 = dense ? s1 : 0;
#pragma unroll
      for (int j = 0; j < R; ++j) v[j] = rsq[o0 + min(lane + 64 * j, len1 - 1)];
    }
  }
  // T: the c-th largest approximate score (c rounds of a wave minimum over
  // score keys; the index part keeps equal scores apart)
  uint64_t prev = 0;
  for (int t = 0; t < c; ++t) {
    uint64_t best = ~uint64_t(0);
    if (R > 0) {
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int p = lane + 64 * j;
        const uint64_t key = (uint64_t(score_key(v[j])) << 32) | uint32_t(p);
        if (p < len1 && (t == 0 || key > prev) && key < best) best = key;
      }
    } else {
      for (int p = lane; p < len1; p += 64) {
        const uint64_t key = (uint64_t(score_key(score_at(p))) << 32) | uint32_t(p);
        if ((t == 0 || key > prev) && key < best) best = key;
      }
    }
    prev = wave_min_u64(best);
  }
  const double E = ecoef * double(qn) * double(cmax) + eadd + esub * (double(qn) + double(cmax));
  const double thr = double(key_score(uint32_t(prev >> 32))) - 2.0 * E;
  // candidates in window order: their window entries in LDS (positions are
  // looked up only for them)
  int n = 0;
  const int nchunk = (len1 + 63) / 64;
  for (int jc = 0; jc < nchunk; ++jc) {
    const int p = jc * 64 + lane;
    float sv = 0.f;
    if (R > 0) {
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (j == jc) sv = v[j];
    } else if (p < len1) {
      sv = score_at(p);
    }
    const bool in = p < len1 && double(sv) >= thr;
    const uint64_t m = __ballot(in);
    const int slot = n + __popcll(m & below);
    if (in && slot < kCandCap) cpos[wave][slot] = p;
    n += __popcll(m);
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  if (n == c) {  // the candidates are the routed set (listed in window order)
    for (int t = lane; t < c; t += 64) routed[q * c + t] = l1_order32[pos_of(cpos[wave][t])];
    if (lane == 0) rcnt[q] = 0;
  } else {
    int32_t* cq = rcand + q * kCandCap;
    const int nl = min(n, kCandCap);
    for (int t = lane; t < nl; t += 64) cq[t] = pos_of(cpos[wave][t]);
    // fewer than c candidates only with non-finite scores (a query holding a
    // NaN or an infinity): the whole window is then decided sequentially,
    // which routes c valid clusters (or -1) whatever the scores
    if (lane == 0) rcnt[q] = (n > kCandCap || n < c) ? kCandCap + 1 : n;
  }
}

// route_rescore_kernel, one wave per query with rcnt[q] > 0.  Each
// candidate's FP64 inner product is summed in parallel (the products are
// exact in FP64) by a group of 16 lanes, four candidates at a time; two FP64
// sums of the same d terms in different orders differ by at most
// 2 (d-1) 2^-53 sum|p| (to first order), so with the band 8 d 2^-53 sum|p|
// around each value, the top c by parallel value are the exact top c whenever
// every chosen band lies above every other band.  Otherwise, and when the
// candidates did not fit (then the whole window), one lane per centroid sums
// the FP64 inner product sequentially in dimension order (the definition) and
// the top c by (score desc, cluster id asc) are taken.
constexpr int kRescoreSteps = 16;  // float4 steps per lane of the fast path: d <= 1024
// one wave per workgroup: a query that needs no rescoring frees its slot at
// once instead of waiting for three busy neighbours
constexpr int kRescoreWaves = 1;

__global__ __launch_bounds__(64 * kRescoreWaves) void route_rescore_kernel(
    const float* __restrict__ Q, int32_t d, int64_t nq, const float* __restrict__ cent_l1,
    const int32_t* __restrict__ l1_order32, const int32_t* __restrict__ l1, int32_t wst,
    const int32_t* __restrict__ lst, int32_t lcap, int32_t c, const int32_t* __restrict__ rcand,
    const int32_t* __restrict__ rcnt, double* __restrict__ rs64, int32_t* __restrict__ routed) {
  __shared__ float sq[kRescoreWaves][64 * kRescoreSteps] __attribute__((aligned(16)));
  __shared__ double clo[kRescoreWaves][kCandCap], chi[kRescoreWaves][kCandCap];
  __shared__ int32_t cid[kRescoreWaves][kCandCap];
  __shared__ uint8_t cpick[kRescoreWaves][kCandCap];
  __shared__ int32_t chosen[kRescoreWaves][LIDER_MAX_C];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const double u = 1.1102230246251565e-16;  // 2^-53
  const bool fast = (d & 3) == 0 && d <= 64 * kRescoreSteps &&
                    ((reinterpret_cast<uintptr_t>(Q) | reinterpret_cast<uintptr_t>(cent_l1)) & 15) == 0;
  for (int64_t q = int64_t(blockIdx.x) * kRescoreWaves + wave; q < nq;
       q += int64_t(gridDim.x) * kRescoreWaves) {
    const int32_t n = rcnt[q];
    if (n == 0) continue;  // decided by the filter (wave-uniform)
    const float* qv = Q + q * d;
    const int32_t* cq = rcand + q * kCandCap;
    if (n > kCandCap) {
      const int32_t s1 = l1[wst * q + 1], len1 = l1[wst * q + 2];
      route_fp64_wave(qv, d, cent_l1, l1_order32, s1, len1, lst ? lst + q * lcap : nullptr, c,
                      rs64 + q * lcap, chosen[wave]);
      for (int t = lane; t < c; t += 64) routed[q * c + t] = chosen[wave][t];
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    // lane j of group g: dims 4 j + 64 i (fast path, query staged in LDS) or
    // j + 16 i
    if (fast) {  // zero beyond d: those products must be exact zeros
      for (int k = 4 * lane; k < 64 * kRescoreSteps; k += 256)
        *reinterpret_cast<float4*>(&sq[wave][k]) =
            k < d ? *reinterpret_cast<const float4*>(qv + k) : float4{0.f, 0.f, 0.f, 0.f};
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
    }
    for (int t0 = 0; t0 < n; t0 += 4) {
      const int t = t0 + g;
      const float* mu = cent_l1 + int64_t(cq[min(t, n - 1)]) * d;
      double ps = 0.0, pa = 0.0;
      if (fast) {
        // the row through a buffer resource: reads past d return zeros
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(mu), 0, d * 4, kBufWord3);
        float4 m[kRescoreSteps];  // every load of the row in flight at once
#pragma unroll
        for (int i = 0; i < kRescoreSteps; ++i) {
          const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, (4 * j + 64 * i) * 4, 0, 0);
          m[i] = float4{__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                        __uint_as_float(v[3])};
        }
#pragma unroll
        for (int i = 0; i < kRescoreSteps; ++i) {
          const float4 x = *reinterpret_cast<const float4*>(&sq[wave][4 * j + 64 * i]);
          const double p0 = double(x.x) * double(m[i].x), p1 = double(x.y) * double(m[i].y);
          const double p2 = double(x.z) * double(m[i].z), p3 = double(x.w) * double(m[i].w);
          ps += p0;
          ps += p1;
          ps += p2;
          ps += p3;
          pa += fabs(p0);
          pa += fabs(p1);
          pa += fabs(p2);
          pa += fabs(p3);
        }
      } else {
        for (int k = j; k < d; k += 16) {
          const double pr = double(qv[k]) * double(mu[k]);
          ps += pr;
          pa += fabs(pr);
        }
      }
      for (int o = 8; o > 0; o >>= 1) {  // within the 16-lane group
        ps += __shfl_xor(ps, o);
        pa += __shfl_xor(pa, o);
      }
      if (j == 0 && t < n) {
        const double band = 8.0 * double(d) * u * pa;
        clo[wave][t] = ps - band;
        chi[wave][t] = ps + band;
        cid[wave][t] = l1_order32[cq[t]];
        cpick[wave][t] = 0;
      }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    // top c by parallel value (band midpoint), ties to the smaller cluster id:
    // a candidate's place is the number of candidates ahead of it in that order
    // (a NaN midpoint counts as -inf, so the order stays total)
    const auto mid = [&](int t) {
      const double v = 0.5 * (clo[wave][t] + chi[wave][t]);
      return v == v ? v : -INFINITY;
    };
    for (int t = lane; t < n; t += 64) {
      const double v = mid(t);
      const int32_t id = cid[wave][t];
      int32_t place = 0;
#pragma unroll 4
      for (int s = 0; s < n; ++s) {
        const double vs = mid(s);
        place += (vs > v || (vs == v && cid[wave][s] < id)) ? 1 : 0;
      }
      cpick[wave][t] = place < c;
      if (place < c) chosen[wave][place] = id;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    // decided when every chosen band lies above every other band
    double lo = INFINITY, hi = -INFINITY;
    for (int t = lane; t < n; t += 64) {
      if (cpick[wave][t])
        lo = fmin(lo, clo[wave][t]);
      else
        hi = fmax(hi, chi[wave][t]);
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, o));
      hi = fmax(hi, __shfl_xor(hi, o));
    }
    if (!(lo > hi))
      route_fp64_wave(qv, d, cent_l1, l1_order32, 0, n, cq, c, rs64 + q * lcap, chosen[wave]);
    for (int t = lane; t < c; t += 64) routed[q * c + t] = chosen[wave][t];
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}


// ------------------------------------------------------------ layer 2 pairs
// The per-cluster pair counts and scatter cursors are kept in kCntCopies
// copies (copy x of cluster j at x C + j), pair t using copy (t / 256) % 8:
// at c = 8 about 80 pairs of 10,000 queries hit each of 1,000 clusters, and
// the atomics on one address queue behind each other; the copies shorten
// each queue eightfold.  A cluster's pairs stay contiguous in the work list,
// copy by copy.

__device__ inline int cnt_copy(int64_t t) { return int((t >> 8) & (kCntCopies - 1)); }

__device__ inline int32_t cluster_count(const int32_t* __restrict__ cnt, int32_t C, int32_t j) {
  int32_t v = 0;
#pragma unroll
  for (int x = 0; x < kCntCopies; ++x) v += cnt[int64_t(x) * C + j];
  return v;
}

// Work-list slot of pair t of cluster j (first slot of the cluster: s0): the
// counts of the copies before t's, then t's place in its own copy.
__device__ inline int32_t copy_slot(const int32_t* __restrict__ cnt, int32_t* __restrict__ fill,
                                    int32_t C, int64_t t, int32_t j, int32_t s0) {
  const int x0 = cnt_copy(t);
  int32_t o = s0;
  for (int x = 0; x < x0; ++x) o += cnt[int64_t(x) * C + j];
  return o + atomicAdd(&fill[int64_t(x0) * C + j], 1);
}

// One thread per (query, routed cluster) pair t.  One array: pairs[t] is the
// window.  H arrays: pw[t H + h] is array h's window (positions of array h)
// and pairs[t] gets the union's hull later (pair_mask_kernel).
__global__ void pairs_kernel(const Model* __restrict__ models, const double* __restrict__ leaves,
                             const int32_t* __restrict__ qdig, int32_t m, int32_t H, int32_t C,
                             int64_t np, int32_t c, int32_t r,
                             const int32_t* __restrict__ routed, Pair* __restrict__ pairs,
                             Pair* __restrict__ pw, int32_t* __restrict__ ccount,
                             uint64_t* __restrict__ kq) {
  // one thread per (pair, array): the H locates of a pair run side by side
  const int64_t u = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (u >= np * H) return;
  const int64_t t = u / H;
  const int32_t h = int32_t(u - t * H);
  const int64_t q = t / c;
  const int32_t j = routed[t];
  Pair ph{-1, 0, 0, 0};
  if (j >= 0) {
    const Model* Mp = models + int64_t(h) * (C + 1) + j;
    const int64_t L = Mp->L;
    uint64_t K = 0;
    const int64_t pos =
        locate(Mp, leaves, qdig + q * 2 * H * m + int64_t(H) * m + int64_t(h) * m, m, &K);
    int64_t s, len;
    window_of(pos, r, L, &s, &len);  // the expansion (if any) replaces s later
    if (kq) kq[t * H + h] = K;
    ph = Pair{j, int32_t(s), int32_t(len), int32_t(pos)};
  }
  if (pw) pw[t * H + h] = ph;
  if (h == 0) {
    if (j >= 0 && ph.len > 0) atomicAdd(&ccount[cnt_copy(t) * C + j], 1);
    pairs[t] = ph;
  }
}

// Block -> tile map of the direct schedules.  Workgroups go to the 8 XCDs
// round-robin (XCD blockIdx % 8); the tiles are cut into chunks of S
// consecutive tiles (about 8,192 rows), chunk k belongs to XCD k % 8, and an
// XCD runs its chunks in order.  Consecutive tiles -- the same clusters, the
// same query rows -- share one XCD's L2, while every XCD gets chunks from all
// over the index: with one contiguous eighth of the tiles per XCD, a
// clustering that numbers its busiest clusters together left one XCD with most
// of the work (1M x 768, c = 8, r = 256: 1.04 ms against 0.81 ms for the same
// clusters in another order).  Grid: 8 S ceil(ceil(ntiles / S) / 8) blocks.
__device__ inline int32_t xcd_chunk_tile(int32_t ntiles, int32_t S) {
  const int32_t xcd = int32_t(blockIdx.x & 7), loc = int32_t(blockIdx.x >> 3);
  const int32_t t = (xcd + 8 * (loc / S)) * S + loc % S;
  return t < ntiles ? t : -1;
}

__host__ __device__ constexpr int32_t tile_chunk(int32_t rows_per_tile) {
  return 8192 / rows_per_tile;
}

inline unsigned chunk_grid(int32_t ntiles, int32_t S) {
  const int32_t nch = (ntiles + S - 1) / S;
  return unsigned(8 * ((nch + 7) / 8) * S);
}

// Pairs per pair-mask workgroup run dealt to one XCD: 4 x 64.
constexpr int32_t kMaskChunk = 64;
// Copies of a pair's LDS bitmap in the pair masks (a power of two): eight or
// four while the 4 waves' copies stay within 24 KB.
__host__ __device__ inline int32_t mask_copies(int32_t mw) {
  return mw <= 192 ? 8 : mw <= 384 ? 4 : 1;
}
// Map segments (8 entries) per lane in flight in the pair masks (8, one
// round for the 297 segments of nine windows of 256 entries, was no faster).
constexpr int kMaskSegs = 4;

// Union of a pair's H windows (several arrays): one wave per pair sets the
// rows (positions of array 0 within the cluster; array h's positions go
// through amap16) in an LDS bitmap of mw words, stores the bitmap as the
// pair's membership mask [mw words] and sets pairs[t] to the hull [first,
// last] of the union.  The bitmap has mask_copies(mw) copies at a stride of
// mw + 1 words (dynamic shared memory, 4 waves x copies x (mw + 1) words):
// lane l marks copy l % copies, so fewer lanes of one atomic instruction hit
// the same word, and the copies are ORed when the mask is stored.
__global__ __launch_bounds__(256) void pair_mask_kernel(
    const Pair* __restrict__ pw, int32_t H, const int32_t* __restrict__ wl,
    const int32_t* __restrict__ wl_end, const int64_t* __restrict__ off,
    const uint16_t* __restrict__ amap16, int64_t n, int32_t mw, Pair* __restrict__ pairs,
    uint32_t* __restrict__ mask, int32_t nblk) {
  extern __shared__ uint32_t bm_all[];
  __shared__ int64_t sea[4][LIDER_MAX_H];  // per wave and array: first map entry read
  __shared__ int32_t slead[4][LIDER_MAX_H], sspan[4][LIDER_MAX_H], sx[4][LIDER_MAX_H];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t nc = mask_copies(mw), nbw = nc * (mw + 1);  // copies, words per wave
  uint32_t* bm = bm_all + wave * nbw;
  uint32_t* mine = bm + (lane & (nc - 1)) * (mw + 1);  // this lane's copy
  // pairs in work-list order, 4 per workgroup, runs of kMaskChunk
  // workgroups dealt to the XCDs in turn: the pairs of a cluster go to one
  // XCD, whose L2 then holds the cluster's position maps
  const int64_t nwl = *wl_end;
  const int32_t blk = xcd_chunk_tile(nblk, kMaskChunk);
  const int64_t u = int64_t(blk) * 4 + wave;
  if (blk >= 0 && u < nwl) {
    const int64_t t = wl[u];
    // the pair's H windows, one per lane (H <= 16), read with one load
    Pair myw{-1, 0, 0, 0};
    if (lane < H) myw = pw[t * H + lane];
    const int32_t j = __shfl(myw.j, 0);
    if (j < 0) return;  // wave-uniform
    const int64_t o = off[j];
    // array 0's window is a range of positions: whole words
    const int32_t s0 = __shfl(myw.s, 0), e0 = s0 + __shfl(myw.len, 0);
    for (int32_t w = lane; w < nbw; w += 64) bm[w] = w < mw ? range_bits(w, s0, e0) : 0u;
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    // the other arrays' window positions mapped to array 0's, in segments of 8
    // consecutive map entries (16 bytes; an array's first segment starts at
    // its window's first entry rounded down to a multiple of 8).  The
    // segments of all H - 1 arrays are numbered in array order and dealt over
    // the lanes, kMaskSegs per lane in flight, so every lane has work whatever
    // the window lengths (one array's window of 256 entries is 33 segments).
    // Lane h (1 <= h < H) sets up array h: map address, lead, span.
    int32_t nseg = 0;
    if (lane >= 1 && lane < H) {
      const int64_t e = int64_t(lane - 1) * n + o + myw.s;
      const int64_t ea = e & ~int64_t(7);
      const int32_t lead = int32_t(e - ea);
      const int32_t span = myw.len > 0 ? lead + myw.len : 0;  // entries from ea through the end
      nseg = (span + 7) >> 3;
      sea[wave][lane] = ea;
      slead[wave][lane] = lead;
      sspan[wave][lane] = span;
    }
    int32_t incl = nseg;  // inclusive prefix of the segment counts over lanes 0..15
#pragma unroll
    for (int o2 = 1; o2 < LIDER_MAX_H; o2 <<= 1) {
      const int32_t y = __shfl_up(incl, o2);
      if (lane >= o2) incl += y;
    }
    if (lane < LIDER_MAX_H) sx[wave][lane] = incl - nseg;  // first segment of array lane
    const int32_t total = __shfl(incl, LIDER_MAX_H - 1);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    for (int32_t g0 = 0; g0 < total; g0 += 64 * kMaskSegs) {
      uint4 v[kMaskSegs];
      int32_t hh[kMaskSegs], cc[kMaskSegs];
#pragma unroll
      for (int u = 0; u < kMaskSegs; ++u) {
        const int32_t g = g0 + 64 * u + lane;
        hh[u] = 1;
        cc[u] = 0;
        v[u] = make_uint4(0u, 0u, 0u, 0u);
        if (g < total) {
          // the array holding segment g: the last one starting at or before g
          // (arrays without segments start where the next one does)
          int32_t h = 1;
          for (int32_t x = 2; x < H; ++x)
            if (sx[wave][x] <= g) h = x;
          hh[u] = h;
          cc[u] = 8 * (g - sx[wave][h]);  // < span: inside the allocation's padding at most
          v[u] = *reinterpret_cast<const uint4*>(amap16 + sea[wave][h] + cc[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < kMaskSegs; ++u) {
        if (g0 + 64 * u + lane >= total) continue;
        const int32_t lead = slead[wave][hh[u]], span = sspan[wave][hh[u]];
        const uint32_t wd[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int32_t c = cc[u] + k;
          const uint32_t row = (wd[k >> 1] >> (16 * (k & 1))) & 0xffffu;
          if (c >= lead && c < span) atomicOr(&mine[row >> 5], 1u << (row & 31));
        }
      }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    int32_t lo = INT32_MAX, hi = -1;
    for (int32_t w = lane; w < mw; w += 64) {
      uint32_t bits = bm[w];
      for (int32_t k = 1; k < nc; ++k) bits |= bm[k * (mw + 1) + w];
      mask[t * mw + w] = bits;
      if (bits) {
        lo = min(lo, w * 32 + __builtin_ctz(bits));
        hi = max(hi, w * 32 + 31 - __builtin_clz(bits));
      }
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
      lo = min(lo, __shfl_xor(lo, o2));
      hi = max(hi, __shfl_xor(hi, o2));
    }
    if (lane == 0) {
      pairs[t].s = hi >= lo ? lo : 0;
      pairs[t].len = hi >= lo ? hi - lo + 1 : 0;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// dist_e-guided bi-directional expansion (Sections 3.3.1, 4.2), one wave per
// item (a query's layer-1 window, or a (query, cluster) pair).  From the
// predicted location the range grows one position at a time on the side whose
// next hashkey is closer to the query's in dist_e (ties to the left, the other
// side once one is exhausted) until min(r, L) positions are taken.  The wave
// scores the next 64 candidates of a side at once into LDS; lane 0 runs the
// sequential two-pointer decisions over them and the exhausted side is
// refilled.  Only the window start changes (the length is min(r, L)).
// Item t belongs to hashkey array h = t % H, whose keys start at
// keys + h * kstride.  Layer 1: items are (query, array) windows, the array is
// the centroids retriever's keys (L = C) and the l1 rows are updated too; else
// items are (pair, array) windows and the array of cluster j starts at off[j].
constexpr int64_t kNoDist = INT64_MAX;

__global__ __launch_bounds__(256) void expand_kernel(const uint64_t* __restrict__ keys,
                                                     const int64_t* __restrict__ off, int64_t L1,
                                                     Pair* __restrict__ items, int64_t nitems,
                                                     const uint64_t* __restrict__ kq, int32_t r,
                                                     int32_t m, int32_t B,
                                                     int32_t* __restrict__ l1, int32_t H,
                                                     int64_t kstride) {
  __shared__ int64_t dl[4][64], dr[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t t = int64_t(blockIdx.x) * 4 + wave;
  if (t >= nitems) return;
  const Pair pr = items[t];
  if (pr.j < 0 || pr.len <= 0) return;
  const uint64_t* kh = keys + (t % H) * kstride;
  const uint64_t* ka = off ? kh + off[pr.j] : kh;
  const int64_t L = off ? off[pr.j + 1] - off[pr.j] : L1;
  const int64_t take = pr.len;  // = min(r, L)
  const uint64_t Kq = kq[t];
  int64_t lo = pr.pos - 1, hi = pr.pos + 1, got = 1;
  int il = 64, ir = 64;
  while (got < take) {
    if (il == 64) {
      const int64_t p = lo - lane;
      dl[wave][lane] = p >= 0 ? dist_e_scaled(ka[p], Kq, m, B) : kNoDist;
      il = 0;
    }
    if (ir == 64) {
      const int64_t p = hi + lane;
      dr[wave][lane] = p < L ? dist_e_scaled(ka[p], Kq, m, B) : kNoDist;
      ir = 0;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      while (got < take && il < 64 && ir < 64) {
        const int64_t a = dl[wave][il], b = dr[wave][ir];
        if (a != kNoDist && (b == kNoDist || a <= b)) {
          ++il;
          --lo;
        } else {
          ++ir;
          ++hi;
        }
        ++got;
      }
    }
    lo = __shfl(lo, 0);
    hi = __shfl(hi, 0);
    got = __shfl(got, 0);
    il = __shfl(il, 0);
    ir = __shfl(ir, 0);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0) {
    items[t].s = int32_t(lo + 1);
    if (l1) l1[3 * t + 1] = int32_t(lo + 1);
  }
}

// Exclusive scan of per-cluster pair counts (single workgroup).
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ cnt, int32_t C,
                                                    int32_t* __restrict__ start) {
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  const int per = (C + 1023) / 1024;
  const int a = tid * per, e = min(C, a + per);
  int32_t s = 0;
  for (int i = a; i < e; ++i) s += cluster_count(cnt, C, i);
  part[tid] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid ? part[tid - 1] : 0;
  for (int i = a; i < e; ++i) {
    start[i] = run;
    run += cluster_count(cnt, C, i);
  }
  if (tid == 1023) start[C] = part[1023];
}

__global__ void scatter_kernel(const Pair* __restrict__ pairs, int64_t np,
                               const int32_t* __restrict__ cnt, int32_t C,
                               const int32_t* __restrict__ start, int32_t* __restrict__ fill,
                               int32_t* __restrict__ wl) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const Pair pr = pairs[t];
  if (pr.j < 0 || pr.len <= 0) return;
  wl[copy_slot(cnt, fill, C, t, pr.j, start[pr.j])] = int32_t(t);
}

// scan_kernel + scatter_kernel in one launch for C <= kFusedScanMax: every
// workgroup scans the cluster counts itself in LDS (they are few), workgroup 0
// also writes start[0..C], then each scatters its 256 pairs.
constexpr int kFusedScanMax = 8192;

__global__ __launch_bounds__(256) void scan_scatter_kernel(const int32_t* __restrict__ cnt,
                                                           int32_t C, const Pair* __restrict__ pairs,
                                                           int64_t np, int32_t* __restrict__ start,
                                                           int32_t* __restrict__ fill,
                                                           int32_t* __restrict__ wl) {
  __shared__ int32_t st[kFusedScanMax + 1];
  __shared__ int32_t part[256];
  const int tid = threadIdx.x;
  const int per = (C + 255) / 256;
  const int a = tid * per, e = min(C, a + per);
  int32_t sum = 0;
  for (int i = a; i < e; ++i) {
    const int32_t v = cluster_count(cnt, C, i);
    st[i] = v;
    sum += v;
  }
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int32_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = tid ? part[tid - 1] : 0;
  for (int i = a; i < e; ++i) {
    const int32_t v = st[i];
    st[i] = run;
    run += v;
  }
  if (tid == 255) st[C] = part[255];
  __syncthreads();
  if (blockIdx.x == 0)
    for (int i = tid; i <= C; i += 256) start[i] = st[i];
  const int64_t t = int64_t(blockIdx.x) * 256 + tid;
  if (t >= np) return;
  const Pair pr = pairs[t];
  if (pr.j < 0 || pr.len <= 0) return;
  wl[copy_slot(cnt, fill, C, t, pr.j, st[pr.j])] = int32_t(t);
}

// Active-tile work list: every pair marks the tiles its window overlaps; the
// first marker of a tile appends it to the list (order unspecified; each
// tile's result does not depend on the order).
__global__ void mark_tiles_kernel(const Pair* __restrict__ pairs, int64_t np, int32_t RT,
                                  const int32_t* __restrict__ tile_base,
                                  int32_t* __restrict__ flag, int32_t* __restrict__ alist,
                                  int32_t* __restrict__ count) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const Pair pr = pairs[t];
  if (pr.j < 0 || pr.len <= 0) return;
  const int32_t b = tile_base[pr.j];
  for (int32_t u = b + pr.s / RT; u <= b + (pr.s + pr.len - 1) / RT; ++u)
    if (atomicExch(&flag[u], 1) == 0) alist[atomicAdd(count, 1)] = u;
}

// ------------------------------------------------------------ rerank
// Per-wave list of the pairs overlapping the wave's current tile.  The pairs
// of the tile's cluster are tested 64 at a time (one ballot round); hits are
// appended until a whole pass (CAP - 64 pairs) is listed, so a round may
// overshoot by up to 63 entries, which carry over to the next pass.
constexpr int kWavePairCap = 64;

template <int CAP>
struct WaveShared {
  int32_t lp[CAP], lq[CAP], ls[CAP], le[CAP];
  uint32_t lm[CAP][4];  // membership bits of the tile's rows (several arrays)
  uint32_t bk[CAP][4];  // block keys of the pass's pairs (32-row blocks of the tile)
};

// Tile fetch, one tile per wave (direct: persistent = 0), one workgroup per
// wave.
__device__ inline int32_t direct_tile(int32_t ntiles, int32_t S) {
  return xcd_chunk_tile(ntiles, S);
}

// Persistent fetch state of one wave.
struct FetchState {
  int32_t v = 0;              // exhausted per-XCD ranges (persistent = 1)
  int32_t cur = 0, end = 0;   // current chunk of tiles (persistent = 1)
  int32_t k = 0;              // list entries taken so far (persistent = 2)
};
constexpr int kFetchChunk = 8;

// Persistent fetch of the wave's next tile.  persistent = 1 (called by lane 0):
// the index's tiles are split into 8 contiguous ranges, one per XCD, each
// drained in chunks of kFetchChunk tiles through its own atomic counter
// (ctr[0..7]; one device-scope atomic per chunk, not per tile); a wave starts
// on its own XCD's range and steals from the others once it is empty.
// persistent = 2: the device-built list of active tiles (ctr[8] entries) is
// dealt to the grid's waves round-robin, without atomics.
__device__ inline int32_t fetch_tile(int persistent, int32_t ntiles, int32_t* __restrict__ ctr,
                                     FetchState& st, const int32_t* __restrict__ alist) {
  if (persistent == 2) {
    const int64_t W = int64_t(gridDim.x) * (blockDim.x >> 6);
    const int64_t idx = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6) + st.k * W;
    ++st.k;
    return idx < ctr[8] ? alist[idx] : -1;
  }
  if (st.cur < st.end) return st.cur++;
  const int32_t per = (ntiles + 7) / 8;
  const int32_t home = blockIdx.x & 7;
  for (; st.v < 8; ++st.v) {
    const int32_t x = (home + st.v) & 7;
    const int32_t lo = x * per, hi = min(ntiles, lo + per);
    if (lo >= hi) continue;
    const int32_t t = lo + atomicAdd(&ctr[x], kFetchChunk);
    if (t < hi) {
      st.cur = t + 1;
      st.end = min(hi, t + kFetchChunk);
      return t;
    }
  }
  return -1;
}

// Rerank of one tile per wave: RT consecutive rows of one cluster (contiguous
// in the reordered corpus) against every (query, cluster) pair whose window
// overlaps the tile.  The wave streams its rows once over the whole dimension
// range and accumulates RT rows x up to 16 * NPCM pairs on MFMA (fp32:
// v_mfma_f32_16x16x4f32, one float4 of both operands feeds 4 MFMAs; bf16:
// v_mfma_f32_16x16x32_bf16, 8 consecutive bf16 per lane), then writes each
// finished score from its accumulator straight into the pair's window score
// row (16 consecutive rows per store).  A workgroup is one wave: no
// cross-wave reduction or barrier, and a wave that finishes early frees its
// slot for the next tile at once (a workgroup of 4 tiles held all 4 slots
// until its slowest tile was done: 2-10 % slower).  A score is one
// accumulator summed over the k-steps in order, so results do not depend on
// the tile size, the schedule or which other pairs share a pass.
constexpr int kRerankNT = 64;  // threads per rerank workgroup (one wave)

// A wave-uniform value, moved to a scalar register.
__device__ inline int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// Operand feeds.  FMT 0: fp32 rows and queries; 1: bf16 rows and queries;
// 2: fp8 e4m3 rows (decoded exactly to bf16) and bf16 queries; 3 / 4: fp32 /
// bf16 with two 16-byte loads per lane and row per k-step, 64 bytes apart, so
// the 4 lanes of a row cover one whole 128-byte line of it per step (the
// streamed corpus feeds: a line is requested by two instructions issued back
// to back instead of by two consecutive k-steps).  Lane slot s covers the
// dimensions [SUBW*s, SUBW*s + SUBW) of the first load and the same range
// plus KS/2 of the second.
enum { kF32 = 0, kBF16 = 1, kFP8 = 2, kF32W = 3, kBF16W = 4 };

template <int FMT, bool VEC>
struct Feed;

// Rows streamed once per launch are loaded with the non-temporal hint.
template <class T>
__device__ inline T stream_load(const T* p, bool nt) {
  return nt ? __builtin_nontemporal_load(p) : *p;
}

// VEC = 16-byte loads; for fp32 VEC also means d % 16 == 0 (every k-step is
// full), so loads carry no bounds branch and the k-loop pipelines.
template <bool VEC>
struct Feed<kF32, VEC> {  // 16 dims per k-step, 4 per lane
  static constexpr int KS = 16, SUBW = 4;
  typedef float XE;
  typedef float QE;
  typedef float4 T;
  __device__ static T load(const float* row, int k, int d) {
    if (VEC) return *reinterpret_cast<const float4*>(row + k);
    float4 v;
    v.x = k < d ? row[k] : 0.f;
    v.y = k + 1 < d ? row[k + 1] : 0.f;
    v.z = k + 2 < d ? row[k + 2] : 0.f;
    v.w = k + 3 < d ? row[k + 3] : 0.f;
    return v;
  }
  __device__ static T loadx(const float* row, int k, int d, bool nt) {
    if (VEC) {
      const floatx4 v = stream_load(reinterpret_cast<const floatx4*>(row + k), nt);
      return float4{v[0], v[1], v[2], v[3]};
    }
    return load(row, k, d);
  }
  typedef T Raw;
  __device__ static Raw raw(const float* row, int k, int d, bool nt) { return loadx(row, k, d, nt); }
  __device__ static T dec(const Raw& v, int, int) { return v; }
  __device__ static void mfma(const T& q, const T& x, floatx4& acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.x, x.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.y, x.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.z, x.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.w, x.w, acc, 0, 0, 0);
  }
};

__device__ inline bf16x8 bf16x8_zero() {
  bf16x8 z;
#pragma unroll
  for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.f;
  return z;
}

// bf16 / fp8 feeds need d % 8 == 0; VEC additionally means d % 32 == 0.  A
// partial last k-step reads a clamped in-bounds address and zeroes the value
// (no branch around the load).
template <bool VEC>
struct Feed<kBF16, VEC> {  // 32 dims per k-step, 8 per lane
  static constexpr int KS = 32, SUBW = 8;
  typedef __hip_bfloat16 XE;
  typedef __hip_bfloat16 QE;
  typedef bf16x8 T;
  __device__ static T load(const __hip_bfloat16* row, int k, int d) {
    if (VEC) return *reinterpret_cast<const bf16x8*>(row + k);
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(row + (k < d ? k : d - 8));
    return k < d ? v : bf16x8_zero();
  }
  __device__ static T loadx(const __hip_bfloat16* row, int k, int d, bool nt) {
    if (VEC) return stream_load(reinterpret_cast<const bf16x8*>(row + k), nt);
    return load(row, k, d);
  }
  typedef T Raw;
  __device__ static Raw raw(const __hip_bfloat16* row, int k, int d, bool nt) {
    return loadx(row, k, d, nt);
  }
  __device__ static T dec(const Raw& v, int, int) { return v; }
  __device__ static void mfma(const T& q, const T& x, floatx4& acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q, x, acc, 0, 0, 0);
  }
};

// Decode one OCP fp8 e4m3 byte (exact in fp32 and in bf16).
__device__ inline float e4m3_value(uint8_t v) {
  const int e = (v >> 3) & 15, mnt = v & 7;
  float a = e == 0 ? float(mnt) * 0.001953125f : ldexpf(1.f + float(mnt) * 0.125f, e - 7);
  if (e == 15 && mnt == 7) a = __uint_as_float(0x7fc00000u);
  return (v & 0x80) ? -a : a;
}

template <bool VEC>
struct Feed<kFP8, VEC> {  // fp8 rows, bf16 queries, 32 dims per k-step
  static constexpr int KS = 32, SUBW = 8;
  typedef uint8_t XE;
  typedef __hip_bfloat16 QE;
  typedef bf16x8 T;
  __device__ static T load(const __hip_bfloat16* row, int k, int d) {
    return Feed<kBF16, VEC>::load(row, k, d);
  }
  typedef uint32_t Raw __attribute__((ext_vector_type(2)));  // 8 undecoded bytes
  __device__ static Raw raw(const uint8_t* row, int k, int d, bool nt) {
    const int kk = VEC ? k : (k < d ? k : d - 8);
    return stream_load(reinterpret_cast<const Raw*>(row + kk), nt);
  }
  __device__ static T dec(const Raw& rv, int k, int d) {
    T v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t w = e < 4 ? rv[0] : rv[1];
      v[e] = (__bf16)e4m3_value(uint8_t(w >> (8 * (e & 3))));
    }
    return (VEC || k < d) ? v : bf16x8_zero();
  }
  __device__ static T loadx(const uint8_t* row, int k, int d, bool nt) {
    return dec(raw(row, k, d, nt), k, d);
  }
  __device__ static void mfma(const T& q, const T& x, floatx4& acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(q, x, acc, 0, 0, 0);
  }
};

struct F32x2 {
  float4 a, b;
};

// VEC: d % 32 == 0 (every k-step is full, loads carry no bounds branch).
template <bool VEC>
struct Feed<kF32W, VEC> {  // 32 dims per k-step: 4 + 4 per lane
  static constexpr int KS = 32, SUBW = 4;
  typedef float XE;
  typedef float QE;
  typedef F32x2 T;
  typedef T Raw;
  __device__ static T load(const float* row, int k, int d) {
    return T{Feed<kF32, VEC>::load(row, k, d), Feed<kF32, VEC>::load(row, k + 16, d)};
  }
  __device__ static T loadx(const float* row, int k, int d, bool nt) {
    return T{Feed<kF32, VEC>::loadx(row, k, d, nt), Feed<kF32, VEC>::loadx(row, k + 16, d, nt)};
  }
  __device__ static Raw raw(const float* row, int k, int d, bool nt) { return loadx(row, k, d, nt); }
  __device__ static T dec(const Raw& v, int, int) { return v; }
  __device__ static void mfma(const T& q, const T& x, floatx4& acc) {
    Feed<kF32, VEC>::mfma(q.a, x.a, acc);
    Feed<kF32, VEC>::mfma(q.b, x.b, acc);
  }
};

struct BF16x2 {
  bf16x8 a, b;
};

// VEC: d % 64 == 0; otherwise d % 8 == 0 and partial steps are zero-filled.
template <bool VEC>
struct Feed<kBF16W, VEC> {  // 64 dims per k-step: 8 + 8 per lane
  static constexpr int KS = 64, SUBW = 8;
  typedef __hip_bfloat16 XE;
  typedef __hip_bfloat16 QE;
  typedef BF16x2 T;
  typedef T Raw;
  __device__ static T load(const __hip_bfloat16* row, int k, int d) {
    return T{Feed<kBF16, VEC>::load(row, k, d), Feed<kBF16, VEC>::load(row, k + 32, d)};
  }
  __device__ static T loadx(const __hip_bfloat16* row, int k, int d, bool nt) {
    return T{Feed<kBF16, VEC>::loadx(row, k, d, nt), Feed<kBF16, VEC>::loadx(row, k + 32, d, nt)};
  }
  __device__ static Raw raw(const __hip_bfloat16* row, int k, int d, bool nt) {
    return loadx(row, k, d, nt);
  }
  __device__ static T dec(const Raw& v, int, int) { return v; }
  __device__ static void mfma(const T& q, const T& x, floatx4& acc) {
    Feed<kBF16, VEC>::mfma(q.a, x.a, acc);
    Feed<kBF16, VEC>::mfma(q.b, x.b, acc);
  }
};

// Row source of a tile read in row-major order: one pointer per 16-row block
// (rows past the tile clamped to its last row).
template <class F, int RC>
struct PtrRows {
  const typename F::XE* xr[RC];
  __device__ typename F::T load(int rc, int k, int d, bool nt) const {
    return F::loadx(xr[rc], k, d, nt);
  }
};


// Rows of an operand-ordered corpus copy (fp32 with 32-dim k-steps, or bf16
// with 64-dim k-steps): the row block rc of the tile starts rc * bstride
// elements after the tile's first block, k-step ks one 2 KB chunk further
// per step; the lane's two 16-byte halves sit at 16 lane bytes into each 1 KB
// half -- each half one contiguous 1 KB wave load, read nontemporally (the
// corpus is streamed once per batch).  Row blocks past the tile's rows are
// not read (zeros).
template <class F, int RC>
struct TileRows {
  typedef typename F::XE XE;
  static constexpr int kHalf = 1024 / int(sizeof(XE));  // elements per 1 KB half
  const XE* base;     // the tile's first block, plus the lane's 16 bytes
  int32_t bstride;    // elements between row blocks
  int32_t rows;       // rows in the tile
  __device__ typename F::T load(int rc, int k, int, bool) const {
    typedef typename F::T T;
    if (16 * rc >= rows) {
      const floatx4 z{0.f, 0.f, 0.f, 0.f};
      return T{__builtin_bit_cast(decltype(T::a), z), __builtin_bit_cast(decltype(T::b), z)};
    }
    const XE* p = base + rc * bstride + (k / F::KS) * (2 * kHalf);
    const floatx4 a = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(p));
    const floatx4 b = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(p + kHalf));
    return T{__builtin_bit_cast(decltype(T::a), a), __builtin_bit_cast(decltype(T::b), b)};
  }
};

// The k-loop of one pass, software-pipelined with two register sets (no
// copies of loaded data): the loads of one step are in flight while the MFMAs
// of the previous step run.  The last load of the paired loop is clamped to
// the final step (a redundant cache hit when the step count is even).
// One k-step's operands: the tile's RC row blocks and the NPC query column
// blocks (q[pc] = the query row of the lane's pair in column block pc).
template <class F, int RC, int NPC, bool NT, class Src>
__device__ __forceinline__ void load_step(const Src& src, const typename F::QE* const* q, int k,
                                          int d, typename F::T (&x)[RC],
                                          typename F::T (&qv)[NPC]) {
#pragma unroll
  for (int rc = 0; rc < RC; ++rc) x[rc] = src.load(rc, k, d, NT);
#pragma unroll
  for (int pc = 0; pc < NPC; ++pc) qv[pc] = F::load(q[pc], k, d);
}

template <class F, int RC, int NPC, int NPCM>
__device__ __forceinline__ void mfma_step(const typename F::T (&x)[RC],
                                          const typename F::T (&qv)[NPC],
                                          floatx4 (&acc)[RC][NPCM]) {
#pragma unroll
  for (int pc = 0; pc < NPC; ++pc) {
#pragma unroll
    for (int rc = 0; rc < RC; ++rc) F::mfma(qv[pc], x[rc], acc[rc][pc]);
  }
}

// The k-loop of one pass over NPC column blocks of 16 pairs, software-
// pipelined with two register sets (no copies of loaded data): the loads of
// one step are in flight while the MFMAs of the previous step run.  The last
// load of the paired loop is clamped to the final step (a redundant cache hit
// when the step count is even).  xa holds the rows' first k-step when `pre`
// is set (issued before the pair scan so that the tile's first HBM reads
// overlap it).
template <class F, int RC, int NPC, int NPCM, bool NT, class Src>
__device__ __forceinline__ void pass_loop(const Src& xr, const typename F::QE* const* q, int ks0,
                                          int ks1, int sub, int d, floatx4 (&acc)[RC][NPCM],
                                          typename F::T (&xa)[RC], bool pre) {
  typename F::T xb[RC], qa[NPC], qb[NPC];
  if (pre) {
#pragma unroll
    for (int pc = 0; pc < NPC; ++pc) qa[pc] = F::load(q[pc], ks0 * F::KS + sub, d);
  } else {
    load_step<F, RC, NPC, NT>(xr, q, ks0 * F::KS + sub, d, xa, qa);
  }
  int ks = ks0;
  for (; ks + 1 < ks1; ks += 2) {
    load_step<F, RC, NPC, NT>(xr, q, (ks + 1) * F::KS + sub, d, xb, qb);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the MFMAs
    mfma_step<F, RC, NPC, NPCM>(xa, qa, acc);
    __builtin_amdgcn_sched_barrier(0);
    const int kn = (ks + 2 < ks1 ? ks + 2 : ks1 - 1) * F::KS + sub;
    load_step<F, RC, NPC, NT>(xr, q, kn, d, xa, qa);
    __builtin_amdgcn_sched_barrier(0);
    mfma_step<F, RC, NPC, NPCM>(xb, qb, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (ks < ks1) mfma_step<F, RC, NPC, NPCM>(xa, qa, acc);
}

// A pass over npc (1..NPCM) column blocks: the register arrays are sized at
// compile time, so each count has its own k-loop.
template <class F, int RC, int NPCM, bool NT, class Src>
__device__ __forceinline__ void pass_any(int npc, const Src& xr, const typename F::QE* const* q,
                                         int nsteps, int sub, int d, floatx4 (&acc)[RC][NPCM],
                                         typename F::T (&xa)[RC], bool pre) {
  switch (npc) {
    case 1: pass_loop<F, RC, 1, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre); break;
    case 2:
      if constexpr (NPCM >= 2) pass_loop<F, RC, 2, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
    case 3:
      if constexpr (NPCM >= 3) pass_loop<F, RC, 3, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
    case 4:
      if constexpr (NPCM >= 4) pass_loop<F, RC, 4, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
    case 5:
      if constexpr (NPCM >= 5) pass_loop<F, RC, 5, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
    case 6:
      if constexpr (NPCM >= 6) pass_loop<F, RC, 6, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
    case 7:
      if constexpr (NPCM >= 7) pass_loop<F, RC, 7, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
    default:
      if constexpr (NPCM >= 8) pass_loop<F, RC, 8, NPCM, NT, Src>(xr, q, 0, nsteps, sub, d, acc, xa, pre);
      break;
  }
}

// pmask (several arrays): pair p's candidates are the rows whose bit is set in
// pmask[p mw ..] (bit = row within the cluster); its window (s, len) is the
// hull of that set, and hull rows outside the set get a NaN score, which
// the selection drops.
// wl == NULL: pair u of the cluster is pair u (identity work list).
// pair_chunk > 0: workgroup (x, y) handles pairs [y*pair_chunk, (y+1)*pair_chunk)
// of its tile's cluster.  row_scale (nullable) multiplies each row's scores.
// NPCM: 16-pair column blocks per MFMA pass (1, 2, 4 or 8).  The pairs that
// overlap the tile are listed across ballot rounds until a whole pass is
// full, so a tile overlapped by P pairs is streamed ceil(P / (16 NPCM))
// times.  Each pair's accumulation is the same in every grouping, so results
// do not depend on NPCM.
// Waves per SIMD the compiler must allow: two where the accumulators and
// double-buffered operands fit 256 registers without spilling, one (with
// accumulators in AGPRs) for the widest passes.
template <int RT, int NPCM>
constexpr int rerank_waves_per_eu() {
  return RT * NPCM <= 128 ? 2 : 1;
}

template <int RT, int FMT, bool VEC, bool NT, int NPCM = 2>
__global__ __launch_bounds__(kRerankNT, (rerank_waves_per_eu<RT, NPCM>())) void rerank_kernel(
    const void* __restrict__ Xv, int32_t d, const int32_t* __restrict__ tiles, int32_t ntiles,
    const int32_t* __restrict__ cstart,
    const int32_t* __restrict__ wl, const Pair* __restrict__ pairs, int32_t c,
    const void* __restrict__ Qv, float* __restrict__ sbuf, int32_t rcap, int persistent,
    int32_t* __restrict__ ctr, int32_t pair_chunk, const float* __restrict__ row_scale,
    const int32_t* __restrict__ alist, const uint32_t* __restrict__ pmask, int32_t mw,
    const int32_t* __restrict__ tblk, uint32_t* __restrict__ bkey, int32_t nbcap) {
  typedef Feed<FMT, VEC> F;
  typedef typename F::XE XE;
  typedef typename F::QE QE;
  constexpr int RC = RT / 16;
  constexpr int PP = 16 * NPCM;  // pairs per pass
  constexpr int CAP = PP + kWavePairCap;
  // the wide feeds stream an operand-ordered copy (Xv = Xt or Xbt, tblk =
  // the tiles' first blocks); the others read row-major rows
  constexpr bool kTiled = VEC && (FMT == kF32W || FMT == kBF16W);
  typedef typename std::conditional<kTiled, TileRows<F, RC>, PtrRows<F, RC>>::type Src;
  __shared__ WaveShared<CAP> sh;
  const XE* X = static_cast<const XE*>(Xv);
  const QE* Q = static_cast<const QE*>(Qv);
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, s = lane >> 4;
  const int nsteps = (d + F::KS - 1) / F::KS;
  const int sub = F::SUBW * s;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  FetchState fs;
  for (int it = 0;; ++it) {
    int32_t tile;
    if (persistent == 1) {
      int32_t t = -1;
      if (lane == 0) t = fetch_tile(1, ntiles, ctr, fs, alist);
      tile = __shfl(t, 0);
    } else if (persistent == 2) {
      tile = fetch_tile(2, ntiles, ctr, fs, alist);
    } else {
      tile = it == 0 ? direct_tile(ntiles, tile_chunk(RT)) : -1;
    }
    if (tile < 0) break;
    // tile descriptor and pair range are wave-uniform: keep them in SGPRs
    const int4 td = reinterpret_cast<const int4*>(tiles)[uni(tile)];
    const int32_t j = uni(td.x), row0 = uni(td.y), rows_here = uni(td.w);
    const int64_t grow = uni(td.z);  // first row of the tile in the reordered corpus
    int32_t plo = uni(cstart[j]), phi = uni(cstart[j + 1]);
    if (pair_chunk > 0) {
      plo += int32_t(blockIdx.y) * pair_chunk;
      phi = min(phi, plo + pair_chunk);
    }
    Src xr;
    if constexpr (kTiled) {
      constexpr int kChunk = 2 * TileRows<F, RC>::kHalf;  // elements per (block, k-step)
      const int32_t nks = d / F::KS;
      xr.base = X + int64_t(uni(tblk[tile])) * nks * kChunk + lane * (16 / int(sizeof(XE)));
      xr.bstride = nks * kChunk;
      xr.rows = rows_here;
    } else {
#pragma unroll
      for (int rc = 0; rc < RC; ++rc)
        xr.xr[rc] = X + (grow + min(16 * rc + i, rows_here - 1)) * d;
    }
    typename F::T xa[RC];
    bool pre = plo < phi;
    if (pre) {  // the first k-step's rows, in flight during the pair scan
#pragma unroll
      for (int rc = 0; rc < RC; ++rc) xa[rc] = xr.load(rc, sub, d, NT);
    }
    int32_t pb = plo;
    int n = 0;  // listed pairs not yet scored (wave-uniform)
    for (;;) {
      // list the overlapping pairs until a pass is full or the cluster's
      // pairs are exhausted
      while (n < PP && pb < phi) {
        const int32_t u = pb + lane;
        bool hit = false;
        int32_t pi = 0;
        Pair pr{0, 0, 0, 0};
        if (u < phi) {
          pi = wl ? wl[u] : u;
          pr = pairs[pi];
          hit = pr.s < row0 + rows_here && pr.s + pr.len > row0;
        }
        const uint64_t m = __ballot(hit);
        if (hit) {
          const int slot = n + __popcll(m & below);
          sh.lp[slot] = pi;
          sh.lq[slot] = pi / c;
          sh.ls[slot] = pr.s;
          sh.le[slot] = pr.s + pr.len;
          if (pmask) {  // tiles start at multiples of 32 rows
#pragma unroll
            for (int w = 0; w < (RT + 31) / 32; ++w)
              sh.lm[slot][w] = pmask[int64_t(pi) * mw + (row0 >> 5) + w];
          }
        }
        n += __popcll(m);
        pb += kWavePairCap;
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      if (n == 0) break;
      const int np = min(PP, n);
      const int npc = NPCM == 1 ? 1 : (np + 15) / 16;
      floatx4 acc[RC][NPCM];
#pragma unroll
      for (int rc = 0; rc < RC; ++rc) {
#pragma unroll
        for (int pc = 0; pc < NPCM; ++pc) acc[rc][pc] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
      const QE* q[NPCM];
#pragma unroll
      for (int pc = 0; pc < NPCM; ++pc) q[pc] = Q + int64_t(sh.lq[min(16 * pc + i, np - 1)]) * d;
      pass_any<F, RC, NPCM, NT, Src>(npc, xr, q, nsteps, sub, d, acc, xa, pre);
      pre = false;
      // D layout: acc[rc][pc][e] = pair 16 pc + 4 s + e, row 16 rc + i.
      // The score stores are nontemporal: the selection reads them once.
      // Block keys: the smallest score key of each (pair, 32-row block of the
      // tile) over the rows stored (NaN, a row outside the union, has the
      // largest key), gathered in LDS and written once per block.
      constexpr int NB = RT / 32;
      if (bkey) {
        for (int u = lane; u < PP * 4; u += 64) sh.bk[u >> 2][u & 3] = 0xffffffffu;
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int pc = 0; pc < NPCM; ++pc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int pp = 16 * pc + 4 * s + e;
          if (pc < npc && pp < np) {
            const int32_t a = sh.ls[pp], en = sh.le[pp];
            float* dst = sbuf + int64_t(sh.lp[pp]) * rcap - a;
            uint32_t km[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) km[b] = 0xffffffffu;
#pragma unroll
            for (int rc = 0; rc < RC; ++rc) {
              const int rr = 16 * rc + i;
              const int32_t row = row0 + rr;
              if (rr < rows_here && row >= a && row < en) {
                float v = acc[rc][pc][e];
                if (row_scale) v *= row_scale[grow + rr];
                if (pmask && !((sh.lm[pp][rr >> 5] >> (rr & 31)) & 1u))
                  v = __builtin_nanf("");
                __builtin_nontemporal_store(v, &dst[row]);
                km[rc >> 1] = min(km[rc >> 1], score_key(v));
              }
            }
            if (bkey) {
#pragma unroll
              for (int b = 0; b < NB; ++b)
                if (km[b] != 0xffffffffu) atomicMin(&sh.bk[pp][b], km[b]);
            }
          }
        }
      }
      if (bkey) {
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        for (int u = lane; u < np * NB; u += 64) {
          const int pp = u / NB, b = u - pp * NB;
          const int32_t a = sh.ls[pp], en = sh.le[pp], b0 = row0 + 32 * b;
          if (32 * b < rows_here && b0 < en && b0 + 32 > a)
            bkey[int64_t(sh.lp[pp]) * nbcap + ((b0 >> 5) - (a >> 5))] = sh.bk[pp][b];
        }
      }
      // the entries past this pass (at most 63) move to the front of the list
      const int rest = n - np;
      if (rest > 0) {
        int32_t vp = 0, vq = 0, vs = 0, ve = 0;
        uint32_t vm[4] = {0u, 0u, 0u, 0u};
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) {
          vp = sh.lp[np + lane];
          vq = sh.lq[np + lane];
          vs = sh.ls[np + lane];
          ve = sh.le[np + lane];
          if (pmask) {
#pragma unroll
            for (int w = 0; w < (RT + 31) / 32; ++w) vm[w] = sh.lm[np + lane][w];
          }
        }
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) {
          sh.lp[lane] = vp;
          sh.lq[lane] = vq;
          sh.ls[lane] = vs;
          sh.le[lane] = ve;
          if (pmask) {
#pragma unroll
            for (int w = 0; w < (RT + 31) / 32; ++w) sh.lm[lane][w] = vm[w];
          }
        }
      }
      n = rest;
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Workgroup rerank of one 128-row tile (the operand-ordered feeds, direct
// schedule).  The 4 waves of a workgroup take 32 rows each and share one list
// of the pairs overlapping the whole tile, so every query row a pass needs is
// read from L2 once per workgroup instead of once per wave: per k-step the
// workgroup stages the pass's query block (16 NPC rows x one k-step) in LDS,
// two steps ahead through registers, and each wave reads it back with 16-byte
// LDS loads.  The registers the per-wave query buffers held now carry a
// deeper row stream: each wave's own rows are loaded three k-steps ahead (a
// ring of four register sets).  One barrier per k-step publishes the next
// query block.  The MFMA sequence of every (pair, row) score is the one of
// rerank_kernel (same feed, same k order), so scores are bit-identical to it.
//
// Per k-step k: issue the staging loads of query block k + 2 and the row
// loads of step k + 3; read query block k from LDS; the MFMAs of step k;
// write the staged block k + 1 to LDS; barrier.  The list is filled by all 4
// waves, 256 pairs per round (each wave 64, slots by an LDS counter); the
// order of the entries is immaterial to the results.  Every loop bound and
// branch around a barrier is workgroup-uniform.
// Row register sets per wave (rows ring - 1 k-steps ahead).
constexpr int wg_ring(int npcm) { return 4; }
constexpr int kWgRound = 256;  // pairs tested per fill round
constexpr int kWgQRow = 144;   // bytes per staged query row: one k-step (128 B) + 16 B pad
constexpr int kWgQBlk = 16 * kWgQRow;

template <int FMT, int NPCM>
struct WgShared {
  static constexpr int CAP = 16 * NPCM + kWgRound;
  int32_t lp[CAP], lq[CAP], ls[CAP], le[CAP];
  uint32_t lm[CAP][4];  // membership bits of the tile's 128 rows (several arrays)
  __attribute__((aligned(16))) unsigned char qs[2][NPCM * kWgQBlk];
  uint32_t bk[4][16 * NPCM];  // block keys of the pass's pairs, per wave
  int32_t n;
};

// One pass over NPC column blocks: acc[rc][pc] of the wave's 32 rows.
template <int FMT, int NPC, int NPCM, int RING>
__device__ __forceinline__ void wg_pass(WgShared<FMT, NPCM>& sh, const TileRows<Feed<FMT, true>, 2>& xr,
                                        const typename Feed<FMT, true>::QE* __restrict__ Q, int32_t d,
                                        int np, int nsteps, floatx4 (&acc)[2][NPCM]) {
  typedef Feed<FMT, true> F;
  typedef typename F::T T;
  typedef typename F::QE QE;
  constexpr int RC = 2;
  constexpr int NCH = (NPC * 128 + 255) / 256;  // 16-byte staging chunks per thread
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = lane & 15, s = lane >> 4;
  const int sub = F::SUBW * s;
  // staging chunk u = tid + 256 j: column block u / 128, pair row (u / 8) % 16,
  // 16-byte part u % 8 of the k-step
  const QE* qsrc[NCH];
  int qdst[NCH];
  bool qon[NCH];
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    const int u = tid + 256 * j;
    const int pc = u >> 7, r = (u >> 3) & 15, part = u & 7;
    qon[j] = pc < NPC;
    const int e = qon[j] ? min(16 * pc + r, np - 1) : 0;
    qsrc[j] = Q + int64_t(sh.lq[e]) * d + part * (16 / int(sizeof(QE)));
    qdst[j] = pc * kWgQBlk + r * kWgQRow + part * 16;
  }
  floatx4 sg[2][NCH];
  auto stage_load = [&](int k, floatx4 (&dst)[NCH]) {
#pragma unroll
    for (int j = 0; j < NCH; ++j)
      if (qon[j]) dst[j] = *reinterpret_cast<const floatx4*>(qsrc[j] + k * F::KS);
  };
  auto stage_store = [&](int slot, const floatx4 (&src)[NCH]) {
#pragma unroll
    for (int j = 0; j < NCH; ++j)
      if (qon[j]) *reinterpret_cast<floatx4*>(&sh.qs[slot][qdst[j]]) = src[j];
  };
  // the wave's query operands of step k from LDS slot k % 2: lane (i, s)
  // reads pair row i of each block at the lane's two 16-byte halves
  auto qread = [&](int slot, T (&qv)[NPC]) {
#pragma unroll
    for (int pc = 0; pc < NPC; ++pc) {
      const unsigned char* b = &sh.qs[slot][pc * kWgQBlk + i * kWgQRow + 16 * s];
      qv[pc] = T{__builtin_bit_cast(decltype(T::a), *reinterpret_cast<const floatx4*>(b)),
                 __builtin_bit_cast(decltype(T::b), *reinterpret_cast<const floatx4*>(b + 64))};
    }
  };
  T xs[RING][RC];
  auto xload = [&](int k, T (&dst)[RC]) {
#pragma unroll
    for (int rc = 0; rc < RC; ++rc) dst[rc] = xr.load(rc, k * F::KS + sub, d, true);
  };
  // prologue: block 0 in LDS slot 0, block 1 staged, rows of steps
  // 0 .. RING - 2 in flight
  stage_load(0, sg[0]);
  if (1 < nsteps) stage_load(1, sg[1]);
#pragma unroll
  for (int u = 0; u + 1 < RING; ++u)
    if (u < nsteps) xload(u, xs[u]);
  stage_store(0, sg[0]);
  __syncthreads();
  // unrolled by U (a multiple of RING and of 2), so every register set index
  // below is a compile-time constant
  constexpr int U = RING % 2 == 0 ? RING : 2 * RING;
  for (int k = 0; k < nsteps; k += U) {
#pragma unroll
    for (int J = 0; J < U; ++J) {
      const int K = k + J;
      if (K < nsteps) {
        if (K + 2 < nsteps) stage_load(K + 2, sg[J & 1]);
        if (K + RING - 1 < nsteps) xload(K + RING - 1, xs[(J + RING - 1) % RING]);
        T qv[NPC];
        qread(J & 1, qv);
        mfma_step<F, RC, NPC, NPCM>(xs[J % RING], qv, acc);
        if (K + 1 < nsteps) stage_store((J + 1) & 1, sg[(J + 1) & 1]);
        __syncthreads();
      }
    }
  }
}

template <int FMT, int NPCM, bool BK>
__global__ __launch_bounds__(256, 2) void rerank_wg_kernel(
    const void* __restrict__ Xv, int32_t d, const int32_t* __restrict__ tiles, int32_t ntiles,
    const int32_t* __restrict__ cstart, const int32_t* __restrict__ wl,
    const Pair* __restrict__ pairs, int32_t c, const void* __restrict__ Qv,
    float* __restrict__ sbuf, int32_t rcap, const uint32_t* __restrict__ pmask, int32_t mw,
    const int32_t* __restrict__ tblk, uint32_t* __restrict__ bkey, int32_t nbcap) {
  typedef Feed<FMT, true> F;
  typedef typename F::XE XE;
  typedef typename F::QE QE;
  constexpr int PP = 16 * NPCM;
  constexpr int CAP = WgShared<FMT, NPCM>::CAP;
  __shared__ WgShared<FMT, NPCM> sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, s = lane >> 4;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int32_t tile = xcd_chunk_tile(ntiles, tile_chunk(128));
  if (tile < 0) return;  // the whole workgroup
  const XE* X = static_cast<const XE*>(Xv);
  const QE* Q = static_cast<const QE*>(Qv);
  const int4 td = reinterpret_cast<const int4*>(tiles)[tile];
  const int32_t j = td.x, row0 = td.y, rows_here = td.w;
  const int32_t plo = cstart[j], phi = cstart[j + 1];
  const int nsteps = d / F::KS;
  TileRows<F, 2> xr;
  {
    constexpr int kChunk = 2 * TileRows<F, 2>::kHalf;
    xr.base = X + (int64_t(tblk[tile]) + 2 * wave) * nsteps * kChunk + lane * (16 / int(sizeof(XE)));
    xr.bstride = nsteps * kChunk;
    xr.rows = max(0, min(32, rows_here - 32 * wave));
  }
  if (tid == 0) sh.n = 0;
  __syncthreads();
  int32_t pb = plo;
  int n = 0;  // listed pairs not yet scored (workgroup-uniform)
  for (;;) {
    while (n < PP && pb < phi) {
      const int32_t u = pb + 64 * wave + lane;
      bool hit = false;
      int32_t pi = 0;
      Pair pr{0, 0, 0, 0};
      if (u < phi) {
        pi = wl ? wl[u] : u;
        pr = pairs[pi];
        hit = pr.s < row0 + rows_here && pr.s + pr.len > row0;
      }
      const uint64_t m = __ballot(hit);
      int base = 0;
      if (lane == 0 && m) base = atomicAdd(&sh.n, __popcll(m));
      base = __shfl(base, 0);
      if (hit) {
        const int slot = base + __popcll(m & below);
        sh.lp[slot] = pi;
        sh.lq[slot] = pi / c;
        sh.ls[slot] = pr.s;
        sh.le[slot] = pr.s + pr.len;
        if (pmask) {  // 128-row tiles start at multiples of 128 rows of the cluster
#pragma unroll
          for (int w = 0; w < 4; ++w) sh.lm[slot][w] = pmask[int64_t(pi) * mw + (row0 >> 5) + w];
        }
      }
      pb += kWgRound;
      __syncthreads();
      n = sh.n;
      __syncthreads();
    }
    if (n == 0) break;
    const int np = min(PP, n);
    const int npc = (np + 15) / 16;
    floatx4 acc[2][NPCM];
#pragma unroll
    for (int rc = 0; rc < 2; ++rc)
#pragma unroll
      for (int pc = 0; pc < NPCM; ++pc) acc[rc][pc] = floatx4{0.f, 0.f, 0.f, 0.f};
    switch (npc) {
      case 1: wg_pass<FMT, 1, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc); break;
      case 2:
        if constexpr (NPCM >= 2) wg_pass<FMT, 2, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
      case 3:
        if constexpr (NPCM >= 3) wg_pass<FMT, 3, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
      case 4:
        if constexpr (NPCM >= 4) wg_pass<FMT, 4, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
      case 5:
        if constexpr (NPCM >= 5) wg_pass<FMT, 5, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
      case 6:
        if constexpr (NPCM >= 6) wg_pass<FMT, 6, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
      case 7:
        if constexpr (NPCM >= 7) wg_pass<FMT, 7, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
      default:
        if constexpr (NPCM >= 8) wg_pass<FMT, 8, NPCM, wg_ring(NPCM)>(sh, xr, Q, d, np, nsteps, acc);
        break;
    }
    // D layout: acc[rc][pc][e] = pair 16 pc + 4 s + e, row 32 wave + 16 rc + i.
    // Block keys: the smallest score key of the rows a wave stores for a pair
    // (NaN, a row outside the union, has the largest key), gathered in LDS.
    if constexpr (BK) {
      for (int u = lane; u < PP; u += 64) sh.bk[wave][u] = 0xffffffffu;
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int pc = 0; pc < NPCM; ++pc) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pp = 16 * pc + 4 * s + e;
        if (pc < npc && pp < np) {
          const int32_t a = sh.ls[pp], en = sh.le[pp];
          float* dst = sbuf + int64_t(sh.lp[pp]) * rcap - a;
          uint32_t km = 0xffffffffu;
#pragma unroll
          for (int rc = 0; rc < 2; ++rc) {
            const int rr = 32 * wave + 16 * rc + i;
            const int32_t row = row0 + rr;
            if (rr < rows_here && row >= a && row < en) {
              float v = acc[rc][pc][e];
              if (pmask && !((sh.lm[pp][rr >> 5] >> (rr & 31)) & 1u)) v = __builtin_nanf("");
              __builtin_nontemporal_store(v, &dst[row]);
              if (BK) km = min(km, score_key(v));
            }
          }
          if (BK && km != 0xffffffffu) atomicMin(&sh.bk[wave][pp], km);
        }
      }
    }
    if constexpr (BK) {
      // the wave's 32 rows are one block of 32 rows of the cluster
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      const int32_t b0 = row0 + 32 * wave;
      for (int pp = lane; pp < np; pp += 64) {
        const int32_t a = sh.ls[pp], en = sh.le[pp];
        if (32 * wave < rows_here && b0 < en && b0 + 32 > a)
          bkey[int64_t(sh.lp[pp]) * nbcap + ((b0 >> 5) - (a >> 5))] = sh.bk[wave][pp];
      }
    }
    // the entries past this pass move to the front of the list
    const int rest = n - np;
    int32_t vp = 0, vq = 0, vs = 0, ve = 0;
    uint32_t vm[4] = {0u, 0u, 0u, 0u};
    if (tid < rest) {
      vp = sh.lp[np + tid];
      vq = sh.lq[np + tid];
      vs = sh.ls[np + tid];
      ve = sh.le[np + tid];
      if (pmask) {
#pragma unroll
        for (int w = 0; w < 4; ++w) vm[w] = sh.lm[np + tid][w];
      }
    }
    __syncthreads();
    if (tid < rest) {
      sh.lp[tid] = vp;
      sh.lq[tid] = vq;
      sh.ls[tid] = vs;
      sh.le[tid] = ve;
      if (pmask) {
#pragma unroll
        for (int w = 0; w < 4; ++w) sh.lm[tid][w] = vm[w];
      }
    }
    if (tid == 0) sh.n = rest;
    n = rest;
    __syncthreads();
  }
}

// Layer-1 scores when every query's centroid window is the whole layer 1
// (r1 = C): the dense product rs[q][p] = <Q[q], cent_l1[p]>, a GEMM on MFMA.
// One (32 MB) x 128 output tile per workgroup; workgroups are dealt to the 8
// XCDs round-robin, so consecutive tiles of one XCD share their query rows in
// its L2.  Each wave owns a (16 MB) x 64 block (MB x 4 MFMA blocks of 16 x 16)
// over the whole dimension range and reads its operand fragments straight
// from the cache hierarchy, double-buffered across k-steps.  MB = 2 halves
// the tile so that small batches still fill the chip in whole rounds.
// row_scale (nullable) multiplies each centroid's scores (fp8 storage).  The
// routing decision only uses these scores through an order-independent error
// bound, so the summation order differs freely from the tiled window kernel.
constexpr int kGemmTileN = 128;

template <class F, int MB>
__device__ __forceinline__ void gemm_load(const typename F::QE* const (&qr)[MB],
                                          const typename F::XE* const (&xr)[4], int k, int d,
                                          typename F::T (&qa)[MB], typename F::Raw (&xa)[4]) {
#pragma unroll
  for (int b = 0; b < MB; ++b) qa[b] = F::load(qr[b], k, d);
#pragma unroll
  for (int b = 0; b < 4; ++b) xa[b] = F::raw(xr[b], k, d, false);
}

// Centroid fragments are decoded (fp8 -> bf16) one block at a time, right
// before their MFMAs, to keep the double-buffered registers small.
template <class F, int MB>
__device__ __forceinline__ void gemm_mfma(const typename F::T (&qa)[MB],
                                          const typename F::Raw (&xa)[4], int k, int d,
                                          floatx4 (&acc)[MB][4]) {
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const typename F::T x = F::dec(xa[nb], k, d);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) F::mfma(qa[mb], x, acc[mb][nb]);
  }
}

template <int FMT, bool VEC, int MB>
__global__ __launch_bounds__(256) void l1_gemm_kernel(const void* __restrict__ Qv, int64_t nq,
                                                      const void* __restrict__ Cv, int32_t C,
                                                      int32_t d, const float* __restrict__ row_scale,
                                                      float* __restrict__ rs) {
  typedef Feed<FMT, VEC> F;
  typedef typename F::XE XE;
  typedef typename F::QE QE;
  constexpr int TM = 32 * MB;  // query rows per workgroup tile
  const QE* Q = static_cast<const QE*>(Qv);
  const XE* X = static_cast<const XE*>(Cv);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, s = lane >> 4;
  const int sub = F::SUBW * s;
  const int64_t ntc = (C + kGemmTileN - 1) / kGemmTileN;
  const int64_t nblk = (nq + TM - 1) / TM * ntc;
  const int64_t per = (nblk + 7) / 8;
  const int64_t t = int64_t(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if ((blockIdx.x >> 3) >= per || t >= nblk) return;
  const int64_t q0 = (t / ntc) * TM + (wave & 1) * (16 * MB);
  const int32_t c0 = int32_t(t % ntc) * kGemmTileN + (wave >> 1) * 64;
  const QE* qr[MB];
  const XE* xr[4];
#pragma unroll
  for (int b = 0; b < MB; ++b) qr[b] = Q + min(q0 + 16 * b + i, nq - 1) * d;
#pragma unroll
  for (int b = 0; b < 4; ++b) xr[b] = X + int64_t(min(c0 + 16 * b + i, C - 1)) * d;
  floatx4 acc[MB][4];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nsteps = (d + F::KS - 1) / F::KS;
  typename F::T qa[MB], qb[MB];
  typename F::Raw xa[4], xb[4];
  gemm_load<F, MB>(qr, xr, sub, d, qa, xa);
  int ks = 0;
  for (; ks + 1 < nsteps; ks += 2) {
    const int k1 = (ks + 1) * F::KS + sub, k2 = (ks + 2 < nsteps ? ks + 2 : nsteps - 1) * F::KS + sub;
    gemm_load<F, MB>(qr, xr, k1, d, qb, xb);
    __builtin_amdgcn_sched_barrier(0);
    gemm_mfma<F, MB>(qa, xa, ks * F::KS + sub, d, acc);
    __builtin_amdgcn_sched_barrier(0);
    gemm_load<F, MB>(qr, xr, k2, d, qa, xa);
    __builtin_amdgcn_sched_barrier(0);
    gemm_mfma<F, MB>(qb, xb, k1, d, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (ks < nsteps) gemm_mfma<F, MB>(qa, xa, ks * F::KS + sub, d, acc);
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int32_t p = c0 + 16 * nb + i;
    if (p >= C) continue;
    const float sc = row_scale ? row_scale[p] : 1.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t q = q0 + 16 * mb + 4 * s + e;
        if (q < nq) rs[q * C + p] = row_scale ? acc[mb][nb][e] * sc : acc[mb][nb][e];
      }
  }
}

// bf16 layer-1 product staged through LDS (d a multiple of 64): a workgroup
// owns a 128 x 128 tile of [queries x centroids], the 4 waves 64 x 64 each
// (4 x 4 blocks of v_mfma_f32_16x16x32_bf16).  K runs in chunks of 64 (32
// with SPLIT below): the workgroup loads the chunk's 128 query rows and 128
// centroid rows (16 KB each) into registers while the
// previous chunk is consumed from LDS, then swaps buffers -- each operand
// byte is read from L2 once per tile instead of once per wave.  Rows are
// padded by 8 bf16 (16 B) so the 16 lanes of a fragment read spread over the
// LDS banks.  Three workgroups fit a CU, so the 632 tiles of 10,000 queries x
// 1,000 centroids run in one round on 256 CUs.  Tiles are dealt to the 8
// XCDs round-robin so consecutive tiles of one XCD share their query rows in
// its L2.
//
// SPLIT: both operands are read in fp32 and each value x is split on its way
// into LDS into h = bf16(x) and l = bf16(x - h) (x - h is exact in fp32), and
// the tile accumulates h_q h_mu + h_q l_mu + l_q h_mu: three MFMAs per
// fragment pair, scores within about 3 2^-16 |q| |mu| plus the fp32
// accumulation error instead of 2^-7 |q| |mu|.  With c > 1 that decides the
// routing for most queries without FP64 rescoring (1M x 768, 1,000 clusters,
// c = 8: 21 candidates per query with the bf16 band, 8.2 with the split one).
constexpr int kLdsK = 64;

__device__ inline void split_bf16x8(const float4& a, const float4& b, bf16x8& hi, bf16x8& lo) {
  const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  __hip_bfloat16 h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    h[e] = __float2bfloat16(v[e]);
    l[e] = __float2bfloat16(v[e] - __bfloat162float(h[e]));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

//
// The first l1_blocks workgroups (a multiple of 8) instead run the layer-1
// locate (l1_item) of 256 items each: both only need the hash kernel's
// output, so one launch runs them side by side.
template <bool SPLIT>
__global__ __launch_bounds__(256, 3) void l1_gemm_lds_kernel(
    const void* __restrict__ Qv, int64_t nq, const void* __restrict__ Cv, int32_t C, int32_t d,
    float* __restrict__ rs, L1Args la, unsigned l1_blocks) {
  constexpr int NP = SPLIT ? 2 : 1;  // operand parts in LDS (high, low)
  // K chunk and padded LDS row (bf16): the split parts double the LDS bytes
  // per value, so SPLIT takes half the chunk and three workgroups still fit a CU
  constexpr int KCH = SPLIT ? kLdsK / 2 : kLdsK, ROW = KCH + 8;
  constexpr int TPR = KCH / 8, RPP = 256 / TPR, NJ = 128 / RPP;  // loader shape
  typedef typename std::conditional<SPLIT, float, __hip_bfloat16>::type E;
  __shared__ __attribute__((aligned(16))) __hip_bfloat16 sa[NP][128 * ROW];
  __shared__ __attribute__((aligned(16))) __hip_bfloat16 sb[NP][128 * ROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (blockIdx.x < l1_blocks) {
    l1_item(la, int64_t(blockIdx.x) * 256 + tid);
    return;
  }
  const E* Q = static_cast<const E*>(Qv);
  const E* Cc = static_cast<const E*>(Cv);
  const unsigned bid = blockIdx.x - l1_blocks;
  const int i = lane & 15, s = lane >> 4;
  const int64_t ntc = (C + 127) / 128;
  const int64_t nblk = (nq + 127) / 128 * ntc;
  const int64_t per = (nblk + 7) / 8;
  const int64_t t = int64_t(bid & 7) * per + (bid >> 3);
  if ((bid >> 3) >= per || t >= nblk) return;
  const int64_t m0 = (t / ntc) * 128;
  const int32_t n0 = int32_t(t % ntc) * 128;
  // loader: thread tid moves 8 values of rows tid / TPR + RPP j, columns
  // 8 (tid % TPR)
  const int lr = tid / TPR, lc = 8 * (tid % TPR);
  const E* qsrc[NJ];
  const E* csrc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    qsrc[j] = Q + min(m0 + lr + RPP * j, nq - 1) * d + lc;
    csrc[j] = Cc + int64_t(min(n0 + lr + RPP * j, C - 1)) * d + lc;
  }
  bf16x8 ra[NJ], rb[NJ];          // bf16 operands in flight
  float4 fa4[NJ][2], fb4[NJ][2];  // fp32 operands in flight (SPLIT)
  auto gload = [&](int kc) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if constexpr (SPLIT) {
        const float4* qa = reinterpret_cast<const float4*>(qsrc[j] + kc * KCH);
        const float4* ca = reinterpret_cast<const float4*>(csrc[j] + kc * KCH);
        fa4[j][0] = qa[0];
        fa4[j][1] = qa[1];
        fb4[j][0] = ca[0];
        fb4[j][1] = ca[1];
      } else {
        ra[j] = *reinterpret_cast<const bf16x8*>(qsrc[j] + kc * KCH);
        rb[j] = *reinterpret_cast<const bf16x8*>(csrc[j] + kc * KCH);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int o = (lr + RPP * j) * ROW + lc;
      if constexpr (SPLIT) {
        bf16x8 h, l;
        split_bf16x8(fa4[j][0], fa4[j][1], h, l);
        *reinterpret_cast<bf16x8*>(&sa[0][o]) = h;
        *reinterpret_cast<bf16x8*>(&sa[NP - 1][o]) = l;
        split_bf16x8(fb4[j][0], fb4[j][1], h, l);
        *reinterpret_cast<bf16x8*>(&sb[0][o]) = h;
        *reinterpret_cast<bf16x8*>(&sb[NP - 1][o]) = l;
      } else {
        *reinterpret_cast<bf16x8*>(&sa[0][o]) = ra[j];
        *reinterpret_cast<bf16x8*>(&sb[0][o]) = rb[j];
      }
    }
  };
  const int wr = (wave & 1) * 64, wc = (wave >> 1) * 64;
  floatx4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nk = d / KCH;
  gload(0);
  lstore();
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    if (kc + 1 < nk) gload(kc + 1);  // in flight while this chunk is consumed
#pragma unroll
    for (int kk = 0; kk < KCH; kk += 32) {
      bf16x8 fa[NP][4], fb[NP][4];
#pragma unroll
      for (int h = 0; h < NP; ++h) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
          fa[h][a] = *reinterpret_cast<const bf16x8*>(&sa[h][(wr + 16 * a + i) * ROW + kk + 8 * s]);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          fb[h][b] = *reinterpret_cast<const bf16x8*>(&sb[h][(wc + 16 * b + i) * ROW + kk + 8 * s]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][a], fb[0][b], acc[a][b], 0, 0, 0);
      if constexpr (SPLIT) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[0][a], fb[NP - 1][b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[NP - 1][a], fb[0][b], acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave is done with this chunk before it is overwritten
    if (kc + 1 < nk) {
      lstore();
      __syncthreads();
    }
  }
  // D layout: acc[a][b][e] = query wr + 16 a + 4 s + e, centroid wc + 16 b + i
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int32_t p = n0 + wc + 16 * b + i;
    if (p >= C) continue;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t q = m0 + wr + 16 * a + 4 * s + e;
        if (q < nq) rs[q * C + p] = acc[a][b][e];
      }
  }
}

// ------------------------------------------------------------ final top-k
constexpr int kSelNT = 256;
constexpr int kKeyCache = 8192;

struct CandView {
  int32_t c;
  const Pair* pr;     // the query's c pairs
  const float* sb;    // its c score rows (stride rcap)
  int32_t rcap;
  int32_t start[LIDER_MAX_C + 1];
};

// Per query: top k (or a shortlist of S) over its windows.  MODE 0 = final
// output; MODE 1 = shortlist of sorted-row indices for the fp32 rerank.
// drop: NaN scores (key 0xffffffff, sorted last) are padding, not candidates.
template <int KPMAX, int MODE>
__global__ __launch_bounds__(kSelNT) void select_kernel(
    const Pair* __restrict__ pairs, const float* __restrict__ sbuf, int32_t rcap, int32_t c,
    int64_t nq, int32_t K, const int64_t* __restrict__ off, const int32_t* __restrict__ perm32,
    int64_t* __restrict__ ids, float* __restrict__ scores, int32_t kout,
    int32_t* __restrict__ slist, int drop, CertArgs ca, int32_t kcap) {
  __shared__ SelShared sh;
  __shared__ uint64_t srt[KPMAX];
  __shared__ int32_t sidx[KPMAX];
  extern __shared__ uint32_t keys[];  // dynamic: kcap keys (at most kKeyCache)
  __shared__ uint32_t s_thr;
  __shared__ int32_t s_m;
  __shared__ int32_t start[LIDER_MAX_C + 1];
  __shared__ int32_t pj[LIDER_MAX_C], ps[LIDER_MAX_C];
  const int tid = threadIdx.x;
  for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
    if (tid == 0) {
      int32_t acc = 0;
      for (int t = 0; t < c; ++t) {
        const Pair pr = pairs[q * c + t];
        start[t] = acc;
        pj[t] = pr.j;
        ps[t] = pr.s;
        acc += pr.j >= 0 ? pr.len : 0;
      }
      start[c] = acc;
    }
    __syncthreads();
    const int32_t n = start[c];
    const float* sbq = sbuf + q * int64_t(c) * rcap;
    auto slot_of = [&](int i) {
      int lo = 0, hi = c;  // largest t with start[t] <= i
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= i)
          lo = mid;
        else
          hi = mid;
      }
      return lo;
    };
    const bool cached = n <= kcap;
    if (cached) {
      for (int t = 0; t < c; ++t) {
        const int32_t a = start[t], len = start[t + 1] - a;
        for (int p = tid; p < len; p += kSelNT) keys[a + p] = score_key(sbq[int64_t(t) * rcap + p]);
      }
      __syncthreads();
    }
    auto key_of = [&](int i) {
      if (cached) return keys[i];
      const int t = slot_of(i);
      return score_key(sbq[int64_t(t) * rcap + (i - start[t])]);
    };
    auto row_of = [&](int i) {
      const int t = slot_of(i);
      return off[pj[t]] + ps[t] + (i - start[t]);
    };
    auto id_of = [&](int i) { return uint32_t(perm32[row_of(i)]); };
    const int KK = K;
    const int KP = pow2_at_least(KK);
    const int got = block_select<kSelNT>(n, KK, KP, key_of, id_of, srt, sidx, sh);
    auto valid = [&](int t) {
      return t < got && !(drop && uint32_t(srt[t] >> 32) == 0xffffffffu);
    };
    if (MODE == 0) {
      for (int t = tid; t < kout; t += kSelNT) {
        if (valid(t)) {
          ids[q * kout + t] = int64_t(srt[t] & 0xffffffffu);
          scores[q * kout + t] = key_score(uint32_t(srt[t] >> 32));
        } else {
          ids[q * kout + t] = -1;
          scores[q * kout + t] = -INFINITY;
        }
      }
    } else if (MODE == 1) {
      for (int t = tid; t < K; t += kSelNT)
        slist[q * K + t] = valid(t) ? int32_t(row_of(sidx[t])) : -1;
    } else {
      // certified shortlist: every candidate within the margin of the k-th
      // best (list order is immaterial: the fp32 rerank ranks by score, id)
      if (tid < 64) {
        const uint32_t T = valid(K - 1) ? uint32_t(srt[K - 1] >> 32) : 0xffffffffu;
        const uint32_t thr = cert_threshold(ca, q, T, tid);
        if (tid == 0) {
          s_thr = thr;
          s_m = 0;
        }
      }
      __syncthreads();
      const uint32_t thr = s_thr;
      for (int i = tid; i < n; i += kSelNT) {
        if (key_of(i) <= thr) slist[q * ca.cap + atomicAdd(&s_m, 1)] = int32_t(row_of(i));
      }
      __syncthreads();
      if (tid == 0) ca.scnt[q] = s_m;
    }
    __syncthreads();
  }
}

// Per query top K (K <= 64), one wave per query: repeated wave minima of
// (key, candidate index) extract the K + 1 best; an exact key tie at the K-th
// place is resolved by original id over all tied candidates; the winners are
// finally ordered by (score desc, id asc).  MODE 0 writes ids / scores, MODE 1
// the shortlist of sorted-row indices.  drop: NaN scores (key 0xffffffff) are
// not candidates (rows of a union's hull outside the union).  R = 0: with
// block keys (bkey), the block form reads only the blocks that can hold the
// K + 1 best; else, or past its limits, the keys are re-read from the score
// rows in one pass that lists the candidates at or below a threshold that it
// tightens as it goes (no LDS copy of the keys: an LDS cache of 2,048 keys
// per wave held the kernel to 3 workgroups per CU).
constexpr int kSelList = 256;
// Block keys per lane in the block form of the selection: queries whose
// windows span more than 64 kSelBlk blocks take the other forms.
constexpr int kSelBlk = 8;

template <int MODE, int R>
__global__ __launch_bounds__(256) void wave_select_kernel(
    const Pair* __restrict__ pairs, const float* __restrict__ sbuf, int32_t rcap, int32_t c,
    int64_t nq, int32_t K, const int64_t* __restrict__ off, const int32_t* __restrict__ perm32,
    int64_t* __restrict__ ids, float* __restrict__ scores, int32_t kout,
    int32_t* __restrict__ slist, int drop, CertArgs ca, const uint32_t* __restrict__ bkey,
    int32_t nbcap) {
  __shared__ int32_t start[4][LIDER_MAX_C + 1];
  __shared__ int64_t pbase[4][LIDER_MAX_C];  // sorted row of each slot's first candidate
  __shared__ int32_t bstart[4][LIDER_MAX_C + 1];  // block form: first block of each slot
  __shared__ int32_t wstart[4][LIDER_MAX_C];      // block form: window start in the cluster
  __shared__ int32_t bsel[4][64];                 // block form: blocks being read
  __shared__ uint64_t ext[4][65];
  __shared__ uint32_t wkey[4][64], wid[4][64];
  __shared__ int64_t wrow[4][64];
  __shared__ uint32_t lkey[4][kSelList];
  __shared__ int32_t lidx[4][kSelList];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));  // uniform, in SGPRs
  const uint64_t below = (uint64_t(1) << lane) - 1;
  // one query per wave, no loop: per-query index arithmetic is not hoisted
  // into registers held across queries
  const int64_t q = int64_t(blockIdx.x) * 4 + wave;
  if (q >= nq) return;
  {
    const float* sbq = sbuf + q * int64_t(c) * rcap;
    // R > 0 (n <= 64 R): candidate i = lane + 64 j keeps its key in register
    // j.  With one slot the scores are sbq[0, len): their loads are issued
    // before the pair is read (an index past the slot re-reads an entry of
    // the query's own buffer and is masked below).
    float fv[R > 0 ? R : 1];
    const bool pre = R > 0 && c == 1;
    if (pre) {
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (64 * j < rcap) fv[j] = sbq[uint32_t(min(lane + 64 * j, rcap - 1))];
    }
    // slot table: lane t reads pair t (64 at a time); start[] is the
    // exclusive prefix sum of the slot lengths, pbase[] each slot's first row.
    // Block form: the window of slot t spans the blocks of 32 cluster rows
    // from (s >> 5) to ((s + len - 1) >> 5); bstart[] is the exclusive
    // prefix sum of their counts
    int32_t n = 0, nbt = 0;
    for (int t0 = 0; t0 < c; t0 += 64) {
      const int t = t0 + lane;
      int32_t len = 0, s0 = 0;
      int64_t base = 0;
      if (t < c) {
        const Pair pr = pairs[q * c + t];
        if (pr.j >= 0) {
          len = pr.len;
          s0 = pr.s;
          base = off[pr.j] + pr.s;
        }
      }
      const int32_t nb = len > 0 ? ((s0 + len - 1) >> 5) - (s0 >> 5) + 1 : 0;
      int32_t incl = len, inclb = nb;
      if (c > 1) {
        for (int o = 1; o < 64; o <<= 1) {
          const int32_t y = __shfl_up(incl, o), yb = __shfl_up(inclb, o);
          if (lane >= o) {
            incl += y;
            inclb += yb;
          }
        }
      }
      if (t < c) {
        start[wave][t] = n + incl - len;
        pbase[wave][t] = base;
        if (bkey) {
          bstart[wave][t] = nbt + inclb - nb;
          wstart[wave][t] = s0;
        }
      }
      n += __shfl(incl, c > 1 ? 63 : 0);
      nbt += __shfl(inclb, c > 1 ? 63 : 0);
    }
    if (lane == 0) {
      start[wave][c] = n;
      bstart[wave][c] = nbt;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    const int32_t* st = start[wave];
    auto slot_of = [&](int32_t i) {
      int lo = 0, hi = c;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (st[mid] <= i)
          lo = mid;
        else
          hi = mid;
      }
      return lo;
    };
    auto row_of = [&](int32_t i) {
      const int t = slot_of(i);
      return pbase[wave][t] + (i - st[t]);
    };
    uint32_t kr[R > 0 ? R : 1];
    if (R > 0) {
      if (!pre && n > 0) {
        // several slots: all R loads issued before any key is formed; the
        // slot of candidate i only moves forward as i grows
        int t = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if (64 * j >= n) continue;  // wave-uniform: register slots past the candidates
          const int32_t i = min(lane + 64 * j, n - 1);
          while (t + 1 < c && st[t + 1] <= i) ++t;
          fv[j] = sbq[int64_t(t) * rcap + (i - st[t])];
        }
      }
#pragma unroll
      for (int j = 0; j < R; ++j) kr[j] = lane + 64 * j < n ? score_key(fv[j]) : 0xffffffffu;
    }
    // extraction of the K + 1 smallest (key, index).  First a threshold: tau =
    // the (K+1)-th smallest of the 64 lane minima, so at least K + 1
    // candidates have key <= tau; those candidates (usually few) are listed
    // in LDS and the extraction runs over the list.  The list holds every
    // candidate the full extraction would take, so the result is the same;
    // a list longer than kSelList falls back to extracting over everything.
    const int want = min(n, K + 1);
    const uint32_t kdrop = drop ? 0xffffffffu : 0u;  // 0: never matches a real key test below
    // f(index, key, valid) over the lane's candidates, the same number of
    // calls on every lane (ballots inside f see the whole wave)
    // R == 0: the scores are re-read from the score rows in chunks of 1,024
    // entries of one slot (16 loads per lane); the next chunk's loads are
    // issued before the current chunk's keys are used
    auto load_chunk = [&](int t, int p0, float(&v)[16]) {
      const int32_t len = st[t + 1] - st[t];
      const float* src = sbq + int64_t(t) * rcap;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int p = p0 + lane + 64 * u;
        v[u] = src[p < len ? p : max(len - 1, 0)];
      }
    };
    auto scan = [&](auto&& f) {
      if (R > 0) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const int32_t i = lane + 64 * j;
          if (64 * j < n) f(i, kr[j], i < n);  // wave-uniform: skips slots past the candidates
        }
      } else {
        int t = 0, p0 = 0;
        float v[16];
        load_chunk(0, 0, v);
        while (true) {
          const int32_t a = __builtin_amdgcn_readfirstlane(st[t]);
          const int32_t len = __builtin_amdgcn_readfirstlane(st[t + 1]) - a;
          int tn = t, pn = p0 + 1024;
          if (pn >= len) {
            tn = t + 1;
            pn = 0;
          }
          float w[16];
          if (tn < c) load_chunk(tn, pn, w);
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int p = p0 + lane + 64 * u;
            if (p0 + 64 * u < len)  // wave-uniform
              f(a + p, p < len ? score_key(v[u]) : 0xffffffffu, p < len);
          }
          if (tn >= c) break;
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = w[u];
          t = tn;
          p0 = pn;
        }
      }
    };
    // the smallest x with at least `want` of the lanes' values <= x, by
    // bisection on ballot counts
    auto bisect = [&](uint32_t lv) {
      uint32_t lo = 0u, hi = 0xffffffffu;
      while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (__popcll(__ballot(lv <= mid)) >= want)
          hi = mid;
        else
          lo = mid + 1;
      }
      return lo;
    };
    // f that lists every candidate with key <= th (the first kSelList in
    // LDS) and takes the lane minima on the way; the slots are formed only
    // for a ballot that lists some candidate
    uint32_t lmin = 0xffffffffu;
    int m = 0;
    auto list_one = [&](int32_t i, uint32_t kk, bool in) {
      const uint64_t bal = __ballot(in);
      if (bal) {  // wave-uniform
        const int slot = m + __popcll(bal & below);
        if (in && slot < kSelList) {
          lkey[wave][slot] = kk;
          lidx[wave][slot] = i;
        }
        m += __popcll(bal);
      }
    };
    auto lister = [&](uint32_t th) {
      m = 0;
      return [&, th](int32_t i, uint32_t kk, bool ok) {
        const bool valid = ok && !(drop && kk == kdrop);
        if (valid) lmin = kk < lmin ? kk : lmin;
        list_one(i, kk, valid && kk <= th);
      };
    };
    auto list_below = [&](uint32_t th) { scan(lister(th)); };
    bool have_min = false, done = false;
    // Block form (R == 0 with block keys: the smallest key of every 32-row
    // block of every window, written by the rerank).  T = the want-th
    // smallest block key: at least `want` candidates (one per block) have
    // key <= T, so the K + 1 smallest all do, and each lies in a block whose
    // key is <= T.  Only those blocks are read (about want of them, against
    // every candidate of the query); their keys <= T are listed.
    uint32_t bk[kSelBlk];
    int32_t bt[kSelBlk];  // (slot << 16) | block of the slot, -1 past the blocks
    const bool bform = R == 0 && bkey && nbt <= 64 * kSelBlk && want > 0;
    // f(index, key, in window) over every candidate of the blocks with key
    // <= th, two blocks per step and four steps' loads in flight
    auto for_blocks = [&](uint32_t th, auto&& f) {
#pragma unroll
      for (int j = 0; j < kSelBlk; ++j) {
        if (64 * j >= nbt) break;  // wave-uniform
        const bool sel = bt[j] >= 0 && bk[j] <= th;
        const uint64_t bal = __ballot(sel);
        if (!bal) continue;  // wave-uniform
        if (sel) bsel[wave][__popcll(bal & below)] = bt[j];
        const int nsel = __popcll(bal);
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        for (int g0 = 0; g0 < nsel; g0 += 8) {
          float v[4];
          int32_t ix[4];
          bool ok[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int g = g0 + 2 * u + (lane >> 5);
            ok[u] = false;
            ix[u] = 0;
            v[u] = 0.f;
            if (g < nsel) {
              const int32_t e = bsel[wave][g], tt = e >> 16;
              const int32_t s0 = wstart[wave][tt], len = st[tt + 1] - st[tt];
              const int32_t pos = (((s0 >> 5) + (e & 0xffff)) << 5) + (lane & 31) - s0;
              ok[u] = pos >= 0 && pos < len;
              ix[u] = st[tt] + pos;
              v[u] = sbq[int64_t(tt) * rcap + (ok[u] ? pos : 0)];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) f(ix[u], score_key(v[u]), ok[u]);
        }
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
      }
    };
    if (bform) {
      int t = 0;
#pragma unroll
      for (int j = 0; j < kSelBlk; ++j) {
        bk[j] = 0xffffffffu;
        bt[j] = -1;
        if (64 * j >= nbt) continue;  // wave-uniform
        const int32_t b = min(lane + 64 * j, nbt - 1);
        while (t + 1 < c && bstart[wave][t + 1] <= b) ++t;
        const int32_t kb = b - bstart[wave][t];
        bk[j] = bkey[(q * c + t) * int64_t(nbcap) + kb];
        if (lane + 64 * j < nbt) bt[j] = (t << 16) | kb;
      }
#pragma unroll
      for (int j = 0; j < kSelBlk; ++j)
        if (bt[j] < 0) bk[j] = 0xffffffffu;
      // T by bisection on the count of block keys <= x
      uint32_t lo = 0u, hi = 0xffffffffu;
      while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < kSelBlk; ++j)
          if (64 * j < nbt) cnt += __popcll(__ballot(bk[j] <= mid));
        if (cnt >= want)
          hi = mid;
        else
          lo = mid + 1;
      }
      const uint32_t T = lo;
      int nsel = 0;
#pragma unroll
      for (int j = 0; j < kSelBlk; ++j)
        if (64 * j < nbt) nsel += __popcll(__ballot(bt[j] >= 0 && bk[j] <= T));
      if (T != 0xffffffffu && nsel <= 16) {
        // up to 16 blocks: their candidates in registers (block g = 2 u +
        // lane / 32, row lane % 32), then a tighter threshold th = the
        // want-th smallest lane minimum of their keys <= T (at least `want`
        // candidates <= th, all of them in these blocks); the keys <= th
        // are listed
        int nb0 = 0;
#pragma unroll
        for (int j = 0; j < kSelBlk; ++j) {
          if (64 * j >= nbt) break;  // wave-uniform
          const bool sel = bt[j] >= 0 && bk[j] <= T;
          const uint64_t bal = __ballot(sel);
          if (sel) bsel[wave][nb0 + __popcll(bal & below)] = bt[j];
          nb0 += __popcll(bal);
        }
        __threadfence_block();
        __builtin_amdgcn_wave_barrier();
        auto cand = [&](int u, int32_t* ixp) {  // window position check and flat index
          const int g = 2 * u + (lane >> 5);
          if (g >= nsel) return -1;
          const int32_t e = bsel[wave][g], tt = e >> 16;
          const int32_t s0 = wstart[wave][tt], len = st[tt + 1] - st[tt];
          const int32_t pos = (((s0 >> 5) + (e & 0xffff)) << 5) + (lane & 31) - s0;
          if (pos < 0 || pos >= len) return -1;
          *ixp = st[tt] + pos;
          return int(int64_t(tt) * rcap + pos);
        };
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int32_t ixu;
          const int at = cand(u, &ixu);
          v[u] = at >= 0 ? sbq[at] : 0.f;
        }
        uint32_t kk[8], lm2 = 0xffffffffu;
        uint32_t okm = 0;  // candidates with key <= T
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int32_t ixu;
          kk[u] = score_key(v[u]);
          if (cand(u, &ixu) >= 0 && !(drop && kk[u] == kdrop) && kk[u] <= T) {
            okm |= 1u << u;
            lm2 = kk[u] < lm2 ? kk[u] : lm2;
          }
        }
        const uint32_t th = min(T, bisect(lm2));
        m = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (2 * u >= nsel) break;  // wave-uniform
          int32_t ixu = 0;
          const bool in = ((okm >> u) & 1u) && kk[u] <= th;
          if (in) cand(u, &ixu);
          list_one(ixu, kk[u], in);
        }
        done = m <= kSelList;
      } else if (T != 0xffffffffu) {
        m = 0;
        for_blocks(T, [&](int32_t i, uint32_t kk, bool ok) {
          list_one(i, kk, ok && !(drop && kk == kdrop) && kk <= T);
        });
        done = m <= kSelList;
      }
    }
    if (R == 0 && !done) {
      // One pass over the chunks.  Each chunk's keys update the lane minima;
      // a chunk holding a key at or below the threshold th first tightens th
      // to the want-th smallest lane minimum (at least `want` candidates seen
      // so far are <= it, so the K + 1 smallest of all are too; th never
      // grows), then lists its keys <= th.  Every candidate <= the final th
      // is listed when its chunk is read, so the list holds all the
      // extraction takes; a list past kSelList falls back to the two passes
      // below.
      uint32_t th = 0xffffffffu;
      int t = 0, p0 = 0;
      float v[16];
      load_chunk(0, 0, v);
      while (true) {
        const int32_t a = __builtin_amdgcn_readfirstlane(st[t]);
        const int32_t len = __builtin_amdgcn_readfirstlane(st[t + 1]) - a;
        int tn = t, pn = p0 + 1024;
        if (pn >= len) {
          tn = t + 1;
          pn = 0;
        }
        float w[16];
        if (tn < c) load_chunk(tn, pn, w);
        uint32_t cmin = 0xffffffffu;
        bool cv = false;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const uint32_t kk = score_key(v[u]);
          if (p0 + lane + 64 * u < len && !(drop && kk == kdrop)) {
            cmin = kk < cmin ? kk : cmin;
            cv = true;
          }
        }
        if (cv) lmin = cmin < lmin ? cmin : lmin;
        if (__ballot(cv && cmin <= th)) {  // wave-uniform
          th = bisect(lmin);
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int p = p0 + lane + 64 * u;
            const uint32_t kk = score_key(v[u]);
            if (p0 + 64 * u < len)  // wave-uniform
              list_one(a + p, kk, p < len && !(drop && kk == kdrop) && kk <= th);
          }
        }
        if (tn >= c) break;
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = w[u];
        t = tn;
        p0 = pn;
      }
      have_min = true;
      done = m <= kSelList;
    }
    if (!done) {
      // tau = the want-th smallest lane minimum: at least `want` candidates
      // have key <= tau, and the list holds them all when it fits
      if (!have_min)
        scan([&](int32_t, uint32_t kk, bool ok) {
          if (ok && !(drop && kk == kdrop)) lmin = kk < lmin ? kk : lmin;
        });
      list_below(bisect(lmin));
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    const bool listed = m <= kSelList;
    uint64_t prev = 0;
    int nx = 0;
    if (listed && m <= 64) {
      // few listed: each lane ranks one entry against all of them, reading
      // the others' (key, index) from their lanes
      uint32_t mk = 0xffffffffu, mi = 0xffffffffu;
      if (lane < m) {
        mk = lkey[wave][lane];
        mi = uint32_t(lidx[wave][lane]);
      }
      int rank = 0;
      for (int u = 0; u < m; ++u) {
        const uint32_t ku = uint32_t(__builtin_amdgcn_readlane(int(mk), u));
        const uint32_t iu = uint32_t(__builtin_amdgcn_readlane(int(mi), u));
        rank += (ku < mk) || (ku == mk && iu < mi);
      }
      if (lane < m && rank < want) ext[wave][rank] = (uint64_t(mk) << 32) | mi;
      nx = min(m, want);
    } else {
      for (int r = 0; r < want; ++r) {
        uint64_t best = ~uint64_t(0);
        if (listed) {
          for (int u = lane; u < m; u += 64) {
            const uint64_t v = (uint64_t(lkey[wave][u]) << 32) | uint32_t(lidx[wave][u]);
            if ((r == 0 || v > prev) && v < best) best = v;
          }
        } else {
          scan([&](int32_t i, uint32_t kk, bool ok) {
            const uint64_t v = (uint64_t(kk) << 32) | uint32_t(i);
            if (ok && !(drop && kk == kdrop) && (r == 0 || v > prev) && v < best) best = v;
          });
        }
        best = wave_min_u64(best);
        if (best == ~uint64_t(0)) break;  // no candidate left (wave-uniform)
        if (lane == 0) ext[wave][r] = best;
        prev = best;
        ++nx;
      }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    const int got = min(nx, K);
    if (lane < got) {
      const uint64_t v = ext[wave][lane];
      const int64_t row = row_of(int32_t(v & 0xffffffffu));
      wkey[wave][lane] = uint32_t(v >> 32);
      wid[wave][lane] = uint32_t(perm32[row]);
      wrow[wave][lane] = row;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    if (nx == K + 1 && uint32_t(ext[wave][K - 1] >> 32) == uint32_t(ext[wave][K] >> 32)) {
      // exact tie at the boundary: the tied places go to the smallest ids
      const uint32_t T = uint32_t(ext[wave][K - 1] >> 32);
      int need = 0;
      for (int t = 0; t < K; ++t) need += wkey[wave][t] == T;
      uint64_t last = 0;
      for (int r = 0; r < need; ++r) {
        uint64_t best = ~uint64_t(0);
        for (int t = 0; t < c; ++t) {
          const int32_t a = st[t], len = st[t + 1] - a;
          for (int p = lane; p < len; p += 64) {
            const uint32_t kk = score_key(sbq[int64_t(t) * rcap + p]);
            if (kk != T) continue;
            const int64_t row = pbase[wave][t] + p;
            const uint64_t v = (uint64_t(uint32_t(perm32[row])) << 32) | uint32_t(row);
            if ((r == 0 || v > last) && v < best) best = v;
          }
        }
        best = wave_min_u64(best);
        if (lane == 0) {
          wid[wave][K - need + r] = uint32_t(best >> 32);
          wrow[wave][K - need + r] = int64_t(uint32_t(best & 0xffffffffu));
        }
        last = best;
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
    }
    // order the winners by (key, id) and write
    uint32_t myk = 0xffffffffu, myid = 0xffffffffu;
    int64_t myrow = 0;
    if (lane < got) {
      myk = wkey[wave][lane];
      myid = wid[wave][lane];
      myrow = wrow[wave][lane];
    }
    int rank = 0;
    for (int u = 0; u < got; ++u) {
      const uint32_t ku = uint32_t(__builtin_amdgcn_readlane(int(myk), u));
      const uint32_t iu = uint32_t(__builtin_amdgcn_readlane(int(myid), u));
      rank += (ku < myk) || (ku == myk && iu < myid);
    }
    if (MODE == 0) {
      if (lane < got) {
        ids[q * kout + rank] = int64_t(myid);
        scores[q * kout + rank] = key_score(myk);
      }
      for (int t = got + lane; t < kout; t += 64) {
        ids[q * kout + t] = -1;
        scores[q * kout + t] = -INFINITY;
      }
    } else if (MODE == 1) {
      if (lane < got) slist[q * K + rank] = int32_t(myrow);
      for (int t = got + lane; t < K; t += 64) slist[q * K + t] = -1;
    } else {
      // certified shortlist: every candidate within the margin of the k-th
      // best key (the largest winner key when all K places are taken)
      uint32_t tk = lane < got ? myk : 0u;
      for (int o = 32; o > 0; o >>= 1) tk = max(tk, uint32_t(__shfl_xor(tk, o)));
      const uint32_t thr = cert_threshold(ca, q, got == K ? tk : 0xffffffffu, lane);
      int m = 0;
      auto cert = [&](int32_t i, uint32_t kk, bool ok) {
        const bool in = ok && kk <= thr;
        const uint64_t bal = __ballot(in);
        if (in) slist[q * ca.cap + m + __popcll(bal & below)] = int32_t(row_of(i));
        m += __popcll(bal);
      };
      if (bform)  // the blocks hold every candidate with key <= thr
        for_blocks(thr, cert);
      else
        scan(cert);
      if (lane == 0) ca.scnt[q] = m;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// Per query top K for 64 < K <= 128 (MODE 0: ids and scores, MODE 2: the
// certified shortlist), one wave per query with the candidates' keys in
// registers (n <= 64 R).  T = the (K+1)-th smallest key, by bisection on
// counts over all candidates; the candidates with key <= T (K + 1 and
// any ties) are listed in LDS and each ranked against the others by (key,
// index), which places the K + 1 smallest.  A list past kSelList (ties)
// extracts by repeated wave minima instead.  Boundary ties go to the smallest
// ids, and the winners are ordered by (score desc, id asc), as in the
// selection for k <= 64.
constexpr int kWideK = 128;

template <int MODE, int R>
__global__ __launch_bounds__(256) void wave_select_wide_kernel(
    const Pair* __restrict__ pairs, const float* __restrict__ sbuf, int32_t rcap, int32_t c,
    int64_t nq, int32_t K, const int64_t* __restrict__ off, const int32_t* __restrict__ perm32,
    int64_t* __restrict__ ids, float* __restrict__ scores, int32_t kout,
    int32_t* __restrict__ slist, int drop, CertArgs ca) {
  __shared__ int32_t start[4][LIDER_MAX_C + 1];
  __shared__ int64_t pbase[4][LIDER_MAX_C];
  __shared__ uint32_t lkey[4][kSelList];
  __shared__ int32_t lidx[4][kSelList];
  __shared__ uint64_t ext[4][kWideK + 1];
  __shared__ uint32_t wk[4][kWideK], wid[4][kWideK];
  __shared__ int64_t wrow[4][kWideK];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int64_t q = int64_t(blockIdx.x) * 4 + wave;
  if (q >= nq) return;
  const float* sbq = sbuf + q * int64_t(c) * rcap;
  // slot table: start[] the exclusive prefix sum of the slot lengths,
  // pbase[] each slot's first row
  int32_t n = 0;
  for (int t0 = 0; t0 < c; t0 += 64) {
    const int t = t0 + lane;
    int32_t len = 0;
    int64_t base = 0;
    if (t < c) {
      const Pair pr = pairs[q * c + t];
      if (pr.j >= 0) {
        len = pr.len;
        base = off[pr.j] + pr.s;
      }
    }
    int32_t incl = len;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (t < c) {
      start[wave][t] = n + incl - len;
      pbase[wave][t] = base;
    }
    n += __shfl(incl, 63);
  }
  if (lane == 0) start[wave][c] = n;
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  const int32_t* st = start[wave];
  auto row_of = [&](int32_t i) {
    int lo = 0, hi = c;  // the largest slot t with st[t] <= i
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (st[mid] <= i)
        lo = mid;
      else
        hi = mid;
    }
    return pbase[wave][lo] + (i - st[lo]);
  };
  // candidate i = lane + 64 j in register j (its score's bits, then its key);
  // all loads issued before any key is formed (the slot of i only moves
  // forward as i grows)
  float fv[R];
  {
    int t = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (64 * j >= n) continue;  // wave-uniform
      const int32_t i = min(lane + 64 * j, n - 1);
      while (t + 1 < c && st[t + 1] <= i) ++t;
      fv[j] = sbq[int64_t(t) * rcap + (i - st[t])];
    }
  }
  uint32_t kr[R];
  uint32_t vm = 0;  // bit j: register j holds a candidate
  uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    kr[j] = lane + 64 * j < n ? score_key(fv[j]) : 0xffffffffu;
    if (lane + 64 * j < n && !(drop && kr[j] == 0xffffffffu)) {
      vm |= 1u << j;
      kmin = min(kmin, kr[j]);
      kmax = max(kmax, kr[j]);
    }
  }
  const int want = min(n, K + 1);
  // T: the smallest x with at least `want` candidates <= x, by bisection
  // over [min, max] of the keys on per-lane counts summed across the wave
  // (no candidate: T = 0xffffffff, which lists nothing)
  uint32_t lo = dpp_min_u32(kmin), hi = ~dpp_min_u32(~kmax);
  if (lo > hi) lo = hi = 0xffffffffu;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    int32_t c0 = 0, c1 = 0;
#pragma unroll
    for (int j = 0; j < R; j += 2) {
      c0 += ((vm >> j) & 1u) && kr[j] <= mid;
      if (j + 1 < R) c1 += ((vm >> (j + 1)) & 1u) && kr[j + 1] <= mid;
    }
    if (dpp_sum_i32(c0 + c1) >= want)
      hi = mid;
    else
      lo = mid + 1;
  }
  const uint32_t T = lo;
  int m = 0;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    if (64 * j >= n) break;  // wave-uniform
    const bool in = ((vm >> j) & 1u) && kr[j] <= T;
    const uint64_t bal = __ballot(in);
    if (bal) {  // wave-uniform
      const int slot = m + __popcll(bal & below);
      if (in && slot < kSelList) {
        lkey[wave][slot] = kr[j];
        lidx[wave][slot] = lane + 64 * j;
      }
      m += __popcll(bal);
    }
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  int nx;
  if (m <= kSelList) {
    // each listed entry's rank among the listed, by (key, index)
    uint64_t me[kSelList / 64];
    int rk[kSelList / 64];
#pragma unroll
    for (int v = 0; v < kSelList / 64; ++v) {
      const int e = lane + 64 * v;
      me[v] = e < m ? (uint64_t(lkey[wave][e]) << 32) | uint32_t(lidx[wave][e]) : ~uint64_t(0);
      rk[v] = 0;
    }
#pragma unroll 4
    for (int u = 0; u < m; ++u) {
      const uint64_t x = (uint64_t(lkey[wave][u]) << 32) | uint32_t(lidx[wave][u]);
#pragma unroll
      for (int v = 0; v < kSelList / 64; ++v) rk[v] += x < me[v];
    }
#pragma unroll
    for (int v = 0; v < kSelList / 64; ++v)
      if (lane + 64 * v < m && rk[v] < want) ext[wave][rk[v]] = me[v];
    nx = min(m, want);
  } else {
    // many ties at T: repeated wave minima over all candidates
    uint64_t prev = 0;
    nx = 0;
    for (int r = 0; r < want; ++r) {
      uint64_t best = ~uint64_t(0);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint64_t v = (uint64_t(kr[j]) << 32) | uint32_t(lane + 64 * j);
        if (((vm >> j) & 1u) && (r == 0 || v > prev) && v < best) best = v;
      }
      best = wave_min_u64(best);
      if (best == ~uint64_t(0)) break;  // wave-uniform
      if (lane == 0) ext[wave][r] = best;
      prev = best;
      ++nx;
    }
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  const int got = min(nx, K);
  for (int t = lane; t < got; t += 64) {
    const uint64_t v = ext[wave][t];
    const int64_t row = row_of(int32_t(v & 0xffffffffu));
    wk[wave][t] = uint32_t(v >> 32);
    wid[wave][t] = uint32_t(perm32[row]);
    wrow[wave][t] = row;
  }
  __threadfence_block();
  __builtin_amdgcn_wave_barrier();
  if (nx == K + 1 && uint32_t(ext[wave][K - 1] >> 32) == uint32_t(ext[wave][K] >> 32)) {
    // exact tie at the boundary: the tied places go to the smallest ids
    const uint32_t TT = uint32_t(ext[wave][K - 1] >> 32);
    int need = 0;
    for (int t = 0; t < K; ++t) need += wk[wave][t] == TT;
    uint64_t last = 0;
    for (int r = 0; r < need; ++r) {
      uint64_t best = ~uint64_t(0);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (!(((vm >> j) & 1u) && kr[j] == TT)) continue;
        const int64_t row = row_of(lane + 64 * j);
        const uint64_t v = (uint64_t(uint32_t(perm32[row])) << 32) | uint32_t(row);
        if ((r == 0 || v > last) && v < best) best = v;
      }
      best = wave_min_u64(best);
      if (lane == 0) {
        wid[wave][K - need + r] = uint32_t(best >> 32);
        wrow[wave][K - need + r] = int64_t(uint32_t(best & 0xffffffffu));
      }
      last = best;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
  // the winners ordered by (key, id); lane holds winners lane and lane + 64
  uint32_t mk[2], mi[2];
  int rank[2] = {0, 0};
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int t = lane + 64 * v;
    mk[v] = t < got ? wk[wave][t] : 0xffffffffu;
    mi[v] = t < got ? wid[wave][t] : 0xffffffffu;
  }
#pragma unroll 4
  for (int u = 0; u < got; ++u) {
    const uint32_t ku = wk[wave][u], iu = wid[wave][u];
#pragma unroll
    for (int v = 0; v < 2; ++v) rank[v] += (ku < mk[v]) || (ku == mk[v] && iu < mi[v]);
  }
  if (MODE == 0) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
      if (lane + 64 * v < got) {
        ids[q * kout + rank[v]] = int64_t(mi[v]);
        scores[q * kout + rank[v]] = key_score(mk[v]);
      }
    for (int t = got + lane; t < kout; t += 64) {
      ids[q * kout + t] = -1;
      scores[q * kout + t] = -INFINITY;
    }
  } else {
    // certified shortlist: every candidate within the margin of the k-th
    // best key (the largest winner key when all K places are taken)
    uint32_t tk = 0u;
#pragma unroll
    for (int v = 0; v < 2; ++v)
      if (lane + 64 * v < got) tk = max(tk, mk[v]);
    for (int o = 32; o > 0; o >>= 1) tk = max(tk, uint32_t(__shfl_xor(tk, o)));
    const uint32_t thr = cert_threshold(ca, q, got == K ? tk : 0xffffffffu, lane);
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (64 * j >= n) break;  // wave-uniform
      const bool in = ((vm >> j) & 1u) && kr[j] <= thr;
      const uint64_t bal = __ballot(in);
      if (in) slist[q * ca.cap + cnt + __popcll(bal & below)] = int32_t(row_of(lane + 64 * j));
      cnt += __popcll(bal);
    }
    if (lane == 0) ca.scnt[q] = cnt;
  }
}

// Precision form, second pass: exact fp32 inner products of the shortlisted
// rows (from the fp32 copy), then the top k.  One workgroup per query; one
// wave per row at a time, lanes over dimensions.
template <int KPMAX>
__global__ __launch_bounds__(kSelNT) void rerank_shortlist_kernel(
    const float* __restrict__ X, int32_t d, const float* __restrict__ Q, int64_t nq,
    const int32_t* __restrict__ slist, int32_t S, const int32_t* __restrict__ perm32, int32_t k,
    int64_t* __restrict__ ids, float* __restrict__ scores) {
  __shared__ SelShared sh;
  __shared__ uint64_t srt[KPMAX];
  __shared__ int32_t sidx[KPMAX];
  __shared__ float sc[4096];
  __shared__ int32_t rows[4096];
  __shared__ int32_t s_n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
    if (tid == 0) s_n = 0;
    __syncthreads();
    for (int t = tid; t < S; t += kSelNT) {
      const int32_t rw = slist[q * S + t];
      rows[t] = rw;
      if (rw >= 0) atomicMax(&s_n, t + 1);
    }
    __syncthreads();
    const int n = s_n;
    const float* qv = Q + q * d;
    for (int t = wave; t < n; t += kSelNT / 64) {
      const float* xr = X + int64_t(rows[t]) * d;
      float acc = 0.f;
      for (int l = lane; l < d; l += 64) acc += qv[l] * xr[l];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if (lane == 0) sc[t] = acc;
    }
    __syncthreads();
    const int KP = pow2_at_least(k);
    const int got = block_select<kSelNT>(
        n, k, KP, [&](int i) { return score_key(sc[i]); },
        [&](int i) { return uint32_t(perm32[rows[i]]); }, srt, sidx, sh);
    for (int t = tid; t < k; t += kSelNT) {
      if (t < got) {
        ids[q * k + t] = int64_t(srt[t] & 0xffffffffu);
        scores[q * k + t] = key_score(uint32_t(srt[t] >> 32));
      } else {
        ids[q * k + t] = -1;
        scores[q * k + t] = -INFINITY;
      }
    }
    __syncthreads();
  }
}

// Precision form, second pass for short lists (S <= 64): one wave per query.
// The wave scores 8 shortlisted rows per round (all their loads in flight
// together), 16 lanes per row, each lane owning the float4 slots
// [4 c + 64 j, 4 c + 64 j + 4) of the dimension range (every load instruction
// reads 256 contiguous bytes of each of 4 rows); lane partials are reduced
// over the 16 lanes by a fixed xor tree.  Then each
// lane ranks one candidate by (score desc, id asc).  Needs d % 4 == 0 and
// 16-byte aligned rows.
__global__ __launch_bounds__(256) void wave_shortlist_kernel(
    const float* __restrict__ X, int32_t d, const float* __restrict__ Q, int64_t nq,
    const int32_t* __restrict__ slist, int32_t S, const int32_t* __restrict__ perm32, int32_t k,
    int64_t* __restrict__ ids, float* __restrict__ scores) {
  __shared__ float sc[4][64];
  __shared__ uint32_t sid[4][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));  // uniform
  const int g = lane >> 4, c16 = lane & 15;
  // one query per wave, no loop
  const int64_t q = int64_t(blockIdx.x) * 4 + wave;
  if (q >= nq) return;
  {
    const int32_t myrow = lane < S ? slist[q * S + lane] : -1;
    const uint64_t valid = __ballot(myrow >= 0);
    const int n = valid == ~uint64_t(0) ? 64 : __ffsll((long long)~valid) - 1;  // valid prefix
    const float* qv = Q + q * d;
    // 8 rows per round (two groups of 4): every load of the round is issued
    // before its products are summed
    for (int t0 = 0; t0 < n; t0 += 8) {
      const int ta = min(t0 + g, n - 1), tb = min(t0 + 4 + g, n - 1);
      const float* xa = X + int64_t(__shfl(myrow, ta)) * d;
      const float* xb = X + int64_t(__shfl(myrow, tb)) * d;
      float acca = 0.f, accb = 0.f;
#pragma unroll 4
      for (int l = 4 * c16; l < d; l += 64) {
        const float4 va = *reinterpret_cast<const float4*>(xa + l);
        const float4 vb = *reinterpret_cast<const float4*>(xb + l);
        const float4 qq = *reinterpret_cast<const float4*>(qv + l);
        acca += va.x * qq.x;
        acca += va.y * qq.y;
        acca += va.z * qq.z;
        acca += va.w * qq.w;
        accb += vb.x * qq.x;
        accb += vb.y * qq.y;
        accb += vb.z * qq.z;
        accb += vb.w * qq.w;
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        acca += __shfl_xor(acca, o);
        accb += __shfl_xor(accb, o);
      }
      if (c16 == 0 && t0 + g < n) sc[wave][t0 + g] = acca;
      if (c16 == 0 && t0 + 4 + g < n) sc[wave][t0 + 4 + g] = accb;
    }
    if (lane < n) sid[wave][lane] = uint32_t(perm32[myrow]);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    if (lane < n) {
      const uint32_t mk = score_key(sc[wave][lane]), mi = sid[wave][lane];
      int rank = 0;
      for (int u = 0; u < n; ++u) {
        const uint32_t ku = score_key(sc[wave][u]), iu = sid[wave][u];
        rank += (ku < mk) || (ku == mk && iu < mi);
      }
      if (rank < k) {
        ids[q * k + rank] = int64_t(mi);
        scores[q * k + rank] = key_score(mk);
      }
    }
    for (int t = n + lane; t < k; t += 64) {
      ids[q * k + t] = -1;
      scores[q * k + t] = -INFINITY;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// Precision form, certified second pass: exact fp32 inner products of every
// listed row (from the fp32 copy) and the top k by (score desc, id asc).  One
// workgroup per query; the list is taken in chunks of kCertChunk rows, each
// merged with the best k so far.  16 lanes per row (float4 slots when d % 4
// == 0 and the rows are 16-byte aligned, else scalar), reduced over the 16
// lanes by a fixed xor tree.
constexpr int kCertChunk = 1024;

template <int KPMAX>
__global__ __launch_bounds__(kSelNT) void cert_rerank_kernel(
    const float* __restrict__ X, int32_t d, const float* __restrict__ Q, int64_t nq,
    const int32_t* __restrict__ slist, int64_t cap, const int32_t* __restrict__ scnt,
    const int32_t* __restrict__ perm32, int32_t k, int vec, int64_t* __restrict__ ids,
    float* __restrict__ scores) {
  __shared__ SelShared sh;
  __shared__ uint64_t srt[KPMAX];
  __shared__ int32_t sidx[KPMAX];
  __shared__ uint64_t best[KPMAX];
  __shared__ float sc[kCertChunk];
  __shared__ int32_t rows[kCertChunk];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int KP = pow2_at_least(k);
  for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const int32_t n = scnt[q];
    const float* qv = Q + q * d;
    int nb = 0;
    for (int32_t c0 = 0; c0 < n; c0 += kCertChunk) {
      const int m = min(kCertChunk, n - c0);
      for (int t = tid; t < m; t += kSelNT) rows[t] = slist[q * cap + c0 + t];
      __syncthreads();
      for (int t0 = 4 * wave; t0 < m; t0 += 4 * (kSelNT / 64)) {
        const int t = t0 + g;
        const float* xr = X + int64_t(rows[min(t, m - 1)]) * d;
        float acc = 0.f;
        if (vec) {
          for (int l = 4 * c16; l < d; l += 64) {
            const float4 v = *reinterpret_cast<const float4*>(xr + l);
            const float4 w = *reinterpret_cast<const float4*>(qv + l);
            acc += v.x * w.x;
            acc += v.y * w.y;
            acc += v.z * w.z;
            acc += v.w * w.w;
          }
        } else {
          for (int l = c16; l < d; l += 16) acc += xr[l] * qv[l];
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (c16 == 0 && t < m) sc[t] = acc;
      }
      __syncthreads();
      const int got = block_select<kSelNT>(
          m + nb, k, KP,
          [&](int i) { return i < m ? score_key(sc[i]) : uint32_t(best[i - m] >> 32); },
          [&](int i) { return i < m ? uint32_t(perm32[rows[i]]) : uint32_t(best[i - m]); }, srt,
          sidx, sh);
      for (int t = tid; t < got; t += kSelNT) best[t] = srt[t];
      nb = got;
      __syncthreads();
    }
    for (int t = tid; t < k; t += kSelNT) {
      if (t < nb) {
        ids[q * k + t] = int64_t(best[t] & 0xffffffffu);
        scores[q * k + t] = key_score(uint32_t(best[t] >> 32));
      } else {
        ids[q * k + t] = -1;
        scores[q * k + t] = -INFINITY;
      }
    }
    __syncthreads();
  }
}

// Certified second pass for k <= 64, one wave per query: the listed rows are
// scored 64 at a time (8 rows per round with all their loads in flight, 16
// lanes per row as in wave_shortlist_kernel), and each chunk is merged with
// the best k so far: every entry of the chunk and of the current best is
// ranked against all others by (score desc, id asc) through readlane, and the
// k first ranks become the new best, kept in LDS in rank order.
__global__ __launch_bounds__(256) void cert_wave_kernel(
    const float* __restrict__ X, int32_t d, const float* __restrict__ Q, int64_t nq,
    const int32_t* __restrict__ slist, int64_t cap, const int32_t* __restrict__ scnt,
    const int32_t* __restrict__ perm32, int32_t k, int vec, int64_t* __restrict__ ids,
    float* __restrict__ scores) {
  __shared__ float sc[4][64];
  __shared__ uint32_t bkey[4][64], bid[4][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));  // uniform
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t q = int64_t(blockIdx.x) * 4 + wave;
  if (q >= nq) return;
  {
    const int32_t n = scnt[q];
    const int32_t* lq = slist + q * cap;
    const float* qv = Q + q * d;
    int nb = 0;  // entries of the best list (wave-uniform)
    for (int32_t c0 = 0; c0 < n; c0 += 64) {
      const int m = min(64, n - c0);
      const int32_t myrow = lane < m ? lq[c0 + lane] : 0;
      for (int t0 = 0; t0 < m; t0 += 8) {
        const int ta = min(t0 + g, m - 1), tb = min(t0 + 4 + g, m - 1);
        const float* xa = X + int64_t(__shfl(myrow, ta)) * d;
        const float* xb = X + int64_t(__shfl(myrow, tb)) * d;
        float acca = 0.f, accb = 0.f;
        if (vec) {
#pragma unroll 4
          for (int l = 4 * c16; l < d; l += 64) {
            const float4 va = *reinterpret_cast<const float4*>(xa + l);
            const float4 vb = *reinterpret_cast<const float4*>(xb + l);
            const float4 qq = *reinterpret_cast<const float4*>(qv + l);
            acca += va.x * qq.x;
            acca += va.y * qq.y;
            acca += va.z * qq.z;
            acca += va.w * qq.w;
            accb += vb.x * qq.x;
            accb += vb.y * qq.y;
            accb += vb.z * qq.z;
            accb += vb.w * qq.w;
          }
        } else {
          for (int l = c16; l < d; l += 16) {
            acca += xa[l] * qv[l];
            accb += xb[l] * qv[l];
          }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
          acca += __shfl_xor(acca, o);
          accb += __shfl_xor(accb, o);
        }
        if (c16 == 0 && t0 + g < m) sc[wave][t0 + g] = acca;
        if (c16 == 0 && t0 + 4 + g < m) sc[wave][t0 + 4 + g] = accb;
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      // entry A of a lane: its chunk row; entry B: its place in the best list
      const uint32_t ka = lane < m ? score_key(sc[wave][lane]) : 0xffffffffu;
      const uint32_t ia = lane < m ? uint32_t(perm32[myrow]) : 0xffffffffu;
      const uint32_t kb = lane < nb ? bkey[wave][lane] : 0xffffffffu;
      const uint32_t ib = lane < nb ? bid[wave][lane] : 0xffffffffu;
      int ra = 0, rb = 0;
      for (int u = 0; u < 64; ++u) {
        const uint32_t ku = uint32_t(__builtin_amdgcn_readlane(int(ka), u));
        const uint32_t iu = uint32_t(__builtin_amdgcn_readlane(int(ia), u));
        const uint32_t kv = uint32_t(__builtin_amdgcn_readlane(int(kb), u));
        const uint32_t iv = uint32_t(__builtin_amdgcn_readlane(int(ib), u));
        const bool uok = u < m, vok = u < nb;
        ra += (uok && ((ku < ka) || (ku == ka && iu < ia))) + (vok && ((kv < ka) || (kv == ka && iv < ia)));
        rb += (uok && ((ku < kb) || (ku == kb && iu < ib))) + (vok && ((kv < kb) || (kv == kb && iv < ib)));
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      if (lane < m && ra < k) {
        bkey[wave][ra] = ka;
        bid[wave][ra] = ia;
      }
      if (lane < nb && rb < k) {
        bkey[wave][rb] = kb;
        bid[wave][rb] = ib;
      }
      nb = min(k, nb + m);
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
    }
    if (lane < k) {
      if (lane < nb) {
        ids[q * k + lane] = int64_t(bid[wave][lane]);
        scores[q * k + lane] = key_score(bkey[wave][lane]);
      } else {
        ids[q * k + lane] = -1;
        scores[q * k + lane] = -INFINITY;
      }
    }
  }
}

// ------------------------------------------------------------ debug exports
__global__ void debug_kernel(const int32_t* __restrict__ l1, const Pair* __restrict__ pairs,
                             const Pair* __restrict__ pw, int32_t H,
                             const int32_t* __restrict__ routed, int64_t nq, int32_t c,
                             int64_t* __restrict__ l1o, int32_t* __restrict__ ro,
                             int64_t* __restrict__ po) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < nq * H && l1o)
    for (int u = 0; u < 3; ++u) l1o[3 * t + u] = l1[3 * t + u];
  if (t < nq * c) {
    if (ro) ro[t] = routed[t];
    if (po)
      for (int32_t h = 0; h < H; ++h) {
        const Pair pr = pw ? pw[t * H + h] : pairs[t];
        int64_t* o = po + 3 * (t * H + h);
        o[0] = pr.j >= 0 ? pr.pos : 0;
        o[1] = pr.j >= 0 ? pr.s : 0;
        o[2] = pr.j >= 0 ? pr.len : 0;
      }
  }
}

// Wave-per-query selection; candidate keys live in registers when every
// query's candidate count (at most c * rcap) fits 64 R of them.
template <int MODE>
void launch_wave_select(hipStream_t st, const Pair* pairs, const float* sbuf, int32_t rcap,
                        int32_t c, int64_t nq, int32_t K, const int64_t* off,
                        const int32_t* perm32, int64_t* ids, float* scores, int32_t kout,
                        int32_t* slist, int drop, CertArgs ca, const uint32_t* bkey,
                        int32_t nbcap) {
  const int64_t nmax = int64_t(c) * rcap;
  const unsigned wgrid = unsigned((nq + 3) / 4);  // one wave per query (nq < 2^31)
  if (bkey)  // the block form (and the re-reading form past its limits)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 0>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca, bkey,
                       nbcap);
  else if (nmax <= 512)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 8>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
  else if (nmax <= 1024)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 16>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
  else if (nmax <= 1280)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 20>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
  else if (nmax <= 2048)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 32>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
  else if (nmax <= 4096)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 64>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
  else if (nmax <= 6144)
    hipLaunchKernelGGL((wave_select_kernel<MODE, 96>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
  else
    hipLaunchKernelGGL((wave_select_kernel<MODE, 0>), dim3(wgrid), dim3(256), 0, st, pairs, sbuf,
                       rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca,
                       (const uint32_t*)nullptr, 0);
}

// 64 < K <= 128 over at most 2,048 candidates per query.
template <int MODE>
void launch_wave_wide(hipStream_t st, const Pair* pairs, const float* sbuf, int32_t rcap,
                      int32_t c, int64_t nq, int32_t K, const int64_t* off, const int32_t* perm32,
                      int64_t* ids, float* scores, int32_t kout, int32_t* slist, int drop,
                      CertArgs ca) {
  const unsigned wgrid = unsigned((nq + 3) / 4);  // one wave per query (nq < 2^31)
  if (int64_t(c) * rcap <= 1024)
    hipLaunchKernelGGL((wave_select_wide_kernel<MODE, 16>), dim3(wgrid), dim3(256), 0, st, pairs,
                       sbuf, rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca);
  else
    hipLaunchKernelGGL((wave_select_wide_kernel<MODE, 32>), dim3(wgrid), dim3(256), 0, st, pairs,
                       sbuf, rcap, c, nq, K, off, perm32, ids, scores, kout, slist, drop, ca);
}

template <int RT, int NPCM>
void launch_score_n(const Index& ix, bool bf16, bool vec, bool bvec, unsigned grid, int ti,
                    const int32_t* cstart, const int32_t* wl, const Pair* pairs, int32_t c,
                    const float* Q, const __hip_bfloat16* Qb, float* sbuf, int32_t rcap,
                    int persistent, int32_t* ctr, const int32_t* alist, const uint32_t* pmask,
                    int32_t mw, uint32_t* bkey, int32_t nbcap, hipStream_t st) {
  const int32_t nt = ix.n_tiles[ti];
  if (bf16 && !bvec)
    hipLaunchKernelGGL((rerank_kernel<RT, kBF16W, false, false, NPCM>), dim3(grid), dim3(kRerankNT), 0,
                       st, (const void*)ix.Xb, ix.d, ix.tiles[ti], nt, cstart, wl, pairs, c,
                       (const void*)Qb, sbuf, rcap, persistent, ctr, 0, (const float*)nullptr,
                       alist, pmask, mw, ix.tile_blk[ti], bkey, nbcap);
  else if (bf16)
    hipLaunchKernelGGL((rerank_kernel<RT, kBF16W, true, false, NPCM>), dim3(grid), dim3(kRerankNT), 0,
                       st, (const void*)ix.Xbt, ix.d, ix.tiles[ti], nt, cstart, wl, pairs, c,
                       (const void*)Qb, sbuf, rcap, persistent, ctr, 0, (const float*)nullptr,
                       alist, pmask, mw, ix.tile_blk[ti], bkey, nbcap);
  else if (vec)
    hipLaunchKernelGGL((rerank_kernel<RT, kF32W, true, false, NPCM>), dim3(grid), dim3(kRerankNT), 0,
                       st, (const void*)ix.Xt, ix.d, ix.tiles[ti], nt, cstart, wl, pairs, c,
                       (const void*)Q, sbuf, rcap, persistent, ctr, 0, (const float*)nullptr,
                       alist, pmask, mw, ix.tile_blk[ti], bkey, nbcap);
  else
    hipLaunchKernelGGL((rerank_kernel<RT, kF32W, false, false, NPCM>), dim3(grid), dim3(kRerankNT), 0,
                       st, (const void*)ix.X, ix.d, ix.tiles[ti], nt, cstart, wl, pairs, c,
                       (const void*)Q, sbuf, rcap, persistent, ctr, 0, (const float*)nullptr,
                       alist, pmask, mw, ix.tile_blk[ti], bkey, nbcap);
}

template <int FMT, int NPCM>
void launch_wg_n(const Index& ix, const void* X, const void* Qv, const int32_t* cstart,
                 const int32_t* wl, const Pair* pairs, int32_t c, float* sbuf, int32_t rcap,
                 const uint32_t* pmask, int32_t mw, uint32_t* bkey, int32_t nbcap,
                 hipStream_t st) {
  const int32_t nt = ix.n_tiles[2];
  // the block keys' epilogue only in the instantiation that writes them
  if (bkey)
    hipLaunchKernelGGL((rerank_wg_kernel<FMT, NPCM, true>), dim3(chunk_grid(nt, tile_chunk(128))),
                       dim3(256), 0, st, X, ix.d, ix.tiles[2], nt, cstart, wl, pairs, c, Qv, sbuf,
                       rcap, pmask, mw, ix.tile_blk[2], bkey, nbcap);
  else
    hipLaunchKernelGGL((rerank_wg_kernel<FMT, NPCM, false>), dim3(chunk_grid(nt, tile_chunk(128))),
                       dim3(256), 0, st, X, ix.d, ix.tiles[2], nt, cstart, wl, pairs, c, Qv, sbuf,
                       rcap, pmask, mw, ix.tile_blk[2], bkey, nbcap);
}

// The workgroup rerank (128-row tiles, direct schedule) on the operand-ordered
// copy of the precision asked for; false when that copy is missing.
bool launch_score_wg(const Index& ix, bool bf16, const int32_t* cstart, const int32_t* wl,
                     const Pair* pairs, int32_t c, const float* Q, const __hip_bfloat16* Qb,
                     float* sbuf, int32_t rcap, int npcm, const uint32_t* pmask, int32_t mw,
                     uint32_t* bkey, int32_t nbcap, hipStream_t st) {
  if (bf16 ? !(ix.d % 64 == 0 && ix.Xbt)
           : !(ix.d % 32 == 0 && ix.Xt && (reinterpret_cast<uintptr_t>(Q) & 15) == 0))
    return false;
#define LIDER_WG(FMT, X, QP)                                                            \
  {                                                                                     \
    if (npcm <= 1)                                                                      \
      launch_wg_n<FMT, 1>(ix, X, QP, cstart, wl, pairs, c, sbuf, rcap, pmask, mw, bkey, \
                          nbcap, st);                                                   \
    else if (npcm == 2)                                                                 \
      launch_wg_n<FMT, 2>(ix, X, QP, cstart, wl, pairs, c, sbuf, rcap, pmask, mw, bkey, \
                          nbcap, st);                                                   \
    else if (npcm <= 4)                                                                 \
      launch_wg_n<FMT, 4>(ix, X, QP, cstart, wl, pairs, c, sbuf, rcap, pmask, mw, bkey, \
                          nbcap, st);                                                   \
    else                                                                                \
      launch_wg_n<FMT, 8>(ix, X, QP, cstart, wl, pairs, c, sbuf, rcap, pmask, mw, bkey, \
                          nbcap, st);                                                   \
  }
  if (bf16)
    LIDER_WG(kBF16W, (const void*)ix.Xbt, (const void*)Qb)
  else
    LIDER_WG(kF32W, (const void*)ix.Xt, (const void*)Q)
#undef LIDER_WG
  return true;
}

// npcm: 16-pair column blocks per pass (1, 2, 4 or 8; the per-wave rerank
// takes at most 2 with 128-row tiles, at most 4 with 64-row tiles).
template <int RT>
void launch_score(const Index& ix, bool bf16, int ti, const int32_t* cstart, const int32_t* wl,
                  const Pair* pairs, int32_t c, const float* Q, const __hip_bfloat16* Qb,
                  float* sbuf, int32_t rcap, int persistent, int grid_mult, int32_t* ctr,
                  const int32_t* alist, int npcm, const uint32_t* pmask, int32_t mw,
                  uint32_t* bkey, int32_t nbcap, hipStream_t st) {
  const int32_t nt = ix.n_tiles[ti];
  unsigned grid;
  if (persistent)  // grid_mult waves per SIMD
    grid = unsigned(std::max(8, 4 * ix.n_cu * grid_mult / 8 * 8));
  else
    grid = chunk_grid(nt, tile_chunk(RT));
  // the wide feeds read the operand-ordered copies; without one (no room at
  // build time), the row-major rows
  const bool vec = (ix.d % 32 == 0) && ((reinterpret_cast<uintptr_t>(Q) & 15) == 0) && ix.Xt;
  const bool bvec = ix.d % 64 == 0 && ix.Xbt;
#define LIDER_SCORE_ARGS                                                                   \
  ix, bf16, vec, bvec, grid, ti, cstart, wl, pairs, c, Q, Qb, sbuf, rcap, persistent, ctr, \
      alist, pmask, mw, bkey, nbcap, st
  if (npcm == 1)
    launch_score_n<RT, 1>(LIDER_SCORE_ARGS);
  else if (npcm == 2 || RT > 64)
    launch_score_n<RT, 2>(LIDER_SCORE_ARGS);
  else if (npcm == 4 || RT > 32)
    launch_score_n<(RT > 64 ? 64 : RT), 4>(LIDER_SCORE_ARGS);
  else
    launch_score_n<32, 8>(LIDER_SCORE_ARGS);
#undef LIDER_SCORE_ARGS
}

// Layer-1 window scores: the centroids (layer-1 order) are one "cluster" of C
// rows tiled by 64, every query is one pair with its r1-window; the query list
// is split over gridDim.y.
constexpr int kL1PairChunk = 256;

void launch_l1_scores(const Index& ix, bool fp8, int64_t nq, const int32_t* l1cs,
                      const Pair* l1pairs, const float* Q, const __hip_bfloat16* Qb, float* rs,
                      int32_t r1, hipStream_t st) {
  const int32_t nt = ix.n_l1_tiles;
  const dim3 grid(chunk_grid(nt, tile_chunk(64)), unsigned((nq + kL1PairChunk - 1) / kL1PairChunk));
  const bool vec = (ix.d % 16 == 0) && ((reinterpret_cast<uintptr_t>(Q) & 15) == 0);
  if (fp8 && ix.d % 32 != 0)
    hipLaunchKernelGGL((rerank_kernel<64, kFP8, false, false>), grid, dim3(kRerankNT), 0, st,
                       (const void*)ix.cent8, ix.d, ix.l1_tiles, nt, l1cs,
                       (const int32_t*)nullptr, l1pairs, 1, (const void*)Qb, rs, r1, 0,
                       (int32_t*)nullptr, kL1PairChunk, (const float*)ix.cent8_scale,
                       (const int32_t*)nullptr, (const uint32_t*)nullptr, 0, (const int32_t*)nullptr,
                       (uint32_t*)nullptr, 0);
  else if (fp8)
    hipLaunchKernelGGL((rerank_kernel<64, kFP8, true, false>), grid, dim3(kRerankNT), 0, st,
                       (const void*)ix.cent8, ix.d, ix.l1_tiles, nt, l1cs,
                       (const int32_t*)nullptr, l1pairs, 1, (const void*)Qb, rs, r1, 0,
                       (int32_t*)nullptr, kL1PairChunk, (const float*)ix.cent8_scale,
                       (const int32_t*)nullptr, (const uint32_t*)nullptr, 0, (const int32_t*)nullptr,
                       (uint32_t*)nullptr, 0);
  else if (vec)
    hipLaunchKernelGGL((rerank_kernel<64, kF32, true, false>), grid, dim3(kRerankNT), 0, st,
                       (const void*)ix.cent_l1, ix.d, ix.l1_tiles, nt, l1cs,
                       (const int32_t*)nullptr, l1pairs, 1, (const void*)Q, rs, r1, 0,
                       (int32_t*)nullptr, kL1PairChunk, (const float*)nullptr,
                       (const int32_t*)nullptr, (const uint32_t*)nullptr, 0, (const int32_t*)nullptr,
                       (uint32_t*)nullptr, 0);
  else
    hipLaunchKernelGGL((rerank_kernel<64, kF32, false, false>), grid, dim3(kRerankNT), 0, st,
                       (const void*)ix.cent_l1, ix.d, ix.l1_tiles, nt, l1cs,
                       (const int32_t*)nullptr, l1pairs, 1, (const void*)Q, rs, r1, 0,
                       (int32_t*)nullptr, kL1PairChunk, (const float*)nullptr,
                       (const int32_t*)nullptr, (const uint32_t*)nullptr, 0, (const int32_t*)nullptr,
                       (uint32_t*)nullptr, 0);
}

// Dense layer-1 scores (r1 = C) on the GEMM kernel: 128-row query tiles when
// that still gives at least 4 workgroups per CU, else 64-row tiles.
template <int MB>
void launch_l1_gemm_mb(const Index& ix, bool fp8, int64_t nq, const float* Q,
                       const __hip_bfloat16* Qb, float* rs, hipStream_t st) {
  const int64_t nblk = (nq + 32 * MB - 1) / (32 * MB) * ((ix.C + kGemmTileN - 1) / kGemmTileN);
  const dim3 grid(unsigned((nblk + 7) / 8 * 8));
  const bool vec = (ix.d % 16 == 0) && ((reinterpret_cast<uintptr_t>(Q) & 15) == 0);
  if (fp8 && ix.d % 32 == 0)
    hipLaunchKernelGGL((l1_gemm_kernel<kFP8, true, MB>), grid, dim3(256), 0, st, (const void*)Qb,
                       nq, (const void*)ix.cent8, ix.C, ix.d, (const float*)ix.cent8_scale, rs);
  else if (fp8)
    hipLaunchKernelGGL((l1_gemm_kernel<kFP8, false, MB>), grid, dim3(256), 0, st, (const void*)Qb,
                       nq, (const void*)ix.cent8, ix.C, ix.d, (const float*)ix.cent8_scale, rs);
  else if (vec)
    hipLaunchKernelGGL((l1_gemm_kernel<kF32, true, MB>), grid, dim3(256), 0, st, (const void*)Q,
                       nq, (const void*)ix.cent_l1, ix.C, ix.d, (const float*)nullptr, rs);
  else
    hipLaunchKernelGGL((l1_gemm_kernel<kF32, false, MB>), grid, dim3(256), 0, st, (const void*)Q,
                       nq, (const void*)ix.cent_l1, ix.C, ix.d, (const float*)nullptr, rs);
}

// bf16 query x bf16 centroid product (candidate scores of the exact routing).
// With la (d a multiple of 64 only), the same launch also runs the layer-1
// locate of every (query, array) item.  Qf (d a multiple of 64, 16-byte
// aligned): the split product of the fp32 queries and centroids instead.
void launch_l1_gemm_bf16(const Index& ix, int64_t nq, const __hip_bfloat16* Qb, float* rs,
                         hipStream_t st, const L1Args* la = nullptr, const float* Qf = nullptr) {
  if (ix.d % kLdsK == 0) {
    const int64_t nblk = (nq + 127) / 128 * ((ix.C + 127) / 128);
    const unsigned l1b = la ? unsigned((la->nq * la->H + 255) / 256 + 7) / 8 * 8 : 0u;
    const dim3 grid(l1b + unsigned((nblk + 7) / 8 * 8));
    if (Qf)
      hipLaunchKernelGGL(l1_gemm_lds_kernel<true>, grid, dim3(256), 0, st, (const void*)Qf, nq,
                         (const void*)ix.cent_l1, ix.C, ix.d, rs, la ? *la : L1Args{}, l1b);
    else
      hipLaunchKernelGGL(l1_gemm_lds_kernel<false>, grid, dim3(256), 0, st, (const void*)Qb, nq,
                         (const void*)ix.cent_l1_b, ix.C, ix.d, rs, la ? *la : L1Args{}, l1b);
    return;
  }
  const int64_t nblk4 = (nq + 127) / 128 * ((ix.C + kGemmTileN - 1) / kGemmTileN);
  const int mb = nblk4 >= int64_t(ix.n_cu) ? 4 : 2;  // operand traffic from L2 bounds it
  const int64_t nblk = (nq + 32 * mb - 1) / (32 * mb) * ((ix.C + kGemmTileN - 1) / kGemmTileN);
  const dim3 grid(unsigned((nblk + 7) / 8 * 8));
  const bool vec = ix.d % 32 == 0;
  if (vec && mb == 4)
    hipLaunchKernelGGL((l1_gemm_kernel<kBF16, true, 4>), grid, dim3(256), 0, st, (const void*)Qb,
                       nq, (const void*)ix.cent_l1_b, ix.C, ix.d, (const float*)nullptr, rs);
  else if (vec)
    hipLaunchKernelGGL((l1_gemm_kernel<kBF16, true, 2>), grid, dim3(256), 0, st, (const void*)Qb,
                       nq, (const void*)ix.cent_l1_b, ix.C, ix.d, (const float*)nullptr, rs);
  else if (mb == 4)
    hipLaunchKernelGGL((l1_gemm_kernel<kBF16, false, 4>), grid, dim3(256), 0, st, (const void*)Qb,
                       nq, (const void*)ix.cent_l1_b, ix.C, ix.d, (const float*)nullptr, rs);
  else
    hipLaunchKernelGGL((l1_gemm_kernel<kBF16, false, 2>), grid, dim3(256), 0, st, (const void*)Qb,
                       nq, (const void*)ix.cent_l1_b, ix.C, ix.d, (const float*)nullptr, rs);
}

void launch_l1_gemm(const Index& ix, bool fp8, int64_t nq, const float* Q,
                    const __hip_bfloat16* Qb, float* rs, hipStream_t st) {
  const int64_t nblk4 = (nq + 127) / 128 * ((ix.C + kGemmTileN - 1) / kGemmTileN);
  if (nblk4 >= 4 * int64_t(ix.n_cu))
    launch_l1_gemm_mb<4>(ix, fp8, nq, Q, Qb, rs, st);
  else
    launch_l1_gemm_mb<2>(ix, fp8, nq, Q, Qb, rs, st);
}

}  // namespace

size_t search_workspace(const Index& ix, int64_t nq, int32_t k, int32_t c, int32_t r,
                        const lider_search_opts& o) {
  return make_plan(ix, nq, k, c, r, o).total;
}

int run_search(const Index& ix, const float* Q, int64_t nq, int32_t k, int32_t c, int32_t r,
               int64_t* ids, float* scores, void* ws, size_t ws_bytes, hipStream_t st,
               const lider_search_opts& o, const lider_search_debug* dbg, hipEvent_t* ev) {
  const Plan p = make_plan(ix, nq, k, c, r, o);
  if (ws_bytes < p.total)
    return set_error(LIDER_EINVAL, "workspace too small: need " + std::to_string(p.total) +
                                       " bytes, got " + std::to_string(ws_bytes));
  char* W = static_cast<char*>(ws);
  int32_t* ctr = reinterpret_cast<int32_t*>(W + p.o_ctr);
  int32_t* qdig = reinterpret_cast<int32_t*>(W + p.o_qdig);
  float* qnorm = reinterpret_cast<float*>(W + p.o_qnorm);
  int32_t* l1 = reinterpret_cast<int32_t*>(W + p.o_l1);
  Pair* l1pairs = reinterpret_cast<Pair*>(W + p.o_l1p);
  int32_t* l1cs = reinterpret_cast<int32_t*>(W + p.o_l1cs);
  float* rs = reinterpret_cast<float*>(W + p.o_rs);
  double* rs64 = reinterpret_cast<double*>(W + p.o_rs64);
  int32_t* routed = reinterpret_cast<int32_t*>(W + p.o_routed);
  Pair* pairs = reinterpret_cast<Pair*>(W + p.o_pairs);
  int32_t* ccount = reinterpret_cast<int32_t*>(W + p.o_ccount);
  int32_t* cstart = reinterpret_cast<int32_t*>(W + p.o_cstart);
  int32_t* cfill = reinterpret_cast<int32_t*>(W + p.o_cfill);
  int32_t* wl = reinterpret_cast<int32_t*>(W + p.o_wl);
  float* sbuf = reinterpret_cast<float*>(W + p.o_sbuf);
  __hip_bfloat16* qb = reinterpret_cast<__hip_bfloat16*>(W + p.o_qb);
  int32_t* slist = reinterpret_cast<int32_t*>(W + p.o_slist);
  int32_t* aflag = reinterpret_cast<int32_t*>(W + p.o_aflag);
  int32_t* alist = reinterpret_cast<int32_t*>(W + p.o_alist);
  uint64_t* kq = reinterpret_cast<uint64_t*>(W + p.o_kq);
  int32_t* lst = reinterpret_cast<int32_t*>(W + p.o_lst);
  int32_t* rw = reinterpret_cast<int32_t*>(W + p.o_rw);
  Pair* pw = reinterpret_cast<Pair*>(W + p.o_pw);
  uint32_t* pmask = reinterpret_cast<uint32_t*>(W + p.o_mask);
  int32_t* rcand = reinterpret_cast<int32_t*>(W + p.o_rcand);
  int32_t* rcnt = reinterpret_cast<int32_t*>(W + p.o_rcnt);
  uint32_t* bkey = p.nbcap ? reinterpret_cast<uint32_t*>(W + p.o_bkey) : nullptr;
  const int32_t m = ix.m, C = ix.C, H = ix.H;
  const int64_t np = nq * c;
  const bool bf16 = o.precision == LIDER_BF16;

  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], st);
  };
  // fp8 centroids (precision form) only feed the window kernel
  const bool fp8 = bf16 && ix.cent8 && !p.l1_dense_rows;
  // Layer-1 scores: dense rows (every centroid; bf16 product unless fp32 is
  // asked for or the bf16 copy is missing) or the window kernel; then the
  // exact routing (or, for fp8 window scores, the approximate routing) over
  // each query's window or union list.  The bf16 queries these need are
  // written by the hash kernel.
  const bool l1b = !fp8 && (o.l1_dense == 0 || o.l1_dense >= 2) && ix.cent_l1_b;
  // the split bf16 product (three MFMAs per fragment pair) when c > 1 or asked
  // for; it reads the fp32 queries with 16-byte loads
  const bool split = l1b && ix.d % kLdsK == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0 &&
                     (o.l1_dense == 3 || (o.l1_dense == 0 && c > 1));
  mark(0);
  // the hash launch also clears the counters (it writes no status: digits are clamped)
  const HashZero zr{ctr, int32_t(kCtrWords), ccount, cfill, kCntCopies * C, 0};
  int rc = run_hash_ex(Q, nq, ix.d, ix.A, ix.b, ix.anorm, 2 * H * m, ix.w, qdig, ctr + 1, 1, qnorm,
                       st, ix.hash_kind, (fp8 || bf16 || l1b) ? qb : nullptr, &zr);
  if (rc != LIDER_OK) return rc;
  mark(1);
  const int64_t nl1 = nq * H;  // (query, array) layer-1 items
  const L1Args la{ix.models, ix.leaves, qdig, m, H, nq, C, p.r1, l1, l1pairs, l1cs,
                  o.expand_bits > 0 ? kq : (uint64_t*)nullptr};
  // the dense bf16 product on the LDS kernel carries the layer-1 locate in its
  // launch; otherwise it has a launch of its own
  const bool l1_fused = p.l1_dense_rows && l1b && ix.d % kLdsK == 0;
  if (l1_fused)
    launch_l1_gemm_bf16(ix, nq, qb, rs, st, &la, split ? Q : nullptr);
  else
    hipLaunchKernelGGL(l1_kernel, dim3(unsigned((nl1 + 255) / 256)), dim3(256), 0, st, la);
  if (o.expand_bits > 0)
    hipLaunchKernelGGL(expand_kernel, dim3(unsigned((nl1 + 3) / 4)), dim3(256), 0, st,
                       ix.l1_keys, (const int64_t*)nullptr, int64_t(C), l1pairs, nl1, kq, p.r1,
                       m, o.expand_bits, l1, H, int64_t(C));
  const unsigned qgrid = unsigned(std::min<int64_t>(nq, 65535));
  const unsigned wgrid = unsigned(std::min<int64_t>((nq + 3) / 4, 65535));
  // the window each routing kernel reads: (l1w[wst q + 1], l1w[wst q + 2]);
  // with several arrays and r1 < C, the union list in rw / lst
  const int32_t* l1w = l1;
  int32_t wst = 3 * H;
  const int32_t* lstp = nullptr;
  if (p.l1_list) {
    const size_t lds = 4 * size_t((C + 31) / 32) * 4;
    hipLaunchKernelGGL(l1_union_kernel, dim3(wgrid), dim3(256), lds, st, l1, H, nq, C, ix.l1map,
                       p.lcap, lst, rw);
    l1w = rw;
    wst = 3;
    lstp = lst;
  }
  double ecoef = dot_err_coef(ix.d);  // fp32 scores
  // absolute terms: subnormal products (d 2^-100) and, for the split product,
  // operand parts flushed or rounded below 2^-126 (a multiple of |q| + max|mu|)
  double eadd = double(ix.d) * 7.888609052210118e-31, esub = 0.0;
  if (!p.l1_dense_rows) {
    launch_l1_scores(ix, fp8, nq, l1cs, l1pairs, Q, qb, rs, p.r1, st);
    if (fp8) {
      // s (bq . e) with e the fp8 codes of mu / s: |q - bq| <= ub |q|;
      // |mu - s e| <= (u8 + 2^-22) |mu| + 2^-10 s sqrt(d) (normal / subnormal
      // codes, s = max|mu_l| / 448, the division's rounding); fp32
      // accumulation of the exact products and the final scaling
      const double ub = 0.00390625, u8 = 0.0625;
      const double sub = 0.0009765625 * std::sqrt(double(ix.d)) / 448.0;
      ecoef = (ub + (1.0 + ub) * (u8 + 2.384185791015625e-07 + sub) +
               1.1 * dot_err_coef(ix.d) * (1.0 + ub) + 2.0 * 5.9604644775390625e-08) * 1.01;
    }
  } else if (split) {
    if (!l1_fused) launch_l1_gemm_bf16(ix, nq, qb, rs, st, nullptr, Q);
    // x = h + l + r with |x - h| <= u |x|, |l| <= u (1 + u) |x|, |r| <= u^2 |x|
    // (u = 2^-8) for q and mu elementwise; the terms the three products drop,
    // h_q r_mu + l_q l_mu + l_q r_mu + r_q mu, are within (2 (1 + u)^2 + 1) u^2
    // sum |q_l mu_l|, and the fp32 accumulation of the 3d exact products within
    // dot_err_coef(3d) of their absolute sum, at most (1 + u)^2 (1 + 2u) sum
    // |q_l mu_l|; sum |q_l mu_l| <= |q| |mu|
    const double u = 0.00390625;
    ecoef = ((2.0 * (1.0 + u) * (1.0 + u) + 1.0) * u * u +
             dot_err_coef(3 * ix.d) * (1.0 + u) * (1.0 + u) * (1.0 + 2.0 * u)) * 1.01;
    eadd = 3.0 * double(ix.d) * 7.888609052210118e-31;
    esub = 3.0 * std::sqrt(double(ix.d)) * 1.1754943508222875e-38;  // 2^-126
  } else if (l1b) {
    if (!l1_fused) launch_l1_gemm_bf16(ix, nq, qb, rs, st);
    const double u = 0.00390625;  // 2^-8: bf16 rounding of each operand
    ecoef = 2.0 * u + u * u + dot_err_coef(ix.d) * (1.0 + u) * (1.0 + u);
  } else {
    launch_l1_gemm(ix, fp8, nq, Q, qb, rs, st);
  }
  const int32_t rstride = p.l1_dense_rows ? C : p.r1;
  const int dense = p.l1_dense_rows ? 1 : 0;
  {
    // every window is the whole dense row when r1 >= C with a single window per query
    const int whole = dense && !lstp && p.r1 >= C && o.expand_bits == 0;
    const unsigned fgrid = unsigned((nq + 3) / 4);  // one wave per query (nq < 2^31)
    if (p.lcap <= 16 * 64)
      hipLaunchKernelGGL(route_filter_kernel<16>, dim3(fgrid), dim3(256), 0, st, ix.d, nq,
                         ix.l1_order32, l1w, wst, lstp, p.lcap, rs, rstride, dense, qnorm,
                         ix.cent_norm_max, ecoef, eadd, esub, c, rcand, rcnt, routed, whole);
    else
      hipLaunchKernelGGL(route_filter_kernel<0>, dim3(fgrid), dim3(256), 0, st, ix.d, nq,
                         ix.l1_order32, l1w, wst, lstp, p.lcap, rs, rstride, dense, qnorm,
                         ix.cent_norm_max, ecoef, eadd, esub, c, rcand, rcnt, routed, whole);
    const unsigned rgrid =
        unsigned(std::min<int64_t>((nq + kRescoreWaves - 1) / kRescoreWaves, 65535));
    hipLaunchKernelGGL(route_rescore_kernel, dim3(rgrid), dim3(64 * kRescoreWaves), 0, st, Q, ix.d, nq,
                       ix.cent_l1, ix.l1_order32, l1w, wst, lstp, p.lcap, c, rcand, rcnt, rs64,
                       routed);
  }
  mark(2);
  Pair* pwp = H > 1 ? pw : nullptr;
  hipLaunchKernelGGL(pairs_kernel, dim3(unsigned((np * H + 255) / 256)), dim3(256), 0, st, ix.models,
                     ix.leaves, qdig, m, H, C, np, c, r, routed, pairs, pwp, ccount,
                     o.expand_bits > 0 ? kq : (uint64_t*)nullptr);
  if (o.expand_bits > 0)
    hipLaunchKernelGGL(expand_kernel, dim3(unsigned((np * H + 3) / 4)), dim3(256), 0, st,
                       ix.keys, ix.off, int64_t(0), H > 1 ? pw : pairs, np * H, kq, r, m,
                       o.expand_bits, (int32_t*)nullptr, H, ix.n);
  if (C <= kFusedScanMax) {
    hipLaunchKernelGGL(scan_scatter_kernel, dim3(unsigned(std::max<int64_t>(1, (np + 255) / 256))),
                       dim3(256), 0, st, ccount, C, pairs, np, cstart, cfill, wl);
  } else {
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, ccount, C, cstart);
    hipLaunchKernelGGL(scatter_kernel, dim3(unsigned((np + 255) / 256)), dim3(256), 0, st, pairs,
                       np, ccount, C, cstart, cfill, wl);
  }
  // several arrays: each listed pair's union of windows as a membership mask
  // over its cluster's rows, and its window set to the union's hull
  if (H > 1) {
    const int32_t nblk = int32_t((np + 3) / 4);
    hipLaunchKernelGGL(pair_mask_kernel, dim3(chunk_grid(nblk, kMaskChunk)), dim3(256),
                       4 * size_t(mask_copies(p.mw)) * (p.mw + 1) * 4, st, pw, H, wl, cstart + C,
                       ix.off, ix.amap16, ix.n, p.mw, pairs, pmask, nblk);
  }
  mark(3);
  const int ti = p.ti;
  const int tr = 32 << ti;
  const int gm = o.grid_mult > 0 ? o.grid_mult : 4;
  const int npcm = p.npcm;
  if (o.persistent == 2) {
    const int32_t nt = ix.n_tiles[ti];
    hipLaunchKernelGGL(zero_kernel, dim3(unsigned(std::min<int64_t>((nt + 255) / 256, 4096))),
                       dim3(256), 0, st, aflag, int64_t(nt));
    hipLaunchKernelGGL(mark_tiles_kernel, dim3(unsigned((np + 255) / 256)), dim3(256), 0, st,
                       pairs, np, tr, ix.tile_base[ti], aflag, alist, ctr + 16);
  }
  if (tr == 32)
    launch_score<32>(ix, bf16, ti, cstart, wl, pairs, c, Q, qb, sbuf, p.rcap, o.persistent, gm,
                     ctr + 8, alist, npcm, H > 1 ? pmask : (const uint32_t*)nullptr, p.mw, bkey,
                     p.nbcap, st);
  else if (tr == 64)
    launch_score<64>(ix, bf16, ti, cstart, wl, pairs, c, Q, qb, sbuf, p.rcap, o.persistent, gm,
                     ctr + 8, alist, npcm, H > 1 ? pmask : (const uint32_t*)nullptr, p.mw, bkey,
                     p.nbcap, st);
  else if (o.persistent || !launch_score_wg(ix, bf16, cstart, wl, pairs, c, Q, qb, sbuf, p.rcap,
                                            npcm, H > 1 ? pmask : (const uint32_t*)nullptr,
                                            p.mw, bkey, p.nbcap, st))
    launch_score<128>(ix, bf16, ti, cstart, wl, pairs, c, Q, qb, sbuf, p.rcap, o.persistent, gm,
                      ctr + 8, alist, npcm, H > 1 ? pmask : (const uint32_t*)nullptr, p.mw, bkey,
                      p.nbcap, st);
  mark(4);
  // the block selection's LDS key cache, sized to the candidates per query
  // (a fixed 32 KB cache held it to three workgroups per CU)
  const int32_t skc = int32_t(std::min<int64_t>(kKeyCache, int64_t(c) * p.rcap));
  if (!bf16) {
    if (k <= 64)
      launch_wave_select<0>(st, pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids,
                            scores, k, slist, int(H > 1), CertArgs(), bkey, p.nbcap);
    else if (k <= 128 && int64_t(c) * p.rcap <= 2048)
      launch_wave_wide<0>(st, pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                          slist, int(H > 1), CertArgs());
    else if (k <= 128)
      hipLaunchKernelGGL((select_kernel<128, 0>), dim3(qgrid), dim3(kSelNT), skc * 4, st,
                         pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                         slist, int(H > 1), CertArgs(), skc);
    else
      hipLaunchKernelGGL((select_kernel<1024, 0>), dim3(qgrid), dim3(kSelNT), skc * 4, st,
                         pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                         slist, int(H > 1), CertArgs(), skc);
  } else if (p.cert) {
    // certified shortlist (every candidate within the bf16 error margin of the
    // k-th best), then the fp32 rerank of each query's list
    CertArgs ca;
    ca.Q = Q;
    ca.Qb = qb;
    ca.d = ix.d;
    ca.xmax = ix.xb_bound[0];
    ca.xres = ix.xb_bound[1];
    ca.xbmax = ix.xb_bound[2];
    ca.scnt = reinterpret_cast<int32_t*>(W + p.o_scnt);
    ca.cap = int64_t(c) * p.rcap;
    if (k <= 64)
      launch_wave_select<2>(st, pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                            slist, int(H > 1), ca, bkey, p.nbcap);
    else if (k <= 128 && int64_t(c) * p.rcap <= 2048)
      launch_wave_wide<2>(st, pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                          slist, int(H > 1), ca);
    else if (k <= 128)
      hipLaunchKernelGGL((select_kernel<128, 2>), dim3(qgrid), dim3(kSelNT), skc * 4, st,
                         pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                         slist, int(H > 1), ca, skc);
    else
      hipLaunchKernelGGL((select_kernel<1024, 2>), dim3(qgrid), dim3(kSelNT), skc * 4, st,
                         pairs, sbuf, p.rcap, c, nq, k, ix.off, ix.perm32, ids, scores, k,
                         slist, int(H > 1), ca, skc);
    const int vec = ix.d % 4 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
    if (k <= 64)
      hipLaunchKernelGGL(cert_wave_kernel, dim3(unsigned((nq + 3) / 4)), dim3(256), 0, st, ix.X,
                         ix.d, Q, nq, slist, ca.cap, ca.scnt, ix.perm32, k, vec, ids, scores);
    else if (k <= 128)
      hipLaunchKernelGGL(cert_rerank_kernel<128>, dim3(qgrid), dim3(kSelNT), 0, st, ix.X, ix.d, Q,
                         nq, slist, ca.cap, ca.scnt, ix.perm32, k, vec, ids, scores);
    else
      hipLaunchKernelGGL(cert_rerank_kernel<1024>, dim3(qgrid), dim3(kSelNT), 0, st, ix.X, ix.d,
                         Q, nq, slist, ca.cap, ca.scnt, ix.perm32, k, vec, ids, scores);
  } else {
    if (p.S <= 64)
      launch_wave_select<1>(st, pairs, sbuf, p.rcap, c, nq, p.S, ix.off, ix.perm32, ids,
                            scores, k, slist, int(H > 1), CertArgs(), bkey, p.nbcap);
    else if (p.S <= 512)
      hipLaunchKernelGGL((select_kernel<512, 1>), dim3(qgrid), dim3(kSelNT), skc * 4, st,
                         pairs, sbuf, p.rcap, c, nq, p.S, ix.off, ix.perm32, ids, scores, k,
                         slist, int(H > 1), CertArgs(), skc);
    else
      hipLaunchKernelGGL((select_kernel<4096, 1>), dim3(qgrid), dim3(kSelNT), skc * 4, st,
                         pairs, sbuf, p.rcap, c, nq, p.S, ix.off, ix.perm32, ids, scores, k,
                         slist, int(H > 1), CertArgs(), skc);
    if (p.S <= 64 && ix.d % 4 == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0)
      hipLaunchKernelGGL(wave_shortlist_kernel, dim3(unsigned((nq + 3) / 4)), dim3(256), 0, st,
                         ix.X, ix.d, Q, nq, slist, p.S, ix.perm32, k, ids, scores);
    else if (k <= 128)
      hipLaunchKernelGGL(rerank_shortlist_kernel<128>, dim3(qgrid), dim3(kSelNT), 0, st, ix.X,
                         ix.d, Q, nq, slist, p.S, ix.perm32, k, ids, scores);
    else
      hipLaunchKernelGGL(rerank_shortlist_kernel<1024>, dim3(qgrid), dim3(kSelNT), 0, st, ix.X,
                         ix.d, Q, nq, slist, p.S, ix.perm32, k, ids, scores);
  }
  mark(5);
  if (dbg) {
    if (dbg->qdigits_dev)
      (void)hipMemcpyAsync(dbg->qdigits_dev, qdig, size_t(nq) * 2 * H * m * 4,
                           hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(debug_kernel, dim3(unsigned((std::max(np, nl1) + 255) / 256 + 1)),
                       dim3(256), 0, st, l1, pairs, H > 1 ? pw : (const Pair*)nullptr, H, routed,
                       nq, c, dbg->l1_dev, dbg->routed_dev, dbg->pairs_dev);
  }
  return check_hip(hipGetLastError(), "search kernels");
}

}  // namespace lider
