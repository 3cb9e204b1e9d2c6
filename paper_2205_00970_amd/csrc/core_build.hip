// Core-model construction (Sections 3.1, 3.3.1, 5) for one layer of LIDER:
// items are hashed (E2LSH digits), each model's digit box gives a mixed-radix
// key, items are stably sorted by (model, key, id), keys are min-max re-scaled
// into [0, L-1] (Eq. (8)) and a two-stage linear RMI (Section 5.2) is fitted by
// least squares on (re-scaled key, location).  The same code builds layer 2
// (one model per cluster over its rows) and layer 1 (one model over the
// centroids).  RMI training is FP64 with the sums in location order and no
// contraction, one thread per model (root) or per (model, leaf).
#include <hip/hip_fp8.h>

#include <algorithm>

#include <cstring>

#include "lider_internal.hpp"

namespace lider {


namespace {


__global__ void fill_i32(int32_t* p, int64_t cnt, int32_t v) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cnt;
       t += int64_t(gridDim.x) * blockDim.x)
    p[t] = v;
}

__global__ void iota_i32(int32_t* p, int64_t n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    p[t] = int32_t(t);
}

__global__ void box_kernel(const int32_t* __restrict__ dig, int32_t m,
                           const int32_t* __restrict__ seg, int64_t n, int32_t* __restrict__ mins,
                           int32_t* __restrict__ maxs) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n * m;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t item = t / m;
    const int i = int(t - item * m);
    const int32_t sg = seg ? seg[item] : 0;
    const int32_t v = dig[t];
    atomicMin(&mins[int64_t(sg) * m + i], v);
    atomicMax(&maxs[int64_t(sg) * m + i], v);
  }
}

__global__ void count_kernel(const int32_t* __restrict__ seg, int64_t n,
                             int32_t* __restrict__ cnt) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    atomicAdd(&cnt[seg ? seg[t] : 0], 1);
}

// Box, effective digit count and leaf slot of each model.
__global__ void model_init_kernel(Model* __restrict__ mb, int32_t nseg, int32_t m, int32_t F,
                                  int64_t leaf_base, const int32_t* __restrict__ mins,
                                  const int32_t* __restrict__ maxs,
                                  const int32_t* __restrict__ cnt) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  Model M;
  M.L = cnt[j];
  M.leaf_off = leaf_base + int64_t(j) * F;
  M.kmin = M.kmax = 0;
  M.scale = 0.0;
  M.root_a = M.root_b = 0.0;
  M.F = F;
  M.m_eff = 0;
  for (int i = 0; i < LIDER_MAX_M; ++i) M.mins[i] = M.maxs[i] = 0;
  if (M.L > 0) {
    for (int i = 0; i < m; ++i) {
      M.mins[i] = mins[int64_t(j) * m + i];
      M.maxs[i] = maxs[int64_t(j) * m + i];
    }
    uint64_t prod = 1;
    int me = 0;
    for (; me < m; ++me) {
      uint64_t R = uint64_t(int64_t(M.maxs[me]) - int64_t(M.mins[me]) + 1);
      if (R > kKeyLimit / prod) break;
      prod *= R;
    }
    M.m_eff = me;
  }
  mb[j] = M;
}

__global__ void key_kernel(const int32_t* __restrict__ dig, int32_t m,
                           const int32_t* __restrict__ seg, int64_t n,
                           const Model* __restrict__ mb, uint64_t* __restrict__ K) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const Model& M = mb[seg ? seg[t] : 0];
    K[t] = encode_data(dig + t * m, M);
  }
}

__global__ void seg_of_kernel(const int32_t* __restrict__ seg, const int32_t* __restrict__ id1,
                              int64_t n, uint32_t* __restrict__ segk) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    segk[t] = seg ? uint32_t(seg[id1[t]]) : 0u;
}

__global__ void final_gather_kernel(const uint64_t* __restrict__ K1,
                                    const int32_t* __restrict__ id1,
                                    const int32_t* __restrict__ idx2, int64_t n,
                                    uint64_t* __restrict__ keys, int64_t* __restrict__ perm) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int32_t q = idx2[t];
    keys[t] = K1[q];
    perm[t] = id1[q];
  }
}

__global__ void lower_bound_u32(const uint32_t* __restrict__ sorted, int64_t n, int32_t nseg,
                                int64_t* __restrict__ off) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nseg) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (sorted[mid] < uint32_t(j))
      lo = mid + 1;
    else
      hi = mid;
  }
  off[j] = lo;
}

// Eq. (8) constants of each model.
__global__ void rescale_param_kernel(Model* __restrict__ mb, int32_t nseg,
                                     const int64_t* __restrict__ off,
                                     const uint64_t* __restrict__ keys) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  const int64_t a = off[j], e = off[j + 1];
  if (e == a) return;
  const uint64_t kmin = keys[a], kmax = keys[e - 1];
  mb[j].kmin = kmin;
  mb[j].kmax = kmax;
  mb[j].scale = kmax > kmin ? double(e - a - 1) / double(kmax - kmin) : 0.0;
}

__global__ void x_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ seg2,
                         int64_t n, const Model* __restrict__ mb, double* __restrict__ x) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    x[t] = rescale(keys[t], mb[seg2[t]]);
}

// Least squares of location on re-scaled key over the positions [a, e) of one
// model whose leaf equals `leaf` (-1: all), sums in location order.
__device__ void ols_range(const double* __restrict__ x, const int32_t* __restrict__ lf, int64_t a,
                          int64_t e, int32_t leaf, double* slope, double* icpt, int64_t* count) {
#pragma clang fp contract(off)
  int64_t n = 0;
  double sx = 0.0, sy = 0.0;
  for (int64_t p = a; p < e; ++p) {
    if (leaf >= 0 && lf[p] != leaf) continue;
    sx = sx + x[p];
    sy = sy + double(p - a);
    ++n;
  }
  *count = n;
  if (n == 0) return;
  const double mx = sx / double(n), my = sy / double(n);
  double sxx = 0.0, sxy = 0.0;
  for (int64_t p = a; p < e; ++p) {
    if (leaf >= 0 && lf[p] != leaf) continue;
    const double dx = x[p] - mx;
    const double dy = double(p - a) - my;
    sxx = sxx + dx * dx;
    sxy = sxy + dx * dy;
  }
  *slope = sxx > 0.0 ? sxy / sxx : 0.0;
  *icpt = my - (*slope) * mx;
}

__global__ void root_kernel(Model* __restrict__ mb, int32_t nseg, const int64_t* __restrict__ off,
                            const double* __restrict__ x) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nseg) return;
  const int64_t a = off[j], e = off[j + 1];
  if (e == a) return;
  double s = 0.0, c = 0.0;
  int64_t cnt;
  ols_range(x, nullptr, a, e, -1, &s, &c, &cnt);
  mb[j].root_a = s;
  mb[j].root_b = c;
}

__global__ void leaf_index_kernel(const double* __restrict__ x, const uint32_t* __restrict__ seg2,
                                  int64_t n, const Model* __restrict__ mb,
                                  int32_t* __restrict__ lf) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x) {
    const Model& M = mb[seg2[t]];
    lf[t] = leaf_of(M.root_a, M.root_b, M.F, M.L, x[t]);
  }
}

// One thread per (model, leaf): fit (empty leaf copies the root), then the
// min / max of (true location - predicted location) over the leaf's items.
__global__ void leaf_fit_kernel(const Model* __restrict__ mb, int32_t nseg, int32_t F,
                                const int64_t* __restrict__ off, const double* __restrict__ x,
                                const int32_t* __restrict__ lf, double* __restrict__ leaves,
                                int32_t* __restrict__ leaf_err) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nseg) * F) return;
  const int32_t j = int32_t(t / F);
  const int32_t leaf = int32_t(t - int64_t(j) * F);
  const Model M = mb[j];
  const int64_t slot = M.leaf_off + leaf;
  const int64_t a = off[j], e = off[j + 1];
  double s = 0.0, c = 0.0;
  int32_t elo = 0, ehi = 0;
  if (e > a) {
    int64_t cnt;
    ols_range(x, lf, a, e, leaf, &s, &c, &cnt);
    if (cnt == 0) {
      s = M.root_a;
      c = M.root_b;
    } else {
      bool seen = false;
      for (int64_t p = a; p < e; ++p) {
        if (lf[p] != leaf) continue;
        const int64_t err = (p - a) - pos_of(s, c, M.L, x[p]);
        if (!seen) {
          elo = ehi = int32_t(err);
          seen = true;
        } else {
          elo = err < elo ? int32_t(err) : elo;
          ehi = err > ehi ? int32_t(err) : ehi;
        }
      }
    }
  }
  leaves[2 * slot] = s;
  leaves[2 * slot + 1] = c;
  leaf_err[2 * slot] = elo;
  leaf_err[2 * slot + 1] = ehi;
}

int sort_bits_for(int64_t v) {
  int b = 1;
  while (b < 63 && (int64_t(1) << b) <= v) ++b;
  return b;
}

struct Bufs {
  std::vector<void*> ptrs;
  ~Bufs() {
    for (void* p : ptrs) hipFree(p);
  }
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    if (hipMalloc(&p, al256(count * sizeof(T) + 1)) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
};

}  // namespace

// Build one layer's core models over n items (digits per item id, model of
// each item in seg, NULL = all in model 0).  Outputs: perm [n] (location ->
// item id), keys [n], off [nseg + 1].
// binary: bit hashkeys; every model's box is [0, 1] (key = Decimal(bits)).
int build_layer(const int32_t* dig, int32_t m, const int32_t* seg, int64_t n, int32_t nseg,
                int32_t F, Model* mb, int64_t leaf_base, double* leaves, int32_t* leaf_err,
                int64_t* perm, uint64_t* keys, int64_t* off, bool binary, hipStream_t st) {
  Bufs B;
  int32_t* mins = B.get<int32_t>(size_t(nseg) * m);
  int32_t* maxs = B.get<int32_t>(size_t(nseg) * m);
  int32_t* cnt = B.get<int32_t>(size_t(nseg));
  uint64_t* K = B.get<uint64_t>(size_t(n));
  uint64_t* K1 = B.get<uint64_t>(size_t(n));
  int32_t* io = B.get<int32_t>(size_t(n));
  int32_t* id1 = B.get<int32_t>(size_t(n));
  uint32_t* segk = B.get<uint32_t>(size_t(n));
  uint32_t* seg2 = B.get<uint32_t>(size_t(n));
  int32_t* idx2 = B.get<int32_t>(size_t(n));
  double* x = B.get<double>(size_t(n));
  int32_t* lf = B.get<int32_t>(size_t(n));
  if (!mins || !maxs || !cnt || !K || !K1 || !io || !id1 || !segk || !seg2 || !idx2 || !x || !lf)
    return set_error(LIDER_ENOMEM, "out of device memory while building core models");
  const dim3 g(1024), blk(256);
  hipLaunchKernelGGL(fill_i32, g, blk, 0, st, mins, int64_t(nseg) * m, binary ? 0 : INT32_MAX);
  hipLaunchKernelGGL(fill_i32, g, blk, 0, st, maxs, int64_t(nseg) * m, binary ? 1 : INT32_MIN);
  hipLaunchKernelGGL(fill_i32, g, blk, 0, st, cnt, int64_t(nseg), 0);
  if (!binary) hipLaunchKernelGGL(box_kernel, g, blk, 0, st, dig, m, seg, n, mins, maxs);
  hipLaunchKernelGGL(count_kernel, g, blk, 0, st, seg, n, cnt);
  hipLaunchKernelGGL(model_init_kernel, dim3((nseg + 255) / 256), blk, 0, st, mb, nseg, m, F,
                     leaf_base, mins, maxs, cnt);
  hipLaunchKernelGGL(key_kernel, g, blk, 0, st, dig, m, seg, n, mb, K);
  hipLaunchKernelGGL(iota_i32, g, blk, 0, st, io, n);
  // stable sort by key (ties keep ascending id), then stable by model
  const size_t tb = radix_sort_temp_bytes(n, 8);
  void* tmp = B.get<char>(tb);
  if (!tmp) return set_error(LIDER_ENOMEM, "out of device memory for the key sort");
  int rc = radix_sort_pairs<uint64_t>(K, io, K1, id1, n, 53, tmp, tb, st);
  if (rc != LIDER_OK) return rc;
  hipLaunchKernelGGL(seg_of_kernel, g, blk, 0, st, seg, id1, n, segk);
  rc = radix_sort_pairs<uint32_t>(segk, io, seg2, idx2, n, sort_bits_for(nseg), tmp, tb, st);
  if (rc != LIDER_OK) return rc;
  hipError_t e;
  hipLaunchKernelGGL(final_gather_kernel, g, blk, 0, st, K1, id1, idx2, n, keys, perm);
  hipLaunchKernelGGL(lower_bound_u32, dim3((nseg + 1 + 255) / 256), blk, 0, st, seg2, n, nseg,
                     off);
  hipLaunchKernelGGL(rescale_param_kernel, dim3((nseg + 255) / 256), blk, 0, st, mb, nseg, off,
                     keys);
  hipLaunchKernelGGL(x_kernel, g, blk, 0, st, keys, seg2, n, mb, x);
  hipLaunchKernelGGL(root_kernel, dim3((nseg + 63) / 64), dim3(64), 0, st, mb, nseg, off, x);
  hipLaunchKernelGGL(leaf_index_kernel, g, blk, 0, st, x, seg2, n, mb, lf);
  const int64_t nl = int64_t(nseg) * F;
  hipLaunchKernelGGL(leaf_fit_kernel, dim3(unsigned((nl + 63) / 64)), dim3(64), 0, st, mb, nseg,
                     F, off, x, lf, leaves, leaf_err);
  e = hipGetLastError();
  if (e != hipSuccess) return check_hip(e, "core-model kernels");
  // temporaries are freed on return: wait for the work that uses them
  return check_hip(hipStreamSynchronize(st), "core-model build");
}

namespace {

__global__ void reorder_kernel(const float* __restrict__ X, int32_t d,
                               const int64_t* __restrict__ perm, int64_t n,
                               float* __restrict__ out, __hip_bfloat16* __restrict__ outb,
                               int32_t* __restrict__ perm32) {
  // one wave per row
  const int lane = threadIdx.x & 63;
  for (int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); r < n;
       r += int64_t(gridDim.x) * 4) {
    const int64_t src = perm[r];
    if (lane == 0 && perm32) perm32[r] = int32_t(src);
    for (int l = lane; l < d; l += 64) {
      const float v = X[src * d + l];
      out[r * d + l] = v;
      if (outb) outb[r * d + l] = __float2bfloat16(v);
    }
  }
}

__global__ void bf16_copy_kernel(const float* __restrict__ a, int64_t cnt,
                                 __hip_bfloat16* __restrict__ b) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cnt;
       t += int64_t(gridDim.x) * blockDim.x)
    b[t] = __float2bfloat16(a[t]);
}

__global__ void i64_to_i32(const int64_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    b[t] = int32_t(a[t]);
}

// fp8 e4m3 (OCP, largest finite 448) with one fp32 scale per row,
// s = max|v| / 448, rounded to nearest even by the HIP conversion.
__global__ void fp8_rows_kernel(const float* __restrict__ cent, int32_t C, int32_t d,
                                uint8_t* __restrict__ out, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= C) return;
  float mx = 0.f;
  for (int l = lane; l < d; l += 64) mx = fmaxf(mx, fabsf(cent[int64_t(j) * d + l]));
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const float s = mx > 0.f ? mx / 448.f : 1.f;
  if (lane == 0) scale[j] = s;
  for (int l = lane; l < d; l += 64) out[int64_t(j) * d + l] = uint8_t(
        __hip_cvt_float_to_fp8(cent[int64_t(j) * d + l] / s, __HIP_SATFINITE, __HIP_E4M3));
}

__global__ void cent_norm_max_kernel(const float* __restrict__ cent, int32_t C, int32_t d,
                                     uint32_t* __restrict__ maxbits) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= C) return;
  double s = 0.0;
  for (int l = lane; l < d; l += 64) s += double(cent[int64_t(j) * d + l]) * double(cent[int64_t(j) * d + l]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) atomicMax(maxbits, __float_as_uint(float(sqrt(s) * (1.0 + 9.5367431640625e-07))));
}

// Precision form: per row, |x|, |x - bf16(x)| and |bf16(x)| (bf16 rounded to
// nearest even like the corpus copy) from FP64 sums of squares, and their
// maxima over the rows as fp32 upper bounds (the squares are exact, the
// factor 1 + 2^-20 covers the sums' and the conversion's roundings).
__global__ void bf16_bounds_kernel(const float* __restrict__ X, int64_t n, int32_t d,
                                   uint32_t* __restrict__ maxbits) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); r < n;
       r += int64_t(gridDim.x) * 4) {
    double sx = 0.0, sr = 0.0, sb = 0.0;
    for (int l = lane; l < d; l += 64) {
      const float v = X[r * d + l];
      const double b = double(__bfloat162float(__float2bfloat16(v)));
      const double e = double(v) - b;
      sx += double(v) * double(v);
      sr += e * e;
      sb += b * b;
    }
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_xor(sx, o);
      sr += __shfl_xor(sr, o);
      sb += __shfl_xor(sb, o);
    }
    if (lane == 0) {
      const double up = 1.0 + 9.5367431640625e-07;
      atomicMax(&maxbits[0], __float_as_uint(float(sqrt(sx) * up)));
      atomicMax(&maxbits[1], __float_as_uint(float(sqrt(sr) * up)));
      atomicMax(&maxbits[2], __float_as_uint(float(sqrt(sb) * up)));
    }
  }
}

// Position maps between hashkey arrays: inv[perm0[p]] = p, then
// map[p] = inv[permh[p]] (array h's sorted position -> array 0's).
__global__ void inverse_kernel(const int64_t* __restrict__ perm, int64_t n,
                               int32_t* __restrict__ inv) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    inv[perm[t]] = int32_t(t);
}

__global__ void compose_kernel(const int64_t* __restrict__ permh, int64_t n,
                               const int32_t* __restrict__ inv, int32_t* __restrict__ map) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    map[t] = inv[permh[t]];
}

// Operand-ordered copy of the reordered corpus, one wave per 16-row block:
// block b takes rows src[b].x .. src[b].x + src[b].y - 1 of X (zeros past
// them).  fp32 (KS = 32): for every k-step and half h, lane l = i + 16 s writes
// dims [32 ks + 16 h + 4 s, + 4) of row i at float offset ((b nks + ks) 2 + h)
// 256 + 4 l.  bf16 (KS = 64): dims [64 ks + 32 h + 8 s, + 8), rounded to
// nearest even like the row-major bf16 copy, at element offset
// ((b nks + ks) 2 + h) 512 + 8 l.
template <bool BF>
__global__ __launch_bounds__(256) void tile_corpus_kernel(const float* __restrict__ X, int32_t d,
                                                          const int2* __restrict__ src,
                                                          int64_t nblk, void* __restrict__ out) {
  constexpr int KS = BF ? 64 : kTileKS, EPL = BF ? 8 : 4;  // dims per k-step, per lane
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, s = lane >> 4;
  const int32_t nks = d / KS;
  for (int64_t b = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6); b < nblk;
       b += int64_t(gridDim.x) * 4) {
    const int2 sr = src[b];
    const bool ok = i < sr.y;
    const float* xr = X + (int64_t(sr.x) + (ok ? i : 0)) * d;
    for (int32_t ks = 0; ks < nks; ++ks)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = ks * KS + (KS / 2) * h + EPL * s;
        const int64_t at = ((b * nks + ks) * 2 + h) * (64 * EPL) + EPL * lane;
        if (BF) {
          __hip_bfloat16* o = static_cast<__hip_bfloat16*>(out) + at;
#pragma unroll
          for (int e = 0; e < 8; ++e) o[e] = __float2bfloat16(ok ? xr[k + e] : 0.f);
        } else {
          const float4 v = ok ? *reinterpret_cast<const float4*>(xr + k) : float4{0.f, 0.f, 0.f, 0.f};
          *reinterpret_cast<float4*>(static_cast<float*>(out) + at) = v;
        }
      }
  }
}

}  // namespace

// Everything after the clustering, for each hashkey array h: layer-2 digits
// and models over the corpus, layer-1 digits and model over the centroids;
// the corpus and centroids reordered by array 0's order, and the maps from
// the other arrays' positions to array 0's.
int build_core_models(Index& ix, const float* Xin, hipStream_t st) {
  const int64_t n = ix.n;
  const int32_t d = ix.d, C = ix.C, m = ix.m, H = ix.H;
  Bufs B;
  int32_t* cs = B.get<int32_t>(64);  // [1] status
  int64_t* l1off = B.get<int64_t>(2);
  int32_t* inv = H > 1 ? B.get<int32_t>(size_t(n)) : nullptr;
  int32_t* inv1 = H > 1 ? B.get<int32_t>(size_t(C)) : nullptr;
  if (!cs || !l1off || (H > 1 && (!inv || !inv1)))
    return set_error(LIDER_ENOMEM, "out of device memory (build scratch)");
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, cs, int64_t(64), 0);
  const bool binary = ix.hash_kind == LIDER_HASH_SIGN;
  const int64_t nleaf = int64_t(C) * ix.F2 + ix.F1;  // leaves of one array
  int rc = LIDER_OK;
  for (int32_t h = 0; h < H; ++h) {
    const size_t r2 = size_t(H) * m + size_t(h) * m;  // layer-2 hash rows of array h
    int32_t* dig = ix.digits + size_t(h) * n * m;
    rc = run_hash_ex(Xin, n, d, ix.A + r2 * d, ix.b + r2, ix.anorm + r2, m, ix.w, dig, cs + 1, 0,
                     nullptr, st, ix.hash_kind);
    if (rc != LIDER_OK) return rc;
    rc = build_layer(dig, m, ix.assign, n, C, ix.F2, ix.models + size_t(h) * (C + 1),
                     int64_t(h) * nleaf, ix.leaves, ix.leaf_err, ix.perm + size_t(h) * n,
                     ix.keys + size_t(h) * n, ix.off, binary, st);
    if (rc != LIDER_OK) return rc;
    // layer 1: the centroids retriever
    const size_t r1 = size_t(h) * m;
    int32_t* dg1 = ix.l1_digits + size_t(h) * C * m;
    rc = run_hash_ex(ix.cent, C, d, ix.A + r1 * d, ix.b + r1, ix.anorm + r1, m, ix.w, dg1, cs + 1,
                     0, nullptr, st, ix.hash_kind);
    if (rc != LIDER_OK) return rc;
    rc = build_layer(dg1, m, nullptr, C, 1, ix.F1, ix.models + size_t(h) * (C + 1) + C,
                     int64_t(h) * nleaf + int64_t(C) * ix.F2, ix.leaves, ix.leaf_err,
                     ix.l1_order + size_t(h) * C, ix.l1_keys + size_t(h) * C, l1off, binary, st);
    if (rc != LIDER_OK) return rc;
  }
  {
    const int64_t blocks = std::min<int64_t>((n + 3) / 4, 65536);
    hipLaunchKernelGGL(reorder_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, Xin, d, ix.perm,
                       n, ix.X, ix.Xb, ix.perm32);
  }
  hipLaunchKernelGGL(reorder_kernel, dim3(unsigned((C + 3) / 4)), dim3(256), 0, st, ix.cent, d,
                     ix.l1_order, int64_t(C), ix.cent_l1, (__hip_bfloat16*)nullptr, ix.l1_order32);
  if (H > 1) {
    hipLaunchKernelGGL(inverse_kernel, dim3(1024), dim3(256), 0, st, ix.perm, n, inv);
    hipLaunchKernelGGL(inverse_kernel, dim3(64), dim3(256), 0, st, ix.l1_order, int64_t(C), inv1);
    for (int32_t h = 1; h < H; ++h) {
      hipLaunchKernelGGL(compose_kernel, dim3(1024), dim3(256), 0, st, ix.perm + size_t(h) * n, n,
                         inv, ix.amap + size_t(h - 1) * n);
      hipLaunchKernelGGL(compose_kernel, dim3(64), dim3(256), 0, st,
                         ix.l1_order + size_t(h) * C, int64_t(C), inv1,
                         ix.l1map + size_t(h - 1) * C);
    }
  }
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int32_t*>(ix.cent_norm_max),
                     int64_t(1), 0);
  hipLaunchKernelGGL(cent_norm_max_kernel, dim3((C + 3) / 4), dim3(256), 0, st, ix.cent, C, d,
                     reinterpret_cast<uint32_t*>(ix.cent_norm_max));
  if (ix.cent8)
    hipLaunchKernelGGL(fp8_rows_kernel, dim3((C + 3) / 4), dim3(256), 0, st, ix.cent_l1, C, d,
                       ix.cent8, ix.cent8_scale);
  if (ix.cent_l1_b)
    hipLaunchKernelGGL(bf16_copy_kernel, dim3(1024), dim3(256), 0, st, ix.cent_l1,
                       int64_t(C) * d, ix.cent_l1_b);
  rc = check_hip(hipGetLastError(), "index finishing kernels");
  if (rc != LIDER_OK) return rc;
  int32_t h_status = 0;
  rc = check_hip(hipMemcpyAsync(&h_status, cs + 1, 4, hipMemcpyDeviceToHost, st), "status");
  if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "index build");
  if (rc != LIDER_OK) return rc;
  if (h_status != 0)
    return set_error(LIDER_ERANGE, "a corpus or centroid hash value does not fit in int32");
  return finish_index(ix);
}

// amap16[h-1][o + p] = amap[h-1][o + p] - o: cluster j = blockIdx.x (rows o ..
// o + L - 1), array h = blockIdx.y + 1.
__global__ void amap16_kernel(const int32_t* __restrict__ amap, const int64_t* __restrict__ off,
                              int64_t n, uint16_t* __restrict__ amap16) {
  const int64_t o = off[blockIdx.x], L = off[blockIdx.x + 1] - o;
  const int64_t base = int64_t(blockIdx.y) * n + o;
  for (int64_t p = threadIdx.x; p < L; p += blockDim.x)
    amap16[base + p] = uint16_t(amap[base + p] - o);
}

// Host copy of the offsets, largest cluster, the 16-bit position maps and the
// rerank tile tables (all derived from the offsets and maps); shared by the
// build and the index loader.
int finish_index(Index& ix) {
  const int32_t C = ix.C;
  int rc = LIDER_OK;
  ix.h_off.resize(size_t(C) + 1);
  rc = check_hip(hipMemcpy(ix.h_off.data(), ix.off, (size_t(C) + 1) * 8, hipMemcpyDeviceToHost),
                 "copy offsets");
  if (rc != LIDER_OK) return rc;
  ix.max_cluster = 0;
  for (int32_t j = 0; j < C; ++j)
    ix.max_cluster = std::max<int64_t>(ix.max_cluster, ix.h_off[j + 1] - ix.h_off[j]);
  if (ix.H > 1 && ix.max_cluster > kMaxMultiCluster)
    return set_error(LIDER_EINVAL, "with n_arrays > 1 no cluster may hold more than 65536 rows");
  // several arrays: the position maps as positions within the cluster, 16 bits
  // each (the search's pair masks read them)
  if (ix.H > 1 && !ix.amap16 && ix.n > 0) {
    const size_t cnt = size_t(ix.H - 1) * size_t(ix.n) + 8;
    if (hipMalloc(&ix.amap16, al256(cnt * 2)) != hipSuccess) {
      ix.amap16 = nullptr;
      return set_error(LIDER_ENOMEM, "out of device memory (array position maps)");
    }
    hipLaunchKernelGGL(amap16_kernel, dim3(unsigned(C), unsigned(ix.H - 1)), dim3(256), 0,
                       nullptr, ix.amap, ix.off, ix.n, ix.amap16);
    rc = check_hip(hipDeviceSynchronize(), "array position maps");
    if (rc != LIDER_OK) return rc;
  }
  // clusters padded to whole 16-row blocks in the operand-ordered copy
  std::vector<int64_t> pblk(size_t(C) + 1, 0);  // first 16-row block of each cluster
  for (int32_t j = 0; j < C; ++j) pblk[j + 1] = pblk[j] + (ix.h_off[j + 1] - ix.h_off[j] + 15) / 16;
  const bool want_t = ix.d % kTileKS == 0;
  const bool want_bt = ix.storage == LIDER_BF16 && ix.d % 64 == 0 && !ix.Xbt;
  if ((want_t || want_bt) && pblk[C] > 0) {
    const int64_t nblk = pblk[C];
    std::vector<int2> src(static_cast<size_t>(nblk));
    for (int32_t j = 0; j < C; ++j)
      for (int64_t b = pblk[j]; b < pblk[j + 1]; ++b) {
        const int64_t r0 = ix.h_off[j] + 16 * (b - pblk[j]);
        src[b] = make_int2(int32_t(r0), int32_t(std::min<int64_t>(16, ix.h_off[j + 1] - r0)));
      }
    int2* dsrc = nullptr;
    const size_t elems = size_t(nblk) * 16 * size_t(ix.d);  // per copy
    if (hipMalloc(&dsrc, al256(src.size() * sizeof(int2))) != hipSuccess)
      return set_error(LIDER_ENOMEM, "out of device memory (operand-ordered corpus)");
    // the copies are an optimisation: without room for one, the rerank reads
    // the row-major rows instead
    if (want_t && hipMalloc(&ix.Xt, al256(elems * 4)) != hipSuccess) {
      (void)hipGetLastError();
      ix.Xt = nullptr;
    }
    if (want_bt && hipMalloc(&ix.Xbt, al256(elems * 2)) != hipSuccess) {
      (void)hipGetLastError();
      ix.Xbt = nullptr;
    }
    rc = check_hip(hipMemcpy(dsrc, src.data(), src.size() * sizeof(int2), hipMemcpyHostToDevice),
                   "copy block table");
    const dim3 grid(unsigned(std::min<int64_t>((nblk + 3) / 4, 65536)));
    if (rc == LIDER_OK && ix.Xt)
      hipLaunchKernelGGL(tile_corpus_kernel<false>, grid, dim3(256), 0, nullptr, ix.X, ix.d, dsrc,
                         nblk, (void*)ix.Xt);
    if (rc == LIDER_OK && ix.Xbt)
      hipLaunchKernelGGL(tile_corpus_kernel<true>, grid, dim3(256), 0, nullptr, ix.X, ix.d, dsrc,
                         nblk, (void*)ix.Xbt);
    if (rc == LIDER_OK) rc = check_hip(hipGetLastError(), "operand-ordered corpus");
    if (rc == LIDER_OK) rc = check_hip(hipDeviceSynchronize(), "operand-ordered corpus");
    (void)hipFree(dsrc);
    if (rc != LIDER_OK) return rc;
  }
  // the row-major bf16 copy only where the operand-ordered one is missing
  // (d not a multiple of 64, or no room for it)
  if (ix.storage == LIDER_BF16 && !ix.Xbt && !ix.Xb && ix.n > 0) {
    if (hipMalloc(&ix.Xb, al256(size_t(ix.n) * size_t(ix.d) * 2)) != hipSuccess) {
      ix.Xb = nullptr;
      return set_error(LIDER_ENOMEM, "out of device memory (bf16 corpus)");
    }
    hipLaunchKernelGGL(bf16_copy_kernel, dim3(4096), dim3(256), 0, nullptr, ix.X,
                       ix.n * int64_t(ix.d), ix.Xb);
    rc = check_hip(hipDeviceSynchronize(), "bf16 corpus");
    if (rc != LIDER_OK) return rc;
  }
  if (ix.storage == LIDER_BF16) {  // bounds of the precision form's certified shortlist
    uint32_t* mb = nullptr;
    uint32_t hb[4] = {0u, 0u, 0u, 0u};
    if (hipMalloc(&mb, 256) != hipSuccess)
      return set_error(LIDER_ENOMEM, "out of device memory (bf16 bounds)");
    rc = check_hip(hipMemcpy(mb, hb, 16, hipMemcpyHostToDevice), "bf16 bounds");
    if (rc == LIDER_OK) {
      hipLaunchKernelGGL(bf16_bounds_kernel, dim3(unsigned(std::min<int64_t>((ix.n + 3) / 4, 65536))),
                         dim3(256), 0, nullptr, ix.X, ix.n, ix.d, mb);
      rc = check_hip(hipGetLastError(), "bf16 bounds");
    }
    if (rc == LIDER_OK) rc = check_hip(hipMemcpy(hb, mb, 16, hipMemcpyDeviceToHost), "bf16 bounds");
    (void)hipFree(mb);
    if (rc != LIDER_OK) return rc;
    for (int i = 0; i < 3; ++i) std::memcpy(&ix.xb_bound[i], &hb[i], 4);
  }
  // rerank tile tables for 32/64/128-row tiles, 4 int32 per tile: cluster,
  // first in-cluster row, first row in the reordered corpus, rows in the tile;
  // and each tile's first 16-row block in the operand-ordered copy
  const int sizes[3] = {32, 64, 128};
  for (int s = 0; s < 3; ++s) {
    std::vector<int32_t> t, tb, tk;
    for (int32_t j = 0; j < C; ++j) {
      tb.push_back(int32_t(t.size() / 4));
      const int64_t L = ix.h_off[j + 1] - ix.h_off[j];
      for (int64_t r0 = 0; r0 < L; r0 += sizes[s]) {
        t.push_back(j);
        t.push_back(int32_t(r0));
        t.push_back(int32_t(ix.h_off[j] + r0));
        t.push_back(int32_t(std::min<int64_t>(sizes[s], L - r0)));
        tk.push_back(int32_t(pblk[j] + r0 / 16));
      }
    }
    tb.push_back(int32_t(t.size() / 4));
    if (hipMalloc(&ix.tile_blk[s], al256(tk.size() * 4 + 4)) != hipSuccess)
      return set_error(LIDER_ENOMEM, "out of device memory (tile table)");
    rc = check_hip(hipMemcpy(ix.tile_blk[s], tk.data(), tk.size() * 4, hipMemcpyHostToDevice),
                   "copy tile blocks");
    if (rc != LIDER_OK) return rc;
    if (hipMalloc(&ix.tile_base[s], al256(tb.size() * 4)) != hipSuccess)
      return set_error(LIDER_ENOMEM, "out of device memory (tile table)");
    rc = check_hip(hipMemcpy(ix.tile_base[s], tb.data(), tb.size() * 4, hipMemcpyHostToDevice),
                   "copy tile bases");
    if (rc != LIDER_OK) return rc;
    ix.n_tiles[s] = int32_t(t.size() / 4);
    if (hipMalloc(&ix.tiles[s], al256(t.size() * 4 + 4)) != hipSuccess)
      return set_error(LIDER_ENOMEM, "out of device memory (tile table)");
    rc = check_hip(hipMemcpy(ix.tiles[s], t.data(), t.size() * 4, hipMemcpyHostToDevice),
                   "copy tile table");
    if (rc != LIDER_OK) return rc;
  }
  {  // layer-1 tiles
    std::vector<int32_t> t;
    for (int32_t r0 = 0; r0 < C; r0 += 64) {
      t.push_back(0);
      t.push_back(r0);
      t.push_back(r0);
      t.push_back(std::min(64, C - r0));
    }
    ix.n_l1_tiles = int32_t(t.size() / 4);
    if (hipMalloc(&ix.l1_tiles, al256(t.size() * 4)) != hipSuccess)
      return set_error(LIDER_ENOMEM, "out of device memory (layer-1 tiles)");
    rc = check_hip(hipMemcpy(ix.l1_tiles, t.data(), t.size() * 4, hipMemcpyHostToDevice),
                   "copy layer-1 tiles");
  }
  return rc;
}

}  // namespace lider
