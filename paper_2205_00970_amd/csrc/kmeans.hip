// k-means clustering of the corpus (Sections 3.2, 3.3.2): Lloyd iterations.
//
// Assignment = argmin_j |x - mu_j|^2 decided in FP64 with ties to the smaller
// j.  The distances come from an fp32 MFMA GEMM (g_j = |mu_j|^2 - 2 x.mu_j, the
// |x|^2 term is common to all j); when the best and second-best fp32 values are
// closer than twice a rigorous rounding-error bound, the point is queued and
// all its distances are recomputed sequentially in FP64 (sum over dimensions of
// (x_l - mu_l)^2, no contraction), which reproduces the FP64 definition.
//
// Update = FP64 mean of each cluster's members summed in ascending id order,
// rounded once to fp32; an empty cluster keeps its centroid.

#include <algorithm>

#include "lider_internal.hpp"

namespace lider {

__global__ void zero_i32_kernel2(int32_t* p, int64_t cnt) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cnt;
       t += int64_t(gridDim.x) * blockDim.x)
    p[t] = 0;
}

// |mu_j|^2 in fp32 and an upper bound of max_j |mu_j| (as float bits, atomicMax).
__global__ void cnorm_kernel(const float* __restrict__ cent, int32_t C, int32_t d,
                             float* __restrict__ cnorm, uint32_t* __restrict__ maxbits) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= C) return;
  float s = 0.f;
  for (int l = lane; l < d; l += 64) {
    float v = cent[int64_t(j) * d + l];
    s += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) {
    cnorm[j] = s;
    const double gam = double(d + 2) * 5.9604644775390625e-08;
    float ub = float(sqrt(double(s) * (1.0 + 2.0 * gam)) * (1.0 + 9.5367431640625e-07));
    atomicMax(maxbits, __float_as_uint(ub));
  }
}

struct Best {
  float bv;
  int32_t bi;
  float sv;
};

__device__ inline void best_push(Best& b, float g, int32_t j) {
  if (g < b.bv || (g == b.bv && j < b.bi)) {
    b.sv = b.bv;
    b.bv = g;
    b.bi = j;
  } else if (g < b.sv) {
    b.sv = g;
  }
}

__device__ inline Best best_merge(const Best& a, const Best& b) {
  Best r;
  if (b.bv < a.bv || (b.bv == a.bv && b.bi < a.bi)) {
    r.bv = b.bv;
    r.bi = b.bi;
    r.sv = fminf(a.bv, b.sv);
  } else {
    r.bv = a.bv;
    r.bi = a.bi;
    r.sv = fminf(b.bv, a.sv);
  }
  return r;
}

// One wave = 16 points; it sweeps all centroids 64 at a time (4 MFMA column
// tiles of 16), keeping per-lane best / second-best, then reduces over the 16
// lanes that hold the same points.
template <bool VEC>
__global__ __launch_bounds__(256) void assign_kernel(
    const float* __restrict__ X, int64_t n, int32_t d, const float* __restrict__ cent,
    const float* __restrict__ cnorm, const uint32_t* __restrict__ maxbits, int32_t C,
    int32_t* __restrict__ assign, const int32_t* __restrict__ prev, int32_t* __restrict__ changed,
    int64_t* __restrict__ amb, int32_t* __restrict__ amb_count) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, s = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 64 + wave * 16;
  if (row0 >= n) return;
  int64_t myrow = row0 + i;
  if (myrow >= n) myrow = n - 1;
  const float* xr = X + myrow * d;
  Best b[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    b[e].bv = INFINITY;
    b[e].bi = 0x7fffffff;
    b[e].sv = INFINITY;
  }
  float ss = 0.f;
  const int dfull = VEC ? (d & ~15) : 0;
  for (int jg = 0; jg < C; jg += 64) {
    floatx4 acc[4];
    const float* cr[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      int j = jg + 16 * t + i;
      cr[t] = cent + int64_t(j < C ? j : C - 1) * d;
    }
    const bool first = jg == 0;
    for (int k0 = 0; k0 < dfull; k0 += 16) {
      const int kk = k0 + 4 * s;
      float4 xv = *reinterpret_cast<const float4*>(xr + kk);
      if (first) ss += xv.x * xv.x + xv.y * xv.y + xv.z * xv.z + xv.w * xv.w;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float4 cv = *reinterpret_cast<const float4*>(cr[t] + kk);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.x, cv.x, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.y, cv.y, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.z, cv.z, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv.w, cv.w, acc[t], 0, 0, 0);
      }
    }
    for (int k0 = dfull; k0 < d; k0 += 16) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int kk = k0 + 4 * s + e;
        const bool in = kk < d;
        float xv = in ? xr[kk] : 0.f;
        if (first) ss += xv * xv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float cv = in ? cr[t][kk] : 0.f;
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv, cv, acc[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = jg + 16 * t + i;
      if (j < C) {
        const float cn = cnorm[j];
#pragma unroll
        for (int e = 0; e < 4; ++e) best_push(b[e], cn - 2.f * acc[t][e], j);
      }
    }
  }
  ss += __shfl_xor(ss, 16);
  ss += __shfl_xor(ss, 32);
  // reduce over the 16 lanes (centroid columns) that share points 4s..4s+3
#pragma unroll
  for (int e = 0; e < 4; ++e) {
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      Best p;
      p.bv = __shfl_xor(b[e].bv, o);
      p.bi = __shfl_xor(b[e].bi, o);
      p.sv = __shfl_xor(b[e].sv, o);
      b[e] = best_merge(b[e], p);
    }
  }
  const double gam = double(d + 2) * 5.9604644775390625e-08;
  const double coef = dot_err_coef(d) + 2.384185791015625e-07;  // + 2^-22 for the fp32 combine
  const double M = double(__uint_as_float(*maxbits));
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ri = 4 * s + e;
    const float ssr = __shfl(ss, ri);
    const int64_t row = row0 + ri;
    if (i != 0 || row >= n) continue;
    const double xn = sqrt(double(ssr) * (1.0 + 2.0 * gam)) * (1.0 + 9.5367431640625e-07);
    const double E = coef * (M * M + 2.0 * xn * M) +
                     double(d + 2) * 8.881784197001252e-16 * (xn + M) * (xn + M) +
                     double(d) * 7.888609052210118e-31;
    const double gap = double(b[e].sv) - double(b[e].bv);
    if (C == 1 || gap > 4.0 * E) {
      assign[row] = b[e].bi;
      if (prev && prev[row] != b[e].bi) atomicAdd(changed, 1);
    } else {
      const int32_t slot = atomicAdd(amb_count, 1);
      amb[slot] = row;
    }
  }
}

// FP64 recompute for queued points: one block per point, threads over
// centroids, each distance a sequential sum without contraction.
__global__ __launch_bounds__(256) void assign_fixup_kernel(
    const float* __restrict__ X, int32_t d, const float* __restrict__ cent, int32_t C,
    int32_t* __restrict__ assign, const int32_t* __restrict__ prev, int32_t* __restrict__ changed,
    const int64_t* __restrict__ amb, const int32_t* __restrict__ amb_count) {
#pragma clang fp contract(off)
  __shared__ double sd[256];
  __shared__ int32_t sj[256];
  const int32_t cnt = *amb_count;
  for (int32_t t = blockIdx.x; t < cnt; t += gridDim.x) {
    const int64_t row = amb[t];
    const float* xr = X + row * d;
    double bd = INFINITY;
    int32_t bj = 0x7fffffff;
    for (int32_t j = threadIdx.x; j < C; j += blockDim.x) {
      const float* mu = cent + int64_t(j) * d;
      double acc = 0.0;
      for (int l = 0; l < d; ++l) {
        double df = double(xr[l]) - double(mu[l]);
        acc = acc + df * df;
      }
      if (acc < bd) {
        bd = acc;
        bj = j;
      }
    }
    sd[threadIdx.x] = bd;
    sj[threadIdx.x] = bj;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        double od = sd[threadIdx.x + o];
        int32_t oj = sj[threadIdx.x + o];
        if (od < sd[threadIdx.x] || (od == sd[threadIdx.x] && oj < sj[threadIdx.x])) {
          sd[threadIdx.x] = od;
          sj[threadIdx.x] = oj;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      assign[row] = sj[0];
      if (prev && prev[row] != sj[0]) atomicAdd(changed, 1);
    }
    __syncthreads();
  }
}

// scratch: cnorm [C] f32 | maxbits u32 | amb_count i32 | amb [n] i64
size_t kmeans_assign_scratch(int64_t n, int32_t C) {
  return (size_t(C) * 4 + 255) / 256 * 256 + 256 + size_t(n) * 8;
}

int run_kmeans_assign(const float* X, int64_t n, int32_t d, const float* cent, int32_t C,
                      int32_t* assign, const int32_t* prev, int32_t* changed, void* scratch,
                      hipStream_t st) {
  char* p = static_cast<char*>(scratch);
  float* cnorm = reinterpret_cast<float*>(p);
  p += (size_t(C) * 4 + 255) / 256 * 256;
  uint32_t* maxbits = reinterpret_cast<uint32_t*>(p);
  int32_t* amb_count = reinterpret_cast<int32_t*>(p + 4);
  p += 256;
  int64_t* amb = reinterpret_cast<int64_t*>(p);
  hipLaunchKernelGGL(zero_i32_kernel2, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<int32_t*>(maxbits), int64_t(2));
  hipLaunchKernelGGL(cnorm_kernel, dim3((C + 3) / 4), dim3(256), 0, st, cent, C, d, cnorm,
                     maxbits);
  const bool vec = (d % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(cent) & 15) == 0);
  const dim3 grid(unsigned((n + 63) / 64));
  if (vec)
    hipLaunchKernelGGL(assign_kernel<true>, grid, dim3(256), 0, st, X, n, d, cent, cnorm,
                       maxbits, C, assign, prev, changed, amb, amb_count);
  else
    hipLaunchKernelGGL(assign_kernel<false>, grid, dim3(256), 0, st, X, n, d, cent, cnorm,
                       maxbits, C, assign, prev, changed, amb, amb_count);
  hipLaunchKernelGGL(assign_fixup_kernel, dim3(1024), dim3(256), 0, st, X, d, cent, C, assign,
                     prev, changed, amb, amb_count);
  return check_hip(hipGetLastError(), "k-means assignment kernels");
}

// ------------------------------------------------------------------ update
__global__ void iota_kernel(int32_t* p, int64_t n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += int64_t(gridDim.x) * blockDim.x)
    p[t] = int32_t(t);
}

// off[j] = first position whose sorted key >= j  (j = 0..C)
__global__ void lower_bound_kernel(const uint32_t* __restrict__ sorted, int64_t n, int32_t C,
                                   int64_t* __restrict__ off) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > C) return;
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

// One thread per (cluster, dim): sequential FP64 sum over members (ascending
// id), mean rounded once to fp32.
__global__ void mean_kernel(const float* __restrict__ X, int32_t d,
                            const int32_t* __restrict__ members, const int64_t* __restrict__ off,
                            int32_t C, float* __restrict__ cent) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(C) * d) return;
  const int32_t j = int32_t(t / d);
  const int32_t l = int32_t(t - int64_t(j) * d);
  const int64_t a = off[j], e = off[j + 1];
  if (e == a) return;
  double s = 0.0;
  for (int64_t p = a; p < e; ++p) s = s + double(X[int64_t(members[p]) * d + l]);
  cent[t] = float(s / double(e - a));
}

static int sort_bits(int32_t C) {
  int b = 1;
  while ((int64_t(1) << b) < int64_t(C) + 1) ++b;
  return b;
}

// scratch: keys_out [n] u32 | iota [n] i32 | members [n] i32 | off [C+1] i64 | sort temp
size_t centroid_means_scratch(int64_t n, int32_t C) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al(size_t(n) * 4) * 3 + al((size_t(C) + 1) * 8) + al(radix_sort_temp_bytes(n, 4));
}

int run_centroid_means(const float* X, int64_t n, int32_t d, const int32_t* assign, int32_t C,
                       float* cent, void* scratch, size_t scratch_bytes, hipStream_t st) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char* p = static_cast<char*>(scratch);
  uint32_t* kout = reinterpret_cast<uint32_t*>(p);
  p += al(size_t(n) * 4);
  int32_t* io = reinterpret_cast<int32_t*>(p);
  p += al(size_t(n) * 4);
  int32_t* members = reinterpret_cast<int32_t*>(p);
  p += al(size_t(n) * 4);
  int64_t* off = reinterpret_cast<int64_t*>(p);
  p += al((size_t(C) + 1) * 8);
  size_t tmp = scratch_bytes - size_t(p - static_cast<char*>(scratch));
  hipLaunchKernelGGL(iota_kernel, dim3(1024), dim3(256), 0, st, io, n);
  const int rc = radix_sort_pairs<uint32_t>(reinterpret_cast<const uint32_t*>(assign), io, kout,
                                            members, n, sort_bits(C), p, tmp, st);
  if (rc != LIDER_OK) return rc;
  hipLaunchKernelGGL(lower_bound_kernel, dim3((C + 1 + 255) / 256), dim3(256), 0, st, kout, n, C,
                     off);
  const int64_t tot = int64_t(C) * d;
  hipLaunchKernelGGL(mean_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, X, d,
                     members, off, C, cent);
  return check_hip(hipGetLastError(), "centroid mean kernels");
}

// ----------------------------------------------------- farthest-first seeding
// Round t: D_i <- min(D_i, |x_i - c_{t-1}|^2) in fp32 (relative error <= e),
// then every row whose fp32 value is within the error band of the maximum is
// rescored exactly (FP64 minimum over all chosen centroids, sequential sums)
// and the FP64 argmax (ties to the smaller id) becomes centroid t.
constexpr double kFFRel = 1.1920928955078125e-07;  // 2^-23 per dimension (fp32 + FP64 side)

__global__ __launch_bounds__(256) void ff_update_kernel(const float* __restrict__ X, int64_t n,
                                                        int32_t d, const float* __restrict__ c,
                                                        float* __restrict__ D,
                                                        uint32_t* __restrict__ maxbits, int first) {
  __shared__ float wmax[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float mx = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 4 + wave; i < n; i += int64_t(gridDim.x) * 4) {
    const float* xr = X + i * d;
    float s = 0.f;
    for (int l = lane; l < d; l += 64) {
      const float t = xr[l] - c[l];
      s += t * t;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    float v = first ? s : fminf(D[i], s);
    if (lane == 0) D[i] = v;
    mx = fmaxf(mx, v);
  }
  if (lane == 0) wmax[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    atomicMax(maxbits, __float_as_uint(m));
  }
}

__global__ void ff_candidates_kernel(const float* __restrict__ D, int64_t n, int32_t d,
                                     const uint32_t* __restrict__ maxbits,
                                     int64_t* __restrict__ cand, int32_t* __restrict__ ncand) {
  const double e = double(d + 3) * kFFRel;
  const double M = double(__uint_as_float(*maxbits));
  const double T = M * (1.0 - 2.0 * e) / (1.0 + 2.0 * e) - double(d) * 7.888609052210118e-31;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (double(D[i]) >= T) cand[atomicAdd(ncand, 1)] = i;
  }
}

// Exact FP64 distance of each candidate to its nearest chosen centroid.
__global__ __launch_bounds__(256) void ff_exact_kernel(const float* __restrict__ X, int32_t d,
                                                       const float* __restrict__ cent, int32_t t,
                                                       const int64_t* __restrict__ cand,
                                                       const int32_t* __restrict__ ncand,
                                                       double* __restrict__ dex) {
#pragma clang fp contract(off)
  __shared__ double sd[256];
  const int32_t cnt = *ncand;
  for (int32_t k = blockIdx.x; k < cnt; k += gridDim.x) {
    const float* xr = X + cand[k] * d;
    double best = INFINITY;
    for (int32_t j = threadIdx.x; j < t; j += blockDim.x) {
      const float* mu = cent + int64_t(j) * d;
      double acc = 0.0;
      for (int l = 0; l < d; ++l) {
        double df = double(xr[l]) - double(mu[l]);
        acc = acc + df * df;
      }
      best = acc < best ? acc : best;
    }
    sd[threadIdx.x] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sd[threadIdx.x] = fmin(sd[threadIdx.x], sd[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) dex[k] = sd[0];
    __syncthreads();
  }
}

// FP64 argmax over the candidates (ties to the smaller row id); writes the
// new centroid row, resets the per-round counters.
__global__ __launch_bounds__(256) void ff_pick_kernel(const float* __restrict__ X, int32_t d,
                                                      float* __restrict__ cent, int32_t t,
                                                      int64_t* __restrict__ cand,
                                                      int32_t* __restrict__ ncand,
                                                      const double* __restrict__ dex,
                                                      uint32_t* __restrict__ maxbits) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int32_t cnt = *ncand;
  double v = -1.0;
  int64_t id = INT64_MAX;
  for (int32_t k = threadIdx.x; k < cnt; k += blockDim.x) {
    const double dv = dex[k];
    const int64_t ci = cand[k];
    if (dv > v || (dv == v && ci < id)) {
      v = dv;
      id = ci;
    }
  }
  bv[threadIdx.x] = v;
  bi[threadIdx.x] = id;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double ov = bv[threadIdx.x + o];
      const int64_t oi = bi[threadIdx.x + o];
      if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int64_t pick = bi[0] == INT64_MAX ? 0 : bi[0];  // no candidate only with NaN input
  for (int l = threadIdx.x; l < d; l += blockDim.x) cent[int64_t(t) * d + l] = X[pick * d + l];
  __syncthreads();
  if (threadIdx.x == 0) {
    *ncand = 0;
    *maxbits = 0;
  }
}

__global__ void gather_rows_kernel(const float* __restrict__ X, int32_t d,
                                   const int64_t* __restrict__ ids, int32_t cnt,
                                   float* __restrict__ out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(cnt) * d) return;
  const int64_t j = t / d;
  out[t] = X[ids[j] * d + (t - j * d)];
}

// Lloyd iterations into ix.cent / ix.assign.
int run_kmeans(Index& ix, const float* X, const int64_t* init_host, int32_t iters,
               int32_t seeding, hipStream_t st) {
  const int64_t n = ix.n;
  const int32_t C = ix.C, d = ix.d;
  int64_t* init_dev = nullptr;
  int32_t* bufs[2] = {nullptr, nullptr};
  int32_t* changed = nullptr;
  void* scr_a = nullptr;
  void* scr_m = nullptr;
  const size_t sa = kmeans_assign_scratch(n, C), sm = centroid_means_scratch(n, C);
  int rc = LIDER_OK;
  auto fail = [&](int code, const char* what) {
    rc = code == LIDER_ENOMEM ? set_error(LIDER_ENOMEM, std::string("out of device memory: ") + what)
                              : code;
  };
  if (hipMalloc(&init_dev, size_t(C) * 8) != hipSuccess ||
      hipMalloc(&bufs[0], size_t(n) * 4) != hipSuccess ||
      hipMalloc(&bufs[1], size_t(n) * 4) != hipSuccess || hipMalloc(&changed, 256) != hipSuccess ||
      hipMalloc(&scr_a, sa) != hipSuccess || hipMalloc(&scr_m, sm) != hipSuccess) {
    fail(LIDER_ENOMEM, "k-means buffers");
  }
  if (rc == LIDER_OK) {
    rc = check_hip(hipMemcpyAsync(init_dev, init_host, size_t(C) * 8, hipMemcpyHostToDevice, st),
                   "copy k-means initial ids");
  }
  if (rc == LIDER_OK) {
    const int64_t tot = int64_t(seeding ? 1 : C) * d;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st,
                       X, d, init_dev, seeding ? 1 : C, ix.cent);
  }
  if (rc == LIDER_OK && seeding == 1 && C > 1) {
    float* D = nullptr;
    int64_t* cand = nullptr;
    double* dex = nullptr;
    if (hipMalloc(&D, size_t(n) * 4) != hipSuccess || hipMalloc(&cand, size_t(n) * 8) != hipSuccess ||
        hipMalloc(&dex, size_t(n) * 8) != hipSuccess)
      fail(LIDER_ENOMEM, "farthest-first buffers");
    int32_t* ncand = changed;  // [0] candidate count, [1] max bits
    uint32_t* maxbits = reinterpret_cast<uint32_t*>(changed + 1);
    if (rc == LIDER_OK) {
      hipLaunchKernelGGL(zero_i32_kernel2, dim3(1), dim3(64), 0, st, changed, int64_t(2));
      const unsigned ub = unsigned(std::min<int64_t>((n + 3) / 4, 8192));
      const unsigned cb = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
      for (int32_t t = 1; t < C; ++t) {
        hipLaunchKernelGGL(ff_update_kernel, dim3(ub), dim3(256), 0, st, X, n, d,
                           ix.cent + int64_t(t - 1) * d, D, maxbits, t == 1 ? 1 : 0);
        hipLaunchKernelGGL(ff_candidates_kernel, dim3(cb), dim3(256), 0, st, D, n, d, maxbits,
                           cand, ncand);
        hipLaunchKernelGGL(ff_exact_kernel, dim3(256), dim3(256), 0, st, X, d, ix.cent, t, cand,
                           ncand, dex);
        hipLaunchKernelGGL(ff_pick_kernel, dim3(1), dim3(256), 0, st, X, d, ix.cent, t, cand,
                           ncand, dex, maxbits);
      }
      rc = check_hip(hipGetLastError(), "farthest-first seeding");
      if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "farthest-first seeding");
    }
    if (D) hipFree(D);
    if (cand) hipFree(cand);
    if (dex) hipFree(dex);
  }
  int cur = 0, fin = 0;
  int32_t it = 0;
  while (rc == LIDER_OK && it < iters) {
    hipLaunchKernelGGL(zero_i32_kernel2, dim3(1), dim3(64), 0, st, changed, int64_t(1));
    rc = run_kmeans_assign(X, n, d, ix.cent, C, bufs[cur], it > 0 ? bufs[cur ^ 1] : nullptr,
                           changed, scr_a, st);
    if (rc != LIDER_OK) break;
    if (it > 0) {
      int32_t h_changed = 0;
      rc = check_hip(hipMemcpyAsync(&h_changed, changed, 4, hipMemcpyDeviceToHost, st),
                     "read k-means change count");
      if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "k-means iteration");
      if (rc != LIDER_OK) break;
      if (h_changed == 0) {  // converged: centroids already are this assignment's means
        fin = cur;
        ++it;
        break;
      }
    }
    rc = run_centroid_means(X, n, d, bufs[cur], C, ix.cent, scr_m, sm, st);
    fin = cur;
    cur ^= 1;
    ++it;
  }
  ix.iters_run = it;
  if (rc == LIDER_OK)
    rc = check_hip(hipMemcpyAsync(ix.assign, bufs[fin], size_t(n) * 4, hipMemcpyDeviceToDevice, st),
                   "copy final assignment");
  if (rc == LIDER_OK) rc = check_hip(hipStreamSynchronize(st), "k-means");
  hipFree(init_dev);
  hipFree(changed);
  hipFree(scr_a);
  hipFree(scr_m);
  hipFree(bufs[0]);
  hipFree(bufs[1]);
  return rc;
}

}  // namespace lider
