// E2LSH projection digits h_i(x) = floor((a_i . x + b_i) / w) (Section 4; the
// integer-valued base hash under SK-LSH's element-wise order, Section 4.2), or
// random-hyperplane bits h_i(x) = [a_i . x >= 0] (the cosine variant, Section
// 4.1).
//
// The projection [rows x d] . [d x nh] runs on fp32 MFMA (v_mfma_f32_16x16x4f32,
// one wave = 16 rows x 16 hashes).  The digit is an integer decided by a
// floating-point value, so it must equal the FP64 definition exactly: a
// projection whose fp32 value lies within a rigorous rounding-error band of a
// bucket edge is queued and recomputed by a sequential FP64 dot product in
// dimension order (fp32 products are exact in FP64, so FMA or not, every
// rounding matches the definition).
#include "lider_internal.hpp"

namespace lider {

// Projection kernel.  Block = 4 waves = 16 rows x (up to) 32 hashes, the
// hashes [32 y, 32 y + 32) of grid row y; the waves split the dimension range (wave w owns a contiguous quarter of the 16-dimension
// steps).  Lane l of a wave owns row / hash (l % 16) and the dimension slot
// s = l / 16: per step it loads 4 consecutive dims [k0 + 4s, k0 + 4s + 4) of
// its row and of its hash vector and feeds them to 4 MFMAs (the k index of an
// MFMA only needs to map to the same dimension on both operands).  Partial
// projections are added in wave order through LDS.
template <bool VEC>
__global__ __launch_bounds__(256) void hash_kernel(
    const float* __restrict__ X, int64_t n, int32_t d, const float* __restrict__ A,
    const float* __restrict__ bvec, const float* __restrict__ anorm, int32_t nh, double w,
    int32_t* __restrict__ out, int64_t* __restrict__ list, int32_t* __restrict__ counter,
    int32_t* __restrict__ status, int clamp, float* __restrict__ rownorm, int kind) {
  __shared__ float part[4][32][16];  // [wave][hash][row]
  __shared__ float pss[4][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, s = lane >> 4;
  const int64_t row0 = int64_t(blockIdx.x) * 16;
  int64_t myrow = row0 + i;
  if (myrow >= n) myrow = n - 1;  // keep loads in bounds; outputs are skipped
  const float* xr = X + myrow * d;
  const int hb = int(blockIdx.y) * 32;  // first hash of this block
  const int nhc = min(32, nh - hb);     // hashes of this block
  const int h0 = hb + (i < nhc ? i : nhc - 1);
  const int h1 = hb + (16 + i < nhc ? 16 + i : nhc - 1);
  const float* a0 = A + int64_t(h0) * d;
  const float* a1 = A + int64_t(h1) * d;
  const bool two = nhc > 16;
  floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  float ss = 0.f;
  const int nk = (d + 15) / 16;
  const int k0s = wave * nk / 4, k1s = (wave + 1) * nk / 4;
  for (int ks = k0s; ks < k1s; ++ks) {
    const int kk = ks * 16 + 4 * s;
    float xe[4], ae[4], be[4];
    if (VEC && kk + 3 < d) {
      const float4 xv = *reinterpret_cast<const float4*>(xr + kk);
      const float4 av = *reinterpret_cast<const float4*>(a0 + kk);
      const float4 bv = *reinterpret_cast<const float4*>(a1 + kk);
      xe[0] = xv.x; xe[1] = xv.y; xe[2] = xv.z; xe[3] = xv.w;
      ae[0] = av.x; ae[1] = av.y; ae[2] = av.z; ae[3] = av.w;
      be[0] = bv.x; be[1] = bv.y; be[2] = bv.z; be[3] = bv.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool in = kk + e < d;
        xe[e] = in ? xr[kk + e] : 0.f;
        ae[e] = in ? a0[kk + e] : 0.f;
        be[e] = in ? a1[kk + e] : 0.f;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ss += xe[e] * xe[e];
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(xe[e], ae[e], acc0, 0, 0, 0);
      if (two) acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(xe[e], be[e], acc1, 0, 0, 0);
    }
  }
  // |x|^2 of row i over this wave's dims: sum the four dimension slots
  ss += __shfl_xor(ss, 16);
  ss += __shfl_xor(ss, 32);
  if (s == 0) pss[wave][i] = ss;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    part[wave][i][4 * s + e] = acc0[e];
    if (two) part[wave][16 + i][4 * s + e] = acc1[e];
  }
  __syncthreads();
  const double coef = dot_err_coef(d);
  const double gam = double(d + 2) * 5.9604644775390625e-08;
  for (int o = threadIdx.x; o < 16 * nhc; o += 256) {
    const int ri = o / nhc, hl = o - ri * nhc, hash = hb + hl;
    const int64_t row = row0 + ri;
    if (row >= n) continue;
    const float ssr = ((pss[0][ri] + pss[1][ri]) + pss[2][ri]) + pss[3][ri];
    const float sv = ((part[0][hl][ri] + part[1][hl][ri]) + part[2][hl][ri]) + part[3][hl][ri];
    const double xn = sqrt(double(ssr) * (1.0 + 2.0 * gam)) * (1.0 + 9.5367431640625e-07);
    if (rownorm && hash == 0) rownorm[row] = float(xn * (1.0 + 9.5367431640625e-07));
    const int64_t oi = row * nh + hash;
    if (kind == LIDER_HASH_SIGN) {  // bit = [a.x >= 0]: decided unless |a.x| is within the band
      const double E = coef * double(anorm[hash]) * xn + double(d) * 7.888609052210118e-31;
      if (!(fabs(double(sv)) > 2.0 * E)) {
        const int32_t slot = atomicAdd(counter, 1);
        list[slot] = oi;
      } else {
        out[oi] = sv > 0.f ? 1 : 0;
      }
      continue;
    }
    const double tv = (double(sv) + double(bvec[hash])) / w;
    const double E = (coef * double(anorm[hash]) * xn + double(d) * 7.888609052210118e-31) / w +
                     8.881784197001252e-16 * fabs(tv);
    const double fl = floor(tv);
    const double fr = tv - fl;
    const double dist = fr < 1.0 - fr ? fr : 1.0 - fr;
    if (!(dist > 2.0 * E)) {
      const int32_t slot = atomicAdd(counter, 1);
      list[slot] = oi;
    } else if (fl >= -2147483648.0 && fl <= 2147483647.0) {
      out[oi] = int32_t(fl);
    } else if (clamp) {
      out[oi] = fl < 0 ? INT32_MIN : INT32_MAX;
    } else {
      atomicExch(status, int32_t(LIDER_ERANGE));
    }
  }
}

// FP64 recompute of queued (row, hash) projections, one wave per entry.  The
// definition is the sequential FP64 sum in dimension order.  The wave first
// sums the same exact products (fp32 x fp32 is exact in FP64) in parallel; two
// FP64 sums of the same d terms in different orders differ by at most
// 2 (d-1) 2^-53 sum|p| (to first order), so when the parallel value is farther
// than a generous multiple of that from a bucket edge, both floors agree.
// Only entries inside that much narrower band run the sequential loop (one
// lane, operands staged in LDS).
constexpr int kFixupLds = 1024;

__device__ inline double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ __launch_bounds__(256) void hash_fixup_kernel(
    const float* __restrict__ X, int32_t d, const float* __restrict__ A,
    const float* __restrict__ bvec, int32_t nh, double w, int32_t* __restrict__ out,
    const int64_t* __restrict__ list, const int32_t* __restrict__ counter,
    int32_t* __restrict__ status, int clamp, int kind) {
  __shared__ float sx[4][kFixupLds], sa[4][kFixupLds];
  __shared__ int s_seq[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t cnt = *counter;
  const bool staged = d <= kFixupLds;
  for (int32_t t = blockIdx.x * 4 + wave; t < cnt; t += gridDim.x * 4) {
    const int64_t o = list[t];
    const int64_t row = o / nh;
    const int hash = int(o - row * nh);
    const float* xr = X + row * d;
    const float* ar = A + int64_t(hash) * d;
    double ps = 0.0, pa = 0.0;
    for (int l = lane; l < d; l += 64) {
      const float xv = xr[l], av = ar[l];
      if (staged) {
        sx[wave][l] = xv;
        sa[wave][l] = av;
      }
      const double pr = double(av) * double(xv);
      ps += pr;
      pa += fabs(pr);
    }
    ps = wave_sum_f64(ps);
    pa = wave_sum_f64(pa);
    const double u = 1.1102230246251565e-16;  // 2^-53
    const bool sign = kind == LIDER_HASH_SIGN;
    const double bh = sign ? 0.0 : double(bvec[hash]);
    const double tp = sign ? ps : (ps + bh) / w;
    const double fp = sign ? (ps >= 0.0 ? 1.0 : 0.0) : floor(tp);
    const double fr = tp - floor(tp);
    const double dist = sign ? fabs(ps) : (fr < 1.0 - fr ? fr : 1.0 - fr);
    const double band = sign ? 8.0 * double(d) * u * pa
                             : 8.0 * (double(d) * u * pa + u * (fabs(ps) + fabs(bh))) / w +
                                   8.0 * u * fabs(tp);
    if (lane == 0) s_seq[wave] = !(dist > band);
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      double fl = fp;
      if (s_seq[wave]) {
        double sacc = 0.0;
        if (staged)
          for (int l = 0; l < d; ++l) sacc = sacc + double(sa[wave][l]) * double(sx[wave][l]);
        else
          for (int l = 0; l < d; ++l) sacc = sacc + double(ar[l]) * double(xr[l]);
        fl = sign ? (sacc >= 0.0 ? 1.0 : 0.0) : floor((sacc + bh) / w);
      }
      if (fl >= -2147483648.0 && fl <= 2147483647.0) {
        out[o] = int32_t(fl);
      } else if (clamp) {
        out[o] = fl < 0 ? INT32_MIN : INT32_MAX;
      } else {
        atomicExch(status, int32_t(LIDER_ERANGE));
      }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// Upper bounds of row norms (FP64, rounded up into fp32).
__global__ void norm_bound_kernel(const float* __restrict__ A, int32_t rows, int32_t d,
                                  float* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int l = 0; l < d; ++l) s += double(A[int64_t(r) * d + l]) * double(A[int64_t(r) * d + l]);
  out[r] = float(sqrt(s) * (1.0 + 9.5367431640625e-07));
}

__global__ void zero_i32_kernel(int32_t* p, int64_t cnt) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < cnt;
       t += int64_t(gridDim.x) * blockDim.x)
    p[t] = 0;
}

void launch_norm_bounds(const float* A, int32_t rows, int32_t d, float* out, hipStream_t st) {
  hipLaunchKernelGGL(norm_bound_kernel, dim3((rows + 63) / 64), dim3(64), 0, st, A, rows, d, out);
}

size_t hash_list_capacity(int64_t n, int32_t nh) { return size_t(n) * size_t(nh); }

// Enqueue digits of n rows into out [n x nh].  list must hold n*nh int64;
// counter and status are single device ints (zeroed here).  rownorm (nullable)
// receives an upper bound of each row's norm.
int run_hash_ex(const float* X, int64_t n, int32_t d, const float* A, const float* b,
                const float* anorm, int32_t nh, double w, int32_t* out, int64_t* list,
                int32_t* counter, int32_t* status, int clamp, float* rownorm, hipStream_t st,
                int kind) {
  if (n <= 0) return LIDER_OK;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(64), 0, st, counter, int64_t(1));
  const bool vec = (d % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const dim3 grid(unsigned((n + 15) / 16), unsigned((nh + 31) / 32));
  if (vec)
    hipLaunchKernelGGL(hash_kernel<true>, grid, dim3(256), 0, st, X, n, d, A, b, anorm, nh, w,
                       out, list, counter, status, clamp, rownorm, kind);
  else
    hipLaunchKernelGGL(hash_kernel<false>, grid, dim3(256), 0, st, X, n, d, A, b, anorm, nh, w,
                       out, list, counter, status, clamp, rownorm, kind);
  int64_t cap = n * nh;
  int64_t blocks = (cap + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(hash_fixup_kernel, dim3(unsigned(blocks)), dim3(256), 0, st, X, d, A, b, nh,
                     w, out, list, counter, status, clamp, kind);
  return check_hip(hipGetLastError(), "hash kernels");
}

}  // namespace lider
