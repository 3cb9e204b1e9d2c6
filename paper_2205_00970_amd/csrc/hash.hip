// E2LSH projection digits h_i(x) = floor((a_i . x + b_i) / w) (Section 4; the
// integer-valued base hash under SK-LSH's element-wise order, Section 4.2), or
// random-hyperplane bits h_i(x) = [a_i . x >= 0] (the cosine variant, Section
// 4.1).
//
// The projection [rows x d] . [d x nh] runs on FP64 MFMA (v_mfma_f64_16x16x4f64,
// one wave = 16 rows x 16 hashes).  The digit is an integer decided by a
// floating-point value, so it must equal the FP64 definition exactly.  The
// fp32 x fp32 products are exact in FP64, so the MFMA sum differs from the
// sequential FP64 sum of the definition only by the rounding of its d + 3
// additions: within 8 (d + 4) 2^-53 |a| |x|.  A projection whose value lies
// within that band of a bucket edge (about 1e-10 relative at d = 768, so almost
// never) is listed and decided by hash_decide_wave in the same kernel, down to
// the sequential FP64 dot product in dimension order where needed.
#include "lider_internal.hpp"

namespace lider {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// FP64 decision of one projection whose MFMA value lay inside the band, by
// one wave.  The wave first sums the same exact products (fp32 x fp32 is
// exact in FP64) in parallel; two FP64 sums of the same d terms in different
// orders differ by at most 2 (d-1) 2^-53 sum|p| (to first order), so when the
// parallel value is farther than a generous multiple of that from a bucket
// edge, both floors agree.  Only entries inside that much narrower band run
// the sequential loop of the definition (one lane, dimension order).  The
// butterfly sums leave bit-identical totals on every lane, so the branch is
// wave-uniform.
__device__ void hash_decide_wave(const float* __restrict__ xr, const float* __restrict__ ar,
                                 int32_t d, double bh, double w, int kind, int clamp,
                                 int32_t* __restrict__ out, int32_t* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  double ps = 0.0, pa = 0.0;
  for (int l = lane; l < d; l += 64) {
    const double pr = double(ar[l]) * double(xr[l]);
    ps += pr;
    pa += fabs(pr);
  }
  ps = wave_sum_f64(ps);
  pa = wave_sum_f64(pa);
  const double u = 1.1102230246251565e-16;  // 2^-53
  const bool sign = kind == LIDER_HASH_SIGN;
  const double tp = sign ? ps : (ps + bh) / w;
  const double fr = tp - floor(tp);
  const double dist = sign ? fabs(ps) : (fr < 1.0 - fr ? fr : 1.0 - fr);
  const double band = sign ? 8.0 * double(d) * u * pa
                           : 8.0 * (double(d) * u * pa + u * (fabs(ps) + fabs(bh))) / w +
                                 8.0 * u * fabs(tp);
  if (lane != 0) return;
  double fl = sign ? (ps >= 0.0 ? 1.0 : 0.0) : floor(tp);
  if (!(dist > band)) {
    double sacc = 0.0;
    for (int l = 0; l < d; ++l) sacc = sacc + double(ar[l]) * double(xr[l]);
    fl = sign ? (sacc >= 0.0 ? 1.0 : 0.0) : floor((sacc + bh) / w);
  }
  if (fl >= -2147483648.0 && fl <= 2147483647.0) {
    *out = int32_t(fl);
  } else if (clamp) {
    *out = fl < 0 ? INT32_MIN : INT32_MAX;
  } else {
    atomicExch(status, int32_t(LIDER_ERANGE));
  }
}

// Projection kernel.  Block = 4 waves = 16 rows x (up to) 32 hashes, the
// hashes [32 y, 32 y + 32) of grid row y; the waves split the dimension range
// (wave w owns a contiguous quarter of the 16-dimension steps).  Lane l of a
// wave owns row / hash (l % 16) and the dimension slot s = l / 16: per step it
// loads 4 consecutive dims [k0 + 4s, k0 + 4s + 4) of its row and of its hash
// vectors and feeds them to 4 MFMAs (the k index of an MFMA only needs to map
// to the same dimension on both operands).  The next step's operands are
// loaded before the current step's MFMAs are issued.  Partial projections are
// added in wave order through LDS; the projections inside the band are listed
// in LDS and decided by hash_decide_wave after the block's other outputs.
// xb (nullable): the rows rounded to bf16 (round to nearest even), written by
// the blocks of grid row 0 from the values they load anyway.  z: counters
// the caller's later kernels need cleared, cleared by the blocks of grid row
// 0 (status must not be among them unless clamp is set: this kernel only
// writes status when it is not).
template <bool VEC>
__global__ __launch_bounds__(256) void hash_kernel(
    const float* __restrict__ X, int64_t n, int32_t d, const float* __restrict__ A,
    const float* __restrict__ bvec, const float* __restrict__ anorm, int32_t nh, double w,
    int32_t* __restrict__ out, int32_t* __restrict__ status, int clamp,
    float* __restrict__ rownorm, int kind, __hip_bfloat16* __restrict__ xb, HashZero z) {
  if (blockIdx.y == 0 && z.nz > 0) {
    for (int32_t t = int32_t(blockIdx.x) * 256 + threadIdx.x; t < z.nz;
         t += int32_t(gridDim.x) * 256) {
      if (z.a && t < z.na) z.a[t] = 0;
      if (z.b && t < z.nb) z.b[t] = 0;
      if (z.c && t < z.nb) z.c[t] = 0;
    }
  }
  __shared__ double part[4][32][16];  // [wave][hash][row]
  __shared__ float pss[4][16];
  __shared__ int32_t qlist[16 * 32];  // (row, hash) entries inside the band
  __shared__ int32_t qn;
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
  __hip_bfloat16* xbr = (xb && blockIdx.y == 0 && row0 + i < n) ? xb + (row0 + i) * d : nullptr;
  doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  float ss = 0.f;
  const int nk = (d + 15) / 16;
  const int k0s = wave * nk / 4, k1s = (wave + 1) * nk / 4;
  float xe[4], ae[4], be[4] = {0.f, 0.f, 0.f, 0.f};
  auto load = [&](int ks, float* xo, float* ao, float* bo) {
    const int kk = ks * 16 + 4 * s;
    if (VEC && kk + 3 < d) {
      const float4 xv = *reinterpret_cast<const float4*>(xr + kk);
      const float4 av = *reinterpret_cast<const float4*>(a0 + kk);
      xo[0] = xv.x; xo[1] = xv.y; xo[2] = xv.z; xo[3] = xv.w;
      ao[0] = av.x; ao[1] = av.y; ao[2] = av.z; ao[3] = av.w;
      if (two) {
        const float4 bv = *reinterpret_cast<const float4*>(a1 + kk);
        bo[0] = bv.x; bo[1] = bv.y; bo[2] = bv.z; bo[3] = bv.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool in = kk + e < d;
        xo[e] = in ? xr[kk + e] : 0.f;
        ao[e] = in ? a0[kk + e] : 0.f;
        if (two) bo[e] = in ? a1[kk + e] : 0.f;
      }
    }
  };
  if (k0s < k1s) load(k0s, xe, ae, be);
  for (int ks = k0s; ks < k1s; ++ks) {
    float xn[4], an[4], bn[4] = {0.f, 0.f, 0.f, 0.f};
    load(ks + 1 < k1s ? ks + 1 : ks, xn, an, bn);
    if (xbr) {
      const int kk = ks * 16 + 4 * s;
      if (VEC && kk + 3 < d) {
        __hip_bfloat16 v4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v4[e] = __float2bfloat16(xe[e]);
        *reinterpret_cast<uint2*>(xbr + kk) = *reinterpret_cast<const uint2*>(v4);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (kk + e < d) xbr[kk + e] = __float2bfloat16(xe[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ss += xe[e] * xe[e];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(double(xe[e]), double(ae[e]), acc0, 0, 0, 0);
      if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(double(xe[e]), double(be[e]), acc1, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      xe[e] = xn[e];
      ae[e] = an[e];
      be[e] = bn[e];
    }
  }
  // |x|^2 of row i over this wave's dims: sum the four dimension slots
  ss += __shfl_xor(ss, 16);
  ss += __shfl_xor(ss, 32);
  if (s == 0) pss[wave][i] = ss;
  // FP64 MFMA result layout: element e of lane l is (row l / 16 + 4 e, hash l % 16)
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    part[wave][i][s + 4 * e] = acc0[e];
    if (two) part[wave][16 + i][s + 4 * e] = acc1[e];
  }
  if (threadIdx.x == 0) qn = 0;
  __syncthreads();
  const double u = 1.1102230246251565e-16;  // 2^-53
  const double gam = double(d + 2) * 5.9604644775390625e-08;
  for (int o = threadIdx.x; o < 16 * nhc; o += 256) {
    const int ri = o / nhc, hl = o - ri * nhc, hash = hb + hl;
    const int64_t row = row0 + ri;
    if (row >= n) continue;
    const float ssr = ((pss[0][ri] + pss[1][ri]) + pss[2][ri]) + pss[3][ri];
    const double sv = ((part[0][hl][ri] + part[1][hl][ri]) + part[2][hl][ri]) + part[3][hl][ri];
    const double xn = sqrt(double(ssr) * (1.0 + 2.0 * gam)) * (1.0 + 9.5367431640625e-07);
    if (rownorm && hash == 0) rownorm[row] = float(xn * (1.0 + 9.5367431640625e-07));
    const int64_t oi = row * nh + hash;
    // sum |a_i x_i| <= |a| |x|; the last term covers fp32 subnormal inputs
    // flushed to zero on the way into FP64.
    const double an = double(anorm[hash]);
    const double pa = an * xn + double(d) * an * 1.1754943508222875e-38;
    if (kind == LIDER_HASH_SIGN) {  // bit = [a.x >= 0]: decided unless |a.x| is within the band
      const double E = 8.0 * double(d + 4) * u * pa;
      if (!(fabs(sv) > E))
        qlist[atomicAdd(&qn, 1)] = o;
      else
        out[oi] = sv > 0.0 ? 1 : 0;
      continue;
    }
    const double bh = double(bvec[hash]);
    const double tv = (sv + bh) / w;
    const double E = 8.0 * (double(d + 4) * u * pa + u * (fabs(sv) + fabs(bh))) / w +
                     8.0 * u * fabs(tv);
    const double fl = floor(tv);
    const double fr = tv - fl;
    const double dist = fr < 1.0 - fr ? fr : 1.0 - fr;
    if (!(dist > E)) {
      qlist[atomicAdd(&qn, 1)] = o;
    } else if (fl >= -2147483648.0 && fl <= 2147483647.0) {
      out[oi] = int32_t(fl);
    } else if (clamp) {
      out[oi] = fl < 0 ? INT32_MIN : INT32_MAX;
    } else {
      atomicExch(status, int32_t(LIDER_ERANGE));
    }
  }
  __syncthreads();
  const int nq = qn;
  for (int e = wave; e < nq; e += 4) {
    const int o = qlist[e];
    const int ri = o / nhc, hash = hb + (o - ri * nhc);
    const int64_t row = row0 + ri;
    hash_decide_wave(X + row * d, A + int64_t(hash) * d, d,
                     kind == LIDER_HASH_SIGN ? 0.0 : double(bvec[hash]), w, kind, clamp,
                     out + row * nh + hash, status);
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

void launch_norm_bounds(const float* A, int32_t rows, int32_t d, float* out, hipStream_t st) {
  hipLaunchKernelGGL(norm_bound_kernel, dim3((rows + 63) / 64), dim3(64), 0, st, A, rows, d, out);
}

// Digits of n rows into out [n x nh].  status is a device int set to
// LIDER_ERANGE when a digit does not fit int32 and clamp is 0.  rownorm
// (nullable) receives an upper bound of each row's norm, xb (nullable) the
// rows rounded to bf16.
int run_hash_ex(const float* X, int64_t n, int32_t d, const float* A, const float* b,
                const float* anorm, int32_t nh, double w, int32_t* out, int32_t* status,
                int clamp, float* rownorm, hipStream_t st, int kind, __hip_bfloat16* xb,
                const HashZero* zero) {
  HashZero z{};
  if (zero) {
    z = *zero;
    z.nz = std::max(z.a ? z.na : 0, (z.b || z.c) ? z.nb : 0);
  }
  if (n <= 0) {
    if (z.nz > 0) return set_error(LIDER_EINVAL, "hash: counters to clear without rows");
    return LIDER_OK;
  }
  const bool vec = (d % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(xb) & 7) == 0);
  const dim3 grid(unsigned((n + 15) / 16), unsigned((nh + 31) / 32));
  if (vec)
    hipLaunchKernelGGL(hash_kernel<true>, grid, dim3(256), 0, st, X, n, d, A, b, anorm, nh, w,
                       out, status, clamp, rownorm, kind, xb, z);
  else
    hipLaunchKernelGGL(hash_kernel<false>, grid, dim3(256), 0, st, X, n, d, A, b, anorm, nh, w,
                       out, status, clamp, rownorm, kind, xb, z);
  return check_hip(hipGetLastError(), "hash kernel");
}

}  // namespace lider
