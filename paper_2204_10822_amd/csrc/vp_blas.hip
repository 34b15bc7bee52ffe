// Vector kernels for the Krylov solvers: deterministic two-stage reductions
// (per-workgroup partials, then one finishing workgroup in fixed order) and the
// fused passes of classical Gram-Schmidt applied twice.
#include "vp_internal.h"

namespace vp {

constexpr int kMaxNV = kMaxRestart + 1;

// out[k] = sum_b partials[b*K + k], fixed order
// mdst (optional, pinned host memory): copy of msrc[0..mn) once the sums are done,
// read by the host after the stream synchronises (no separate copy).
__global__ void k_finish_sum(const double* __restrict__ partials, int nblocks, int K, double* out,
                             const double* msrc, double* mdst, int mn) {
  __shared__ double lds[1024];
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partials[(size_t)b * K + k];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = lds[0];
    __syncthreads();
  }
  if (mdst && threadIdx.x == 0)
    for (int m = 0; m < mn; ++m) mdst[m] = msrc[m];
}

void launch_finish_sum(hipStream_t s, const double* partials, int nblocks, int K, double* out, const double* msrc,
                       double* mdst, int mn) {
  hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(512), 0, s, partials, nblocks, K, out, msrc, mdst, mn);
  VP_LAUNCH_CHECK();
}

// Per-workgroup partial sums of v[k] (k < nv, compile-time bound NV) and, if
// with_extra, of one more value stored after them: partials[block*K + k],
// K = nv + with_extra.  Unrolled with guards so v stays in registers.
template <int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], int nv, double extra,
                                               bool with_extra, double* lds /* 16*(NV+1) */,
                                               double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int K = nv + (with_extra ? 1 : 0);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    if (k < nv) {
      const double t = wave_sum(v[k]);
      if (lane == 0) lds[wid * (NV + 1) + k] = t;
    }
  }
  if (with_extra) {
    const double t = wave_sum(extra);
    if (lane == 0) lds[wid * (NV + 1) + NV] = t;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const int src = k < nv ? k : NV;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[w * (NV + 1) + src];
    partials[(size_t)blockIdx.x * K + k] = s;
  }
}

__global__ void __launch_bounds__(kBlock) k_dot(const double* __restrict__ x, const double* __restrict__ y,
                                                size_t n, double* __restrict__ partials) {
  __shared__ double lds[16];
  double a[1] = {0.0};
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    a[0] = fma(x[e], y[e], a[0]);
  block_sum<1>(a, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = a[0];
}

void launch_dot(hipStream_t s, const double* x, const double* y, size_t n, double* partials) {
  hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(kBlock), 0, s, x, y, n, partials);
  VP_LAUNCH_CHECK();
}

// h_k = V_k . w, k < nv
template <int NV>
__global__ void __launch_bounds__(kBlock)
k_mdot(const double* __restrict__ V, size_t ld, int nv, const double* __restrict__ w, size_t n,
       double* __restrict__ partials) {
  __shared__ double lds[16 * (NV + 1)];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double we = w[e];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) acc[k] = fma(V[k * ld + e], we, acc[k]);
  }
  block_partials<NV>(acc, nv, 0.0, false, lds, partials);
}

// w <- w - sum_k h_k V_k ;  partials: V_k . w_new (k < nv) and w_new . w_new (slot nv)
template <int NV>
__global__ void __launch_bounds__(kBlock)
k_maxpy_mdot(const double* __restrict__ V, size_t ld, int nv, const double* __restrict__ h,
             double* __restrict__ w, size_t n, double* __restrict__ partials) {
  __shared__ double lds[16 * (NV + 1)];
  __shared__ double hs[NV];
  for (int k = threadIdx.x; k < nv; k += blockDim.x) hs[k] = h[k];
  __syncthreads();
  double acc[NV];
  double nrm = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double vk[NV];
    double we = w[e];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) {
        vk[k] = V[k * ld + e];
        we = fma(-hs[k], vk[k], we);
      }
    w[e] = we;
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) acc[k] = fma(vk[k], we, acc[k]);
    nrm = fma(we, we, nrm);
  }
  block_partials<NV>(acc, nv, nrm, true, lds, partials);
}

// out <- (w - sum_k h_k V_k) / sqrt(nrm2[0] - sum_k h_k^2)
template <int NV>
__global__ void __launch_bounds__(kBlock)
k_maxpy_scale(const double* __restrict__ V, size_t ld, int nv, const double* __restrict__ h,
              const double* __restrict__ w, const double* __restrict__ nrm2,
              double* __restrict__ out, size_t n) {
  __shared__ double hs[NV];
  __shared__ double inv;
  for (int k = threadIdx.x; k < nv; k += blockDim.x) hs[k] = h[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = nrm2[0];
    for (int k = 0; k < nv; ++k) s -= hs[k] * hs[k];
    inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  }
  __syncthreads();
  const double sc = inv;
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double we = w[e];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv) we = fma(-hs[k], V[k * ld + e], we);
    out[e] = we * sc;
  }
}

// x += sum_k y_k Z_k
template <int NV>
__global__ void __launch_bounds__(kBlock)
k_gemv_add(const double* __restrict__ Z, size_t ld, int nz, const double* __restrict__ y,
           double* __restrict__ x, size_t n) {
  __shared__ double ys[NV];
  for (int k = threadIdx.x; k < nz; k += blockDim.x) ys[k] = y[k];
  __syncthreads();
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double xe = x[e];
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nz) xe = fma(ys[k], Z[k * ld + e], xe);
    x[e] = xe;
  }
}

#define VP_DISPATCH_NV(nv, KERNEL, ...)                                                       \
  do {                                                                                        \
    if ((nv) <= 8) hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                                \
    else if ((nv) <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);                         \
    else if ((nv) <= 32) hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__);                         \
    else hipLaunchKernelGGL(KERNEL<kMaxNV>, __VA_ARGS__);                                     \
  } while (0)

void launch_mdot(hipStream_t s, const double* V, size_t ld, int nv, const double* w, size_t n,
                 double* partials) {
  if (nv > kMaxNV) throw Error(VP_EINVAL, "mdot: too many vectors");
  VP_DISPATCH_NV(nv, k_mdot, dim3(kRedBlocks), dim3(kBlock), 0, s, V, ld, nv, w, n, partials);
  VP_LAUNCH_CHECK();
}

void launch_maxpy_mdot(hipStream_t s, const double* V, size_t ld, int nv, const double* h,
                       double* w, size_t n, double* partials) {
  if (nv > kMaxNV) throw Error(VP_EINVAL, "maxpy_mdot: too many vectors");
  VP_DISPATCH_NV(nv, k_maxpy_mdot, dim3(kRedBlocks), dim3(kBlock), 0, s, V, ld, nv, h, w, n, partials);
  VP_LAUNCH_CHECK();
}

void launch_maxpy_scale(hipStream_t s, const double* V, size_t ld, int nv, const double* h,
                        const double* w, const double* nrm2, double* out, size_t n) {
  if (nv > kMaxNV) throw Error(VP_EINVAL, "maxpy_scale: too many vectors");
  VP_DISPATCH_NV(nv, k_maxpy_scale, dim3(grid_for(n)), dim3(kBlock), 0, s, V, ld, nv, h, w, nrm2, out, n);
  VP_LAUNCH_CHECK();
}

void launch_gemv_add(hipStream_t s, const double* Z, size_t ld, int nz, const double* y, double* x,
                     size_t n) {
  if (nz > kMaxNV) throw Error(VP_EINVAL, "gemv_add: too many vectors");
  VP_DISPATCH_NV(nz, k_gemv_add, dim3(grid_for(n)), dim3(kBlock), 0, s, Z, ld, nz, y, x, n);
  VP_LAUNCH_CHECK();
}

__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, size_t n) {
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + (b == 0.0 ? 0.0 : b * y[e]);
}

void launch_axpby(hipStream_t s, double a, const double* x, double b, double* y, size_t n) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kBlock), 0, s, a, x, b, y, n);
  VP_LAUNCH_CHECK();
}

// y = x * scal[0] (invert = 0) or y = x / scal[0] (invert = 1); scal on the device
__global__ void k_scale_copy(const double* __restrict__ x, const double* __restrict__ scal, int invert,
                             double* __restrict__ y, size_t n) {
  const double sv = scal[0];
  const double f = invert ? (sv != 0.0 ? 1.0 / sv : 0.0) : sv;
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = x[e] * f;
}

void launch_scale_copy(hipStream_t s, const double* x, const double* scal, int invert, double* y,
                       size_t n) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(kBlock), 0, s, x, scal, invert, y, n);
  VP_LAUNCH_CHECK();
}

// flexible CG, dev = [rz, pq, ...]: alpha = rz/pq; x += alpha p; r -= alpha q;
// partials: r.r.  r32 (optional): the new r in FP32 for the V-cycle, divided by
// dsc if that is given.
__global__ void __launch_bounds__(kBlock)
k_fcg_update(const double* __restrict__ dev, double* __restrict__ x, double* __restrict__ r,
             const double* __restrict__ p, const double* __restrict__ q, size_t n,
             double* __restrict__ partials, float* __restrict__ r32, const double* __restrict__ dsc) {
  __shared__ double lds[16];
  const double alpha = dev[1] != 0.0 ? dev[0] / dev[1] : 0.0;
  double a[1] = {0.0};
  // node pairs (two dofs) per step: 16-byte loads and stores
  const size_t n2 = n / 2;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += stride) {
    const double2 pe = reinterpret_cast<const double2*>(p)[e];
    const double2 qe = reinterpret_cast<const double2*>(q)[e];
    double2 xe = reinterpret_cast<const double2*>(x)[e];
    double2 re = reinterpret_cast<const double2*>(r)[e];
    xe.x = fma(alpha, pe.x, xe.x);
    xe.y = fma(alpha, pe.y, xe.y);
    re.x = fma(-alpha, qe.x, re.x);
    re.y = fma(-alpha, qe.y, re.y);
    reinterpret_cast<double2*>(x)[e] = xe;
    reinterpret_cast<double2*>(r)[e] = re;
    if (r32) {
      float2 o;
      if (dsc) {
        const double2 de = reinterpret_cast<const double2*>(dsc)[e];
        o = make_float2((float)(re.x / de.x), (float)(re.y / de.y));
      } else {
        o = make_float2((float)re.x, (float)re.y);
      }
      reinterpret_cast<float2*>(r32)[e] = o;
    }
    a[0] = fma(re.x, re.x, a[0]);
    a[0] = fma(re.y, re.y, a[0]);
  }
  if (n & 1) {  // odd length: last element by the first thread
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      const size_t e = n - 1;
      x[e] = fma(alpha, p[e], x[e]);
      const double re = fma(-alpha, q[e], r[e]);
      r[e] = re;
      if (r32) r32[e] = (float)(dsc ? re / dsc[e] : re);
      a[0] = fma(re, re, a[0]);
    }
  }
  block_sum<1>(a, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = a[0];
}

int launch_fcg_update(hipStream_t s, const double* dev, double* x, double* r, const double* p,
                      const double* q, size_t n, double* partials, float* r32, const double* dsc) {
  hipLaunchKernelGGL(k_fcg_update, dim3(kDotBlocks), dim3(kBlock), 0, s, dev, x, r, p, q, n, partials, r32, dsc);
  VP_LAUNCH_CHECK();
  return kDotBlocks;
}

// The V-cycle's output to the Krylov solver: z = x (widened, divided by dsc if
// given; z may alias x, or be null when the caller reads x itself), with
// per-workgroup partials of z.r and, if q is given, z.q (partials[block*K + k],
// K = 1 or 2).
template <typename TX>
__global__ void __launch_bounds__(kBlock)
k_out_dots(const TX* x, const double* __restrict__ dsc, double* z, const double* __restrict__ r,
           const double* __restrict__ q, size_t n, double* __restrict__ partials) {
  __shared__ double lds[32];
  double a[2] = {0.0, 0.0};
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double ze = (double)x[e];
    if (dsc) ze /= dsc[e];
    if (z && (const void*)z != (const void*)x) z[e] = ze;
    a[0] = fma(ze, r[e], a[0]);
    if (q) a[1] = fma(ze, q[e], a[1]);
  }
  block_sum<2>(a, lds);
  if (threadIdx.x == 0) {
    partials[(size_t)blockIdx.x * (q ? 2 : 1)] = a[0];
    if (q) partials[(size_t)blockIdx.x * 2 + 1] = a[1];
  }
}

template <typename TX>
int launch_out_dots(hipStream_t s, const TX* x, const double* dsc, double* z, const double* r, const double* q,
                    size_t n, double* partials) {
  hipLaunchKernelGGL((k_out_dots<TX>), dim3(kDotBlocks), dim3(kBlock), 0, s, x, dsc, z, r, q, n, partials);
  VP_LAUNCH_CHECK();
  return kDotBlocks;
}
template int launch_out_dots<float>(hipStream_t, const float*, const double*, double*, const double*,
                                    const double*, size_t, double*);
template int launch_out_dots<double>(hipStream_t, const double*, const double*, double*, const double*,
                                     const double*, size_t, double*);

// p = z + beta p with beta = -dev[6]/dev[1] (flexible CG: beta = -alpha z.q / r.z_old,
// alpha = r.z_old / p.q); first: p = z.  Thread 0 of workgroup 0 moves the new r.z
// (dev[5]) to dev[0]; no other thread reads dev[0] here.
__global__ void k_fcg_dir(double* __restrict__ dev, const double* __restrict__ z,
                          double* __restrict__ p, size_t n, int first) {
  const double beta = (first || dev[1] == 0.0) ? 0.0 : -dev[6] / dev[1];
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    p[e] = first ? z[e] : fma(beta, p[e], z[e]);
  if (!first && blockIdx.x == 0 && threadIdx.x == 0) dev[0] = dev[5];
}

void launch_fcg_dir(hipStream_t s, double* dev, const double* z, double* p, size_t n, int first) {
  hipLaunchKernelGGL(k_fcg_dir, dim3(grid_for(n)), dim3(kBlock), 0, s, dev, z, p, n, first);
  VP_LAUNCH_CHECK();
}

// The same update with z read from the FP32 V-cycle output: z = x32 (divided by
// dsc if given), widened exactly as the output conversion does it, so p is bitwise
// the one computed from the FP64 copy, without that copy's write and read.
__global__ void k_fcg_dir32(double* __restrict__ dev, const float* __restrict__ x32, const double* __restrict__ dsc,
                            double* __restrict__ p, size_t n, int first) {
  const double beta = (first || dev[1] == 0.0) ? 0.0 : -dev[6] / dev[1];
  // two entries per step (16-byte loads of p, 8-byte loads of x32); n is even
  const size_t n2 = n / 2;
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n2; e += (size_t)gridDim.x * blockDim.x) {
    const float2 xv = reinterpret_cast<const float2*>(x32)[e];
    double z0 = (double)xv.x, z1 = (double)xv.y;
    if (dsc) {
      const double2 dv = reinterpret_cast<const double2*>(dsc)[e];
      z0 /= dv.x;
      z1 /= dv.y;
    }
    double2 pv;
    if (first) {
      pv = make_double2(z0, z1);
    } else {
      pv = reinterpret_cast<const double2*>(p)[e];
      pv.x = fma(beta, pv.x, z0);
      pv.y = fma(beta, pv.y, z1);
    }
    reinterpret_cast<double2*>(p)[e] = pv;
  }
  if (!first && blockIdx.x == 0 && threadIdx.x == 0) dev[0] = dev[5];
}

void launch_fcg_dir32(hipStream_t s, double* dev, const float* x32, const double* dsc, double* p, size_t n,
                      int first) {
  if (n % 2) throw Error(VP_EINVAL, "FCG direction: odd vector length");
  hipLaunchKernelGGL(k_fcg_dir32, dim3(grid_for(n / 2)), dim3(kBlock), 0, s, dev, x32, dsc, p, n, first);
  VP_LAUNCH_CHECK();
}

__global__ void k_cast_df(const double* __restrict__ x, float* __restrict__ y, size_t n) {
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = (float)x[e];
}
__global__ void k_cast_fd(const float* __restrict__ x, double* __restrict__ y, size_t n) {
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = (double)x[e];
}
void launch_cast(hipStream_t s, const double* x, float* y, size_t n) {
  hipLaunchKernelGGL(k_cast_df, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  VP_LAUNCH_CHECK();
}
void launch_cast(hipStream_t s, const float* x, double* y, size_t n) {
  hipLaunchKernelGGL(k_cast_fd, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, n);
  VP_LAUNCH_CHECK();
}

__global__ void k_fill(double* __restrict__ x, double v, size_t n) {
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    x[e] = v;
}
void launch_fill(hipStream_t s, double* x, double v, size_t n) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, x, v, n);
  VP_LAUNCH_CHECK();
}

}  // namespace vp
