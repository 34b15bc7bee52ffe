// Learned warm start: a 4-level convolutional U-Net run and trained with
// hand-written BF16 matrix-core (MFMA) kernels and FP32 accumulation.
//
// Every layer is lowered to one GEMM C[M,N] = A[M,K] B[K,N] on the matrix cores
// plus cheap layout kernels:
//   3x3 conv (pad 1)      : im2col (two inputs = skip concat without a copy) + GEMM
//   3x3 conv input grad   : GEMM dcol = dY W^T, then a gather col2im (no atomics)
//   weight grads          : split-K GEMM col^T dY over pixels + fixed-order reduction
//   2x2 stride-2 down     : space-to-depth (a reshape) + GEMM
//   2x2 stride-2 up       : GEMM to 4*Cout channels + depth-to-space
//   1x1 output            : GEMM
// Activations are NHWC BF16; the output head, loss and Adam are FP32.
#include "vp_internal.h"
#include "../../include/vpnet.h"

#include <cstring>
#include <memory>

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// eight consecutive BF16 values of an LDS row (8-byte aligned: two 8-byte loads)
__device__ __forceinline__ v8bf lds_frag8(const short* p) {
  const v4s lo = *reinterpret_cast<const v4s*>(p), hi = *reinterpret_cast<const v4s*>(p + 4);
  const v8s v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(v8bf, v);
}
typedef float v4f __attribute__((ext_vector_type(4)));
using bf16 = __hip_bfloat16;

namespace vp {
namespace net {

// ---------------------------------------------------------------------------
// GEMM on the matrix cores.  A is [M][K] (lda) or, with AT, [K][M]; B is [K][N]
// or, with BT, [N][K].  Workgroup tile 64x64, K step 32, four waves each owning a
// 32x32 quadrant computed as 2x2 tiles of the 16x16x32 BF16 MFMA (gfx950's
// double-K form: one instruction per 32-deep K step).
// Epilogue: OUT_BF16 stores relu?(C + bias) in BF16; otherwise FP32 C (+ bias) is
// stored to C32 + split*M*ldc (split-K partial when gridDim.z > 1).
// ---------------------------------------------------------------------------
constexpr int BM = 64, BN = 64, BK = 32, KPAD = 4;   // LDS rows padded to 72 B (fewer bank conflicts than 80)

__device__ __forceinline__ short bf_bits(bf16 x) {
  short s;
  __builtin_memcpy(&s, &x, 2);
  return s;
}

// Stage one 64 x 32 operand tile into LDS as T[row][k] (row = m for A, n for B).
// `kmajor` operands are stored [K][rows] (contiguous along rows), the others
// [rows][K] (contiguous along K).  Each thread moves 8 consecutive elements with
// one 16-byte load when the ld is a multiple of 8 and the vector is in bounds.
template <bool KMAJOR>
__device__ __forceinline__ void stage_tile(const bf16* __restrict__ X, int rows, int kend, int ld, int r0, int k0,
                                           short (*T)[BK + KPAD], int tid) {
  const unsigned short* Xs = reinterpret_cast<const unsigned short*>(X);
  if (!KMAJOR) {
    const int r = tid >> 2, c = (tid & 3) * 8;
    const int gr = r0 + r, gk = k0 + c;
    if ((ld & 7) == 0 && gr < rows && gk + 8 <= kend) {
      const uint4 v = *reinterpret_cast<const uint4*>(Xs + (size_t)gr * ld + gk);
      const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T[r][c + 2 * q] = (short)(w[q] & 0xffff);
        T[r][c + 2 * q + 1] = (short)(w[q] >> 16);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        T[r][c + q] = (gr < rows && gk + q < kend) ? (short)Xs[(size_t)gr * ld + gk + q] : (short)0;
    }
  } else {
    const int c = tid >> 3, r = (tid & 7) * 8;
    const int gr = r0 + r, gk = k0 + c;
    if ((ld & 7) == 0 && gk < kend && gr + 8 <= rows) {
      const uint4 v = *reinterpret_cast<const uint4*>(Xs + (size_t)gk * ld + gr);
      const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T[r + 2 * q][c] = (short)(w[q] & 0xffff);
        T[r + 2 * q + 1][c] = (short)(w[q] >> 16);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        T[r + q][c] = (gk < kend && gr + q < rows) ? (short)Xs[(size_t)gk * ld + gr + q] : (short)0;
    }
  }
}

template <bool AT, bool BT, bool OUT_BF16>
__global__ void __launch_bounds__(256)
k_gemm(const bf16* __restrict__ A, const bf16* __restrict__ B, int M, int N, int K, int lda, int ldb,
       const float* __restrict__ bias, int relu, bf16* __restrict__ Cb, float* __restrict__ C32, int ldc,
       int k_per_split) {
  __shared__ short As[BM][BK + KPAD];   // [m][k]
  __shared__ short Bs[BN][BK + KPAD];   // [n][k] (B kept transposed: fragments are contiguous)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * k_per_split;
  const int kend = min(K, kbeg + k_per_split);
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    stage_tile<AT>(A, M, kend, lda, m0, k0, As, tid);
    stage_tile<!BT>(B, N, kend, ldb, n0, k0, Bs, tid);
    __syncthreads();
    {
      // lane: row (A) or column (B) lane % 16, k = 8 (lane / 16) .. + 7 of the step
      v8bf af[2], bfr[2];
      const int kq = 8 * (lane >> 4);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + 16 * i + (lane & 15);
        af[i] = lds_frag8(&As[row][kq]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = wn + 16 * j + (lane & 15);
        bfr[j] = lds_frag8(&Bs[col][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane holds rows 4*(lane/16) + q, column lane%16 of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][q];
        if (bias) v += bias[gn];
        if (OUT_BF16) {
          if (relu) v = fmaxf(v, 0.f);
          Cb[(size_t)gm * ldc + gn] = __float2bfloat16(v);
        } else {
          C32[(size_t)blockIdx.z * M * ldc + (size_t)gm * ldc + gn] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// layout kernels (NHWC)
// ---------------------------------------------------------------------------
// col[p][(ky*3+kx)*(C1+C2) + c] = X(p + (ky-1, kx-1), c), X = concat(X1, X2) along
// channels.  One thread per (pixel, tap, 8-channel group): a 16-byte copy (C1, C2
// are multiples of 8).
__global__ void k_im2col3(const bf16* __restrict__ X1, int C1, const bf16* __restrict__ X2, int C2,
                          int Bn, int H, int W, bf16* __restrict__ col) {
  const int C = C1 + C2, G = C >> 3;
  const unsigned total = (unsigned)Bn * H * W * 9 * G;
  for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const unsigned g = e % G, t = e / G;
    const unsigned kp = t % 9, p = t / 9;
    const unsigned x = p % W, y = (p / W) % H, b = p / (W * H);
    const int yy = (int)y + (int)(kp / 3) - 1, xx = (int)x + (int)(kp % 3) - 1;
    const int c = 8 * (int)g;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
      const size_t q = ((size_t)b * H + yy) * W + xx;
      v = c < C1 ? *reinterpret_cast<const uint4*>(X1 + q * C1 + c)
                 : *reinterpret_cast<const uint4*>(X2 + q * C2 + (c - C1));
    }
    *reinterpret_cast<uint4*>(col + ((size_t)p * 9 + kp) * C + c) = v;
  }
}

// dX(q, c) = sum_{kp} dcol[q - off(kp)][kp*C + c]; split into the two inputs'
// gradients.  One thread per (pixel, 4-channel group), float4 accesses.
__global__ void k_col2im3(const float* __restrict__ dcol, int C1, int C2, int Bn, int H, int W,
                          float* __restrict__ dX1, float* __restrict__ dX2) {
  const int C = C1 + C2, G = C >> 2;
  const unsigned total = (unsigned)Bn * H * W * G;
  for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const unsigned g = e % G, q = e / G;
    const unsigned x = q % W, y = (q / W) % H, b = q / (W * H);
    const int c = 4 * (int)g;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int kp = 0; kp < 9; ++kp) {
      const int py = (int)y - (kp / 3 - 1), px = (int)x - (kp % 3 - 1);
      if (py < 0 || py >= H || px < 0 || px >= W) continue;
      const size_t p = ((size_t)b * H + py) * W + px;
      const float4 d = *reinterpret_cast<const float4*>(dcol + (p * 9 + kp) * C + c);
      s.x += d.x; s.y += d.y; s.z += d.z; s.w += d.w;
    }
    if (c < C1) *reinterpret_cast<float4*>(dX1 + (size_t)q * C1 + c) = s;
    else if (dX2) *reinterpret_cast<float4*>(dX2 + (size_t)q * C2 + (c - C1)) = s;
  }
}

// space-to-depth: Y[b][y][x][(dy*2+dx)*C + c] = X[b][2y+dy][2x+dx][c]  (H, W of Y)
template <typename T>
__global__ void k_s2d(const T* __restrict__ X, int Bn, int H, int W, int C, T* __restrict__ Y) {
  const size_t total = (size_t)Bn * H * W * 4 * C;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int k = (int)((e / C) % 4);
    const size_t p = e / ((size_t)4 * C);
    const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((size_t)W * H));
    const size_t q = ((size_t)b * 2 * H + 2 * y + k / 2) * 2 * W + 2 * x + k % 2;
    Y[e] = X[q * C + c];
  }
}

// depth-to-space: Y[b][2y+dy][2x+dx][c] = op(X[b][y][x][(dy*2+dx)*C + c] + bias[c])  (H, W of X)
template <typename TI, typename TO>
__global__ void k_d2s(const TI* __restrict__ X, int Bn, int H, int W, int C, const float* __restrict__ bias,
                      int relu, TO* __restrict__ Y) {
  const size_t total = (size_t)Bn * H * W * 4 * C;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const int k = (int)((e / C) % 4);
    const size_t p = e / ((size_t)4 * C);
    const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((size_t)W * H));
    const size_t q = ((size_t)b * 2 * H + 2 * y + k / 2) * 2 * W + 2 * x + k % 2;
    float v = (float)X[e];
    if (bias) v += bias[c];
    if (relu) v = fmaxf(v, 0.f);
    Y[q * C + c] = (TO)v;
  }
}

// g = dY * (Y > 0) (ReLU derivative from the stored output), to BF16 for the GEMMs
__global__ void k_relu_grad(const float* __restrict__ dY, const bf16* __restrict__ Y, size_t n, int relu,
                            bf16* __restrict__ g) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float d = dY[e];
    g[e] = __float2bfloat16((!relu || (float)Y[e] > 0.f) ? d : 0.f);
  }
}

__global__ void k_bf16_to_f32(const bf16* __restrict__ x, size_t n, float* __restrict__ y) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = (float)x[e];
}

// sum of two FP32 gradients (skip connection receives from two consumers)
__global__ void k_add_into(float* __restrict__ a, const float* __restrict__ b, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    a[e] += b[e];
}

// out[i] = sum_s part[s][i]  (fixed order)
__global__ void k_sum_splits(const float* __restrict__ part, int splits, size_t n, float* __restrict__ out) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[(size_t)k * n + e];
    out[e] = s;
  }
}

// Column sums over pixels in two fixed-order stages: workgroup b sums pixels
// [b*chunk, (b+1)*chunk) for every column (thread t owns columns t, t+256, ...),
// writing part[b][col]; k_sum_splits then adds the parts in order.
// Used for bias gradients (BF16 g) and for the head gradients.
__global__ void k_colsum_bf16(const bf16* __restrict__ g, size_t P, int C, size_t chunk, float* __restrict__ part) {
  const size_t p0 = (size_t)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
  for (int c = threadIdx.x; c < C; c += blockDim.x) {
    float s = 0.f;
    for (size_t p = p0; p < p1; ++p) s += (float)g[p * C + c];
    part[(size_t)blockIdx.x * C + c] = s;
  }
}

// head: part[b][c*O + o] = sum_p X[p][c] G[p][o], part[b][C*O + o] = sum_p G[p][o]
// over pixel chunk b; one thread per output entry
// out[col] = sum_k part[k][col] for k < parts: one workgroup per column, fixed order
__global__ void k_reduce_parts(const float* __restrict__ part, int parts, int ncol, float* __restrict__ out) {
  __shared__ float lds[256];
  const int col = blockIdx.x;
  float s = 0.f;
  for (int k = threadIdx.x; k < parts; k += blockDim.x) s += part[(size_t)k * ncol + col];
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = lds[0];
}

__global__ void k_head_wgrad_part(const bf16* __restrict__ X, const float* __restrict__ G, size_t P, int C,
                                  int O, size_t chunk, float* __restrict__ part) {
  const int K = C * O + O;
  const size_t p0 = (size_t)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
  for (int e = threadIdx.x; e < K; e += blockDim.x) {
    float s = 0.f;
    if (e < C * O) {
      const int c = e / O, o = e % O;
      for (size_t p = p0; p < p1; ++p) s += (float)X[p * C + c] * G[p * O + o];
    } else {
      const int o = e - C * O;
      for (size_t p = p0; p < p1; ++p) s += G[p * O + o];
    }
    part[(size_t)blockIdx.x * K + e] = s;
  }
}

// 1x1 output head in FP32: out[p][o] = sum_c X[p][c] W[c][o] + b[o]
__global__ void k_head_fwd(const bf16* __restrict__ X, size_t P, int C, const float* __restrict__ Wt,
                           const float* __restrict__ b, int O, float* __restrict__ out) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < P * O; e += (size_t)gridDim.x * blockDim.x) {
    const int o = (int)(e % O);
    const size_t p = e / O;
    float s = b[o];
    for (int c = 0; c < C; ++c) s += (float)X[p * C + c] * Wt[c * O + o];
    out[e] = s;
  }
}

// MSE loss over n outputs: partial sums per workgroup, grad = 2 (out - t) / n
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ t, size_t n,
                      float* __restrict__ grad, double* __restrict__ partials) {
  __shared__ double lds[16];
  double a[1] = {0.0};
  const float sc = 2.f / (float)n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float d = out[e] - t[e];
    grad[e] = sc * d;
    a[0] += (double)d * d;
  }
  block_sum<1>(a, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = a[0];
}

// head input grad: dX[p][c] = sum_o G[p][o] W[c][o]
__global__ void k_head_dgrad(const float* __restrict__ G, size_t P, int C, const float* __restrict__ Wt, int O,
                             float* __restrict__ dX) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < P * C; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const size_t p = e / C;
    float s = 0.f;
    for (int o = 0; o < O; ++o) s += G[p * O + o] * Wt[c * O + o];
    dX[e] = s;
  }
}

__global__ void k_to_bf16(const float* __restrict__ x, bf16* __restrict__ y, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = __float2bfloat16(x[e]);
}

// Adam on FP32 master weights, BF16 copy refreshed in the same pass
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2, bf16* __restrict__ wb) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    const float ww = w[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    w[e] = ww;
    wb[e] = __float2bfloat16(ww);
  }
}

// ---------------------------------------------------------------------------
// features and guesses (solver <-> network)
// ---------------------------------------------------------------------------
// 8 normalised input channels on the coarse cell grid (f x f box average of the
// mesh cells): H/2, (A-0.85)/0.15, v_air/25 (2), v_ocean/0.1 (2), v_prev/0.3 (2);
// node fields are first averaged to cells (mean of the 4 corners).
__global__ void k_features(int nx, int ny, int f, const double* __restrict__ H, const double* __restrict__ A,
                           const double* __restrict__ va, const double* __restrict__ vo,
                           const double* __restrict__ vp, float* __restrict__ out) {
  const int Wc = nx / f, Hc = ny / f;
  const size_t total = (size_t)Wc * Hc;
  const int nxn = nx + 1;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int X = (int)(e % Wc), Y = (int)(e / Wc);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int ci = X * f + dx, cj = Y * f + dy;
        const size_t cell = (size_t)cj * nx + ci;
        acc[0] += H[cell];
        acc[1] += A[cell];
        const size_t sw = (size_t)cj * nxn + ci;
        const size_t id[4] = {sw, sw + 1, sw + nxn, sw + nxn + 1};
        for (int a = 0; a < 4; ++a)
          for (int d = 0; d < 2; ++d) {
            acc[2 + d] += 0.25 * va[2 * id[a] + d];
            acc[4 + d] += 0.25 * vo[2 * id[a] + d];
            acc[6 + d] += 0.25 * vp[2 * id[a] + d];
          }
      }
    const double s = 1.0 / (f * f);
    float* o = out + e * 8;
    o[0] = (float)(acc[0] * s / 2.0);
    o[1] = (float)((acc[1] * s - 0.85) / 0.15);
    o[2] = (float)(acc[2] * s / 25.0);
    o[3] = (float)(acc[3] * s / 25.0);
    o[4] = (float)(acc[4] * s / 0.1);
    o[5] = (float)(acc[5] * s / 0.1);
    o[6] = (float)(acc[6] * s / 0.3);
    o[7] = (float)(acc[7] * s / 0.3);
  }
}

// training targets on the cell grid: the velocity change v - v_prev (mean of the 4
// corners)/0.3 (v_prev nullable: 0), pi (mean of the 4 points)
__global__ void k_targets(int nx, int ny, const double* __restrict__ v, const double* __restrict__ pi,
                          const double* __restrict__ vprev, float* __restrict__ out) {
  const size_t ncell = (size_t)nx * ny;
  const int nxn = nx + 1;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ncell; e += (size_t)gridDim.x * blockDim.x) {
    const int ci = (int)(e % nx), cj = (int)(e / nx);
    const size_t sw = (size_t)cj * nxn + ci;
    const size_t id[4] = {sw, sw + 1, sw + nxn, sw + nxn + 1};
    double vx = 0, vy = 0;
    for (int a = 0; a < 4; ++a) {
      const double px = vprev ? vprev[2 * id[a]] : 0.0, py = vprev ? vprev[2 * id[a] + 1] : 0.0;
      vx += 0.25 * (v[2 * id[a]] - px);
      vy += 0.25 * (v[2 * id[a] + 1] - py);
    }
    float* o = out + e * 5;
    o[0] = (float)(vx / 0.3);
    o[1] = (float)(vy / 0.3);
    for (int k = 0; k < 3; ++k) {
      double s = 0;
      for (int q = 0; q < 4; ++q) s += 0.25 * pi[(size_t)(q * 3 + k) * ncell + e];
      o[2 + k] = (float)s;
    }
  }
}

// bilinear sample of a cell-centred coarse field (Wc x Hc cells over [0,1]^2), clamped
__device__ __forceinline__ float sample(const float* __restrict__ F, int Wc, int Hc, int C, int ch, double x,
                                        double y) {
  const double gx = x * Wc - 0.5, gy = y * Hc - 0.5;
  int i0 = (int)floor(gx), j0 = (int)floor(gy);
  const double tx = gx - i0, ty = gy - j0;
  const int i1 = min(max(i0 + 1, 0), Wc - 1), j1 = min(max(j0 + 1, 0), Hc - 1);
  i0 = min(max(i0, 0), Wc - 1);
  j0 = min(max(j0, 0), Hc - 1);
  const double a = F[((size_t)j0 * Wc + i0) * C + ch], b = F[((size_t)j0 * Wc + i1) * C + ch];
  const double c = F[((size_t)j1 * Wc + i0) * C + ch], d = F[((size_t)j1 * Wc + i1) * C + ch];
  return (float)((1 - ty) * ((1 - tx) * a + tx * b) + ty * ((1 - tx) * c + tx * d));
}

// network output (Wc x Hc x 5) -> v0 = v_prev + the sampled change (de-normalised by
// 0.3 m/s) at the mesh nodes (zero on the boundary; v_prev nullable: 0), pi0 at the
// Gauss points, both by bilinear sampling
__global__ void k_guess(int nx, int ny, const float* __restrict__ outp, int Wc, int Hc,
                        const double* __restrict__ vprev, double* __restrict__ v0, double* __restrict__ pi0) {
  const size_t nn = (size_t)(nx + 1) * (ny + 1), ncell = (size_t)nx * ny;
  const double g0 = 0.21132486540518711775, g1 = 0.78867513459481288225;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn + ncell; e += (size_t)gridDim.x * blockDim.x) {
    if (e < nn) {
      const int i = (int)(e % (nx + 1)), j = (int)(e / (nx + 1));
      const bool bnd = i == 0 || j == 0 || i == nx || j == ny;
      const double x = (double)i / nx, y = (double)j / ny;
      const double px = vprev ? vprev[2 * e] : 0.0, py = vprev ? vprev[2 * e + 1] : 0.0;
      v0[2 * e] = bnd ? 0.0 : px + 0.3 * sample(outp, Wc, Hc, 5, 0, x, y);
      v0[2 * e + 1] = bnd ? 0.0 : py + 0.3 * sample(outp, Wc, Hc, 5, 1, x, y);
    } else if (pi0) {
      const size_t cell = e - nn;
      const int ci = (int)(cell % nx), cj = (int)(cell / nx);
      for (int q = 0; q < 4; ++q) {
        const double x = (ci + ((q & 1) ? g1 : g0)) / nx, y = (cj + ((q & 2) ? g1 : g0)) / ny;
        for (int k = 0; k < 3; ++k) pi0[(size_t)(q * 3 + k) * ncell + cell] = sample(outp, Wc, Hc, 5, 2 + k, x, y);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side: the network
// ---------------------------------------------------------------------------
template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  VP_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
  return static_cast<T*>(p);
}

inline unsigned gs(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 16384); }

enum Kind { CONV3 = 0, DOWN = 1, UP = 2, HEAD = 3 };
constexpr int kSumParts = 1024;  // pixel chunks of the two-stage column sums

struct Layer {
  Kind kind;
  int cin, cin2, cout;     // cin2: second (skip) input channels for CONV3
  int H, W;                // spatial size of the OUTPUT
  size_t woff, boff;       // parameter offsets (elements) into the flat arrays
  int in, in2, out;        // activation ids
};

struct Act {
  int C, H, W;
  bf16* y = nullptr;       // BF16 output (post-ReLU)
  float* g = nullptr;      // FP32 gradient w.r.t. y
};

}  // namespace net
}  // namespace vp

struct vpnet_s {
  hipStream_t stream = nullptr;
  int Bn = 0, H = 0, W = 0;
  std::string err;
  std::vector<vp::net::Layer> layers;
  std::vector<vp::net::Act> acts;
  size_t nparam = 0;
  float* w = nullptr;        // FP32 master
  bf16* wb = nullptr;  // BF16 copy used by the GEMMs
  float* g = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  long step = 0;
  // scratch
  bf16* col = nullptr;  size_t col_n = 0;
  float* fcol = nullptr;     size_t fcol_n = 0;
  float* part = nullptr;     size_t part_n = 0;
  bf16* gb = nullptr;   size_t gb_n = 0;
  float* tmp = nullptr;      size_t tmp_n = 0;
  float* out = nullptr;      // [B][H][W][5]
  float* gout = nullptr;
  double* red = nullptr;     // reduction partials
  double* hred = nullptr;    // pinned
  float* feat = nullptr;     // [H][W][8] input features of vpnet_infer
  bf16* xin = nullptr;  // BF16 input
};

namespace vp {
namespace net {

constexpr int kCin = 8, kCout = 5;

void build(vpnet_s* n) {
  const int Hs[4] = {n->H, n->H / 2, n->H / 4, n->H / 8};
  const int Ws[4] = {n->W, n->W / 2, n->W / 4, n->W / 8};
  const int ch[4] = {16, 32, 64, 128};
  auto act = [&](int C, int l) {
    n->acts.push_back(Act{C, Hs[l], Ws[l]});
    return (int)n->acts.size() - 1;
  };
  size_t off = 0;
  auto layer = [&](Kind k, int cin, int cin2, int cout, int l, int in, int in2) {
    Layer L{k, cin, cin2, cout, Hs[l], Ws[l], 0, 0, in, in2, -1};
    const int kin = k == CONV3 ? 9 * (cin + cin2) : k == DOWN ? 4 * cin : cin;
    const int kout = k == UP ? 4 * cout : cout;
    L.woff = off;
    off += (size_t)kin * kout;
    L.boff = off;
    off += cout;
    L.out = k == HEAD ? -1 : act(cout, l);
    n->layers.push_back(L);
    return L.out;
  };
  const int x = act(kCin, 0);
  int e0 = layer(CONV3, kCin, 0, ch[0], 0, x, -1);
  e0 = layer(CONV3, ch[0], 0, ch[0], 0, e0, -1);
  int t = layer(DOWN, ch[0], 0, ch[1], 1, e0, -1);
  int e1 = layer(CONV3, ch[1], 0, ch[1], 1, t, -1);
  e1 = layer(CONV3, ch[1], 0, ch[1], 1, e1, -1);
  t = layer(DOWN, ch[1], 0, ch[2], 2, e1, -1);
  int e2 = layer(CONV3, ch[2], 0, ch[2], 2, t, -1);
  e2 = layer(CONV3, ch[2], 0, ch[2], 2, e2, -1);
  t = layer(DOWN, ch[2], 0, ch[3], 3, e2, -1);
  int e3 = layer(CONV3, ch[3], 0, ch[3], 3, t, -1);
  e3 = layer(CONV3, ch[3], 0, ch[3], 3, e3, -1);
  t = layer(UP, ch[3], 0, ch[2], 2, e3, -1);
  int c2 = layer(CONV3, ch[2], ch[2], ch[2], 2, t, e2);
  c2 = layer(CONV3, ch[2], 0, ch[2], 2, c2, -1);
  t = layer(UP, ch[2], 0, ch[1], 1, c2, -1);
  int c1 = layer(CONV3, ch[1], ch[1], ch[1], 1, t, e1);
  c1 = layer(CONV3, ch[1], 0, ch[1], 1, c1, -1);
  t = layer(UP, ch[1], 0, ch[0], 0, c1, -1);
  int c0 = layer(CONV3, ch[0], ch[0], ch[0], 0, t, e0);
  c0 = layer(CONV3, ch[0], 0, ch[0], 0, c0, -1);
  layer(HEAD, ch[0], 0, kCout, 0, c0, -1);
  n->nparam = off;
}

template <bool AT, bool BT, bool OB>
void gemm(hipStream_t s, const bf16* A, const bf16* B, int M, int N, int K, int lda, int ldb, const float* bias,
          int relu, bf16* Cb, float* C32, int ldc, int splits) {
  const int kps = ((K + splits - 1) / splits + BK - 1) / BK * BK;
  splits = (K + kps - 1) / kps;
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, splits);
  hipLaunchKernelGGL((k_gemm<AT, BT, OB>), grid, dim3(256), 0, s, A, B, M, N, K, lda, ldb, bias, relu, Cb, C32,
                     ldc, kps);
  VP_LAUNCH_CHECK();
}

// FP32 result of a split-K GEMM (partials summed in fixed order)
void gemm_f32(vpnet_s* n, bool AT, bool BT, const bf16* A, const bf16* B, int M, int N, int K, int lda, int ldb,
              float* C) {
  int splits = std::max(1, std::min(64, K / 2048));
  const int kps = ((K + splits - 1) / splits + BK - 1) / BK * BK;
  splits = (K + kps - 1) / kps;
  const size_t need = (size_t)splits * M * N;
  if (need > n->part_n) {
    if (n->part) (void)hipFree(n->part);
    n->part = dalloc<float>(need);
    n->part_n = need;
  }
  hipStream_t s = n->stream;
  if (AT && !BT) gemm<true, false, false>(s, A, B, M, N, K, lda, ldb, nullptr, 0, nullptr, n->part, N, splits);
  else if (!AT && BT) gemm<false, true, false>(s, A, B, M, N, K, lda, ldb, nullptr, 0, nullptr, n->part, N, splits);
  else if (!AT && !BT) gemm<false, false, false>(s, A, B, M, N, K, lda, ldb, nullptr, 0, nullptr, n->part, N, splits);
  else throw Error(VP_EINVAL, "unsupported GEMM layout");
  hipLaunchKernelGGL(k_sum_splits, dim3(gs((size_t)M * N)), dim3(256), 0, s, n->part, splits, (size_t)M * N, C);
  VP_LAUNCH_CHECK();
}

template <typename T>
void ensure(T*& p, size_t& have, size_t need) {
  if (need <= have) return;
  if (p) (void)hipFree(p);
  p = dalloc<T>(need);
  have = need;
}

void forward(vpnet_s* n) {
  hipStream_t s = n->stream;
  const int Bn = n->Bn;
  for (const Layer& L : n->layers) {
    const Act& X = n->acts[L.in];
    const size_t P = (size_t)Bn * L.H * L.W;
    const bf16* Wt = n->wb + L.woff;
    const float* b = n->w + L.boff;
    if (L.kind == CONV3) {
      const Act& X2 = L.in2 >= 0 ? n->acts[L.in2] : X;
      const int C = L.cin + L.cin2;
      ensure(n->col, n->col_n, P * 9 * C);
      hipLaunchKernelGGL(k_im2col3, dim3(gs(P * 9 * C / 8)), dim3(256), 0, s, X.y, L.cin,
                         L.in2 >= 0 ? X2.y : nullptr, L.cin2, Bn, L.H, L.W, n->col);
      VP_LAUNCH_CHECK();
      gemm<false, false, true>(s, n->col, Wt, (int)P, L.cout, 9 * C, 9 * C, L.cout, b, 1, n->acts[L.out].y, nullptr,
                               L.cout, 1);
    } else if (L.kind == DOWN) {
      ensure(n->col, n->col_n, P * 4 * L.cin);
      hipLaunchKernelGGL(k_s2d<bf16>, dim3(gs(P * 4 * L.cin)), dim3(256), 0, s, X.y, Bn, L.H, L.W, L.cin, n->col);
      VP_LAUNCH_CHECK();
      gemm<false, false, true>(s, n->col, Wt, (int)P, L.cout, 4 * L.cin, 4 * L.cin, L.cout, b, 1, n->acts[L.out].y,
                               nullptr, L.cout, 1);
    } else if (L.kind == UP) {
      const size_t Pin = (size_t)Bn * X.H * X.W;
      ensure(n->col, n->col_n, Pin * 4 * L.cout);
      gemm<false, false, true>(s, X.y, Wt, (int)Pin, 4 * L.cout, L.cin, L.cin, 4 * L.cout, nullptr, 0, n->col,
                               nullptr, 4 * L.cout, 1);
      hipLaunchKernelGGL((k_d2s<bf16, bf16>), dim3(gs(Pin * 4 * L.cout)), dim3(256), 0, s, n->col, Bn, X.H, X.W,
                         L.cout, b, 1, n->acts[L.out].y);
      VP_LAUNCH_CHECK();
    } else {
      hipLaunchKernelGGL(k_head_fwd, dim3(gs(P * kCout)), dim3(256), 0, s, X.y, P, L.cin, n->w + L.woff, b, kCout,
                         n->out);
      VP_LAUNCH_CHECK();
    }
  }
}

void backward(vpnet_s* n) {
  hipStream_t s = n->stream;
  const int Bn = n->Bn;
  for (auto& a : n->acts) {
    if (!a.g) a.g = dalloc<float>((size_t)Bn * a.H * a.W * a.C);
    VP_HIP(hipMemsetAsync(a.g, 0, (size_t)Bn * a.H * a.W * a.C * sizeof(float), s));
  }
  for (int li = (int)n->layers.size() - 1; li >= 0; --li) {
    const Layer& L = n->layers[li];
    Act& X = n->acts[L.in];
    const size_t P = (size_t)Bn * L.H * L.W;
    float* dW = n->g + L.woff;
    float* db = n->g + L.boff;
    if (L.kind == HEAD) {
      const int K = L.cin * kCout + kCout;  // dW then db, contiguous in the parameter vector
      const size_t chunk = (P + kSumParts - 1) / kSumParts;
      ensure(n->part, n->part_n, (size_t)kSumParts * K);
      hipLaunchKernelGGL(k_head_wgrad_part, dim3(kSumParts), dim3(128), 0, s, X.y, n->gout, P, L.cin, kCout,
                         chunk, n->part);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_reduce_parts, dim3(K), dim3(256), 0, s, n->part, kSumParts, K, dW);
      VP_LAUNCH_CHECK();
      ensure(n->tmp, n->tmp_n, P * L.cin);
      hipLaunchKernelGGL(k_head_dgrad, dim3(gs(P * L.cin)), dim3(256), 0, s, n->gout, P, L.cin, n->w + L.woff, kCout,
                         n->tmp);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_add_into, dim3(gs(P * L.cin)), dim3(256), 0, s, X.g, n->tmp, P * L.cin);
      VP_LAUNCH_CHECK();
      continue;
    }
    Act& Y = n->acts[L.out];
    const size_t ny = P * L.cout;
    ensure(n->gb, n->gb_n, ny);
    hipLaunchKernelGGL(k_relu_grad, dim3(gs(ny)), dim3(256), 0, s, Y.g, Y.y, ny, 1, n->gb);
    VP_LAUNCH_CHECK();
    {
      const size_t chunk = (P + kSumParts - 1) / kSumParts;
      ensure(n->part, n->part_n, (size_t)kSumParts * L.cout);
      hipLaunchKernelGGL(k_colsum_bf16, dim3(kSumParts), dim3(128), 0, s, n->gb, P, L.cout, chunk, n->part);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_reduce_parts, dim3(L.cout), dim3(256), 0, s, n->part, kSumParts, L.cout, db);
      VP_LAUNCH_CHECK();
    }
    const bf16* Wt = n->wb + L.woff;
    if (L.kind == CONV3) {
      const Act& X2 = L.in2 >= 0 ? n->acts[L.in2] : X;
      const int C = L.cin + L.cin2;
      ensure(n->col, n->col_n, P * 9 * C);
      hipLaunchKernelGGL(k_im2col3, dim3(gs(P * 9 * C / 8)), dim3(256), 0, s, X.y, L.cin,
                         L.in2 >= 0 ? X2.y : nullptr, L.cin2, Bn, L.H, L.W, n->col);
      VP_LAUNCH_CHECK();
      // dW = col^T g  [9C x cout]
      gemm_f32(n, true, false, n->col, n->gb, 9 * C, L.cout, (int)P, 9 * C, L.cout, dW);
      // dcol = g W^T  [P x 9C]
      ensure(n->fcol, n->fcol_n, P * 9 * C);
      gemm<false, true, false>(s, n->gb, Wt, (int)P, 9 * C, L.cout, L.cout, L.cout, nullptr, 0, nullptr, n->fcol,
                               9 * C, 1);
      ensure(n->tmp, n->tmp_n, P * C);
      float* t1 = n->tmp;
      float* t2 = L.in2 >= 0 ? n->tmp + P * L.cin : nullptr;
      hipLaunchKernelGGL(k_col2im3, dim3(gs(P * C / 4)), dim3(256), 0, s, n->fcol, L.cin, L.cin2, Bn, L.H, L.W, t1,
                         t2);
      VP_LAUNCH_CHECK();
      if (L.in > 0) {
        hipLaunchKernelGGL(k_add_into, dim3(gs(P * L.cin)), dim3(256), 0, s, X.g, t1, P * L.cin);
        VP_LAUNCH_CHECK();
      }
      if (L.in2 >= 0) {
        hipLaunchKernelGGL(k_add_into, dim3(gs(P * L.cin2)), dim3(256), 0, s, n->acts[L.in2].g, t2, P * L.cin2);
        VP_LAUNCH_CHECK();
      }
    } else if (L.kind == DOWN) {
      ensure(n->col, n->col_n, P * 4 * L.cin);
      hipLaunchKernelGGL(k_s2d<bf16>, dim3(gs(P * 4 * L.cin)), dim3(256), 0, s, X.y, Bn, L.H, L.W, L.cin, n->col);
      VP_LAUNCH_CHECK();
      gemm_f32(n, true, false, n->col, n->gb, 4 * L.cin, L.cout, (int)P, 4 * L.cin, L.cout, dW);
      ensure(n->fcol, n->fcol_n, P * 4 * L.cin);
      gemm<false, true, false>(s, n->gb, Wt, (int)P, 4 * L.cin, L.cout, L.cout, L.cout, nullptr, 0, nullptr, n->fcol,
                               4 * L.cin, 1);
      ensure(n->tmp, n->tmp_n, P * 4 * L.cin);
      hipLaunchKernelGGL((k_d2s<float, float>), dim3(gs(P * 4 * L.cin)), dim3(256), 0, s, n->fcol, Bn, L.H, L.W,
                         L.cin, (const float*)nullptr, 0, n->tmp);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_add_into, dim3(gs(P * 4 * L.cin)), dim3(256), 0, s, X.g, n->tmp, P * 4 * L.cin);
      VP_LAUNCH_CHECK();
    } else {  // UP: Y4 = X W [Pin x 4cout], then depth-to-space
      const size_t Pin = (size_t)Bn * X.H * X.W;
      ensure(n->col, n->col_n, Pin * 4 * L.cout);
      hipLaunchKernelGGL(k_s2d<bf16>, dim3(gs(Pin * 4 * L.cout)), dim3(256), 0, s, n->gb, Bn, X.H, X.W, L.cout,
                         n->col);
      VP_LAUNCH_CHECK();
      // dW = X^T g4  [cin x 4cout]
      gemm_f32(n, true, false, X.y, n->col, L.cin, 4 * L.cout, (int)Pin, L.cin, 4 * L.cout, dW);
      ensure(n->tmp, n->tmp_n, Pin * L.cin);
      gemm<false, true, false>(s, n->col, Wt, (int)Pin, L.cin, 4 * L.cout, 4 * L.cout, 4 * L.cout, nullptr, 0,
                               nullptr, n->tmp, L.cin, 1);
      hipLaunchKernelGGL(k_add_into, dim3(gs(Pin * L.cin)), dim3(256), 0, s, X.g, n->tmp, Pin * L.cin);
      VP_LAUNCH_CHECK();
    }
  }
}

}  // namespace net
}  // namespace vp

using namespace vp;
using namespace vp::net;

namespace {
template <typename F>
int nguard(vpnet_s* n, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    if (n) n->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (n) n->err = e.what();
    return VP_EHIP;
  }
}
void nreq(bool ok, const char* msg) {
  if (!ok) throw Error(VP_EINVAL, msg);
}
}  // namespace

extern "C" {

int vpnet_create(int batch, int height, int width, void* stream, vpnet_s** out) {
  if (!out) return VP_EINVAL;
  *out = nullptr;
  if (batch < 1 || height < 8 || width < 8 || height % 8 || width % 8) return VP_EINVAL;
  vpnet_s* n = new vpnet_s();
  const int rc = nguard(n, [&] {
    n->stream = (hipStream_t)stream;
    n->Bn = batch;
    n->H = height;
    n->W = width;
    build(n);
    for (auto& a : n->acts) a.y = dalloc<bf16>((size_t)batch * a.H * a.W * a.C);
    n->w = dalloc<float>(n->nparam);
    n->wb = dalloc<bf16>(n->nparam);
    n->g = dalloc<float>(n->nparam);
    n->m = dalloc<float>(n->nparam);
    n->v = dalloc<float>(n->nparam);
    VP_HIP(hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->stream));
    VP_HIP(hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->stream));
    const size_t P = (size_t)batch * height * width;
    n->out = dalloc<float>(P * kCout);
    n->gout = dalloc<float>(P * kCout);
    n->red = dalloc<double>(1024);
    VP_HIP(hipHostMalloc((void**)&n->hred, 16 * sizeof(double), hipHostMallocDefault));
    return VP_OK;
  });
  if (rc != VP_OK) {
    vpnet_destroy(n);
    return rc;
  }
  *out = n;
  return VP_OK;
}

void vpnet_destroy(vpnet_s* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  for (auto& a : n->acts) {
    if (a.y) (void)hipFree(a.y);
    if (a.g) (void)hipFree(a.g);
  }
  void* bufs[] = {n->w, n->wb, n->g, n->m, n->v, n->col, n->fcol, n->part, n->gb, n->tmp, n->out, n->gout, n->red,
                  n->feat};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (n->hred) (void)hipHostFree(n->hred);
  delete n;
}

const char* vpnet_last_error(vpnet_s* n) { return n ? n->err.c_str() : ""; }

int64_t vpnet_param_count(vpnet_s* n) { return n ? (int64_t)n->nparam : -1; }

int vpnet_set_params(vpnet_s* n, const float* src) {
  return nguard(n, [&] {
    nreq(n && src, "null argument");
    VP_HIP(hipMemcpyAsync(n->w, src, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3(gs(n->nparam)), dim3(256), 0, n->stream, n->w, n->wb, n->nparam);
    VP_LAUNCH_CHECK();
    VP_HIP(hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->stream));
    VP_HIP(hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->stream));
    n->step = 0;
    return VP_OK;
  });
}

int vpnet_get_params(vpnet_s* n, float* dst) {
  return nguard(n, [&] {
    nreq(n && dst, "null argument");
    VP_HIP(hipMemcpyAsync(dst, n->w, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return VP_OK;
  });
}

int vpnet_get_grads(vpnet_s* n, float* dst) {
  return nguard(n, [&] {
    nreq(n && dst, "null argument");
    VP_HIP(hipMemcpyAsync(dst, n->g, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return VP_OK;
  });
}

int vpnet_forward(vpnet_s* n, const float* input, float* output) {
  return nguard(n, [&] {
    nreq(n && input && output, "null argument");
    const size_t P = (size_t)n->Bn * n->H * n->W;
    hipLaunchKernelGGL(k_to_bf16, dim3(gs(P * kCin)), dim3(256), 0, n->stream, input, n->acts[0].y, P * kCin);
    VP_LAUNCH_CHECK();
    forward(n);
    VP_HIP(hipMemcpyAsync(output, n->out, P * kCout * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    return VP_OK;
  });
}

int vpnet_backward(vpnet_s* n, const float* input, const float* target, float* loss) {
  return nguard(n, [&] {
    nreq(n && input && target, "null argument");
    const size_t P = (size_t)n->Bn * n->H * n->W;
    hipLaunchKernelGGL(k_to_bf16, dim3(gs(P * kCin)), dim3(256), 0, n->stream, input, n->acts[0].y, P * kCin);
    VP_LAUNCH_CHECK();
    forward(n);
    const size_t no = P * kCout;
    hipLaunchKernelGGL(k_mse, dim3(512), dim3(256), 0, n->stream, n->out, target, no, n->gout, n->red);
    VP_LAUNCH_CHECK();
    launch_finish_sum(n->stream, n->red, 512, 1, n->red + 600);
    backward(n);
    if (loss) {
      VP_HIP(hipMemcpyAsync(n->hred, n->red + 600, sizeof(double), hipMemcpyDeviceToHost, n->stream));
      VP_HIP(hipStreamSynchronize(n->stream));
      *loss = (float)(n->hred[0] / (double)no);
    }
    return VP_OK;
  });
}

int vpnet_adam(vpnet_s* n, float lr) {
  return nguard(n, [&] {
    nreq(n != nullptr && lr > 0.f, "bad argument");
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)n->step), c2 = 1.f - powf(b2, (float)n->step);
    hipLaunchKernelGGL(k_adam, dim3(gs(n->nparam)), dim3(256), 0, n->stream, n->w, n->g, n->m, n->v, n->nparam, lr,
                       b1, b2, 1e-8f, c1, c2, n->wb);
    VP_LAUNCH_CHECK();
    return VP_OK;
  });
}

int vpnet_train_step(vpnet_s* n, const float* input, const float* target, float lr, float* loss) {
  const int rc = vpnet_backward(n, input, target, loss);
  if (rc != VP_OK) return rc;
  return vpnet_adam(n, lr);
}

int vpnet_features(int nx, int ny, int f, const double* H, const double* A, const double* va, const double* vo,
                   const double* vp_, float* out, void* stream) {
  if (nx < 1 || ny < 1 || f < 1 || nx % f || ny % f || !H || !A || !va || !vo || !vp_ || !out) return VP_EINVAL;
  hipLaunchKernelGGL(k_features, dim3(gs((size_t)(nx / f) * (ny / f))), dim3(256), 0, (hipStream_t)stream, nx, ny, f,
                     H, A, va, vo, vp_, out);
  return hipGetLastError() == hipSuccess ? VP_OK : VP_EHIP;
}

int vpnet_targets(int nx, int ny, const double* v, const double* pi, const double* v_prev, float* out,
                  void* stream) {
  if (nx < 1 || ny < 1 || !v || !pi || !out) return VP_EINVAL;
  hipLaunchKernelGGL(k_targets, dim3(gs((size_t)nx * ny)), dim3(256), 0, (hipStream_t)stream, nx, ny, v, pi, v_prev,
                     out);
  return hipGetLastError() == hipSuccess ? VP_OK : VP_EHIP;
}

int vpnet_guess(int nx, int ny, const float* outp, int wc, int hc, const double* v_prev, double* v0, double* pi0,
                void* stream) {
  if (nx < 1 || ny < 1 || wc < 1 || hc < 1 || !outp || !v0) return VP_EINVAL;
  const size_t n = (size_t)(nx + 1) * (ny + 1) + (size_t)nx * ny;
  hipLaunchKernelGGL(k_guess, dim3(gs(n)), dim3(256), 0, (hipStream_t)stream, nx, ny, outp, wc, hc, v_prev, v0,
                     pi0);
  return hipGetLastError() == hipSuccess ? VP_OK : VP_EHIP;
}

constexpr int kMaxPool = VPNET_MAX_POOL;

int vpnet_infer(vpnet_s* n, vp_ctx c, int candidates, double* v0, double* pi0, int* chosen) {
  return nguard(n, [&] {
    nreq(n && c && v0 && pi0, "null argument");
    nreq(candidates > 0 && candidates <= (VPNET_START_LEARNED | VPNET_START_PREVIOUS | VPNET_START_ZERO),
         "candidates must be a non-empty set of VPNET_START_* flags");
    nreq(n->Bn == 1, "vpnet_infer needs a network of batch 1");
    nreq(c->order == 1, "the learned start takes Q1 velocity elements");
    nreq(c->stream == n->stream, "the network and the context must share a stream");
    const int nx = c->ec.nx, ny = c->ec.ny;
    nreq(nx % n->W == 0 && ny % n->H == 0 && nx / n->W == ny / n->H,
         "the mesh must be f times the network's grid on both sides (integer f)");
    if (!c->have_state) throw Error(VP_ESTATE, "vp_set_state not called");
    const int f = nx / n->W;
    if (f > kMaxPool) {
      // pooled further than measured: the learned start is not a candidate
      nreq(candidates != VPNET_START_LEARNED, "mesh finer than the network's grid times VPNET_MAX_POOL");
      candidates &= ~VPNET_START_LEARNED;
    }
    const size_t P = (size_t)n->H * n->W;
    if (!n->feat) n->feat = dalloc<float>(P * kCin);
    hipStream_t s = n->stream;
    if (candidates & VPNET_START_LEARNED) {
      hipLaunchKernelGGL(k_features, dim3(gs(P)), dim3(256), 0, s, nx, ny, f, c->Hs, c->As, c->vas, c->vo, c->vps,
                         n->feat);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_to_bf16, dim3(gs(P * kCin)), dim3(256), 0, s, n->feat, n->acts[0].y, P * kCin);
      VP_LAUNCH_CHECK();
      forward(n);
      const size_t m = (size_t)(nx + 1) * (ny + 1) + (size_t)nx * ny;
      hipLaunchKernelGGL(k_guess, dim3(gs(m)), dim3(256), 0, s, nx, ny, n->out, n->W, n->H, c->vps, v0, pi0);
      VP_LAUNCH_CHECK();
      if (f > 1) {
        // pooled inputs: the proposed change damped, pi consistent with the result
        launch_axpby(s, 1.0 - VPNET_POOLED_SCALE, c->vps, VPNET_POOLED_SCALE, v0, c->ndof);
        launch_pi_init(c, v0, pi0);
      }
    }
    // the start with the lowest energy Phi (eq. energy), first in the order
    // learned, previous, zero on ties
    int best = 0;
    double be = 0.0;
    auto consider = [&](int flag, const double* v) {
      const double e = energy_at(c, v);
      if (!best || e < be) {
        best = flag;
        be = e;
      }
    };
    if (candidates & VPNET_START_LEARNED) consider(VPNET_START_LEARNED, v0);
    if (candidates & VPNET_START_PREVIOUS) consider(VPNET_START_PREVIOUS, c->vps);
    if (candidates & VPNET_START_ZERO) {
      double* z = c->work + 4 * c->ndof;
      launch_fill(s, z, 0.0, c->ndof);
      consider(VPNET_START_ZERO, z);
    }
    if (best == VPNET_START_PREVIOUS) {
      VP_HIP(hipMemcpyAsync(v0, c->vps, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_pi_init(c, v0, pi0);
    } else if (best == VPNET_START_ZERO) {
      launch_fill(s, v0, 0.0, c->ndof);
      launch_fill(s, pi0, 0.0, 4 * 3 * c->ncell);
    }
    if (chosen) *chosen = best;
    return VP_OK;
  });
}

int vpnet_inspect(vpnet_s* n, int act, float* y, float* g, int64_t* count) {
  return nguard(n, [&] {
    nreq(n != nullptr, "null network");
    nreq(act >= 0 && act < (int)n->acts.size(), "activation index out of range");
    const Act& a = n->acts[act];
    const size_t m = (size_t)n->Bn * a.H * a.W * a.C;
    if (count) *count = (int64_t)m;
    if (y) {
      hipLaunchKernelGGL(k_bf16_to_f32, dim3(gs(m)), dim3(256), 0, n->stream, a.y, m, y);
      VP_LAUNCH_CHECK();
    }
    if (g) {
      if (!a.g) throw Error(VP_ESTATE, "no gradients before vpnet_backward");
      VP_HIP(hipMemcpyAsync(g, a.g, m * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    }
    return VP_OK;
  });
}

int vpnet_gemm(const void* A, const void* B, float* C, int M, int N, int K, int a_trans, int b_trans, void* stream) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return VP_EINVAL;
  try {
    hipStream_t s = (hipStream_t)stream;
    const int lda = a_trans ? M : K, ldb = b_trans ? K : N;
    const bf16* a = (const bf16*)A;
    const bf16* b = (const bf16*)B;
    if (a_trans && b_trans) gemm<true, true, false>(s, a, b, M, N, K, lda, ldb, nullptr, 0, nullptr, C, N, 1);
    else if (a_trans) gemm<true, false, false>(s, a, b, M, N, K, lda, ldb, nullptr, 0, nullptr, C, N, 1);
    else if (b_trans) gemm<false, true, false>(s, a, b, M, N, K, lda, ldb, nullptr, 0, nullptr, C, N, 1);
    else gemm<false, false, false>(s, a, b, M, N, K, lda, ldb, nullptr, 0, nullptr, C, N, 1);
  } catch (const Error& e) {
    return e.code;
  }
  return VP_OK;
}

}  // extern "C"
