// Structured smoothed-aggregation AMG on block 9-point stencils.
//
// Every level is a structured grid of nxn x nyn nodes carrying B dofs per node
// (B = 2 on the finest level, 3 on coarse levels: the rigid-body modes), and its
// operator is a symmetric block 9-point stencil stored as five B x B blocks per
// node (self, E, N, NE, NW; the W, S, SW, SE couplings are the transposes held by
// the neighbours), block-interleaved: A[aidx(B, nn, blk, node, r, c)].
//
// Aggregates are 3x3 node blocks (the last one per direction takes the 3..5
// remaining nodes).  One block-Jacobi smoothing step of the tentative
// prolongator widens each column's support by one node ring, which keeps the
// Galerkin operator P^T A P a block 9-point stencil on the aggregate grid, so
// every level reuses the same stencil kernels and no sparse-matrix product with
// run-time sparsity is needed.  This replaces the paper's classical AMG
// (BoomerAMG, Sec. 5.4); its role there is the preconditioner of FGMRES for the
// SPD linearisations with strongly varying coefficients.
#include "vp_internal.h"

namespace vp {

namespace {

template <typename T> struct Acc { using type = float; };
template <> struct Acc<double> { using type = double; };

// ---- aggregation along one direction ---------------------------------------
__device__ __forceinline__ int agg_of(int i, int nagg) {
  const int a = i / 3;
  return a < nagg ? a : nagg - 1;
}
__device__ __forceinline__ int agg_last(int a, int n, int nagg) { return a == nagg - 1 ? n - 1 : 3 * a + 2; }
// aggregate adjacent to node i through the 9-point stencil, other than its own (-1: none)
__device__ __forceinline__ int agg_other(int i, int n, int nagg) {
  const int a = agg_of(i, nagg);
  if (i == 3 * a && a > 0) return a - 1;
  if (i == agg_last(a, n, nagg) && a < nagg - 1) return a + 1;
  return -1;
}
// slot (0/1) of coarse index J for node i along one direction, -1 if none
__device__ __forceinline__ int slot1(int i, int n, int nagg, int J) {
  if (agg_of(i, nagg) == J) return 0;
  if (agg_other(i, n, nagg) == J) return 1;
  return -1;
}

// Aggregate-major order of the fine nodes for the Galerkin scratch W: the nodes at
// position (px, py) < 3 inside their aggregate form one plane indexed like the
// coarse nodes, so the threads of consecutive coarse nodes read consecutive
// addresses; the extra nodes of a last aggregate longer than three (at most two
// columns and two rows, nxn - 3 ncx and nyn - 3 ncy) follow the nine planes.
__host__ __device__ __forceinline__ size_t gw_size(int nxn, int nyn, int ncx, int ncy) {
  return (size_t)9 * ncx * ncy + (size_t)(nxn - 3 * ncx) * nyn + (size_t)(nyn - 3 * ncy) * nxn;
}
__device__ __forceinline__ size_t gw_index(int i, int j, int nxn, int nyn, int ncx, int ncy) {
  const int ax = agg_of(i, ncx), ay = agg_of(j, ncy);
  const int px = i - 3 * ax, py = j - 3 * ay;
  const size_t ncn = (size_t)ncx * ncy;
  if (px < 3 && py < 3) return (size_t)(py * 3 + px) * ncn + (size_t)ay * ncx + ax;
  if (px >= 3) return 9 * ncn + (size_t)(px - 3) * nyn + j;
  return 9 * ncn + (size_t)(nxn - 3 * ncx) * nyn + (size_t)(py - 3) * nxn + i;
}

// ---- block access ------------------------------------------------------------
// 9 directions: 0 self, 1 E, 2 N, 3 NE, 4 NW, 5 W, 6 S, 7 SW, 8 SE
__constant__ int kDI[9] = {0, 1, 0, 1, -1, -1, 0, -1, 1};
__constant__ int kDJ[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};

// Raw B*B values of one stored block (contiguous), widened to TA.  2x2 FP32 and
// FP64 blocks use 16-byte vector loads.
template <int B, typename TM, typename TA>
__device__ __forceinline__ void load_raw(const TM* __restrict__ p, TA (&v)[B * B]) {
  if constexpr (B == 2 && std::is_same<TM, float>::value) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = (TA)t.x; v[1] = (TA)t.y; v[2] = (TA)t.z; v[3] = (TA)t.w;
  } else if constexpr (B == 2 && std::is_same<TM, __hip_bfloat16>::value) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);   // 4 BF16 = 8 bytes
    v[0] = (TA)__uint_as_float(t.x << 16); v[1] = (TA)__uint_as_float(t.x & 0xffff0000u);
    v[2] = (TA)__uint_as_float(t.y << 16); v[3] = (TA)__uint_as_float(t.y & 0xffff0000u);
  } else if constexpr (B == 2 && std::is_same<TM, _Float16>::value) {
    typedef _Float16 half4 __attribute__((ext_vector_type(4)));
    const half4 t = *reinterpret_cast<const half4*>(p);   // 4 FP16 = 8 bytes
    v[0] = (TA)t.x; v[1] = (TA)t.y; v[2] = (TA)t.z; v[3] = (TA)t.w;
  } else if constexpr (B == 2 && std::is_same<TM, double>::value) {
    const double2 t0 = reinterpret_cast<const double2*>(p)[0];
    const double2 t1 = reinterpret_cast<const double2*>(p)[1];
    v[0] = (TA)t0.x; v[1] = (TA)t0.y; v[2] = (TA)t1.x; v[3] = (TA)t1.y;
  } else {
#pragma unroll
    for (int k = 0; k < B * B; ++k) v[k] = (TA)ld(p + k);
  }
}

// B values of one node of a vector (2-dof nodes as one 8/16-byte load or store)
template <int B, typename TV, typename TA>
__device__ __forceinline__ void load_node(const TV* __restrict__ x, size_t n, TA (&v)[B]) {
  if constexpr (B == 2 && std::is_same<TV, float>::value) {
    const float2 t = reinterpret_cast<const float2*>(x)[n];
    v[0] = (TA)t.x; v[1] = (TA)t.y;
  } else if constexpr (B == 2 && std::is_same<TV, double>::value) {
    const double2 t = reinterpret_cast<const double2*>(x)[n];
    v[0] = (TA)t.x; v[1] = (TA)t.y;
  } else {
#pragma unroll
    for (int k = 0; k < B; ++k) v[k] = (TA)x[n * B + k];
  }
}
template <int B, typename TV, typename TA>
__device__ __forceinline__ void store_node(TV* __restrict__ x, size_t n, const TA (&v)[B]) {
  if constexpr (B == 2 && std::is_same<TV, float>::value) {
    reinterpret_cast<float2*>(x)[n] = make_float2((float)v[0], (float)v[1]);
  } else if constexpr (B == 2 && std::is_same<TV, double>::value) {
    reinterpret_cast<double2*>(x)[n] = make_double2((double)v[0], (double)v[1]);
  } else {
#pragma unroll
    for (int k = 0; k < B; ++k) x[n * B + k] = (TV)v[k];
  }
}

// Load the B x B block coupling node (i,j) (rows) to its neighbour in direction d
// (columns).  Caller guarantees the neighbour exists.
template <int B, typename TM, typename TA>
__device__ __forceinline__ void load_block(const TM* __restrict__ A, size_t nn, int nxn, int i, int j,
                                           int d, TA (&out)[B][B]) {
  const size_t n = (size_t)j * nxn + i;
  TA v[B * B];
  if (d <= 4) {
    load_raw<B>(A + aidx(B, nn, d, n, 0, 0), v);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) out[r][c] = v[r * B + c];
  } else {
    const int blk = d - 4;  // W->E(1), S->N(2), SW->NE(3), SE->NW(4)
    const size_t m = (size_t)(j + kDJ[d]) * nxn + (i + kDI[d]);
    load_raw<B>(A + aidx(B, nn, blk, m, 0, 0), v);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) out[r][c] = v[c * B + r];
  }
}

// Inverse of a B x B block.  The block is first scaled by its largest entry:
// operator entries reach ~1e17 and the cofactor products (~1e51 for B = 3) would
// overflow FP32 otherwise.
template <int B, typename TA>
__device__ __forceinline__ void invert_block(const TA (&Din)[B][B], TA (&Di)[B][B]) {
  TA m = TA(0);
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c) m = fmax(m, fabs(Din[r][c]));
  const TA is = m > TA(0) ? TA(1) / m : TA(1);
  TA D[B][B];
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c) D[r][c] = Din[r][c] * is;
  if constexpr (B == 2) {
    const TA det = D[0][0] * D[1][1] - D[0][1] * D[1][0];
    const TA id = det != TA(0) ? is / det : TA(0);
    Di[0][0] = D[1][1] * id; Di[0][1] = -D[0][1] * id;
    Di[1][0] = -D[1][0] * id; Di[1][1] = D[0][0] * id;
  } else {
    const TA c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
    const TA c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
    const TA c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
    const TA det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
    const TA id = det != TA(0) ? is / det : TA(0);
    Di[0][0] = c00 * id;
    Di[1][0] = c01 * id;
    Di[2][0] = c02 * id;
    Di[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * id;
    Di[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * id;
    Di[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * id;
    Di[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * id;
    Di[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * id;
    Di[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * id;
  }
}

// (A x)_n for node (i, j) of the stencil; getx(m, ii, jj, xm) supplies the B
// values of x at neighbour node m = (ii, jj) (global memory or a staged tile).
template <int B, typename TM, typename TA, typename GetX>
__device__ __forceinline__ void stencil_row_f(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int i, int j,
                                              GetX getx, TA (&y)[B], TA (&D)[B][B]) {
#pragma unroll
  for (int r = 0; r < B; ++r) y[r] = TA(0);
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int ii = i + kDI[d], jj = j + kDJ[d];
    if (ii < 0 || jj < 0 || ii >= nxn || jj >= nyn) continue;
    TA blk[B][B];
    load_block<B>(A, nn, nxn, i, j, d, blk);
    if (d == 0) {
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < B; ++c) D[r][c] = blk[r][c];
    }
    const size_t m = (size_t)jj * nxn + ii;
    TA xm[B];
    getx(m, ii, jj, xm);
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) y[r] += blk[r][c] * xm[c];
  }
}

// (A x)_n of the symmetric block 25-point stencil of Q2 elements (ST = 1, B = 2):
// the 13 stored blocks of node n times x at their offsets, plus the transposes of
// the blocks stored at n - o for the 12 non-self offsets o.
template <typename TM, typename TA, typename GetX>
__device__ __forceinline__ void stencil_row25_f(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int i, int j,
                                                GetX getx, TA (&y)[2], TA (&D)[2][2]) {
  y[0] = y[1] = TA(0);
  const size_t n = (size_t)j * nxn + i;
#pragma unroll
  for (int d = 0; d < 13; ++d) {
    const int ox = q2_ox(d), oy = q2_oy(d);
    {
      const int ii = i + ox, jj = j + oy;
      if (ii >= 0 && ii < nxn && jj < nyn) {
        TA v[4];
        load_raw<2>(A + aidx(2, nn, d, n, 0, 0), v);
        if (d == 0) {
          D[0][0] = v[0]; D[0][1] = v[1]; D[1][0] = v[2]; D[1][1] = v[3];
        }
        TA xm[2];
        getx((size_t)jj * nxn + ii, ii, jj, xm);
        y[0] += v[0] * xm[0] + v[1] * xm[1];
        y[1] += v[2] * xm[0] + v[3] * xm[1];
      }
    }
    if (d > 0) {
      const int ii = i - ox, jj = j - oy;
      if (ii >= 0 && ii < nxn && jj >= 0) {
        const size_t m = (size_t)jj * nxn + ii;
        TA v[4];
        load_raw<2>(A + aidx(2, nn, d, m, 0, 0), v);
        TA xm[2];
        getx(m, ii, jj, xm);
        y[0] += v[0] * xm[0] + v[2] * xm[1];
        y[1] += v[1] * xm[0] + v[3] * xm[1];
      }
    }
  }
}

// (A x)_n: ST = 0 the block 9-point stencil of every AMG level, ST = 1 the
// 25-point stencil of Q2 elements on the finest level
template <int B, int ST = 0, typename TM, typename TV, typename TA>
__device__ __forceinline__ void stencil_row(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int i,
                                            int j, const TV* __restrict__ x, TA (&y)[B],
                                            TA (&D)[B][B]) {
  if constexpr (ST == 1) {
    static_assert(B == 2, "the 25-point stencil has 2x2 blocks");
    stencil_row25_f<TM, TA>(A, nn, nxn, nyn, i, j, [&](size_t m, int, int, TA (&xm)[2]) { load_node<2>(x, m, xm); },
                            y, D);
  } else {
    stencil_row_f<B>(A, nn, nxn, nyn, i, j, [&](size_t m, int, int, TA (&xm)[B]) { load_node<B>(x, m, xm); }, y, D);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// stencil kernels
// ---------------------------------------------------------------------------
// Per-node bodies of the stencil and transfer kernels.  Each __global__ kernel
// below maps one thread to one node (eight lanes to one coarse node for the
// restriction); the single-workgroup kernel for the smallest levels loops the
// same bodies over the nodes, so both give identical results.

// r = b - A x at node n (b may be null: r = -A x); in-place r == b is allowed.
template <int B, typename TM, typename TV, int ST = 0>
__device__ __forceinline__ void node_sten_resid(const TM* __restrict__ A, size_t nn, int nxn, int nyn,
                                                const TV* __restrict__ x, const TV* b, TV* r, size_t n) {
  using TA = typename Acc<TV>::type;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  TA y[B], D[B][B], bb[B];
  stencil_row<B, ST>(A, nn, nxn, nyn, i, j, x, y, D);
  if (b) load_node<B>(b, n, bb);
#pragma unroll
  for (int k = 0; k < B; ++k) bb[k] = (b ? bb[k] : TA(0)) - y[k];
  store_node<B>(r, n, bb);
}

// Chebyshev first step: d = D^{-1} src * inv_theta.  x (if given) = d, or x += d
// with add; r (if given) = src.
template <int B, typename TM, typename TV>
__device__ __forceinline__ void node_cheb_first(const TM* __restrict__ A, size_t nn, const TV* __restrict__ src,
                                                TV* __restrict__ r, TV* __restrict__ d, TV* __restrict__ x,
                                                typename Acc<TV>::type inv_theta, int add, size_t n) {
  using TA = typename Acc<TV>::type;
  TA v[B * B], D[B][B], Di[B][B], sv[B], dk[B];
  load_raw<B>(A + aidx(B, nn, 0, n, 0, 0), v);
#pragma unroll
  for (int rr = 0; rr < B; ++rr)
#pragma unroll
    for (int c = 0; c < B; ++c) D[rr][c] = v[rr * B + c];
  invert_block<B>(D, Di);
  load_node<B>(src, n, sv);
#pragma unroll
  for (int k = 0; k < B; ++k) {
    TA t = TA(0);
#pragma unroll
    for (int c = 0; c < B; ++c) t += Di[k][c] * sv[c];
    dk[k] = t * inv_theta;
  }
  store_node<B>(d, n, dk);
  if (x) {
    TA xn[B];
    if (add) {
      load_node<B>(x, n, xn);
#pragma unroll
      for (int k = 0; k < B; ++k) xn[k] += dk[k];
    } else {
#pragma unroll
      for (int k = 0; k < B; ++k) xn[k] = dk[k];
    }
    store_node<B>(x, n, xn);
  }
  if (r) store_node<B>(r, n, sv);
}

// Residual and first Chebyshev step of post-smoothing in one sweep:
// r = b - A x, d = D^{-1} r * inv_theta.  x itself is not updated here (its
// neighbours are still being read); the following step adds d (xmode 1).
template <int B, typename TM, typename TV, int ST = 0>
__device__ __forceinline__ void node_resid_first(const TM* __restrict__ A, size_t nn, int nxn, int nyn,
                                                 const TV* __restrict__ x, const TV* __restrict__ b,
                                                 TV* __restrict__ r, TV* __restrict__ d,
                                                 typename Acc<TV>::type inv_theta, size_t n) {
  using TA = typename Acc<TV>::type;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  TA y[B], D[B][B], Di[B][B], rn[B], dk[B];
  stencil_row<B, ST>(A, nn, nxn, nyn, i, j, x, y, D);
  invert_block<B>(D, Di);
  load_node<B>(b, n, rn);
#pragma unroll
  for (int k = 0; k < B; ++k) rn[k] -= y[k];
  store_node<B>(r, n, rn);
#pragma unroll
  for (int k = 0; k < B; ++k) {
    TA t = TA(0);
#pragma unroll
    for (int c = 0; c < B; ++c) t += Di[k][c] * rn[c];
    dk[k] = t * inv_theta;
  }
  store_node<B>(d, n, dk);
}

// Chebyshev step: r = rin - A dp; dn = cdd dp + cdr D^{-1} r;
//   xmode 0: xout = xin + dn;  1: xout = (xin + dp) + dn;  2: xout = dp + dn (xin not read).
// rin may equal rout and xin may equal xout.
template <int B, typename TM, typename TV, int ST = 0>
__device__ __forceinline__ void node_cheb_step(const TM* __restrict__ A, size_t nn, int nxn, int nyn,
                                               const TV* __restrict__ dp, const TV* rin, TV* rout,
                                               TV* __restrict__ dn, const TV* xin, TV* xout,
                                               typename Acc<TV>::type cdd, typename Acc<TV>::type cdr, int xmode,
                                               size_t n) {
  using TA = typename Acc<TV>::type;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  TA y[B], D[B][B], Di[B][B], rn[B], dpn[B], xn[B], dk[B];
  stencil_row<B, ST>(A, nn, nxn, nyn, i, j, dp, y, D);
  invert_block<B>(D, Di);
  load_node<B>(rin, n, rn);
  load_node<B>(dp, n, dpn);
  if (xmode == 2) {
#pragma unroll
    for (int k = 0; k < B; ++k) xn[k] = dpn[k];
  } else {
    load_node<B>(xin, n, xn);
    if (xmode == 1) {
#pragma unroll
      for (int k = 0; k < B; ++k) xn[k] += dpn[k];
    }
  }
#pragma unroll
  for (int k = 0; k < B; ++k) rn[k] -= y[k];
  store_node<B>(rout, n, rn);
#pragma unroll
  for (int k = 0; k < B; ++k) {
    TA t = TA(0);
#pragma unroll
    for (int c = 0; c < B; ++c) t += Di[k][c] * rn[c];
    dk[k] = fma(cdd, dpn[k], cdr * t);   // the contraction every sweep kernel writes
    xn[k] += dk[k];
  }
  store_node<B>(dn, n, dk);
  store_node<B>(xout, n, xn);
}

// ---------------------------------------------------------------------------
// transfers: P stored per fine node as 4 slots x (B x 3), one plane per component
//   P[pidx(B, nn, slot, node, r, c)]
// slot = sx + 2 sy, sx = 0: own aggregate in x, 1: the adjacent one (agg_other)
// ---------------------------------------------------------------------------
// Restriction with eight lanes per coarse node I (lane sub of the group, gid / 8 =
// I): I's window spans at most 6 x 6 fine nodes (the aggregate, one node on each
// side, a last aggregate of up to 5); lane k sums the window nodes k, k+8, ... and
// the eight partial sums are combined by a fixed butterfly within the lane group
// (deterministic).  All eight lanes of a group must call this together.
constexpr int kRestrictLanes = 8;
template <int B, typename TP, typename TV>
__device__ __forceinline__ void group_restrict(const TP* __restrict__ P, size_t nn, int nxn, int nyn, int ncx,
                                               int ncy, const TV* __restrict__ r, TV* __restrict__ bc, size_t I,
                                               int sub) {
  using TA = typename Acc<TV>::type;
  const int Ix = (int)(I % ncx), Iy = (int)(I / ncx);
  const int i0 = max(3 * Ix - 1, 0), i1 = min(agg_last(Ix, nxn, ncx) + 1, nxn - 1);
  const int j0 = max(3 * Iy - 1, 0), j1 = min(agg_last(Iy, nyn, ncy) + 1, nyn - 1);
  TA acc[3] = {TA(0), TA(0), TA(0)};
#pragma unroll
  for (int w = sub; w < 36; w += kRestrictLanes) {
    const int i = i0 + w % 6, j = j0 + w / 6;
    if (i > i1 || j > j1) continue;
    const int sx = slot1(i, nxn, ncx, Ix), sy = slot1(j, nyn, ncy, Iy);
    if (sx < 0 || sy < 0) continue;
    const int s = sx + 2 * sy;
    const size_t n = (size_t)j * nxn + i;
    TA rv[B];
    load_node<B>(r, n, rv);
#pragma unroll
    for (int rr = 0; rr < B; ++rr)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += (TA)ld(P + pidx(B, nn, s, n, rr, c)) * rv[rr];
  }
#pragma unroll
  for (int o = 1; o < kRestrictLanes; o <<= 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
  if (sub == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) bc[I * 3 + c] = (TV)acc[c];
  }
}

// x += P xc at fine node n
template <int B, typename TP, typename TV>
__device__ __forceinline__ void prolong_value(const TP* __restrict__ P, size_t nn, int nxn, int nyn, int ncx,
                                              int ncy, const TV* __restrict__ xc, const TV* xi, size_t n,
                                              typename Acc<TV>::type (&acc)[B]) {
  using TA = typename Acc<TV>::type;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  const int ax[2] = {agg_of(i, ncx), agg_other(i, nxn, ncx)};
  const int ay[2] = {agg_of(j, ncy), agg_other(j, nyn, ncy)};
#pragma unroll
  for (int rr = 0; rr < B; ++rr) acc[rr] = (TA)xi[n * B + rr];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int Jx = ax[s & 1], Jy = ay[s >> 1];
    if (Jx < 0 || Jy < 0) continue;
    const size_t J = (size_t)Jy * ncx + Jx;
    TA xj[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) xj[c] = (TA)xc[J * 3 + c];
#pragma unroll
    for (int rr = 0; rr < B; ++rr)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[rr] += (TA)ld(P + pidx(B, nn, s, n, rr, c)) * xj[c];
  }
}

// x = xi + P xc at fine node n
template <int B, typename TP, typename TV>
__device__ __forceinline__ void node_prolong_add(const TP* __restrict__ P, size_t nn, int nxn, int nyn, int ncx,
                                                 int ncy, const TV* __restrict__ xc, const TV* xi, TV* x, size_t n) {
  typename Acc<TV>::type acc[B];
  prolong_value<B>(P, nn, nxn, nyn, ncx, ncy, xc, xi, n, acc);
#pragma unroll
  for (int rr = 0; rr < B; ++rr) x[n * B + rr] = (TV)acc[rr];
}

// x = M b for the dense coarsest inverse, row rw
template <typename TM, typename TV>
__device__ __forceinline__ void row_dense_apply(const TM* __restrict__ M, int nd, const TV* __restrict__ b,
                                                TV* __restrict__ x, int rw) {
  using TA = typename Acc<TV>::type;
  TA s = TA(0);
  for (int c = 0; c < nd; ++c) s += (TA)M[(size_t)rw * nd + c] * (TA)b[c];
  x[rw] = (TV)s;
}

// ---- one thread per node ----------------------------------------------------
template <int B, typename TM, typename TV, int ST = 0>
__global__ void __launch_bounds__(kBlock)
k_sten_resid(const TM* __restrict__ A, size_t nn, int nxn, int nyn, const TV* __restrict__ x, const TV* b, TV* r) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n < nn) node_sten_resid<B, TM, TV, ST>(A, nn, nxn, nyn, x, b, r, n);
}

// y = A x (FP64 finest level), partial sums of x.y per workgroup (for CG).
// Each wave covers 64 columns of a strip of TR node rows and walks up it: the
// stored blocks of the row below (north, north-east, north-west planes) and x
// of the rows below/at/above stay in registers from the previous step, and the
// left and right neighbours' values come from the adjacent lanes, so every
// stored block and x value is read from memory once per strip (lanes at a
// wave's edge load their outside neighbour's values).  A workgroup is four
// waves: WX side by side along x times 4/WX strips along y.
struct Blk4 {
  double a, b, c, d;  // block entries (0,0), (0,1), (1,0), (1,1)
};

__device__ __forceinline__ Blk4 walk_block(const double* __restrict__ A, size_t nn, int p, int nxn, int nyn, int i,
                                           int j) {
  if (i < 0 || i >= nxn || j < 0 || j >= nyn) return Blk4{0.0, 0.0, 0.0, 0.0};
  const double2* q = reinterpret_cast<const double2*>(A + aidx(2, nn, p, (size_t)j * nxn + i, 0, 0));
  const double2 u = q[0], v = q[1];
  return Blk4{u.x, u.y, v.x, v.y};
}

__device__ __forceinline__ double2 walk_x(const double* __restrict__ x, int nxn, int nyn, int i, int j) {
  if (i < 0 || i >= nxn || j < 0 || j >= nyn) return make_double2(0.0, 0.0);
  return reinterpret_cast<const double2*>(x)[(size_t)j * nxn + i];
}

__device__ __forceinline__ double2 lane_d2(double2 v, int src) {
  return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__device__ __forceinline__ Blk4 lane_blk(const Blk4& b, int src) {
  return Blk4{__shfl(b.a, src, 64), __shfl(b.b, src, 64), __shfl(b.c, src, 64), __shfl(b.d, src, 64)};
}

template <int TR, int WX>
__global__ void __launch_bounds__(kBlock)
k_apply_fine(const double* __restrict__ A, size_t nn, int nxn, int nyn, const double* __restrict__ x,
             double* __restrict__ y, double* __restrict__ partials) {
  constexpr int kWalkRows = TR;
  constexpr int WY = kBlock / 64 / WX;   // waves along y
  __shared__ double lds[16];
  const int lane = threadIdx.x & 63, wv = (int)(threadIdx.x >> 6);
  const int i = (blockIdx.x * WX + wv % WX) * 64 + lane;
  const int j0 = (blockIdx.y * WY + wv / WX) * kWalkRows;
  const bool in = i < nxn;
  const int ic = in ? i : -1;  // -1: every load of an idle lane returns zeros
  const int lm = (lane + 63) & 63, lp = (lane + 1) & 63;
  Blk4 cN = walk_block(A, nn, 2, nxn, nyn, ic, j0 - 1);
  Blk4 cNE = walk_block(A, nn, 3, nxn, nyn, ic, j0 - 1);
  Blk4 cNW = walk_block(A, nn, 4, nxn, nyn, ic, j0 - 1);
  double2 xs = walk_x(x, nxn, nyn, ic, j0 - 1);
  double2 xc = walk_x(x, nxn, nyn, ic, j0);
  double acc[1] = {0.0};
#pragma unroll
  for (int t = 0; t < kWalkRows; ++t) {
    const int j = j0 + t;   // uniform across the wave
    if (j >= nyn) break;
    const Blk4 P0 = walk_block(A, nn, 0, nxn, nyn, ic, j);
    const Blk4 PE = walk_block(A, nn, 1, nxn, nyn, ic, j);
    const Blk4 PN = walk_block(A, nn, 2, nxn, nyn, ic, j);
    const Blk4 PNE = walk_block(A, nn, 3, nxn, nyn, ic, j);
    const Blk4 PNW = walk_block(A, nn, 4, nxn, nyn, ic, j);
    const double2 xn = walk_x(x, nxn, nyn, ic, j + 1);
    double2 xcL = lane_d2(xc, lm), xcR = lane_d2(xc, lp);
    double2 xnL = lane_d2(xn, lm), xnR = lane_d2(xn, lp);
    double2 xsL = lane_d2(xs, lm), xsR = lane_d2(xs, lp);
    Blk4 PEL = lane_blk(PE, lm), cNEL = lane_blk(cNE, lm), cNWR = lane_blk(cNW, lp);
    if (lane == 0) {
      xcL = walk_x(x, nxn, nyn, i - 1, j);
      xnL = walk_x(x, nxn, nyn, i - 1, j + 1);
      xsL = walk_x(x, nxn, nyn, i - 1, j - 1);
      PEL = walk_block(A, nn, 1, nxn, nyn, i - 1, j);
      cNEL = walk_block(A, nn, 3, nxn, nyn, i - 1, j - 1);
    }
    if (lane == 63) {
      xcR = walk_x(x, nxn, nyn, i + 1, j);
      xnR = walk_x(x, nxn, nyn, i + 1, j + 1);
      xsR = walk_x(x, nxn, nyn, i + 1, j - 1);
      cNWR = walk_block(A, nn, 4, nxn, nyn, i + 1, j - 1);
    }
    if (i == 0) xcL = xnL = xsL = make_double2(0.0, 0.0);
    if (i + 1 >= nxn) xcR = xnR = xsR = make_double2(0.0, 0.0);
    if (in) {
      double y0 = 0.0, y1 = 0.0;
      auto fwd = [&](const Blk4& b, double2 v) {
        y0 += b.a * v.x + b.b * v.y;
        y1 += b.c * v.x + b.d * v.y;
      };
      auto bwd = [&](const Blk4& b, double2 v) {   // transpose of a block stored at the neighbour
        y0 += b.a * v.x + b.c * v.y;
        y1 += b.b * v.x + b.d * v.y;
      };
      fwd(P0, xc);
      fwd(PE, xcR);
      fwd(PN, xn);
      fwd(PNE, xnR);
      fwd(PNW, xnL);
      bwd(PEL, xcL);
      bwd(cN, xs);
      bwd(cNEL, xsL);
      bwd(cNWR, xsR);
      reinterpret_cast<double2*>(y)[(size_t)j * nxn + i] = make_double2(y0, y1);
      acc[0] += y0 * xc.x + y1 * xc.y;
    }
    cN = PN;
    cNE = PNE;
    cNW = PNW;
    xs = xc;
    xc = xn;
  }
  if (partials) {
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = acc[0];
  }
}

template <int B, typename TM, typename TV>
__global__ void __launch_bounds__(kBlock)
k_cheb_first(const TM* __restrict__ A, size_t nn, const TV* __restrict__ src, TV* __restrict__ r,
             TV* __restrict__ d, TV* __restrict__ x, typename Acc<TV>::type inv_theta, int add) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n < nn) node_cheb_first<B>(A, nn, src, r, d, x, inv_theta, add, n);
}

template <int B, typename TM, typename TV, int ST = 0>
__global__ void __launch_bounds__(kBlock)
k_resid_first(const TM* __restrict__ A, size_t nn, int nxn, int nyn, const TV* __restrict__ x,
              const TV* __restrict__ b, TV* __restrict__ r, TV* __restrict__ d,
              typename Acc<TV>::type inv_theta) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n < nn) node_resid_first<B, TM, TV, ST>(A, nn, nxn, nyn, x, b, r, d, inv_theta, n);
}

template <int B, typename TM, typename TV, int ST = 0>
__global__ void __launch_bounds__(kBlock)
k_cheb_step(const TM* __restrict__ A, size_t nn, int nxn, int nyn, const TV* __restrict__ dp,
            const TV* rin, TV* rout, TV* __restrict__ dn, const TV* xin, TV* xout, typename Acc<TV>::type cdd,
            typename Acc<TV>::type cdr, int xmode) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n < nn) node_cheb_step<B, TM, TV, ST>(A, nn, nxn, nyn, dp, rin, rout, dn, xin, xout, cdd, cdr, xmode, n);
}

template <int B, typename TP, typename TV>
__global__ void __launch_bounds__(kBlock)
k_restrict(const TP* __restrict__ P, size_t nn, int nxn, int nyn, int ncx, int ncy,
           const TV* __restrict__ r, TV* __restrict__ bc) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t I = gid / kRestrictLanes;
  if (I >= (size_t)ncx * ncy) return;  // whole lane groups leave together
  group_restrict<B>(P, nn, nxn, nyn, ncx, ncy, r, bc, I, (int)(gid % kRestrictLanes));
}

template <int B, typename TP, typename TV>
__global__ void __launch_bounds__(kBlock)
k_prolong_add(const TP* __restrict__ P, size_t nn, int nxn, int nyn, int ncx, int ncy,
              const TV* __restrict__ xc, const TV* xi, TV* x) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n < nn) node_prolong_add<B>(P, nn, nxn, nyn, ncx, ncy, xc, xi, x, n);
}

// ---------------------------------------------------------------------------
// two smoother sweeps per pass on the finest level
// ---------------------------------------------------------------------------
// A pass covers a tile of kPairTX x kPairTY nodes.  The first sweep is evaluated
// on the tile and a one-node ring around it (its results for the ring are what
// the second sweep's stencil needs), kept in LDS; the second sweep then runs on
// the tile and writes the outputs.  Each node's arithmetic is exactly that of the
// single-sweep kernels (same per-node expressions, same storage type of every
// intermediate), so the results are bitwise those of two launches, while the
// intermediate direction, residual and iterate never travel through HBM.
//   PAIR_STEP_STEP  : Chebyshev steps k and k+1.  vin = d_{k-1}, rin = residual
//                     before step k, xin = iterate (not read for xmode1 = 2).
//                     Out: residual, direction and iterate after step k+1.
//   PAIR_STEP_RESID : Chebyshev step k, then the residual r - A d_k of
//                     pre-smoothing.  Out: that residual and the iterate.
//   PAIR_RFIRST_STEP: residual r = b - A x with the first correction
//                     d0 = D^{-1} r / theta (vin = x, rin = b), then step 1
//                     (xmode 1).  Out: residual, direction, iterate; xout must
//                     not alias xin (neighbouring tiles still read x).
// rin and rout, and vin and dout, must not alias (ring nodes of one tile are
// interior nodes of another).
enum { PAIR_STEP_STEP = 0, PAIR_STEP_RESID = 1, PAIR_RFIRST_STEP = 2 };
// On the tiled coarse-level pairs two more passes come first, formed on the tile and
// two rings in LDS: PAIR_FIRST_STEP starts a pre-smoothing from x = 0 (the first
// step d0 = D^-1 b / theta, then the sweeps of PAIR_STEP_STEP with xmode 2), and
// PAIR_PROLONG_RFIRST starts a post-smoothing from the coarse-grid correction
// (x + P xc, then the sweeps of PAIR_RFIRST_STEP).
enum { PAIR_FIRST_STEP = 3, PAIR_PROLONG_RFIRST = 4 };
struct PairExtra {
  const void* P;      // prolongator (PAIR_PROLONG_RFIRST; stored in the vector type on coarse levels)
  const void* xc;     // coarse correction (TV)
  int ncx, ncy;
  double c0;          // 1/theta (PAIR_FIRST_STEP)
};
constexpr int kPairTX = 64, kPairTY = 16, kPairThreads = 256;   // defaults; launch_pair picks per type

template <int MODE, int XM, typename TM, typename TV, int TX, int TY, int NT, int B>
__device__ __forceinline__ void cheb_pair_body(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int tiles_x,
                                               int tiles, const TV* __restrict__ vin, const TV* __restrict__ rin,
                                               const TV* xin, TV* __restrict__ rout, TV* __restrict__ dout,
                                               TV* xout, typename Acc<TV>::type c1a, typename Acc<TV>::type c1b,
                                               typename Acc<TV>::type c2a, typename Acc<TV>::type c2b,
                                               const PairExtra& ex) {
  using TA = typename Acc<TV>::type;
  constexpr bool pre0 = MODE == PAIR_FIRST_STEP || MODE == PAIR_PROLONG_RFIRST;   // input formed in LDS
  constexpr bool rfirst = MODE == PAIR_RFIRST_STEP || MODE == PAIR_PROLONG_RFIRST;
  constexpr int xmode1 = MODE == PAIR_FIRST_STEP ? 2 : XM;   // xmode of the first sweep's step (STEP modes)
  constexpr int W2 = TX + 4;                                   // row length of the twice-ringed tile
  __shared__ TV s_d[(TX + 2) * (TY + 2)][B];   // first sweep's direction on the ringed tile
  __shared__ TV s_r[(TX + 2) * (TY + 2)][B];   // first sweep's residual
  __shared__ TV s_v[pre0 ? (TX + 4) * (TY + 4) : 1][B];   // the first sweep's input on the twice-ringed tile
  const int tb = (int)xcd_block();
  if (tb >= tiles) return;                   // whole workgroup
  const int i0 = (tb % tiles_x) * TX, j0 = (tb / tiles_x) * TY;
  if constexpr (pre0) {
#pragma unroll 1
    for (int k = threadIdx.x; k < (TX + 4) * (TY + 4); k += NT) {
      const int i = i0 - 2 + k % W2, j = j0 - 2 + k / W2;
      if (i < 0 || j < 0 || i >= nxn || j >= nyn) continue;
      const size_t n = (size_t)j * nxn + i;
      TA v[B];
      if constexpr (MODE == PAIR_FIRST_STEP) {   // d0 = D^-1 b / theta (node_cheb_first)
        TA raw[B * B], D[B][B], Di[B][B], sv[B];
        load_raw<B>(A + aidx(B, nn, 0, n, 0, 0), raw);
#pragma unroll
        for (int rr = 0; rr < B; ++rr)
#pragma unroll
          for (int c = 0; c < B; ++c) D[rr][c] = raw[rr * B + c];
        invert_block<B>(D, Di);
        load_node<B>(rin, n, sv);
#pragma unroll
        for (int q = 0; q < B; ++q) {
          TA t = TA(0);
#pragma unroll
          for (int c = 0; c < B; ++c) t += Di[q][c] * sv[c];
          v[q] = t * (TA)ex.c0;
        }
      } else {                                   // x + P xc (node_prolong_add)
        prolong_value<B>((const TV*)ex.P, nn, nxn, nyn, ex.ncx, ex.ncy, (const TV*)ex.xc, xin, n, v);
      }
#pragma unroll
      for (int q = 0; q < B; ++q) s_v[k][q] = (TV)v[q];
    }
    __syncthreads();
  }
  // the first sweep's input and the node's own value of it
  auto vget = [&](size_t m, int ii, int jj, TA (&xm)[B]) {
    if constexpr (pre0) {
      const int l = (jj - j0 + 2) * W2 + (ii - i0 + 2);
#pragma unroll
      for (int q = 0; q < B; ++q) xm[q] = (TA)s_v[l][q];
    } else {
      load_node<B>(vin, m, xm);
    }
  };
  // first sweep on the tile and its ring (loops kept rolled: the unrolled body
  // would not fit the instruction cache)
#pragma unroll 1
  for (int k = threadIdx.x; k < (TX + 2) * (TY + 2); k += NT) {
    const int i = i0 - 1 + k % (TX + 2), j = j0 - 1 + k / (TX + 2);
    if (i < 0 || j < 0 || i >= nxn || j >= nyn) continue;
    const size_t n = (size_t)j * nxn + i;
    TA y[B], D[B][B], Di[B][B], rn[B], dk[B];
    stencil_row_f<B>(A, nn, nxn, nyn, i, j, vget, y, D);
    invert_block<B>(D, Di);
    load_node<B>(rin, n, rn);
#pragma unroll
    for (int q = 0; q < B; ++q) rn[q] -= y[q];
    if constexpr (rfirst) {
#pragma unroll
      for (int q = 0; q < B; ++q) {
        TA t = TA(0);
#pragma unroll
        for (int c = 0; c < B; ++c) t += Di[q][c] * rn[c];
        dk[q] = t * c1a;
      }
    } else {
      TA dpn[B];
      vget(n, i, j, dpn);
#pragma unroll
      for (int q = 0; q < B; ++q) {
        TA t = TA(0);
#pragma unroll
        for (int c = 0; c < B; ++c) t += Di[q][c] * rn[c];
        dk[q] = fma(c1a, dpn[q], c1b * t);
      }
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      s_d[k][q] = (TV)dk[q];
      s_r[k][q] = (TV)rn[q];
    }
  }
  __syncthreads();
  // second sweep on the tile
#pragma unroll 1
  for (int k = threadIdx.x; k < TX * TY; k += NT) {
    const int li = k % TX, lj = k / TX;
    const int i = i0 + li, j = j0 + lj;
    if (i >= nxn || j >= nyn) continue;
    const size_t n = (size_t)j * nxn + i;
    const int lk = (lj + 1) * (TX + 2) + li + 1;
    TA d1[B], r1[B], x1[B], y[B], D[B][B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      d1[q] = (TA)s_d[lk][q];
      r1[q] = (TA)s_r[lk][q];
    }
    // iterate after the first sweep (as the single-sweep kernels store it)
    if constexpr (rfirst) {
      if constexpr (pre0) vget(n, i, j, x1);           // the corrected x
      else load_node<B>(xin, n, x1);                   // the first sweep leaves x unchanged
    } else {
      TA dpn[B];
      vget(n, i, j, dpn);
      if constexpr (xmode1 == 2) {
#pragma unroll
        for (int q = 0; q < B; ++q) x1[q] = dpn[q];
      } else {
        load_node<B>(xin, n, x1);
        if constexpr (xmode1 == 1) {
#pragma unroll
          for (int q = 0; q < B; ++q) x1[q] += dpn[q];
        }
      }
#pragma unroll
      for (int q = 0; q < B; ++q) x1[q] = (TA)(TV)(x1[q] + d1[q]);
    }
    stencil_row_f<B>(A, nn, nxn, nyn, i, j,
                     [&](size_t, int ii, int jj, TA (&xm)[B]) {
                       const int l = (jj - j0 + 1) * (TX + 2) + (ii - i0 + 1);
#pragma unroll
                       for (int q = 0; q < B; ++q) xm[q] = (TA)s_d[l][q];
                     },
                     y, D);
    TA r2[B];
#pragma unroll
    for (int q = 0; q < B; ++q) r2[q] = r1[q] - y[q];
    store_node<B>(rout, n, r2);
    if constexpr (MODE == PAIR_STEP_RESID) {
      store_node<B>(xout, n, x1);
    } else {
      TA Di[B][B], d2[B], x2[B];
      invert_block<B>(D, Di);
      if constexpr (rfirst) {
#pragma unroll
        for (int q = 0; q < B; ++q) x1[q] += d1[q];     // step 1 in xmode 1: (x + d0) + d1
      }
#pragma unroll
      for (int q = 0; q < B; ++q) {
        TA t = TA(0);
#pragma unroll
        for (int c = 0; c < B; ++c) t += Di[q][c] * r2[c];
        d2[q] = fma(c2a, d1[q], c2b * t);
        x2[q] = x1[q] + d2[q];
      }
      store_node<B>(dout, n, d2);
      store_node<B>(xout, n, x2);
    }
  }
}

template <int MODE, int XM, typename TM, typename TV, int TX = kPairTX, int TY = kPairTY, int NT = kPairThreads,
          int WMAX = 8>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, WMAX)))
k_cheb_pair(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int tiles_x, int tiles,
            const TV* __restrict__ vin, const TV* __restrict__ rin, const TV* xin, TV* __restrict__ rout,
            TV* __restrict__ dout, TV* xout, typename Acc<TV>::type c1a, typename Acc<TV>::type c1b,
            typename Acc<TV>::type c2a, typename Acc<TV>::type c2b) {
  cheb_pair_body<MODE, XM, TM, TV, TX, TY, NT, 2>(A, nn, nxn, nyn, tiles_x, tiles, vin, rin, xin, rout, dout, xout,
                                                  c1a, c1b, c2a, c2b, PairExtra{});
}

// The same paired sweeps on a small structured coarse level (3 x 3 blocks, any
// storage): 14 x 14 tiles, the ringed tile one node per thread of 256.  On levels of
// a few ten thousand nodes or fewer each launch is mostly latency, and one launch
// for two sweeps replaces two.
constexpr int kPair3Tile = 14;
template <int MODE, int XM, typename TM, typename TV>
__global__ void __launch_bounds__(256)
k_cheb_pair3(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int tiles_x, int tiles,
             const TV* __restrict__ vin, const TV* __restrict__ rin, const TV* xin, TV* __restrict__ rout,
             TV* __restrict__ dout, TV* xout, typename Acc<TV>::type c1a, typename Acc<TV>::type c1b,
             typename Acc<TV>::type c2a, typename Acc<TV>::type c2b, PairExtra ex) {
  cheb_pair_body<MODE, XM, TM, TV, kPair3Tile, kPair3Tile, 256, 3>(A, nn, nxn, nyn, tiles_x, tiles, vin, rin, xin,
                                                                   rout, dout, xout, c1a, c1b, c2a, c2b, ex);
}

// The same two sweeps by column walks, for operators stored in the vector type
// (FP64 and FP32 finest levels): a wave covers 64 columns, the 62 inner ones its
// outputs, and walks up a strip of TR rows, evaluating the first sweep one row
// ahead of the second (on the strip and one row on each side).  The stored blocks
// of the last three rows, the first-sweep results of the last three rows and the
// input vector's last three rows stay in registers; left and right neighbours come
// from the adjacent lanes (the outer lanes load their outside neighbours).  No LDS,
// no barrier, every value read once per strip.  Per node the operations are those
// of k_cheb_pair in the same order, so the outputs are bitwise the same.
template <typename TA>
struct WBlk {
  TA a, b, c, d;   // block entries (0,0), (0,1), (1,0), (1,1)
};
template <typename TA>
struct WVec {
  TA x, y;
};
template <typename TA>
__device__ __forceinline__ WBlk<TA> wshb(const WBlk<TA>& v, int src) {
  return WBlk<TA>{__shfl(v.a, src, 64), __shfl(v.b, src, 64), __shfl(v.c, src, 64), __shfl(v.d, src, 64)};
}
template <typename TA>
__device__ __forceinline__ WVec<TA> wshv(WVec<TA> v, int src) {
  return WVec<TA>{__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}
template <typename TA>
__device__ __forceinline__ WBlk<TA> wblk(const TA* __restrict__ A, size_t nn, int p, int nxn, int nyn, int i, int j) {
  if (i < 0 || i >= nxn || j < 0 || j >= nyn) return WBlk<TA>{TA(0), TA(0), TA(0), TA(0)};
  const TA* q = A + aidx(2, nn, p, (size_t)j * nxn + i, 0, 0);
  if constexpr (std::is_same<TA, double>::value) {
    const double2 u = reinterpret_cast<const double2*>(q)[0], w = reinterpret_cast<const double2*>(q)[1];
    return WBlk<TA>{u.x, u.y, w.x, w.y};
  } else {
    const float4 v = *reinterpret_cast<const float4*>(q);
    return WBlk<TA>{v.x, v.y, v.z, v.w};
  }
}
template <typename TA>
__device__ __forceinline__ WVec<TA> wvec(const TA* __restrict__ p, int nxn, int nyn, int i, int j) {
  if (i < 0 || i >= nxn || j < 0 || j >= nyn) return WVec<TA>{TA(0), TA(0)};
  const size_t n = (size_t)j * nxn + i;
  return WVec<TA>{p[2 * n], p[2 * n + 1]};
}
// y += b x, or b^T x for a block stored at the neighbour (the order of stencil_row_f)
template <typename TA>
__device__ __forceinline__ void wfwd(TA (&y)[2], const WBlk<TA>& b, WVec<TA> x) {
  y[0] += b.a * x.x; y[0] += b.b * x.y;
  y[1] += b.c * x.x; y[1] += b.d * x.y;
}
template <typename TA>
__device__ __forceinline__ void wbwd(TA (&y)[2], const WBlk<TA>& b, WVec<TA> x) {
  y[0] += b.a * x.x; y[0] += b.c * x.y;
  y[1] += b.b * x.x; y[1] += b.d * x.y;
}

template <int MODE, int XM, typename TV, int TR>
__global__ void __launch_bounds__(256)
k_cheb_walk(const TV* __restrict__ A, size_t nn, int nxn, int nyn, const TV* __restrict__ vin,
            const TV* __restrict__ rin, const TV* xin, TV* __restrict__ rout, TV* __restrict__ dout, TV* xout,
            TV c1a, TV c1b, TV c2a, TV c2b) {
  using Bk = WBlk<TV>;
  using Vc = WVec<TV>;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 62 - 1 + lane;
  const int j0 = (blockIdx.y * 4 + (int)(threadIdx.x >> 6)) * TR;
  const bool in = i >= 0 && i < nxn;
  const int ic = in ? i : -(1 << 29);   // idle lanes load nothing
  const int lm = (lane + 63) & 63, lp = (lane + 1) & 63;
  const Bk z{TV(0), TV(0), TV(0), TV(0)};
  // rows r-1 (q*) and r-2 (s*: north, north-east, north-west) of the stored blocks
  Bk q0 = wblk(A, nn, 0, nxn, nyn, ic, j0 - 2), qE = wblk(A, nn, 1, nxn, nyn, ic, j0 - 2),
     qN = wblk(A, nn, 2, nxn, nyn, ic, j0 - 2), qNE = wblk(A, nn, 3, nxn, nyn, ic, j0 - 2),
     qNW = wblk(A, nn, 4, nxn, nyn, ic, j0 - 2);
  Bk sN = z, sNE = z, sNW = z;
  Vc vS = wvec(vin, nxn, nyn, ic, j0 - 2), vC = wvec(vin, nxn, nyn, ic, j0 - 1);
  Vc d1pp{TV(0), TV(0)}, d1p{TV(0), TV(0)}, r1p{TV(0), TV(0)};
  for (int r = j0 - 1; r <= j0 + TR; ++r) {
    if (r > nyn) break;   // uniform across the wave
    const Bk P0 = wblk(A, nn, 0, nxn, nyn, ic, r), PE = wblk(A, nn, 1, nxn, nyn, ic, r),
             PN = wblk(A, nn, 2, nxn, nyn, ic, r), PNE = wblk(A, nn, 3, nxn, nyn, ic, r),
             PNW = wblk(A, nn, 4, nxn, nyn, ic, r);
    const Vc vN = wvec(vin, nxn, nyn, ic, r + 1);
    const Vc rC = wvec(rin, nxn, nyn, ic, r);
    // first sweep at row r
    Vc vCL = wshv(vC, lm), vCR = wshv(vC, lp), vNL = wshv(vN, lm), vNR = wshv(vN, lp), vSL = wshv(vS, lm),
       vSR = wshv(vS, lp);
    Bk PEL = wshb(PE, lm), qNEL = wshb(qNE, lm), qNWR = wshb(qNW, lp);
    if (lane == 0) {
      vCL = wvec(vin, nxn, nyn, i - 1, r);
      vNL = wvec(vin, nxn, nyn, i - 1, r + 1);
      vSL = wvec(vin, nxn, nyn, i - 1, r - 1);
      PEL = wblk(A, nn, 1, nxn, nyn, i - 1, r);
      qNEL = wblk(A, nn, 3, nxn, nyn, i - 1, r - 1);
    }
    if (lane == 63) {
      vCR = wvec(vin, nxn, nyn, i + 1, r);
      vNR = wvec(vin, nxn, nyn, i + 1, r + 1);
      vSR = wvec(vin, nxn, nyn, i + 1, r - 1);
      qNWR = wblk(A, nn, 4, nxn, nyn, i + 1, r - 1);
    }
    Vc d1c{TV(0), TV(0)}, r1c{TV(0), TV(0)};
    if (in && r >= 0 && r < nyn) {
      TV y[2] = {TV(0), TV(0)};
      const bool hE = i + 1 < nxn, hW = i > 0, hN = r + 1 < nyn, hS = r > 0;
      wfwd(y, P0, vC);
      if (hE) wfwd(y, PE, vCR);
      if (hN) wfwd(y, PN, vN);
      if (hE && hN) wfwd(y, PNE, vNR);
      if (hW && hN) wfwd(y, PNW, vNL);
      if (hW) wbwd(y, PEL, vCL);
      if (hS) wbwd(y, qN, vS);
      if (hW && hS) wbwd(y, qNEL, vSL);
      if (hE && hS) wbwd(y, qNWR, vSR);
      TV D[2][2] = {{P0.a, P0.b}, {P0.c, P0.d}}, Di[2][2];
      invert_block<2>(D, Di);
      const TV rn[2] = {rC.x - y[0], rC.y - y[1]};
      TV t[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        t[q] = TV(0);
        t[q] += Di[q][0] * rn[0];
        t[q] += Di[q][1] * rn[1];
      }
      if constexpr (MODE == PAIR_RFIRST_STEP) d1c = Vc{t[0] * c1a, t[1] * c1a};
      else d1c = Vc{fma(c1a, vC.x, c1b * t[0]), fma(c1a, vC.y, c1b * t[1])};
      r1c = Vc{rn[0], rn[1]};
    }
    // second sweep at row j = r - 1, inner lanes
    const int j = r - 1;
    const Vc dL = wshv(d1p, lm), dR = wshv(d1p, lp), dNL = wshv(d1c, lm), dNR = wshv(d1c, lp), dSL = wshv(d1pp, lm),
             dSR = wshv(d1pp, lp);
    const Bk qEL = wshb(qE, lm), sNEL = wshb(sNE, lm), sNWR = wshb(sNW, lp);
    if (j >= j0 && j < nyn && in && lane >= 1 && lane <= 62) {
      const size_t n = (size_t)j * nxn + i;
      TV x1[2];
      if constexpr (MODE == PAIR_RFIRST_STEP) {
        x1[0] = xin[2 * n]; x1[1] = xin[2 * n + 1];      // the first sweep leaves x unchanged
      } else {
        const Vc dpn = vS;                                 // vin at row j
        if constexpr (XM == 2) {
          x1[0] = dpn.x; x1[1] = dpn.y;
        } else {
          x1[0] = xin[2 * n]; x1[1] = xin[2 * n + 1];
          if constexpr (XM == 1) {
            x1[0] += dpn.x; x1[1] += dpn.y;
          }
        }
        x1[0] = x1[0] + d1p.x; x1[1] = x1[1] + d1p.y;
      }
      TV y[2] = {TV(0), TV(0)};
      const bool hE = i + 1 < nxn, hW = i > 0, hN = j + 1 < nyn, hS = j > 0;
      wfwd(y, q0, d1p);
      if (hE) wfwd(y, qE, dR);
      if (hN) wfwd(y, qN, d1c);
      if (hE && hN) wfwd(y, qNE, dNR);
      if (hW && hN) wfwd(y, qNW, dNL);
      if (hW) wbwd(y, qEL, dL);
      if (hS) wbwd(y, sN, d1pp);
      if (hW && hS) wbwd(y, sNEL, dSL);
      if (hE && hS) wbwd(y, sNWR, dSR);
      const TV r2[2] = {r1p.x - y[0], r1p.y - y[1]};
      rout[2 * n] = r2[0];
      rout[2 * n + 1] = r2[1];
      if constexpr (MODE == PAIR_STEP_RESID) {
        xout[2 * n] = x1[0];
        xout[2 * n + 1] = x1[1];
      } else {
        TV D[2][2] = {{q0.a, q0.b}, {q0.c, q0.d}}, Di[2][2];
        invert_block<2>(D, Di);
        if constexpr (MODE == PAIR_RFIRST_STEP) {
          x1[0] += d1p.x;                                 // step 1 in xmode 1: (x + d0) + d1
          x1[1] += d1p.y;
        }
        const TV d1v[2] = {d1p.x, d1p.y};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          TV t = TV(0);
          t += Di[q][0] * r2[0];
          t += Di[q][1] * r2[1];
          const TV d2 = fma(c2a, d1v[q], c2b * t);
          dout[2 * n + q] = d2;
          xout[2 * n + q] = x1[q] + d2;
        }
      }
    }
    sN = qN; sNE = qNE; sNW = qNW;
    q0 = P0; qE = PE; qN = PN; qNE = PNE; qNW = PNW;
    vS = vC; vC = vN;
    d1pp = d1p; d1p = d1c; r1p = r1c;
  }
}

// All four sweeps of a degree-4 Chebyshev smoothing in one column walk (operators
// stored in the vector type).  A wave covers 64 columns and walks up a strip of TR
// rows; at the step to row R it loads row R and evaluates stage k (k = 1..4) at row
// R - k, so stage k finds the previous stage's result at rows R - k - 1, R - k and
// R - k + 1 in registers (the last two rows kept, the newest just computed).  Each
// stage narrows the valid lanes by one per side: lanes 4..59 of a wave are its
// outputs (56 columns per wave) and the strip is evaluated 4 rows beyond its ends by
// the earlier stages.  The blocks of the last five rows, their block inverses and each
// stage's last two rows are register-resident (no LDS, no barrier).  Every node's
// arithmetic is that of the paired kernels in the same order, so the results are
// bitwise the same as two paired or four single sweeps.  The next row's loads are
// issued before the current row is evaluated.
//   W4_PRE:  x = 0 on entry.  d0 = D^-1 b / theta, three Chebyshev steps, then the
//            residual: writes x and r = b - A x.
//   W4_POST: four Chebyshev steps from x (the first from r = b - A x): writes x.
//            x is read around the strip, so the output goes to another buffer.
// c0 = 1/theta; (a_k, b_k) are the (cdd, cdr) of steps 1..3.
enum { W4_PRE = 0, W4_POST = 1 };
template <typename T>
struct WRow {
  WBlk<T> p0, e, n, ne, nw;
};
template <typename T>
__device__ __forceinline__ WRow<T> wrow(const T* __restrict__ A, size_t nn, int nxn, int nyn, int i, int j) {
  return WRow<T>{wblk(A, nn, 0, nxn, nyn, i, j), wblk(A, nn, 1, nxn, nyn, i, j), wblk(A, nn, 2, nxn, nyn, i, j),
                 wblk(A, nn, 3, nxn, nyn, i, j), wblk(A, nn, 4, nxn, nyn, i, j)};
}
template <typename T>
__device__ __forceinline__ WBlk<T> winv(const WBlk<T>& p) {
  T D[2][2] = {{p.a, p.b}, {p.c, p.d}}, Di[2][2];
  invert_block<2>(D, Di);
  return WBlk<T>{Di[0][0], Di[0][1], Di[1][0], Di[1][1]};
}
// y = (A u) at one node in the order of stencil_row_f: own row o, south row s (its
// n, ne, nw blocks), u at rows j - 1, j, j + 1.  Every lane takes part in the shuffles.
template <typename T>
__device__ __forceinline__ void wapply(T (&y)[2], const WRow<T>& o, const WRow<T>& s, WVec<T> uS, WVec<T> uC,
                                       WVec<T> uN, int lm, int lp, bool hE, bool hW, bool hN, bool hS) {
  const WVec<T> uCL = wshv(uC, lm), uCR = wshv(uC, lp), uNL = wshv(uN, lm), uNR = wshv(uN, lp), uSL = wshv(uS, lm),
                uSR = wshv(uS, lp);
  const WBlk<T> eL = wshb(o.e, lm), sneL = wshb(s.ne, lm), snwR = wshb(s.nw, lp);
  y[0] = T(0);
  y[1] = T(0);
  wfwd(y, o.p0, uC);
  if (hE) wfwd(y, o.e, uCR);
  if (hN) wfwd(y, o.n, uN);
  if (hE && hN) wfwd(y, o.ne, uNR);
  if (hW && hN) wfwd(y, o.nw, uNL);
  if (hW) wbwd(y, eL, uCL);
  if (hS) wbwd(y, s.n, uS);
  if (hW && hS) wbwd(y, sneL, uSL);
  if (hE && hS) wbwd(y, snwR, uSR);
}
template <typename T>
__device__ __forceinline__ WVec<T> wsolve(const WBlk<T>& Di, const T (&r)[2]) {
  T t0 = T(0), t1 = T(0);
  t0 += Di.a * r[0];
  t0 += Di.b * r[1];
  t1 += Di.c * r[0];
  t1 += Di.d * r[1];
  return WVec<T>{t0, t1};
}


// One strip of the four-sweep walk.  UP walks from the strip's bottom (sweep k at
// row R - k, the south neighbour of a sweep's row is older than its row); the
// mirror image (UP = false) walks from the top (sweep k at row R + k: the south
// neighbour is the row the previous sweep has just produced, and the operator
// rows R .. R + 4 suffice, one fewer than upward).  Every node gets the same
// arithmetic in the same order either way, so both give the outputs bitwise.
template <int KIND, typename T, bool UP>
__device__ __forceinline__ void walk4_strip(int TR, int i, int j0, int lane, const T* __restrict__ A, size_t nn,
                                            int nxn, int nyn, const T* __restrict__ b, const T* __restrict__ xin,
                                            T* __restrict__ rout, T* __restrict__ xout, T c0, T a1, T b1, T a2, T b2,
                                            T a3, T b3) {
  using Bk = WBlk<T>;
  using Vc = WVec<T>;
  using Rw = WRow<T>;
  constexpr int sg = UP ? -1 : 1;   // sweep k works on row R + sg k
  const bool in = i >= 0 && i < nxn;
  const int ic = in ? i : -(1 << 29);   // idle lanes load nothing
  const int lm = (lane + 63) & 63, lp = (lane + 1) & 63;
  const bool hE = i + 1 < nxn, hW = i > 0;
  const Bk z{T(0), T(0), T(0), T(0)};
  const Vc zv{T(0), T(0)};
  const Rw zr{z, z, z, z, z};
  Rw W1 = zr, W2 = zr, W3 = zr, W4 = zr, W5 = zr;   // blocks of rows R + sg, ..., R + 5 sg (W5 upward only)
  Bk D1 = z, D2 = z, D3 = z, D4 = z;                  // block inverses of rows R + sg .. R + 4 sg
  // sweep k's input vector at its row's far neighbour (uO: the row below upward,
  // above downward) and at its row (uC)
  Vc uO1 = zv, uC1 = zv, uO2 = zv, uC2 = zv, uO3 = zv, uC3 = zv, uO4 = zv, uC4 = zv;
  Vc rc1 = zv, rc2 = zv, rc3 = zv, rc4 = zv;          // residual entering sweep k at its row
  Vc xc2 = zv, xc3 = zv, xc4 = zv;                    // iterate entering sweep k at its row
  // sweep k covers rows j0 - 4 + k .. j0 + TR + 3 - k of the grid
  const int Rfirst = UP ? j0 - 4 : min(j0 + TR + 3, nyn - 1);
  const int Rlast = UP ? min(j0 + TR + 3, nyn + 3) : j0 - 4;
  auto active = [&](int j, int k) {
    return j >= 0 && j < nyn && (UP ? j >= j0 - 4 + k : j <= j0 + TR + 3 - k);
  };
  // row R - sg is loaded while row R is evaluated
  Rw Wn = wrow(A, nn, nxn, nyn, ic, Rfirst);
  Vc bn = wvec(b, nxn, nyn, ic, Rfirst), xn = zv;
  if constexpr (KIND == W4_POST) xn = wvec(xin, nxn, nyn, ic, Rfirst);
  // One row step; the shifts at its end rotate the register window.
  auto row = [&] __device__ (const int R) {
    const Rw W0 = Wn;
    const Vc bR = bn, xR = xn;
    Wn = wrow(A, nn, nxn, nyn, ic, R - sg);
    bn = wvec(b, nxn, nyn, ic, R - sg);
    if constexpr (KIND == W4_POST) xn = wvec(xin, nxn, nyn, ic, R - sg);
    const Bk D0 = winv(W0.p0);
    Vc u0;   // sweep 1's input at row R
    if constexpr (KIND == W4_PRE) {
      const T bb[2] = {bR.x, bR.y};
      const Vc t = wsolve(D0, bb);
      u0 = Vc{t.x * c0, t.y * c0};
    } else {
      u0 = xR;
    }
    // y = A u at row j of sweep k: own blocks Wk, the south row's blocks and the
    // input at rows j - 1, j, j + 1 (the new value un is on the near side)
    auto apply = [&](T (&y)[2], int j, const Rw& Wk, const Rw& Wfar, const Rw& Wnear, const Vc& uO, const Vc& uC,
                     const Vc& un) {
      if constexpr (UP)
        wapply(y, Wk, Wfar, uO, uC, un, lm, lp, hE, hW, j + 1 < nyn, j > 0);
      else
        wapply(y, Wk, Wnear, un, uC, uO, lm, lp, hE, hW, j + 1 < nyn, j > 0);
    };
    Vc d1 = zv, r1 = zv, x1 = zv;
    {
      const int j = R + sg;
      if (active(j, 1)) {
        T y[2];
        apply(y, j, W1, W2, W0, uO1, uC1, u0);
        const T r[2] = {rc1.x - y[0], rc1.y - y[1]};
        const Vc t = wsolve(D1, r);
        if constexpr (KIND == W4_PRE) {
          d1 = Vc{fma(a1, uC1.x, b1 * t.x), fma(a1, uC1.y, b1 * t.y)};
          x1 = Vc{uC1.x + d1.x, uC1.y + d1.y};
        } else {
          d1 = Vc{t.x * c0, t.y * c0};
          {
            // the paired kernels add this step to x in their next sweep, to the
            // rounded product: no contraction into a fused multiply-add here
#pragma clang fp contract(off)
            x1 = Vc{uC1.x + d1.x, uC1.y + d1.y};
          }
        }
        r1 = Vc{r[0], r[1]};
      }
    }
    Vc d2 = zv, r2 = zv, x2 = zv;
    {
      const int j = R + 2 * sg;
      if (active(j, 2)) {
        T y[2];
        apply(y, j, W2, W3, W1, uO2, uC2, d1);
        const T r[2] = {rc2.x - y[0], rc2.y - y[1]};
        const Vc t = wsolve(D2, r);
        const T a = KIND == W4_PRE ? a2 : a1, bq = KIND == W4_PRE ? b2 : b1;
        d2 = Vc{fma(a, uC2.x, bq * t.x), fma(a, uC2.y, bq * t.y)};
        x2 = Vc{xc2.x + d2.x, xc2.y + d2.y};
        r2 = Vc{r[0], r[1]};
      }
    }
    Vc d3 = zv, r3 = zv, x3 = zv;
    {
      const int j = R + 3 * sg;
      if (active(j, 3)) {
        T y[2];
        apply(y, j, W3, W4, W2, uO3, uC3, d2);
        const T r[2] = {rc3.x - y[0], rc3.y - y[1]};
        const Vc t = wsolve(D3, r);
        const T a = KIND == W4_PRE ? a3 : a2, bq = KIND == W4_PRE ? b3 : b2;
        d3 = Vc{fma(a, uC3.x, bq * t.x), fma(a, uC3.y, bq * t.y)};
        x3 = Vc{xc3.x + d3.x, xc3.y + d3.y};
        r3 = Vc{r[0], r[1]};
      }
    }
    {
      const int j = R + 4 * sg;   // sweep 4: the outputs, rows j0 .. j0 + TR - 1
      if (j >= j0 && j < j0 + TR && j < nyn) {
        T y[2];
        apply(y, j, W4, W5, W3, uO4, uC4, d3);
        const T r[2] = {rc4.x - y[0], rc4.y - y[1]};
        if (in && lane >= 4 && lane < 60) {
          const size_t n = (size_t)j * nxn + i;
          if constexpr (KIND == W4_PRE) {
            rout[2 * n] = r[0];
            rout[2 * n + 1] = r[1];
            xout[2 * n] = xc4.x;
            xout[2 * n + 1] = xc4.y;
          } else {
            const Vc t = wsolve(D4, r);
            const T d[2] = {fma(a3, uC4.x, b3 * t.x), fma(a3, uC4.y, b3 * t.y)};
            xout[2 * n] = xc4.x + d[0];
            xout[2 * n + 1] = xc4.y + d[1];
          }
        }
      }
    }
    if constexpr (UP) W5 = W4;
    W4 = W3; W3 = W2; W2 = W1; W1 = W0;
    D4 = D3; D3 = D2; D2 = D1; D1 = D0;
    uO4 = uC4; uC4 = d3; uO3 = uC3; uC3 = d2; uO2 = uC2; uC2 = d1; uO1 = uC1; uC1 = u0;
    rc4 = r3; rc3 = r2; rc2 = r1; rc1 = bR;
    xc4 = x3; xc3 = x2; xc2 = x1;
  };
  // Steps issued as many at a time as the window has row slots (seven upward: the
  // prefetched row, the current one and five more; six downward): after inlining,
  // most of the rotation becomes a renaming of registers instead of copies.  R is
  // uniform across the wave.
  int R = Rfirst;
  if constexpr (UP) {
    for (; R + 6 <= Rlast; R += 7) {
      row(R);
      row(R + 1);
      row(R + 2);
      row(R + 3);
      row(R + 4);
      row(R + 5);
      row(R + 6);
    }
    for (; R <= Rlast; ++R) row(R);
  } else {
    for (; R - 5 >= Rlast; R -= 6) {
      row(R);
      row(R - 1);
      row(R - 2);
      row(R - 3);
      row(R - 4);
      row(R - 5);
    }
    for (; R >= Rlast; --R) row(R);
  }
}

// A workgroup takes two vertically adjacent strips; the lower one walks upward and
// the upper one downward, so the eight rows the two strips share come in at about
// the same time, and the upper strip starts where the next workgroup's lower strip
// starts.  With FP64 blocks each strip is two waves (112 columns) wide, so the waves
// side by side also read their eight shared columns at the same time on one CU
// (measured at 2049^2: FP32 131 us with one wave per strip, 135 with two; FP64 314
// us with two, 332 with one).  Workgroups are dealt to the XCDs in contiguous runs
// of a column-major order, so vertical and horizontal neighbours mostly share an L2.
template <typename T>
constexpr int walk4_cols() { return std::is_same<T, double>::value ? 2 : 1; }
constexpr int kWalk4Strips = 2;
template <int KIND, typename T>
__global__ void __launch_bounds__(64 * kWalk4Strips * walk4_cols<T>())
k_cheb_walk4(int TR, int ntx, int nty, const T* __restrict__ A, size_t nn, int nxn, int nyn,
             const T* __restrict__ b, const T* __restrict__ xin, T* __restrict__ rout, T* __restrict__ xout, T c0,
             T a1, T b1, T a2, T b2, T a3, T b3) {
  constexpr int cols = walk4_cols<T>();
  const unsigned t = xcd_block();
  const int tx = (int)(t / nty), ty = (int)(t % nty);
  if (tx >= ntx) return;
  const int lane = threadIdx.x & 63, wave = (int)(threadIdx.x >> 6);
  const int col = wave % cols, strip = wave / cols;
  const int i = (tx * cols + col) * 56 - 4 + lane;
  const int j0 = (ty * kWalk4Strips + strip) * TR;
  if (strip == 0)
    walk4_strip<KIND, T, true>(TR, i, j0, lane, A, nn, nxn, nyn, b, xin, rout, xout, c0, a1, b1, a2, b2, a3, b3);
  else
    walk4_strip<KIND, T, false>(TR, i, j0, lane, A, nn, nxn, nyn, b, xin, rout, xout, c0, a1, b1, a2, b2, a3, b3);
}

// Paired sweeps by column walks on the structured coarse levels (3 x 3 blocks, FP32
// operator and vectors): the scheme of k_cheb_walk with runtime strip height TR and
// register blocks of 9 values.  The two Chebyshev combinations are written as
// explicit fused multiply-adds, fma(c_dd, d, c_dr * t), which is how the single-sweep
// kernels contract them, so the outputs are bitwise those of two single sweeps.
struct W3Blk {
  float v[9];
};
struct W3Vec {
  float v[3];
};
__device__ __forceinline__ W3Blk w3shb(const W3Blk& x, int src) {
  W3Blk o;
#pragma unroll
  for (int k = 0; k < 9; ++k) o.v[k] = __shfl(x.v[k], src, 64);
  return o;
}
__device__ __forceinline__ W3Vec w3shv(const W3Vec& x, int src) {
  W3Vec o;
#pragma unroll
  for (int k = 0; k < 3; ++k) o.v[k] = __shfl(x.v[k], src, 64);
  return o;
}
__device__ __forceinline__ W3Blk w3blk(const float* __restrict__ A, size_t nn, int p, int nxn, int nyn, int i,
                                       int j) {
  W3Blk o;
  if (i < 0 || i >= nxn || j < 0 || j >= nyn) {
#pragma unroll
    for (int k = 0; k < 9; ++k) o.v[k] = 0.0f;
    return o;
  }
  const float* q = A + aidx(3, nn, p, (size_t)j * nxn + i, 0, 0);
#pragma unroll
  for (int k = 0; k < 9; ++k) o.v[k] = q[k];
  return o;
}
__device__ __forceinline__ W3Vec w3vec(const float* __restrict__ p, int nxn, int nyn, int i, int j) {
  W3Vec o;
  if (i < 0 || i >= nxn || j < 0 || j >= nyn) {
#pragma unroll
    for (int k = 0; k < 3; ++k) o.v[k] = 0.0f;
    return o;
  }
  const size_t n = (size_t)j * nxn + i;
#pragma unroll
  for (int k = 0; k < 3; ++k) o.v[k] = p[3 * n + k];
  return o;
}
// y += b x, or b^T x for a block stored at the neighbour (the order of stencil_row_f)
__device__ __forceinline__ void w3fwd(float (&y)[3], const W3Blk& b, const W3Vec& x) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) y[r] += b.v[r * 3 + c] * x.v[c];
}
__device__ __forceinline__ void w3bwd(float (&y)[3], const W3Blk& b, const W3Vec& x) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) y[r] += b.v[c * 3 + r] * x.v[c];
}

template <int MODE, int XM>
__global__ void __launch_bounds__(256)
k_cheb_walk3(int TR, const float* __restrict__ A, size_t nn, int nxn, int nyn, const float* __restrict__ vin,
             const float* __restrict__ rin, const float* xin, float* __restrict__ rout, float* __restrict__ dout,
             float* xout, float c1a, float c1b, float c2a, float c2b) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 62 - 1 + lane;
  const int j0 = (blockIdx.y * 4 + (int)(threadIdx.x >> 6)) * TR;
  const bool in = i >= 0 && i < nxn;
  const int ic = in ? i : -(1 << 29);   // idle lanes load nothing
  const int lm = (lane + 63) & 63, lp = (lane + 1) & 63;
  W3Vec zv;
#pragma unroll
  for (int k = 0; k < 3; ++k) zv.v[k] = 0.0f;
  W3Blk z;
#pragma unroll
  for (int k = 0; k < 9; ++k) z.v[k] = 0.0f;
  // rows r-1 (q*) and r-2 (s*: north, north-east, north-west) of the stored blocks
  W3Blk q0 = w3blk(A, nn, 0, nxn, nyn, ic, j0 - 2), qE = w3blk(A, nn, 1, nxn, nyn, ic, j0 - 2),
        qN = w3blk(A, nn, 2, nxn, nyn, ic, j0 - 2), qNE = w3blk(A, nn, 3, nxn, nyn, ic, j0 - 2),
        qNW = w3blk(A, nn, 4, nxn, nyn, ic, j0 - 2);
  W3Blk sN = z, sNE = z, sNW = z;
  W3Vec vS = w3vec(vin, nxn, nyn, ic, j0 - 2), vC = w3vec(vin, nxn, nyn, ic, j0 - 1);
  W3Vec d1pp = zv, d1p = zv, r1p = zv;
  for (int r = j0 - 1; r <= j0 + TR; ++r) {
    if (r > nyn) break;   // uniform across the wave
    const W3Blk P0 = w3blk(A, nn, 0, nxn, nyn, ic, r), PE = w3blk(A, nn, 1, nxn, nyn, ic, r),
                PN = w3blk(A, nn, 2, nxn, nyn, ic, r), PNE = w3blk(A, nn, 3, nxn, nyn, ic, r),
                PNW = w3blk(A, nn, 4, nxn, nyn, ic, r);
    const W3Vec vN = w3vec(vin, nxn, nyn, ic, r + 1);
    const W3Vec rC = w3vec(rin, nxn, nyn, ic, r);
    // first sweep at row r
    W3Vec vCL = w3shv(vC, lm), vCR = w3shv(vC, lp), vNL = w3shv(vN, lm), vNR = w3shv(vN, lp), vSL = w3shv(vS, lm),
          vSR = w3shv(vS, lp);
    W3Blk PEL = w3shb(PE, lm), qNEL = w3shb(qNE, lm), qNWR = w3shb(qNW, lp);
    if (lane == 0) {
      vCL = w3vec(vin, nxn, nyn, i - 1, r);
      vNL = w3vec(vin, nxn, nyn, i - 1, r + 1);
      vSL = w3vec(vin, nxn, nyn, i - 1, r - 1);
      PEL = w3blk(A, nn, 1, nxn, nyn, i - 1, r);
      qNEL = w3blk(A, nn, 3, nxn, nyn, i - 1, r - 1);
    }
    if (lane == 63) {
      vCR = w3vec(vin, nxn, nyn, i + 1, r);
      vNR = w3vec(vin, nxn, nyn, i + 1, r + 1);
      vSR = w3vec(vin, nxn, nyn, i + 1, r - 1);
      qNWR = w3blk(A, nn, 4, nxn, nyn, i + 1, r - 1);
    }
    W3Vec d1c = zv, r1c = zv;
    if (in && r >= 0 && r < nyn) {
      float y[3] = {0.0f, 0.0f, 0.0f};
      const bool hE = i + 1 < nxn, hW = i > 0, hN = r + 1 < nyn, hS = r > 0;
      w3fwd(y, P0, vC);
      if (hE) w3fwd(y, PE, vCR);
      if (hN) w3fwd(y, PN, vN);
      if (hE && hN) w3fwd(y, PNE, vNR);
      if (hW && hN) w3fwd(y, PNW, vNL);
      if (hW) w3bwd(y, PEL, vCL);
      if (hS) w3bwd(y, qN, vS);
      if (hW && hS) w3bwd(y, qNEL, vSL);
      if (hE && hS) w3bwd(y, qNWR, vSR);
      float D[3][3], Di[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) D[a][c] = P0.v[a * 3 + c];
      invert_block<3>(D, Di);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float rn = rC.v[k] - y[k];
        r1c.v[k] = rn;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float t = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) t += Di[k][c] * r1c.v[c];
        if constexpr (MODE == PAIR_RFIRST_STEP) d1c.v[k] = t * c1a;
        else d1c.v[k] = fma(c1a, vC.v[k], c1b * t);
      }
    }
    // second sweep at row j = r - 1, inner lanes
    const int j = r - 1;
    const W3Vec dL = w3shv(d1p, lm), dR = w3shv(d1p, lp), dNL = w3shv(d1c, lm), dNR = w3shv(d1c, lp),
                dSL = w3shv(d1pp, lm), dSR = w3shv(d1pp, lp);
    const W3Blk qEL = w3shb(qE, lm), sNEL = w3shb(sNE, lm), sNWR = w3shb(sNW, lp);
    if (j >= j0 && j < nyn && in && lane >= 1 && lane <= 62) {
      const size_t n = (size_t)j * nxn + i;
      float x1[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if constexpr (MODE == PAIR_RFIRST_STEP) {
          x1[k] = xin[3 * n + k];   // the first sweep leaves x unchanged
        } else {
          if constexpr (XM == 2) {
            x1[k] = vS.v[k];        // vin at row j
          } else {
            x1[k] = xin[3 * n + k];
            if constexpr (XM == 1) x1[k] += vS.v[k];
          }
          x1[k] = x1[k] + d1p.v[k];
        }
      }
      float y[3] = {0.0f, 0.0f, 0.0f};
      const bool hE = i + 1 < nxn, hW = i > 0, hN = j + 1 < nyn, hS = j > 0;
      w3fwd(y, q0, d1p);
      if (hE) w3fwd(y, qE, dR);
      if (hN) w3fwd(y, qN, d1c);
      if (hE && hN) w3fwd(y, qNE, dNR);
      if (hW && hN) w3fwd(y, qNW, dNL);
      if (hW) w3bwd(y, qEL, dL);
      if (hS) w3bwd(y, sN, d1pp);
      if (hW && hS) w3bwd(y, sNEL, dSL);
      if (hE && hS) w3bwd(y, sNWR, dSR);
      float r2[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        r2[k] = r1p.v[k] - y[k];
        rout[3 * n + k] = r2[k];
      }
      if constexpr (MODE == PAIR_STEP_RESID) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xout[3 * n + k] = x1[k];
      } else {
        float D[3][3], Di[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) D[a][c] = q0.v[a * 3 + c];
        invert_block<3>(D, Di);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if constexpr (MODE == PAIR_RFIRST_STEP) x1[k] += d1p.v[k];   // (x + d0) + d1
          float t = 0.0f;
#pragma unroll
          for (int c = 0; c < 3; ++c) t += Di[k][c] * r2[c];
          const float d2 = fma(c2a, d1p.v[k], c2b * t);
          dout[3 * n + k] = d2;
          xout[3 * n + k] = x1[k] + d2;
        }
      }
    }
    sN = qN; sNE = qNE; sNW = qNW;
    q0 = P0; qE = PE; qN = PN; qNE = PNE; qNW = PNW;
    vS = vC; vC = vN;
    d1pp = d1p; d1p = d1c; r1p = r1c;
  }
}

// ---------------------------------------------------------------------------
// the smallest levels in one workgroup
// ---------------------------------------------------------------------------
// Below a few thousand nodes every kernel of the V-cycle is launch- and
// latency-bound (a few microseconds for a handful of waves).  The part of the
// cycle from level l0 (coarse, B = 3) down to the dense coarsest solve and back
// runs in one workgroup instead: the same per-node bodies, looped over the nodes
// of each sweep, with a workgroup barrier between sweeps.
constexpr int kTailNodes = 1024;   // levels with at most this many nodes
constexpr int kTailLevels = 6;
constexpr int kTailDegree = 8;
constexpr int kTailThreads = 1024;

struct TailLevel {
  const void* A;     // operator (storage type TM)
  const void* P;     // prolongator to the next level (TP)
  void *b, *x, *r, *d0, *d1;
  unsigned nn;
  int nxn, nyn, ncx, ncy;
  double inv_theta;
  double cdd[kTailDegree], cdr[kTailDegree];   // Chebyshev step coefficients, index 1..degree-1
};
struct TailArgs {
  TailLevel L[kTailLevels];
  const void* Ainv;  // dense inverse of the coarsest level (TV)
  int nlev, degree, nd;
};

template <typename TM, typename TV>
__device__ void tail_smooth(const TailLevel& L, const TV* b, TV* x, bool pre, int degree) {
  using TA = typename Acc<TV>::type;
  const TM* A = (const TM*)L.A;
  TV* r = (TV*)L.r;
  TV* d[2] = {(TV*)L.d0, (TV*)L.d1};
  const size_t nn = L.nn;
  const TA inv_theta = (TA)L.inv_theta;
  const unsigned t0 = threadIdx.x, nt = blockDim.x;
  if (pre) {
    for (size_t n = t0; n < nn; n += nt)
      node_cheb_first<3>(A, nn, b, degree == 1 ? r : (TV*)nullptr, d[0], degree == 1 ? x : (TV*)nullptr, inv_theta, 0,
                         n);
  } else if (degree == 1) {
    for (size_t n = t0; n < nn; n += nt) node_sten_resid<3>(A, nn, L.nxn, L.nyn, (const TV*)x, b, r, n);
    __syncthreads();
    for (size_t n = t0; n < nn; n += nt) node_cheb_first<3>(A, nn, (const TV*)r, (TV*)nullptr, d[0], x, inv_theta, 1, n);
  } else {
    for (size_t n = t0; n < nn; n += nt) node_resid_first<3>(A, nn, L.nxn, L.nyn, (const TV*)x, b, r, d[0], inv_theta, n);
  }
  __syncthreads();
  for (int k = 1; k < degree; ++k) {
    const int xmode = k > 1 ? 0 : pre ? 2 : 1;
    const TV* rin = (pre && k == 1) ? b : (const TV*)r;
    for (size_t n = t0; n < nn; n += nt)
      node_cheb_step<3>(A, nn, L.nxn, L.nyn, (const TV*)d[(k - 1) & 1], rin, r, d[k & 1], (const TV*)x, x,
                        (TA)L.cdd[k], (TA)L.cdr[k], xmode, n);
    __syncthreads();
  }
  if (pre) {
    for (size_t n = t0; n < nn; n += nt)
      node_sten_resid<3>(A, nn, L.nxn, L.nyn, (const TV*)d[(degree - 1) & 1], (const TV*)r, r, n);
    __syncthreads();
  }
}

template <typename TM, typename TP, typename TV>
__global__ void __launch_bounds__(kTailThreads) k_vcycle_tail(TailArgs a) {
  const unsigned t0 = threadIdx.x, nt = blockDim.x;   // nt is a multiple of the restriction lane group
  for (int l = 0; l + 1 < a.nlev; ++l) {
    const TailLevel& L = a.L[l];
    const TailLevel& N = a.L[l + 1];
    tail_smooth<TM, TV>(L, (const TV*)L.b, (TV*)L.x, true, a.degree);
    const size_t ng = (size_t)N.nn * kRestrictLanes;
    for (size_t g = t0; g < ng; g += nt)
      group_restrict<3>((const TP*)L.P, (size_t)L.nn, L.nxn, L.nyn, L.ncx, L.ncy, (const TV*)L.r, (TV*)N.b,
                        g / kRestrictLanes, (int)(g % kRestrictLanes));
    __syncthreads();
  }
  const TailLevel& C = a.L[a.nlev - 1];
  for (int rw = (int)t0; rw < a.nd; rw += (int)nt) row_dense_apply((const TV*)a.Ainv, a.nd, (const TV*)C.b, (TV*)C.x, rw);
  __syncthreads();
  for (int l = a.nlev - 2; l >= 0; --l) {
    const TailLevel& L = a.L[l];
    const TailLevel& N = a.L[l + 1];
    for (size_t n = t0; n < L.nn; n += nt)
      node_prolong_add<3>((const TP*)L.P, (size_t)L.nn, L.nxn, L.nyn, L.ncx, L.ncy, (const TV*)N.x, (const TV*)L.x,
                          (TV*)L.x, n);
    __syncthreads();
    tail_smooth<TM, TV>(L, (const TV*)L.b, (TV*)L.x, false, a.degree);
  }
}

// The same V-cycle over the tail levels with FP32 vectors, restructured for
// latency: every vector of every tail level lives in LDS (read through generic
// pointers by the shared restriction, prolongation and dense-solve helpers), and
// each thread keeps its node's nine stencil blocks and its diagonal inverse in
// registers for the whole smoothing of a level, so a sweep waits only on LDS and the
// barrier.  Per node the arithmetic is that of the node kernels in the same order
// (stencil_row_f's neighbour order, the same fused multiply-adds): bitwise the
// results of k_vcycle_tail.  Chebyshev degree >= 2; the levels' vectors must fit
// kTailLdsFloats (15 floats per node) and the first tail level kTailLdsThreads nodes
// (one node per thread; 768 threads leave 170 registers per thread, enough to hold
// the 81 block entries without spilling, which 1024 threads' 128 are not).
constexpr int kTailLdsFloats = 18000;
constexpr int kTailLdsThreads = 768;

__device__ __forceinline__ float* tail_vec(float* sv, const TailArgs& a, int l, int q) {
  int off = 0;
  for (int k = 0; k < l; ++k) off += 15 * (int)a.L[k].nn;
  return sv + off + q * 3 * (int)a.L[l].nn;
}

template <typename TM>
__device__ void tail_smooth_reg(const TailLevel& L, float* b, float* x, float* r, float* d0, float* d1, bool pre,
                                int degree) {
  const int t = (int)threadIdx.x;
  const int nn = (int)L.nn, nxn = L.nxn, nyn = L.nyn;
  const bool own = t < nn;
  const int i = own ? t % nxn : 0, j = own ? t / nxn : 0;
  float blk[9][3][3];
  unsigned valid = 0u;
  float Di[3][3];
  if (own) {
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      if (ii < 0 || jj < 0 || ii >= nxn || jj >= nyn) continue;
      valid |= 1u << d;
      load_block<3>((const TM*)L.A, (size_t)nn, nxn, i, j, d, blk[d]);
    }
    invert_block<3>(blk[0], Di);
  }
  auto stencil = [&](const float* v, float (&y)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] = 0.0f;
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      if (!((valid >> d) & 1u)) continue;
      const int m = (j + kDJ[d]) * nxn + (i + kDI[d]);
      float xm[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) xm[c] = v[3 * m + c];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) y[k] += blk[d][k][c] * xm[c];
    }
  };
  const float inv_theta = (float)L.inv_theta;
  float* d[2] = {d0, d1};
  if (own) {
    if (pre) {   // d0 = D^-1 b / theta
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float tt = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) tt += Di[k][c] * b[3 * t + c];
        d0[3 * t + k] = tt * inv_theta;
      }
    } else {     // r = b - A x, d0 = D^-1 r / theta
      float y[3], rn[3];
      stencil(x, y);
#pragma unroll
      for (int k = 0; k < 3; ++k) rn[k] = b[3 * t + k];
#pragma unroll
      for (int k = 0; k < 3; ++k) rn[k] -= y[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) r[3 * t + k] = rn[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float tt = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) tt += Di[k][c] * rn[c];
        d0[3 * t + k] = tt * inv_theta;
      }
    }
  }
  __syncthreads();
  for (int s = 1; s < degree; ++s) {
    const int xmode = s > 1 ? 0 : pre ? 2 : 1;
    const float* dp = d[(s - 1) & 1];
    float* dn = d[s & 1];
    const float* rin = (pre && s == 1) ? b : r;
    if (own) {
      float y[3], rn[3], dpn[3], xn[3], dk[3];
      stencil(dp, y);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        rn[k] = rin[3 * t + k];
        dpn[k] = dp[3 * t + k];
      }
      if (xmode == 2) {
#pragma unroll
        for (int k = 0; k < 3; ++k) xn[k] = dpn[k];
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) xn[k] = x[3 * t + k];
        if (xmode == 1) {
#pragma unroll
          for (int k = 0; k < 3; ++k) xn[k] += dpn[k];
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) rn[k] -= y[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) r[3 * t + k] = rn[k];
      const float cdd = (float)L.cdd[s], cdr = (float)L.cdr[s];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float tt = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) tt += Di[k][c] * rn[c];
        dk[k] = fma(cdd, dpn[k], cdr * tt);
        xn[k] += dk[k];
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        dn[3 * t + k] = dk[k];
        x[3 * t + k] = xn[k];
      }
    }
    __syncthreads();
  }
  if (pre) {   // r = r - A d: the residual after the last step
    if (own) {
      float y[3], bb[3];
      stencil(d[(degree - 1) & 1], y);
#pragma unroll
      for (int k = 0; k < 3; ++k) bb[k] = r[3 * t + k];
#pragma unroll
      for (int k = 0; k < 3; ++k) bb[k] = bb[k] - y[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) r[3 * t + k] = bb[k];
    }
    __syncthreads();
  }
}

template <typename TM, typename TP>
__global__ void __launch_bounds__(kTailLdsThreads) k_vcycle_tail_lds(TailArgs a) {
  __shared__ float sv[kTailLdsFloats];
  const int t0 = (int)threadIdx.x, nt = (int)blockDim.x;
  {
    const float* b0 = (const float*)a.L[0].b;
    float* vb = tail_vec(sv, a, 0, 0);
    for (int e = t0; e < 3 * (int)a.L[0].nn; e += nt) vb[e] = b0[e];
  }
  __syncthreads();
  for (int l = 0; l + 1 < a.nlev; ++l) {
    const TailLevel& L = a.L[l];
    const TailLevel& N = a.L[l + 1];
    tail_smooth_reg<TM>(L, tail_vec(sv, a, l, 0), tail_vec(sv, a, l, 1), tail_vec(sv, a, l, 2),
                        tail_vec(sv, a, l, 3), tail_vec(sv, a, l, 4), true, a.degree);
    const float* rl = tail_vec(sv, a, l, 2);
    float* bn = tail_vec(sv, a, l + 1, 0);
    const size_t ng = (size_t)N.nn * kRestrictLanes;
    for (size_t g = t0; g < ng; g += nt)
      group_restrict<3>((const TP*)L.P, (size_t)L.nn, L.nxn, L.nyn, L.ncx, L.ncy, rl, bn, g / kRestrictLanes,
                        (int)(g % kRestrictLanes));
    __syncthreads();
  }
  {
    const int lc = a.nlev - 1;
    const float* bc = tail_vec(sv, a, lc, 0);
    float* xc = tail_vec(sv, a, lc, 1);
    for (int rw = t0; rw < a.nd; rw += nt) row_dense_apply((const float*)a.Ainv, a.nd, bc, xc, rw);
  }
  __syncthreads();
  for (int l = a.nlev - 2; l >= 0; --l) {
    const TailLevel& L = a.L[l];
    const TailLevel& N = a.L[l + 1];
    float* xl = tail_vec(sv, a, l, 1);
    const float* xn = tail_vec(sv, a, l + 1, 1);
    for (int n = t0; n < (int)L.nn; n += nt)
      node_prolong_add<3>((const TP*)L.P, (size_t)L.nn, L.nxn, L.nyn, L.ncx, L.ncy, xn, (const float*)xl, xl,
                          (size_t)n);
    __syncthreads();
    tail_smooth_reg<TM>(L, tail_vec(sv, a, l, 0), xl, tail_vec(sv, a, l, 2), tail_vec(sv, a, l, 3),
                        tail_vec(sv, a, l, 4), false, a.degree);
  }
  {
    float* x0 = (float*)a.L[0].x;
    const float* vx = tail_vec(sv, a, 0, 1);
    for (int e = t0; e < 3 * (int)a.L[0].nn; e += nt) x0[e] = vx[e];
  }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// Near-null-space row block of node (i,j) on the finest level: rigid motions
// (1,0), (0,1), (-y,x); zero rows at Dirichlet nodes.  (cx, cy, sc) shift and
// scale the coordinates.
__device__ __forceinline__ void rigid_rows(int i, int j, int nxn, int nyn, double cx, double cy,
                                           double sc, double (&b)[3][3]) {
  const bool bnd = i == 0 || j == 0 || i == nxn - 1 || j == nyn - 1;
  const double x = (i - cx) * sc, y = (j - cy) * sc;
  b[0][0] = 1.0; b[0][1] = 0.0; b[0][2] = -y;
  b[1][0] = 0.0; b[1][1] = 1.0; b[1][2] = x;
  b[2][0] = b[2][1] = b[2][2] = 0.0;
  if (bnd) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) b[r][c] = 0.0;
  }
}

// Cholesky of a 3x3 SPD matrix G = R^T R (R upper).  Tiny pivots -> zero column.
__device__ __forceinline__ void chol3(const double (&G)[3][3], double (&R)[3][3]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[r][c] = 0.0;
  const double scale = fmax(fmax(G[0][0], G[1][1]), G[2][2]);
  for (int k = 0; k < 3; ++k) {
    double s = G[k][k];
    for (int m = 0; m < k; ++m) s -= R[m][k] * R[m][k];
    if (s <= 1e-24 * scale) continue;  // dependent column: leave R row k zero
    R[k][k] = sqrt(s);
    for (int c = k + 1; c < 3; ++c) {
      double t = G[k][c];
      for (int m = 0; m < k; ++m) t -= R[m][k] * R[m][c];
      R[k][c] = t / R[k][k];
    }
  }
}

// q = b R^{-1} for a row vector b (R upper triangular; zero pivots give zero q)
__device__ __forceinline__ void rsolve_row(const double (&R)[3][3], const double (&b)[3], double (&q)[3]) {
  for (int c = 0; c < 3; ++c) {
    double t = b[c];
    for (int m = 0; m < c; ++m) t -= q[m] * R[m][c];
    q[c] = R[c][c] != 0.0 ? t / R[c][c] : 0.0;
  }
}

// Tentative prolongator by Cholesky-QR applied twice per aggregate, and the
// coarse near-null space Bc = Q^T B (B with global coordinates on the finest level).
template <int B>
__global__ void k_tentative(int nxn, int nyn, int ncx, int ncy, const double* __restrict__ Bnull,
                            double* __restrict__ Ptent, double* __restrict__ Bc) {
  const size_t I = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= (size_t)ncx * ncy) return;
  const size_t nn = (size_t)nxn * nyn, ncn = (size_t)ncx * ncy;
  const int Ix = (int)(I % ncx), Iy = (int)(I / ncx);
  const int i0 = 3 * Ix, i1 = agg_last(Ix, nxn, ncx), j0 = 3 * Iy, j1 = agg_last(Iy, nyn, ncy);
  const double cx = 0.5 * (i0 + i1), cy = 0.5 * (j0 + j1);
  const double gsc = 1.0 / (double)max(nxn, nyn);
  auto rows = [&](int i, int j, bool local, double (&b)[3][3]) {
    if constexpr (B == 2) {
      if (local) rigid_rows(i, j, nxn, nyn, cx, cy, 1.0 / 3.0, b);
      else rigid_rows(i, j, nxn, nyn, 0.0, 0.0, gsc, b);
    } else {
      const size_t n = (size_t)j * nxn + i;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) b[r][c] = Bnull[(size_t)(r * 3 + c) * nn + n];
    }
  };
  double R1[3][3], R2[3][3];
  // pass 1: G = B^T B
  double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      double b[3][3];
      rows(i, j, true, b);
      for (int r = 0; r < B; ++r)
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) G[a][c] += b[r][a] * b[r][c];
    }
  chol3(G, R1);
  // pass 2: G2 = (B R1^-1)^T (B R1^-1)
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) G[a][c] = 0.0;
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      double b[3][3];
      rows(i, j, true, b);
      for (int r = 0; r < B; ++r) {
        double q[3];
        rsolve_row(R1, b[r], q);
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) G[a][c] += q[a] * q[c];
      }
    }
  chol3(G, R2);
  // pass 3: Q = B R1^-1 R2^-1 written per node; Bc = Q^T B_global
  double Bcl[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int j = j0; j <= j1; ++j)
    for (int i = i0; i <= i1; ++i) {
      double b[3][3], bg[3][3];
      rows(i, j, true, b);
      rows(i, j, false, bg);
      const size_t n = (size_t)j * nxn + i;
      for (int r = 0; r < B; ++r) {
        double q1[3], q[3];
        rsolve_row(R1, b[r], q1);
        rsolve_row(R2, q1, q);
        for (int c = 0; c < 3; ++c) Ptent[(size_t)(r * 3 + c) * nn + n] = q[c];
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) Bcl[a][c] += q[a] * bg[r][c];
      }
    }
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) Bc[(size_t)(a * 3 + c) * ncn + I] = Bcl[a][c];
}

// Per-workgroup max of the Gershgorin bound of D^{-1} A (block Jacobi):
// max over rows of sum over blocks of |D^{-1} A_nm| row sums.
template <int B, typename TM = double>
__global__ void __launch_bounds__(kBlock)
k_gershgorin(const TM* __restrict__ A, size_t nn, int nxn, int nyn, double* __restrict__ partials) {
  __shared__ double lds[16];
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double best = 0.0;
  if (n < nn) {
    const int i = (int)(n % nxn), j = (int)(n / nxn);
    double D[B][B], Di[B][B];
    load_block<B>(A, nn, nxn, i, j, 0, D);
    invert_block<B>(D, Di);
    double rs[B];
    for (int r = 0; r < B; ++r) rs[r] = 0.0;
    for (int d = 0; d < 9; ++d) {
      const int ii = i + kDI[d], jj = j + kDJ[d];
      if (ii < 0 || jj < 0 || ii >= nxn || jj >= nyn) continue;
      double blk[B][B];
      load_block<B>(A, nn, nxn, i, j, d, blk);
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) {
          double t = 0.0;
          for (int k = 0; k < B; ++k) t += Di[r][k] * blk[k][c];
          rs[r] += fabs(t);
        }
    }
    for (int r = 0; r < B; ++r) best = fmax(best, rs[r]);
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, lds[w]);
    partials[blockIdx.x] = m;
  }
}

// The same bound for the symmetric block 25-point stencil of Q2 elements: the
// stored blocks of node n and the transposes of the blocks stored at n - o.
__global__ void __launch_bounds__(kBlock)
k_gershgorin25(const double* __restrict__ A, size_t nn, int nxn, int nyn, double* __restrict__ partials) {
  __shared__ double lds[16];
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double best = 0.0;
  if (n < nn) {
    const int i = (int)(n % nxn), j = (int)(n / nxn);
    double D[2][2], Di[2][2];
    for (int r = 0; r < 2; ++r)
      for (int q = 0; q < 2; ++q) D[r][q] = A[aidx(2, nn, 0, n, r, q)];
    invert_block<2>(D, Di);
    double rs[2] = {0.0, 0.0};
    auto add = [&](const double (&blk)[2][2]) {
      for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) rs[r] += fabs(Di[r][0] * blk[0][q] + Di[r][1] * blk[1][q]);
    };
    for (int d = 0; d < 13; ++d) {
      const int ox = q2_ox(d), oy = q2_oy(d);
      if (i + ox >= 0 && i + ox < nxn && j + oy < nyn) {
        double blk[2][2];
        for (int r = 0; r < 2; ++r)
          for (int q = 0; q < 2; ++q) blk[r][q] = A[aidx(2, nn, d, n, r, q)];
        add(blk);
      }
      if (d > 0 && i - ox >= 0 && i - ox < nxn && j - oy >= 0) {
        const size_t m = (size_t)(j - oy) * nxn + (i - ox);
        double blk[2][2];
        for (int r = 0; r < 2; ++r)
          for (int q = 0; q < 2; ++q) blk[r][q] = A[aidx(2, nn, d, m, q, r)];
        add(blk);
      }
    }
    best = fmax(rs[0], rs[1]);
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, lds[w]);
    partials[blockIdx.x] = m;
  }
}

// Power iteration for lmax(D^{-1} A) (block Jacobi), device resident and warm
// started across setups.  One step: y = D^{-1} A x / |x|, partial sums of |y|^2;
// |x|^2 is read from nrm2_in (device), so no host synchronisation is needed.
__global__ void k_power_init(double* __restrict__ x, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    // deterministic pseudo-random start (splitmix-style hash of the index)
    unsigned long long z = (unsigned long long)e * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[e] = 0.5 + (double)(z >> 11) * (1.0 / 9007199254740992.0);
  }
}

template <int B, int ST = 0, typename TM = double>
__global__ void __launch_bounds__(kBlock)
k_power_step(const TM* __restrict__ A, size_t nn, int nxn, int nyn, const double* __restrict__ x,
             const double* __restrict__ nrm2_in, double* __restrict__ y, double* __restrict__ partials) {
  __shared__ double lds[16];
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (n < nn) {
    const int i = (int)(n % nxn), j = (int)(n / nxn);
    const double s = nrm2_in[0] > 0.0 ? 1.0 / sqrt(nrm2_in[0]) : 0.0;
    double Ax[B], D[B][B], Di[B][B];
    stencil_row<B, ST>(A, nn, nxn, nyn, i, j, x, Ax, D);
    invert_block<B>(D, Di);
    for (int r = 0; r < B; ++r) {
      double t = 0.0;
      for (int c = 0; c < B; ++c) t += Di[r][c] * Ax[c];
      t *= s;
      y[n * B + r] = t;
      acc[0] += t * t;
    }
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// lmax = factor * |y| (|x| = 1 after scaling), never above the Gershgorin bound
__global__ void k_power_final(const double* __restrict__ nrm2, double factor, double* __restrict__ lmax) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double est = factor * sqrt(fmax(nrm2[0], 0.0));
    const double g = lmax[0];
    lmax[0] = (est > 0.0 && est < g) ? est : g;
  }
}

// One device scalar from each of up to kMaxLevels + 1 places into out[0 .. n)
struct ScalarPtrs {
  const double* p[kMaxLevels + 1];
  int n;
};
__global__ void k_gather_scalars(ScalarPtrs a, double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t < a.n) out[t] = a.p[t][0];
}

__global__ void k_finish_max(const double* __restrict__ partials, int nblocks, double* __restrict__ out) {
  __shared__ double lds[512];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) m = fmax(m, partials[b]);
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = lds[0];
}

// Smoothed prolongator P = (I - omega D^{-1} A) Ptent, omega = omega_scale * 4/(3 lmax),
// computed in FP64 and stored in FP64 (P), FP32 (P32) or both.  TM = float: from the
// FP32 copy of the operator (the FP32 modes, whose V-cycle and Galerkin products use
// the FP32 prolongator only).
template <int B, typename TM = double>
__global__ void __launch_bounds__(kBlock)
k_smooth_p(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int ncx, int ncy,
           const double* __restrict__ Ptent, const double* __restrict__ lmax, double omega_scale,
           double* __restrict__ P, float* __restrict__ P32) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  const double omega = omega_scale * 4.0 / (3.0 * lmax[0]);
  double D[B][B], Di[B][B];
  load_block<B>(A, nn, nxn, i, j, 0, D);
  invert_block<B>(D, Di);
  const int ax[2] = {agg_of(i, ncx), agg_other(i, nxn, ncx)};
  const int ay[2] = {agg_of(j, ncy), agg_other(j, nyn, ncy)};
  // (A Ptent) restricted to each slot's aggregate: every neighbour lies in the
  // node's own aggregate or the adjacent one along each axis, so one pass over the
  // nine neighbours adds each term to its slot (in the order of d, per slot)
  double acc[4][B][3];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[sl][r][c] = 0.0;
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int ii = i + kDI[d], jj = j + kDJ[d];
    if (ii < 0 || jj < 0 || ii >= nxn || jj >= nyn) continue;
    const int sl = (agg_of(ii, ncx) == ax[0] ? 0 : 1) + (agg_of(jj, ncy) == ay[0] ? 0 : 2);
    double blk[B][B];
    load_block<B>(A, nn, nxn, i, j, d, blk);
    const size_t m = (size_t)jj * nxn + ii;
    double pt[B][3];
#pragma unroll
    for (int k = 0; k < B; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) pt[k][c] = Ptent[(size_t)(k * 3 + c) * nn + m];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s != sl) continue;
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int k = 0; k < B; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[s][r][c] += blk[r][k] * pt[k][c];
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const bool ok = ax[s & 1] >= 0 && ay[s >> 1] >= 0;
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k) t += Di[r][k] * acc[s][k][c];
        double val = -omega * t;
        if (s == 0) val += Ptent[(size_t)(r * 3 + c) * nn + n];
        if (!ok) val = 0.0;
        if (P) P[pidx(B, nn, s, n, r, c)] = val;
        if (P32) P32[pidx(B, nn, s, n, r, c)] = (float)val;
      }
  }
}

// Galerkin coarse operator Ac = P^T A P in the 5-block symmetric storage (3x3
// blocks), in two coalesced passes.
//
// Pass 1 (one thread per fine node i): W(i, J) = sum_k A(i,k) P(k,J) for the
// coarse nodes J = agg(i) + (qx-1, qy-1), q = qy*3 + qx in 0..8 (A P vanishes for
// every other J: the prolongator columns of k's neighbours reach at most one
// aggregate further).  W[((q*B + r)*3 + c)*nw + gw_index(i)], nw = gw_size, zero
// where J is absent.  TM is the operator's and prolongator's storage type and TW
// that of W, which is also the accumulation type: FP64 throughout, or, in the FP32
// modes, the FP32 copies of A and P the V-cycle applies with W accumulated and
// stored in FP32 (half the bytes; the coarse sums of the second pass stay FP64).
template <int B, typename TM, typename TW>
__device__ __forceinline__ void galerkin_ap_compute(const TM* __restrict__ A, size_t nn, int nxn, int nyn,
                                                    int ncx, int ncy, const TM* __restrict__ P, int i, int j,
                                                    TW (&w)[9][B][3]) {
  const int ax = agg_of(i, ncx), ay = agg_of(j, ncy);
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) w[q][r][c] = (TW)0;
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int ii = i + kDI[d], jj = j + kDJ[d];
    if (ii < 0 || jj < 0 || ii >= nxn || jj >= nyn) continue;
    TW blk[B][B];
    load_block<B>(A, nn, nxn, i, j, d, blk);
    const size_t m = (size_t)jj * nxn + ii;
#pragma unroll
    for (int qy = 0; qy < 3; ++qy) {
      const int sy = slot1(jj, nyn, ncy, ay + qy - 1);
      if (sy < 0) continue;
#pragma unroll
      for (int qx = 0; qx < 3; ++qx) {
        const int sx = slot1(ii, nxn, ncx, ax + qx - 1);
        if (sx < 0) continue;
        const int sl = sx + 2 * sy;
#pragma unroll
        for (int k = 0; k < B; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const TW pv = (TW)P[pidx(B, nn, sl, m, k, c)];
#pragma unroll
            for (int r = 0; r < B; ++r) w[qy * 3 + qx][r][c] += blk[r][k] * pv;
          }
      }
    }
  }
}

// One thread per fine node in row order (coalesced loads of A and P); the stores
// follow the aggregate-major order of W, three runs of consecutive addresses per
// wave.  Measured against the alternatives at 2049^2: threads in the order of W
// (loads three nodes apart) and a row-order tile transposed through LDS before the
// stores were both slower.
template <int B, typename TM = double, typename TW = double>
__global__ void __launch_bounds__(kBlock)
k_galerkin_ap(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int ncx, int ncy,
              const TM* __restrict__ P, TW* __restrict__ W) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  TW w[9][B][3];
  galerkin_ap_compute<B>(A, nn, nxn, nyn, ncx, ncy, P, i, j, w);
  const size_t nw = gw_size(nxn, nyn, ncx, ncy), gi = gw_index(i, j, nxn, nyn, ncx, ncy);
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) W[(size_t)((q * B + r) * 3 + c) * nw + gi] = w[q][r][c];
}

// Pass 1 with threads in the order of W, for FP32 W: a workgroup of three waves
// takes 64 aggregates of one fine row, wave w the nodes at position w in them, so
// each store writes 64 consecutive values of a class plane (whole lines; measured
// faster than the row-order threads' three partial runs per store); the loads are
// three nodes apart and the three waves share their lines.  Per row, one more workgroup takes the nodes past
// the last full run of 3 (positions 3 and 4 of a longer last run), and the rows past
// the last full run in y go in row order (their W entries are stored in row order).
// Workgroups are numbered row by row and dealt to the XCDs in contiguous runs.
constexpr int kApWThreads = 192;
template <int B, typename TM, typename TW>
__global__ void __launch_bounds__(kApWThreads)
k_galerkin_ap_w(const TM* __restrict__ A, size_t nn, int nxn, int nyn, int ncx, int ncy, int gx,
                const TM* __restrict__ P, TW* __restrict__ W) {
  const unsigned t = xcd_block();
  const int j = (int)(t / (unsigned)gx), b = (int)(t % (unsigned)gx);
  if (j >= nyn) return;
  const int nbx = (ncx + 63) / 64;
  int i;
  if (j < 3 * ncy) {
    if (b < nbx) {
      const int ax = b * 64 + (int)(threadIdx.x & 63);
      if (ax >= ncx) return;
      i = 3 * ax + (int)(threadIdx.x >> 6);
    } else if (b == nbx) {
      i = 3 * ncx + (int)threadIdx.x;
      if (i >= nxn) return;
    } else {
      return;
    }
  } else {
    i = b * kApWThreads + (int)threadIdx.x;
    if (i >= nxn) return;
  }
  TW w[9][B][3];
  galerkin_ap_compute<B>(A, nn, nxn, nyn, ncx, ncy, P, i, j, w);
  const size_t nw = gw_size(nxn, nyn, ncx, ncy), gi = gw_index(i, j, nxn, nyn, ncx, ncy);
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) W[(size_t)((q * B + r) * 3 + c) * nw + gi] = w[q][r][c];
}
template <int B, typename TM, typename TW>
void launch_galerkin_ap_w(hipStream_t s, const Level& L, const TM* A, const TM* P, TW* W) {
  const int gx = std::max((L.ncx + 63) / 64 + 1, (L.nxn + kApWThreads - 1) / kApWThreads);
  hipLaunchKernelGGL((k_galerkin_ap_w<B, TM, TW>), dim3(grid_for((size_t)gx * L.nyn, 1)), dim3(kApWThreads), 0, s, A,
                     L.nn, L.nxn, L.nyn, L.ncx, L.ncy, gx, P, W);
  VP_LAUNCH_CHECK();
}

// Pass 2 (one thread per coarse node I): Ac(I, J_t) = sum over the fine nodes i of
// I's prolongator support of P(i,I)^T W(i, J_t) for the 5 stored targets
// J_t = I + {(0,0), (1,0), (0,1), (1,1), (-1,1)}; the diagonal block is
// symmetrised and empty coarse dofs get a unit diagonal.  A workgroup takes a tile
// of kPtwTX x kPtwTY coarse nodes (a wave per tile row), so the fine rows that
// vertically adjacent coarse nodes share are read from L2 within the workgroup;
// tiles are dealt to the XCDs in contiguous runs (xcd_block), so a tile's
// neighbours above and below mostly share its L2 too.
constexpr int kPtwTX = 64, kPtwTY = 4;
template <int B, typename TM = double, typename TW = double>
__global__ void __launch_bounds__(kPtwTX * kPtwTY)
k_galerkin_ptw(const TM* __restrict__ P, const TW* __restrict__ W, size_t nn, int nxn, int nyn,
               int ncx, int ncy, double* __restrict__ Ac) {
  const size_t ncn = (size_t)ncx * ncy;
  const int ntx = (ncx + kPtwTX - 1) / kPtwTX;
  const unsigned tile = xcd_block();
  const int Ix = (int)(tile % ntx) * kPtwTX + (int)(threadIdx.x % kPtwTX);
  const int Iy = (int)(tile / ntx) * kPtwTY + (int)(threadIdx.x / kPtwTX);
  if (Ix >= ncx || Iy >= ncy) return;
  const size_t I = (size_t)Iy * ncx + Ix;
  const size_t nw = gw_size(nxn, nyn, ncx, ncy);
  const int tJx[5] = {Ix, Ix + 1, Ix, Ix + 1, Ix - 1};
  const int tJy[5] = {Iy, Iy, Iy + 1, Iy + 1, Iy + 1};
  double acc[5][3][3];
#pragma unroll
  for (int t = 0; t < 5; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[t][a][c] = 0.0;
  const int i0 = max(3 * Ix - 1, 0), i1 = min(agg_last(Ix, nxn, ncx) + 1, nxn - 1);
  const int j0 = max(3 * Iy - 1, 0), j1 = min(agg_last(Iy, nyn, ncy) + 1, nyn - 1);
  for (int j = j0; j <= j1; ++j) {
    const int sy = slot1(j, nyn, ncy, Iy);
    if (sy < 0) continue;
    const int ay = agg_of(j, ncy);
    for (int i = i0; i <= i1; ++i) {
      const int sx = slot1(i, nxn, ncx, Ix);
      if (sx < 0) continue;
      const int sl = sx + 2 * sy;
      const size_t n = (size_t)j * nxn + i;
      const size_t gi = gw_index(i, j, nxn, nyn, ncx, ncy);
      const int ax = agg_of(i, ncx);
      double PI[B][3];
#pragma unroll
      for (int r = 0; r < B; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) PI[r][c] = (double)P[pidx(B, nn, sl, n, r, c)];
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        const int qx = tJx[t] - ax + 1, qy = tJy[t] - ay + 1;
        if (tJx[t] < 0 || tJx[t] >= ncx || tJy[t] >= ncy || qx < 0 || qx > 2 || qy > 2) continue;
        const int q = qy * 3 + qx;
#pragma unroll
        for (int k = 0; k < B; ++k)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double wv = (double)W[(size_t)((q * B + k) * 3 + c) * nw + gi];
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[t][a][c] += PI[k][a] * wv;
          }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = a + 1; c < 3; ++c) {
      const double sv = 0.5 * (acc[0][a][c] + acc[0][c][a]);
      acc[0][a][c] = acc[0][c][a] = sv;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (acc[0][a][a] == 0.0) acc[0][a][a] = 1.0;
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    const bool valid = !(tJx[t] < 0 || tJx[t] >= ncx || tJy[t] >= ncy);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) Ac[aidx(3, ncn, t, I, a, c)] = valid ? acc[t][a][c] : 0.0;
  }
}

// ---- Q2 elements: unsmoothed first level --------------------------------------
// P = Ptent in slot 0 (the node's own aggregate), the other slots zero.
__global__ void k_tent_to_p(const double* __restrict__ Ptent, size_t nn, double* __restrict__ P) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  for (int sl = 0; sl < 4; ++sl)
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) P[pidx(2, nn, sl, n, r, c)] = sl == 0 ? Ptent[(size_t)(r * 3 + c) * nn + n] : 0.0;
}

// storage plane of the forward offset (ox, oy) of the Q2 25-point stencil
__device__ __forceinline__ int q2_plane(int ox, int oy) { return oy == 0 ? ox : 3 + (oy - 1) * 5 + (ox + 2); }

// Level-1 operator of Q2 elements: Ac = Ptent^T K2 Ptent with the tentative
// (unsmoothed) prolongator, one thread per coarse node.  Nodes of aggregates I and
// J couple through K2 only within two nodes of each other, so Ac is again a block
// 9-point stencil (5 stored 3x3 blocks); the diagonal block is symmetrised and
// empty coarse dofs get a unit diagonal, as in the smoothed Galerkin product.
__global__ void __launch_bounds__(kBlock)
k_galerkin_tent25(const double* __restrict__ K, const double* __restrict__ Ptent, size_t nn, int nxn, int nyn,
                  int ncx, int ncy, double* __restrict__ Ac) {
  const size_t ncn = (size_t)ncx * ncy;
  const size_t I = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= ncn) return;
  const int Ix = (int)(I % ncx), Iy = (int)(I / ncx);
#pragma unroll 1
  for (int t = 0; t < 5; ++t) {
    const int Jx = Ix + (t == 1 || t == 3 ? 1 : t == 4 ? -1 : 0);
    const int Jy = Iy + (t >= 2 ? 1 : 0);
    const bool valid = !(Jx < 0 || Jx >= ncx || Jy >= ncy);
    double acc[3][3];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) acc[a][c] = 0.0;
    if (valid) {
      for (int j = 3 * Iy; j <= agg_last(Iy, nyn, ncy); ++j)
        for (int i = 3 * Ix; i <= agg_last(Ix, nxn, ncx); ++i) {
          const size_t n = (size_t)j * nxn + i;
          double W[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
          for (int jj = max(3 * Jy, j - 2); jj <= min(agg_last(Jy, nyn, ncy), j + 2); ++jj)
            for (int ii = max(3 * Jx, i - 2); ii <= min(agg_last(Jx, nxn, ncx), i + 2); ++ii) {
              const int ox = ii - i, oy = jj - j;
              const size_t m = (size_t)jj * nxn + ii;
              double kb[2][2];
              if (oy > 0 || (oy == 0 && ox >= 0)) {
                const int pl = q2_plane(ox, oy);
                for (int r = 0; r < 2; ++r)
                  for (int c = 0; c < 2; ++c) kb[r][c] = K[aidx(2, nn, pl, n, r, c)];
              } else {
                const int pl = q2_plane(-ox, -oy);
                for (int r = 0; r < 2; ++r)
                  for (int c = 0; c < 2; ++c) kb[r][c] = K[aidx(2, nn, pl, m, c, r)];
              }
              for (int k = 0; k < 2; ++k)
                for (int c = 0; c < 3; ++c) {
                  const double pv = Ptent[(size_t)(k * 3 + c) * nn + m];
                  for (int r = 0; r < 2; ++r) W[r][c] += kb[r][k] * pv;
                }
            }
          for (int k = 0; k < 2; ++k)
            for (int c = 0; c < 3; ++c) {
              const double wv = W[k][c];
              for (int a = 0; a < 3; ++a) acc[a][c] += Ptent[(size_t)(k * 3 + a) * nn + n] * wv;
            }
        }
    }
    if (t == 0) {
      for (int a = 0; a < 3; ++a)
        for (int c = a + 1; c < 3; ++c) {
          const double sv = 0.5 * (acc[a][c] + acc[c][a]);
          acc[a][c] = acc[c][a] = sv;
        }
      for (int a = 0; a < 3; ++a)
        if (acc[a][a] == 0.0) acc[a][a] = 1.0;
    }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) Ac[aidx(3, ncn, t, I, a, c)] = valid ? acc[a][c] : 0.0;
  }
}

// ---- BF16 coarse storage: Jacobi-scaled operators --------------------------
// dsc = sqrt(diag(A)) per dof (point diagonal of the self block)
template <int B>
__global__ void k_diag_sqrt(const double* __restrict__ A, size_t nn, double* __restrict__ dsc) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  for (int r = 0; r < B; ++r) {
    const double d = A[aidx(B, nn, 0, n, r, r)];
    dsc[n * B + r] = d > 0.0 ? sqrt(d) : 1.0;
  }
}

__device__ __forceinline__ void store16(__hip_bfloat16* p, double v) { *p = __float2bfloat16((float)v); }
__device__ __forceinline__ void store16(_Float16* p, double v) { *p = (_Float16)(float)v; }
__device__ __forceinline__ void store16(float* p, double v) { *p = (float)v; }

// S = D^{-1/2} A D^{-1/2} stored in 16 bits (BF16 or FP16; same 5-block layout).
// One thread per stored entry, so consecutive lanes write consecutive values and
// every store covers whole lines (one thread per node, writing 2 bytes per lane at a
// stride of B*B entries, was measured slower).
// Entry k = (blk*nn + n)*B*B + r*B + c; the host guarantees 5*B*B*nn < 2^32.
template <int B, typename T16>
__global__ void __launch_bounds__(kBlock)
k_scale_to_16(const double* __restrict__ A, unsigned nn, int nxn, int nyn, const double* __restrict__ dsc,
              T16* __restrict__ S) {
  constexpr int DI[5] = {0, 1, 0, 1, -1};
  constexpr int DJ[5] = {0, 0, 1, 1, 1};
  const unsigned total = 5u * B * B * nn;
  for (unsigned k = (unsigned)xcd_block() * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
    const unsigned bn = k / (B * B);   // blk*nn + n
    const int rc = (int)(k - bn * (B * B));
    const int r = rc / B, c = rc - r * B;
    const int blk = (int)(bn / nn);
    const unsigned n = bn - (unsigned)blk * nn;
    const int j = (int)(n / (unsigned)nxn), i = (int)(n - (unsigned)j * nxn);
    int ii = i, jj = j;
#pragma unroll
    for (int b = 1; b < 5; ++b)
      if (blk == b) { ii = i + DI[b]; jj = j + DJ[b]; }
    const bool ok = ii >= 0 && jj >= 0 && ii < nxn && jj < nyn;
    const size_t m = ok ? (size_t)jj * nxn + ii : n;
    const double v = ok ? A[k] / (dsc[(size_t)n * B + r] * dsc[m * B + c]) : 0.0;
    store16(S + k, v);
  }
}
template <int B, typename T16>
void launch_scale_to_16(hipStream_t s, const Level& L, T16* S) {
  const size_t total = (size_t)5 * B * B * L.nn;
  if (total >= ((size_t)1 << 32)) throw Error(VP_EINVAL, "operator too large for the 16-bit scaling kernel");
  hipLaunchKernelGGL((k_scale_to_16<B, T16>), dim3(grid_for(total)), dim3(kBlock), 0, s, (const double*)L.A64,
                     (unsigned)L.nn, L.nxn, L.nyn, (const double*)L.dsc64, S);
  VP_LAUNCH_CHECK();
}

// P^ = diag(dsc_f) P diag(1/dsc_c) in FP32 (dsc_f = null: no row scaling, finest level)
template <int B, typename TP = double>
__global__ void k_scale_p(const TP* __restrict__ P, size_t nn, int nxn, int nyn, int ncx, int ncy,
                          const double* __restrict__ dsc_f, const double* __restrict__ dsc_c,
                          float* __restrict__ Ps) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  const int ax[2] = {agg_of(i, ncx), agg_other(i, nxn, ncx)};
  const int ay[2] = {agg_of(j, ncy), agg_other(j, nyn, ncy)};
  // every load is unconditional (an absent slot reads coarse node 0 and stores 0),
  // so a thread's loads are all in flight at once
  double fr[B];
#pragma unroll
  for (int r = 0; r < B; ++r) fr[r] = dsc_f ? dsc_f[n * B + r] : 1.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int Jx = ax[s & 1], Jy = ay[s >> 1];
    const bool ok = Jx >= 0 && Jy >= 0;
    const size_t J = ok ? (size_t)Jy * ncx + Jx : 0;
    double dc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dc[c] = dsc_c[J * 3 + c];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const size_t k = pidx(B, nn, s, n, r, c);
        const float v = (float)(fr[r] * (double)P[k] / dc[c]);
        Ps[k] = ok ? v : 0.0f;
      }
  }
}

// y = (float)(x / dsc) and y = (double)(x) / dsc: the V-cycle's input and output
// in the Jacobi-scaled variables of a BF16 finest level
__global__ void k_scale_cast_df(const double* __restrict__ x, const double* __restrict__ dsc, float* __restrict__ y,
                                size_t n) {
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = (float)(x[e] / dsc[e]);
}
__global__ void k_scale_cast_fd(const float* __restrict__ x, const double* __restrict__ dsc, double* __restrict__ y,
                                size_t n) {
  for (size_t e = (size_t)xcd_block() * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    y[e] = (double)x[e] / dsc[e];
}

// (D^{1/2} A^{-1} D^{1/2}) of the coarsest level in FP32 (inverse of the scaled operator)
__global__ void k_scale_dense(const double* __restrict__ M, int nd, const double* __restrict__ dsc,
                              float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nd * nd) return;
  const int r = (int)(e / nd), c = (int)(e % nd);
  out[e] = (float)(dsc[r] * M[e] * dsc[c]);
}

// Dense matrix (row-major nd x nd, nd = B*nn) of a stencil level.  Zero-filled by caller.
template <int B>
__global__ void k_to_dense(const double* __restrict__ A, size_t nn, int nxn, int nyn, double* __restrict__ M) {
  const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  const size_t nd = (size_t)B * nn;
  for (int d = 0; d < 9; ++d) {
    const int ii = i + kDI[d], jj = j + kDJ[d];
    if (ii < 0 || jj < 0 || ii >= nxn || jj >= nyn) continue;
    double blk[B][B];
    load_block<B>(A, nn, nxn, i, j, d, blk);
    const size_t m = (size_t)jj * nxn + ii;
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) M[(n * B + r) * nd + m * B + c] = blk[r][c];
  }
}

// In-place Gauss-Jordan inversion of an SPD matrix (no pivoting needed), one workgroup.
__global__ void __launch_bounds__(1024) k_gauss_jordan(double* __restrict__ M, int nd) {
  __shared__ double rowk[1024];
  __shared__ double colk[1024];
  for (int k = 0; k < nd; ++k) {
    const double piv = M[(size_t)k * nd + k];
    const double ip = piv != 0.0 ? 1.0 / piv : 0.0;
    for (int t = threadIdx.x; t < nd; t += blockDim.x) {
      rowk[t] = M[(size_t)k * nd + t];
      colk[t] = M[(size_t)t * nd + k];
    }
    __syncthreads();
    for (size_t e = threadIdx.x; e < (size_t)nd * nd; e += blockDim.x) {
      const int r = (int)(e / nd), c = (int)(e % nd);
      double v;
      if (r == k && c == k) v = ip;
      else if (r == k) v = rowk[c] * ip;
      else if (c == k) v = -colk[r] * ip;
      else v = M[e] - colk[r] * rowk[c] * ip;
      M[e] = v;
    }
    __syncthreads();
  }
}

// Same inversion with the whole matrix resident in LDS (nd <= kLdsGJ; gfx950 has
// 160 KB of LDS per CU): one global read and write instead of nd passes.
constexpr int kLdsGJ = 140;
__global__ void __launch_bounds__(1024) k_gauss_jordan_lds(double* __restrict__ M, int nd) {
  __shared__ double S[kLdsGJ * kLdsGJ];
  __shared__ double rowk[kLdsGJ];
  __shared__ double colk[kLdsGJ];
  const int n2 = nd * nd;
  for (int e = threadIdx.x; e < n2; e += blockDim.x) S[e] = M[e];
  __syncthreads();
  for (int k = 0; k < nd; ++k) {
    const double piv = S[k * nd + k];
    const double ip = piv != 0.0 ? 1.0 / piv : 0.0;
    for (int t = threadIdx.x; t < nd; t += blockDim.x) {
      rowk[t] = S[k * nd + t];
      colk[t] = S[t * nd + k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n2; e += blockDim.x) {
      const int r = e / nd, c = e % nd;
      double v;
      if (r == k && c == k) v = ip;
      else if (r == k) v = rowk[c] * ip;
      else if (c == k) v = -colk[r] * ip;
      else v = S[e] - colk[r] * rowk[c] * ip;
      S[e] = v;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n2; e += blockDim.x) M[e] = S[e];
}

template <typename TM, typename TV>
__global__ void k_dense_apply(const TM* __restrict__ M, int nd, const TV* __restrict__ b, TV* __restrict__ x) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nd) row_dense_apply(M, nd, b, x, r);
}

// d = (TD)s, four entries per step with one aligned vector load and store each (the
// buffers are allocation bases, so 4-entry groups are aligned), the last n % 4 singly
template <typename T>
struct alignas(4 * sizeof(T)) Vec4 {
  T v[4];
};
template <typename TS, typename TD>
__global__ void k_convert(const TS* __restrict__ s, TD* __restrict__ d, size_t n) {
  const size_t n4 = n / 4, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += stride) {
    const Vec4<TS> a = reinterpret_cast<const Vec4<TS>*>(s)[e];
    Vec4<TD> b;
#pragma unroll
    for (int k = 0; k < 4; ++k) b.v[k] = (TD)a.v[k];
    reinterpret_cast<Vec4<TD>*>(d)[e] = b;
  }
  for (size_t e = 4 * n4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) d[e] = (TD)s[e];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  VP_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
  return static_cast<T*>(p);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void free_vectors(Level& L) {
  void** v[7] = {&L.x, &L.b, &L.r, &L.d0, &L.d1, &L.r2, &L.x2};
  for (auto pp : v) {
    if (*pp) (void)hipFree(*pp);
    *pp = nullptr;
  }
}

template <typename TS, typename TD>
void convert(hipStream_t s, const TS* src, TD* dst, size_t n) {
  if ((reinterpret_cast<uintptr_t>(src) % (4 * sizeof(TS))) || (reinterpret_cast<uintptr_t>(dst) % (4 * sizeof(TD))))
    throw Error(VP_EINVAL, "convert: buffers not aligned to 4 entries");
  hipLaunchKernelGGL((k_convert<TS, TD>), dim3(std::min<size_t>((n / 4 + 255) / 256, 4096) + 1), dim3(256), 0, s,
                     src, dst, n);
  VP_LAUNCH_CHECK();
}

}  // namespace

// The smoothed prolongator of a level in FP64 (12*B*nn values): the FP64 one, or
// the FP32 one widened where only that exists (the FP32 modes).
void amg_export_p(vp_ctx c, int level, double* P) {
  const Level& L = c->lev[level];
  const size_t np = (size_t)12 * L.B * L.nn;
  if (L.p64_stale)
    launch_cast(c->stream, (const float*)(c->amg_prec == VP_PREC_FP32_BF16COARSE ? L.P32u : L.P32), P, np);
  else
    VP_HIP(hipMemcpyAsync(P, L.P64, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
}

void amg_free(vp_ctx c) {
  c->a32_assembled = false;
  for (int l = 0; l < kMaxLevels; ++l) {
    Level& L = c->lev[l];
    if (l > 0) dfree(L.A64);
    dfree(L.A32);
    dfree(L.Ptent);
    dfree(L.P64);
    dfree(L.P32);
    dfree(L.P32u);
    dfree(L.Ph);
    dfree(L.Bnull);
    dfree(L.lmax);
    dfree(L.pv0);
    dfree(L.pv1);
    dfree(L.pnrm);
    dfree(L.Ainv64);
    dfree(L.Ainv32);
    dfree(L.Abf);
    dfree(L.Ah);
    dfree(L.dsc64);
    free_vectors(L);
    L = Level();
  }
  dfree(c->dense);
  dfree(c->gal_work);
  dfree(c->lmax_all);
  c->nlev = 0;
  c->amg_struct = false;
  c->amg_ready = false;
}

// Build the level structure (geometry only: grids, tentative prolongators,
// near-null spaces).  The finest operator is the context's assembled K.
void amg_build_structure(vp_ctx c, double* K, int max_coarse) {
  amg_free(c);
  c->max_coarse = max_coarse;
  int nxn = c->ec.nxn, nyn = c->ec.nyn, B = 2;
  int l = 0;
  for (;; ++l) {
    Level& L = c->lev[l];
    L.nxn = nxn; L.nyn = nyn; L.B = B;
    L.nn = (size_t)nxn * nyn;
    L.A64 = (l == 0) ? K : dalloc<double>((size_t)5 * B * B * L.nn);
    L.lmax = dalloc<double>(1);
    const bool last = (size_t)B * L.nn <= (size_t)max_coarse || nxn < 6 || nyn < 6 || l == kMaxLevels - 1;
    if (last) break;
    L.ncx = nxn / 3;
    L.ncy = nyn / 3;
    L.Ptent = dalloc<double>((size_t)B * 3 * L.nn);
    L.P64 = dalloc<double>((size_t)4 * B * 3 * L.nn);
    Level& Nx = c->lev[l + 1];
    const size_t ncn = (size_t)L.ncx * L.ncy;
    Nx.Bnull = dalloc<double>(9 * ncn);
    const unsigned g = (unsigned)((ncn + 127) / 128);
    if (B == 2)
      hipLaunchKernelGGL(k_tentative<2>, dim3(g), dim3(128), 0, c->stream, nxn, nyn, L.ncx, L.ncy,
                         (const double*)nullptr, L.Ptent, Nx.Bnull);
    else
      hipLaunchKernelGGL(k_tentative<3>, dim3(g), dim3(128), 0, c->stream, nxn, nyn, L.ncx, L.ncy,
                         (const double*)L.Bnull, L.Ptent, Nx.Bnull);
    VP_LAUNCH_CHECK();
    nxn = L.ncx;
    nyn = L.ncy;
    B = 3;
  }
  c->nlev = l + 1;
  Level& C = c->lev[c->nlev - 1];
  const size_t nd = (size_t)C.B * C.nn;
  if (nd > 1024) throw Error(VP_EINVAL, "coarsest level too large for the dense solve");
  C.Ainv64 = dalloc<double>(nd * nd);
  c->amg_struct = true;
}

namespace {

template <typename TV>
void alloc_vectors(vp_ctx c) {
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    free_vectors(L);
    const size_t n = (size_t)L.B * L.nn;
    L.x = dalloc<TV>(n);
    L.b = dalloc<TV>(n);
    L.r = dalloc<TV>(n);
    L.d0 = dalloc<TV>(n);
    L.d1 = dalloc<TV>(n);
    L.r2 = dalloc<TV>(n);   // paired sweeps (finest level; coarse levels in FP32)
    L.x2 = dalloc<TV>(n);
  }
}

}  // namespace

// BF16-coarse mode: level 0 keeps an FP32 operator; every coarser level l stores
// S_l = D_l^{-1/2} A_l D_l^{-1/2} in BF16 and the V-cycle works there in the
// scaled variables, with prolongators P^_l = D_l^{1/2} P_l D_{l+1}^{-1/2} (FP32;
// D_0 = I) and the coarsest inverse D^{1/2} A^{-1} D^{1/2} (FP32).
// Reduced-precision copies of the operators for the mixed modes.  finest: 0 FP32
// (unscaled), 1 BF16 Jacobi-scaled, 2 FP16 Jacobi-scaled; coarse levels are
// Jacobi-scaled in BF16 (coarse 0), FP16 (1) or FP32 (2).
void bf16_copies(vp_ctx c, hipStream_t s, int finest, int coarse) {
  const bool coarse_fp16 = coarse == 1;
  const bool finest_scaled = finest != 0;
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    const size_t na = (size_t)5 * L.B * L.B * L.nn;
    const unsigned g = (unsigned)((L.nn + 255) / 256);
    if (l == 0 && finest == 0) continue;   // FP32 finest operator made first (Q2: the finest level runs on K2_32)
    if (!L.dsc64) L.dsc64 = dalloc<double>((size_t)L.B * L.nn);
    if (L.B == 2)
      hipLaunchKernelGGL(k_diag_sqrt<2>, dim3(g), dim3(256), 0, s, L.A64, L.nn, L.dsc64);
    else
      hipLaunchKernelGGL(k_diag_sqrt<3>, dim3(g), dim3(256), 0, s, L.A64, L.nn, L.dsc64);
    VP_LAUNCH_CHECK();
    if (l > 0 && coarse == 2) {
      if (!L.A32) L.A32 = dalloc<float>(na);
      if (L.B == 2)
        launch_scale_to_16<2>(s, L, L.A32);
      else
        launch_scale_to_16<3>(s, L, L.A32);
    } else if ((l == 0 && finest == 2) || (l > 0 && coarse_fp16)) {
      if (!L.Ah) L.Ah = dalloc<_Float16>(na);
      if (L.B == 2)
        launch_scale_to_16<2>(s, L, L.Ah);
      else
        launch_scale_to_16<3>(s, L, L.Ah);
    } else {
      if (!L.Abf) L.Abf = dalloc<__hip_bfloat16>(na);
      if (L.B == 2)
        launch_scale_to_16<2>(s, L, L.Abf);
      else
        launch_scale_to_16<3>(s, L, L.Abf);
    }
    VP_LAUNCH_CHECK();
  }
  for (int l = 0; l + 1 < c->nlev; ++l) {
    Level& L = c->lev[l];
    Level& N = c->lev[l + 1];
    const size_t np = (size_t)4 * L.B * 3 * L.nn;
    if (!L.P32) L.P32 = dalloc<float>(np);
    const unsigned g = (unsigned)((L.nn + 255) / 256);
    if (L.p64_stale && L.B == 2)   // the FP32 + BF16-coarse mode's prolongators exist in FP32 only
      hipLaunchKernelGGL((k_scale_p<2, float>), dim3(g), dim3(256), 0, s, (const float*)L.P32u, L.nn, L.nxn, L.nyn,
                         L.ncx, L.ncy, (const double*)(finest_scaled ? L.dsc64 : nullptr), (const double*)N.dsc64,
                         L.P32);
    else if (L.p64_stale)
      hipLaunchKernelGGL((k_scale_p<3, float>), dim3(g), dim3(256), 0, s, (const float*)L.P32u, L.nn, L.nxn, L.nyn,
                         L.ncx, L.ncy, (const double*)L.dsc64, (const double*)N.dsc64, L.P32);
    else if (L.B == 2)
      hipLaunchKernelGGL(k_scale_p<2>, dim3(g), dim3(256), 0, s, L.P64, L.nn, L.nxn, L.nyn, L.ncx, L.ncy,
                         (const double*)(finest_scaled ? L.dsc64 : nullptr), (const double*)N.dsc64, L.P32);
    else
      hipLaunchKernelGGL(k_scale_p<3>, dim3(g), dim3(256), 0, s, L.P64, L.nn, L.nxn, L.nyn, L.ncx, L.ncy,
                         (const double*)L.dsc64, (const double*)N.dsc64, L.P32);
    VP_LAUNCH_CHECK();
    if (l == 0 && finest == 2) {   // the finest transfers read the scaled prolongator in FP16
      if (!L.Ph) L.Ph = dalloc<_Float16>(np);
      convert(s, (const float*)L.P32, L.Ph, np);
    }
  }
  Level& C = c->lev[c->nlev - 1];
  const int nd = C.B * (int)C.nn;
  if (!C.Ainv32) C.Ainv32 = dalloc<float>((size_t)nd * nd);
  if (c->nlev == 1 && !finest_scaled) {
    convert(s, C.Ainv64, C.Ainv32, (size_t)nd * nd);
  } else {
    hipLaunchKernelGGL(k_scale_dense, dim3((unsigned)(((size_t)nd * nd + 255) / 256)), dim3(256), 0, s, C.Ainv64, nd,
                       (const double*)C.dsc64, C.Ainv32);
    VP_LAUNCH_CHECK();
  }
}

// Scratch for the Galerkin products: the largest 9*3*B*gw_size over the levels
// that have a coarser level (allocated once per hierarchy).
double* galerkin_work(vp_ctx c) {
  if (!c->gal_work) {
    size_t mx = 0;
    for (int l = 0; l + 1 < c->nlev; ++l) {
      const Level& L = c->lev[l];
      mx = std::max(mx, (size_t)27 * L.B * gw_size(L.nxn, L.nyn, L.ncx, L.ncy));
    }
    c->gal_work = dalloc<double>(std::max<size_t>(mx, 1));
  }
  return c->gal_work;
}

// Restart the spectral estimates from the fixed start vector at the next setup.
void amg_reset_estimates(vp_ctx c) {
  for (int l = 0; l < kMaxLevels; ++l) c->lev[l].pv_warm = false;
  c->pq_warm = false;
}

// Numeric setup on the current finest operator.
// First level handled by the single-workgroup tail kernel, or -1 (also with
// VP_AMG_VAR_NO_TAIL, which keeps one launch per sweep everywhere).
int tail_start(vp_ctx c) {
  if (c->amg_variant & VP_AMG_VAR_NO_TAIL) return -1;
  if (c->cheb_degree > kTailDegree) return -1;
  for (int l = 1; l + 1 < c->nlev; ++l)
    if (c->lev[l].B == 3 && c->lev[l].nn <= (size_t)kTailNodes && c->nlev - l <= kTailLevels) return l;
  return -1;
}

// Q2 elements: the V-cycle smooths the finest level with the 25-point Q2
// operator itself (level 1 is Ptent^T K2 Ptent), so its Chebyshev interval
// needs lmax(D^{-1} K2): Gershgorin bound, then the power
// iteration warm started across setups.  FP32 V-cycles get an FP32 copy.
void q2_smoother_setup(vp_ctx c, int precision) {
  hipStream_t s = c->stream;
  const size_t nn = c->nn, nd = 2 * nn;
  const int nxn = c->ec.nxn, nyn = c->ec.nyn;
  const unsigned g = (unsigned)((nn + kBlock - 1) / kBlock);
  if (!c->lmax_q2) {
    c->lmax_q2 = dalloc<double>(1);
    c->pq0 = dalloc<double>(nd);
    c->pq1 = dalloc<double>(nd);
    c->pqn = dalloc<double>(2);
  }
  hipLaunchKernelGGL(k_gershgorin25, dim3(g), dim3(kBlock), 0, s, c->K2, nn, nxn, nyn, c->partials);
  VP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_finish_max, dim3(1), dim3(512), 0, s, c->partials, (int)g, c->lmax_q2);
  VP_LAUNCH_CHECK();
  int its = c->power_its_warm;
  if (!c->pq_warm) {
    hipLaunchKernelGGL(k_power_init, dim3(1024), dim3(256), 0, s, c->pq0, nd);
    VP_LAUNCH_CHECK();
    its = c->power_its_cold;
    c->pq_warm = true;
  }
  launch_dot(s, c->pq0, c->pq0, nd, c->partials);
  launch_finish_sum(s, c->partials, kRedBlocks, 1, c->pqn);
  for (int k = 0; k < its; ++k) {
    double* xin = (k & 1) ? c->pq1 : c->pq0;
    double* yout = (k & 1) ? c->pq0 : c->pq1;
    hipLaunchKernelGGL((k_power_step<2, 1>), dim3(g), dim3(kBlock), 0, s, c->K2, nn, nxn, nyn, xin,
                       c->pqn + (k & 1), yout, c->partials);
    VP_LAUNCH_CHECK();
    launch_finish_sum(s, c->partials, (int)g, 1, c->pqn + ((k + 1) & 1));
  }
  hipLaunchKernelGGL(k_power_final, dim3(1), dim3(64), 0, s, c->pqn + (its & 1), c->power_factor, c->lmax_q2);
  VP_LAUNCH_CHECK();
  if (its & 1) std::swap(c->pq0, c->pq1);
  if (precision != VP_PREC_FP64) {
    const size_t na = (size_t)52 * nn;
    if (!c->K2_32) c->K2_32 = dalloc<float>(na);
    convert(s, c->K2, c->K2_32, na);
  }
}

void amg_setup_numeric(vp_ctx c, int precision, double omega_scale) {
  if (!c->amg_struct) throw Error(VP_ESTATE, "AMG structure missing");
  hipStream_t s = c->stream;
  const bool q2u = c->order == 2;
  if (c->order == 2) q2_smoother_setup(c, precision);
  // Modes whose V-cycle smooths with FP32 (or BF16) operators build the hierarchy
  // from FP32 copies: each level's operator is copied to FP32 as soon as it exists,
  // and its spectral bounds, smoothed prolongator (kept in FP32 only) and Galerkin
  // product read that copy (half the bytes).  The coarse operators themselves are
  // summed in FP64 and kept in FP64 for the next level's copy and the scalings.
  const bool fine32 = c->order == 1 && (precision == VP_PREC_FP32 || precision == VP_PREC_FP32_BF16COARSE);
  for (int l = 0; l < c->nlev; ++l) c->lev[l].p64_stale = false;
  if (!fine32) c->a32_assembled = false;   // other modes may overwrite the finest FP32 buffer
  for (int l = 0; l < c->nlev; ++l) {
    Level& L = c->lev[l];
    const unsigned g = (unsigned)((L.nn + kBlock - 1) / kBlock);
    if (l == 0 && q2u) {
      // Q2 elements: the finest level is smoothed with K2 (its bound from
      // q2_smoother_setup) and restricted with the tentative prolongator
      VP_HIP(hipMemcpyAsync(L.lmax, c->lmax_q2, sizeof(double), hipMemcpyDeviceToDevice, s));
      if (c->nlev == 1) break;
      hipLaunchKernelGGL(k_tent_to_p, dim3(g), dim3(kBlock), 0, s, L.Ptent, L.nn, L.P64);
      VP_LAUNCH_CHECK();
      Level& N = c->lev[1];
      hipLaunchKernelGGL(k_galerkin_tent25, dim3((unsigned)((N.nn + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                         (const double*)c->K2, (const double*)L.Ptent, L.nn, L.nxn, L.nyn, L.ncx, L.ncy, N.A64);
      VP_LAUNCH_CHECK();
      continue;
    }
    const float* A32 = nullptr;
    if (fine32) {
      const size_t na = (size_t)5 * L.B * L.B * L.nn;
      if (!L.A32) L.A32 = dalloc<float>(na);
      if (!(l == 0 && c->a32_assembled)) convert(s, L.A64, L.A32, na);   // else written by the assembly
      A32 = L.A32;
    }
    if (A32 && L.B == 2)
      hipLaunchKernelGGL((k_gershgorin<2, float>), dim3(g), dim3(kBlock), 0, s, A32, L.nn, L.nxn, L.nyn, c->partials);
    else if (A32)
      hipLaunchKernelGGL((k_gershgorin<3, float>), dim3(g), dim3(kBlock), 0, s, A32, L.nn, L.nxn, L.nyn, c->partials);
    else if (L.B == 2)
      hipLaunchKernelGGL(k_gershgorin<2>, dim3(g), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, c->partials);
    else
      hipLaunchKernelGGL(k_gershgorin<3>, dim3(g), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, c->partials);
    VP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finish_max, dim3(1), dim3(512), 0, s, c->partials, (int)g, L.lmax);
    VP_LAUNCH_CHECK();
    if (l == c->nlev - 1) break;
    // power iteration on D^{-1} A, warm started from the previous setup's vector
    {
      const size_t nd = (size_t)L.B * L.nn;
      int its = c->power_its_warm;
      if (!L.pv0) {
        L.pv0 = dalloc<double>(nd);
        L.pv1 = dalloc<double>(nd);
        L.pnrm = dalloc<double>(2);
      }
      if (!L.pv_warm) {
        hipLaunchKernelGGL(k_power_init, dim3(1024), dim3(256), 0, s, L.pv0, nd);
        VP_LAUNCH_CHECK();
        its = c->power_its_cold;
        L.pv_warm = true;
      }
      // |x|^2 of the start vector
      launch_dot(s, L.pv0, L.pv0, nd, c->partials);
      launch_finish_sum(s, c->partials, kRedBlocks, 1, L.pnrm);
      for (int k = 0; k < its; ++k) {
        double* xin = (k & 1) ? L.pv1 : L.pv0;
        double* yout = (k & 1) ? L.pv0 : L.pv1;
        const double* nrm = L.pnrm + (k & 1);
        if (A32 && L.B == 2)
          hipLaunchKernelGGL((k_power_step<2, 0, float>), dim3(g), dim3(kBlock), 0, s, A32, L.nn, L.nxn, L.nyn, xin,
                             nrm, yout, c->partials);
        else if (A32)
          hipLaunchKernelGGL((k_power_step<3, 0, float>), dim3(g), dim3(kBlock), 0, s, A32, L.nn, L.nxn, L.nyn, xin,
                             nrm, yout, c->partials);
        else if (L.B == 2)
          hipLaunchKernelGGL(k_power_step<2>, dim3(g), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, xin, nrm, yout,
                             c->partials);
        else
          hipLaunchKernelGGL(k_power_step<3>, dim3(g), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, xin, nrm, yout,
                             c->partials);
        VP_LAUNCH_CHECK();
        launch_finish_sum(s, c->partials, (int)g, 1, L.pnrm + ((k + 1) & 1));
      }
      hipLaunchKernelGGL(k_power_final, dim3(1), dim3(64), 0, s, L.pnrm + (its & 1), c->power_factor, L.lmax);
      VP_LAUNCH_CHECK();
      if (its & 1) std::swap(L.pv0, L.pv1);  // keep the latest iterate in pv0
    }
    // The FP32 mode's FP32 prolongator is written by the smoothing itself.  In the
    // FP32 modes only the FP32 prolongator is made, from the FP32 operator: the
    // V-cycle and the Galerkin product read nothing else (the BF16-coarse mode keeps
    // it unscaled in P32u; its scaled copy for the V-cycle is made once the coarse
    // diagonal is known).
    float* p32 = nullptr;
    float*& pdst = A32 && precision == VP_PREC_FP32_BF16COARSE ? L.P32u : L.P32;
    if (precision == VP_PREC_FP32 || A32) {
      if (!pdst) pdst = dalloc<float>((size_t)4 * L.B * 3 * L.nn);
      p32 = pdst;
    }
    L.p64_stale = A32 != nullptr;
    if (A32 && L.B == 2)
      hipLaunchKernelGGL((k_smooth_p<2, float>), dim3(g), dim3(kBlock), 0, s, A32, L.nn, L.nxn, L.nyn, L.ncx, L.ncy,
                         L.Ptent, L.lmax, omega_scale, (double*)nullptr, p32);
    else if (A32)
      hipLaunchKernelGGL((k_smooth_p<3, float>), dim3(g), dim3(kBlock), 0, s, A32, L.nn, L.nxn, L.nyn, L.ncx, L.ncy,
                         L.Ptent, L.lmax, omega_scale, (double*)nullptr, p32);
    else if (L.B == 2)
      hipLaunchKernelGGL(k_smooth_p<2>, dim3(g), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, L.ncx, L.ncy,
                         L.Ptent, L.lmax, omega_scale, L.P64, p32);
    else
      hipLaunchKernelGGL(k_smooth_p<3>, dim3(g), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, L.ncx, L.ncy,
                         L.Ptent, L.lmax, omega_scale, L.P64, p32);
    VP_LAUNCH_CHECK();
    Level& N = c->lev[l + 1];
    const size_t ptw_tiles = (size_t)((L.ncx + kPtwTX - 1) / kPtwTX) * ((L.ncy + kPtwTY - 1) / kPtwTY);
    const unsigned gc = grid_for(ptw_tiles, 1);   // one workgroup per tile, a multiple of 8
    double* Wap = galerkin_work(c);
    float* W32 = reinterpret_cast<float*>(Wap);
    if (A32 && L.B == 2) {
      launch_galerkin_ap_w<2>(s, L, A32, (const float*)p32, W32);
      hipLaunchKernelGGL((k_galerkin_ptw<2, float, float>), dim3(gc), dim3(kPtwTX * kPtwTY), 0, s,
                         (const float*)p32, (const float*)W32, L.nn, L.nxn, L.nyn, L.ncx, L.ncy, N.A64);
    } else if (A32) {
      launch_galerkin_ap_w<3>(s, L, A32, (const float*)p32, W32);
      hipLaunchKernelGGL((k_galerkin_ptw<3, float, float>), dim3(gc), dim3(kPtwTX * kPtwTY), 0, s,
                         (const float*)p32, (const float*)W32, L.nn, L.nxn, L.nyn, L.ncx, L.ncy, N.A64);
    } else if (L.B == 2) {
      hipLaunchKernelGGL(k_galerkin_ap<2>, dim3(grid_for(L.nn)), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, L.ncx,
                         L.ncy, L.P64, Wap);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_galerkin_ptw<2>, dim3(gc), dim3(kPtwTX * kPtwTY), 0, s, L.P64, Wap, L.nn, L.nxn, L.nyn, L.ncx,
                         L.ncy, N.A64);
    } else {
      hipLaunchKernelGGL(k_galerkin_ap<3>, dim3(grid_for(L.nn)), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, L.ncx,
                         L.ncy, L.P64, Wap);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_galerkin_ptw<3>, dim3(gc), dim3(kPtwTX * kPtwTY), 0, s, L.P64, Wap, L.nn, L.nxn, L.nyn, L.ncx,
                         L.ncy, N.A64);
    }
    VP_LAUNCH_CHECK();
  }
  // coarsest: dense inverse
  Level& C = c->lev[c->nlev - 1];
  const int nd = C.B * (int)C.nn;
  VP_HIP(hipMemsetAsync(C.Ainv64, 0, (size_t)nd * nd * sizeof(double), s));
  const unsigned gd = (unsigned)((C.nn + 127) / 128);
  if (C.B == 2)
    hipLaunchKernelGGL(k_to_dense<2>, dim3(gd), dim3(128), 0, s, C.A64, C.nn, C.nxn, C.nyn, C.Ainv64);
  else
    hipLaunchKernelGGL(k_to_dense<3>, dim3(gd), dim3(128), 0, s, C.A64, C.nn, C.nxn, C.nyn, C.Ainv64);
  VP_LAUNCH_CHECK();
  if (nd <= kLdsGJ) hipLaunchKernelGGL(k_gauss_jordan_lds, dim3(1), dim3(1024), 0, s, C.Ainv64, nd);
  else hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, s, C.Ainv64, nd);
  VP_LAUNCH_CHECK();
  // reduced-precision copies
  if (precision == VP_PREC_FP32_BF16COARSE || precision == VP_PREC_BF16 || precision == VP_PREC_FP16_BF16COARSE ||
      precision == VP_PREC_FP16 || precision == VP_PREC_FP16_FP32COARSE) {
    const int finest = precision == VP_PREC_BF16 ? 1 : precision == VP_PREC_FP32_BF16COARSE ? 0 : 2;
    const int coarse = precision == VP_PREC_FP16 ? 1 : precision == VP_PREC_FP16_FP32COARSE ? 2 : 0;
    bf16_copies(c, s, finest, coarse);
    if (precision == VP_PREC_FP16_FP32COARSE) {   // FP32 scaled finest operator for the post-correction residual
      Level& L0 = c->lev[0];
      const size_t na0 = (size_t)20 * L0.nn;
      if (!L0.A32) L0.A32 = dalloc<float>(na0);
      launch_scale_to_16<2>(s, L0, L0.A32);
      VP_LAUNCH_CHECK();
    }
  } else if (precision != VP_PREC_FP64) {
    for (int l = 0; l < c->nlev; ++l) {
      Level& L = c->lev[l];
      const size_t na = (size_t)5 * L.B * L.B * L.nn;
      // Q1: every FP32 operator was made in the level loop; Q2: the coarse ones here
      // (the finest level runs on K2_32)
      if (l > 0 && c->order == 2) {
        if (!L.A32) L.A32 = dalloc<float>(na);
        convert(s, L.A64, L.A32, na);
      }
      if (L.P64 && (c->order == 2 && l == 0)) {   // smoothed prolongators got theirs from k_smooth_p
        const size_t np = (size_t)4 * L.B * 3 * L.nn;
        if (!L.P32) L.P32 = dalloc<float>(np);
        convert(s, L.P64, L.P32, np);
      }
      if (L.Ainv64) {
        if (!L.Ainv32) L.Ainv32 = dalloc<float>((size_t)nd * nd);
        convert(s, L.Ainv64, L.Ainv32, (size_t)nd * nd);
      }
    }
  }
  const bool vec64 = precision == VP_PREC_FP64;
  if (c->lev[0].x == nullptr || vec64 != c->sa_vec64) {
    if (vec64) alloc_vectors<double>(c);
    else alloc_vectors<float>(c);
    c->sa_vec64 = vec64;
  }
  c->amg_prec = precision;
  // spectral bounds to the host: gathered on the device, one copy and one
  // synchronisation per setup
  {
    ScalarPtrs g{};
    g.n = c->nlev + (c->order == 2 ? 1 : 0);
    for (int l = 0; l < c->nlev; ++l) g.p[l] = c->lev[l].lmax;
    if (c->order == 2) g.p[c->nlev] = c->lmax_q2;
    if (!c->lmax_all) c->lmax_all = dalloc<double>(kMaxLevels + 1);
    hipLaunchKernelGGL(k_gather_scalars, dim3(1), dim3(64), 0, s, g, c->lmax_all);
    VP_LAUNCH_CHECK();
    VP_HIP(hipMemcpyAsync(c->hscal, c->lmax_all, g.n * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  VP_HIP(hipStreamSynchronize(s));
  for (int l = 0; l < c->nlev + (c->order == 2 ? 1 : 0); ++l)
    if (!(c->hscal[l] > 0.0) || !std::isfinite(c->hscal[l]))
      throw Error(VP_ENONFINITE, "AMG setup: non-finite or non-positive spectral bound");
  for (int l = 0; l < c->nlev; ++l) c->lev[l].lmax_h = c->hscal[l];
  if (c->order == 2) c->lmax_q2_h = c->hscal[c->nlev];
  c->tail_level = tail_start(c);
  {
    c->pair_sweeps = !(c->amg_variant & VP_AMG_VAR_NO_PAIRS);
    c->tail_lds = !(c->amg_variant & VP_AMG_VAR_NO_TAIL_LDS);
    c->ph_transfers = !(c->amg_variant & VP_AMG_VAR_NO_P16) && c->lev[0].Ph != nullptr &&
                      (precision == VP_PREC_FP16_BF16COARSE || precision == VP_PREC_FP16 ||
                       precision == VP_PREC_FP16_FP32COARSE);
  }
  c->amg_ready = true;
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------
namespace {

template <int B, typename TM, typename TV, int ST = 0>
void sten_resid(vp_ctx c, int l, const Level& L, const TM* A, const TV* x, const TV* b, TV* r) {
  const int pr = l == 0 ? prof_begin(c, VP_KID_STEN_RESID0) : -1;
  hipLaunchKernelGGL((k_sten_resid<B, TM, TV, ST>), dim3(grid_for(L.nn)), dim3(kBlock), 0, c->stream, A, L.nn,
                     L.nxn, L.nyn, x, b, r);
  VP_LAUNCH_CHECK();
  prof_end(c, pr);
}

// Chebyshev smoothing of degree `degree` on [lmax/ratio, lmax] with the block
// diagonal as preconditioner.  pre: x = 0 on entry and r = b - A x on exit (for
// the restriction); otherwise x is updated in place from the residual of b.
// ST = 1 with lmax_h: the finest level of Q2 elements (25-point stencil, its own
// spectral bound).
template <int B, typename TM, typename TV, int ST = 0>
void smooth(vp_ctx c, int l, const Level& L, const TM* A, const TV* b, TV* x, bool pre, int degree,
            double ratio, double lmax_h = 0.0, const float* Ares = nullptr) {
  hipStream_t s = c->stream;
  using TA = typename Acc<TV>::type;
  TV* r = (TV*)L.r;
  TV* d[2] = {(TV*)L.d0, (TV*)L.d1};
  const double lmax = ST == 1 ? lmax_h : L.lmax_h, lmin = lmax / ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  const unsigned g = grid_for(L.nn);
  const TA inv_theta = (TA)(1.0 / theta);
  if (pre) {
    // zero initial guess: the residual starts at b, the first correction is D^{-1} b / theta
    hipLaunchKernelGGL((k_cheb_first<B, TM, TV>), dim3(g), dim3(kBlock), 0, s, A, L.nn, b,
                       degree == 1 ? r : nullptr, d[0], degree == 1 ? x : nullptr, inv_theta, 0);
    VP_LAUNCH_CHECK();
  } else if (degree == 1) {
    if constexpr (std::is_same<TV, float>::value && ST == 0) {
      if (Ares) sten_resid<B, float, TV, ST>(c, l, L, Ares, (const TV*)x, b, r);
      else sten_resid<B, TM, TV, ST>(c, l, L, A, (const TV*)x, b, r);
    } else {
      sten_resid<B, TM, TV, ST>(c, l, L, A, (const TV*)x, b, r);
    }
    hipLaunchKernelGGL((k_cheb_first<B, TM, TV>), dim3(g), dim3(kBlock), 0, s, A, L.nn, (const TV*)r,
                       (TV*)nullptr, d[0], x, inv_theta, 1);
    VP_LAUNCH_CHECK();
  } else {
    bool done = false;
    if constexpr (std::is_same<TV, float>::value && ST == 0) {
      if (Ares) {   // post-correction residual from the FP32 operator (see smooth_post_pairs)
        hipLaunchKernelGGL((k_resid_first<B, float, TV, ST>), dim3(g), dim3(kBlock), 0, s, Ares, L.nn, L.nxn, L.nyn,
                           (const TV*)x, b, r, d[0], inv_theta);
        done = true;
      }
    }
    if (!done)
      hipLaunchKernelGGL((k_resid_first<B, TM, TV, ST>), dim3(g), dim3(kBlock), 0, s, A, L.nn, L.nxn, L.nyn,
                         (const TV*)x, b, r, d[0], inv_theta);
    VP_LAUNCH_CHECK();
  }
  for (int k = 1; k < degree; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    const double cdd = rn * rho, cdr = 2.0 * rn / delta;
    const int xmode = k > 1 ? 0 : pre ? 2 : 1;
    const TV* rin = (pre && k == 1) ? b : (const TV*)r;
    const int pr = (l == 0 && xmode == 0) ? prof_begin(c, VP_KID_CHEB_STEP0) : -1;
    bool done = false;
    if constexpr (std::is_same<TV, float>::value && ST == 0) {
      if (Ares && !pre && k == 1) {   // the first post-correction pass: residual and step 1 in FP32
        hipLaunchKernelGGL((k_cheb_step<B, float, TV, ST>), dim3(g), dim3(kBlock), 0, s, Ares, L.nn, L.nxn, L.nyn,
                           (const TV*)d[(k - 1) & 1], rin, r, d[k & 1], (const TV*)x, x, (TA)cdd, (TA)cdr, xmode);
        done = true;
      }
    }
    if (!done)
      hipLaunchKernelGGL((k_cheb_step<B, TM, TV, ST>), dim3(g), dim3(kBlock), 0, s, A, L.nn, L.nxn, L.nyn,
                         (const TV*)d[(k - 1) & 1], rin, r, d[k & 1], (const TV*)x, x, (TA)cdd, (TA)cdr, xmode);
    VP_LAUNCH_CHECK();
    prof_end(c, pr);
    rho = rn;
  }
  // r = b - A x after pre-smoothing (r holds the residual before the last correction)
  if (pre) sten_resid<B, TM, TV, ST>(c, l, L, A, (const TV*)d[(degree - 1) & 1], (const TV*)r, r);
}

template <typename TV>
void launch_tail(vp_ctx c, int l0) {
  TailArgs a{};
  a.nlev = c->nlev - l0;
  a.degree = c->cheb_degree;
  const bool fp64 = std::is_same<TV, double>::value;
  const int prec = c->amg_prec;
  for (int k = 0; k < a.nlev; ++k) {
    const Level& L = c->lev[l0 + k];
    TailLevel& T = a.L[k];
    T.nn = (unsigned)L.nn;
    T.nxn = L.nxn; T.nyn = L.nyn; T.ncx = L.ncx; T.ncy = L.ncy;
    T.b = L.b; T.x = L.x; T.r = L.r; T.d0 = L.d0; T.d1 = L.d1;
    T.P = fp64 ? (const void*)L.P64 : (const void*)L.P32;
    if (fp64) T.A = L.A64;
    else if (prec == VP_PREC_FP32 || prec == VP_PREC_FP16_FP32COARSE) T.A = L.A32;
    else if (prec == VP_PREC_FP16) T.A = L.Ah;
    else T.A = L.Abf;
    // the coefficients of smooth(), in the same arithmetic
    const double lmax = L.lmax_h, lmin = lmax / c->cheb_ratio;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    T.inv_theta = 1.0 / theta;
    for (int s = 1; s < a.degree; ++s) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      T.cdd[s] = rn * rho;
      T.cdr[s] = 2.0 * rn / delta;
      rho = rn;
    }
  }
  const Level& C = c->lev[c->nlev - 1];
  a.nd = C.B * (int)C.nn;
  a.Ainv = fp64 ? (const void*)C.Ainv64 : (const void*)C.Ainv32;
  hipStream_t s = c->stream;
  int lds_floats = 0;
  for (int k = 0; k < a.nlev; ++k) lds_floats += 15 * (int)a.L[k].nn;
  const bool lds = c->tail_lds && !fp64 && a.degree >= 2 && lds_floats <= kTailLdsFloats &&
                   a.L[0].nn <= (unsigned)kTailLdsThreads;
  if (lds) {
    if (prec == VP_PREC_FP32 || prec == VP_PREC_FP16_FP32COARSE)
      hipLaunchKernelGGL((k_vcycle_tail_lds<float, float>), dim3(1), dim3(kTailLdsThreads), 0, s, a);
    else if (prec == VP_PREC_FP16)
      hipLaunchKernelGGL((k_vcycle_tail_lds<_Float16, float>), dim3(1), dim3(kTailLdsThreads), 0, s, a);
    else
      hipLaunchKernelGGL((k_vcycle_tail_lds<__hip_bfloat16, float>), dim3(1), dim3(kTailLdsThreads), 0, s, a);
  } else if (fp64)
    hipLaunchKernelGGL((k_vcycle_tail<double, double, double>), dim3(1), dim3(kTailThreads), 0, s, a);
  else if (prec == VP_PREC_FP32 || prec == VP_PREC_FP16_FP32COARSE)
    hipLaunchKernelGGL((k_vcycle_tail<float, float, float>), dim3(1), dim3(kTailThreads), 0, s, a);
  else if (prec == VP_PREC_FP16)
    hipLaunchKernelGGL((k_vcycle_tail<_Float16, float, float>), dim3(1), dim3(kTailThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_vcycle_tail<__hip_bfloat16, float, float>), dim3(1), dim3(kTailThreads), 0, s, a);
  VP_LAUNCH_CHECK();
}

// Finest-level smoothing with the sweeps fused in pairs (k_cheb_pair); the same
// sequence of per-node operations as smooth().  Pre-smoothing from x = 0 returns
// the buffer holding r = b - A x; post-smoothing leaves x updated in place.
// Tile shape and workgroup per value type, measured at 2049^2 nodes: FP32
// vectors 62 x 14 tiles, 1024 threads, at most 4 waves per SIMD (5% faster
// V-cycles than 64 x 16); FP64 30 x 30 tiles, 256 threads (1.5% faster than
// 128 x 8).  Ringed tiles of 32^2 and 64 x 16 nodes fill whole rounds of threads.
template <int MODE, int XM, typename TM, typename TV>
void launch_pair(vp_ctx c, const Level& L, const TM* A, const TV* vin, const TV* rin, const TV* xin, TV* rout,
                 TV* dout, TV* xout, double c1a, double c1b, double c2a, double c2b) {
  using TA = typename Acc<TV>::type;
  auto go = [&](auto tx_, auto ty_, auto nt_, auto w_) {
    constexpr int TX = decltype(tx_)::value, TY = decltype(ty_)::value, NT = decltype(nt_)::value,
                  W = decltype(w_)::value;
    const int tx = (L.nxn + TX - 1) / TX, ty = (L.nyn + TY - 1) / TY;
    const int tiles = tx * ty;
    const unsigned g = (unsigned)((tiles + 7) / 8 * 8);
    hipLaunchKernelGGL((k_cheb_pair<MODE, XM, TM, TV, TX, TY, NT, W>), dim3(g), dim3(NT), 0, c->stream, A, L.nn,
                       L.nxn, L.nyn, tx, tiles, vin, rin, xin, rout, dout, xout, (TA)c1a, (TA)c1b, (TA)c2a, (TA)c2b);
    VP_LAUNCH_CHECK();
  };
  using std::integral_constant;
  if constexpr (std::is_same<TM, TV>::value) {
    // operator in the vector type: column walks (strips of 12 rows FP64, 10 FP32)
    constexpr int TR = std::is_same<TV, double>::value ? 12 : 10;
    const dim3 g((unsigned)((L.nxn + 61) / 62), (unsigned)((L.nyn + 4 * TR - 1) / (4 * TR)));
    hipLaunchKernelGGL((k_cheb_walk<MODE, XM, TV, TR>), g, dim3(256), 0, c->stream, A, L.nn, L.nxn, L.nyn, vin, rin,
                       xin, rout, dout, xout, (TV)c1a, (TV)c1b, (TV)c2a, (TV)c2b);
    VP_LAUNCH_CHECK();
  } else if constexpr (std::is_same<TV, double>::value) {
    go(integral_constant<int, 30>(), integral_constant<int, 30>(), integral_constant<int, 256>(),
       integral_constant<int, 8>());
  } else {  // the ringed tile (64 x 16) is exactly one node per thread for the first sweep
    go(integral_constant<int, 62>(), integral_constant<int, 14>(), integral_constant<int, 1024>(),
       integral_constant<int, 4>());
  }
}

// Paired sweeps on a structured coarse level (B = 3, FP32): column walks whose strip
// height is the smallest with every workgroup resident at once.  Used on levels of
// at least kCoarsePairNodes nodes.
constexpr size_t kCoarsePairNodes = 100000;
// whether a 3 x 3-block level's pairs run as tiles (k_cheb_pair3), which also take the
// first step of a pre-smoothing and the prolongation before a post-smoothing
template <typename TM, typename TV>
bool coarse_tiles(const Level& L) {
  return !(std::is_same<TM, float>::value && std::is_same<TV, float>::value && L.nn >= kCoarsePairNodes);
}
template <int MODE, int XM>
void launch_walk3(vp_ctx c, const Level& L, const float* A, const float* vin, const float* rin, const float* xin,
                  float* rout, float* dout, float* xout, double c1a, double c1b, double c2a, double c2b) {
  int& resident = c->walk3_resident;
  if (resident == 0) {
    int ncu = 0, per_cu = 0;
    VP_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    VP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_cheb_walk3<PAIR_STEP_STEP, 0>), 256, 0));
    resident = std::max(1, ncu * per_cu);
  }
  const int gx = (L.nxn + 61) / 62;
  const int gy_fit = std::max(1, resident / gx);
  const int tr = std::max(2, (L.nyn + 4 * gy_fit - 1) / (4 * gy_fit));
  const int gy = (L.nyn + 4 * tr - 1) / (4 * tr);
  hipLaunchKernelGGL((k_cheb_walk3<MODE, XM>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, c->stream, tr, A, L.nn,
                     L.nxn, L.nyn, vin, rin, xin, rout, dout, xout, (float)c1a, (float)c1b, (float)c2a, (float)c2b);
  VP_LAUNCH_CHECK();
}

// Two Chebyshev steps in one pass: the finest level (B = 2, any storage) or a
// structured coarse level (B = 3, FP32 operator and vectors only).
template <int B, int MODE, int XM, typename TM, typename TV>
void launch_pairb(vp_ctx c, const Level& L, const TM* A, const TV* vin, const TV* rin, const TV* xin, TV* rout,
                  TV* dout, TV* xout, double c1a, double c1b, double c2a, double c2b,
                  const PairExtra& ex = PairExtra{}) {
  using TA = typename Acc<TV>::type;
  if constexpr (B == 2) {
    launch_pair<MODE, XM>(c, L, A, vin, rin, xin, rout, dout, xout, c1a, c1b, c2a, c2b);
  } else {
    if constexpr (std::is_same<TM, float>::value && std::is_same<TV, float>::value) {
      if (L.nn >= kCoarsePairNodes) {
        launch_walk3<MODE, XM>(c, L, A, vin, rin, xin, rout, dout, xout, c1a, c1b, c2a, c2b);
        return;
      }
    }
    const int tx = (L.nxn + kPair3Tile - 1) / kPair3Tile, ty = (L.nyn + kPair3Tile - 1) / kPair3Tile;
    const int tiles = tx * ty;
    const unsigned g = (unsigned)((tiles + 7) / 8 * 8);   // xcd_block() needs a multiple of 8
    hipLaunchKernelGGL((k_cheb_pair3<MODE, XM, TM, TV>), dim3(g), dim3(256), 0, c->stream, A, L.nn, L.nxn, L.nyn, tx,
                       tiles, vin, rin, xin, rout, dout, xout, (TA)c1a, (TA)c1b, (TA)c2a, (TA)c2b, ex);
    VP_LAUNCH_CHECK();
  }
}

struct ChebCoef {
  double inv_theta;
  double cdd[32], cdr[32];   // index 1..degree-1
};
inline ChebCoef cheb_coefficients(double lmax_h, double ratio, int degree) {
  ChebCoef k{};
  const double lmax = lmax_h, lmin = lmax / ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  k.inv_theta = 1.0 / theta;
  for (int s = 1; s < degree && s < 32; ++s) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    k.cdd[s] = rn * rho;
    k.cdr[s] = 2.0 * rn / delta;
    rho = rn;
  }
  return k;
}

// Degree-4 smoothing by one four-sweep column walk.  The strip height is the
// smallest whose workgroups are all resident at once: a second, partial round of
// workgroups costs up to half the kernel's time.
template <int KIND, typename T>
void launch_walk4(vp_ctx c, const Level& L, const T* A, const T* b, const T* xin, T* rout, T* xout,
                  const ChebCoef& k) {
  int& resident = c->walk4_resident[std::is_same<T, double>::value ? 1 : 0][KIND];
  constexpr int cols = walk4_cols<T>(), threads = 64 * kWalk4Strips * cols;
  if (resident == 0) {
    int ncu = 0, per_cu = 0;
    VP_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    VP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_cheb_walk4<KIND, T>), threads, 0));
    resident = std::max(1, ncu * per_cu);
  }
  const int gx = (L.nxn + 56 * cols - 1) / (56 * cols);
  const int gy_fit = std::max(1, resident / gx);   // workgroup rows (kWalk4Strips strips each) that fit
  const int tr = c->walk4_rows > 0 ? c->walk4_rows
                                   : std::max(8, (L.nyn + kWalk4Strips * gy_fit - 1) / (kWalk4Strips * gy_fit));
  const int gy = (L.nyn + kWalk4Strips * tr - 1) / (kWalk4Strips * tr);
  hipLaunchKernelGGL((k_cheb_walk4<KIND, T>), dim3(grid_for((size_t)gx * gy, 1)), dim3(threads), 0,
                     c->stream, tr, gx, gy, A, L.nn, L.nxn, L.nyn, b, xin, rout, xout, (T)k.inv_theta, (T)k.cdd[1],
                     (T)k.cdr[1], (T)k.cdd[2], (T)k.cdr[2], (T)k.cdd[3], (T)k.cdr[3]);
  VP_LAUNCH_CHECK();
}

template <int B, typename TM, typename TV>
const TV* smooth_pre_pairs(vp_ctx c, const Level& L, const TM* A, const TV* b, TV* x) {
  using TA = typename Acc<TV>::type;
  const bool fine = &L == &c->lev[0];
  const int m = c->cheb_degree - 1;
  const ChebCoef k = cheb_coefficients(L.lmax_h, c->cheb_ratio, c->cheb_degree);
  if constexpr (B == 2 && std::is_same<TM, TV>::value) {
    if (c->cheb_degree == 4) {
      const int pr = prof_begin(c, VP_KID_CHEB_WALK4);
      launch_walk4<W4_PRE, TV>(c, L, A, b, nullptr, (TV*)L.r, x, k);
      prof_end(c, pr);
      return (const TV*)L.r;
    }
  }
  TV* d[2] = {(TV*)L.d0, (TV*)L.d1};
  TV* rb[2] = {(TV*)L.r, (TV*)L.r2};
  bool fused_first = false;   // the tiles form d0 themselves
  if constexpr (B == 3) fused_first = m >= 2 && coarse_tiles<TM, TV>(L);
  if (!fused_first) {
    hipLaunchKernelGGL((k_cheb_first<B, TM, TV>), dim3(grid_for(L.nn)), dim3(kBlock), 0, c->stream, A, L.nn, b,
                       (TV*)nullptr, d[0], (TV*)nullptr, (TA)k.inv_theta, 0);
    VP_LAUNCH_CHECK();
  }
  const TV* rcur = b;
  int di = 0, ri = 0;
  for (int s = 1; s <= m;) {
    if (s + 1 <= m) {
      if (s == 1 && fused_first)
        launch_pairb<B, PAIR_FIRST_STEP, 2>(c, L, A, (const TV*)nullptr, rcur, (const TV*)x, rb[ri], d[di ^ 1], x,
                                            k.cdd[s], k.cdr[s], k.cdd[s + 1], k.cdr[s + 1],
                                            PairExtra{nullptr, nullptr, 0, 0, k.inv_theta});
      else if (s == 1)
        launch_pairb<B, PAIR_STEP_STEP, 2>(c, L, A, (const TV*)d[di], rcur, (const TV*)x, rb[ri], d[di ^ 1], x,
                                           k.cdd[s], k.cdr[s], k.cdd[s + 1], k.cdr[s + 1]);
      else {
        const int pr = fine ? prof_begin(c, VP_KID_CHEB_PAIR0) : -1;
        launch_pairb<B, PAIR_STEP_STEP, 0>(c, L, A, (const TV*)d[di], rcur, (const TV*)x, rb[ri], d[di ^ 1], x,
                                           k.cdd[s], k.cdr[s], k.cdd[s + 1], k.cdr[s + 1]);
        prof_end(c, pr);
      }
      rcur = rb[ri];
      ri ^= 1;
      di ^= 1;
      s += 2;
    } else {
      if (s == 1)
        launch_pairb<B, PAIR_STEP_RESID, 2>(c, L, A, (const TV*)d[di], rcur, (const TV*)x, rb[ri], (TV*)nullptr, x,
                                            k.cdd[s], k.cdr[s], 0.0, 0.0);
      else
        launch_pairb<B, PAIR_STEP_RESID, 0>(c, L, A, (const TV*)d[di], rcur, (const TV*)x, rb[ri], (TV*)nullptr, x,
                                            k.cdd[s], k.cdr[s], 0.0, 0.0);
      return rb[ri];
    }
  }
  // even number of steps: the final residual alone, in place
  sten_resid<B>(c, fine ? 0 : 1, L, A, (const TV*)d[di], rcur, (TV*)rcur);
  return rcur;
}

// Ares (FP32 vectors only, nullable): operator for the first pass (the residual
// b - A x after the coarse-grid correction and the first Chebyshev step).  That
// residual is small next to A x, so a 16-bit operator's rounding would dominate it.
// xin (nullable): the corrected x in another buffer, for the four-sweep walk.
template <int B, typename TM, typename TV>
void smooth_post_pairs(vp_ctx c, const Level& L, const TM* A, const TV* b, TV* x, const float* Ares = nullptr,
                       const TV* xin = nullptr, const PairExtra* pro = nullptr) {
  using TA = typename Acc<TV>::type;
  const bool fine = &L == &c->lev[0];
  const int m = c->cheb_degree - 1;
  const ChebCoef k = cheb_coefficients(L.lmax_h, c->cheb_ratio, c->cheb_degree);
  TV* d[2] = {(TV*)L.d0, (TV*)L.d1};
  TV* rb[2] = {(TV*)L.r, (TV*)L.r2};
  TV* x2 = (TV*)L.x2;
  if constexpr (B == 2 && std::is_same<TM, TV>::value) {
    if (c->cheb_degree == 4 && !Ares && xin) {
      const int pr = prof_begin(c, VP_KID_CHEB_WALK4);
      launch_walk4<W4_POST, TV>(c, L, A, b, xin, nullptr, x, k);
      prof_end(c, pr);
      return;
    }
  }
  bool done = false;
  if constexpr (B == 2 && std::is_same<TV, float>::value) {
    if (Ares) {
      launch_pair<PAIR_RFIRST_STEP, 1>(c, L, Ares, (const TV*)x, b, (const TV*)x, rb[0], d[1], x2, k.inv_theta, 0.0,
                                       k.cdd[1], k.cdr[1]);
      done = true;
    }
  }
  if (!done && pro)   // x + P xc formed by the tiles themselves (x is the uncorrected iterate)
    launch_pairb<B, PAIR_PROLONG_RFIRST, 1>(c, L, A, (const TV*)nullptr, b, (const TV*)x, rb[0], d[1], x2,
                                            k.inv_theta, 0.0, k.cdd[1], k.cdr[1], *pro);
  else if (!done)
    launch_pairb<B, PAIR_RFIRST_STEP, 1>(c, L, A, (const TV*)x, b, (const TV*)x, rb[0], d[1], x2, k.inv_theta, 0.0,
                                         k.cdd[1], k.cdr[1]);
  const TV* xcur = x2;
  TV* rcur = rb[0];
  int di = 1, ri = 1;
  for (int s = 2; s <= m;) {
    if (s + 1 <= m) {
      const int pr = fine ? prof_begin(c, VP_KID_CHEB_PAIR0) : -1;
      launch_pairb<B, PAIR_STEP_STEP, 0>(c, L, A, (const TV*)d[di], (const TV*)rcur, xcur, rb[ri], d[di ^ 1], x,
                                         k.cdd[s], k.cdr[s], k.cdd[s + 1], k.cdr[s + 1]);
      prof_end(c, pr);
      rcur = rb[ri];
      ri ^= 1;
      di ^= 1;
      s += 2;
    } else {
      hipLaunchKernelGGL((k_cheb_step<B, TM, TV>), dim3(grid_for(L.nn)), dim3(kBlock), 0, c->stream, A, L.nn, L.nxn,
                         L.nyn, (const TV*)d[di], (const TV*)rcur, rcur, d[di ^ 1], xcur, x, (TA)k.cdd[s],
                         (TA)k.cdr[s], 0);
      VP_LAUNCH_CHECK();
      di ^= 1;
      s += 1;
    }
    xcur = x;
  }
  if (xcur != x) VP_HIP(hipMemcpyAsync(x, xcur, sizeof(TV) * B * L.nn, hipMemcpyDeviceToDevice, c->stream));
}

template <typename TV>
void vcycle_level(vp_ctx c, int l, const TV* b, TV* x) {
  hipStream_t s = c->stream;
  if (l > 0 && l == c->tail_level) {
    if constexpr (std::is_same<TV, double>::value) launch_tail<double>(c, l);
    else launch_tail<float>(c, l);
    return;
  }
  Level& L = c->lev[l];
  const bool fp64 = std::is_same<TV, double>::value;
  if (l == c->nlev - 1) {
    const int nd = L.B * (int)L.nn;
    if (fp64)
      hipLaunchKernelGGL((k_dense_apply<double, TV>), dim3((nd + 127) / 128), dim3(128), 0, s, L.Ainv64, nd, b, x);
    else
      hipLaunchKernelGGL((k_dense_apply<float, TV>), dim3((nd + 127) / 128), dim3(128), 0, s, L.Ainv32, nd, b, x);
    VP_LAUNCH_CHECK();
    return;
  }
  Level& N = c->lev[l + 1];
  if (l == 0 && c->order == 2) {
    // Q2 elements: smooth with the 25-point operator, restrict/prolong with the
    // tentative prolongator (stored in slot 0 of P)
    auto q2 = [&](auto tm_tag, const void* Kv) {
      using TM = decltype(tm_tag);
      const TM* K = (const TM*)Kv;
      smooth<2, TM, TV, 1>(c, 0, L, K, b, x, true, c->cheb_degree, c->cheb_ratio, c->lmax_q2_h);
      using TPv = typename std::conditional<std::is_same<TV, double>::value, double, float>::type;
      const TPv* Pp = (const TPv*)(std::is_same<TV, double>::value ? (const void*)L.P64 : (const void*)L.P32);
      hipLaunchKernelGGL((k_restrict<2, TPv, TV>), dim3((unsigned)((N.nn * kRestrictLanes + kBlock - 1) / kBlock)),
                         dim3(kBlock), 0, s, Pp, L.nn, L.nxn, L.nyn, L.ncx, L.ncy, (const TV*)L.r, (TV*)N.b);
      VP_LAUNCH_CHECK();
      vcycle_level<TV>(c, 1, (const TV*)N.b, (TV*)N.x);
      hipLaunchKernelGGL((k_prolong_add<2, TPv, TV>), dim3(grid_for(L.nn)), dim3(kBlock), 0, s, Pp, L.nn, L.nxn,
                         L.nyn, L.ncx, L.ncy, (const TV*)N.x, (const TV*)x, x);
      VP_LAUNCH_CHECK();
      smooth<2, TM, TV, 1>(c, 0, L, K, b, x, false, c->cheb_degree, c->cheb_ratio, c->lmax_q2_h);
    };
    if constexpr (std::is_same<TV, double>::value) q2(double(), c->K2);
    else q2(float(), c->K2_32);
    return;
  }
  auto run = [&](auto bconst, auto tm_tag, auto tp_tag, const void* Av, const void* Pv) {
    constexpr int B = decltype(bconst)::value;
    using TM = decltype(tm_tag);
    using TP = decltype(tp_tag);
    const TM* A = (const TM*)Av;
    const TP* P = (const TP*)Pv;
    // paired sweeps on every level above the tail: column walks on the finest level and
    // on large FP32 coarse levels, tiles elsewhere (on levels of a few ten thousand
    // nodes a walk's strips are a few rows long and load latency makes it slower than
    // two single sweeps: 15 us against 10 us at 227^2 nodes, 36 us against 50 us at 683^2)
    constexpr bool pairable = true;
    const bool pairs = (B == 2 ? l == 0 : l > 0) && c->pair_sweeps && c->cheb_degree >= 2 && c->cheb_degree <= 32;
    const TV* rres = (const TV*)L.r;
    if constexpr (pairable) {
      if (pairs) rres = smooth_pre_pairs<B, TM, TV>(c, L, A, b, x);
      else smooth<B, TM, TV>(c, l, L, A, b, x, true, c->cheb_degree, c->cheb_ratio);
    } else {
      smooth<B, TM, TV>(c, l, L, A, b, x, true, c->cheb_degree, c->cheb_ratio);
    }
    hipLaunchKernelGGL((k_restrict<B, TP, TV>), dim3((unsigned)((N.nn * kRestrictLanes + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0,
                       s, P, L.nn, L.nxn, L.nyn, L.ncx, L.ncy, rres, (TV*)N.b);
    VP_LAUNCH_CHECK();
    vcycle_level<TV>(c, l + 1, (const TV*)N.b, (TV*)N.x);
    const float* Ares = (B == 2 && l == 0 && c->amg_prec == VP_PREC_FP16_FP32COARSE) ? L.A32 : nullptr;
    // the four-sweep walk reads the corrected x around its strips, so the correction
    // goes to a second buffer and the walk writes x
    const bool walk4 = B == 2 && pairs && std::is_same<TM, TV>::value && c->cheb_degree == 4 && !Ares;
    // tiled coarse pairs take the correction x + P xc into their first pass
    const bool fused_pro = B == 3 && pairs && std::is_same<TP, TV>::value && coarse_tiles<TM, TV>(L);
    TV* xcor = walk4 ? (TV*)L.x2 : x;
    if (!fused_pro) {
      hipLaunchKernelGGL((k_prolong_add<B, TP, TV>), dim3(grid_for(L.nn)), dim3(kBlock), 0, s, P, L.nn, L.nxn,
                         L.nyn, L.ncx, L.ncy, (const TV*)N.x, (const TV*)x, xcor);
      VP_LAUNCH_CHECK();
    }
    const PairExtra pro{(const void*)P, (const void*)N.x, L.ncx, L.ncy, 0.0};
    if constexpr (B == 2) {
      if (walk4) smooth_post_pairs<B, TM, TV>(c, L, A, b, x, nullptr, (const TV*)xcor);
      else if (pairs) smooth_post_pairs<B, TM, TV>(c, L, A, b, x, Ares);
      else smooth<B, TM, TV>(c, l, L, A, b, x, false, c->cheb_degree, c->cheb_ratio, 0.0, Ares);
    } else if constexpr (pairable) {
      if (pairs) smooth_post_pairs<B, TM, TV>(c, L, A, b, x, nullptr, nullptr, fused_pro ? &pro : nullptr);
      else smooth<B, TM, TV>(c, l, L, A, b, x, false, c->cheb_degree, c->cheb_ratio);
    } else {
      smooth<B, TM, TV>(c, l, L, A, b, x, false, c->cheb_degree, c->cheb_ratio);
    }
  };
  if constexpr (std::is_same<TV, double>::value) {
    if (L.B == 2) run(std::integral_constant<int, 2>(), double(), double(), L.A64, L.P64);
    else run(std::integral_constant<int, 3>(), double(), double(), L.A64, L.P64);
  } else {
    const bool bf = ((c->amg_prec == VP_PREC_FP32_BF16COARSE || c->amg_prec == VP_PREC_FP16_BF16COARSE) && l > 0) ||
                    c->amg_prec == VP_PREC_BF16;
    if ((l == 0 && (c->amg_prec == VP_PREC_FP16_BF16COARSE || c->amg_prec == VP_PREC_FP16_FP32COARSE)) ||
        c->amg_prec == VP_PREC_FP16) {
      if (l == 0 && c->ph_transfers) run(std::integral_constant<int, 2>(), _Float16(), _Float16(), L.Ah, L.Ph);
      else if (L.B == 2) run(std::integral_constant<int, 2>(), _Float16(), float(), L.Ah, L.P32);
      else run(std::integral_constant<int, 3>(), _Float16(), float(), L.Ah, L.P32);
    } else if (L.B == 2 && bf) run(std::integral_constant<int, 2>(), __hip_bfloat16(), float(), L.Abf, L.P32);
    else if (L.B == 2) run(std::integral_constant<int, 2>(), float(), float(), L.A32, L.P32);
    else if (bf) run(std::integral_constant<int, 3>(), __hip_bfloat16(), float(), L.Abf, L.P32);
    else run(std::integral_constant<int, 3>(), float(), float(), L.A32, L.P32);
  }
}

}  // namespace

// The finest level runs in Jacobi-scaled variables (16-bit finest storage).
bool scaled_finest(vp_ctx c) {
  return c->amg_prec == VP_PREC_BF16 || c->amg_prec == VP_PREC_FP16_BF16COARSE || c->amg_prec == VP_PREC_FP16 ||
         c->amg_prec == VP_PREC_FP16_FP32COARSE;
}

// z = M^{-1} r (FP64 in/out; V-cycle in the setup's precision)
void amg_apply(vp_ctx c, const double* r, double* z) {
  if (!c->amg_ready) throw Error(VP_ESTATE, "AMG not set up");
  if (c->amg_kind == VP_AMG_RS) {
    const int pr = prof_begin(c, VP_KID_VCYCLE);
    rs_apply(c, r, z);
    prof_end(c, pr);
    return;
  }
  Level& L = c->lev[0];
  const size_t n = (size_t)L.B * L.nn;
  struct End {
    vp_ctx c;
    int idx;
    ~End() {
      try { prof_end(c, idx); } catch (...) {}
    }
  } end_{c, prof_begin(c, VP_KID_VCYCLE)};
  if (c->amg_prec == VP_PREC_FP64) {
    vcycle_level<double>(c, 0, r, z);
  } else if (scaled_finest(c)) {
    // finest level in the scaled variables: b^ = D^{-1/2} r, z = D^{-1/2} x^
    hipLaunchKernelGGL(k_scale_cast_df, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, r, L.dsc64, (float*)L.b, n);
    VP_LAUNCH_CHECK();
    vcycle_level<float>(c, 0, (const float*)L.b, (float*)L.x);
    hipLaunchKernelGGL(k_scale_cast_fd, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, (const float*)L.x, L.dsc64,
                       z, n);
    VP_LAUNCH_CHECK();
  } else {
    launch_cast(c->stream, r, (float*)L.b, n);
    // level-0 x must not alias L.b; the cycle writes L.x
    vcycle_level<float>(c, 0, (const float*)L.b, (float*)L.x);
    launch_cast(c->stream, (const float*)L.x, z, n);
  }
}

// FP32 input buffer of the V-cycle (and the finest level's Jacobi scaling when
// the V-cycle runs in scaled variables), or null for an FP64 V-cycle: callers
// that produce the residual can write it there directly and pass input_ready.

float* amg_input32(vp_ctx c, const double** dsc) {
  if (dsc) *dsc = scaled_finest(c) ? c->lev[0].dsc64 : nullptr;
  return c->amg_prec == VP_PREC_FP64 ? nullptr : (float*)c->lev[0].b;
}

// The FP32 V-cycle output (SA hierarchy in a mixed precision) and its scaling, or
// null where the V-cycle works in FP64.
const float* amg_output32(vp_ctx c, const double** dsc) {
  const bool f32 = c->amg_kind == VP_AMG_SA && c->amg_prec != VP_PREC_FP64;
  if (dsc) *dsc = f32 && scaled_finest(c) ? c->lev[0].dsc64 : nullptr;
  return f32 ? (const float*)c->lev[0].x : nullptr;
}

// z = M^{-1} r followed, in the same pass as the V-cycle's output conversion, by
// the per-workgroup partials of z.r and (q given) z.q.  Returns the number of
// workgroups (the partials hold 1 or 2 values each).  z may be null for an FP32
// V-cycle (the caller reads its output through amg_output32).
int amg_apply_dots(vp_ctx c, const double* r, const double* q, double* z, bool input_ready) {
  if (!c->amg_ready) throw Error(VP_ESTATE, "AMG not set up");
  Level& L = c->lev[0];
  const size_t n = (size_t)L.B * L.nn;
  hipStream_t s = c->stream;
  const int pr = prof_begin(c, VP_KID_VCYCLE);
  int nb;
  if (c->amg_kind == VP_AMG_RS) {
    rs_apply(c, r, z);
    nb = launch_out_dots<double>(s, z, nullptr, z, r, q, n, c->partials);
  } else if (c->amg_prec == VP_PREC_FP64) {
    vcycle_level<double>(c, 0, r, z);
    nb = launch_out_dots<double>(s, z, nullptr, z, r, q, n, c->partials);
  } else {
    const bool scaled = scaled_finest(c);
    if (!input_ready) {
      if (scaled) {
        hipLaunchKernelGGL(k_scale_cast_df, dim3(grid_for(n)), dim3(kBlock), 0, s, r, L.dsc64, (float*)L.b, n);
        VP_LAUNCH_CHECK();
      } else {
        launch_cast(s, r, (float*)L.b, n);
      }
    }
    vcycle_level<float>(c, 0, (const float*)L.b, (float*)L.x);
    nb = launch_out_dots<float>(s, (const float*)L.x, scaled ? L.dsc64 : nullptr, z, r, q, n, c->partials);
  }
  prof_end(c, pr);
  return nb;
}

void launch_dense_inverse(hipStream_t s, double* M, int nd) {
  if (nd <= kLdsGJ) hipLaunchKernelGGL(k_gauss_jordan_lds, dim3(1), dim3(1024), 0, s, M, nd);
  else hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, s, M, nd);
  VP_LAUNCH_CHECK();
}

template <int TR, int WX>
int launch_walk(hipStream_t s, const Level& L, const double* x, double* y, double* partials) {
  constexpr int WY = kBlock / 64 / WX;
  const unsigned gx = (unsigned)((L.nxn + 64 * WX - 1) / (64 * WX));
  const unsigned gy = (unsigned)((L.nyn + TR * WY - 1) / (TR * WY));
  hipLaunchKernelGGL((k_apply_fine<TR, WX>), dim3(gx, gy), dim3(kBlock), 0, s, L.A64, L.nn, L.nxn, L.nyn, x, y,
                     partials);
  VP_LAUNCH_CHECK();
  return (int)(gx * gy);
}

int launch_apply_fine(hipStream_t s, const Level& L, const double* x, double* y, double* partials) {
  // two-row strips, four waves side by side (256 columns): measured best of strip
  // heights 2-16 and 1-4 waves across on 2049^2 nodes
  return launch_walk<2, 4>(s, L, x, y, partials);
}

}  // namespace vp
