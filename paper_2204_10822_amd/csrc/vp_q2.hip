// Q2 (biquadratic) velocity elements: the same implicit momentum step on the
// (2nx+1) x (2ny+1) node grid of the nx x ny cells, with 3x3 Gauss quadrature
// (the paper's higher-order option, Sec. 5; everything else as for Q1).
//
// The linearised operator couples nodes up to two grid steps apart: a symmetric
// block 25-point stencil stored as 13 2x2 blocks per node, the self block and the
// 12 "forward" offsets (ox, oy) with oy > 0 or (oy = 0, ox > 0):
//   K2[aidx(2, nn, dir, node, r, c)],  dir = q2_dir(ox, oy).
// Kernels are node-centred (gather over the up to four cells holding the node),
// so outputs are written by one thread each and results are deterministic.
// Quadrature-point quantities use the Mandel form of the Q1 kernels.
#include "vp_internal.h"

namespace vp {

namespace {

constexpr double kSqrt2 = 1.41421356237309504880;
// 3-point Gauss rule on [0, 1]: points 1/2 -+ sqrt(3/5)/2 and 1/2, weights 5/18, 8/18, 5/18
__device__ __forceinline__ double gauss3_pt(int k) {
  return k == 0 ? 0.11270166537925831148 : (k == 1 ? 0.5 : 0.88729833462074168852);
}
__device__ __forceinline__ double gauss3_wt(int k) { return k == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }

// 1-D quadratic Lagrange basis at nodes 0, 1/2, 1 and its derivative
__device__ __forceinline__ double lag(int k, double t) {
  return k == 0 ? 2.0 * (t - 0.5) * (t - 1.0) : (k == 1 ? 4.0 * t * (1.0 - t) : 2.0 * t * (t - 0.5));
}
__device__ __forceinline__ double dlag(int k, double t) {
  return k == 0 ? 4.0 * t - 3.0 : (k == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0);
}

struct Shape9 {
  double N[9], gx[9], gy[9];
  double w;
};

// shape functions of the 9 element nodes (a = ax + 3 ay) at Gauss point q = qx + 3 qy
__device__ __forceinline__ Shape9 shape9(int q, double hx, double hy) {
  const int qx = q % 3, qy = q / 3;
  const double tx = gauss3_pt(qx), ty = gauss3_pt(qy);
  double lx[3], ly[3], dx[3], dy[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lx[k] = lag(k, tx); ly[k] = lag(k, ty);
    dx[k] = dlag(k, tx) / hx; dy[k] = dlag(k, ty) / hy;
  }
  Shape9 s;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    s.N[a] = lx[a % 3] * ly[a / 3];
    s.gx[a] = dx[a % 3] * ly[a / 3];
    s.gy[a] = lx[a % 3] * dy[a / 3];
  }
  s.w = gauss3_wt(qx) * gauss3_wt(qy) * hx * hy;
  return s;
}

struct CellVel9 {
  double x[9], y[9];
};

__device__ __forceinline__ void load_cell9(const ElemConst& c, const double* __restrict__ v,
                                           const double* __restrict__ dv, double alpha, int ci, int cj,
                                           CellVel9& out) {
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const size_t id = (size_t)(2 * cj + a / 3) * c.nxn + (2 * ci + a % 3);
    const double2 t = reinterpret_cast<const double2*>(v)[id];
    out.x[a] = t.x;
    out.y[a] = t.y;
    if (dv) {
      const double2 d = reinterpret_cast<const double2*>(dv)[id];
      out.x[a] = fma(alpha, d.x, out.x[a]);
      out.y[a] = fma(alpha, d.y, out.y[a]);
    }
  }
}

struct Kin9 {
  double u, w, ux, uy, wx, wy, t1, t2, t3, delta;
};

__device__ __forceinline__ Kin9 kin9(const ElemConst& c, const Shape9& s, const CellVel9& v) {
  Kin9 k;
  k.u = k.w = k.ux = k.uy = k.wx = k.wy = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    k.u = fma(s.N[a], v.x[a], k.u);
    k.w = fma(s.N[a], v.y[a], k.w);
    k.ux = fma(s.gx[a], v.x[a], k.ux);
    k.uy = fma(s.gy[a], v.x[a], k.uy);
    k.wx = fma(s.gx[a], v.y[a], k.wx);
    k.wy = fma(s.gy[a], v.y[a], k.wy);
  }
  k.t1 = c.c1 * k.ux + c.c2 * k.wy;
  k.t2 = c.c2 * k.ux + c.c1 * k.wy;
  k.t3 = c.s2e * (k.uy + k.wx);
  k.delta = sqrt(c.dmin2 + 2.0 * (k.t1 * k.t1 + k.t2 * k.t2 + k.t3 * k.t3));
  return k;
}

__device__ __forceinline__ double interp9(const Shape9& s, const double f[9]) {
  double r = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) r = fma(s.N[a], f[a], r);
  return r;
}

__device__ __forceinline__ bool q2_boundary(const ElemConst& c, int I, int J) {
  return I == 0 || J == 0 || I == c.nxn - 1 || J == c.nyn - 1;
}

// Cells holding node index I along one direction: up to two (cell, local index)
// pairs; returns the count.
__device__ __forceinline__ int q2_cells(int I, int ncell, int (&ci)[2], int (&ai)[2]) {
  int k = 0;
  if (I & 1) {
    ci[k] = (I - 1) / 2; ai[k] = 1; ++k;
  } else {
    if (I / 2 - 1 >= 0) { ci[k] = I / 2 - 1; ai[k] = 2; ++k; }
    if (I / 2 < ncell) { ci[k] = I / 2; ai[k] = 0; ++k; }
  }
  return k;
}

}  // namespace

// stored block index of offset (ox, oy), -1 for the transposed (backward) half
__host__ __device__ constexpr int q2_dir(int ox, int oy) {
  return (ox == 0 && oy == 0) ? 0
         : (oy == 0 && ox > 0) ? ox
         : (oy == 1 || oy == 2) ? 3 + 5 * (oy - 1) + (ox + 2)
         : -1;
}

// ---------------------------------------------------------------------------
// per-step precompute: the load vector
__global__ void __launch_bounds__(kBlock)
k_q2_load_vector(ElemConst c, const double* __restrict__ rhoH, const double* __restrict__ va,
                 const double* __restrict__ vo, const double* __restrict__ vn, double* __restrict__ F) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n >= (size_t)c.nxn * c.nyn) return;
  const int I = (int)(n % c.nxn), J = (int)(n / c.nxn);
  int cx[2], ax[2], cy[2], ay[2];
  const int kx = q2_cells(I, c.nx, cx, ax), ky = q2_cells(J, c.ny, cy, ay);
  double fx = 0.0, fy = 0.0;
  for (int b = 0; b < ky; ++b)
    for (int a = 0; a < kx; ++a) {
      const int ci = cx[a], cj = cy[b];
      CellVel9 A_, O_, Nv;
      load_cell9(c, va, nullptr, 0.0, ci, cj, A_);
      load_cell9(c, vo, nullptr, 0.0, ci, cj, O_);
      load_cell9(c, vn, nullptr, 0.0, ci, cj, Nv);
      const double rh = rhoH[(size_t)cj * c.nx + ci];
      for (int q = 0; q < 9; ++q) {
        const Shape9 s = shape9(q, c.hx, c.hy);
        const double Na = lag(ax[a], gauss3_pt(q % 3)) * lag(ay[b], gauss3_pt(q / 3));
        const double axq = interp9(s, A_.x), ayq = interp9(s, A_.y);
        const double oxq = interp9(s, O_.x), oyq = interp9(s, O_.y);
        const double nxq = interp9(s, Nv.x), nyq = interp9(s, Nv.y);
        const double sa = c.cda * sqrt(axq * axq + ayq * ayq);
        const double gx_ = rh * nxq + c.dt * rh * c.fc * (nyq - oyq) + c.dt * sa * axq;
        const double gy_ = rh * nyq - c.dt * rh * c.fc * (nxq - oxq) + c.dt * sa * ayq;
        fx = fma(s.w * Na, gx_, fx);
        fy = fma(s.w * Na, gy_, fy);
      }
    }
  reinterpret_cast<double2*>(F)[n] = make_double2(fx, fy);
}

// ---------------------------------------------------------------------------
// residual R(v) = A(v, phi) - F(phi) and energy Phi (eq. A, eq. sigma, eq. energy)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_q2_residual(ElemConst c, const double* __restrict__ v, const double* __restrict__ dv, double alpha,
              const double* __restrict__ vo, const double* __restrict__ F, const double* __restrict__ P,
              const double* __restrict__ rhoH, double* __restrict__ r, double* __restrict__ partials) {
  __shared__ double lds[16 * 3];
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  if (n < (size_t)c.nxn * c.nyn) {
    const int I = (int)(n % c.nxn), J = (int)(n / c.nxn);
    int cx[2], ax[2], cy[2], ay[2];
    const int kx = q2_cells(I, c.nx, cx, ax), ky = q2_cells(J, c.ny, cy, ay);
    double rx = 0.0, ry = 0.0, ecell = 0.0, eabs = 0.0;
    for (int b = 0; b < ky; ++b)
      for (int a = 0; a < kx; ++a) {
        const int ci = cx[a], cj = cy[b];
        const bool owner = ax[a] == 0 && ay[b] == 0;   // the node is the cell's south-west corner
        CellVel9 V, O;
        load_cell9(c, v, dv, alpha, ci, cj, V);
        load_cell9(c, vo, nullptr, 0.0, ci, cj, O);
        const size_t e = (size_t)cj * c.nx + ci;
        const double Pc = P[e], rh = rhoH[e];
        double en = 0.0;
        for (int q = 0; q < 9; ++q) {
          const Shape9 s = shape9(q, c.hx, c.hy);
          const Kin9 k = kin9(c, s, V);
          const double tx = gauss3_pt(q % 3), ty = gauss3_pt(q / 3);
          const double Na = lag(ax[a], tx) * lag(ay[b], ty);
          const double gxa = dlag(ax[a], tx) * lag(ay[b], ty) / c.hx;
          const double gya = lag(ax[a], tx) * dlag(ay[b], ty) / c.hy;
          const double kd = c.dt * Pc / k.delta, hp = 0.5 * c.dt * Pc;
          const double Sx = kd * (c.c1 * k.t1 + c.c2 * k.t2) - hp;
          const double Sy = kd * (c.c2 * k.t1 + c.c1 * k.t2) - hp;
          const double Sxy = kd * c.s2e * k.t3;
          const double wx_ = interp9(s, O.x) - k.u, wy_ = interp9(s, O.y) - k.w;
          const double wn = sqrt(wx_ * wx_ + wy_ * wy_);
          const double fx = rh * k.u - c.dt * c.cdo * wn * wx_;
          const double fy = rh * k.w - c.dt * c.cdo * wn * wy_;
          rx += s.w * (Sx * gxa + Sxy * gya + fx * Na);
          ry += s.w * (Sy * gya + Sxy * gxa + fy * Na);
          if (owner)
            en += s.w * (0.5 * rh * (k.u * k.u + k.w * k.w) +
                         c.dt * (0.5 * Pc * (k.delta - (k.ux + k.wy)) + c.cdo * wn * wn * wn / 3.0));
        }
        if (owner) { ecell += en; eabs += fabs(en); }
      }
    const double2 Fn = reinterpret_cast<const double2*>(F)[n];
    double2 vn = reinterpret_cast<const double2*>(v)[n];
    if (dv) {
      const double2 d = reinterpret_cast<const double2*>(dv)[n];
      vn.x = fma(alpha, d.x, vn.x);
      vn.y = fma(alpha, d.y, vn.y);
    }
    rx -= Fn.x;
    ry -= Fn.y;
    if (q2_boundary(c, I, J)) rx = ry = 0.0;
    if (r) reinterpret_cast<double2*>(r)[n] = make_double2(rx, ry);
    const double fv = Fn.x * vn.x + Fn.y * vn.y;
    acc[0] = rx * rx + ry * ry;
    acc[1] = ecell - fv;
    acc[2] = eabs + fabs(fv);
  }
  block_sum<3>(acc, lds);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 3 + 0] = acc[0];
    partials[blockIdx.x * 3 + 1] = acc[1];
    partials[blockIdx.x * 3 + 2] = acc[2];
  }
}

// ---------------------------------------------------------------------------
// operator assembly (eq. linearSVNewton + eq. modification; eq. standardNewton1/2)
// ---------------------------------------------------------------------------
// One cell's contribution to the block row of its node (AX, AY): every block index
// is a compile-time constant, so the 13 accumulators stay in registers.
template <int AX, int AY>
__device__ __forceinline__ void q2_cell_row(const ElemConst& c, const CellVel9& V, const CellVel9& O, double Pc,
                                            double rh, const double* __restrict__ pi, size_t e, size_t ncell,
                                            int variant, double (&blk)[13][4]) {
  constexpr int a = AX + 3 * AY;
  for (int q = 0; q < 9; ++q) {
    const Shape9 s = shape9(q, c.hx, c.hy);
    const Kin9 k = kin9(c, s, V);
    const double d = k.delta;
    const double base = c.dt * Pc / d;
    double C11, C12, C13, C22, C23, C33;
    if (variant == VP_SVN) {
      const double p1 = pi[(size_t)(q * 3 + 0) * ncell + e];
      const double p2 = pi[(size_t)(q * 3 + 1) * ncell + e];
      const double p3 = kSqrt2 * pi[(size_t)(q * 3 + 2) * ncell + e];
      const double sn = fmax(1.0, sqrt(2.0 * (p1 * p1 + p2 * p2 + p3 * p3)));
      const double f = base / (d * sn);
      C11 = base - f * 2.0 * k.t1 * p1;
      C22 = base - f * 2.0 * k.t2 * p2;
      C33 = base - f * 2.0 * k.t3 * p3;
      C12 = -f * (k.t1 * p2 + p1 * k.t2);
      C13 = -f * (k.t1 * p3 + p1 * k.t3);
      C23 = -f * (k.t2 * p3 + p2 * k.t3);
    } else {
      const double f = 2.0 * base / (d * d);
      C11 = base - f * k.t1 * k.t1;
      C22 = base - f * k.t2 * k.t2;
      C33 = base - f * k.t3 * k.t3;
      C12 = -f * k.t1 * k.t2;
      C13 = -f * k.t1 * k.t3;
      C23 = -f * k.t2 * k.t3;
    }
    const double wx_ = interp9(s, O.x) - k.u, wy_ = interp9(s, O.y) - k.w;
    const double wn = sqrt(wx_ * wx_ + wy_ * wy_);
    const double dr = c.dt * c.cdo;
    double Mxx = rh + dr * wn, Myy = Mxx, Mxy = 0.0;
    if (wn > 0.0) {
      Mxx += dr * wx_ * wx_ / wn;
      Myy += dr * wy_ * wy_ / wn;
      Mxy = dr * wx_ * wy_ / wn;
    }
    const double gxa = s.gx[a], gya = s.gy[a];
    const double bx0 = c.c1 * gxa, bx1 = c.c2 * gxa, bx2 = c.s2e * gya;
    const double by0 = c.c2 * gya, by1 = c.c1 * gya, by2 = c.s2e * gxa;
    const double X00 = bx0 * C11 + bx1 * C12 + bx2 * C13;
    const double X01 = bx0 * C12 + bx1 * C22 + bx2 * C23;
    const double X02 = bx0 * C13 + bx1 * C23 + bx2 * C33;
    const double X10 = by0 * C11 + by1 * C12 + by2 * C13;
    const double X11 = by0 * C12 + by1 * C22 + by2 * C23;
    const double X12 = by0 * C13 + by1 * C23 + by2 * C33;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
      const int dir = q2_dir(b % 3 - AX, b / 3 - AY);
      if (dir < 0) continue;
      const double gxb = s.gx[b], gyb = s.gy[b];
      const double cx0 = c.c1 * gxb, cx1 = c.c2 * gxb, cx2 = c.s2e * gyb;
      const double cy0 = c.c2 * gyb, cy1 = c.c1 * gyb, cy2 = c.s2e * gxb;
      const double nn_ = s.N[a] * s.N[b];
      blk[dir][0] += s.w * (X00 * cx0 + X01 * cx1 + X02 * cx2 + nn_ * Mxx);
      blk[dir][1] += s.w * (X00 * cy0 + X01 * cy1 + X02 * cy2 + nn_ * Mxy);
      blk[dir][2] += s.w * (X10 * cx0 + X11 * cx1 + X12 * cx2 + nn_ * Mxy);
      blk[dir][3] += s.w * (X10 * cy0 + X11 * cy1 + X12 * cy2 + nn_ * Myy);
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_q2_assemble(ElemConst c, const double* __restrict__ v, const double* __restrict__ pi, int variant,
              const double* __restrict__ vo, const double* __restrict__ P, const double* __restrict__ rhoH,
              double* __restrict__ K) {
  const size_t nn = (size_t)c.nxn * c.nyn;
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int I = (int)(n % c.nxn), J = (int)(n / c.nxn);
  const size_t ncell = (size_t)c.nx * c.ny;
  double blk[13][4];
#pragma unroll
  for (int b = 0; b < 13; ++b)
#pragma unroll
    for (int k = 0; k < 4; ++k) blk[b][k] = 0.0;
  int cx[2], ax[2], cy[2], ay[2];
  const int kx = q2_cells(I, c.nx, cx, ax), ky = q2_cells(J, c.ny, cy, ay);
  for (int b = 0; b < ky; ++b)
    for (int a = 0; a < kx; ++a) {
      const int ci = cx[a], cj = cy[b];
      CellVel9 V, O;
      load_cell9(c, v, nullptr, 0.0, ci, cj, V);
      load_cell9(c, vo, nullptr, 0.0, ci, cj, O);
      const size_t e = (size_t)cj * c.nx + ci;
      const double Pc = P[e], rh = rhoH[e];
      switch (ax[a] + 3 * ay[b]) {
        case 0: q2_cell_row<0, 0>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 1: q2_cell_row<1, 0>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 2: q2_cell_row<2, 0>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 3: q2_cell_row<0, 1>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 4: q2_cell_row<1, 1>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 5: q2_cell_row<2, 1>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 6: q2_cell_row<0, 2>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        case 7: q2_cell_row<1, 2>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
        default: q2_cell_row<2, 2>(c, V, O, Pc, rh, pi, e, ncell, variant, blk); break;
      }
    }
  // Dirichlet rows and columns: identity at boundary nodes, no coupling to them
  const bool bn = q2_boundary(c, I, J);
#pragma unroll
  for (int d = 0; d < 13; ++d) {
    const int ii = I + q2_ox(d), jj = J + q2_oy(d);
    bool zero;
    if (d == 0) zero = bn;
    else zero = bn || ii < 0 || ii >= c.nxn || jj >= c.nyn || q2_boundary(c, ii, jj);
    double val[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      val[k] = zero ? 0.0 : blk[d][k];
      if (d == 0 && bn) val[k] = (k == 0 || k == 3) ? 1.0 : 0.0;
    }
    double2* dst = reinterpret_cast<double2*>(K + aidx(2, nn, d, n, 0, 0));
    dst[0] = make_double2(val[0], val[1]);
    dst[1] = make_double2(val[2], val[3]);
  }
}

// y = K2 x (block 25-point, transposed halves read from the neighbours), with
// per-workgroup partial sums of x.y
__global__ void __launch_bounds__(kBlock)
k_q2_apply(const double* __restrict__ K, int nxn, int nyn, const double* __restrict__ x, double* __restrict__ y,
           double* __restrict__ partials) {
  __shared__ double lds[16];
  const size_t nn = (size_t)nxn * nyn;
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (n < nn) {
    const int I = (int)(n % nxn), J = (int)(n / nxn);
    double y0 = 0.0, y1 = 0.0;
#pragma unroll
    for (int d = 0; d < 13; ++d) {
      const int ox = q2_ox(d), oy = q2_oy(d);
      // forward block at this node
      {
        const int ii = I + ox, jj = J + oy;
        if (ii >= 0 && ii < nxn && jj < nyn) {
          const size_t m = (size_t)jj * nxn + ii;
          const double2 b0 = reinterpret_cast<const double2*>(K + aidx(2, nn, d, n, 0, 0))[0];
          const double2 b1 = reinterpret_cast<const double2*>(K + aidx(2, nn, d, n, 0, 0))[1];
          const double2 xm = reinterpret_cast<const double2*>(x)[m];
          y0 += b0.x * xm.x + b0.y * xm.y;
          y1 += b1.x * xm.x + b1.y * xm.y;
        }
      }
      // the transposed block held by the neighbour at the opposite offset
      if (d > 0) {
        const int ii = I - ox, jj = J - oy;
        if (ii >= 0 && ii < nxn && jj >= 0) {
          const size_t m = (size_t)jj * nxn + ii;
          const double2 b0 = reinterpret_cast<const double2*>(K + aidx(2, nn, d, m, 0, 0))[0];
          const double2 b1 = reinterpret_cast<const double2*>(K + aidx(2, nn, d, m, 0, 0))[1];
          const double2 xm = reinterpret_cast<const double2*>(x)[m];
          y0 += b0.x * xm.x + b1.x * xm.y;
          y1 += b0.y * xm.x + b1.y * xm.y;
        }
      }
    }
    reinterpret_cast<double2*>(y)[n] = make_double2(y0, y1);
    const double2 xn = reinterpret_cast<const double2*>(x)[n];
    acc[0] = y0 * xn.x + y1 * xn.y;
  }
  if (partials) {
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
  }
}

// ---------------------------------------------------------------------------
// dual update (eq. tautilde with eq. modification) and consistent initialisation
// ---------------------------------------------------------------------------
__global__ void k_q2_pi_update(ElemConst c, const double* __restrict__ v, const double* __restrict__ dv,
                               double* __restrict__ pi, double alpha) {
  const size_t ncell = (size_t)c.nx * c.ny;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const int ci = (int)(e % c.nx), cj = (int)(e / c.nx);
  CellVel9 V, D;
  load_cell9(c, v, nullptr, 0.0, ci, cj, V);
  load_cell9(c, dv, nullptr, 0.0, ci, cj, D);
  for (int q = 0; q < 9; ++q) {
    const Shape9 s = shape9(q, c.hx, c.hy);
    const Kin9 k = kin9(c, s, V);
    const Kin9 kd = kin9(c, s, D);
    double* pq = pi + (size_t)(q * 3) * ncell + e;
    const double p1 = pq[0], p2 = pq[ncell], p3 = kSqrt2 * pq[2 * ncell];
    const double sn = fmax(1.0, sqrt(2.0 * (p1 * p1 + p2 * p2 + p3 * p3)));
    const double id = 1.0 / k.delta;
    const double at = k.t1 * kd.t1 + k.t2 * kd.t2 + k.t3 * kd.t3;
    const double pt = p1 * kd.t1 + p2 * kd.t2 + p3 * kd.t3;
    const double g = id * id / sn;
    const double d1 = -p1 + (k.t1 + kd.t1) * id - g * (at * p1 + pt * k.t1);
    const double d2 = -p2 + (k.t2 + kd.t2) * id - g * (at * p2 + pt * k.t2);
    const double d3 = -p3 + (k.t3 + kd.t3) * id - g * (at * p3 + pt * k.t3);
    pq[0] = p1 + alpha * d1;
    pq[ncell] = p2 + alpha * d2;
    pq[2 * ncell] = (p3 + alpha * d3) / kSqrt2;
  }
}

__global__ void k_q2_pi_init(ElemConst c, const double* __restrict__ v, double* __restrict__ pi) {
  const size_t ncell = (size_t)c.nx * c.ny;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const int ci = (int)(e % c.nx), cj = (int)(e / c.nx);
  CellVel9 V;
  load_cell9(c, v, nullptr, 0.0, ci, cj, V);
  for (int q = 0; q < 9; ++q) {
    const Shape9 s = shape9(q, c.hx, c.hy);
    const Kin9 k = kin9(c, s, V);
    const double id = 1.0 / k.delta;
    double* pq = pi + (size_t)(q * 3) * ncell + e;
    pq[0] = k.t1 * id;
    pq[ncell] = k.t2 * id;
    pq[2 * ncell] = k.t3 * id / kSqrt2;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_q2_precompute(vp_ctx c, const double* va, const double* vo, const double* vprev) {
  hipLaunchKernelGGL(k_q2_load_vector, dim3(grid_for(c->nn)), dim3(kBlock), 0, c->stream, c->ec, c->rhoH, va, vo,
                     vprev, c->F);
  VP_LAUNCH_CHECK();
}

void launch_q2_residual(vp_ctx c, const double* v, const double* dv, double alpha, double* r, double* partials,
                        unsigned* nblocks) {
  const unsigned g = grid_for(c->nn);
  hipLaunchKernelGGL(k_q2_residual, dim3(g), dim3(kBlock), 0, c->stream, c->ec, v, dv, alpha, c->vo, c->F, c->P,
                     c->rhoH, r, partials);
  VP_LAUNCH_CHECK();
  *nblocks = g;
}

void launch_q2_assemble(vp_ctx c, const double* v, const double* pi, int variant) {
  hipLaunchKernelGGL(k_q2_assemble, dim3(grid_for(c->nn)), dim3(kBlock), 0, c->stream, c->ec, v, pi, variant,
                     c->vo, c->P, c->rhoH, c->K2);
  VP_LAUNCH_CHECK();
}

void launch_q2_apply(vp_ctx c, const double* x, double* y, double* partials) {
  hipLaunchKernelGGL(k_q2_apply, dim3(grid_for(c->nn)), dim3(kBlock), 0, c->stream, c->K2, c->ec.nxn, c->ec.nyn, x,
                     y, partials);
  VP_LAUNCH_CHECK();
}

void launch_q2_pi_update(vp_ctx c, const double* v, const double* dv, double* pi, double alpha) {
  hipLaunchKernelGGL(k_q2_pi_update, dim3((unsigned)((c->ncell + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, c->ec, v, dv, pi, alpha);
  VP_LAUNCH_CHECK();
}

void launch_q2_pi_init(vp_ctx c, const double* v, double* pi) {
  hipLaunchKernelGGL(k_q2_pi_init, dim3((unsigned)((c->ncell + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, c->ec, v, pi);
  VP_LAUNCH_CHECK();
}

}  // namespace vp
