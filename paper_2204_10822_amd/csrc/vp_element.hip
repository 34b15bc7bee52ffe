// Element kernels on the structured Q1 mesh: per-step precompute, residual and
// energy, linearised-operator assembly, dual (pi) update.
//
// Every quadrature-point quantity is computed in Mandel form: for a symmetric
// 2x2 tensor X, m(X) = (X11, X22, sqrt2 X12), so m(X).m(Y) = X:Y.  With e the
// ellipse ratio, tau(v) = e^-1 eps'(v) + tr(eps)/2 I (Sec. 4) becomes
//   m(tau) = (c1 ux + c2 vy, c2 ux + c1 vy, s2e (uy + vx)),
//   c1 = (1 + 1/e)/2, c2 = (1 - 1/e)/2, s2e = 1/(sqrt2 e),
// and Delta = sqrt(Delta_min^2 + 2 m(tau).m(tau)).
//
// The residual and the assembly run on element patches staged in LDS (each cell's
// Gauss points evaluated once per tile, then gathered by the nodes of the tile in
// a fixed order), the dual update per cell; no two threads write the same output
// and results are deterministic without atomics.
#include "vp_internal.h"

namespace vp {

namespace {

constexpr double kG0 = 0.21132486540518711775;  // 1/2 - 1/(2 sqrt 3)
constexpr double kG1 = 0.78867513459481288225;  // 1/2 + 1/(2 sqrt 3)
constexpr double kSqrt2 = 1.41421356237309504880;

struct Shape {
  double N[4], gx[4], gy[4];
};

// Q1 shape functions on the cell at Gauss point q = qx + 2 qy; corners SW, SE, NW, NE.
__device__ __forceinline__ Shape shape_at(int q, double ihx, double ihy) {
  const double xi = (q & 1) ? kG1 : kG0, eta = (q & 2) ? kG1 : kG0;
  Shape s;
  s.N[0] = (1 - xi) * (1 - eta); s.N[1] = xi * (1 - eta);
  s.N[2] = (1 - xi) * eta;       s.N[3] = xi * eta;
  s.gx[0] = -(1 - eta) * ihx; s.gx[1] = (1 - eta) * ihx; s.gx[2] = -eta * ihx; s.gx[3] = eta * ihx;
  s.gy[0] = -(1 - xi) * ihy;  s.gy[1] = -xi * ihy;       s.gy[2] = (1 - xi) * ihy; s.gy[3] = xi * ihy;
  return s;
}

struct CellVel {
  double x[4], y[4];
};

__device__ __forceinline__ void load_cell(const ElemConst& c, const double* __restrict__ v,
                                          const double* __restrict__ dv, double alpha, int ci,
                                          int cj, CellVel& out) {
  const size_t sw = (size_t)cj * c.nxn + ci;
  const size_t id[4] = {sw, sw + 1, sw + c.nxn, sw + c.nxn + 1};
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double2 t = reinterpret_cast<const double2*>(v)[id[a]];
    out.x[a] = t.x;
    out.y[a] = t.y;
    if (dv) {
      const double2 d = reinterpret_cast<const double2*>(dv)[id[a]];
      out.x[a] = fma(alpha, d.x, out.x[a]);
      out.y[a] = fma(alpha, d.y, out.y[a]);
    }
  }
}

// 1/sqrt(x) for a positive, normal x: the hardware estimate refined by two steps of
// Newton's method for f(y) = 1/y^2 - x (y <- y (3 - x y^2) / 2, each step squaring
// the relative error), so the result is within a few ulp.  Replaces a square root
// and a division (each a multi-instruction sequence in FP64) where both are needed.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

struct Kin {
  double u, w;       // velocity at the point
  double ux, uy, wx, wy;
  double t1, t2, t3; // m(tau(v))
  double delta;      // Delta = sqrt(Delta_min^2 + 2 m(tau).m(tau))
  double idelta;     // 1 / Delta
};

__device__ __forceinline__ Kin kinematics(const ElemConst& c, const Shape& s, const CellVel& v) {
  Kin k;
  k.u = k.w = k.ux = k.uy = k.wx = k.wy = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
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
  const double d2 = c.dmin2 + 2.0 * (k.t1 * k.t1 + k.t2 * k.t2 + k.t3 * k.t3);
  k.idelta = rsqrt_nr(d2);   // d2 >= Delta_min^2 > 0
  k.delta = d2 * k.idelta;
  return k;
}

// |w| and 1/|w| (0 and 0 for w = 0)
__device__ __forceinline__ void norm_inv(double wx, double wy, double& n, double& in) {
  const double n2 = wx * wx + wy * wy;
  in = n2 > 0.0 ? rsqrt_nr(n2) : 0.0;
  n = n2 * in;
}

__device__ __forceinline__ double interp(const Shape& s, const double f[4]) {
  return s.N[0] * f[0] + s.N[1] * f[1] + s.N[2] * f[2] + s.N[3] * f[3];
}

__device__ __forceinline__ bool is_boundary(const ElemConst& c, int i, int j) {
  return i == 0 || j == 0 || i == c.nx || j == c.ny;
}

}  // namespace

// ---------------------------------------------------------------------------
// per-step precompute: P, rho*H per cell; load vector F per node (eq. F)
// ---------------------------------------------------------------------------
__global__ void k_cell_coeffs(ElemConst c, const double* __restrict__ H, const double* __restrict__ A,
                              double* __restrict__ P, double* __restrict__ rhoH) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)c.nx * c.ny) return;
  const double h = H[e];
  P[e] = c.P_star * h * exp(-c.C_strength * (1.0 - A[e]));
  rhoH[e] = c.rho_ice * h;
}

__global__ void k_load_vector(ElemConst c, const double* __restrict__ rhoH,
                              const double* __restrict__ va, const double* __restrict__ vo,
                              const double* __restrict__ vn, double* __restrict__ F) {
  const size_t n = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (n >= (size_t)c.nxn * c.nyn) return;
  const int i = (int)(n % c.nxn), j = (int)(n / c.nxn);
  const double ihx = c.ihx, ihy = c.ihy;
  double fx = 0.0, fy = 0.0;
  for (int dyc = 0; dyc < 2; ++dyc)
    for (int dxc = 0; dxc < 2; ++dxc) {
      const int ci = i - 1 + dxc, cj = j - 1 + dyc;
      if (ci < 0 || cj < 0 || ci >= c.nx || cj >= c.ny) continue;
      const int a = (dxc ? 0 : 1) + (dyc ? 0 : 2);
      CellVel A_, O_, Nv;
      load_cell(c, va, nullptr, 0.0, ci, cj, A_);
      load_cell(c, vo, nullptr, 0.0, ci, cj, O_);
      load_cell(c, vn, nullptr, 0.0, ci, cj, Nv);
      const double rh = rhoH[(size_t)cj * c.nx + ci];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const Shape s = shape_at(q, ihx, ihy);
        const double ax = interp(s, A_.x), ay = interp(s, A_.y);
        const double ox = interp(s, O_.x), oy = interp(s, O_.y);
        const double nxq = interp(s, Nv.x), nyq = interp(s, Nv.y);
        const double sa = c.cda * sqrt(ax * ax + ay * ay);
        // rhoH v^n - dt rhoH f_c e_r x (v^n - v_o) + dt tau_atm,  e_r x u = (-u_y, u_x)
        const double gx_ = rh * nxq + c.dt * rh * c.fc * (nyq - oy) + c.dt * sa * ax;
        const double gy_ = rh * nyq - c.dt * rh * c.fc * (nxq - ox) + c.dt * sa * ay;
        fx = fma(c.wq * s.N[a], gx_, fx);
        fy = fma(c.wq * s.N[a], gy_, fy);
      }
    }
  reinterpret_cast<double2*>(F)[n] = make_double2(fx, fy);
}

// Count of invalid step data per workgroup: H negative or not finite, A outside
// [0, 1] or not finite, a velocity component not finite.  partials[b] (K = 1).
__global__ void __launch_bounds__(kBlock)
k_state_check(const double* __restrict__ H, const double* __restrict__ A, const double* __restrict__ va,
              const double* __restrict__ vo, const double* __restrict__ vprev, size_t ncell, size_t ndof,
              double* __restrict__ partials) {
  __shared__ double lds[16];
  double bad[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ncell; e += stride) {
    const double h = H[e], a = A[e];
    if (!(isfinite(h) && h >= 0.0)) bad[0] += 1.0;
    if (!(isfinite(a) && a >= 0.0 && a <= 1.0)) bad[0] += 1.0;
  }
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < ndof; e += stride)
    if (!(isfinite(va[e]) && isfinite(vo[e]) && isfinite(vprev[e]))) bad[0] += 1.0;
  block_sum<1>(bad, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = bad[0];
}

int launch_state_check(vp_ctx c, const double* H, const double* A, const double* va, const double* vo,
                       const double* vprev) {
  hipLaunchKernelGGL(k_state_check, dim3(kRedBlocks), dim3(kBlock), 0, c->stream, H, A, va, vo, vprev,
                     c->ncell, c->ndof, c->partials);
  VP_LAUNCH_CHECK();
  return kRedBlocks;
}

void launch_precompute(vp_ctx c, const double* H, const double* A, const double* va,
                       const double* vo, const double* vprev) {
  const size_t nc = c->ncell;
  hipLaunchKernelGGL(k_cell_coeffs, dim3((unsigned)((nc + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, c->ec, H, A, c->P, c->rhoH);
  VP_LAUNCH_CHECK();
  if (c->order == 2) {
    launch_q2_precompute(c, va, vo, vprev);
  } else {
    hipLaunchKernelGGL(k_load_vector, dim3(grid_for(c->nn)), dim3(kBlock), 0, c->stream, c->ec,
                       c->rhoH, va, vo, vprev, c->F);
    VP_LAUNCH_CHECK();
  }
  VP_HIP(hipMemcpyAsync(c->vo, vo, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  // the step's data, kept for the learned start's input features
  VP_HIP(hipMemcpyAsync(c->Hs, H, c->ncell * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  VP_HIP(hipMemcpyAsync(c->As, A, c->ncell * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  VP_HIP(hipMemcpyAsync(c->vas, va, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  VP_HIP(hipMemcpyAsync(c->vps, vprev, c->ndof * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
}

// ---------------------------------------------------------------------------
// Element patches.  A workgroup owns a tile of kTN x kTN nodes and the
// (kTN+1) x (kTN+1) = 256 cells around them (one cell per thread).  Phase 1:
// every thread evaluates its cell's four Gauss points once and leaves the
// cell's element contributions in LDS (plane per value: lds[k * 256 + cell]).
// Phase 2: every node thread sums, in a fixed order, what the (up to) four cells
// around it hold for it and writes its outputs.  Each cell is evaluated by at
// most four tiles at their seams (~1.14x on average) instead of by its four
// corner nodes (4x), and the sums are deterministic without atomics.
// Tile-local cell (cx, cy), cx, cy in [0, 16): global cell (i0 - 1 + cx, j0 - 1 + cy);
// tile-local node (x, y), x, y in [0, kTN): global node (i0 + x, j0 + y), whose
// cells are NE = (x+1, y+1) (node = its SW corner a=0), NW = (x, y+1) (a=1),
// SE = (x+1, y) (a=2), SW = (x, y) (a=3).
// ---------------------------------------------------------------------------
constexpr int kTC = 16;            // cells per tile side
constexpr int kTN = kTC - 1;       // nodes per tile side
constexpr int kTCells = kTC * kTC; // = threads per workgroup

inline dim3 tile_grid(const ElemConst& c) {
  return dim3((unsigned)((c.nxn + kTN - 1) / kTN), (unsigned)((c.nyn + kTN - 1) / kTN));
}

// The integral terms of one cell's residual element vector (corner a: x at ev[2a],
// y at ev[2a+1]) and its integrated energy density, by the cell's 2x2 Gauss rule.
__device__ __forceinline__ void cell_residual(const ElemConst& c, const CellVel& V, const CellVel& O, double Pc,
                                              double rh, double (&ev)[8], double& en) {
  const double ihx = c.ihx, ihy = c.ihy;
#pragma unroll 1   // fewer live registers (126 instead of 162), same speed or better
  for (int q = 0; q < 4; ++q) {
    const Shape s = shape_at(q, ihx, ihy);
    const Kin k = kinematics(c, s, V);
    // (P/Delta) tau(v):tau(phi) - (P/2) tr eps(phi), times dt
    const double kd = c.dt * Pc * k.idelta, hp = 0.5 * c.dt * Pc;
    const double Sx = kd * (c.c1 * k.t1 + c.c2 * k.t2) - hp;
    const double Sy = kd * (c.c2 * k.t1 + c.c1 * k.t2) - hp;
    const double Sxy = kd * c.s2e * k.t3;
    // mass and ocean drag: rhoH v - dt tau_ocean(v)
    const double wx_ = interp(s, O.x) - k.u, wy_ = interp(s, O.y) - k.w;
    double wn, iwn;
    norm_inv(wx_, wy_, wn, iwn);
    const double fx = rh * k.u - c.dt * c.cdo * wn * wx_;
    const double fy = rh * k.w - c.dt * c.cdo * wn * wy_;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ev[2 * a] += c.wq * (Sx * s.gx[a] + Sxy * s.gy[a] + fx * s.N[a]);
      ev[2 * a + 1] += c.wq * (Sy * s.gy[a] + Sxy * s.gx[a] + fy * s.N[a]);
    }
    en += c.wq * (0.5 * rh * (k.u * k.u + k.w * k.w) +
                  c.dt * (0.5 * Pc * (k.delta - (k.ux + k.wy)) + c.cdo * wn * wn * wn * (1.0 / 3.0)));
  }
}

// ---------------------------------------------------------------------------
// residual R(v) = A(v, phi) - F(phi) (eq. A with eq. sigma) and energy Phi (eq. energy)
// ---------------------------------------------------------------------------
// Cell values in LDS: 0..7 the element vector (corner a: x at 2a, y at 2a+1) of
// the integral terms, 8 the cell's integrated energy density.
__global__ void __launch_bounds__(kTCells)
k_residual(ElemConst c, const double* __restrict__ v, const double* __restrict__ dv, double alpha,
           const double* __restrict__ vo, const double* __restrict__ F,
           const double* __restrict__ P, const double* __restrict__ rhoH,
           double* __restrict__ r, double* __restrict__ partials) {
  __shared__ double cv[9 * kTCells];
  __shared__ double lds[16 * 3];
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * kTN, j0 = blockIdx.y * kTN;
  {
    const int ci = i0 - 1 + (t % kTC), cj = j0 - 1 + (t / kTC);
    double ev[8] = {0, 0, 0, 0, 0, 0, 0, 0}, en = 0.0;
    if (ci >= 0 && cj >= 0 && ci < c.nx && cj < c.ny) {
      CellVel V, O;
      load_cell(c, v, dv, alpha, ci, cj, V);
      load_cell(c, vo, nullptr, 0.0, ci, cj, O);
      const size_t e = (size_t)cj * c.nx + ci;
      cell_residual(c, V, O, P[e], rhoH[e], ev, en);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) cv[k * kTCells + t] = ev[k];
    cv[8 * kTCells + t] = en;
  }
  __syncthreads();
  double acc[3] = {0.0, 0.0, 0.0};
  const int x = t % kTN, y = t / kTN;
  const int i = i0 + x, j = j0 + y;
  if (t < kTN * kTN && i < c.nxn && j < c.nyn) {
    const int cNE = (y + 1) * kTC + x + 1, cNW = (y + 1) * kTC + x, cSE = y * kTC + x + 1, cSW = y * kTC + x;
    // corner a of the cells NE, NW, SE, SW is 0, 1, 2, 3 (cells outside the mesh hold 0)
    double rx = cv[0 * kTCells + cNE] + cv[2 * kTCells + cNW] + cv[4 * kTCells + cSE] + cv[6 * kTCells + cSW];
    double ry = cv[1 * kTCells + cNE] + cv[3 * kTCells + cNW] + cv[5 * kTCells + cSE] + cv[7 * kTCells + cSW];
    const size_t n = (size_t)j * c.nxn + i;
    const double2 Fn = reinterpret_cast<const double2*>(F)[n];
    double2 vn = reinterpret_cast<const double2*>(v)[n];
    if (dv) {
      const double2 d = reinterpret_cast<const double2*>(dv)[n];
      vn.x = fma(alpha, d.x, vn.x);
      vn.y = fma(alpha, d.y, vn.y);
    }
    rx -= Fn.x;
    ry -= Fn.y;
    if (is_boundary(c, i, j)) rx = ry = 0.0;
    if (r) reinterpret_cast<double2*>(r)[n] = make_double2(rx, ry);
    // the cell whose SW corner is this node is counted here (each cell once)
    const double ecell = cv[8 * kTCells + cNE];
    const double fv = Fn.x * vn.x + Fn.y * vn.y;
    acc[0] = rx * rx + ry * ry;
    acc[1] = ecell - fv;
    acc[2] = fabs(ecell) + fabs(fv);
  }
  block_sum<3>(acc, lds);
  if (t == 0) {
    const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    partials[b * 3 + 0] = acc[0];
    partials[b * 3 + 1] = acc[1];
    partials[b * 3 + 2] = acc[2];
  }
}




// ---------------------------------------------------------------------------
// operator assembly (eq. linearSVNewton + eq. modification; eq. standardNewton1/2)
// ---------------------------------------------------------------------------
// Per Gauss point the viscous part is a symmetric 3x3 Mandel matrix C:
//   svN : C = dt P/Delta [I - (a p^T + p a^T)/(Delta s)], a = m(tau(v_l)), p = m(pi_l),
//         s = max(1, sqrt(2 p.p))
//   stdN: C = dt P/Delta [I - 2 a a^T / Delta^2]
// and the mass/drag part is the symmetric 2x2 matrix
//   M = rhoH I + dt C_o rho_o (|w| I + w w^T / |w|),  w = v_o - v_l.
// The element block of corners (a, b) is sum_q wq [B_a^T C B_b + N_a N_b M], where
// B_a maps the two nodal dofs of corner a to m(tau(N_a e_d)).  A cell keeps its
// ten blocks with a <= b in LDS: the diagonal blocks as (xx, xy, yy) (symmetric),
// the others as [r][c] with the rows of corner a:
//   values  0.. 11: D0, D1, D2, D3          (diagonal blocks, 3 each)
//   values 12.. 35: B01, B23, B02, B13, B03, B12 (4 each)
// and the node sums self = D0(NE)+D1(NW)+D2(SE)+D3(SW), east = B01(NE)+B23(SE),
// north = B02(NE)+B13(NW), north-east = B03(NE), north-west = B12(NW).
namespace {
constexpr int kB01 = 12, kB23 = 16, kB02 = 20, kB13 = 24, kB03 = 28, kB12 = 32;

// acc[0..3] += B_a^T C B_b + N_a N_b M for corner b given X = B_a^T C (C and M
// already carry the Gauss weight)
__device__ __forceinline__ void add_block(const ElemConst& c, const Shape& s, int a, int b, const double X[6],
                                          double Mxx, double Mxy, double Myy, double* acc) {
  const double gxb = s.gx[b], gyb = s.gy[b];
  const double cx0 = c.c1 * gxb, cx1 = c.c2 * gxb, cx2 = c.s2e * gyb;
  const double cy0 = c.c2 * gyb, cy1 = c.c1 * gyb, cy2 = c.s2e * gxb;
  const double nn_ = s.N[a] * s.N[b];
  acc[0] += X[0] * cx0 + X[1] * cx1 + X[2] * cx2 + nn_ * Mxx;
  acc[1] += X[0] * cy0 + X[1] * cy1 + X[2] * cy2 + nn_ * Mxy;
  acc[2] += X[3] * cx0 + X[4] * cx1 + X[5] * cx2 + nn_ * Mxy;
  acc[3] += X[3] * cy0 + X[4] * cy1 + X[5] * cy2 + nn_ * Myy;
}

__device__ __forceinline__ void add_diag(const ElemConst& c, const Shape& s, int a, const double X[6],
                                         double Mxx, double Mxy, double Myy, double* acc) {
  const double gxb = s.gx[a], gyb = s.gy[a];
  const double cx0 = c.c1 * gxb, cx1 = c.c2 * gxb, cx2 = c.s2e * gyb;
  const double cy0 = c.c2 * gyb, cy1 = c.c1 * gyb, cy2 = c.s2e * gxb;
  const double nn_ = s.N[a] * s.N[a];
  acc[0] += X[0] * cx0 + X[1] * cx1 + X[2] * cx2 + nn_ * Mxx;
  acc[1] += X[0] * cy0 + X[1] * cy1 + X[2] * cy2 + nn_ * Mxy;
  acc[2] += X[3] * cy0 + X[4] * cy1 + X[5] * cy2 + nn_ * Myy;
}
}  // namespace

// The ten upper element blocks (a <= b) of one cell in the layout described
// above, by the cell's 2x2 Gauss rule; pi points at the cell's value of the first
// Mandel component at the first Gauss point (planes ncell apart), unused for stdN.
__device__ __forceinline__ void cell_blocks(const ElemConst& c, const CellVel& V, const CellVel& O, double Pc,
                                            double rh, int variant, const double* __restrict__ pi, size_t ncell,
                                            double (&acc)[36]) {
  const double ihx = c.ihx, ihy = c.ihy;
#pragma unroll 1   // 198 registers instead of 222 and ~3% faster (still two waves per SIMD)
  for (int q = 0; q < 4; ++q) {
    const Shape s = shape_at(q, ihx, ihy);
    const Kin k = kinematics(c, s, V);
    // C and M carry the Gauss weight wq
    const double base = c.wq * c.dt * Pc * k.idelta;
    double C11, C12, C13, C22, C23, C33;
    if (variant == VP_SVN) {
      const double p1 = pi[(size_t)(q * 3 + 0) * ncell];
      const double p2 = pi[(size_t)(q * 3 + 1) * ncell];
      const double p3 = kSqrt2 * pi[(size_t)(q * 3 + 2) * ncell];
      const double s2 = 2.0 * (p1 * p1 + p2 * p2 + p3 * p3);
      const double isn = s2 > 1.0 ? rsqrt_nr(s2) : 1.0;   // 1 / max(1, sqrt(2 p.p))
      const double f = base * k.idelta * isn;
      C11 = base - f * 2.0 * k.t1 * p1;
      C22 = base - f * 2.0 * k.t2 * p2;
      C33 = base - f * 2.0 * k.t3 * p3;
      C12 = -f * (k.t1 * p2 + p1 * k.t2);
      C13 = -f * (k.t1 * p3 + p1 * k.t3);
      C23 = -f * (k.t2 * p3 + p2 * k.t3);
    } else {
      const double f = 2.0 * base * k.idelta * k.idelta;
      C11 = base - f * k.t1 * k.t1;
      C22 = base - f * k.t2 * k.t2;
      C33 = base - f * k.t3 * k.t3;
      C12 = -f * k.t1 * k.t2;
      C13 = -f * k.t1 * k.t3;
      C23 = -f * k.t2 * k.t3;
    }
    const double wx_ = interp(s, O.x) - k.u, wy_ = interp(s, O.y) - k.w;
    double wn, iwn;
    norm_inv(wx_, wy_, wn, iwn);   // iwn = 0 for w = 0: the rank-one term vanishes
    const double dr = c.wq * c.dt * c.cdo;
    const double Mxx = c.wq * rh + dr * wn + dr * wx_ * wx_ * iwn;
    const double Myy = c.wq * rh + dr * wn + dr * wy_ * wy_ * iwn;
    const double Mxy = dr * wx_ * wy_ * iwn;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      // X = B_a^T C (2x3), B_a columns: dof x (c1 gx, c2 gx, s2e gy), dof y (c2 gy, c1 gy, s2e gx)
      const double gxa = s.gx[a], gya = s.gy[a];
      const double bx0 = c.c1 * gxa, bx1 = c.c2 * gxa, bx2 = c.s2e * gya;
      const double by0 = c.c2 * gya, by1 = c.c1 * gya, by2 = c.s2e * gxa;
      const double X[6] = {bx0 * C11 + bx1 * C12 + bx2 * C13, bx0 * C12 + bx1 * C22 + bx2 * C23,
                           bx0 * C13 + bx1 * C23 + bx2 * C33, by0 * C11 + by1 * C12 + by2 * C13,
                           by0 * C12 + by1 * C22 + by2 * C23, by0 * C13 + by1 * C23 + by2 * C33};
      add_diag(c, s, a, X, Mxx, Mxy, Myy, acc + 3 * a);
      if (a == 0) {
        add_block(c, s, 0, 1, X, Mxx, Mxy, Myy, acc + kB01);
        add_block(c, s, 0, 2, X, Mxx, Mxy, Myy, acc + kB02);
        add_block(c, s, 0, 3, X, Mxx, Mxy, Myy, acc + kB03);
      } else if (a == 1) {
        add_block(c, s, 1, 3, X, Mxx, Mxy, Myy, acc + kB13);
        add_block(c, s, 1, 2, X, Mxx, Mxy, Myy, acc + kB12);
      } else if (a == 2) {
        add_block(c, s, 2, 3, X, Mxx, Mxy, Myy, acc + kB23);
      }
    }
  }
}

// Write node (i, j)'s five stored blocks (self, E, N, NE, NW) with the Dirichlet
// rows and columns: identity at boundary nodes, no coupling to them.
__device__ __forceinline__ void store_node_blocks(const ElemConst& c, double* __restrict__ K, int i, int j,
                                                  const double (&blk)[5][4], float* __restrict__ K32 = nullptr) {
  const size_t nn = (size_t)c.nxn * c.nyn;
  const size_t n = (size_t)j * c.nxn + i;
  const bool bn = is_boundary(c, i, j);
  const int nbi[5] = {i, i + 1, i, i + 1, i - 1};
  const int nbj[5] = {j, j, j + 1, j + 1, j + 1};
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    bool zero;
    if (b == 0) zero = bn;
    else zero = bn || nbi[b] < 0 || nbi[b] > c.nx || nbj[b] > c.ny || is_boundary(c, nbi[b], nbj[b]);
    double val[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      val[k] = zero ? 0.0 : blk[b][k];
      if (b == 0 && bn) val[k] = (k == 0 || k == 3) ? 1.0 : 0.0;
    }
    // block-interleaved storage: the block's 4 values are contiguous (32 bytes)
    double2* dst = reinterpret_cast<double2*>(K + aidx(2, nn, b, n, 0, 0));
    dst[0] = make_double2(val[0], val[1]);
    dst[1] = make_double2(val[2], val[3]);
    if (K32)   // the FP32 copy the FP32 modes' AMG setup reads (the same rounding as a conversion)
      *reinterpret_cast<float4*>(K32 + aidx(2, nn, b, n, 0, 0)) =
          make_float4((float)val[0], (float)val[1], (float)val[2], (float)val[3]);
  }
}

template <int TCX, int TCY>
__global__ void __launch_bounds__(TCX * TCY)
k_assemble(ElemConst c, const double* __restrict__ v, const double* __restrict__ pi, int variant,
           const double* __restrict__ vo, const double* __restrict__ P,
           const double* __restrict__ rhoH, double* __restrict__ K, float* __restrict__ K32) {
  constexpr int NT = TCX * TCY, NX = TCX - 1, NY = TCY - 1;   // threads = cells; nodes NX x NY
  __shared__ double cv[36 * NT];
  const size_t ncell = (size_t)c.nx * c.ny;
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * NX, j0 = blockIdx.y * NY;
  {
    const int ci = i0 - 1 + (t % TCX), cj = j0 - 1 + (t / TCX);
    double acc[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) acc[k] = 0.0;
    if (ci >= 0 && cj >= 0 && ci < c.nx && cj < c.ny) {
      CellVel V, O;
      load_cell(c, v, nullptr, 0.0, ci, cj, V);
      load_cell(c, vo, nullptr, 0.0, ci, cj, O);
      const size_t e = (size_t)cj * c.nx + ci;
      cell_blocks(c, V, O, P[e], rhoH[e], variant, pi + e, ncell, acc);
    }
#pragma unroll
    for (int k = 0; k < 36; ++k) cv[k * NT + t] = acc[k];
  }
  __syncthreads();
  const int x = t % NX, y = t / NX;
  const int i = i0 + x, j = j0 + y;
  if (t >= NX * NY || i >= c.nxn || j >= c.nyn) return;
  const int cNE = (y + 1) * TCX + x + 1, cNW = (y + 1) * TCX + x, cSE = y * TCX + x + 1, cSW = y * TCX + x;
  auto at = [&](int k, int cell) { return cv[k * NT + cell]; };
  double blk[5][4];
  {
    const double sxx = ((at(0, cNE) + at(3, cNW)) + at(6, cSE)) + at(9, cSW);
    const double sxy = ((at(1, cNE) + at(4, cNW)) + at(7, cSE)) + at(10, cSW);
    const double syy = ((at(2, cNE) + at(5, cNW)) + at(8, cSE)) + at(11, cSW);
    blk[0][0] = sxx; blk[0][1] = sxy; blk[0][2] = sxy; blk[0][3] = syy;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    blk[1][k] = at(kB01 + k, cNE) + at(kB23 + k, cSE);
    blk[2][k] = at(kB02 + k, cNE) + at(kB13 + k, cNW);
    blk[3][k] = at(kB03 + k, cNE);
    blk[4][k] = at(kB12 + k, cNW);
  }
  store_node_blocks(c, K, i, j, blk, K32);
}


void launch_residual(vp_ctx c, const double* v, const double* dv, double alpha, double* r,
                     double* partials, unsigned* nblocks) {
  if (c->order == 2) {
    launch_q2_residual(c, v, dv, alpha, r, partials, nblocks);
    return;
  }
  const dim3 g = tile_grid(c->ec);
  hipLaunchKernelGGL(k_residual, g, dim3(kTCells), 0, c->stream, c->ec, v, dv, alpha, c->vo,
                     c->F, c->P, c->rhoH, r, partials);
  VP_LAUNCH_CHECK();
  *nblocks = g.x * g.y;
}

unsigned residual_blocks(const ElemConst& c) {
  const dim3 g = tile_grid(c);
  return g.x * g.y;
}

// K receives the Q1 operator; with Q2 elements the operator goes to c->K2 (the AMG
// builds its first coarse level from it and K is not used).
// When the last AMG setup ran in an FP32 mode (its hierarchy starts from an FP32
// copy of this operator), the assembly writes that copy too and the next setup
// skips the conversion.
void launch_assemble(vp_ctx c, const double* v, const double* pi, int variant, double* K) {
  c->a32_assembled = false;
  if (c->order == 2) {
    launch_q2_assemble(c, v, pi, variant);
    return;
  }
  float* K32 = nullptr;
  if (K == c->lev[0].A64 && c->lev[0].A32 && c->amg_kind == VP_AMG_SA &&
      (c->amg_prec == VP_PREC_FP32 || c->amg_prec == VP_PREC_FP32_BF16COARSE))
    K32 = c->lev[0].A32;
  constexpr int TX = kTC, TY = kTC;   // 8-row tiles measured no faster, 4-row tiles slower
  const dim3 g((unsigned)((c->ec.nxn + TX - 2) / (TX - 1)), (unsigned)((c->ec.nyn + TY - 2) / (TY - 1)));
  hipLaunchKernelGGL((k_assemble<TX, TY>), g, dim3(TX * TY), 0, c->stream, c->ec, v, pi, variant, c->vo, c->P,
                     c->rhoH, K, K32);
  VP_LAUNCH_CHECK();
  c->a32_assembled = K32 != nullptr;
}

// ---------------------------------------------------------------------------
// dual update (eq. tautilde with eq. modification) and consistent initialisation (eq. pi)
// ---------------------------------------------------------------------------
//   pi~ = -p + a/D + t~/D - [(a.t~) p + (p.t~) a] / (D^2 s)   (Mandel vectors)
__global__ void k_pi_update(ElemConst c, const double* __restrict__ v, const double* __restrict__ dv,
                            double* __restrict__ pi, double alpha) {
  const size_t ncell = (size_t)c.nx * c.ny;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const int ci = (int)(e % c.nx), cj = (int)(e / c.nx);
  const double ihx = c.ihx, ihy = c.ihy;
  CellVel V, D;
  load_cell(c, v, nullptr, 0.0, ci, cj, V);
  load_cell(c, dv, nullptr, 0.0, ci, cj, D);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const Shape s = shape_at(q, ihx, ihy);
    const Kin k = kinematics(c, s, V);
    const Kin kd = kinematics(c, s, D);
    double* pq = pi + (size_t)(q * 3) * ncell + e;
    const double p1 = pq[0], p2 = pq[ncell], p3 = kSqrt2 * pq[2 * ncell];
    const double sn = fmax(1.0, sqrt(2.0 * (p1 * p1 + p2 * p2 + p3 * p3)));
    const double id = k.idelta;
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

__global__ void k_pi_init(ElemConst c, const double* __restrict__ v, double* __restrict__ pi) {
  const size_t ncell = (size_t)c.nx * c.ny;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const int ci = (int)(e % c.nx), cj = (int)(e / c.nx);
  const double ihx = c.ihx, ihy = c.ihy;
  CellVel V;
  load_cell(c, v, nullptr, 0.0, ci, cj, V);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const Shape s = shape_at(q, ihx, ihy);
    const Kin k = kinematics(c, s, V);
    const double id = k.idelta;
    double* pq = pi + (size_t)(q * 3) * ncell + e;
    pq[0] = k.t1 * id;
    pq[ncell] = k.t2 * id;
    pq[2 * ncell] = k.t3 * id / kSqrt2;
  }
}

void launch_pi_update(vp_ctx c, const double* v, const double* dv, double* pi, double alpha) {
  if (c->order == 2) {
    launch_q2_pi_update(c, v, dv, pi, alpha);
    return;
  }
  hipLaunchKernelGGL(k_pi_update, dim3((unsigned)((c->ncell + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, c->stream, c->ec, v, dv, pi, alpha);
  VP_LAUNCH_CHECK();
}

void launch_pi_init(vp_ctx c, const double* v, double* pi) {
  if (c->order == 2) {
    launch_q2_pi_init(c, v, pi);
    return;
  }
  hipLaunchKernelGGL(k_pi_init, dim3((unsigned)((c->ncell + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     c->stream, c->ec, v, pi);
  VP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// transport of A and H (eq. model:A, eq. model:H): one explicit Euler step
// (Sec. 3) of cell-wise constant fields (finite volumes, Sec. 5) with the Q1
// velocity.  Face normal velocity = mean of the face's two nodal values (exact
// for Q1; Simpson's rule on the face's end and midpoint nodes for Q2), first-order
// upwind flux (v.n)|f| Q_up, no flux through the boundary
// (v = 0 there).  Each face flux is evaluated by both adjacent cells with the
// same operands, so the update is conservative.  A is clipped to [0, 1] and H to
// [0, inf).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_advect(const double* __restrict__ v, const double* __restrict__ A, const double* __restrict__ H, int nx,
         int ny, int order, double hx, double hy, double dt, double* __restrict__ Ao, double* __restrict__ Ho) {
  const size_t c = (size_t)xcd_block() * blockDim.x + threadIdx.x;
  if (c >= (size_t)nx * ny) return;
  const int i = (int)(c % nx), j = (int)(c / nx);
  const double2* V = reinterpret_cast<const double2*>(v);
  double uw, ue, us, un;
  if (order == 2) {
    // Q2 velocity: Simpson's rule on each face's end and midpoint nodes
    const size_t nxn = (size_t)2 * nx + 1;
    auto at = [&](int I, int J) { return V[(size_t)J * nxn + I]; };
    const int I0 = 2 * i, J0 = 2 * j;
    uw = i > 0 ? (at(I0, J0).x + 4.0 * at(I0, J0 + 1).x + at(I0, J0 + 2).x) / 6.0 : 0.0;
    ue = i < nx - 1 ? (at(I0 + 2, J0).x + 4.0 * at(I0 + 2, J0 + 1).x + at(I0 + 2, J0 + 2).x) / 6.0 : 0.0;
    us = j > 0 ? (at(I0, J0).y + 4.0 * at(I0 + 1, J0).y + at(I0 + 2, J0).y) / 6.0 : 0.0;
    un = j < ny - 1 ? (at(I0, J0 + 2).y + 4.0 * at(I0 + 1, J0 + 2).y + at(I0 + 2, J0 + 2).y) / 6.0 : 0.0;
  } else {
    const size_t nxn = (size_t)nx + 1;
    const double2 v00 = V[(size_t)j * nxn + i], v10 = V[(size_t)j * nxn + i + 1];
    const double2 v01 = V[(size_t)(j + 1) * nxn + i], v11 = V[(size_t)(j + 1) * nxn + i + 1];
    uw = i > 0 ? 0.5 * (v00.x + v01.x) : 0.0;
    ue = i < nx - 1 ? 0.5 * (v10.x + v11.x) : 0.0;
    us = j > 0 ? 0.5 * (v00.y + v10.y) : 0.0;
    un = j < ny - 1 ? 0.5 * (v01.y + v11.y) : 0.0;
  }
  const double s = dt / (hx * hy);
  const double* Q[2] = {A, H};
  double out[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const double* q = Q[f];
    const double qc = q[c];
    const double qw = i > 0 ? q[c - 1] : qc, qe = i < nx - 1 ? q[c + 1] : qc;
    const double qs = j > 0 ? q[c - nx] : qc, qn = j < ny - 1 ? q[c + nx] : qc;
    const double Fw = uw * hy * (uw > 0.0 ? qw : qc), Fe = ue * hy * (ue > 0.0 ? qc : qe);
    const double Fs = us * hx * (us > 0.0 ? qs : qc), Fn = un * hx * (un > 0.0 ? qc : qn);
    out[f] = qc - s * ((Fe - Fw) + (Fn - Fs));
  }
  Ao[c] = fmin(fmax(out[0], 0.0), 1.0);
  Ho[c] = fmax(out[1], 0.0);
}

void launch_advect(vp_ctx c, const double* v, const double* A, const double* H, double* Ao, double* Ho) {
  hipLaunchKernelGGL(k_advect, dim3(grid_for(c->ncell)), dim3(kBlock), 0, c->stream, v, A, H, c->ec.nx, c->ec.ny,
                     c->order, c->ec.hx, c->ec.hy, c->ec.dt, Ao, Ho);
  VP_LAUNCH_CHECK();
}

}  // namespace vp
