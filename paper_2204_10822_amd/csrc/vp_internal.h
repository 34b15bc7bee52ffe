// Internal declarations shared by the libvp translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <type_traits>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vp.h"

namespace vp {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define VP_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::vp::Error(e_ == hipErrorOutOfMemory ? VP_ENOMEM : VP_EHIP,          \
                        std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define VP_LAUNCH_CHECK() VP_HIP(hipGetLastError())

constexpr int kBlock = 256;     // threads per workgroup for node/vector kernels
constexpr int kRedBlocks = 512; // workgroups of a grid-stride reduction
constexpr int kDotBlocks = 2048; // workgroups of the V-cycle output + dot products
constexpr int kMaxLevels = 16;
constexpr int kMaxRestart = 64;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum K values over the workgroup (blockDim.x a multiple of 64, <= 1024); the
// result is valid in thread 0.  Fixed order => deterministic.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds /* >= 16*K */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[wid * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[w * K + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Remap the linear workgroup id so that each of the 8 XCDs (which receive
// workgroups round-robin) processes one contiguous eighth of the index range;
// neighbouring rows of a structured grid then share that XCD's L2.
// Requires gridDim.x % 8 == 0 (launchers round the grid up).
__device__ __forceinline__ unsigned xcd_block() {
  const unsigned b = blockIdx.x, g = gridDim.x;
  return (b & 7u) * (g >> 3) + (b >> 3);
}

inline unsigned grid_for(size_t n, int block = kBlock) {
  size_t g = (n + block - 1) / block;
  g = (g + 7) / 8 * 8;
  if (g == 0) g = 8;
  return (unsigned)g;
}

// Operator storage (every level): block-interleaved, five B x B blocks per node
// (self, E, N, NE, NW), each block's B*B values contiguous:
//   A[aidx(B, nn, blk, n, r, c)] = ((blk * nn + n) * B + r) * B + c
// so a 2x2 FP32 block is one 16-byte load and a wave reads contiguous memory.
__host__ __device__ __forceinline__ size_t aidx(int B, size_t nn, int blk, size_t n, int r, int c) {
  return (((size_t)blk * nn + n) * B + r) * B + c;
}
// Smoothed prolongator: per fine node 4 slots x (B x 3), one plane per
// (slot, row, column) component so consecutive nodes are consecutive in memory:
//   P[pidx(B, nn, s, n, r, c)] = ((s * B + r) * 3 + c) * nn + n
__host__ __device__ __forceinline__ size_t pidx(int B, size_t nn, int s, size_t n, int r, int c) {
  return (size_t)((s * B + r) * 3 + c) * nn + n;
}

// Symmetric block 25-point stencil of Q2 elements: 13 stored blocks per node, the
// self block (dir 0) and the forward offsets (1,0), (2,0), (-2..2, 1), (-2..2, 2).
__host__ __device__ constexpr int q2_ox(int dir) { return dir == 0 ? 0 : dir <= 2 ? dir : (dir - 3) % 5 - 2; }
__host__ __device__ constexpr int q2_oy(int dir) { return dir <= 2 ? 0 : (dir - 3) / 5 + 1; }

// bf16 storage helpers (round to nearest even)
__device__ __forceinline__ float ld(const float* p) { return *p; }
__device__ __forceinline__ double ld(const double* p) { return *p; }
__device__ __forceinline__ float ld(const __hip_bfloat16* p) { return __bfloat162float(*p); }
__device__ __forceinline__ float ld(const _Float16* p) { return (float)*p; }

// ---------------------------------------------------------------------------
// element constants (uniform structured mesh, 2x2 Gauss)
// ---------------------------------------------------------------------------
struct ElemConst {
  int nx, ny, nxn, nyn;
  double hx, hy, wq;             // wq = hx*hy/4, the weight of each Gauss point
  double dt, dmin2;              // dt, Delta_min^2
  double c1, c2, s2e;            // tau map: c1 = (1+1/e)/2, c2 = (1-1/e)/2, s2e = 1/(sqrt2 e)
  double rho_ice, cdo, cda, fc;  // rho_ice, C_o rho_o, C_a rho_a, f_c
  double P_star, C_strength;
  double ihx, ihy;               // 1/hx, 1/hy
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Level {
  int nxn = 0, nyn = 0, B = 2;   // node grid and dofs per node
  size_t nn = 0;                 // nodes
  // operator: 5*B*B planes of nn values (self, E, N, NE, NW blocks)
  double* A64 = nullptr;
  float* A32 = nullptr;
  __hip_bfloat16* Abf = nullptr; // Jacobi-scaled values (mixed+bf16 mode, levels >= 1)
  _Float16* Ah = nullptr;         // Jacobi-scaled FP16 values (finest level, FP16 mode)
  _Float16* Ph = nullptr;         // FP16 copy of the scaled prolongator (finest level, FP16 modes)
  double* dsc64 = nullptr;       // sqrt(diag A) per dof (bf16 mode, levels >= 1)
  bool own_A64 = true;
  // transfer to the next level (aggregation of 3x3 nodes)
  int ncx = 0, ncy = 0;
  double* Ptent = nullptr;       // [B*3][nn]  own-aggregate tentative block per node
  double* P64 = nullptr;         // [4 slots][B*3][nn] smoothed prolongator
  float* P32 = nullptr;
  float* P32u = nullptr;         // unscaled FP32 prolongator (finest level, FP32 + BF16-coarse mode)
  bool p64_stale = false;        // finest level of the FP32 modes: the prolongator exists in FP32 only
  double* Bnull = nullptr;       // near-null space at this level [B*3][nn] (levels >= 1)
  double* lmax = nullptr;        // device scalar: bound on lmax(D^-1 A)
  double* pv0 = nullptr;         // power-iteration vectors (FP64, B*nn), warm across setups
  double* pv1 = nullptr;
  double* pnrm = nullptr;        // device [2]: squared norms of the power iterates
  bool pv_warm = false;          // pv0 holds the previous setup's iterate
  double lmax_h = 0.0;
  // V-cycle vectors, B*nn each, in the V-cycle precision
  void* x = nullptr; void* b = nullptr; void* r = nullptr; void* d0 = nullptr; void* d1 = nullptr;
  void* r2 = nullptr; void* x2 = nullptr;   // second residual / iterate (finest level, paired sweeps)
  // coarsest level: dense inverse (row-major, ndof x ndof)
  double* Ainv64 = nullptr;
  float* Ainv32 = nullptr;
};

}  // namespace vp

namespace vp {
// HIP-event timing of selected launches (see vp_profile)
struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev;   // pool, two events per record
  std::vector<int> kid;         // kernel id per record
  size_t used = 0;
};
}  // namespace vp

namespace vp {
struct RSHier;
}

struct vp_ctx_s {
  vp::Prof prof;
  vp_problem_desc desc{};
  hipStream_t stream = nullptr;
  int device = 0;
  int walk4_resident[2][2] = {{0, 0}, {0, 0}};   // workgroups of k_cheb_walk4 resident at once ([FP64][kind])
  int walk3_resident = 0;                          // workgroups of k_cheb_walk3 resident at once
  vp::ElemConst ec{};
  size_t nn = 0, ncell = 0, ndof = 0;
  int order = 1;                   // velocity elements: 1 = Q1, 2 = Q2
  double* K2 = nullptr;            // Q2: the operator, 13 blocks per node
  float* K2_32 = nullptr;          // Q2: FP32 copy for the V-cycle's finest level
  double* lmax_q2 = nullptr;       // Q2: lmax(D^{-1} K2) for the finest smoother (device)
  double lmax_q2_h = 0.0;
  double *pq0 = nullptr, *pq1 = nullptr, *pqn = nullptr;  // Q2: its power-iteration vectors
  bool pq_warm = false;
  std::string err;
  // state
  double* P = nullptr;      // [ncell]
  double* rhoH = nullptr;   // [ncell]
  double* F = nullptr;      // [ndof]
  double* vo = nullptr;     // [ndof]
  double *Hs = nullptr, *As = nullptr;    // copies of the step's H, A [ncell]
  double *vas = nullptr, *vps = nullptr;  // copies of v_air, v_prev [ndof]
  bool have_state = false;
  double rnorm_zero = -1.0;
  // operator
  bool have_K = false;
  // AMG
  int nlev = 0;
  vp::Level lev[vp::kMaxLevels];
  bool amg_ready = false;
  bool amg_struct = false;
  int amg_prec = 0;
  bool a32_assembled = false;      // the last assembly also wrote lev[0].A32 (FP32 copy, FP32 modes)
  int amg_kind = 0;                // VP_AMG_SA or VP_AMG_RS
  bool sa_vec64 = false;           // the SA V-cycle vectors are FP64
  bool ph_transfers = false;       // finest restriction/prolongation read the FP16 prolongator
  vp::RSHier* rs = nullptr;        // classical AMG hierarchy
  int cheb_degree = 3;
  int tail_level = -1;             // first level run by the single-workgroup tail kernel
  bool pair_sweeps = true;         // finest-level smoother sweeps fused in pairs
  bool tail_lds = true;            // FP32-vector tail with LDS vectors and register blocks
  int amg_variant = 0;             // VP_AMG_VAR_* flags of the last setup (verification)
  int walk4_rows = 0;              // fixed strip height of the four-sweep walk (0 = automatic)
  double cheb_ratio = 30.0;
  int max_coarse = 140;
  int power_its_cold = 16, power_its_warm = 6;
  double power_factor = 1.15;
  // scratch
  double* partials = nullptr;      // [kRedBlocks * 64]
  double* dscal = nullptr;         // device scalars [256]
  double* hscal = nullptr;         // pinned host scalars [256]
  double* work = nullptr;          // [6*ndof] Newton/line-search temporaries
  double* kv = nullptr;            // Krylov bases [(2*restart+1 + 4) * ndof]
  double* static_ws = nullptr;     // device address of the static workspace (allocation-free solve)
  int kv_restart = 0;
  double* dense = nullptr;         // coarse dense matrix scratch
  double* lmax_all = nullptr;      // the levels' spectral bounds gathered for one copy to the host
  double* gal_work = nullptr;      // A P per fine node for the Galerkin product [9*3*B*nn]
  // Newton history (Eisenstat-Walker state)
  double ew_rn_prev = -1.0, ew_eta_prev = 0.1;
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
namespace vp {
// Bracket a launch (or a nested group of launches) with events when profiling is
// on.  prof_begin returns the record index for prof_end (-1 when off).
inline int prof_begin(vp_ctx c, int kid) {
  Prof& p = c->prof;
  if (!p.on) return -1;
  const size_t idx = p.used++;
  while (p.ev.size() < 2 * p.used) {
    hipEvent_t e;
    VP_HIP(hipEventCreate(&e));
    p.ev.push_back(e);
  }
  if (p.kid.size() < p.used) p.kid.resize(p.used);
  p.kid[idx] = kid;
  VP_HIP(hipEventRecord(p.ev[2 * idx], c->stream));
  return (int)idx;
}
inline void prof_end(vp_ctx c, int idx) {
  if (idx < 0) return;
  VP_HIP(hipEventRecord(c->prof.ev[2 * (size_t)idx + 1], c->stream));
}
void launch_precompute(vp_ctx c, const double* H, const double* A, const double* va,
                       const double* vo, const double* vprev);
// residual/energy at v + alpha*dv (dv may be null); writes r (nullable) and
// 3 partial sums per workgroup: |R|^2, Phi, sum|Phi terms|
void launch_residual(vp_ctx c, const double* v, const double* dv, double alpha, double* r,
                     double* partials, unsigned* nblocks);
void launch_assemble(vp_ctx c, const double* v, const double* pi, int variant, double* K);
void launch_pi_update(vp_ctx c, const double* v, const double* dv, double* pi, double alpha);
void launch_pi_init(vp_ctx c, const double* v, double* pi);
// workgroups of the Q1 residual kernel (one per element-patch tile)
unsigned residual_blocks(const ElemConst& c);
// per-workgroup counts of invalid step data into c->partials (K = 1); returns the workgroups
int launch_state_check(vp_ctx c, const double* H, const double* A, const double* va, const double* vo,
                       const double* vprev);
// Phi(v) of eq. energy on the context's state (synchronises); VP_ENONFINITE if not finite
double energy_at(vp_ctx c, const double* v);
void launch_advect(vp_ctx c, const double* v, const double* A, const double* H, double* Ao, double* Ho);
// Q2 velocity elements
void launch_q2_precompute(vp_ctx c, const double* va, const double* vo, const double* vprev);
void launch_q2_residual(vp_ctx c, const double* v, const double* dv, double alpha, double* r, double* partials,
                        unsigned* nblocks);
void launch_q2_assemble(vp_ctx c, const double* v, const double* pi, int variant);
void launch_q2_apply(vp_ctx c, const double* x, double* y, double* partials);
// classical AMG (vp_rs.hip)
void rs_setup(vp_ctx c, double theta, double max_row_sum, int sweeps, int max_coarse);
void rs_apply(vp_ctx c, const double* r, double* z);
void rs_free(vp_ctx c);
int rs_levels(vp_ctx c);
void rs_info(vp_ctx c, int level, long long* out);
void rs_export(vp_ctx c, int level, int* A_ptr, int* A_col, double* A_val, int* cf, int* P_ptr, int* P_col,
               double* P_val, int* colour);
void launch_q2_pi_update(vp_ctx c, const double* v, const double* dv, double* pi, double alpha);
void launch_q2_pi_init(vp_ctx c, const double* v, double* pi);
// the Krylov operator of the context: the Q1 stencil in lev[0], or the Q2 operator
int launch_apply_K(vp_ctx c, const double* x, double* y, double* partials);

// reductions / BLAS-1 (vector length n doubles)
void launch_finish_sum(hipStream_t s, const double* partials, int nblocks, int K, double* out,
                       const double* msrc = nullptr, double* mdst = nullptr, int mn = 0);
void launch_dot(hipStream_t s, const double* x, const double* y, size_t n, double* partials);
void launch_mdot(hipStream_t s, const double* V, size_t ld, int nv, const double* w, size_t n,
                 double* partials);
void launch_maxpy_mdot(hipStream_t s, const double* V, size_t ld, int nv, const double* h,
                       double* w, size_t n, double* partials);
void launch_maxpy_scale(hipStream_t s, const double* V, size_t ld, int nv, const double* h,
                        const double* w, const double* nrm2, double* out, size_t n);
void launch_gemv_add(hipStream_t s, const double* Z, size_t ld, int nz, const double* y,
                     double* x, size_t n);
void launch_axpby(hipStream_t s, double a, const double* x, double b, double* y, size_t n);
void launch_scale_copy(hipStream_t s, const double* x, const double* scal, int invert,
                       double* y, size_t n);
int launch_fcg_update(hipStream_t s, const double* dev, double* x, double* r, const double* p,
                      const double* q, size_t n, double* partials, float* r32 = nullptr,
                      const double* dsc = nullptr);
void launch_fcg_dir(hipStream_t s, double* dev, const double* z, double* p, size_t n, int first);
void launch_fcg_dir32(hipStream_t s, double* dev, const float* x32, const double* dsc, double* p, size_t n,
                      int first);
void launch_cast(hipStream_t s, const double* x, float* y, size_t n);
template <typename TX>
int launch_out_dots(hipStream_t s, const TX* x, const double* dsc, double* z, const double* r, const double* q,
                    size_t n, double* partials);
void launch_cast(hipStream_t s, const float* x, double* y, size_t n);
void launch_fill(hipStream_t s, double* x, double v, size_t n);

// structured stencil operators (AMG levels)
template <typename TM, typename TV>
void launch_stencil_residual(hipStream_t s, const Level& L, const TM* A, const TV* x, const TV* b,
                             TV* r);
// y = A x on the finest level (FP64), x.y partials; returns the number of partials
int launch_apply_fine(hipStream_t s, const Level& L, const double* x, double* y, double* partials);
}  // namespace vp
