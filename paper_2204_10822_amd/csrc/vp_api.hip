// C ABI of libvp: context, state, residual, assembly, AMG, Krylov and Newton.
#include "vp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

namespace vp {
void amg_free(vp_ctx c);
void amg_export_p(vp_ctx c, int level, double* P);
void amg_build_structure(vp_ctx c, double* K, int max_coarse);
void amg_setup_numeric(vp_ctx c, int precision, double omega_scale);
void amg_apply(vp_ctx c, const double* r, double* z);
int amg_apply_dots(vp_ctx c, const double* r, const double* q, double* z, bool input_ready);
float* amg_input32(vp_ctx c, const double** dsc);
const float* amg_output32(vp_ctx c, const double** dsc);
void amg_reset_estimates(vp_ctx c);
}  // namespace vp

using namespace vp;

// Workspace of vp_krylov_solve_noalloc: the four flexible-CG vectors (r, q, z, p) of
// at most kNoAllocDofs doubles each (72 MiB), one copy per GPU, held until the
// process ends.  Host code never passes this name to a kernel: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress, per device.
static constexpr size_t kNoAllocDofs = 2359296;
static __device__ __align__(256) double scratch[4 * kNoAllocDofs];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device;
// resolved once per device.
double* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(VP_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    VP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(VP_EHIP, "hipGetSymbolAddress returned no address for the Krylov workspace");
    g_scratch_dev[device] = static_cast<double*>(p);
  }
  return g_scratch_dev[device];
}

thread_local std::string g_create_error;

template <typename F>
int guarded(vp_ctx c, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    if (c) c->err = e.what();
    else g_create_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    else g_create_error = e.what();
    return VP_EHIP;
  } catch (...) {
    if (c) c->err = "unknown error";
    return VP_EHIP;
  }
}

void require(bool ok, int code, const char* msg) {
  if (!ok) throw Error(code, msg);
}

template <typename T>
T* dalloc(size_t n) {
  void* p = nullptr;
  VP_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
  return static_cast<T*>(p);
}

size_t partial_slots(vp_ctx c) {
  const size_t red = std::max<size_t>((size_t)kRedBlocks * (kMaxRestart + 4), 3 * (size_t)grid_for(c->nn) + 64);
  return std::max<size_t>(red, 3 * (size_t)residual_blocks(c->ec) + 64);
}

// sum the first K partial columns of nblocks workgroups into dscal[off..off+K)
void finish(vp_ctx c, int nblocks, int K, int off) {
  launch_finish_sum(c->stream, c->partials, nblocks, K, c->dscal + off);
}

// finish into dscal[off..off+K) and hand dscal[0..mn) to the host (pinned scalars
// written by the finishing kernel itself), then wait for the stream
void finish_fetch(vp_ctx c, int nblocks, int K, int off, int mn) {
  launch_finish_sum(c->stream, c->partials, nblocks, K, c->dscal + off, c->dscal, c->hscal, mn);
  VP_HIP(hipStreamSynchronize(c->stream));
}

void fetch(vp_ctx c, int off, int K) {
  VP_HIP(hipMemcpyAsync(c->hscal + off, c->dscal + off, K * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  VP_HIP(hipStreamSynchronize(c->stream));
}

struct ResidOut {
  double rnorm, energy, eabs;
};

ResidOut residual_eval(vp_ctx c, const double* v, const double* dv, double alpha, double* r) {
  unsigned g = 0;
  const int pr = prof_begin(c, VP_KID_RESIDUAL);
  launch_residual(c, v, dv, alpha, r, c->partials, &g);
  prof_end(c, pr);
  finish(c, (int)g, 3, 0);
  fetch(c, 0, 3);
  ResidOut o{std::sqrt(std::max(c->hscal[0], 0.0)), c->hscal[1], c->hscal[2]};
  if (!std::isfinite(o.rnorm) || !std::isfinite(o.energy))
    throw Error(VP_ENONFINITE, "non-finite residual norm or energy");
  return o;
}

}  // namespace

double vp::energy_at(vp_ctx c, const double* v) {
  if (!c->have_state) throw Error(VP_ESTATE, "vp_set_state not called");
  return residual_eval(c, v, nullptr, 0.0, nullptr).energy;
}

namespace {

double norm2(vp_ctx c, const double* x, size_t n) {
  launch_dot(c->stream, x, x, n, c->partials);
  finish(c, kRedBlocks, 1, 0);
  fetch(c, 0, 1);
  return std::sqrt(std::max(c->hscal[0], 0.0));
}

double rnorm_zero(vp_ctx c) {
  if (c->rnorm_zero < 0.0) {
    double* z = c->work + 4 * c->ndof;
    launch_fill(c->stream, z, 0.0, c->ndof);
    c->rnorm_zero = residual_eval(c, z, nullptr, 0.0, nullptr).rnorm;
  }
  return c->rnorm_zero;
}

void ensure_krylov(vp_ctx c, int restart) {
  if (c->kv && c->kv_restart >= restart) return;
  if (c->kv) (void)hipFree(c->kv);
  c->kv = nullptr;
  c->kv = dalloc<double>((size_t)(2 * restart + 4) * c->ndof);
  c->kv_restart = restart;
}

// ---------------------------------------------------------------------------
// FGMRES(m), right preconditioned, CGS2 with one host synchronisation per iteration
// ---------------------------------------------------------------------------
}  // namespace

int vp::launch_apply_K(vp_ctx c, const double* x, double* y, double* partials) {
  if (c->order == 2) {
    launch_q2_apply(c, x, y, partials);
    return (int)grid_for(c->nn);
  }
  return launch_apply_fine(c->stream, c->lev[0], x, y, partials);
}

namespace {

int fgmres(vp_ctx c, const double* b, double* x, const vp_krylov_opts& o, vp_krylov_info* info) {
  const size_t n = c->ndof;
  const int m = o.restart;
  ensure_krylov(c, m);
  double* V = c->kv;                       // m+1 vectors
  double* Z = c->kv + (size_t)(m + 1) * n; // m vectors
  double* w = Z + (size_t)m * n;           // 1 vector
  hipStream_t s = c->stream;
  const double bnorm = norm2(c, b, n);
  if (info) { info->iters = 0; info->rel_resid = 0.0; }
  if (bnorm == 0.0) {
    launch_fill(s, x, 0.0, n);
    return VP_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), y(m);
  int total = 0;
  double rel = 1.0;
  while (true) {
    // r0 = b - K x  -> V0 = r0 / |r0|
    launch_apply_K(c, x, w, nullptr);
    launch_axpby(s, 1.0, b, -1.0, w, n);
    const double beta = norm2(c, w, n);
    rel = beta / bnorm;
    if (rel <= o.rtol || total >= o.maxit) break;
    launch_axpby(s, 1.0 / beta, w, 0.0, V, n);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    bool done = false;
    for (; j < m && total < o.maxit; ++j) {
      double* vj = V + (size_t)j * n;
      double* zj = Z + (size_t)j * n;
      amg_apply(c, vj, zj);
      const int pr = prof_begin(c, VP_KID_APPLY_FINE);
      launch_apply_K(c, zj, w, nullptr);
      prof_end(c, pr);
      const int nv = j + 1;
      // pass 1: h1 = V^T w
      launch_mdot(s, V, n, nv, w, n, c->partials);
      finish(c, kRedBlocks, nv, 0);
      // pass 2: w -= V h1 ; h2 = V^T w, |w|^2
      launch_maxpy_mdot(s, V, n, nv, c->dscal, w, n, c->partials);
      finish(c, kRedBlocks, nv + 1, 100);
      // pass 3: v_{j+1} = (w - V h2) / sqrt(|w|^2 - |h2|^2)
      launch_maxpy_scale(s, V, n, nv, c->dscal + 100, w, c->dscal + 100 + nv, V + (size_t)(j + 1) * n, n);
      fetch(c, 0, 100 + nv + 1);
      double hh = c->hscal[100 + nv];
      for (int k = 0; k < nv; ++k) {
        const double h2 = c->hscal[100 + k];
        H[(size_t)k * m + j] = c->hscal[k] + h2;
        hh -= h2 * h2;
      }
      for (int k = 0; k <= nv; ++k)
        if (!std::isfinite(c->hscal[k < nv ? k : 100 + nv]))
          throw Error(VP_ENONFINITE, "non-finite Krylov scalar");
      const double hnext = hh > 0.0 ? std::sqrt(hh) : 0.0;
      H[(size_t)(j + 1) * m + j] = hnext;
      // Givens rotations
      for (int k = 0; k < j; ++k) {
        const double a = H[(size_t)k * m + j], bb = H[(size_t)(k + 1) * m + j];
        H[(size_t)k * m + j] = cs[k] * a + sn[k] * bb;
        H[(size_t)(k + 1) * m + j] = -sn[k] * a + cs[k] * bb;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      const double rr = std::hypot(a, bb);
      if (rr == 0.0) throw Error(VP_EBREAKDOWN, "FGMRES breakdown");
      cs[j] = a / rr;
      sn[j] = bb / rr;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      rel = std::fabs(g[j + 1]) / bnorm;
      if (rel <= o.rtol || hnext <= 1e-14 * std::fabs(g[0])) {
        ++j;
        done = true;
        break;
      }
    }
    // y = H^{-1} g, x += Z y
    const int k = j;
    for (int r = k - 1; r >= 0; --r) {
      double t = g[r];
      for (int q = r + 1; q < k; ++q) t -= H[(size_t)r * m + q] * y[q];
      y[r] = t / H[(size_t)r * m + r];
    }
    // the pinned staging area is read by the copy engine: synchronise before reuse
    std::memcpy(c->hscal + 300, y.data(), k * sizeof(double));
    VP_HIP(hipMemcpyAsync(c->dscal + 180, c->hscal + 300, k * sizeof(double), hipMemcpyHostToDevice, s));
    launch_gemv_add(s, Z, n, k, c->dscal + 180, x, n);
    VP_HIP(hipStreamSynchronize(s));
    if (done || total >= o.maxit) {
      // true residual for the report
      launch_apply_K(c, x, w, nullptr);
      launch_axpby(s, 1.0, b, -1.0, w, n);
      rel = norm2(c, w, n) / bnorm;
      break;
    }
  }
  if (info) { info->iters = total; info->rel_resid = rel; }
  return rel <= o.rtol * 1.0001 ? VP_OK : VP_KRYLOV_MAXIT;
}

// ---------------------------------------------------------------------------
// flexible CG (Polak-Ribiere form), one host synchronisation per iteration
// dscal layout: [0] r.z  [1] p.q  [4] r.r  [5] z.r new  [6] z.q
// ---------------------------------------------------------------------------
// ws: four vectors of ndof doubles (r, q, z, p)
int fcg(vp_ctx c, const double* b, double* x, const vp_krylov_opts& o, vp_krylov_info* info, double* ws) {
  const size_t n = c->ndof;
  double* r = ws;             // r and q adjacent: mdot over [r, q]
  double* q = r + n;
  double* z = q + n;
  double* p = z + n;
  hipStream_t s = c->stream;
  const double bnorm = norm2(c, b, n);
  if (info) { info->iters = 0; info->rel_resid = 0.0; }
  if (bnorm == 0.0) {
    launch_fill(s, x, 0.0, n);
    return VP_OK;
  }
  launch_apply_K(c, x, r, nullptr);
  launch_axpby(s, 1.0, b, -1.0, r, n);
  double rel = norm2(c, r, n) / bnorm;
  int it = 0;
  if (rel > o.rtol) {
    const double* dsc = nullptr;
    float* r32 = amg_input32(c, &dsc);  // the update writes the V-cycle's FP32 input directly
    const double* zdsc = nullptr;
    const float* z32 = amg_output32(c, &zdsc);  // the direction reads the V-cycle's FP32 output directly
    auto direction = [&](int first) {
      if (z32) launch_fcg_dir32(s, c->dscal, z32, zdsc, p, n, first);
      else launch_fcg_dir(s, c->dscal, z, p, n, first);
    };
    int nb = amg_apply_dots(c, r, nullptr, z32 ? nullptr : z, false);  // r.z
    finish(c, nb, 1, 0);
    direction(1);
    while (it < o.maxit) {
      const int pr = prof_begin(c, VP_KID_APPLY_FINE);
      const int nbq = launch_apply_K(c, p, q, c->partials);  // q = K p, p.q
      prof_end(c, pr);
      finish(c, nbq, 1, 1);
      nb = launch_fcg_update(s, c->dscal, x, r, p, q, n, c->partials, r32, dsc);
      finish_fetch(c, nb, 1, 4, 5);
      ++it;
      if (!std::isfinite(c->hscal[4]) || !std::isfinite(c->hscal[1]))
        throw Error(VP_ENONFINITE, "non-finite Krylov scalar");
      if (c->hscal[1] <= 0.0) throw Error(VP_EBREAKDOWN, "FCG breakdown: p.Kp <= 0");
      rel = std::sqrt(std::max(c->hscal[4], 0.0)) / bnorm;
      if (rel <= o.rtol) break;
      nb = amg_apply_dots(c, r, q, z32 ? nullptr : z, r32 != nullptr);  // z.r, z.q
      finish(c, nb, 2, 5);
      direction(0);
    }
  }
  if (info) { info->iters = it; info->rel_resid = rel; }
  return rel <= o.rtol ? VP_OK : VP_KRYLOV_MAXIT;
}

int krylov(vp_ctx c, const double* b, double* x, const vp_krylov_opts& o, vp_krylov_info* info) {
  require(c->have_K, VP_ESTATE, "no assembled operator");
  require(c->amg_ready, VP_ESTATE, "AMG not set up");
  require(o.maxit >= 1 && o.rtol > 0.0, VP_EINVAL, "bad Krylov options");
  if (o.method == VP_KRYLOV_FCG) {
    ensure_krylov(c, 2);
    return fcg(c, b, x, o, info, c->kv);
  }
  require(o.restart >= 1 && o.restart <= kMaxRestart, VP_EINVAL, "restart out of range");
  return fgmres(c, b, x, o, info);
}

void amg_setup(vp_ctx c, const vp_amg_opts& a) {
  require(c->have_K, VP_ESTATE, "no assembled operator");
  require(a.kind == VP_AMG_SA || a.kind == VP_AMG_RS, VP_EINVAL, "bad AMG kind");
  if (a.kind == VP_AMG_RS) {
    require(a.precision == VP_PREC_FP64, VP_EINVAL, "classical AMG runs in FP64");
    require(a.sweeps >= 1 && a.sweeps <= 16, VP_EINVAL, "sweeps out of range");
    require(a.strong_threshold > 0.0 && a.strong_threshold < 1.0, VP_EINVAL, "strong threshold out of (0, 1)");
    require(a.max_row_sum > 0.0 && a.max_row_sum <= 1.0, VP_EINVAL, "max_row_sum out of (0, 1]");
    require(a.max_coarse >= 8 && a.max_coarse <= 1024, VP_EINVAL, "max_coarse out of range");
    c->amg_ready = false;
    rs_setup(c, a.strong_threshold, a.max_row_sum, a.sweeps, a.max_coarse);
    c->amg_kind = VP_AMG_RS;
    c->amg_prec = VP_PREC_FP64;
    c->amg_ready = true;
    return;
  }
  c->amg_kind = VP_AMG_SA;
  require(a.cheb_degree >= 1 && a.cheb_degree <= 16, VP_EINVAL, "cheb_degree out of range");
  require(a.max_coarse >= 8 && a.max_coarse <= 1024, VP_EINVAL, "max_coarse out of range");
  require(a.precision >= 0 && a.precision <= VP_PREC_FP16_FP32COARSE, VP_EINVAL, "bad precision");
  require(c->order == 1 || a.precision <= VP_PREC_FP32_BF16COARSE, VP_EINVAL,
          "Q2 elements take the FP64, FP32 or FP32 + BF16-coarse V-cycle");
  require(a.cheb_ratio > 1.0 && a.omega_scale > 0.0, VP_EINVAL, "bad smoother options");
  require(a.variant >= 0 && a.variant <= 15, VP_EINVAL, "unknown AMG variant flags");
  require(a.walk4_rows >= 0 && a.walk4_rows <= 4096, VP_EINVAL, "walk4_rows out of range");
  c->amg_variant = a.variant;
  c->walk4_rows = a.walk4_rows;
  if (!c->amg_struct || c->max_coarse != a.max_coarse) amg_build_structure(c, c->lev[0].A64, a.max_coarse);
  c->cheb_degree = a.cheb_degree;
  c->cheb_ratio = a.cheb_ratio;
  amg_setup_numeric(c, a.precision, a.omega_scale);
}

double ew_eta(vp_ctx c, double rn, double tol_abs, double eta_max) {
  double eta;
  if (c->ew_rn_prev < 0.0) {
    eta = eta_max;
  } else {
    eta = 0.9 * (rn / c->ew_rn_prev) * (rn / c->ew_rn_prev);
    const double sg = 0.9 * c->ew_eta_prev * c->ew_eta_prev;
    if (sg > 0.1) eta = std::max(eta, sg);
  }
  // no oversolving near the end: a linear residual of half the distance to the
  // Newton tolerance is enough (Kelley's safeguard of the Eisenstat-Walker choice)
  eta = std::max(eta, 0.5 * tol_abs / rn);
  return std::min(eta, eta_max);
}

bool ls_accept(int mode, const ResidOut& t, const ResidOut& o) {
  if (mode == VP_LS_RESIDUAL) return t.rnorm < o.rnorm;
  const double floor = 1e-14 * std::max(o.eabs, t.eabs);
  const double d = t.energy - o.energy;
  if (d < -floor) return true;
  if (d > floor) return false;
  return t.rnorm < o.rnorm;
}

// One Newton iteration; when rcache is true the residual of v is already in work[0].
int newton_step(vp_ctx c, double* v, double* pi, const vp_newton_opts& no, const vp_amg_opts& ao,
                const vp_krylov_opts& ko, vp_newton_info* info, bool rcache, ResidOut* cur) {
  require(c->have_state, VP_ESTATE, "vp_set_state not called");
  require(v != nullptr && (no.variant == VP_STDN || pi != nullptr), VP_EINVAL, "null v or pi");
  require(no.variant == VP_SVN || no.variant == VP_STDN, VP_EINVAL, "bad variant");
  require(no.max_backtracks >= 0 && no.eta_max > 0.0 && no.tol > 0.0, VP_EINVAL, "bad Newton options");
  const size_t n = c->ndof;
  hipStream_t s = c->stream;
  double* R = c->work;
  double* rhs = c->work + n;
  double* dv = c->work + 2 * n;
  double* Rt = c->work + 3 * n;
  const double r0 = rnorm_zero(c);
  ResidOut o = rcache && cur ? *cur : residual_eval(c, v, nullptr, 0.0, R);
  const int pr = prof_begin(c, VP_KID_ASSEMBLE);
  launch_assemble(c, v, pi, no.variant, c->lev[0].A64);
  prof_end(c, pr);
  c->have_K = true;
  amg_setup(c, ao);
  const double eta = ew_eta(c, o.rnorm, no.tol * r0, no.eta_max);
  launch_axpby(s, -1.0, R, 0.0, rhs, n);
  launch_fill(s, dv, 0.0, n);
  vp_krylov_opts kk = ko;
  kk.rtol = eta;
  vp_krylov_info ki{};
  const int kst = krylov(c, rhs, dv, kk, &ki);
  if (kst < 0) return kst;
  double alpha = 1.0;
  int bt = 0;
  bool ok = false;
  ResidOut t{};
  for (; bt <= no.max_backtracks; ++bt) {
    t = residual_eval(c, v, dv, alpha, Rt);
    if (ls_accept(no.ls_mode, t, o)) {
      ok = true;
      break;
    }
    alpha *= 0.5;
  }
  if (info) {
    info->rnorm = o.rnorm;
    info->rnorm0 = r0;
    info->energy = o.energy;
    info->eta = eta;
    info->krylov_iters = ki.iters;
    info->backtracks = std::min(bt, no.max_backtracks);
    info->alpha = ok ? alpha : 0.0;
    info->rnorm_new = ok ? t.rnorm : o.rnorm;
    info->energy_new = ok ? t.energy : o.energy;
  }
  if (!ok) return VP_LINESEARCH_FAIL;
  if (no.variant == VP_SVN) launch_pi_update(c, v, dv, pi, alpha);
  launch_axpby(s, alpha, dv, 1.0, v, n);
  if (no.variant == VP_STDN && pi) launch_pi_init(c, v, pi);
  VP_HIP(hipMemcpyAsync(R, Rt, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  c->ew_rn_prev = o.rnorm;
  c->ew_eta_prev = eta;
  if (cur) *cur = t;
  return VP_OK;
}

void check_desc(const vp_problem_desc* d) {
  require(d != nullptr, VP_EINVAL, "null problem description");
  require(d->nx >= 2 && d->ny >= 2, VP_EINVAL, "nx and ny must be >= 2");
  require(d->order >= 0 && d->order <= 2, VP_EINVAL, "order must be 1 (Q1) or 2 (Q2)");
  const int64_t o = d->order == 2 ? 2 : 1;
  require((o * d->nx + 1) * (o * d->ny + 1) < (int64_t)1 << 31, VP_EINVAL, "mesh too large");
  require(d->Lx > 0 && d->Ly > 0 && d->dt > 0 && d->delta_min > 0 && d->e_ratio > 0, VP_EINVAL,
          "Lx, Ly, dt, delta_min and e_ratio must be positive");
  require(d->P_star >= 0 && d->rho_ice > 0 && d->rho_air >= 0 && d->rho_ocean >= 0 && d->C_air >= 0 &&
              d->C_ocean >= 0,
          VP_EINVAL, "negative physical constant");
}

}  // namespace

extern "C" {

void vp_default_opts(vp_newton_opts* n, vp_amg_opts* a, vp_krylov_opts* k) {
  if (n) *n = vp_newton_opts{VP_SVN, 1e-8, 0.1, 30, VP_LS_ENERGY};
  if (a) *a = vp_amg_opts{4, 140, VP_PREC_FP64, 30.0, 1.0, VP_AMG_SA, 3, 0.5, 0.9, 0, 0};
  if (k) *k = vp_krylov_opts{VP_KRYLOV_FCG, 30, 500, 1e-2};
}

const char* vp_last_error(vp_ctx c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int vp_create(const vp_problem_desc* desc, void* stream, vp_ctx* out) {
  return guarded(nullptr, [&] {
    require(out != nullptr, VP_EINVAL, "null output handle");
    *out = nullptr;
    check_desc(desc);
    vp_ctx c = new vp_ctx_s();
    try {
      c->desc = *desc;
      c->stream = (hipStream_t)stream;
      VP_HIP(hipGetDevice(&c->device));
      c->static_ws = scratch_address(c->device);
      c->order = desc->order == 2 ? 2 : 1;
      ElemConst& e = c->ec;
      e.nx = desc->nx; e.ny = desc->ny;
      e.nxn = c->order * desc->nx + 1; e.nyn = c->order * desc->ny + 1;
      e.hx = desc->Lx / desc->nx; e.hy = desc->Ly / desc->ny; e.wq = 0.25 * e.hx * e.hy;
      e.ihx = 1.0 / e.hx; e.ihy = 1.0 / e.hy;
      e.dt = desc->dt; e.dmin2 = desc->delta_min * desc->delta_min;
      e.c1 = 0.5 * (1.0 + 1.0 / desc->e_ratio); e.c2 = 0.5 * (1.0 - 1.0 / desc->e_ratio);
      e.s2e = 1.0 / (std::sqrt(2.0) * desc->e_ratio);
      e.rho_ice = desc->rho_ice; e.cdo = desc->C_ocean * desc->rho_ocean; e.cda = desc->C_air * desc->rho_air;
      e.fc = desc->f_coriolis; e.P_star = desc->P_star; e.C_strength = desc->C_strength;
      c->nn = (size_t)e.nxn * e.nyn;
      c->ncell = (size_t)e.nx * e.ny;
      c->ndof = 2 * c->nn;
      c->P = dalloc<double>(c->ncell);
      c->rhoH = dalloc<double>(c->ncell);
      c->F = dalloc<double>(c->ndof);
      c->vo = dalloc<double>(c->ndof);
      c->Hs = dalloc<double>(c->ncell);
      c->As = dalloc<double>(c->ncell);
      c->vas = dalloc<double>(c->ndof);
      c->vps = dalloc<double>(c->ndof);
      c->partials = dalloc<double>(partial_slots(c));
      c->dscal = dalloc<double>(256);
      VP_HIP(hipHostMalloc((void**)&c->hscal, 512 * sizeof(double), hipHostMallocDefault));
      c->work = dalloc<double>(5 * c->ndof);
      c->lev[0].A64 = dalloc<double>(20 * c->nn);
      c->lev[0].nxn = e.nxn; c->lev[0].nyn = e.nyn; c->lev[0].B = 2; c->lev[0].nn = c->nn;
      if (c->order == 2) {
        c->K2 = dalloc<double>((size_t)52 * c->nn);
        // the Q1 stencil storage only carries the AMG structure for Q2 elements
        VP_HIP(hipMemsetAsync(c->lev[0].A64, 0, 20 * c->nn * sizeof(double), c->stream));
      }
    } catch (...) {
      vp_destroy(c);
      throw;
    }
    *out = c;
    return VP_OK;
  });
}

void vp_destroy(vp_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  double* K = c->lev[0].A64;
  rs_free(c);
  amg_free(c);
  if (K) (void)hipFree(K);
  void* bufs[] = {c->P, c->rhoH, c->F, c->vo, c->Hs, c->As, c->vas, c->vps, c->partials, c->dscal, c->work, c->kv, c->dense,
                  c->K2, c->K2_32, c->lmax_q2, c->pq0, c->pq1, c->pqn};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (c->hscal) (void)hipHostFree(c->hscal);
  for (hipEvent_t e : c->prof.ev) (void)hipEventDestroy(e);
  delete c;
}

int vp_set_state(vp_ctx c, const double* H, const double* A, const double* va, const double* vo,
                 const double* vp_) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    require(H && A && va && vo && vp_, VP_EINVAL, "null state array");
    const int nb = launch_state_check(c, H, A, va, vo, vp_);
    finish_fetch(c, nb, 1, 0, 1);
    require(c->hscal[0] == 0.0, VP_EINVAL,
            "invalid step data: H must be finite and >= 0, A finite in [0, 1], velocities finite");
    launch_precompute(c, H, A, va, vo, vp_);
    c->have_state = true;
    c->rnorm_zero = -1.0;
    c->ew_rn_prev = -1.0;
    c->ew_eta_prev = 0.1;
    return VP_OK;
  });
}

int vp_residual(vp_ctx c, const double* v, double* r, double* rnorm, double* energy) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    require(c->have_state, VP_ESTATE, "vp_set_state not called");
    require(v != nullptr, VP_EINVAL, "null v");
    if (!rnorm && !energy) {
      unsigned g;
      launch_residual(c, v, nullptr, 0.0, r, c->partials, &g);
      return VP_OK;
    }
    const ResidOut o = residual_eval(c, v, nullptr, 0.0, r);
    if (rnorm) *rnorm = o.rnorm;
    if (energy) *energy = o.energy;
    return VP_OK;
  });
}

int vp_newton_assemble(vp_ctx c, const double* v, const double* pi, int variant) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    require(c->have_state, VP_ESTATE, "vp_set_state not called");
    require(variant == VP_SVN || variant == VP_STDN, VP_EINVAL, "bad variant");
    require(v != nullptr && (variant == VP_STDN || pi != nullptr), VP_EINVAL, "null v or pi");
    launch_assemble(c, v, pi, variant, c->lev[0].A64);
    c->have_K = true;
    c->amg_ready = false;
    return VP_OK;
  });
}

int vp_operator_apply(vp_ctx c, const double* x, double* y) {
  return guarded(c, [&] {
    require(c != nullptr && x && y, VP_EINVAL, "null argument");
    require(c->have_K, VP_ESTATE, "no assembled operator");
    launch_apply_K(c, x, y, nullptr);
    return VP_OK;
  });
}

int vp_operator_export(vp_ctx c, double* blocks) {
  return guarded(c, [&] {
    require(c != nullptr && blocks, VP_EINVAL, "null argument");
    require(c->have_K, VP_ESTATE, "no assembled operator");
    if (c->order == 2)
      VP_HIP(hipMemcpyAsync(blocks, c->K2, 52 * c->nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    else
      VP_HIP(hipMemcpyAsync(blocks, c->lev[0].A64, 20 * c->nn * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
    return VP_OK;
  });
}

int vp_amg_setup(vp_ctx c, const vp_amg_opts* a) {
  return guarded(c, [&] {
    require(c != nullptr && a, VP_EINVAL, "null argument");
    amg_setup(c, *a);
    return VP_OK;
  });
}

int vp_amg_apply(vp_ctx c, const double* r, double* z) {
  return guarded(c, [&] {
    require(c != nullptr && r && z, VP_EINVAL, "null argument");
    require(r != z, VP_EINVAL, "r and z must not alias");
    amg_apply(c, r, z);
    return VP_OK;
  });
}

int vp_amg_info(vp_ctx c, int* levels, int* nxn, int* nyn, int* dpn) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    if (c->amg_ready && c->amg_kind == VP_AMG_RS) {
      const int nl = rs_levels(c);
      if (levels) *levels = nl;
      for (int l = 0; l < nl; ++l) {
        long long info[5];
        rs_info(c, l, info);
        if (nxn) nxn[l] = (int)info[0];
        if (nyn) nyn[l] = 1;
        if (dpn) dpn[l] = 1;
      }
      return VP_OK;
    }
    require(c->amg_struct, VP_ESTATE, "AMG not set up");
    if (levels) *levels = c->nlev;
    for (int l = 0; l < c->nlev; ++l) {
      if (nxn) nxn[l] = c->lev[l].nxn;
      if (nyn) nyn[l] = c->lev[l].nyn;
      if (dpn) dpn[l] = c->lev[l].B;
    }
    return VP_OK;
  });
}

int vp_amg_export(vp_ctx c, int level, double* A, double* P) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    require(c->amg_ready, VP_ESTATE, "AMG not set up");
    require(c->amg_kind == VP_AMG_SA, VP_ESTATE, "classical AMG: use vp_amg_rs_export");
    require(level >= 0 && level < c->nlev, VP_EINVAL, "level out of range");
    require(!P || level + 1 < c->nlev, VP_EINVAL, "the coarsest level has no prolongator");
    const Level& L = c->lev[level];
    if (A)
      VP_HIP(hipMemcpyAsync(A, L.A64, (size_t)5 * L.B * L.B * L.nn * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
    if (P) amg_export_p(c, level, P);
    return VP_OK;
  });
}

int vp_amg_rs_info(vp_ctx c, int level, int64_t* out) {
  return guarded(c, [&] {
    require(c != nullptr && out, VP_EINVAL, "null argument");
    require(c->amg_ready && c->amg_kind == VP_AMG_RS, VP_ESTATE, "classical AMG not set up");
    require(level >= 0 && level < rs_levels(c), VP_EINVAL, "level out of range");
    long long info[5];
    rs_info(c, level, info);
    for (int k = 0; k < 5; ++k) out[k] = info[k];
    return VP_OK;
  });
}

int vp_amg_rs_export(vp_ctx c, int level, int32_t* A_ptr, int32_t* A_col, double* A_val, int32_t* cf,
                     int32_t* P_ptr, int32_t* P_col, double* P_val, int32_t* colour) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    require(c->amg_ready && c->amg_kind == VP_AMG_RS, VP_ESTATE, "classical AMG not set up");
    require(level >= 0 && level < rs_levels(c), VP_EINVAL, "level out of range");
    require(level + 1 < rs_levels(c) || !(cf || P_ptr || P_col || P_val || colour), VP_EINVAL,
            "the coarsest level has no splitting, prolongator or colouring");
    rs_export(c, level, A_ptr, A_col, A_val, cf, P_ptr, P_col, P_val, colour);
    return VP_OK;
  });
}

int vp_krylov_solve(vp_ctx c, const double* b, double* x, const vp_krylov_opts* o, vp_krylov_info* info) {
  return guarded(c, [&] {
    require(c != nullptr && b && x && o, VP_EINVAL, "null argument");
    return krylov(c, b, x, *o, info);
  });
}

int vp_krylov_solve_noalloc(vp_ctx c, const double* b, double* x, const vp_krylov_opts* o,
                            vp_krylov_info* info) {
  return guarded(c, [&] {
    require(c != nullptr && b && x && o, VP_EINVAL, "null argument");
    require(o->method == VP_KRYLOV_FCG, VP_EINVAL, "the allocation-free Krylov solve runs flexible CG only");
    require(c->ndof <= kNoAllocDofs, VP_EINVAL,
            "mesh too large for the static Krylov workspace (at most 2359296 dofs)");
    require(c->have_K, VP_ESTATE, "no assembled operator");
    require(c->amg_ready, VP_ESTATE, "AMG not set up");
    require(o->maxit >= 1 && o->rtol > 0.0, VP_EINVAL, "bad Krylov options");
    require(c->static_ws != nullptr, VP_ESTATE, "no workspace address for this device");
    // profiling creates events on demand: leave it off for this call
    struct ProfOff {
      Prof& p;
      bool on;
      explicit ProfOff(Prof& q) : p(q), on(q.on) { p.on = false; }
      ~ProfOff() { p.on = on; }
    } off(c->prof);
    return fcg(c, b, x, *o, info, c->static_ws);
  });
}

int vp_pi_update(vp_ctx c, const double* v, const double* dv, double* pi, double alpha) {
  return guarded(c, [&] {
    require(c != nullptr && v && dv && pi, VP_EINVAL, "null argument");
    launch_pi_update(c, v, dv, pi, alpha);
    return VP_OK;
  });
}

int vp_pi_init(vp_ctx c, const double* v, double* pi) {
  return guarded(c, [&] {
    require(c != nullptr && v && pi, VP_EINVAL, "null argument");
    launch_pi_init(c, v, pi);
    return VP_OK;
  });
}

int vp_advect(vp_ctx c, const double* v, const double* A, const double* H, double* A_out, double* H_out) {
  return guarded(c, [&] {
    require(c != nullptr && v && A && H && A_out && H_out, VP_EINVAL, "null argument");
    require(A_out != A && A_out != H && H_out != A && H_out != H && A_out != H_out, VP_EINVAL,
            "outputs must not alias the inputs or each other");
    launch_advect(c, v, A, H, A_out, H_out);
    return VP_OK;
  });
}

int vp_profile(vp_ctx c, int enable) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    if (enable) c->prof.used = 0;
    c->prof.on = enable != 0;
    return VP_OK;
  });
}

int vp_profile_read(vp_ctx c, int kid, double* total_ms, int* launches, double* bytes) {
  return guarded(c, [&] {
    require(c != nullptr, VP_EINVAL, "null context");
    require(kid >= 0 && kid < VP_KID_COUNT, VP_EINVAL, "unknown kernel id");
    VP_HIP(hipStreamSynchronize(c->stream));
    double ms = 0.0;
    int cnt = 0;
    for (size_t k = 0; k < c->prof.used; ++k) {
      if (c->prof.kid[k] != kid) continue;
      float t = 0.0f;
      VP_HIP(hipEventElapsedTime(&t, c->prof.ev[2 * k], c->prof.ev[2 * k + 1]));
      ms += t;
      ++cnt;
    }
    const double nn = (double)c->nn, nc = (double)c->ncell;
    const bool f32 = c->amg_prec != VP_PREC_FP64;
    double b = 0.0;
    switch (kid) {
      case VP_KID_APPLY_FINE: b = nn * (20 * 8 + 2 * 16); break;
      case VP_KID_CHEB_STEP0:
        b = c->amg_prec >= VP_PREC_BF16 ? nn * (20 * 2 + 6 * 8) : f32 ? nn * (20 * 4 + 6 * 8) : nn * (20 * 8 + 6 * 16);
        break;
      case VP_KID_STEN_RESID0:
        b = c->amg_prec >= VP_PREC_BF16 ? nn * (20 * 2 + 3 * 8) : f32 ? nn * (20 * 4 + 3 * 8) : nn * (20 * 8 + 3 * 16);
        break;
      case VP_KID_CHEB_PAIR0:   // A once + three vectors read and three written, for two steps
        b = c->amg_prec >= VP_PREC_BF16 ? nn * (20 * 2 + 6 * 8) : f32 ? nn * (20 * 4 + 6 * 8) : nn * (20 * 8 + 6 * 16);
        break;
      case VP_KID_CHEB_WALK4:   // A once, b, and x in + x out (post) or x and r out (pre)
        b = f32 ? nn * (20 * 4 + 3 * 8) : nn * (20 * 8 + 3 * 16);
        break;
      case VP_KID_RESIDUAL: b = nn * 64 + nc * 16; break;
      case VP_KID_ASSEMBLE: b = nn * (32 + 160) + nc * (16 + 96); break;
      default: b = 0.0;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = cnt;
    if (bytes) *bytes = b;
    return VP_OK;
  });
}

int vp_newton_step(vp_ctx c, double* v, double* pi, const vp_newton_opts* no, const vp_amg_opts* ao,
                   const vp_krylov_opts* ko, vp_newton_info* info) {
  return guarded(c, [&] {
    require(c != nullptr && no && ao && ko, VP_EINVAL, "null argument");
    return newton_step(c, v, pi, *no, *ao, *ko, info, false, nullptr);
  });
}

int vp_newton_solve(vp_ctx c, double* v, double* pi, int maxit, const vp_newton_opts* no,
                    const vp_amg_opts* ao, const vp_krylov_opts* ko, vp_solve_info* info,
                    double* history) {
  return guarded(c, [&] {
    require(c != nullptr && no && ao && ko && v, VP_EINVAL, "null argument");
    require(maxit >= 0, VP_EINVAL, "maxit < 0");
    require(c->have_state, VP_ESTATE, "vp_set_state not called");
    c->ew_rn_prev = -1.0;
    c->ew_eta_prev = no->eta_max;
    amg_reset_estimates(c);  // a solve is a function of its inputs only
    const double r0 = rnorm_zero(c);
    ResidOut cur = residual_eval(c, v, nullptr, 0.0, c->work);
    int it = 0, kits = 0, st = VP_NOT_CONVERGED;
    if (history) history[0] = r0 > 0 ? cur.rnorm / r0 : 0.0;
    while (true) {
      if (cur.rnorm <= no->tol * r0) { st = VP_OK; break; }
      if (it >= maxit) { st = VP_NOT_CONVERGED; break; }
      vp_newton_info ni{};
      const int rc = newton_step(c, v, pi, *no, *ao, *ko, &ni, true, &cur);
      if (rc < 0) return rc;
      kits += ni.krylov_iters;
      if (rc == VP_LINESEARCH_FAIL) { st = rc; break; }
      ++it;
      if (history) history[it] = r0 > 0 ? cur.rnorm / r0 : 0.0;
    }
    if (info) {
      info->iterations = it;
      info->krylov_iters = kits;
      info->rnorm0 = r0;
      info->rel_resid = r0 > 0 ? cur.rnorm / r0 : 0.0;
    }
    return st;
  });
}

}  // extern "C"
