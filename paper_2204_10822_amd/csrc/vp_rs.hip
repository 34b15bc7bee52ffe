// Classical (Ruge-Stueben) AMG on the GPU with the settings the paper reports
// for its preconditioner (Sec. 5.4): strong threshold 0.5, three symmetric
// Gauss-Seidel sweeps per smoothing on every level, Gaussian elimination on the
// coarsest level, V-cycle, FP64 throughout.  An alternative to the structured
// smoothed aggregation of vp_amg.hip, on the same operators.
//
// Every step runs in the kernels below; the host only sizes buffers from scan
// totals and loops over coarsening / colouring rounds.
//  * the finest level is the assembled block stencil (Q1 9-point or Q2
//    25-point) converted to scalar CSR with the dof numbering of the vectors
//    (2 node + component), rows sorted by column, exact zeros dropped;
//  * strength: j strongly influences i when -s a_ij >= theta max_k(-s a_ik),
//    s = sign(a_ii); rows with |row sum| > max_row_sum |a_ii| have none;
//  * coarsening: the Ruge-Stueben first pass done in parallel rounds: every
//    undecided point whose key (measure, hash, index) beats its undecided strong
//    neighbours (either direction) becomes C, its undecided strong dependents
//    become F, and the measures are updated as in the sequential pass (-1 for the
//    points a new C depends on, +1 for the points a new F depends on); points
//    nothing undecided depends on become F;
//  * classical interpolation (strong F neighbours distributed over the common
//    strong C neighbours by couplings of sign opposite to their diagonal, weak
//    couplings lumped into the diagonal);
//  * R = P^T built row by row from the symmetric sparsity of A, Galerkin
//    A_c = R (A P) by a row-wise k-way merge of sorted rows (deterministic);
//  * multicolour symmetric Gauss-Seidel: a parallel greedy colouring (rounds of
//    hash-key local maxima, each taking the smallest colour its neighbours do
//    not hold), one launch per colour on the large levels and one workgroup for
//    all levels below kRsSmall rows (their whole V-cycle in one kernel).
#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "vp_internal.h"

namespace vp {

void launch_dense_inverse(hipStream_t s, double* M, int nd);

namespace {

constexpr int kRsBlock = 256;
constexpr int kMergeBlock = 64;
constexpr int kMaxMergeList = 480;  // longest left-factor row of a sparse product (LDS < 64 KB)
constexpr int kRsSmall = 2048;      // levels handled by the one-workgroup tail kernel
constexpr int kMaxColours = 128;
constexpr int kMaxRsLevels = 25;
constexpr int kMaxRounds = 4096;
constexpr int kDenseMax = 1024;     // coarsest levels above this are only smoothed
constexpr int8_t kU = -1, kF = 0, kC = 1, kNewF = 2;

template <typename T>
void ensure(T*& p, size_t& cap, size_t n) {
  if (n <= cap && p) return;
  if (p) VP_HIP(hipFree(p));
  p = nullptr;
  cap = 0;
  const size_t m = std::max<size_t>(n, 1);
  VP_HIP(hipMalloc((void**)&p, m * sizeof(T)));
  cap = m;
}

inline unsigned rs_grid(size_t n, int block = kRsBlock) { return (unsigned)((n + block - 1) / block); }

}  // namespace

struct RSLevel {
  int n = 0, nc = 0, ncol = 0;
  size_t nnz = 0, nnzP = 0, nnzR = 0;
  int* ptr = nullptr; size_t c_ptr = 0;
  int* col = nullptr; size_t c_col = 0;
  double* val = nullptr; size_t c_val = 0;
  double* diag = nullptr; size_t c_diag = 0;
  int8_t* cf = nullptr; size_t c_cf = 0;
  int* cidx = nullptr; size_t c_cidx = 0;
  int* pptr = nullptr; size_t c_pptr = 0;
  int* pcol = nullptr; size_t c_pcol = 0;
  double* pval = nullptr; size_t c_pval = 0;
  int* rptr = nullptr; size_t c_rptr = 0;
  int* rcol = nullptr; size_t c_rcol = 0;
  double* rval = nullptr; size_t c_rval = 0;
  int* colour = nullptr; size_t c_colour = 0;
  int* corder = nullptr; size_t c_corder = 0;
  int* coff = nullptr; size_t c_coff = 0;  // device copy of the colour offsets
  std::vector<int> coff_h;
  // the rows of each colour again in ELL form (slot-major, padded with zero
  // couplings to the row itself) for coalesced smoother reads
  int* ecol = nullptr; size_t c_ecol = 0;
  double* eval = nullptr; size_t c_eval = 0;
  int* eoff = nullptr; size_t c_eoff = 0;  // device [base, width] per colour
  std::vector<long long> ebase_h;
  std::vector<int> ewidth_h;
  double* x = nullptr; size_t c_x = 0;
  double* b = nullptr; size_t c_b = 0;
  double* r = nullptr; size_t c_r = 0;
  double* Ainv = nullptr; size_t c_ainv = 0;
  bool smooth_only = false;  // coarsest level that could not be coarsened and is too large to factor
};

struct RSHier {
  RSLevel lev[kMaxRsLevels];
  int nlev = 0, tail = -1, sweeps = 3;
  // setup scratch
  int* cnt = nullptr; size_t c_cnt = 0;
  int* lam = nullptr; size_t c_lam = 0;
  int8_t* sel = nullptr; size_t c_sel = 0;
  uint8_t* strong = nullptr; size_t c_strong = 0;
  int* tpos = nullptr; size_t c_tpos = 0;
  int* cfine = nullptr; size_t c_cfine = 0;
  int* apptr = nullptr; size_t c_apptr = 0;
  int* apcol = nullptr; size_t c_apcol = 0;
  double* apval = nullptr; size_t c_apval = 0;
  long long* bsum = nullptr; size_t c_bsum = 0;
  int* dint = nullptr;          // device counters [64]
  long long* hint = nullptr;    // pinned host mirror [64]
  void* targs = nullptr;        // device copy of the tail arguments
};

namespace {

// ---------------------------------------------------------------------------
// exclusive scan of int counts into ptr[0..n] (ptr[n] = total), total returned
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 256, kScanPer = 4, kScanChunk = kScanBlock * kScanPer;

__global__ void __launch_bounds__(kScanBlock) k_scan_local(const int* __restrict__ cnt, size_t n,
                                                           int* __restrict__ out, long long* __restrict__ bsum) {
  __shared__ long long s[kScanBlock];
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanPer;
  long long v[kScanPer], t = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? cnt[base + k] : 0;
    t += v[k];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const long long a = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += a;
    __syncthreads();
  }
  long long run = s[threadIdx.x] - t;
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = (int)run;  // block-local offset (< 2^31)
    run += v[k];
  }
  if (threadIdx.x == kScanBlock - 1) bsum[blockIdx.x] = s[threadIdx.x];
}

__global__ void __launch_bounds__(1024) k_scan_top(long long* __restrict__ bsum, int nb, long long* __restrict__ total) {
  __shared__ long long s[1024];
  long long carry = 0;
  for (int c0 = 0; c0 < nb; c0 += 1024) {
    const int i = c0 + (int)threadIdx.x;
    const long long v = i < nb ? bsum[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const long long a = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;
    const long long blk = s[1023];
    __syncthreads();
    carry += blk;
  }
  if (threadIdx.x == 0) total[0] = carry;
}

__global__ void k_scan_add(int* __restrict__ out, size_t n, const long long* __restrict__ boff,
                           const long long* __restrict__ total) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int)(out[i] + boff[i / kScanChunk]);
  if (i == 0) out[n] = (int)total[0];
}

// ---------------------------------------------------------------------------
// finest level: block stencil -> scalar CSR
// ---------------------------------------------------------------------------
// storage plane of the forward offset (dx, dy) (dy > 0, or dy = 0 and dx >= 0)
template <int RAD>
__device__ __forceinline__ int stencil_plane(int dx, int dy) {
  if constexpr (RAD == 1) return dy == 0 ? dx : (dx == 0 ? 2 : dx == 1 ? 3 : 4);
  else return dy == 0 ? dx : 3 + (dy - 1) * 5 + (dx + 2);
}

template <int RAD>
__device__ __forceinline__ double stencil_entry(const double* __restrict__ A, size_t nn, int nxn, size_t n, int dx,
                                                int dy, int r, int c) {
  if (dy > 0 || (dy == 0 && dx >= 0)) return A[aidx(2, nn, stencil_plane<RAD>(dx, dy), n, r, c)];
  const size_t m = (size_t)((long long)n + (long long)dy * nxn + dx);
  return A[aidx(2, nn, stencil_plane<RAD>(-dx, -dy), m, c, r)];
}

template <int RAD, bool FILL>
__global__ void __launch_bounds__(kRsBlock)
k_rs_from_stencil(const double* __restrict__ A, size_t nn, int nxn, int nyn, const int* __restrict__ ptr,
                  int* __restrict__ cnt, int* __restrict__ col, double* __restrict__ val) {
  const size_t row = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= 2 * nn) return;
  const size_t n = row >> 1;
  const int r = (int)(row & 1);
  const int i = (int)(n % nxn), j = (int)(n / nxn);
  int k = FILL ? ptr[row] : 0;
  for (int dy = -RAD; dy <= RAD; ++dy)
    for (int dx = -RAD; dx <= RAD; ++dx) {
      const int ii = i + dx, jj = j + dy;
      if (ii < 0 || ii >= nxn || jj < 0 || jj >= nyn) continue;
      const size_t m = (size_t)jj * nxn + ii;
      for (int c = 0; c < 2; ++c) {
        const double a = stencil_entry<RAD>(A, nn, nxn, n, dx, dy, r, c);
        if (a != 0.0 || (m == n && c == r)) {
          if (FILL) {
            col[k] = (int)(2 * m + c);
            val[k] = a;
          }
          ++k;
        }
      }
    }
  if (!FILL) cnt[row] = k;
}

// ---------------------------------------------------------------------------
// strength, transposed positions, longest row
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kRsBlock)
k_rs_strength(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
              double theta, double max_row_sum, uint8_t* __restrict__ strong, int* __restrict__ lam,
              double* __restrict__ diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int lo = ptr[i], hi = ptr[i + 1];
  double d = 0.0, rs = 0.0;
  for (int k = lo; k < hi; ++k) {
    rs += val[k];
    if (col[k] == i) d += val[k];
  }
  const double sg = d >= 0.0 ? -1.0 : 1.0;
  double mx = 0.0;
  for (int k = lo; k < hi; ++k)
    if (col[k] != i) mx = fmax(mx, sg * val[k]);
  diag[i] = d;
  const bool none = (max_row_sum < 1.0 && fabs(rs) > max_row_sum * fabs(d)) || !(mx > 0.0);
  for (int k = lo; k < hi; ++k) {
    const bool s = !none && col[k] != i && sg * val[k] >= theta * mx;
    strong[k] = s ? 1 : 0;
    if (s) atomicAdd(&lam[col[k]], 1);
  }
}

__global__ void __launch_bounds__(kRsBlock)
k_rs_diag(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
          double* __restrict__ diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k)
    if (col[k] == i) d += val[k];
  diag[i] = d;
}

__global__ void __launch_bounds__(kRsBlock)
k_rs_tpos(int n, const int* __restrict__ ptr, const int* __restrict__ col, int* __restrict__ tpos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    int lo = ptr[j], hi = ptr[j + 1] - 1, hit = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int c = col[mid];
      if (c == i) { hit = mid; break; }
      if (c < i) lo = mid + 1;
      else hi = mid - 1;
    }
    tpos[k] = hit;
  }
}

// ---------------------------------------------------------------------------
// parallel Ruge-Stueben first pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned rs_hash(unsigned i, unsigned seed) {
  unsigned z = i * 0x9E3779B9u + seed;
  z = (z ^ (z >> 16)) * 0x85EBCA6Bu;
  z = (z ^ (z >> 13)) * 0xC2B2AE35u;
  return z ^ (z >> 16);
}

__device__ __forceinline__ bool key_gt(int la, unsigned ha, int ia, int lb, unsigned hb, int ib) {
  return la != lb ? la > lb : (ha != hb ? ha > hb : ia > ib);
}

__device__ __forceinline__ bool dep_on_me(const uint8_t* strong, const int* tpos, int k) {
  const int t = tpos[k];
  return t >= 0 && strong[t];
}

__global__ void k_rs_cf_init(int n, const int* __restrict__ lam, int8_t* __restrict__ cf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cf[i] = lam[i] == 0 ? kF : kU;
}

__global__ void __launch_bounds__(kRsBlock)
k_rs_select(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
            const int* __restrict__ tpos, const int8_t* __restrict__ cf, const int* __restrict__ lam,
            int8_t* __restrict__ sel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cf[i] != kU) { sel[i] = 0; return; }
  const int li = lam[i];
  const unsigned hi_ = rs_hash((unsigned)i, 0x51ED270Bu);
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    if (j == i || cf[j] != kU) continue;
    if (!strong[k] && !dep_on_me(strong, tpos, k)) continue;
    if (key_gt(lam[j], rs_hash((unsigned)j, 0x51ED270Bu), j, li, hi_, i)) { sel[i] = 0; return; }
  }
  sel[i] = 1;
}

__global__ void __launch_bounds__(kRsBlock)
k_rs_mark(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
          const int* __restrict__ tpos, const int8_t* __restrict__ sel, int8_t* cf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !sel[i]) return;
  cf[i] = kC;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    if (j != i && dep_on_me(strong, tpos, k) && cf[j] == kU) cf[j] = kNewF;
  }
}

__global__ void __launch_bounds__(kRsBlock)
k_rs_update(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
            const int8_t* __restrict__ sel, const int8_t* __restrict__ cf, int* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = sel[i] ? -1 : (cf[i] == kNewF ? 1 : 0);
  if (d == 0) return;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    if (strong[k] && cf[j] == kU) atomicAdd(&lam[j], d);
  }
}

__global__ void k_rs_finish_round(int n, int8_t* __restrict__ cf, const int* __restrict__ lam,
                                  int* __restrict__ undecided) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int8_t s = cf[i];
  if (s == kNewF) s = kF;
  else if (s == kU && lam[i] <= 0) s = kF;
  cf[i] = s;
  if (s == kU) atomicAdd(undecided, 1);
}

__global__ void k_rs_zero_ints(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_rs_is_c(int n, const int8_t* __restrict__ cf, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = cf[i] == kC ? 1 : 0;
}

__global__ void k_rs_cfine(int n, const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                           int* __restrict__ cfine) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && cf[i] == kC) cfine[cidx[i]] = i;
}

// ---------------------------------------------------------------------------
// classical interpolation
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kRsBlock)
k_rs_pcount(int n, const int* __restrict__ ptr, const int* __restrict__ col, const uint8_t* __restrict__ strong,
            const int8_t* __restrict__ cf, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cf[i] == kC) { cnt[i] = 1; return; }
  int c = 0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k)
    if (strong[k] && cf[col[k]] == kC) ++c;
  cnt[i] = c;
}

__device__ __forceinline__ double sign_of(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

__global__ void __launch_bounds__(kRsBlock)
k_rs_pfill(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
           const uint8_t* __restrict__ strong, const int8_t* __restrict__ cf, const int* __restrict__ cidx,
           const double* __restrict__ diag, const int* __restrict__ pptr, int* __restrict__ pcol,
           double* __restrict__ pval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = pptr[i], p1 = pptr[i + 1];
  if (cf[i] == kC) {
    pcol[p0] = cidx[i];
    pval[p0] = 1.0;
    return;
  }
  if (p1 == p0) return;
  const int lo = ptr[i], hi = ptr[i + 1];
  // strong C neighbours (fine indices, ascending) with a_ik; diagonal plus weak couplings
  double dg = 0.0;
  int q = p0;
  for (int k = lo; k < hi; ++k) {
    const int j = col[k];
    if (j == i) dg += val[k];
    else if (strong[k] && cf[j] == kC) { pcol[q] = j; pval[q] = val[k]; ++q; }
    else if (!strong[k]) dg += val[k];
  }
  // strong F neighbours m: distribute a_im over the C_i couplings of row m
  for (int k = lo; k < hi; ++k) {
    const int m = col[k];
    if (m == i || !strong[k] || cf[m] == kC) continue;
    const double aim = val[k], smm = sign_of(diag[m]);
    const int mlo = ptr[m], mhi = ptr[m + 1];
    double den = 0.0;
    for (int a = mlo, t = p0; a < mhi && t < p1;) {
      const int ca = col[a], ct = pcol[t];
      if (ca < ct) ++a;
      else if (ct < ca) ++t;
      else {
        if (val[a] * smm < 0.0) den += val[a];
        ++a; ++t;
      }
    }
    if (den == 0.0) { dg += aim; continue; }
    for (int a = mlo, t = p0; a < mhi && t < p1;) {
      const int ca = col[a], ct = pcol[t];
      if (ca < ct) ++a;
      else if (ct < ca) ++t;
      else {
        if (val[a] * smm < 0.0) pval[t] += aim * val[a] / den;
        ++a; ++t;
      }
    }
  }
  for (int t = p0; t < p1; ++t) {
    pval[t] = -pval[t] / dg;
    pcol[t] = cidx[pcol[t]];
  }
}

// R = P^T, one coarse row per thread: the fine rows j holding coarse point I lie in
// row i = cfine[I] of A (symmetric sparsity), so R's rows come out sorted.
template <bool FILL>
__global__ void __launch_bounds__(kRsBlock)
k_rs_restrictor(int nc, const int* __restrict__ cfine, const int* __restrict__ ptr, const int* __restrict__ col,
                const int8_t* __restrict__ cf, const int* __restrict__ pptr, const int* __restrict__ pcol,
                const double* __restrict__ pval, const int* __restrict__ rptr, int* __restrict__ cnt,
                int* __restrict__ rcol, double* __restrict__ rval) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int i = cfine[I];
  int q = FILL ? rptr[I] : 0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    double w = 0.0;
    bool hit = false;
    if (j == i) { w = 1.0; hit = true; }
    else if (cf[j] != kC) {
      for (int t = pptr[j]; t < pptr[j + 1]; ++t)
        if (pcol[t] == I) { w = pval[t]; hit = true; break; }
    }
    if (hit) {
      if (FILL) { rcol[q] = j; rval[q] = w; }
      ++q;
    }
  }
  if (!FILL) cnt[I] = q;
}

// ---------------------------------------------------------------------------
// sparse product C = L * Rm, one output row per thread: a k-way merge of the
// sorted rows of Rm named by row t of L (cursor offsets in LDS)
// ---------------------------------------------------------------------------
template <bool FILL>
__global__ void __launch_bounds__(kMergeBlock)
k_rs_spgemm(int nrows, const int* __restrict__ Lptr, const int* __restrict__ Lcol, const double* __restrict__ Lval,
            const int* __restrict__ Rptr, const int* __restrict__ Rcol, const double* __restrict__ Rval,
            const int* __restrict__ Cptr, int* __restrict__ Ccnt, int* __restrict__ Ccol,
            double* __restrict__ Cval) {
  extern __shared__ unsigned short cur[];
  const int t = blockIdx.x * kMergeBlock + threadIdx.x;
  if (t >= nrows) return;
  const int lo = Lptr[t], K = Lptr[t + 1] - lo;
  for (int e = 0; e < K; ++e) cur[e * kMergeBlock + threadIdx.x] = 0;
  int out = FILL ? Cptr[t] : 0;
  for (;;) {
    int mn = INT_MAX;
    for (int e = 0; e < K; ++e) {
      const int j = Lcol[lo + e];
      const int p = Rptr[j] + cur[e * kMergeBlock + threadIdx.x];
      if (p < Rptr[j + 1]) mn = min(mn, Rcol[p]);
    }
    if (mn == INT_MAX) break;
    double s = 0.0;
    for (int e = 0; e < K; ++e) {
      const int j = Lcol[lo + e];
      const int p = Rptr[j] + cur[e * kMergeBlock + threadIdx.x];
      if (p < Rptr[j + 1] && Rcol[p] == mn) {
        s += Lval[lo + e] * Rval[p];
        cur[e * kMergeBlock + threadIdx.x] += 1;
      }
    }
    if (FILL) {
      Ccol[out] = mn;
      Cval[out] = s;
    }
    ++out;
  }
  if (!FILL) Ccnt[t] = out;
}

__global__ void k_rs_rowmax(int n, const int* __restrict__ ptr, int* __restrict__ mx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicMax(mx, ptr[i + 1] - ptr[i]);
}

// ---------------------------------------------------------------------------
// parallel greedy colouring
// ---------------------------------------------------------------------------
__global__ void k_col_init(int n, int* __restrict__ colour) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) colour[i] = -1;
}

__global__ void __launch_bounds__(kRsBlock)
k_col_select(int n, const int* __restrict__ ptr, const int* __restrict__ col, const int* __restrict__ colour,
             int8_t* __restrict__ sel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (colour[i] >= 0) { sel[i] = 0; return; }
  const unsigned hi_ = rs_hash((unsigned)i, 0x2545F491u);
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    if (j == i || colour[j] >= 0) continue;
    if (key_gt(0, rs_hash((unsigned)j, 0x2545F491u), j, 0, hi_, i)) { sel[i] = 0; return; }
  }
  sel[i] = 1;
}

__global__ void __launch_bounds__(kRsBlock)
k_col_assign(int n, const int* __restrict__ ptr, const int* __restrict__ col, const int8_t* __restrict__ sel,
             int* colour, int* __restrict__ ctr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!sel[i]) {
    if (colour[i] < 0) atomicAdd(&ctr[0], 1);
    return;
  }
  unsigned long long m0 = 0, m1 = 0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = col[k];
    const int c = j == i ? -1 : colour[j];
    if (c >= 0 && c < 64) m0 |= 1ull << c;
    else if (c >= 64 && c < 128) m1 |= 1ull << (c - 64);
  }
  int c;
  if (~m0) c = __builtin_ctzll(~m0);
  else if (~m1) c = 64 + __builtin_ctzll(~m1);
  else { c = kMaxColours - 1; atomicAdd(&ctr[2], 1); }  // reported as an error by the host
  colour[i] = c;
}

__global__ void k_col_count(int n, const int* __restrict__ colour, int* __restrict__ counts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&counts[colour[i]], 1);
}

__global__ void k_col_scatter(int n, const int* __restrict__ colour, int* __restrict__ cursor,
                              int* __restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) order[atomicAdd(&cursor[colour[i]], 1)] = i;
}

__global__ void k_col_width(int n, const int* __restrict__ ptr, const int* __restrict__ colour,
                            int* __restrict__ width) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicMax(&width[colour[i]], ptr[i + 1] - ptr[i]);
}

// ELL copy: position t of the colour-sorted order, row i = order[t] of colour c
// goes to column t - coff[c] of colour c's slot-major block at base(c).
__global__ void __launch_bounds__(kRsBlock)
k_ell_fill(int n, const int* __restrict__ order, const int* __restrict__ colour, const int* __restrict__ coff,
           const long long* __restrict__ ebase, const int* __restrict__ ewidth, const int* __restrict__ ptr,
           const int* __restrict__ col, const double* __restrict__ val, int* __restrict__ ecol,
           double* __restrict__ eval) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int i = order[t], c = colour[i];
  const int cnt = coff[c + 1] - coff[c], tl = t - coff[c], w = ewidth[c];
  const long long base = ebase[c];
  const int lo = ptr[i], len = ptr[i + 1] - lo;
  for (int e = 0; e < w; ++e) {
    const long long q = base + (long long)e * cnt + tl;
    ecol[q] = e < len ? col[lo + e] : i;
    eval[q] = e < len ? val[lo + e] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// cycle kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ void relax_row(int i, const int* __restrict__ ptr, const int* __restrict__ col,
                                          const double* __restrict__ val, const double* __restrict__ diag,
                                          const double* __restrict__ b, double* x) {
  double ax = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) ax += val[k] * x[col[k]];
  x[i] += (b[i] - ax) / diag[i];
}

// one colour's rows from its ELL block (the same sums, in the same order, as the CSR rows)
__global__ void __launch_bounds__(kRsBlock)
k_rs_relax(const int* __restrict__ rows, int cnt, int w, const int* __restrict__ ecol,
           const double* __restrict__ eval, const double* __restrict__ diag, const double* __restrict__ b, double* x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const int i = rows[t];
  double ax = 0.0;
  for (int e = 0; e < w; ++e) ax += eval[(size_t)e * cnt + t] * x[ecol[(size_t)e * cnt + t]];
  x[i] += (b[i] - ax) / diag[i];
}

__global__ void __launch_bounds__(kRsBlock)
k_rs_resid(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
           const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ax = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) ax += val[k] * x[col[k]];
  r[i] = b[i] - ax;
}

// y = M v (add = 0) or y += M v (add = 1)
__global__ void __launch_bounds__(kRsBlock)
k_rs_spmv(int n, const int* __restrict__ ptr, const int* __restrict__ col, const double* __restrict__ val,
          const double* __restrict__ v, double* __restrict__ y, int add) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * v[col[k]];
  y[i] = add ? y[i] + s : s;
}

__global__ void k_rs_fill(double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

__global__ void k_rs_to_dense(int n, const int* __restrict__ ptr, const int* __restrict__ col,
                              const double* __restrict__ val, double* __restrict__ D) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < n; ++j) D[(size_t)i * n + j] = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) D[(size_t)i * n + col[k]] = val[k];
}

__global__ void k_rs_dense_apply(int n, const double* __restrict__ M, const double* __restrict__ b,
                                 double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += M[(size_t)i * n + j] * b[j];
  x[i] = s;
}

// The V-cycle below level `first` in one workgroup (levels of < kRsSmall rows).
struct RsTailLevel {
  int n, nc, ncol;
  const int *ptr, *col, *pptr, *pcol, *rptr, *rcol, *corder, *coff;
  const double *val, *diag, *pval, *rval;
  double *x, *b, *r;
};
struct RsTailArgs {
  RsTailLevel L[kMaxRsLevels];
  int nlev, sweeps;
  const double* Ainv;  // coarsest dense inverse
  int ncoarse;
};

__device__ void tail_sweeps(const RsTailLevel& L, int sweeps) {
  for (int s = 0; s < sweeps; ++s)
    for (int dir = 0; dir < 2; ++dir)
      for (int cc = 0; cc < L.ncol; ++cc) {
        const int c = dir ? L.ncol - 1 - cc : cc;
        for (int t = L.coff[c] + (int)threadIdx.x; t < L.coff[c + 1]; t += blockDim.x)
          relax_row(L.corder[t], L.ptr, L.col, L.val, L.diag, L.b, L.x);
        __syncthreads();
      }
}

__global__ void __launch_bounds__(1024) k_rs_tail(const RsTailArgs* __restrict__ A) {
  const int nl = A->nlev;
  // down
  for (int l = 0; l < nl - 1; ++l) {
    const RsTailLevel& L = A->L[l];
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) L.x[i] = 0.0;
    __syncthreads();
    tail_sweeps(L, A->sweeps);
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
      double ax = 0.0;
      for (int k = L.ptr[i]; k < L.ptr[i + 1]; ++k) ax += L.val[k] * L.x[L.col[k]];
      L.r[i] = L.b[i] - ax;
    }
    __syncthreads();
    const RsTailLevel& N = A->L[l + 1];
    for (int I = threadIdx.x; I < L.nc; I += blockDim.x) {
      double s = 0.0;
      for (int k = L.rptr[I]; k < L.rptr[I + 1]; ++k) s += L.rval[k] * L.r[L.rcol[k]];
      N.b[I] = s;
    }
    __syncthreads();
  }
  // coarsest
  if (!A->Ainv) {
    const RsTailLevel& C = A->L[nl - 1];
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) C.x[i] = 0.0;
    __syncthreads();
    tail_sweeps(C, A->sweeps);
    tail_sweeps(C, A->sweeps);
  } else {
    const RsTailLevel& C = A->L[nl - 1];
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) {
      double s = 0.0;
      for (int j = 0; j < C.n; ++j) s += A->Ainv[(size_t)i * C.n + j] * C.b[j];
      C.x[i] = s;
    }
    __syncthreads();
  }
  // up
  for (int l = nl - 2; l >= 0; --l) {
    const RsTailLevel& L = A->L[l];
    const RsTailLevel& N = A->L[l + 1];
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
      double s = 0.0;
      for (int k = L.pptr[i]; k < L.pptr[i + 1]; ++k) s += L.pval[k] * N.x[L.pcol[k]];
      L.x[i] += s;
    }
    __syncthreads();
    tail_sweeps(L, A->sweeps);
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
long long read_ll(RSHier& H, hipStream_t s, const long long* dptr) {
  VP_HIP(hipMemcpyAsync(H.hint, dptr, sizeof(long long), hipMemcpyDeviceToHost, s));
  VP_HIP(hipStreamSynchronize(s));
  return H.hint[0];
}

int read_int(RSHier& H, hipStream_t s, const int* dptr, int count = 1, int* out = nullptr) {
  VP_HIP(hipMemcpyAsync(H.hint, dptr, count * sizeof(int), hipMemcpyDeviceToHost, s));
  VP_HIP(hipStreamSynchronize(s));
  const int* v = reinterpret_cast<const int*>(H.hint);
  if (out) std::memcpy(out, v, count * sizeof(int));
  return v[0];
}

// ptr[0..n] from cnt[0..n), total returned
size_t scan(RSHier& H, hipStream_t s, const int* cnt, int* ptr, size_t n) {
  const int nb = (int)std::max<size_t>(1, (n + kScanChunk - 1) / kScanChunk);
  ensure(H.bsum, H.c_bsum, (size_t)nb + 1);
  hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanBlock), 0, s, cnt, n, ptr, H.bsum);
  VP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, H.bsum, nb, H.bsum + nb);
  VP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_add, dim3(rs_grid(std::max<size_t>(n, 1))), dim3(kRsBlock), 0, s, ptr, n, H.bsum,
                     H.bsum + nb);
  VP_LAUNCH_CHECK();
  const long long tot = read_ll(H, s, H.bsum + nb);
  if (tot > (long long)INT_MAX) throw Error(VP_EINVAL, "classical AMG: a level exceeds 2^31 entries");
  return (size_t)tot;
}

int row_max(RSHier& H, hipStream_t s, const int* ptr, int n) {
  hipLaunchKernelGGL(k_rs_zero_ints, dim3(1), dim3(64), 0, s, H.dint, 64);
  VP_LAUNCH_CHECK();
  if (n > 0) {
    hipLaunchKernelGGL(k_rs_rowmax, dim3(rs_grid(n)), dim3(kRsBlock), 0, s, n, ptr, H.dint);
    VP_LAUNCH_CHECK();
  }
  return read_int(H, s, H.dint);
}

// C = L * R (rows nrows), C's arrays sized here
void spgemm(RSHier& H, hipStream_t s, int nrows, const int* Lptr, const int* Lcol, const double* Lval,
            const int* Rptr, const int* Rcol, const double* Rval, int*& Cptr, size_t& cCptr, int*& Ccol,
            size_t& cCcol, double*& Cval, size_t& cCval, size_t* nnz_out) {
  const int K = row_max(H, s, Lptr, nrows);
  if (K > kMaxMergeList) throw Error(VP_EINVAL, "classical AMG: operator row longer than the merge limit");
  const size_t lds = (size_t)std::max(K, 1) * kMergeBlock * sizeof(unsigned short);
  ensure(Cptr, cCptr, (size_t)nrows + 1);
  ensure(H.cnt, H.c_cnt, (size_t)nrows + 1);
  const unsigned g = rs_grid(nrows, kMergeBlock);
  hipLaunchKernelGGL((k_rs_spgemm<false>), dim3(g), dim3(kMergeBlock), lds, s, nrows, Lptr, Lcol, Lval, Rptr,
                     Rcol, Rval, (const int*)nullptr, H.cnt, (int*)nullptr, (double*)nullptr);
  VP_LAUNCH_CHECK();
  const size_t nnz = scan(H, s, H.cnt, Cptr, nrows);
  ensure(Ccol, cCcol, nnz);
  ensure(Cval, cCval, nnz);
  hipLaunchKernelGGL((k_rs_spgemm<true>), dim3(g), dim3(kMergeBlock), lds, s, nrows, Lptr, Lcol, Lval, Rptr, Rcol,
                     Rval, (const int*)Cptr, (int*)nullptr, Ccol, Cval);
  VP_LAUNCH_CHECK();
  *nnz_out = nnz;
}

void colour_level(RSHier& H, hipStream_t s, RSLevel& L) {
  const int n = L.n;
  ensure(L.colour, L.c_colour, n);
  ensure(L.corder, L.c_corder, n);
  ensure(H.sel, H.c_sel, n);
  const unsigned g = rs_grid(n);
  hipLaunchKernelGGL(k_col_init, dim3(g), dim3(kRsBlock), 0, s, n, L.colour);
  VP_LAUNCH_CHECK();
  int ctr[3] = {0, 0, 0};
  for (int round = 0;; ++round) {
    if (round >= kMaxRounds) throw Error(VP_EINVAL, "classical AMG: colouring did not finish");
    hipLaunchKernelGGL(k_rs_zero_ints, dim3(1), dim3(64), 0, s, H.dint, 64);
    hipLaunchKernelGGL(k_col_select, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, L.colour, H.sel);
    VP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_col_assign, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, H.sel, L.colour, H.dint);
    VP_LAUNCH_CHECK();
    read_int(H, s, H.dint, 3, ctr);
    if (ctr[2] > 0) throw Error(VP_EINVAL, "classical AMG: more than 128 colours needed");
    if (ctr[0] == 0) break;
  }
  // rows per colour, offsets, rows sorted by colour
  hipLaunchKernelGGL(k_rs_zero_ints, dim3(1), dim3(kMaxColours + 1), 0, s, H.dint, kMaxColours + 1);
  hipLaunchKernelGGL(k_col_count, dim3(g), dim3(kRsBlock), 0, s, n, L.colour, H.dint);
  VP_LAUNCH_CHECK();
  std::vector<int> counts(kMaxColours);
  read_int(H, s, H.dint, kMaxColours, counts.data());
  int ncol = 0;
  for (int c = 0; c < kMaxColours; ++c)
    if (counts[c] > 0) ncol = c + 1;
  L.ncol = ncol;
  L.coff_h.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) L.coff_h[c + 1] = L.coff_h[c] + counts[c];
  ensure(L.coff, L.c_coff, (size_t)ncol + 1);
  VP_HIP(hipMemcpyAsync(L.coff, L.coff_h.data(), (ncol + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  VP_HIP(hipMemcpyAsync(H.dint, L.coff_h.data(), ncol * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_col_scatter, dim3(g), dim3(kRsBlock), 0, s, n, L.colour, H.dint, L.corder);
  VP_LAUNCH_CHECK();
  // ELL blocks: widths per colour, bases, fill
  hipLaunchKernelGGL(k_rs_zero_ints, dim3(1), dim3(kMaxColours), 0, s, H.dint, kMaxColours);
  hipLaunchKernelGGL(k_col_width, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.colour, H.dint);
  VP_LAUNCH_CHECK();
  L.ewidth_h.assign(ncol, 0);
  read_int(H, s, H.dint, ncol, L.ewidth_h.data());
  L.ebase_h.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) L.ebase_h[c + 1] = L.ebase_h[c] + (long long)L.ewidth_h[c] * counts[c];
  const size_t ne = (size_t)L.ebase_h[ncol];
  ensure(L.ecol, L.c_ecol, ne);
  ensure(L.eval, L.c_eval, ne);
  ensure(L.eoff, L.c_eoff, (size_t)3 * ncol + 2);  // ebase as long long (2 ints each) then widths
  long long* ebase_d = reinterpret_cast<long long*>(L.eoff);
  int* ewidth_d = L.eoff + 2 * ncol;
  VP_HIP(hipMemcpyAsync(ebase_d, L.ebase_h.data(), ncol * sizeof(long long), hipMemcpyHostToDevice, s));
  VP_HIP(hipMemcpyAsync(ewidth_d, L.ewidth_h.data(), ncol * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_ell_fill, dim3(g), dim3(kRsBlock), 0, s, n, L.corder, L.colour, L.coff, ebase_d, ewidth_d,
                     L.ptr, L.col, L.val, L.ecol, L.eval);
  VP_LAUNCH_CHECK();
  VP_HIP(hipStreamSynchronize(s));  // the host vectors are read by the copies above
}

void free_level(RSLevel& L) {
  void* bufs[] = {L.ptr, L.col, L.val, L.diag, L.cf, L.cidx, L.pptr, L.pcol, L.pval, L.rptr, L.rcol,
                  L.rval, L.colour, L.corder, L.coff, L.ecol, L.eval, L.eoff, L.x, L.b, L.r, L.Ainv};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  L = RSLevel();
}

}  // namespace

void rs_free(vp_ctx c) {
  if (!c->rs) return;
  RSHier& H = *c->rs;
  for (RSLevel& L : H.lev) free_level(L);
  void* bufs[] = {H.cnt, H.lam, H.sel, H.strong, H.tpos, H.cfine, H.apptr, H.apcol, H.apval, H.bsum, H.dint,
                  H.targs};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (H.hint) (void)hipHostFree(H.hint);
  delete c->rs;
  c->rs = nullptr;
}

void rs_setup(vp_ctx c, double theta, double max_row_sum, int sweeps, int max_coarse) {
  if (!c->rs) {
    c->rs = new RSHier();
    RSHier& H = *c->rs;
    VP_HIP(hipMalloc((void**)&H.dint, 256 * sizeof(int)));
    VP_HIP(hipHostMalloc((void**)&H.hint, 256 * sizeof(long long), hipHostMallocDefault));
    VP_HIP(hipMalloc(&H.targs, sizeof(RsTailArgs)));
  }
  RSHier& H = *c->rs;
  hipStream_t s = c->stream;
  H.sweeps = sweeps;
  // finest level from the assembled stencil
  {
    RSLevel& L = H.lev[0];
    const size_t nn = c->nn;
    const int nxn = c->ec.nxn, nyn = c->ec.nyn;
    const double* A = c->order == 2 ? c->K2 : c->lev[0].A64;
    L.n = (int)(2 * nn);
    ensure(L.ptr, L.c_ptr, 2 * nn + 1);
    ensure(H.cnt, H.c_cnt, 2 * nn + 1);
    const unsigned g = rs_grid(2 * nn);
    if (c->order == 2)
      hipLaunchKernelGGL((k_rs_from_stencil<2, false>), dim3(g), dim3(kRsBlock), 0, s, A, nn, nxn, nyn,
                         (const int*)nullptr, H.cnt, (int*)nullptr, (double*)nullptr);
    else
      hipLaunchKernelGGL((k_rs_from_stencil<1, false>), dim3(g), dim3(kRsBlock), 0, s, A, nn, nxn, nyn,
                         (const int*)nullptr, H.cnt, (int*)nullptr, (double*)nullptr);
    VP_LAUNCH_CHECK();
    L.nnz = scan(H, s, H.cnt, L.ptr, 2 * nn);
    ensure(L.col, L.c_col, L.nnz);
    ensure(L.val, L.c_val, L.nnz);
    if (c->order == 2)
      hipLaunchKernelGGL((k_rs_from_stencil<2, true>), dim3(g), dim3(kRsBlock), 0, s, A, nn, nxn, nyn,
                         (const int*)L.ptr, (int*)nullptr, L.col, L.val);
    else
      hipLaunchKernelGGL((k_rs_from_stencil<1, true>), dim3(g), dim3(kRsBlock), 0, s, A, nn, nxn, nyn,
                         (const int*)L.ptr, (int*)nullptr, L.col, L.val);
    VP_LAUNCH_CHECK();
  }
  int l = 0;
  for (;; ++l) {
    RSLevel& L = H.lev[l];
    const int n = L.n;
    const unsigned g = rs_grid(n);
    ensure(L.diag, L.c_diag, n);
    if (n <= max_coarse || l + 1 >= kMaxRsLevels) break;
    // strength and measures
    ensure(H.strong, H.c_strong, L.nnz);
    ensure(H.tpos, H.c_tpos, L.nnz);
    ensure(H.lam, H.c_lam, n);
    ensure(H.sel, H.c_sel, n);
    ensure(L.cf, L.c_cf, n);
    hipLaunchKernelGGL(k_rs_zero_ints, dim3(g), dim3(kRsBlock), 0, s, H.lam, n);
    hipLaunchKernelGGL(k_rs_strength, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, L.val, theta, max_row_sum,
                       H.strong, H.lam, L.diag);
    VP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rs_tpos, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, H.tpos);
    VP_LAUNCH_CHECK();
    // coarsening rounds
    hipLaunchKernelGGL(k_rs_cf_init, dim3(g), dim3(kRsBlock), 0, s, n, H.lam, L.cf);
    VP_LAUNCH_CHECK();
    for (int round = 0;; ++round) {
      if (round >= kMaxRounds) throw Error(VP_EINVAL, "classical AMG: coarsening did not finish");
      hipLaunchKernelGGL(k_rs_select, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, H.strong, H.tpos, L.cf,
                         H.lam, H.sel);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_rs_mark, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, H.strong, H.tpos, H.sel, L.cf);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_rs_update, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, H.strong, H.sel, L.cf, H.lam);
      VP_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_rs_zero_ints, dim3(1), dim3(64), 0, s, H.dint, 64);
      hipLaunchKernelGGL(k_rs_finish_round, dim3(g), dim3(kRsBlock), 0, s, n, L.cf, H.lam, H.dint);
      VP_LAUNCH_CHECK();
      if (read_int(H, s, H.dint) == 0) break;
    }
    // coarse numbering
    ensure(L.cidx, L.c_cidx, (size_t)n + 1);
    hipLaunchKernelGGL(k_rs_is_c, dim3(g), dim3(kRsBlock), 0, s, n, L.cf, H.cnt);
    VP_LAUNCH_CHECK();
    const int nc = (int)scan(H, s, H.cnt, L.cidx, n);
    if (nc == 0 || nc == n) break;  // no further coarsening possible
    L.nc = nc;
    ensure(H.cfine, H.c_cfine, nc);
    hipLaunchKernelGGL(k_rs_cfine, dim3(g), dim3(kRsBlock), 0, s, n, L.cf, L.cidx, H.cfine);
    VP_LAUNCH_CHECK();
    // interpolation
    ensure(L.pptr, L.c_pptr, (size_t)n + 1);
    hipLaunchKernelGGL(k_rs_pcount, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, H.strong, L.cf, H.cnt);
    VP_LAUNCH_CHECK();
    L.nnzP = scan(H, s, H.cnt, L.pptr, n);
    ensure(L.pcol, L.c_pcol, L.nnzP);
    ensure(L.pval, L.c_pval, L.nnzP);
    hipLaunchKernelGGL(k_rs_pfill, dim3(g), dim3(kRsBlock), 0, s, n, L.ptr, L.col, L.val, H.strong, L.cf, L.cidx,
                       L.diag, L.pptr, L.pcol, L.pval);
    VP_LAUNCH_CHECK();
    // restriction R = P^T
    ensure(L.rptr, L.c_rptr, (size_t)nc + 1);
    const unsigned gc = rs_grid(nc);
    hipLaunchKernelGGL((k_rs_restrictor<false>), dim3(gc), dim3(kRsBlock), 0, s, nc, H.cfine, L.ptr, L.col, L.cf,
                       L.pptr, L.pcol, L.pval, (const int*)nullptr, H.cnt, (int*)nullptr, (double*)nullptr);
    VP_LAUNCH_CHECK();
    L.nnzR = scan(H, s, H.cnt, L.rptr, nc);
    ensure(L.rcol, L.c_rcol, L.nnzR);
    ensure(L.rval, L.c_rval, L.nnzR);
    hipLaunchKernelGGL((k_rs_restrictor<true>), dim3(gc), dim3(kRsBlock), 0, s, nc, H.cfine, L.ptr, L.col, L.cf,
                       L.pptr, L.pcol, L.pval, (const int*)L.rptr, (int*)nullptr, L.rcol, L.rval);
    VP_LAUNCH_CHECK();
    // Galerkin: AP = A P, A_c = R (AP)
    size_t nnzAP = 0;
    spgemm(H, s, n, L.ptr, L.col, L.val, L.pptr, L.pcol, L.pval, H.apptr, H.c_apptr, H.apcol, H.c_apcol, H.apval,
           H.c_apval, &nnzAP);
    RSLevel& N = H.lev[l + 1];
    N.n = nc;
    spgemm(H, s, nc, L.rptr, L.rcol, L.rval, H.apptr, H.apcol, H.apval, N.ptr, N.c_ptr, N.col, N.c_col, N.val,
           N.c_val, &N.nnz);
    colour_level(H, s, L);
    ensure(L.x, L.c_x, (size_t)n);
    ensure(L.b, L.c_b, (size_t)n);
    ensure(L.r, L.c_r, (size_t)n);
  }
  H.nlev = l + 1;
  // coarsest: dense inverse, or (coarsening stalled on a large level) smoothing only
  {
    RSLevel& C = H.lev[H.nlev - 1];
    const int n = C.n;
    C.nc = 0;
    C.smooth_only = n > kDenseMax;
    if (C.smooth_only) {
      hipLaunchKernelGGL(k_rs_diag, dim3(rs_grid(n)), dim3(kRsBlock), 0, s, n, C.ptr, C.col, C.val, C.diag);
      VP_LAUNCH_CHECK();
      colour_level(H, s, C);
    } else {
      ensure(C.Ainv, C.c_ainv, (size_t)n * n);
      hipLaunchKernelGGL(k_rs_to_dense, dim3(rs_grid(n)), dim3(kRsBlock), 0, s, n, C.ptr, C.col, C.val, C.Ainv);
      VP_LAUNCH_CHECK();
      launch_dense_inverse(s, C.Ainv, n);
    }
    ensure(C.x, C.c_x, (size_t)n);
    ensure(C.b, C.c_b, (size_t)n);
  }
  // the one-workgroup tail: the first level from which every level is small
  H.tail = -1;
  for (int k = 1; k < H.nlev; ++k)
    if (H.lev[k].n < kRsSmall) { H.tail = k; break; }
  if (H.tail > 0) {
    RsTailArgs a{};
    a.nlev = H.nlev - H.tail;
    a.sweeps = H.sweeps;
    for (int k = 0; k < a.nlev; ++k) {
      const RSLevel& L = H.lev[H.tail + k];
      RsTailLevel& T = a.L[k];
      T.n = L.n; T.nc = L.nc; T.ncol = L.ncol;
      T.ptr = L.ptr; T.col = L.col; T.val = L.val; T.diag = L.diag;
      T.pptr = L.pptr; T.pcol = L.pcol; T.pval = L.pval;
      T.rptr = L.rptr; T.rcol = L.rcol; T.rval = L.rval;
      T.corder = L.corder; T.coff = L.coff;
      T.x = L.x; T.b = L.b; T.r = L.r;
    }
    a.Ainv = H.lev[H.nlev - 1].smooth_only ? nullptr : H.lev[H.nlev - 1].Ainv;
    a.ncoarse = H.lev[H.nlev - 1].n;
    VP_HIP(hipMemcpyAsync(H.targs, &a, sizeof(a), hipMemcpyHostToDevice, s));
    VP_HIP(hipStreamSynchronize(s));
  }
  VP_HIP(hipStreamSynchronize(s));
}

namespace {

void relax_level(vp_ctx c, const RSLevel& L, const double* b, double* x, int sweeps) {
  hipStream_t s = c->stream;
  for (int sw = 0; sw < sweeps; ++sw)
    for (int dir = 0; dir < 2; ++dir)
      for (int cc = 0; cc < L.ncol; ++cc) {
        const int col = dir ? L.ncol - 1 - cc : cc;
        const int cnt = L.coff_h[col + 1] - L.coff_h[col];
        if (cnt == 0) continue;
        hipLaunchKernelGGL(k_rs_relax, dim3(rs_grid(cnt)), dim3(kRsBlock), 0, s, L.corder + L.coff_h[col], cnt,
                           L.ewidth_h[col], L.ecol + L.ebase_h[col], L.eval + L.ebase_h[col], L.diag, b, x);
        VP_LAUNCH_CHECK();
      }
}

void rs_level(vp_ctx c, int l, const double* b, double* x) {
  RSHier& H = *c->rs;
  hipStream_t s = c->stream;
  RSLevel& L = H.lev[l];
  if (l == H.nlev - 1) {
    if (L.smooth_only) {
      hipLaunchKernelGGL(k_rs_fill, dim3(rs_grid(L.n)), dim3(kRsBlock), 0, s, x, L.n);
      VP_LAUNCH_CHECK();
      relax_level(c, L, b, x, 2 * H.sweeps);
      return;
    }
    hipLaunchKernelGGL(k_rs_dense_apply, dim3(rs_grid(L.n)), dim3(kRsBlock), 0, s, L.n, L.Ainv, b, x);
    VP_LAUNCH_CHECK();
    return;
  }
  RSLevel& N = H.lev[l + 1];
  const unsigned g = rs_grid(L.n);
  hipLaunchKernelGGL(k_rs_fill, dim3(g), dim3(kRsBlock), 0, s, x, L.n);
  VP_LAUNCH_CHECK();
  relax_level(c, L, b, x, H.sweeps);
  hipLaunchKernelGGL(k_rs_resid, dim3(g), dim3(kRsBlock), 0, s, L.n, L.ptr, L.col, L.val, x, b, L.r);
  VP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_rs_spmv, dim3(rs_grid(L.nc)), dim3(kRsBlock), 0, s, L.nc, L.rptr, L.rcol, L.rval, L.r, N.b,
                     0);
  VP_LAUNCH_CHECK();
  if (l + 1 == H.tail) {
    hipLaunchKernelGGL(k_rs_tail, dim3(1), dim3(1024), 0, s, (const RsTailArgs*)H.targs);
    VP_LAUNCH_CHECK();
  } else {
    rs_level(c, l + 1, N.b, N.x);
  }
  hipLaunchKernelGGL(k_rs_spmv, dim3(g), dim3(kRsBlock), 0, s, L.n, L.pptr, L.pcol, L.pval, N.x, x, 1);
  VP_LAUNCH_CHECK();
  relax_level(c, L, b, x, H.sweeps);
}

}  // namespace

void rs_apply(vp_ctx c, const double* r, double* z) {
  if (!c->rs || c->rs->nlev == 0) throw Error(VP_ESTATE, "classical AMG not set up");
  rs_level(c, 0, r, z);
}

int rs_levels(vp_ctx c) { return c->rs ? c->rs->nlev : 0; }

void rs_info(vp_ctx c, int level, long long* out) {
  const RSLevel& L = c->rs->lev[level];
  out[0] = L.n;
  out[1] = (long long)L.nnz;
  out[2] = L.nc;
  out[3] = (long long)L.nnzP;
  out[4] = L.ncol;
}

void rs_export(vp_ctx c, int level, int* A_ptr, int* A_col, double* A_val, int* cf, int* P_ptr, int* P_col,
               double* P_val, int* colour) {
  const RSLevel& L = c->rs->lev[level];
  hipStream_t s = c->stream;
  const bool coarsest = level == c->rs->nlev - 1;
  if (A_ptr) VP_HIP(hipMemcpyAsync(A_ptr, L.ptr, (L.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (A_col) VP_HIP(hipMemcpyAsync(A_col, L.col, L.nnz * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (A_val) VP_HIP(hipMemcpyAsync(A_val, L.val, L.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (coarsest) return;
  if (cf) {
    std::vector<int8_t> h(L.n);
    VP_HIP(hipMemcpyAsync(h.data(), L.cf, L.n, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    std::vector<int> hi(h.begin(), h.end());
    VP_HIP(hipMemcpyAsync(cf, hi.data(), L.n * sizeof(int), hipMemcpyHostToDevice, s));
    VP_HIP(hipStreamSynchronize(s));
  }
  if (P_ptr) VP_HIP(hipMemcpyAsync(P_ptr, L.pptr, (L.n + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (P_col) VP_HIP(hipMemcpyAsync(P_col, L.pcol, L.nnzP * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (P_val) VP_HIP(hipMemcpyAsync(P_val, L.pval, L.nnzP * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (colour) VP_HIP(hipMemcpyAsync(colour, L.colour, L.n * sizeof(int), hipMemcpyDeviceToDevice, s));
}

}  // namespace vp
