// 1D moments of basis pairs against the Lagrange basis on the Chebyshev
// nodes (eq. defV in node form), FP64:
//
//   M[d][a][p] = int_{-L}^{L} g_{mu,d}(x) g_{nu,d}(x) l_a(x) dx.
//
// By the Gaussian product rule (Prop. 2.1, eq. gauss_prod) the integrand is
//   N N' (x-A)^l (x-B)^l' E exp(-p (x-P)^2),  p = a+b, P = (aA+bB)/p,
//   E = exp(-ab/p (A-B)^2).
// One thread owns one (pair, direction).  It integrates over the box
// intersected with P +- 9/sqrt(p) (beyond which the Gaussian is below e^-81
// of its peak) with a fixed composite Gauss-Legendre rule, accumulating the
// Chebyshev moments int f(x) T_k(x/L) dx by the three-term recurrence -- the
// paper's own W matrices of eq. defV in the T_k basis -- and maps them to the
// Lagrange basis with the fixed n x n matrix gam.  Every thread runs the same
// instruction stream, so the wavefront never diverges.
#include "tai_internal.h"
#include "tai_device.h"

#include <algorithm>

#include <cmath>

namespace tai {
namespace {

__device__ inline double norm_1d(double a, int l) {
  // [(2a/pi)^(1/2) (4a)^l / (2l-1)!!]^(1/2)
  double df = 1.0;
  for (int k = 2 * l - 1; k > 0; k -= 2) df *= k;
  double p4 = 1.0;
  for (int k = 0; k < l; ++k) p4 *= 4.0 * a;
  return sqrt(sqrt(2.0 * a / M_PI) * p4 / df);
}

__device__ inline double ipow(double x, int l) {
  double r = 1.0;
  for (int k = 0; k < l; ++k) r *= x;
  return r;
}

template <int NMAX>
__device__ inline void moments_body(const DevBasis& bs, int n, double L, const NodeTables& tb,
                                    double* __restrict__ M, int64_t npair, const int32_t* __restrict__ pairs = nullptr) {
  // the GL panel rule and the Chebyshev-to-node map, read at uniform
  // addresses by every thread, come from LDS
  __shared__ double s_pz[kMomOrder], s_pw[kMomOrder];
  __shared__ double s_gam[NMAX * NMAX];
  for (int i = threadIdx.x; i < NMAX * NMAX; i += blockDim.x) {
    const int ai = i / NMAX, k = i - ai * NMAX;
    s_gam[i] = (ai < n && k < n) ? tb.gam[ai * n + k] : 0.0;
  }
  for (int i = threadIdx.x; i < kMomOrder; i += blockDim.x) {
    s_pz[i] = tb.pz[i];
    s_pw[i] = tb.pw[i];
  }
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * npair) return;
  const int d = (int)(g / npair);
  const int64_t p = g - d * npair;
  // column p is pair pairs[p] of the full list when a screened list is given
  int64_t gp = p;
  bool valid = true;
  if (pairs) {
    gp = pairs[p];
    valid = gp >= 0 && gp < (int64_t)bs.nb * (bs.nb + 1) / 2;
    if (!valid) gp = 0;
  }
  int mu, nu;
  decode_pair(bs.nb, gp, mu, nu);

  const double a = bs.alpha[mu], b = bs.alpha[nu];
  const double A = bs.center[3 * mu + d], B = bs.center[3 * nu + d];
  const int la = bs.lxyz[3 * mu + d], lb = bs.lxyz[3 * nu + d];
  double nrm;
  if (bs.coef) {
    nrm = (d == 0) ? bs.coef[mu] * bs.coef[nu] : 1.0;
  } else {
    nrm = norm_1d(a, la) * norm_1d(b, lb);
  }
  const double pp = a + b;
  const double P = (a * A + b * B) / pp;
  const double E = exp(-a * b / pp * (A - B) * (A - B));
  const double pref = valid ? nrm * E : 0.0;
  const double half = 9.0 / sqrt(pp);
  const double lo = fmax(-L, P - half);
  const double hi = fmin(L, P + half);
  const double h = (hi > lo) ? (hi - lo) / kMomPanels : 0.0;
  const double invL = 1.0 / L;

  double mom[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) mom[k] = 0.0;

  for (int s = 0; s < kMomPanels; ++s) {
    const double mid = lo + (s + 0.5) * h;
    for (int j = 0; j < kMomOrder; ++j) {
      const double x = mid + 0.5 * h * s_pz[j];
      const double dxp = x - P;
      const double f = pref * (0.5 * h * s_pw[j]) * ipow(x - A, la) * ipow(x - B, lb) * exp(-pp * dxp * dxp);
      const double u = x * invL;
      double t0 = 1.0, t1 = u;
      mom[0] += f;
      if (NMAX > 1) mom[1] += f * u;
#pragma unroll
      for (int k = 2; k < NMAX; ++k) {
        const double t2 = 2.0 * u * t1 - t0;
        mom[k] += f * t2;
        t0 = t1;
        t1 = t2;
      }
    }
  }

  double* out = M + (int64_t)d * n * npair + p;
  for (int ai = 0; ai < n; ++ai) {
    const double* gr = s_gam + ai * NMAX;  // zero beyond n
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) s += gr[k] * mom[k];
    out[(int64_t)ai * npair] = s;
  }
}

template <int NMAX>
__global__ void __launch_bounds__(128)
moments_kernel(DevBasis bs, int n, double L, NodeTables tb, double* __restrict__ M, int64_t npair,
               const int32_t* __restrict__ pairs) {
  moments_body<NMAX>(bs, n, L, tb, M, npair, pairs);
}

// Screening (section 6.3, compression by screening).  One wave per row mu of
// the pair list counts, then writes, the pairs (mu, nu >= mu) whose Gaussian
// product prefactor exp(-ab/(a+b) |A - B|^2) exceeds tau, 64 columns nu at a
// time: a ballot of the lanes that keep their pair gives each kept lane its
// slot (the kept lanes below it) and the chunk's count.  A single work group
// turns the row counts into offsets in between, so the kept indices come out
// in ascending order.  The exponent is formed with unfused, left-to-right
// operations.
__device__ inline bool keep_pair(const DevBasis& bs, double tau, int mu, int nu) {
#pragma clang fp contract(off)
  const double a = bs.alpha[mu], b = bs.alpha[nu];
  double r2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double x = bs.center[3 * mu + d] - bs.center[3 * nu + d];
    r2 = r2 + x * x;
  }
  const double e = (a * b) / (a + b) * r2;
  return tau <= 0.0 || exp(-e) > tau;
}

constexpr int kScreenRows = 4;  // rows (one wave each) per work group
constexpr int kScreenThreads = 64 * kScreenRows;

__global__ void __launch_bounds__(kScreenThreads) screen_count_kernel(DevBasis bs, double tau, int32_t* rows) {
  const int mu = blockIdx.x * kScreenRows + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (mu >= bs.nb) return;  // whole waves
  int c = 0;
  for (int nu0 = mu; nu0 < bs.nb; nu0 += 64) {
    const int nu = nu0 + lane;
    c += __popcll(__ballot(nu < bs.nb && keep_pair(bs, tau, mu, nu)));
  }
  if (lane == 0) rows[mu] = c;
}

// exclusive scan of rows[0 .. nb) in place, total to rows[nb] and *count
__global__ void __launch_bounds__(1024) screen_scan_kernel(int nb, int32_t* rows, int32_t* count) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x, per = (nb + 1023) / 1024;
  const int lo = min(nb, t * per), hi = min(nb, lo + per);
  int32_t sum = 0;
  for (int i = lo; i < hi; ++i) sum += rows[i];
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    int32_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const int32_t v = part[i];
      part[i] = acc;
      acc += v;
    }
    rows[nb] = acc;
    *count = acc;
  }
  __syncthreads();
  int32_t acc = part[t];
  for (int i = lo; i < hi; ++i) {
    const int32_t v = rows[i];
    rows[i] = acc;
    acc += v;
  }
}

__global__ void __launch_bounds__(kScreenThreads)
screen_write_kernel(DevBasis bs, double tau, const int32_t* __restrict__ rows, int32_t* __restrict__ pairs) {
  const int mu = blockIdx.x * kScreenRows + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (mu >= bs.nb) return;  // whole waves
  int32_t o = rows[mu];
  const uint64_t below = __lanemask_lt();
  const int64_t p0 = pair_row_start(bs.nb, mu);
  for (int nu0 = mu; nu0 < bs.nb; nu0 += 64) {
    const int nu = nu0 + lane;
    const bool k = nu < bs.nb && keep_pair(bs, tau, mu, nu);
    const uint64_t m = __ballot(k);
    if (k) pairs[o + __popcll(m & below)] = (int32_t)(p0 + (nu - mu));
    o += __popcll(m);
  }
}

// blockIdx.y = partition z of the adaptive boxes: pairs pairs[off[z] ..),
// box half-width L[z], moment block M + 3 n off[z].  Only L depends on the
// box (the node map and panel rule do not), so one launch serves all boxes;
// blocks past a partition's 3 count threads return as a whole.
template <int NMAX>
__global__ void __launch_bounds__(128)
moments_parts_kernel(DevBasis bs, int n, PartSpans sp, NodeTables tb, double* __restrict__ M,
                     const int32_t* __restrict__ pairs) {
  const int z = blockIdx.y;
  const int64_t o = sp.off[z], cnt = sp.off[z + 1] - o;
  if ((int64_t)blockIdx.x * 128 >= 3 * cnt) return;
  moments_body<NMAX>(bs, n, sp.L[z], tb, M + 3 * (int64_t)n * o, cnt, pairs + o);
}

// blockIdx.y = molecule; blocks past a molecule's 3*npair threads return
template <int NMAX>
__global__ void __launch_bounds__(128)
moments_batch_kernel(const PrepMol* __restrict__ mols, int n) {
  const PrepMol& m = mols[blockIdx.y];
  moments_body<NMAX>(m.basis, n, m.L, m.tb, m.M, m.npair);
}

// Coefficient moments mu_d[j][p] = sum_a T_j(xi_a / L) M_d[a][p], the
// moments against T_j (j < n) that the per-node degree form contracts (eq.
// tensors with the nested moments of section 3.2): T_j = sum_a T_j(xi_a) l_a
// for every j < n.  One thread per (pair, direction); the n x n table of
// T_j(xi_a/L) in LDS.
constexpr int kCoefThreads = 256;

template <int NMAX>
__device__ inline void coef_moments_body(const double* __restrict__ M, int n, int64_t npair, int kind,
                                         double* __restrict__ mu) {
  __shared__ double V[NMAX * NMAX];
  for (int e = threadIdx.x; e < n * n; e += kCoefThreads) V[e] = cheb_at_node(kind, n, e / n, e % n);
  __syncthreads();
  const int d = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * kCoefThreads + threadIdx.x;
  if (p >= npair) return;
  double m[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) m[a] = a < n ? M[((int64_t)d * n + a) * npair + p] : 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
      if (a < n) s += V[a * n + j] * m[a];
    mu[((int64_t)d * n + j) * npair + p] = s;
  }
}

template <int NMAX>
__global__ void __launch_bounds__(kCoefThreads)
coef_moments_kernel(const double* __restrict__ M, int n, int64_t npair, int kind, double* __restrict__ mu) {
  coef_moments_body<NMAX>(M, n, npair, kind, mu);
}

// blockIdx.z = molecule; molecules without coefficient moments are skipped
template <int NMAX>
__global__ void __launch_bounds__(kCoefThreads)
coef_moments_batch_kernel(const PrepMol* __restrict__ mols, int n, int kind) {
  const PrepMol& m = mols[blockIdx.z];
  if (m.Mu == nullptr || (int64_t)blockIdx.x * kCoefThreads >= m.npair) return;
  coef_moments_body<NMAX>(m.M, n, m.npair, kind, m.Mu);
}

}  // namespace

hipError_t launch_coef_moments(const double* M, int n, int64_t npair, int kind, double* mu, hipStream_t s) {
  const dim3 grid((unsigned)((npair + kCoefThreads - 1) / kCoefThreads), 3);
  if (n <= 16) hipLaunchKernelGGL(coef_moments_kernel<16>, grid, dim3(kCoefThreads), 0, s, M, n, npair, kind, mu);
  else if (n <= 32) hipLaunchKernelGGL(coef_moments_kernel<32>, grid, dim3(kCoefThreads), 0, s, M, n, npair, kind, mu);
  else if (n <= 48) hipLaunchKernelGGL(coef_moments_kernel<48>, grid, dim3(kCoefThreads), 0, s, M, n, npair, kind, mu);
  else hipLaunchKernelGGL(coef_moments_kernel<64>, grid, dim3(kCoefThreads), 0, s, M, n, npair, kind, mu);
  return hipGetLastError();
}

hipError_t launch_coef_moments_batch(const PrepMol* mols, int nmol, int64_t max_npair, int n, int kind,
                                     hipStream_t s) {
  const dim3 grid((unsigned)((max_npair + kCoefThreads - 1) / kCoefThreads), 3, nmol);
  if (n <= 16) hipLaunchKernelGGL(coef_moments_batch_kernel<16>, grid, dim3(kCoefThreads), 0, s, mols, n, kind);
  else if (n <= 32) hipLaunchKernelGGL(coef_moments_batch_kernel<32>, grid, dim3(kCoefThreads), 0, s, mols, n, kind);
  else if (n <= 48) hipLaunchKernelGGL(coef_moments_batch_kernel<48>, grid, dim3(kCoefThreads), 0, s, mols, n, kind);
  else hipLaunchKernelGGL(coef_moments_batch_kernel<64>, grid, dim3(kCoefThreads), 0, s, mols, n, kind);
  return hipGetLastError();
}

hipError_t launch_moments_batch(const PrepMol* mols, int nmol, int64_t max_npair, int n, hipStream_t s) {
  const unsigned blocks = (unsigned)((3 * max_npair + 127) / 128);
  const dim3 grid(blocks, nmol);
  if (n <= 16) hipLaunchKernelGGL(moments_batch_kernel<16>, grid, dim3(128), 0, s, mols, n);
  else if (n <= 32) hipLaunchKernelGGL(moments_batch_kernel<32>, grid, dim3(128), 0, s, mols, n);
  else if (n <= 48) hipLaunchKernelGGL(moments_batch_kernel<48>, grid, dim3(128), 0, s, mols, n);
  else hipLaunchKernelGGL(moments_batch_kernel<64>, grid, dim3(128), 0, s, mols, n);
  return hipGetLastError();
}

hipError_t launch_moments_pairs(const DevBasis& b, int n, double L, const NodeTables& tb, const int32_t* pairs,
                                int64_t npair, double* M, hipStream_t s) {
  const int64_t total = 3 * npair;
  const int threads = 128;
  const unsigned blocks = (unsigned)((total + threads - 1) / threads);
  if (n <= 16)
    hipLaunchKernelGGL(moments_kernel<16>, dim3(blocks), dim3(threads), 0, s, b, n, L, tb, M, npair, pairs);
  else if (n <= 32)
    hipLaunchKernelGGL(moments_kernel<32>, dim3(blocks), dim3(threads), 0, s, b, n, L, tb, M, npair, pairs);
  else if (n <= 48)
    hipLaunchKernelGGL(moments_kernel<48>, dim3(blocks), dim3(threads), 0, s, b, n, L, tb, M, npair, pairs);
  else
    hipLaunchKernelGGL(moments_kernel<64>, dim3(blocks), dim3(threads), 0, s, b, n, L, tb, M, npair, pairs);
  return hipGetLastError();
}

hipError_t launch_moments_parts(const DevBasis& b, int n, const NodeTables& tb, const int32_t* pairs,
                                const PartSpans& sp, int nparts, double* M, hipStream_t s) {
  int64_t maxc = 0;
  for (int z = 0; z < nparts; ++z) maxc = std::max<int64_t>(maxc, sp.off[z + 1] - sp.off[z]);
  if (maxc == 0) return hipSuccess;
  const dim3 grid((unsigned)((3 * maxc + 127) / 128), (unsigned)nparts);
  if (n <= 16) hipLaunchKernelGGL(moments_parts_kernel<16>, grid, dim3(128), 0, s, b, n, sp, tb, M, pairs);
  else if (n <= 32) hipLaunchKernelGGL(moments_parts_kernel<32>, grid, dim3(128), 0, s, b, n, sp, tb, M, pairs);
  else if (n <= 48) hipLaunchKernelGGL(moments_parts_kernel<48>, grid, dim3(128), 0, s, b, n, sp, tb, M, pairs);
  else hipLaunchKernelGGL(moments_parts_kernel<64>, grid, dim3(128), 0, s, b, n, sp, tb, M, pairs);
  return hipGetLastError();
}

hipError_t launch_moments(const DevBasis& b, int n, double L, const NodeTables& tb,
                          double* M, hipStream_t s) {
  return launch_moments_pairs(b, n, L, tb, nullptr, (int64_t)b.nb * (b.nb + 1) / 2, M, s);
}

hipError_t launch_screen(const DevBasis& b, double tau, int32_t* rows, int32_t* pairs, int32_t* count,
                         hipStream_t s) {
  const unsigned blocks = (unsigned)((b.nb + kScreenRows - 1) / kScreenRows);
  hipLaunchKernelGGL(screen_count_kernel, dim3(blocks), dim3(kScreenThreads), 0, s, b, tau, rows);
  hipLaunchKernelGGL(screen_scan_kernel, dim3(1), dim3(1024), 0, s, b.nb, rows, count);
  hipLaunchKernelGGL(screen_write_kernel, dim3(blocks), dim3(kScreenThreads), 0, s, b, tau, rows, pairs);
  return hipGetLastError();
}

}  // namespace tai
