// Quadrature and interpolation tables on the device, FP64.
//
// * Gauss-Legendre nodes/weights for int_0^omega ds (eq. TEI2 with the
//   Gauss rule of Prop. 2.4), by Newton's method on the Legendre polynomial.
// * Chebyshev nodes on [-L, L], Lobatto or first kind (Def. 2.2).
// * K_k(a,b) = exp(-t_k^2 (xi_a - xi_b)^2): the 1D Gaussian factor of
//   eq. TEI2 on the Chebyshev grid, i.e. the node-value form of the
//   interpolant of eq. chebcheb.
// * The map from Chebyshev moments to Lagrange moments used by the moment
//   kernel: l_a(x) = sum_k gam[a][k] T_k(x/L).
// * The composite Gauss-Legendre panel rule of the moment kernel.
// * Per-node degrees (eq. chebcheb with N_k points for node k): the Chebyshev
//   coefficients of each node's factor, the smallest degree whose dropped
//   coefficients sum to at most a tolerance, and the truncated K tables.
#include "tai_internal.h"
#include "tai_device.h"

#include <cmath>

namespace tai {
namespace {

constexpr int kNodeThreads = 256;
constexpr int kPanelBase = 128;  // threads [128, 128 + kMomOrder) build the panel rule
constexpr int kXiBase = 160;     // threads [160, 160 + n) build the Chebyshev nodes

// Legendre P_m and P_{m-1} at x by the three-term recurrence.
__device__ inline void legendre_pair(int m, double x, double& pm, double& pm1) {
  double p0 = 1.0, p1 = x;
  for (int j = 1; j < m; ++j) {
    const double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pm = p1;
  pm1 = p0;
}

// Root `i` (0-based, descending) of P_m and its Gauss weight.
__device__ inline void gauss_root(int m, int i, double& x, double& wt) {
  x = cos(M_PI * (i + 0.75) / (m + 0.5));
  for (int it = 0; it < 100; ++it) {
    double pm, pm1;
    legendre_pair(m, x, pm, pm1);
    const double dp = m * (x * pm - pm1) / (x * x - 1.0);
    const double dx = pm / dp;
    x -= dx;
    if (fabs(dx) < 1e-15) break;
  }
  double pm, pm1;
  legendre_pair(m, x, pm, pm1);
  const double dp = m * (x * pm - pm1) / (x * x - 1.0);
  wt = 2.0 / ((1.0 - x * x) * dp * dp);
}

__device__ inline void nodes_body(double omega, int nq, int n, double L, int kind, const NodeTables& tb) {
  const int tid = threadIdx.x;
  if (tid < nq) {
    double z, zw;
    gauss_root(nq, tid, z, zw);
    const int k = nq - 1 - tid;  // ascending order
    tb.t[k] = 0.5 * omega * (1.0 + z);
    tb.w[k] = 0.5 * omega * zw;
  } else if (tid >= kPanelBase && tid < kPanelBase + kMomOrder) {
    const int i = tid - kPanelBase;
    double z, zw;
    gauss_root(kMomOrder, i, z, zw);
    tb.pz[kMomOrder - 1 - i] = z;
    tb.pw[kMomOrder - 1 - i] = zw;
  } else if (tid >= kXiBase && tid < kXiBase + n) {
    const int a = tid - kXiBase;
    const double th = (kind == 0) ? M_PI * a / (n - 1) : (2.0 * a + 1.0) * M_PI / (2.0 * n);
    tb.xi[a] = L * cos(th);
  }
}

__global__ void __launch_bounds__(kNodeThreads)
nodes_kernel(double omega, int nq, int n, double L, int kind, NodeTables tb) {
  nodes_body(omega, nq, n, L, kind, tb);
}

// one work group per molecule (blockIdx.y)
__global__ void __launch_bounds__(kNodeThreads)
nodes_batch_kernel(const PrepMol* __restrict__ mols, int nq, int n, int kind) {
  const PrepMol& m = mols[blockIdx.y];
  nodes_body(m.omega, nq, n, m.L, kind, m.tb);
}

// K tables (nq*n*n entries) followed by the n*n Chebyshev-to-Lagrange map.
__device__ inline void ktables_body(int nq, int n, int kind, const NodeTables& tb) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nk = (int64_t)nq * n * n;
  if (g < nk) {
    const int k = (int)(g / ((int64_t)n * n));
    const int ab = (int)(g % ((int64_t)n * n));
    const int a = ab / n, b = ab % n;
    const double dx = tb.xi[a] - tb.xi[b];
    const double t = tb.t[k];
    tb.K[g] = exp(-t * t * dx * dx);
  } else if (g < nk + (int64_t)n * n) {
    const int ak = (int)(g - nk);
    const int a = ak / n, k = ak % n;
    double v;
    if (kind == 0) {
      // Lobatto: l_a(u) = sum_k 2/(N c_a c_k) T_k(u_a) T_k(u), N = n-1,
      // c_0 = c_N = 2, other c = 1; T_k(u_a) = cos(pi a k / N)
      const int N = n - 1;
      const double ca = (a == 0 || a == N) ? 2.0 : 1.0;
      const double ck = (k == 0 || k == N) ? 2.0 : 1.0;
      v = 2.0 / (N * ca * ck) * cos(M_PI * (double)((int64_t)a * k % (2 * N)) / N);
    } else {
      // first kind: l_a(u) = sum_k (2 - delta_k0)/n T_k(u_a) T_k(u),
      // T_k(u_a) = cos(k (2a+1) pi / (2n))
      const double ck = (k == 0) ? 1.0 : 2.0;
      v = ck / n * cos(M_PI * (double)((int64_t)k * (2 * a + 1) % (4 * n)) / (2.0 * n));
    }
    tb.gam[ak] = v;
  }
}

__global__ void __launch_bounds__(256)
ktables_kernel(int nq, int n, int kind, NodeTables tb) {
  ktables_body(nq, n, kind, tb);
}

__global__ void __launch_bounds__(256)
ktables_batch_kernel(const PrepMol* __restrict__ mols, int nq, int n, int kind) {
  ktables_body(nq, n, kind, mols[blockIdx.y].tb);
}

constexpr int kDegThreads = 256;
constexpr int kDegMaxN = 64;
constexpr int kDegPer = kDegMaxN * kDegMaxN / kDegThreads;  // entries per thread

// One work group per node k.  With gam the Chebyshev-to-Lagrange map
// (l_a = sum_j gam[a][j] T_j), the node's interpolant
// sum_ab K_k(a,b) l_a(x) l_b(y) has coefficients C = gam^T K_k gam.  The
// coefficients are summed in absolute value over the shells max(i,j) = s,
// and the tail sums tail(m) = sum_{s >= m} shell(s) taken from the outside
// in: N_k is the smallest m >= 1 with tail(m) <= tol (n if tol <= 0).
// Dropping the rest moves the factor by at most tail(N_k) on the box since
// |T_j| <= 1.  With tol > 0, K_k becomes V C V^T, V[a][j] = T_j(xi_a/L): the
// node values of the kept polynomial, which every node-form stage uses.
__device__ inline void degrees_body(int n, int kind, double tol, const NodeTables& tb, int k) {
  __shared__ double buf[kDegMaxN * kDegMaxN];
  __shared__ double shell[kDegMaxN];
  __shared__ int nk_s;
  const int tid = threadIdx.x, nn = n * n;
  const double* Kk = tb.K + (int64_t)k * nn;
  double v[kDegPer];
  // X = K_k gam
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) {
      const int a = e / n, j = e % n;
      double x = 0.0;
      for (int b = 0; b < n; ++b) x += Kk[a * n + b] * tb.gam[b * n + j];
      buf[e] = x;
    }
  }
  __syncthreads();
  // C = gam^T X
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) {
      const int i = e / n, j = e % n;
      double x = 0.0;
      for (int a = 0; a < n; ++a) x += tb.gam[a * n + i] * buf[a * n + j];
      v[r] = x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) buf[e] = v[r];
  }
  __syncthreads();
  if (tid < n) {
    const int s = tid;
    double x = 0.0;
    for (int j = 0; j <= s; ++j) x += fabs(buf[s * n + j]);
    for (int i = 0; i < s; ++i) x += fabs(buf[i * n + s]);
    shell[s] = x;
  }
  __syncthreads();
  if (tid == 0) {
    int m = n;
    if (tol > 0) {
      double tail = 0.0;
      for (int c = n - 1; c >= 1; --c) {
        tail += shell[c];
        if (tail <= tol) m = c;
        else break;
      }
    }
    nk_s = m;
    tb.nk[k] = m;
  }
  __syncthreads();
  const int m = nk_s;
  double* Ck = tb.C + (int64_t)k * nn;
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) {
      const int i = e / n, j = e % n;
      const double c = (i < m && j < m) ? buf[e] : 0.0;
      Ck[e] = c;
      v[r] = c;
    }
  }
  if (!(tol > 0)) return;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) buf[e] = v[r];
  }
  __syncthreads();
  // Z = C V^T (rows i < m only are nonzero)
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) {
      const int i = e / n, b = e % n;
      double x = 0.0;
      for (int j = 0; j < m; ++j) x += buf[i * n + j] * cheb_at_node(kind, n, b, j);
      v[r] = x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) buf[e] = v[r];
  }
  __syncthreads();
  // K~ = V Z
  double* Kw = tb.K + (int64_t)k * nn;
#pragma unroll
  for (int r = 0; r < kDegPer; ++r) {
    const int e = tid + kDegThreads * r;
    if (e < nn) {
      const int a = e / n, b = e % n;
      double x = 0.0;
      for (int i = 0; i < m; ++i) x += cheb_at_node(kind, n, a, i) * buf[i * n + b];
      Kw[e] = x;
    }
  }
}

__global__ void __launch_bounds__(kDegThreads)
degrees_kernel(int n, int kind, double tol, NodeTables tb) {
  degrees_body(n, kind, tol, tb, blockIdx.x);
}

// one work group per (node, molecule); molecules with tol <= 0 are skipped
__global__ void __launch_bounds__(kDegThreads)
degrees_batch_kernel(const PrepMol* __restrict__ mols, int n, int kind) {
  const PrepMol& m = mols[blockIdx.y];
  if (!(m.degree_tol > 0)) return;
  degrees_body(n, kind, m.degree_tol, m.tb, blockIdx.x);
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t node_tables_bytes(int nq, int n) {
  return align256(sizeof(double) * nq) * 2 + align256(sizeof(double) * n) +
         align256(sizeof(double) * (size_t)nq * n * n) + align256(sizeof(double) * n * n) +
         align256(sizeof(double) * kMomOrder) * 2 + align256(sizeof(double) * (size_t)nq * n * n) +
         align256(sizeof(int32_t) * nq);
}

NodeTables carve_node_tables(void* base, int nq, int n) {
  char* p = static_cast<char*>(base);
  NodeTables tb;
  tb.t = reinterpret_cast<double*>(p); p += align256(sizeof(double) * nq);
  tb.w = reinterpret_cast<double*>(p); p += align256(sizeof(double) * nq);
  tb.xi = reinterpret_cast<double*>(p); p += align256(sizeof(double) * n);
  tb.K = reinterpret_cast<double*>(p); p += align256(sizeof(double) * (size_t)nq * n * n);
  tb.gam = reinterpret_cast<double*>(p); p += align256(sizeof(double) * n * n);
  tb.pz = reinterpret_cast<double*>(p); p += align256(sizeof(double) * kMomOrder);
  tb.pw = reinterpret_cast<double*>(p); p += align256(sizeof(double) * kMomOrder);
  tb.C = reinterpret_cast<double*>(p); p += align256(sizeof(double) * (size_t)nq * n * n);
  tb.nk = reinterpret_cast<int32_t*>(p);
  return tb;
}

hipError_t launch_degrees(int nq, int n, int kind, double degree_tol, const NodeTables& tb, hipStream_t s) {
  if (n > kDegMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(degrees_kernel, dim3(nq), dim3(kDegThreads), 0, s, n, kind, degree_tol, tb);
  return hipGetLastError();
}

hipError_t launch_nodes(double omega, int nq, int n, double L, int kind, double degree_tol,
                        const NodeTables& tb, hipStream_t s) {
  hipLaunchKernelGGL(nodes_kernel, dim3(1), dim3(kNodeThreads), 0, s, omega, nq, n, L, kind, tb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)nq * n * n + (int64_t)n * n;
  const int blocks = (int)((total + 255) / 256);
  hipLaunchKernelGGL(ktables_kernel, dim3(blocks), dim3(256), 0, s, nq, n, kind, tb);
  e = hipGetLastError();
  if (e != hipSuccess || !(degree_tol > 0)) return e;
  return launch_degrees(nq, n, kind, degree_tol, tb, s);
}

hipError_t launch_nodes_batch(const PrepMol* mols, int nmol, int nq, int n, int kind, bool any_degree,
                              hipStream_t s) {
  hipLaunchKernelGGL(nodes_batch_kernel, dim3(1, nmol), dim3(kNodeThreads), 0, s, mols, nq, n, kind);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)nq * n * n + (int64_t)n * n;
  const int blocks = (int)((total + 255) / 256);
  hipLaunchKernelGGL(ktables_batch_kernel, dim3(blocks, nmol), dim3(256), 0, s, mols, nq, n, kind);
  e = hipGetLastError();
  if (e != hipSuccess || !any_degree) return e;
  if (n > kDegMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(degrees_batch_kernel, dim3(nq, nmol), dim3(kDegThreads), 0, s, mols, n, kind);
  return hipGetLastError();
}

}  // namespace tai
