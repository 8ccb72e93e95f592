// Low-rank compression of the moments (section 6.1, eqs. SVD and
// approxepsilon), FP64.  The moment matrices of the three directions are
// stacked side by side, W = [M_1 | M_2 | M_3] (n x 3 npair); its leading left
// singular vectors V (n x R) give compressed moments U_d = V^T M_d and tables
// Kc_k = V^T K_k V, so every factor m_p^T K_k m_q of Theorem 3.1 becomes
// u_p^T Kc_k u_q with inner length R instead of n.
//
//  * Gram matrix G = W W^T = sum_d M_d M_d^T: chunks of pairs per work group,
//    partial G per chunk, the partials summed in a fixed order.
//  * Eigenpairs of G (sigma_r^2 and the left singular vectors of W) by the
//    cyclic Jacobi method in one work group: the n(n-1)/2 rotations of a
//    sweep are applied in n-1 rounds of n/2 disjoint pairs (round-robin
//    order), each round one parallel in-place pass over the 2 x 2 blocks of G
//    in LDS, the columns of V rotated alongside.  Sweeps stop when a whole
//    sweep finds every off-diagonal entry negligible against its diagonal
//    pair.  Eigenvalues are sorted in decreasing order; the rank R is the
//    count of sigma_r > tol * sigma_1 (at least one), the cut of section 6.1.
//    The contractions run their inner index in chunks of 8, so the operands
//    are written at the padded length min(n, 8 ceil(R / 8)) with the basis
//    columns from R on taken as zero: zero rows of U and zero rows and
//    columns of Kc add nothing to any product, and the result is that of
//    rank R.
//  * One refinement pass: Y = V1^T W in the first basis V1, then the Gram
//    matrix of Y (nearly diagonal, its entries (r, s) rounded relative to
//    sigma_r sigma_s rather than sigma_1^2) and its Jacobi eigenvectors V2;
//    the basis is V = V1 V2.  Forming W W^T alone resolves sigma_r only to
//    about 1e-16 sigma_1^2 / sigma_r; after the pass the values and the kept
//    subspace carry errors of about 1e-16 sigma_1 / sigma_r, as an SVD of W.
//  * U and Kc: plain FP64 products with V in LDS.
#include "tai_internal.h"

namespace tai {
namespace {

constexpr int kMaxN = 64;        // largest n the library accepts
constexpr int kGramPairs = 32;   // pairs staged per LDS tile of the Gram kernel
constexpr int kMaxSweeps = 40;

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Partial Gram matrix of the pairs [c*chunk, min((c+1)*chunk, npair)) of the
// three directions: part[c][a][b] = sum_d sum_q M_d(a, q) M_d(b, q).  Thread t
// owns the 4 x 4 block (a0 + i, b0 + j) of G, a0 = 4 (t / 16), b0 = 4 (t % 16).
__global__ void __launch_bounds__(256)
gram_kernel(const double* __restrict__ M, int n, int64_t npair, int64_t chunk, double* __restrict__ part) {
  __shared__ double s_m[kGramPairs][kMaxN + 2];
  const int64_t q0 = (int64_t)blockIdx.x * chunk;
  const int64_t q1 = q0 + chunk < npair ? q0 + chunk : npair;
  const int a0 = 4 * (threadIdx.x / 16), b0 = 4 * (threadIdx.x % 16);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double* Md = M + (int64_t)d * n * npair;
    for (int64_t qb = q0; qb < q1; qb += kGramPairs) {
      __syncthreads();
      for (int e = threadIdx.x; e < kMaxN * kGramPairs; e += 256) {
        const int a = e / kGramPairs, j = e % kGramPairs;
        const int64_t q = qb + j;
        s_m[j][a] = (a < n && q < q1) ? Md[(int64_t)a * npair + q] : 0.0;
      }
      __syncthreads();
      for (int j = 0; j < kGramPairs; ++j) {
        double x[4], y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x[i] = s_m[j][a0 + i];
          y[i] = s_m[j][b0 + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[i][k] += x[i] * y[k];
      }
    }
  }
  double* out = part + (int64_t)blockIdx.x * n * n;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (a0 + i < n && b0 + k < n) out[(a0 + i) * n + b0 + k] = acc[i][k];
}

// G[e] = sum over the chunks of part[c][e]: 64 entries per work group, four
// groups of threads each summing every fourth chunk in order, the four group
// sums then added in a fixed order.
__global__ void __launch_bounds__(256)
gram_sum_kernel(const double* __restrict__ part, int nchunk, int nn, double* __restrict__ G) {
  __shared__ double s_sum[4][64];
  const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + l;
  double s = 0.0;
  if (e < nn)
    for (int c = g; c < nchunk; c += 4) s += part[(int64_t)c * nn + e];
  s_sum[g][l] = s;
  __syncthreads();
  if (g == 0 && e < nn) G[e] = ((s_sum[0][l] + s_sum[1][l]) + s_sum[2][l]) + s_sum[3][l];
}

// Cyclic Jacobi on the symmetric n x n matrix G (n <= 64, padded to an even
// order m with a zero row and column, which no rotation touches).  Outputs
// sigma[r] = sqrt(max(lambda_r, 0)) in decreasing order, V[a][r] the matching
// unit eigenvectors, and *rank.
constexpr int kJacobiThreads = 1024;

// Off-diagonal entries at most rel * sqrt(|a_pp a_qq|), or at most
// floor_rel * trace(G), are left alone: below the floor an entry is rounding
// noise of the Gram matrix itself, and rotating on it would never settle.
__global__ void __launch_bounds__(kJacobiThreads)
jacobi_kernel(const double* __restrict__ G, int n, double tol, double rel, double floor_rel,
              double* __restrict__ sigma, double* __restrict__ V, int32_t* __restrict__ rank) {
  constexpr int S = kMaxN + 1;
  __shared__ double A[kMaxN * S];
  __shared__ double Q[kMaxN * S];
  __shared__ double rc[kMaxN / 2], rs[kMaxN / 2];
  __shared__ int rp[kMaxN / 2], rq[kMaxN / 2];
  __shared__ int order[kMaxN];
  __shared__ int rotated;
  __shared__ double floor_abs;
  const int m = n + (n & 1), half = m / 2;
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += fabs(G[i * n + i]);
    floor_abs = fmax(floor_rel * tr, 1e-290);
  }
  for (int e = threadIdx.x; e < m * m; e += kJacobiThreads) {
    const int i = e / m, j = e % m;
    A[i * S + j] = (i < n && j < n) ? G[i * n + j] : 0.0;
    Q[i * S + j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      // round-robin pairing: slot 0 fixed, the other m-1 slots rotate
      if (threadIdx.x < half) {
        const int i = threadIdx.x;
        auto slot = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + round) % (m - 1); };
        int p = slot(i), q = slot(m - 1 - i);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        const double app = A[p * S + p], aqq = A[q * S + q], apq = A[p * S + q];
        double c = 1.0, s = 0.0;
        // rotate unless apq is negligible against the diagonal pair (a
        // relative test, so tiny eigenvalues of a semi-definite G are still
        // resolved) or below the underflow range
        if (fabs(apq) > rel * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
          // the rotation that zeroes A'(p, q): tan = t, the root of
          // t^2 + 2 theta t - 1 = 0 of smaller size, theta = (aqq - app) / (2 apq)
          const double theta = (aqq - app) / (2.0 * apq);
          const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          rotated = 1;
        }
        rp[i] = p;
        rq[i] = q;
        rc[i] = c;
        rs[i] = s;
      }
      __syncthreads();
      // A <- J^T A J and V <- V J for the block-diagonal J of this round's
      // disjoint rotations: entry block (p_i, q_i) x (p_j, q_j) of A depends
      // only on the same block, so every 2 x 2 block is updated in place by
      // one thread (columns by rotation j, then rows by rotation i); the
      // rotated entries (p, q), (q, p) are zero by construction of the angle
      const int nblkA = half * half;
      for (int e = threadIdx.x; e < nblkA + m * half; e += kJacobiThreads) {
        if (e < nblkA) {
          const int i = e / half, j = e % half;
          const int p = rp[i], q = rq[i], u = rp[j], v = rq[j];
          const double ci = rc[i], si = rs[i], cj = rc[j], sj = rs[j];
          const double a_pu = A[p * S + u], a_pv = A[p * S + v], a_qu = A[q * S + u], a_qv = A[q * S + v];
          const double b_pu = cj * a_pu - sj * a_pv, b_pv = sj * a_pu + cj * a_pv;
          const double b_qu = cj * a_qu - sj * a_qv, b_qv = sj * a_qu + cj * a_qv;
          const bool hit = i == j && si != 0.0;
          A[p * S + u] = ci * b_pu - si * b_qu;
          A[q * S + u] = hit ? 0.0 : si * b_pu + ci * b_qu;
          A[p * S + v] = hit ? 0.0 : ci * b_pv - si * b_qv;
          A[q * S + v] = si * b_pv + ci * b_qv;
        } else {
          const int f = e - nblkA, r = f / half, j = f % half;
          const int u = rp[j], v = rq[j];
          const double c = rc[j], sn = rs[j];
          const double x = Q[r * S + u], y = Q[r * S + v];
          Q[r * S + u] = c * x - sn * y;
          Q[r * S + v] = sn * x + c * y;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // decreasing eigenvalues over the n real indices (the pad index n, when n
  // is odd, keeps its zero eigenvalue and unit vector and is left out)
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 0; i < n; ++i) {
      int best = i;
      for (int j = i + 1; j < n; ++j)
        if (A[order[j] * S + order[j]] > A[order[best] * S + order[best]]) best = j;
      const int t = order[i];
      order[i] = order[best];
      order[best] = t;
    }
    const double s0 = sqrt(fmax(A[order[0] * S + order[0]], 0.0));
    int r = 0;
    for (int i = 0; i < n; ++i)
      if (sqrt(fmax(A[order[i] * S + order[i]], 0.0)) > tol * s0) ++r;
    *rank = r < 1 ? 1 : r;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += kJacobiThreads) {
    const int a = e / n, r = e % n;
    V[a * n + r] = Q[a * S + order[r]];
  }
  if (threadIdx.x < n) sigma[threadIdx.x] = sqrt(fmax(A[order[threadIdx.x] * S + order[threadIdx.x]], 0.0));
}

// U[d][r][q] = sum_a V[a][r] M[d][a][q] for r < R (V is n x n, its first R
// columns used), with the columns from `keep` on taken as zero: rows
// keep..R-1 of U are the zero padding of the kept rank up to the inner
// length the contractions run at.  One thread per pair with the moment
// column in registers.
template <int NMAX>
__global__ void __launch_bounds__(256)
compress_moments_kernel(const double* __restrict__ M, int n, int64_t npair, const double* __restrict__ V, int R,
                        int keep, double* __restrict__ U) {
  __shared__ __align__(16) double s_v[NMAX * NMAX];
  for (int e = threadIdx.x; e < n * R; e += 256) {
    const int a = e / R, r = e % R;
    s_v[a * NMAX + r] = r < keep ? V[a * n + r] : 0.0;
  }
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= npair) return;
  const int d = blockIdx.y;
  const double* Md = M + (int64_t)d * n * npair;
  double m[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) m[a] = a < n ? Md[(int64_t)a * npair + q] : 0.0;
  double* Ud = U + (int64_t)d * R * npair;
  int r = 0;
  for (; r + 1 < R; r += 2) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
      if (a < n) {
        const double2 v = *reinterpret_cast<const double2*>(&s_v[a * NMAX + r]);
        s0 += v.x * m[a];
        s1 += v.y * m[a];
      }
    Ud[(int64_t)r * npair + q] = s0;
    Ud[(int64_t)(r + 1) * npair + q] = s1;
  }
  if (r < R) {
    double s0 = 0.0;
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
      if (a < n) s0 += s_v[a * NMAX + r] * m[a];
    Ud[(int64_t)r * npair + q] = s0;
  }
}

// V = V1 V2 (n x n), one work group.
__global__ void __launch_bounds__(256)
basis_product_kernel(const double* __restrict__ V1, const double* __restrict__ V2, int n, double* __restrict__ V) {
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int a = e / n, r = e % n;
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += V1[a * n + b] * V2[b * n + r];
    V[e] = s;
  }
}

// Kc[k] = V_R^T K[k] V_R (R x R), one work group per node; the columns of V
// from `keep` on are taken as zero (zero rows and columns of Kc).
__global__ void __launch_bounds__(256)
compress_tables_kernel(const double* __restrict__ K, int n, const double* __restrict__ V, int R, int keep,
                       double* __restrict__ Kc) {
  constexpr int S = kMaxN + 1;
  __shared__ double s_k[kMaxN * S];
  __shared__ double s_v[kMaxN * S];
  __shared__ double s_t[kMaxN * S];
  const int k = blockIdx.x;
  const double* Kk = K + (int64_t)k * n * n;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int a = e / n, b = e % n;
    s_k[a * S + b] = Kk[e];
    s_v[a * S + b] = b < keep ? V[e] : 0.0;
  }
  __syncthreads();
  // T = K V_R  (n x R)
  for (int e = threadIdx.x; e < n * R; e += 256) {
    const int a = e / R, r = e % R;
    double s = 0.0;
    for (int b = 0; b < n; ++b) s += s_k[a * S + b] * s_v[b * S + r];
    s_t[a * S + r] = s;
  }
  __syncthreads();
  double* out = Kc + (int64_t)k * R * R;
  for (int e = threadIdx.x; e < R * R; e += 256) {
    const int r = e / R, u = e % R;
    double s = 0.0;
    for (int a = 0; a < n; ++a) s += s_v[a * S + r] * s_t[a * S + u];
    out[e] = s;
  }
}

}  // namespace

int compress_nchunk(int64_t npair) {
  const int64_t c = (npair + kGramPairs - 1) / kGramPairs;
  return (int)(c < 2048 ? c : 2048);
}

size_t compress_work_bytes(int n, int nq, int64_t npair) {
  const size_t nn = (size_t)n * n;
  return align256(8 * nn * compress_nchunk(npair)) + align256(8 * nn) * 4 + align256(8 * (size_t)n) +
         align256(8 * (size_t)nq * nn) + align256(sizeof(int32_t));
}

CompressWork carve_compress_work(void* base, int n, int nq, int64_t npair) {
  const size_t nn = (size_t)n * n;
  CompressWork w;
  w.nchunk = compress_nchunk(npair);
  char* p = static_cast<char*>(base);
  w.part = reinterpret_cast<double*>(p); p += align256(8 * nn * w.nchunk);
  w.G = reinterpret_cast<double*>(p); p += align256(8 * nn);
  w.V = reinterpret_cast<double*>(p); p += align256(8 * nn);
  w.V1 = reinterpret_cast<double*>(p); p += align256(8 * nn);
  w.V2 = reinterpret_cast<double*>(p); p += align256(8 * nn);
  w.sigma = reinterpret_cast<double*>(p); p += align256(8 * (size_t)n);
  w.Kc = reinterpret_cast<double*>(p); p += align256(8 * (size_t)nq * nn);
  w.rank = reinterpret_cast<int32_t*>(p);
  return w;
}

namespace {
void launch_moments_in(const double* M, int n, int64_t npair, const double* V, int R, int keep, double* U,
                       hipStream_t s) {
  const dim3 g(nblk(npair, 256), 3);
  if (n <= 16) hipLaunchKernelGGL(compress_moments_kernel<16>, g, dim3(256), 0, s, M, n, npair, V, R, keep, U);
  else if (n <= 32) hipLaunchKernelGGL(compress_moments_kernel<32>, g, dim3(256), 0, s, M, n, npair, V, R, keep, U);
  else if (n <= 48) hipLaunchKernelGGL(compress_moments_kernel<48>, g, dim3(256), 0, s, M, n, npair, V, R, keep, U);
  else hipLaunchKernelGGL(compress_moments_kernel<64>, g, dim3(256), 0, s, M, n, npair, V, R, keep, U);
}
void launch_gram_eig(const double* M, int n, int64_t npair, double tol, double rel, double floor_rel,
                     const CompressWork& w, double* V, hipStream_t s) {
  const int64_t chunk = (npair + w.nchunk - 1) / w.nchunk;
  const int nchunk = (int)((npair + chunk - 1) / chunk);
  hipLaunchKernelGGL(gram_kernel, dim3(nchunk), dim3(256), 0, s, M, n, npair, chunk, w.part);
  hipLaunchKernelGGL(gram_sum_kernel, dim3(nblk(n * n, 64)), dim3(256), 0, s, w.part, nchunk, n * n, w.G);
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kJacobiThreads), 0, s, w.G, n, tol, rel, floor_rel, w.sigma, V,
                     w.rank);
}
}  // namespace

hipError_t launch_compress_basis(const double* M, int n, int64_t npair, double tol, const CompressWork& w,
                                 double* Y, hipStream_t s) {
  // V1 from W W^T need only be close: the refinement pass corrects it, and
  // entries below 1e-14 of the trace are the Gram matrix's own rounding
  launch_gram_eig(M, n, npair, tol, 1e-10, 1e-14, w, w.V1, s);
  launch_moments_in(M, n, npair, w.V1, n, n, Y, s);   // Y = V1^T W
  // V2, sigma, rank from Y Y^T: a relative test only (its entries are
  // rounded relative to sigma_r sigma_s)
  launch_gram_eig(Y, n, npair, tol, 1e-13, 0.0, w, w.V2, s);
  hipLaunchKernelGGL(basis_product_kernel, dim3(1), dim3(256), 0, s, w.V1, w.V2, n, w.V);
  return hipGetLastError();
}

hipError_t launch_compress_operands(const double* M, int n, int64_t npair, int R, int keep, int nq,
                                    const double* K, const CompressWork& w, double* U, hipStream_t s) {
  launch_moments_in(M, n, npair, w.V, R, keep, U, s);
  hipLaunchKernelGGL(compress_tables_kernel, dim3(nq), dim3(256), 0, s, K, n, w.V, R, keep, w.Kc);
  return hipGetLastError();
}

}  // namespace tai
