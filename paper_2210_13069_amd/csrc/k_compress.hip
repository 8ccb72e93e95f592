// Low-rank compression of the moments (section 6.1, eqs. SVD and
// approxepsilon), FP64.  The moment matrices of the three directions are
// stacked side by side, W = [M_1 | M_2 | M_3] (n x 3 npair); its leading left
// singular vectors V (n x R) give compressed moments U_d = V^T M_d and tables
// Kc_k = V^T K_k V, so every factor m_p^T K_k m_q of Theorem 3.1 becomes
// u_p^T Kc_k u_q with inner length R instead of n.
//
//  * Gram matrix G = W W^T = sum_d M_d M_d^T: chunks of pairs per work group,
//    partial G per chunk, the partials of each entry summed in a fixed order
//    by one work group per entry.
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
//  * One refinement pass: Y = V1^T W in the first basis V1 (formed batch by
//    batch inside the Gram kernel, never stored), then the Gram matrix of Y
//    (nearly diagonal, its entries (r, s) rounded relative to sigma_r
//    sigma_s rather than sigma_1^2) and its Jacobi eigenvectors V2;
//    the basis is V = V1 V2.  Forming W W^T alone resolves sigma_r only to
//    about 1e-16 sigma_1^2 / sigma_r; after the pass the values and the kept
//    subspace carry errors of about 1e-16 sigma_1 / sigma_r, as an SVD of W.
//  * U and Kc: plain FP64 products with V in LDS.
#include "tai_internal.h"

namespace tai {
namespace {

constexpr int kMaxN = 64;        // largest n the library accepts
constexpr int kGramPairs = 32;   // pairs per Gram chunk, at least
constexpr int kMaxSweeps = 40;

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Partial Gram matrix of the pairs [c*chunk, min((c+1)*chunk, npair)) of the
// three directions on the FP64 matrix cores: part[a][b][c] =
// sum_d sum_q M_d(a, q) M_d(b, q) (chunk index fastest, so that each entry's
// partials are contiguous for the sum).  The pairs are staged kGramKB at a
// time for the three directions (one batch ahead in registers), k = (d, pair)
// running over the 3 kGramKB values, in LDS as s_m[k][a].  Every wave keeps
// all the 16 x 16 tiles (I <= J) of G, independent MFMA chains, over its own
// quarter of each batch's k values; the four waves' tiles are added in a
// fixed order at the end, and each tile is written with its mirror.  The
// v_mfma_f64_16x16x4 operands of both sides come from s_m (lane l: row
// 16 I + l % 16, k0 + l / 16).
//
// With XF (the refinement pass) the Gram matrix is that of Y = V1^T W: each
// staged batch is first turned into its columns of Y in place, y_k =
// V1^T w_k, on the matrix cores (V1 in dynamic LDS, padded with zeros to
// whole 16 x 16 tiles); a wave takes whole groups of 16 k values, reads
// all their rows before it writes them, and one barrier separates the
// transform from the Gram products.  Y itself never reaches memory.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kGramKB = 32;               // pairs per staged batch and direction
constexpr int kGramK = 3 * kGramKB;       // k values per batch
constexpr int kGramKW = kGramK / 4;       // k values per wave and batch
constexpr int kGramPad = 65;              // LDS length of one k value's row (doubles; odd, so
                                          // the staging stores of 32 pairs hit distinct banks)
constexpr int kGramTiles = 10;            // tiles I <= J of G for n <= 64

template <bool XF>
__device__ __forceinline__ void gram_body(const double* __restrict__ M, const double* __restrict__ V1, int n,
                                          int64_t npair, int64_t chunk, int nchunk, double* __restrict__ part) {
  // the staged batch, and at the end the tiles of waves 1..3
  constexpr int kStage = kGramK * kGramPad, kSums = 3 * kGramTiles * 4 * 64;
  __shared__ double s_m[kStage > kSums ? kStage : kSums];
  extern __shared__ double s_v1[];   // XF: [16 T][16 T] V1 with zero padding
  const int64_t q0 = (int64_t)blockIdx.x * chunk;
  const int64_t q1 = q0 + chunk < npair ? q0 + chunk : npair;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int T = (n + 15) / 16, ntile = T * (T + 1) / 2, NP = 16 * T;
  int ti[kGramTiles], tj[kGramTiles];
  v4d acc[kGramTiles];
#pragma unroll
  for (int u = 0; u < kGramTiles; ++u) {
    acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
    int t = u, I = 0;
    while (I < T && t >= T - I) {   // row I holds the tiles (I, I .. T-1)
      t -= T - I;
      ++I;
    }
    ti[u] = I;
    tj[u] = I + t;
  }
  // rows n .. 16 T - 1 of every k stay zero (with XF the transform writes
  // zeros there too: the padded columns of V1 are zero)
  for (int e = threadIdx.x; e < kStage; e += 256) s_m[e] = 0.0;
  if (XF)
    for (int e = threadIdx.x; e < NP * NP; e += 256) {
      const int a = e / NP, r = e % NP;
      s_v1[e] = (a < n && r < n) ? V1[a * n + r] : 0.0;
    }
  // staging: thread t reads pair qb + t % 32 of rows t / 32 + 8 i of each
  // direction (256-byte runs of a moment row), one batch ahead in registers
  constexpr int kRowStep = 256 / kGramKB, kRowsPer = (kMaxN + kRowStep - 1) / kRowStep;
  const int j = threadIdx.x % kGramKB, a0 = threadIdx.x / kGramKB;
  double pre[3][kRowsPer];
  auto fetch = [&](int64_t qb) {
    const bool inb = qb + j < q1;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int i = 0; i < kRowsPer; ++i) {
        const int a = a0 + kRowStep * i;
        pre[d][i] = (inb && a < n) ? M[((int64_t)d * n + a) * npair + qb + j] : 0.0;
      }
  };
  fetch(q0);
  const double* base = s_m + (wave * kGramKW + (lane >> 4)) * kGramPad + (lane & 15);
  for (int64_t qb = q0; qb < q1; qb += kGramKB) {
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int i = 0; i < kRowsPer; ++i) {
        const int a = a0 + kRowStep * i;
        if (a < n) s_m[(d * kGramKB + j) * kGramPad + a] = pre[d][i];
      }
    __syncthreads();
    if (qb + kGramKB < q1) fetch(qb + kGramKB);
    if (XF) {
      // y_k(r) = sum_a V1(a, r) w_k(a) for the k groups kt = wave, wave + 4,
      // in steps of 4 values of a from ab: lane l holds the A operand
      // w_{16 kt + l % 16}(ab + l / 16) and the B operand V1(ab + l / 16,
      // 16 rt + l % 16) of column tile rt; the result tile (k, r) lands on
      // lane l as rows k = 16 kt + l / 16 + 4 x, column 16 rt + l % 16
      constexpr int kKT = kGramK / 16;
      for (int kt = wave; kt < kKT; kt += 4) {
        v4d y[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) y[rt] = v4d{0.0, 0.0, 0.0, 0.0};
        const double* arow = s_m + (16 * kt + (lane & 15)) * kGramPad + (lane >> 4);
        const double* brow = s_v1 + (lane >> 4) * NP + (lane & 15);
        for (int ab = 0; ab < NP; ab += 4) {
          const double av = arow[ab];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
            if (rt < T) y[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, brow[ab * NP + 16 * rt], y[rt], 0, 0, 0);
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
          if (rt < T)
#pragma unroll
            for (int x = 0; x < 4; ++x)
              s_m[(16 * kt + (lane >> 4) + 4 * x) * kGramPad + 16 * rt + (lane & 15)] = y[rt][x];
      }
      __syncthreads();
    }
#pragma unroll
    for (int k0 = 0; k0 < kGramKW; k0 += 4) {
#pragma unroll
      for (int u = 0; u < kGramTiles; ++u)
        if (u < ntile)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(base[k0 * kGramPad + 16 * ti[u]],
                                                        base[k0 * kGramPad + 16 * tj[u]], acc[u], 0, 0, 0);
    }
  }
  // the four waves' tiles, added in wave order by wave 0 through LDS
  __syncthreads();
  double* s_acc = s_m;   // [wave 1..3][tile][4][64]
  if (wave > 0) {
#pragma unroll
    for (int u = 0; u < kGramTiles; ++u)
      if (u < ntile)
#pragma unroll
        for (int r = 0; r < 4; ++r) s_acc[(((wave - 1) * kGramTiles + u) * 4 + r) * 64 + lane] = acc[u][r];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int u = 0; u < kGramTiles; ++u) {
    if (u >= ntile) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = acc[u][r];
#pragma unroll
      for (int w = 1; w < 4; ++w) v += s_acc[(((w - 1) * kGramTiles + u) * 4 + r) * 64 + lane];
      const int a = 16 * ti[u] + (lane >> 4) + 4 * r, b = 16 * tj[u] + (lane & 15);
      if (a < n && b < n) {
        part[((int64_t)a * n + b) * nchunk + blockIdx.x] = v;
        if (ti[u] != tj[u]) part[((int64_t)b * n + a) * nchunk + blockIdx.x] = v;
      }
    }
  }
}

// pass 0: the Gram matrix of W; pass 1 (dynamic LDS of gram_v1_bytes):
// that of Y = V1^T W
__global__ void __launch_bounds__(256)
gram_kernel(const double* __restrict__ M, int n, int64_t npair, int64_t chunk, double* __restrict__ part) {
  gram_body<false>(M, nullptr, n, npair, chunk, (int)gridDim.x, part);
}

__global__ void __launch_bounds__(256)
gram_y_kernel(const double* __restrict__ M, const double* __restrict__ V1, int n, int64_t npair, int64_t chunk,
              double* __restrict__ part) {
  gram_body<true>(M, V1, n, npair, chunk, (int)gridDim.x, part);
}

// batched: molecule blockIdx.y
__global__ void __launch_bounds__(256)
gram_batch_kernel(const CmpMol* __restrict__ tab, int n) {
  const CmpMol& m = tab[blockIdx.y];
  if ((int)blockIdx.x >= m.nchunk) return;
  gram_body<false>(m.M, nullptr, n, m.npair, m.chunk, m.nchunk, m.part);
}

__global__ void __launch_bounds__(256)
gram_y_batch_kernel(const CmpMol* __restrict__ tab, int n) {
  const CmpMol& m = tab[blockIdx.y];
  if ((int)blockIdx.x >= m.nchunk) return;
  gram_body<true>(m.M, m.V1, n, m.npair, m.chunk, m.nchunk, m.part);
}

inline size_t gram_v1_bytes(int n) {
  const size_t np = 16 * (size_t)((n + 15) / 16);
  return 8 * np * np;
}

// G[e] = sum over the chunks of part[e][c], one work group per entry: thread
// t sums the chunks t, t + 256, ... in order, then a fixed-order tree over
// the 256 thread sums.
constexpr int kGramSumThreads = 256;
__device__ __forceinline__ void gram_sum_body(const double* __restrict__ part, int nchunk, double* __restrict__ G) {
  __shared__ double s_sum[kGramSumThreads];
  const int e = blockIdx.x, t = threadIdx.x;
  const double* pe = part + (int64_t)e * nchunk;
  double s = 0.0;
  for (int c = t; c < nchunk; c += kGramSumThreads) s += pe[c];
  s_sum[t] = s;
  __syncthreads();
  for (int w = kGramSumThreads / 2; w > 0; w >>= 1) {
    if (t < w) s_sum[t] += s_sum[t + w];
    __syncthreads();
  }
  if (t == 0) G[e] = s_sum[0];
}

__global__ void __launch_bounds__(kGramSumThreads)
gram_sum_kernel(const double* __restrict__ part, int nchunk, double* __restrict__ G) {
  gram_sum_body(part, nchunk, G);
}

__global__ void __launch_bounds__(kGramSumThreads)
gram_sum_batch_kernel(const CmpMol* __restrict__ tab) {
  const CmpMol& m = tab[blockIdx.y];
  gram_sum_body(m.part, m.nchunk, m.G);
}

// Cyclic Jacobi on the symmetric n x n matrix G (n <= 64, padded to an even
// order m with a zero row and column, which no rotation touches).  Outputs
// sigma[r] = sqrt(max(lambda_r, 0)) in decreasing order, V[a][r] the matching
// unit eigenvectors, and *rank.
constexpr int kJacobiThreads = 1024;

// Off-diagonal entries at most rel * sqrt(|a_pp a_qq|), or at most
// floor_rel * trace(G), are left alone: below the floor an entry is rounding
// noise of the Gram matrix itself, and rotating on it would never settle.
__device__ __forceinline__ void jacobi_body(const double* __restrict__ G, int n, double tol, double rel, double floor_rel,
                                   double* __restrict__ sigma, double* __restrict__ V, int32_t* __restrict__ rank) {
  constexpr int S = kMaxN + 1;
  __shared__ double A[kMaxN * S];
  __shared__ double Q[kMaxN * S];
  __shared__ double2 rcs[kMaxN / 2];  // (c, s) of the rotations of a round
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
  // This thread's share of a round, the same in every round: at most
  // kAItems 2 x 2 blocks (ai, aj) of A (half^2 of them) and at most kQItems
  // (row, rotation) pairs of the eigenvector update (m half of them).
  constexpr int kAItems = ((kMaxN / 2) * (kMaxN / 2) + kJacobiThreads - 1) / kJacobiThreads;
  constexpr int kQItems = (kMaxN * (kMaxN / 2) + kJacobiThreads - 1) / kJacobiThreads;
  const int tid = threadIdx.x;
  int ai[kAItems], aj[kAItems];
#pragma unroll
  for (int k = 0; k < kAItems; ++k) {
    const int f = tid + k * kJacobiThreads;
    ai[k] = f < half * half ? f / half : -1;
    aj[k] = f < half * half ? f % half : 0;
  }
  int qr[kQItems], qj[kQItems];
#pragma unroll
  for (int k = 0; k < kQItems; ++k) {
    const int f = tid + k * kJacobiThreads;
    qr[k] = f < m * half ? f / half : -1;
    qj[k] = f < m * half ? f % half : 0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      // round-robin pairing: slot 0 fixed, the other m-1 slots rotate; the
      // pair (p_i, q_i), p_i < q_i, of rotation i is recomputed wherever used
      auto slot = [&](int k) {
        int x = k - 1 + round;
        x = x >= m - 1 ? x - (m - 1) : x;
        return k == 0 ? 0 : 1 + x;
      };
      auto pair_of = [&](int i, int& p, int& q) {
        const int a = slot(i), b = slot(m - 1 - i);
        p = a < b ? a : b;
        q = a < b ? b : a;
      };
      if (threadIdx.x < half) {
        const int i = threadIdx.x;
        int p, q;
        pair_of(i, p, q);
        const double app = A[p * S + p], aqq = A[q * S + q], apq = A[p * S + q];
        double c = 1.0, s = 0.0;
        // rotate unless apq is negligible against the diagonal pair (a
        // relative test, so tiny eigenvalues of a semi-definite G are still
        // resolved) or below the underflow range
        if (fabs(apq) > rel * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
          // the rotation that zeroes A'(p, q): tan = t, the root of smaller
          // size of t^2 + 2 theta t - 1 = 0, theta = x / y with
          // x = aqq - app, y = 2 apq, i.e. t = sgn(x) y / (|x| + sqrt(x^2 + y^2))
          const double x = aqq - app, y = 2.0 * apq;
          const double t = (x >= 0 ? y : -y) / (fabs(x) + sqrt(x * x + y * y));
          c = rsqrt(t * t + 1.0);
          s = t * c;
          rotated = 1;
        }
        rcs[i] = double2{c, s};
      }
      __syncthreads();
      // A <- J^T A J and V <- V J for the block-diagonal J of this round's
      // disjoint rotations: entry block (p_i, q_i) x (p_j, q_j) of A depends
      // only on the same block, so every 2 x 2 block is updated in place by
      // one thread (columns by rotation j, then rows by rotation i); the
      // rotated entries (p, q), (q, p) are zero by construction of the angle
      // (each thread's items are fixed for the kernel: see below)
#pragma unroll
      for (int k = 0; k < kAItems; ++k) {
        if (ai[k] < 0) continue;
        const int i = ai[k], j = aj[k];
        int p, q, u, v;
        pair_of(i, p, q);
        pair_of(j, u, v);
        const double2 ri = rcs[i], rj = rcs[j];
        const double ci = ri.x, si = ri.y, cj = rj.x, sj = rj.y;
        // two identity rotations (c = 1, s = 0) give back the block exactly:
        // in late sweeps most blocks are left as they are
        if (si == 0.0 && sj == 0.0) continue;
        const double a_pu = A[p * S + u], a_pv = A[p * S + v], a_qu = A[q * S + u], a_qv = A[q * S + v];
        const double b_pu = cj * a_pu - sj * a_pv, b_pv = sj * a_pu + cj * a_pv;
        const double b_qu = cj * a_qu - sj * a_qv, b_qv = sj * a_qu + cj * a_qv;
        const bool hit = i == j && si != 0.0;
        A[p * S + u] = ci * b_pu - si * b_qu;
        A[q * S + u] = hit ? 0.0 : si * b_pu + ci * b_qu;
        A[p * S + v] = hit ? 0.0 : ci * b_pv - si * b_qv;
        A[q * S + v] = si * b_pv + ci * b_qv;
      }
#pragma unroll
      for (int k = 0; k < kQItems; ++k) {
        if (qr[k] < 0) continue;
        const int r = qr[k];
        int u, v;
        pair_of(qj[k], u, v);
        const double2 rj = rcs[qj[k]];
        const double c = rj.x, sn = rj.y;
        if (sn == 0.0) continue;   // the identity rotation
        const double x = Q[r * S + u], y = Q[r * S + v];
        Q[r * S + u] = c * x - sn * y;
        Q[r * S + v] = sn * x + c * y;
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

__global__ void __launch_bounds__(kJacobiThreads)
jacobi_kernel(const double* __restrict__ G, int n, double tol, double rel, double floor_rel,
              double* __restrict__ sigma, double* __restrict__ V, int32_t* __restrict__ rank) {
  jacobi_body(G, n, tol, rel, floor_rel, sigma, V, rank);
}

// batched: molecule blockIdx.x; pass 0 writes V1, pass 1 V2 (and both the
// singular values and the rank, the second pass's final)
__global__ void __launch_bounds__(kJacobiThreads)
jacobi_batch_kernel(const CmpMol* __restrict__ tab, int n, int pass, double rel, double floor_rel) {
  const CmpMol& m = tab[blockIdx.x];
  jacobi_body(m.G, n, m.tol, rel, floor_rel, m.sigma, pass == 0 ? m.V1 : m.V2, m.rank);
}

// U[d][r][q] = sum_a V[a][r] M[d][a][q] for r < R (V is n x n, its first R
// columns used), with the columns from `keep` on taken as zero: rows
// keep..R-1 of U are the zero padding of the kept rank up to the inner
// length the contractions run at.  One thread per pair with the moment
// column in registers.
template <int NMAX>
__device__ __forceinline__ void compress_moments_body(const double* __restrict__ M, int n, int64_t npair,
                                             const double* __restrict__ V, int R, int keep, double* __restrict__ U) {
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

template <int NMAX>
__global__ void __launch_bounds__(256)
compress_moments_kernel(const double* __restrict__ M, int n, int64_t npair, const double* __restrict__ V, int R,
                        int keep, double* __restrict__ U) {
  compress_moments_body<NMAX>(M, n, npair, V, R, keep, U);
}

// batched, molecule blockIdx.z: U = V^T M at length n with the columns of V
// from the molecule's rank on taken as zero
template <int NMAX>
__global__ void __launch_bounds__(256)
compress_moments_batch_kernel(const CmpMol* __restrict__ tab, int n) {
  const CmpMol& m = tab[blockIdx.z];
  if ((int64_t)blockIdx.x * 256 >= m.npair) return;
  compress_moments_body<NMAX>(m.M, n, m.npair, m.V, n, *m.rank, m.U);
}

// V = V1 V2 (n x n): one work group per row a, one thread per column r.
__device__ __forceinline__ void basis_product_body(const double* __restrict__ V1, const double* __restrict__ V2, int n,
                                          double* __restrict__ V) {
  const int a = blockIdx.x, r = threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (int b = 0; b < n; ++b) s += V1[a * n + b] * V2[b * n + r];
  V[a * n + r] = s;
}

__global__ void __launch_bounds__(64)
basis_product_kernel(const double* __restrict__ V1, const double* __restrict__ V2, int n, double* __restrict__ V) {
  basis_product_body(V1, V2, n, V);
}

__global__ void __launch_bounds__(64)
basis_product_batch_kernel(const CmpMol* __restrict__ tab, int n) {
  const CmpMol& m = tab[blockIdx.y];
  basis_product_body(m.V1, m.V2, n, m.V);
}

// Kc[k] = V_R^T K[k] V_R (R x R), one work group per node; the columns of V
// from `keep` on are taken as zero (zero rows and columns of Kc).
__device__ __forceinline__ void compress_tables_body(const double* __restrict__ K, int n, const double* __restrict__ V, int R,
                                            int keep, double* __restrict__ Kc) {
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

__global__ void __launch_bounds__(256)
compress_tables_kernel(const double* __restrict__ K, int n, const double* __restrict__ V, int R, int keep,
                       double* __restrict__ Kc) {
  compress_tables_body(K, n, V, R, keep, Kc);
}

// batched, molecule blockIdx.y: tables at length n with the columns of V from
// the rank on taken as zero, and the molecule's per-node inner length (its
// rank) for the assembly kernels that skip the zero inner steps
__global__ void __launch_bounds__(256)
compress_tables_batch_kernel(const CmpMol* __restrict__ tab, int n, int nq) {
  const CmpMol& m = tab[blockIdx.y];
  const int keep = *m.rank;
  compress_tables_body(m.K, n, m.V, n, keep, m.Kc);
  if (blockIdx.x == 0 && m.nk)
    for (int k = threadIdx.x; k < nq; k += 256) m.nk[k] = keep;
}

}  // namespace

// Gram chunks: at most 512 (two work groups per compute unit), so that the
// transposed partials stay small.
int compress_nchunk(int64_t npair) {
  const int64_t c = (npair + kGramPairs - 1) / kGramPairs;
  return (int)(c < 512 ? c : 512);
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
// eigenpairs of the Gram matrix of W (V1 null) or of Y = V1^T W
void launch_gram_eig(const double* M, const double* V1, int n, int64_t npair, double tol, double rel,
                     double floor_rel, const CompressWork& w, double* V, hipStream_t s) {
  const int64_t chunk = (npair + w.nchunk - 1) / w.nchunk;
  const int nchunk = (int)((npair + chunk - 1) / chunk);
  if (V1)
    hipLaunchKernelGGL(gram_y_kernel, dim3(nchunk), dim3(256), gram_v1_bytes(n), s, M, V1, n, npair, chunk, w.part);
  else
    hipLaunchKernelGGL(gram_kernel, dim3(nchunk), dim3(256), 0, s, M, n, npair, chunk, w.part);
  hipLaunchKernelGGL(gram_sum_kernel, dim3(n * n), dim3(kGramSumThreads), 0, s, w.part, nchunk, w.G);
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(kJacobiThreads), 0, s, w.G, n, tol, rel, floor_rel, w.sigma, V,
                     w.rank);
}
}  // namespace

hipError_t launch_compress_basis(const double* M, int n, int64_t npair, double tol, const CompressWork& w,
                                 hipStream_t s) {
  // V1 from W W^T need only be close: the refinement pass corrects it, and
  // entries below 1e-14 of the trace are the Gram matrix's own rounding
  launch_gram_eig(M, nullptr, n, npair, tol, 1e-10, 1e-14, w, w.V1, s);
  // V2, sigma, rank from Y Y^T, Y = V1^T W formed inside the Gram kernel: a
  // relative test (its entries are rounded relative to sigma_r sigma_s), and
  // a floor of 1e-28 of the trace, i.e. (1e-14 sigma_1)^2: rotating entries
  // below it moves no singular value above 1e-14 sigma_1 and only lengthens
  // the sweeps over the noise block
  launch_gram_eig(M, w.V1, n, npair, tol, 1e-13, 1e-28, w, w.V2, s);
  hipLaunchKernelGGL(basis_product_kernel, dim3(n), dim3(64), 0, s, w.V1, w.V2, n, w.V);
  return hipGetLastError();
}

size_t cmp_mol_bytes(int n, int nq, int64_t npair) {
  const size_t nn = (size_t)n * n;
  return align256(8 * nn * compress_nchunk(npair)) + align256(8 * nn) * 4 + align256(8 * (size_t)n) +
         align256(sizeof(int32_t)) + align256(8 * 3 * (size_t)n * npair) + align256(8 * (size_t)nq * nn);
}

CmpMol carve_cmp_mol(void* base, int n, int nq, int64_t npair, const double* M, double tol, const double* K,
                     int32_t* nk) {
  const size_t nn = (size_t)n * n;
  CmpMol m;
  m.M = M;
  m.npair = npair;
  const int64_t c0 = compress_nchunk(npair);
  m.chunk = (npair + c0 - 1) / c0;
  m.nchunk = (int32_t)((npair + m.chunk - 1) / m.chunk);
  m.tol = tol;
  char* p = static_cast<char*>(base);
  m.part = reinterpret_cast<double*>(p); p += align256(8 * nn * c0);
  m.G = reinterpret_cast<double*>(p); p += align256(8 * nn);
  m.V1 = reinterpret_cast<double*>(p); p += align256(8 * nn);
  m.V2 = reinterpret_cast<double*>(p); p += align256(8 * nn);
  m.V = reinterpret_cast<double*>(p); p += align256(8 * nn);
  m.sigma = reinterpret_cast<double*>(p); p += align256(8 * (size_t)n);
  m.rank = reinterpret_cast<int32_t*>(p); p += align256(sizeof(int32_t));
  m.U = reinterpret_cast<double*>(p); p += align256(8 * 3 * (size_t)n * npair);
  m.K = K;
  m.Kc = reinterpret_cast<double*>(p);
  m.nk = nk;
  return m;
}

hipError_t launch_compress_batch(const CmpMol* tab, int ncm, int n, int nq, int64_t max_npair, int max_nchunk,
                                 hipStream_t s) {
  const unsigned mb = nblk(max_npair, 256);
  auto moments_in = [&]() {
    const dim3 g(mb, 3, ncm);
    if (n <= 16) hipLaunchKernelGGL(compress_moments_batch_kernel<16>, g, dim3(256), 0, s, tab, n);
    else if (n <= 32) hipLaunchKernelGGL(compress_moments_batch_kernel<32>, g, dim3(256), 0, s, tab, n);
    else if (n <= 48) hipLaunchKernelGGL(compress_moments_batch_kernel<48>, g, dim3(256), 0, s, tab, n);
    else hipLaunchKernelGGL(compress_moments_batch_kernel<64>, g, dim3(256), 0, s, tab, n);
  };
  auto gram_eig = [&](int pass, double rel, double floor_rel) {
    if (pass == 0) hipLaunchKernelGGL(gram_batch_kernel, dim3(max_nchunk, ncm), dim3(256), 0, s, tab, n);
    else hipLaunchKernelGGL(gram_y_batch_kernel, dim3(max_nchunk, ncm), dim3(256), gram_v1_bytes(n), s, tab, n);
    hipLaunchKernelGGL(gram_sum_batch_kernel, dim3(n * n, ncm), dim3(kGramSumThreads), 0, s, tab);
    hipLaunchKernelGGL(jacobi_batch_kernel, dim3(ncm), dim3(kJacobiThreads), 0, s, tab, n, pass, rel, floor_rel);
  };
  // the two passes of launch_compress_basis, with its tolerances
  gram_eig(0, 1e-10, 1e-14);
  gram_eig(1, 1e-13, 1e-28);
  hipLaunchKernelGGL(basis_product_batch_kernel, dim3(n, ncm), dim3(64), 0, s, tab, n);
  moments_in();
  hipLaunchKernelGGL(compress_tables_batch_kernel, dim3(nq, ncm), dim3(256), 0, s, tab, n, nq);
  return hipGetLastError();
}

hipError_t launch_compress_operands(const double* M, int n, int64_t npair, int R, int keep, int nq,
                                    const double* K, const CompressWork& w, double* U, hipStream_t s) {
  launch_moments_in(M, n, npair, w.V, R, keep, U, s);
  hipLaunchKernelGGL(compress_tables_kernel, dim3(nq), dim3(256), 0, s, K, n, w.V, R, keep, w.Kc);
  return hipGetLastError();
}

}  // namespace tai
