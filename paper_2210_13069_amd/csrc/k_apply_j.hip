// Coulomb matrix through the n^3 Chebyshev grid tensor, B never formed
// (eq. coulapprox with the mode products of eq. ig1), FP64:
//
//   Dt_q       = D(k,l) (2 - delta_kl)                     q = (k,l), k <= l
//   rho(a)     = sum_q Dt_q m_{q,0}(a0) m_{q,1}(a1) m_{q,2}(a2)
//   Phi        = (2/sqrt(pi)) sum_k w_k  rho x_0 K_k x_1 K_k x_2 K_k
//   J_p        = sum_a m_{p,0}(a0) m_{p,1}(a1) m_{p,2}(a2) Phi(a)
//   J(mu,nu)   = J(nu,mu) = J_p,                           p = (mu,nu)
//
// Both pair contractions run on the FP64 matrix cores (v_mfma_f64_16x16x4):
//  * rho: for each a0, rho_a0 = (c_a0 o M_1) M_2^T with c_a0(q) = Dt_q m_{q,0}(a0),
//    an n x n product over the pairs.  A work group owns 8*A0W values of a0
//    and one chunk of pairs, stages the chunk's moments in LDS 64 pairs at a
//    time (loads for the next batch in flight during the MFMAs) and writes an
//    n^3 partial; the partials are summed in a fixed order, so the result does
//    not depend on scheduling.
//  * J_p: for a tile of 16 pairs, X(a0, a1, p) = sum_a2 Phi(a0, a1, a2) m_{p,2}(a2)
//    is an MFMA product with Phi staged in LDS one a0 slab at a time; the
//    output fragment is contracted at once with m_{p,1} (in registers) and
//    m_{p,0}, so X is never stored.
#include "tai_internal.h"
#include "tai_device.h"

namespace tai {
namespace {

constexpr double kTwoOverSqrtPi = 1.1283791670955126;

// Pair p of the moments is pair pairs[p] of the full list when a screened
// list is given (entries outside the full list contribute nothing).
__device__ inline bool pair_of(const int32_t* pairs, int nb, int64_t p, int& mu, int& nu) {
  int64_t g = p;
  if (pairs) {
    g = pairs[p];
    if (g < 0 || g >= (int64_t)nb * (nb + 1) / 2) return false;
  }
  decode_pair(nb, g, mu, nu);
  return true;
}

__global__ void __launch_bounds__(256)
density_pairs_kernel(const double* __restrict__ D, int nb, int64_t npair, const int32_t* __restrict__ pairs,
                     double* __restrict__ Dt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int mu, nu;
  Dt[p] = pair_of(pairs, nb, p, mu, nu) ? D[(int64_t)mu * nb + nu] * (mu == nu ? 1.0 : 2.0) : 0.0;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kKB = 64;          // pairs per LDS batch of the rho kernel
constexpr int kRhoGroups = 512;  // target work groups of the rho kernel

// The arithmetic of the two pair contractions: FP64, or FP32 with the
// products summed in FP32 within one LDS batch of pairs (rho) or one a1
// block (J_p) and in FP64 beyond.  Both use 16x16x4 MFMAs, whose operand
// fragments have the same lane layout; the output rows differ (row_of).
struct JF64 {
  using T = double;
  using Acc = v4d;
  static constexpr bool kSplitSum = false;
  __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row_of(int kg, int r) { return kg + 4 * r; }
};
struct JF32 {
  using T = float;
  using Acc = v4f;
  static constexpr bool kSplitSum = true;
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row_of(int kg, int r) { return 4 * kg + r; }
};

// grid (ceil(n / (8*A0W)), nchunk), 512 threads.  Wave w owns
// a0 = blockIdx.x*8*A0W + w*A0W + {0..A0W-1} and all (a1, a2) in NT x NT
// output tiles of 16 x 16 (n padded to 16*NT with zeros).
// MT: the element type the moments are read in (the FP32 form reads an FP32
// copy, half the bytes of the staging loads that bound it).
template <class Op, int NT, int A0W, class MT = double>
__global__ void __launch_bounds__(512, 1)
rho_mfma_kernel(const MT* __restrict__ M, const double* __restrict__ Dt, int n, int64_t npair,
                int64_t chunk, double* __restrict__ part) {
  constexpr int NP = 16 * NT;                  // padded extent of a1 and a2
  constexpr int A0G = 8 * A0W;                 // a0 per work group
  constexpr int ROWS = A0G + 2 * NP;           // staged rows: c (A0G), m1 (NP), m2 (NP)
  constexpr int PER = ROWS * kKB / 512;        // staged values per thread
  constexpr int CS = A0G + 1, MS = NP + 1;     // LDS row strides (doubles)
  using T = typename Op::T;
  using Acc = typename Op::Acc;
  // two LDS buffers: batch b is read from buffer b & 1 while batch b + 1 is
  // stored into the other after the MFMAs, one barrier per batch
  __shared__ T s_c2[2][kKB * CS];
  __shared__ T s_m12[2][kKB * MS];
  __shared__ T s_m22[2][kKB * MS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int a0base = blockIdx.x * A0G;
  const int64_t q0 = (int64_t)blockIdx.y * chunk;
  const int64_t q1 = (q0 + chunk < npair) ? q0 + chunk : npair;
  const MT* M0 = M;
  const MT* M1 = M + (int64_t)n * npair;
  const MT* M2 = M + 2 * (int64_t)n * npair;

  // staged value e = threadIdx.x + 512 i of a batch: row e / kKB, pair e % kKB
  T pre[PER];
  auto load = [&](int64_t qb) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      const int row = e / kKB;
      const int64_t q = qb + (e % kKB);
      double v = 0.0;
      if (q < q1) {
        if (row < A0G) {
          const int a0 = a0base + row;
          if (a0 < n) v = Dt[q] * (double)M0[(int64_t)a0 * npair + q];
        } else if (row < A0G + NP) {
          const int a = row - A0G;
          if (a < n) v = (double)M1[(int64_t)a * npair + q];
        } else {
          const int a = row - A0G - NP;
          if (a < n) v = (double)M2[(int64_t)a * npair + q];
        }
      }
      pre[i] = (T)v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      const int row = e / kKB, qq = e % kKB;
      if (row < A0G) s_c2[buf][qq * CS + row] = pre[i];
      else if (row < A0G + NP) s_m12[buf][qq * MS + row - A0G] = pre[i];
      else s_m22[buf][qq * MS + row - A0G - NP] = pre[i];
    }
  };

  Acc acc[A0W][NT][NT];
  v4d tot[Op::kSplitSum ? A0W : 1][NT][NT];  // FP64 sums of the FP32 batches
#pragma unroll
  for (int a = 0; a < A0W; ++a)
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        acc[a][i][j] = Acc{0, 0, 0, 0};
        if constexpr (Op::kSplitSum) tot[a][i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      }

  load(q0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t qb = q0; qb < q1; qb += kKB, buf ^= 1) {
    const bool more = qb + kKB < q1;
    if (more) load(qb + kKB);  // next batch in flight during the MFMAs
    const T* s_c = s_c2[buf];
    const T* s_m1 = s_m12[buf];
    const T* s_m2 = s_m22[buf];
#pragma unroll 2
    for (int st = 0; st < kKB / 4; ++st) {
      const int kk = 4 * st + kg;  // this lane's pair within the batch
      T bm[NT], am[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j) bm[j] = s_m2[kk * MS + 16 * j + r16];
#pragma unroll
      for (int i = 0; i < NT; ++i) am[i] = s_m1[kk * MS + 16 * i + r16];
#pragma unroll
      for (int a = 0; a < A0W; ++a) {
        const T cq = s_c[kk * CS + wave * A0W + a];
#pragma unroll
        for (int i = 0; i < NT; ++i) {
          const T av = cq * am[i];
#pragma unroll
          for (int j = 0; j < NT; ++j) acc[a][i][j] = Op::mma(av, bm[j], acc[a][i][j]);
        }
      }
    }
    if constexpr (Op::kSplitSum) {
#pragma unroll
      for (int a = 0; a < A0W; ++a)
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int j = 0; j < NT; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[a][i][j][r] += (double)acc[a][i][j][r];
            acc[a][i][j] = Acc{0, 0, 0, 0};
          }
    }
    // the other buffer was last read in the previous batch, which every wave
    // finished before the barrier that ended it
    if (more) store(buf ^ 1);
    __syncthreads();
  }

  // lane l holds column a2 = 16 j + l%16 and rows a1 = 16 i + row_of(l/16, r)
  const int64_t n2 = (int64_t)n * n;
#pragma unroll
  for (int a = 0; a < A0W; ++a) {
    const int a0 = a0base + wave * A0W + a;
    if (a0 >= n) continue;
    double* out = part + ((int64_t)blockIdx.y * n + a0) * n2;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a1 = 16 * i + Op::row_of(kg, r), a2 = 16 * j + r16;
          double v;
          if constexpr (Op::kSplitSum) v = tot[a][i][j][r];
          else v = acc[a][i][j][r];
          if (a1 < n && a2 < n) out[a1 * n + a2] = v;
        }
  }
}

__global__ void __launch_bounds__(256)
sum_parts_kernel(const double* __restrict__ part, int nchunk, int64_t len, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * len + i];
  out[i] = s;
}

// Phi = (2/sqrt(pi)) sum_k w_k rho x_0 K_k x_1 K_k x_2 K_k in two passes.
// Pass 1, one work group per (a0 slab, node k): S = K_k rho(a0, :, :) K_k^T,
// both products in LDS, written to T[k][a0][:][:].
template <int NMAX>
__global__ void __launch_bounds__(256)
slab_modes_kernel(const double* __restrict__ K, const double* __restrict__ rho, int n,
                  double* __restrict__ T) {
  constexpr int ST = NMAX + 1;
  __shared__ double s_k[NMAX * ST];
  __shared__ double s_r[NMAX * ST];
  __shared__ double s_u[NMAX * ST];
  const int a0 = blockIdx.x, k = blockIdx.y;
  const int64_t n2 = (int64_t)n * n;
  const double* Kk = K + (int64_t)k * n2;
  const double* R = rho + a0 * n2;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    s_k[i * ST + j] = Kk[e];
    s_r[i * ST + j] = R[e];
  }
  __syncthreads();
  // U(i1, b) = sum_a K(i1, a) rho(a, b)
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i1 = e / n, b = e % n;
    double u = 0.0;
    for (int a = 0; a < n; ++a) u += s_k[i1 * ST + a] * s_r[a * ST + b];
    s_u[i1 * ST + b] = u;
  }
  __syncthreads();
  // S(i1, i2) = sum_b U(i1, b) K(i2, b)
  double* out = T + ((int64_t)k * n + a0) * n2;
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i1 = e / n, i2 = e % n;
    double v = 0.0;
    for (int b = 0; b < n; ++b) v += s_u[i1 * ST + b] * s_k[i2 * ST + b];
    out[e] = v;
  }
}

// Pass 2: P[k](i0, c) = sum_a K_k(i0, a) T[k][a][c] for c = (i1, i2); one
// thread per (c, k) with all i0 in registers, K_k read at uniform addresses.
template <int NMAX>
__global__ void __launch_bounds__(256)
mode0_kernel(const double* __restrict__ K, const double* __restrict__ T, int n, double* __restrict__ P) {
  const int64_t n2 = (int64_t)n * n;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int k = blockIdx.y;
  const int64_t cc = c < n2 ? c : 0;
  const double* Kk = K + (int64_t)k * n2;
  const double* Tk = T + (int64_t)k * n * n2;
  double acc[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) acc[i] = 0.0;
  for (int a = 0; a < n; ++a) {
    const double t = Tk[a * n2 + cc];
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) acc[i] += Kk[i * n + a] * t;
  }
  if (c >= n2) return;
  double* out = P + (int64_t)k * n * n2;
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n) out[i * n2 + c] = acc[i];
}

// Phi = (2/sqrt(pi)) sum_k w_k P[k], summed in node order.
__global__ void __launch_bounds__(256)
phi_kernel(const double* __restrict__ P, const double* __restrict__ w, int nq, int64_t n3,
           double* __restrict__ Phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double s = 0.0;
  for (int k = 0; k < nq; ++k) s += w[k] * P[(int64_t)k * n3 + i];
  Phi[i] = kTwoOverSqrtPi * s;
}

// J_p for 256 pairs per work group of 512 threads: wave w owns the two
// 16-pair tiles at blockIdx.x*256 + 32 w.  Per a0 the slab Phi(a0, :, :) is
// staged in LDS (double-buffered, the next slab's loads in flight during the
// MFMAs); X = Phi(a0) m_2 comes out of the matrix cores one 16-row block of
// a1 at a time and is contracted at once with m_1 and m_0.
template <class Op, int NT>
__global__ void __launch_bounds__(512, 1)
jp_mfma_kernel(const double* __restrict__ M, const double* __restrict__ Phi, int n, int64_t npair,
               double* __restrict__ Jp) {
  constexpr int NP = 16 * NT, NK = NP / 4, PT = 2;
  constexpr int PS = NP + 1;                        // LDS row stride (doubles)
  constexpr int SLAB = NP * NP;                     // padded slab values
  constexpr int PER = (SLAB + 511) / 512;           // staged values per thread
  using T = typename Op::T;
  using Acc = typename Op::Acc;
  __shared__ T s_phi[2][NP * PS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const double* M0 = M;
  const double* M1 = M + (int64_t)n * npair;
  const double* M2 = M + 2 * (int64_t)n * npair;
  const int64_t n2 = (int64_t)n * n;

  int64_t pc[PT];
  bool pok[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int64_t p = (int64_t)blockIdx.x * 256 + wave * 32 + 16 * t + r16;
    pok[t] = p < npair;
    pc[t] = pok[t] ? p : 0;
  }
  // B fragments m_2(a2 = 4 s + l/16, p) and the weights m_1(a1, p) of this
  // lane's output rows a1 = 16 i + row_of(l/16, r)
  T bm[PT][NK];
  double w1[PT][NT][4];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
#pragma unroll
    for (int st = 0; st < NK; ++st) {
      const int a2 = 4 * st + kg;
      bm[t][st] = (T)((pok[t] && a2 < n) ? M2[(int64_t)a2 * npair + pc[t]] : 0.0);
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a1 = 16 * i + Op::row_of(kg, r);
        w1[t][i][r] = (pok[t] && a1 < n) ? M1[(int64_t)a1 * npair + pc[t]] : 0.0;
      }
  }

  double pre[PER];
  auto load = [&](int a0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      const int a1 = e / NP, a2 = e % NP;
      pre[i] = (e < SLAB && a1 < n && a2 < n) ? Phi[a0 * n2 + (int64_t)a1 * n + a2] : 0.0;
    }
  };
  auto store = [&](T* buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      if (e < SLAB) buf[(e / NP) * PS + (e % NP)] = (T)pre[i];
    }
  };

  double jacc[PT] = {};
  load(0);
  for (int a0 = 0; a0 < n; ++a0) {
    T* buf = s_phi[a0 & 1];
    store(buf);
    __syncthreads();  // slab a0 in LDS; every wave is past slab a0-2 in this buffer
    if (a0 + 1 < n) load(a0 + 1);
    double m0v[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) m0v[t] = pok[t] ? M0[(int64_t)a0 * npair + pc[t]] : 0.0;
    double y[PT] = {};
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      Acc X[PT];
#pragma unroll
      for (int t = 0; t < PT; ++t) X[t] = Acc{0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < NK; ++st) {
        const T av = buf[(16 * i + r16) * PS + 4 * st + kg];
#pragma unroll
        for (int t = 0; t < PT; ++t) X[t] = Op::mma(av, bm[t][st], X[t]);
      }
#pragma unroll
      for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) y[t] += w1[t][i][r] * (double)X[t][r];
    }
#pragma unroll
    for (int t = 0; t < PT; ++t) jacc[t] += m0v[t] * y[t];
  }
  // the four lanes l/16 = 0..3 of a column hold partial sums over a1
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    double v = jacc[t];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (kg == 0 && pok[t]) Jp[pc[t]] = v;
  }
}

__global__ void __launch_bounds__(256)
unpack_kernel(const double* __restrict__ Jp, int nb, int64_t npair, const int32_t* __restrict__ pairs,
              double* __restrict__ J) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int mu, nu;
  if (!pair_of(pairs, nb, p, mu, nu)) return;
  J[(int64_t)mu * nb + nu] = Jp[p];
  J[(int64_t)nu * nb + mu] = Jp[p];
}

// Pair density of one orbital, D = q q^T folded over the ordered pairs:
// Dt_p = q(mu) q(nu) (2 - delta_mu,nu).
__global__ void __launch_bounds__(256)
orbital_pairs_kernel(const double* __restrict__ q, int nb, int64_t npair, const int32_t* __restrict__ pairs,
                     double* __restrict__ Dt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int mu, nu;
  Dt[p] = pair_of(pairs, nb, p, mu, nu) ? q[mu] * q[nu] * (mu == nu ? 1.0 : 2.0) : 0.0;
}

// Exchange (appendix B): the pair weights of X_{j mu} = sum_lambda q_j(lambda)
// m_(mu lambda), over the pairs that hold mu: Dt_p = q(other index of p), and
// q(mu) for the pair (mu, mu).
__global__ void __launch_bounds__(256)
exchange_pairs_kernel(const double* __restrict__ q, int nb, int row, int64_t npair, const int32_t* __restrict__ pairs,
                      double* __restrict__ Dt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int mu, nu;
  double v = 0.0;
  if (pair_of(pairs, nb, p, mu, nu)) v = mu == row ? q[nu] : (nu == row ? q[mu] : 0.0);
  Dt[p] = v;
}

// K(mu, nu) = 2 sum_j sum_a X_{j mu}(a) Phi_{j nu}(a), one work group per
// (mu, nu), the orbitals and grid points in a fixed order, then a tree sum.
__global__ void __launch_bounds__(256)
exchange_dot_kernel(const double* __restrict__ R, const double* __restrict__ F, int64_t n3, int nb, int norb,
                    double* __restrict__ Kx) {
  __shared__ double red[256];
  const int mu = blockIdx.y, nu = blockIdx.x;
  double acc = 0.0;
  for (int j = 0; j < norb; ++j) {
    const double* r = R + ((int64_t)j * nb + mu) * n3;
    const double* f = F + ((int64_t)j * nb + nu) * n3;
    for (int64_t a = threadIdx.x; a < n3; a += 256) acc += r[a] * f[a];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) Kx[(int64_t)mu * nb + nu] = 2.0 * red[0];
}

// J_mo(i, j) = sum_a rho_i(a) Phi_j(a) over the n^3 grid, one work group per
// (i, j), a fixed-order tree sum.
__global__ void __launch_bounds__(256)
mo_dot_kernel(const double* __restrict__ R, const double* __restrict__ F, int64_t n3, int norb,
              double* __restrict__ Jmo) {
  __shared__ double red[256];
  const int i = blockIdx.y, j = blockIdx.x;
  const double* r = R + (int64_t)i * n3;
  const double* f = F + (int64_t)j * n3;
  double acc = 0.0;
  for (int64_t a = threadIdx.x; a < n3; a += 256) acc += r[a] * f[a];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) Jmo[(int64_t)i * norb + j] = red[0];
}

// J entries of the pairs that screening dropped are zero.
__global__ void __launch_bounds__(256) zero_kernel(double* __restrict__ x, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] = 0.0;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

namespace {
// a0 values per wave of the rho kernel: two where the accumulators allow
int rho_a0_per_wave(int prec, int n) { return (prec == kFP64 && n <= 48) ? 2 : 1; }
int rho_groups(int prec, int n) { return (n + 8 * rho_a0_per_wave(prec, n) - 1) / (8 * rho_a0_per_wave(prec, n)); }
}  // namespace

int j_nchunk(int prec, int n, int npair) {
  int c = kRhoGroups / rho_groups(prec, n);
  if (c < 1) c = 1;
  const int maxc = (npair + 4 * kKB - 1) / (4 * kKB);  // at least four batches per chunk
  if (c > maxc) c = maxc;
  return c < 1 ? 1 : c;
}

size_t j_work_bytes(int prec, int nq, int n, int npair) {
  const size_t n3 = (size_t)n * n * n;
  const int nc = j_nchunk(prec, n, npair);
  const size_t m32 = prec == kFP32 ? align256(4 * 3 * (size_t)n * npair) : 0;
  return align256(8 * (size_t)npair) * 2 + align256(8 * n3 * nc) + align256(8 * n3) * 2 + align256(8 * n3 * nq) * 2 +
         m32;
}

JWork carve_j_work(void* base, int prec, int nq, int n, int npair) {
  const size_t n3 = (size_t)n * n * n;
  JWork w;
  w.nchunk = j_nchunk(prec, n, npair);
  char* p = static_cast<char*>(base);
  w.Dt = reinterpret_cast<double*>(p); p += align256(8 * (size_t)npair);
  w.Jp = reinterpret_cast<double*>(p); p += align256(8 * (size_t)npair);
  w.rho_part = reinterpret_cast<double*>(p); p += align256(8 * n3 * w.nchunk);
  w.rho = reinterpret_cast<double*>(p); p += align256(8 * n3);
  w.Phi = reinterpret_cast<double*>(p); p += align256(8 * n3);
  w.T1 = reinterpret_cast<double*>(p); p += align256(8 * n3 * nq);
  w.T2 = reinterpret_cast<double*>(p); p += align256(8 * n3 * nq);
  w.M32 = prec == kFP32 ? reinterpret_cast<float*>(p) : nullptr;
  return w;
}

template <class Op, int A0W, class MT>
void launch_pair_contraction_rho(const MT* M, int n, int npair, const JWork& w, hipStream_t s) {
  const int64_t chunk = ((int64_t)npair + w.nchunk - 1) / w.nchunk;
  const dim3 rg((n + 8 * A0W - 1) / (8 * A0W), w.nchunk);
  if (n <= 16) hipLaunchKernelGGL((rho_mfma_kernel<Op, 1, A0W, MT>), rg, dim3(512), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  else if (n <= 32) hipLaunchKernelGGL((rho_mfma_kernel<Op, 2, A0W, MT>), rg, dim3(512), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  else if (n <= 48) hipLaunchKernelGGL((rho_mfma_kernel<Op, 3, A0W, MT>), rg, dim3(512), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  else hipLaunchKernelGGL((rho_mfma_kernel<Op, 4, 1, MT>), rg, dim3(512), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
}

__global__ void __launch_bounds__(256) to_fp32_kernel(const double* __restrict__ x, int64_t count, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = (float)x[i];
}

template <class Op>
void launch_pair_contraction_jp(const double* M, int n, int npair, const JWork& w, hipStream_t s) {
  const unsigned jb = nblk(npair, 256);
  if (n <= 16) hipLaunchKernelGGL((jp_mfma_kernel<Op, 1>), dim3(jb), dim3(512), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  else if (n <= 32) hipLaunchKernelGGL((jp_mfma_kernel<Op, 2>), dim3(jb), dim3(512), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  else if (n <= 48) hipLaunchKernelGGL((jp_mfma_kernel<Op, 3>), dim3(jb), dim3(512), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  else hipLaunchKernelGGL((jp_mfma_kernel<Op, 4>), dim3(jb), dim3(512), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
}

namespace {
// the FP32 pair contraction reads an FP32 copy of the moments (in w.M32),
// made once per call
void convert_moments(int prec, const double* M, int n, int npair, const JWork& w, hipStream_t s) {
  if (prec != kFP32) return;
  const int64_t count = 3 * (int64_t)n * npair;
  hipLaunchKernelGGL(to_fp32_kernel, dim3(nblk(count, 256)), dim3(256), 0, s, M, count, w.M32);
}

// rho from the pair densities in w.Dt, then Phi = (2/sqrt(pi)) sum_k w_k rho x_d K_k
// (into w.rho and w.Phi)
void launch_rho_phi(int prec, const double* M, int npair, int n, int nq, const NodeTables& tb, const JWork& w,
                    hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  if (prec == kFP32) launch_pair_contraction_rho<JF32, 1>(static_cast<const float*>(w.M32), n, npair, w, s);
  else if (n <= 48) launch_pair_contraction_rho<JF64, 2>(M, n, npair, w, s);
  else launch_pair_contraction_rho<JF64, 1>(M, n, npair, w, s);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, w.rho_part, w.nchunk, n3, w.rho);
  if (n <= 16) hipLaunchKernelGGL(slab_modes_kernel<16>, dim3(n, nq), dim3(256), 0, s, tb.K, w.rho, n, w.T1);
  else if (n <= 32) hipLaunchKernelGGL(slab_modes_kernel<32>, dim3(n, nq), dim3(256), 0, s, tb.K, w.rho, n, w.T1);
  else if (n <= 48) hipLaunchKernelGGL(slab_modes_kernel<48>, dim3(n, nq), dim3(256), 0, s, tb.K, w.rho, n, w.T1);
  else hipLaunchKernelGGL(slab_modes_kernel<64>, dim3(n, nq), dim3(256), 0, s, tb.K, w.rho, n, w.T1);
  const dim3 mg(nblk((int64_t)n * n, 256), nq);
  if (n <= 16) hipLaunchKernelGGL(mode0_kernel<16>, mg, dim3(256), 0, s, tb.K, w.T1, n, w.T2);
  else if (n <= 32) hipLaunchKernelGGL(mode0_kernel<32>, mg, dim3(256), 0, s, tb.K, w.T1, n, w.T2);
  else if (n <= 48) hipLaunchKernelGGL(mode0_kernel<48>, mg, dim3(256), 0, s, tb.K, w.T1, n, w.T2);
  else hipLaunchKernelGGL(mode0_kernel<64>, mg, dim3(256), 0, s, tb.K, w.T1, n, w.T2);
  hipLaunchKernelGGL(phi_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, w.T2, tb.w, nq, n3, w.Phi);
}
}  // namespace

hipError_t launch_apply_j(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                          const NodeTables& tb, const double* D, double* J, const JWork& w, hipStream_t s) {
  hipLaunchKernelGGL(density_pairs_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, D, nb, (int64_t)npair, pairs,
                     w.Dt);
  convert_moments(prec, M, n, npair, w, s);
  launch_rho_phi(prec, M, npair, n, nq, tb, w, s);
  if (prec == kFP32) launch_pair_contraction_jp<JF32>(M, n, npair, w, s);
  else launch_pair_contraction_jp<JF64>(M, n, npair, w, s);
  if (pairs) {
    const int64_t nn = (int64_t)nb * nb;
    hipLaunchKernelGGL(zero_kernel, dim3(nblk(nn, 256)), dim3(256), 0, s, J, nn);
  }
  hipLaunchKernelGGL(unpack_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, w.Jp, nb, (int64_t)npair, pairs, J);
  return hipGetLastError();
}

hipError_t launch_coulomb_mo(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                             const NodeTables& tb, const double* Q, int norb, double* R, double* F, double* Jmo,
                             const JWork& w, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  convert_moments(prec, M, n, npair, w, s);
  for (int i = 0; i < norb; ++i) {
    JWork wi = w;
    wi.rho = R + (int64_t)i * n3;
    wi.Phi = F + (int64_t)i * n3;
    hipLaunchKernelGGL(orbital_pairs_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, Q + (int64_t)i * nb, nb,
                       (int64_t)npair, pairs, wi.Dt);
    launch_rho_phi(prec, M, npair, n, nq, tb, wi, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(mo_dot_kernel, dim3(norb, norb), dim3(256), 0, s, R, F, n3, norb, Jmo);
  return hipGetLastError();
}

hipError_t launch_exchange(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                           const NodeTables& tb, const double* Q, int norb, double* R, double* F, double* Kx,
                           const JWork& w, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  convert_moments(prec, M, n, npair, w, s);
  for (int j = 0; j < norb; ++j)
    for (int mu = 0; mu < nb; ++mu) {
      JWork wi = w;
      const int64_t slot = (int64_t)j * nb + mu;
      wi.rho = R + slot * n3;
      wi.Phi = F + slot * n3;
      hipLaunchKernelGGL(exchange_pairs_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, Q + (int64_t)j * nb, nb, mu,
                         (int64_t)npair, pairs, wi.Dt);
      launch_rho_phi(prec, M, npair, n, nq, tb, wi, s);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  hipLaunchKernelGGL(exchange_dot_kernel, dim3(nb, nb), dim3(256), 0, s, R, F, n3, nb, norb, Kx);
  return hipGetLastError();
}

}  // namespace tai
