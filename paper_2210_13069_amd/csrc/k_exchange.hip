// Long-range exchange matrix in the factorized form of appendix B:
//
//   X_{j mu}(a)  = sum_lambda q_j(lambda) prod_d m_{(mu lambda),d}(a_d)    (a in [n]^3)
//   Phi_{j mu}   = sum_k w_k (K_k (x) K_k (x) K_k) X_{j mu}
//   K(mu, nu)    = 2 (2/sqrt(pi)) sum_j < X_{j mu}, Phi_{j nu} >
//
// where (mu lambda) is the pair holding mu and lambda (mu lambda = lambda mu),
// so each X_{j mu} gathers the nb pairs of row mu of the pair list, not all of
// them.  All T = norb nb grid tensors are then taken through the mode products
// together, as matrix-core products batched over tensors:
//
//  * exch_x_kernel: per (a0 group, mu, j) one work group forms X_{j mu} for its
//    a0 values over the nb pairs (mu, lambda), staged in LDS 64 pairs at a
//    time (v_mfma_f64_16x16x4, or the FP32 form);
//  * exch_slab_kernel: per slab (t, a0) and node k, S = K_k X_t(a0) K_k^T (both
//    products on the FP64 matrix cores, the slab and K_k in LDS), written to an
//    intermediate T1[t][k][a0] that holds a bounded chunk of tensors;
//  * exch_mode0_kernel: Phi_t(i0, c) = sum_{k, a0} w_k K_k(i0, a0) T1[t][k][a0][c]
//    for c = (a1, a2): one FP64 product with inner length nq n per tensor;
//  * exch_dot_kernel: K = 2 (2/sqrt(pi)) X Phi^T over the flattened (j, a)
//    index, the 64 x 64 output tiles on and above the diagonal staged through
//    LDS, split along the inner index into partials that exch_dot_sum_kernel
//    adds in a fixed order (each entry and its mirror from the same tile).
//
// No atomics: every sum runs in a fixed order, so the result is deterministic.
#include "tai_internal.h"
#include "tai_device.h"

#include <algorithm>
#include <cstdint>
#include <cstdlib>

namespace tai {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr double kTwoOverSqrtPi = 1.1283791670955126;

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

struct XF64 {
  using T = double;
  using Acc = v4d;
  static constexpr bool kSplitSum = false;
  __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row_of(int kg, int r) { return kg + 4 * r; }
};
struct XF32 {
  using T = float;
  using Acc = v4f;
  static constexpr bool kSplitSum = true;
  __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row_of(int kg, int r) { return 4 * kg + r; }
};

constexpr int kXB = 64;  // pairs per LDS batch of the X kernel

// Column of pair (mu, lambda) in the moments: its index in the full pair
// list, or through inv (full index -> list position, -1 if not listed) for a
// screened list.  -1: the pair is not there.
__device__ inline int64_t pair_col(int nb, int mu, int lam, const int32_t* inv) {
  const int a = mu < lam ? mu : lam, b = mu < lam ? lam : mu;
  const int64_t p = pair_row_start(nb, a) + (b - a);
  return inv ? (int64_t)inv[p] : p;
}

// X_{j mu} for the a0 values of this work group: grid (ceil(n / (8 A0W)),
// nb, norb), 512 threads.  Wave w owns a0 = blockIdx.x 8 A0W + w A0W + {0..A0W-1}
// and all (a1, a2) in NT x NT tiles of 16 x 16.  Per batch of 64 values of
// lambda the rows c(a0, lambda) = q_j(lambda) m_{(mu lambda),0}(a0), m_1 and
// m_2 of the gathered pairs are staged in LDS (the next batch in flight in
// registers during the MFMAs).
template <class Op, int NT, int A0W>
__global__ void __launch_bounds__(512, 1)
exch_x_kernel(const double* __restrict__ M, int64_t npair, int n, int nb, const int32_t* __restrict__ inv,
              const double* __restrict__ Q, double* __restrict__ X) {
  constexpr int NP = 16 * NT;
  constexpr int A0G = 8 * A0W;
  constexpr int ROWS = A0G + 2 * NP;
  constexpr int PER = ROWS * kXB / 512;
  constexpr int CS = A0G + 1, MS = NP + 1;
  using T = typename Op::T;
  using Acc = typename Op::Acc;
  __shared__ T s_c2[2][kXB * CS];
  __shared__ T s_m12[2][kXB * MS];
  __shared__ T s_m22[2][kXB * MS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int a0base = blockIdx.x * A0G;
  const int mu = blockIdx.y, j = blockIdx.z;
  const double* qj = Q + (int64_t)j * nb;
  const double* M0 = M;
  const double* M1 = M + (int64_t)n * npair;
  const double* M2 = M + 2 * (int64_t)n * npair;

  T pre[PER];
  auto load = [&](int lb) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      const int row = e / kXB;
      const int lam = lb + (e % kXB);
      double v = 0.0;
      if (lam < nb) {
        const int64_t col = pair_col(nb, mu, lam, inv);
        if (col >= 0) {
          if (row < A0G) {
            const int a0 = a0base + row;
            if (a0 < n) v = qj[lam] * M0[(int64_t)a0 * npair + col];
          } else if (row < A0G + NP) {
            const int a = row - A0G;
            if (a < n) v = M1[(int64_t)a * npair + col];
          } else {
            const int a = row - A0G - NP;
            if (a < n) v = M2[(int64_t)a * npair + col];
          }
        }
      }
      pre[i] = (T)v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      const int row = e / kXB, qq = e % kXB;
      if (row < A0G) s_c2[buf][qq * CS + row] = pre[i];
      else if (row < A0G + NP) s_m12[buf][qq * MS + row - A0G] = pre[i];
      else s_m22[buf][qq * MS + row - A0G - NP] = pre[i];
    }
  };

  Acc acc[A0W][NT][NT];
  v4d tot[Op::kSplitSum ? A0W : 1][NT][NT];
#pragma unroll
  for (int a = 0; a < A0W; ++a)
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int jj = 0; jj < NT; ++jj) {
        acc[a][i][jj] = Acc{0, 0, 0, 0};
        if constexpr (Op::kSplitSum) tot[a][i][jj] = v4d{0.0, 0.0, 0.0, 0.0};
      }

  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int lb = 0; lb < nb; lb += kXB, buf ^= 1) {
    const bool more = lb + kXB < nb;
    if (more) load(lb + kXB);
    const T* s_c = s_c2[buf];
    const T* s_m1 = s_m12[buf];
    const T* s_m2 = s_m22[buf];
#pragma unroll 2
    for (int st = 0; st < kXB / 4; ++st) {
      const int kk = 4 * st + kg;
      T bm[NT], am[NT];
#pragma unroll
      for (int jj = 0; jj < NT; ++jj) bm[jj] = s_m2[kk * MS + 16 * jj + r16];
#pragma unroll
      for (int i = 0; i < NT; ++i) am[i] = s_m1[kk * MS + 16 * i + r16];
#pragma unroll
      for (int a = 0; a < A0W; ++a) {
        const T cq = s_c[kk * CS + wave * A0W + a];
#pragma unroll
        for (int i = 0; i < NT; ++i) {
          const T av = cq * am[i];
#pragma unroll
          for (int jj = 0; jj < NT; ++jj) acc[a][i][jj] = Op::mma(av, bm[jj], acc[a][i][jj]);
        }
      }
    }
    if constexpr (Op::kSplitSum) {
#pragma unroll
      for (int a = 0; a < A0W; ++a)
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int jj = 0; jj < NT; ++jj) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tot[a][i][jj][r] += (double)acc[a][i][jj][r];
            acc[a][i][jj] = Acc{0, 0, 0, 0};
          }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  const int64_t n2 = (int64_t)n * n;
  double* out = X + ((int64_t)j * nb + mu) * n2 * n;
#pragma unroll
  for (int a = 0; a < A0W; ++a) {
    const int a0 = a0base + wave * A0W + a;
    if (a0 >= n) continue;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int jj = 0; jj < NT; ++jj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a1 = 16 * i + Op::row_of(kg, r), a2 = 16 * jj + r16;
          double v;
          if constexpr (Op::kSplitSum) v = tot[a][i][jj][r];
          else v = acc[a][i][jj][r];
          if (a1 < n && a2 < n) out[a0 * n2 + a1 * n + a2] = v;
        }
  }
}

// Work-group barrier for LDS hand-offs only: waits for this wave's LDS
// operations, not for its global stores (a __syncthreads would drain the
// slab outputs already on their way to memory at every node).
__device__ inline void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One 16 x 16 FP64 tile product per wave and step on the matrix cores, the
// fragments of a wave's next tile read from LDS while the MFMAs of the
// current one run.  Wave w takes tiles w, w + 4, ...; frag(t, st, a, b)
// reads tile t's A and B fragments of inner step st, put(t, acc) stores its
// result.
template <int NK, int TILES, class Frag, class Put>
__device__ inline void tile_products(int wave, Frag&& frag, Put&& put) {
  constexpr int MAXIT = (TILES + 3) / 4;
  double fa[2][NK], fb[2][NK];
  if (wave < TILES) {
#pragma unroll
    for (int st = 0; st < NK; ++st) frag(wave, st, fa[0][st], fb[0][st]);
  }
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int tt = wave + 4 * it;
    if (tt + 4 < TILES) {
#pragma unroll
      for (int st = 0; st < NK; ++st) frag(tt + 4, st, fa[(it + 1) & 1][st], fb[(it + 1) & 1][st]);
    }
    if (tt < TILES) {
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < NK; ++st)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[it & 1][st], fb[it & 1][st], acc, 0, 0, 0);
      put(tt, acc);
    }
  }
}

// Slab products of a chunk of tensors: grid (ceil(Tc n / SB), KC), 256
// threads.  The work group takes SB slabs (t, a0) of consecutive index
// s = t n + a0, keeps them in LDS (zero padded to NP x NP) and for every node
// k of its share (grid y splits the nodes into KC equal runs, so that few
// tensors still fill the device) forms U = K_k X(a0) and S = U K_k^T on the
// FP64 matrix cores, K_k staged in LDS, writing S to T1[t][k][a0][a1 n + a2].
// The next node's K_k values are loaded into registers while the current
// node's products run.  Tensor t reads X[t % xmod] and the tables
// K + t kstride (kstride 0: one table set; with kstride > 0 a work group
// holds one slab, SB = 1).
template <int NT, int SB>
__global__ void __launch_bounds__(256)
exch_slab_kernel(const double* __restrict__ X, const double* __restrict__ K, int n, int nq, int64_t nslab,
                 double* __restrict__ T1, int64_t xmod, int64_t kstride) {
  constexpr int NP = 16 * NT, PS = NP + 1, NK = NP / 4;
  constexpr int TILES = SB * NT * NT;
  constexpr int XPER = (SB * NP * NP + 255) / 256, KPER = (NP * NP + 255) / 256;
  __shared__ double Xs[SB * NP * PS];   // [SB][NP][PS]
  __shared__ double Us[SB * NP * PS];   // [SB][NP][PS]
  __shared__ double Ks[NP * PS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * SB;
  const int64_t n2 = (int64_t)n * n;
  {
    double xr[XPER];
#pragma unroll
    for (int i = 0; i < XPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int sb = e / (NP * NP), rem = e - sb * NP * NP;
      const int a1 = rem / NP, a2 = rem - a1 * NP;
      const int64_t sl = s0 + sb;
      xr[i] = 0.0;
      if (e < SB * NP * NP && sl < nslab && a1 < n && a2 < n) {
        const int64_t t = sl / n, a0 = sl - t * n;
        xr[i] = X[((t % xmod) * n + a0) * n2 + a1 * n + a2];
      }
    }
#pragma unroll
    for (int i = 0; i < XPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int sb = e / (NP * NP), rem = e - sb * NP * NP;
      if (e < SB * NP * NP) Xs[(sb * NP + rem / NP) * PS + rem % NP] = xr[i];
    }
  }
  const double* Kt = K + (s0 / n) * kstride;
  // T1 offset of each slab's node 0 (the node adds k n^3), -1 past the end
  int64_t tbase[SB];
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
    const int64_t sl = s0 + sb, t = sl / n, a0 = sl - t * n;
    tbase[sb] = sl < nslab ? (t * nq * n + a0) * n2 : -1;
  }
  const int kper = (nq + (int)gridDim.y - 1) / (int)gridDim.y;
  const int k0 = (int)blockIdx.y * kper, k1 = min(nq, k0 + kper);
  double kr[KPER];
  auto load_k = [&](int k) {
    const double* Kk = Kt + (int64_t)k * n2;
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int a = e / NP, b = e - a * NP;
      kr[i] = (e < NP * NP && a < n && b < n) ? Kk[a * n + b] : 0.0;
    }
  };
  if (k0 < k1) load_k(k0);
  for (int k = k0; k < k1; ++k) {
    lds_barrier();  // the previous node's Ks and Us reads are done (and Xs written)
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < NP * NP) Ks[(e / NP) * PS + e % NP] = kr[i];
    }
    if (k + 1 < k1) load_k(k + 1);
    lds_barrier();
    // U_sb = K_k X_sb
    tile_products<NK, TILES>(
        wave,
        [&](int tt, int st, double& a, double& b) {
          const int sb = tt / (NT * NT), ij = tt - sb * NT * NT, i = ij / NT, jj = ij - i * NT;
          a = Ks[(16 * i + r16) * PS + 4 * st + kg];
          b = Xs[(sb * NP + 4 * st + kg) * PS + 16 * jj + r16];
        },
        [&](int tt, const v4d& acc) {
          const int sb = tt / (NT * NT), ij = tt - sb * NT * NT, i = ij / NT, jj = ij - i * NT;
          double* us = Us + sb * NP * PS;
#pragma unroll
          for (int r = 0; r < 4; ++r) us[(16 * i + kg + 4 * r) * PS + 16 * jj + r16] = acc[r];
        });
    lds_barrier();
    // S_sb = U_sb K_k^T, straight to T1
    tile_products<NK, TILES>(
        wave,
        [&](int tt, int st, double& a, double& b) {
          const int sb = tt / (NT * NT), ij = tt - sb * NT * NT, i = ij / NT, jj = ij - i * NT;
          a = Us[(sb * NP + 16 * i + r16) * PS + 4 * st + kg];
          b = Ks[(16 * jj + r16) * PS + 4 * st + kg];
        },
        [&](int tt, const v4d& acc) {
          const int sb = tt / (NT * NT), ij = tt - sb * NT * NT, i = ij / NT, jj = ij - i * NT;
          if (tbase[sb] < 0) return;
          double* out = T1 + tbase[sb] + (int64_t)k * n * n2;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a1 = 16 * i + kg + 4 * r, a2 = 16 * jj + r16;
            if (a1 < n && a2 < n) out[a1 * n + a2] = acc[r];
          }
        });
  }
}

// The slab products of exch_slab_kernel for 33 <= n <= 40 and one table set,
// two slabs per work group side by side: U = K_k [X(s0) X(s0 + 1)] is one
// n x 2n product and S = [U(s0); U(s0 + 1)] K_k^T one 2n x n product, so the
// 16-wide tiles pad only K_k's side (n to 48; 2n is at most 80 = 5 tiles)
// and the inner index runs to 40 instead of 48: 15 tiles per product on four
// waves instead of 9 per slab.  Grid (ceil(nslab / 2), KC), 256 threads; the
// node runs, the K_k prefetch and the output T1[t][k][a0][a1 n + a2] are
// those of exch_slab_kernel.
template <int NT, int CT, int NK>
__global__ void __launch_bounds__(256)
exch_slab2_kernel(const double* __restrict__ X, const double* __restrict__ K, int n, int nq, int64_t nslab,
                  double* __restrict__ T1, int64_t xmod) {
  constexpr int SB = 2;
  constexpr int XR = 4 * NK;                 // rows of Xs and Us: the inner index, zero from n on
  constexpr int XC = 16 * CT, XPS = XC + 1;  // packed columns sb n + a2, zero from SB n on
  constexpr int KR = 16 * NT, KC4 = 4 * NK, KPS = KC4 + 1;
  constexpr int TILES = NT * CT;
  constexpr int XPER = (XR * XC + 255) / 256, KPER = (KR * KC4 + 255) / 256;
  __shared__ double Xs[XR * XPS];
  __shared__ double Us[XR * XPS];
  __shared__ double Ks[KR * KPS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * SB;
  const int64_t n2 = (int64_t)n * n;
  // slab of a packed index x < 16 CT = 80 <= 3 n: two compares, no division
  auto slab_of = [n](int x) { return (x >= n ? 1 : 0) + (x >= 2 * n ? 1 : 0); };
  {
    double xr[XPER];
#pragma unroll
    for (int i = 0; i < XPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int a1 = e / XC, col = e - a1 * XC;
      const int sb = slab_of(col), a2 = col - sb * n;
      const int64_t sl = s0 + sb;
      xr[i] = 0.0;
      if (e < XR * XC && a1 < n && sb < SB && sl < nslab) {
        const int64_t t = sl / n, a0 = sl - t * n;
        xr[i] = X[((t % xmod) * n + a0) * n2 + a1 * n + a2];
      }
    }
#pragma unroll
    for (int i = 0; i < XPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < XR * XC) Xs[(e / XC) * XPS + e % XC] = xr[i];
    }
  }
  // T1 offset of each slab's node 0 (the node adds k n^3), -1 past the end
  int64_t tbase[SB];
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
    const int64_t sl = s0 + sb, t = sl / n, a0 = sl - t * n;
    tbase[sb] = sl < nslab ? (t * nq * n + a0) * n2 : -1;
  }
  const int kper = (nq + (int)gridDim.y - 1) / (int)gridDim.y;
  const int k0 = (int)blockIdx.y * kper, k1 = min(nq, k0 + kper);
  double kr[KPER];
  auto load_k = [&](int k) {
    const double* Kk = K + (int64_t)k * n2;
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int a = e / KC4, b = e - a * KC4;
      kr[i] = (e < KR * KC4 && a < n && b < n) ? Kk[a * n + b] : 0.0;
    }
  };
  if (k0 < k1) load_k(k0);
  for (int k = k0; k < k1; ++k) {
    lds_barrier();  // the previous node's Ks and Us reads are done (and Xs written)
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < KR * KC4) Ks[(e / KC4) * KPS + e % KC4] = kr[i];
    }
    if (k + 1 < k1) load_k(k + 1);
    lds_barrier();
    // U = K_k [X(s0) X(s0 + 1)]: tile (i, jj) of rows 16 i (i1) and packed
    // columns 16 jj; rows from XR on are K_k's zero padding and are dropped
    tile_products<NK, TILES>(
        wave,
        [&](int tt, int st, double& a, double& b) {
          const int i = tt / CT, jj = tt - i * CT;
          a = Ks[(16 * i + r16) * KPS + 4 * st + kg];
          b = Xs[(4 * st + kg) * XPS + 16 * jj + r16];
        },
        [&](int tt, const v4d& acc) {
          const int i = tt / CT, jj = tt - i * CT;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i1 = 16 * i + kg + 4 * r;
            if (i1 < XR) Us[i1 * XPS + 16 * jj + r16] = acc[r];
          }
        });
    lds_barrier();
    // S = [U(s0); U(s0 + 1)] K_k^T: tile (ri, jj) of packed rows 16 ri
    // (sb n + i1) and columns 16 jj (i2).  An inner index a2 >= n reads the
    // next slab's column of U, against a zero column of K_k.
    tile_products<NK, TILES>(
        wave,
        [&](int tt, int st, double& a, double& b) {
          const int ri = tt / NT, jj = tt - ri * NT;
          const int r = 16 * ri + r16, sb = slab_of(r), i1 = r - sb * n;
          a = sb < SB ? Us[i1 * XPS + sb * n + 4 * st + kg] : 0.0;
          b = Ks[(16 * jj + r16) * KPS + 4 * st + kg];
        },
        [&](int tt, const v4d& acc) {
          const int ri = tt / NT, jj = tt - ri * NT;
          const int i2 = 16 * jj + r16;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int r = 16 * ri + kg + 4 * rr, sb = slab_of(r), i1 = r - sb * n;
            const int64_t base = sb == 0 ? tbase[0] : sb == 1 ? tbase[1] : -1;
            if (base >= 0 && i2 < n) T1[base + (int64_t)k * n * n2 + i1 * n + i2] = acc[rr];
          }
        });
  }
}

// Phi_t(i0, c) = sum_k w_k sum_a K_k(i0, a) T1[t][k][a][c], c = (a1, a2): grid
// (ceil(n^2 / (64 CW)), Tc, G), 256 threads; wave w owns the CW tiles of 16
// columns from c0 + 16 CW w and all NT tiles of i0 (with CW = 2 each read of
// w_k K_k from LDS feeds two MFMAs and a wave has twice the T1 loads in
// flight).  Per node, w_k K_k is staged in
// LDS; the T1 fragments stream from memory once, and the next node's w_k K_k
// and T1 fragments are loaded into registers while the current node's MFMAs
// run.  Tensor t's tables start at K + t kstride.  With G > 1 the nodes are
// split into G equal runs and run g writes its partial sums to the g-th
// block of Tc tensors at Phi.  NK inner steps of 4 (NP / 4, or 10 for
// 33 <= n <= 40: the inner index stops at 40).
template <int NT, int NK = 4 * NT, int CW = 1>
__global__ void __launch_bounds__(256)
exch_mode0_kernel(const double* __restrict__ T1, const double* __restrict__ K, const double* __restrict__ w, int n,
                  int nq, double* __restrict__ Phi, int64_t kstride) {
  constexpr int NP = 16 * NT, PS = NP + 1;
  constexpr int KPER = (NP * NP + 255) / 256;
  __shared__ double Ws[NP * PS];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t n2 = (int64_t)n * n;
  const int64_t t = blockIdx.y;
  int64_t c[CW];
  bool cok[CW];
#pragma unroll
  for (int j = 0; j < CW; ++j) {
    c[j] = (int64_t)blockIdx.x * (64 * CW) + 16 * (CW * wave + j) + r16;
    cok[j] = c[j] < n2;
  }
  const double* Tt = T1 + t * nq * n * n2;
  const double* Kt = K + t * kstride;
  const int kper = (nq + (int)gridDim.z - 1) / (int)gridDim.z;
  const int k0 = (int)blockIdx.z * kper, k1 = min(nq, k0 + kper);
  v4d acc[CW][NT];
#pragma unroll
  for (int j = 0; j < CW; ++j)
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[j][i] = v4d{0.0, 0.0, 0.0, 0.0};
  double kr[KPER], bv[2][CW][NK];
  auto load = [&](int k, double (&b)[CW][NK]) {
    const double wk = w[k];
    const double* Kk = Kt + (int64_t)k * n2;
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int a = e / NP, bb = e - a * NP;
      kr[i] = (e < NP * NP && a < n && bb < n) ? wk * Kk[a * n + bb] : 0.0;
    }
    const double* Tk = Tt + (int64_t)k * n * n2;
#pragma unroll
    for (int j = 0; j < CW; ++j)
#pragma unroll
      for (int st = 0; st < NK; ++st) {
        const int a = 4 * st + kg;
        b[j][st] = (cok[j] && a < n) ? Tk[a * n2 + c[j]] : 0.0;
      }
  };
  auto node = [&](int k, double (&cur)[CW][NK], double (&nxt)[CW][NK]) {
    lds_barrier();  // the previous node's Ws reads are done
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < NP * NP) Ws[(e / NP) * PS + e % NP] = kr[i];
    }
    if (k + 1 < k1) load(k + 1, nxt);
    lds_barrier();
#pragma unroll
    for (int st = 0; st < NK; ++st) {
      const int a = 4 * st + kg;
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const double av = Ws[(16 * i + r16) * PS + a];
#pragma unroll
        for (int j = 0; j < CW; ++j)
          acc[j][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cur[j][st], acc[j][i], 0, 0, 0);
      }
    }
  };
  if (k0 < k1) load(k0, bv[0]);
  for (int k = k0; k < k1; k += 2) {
    node(k, bv[0], bv[1]);
    if (k + 1 < k1) node(k + 1, bv[1], bv[0]);
  }
  double* out = Phi + ((int64_t)blockIdx.z * gridDim.y + t) * n * n2;
#pragma unroll
  for (int j = 0; j < CW; ++j) {
    if (!cok[j]) continue;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i0 = 16 * i + kg + 4 * r;
        if (i0 < n) out[i0 * n2 + c[j]] = acc[j][i][r];
      }
  }
}

// Partial exchange matrix over one slice of the inner index: grid
// (ceil(nb / 64), ceil(nb / 64), nsplit), 256 threads.  The inner index is
// f = (j, a) over norb n^3 values, split into nsplit equal slices; rows mu of
// X and nu of Phi are staged in LDS 32 inner values at a time (rows
// contiguous in memory).  Wave w owns the 32 x 32 quarter (w / 2, w % 2) of the
// 64 x 64 tile.  part[s][mu][nu] = sum over slice s of X(mu, f) Phi(nu, f),
// for the tiles on and above the diagonal only (K is symmetric; the sum
// kernel reads entry (min, max) for both orders, so K comes out exactly
// symmetric).
constexpr int kDK = 32;
__global__ void __launch_bounds__(256)
exch_dot_kernel(const double* __restrict__ X, const double* __restrict__ Phi, int nb, int norb, int64_t n3,
                int64_t slice, double* __restrict__ part) {
  constexpr int DS = kDK + 1;
  __shared__ double xs[64 * DS];
  __shared__ double ps[64 * DS];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  // K is symmetric: only the tiles on and above the diagonal are formed
  if (blockIdx.y < blockIdx.x) return;
  const int mu0 = blockIdx.x * 64, nu0 = blockIdx.y * 64;
  const int64_t total = (int64_t)norb * n3;
  const int64_t f0 = (int64_t)blockIdx.z * slice;
  const int64_t f1 = f0 + slice < total ? f0 + slice : total;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = v4d{0.0, 0.0, 0.0, 0.0};
  const int wi = wave >> 1, wj = wave & 1;
  // this thread stages column col of every batch, rows row0, row0 + 8, ...
  static_assert(256 % kDK == 0, "a thread's column is the same in every row step");
  const int col = threadIdx.x % kDK, row0 = threadIdx.x / kDK;
  for (int64_t fb = f0; fb < f1; fb += kDK) {
    __syncthreads();
    const int64_t f = fb + col;
    const bool fin = f < f1;
    const int64_t fc = fin ? f : f0;              // past the slice: no load
    const int64_t j = fc / n3, a = fc - j * n3;   // once per batch, not per row
    const double* xcol = X + (j * nb + mu0) * n3 + a;
    const double* pcol = Phi + (j * nb + nu0) * n3 + a;
    for (int row = row0; row < 64; row += 256 / kDK) {
      double xv = 0.0, pv = 0.0;
      if (fin) {
        if (mu0 + row < nb) xv = xcol[row * n3];
        if (nu0 + row < nb) pv = pcol[row * n3];
      }
      xs[row * DS + col] = xv;
      ps[row * DS + col] = pv;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kDK / 4; ++st) {
      const int kk = 4 * st + kg;
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = xs[(32 * wi + 16 * i + r16) * DS + kk];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) bv[jj] = ps[(32 * wj + 16 * jj + r16) * DS + kk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[jj], acc[i][jj], 0, 0, 0);
    }
  }
  double* out = part + (int64_t)blockIdx.z * nb * nb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = mu0 + 32 * wi + 16 * i + kg + 4 * r, nu = nu0 + 32 * wj + 16 * jj + r16;
        if (mu < nb && nu < nb) out[(int64_t)mu * nb + nu] = acc[i][jj][r];
      }
}

// out[i] = sum_g part[g][i], runs in order
__global__ void __launch_bounds__(256)
sum_runs_kernel(const double* __restrict__ part, int nrun, int64_t len, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = 0.0;
  for (int g = 0; g < nrun; ++g) s += part[(int64_t)g * len + i];
  out[i] = s;
}

// K(mu, nu) = 2 (2/sqrt(pi)) sum_s part[s][mu][nu], slices in order.
__global__ void __launch_bounds__(256)
exch_dot_sum_kernel(const double* __restrict__ part, int nsplit, int nb, double* __restrict__ Kx) {
  const int64_t nn = (int64_t)nb * nb;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  // both (mu, nu) and (nu, mu) take the entry of the upper tiles
  const int64_t mu = i / nb, nu = i - mu * nb;
  const int64_t src = mu <= nu ? i : nu * nb + mu;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * nn + src];
  Kx[i] = 2.0 * kTwoOverSqrtPi * s;
}

// full pair index -> position in the listed pairs (-1 elsewhere)
__global__ void __launch_bounds__(256) fill_kernel(int32_t* __restrict__ x, int64_t count, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] = v;
}
__global__ void __launch_bounds__(256)
invert_pairs_kernel(const int32_t* __restrict__ pairs, int64_t npk, int64_t npair_full, int32_t* __restrict__ inv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npk) return;
  const int64_t p = pairs[i];
  if (p >= 0 && p < npair_full) inv[p] = (int32_t)i;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// SB slabs per work group: LDS (2 SB + 1) NP (NP + 1) doubles.  The
// launches take SB 4 at n <= 16, 2 at n <= 32 (41 KB: three work groups per
// compute unit) and 1 beyond (56 KB at n <= 48: two work groups, two waves
// per SIMD to hide each other's waits, 13% faster at Nb = 400 than one work
// group of two slabs; 100 KB at n <= 64).
// kc: node runs (grid y), 1 unless few tensors leave the device idle
template <int NT, int SB>
void launch_slab(const double* X, const double* K, int n, int nq, int64_t nslab, double* T1, hipStream_t s,
                 int64_t xmod = INT64_MAX, int64_t kstride = 0, int kc = 1) {
  hipLaunchKernelGGL((exch_slab_kernel<NT, SB>), dim3(nblk(nslab, SB), kc), dim3(256), 0, s, X, K, n, nq, nslab,
                     T1, xmod, kstride);
}

// two slabs per work group for 33 <= n <= 40 (NT 3), one table set
void launch_slab2(const double* X, const double* K, int n, int nq, int64_t nslab, double* T1, hipStream_t s,
                  int64_t xmod = INT64_MAX, int kc = 1) {
  hipLaunchKernelGGL((exch_slab2_kernel<3, 5, 10>), dim3(nblk(nslab, 2), kc), dim3(256), 0, s, X, K, n, nq, nslab,
                     T1, xmod);
}

// Work groups a launch of the mode products should hold at least: several
// per compute unit, so that the latency of the staged loads is hidden.
constexpr int64_t kModeGroups = 2048;

// node runs for `groups` work groups over `nq` nodes: enough runs to reach
// kModeGroups, at most one node per run
int node_runs(int64_t groups, int nq) {
  const int64_t r = (kModeGroups + groups - 1) / groups;
  return (int)std::max<int64_t>(1, std::min<int64_t>(r, nq));
}

}  // namespace

hipError_t launch_mode_products(const double* X, int64_t T, int64_t xmod, const double* K, int64_t kstride,
                                const double* w, int n, int nq, double* T1, int64_t T0, int64_t kstride0,
                                int nq0, double* Phi, double* part, int64_t part_len, hipStream_t s) {
  const int NT = (n + 15) / 16;
  const int64_t nslab = T * n, n2 = (int64_t)n * n;
  if (kstride != 0) {
    const int kc = node_runs(nslab, nq);
    if (NT == 1) launch_slab<1, 1>(X, K, n, nq, nslab, T1, s, xmod, kstride, kc);
    else if (NT == 2) launch_slab<2, 1>(X, K, n, nq, nslab, T1, s, xmod, kstride, kc);
    else if (NT == 3) launch_slab<3, 1>(X, K, n, nq, nslab, T1, s, xmod, kstride, kc);
    else launch_slab<4, 1>(X, K, n, nq, nslab, T1, s, xmod, kstride, kc);
  } else {
    if (NT == 1) launch_slab<1, 4>(X, K, n, nq, nslab, T1, s, xmod, 0, node_runs(nblk(nslab, 4), nq));
    else if (NT == 2) launch_slab<2, 2>(X, K, n, nq, nslab, T1, s, xmod, 0, node_runs(nblk(nslab, 2), nq));
    else if (NT == 3 && n <= 40) launch_slab2(X, K, n, nq, nslab, T1, s, xmod, node_runs(nblk(nslab, 2), nq));
    else if (NT == 3) launch_slab<3, 1>(X, K, n, nq, nslab, T1, s, xmod, 0, node_runs(nslab, nq));
    else launch_slab<4, 1>(X, K, n, nq, nslab, T1, s, xmod, 0, node_runs(nslab, nq));
  }
  // mode 0: with few output tensors the node sum is split into runs whose
  // partial tensors (in part, part_len doubles) are added in run order
  const int64_t len = T0 * n * n2;
  const int cw = (NT == 3 && n <= 40) ? 2 : 1;   // 16-column tiles per wave of the mode-0 pass
  int g = node_runs((int64_t)nblk(n2, 64 * cw) * T0, nq0);
  if (part == nullptr || part_len < 2 * len) g = 1;
  else g = (int)std::min<int64_t>(g, part_len / len);
  double* out = g > 1 ? part : Phi;
  const dim3 mg(nblk(n2, 64 * cw), (unsigned)T0, (unsigned)g);
  if (NT == 1) hipLaunchKernelGGL((exch_mode0_kernel<1>), mg, dim3(256), 0, s, T1, K, w, n, nq0, out, kstride0);
  else if (NT == 2) hipLaunchKernelGGL((exch_mode0_kernel<2>), mg, dim3(256), 0, s, T1, K, w, n, nq0, out, kstride0);
  else if (NT == 3 && n <= 40)
    hipLaunchKernelGGL((exch_mode0_kernel<3, 10, 2>), mg, dim3(256), 0, s, T1, K, w, n, nq0, out, kstride0);
  else if (NT == 3) hipLaunchKernelGGL((exch_mode0_kernel<3>), mg, dim3(256), 0, s, T1, K, w, n, nq0, out, kstride0);
  else hipLaunchKernelGGL((exch_mode0_kernel<4>), mg, dim3(256), 0, s, T1, K, w, n, nq0, out, kstride0);
  if (g > 1) hipLaunchKernelGGL(sum_runs_kernel, dim3(nblk(len, 256)), dim3(256), 0, s, part, g, len, Phi);
  return hipGetLastError();
}

ExchangeWork exchange_work_plan(int n, int nq, int nb, int norb, bool listed, int64_t npair_full) {
  ExchangeWork p{};
  const int64_t n3 = (int64_t)n * n * n;
  p.ntensor = (int64_t)norb * nb;
  const int64_t per = (int64_t)nq * n3 * 8;                  // T1 bytes per tensor
  p.tchunk = (int64_t)std::max<int64_t>(1, std::min<int64_t>(p.ntensor, (int64_t(4) << 30) / per));
  // TAI_EXCHANGE_CHUNK=<c> caps the tensors per chunk (tests of the chunked path)
  if (const char* env = std::getenv("TAI_EXCHANGE_CHUNK")) {
    const long long cap = std::atoll(env);
    if (cap > 0) p.tchunk = std::min<int64_t>(p.tchunk, cap);
  }
  const int64_t total = (int64_t)norb * n3;
  const int64_t tb64 = (nb + 63) / 64, tiles = tb64 * (tb64 + 1) / 2;   // tiles on and above the diagonal
  int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(1024, 2048 / tiles));
  const int64_t slice = ((total + nsplit - 1) / nsplit + kDK - 1) / kDK * kDK;
  p.nsplit = (int)((total + slice - 1) / slice);
  p.slice = slice;
  size_t b = 0;
  p.off_X = b; b += align256(8 * (size_t)p.ntensor * n3);
  p.off_Phi = b; b += align256(8 * (size_t)p.ntensor * n3);
  p.off_T1 = b; b += align256((size_t)per * p.tchunk);
  p.off_part = b; b += align256(8 * (size_t)p.nsplit * nb * nb);
  p.off_inv = b; b += listed ? align256(4 * (size_t)npair_full) : 0;
  p.bytes = b;
  return p;
}

hipError_t launch_exchange(int prec, const double* M, int nb, int64_t npair, const int32_t* pairs, int n, int nq,
                           const NodeTables& tb, const double* Q, int norb, void* work, const ExchangeWork& p,
                           double* Kx, hipStream_t s) {
  char* base = static_cast<char*>(work);
  double* X = reinterpret_cast<double*>(base + p.off_X);
  double* Phi = reinterpret_cast<double*>(base + p.off_Phi);
  double* T1 = reinterpret_cast<double*>(base + p.off_T1);
  double* part = reinterpret_cast<double*>(base + p.off_part);
  int32_t* inv = nullptr;
  if (pairs) {
    const int64_t full = (int64_t)nb * (nb + 1) / 2;
    inv = reinterpret_cast<int32_t*>(base + p.off_inv);
    hipLaunchKernelGGL(fill_kernel, dim3(nblk(full, 256)), dim3(256), 0, s, inv, full, -1);
    hipLaunchKernelGGL(invert_pairs_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, pairs, npair, full, inv);
  }
  // X_{j mu}: one work group per (a0 group, mu, j)
  const int NT = (n + 15) / 16;
  if (prec == kFP32) {
    const dim3 g((n + 7) / 8, nb, norb);
#define TAI_XK(nt) hipLaunchKernelGGL((exch_x_kernel<XF32, nt, 1>), g, dim3(512), 0, s, M, npair, n, nb, inv, Q, X)
    if (NT == 1) TAI_XK(1); else if (NT == 2) TAI_XK(2); else if (NT == 3) TAI_XK(3); else TAI_XK(4);
#undef TAI_XK
  } else if (n <= 48) {
    const dim3 g((n + 15) / 16, nb, norb);
#define TAI_XK(nt) hipLaunchKernelGGL((exch_x_kernel<XF64, nt, 2>), g, dim3(512), 0, s, M, npair, n, nb, inv, Q, X)
    if (NT == 1) TAI_XK(1); else if (NT == 2) TAI_XK(2); else TAI_XK(3);
#undef TAI_XK
  } else {
    const dim3 g((n + 7) / 8, nb, norb);
    hipLaunchKernelGGL((exch_x_kernel<XF64, 4, 1>), g, dim3(512), 0, s, M, npair, n, nb, inv, Q, X);
  }
  // Phi of every tensor, the slab products of a bounded chunk at a time
  const int64_t n3 = (int64_t)n * n * n, n2 = (int64_t)n * n;
  for (int64_t t0 = 0; t0 < p.ntensor; t0 += p.tchunk) {
    const int64_t tc = std::min<int64_t>(p.tchunk, p.ntensor - t0);
    const double* Xc = X + t0 * n3;
    const int64_t nslab = tc * n;
    if (NT == 1) launch_slab<1, 4>(Xc, tb.K, n, nq, nslab, T1, s);
    else if (NT == 2) launch_slab<2, 2>(Xc, tb.K, n, nq, nslab, T1, s);
    else if (NT == 3 && n <= 40) launch_slab2(Xc, tb.K, n, nq, nslab, T1, s);
    else if (NT == 3) launch_slab<3, 1>(Xc, tb.K, n, nq, nslab, T1, s);
    else launch_slab<4, 1>(Xc, tb.K, n, nq, nslab, T1, s);
    const dim3 mg(nblk(n2, NT == 3 && n <= 40 ? 128 : 64), (unsigned)tc);
    double* Pc = Phi + t0 * n3;
    if (NT == 1) hipLaunchKernelGGL((exch_mode0_kernel<1>), mg, dim3(256), 0, s, T1, tb.K, tb.w, n, nq, Pc, 0);
    else if (NT == 2) hipLaunchKernelGGL((exch_mode0_kernel<2>), mg, dim3(256), 0, s, T1, tb.K, tb.w, n, nq, Pc, 0);
    else if (NT == 3 && n <= 40)
      hipLaunchKernelGGL((exch_mode0_kernel<3, 10, 2>), mg, dim3(256), 0, s, T1, tb.K, tb.w, n, nq, Pc, 0);
    else if (NT == 3) hipLaunchKernelGGL((exch_mode0_kernel<3>), mg, dim3(256), 0, s, T1, tb.K, tb.w, n, nq, Pc, 0);
    else hipLaunchKernelGGL((exch_mode0_kernel<4>), mg, dim3(256), 0, s, T1, tb.K, tb.w, n, nq, Pc, 0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // K = 2 (2/sqrt(pi)) X Phi^T
  const dim3 dg(nblk(nb, 64), nblk(nb, 64), p.nsplit);
  hipLaunchKernelGGL(exch_dot_kernel, dg, dim3(256), 0, s, X, Phi, nb, norb, n3, p.slice, part);
  const int64_t nn = (int64_t)nb * nb;
  hipLaunchKernelGGL(exch_dot_sum_kernel, dim3(nblk(nn, 256)), dim3(256), 0, s, part, p.nsplit, nb, Kx);
  return hipGetLastError();
}

}  // namespace tai
