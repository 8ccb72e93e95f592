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

#include <type_traits>

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
template <class Op, int NT, int A0W, class MT>
__device__ __forceinline__ void rho_mfma_body(const MT* __restrict__ M, const double* __restrict__ Dt, int n,
                                              int64_t npair, int64_t chunk, double* __restrict__ part) {
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

template <class Op, int NT, int A0W, class MT = double>
__global__ void __launch_bounds__(512, 1)
rho_mfma_kernel(const MT* __restrict__ M, const double* __restrict__ Dt, int n, int64_t npair,
                int64_t chunk, double* __restrict__ part) {
  // batched densities (several orbitals in one launch): density z, its
  // partial grids after those of densities 0 .. z-1
  rho_mfma_body<Op, NT, A0W, MT>(M, Dt + (int64_t)blockIdx.z * npair, n, npair, chunk,
                                 part + (int64_t)blockIdx.z * gridDim.y * n * n * n);
}

// Pair lists cut into consecutive spans (the partitions of the adaptive
// boxes): span z holds pairs off[z] .. off[z+1] of the list, its moments the
// block M + 3 n off[z] (each span's own pair count as the stride); blk[z] is
// the first work group of span z in a launch that covers all spans.
struct Spans {
  int64_t off[kMaxParts + 1];
  int64_t blk[kMaxParts + 1];
};

// rho of every span in one launch: grid (ceil(n / (8*A0W)), nchunk, nspan),
// span z's pairs cut into nchunk chunks, its partial grids after those of
// spans 0 .. z-1.  An empty span writes zero partial grids.
template <class Op, int NT, int A0W, class MT>
__global__ void __launch_bounds__(512, 1)
rho_spans_kernel(const MT* __restrict__ M, const double* __restrict__ Dt, int n, Spans sp, double* __restrict__ part) {
  const int z = blockIdx.z;
  const int64_t cnt = sp.off[z + 1] - sp.off[z];
  const int64_t chunk = (cnt + gridDim.y - 1) / gridDim.y;
  rho_mfma_body<Op, NT, A0W, MT>(M + 3 * (int64_t)n * sp.off[z], Dt + sp.off[z], n, cnt, chunk,
                                 part + (int64_t)z * gridDim.y * n * n * n);
}

// ---------------------------------------------------------------------------
// Split-BF16 forms of the two pair contractions (TAI_BF16X3, TAI_BF16X6).
// Each FP32 operand value x is cut into S bfloat16 slices, s0 = bf16(x),
// s1 = bf16(x - s0), s2 = bf16(x - s0 - s1), and a product sums s_i t_j over
// i + j <= S - 1 on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation): S = 2 gives 3 products, S = 3 gives 6.  bfloat16 keeps
// FP32's exponent range, so no operand scaling is needed.  The moments are
// read from the FP32 copy, the grid sums and mode products stay FP64.
//
// Measured on the device, sums on these MFMAs lose more than an exactly
// rounded FP32 accumulation would: J on the Nb = 64 workload was about 4x
// less accurate than a host model with round-to-nearest accumulation, close
// to one with truncating accumulation.  Each accumulator therefore takes few
// MFMA additions: in rho the small cross products of a K-step are summed in
// a fresh accumulator and folded into the running sum with one VALU add
// (round-to-nearest), and in J_p the 32-wide K-chunks go round-robin into
// three accumulators that are added the same way.  The pair sums of rho
// cancel heavily, and even so the 6-product rho stayed several times less
// accurate than the FP32 one (1.3e-6 against 1.9e-7 relative 2-norm of J
// on a 300-function basis), so TAI_BF16X6 takes the FP32 rho and splits
// only the projection; TAI_BF16X3 runs both contractions split.
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int S>
__device__ inline void split8(const float (&x)[8], v8bf (&out)[S]) {
  float r[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = x[e];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const __bf16 h = (__bf16)r[e];
      out[s][e] = h;
      r[e] -= (float)h;
    }
}

__device__ inline v4f mma_bf16(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// slice pairs (A slice, B slice) summed by an S-slice product
template <int S> struct SlicePairs;
template <> struct SlicePairs<2> {
  static constexpr int kN = 3;
  static constexpr int a[3] = {0, 0, 1};
  static constexpr int b[3] = {0, 1, 0};
};
template <> struct SlicePairs<3> {
  static constexpr int kN = 6;
  static constexpr int a[6] = {0, 0, 1, 0, 1, 2};
  static constexpr int b[6] = {0, 1, 0, 2, 1, 0};
};

constexpr int kKB16 = 64;   // pairs per LDS batch of the split rho kernel (two K-steps of 32)

// rho partials in split BF16.  1D grid; block b runs on XCD b % 8 and takes
// a0 group g and pair chunk c with the ngroups groups of one chunk on one XCD
// one after another, so that the chunk's moments are read from that XCD's L2
// by all its groups.  Wave w owns a0 = 8 A0W g + A0W w + {0 .. A0W-1} and all (a1, a2)
// in NT x NT tiles of 16 x 16; per batch of 64 pairs the chunk's rows
// c(a0, q) = Dt_q m_{q,0}(a0) (FP32), m_1 (FP32) and the slices of m_2 are
// staged in LDS, K-contiguous per row.  The A operand c(a0, q) m_{q,1}(a1) is
// formed in FP32 per lane and split on the fly.  Products are summed in FP32
// within one batch and in FP64 across the batches of the chunk; the chunk
// partials are summed in FP64 in a fixed order.
template <int NT, int S, int A0W>
__global__ void __launch_bounds__(512, 1)
rho16_kernel(const float* __restrict__ M, const double* __restrict__ Dt, int n, int64_t npair, int64_t chunk,
             int nchunk, int ngroups, double* __restrict__ part) {
  constexpr int NP = 16 * NT;
  constexpr int A0G = 8 * A0W;
  constexpr int CST = kKB16 + 4;          // FP32 row stride of s_c, s_m1 (floats)
  constexpr int BST = kKB16 + 8;          // bf16 row stride of the m_2 slices
  constexpr int ROWS = A0G + 2 * NP;      // staged rows per batch
  constexpr int PER = ROWS * kKB16 / 512; // staged values per thread
  using SP = SlicePairs<S>;
  __shared__ __align__(16) float s_c[2][A0G * CST];
  __shared__ __align__(16) float s_m1[2][NP * CST];
  __shared__ __align__(16) __bf16 s_m2[2][S * NP * BST];
  const int b = blockIdx.x;
  const int xcd = b & 7, r8 = b >> 3;
  const int g = r8 % ngroups;
  const int c = (r8 / ngroups) * 8 + xcd;
  if (c >= nchunk) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int a0base = g * A0G;
  const int64_t q0 = (int64_t)c * chunk;
  const int64_t q1 = (q0 + chunk < npair) ? q0 + chunk : npair;
  const float* M0 = M;
  const float* M1 = M + (int64_t)n * npair;
  const float* M2 = M + 2 * (int64_t)n * npair;
  // staged value e = threadIdx.x + 512 i: row e / 64, pair e % 64 (the pair
  // column is threadIdx.x % 64 for every i)
  const int qq = threadIdx.x & 63;
  float pre[PER];
  auto load = [&](int64_t qb) {
    const int64_t q = qb + qq;
    const bool ok = q < q1;
    const float dt = ok ? (float)Dt[q] : 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int row = (threadIdx.x + 512 * i) >> 6;
      float v = 0.f;
      if (ok) {
        if (row < A0G) {
          const int a0 = a0base + row;
          if (a0 < n) v = dt * M0[(int64_t)a0 * npair + q];
        } else if (row < A0G + NP) {
          const int a = row - A0G;
          if (a < n) v = M1[(int64_t)a * npair + q];
        } else {
          const int a = row - A0G - NP;
          if (a < n) v = M2[(int64_t)a * npair + q];
        }
      }
      pre[i] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int row = (threadIdx.x + 512 * i) >> 6;
      if (row < A0G) s_c[buf][row * CST + qq] = pre[i];
      else if (row < A0G + NP) s_m1[buf][(row - A0G) * CST + qq] = pre[i];
      else {
        const int a = row - A0G - NP;
        float rr = pre[i];
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
          const __bf16 h = (__bf16)rr;
          s_m2[buf][(sl * NP + a) * BST + qq] = h;
          rr -= (float)h;
        }
      }
    }
  };

  v4f acc[A0W][NT][NT];
  v4d tot[A0W][NT][NT];
#pragma unroll
  for (int a = 0; a < A0W; ++a)
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        acc[a][i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        tot[a][i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      }

  load(q0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int64_t qb = q0; qb < q1; qb += kKB16, buf ^= 1) {
    const bool more = qb + kKB16 < q1;
    if (more) load(qb + kKB16);
#pragma unroll
    for (int ks = 0; ks < kKB16 / 32; ++ks) {
      const int k0 = 32 * ks + 8 * kg;   // this lane's 8 pairs of the K-step
      v8bf bm[NT][S];
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int sl = 0; sl < S; ++sl)
          bm[j][sl] = *reinterpret_cast<const v8bf*>(&s_m2[buf][(sl * NP + 16 * j + r16) * BST + k0]);
      float cv[A0W][8];
#pragma unroll
      for (int a = 0; a < A0W; ++a) {
        const float4* src = reinterpret_cast<const float4*>(&s_c[buf][(A0W * wave + a) * CST + k0]);
        const float4 u = src[0], v = src[1];
        cv[a][0] = u.x; cv[a][1] = u.y; cv[a][2] = u.z; cv[a][3] = u.w;
        cv[a][4] = v.x; cv[a][5] = v.y; cv[a][6] = v.z; cv[a][7] = v.w;
      }
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const float4* src = reinterpret_cast<const float4*>(&s_m1[buf][(16 * i + r16) * CST + k0]);
        const float4 u = src[0], v = src[1];
        const float m1v[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
        for (int a = 0; a < A0W; ++a) {
          float x[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = cv[a][e] * m1v[e];
          v8bf as[S];
          split8<S>(x, as);
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            // cross products of the slices in a fresh accumulator, the
            // leading product into the running sum, then one rounded add
            v4f lo = mma_bf16(as[SP::a[1]], bm[j][SP::b[1]], v4f{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int pp = 2; pp < SP::kN; ++pp) lo = mma_bf16(as[SP::a[pp]], bm[j][SP::b[pp]], lo);
            acc[a][i][j] = mma_bf16(as[0], bm[j][0], acc[a][i][j]);
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][i][j][r] += lo[r];
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < A0W; ++a)
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) tot[a][i][j][r] += (double)acc[a][i][j][r];
          acc[a][i][j] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    if (more) store(buf ^ 1);
    __syncthreads();
  }
  // lane l holds column a2 = 16 j + l%16 and rows a1 = 16 i + 4 (l/16) + r
  const int64_t n2 = (int64_t)n * n;
#pragma unroll
  for (int a = 0; a < A0W; ++a) {
    const int a0 = a0base + A0W * wave + a;
    if (a0 >= n) continue;
    double* out = part + ((int64_t)c * n + a0) * n2;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a1 = 16 * i + 4 * kg + r, a2 = 16 * j + r16;
          if (a1 < n && a2 < n) out[a1 * n + a2] = tot[a][i][j][r];
        }
  }
}

// Inner layout of the split J_p contraction: position pos = nseg a2 + s
// (segment-minor) holds slice a[s] of Phi(.., a2) on the A side and slice
// b[s] of m_2(a2) on the B side, zero padded to kc = 32 ceil(nseg n / 32).
// Eight consecutive positions (one lane's share of a 32-wide K-step) then
// touch at most three values of a2 for nseg = 6.
template <int S> struct JSeg;
template <> struct JSeg<2> {
  static constexpr int kSeg = 3;
  static constexpr int a[3] = {0, 0, 1};
  static constexpr int b[3] = {0, 1, 0};
};
template <> struct JSeg<3> {
  static constexpr int kSeg = 6;
  static constexpr int a[6] = {0, 0, 1, 0, 1, 2};
  static constexpr int b[6] = {0, 1, 0, 2, 1, 0};
};
__host__ __device__ inline int j16_kc(int S, int n) {
  const int nseg = S == 2 ? 3 : 6;
  return (nseg * n + 31) / 32 * 32;
}

// Phi split into its slices in the A layout: Ps[a0][a1][kc] (bf16).
template <int S>
__global__ void __launch_bounds__(256)
phi_split_kernel(const double* __restrict__ Phi, int n, int kc, __bf16* __restrict__ Ps) {
  const int64_t row = blockIdx.x;            // (a0, a1)
  const double* src = Phi + row * n;
  __bf16* dst = Ps + row * kc;
  constexpr int NS = JSeg<S>::kSeg;
  for (int pos = threadIdx.x; pos < kc; pos += 256) {
    const int a2 = pos / NS, seg = pos - a2 * NS;
    __bf16 v = (__bf16)0.f;
    if (a2 < n) {
      const int want = JSeg<S>::a[seg];
      double r = src[a2];
      for (int sl = 0; sl < want; ++sl) r -= (double)(float)(__bf16)(float)r;
      v = (__bf16)(float)r;
    }
    dst[pos] = v;
  }
}

// J_p in split BF16 for 256 pairs per work group of 512 threads (wave w owns
// the two 16-pair tiles at blockIdx.x*256 + 32 w).  Each lane holds the m_2
// slices of its pair in the B layout for the whole kernel; per a0 the slab
// Ps(a0, :, :) is staged in LDS (double-buffered) and X = Phi(a0) m_2 comes
// out of the matrix cores one 16-row block of a1 at a time, contracted at
// once with m_1 (FP32) and, per a0, with m_0 (FP64).
template <int NT, int S, int KC>
__global__ void __launch_bounds__(512, 1)
jp16_kernel(const float* __restrict__ M, const __bf16* __restrict__ Ps, int n, int64_t npair,
            double* __restrict__ Jp) {
  constexpr int PT = 2;
  constexpr int kc = 32 * KC;
  constexpr int RS = kc + 8;                       // LDS row stride (bf16)
  constexpr int Q16 = kc / 8;                      // 16-byte pieces per row
  __shared__ __align__(16) __bf16 s_p[2][NT * 16 * RS];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const float* M0 = M;
  const float* M1 = M + (int64_t)n * npair;
  const float* M2 = M + 2 * (int64_t)n * npair;
  const int64_t n2kc = (int64_t)n * kc;

  int64_t pc[PT];
  bool pok[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int64_t p = (int64_t)blockIdx.x * 256 + wave * 32 + 16 * t + r16;
    pok[t] = p < npair;
    pc[t] = pok[t] ? p : 0;
  }
  // B fragments: K positions 32 c + 8 kg + e of the B layout; the lane's
  // eight positions hold the slices of at most NA consecutive values of a2.
  // One code path per kg, so that every position maps to its (a2, slice) at
  // compile time.
  constexpr int NS = JSeg<S>::kSeg;
  constexpr int NA = (7 + NS - 1) / NS + 1;
  v8bf bm[PT][KC];
  auto build_b = [&](auto kgc) {
    constexpr int KG = decltype(kgc)::value;
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
      for (int cc = 0; cc < KC; ++cc) {
        const int pos0 = 32 * cc + 8 * KG;
        const int a2f = pos0 / NS;
        float sl[NA][S];
#pragma unroll
        for (int u = 0; u < NA; ++u) {
          const int a2 = a2f + u;
          float r = (pok[t] && a2 < n) ? M2[(int64_t)a2 * npair + pc[t]] : 0.f;
#pragma unroll
          for (int q = 0; q < S; ++q) {
            const __bf16 h = (__bf16)r;
            sl[u][q] = (float)h;
            r -= (float)h;
          }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int pos = pos0 + e;
          bm[t][cc][e] = (__bf16)sl[pos / NS - a2f][JSeg<S>::b[pos % NS]];
        }
      }
  };
  switch (kg) {
    case 0: build_b(std::integral_constant<int, 0>{}); break;
    case 1: build_b(std::integral_constant<int, 1>{}); break;
    case 2: build_b(std::integral_constant<int, 2>{}); break;
    default: build_b(std::integral_constant<int, 3>{}); break;
  }
  // m_1 at this lane's output rows a1 = 16 i + 4 kg + r
  float w1[PT][NT][4];
#pragma unroll
  for (int t = 0; t < PT; ++t)
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a1 = 16 * i + 4 * kg + r;
        w1[t][i][r] = (pok[t] && a1 < n) ? M1[(int64_t)a1 * npair + pc[t]] : 0.f;
      }

  // slab staging: rows a1 < 16 NT (zero beyond n), Q16 pieces of 16 bytes each
  constexpr int PIECES = NT * 16 * Q16;
  constexpr int PER = (PIECES + 511) / 512;
  uint4 pre[PER];
  auto load = [&](int a0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      const int a1 = e / Q16, q = e - a1 * Q16;
      uint4 v = uint4{0u, 0u, 0u, 0u};
      if (e < PIECES && a1 < n) v = reinterpret_cast<const uint4*>(Ps + a0 * n2kc + (int64_t)a1 * kc)[q];
      pre[i] = v;
    }
  };
  auto store = [&](__bf16* bufp) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + 512 * i;
      if (e < PIECES) {
        const int a1 = e / Q16, q = e - a1 * Q16;
        *reinterpret_cast<uint4*>(bufp + a1 * RS + 8 * q) = pre[i];
      }
    }
  };

  double jacc[PT] = {};
  load(0);
  for (int a0 = 0; a0 < n; ++a0) {
    __bf16* bufp = s_p[a0 & 1];
    store(bufp);
    __syncthreads();  // slab a0 in LDS; every wave is past slab a0-2 in this buffer
    if (a0 + 1 < n) load(a0 + 1);
    double y[PT] = {};
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      // the K-chunks go round-robin into NR accumulators (at most three
      // MFMA additions each), summed with rounded adds at the end
      constexpr int NR = KC < 3 ? KC : 3;
      v4f Xr[NR][PT];
#pragma unroll
      for (int u = 0; u < NR; ++u)
#pragma unroll
        for (int t = 0; t < PT; ++t) Xr[u][t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int cc = 0; cc < KC; ++cc) {
        const v8bf av = *reinterpret_cast<const v8bf*>(bufp + (16 * i + r16) * RS + 32 * cc + 8 * kg);
#pragma unroll
        for (int t = 0; t < PT; ++t) Xr[cc % NR][t] = mma_bf16(av, bm[t][cc], Xr[cc % NR][t]);
      }
      v4f X[PT];
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        X[t] = Xr[0][t];
#pragma unroll
        for (int u = 1; u < NR; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) X[t][r] += Xr[u][t][r];
      }
#pragma unroll
      for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) y[t] += (double)w1[t][i][r] * (double)X[t][r];
    }
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const double m0 = pok[t] ? (double)M0[(int64_t)a0 * npair + pc[t]] : 0.0;
      jacc[t] += m0 * y[t];
    }
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
sum_parts_kernel(const double* __restrict__ part, int nchunk, int64_t len, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  part += (int64_t)blockIdx.y * nchunk * len;   // batched: grid y
  out += (int64_t)blockIdx.y * len;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * len + i];
  out[i] = s;
}

// out[i] = scale w[i % nq] for i < nq reps: the quadrature weights, repeated
// for each source box of the adaptive J, with 2/sqrt(pi) folded in.
__global__ void __launch_bounds__(256)
repeat_weights_kernel(const double* __restrict__ w, int nq, int reps, double scale, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nq * reps) out[i] = scale * w[i % nq];
}

// J_p for 256 pairs per work group of 512 threads: wave w owns the two
// 16-pair tiles at blockIdx.x*256 + 32 w.  Per a0 the slab Phi(a0, :, :) is
// staged in LDS (double-buffered, the next slab's loads in flight during the
// MFMAs); X = Phi(a0) m_2 comes out of the matrix cores one 16-row block of
// a1 at a time and is contracted at once with m_1 and m_0.
template <class Op, int NT>
__device__ __forceinline__ void jp_mfma_body(const double* __restrict__ M, const double* __restrict__ Phi, int n,
                                             int64_t npair, double* __restrict__ Jp, int64_t blk) {
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
    const int64_t p = blk * 256 + wave * 32 + 16 * t + r16;
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

template <class Op, int NT>
__global__ void __launch_bounds__(512, 1)
jp_mfma_kernel(const double* __restrict__ M, const double* __restrict__ Phi, int n, int64_t npair,
               double* __restrict__ Jp) {
  jp_mfma_body<Op, NT>(M, Phi, n, npair, Jp, blockIdx.x);
}

// J_p of every span in one launch: work groups blk[z] .. blk[z+1] take the
// pairs of span z (256 each) against its own Phi (Phi + z n^3).
template <class Op, int NT>
__global__ void __launch_bounds__(512, 1)
jp_spans_kernel(const double* __restrict__ M, const double* __restrict__ Phi, int n, int nspan, Spans sp,
                double* __restrict__ Jp) {
  int z = 0;
  while (z + 1 < nspan && (int64_t)blockIdx.x >= sp.blk[z + 1]) ++z;
  const int64_t o = sp.off[z];
  jp_mfma_body<Op, NT>(M + 3 * (int64_t)n * o, Phi + (int64_t)z * n * n * n, n, sp.off[z + 1] - o, Jp + o,
                       (int64_t)blockIdx.x - sp.blk[z]);
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
  q += (int64_t)blockIdx.y * nb;   // orbital blockIdx.y
  Dt += (int64_t)blockIdx.y * npair;
  int mu, nu;
  Dt[p] = pair_of(pairs, nb, p, mu, nu) ? q[mu] * q[nu] * (mu == nu ? 1.0 : 2.0) : 0.0;
}

// J_mo(i, j) = sum_a rho_i(a) Phi_j(a) over the n^3 grid, one work group per
// (i, j), a fixed-order tree sum.
__global__ void __launch_bounds__(256)
mo_dot_kernel(const double* __restrict__ R, const double* __restrict__ F, int64_t n3, int norb, double scale,
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
  if (threadIdx.x == 0) Jmo[(int64_t)i * norb + j] = scale * red[0];
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

// the split-BF16 forms of J, TAI_BF16X3 (2 slices) and TAI_BF16X6 (3)
inline bool split_j(int prec) { return prec == kBF16X3 || prec == kBF16X6; }
inline int j_slices(int prec) { return prec == kBF16X6 ? 3 : 2; }

size_t j_work_bytes(int prec, int nq, int n, int npair) {
  const size_t n3 = (size_t)n * n * n;
  const int nc = j_nchunk(prec, n, npair);
  const size_t m32 = (prec == kFP32 || split_j(prec)) ? align256(4 * 3 * (size_t)n * npair) : 0;
  const size_t ps = split_j(prec) ? align256(2 * (size_t)n * n * j16_kc(j_slices(prec), n)) : 0;
  return align256(8 * (size_t)npair) * 2 + align256(8 * n3 * nc) + align256(8 * n3) * 2 + align256(8 * n3 * nq) * 2 +
         align256(8 * (size_t)nq) + m32 + ps;
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
  w.wsc = reinterpret_cast<double*>(p); p += align256(8 * (size_t)nq);
  w.M32 = (prec == kFP32 || split_j(prec)) ? reinterpret_cast<float*>(p) : nullptr;
  if (w.M32) p += align256(4 * 3 * (size_t)n * npair);
  w.Ps = split_j(prec) ? reinterpret_cast<void*>(p) : nullptr;
  return w;
}

template <class Op, int A0W, class MT>
void launch_pair_contraction_rho(const MT* M, int n, int npair, const JWork& w, hipStream_t s, int ndens = 1) {
  const int64_t chunk = ((int64_t)npair + w.nchunk - 1) / w.nchunk;
  const dim3 rg((n + 8 * A0W - 1) / (8 * A0W), w.nchunk, ndens);
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
template <int NT, int S>
void launch_rho16_t(const float* M, int n, int npair, const JWork& w, hipStream_t s) {
  constexpr int A0W = 1;   // one a0 per wave: FP32 and FP64 accumulators for 16 NT^2 outputs
  const int ng = (n + 8 * A0W - 1) / (8 * A0W);
  const int64_t chunk = ((int64_t)npair + w.nchunk - 1) / w.nchunk;
  const unsigned blocks = (unsigned)((w.nchunk + 7) / 8 * 8 * ng);
  hipLaunchKernelGGL((rho16_kernel<NT, S, A0W>), dim3(blocks), dim3(512), 0, s, M, w.Dt, n, (int64_t)npair, chunk,
                     w.nchunk, ng, w.rho_part);
}
template <int S>
void launch_rho16_s(const float* M, int n, int npair, const JWork& w, hipStream_t s) {
  if (n <= 16) launch_rho16_t<1, S>(M, n, npair, w, s);
  else if (n <= 32) launch_rho16_t<2, S>(M, n, npair, w, s);
  else if (n <= 48) launch_rho16_t<3, S>(M, n, npair, w, s);
  else launch_rho16_t<4, S>(M, n, npair, w, s);
}
// rho in split BF16 for TAI_BF16X3 only: TAI_BF16X6 takes the FP32 rho (the
// bf16 matrix cores' accumulation of the pair sums, which cancel heavily,
// left the 6-product rho several times less accurate than the FP32 one:
// 1.3e-6 against 1.9e-7 relative 2-norm of J on a 300-function basis)
void launch_rho16(int prec, const float* M, int n, int npair, const JWork& w, hipStream_t s) {
  (void)prec;
  launch_rho16_s<2>(M, n, npair, w, s);
}
inline bool rho_split(int prec) { return prec == kBF16X3; }

template <int NT, int S, int KC>
void launch_jp16_k(const float* M, const __bf16* Ps, int n, int npair, double* Jp, hipStream_t s) {
  hipLaunchKernelGGL((jp16_kernel<NT, S, KC>), dim3(nblk(npair, 256)), dim3(512), 0, s, M, Ps, n, (int64_t)npair, Jp);
}
// J_p in split BF16: Phi cut into its slices, then the contraction; the
// inner length kc (a multiple of 32) selects the compiled variant.
template <int S>
void launch_jp16_s(const float* M, const double* Phi, void* Psv, int n, int npair, double* Jp, hipStream_t s) {
  const int kc = j16_kc(S, n);
  __bf16* Ps = static_cast<__bf16*>(Psv);
  hipLaunchKernelGGL((phi_split_kernel<S>), dim3(n * n), dim3(256), 0, s, Phi, n, kc, Ps);
  const int NT = (n + 15) / 16, KC = kc / 32;
#define TAI_JP16(nt, kcc) if (NT == nt && KC == kcc) return launch_jp16_k<nt, S, kcc>(M, Ps, n, npair, Jp, s)
  if constexpr (S == 2) {
    // 3 n rounded up to 32: n <= 16 -> KC <= 2; <= 32 -> <= 3; <= 48 -> <= 5; <= 64 -> <= 6
    TAI_JP16(1, 1); TAI_JP16(1, 2);
    TAI_JP16(2, 2); TAI_JP16(2, 3);
    TAI_JP16(3, 4); TAI_JP16(3, 5);
    TAI_JP16(4, 5); TAI_JP16(4, 6);
  } else {
    // 6 n rounded up to 32: n <= 16 -> KC <= 3; <= 32 -> <= 6; <= 48 -> <= 9; <= 64 -> <= 12
    TAI_JP16(1, 1); TAI_JP16(1, 2); TAI_JP16(1, 3);
    TAI_JP16(2, 4); TAI_JP16(2, 5); TAI_JP16(2, 6);
    TAI_JP16(3, 7); TAI_JP16(3, 8); TAI_JP16(3, 9);
    TAI_JP16(4, 10); TAI_JP16(4, 11); TAI_JP16(4, 12);
  }
#undef TAI_JP16
}

// the FP32 pair contraction reads an FP32 copy of the moments (in w.M32),
// made once per call
void convert_moments(int prec, const double* M, int n, int npair, const JWork& w, hipStream_t s) {
  if (prec != kFP32 && !split_j(prec)) return;
  const int64_t count = 3 * (int64_t)n * npair;
  hipLaunchKernelGGL(to_fp32_kernel, dim3(nblk(count, 256)), dim3(256), 0, s, M, count, w.M32);
}

// Phi = sum_k wsc_k rho x_0 K_k x_1 K_k x_2 K_k (wsc = (2/sqrt(pi)) w) on the
// FP64 matrix cores: the slab products into w.T1, the mode-0 products and
// node sum with the node runs' partial tensors in w.T2.  The plain J and the
// one-box adaptive J both take this exact sequence.
hipError_t launch_phi_grid(const double* rho, const double* K, const double* wsc, int n, int nq, const JWork& w,
                           double* Phi, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  return launch_mode_products(rho, 1, 1, K, 0, wsc, n, nq, w.T1, 1, 0, nq, Phi, w.T2, (int64_t)nq * n3, s);
}

// rho from the pair densities in w.Dt, then Phi = (2/sqrt(pi)) sum_k w_k rho x_d K_k
// (into w.rho and w.Phi)
hipError_t launch_rho_phi(int prec, const double* M, int npair, int n, int nq, const NodeTables& tb, const JWork& w,
                          hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  if (rho_split(prec)) launch_rho16(prec, w.M32, n, npair, w, s);
  else if (prec == kFP32 || split_j(prec))
    launch_pair_contraction_rho<JF32, 1>(static_cast<const float*>(w.M32), n, npair, w, s);
  else if (n <= 48) launch_pair_contraction_rho<JF64, 2>(M, n, npair, w, s);
  else launch_pair_contraction_rho<JF64, 1>(M, n, npair, w, s);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, w.rho_part, w.nchunk, n3, w.rho);
  hipLaunchKernelGGL(repeat_weights_kernel, dim3(nblk(nq, 256)), dim3(256), 0, s, tb.w, nq, 1, kTwoOverSqrtPi, w.wsc);
  return launch_phi_grid(w.rho, tb.K, w.wsc, n, nq, w, w.Phi, s);
}
}  // namespace

hipError_t launch_apply_j(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                          const NodeTables& tb, const double* D, double* J, const JWork& w, hipStream_t s) {
  hipLaunchKernelGGL(density_pairs_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, D, nb, (int64_t)npair, pairs,
                     w.Dt);
  convert_moments(prec, M, n, npair, w, s);
  const hipError_t e = launch_rho_phi(prec, M, npair, n, nq, tb, w, s);
  if (e != hipSuccess) return e;
  if (split_j(prec)) {
    if (j_slices(prec) == 3) launch_jp16_s<3>(w.M32, w.Phi, w.Ps, n, npair, w.Jp, s);
    else launch_jp16_s<2>(w.M32, w.Phi, w.Ps, n, npair, w.Jp, s);
  } else if (prec == kFP32) launch_pair_contraction_jp<JF32>(M, n, npair, w, s);
  else launch_pair_contraction_jp<JF64>(M, n, npair, w, s);
  if (pairs) {
    const int64_t nn = (int64_t)nb * nb;
    hipLaunchKernelGGL(zero_kernel, dim3(nblk(nn, 256)), dim3(256), 0, s, J, nn);
  }
  hipLaunchKernelGGL(unpack_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, w.Jp, nb, (int64_t)npair, pairs, J);
  return hipGetLastError();
}


// J over adaptive boxes (section 6.2 with eq. coulapprox): rho_s of every
// partition on its own grid, then for every partition s
//   Phi_s = (2/sqrt(pi)) sum_s' sum_k w_k rho_s' x_d K_k^(s,s')
// (the slab and mode-0 passes of each partition pair write their node
// products side by side, one weighted sum over the (s', k) blocks follows),
// J_p for the pairs of s, unpacked into J.
//
// One box runs the plain path's kernels (the same bits as tai_apply_J).
// More boxes: rho of all partitions in one launch (the single list's chunk
// count shared out among them), the mode products of all box pairs at once
// on the matrix cores with 2/sqrt(pi) folded into the repeated weights, and
// J_p of all partitions in one launch; the split-BF16 contractions keep a
// launch per partition.
namespace {
template <class Op, int A0W, class MT>
void launch_rho_spans(const MT* M, int n, const Spans& sp, int nspan, int nchunk, const double* Dt, double* part,
                      hipStream_t s) {
  const dim3 rg((n + 8 * A0W - 1) / (8 * A0W), nchunk, nspan);
  if (n <= 16) hipLaunchKernelGGL((rho_spans_kernel<Op, 1, A0W, MT>), rg, dim3(512), 0, s, M, Dt, n, sp, part);
  else if (n <= 32) hipLaunchKernelGGL((rho_spans_kernel<Op, 2, A0W, MT>), rg, dim3(512), 0, s, M, Dt, n, sp, part);
  else if (n <= 48) hipLaunchKernelGGL((rho_spans_kernel<Op, 3, A0W, MT>), rg, dim3(512), 0, s, M, Dt, n, sp, part);
  else hipLaunchKernelGGL((rho_spans_kernel<Op, 4, 1, MT>), rg, dim3(512), 0, s, M, Dt, n, sp, part);
}
template <class Op>
void launch_jp_spans(const double* M, int n, const Spans& sp, int nspan, const double* Phi, double* Jp,
                     hipStream_t s) {
  const unsigned jb = (unsigned)sp.blk[nspan];
  if (jb == 0) return;
  if (n <= 16) hipLaunchKernelGGL((jp_spans_kernel<Op, 1>), dim3(jb), dim3(512), 0, s, M, Phi, n, nspan, sp, Jp);
  else if (n <= 32) hipLaunchKernelGGL((jp_spans_kernel<Op, 2>), dim3(jb), dim3(512), 0, s, M, Phi, n, nspan, sp, Jp);
  else if (n <= 48) hipLaunchKernelGGL((jp_spans_kernel<Op, 3>), dim3(jb), dim3(512), 0, s, M, Phi, n, nspan, sp, Jp);
  else hipLaunchKernelGGL((jp_spans_kernel<Op, 4>), dim3(jb), dim3(512), 0, s, M, Phi, n, nspan, sp, Jp);
}
}  // namespace

hipError_t launch_apply_j_parts(int prec, const double* M, int nb, const int32_t* pairs, const int64_t* offs,
                                int nparts, int n, int nq, const double* w, const double* Kx, const double* D,
                                double* J, const JWork& wk, double* rho_all, double* T2_all, double* Phi_all,
                                double* wrep, hipStream_t s) {
  const int64_t total = offs[nparts];
  const int64_t n3 = (int64_t)n * n * n, n2 = (int64_t)n * n;
  hipLaunchKernelGGL(density_pairs_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, D, nb, total, pairs, wk.Dt);
  convert_moments(prec, M, n, (int)total, wk, s);
  // one box: the plain path's sequence (the same bits as tai_apply_J); the
  // weights carry 2/sqrt(pi) either way
  const bool one = nparts == 1;
  hipLaunchKernelGGL(repeat_weights_kernel, dim3(nblk((int64_t)nq * nparts, 256)), dim3(256), 0, s, w, nq, nparts,
                     kTwoOverSqrtPi, wrep);
  Spans sp{};
  for (int p = 0; p <= nparts; ++p) {
    sp.off[p] = offs[p];
    sp.blk[p] = p == 0 ? 0 : sp.blk[p - 1] + nblk(offs[p] - offs[p - 1], 256);
  }
  // chunks per partition: the single list's count shared out, so that the
  // partial grids of all partitions fit where the list's would
  const int pchunk = wk.nchunk / nparts;
  if (!one && !rho_split(prec) && pchunk >= 1) {
    if (prec == kFP32 || split_j(prec))
      launch_rho_spans<JF32, 1>(static_cast<const float*>(wk.M32), n, sp, nparts, pchunk, wk.Dt, wk.rho_part, s);
    else if (n <= 48) launch_rho_spans<JF64, 2>(M, n, sp, nparts, pchunk, wk.Dt, wk.rho_part, s);
    else launch_rho_spans<JF64, 1>(M, n, sp, nparts, pchunk, wk.Dt, wk.rho_part, s);
    hipLaunchKernelGGL(sum_parts_kernel, dim3(nblk(n3, 256), nparts), dim3(256), 0, s, wk.rho_part, pchunk, n3,
                       rho_all);
  } else {
    for (int p = 0; p < nparts; ++p) {
      const int64_t cnt = offs[p + 1] - offs[p];
      double* rho_p = rho_all + p * n3;
      if (cnt == 0) {
        hipLaunchKernelGGL(zero_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, rho_p, n3);
        continue;
      }
      JWork wp = wk;
      wp.Dt = wk.Dt + offs[p];
      const double* Mp = M + 3 * (int64_t)n * offs[p];
      if (rho_split(prec)) launch_rho16(prec, wk.M32 + 3 * (int64_t)n * offs[p], n, (int)cnt, wp, s);
      else if (prec == kFP32 || split_j(prec))
        launch_pair_contraction_rho<JF32, 1>(static_cast<const float*>(wk.M32 + 3 * (int64_t)n * offs[p]), n,
                                             (int)cnt, wp, s);
      else if (n <= 48) launch_pair_contraction_rho<JF64, 2>(Mp, n, (int)cnt, wp, s);
      else launch_pair_contraction_rho<JF64, 1>(Mp, n, (int)cnt, wp, s);
      hipLaunchKernelGGL(sum_parts_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, wk.rho_part, wk.nchunk, n3, rho_p);
    }
  }
  if (!one) {
    // T1 of box pair (p, q) = rho_q through the tables K^(p,q), at
    // T2_all[(p nparts + q) nq]; Phi_p sums its nparts nq node blocks (the
    // partial grids of rho are free again and hold the node runs' sums)
    const hipError_t e = launch_mode_products(rho_all, (int64_t)nparts * nparts, nparts, Kx, (int64_t)nq * n2, wrep,
                                              n, nq, T2_all, nparts, (int64_t)nparts * nq * n2, nparts * nq, Phi_all,
                                              wk.rho_part, (int64_t)wk.nchunk * n3, s);
    if (e != hipSuccess) return e;
    if (!split_j(prec)) {
      if (prec == kFP32) launch_jp_spans<JF32>(M, n, sp, nparts, Phi_all, wk.Jp, s);
      else launch_jp_spans<JF64>(M, n, sp, nparts, Phi_all, wk.Jp, s);
      hipLaunchKernelGGL(unpack_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, wk.Jp, nb, total, pairs, J);
      return hipGetLastError();
    }
  }
  for (int p = 0; p < nparts; ++p) {
    const int64_t cnt = offs[p + 1] - offs[p];
    if (cnt == 0) continue;
    if (one) {
      const hipError_t e = launch_phi_grid(rho_all, Kx, wrep, n, nq, wk, wk.Phi, s);
      if (e != hipSuccess) return e;
    }
    JWork wp = wk;
    wp.Jp = wk.Jp + offs[p];
    wp.Phi = one ? wk.Phi : Phi_all + (int64_t)p * n3;
    if (split_j(prec)) {
      const float* M32p = wk.M32 + 3 * (int64_t)n * offs[p];
      if (j_slices(prec) == 3) launch_jp16_s<3>(M32p, wp.Phi, wk.Ps, n, (int)cnt, wp.Jp, s);
      else launch_jp16_s<2>(M32p, wp.Phi, wk.Ps, n, (int)cnt, wp.Jp, s);
    } else if (prec == kFP32) {
      launch_pair_contraction_jp<JF32>(M + 3 * (int64_t)n * offs[p], n, (int)cnt, wp, s);
    } else {
      launch_pair_contraction_jp<JF64>(M + 3 * (int64_t)n * offs[p], n, (int)cnt, wp, s);
    }
    hipLaunchKernelGGL(unpack_kernel, dim3(nblk(cnt, 256)), dim3(256), 0, s, wp.Jp, nb, cnt, pairs + offs[p], J);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Orbitals per launch of the batched orbital densities, and the chunks of
// pairs each orbital's density is split into (the launch holds enough work
// groups for the device either way).
constexpr int kMoBlock = 32;
// The pair contraction runs one work group per compute unit: the chunk
// count is the one between 2 and 4 waves of work groups over the device's
// `cus` units whose last wave is fullest (the first such, at most the
// single-density count).
int mo_chunks(int prec, int n, int npair, int ob, int cus) {
  const int groups = rho_groups(prec, n) * ob;
  const int cap = j_nchunk(prec, n, npair);
  int best = 1;
  double best_eff = -1.0;
  for (int c = (2 * cus + groups - 1) / groups; c <= (4 * cus + groups - 1) / groups && c <= cap; ++c) {
    const int64_t total = (int64_t)groups * c;
    const double eff = (double)total / (double)(((total + cus - 1) / cus) * cus);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = c;
    }
  }
  if (best_eff < 0) best = cap < (2 * cus + groups - 1) / groups ? cap : (2 * cus + groups - 1) / groups;
  return best < 1 ? 1 : best;
}

size_t mo_work_bytes(int prec, int n, int nq, int npair, int norb, int cus) {
  const size_t n3 = (size_t)n * n * n;
  const int ob = norb < kMoBlock ? norb : kMoBlock;
  return align256(8 * n3 * norb) * 2 + align256(8 * (size_t)npair * ob) +
         align256(8 * n3 * ob * mo_chunks(prec, n, npair, ob, cus)) + align256(8 * n3 * nq * ob);
}

// All orbitals' grid densities rho_i = Q(i,:) M_max (the paper's Q M_max,
// eq. Coul) and Phi_i, in blocks of kMoBlock orbitals with one launch per
// stage for the whole block: the orbital pair densities, the pair
// contraction (grid z = orbital, each orbital's chunks of pairs), the chunk
// sums, the mode products and the node sums; then J_mo(i, j) = <rho_i, Phi_j>.
hipError_t launch_coulomb_mo(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                             const NodeTables& tb, const double* Q, int norb, int cus, void* work, double* Jmo,
                             const JWork& w, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  convert_moments(prec, M, n, npair, w, s);
  const int obmax = norb < kMoBlock ? norb : kMoBlock;
  const int nc = mo_chunks(prec, n, npair, obmax, cus);
  char* p = static_cast<char*>(work);
  double* R = reinterpret_cast<double*>(p); p += align256(8 * n3 * norb);
  double* F = reinterpret_cast<double*>(p); p += align256(8 * n3 * norb);
  double* Dt = reinterpret_cast<double*>(p); p += align256(8 * (size_t)npair * obmax);
  double* part = reinterpret_cast<double*>(p); p += align256(8 * n3 * obmax * nc);
  double* T1 = reinterpret_cast<double*>(p);
  for (int i0 = 0; i0 < norb; i0 += obmax) {
    const int ob = norb - i0 < obmax ? norb - i0 : obmax;
    hipLaunchKernelGGL(orbital_pairs_kernel, dim3(nblk(npair, 256), ob), dim3(256), 0, s, Q + (int64_t)i0 * nb, nb,
                       (int64_t)npair, pairs, Dt);
    JWork wb = w;
    wb.Dt = Dt;
    wb.nchunk = nc;
    wb.rho_part = part;
    if (prec == kFP32)
      launch_pair_contraction_rho<JF32, 1>(static_cast<const float*>(w.M32), n, npair, wb, s, ob);
    else if (n <= 48) launch_pair_contraction_rho<JF64, 2>(M, n, npair, wb, s, ob);
    else launch_pair_contraction_rho<JF64, 1>(M, n, npair, wb, s, ob);
    double* Rb = R + (int64_t)i0 * n3;
    hipLaunchKernelGGL(sum_parts_kernel, dim3(nblk(n3, 256), ob), dim3(256), 0, s, part, nc, n3, Rb);
    // the block's mode products on the matrix cores (Phi without 2/sqrt(pi),
    // which the dot products apply)
    // (the partial grids of rho are free again and hold the node runs' sums)
    const hipError_t e = launch_mode_products(Rb, ob, ob, tb.K, 0, tb.w, n, nq, T1, ob, 0, nq,
                                              F + (int64_t)i0 * n3, part, (int64_t)ob * nc * n3, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(mo_dot_kernel, dim3(norb, norb), dim3(256), 0, s, R, F, n3, norb, kTwoOverSqrtPi, Jmo);
  return hipGetLastError();
}


}  // namespace tai
