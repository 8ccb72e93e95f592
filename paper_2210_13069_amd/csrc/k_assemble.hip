// Assembly of the pair matrix B (Theorem 3.1 in Hadamard form, eq. Fi):
//
//   B(p,q) = (2/sqrt(pi)) sum_k w_k prod_{d=0..2} G_{k,d}(p,q),
//   G_{k,d} = M_d^T (K_k M_d).
//
// Three kernels:
//   pack     A_d[p][:]    = M_d(:,p) scaled by 2^-e(p,d), split into slices
//   project  Y_{k,d}[q][:] = (K_k M_d)(:,q) scaled by 2^-e(q,d) (and by w_k
//            for d = 2), split into slices; FP64 arithmetic.  This k-dependent
//            operand is written to HBM once per call (1.98 GB for F16X3 at
//            Nb = 400) and streamed back by the assembly.
//   assemble one work group per output tile; for each k it forms the three
//            G tiles with MFMA (inner dimension = the concatenated slice
//            products), multiplies them elementwise in registers and
//            accumulates into the tile: the G tiles and their products never
//            reach memory.  The tile (P,Q), P <= Q, is stored together with
//            its mirror.
//
// Operand rows are K-contiguous ("NT" product): G(p,q) = sum_c A[p][c] Y[q][c],
// so both MFMA operands are read with the same per-lane addressing, and a
// consistent permutation of the inner index inside a 16-byte lane load is
// harmless.  Slice layouts (each segment n long, zero padded to kc):
//   BF16X3 / F16X3:  A = [s0 | s0 | s1],          Y = [s0 | s1 | s0]
//   BF16X6:          A = [s0|s0|s1|s0|s1|s2],     Y = [s0|s1|s0|s2|s1|s0]
// so the inner product sums s_i s_j over i + j <= S-1.
#include "tai_internal.h"

#include <cmath>
#include <type_traits>

namespace tai {
namespace {

typedef double v2d __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr double kTwoOverSqrtPi = 1.1283791670955126;  // 2/sqrt(pi)

// ---------------------------------------------------------------------------
// operand formats
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline T to_slice(double x);
template <>
__device__ inline __bf16 to_slice<__bf16>(double x) { return (__bf16)(float)x; }
// FP64 -> FP32 -> FP16 rounds exactly as FP64 -> FP16 does (24 >= 2*11 + 2
// bits), so the compiler folds the two conversions into one, which has no
// instruction and is expanded into ~35 integer operations.  The empty asm
// keeps the two hardware conversions.
template <>
__device__ inline _Float16 to_slice<_Float16>(double x) {
  float f = (float)x;
  __asm__("" : "+v"(f));
  return (_Float16)f;
}

// Operand rows are staged through LDS so that the global writes coalesce: a
// work group of kRowsPerTile threads builds that many consecutive rows (one
// per thread) in an LDS tile whose row stride is an odd number of 32-bit
// words (per-thread element writes hit distinct banks), then copies the tile
// out word by word.
constexpr int kRowsPerTile = 64;

__device__ inline int tile_stride_words(int prec, int kc) {
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  return kc * es / 4 + 1;
}

template <typename T>
__device__ inline void put16(uint32_t* row, int x, T v) {
  reinterpret_cast<T*>(row)[x] = v;
}

// Write element a (all its slice segments) of an operand row held in LDS.
// side 0 = A layout, side 1 = Y layout.
__device__ inline void tile_elem(int prec, int side, double x, int n, int a, uint32_t* row) {
  if (prec == kFP64) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    row[2 * a] = (uint32_t)u;
    row[2 * a + 1] = (uint32_t)(u >> 32);
  } else if (prec == kFP32) {
    row[a] = __float_as_uint((float)x);
  } else if (prec == kF16X3) {
    // A = [h0 | h0 | h1], Y = [h0 | h1 | h0]
    const _Float16 h0 = to_slice<_Float16>(x);
    const _Float16 h1 = to_slice<_Float16>(x - (double)h0);
    put16(row, seg_pos(prec, n, 0, a), h0);
    put16(row, seg_pos(prec, n, 1, a), side ? h1 : h0);
    put16(row, seg_pos(prec, n, 2, a), side ? h0 : h1);
  } else {
    // BF16X3: A = [s0 | s0 | s1], Y = [s0 | s1 | s0]
    // BF16X6: A = [s0|s0|s1|s0|s1|s2], Y = [s0|s1|s0|s2|s1|s0]
    const __bf16 s0 = to_slice<__bf16>(x);
    const double r1 = x - (double)(float)s0;
    const __bf16 s1 = to_slice<__bf16>(r1);
    put16(row, seg_pos(prec, n, 0, a), s0);
    put16(row, seg_pos(prec, n, 1, a), side ? s1 : s0);
    put16(row, seg_pos(prec, n, 2, a), side ? s0 : s1);
    if (prec == kBF16X6) {
      const __bf16 s2 = to_slice<__bf16>(r1 - (double)(float)s1);
      put16(row, seg_pos(prec, n, 3, a), side ? s2 : s0);
      put16(row, seg_pos(prec, n, 4, a), s1);
      put16(row, seg_pos(prec, n, 5, a), side ? s0 : s2);
    }
  }
}

// Zero the padding [nseg*n, kc) of a row held in LDS.
__device__ inline void tile_pad(int prec, int n, int kc, uint32_t* row) {
  if (prec == kFP64 || prec == kFP32) {
    const int w = prec == kFP64 ? 2 : 1;
    for (int x = n * w; x < kc * w; ++x) row[x] = 0u;
  } else {
    const int nseg = prec == kBF16X6 ? 6 : 3;
    for (int x = nseg * n; x < kc; ++x) put16<unsigned short>(row, x, 0);
  }
}

// Copy the LDS tile of kRowsPerTile rows to dst (rows contiguous, kc elements
// each) in 16-byte stores: a row is kc * es bytes, a multiple of 16 for every
// operand format (kc is a multiple of 8, or of 32 for the 16-bit slices), and
// dst is 16-byte aligned.
__device__ inline void tile_store(int prec, int kc, const uint32_t* tile, int stride_w, uint32_t* __restrict__ dst) {
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  const int qpr = kc * es / 16;  // 16-byte quads per row
  const int total = kRowsPerTile * qpr;
  uint4* __restrict__ dst4 = reinterpret_cast<uint4*>(dst);
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int r = e / qpr, q = e - r * qpr;
    const uint32_t* src = tile + r * stride_w + 4 * q;
    dst4[e] = uint4{src[0], src[1], src[2], src[3]};
  }
}

__device__ inline int scale_exponent(double mx) {
  if (!(mx > 0.0)) return 0;
  int e = ilogb(mx) + 1;  // mx * 2^-e in [0.5, 1)
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// grid (prow / kRowsPerTile, 3): A_d rows and the exponents e(p, d).
template <int NMAX>
__device__ inline void pack_body(int prec, const double* __restrict__ M, int n, int64_t npair, int prow, int kc,
                                 char* __restrict__ A, int32_t* __restrict__ ex) {
  extern __shared__ uint32_t tile[];
  const int d = blockIdx.y;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsPerTile;
  const int64_t p = row0 + threadIdx.x;
  const int sw = tile_stride_words(prec, kc);
  uint32_t* row = tile + threadIdx.x * sw;
  double v[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) v[a] = 0.0;
  int e = 0;
  if (p < npair) {
    double mx = 0.0;
#pragma unroll
    for (int a = 0; a < NMAX; ++a) {
      if (a < n) {
        v[a] = M[((int64_t)d * n + a) * npair + p];
        mx = fmax(mx, fabs(v[a]));
      }
    }
    if (prec != kFP64) e = scale_exponent(mx);
  }
  ex[(int64_t)d * prow + p] = e;
#pragma unroll
  for (int a = 0; a < NMAX; ++a)
    if (a < n) tile_elem(prec, 0, ldexp(v[a], -e), n, a, row);
  tile_pad(prec, n, kc, row);
  __syncthreads();
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  tile_store(prec, kc, tile, sw, reinterpret_cast<uint32_t*>(A + (((int64_t)d * prow + row0) * kc) * es));
}

// Y_{k,d} rows, (K_k M_d)(:, q) scaled by 2^-e(q,d) (and by w_k 2^ysh for d = 2),
// in the operand format of prec, for 64 rows q and one direction d over all
// nodes k.  The product runs on the FP64 matrix cores (v_mfma_f64_16x16x4):
// wave w holds the A fragments M_d(b, q) of rows q0 + 16 w .. +16 for the
// whole kernel; per node, K_k is staged in LDS (zero padded to NP x NP, the
// next node's values in registers during the MFMAs), the 16 x NP output of
// each wave is split into slices into an LDS tile of 64 rows, and the tile
// leaves as one contiguous block of Y.
typedef double v4d_t __attribute__((ext_vector_type(4)));

template <int NT, int PREC>
__device__ inline void project_mfma_body(const double* __restrict__ M, int n, int64_t npair, int prow,
                                         int nq, int kc, const double* __restrict__ K,
                                         const double* __restrict__ w, const int32_t* __restrict__ ex,
                                         int ysh, char* __restrict__ Y) {
  constexpr int prec = PREC;
  constexpr int NP = 16 * NT, NK = NP / 4, PS = NP + 1;
  constexpr int KPER = (NP * NP + 255) / 256;  // staged K values per thread
  extern __shared__ double smem[];
  double* Ks = smem;                                            // [NP][PS]
  uint32_t* tile = reinterpret_cast<uint32_t*>(smem + NP * PS);  // [64][sw]
  const int d = blockIdx.y;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsPerTile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int sw = tile_stride_words(prec, kc);
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);

  // A fragments: row q = row0 + 16 w + l%16, inner index b = 4 s + l/16
  double am[NK];
  {
    const int64_t q = row0 + 16 * wave + r16;
#pragma unroll
    for (int st = 0; st < NK; ++st) {
      const int bb = 4 * st + kg;
      am[st] = (q < npair && bb < n) ? M[((int64_t)d * n + bb) * npair + q] : 0.0;
    }
  }
  // the scale 2^-e of this lane's output rows 16 w + l/16 + 4 r
  double rs[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t q = row0 + 16 * wave + kg + 4 * r;
    rs[r] = q < npair ? ldexp(1.0, -ex[(int64_t)d * prow + q]) : 0.0;
  }
  // padding columns of the tile are zero for every node
  for (int r = threadIdx.x; r < kRowsPerTile; r += 256) tile_pad(prec, n, kc, tile + r * sw);

  double kp[KPER];
  auto load_k = [&](int k) {
    const double* Kk = K + (int64_t)k * n * n;
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int a = e / NP, bb = e % NP;
      kp[i] = (e < NP * NP && a < n && bb < n) ? Kk[a * n + bb] : 0.0;
    }
  };
  load_k(0);
  for (int k = 0; k < nq; ++k) {
    __syncthreads();  // previous node: Ks read and the tile copied out
#pragma unroll
    for (int i = 0; i < KPER; ++i) {
      const int e = threadIdx.x + 256 * i;
      if (e < NP * NP) Ks[(e / NP) * PS + e % NP] = kp[i];
    }
    __syncthreads();
    if (k + 1 < nq) load_k(k + 1);
    const double wk = (d == 2) ? ldexp(w[k], ysh) : 1.0;
    // one column tile at a time: its fragments, MFMAs and slices
#pragma unroll 1
    for (int j = 0; j < NT; ++j) {
      v4d_t acc = v4d_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < NK; ++st)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(am[st], Ks[(16 * j + r16) * PS + 4 * st + kg], acc, 0, 0, 0);
      // lane l holds column a = 16 j + l%16, rows l/16 + 4 r
      const int a = 16 * j + r16;
      if (a < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          tile_elem(prec, 1, acc[r] * (rs[r] * wk), n, a, tile + (16 * wave + kg + 4 * r) * sw);
      }
    }
    __syncthreads();
    tile_store(prec, kc, tile, sw, reinterpret_cast<uint32_t*>(Y + ((((int64_t)k * 3 + d) * prow + row0) * kc) * es));
  }
}

// ---------------------------------------------------------------------------
// MFMA wrappers.  16x16 output blocks; lane l holds 4 entries of column l%16:
// rows 4*(l/16)+r for the f32/f16/bf16 instructions and rows (l/16)+4r for
// the f64 one (row_of).  Each lane loads 16 (f32: 8) contiguous bytes of its
// row's K-vector.
// ---------------------------------------------------------------------------
struct OpF64 {
  using Frag = v2d;           // 2 K-steps of the 16x16x4 f64 MFMA
  using Acc = v4d;
  static constexpr int kChunk = 8;   // K elements per 64-lane load
  static constexpr int kPerLane = 2;
  __device__ static inline int row_of(int kg, int r) { return kg + 4 * r; }
  __device__ static inline Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline Acc mma(Frag a, Frag b, Acc c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.y, c, 0, 0, 0);
    return c;
  }
};
struct OpF32 {
  using Frag = v2f;
  using Acc = v4f;
  static constexpr int kChunk = 8;
  static constexpr int kPerLane = 2;
  __device__ static inline int row_of(int kg, int r) { return 4 * kg + r; }
  __device__ static inline Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline Acc mma(Frag a, Frag b, Acc c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c, 0, 0, 0);
    return c;
  }
};
struct OpF16 {
  using Frag = v8h;
  using Acc = v4f;
  static constexpr int kChunk = 32;
  static constexpr int kPerLane = 8;
  __device__ static inline int row_of(int kg, int r) { return 4 * kg + r; }
  __device__ static inline Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
struct OpBF16 {
  using Frag = v8bf;
  using Acc = v4f;
  static constexpr int kChunk = 32;
  static constexpr int kPerLane = 8;
  __device__ static inline int row_of(int kg, int r) { return 4 * kg + r; }
  __device__ static inline Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <class Op> struct ElemOf;
template <> struct ElemOf<OpF64> { using T = double; };
template <> struct ElemOf<OpF32> { using T = float; };
template <> struct ElemOf<OpF16> { using T = _Float16; };
template <> struct ElemOf<OpBF16> { using T = __bf16; };

// FP64 accumulates across k in FP64 directly; the others accumulate groups
// of kGroup nodes in FP32 and the groups in FP64.
constexpr int kGroup = 8;

__device__ inline int64_t tri_start(int64_t T, int64_t I) { return I * T - (I * (I - 1)) / 2; }

__device__ inline void decode_tile(int64_t T, int64_t t, int& I, int& J) {
  const double b2 = 2.0 * T + 1.0;
  int64_t i = (int64_t)floor(0.5 * (b2 - sqrt(b2 * b2 - 8.0 * (double)t)));
  if (i < 0) i = 0;
  if (i > T - 1) i = T - 1;
  while (i > 0 && tri_start(T, i) > t) --i;
  while (i + 1 < T && tri_start(T, i + 1) <= t) ++i;
  I = (int)i;
  J = (int)(i + (t - tri_start(T, i)));
}

// Wave tile = (16*WM) x (16*WN); work group = 2 x 2 waves.
template <class Op, int WM, int WN>
__device__ inline void assemble_tile(const AsmMol& m, int I, int J) {
  using T = typename ElemOf<Op>::T;
  using Acc = typename Op::Acc;
  using Frag = typename Op::Frag;
  constexpr int TILE = 32 * WM;  // == 32 * WN
  static_assert(WM == WN, "square tiles");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t row0 = (int64_t)I * TILE + wr * 16 * WM;
  const int64_t col0 = (int64_t)J * TILE + wc * 16 * WN;
  const int kc = m.kc;
  const int64_t prow = m.prow;
  const T* __restrict__ Abase = static_cast<const T*>(m.A);
  const T* __restrict__ Ybase = static_cast<const T*>(m.Y);

  constexpr bool kF64 = sizeof(T) == 8;
  Acc acc[WM][WN];
  v4d acc64[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) { acc[i][j] = Op::zero(); acc64[i][j] = v4d{0.0, 0.0, 0.0, 0.0}; }

  for (int k = 0; k < m.nq; ++k) {
    Acc H[WM][WN];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Acc G[WM][WN];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) G[i][j] = Op::zero();
      const T* Ad = Abase + ((int64_t)d * prow + row0 + r16) * kc + kg * Op::kPerLane;
      const T* Yd = Ybase + (((int64_t)k * 3 + d) * prow + col0 + r16) * kc + kg * Op::kPerLane;
      for (int c0 = 0; c0 < kc; c0 += Op::kChunk) {
        Frag fa[WM], fb[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i) fa[i] = *reinterpret_cast<const Frag*>(Ad + (int64_t)i * 16 * kc + c0);
#pragma unroll
        for (int j = 0; j < WN; ++j) fb[j] = *reinterpret_cast<const Frag*>(Yd + (int64_t)j * 16 * kc + c0);
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) G[i][j] = Op::mma(fa[i], fb[j], G[i][j]);
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          if (d == 0) H[i][j] = G[i][j];
          else if (d == 1) H[i][j] = H[i][j] * G[i][j];
          else acc[i][j] += H[i][j] * G[i][j];
        }
    }
    if (!kF64 && ((k + 1) % kGroup == 0 || k + 1 == m.nq)) {
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = Op::zero();
        }
    }
  }

  const int64_t npair = m.npair;
  const int64_t ldb = m.ldb;
#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int64_t col = col0 + j * 16 + r16;
      const int ecol = kF64 ? 0 : m.ex[col] + m.ex[prow + col] + m.ex[2 * prow + col] - m.ysh;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + i * 16 + Op::row_of(kg, r);
        if (row >= npair || col >= npair) continue;
        double v;
        if (kF64) {
          v = (double)acc[i][j][r] * kTwoOverSqrtPi;
        } else {
          const int erow = m.ex[row] + m.ex[prow + row] + m.ex[2 * prow + row];
          v = ldexp(acc64[i][j][r] * kTwoOverSqrtPi, erow + ecol);
        }
        if (kF64) {
          double* B = static_cast<double*>(m.B);
          B[row * ldb + col] = v;
          if (I != J) B[col * ldb + row] = v;
        } else {
          float* B = static_cast<float*>(m.B);
          B[row * ldb + col] = (float)v;
          if (I != J) B[col * ldb + row] = (float)v;
        }
      }
    }
  }
}

// FP64 / FP32 tile with the k-invariant A operand held in registers: the
// same arithmetic in the same order as assemble_tile (identical results),
// but A is loaded once per tile instead of once per node, and the Y
// fragments of the next PD (node, direction, chunk) steps are loaded while
// the MFMAs of the current one run.  KC is the inner length (n rounded up
// to 8).
// Call f(integral_constant<int, c>) for the compile-time count c == v
// (1 <= v <= N).
template <int N, class F>
__device__ inline void with_count(int v, F&& f) {
  if constexpr (N == 1) {
    f(std::integral_constant<int, 1>{});
  } else {
    if (v >= N) f(std::integral_constant<int, N>{});
    else with_count<N - 1>(v, f);
  }
}

// DEG: the operands are in coefficient form and node k contracts only its
// first ceil(N_k / chunk) inner chunks (the Y rows beyond N_k are zero).
template <class Op, int KC, int WN, int PD, bool DEG = false, int WM = 2>
__device__ inline void assemble_tile_as(const AsmMol& m, int I, int J) {
  using T = typename ElemOf<Op>::T;
  using Acc = typename Op::Acc;
  using Frag = typename Op::Frag;
  // 64 x 64 tile; waves (4 / WM) x (4 / WN), each 16*WM rows x 16*WN columns
  constexpr int TILE = 64, WC = 4 / WN, NCK = KC / Op::kChunk, NSTEP = 3 * NCK;
  static_assert(WM == 2 || WM == 4, "rows per wave");
  static_assert(KC % Op::kChunk == 0, "inner length");
  constexpr bool kF64 = sizeof(T) == 8;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t row0 = (int64_t)I * TILE + wr * 16 * WM;
  const int64_t col0 = (int64_t)J * TILE + wc * 16 * WN;
  const int64_t prow = m.prow;
  const T* __restrict__ Abase = static_cast<const T*>(m.A);
  // Y addressing: a wave-uniform base per step plus one 32-bit lane offset
  typedef __attribute__((address_space(1))) const Frag gFrag;
  const char* __restrict__ Yw = static_cast<const char*>(m.Y) + col0 * KC * (int64_t)sizeof(T);
  const uint32_t ylane = (uint32_t)((r16 * KC + kg * Op::kPerLane) * sizeof(T));

  Frag fa[3][NCK][WM];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < NCK; ++c)
#pragma unroll
      for (int i = 0; i < WM; ++i)
        fa[d][c][i] = *reinterpret_cast<const Frag*>(Abase + ((int64_t)d * prow + row0 + 16 * i + r16) * KC +
                                                     kg * Op::kPerLane + c * Op::kChunk);
  // Y fragments of step s = (k, d, c): Y[k][d][col0 + 16 j + r16][c * chunk + ...]
  auto loadY = [&](int k, int st, Frag (&dst)[WN]) {
    const int d = st / NCK, c = st % NCK;
    const char* y = Yw + (((int64_t)k * 3 + d) * prow * KC + c * Op::kChunk) * (int64_t)sizeof(T);
#pragma unroll
    for (int j = 0; j < WN; ++j) dst[j] = *(gFrag*)(y + ylane + j * 16 * KC * (int)sizeof(T));
  };

  Acc acc[WM][WN];
  v4d acc64[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) { acc[i][j] = Op::zero(); acc64[i][j] = v4d{0.0, 0.0, 0.0, 0.0}; }

  const int nq = m.nq;
  // ring[0] holds the current step's Y fragments, ring[1..PD] the next PD
  // steps' (loads in flight)
  Frag ring[PD + 1][WN];
  const int32_t* __restrict__ nkp = DEG ? m.nk : nullptr;
  if (DEG && nkp != nullptr) {
    // Per-node chunk counts: node k runs 3 * nck(k) steps; the ring still
    // runs PD steps ahead, into the next node's first steps.
    auto nck_of = [&](int k) { return (nkp[k] + Op::kChunk - 1) / Op::kChunk; };
    auto loadY3 = [&](int k, int d, int c, Frag (&dst)[WN]) {
      const char* y = Yw + (((int64_t)k * 3 + d) * prow * KC + c * Op::kChunk) * (int64_t)sizeof(T);
#pragma unroll
      for (int j = 0; j < WN; ++j) dst[j] = *(gFrag*)(y + ylane + j * 16 * KC * (int)sizeof(T));
    };
    int nck_cur = nck_of(0);
#pragma unroll
    for (int a = 0; a < PD; ++a) loadY3(0, a / nck_cur, a % nck_cur, ring[a]);  // 3 * nck >= 3 > PD
    for (int k = 0; k < nq; ++k) {
      const int nck_next = k + 1 < nq ? nck_of(k + 1) : 1;
      with_count<NCK>(nck_cur, [&](auto nc) {
        constexpr int NC = decltype(nc)::value, NS = 3 * NC;
        Acc H[WM][WN], G[WM][WN];
#pragma unroll
        for (int st = 0; st < NS; ++st) {
          const int d = st / NC, c = st % NC;
          if (st + PD < NS) {
            loadY3(k, (st + PD) / NC, (st + PD) % NC, ring[PD]);
          } else if (k + 1 < nq) {
            const int s2 = st + PD - NS;  // step of the next node, < PD
            loadY3(k + 1, s2 / nck_next, s2 % nck_next, ring[PD]);
          }
#pragma unroll
          for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) G[i][j] = Op::mma(fa[d][c][i], ring[0][j], c == 0 ? Op::zero() : G[i][j]);
          if (c == NC - 1) {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
              for (int j = 0; j < WN; ++j) {
                if (d == 0) H[i][j] = G[i][j];
                else if (d == 1) H[i][j] = H[i][j] * G[i][j];
                else acc[i][j] += H[i][j] * G[i][j];
              }
          }
#pragma unroll
          for (int a = 0; a < PD; ++a)
#pragma unroll
            for (int j = 0; j < WN; ++j) ring[a][j] = ring[a + 1][j];
        }
      });
      nck_cur = nck_next;
      if (!kF64 && ((k + 1) % kGroup == 0 || k + 1 == nq)) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
            acc[i][j] = Op::zero();
          }
      }
    }
  } else {
#pragma unroll
  for (int a = 0; a < PD; ++a)
    if (a / NSTEP < nq) loadY(a / NSTEP, a % NSTEP, ring[a]);
  for (int k = 0; k < nq; ++k) {
    Acc H[WM][WN], G[WM][WN];
#pragma unroll
    for (int st = 0; st < NSTEP; ++st) {
      const int d = st / NCK, c = st % NCK;
      {
        const int k2 = k + (st + PD) / NSTEP, st2 = (st + PD) % NSTEP;
        if (k2 < nq) loadY(k2, st2, ring[PD]);
      }
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) G[i][j] = Op::mma(fa[d][c][i], ring[0][j], c == 0 ? Op::zero() : G[i][j]);
      if (c == NCK - 1) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            if (d == 0) H[i][j] = G[i][j];
            else if (d == 1) H[i][j] = H[i][j] * G[i][j];
            else acc[i][j] += H[i][j] * G[i][j];
          }
      }
#pragma unroll
      for (int a = 0; a < PD; ++a)
#pragma unroll
        for (int j = 0; j < WN; ++j) ring[a][j] = ring[a + 1][j];
    }
    if (!kF64 && ((k + 1) % kGroup == 0 || k + 1 == nq)) {
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = Op::zero();
        }
    }
  }
  }

  const int64_t npair = m.npair;
  const int64_t ldb = m.ldb;
#pragma unroll
  for (int i = 0; i < WM; ++i) {
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int64_t col = col0 + j * 16 + r16;
      const int ecol = kF64 ? 0 : m.ex[col] + m.ex[prow + col] + m.ex[2 * prow + col] - m.ysh;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + i * 16 + Op::row_of(kg, r);
        if (row >= npair || col >= npair) continue;
        if (kF64) {
          const double v = (double)acc[i][j][r] * kTwoOverSqrtPi;
          double* B = static_cast<double*>(m.B);
          B[row * ldb + col] = v;
          if (I != J) B[col * ldb + row] = v;
        } else {
          const int erow = m.ex[row] + m.ex[prow + row] + m.ex[2 * prow + row];
          const float v = (float)ldexp(acc64[i][j][r] * kTwoOverSqrtPi, erow + ecol);
          float* B = static_cast<float*>(m.B);
          B[row * ldb + col] = v;
          if (I != J) B[col * ldb + row] = v;
        }
      }
    }
  }
}

// Wave tiles of (16 WM) x (16 WN) in a 64 x 64 tile: WM 2, WN 2: four waves
// of 32 x 32; WM 2, WN 1: eight waves of 32 x 16 (half the accumulator
// registers per wave, for the FP64 operands of the longer inner lengths);
// WM 4, WN 1: four waves of 64 x 16 (each Y fragment feeds four MFMAs).  Two
// waves per SIMD in every form.
template <int WM, int WN>
constexpr int as_threads() { return 64 * (4 / WM) * (4 / WN); }

template <class Op, int KC, int WN, bool DEG, int WM>
__global__ void __launch_bounds__((as_threads<WM, WN>()), (512 / as_threads<WM, WN>()))
assemble_as_kernel(AsmMol m) {
  int I, J;
  decode_tile(m.tiles, blockIdx.x, I, J);
  // FP32 MFMAs take half the cycles of FP64 ones: look two steps ahead
  assemble_tile_as<Op, KC, WN, sizeof(typename ElemOf<Op>::T) == 8 ? 1 : 2, DEG, WM>(m, I, J);
}

template <class Op, int WM, int WN>
__global__ void __launch_bounds__(256)
assemble_kernel(AsmMol m) {
  int I, J;
  decode_tile(m.tiles, blockIdx.x, I, J);
  assemble_tile<Op, WM, WN>(m, I, J);
}

// Persistent variants: work groups take (molecule, tile) items from a queue
// and hand each to `tile(m, I, J)`.
template <class F>
__device__ inline void drain_tile_queue(const AsmMol* __restrict__ mols, int nmol, int64_t nitems, unsigned* counter,
                                        F&& tile) {
  __shared__ int64_t item_s;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_s = (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t item = item_s;
    if (item >= nitems) break;
    // molecule whose item range holds `item` (items are grouped by molecule)
    int lo = 0, hi = nmol - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (mols[mid].tile0 <= item) lo = mid; else hi = mid - 1;
    }
    const AsmMol m = mols[lo];
    int I, J;
    decode_tile(m.tiles, item - m.tile0, I, J);
    tile(m, I, J);
  }
}

template <class Op, int WM, int WN>
__global__ void __launch_bounds__(256)
assemble_queue_kernel(const AsmMol* __restrict__ mols, int nmol, int64_t nitems, unsigned* counter) {
  drain_tile_queue(mols, nmol, nitems, counter,
                   [](const AsmMol& m, int I, int J) { assemble_tile<Op, WM, WN>(m, I, J); });
}

template <class Op, int KC, int WN, bool DEG, int WM>
__global__ void __launch_bounds__((as_threads<WM, WN>()), (512 / as_threads<WM, WN>()))
assemble_as_queue_kernel(const AsmMol* __restrict__ mols, int nmol, int64_t nitems, unsigned* counter) {
  drain_tile_queue(mols, nmol, nitems, counter, [](const AsmMol& m, int I, int J) {
    assemble_tile_as<Op, KC, WN, sizeof(typename ElemOf<Op>::T) == 8 ? 1 : 2, DEG, WM>(m, I, J);
  });
}

__global__ void reset_counter_kernel(unsigned* c) {
  if (threadIdx.x < kAsm16Queues) c[threadIdx.x] = 0u;
}

// Single-molecule kernels and their batch forms: blockIdx.z = molecule of
// the batch; blocks beyond a molecule's padded rows return at once (the
// test is uniform per work group, before any barrier).
template <int NMAX>
__global__ void __launch_bounds__(kRowsPerTile)
pack_kernel(int prec, const double* __restrict__ M, int n, int64_t npair, int prow, int kc,
            char* __restrict__ A, int32_t* __restrict__ ex) {
  pack_body<NMAX>(prec, M, n, npair, prow, kc, A, ex);
}

template <int NMAX>
__global__ void __launch_bounds__(kRowsPerTile)
pack_batch_kernel(int prec, const PrepMol* __restrict__ mols, int n, int kc) {
  const PrepMol& m = mols[blockIdx.z];
  if ((int64_t)blockIdx.x * kRowsPerTile >= m.prow) return;
  pack_body<NMAX>(prec, m.U ? m.U : (m.Mu ? m.Mu : m.M), n, m.npair, m.prow, kc, static_cast<char*>(m.A), m.ex);
}

template <int NT, int PREC>
__global__ void __launch_bounds__(256, 3)
project_kernel(const double* __restrict__ M, int n, int64_t npair, int prow, int nq,
               int kc, const double* __restrict__ K, const double* __restrict__ w,
               const int32_t* __restrict__ ex, int ysh, char* __restrict__ Y) {
  project_mfma_body<NT, PREC>(M, n, npair, prow, nq, kc, K, w, ex, ysh, Y);
}

template <int NT, int PREC>
__global__ void __launch_bounds__(256, 3)
project_batch_kernel(const PrepMol* __restrict__ mols, int n, int nq, int kc) {
  const PrepMol& m = mols[blockIdx.z];
  if ((int64_t)blockIdx.x * kRowsPerTile >= m.prow) return;
  // compressed operands (rank_tol > 0), or the coefficient form (per-node
  // degrees: moments against T_j, kept coefficients), or the node form
  const double* src = m.U ? m.U : (m.Mu ? m.Mu : m.M);
  const double* tab = m.U ? m.Kc : (m.Mu ? m.tb.C : m.tb.K);
  project_mfma_body<NT, PREC>(src, n, m.npair, m.prow, nq, kc, tab, m.tb.w, m.ex, m.ysh, static_cast<char*>(m.Y));
}

size_t project_lds(int prec, int n) {
  const int NP = (n + 15) / 16 * 16;
  const int kc = operand_kc(prec, n);
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  return sizeof(double) * NP * (NP + 1) + sizeof(uint32_t) * kRowsPerTile * (kc * es / 4 + 1);
}

template <int NMAX>
hipError_t launch_pack_t(int prec, const double* M, int n, int npair, int prow, void* A,
                         int32_t* ex, hipStream_t s) {
  const int kc = operand_kc(prec, n);
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  const size_t lds = sizeof(uint32_t) * kRowsPerTile * (kc * es / 4 + 1);
  hipLaunchKernelGGL(pack_kernel<NMAX>, dim3(prow / kRowsPerTile, 3), dim3(kRowsPerTile), lds, s,
                     prec, M, n, (int64_t)npair, prow, kc, static_cast<char*>(A), ex);
  return hipGetLastError();
}

template <int NT, int PREC>
hipError_t launch_project_p(const double* M, int n, int npair, int prow, int nq, const NodeTables& tb,
                            const int32_t* ex, int ysh, void* Y, hipStream_t s) {
  hipLaunchKernelGGL((project_kernel<NT, PREC>), dim3(prow / kRowsPerTile, 3), dim3(256), project_lds(PREC, n), s,
                     M, n, (int64_t)npair, prow, nq, operand_kc(PREC, n), tb.K, tb.w, ex, ysh, static_cast<char*>(Y));
  return hipGetLastError();
}

template <int NT>
hipError_t launch_project_t(int prec, const double* M, int n, int npair, int prow, int nq,
                            const NodeTables& tb, const int32_t* ex, int ysh, void* Y, hipStream_t s) {
  switch (prec) {
    case kFP64: return launch_project_p<NT, kFP64>(M, n, npair, prow, nq, tb, ex, ysh, Y, s);
    case kFP32: return launch_project_p<NT, kFP32>(M, n, npair, prow, nq, tb, ex, ysh, Y, s);
    case kF16X3: return launch_project_p<NT, kF16X3>(M, n, npair, prow, nq, tb, ex, ysh, Y, s);
    case kBF16X3: return launch_project_p<NT, kBF16X3>(M, n, npair, prow, nq, tb, ex, ysh, Y, s);
    default: return launch_project_p<NT, kBF16X6>(M, n, npair, prow, nq, tb, ex, ysh, Y, s);
  }
}

template <int NMAX>
hipError_t launch_pack_batch_t(int prec, const PrepMol* mols, int nmol, int max_prow, int n, hipStream_t s) {
  const int kc = operand_kc(prec, n);
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  const size_t lds = sizeof(uint32_t) * kRowsPerTile * (kc * es / 4 + 1);
  hipLaunchKernelGGL(pack_batch_kernel<NMAX>, dim3(max_prow / kRowsPerTile, 3, nmol), dim3(kRowsPerTile), lds, s,
                     prec, mols, n, kc);
  return hipGetLastError();
}

template <int NT, int PREC>
hipError_t launch_project_batch_p(const PrepMol* mols, int nmol, int max_prow, int n, int nq, hipStream_t s) {
  hipLaunchKernelGGL((project_batch_kernel<NT, PREC>), dim3(max_prow / kRowsPerTile, 3, nmol), dim3(256),
                     project_lds(PREC, n), s, mols, n, nq, operand_kc(PREC, n));
  return hipGetLastError();
}

template <int NT>
hipError_t launch_project_batch_t(int prec, const PrepMol* mols, int nmol, int max_prow, int n, int nq,
                                  hipStream_t s) {
  switch (prec) {
    case kFP64: return launch_project_batch_p<NT, kFP64>(mols, nmol, max_prow, n, nq, s);
    case kFP32: return launch_project_batch_p<NT, kFP32>(mols, nmol, max_prow, n, nq, s);
    case kF16X3: return launch_project_batch_p<NT, kF16X3>(mols, nmol, max_prow, n, nq, s);
    case kBF16X3: return launch_project_batch_p<NT, kBF16X3>(mols, nmol, max_prow, n, nq, s);
    default: return launch_project_batch_p<NT, kBF16X6>(mols, nmol, max_prow, n, nq, s);
  }
}

}  // namespace

hipError_t launch_pack_batch(int prec, const PrepMol* mols, int nmol, int max_prow, int n, hipStream_t s) {
  if (n <= 16) return launch_pack_batch_t<16>(prec, mols, nmol, max_prow, n, s);
  if (n <= 32) return launch_pack_batch_t<32>(prec, mols, nmol, max_prow, n, s);
  if (n <= 48) return launch_pack_batch_t<48>(prec, mols, nmol, max_prow, n, s);
  return launch_pack_batch_t<64>(prec, mols, nmol, max_prow, n, s);
}

hipError_t launch_project_batch(int prec, const PrepMol* mols, int nmol, int max_prow, int n, int nq,
                                hipStream_t s) {
  if (n <= 16) return launch_project_batch_t<1>(prec, mols, nmol, max_prow, n, nq, s);
  if (n <= 32) return launch_project_batch_t<2>(prec, mols, nmol, max_prow, n, nq, s);
  if (n <= 48) return launch_project_batch_t<3>(prec, mols, nmol, max_prow, n, nq, s);
  return launch_project_batch_t<4>(prec, mols, nmol, max_prow, n, nq, s);
}

int operand_esize(int prec) {
  return prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
}

int operand_kc(int prec, int n) {
  auto up = [](int x, int m) { return (x + m - 1) / m * m; };
  switch (prec) {
    case kFP64:
    case kFP32: return up(n, 8);
    case kBF16X6: return up(6 * n, 32);
    default: return up(3 * n, 32);
  }
}

// Edge of the generic kernel's square output tiles, for every arithmetic
// (operand rows are padded further, to a multiple of 256, by the host).
int assemble_tile(int) { return 64; }

hipError_t launch_pack(int prec, const double* M, int n, int npair, int prow, void* A,
                       int32_t* ex, hipStream_t s) {
  if (n <= 16) return launch_pack_t<16>(prec, M, n, npair, prow, A, ex, s);
  if (n <= 32) return launch_pack_t<32>(prec, M, n, npair, prow, A, ex, s);
  if (n <= 48) return launch_pack_t<48>(prec, M, n, npair, prow, A, ex, s);
  return launch_pack_t<64>(prec, M, n, npair, prow, A, ex, s);
}

hipError_t launch_project(int prec, const double* M, int n, int npair, int prow, int nq,
                          const NodeTables& tb, const int32_t* ex, int ysh, void* Y, hipStream_t s) {
  if (n <= 16) return launch_project_t<1>(prec, M, n, npair, prow, nq, tb, ex, ysh, Y, s);
  if (n <= 32) return launch_project_t<2>(prec, M, n, npair, prow, nq, tb, ex, ysh, Y, s);
  if (n <= 48) return launch_project_t<3>(prec, M, n, npair, prow, nq, tb, ex, ysh, Y, s);
  return launch_project_t<4>(prec, M, n, npair, prow, nq, tb, ex, ysh, Y, s);
}

// FP64 uses the eight-wave form from inner length 32 on (the four-wave form
// spills there); FP32 the four waves of 64 x 16.
template <class Op, int KC>
constexpr int as_wn() {
  return sizeof(typename ElemOf<Op>::T) == 8 ? (KC >= 32 ? 1 : 2) : 1;
}
template <class Op, int KC>
constexpr int as_wm() {
  return sizeof(typename ElemOf<Op>::T) == 8 ? 2 : 4;
}

// grid: tiles (one work group each), or, for the queue form, work groups
// of four waves' worth of threads (halved for the eight-wave form).
template <class Op, int KC, bool DEG>
void launch_as_kc(const dim3& grid, const AsmMol* mols, int nmol, int64_t nitems, unsigned* counter,
                  const AsmMol& m, bool queue, hipStream_t s) {
  constexpr int WN = as_wn<Op, KC>(), WM = as_wm<Op, KC>(), NT = as_threads<WM, WN>();
  const dim3 block(NT);
  if (queue) {
    // grid.x counts 256-thread work groups
    const dim3 g((unsigned)(((int64_t)grid.x * 256 + NT - 1) / NT));
    hipLaunchKernelGGL((assemble_as_queue_kernel<Op, KC, WN, DEG, WM>), g, block, 0, s, mols, nmol, nitems, counter);
  } else {
    hipLaunchKernelGGL((assemble_as_kernel<Op, KC, WN, DEG, WM>), grid, block, 0, s, m);
  }
}

template <class Op, int KC>
void launch_as_kc(bool deg, const dim3& grid, const AsmMol* mols, int nmol, int64_t nitems, unsigned* counter,
                  const AsmMol& m, bool queue, hipStream_t s) {
  if (deg) launch_as_kc<Op, KC, true>(grid, mols, nmol, nitems, counter, m, queue, s);
  else launch_as_kc<Op, KC, false>(grid, mols, nmol, nitems, counter, m, queue, s);
}

// deg: molecules may carry per-node degrees (AsmMol::nk).
template <class Op>
bool launch_as(int kc, bool deg, const dim3& grid, const AsmMol* mols, int nmol, int64_t nitems, unsigned* counter,
               const AsmMol& m, bool queue, hipStream_t s) {
  switch (kc) {
    case 8: launch_as_kc<Op, 8>(deg, grid, mols, nmol, nitems, counter, m, queue, s); return true;
    case 16: launch_as_kc<Op, 16>(deg, grid, mols, nmol, nitems, counter, m, queue, s); return true;
    case 24: launch_as_kc<Op, 24>(deg, grid, mols, nmol, nitems, counter, m, queue, s); return true;
    case 32: launch_as_kc<Op, 32>(deg, grid, mols, nmol, nitems, counter, m, queue, s); return true;
    case 40: launch_as_kc<Op, 40>(deg, grid, mols, nmol, nitems, counter, m, queue, s); return true;
    default: return false;
  }
}

hipError_t launch_assemble(int prec, const AsmMol& m, hipStream_t s) {
  const int64_t ntiles = (int64_t)m.tiles * (m.tiles + 1) / 2;
  const dim3 grid((unsigned)ntiles), block(256);
  // inner lengths up to 40: A-stationary tiles (the A operand fits the registers)
  const bool deg = m.nk != nullptr;
  if (prec == kFP64 && launch_as<OpF64>(m.kc, deg, grid, nullptr, 0, 0, nullptr, m, false, s)) return hipGetLastError();
  if (prec == kFP32 && launch_as<OpF32>(m.kc, deg, grid, nullptr, 0, 0, nullptr, m, false, s)) return hipGetLastError();
  switch (prec) {
    case kFP64: hipLaunchKernelGGL((assemble_kernel<OpF64, 2, 2>), grid, block, 0, s, m); break;
    case kFP32: hipLaunchKernelGGL((assemble_kernel<OpF32, 2, 2>), grid, block, 0, s, m); break;
    case kF16X3: hipLaunchKernelGGL((assemble_kernel<OpF16, 2, 2>), grid, block, 0, s, m); break;
    default: hipLaunchKernelGGL((assemble_kernel<OpBF16, 2, 2>), grid, block, 0, s, m); break;
  }
  return hipGetLastError();
}

hipError_t launch_reset_counter(unsigned* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  return hipGetLastError();
}

int assemble_queue_blocks(int /*prec*/, int device) {
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  return cus * 4;
}

hipError_t launch_assemble_queue(int prec, int kc, bool deg, const AsmMol* mols_dev, int nmol, int64_t nitems,
                                 unsigned* counter, int nblocks, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block(256);
  const AsmMol none{};
  if (prec == kFP64 && launch_as<OpF64>(kc, deg, grid, mols_dev, nmol, nitems, counter, none, true, s))
    return hipGetLastError();
  if (prec == kFP32 && launch_as<OpF32>(kc, deg, grid, mols_dev, nmol, nitems, counter, none, true, s))
    return hipGetLastError();
  switch (prec) {
    case kFP64: hipLaunchKernelGGL((assemble_queue_kernel<OpF64, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
    case kFP32: hipLaunchKernelGGL((assemble_queue_kernel<OpF32, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
    case kF16X3: hipLaunchKernelGGL((assemble_queue_kernel<OpF16, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
    default: hipLaunchKernelGGL((assemble_queue_kernel<OpBF16, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
  }
  return hipGetLastError();
}

}  // namespace tai
