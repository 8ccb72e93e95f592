// Assembly of the pair matrix B (Theorem 3.1 in Hadamard form, eq. Fi):
//
//   B(p,q) = (2/sqrt(pi)) sum_k w_k prod_{d=0..2} G_{k,d}(p,q),
//   G_{k,d} = M_d^T (K_k M_d).
//
// Three kernels:
//   pack     A_d[p][:]    = M_d(:,p) scaled by 2^-e(p,d), split into slices
//   project  Y_{k,d}[q][:] = (K_k M_d)(:,q) scaled by 2^-e(q,d) (and by w_k
//            for d = 2), split into slices; FP64 arithmetic
//   assemble one work group per output tile; for each k it forms the three
//            G tiles with MFMA (inner dimension = the concatenated slice
//            products), multiplies them elementwise in registers and
//            accumulates into the tile; no per-k matrix ever reaches memory.
//            The tile (P,Q), P <= Q, is stored together with its mirror.
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
__device__ inline int scale_exponent(double mx) {
  if (!(mx > 0.0)) return 0;
  int e = ilogb(mx) + 1;  // mx * 2^-e in [0.5, 1)
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

template <typename T>
__device__ inline T to_slice(double x);
template <>
__device__ inline __bf16 to_slice<__bf16>(double x) { return (__bf16)(float)x; }
template <>
__device__ inline _Float16 to_slice<_Float16>(double x) { return (_Float16)(float)x; }

// Write element a of an operand row (all its slice segments); pad writes
// the zero tail [nseg*n, kc).
__device__ inline void write_elem(int prec, int side, double x, int n, int a, void* rowp) {
  if (prec == kFP64) {
    static_cast<double*>(rowp)[a] = x;
  } else if (prec == kFP32) {
    static_cast<float*>(rowp)[a] = (float)x;
  } else if (prec == kF16X3) {
    _Float16* r = static_cast<_Float16*>(rowp);
    const _Float16 h0 = to_slice<_Float16>(x);
    const _Float16 h1 = to_slice<_Float16>(x - (double)h0);
    r[a] = h0;
    r[n + a] = side ? h1 : h0;
    r[2 * n + a] = side ? h0 : h1;
  } else {
    __bf16* r = static_cast<__bf16*>(rowp);
    const __bf16 s0 = to_slice<__bf16>(x);
    const double r1 = x - (double)(float)s0;
    const __bf16 s1 = to_slice<__bf16>(r1);
    r[a] = s0;
    r[n + a] = side ? s1 : s0;
    r[2 * n + a] = side ? s0 : s1;
    if (prec == kBF16X6) {
      const __bf16 s2 = to_slice<__bf16>(r1 - (double)(float)s1);
      r[3 * n + a] = side ? s2 : s0;
      r[4 * n + a] = s1;
      r[5 * n + a] = side ? s0 : s2;
    }
  }
}

__device__ inline void write_pad(int prec, int n, int kc, void* rowp) {
  const int nseg = prec == kFP64 || prec == kFP32 ? 1 : (prec == kBF16X6 ? 6 : 3);
  for (int c = nseg * n; c < kc; ++c) {
    if (prec == kFP64) static_cast<double*>(rowp)[c] = 0.0;
    else if (prec == kFP32) static_cast<float*>(rowp)[c] = 0.0f;
    else if (prec == kF16X3) static_cast<_Float16*>(rowp)[c] = (_Float16)0.0f;
    else static_cast<__bf16*>(rowp)[c] = (__bf16)0.0f;
  }
}

// Write one operand row from the n FP64 values v (already scaled).
// side 0 = A layout, side 1 = Y layout.  v is indexed only at compile-time
// positions so it stays in registers.
template <int NMAX>
__device__ inline void write_row(int prec, int side, const double (&v)[NMAX], int n, int kc, void* rowp) {
  if (prec == kFP64) {
    double* r = static_cast<double*>(rowp);
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
      if (a < n) r[a] = v[a];
    for (int c = n; c < kc; ++c) r[c] = 0.0;
    return;
  }
  if (prec == kFP32) {
    float* r = static_cast<float*>(rowp);
#pragma unroll
    for (int a = 0; a < NMAX; ++a)
      if (a < n) r[a] = (float)v[a];
    for (int c = n; c < kc; ++c) r[c] = 0.0f;
    return;
  }
  if (prec == kF16X3) {
    // A = [h0 | h0 | h1], Y = [h0 | h1 | h0]
    _Float16* r = static_cast<_Float16*>(rowp);
#pragma unroll
    for (int a = 0; a < NMAX; ++a) {
      if (a < n) {
        const _Float16 h0 = to_slice<_Float16>(v[a]);
        const _Float16 h1 = to_slice<_Float16>(v[a] - (double)h0);
        r[a] = h0;
        r[n + a] = side ? h1 : h0;
        r[2 * n + a] = side ? h0 : h1;
      }
    }
    for (int c = 3 * n; c < kc; ++c) r[c] = (_Float16)0.0f;
    return;
  }
  __bf16* r = static_cast<__bf16*>(rowp);
  const bool six = prec == kBF16X6;
#pragma unroll
  for (int a = 0; a < NMAX; ++a) {
    if (a < n) {
      const __bf16 s0 = to_slice<__bf16>(v[a]);
      const double r1 = v[a] - (double)(float)s0;
      const __bf16 s1 = to_slice<__bf16>(r1);
      if (!six) {
        // A = [s0 | s0 | s1], Y = [s0 | s1 | s0]
        r[a] = s0;
        r[n + a] = side ? s1 : s0;
        r[2 * n + a] = side ? s0 : s1;
      } else {
        // A = [s0|s0|s1|s0|s1|s2], Y = [s0|s1|s0|s2|s1|s0]
        const __bf16 s2 = to_slice<__bf16>(r1 - (double)(float)s1);
        r[a] = s0;
        r[n + a] = side ? s1 : s0;
        r[2 * n + a] = side ? s0 : s1;
        r[3 * n + a] = side ? s2 : s0;
        r[4 * n + a] = s1;
        r[5 * n + a] = side ? s0 : s2;
      }
    }
  }
  for (int c = (six ? 6 : 3) * n; c < kc; ++c) r[c] = (__bf16)0.0f;
}

template <int NMAX>
__global__ void __launch_bounds__(256)
pack_kernel(int prec, const double* __restrict__ M, int n, int64_t npair, int prow, int kc,
            char* __restrict__ A, int32_t* __restrict__ ex) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * (int64_t)prow) return;
  const int d = (int)(g / prow);
  const int64_t p = g - (int64_t)d * prow;
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  char* rowp = A + g * kc * es;
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
    if (prec != kFP64) {
      e = scale_exponent(mx);
#pragma unroll
      for (int a = 0; a < NMAX; ++a) v[a] = ldexp(v[a], -e);
    }
  }
  ex[g] = e;
  write_row<NMAX>(prec, 0, v, n, kc, rowp);
}

template <int NMAX>
__global__ void __launch_bounds__(256)
project_kernel(int prec, const double* __restrict__ M, int n, int64_t npair, int prow, int nq,
               int kc, const double* __restrict__ K, const double* __restrict__ w,
               const int32_t* __restrict__ ex, char* __restrict__ Y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nq * 3 * prow) return;
  const int k = (int)(g / (3 * (int64_t)prow));
  const int64_t rem = g - (int64_t)k * 3 * prow;
  const int d = (int)(rem / prow);
  const int64_t q = rem - (int64_t)d * prow;
  const int es = prec == kFP64 ? 8 : (prec == kFP32 ? 4 : 2);
  char* rowp = Y + g * kc * es;
  double m[NMAX];
#pragma unroll
  for (int b = 0; b < NMAX; ++b) m[b] = 0.0;
  double scale = 0.0;
  if (q < npair) {
#pragma unroll
    for (int b = 0; b < NMAX; ++b)
      if (b < n) m[b] = M[((int64_t)d * n + b) * npair + q];
    scale = ldexp(1.0, -ex[(int64_t)d * prow + q]);
    if (d == 2) scale *= w[k];
  }
  const double* Kk = K + (int64_t)k * n * n;
  for (int a = 0; a < n; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NMAX; ++b)
      if (b < n) s += Kk[a * n + b] * m[b];
    write_elem(prec, 1, s * scale, n, a, rowp);
  }
  write_pad(prec, n, kc, rowp);
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
      const int ecol = kF64 ? 0 : m.ex[col] + m.ex[prow + col] + m.ex[2 * prow + col];
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

template <class Op, int WM, int WN>
__global__ void __launch_bounds__(256)
assemble_kernel(AsmMol m) {
  int I, J;
  decode_tile(m.tiles, blockIdx.x, I, J);
  assemble_tile<Op, WM, WN>(m, I, J);
}

// Persistent variant: work groups take (molecule, tile) items from a queue.
template <class Op, int WM, int WN>
__global__ void __launch_bounds__(256)
assemble_queue_kernel(const AsmMol* __restrict__ mols, int nmol, int64_t nitems, unsigned* counter) {
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
    assemble_tile<Op, WM, WN>(m, I, J);
  }
}

__global__ void reset_counter_kernel(unsigned* c) { *c = 0u; }

template <int NMAX>
hipError_t launch_pack_t(int prec, const double* M, int n, int npair, int prow, void* A,
                         int32_t* ex, hipStream_t s) {
  const int kc = operand_kc(prec, n);
  const int64_t total = 3 * (int64_t)prow;
  hipLaunchKernelGGL(pack_kernel<NMAX>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     prec, M, n, (int64_t)npair, prow, kc, static_cast<char*>(A), ex);
  return hipGetLastError();
}

template <int NMAX>
hipError_t launch_project_t(int prec, const double* M, int n, int npair, int prow, int nq,
                            const NodeTables& tb, const int32_t* ex, void* Y, hipStream_t s) {
  const int kc = operand_kc(prec, n);
  const int64_t total = (int64_t)nq * 3 * prow;
  hipLaunchKernelGGL(project_kernel<NMAX>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     prec, M, n, (int64_t)npair, prow, nq, kc, tb.K, tb.w, ex, static_cast<char*>(Y));
  return hipGetLastError();
}

}  // namespace

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

int assemble_tile(int /*prec*/) { return 64; }

hipError_t launch_pack(int prec, const double* M, int n, int npair, int prow, void* A,
                       int32_t* ex, hipStream_t s) {
  if (n <= 16) return launch_pack_t<16>(prec, M, n, npair, prow, A, ex, s);
  if (n <= 32) return launch_pack_t<32>(prec, M, n, npair, prow, A, ex, s);
  if (n <= 48) return launch_pack_t<48>(prec, M, n, npair, prow, A, ex, s);
  return launch_pack_t<64>(prec, M, n, npair, prow, A, ex, s);
}

hipError_t launch_project(int prec, const double* M, int n, int npair, int prow, int nq,
                          const NodeTables& tb, const int32_t* ex, void* Y, hipStream_t s) {
  if (n <= 16) return launch_project_t<16>(prec, M, n, npair, prow, nq, tb, ex, Y, s);
  if (n <= 32) return launch_project_t<32>(prec, M, n, npair, prow, nq, tb, ex, Y, s);
  if (n <= 48) return launch_project_t<48>(prec, M, n, npair, prow, nq, tb, ex, Y, s);
  return launch_project_t<64>(prec, M, n, npair, prow, nq, tb, ex, Y, s);
}

hipError_t launch_assemble(int prec, const AsmMol& m, hipStream_t s) {
  const int64_t ntiles = (int64_t)m.tiles * (m.tiles + 1) / 2;
  const dim3 grid((unsigned)ntiles), block(256);
  switch (prec) {
    case kFP64: hipLaunchKernelGGL((assemble_kernel<OpF64, 2, 2>), grid, block, 0, s, m); break;
    case kFP32: hipLaunchKernelGGL((assemble_kernel<OpF32, 2, 2>), grid, block, 0, s, m); break;
    case kF16X3: hipLaunchKernelGGL((assemble_kernel<OpF16, 2, 2>), grid, block, 0, s, m); break;
    default: hipLaunchKernelGGL((assemble_kernel<OpBF16, 2, 2>), grid, block, 0, s, m); break;
  }
  return hipGetLastError();
}

hipError_t launch_reset_counter(unsigned* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

int assemble_queue_blocks(int /*prec*/, int device) {
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  return cus * 4;
}

hipError_t launch_assemble_queue(int prec, const AsmMol* mols_dev, int nmol, int64_t nitems,
                                 unsigned* counter, int nblocks, hipStream_t s) {
  const dim3 grid((unsigned)nblocks), block(256);
  switch (prec) {
    case kFP64: hipLaunchKernelGGL((assemble_queue_kernel<OpF64, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
    case kFP32: hipLaunchKernelGGL((assemble_queue_kernel<OpF32, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
    case kF16X3: hipLaunchKernelGGL((assemble_queue_kernel<OpF16, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
    default: hipLaunchKernelGGL((assemble_queue_kernel<OpBF16, 2, 2>), grid, block, 0, s, mols_dev, nmol, nitems, counter); break;
  }
  return hipGetLastError();
}

}  // namespace tai
