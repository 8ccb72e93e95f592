// Assembly of B in FP32 on the matrix cores (v_mfma_f32_16x16x4f32): the
// same contraction as the other assembly kernels (Theorem 3.1 in Hadamard
// form, G_{k,d} = M_d^T (K_k M_d), B = (2/sqrt(pi)) sum_k w_k G_{k,0} o
// G_{k,1} o G_{k,2}), organised like the 16-bit persistent kernel:
//
// * A-stationary: each wave keeps the FP32 A_d operand of its 16*RB rows,
//   all three directions and the whole inner length, in VGPRs for a work item.
// * The Y_{k,d} operand of a 16-column block is streamed per node k through a
//   two-deep LDS ring with direct-to-LDS dword loads shared by the eight
//   waves.  One 256-byte fragment holds, in lane order, the 4-byte operand
//   of one MFMA (an inner step of 4), so any inner length that is a multiple
//   of 4 runs without padding; the LDS fragment reads are conflict-free.
// * Per node the three G tiles are multiplied elementwise and accumulated in
//   FP32; every kGroup32 nodes the FP32 sums are added into FP64 partial sums
//   held in wave-private LDS.
// * A finished column block leaves straight from registers: rows for
//   row <= col, 16-byte mirrored columns for row < col.
// * Persistent work groups take (molecule, row panel, column-block range)
//   items from per-XCD queues, as the 16-bit kernel does.
// * With per-node degrees (operands in coefficient form, AsmMol::nk) node k
//   loads and contracts only its first ceil(N_k / 4) inner steps; the Y rows
//   beyond N_k are zero.
#include "tai_internal.h"

#include <cmath>
#include <type_traits>

namespace tai {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr double kTwoOverSqrtPi = 1.1283791670955126;

// Raw buffer resource on a step's base pointer (fourth word: the gfx9 value,
// 32-bit data format, no swizzle or index stride).  The FP64 kernel's Y
// fragments go to LDS through buffer loads: a load into LDS through the
// global segment makes the compiler treat every later LDS read as possibly
// out of order and wait for all of them before each MFMA step (9% of the
// FP64 kernel's time at Nb = 400).
__device__ inline __amdgpu_buffer_rsrc_t y_rsrc(const char* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, 0x7fffffff, 0x00020000);
}
// FP32 accumulation group of quadrature nodes (as in the FP32 tile kernel)
constexpr int kGroup32 = 8;
constexpr int kQueues = kAsm16Queues;
constexpr int kNW32 = 8;  // waves per work group (two per SIMD)

template <int KC, int RB>
struct Cfg32 {
  static constexpr int KC_ = KC, RB_ = RB, NW = kNW32;
  static constexpr int NCH = KC / 4;                   // inner steps of 4
  static constexpr int NT = 64 * NW;
  static constexpr int ROWS = 16 * RB * NW;            // rows per panel
  static constexpr int COLS = 16;                      // columns per block
  static constexpr int NFRAG = 3 * NCH;                // 256-byte fragments per node
  static constexpr int LPW = (NFRAG + NW - 1) / NW;    // loads per wave (some waves one fewer)
  static constexpr int NV = RB * 4;                    // accumulator values per lane
  static constexpr int SUM_BYTES = NW * NV * 64 * 8;
  static constexpr int ITEM_COLS = 512;
  static constexpr int LDS_BYTES = 2 * NFRAG * 256 + SUM_BYTES + 4 * (ROWS + ITEM_COLS);
  static_assert(KC % 4 == 0, "inner length");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

__device__ inline void wait_vmcnt0() { __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Call f(integral_constant<int, c>) for the compile-time count c == v (1 <= v <= N).
template <int N, class F>
__device__ inline void with_steps(int v, F&& f) {
  if constexpr (N == 1) {
    f(std::integral_constant<int, 1>{});
  } else {
    if (v >= N) f(std::integral_constant<int, N>{});
    else with_steps<N - 1>(v, f);
  }
}

template <class C, bool DEG>
__device__ inline void run_item32(const AsmMol& m, int rp, int cb0, int cb1, float* yb0, float* yb1, double* sums,
                                  int* erow_s, int* ecol_s) {
  constexpr int RB = C::RB_, NCH = C::NCH, NT = C::NT, NV = C::NV, ROWS = C::ROWS, COLS = C::COLS;
  constexpr int NW = C::NW, NFRAG = C::NFRAG, LPW = C::LPW;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t prow = m.prow;
  // a rectangular block's columns have their own operand rows and exponents
  const bool rect = m.rect != 0;
  const int64_t pcol = rect ? (int64_t)m.pcol : prow;
  const int32_t* __restrict__ exc = rect ? m.exc : m.ex;
  const int64_t row_wg = (int64_t)rp * ROWS;
  const int64_t row_base = row_wg + wave * 16 * RB;
  const float* __restrict__ Af = static_cast<const float*>(m.A);
  const char* __restrict__ Yb = static_cast<const char*>(m.Y);
  const int nq = m.nq;
  const int64_t npair = m.npair;
  const int64_t ldb = m.ldb;
  float* __restrict__ Bout = static_cast<float*>(m.B);
  float* __restrict__ Tout = static_cast<float*>(rect ? m.Bt : m.B);
  const bool vec_ok = ((ldb & 3) == 0) && ((reinterpret_cast<uintptr_t>(Tout) & 15) == 0);
  double* mysum = sums + wave * NV * 64 + lane;  // value v at mysum[v * 64]
  const int nblk = cb1 - cb0;
  const int64_t col_first = (int64_t)cb0 * COLS;

  for (int i = threadIdx.x; i < ROWS; i += NT) {
    const int64_t row = row_wg + i;
    erow_s[i] = m.ex[row] + m.ex[prow + row] + m.ex[2 * prow + row];
  }
  for (int i = threadIdx.x; i < nblk * COLS; i += NT) {
    const int64_t col = col_first + i;
    ecol_s[i] = exc[col] + exc[pcol + col] + exc[2 * pcol + col] - m.ysh;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) mysum[v * 64] = 0.0;

  // k-invariant A operand: lane l holds A_d[row][4 ch + l/16] for MFMA step ch
  float af[3][RB][NCH];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        af[d][rb][ch] = Af[((int64_t)d * prow + row_base + 16 * rb + r16) * C::KC_ + 4 * ch + kg];
  __syncthreads();  // exponent tables written

  // Y fragment f = d * NCH + ch of a (node, block): lane l loads
  // Y[k][d][col0 + l%16][4 ch + l/16]; wave w loads fragments w, w + NW, ...
  const int64_t node_bytes = 3 * pcol * C::KC_ * 4;
  const int64_t block_bytes = (int64_t)COLS * C::KC_ * 4;
  uint32_t off[LPW];
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    int f = wave + NW * i;
    f = f < NFRAG ? f : 0;
    const int d = f / NCH, ch = f % NCH;
    off[i] = (uint32_t)((((int64_t)d * pcol + col_first + r16) * C::KC_ + 4 * ch + kg) * 4);
  }
  const int T = nblk * nq;
  const int32_t* __restrict__ nkp = DEG ? m.nk : nullptr;
  auto steps_of = [&](int node) { return (DEG && nkp) ? (nkp[node] + 3) / 4 : NCH; };
  int ib = 0, ik = 0;  // (block, node) of the next step to load
  auto issue_next = [&](float* buf) {
    // (global-segment loads here: the buffer form, which helps the FP64
    // kernel, measured 1.4% slower for this one)
    const char* base = Yb + ik * node_bytes + ib * block_bytes;
    const int nch = steps_of(ik);
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const int f = wave + NW * i;
      if (f < NFRAG && f % NCH < nch)
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(base + off[i]), (lds_ptr_t)(buf + f * 64), 4,
                                         0, 0);
    }
    if (++ik == nq) {
      ik = 0;
      ++ib;
    }
  };
  issue_next(yb0);

  v4f acc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};

  typedef __attribute__((address_space(1))) float gfloat;
  typedef __attribute__((address_space(1))) v4f gv4f;
  typedef __attribute__((address_space(1))) char gchar;
  gchar* Bbytes = (gchar*)Bout;
  gchar* Tbytes = (gchar*)Tout;
  const uint32_t ldb4 = (uint32_t)ldb * 4u;
  const int ncol32 = rect ? m.ncol : (int)npair;
  auto finish_block = [&](int fb) {
    const int64_t colu = col_first + (int64_t)fb * COLS;  // uniform first column
    const int ecol = ecol_s[fb * COLS + r16];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int rl0 = wave * 16 * RB + 16 * rb + 4 * kg;
      const int4 er = *reinterpret_cast<const int4*>(erow_s + rl0);
      const int erow[4] = {er.x, er.y, er.z, er.w};
      const int64_t rowu = row_wg + wave * 16 * RB + 16 * rb;  // uniform first row of the block
      const int row0 = 4 * kg;                                 // this lane's first row, relative
      const int dc = (int)(colu - rowu) + r16;                 // col - rowu for this lane
      // rows kept: row - rowu <= lim_row (upper triangle: row <= col);
      // mirrored: row - rowu < lim_mir (row < col); a rectangular block keeps
      // and mirrors every row below its row count
      const int lim_row = rect ? (int)(npair - rowu) - 1 : dc;
      const int lim_mir = rect ? (int)(npair - rowu) : dc;
      float val[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int v = rb * 4 + r;
        val[r] = (float)ldexp(mysum[v * 64] * kTwoOverSqrtPi, erow[r] + ecol);
        mysum[v * 64] = 0.0;
      }
      if ((int)colu + r16 < ncol32) {
        gchar* rbase = Bbytes + (rowu * ldb + colu) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row0 + r <= lim_row) *(gfloat*)(rbase + ((uint32_t)(row0 + r) * ldb4 + (uint32_t)r16 * 4u)) = val[r];
        gchar* mbase = Tbytes + (colu * ldb + rowu) * 4;
        gfloat* dst = (gfloat*)(mbase + ((uint32_t)r16 * ldb4 + (uint32_t)row0 * 4u));
        if (vec_ok && row0 + 3 < lim_mir) {
          *(gv4f*)dst = v4f{val[0], val[1], val[2], val[3]};
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (row0 + r < lim_mir) dst[r] = val[r];
        }
      }
    }
  };
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) mysum[(rb * 4 + r) * 64] += (double)acc[rb][r];
      acc[rb] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  };

  int k = 0, blk = 0;  // (block, node) of the current step
  float* cur = yb0;
  float* nxt = yb1;
  for (int t = 0; t < T; ++t) {
    // this wave's loads of step t have landed; after the barrier everyone's
    // have, and every wave is done with step t-1, whose buffer is reloaded
    wait_vmcnt0();
    __asm__ volatile("s_barrier" ::: "memory");
    const int nch = steps_of(k);  // inner steps of this node (uniform)
    if (t + 1 < T) issue_next(nxt);
    // the node's MFMAs with NC inner steps per direction: fragment (d, ch) of
    // the LDS buffer for g = d * NC + ch, the next fragment read one ahead
    auto node = [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      v4f H[RB], G[RB];
      float b[2];
      b[0] = cur[lane];
#pragma unroll
      for (int g = 0; g < 3 * NC; ++g) {
        const int d = g / NC, ch = g % NC;
        if (g + 1 < 3 * NC) b[(g + 1) & 1] = cur[(((g + 1) / NC) * NCH + (g + 1) % NC) * 64 + lane];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
          G[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[d][rb][ch], b[g & 1],
                                                       ch == 0 ? v4f{0.f, 0.f, 0.f, 0.f} : G[rb], 0, 0, 0);
        if (ch == NC - 1) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            if (d == 0) H[rb] = G[rb];
            else if (d == 1) H[rb] *= G[rb];
            else acc[rb] += H[rb] * G[rb];
          }
        }
      }
    };
    if constexpr (DEG) with_steps<NCH>(nch, node);
    else node(std::integral_constant<int, NCH>{});
    if ((k + 1) % kGroup32 == 0 || k + 1 == nq) flush();
    if (++k == nq) {
      finish_block(blk);
      k = 0;
      ++blk;
    }
    float* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

template <class C, bool DEG>
__global__ void __launch_bounds__(C::NT, 1)
assemble32_kernel(const AsmMol* __restrict__ mols, const int4* __restrict__ items, const int* __restrict__ seg,
                  unsigned* __restrict__ counters) {
  __shared__ float yb0[C::NFRAG * 64];
  __shared__ float yb1[C::NFRAG * 64];
  __shared__ double sums[C::SUM_BYTES / 8];
  __shared__ int erow_s[C::ROWS];
  __shared__ int ecol_s[C::ITEM_COLS];
  __shared__ int item_s;
  const int home = blockIdx.x % kQueues;
  for (int probe = 0; probe < kQueues;) {
    const int qi = (home + probe) % kQueues;
    __syncthreads();  // the previous item is done with every LDS buffer
    if (threadIdx.x == 0) {
      const int i = (int)atomicAdd(counters + qi, 1u);
      item_s = (i < seg[qi + 1] - seg[qi]) ? seg[qi] + i : -1;
    }
    __syncthreads();
    const int it = item_s;
    if (it < 0) {
      ++probe;
      continue;
    }
    const int4 item = items[it];
    const AsmMol m = mols[item.x];
    run_item32<C, DEG>(m, item.y, item.z, item.w, yb0, yb1, sums, erow_s, ecol_s);
  }
}

// ---------------------------------------------------------------------------
// FP64 form (v_mfma_f64_16x16x4f64): the same persistent design with 1 KB
// fragments of two doubles per lane (dwordx4 loads), two MFMAs per fragment,
// so inner lengths that are multiples of 8 run without padding.  Products
// and sums are FP64 throughout, as in the FP64 tile kernel; the accumulators
// stay in registers and no exponent scaling applies.
// ---------------------------------------------------------------------------
typedef double v2d __attribute__((ext_vector_type(2)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <int KC, int RB>
struct Cfg64 {
  static constexpr int KC_ = KC, RB_ = RB, NW = kNW32;
  static constexpr int NCH = KC / 8;                   // 1 KB fragments per direction (8 inner indices)
  static constexpr int NT = 64 * NW;
  static constexpr int ROWS = 16 * RB * NW;
  static constexpr int COLS = 16;
  static constexpr int NFRAG = 3 * NCH;
  static constexpr int LPW = (NFRAG + NW - 1) / NW;
  static_assert(KC % 8 == 0, "inner length");
  static_assert(2 * NFRAG * 1024 <= 160 * 1024, "LDS");
};

template <class C, bool DEG>
__device__ inline void run_item64(const AsmMol& m, int rp, int cb0, int cb1, uint4* yb0, uint4* yb1) {
  constexpr int RB = C::RB_, NCH = C::NCH, NW = C::NW, NFRAG = C::NFRAG, LPW = C::LPW, ROWS = C::ROWS;
  constexpr int COLS = C::COLS;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t prow = m.prow;
  const int64_t row_wg = (int64_t)rp * ROWS;
  const int64_t row_base = row_wg + wave * 16 * RB;
  const double* __restrict__ Ad = static_cast<const double*>(m.A);
  const char* __restrict__ Yb = static_cast<const char*>(m.Y);
  const int nq = m.nq;
  const int64_t ldb = m.ldb;
  const int npair32 = (int)m.npair;
  // a rectangular block: its own column operand rows, every entry, mirror to Bt
  const bool rect = m.rect != 0;
  const int64_t pcol = rect ? (int64_t)m.pcol : prow;
  const int ncol32 = rect ? m.ncol : npair32;
  const int nblk = cb1 - cb0;
  const int64_t col_first = (int64_t)cb0 * COLS;

  // k-invariant A operand: lane l holds A_d[row][8 ch + 2 (l/16) + {0, 1}]
  v2d af[3][RB][NCH];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        af[d][rb][ch] = *(const __attribute__((address_space(1))) v2d*)(
            Ad + ((int64_t)d * prow + row_base + 16 * rb + r16) * C::KC_ + 8 * ch + 2 * kg);

  const int64_t node_bytes = 3 * pcol * C::KC_ * 8;
  const int64_t block_bytes = (int64_t)COLS * C::KC_ * 8;
  uint32_t off[LPW];
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    int f = wave + NW * i;
    f = f < NFRAG ? f : 0;
    const int d = f / NCH, ch = f % NCH;
    off[i] = (uint32_t)((((int64_t)d * pcol + col_first + r16) * C::KC_ + 8 * ch + 2 * kg) * 8);
  }
  const int T = nblk * nq;
  const int32_t* __restrict__ nkp = DEG ? m.nk : nullptr;
  auto steps_of = [&](int node) { return (DEG && nkp) ? (nkp[node] + 7) / 8 : NCH; };
  int ib = 0, ik = 0;
  auto issue_next = [&](uint4* buf) {
    const __amdgpu_buffer_rsrc_t rs = y_rsrc(Yb + ik * node_bytes + ib * block_bytes);
    const int nch = steps_of(ik);
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const int f = wave + NW * i;
      if (f < NFRAG && f % NCH < nch)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)(buf + f * 64), 16, off[i], 0, 0, 0);
    }
    if (++ik == nq) {
      ik = 0;
      ++ib;
    }
  };
  issue_next(yb0);

  v4d acc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = v4d{0.0, 0.0, 0.0, 0.0};

  typedef __attribute__((address_space(1))) double gdouble;
  gdouble* Bd = (gdouble*)static_cast<double*>(m.B);
  gdouble* Td = (gdouble*)static_cast<double*>(rect ? m.Bt : m.B);
  // lane l holds column col0 + l%16 and rows kg + 4 r of each 16-row block
  auto finish_block = [&](int fb) {
    const int64_t colu = col_first + (int64_t)fb * COLS;
    const int col = (int)colu + r16;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t rowu = row_wg + wave * 16 * RB + 16 * rb;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (int)rowu + kg + 4 * r;
        const double v = acc[rb][r] * kTwoOverSqrtPi;
        if (rect) {
          if (col < ncol32 && row < npair32) {
            Bd[(int64_t)row * ldb + col] = v;
            Td[(int64_t)col * ldb + row] = v;
          }
        } else if (col < npair32 && row <= col) {
          Bd[(int64_t)row * ldb + col] = v;
          if (row < col) Bd[(int64_t)col * ldb + row] = v;
        }
      }
      acc[rb] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  };

  int k = 0, blk = 0;
  uint4* cur = yb0;
  uint4* nxt = yb1;
  for (int t = 0; t < T; ++t) {
    wait_vmcnt0();
    __asm__ volatile("s_barrier" ::: "memory");
    const int nch = steps_of(k);
    if (t + 1 < T) issue_next(nxt);
    auto node = [&](auto nc) {
      constexpr int NC = decltype(nc)::value;
      v4d H[RB], G[RB];
      v2d b[2];
      b[0] = *reinterpret_cast<const v2d*>(cur + lane);
#pragma unroll
      for (int g = 0; g < 3 * NC; ++g) {
        const int d = g / NC, ch = g % NC;
        if (g + 1 < 3 * NC)
          b[(g + 1) & 1] = *reinterpret_cast<const v2d*>(cur + (((g + 1) / NC) * NCH + (g + 1) % NC) * 64 + lane);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          v4d x = __builtin_amdgcn_mfma_f64_16x16x4f64(af[d][rb][ch].x, b[g & 1].x,
                                                       ch == 0 ? v4d{0.0, 0.0, 0.0, 0.0} : G[rb], 0, 0, 0);
          G[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[d][rb][ch].y, b[g & 1].y, x, 0, 0, 0);
        }
        if (ch == NC - 1) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            if (d == 0) H[rb] = G[rb];
            else if (d == 1) H[rb] *= G[rb];
            else acc[rb] += H[rb] * G[rb];
          }
        }
      }
    };
    if constexpr (DEG) with_steps<NCH>(nch, node);
    else node(std::integral_constant<int, NCH>{});
    if (++k == nq) {
      finish_block(blk);
      k = 0;
      ++blk;
    }
    uint4* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
}

template <class C, bool DEG>
__global__ void __launch_bounds__(C::NT, 1)
assemble64_kernel(const AsmMol* __restrict__ mols, const int4* __restrict__ items, const int* __restrict__ seg,
                  unsigned* __restrict__ counters) {
  __shared__ uint4 yb0[C::NFRAG * 64];
  __shared__ uint4 yb1[C::NFRAG * 64];
  __shared__ int item_s;
  const int home = blockIdx.x % kQueues;
  for (int probe = 0; probe < kQueues;) {
    const int qi = (home + probe) % kQueues;
    __syncthreads();  // the previous item is done with every LDS buffer
    if (threadIdx.x == 0) {
      const int i = (int)atomicAdd(counters + qi, 1u);
      item_s = (i < seg[qi + 1] - seg[qi]) ? seg[qi] + i : -1;
    }
    __syncthreads();
    const int it = item_s;
    if (it < 0) {
      ++probe;
      continue;
    }
    const int4 item = items[it];
    const AsmMol m = mols[item.x];
    run_item64<C, DEG>(m, item.y, item.z, item.w, yb0, yb1);
  }
}

template <int KC, int RB>
hipError_t launch64(bool deg, const AsmMol* mols, const int4* items, const int* seg, unsigned* counters, int nblocks,
                    hipStream_t s) {
  if (deg)
    hipLaunchKernelGGL((assemble64_kernel<Cfg64<KC, RB>, true>), dim3(nblocks), dim3(Cfg64<KC, RB>::NT), 0, s, mols,
                       items, seg, counters);
  else
    hipLaunchKernelGGL((assemble64_kernel<Cfg64<KC, RB>, false>), dim3(nblocks), dim3(Cfg64<KC, RB>::NT), 0, s, mols,
                       items, seg, counters);
  return hipGetLastError();
}

// row blocks per wave: the FP64 A operand takes 24 VGPRs per row block and
// 8 inner indices
constexpr int rb64(int kc) { return kc <= 8 ? 4 : (kc <= 40 ? 2 : 1); }

template <int KC, int RB>
hipError_t launch32(bool deg, const AsmMol* mols, const int4* items, const int* seg, unsigned* counters, int nblocks,
                    hipStream_t s) {
  if (deg)
    hipLaunchKernelGGL((assemble32_kernel<Cfg32<KC, RB>, true>), dim3(nblocks), dim3(Cfg32<KC, RB>::NT), 0, s, mols,
                       items, seg, counters);
  else
    hipLaunchKernelGGL((assemble32_kernel<Cfg32<KC, RB>, false>), dim3(nblocks), dim3(Cfg32<KC, RB>::NT), 0, s, mols,
                       items, seg, counters);
  return hipGetLastError();
}

// four row blocks per wave while the A operand leaves room (inner length up
// to 40), two beyond
constexpr int rb32(int kc) { return kc <= 40 ? 4 : 2; }

}  // namespace

int asm32_rows(int kc) { return 16 * rb32(kc) * kNW32; }
int asm64_rows(int kc) { return 16 * rb64(kc) * kNW32; }

hipError_t launch_assemble64(int kc, bool deg, const AsmMol* mols_dev, const int4* items_dev, const int* seg_dev,
                             unsigned* counters, int nblocks, hipStream_t s) {
  switch (kc) {
    case 8: return launch64<8, rb64(8)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 16: return launch64<16, rb64(16)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 24: return launch64<24, rb64(24)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 32: return launch64<32, rb64(32)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 40: return launch64<40, rb64(40)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 48: return launch64<48, rb64(48)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 56: return launch64<56, rb64(56)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 64: return launch64<64, rb64(64)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_assemble32(int kc, bool deg, const AsmMol* mols_dev, const int4* items_dev, const int* seg_dev,
                             unsigned* counters, int nblocks, hipStream_t s) {
  switch (kc) {
    case 8: return launch32<8, rb32(8)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 16: return launch32<16, rb32(16)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 24: return launch32<24, rb32(24)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 32: return launch32<32, rb32(32)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 40: return launch32<40, rb32(40)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 48: return launch32<48, rb32(48)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 56: return launch32<56, rb32(56)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    case 64: return launch32<64, rb32(64)>(deg, mols_dev, items_dev, seg_dev, counters, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tai
