// Assembly of B for the 16-bit split arithmetics (F16X3, BF16X3, BF16X6):
// the same contraction as the generic kernel (Theorem 3.1 in Hadamard form,
// G_{k,d} = M_d^T (K_k M_d), B = (2/sqrt(pi)) sum_k w_k G_{k,0} o G_{k,1} o G_{k,2}),
// organised around the MI355X matrix cores:
//
// * A-stationary: each wave keeps the A_d operand (the k-invariant moments)
//   of its 16*RB rows, all three directions and the whole inner dimension,
//   in VGPRs for a whole work item.  RB is chosen per inner length so that
//   the operand, the Hadamard product and the FP32 accumulators fit in the
//   256 architectural VGPRs (no AGPR round trips before each MFMA).
// * The Y_{k,d} operand of one 32-column block is streamed per k through LDS
//   with direct-to-LDS buffer loads (buffer_load_dwordx4 ... lds), NBUF-buffered so the
//   loads run NBUF-1 nodes ahead, and shared by the four waves.  Each 1 KB
//   fragment holds the 16-byte MFMA operand of every lane in lane order, so
//   the fragment reads are bank-conflict-free.  Each wave issues the same
//   number of loads per node, so the waits count loads exactly.
// * Per k the three G tiles come out of v_mfma_f32_16x16x32_{f16,bf16}, are
//   multiplied elementwise and accumulated in FP32; every kGroup nodes the
//   FP32 sums are added into FP64 partial sums held in wave-private LDS.
// * A finished 32-column block goes through an LDS tile and leaves as
//   coalesced rows (entries row <= col) and mirrored columns (row < col).
// * Persistent work groups take (molecule, row panel, column-block range)
//   items from a queue ordered column-chunk-major, so work groups running at
//   the same time read the same Y blocks from L2.
#include "tai_internal.h"

#include <cmath>
#include <cstdlib>
#include <type_traits>

namespace tai {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr double kTwoOverSqrtPi = 1.1283791670955126;
// fourth word of a raw buffer resource on gfx9 parts (32-bit data format,
// no swizzle, no index stride)
constexpr int kBufferWord3 = 0x00020000;
// FP32 accumulation group of quadrature nodes: sixteen keep the FP32 part of
// the error well below the split's own (F16X3 normwise 4e-8 at Nb = 400)
// and flush the FP64 partial sums half as often as eight.
constexpr int kGroup16 = 16;
constexpr int kQueues = kAsm16Queues;

// Compile-time shape: NW waves per work group, RB row blocks of 16 per wave,
// CB column blocks of 16 per item block, an LDS ring of NBUF steps of NPS
// quadrature nodes each (two nodes per step halve the waits, barriers and
// load issues per node; the ring slot doubles).
template <int KC, int Q, int NW, int RB, int CB, int NBUF, int NPS = 1>
struct Cfg16 {
  static constexpr int KC_ = KC, Q_ = Q, NW_ = NW, RB_ = RB, CB_ = CB, NBUF_ = NBUF, NPS_ = NPS;
  static constexpr int NCH = KC / 32;                    // 32-wide inner chunks
  static constexpr int U = Q >= kX6Key ? NCH - 3 * (Q - kX6Key) : NCH - Q;  // distinct A fragments
  static constexpr int NT = 64 * NW;                     // threads per work group
  static constexpr int ROWS = 16 * RB * NW;              // rows per panel
  static constexpr int COLS = 16 * CB;                   // columns per block
  static constexpr int NFRAG_NODE = 3 * CB * NCH;        // 1 KB fragments per node
  static constexpr int NFRAG = NFRAG_NODE * NPS;         // per step
  static constexpr int LPW_HI = (NFRAG + NW - 1) / NW;   // loads of waves < N_HI
  static constexpr int LPW_LO = NFRAG / NW;              // loads of the others
  static constexpr int N_HI = NFRAG % NW == 0 ? NW : NFRAG % NW;
  static constexpr int NV = RB * CB * 4;                 // accumulator values per lane
  static constexpr int SUM_BYTES = NW * NV * 64 * 8;     // FP64 partial sums, all waves
  static constexpr int ITEM_COLS = COLS * (512 / COLS);  // columns of the longest item
  static constexpr int LDS_BYTES = NBUF * NFRAG * 1024 + SUM_BYTES + 4 * (ROWS + ITEM_COLS);
  static_assert(NBUF == 2 || NBUF == 3, "ring depth");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS");
};

// A fragment register index of MFMA chunk ch, and the K chunk a register
// fragment is loaded from.  X3 layouts: chunks Q..2Q-1 repeat 0..Q-1.  BF16X6
// layouts (Q = kX6Key + Q6): in range r < Q6 the six segment chunks 6r + s
// use fragments 3r + {0, 0, 1, 0, 1, 2}[s]; later chunks follow.
template <int Q> __device__ constexpr int a_slot(int ch) {
  if constexpr (Q >= kX6Key) {
    constexpr int Q6 = Q - kX6Key;
    return ch < 6 * Q6 ? 3 * (ch / 6) + (ch % 6 == 5 ? 2 : (ch % 6 == 2 || ch % 6 == 4) ? 1 : 0)
                       : 3 * Q6 + (ch - 6 * Q6);
  } else {
    return ch < Q ? ch : ch - Q;
  }
}
template <int Q> __device__ constexpr int a_chunk(int u) {
  if constexpr (Q >= kX6Key) {
    constexpr int Q6 = Q - kX6Key;
    return u < 3 * Q6 ? 6 * (u / 3) + (u % 3 == 0 ? 0 : (u % 3 == 1 ? 2 : 5)) : 6 * Q6 + (u - 3 * Q6);
  } else {
    return u < Q ? u : u + Q;
  }
}

template <int N>
__device__ inline void wait_vmcnt() {
  __asm__ volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ inline v4f mma(v8h a, v8h b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
__device__ inline v4f mma(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// Direct-to-LDS loads of the Y fragments of one step.  Fragment
// f = (d*CB + c)*NCH + ch holds, for lane l, the 16 bytes
// Y[k][d][col0 + 16c + l%16][32ch + 8(l/16) .. +8].  Wave w loads fragments
// w, w + NW, ... (LPW_HI of them for w < N_HI, else LPW_LO), the same count
// for every step, so that a wave's wait can count its own loads.  The byte
// offsets of a wave's fragments are fixed for an item (off); a step's
// (node, column block) only moves the uniform base pointer.
template <class C>
struct YLoads {
  uint32_t off[C::LPW_HI];
  __device__ void init(int64_t prow, int64_t col0, int64_t node_bytes, int wave, int lane) {
    const int r16 = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int i = 0; i < C::LPW_HI; ++i) {
      int f = wave + C::NW_ * i;
      f = f < C::NFRAG ? f : 0;
      const int j = f / C::NFRAG_NODE, g = f % C::NFRAG_NODE;
      const int ch = g % C::NCH;
      const int c = (g / C::NCH) % C::CB_;
      const int d = g / (C::NCH * C::CB_);
      off[i] = (uint32_t)(j * node_bytes + (((int64_t)d * prow + col0 + 16 * c + r16) * C::KC_ + 32 * ch + 8 * kg) * 2);
    }
  }
  // Buffer loads (a resource built on the step's base pointer, the fixed
  // offsets per lane): a load into LDS through the global segment would
  // make the compiler count every later LDS read as possibly out of order,
  // so each fragment read would wait for all of them (lgkmcnt(0)) instead of
  // only the one the MFMAs need.
  __device__ void issue(const char* base, uint4* buf, int wave) const {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, 0x7fffffff, kBufferWord3);
#pragma unroll
    for (int i = 0; i < C::LPW_HI; ++i) {
      const int f = wave + C::NW_ * i;
      if (f < C::NFRAG) __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)(buf + f * 64), 16, off[i], 0, 0, 0);
    }
  }
};

// Wait until this wave's loads of the current step have landed.  Loads
// complete in issue order, so with the next step's loads already issued
// (ring of 3) it is enough to leave this wave's per-step count outstanding.
template <class C>
__device__ inline void wait_step(bool next_issued, int wave) {
  if constexpr (C::NBUF_ == 3) {
    if (next_issued) {
      if (wave < C::N_HI) wait_vmcnt<C::LPW_HI>();
      else wait_vmcnt<C::LPW_LO>();
      return;
    }
  }
  wait_vmcnt<0>();
}

// The MFMA work of the NPS nodes of one step on one column block: for each
// node, the three G_d tiles from the A fragments in registers and the Y
// fragments in buffer cur, then acc += G_0 o G_1 o G_2 (w_k is folded into
// Y of direction 2), then node_end(j).  The Y fragments are read one chunk
// ahead of the MFMAs that use them (two register sets), across the node
// boundary too, so the LDS latency hides behind the RB*CB MFMAs of the
// current chunk and the next node's first reads overlap this node's
// Hadamard products and sum flushes.
template <class C, bool BF, class NodeEnd>
__device__ inline void step_mfma(const uint4* cur,
                                 const typename std::conditional<BF, v8bf, v8h>::type (&af)[3][C::RB_][C::U],
                                 v4f (&acc)[C::RB_][C::CB_], int lane, NodeEnd&& node_end) {
  using Frag = typename std::conditional<BF, v8bf, v8h>::type;
  constexpr int RB = C::RB_, CB = C::CB_, NCH = C::NCH, NF = 3 * NCH, NFS = NF * C::NPS_;
  // fragment f of the step: node f / NF, then ((d * CB + c) * NCH + ch) within the node
  auto frag = [&](int f, int c) {
    const int j = f / NF, g = f % NF;
    return *reinterpret_cast<const Frag*>(cur + (j * C::NFRAG_NODE + ((g / NCH) * CB + c) * NCH + g % NCH) * 64 + lane);
  };
  Frag bf[2][CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) bf[0][c] = frag(0, c);
  v4f H[RB][CB], G[RB][CB];
#pragma unroll
  for (int f = 0; f < NFS; ++f) {
    const int g = f % NF, d = g / NCH, ch = g % NCH;
    if (f + 1 < NFS) {
#pragma unroll
      for (int c = 0; c < CB; ++c) bf[(f + 1) & 1][c] = frag(f + 1, c);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int c = 0; c < CB; ++c)
        G[rb][c] = mma(af[d][rb][a_slot<C::Q_>(ch)], bf[f & 1][c], ch == 0 ? v4f{0.f, 0.f, 0.f, 0.f} : G[rb][c]);
    if (ch == NCH - 1) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          if (d == 0) H[rb][c] = G[rb][c];
          else if (d == 1) H[rb][c] *= G[rb][c];
          else acc[rb][c] += H[rb][c] * G[rb][c];
        }
      if (d == 2) node_end(f / NF);
    }
  }
}

// One work item: the rows of panel rp against column blocks [cb0, cb1).
// The steps (column block, node) run as one stream through the LDS ring, so
// the loads of the next block start while the current one finishes.  Each
// wave owns its rows: FP32 sums over kGroup16 nodes are added into its FP64
// partial sums in LDS, and a finished block leaves straight from registers
// (rows for row <= col, the mirror for row < col) without a work-group barrier.
template <class C, bool BF>
__device__ inline void run_item(const AsmMol& m, int rp, int cb0, int cb1, uint4* yb0, uint4* yb1, uint4* yb2,
                                double* sums, int* erow_s, int* ecol_s) {
  using Frag = typename std::conditional<BF, v8bf, v8h>::type;
  constexpr int RB = C::RB_, CB = C::CB_, U = C::U, NBUF = C::NBUF_;
  constexpr int ROWS = C::ROWS, COLS = C::COLS, NT = C::NT, NV = C::NV;
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
  const char* __restrict__ Ab = static_cast<const char*>(m.A);
  const char* __restrict__ Yb = static_cast<const char*>(m.Y);
  const int nq = m.nq;
  const int64_t npair = m.npair;
  const int64_t ldb = m.ldb;
  float* __restrict__ Bout = static_cast<float*>(m.B);
  float* __restrict__ Tout = static_cast<float*>(rect ? m.Bt : m.B);
  const bool vec_ok = ((ldb & 3) == 0) && ((reinterpret_cast<uintptr_t>(Tout) & 15) == 0);
  double* mysum = sums + wave * NV * 64 + lane;   // value v at mysum[v * 64]
  const int nblk = cb1 - cb0;
  const int64_t col_first = (int64_t)cb0 * COLS;

  // summed power-of-two exponents of the panel's rows and the item's columns
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

  // k-invariant A operand of this wave's rows, all directions
  Frag af[3][RB][U];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t row = (int64_t)d * prow + row_base + 16 * rb + r16;
        af[d][rb][u] = *(const __attribute__((address_space(1))) Frag*)(Ab + (row * C::KC_ + 32 * a_chunk<C::Q_>(u) + 8 * kg) * 2);
      }
  __syncthreads();  // exponent tables written

  // step t = (block t / nq, node t % nq); its Y base pointer
  const int64_t node_bytes = 3 * pcol * C::KC_ * 2;
  const int64_t block_bytes = (int64_t)COLS * C::KC_ * 2;
  const int T = nblk * (nq / C::NPS_);
  YLoads<C> yl;
  yl.init(pcol, col_first, node_bytes, wave, lane);
  int ib = 0, ik = 0;  // (block, node) of the next step to load
  auto issue_next = [&](uint4* buf) {
    yl.issue(Yb + ik * node_bytes + ib * block_bytes, buf, wave);
    ik += C::NPS_;
    if (ik == nq) {
      ik = 0;
      ++ib;
    }
  };
  issue_next(yb0);
  if (NBUF == 3) issue_next(yb1);

  v4f acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[rb][c] = v4f{0.f, 0.f, 0.f, 0.f};
  int k = 0, blk = 0;  // (block, node) of the current step

  // Output addressing: a uniform base per (row block, column block) plus
  // 32-bit per-lane byte offsets, and 32-bit row/column tests relative to
  // the block, so that nothing 64-bit per lane stays live across the node
  // loop.  Stores go through the global address space (a generic pointer
  // could alias LDS and would make the compiler drain the Y loads).
  typedef __attribute__((address_space(1))) float gfloat;
  typedef __attribute__((address_space(1))) v4f gv4f;
  typedef __attribute__((address_space(1))) char gchar;
  gchar* Bbytes = (gchar*)Bout;
  gchar* Tbytes = (gchar*)Tout;
  const uint32_t ldb4 = (uint32_t)ldb * 4u;
  const int ncol32 = rect ? m.ncol : (int)npair;
  auto finish_block = [&](int fb) {
    const int64_t col0 = col_first + (int64_t)fb * COLS;
    int ecol[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) ecol[c] = ecol_s[fb * COLS + 16 * c + r16];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int rl0 = wave * 16 * RB + 16 * rb + 4 * kg;
      const int4 er = *reinterpret_cast<const int4*>(erow_s + rl0);
      const int erow[4] = {er.x, er.y, er.z, er.w};
      const int64_t rowu = row_wg + wave * 16 * RB + 16 * rb;  // uniform first row of the block
      const int row0 = 4 * kg;                                 // this lane's first row, relative
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int64_t colu = col0 + 16 * c;                    // uniform first column
        const int dc = (int)(colu - rowu) + r16;               // col - rowu for this lane
        // rows kept: row - rowu <= lim_row (upper triangle: row <= col);
        // mirrored: row - rowu < lim_mir (row < col); a rectangular block
        // keeps and mirrors every row below its row count
        const int lim_row = rect ? (int)(npair - rowu) - 1 : dc;
        const int lim_mir = rect ? (int)(npair - rowu) : dc;
        float val[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int v = (rb * CB + c) * 4 + r;
          val[r] = (float)ldexp(mysum[v * 64] * kTwoOverSqrtPi, erow[r] + ecol[c]);
          mysum[v * 64] = 0.0;
        }
        if ((int)colu + r16 < ncol32) {
          // rows: B[row][col]
          gchar* rbase = Bbytes + (rowu * ldb + colu) * 4;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (row0 + r <= lim_row) *(gfloat*)(rbase + ((uint32_t)(row0 + r) * ldb4 + (uint32_t)r16 * 4u)) = val[r];
          // mirror: B[col][row .. row+3] (Bt[col][row ..] for a rectangular block)
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
    }
  };

  // FP32 group sums into the FP64 partial sums.  With a two-deep ring a
  // wave has no loads in flight between its barrier and its next load issue,
  // so the flush of a group that ends a step waits for that point and uses
  // LDS atomic adds (ds_add_f64, no return value): no read-modify-write
  // round trip, and the wait the compiler puts before an LDS atomic (for
  // loads into LDS) finds nothing outstanding.  Elsewhere the flush is a
  // plain read-modify-write.  Each lane owns its addresses, so the additions
  // keep their node order either way.
  constexpr bool kDeferFlush = NBUF == 2;
  bool flush_pending = false;
  auto flush = [&](auto atomic) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          double* sp = mysum + ((rb * CB + c) * 4 + r) * 64;
          if constexpr (decltype(atomic)::value) atomicAdd(sp, (double)acc[rb][c][r]);
          else *sp += (double)acc[rb][c][r];
        }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[rb][c] = v4f{0.f, 0.f, 0.f, 0.f};
    flush_pending = false;
  };

  // With nq a multiple of NPS and at least NBUF * NPS (the host routes other
  // node counts to another shape or the generic kernel) a block ends at most
  // once per group of NBUF steps, and the next block's first flush comes more
  // than NBUF-1 steps later, so the finished block's sums can wait for the
  // end of the group.
  int done = -1;  // block finished within the current group
  auto step = [&](int t, const uint4* cur, uint4* nxt) {
    // Every wave waits for its own loads of step t, then all waves meet:
    // step t is in LDS for everyone and every wave has consumed step t-1,
    // whose buffer the loads below reuse.  A plain s_barrier (memory clobber
    // for the compiler) instead of __syncthreads, whose fence would also
    // drain the loads still in flight.
    wait_step<C>(t + 1 < T, wave);
    __asm__ volatile("s_barrier" ::: "memory");
    if (flush_pending) flush(std::true_type{});
    if (t + NBUF - 1 < T) issue_next(nxt);
    step_mfma<C, BF>(cur, af, acc, lane, [&](int j) {
      if ((k + 1) % kGroup16 == 0 || k + 1 == nq) {
        // a group that ends the step waits for the next step's start
        if (kDeferFlush && j == C::NPS_ - 1) flush_pending = true;
        else flush(std::false_type{});
      }
      if (++k == nq) {
        done = blk;
        k = 0;
        ++blk;
      }
    });
  };

  if constexpr (NBUF == 3) {
    for (int t = 0; t < T; t += 3) {
      step(t, yb0, yb2);
      if (t + 1 < T) step(t + 1, yb1, yb0);
      if (t + 2 < T) step(t + 2, yb2, yb1);
      if (done >= 0) {
        if (flush_pending) flush(std::false_type{});
        finish_block(done);
        done = -1;
      }
    }
  } else {
    for (int t = 0; t < T; t += 2) {
      step(t, yb0, yb1);
      if (t + 1 < T) step(t + 1, yb1, yb0);
      if (done >= 0) {
        if (flush_pending) flush(std::false_type{});
        finish_block(done);
        done = -1;
      }
    }
  }
}

// Two waves per SIMD: one work group of 8 waves, or two of 4.
// Work groups are dealt to the 8 XCDs round-robin by index, so work group b
// drains queue b % 8 first: queue x holds the column runs x, x + 8, ... of
// every molecule, and the work groups sharing an XCD's L2 share their Y
// blocks.  A drained queue sends the work group on to the next one.
template <class C, bool BF>
__global__ void __launch_bounds__(C::NT, C::NW_ >= 8 ? 1 : 8 / C::NW_)
assemble16_kernel(const AsmMol* __restrict__ mols, const int4* __restrict__ items, const int* __restrict__ seg,
                  unsigned* __restrict__ counters) {
  __shared__ uint4 yb0[C::NFRAG * 64];
  __shared__ uint4 yb1[C::NFRAG * 64];
  __shared__ uint4 yb2[C::NBUF_ == 3 ? C::NFRAG * 64 : 1];
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
    run_item<C, BF>(m, item.y, item.z, item.w, yb0, yb1, yb2, sums, erow_s, ecol_s);
  }
}

template <class C>
hipError_t launch_shape(bool bf, const AsmMol* mols, const int4* items, const int* seg, unsigned* counters,
                        int nblocks, hipStream_t s) {
  if (bf)
    hipLaunchKernelGGL((assemble16_kernel<C, true>), dim3(nblocks), dim3(C::NT), 0, s, mols, items, seg, counters);
  else
    hipLaunchKernelGGL((assemble16_kernel<C, false>), dim3(nblocks), dim3(C::NT), 0, s, mols, items, seg, counters);
  return hipGetLastError();
}

template <class C>
int resident_wgs() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&assemble16_kernel<C, false>),
                                                    C::NT, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

using LaunchFn = hipError_t (*)(bool, const AsmMol*, const int4*, const int*, unsigned*, int, hipStream_t);
struct ShapeEntry {
  int kc, q, nw, rb, cb, nbuf, nps;
  LaunchFn launch;
  int (*occupancy)();
};

#define TAI_S16(KC, Q, NW, RB, CB, NBUF) \
  {KC, Q, NW, RB, CB, NBUF, 1, &launch_shape<Cfg16<KC, Q, NW, RB, CB, NBUF>>, &resident_wgs<Cfg16<KC, Q, NW, RB, CB, NBUF>>}
#define TAI_S16P(KC, Q, NW, RB, CB, NBUF, NPS)                                   \
  {KC, Q, NW, RB, CB, NBUF, NPS, &launch_shape<Cfg16<KC, Q, NW, RB, CB, NBUF, NPS>>, \
   &resident_wgs<Cfg16<KC, Q, NW, RB, CB, NBUF, NPS>>}

// Per inner length (kc) and duplicated chunk count (q): the shapes that fit
// the register file (A operand 12*RB*U VGPRs plus 12*RB*CB for the
// accumulators) and the LDS, in order of preference.
const ShapeEntry kShapes[] = {
    TAI_S16(32, 0, 8, 4, 2, 3),   TAI_S16(32, 0, 8, 4, 1, 3),
    TAI_S16(64, 0, 8, 4, 1, 3),   TAI_S16(64, 0, 8, 3, 2, 2),
    TAI_S16(96, 0, 8, 4, 1, 3),   TAI_S16(96, 0, 8, 3, 2, 2),
    TAI_S16P(96, 1, 8, 4, 1, 2, 2),
    TAI_S16(96, 1, 8, 4, 1, 3),   TAI_S16(96, 1, 8, 3, 2, 2),   TAI_S16(96, 1, 4, 4, 1, 3),
    TAI_S16(96, 1, 4, 2, 1, 3),   TAI_S16(96, 1, 4, 2, 2, 2),
    TAI_S16(128, 0, 8, 2, 2, 3),  TAI_S16(128, 0, 8, 3, 1, 3),
    TAI_S16P(128, 1, 8, 4, 1, 2, 2), TAI_S16P(128, 1, 8, 4, 1, 3, 2),
    TAI_S16(128, 1, 4, 4, 1, 3),  TAI_S16(128, 1, 8, 4, 1, 3),  TAI_S16(128, 1, 4, 4, 1, 2),
    TAI_S16(128, 1, 4, 3, 1, 3),  TAI_S16(128, 1, 8, 2, 2, 3),  TAI_S16(128, 1, 4, 2, 1, 3),
    TAI_S16(160, 0, 8, 2, 2, 3),  TAI_S16(160, 0, 8, 1, 2, 3),
    TAI_S16(160, 1, 8, 2, 2, 3),  TAI_S16(160, 1, 8, 3, 1, 3),
    TAI_S16(192, 0, 8, 2, 2, 2),  TAI_S16(192, 0, 8, 1, 2, 3),
    TAI_S16(192, 1, 8, 2, 2, 2),  TAI_S16(192, 2, 8, 2, 2, 2),
    TAI_S16P(192, kX6Key + 1, 8, 4, 1, 2, 2),
    TAI_S16(192, kX6Key + 1, 8, 4, 1, 3), TAI_S16(192, kX6Key + 1, 8, 3, 1, 3),
    TAI_S16(224, 0, 8, 1, 2, 2),  TAI_S16(256, 0, 8, 1, 2, 2),
    TAI_S16P(256, kX6Key + 1, 8, 2, 1, 2, 2),
    TAI_S16(256, kX6Key + 1, 8, 2, 1, 3), TAI_S16(256, kX6Key + 1, 8, 2, 1, 2),
    TAI_S16P(288, kX6Key + 1, 8, 2, 1, 2, 2),
    TAI_S16(288, kX6Key + 1, 8, 2, 1, 3), TAI_S16(288, kX6Key + 1, 8, 1, 2, 2),
    TAI_S16(352, kX6Key + 1, 8, 1, 1, 2),
    TAI_S16(288, 0, 8, 1, 2, 2),  TAI_S16(320, 0, 8, 1, 2, 2),
    TAI_S16(352, 0, 8, 1, 1, 2),
};
#undef TAI_S16
#undef TAI_S16P

Asm16Shape to_shape(int id) {
  const ShapeEntry& e = kShapes[id];
  Asm16Shape sh;
  sh.id = id;
  sh.waves = e.nw;
  sh.rb = e.rb;
  sh.cb = e.cb;
  sh.nbuf = e.nbuf;
  sh.nps = e.nps;
  sh.rows = 16 * e.rb * e.nw;
  sh.cols = 16 * e.cb;
  sh.wgs_per_cu = 1;  // asm16_shape asks the runtime
  sh.kc_key = e.kc;
  sh.q_key = e.q;
  return sh;
}

}  // namespace

int asm16_max_kc() { return 352; }

int asm16_shapes(int kc, int q, Asm16Shape* out, int cap) {
  int n = 0;
  for (int i = 0; i < (int)(sizeof(kShapes) / sizeof(kShapes[0])); ++i)
    if (kShapes[i].kc == kc && kShapes[i].q == q) {
      if (n < cap) out[n] = to_shape(i);
      ++n;
    }
  return n;
}

Asm16Shape asm16_shape(int kc, int q, int pick) {
  Asm16Shape c[16];
  const int n = asm16_shapes(kc, q, c, 16);
  if (n == 0) {
    Asm16Shape none{};
    none.id = -1;
    return none;
  }
  Asm16Shape sh = c[(pick >= 0 && pick < n && pick < 16) ? pick : 0];
  sh.wgs_per_cu = kShapes[sh.id].occupancy();
  return sh;
}

hipError_t launch_assemble16(int prec, int kc, int q, const Asm16Shape& shape, const AsmMol* mols_dev,
                             const int4* items_dev, const int* seg_dev, unsigned* counters, int nblocks,
                             hipStream_t s) {
  if (shape.id < 0 || shape.id >= (int)(sizeof(kShapes) / sizeof(kShapes[0])) || kShapes[shape.id].kc != kc ||
      kShapes[shape.id].q != q)
    return hipErrorInvalidValue;
  return kShapes[shape.id].launch(prec != kF16X3, mols_dev, items_dev, seg_dev, counters, nblocks, s);
}

}  // namespace tai
