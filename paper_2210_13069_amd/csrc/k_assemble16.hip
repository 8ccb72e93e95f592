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
//   with direct-to-LDS loads (global_load_lds_dwordx4), NBUF-buffered so the
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
#include <type_traits>

namespace tai {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr double kTwoOverSqrtPi = 1.1283791670955126;
constexpr int kCB = 2;      // 16-column blocks per 32-column block
constexpr int kGroup16 = 8; // FP32 accumulation group of quadrature nodes
constexpr int kOutStride = 33;  // floats per row of the output tile

template <int KC, int Q>
struct Cfg16 {
  static constexpr int NCH = KC / 32;                       // 32-wide inner chunks
  static constexpr int U = NCH - Q;                         // distinct A fragments
  static constexpr int RB = U <= 3 ? 4 : (U <= 4 ? 3 : (U <= 6 ? 2 : 1));
  static constexpr int ROWS = 64 * RB;                      // rows per work group
  static constexpr int NFRAG = 3 * kCB * NCH;               // 1 KB fragments per node
  static constexpr int LPW = (NFRAG + 3) / 4;               // loads per wave per node
  static constexpr int NV = RB * kCB * 4;                   // accumulator values per lane
  static constexpr int ACC_BYTES = 4 * NV * 64 * 8;         // FP64 partial sums, all waves
  static constexpr int NBUF = (3 * NFRAG * 1024 + ACC_BYTES <= 150 * 1024) ? 3 : 2;
};

// A fragment register index of MFMA chunk ch (chunks Q..2Q-1 repeat 0..Q-1),
// and the K chunk a register fragment is loaded from.
template <int Q> __device__ constexpr int a_slot(int ch) { return ch < Q ? ch : ch - Q; }
template <int Q> __device__ constexpr int a_chunk(int u) { return u < Q ? u : u + Q; }

template <int N>
__device__ inline void wait_vmcnt() {
  __asm__ volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ inline v4f mma(v8h a, v8h b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
__device__ inline v4f mma(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// Issue the direct-to-LDS loads of the Y fragments of node k into buf.
// Fragment f = (d*kCB + c)*NCH + ch holds, for lane l, the 16 bytes
// Y[k][d][col0 + 16c + l%16][32ch + 8(l/16) .. +8].  Wave w loads fragments
// w, w+4, ...; the index is clamped so that every wave issues exactly LPW
// loads (a clamped duplicate rewrites identical bytes).
template <int KC, int Q>
__device__ inline void stage_y(const char* __restrict__ Y, int64_t prow, int k, int64_t col0, uint4* buf,
                               int wave, int lane) {
  using C = Cfg16<KC, Q>;
  const int r16 = lane & 15, kg = lane >> 4;
#pragma unroll
  for (int i = 0; i < C::LPW; ++i) {
    int f = wave + 4 * i;
    f = f < C::NFRAG ? f : C::NFRAG - 1;
    const int ch = f % C::NCH;
    const int c = (f / C::NCH) % kCB;
    const int d = f / (C::NCH * kCB);
    const int64_t row = ((int64_t)k * 3 + d) * prow + col0 + 16 * c + r16;
    const char* src = Y + (row * KC + 32 * ch + 8 * kg) * 2;
    __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src), (lds_ptr_t)(buf + f * 64), 16, 0, 0);
  }
}

template <int KC, int Q>
__device__ inline void wait_stage(int k, int nq) {
  using C = Cfg16<KC, Q>;
  if constexpr (C::NBUF == 3) {
    if (k + 1 < nq) wait_vmcnt<C::LPW>();  // stage k+1 may stay in flight
    else wait_vmcnt<0>();
  } else {
    wait_vmcnt<0>();
  }
}

// One node k of a 32-column block: wait for its Y fragments (buffer CUR),
// issue the loads of node k + NBUF - 1 into buffer NXT, and accumulate.
// The buffers are distinct __shared__ objects chosen at compile time, so the
// compiler can tell the in-flight direct-to-LDS writes from the reads.
template <int KC, int Q, bool BF, int RB, int NCH>
__device__ inline void node_step(int k, int nq, int64_t prow, int64_t col0, const char* __restrict__ Yb,
                                 const uint4* cur, uint4* nxt,
                                 const typename std::conditional<BF, v8bf, v8h>::type (&af)[3][RB][NCH - Q],
                                 v4f (&acc)[RB][kCB], int wave, int lane) {
  using C = Cfg16<KC, Q>;
  using Frag = typename std::conditional<BF, v8bf, v8h>::type;
  constexpr int D = C::NBUF - 1;
  // Every wave waits for its own loads of node k, then all waves meet: node
  // k is then in LDS for everyone, and every wave has consumed node k-1 (its
  // fragments fed MFMAs that already issued), whose buffer the loads below
  // reuse.  A plain s_barrier (memory clobber for the compiler) instead of
  // __syncthreads, whose fence would also drain the loads still in flight.
  wait_stage<KC, Q>(k, nq);
  __asm__ volatile("s_barrier" ::: "memory");
  if (k + D < nq) stage_y<KC, Q>(Yb, prow, k + D, col0, nxt, wave, lane);
  v4f H[RB][kCB];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    v4f G[RB][kCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int c = 0; c < kCB; ++c) G[rb][c] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      Frag bfr[kCB];
#pragma unroll
      for (int c = 0; c < kCB; ++c)
        bfr[c] = *reinterpret_cast<const Frag*>(cur + ((d * kCB + c) * NCH + ch) * 64 + lane);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < kCB; ++c) G[rb][c] = mma(af[d][rb][a_slot<Q>(ch)], bfr[c], G[rb][c]);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int c = 0; c < kCB; ++c) {
        if (d == 0) H[rb][c] = G[rb][c];
        else if (d == 1) H[rb][c] *= G[rb][c];
        else acc[rb][c] += H[rb][c] * G[rb][c];
      }
  }
}

template <int KC, int Q, bool BF>
__device__ inline void run_item(const AsmMol& m, int rp, int cb0, int cb1, uint4* yb0, uint4* yb1, uint4* yb2,
                                double* accs, float* outt) {
  using C = Cfg16<KC, Q>;
  using Frag = typename std::conditional<BF, v8bf, v8h>::type;
  constexpr int RB = C::RB, NCH = C::NCH, NBUF = C::NBUF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int64_t prow = m.prow;
  const int64_t row_wg = (int64_t)rp * C::ROWS;
  const int64_t row_base = row_wg + wave * 16 * RB;
  const char* __restrict__ Ab = static_cast<const char*>(m.A);
  const char* __restrict__ Yb = static_cast<const char*>(m.Y);
  const int nq = m.nq;
  const int64_t npair = m.npair;
  const int64_t ldb = m.ldb;
  float* __restrict__ Bout = static_cast<float*>(m.B);
  const bool vec_ok = ((ldb & 3) == 0) && ((reinterpret_cast<uintptr_t>(Bout) & 15) == 0);
  double* myacc = accs + wave * C::NV * 64 + lane;   // value v at myacc[v * 64]

  // k-invariant A operand of this wave's rows, all directions
  Frag af[3][RB][NCH - Q];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int u = 0; u < NCH - Q; ++u) {
        const int64_t row = (int64_t)d * prow + row_base + 16 * rb + r16;
        af[d][rb][u] = *reinterpret_cast<const Frag*>(Ab + (row * KC + 32 * a_chunk<Q>(u) + 8 * kg) * 2);
      }

  for (int cb = cb0; cb < cb1; ++cb) {
    const int64_t col0 = (int64_t)cb * 32;
    // prologue: the first NBUF-1 nodes
    stage_y<KC, Q>(Yb, prow, 0, col0, yb0, wave, lane);
    if (NBUF == 3 && nq > 1) stage_y<KC, Q>(Yb, prow, 1, col0, yb1, wave, lane);

    v4f acc[RB][kCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int c = 0; c < kCB; ++c) acc[rb][c] = v4f{0.f, 0.f, 0.f, 0.f};
    bool first_flush = true;
    auto flush = [&](int k) {
      if ((k + 1) % kGroup16 == 0 || k + 1 == nq) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int c = 0; c < kCB; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int v = (rb * kCB + c) * 4 + r;
              const double x = (double)acc[rb][c][r];
              myacc[v * 64] = first_flush ? x : myacc[v * 64] + x;
            }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int c = 0; c < kCB; ++c) acc[rb][c] = v4f{0.f, 0.f, 0.f, 0.f};
        first_flush = false;
      }
    };

    if constexpr (NBUF == 3) {
      for (int k = 0; k < nq; k += 3) {
        node_step<KC, Q, BF, RB, NCH>(k, nq, prow, col0, Yb, yb0, yb2, af, acc, wave, lane);
        flush(k);
        if (k + 1 < nq) {
          node_step<KC, Q, BF, RB, NCH>(k + 1, nq, prow, col0, Yb, yb1, yb0, af, acc, wave, lane);
          flush(k + 1);
        }
        if (k + 2 < nq) {
          node_step<KC, Q, BF, RB, NCH>(k + 2, nq, prow, col0, Yb, yb2, yb1, af, acc, wave, lane);
          flush(k + 2);
        }
      }
    } else {
      for (int k = 0; k < nq; k += 2) {
        node_step<KC, Q, BF, RB, NCH>(k, nq, prow, col0, Yb, yb0, yb1, af, acc, wave, lane);
        flush(k);
        if (k + 1 < nq) {
          node_step<KC, Q, BF, RB, NCH>(k + 1, nq, prow, col0, Yb, yb1, yb0, af, acc, wave, lane);
          flush(k + 1);
        }
      }
    }

    // finished block: FP64 sums -> scaled floats in the output tile
    double fin[C::NV];
#pragma unroll
    for (int v = 0; v < C::NV; ++v) fin[v] = myacc[v * 64];
    __syncthreads();  // every wave has read its sums before the tile reuses the space
    int ecol[kCB];
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      const int64_t col = col0 + 16 * c + r16;
      ecol[c] = m.ex[col] + m.ex[prow + col] + m.ex[2 * prow + col];
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wave * 16 * RB + 16 * rb + 4 * kg + r;
        const int64_t row = row_wg + rl;
        const int erow = m.ex[row] + m.ex[prow + row] + m.ex[2 * prow + row];
#pragma unroll
        for (int c = 0; c < kCB; ++c) {
          const int v = (rb * kCB + c) * 4 + r;
          outt[rl * kOutStride + 16 * c + r16] = (float)ldexp(fin[v] * kTwoOverSqrtPi, erow + ecol[c]);
        }
      }
    __syncthreads();

    // rows: B[row][col0 .. col0+31] for row <= col
    for (int i = threadIdx.x; i < C::ROWS * 8; i += 256) {
      const int rl = i >> 3, c4 = (i & 7) * 4;
      const int64_t row = row_wg + rl;
      const int64_t col = col0 + c4;
      const float* src = outt + rl * kOutStride + c4;
      float* dst = Bout + row * ldb + col;
      if (vec_ok && row <= col && col + 3 < npair) {
        *reinterpret_cast<float4*>(dst) = make_float4(src[0], src[1], src[2], src[3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (row <= col + e && col + e < npair) dst[e] = src[e];
      }
    }
    // mirrored columns: B[col][row .. row+3] for row < col
    for (int i = threadIdx.x; i < 32 * (C::ROWS / 4); i += 256) {
      const int cl = i / (C::ROWS / 4), r4 = (i % (C::ROWS / 4)) * 4;
      const int64_t col = col0 + cl;
      const int64_t row = row_wg + r4;
      if (col >= npair) continue;
      const float* src = outt + r4 * kOutStride + cl;
      float* dst = Bout + col * ldb + row;
      if (vec_ok && row + 3 < col) {
        *reinterpret_cast<float4*>(dst) =
            make_float4(src[0], src[kOutStride], src[2 * kOutStride], src[3 * kOutStride]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (row + e < col) dst[e] = src[e * kOutStride];
      }
    }
    __syncthreads();  // tile and sums space free for the next block
  }
}

template <int KC, int Q, bool BF>
__global__ void __launch_bounds__(256, 1)
assemble16_kernel(const AsmMol* __restrict__ mols, const int4* __restrict__ items, int nitems,
                  unsigned* __restrict__ counter) {
  using C = Cfg16<KC, Q>;
  __shared__ uint4 yb0[C::NFRAG * 64];
  __shared__ uint4 yb1[C::NFRAG * 64];
  __shared__ uint4 yb2[C::NBUF == 3 ? C::NFRAG * 64 : 1];
  __shared__ double accs[C::ACC_BYTES / 8];  // FP64 sums; reused as the output tile
  __shared__ int item_s;
  static_assert(C::ROWS * kOutStride * 4 <= C::ACC_BYTES, "output tile fits in the sums space");
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item_s = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int it = item_s;
    if (it >= nitems) break;
    const int4 item = items[it];
    const AsmMol m = mols[item.x];
    run_item<KC, Q, BF>(m, item.y, item.z, item.w, yb0, yb1, yb2, accs, reinterpret_cast<float*>(accs));
  }
}

template <int KC, int Q>
hipError_t launch16(bool bf, const AsmMol* mols, const int4* items, int nitems, unsigned* counter, int nblocks,
                    hipStream_t s) {
  if (bf)
    hipLaunchKernelGGL((assemble16_kernel<KC, Q, true>), dim3(nblocks), dim3(256), 0, s, mols, items, nitems, counter);
  else
    hipLaunchKernelGGL((assemble16_kernel<KC, Q, false>), dim3(nblocks), dim3(256), 0, s, mols, items, nitems, counter);
  return hipGetLastError();
}

}  // namespace

int asm16_max_kc() { return 352; }

int asm16_rows_for(int kc, int q) {
  const int u = kc / 32 - q;
  return 64 * (u <= 3 ? 4 : (u <= 4 ? 3 : (u <= 6 ? 2 : 1)));
}

hipError_t launch_assemble16(int prec, int kc, int q, const AsmMol* mols_dev, const int4* items_dev, int nitems,
                             unsigned* counter, int nblocks, hipStream_t s) {
  const bool bf = prec != kF16X3;
#define TAI_L16(KC_, Q_) \
  if (kc == KC_ && q == Q_) return launch16<KC_, Q_>(bf, mols_dev, items_dev, nitems, counter, nblocks, s);
  TAI_L16(32, 0) TAI_L16(64, 0) TAI_L16(96, 0) TAI_L16(96, 1) TAI_L16(128, 0) TAI_L16(128, 1)
  TAI_L16(160, 0) TAI_L16(160, 1) TAI_L16(192, 0) TAI_L16(192, 1) TAI_L16(192, 2)
  TAI_L16(224, 0) TAI_L16(256, 0) TAI_L16(288, 0) TAI_L16(320, 0) TAI_L16(352, 0)
#undef TAI_L16
  return hipErrorInvalidValue;
}

}  // namespace tai
