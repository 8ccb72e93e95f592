// Host layer of libtai: the C ABI of include/tai.h.  Validates arguments
// before any device work, owns the context's workspace, and enqueues the
// kernels of the hot path on the caller's stream.
#include "tai_internal.h"
#include "../../include/tai.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// Static device scratch of tai_apply_J_noalloc: the node tables and the J
// intermediates of one call, for callers that cannot allocate.  Every device
// the library runs on holds its own copy until the process ends.  In host
// code `scratch` is only a stand-in symbol: its device address comes from
// hipGetSymbolAddress, once per device (scratch_address), and only that
// address is ever handed to a kernel or a copy.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

using tai::NodeTables;

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct tai_ctx {
  int device = -1;        // -1: host-only context (validation only)
  std::string err;
  size_t limit = 0;       // workspace limit in bytes (0 = none)
  size_t total = 0;       // bytes currently allocated
  Buf nodes;              // NodeTables for single-molecule calls
  Buf basis;              // device copy of a basis
  Buf host_basis;         // pinned staging of a basis
  hipEvent_t host_basis_done = nullptr;
  Buf opA, opEx, opY;     // assembly operands
  Buf opMu;               // coefficient moments (per-node degrees)
  Buf cmp, cmpU;          // low-rank compression: basis, Gram, tables; compressed moments
  Buf screen;             // screening: row counts / offsets and the kept count
  Buf part, partJ;        // adaptive boxes: supports, sort and lists; partitioned J intermediates
  Buf partB;              // partitioned B: cross tables and every block's operands
  Buf mo;                 // orbital-basis Coulomb matrix: rho and Phi of every orbital
  Buf ct, ct_work;        // contraction: member tables; primitive-basis D and J
  Buf ct_host;            // pinned staging of the member tables
  hipEvent_t ct_host_done = nullptr;
  Buf asm_tab, asm_counter;  // 16-bit kernel: device molecule table + items, queue counter
  Buf asm_host;           // pinned staging of the table
  hipEvent_t asm_host_done = nullptr;
  int cus = 0;            // compute units of the device
  void* scratch = nullptr;  // this device's address of the static scratch
  // 16-bit kernel shapes: runtime facts per table entry, the tuned choice
  // (candidate index) per call signature, and the tuning state
  std::vector<tai::Asm16Shape> shapes16;
  struct Tuned { int prec, n, nq; uint64_t key; int pick; };
  std::vector<Tuned> tuned;
  int tune_mode = 1;      // 0: table defaults, 1: tune each new signature once
  int force_pick = -1;    // candidate forced while tuning
  uint64_t size_key = 0;  // size class of the call in progress
  Buf jwork;              // apply_J intermediates
  // batched path
  Buf b_nodes, b_basis, b_opA, b_opEx, b_opY, b_opMu, b_mols, b_counter;
  Buf b_cmp;              // batched compression: per-molecule buffers and per-node ranks
  Buf b_host;             // pinned staging of all bases of a batch
  hipEvent_t b_host_done = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<unsigned char> graph_key;
  // per-stage device timing (tai_profile_enable / tai_profile_read)
  bool prof_on = false;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms[8] = {0};
  int64_t prof_n[8] = {0};
};

namespace {

int fail(tai_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(tai_ctx* c, hipError_t e, const char* where) {
  return fail(c, TAI_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool finite(double x) { return std::isfinite(x); }

// check_L = false where the half-widths come from elsewhere (the boxes of
// the partitioned J) and params->L is not read.
int validate_params(tai_ctx* c, const tai_params* p, bool check_L = true) {
  if (!p) return fail(c, TAI_ERR_INVALID_ARG, "params is NULL");
  if (!finite(p->omega) || !(p->omega > 0)) return fail(c, TAI_ERR_INVALID_ARG, "omega must be finite and > 0");
  if (p->nq < 1 || p->nq > 128) return fail(c, TAI_ERR_INVALID_ARG, "nq must be in [1, 128]");
  if (p->n < 2 || p->n > 64) return fail(c, TAI_ERR_INVALID_ARG, "n must be in [2, 64]");
  if (check_L && (!finite(p->L) || !(p->L > 0))) return fail(c, TAI_ERR_INVALID_ARG, "L must be finite and > 0");
  if (p->nodes != TAI_NODES_LOBATTO && p->nodes != TAI_NODES_GAUSS)
    return fail(c, TAI_ERR_INVALID_ARG, "nodes must be TAI_NODES_LOBATTO or TAI_NODES_GAUSS");
  if (p->prec < TAI_FP64 || p->prec > TAI_F16X3) return fail(c, TAI_ERR_INVALID_ARG, "unknown prec");
  if (!finite(p->degree_tol) || p->degree_tol < 0)
    return fail(c, TAI_ERR_INVALID_ARG, "degree_tol must be finite and >= 0");
  if (!finite(p->rank_tol) || p->rank_tol < 0 || !(p->rank_tol < 1))
    return fail(c, TAI_ERR_INVALID_ARG, "rank_tol must be finite and in [0, 1)");
  return TAI_OK;
}

int validate_basis(tai_ctx* c, const tai_basis* b) {
  if (!b) return fail(c, TAI_ERR_INVALID_ARG, "basis is NULL");
  if (b->nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  const int64_t npair = (int64_t)b->nb * (b->nb + 1) / 2;
  if (npair > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (!b->center || !b->alpha || !b->lxyz) return fail(c, TAI_ERR_INVALID_ARG, "basis center/alpha/lxyz is NULL");
  for (int i = 0; i < b->nb; ++i) {
    if (!finite(b->alpha[i]) || !(b->alpha[i] > 0))
      return fail(c, TAI_ERR_INVALID_ARG, "alpha[" + std::to_string(i) + "] must be finite and > 0");
    for (int d = 0; d < 3; ++d) {
      if (!finite(b->center[3 * i + d]))
        return fail(c, TAI_ERR_INVALID_ARG, "center[" + std::to_string(i) + "] is not finite");
      const int l = b->lxyz[3 * i + d];
      if (l < 0 || l > 4) return fail(c, TAI_ERR_INVALID_ARG, "lxyz[" + std::to_string(i) + "] out of [0, 4]");
    }
    if (b->coef && !finite(b->coef[i]))
      return fail(c, TAI_ERR_INVALID_ARG, "coef[" + std::to_string(i) + "] is not finite");
  }
  return TAI_OK;
}

int check_ctx(tai_ctx* c) {
  if (!c) return TAI_ERR_INVALID_ARG;
  c->err.clear();
  return TAI_OK;
}

int need_device(tai_ctx* c) {
  if (c->device < 0) return fail(c, TAI_ERR_NOT_READY, "host-only context: no device work possible");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return TAI_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Arithmetics of the pair contractions of J: FP64, FP32, and the split-BF16
// forms (F16X3 would need the operands scaled across the sum over pairs).
bool j_prec_ok(int prec) { return prec == TAI_FP64 || prec == TAI_FP32 || prec == TAI_BF16X3 || prec == TAI_BF16X6; }

const char* const kStageNames[] = {"nodes", "moments", "pack", "project", "assemble", "apply_J", "batched", "compress"};
constexpr int kNumStages = 8;
enum { kStNodes = 0, kStMoments, kStPack, kStProject, kStAssemble, kStApplyJ, kStBatched, kStCompress };

hipEvent_t take_event(tai_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one stage's launches with timing events on the stream it runs on.
struct Timed {
  tai_ctx* c;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Timed(tai_ctx* c_, int st, hipStream_t s_) : c(c_), stage(st), s(s_) {
    if (c->prof_on && (a = take_event(c)) && hipEventRecord(a, s) != hipSuccess) {
      c->ev_pool.push_back(a);
      a = nullptr;
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (b && hipEventRecord(b, s) == hipSuccess) {
      c->prof_pending.push_back({stage, a, b});
    } else {
      c->ev_pool.push_back(a);
      if (b) c->ev_pool.push_back(b);
    }
  }
};


// Grow a device buffer to at least `bytes`.
int ensure(tai_ctx* c, Buf& b, size_t bytes) {
  bytes = align256(bytes ? bytes : 256);
  if (b.cap >= bytes) return TAI_OK;
  if (c->limit && c->total - b.cap + bytes > c->limit)
    return fail(c, TAI_ERR_NOMEM, "workspace of " + std::to_string(c->total - b.cap + bytes) +
                                      " bytes exceeds TAI_WORKSPACE_LIMIT");
  if (b.p) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    hipFree(b.p);
    c->total -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, TAI_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.cap = bytes;
  c->total += bytes;
  return TAI_OK;
}

// Grow a pinned host buffer; waits for the copy that last read it.
int ensure_host(tai_ctx* c, Buf& b, hipEvent_t& done, size_t bytes) {
  if (done) {
    hipError_t e = hipEventSynchronize(done);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
  } else {
    hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
  }
  bytes = align256(bytes ? bytes : 256);
  if (b.cap >= bytes) return TAI_OK;
  if (b.p) hipHostFree(b.p);
  b.p = nullptr;
  b.cap = 0;
  hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, TAI_ERR_NOMEM, "hipHostMalloc failed");
  }
  b.cap = bytes;
  return TAI_OK;
}

void free_buf(tai_ctx* c, Buf& b) {
  if (b.p) hipFree(b.p);
  c->total -= b.cap;
  b.p = nullptr;
  b.cap = 0;
}

int64_t npair_of(int nb) { return (int64_t)nb * (nb + 1) / 2; }

// Serialised basis: center[3nb] alpha[nb] coef[nb] (doubles), lxyz[3nb] (int32).
size_t basis_bytes(int nb) { return align256(sizeof(double) * 5 * (size_t)nb) + align256(sizeof(int32_t) * 3 * (size_t)nb); }

void pack_basis_host(const tai_basis* b, char* dst) {
  double* dd = reinterpret_cast<double*>(dst);
  std::memcpy(dd, b->center, sizeof(double) * 3 * b->nb);
  std::memcpy(dd + 3 * b->nb, b->alpha, sizeof(double) * b->nb);
  if (b->coef) std::memcpy(dd + 4 * b->nb, b->coef, sizeof(double) * b->nb);
  else std::memset(dd + 4 * b->nb, 0, sizeof(double) * b->nb);
  std::memcpy(dst + align256(sizeof(double) * 5 * (size_t)b->nb), b->lxyz, sizeof(int32_t) * 3 * b->nb);
}

tai::DevBasis dev_basis_view(const tai_basis* b, char* dev) {
  tai::DevBasis d;
  d.nb = b->nb;
  double* dd = reinterpret_cast<double*>(dev);
  d.center = dd;
  d.alpha = dd + 3 * b->nb;
  d.coef = b->coef ? dd + 4 * b->nb : nullptr;
  d.lxyz = reinterpret_cast<const int32_t*>(dev + align256(sizeof(double) * 5 * (size_t)b->nb));
  return d;
}

// Index of the 16-bit kernel shape used for (prec, n, nq) at the current
// call's size class: TAI_ASM16_SHAPE if set, else the candidate being timed
// while tuning, else the tuned choice, else the table default (0).
int shape_pick(tai_ctx* c, int prec, int n, int nq) {
  if (const char* v = std::getenv("TAI_ASM16_SHAPE")) return std::atoi(v);
  if (c->force_pick >= 0) return c->force_pick;
  for (const auto& t : c->tuned)
    if (t.prec == prec && t.n == n && t.nq == nq && t.key == c->size_key) return t.pick;
  return 0;
}

// Whether a shape can stream nq nodes: its ring steps hold nps nodes each,
// and the deferred end-of-block epilogue needs at least nbuf steps per block.
bool shape_fits(const tai::Asm16Shape& sh, int nq) { return nq % sh.nps == 0 && nq >= sh.nbuf * sh.nps; }

// Shape of the 16-bit kernel for this call (runtime facts cached per table
// entry; the device must be current): the picked candidate if it fits nq,
// else the first one in table order that does; id -1 if none does.
tai::Asm16Shape shape16(tai_ctx* c, int prec, int n, int nq) {
  const int kc = tai::operand_kc(prec, n), q = tai::operand_dup_chunks(prec, n);
  tai::Asm16Shape list[16];
  const int cnt = std::min(tai::asm16_shapes(kc, q, list, 16), 16);
  int pick = shape_pick(c, prec, n, nq);
  if (pick < 0 || pick >= cnt || !shape_fits(list[pick], nq)) {
    pick = -1;
    for (int i = 0; i < cnt && pick < 0; ++i)
      if (shape_fits(list[i], nq)) pick = i;
  }
  if (pick < 0) {
    tai::Asm16Shape none{};
    none.id = -1;
    return none;
  }
  for (const auto& sh : c->shapes16)
    if (sh.id == list[pick].id) return sh;
  tai::Asm16Shape sh = tai::asm16_shape(kc, q, pick);
  c->shapes16.push_back(sh);
  return sh;
}

// Whether the 16-bit persistent kernel takes this call: a split 16-bit
// arithmetic whose inner length it supports, and a shape that fits the node
// count (too few nodes for any ring go to the generic kernel).
bool use16(tai_ctx* c, int prec, int n, int nq) {
  if (!tai::is_split16(prec) || tai::operand_kc(prec, n) > tai::asm16_max_kc() || std::getenv("TAI_ASM16_GENERIC"))
    return false;
  return shape16(c, prec, n, nq).id >= 0;
}

// Whether FP32 / FP64 assembly takes the persistent LDS-ring kernel
// (k_assemble32.hip), for the inner lengths it is built for (it skips each
// node's unused inner steps with per-node degrees too).  TAI_TILE_ASSEMBLY
// selects the tile kernels instead.
bool use32(int prec, int n) {
  return (prec == tai::kFP32 || prec == tai::kFP64) && tai::operand_kc(prec, n) <= tai::kAsm32MaxKc &&
         !std::getenv("TAI_TILE_ASSEMBLY");
}
int ring_rows(int prec, int n) {
  const int kc = tai::operand_kc(prec, n);
  return prec == tai::kFP64 ? tai::asm64_rows(kc) : tai::asm32_rows(kc);
}
// Always the form that reads per-node degrees (a molecule without them runs
// every inner step): a molecule then gives the same bits alone and in any
// batch.
hipError_t launch_ring(int prec, int kc, bool /*deg*/, const tai::AsmMol* mols, const int4* items, const int* seg,
                       unsigned* counters, int nblocks, hipStream_t s) {
  return prec == tai::kFP64 ? tai::launch_assemble64(kc, true, mols, items, seg, counters, nblocks, s)
                            : tai::launch_assemble32(kc, true, mols, items, seg, counters, nblocks, s);
}

int prow_of(tai_ctx* c, int prec, int n, int nq, int64_t npair) {
  int64_t t = 256;
  const bool p16 = use16(c, prec, n, nq), p32 = use32(prec, n);
  if (p16 || p32) {
    const int64_t r = p16 ? shape16(c, prec, n, nq).rows : ring_rows(prec, n);
    int64_t a = r, b = 256;
    while (b) {
      const int64_t tmp = a % b;
      a = b;
      b = tmp;
    }
    t = r / a * 256;  // lcm(r, 256)
  }
  return (int)((npair + t - 1) / t * t);
}

size_t opA_bytes(int prec, int n, int prow) {
  return align256((size_t)3 * prow * tai::operand_kc(prec, n) * tai::operand_esize(prec));
}
size_t opY_bytes(int prec, int n, int nq, int prow) {
  return align256((size_t)nq * 3 * prow * tai::operand_kc(prec, n) * tai::operand_esize(prec));
}
size_t opEx_bytes(int prow) { return align256(sizeof(int32_t) * 3 * (size_t)prow); }

// Work items of the 16-bit assembly kernel for one molecule: row panels of
// Work items of the 16-bit kernel: (molecule, row panel of R rows, run of up
// to 512 columns in blocks of C), upper triangle only.  Column runs are
// dealt round-robin to the kAsm16Queues queues (one per XCD; `rr` carries
// the deal across molecules), each queue ordered column-run-major so that
// the work groups of an XCD share the Y blocks of a run in its L2.
struct Items16 {
  std::vector<int4> q[tai::kAsm16Queues];
  int rr = 0;
  // Items of (row panel, run of column blocks) in the upper triangle, with
  // runs of up to 512 columns.  With min_items > 0 the runs are halved
  // until there are at least that many items (or one block per item), so
  // that a small molecule still spreads over the device; the entries and
  // the order of every entry's node sum do not depend on the runs.
  void add(int mol, int64_t npair, int64_t R, int64_t C, int64_t min_items = 0) {
    const int64_t ncb = (npair + C - 1) / C;
    const int64_t nrp = (npair + R - 1) / R;
    int64_t chunk = std::max<int64_t>(1, 512 / C);
    auto items_for = [&](int64_t ch) {
      int64_t n = 0;
      for (int64_t j = 0; j * ch < ncb; ++j)
        for (int64_t rp = 0; rp < nrp; ++rp)
          n += std::max(j * ch, rp * R / C) < std::min((j + 1) * ch, ncb) ? 1 : 0;
      return n;
    };
    while (chunk > 1 && items_for(chunk) < min_items) chunk = (chunk + 1) / 2;
    for (int64_t j = 0; j * chunk < ncb; ++j) {
      std::vector<int4>& out = q[rr++ % tai::kAsm16Queues];
      for (int64_t rp = 0; rp < nrp; ++rp) {
        const int64_t lo = std::max(j * chunk, rp * R / C);
        const int64_t hi = std::min((j + 1) * chunk, ncb);
        if (lo < hi) out.push_back(int4{mol, (int)rp, (int)lo, (int)hi});
      }
    }
  }
  // Items of a rectangular block (nrow rows against ncol columns, every
  // entry): all (row panel, run of column blocks), runs as in add.
  void add_rect(int mol, int64_t nrow, int64_t ncol, int64_t R, int64_t C, int64_t min_items = 0) {
    const int64_t ncb = (ncol + C - 1) / C;
    const int64_t nrp = (nrow + R - 1) / R;
    int64_t chunk = std::max<int64_t>(1, 512 / C);
    while (chunk > 1 && ((ncb + chunk - 1) / chunk) * nrp < min_items) chunk = (chunk + 1) / 2;
    for (int64_t j = 0; j * chunk < ncb; ++j) {
      std::vector<int4>& out = q[rr++ % tai::kAsm16Queues];
      for (int64_t rp = 0; rp < nrp; ++rp)
        out.push_back(int4{mol, (int)rp, (int)(j * chunk), (int)std::min((j + 1) * chunk, ncb)});
    }
  }
  size_t count() const {
    size_t n = 0;
    for (const auto& v : q) n += v.size();
    return n;
  }
  // seg[kAsm16Queues + 1] offsets followed (at 256 bytes) by the items
  static size_t seg_bytes() { return align256(sizeof(int) * (tai::kAsm16Queues + 1)); }
  size_t bytes() const { return seg_bytes() + sizeof(int4) * count(); }
  void write(char* dst) const {
    int* seg = reinterpret_cast<int*>(dst);
    int4* it = reinterpret_cast<int4*>(dst + seg_bytes());
    int off = 0;
    for (int x = 0; x < tai::kAsm16Queues; ++x) {
      seg[x] = off;
      std::memcpy(it + off, q[x].data(), sizeof(int4) * q[x].size());
      off += (int)q[x].size();
    }
    seg[tai::kAsm16Queues] = off;
  }
};

// Whether calls of this arithmetic and degree have 16-bit kernel shapes to
// choose between (and nobody forced one).
bool tunable(int prec, int n) {
  if (!tai::is_split16(prec) || tai::operand_kc(prec, n) > tai::asm16_max_kc()) return false;
  if (std::getenv("TAI_ASM16_GENERIC") || std::getenv("TAI_ASM16_SHAPE")) return false;
  tai::Asm16Shape list[16];
  return tai::asm16_shapes(tai::operand_kc(prec, n), tai::operand_dup_chunks(prec, n), list, 16) > 1;
}

// Autotuner of the 16-bit kernel shape: on the first call of a signature
// (arithmetic, degree, nodes, size class) every candidate shape runs the
// whole call once to warm up and once timed on the caller's stream; the
// fastest is kept for the signature (the table's first fitting shape unless
// another is more than 2% faster).  All candidates compute every entry
// with the same arithmetic in the same order, so the choice never changes
// results.  `run` performs the call without a graph.
template <class Run>
int tune16(tai_ctx* c, int prec, int n, int nq, hipStream_t s, Run run) {
  for (const auto& t : c->tuned)
    if (t.prec == prec && t.n == n && t.nq == nq && t.key == c->size_key) return TAI_OK;
  tai::Asm16Shape list[16];
  const int cnt = tai::asm16_shapes(tai::operand_kc(prec, n), tai::operand_dup_chunks(prec, n), list, 16);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) hipEventDestroy(a);
    return hip_fail(c, hipErrorUnknown, "hipEventCreate");
  }
  const bool prof = c->prof_on;
  c->prof_on = false;
  int best = -1, r = TAI_OK;
  float best_ms = 0.f;
  for (int i = 0; i < cnt && i < 16; ++i) {
    if (!shape_fits(list[i], nq)) continue;  // shape16 would not take it
    c->force_pick = i;
    if ((r = run())) break;
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess && (r = run())) break;
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (e != hipSuccess) {
      r = hip_fail(c, e, "autotune timing");
      break;
    }
    // the first candidate that fits (table order) holds unless another one
    // is more than 2% faster, so that run-to-run noise does not flip the
    // choice between shapes that are within it
    if (best < 0 || ms < best_ms * 0.98f) {
      best_ms = ms;
      best = i;
    }
  }
  c->force_pick = -1;
  c->prof_on = prof;
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (r) return r;
  c->tuned.push_back({prec, n, nq, c->size_key, best < 0 ? 0 : best});
  return TAI_OK;
}

uint64_t pow2_at_least(int64_t v) {
  uint64_t k = 1;
  while ((int64_t)k < v) k <<= 1;
  return k;
}

}  // namespace

extern "C" {

// Device address of the static scratch on `device`, looked up once per
// device with that device current (each device holds its own copy of the
// array at its own address).  nullptr if the lookup fails.
static void* scratch_address(int device) {
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    void* p = nullptr;
    if (hipSetDevice(device) == hipSuccess && hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) addr[device] = p;
    else (void)hipGetLastError();
    if (prev >= 0) hipSetDevice(prev);
  }
  return addr[device];
}

int tai_create(tai_ctx** ctx, int hip_device) {
  if (!ctx) return TAI_ERR_INVALID_ARG;
  *ctx = nullptr;
  if (hip_device < -1) return TAI_ERR_INVALID_ARG;
  tai_ctx* c = new (std::nothrow) tai_ctx();
  if (!c) return TAI_ERR_NOMEM;
  if (const char* lim = std::getenv("TAI_WORKSPACE_LIMIT")) c->limit = (size_t)std::strtoull(lim, nullptr, 10);
  if (hip_device >= 0) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || hip_device >= count) {
      (void)hipGetLastError();
      delete c;
      return TAI_ERR_HIP;
    }
    c->device = hip_device;
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, hip_device) != hipSuccess) c->cus = 256;
    c->scratch = scratch_address(hip_device);
  }
  *ctx = c;
  return TAI_OK;
}

int tai_destroy(tai_ctx* c) {
  if (!c) return TAI_OK;
  if (c->device >= 0) {
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (Buf* b : {&c->nodes, &c->basis, &c->opA, &c->opEx, &c->opY, &c->opMu, &c->cmp, &c->cmpU, &c->screen, &c->part,
                   &c->partJ, &c->partB, &c->mo, &c->ct, &c->ct_work, &c->asm_tab,
                   &c->asm_counter,
                   &c->jwork,
                   &c->b_nodes, &c->b_basis, &c->b_opA, &c->b_opEx, &c->b_opY, &c->b_opMu, &c->b_mols, &c->b_counter, &c->b_cmp})
      free_buf(c, *b);
    if (c->host_basis.p) hipHostFree(c->host_basis.p);
    if (c->b_host.p) hipHostFree(c->b_host.p);
    if (c->asm_host.p) hipHostFree(c->asm_host.p);
    if (c->ct_host.p) hipHostFree(c->ct_host.p);
    if (c->ct_host_done) hipEventDestroy(c->ct_host_done);
    if (c->asm_host_done) hipEventDestroy(c->asm_host_done);
    if (c->host_basis_done) hipEventDestroy(c->host_basis_done);
    if (c->b_host_done) hipEventDestroy(c->b_host_done);
    if (c->graph) hipGraphExecDestroy(c->graph);
    for (auto& rec : c->prof_pending) {
      hipEventDestroy(rec.a);
      hipEventDestroy(rec.b);
    }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  }
  delete c;
  return TAI_OK;
}

const char* tai_status_string(int status) {
  switch (status) {
    case TAI_OK: return "TAI_OK";
    case TAI_ERR_INVALID_ARG: return "TAI_ERR_INVALID_ARG: invalid argument";
    case TAI_ERR_NOMEM: return "TAI_ERR_NOMEM: workspace allocation failed or over the limit";
    case TAI_ERR_HIP: return "TAI_ERR_HIP: HIP runtime error";
    case TAI_ERR_UNSUPPORTED: return "TAI_ERR_UNSUPPORTED: unsupported combination";
    case TAI_ERR_NOT_READY: return "TAI_ERR_NOT_READY: context not usable";
    default: return "unknown tai status";
  }
}

const char* tai_last_error(const tai_ctx* c) { return c ? c->err.c_str() : ""; }

int tai_sync(tai_ctx* c, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = need_device(c))) return r;
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "pending error");
  return TAI_OK;
}

int tai_quadrature(tai_ctx* c, const tai_params* p, double* t, double* w, double* xi, double* K, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(p->nq, p->n)))) return r;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, p->nq, p->n);
  hipError_t e;
  {
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, p->nq, p->n, p->L, p->nodes, p->degree_tol, tb, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  const size_t nq = p->nq, n = p->n;
  if (t && (e = hipMemcpyAsync(t, tb.t, 8 * nq, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(c, e, "copy t");
  if (w && (e = hipMemcpyAsync(w, tb.w, 8 * nq, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(c, e, "copy w");
  if (xi && (e = hipMemcpyAsync(xi, tb.xi, 8 * n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(c, e, "copy xi");
  if (K && (e = hipMemcpyAsync(K, tb.K, 8 * nq * n * n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(c, e, "copy K");
  return TAI_OK;
}

int tai_degrees(tai_ctx* c, const tai_params* p, int32_t* nk, double* C, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!nk && !C) return fail(c, TAI_ERR_INVALID_ARG, "nk and C are both NULL");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(p->nq, p->n)))) return r;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, p->nq, p->n);
  hipError_t e;
  {
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, p->nq, p->n, p->L, p->nodes, 0.0, tb, s);
    if (e == hipSuccess) e = tai::launch_degrees(p->nq, p->n, p->nodes, p->degree_tol, tb, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "degrees kernel");
  const size_t nq = p->nq, n = p->n;
  if (nk && (e = hipMemcpyAsync(nk, tb.nk, 4 * nq, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(c, e, "copy nk");
  if (C && (e = hipMemcpyAsync(C, tb.C, 8 * nq * n * n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return hip_fail(c, e, "copy C");
  return TAI_OK;
}

static int compress_impl(tai_ctx* c, const double* M, int64_t npair, const tai_params* p, const NodeTables& tb,
                         bool operands, hipStream_t s, tai::CompressWork* w, int* R);

int tai_compress(tai_ctx* c, const double* M, int32_t npair, const tai_params* p, int32_t* rank, double* sigma,
                 double* V, double* U, double* Kc, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !rank) return fail(c, TAI_ERR_INVALID_ARG, "M or rank is NULL");
  if (npair < 1) return fail(c, TAI_ERR_INVALID_ARG, "npair must be >= 1");
  if (!(p->rank_tol > 0)) return fail(c, TAI_ERR_INVALID_ARG, "rank_tol must be > 0");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  tai::CompressWork w;
  int R = 0;
  hipError_t e;
  const bool operands = U || Kc;
  NodeTables tb{};
  if (operands) {
    if ((r = ensure(c, c->nodes, tai::node_tables_bytes(p->nq, p->n)))) return r;
    tb = tai::carve_node_tables(c->nodes.p, p->nq, p->n);
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, p->nq, p->n, p->L, p->nodes, p->degree_tol, tb, s);
    if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  }
  if ((r = compress_impl(c, M, npair, p, tb, operands, s, &w, &R))) return r;
  const size_t n = p->n;
  const size_t Rp = tai::padded_rank(R, p->n);
  if (sigma && (e = hipMemcpyAsync(sigma, w.sigma, 8 * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(c, e, "copy sigma");
  if (V && (e = hipMemcpyAsync(V, w.V, 8 * n * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(c, e, "copy V");
  if (U && (e = hipMemcpyAsync(U, c->cmpU.p, 8 * 3 * Rp * npair, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(c, e, "copy U");
  if (Kc && (e = hipMemcpyAsync(Kc, w.Kc, 8 * (size_t)p->nq * Rp * Rp, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(c, e, "copy Kc");
  *rank = R;
  return TAI_OK;
}

int tai_apply_J_compressed(tai_ctx* c, const double* U, int32_t nb, const int32_t* pairs, int32_t npk, int32_t R,
                           const double* Kc, const tai_params* p, const double* D, double* J, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!U || !Kc || !D || !J) return fail(c, TAI_ERR_INVALID_ARG, "U, Kc, D or J is NULL");
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  if (npair_of(nb) > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (pairs && (npk < 1 || npk > npair_of(nb))) return fail(c, TAI_ERR_INVALID_ARG, "npk must be in [1, npair]");
  if (R < 1 || R > p->n) return fail(c, TAI_ERR_INVALID_ARG, "R must be in [1, n]");
  if (!j_prec_ok(p->prec))
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J_compressed supports prec TAI_FP64, TAI_FP32, TAI_BF16X3 and TAI_BF16X6");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nq = p->nq;
  const int64_t npair = pairs ? npk : npair_of(nb);
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(nq, p->n)))) return r;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, nq, p->n);
  hipError_t e;
  {
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, nq, p->n, p->L, p->nodes, 0.0, tb, s);  // the weights w_k
  }
  if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  NodeTables tbp = tb;
  tbp.K = const_cast<double*>(Kc);
  const int Rp = tai::padded_rank(R, p->n);   // U and Kc are laid out at the padded length
  if ((r = ensure(c, c->jwork, tai::j_work_bytes(p->prec, nq, Rp, (int)npair)))) return r;
  tai::JWork w = tai::carve_j_work(c->jwork.p, p->prec, nq, Rp, (int)npair);
  {
    Timed tm(c, kStApplyJ, s);
    e = tai::launch_apply_j(p->prec, U, nb, (int)npair, pairs, Rp, nq, tbp, D, J, w, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "apply_J kernels");
  return TAI_OK;
}

// Copy a validated basis to the device (through pinned staging) on s.
static int upload_basis(tai_ctx* c, const tai_basis* b, hipStream_t s, tai::DevBasis* db) {
  int r;
  const size_t bb = basis_bytes(b->nb);
  if ((r = ensure(c, c->basis, bb))) return r;
  if ((r = ensure_host(c, c->host_basis, c->host_basis_done, bb))) return r;
  pack_basis_host(b, static_cast<char*>(c->host_basis.p));
  hipError_t e = hipMemcpyAsync(c->basis.p, c->host_basis.p, bb, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(c, e, "basis upload");
  if ((e = hipEventRecord(c->host_basis_done, s)) != hipSuccess) return hip_fail(c, e, "hipEventRecord");
  *db = dev_basis_view(b, static_cast<char*>(c->basis.p));
  return TAI_OK;
}

int tai_screen_pairs(tai_ctx* c, const tai_basis* b, double tau, int32_t* pairs, int32_t* nkept, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_basis(c, b))) return r;
  if (!std::isfinite(tau) || !(tau < 1.0)) return fail(c, TAI_ERR_INVALID_ARG, "tau must be finite and < 1");
  if (!pairs || !nkept) return fail(c, TAI_ERR_INVALID_ARG, "pairs or nkept is NULL");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  tai::DevBasis db;
  if ((r = upload_basis(c, b, s, &db))) return r;
  if ((r = ensure(c, c->screen, sizeof(int32_t) * ((size_t)b->nb + 2)))) return r;
  int32_t* rows = static_cast<int32_t*>(c->screen.p);
  int32_t* count = rows + b->nb + 1;
  hipError_t e;
  {
    Timed tm(c, kStMoments, s);
    e = tai::launch_screen(db, tau, rows, pairs, count, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "screening kernels");
  int32_t host = 0;
  if ((e = hipMemcpyAsync(&host, count, sizeof host, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "count copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  *nkept = host;
  return TAI_OK;
}

int tai_partition_pairs(tai_ctx* c, const tai_basis* b, double tau, int32_t nparts, int32_t* pairs, int32_t* counts,
                        double* boxes, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_basis(c, b))) return r;
  if (!std::isfinite(tau) || !(tau > 0.0) || !(tau < 1.0)) return fail(c, TAI_ERR_INVALID_ARG, "tau must be in (0, 1)");
  if (nparts < 1 || nparts > tai::kMaxParts)
    return fail(c, TAI_ERR_INVALID_ARG, "nparts must be in [1, " + std::to_string(tai::kMaxParts) + "]");
  if (!pairs || !counts || !boxes) return fail(c, TAI_ERR_INVALID_ARG, "pairs, counts or boxes is NULL");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  tai::DevBasis db;
  if ((r = upload_basis(c, b, s, &db))) return r;
  if ((r = ensure(c, c->part, tai::partition_work_bytes(b->nb, nparts)))) return r;
  const tai::PartWork w = tai::carve_partition_work(c->part.p, b->nb, nparts);
  hipError_t e;
  {
    Timed tm(c, kStMoments, s);
    e = tai::launch_partition(db, std::log(1.0 / tau), nparts, w, pairs, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "partition kernels");
  double hb[tai::kMaxParts];
  int32_t hc[tai::kMaxParts];
  if ((e = hipMemcpyAsync(hb, w.boxes, sizeof(double) * nparts, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "boxes copy");
  if ((e = hipMemcpyAsync(hc, w.totals, sizeof(int32_t) * nparts, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "counts copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  for (int i = 0; i < nparts; ++i) {
    boxes[i] = hb[i];
    counts[i] = hc[i];
  }
  return TAI_OK;
}

int tai_moments_partitioned(tai_ctx* c, const tai_basis* b, const tai_params* p, const int32_t* pairs,
                            const int32_t* counts, const double* boxes, int32_t nparts, double* M, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_basis(c, b))) return r;
  if ((r = validate_params(c, p, false))) return r;
  if (!M || !pairs || !counts || !boxes) return fail(c, TAI_ERR_INVALID_ARG, "a pointer is NULL");
  if (nparts < 1 || nparts > tai::kMaxParts)
    return fail(c, TAI_ERR_INVALID_ARG, "nparts must be in [1, " + std::to_string(tai::kMaxParts) + "]");
  tai::PartSpans sp{};
  sp.off[0] = 0;
  for (int i = 0; i < nparts; ++i) {
    if (counts[i] < 0) return fail(c, TAI_ERR_INVALID_ARG, "counts must be >= 0");
    if (!std::isfinite(boxes[i]) || !(boxes[i] > 0)) return fail(c, TAI_ERR_INVALID_ARG, "boxes must be finite and > 0");
    sp.off[i + 1] = sp.off[i] + counts[i];
    sp.L[i] = boxes[i];
  }
  if (sp.off[nparts] < 1 || sp.off[nparts] > npair_of(b->nb))
    return fail(c, TAI_ERR_INVALID_ARG, "the partition counts must add up to a number in [1, npair]");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(p->nq, p->n)))) return r;
  tai::DevBasis db;
  if ((r = upload_basis(c, b, s, &db))) return r;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, p->nq, p->n);
  hipError_t e;
  {
    // the node map and the panel rule of the moments do not depend on the box
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, p->nq, p->n, boxes[nparts - 1], p->nodes, 0.0, tb, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  {
    Timed tm(c, kStMoments, s);
    e = tai::launch_moments_parts(db, p->n, tb, pairs, sp, nparts, M, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "moments kernel");
  return TAI_OK;
}

// B over adaptive boxes (section 6.2 with Theorem 3.1): for every pair of
// partitions s <= s' the columns' operand Y^(s,s')_{k,d} = (K_k^(s,s') M_d)^T
// of partition s' (the cross tables of the two boxes), then one persistent
// assembly launch over all blocks: the diagonal blocks s = s' as symmetric
// molecules, the others as rectangular blocks mirrored into B^T's block.
int tai_assemble_B_partitioned(tai_ctx* c, const double* M, const int32_t* counts, const double* boxes,
                               int32_t nparts, const tai_params* p, void* B, int64_t ldb, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p, false))) return r;
  if (!M || !counts || !boxes || !B) return fail(c, TAI_ERR_INVALID_ARG, "a pointer is NULL");
  if (nparts < 1 || nparts > tai::kMaxParts)
    return fail(c, TAI_ERR_INVALID_ARG, "nparts must be in [1, " + std::to_string(tai::kMaxParts) + "]");
  int64_t offs[tai::kMaxParts + 1];
  offs[0] = 0;
  tai::PartBoxes bx{};
  bx.nparts = nparts;
  for (int i = 0; i < nparts; ++i) {
    if (counts[i] < 0) return fail(c, TAI_ERR_INVALID_ARG, "counts must be >= 0");
    if (!std::isfinite(boxes[i]) || !(boxes[i] > 0)) return fail(c, TAI_ERR_INVALID_ARG, "boxes must be finite and > 0");
    offs[i + 1] = offs[i] + counts[i];
    bx.b[i] = boxes[i];
  }
  const int64_t total = offs[nparts];
  if (total < 1 || total > 2147483647LL)
    return fail(c, TAI_ERR_INVALID_ARG, "the partition counts must add up to a number in [1, 2^31-1]");
  if (ldb < total) return fail(c, TAI_ERR_INVALID_ARG, "ldb must be >= the total pair count");
  if (p->rank_tol > 0 || p->degree_tol > 0)
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_assemble_B_partitioned: rank_tol and degree_tol must be 0");
  const int prec = p->prec, n = p->n, nq = p->nq;
  if ((r = need_device(c))) return r;
  c->size_key = pow2_at_least(total);
  const bool p16 = use16(c, prec, n, nq), p32 = !p16 && use32(prec, n);
  if (!p16 && !p32)
    return fail(c, TAI_ERR_UNSUPPORTED,
                "tai_assemble_B_partitioned runs on the persistent kernels only (FP64 and FP32 up to their inner "
                "length, the split 16-bit forms with a shape for nq)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(nq, n)))) return r;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, nq, n);
  // workspace: cross tables, then per partition A and exponents, then the
  // column operands of the blocks s <= s'
  int prow[tai::kMaxParts];
  size_t oA[tai::kMaxParts], oE[tai::kMaxParts], oY[tai::kMaxParts * tai::kMaxParts];
  const size_t kx_bytes = align256(sizeof(double) * (size_t)nparts * nparts * nq * n * n);
  size_t bytes = kx_bytes;
  for (int i = 0; i < nparts; ++i) {
    prow[i] = prow_of(c, prec, n, nq, std::max<int64_t>(1, counts[i]));
    oA[i] = bytes;
    bytes += opA_bytes(prec, n, prow[i]);
    oE[i] = bytes;
    bytes += opEx_bytes(prow[i]);
  }
  for (int i = 0; i < nparts; ++i)
    for (int j = i; j < nparts; ++j) {
      oY[i * nparts + j] = bytes;
      if (counts[i] > 0 && counts[j] > 0) bytes += opY_bytes(prec, n, nq, prow[j]);
    }
  if ((r = ensure(c, c->partB, bytes))) return r;
  char* base = static_cast<char*>(c->partB.p);
  double* Kx = reinterpret_cast<double*>(base);
  const int ysh = tai::y_shift(prec, p->omega, nq);
  const size_t es = prec == tai::kFP64 ? 8 : 4;
  hipError_t e;
  {
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, nq, n, boxes[nparts - 1], p->nodes, 0.0, tb, s);
    if (e == hipSuccess) e = tai::launch_cross_tables(tb.t, nq, n, p->nodes, bx, Kx, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "node kernels");
  for (int i = 0; i < nparts && e == hipSuccess; ++i) {
    if (counts[i] == 0) continue;
    Timed tm(c, kStPack, s);
    e = tai::launch_pack(prec, M + 3 * (int64_t)n * offs[i], n, counts[i], prow[i], base + oA[i],
                         reinterpret_cast<int32_t*>(base + oE[i]), s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "pack kernel");
  std::vector<tai::AsmMol> am;
  for (int i = 0; i < nparts && e == hipSuccess; ++i)
    for (int j = i; j < nparts && e == hipSuccess; ++j) {
      if (counts[i] == 0 || counts[j] == 0) continue;
      // Y of the columns (partition j) through K^(i,j): rows on box i's grid
      NodeTables tbp = tb;
      tbp.K = Kx + ((int64_t)i * nparts + j) * nq * n * n;
      {
        Timed tm(c, kStProject, s);
        e = tai::launch_project(prec, M + 3 * (int64_t)n * offs[j], n, counts[j], prow[j], nq, tbp,
                                reinterpret_cast<int32_t*>(base + oE[j]), ysh, base + oY[i * nparts + j], s);
      }
      tai::AsmMol m;
      m.A = base + oA[i];
      m.Y = base + oY[i * nparts + j];
      m.ex = reinterpret_cast<int32_t*>(base + oE[i]);
      m.B = static_cast<char*>(B) + ((int64_t)offs[i] * ldb + offs[j]) * es;
      m.ldb = ldb;
      m.npair = counts[i];
      m.prow = prow[i];
      m.nq = nq;
      m.kc = tai::operand_kc(prec, n);
      m.tiles = prow[i] / tai::assemble_tile(prec);
      m.tile0 = 0;
      m.nk = nullptr;
      m.ysh = ysh;
      if (i != j) {
        m.rect = 1;
        m.exc = reinterpret_cast<int32_t*>(base + oE[j]);
        m.pcol = prow[j];
        m.ncol = counts[j];
        m.Bt = static_cast<char*>(B) + ((int64_t)offs[j] * ldb + offs[i]) * es;
      }
      am.push_back(m);
    }
  if (e != hipSuccess) return hip_fail(c, e, "project kernel");
  Items16 items;
  const tai::Asm16Shape sh = p16 ? shape16(c, prec, n, nq) : tai::Asm16Shape{};
  const int64_t R = p16 ? sh.rows : ring_rows(prec, n), Cc = p16 ? sh.cols : tai::kAsm32Cols;
  const int64_t slots = (int64_t)(c->cus > 0 ? c->cus : 256) * (p16 ? sh.wgs_per_cu : 1);
  for (size_t k = 0; k < am.size(); ++k) {
    if (am[k].rect) items.add_rect((int)k, am[k].npair, am[k].ncol, R, Cc, 2 * slots / (int64_t)am.size());
    else items.add((int)k, am[k].npair, R, Cc, 2 * slots / (int64_t)am.size());
  }
  const size_t mol_bytes = align256(sizeof(tai::AsmMol) * am.size());
  const size_t tab_bytes = mol_bytes + items.bytes();
  if ((r = ensure(c, c->asm_tab, tab_bytes))) return r;
  if ((r = ensure(c, c->asm_counter, 256))) return r;
  if ((r = ensure_host(c, c->asm_host, c->asm_host_done, tab_bytes))) return r;
  char* hb = static_cast<char*>(c->asm_host.p);
  std::memcpy(hb, am.data(), sizeof(tai::AsmMol) * am.size());
  items.write(hb + mol_bytes);
  if ((e = hipMemcpyAsync(c->asm_tab.p, hb, tab_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(c, e, "table upload");
  if ((e = hipEventRecord(c->asm_host_done, s)) != hipSuccess) return hip_fail(c, e, "hipEventRecord");
  unsigned* counter = static_cast<unsigned*>(c->asm_counter.p);
  if ((e = tai::launch_reset_counter(counter, s)) != hipSuccess) return hip_fail(c, e, "reset kernel");
  const int nitems = (int)items.count();
  const int nblocks = (int)std::min<int64_t>(nitems, slots);
  const auto* mols_dev = static_cast<const tai::AsmMol*>(c->asm_tab.p);
  const char* tab = static_cast<const char*>(c->asm_tab.p) + mol_bytes;
  const auto* seg_dev = reinterpret_cast<const int*>(tab);
  const auto* items_dev = reinterpret_cast<const int4*>(tab + Items16::seg_bytes());
  {
    Timed tm(c, kStAssemble, s);
    if (p16)
      e = tai::launch_assemble16(prec, tai::operand_kc(prec, n), tai::operand_dup_chunks(prec, n), sh, mols_dev,
                                 items_dev, seg_dev, counter, nblocks, s);
    else
      e = launch_ring(prec, tai::operand_kc(prec, n), false, mols_dev, items_dev, seg_dev, counter, nblocks, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "assemble kernel");
  return TAI_OK;
}

int tai_apply_J_partitioned(tai_ctx* c, const double* M, int32_t nb, const int32_t* pairs, const int32_t* counts,
                            const double* boxes, int32_t nparts, const tai_params* p, const double* D, double* J,
                            void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p, false))) return r;
  if (!M || !pairs || !counts || !boxes || !D || !J) return fail(c, TAI_ERR_INVALID_ARG, "a pointer is NULL");
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  const int64_t npair = npair_of(nb);
  if (npair > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (nparts < 1 || nparts > tai::kMaxParts)
    return fail(c, TAI_ERR_INVALID_ARG, "nparts must be in [1, " + std::to_string(tai::kMaxParts) + "]");
  int64_t offs[tai::kMaxParts + 1];
  offs[0] = 0;
  tai::PartBoxes bx{};
  bx.nparts = nparts;
  for (int i = 0; i < nparts; ++i) {
    if (counts[i] < 0) return fail(c, TAI_ERR_INVALID_ARG, "counts must be >= 0");
    if (!std::isfinite(boxes[i]) || !(boxes[i] > 0)) return fail(c, TAI_ERR_INVALID_ARG, "boxes must be finite and > 0");
    offs[i + 1] = offs[i] + counts[i];
    bx.b[i] = boxes[i];
  }
  if (offs[nparts] != npair) return fail(c, TAI_ERR_INVALID_ARG, "the partition counts must add up to npair");
  if (!j_prec_ok(p->prec))
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J_partitioned supports prec TAI_FP64, TAI_FP32, TAI_BF16X3 and TAI_BF16X6");
  if (p->rank_tol > 0 || p->degree_tol > 0)
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J_partitioned: rank_tol and degree_tol must be 0");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nq = p->nq, n = p->n;
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(nq, n)))) return r;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, nq, n);
  const size_t n3 = (size_t)n * n * n;
  const size_t jb = align256(tai::j_work_bytes(p->prec, nq, n, (int)npair));
  // rho and Phi of every box; the node products of every box pair
  const size_t rb = align256(8 * n3 * nparts), tb2 = align256(8 * n3 * nq * nparts * nparts),
               wb = align256(8 * nq * nparts);
  const size_t kb = align256(8 * (size_t)nparts * nparts * nq * n * n);
  if ((r = ensure(c, c->partJ, jb + rb * 2 + tb2 + wb + kb))) return r;
  char* base = static_cast<char*>(c->partJ.p);
  tai::JWork w = tai::carve_j_work(base, p->prec, nq, n, (int)npair);
  double* rho_all = reinterpret_cast<double*>(base + jb);
  double* Phi_all = reinterpret_cast<double*>(base + jb + rb);
  double* T2_all = reinterpret_cast<double*>(base + jb + 2 * rb);
  double* wrep = reinterpret_cast<double*>(base + jb + 2 * rb + tb2);
  double* Kx = reinterpret_cast<double*>(base + jb + 2 * rb + tb2 + wb);
  hipError_t e;
  {
    Timed tm(c, kStNodes, s);
    // t_k, w_k (the plain tables on the largest box are not used)
    e = tai::launch_nodes(p->omega, nq, n, boxes[nparts - 1], p->nodes, 0.0, tb, s);
    if (e == hipSuccess) e = tai::launch_cross_tables(tb.t, nq, n, p->nodes, bx, Kx, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "node kernels");
  {
    Timed tm(c, kStApplyJ, s);
    e = tai::launch_apply_j_parts(p->prec, M, nb, pairs, offs, nparts, n, nq, tb.w, Kx, D, J, w, rho_all, T2_all,
                                  Phi_all, wrep, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "partitioned apply_J kernels");
  return TAI_OK;
}

static int moments_impl(tai_ctx* c, const tai_basis* b, const tai_params* p, const int32_t* pairs, int64_t npk,
                        double* M, hipStream_t s) {
  int r;
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(p->nq, p->n)))) return r;
  tai::DevBasis db;
  if ((r = upload_basis(c, b, s, &db))) return r;
  hipError_t e;
  NodeTables tb = tai::carve_node_tables(c->nodes.p, p->nq, p->n);
  {
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, p->nq, p->n, p->L, p->nodes, 0.0, tb, s);  // the moments need no K tables
  }
  if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  {
    Timed tm(c, kStMoments, s);
    e = tai::launch_moments_pairs(db, p->n, p->L, tb, pairs, npk, M, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "moments kernel");
  return TAI_OK;
}

int tai_moments(tai_ctx* c, const tai_basis* b, const tai_params* p, double* M, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_basis(c, b))) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M) return fail(c, TAI_ERR_INVALID_ARG, "M is NULL");
  if ((r = need_device(c))) return r;
  return moments_impl(c, b, p, nullptr, npair_of(b->nb), M, static_cast<hipStream_t>(stream));
}

int tai_moments_pairs(tai_ctx* c, const tai_basis* b, const tai_params* p, const int32_t* pairs, int32_t npk,
                      double* M, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_basis(c, b))) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !pairs) return fail(c, TAI_ERR_INVALID_ARG, "pairs or M is NULL");
  if (npk < 1 || npk > npair_of(b->nb)) return fail(c, TAI_ERR_INVALID_ARG, "npk must be in [1, npair]");
  if ((r = need_device(c))) return r;
  return moments_impl(c, b, p, pairs, npk, M, static_cast<hipStream_t>(stream));
}

// Low-rank compression of the moments (section 6.1, eqs. SVD and
// approxepsilon) on s: basis and rank, then the compressed moments
// (c->cmpU, [3][R][npair]) and tables (w->Kc, [nq][R][R]) from the node tables
// tb.  The call waits on the host for the rank.
static int compress_impl(tai_ctx* c, const double* M, int64_t npair, const tai_params* p, const NodeTables& tb,
                         bool operands, hipStream_t s, tai::CompressWork* w, int* R) {
  int r;
  const int n = p->n, nq = p->nq;
  if ((r = ensure(c, c->cmp, tai::compress_work_bytes(n, nq, npair)))) return r;
  if ((r = ensure(c, c->cmpU, sizeof(double) * 3 * (size_t)n * npair))) return r;
  *w = tai::carve_compress_work(c->cmp.p, n, nq, npair);
  hipError_t e;
  {
    Timed tm(c, kStCompress, s);
    e = tai::launch_compress_basis(M, n, npair, p->rank_tol, *w, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "compression basis kernels");
  int32_t host = 0;
  if ((e = hipMemcpyAsync(&host, w->rank, sizeof host, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(c, e, "rank copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  if (host < 1 || host > n) return fail(c, TAI_ERR_HIP, "compression rank out of range");
  *R = host;
  if (!operands) return TAI_OK;
  {
    Timed tm(c, kStCompress, s);
    e = tai::launch_compress_operands(M, n, npair, tai::padded_rank(host, n), host, nq, tb.K, *w,
                                      static_cast<double*>(c->cmpU.p), s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "compression operand kernels");
  return TAI_OK;
}

// Node tables of p on s, then the operands a path contracts: M, n and the K
// tables, or with p->rank_tol > 0 the compressed U, R and Kc.
static int prepare_operands(tai_ctx* c, const double* M, int64_t npair, const tai_params* p, hipStream_t s,
                            NodeTables* tb, const double** Mop, int* ne, NodeTables* tbp) {
  int r;
  if ((r = ensure(c, c->nodes, tai::node_tables_bytes(p->nq, p->n)))) return r;
  *tb = tai::carve_node_tables(c->nodes.p, p->nq, p->n);
  hipError_t e;
  {
    Timed tm(c, kStNodes, s);
    e = tai::launch_nodes(p->omega, p->nq, p->n, p->L, p->nodes, p->degree_tol, *tb, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  *Mop = M;
  *ne = p->n;
  *tbp = *tb;
  if (p->rank_tol > 0) {
    tai::CompressWork w;
    if ((r = compress_impl(c, M, npair, p, *tb, true, s, &w, ne))) return r;
    *ne = tai::padded_rank(*ne, p->n);   // the zero-padded inner length of U and Kc
    *Mop = static_cast<const double*>(c->cmpU.p);
    tbp->K = w.Kc;
  }
  return TAI_OK;
}

static int assemble_impl(tai_ctx* c, const double* M, int32_t npair, const tai_params* p, void* B, int64_t ldb,
                         hipStream_t s) {
  int r;
  const int prec = p->prec, nq = p->nq;
  NodeTables tb, tbp;
  const double* Mop = M;
  int n = p->n;
  if ((r = prepare_operands(c, M, npair, p, s, &tb, &Mop, &n, &tbp))) return r;
  // per-node degrees in FP64 / FP32: operands in coefficient form (moments
  // against T_j and the kept coefficients), each node contracting its
  // leading N_k indices.  The split 16-bit arithmetics keep the node form
  // with the truncated K tables: in coefficient form the moments of narrow
  // pairs cancel across indices and the slices lose about a factor of three
  // in accuracy.
  // With rank_tol > 0 the compressed tables already hold the truncated
  // factors (Kc_k = V^T Kt_k V) and the operands are U, not moments: the
  // node form throughout.
  const bool deg = p->degree_tol > 0 && !tai::is_split16(prec) && !(p->rank_tol > 0);
  const int prow = prow_of(c, prec, n, nq, npair);
  if ((r = ensure(c, c->opA, opA_bytes(prec, n, prow)))) return r;
  if ((r = ensure(c, c->opEx, opEx_bytes(prow)))) return r;
  if ((r = ensure(c, c->opY, opY_bytes(prec, n, nq, prow)))) return r;
  if (deg && (r = ensure(c, c->opMu, sizeof(double) * 3 * (size_t)n * npair))) return r;
  hipError_t e;
  int32_t* ex = static_cast<int32_t*>(c->opEx.p);
  if (deg) {
    double* mu = static_cast<double*>(c->opMu.p);
    {
      Timed tm(c, kStPack, s);
      e = tai::launch_coef_moments(M, n, npair, p->nodes, mu, s);
    }
    if (e != hipSuccess) return hip_fail(c, e, "coefficient moments kernel");
    Mop = mu;
    tbp.K = tb.C;
  }
  {
    Timed tm(c, kStPack, s);
    e = tai::launch_pack(prec, Mop, n, npair, prow, c->opA.p, ex, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "pack kernel");
  {
    Timed tm(c, kStProject, s);
    e = tai::launch_project(prec, Mop, n, npair, prow, nq, tbp, ex, tai::y_shift(prec, p->omega, nq), c->opY.p, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "project kernel");
  tai::AsmMol m;
  m.A = c->opA.p;
  m.Y = c->opY.p;
  m.ex = ex;
  m.B = B;
  m.ldb = ldb;
  m.npair = npair;
  m.prow = prow;
  m.nq = nq;
  m.kc = tai::operand_kc(prec, n);
  m.tiles = prow / tai::assemble_tile(prec);
  m.tile0 = 0;
  m.nk = deg ? tb.nk : nullptr;
  m.ysh = tai::y_shift(prec, p->omega, nq);
  const bool p16 = use16(c, prec, n, nq), p32 = !p16 && use32(prec, n);
  if (p16 || p32) {
    Items16 items;
    const tai::Asm16Shape sh = p16 ? shape16(c, prec, n, nq) : tai::Asm16Shape{};
    const int64_t slots = (int64_t)(c->cus > 0 ? c->cus : 256) * (p16 ? sh.wgs_per_cu : 1);
    if (p16) items.add(0, npair, sh.rows, sh.cols, 2 * slots);
    else items.add(0, npair, ring_rows(prec, n), tai::kAsm32Cols, 2 * slots);
    const size_t tab_bytes = align256(sizeof(tai::AsmMol)) + items.bytes();
    if ((r = ensure(c, c->asm_tab, tab_bytes))) return r;
    if ((r = ensure(c, c->asm_counter, 256))) return r;
    if ((r = ensure_host(c, c->asm_host, c->asm_host_done, tab_bytes))) return r;
    char* hb = static_cast<char*>(c->asm_host.p);
    std::memcpy(hb, &m, sizeof m);
    items.write(hb + align256(sizeof(tai::AsmMol)));
    if ((e = hipMemcpyAsync(c->asm_tab.p, hb, tab_bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(c, e, "table upload");
    if ((e = hipEventRecord(c->asm_host_done, s)) != hipSuccess) return hip_fail(c, e, "hipEventRecord");
    unsigned* counter = static_cast<unsigned*>(c->asm_counter.p);
    if ((e = tai::launch_reset_counter(counter, s)) != hipSuccess) return hip_fail(c, e, "reset kernel");
    const int nitems = (int)items.count();
    const int nblocks = std::min(nitems, (c->cus > 0 ? c->cus : 256) * (p16 ? sh.wgs_per_cu : 1));
    const auto* mols_dev = static_cast<const tai::AsmMol*>(c->asm_tab.p);
    const char* tab = static_cast<const char*>(c->asm_tab.p) + align256(sizeof(tai::AsmMol));
    const auto* seg_dev = reinterpret_cast<const int*>(tab);
    const auto* items_dev = reinterpret_cast<const int4*>(tab + Items16::seg_bytes());
    {
      Timed tm(c, kStAssemble, s);
      if (p16)
        e = tai::launch_assemble16(prec, m.kc, tai::operand_dup_chunks(prec, n), sh, mols_dev, items_dev, seg_dev,
                                   counter, nblocks, s);
      else
        e = launch_ring(prec, m.kc, deg, mols_dev, items_dev, seg_dev, counter, nblocks, s);
    }
  } else {
    Timed tm(c, kStAssemble, s);
    e = tai::launch_assemble(prec, m, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "assemble kernel");
  return TAI_OK;
}

int tai_assemble_B(tai_ctx* c, const double* M, int32_t npair, const tai_params* p, void* B, int64_t ldb,
                   void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !B) return fail(c, TAI_ERR_INVALID_ARG, "M or B is NULL");
  if (npair < 1) return fail(c, TAI_ERR_INVALID_ARG, "npair must be >= 1");
  if (ldb < npair) return fail(c, TAI_ERR_INVALID_ARG, "ldb must be >= npair");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  c->size_key = pow2_at_least(npair);
  if (c->tune_mode == 1 && tunable(p->prec, p->n) && !(p->rank_tol > 0)) {
    r = tune16(c, p->prec, p->n, p->nq, s, [&]() { return assemble_impl(c, M, npair, p, B, ldb, s); });
    if (r) return r;
  }
  return assemble_impl(c, M, npair, p, B, ldb, s);
}

static int batched_impl(tai_ctx* c, int32_t nmol, const tai_mol* mols, hipStream_t s, bool allow_graph);

int tai_assemble_B_batched(tai_ctx* c, int32_t nmol, const tai_mol* mols, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if (nmol < 1 || nmol > 65535 || !mols)
    return fail(c, TAI_ERR_INVALID_ARG, "nmol must be in 1..65535 and mols non-NULL");
  for (int i = 0; i < nmol; ++i) {
    if ((r = validate_basis(c, &mols[i].basis))) return fail(c, r, "molecule " + std::to_string(i) + ": " + c->err);
    if ((r = validate_params(c, &mols[i].params))) return fail(c, r, "molecule " + std::to_string(i) + ": " + c->err);
    if (!mols[i].M || !mols[i].B) return fail(c, TAI_ERR_INVALID_ARG, "molecule " + std::to_string(i) + ": M or B is NULL");
    if (mols[i].ldb < npair_of(mols[i].basis.nb))
      return fail(c, TAI_ERR_INVALID_ARG, "molecule " + std::to_string(i) + ": ldb must be >= npair");
    const tai_params& p0 = mols[0].params;
    const tai_params& pi = mols[i].params;
    if (pi.nq != p0.nq || pi.n != p0.n || pi.nodes != p0.nodes || pi.prec != p0.prec)
      return fail(c, TAI_ERR_INVALID_ARG, "molecules of a batch must share nq, n, nodes and prec");
  }
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // size class of a batch: a hash of its molecule sizes
  uint64_t h = 1469598103934665603ull ^ (uint64_t)nmol;
  for (int i = 0; i < nmol; ++i) h = (h ^ (uint64_t)mols[i].basis.nb) * 1099511628211ull;
  c->size_key = h | (1ull << 63);
  const tai_params& p0 = mols[0].params;
  if (c->tune_mode == 1 && tunable(p0.prec, p0.n)) {
    r = tune16(c, p0.prec, p0.n, p0.nq, s, [&]() { return batched_impl(c, nmol, mols, s, false); });
    if (r) return r;
  }
  return batched_impl(c, nmol, mols, s, true);
}

static int batched_impl(tai_ctx* c, int32_t nmol, const tai_mol* mols, hipStream_t s, bool allow_graph) {
  int r;
  const int prec = mols[0].params.prec, n = mols[0].params.n, nq = mols[0].params.nq;
  const int tile = tai::assemble_tile(prec);
  // molecules with per-node degrees take their operands in coefficient form
  // in FP64 / FP32 (the split arithmetics keep the node form, see assemble_impl)
  // Molecules with rank_tol > 0 are compressed on the device (no host wait
  // for their ranks): operands at the full length n with zero directions
  // beyond the rank, which the FP64 / FP32 kernels skip node by node.
  auto compressed = [&](int i) { return mols[i].params.rank_tol > 0; };
  auto coef_form = [&](int i) {
    return mols[i].params.degree_tol > 0 && !tai::is_split16(prec) && !compressed(i);
  };
  bool any_degree = false, any_tol = false, any_cmp = false;
  for (int i = 0; i < nmol; ++i) {
    any_degree = any_degree || coef_form(i);
    any_tol = any_tol || mols[i].params.degree_tol > 0;
    any_cmp = any_cmp || compressed(i);
  }

  // layout of the batch workspace
  std::vector<size_t> off_nodes(nmol), off_basis(nmol), off_A(nmol), off_Ex(nmol), off_Y(nmol), off_Mu(nmol),
      off_cmp(nmol);
  std::vector<int> prow(nmol);
  size_t sz_nodes = 0, sz_basis = 0, sz_A = 0, sz_Ex = 0, sz_Y = 0, sz_Mu = 0, sz_cmp = 0;
  int64_t nitems = 0;
  std::vector<tai::AsmMol> am(nmol);
  for (int i = 0; i < nmol; ++i) {
    const int64_t np = npair_of(mols[i].basis.nb);
    prow[i] = prow_of(c, prec, n, nq, np);
    off_nodes[i] = sz_nodes; sz_nodes += align256(tai::node_tables_bytes(nq, n));
    off_basis[i] = sz_basis; sz_basis += basis_bytes(mols[i].basis.nb);
    off_A[i] = sz_A; sz_A += opA_bytes(prec, n, prow[i]);
    off_Ex[i] = sz_Ex; sz_Ex += opEx_bytes(prow[i]);
    off_Y[i] = sz_Y; sz_Y += opY_bytes(prec, n, nq, prow[i]);
    off_Mu[i] = sz_Mu;
    if (coef_form(i)) sz_Mu += align256(sizeof(double) * 3 * (size_t)n * np);
    off_cmp[i] = sz_cmp;
    if (compressed(i)) sz_cmp += align256(tai::cmp_mol_bytes(n, nq, np)) + align256(sizeof(int32_t) * nq);
  }
  if ((r = ensure(c, c->b_nodes, sz_nodes))) return r;
  if ((r = ensure(c, c->b_basis, sz_basis))) return r;
  if ((r = ensure(c, c->b_opA, sz_A))) return r;
  if ((r = ensure(c, c->b_opEx, sz_Ex))) return r;
  if ((r = ensure(c, c->b_opY, sz_Y))) return r;
  if (sz_Mu > 0 && (r = ensure(c, c->b_opMu, sz_Mu))) return r;
  if (sz_cmp > 0 && (r = ensure(c, c->b_cmp, sz_cmp))) return r;
  if ((r = ensure(c, c->b_counter, 256))) return r;
  for (int i = 0; i < nmol; ++i) {
    tai::AsmMol& m = am[i];
    m.A = static_cast<char*>(c->b_opA.p) + off_A[i];
    m.Y = static_cast<char*>(c->b_opY.p) + off_Y[i];
    m.ex = reinterpret_cast<const int32_t*>(static_cast<char*>(c->b_opEx.p) + off_Ex[i]);
    m.B = mols[i].B;
    m.ldb = mols[i].ldb;
    m.npair = (int32_t)npair_of(mols[i].basis.nb);
    m.prow = prow[i];
    m.nq = nq;
    m.kc = tai::operand_kc(prec, n);
    m.tiles = prow[i] / tile;
    m.tile0 = nitems;
    nitems += (int64_t)m.tiles * (m.tiles + 1) / 2;
    m.nk = nullptr;  // set below from the molecule's node tables
    m.ysh = tai::y_shift(prec, mols[i].params.omega, nq);
  }
  // the 16-bit kernel drains (molecule, row panel, column range) items,
  // largest molecules first so the tail of the queue holds small items
  const bool split16 = use16(c, prec, n, nq);
  const bool fp32p = !split16 && use32(prec, n);
  Items16 items16;
  const tai::Asm16Shape sh16 = split16 ? shape16(c, prec, n, nq) : tai::Asm16Shape{};
  if (split16 || fp32p) {
    std::vector<int> order(nmol);
    for (int i = 0; i < nmol; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return am[a].npair > am[b].npair; });
    const int kc = tai::operand_kc(prec, n);
    for (int i : order)
      items16.add(i, am[i].npair, split16 ? sh16.rows : ring_rows(prec, n), split16 ? sh16.cols : tai::kAsm32Cols);
  }
  // device tables: [AsmMol x nmol | PrepMol x nmol | CmpMol x ncm | items]
  const size_t off_prep = align256(sizeof(tai::AsmMol) * nmol);
  int ncm = 0;
  for (int i = 0; i < nmol; ++i) ncm += compressed(i) ? 1 : 0;
  const size_t off_cmptab = off_prep + align256(sizeof(tai::PrepMol) * nmol);
  const size_t off_items = off_cmptab + align256(sizeof(tai::CmpMol) * (ncm > 0 ? ncm : 1));
  const size_t tab_bytes = off_items + (split16 || fp32p ? items16.bytes() : 0);
  if ((r = ensure(c, c->b_mols, tab_bytes))) return r;
  std::vector<tai::PrepMol> prep(nmol);
  std::vector<tai::CmpMol> cmp;
  int64_t max_npair = 0, max_npair_cmp = 0;
  int max_prow = 0, max_nchunk = 0;
  for (int i = 0; i < nmol; ++i) {
    tai::PrepMol& q = prep[i];
    q.omega = mols[i].params.omega;
    q.L = mols[i].params.L;
    q.degree_tol = mols[i].params.degree_tol;
    q.tb = tai::carve_node_tables(static_cast<char*>(c->b_nodes.p) + off_nodes[i], nq, n);
    q.Mu = coef_form(i) ? reinterpret_cast<double*>(static_cast<char*>(c->b_opMu.p) + off_Mu[i]) : nullptr;
    am[i].nk = q.Mu ? q.tb.nk : nullptr;
    q.U = nullptr;
    q.Kc = nullptr;
    if (compressed(i)) {
      char* cb = static_cast<char*>(c->b_cmp.p) + off_cmp[i];
      int32_t* nk = reinterpret_cast<int32_t*>(cb + align256(tai::cmp_mol_bytes(n, nq, am[i].npair)));
      tai::CmpMol cm = tai::carve_cmp_mol(cb, n, nq, am[i].npair, mols[i].M, mols[i].params.rank_tol, q.tb.K,
                                          tai::is_split16(prec) ? nullptr : nk);
      q.U = cm.U;
      q.Kc = cm.Kc;
      am[i].nk = cm.nk;
      cmp.push_back(cm);
      max_npair_cmp = std::max<int64_t>(max_npair_cmp, am[i].npair);
      max_nchunk = std::max(max_nchunk, (int)cm.nchunk);
    }
    q.basis = dev_basis_view(&mols[i].basis, static_cast<char*>(c->b_basis.p) + off_basis[i]);
    q.M = mols[i].M;
    q.npair = am[i].npair;
    q.prow = prow[i];
    q.A = const_cast<void*>(am[i].A);
    q.ex = const_cast<int32_t*>(am[i].ex);
    q.Y = const_cast<void*>(am[i].Y);
    q.ysh = am[i].ysh;
    max_npair = std::max<int64_t>(max_npair, am[i].npair);
    max_prow = std::max(max_prow, prow[i]);
  }

  // upload bases, the molecule table and the items (outside any graph)
  const size_t host_bytes = sz_basis + tab_bytes;
  if ((r = ensure_host(c, c->b_host, c->b_host_done, host_bytes))) return r;
  char* hb = static_cast<char*>(c->b_host.p);
  for (int i = 0; i < nmol; ++i) pack_basis_host(&mols[i].basis, hb + off_basis[i]);
  std::memcpy(hb + sz_basis, am.data(), sizeof(tai::AsmMol) * nmol);
  std::memcpy(hb + sz_basis + off_prep, prep.data(), sizeof(tai::PrepMol) * nmol);
  if (ncm > 0) std::memcpy(hb + sz_basis + off_cmptab, cmp.data(), sizeof(tai::CmpMol) * ncm);
  if (split16 || fp32p) items16.write(hb + sz_basis + off_items);
  hipError_t e = hipMemcpyAsync(c->b_basis.p, hb, sz_basis, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->b_mols.p, hb + sz_basis, tab_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(c->b_host_done, s);
  if (e != hipSuccess) return hip_fail(c, e, "batch upload");

  // the kernel sequence; recorded into a graph when a stream is given
  auto enqueue = [&](hipStream_t st) -> hipError_t {
    // preparation of every molecule, one launch per stage
    const auto* prep_dev = reinterpret_cast<const tai::PrepMol*>(static_cast<char*>(c->b_mols.p) + off_prep);
    hipError_t err = tai::launch_nodes_batch(prep_dev, nmol, nq, n, mols[0].params.nodes, any_tol, st);
    if (err == hipSuccess) err = tai::launch_moments_batch(prep_dev, nmol, max_npair, n, st);
    if (err == hipSuccess && ncm > 0) {
      const auto* cmp_dev = reinterpret_cast<const tai::CmpMol*>(static_cast<char*>(c->b_mols.p) + off_cmptab);
      err = tai::launch_compress_batch(cmp_dev, ncm, n, nq, max_npair_cmp, max_nchunk, st);
    }
    if (err == hipSuccess && any_degree)
      err = tai::launch_coef_moments_batch(prep_dev, nmol, max_npair, n, mols[0].params.nodes, st);
    if (err == hipSuccess) err = tai::launch_pack_batch(prec, prep_dev, nmol, max_prow, n, st);
    if (err == hipSuccess) err = tai::launch_project_batch(prec, prep_dev, nmol, max_prow, n, nq, st);
    if (err != hipSuccess) return err;
    unsigned* counter = static_cast<unsigned*>(c->b_counter.p);
    err = tai::launch_reset_counter(counter, st);
    if (err != hipSuccess) return err;
    const auto* mols_dev = static_cast<const tai::AsmMol*>(c->b_mols.p);
    if (split16 || fp32p) {
      const char* tab = static_cast<const char*>(c->b_mols.p) + off_items;
      const auto* seg_dev = reinterpret_cast<const int*>(tab);
      const auto* items_dev = reinterpret_cast<const int4*>(tab + Items16::seg_bytes());
      const int ni = (int)items16.count();
      const int blocks = std::min(ni, (c->cus > 0 ? c->cus : 256) * (split16 ? sh16.wgs_per_cu : 1));
      if (fp32p)
        return launch_ring(prec, am[0].kc, any_degree || any_cmp, mols_dev, items_dev, seg_dev, counter, blocks, st);
      return tai::launch_assemble16(prec, am[0].kc, tai::operand_dup_chunks(prec, n), sh16, mols_dev, items_dev,
                                    seg_dev, counter, blocks, st);
    }
    int blocks = tai::assemble_queue_blocks(prec, c->device);
    if (blocks > nitems) blocks = (int)nitems;
    return tai::launch_assemble_queue(prec, am[0].kc, any_degree || any_cmp, mols_dev, nmol, nitems, counter, blocks,
                                      st);
  };

  const bool use_graph = allow_graph && s != nullptr && !std::getenv("TAI_NO_GRAPH");
  if (!use_graph) {
    {
      Timed tm(c, kStBatched, s);
      e = enqueue(s);
    }
    if (e != hipSuccess) return hip_fail(c, e, "batched launch");
    return TAI_OK;
  }
  // graph key: everything the recorded kernels capture by value
  std::vector<unsigned char> key;
  auto put = [&key](const void* v, size_t nbytes) {
    const unsigned char* b = static_cast<const unsigned char*>(v);
    key.insert(key.end(), b, b + nbytes);
  };
  put(&nmol, sizeof nmol);
  for (int i = 0; i < nmol; ++i) {
    put(&mols[i].params, sizeof(tai_params));
    put(&mols[i].basis.nb, sizeof(int32_t));
    const int has_coef = mols[i].basis.coef != nullptr;
    put(&has_coef, sizeof has_coef);
    put(&mols[i].M, sizeof(void*));
    put(&mols[i].B, sizeof(void*));
    put(&mols[i].ldb, sizeof(int64_t));
  }
  void* bases[] = {c->b_nodes.p, c->b_basis.p, c->b_opA.p, c->b_opEx.p, c->b_opY.p, c->b_opMu.p, c->b_mols.p,
                   c->b_counter.p, c->b_cmp.p};
  put(bases, sizeof bases);
  put(&sh16.id, sizeof sh16.id);
  if (!c->graph || key != c->graph_key) {
    if (c->graph) {
      hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) return hip_fail(c, e, "begin capture");
    hipError_t le = enqueue(s);
    e = hipStreamEndCapture(s, &g);
    if (le != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return hip_fail(c, le, "batched capture");
    }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph = nullptr;
      return hip_fail(c, e, "graph instantiate");
    }
    c->graph_key = key;
  }
  {
    Timed tm(c, kStBatched, s);
    e = hipGraphLaunch(c->graph, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "graph launch");
  return TAI_OK;
}

static int apply_j_impl(tai_ctx* c, const double* M, int32_t nb, const int32_t* pairs, int64_t npair,
                        const tai_params* p, const double* D, double* J, void* stream) {
  int r;
  if (!j_prec_ok(p->prec))
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J supports prec TAI_FP64, TAI_FP32, TAI_BF16X3 and TAI_BF16X6");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nq = p->nq;
  NodeTables tb, tbp;
  const double* Mop = M;
  int n = p->n;
  if ((r = prepare_operands(c, M, npair, p, s, &tb, &Mop, &n, &tbp))) return r;
  if ((r = ensure(c, c->jwork, tai::j_work_bytes(p->prec, nq, n, (int)npair)))) return r;
  hipError_t e;
  tai::JWork w = tai::carve_j_work(c->jwork.p, p->prec, nq, n, (int)npair);
  {
    Timed tm(c, kStApplyJ, s);
    e = tai::launch_apply_j(p->prec, Mop, nb, (int)npair, pairs, n, nq, tbp, D, J, w, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "apply_J kernels");
  return TAI_OK;
}

int tai_apply_J_noalloc(tai_ctx* c, const double* M, int32_t nb, const tai_params* p, const double* D, double* J,
                        void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !D || !J) return fail(c, TAI_ERR_INVALID_ARG, "M, D or J is NULL");
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  const int64_t npair = npair_of(nb);
  if (npair > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (p->prec != TAI_FP64 && p->prec != TAI_FP32)
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J_noalloc supports prec TAI_FP64 and TAI_FP32");
  if (p->rank_tol > 0)
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J_noalloc: rank_tol > 0 needs the compression workspace");
  const int nq = p->nq, n = p->n;
  const size_t tab = align256(tai::node_tables_bytes(nq, n));
  const size_t need = tab + tai::j_work_bytes(p->prec, nq, n, (int)npair);
  if (need > kScratchBytes)
    return fail(c, TAI_ERR_INVALID_ARG, "tai_apply_J_noalloc needs " + std::to_string(need) +
                                            " bytes of scratch; the static scratch holds " +
                                            std::to_string(kScratchBytes));
  if ((r = need_device(c))) return r;
  if (!c->scratch) return fail(c, TAI_ERR_HIP, "the static scratch has no device address on this device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(c->scratch);
  NodeTables tb = tai::carve_node_tables(base, nq, n);
  tai::JWork w = tai::carve_j_work(base + tab, p->prec, nq, n, (int)npair);
  hipError_t e = tai::launch_nodes(p->omega, nq, n, p->L, p->nodes, p->degree_tol, tb, s);
  if (e != hipSuccess) return hip_fail(c, e, "nodes kernel");
  e = tai::launch_apply_j(p->prec, M, nb, (int)npair, nullptr, n, nq, tb, D, J, w, s);
  if (e != hipSuccess) return hip_fail(c, e, "apply_J kernels");
  return TAI_OK;
}

int tai_apply_J(tai_ctx* c, const double* M, int32_t nb, const tai_params* p, const double* D, double* J,
                void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !D || !J) return fail(c, TAI_ERR_INVALID_ARG, "M, D or J is NULL");
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  const int64_t npair = npair_of(nb);
  if (npair > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  return apply_j_impl(c, M, nb, nullptr, npair, p, D, J, stream);
}

int tai_apply_J_pairs(tai_ctx* c, const double* M, int32_t nb, const int32_t* pairs, int32_t npk,
                      const tai_params* p, const double* D, double* J, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !D || !J || !pairs) return fail(c, TAI_ERR_INVALID_ARG, "M, pairs, D or J is NULL");
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  if (npair_of(nb) > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (npk < 1 || npk > npair_of(nb)) return fail(c, TAI_ERR_INVALID_ARG, "npk must be in [1, npair]");
  return apply_j_impl(c, M, nb, pairs, npk, p, D, J, stream);
}

int tai_coulomb_mo(tai_ctx* c, const double* M, int32_t nb, const int32_t* pairs, int32_t npk,
                   const tai_params* p, const double* Q, int32_t norb, double* Jmo, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !Q || !Jmo) return fail(c, TAI_ERR_INVALID_ARG, "M, Q or Jmo is NULL");
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "nb must be >= 1");
  if (npair_of(nb) > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (norb < 1 || norb > 1024) return fail(c, TAI_ERR_INVALID_ARG, "norb must be in [1, 1024]");
  if (pairs && (npk < 1 || npk > npair_of(nb))) return fail(c, TAI_ERR_INVALID_ARG, "npk must be in [1, npair]");
  if (p->prec != TAI_FP64 && p->prec != TAI_FP32)
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_coulomb_mo supports prec TAI_FP64 and TAI_FP32");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nq = p->nq;
  const int64_t npair = pairs ? npk : npair_of(nb);
  NodeTables tb, tbp;
  const double* Mop = M;
  int n = p->n;
  if ((r = prepare_operands(c, M, npair, p, s, &tb, &Mop, &n, &tbp))) return r;
  if ((r = ensure(c, c->jwork, tai::j_work_bytes(p->prec, nq, n, (int)npair)))) return r;
  const int cus = c->cus > 0 ? c->cus : 256;
  if ((r = ensure(c, c->mo, tai::mo_work_bytes(p->prec, n, nq, (int)npair, norb, cus)))) return r;
  hipError_t e;
  tai::JWork w = tai::carve_j_work(c->jwork.p, p->prec, nq, n, (int)npair);
  {
    Timed tm(c, kStApplyJ, s);
    e = tai::launch_coulomb_mo(p->prec, Mop, nb, (int)npair, pairs, n, nq, tbp, Q, norb, cus, c->mo.p, Jmo, w, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "coulomb_mo kernels");
  return TAI_OK;
}

int tai_exchange(tai_ctx* c, const double* M, int32_t nb, const int32_t* pairs, int32_t npk, const tai_params* p,
                 const double* Q, int32_t norb, double* Kx, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !Q || !Kx) return fail(c, TAI_ERR_INVALID_ARG, "M, Q or Kx is NULL");
  if (nb < 1 || nb > 65535) return fail(c, TAI_ERR_INVALID_ARG, "nb must be in [1, 65535]");
  if (npair_of(nb) > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "npair exceeds 2^31-1");
  if (norb < 1 || norb > 1024) return fail(c, TAI_ERR_INVALID_ARG, "norb must be in [1, 1024]");
  if (pairs && (npk < 1 || npk > npair_of(nb))) return fail(c, TAI_ERR_INVALID_ARG, "npk must be in [1, npair]");
  const double work = 16.0 * norb * (double)nb * p->n * p->n * p->n;
  if (work > 64.0 * (1ull << 30))
    return fail(c, TAI_ERR_INVALID_ARG, "norb * nb * n^3 too large: the X and Phi tensors exceed 64 GiB");
  if (p->prec != TAI_FP64 && p->prec != TAI_FP32)
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_exchange supports prec TAI_FP64 and TAI_FP32");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nq = p->nq;
  const int64_t npair = pairs ? npk : npair_of(nb);
  NodeTables tb, tbp;
  const double* Mop = M;
  int n = p->n;
  if ((r = prepare_operands(c, M, npair, p, s, &tb, &Mop, &n, &tbp))) return r;
  const tai::ExchangeWork plan = tai::exchange_work_plan(n, nq, nb, norb, pairs != nullptr, npair_of(nb));
  if ((r = ensure(c, c->mo, plan.bytes))) return r;
  hipError_t e;
  {
    Timed tm(c, kStApplyJ, s);
    e = tai::launch_exchange(p->prec, Mop, nb, npair, pairs, n, nq, tbp, Q, norb, c->mo.p, plan, Kx, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "exchange kernels");
  return TAI_OK;
}

// A contraction map: fmap[0] = 0 and each step adds 0 or 1 (primitives listed
// function by function, every function at least one); returns nb or 0.
static int32_t contraction_nb(const int32_t* fmap, int32_t nbp) {
  if (!fmap || nbp < 1 || fmap[0] != 0) return 0;
  for (int32_t i = 1; i < nbp; ++i)
    if (fmap[i] != fmap[i - 1] && fmap[i] != fmap[i - 1] + 1) return 0;
  return fmap[nbp - 1] + 1;
}

int tai_contract_pairs(tai_ctx* c, const void* Bp, int64_t ldbp, int32_t nbp, const int32_t* fmap, int32_t prec,
                       void* B, int64_t ldb, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if (!Bp || !B) return fail(c, TAI_ERR_INVALID_ARG, "Bp or B is NULL");
  if (nbp < 1 || npair_of(nbp) > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "nbp out of range");
  const int32_t nb = contraction_nb(fmap, nbp);
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "fmap must start at 0 and step by 0 or 1");
  const int64_t npp = npair_of(nbp), npc = npair_of(nb);
  if (ldbp < npp || ldb < npc) return fail(c, TAI_ERR_INVALID_ARG, "ldbp < npair(nbp) or ldb < npair(nb)");
  if (prec < TAI_FP64 || prec > TAI_F16X3) return fail(c, TAI_ERR_INVALID_ARG, "unknown prec");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // member lists of the contracted pairs (CSR over primitive pairs, row-major order)
  const size_t tab = align256(sizeof(int32_t) * (npc + 1)) + align256(sizeof(int32_t) * npp) +
                     align256(sizeof(double) * npp);
  if ((r = ensure(c, c->ct, tab))) return r;
  if ((r = ensure_host(c, c->ct_host, c->ct_host_done, tab))) return r;
  char* hb = static_cast<char*>(c->ct_host.p);
  int32_t* off = reinterpret_cast<int32_t*>(hb);
  int32_t* idx = reinterpret_cast<int32_t*>(hb + align256(sizeof(int32_t) * (npc + 1)));
  double* wt = reinterpret_cast<double*>(hb + align256(sizeof(int32_t) * (npc + 1)) + align256(sizeof(int32_t) * npp));
  std::vector<int64_t> P(npp);
  std::fill(off, off + npc + 1, 0);
  int64_t p = 0;
  for (int32_t i = 0; i < nbp; ++i)
    for (int32_t j = i; j < nbp; ++j, ++p) {
      const int64_t mu = fmap[i], nu = fmap[j];
      P[p] = mu * nb - mu * (mu - 1) / 2 + (nu - mu);
      ++off[P[p] + 1];
    }
  for (int64_t q = 0; q < npc; ++q) off[q + 1] += off[q];
  std::vector<int32_t> fill(off, off + npc);
  p = 0;
  for (int32_t i = 0; i < nbp; ++i)
    for (int32_t j = i; j < nbp; ++j, ++p) {
      const int32_t slot = fill[P[p]]++;
      idx[slot] = (int32_t)p;
      wt[slot] = (fmap[i] == fmap[j] && i != j) ? 2.0 : 1.0;
    }
  hipError_t e = hipMemcpyAsync(c->ct.p, hb, tab, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(c->ct_host_done, s);
  if (e != hipSuccess) return hip_fail(c, e, "contraction table upload");
  char* db = static_cast<char*>(c->ct.p);
  e = tai::launch_contract_pairs(prec == TAI_FP64, Bp, ldbp, reinterpret_cast<const int32_t*>(db),
                                 reinterpret_cast<const int32_t*>(db + align256(sizeof(int32_t) * (npc + 1))),
                                 reinterpret_cast<const double*>(db + align256(sizeof(int32_t) * (npc + 1)) +
                                                                 align256(sizeof(int32_t) * npp)),
                                 npc, B, ldb, s);
  if (e != hipSuccess) return hip_fail(c, e, "contraction kernel");
  return TAI_OK;
}

int tai_apply_J_contracted(tai_ctx* c, const double* M, int32_t nbp, const int32_t* fmap, const tai_params* p,
                           const double* D, double* J, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = validate_params(c, p))) return r;
  if (!M || !D || !J) return fail(c, TAI_ERR_INVALID_ARG, "M, D or J is NULL");
  if (nbp < 1 || npair_of(nbp) > 2147483647LL) return fail(c, TAI_ERR_INVALID_ARG, "nbp out of range");
  const int32_t nb = contraction_nb(fmap, nbp);
  if (nb < 1) return fail(c, TAI_ERR_INVALID_ARG, "fmap must start at 0 and step by 0 or 1");
  if (!j_prec_ok(p->prec))
    return fail(c, TAI_ERR_UNSUPPORTED, "tai_apply_J_contracted supports prec TAI_FP64, TAI_FP32, TAI_BF16X3 and TAI_BF16X6");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // device tables: fmap [nbp], first primitive of each function [nb + 1]
  const size_t tab = align256(sizeof(int32_t) * nbp) + align256(sizeof(int32_t) * (nb + 1));
  if ((r = ensure(c, c->ct, tab))) return r;
  if ((r = ensure_host(c, c->ct_host, c->ct_host_done, tab))) return r;
  char* hb = static_cast<char*>(c->ct_host.p);
  std::memcpy(hb, fmap, sizeof(int32_t) * nbp);
  int32_t* first = reinterpret_cast<int32_t*>(hb + align256(sizeof(int32_t) * nbp));
  first[0] = 0;
  for (int32_t i = 1; i < nbp; ++i)
    if (fmap[i] != fmap[i - 1]) first[fmap[i]] = i;
  first[nb] = nbp;
  hipError_t e = hipMemcpyAsync(c->ct.p, hb, tab, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(c->ct_host_done, s);
  if (e != hipSuccess) return hip_fail(c, e, "contraction table upload");
  const int32_t* fmap_d = static_cast<const int32_t*>(c->ct.p);
  const int32_t* first_d = reinterpret_cast<const int32_t*>(static_cast<char*>(c->ct.p) + align256(sizeof(int32_t) * nbp));
  const size_t nn = (size_t)nbp * nbp;
  if ((r = ensure(c, c->ct_work, 2 * sizeof(double) * nn))) return r;
  double* Dp = static_cast<double*>(c->ct_work.p);
  double* Jp = Dp + nn;
  if ((e = tai::launch_expand_density(D, nb, fmap_d, nbp, Dp, s)) != hipSuccess) return hip_fail(c, e, "expand density");
  if ((r = apply_j_impl(c, M, nbp, nullptr, npair_of(nbp), p, Dp, Jp, stream))) return r;
  if ((e = tai::launch_contract_functions(Jp, nbp, first_d, nb, J, s)) != hipSuccess)
    return hip_fail(c, e, "contract functions");
  return TAI_OK;
}

int tai_tune(tai_ctx* c, int mode) {
  int r = check_ctx(c);
  if (r) return r;
  if (mode < 0 || mode > 2) return fail(c, TAI_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
  if (mode == 2) c->tuned.clear();
  else c->tune_mode = mode;
  return TAI_OK;
}

int tai_peak_probe(tai_ctx* c, int what, double* value, void* stream) {
  int r = check_ctx(c);
  if (r) return r;
  if (what < 0 || what > 2) return fail(c, TAI_ERR_INVALID_ARG, "what must be 0, 1 or 2");
  if (!value) return fail(c, TAI_ERR_INVALID_ARG, "value is NULL");
  if ((r = need_device(c))) return r;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess || cus < 1) return hip_fail(c, e == hipSuccess ? hipErrorUnknown : e, "CU count");
  const int iters = what == 0 ? 20000 : 4000;
  const int64_t n16 = what == 2 ? (int64_t{1} << 26) : 0;  // 1 GiB each way
  float* out = nullptr;
  void* src = nullptr;
  void* dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 0.0;
  auto done = [&](int code) {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (out) hipFree(out);
    if (src) hipFree(src);
    if (dst) hipFree(dst);
    return code;
  };
  if (hipMalloc(&out, sizeof(float) * 2 * cus * 256) != hipSuccess ||
      (n16 && (hipMalloc(&src, 16 * n16) != hipSuccess || hipMalloc(&dst, 16 * n16) != hipSuccess))) {
    (void)hipGetLastError();
    return done(fail(c, TAI_ERR_NOMEM, "probe buffers"));
  }
  if (n16 && (e = hipMemsetAsync(src, 0, 16 * n16, s)) != hipSuccess) return done(hip_fail(c, e, "probe fill"));
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
    return done(hip_fail(c, e, "hipEventCreate"));
  for (int rep = 0; rep < 4; ++rep) {  // the first launch warms up and is not counted
    if ((e = hipEventRecord(e0, s)) != hipSuccess) return done(hip_fail(c, e, "hipEventRecord"));
    if ((e = tai::launch_probe(what, cus, out, src, dst, n16, iters, s)) != hipSuccess)
      return done(hip_fail(c, e, "probe launch"));
    if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
      return done(hip_fail(c, e, "probe timing"));
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return done(hip_fail(c, e, "hipEventElapsedTime"));
    if (rep > 0 && ms > 0.f) best = std::max(best, tai::probe_work(what, cus, n16, iters) / (ms * 1e-3));
  }
  *value = what == 2 ? best / 1e9 : best / 1e12;
  return done(TAI_OK);
}

int tai_profile_enable(tai_ctx* c, int enable) {
  int r = check_ctx(c);
  if (r) return r;
  if ((r = need_device(c))) return r;
  for (auto& rec : c->prof_pending) {
    hipEventSynchronize(rec.b);
    c->ev_pool.push_back(rec.a);
    c->ev_pool.push_back(rec.b);
  }
  c->prof_pending.clear();
  for (int i = 0; i < kNumStages; ++i) {
    c->prof_ms[i] = 0.0;
    c->prof_n[i] = 0;
  }
  c->prof_on = enable != 0;
  return TAI_OK;
}

int tai_profile_read(tai_ctx* c, const char* stage, double* total_ms, int64_t* count) {
  int r = check_ctx(c);
  if (r) return r;
  if (!stage || !total_ms || !count) return fail(c, TAI_ERR_INVALID_ARG, "stage, total_ms or count is NULL");
  int st = -1;
  for (int i = 0; i < kNumStages; ++i)
    if (std::strcmp(stage, kStageNames[i]) == 0) st = i;
  if (st < 0) return fail(c, TAI_ERR_INVALID_ARG, std::string("unknown stage ") + stage);
  if ((r = need_device(c))) return r;
  for (auto& rec : c->prof_pending) {
    hipError_t e = hipEventSynchronize(rec.b);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, rec.a, rec.b);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
    c->prof_ms[rec.stage] += ms;
    c->prof_n[rec.stage] += 1;
    c->ev_pool.push_back(rec.a);
    c->ev_pool.push_back(rec.b);
  }
  c->prof_pending.clear();
  *total_ms = c->prof_ms[st];
  *count = c->prof_n[st];
  return TAI_OK;
}

}  // extern "C"
