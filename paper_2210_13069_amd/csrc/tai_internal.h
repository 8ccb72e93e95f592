// Internal declarations shared by the host layer and the kernel files of
// libtai.  Not part of the public ABI (include/tai.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace tai {

enum Prec { kFP64 = 0, kFP32 = 1, kBF16X3 = 2, kBF16X6 = 3, kF16X3 = 4 };

// Composite Gauss-Legendre rule used for the 1D moments: the pair's support
// is split into kMomPanels equal panels of kMomOrder nodes each.
constexpr int kMomPanels = 4;
constexpr int kMomOrder = 24;

// Device-resident FP64 tables for one (omega, nq, n, L, nodes).
struct NodeTables {
  double* t;     // [nq]      Gauss-Legendre nodes on (0, omega)
  double* w;     // [nq]      weights
  double* xi;    // [n]       Chebyshev nodes on [-L, L]
  double* K;     // [nq][n][n] exp(-t_k^2 (xi_a - xi_b)^2)
  double* gam;   // [n][n]    Chebyshev-to-Lagrange map: l_a(x) = sum_k gam[a][k] T_k(x/L)
  double* pz;    // [kMomOrder] panel rule nodes on [-1, 1]
  double* pw;    // [kMomOrder] panel rule weights
  double* C;     // [nq][n][n] Chebyshev coefficients of each node's factor,
                 //            zero beyond its degree (launch_degrees)
  int32_t* nk;   // [nq]      per-node degree N_k (launch_degrees)
};

// Bytes needed by the node tables (each array 256-byte aligned).
size_t node_tables_bytes(int nq, int n);
NodeTables carve_node_tables(void* base, int nq, int n);

// Nodes, weights, Chebyshev nodes and K tables; with degree_tol > 0 also the
// per-node degrees, after which K holds the truncated tables (launch_degrees).
hipError_t launch_nodes(double omega, int nq, int n, double L, int kind, double degree_tol,
                        const NodeTables& tb, hipStream_t s);
// Per-node degree (eq. chebcheb with N_k points for node k): C_k, N_k, and,
// for degree_tol > 0, K_k replaced by the node values of the kept part.
// Needs the tables of launch_nodes.
hipError_t launch_degrees(int nq, int n, int kind, double degree_tol, const NodeTables& tb, hipStream_t s);

// Device copy of one molecule's basis.
struct DevBasis {
  int32_t nb;
  const double* center;   // [nb][3]
  const double* alpha;    // [nb]
  const int32_t* lxyz;    // [nb][3]
  const double* coef;     // [nb] or nullptr
};

hipError_t launch_moments(const DevBasis& b, int n, double L, const NodeTables& tb,
                          double* M, hipStream_t s);
// Moments of the listed pairs (indices into the full pair list; entries
// outside it give zero moments): M[d][a][i] for pair pairs[i], i < npk.
hipError_t launch_moments_pairs(const DevBasis& b, int n, double L, const NodeTables& tb, const int32_t* pairs,
                                int64_t npk, double* M, hipStream_t s);
// Screening (section 6.3): pair p(mu, nu) is kept when
// exp(-ab/(a+b) |A - B|^2) > tau (every pair when tau <= 0).  Writes the kept
// indices in ascending order to pairs and their count to *count (device);
// rows: device scratch of nb + 1 int32.
hipError_t launch_screen(const DevBasis& b, double tau, int32_t* rows, int32_t* pairs, int32_t* count,
                         hipStream_t s);
// Coefficient moments mu_d[j][p] = sum_a T_j(xi_a / L) M_d[a][p] (the
// moments against T_j, j < n), FP64.
hipError_t launch_coef_moments(const double* M, int n, int64_t npair, int kind, double* mu, hipStream_t s);

// ---- assembly -------------------------------------------------------------

// Length of one operand K-vector (all slices concatenated, zero padded).
int operand_kc(int prec, int n);

// Order of the inner (K) index of the split operands.  The three slice
// segments of the X3 modes (A = [s0|s0|s1], Y = [s0|s1|s0]) are laid out in
// groups of 8 so that, for n % 8 == 0, the first dup_chunks(n) 32-wide
// chunks of segment 0 and segment 1 sit in chunks c and c + Q: the A
// operand then has Q pairs of identical MFMA fragments, which the 16-bit
// kernel keeps in registers once.  Any such permutation of K, applied to A
// and Y alike, leaves every inner product unchanged.
//
// BF16X6 (A = [s0|s0|s1|s0|s1|s2], Y = [s0|s1|s0|s2|s1|s0]) with n % 8 == 0
// and n >= 32 takes the same idea with six segments: each of the first
// n / 32 full 32-index ranges r comes as six chunks, segment 0 .. 5 of its
// indices; chunks 6r, 6r+1, 6r+3 of A are then equal (s0), and 6r+2, 6r+4
// (s1), so A has three distinct fragments per range.  The remaining indices
// follow in groups of 8, the six segments of a group side by side.  Its
// shape key is kX6Key + n / 32.
constexpr int kX6Key = 100;
__host__ __device__ inline int operand_dup_chunks(int prec, int n) {
  if ((prec == kBF16X3 || prec == kF16X3) && n % 8 == 0) return n / 32;
  if (prec == kBF16X6 && n % 8 == 0 && n >= 32) return kX6Key + n / 32;
  return 0;
}
__host__ __device__ inline int seg_pos(int prec, int n, int s, int a) {
  const int Q = operand_dup_chunks(prec, n);
  if (Q >= kX6Key) {
    const int Q6 = Q - kX6Key, g = a >> 3, o = a & 7;
    const int p = g < 4 * Q6 ? 24 * (g >> 2) + 4 * s + (g & 3) : 24 * Q6 + 6 * (g - 4 * Q6) + s;
    return 8 * p + o;
  }
  if (Q == 0) return s * n + a;
  const int G = n / 8, g = a >> 3, o = a & 7;
  int p;
  if (s == 0) p = g < 4 * Q ? g : 8 * Q + (g - 4 * Q);
  else if (s == 1) p = g < 4 * Q ? 4 * Q + g : 8 * Q + (G - 4 * Q) + (g - 4 * Q);
  else p = 8 * Q + 2 * (G - 4 * Q) + g;
  return 8 * p + o;
}
// Bytes per operand element.
int operand_esize(int prec);
// Square output tile edge of the assembly kernel (rows of operands are
// padded to a multiple of it).
int assemble_tile(int prec);

struct AsmMol {
  // operands (device): A[d][prow][kc], Y[k][d][prow][kc]; prow = padded rows
  const void* A;
  const void* Y;
  const int32_t* ex;     // [3][prow] power-of-two exponents (zeros for FP64)
  void* B;               // output
  int64_t ldb;
  int32_t npair;
  int32_t prow;          // padded row count
  int32_t nq;
  int32_t kc;
  int32_t tiles;         // tiles per side
  int64_t tile0;         // first linear work item of this molecule
  // per-node degrees N_k [nq] when the operands are in coefficient form
  // (FP64 and FP32 only; nullptr: every node runs the full inner length)
  const int32_t* nk;
  // power of two folded into Y_{k,2} with w_k (y_shift); the column
  // exponents are lowered by it when B is scaled back
  int32_t ysh;
  // Rectangular block (the persistent ring and 16-bit kernels only): rows
  // from A (npair of them, exponents ex over prow), columns from Y (ncol of
  // them, padded count pcol, exponents exc), every entry computed, written
  // to B and mirrored to Bt (B^T's block).  rect 0: the symmetric block
  // (upper triangle, mirror into B itself; exc, pcol, ncol, Bt unused).
  int32_t rect = 0;
  const int32_t* exc = nullptr;
  int32_t pcol = 0;
  int32_t ncol = 0;
  void* Bt = nullptr;
};

// Per-molecule arguments of the preparation stages of a batch (nodes,
// moments, operand packing and projection), read by the batch kernels at
// blockIdx.y (nodes, moments) or blockIdx.z (pack, project).
struct PrepMol {
  double omega, L, degree_tol;
  NodeTables tb;
  DevBasis basis;
  double* M;
  double* Mu;            // coefficient moments (per-node degrees, FP64 and FP32), else nullptr
  const double* U;       // compressed moments [3][n][npair] (rank_tol > 0), else nullptr
  const double* Kc;      // their tables [nq][n][n]
  int64_t npair;
  int32_t prow;
  void* A;
  int32_t* ex;
  void* Y;
  int32_t ysh;           // y_shift of the molecule
};
// any_degree: some molecule has degree_tol > 0 (then the degree stage runs
// for the batch; molecules with degree_tol <= 0 keep their tables).
hipError_t launch_nodes_batch(const PrepMol* mols, int nmol, int nq, int n, int kind, bool any_degree,
                              hipStream_t s);
hipError_t launch_moments_batch(const PrepMol* mols, int nmol, int64_t max_npair, int n, hipStream_t s);
// launch_coef_moments for the molecules with PrepMol::Mu set.
hipError_t launch_coef_moments_batch(const PrepMol* mols, int nmol, int64_t max_npair, int n, int kind,
                                     hipStream_t s);
hipError_t launch_pack_batch(int prec, const PrepMol* mols, int nmol, int max_prow, int n, hipStream_t s);
hipError_t launch_project_batch(int prec, const PrepMol* mols, int nmol, int max_prow, int n, int nq,
                                hipStream_t s);

hipError_t launch_pack(int prec, const double* M, int n, int npair, int prow,
                       void* A, int32_t* ex, hipStream_t s);
hipError_t launch_project(int prec, const double* M, int n, int npair, int prow, int nq,
                          const NodeTables& tb, const int32_t* ex, int ysh, void* Y, hipStream_t s);
// Single molecule, one work group per tile.
hipError_t launch_assemble(int prec, const AsmMol& m, hipStream_t s);
// Persistent launch over a device work list of molecules; `counter` is a
// device int zeroed by launch_reset_counter before each launch (which
// zeroes the kAsm16Queues counters starting there).
hipError_t launch_assemble_queue(int prec, int kc, bool deg, const AsmMol* mols_dev, int nmol, int64_t nitems,
                                 unsigned* counter, int nblocks, hipStream_t s);
hipError_t launch_reset_counter(unsigned* counter, hipStream_t s);
int assemble_queue_blocks(int prec, int device);

// 16-bit split arithmetics: A-stationary persistent kernel over work items
// int4 {molecule, row panel, first column block, end column block}.  A shape
// fixes the waves per work group, the row blocks (16 rows) per wave, the
// column blocks (16 columns) per item block and the depth of the LDS ring;
// rows = 16 * rb * waves per panel, cols = 16 * cb per column block.
struct Asm16Shape {
  int id;          // index into the shape table (-1: none fits)
  int waves, rb, cb, nbuf;
  int nps;         // quadrature nodes per LDS ring step (nq must be a multiple, >= nbuf * nps)
  int rows, cols;  // panel rows, block columns
  int wgs_per_cu;  // resident work groups per CU (register / LDS bound)
  int kc_key, q_key;  // the (kc, q) the shape was chosen for
};
int asm16_max_kc();
// Shapes that compile for (kc, q), the table default first; asm16_shape
// returns candidate `pick` (0 if out of range) with its resident work
// groups per CU filled in from the runtime (device must be current).
int asm16_shapes(int kc, int q, Asm16Shape* out, int cap);
Asm16Shape asm16_shape(int kc, int q, int pick);
// The items are split into kAsm16Queues queues (one per XCD): queue x is
// items[seg[x] .. seg[x+1]); counters[x] are zeroed by launch_reset_counter.
constexpr int kAsm16Queues = 8;
hipError_t launch_assemble16(int prec, int kc, int q, const Asm16Shape& shape, const AsmMol* mols_dev,
                             const int4* items_dev, const int* seg_dev, unsigned* counters, int nblocks,
                             hipStream_t s);
inline bool is_split16(int prec) { return prec == kBF16X3 || prec == kBF16X6 || prec == kF16X3; }

// FP32 persistent kernel (k_assemble32.hip): the same items and queues as the
// 16-bit kernel, panels of asm32_rows(kc) rows, column blocks of 16; one work
// group of eight waves per CU.  kc a multiple of 8 up to 64.
constexpr int kAsm32Cols = 16;
constexpr int kAsm32MaxKc = 64;
int asm32_rows(int kc);
// The FP64 form: panels of asm64_rows(kc) rows.
int asm64_rows(int kc);
hipError_t launch_assemble64(int kc, bool deg, const AsmMol* mols_dev, const int4* items_dev, const int* seg_dev,
                             unsigned* counters, int nblocks, hipStream_t s);
// deg: the molecules may carry per-node degrees (AsmMol::nk).
hipError_t launch_assemble32(int kc, bool deg, const AsmMol* mols_dev, const int4* items_dev, const int* seg_dev,
                             unsigned* counters, int nblocks, hipStream_t s);

// ---- Coulomb matrix through the grid tensor --------------------------------

struct JWork {
  double* Dt;      // [npair]
  double* rho_part;// [nchunk][n^3]
  double* rho;     // [n^3]
  double* T1;      // [nq][n^3] slab products K_k rho(a0) K_k^T
  double* T2;      // [nq][n^3] mode-0 partial sums over runs of nodes
  double* wsc;     // [nq] quadrature weights times 2/sqrt(pi)
  double* Phi;     // [n^3]
  double* Jp;      // [npair]
  float* M32;      // [3][n][npair] FP32 copy of the moments (FP32 and split BF16, else null)
  void* Ps;        // [n][n][kc] bfloat16 slices of Phi (split BF16 only, else null)
  int nchunk;
};
int j_nchunk(int prec, int n, int npair);
size_t j_work_bytes(int prec, int nq, int n, int npair);
JWork carve_j_work(void* base, int prec, int nq, int n, int npair);
// Low-rank compression of the moments (k_compress.hip): Gram matrix of
// W = [M_1 | M_2 | M_3], its eigenpairs by Jacobi (V[a][r], sigma[r]
// decreasing, *rank = #{sigma_r > tol sigma_1}, at least 1), then compressed
// moments U[d][r][q] = sum_a V[a][r] M[d][a][q] and tables Kc[k] = V_R^T K[k] V_R.
struct CompressWork {
  double* part;    // [nchunk][n][n] partial Gram matrices
  double* G;       // [n][n]
  double* V;       // [n][n] the basis V1 V2
  double* V1;      // [n][n] eigenvectors of W W^T
  double* V2;      // [n][n] eigenvectors of Y Y^T, Y = V1^T W (never stored)
  double* sigma;   // [n]
  double* Kc;      // [nq][R][R]
  int32_t* rank;   // [1]
  int nchunk;
};
size_t compress_work_bytes(int n, int nq, int64_t npair);
CompressWork carve_compress_work(void* base, int n, int nq, int64_t npair);
hipError_t launch_compress_basis(const double* M, int n, int64_t npair, double tol, const CompressWork& w,
                                 hipStream_t s);
// U [3][R][npair] and Kc [nq][R][R] at inner length R with the basis columns
// from `keep` on taken as zero (keep <= R: the kept rank, R its padding).
hipError_t launch_compress_operands(const double* M, int n, int64_t npair, int R, int keep, int nq,
                                    const double* K, const CompressWork& w, double* U, hipStream_t s);
// One molecule of a batched compression: every buffer is the molecule's
// own, the rank stays on the device, and the operands are written at the
// full length n with the basis columns from the rank on taken as zero
// (U [3][n][npair], Kc [nq][n][n]); nk (if set) receives the rank for every
// node, the inner length the FP64 / FP32 assembly kernels then run.
struct CmpMol {
  const double* M;     // [3][n][npair] moments
  int64_t npair;
  int64_t chunk;       // pairs per Gram chunk
  int32_t nchunk;
  double tol;
  double* part;        // [n * n][nchunk]
  double* G;           // [n][n]
  double* V1;          // [n][n]
  double* V2;          // [n][n]
  double* V;           // [n][n]
  double* sigma;       // [n]
  int32_t* rank;       // [1]
  double* U;           // [3][n][npair]
  const double* K;     // [nq][n][n] the molecule's node tables
  double* Kc;          // [nq][n][n]
  int32_t* nk;         // [nq] or nullptr
};
// Bytes of one molecule's compression buffers (without the tables K), and
// its Gram chunking.
size_t cmp_mol_bytes(int n, int nq, int64_t npair);
CmpMol carve_cmp_mol(void* base, int n, int nq, int64_t npair, const double* M, double tol, const double* K,
                     int32_t* nk);
// The whole compression of ncm molecules (tab on the device), no host wait.
hipError_t launch_compress_batch(const CmpMol* tab, int ncm, int n, int nq, int64_t max_npair, int max_nchunk,
                                 hipStream_t s);

// Power of two 2^ysh that the projection folds into Y_{k,2} together with
// the quadrature weight w_k, so that the split 16-bit operands stay clear of
// the FP16 subnormals: without it w_k (about omega pi / (2 nq), 1e-3 .. 3e-2)
// pushes the low slice of every Y_{k,2} entry below FP16's smallest normal.
// ysh puts the largest weight near [8, 16); products of a B entry stay far
// below FP32 and FP16 overflow (|Y| <= 16 n).  Zero for FP64 and FP32.  The
// value is any power of two of that size: the assembly lowers every column
// exponent by ysh, which is exact.
inline int y_shift(int prec, double omega, int nq) {
  if (prec == 0 || prec == 1) return 0;
  const double west = 0.5 * omega * 3.141592653589793 / (nq + 0.5);
  return 3 - ilogb(west);
}

// Inner length the compressed operands of kept rank R are written at.
inline int padded_rank(int R, int n) {
  const int r8 = (R + 7) / 8 * 8;
  return r8 < n ? r8 : n;
}

// Contracted basis functions (k_contract.hip).  B_c[P][Q] = sum over the
// CSR members a of P and b of Q of wt[a] wt[b] Bp[idx[a]][idx[b]] (double or
// float matrices, FP64 sums); D_prim[i][j] = D[fmap[i]][fmap[j]];
// J[mu][nu] = sum of Jp over primitives first[mu] .. first[mu+1] by first[nu] .. first[nu+1].
hipError_t launch_contract_pairs(bool fp64, const void* Bp, int64_t ldbp, const int32_t* off, const int32_t* idx,
                                 const double* wt, int64_t npc, void* B, int64_t ldb, hipStream_t s);
hipError_t launch_expand_density(const double* D, int nb, const int32_t* fmap, int nbp, double* Dp, hipStream_t s);
hipError_t launch_contract_functions(const double* Jp, int nbp, const int32_t* first, int nb, double* J,
                                     hipStream_t s);
// Coulomb matrix in the orbital basis: per orbital i (row i of Q, length nb)
// the pair density of q_i q_i^T, rho_i and Phi_i (n^3 each) for blocks of
// orbitals at a time, then Jmo[i][j] = <rho_i, Phi_j>.  work: mo_work_bytes.
// cus: compute units of the device (the pair contraction's chunking).
size_t mo_work_bytes(int prec, int n, int nq, int npair, int norb, int cus);
hipError_t launch_coulomb_mo(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                             const NodeTables& tb, const double* Q, int norb, int cus, void* work, double* Jmo,
                             const JWork& w, hipStream_t s);
// Long-range exchange matrix (appendix B): X_{j mu} and Phi_{j nu} for every
// orbital j and function mu into R and F ([norb][nb][n^3] each), then
// Kx(mu, nu) = 2 sum_j <X_{j mu}, Phi_{j nu}>.
// Adaptive integration boxes (section 6.2, k_partition.hip): the pair
// supports, equal-count quantile boxes (sorted supports), the partitions'
// pair lists (concatenated, each ascending) and the cross tables between the
// boxes' Chebyshev grids.
constexpr int kMaxParts = 16;
struct PartBoxes {
  double b[kMaxParts];
  int nparts;
};
// The partitions' spans of the concatenated pair list (off[s] .. off[s+1])
// and their box half-widths, passed by value to the batched moments kernel.
struct PartSpans {
  int64_t off[kMaxParts + 1];
  double L[kMaxParts];
};
// Moments of every partition's pairs on its own box (k_moments.hip): block s
// of M = [3][n][counts[s]] at M + 3 n off[s], the pairs pairs[off[s] ..),
// box [-L[s], L[s]]; one launch, the partition as a grid dimension.
hipError_t launch_moments_parts(const DevBasis& b, int n, const NodeTables& tb, const int32_t* pairs,
                                const PartSpans& sp, int nparts, double* M, hipStream_t s);
struct PartWork {
  double* sup;        // [npair] support half-widths
  double* sorted;     // [npair]
  int32_t* counts;    // [nparts][nb] per-row counts, then list offsets
  double* boxes;      // [nparts] box half-widths
  int32_t* totals;    // [nparts] pairs per partition
  void* temp;         // sort workspace
  size_t temp_bytes;
};
size_t partition_work_bytes(int nb, int nparts);
PartWork carve_partition_work(void* base, int nb, int nparts);
// c = ln(1/tau)
hipError_t launch_partition(const DevBasis& bs, double c, int nparts, const PartWork& w, int32_t* pairs,
                            hipStream_t s);
// Kx[s nparts + s'][k][a][b] = exp(-t_k^2 (b_s xi_a - b_s' xi_b)^2), xi the unit Chebyshev nodes
hipError_t launch_cross_tables(const double* t, int nq, int n, int kind, const PartBoxes& bx, double* Kx,
                               hipStream_t s);
// J over adaptive boxes: M holds the partitions' moment blocks [3][n][count_s]
// one after another (each on its own box), pairs the concatenated lists.
// Kx from launch_cross_tables; w the node weights.
hipError_t launch_apply_j_parts(int prec, const double* M, int nb, const int32_t* pairs, const int64_t* offs,
                                int nparts, int n, int nq, const double* w, const double* Kx, const double* D,
                                double* J, const JWork& wk, double* rho_all, double* T2_all, double* Phi_all,
                                double* wrep, hipStream_t s);

// Exchange matrix, factorized form (k_exchange.hip).  exchange_work_plan
// lays out one workspace: the X and Phi grid tensors of all norb nb
// (orbital, function) slots, the slab products of a chunk of tensors (at
// most 4 GiB), the partial sums of the final product and, for a screened
// pair list, the inverse map of the list.
struct ExchangeWork {
  int64_t ntensor, tchunk, slice;
  int nsplit;
  size_t off_X, off_Phi, off_T1, off_part, off_inv, bytes;
};
ExchangeWork exchange_work_plan(int n, int nq, int nb, int norb, bool listed, int64_t npair_full);
// Mode products on the FP64 matrix cores for many tensors (k_exchange.hip):
// slab products T1[t][k][a0] = K_k X_t(a0) K_k^T for T tensors, tensor t
// reading X[t % xmod] and the tables K + t kstride; then for T0 groups of
// consecutive T1 blocks, Phi_g = sum_k w_k K_k x_0 (group g's nq0 node
// blocks, tables K + g kstride0), without the factor 2/sqrt(pi).  part
// (part_len doubles, may be null) lets a launch with few groups split the
// node sum into runs whose partial Phi are then added in order.
hipError_t launch_mode_products(const double* X, int64_t T, int64_t xmod, const double* K, int64_t kstride,
                                const double* w, int n, int nq, double* T1, int64_t T0, int64_t kstride0,
                                int nq0, double* Phi, double* part, int64_t part_len, hipStream_t s);
hipError_t launch_exchange(int prec, const double* M, int nb, int64_t npair, const int32_t* pairs, int n, int nq,
                           const NodeTables& tb, const double* Q, int norb, void* work, const ExchangeWork& p,
                           double* Kx, hipStream_t s);
// Achievable-peak probes (k_probe.hip): what 0 = FP16 MFMA, 1 = FP64 MFMA,
// 2 = HBM copy.  probe_work is the flops (0, 1) or bytes (2) of one launch.
hipError_t launch_probe(int what, int cus, float* out, const void* src, void* dst, int64_t n16, int iters,
                        hipStream_t s);
double probe_work(int what, int cus, int64_t n16, int iters);

// pairs: nullptr (all pairs), or the screened list: M holds the moments of
// pairs[0 .. npair), and the J entries of the other pairs are set to zero.
hipError_t launch_apply_j(int prec, const double* M, int nb, int npair, const int32_t* pairs, int n, int nq,
                          const NodeTables& tb, const double* D, double* J,
                          const JWork& w, hipStream_t s);

}  // namespace tai
