/*
 * tai.h -- C ABI of the MI355X (gfx950) library for the tensorized
 * approximation (TA) of the long-range two-electron integrals tensor
 * (Badreddine, Chollet, Grigori, arXiv 2210.13069).
 *
 * Method (section 3 of the paper).  The long-range kernel is written as
 *     erf(w r)/r = (2/sqrt(pi)) int_0^w exp(-s^2 r^2) ds             (eq. kernel)
 * and discretised by Gauss-Legendre nodes t_k, weights w_k on [0, w]
 * (eq. TEI2).  Each 1D factor exp(-t_k^2 (x-y)^2) on the box [-L,L]^2 is
 * replaced by its tensor Chebyshev interpolant (eq. chebcheb), kept here in
 * node-value (Lagrange) form with the n x n matrices
 *     K_k(a,b) = exp(-t_k^2 (xi_a - xi_b)^2),
 * xi_a the Chebyshev nodes on [-L,L].  With the 1D moments of every basis pair
 * p = (mu,nu), mu <= nu, against the Lagrange basis l_a (eq. defV),
 *     m_{p,d}(a) = int_{-L}^{L} g_{mu,d}(x) g_{nu,d}(x) l_a(x) dx,
 * Theorem 3.1 with eq. tensors gives
 *     B(p,q) = (2/sqrt(pi)) sum_k w_k prod_{d=1..3} m_{p,d}^T K_k m_{q,d}.
 * The Coulomb matrix (eqs. Coul, coulapprox; atomic-orbital form)
 *     J(mu,nu) = sum over all ordered (k,l) of B(mu nu, k l) D(k,l)
 * is applied through the n^3 Chebyshev-grid tensor (eq. ig1), never forming B.
 *
 * Conventions for every entry point
 *   - Return value: TAI_OK (0) or a negative TAI_ERR_* code; nothing throws
 *     across the ABI.  tai_last_error() gives a message for the last failure
 *     on a context.
 *   - Arguments are validated before any device work; on TAI_ERR_INVALID_ARG
 *     and TAI_ERR_UNSUPPORTED no output is written.
 *   - Pointers marked DEVICE are device memory owned by the caller, on the
 *     context's device; HOST pointers are read during the call only.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     stream-ordered and asynchronous: they return once the work is enqueued.
 *     A device fault surfaces from a later call or from tai_sync().
 *   - A context owns its workspace and caches; it is not thread-safe (use one
 *     context per host thread).  Calls on one context that run concurrently
 *     on different streams must not overlap in time, since they share the
 *     context's workspace.
 *   - Pair index (0-based, mu <= nu, row-major upper triangle):
 *         p(mu,nu) = mu*nb - mu*(mu-1)/2 + (nu - mu),  npair = nb*(nb+1)/2.
 */
#ifndef TAI_H
#define TAI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TAI_OK = 0,
  TAI_ERR_INVALID_ARG = -1,   /* a bad argument; nothing was written           */
  TAI_ERR_NOMEM = -2,         /* workspace allocation failed or over the limit
                                 set by the environment variable
                                 TAI_WORKSPACE_LIMIT (bytes)                   */
  TAI_ERR_HIP = -3,           /* a HIP runtime error (launch, fault, ...)      */
  TAI_ERR_UNSUPPORTED = -4,   /* valid but unsupported combination             */
  TAI_ERR_NOT_READY = -5      /* context not usable (e.g. failed creation)     */
};

/* Chebyshev node family (Def. 2.2): Lobatto (second kind) is the paper's
   choice for TA (remark closing section 4.3); Gauss is the first kind. */
enum { TAI_NODES_LOBATTO = 0, TAI_NODES_GAUSS = 1 };

/* Arithmetic of the B contraction (tai_assemble_B) and of the grid
   projections of tai_apply_J.  Node generation, moments and the K tables are
   FP64 in every mode; the cross-k accumulation of B is FP32 within the
   low-precision modes and FP64 for TAI_FP64.
     TAI_FP64   FP64 MFMA.
     TAI_FP32   FP32 MFMA.
     TAI_BF16X3 each operand split into 2 bfloat16 slices, 3 products
                (hi*hi + hi*lo + lo*hi), FP32 MFMA accumulation.
     TAI_BF16X6 3 bfloat16 slices, 6 products.
     TAI_F16X3  2 float16 slices, 3 products; operands are scaled per
                (pair, direction) by powers of two so the slices stay in range.
   Low-precision modes write B as float32. */
enum { TAI_FP64 = 0, TAI_FP32 = 1, TAI_BF16X3 = 2, TAI_BF16X6 = 3, TAI_F16X3 = 4 };

/* One molecule's basis: nb functions, each ONE primitive Cartesian Gaussian
     g_mu(x) = c_mu prod_d (x_d - A_mu,d)^{l_mu,d} exp(-alpha_mu |x - A_mu|^2)
   (eqs. basis and primi with I_mu = 1).  HOST pointers. */
typedef struct {
  int32_t        nb;      /* 1 <= nb, npair = nb(nb+1)/2 <= 2^31 - 1          */
  const double*  center;  /* [nb][3], finite                                  */
  const double*  alpha;   /* [nb], finite and > 0                             */
  const int32_t* lxyz;    /* [nb][3], each power in 0..4                      */
  const double*  coef;    /* [nb] multiplier c_mu, or NULL: then c_mu makes
                             each Cartesian factor unit-norm,
                             prod_d [(2a/pi)^(1/2) (4a)^l / (2l-1)!!]^(1/2)   */
} tai_basis;

/* Method parameters.  omega > 0; 1 <= nq <= 128 Gauss-Legendre nodes in t;
   2 <= n <= 64 Chebyshev nodes per direction; L > 0 the half-width of the box
   [-L,L]^3 (the paper's b, eq. compact); nodes and prec from the enums.
   degree_tol >= 0 (finite) selects a degree per quadrature node (the
   paper's N_i, eq. chebcheb): 0 keeps every node at n; with degree_tol > 0
   node k keeps the Chebyshev coefficients of its factor below N_k, the
   smallest degree whose dropped coefficients sum in absolute value to at
   most degree_tol, so each factor moves by at most degree_tol on the box
   (tai_degrees).  Every entry point then uses the truncated factors.
   rank_tol in [0, 1) selects the low-rank compression of the moments
   (section 6.1, eqs. SVD and approxepsilon): 0 keeps the n node values;
   with rank_tol > 0 tai_assemble_B, tai_apply_J(_pairs), tai_apply_J_contracted
   and tai_coulomb_mo contract U_d = V^T M_d and Kc_k = V^T K_k V instead,
   V the R leading left singular vectors of [M_1 | M_2 | M_3] with
   sigma_r > rank_tol * sigma_1 (tai_compress); those calls then wait on the
   host for R.  Both together: the moments are compressed as above and the
   tables are those of the truncated factors, Kc_k = V^T Kt_k V with Kt_k the
   node values of node k's degree-N_k polynomial (the nested tables of
   section 3.2.2 in the compressed basis); the work is that of rank R at
   every node.  In tai_assemble_B_batched each molecule with rank_tol > 0 is
   compressed on the device with no host wait: its operands keep the full
   length n with zero directions beyond its rank, which the FP64 and FP32
   kernels skip node by node (the split 16-bit kernels run the full
   length). */
typedef struct {
  double  omega;
  int32_t nq;
  int32_t n;
  double  L;
  int32_t nodes;
  int32_t prec;
  double  degree_tol;
  double  rank_tol;
} tai_params;

/* ---- context ------------------------------------------------------------ */

typedef struct tai_ctx tai_ctx;   /* opaque */

/* Create a context on HIP device `hip_device` (>= 0).  hip_device == -1
   makes a host-only context: every entry point validates its arguments and
   then returns TAI_ERR_NOT_READY instead of touching a device (used to check
   argument handling on machines without a GPU).  *ctx is set to NULL on
   error; TAI_ERR_HIP if the device does not exist. */
int tai_create(tai_ctx** ctx, int hip_device);

/* Free the context's workspace and caches.  NULL is accepted. */
int tai_destroy(tai_ctx* ctx);

/* Static description of a status code; never NULL. */
const char* tai_status_string(int status);

/* Message of the last failure on ctx (empty string if none); never NULL.
   The string stays valid until the next call on ctx. */
const char* tai_last_error(const tai_ctx* ctx);

/* Wait for `stream` and report any pending device error as TAI_ERR_HIP. */
int tai_sync(tai_ctx* ctx, void* stream);

/* ---- hot path ----------------------------------------------------------- */

/* Quadrature nodes and interpolation tables, computed on the device in FP64.
   t[k], w[k] (k < nq): Gauss-Legendre nodes/weights of int_0^omega (eq. TEI2,
   Prop. 2.4); xi[a] (a < n): Chebyshev nodes on [-L,L] (Def. 2.2);
   K[k][a][b] = exp(-t_k^2 (xi_a - xi_b)^2) (eq. chebcheb, node form), or
   with degree_tol > 0 the values at the grid of node k's polynomial cut to
   degree N_k (tai_degrees).
   All DEVICE double; any of the four pointers may be NULL to skip it. */
int tai_quadrature(tai_ctx* ctx, const tai_params* params,
                   double* t, double* w, double* xi, double* K, void* stream);

/* Per-node degrees (eq. chebcheb with N_k interpolation points for node k,
   and the nested coefficient moments of section 3.2).  For each node the
   Chebyshev coefficients C_k[i][j] of the n x n interpolant of
   exp(-t_k^2 (x-y)^2) in T_i(x/L) T_j(y/L) are computed in FP64; N_k is the
   smallest m >= 1 with sum_{max(i,j) >= m} |C_k[i][j]| <= degree_tol (n when
   degree_tol == 0), and entries with i or j >= N_k are set to zero.
   nk: DEVICE int32 [nq] or NULL; C: DEVICE double [nq][n][n] or NULL (not
   both NULL).  With degree_tol > 0, tai_quadrature's K holds the node values
   of the kept polynomials. */
int tai_degrees(tai_ctx* ctx, const tai_params* params, int32_t* nk, double* C, void* stream);

/* Low-rank compression of the moments (section 6.1, eqs. SVD and
   approxepsilon).  M: DEVICE double [3][n][npair] (tai_moments).  The
   singular values and left singular vectors of W = [M_1 | M_2 | M_3]
   (n x 3 npair) are computed in FP64 from the eigenpairs of W W^T (cyclic
   Jacobi): sigma (DEVICE double [n] or NULL) in decreasing order, V (DEVICE
   double [n][n] or NULL) with V[a][r] the r-th singular vector, and
   *rank (HOST) R = #{r : sigma_r > rank_tol * sigma_1}, at least 1 (the cut
   of section 6.1).  One basis serves the three directions and every
   quadrature node.  Forming W W^T resolves sigma_r to about
   1e-16 sigma_1^2 / sigma_r, so ranks cut at rank_tol >= 1e-7 rest on
   well-resolved values.  rank_tol must be > 0 (TAI_ERR_INVALID_ARG
   otherwise).  The call waits on the host for the rank.
   With U (DEVICE double, room for [3][n][npair]) and/or Kc (DEVICE double,
   room for [nq][n][n]) non-NULL the compressed operands are written too, at
   the padded inner length Rp = min(n, 8 ceil(R / 8)) that the contractions
   run at (their inner index goes in chunks of 8):
   U[d][r][q] = sum_a V[a][r] M[d][a][q] for r < R and 0 for R <= r < Rp,
   packed as [3][Rp][npair], and Kc[k] = V_R^T K_k V_R (eq. approxepsilon)
   bordered by zero rows and columns up to Rp, packed as [nq][Rp][Rp].  The
   zero padding adds nothing to any product: results are those of rank R.
   They serve tai_apply_J_compressed for as long as the moments do not
   change. */
int tai_compress(tai_ctx* ctx, const double* M, int32_t npair, const tai_params* params, int32_t* rank,
                 double* sigma, double* V, double* U, double* Kc, void* stream);

/* J from prepared compressed operands (tai_compress with U and Kc): the J of
   tai_apply_J (or tai_apply_J_pairs when pairs != NULL, npk pairs listed) on
   the grid of the compressed directions, with no basis computed and no host
   wait, so that one compression serves every J build while the moments stay
   fixed (a self-consistent-field loop changes D only).  R is the rank
   tai_compress returned (1 <= R <= params->n); U: DEVICE double
   [3][Rp][npk or npair] and Kc: DEVICE double [nq][Rp][Rp] as tai_compress
   wrote them, Rp = min(n, 8 ceil(R / 8)); params gives omega, nq, n, L, nodes
   (for the weights w_k) and prec (TAI_FP64, TAI_FP32, TAI_BF16X3 or TAI_BF16X6, as for tai_apply_J); rank_tol and
   degree_tol are not read.  The result equals that of tai_apply_J with the
   same rank_tol bit for bit. */
int tai_apply_J_compressed(tai_ctx* ctx, const double* U, int32_t nb, const int32_t* pairs, int32_t npk,
                           int32_t R, const double* Kc, const tai_params* params, const double* D, double* J,
                           void* stream);

/* 1D moments (eq. defV, Lagrange basis), FP64 on the device:
     M[d][a][p] = int_{-L}^{L} g_{mu,d}(x) g_{nu,d}(x) l_a(x) dx
   for d < 3, a < n, p < npair.  M is DEVICE double [3][n][npair].  With
   coef == NULL the unit-norm constants are applied per direction; with coef
   the factor c_mu c_nu goes into the d = 0 moments.  params->prec is ignored. */
int tai_moments(tai_ctx* ctx, const tai_basis* basis, const tai_params* params,
                double* M, void* stream);

/* The full pair matrix (Theorem 3.1, Algorithm 1 for all pairs):
     B[p*ldb + q] = (2/sqrt(pi)) sum_k w_k prod_d (M_d^T K_k M_d)(p,q)
   for p, q < npair, written for both triangles (B is symmetric; each tile
   p-block <= q-block is computed once and stored with its mirror).
   M: DEVICE double [3][n][npair] (as from tai_moments).  B: DEVICE, row-major
   npair x ldb (ldb >= npair), double if params->prec == TAI_FP64 else float.
   Columns npair..ldb-1 are not touched. */
int tai_assemble_B(tai_ctx* ctx, const double* M, int32_t npair, const tai_params* params,
                   void* B, int64_t ldb, void* stream);

/* One molecule of a batch: its own basis (HOST), parameters, moment buffer M
   (DEVICE double [3][n][npair], written by the call) and output B (DEVICE,
   as in tai_assemble_B).  All molecules of one batch must share nq, n, nodes
   and prec; omega and L may differ. */
typedef struct {
  tai_basis  basis;
  tai_params params;
  double*    M;
  void*      B;
  int64_t    ldb;
} tai_mol;

/* Moments and B for every molecule of a batch (1 <= nmol <= 65535; the
   molecules share nq, n, nodes and prec, each has its own omega, L, basis,
   M and B): one launch per preparation stage (nodes, moments, operand
   packing, projection) covering all molecules, then ONE persistent assembly
   launch whose work groups drain a queue of (molecule, tile) items.  With a non-NULL stream the
   kernel sequence is recorded once into a HIP graph and replayed while the
   batch description (sizes, parameters, M/B pointers) is unchanged; the
   bases themselves are uploaded on every call.  Setting the environment
   variable TAI_NO_GRAPH launches the kernels directly.  Results equal those
   of tai_moments + tai_assemble_B per molecule (bit for bit in FP64 and
   FP32, also for compressed molecules; the split 16-bit forms of a
   compressed molecule run at inner length n instead of the padded rank and
   agree to their tolerance).  Molecules with rank_tol > 0 are compressed
   inside the launch sequence (section 6.1) without a host wait, so the
   graph holds the compression too. */
int tai_assemble_B_batched(tai_ctx* ctx, int32_t nmol, const tai_mol* mols, void* stream);

/* Coulomb matrix through the grid tensor, B never formed (eq. coulapprox with
   the mode products of eq. ig1):
     Dt_q   = D(k,l) (2 - delta_kl),  q = (k,l), k <= l
     rho(a) = sum_q Dt_q prod_d m_{q,d}(a_d)                 (a in [n]^3)
     Phi    = (2/sqrt(pi)) sum_k w_k rho x_1 K_k x_2 K_k x_3 K_k
     J(mu,nu) = J(nu,mu) = sum_a prod_d m_{p,d}(a_d) Phi(a),  p = (mu,nu)
   which equals sum over all ordered (k,l) of B(mu nu, k l) D(k,l) for a
   symmetric D.  M: DEVICE double [3][n][npair]; D: DEVICE double [nb][nb],
   only its upper triangle is read; J: DEVICE double [nb][nb], fully written.
   params->prec selects the arithmetic of the two pair contractions (rho and
   the projection onto the pairs), both on the matrix cores:
     TAI_FP64   FP64 throughout;
     TAI_FP32   FP32 operands and products, summed in FP32 within a batch of
                64 pairs (rho) or one 16-row block (projection) and in FP64
                beyond; the mode products and the contraction with m_{p,0},
                m_{p,1} stay FP64.
     TAI_BF16X6 the projection onto the pairs in split BF16: Phi and the
                FP32 moments cut into 3 bfloat16 slices, 6 slice products
                per term (bf16 MFMA, FP32 accumulation, FP64 across a1);
                rho as for TAI_FP32 (in split BF16 the matrix cores'
                accumulation of the heavily cancelling pair sums costs
                several times the FP32 accuracy).
     TAI_BF16X3 both contractions in split BF16 with 2 slices and 3
                products (16 significant bits: a few 1e-6 relative): rho's
                operand Dt_q m_{q,0}(a0) m_{q,1}(a1) formed in FP32 and
                split, summed in FP32 within a batch of 64 pairs and in FP64
                beyond.
   TAI_F16X3 returns TAI_ERR_UNSUPPORTED (its range scaling does not carry
   across the sum over pairs). */
int tai_apply_J(tai_ctx* ctx, const double* M, int32_t nb, const tai_params* params,
                const double* D, double* J, void* stream);

/* tai_apply_J for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same J, bit for bit, with every intermediate (node tables, pair
   density, partial and final grid tensors, mode products, J on the pairs)
   carved from a static device array of 256 MiB that the library holds on
   each device it runs on until the process ends, looked up once per device
   when a context is created.  The call makes no hipMalloc, hipFree or other
   allocating call and does no host synchronisation; the caller passes M, D
   and J as for tai_apply_J.
   Limits: prec TAI_FP64 or TAI_FP32; rank_tol must be 0 (the compression
   needs its own workspace: TAI_ERR_UNSUPPORTED); the call's scratch need,
   the node tables plus 16 npair + 8 n^3 (nchunk + 2 + 2 nq) + 8 nq bytes (+ 12 n
   npair for TAI_FP32), with nchunk = 512 / g for the g groups of the rho
   contraction (g = ceil(n / 16) in FP64 up to n = 48, else ceil(n / 8)) and
   at most ceil(npair / 256), must fit in 256 MiB, else TAI_ERR_INVALID_ARG
   with the size in tai_last_error (Nb = 1000, n = 48, nq = 32 in FP64 needs
   207 MiB).  Every call on a
   device shares that device's array, which keeps the last call's contents;
   nothing in it needs to start at zero (every intermediate is written
   before it is read).  Calls that overlap in time on one device, from any
   context or stream, race on the array: order them on one stream or
   synchronise between them. */
int tai_apply_J_noalloc(tai_ctx* ctx, const double* M, int32_t nb, const tai_params* params,
                        const double* D, double* J, void* stream);

/* Coulomb matrix in the molecular-orbital basis (section 5, eq. Coul):
     Jmo[i][j] = sum over all ordered (mu,nu), (kappa,lambda) of
                 q_i(mu) q_i(nu) B(mu nu, kappa lambda) q_j(kappa) q_j(lambda)
   = < q_i q_i^T, B (q_j q_j^T) > for the orbitals q_i = Q[i][0 .. nb).
   Through the grid, with neither B nor any AO Coulomb matrix formed: for each
   orbital the pair density of q_i q_i^T gives rho_i and Phi_i as in
   tai_apply_J, and Jmo[i][j] = sum_a rho_i(a) Phi_j(a) over the n^3 grid.
   M: DEVICE double [3][n][npair], or [3][n][npk] for the DEVICE pair list
   pairs [npk] of tai_moments_pairs (pairs NULL: all pairs, npk ignored).
   Q: DEVICE double [norb][nb], 1 <= norb <= 1024.  Jmo: DEVICE double
   [norb][norb].  params->prec TAI_FP64 or TAI_FP32 as for tai_apply_J (the
   rho contraction); the grid sums are FP64.  Workspace 2 * norb * n^3 doubles. */
int tai_coulomb_mo(tai_ctx* ctx, const double* M, int32_t nb, const int32_t* pairs, int32_t npk,
                   const tai_params* params, const double* Q, int32_t norb, double* Jmo, void* stream);

/* Long-range exchange matrix (appendix B, eq. exchange):
   Kx(mu, nu) = 2 sum_j sum_{lambda, kappa} q_j(lambda) q_j(kappa) B(mu lambda, kappa nu)
   over ordered index pairs, for the orbitals Q (DEVICE double [norb][nb],
   1 <= norb <= 1024), by the paper's factorized form: for each orbital j and
   function mu the n^3 grid tensor X_{j mu} = sum_lambda q_j(lambda) m_(mu lambda)
   (a rho over the pairs that hold mu) and its Phi_{j nu} as in tai_apply_J,
   then Kx(mu, nu) = 2 sum_j <X_{j mu}, Phi_{j nu}>.  M: DEVICE double
   [3][n][npair] (or [3][n][npk] with a pair list, as tai_apply_J_pairs);
   Kx: DEVICE double [nb][nb], written in full.  The context keeps
   2 norb nb n^3 doubles of grid tensors (at most 64 GiB, else
   TAI_ERR_INVALID_ARG).  prec TAI_FP64 or TAI_FP32 (the rho contractions);
   rank_tol > 0 runs it on the compressed grid.  Each (j, mu) costs a
   contraction over the Nb pairs that hold mu (2 n^3 Nb flops) and the mode
   products of one grid tensor (6 nq n^4); the grid tensors of all (j, mu)
   run through the mode products in chunks of at most 4 GiB. */
int tai_exchange(tai_ctx* ctx, const double* M, int32_t nb, const int32_t* pairs, int32_t npk,
                 const tai_params* params, const double* Q, int32_t norb, double* Kx, void* stream);

/* ---- contracted basis functions (eq. basis, I_mu > 1 primitives) ---------- */

/* A contracted basis is passed as its primitives: a tai_basis of nbp
   primitive functions listed function by function, whose coef holds each
   primitive's contraction coefficient (times any normalisation wanted), and
   fmap [nbp] (HOST int32), the contracted function of each primitive:
   fmap[0] = 0 and each step adds 0 or 1, so nb = fmap[nbp-1] + 1.  Moments
   and B are formed over the primitive pairs (tai_moments, tai_assemble_B with
   the primitive basis); the contracted results are segment sums of them. */

/* B over contracted pairs from B over primitive pairs:
     B[P*ldb + Q] = sum_{p -> P} sum_{q -> Q} w_p w_q Bp[p*ldbp + q],
   where primitive pair p = (i, j), i <= j, belongs to P = (fmap[i], fmap[j])
   and w_p = 2 when i != j are primitives of one function (the product
   g_mu g_mu holds both orders), else 1.  Bp: DEVICE, npair(nbp) rows, ldbp
   >= npair(nbp); B: DEVICE, npair(nb) x ldb, ldb >= npair(nb); both double
   if prec == TAI_FP64, else float (sums in FP64).  Writes every entry of B. */
int tai_contract_pairs(tai_ctx* ctx, const void* Bp, int64_t ldbp, int32_t nbp, const int32_t* fmap, int32_t prec,
                       void* B, int64_t ldb, void* stream);

/* tai_apply_J for a contracted basis: M is DEVICE double [3][n][npair(nbp)],
   the moments of the primitive basis; D and J are DEVICE double [nb][nb]
   over contracted functions.  The density is expanded to the primitives,
   D_prim(i,j) = D(fmap[i], fmap[j]), J_prim is formed as in tai_apply_J, and
   J(mu,nu) = sum over primitives i of mu and j of nu of J_prim(i,j).
   Workspace 2 * nbp^2 doubles. */
int tai_apply_J_contracted(tai_ctx* ctx, const double* M, int32_t nbp, const int32_t* fmap,
                           const tai_params* params, const double* D, double* J, void* stream);

/* ---- screening (section 6.3, compression by screening) --------------------- */

/* Pairs that survive screening: pair p(mu,nu), mu <= nu, is dropped when its
   Gaussian product prefactor exp(-a_mu a_nu/(a_mu + a_nu) |A_mu - A_nu|^2)
   is at most tau (every pair is kept when tau <= 0; 0 < tau < 1 keeps at
   least the diagonal pairs).  pairs: DEVICE int32 with room for npair
   entries; the kept pair indices are written in ascending order.  nkept:
   HOST, set to their count.  The call waits for `stream` to read the count.
   tau must be finite and < 1. */
int tai_screen_pairs(tai_ctx* ctx, const tai_basis* basis, double tau, int32_t* pairs, int32_t* nkept,
                     void* stream);

/* tai_moments for a list of pairs: M[d][a][i] is the moment of pair pairs[i]
   (an index into the full pair list, e.g. from tai_screen_pairs), i < npk.
   pairs: DEVICE int32 [npk], 1 <= npk <= npair; entries outside the full
   list give zero moments.  M: DEVICE double [3][n][npk].  tai_assemble_B with
   npair = npk then returns B restricted to the listed pairs, in list order. */
int tai_moments_pairs(tai_ctx* ctx, const tai_basis* basis, const tai_params* params, const int32_t* pairs,
                      int32_t npk, double* M, void* stream);

/* tai_apply_J with the pair sums restricted to a list of pairs (screening):
   M is DEVICE double [3][n][npk] from tai_moments_pairs for the same DEVICE
   list pairs [npk]; rho sums over the listed pairs only, J is computed for
   them and its entries of the other pairs are written as zero.  Otherwise as
   tai_apply_J. */
int tai_apply_J_pairs(tai_ctx* ctx, const double* M, int32_t nb, const int32_t* pairs, int32_t npk,
                      const tai_params* params, const double* D, double* J, void* stream);

/* ---- adaptive integration boxes (section 6.2) ----------------------------- */

/* Clusters the pairs into nparts boxes.  The numerical support of pair p
   (mu <= nu) is the centred box [-b_p, b_p]^3 outside which its Gaussian
   factor exp(-p (x_d - P_d)^2) (Gaussian product rule, eq. gauss_prod) is
   below tau in every direction: b_p = max_d |P_d| + sqrt(ln(1/tau) / p),
   p = a_mu + a_nu, P = (a_mu A_mu + a_nu A_nu) / p.  The supports are cut
   into equal-count quantiles (the paper leaves the clustering open): box s
   (s = 0 .. nparts-1) is [-v_s, v_s] with v_s the ceil((s+1) npair / nparts)-th
   smallest support, and pair p goes to the first box that holds its
   support (v_{s-1} < b_p <= v_s), so equal supports share a partition and a
   partition can be empty.  0 < tau < 1; 1 <= nparts <= 16.
   pairs: DEVICE int32 [npair], written with the pair indices of partition 0,
   then 1, ..., each partition's in ascending order; counts: HOST int32
   [nparts], pairs per partition; boxes: HOST double [nparts], v_s
   (ascending).  The call waits for `stream` to return counts and boxes. */
int tai_partition_pairs(tai_ctx* ctx, const tai_basis* basis, double tau, int32_t nparts, int32_t* pairs,
                        int32_t* counts, double* boxes, void* stream);

/* The moments of every partition's pairs on its own box (section 6.2: each
   pair's interpolant on the grid of its partition's box), in one launch:
   block s of M, [3][n][counts[s]] at M + 3 n (counts[0] + ... +
   counts[s-1]), holds what tai_moments_pairs writes for the pairs of
   partition s with params->L = boxes[s], bit for bit.  pairs: DEVICE int32,
   the partitions' lists one after another; counts: HOST int32 [nparts]
   (>= 0, adding up to a number in [1, npair(nb)]); boxes: HOST double
   [nparts] (finite, > 0); 1 <= nparts <= 16 (TAI_ERR_INVALID_ARG
   otherwise).  params->L is not read; M: DEVICE double, written. */
int tai_moments_partitioned(tai_ctx* ctx, const tai_basis* basis, const tai_params* params, const int32_t* pairs,
                            const int32_t* counts, const double* boxes, int32_t nparts, double* M, void* stream);

/* J with adaptive boxes (eq. coulapprox with the boxes of section 6.2,
   tai_partition_pairs): every pair of partition s carries its moments on
   the Chebyshev grid of box s, and two partitions s, s' interact through the
   interpolant of exp(-t_k^2 (x - y)^2) on [-v_s, v_s] x [-v_s', v_s'], with
   node values K_k^(s,s')(a, b) = exp(-t_k^2 (xi^s_a - xi^s'_b)^2):
     rho_s  = sum_{q in s} Dt_q (x)_d m_{q,d}                 (grid of box s)
     Phi_s  = (2/sqrt(pi)) sum_k w_k sum_s' rho_s' x_1 K_k^(s,s') x_2 K_k^(s,s') x_3 K_k^(s,s')
     J_p    = < (x)_d m_{p,d}, Phi_s >,  p in s,
   i.e. sum over all pairs q of B(p, q) Dt_q with B(p, q) from Theorem 3.1 on
   the two pairs' boxes.  M: DEVICE double, the partitions' moment blocks one
   after another, block s = [3][n][counts[s]] as tai_moments_pairs writes it
   for the pairs of partition s with params->L = boxes[s]; pairs, counts,
   boxes as from tai_partition_pairs (counts adding up to npair(nb), boxes
   > 0); D, J as for tai_apply_J.  params gives omega, nq, n, nodes and prec
   (TAI_FP64, TAI_FP32, TAI_BF16X3, TAI_BF16X6; the mode products stay FP64);
   params->L is not read; rank_tol and degree_tol must be 0
   (TAI_ERR_UNSUPPORTED). */
int tai_apply_J_partitioned(tai_ctx* ctx, const double* M, int32_t nb, const int32_t* pairs, const int32_t* counts,
                            const double* boxes, int32_t nparts, const tai_params* params, const double* D, double* J,
                            void* stream);

/* B over adaptive boxes (section 6.2 with Theorem 3.1): B(p, q) =
   (2/sqrt(pi)) sum_k w_k prod_d m_{p,d}^T K_k^(s,s') m_{q,d}, p in partition s
   (moments on box s), q in s' (moments on box s'), K^(s,s') the interpolant
   of exp(-t_k^2 (x - y)^2) on the two boxes' grids, the matrix whose products
   with the pair densities tai_apply_J_partitioned applies.  Rows and columns
   follow the concatenated partition lists (the order of the pairs of
   tai_partition_pairs).  M: DEVICE double, the moment blocks of
   tai_moments_partitioned; counts: HOST int32 [nparts] (>= 0, adding up to a
   total of at least 1); boxes: HOST double [nparts] (finite, > 0);
   1 <= nparts <= 16.  B: DEVICE, row-major total x ldb (ldb >= total),
   double for TAI_FP64 else float, written in full (both triangles).  params
   gives omega, nq, n, nodes and prec; params->L is not read; rank_tol and
   degree_tol must be 0.  Runs on the persistent assembly kernels: TAI_FP64
   and TAI_FP32 (n up to their inner length) and the split 16-bit forms with
   a compiled shape for nq; otherwise TAI_ERR_UNSUPPORTED.  The library keeps
   the cross tables and, per partition pair s <= s', the column operand
   (about nparts (nparts + 1) / 2 times the single-box projection). */
int tai_assemble_B_partitioned(tai_ctx* ctx, const double* M, const int32_t* counts, const double* boxes,
                               int32_t nparts, const tai_params* params, void* B, int64_t ldb, void* stream);

/* ---- tuning ------------------------------------------------------------- */

/* Shape autotuner of the split 16-bit assembly (TAI_BF16X3, TAI_BF16X6,
   TAI_F16X3).  Its persistent kernel has several compiled shapes per inner
   length (waves per work group, row and column blocks per wave, LDS ring
   depth).  With mode 1 (the default) the first tai_assemble_B or
   tai_assemble_B_batched call of a signature -- arithmetic, n, nq and a size
   class (npair rounded up to a power of two; for a batch, its list of basis
   sizes) -- runs every candidate twice on the call's stream, times the second
   run with HIP events and keeps the fastest for later calls of the
   signature (the table default stays unless another candidate is more than
   2% faster).  That first call therefore takes about twice the number of
   candidates times longer and synchronizes the stream.  Candidates compute
   every entry with the same arithmetic in the same order: results do not
   depend on the choice.  mode 0 uses the table default shape without
   timing; mode 2 forgets the choices made so far (the mode is unchanged).
   The environment variable TAI_ASM16_SHAPE=<k> forces candidate k.
   TAI_ERR_INVALID_ARG for another mode. */
int tai_tune(tai_ctx* ctx, int mode);

/* ---- timing ------------------------------------------------------------- */

/* Per-stage device timing.  While enabled, every call brackets each stage it
   enqueues with HIP events recorded on the call's stream (outside graph
   capture).  Stages: "nodes", "moments", "pack", "project", "assemble",
   "apply_J", "batched" (a whole tai_assemble_B_batched launch or graph
   replay), "compress" (basis and compressed operands of rank_tol > 0).  tai_profile_enable clears the totals (enable = 0 turns timing
   off); tai_profile_read waits for the recorded events and returns the total
   milliseconds and the number of timed launches of one stage. */
int tai_profile_enable(tai_ctx* ctx, int enable);
int tai_profile_read(tai_ctx* ctx, const char* stage, double* total_ms, int64_t* count);

/* What this device sustains, for reporting measured kernels against the
   device's own ceiling beside the published one: what 0 = dense FP16 matrix
   throughput (back-to-back independent v_mfma_f32_16x16x32_f16 on every
   SIMD), 1 = FP64 matrix throughput (v_mfma_f64_16x16x4_f64), both in
   TFLOP/s; 2 = HBM streaming copy, bytes read plus written, in GB/s.  The
   best of three timed launches after one warm-up, on `stream`.  The call
   allocates its own buffers (2 GiB for what 2), synchronizes the stream and
   takes a few milliseconds.  TAI_ERR_INVALID_ARG for another `what` or a NULL
   `value`, TAI_ERR_NOMEM if the buffers cannot be allocated. */
int tai_peak_probe(tai_ctx* ctx, int what, double* value, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TAI_H */
