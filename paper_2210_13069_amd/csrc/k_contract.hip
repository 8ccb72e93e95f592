// Contracted basis functions (eq. basis with I_mu > 1 primitives each).
// A contracted function is the sum of its primitives (their contraction
// coefficients go into the primitive basis' coef), so the pair product of
// two contracted functions is the sum over ordered primitive pairs:
//
//   B_c(P, Q) = sum_{p -> P} sum_{q -> Q} w_p w_q B(p, q),
//
// with w_p = 2 for the pair (i, j), i != j, of two primitives of one function
// (both orders) and 1 otherwise; likewise J over contracted functions is the
// sum of the primitive-basis J over the members of each function, for the
// density expanded to the primitives, D_prim(i, j) = D(f(i), f(j)).
#include "tai_internal.h"

namespace tai {
namespace {

constexpr int kTile = 16;

// One thread per contracted entry (P, Q); the member lists of contracted
// pairs are CSR: primitive pairs idx[off[P] .. off[P+1]) with weights wt.
template <typename T>
__global__ void __launch_bounds__(kTile* kTile)
contract_pairs_kernel(const T* __restrict__ Bp, int64_t ldbp, const int32_t* __restrict__ off,
                      const int32_t* __restrict__ idx, const double* __restrict__ wt, int64_t npc, T* __restrict__ B,
                      int64_t ldb) {
  const int64_t P = (int64_t)blockIdx.y * kTile + threadIdx.y;
  const int64_t Q = (int64_t)blockIdx.x * kTile + threadIdx.x;
  if (P >= npc || Q >= npc) return;
  double s = 0.0;
  for (int a = off[P]; a < off[P + 1]; ++a) {
    const T* row = Bp + (int64_t)idx[a] * ldbp;
    double r = 0.0;
    for (int b = off[Q]; b < off[Q + 1]; ++b) r += wt[b] * (double)row[idx[b]];
    s += wt[a] * r;
  }
  B[P * ldb + Q] = (T)s;
}

__global__ void __launch_bounds__(256)
expand_density_kernel(const double* __restrict__ D, int nb, const int32_t* __restrict__ fmap, int nbp,
                      double* __restrict__ Dp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nbp * nbp) return;
  const int i = (int)(e / nbp), j = (int)(e % nbp);
  Dp[e] = D[(int64_t)fmap[i] * nb + fmap[j]];
}

// J(mu, nu) = sum of Jp over the primitives first[mu] .. first[mu+1] and
// first[nu] .. first[nu+1]
__global__ void __launch_bounds__(256)
contract_functions_kernel(const double* __restrict__ Jp, int nbp, const int32_t* __restrict__ first, int nb,
                          double* __restrict__ J) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * nb) return;
  const int mu = (int)(e / nb), nu = (int)(e % nb);
  double s = 0.0;
  for (int i = first[mu]; i < first[mu + 1]; ++i)
    for (int j = first[nu]; j < first[nu + 1]; ++j) s += Jp[(int64_t)i * nbp + j];
  J[e] = s;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_contract_pairs(bool fp64, const void* Bp, int64_t ldbp, const int32_t* off, const int32_t* idx,
                                 const double* wt, int64_t npc, void* B, int64_t ldb, hipStream_t s) {
  const dim3 grid(nblk(npc, kTile), nblk(npc, kTile)), block(kTile, kTile);
  if (fp64)
    hipLaunchKernelGGL(contract_pairs_kernel<double>, grid, block, 0, s, static_cast<const double*>(Bp), ldbp, off,
                       idx, wt, npc, static_cast<double*>(B), ldb);
  else
    hipLaunchKernelGGL(contract_pairs_kernel<float>, grid, block, 0, s, static_cast<const float*>(Bp), ldbp, off, idx,
                       wt, npc, static_cast<float*>(B), ldb);
  return hipGetLastError();
}

hipError_t launch_expand_density(const double* D, int nb, const int32_t* fmap, int nbp, double* Dp, hipStream_t s) {
  hipLaunchKernelGGL(expand_density_kernel, dim3(nblk((int64_t)nbp * nbp, 256)), dim3(256), 0, s, D, nb, fmap, nbp,
                     Dp);
  return hipGetLastError();
}

hipError_t launch_contract_functions(const double* Jp, int nbp, const int32_t* first, int nb, double* J,
                                     hipStream_t s) {
  hipLaunchKernelGGL(contract_functions_kernel, dim3(nblk((int64_t)nb * nb, 256)), dim3(256), 0, s, Jp, nbp, first,
                     nb, J);
  return hipGetLastError();
}

}  // namespace tai
