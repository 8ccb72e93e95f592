// Coulomb matrix through the n^3 Chebyshev grid tensor, B never formed
// (eq. coulapprox with the mode products of eq. ig1), FP64:
//
//   Dt_q       = D(k,l) (2 - delta_kl)                     q = (k,l), k <= l
//   rho(a)     = sum_q Dt_q m_{q,0}(a0) m_{q,1}(a1) m_{q,2}(a2)
//   Phi        = (2/sqrt(pi)) sum_k w_k  rho x_0 K_k x_1 K_k x_2 K_k
//   J_p        = sum_a m_{p,0}(a0) m_{p,1}(a1) m_{p,2}(a2) Phi(a)
//   J(mu,nu)   = J(nu,mu) = J_p,                           p = (mu,nu)
//
// rho is a split-K contraction over pairs: each work group owns one a0 and
// one chunk of pairs and writes an n x n partial; the partials are summed in
// a fixed order, so the result does not depend on scheduling.
#include "tai_internal.h"
#include "tai_device.h"

namespace tai {
namespace {

constexpr double kTwoOverSqrtPi = 1.1283791670955126;
constexpr int kQB = 32;          // pairs staged per LDS batch in the rho kernel
constexpr int kRhoBlocks = 2048; // target work groups of the rho kernel

__global__ void __launch_bounds__(256)
density_pairs_kernel(const double* __restrict__ D, int nb, int64_t npair, double* __restrict__ Dt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int mu, nu;
  decode_pair(nb, p, mu, nu);
  Dt[p] = D[(int64_t)mu * nb + nu] * (mu == nu ? 1.0 : 2.0);
}

// grid (n, nchunk); 256 threads as 16 x 16, each an MT x MT micro-tile of
// (a1, a2) = (ty + 16 i, tx + 16 j).
template <int MT>
__global__ void __launch_bounds__(256)
rho_kernel(const double* __restrict__ M, const double* __restrict__ Dt, int n, int64_t npair,
           int64_t chunk, double* __restrict__ part) {
  constexpr int NM = 16 * MT;
  __shared__ double c_s[kQB];
  __shared__ double m1_s[kQB][NM];
  __shared__ double m2_s[kQB][NM];
  const int a0 = blockIdx.x;
  const int64_t q0 = (int64_t)blockIdx.y * chunk;
  const int64_t q1 = (q0 + chunk < npair) ? q0 + chunk : npair;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const double* M0 = M;
  const double* M1 = M + (int64_t)n * npair;
  const double* M2 = M + 2 * (int64_t)n * npair;
  double acc[MT][MT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < MT; ++j) acc[i][j] = 0.0;

  for (int64_t qb = q0; qb < q1; qb += kQB) {
    __syncthreads();
    // stage: thread t loads column (t % kQB) for rows a = t / kQB + 8 r
    {
      const int qq = threadIdx.x % kQB;
      const int64_t q = qb + qq;
      const bool ok = q < q1;
      if (threadIdx.x < kQB) c_s[qq] = ok ? Dt[q] * M0[(int64_t)a0 * npair + q] : 0.0;
      for (int a = threadIdx.x / kQB; a < NM; a += 256 / kQB) {
        const bool in = ok && a < n;
        m1_s[qq][a] = in ? M1[(int64_t)a * npair + q] : 0.0;
        m2_s[qq][a] = in ? M2[(int64_t)a * npair + q] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int qq = 0; qq < kQB; ++qq) {
      const double cq = c_s[qq];
      double x[MT], y[MT];
#pragma unroll
      for (int i = 0; i < MT; ++i) x[i] = cq * m1_s[qq][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < MT; ++j) y[j] = m2_s[qq][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < MT; ++j) acc[i][j] += x[i] * y[j];
    }
  }
  double* out = part + ((int64_t)blockIdx.y * n + a0) * n * n;
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < MT; ++j) {
      const int a1 = ty + 16 * i, a2 = tx + 16 * j;
      if (a1 < n && a2 < n) out[a1 * n + a2] = acc[i][j];
    }
}

__global__ void __launch_bounds__(256)
sum_parts_kernel(const double* __restrict__ part, int nchunk, int64_t len, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * len + i];
  out[i] = s;
}

// out[k][...] = mode-`mode` product of K_k with in (in shared by all k when
// in_stride == 0).  Index (i0, i1, i2) of an n^3 tensor, i0 slowest.
__global__ void __launch_bounds__(256)
mode_product_kernel(const double* __restrict__ K, const double* __restrict__ in, int64_t in_stride,
                    double* __restrict__ out, int n, int nq, int mode) {
  const int64_t n3 = (int64_t)n * n * n;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n3 * nq) return;
  const int k = (int)(g / n3);
  const int64_t e = g - k * n3;
  const int i0 = (int)(e / (n * n)), i1 = (int)((e / n) % n), i2 = (int)(e % n);
  const double* Kk = K + (int64_t)k * n * n;
  const double* src = in + k * in_stride;
  double s = 0.0;
  if (mode == 0) {
    for (int a = 0; a < n; ++a) s += Kk[i0 * n + a] * src[((int64_t)a * n + i1) * n + i2];
  } else if (mode == 1) {
    for (int a = 0; a < n; ++a) s += Kk[i1 * n + a] * src[((int64_t)i0 * n + a) * n + i2];
  } else {
    for (int a = 0; a < n; ++a) s += Kk[i2 * n + a] * src[((int64_t)i0 * n + i1) * n + a];
  }
  out[g] = s;
}

__global__ void __launch_bounds__(256)
phi_kernel(const double* __restrict__ T3, const double* __restrict__ w, int nq, int64_t n3,
           double* __restrict__ Phi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double s = 0.0;
  for (int k = 0; k < nq; ++k) s += w[k] * T3[(int64_t)k * n3 + i];
  Phi[i] = kTwoOverSqrtPi * s;
}

// One thread per pair: J_p = sum_a0 m0(a0) sum_a1 m1(a1) sum_a2 m2(a2) Phi,
// with the pair's m2 column in registers; Phi rows are read at wave-uniform
// addresses.
template <int NMAX>
__global__ void __launch_bounds__(128)
jp_kernel(const double* __restrict__ M, const double* __restrict__ Phi, int n, int64_t npair,
          double* __restrict__ Jp) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = p < npair;
  const int64_t pc = ok ? p : 0;
  const double* M0 = M;
  const double* M1 = M + (int64_t)n * npair;
  const double* M2 = M + 2 * (int64_t)n * npair;
  double m2[NMAX];
#pragma unroll
  for (int a = 0; a < NMAX; ++a) m2[a] = (a < n) ? M2[(int64_t)a * npair + pc] : 0.0;
  double jp = 0.0;
  for (int a0 = 0; a0 < n; ++a0) {
    double y = 0.0;
    for (int a1 = 0; a1 < n; ++a1) {
      const double* row = Phi + ((int64_t)a0 * n + a1) * n;
      double z = 0.0;
#pragma unroll
      for (int a2 = 0; a2 < NMAX; ++a2)
        if (a2 < n) z += m2[a2] * row[a2];
      y += M1[(int64_t)a1 * npair + pc] * z;
    }
    jp += M0[(int64_t)a0 * npair + pc] * y;
  }
  if (ok) Jp[p] = jp;
}

__global__ void __launch_bounds__(256)
unpack_kernel(const double* __restrict__ Jp, int nb, int64_t npair, double* __restrict__ J) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int mu, nu;
  decode_pair(nb, p, mu, nu);
  J[(int64_t)mu * nb + nu] = Jp[p];
  J[(int64_t)nu * nb + mu] = Jp[p];
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int j_nchunk(int n, int npair) {
  int c = kRhoBlocks / (n > 0 ? n : 1);
  if (c < 1) c = 1;
  const int maxc = (npair + 255) / 256;  // at least 256 pairs per chunk
  if (c > maxc) c = maxc;
  return c < 1 ? 1 : c;
}

size_t j_work_bytes(int nq, int n, int npair) {
  const size_t n3 = (size_t)n * n * n;
  const int nc = j_nchunk(n, npair);
  return align256(8 * (size_t)npair) * 2 + align256(8 * n3 * nc) + align256(8 * n3) * 2 +
         align256(8 * n3 * nq) * 3;
}

JWork carve_j_work(void* base, int nq, int n, int npair) {
  const size_t n3 = (size_t)n * n * n;
  JWork w;
  w.nchunk = j_nchunk(n, npair);
  char* p = static_cast<char*>(base);
  w.Dt = reinterpret_cast<double*>(p); p += align256(8 * (size_t)npair);
  w.Jp = reinterpret_cast<double*>(p); p += align256(8 * (size_t)npair);
  w.rho_part = reinterpret_cast<double*>(p); p += align256(8 * n3 * w.nchunk);
  w.rho = reinterpret_cast<double*>(p); p += align256(8 * n3);
  w.Phi = reinterpret_cast<double*>(p); p += align256(8 * n3);
  w.T1 = reinterpret_cast<double*>(p); p += align256(8 * n3 * nq);
  w.T2 = reinterpret_cast<double*>(p); p += align256(8 * n3 * nq);
  w.T3 = reinterpret_cast<double*>(p);
  return w;
}

hipError_t launch_apply_j(const double* M, int nb, int npair, int n, int nq, const NodeTables& tb,
                          const double* D, double* J, const JWork& w, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  hipLaunchKernelGGL(density_pairs_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, D, nb, (int64_t)npair, w.Dt);
  const int64_t chunk = ((int64_t)npair + w.nchunk - 1) / w.nchunk;
  const dim3 rg(n, w.nchunk);
  if (n <= 16) hipLaunchKernelGGL(rho_kernel<1>, rg, dim3(256), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  else if (n <= 32) hipLaunchKernelGGL(rho_kernel<2>, rg, dim3(256), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  else if (n <= 48) hipLaunchKernelGGL(rho_kernel<3>, rg, dim3(256), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  else hipLaunchKernelGGL(rho_kernel<4>, rg, dim3(256), 0, s, M, w.Dt, n, (int64_t)npair, chunk, w.rho_part);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, w.rho_part, w.nchunk, n3, w.rho);
  const unsigned mb = nblk(n3 * nq, 256);
  hipLaunchKernelGGL(mode_product_kernel, dim3(mb), dim3(256), 0, s, tb.K, w.rho, (int64_t)0, w.T1, n, nq, 0);
  hipLaunchKernelGGL(mode_product_kernel, dim3(mb), dim3(256), 0, s, tb.K, w.T1, n3, w.T2, n, nq, 1);
  hipLaunchKernelGGL(mode_product_kernel, dim3(mb), dim3(256), 0, s, tb.K, w.T2, n3, w.T3, n, nq, 2);
  hipLaunchKernelGGL(phi_kernel, dim3(nblk(n3, 256)), dim3(256), 0, s, w.T3, tb.w, nq, n3, w.Phi);
  const unsigned jb = nblk(npair, 128);
  if (n <= 16) hipLaunchKernelGGL(jp_kernel<16>, dim3(jb), dim3(128), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  else if (n <= 32) hipLaunchKernelGGL(jp_kernel<32>, dim3(jb), dim3(128), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  else if (n <= 48) hipLaunchKernelGGL(jp_kernel<48>, dim3(jb), dim3(128), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  else hipLaunchKernelGGL(jp_kernel<64>, dim3(jb), dim3(128), 0, s, M, w.Phi, n, (int64_t)npair, w.Jp);
  hipLaunchKernelGGL(unpack_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, w.Jp, nb, (int64_t)npair, J);
  return hipGetLastError();
}

}  // namespace tai
