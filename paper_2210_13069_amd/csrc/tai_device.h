// Device helpers shared by the kernel files of libtai.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tai {

// First pair index of row mu in the row-major upper triangle of an
// nb x nb pair list: p(mu, nu) = mu*nb - mu(mu-1)/2 + (nu - mu).
__device__ inline int64_t pair_row_start(int64_t nb, int64_t mu) { return mu * nb - (mu * (mu - 1)) / 2; }

// Inverse of the pair index.
__device__ inline void decode_pair(int64_t nb, int64_t p, int& mu, int& nu) {
  const double b2 = 2.0 * nb + 1.0;
  int64_t m = (int64_t)floor(0.5 * (b2 - sqrt(b2 * b2 - 8.0 * (double)p)));
  if (m < 0) m = 0;
  if (m > nb - 1) m = nb - 1;
  while (m > 0 && pair_row_start(nb, m) > p) --m;
  while (m + 1 < nb && pair_row_start(nb, m + 1) <= p) ++m;
  mu = (int)m;
  nu = (int)(m + (p - pair_row_start(nb, m)));
}

// T_j(xi_a / L) on the Chebyshev grid, the angle reduced exactly in
// integers: Lobatto (kind 0) xi_a = L cos(pi a / (n-1)), first kind
// xi_a = L cos((2a+1) pi / (2n)).
__device__ inline double cheb_at_node(int kind, int n, int a, int j) {
  if (kind == 0) {
    const int N = n - 1;
    return cos(M_PI * (double)((int64_t)a * j % (2 * N)) / N);
  }
  return cos(M_PI * (double)((int64_t)j * (2 * a + 1) % (4 * n)) / (2.0 * n));
}

}  // namespace tai
