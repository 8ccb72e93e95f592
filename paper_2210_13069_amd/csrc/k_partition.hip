// Adaptive integration boxes (section 6.2).
//
//  * support_kernel: per pair p = (mu, nu) the half-width
//        b_p = max_d |P_d| + sqrt(c / p),  p = a + b,  P = (a A + b B) / p,
//    c = ln(1/tau) (from the host), outside which the pair's exponential
//    factor exp(-p (x - P_d)^2) is below tau in every direction.  Contraction
//    into fused multiply-adds is off here: every operation is the correctly
//    rounded FP64 one (division and square root included), the same value in
//    every implementation of the formula, so that ties at the box edges fall
//    the same way.
//  * the supports are sorted (hipCUB radix sort of the FP64 keys) and box s
//    is the ceil(s npair / nparts)-th smallest support: equal-count quantile
//    boxes; a pair belongs to the first box that holds its support.
//  * part_count_kernel / part_scan_kernel / part_write_kernel: the pair
//    lists of the partitions, concatenated in partition order, each
//    ascending, as the screening kernels build the kept list (one wave per
//    row, a ballot per partition).
//  * cross_tables_kernel: K_k^(s,s')(a, b) = exp(-t_k^2 (xi^s_a - xi^s'_b)^2),
//    xi^s the Chebyshev nodes of box s: the node values of the interpolant of
//    exp(-t_k^2 (x - y)^2) on [-b_s, b_s] x [-b_s', b_s'].
#include "tai_internal.h"
#include "tai_device.h"

#include <hipcub/hipcub.hpp>

namespace tai {
namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__global__ void __launch_bounds__(256)
support_kernel(DevBasis bs, double c, int64_t npair, double* __restrict__ sup) {
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npair) return;
  int mu, nu;
  decode_pair(bs.nb, g, mu, nu);
  const double a = bs.alpha[mu], b = bs.alpha[nu];
  const double p = a + b;
  double m = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double P = (a * bs.center[3 * mu + d] + b * bs.center[3 * nu + d]) / p;
    m = fmax(m, fabs(P));
  }
  sup[g] = m + sqrt(c / p);
}

// boxes[s] = sorted[ceil((s+1) npair / nparts) - 1]
__global__ void box_kernel(const double* __restrict__ sorted, int64_t npair, int nparts, double* __restrict__ boxes) {
  const int s = threadIdx.x;
  if (s >= nparts) return;
  const int64_t k = ((int64_t)(s + 1) * npair + nparts - 1) / nparts;
  boxes[s] = sorted[k - 1];
}

__device__ inline int part_of(double v, const double* boxes, int nparts) {
  int s = 0;
  while (s < nparts - 1 && boxes[s] < v) ++s;
  return s;
}

// One wave per row mu, 64 columns nu at a time.  Partition indices are
// compared against every s < kMaxParts with static register indices (no
// scratch arrays): counts[s][mu] = pairs (mu, nu >= mu) of partition s.
constexpr int kPartRows = 4;  // rows (one wave each) per work group

__global__ void __launch_bounds__(64 * kPartRows)
part_count_kernel(int nb, const double* __restrict__ sup, const double* __restrict__ boxes, int nparts,
                  int32_t* __restrict__ counts) {
  const int mu = blockIdx.x * kPartRows + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (mu >= nb) return;  // whole waves
  int32_t c[kMaxParts];
#pragma unroll
  for (int s = 0; s < kMaxParts; ++s) c[s] = 0;
  const int64_t p0 = pair_row_start(nb, mu);
  for (int nu0 = mu; nu0 < nb; nu0 += 64) {
    const int nu = nu0 + lane;
    const int sl = nu < nb ? part_of(sup[p0 + (nu - mu)], boxes, nparts) : kMaxParts;
#pragma unroll
    for (int s = 0; s < kMaxParts; ++s)
      if (s < nparts) c[s] += __popcll(__ballot(sl == s));
  }
  if (lane == 0) {
#pragma unroll
    for (int s = 0; s < kMaxParts; ++s)
      if (s < nparts) counts[(int64_t)s * nb + mu] = c[s];
  }
}

// exclusive scan of counts[0 .. len) in place (partition-major order), the
// per-partition totals to totals[s]
__global__ void __launch_bounds__(1024)
part_scan_kernel(int nb, int nparts, int32_t* __restrict__ counts, int32_t* __restrict__ totals) {
  __shared__ int32_t part[1024];
  const int64_t len = (int64_t)nb * nparts;
  const int t = threadIdx.x;
  const int64_t per = (len + 1023) / 1024;
  const int64_t lo = min(len, t * per), hi = min(len, lo + per);
  int32_t sum = 0;
  for (int64_t i = lo; i < hi; ++i) sum += counts[i];
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    int32_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const int32_t v = part[i];
      part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int32_t acc = part[t];
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t v = counts[i];
    counts[i] = acc;
    acc += v;
  }
  __syncthreads();
  if (t < nparts) {
    // total of partition t = start of t+1 - start of t
    const int32_t start = counts[(int64_t)t * nb];
    int32_t end;
    if (t + 1 < nparts) end = counts[(int64_t)(t + 1) * nb];
    else end = (int32_t)((int64_t)nb * (nb + 1) / 2);
    totals[t] = end - start;
  }
}

// each lane's slot: its partition's running offset plus the lanes below it
// in the same partition
__global__ void __launch_bounds__(64 * kPartRows)
part_write_kernel(int nb, const double* __restrict__ sup, const double* __restrict__ boxes, int nparts,
                  const int32_t* __restrict__ starts, int32_t* __restrict__ pairs) {
  const int mu = blockIdx.x * kPartRows + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (mu >= nb) return;  // whole waves
  int32_t pos[kMaxParts];
#pragma unroll
  for (int s = 0; s < kMaxParts; ++s) pos[s] = s < nparts ? starts[(int64_t)s * nb + mu] : 0;
  const uint64_t below = __lanemask_lt();
  const int64_t p0 = pair_row_start(nb, mu);
  for (int nu0 = mu; nu0 < nb; nu0 += 64) {
    const int nu = nu0 + lane;
    const int64_t p = p0 + (nu - mu);
    const int sl = nu < nb ? part_of(sup[p], boxes, nparts) : kMaxParts;
    int32_t slot = 0;
#pragma unroll
    for (int s = 0; s < kMaxParts; ++s) {
      if (s < nparts) {
        const uint64_t m = __ballot(sl == s);
        if (sl == s) slot = pos[s] + __popcll(m & below);
        pos[s] += __popcll(m);
      }
    }
    if (sl < kMaxParts) pairs[slot] = (int32_t)p;
  }
}

__global__ void __launch_bounds__(256)
cross_tables_kernel(const double* __restrict__ t, int nq, int n, int kind, PartBoxes bx, double* __restrict__ Kx) {
  // no contraction: each node b_s cos(theta_a) is rounded on its own, as
  // the plain tables store it, so that one box gives the plain K_k bit for bit
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nq * n * n;
  const int64_t total = per * bx.nparts * bx.nparts;
  if (g >= total) return;
  const int ss = (int)(g / per);
  const int64_t r = g - ss * per;
  const int k = (int)(r / ((int64_t)n * n));
  const int ab = (int)(r % ((int64_t)n * n));
  const int a = ab / n, b = ab % n;
  const int s = ss / bx.nparts, s2 = ss % bx.nparts;
  const double tha = (kind == 0) ? M_PI * a / (n - 1) : (2.0 * a + 1.0) * M_PI / (2.0 * n);
  const double thb = (kind == 0) ? M_PI * b / (n - 1) : (2.0 * b + 1.0) * M_PI / (2.0 * n);
  const double dx = bx.b[s] * cos(tha) - bx.b[s2] * cos(thb);
  const double tk = t[k];
  Kx[g] = exp(-tk * tk * dx * dx);
}

}  // namespace

namespace {
inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
size_t sort_temp_bytes(int64_t npair) {
  size_t temp = 0;
  hipcub::DeviceRadixSort::SortKeys(nullptr, temp, (const double*)nullptr, (double*)nullptr, (int)npair);
  return temp;
}
}  // namespace

size_t partition_work_bytes(int nb, int nparts) {
  const int64_t npair = (int64_t)nb * (nb + 1) / 2;
  return al256(8 * npair) * 2 + al256(4 * (size_t)nb * nparts) + al256(8 * kMaxParts) + al256(4 * kMaxParts) +
         al256(sort_temp_bytes(npair));
}

PartWork carve_partition_work(void* base, int nb, int nparts) {
  const int64_t npair = (int64_t)nb * (nb + 1) / 2;
  PartWork w;
  char* p = static_cast<char*>(base);
  w.sup = reinterpret_cast<double*>(p); p += al256(8 * npair);
  w.sorted = reinterpret_cast<double*>(p); p += al256(8 * npair);
  w.counts = reinterpret_cast<int32_t*>(p); p += al256(4 * (size_t)nb * nparts);
  w.boxes = reinterpret_cast<double*>(p); p += al256(8 * kMaxParts);
  w.totals = reinterpret_cast<int32_t*>(p); p += al256(4 * kMaxParts);
  w.temp = p;
  w.temp_bytes = sort_temp_bytes(npair);
  return w;
}

hipError_t launch_partition(const DevBasis& bs, double c, int nparts, const PartWork& w, int32_t* pairs,
                            hipStream_t s) {
  const int nb = bs.nb;
  const int64_t npair = (int64_t)nb * (nb + 1) / 2;
  hipLaunchKernelGGL(support_kernel, dim3(nblk(npair, 256)), dim3(256), 0, s, bs, c, npair, w.sup);
  size_t temp = w.temp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortKeys(w.temp, temp, w.sup, w.sorted, (int)npair, 0, 64, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(box_kernel, dim3(1), dim3(64), 0, s, w.sorted, npair, nparts, w.boxes);
  hipLaunchKernelGGL(part_count_kernel, dim3(nblk(nb, kPartRows)), dim3(64 * kPartRows), 0, s, nb, w.sup, w.boxes,
                     nparts, w.counts);
  hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, s, nb, nparts, w.counts, w.totals);
  hipLaunchKernelGGL(part_write_kernel, dim3(nblk(nb, kPartRows)), dim3(64 * kPartRows), 0, s, nb, w.sup, w.boxes,
                     nparts, w.counts, pairs);
  return hipGetLastError();
}

hipError_t launch_cross_tables(const double* t, int nq, int n, int kind, const PartBoxes& bx, double* Kx,
                               hipStream_t s) {
  const int64_t total = (int64_t)nq * n * n * bx.nparts * bx.nparts;
  hipLaunchKernelGGL(cross_tables_kernel, dim3(nblk(total, 256)), dim3(256), 0, s, t, nq, n, kind, bx, Kx);
  return hipGetLastError();
}

}  // namespace tai
