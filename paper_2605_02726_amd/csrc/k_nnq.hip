// Quantisation of the decoder parameters and their Exp-Golomb rate
// (Section IV-E): every parameter belongs to one group (submodule ARM,
// synthesis, upsampling or IFCE; weights or biases) with its own
// quantisation step; a quantised parameter becomes step * rint(p / step)
// (ties to even) and its integer v is coded as u = 2v - 1 (v > 0) or -2v
// (v <= 0) with an order-k Exp-Golomb code of 2 floor(log2(u + 2^k)) - k + 1
// bits.  One workgroup per image writes the (quantised or unquantised)
// parameters from the kept copy into theta and totals, per group and per
// order k = 0..CC_NNQ_NK-1, the code lengths (integer sums: exact and
// independent of order).
#include "cc_internal.h"

#include <math.h>

namespace {

__global__ __launch_bounds__(1024) void k_nnq(Launch L, NnqPack A) {
  __shared__ unsigned long long cnt[CC_NNQ_NG * CC_NNQ_NK];
  const int im = blockIdx.x;
  const CDesc* d = (const CDesc*)L.d[im];
  const int tid = threadIdx.x;
  for (int i = tid; i < CC_NNQ_NG * CC_NNQ_NK; i += blockDim.x) cnt[i] = 0ull;
  __syncthreads();
  float* theta = d->theta + d->n_lat;
  for (int p = tid; p < d->n_par; p += blockDim.x) {
    const int g = d->nnq_group[p];
    const float x = d->nnq_keep[p];
    const float st = A.step[im][g];
    if (st > 0.0f) {
      const float q = rintf(x / st);
      theta[p] = st * q;
      const long long v = (long long)q;
      const unsigned long long u = v > 0 ? (unsigned long long)(2 * v - 1) : (unsigned long long)(-2 * v);
      for (int k = 0; k < CC_NNQ_NK; ++k) {
        const unsigned long long x2 = u + (1ull << k);
        const int m = 63 - __clzll((long long)x2);
        atomicAdd(&cnt[g * CC_NNQ_NK + k], (unsigned long long)(2 * m - k + 1));
      }
    } else {
      theta[p] = x;
    }
  }
  __syncthreads();
  for (int i = tid; i < CC_NNQ_NG * CC_NNQ_NK; i += blockDim.x) d->nnq_bits[i] = (long long)cnt[i];
}

}  // namespace

int cc_launch_nnq(const Launch& l, const NnqPack& a, hipStream_t st) {
  hipLaunchKernelGGL(k_nnq, dim3(l.n), dim3(1024), 0, st, l, a);
  return hipGetLastError() == hipSuccess ? CC_OK : CC_EDEVICE;
}
