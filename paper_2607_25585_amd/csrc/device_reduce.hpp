// Fixed-order device reductions shared by the HIP kernels: wave butterflies,
// then the block's waves in order, then per-block partials stored to memory and
// summed in block order by a finishing launch, so every dot product is bitwise
// reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

#include "ftlm_internal.hpp"

namespace ftlm {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-level (NT threads) fixed-order sums of NV*KC per-lane values, stored to
// part[slot*NV*KC ...] with plain stores.  The grid-level sum runs in a
// separate finishing kernel launched behind this one on the same stream (the
// kernel boundary orders the stores): no device-scope fence or atomic per
// block, which on this GPU cost a write-back of the L2 each and serialise the
// grid's tail.
template <int NV, int KC, int NT = kBlock>
__device__ __forceinline__ void block_partials_store(const double (&val)[NV][KC], double *part, int slot) {
  __shared__ double red[NT / 64][NV * KC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NV; a++)
#pragma unroll
    for (int q = 0; q < KC; q++) {
      double s = wave_sum(val[a][q]);
      if (lane == 0) red[wv][a * KC + q] = s;
    }
  __syncthreads();
  if (threadIdx.x < NV * KC) {
    double s = 0;
    for (int w2 = 0; w2 < NT / 64; w2++) s += red[w2][threadIdx.x];
    part[(size_t)slot * NV * KC + threadIdx.x] = s;
  }
}

// Sum of x[bx * stride] over bx < n by the whole block in a fixed order (thread
// t takes bx = t, t + 256, ...; then wave butterflies and the waves in order).
// Every thread gets the total.  Called uniformly by all threads of the block.
__device__ __forceinline__ double block_sum_strided(const double *x, unsigned n, size_t stride) {
  __shared__ double sh[kBlock / 64];
  double s = 0;
  for (unsigned bx = threadIdx.x; bx < n; bx += kBlock) s += x[(size_t)bx * stride];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0;
#pragma unroll
  for (int w2 = 0; w2 < kBlock / 64; w2++) tot += sh[w2];
  __syncthreads();
  return tot;
}

}  // namespace ftlm
