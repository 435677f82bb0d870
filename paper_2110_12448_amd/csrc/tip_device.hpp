// tip_device.hpp -- the FP64 tip / solid-fraction / finiteness record of the
// reduction kernels and its wave, workgroup and grid combination (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "pf_internal.hpp"

namespace pf {

struct TipAcc {
  double y;       // best crossing height, -inf if none
  long long idx;  // linear index of its lower cell (ties: smallest)
  double fs;      // sum of (1 + phi)/2
  unsigned bad;   // count of non-finite psi or U
};

__device__ __forceinline__ void tip_init(TipAcc &a) {
  a.y = -__builtin_inf();
  a.idx = 0x7fffffffffffffffLL;
  a.fs = 0.0;
  a.bad = 0u;
}

__device__ __forceinline__ void tip_merge(TipAcc &a, double y, long long idx, double fs,
                                          unsigned bad) {
  if (y > a.y || (y == a.y && idx < a.idx)) {
    a.y = y;
    a.idx = idx;
  }
  a.fs += fs;
  a.bad += bad;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  return __shfl_xor(v, m, 64);
}
__device__ __forceinline__ long long shfl_xor_ll(long long v, int m) {
  return __shfl_xor(v, m, 64);
}

// Butterfly over the 64 lanes; every lane ends with the wave total.
__device__ __forceinline__ void tip_wave_reduce(TipAcc &a) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    double y = shfl_xor_d(a.y, m);
    long long i = shfl_xor_ll(a.idx, m);
    double f = shfl_xor_d(a.fs, m);
    unsigned b = (unsigned)__shfl_xor((int)a.bad, m, 64);
    tip_merge(a, y, i, f, b);
  }
}

// Block reduction of one TipAcc per wave (blockDim = 64 * nwaves <= 1024):
// the block's total is written to partials[blockIdx.x].  `lds` needs room for
// one TipAcc per wave.  No grid-wide fence or counter: a second launch (tip_combine)
// combines the partials, the kernel boundary ordering the two.
__device__ __forceinline__ void tip_block_partial(TipAcc a, TipAcc *partials, TipAcc *lds) {
  tip_wave_reduce(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  if (lane == 0) lds[wave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    TipAcc b = lds[0];
    for (int w = 1; w < nw; ++w) tip_merge(b, lds[w].y, lds[w].idx, lds[w].fs, lds[w].bad);
    partials[blockIdx.x] = b;
  }
}

// One block of kWaves waves combines n <= kPer * blockDim.x partials in a
// fixed order (thread t takes partials t, t + blockDim.x, ... in turn, then
// the butterfly and the waves in order: deterministic for a given n and block
// size) and returns the total in thread 0.  Each thread issues its loads
// before merging any of them.  `lds` needs room for kWaves TipAcc.
template <int kPer, int kWaves>
__device__ __forceinline__ TipAcc tip_combine(const TipAcc *partials, int n, TipAcc *lds) {
  TipAcc p[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = (int)threadIdx.x + k * (int)blockDim.x;
    if (b < n)
      p[k] = partials[b];
    else
      tip_init(p[k]);
  }
  TipAcc c = p[0];
#pragma unroll
  for (int k = 1; k < kPer; ++k) tip_merge(c, p[k].y, p[k].idx, p[k].fs, p[k].bad);
  tip_wave_reduce(c);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds[wave] = c;
  __syncthreads();
  TipAcc t = lds[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) tip_merge(t, lds[w].y, lds[w].idx, lds[w].fs, lds[w].bad);
  return t;
}

}  // namespace pf
