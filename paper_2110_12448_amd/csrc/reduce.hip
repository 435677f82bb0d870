// reduce.hip -- grid-wide tip / solid-fraction / finiteness reduction of a
// stored state (gfx950).
//
// Tip (most advanced solid-liquid interface along y, Sec. 4.3.2 and 6.2.1):
// over every vertical cell pair with phi >= 0 below and phi < 0 above, the
// phi = 0 crossing y = (j + phi_j / (phi_j - phi_{j+1})) h by linear
// interpolation; the largest y wins, ties go to the smallest linear index.
// Solid fraction: (1/N) sum (1 + phi)/2.  All accumulation in FP64; phi itself
// is evaluated in the field precision exactly as the step kernels do.
#include "pf_device.hpp"

namespace pf {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs<T> a) {
  using M = Math<T>;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int pend = a.frame->pending;
  const int lines = ny * nz;
  const T isq2 = T(0.70710678118654752);
  TipAcc acc;
  tip_init(acc);
  for (int line = blockIdx.x; line < lines; line += gridDim.x) {
    const int j = line % ny;
    const int l = line / ny;
    const int jp = pend ? min(j + 1, ny - 1) : j;
    const int jq = pend ? min(j + 2, ny - 1) : j + 1;
    const size_t base = (size_t)l * (size_t)ny * (size_t)nx;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
      T p = a.psi[base + (size_t)jp * nx + x];
      T u = a.U[base + (size_t)jp * nx + x];
      T f = M::tanh_(p * isq2);
      double fd = (double)f;
      acc.fs += 0.5 * (1.0 + fd);
      acc.bad += (M::finite(p) && M::finite(u)) ? 0u : 1u;
      if (j <= ny - 2 && f >= T(0)) {
        T fn = M::tanh_(a.psi[base + (size_t)jq * nx + x] * isq2);
        if (fn < T(0)) {
          double fnd = (double)fn;
          double yy = ((double)j + fd / (fd - fnd)) * a.hd;
          long long id = (long long)x + (long long)nx * ((long long)j + (long long)ny * l);
          if (yy > acc.y || (yy == acc.y && id < acc.idx)) {
            acc.y = yy;
            acc.idx = id;
          }
        }
      }
    }
  }
  __shared__ TipAcc lds[16];
  TipResult *res = a.red.result;
  tip_block_and_grid(acc, a.red.partials, a.red.counter, lds, [res](const TipAcc &t) {
    res->y = t.y;
    res->idx = t.idx;
    res->fs_sum = t.fs;
    res->bad = t.bad;
    res->found = t.y > -__builtin_inf() ? 1 : 0;
  });
}

}  // namespace

size_t tip_acc_bytes() { return sizeof(TipAcc); }

int reduce_blocks(int nx, int ny, int nz) {
  (void)nx;
  long long lines = (long long)ny * nz;
  return (int)(lines < 256 ? lines : 256);  // one block per CU: few grid-wide fences
}

template <typename T>
hipError_t launch_reduce(const ReduceArgs<T> &a, hipStream_t st) {
  int blocks = reduce_blocks(a.nx, a.ny, a.nz);
  hipLaunchKernelGGL((reduce_kernel<T>), dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_reduce<float>(const ReduceArgs<float> &, hipStream_t);
template hipError_t launch_reduce<double>(const ReduceArgs<double> &, hipStream_t);

}  // namespace pf
