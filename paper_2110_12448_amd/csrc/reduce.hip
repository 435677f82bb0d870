// reduce.hip -- grid-wide tip / solid-fraction / finiteness reduction of a
// stored state (gfx950).
//
// Tip (most advanced solid-liquid interface along y, Sec. 4.3.2 and 6.2.1):
// over every vertical cell pair with phi >= 0 below and phi < 0 above, the
// phi = 0 crossing y = (j + phi_j / (phi_j - phi_{j+1})) h by linear
// interpolation; the largest y wins, ties go to the smallest linear index.
// Solid fraction: (1/N) sum (1 + phi)/2.  All accumulation in FP64; phi itself
// is evaluated in the field precision exactly as the step kernels do.
//
// Schedule: each wave64 walks up 64 adjacent columns of one z layer over a
// run of `rows` rows, loading psi and U once per cell and evaluating tanh
// once per cell (phi of the row above is carried to the next row; a run
// evaluates one extra row above its end for the last crossing test).  The
// walk goes in chunks of kChunk rows whose loads are all issued before any
// is used; per column the highest crossing row of the run is kept by selects
// and its FP64 height formed once at the end of the run.  Runs are ordered
// strip-fastest, so consecutive waves read adjacent 256-byte row pieces; the
// grid holds up to kMaxReduceBlocks workgroups of kReduceWaves waves and
// strides over the runs.  Per-wave FP64 partials are combined by wave
// shuffles and per workgroup, then in workgroup order by a second,
// one-workgroup launch (deterministic for a given lattice; no grid-wide fence
// and arrival counter, whose device-scope fences cost far more on this device
// than the extra launch).
#include "pf_device.hpp"
#include "tip_device.hpp"

namespace pf {

namespace {

// waves per workgroup of the main pass (one partial per workgroup)
constexpr int kReduceWaves = 4;
// rows of a column walk whose loads are issued together
constexpr int kChunk = 8;

template <typename T>
__global__ __launch_bounds__(64 * kReduceWaves) void reduce_kernel(ReduceArgs<T> a) {
  using M = Math<T>;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  // the frame record (its pending shift decides which stored row a frame
  // row reads); workgroup 0 also copies it into the result record
  const FrameState fr = a.frame ? *a.frame : FrameState{0, a.pending, 0};
  const int pend = fr.pending;
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const long long wave = (long long)blockIdx.x * wpb + (threadIdx.x >> 6);
  const long long nwaves = (long long)gridDim.x * wpb;
  const int nstrips = (nx + 63) >> 6;
  const int rows = a.rows;
  const int nsegs = (ny + rows - 1) / rows;
  const long long items = (long long)nstrips * nsegs * nz;
  const T isq2 = T(0.70710678118654752);
  const size_t plane = (size_t)nx * (size_t)ny;
  TipAcc acc;
  tip_init(acc);
  // stored row of frame row j (a pending shift reads one row up, the top
  // row repeated)
  auto srow = [&](int j) -> size_t { return (size_t)(pend ? min(j + 1, ny - 1) : j) * nx; };
  for (long long it = wave; it < items; it += nwaves) {
    const int strip = (int)(it % nstrips);
    const long long r2 = it / nstrips;
    const int seg = (int)(r2 % nsegs);
    const int l = (int)(r2 / nsegs);
    const int x = strip * 64 + lane;
    const bool in = x < nx;
    const size_t base = (size_t)l * plane + (size_t)(in ? x : nx - 1);
    const int y0 = seg * rows;
    const int ye = min(y0 + rows, ny);
    // per column the highest crossing row wins: crossing heights lie in
    // [j, j + 1) h, so a higher row is always further up; the walk keeps
    // that row and its two phi values with selects (no branch) and the FP64
    // height is formed once per run.  Rows go in chunks of kChunk whose loads
    // are all issued before any is used (rows past the run reload its last
    // row and are not counted).
    int bj = -1;
    T bf = T(0), bfn = T(0);
    double sf = 0.0;
    unsigned bad = 0u;
    T p = a.psi[base + srow(y0)];
    T f = T(0);  // phi of the first row: formed once the first chunk's loads are issued
    for (int j0 = y0; j0 < ye; j0 += kChunk) {
      T uv[kChunk], pv[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        const int j = min(j0 + k, ye - 1);
        uv[k] = a.U[base + srow(j)];
        pv[k] = a.psi[base + srow(min(j + 1, ny - 1))];
      }
      if (j0 == y0) f = M::tanh_(p * isq2);
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        const int j = j0 + k;
        if (j < ye) {
          const bool up = j + 1 < ny;
          const T pn = pv[k];
          const T fn = M::tanh_(pn * isq2);
          sf += (double)f;
          bad += (M::finite(p) && M::finite(uv[k])) ? 0u : 1u;
          const bool cr = up && f >= T(0) && fn < T(0);
          bj = cr ? j : bj;
          bf = cr ? f : bf;
          bfn = cr ? fn : bfn;
          p = pn;
          f = fn;
        }
      }
    }
    if (in) {
      // sum over the run of (1 + phi)/2
      acc.fs += 0.5 * ((double)(ye - y0) + sf);
      acc.bad += bad;
      if (bj >= 0) {
        const double fd = (double)bf, fnd = (double)bfn;
        const double yy = ((double)bj + fd / (fd - fnd)) * a.hd;
        const long long id = (long long)x + (long long)nx * ((long long)bj + (long long)ny * l);
        if (yy > acc.y || (yy == acc.y && id < acc.idx)) {
          acc.y = yy;
          acc.idx = id;
        }
      }
    }
  }
  __shared__ TipAcc lds[kReduceWaves];
  tip_block_partial(acc, a.red.partials, lds);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.red.result->frame = a.frame ? fr : FrameState{0, 0, 0};
}

// The grid's partials in block order -> the result record (one workgroup of
// kFinishThreads; each thread holds at most kFinishPer partials).
constexpr int kFinishThreads = 256;
constexpr int kFinishPer = kMaxReduceBlocks / kFinishThreads;
static_assert(kFinishPer * kFinishThreads >= kMaxReduceBlocks, "every partial has a thread");

__global__ __launch_bounds__(kFinishThreads) void reduce_finish_kernel(Reduce red, int nblocks) {
  __shared__ TipAcc lds[kFinishThreads / 64];
  const TipAcc t = tip_combine<kFinishPer, kFinishThreads / 64>(red.partials, nblocks, lds);
  if (threadIdx.x == 0) {
    TipResult *res = red.result;
    res->y = t.y;
    res->idx = t.idx;
    res->fs_sum = t.fs;
    res->bad = t.bad;
    res->found = t.y > -__builtin_inf() ? 1 : 0;
  }
}

}  // namespace

size_t tip_acc_bytes() { return sizeof(TipAcc); }

// Runs of 32 rows, halved (down to kMinRunRows) until there are kRunTarget of
// them, so small lattices still spread over the chip.
constexpr int kRunTarget = 4096;
constexpr int kMinRunRows = 4;

GeomReduce reduce_geometry(int nx, int ny, int nz) {
  const long long cols = (long long)((nx + 63) / 64) * nz;
  int rows = 32;
  while (rows > kMinRunRows && cols * ((ny + rows - 1) / rows) < kRunTarget) rows /= 2;
  const long long items = cols * ((ny + rows - 1) / rows);
  const long long blocks = (items + kReduceWaves - 1) / kReduceWaves;
  return GeomReduce{rows, (int)(blocks < kMaxReduceBlocks ? blocks : kMaxReduceBlocks)};
}

int reduce_blocks(int nx, int ny, int nz) { return reduce_geometry(nx, ny, nz).blocks; }

template <typename T>
hipError_t launch_reduce(const ReduceArgs<T> &a, hipStream_t st) {
  const GeomReduce g = reduce_geometry(a.nx, a.ny, a.nz);
  ReduceArgs<T> b = a;
  b.rows = g.rows;
  hipLaunchKernelGGL((reduce_kernel<T>), dim3(g.blocks), dim3(64 * kReduceWaves), 0, st, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_finish_kernel, dim3(1), dim3(kFinishThreads), 0, st, b.red, g.blocks);
  return hipGetLastError();
}

template hipError_t launch_reduce<float>(const ReduceArgs<float> &, hipStream_t);
template hipError_t launch_reduce<double>(const ReduceArgs<double> &, hipStream_t);

}  // namespace pf
