// pf_device.hpp -- device-side building blocks shared by the gfx950 step and
// reduction kernels: per-precision math, wave64 cross-lane moves, boundary
// ghost maps and buffer stores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf_internal.hpp"

namespace pf {

// ------------------------------------------------------------------ math

template <typename T> struct Math;

template <> struct Math<float> {
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
  // tanh(x) = sign(x) (1 - e) / (1 + e), e = exp(-2|x|), with the hardware
  // base-2 exponential; absolute error a few ulp of 1.
  static __device__ __forceinline__ float tanh_(float x) {
    const float m2log2e = -2.8853900817779268f;  // -2 / ln 2
    float e = __builtin_amdgcn_exp2f(m2log2e * __builtin_fabsf(x));
    float t = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
    return __builtin_copysignf(t, x);
  }
  static __device__ __forceinline__ bool finite(float x) { return __builtin_isfinite(x); }
};

template <> struct Math<double> {
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
  static __device__ __forceinline__ double tanh_(double x) { return tanh(x); }
  static __device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }
};

// ------------------------------------------------------- frame decision
// A phi = 0 crossing between rows m and m + 1 (phi_m >= 0 > phi_{m+1}) lies
// at height y = (m + phi_m / (phi_m - phi_{m+1})) h; the frame moves when some
// y >= shift_row h, both sides rounded in FP64 (thr = shift_row h).  The
// fraction lies in [0, 1], so a crossing from a row at or above shift_row
// always qualifies and one from a row below shift_row - 1 never does (FP64
// rounding is monotone and cannot close a gap of h): callers skip those rows
// and only the row just below shift_row evaluates the quotient.
template <typename T>
__device__ __forceinline__ bool crossing_reaches(T fC, T fN, int m, int shift_row, double thr,
                                                 double hd) {
  if (m >= shift_row) return true;
  const double fc = (double)fC, fn = (double)fN;
  return ((double)m + fc / (fc - fn)) * hd >= thr;
}

// ------------------------------------------------------- cross-lane moves
// Lane i of a wave64 holds lattice column x0 + i.  from_right() returns the
// value of lane i + 1 (column x + 1), from_left() the value of lane i - 1;
// the end lanes receive 0.  Both are single DPP wave shifts.

#define PF_DPP_WAVE_SHL1 0x130  // lane i reads lane i + 1
#define PF_DPP_WAVE_SHR1 0x138  // lane i reads lane i - 1

__device__ __forceinline__ float from_right(float v) {
  return __builtin_amdgcn_update_dpp(0.0f, v, PF_DPP_WAVE_SHL1, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_left(float v) {
  return __builtin_amdgcn_update_dpp(0.0f, v, PF_DPP_WAVE_SHR1, 0xF, 0xF, true);
}
__device__ __forceinline__ double from_right(double v) {
  int2 a = __builtin_bit_cast(int2, v);
  a.x = __builtin_amdgcn_update_dpp(0, a.x, PF_DPP_WAVE_SHL1, 0xF, 0xF, true);
  a.y = __builtin_amdgcn_update_dpp(0, a.y, PF_DPP_WAVE_SHL1, 0xF, 0xF, true);
  return __builtin_bit_cast(double, a);
}
__device__ __forceinline__ double from_left(double v) {
  int2 a = __builtin_bit_cast(int2, v);
  a.x = __builtin_amdgcn_update_dpp(0, a.x, PF_DPP_WAVE_SHR1, 0xF, 0xF, true);
  a.y = __builtin_amdgcn_update_dpp(0, a.y, PF_DPP_WAVE_SHR1, 0xF, 0xF, true);
  return __builtin_bit_cast(double, a);
}
__device__ __forceinline__ int from_right(int v) {
  return __builtin_amdgcn_update_dpp(0, v, PF_DPP_WAVE_SHL1, 0xF, 0xF, true);
}
__device__ __forceinline__ int from_left(int v) {
  return __builtin_amdgcn_update_dpp(0, v, PF_DPP_WAVE_SHR1, 0xF, 0xF, true);
}

// ------------------------------------------------------------- ghost maps
// Lattice index i (possibly outside [0, n)) -> stored index.  PERIODIC wraps;
// NOFLUX mirrors about the boundary face (-1 -> 0, -2 -> 1, n -> n-1, ...).
__device__ __forceinline__ int ghost(int i, int n, int bc) {
  if (bc == PF_BC_PERIODIC) {
    int m = i % n;
    return m < 0 ? m + n : m;
  }
  int p = 2 * n;
  int m = i % p;
  if (m < 0) m += p;
  return m < n ? m : p - 1 - m;
}

// Same map for indices within one period of the lattice (-n <= i < 2n), with
// no division: used for row indices inside the time-step loops.
__device__ __forceinline__ int ghost_near(int i, int n, int bc) {
  if (i < 0) return bc == PF_BC_PERIODIC ? i + n : -i - 1;
  if (i >= n) return bc == PF_BC_PERIODIC ? i - n : 2 * n - 1 - i;
  return i;
}

// Store v at column x of the row starting at `row` (nx elements) from the
// lanes with ok set, without a branch: a raw buffer store whose record is the
// row, the other lanes given an offset beyond it, which the hardware drops.
// Straight-line stores keep the row pipelines of the step kernels in fewer
// basic blocks.
template <typename T>
__device__ __forceinline__ void store_row(T *row, int nx, int x, bool ok, T v) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(row, 0, nx * (int)sizeof(T), 0x00020000);  // word 3: raw 32-bit access (gfx9 family)
  // the dropped lanes' offset 2^31 lies past every record: nx * 8 < 2^31
  // because the x-y plane is at most 2^30 - 1 cells and ny >= 4
  const int off = ok ? x * (int)sizeof(T) : (int)0x80000000u;
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off, 0, 0);
  } else {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, off, 0, 0);
  }
}

}  // namespace pf
