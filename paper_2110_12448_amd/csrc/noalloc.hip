// noalloc.hip -- pf_tip_fields: the reduction of pf_tip_state on caller-held
// device fields, with its partials and result in a fixed device
// array of this library (no device memory is allocated by the call).
//
// The array below is a device symbol.  Its host-side name is only a stand-in
// for the symbol: its device address is obtained once per device with
// hipGetSymbolAddress and only that address is passed to kernels and copies.
// Every call on one device shares that device's array, so calls that overlap
// on one device (two streams, two host threads) race; calls on different
// devices do not.
#include <string.h>

#include <mutex>
#include <string>

#include "pf_device.hpp"
#include "tip_device.hpp"
#include "pf_internal.hpp"

using namespace pf;

namespace {

constexpr int kMaxDev = 64;
// partials of every workgroup of the reduction, then its result
constexpr size_t kPartialsBytes = (size_t)kMaxReduceBlocks * sizeof(TipAcc);
constexpr size_t kResultOff = (kPartialsBytes + 255) & ~(size_t)255;
constexpr size_t kScratchBytes = kResultOff + 256;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDev];  // device address of `scratch` per device (set once)

int fail_na(int code, const std::string &m) { return report_error(code, m.c_str()); }

// Device address of this device's scratch array (looked up once per device).
int scratch_ptr(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail_na(PF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
    g_ptr[dev] = ptr;
  }
  *out = reinterpret_cast<unsigned char *>(g_ptr[dev]);
  return PF_OK;
}

template <typename T>
int run(const void *psi, const void *U, int nx, int ny, int nz, double h, int pending,
        unsigned char *base, hipStream_t st, TipResult *res) {
  ReduceArgs<T> a;
  a.psi = reinterpret_cast<const T *>(psi);
  a.U = reinterpret_cast<const T *>(U);
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.rows = 0;
  a.hd = h;
  a.frame = nullptr;
  a.pending = pending;
  a.red = Reduce{reinterpret_cast<TipAcc *>(base), reinterpret_cast<TipResult *>(base + kResultOff)};
  hipError_t e = launch_reduce<T>(a, st);
  if (e == hipSuccess) e = hipMemcpyAsync(res, a.red.result, sizeof(TipResult), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail_na(PF_ERR_DEVICE, std::string("reduction: ") + hipGetErrorString(e));
  return PF_OK;
}

}  // namespace

extern "C" {

int pf_tip_fields(const void *psi, const void *U, int32_t precision, int32_t nx, int32_t ny,
                  int32_t nz, double h, int32_t pending, void *stream, pf_tip *out) {
  if (!psi || !U || !out) return fail_na(PF_ERR_ARG, "psi, U and out must not be NULL");
  if (precision != PF_F32 && precision != PF_F64)
    return fail_na(PF_ERR_ARG, "precision must be PF_F32 or PF_F64");
  if (nx < 1 || ny < 2 || nz < 1) return fail_na(PF_ERR_ARG, "need nx >= 1, ny >= 2, nz >= 1");
  if ((long long)nx * ny > (1LL << 30) - 1 || (long long)ny * nz > (1LL << 30) - 1 ||
      (double)nx * ny * nz > 4.0e9)
    return fail_na(PF_ERR_ARG, "lattice beyond the library's limits (x-y and y-z planes below "
                               "2^30 cells, at most 4e9 cells)");
  if (!(h > 0.0)) return fail_na(PF_ERR_ARG, "h must be > 0");
  if (pending != 0 && pending != 1) return fail_na(PF_ERR_ARG, "pending must be 0 or 1");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev)
    return fail_na(PF_ERR_DEVICE, "no usable current device");
  unsigned char *base = nullptr;
  int rc = scratch_ptr(dev, &base);
  if (rc != PF_OK) return rc;
  TipResult r;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  rc = precision == PF_F64 ? run<double>(psi, U, nx, ny, nz, h, pending, base, st, &r)
                           : run<float>(psi, U, nx, ny, nz, h, pending, base, st, &r);
  if (rc != PF_OK) return rc;
  pf_tip t;
  memset(&t, 0, sizeof(t));
  t.found = r.found;
  t.nonfinite = r.bad ? 1 : 0;
  t.solid_fraction = r.fs_sum / ((double)nx * ny * nz);
  if (r.found) {
    t.index = r.idx;
    t.x = (double)(r.idx % nx) * h;
    t.z = nz > 1 ? (double)(r.idx / ((long long)nx * ny)) * h : 0.0;
    t.y_frame = r.y;
    t.y_lab = r.y;
  } else {
    t.index = -1;
  }
  *out = t;
  if (r.bad) return fail_na(PF_ERR_NONFINITE, "fields hold NaN or Inf values");
  return PF_OK;
}

}  // extern "C"
