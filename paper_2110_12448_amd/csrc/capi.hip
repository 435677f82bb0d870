// capi.hip -- the C ABI of include/pf.h: parameter validation, workspace
// layout, state upload/download and the per-step launch sequence.
#include <math.h>
#include <cmath>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "pf_device.hpp"
#include "pf_internal.hpp"

using namespace pf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

}  // namespace

namespace pf {
int report_error(int code, const char *msg) { return fail(code, msg); }
}  // namespace pf

namespace {

#define PF_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail(PF_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// thin-interface constant a2 = 47/75 (Sec. 2.1): default lambda = D~ / a2
constexpr double kA2 = 47.0 / 75.0;
// Default 2D geometry, -k: k waves per SIMD, so that the launch fills whole
// rounds of the device (a fraction of a round leaves the SIMDs that hold one
// wave more to finish alone).  Each segment recomputes about 1.5 rows of
// work below it, so fewer, longer segments cost less, while more waves per
// SIMD hide more latency.  With R = strips * ny / SIMDs rows per SIMD, k =
// round(R^0.4) in FP32 and round(0.75 R^0.4) in FP64 (at most 3 waves of
// the FP64 kernel fit a SIMD), within [1, 64]: fitted to sweeps of k on
// 256^2 .. 8192^2 lattices (1024x2048: 4 waves per SIMD); on the lattices
// measured it is within 5% of the fastest k, which pf_autotune finds.
int default_seg2d(int nx, int ny, int precision, int ncu) {
  const double strips = (nx + 59) / 60;
  const double R = strips * ny / (4.0 * std::max(1, ncu));
  const double k = (precision == PF_F64 ? 0.75 : 1.0) * std::pow(R, 0.4);
  return -std::min(64, std::max(1, (int)std::lround(k)));
}
// Batched members keep segments of at least 8 rows: the batch fills the chip
// by itself.
constexpr int kMinSegBatch2D = 8;
constexpr size_t kMaxLds3DBytes = 163840;  // LDS one gfx950 workgroup may allocate
constexpr size_t kMaxLds3D = kMaxLds3DBytes;
// Default 3D geometry.  z rows per wide workgroup: 14 in FP32 (16 waves, the
// most one workgroup holds: one workgroup per CU at the kernel's 100-128
// VGPRs, ring rows costing 16/14), 6 in FP64 (8 waves, its launch bound:
// two waves per SIMD at its ~230 VGPRs, ring rows costing 8/6).
// Segments: the count that minimises the estimated time rounds x (rows + 2.5),
// where rounds = ceil(workgroups / resident workgroups) and a segment's
// prologue costs about 2.5 rows; the rows of a column are split evenly.  On
// 256^3 FP32 (4 wide strips of 19 z tiles and a thin strip of 6) that is 3
// segments of 85-86 rows (the thin strip 4 of 64), 252 workgroups in one
// round; pf_autotune refines it per lattice.
std::pair<int, int> default_geom3d(const pf_params *p, int ncu) {
  const bool f64 = p->precision == PF_F64;
  const int zt = std::min(f64 ? 6 : 14, std::max(1, p->nz));
  const int nw = zt + 2;
  const size_t lds = step3d_lds_bytes(p->nx, zt, f64 ? 8 : 4);
  const int by_waves = std::max(1, (f64 ? 8 : 16) / nw);
  const int by_lds = std::max(1, (int)(kMaxLds3DBytes / lds));
  const long long resident = (long long)std::max(1, ncu) * std::min(by_waves, by_lds);
  int best = p->ny;
  double best_cost = 1e300;
  for (int n = 1; n <= std::max(1, p->ny / 4); ++n) {
    const int rows = (p->ny + n - 1) / n;
    const long long blocks = geom3d(p->nx, p->ny, p->nz, rows, zt).blocks;
    const double cost = (double)((blocks + resident - 1) / resident) * (rows + 2.5);
    if (cost < best_cost - 1e-9) {
      best_cost = cost;
      best = rows;
    }
  }
  return {best, zt};
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t cells(const pf_params *p) {
  return (size_t)p->nx * (size_t)p->ny * (size_t)(p->dim == 3 ? p->nz : 1);
}

void weights_of(const pf_params *p, double w[3]) {
  if (p->scheme == PF_SCHEME_STD) {
    w[0] = 1.0; w[1] = 0.0; w[2] = 0.0;
  } else if (p->scheme == PF_SCHEME_WEIGHTS) {
    double s = p->weights[0] + p->weights[1] + (p->dim == 3 ? p->weights[2] : 0.0);
    w[0] = p->weights[0] / s;
    w[1] = p->weights[1] / s;
    w[2] = p->dim == 3 ? p->weights[2] / s : 0.0;
  } else if (p->dim == 2) {
    w[0] = 2.0 / 3.0; w[1] = 1.0 / 3.0; w[2] = 0.0;
  } else {
    w[0] = 1.0 / 3.0; w[1] = 2.0 / 3.0; w[2] = 0.0;
  }
}

// smallest F1 of Eq. Thermal_F1 over the lattice rows for the zeta offset
// off = s h - y0 - Vp t (zeta = y + off is linear in y, so the extreme rows
// bound it); 1 if isothermal
double f1_min_at(const pf_params *p, double off) {
  if (!(p->lT > 0.0)) return 1.0;
  double zmax = (p->ny - 1) * p->h + off;
  double zmin = off;
  double a = 1.0 - (1.0 - p->k) * zmax / p->lT;
  double b = 1.0 - (1.0 - p->k) * zmin / p->lT;
  return a < b ? a : b;
}

// at t = 0 with no frame shift
double f1_min(const pf_params *p) { return f1_min_at(p, -p->y0); }

// explicit limit h^2 / (2 dim max(D~, 1/F1_min))
double stable_dt_for(const pf_params *p, double f1) {
  return p->h * p->h / (2.0 * p->dim * std::max(p->D, 1.0 / f1));
}

struct Layout {
  size_t psi[2], U[2], grain, grain2, rot, frame[3], partials, result, total;
};

Layout layout_of(const pf_params *p) {
  Layout L;
  size_t es = p->precision == PF_F64 ? 8 : 4;
  size_t n = cells(p);
  size_t o = 0;
  for (int i = 0; i < 2; ++i) { L.psi[i] = o; o += align256(n * es); }
  for (int i = 0; i < 2; ++i) { L.U[i] = o; o += align256(n * es); }
  L.grain = o; o += align256(p->n_grains > 1 ? n : 1);
  L.grain2 = o; o += align256(p->dynamic_grains ? n : 1);  // the next level's map
  L.rot = o; o += align256((size_t)(p->n_grains > 0 ? p->n_grains : 1) * 9 * es);
  for (int i = 0; i < 3; ++i) { L.frame[i] = o; o += 256; }
  // one partial per workgroup of the reduction
  int nb = reduce_blocks(p->nx, p->ny, p->dim == 3 ? p->nz : 1);
  L.partials = o; o += align256((size_t)(nb + 64) * tip_acc_bytes());
  L.result = o; o += 256;
  L.total = o;
  return L;
}

int validate(const pf_params *p) {
  if (!p) return fail(PF_ERR_ARG, "params is NULL");
  if (p->dim != 2 && p->dim != 3) return fail(PF_ERR_ARG, "dim must be 2 or 3");
  if (p->nx < 4 || p->ny < 4 || (p->dim == 3 && p->nz < 4))
    return fail(PF_ERR_ARG, "every lattice side must be >= 4");
  if ((double)p->nx * p->ny * (p->dim == 3 ? p->nz : 1) > 4.0e9)
    return fail(PF_ERR_ARG, "lattice larger than 4e9 cells");
  if ((long long)p->nx * p->ny > 2147483647LL / 2 ||
      (long long)p->ny * (p->dim == 3 ? p->nz : 1) > 2147483647LL / 2)
    return fail(PF_ERR_ARG, "x-y plane or y-z plane too large");
  if (p->precision != PF_F32 && p->precision != PF_F64)
    return fail(PF_ERR_ARG, "precision must be PF_F32 or PF_F64");
  if (p->scheme < PF_SCHEME_ISO || p->scheme > PF_SCHEME_WEIGHTS)
    return fail(PF_ERR_ARG, "unknown scheme");
  if (p->scheme == PF_SCHEME_WEIGHTS) {
    double s = p->weights[0] + p->weights[1] + (p->dim == 3 ? p->weights[2] : 0.0);
    if (!(fabs(s) > 1e-12)) return fail(PF_ERR_ARG, "shell weights sum to zero");
    if (p->dim == 2 && p->weights[2] != 0.0)
      return fail(PF_ERR_ARG, "2D has two shells: weights[2] must be 0");
  }
  if (p->antitrapping != PF_AT_APPROX && p->antitrapping != PF_AT_FULL)
    return fail(PF_ERR_ARG, "antitrapping must be PF_AT_APPROX or PF_AT_FULL");
  if (p->divergence != PF_DIV_SHELLS && p->divergence != PF_DIV_TWO_POINT)
    return fail(PF_ERR_ARG, "divergence must be PF_DIV_SHELLS or PF_DIV_TWO_POINT");
  if (p->dim == 3 && (p->antitrapping != PF_AT_APPROX || p->divergence != PF_DIV_SHELLS))
    return fail(PF_ERR_ARG, "3D runs the approximated current with shell divergences only");
  if (!(p->k > 0.0 && p->k < 1.0)) return fail(PF_ERR_ARG, "k must lie in (0, 1)");
  if (!(p->eps4 >= 0.0 && p->eps4 < 1.0 / 15.0))
    return fail(PF_ERR_ARG, "eps4 must lie in [0, 1/15)");
  if (!(p->D > 0.0)) return fail(PF_ERR_ARG, "D must be > 0");
  if (!(p->h > 0.0)) return fail(PF_ERR_ARG, "h must be > 0");
  if (!isfinite(p->lambda) || !isfinite(p->dt) || !isfinite(p->Vp) || !isfinite(p->lT) ||
      !isfinite(p->y0))
    return fail(PF_ERR_ARG, "non-finite scalar parameter");
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != PF_BC_NOFLUX && p->bc[a] != PF_BC_PERIODIC)
      return fail(PF_ERR_ARG, "bc must be PF_BC_NOFLUX or PF_BC_PERIODIC");
  if (p->frame) {
    if (p->bc[1] != PF_BC_NOFLUX) return fail(PF_ERR_ARG, "the moving frame needs no-flux y walls");
    if (p->shift_row < 1 || p->shift_row > p->ny - 2)
      return fail(PF_ERR_ARG, "shift_row must lie in [1, ny-2]");
  }
  if (p->n_grains < 1 || p->n_grains > 127) return fail(PF_ERR_ARG, "n_grains must be 1..127");
  if (p->dynamic_grains != 0 && p->dynamic_grains != 1)
    return fail(PF_ERR_ARG, "dynamic_grains must be 0 or 1");
  if (p->dynamic_grains && p->n_grains < 2)
    return fail(PF_ERR_ARG, "dynamic grains need n_grains >= 2");
  if (!p->grain_rot) return fail(PF_ERR_ARG, "grain_rot is NULL");
  for (int g = 0; g < p->n_grains; ++g) {
    const double *R = p->grain_rot + 9 * g;
    for (int i = 0; i < 9; ++i)
      if (!isfinite(R[i])) return fail(PF_ERR_ARG, "non-finite rotation entry");
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double d = 0.0;
        for (int m = 0; m < 3; ++m) d += R[m * 3 + i] * R[m * 3 + j];
        if (fabs(d - (i == j ? 1.0 : 0.0)) > 1e-9)
          return fail(PF_ERR_ARG, "grain rotation is not orthonormal");
      }
    double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                 R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (det < 0.0) return fail(PF_ERR_ARG, "grain rotation is improper (det < 0)");
    if (p->dim == 2 && (fabs(R[2]) > 1e-12 || fabs(R[5]) > 1e-12 || fabs(R[6]) > 1e-12 ||
                        fabs(R[7]) > 1e-12))
      return fail(PF_ERR_ARG, "2D grain rotations must be rotations about z");
  }
  if (p->lT > 0.0 && !(f1_min(p) > 0.0))
    return fail(PF_ERR_ARG, "F1 = 1 - (1-k) zeta / lT is not positive over the lattice");
  return PF_OK;
}

}  // namespace

struct pf_solver {
  pf_params p;
  std::vector<double> rot;
  double w[3];
  double lambda, dt;
  size_t n;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  bool own;
  Layout L;
  int cur;    // current field buffers
  int fcur;   // current frame record (0..2, advances with the frame on)
  long long step;
  int seg, ztile;  // launch geometry (2D seg < 0: -(waves per SIMD))
  int ncu;         // compute units of the device the solver was created on
  bool have_prev;
  double prev_t, prev_y;
};

namespace {

// Rows per segment of the solver's 2D geometry (the longest segment when it
// asks for waves per SIMD).
int rows2d(const pf_solver *s) {
  if (s->seg > 0) return s->seg;
  const Geom2D g = geom2d(s->p.nx, s->p.ny, s->seg, s->ncu);
  return g.segbase + (g.segrem ? 1 : 0);
}

template <typename T>
T *field(pf_solver *s, size_t off) {
  return reinterpret_cast<T *>(s->ws + off);
}

template <typename T>
Coef<T> coef_of(const pf_solver *s) {
  const pf_params &p = s->p;
  const double h = p.h, h2 = h * h;
  Coef<T> c = {};
  c.dt = (T)s->dt;
  c.k = (T)p.k;
  c.omk = (T)(1.0 - p.k);
  c.eps4 = (T)p.eps4;
  c.an0 = (T)(1.0 - 3.0 * p.eps4);
  c.an4 = (T)(4.0 * p.eps4);
  c.an16 = (T)(16.0 * p.eps4);
  c.D = (T)p.D;
  c.lambda = (T)s->lambda;
  c.inv_h = (T)(1.0 / h);
  c.h = (T)h;
  c.cStd = (T)(1.0 / h2);
  c.inv_lT = (T)(p.lT > 0.0 ? 1.0 / p.lT : 0.0);
  if (p.dim == 2) {
    // L_{1,0} = s10/h^2, L_{0,1} = s11/(2h^2) (Eqs. 2D_L10, 2D_L01)
    c.cL1 = (T)(s->w[0] / h2);
    c.cL2 = (T)(s->w[1] / (2.0 * h2));
    c.cL3 = (T)0;
    // G_{1,0} = (...)/(4h^2), G_{0,1} = (...)/(8h^2) (Eqs. Grad_10, Grad_11)
    c.cG1 = (T)(s->w[0] / (4.0 * h2));
    c.cG2 = (T)(s->w[1] / (8.0 * h2));
    c.cG3 = (T)0;
    // D_{1,0}: fluxes carry the 4-point alpha sum, /(4h^2); D_{0,1}: plaquette
    // means times dbeta, /(2h^2) (Eqs. flux_10, flux_11)
    c.cD1 = (T)(s->w[0] / (4.0 * h2));
    c.cD2 = (T)(s->w[1] / (2.0 * h2));
    c.cD3 = (T)0;
    // two-point faces carry (alpha_0 + alpha_e) dbeta: /(2h^2); links of the
    // full current carry h / |h grad psi| and enter with a factor h
    c.cT = (T)(1.0 / (2.0 * h2));
    c.at_eps = (T)(1e-12 * h2);
    c.ac_eps = (T)(4e-12 * h2);
    c.an1 = (T)(1.0 + p.eps4);
    c.an8 = (T)(8.0 * p.eps4);
  } else {
    // L_{1,0,0} = s/h^2, L_{0,1,0} = s/(4h^2), L_{0,0,1} = s/(4h^2)
    c.cL1 = (T)(s->w[0] / h2);
    c.cL2 = (T)(s->w[1] / (4.0 * h2));
    c.cL3 = (T)(s->w[2] / (4.0 * h2));
    // G_{1,0,0} = /(4h^2), G_{0,1,0} = /(16h^2), G_{0,0,1} = /(16h^2)
    c.cG1 = (T)(s->w[0] / (4.0 * h2));
    c.cG2 = (T)(s->w[1] / (16.0 * h2));
    c.cG3 = (T)(s->w[2] / (16.0 * h2));
    // D_{1,0,0} = sum abar dbeta / h^2; D_{0,1,0}, D_{0,0,1} = / (4h^2)
    c.cD1 = (T)(s->w[0] / h2);
    c.cD2 = (T)(s->w[1] / (4.0 * h2));
    c.cD3 = (T)(s->w[2] / (4.0 * h2));
    c.k1a = (T)(s->w[0] / h2 / 4.0);
    c.k1b = (T)(s->w[0] / h2 / 16.0);
    c.k2a = (T)(s->w[1] / (4.0 * h2) * 3.0 / 16.0);
    c.k2b = (T)(s->w[1] / (4.0 * h2) / 32.0);
    c.k3 = (T)(s->w[2] / (4.0 * h2) / 8.0);
    c.ac_eps = (T)(4e-12 * h2);
    c.f3_eps = (T)(16e-12 * h2);
    c.f3_scale = (T)(1.0 / (4.0 * h2));
  }
  return c;
}

template <typename T>
int upload(pf_solver *s, const pf_init *init) {
  const size_t n = s->n;
  std::vector<T> tmp(n);
  for (size_t i = 0; i < n; ++i) tmp[i] = (T)init->psi[i];
  PF_HIP(hipMemcpy(field<T>(s, s->L.psi[0]), tmp.data(), n * sizeof(T), hipMemcpyHostToDevice));
  for (size_t i = 0; i < n; ++i) tmp[i] = (T)init->U[i];
  PF_HIP(hipMemcpy(field<T>(s, s->L.U[0]), tmp.data(), n * sizeof(T), hipMemcpyHostToDevice));
  // rotation table: 2D (r00, r01, r10, r11) per grain, 3D all 9
  const int ng = s->p.n_grains;
  std::vector<T> rt((size_t)ng * 9, (T)0);
  for (int g = 0; g < ng; ++g) {
    const double *R = s->rot.data() + 9 * g;
    if (s->p.dim == 2) {
      rt[4 * g + 0] = (T)R[0];
      rt[4 * g + 1] = (T)R[1];
      rt[4 * g + 2] = (T)R[3];
      rt[4 * g + 3] = (T)R[4];
    } else {
      for (int i = 0; i < 9; ++i) rt[9 * g + i] = (T)R[i];
    }
  }
  PF_HIP(hipMemcpy(s->ws + s->L.rot, rt.data(), rt.size() * sizeof(T), hipMemcpyHostToDevice));
  return PF_OK;
}

// Grain map k (0, 1): the static map, or the two levels of a dynamic one
// (the current level is the solver's buffer parity, like psi and U).
int8_t *grain_buf(pf_solver *s, int k) {
  return reinterpret_cast<int8_t *>(s->ws + (k == 0 || !s->p.dynamic_grains ? s->L.grain
                                                                            : s->L.grain2));
}

// Argument block of the 2D step of solver s (pointers set per launch).
template <typename T>
Geom2D fill2d(pf_solver *s, Step2DArgs<T> &a, int min_seg = 1, int seg_fixed = 0) {
  const pf_params &p = s->p;
  memset(&a, 0, sizeof(a));
  Geom2D g = seg_fixed > 0   ? geom2d(p.nx, p.ny, seg_fixed)
             : min_seg <= 1 ? geom2d(p.nx, p.ny, s->seg, s->ncu)
                            : geom2d(p.nx, p.ny, std::max(rows2d(s), min_seg));
  a.grain = p.n_grains > 1 ? grain_buf(s, s->cur) : nullptr;
  a.grain_out = p.dynamic_grains ? grain_buf(s, 1 - s->cur) : nullptr;
  a.rot = field<T>(s, s->L.rot);
  a.r00 = (T)s->rot[0]; a.r01 = (T)s->rot[1]; a.r10 = (T)s->rot[3]; a.r11 = (T)s->rot[4];
  a.nx = p.nx; a.ny = p.ny; a.bcx = p.bc[0]; a.bcy = p.bc[1];
  a.wout = g.wout; a.nstrips = g.nstrips; a.nsegs = g.nsegs;
  a.segbase = g.segbase; a.segrem = g.segrem;
  a.c = coef_of<T>(s);
  a.hd = p.h; a.y0 = p.y0; a.Vp = p.Vp; a.dtd = s->dt;
  a.frame = p.frame; a.shift_row = p.shift_row;
  return g;
}

template <typename T>
int step_impl(pf_solver *s, long long nsteps, bool diffusion_only = false) {
  const pf_params &p = s->p;
  const bool frozen = p.lT > 0.0;
  const bool reduce = p.frame != 0;
  const bool multi = p.n_grains > 1;
  const Coef<T> c = coef_of<T>(s);
  auto frec = [&](int i) { return reinterpret_cast<FrameState *>(s->ws + s->L.frame[i % 3]); };
  if (p.dim == 2) {
    Step2DArgs<T> a;
    Geom2D g = fill2d<T>(s, a);
    (void)c;
    const bool two = p.divergence == PF_DIV_TWO_POINT;
    const int at = diffusion_only ? kAtDiffusionOnly
                   : p.antitrapping == PF_AT_FULL ? (two ? kAtFullTwoPoint : kAtFullShells)
                                                  : (two ? kAtApproxTwoPoint : kAtApproxShells);
    for (long long i = 0; i < nsteps; ++i) {
      a.psi_in = field<T>(s, s->L.psi[s->cur]);
      a.U_in = field<T>(s, s->L.U[s->cur]);
      a.psi_out = field<T>(s, s->L.psi[1 - s->cur]);
      a.U_out = field<T>(s, s->L.U[1 - s->cur]);
      if (multi) a.grain = grain_buf(s, s->cur);
      if (p.dynamic_grains) a.grain_out = grain_buf(s, 1 - s->cur);
      a.frame_in = frec(s->fcur);
      a.frame_out = frec(s->fcur + 1);
      a.frame_clear = frec(s->fcur + 2);
      a.step = s->step;
      PF_HIP(launch_step2d<T>(a, g, frozen, reduce, multi, at, s->stream));
      s->cur = 1 - s->cur;
      if (reduce) s->fcur = (s->fcur + 1) % 3;
      s->step += 1;
    }
  } else {
    Step3DArgs<T> a;
    memset(&a, 0, sizeof(a));
    Geom3D g = geom3d(p.nx, p.ny, p.nz, s->seg, s->ztile);
    a.grain = multi ? grain_buf(s, s->cur) : nullptr;
    a.grain_out = p.dynamic_grains ? grain_buf(s, 1 - s->cur) : nullptr;
    a.rot = field<T>(s, s->L.rot);
    for (int i = 0; i < 9; ++i) a.R[i] = (T)s->rot[i];
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz;
    a.bcx = p.bc[0]; a.bcy = p.bc[1]; a.bcz = p.bc[2];
    a.wout = g.wout; a.nstrips = g.nstrips; a.nzt = g.nzt; a.nsegs = g.nsegs; a.seg = g.seg;
    a.ztile = g.ztile;
    a.segbase = g.segbase; a.segrem = g.segrem;
    a.ncols = g.ncols; a.ncols_wide = g.ncols_wide;
    a.thin_g = g.thin_g; a.thin_G = g.thin_G; a.thin_wout = g.thin_wout;
    a.thin_nzt = g.thin_nzt; a.thin_segbase = g.thin_segbase; a.thin_segrem = g.thin_segrem;
    a.c = c;
    a.hd = p.h; a.y0 = p.y0; a.Vp = p.Vp; a.dtd = s->dt;
    a.frame = p.frame; a.shift_row = p.shift_row;
    for (long long i = 0; i < nsteps; ++i) {
      a.psi_in = field<T>(s, s->L.psi[s->cur]);
      a.U_in = field<T>(s, s->L.U[s->cur]);
      a.psi_out = field<T>(s, s->L.psi[1 - s->cur]);
      a.U_out = field<T>(s, s->L.U[1 - s->cur]);
      if (multi) a.grain = grain_buf(s, s->cur);
      if (p.dynamic_grains) a.grain_out = grain_buf(s, 1 - s->cur);
      a.frame_in = frec(s->fcur);
      a.frame_out = frec(s->fcur + 1);
      a.frame_clear = frec(s->fcur + 2);
      a.step = s->step;
      PF_HIP(launch_step3d<T>(a, g, frozen, reduce, multi, s->stream));
      s->cur = 1 - s->cur;
      if (reduce) s->fcur = (s->fcur + 1) % 3;
      s->step += 1;
    }
  }
  return PF_OK;
}

template <typename T>
int reduce_impl(pf_solver *s, TipResult *res, FrameState *fr) {
  ReduceArgs<T> a;
  a.psi = field<T>(s, s->L.psi[s->cur]);
  a.U = field<T>(s, s->L.U[s->cur]);
  a.nx = s->p.nx; a.ny = s->p.ny; a.nz = s->p.dim == 3 ? s->p.nz : 1;
  a.hd = s->p.h;
  a.rows = 0;  // set by the launcher
  a.frame = reinterpret_cast<const FrameState *>(s->ws + s->L.frame[s->fcur]);
  a.pending = 0;
  a.red = Reduce{reinterpret_cast<TipAcc *>(s->ws + s->L.partials),
                 reinterpret_cast<TipResult *>(s->ws + s->L.result)};
  PF_HIP(launch_reduce<T>(a, s->stream));
  // the result record carries a copy of the frame record the reduction read
  PF_HIP(hipMemcpyAsync(res, a.red.result, sizeof(TipResult), hipMemcpyDeviceToHost, s->stream));
  PF_HIP(hipStreamSynchronize(s->stream));
  *fr = res->frame;
  return PF_OK;
}

template <typename T>
int read_impl(pf_solver *s, double *phi, double *U, double *psi) {
  const pf_params &p = s->p;
  const size_t n = s->n;
  FrameState fr;
  PF_HIP(hipStreamSynchronize(s->stream));
  PF_HIP(hipMemcpy(&fr, s->ws + s->L.frame[s->fcur], sizeof(fr), hipMemcpyDeviceToHost));
  std::vector<T> hp(n), hu(n);
  PF_HIP(hipMemcpy(hp.data(), field<T>(s, s->L.psi[s->cur]), n * sizeof(T), hipMemcpyDeviceToHost));
  PF_HIP(hipMemcpy(hu.data(), field<T>(s, s->L.U[s->cur]), n * sizeof(T), hipMemcpyDeviceToHost));
  const int nx = p.nx, ny = p.ny, nz = p.dim == 3 ? p.nz : 1;
  for (int l = 0; l < nz; ++l)
    for (int j = 0; j < ny; ++j) {
      int jp = fr.pending ? std::min(j + 1, ny - 1) : j;
      size_t dst = ((size_t)l * ny + j) * nx, src = ((size_t)l * ny + jp) * nx;
      for (int i = 0; i < nx; ++i) {
        double vp = (double)hp[src + i];
        if (psi) psi[dst + i] = vp;
        if (phi) phi[dst + i] = tanh(vp / sqrt(2.0));
        if (U) U[dst + i] = (double)hu[src + i];
      }
    }
  return PF_OK;
}

}  // namespace

struct pf_batch {
  std::vector<pf_solver *> s;
  int precision;
  bool frozen, frame, multi;
  hipStream_t stream;
  void *table;  // device BatchSolve2D<T>[n]
  int2 *map;    // device workgroup map
  int blocks;
  std::vector<long long> expect;  // solver steps the device table assumes
  std::vector<int> seg;           // segment lengths the table was built with
  int graph_steps;
  int seg_fixed;  // > 0: rows per segment of every member (pf_batch_autotune)
  hipStream_t cap;
  hipGraph_t graph;
  hipGraphExec_t gexec;
};

namespace {

int xcd_remap_host(int b, int nb) {
  const int X = 8;
  int q = nb / X, r = nb % X, x = b % X;
  return x * q + (x < r ? x : r) + b / X;
}

// (Re)build the device table and workgroup map from the solvers' state.
template <typename T>
int batch_build(pf_batch *b) {
  const int n = (int)b->s.size();
  std::vector<BatchSolve2D<T>> tab(n);
  std::vector<int2> list;
  for (int i = 0; i < n; ++i) {
    pf_solver *s = b->s[i];
    BatchSolve2D<T> &e = tab[i];
    memset(&e, 0, sizeof(e));
    Geom2D g = fill2d<T>(s, e.a, kMinSegBatch2D, b->seg_fixed);
    for (int k = 0; k < 2; ++k) {
      e.psi[k] = field<T>(s, s->L.psi[k]);
      e.U[k] = field<T>(s, s->L.U[k]);
    }
    for (int k = 0; k < 3; ++k) e.frames[k] = reinterpret_cast<FrameState *>(s->ws + s->L.frame[k]);
    e.n0 = s->step;
    e.par0 = s->cur;
    e.f0 = s->fcur;
    for (int lb = 0; lb < g.blocks; ++lb) list.push_back(int2{i, lb});
    b->expect[i] = s->step;
    b->seg[i] = s->seg;
  }
  const int total = (int)list.size();
  std::vector<int2> map(total);
  for (int k = 0; k < total; ++k) map[k] = list[xcd_remap_host(k, total)];
  PF_HIP(hipStreamSynchronize(b->stream));
  if (b->table) (void)hipFree(b->table);
  if (b->map) (void)hipFree(b->map);
  b->table = nullptr;
  b->map = nullptr;
  PF_HIP(hipMalloc(&b->table, sizeof(BatchSolve2D<T>) * n));
  PF_HIP(hipMalloc((void **)&b->map, sizeof(int2) * total));
  PF_HIP(hipMemcpy(b->table, tab.data(), sizeof(BatchSolve2D<T>) * n, hipMemcpyHostToDevice));
  PF_HIP(hipMemcpy(b->map, map.data(), sizeof(int2) * total, hipMemcpyHostToDevice));
  b->blocks = total;
  return PF_OK;
}

void batch_drop_graph(pf_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

template <typename T>
int batch_capture(pf_batch *b) {
  batch_drop_graph(b);
  if (b->graph_steps <= 0) return PF_OK;
  auto *tab = reinterpret_cast<BatchSolve2D<T> *>(b->table);
  PF_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  for (int k = 0; k < b->graph_steps; ++k)
    (void)launch_batch2d<T>(tab, b->map, b->blocks, k, b->frozen, b->frame, b->multi, b->cap);
  (void)launch_batch2d_advance<T>(tab, (int)b->s.size(), b->graph_steps, b->frame, b->cap);
  PF_HIP(hipStreamEndCapture(b->cap, &b->graph));
  PF_HIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
  return PF_OK;
}

template <typename T>
int batch_step(pf_batch *b, long long nsteps) {
  bool stale = false;
  for (size_t i = 0; i < b->s.size(); ++i)
    if (b->s[i]->step != b->expect[i] || b->s[i]->seg != b->seg[i]) stale = true;
  if (stale) {
    int rc = batch_build<T>(b);
    if (rc != PF_OK) return rc;
    rc = batch_capture<T>(b);
    if (rc != PF_OK) return rc;
  }
  auto *tab = reinterpret_cast<BatchSolve2D<T> *>(b->table);
  long long done = 0;
  if (b->gexec) {
    for (; done + b->graph_steps <= nsteps; done += b->graph_steps)
      PF_HIP(hipGraphLaunch(b->gexec, b->stream));
  }
  const int rem = (int)(nsteps - done);
  if (rem > 0) {
    for (int k = 0; k < rem; ++k)
      PF_HIP(launch_batch2d<T>(tab, b->map, b->blocks, k, b->frozen, b->frame, b->multi,
                               b->stream));
    PF_HIP(launch_batch2d_advance<T>(tab, (int)b->s.size(), rem, b->frame, b->stream));
  }
  for (size_t i = 0; i < b->s.size(); ++i) {
    pf_solver *s = b->s[i];
    s->step += nsteps;
    s->cur = (int)((s->cur + nsteps) & 1);
    if (b->frame) s->fcur = (int)((s->fcur + nsteps) % 3);
    b->expect[i] = s->step;
  }
  return PF_OK;
}

}  // namespace

namespace {

// Seconds of `steps` steps of `run` on `st` (after 2 warm-up steps), or a
// negative value when a HIP call failed.
template <typename F>
double time_steps(hipStream_t st, int steps, F run) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double out = -1.0;
  float ms = 0.f;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess && run(2) == PF_OK &&
      hipEventRecord(e0, st) == hipSuccess && run(steps) == PF_OK &&
      hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
      hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
    out = ms * 1e-3;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return out;
}

// Longest trial a caller may ask for: the confirming passes run four times as
// many steps, which must stay within an int.
constexpr int kMaxTrialSteps = 1 << 20;

// Index of the fastest of n candidates timed by trial(i, m) (seconds of m
// times the trial's base step count, negative on failure; -1 returned then).
// Candidate 0 is the geometry in use: each candidate is timed in two
// interleaved passes and keeps its better time.  A candidate more than 3%
// faster than candidate 0 is then confirmed against it in three interleaved
// passes four times as long, and replaces it only when it is still more than
// 2% faster there: a short trial can misjudge near-equal geometries, and the
// choice should not flip from run to run on timing noise.
template <typename F>
int pick_fastest(int n, F trial) {
  std::vector<double> best(n, 1e300);
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < n; ++i) {
      double sec = trial(i, 1);
      if (sec < 0.0) return -1;
      best[i] = std::min(best[i], sec);
    }
  int k = 0;
  for (int i = 1; i < n; ++i)
    if (best[i] < best[k]) k = i;
  if (!(best[k] < 0.97 * best[0])) return 0;
  double b0 = 1e300, bk = 1e300;
  for (int pass = 0; pass < 3; ++pass) {
    const double s0 = trial(0, 4), sk = trial(k, 4);
    if (s0 < 0.0 || sk < 0.0) return -1;
    b0 = std::min(b0, s0);
    bk = std::min(bk, sk);
  }
  return bk < 0.98 * b0 ? k : 0;
}

// A copy of solver s whose workspace is a fresh device copy of s's (the
// caller frees clone.ws).  Stepping the copy leaves s untouched.
int clone_solver(pf_solver *s, pf_solver &clone) {
  void *d = nullptr;
  PF_HIP(hipStreamSynchronize(s->stream));
  if (hipMalloc(&d, s->L.total) != hipSuccess)
    return fail(PF_ERR_OOM, "autotune scratch allocation of " + std::to_string(s->L.total) +
                                " bytes failed");
  if (hipMemcpy(d, s->ws, s->L.total, hipMemcpyDeviceToDevice) != hipSuccess) {
    (void)hipFree(d);
    return fail(PF_ERR_DEVICE, "autotune scratch copy failed");
  }
  clone = *s;
  clone.ws = reinterpret_cast<char *>(d);
  clone.ws_bytes = s->L.total;
  clone.own = false;
  return PF_OK;
}

template <typename T>
int autotune_impl(pf_solver *s, int steps) {
  pf_solver t;
  int rc = clone_solver(s, t);
  if (rc != PF_OK) return rc;
  // (rows per segment, z rows per workgroup); the geometry in use first
  std::vector<std::pair<int, int>> cand = {{s->seg, s->ztile}};
  auto add = [&](int seg, int zt) {
    if (seg != s->seg || zt != s->ztile) cand.push_back({seg, zt});
  };
  if (s->p.dim == 2) {
    // waves per SIMD; counts that give the same segments as one already
    // listed are skipped
    std::vector<int> nsegs = {geom2d(s->p.nx, s->p.ny, s->seg, s->ncu).nsegs};
    for (int k : {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32}) {
      const int n = geom2d(s->p.nx, s->p.ny, -k, s->ncu).nsegs;
      if (std::find(nsegs.begin(), nsegs.end(), n) != nsegs.end()) continue;
      nsegs.push_back(n);
      add(-k, s->ztile);
    }
  } else {
    // rows per segment, each candidate kept only when it gives a segment
    // count not listed yet for its z rows (the rows are split evenly)
    const int zmax = s->p.precision == PF_F64 ? 6 : 14;
    for (int zt : {1, 2, 4, 6, 8, 10, 12, 14}) {
      std::vector<int> seen;
      if (zt == s->ztile) seen.push_back(geom3d(s->p.nx, s->p.ny, s->p.nz, s->seg, zt).nsegs);
      for (int seg : {8, 12, 16, 24, 32, 43, 64, 86, 128, 256}) {
        if (zt > zmax || zt > s->p.nz || seg > std::max(8, s->p.ny) ||
            step3d_lds_bytes(s->p.nx, zt, sizeof(T)) > kMaxLds3D)
          continue;
        const int ns = geom3d(s->p.nx, s->p.ny, s->p.nz, seg, zt).nsegs;
        if (std::find(seen.begin(), seen.end(), ns) != seen.end()) continue;
        seen.push_back(ns);
        add(seg, zt);
      }
    }
  }
  const int k = pick_fastest((int)cand.size(), [&](int i, int m) {
    t.seg = cand[i].first;
    t.ztile = cand[i].second;
    return time_steps(s->stream, steps * m, [&](int n) { return step_impl<T>(&t, n); });
  });
  (void)hipStreamSynchronize(s->stream);
  (void)hipFree(t.ws);
  if (k < 0) return fail(PF_ERR_DEVICE, "autotune trial failed");
  s->seg = cand[k].first;
  s->ztile = cand[k].second;
  return PF_OK;
}

template <typename T>
int batch_autotune_impl(pf_batch *b, int steps) {
  PF_HIP(hipStreamSynchronize(b->stream));
  const int n = (int)b->s.size();
  std::vector<pf_solver> clones(n);
  int made = 0, rc = PF_OK;
  for (; made < n && rc == PF_OK; ++made) rc = clone_solver(b->s[made], clones[made]);
  if (rc != PF_OK) --made;
  pf_batch tb;
  tb.precision = b->precision;
  tb.frozen = b->frozen;
  tb.frame = b->frame;
  tb.multi = b->multi;
  tb.stream = b->stream;
  tb.table = nullptr;
  tb.map = nullptr;
  tb.graph_steps = 0;
  tb.cap = nullptr;
  tb.graph = nullptr;
  tb.gexec = nullptr;
  for (int i = 0; i < made; ++i) tb.s.push_back(&clones[i]);
  tb.expect.assign(made, -1);
  tb.seg.assign(made, 0);
  // candidate 0: the segment length in use (0 = each member's own)
  std::vector<int> cand = {b->seg_fixed};
  for (int seg : {4, 6, 8, 12, 16, 24, 32})
    if (seg != b->seg_fixed) cand.push_back(seg);
  int bseg = b->seg_fixed;
  if (rc == PF_OK) {
    const int k = pick_fastest((int)cand.size(), [&](int i, int mult) {
      tb.seg_fixed = cand[i];
      tb.expect.assign(made, -1);  // rebuild with this segment length
      return time_steps(b->stream, steps * mult, [&](int m) { return batch_step<T>(&tb, m); });
    });
    if (k < 0)
      rc = fail(PF_ERR_DEVICE, "batch autotune trial failed");
    else
      bseg = cand[k];
  }
  (void)hipStreamSynchronize(b->stream);
  if (tb.table) (void)hipFree(tb.table);
  if (tb.map) (void)hipFree(tb.map);
  for (int i = 0; i < made; ++i) (void)hipFree(clones[i].ws);
  if (rc != PF_OK) return rc;
  b->seg_fixed = bseg;
  rc = batch_build<T>(b);
  if (rc != PF_OK) return rc;
  return batch_capture<T>(b);
}

}  // namespace

extern "C" {

int pf_batch_create(pf_solver *const *solvers, int32_t n, pf_batch **out) {
  if (!solvers || n < 1 || !out) return fail(PF_ERR_ARG, "need n >= 1 solvers and an out pointer");
  for (int i = 0; i < n; ++i)
    if (!solvers[i]) return fail(PF_ERR_ARG, "solver is NULL");
  const pf_solver *s0 = solvers[0];
  for (int i = 0; i < n; ++i) {
    const pf_solver *s = solvers[i];
    if (s->p.dim != 2) return fail(PF_ERR_ARG, "batched stepping is 2D only");
    if (s->p.antitrapping != PF_AT_APPROX || s->p.divergence != PF_DIV_SHELLS)
      return fail(PF_ERR_ARG, "batched stepping runs the approximated current on shell divergences");
    if (s->p.dynamic_grains) return fail(PF_ERR_ARG, "batched stepping takes static grain maps");
    if (s->p.precision != s0->p.precision) return fail(PF_ERR_ARG, "mixed precisions in a batch");
    if ((s->p.lT > 0.0) != (s0->p.lT > 0.0) || (s->p.frame != 0) != (s0->p.frame != 0) ||
        (s->p.n_grains > 1) != (s0->p.n_grains > 1))
      return fail(PF_ERR_ARG, "a batch needs one kind: all frozen or all isothermal, all with or "
                              "without frame, all single- or all multi-grain");
    if (s->stream != s0->stream) return fail(PF_ERR_ARG, "solvers of a batch share one stream");
    for (int j = 0; j < i; ++j)
      if (solvers[j] == s) return fail(PF_ERR_ARG, "a solver appears twice in the batch");
  }
  pf_batch *b = new (std::nothrow) pf_batch();
  if (!b) return fail(PF_ERR_OOM, "host allocation failed");
  b->s.assign(solvers, solvers + n);
  b->precision = s0->p.precision;
  b->frozen = s0->p.lT > 0.0;
  b->frame = s0->p.frame != 0;
  b->multi = s0->p.n_grains > 1;
  b->stream = s0->stream;
  b->table = nullptr;
  b->map = nullptr;
  b->expect.assign(n, -1);
  b->seg.assign(n, 0);
  b->graph_steps = 0;
  b->seg_fixed = 0;
  b->graph = nullptr;
  b->gexec = nullptr;
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(PF_ERR_DEVICE, "capture stream creation failed");
  }
  int rc = b->precision == PF_F64 ? batch_build<double>(b) : batch_build<float>(b);
  if (rc != PF_OK) {
    pf_batch_destroy(b);
    return rc;
  }
  *out = b;
  return PF_OK;
}

int pf_batch_step(pf_batch *b, int64_t nsteps) {
  if (!b) return fail(PF_ERR_ARG, "batch is NULL");
  if (nsteps < 0) return fail(PF_ERR_ARG, "nsteps must be >= 0");
  return b->precision == PF_F64 ? batch_step<double>(b, nsteps) : batch_step<float>(b, nsteps);
}

int pf_batch_use_graph(pf_batch *b, int32_t steps_per_graph) {
  if (!b) return fail(PF_ERR_ARG, "batch is NULL");
  if (steps_per_graph < 0) return fail(PF_ERR_ARG, "steps_per_graph must be >= 0");
  if (steps_per_graph > 0 && steps_per_graph % (b->frame ? 6 : 2) != 0)
    return fail(PF_ERR_ARG, "steps_per_graph must be a multiple of 2 (6 with the moving frame)");
  b->graph_steps = steps_per_graph;
  PF_HIP(hipStreamSynchronize(b->stream));
  int rc = b->precision == PF_F64 ? batch_build<double>(b) : batch_build<float>(b);
  if (rc != PF_OK) return rc;
  return b->precision == PF_F64 ? batch_capture<double>(b) : batch_capture<float>(b);
}

void pf_batch_destroy(pf_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  batch_drop_graph(b);
  if (b->table) (void)hipFree(b->table);
  if (b->map) (void)hipFree(b->map);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

int pf_autotune(pf_solver *s, int32_t steps_per_trial, int32_t *seg, int32_t *ztile) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  if (steps_per_trial < 1 || steps_per_trial > kMaxTrialSteps)
    return fail(PF_ERR_ARG, "steps_per_trial must be in [1, 2^20]");
  int rc = s->p.precision == PF_F64 ? autotune_impl<double>(s, steps_per_trial)
                                    : autotune_impl<float>(s, steps_per_trial);
  if (rc != PF_OK) return rc;
  if (seg) *seg = s->seg;
  if (ztile) *ztile = s->p.dim == 3 ? s->ztile : 1;
  return PF_OK;
}

int pf_batch_autotune(pf_batch *b, int32_t steps_per_trial, int32_t *seg) {
  if (!b) return fail(PF_ERR_ARG, "batch is NULL");
  if (steps_per_trial < 1 || steps_per_trial > kMaxTrialSteps)
    return fail(PF_ERR_ARG, "steps_per_trial must be in [1, 2^20]");
  int rc = b->precision == PF_F64 ? batch_autotune_impl<double>(b, steps_per_trial)
                                  : batch_autotune_impl<float>(b, steps_per_trial);
  if (rc != PF_OK) return rc;
  if (seg) *seg = b->seg_fixed;
  return PF_OK;
}

int pf_version(void) { return PF_VERSION; }

const char *pf_last_error(void) { return g_err.c_str(); }

double pf_stable_dt(const pf_params *p) {
  if (validate(p) != PF_OK) return -1.0;
  return stable_dt_for(p, f1_min(p));
}

size_t pf_workspace_bytes(const pf_params *p) {
  if (validate(p) != PF_OK) return 0;
  return layout_of(p).total;
}

int pf_create(const pf_params *p, const pf_init *init, void *workspace, size_t workspace_bytes,
              void *stream, pf_solver **out) {
  int rc = validate(p);
  if (rc != PF_OK) return rc;
  if (!init || !init->psi || !init->U) return fail(PF_ERR_ARG, "init arrays are NULL");
  if (!out) return fail(PF_ERR_ARG, "out is NULL");
  const size_t n = cells(p);
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(init->psi[i]) || !isfinite(init->U[i]))
      return fail(PF_ERR_NONFINITE, "initial psi or U holds NaN or Inf");
  if (init->grain) {
    for (size_t i = 0; i < n; ++i)
      if (init->grain[i] < 0 || init->grain[i] >= p->n_grains)
        return fail(PF_ERR_ARG, "grain index outside [0, n_grains)");
    if (p->frame && !p->dynamic_grains) {  // a static map does not shift with the frame
      const int nx = p->nx, ny = p->ny, nz = p->dim == 3 ? p->nz : 1;
      for (int l = 0; l < nz; ++l)
        for (int j = 1; j < ny; ++j)
          for (int i = 0; i < nx; ++i)
            if (init->grain[((size_t)l * ny + j) * nx + i] != init->grain[(size_t)l * ny * nx + i])
              return fail(PF_ERR_ARG, "with the moving frame the grain map must not vary along y");
    }
  }
  double lambda = p->lambda > 0.0 ? p->lambda : p->D / kA2;
  double dtmax = pf_stable_dt(p);
  double dt = p->dt > 0.0 ? p->dt : 0.8 * dtmax;
  if (dt > dtmax * (1.0 + 1e-12))
    return fail(PF_ERR_UNSTABLE_DT, "dt = " + std::to_string(dt) + " exceeds the stability limit " +
                                        std::to_string(dtmax));
  Layout L = layout_of(p);
  pf_solver *s = new (std::nothrow) pf_solver();
  if (!s) return fail(PF_ERR_OOM, "host allocation failed");
  s->p = *p;
  s->rot.assign(p->grain_rot, p->grain_rot + 9 * p->n_grains);
  s->p.grain_rot = s->rot.data();
  weights_of(p, s->w);
  s->lambda = lambda;
  s->dt = dt;
  s->n = n;
  s->stream = reinterpret_cast<hipStream_t>(stream);
  s->L = L;
  s->cur = 0;
  s->fcur = 0;
  s->step = 0;
  s->have_prev = false;
  if (workspace) {
    if (workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
      delete s;
      return fail(PF_ERR_OOM, "workspace smaller than pf_workspace_bytes() or not 256-byte aligned");
    }
    s->ws = reinterpret_cast<char *>(workspace);
    s->ws_bytes = workspace_bytes;
    s->own = false;
  } else {
    void *d = nullptr;
    if (hipMalloc(&d, L.total) != hipSuccess) {
      delete s;
      return fail(PF_ERR_OOM, "hipMalloc of " + std::to_string(L.total) + " bytes failed");
    }
    s->ws = reinterpret_cast<char *>(d);
    s->ws_bytes = L.total;
    s->own = true;
  }
  int r2 = PF_OK;
  {
    int dev = 0;
    s->ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&s->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        s->ncu < 1)
      r2 = fail(PF_ERR_DEVICE, "cannot read the device's compute unit count");
  }
  if (p->dim == 2) {
    s->seg = default_seg2d(p->nx, p->ny, p->precision, s->ncu);
    s->ztile = 1;
  } else {
    std::tie(s->seg, s->ztile) = default_geom3d(p, s->ncu);
  }
  if (r2 == PF_OK)
    r2 = p->precision == PF_F64 ? upload<double>(s, init) : upload<float>(s, init);
  if (r2 == PF_OK && p->n_grains > 1) {
    std::vector<int8_t> g(n, 0);
    if (init->grain) memcpy(g.data(), init->grain, n);
    if (hipMemcpy(s->ws + L.grain, g.data(), n, hipMemcpyHostToDevice) != hipSuccess)
      r2 = fail(PF_ERR_DEVICE, "grain upload failed");
  }
  if (r2 == PF_OK) {
    FrameState z{0, 0, 0};
    if (hipMemcpy(s->ws + L.frame[0], &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->ws + L.frame[1], &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->ws + L.frame[2], &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess)
      r2 = fail(PF_ERR_DEVICE, "state initialisation failed");
  }
  if (r2 != PF_OK) {
    if (s->own) (void)hipFree(s->ws);
    delete s;
    return r2;
  }
  *out = s;
  return PF_OK;
}

int pf_step(pf_solver *s, int64_t nsteps) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  if (nsteps < 0) return fail(PF_ERR_ARG, "nsteps must be >= 0");
  return s->p.precision == PF_F64 ? step_impl<double>(s, nsteps) : step_impl<float>(s, nsteps);
}

int pf_step_diffusion(pf_solver *s, int64_t nsteps) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  if (nsteps < 0) return fail(PF_ERR_ARG, "nsteps must be >= 0");
  if (s->p.dim != 2) return fail(PF_ERR_ARG, "the diffusion-only step is 2D only");
  if (s->p.divergence != PF_DIV_SHELLS)
    return fail(PF_ERR_ARG, "the diffusion-only step uses the shell divergence");
  return s->p.precision == PF_F64 ? step_impl<double>(s, nsteps, true)
                                  : step_impl<float>(s, nsteps, true);
}

int pf_synchronize(pf_solver *s) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  PF_HIP(hipStreamSynchronize(s->stream));
  return PF_OK;
}

int pf_read_fields(pf_solver *s, double *phi, double *U, double *psi, int8_t *grain) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  int rc = s->p.precision == PF_F64 ? read_impl<double>(s, phi, U, psi)
                                    : read_impl<float>(s, phi, U, psi);
  if (rc != PF_OK) return rc;
  if (grain) {
    if (s->p.dynamic_grains) {
      // the current level's map, with the frame shift it may still owe
      FrameState fr;
      PF_HIP(hipMemcpy(&fr, s->ws + s->L.frame[s->fcur], sizeof(fr), hipMemcpyDeviceToHost));
      std::vector<int8_t> hg(s->n);
      PF_HIP(hipMemcpy(hg.data(), grain_buf(s, s->cur), s->n, hipMemcpyDeviceToHost));
      const int nx = s->p.nx, ny = s->p.ny, nz = s->p.dim == 3 ? s->p.nz : 1;
      for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j) {
          int jp = (s->p.frame && fr.pending) ? std::min(j + 1, ny - 1) : j;
          memcpy(grain + ((size_t)l * ny + j) * nx, hg.data() + ((size_t)l * ny + jp) * nx, nx);
        }
    } else if (s->p.n_grains > 1) {
      PF_HIP(hipMemcpy(grain, s->ws + s->L.grain, s->n, hipMemcpyDeviceToHost));
    } else {
      memset(grain, 0, s->n);
    }
  }
  return PF_OK;
}

int pf_tip_state(pf_solver *s, pf_tip *out) {
  if (!s || !out) return fail(PF_ERR_ARG, "solver or out is NULL");
  TipResult r;
  FrameState fr;
  int rc = s->p.precision == PF_F64 ? reduce_impl<double>(s, &r, &fr)
                                    : reduce_impl<float>(s, &r, &fr);
  if (rc != PF_OK) return rc;
  const pf_params &p = s->p;
  pf_tip t;
  memset(&t, 0, sizeof(t));
  t.step = s->step;
  t.t = (double)s->step * s->dt;
  t.found = r.found;
  t.nonfinite = r.bad ? 1 : 0;
  t.frame_shift = fr.base + fr.pending;
  t.solid_fraction = r.fs_sum / (double)s->n;
  if (r.found) {
    const long long nx = p.nx, ny = p.ny;
    t.index = r.idx;
    t.x = (double)(r.idx % nx) * p.h;
    t.z = p.dim == 3 ? (double)(r.idx / (nx * ny)) * p.h : 0.0;
    t.y_frame = r.y;
    t.y_lab = r.y + (double)t.frame_shift * p.h;
    if (s->have_prev && t.t > s->prev_t) t.velocity = (t.y_lab - s->prev_y) / (t.t - s->prev_t);
    s->have_prev = true;
    s->prev_t = t.t;
    s->prev_y = t.y_lab;
  } else {
    t.index = -1;
  }
  *out = t;
  if (r.bad) return fail(PF_ERR_NONFINITE, "state holds NaN or Inf values");
  if (p.lT > 0.0) {
    // the thermal coordinate has moved with the frame shift and the clock:
    // F1 must stay positive and dt within the limit it sets
    const double f1 = f1_min_at(&p, (double)t.frame_shift * p.h - p.y0 - p.Vp * t.t);
    if (!(f1 > 0.0))
      return fail(PF_ERR_UNSTABLE_DT, "F1 = 1 - (1-k) zeta / lT is no longer positive over the "
                                      "lattice (frame shift " + std::to_string(t.frame_shift) +
                                      ", t = " + std::to_string(t.t) + ")");
    const double dtmax = stable_dt_for(&p, f1);
    if (s->dt > dtmax * (1.0 + 1e-12))
      return fail(PF_ERR_UNSTABLE_DT, "dt = " + std::to_string(s->dt) +
                                          " now exceeds the stability limit " +
                                          std::to_string(dtmax) + " (F1 min " +
                                          std::to_string(f1) + ")");
  }
  return PF_OK;
}

int pf_device_fields(pf_solver *s, void **psi, void **U) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  if (psi) *psi = s->ws + s->L.psi[s->cur];
  if (U) *U = s->ws + s->L.U[s->cur];
  return PF_OK;
}

int pf_frame_state(pf_solver *s, int64_t *shift, int32_t *pending) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  FrameState fr;
  PF_HIP(hipStreamSynchronize(s->stream));
  PF_HIP(hipMemcpy(&fr, s->ws + s->L.frame[s->fcur], sizeof(fr), hipMemcpyDeviceToHost));
  if (shift) *shift = fr.base + fr.pending;
  if (pending) *pending = fr.pending;
  return PF_OK;
}

int pf_tune(pf_solver *s, int32_t rows_per_segment, int32_t z_tile) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  if (s->p.dim == 2 && rows_per_segment >= -64 && rows_per_segment <= -1) {
    s->seg = rows_per_segment;  // -k: k waves per SIMD
    return PF_OK;
  }
  if (rows_per_segment < 4 || rows_per_segment > 256)
    return fail(PF_ERR_ARG, s->p.dim == 2 ? "rows_per_segment must lie in [4, 256] or [-64, -1]"
                                          : "rows_per_segment must lie in [4, 256]");
  if (s->p.dim == 3 && (z_tile < 1 || z_tile > 14))
    return fail(PF_ERR_ARG, "z_tile must lie in [1, 14]");
  if (s->p.dim == 3 && s->p.precision == PF_F64 && z_tile > 6)
    return fail(PF_ERR_ARG, "FP64 3D workgroups hold at most 6 z rows (8 waves)");
  if (s->p.dim == 3 &&
      step3d_lds_bytes(s->p.nx, z_tile, s->p.precision == PF_F64 ? 8 : 4) > kMaxLds3D)
    return fail(PF_ERR_ARG, "z_tile too large for the LDS of one workgroup at this precision");
  s->seg = rows_per_segment;
  if (s->p.dim == 3) s->ztile = z_tile;
  return PF_OK;
}

int pf_geometry(pf_solver *s, int32_t *rows_per_segment, int32_t *z_tile) {
  if (!s) return fail(PF_ERR_ARG, "solver is NULL");
  if (rows_per_segment) *rows_per_segment = s->seg;
  if (z_tile) *z_tile = s->p.dim == 3 ? s->ztile : 1;
  return PF_OK;
}

void pf_destroy(pf_solver *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->own) (void)hipFree(s->ws);
  delete s;
}

}  // extern "C"
