// step3d.hip -- fused psi/U explicit step on the 3D cubic lattice (gfx950).
//
// One launch advances psi and U by one explicit Euler step (Sec. 4.3.1 and
// 6.2.1) with the three-shell operators of Sec. 5 and App. A:
//   L = w1 L_{1,0,0} + w2 L_{0,1,0} + w3 L_{0,0,1}  (Eqs. 3D_L100, 3D_L110,
//       3D_L111), G likewise (Eqs. Grad_100, Grad_110, Grad_111, with the
//       <111> prefactor 1/(16 h^2) that reproduces the printed symbol), and the
//       divergence D_{s1,s2,s3} of Eqs. divergence_100, divergence_110,
//       divergence_111 with their averaged alpha on each flux;
//   the cubic anisotropy a_s = 1 - 3 eps4 + 4 eps4 sum n'^4, n' = R_g^T n, per
//       grain g, whose eps4-linear terms use the standard <100> face fluxes;
//   frozen temperature along y (Eqs. Thermal_F1, Thermal_F2);
//   U with D~ div[(1 - phi) grad U] + div[alpha_A grad psi] + sqrt2 alpha_A
//       (Eq. PF_b with the approximated anti-trapping current, Eq. Anti_approx).
// Default weights (1/3, 2/3, 0) give the isotropic S-bar_{1,2,0} scheme.
//
// Schedule.  A workgroup owns 60 x-columns (wave64 lanes, 2-column halo on
// each side), `ztile` output z-rows and a segment of `seg` y-rows.  It runs
// ztile + 2 waves, one per z-row including a ring row on each side (the ring
// waves also load the outer psi halo rows), which march up the segment in
// lock-step.  Each iteration publishes the newest psi, U, phi row in LDS rings
// of 5 rows, then (barrier) computes the psi rate of the row below from the
// LDS 3x3x3 neighbourhood and publishes alpha_A, then (barrier) the output
// waves update U two rows below from the 3x3x3 neighbourhoods of alpha_D =
// 1 - phi, alpha_A, U and psi.  No-flux walls: psi, U and phi are read through
// the mirror map, alpha_A of a mirrored cell is replaced by its image.
#include <type_traits>

#include "pf_device.hpp"

namespace pf {

namespace {

constexpr float kGradEps3 = 1e-12f;

template <typename T>
struct Rot3 {
  T m[9];  // row-major crystal -> lab
};

// a_s and, optionally, one lab component of J = a^2 g + |g|^2 a da/dg
// (J = R [g'(a^2 - 16 eps4 a s4) + 16 eps4 a g'^3/|g|^2], g' = R^T g).
template <typename T, int comp>
__device__ __forceinline__ T aniso3(T gx, T gy, T gz, const Rot3<T> &R, const Coef<T> &c) {
  T g2 = gx * gx + gy * gy + gz * gz;
  T r2 = Math<T>::rcp(g2 > T(kGradEps3) ? g2 : T(kGradEps3));
  T c0 = R.m[0] * gx + R.m[3] * gy + R.m[6] * gz;
  T c1 = R.m[1] * gx + R.m[4] * gy + R.m[7] * gz;
  T c2 = R.m[2] * gx + R.m[5] * gy + R.m[8] * gz;
  T q0 = c0 * c0, q1 = c1 * c1, q2 = c2 * c2;
  T s4 = (q0 * q0 + q1 * q1 + q2 * q2) * (r2 * r2);
  T a = c.an0 + c.an4 * s4;
  if constexpr (comp < 0) {
    return g2 > T(kGradEps3) ? a : T(1);
  } else {
    T t = c.an16 * a;
    T base = a * a - t * s4;
    T tr = t * r2;
    T j0 = c0 * (base + tr * q0);
    T j1 = c1 * (base + tr * q1);
    T j2 = c2 * (base + tr * q2);
    T j = R.m[3 * comp + 0] * j0 + R.m[3 * comp + 1] * j1 + R.m[3 * comp + 2] * j2;
    T plain = comp == 0 ? gx : (comp == 1 ? gy : gz);
    return g2 > T(kGradEps3) ? j : plain;
  }
}

__device__ __forceinline__ int xcd_remap3(int b, int nb) {
  const int X = 8;
  int q = nb / X, r = nb % X, x = b % X;
  return x * q + (x < r ? x : r) + b / X;
}

// index into a 3x3x3 neighbourhood, offsets in {-1, 0, 1}
__host__ __device__ constexpr int nb(int dx, int dy, int dz) {
  return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
}

constexpr int kRS = 66;  // LDS row stride: lane l at l + 1, pads at 0 and 65

// Generalised divergence sum_links abar (beta_d - beta_0) over the three
// shells for one cell, from its 3x3x3 alpha and beta neighbourhoods; returns
// cD1 S100 + cD2 S110 + cD3 S111.
template <typename T, bool kShell3>
__device__ __forceinline__ T divergence27(const T (&A)[27], const T (&B)[27], const Coef<T> &c) {
  const T b0 = B[nb(0, 0, 0)];
  // <100>: abar = 1/4 (alpha_0 + alpha_d) + 1/16 sum over the 4 tangential
  // offsets t of (alpha_t + alpha_{d+t})
  T s100 = T(0);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
      int d[3] = {0, 0, 0};
      d[ax] = sg;
      T near = A[nb(0, 0, 0)] + A[nb(d[0], d[1], d[2])];
      T far = T(0);
#pragma unroll
      for (int tx = 0; tx < 3; ++tx) {
        if (tx == ax) continue;
#pragma unroll
        for (int ts = -1; ts <= 1; ts += 2) {
          int t[3] = {0, 0, 0};
          t[tx] = ts;
          far += A[nb(t[0], t[1], t[2])] + A[nb(d[0] + t[0], d[1] + t[1], d[2] + t[2])];
        }
      }
      T abar = T(0.25) * near + T(0.0625) * far;
      s100 += abar * (B[nb(d[0], d[1], d[2])] - b0);
    }
  }
  // <110>: abar = 3/16 (in-plane plaquette) + 1/32 (the plaquettes above and
  // below along the third axis)
  T s110 = T(0);
#pragma unroll
  for (int a1 = 0; a1 < 3; ++a1) {
#pragma unroll
    for (int a2 = a1 + 1; a2 < 3; ++a2) {
      const int am = 3 - a1 - a2;
#pragma unroll
      for (int s1 = -1; s1 <= 1; s1 += 2) {
#pragma unroll
        for (int s2 = -1; s2 <= 1; s2 += 2) {
          int e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0}, d[3] = {0, 0, 0};
          e1[a1] = s1;
          e2[a2] = s2;
          d[a1] = s1;
          d[a2] = s2;
          T in = A[nb(0, 0, 0)] + A[nb(e1[0], e1[1], e1[2])] + A[nb(e2[0], e2[1], e2[2])] +
                 A[nb(d[0], d[1], d[2])];
          T out = T(0);
#pragma unroll
          for (int sm = -1; sm <= 1; sm += 2) {
            int m[3] = {0, 0, 0};
            m[am] = sm;
            out += A[nb(m[0], m[1], m[2])] + A[nb(e1[0] + m[0], e1[1] + m[1], e1[2] + m[2])] +
                   A[nb(e2[0] + m[0], e2[1] + m[1], e2[2] + m[2])] +
                   A[nb(d[0] + m[0], d[1] + m[1], d[2] + m[2])];
          }
          T abar = T(0.1875) * in + T(0.03125) * out;
          s110 += abar * (B[nb(d[0], d[1], d[2])] - b0);
        }
      }
    }
  }
  T res = c.cD1 * s100 + c.cD2 * s110;
  if constexpr (kShell3) {
    // <111>: abar = mean of the 8 corners of the cube spanned by 0 and d
    T s111 = T(0);
#pragma unroll
    for (int sx = -1; sx <= 1; sx += 2)
#pragma unroll
      for (int sy = -1; sy <= 1; sy += 2)
#pragma unroll
        for (int sz = -1; sz <= 1; sz += 2) {
          T cube = A[nb(0, 0, 0)] + A[nb(sx, 0, 0)] + A[nb(0, sy, 0)] + A[nb(0, 0, sz)] +
                   A[nb(sx, sy, 0)] + A[nb(sx, 0, sz)] + A[nb(0, sy, sz)] + A[nb(sx, sy, sz)];
          s111 += T(0.125) * cube * (B[nb(sx, sy, sz)] - b0);
        }
    res += c.cD3 * s111;
  }
  return res;
}

// FP32 workgroups run up to 10 waves (ztile <= 8); FP64 ones up to 4
// (ztile <= 2, bounded by LDS), which leaves them the whole register file.
template <typename T>
constexpr int max_threads3d() { return sizeof(T) == 8 ? 256 : 640; }

template <typename T, bool kFrozen, bool kReduce, bool kMulti, bool kShell3>
__global__ __launch_bounds__(max_threads3d<T>()) void step3d_kernel(Step3DArgs<T> a) {
  using M = Math<T>;
  const Coef<T> &c = a.c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int Z = a.ztile, NZR = Z + 4;
  const int SLOT = NZR * kRS;
  T *psiL = sm;              // 5 row slots each
  T *UL = psiL + 5 * SLOT;
  T *phL = UL + 5 * SLOT;
  T *aAL = phL + 5 * SLOT;

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lb = xcd_remap3((int)blockIdx.x, (int)gridDim.x);
  const int strip = lb % a.nstrips;
  const int rest = lb / a.nstrips;
  const int zt = rest % a.nzt;
  const int segi = rest / a.nzt;

  const int x = strip * a.wout - 2 + lane;
  const int gx = ghost(x, nx, a.bcx);
  const bool out_lane = lane >= 2 && lane < 2 + a.wout && x < nx;
  const int z0 = zt * Z;
  const int z = z0 - 1 + w;
  const int zi = w + 1;
  const bool out_wave = w >= 1 && w <= Z && z < nz;
  const bool ring = (w == 0) || (w == Z + 1);
  const int zh = (w == 0) ? z0 - 2 : z0 + Z + 1;
  const int zih = (w == 0) ? 0 : Z + 3;
  const size_t plane = (size_t)nx * (size_t)ny;
  const size_t pz = (size_t)ghost(z, nz, a.bcz) * plane + (size_t)gx;
  const size_t pzh = (size_t)ghost(zh, nz, a.bcz) * plane + (size_t)gx;
  const size_t pzd = (size_t)ghost(z - 1, nz, a.bcz) * plane + (size_t)gx;
  const int y0 = segi * a.seg;
  const int ye = min(y0 + a.seg, ny);

  const int pend = a.frame ? a.frame_in->pending : 0;
  const long long shift = a.frame ? a.frame_in->base + pend : 0;
  T off = T(0);
  if (kFrozen) off = (T)((double)shift * a.hd - a.y0 - a.Vp * ((double)a.step * a.dtd));
  const double ythr = (double)a.shift_row * a.hd;
  bool over = false;
  const T sq2 = T(1.4142135623730951);
  const T isq2 = T(0.70710678118654752);

  auto rowoff = [&](int r) -> size_t {
    int j = ghost_near(r, ny, a.bcy);
    if (pend) j = min(j + 1, ny - 1);
    return (size_t)j * (size_t)nx;
  };
  auto slot5 = [](int r) { return (r + 10) % 5; };
  auto rot_of = [&](int g) -> Rot3<T> {
    Rot3<T> R;
    const T *q = kMulti ? a.rot + 9 * g : a.R;
#pragma unroll
    for (int i = 0; i < 9; ++i) R.m[i] = q[i];
    return R;
  };
  // LDS element of field F at row slot s, z index zz, lane offset dx
  auto L = [&](const T *F, int s, int zz, int dx) -> T {
    return F[(s * NZR + zz) * kRS + lane + 1 + dx];
  };

  // z index of the neighbour below / above for the divergence: a mirrored
  // (no-flux) neighbour is the cell itself
  const int ziD = (a.bcz == PF_BC_NOFLUX && z == 0) ? zi : zi - 1;
  const int ziU = (a.bcz == PF_BC_NOFLUX && z == nz - 1) ? zi : zi + 1;

  // own-row window (rows r-2, r-1, r) and carries
  T pS = 0, pC = 0, pN = 0, uS = 0, uC = 0, uN = 0, fS = 0, fC = 0, fN = 0;
  T aAown[3] = {0, 0, 0};  // alpha_A of own cell at rows m-1, m (index by m mod 3)
  T FyS = 0;               // y face flux below row r-1
  int gC = 0, gN = 0;

  T nxt_p, nxt_u, nxt_h = 0;
  int nxt_g = 0;
  {
    size_t ro = rowoff(y0 - 2);
    nxt_p = a.psi_in[pz + ro];
    nxt_u = a.U_in[pz + ro];
    if (ring) nxt_h = a.psi_in[pzh + ro];
    if (kMulti) nxt_g = a.grain[pz + ro];
  }

  auto iter = [&](auto phase, int r) {
    constexpr int P = decltype(phase)::value;
    // ---------------- phase A: publish row r
    pS = pC; pC = pN; uS = uC; uC = uN; fS = fC; fC = fN; gC = gN;
    pN = nxt_p; uN = nxt_u; gN = nxt_g;
    const T hN = nxt_h;
    if (r + 1 <= ye + 1) {
      size_t ro = rowoff(r + 1);
      nxt_p = a.psi_in[pz + ro];
      nxt_u = a.U_in[pz + ro];
      if (ring) nxt_h = a.psi_in[pzh + ro];
      if (kMulti) nxt_g = a.grain[pz + ro];
    }
    fN = M::tanh_(pN * isq2);
    const int sN = slot5(r);
    {
      const int o = (sN * NZR + zi) * kRS + lane + 1;
      psiL[o] = pN;
      UL[o] = uN;
      phL[o] = fN;
      if (ring) psiL[(sN * NZR + zih) * kRS + lane + 1] = hN;
    }
    __syncthreads();
    if constexpr (P == 0) {
      __syncthreads();
      return;
    }
    const int m = r - 1;
    const int sm1 = slot5(m - 1), s0 = slot5(m), sp1 = slot5(m + 1);
    const T ih = c.inv_h, qh = T(0.25) * c.inv_h;

    if constexpr (P == 1) {
      // only the y face between rows m and m+1 (lower cell (x, m, z))
      T gyn = (L(psiL, sp1, zi, 0) - L(psiL, s0, zi, 0)) * ih;
      T gxt = (L(psiL, s0, zi, 1) + L(psiL, sp1, zi, 1) - L(psiL, s0, zi, -1) -
               L(psiL, sp1, zi, -1)) * qh;
      T gzt = (L(psiL, s0, zi + 1, 0) + L(psiL, sp1, zi + 1, 0) - L(psiL, s0, zi - 1, 0) -
               L(psiL, sp1, zi - 1, 0)) * qh;
      FyS = aniso3<T, 1>(gxt, gyn, gzt, rot_of(gC), c);
      __syncthreads();
      return;
    } else {
      // ---------------- phase B: psi rate at row m from the LDS neighbourhood
      T Pn[27];
      const int sy[3] = {sm1, s0, sp1};
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            if (!kShell3 && dx != 0 && dy != 0 && dz != 0) continue;  // corners unused
            Pn[nb(dx, dy, dz)] = L(psiL, sy[dy + 1], zi + dz, dx);
          }
      const T p0 = Pn[nb(0, 0, 0)];
      T s1 = T(0), s2 = T(0), s3 = T(0);
      T g1 = T(0), g2 = T(0), g3 = T(0);
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int sh = (dx != 0) + (dy != 0) + (dz != 0);
            if (sh == 0 || (sh == 3 && !kShell3)) continue;
            T d = Pn[nb(dx, dy, dz)] - p0;
            if (sh == 1) s1 += d; else if (sh == 2) s2 += d; else s3 += d;
            // gradient-square pairs: one term per opposite pair (first
            // non-zero offset positive)
            const int first = dx != 0 ? dx : (dy != 0 ? dy : dz);
            if (first > 0) {
              T e = Pn[nb(dx, dy, dz)] - Pn[nb(-dx, -dy, -dz)];
              if (sh == 1) g1 += e * e; else if (sh == 2) g2 += e * e; else g3 += e * e;
            }
          }
      T Lap = c.cL1 * s1 + c.cL2 * s2;
      T G = c.cG1 * g1 + c.cG2 * g2;
      if constexpr (kShell3) {
        Lap += c.cL3 * s3;
        G += c.cG3 * g3;
      }
      const Rot3<T> R = rot_of(gC);
      const T hh = T(0.5) * c.inv_h;
      T ac = aniso3<T, -1>((Pn[nb(1, 0, 0)] - Pn[nb(-1, 0, 0)]) * hh,
                           (Pn[nb(0, 1, 0)] - Pn[nb(0, -1, 0)]) * hh,
                           (Pn[nb(0, 0, 1)] - Pn[nb(0, 0, -1)]) * hh, R, c);
      // x face east of the cell
      T FxE = aniso3<T, 0>(
          (Pn[nb(1, 0, 0)] - p0) * ih,
          (Pn[nb(0, 1, 0)] + Pn[nb(1, 1, 0)] - Pn[nb(0, -1, 0)] - Pn[nb(1, -1, 0)]) * qh,
          (Pn[nb(0, 0, 1)] + Pn[nb(1, 0, 1)] - Pn[nb(0, 0, -1)] - Pn[nb(1, 0, -1)]) * qh, R, c);
      T FxW = from_left(FxE);
      // y face north of the cell
      T FyN = aniso3<T, 1>(
          (Pn[nb(1, 0, 0)] + Pn[nb(1, 1, 0)] - Pn[nb(-1, 0, 0)] - Pn[nb(-1, 1, 0)]) * qh,
          (Pn[nb(0, 1, 0)] - p0) * ih,
          (Pn[nb(0, 0, 1)] + Pn[nb(0, 1, 1)] - Pn[nb(0, 0, -1)] - Pn[nb(0, 1, -1)]) * qh, R, c);
      // z faces above (own grain) and below (grain of the cell below)
      T FzU = aniso3<T, 2>(
          (Pn[nb(1, 0, 0)] + Pn[nb(1, 0, 1)] - Pn[nb(-1, 0, 0)] - Pn[nb(-1, 0, 1)]) * qh,
          (Pn[nb(0, 1, 0)] + Pn[nb(0, 1, 1)] - Pn[nb(0, -1, 0)] - Pn[nb(0, -1, 1)]) * qh,
          (Pn[nb(0, 0, 1)] - p0) * ih, R, c);
      Rot3<T> Rd = R;
      if (kMulti) Rd = rot_of(a.grain[pzd + rowoff(m)]);
      T FzD = aniso3<T, 2>(
          (Pn[nb(1, 0, -1)] + Pn[nb(1, 0, 0)] - Pn[nb(-1, 0, -1)] - Pn[nb(-1, 0, 0)]) * qh,
          (Pn[nb(0, 1, -1)] + Pn[nb(0, 1, 0)] - Pn[nb(0, -1, -1)] - Pn[nb(0, -1, 0)]) * qh,
          (p0 - Pn[nb(0, 0, -1)]) * ih, Rd, c);
      const T ac2 = ac * ac;
      T std6 = Pn[nb(1, 0, 0)] + Pn[nb(-1, 0, 0)] + Pn[nb(0, 1, 0)] + Pn[nb(0, -1, 0)] +
               Pn[nb(0, 0, 1)] + Pn[nb(0, 0, -1)] - T(6) * p0;
      T Nn = (FxE - FxW + FyN - FyS + FzU - FzD) * ih - ac2 * (std6 * c.cStd);
      FyS = FyN;
      T F1 = T(1), F2 = uC;
      if (kFrozen) {
        T zeta = (T)ghost_near(m, ny, a.bcy) * c.h + off;
        F1 = T(1) - c.omk * zeta * c.inv_lT;
        F2 = uC + zeta * c.inv_lT;
      }
      const T ph = fC;
      const T omp = T(1) - ph * ph;
      T rhs = ac2 * (Lap - sq2 * ph * G) + Nn + sq2 * (ph - c.lambda * omp * F2);
      T rate = rhs * M::rcp(F1 * ac2);
      T aA = (T(1) + c.omk * uC) * omp * rate * T(0.5);
      if (a.bcx == PF_BC_NOFLUX) {  // mirrored columns take their image's value
        T fr = from_right(aA), fl = from_left(aA);
        aA = (x == -1) ? fr : ((x == nx) ? fl : aA);
      }
      aAL[(s0 * NZR + zi) * kRS + lane + 1] = aA;
      aAown[(m + 3) % 3] = aA;
      if (P >= 3 && m < ye && out_wave && out_lane) {
        a.psi_out[pz + (size_t)m * nx - (size_t)gx + (size_t)x] = pC + c.dt * rate;
        if (kReduce && m <= ny - 2 && fC >= T(0) && fN < T(0)) {
          double fc = (double)fC, fn = (double)fN;
          over |= ((double)m + fc / (fc - fn)) * a.hd >= ythr;
        }
      }
    }
    __syncthreads();

    if constexpr (P >= 3) {
      // ---------------- phase C: U update at row q = m - 1 (output waves)
      const int q = m - 1;
      if (P == 4 && out_wave) {
        // rows of the neighbourhood; a mirrored (no-flux) row is the row itself
        const int syq[3] = {(a.bcy == PF_BC_NOFLUX && q == 0) ? slot5(q) : slot5(q - 1), slot5(q),
                            (a.bcy == PF_BC_NOFLUX && q == ny - 1) ? slot5(q) : slot5(q + 1)};
        const int zq[3] = {ziD, zi, ziU};
        // alpha_A of a mirrored (no-flux) row is its image's value
        const bool fixS = (a.bcy == PF_BC_NOFLUX && q == 0);
        const bool fixN = (a.bcy == PF_BC_NOFLUX && q == ny - 1);
        (void)fixS;
        (void)fixN;
        T A[27], B[27];
        // field D: alpha = 1 - phi, beta = U
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              A[nb(dx, dy, dz)] = T(1) - L(phL, syq[dy + 1], zq[dz + 1], dx);
              const int sh = (dx != 0) + (dy != 0) + (dz != 0);
              if (sh < 3 || kShell3) B[nb(dx, dy, dz)] = L(UL, syq[dy + 1], zq[dz + 1], dx);
            }
        T divD = divergence27<T, kShell3>(A, B, c);
        // field A: alpha = alpha_A, beta = psi
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
              A[nb(dx, dy, dz)] = L(aAL, syq[dy + 1], zq[dz + 1], dx);
              const int sh = (dx != 0) + (dy != 0) + (dz != 0);
              if (sh < 3 || kShell3) B[nb(dx, dy, dz)] = L(psiL, syq[dy + 1], zq[dz + 1], dx);
            }
        T divA = divergence27<T, kShell3>(A, B, c);
        const T aAq = aAown[(q + 3) % 3];
        T rU = (c.D * divD + divA + sq2 * aAq) * M::rcp(T(1) + c.k - c.omk * fS);
        if (out_lane) a.U_out[pz + (size_t)q * nx - (size_t)gx + (size_t)x] = uS + c.dt * rU;
      }
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  iter(I0{}, y0 - 2);
  iter(I1{}, y0 - 1);
  iter(I2{}, y0);
  iter(I3{}, y0 + 1);
  for (int r = y0 + 2; r <= ye + 1; ++r) iter(I4{}, r);

  if (kReduce) {
    const bool any = __any(over && out_wave);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      const FrameState fi = *a.frame_in;
      a.frame_out->base = fi.base + fi.pending;
      a.frame_clear->pending = 0;
    }
    if (any && lane == 0)
      __hip_atomic_fetch_or(&a.frame_out->pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

Geom3D geom3d(int nx, int ny, int nz, int seg, int ztile) {
  Geom3D g;
  g.nstrips = (nx + 59) / 60;
  g.wout = (nx + g.nstrips - 1) / g.nstrips;
  g.ztile = ztile < 1 ? 1 : (ztile > 8 ? 8 : ztile);
  g.nzt = (nz + g.ztile - 1) / g.ztile;
  g.seg = seg < 1 ? 1 : seg;
  g.nsegs = (ny + g.seg - 1) / g.seg;
  g.threads = 64 * (g.ztile + 2);
  g.blocks = g.nstrips * g.nzt * g.nsegs;
  return g;
}

size_t step3d_lds_bytes(int ztile, size_t elem) {
  return (size_t)20 * (size_t)(ztile + 4) * (size_t)kRS * elem;
}

template <typename T>
hipError_t launch_step3d(const Step3DArgs<T> &a, const Geom3D &g, bool frozen, bool reduce,
                         bool multi, hipStream_t st) {
  dim3 grid(g.blocks), block(g.threads);
  size_t lds = step3d_lds_bytes(g.ztile, sizeof(T));
  const bool shell3 = a.c.cD3 != T(0) || a.c.cL3 != T(0) || a.c.cG3 != T(0);
#define PF_L3(F, R, MU, S3) \
  hipLaunchKernelGGL((step3d_kernel<T, F, R, MU, S3>), grid, block, lds, st, a)
#define PF_L3S(F, R, MU) \
  do { if (shell3) PF_L3(F, R, MU, true); else PF_L3(F, R, MU, false); } while (0)
  if (frozen) {
    if (reduce) { if (multi) PF_L3S(true, true, true); else PF_L3S(true, true, false); }
    else { if (multi) PF_L3S(true, false, true); else PF_L3S(true, false, false); }
  } else {
    if (reduce) { if (multi) PF_L3S(false, true, true); else PF_L3S(false, true, false); }
    else { if (multi) PF_L3S(false, false, true); else PF_L3S(false, false, false); }
  }
#undef PF_L3S
#undef PF_L3
  return hipGetLastError();
}

template hipError_t launch_step3d<float>(const Step3DArgs<float> &, const Geom3D &, bool, bool,
                                         bool, hipStream_t);
template hipError_t launch_step3d<double>(const Step3DArgs<double> &, const Geom3D &, bool, bool,
                                          bool, hipStream_t);

}  // namespace pf
