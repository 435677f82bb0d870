// step2d.hip -- fused psi/U explicit step on the 2D square lattice (gfx950).
//
// One launch advances psi and U by one explicit Euler step (Sec. 4.3.1):
//   psi^{n+1} = psi^n + dt R_psi,  R_psi from Eq. PF_a with the isotropic
//     Laplacian L_{s1,s2} (Eqs. 2D_L10, 2D_L01, 2D_L21), gradient square
//     G_{s1,s2} (App. A, Eqs. Grad_10, Grad_11), the rotated cubic
//     anisotropy (Eq. anis_function) whose eps4-linear terms use the standard
//     <10> face fluxes (Sec. 2.2), and the frozen-temperature functions
//     (Eqs. Thermal_F1, Thermal_F2);
//   U^{n+1} = U^n + dt R_U,  R_U from Eq. PF_b with D~ div[(1-phi) grad U]
//     and the approximated anti-trapping term div[alpha_A grad psi]
//     (Eq. Anti_approx), both through the two-shell divergence
//     D_{s1,s2} (Eqs. divergence_10, flux_10, divergence_11, flux_11).
//
// Schedule.  Each wave64 owns a strip of 64 lattice columns (60 outputs plus
// a 2-column halo on each side) and a segment of `seg` rows, and marches up
// the segment one row per iteration, holding a 3-row window of psi, U, phi
// and alpha_A in registers.  x neighbours come from DPP wave shifts, so the
// kernel uses no LDS and no barrier outside the final reduction.  With the
// newest row r loaded, an iteration computes the y face flux r-1/2, the psi
// rate of row r-1 (written out as psi^{n+1} and turned into alpha_A), and the
// U update of row r-2, which needs alpha_A on rows r-3..r-1.  Fluxes shared
// between neighbouring cells are computed once: x-direction ones are passed
// across lanes, y-direction ones carried to the next row; the two divergences
// of Eq. PF_b are combined link by link.  With the moving frame the same pass
// decides from the phi = 0 crossings of state n whether state n+1 moves one
// row (FP64 crossing heights, one flag per wave); with dynamic grains it
// writes the next level's grain map.
//
// Variants (template kAT) for the scheme comparison of Sec. 4.3 (Table 1):
//   kAtApproxShells    the approximated current on shell fluxes (S-bar_{2,1});
//   kAtFullShells      the full current div[alpha grad psi/|grad psi|] of
//                      Eq. Anti_convention: each shell flux of the A
//                      divergence divided by |grad psi| at its flux point, from
//                      the fourth-order stencils of App. B (S_{2,1}).  These
//                      reach rows q-2..q+2 and columns x-2..x+2 of the U row q,
//                      so the window keeps two more psi rows and the +-2
//                      columns of two rows; the 2-lane halo already covers them;
//   kAtFullTwoPoint    both divergences on the <10> faces alone with the mean
//                      of the two cells as face alpha, the full current with
//                      the face gradient from the normal difference and the
//                      four-point tangential difference (S_{1,0});
//   kAtApproxTwoPoint  the same faces with the approximated current;
//   kAtDiffusionOnly   psi held (copied), U advanced by the diffusion term of
//                      Eq. PF_b alone on the shell divergence: the same bytes
//                      per cell with a fraction of the arithmetic.
#include <type_traits>

#include "pf_device.hpp"

namespace pf {

namespace {

template <typename T>
struct Rot2 {
  T r00, r01, r10, r11;  // crystal -> lab
};

// Both functions take the gradient in any positive multiple of its true
// value (g~ = s g): a_s does not depend on the scale and J is homogeneous of
// degree 1, so J(g~) = s J(g).  g2eps is the guard |g|^2 <= 1e-12 expressed
// for g~ (1e-12 s^2): at or below it a_s = 1 and J = g~.
//
// In 2D the cubic form of Eq. anis_function, a_s = 1 - 3 eps4 + 4 eps4
// (u^4 + v^4) with (u, v) = R^T g/|g|, equals 1 + eps4 - 8 eps4 u^2 v^2
// (= 1 + eps4 cos 4(theta - alpha0)).
template <typename T>
__device__ __forceinline__ T aniso_a(T gx, T gy, T g2eps, const Rot2<T> &R, const Coef<T> &c) {
  T g2 = gx * gx + gy * gy;
  T r2 = Math<T>::rcp(g2 > g2eps ? g2 : g2eps);
  T cx = R.r00 * gx + R.r10 * gy;
  T cy = R.r01 * gx + R.r11 * gy;
  T w = cx * cy * r2;
  T a = c.an1 - c.an8 * w * w;
  return g2 > g2eps ? a : T(1);
}

// Component `comp` (0: x, 1: y) of the anisotropic flux
// J = a^2 g + |g|^2 a da/dg.  In 2D the second term is a (da/dtheta) g_perp,
// g_perp = (-gy, gx), with da/dtheta = -16 eps4 u v (u^2 - v^2).
template <typename T, int comp>
__device__ __forceinline__ T aniso_flux(T gx, T gy, T g2eps, const Rot2<T> &R,
                                        const Coef<T> &c) {
  T g2 = gx * gx + gy * gy;
  T r2 = Math<T>::rcp(g2 > g2eps ? g2 : g2eps);
  T cx = R.r00 * gx + R.r10 * gy;
  T cy = R.r01 * gx + R.r11 * gy;
  T w = cx * cy * r2;
  T a = c.an1 - c.an8 * w * w;
  T ath = c.an16 * w * ((cx * cx - cy * cy) * r2);  // -da/dtheta
  T j = comp == 0 ? a * (a * gx + ath * gy) : a * (a * gy - ath * gx);
  T plain = comp == 0 ? gx : gy;
  return g2 > g2eps ? j : plain;
}

// Logical blocks -> hardware blocks so that each of the 8 XCDs (which take
// consecutive hardware blocks round-robin) runs a contiguous range of strips
// and shares their halo rows in its own L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int X = 8;
  int q = nb / X, r = nb % X, x = b % X;
  return x * q + (x < r ? x : r) + b / X;
}

// Waves per SIMD the register budget must leave room for.  The steady-state
// row group is one basic block, so the scheduler overlaps rows freely: FP32
// variants settle at 85-132 VGPRs (3-5 waves per SIMD) and run fastest
// unconstrained; the FP64 approximated-current single-grain variants would
// take 200+ VGPRs (2 waves) and run 6-18% faster held to 3 waves (168 VGPRs,
// no spills).  The other FP64 variants would spill there and stay
// unconstrained.
template <typename T, bool kMulti, int kAT>
constexpr int kMinWaves2D =
    sizeof(T) == 8 && !kMulti &&
            (kAT == kAtApproxShells || kAT == kAtApproxTwoPoint || kAT == kAtDiffusionOnly)
        ? 3
        : 1;
// The batched kernel's FP32 variants hold 4 waves per SIMD: unconstrained,
// its frozen variants settle at 124-132 VGPRs, where the 4th wave comes and
// goes with small changes to the body; held to 128, two spill a register or
// two outside the row loop.
template <typename T, bool kMulti>
constexpr int kMinWavesBatch2D = sizeof(T) == 4 ? 4 : kMinWaves2D<T, kMulti, kAtApproxShells>;

// One logical workgroup `lb` (4 waves) of the step of one solve `a`.
template <typename T, bool kFrozen, bool kReduce, bool kMulti, int kAT, bool kRowTail = true>
__device__ __forceinline__ void step2d_body(const Step2DArgs<T> &a, const int lb) {
  constexpr bool kTwoPoint = kAT == kAtFullTwoPoint || kAT == kAtApproxTwoPoint;
  constexpr bool kDiff = kAT == kAtDiffusionOnly;
  using M = Math<T>;
  const Coef<T> &c = a.c;
  const int lane = threadIdx.x & 63;
  // wave-uniform: keeps strip, segment and row counters in scalar registers
  const int wave = lb * 4 + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int nx = a.nx, ny = a.ny;

  bool over_any = false;

  if (wave < a.nstrips * a.nsegs) {
    const int strip = wave % a.nstrips, segi = wave / a.nstrips;
    const int x = strip * a.wout - 2 + lane;
    const int gx = ghost(x, nx, a.bcx);
    const bool out_lane = lane >= 2 && lane < 2 + a.wout && x < nx;
    // rows split evenly: the first segrem segments take one row more
    const int y0 = segi * a.segbase + min(segi, a.segrem);
    const int ye = y0 + a.segbase + (segi < a.segrem ? 1 : 0);
    const int pend = a.frame ? a.frame_in->pending : 0;
    const long long shift = a.frame ? a.frame_in->base + pend : 0;
    T off = T(0);
    if (kFrozen) off = (T)((double)shift * a.hd - a.y0 - a.Vp * ((double)a.step * a.dtd));
    const double ythr = (double)a.shift_row * a.hd;
    bool over = false;  // this lane saw a crossing at or above the shift row
    const T sq2 = T(1.4142135623730951);
    const T isq2 = T(0.70710678118654752);

    auto prow = [&](int r) -> size_t {
      int j = ghost_near(r, ny, a.bcy);
      if (pend) j = min(j + 1, ny - 1);
      return (size_t)j * (size_t)nx + (size_t)gx;
    };
    // the same for the steady state, whose rows (y0 + 5 .. ye + 1) can only
    // cross the top boundary, in plain arithmetic: no branch splits the row
    const int top_per = a.bcy == PF_BC_PERIODIC ? ny : 0;
    const int top_mir = a.bcy == PF_BC_PERIODIC ? 0 : 1;
    auto prow_top = [&](int r) -> size_t {
      const int over = max(r - (ny - 1), 0);  // 0, 1 or 2 rows past the top
      const int j = r - top_per * min(over, 1) - top_mir * max(2 * over - 1, 0);
      return (size_t)min(j + pend, ny - 1) * (size_t)nx + (size_t)gx;
    };
    auto rot_of = [&](int g) -> Rot2<T> {
      if (kMulti) {
        const T *q = a.rot + 4 * g;
        return Rot2<T>{q[0], q[1], q[2], q[3]};
      }
      return Rot2<T>{a.r00, a.r01, a.r10, a.r11};
    };

    // register window: S = row r-2, C = row r-1, N = row r (newest)
    T pS = 0, pSW = 0, pSE = 0, pC = 0, pCW = 0, pCE = 0, pN = 0, pNW = 0, pNE = 0;
    T uS = 0, uC = 0, uN = 0;
    T fS = 0, fC = 0, fN = 0;
    T aAS = 0, aAC = 0;
    int gS = 0, gC = 0, gN = 0;
    T FyS = 0;  // y face flux below row r-1
    // carries of the divergence for the row pair below (q-1, q): the combined
    // north and diagonal links, and the plaquette alphas of both fields
    T cN = 0, c1 = 0, c2 = 0, cPD = 0, cPA = 0;
    // full current only: B1 = row r-3, B2 = row r-4, and the x+-2 columns of
    // rows r-1 (C) and r-2 (S)
    T pB1 = 0, pB1W = 0, pB1E = 0, pB1E2 = 0, pB2 = 0, pB2E = 0;
    T pCE2 = 0, pCW2 = 0, pSE2 = 0, pSW2 = 0;

    // rows r, r+1, r+2 in flight (loads issued two iterations ahead)
    T lp0, lu0, lp1, lu1, lp2, lu2;
    int lg0 = 0, lg1 = 0, lg2 = 0;
    {
      size_t o0 = prow(y0 - 2), o1 = prow(y0 - 1), o2 = prow(y0);
      lp0 = a.psi_in[o0]; lu0 = a.U_in[o0];
      lp1 = a.psi_in[o1]; lu1 = a.U_in[o1];
      lp2 = a.psi_in[o2]; lu2 = a.U_in[o2];
      if (kMulti) { lg0 = a.grain[o0]; lg1 = a.grain[o1]; lg2 = a.grain[o2]; }
    }

    // One row of the pipeline.  P is the pipeline phase: 0 loads only (row
    // y0-2), 1 adds the y face flux, 2 the psi rate of row y0-1, 3 the first
    // stored psi row and the divergence carries of the pair (y0-1, y0), 4 is
    // the steady state with every stage active.
    // moving-frame decision: an interface cell of row m whose
    // phi = 0 crossing lies at or above the shift row.  Rows at or above it
    // qualify outright and rows below the one under it cannot (the crossing
    // lies within one row), so the loop votes with plain masks; the FP64
    // crossing height of the row under the shift row is taken once, below.
    auto frame_vote = [&](int m, T f0, T f1) -> bool {
      return out_lane & (m >= a.shift_row) & (m <= ny - 2) & (f0 >= T(0)) & (f1 < T(0));
    };
    auto iter = [&](auto phase, int r) {
      constexpr int P = decltype(phase)::value;
      if constexpr (kAT == kAtFullShells) {
        pB2 = pB1; pB2E = pB1E; pB1E2 = pSE2;
        pSE2 = pCE2; pSW2 = pCW2;
      }
      if constexpr (kAT == kAtFullShells || kAT == kAtFullTwoPoint) {
        pB1 = pS; pB1W = pSW; pB1E = pSE;
      }
      pS = pC; pSW = pCW; pSE = pCE;
      pC = pN; pCW = pNW; pCE = pNE;
      uS = uC; uC = uN;
      fS = fC; fC = fN;
      aAS = aAC;
      gS = gC;
      gC = gN;
      pN = lp0; uN = lu0; gN = lg0;
      lp0 = lp1; lu0 = lu1; lg0 = lg1;
      lp1 = lp2; lu1 = lu2; lg1 = lg2;
      if (P >= 5 || r + 3 <= ye + 1) {
        // steady state: the last rows reload row ye + 1 (never consumed)
        // instead of branching around the load
        size_t on = P >= 5 ? prow_top(min(r + 3, ye + 1)) : prow(r + 3);
        lp2 = a.psi_in[on];
        lu2 = a.U_in[on];
        if (kMulti) lg2 = a.grain[on];
      }
      pNW = from_left(pN);
      pNE = from_right(pN);
      fN = M::tanh_(pN * isq2);
      if constexpr (P == 0) return;
      if constexpr (kAT == kAtFullShells && P >= 2) {
        pCE2 = from_right(pCE);
        pCW2 = from_left(pCW);
      }

      // y face between rows r-1 and r, grain of the lower cell; face
      // fluxes are h J (gradients passed as h g)
      T FyN = T(0);
      if constexpr (!kDiff)
        FyN = aniso_flux<T, 1>(T(0.25) * (pNE + pCE - pNW - pCW), pN - pC, c.at_eps, rot_of(gC),
                               c);
      // dynamic grains: the grain of row m at the next level (a liquid cell,
      // psi < 0, with a solid face neighbour takes the grain of the solid
      // neighbour with the largest psi, first of -x, +x, -y, +y on ties)
      auto grain_next = [&](int m) {
        if constexpr (kMulti) {
          if (a.grain_out != nullptr && P >= 3 && m < ye) {
            const int gW = from_left(gC), gE = from_right(gC);
            int gn = gC;
            if (pC < T(0)) {
              T best = T(0);
              bool found = false;
              auto take = [&](T v, int g) {
                if (v >= T(0) && (!found || v > best)) {
                  best = v;
                  gn = g;
                  found = true;
                }
              };
              take(pCW, gW);
              take(pCE, gE);
              take(pS, gS);
              take(pN, gN);
            }
            if (out_lane) a.grain_out[(size_t)m * (size_t)nx + (size_t)x] = (int8_t)gn;
          }
        }
      };
      if constexpr (P >= 2 && kDiff) {
        // psi is held: copy row m and take the frame decision on it
        const int m = r - 1;
        grain_next(m);
        if (P >= 3 && m < ye) {
          store_row(a.psi_out + (size_t)m * (size_t)nx, nx, x, out_lane, pC);
          if (kReduce) over = over | frame_vote(m, fC, fN);
        }
      } else if constexpr (P >= 2) {
        // ---------------- psi rate at row m (window rows S, C, N = m-1, m, m+1)
        const int m = r - 1;
        grain_next(m);
        const Rot2<T> R = rot_of(gC);
        T dE = pCE - pC, dW = pCW - pC, dN = pN - pC, dS = pS - pC;
        T s10 = dE + dW + dN + dS;
        T s11 = (pNE - pC) + (pNW - pC) + (pSE - pC) + (pSW - pC);
        T L = c.cL1 * s10 + c.cL2 * s11;
        T ex = pCE - pCW, ey = pN - pS;
        T e1 = pNE - pSW, e2 = pSE - pNW;
        T G = c.cG1 * (ex * ex + ey * ey) + c.cG2 * (e1 * e1 + e2 * e2);
        T ac = aniso_a(ex, ey, c.ac_eps, R, c);  // (ex, ey) = 2h g
        T FxE = aniso_flux<T, 0>(dE, T(0.25) * (pN + pNE - pS - pSE), c.at_eps, R, c);
        T FxW = from_left(FxE);
        T ac2 = ac * ac;
        T Nn = (FxE - FxW + FyN - FyS - ac2 * s10) * c.cStd;
        T F1 = T(1), F2 = uC;
        if (kFrozen) {
          T zeta = (T)(P >= 5 ? m : ghost_near(m, ny, a.bcy)) * c.h + off;
          F1 = T(1) - c.omk * zeta * c.inv_lT;
          F2 = uC + zeta * c.inv_lT;
        }
        T ph = fC;
        T omp = T(1) - ph * ph;
        T rhs = ac2 * (L - sq2 * ph * G) + Nn + sq2 * (ph - c.lambda * omp * F2);
        T rate = rhs * M::rcp(F1 * ac2);
        T aA = (T(1) + c.omk * uC) * omp * rate * T(0.5);
        if (P == 6 || (P < 5 && a.bcx == PF_BC_NOFLUX)) {  // mirrored columns copy their image
          T fr = from_right(aA), fl = from_left(aA);
          aA = (x == -1) ? fr : ((x == nx) ? fl : aA);
        }
        aAC = aA;
        // mirrored rows copy their image (rows 0 and ny, never met inside the
        // unrolled steady state: phase 5)
        if (P < 5 && a.bcy == PF_BC_NOFLUX) {
          if (m == 0) aAS = aAC;
          if (m == ny) aAC = aAS;
        }
        if (P >= 5 || (P >= 3 && m < ye)) {
          store_row(a.psi_out + (size_t)m * (size_t)nx, nx, x, out_lane, pC + c.dt * rate);
          if (kReduce) over = over | frame_vote(m, fC, fN);
        }
      }
      FyS = FyN;

      // ---------------- divergences of row q = r-2.  Both fields of Eq. PF_b
      // are combined link by link, D~ f_D + lambda f_A with D~ folded into
      // alpha_D = D~ (1 - phi) and lambda = 1, or h for the full current (whose
      // links carry h / |h grad psi|): one set of sums, lane moves and carries.
      constexpr bool kFullAT = kAT == kAtFullShells || kAT == kAtFullTwoPoint;
      if constexpr (P >= 3 && kTwoPoint) {
        // <10> faces: east face of row q and north face (q+1/2)
        const int q = r - 2;
        T aq = c.D - c.D * fS, aq1 = c.D - c.D * fC;
        const T kE = aq + from_right(aq), kN = aq + aq1;
        const T gE = from_right(uS) - uS, gN = uC - uS;
        T fE = kE * gE, fN = kN * gN;
        T dE = pSE - pS, dN = pC - pS;
        T fEA = (aAS + from_right(aAS)) * dE;
        T fNA = (aAS + aAC) * dN;
        if constexpr (kFullAT) {
          // |grad psi| h at the faces: normal difference and a quarter of the
          // four-point tangential difference
          T tE = pC + pCE - pB1 - pB1E;
          T tN = pSW + pCW - pSE - pCE;
          T gE = dE * dE + T(0.0625) * (tE * tE);
          T gN = dN * dN + T(0.0625) * (tN * tN);
          fEA *= gE > c.at_eps ? M::rsq(gE) : T(0);
          fNA *= gN > c.at_eps ? M::rsq(gN) : T(0);
          fE += c.h * fEA;
          fN += c.h * fNA;
        } else {
          fE = fEA + kE * gE;
          fN = fNA + kN * gN;
        }
        if constexpr (P >= 4) {
          T div = c.cT * (fE - from_left(fE) + fN - cN);
          T rU = (div + sq2 * aAS) * M::rcp(T(1) + c.k - c.omk * fS);
          store_row(a.U_out + (size_t)q * (size_t)nx, nx, x, out_lane, uS + c.dt * rU);
        }
        cN = fN;
      } else if constexpr (P >= 3) {
        // shells on the row pair (q, q+1) = (S, C): field D alpha = D~(1 - phi),
        // beta = U; field A alpha = alpha_A, beta = psi
        const int q = r - 2;
        T aq = c.D - c.D * fS, aq1 = c.D - c.D * fC;
        T aE = from_right(aq), aNE = from_right(aq1);
        T PD = (aq + aE + aq1 + aNE) * T(0.25);
        T PDW = from_left(PD);
        T uE = from_right(uS), uNE = from_right(uC), uNW = from_left(uC);
        const T kE = aq + aE + PD + cPD, kN = aq + aq1 + PD + PDW;
        const T gE = uE - uS, gN = uC - uS, gNE = uNE - uS, gNW = uNW - uS;
        T fE = kE * gE, fN = kN * gN;
        T d1 = PD * gNE, d2 = PDW * gNW;

        T PA = T(0);
        if constexpr (!kDiff) {
          T bE = from_right(aAS), bNE = from_right(aAC);
          PA = (aAS + bE + aAC + bNE) * T(0.25);
          T PAW = from_left(PA);
          T fEA = (aAS + bE + PA + cPA) * (pSE - pS);
          T fNA = (aAS + aAC + PA + PAW) * (pC - pS);
          T d1A = PA * (pCE - pS);
          T d2A = PAW * (pCW - pS);
          if constexpr (kAT == kAtFullShells) {
            // App. B gradients (times h) at the north face (q+1/2), the
            // north-east corner (q+1/2, x+1/2) and, for the U row, the east face
            // (q, x+1/2); the west, north-west and south links reuse the
            // neighbours' values
            auto inv = [&](T gx, T gy) {
              T g2 = gx * gx + gy * gy;
              return g2 > c.at_eps ? M::rsq(g2) : T(0);
            };
            const T k1 = T(35.0 / 48.0), k2 = T(1.0 / 48.0), k3 = T(1.0 / 6.0);
            const T m1 = T(35.0 / 96.0), m2 = T(1.0 / 32.0), m3 = T(1.0 / 24.0);
            T invN;
            {  // face (0, 1/2): the (1/2, 0) stencil turned a quarter
              T a1 = pCW - pSE, b1 = pCE - pSW;
              T a2 = pNW - pB1E, b2 = pNE - pB1W;
              T a3 = pCW2 - pSE2, b3 = pCE2 - pSW2;
              T gx = k1 * (a1 + b1) - k2 * (a2 + b2) - k3 * (a3 + b3);
              T gy = m1 * (a1 - b1) - m2 * (a2 - b2) - m3 * (a3 - b3);
              invN = inv(gx, gy);
            }
            T invNE;
            {  // corner (1/2, 1/2)
              T a1 = pCE - pS, b1 = pSE - pC;
              T a2 = pCE2 - pSW, b2 = pSE2 - pCW;
              T a3 = pNE - pB1, b3 = pB1E - pN;
              T gx = T(5.0 / 8.0) * (a1 + b1) - T(1.0 / 48.0) * (a2 + b2) -
                     T(1.0 / 16.0) * (a3 + b3);
              T gy = T(5.0 / 8.0) * (a1 - b1) - T(1.0 / 16.0) * (a2 - b2) -
                     T(1.0 / 48.0) * (a3 - b3);
              invNE = inv(gx, gy);
            }
            fNA *= invN;
            d1A *= invNE;
            d2A *= from_left(invNE);
            if constexpr (P >= 4) {  // face (1/2, 0)
              T a1 = pCE - pB1, b1 = pB1E - pC;
              T a2 = pCE2 - pB1W, b2 = pB1E2 - pCW;
              T a3 = pNE - pB2, b3 = pB2E - pN;
              T gx = k1 * (a1 + b1) - k2 * (a2 + b2) - k3 * (a3 + b3);
              T gy = m1 * (a1 - b1) - m2 * (a2 - b2) - m3 * (a3 - b3);
              fEA *= inv(gx, gy);
            }
            fE += c.h * fEA;
            fN += c.h * fNA;
            d1 += c.h * d1A;
            d2 += c.h * d2A;
          } else {
            // one expression per link, so each U product fuses with the
            // psi link into a multiply-add
            fE = fEA + kE * gE;
            fN = fNA + kN * gN;
            d1 = d1A + PD * gNE;
            d2 = d2A + PDW * gNW;
          }
        }

        if constexpr (P >= 4) {
          T div = c.cD1 * (fE - from_left(fE) + fN - cN) +
                  c.cD2 * (d1 + d2 - from_left(c1) - from_right(c2));
          // the held psi has no anti-trapping current and no source
          T rU = (kDiff ? div : div + sq2 * aAS) * M::rcp(T(1) + c.k - c.omk * fS);
          store_row(a.U_out + (size_t)q * (size_t)nx, nx, x, out_lane, uS + c.dt * rU);
        }
        cN = fN; c1 = d1; c2 = d2; cPD = PD; cPA = PA;
      }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;  // phase 4 on rows 1..ny-1
    using I6 = std::integral_constant<int, 6>;  // phase 5, mirrored x columns
    iter(I0{}, y0 - 2);
    iter(I1{}, y0 - 1);
    iter(I2{}, y0);
    iter(I3{}, y0 + 1);
    // steady state unrolled by 6, a multiple of every register-rotation
    // period (3 for the row window, the grains and the loads in flight, 2 for
    // alpha_A, 1 for the carries), so the rotation costs no register moves.
    // Its psi rows m = r - 1 run from y0 + 1 to at most ye - 1, so none is
    // row 0 or ny.
    // The rows left over (fewer than 6) run one at a time, still straight-line
    // (the window then rotates by register moves); only the last iteration,
    // whose psi row ye belongs to the next segment, takes the checked phase 4.
    // Without kRowTail (batched launches: long segments, and waves of many
    // solves at different points of the code) they take phase 4, which keeps
    // the code smaller.
    int r = y0 + 2;
    if (a.bcx == PF_BC_NOFLUX) {  // phase 6: phase 5 with mirrored columns
      for (; r + 5 <= ye; r += 6) {
        iter(I6{}, r);
        iter(I6{}, r + 1);
        iter(I6{}, r + 2);
        iter(I6{}, r + 3);
        iter(I6{}, r + 4);
        iter(I6{}, r + 5);
      }
      if constexpr (kRowTail)
        for (; r <= ye; ++r) iter(I6{}, r);
    } else {
      for (; r + 5 <= ye; r += 6) {
        iter(I5{}, r);
        iter(I5{}, r + 1);
        iter(I5{}, r + 2);
        iter(I5{}, r + 3);
        iter(I5{}, r + 4);
        iter(I5{}, r + 5);
      }
      if constexpr (kRowTail)
        for (; r <= ye; ++r) iter(I5{}, r);
    }
    for (; r <= ye + 1; ++r) iter(I4{}, r);
    if (kReduce) {
      // the row under the shift row: its crossing height in FP64, on the phi
      // the pipeline computed from the same loads
      const int ms = a.shift_row - 1;
      if (ms >= y0 && ms < ye && ms <= ny - 2) {
        const T f0 = M::tanh_(a.psi_in[prow(ms)] * isq2);
        const T f1 = M::tanh_(a.psi_in[prow(ms + 1)] * isq2);
        if (out_lane && f0 >= T(0) && f1 < T(0))
          over |= crossing_reaches(f0, f1, ms, a.shift_row, ythr, a.hd);
      }
      over_any = __any(over);
    }
  }

  if (kReduce) {
    // moving frame: publish the shift count of this level, flag the next
    // level for a one-row shift if any crossing reached the shift row, and
    // clear the record the next step will write into
    if (lb == 0 && threadIdx.x == 0) {
      const FrameState fi = *a.frame_in;
      a.frame_out->base = fi.base + fi.pending;
      a.frame_clear->pending = 0;
    }
    if (over_any && lane == 0)
      __hip_atomic_fetch_or(&a.frame_out->pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T, bool kFrozen, bool kReduce, bool kMulti, int kAT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMinWaves2D<T, kMulti, kAT>)))
void step2d_kernel(Step2DArgs<T> a) {
  step2d_body<T, kFrozen, kReduce, kMulti, kAT>(a, xcd_remap((int)blockIdx.x, (int)gridDim.x));
}

// Many solves in one launch: workgroup b runs logical workgroup map[b].y of
// solve map[b].x.  Launch k of an epoch steps every solve from its level
// n0 + k: buffers and frame records are picked from the epoch's parities.
template <typename T, bool kFrozen, bool kReduce, bool kMulti>
__global__ __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(kMinWavesBatch2D<T, kMulti>)))
void batch2d_kernel(const BatchSolve2D<T> *table,
                                                      const int2 *map, int k) {
  const int2 bm = map[blockIdx.x];
  const BatchSolve2D<T> &e = table[bm.x];
  Step2DArgs<T> a = e.a;
  const long long n = e.n0 + k;
  const int par = (int)((e.par0 + k) & 1);
  a.psi_in = e.psi[par];
  a.U_in = e.U[par];
  a.psi_out = e.psi[par ^ 1];
  a.U_out = e.U[par ^ 1];
  a.step = n;
  if (kReduce) {
    const int f = (e.f0 + k) % 3;
    a.frame_in = e.frames[f];
    a.frame_out = e.frames[(f + 1) % 3];
    a.frame_clear = e.frames[(f + 2) % 3];
  }
  step2d_body<T, kFrozen, kReduce, kMulti, kAtApproxShells, false>(a, bm.y);
}

// Advance the epoch origin of every solve by `steps` (end of a captured graph).
template <typename T>
__global__ void batch2d_advance(BatchSolve2D<T> *table, int n, int steps, int frame) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    table[i].n0 += steps;
    table[i].par0 = (table[i].par0 + steps) & 1;
    if (frame) table[i].f0 = (table[i].f0 + steps) % 3;
  }
}

}  // namespace

Geom2D geom2d(int nx, int ny, int seg, int ncu) {
  Geom2D g;
  g.nstrips = (nx + 59) / 60;
  g.wout = (nx + g.nstrips - 1) / g.nstrips;
  g.seg = seg == 0 ? 1 : seg;
  if (g.seg > 0) {
    g.nsegs = (ny + g.seg - 1) / g.seg;
  } else {
    // -k: k waves per SIMD, i.e. k * 4 * ncu waves in all (4 SIMDs per CU)
    const long long want = (long long)(-g.seg) * 4 * (ncu > 0 ? ncu : 1) / g.nstrips;
    g.nsegs = (int)std::max(1LL, std::min((long long)ny, want));
  }
  g.segbase = ny / g.nsegs;
  g.segrem = ny % g.nsegs;
  int waves = g.nstrips * g.nsegs;
  g.blocks = (waves + 3) / 4;
  return g;
}

template <typename T, int kAT>
void launch_step2d_at(const Step2DArgs<T> &a, const Geom2D &g, bool frozen, bool reduce,
                      bool multi, hipStream_t st) {
  dim3 grid(g.blocks), block(256);
#define PF_L2(F, R, MU) \
  hipLaunchKernelGGL((step2d_kernel<T, F, R, MU, kAT>), grid, block, 0, st, a)
  if (frozen) {
    if (reduce) { if (multi) PF_L2(true, true, true); else PF_L2(true, true, false); }
    else { if (multi) PF_L2(true, false, true); else PF_L2(true, false, false); }
  } else {
    if (reduce) { if (multi) PF_L2(false, true, true); else PF_L2(false, true, false); }
    else { if (multi) PF_L2(false, false, true); else PF_L2(false, false, false); }
  }
#undef PF_L2
}

template <typename T>
hipError_t launch_step2d(const Step2DArgs<T> &a, const Geom2D &g, bool frozen, bool reduce,
                         bool multi, int at, hipStream_t st) {
  switch (at) {
    case kAtApproxShells: launch_step2d_at<T, kAtApproxShells>(a, g, frozen, reduce, multi, st); break;
    case kAtFullShells: launch_step2d_at<T, kAtFullShells>(a, g, frozen, reduce, multi, st); break;
    case kAtFullTwoPoint: launch_step2d_at<T, kAtFullTwoPoint>(a, g, frozen, reduce, multi, st); break;
    case kAtApproxTwoPoint:
      launch_step2d_at<T, kAtApproxTwoPoint>(a, g, frozen, reduce, multi, st);
      break;
    case kAtDiffusionOnly:
      launch_step2d_at<T, kAtDiffusionOnly>(a, g, frozen, reduce, multi, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch2d(const BatchSolve2D<T> *table, const int2 *map, int blocks, int k,
                          bool frozen, bool reduce, bool multi, hipStream_t st) {
  dim3 grid(blocks), block(256);
#define PF_LB(F, R, MU) \
  hipLaunchKernelGGL((batch2d_kernel<T, F, R, MU>), grid, block, 0, st, table, map, k)
  if (frozen) {
    if (reduce) { if (multi) PF_LB(true, true, true); else PF_LB(true, true, false); }
    else { if (multi) PF_LB(true, false, true); else PF_LB(true, false, false); }
  } else {
    if (reduce) { if (multi) PF_LB(false, true, true); else PF_LB(false, true, false); }
    else { if (multi) PF_LB(false, false, true); else PF_LB(false, false, false); }
  }
#undef PF_LB
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch2d_advance(BatchSolve2D<T> *table, int n, int steps, bool frame,
                                  hipStream_t st) {
  hipLaunchKernelGGL((batch2d_advance<T>), dim3((n + 63) / 64), dim3(64), 0, st, table, n, steps,
                     frame ? 1 : 0);
  return hipGetLastError();
}

template hipError_t launch_batch2d<float>(const BatchSolve2D<float> *, const int2 *, int, int,
                                          bool, bool, bool, hipStream_t);
template hipError_t launch_batch2d<double>(const BatchSolve2D<double> *, const int2 *, int, int,
                                           bool, bool, bool, hipStream_t);
template hipError_t launch_batch2d_advance<float>(BatchSolve2D<float> *, int, int, bool,
                                                  hipStream_t);
template hipError_t launch_batch2d_advance<double>(BatchSolve2D<double> *, int, int, bool,
                                                   hipStream_t);

template hipError_t launch_step2d<float>(const Step2DArgs<float> &, const Geom2D &, bool, bool,
                                         bool, int, hipStream_t);
template hipError_t launch_step2d<double>(const Step2DArgs<double> &, const Geom2D &, bool, bool,
                                          bool, int, hipStream_t);

}  // namespace pf
