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
// lock-step.  Each iteration publishes the newest psi, U and D~(1 - phi) row
// in LDS rings of 5 rows, then (barrier) computes the psi rate of the row
// below from the LDS 3x3x3 neighbourhood (its z-down face flux is the wave
// below's z-up one, read after a barrier) and publishes alpha_A, then
// (barrier) evaluates the divergence links of the row below that.  Every
// link is evaluated once: a cell owns the links towards +x, +y or +z (9, and
// 4 of the <111> shell) and takes the others with the opposite sign from the
// lane to its left, from the row below (register carries) and, for links to
// the z-rows below and the links to the row below in other z-rows, from an
// exchange buffer in which each wave publishes two sums per lane and row.  A
// row's U is therefore finished one iteration later, after the next barriers.
// With the moving frame the pass takes the frame decision as in 2D; with
// dynamic grains it writes the next level's grain map.  No-flux walls: psi, U and phi
// are read through the mirror map, and every field beyond a wall is read at
// its image (alpha_A of a mirrored cell included).
#include <atomic>
#include <type_traits>

#include "pf_device.hpp"

namespace pf {

namespace {

template <typename T>
struct Rot3 {
  T m[9];  // row-major crystal -> lab
};

// a_s and, optionally, one lab component of J = a^2 g + |g|^2 a da/dg
// (J = R [g'(a^2 - 16 eps4 a s4) + 16 eps4 a g'^3/|g|^2], g' = R^T g).
// a_s is scale-free and J homogeneous of degree 1, so callers pass a scaled
// gradient (4h g at faces, 2h g at the centre) with the |g|^2 <= 1e-12 guard
// scaled alike (eps), and unscale J once.
template <typename T, int comp>
__device__ __forceinline__ T aniso3(T gx, T gy, T gz, const Rot3<T> &R, const Coef<T> &c,
                                    T eps) {
  T g2 = gx * gx + gy * gy + gz * gz;
  T r2 = Math<T>::rcp(g2 > eps ? g2 : eps);
  T c0 = R.m[0] * gx + R.m[3] * gy + R.m[6] * gz;
  T c1 = R.m[1] * gx + R.m[4] * gy + R.m[7] * gz;
  T c2 = R.m[2] * gx + R.m[5] * gy + R.m[8] * gz;
  T q0 = c0 * c0, q1 = c1 * c1, q2 = c2 * c2;
  T s4 = (q0 * q0 + q1 * q1 + q2 * q2) * (r2 * r2);
  T a = c.an0 + c.an4 * s4;
  if constexpr (comp < 0) {
    return g2 > eps ? a : T(1);
  } else {
    T t = c.an16 * a;
    T base = a * a - t * s4;
    T tr = t * r2;
    T j0 = c0 * (base + tr * q0);
    T j1 = c1 * (base + tr * q1);
    T j2 = c2 * (base + tr * q2);
    T j = R.m[3 * comp + 0] * j0 + R.m[3 * comp + 1] * j1 + R.m[3 * comp + 2] * j2;
    T plain = comp == 0 ? gx : (comp == 1 ? gy : gz);
    return g2 > eps ? j : plain;
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
enum LdsField { kPsi = 0, kU = 1, kAD = 2, kAA = 3 };  // alpha_D = D~ (1 - phi), alpha_A

// alpha averages of the links a cell owns, times their shell coefficient
// (Eqs. divergence_100, divergence_110): <100> links abar = P(0) + P(d) with
// P = alpha/4 + (sum of the 4 neighbours across the link axis)/16; <110>
// links abar = 3/16 (in-plane plaquette) + 1/32 (the two plaquettes beside
// it along the third axis).  Py1 is P_y of the cell one row up, carried.
// <111> links (sx, +1, sz): abar = mean of the 8 corners of the cube.
template <typename T>
struct Abar9 {
  T E, N, Up, NE, NW, EU, WU, NU, ND, Py1;
  T Tpp, Tmp, Tpm, Tmm;  // <111> links (+1,+1,+1), (-1,+1,+1), (+1,+1,-1), (-1,+1,-1)
};
template <typename T>
struct Diff9 {
  T E, N, Up, NE, NW, EU, WU, NU, ND;
  T Tpp, Tmp, Tpm, Tmm;
};

// FP32 workgroups run up to 16 waves (ztile <= 14, at most 128 VGPRs per
// lane); FP64 ones, which need about 230 VGPRs, up to 8 (ztile <= 6, two
// waves per SIMD).
template <typename T>
constexpr int max_threads3d() { return sizeof(T) == 8 ? 512 : 1024; }

// One tile of the step: a workgroup of nw waves marching up one y segment.
// Wide tiles (kG = 1): each wave is one z row of 64 lanes holding a strip of
// up to 60 output columns with a 2-column halo on each side.  Thin tiles
// hold the strip of the last nx mod 60 columns: each wave is kG = 3 or 4 lane
// groups of 21 or 16 lanes, each group its own z row, so that a narrow strip
// does not leave most lanes idle; the tile then spans kG times as many z rows.
// The group width is a compile-time constant, so LDS offsets other than the
// lane's own part fold into the instructions' immediate offsets.
// In both, the lowest and highest z rows of the tile are ring rows whose
// results only feed their neighbours.  Lane moves (DPP) cross group
// boundaries only in halo lanes, whose results are never used; lanes past the
// last group repeat its last lane.  Returns the lane's moving-frame vote.
template <int kG>
constexpr int group_lanes() { return kG == 1 ? 64 : (kG == 3 ? 21 : 16); }

template <typename T, bool kFrozen, bool kReduce, bool kMulti, bool kShell3, int kG>
__device__ __forceinline__ bool step3d_tile(const Step3DArgs<T> &a, int strip, int zt, int segi,
                                            unsigned char *smem_raw) {
  using M = Math<T>;
  const Coef<T> &c = a.c;
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int nwv = (int)(blockDim.x >> 6);
  constexpr bool kWide = kG == 1;
  constexpr int GL = group_lanes<kG>();   // lanes per group
  constexpr int g = kG;                   // groups (z rows) per wave
  constexpr int RS = GL + 2;              // LDS row stride: lane l at l + 1, pads at 0 and GL + 1
  const int NW = nwv * g;                 // z rows of the tile, ring rows included
  const int Z = NW - 2, NZR = Z + 4;
  const int SLOT = NZR * RS;
  // Field rings, 5 row slots of NZR z layers, stored [slot][layer][field][lane]
  // so that the four fields of one (row, layer) sit at fixed offsets from one
  // another and share one address computation.
  T *XL = sm + 4 * 5 * SLOT;  // link exchange [row parity][to above, to below][z row][lane]
  T *FZ = XL + 4 * NW * GL;   // z-up face flux of each z row [z row][lane]
  int8_t *gL = reinterpret_cast<int8_t *>(FZ + NW * GL);  // grains, 5 row slots

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int grp = 0, lx = lane;
  if (!kWide) {
    grp = min(lane / GL, g - 1);
    lx = min(lane - grp * GL, GL - 1);
  }
  const bool valid = kWide || lane < g * GL;
  const int zr = kWide ? w : w * g + grp;  // z row within the tile
  const int wout = kWide ? a.wout : a.thin_wout;
  const int x = (kWide ? strip * a.wout : a.nstrips * a.wout) - 2 + lx;
  const int gx = ghost(x, nx, a.bcx);
  const bool out_lane = valid && lx >= 2 && lx < 2 + wout && x < nx;
  const int z0 = zt * Z;
  const int z = z0 - 1 + zr;
  const int zi = zr + 1;
  const bool out_wave = zr >= 1 && zr <= Z && z < nz;  // uniform over a wave in wide tiles
  const bool ring = (zr == 0) || (zr == Z + 1);
  const int zh = (zr == 0) ? z0 - 2 : z0 + Z + 1;
  const int zih = (zr == 0) ? 0 : Z + 3;
  const size_t plane = (size_t)nx * (size_t)ny;
  const size_t pz = (size_t)ghost(z, nz, a.bcz) * plane + (size_t)gx;
  const size_t pzh = (size_t)ghost(zh, nz, a.bcz) * plane + (size_t)gx;
  const size_t pzd = (size_t)ghost(z - 1, nz, a.bcz) * plane + (size_t)gx;
  // the rows of a column are split evenly between its segments (thin
  // columns have their own, shorter segments)
  const int segbase = kWide ? a.segbase : a.thin_segbase;
  const int segrem = kWide ? a.segrem : a.thin_segrem;
  const int y0 = segi * segbase + min(segi, segrem);
  const int ye = y0 + segbase + (segi < segrem ? 1 : 0);

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
  // slot of the row k rows below the row in slot s
  auto back = [](int s, int k) { return s >= k ? s - k : s + 5 - k; };
  // LDS index of field f at row slot s in z layer zi + dz, this lane's column:
  // the lane's part of the index is computed once (thin tiles have a z row
  // per lane group)
  const int LAY = 4 * RS;              // elements per z layer of a slot
  const int SLOTF = NZR * LAY;         // elements per row slot
  const int zoc = zi * LAY + lx + 1;
  auto at = [&](int f, int s, int dz) -> int { return s * SLOTF + f * RS + dz * LAY + zoc; };
  auto rot_of = [&](int g) -> Rot3<T> {
    Rot3<T> R;
    const T *q = kMulti ? a.rot + 9 * g : a.R;
#pragma unroll
    for (int i = 0; i < 9; ++i) R.m[i] = q[i];
    return R;
  };
  // LDS element of field f at row slot s, z layer zz, lane offset dx
  auto L = [&](int f, int s, int dz, int dx) -> T { return sm[at(f, s, dz) + dx]; };

  // Divergence neighbourhoods: a z-row or y-row beyond a no-flux wall is read
  // as its mirror image (alpha_A included, which the ring waves cannot
  // produce for a mirrored row).  Layers are clamped to the LDS tile: only
  // waves whose results are unused can reach the clamp.
  auto zlayer = [&](int zz) -> int {
    if (a.bcz == PF_BC_NOFLUX) {
      if (zz < 0) zz = -zz - 1;
      else if (zz >= nz) zz = 2 * nz - 1 - zz;
    }
    return min(max(zz - z0 + 2, 0), NZR - 1);
  };
  const int zl[3] = {zlayer(z - 1), zlayer(z), zlayer(z + 1)};
  const int zlo[3] = {zl[0] * LAY + lx + 1, zl[1] * LAY + lx + 1, zl[2] * LAY + lx + 1};
  const int gzo = zi * RS + lx + 1;  // the same for the int8 grain ring (no field axis)
  auto yslot = [&](int j) {
    if (a.bcy == PF_BC_NOFLUX) {
      if (j < 0) j = -j - 1;
      else if (j >= ny) j = 2 * ny - 1 - j;
    }
    return slot5(j);
  };

  // own-row window (rows r-2, r-1, r) and carries
  T pS = 0, pC = 0, pN = 0, uS = 0, uC = 0, uN = 0, fS = 0, fC = 0, fN = 0;
  T aAq = 0, aAm = 0;      // alpha_A of own cell at rows m-1 and m
  T FyS = 0;               // y face flux below row r-1
  int gS = 0, gC = 0, gN = 0;
  // shared divergence links: P_y of the next row (fields D, A), the south
  // links of the row (N, NE, NW of the row below), this wave's NU and ND of
  // the row below (sent to the neighbouring waves one row late), and the row
  // waiting for its neighbours' links (U, the own part of the update, 1/den)
  T PyD = 0, PyA = 0, southSum = 0, NUprev = 0, NDprev = 0;
  T waitU = 0, waitBase = 0, waitDen = 0;

  T nxt_p, nxt_u, nxt_h = 0;
  int nxt_g = 0;
  // slot of the row the next iteration publishes, advanced by one per
  // iteration (the slots of the rows below follow from it without a division)
  int sr = slot5(y0 - 2);
  {
    size_t ro = rowoff(y0 - 2);
    nxt_p = a.psi_in[pz + ro];
    nxt_u = a.U_in[pz + ro];
    if (ring) nxt_h = a.psi_in[pzh + ro];
    if (kMulti) nxt_g = a.grain[pz + ro];
  }

  // U of the waiting row qf from its own part and the neighbours' links
  // (output rows only: their neighbours zr - 1 and zr + 1 exist in the tile)
  auto finalize = [&](int qf) {
    if (!out_wave) return;
    const int par = qf & 1;
    const T below = XL[((par * 2 + 0) * NW + (zr - 1)) * GL + lx];
    const T above = XL[((par * 2 + 1) * NW + (zr + 1)) * GL + lx];
    store_row(a.U_out + (pz - (size_t)gx) + (size_t)qf * nx, nx, x, out_lane,
               waitU + c.dt * waitDen * (waitBase - below - above));
  };

  auto iter = [&](auto phase, int r) {
    constexpr int P = decltype(phase)::value;
    // ---------------- phase A: publish row r
    pS = pC; pC = pN; uS = uC; uC = uN; fS = fC; fC = fN; gS = gC; gC = gN;
    pN = nxt_p; uN = nxt_u; gN = nxt_g;
    const T hN = nxt_h;
    {
      // the last iteration reloads row ye + 1 (never consumed) rather than
      // branching around the loads
      size_t ro = rowoff(min(r + 1, ye + 1));
      nxt_p = a.psi_in[pz + ro];
      nxt_u = a.U_in[pz + ro];
      if (ring) nxt_h = a.psi_in[pzh + ro];
      if (kMulti) nxt_g = a.grain[pz + ro];
    }
    const int sN = sr;
    sr = sN == 4 ? 0 : sN + 1;
    const int oN = at(kPsi, sN, 0);
    // phi and alpha_D of row r are first read by the links of the next
    // iteration: phi is formed after the psi phase's first LDS reads are
    // issued, while they are in flight, and alpha_D stored after them (the
    // empty asm statements hold that order against the compiler's hoisting
    // and sinking).  With <111> links (more reads in flight) that order ran
    // slower, so there both are formed here, before the barrier.
    constexpr bool kLatePhi = !kShell3;
    auto form_fN = [&]() {
      T pNb = pN;
      if constexpr (kLatePhi) asm volatile("" : "+v"(pNb));
      fN = M::tanh_(pNb * isq2);
      if constexpr (kLatePhi) asm volatile("" : "+v"(fN));
    };
    auto publish_aD = [&]() { sm[oN + (kAD - kPsi) * RS] = c.D * (T(1) - fN); };
    sm[oN] = pN;
    sm[oN + (kU - kPsi) * RS] = uN;
    if (kMulti) gL[sN * NZR * RS + gzo] = (int8_t)gN;
    if (ring) sm[sN * SLOTF + zih * LAY + lx + 1] = hN;
    if constexpr (!kLatePhi) {
      form_fN();
      publish_aD();
    }
    // The psi phase's neighbourhood in rows r-2 and r-1 (its rows m-1 and m)
    // was published in earlier iterations: part of it is read before the
    // barrier, whose wait then covers those reads.  Row m always; row m-1
    // too with <111> links (18 of the 27 points).  Without them, reading row
    // m-1 early as well ran slower than row m alone.
    constexpr int kEarlyFrom = kShell3 ? -1 : 0;  // rows dy = kEarlyFrom .. 0
    T Pn[27];
    if constexpr (P >= 2) {
      const int syb[2] = {back(sN, 2), back(sN, 1)};
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = kEarlyFrom; dy <= 0; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            if (!kShell3 && dx != 0 && dy != 0 && dz != 0) continue;  // corners unused
            Pn[nb(dx, dy, dz)] = L(kPsi, syb[dy + 1], dz, dx);
          }
    }
    __syncthreads();
    if constexpr (P == 0) {
      if constexpr (kLatePhi) {
        form_fN();
        publish_aD();
      }
      __syncthreads();
      return;
    }
    const int m = r - 1;
    const int s0 = back(sN, 1), sp1 = sN;

    if constexpr (P == 1) {
      // only the y face between rows m and m+1 (lower cell (x, m, z)), in
      // the same form as the steady state's north face
      const T cx0 = L(kPsi, s0, 0, 1) - L(kPsi, s0, 0, -1);
      const T cx1 = L(kPsi, sp1, 0, 1) - L(kPsi, sp1, 0, -1);
      const T cz0 = L(kPsi, s0, 1, 0) - L(kPsi, s0, -1, 0);
      const T cz1 = L(kPsi, sp1, 1, 0) - L(kPsi, sp1, -1, 0);
      FyS = aniso3<T, 1>(cx0 + cx1, T(4) * (L(kPsi, sp1, 0, 0) - L(kPsi, s0, 0, 0)), cz0 + cz1,
                         rot_of(gC), c, c.f3_eps);
      if constexpr (kLatePhi) {
        form_fN();
        publish_aD();
      }
      __syncthreads();
      return;
    } else {
      // ---------------- phase B: psi rate at row m from the LDS neighbourhood
      // (the rows not read before the barrier; row m+1 = r)
      const int sy[3] = {back(sN, 2), s0, sp1};
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            if (dy >= kEarlyFrom && dy <= 0) continue;  // read before the barrier
            if (!kShell3 && dx != 0 && dy != 0 && dz != 0) continue;  // corners unused
            Pn[nb(dx, dy, dz)] = L(kPsi, sy[dy + 1], dz, dx);
          }
      if constexpr (kLatePhi) form_fN();
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
      // central differences (2h g at the centre); the face gradients below
      // are 4h g: the normal difference times 4 and, for each tangential
      // axis, the sum of the central differences of the two cells
      const T cx = Pn[nb(1, 0, 0)] - Pn[nb(-1, 0, 0)];
      const T cy = Pn[nb(0, 1, 0)] - Pn[nb(0, -1, 0)];
      const T cz = Pn[nb(0, 0, 1)] - Pn[nb(0, 0, -1)];
      T ac = aniso3<T, -1>(cx, cy, cz, R, c, c.ac_eps);
      // x face east of the cell (the right lane's differences by DPP)
      T FxE = aniso3<T, 0>(T(4) * (Pn[nb(1, 0, 0)] - p0), cy + from_right(cy),
                           cz + from_right(cz), R, c, c.f3_eps);
      T FxW = from_left(FxE);
      // y face north of the cell
      T FyN = aniso3<T, 1>(cx + (Pn[nb(1, 1, 0)] - Pn[nb(-1, 1, 0)]),
                           T(4) * (Pn[nb(0, 1, 0)] - p0),
                           cz + (Pn[nb(0, 1, 1)] - Pn[nb(0, 1, -1)]), R, c, c.f3_eps);
      // z face above (own grain); the face below is the wave below's face
      // above (the same points in the same order, the grain of the lower
      // cell), read after a barrier; the lowest wave computes its own
      T FzU = aniso3<T, 2>(cx + (Pn[nb(1, 0, 1)] - Pn[nb(-1, 0, 1)]),
                           cy + (Pn[nb(0, 1, 1)] - Pn[nb(0, -1, 1)]),
                           T(4) * (Pn[nb(0, 0, 1)] - p0), R, c, c.f3_eps);
      FZ[zr * GL + lx] = FzU;
      T FzD;
      if (w == 0) {
        Rot3<T> Rd = R;
        if (kMulti) Rd = rot_of(a.grain[pzd + rowoff(m)]);
        FzD = aniso3<T, 2>((Pn[nb(1, 0, -1)] - Pn[nb(-1, 0, -1)]) + cx,
                           (Pn[nb(0, 1, -1)] - Pn[nb(0, -1, -1)]) + cy,
                           T(4) * (p0 - Pn[nb(0, 0, -1)]), Rd, c, c.f3_eps);
      }
      __syncthreads();
      if (zr != 0) FzD = FZ[(zr - 1) * GL + lx];
      const T ac2 = ac * ac;
      // the standard Laplacian of the remainder is the <100> sum s1 / h^2
      T Nn = (FxE - FxW + FyN - FyS + FzU - FzD) * c.f3_scale - ac2 * (s1 * c.cStd);
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
      sm[at(kAA, s0, 0)] = aA;
      if constexpr (kLatePhi) publish_aD();
      aAq = aAm;
      aAm = aA;
      // dynamic grains: the grain of row m at the next level (a liquid cell,
      // psi < 0, with a solid face neighbour takes the grain of the solid
      // neighbour with the largest psi, first of -x, +x, -y, +y, -z, +z)
      if constexpr (kMulti) {
        if (a.grain_out != nullptr && P >= 3 && m < ye) {
          const int gW = from_left(gC), gE = from_right(gC);
          int gn = gC;
          if (p0 < T(0)) {
            T best = T(0);
            bool found = false;
            auto take = [&](T v, int g) {
              if (v >= T(0) && (!found || v > best)) {
                best = v;
                gn = g;
                found = true;
              }
            };
            take(Pn[nb(-1, 0, 0)], gW);
            take(Pn[nb(1, 0, 0)], gE);
            take(Pn[nb(0, -1, 0)], gS);
            take(Pn[nb(0, 1, 0)], gN);
            take(Pn[nb(0, 0, -1)], (int)gL[s0 * NZR * RS + gzo - RS]);
            take(Pn[nb(0, 0, 1)], (int)gL[s0 * NZR * RS + gzo + RS]);
          }
          if (out_wave && out_lane)
            a.grain_out[pz + (size_t)m * nx - (size_t)gx + (size_t)x] = (int8_t)gn;
        }
      }
      if (P >= 3 && m < ye && out_wave) {
        store_row(a.psi_out + (pz - (size_t)gx) + (size_t)m * nx, nx, x, out_lane, pC + c.dt * rate);
        // moving-frame vote as a mask: rows at or above the shift row
        // qualify outright; the crossing height of the row under it is
        // taken in FP64 once, after the rows
        if (kReduce)
          over = over | (out_lane & (m >= a.shift_row) & (m <= ny - 2) & (fC >= T(0)) & (fN < T(0)));
      }
    }
    // ---------------- phase C's operands that this iteration's alpha_A does
    // not feed (psi, U and alpha_D of rows q-1 .. q+1, q = m - 1, all
    // published before the first barrier): read before the last barrier, so
    // that after it only the alpha_A reads are waited on.  (At P == 3, whose
    // q = y0 - 1 can lie below a no-flux wall with row q-1's image at row r,
    // nothing of row q-1 is read.)
    const int q = m - 1;
    int sl[3] = {0, 0, 0};
    if constexpr (P >= 3) {
      if (a.bcy != PF_BC_NOFLUX || (q >= 1 && q <= ny - 2)) {
        sl[0] = back(sN, 3);  // rows q-1, q, q+1 = r-3, r-2, r-1
        sl[1] = back(sN, 2);
        sl[2] = back(sN, 1);
      } else {
        sl[0] = yslot(q - 1);
        sl[1] = yslot(q);
        sl[2] = yslot(q + 1);
      }
    }
    auto rd = [&](int f, int dy, int dz, int dx) -> T {
      return sm[sl[dy + 1] * SLOTF + f * RS + zlo[dz + 1] + dx];
    };
    constexpr bool kFull = P == 4;
    auto abars = [&](int AL, T Pyq) -> Abar9<T> {
      Abar9<T> o;
      const T a00 = rd(AL, 0, 0, 0), a10 = rd(AL, 1, 0, 0);
      const T a0m = rd(AL, 0, -1, 0), a0p = rd(AL, 0, 1, 0);
      const T a1m = rd(AL, 1, -1, 0), a1p = rd(AL, 1, 1, 0);
      o.Py1 = c.k1a * a10 + c.k1b * (rd(AL, 1, 0, -1) + rd(AL, 1, 0, 1) + a1m + a1p);
      o.N = Pyq + o.Py1;
      // xy plaquettes {x, x+1} x {q, q+1} at z-1, z, z+1
      const T cm = a0m + a1m, c0 = a00 + a10, cp = a0p + a1p;
      const T Xm = cm + from_right(cm), X0 = c0 + from_right(c0), Xp = cp + from_right(cp);
      o.NE = c.k2a * X0 + c.k2b * (Xm + Xp);
      o.NW = from_left(o.NE);
      // yz plaquettes {q, q+1} x {z, z+1} (NU) and {z-1, z} (ND) at x-1, x, x+1
      const T S = c0 + cp, Sd = cm + c0;
      o.NU = c.k2a * S + c.k2b * (from_left(S) + from_right(S));
      o.ND = c.k2a * Sd + c.k2b * (from_left(Sd) + from_right(Sd));
      if constexpr (kShell3) {
        // the cube {x, x+1} x {q, q+1} x {z, z+1} is two stacked plaquettes
        o.Tpp = c.k3 * (X0 + Xp);
        o.Tpm = c.k3 * (X0 + Xm);
        o.Tmp = from_left(o.Tpp);
        o.Tmm = from_left(o.Tpm);
      } else {
        o.Tpp = o.Tpm = o.Tmp = o.Tmm = T(0);
      }
      if constexpr (kFull) {
        const T am0 = rd(AL, -1, 0, 0), am1 = rd(AL, -1, 1, 0);
        const T Px = c.k1a * a00 + c.k1b * (am0 + a10 + a0m + a0p);
        o.E = Px + from_right(Px);
        const T Pz0 = c.k1a * a00 + c.k1b * (rd(AL, 0, 0, -1) + rd(AL, 0, 0, 1) + am0 + a10);
        const T Pz1 = c.k1a * a0p + c.k1b * (rd(AL, 0, 1, -1) + rd(AL, 0, 1, 1) + am1 + a1p);
        o.Up = Pz0 + Pz1;
        // xz plaquettes {x, x+1} x {z, z+1} at q-1, q, q+1
        const T ym = am0 + am1, y0s = a00 + a0p, yp = a10 + a1p;
        const T Ym = ym + from_right(ym), Y0 = y0s + from_right(y0s), Yp = yp + from_right(yp);
        o.EU = c.k2a * Y0 + c.k2b * (Ym + Yp);
        o.WU = from_left(o.EU);
      } else {
        o.E = o.Up = o.EU = o.WU = T(0);
      }
      return o;
    };
    auto diffs = [&](int BL) -> Diff9<T> {
      Diff9<T> o;
      const T b0 = rd(BL, 0, 0, 0);
      o.N = rd(BL, 1, 0, 0) - b0;
      o.NE = rd(BL, 1, 0, 1) - b0;
      o.NW = rd(BL, 1, 0, -1) - b0;
      o.NU = rd(BL, 1, 1, 0) - b0;
      o.ND = rd(BL, 1, -1, 0) - b0;
      if constexpr (kShell3) {
        o.Tpp = rd(BL, 1, 1, 1) - b0;
        o.Tmp = rd(BL, 1, 1, -1) - b0;
        o.Tpm = rd(BL, 1, -1, 1) - b0;
        o.Tmm = rd(BL, 1, -1, -1) - b0;
      } else {
        o.Tpp = o.Tmp = o.Tpm = o.Tmm = T(0);
      }
      if constexpr (kFull) {
        o.E = rd(BL, 0, 0, 1) - b0;
        o.Up = rd(BL, 0, 1, 0) - b0;
        o.EU = rd(BL, 0, 1, 1) - b0;
        o.WU = rd(BL, 0, 1, -1) - b0;
      } else {
        o.E = o.Up = o.EU = o.WU = T(0);
      }
      return o;
    };
    // P_y of row q itself: carried from the row below except at the start
    auto py_here = [&](int AL) -> T {
      return c.k1a * rd(AL, 0, 0, 0) +
             c.k1b * (rd(AL, 0, 0, -1) + rd(AL, 0, 0, 1) + rd(AL, 0, -1, 0) + rd(AL, 0, 1, 0));
    };
    Diff9<T> dU{}, dP{};
    Abar9<T> bD{};
    if constexpr (P >= 3) {
      dU = diffs(kU);
      dP = diffs(kPsi);
      if constexpr (!kFull) PyD = py_here(kAD);
      bD = abars(kAD, PyD);
    }
    __syncthreads();

    if constexpr (P >= 3) {
      // ---------------- phase C: the links this wave owns at row q
      // (P == 3: only those towards row q+1, which the first U row needs)
      if constexpr (!kFull) PyA = py_here(kAA);
      const Abar9<T> bA = abars(kAA, PyA);
      PyD = bD.Py1;
      PyA = bA.Py1;
      // link values: D~ abar_D dU + abar_A dpsi (D~ is inside alpha_D)
      const T fN_ = bD.N * dU.N + bA.N * dP.N;
      const T fNE = bD.NE * dU.NE + bA.NE * dP.NE;
      const T fNW = bD.NW * dU.NW + bA.NW * dP.NW;
      const T fNU = bD.NU * dU.NU + bA.NU * dP.NU;
      const T fND = bD.ND * dU.ND + bA.ND * dP.ND;
      // <111> links towards +y; the wave above takes (-1,+1,+1) of lane x+1 and
      // (+1,+1,+1) of lane x-1 as its south-down links, the wave below the
      // (.,+1,-1) pair alike (both one row late)
      T f111 = T(0), up111 = T(0), dn111 = T(0);
      if constexpr (kShell3) {
        const T fpp = bD.Tpp * dU.Tpp + bA.Tpp * dP.Tpp;
        const T fmp = bD.Tmp * dU.Tmp + bA.Tmp * dP.Tmp;
        const T fpm = bD.Tpm * dU.Tpm + bA.Tpm * dP.Tpm;
        const T fmm = bD.Tmm * dU.Tmm + bA.Tmm * dP.Tmm;
        f111 = (fpp + fmp) + (fpm + fmm);
        up111 = from_right(fmp) + from_left(fpp);
        dn111 = from_right(fmm) + from_left(fpm);
      }
      if constexpr (kFull) {
        const T fE = bD.E * dU.E + bA.E * dP.E;
        const T fUp = bD.Up * dU.Up + bA.Up * dP.Up;
        const T fEU = bD.EU * dU.EU + bA.EU * dP.EU;
        const T fWU = bD.WU * dU.WU + bA.WU * dP.WU;
        // links the waves above and below take with the opposite sign
        const int par = q & 1;
        XL[((par * 2 + 0) * NW + zr) * GL + lx] = fUp + from_left(fEU) + from_right(fWU) + NUprev;
        XL[((par * 2 + 1) * NW + zr) * GL + lx] = NDprev;
        T own = ((fE + fN_) + (fUp + fNE)) + ((fNW + fEU) + (fWU + fNU)) + fND + f111;
        T part = own - from_left(fE) - southSum;
        // finish the row below with its neighbours' links (published one
        // iteration ago), then let row q wait
        if (q - 1 >= y0) finalize(q - 1);
        waitU = uS;
        waitBase = part + sq2 * aAq;
        waitDen = M::rcp(T(1) + c.k - c.omk * fS);
      }
      southSum = fN_ + from_left(fNE) + from_right(fNW);
      NUprev = fNU + up111;
      NDprev = fND + dn111;
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
  // the last row's neighbours published their links in the last iteration
  __syncthreads();
  finalize(ye - 1);

  if (kReduce && out_wave) {
    const int ms = a.shift_row - 1;  // the row under the shift row
    if (ms >= y0 && ms < ye && ms <= ny - 2) {
      const T f0 = M::tanh_(a.psi_in[pz + rowoff(ms)] * isq2);
      const T f1 = M::tanh_(a.psi_in[pz + rowoff(ms + 1)] * isq2);
      if (out_lane && f0 >= T(0) && f1 < T(0))
        over |= crossing_reaches(f0, f1, ms, a.shift_row, ythr, a.hd);
    }
  }
  return over;
}

template <typename T, bool kFrozen, bool kReduce, bool kMulti, bool kShell3>
__global__ __launch_bounds__(max_threads3d<T>()) void step3d_kernel(Step3DArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // Wide tiles first, segment by segment (strip fastest, then z tile), then
  // the thin strip's tiles likewise (thin tiles have their own, shorter
  // segments: their rows cost more)
  const int lb = xcd_remap3((int)blockIdx.x, (int)gridDim.x);
  const int nwide = a.ncols_wide * a.nsegs;
  bool over;
  if (lb < nwide) {
    const int segi = lb / a.ncols_wide;
    const int col = lb - segi * a.ncols_wide;
    over = step3d_tile<T, kFrozen, kReduce, kMulti, kShell3, 1>(a, col % a.nstrips,
                                                               col / a.nstrips, segi, smem_raw);
  } else {
    const int t = lb - nwide;
    const int segi = t / a.thin_nzt;
    const int zt = t - segi * a.thin_nzt;
    if (a.thin_g == 3)
      over = step3d_tile<T, kFrozen, kReduce, kMulti, kShell3, 3>(a, 0, zt, segi, smem_raw);
    else
      over = step3d_tile<T, kFrozen, kReduce, kMulti, kShell3, 4>(a, 0, zt, segi, smem_raw);
  }
  if (kReduce) {
    const bool any = __any(over);
    const int lane = threadIdx.x & 63;
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
  g.ztile = ztile < 1 ? 1 : (ztile > 14 ? 14 : ztile);
  const int nw = g.ztile + 2;
  // strips of 60 output columns; the last nx mod 60 columns form a thin
  // strip of lane groups when three (21 lanes, up to 17 columns) or four (16
  // lanes, up to 12 columns) groups fit a wave, else the strips share the
  // columns evenly
  const int nfull = nx / 60, r = nx - 60 * nfull;
  const int gr = r == 0 ? 0 : (r <= 12 ? 4 : (r <= 17 ? 3 : 1));
  g.thin_g = 0;
  g.thin_G = 0;
  g.thin_wout = 0;
  g.thin_nzt = 0;
  if (r == 0 || gr >= 3) {
    g.nstrips = nfull;
    g.wout = 60;
    if (r > 0) {
      g.thin_g = gr;
      g.thin_G = gr == 3 ? 21 : 16;
      g.thin_wout = r;
      const int zt_thin = nw * gr - 2;
      g.thin_nzt = (nz + zt_thin - 1) / zt_thin;
    }
  } else {
    g.nstrips = (nx + 59) / 60;
    g.wout = (nx + g.nstrips - 1) / g.nstrips;
  }
  g.nzt = (nz + g.ztile - 1) / g.ztile;
  g.ncols_wide = g.nstrips * g.nzt;
  g.ncols = g.ncols_wide + g.thin_nzt;
  g.seg = seg < 1 ? 1 : seg;
  g.nsegs = (ny + g.seg - 1) / g.seg;
  g.segbase = ny / g.nsegs;
  g.segrem = ny - g.segbase * g.nsegs;
  // a thin tile's row costs more than a wide one's (its LDS addresses have a
  // per-lane part and its three or four z rows share each wave), so its
  // segments are 3/4 as long
  const int seg_thin = g.seg * 3 / 4 < 1 ? 1 : g.seg * 3 / 4;
  g.thin_nsegs = g.thin_nzt > 0 ? (ny + seg_thin - 1) / seg_thin : 0;
  g.thin_segbase = g.thin_nsegs > 0 ? ny / g.thin_nsegs : 0;
  g.thin_segrem = g.thin_nsegs > 0 ? ny - g.thin_segbase * g.thin_nsegs : 0;
  g.threads = 64 * nw;
  g.blocks = g.ncols_wide * g.nsegs + g.thin_nzt * g.thin_nsegs;
  return g;
}

size_t step3d_lds_bytes(int nx, int ztile, size_t elem) {
  // four 5-row rings of (z rows + 2) z layers, the link exchange, the z-face
  // fluxes, and a 5-row int8 ring of grains; the larger of a wide tile's
  // and a thin tile's
  const Geom3D g = geom3d(nx, 8, 8, 8, ztile);
  const size_t nw = (size_t)g.ztile + 2;
  size_t wide = ((size_t)20 * (nw + 2) * (size_t)kRS + (size_t)5 * nw * 64) * elem +
                (((size_t)5 * (nw + 2) * (size_t)kRS + 15) & ~(size_t)15);
  size_t thin = 0;
  if (g.thin_g > 0) {
    const size_t NW = nw * (size_t)g.thin_g, RS = (size_t)g.thin_G + 2;
    thin = ((size_t)20 * (NW + 2) * RS + (size_t)5 * NW * (size_t)g.thin_G) * elem +
           (((size_t)5 * (NW + 2) * RS + 15) & ~(size_t)15);
  }
  return wide > thin ? wide : thin;
}

// Launch one instantiation; workgroups above 64 KB of LDS need the kernel's
// dynamic-LDS limit raised once per device (gfx950 allows up to 160 KB per
// workgroup).  Safe to call from several host threads.
constexpr int kMaxDevices = 64;
template <typename T, bool F, bool R, bool MU, bool S3>
hipError_t launch3(const Step3DArgs<T> &a, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
  // dynamic-LDS limit already raised for this instantiation, per device
  static std::atomic<size_t> allowed[kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (lds > 65536 && lds > allowed[dev].load(std::memory_order_relaxed)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step3d_kernel<T, F, R, MU, S3>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    size_t cur = allowed[dev].load(std::memory_order_relaxed);
    while (cur < lds && !allowed[dev].compare_exchange_weak(cur, lds)) {
    }
  }
  hipLaunchKernelGGL((step3d_kernel<T, F, R, MU, S3>), grid, block, lds, st, a);
  return hipSuccess;
}

template <typename T>
hipError_t launch_step3d(const Step3DArgs<T> &a, const Geom3D &g, bool frozen, bool reduce,
                         bool multi, hipStream_t st) {
  dim3 grid(g.blocks), block(g.threads);
  size_t lds = step3d_lds_bytes(a.nx, g.ztile, sizeof(T));
  const bool shell3 = a.c.cD3 != T(0) || a.c.cL3 != T(0) || a.c.cG3 != T(0);
  hipError_t e = hipSuccess;
#define PF_L3(F, R, MU, S3) e = launch3<T, F, R, MU, S3>(a, grid, block, lds, st)
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
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template hipError_t launch_step3d<float>(const Step3DArgs<float> &, const Geom3D &, bool, bool,
                                         bool, hipStream_t);
template hipError_t launch_step3d<double>(const Step3DArgs<double> &, const Geom3D &, bool, bool,
                                          bool, hipStream_t);

}  // namespace pf
