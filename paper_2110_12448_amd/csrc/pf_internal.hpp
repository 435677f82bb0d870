// pf_internal.hpp -- host/device shared definitions of the phase-field
// library: kernel argument blocks, device-resident frame and tip records,
// and the launchers the C ABI calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pf.h"

namespace pf {

// Moving-frame record of one time level, device resident.  The rows the
// frame has moved for this level are base + pending; pending = 1 means the
// stored arrays still owe one downward shift, applied when they are next
// read.  Step n reads record n % 3, publishes base and ORs pending into record
// (n+1) % 3, and clears pending of record (n+2) % 3 for step n+1: no grid-wide
// synchronisation or fence is needed inside a step.
struct alignas(16) FrameState {
  long long base;
  int pending;
  int pad;
};

// Result of a grid-wide tip / solid-fraction / finiteness reduction, with a
// copy of the frame record the reduction read (zero when it was given none;
// written by the main pass, the rest by the combining launch), so that one
// copy to the host returns both.
struct alignas(16) TipResult {
  double y;          // crossing height in the frame, valid when found
  long long idx;     // linear frame index of the cell below the crossing
  double fs_sum;     // sum over cells of (1 + phi)/2
  unsigned bad;      // number of non-finite psi or U values
  int found;
  FrameState frame;
};

struct TipAcc;  // per-block partial (tip_device.hpp)

// Workspace pieces of the reduction: one partial per workgroup and the
// result record.
struct Reduce {
  TipAcc *partials;
  TipResult *result;
};

// Physical constants of one step, precomputed on the host in FP64 and cast
// to the working precision T.
template <typename T>
struct Coef {
  T dt, k, omk, eps4, D, lambda;
  T an0, an4, an16;  // 1 - 3 eps4, 4 eps4, 16 eps4 (cubic a_s and its torque)
  T inv_h;          // 1/h
  T cL1, cL2, cL3;  // shell weights of L over their prefactors
  T cG1, cG2, cG3;  // shell weights of G over their prefactors
  T cD1, cD2, cD3;  // shell weights of the divergence over their prefactors
  T cStd;           // 1/h^2 (standard Laplacian of the eps4 remainder)
  T inv_lT;         // 1/lT (frozen temperature)
  T h;
  T cT;             // two-point <10> faces: 1/(2h^2) (2D)
  T at_eps;         // 1e-12 h^2: the |g|^2 <= 1e-12 guard for h g (face gradients, 2D)
  T ac_eps;         // 4e-12 h^2: the same guard for 2h g (centre differences)
  T an1, an8;       // 1 + eps4, 8 eps4 (2D a_s = 1 + eps4 - 8 eps4 u^2 v^2)
  T k1a, k1b;       // cD1/4, cD1/16: <100> link alpha weights times the shell coefficient (3D)
  T k2a, k2b;       // 3 cD2/16, cD2/32: the same for <110> links (3D)
  T k3;             // cD3/8: <111> links, mean of the 8 cube corners (3D)
  T f3_eps;         // 16e-12 h^2: the |g|^2 <= 1e-12 guard for 4h g (face gradients, 3D)
  T f3_scale;       // 1/(4 h^2): unscales the sum of the 4h-scaled face fluxes (3D)
};

template <typename T>
struct Step2DArgs {
  const T *psi_in, *U_in;
  T *psi_out, *U_out;
  const int8_t *grain;   // multi-grain only
  int8_t *grain_out;     // dynamic grains only: grain map of the next level
  const T *rot;          // multi-grain only: 4 per grain (r00, r01, r10, r11)
  T r00, r01, r10, r11;  // single grain
  int nx, ny, bcx, bcy;
  int wout, nstrips, nsegs, segbase, segrem;
  Coef<T> c;
  double hd, y0, Vp, dtd;
  long long step;
  int frame, shift_row;
  const FrameState *frame_in;
  FrameState *frame_out, *frame_clear;
};

// One solve of a batched 2D launch: its argument block plus both buffer
// pairs, its three frame records and the epoch origin (level n0, buffer
// parity and frame-record index at launch k = 0).
template <typename T>
struct BatchSolve2D {
  Step2DArgs<T> a;
  T *psi[2];
  T *U[2];
  FrameState *frames[3];
  long long n0;
  int par0, f0;
};

template <typename T>
struct Step3DArgs {
  const T *psi_in, *U_in;
  T *psi_out, *U_out;
  const int8_t *grain;   // multi-grain only
  int8_t *grain_out;     // dynamic grains only: grain map of the next level
  const T *rot;          // 9 per grain, row-major crystal -> lab
  T R[9];                // single grain
  int nx, ny, nz, bcx, bcy, bcz;
  int wout, nstrips, nzt, nsegs, seg, ztile;
  int segbase, segrem;          // rows of a segment: segbase, one more for the first segrem
  int ncols, ncols_wide;        // tile columns (strip, z tile), wide ones first
  int thin_g, thin_G, thin_wout;  // thin strip: lane groups per wave, lanes per group, width
  int thin_nzt, thin_segbase, thin_segrem;  // its z tiles and segments
  Coef<T> c;
  double hd, y0, Vp, dtd;
  long long step;
  int frame, shift_row;
  const FrameState *frame_in;
  FrameState *frame_out, *frame_clear;
};

template <typename T>
struct ReduceArgs {
  const T *psi, *U;
  int nx, ny, nz;
  int rows;                 // rows per column walk (reduce_geometry)
  double hd;
  const FrameState *frame;  // pending shift of the arrays read, or NULL:
  int pending;              // then this host value is used
  Reduce red;
};

// Launch geometry of the 2D step: wave64 strips of up to 60 output columns
// and, per strip, ceil(ny / seg) segments for seg > 0, or for seg = -k as
// many as give k waves per SIMD over ncu compute units (at most ny); the rows
// are split evenly (segbase rows each, one more for the first segrem).
struct Geom2D {
  int wout, nstrips, nsegs, seg, segbase, segrem, blocks;
};
Geom2D geom2d(int nx, int ny, int seg, int ncu = 0);

// Launch geometry of the 3D step: nstrips strips of wout output columns
// (wide tiles, one z row per wave) and, when at most 17 of nx mod 60 columns
// remain, a thin strip of thin_g = 3 or 4 groups of thin_G = 21 or 16 lanes
// per wave (thin_nzt z tiles); ztile z rows per wide workgroup of ztile + 2
// waves; each column's ny rows split evenly between nsegs segments of at
// most seg rows (thin columns: thin_nsegs of at most 3/4 of that).
struct Geom3D {
  int wout, nstrips, ztile, nzt, nsegs, seg, segbase, segrem, blocks, threads;
  int thin_g, thin_G, thin_wout, thin_nzt, ncols_wide, ncols;
  int thin_nsegs, thin_segbase, thin_segrem;
};
Geom3D geom3d(int nx, int ny, int nz, int seg, int ztile);
size_t step3d_lds_bytes(int nx, int ztile, size_t elem);

size_t tip_acc_bytes();
// Launch geometry of the reduction: rows per column walk and workgroups
// (at most kMaxReduceBlocks).
constexpr int kMaxReduceBlocks = 4096;
struct GeomReduce {
  int rows, blocks;
};
GeomReduce reduce_geometry(int nx, int ny, int nz);
int reduce_blocks(int nx, int ny, int nz);

// Divergence / anti-trapping variants of the 2D step.
enum At2D : int {
  kAtApproxShells = 0,    // approximated current, shell fluxes (S-bar_{s1,s2})
  kAtFullShells = 1,      // full current, App. B |grad psi| at the flux points (S_{2,1})
  kAtFullTwoPoint = 2,    // full current, two-point <10> faces (S_{1,0})
  kAtApproxTwoPoint = 3,  // approximated current, two-point <10> faces
  kAtDiffusionOnly = 4,   // psi held, U by D~ div[(1 - phi) grad U] alone (shells)
};

// Record msg as the calling thread's last error (pf_last_error) and return
// code.
int report_error(int code, const char *msg);

template <typename T>
hipError_t launch_step2d(const Step2DArgs<T> &a, const Geom2D &g, bool frozen, bool reduce,
                         bool multi, int at, hipStream_t st);
template <typename T>
hipError_t launch_step3d(const Step3DArgs<T> &a, const Geom3D &g, bool frozen, bool reduce,
                         bool multi, hipStream_t st);
template <typename T>
hipError_t launch_reduce(const ReduceArgs<T> &a, hipStream_t st);
template <typename T>
hipError_t launch_batch2d(const BatchSolve2D<T> *table, const int2 *map, int blocks, int k,
                          bool frozen, bool reduce, bool multi, hipStream_t st);
template <typename T>
hipError_t launch_batch2d_advance(BatchSolve2D<T> *table, int n, int steps, bool frame,
                                  hipStream_t st);

}  // namespace pf
