/*
 * pf_oracle.h -- plain FP64 CPU oracle for the isotropic phase-field step of
 * Ji, Molavi Tabrizi & Karma, "Isotropic finite-difference approximations for
 * phase-field simulations of polycrystalline alloy solidification"
 * (arXiv:2110.12448).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library under paper_2110_12448_amd/.
 *
 * Conventions: lengths in units of the interface width W, times in units of
 * tau_0 (Sec. 2.1).  Cell (i, j, l) sits at (i h, j h, l h); storage is
 * row-major with x fastest: idx = i + nx*(j + ny*l).  y is the growth and
 * thermal axis.  2D problems use nz = 1.
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_NOFLUX 0   /* cell-centred mirror about the boundary face */
#define OR_PERIODIC 1

typedef struct or_params {
  int32_t dim;              /* 2 or 3 */
  int32_t nx, ny, nz;       /* nz = 1 in 2D */
  double w[3];              /* shell weights (Eq. tau_2D / tau_3D), sum to 1 */
  double k;                 /* partition coefficient */
  double eps4;              /* anisotropy strength (Eq. anis_function) */
  double D;                 /* dimensionless diffusivity D~ */
  double lambda;            /* coupling constant */
  double h;                 /* lattice spacing in W */
  double dt;                /* explicit Euler step in tau_0 */
  double Vp;                /* pulling speed V~p */
  double lT;                /* thermal length l~T; <= 0 selects isothermal */
  double y0;                /* isotherm origin: zeta = y + s*h - y0 - Vp*t */
  int32_t bc[3];            /* OR_NOFLUX or OR_PERIODIC per axis */
  int32_t frame;            /* 1: moving frame along y */
  int32_t shift_row;        /* frame shifts when y_tip >= shift_row*h */
  int32_t n_grains;
  const double *rot;        /* n_grains x 9 row-major, crystal -> lab */
  int32_t round_f32;        /* 1: round stored psi, U to float after a step */
  int32_t antitrapping;     /* 0: approximated current (Sec. 2.3); 1: full
                               current of Eq. Anti_convention (2D only) */
  int32_t two_point;        /* 1: standard <10> divergences with two-point
                               face averages of alpha (2D scheme S_{1,0}) */
  int32_t frozen_psi;       /* 1: psi held fixed (d psi/dt = 0), U evolves by
                               Eq. PF_b alone: solute diffusion through a
                               frozen phase field */
  int32_t dynamic_grains;   /* 1: grain indices follow solidification
                               (or_grain_update), shifted with the frame */
} or_params;

typedef struct or_tip {
  int32_t found;            /* 0 when no cell pair crosses phi = 0 along y */
  int64_t idx;              /* linear index of the lower cell of the crossing */
  double x, y, z;           /* tip position in the frame (units of W) */
} or_tip;

typedef struct or_state {
  int64_t step;             /* n: number of steps taken, t = n*dt */
  int64_t shift;            /* s: rows the frame has moved */
  int64_t nonfinite;        /* non-finite psi/U values after the last step */
} or_state;

/* Whole-field operators: evaluate the discretisation at every cell, with the
 * boundary ghost map of p->bc.  `out` has nx*ny*nz entries. */
void or_phi(const or_params *p, const double *psi, double *phi);
void or_laplacian(const or_params *p, const double *psi, double *out);
void or_grad_square(const or_params *p, const double *psi, double *out);
void or_divergence(const or_params *p, const double *alpha, const double *beta,
                   double *out);
/* Divergence with two-point face averages on the <10> (<100>) shell:
 * (1/h^2) sum_faces (alpha_0 + alpha_e)/2 (beta_e - beta_0). */
void or_divergence_two_point(const or_params *p, const double *alpha, const double *beta,
                             double *out);
/* Full anti-trapping divergence div(alpha grad(beta)/|grad beta|) (2D):
 * shell fluxes of the divergence with |grad beta| at each flux point from the
 * O(h^4) formulas of App. B (two_point = 0), or <10> fluxes with two-point
 * alpha and the standard face gradient (two_point = 1). */
void or_antitrapping_full(const or_params *p, const double *alpha, const double *beta,
                          double *out);
/* App. B gradient of beta at the flux point of cell (i, j) in direction
 * dir: 0..3 = (+1/2,0), (0,+1/2), (-1/2,0), (0,-1/2); 4..7 = (+1/2,+1/2),
 * (-1/2,+1/2), (-1/2,-1/2), (+1/2,-1/2). */
void or_flux_gradient_appB(const or_params *p, const double *beta, long i, long j, int dir,
                           double *gx, double *gy);
void or_anis_center(const or_params *p, const double *psi, const int8_t *grain,
                    double *a_c);
void or_anis_remainder(const or_params *p, const double *psi,
                       const int8_t *grain, double *N);
/* Right-hand sides: rate_psi = d(psi)/dt and rate_U = dU/dt of one step at
 * time level n with frame shift s. */
void or_rates(const or_params *p, const double *psi, const double *U,
              const int8_t *grain, int64_t n, int64_t s, double *rate_psi,
              double *rate_U);

/* Grain indices of level n+1 from psi and the grains of level n (READING):
 * a liquid cell (psi < 0) with a solid face neighbour (psi >= 0) takes the
 * grain of the solid face neighbour with the largest psi, the first in the
 * order -x, +x, -y, +y, -z, +z on ties; other cells keep theirs. */
void or_grain_update(const or_params *p, const double *psi, const int8_t *g, int8_t *gn);

/* Advance nsteps explicit Euler steps in place; updates *st, and the grain
 * map in place when p->dynamic_grains. */
int or_step(const or_params *p, double *psi, double *U, int8_t *grain,
            int64_t nsteps, or_state *st);

/* Tip of the phase field phi and the solid fraction. */
void or_tip_find(const or_params *p, const double *phi, or_tip *out);
double or_solid_fraction(const or_params *p, const double *phi);

int or_num_threads(void);
/* Threads of the OpenMP loops over rows (results do not depend on it). */
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
