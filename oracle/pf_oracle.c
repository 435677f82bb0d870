/*
 * pf_oracle.c -- plain FP64 CPU oracle of the explicit phi/U step of the
 * quantitative binary-alloy phase-field model with the O(h^2)-isotropic
 * finite-difference operators of arXiv:2110.12448.
 *
 * TEST INFRASTRUCTURE ONLY: read by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.
 *
 * Everything here is written for a reader holding the paper: one function per
 * discretised term, evaluated cell by cell, with no blocking or fusion.  Each
 * function names the passage it follows.  Readings of points the paper leaves
 * open are marked READING and listed in the design notes.
 *
 * Pinned by tests/test_oracle_*.py against closed forms (Fourier symbols of
 * Sec. 4.2, 6.1 and App. A; Taylor expansions of Sec. 4.1; exact results on
 * polynomials), an exact planar-front fixed point, the 1D reduction, lattice
 * rotation invariance, a pure-diffusion mode, and brute-force tip / solid
 * fraction cases.
 */
#include "pf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SQRT2 1.41421356237309504880
/* READING: |grad psi|^2 at or below this value (units W^-2) counts as a
 * vanishing gradient: a_s = 1 and no anisotropic torque (the paper is silent). */
#define GRAD_EPS 1e-12

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- ghosts */

/* Boundary ghost map of one axis.  PERIODIC wraps; NOFLUX mirrors about the
 * boundary face (-1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2), the cell-centred
 * reflection used for the no-flux walls of Sec. 4.3.2 and 6.2.2. */
static long ghost(long i, long n, int bc) {
  if (bc == OR_PERIODIC) {
    i %= n;
    if (i < 0) i += n;
    return i;
  }
  while (i < 0 || i >= n) {
    if (i < 0) i = -i - 1;
    if (i >= n) i = 2 * n - 1 - i;
  }
  return i;
}

static size_t cell(const or_params *p, long i, long j, long l) {
  size_t a = (size_t)ghost(i, p->nx, p->bc[0]);
  size_t b = (size_t)ghost(j, p->ny, p->bc[1]);
  size_t c = (p->dim == 3) ? (size_t)ghost(l, p->nz, p->bc[2]) : 0;
  return a + (size_t)p->nx * (b + (size_t)p->ny * c);
}

static size_t ncells(const or_params *p) {
  return (size_t)p->nx * (size_t)p->ny * (size_t)(p->dim == 3 ? p->nz : 1);
}

/* Value of field f at cell (i,j,l) + (a,b,c). */
#define F(f, a, b, c) (f)[cell(p, i + (a), j + (b), l + (c))]

/* Loop over every cell; rows are independent, so they may run in parallel. */
#define FOR_CELLS                                                     \
  _Pragma("omp parallel for collapse(2) schedule(static)")            \
  for (long l = 0; l < (long)(p->dim == 3 ? p->nz : 1); ++l)          \
    for (long j = 0; j < (long)p->ny; ++j)                            \
      for (long i = 0; i < (long)p->nx; ++i)

#define HERE ((size_t)i + (size_t)p->nx * ((size_t)j + (size_t)p->ny * (size_t)l))

/* Lattice shells of the cubic lattice: <100> has one non-zero component,
 * <110> two and <111> three (Sec. 5). */
static int shell_of(int a, int b, int c) {
  return (a != 0) + (b != 0) + (c != 0);
}

/* ------------------------------------------------------------- phi field */

/* Preconditioned phase field: phi = tanh(psi / sqrt 2) (Sec. 2, first eq.). */
void or_phi(const or_params *p, const double *psi, double *phi) {
  size_t n = ncells(p);
  for (size_t c = 0; c < n; ++c) phi[c] = tanh(psi[c] / SQRT2);
}

/* -------------------------------------------------------------- Laplacian */

/* 2D: L_{1,0} (Eq. 2D_L10), L_{0,1} (Eq. 2D_L01), mixed by Eq. tau_2D.
 * 3D: L_{1,0,0}, L_{0,1,0}, L_{0,0,1} (Eqs. 3D_L100, 3D_L110, 3D_L111),
 * mixed by Eq. tau_3D. */
void or_laplacian(const or_params *p, const double *psi, double *out) {
  const double h2 = p->h * p->h;
  if (p->dim == 2) {
    FOR_CELLS {
      double c0 = F(psi, 0, 0, 0);
      double L10 = (F(psi, 1, 0, 0) + F(psi, -1, 0, 0) + F(psi, 0, 1, 0) +
                    F(psi, 0, -1, 0) - 4.0 * c0) / h2;
      double L01 = (F(psi, 1, 1, 0) + F(psi, -1, 1, 0) + F(psi, 1, -1, 0) +
                    F(psi, -1, -1, 0) - 4.0 * c0) / (2.0 * h2);
      out[HERE] = p->w[0] * L10 + p->w[1] * L01;
    }
  } else {
    FOR_CELLS {
      double c0 = F(psi, 0, 0, 0);
      double s[4] = {0, 0, 0, 0};
      int cnt[4] = {0, 0, 0, 0};
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            int sh = shell_of(a, b, c);
            if (sh == 0) continue;
            s[sh] += F(psi, a, b, c);
            cnt[sh] += 1;
          }
      double L100 = (s[1] - cnt[1] * c0) / h2;          /* 6 points */
      double L010 = (s[2] - cnt[2] * c0) / (4.0 * h2);  /* 12 points */
      double L001 = (s[3] - cnt[3] * c0) / (4.0 * h2);  /* 8 points */
      out[HERE] = p->w[0] * L100 + p->w[1] * L010 + p->w[2] * L001;
    }
  }
}

/* -------------------------------------------------------- gradient square */

/* App. A.  2D: G_{1,0} (Eq. Grad_10), G_{0,1} (Eq. Grad_11).  3D: G_{1,0,0},
 * G_{0,1,0}, G_{0,0,1} (Eqs. Grad_100, Grad_110, Grad_111).  READING: the
 * printed 1/(144 h^2) prefactor of G_{0,0,1} is taken as 1/(16 h^2), the
 * value that reproduces the printed Fourier symbol and |grad psi|^2 exactly
 * on linear fields. */
void or_grad_square(const or_params *p, const double *psi, double *out) {
  const double h2 = p->h * p->h;
  if (p->dim == 2) {
    FOR_CELLS {
      double ex = F(psi, 1, 0, 0) - F(psi, -1, 0, 0);
      double ey = F(psi, 0, 1, 0) - F(psi, 0, -1, 0);
      double d1 = F(psi, 1, 1, 0) - F(psi, -1, -1, 0);
      double d2 = F(psi, 1, -1, 0) - F(psi, -1, 1, 0);
      double G10 = (ex * ex + ey * ey) / (4.0 * h2);
      double G01 = (d1 * d1 + d2 * d2) / (8.0 * h2);
      out[HERE] = p->w[0] * G10 + p->w[1] * G01;
    }
  } else {
    FOR_CELLS {
      /* One term per opposite pair: the half shell whose first non-zero
       * component is +1. */
      double s[4] = {0, 0, 0, 0};
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            int sh = shell_of(a, b, c);
            if (sh == 0) continue;
            int first = (a != 0) ? a : ((b != 0) ? b : c);
            if (first < 0) continue;
            double d = F(psi, a, b, c) - F(psi, -a, -b, -c);
            s[sh] += d * d;
          }
      double G100 = s[1] / (4.0 * h2);
      double G010 = s[2] / (16.0 * h2);
      double G001 = s[3] / (16.0 * h2);
      out[HERE] = p->w[0] * G100 + p->w[1] * G010 + p->w[2] * G001;
    }
  }
}

/* ------------------------------------------------------------ divergence */

/* Generalised divergence div(alpha grad beta).
 * 2D: D_{1,0} with the <10> fluxes of Eqs. divergence_10 and flux_10 (face
 * alpha = [alpha_0 + alpha_nb + two plaquette means] / 4), D_{0,1} with the
 * <11> fluxes of Eqs. divergence_11 and flux_11.
 * 3D: D_{1,0,0} (Eq. divergence_100; face alpha = 1/4 on the 2 nearest and
 * 1/16 on the 8 next-nearest points), D_{0,1,0} (Eq. divergence_110; edge
 * alpha = 3/16 on the 4 in-plane points, 1/32 on the 8 above and below),
 * D_{0,0,1} (Eq. divergence_111; corner alpha = mean of the cube). */
void or_divergence(const or_params *p, const double *alpha, const double *beta,
                   double *out) {
  const double h = p->h;
  if (p->dim == 2) {
    FOR_CELLS {
#define A(a, b) F(alpha, a, b, 0)
#define B(a, b) F(beta, a, b, 0)
      /* plaquette means abar at the four corners (1/2,1/2) etc. */
      double q_pp = (A(1, 1) + A(1, 0) + A(0, 1) + A(0, 0)) / 4.0;
      double q_pm = (A(1, -1) + A(1, 0) + A(0, -1) + A(0, 0)) / 4.0;
      double q_mp = (A(-1, 1) + A(-1, 0) + A(0, 1) + A(0, 0)) / 4.0;
      double q_mm = (A(-1, -1) + A(-1, 0) + A(0, -1) + A(0, 0)) / 4.0;
      /* <10> fluxes, positive out of the cell */
      double F_e = (A(1, 0) + A(0, 0) + q_pp + q_pm) * (B(1, 0) - B(0, 0)) / (4.0 * h);
      double F_n = (A(0, 1) + A(0, 0) + q_pp + q_mp) * (B(0, 1) - B(0, 0)) / (4.0 * h);
      double F_w = (A(0, 0) + A(-1, 0) + q_mp + q_mm) * (B(-1, 0) - B(0, 0)) / (4.0 * h);
      double F_s = (A(0, 0) + A(0, -1) + q_pm + q_mm) * (B(0, -1) - B(0, 0)) / (4.0 * h);
      double D10 = (F_e + F_w + F_n + F_s) / h;
      /* <11> fluxes */
      const double r2h = SQRT2 * h;
      double F_ne = (A(1, 1) + A(0, 0) + A(0, 1) + A(1, 0)) * (B(1, 1) - B(0, 0)) / (4.0 * r2h);
      double F_nw = (A(-1, 1) + A(0, 0) + A(0, 1) + A(-1, 0)) * (B(-1, 1) - B(0, 0)) / (4.0 * r2h);
      double F_se = (A(1, -1) + A(0, 0) + A(1, 0) + A(0, -1)) * (B(1, -1) - B(0, 0)) / (4.0 * r2h);
      double F_sw = (A(-1, -1) + A(0, 0) + A(0, -1) + A(-1, 0)) * (B(-1, -1) - B(0, 0)) / (4.0 * r2h);
      double D01 = (F_ne + F_nw + F_se + F_sw) / r2h;
      out[HERE] = p->w[0] * D10 + p->w[1] * D01;
#undef A
#undef B
    }
  } else {
    FOR_CELLS {
      double b0 = F(beta, 0, 0, 0);
      double D[4] = {0, 0, 0, 0};
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int c = -1; c <= 1; ++c) {
            int sh = shell_of(a, b, c);
            if (sh == 0) continue;
            int d[3] = {a, b, c};
            double abar = 0.0;
            if (sh == 1) {
              /* face (1/2,0,0)-type: 1/4 on the two nearest points, 1/16 on
               * the eight points one tangential step away from them. */
              abar = (F(alpha, 0, 0, 0) + F(alpha, a, b, c)) / 4.0;
              for (int ax = 0; ax < 3; ++ax) {
                if (d[ax] != 0) continue;
                for (int sg = -1; sg <= 1; sg += 2) {
                  int t[3] = {0, 0, 0};
                  t[ax] = sg;
                  abar += (F(alpha, t[0], t[1], t[2]) +
                           F(alpha, a + t[0], b + t[1], c + t[2])) / 16.0;
                }
              }
              D[1] += abar * (F(beta, a, b, c) - b0) / h / h;
            } else if (sh == 2) {
              /* edge (1/2,1/2,0)-type: 3/16 on the 4 points of the in-plane
               * plaquette, 1/32 on the 8 points above and below it. */
              int m = (d[0] == 0) ? 0 : ((d[1] == 0) ? 1 : 2);
              int e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
              int first = 1;
              for (int ax = 0; ax < 3; ++ax) {
                if (d[ax] == 0) continue;
                if (first) { e1[ax] = d[ax]; first = 0; } else { e2[ax] = d[ax]; }
              }
              int pts[4][3] = {{0, 0, 0},
                               {e1[0], e1[1], e1[2]},
                               {e2[0], e2[1], e2[2]},
                               {a, b, c}};
              for (int q = 0; q < 4; ++q) {
                abar += 3.0 / 16.0 * F(alpha, pts[q][0], pts[q][1], pts[q][2]);
                for (int sg = -1; sg <= 1; sg += 2) {
                  int t[3] = {0, 0, 0};
                  t[m] = sg;
                  abar += 1.0 / 32.0 * F(alpha, pts[q][0] + t[0], pts[q][1] + t[1],
                                         pts[q][2] + t[2]);
                }
              }
              /* flux abar * dbeta / (sqrt2 h), summed with prefactor 1/(2 sqrt2 h) */
              D[2] += abar * (F(beta, a, b, c) - b0) / (SQRT2 * h) / (2.0 * SQRT2 * h);
            } else {
              /* corner (1/2,1/2,1/2)-type: mean of the 8 cube corners */
              for (int x = 0; x <= 1; ++x)
                for (int y = 0; y <= 1; ++y)
                  for (int z = 0; z <= 1; ++z)
                    abar += F(alpha, x * a, y * b, z * c) / 8.0;
              /* flux abar * dbeta / (sqrt3 h), prefactor sqrt3 / (4 h) */
              D[3] += abar * (F(beta, a, b, c) - b0) / (sqrt(3.0) * h) * sqrt(3.0) / (4.0 * h);
            }
          }
      out[HERE] = p->w[0] * D[1] + p->w[1] * D[2] + p->w[2] * D[3];
    }
  }
}

/* Two-point divergence of the standard scheme S_{1,0} (Sec. 4.3.1, the
 * <10> discretisation the paper takes from its Ref. Tourret 2015; READING:
 * face alpha = mean of the two cells). */
void or_divergence_two_point(const or_params *p, const double *alpha, const double *beta,
                             double *out) {
  const double h2 = p->h * p->h;
  FOR_CELLS {
    double a0 = F(alpha, 0, 0, 0), b0 = F(beta, 0, 0, 0);
    double s = 0.0;
    for (int ax = 0; ax < p->dim; ++ax)
      for (int sg = -1; sg <= 1; sg += 2) {
        int e[3] = {0, 0, 0};
        e[ax] = sg;
        s += (a0 + F(alpha, e[0], e[1], e[2])) / 2.0 * (F(beta, e[0], e[1], e[2]) - b0);
      }
    out[HERE] = s / h2;
  }
}

/* ---------------------------------------------- full anti-trapping (App. B) */

/* Rotate offset (a, b) by dir quarter turns counter-clockwise. */
static void quarter(int q, int a, int b, int *x, int *y) {
  for (int k = 0; k < q; ++k) {
    int t = a;
    a = -b;
    b = t;
  }
  *x = a;
  *y = b;
}

/* beta at cell (i, j) + (a, b) rotated by q quarter turns. */
static double beta_rot(const or_params *p, const double *beta, long i, long j, int q, int a,
                       int b) {
  int x, y;
  quarter(q, a, b, &x, &y);
  const long l = 0;
  return F(beta, x, y, 0);
}

/* App. B: |grad beta| at the flux points with vanishing O(h^2) error.  The
 * formulas are printed for (1/2, 0) and (1/2, 1/2); the other points follow
 * by rotating the stencil (the gradient rotates with it). */
void or_flux_gradient_appB(const or_params *p, const double *beta, long i, long j, int dir,
                           double *gx, double *gy) {
  const double h = p->h;
  int q = dir & 3;
  double dx, dy;  /* derivatives in the rotated frame */
#define BR(a, b) beta_rot(p, beta, i, j, q, (a), (b))
  if (dir < 4) {
    /* point (1/2, 0) of the rotated frame */
    double t1 = (BR(1, 1) - BR(0, -1)) - (BR(0, 1) - BR(1, -1));
    double t2 = (BR(2, 1) - BR(-1, -1)) - (BR(-1, 1) - BR(2, -1));
    double t3 = (BR(1, 2) - BR(0, -2)) - (BR(0, 2) - BR(1, -2));
    dx = 35.0 / 24.0 * t1 / (2.0 * h) - 1.0 / 8.0 * t2 / (6.0 * h) - 1.0 / 3.0 * t3 / (2.0 * h);
    double u1 = (BR(1, 1) - BR(0, -1)) + (BR(0, 1) - BR(1, -1));
    double u2 = (BR(2, 1) - BR(-1, -1)) + (BR(-1, 1) - BR(2, -1));
    double u3 = (BR(1, 2) - BR(0, -2)) + (BR(0, 2) - BR(1, -2));
    dy = 35.0 / 24.0 * u1 / (4.0 * h) - 1.0 / 8.0 * u2 / (4.0 * h) - 1.0 / 3.0 * u3 / (8.0 * h);
  } else {
    /* point (1/2, 1/2) of the rotated frame */
    double t1 = (BR(1, 1) - BR(0, 0)) - (BR(0, 1) - BR(1, 0));
    double t2 = (BR(2, 1) - BR(-1, 0)) - (BR(-1, 1) - BR(2, 0));
    double t3 = (BR(1, 2) - BR(0, -1)) - (BR(0, 2) - BR(1, -1));
    dx = 5.0 / 4.0 * t1 / (2.0 * h) - 1.0 / 8.0 * t2 / (6.0 * h) - 1.0 / 8.0 * t3 / (2.0 * h);
    double u1 = (BR(1, 1) - BR(0, 0)) + (BR(0, 1) - BR(1, 0));
    double u2 = (BR(2, 1) - BR(-1, 0)) + (BR(-1, 1) - BR(2, 0));
    double u3 = (BR(1, 2) - BR(0, -1)) + (BR(0, 2) - BR(1, -1));
    dy = 5.0 / 4.0 * u1 / (2.0 * h) - 1.0 / 8.0 * u2 / (2.0 * h) - 1.0 / 8.0 * u3 / (6.0 * h);
  }
#undef BR
  /* back to the lattice frame: rotate (dx, dy) by q quarter turns */
  double x = dx, y = dy;
  for (int k = 0; k < q; ++k) {
    double t = x;
    x = -y;
    y = t;
  }
  *gx = x;
  *gy = y;
}

/* READING: a flux point whose |grad beta|^2 is at or below the guard carries
 * no anti-trapping flux (the normal is undefined there). */
static double inv_norm(double gx, double gy) {
  double g2 = gx * gx + gy * gy;
  return g2 > GRAD_EPS ? 1.0 / sqrt(g2) : 0.0;
}

/* Full anti-trapping term A = div(alpha grad beta / |grad beta|), 2D. */
void or_antitrapping_full(const or_params *p, const double *alpha, const double *beta,
                          double *out) {
  const double h = p->h;
  FOR_CELLS {
#define A(a, b) F(alpha, a, b, 0)
#define B(a, b) F(beta, a, b, 0)
    double b0 = B(0, 0);
    if (p->two_point) {
      /* <10> fluxes: two-point alpha, face gradient from the normal difference
       * and the tangential four-point average */
      double s = 0.0;
      for (int q = 0; q < 4; ++q) {
        int ex, ey, tx, ty;
        quarter(q, 1, 0, &ex, &ey);
        quarter(q, 0, 1, &tx, &ty);
        double gn = (B(ex, ey) - b0) / h;
        double gt = (B(tx, ty) + B(ex + tx, ey + ty) - B(-tx, -ty) - B(ex - tx, ey - ty)) /
                    (4.0 * h);
        s += (A(0, 0) + A(ex, ey)) / 2.0 * gn * inv_norm(gn, gt) / h;
      }
      out[HERE] = s;
    } else {
      double s10 = 0.0, s01 = 0.0;
      for (int q = 0; q < 4; ++q) {
        /* <10> flux of Eq. flux_10): face alpha from the two cells and the two
         * plaquettes beside the face */
        int ex, ey, tx, ty;
        quarter(q, 1, 0, &ex, &ey);
        quarter(q, 0, 1, &tx, &ty);
        double qp = (A(0, 0) + A(ex, ey) + A(tx, ty) + A(ex + tx, ey + ty)) / 4.0;
        double qm = (A(0, 0) + A(ex, ey) + A(-tx, -ty) + A(ex - tx, ey - ty)) / 4.0;
        double abar = (A(0, 0) + A(ex, ey) + qp + qm) / 4.0;
        double gx, gy;
        or_flux_gradient_appB(p, beta, i, j, q, &gx, &gy);
        s10 += abar * (B(ex, ey) - b0) / h * inv_norm(gx, gy) / h;
        /* <11> flux of Eq. flux_11): plaquette mean */
        int dx, dy;
        quarter(q, 1, 1, &dx, &dy);
        double qd = (A(0, 0) + A(dx, 0) + A(0, dy) + A(dx, dy)) / 4.0;
        or_flux_gradient_appB(p, beta, i, j, 4 + q, &gx, &gy);
        s01 += qd * (B(dx, dy) - b0) / (SQRT2 * h) * inv_norm(gx, gy) / (SQRT2 * h);
      }
      out[HERE] = p->w[0] * s10 + p->w[1] * s01;
    }
#undef A
#undef B
  }
}

/* ------------------------------------------------------------ anisotropy */

/* Cubic anisotropy of Eq. anis_function, rotated per grain.  READING (3D
 * form): a_s(n) = 1 - 3 eps4 + 4 eps4 sum_i n'_i^4 with n' = R^T n the normal
 * in the crystal frame; in 2D with R a rotation by alpha_0 this equals
 * 1 + eps4 cos 4(theta - alpha_0).  Returns a_s and, in dadg, the derivative
 * of a_s with respect to the lab-frame gradient g (the normal is g/|g|). */
static double anis(const or_params *p, int grain, const double g[3],
                   double dadg[3]) {
  const double *R = p->rot + 9 * grain;
  double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  dadg[0] = dadg[1] = dadg[2] = 0.0;
  if (!(g2 > GRAD_EPS)) return 1.0;
  double gl = sqrt(g2);
  double n[3] = {g[0] / gl, g[1] / gl, g[2] / gl};
  double nc[3];
  for (int r = 0; r < 3; ++r)
    nc[r] = R[0 * 3 + r] * n[0] + R[1 * 3 + r] * n[1] + R[2 * 3 + r] * n[2];
  double s4 = 0.0;
  for (int r = 0; r < 3; ++r) s4 += nc[r] * nc[r] * nc[r] * nc[r];
  double a = 1.0 - 3.0 * p->eps4 + 4.0 * p->eps4 * s4;
  /* d a / d g' in the crystal frame: 16 eps4 (n'^3 - s4 n') / |g| */
  double dc[3];
  for (int r = 0; r < 3; ++r)
    dc[r] = 16.0 * p->eps4 * (nc[r] * nc[r] * nc[r] - s4 * nc[r]) / gl;
  for (int r = 0; r < 3; ++r)
    dadg[r] = R[r * 3 + 0] * dc[0] + R[r * 3 + 1] * dc[1] + R[r * 3 + 2] * dc[2];
  return a;
}

/* a_s at the cell centre from the central-difference gradient. */
void or_anis_center(const or_params *p, const double *psi, const int8_t *grain,
                    double *a_c) {
  const double h = p->h;
  FOR_CELLS {
    double g[3];
    g[0] = (F(psi, 1, 0, 0) - F(psi, -1, 0, 0)) / (2.0 * h);
    g[1] = (F(psi, 0, 1, 0) - F(psi, 0, -1, 0)) / (2.0 * h);
    g[2] = (p->dim == 3) ? (F(psi, 0, 0, 1) - F(psi, 0, 0, -1)) / (2.0 * h) : 0.0;
    double dadg[3];
    int gr = grain ? grain[HERE] : 0;
    a_c[HERE] = anis(p, gr, g, dadg);
  }
}

/* Component `ax` of the anisotropic flux J = a^2 grad psi + |grad psi|^2 a
 * d a / d(grad psi) on the face between cell (i,j,l) and its +ax neighbour.
 * The face gradient takes the normal derivative across the face and the
 * tangential derivatives averaged over the two cells (the standard <10>-shell
 * discretisation the paper keeps for the eps4-linear terms, Sec. 2.2 and
 * Sec. 4.3.1).  READING: the face uses the grain of its lower cell. */
static double face_flux(const or_params *p, const double *psi,
                        const int8_t *grain, long i, long j, long l, int ax) {
  const double h = p->h;
  int e[3] = {0, 0, 0};
  e[ax] = 1;
  double g[3] = {0, 0, 0};
  g[ax] = (F(psi, e[0], e[1], e[2]) - F(psi, 0, 0, 0)) / h;
  for (int t = 0; t < p->dim; ++t) {
    if (t == ax) continue;
    int u[3] = {0, 0, 0};
    u[t] = 1;
    g[t] = (F(psi, u[0], u[1], u[2]) + F(psi, e[0] + u[0], e[1] + u[1], e[2] + u[2]) -
            F(psi, -u[0], -u[1], -u[2]) - F(psi, e[0] - u[0], e[1] - u[1], e[2] - u[2])) /
           (4.0 * h);
  }
  int gr = grain ? grain[cell(p, i, j, l)] : 0;
  double dadg[3];
  double a = anis(p, gr, g, dadg);
  double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  return a * a * g[ax] + g2 * a * dadg[ax];
}

/* The eps4-dependent part of the psi equation (Eq. PF_a):
 * grad(a_s^2) . grad psi + sum_q d_q(|grad psi|^2 a_s da_s/d(d_q psi))
 * = div J - a_s^2 lap psi.  READING: discretised on the <10> shell as
 * N = div_{10} J - a_c^2 L_std, which vanishes identically when eps4 = 0. */
void or_anis_remainder(const or_params *p, const double *psi,
                       const int8_t *grain, double *N) {
  const double h = p->h;
  FOR_CELLS {
    double divJ = 0.0;
    for (int ax = 0; ax < p->dim; ++ax) {
      int e[3] = {0, 0, 0};
      e[ax] = 1;
      divJ += (face_flux(p, psi, grain, i, j, l, ax) -
               face_flux(p, psi, grain, i - e[0], j - e[1], l - e[2], ax)) / h;
    }
    double c0 = F(psi, 0, 0, 0);
    double Lstd = F(psi, 1, 0, 0) + F(psi, -1, 0, 0) + F(psi, 0, 1, 0) + F(psi, 0, -1, 0) -
                  2.0 * p->dim * c0;
    if (p->dim == 3) Lstd += F(psi, 0, 0, 1) + F(psi, 0, 0, -1);
    Lstd /= h * h;
    double gc[3];
    gc[0] = (F(psi, 1, 0, 0) - F(psi, -1, 0, 0)) / (2.0 * h);
    gc[1] = (F(psi, 0, 1, 0) - F(psi, 0, -1, 0)) / (2.0 * h);
    gc[2] = (p->dim == 3) ? (F(psi, 0, 0, 1) - F(psi, 0, 0, -1)) / (2.0 * h) : 0.0;
    double dadg[3];
    double ac = anis(p, grain ? grain[HERE] : 0, gc, dadg);
    N[HERE] = divJ - ac * ac * Lstd;
  }
}

/* ----------------------------------------------------------------- rates */

/* Time derivatives of psi (Eq. PF_a) and U (Eq. PF_b with the approximated
 * anti-trapping current of Eq. Anti_approx), both at time level n.
 * Frozen temperature: F1, F2 of Eqs. Thermal_F1, Thermal_F2 with the thermal
 * coordinate zeta = y + s h - y0 - Vp n dt (READING: y is the thermal axis);
 * isothermal limit F1 = 1, F2 = U (Sec. 2.1).
 * Approximated anti-trapping (Sec. 2.3): Abar = div(alpha_A grad psi) with
 * alpha_A = (1 + (1-k)U) d(phi)/dt / sqrt2 = (1 + (1-k)U)(1 - phi^2) dpsi/dt / 2.
 * The source term of Eq. PF_b equals sqrt2 alpha_A.  With p->antitrapping the
 * full current div(alpha_A grad psi/|grad psi|) of Eq. Anti_convention (App. B
 * for its discretisation) replaces the approximated one. */
void or_rates(const or_params *p, const double *psi, const double *U,
              const int8_t *grain, int64_t n, int64_t s, double *rate_psi,
              double *rate_U) {
  size_t nc = ncells(p);
  double *phi = malloc(nc * sizeof(double));
  double *L = malloc(nc * sizeof(double));
  double *G = malloc(nc * sizeof(double));
  double *ac = malloc(nc * sizeof(double));
  double *N = malloc(nc * sizeof(double));
  double *aD = malloc(nc * sizeof(double));
  double *aA = malloc(nc * sizeof(double));
  double *divD = malloc(nc * sizeof(double));
  double *divA = malloc(nc * sizeof(double));

  or_phi(p, psi, phi);
  or_laplacian(p, psi, L);
  or_grad_square(p, psi, G);
  or_anis_center(p, psi, grain, ac);
  or_anis_remainder(p, psi, grain, N);

  const double k = p->k;
  const double t = (double)n * p->dt;
  const double off = (double)s * p->h - p->y0 - p->Vp * t;
  FOR_CELLS {
    size_t c = HERE;
    double F1 = 1.0, F2 = U[c];
    if (p->lT > 0.0) {
      double zeta = (double)j * p->h + off;
      F1 = 1.0 - (1.0 - k) * zeta / p->lT;
      F2 = U[c] + zeta / p->lT;
    }
    double ph = phi[c];
    double a2 = ac[c] * ac[c];
    double rhs = a2 * (L[c] - SQRT2 * ph * G[c]) + N[c] +
                 SQRT2 * (ph - p->lambda * (1.0 - ph * ph) * F2);
    rate_psi[c] = p->frozen_psi ? 0.0 : rhs / (F1 * a2);
    aD[c] = 1.0 - ph;
    aA[c] = (1.0 + (1.0 - k) * U[c]) * (1.0 - ph * ph) * rate_psi[c] / 2.0;
  }

  if (p->two_point)
    or_divergence_two_point(p, aD, U, divD);
  else
    or_divergence(p, aD, U, divD);
  if (p->antitrapping)
    or_antitrapping_full(p, aA, psi, divA);
  else if (p->two_point)
    or_divergence_two_point(p, aA, psi, divA);
  else
    or_divergence(p, aA, psi, divA);
  for (size_t c = 0; c < nc; ++c) {
    double rhs = p->D * divD[c] + divA[c] + SQRT2 * aA[c];
    rate_U[c] = rhs / (1.0 + k - (1.0 - k) * phi[c]);
  }

  free(phi); free(L); free(G); free(ac); free(N);
  free(aD); free(aA); free(divD); free(divA);
}

/* --------------------------------------------------------- tip, fraction */

/* Most advanced solid-liquid interface along y (Sec. 4.3.2, Sec. 6.2.1).
 * READING: over every pair of cells (i,j,l), (i,j+1,l) with phi >= 0 > phi
 * above it, the phi = 0 crossing y = (j + phi_j / (phi_j - phi_{j+1})) h by
 * linear interpolation; the tip is the largest such y, ties going to the
 * smallest linear index of the lower cell. */
void or_tip_find(const or_params *p, const double *phi, or_tip *out) {
  out->found = 0;
  out->idx = -1;
  out->x = out->y = out->z = 0.0;
  long nz = p->dim == 3 ? p->nz : 1;
  for (long l = 0; l < nz; ++l)
    for (long j = 0; j + 1 < p->ny; ++j)
      for (long i = 0; i < p->nx; ++i) {
        size_t c = (size_t)i + (size_t)p->nx * ((size_t)j + (size_t)p->ny * (size_t)l);
        size_t up = c + (size_t)p->nx;
        double f0 = phi[c], f1 = phi[up];
        if (!(f0 >= 0.0 && f1 < 0.0)) continue;
        double y = ((double)j + f0 / (f0 - f1)) * p->h;
        if (!out->found || y > out->y || (y == out->y && (int64_t)c < out->idx)) {
          out->found = 1;
          out->idx = (int64_t)c;
          out->x = (double)i * p->h;
          out->y = y;
          out->z = (double)l * p->h;
        }
      }
}

/* Solid fraction (1/N) sum (1 + phi)/2, summed in FP64 in index order. */
double or_solid_fraction(const or_params *p, const double *phi) {
  size_t n = ncells(p);
  double s = 0.0;
  for (size_t c = 0; c < n; ++c) s += (1.0 + phi[c]) / 2.0;
  return s / (double)n;
}

/* ------------------------------------------------------------------ step */

/* Moving frame: drop the bottom row, move every row down by one and keep the
 * old top row as the new top row (the far field is copied in). */
static void shift_down_bytes(const or_params *p, void *f, size_t elem) {
  long nz = p->dim == 3 ? p->nz : 1;
  size_t row = (size_t)p->nx * elem;
  for (long l = 0; l < nz; ++l) {
    char *plane = (char *)f + (size_t)l * row * (size_t)p->ny;
    memmove(plane, plane + row, row * (size_t)(p->ny - 1));
  }
}

static void shift_down(const or_params *p, double *f) { shift_down_bytes(p, f, sizeof(double)); }

/* READING (dynamic grains; the paper follows single grains and prints no
 * rule): a cell that is liquid at level n (phi < 0, i.e. psi < 0) and has a
 * solid face neighbour (psi >= 0) takes, at level n+1, the grain of the solid
 * face neighbour with the largest psi (largest phi), the first in the order
 * -x, +x, -y, +y, -z, +z on ties; every other cell keeps its grain.  Beyond a
 * no-flux wall the neighbour is the cell's image. */
void or_grain_update(const or_params *p, const double *psi, const int8_t *g, int8_t *gn) {
  FOR_CELLS {
    size_t c = HERE;
    int8_t out = g[c];
    if (psi[c] < 0.0) {
      int found = 0;
      double best = 0.0;
      for (int ax = 0; ax < p->dim; ++ax)
        for (int sg = -1; sg <= 1; sg += 2) {
          int e[3] = {0, 0, 0};
          e[ax] = sg;
          double v = F(psi, e[0], e[1], e[2]);
          if (v >= 0.0 && (!found || v > best)) {
            best = v;
            out = F(g, e[0], e[1], e[2]);
            found = 1;
          }
        }
    }
    gn[c] = out;
  }
}

/* Explicit Euler (Sec. 4.3.1): psi^{n+1} = psi^n + dt rate_psi, then
 * U^{n+1} = U^n + dt rate_U with rate_U built from psi^n, U^n and
 * dpsi/dt = rate_psi (READING: psi first, then U, all coefficients at level n).
 * With the moving frame on, the tip of phi^n decides after step n whether the
 * new state is shifted down one row (READING: at most one row per step). */
int or_step(const or_params *p, double *psi, double *U, int8_t *grain,
            int64_t nsteps, or_state *st) {
  size_t nc = ncells(p);
  double *rp = malloc(nc * sizeof(double));
  double *ru = malloc(nc * sizeof(double));
  double *phi = malloc(nc * sizeof(double));
  int8_t *gn = (p->dynamic_grains && grain) ? malloc(nc) : NULL;
  if (!rp || !ru || !phi || (p->dynamic_grains && grain && !gn)) {
    free(rp); free(ru); free(phi); free(gn);
    return -1;
  }
  for (int64_t it = 0; it < nsteps; ++it) {
    or_tip tip = {0, -1, 0, 0, 0};
    if (p->frame) {
      or_phi(p, psi, phi);
      or_tip_find(p, phi, &tip);
    }
    or_rates(p, psi, U, grain, st->step, st->shift, rp, ru);
    if (gn) or_grain_update(p, psi, grain, gn);  /* from level n */
    for (size_t c = 0; c < nc; ++c) {
      psi[c] += p->dt * rp[c];
      U[c] += p->dt * ru[c];
      if (p->round_f32) {
        psi[c] = (double)(float)psi[c];
        U[c] = (double)(float)U[c];
      }
    }
    st->step += 1;
    if (gn) memcpy(grain, gn, nc);
    if (p->frame && tip.found && tip.y >= (double)p->shift_row * p->h) {
      shift_down(p, psi);
      shift_down(p, U);
      if (gn) shift_down_bytes(p, grain, 1);
      st->shift += 1;
    }
  }
  int64_t bad = 0;
  for (size_t c = 0; c < nc; ++c)
    if (!isfinite(psi[c]) || !isfinite(U[c])) ++bad;
  st->nonfinite = bad;
  free(rp); free(ru); free(phi); free(gn);
  return 0;
}
