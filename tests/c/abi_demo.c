/* A C program driving the library through include/pf.h alone (no Python, no
 * torch): a disc of solid in an undercooled melt on a 96 x 96 lattice,
 * stepped in FP64 and FP32 with library-owned workspaces on the null stream.
 * Prints one line of results; with an output path it also writes the FP64
 * psi and U arrays (raw doubles, psi then U) for comparison with the Python
 * binding.  Exit status 0 only if every call behaved as documented. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pf.h"

#define NX 96
#define NY 96
#define STEPS 200

static int check(int rc, const char *what) {
  if (rc != PF_OK) {
    fprintf(stderr, "%s failed: %d %s\n", what, rc, pf_last_error());
    return 1;
  }
  return 0;
}

static void params(pf_params *p, int precision, const double *rot) {
  memset(p, 0, sizeof *p);
  p->dim = 2;
  p->nx = NX;
  p->ny = NY;
  p->nz = 1;
  p->precision = precision;
  p->scheme = PF_SCHEME_ISO;
  p->k = 0.15;
  p->eps4 = 0.02;
  p->D = 2.0;
  p->lambda = 0.0;          /* D / a2 */
  p->h = 0.8;
  p->dt = 0.8 * 0.64 / 8.0; /* the paper's rule 0.8 h^2 / (4 D) */
  p->lT = 0.0;              /* isothermal */
  p->bc[0] = PF_BC_NOFLUX;
  p->bc[1] = PF_BC_NOFLUX;
  p->bc[2] = PF_BC_NOFLUX;
  p->n_grains = 1;
  p->grain_rot = rot;
}

int main(int argc, char **argv) {
  static double psi[NX * NY], U[NX * NY], out_psi[2][NX * NY], out_U[2][NX * NY];
  const double a = 10.0 * 3.14159265358979323846 / 180.0;
  const double rot[9] = {cos(a), -sin(a), 0.0, sin(a), cos(a), 0.0, 0.0, 0.0, 1.0};
  for (int j = 0; j < NY; ++j)
    for (int i = 0; i < NX; ++i) {
      const double x = i * 0.8 - 48 * 0.8, y = j * 0.8 - 48 * 0.8;
      psi[i + NX * j] = 8.0 - sqrt(x * x + y * y);
      U[i + NX * j] = -0.55;
    }
  const pf_init init = {psi, U, NULL};
  pf_tip tip[2];
  int bad = 0;
  if (pf_version() != PF_VERSION) return 2;

  for (int prec = 0; prec < 2; ++prec) {
    pf_params p;
    params(&p, prec == 0 ? PF_F64 : PF_F32, rot);
    pf_solver *s = NULL;
    bad |= check(pf_create(&p, &init, NULL, 0, NULL, &s), "pf_create");
    if (bad) return 1;
    bad |= check(pf_step(s, STEPS), "pf_step");
    bad |= check(pf_read_fields(s, NULL, out_U[prec], out_psi[prec], NULL), "pf_read_fields");
    bad |= check(pf_tip_state(s, &tip[prec]), "pf_tip_state");
    pf_destroy(s);
  }

  /* documented failures: an unstable time step and a bad lattice */
  pf_params p;
  params(&p, PF_F32, rot);
  p.dt = 10.0;
  pf_solver *s = NULL;
  if (pf_create(&p, &init, NULL, 0, NULL, &s) != PF_ERR_UNSTABLE_DT || s != NULL) bad = 1;
  params(&p, PF_F32, rot);
  p.nx = 2;
  if (pf_create(&p, &init, NULL, 0, NULL, &s) != PF_ERR_ARG || s != NULL) bad = 1;

  double du = 0.0;
  for (int c = 0; c < NX * NY; ++c) {
    const double d = fabs(out_U[0][c] - out_U[1][c]);
    if (!(d <= du)) du = d;  /* NaN-propagating max */
  }
  printf("steps %d  tip64 %.6f  tip32 %.6f  fs64 %.6f  fs32 %.6f  max|dU| %.3e  bad %d\n", STEPS,
         tip[0].y_frame, tip[1].y_frame, tip[0].solid_fraction, tip[1].solid_fraction, du, bad);
  if (!tip[0].found || !tip[1].found || tip[0].nonfinite || !(du <= 1e-5)) bad = 1;
  if (argc > 1) {
    FILE *f = fopen(argv[1], "wb");
    if (!f) return 1;
    fwrite(out_psi[0], sizeof(double), NX * NY, f);
    fwrite(out_U[0], sizeof(double), NX * NY, f);
    fclose(f);
  }
  return bad;
}
