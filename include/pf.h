/*
 * pf.h -- C ABI of the MI355X phase-field library (libpfiso.so).
 *
 * One explicit time step of the quantitative phase-field model of dilute
 * binary-alloy solidification with the O(h^2)-isotropic finite-difference
 * operators of K. Ji, A. Molavi Tabrizi & A. Karma, "Isotropic
 * finite-difference approximations for phase-field simulations of
 * polycrystalline alloy solidification" (arXiv:2110.12448):
 *   - the preconditioned phase field psi, phi = tanh(psi/sqrt2) (Sec. 2),
 *     evolved by Eq. PF_a, and the supersaturation U evolved by Eq. PF_b with
 *     the approximated anti-trapping current of Eq. Anti_approx (Sec. 2.3);
 *   - Laplacian, gradient square and divergence mixed from lattice-shell
 *     bases (Eqs. tau_2D, tau_3D; Sec. 3, Sec. 5, App. A): S-bar_{2,1} in 2D
 *     and S-bar_{1,2,0} in 3D by default;
 *   - cubic interface anisotropy rotated per grain (Eq. anis_function), its
 *     eps4-linear terms on the standard <10>/<100> shell (Sec. 2.2, 4.3.1);
 *   - frozen temperature (Eqs. Thermal_F1, Thermal_F2) or isothermal growth;
 *   - explicit Euler in time (Sec. 4.3.1).
 *
 * Units: lengths in the interface width W, times in tau_0.  Lattice cell
 * (i, j, l) sits at (i h, j h, l h); y (index j) is the growth and thermal
 * axis.  Host arrays are row-major with x fastest: idx = i + nx*(j + ny*l).
 *
 * Errors: every int-returning call returns PF_OK (0) or a negative PF_ERR_*
 * code and leaves out-parameters untouched on failure; pf_last_error()
 * describes the last failure of the calling thread.  No exception crosses
 * this interface.  Threading: a solver belongs to the stream it was created
 * on; distinct solvers are independent and may run concurrently.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_VERSION 1

/* return codes */
#define PF_OK 0
#define PF_ERR_ARG (-1)          /* invalid argument or inconsistent parameters */
#define PF_ERR_UNSTABLE_DT (-2)  /* dt above the explicit stability limit */
#define PF_ERR_OOM (-3)          /* device allocation failed or workspace too small */
#define PF_ERR_DEVICE (-4)       /* a HIP runtime call failed */
#define PF_ERR_NONFINITE (-5)    /* the state holds NaN or Inf values */
#define PF_ERR_STATE (-6)        /* call not valid in the solver's state */

/* precision of the stored and stepped fields */
#define PF_F32 0
#define PF_F64 1

/* boundary condition per axis (no-flux: Sec. 4.3.2, 6.2.2; periodic: Sec. 4.3.3, 6.2.3) */
#define PF_BC_NOFLUX 0           /* mirror about the boundary face */
#define PF_BC_PERIODIC 1

/* finite-difference scheme: shell weights of Eq. tau_2D / tau_3D applied to
 * the Laplacian, the gradient square and both divergences */
#define PF_SCHEME_ISO 0          /* 2D (2/3, 1/3); 3D (1/3, 2/3, 0) */
#define PF_SCHEME_STD 1          /* 2D (1, 0);     3D (1, 0, 0) */
#define PF_SCHEME_WEIGHTS 2      /* pf_params.weights, normalised to sum 1 */

/* anti-trapping current in Eq. PF_b (2D may take either; 3D is approximated
 * only, as in Sec. 6: the full form would need a 3D analogue of App. B) */
#define PF_AT_APPROX 0           /* div[alpha grad psi], Eq. Anti_approx (Sec. 2.3) */
#define PF_AT_FULL 1             /* div[alpha grad psi / |grad psi|], Eq. Anti_convention;
                                    with shell fluxes |grad psi| at each flux point
                                    comes from the fourth-order stencils of App. B */

/* discretisation of the two divergences of Eq. PF_b (2D only) */
#define PF_DIV_SHELLS 0          /* shell fluxes with the scheme's weights (Sec. 4.1) */
#define PF_DIV_TWO_POINT 1       /* <10> faces only, face alpha the mean of the two
                                    cells and, for the full current, the face
                                    gradient from the normal difference and the
                                    four-point tangential difference: the standard
                                    scheme S_{1,0} of Sec. 4.3.1 (with PF_SCHEME_STD) */

typedef struct pf_params {
  int32_t dim;          /* 2 or 3 */
  int32_t nx, ny, nz;   /* lattice size, each >= 4 (nz ignored in 2D) */
  int32_t precision;    /* PF_F32 or PF_F64 */
  int32_t scheme;       /* PF_SCHEME_* */
  double weights[3];    /* shell weights for PF_SCHEME_WEIGHTS (3D: <100>,<110>,<111>) */
  double k;             /* interface partition coefficient, 0 < k < 1 */
  double eps4;          /* anisotropy strength, 0 <= eps4 < 1/15 */
  double D;             /* dimensionless diffusivity D~ = D tau0 / W^2 > 0 */
  double lambda;        /* coupling constant; <= 0 selects D~/a2, a2 = 47/75 (Sec. 2.1) */
  double h;             /* lattice spacing in units of W (the paper's h/W) */
  double dt;            /* time step in tau0; <= 0 selects 0.8 x pf_stable_dt() */
  double Vp;            /* pulling speed V~p (frozen temperature) */
  double lT;            /* thermal length l~T; <= 0 selects the isothermal limit */
  double y0;            /* isotherm origin: zeta = y + s h - y0 - Vp t */
  int32_t bc[3];        /* PF_BC_* for x, y, z */
  int32_t frame;        /* 1: moving frame along +y (requires bc[1] == PF_BC_NOFLUX) */
  int32_t shift_row;    /* frame moves one row when y_tip >= shift_row * h; 1..ny-2 */
  int32_t n_grains;     /* 1..127 */
  const double *grain_rot; /* n_grains x 9, row-major proper rotations, crystal -> lab */
  int32_t antitrapping; /* PF_AT_APPROX (0, default) or PF_AT_FULL */
  int32_t divergence;   /* PF_DIV_SHELLS (0, default) or PF_DIV_TWO_POINT */
  int32_t dynamic_grains; /* 0: static grain map.  1 (n_grains > 1): each step a
                             cell that is liquid (psi < 0) with a solid face
                             neighbour (psi >= 0) takes the grain of the solid
                             face neighbour with the largest psi (first of -x,
                             +x, -y, +y, -z, +z on ties), so orientations grow
                             with the solid; the map then shifts with the
                             moving frame and may vary along y */
} pf_params;

typedef struct pf_init {
  const double *psi;    /* nx*ny*nz initial psi (host, FP64, finite) */
  const double *U;      /* nx*ny*nz initial U (host, FP64, finite) */
  const int8_t *grain;  /* nx*ny*nz grain index in [0, n_grains), or NULL for all 0;
                           with the frame on it must not vary along y */
} pf_init;

typedef struct pf_tip {
  int64_t step;          /* steps taken */
  double t;              /* step * dt */
  int32_t found;         /* 0 when no cell pair crosses phi = 0 along y */
  int32_t nonfinite;     /* 1 when any psi or U value is NaN or Inf */
  int64_t index;         /* linear frame index of the cell below the crossing */
  double x, y_frame, z;  /* tip position in the frame (W) */
  double y_lab;          /* y_frame + frame_shift * h, in FP64 */
  double velocity;       /* d y_lab / dt between the last two pf_tip_state calls (0 at first) */
  double solid_fraction; /* (1/N) sum (1 + phi)/2, FP64 */
  int64_t frame_shift;   /* rows the frame has moved */
} pf_tip;

typedef struct pf_solver pf_solver;

/* Library version (PF_VERSION). */
int pf_version(void);

/* Message of the calling thread's last failure ("" if none). */
const char *pf_last_error(void);

/* Explicit stability limit used by pf_create: h^2 / (2 dim max(D~, 1/F1_min))
 * with F1_min the smallest F1 of Eq. Thermal_F1 over the initial lattice
 * (1 when isothermal).  This is the paper's rule for explicit Euler
 * (Sec. 4.3.1 and 6.2.1: dt = 0.8 h^2 / (2 dim D~) at 0.8 of the limit)
 * extended by the isotropic diffusivity 1/F1 of the psi equation (Eq. PF_a
 * divided by a_s^2 F1).  It leaves out the anisotropic interface stiffness,
 * which lowers the limit when the psi diffusivity binds (isothermal, D~ =
 * 0.5, eps4 = 0.06: 0.95 of this limit goes unstable, 0.8 does not): keep dt
 * at the default 0.8 of this limit when eps4 is large.  F1 changes
 * as zeta = y + s h - y0 - Vp t moves; pf_tip_state re-checks the limit for
 * the current s and t.  Returns a negative value on bad input. */
double pf_stable_dt(const pf_params *p);

/* Device bytes pf_create needs when the caller provides the memory. */
size_t pf_workspace_bytes(const pf_params *p);

/* Create a solver on `stream` (a hipStream_t; NULL for the null stream) of
 * the current device for the problem of Sec. 2.1: psi and U evolve by Eqs.
 * PF_a and PF_b (phi = tanh(psi / sqrt2)), with the anti-trapping current of
 * Eq. Anti_approx (or Eq. Anti_convention, 2D), the coupling lambda = a1
 * W/d0 = D~/a2 unless given, frozen temperature by Eqs. Thermal_F1 and
 * Thermal_F2 when lT > 0, and the cubic anisotropy of Eq. anis_function
 * rotated per grain by p->grain_rot; the operators are the shell mixes of
 * Eqs. tau_2D / tau_3D with the scheme's weights (Sec. 3, 5, App. A).  Copies
 * p, p->grain_rot and the init arrays; the caller keeps ownership of every
 * host pointer.  If `workspace` is non-NULL it is caller-owned device memory
 * of at least pf_workspace_bytes(p) bytes, 256-byte aligned, that must
 * outlive the solver; otherwise the library allocates and pf_destroy frees.
 * Validates the parameters (PF_ERR_ARG), dt against pf_stable_dt
 * (PF_ERR_UNSTABLE_DT) and the init arrays (PF_ERR_NONFINITE); *out is set
 * only on success. */
int pf_create(const pf_params *p, const pf_init *init, void *workspace,
              size_t workspace_bytes, void *stream, pf_solver **out);

/* Enqueue nsteps (>= 0) explicit Euler time steps (Sec. 4.3.1 and 6.2.1):
 * psi^{n+1} = psi^n + dt R_psi(psi^n, U^n) from Eq. PF_a, then U^{n+1} = U^n +
 * dt R_U(psi^n, U^n, d psi/dt) from Eq. PF_b, every coefficient at level n,
 * one fused kernel launch per step on the solver's stream; with the moving
 * frame the tip of phi^n decides whether level n+1 moves down one row.
 * Returns without waiting; non-finite values surface at the next
 * pf_tip_state.  PF_ERR_ARG for nsteps < 0, PF_ERR_DEVICE when a launch
 * fails. */
int pf_step(pf_solver *s, int64_t nsteps);

/* Enqueue nsteps steps of the solute-diffusion part of Eq. PF_b alone, with
 * psi held fixed (d psi/dt = 0, so the anti-trapping current and the source
 * vanish): U <- U + dt D~ D_{s1,s2}(1 - phi, U) / (1 + k - (1-k) phi) on the
 * shell divergence of the solver's weights (Sec. 4.1), psi copied to the next
 * buffer.  Each step reads and writes the same arrays as pf_step (16 bytes per
 * cell in FP32) with a fraction of its arithmetic, so it shows the
 * memory-bound regime of the same layout.  The moving-frame rule applies as in
 * pf_step.  2D only and shell divergences only (PF_ERR_ARG otherwise). */
int pf_step_diffusion(pf_solver *s, int64_t nsteps);

/* Wait for the solver's stream. */
int pf_synchronize(pf_solver *s);

/* Synchronise and copy the state to host FP64 arrays of nx*ny*nz values in
 * frame coordinates (x fastest): phi = tanh(psi/sqrt2), the change of
 * variable of Sec. 2.1 (phi = +1 solid, -1 liquid), U, and psi itself.  Any
 * pointer may be NULL; grain (int8, the current map) likewise.  psi and U
 * are copied in the field precision and widened, and phi is formed from the
 * copied psi, on the host in FP64 (a conversion of the output only: the
 * steps take their own phi on the device).  The caller owns the arrays.
 * PF_ERR_DEVICE when a copy fails. */
int pf_read_fields(pf_solver *s, double *phi, double *U, double *psi, int8_t *grain);

/* Synchronise, reduce the current state on the device and fill *out: the
 * tip, the most advanced solid-liquid interface along y (Sec. 4.3.2 and
 * 6.2.1), as the largest height y = (j + phi_j / (phi_j - phi_{j+1})) h of a
 * phi = 0 crossing between vertically adjacent cells (phi_j >= 0 > phi_{j+1};
 * ties to the smallest linear index), with its x and z; the solid fraction
 * (1/N) sum (1 + phi)/2; and a non-finite check.  Accumulation is FP64.
 * Returns PF_ERR_NONFINITE (with *out filled) when the state holds NaN or
 * Inf, and PF_ERR_UNSTABLE_DT (with *out filled) when, for the frame shift s
 * and time t now reached, F1 of Eq. Thermal_F1 is no longer positive over the
 * lattice or dt exceeds pf_stable_dt's limit with that F1. */
int pf_tip_state(pf_solver *s, pf_tip *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * reduction of pf_tip_state on caller-held device fields, with no solver.
 * psi and U are device arrays of nx*ny*nz values (float for PF_F32, double
 * for PF_F64), x fastest; pending = 1 reads them as owing one downward frame
 * shift (as pf_device_fields / pf_frame_state report), else 0.  Fills the
 * tip (found, index, x, y_frame, z; y_lab = y_frame), solid_fraction and
 * nonfinite of *out; step, t, velocity and frame_shift are 0.  Runs on
 * `stream` (NULL: the null stream) of the current device and waits for it.
 * Its partials and result live in a fixed array of this library on
 * each device (about 132 KB, held until the process ends), so it never
 * allocates device memory; every call on one device shares that array, so
 * calls that overlap on one device (several streams or host threads) race.
 * Any lattice the library accepts fits (x-y and y-z planes below 2^30
 * cells, at most 4e9 cells; ny >= 2): PF_ERR_ARG beyond that or for NULL
 * pointers, PF_ERR_NONFINITE (with *out filled) when a value is NaN or Inf,
 * PF_ERR_DEVICE when a HIP call fails. */
int pf_tip_fields(const void *psi, const void *U, int32_t precision, int32_t nx, int32_t ny,
                  int32_t nz, double h, int32_t pending, void *stream, pf_tip *out);

/* Device pointers of the current psi and U arrays (element type per
 * precision, nx*ny*nz each, frame rows possibly pending one shift: see
 * pf_frame_state).  Valid until the next pf_step. */
int pf_device_fields(pf_solver *s, void **psi, void **U);

/* Rows moved so far and whether the current device arrays still owe one
 * downward shift (applied on the fly by the next step and by the readers). */
int pf_frame_state(pf_solver *s, int64_t *shift, int32_t *pending);

/* Launch geometry of the step kernels: rows per wave segment (2D and 3D,
 * 4..256; in 2D also -k for k = 1..64, asking for k waves per SIMD of the
 * device: each 60-column strip then takes as many segments as give k * 4 *
 * (compute units) waves in all, at most one per row, and the rows are split
 * evenly between them) and z rows per workgroup (3D, 1..14 in FP32, 1..6 in
 * FP64, within the LDS of one workgroup; ignored in 2D).  Results do not
 * depend on it (only the work split changes); used by the tile autotuner.
 * PF_ERR_ARG outside these ranges. */
int pf_tune(pf_solver *s, int32_t rows_per_segment, int32_t z_tile);

/* The launch geometry in use (the library's default for the lattice and
 * precision until pf_tune or pf_autotune changes it; the 2D default is a
 * number of waves per SIMD, so rows_per_segment is negative); z_tile is 1
 * in 2D.
 * Either pointer may be NULL.  PF_ERR_ARG for a NULL solver.  (Launch
 * geometry is not part of the paper's method: results never depend on it.) */
int pf_geometry(pf_solver *s, int32_t *rows_per_segment, int32_t *z_tile);

/* Tile autotuner: time each candidate launch geometry (2D: 1..32 waves per
 * SIMD, as pf_tune's -k; 3D: rows per segment 8..256 times z rows per workgroup, within the
 * LDS of one workgroup and at most 6 z rows in FP64) over steps_per_trial
 * steps (after 2 warm-up steps) with HIP events on the solver's stream, two
 * interleaved passes keeping each candidate's better time, and keep the
 * fastest as if set by pf_tune; the geometry in use stays unless another is
 * more than 3% faster there and, re-timed against it in three interleaved
 * passes of 4 x steps_per_trial steps, still more than 2% faster (near-equal
 * candidates do not flip with noise).  Trials run on a scratch device copy
 * of the workspace (one extra workspace allocated and freed here), so the
 * solve itself neither advances nor changes; results never depend on the
 * choice.  Synchronises.  seg and ztile (either may be NULL) receive the
 * choice (ztile 1 in 2D).  PF_ERR_ARG for a NULL solver or steps_per_trial
 * outside [1, 2^20], PF_ERR_OOM when the scratch copy does not fit, PF_ERR_DEVICE when a
 * trial launch fails (the solve is then unchanged). */
int pf_autotune(pf_solver *s, int32_t steps_per_trial, int32_t *seg, int32_t *ztile);

/* Release the solver (and its workspace if the library allocated it). */
void pf_destroy(pf_solver *s);

/* ------------------------------------------------------------- batching
 * Many 2D solves advanced together: every step of every solve in ONE kernel
 * launch (each workgroup runs one tile of one solve), optionally replayed from
 * a captured HIP graph.  The solves keep their own workspaces and stay
 * usable through the calls above (read-back, tip state, single steps); a
 * batch only needs its solvers to be alive, 2D, of one precision, of one kind
 * (all frozen or all isothermal, all with or without the moving frame, all
 * single- or all multi-grain), on the approximated current with shell
 * divergences (the defaults) and bound to one stream.  Results are bitwise
 * those of stepping each solve on its own with the same launch geometry.  A
 * batch of one solver is valid: it replays a single small solve from a graph,
 * without a launch per step. */
typedef struct pf_batch pf_batch;

/* Build a batch over n solvers (the caller keeps the solvers). */
int pf_batch_create(pf_solver *const *solvers, int32_t n, pf_batch **out);

/* Enqueue nsteps steps of every solve; no host synchronisation (a solver
 * stepped on its own since the last call is picked up, at the cost of one
 * synchronisation). */
int pf_batch_step(pf_batch *b, int64_t nsteps);

/* Capture steps_per_graph launches (a multiple of 2; of 6 with the moving
 * frame) into a HIP graph replayed by pf_batch_step; 0 launches directly. */
int pf_batch_use_graph(pf_batch *b, int32_t steps_per_graph);

/* Batch autotuner: time the batched step for one segment length shared by
 * every member (4..32 rows) against the one in use (initially each member's
 * own segment length, at least 8 rows; for a member whose geometry asks for
 * waves per SIMD, the longest segment that gives alone) over
 * steps_per_trial steps on scratch copies of all
 * member workspaces, with the same passes and margins as pf_autotune,
 * then rebuild the batch with the choice (kept until the batch is destroyed;
 * it overrides the members' own pf_tune settings inside the batch only).  The
 * members do not advance.  Synchronises.  *seg (may be NULL) receives the
 * choice, 0 meaning each member's own segment length.  PF_ERR_ARG for a
 * NULL batch or steps_per_trial outside [1, 2^20], PF_ERR_OOM when the copies do not fit,
 * PF_ERR_DEVICE when a trial launch fails. */
int pf_batch_autotune(pf_batch *b, int32_t steps_per_trial, int32_t *seg);

/* Release the batch (not its solvers). */
void pf_batch_destroy(pf_batch *b);

#ifdef __cplusplus
}
#endif
#endif
