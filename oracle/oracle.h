/*
 * oracle.h -- C interface of the FP64 reference ("oracle") of the
 * special-relativistic curvilinear PIC particle step
 * (Entity paper I, arXiv 2511.17710).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this library: only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py use it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Conventions (all restated from the paper):
 *   - code coordinates x^i in [0, N_i), cell size 1 in code units (Sec. 2.4);
 *   - field arrays are [6][np3][np2][np1] with x fastest, components
 *     (E1,E2,E3,B1,B2,B3) in that order, 2 ghost cells on each side of every
 *     active dimension (np_d = N_d + 4; in 2D np3 = 1); element (i,j,k)
 *     holds the component at its own Yee point (Sec. 3.1, App. A);
 *   - current arrays are [3][np3][np2][np1] with the same layout;
 *   - particles: per-dimension cell index i_d and offset delta_d in [0,1)
 *     (Sec. 3.1), four-velocity u in the global Cartesian basis (Sec. 2.3).
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t geom;        /* 0 Cartesian, 1 axisymmetric spherical, 2 quasi-spherical */
  int32_t dim;         /* Cartesian: 2 or 3; (quasi-)spherical: 2 */
  int32_t n[3];        /* active cells per dimension (unused = 1) */
  double lo[3], hi[3]; /* Cartesian extents; (quasi-)spherical: lo[0]=r_min, hi[0]=r_max */
  double r0, vartheta; /* quasi-spherical stretching parameters */
  int32_t periodic[3]; /* Cartesian only; must be 1 for every active dimension */
  double rho0;         /* fiducial Larmor radius */
} orc_grid;

typedef struct {
  int64_t n;
  int32_t *cell;      /* n x 3 (i1,i2,i3); unused dims 0 */
  double *offs;       /* n x 3, in [0,1); unused dims 0 */
  double *u;          /* n x 3 */
  double *w;          /* n */
  double *phi;        /* n, axisymmetric only (NULL otherwise) */
  int32_t *alive;     /* n, 1 alive / 0 dead */
  int32_t *cell_prev; /* n x 3, written on the last step of orc_run (may be NULL) */
  double *offs_prev;  /* n x 3, idem */
  int32_t *perm;      /* n, permutation of the last sort (may be NULL) */
} orc_species;

int32_t orc_version(void);
int64_t orc_field_points(const orc_grid *g); /* np1*np2*np3 */
double orc_dt_from_cfl(const orc_grid *g, double cfl);
void orc_sqrt_h(const orc_grid *g, const double *x, double *h);
double orc_theta_of_T(const orc_grid *g, double T);
double orc_T_of_theta(const orc_grid *g, double theta);
void orc_code_to_cart(const orc_grid *g, const double *x, double phi, double *X);
void orc_cart_to_code(const orc_grid *g, const double *X, double *x, double *phi);
int orc_fields_from_tetrad(const orc_grid *g, const double *in, int32_t includes_ghosts,
                           double *out);
void orc_interp(const orc_grid *g, const double *EB, int64_t n, const int32_t *cell,
                const double *offs, double *out6);
void orc_to_cart(const orc_grid *g, int64_t n, const int32_t *cell, const double *offs,
                 const double *phi, const double *F6, double *E3, double *B3);
void orc_boris(int64_t n, double k, const double *E3, const double *B3, double *u3);
void orc_vay(int64_t n, double k, const double *E3, const double *B3, double *u3);
void orc_gca(int64_t n, double k, const double *E3, const double *B3, double *u3);
void orc_move(const orc_grid *g, double dt, int64_t n, int32_t *cell, double *offs,
              double *phi, const double *u3, int32_t *alive, int32_t *m3, double *dx3);
void orc_move_literal(const orc_grid *g, double dt, int64_t n, const int32_t *cell,
                      const double *offs, const double *phi, const double *u3,
                      double *xnew, double *phinew);
void orc_sort_perm(int64_t n, const int32_t *keys, int32_t *perm);
/* the sort key of every particle (cell n x 3, alive n), as the sorts of orc_run form it */
int orc_sort_keys(const orc_grid *g, int64_t n, const int32_t *cell, const int32_t *alive,
                  int32_t *keys);
int orc_run(const orc_grid *g, double dt, int32_t nsteps, int32_t sort_every,
            int64_t step0, const double *EB, int32_t nspecies, const double *q,
            const double *m, orc_species *sp, double *J);
/* field solver (Sec. 2.3 steps 2, 9-11; App. A; Sec. 2.5, 2.6), in place on
 * padded arrays: Faraday B -= f curl E / sqrt(h); Ampere E += dt curl B /
 * sqrt(h) - coupling dt J / sqrt(h) with the axis rules; filter passes */
int orc_faraday(const orc_grid *g, double *EB, double f);
int orc_ampere(const orc_grid *g, double *EB, const double *J, double dt, double coupling);
int orc_filter(const orc_grid *g, double *J, int32_t passes);
double orc_polar_area(const orc_grid *g, double x1);
int orc_run_pushers(const orc_grid *g, double dt, int32_t nsteps, int32_t sort_every,
                    int64_t step0, const double *EB, int32_t nspecies, const double *q,
                    const double *m, const int32_t *pusher, const double *e_ovr,
                    const double *larmor_max, orc_species *sp, double *J);
int orc_adjoint(const orc_grid *g, double dt, int32_t K, const double *EB,
                int32_t nspecies, const double *q, const double *m,
                const orc_species *sp, const double *lamJ,
                const double *const *lam_u, const double *const *lam_d,
                double *dEB, double **du0, double **dd0, double *loss);
int orc_jvp(const orc_grid *g, double dt, int32_t K, const double *EB, const double *vEB,
            int32_t nspecies, const double *q, const double *m, const orc_species *sp,
            const double *const *vu0, const double *const *vd0, const double *lamJ,
            const double *const *lam_u, const double *const *lam_d, double *loss,
            double *dloss);

#ifdef __cplusplus
}
#endif
#endif
