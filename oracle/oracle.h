/* FP64 CPU oracle for biased Langevin trial paths and the variational
 * functional.  TEST INFRASTRUCTURE ONLY: it is linked by the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product
 * library.  It shares no code or header with the HIP path.
 *
 * Plain, single-threaded, slow and written to be read against the paper:
 *   - Langevin equations of motion for solute X and solvent Y      (Eq. Lang)
 *   - external bias force on solute atoms only, harmonic in a collective
 *     variable z(X) toward a ramped reference                      (text after Eq. Lang)
 *   - ratchet-and-pawl bias with running minimum z_m               (Eq. VR)
 *   - contact-map collective variable                              (supplement, "Collective coordinate")
 *   - variational functional  int dt sum_i |F_i^bias|^2/(gamma_i m_i)
 *     with the 1/(4 kT) prefactor of the path action              (Eq. StrVMD, Eq. VMDcondition)
 *   - selection of the trial with the least functional among
 *     trials that reached the product                             (main text, folding-event criterion)
 *   - derivative of the functional with respect to the bias stiffness and
 *     ramp rate along a trajectory, the noise held fixed (dual numbers)
 *
 * Parity status per function is stated in the comment above it.
 */
#ifndef VP_ORACLE_H
#define VP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_atoms, n_solute;
  const double *mass, *gamma, *charge, *sigma, *epsilon; /* [n_atoms] */
  int32_t n_bonds;
  const int32_t *bonds; /* [n_bonds][2] */
  const double *bond_k, *bond_r0;
  int32_t n_angles;
  const int32_t *angles; /* [n_angles][3] (a, vertex, b) */
  const double *angle_k, *angle_theta0;
  int32_t n_excl;
  const int32_t *excl; /* [n_excl][2] */
  double box[3], r_cut, eps_rf, kT, dt;
  const double *x_final; /* [n_solute][3] or NULL */
  int32_t bias;
  double bias_k, ramp_rate, z_target;
  double contact_r0, contact_rs, contact_rc;
  int32_t contact_min_sep;
  double reach_tol;
  uint64_t seed;
  const double *const_force; /* [n_solute][3] for ORA_BIAS_CONST */
  double reach_rmsd;         /* nm: RMSD to X_f after optimal superposition; +inf = not used */
} ora_sys;

enum { ORA_BIAS_NONE = 0, ORA_BIAS_CONST = 1, ORA_BIAS_RG = 2, ORA_BIAS_CONTACT = 3,
       ORA_BIAS_RMD_CONTACT = 4 };

/* trajectory state carried between segments */
typedef struct {
  int64_t step;
  double phi_acc; /* sum_n w_n S_n so far, with w_0 = 1/2 */
  double s_last;  /* S at the latest step: Phi drops half of it (trapezoid end) */
  double z0;      /* z(X_0): start of the bias ramp */
  double z_m;     /* ratchet minimum */
  double z_last;
  int32_t status; /* 0 ok, 1 unstable */
  int32_t pad;
} ora_state;

/* energies/diagnostics of one force evaluation: the four terms of U(X,Y),
 * the bias energy, z, z_ref, S = sum_i |F_i^bias|^2/(gamma_i m_i), the total
 * U + U_bias, and the virial W_ab = sum over the pair and bonded terms of U of
 * r_a F_b (row-major, a, b in x, y, z; r the separation vector of a term's
 * atoms from a reference atom of the term, F the force on the displaced atom;
 * the bias is an external force and takes no part) */
enum { ORA_E_LJ = 0, ORA_E_RF, ORA_E_BOND, ORA_E_ANGLE, ORA_E_BIAS, ORA_Z, ORA_ZREF, ORA_S,
       ORA_U_TOTAL, ORA_VIR, ORA_N_TERMS = ORA_VIR + 9 };

typedef struct ora_ctx ora_ctx;

ora_ctx *ora_create(const ora_sys *s);
void ora_destroy(ora_ctx *c);

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void ora_uniforms(uint64_t seed, uint32_t atom, uint32_t step, uint32_t tag, double u[4]);
void ora_normals(uint64_t seed, uint32_t atom, uint32_t step, uint32_t tag, double g[3]);

int64_t ora_pairs(const ora_ctx *c, const double *x, int32_t use_cells, int32_t *out, int64_t cap);
int ora_forces(ora_ctx *c, const double *x, double t, const ora_state *st, int32_t use_cells,
               double *f, double *fbias, double *terms);
double ora_cv(const ora_ctx *c, const double *x, double *grad);
double ora_contact_value(double r, double r0, double rs, double rc, double *dcdr);
int ora_init(ora_ctx *c, const double *x0, ora_state *st);
void ora_maxwell(const ora_ctx *c, double *v);
int ora_run(ora_ctx *c, double *x, double *v, ora_state *st, int32_t nsteps, int32_t use_cells,
            double *traj);
double ora_phi(const ora_ctx *c, const ora_state *st);
/* root-mean-square deviation of the solute positions x (first n_solute rows
 * of [n][3]) from X_f after the optimal rigid superposition (rotation and
 * translation, no reflection), unweighted; NAN without x_final */
double ora_rmsd(const ora_ctx *c, const double *x);
/* product reached (main text, folding-event criterion): stable trajectory,
 * |z(X_t) - z_target| <= reach_tol and, when reach_rmsd is finite,
 * ora_rmsd(x) <= reach_rmsd; x are the current positions (may be NULL when
 * reach_rmsd is infinite) */
int ora_reached(const ora_ctx *c, const ora_state *st, const double *x);
int ora_select(int32_t n, const double *phi, const uint8_t *reached, const uint8_t *eligible,
               int32_t *best, double *best_phi);

/* Pathwise derivative with respect to theta = (bias_k, ramp_rate), the noise
 * held fixed, by dual-number evaluation of the functions above.
 *
 * ora_forces_dir: F = -grad U + F^bias at (x, t) and its derivatives along
 *   two directions: a displacement dx ([2][n][3], NULL = none) and, if
 *   theta != 0, the parameters (direction 0: bias_k, 1: ramp_rate).
 *   f [n][3], fdot [2][n][3], S and Sdot[2] may each be NULL.
 * ora_init_tangent: trapezoid accumulators pd[4] = (sum w dS/dk,
 *   sum w dS/drho, last dS/dk, last dS/drho) at step 0 (tangents zero).
 * ora_run_tangent: as ora_run, also advancing xt, vt ([2][n][3]: dx/dtheta,
 *   dv/dtheta) and pd.  Returns -1 for the ratchet bias (not differentiable
 *   through its running minimum).
 * ora_phi_grad: dPhi/dtheta [2] from pd (NaN for an unstable trajectory). */
int ora_forces_dir(ora_ctx *c, const double *x, const double *dx, int32_t theta, double t,
                   const ora_state *st, int32_t use_cells, double *f, double *fdot, double *S,
                   double *Sdot);
int ora_init_tangent(ora_ctx *c, const double *x0, const ora_state *st, double *pd);
int ora_run_tangent(ora_ctx *c, double *x, double *v, ora_state *st, double *xt, double *vt,
                    double *pd, int32_t nsteps, int32_t use_cells);
void ora_phi_grad(const ora_ctx *c, const ora_state *st, const double *pd, double *out);

/* ------------------------------------------------------------------------ */
/* Toy model (supplement, "Illustrative Application in a Toy Model"): a point  */
/* particle on the 2-D surface                                                 */
/*   U(x,y) = w^2 (x^2+y^2)^2 - A1 s1^2/(x^2+y^2+s1^2)^2                       */
/*          + A2 s2^2/(x^2+y^2+s2^2)^2 - A3 s3^2/((x-xm)^2+(y-ym)^2+s3^2)^2     */
/* with underdamped Langevin dynamics (BAOAB, as for the atomistic system),  */
/* noise normals (g0, g1) of Philox counter (0, step, 2, 0) under the trial's  */
/* key, and a bias on z = sqrt(x^2 + y^2): none (plain), the ratchet of Eq. VR  */
/* (rMD) or the harmonic steering force -K z grad z (steered MD).  The        */
/* functional of Eq. VMDcondition accumulates over every step (trapezoid).   */
/* ------------------------------------------------------------------------ */
typedef struct {
  double A1, A2, A3, s1, s2, s3, w, xm, ym;
  double gamma, mass, kT, dt;
  double x0, y0;
  double r_product; /* reached: first step with z <= r_product */
  double r_gate;    /* theta_gate: polar angle at the first step with z <= r_gate */
  int32_t n_steps;
  int32_t pad;
} ora_toy_params;

enum { ORA_TOY_PLAIN = 0, ORA_TOY_RMD = 1, ORA_TOY_SMD = 2 };
/* per-trial results: Phi, reached (0/1), first step with z <= r_product (-1),
 * final x, y, ratchet minimum z_m, polar angle at the first step with
 * z <= r_gate (NAN if none) */
enum { ORA_TOY_PHI = 0, ORA_TOY_REACHED, ORA_TOY_T_REACH, ORA_TOY_X, ORA_TOY_Y, ORA_TOY_ZMIN,
       ORA_TOY_THETA_GATE, ORA_TOY_COUNT };

/* U and its gradient at (x, y) */
double ora_toy_potential(const ora_toy_params *p, double x, double y, double *gx, double *gy);
/* one trial: out[ORA_TOY_COUNT]; path (may be NULL): [n_steps + 1][2] positions */
void ora_toy_run(const ora_toy_params *p, int32_t kind, double k_bias, uint64_t seed, double *out,
                 double *path);

/* ------------------------------------------------------------------------ */
/* Order of native-contact formation and path similarity (main text, the    */
/* matrix M of the mechanism analysis).  t: formation step of each of nc      */
/* contacts in trajectories a and b (a contact never formed carries the same  */
/* value as every other unformed one).  M_ij = 1 if t_i < t_j, 0 if t_i > t_j, */
/* 1/2 if equal; s = (number of ordered pairs i != j with M_ij(a) = M_ij(b))   */
/* / (nc (nc - 1)).                                                            */
/* ------------------------------------------------------------------------ */
double ora_path_similarity(int32_t nc, const int64_t *ta, const int64_t *tb);

/* Native contacts (reading of the main text's "native contacts"): solute
 * pairs i < j with j - i > contact_min_sep whose distance in X_f is at most
 * contact_r0 (where C = 3/5); a contact is formed at a configuration where
 * its distance is at most contact_r0.  Both decisions are taken exactly, on
 * positions and r0 rounded to the 2^-22 nm grid (squared integer distances).
 * ora_native_contacts writes up to cap pairs [cap][2] and returns the count;
 * ora_contacts_formed sets formed[k] for the listed pairs at positions x. */
int64_t ora_native_contacts(const ora_ctx *c, int32_t *pairs, int64_t cap);
void ora_contacts_formed(const ora_ctx *c, const double *x, const int32_t *pairs, int64_t nc,
                         uint8_t *formed);

#ifdef __cplusplus
}
#endif
#endif
