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

#ifdef __cplusplus
}
#endif
#endif
