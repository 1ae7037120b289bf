/* vp.h — C ABI of the MI355X (gfx950) library for batched biased-Langevin
 * trial paths scored by the variational functional of
 * S. a Beccara, L. Fant, P. Faccioli, "Variational scheme to compute protein
 * reaction pathways using atomistic force fields with explicit solvent"
 * (arXiv:1405.6104).
 *
 * The library integrates many independent trial trajectories of a solute X
 * (atoms [0, n_solute)) in explicit solvent Y (the remaining atoms) with the
 * Langevin equations of motion of the paper (Eq. Lang), adds an external,
 * time-dependent bias force on the solute only (text after Eq. Lang; the
 * ratchet form is Eq. VR), accumulates per trajectory the functional
 *     Phi = 1/(4 kT) * int_0^t dtau sum_{i in X} |F_i^bias|^2 / (gamma_i m_i)
 * (Eq. VMDcondition with the prefactor of the path action, Eq. StrVMD), and
 * selects the trajectory with the least Phi among those that reached the
 * product (main text, folding-event criterion).
 *
 * Conventions for every entry point:
 *   - units: nm, ps, amu, kJ/mol, elementary charge; angles in radians;
 *   - every function returns vp_status (VP_OK == 0); nothing throws or exits;
 *     on error vp_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread);
 *   - "host" pointers are read synchronously and may be freed on return;
 *     "device" pointers are HIP device allocations that must stay valid
 *     until the work enqueued on the given stream has completed;
 *   - per-atom arrays of a batch concatenate the replicas in the order given
 *     to vp_system_create, each replica's atoms in their original order
 *     ("user order"); 3-vectors are stored as [atom][3] (AoS), FP32 unless
 *     stated otherwise;
 *   - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *     The calls of one system are ordered: each asynchronous call records an
 *     event on its stream, and a later call on another stream first waits on
 *     it, so work enqueued on different streams never overlaps (the calls
 *     share device buffers); synchronising calls wait on that event.
 *   - one vp_system must not be used from two threads at once.
 */
#ifndef VP_H
#define VP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vp_system vp_system; /* opaque; owned by the library */

typedef enum {
  VP_OK = 0,
  VP_ERR_ARG = -1,    /* invalid argument (message says which) */
  VP_ERR_HIP = -2,    /* a HIP runtime call or kernel failed */
  VP_ERR_NOMEM = -3,  /* device or host allocation failed */
  VP_ERR_STATE = -4,  /* call not valid in the current state */
  VP_ERR_NOPATH = -5  /* vp_select_path: no eligible finite trajectory */
} vp_status;

typedef enum {
  VP_BIAS_NONE = 0,
  VP_BIAS_CONST = 1,       /* fixed force vector per solute atom (tests) */
  VP_BIAS_RG = 2,          /* harmonic in the mass-weighted radius of gyration */
  VP_BIAS_CONTACT = 3,     /* harmonic in the contact-map distance (supplement) */
  VP_BIAS_RMD_CONTACT = 4  /* ratchet-and-pawl on the contact-map distance (Eq. VR) */
} vp_bias_kind;

/* Per-replica status word (vp_observables, column VP_OBS_STATUS).  Either
 * flag freezes the replica at the step where it was raised: a force above
 * 1e6 kJ/mol/nm or a non-finite force (UNSTABLE), or a pair list that did
 * not fit its per-atom capacity or its block's staging capacity, so that
 * pairs were left out of the forces (LIST_OVERFLOW).  A flagged replica's
 * functional is +inf and it is never selected. */
enum { VP_REPLICA_OK = 0, VP_REPLICA_UNSTABLE = 1, VP_REPLICA_LIST_OVERFLOW = 2 };

/* One trial trajectory: the problem statement of the paper (masses m_i,
 * frictions gamma_i, kT, the potential U(X,Y), the bias F^bias(X,t), the
 * initial configuration X_i (+ solvent) and the product X_f).  All pointers
 * are HOST pointers, deep-copied by vp_system_create.
 *
 * Potential U(X,Y): Lennard-Jones, potential-shifted to zero at r_cut, with
 * sigma_ij = (sigma_i+sigma_j)/2 and eps_ij = sqrt(eps_i eps_j); reaction-field
 * Coulomb with dielectric eps_rf beyond r_cut (zero at r_cut); both over
 * non-excluded pairs closer than r_cut under the minimum-image convention in
 * an orthorhombic periodic box (r_cut < box/2); harmonic bonds 1/2 k (r-r0)^2
 * and angles 1/2 k (theta-theta0)^2 on unwrapped coordinates.
 *
 * Bias (solute only): U_b = 1/2 bias_k (z(X) - z_ref(t))^2 with
 * z_ref(t) = z_target + (z(X_0) - z_target) * max(0, 1 - ramp_rate * t);
 * z is the radius of gyration (VP_BIAS_RG) or the contact-map distance
 * sum_{i<j, j-i > contact_min_sep} (C~_ij(X) - C~_ij(X_f))^2 with
 * C~ = C(r) S(r), C = (1-(r/r0)^6)/(1-(r/r0)^10), S a quintic switch from 1 at
 * contact_rs to 0 at contact_rc.  VP_BIAS_RMD_CONTACT applies
 * -(bias_k/2)(z - z_m) grad z while z > z_m, z_m the running minimum of z. */
typedef struct {
  int32_t n_atoms;   /* > 0 and <= 65536 */
  int32_t n_solute;  /* 0 <= n_solute <= n_atoms; atoms [0, n_solute) are X */
  const double *mass, *gamma, *charge, *sigma, *epsilon; /* [n_atoms] */
  int32_t n_bonds;
  const int32_t *bonds; /* [n_bonds][2], two distinct atoms */
  const double *bond_k, *bond_r0;
  int32_t n_angles;
  const int32_t *angles; /* [n_angles][3]: end, vertex, end (three distinct atoms) */
  const double *angle_k, *angle_theta0;
  int32_t n_excl;
  const int32_t *excl; /* [n_excl][2]: pairs without nonbonded interaction */
  double box[3];       /* orthorhombic box edges */
  double r_cut, eps_rf, kT, dt;
  const double *x0;      /* [n_atoms][3] X_i (+ solvent), unwrapped; |x| < 238 nm */
  const double *v0;      /* [n_atoms][3] or NULL: Maxwell-Boltzmann from the seed */
  const double *x_final; /* [n_solute][3] X_f (defines the target contact map) or NULL */
  int32_t bias;          /* vp_bias_kind */
  double bias_k, ramp_rate, z_target;
  double contact_r0, contact_rs, contact_rc;
  int32_t contact_min_sep;
  double reach_tol;          /* reached requires |z(X_t) - z_target| <= reach_tol */
  uint64_t seed;             /* Philox4x32-10 key of this trajectory's noise */
  const double *const_force; /* [n_solute][3] for VP_BIAS_CONST (the force of
                                U_b = -sum_i F0_i . x_i; z reports sum_i F0_i . x_i),
                                else NULL */
  double reach_rmsd;         /* nm; when finite, reached also requires the RMSD of
                                the solute from X_f after the optimal rotation and
                                translation (unweighted, no reflection; the folding
                                criterion of the main text) to be <= reach_rmsd;
                                needs x_final.  +inf: not used */
} vp_replica_desc;

typedef struct {
  int32_t nstlist;     /* pair lists are rebuilt when the step count n + 1 is a
                          multiple of nstlist and whenever an atom has moved
                          half the skin since its replica's last build.
                          0: per replica, the largest power of two (<= 32) in
                          which a fast atom (5 sigma of the lightest atom's
                          Maxwell speed at kT) moves less than half of the
                          largest admissible skin (8 for 12,560-atom water at
                          300 K and 1 fs); powers of two keep the rebuild steps
                          of different replicas aligned */
  double skin;         /* pair-list buffer in nm.  0: per replica, just large
                          enough for the interval (rounded up to 0.01 nm; 0.13
                          in the case above) and at most the largest of 0.14,
                          0.13, ... nm whose staged neighbourhood fits the
                          force kernel's LDS and whose r_cut + skin stays below
                          half the box (VP_OBS_SKIN and VP_OBS_NSTLIST report
                          the values taken) */
  int32_t steps_per_graph; /* steps captured per hipGraph launch (0: 20) */
  int32_t use_graph;       /* 1: replay captured graphs; 0: launch every kernel */
  int32_t max_neighbors;   /* per-atom list capacity (0: derived from density) */
  int32_t tangent;         /* 1: also propagate dPhi/d(bias_k, ramp_rate) (vp_functional);
                              harmonic and constant biases only */
  int32_t force_shape;     /* tile shape of the force kernel (waves per 64-atom block x list
                              entries per batch): 0: 8x4 (default), 1: 8x2, 2: 4x4, 3: 16x2 */
  int32_t autotune;        /* 1: time every tile shape on each size bucket at creation and
                              launch each bucket with its fastest (force_shape is ignored);
                              the forces are bitwise the same for every shape */
  int32_t nst_out;         /* > 0: an energy record (VP_REC_*) of every replica at creation and
                              after every step whose count is a multiple of nst_out
                              (vp_energy_records); 0: none */
  int32_t out_capacity;    /* records kept per replica, the latest ones (0: 1024) */
  int32_t stage_cap;       /* > 0: staged neighbourhood atoms per 64-atom block at most this
                              (a diagnostic: blocks that need more are built again in exact
                              mode, which stages only atoms within the list radius of one of
                              the block's atoms); 0: as large as the force kernel's LDS allows */
  int32_t contact_order;   /* 1: record the step at which each native contact of the replicas
                              that give x_final first forms (vp_contact_order,
                              vp_path_similarity); 0: off */
  /* Device memory: when dev_alloc is not NULL every device buffer the system
   * holds is obtained from dev_alloc(bytes, alloc_ctx) (NULL = out of memory)
   * and returned with dev_free(ptr, alloc_ctx) by vp_system_destroy, or by a
   * failing vp_system_create; temporary buffers of the diagnostic calls too.
   * The memory must be device memory usable on every stream the system is
   * used with.  NULL: hipMalloc / hipFree. */
  void *(*dev_alloc)(size_t bytes, void *alloc_ctx);
  void (*dev_free)(void *ptr, void *alloc_ctx);
  void *alloc_ctx;
} vp_options;

/* Columns of the FP64 energy table written by vp_forces (one row per
 * replica) and the first columns of an energy record: Lennard-Jones,
 * reaction field, bond and angle energies, bias energy, z, z_ref (the ratchet
 * minimum for VP_BIAS_RMD_CONTACT), S = sum_i |F_i^bias|^2/(gamma_i m_i), the
 * total U + U_b, the virial W_ab = sum over the pair and bonded terms of U of
 * r_a F_b (r the separation of a moved atom from the term's other atom or
 * vertex, F the force on the moved atom; row-major; the bias, an external
 * force, takes no part), and the replica's status bits of that evaluation. */
enum { VP_E_LJ = 0, VP_E_RF, VP_E_BOND, VP_E_ANGLE, VP_E_BIAS, VP_E_Z, VP_E_ZREF, VP_E_S,
       VP_E_TOTAL, VP_E_WXX, VP_E_WXY, VP_E_WXZ, VP_E_WYX, VP_E_WYY, VP_E_WYZ, VP_E_WZX,
       VP_E_WZY, VP_E_WZZ, VP_E_STATUS, VP_E_COUNT };

/* An energy record of a trajectory (vp_energy_records): the VP_E_* columns at
 * step n, then n, the kinetic energy (1/2) sum m v^2 of the velocities of step
 * n, and Phi accumulated up to step n (trapezoid rule closed at n). */
enum { VP_REC_STEP = VP_E_COUNT, VP_REC_KE, VP_REC_PHI, VP_REC_COUNT };

#define VP_FORCE_SHAPES 4

/* One size bucket of a batch: the replicas that share a cutoff and
 * floor(log2 n_atoms), and the force-kernel tile shape their blocks run with.
 * With vp_options.autotune, ms[k] is the shortest of several timed force
 * launches of shape k over the bucket's blocks alone; otherwise ms is zero. */
typedef struct {
  double r_cut;        /* nm */
  int32_t log2_atoms;  /* floor(log2 n_atoms) of its replicas */
  int32_t n_replicas;
  int32_t n_blocks;    /* 64-atom blocks (padding included) */
  int32_t shape;       /* the vp_options.force_shape index its blocks run with */
  int32_t waves, entries;  /* that shape: waves per block, list entries per batch */
  double ms[VP_FORCE_SHAPES];
} vp_tile_bucket;

/* Positions are held as 32-bit fixed point in units of 2^-22 nm, so that
 * periodic images are exact integer shifts: x0 and x_dev are rounded to the
 * nearest multiple of 2^-22 nm (ties to even) on entry and every drift of the
 * integrator is rounded to that grid.  Coordinates must stay within 238 nm of
 * the origin.
 *
 * Create a batch of trial trajectories.  reps: HOST array of n_reps
 * descriptions (deep-copied).  opt: HOST, may be NULL for defaults.  Uploads
 * parameters, draws Maxwell velocities where v0 is NULL, builds the pair
 * lists and evaluates the forces and the functional integrand at t = 0.
 * Returns VP_ERR_ARG for NULL pointers, n_reps <= 0, n_atoms out of range,
 * r_cut >= box/2, indices out of range, negative masses/frictions, or a bias
 * kind that lacks its data (x_final, const_force).  *out is NULL on error. */
vp_status vp_system_create(const vp_replica_desc *reps, int32_t n_reps, const vp_options *opt,
                           vp_system **out);

/* Release every device and host resource.  NULL is accepted. */
vp_status vp_system_destroy(vp_system *s);

/* Total force F = -grad U + F^bias (Eq. Lang with the bias of the text after
 * it) at time t for the positions x_dev of every replica, without touching
 * the trajectory state.  x_dev: DEVICE [sum N][3] FP32 in user order;
 * f_dev: DEVICE [sum N][3] FP32 output; energy_dev: DEVICE [n_reps][VP_E_COUNT]
 * FP64 output (or NULL), the columns VP_E_*.  Ratchet replicas use their
 * current running minimum.  Asynchronous on hip_stream, so a replica whose
 * pair list overflowed (positions denser than the capacities sized at
 * creation allow) cannot be reported by the return value: its forces are
 * written as NaN and its VP_E_STATUS column and its VP_OBS_EVAL_STATUS
 * observable carry VP_REPLICA_LIST_OVERFLOW. */
vp_status vp_forces(vp_system *s, const float *x_dev, float *f_dev, double *energy_dev, double t,
                    void *hip_stream);

/* vp_forces for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same evaluation, results bit for bit those of vp_forces, with the evaluation
 * context (lists, staging, cell index, partial sums) in a static device array
 * of 64 MiB per GPU that the library holds until the process ends, instead
 * of buffers it allocates.  Allocates nothing.  Returns VP_ERR_ARG when the
 * system's context does not fit (about 30 MB for a 12,560-atom replica; a
 * batch that needs more uses vp_forces).  Every call on a GPU uses that GPU's
 * one array, so calls that overlap on one GPU -- on different streams, or
 * from different systems or threads -- race and must be ordered by the
 * caller.  Overflow reporting as for vp_forces (NaN forces and the status
 * column), except that VP_OBS_EVAL_STATUS follows vp_forces calls only. */
vp_status vp_forces_noalloc(vp_system *s, const float *x_dev, float *f_dev, double *energy_dev,
                            double t, void *hip_stream);

/* Advance every replica by n_steps BAOAB steps of Eq. Lang (>= 0),
 * accumulating Phi.  Asynchronous on hip_stream. */
vp_status vp_step_batch(vp_system *s, int32_t n_steps, void *hip_stream);

/* Phi of every replica since creation (Eq. VMDcondition, trapezoid rule in
 * time, 1/(4 kT) prefactor): phi_host HOST [n_reps]; +inf for an unstable
 * replica.  dphi_dtheta_host: HOST [n_reps][2] or NULL; if given, receives
 * dPhi/d(bias_k) and dPhi/d(ramp_rate) along each trajectory with its noise
 * held fixed (pathwise derivative of the discrete BAOAB trajectory, carried
 * forward by tangents), NaN for an unstable replica; VP_ERR_STATE unless
 * the system was created with vp_options.tangent = 1.  Synchronises the
 * system's last stream. */
vp_status vp_functional(vp_system *s, double *phi_host, double *dphi_dtheta_host);

/* Variational selection: the replica with the least finite Phi among those
 * that reached the product (status clear, |z - z_target| <= reach_tol at the
 * current step and, where reach_rmsd is finite, RMSD to X_f <= reach_rmsd)
 * and whose eligible flag (HOST [n_reps], NULL = all) is nonzero; ties go to
 * the lowest index.  Returns VP_ERR_NOPATH with *best = -1 when none
 * qualifies.  Synchronises. */
vp_status vp_select_path(vp_system *s, const uint8_t *eligible, int32_t *best, double *best_phi);

/* Copy the current positions and velocities in user order into DEVICE
 * buffers x_dev, v_dev ([sum N][3] FP32; either may be NULL).  Asynchronous.
 * The trajectory state itself lives in the library's own sorted, fixed-point
 * layout (positions in units of 2^-22 nm, reordered at every list rebuild),
 * so it is copied out rather than lent as views. */
vp_status vp_get_state(vp_system *s, float *x_dev, float *v_dev, void *hip_stream);

/* Per-replica observables: obs_host HOST [n_reps][VP_OBS_COUNT] FP64.
 * Pair-list statistics since creation: largest staged neighbourhood of a
 * 64-atom block and its capacity, longest per-atom list and its capacity,
 * number of blocks built again in exact mode (staging capacity reached);
 * the replica's pair-list buffer (nm) and rebuild interval. */
/* Also: the RMSD of the solute from X_f after optimal superposition (NaN
 * without x_final), whether the replica counts as having reached the product
 * (the criterion of vp_select_path), and the status bits of its latest
 * vp_forces evaluation.  Synchronises. */
enum { VP_OBS_STEP = 0, VP_OBS_Z, VP_OBS_ZREF, VP_OBS_ZMIN, VP_OBS_PHI, VP_OBS_STATUS,
       VP_OBS_REBUILDS, VP_OBS_KE, VP_OBS_STAGE_MAX, VP_OBS_STAGE_CAP, VP_OBS_LIST_MAX,
       VP_OBS_LIST_CAP, VP_OBS_EXACT_BUILDS, VP_OBS_SKIN, VP_OBS_NSTLIST, VP_OBS_RMSD,
       VP_OBS_REACHED, VP_OBS_EVAL_STATUS, VP_OBS_COUNT };
vp_status vp_observables(vp_system *s, double *obs_host);

/* Energy records of the trajectories (vp_options.nst_out > 0): writes the
 * number of records held per replica to *n_records (the same for every
 * replica: at most vp_options.out_capacity, the latest ones) and, if out_host
 * is not NULL, min(cap, *n_records) of them per replica, oldest first, as
 * HOST FP64 [n_reps][min(cap, *n_records)][VP_REC_COUNT].  VP_ERR_STATE when
 * the system records nothing.  Synchronises. */
vp_status vp_energy_records(vp_system *s, double *out_host, int32_t cap, int32_t *n_records);

/* Order of native-contact formation (main text, mechanism analysis; needs
 * vp_options.contact_order = 1).  The native contacts of a replica are its
 * solute pairs i < j with j - i > contact_min_sep and |X_f,i - X_f,j| <=
 * contact_r0; a contact forms at the first step (0 = the initial state) at
 * which its distance is <= contact_r0.  Both tests are exact, on squared
 * integer distances of positions and r0 on the 2^-22 nm grid.  Writes the
 * number of contacts of replica rep to *n_contacts and, where not NULL, the
 * first min(cap, n) pairs (HOST int32 [cap][2], replica-local user indices)
 * and formation steps (HOST int64 [cap], -1 = not formed yet).  Synchronises. */
vp_status vp_contact_order(vp_system *s, int32_t rep, int32_t *pairs_host, int64_t *steps_host,
                           int32_t cap, int32_t *n_contacts);

/* Path similarity s(k, k') = (number of ordered contact pairs i != j with
 * M_ij(k) = M_ij(k')) / (N_c (N_c - 1)), M_ij = 1, 0, 1/2 when contact i forms
 * before, after or at the same step as j (contacts not formed yet count as
 * forming together, after all others), for every pair of replicas with the
 * same native contacts: sim_host HOST [n_reps][n_reps] FP64, NaN where the
 * contact sets differ or N_c < 2.  Computed on the GPU; synchronises. */
vp_status vp_path_similarity(vp_system *s, double *sim_host);

/* Device bytes held by the system (its buffers, whichever allocator). */
vp_status vp_device_bytes(const vp_system *s, int64_t *bytes);

/* Force-kernel timing.  While on != 0, vp_step_batch enqueues its steps by
 * direct kernel launches (no graph replay) with a HIP event recorded on the
 * caller's stream before and after every nonbonded+bonded force launch, and
 * waits for each block of steps to accumulate the elapsed times.  Results are
 * bit-identical to the graph path. */
vp_status vp_set_timing(vp_system *s, int32_t on);

/* Mean duration (*avg_ms) and number (*count) of the force launches timed
 * since the last reset; reset != 0 clears the accumulators. */
vp_status vp_kernel_timing(vp_system *s, double *avg_ms, int64_t *count, int32_t reset);

/* Number of unordered pairs of replica rep whose current separation passes
 * the force kernel's membership predicate (a diagnostic; synchronises). */
vp_status vp_pair_count(vp_system *s, int32_t rep, int64_t *count);

/* Sizes: total atoms of the batch and number of replicas. */
vp_status vp_sizes(const vp_system *s, int64_t *n_atoms_total, int32_t *n_reps);

/* The size buckets of the batch and their force tile shapes, in order of
 * first appearance in the batch: writes min(cap, count) entries to out (HOST,
 * may be NULL when cap is 0) and the count to *n_buckets.  With autotuning,
 * *split (may be NULL) is 1 when the buckets run as one launch per chosen
 * shape and 0 when one shape over every block timed faster. */
vp_status vp_tile_buckets(vp_system *s, vp_tile_bucket *out, int32_t cap, int32_t *n_buckets,
                          int32_t *split);

/* Diagnostic (tests of the launch plan): runs the force kernel of size bucket
 * i (in vp_tile_buckets order) with tile shape shapes[i] (HOST, n = number of
 * buckets), as one launch per shape over its buckets' blocks, whatever the
 * shapes.  Synchronises; captured step graphs are rebuilt on the next call. */
vp_status vp_debug_set_tiles(vp_system *s, const int32_t *shapes, int32_t n);

/* Diagnostic (derivative checks): the directional derivatives of the total
 * force of vp_forces along two displacements of the positions, parameters
 * fixed -- the Hessian-vector products that carry the tangents.
 * x_dev: DEVICE [sum N][3] FP32 positions; dx_dev: DEVICE [2][sum N][3] FP32
 * directions; out_dev: DEVICE [2][sum N][3] FP32.  VP_ERR_STATE unless the
 * system was created with vp_options.tangent = 1.  Asynchronous. */
vp_status vp_debug_force_dir(vp_system *s, const float *x_dev, const float *dx_dev, float *out_dev,
                             double t, void *hip_stream);

/* Diagnostic (derivative checks): the exact trajectory state in user order,
 * HOST FP64 buffers: x_host, v_host [sum N][3] (positions are the grid values);
 * xt_host, vt_host [2][sum N][3] dx/dtheta, dv/dtheta and pd_host [n_reps][4]
 * (sum_n w_n dS_n/dtheta for bias_k and ramp_rate, then the latest dS/dtheta),
 * each NULL or, when given, requiring vp_options.tangent = 1.  Synchronises. */
vp_status vp_debug_trajectory_state(vp_system *s, double *x_host, double *v_host, double *xt_host,
                                    double *vt_host, double *pd_host);

/* Diagnostics for tests: copy the pair list of replica rep as unordered
 * pairs (i < j, replica-local user indices) whose current FP32 separation
 * passes the membership predicate, into pairs_host HOST [cap][2].
 * *count receives the number of such pairs (which may exceed cap). */
vp_status vp_debug_pairs(vp_system *s, int32_t rep, int32_t *pairs_host, int64_t cap,
                         int64_t *count);

/* Diagnostics for tests: draw the three Box-Muller normals the integrator
 * uses for (seed, atom, step, tag) for n consecutive atoms starting at
 * atom0.  out_dev: DEVICE [n][4] FP32 (g0, g1, g2, first uniform). */
vp_status vp_debug_noise(uint64_t seed, uint32_t atom0, uint32_t step, uint32_t tag, int32_t n,
                         float *out_dev, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Toy model (supplement, "Illustrative Application in a Toy Model"): trial
 * paths of one particle on the 2-D surface
 *   U(x,y) = w^2 (x^2+y^2)^2 - A1 s1^2/(x^2+y^2+s1^2)^2 + A2 s2^2/(x^2+y^2+s2^2)^2
 *            - A3 s3^2/((x-xm)^2+(y-ym)^2+s3^2)^2
 * with the BAOAB Langevin steps of the atomistic trials (FP64; noise normals
 * of Philox counter (0, step, 2, 0) under the trial's key, Maxwell velocities
 * from counter (0, 0, 1, 0)), biased on z = sqrt(x^2 + y^2) by nothing
 * (VP_TOY_PLAIN), the ratchet of Eq. VR with k_R = k (VP_TOY_RMD) or the
 * steering force -k z grad z (VP_TOY_SMD), each scored by Phi of Eq.
 * VMDcondition over the whole run.
 * ------------------------------------------------------------------------- */
typedef struct {
  double A1, A2, A3, s1, s2, s3, w, xm, ym;  /* the surface (paper: 30, 20, 6, 1, 2, 2, 0.03, 1.5, 0) */
  double gamma, mass, kT, dt;                /* paper: 1, 1, 0.2, 0.02 */
  double x0, y0;                             /* start (paper: 0, 5) */
  double r_product;                          /* reached: z <= r_product at some step */
  double r_gate;                             /* VP_TOY_THETA_GATE: polar angle at the first step
                                                with z <= r_gate */
  int32_t n_steps;                           /* steps per trial */
  int32_t path_stride;                       /* > 0: positions every path_stride steps */
} vp_toy_params;

enum { VP_TOY_PLAIN = 0, VP_TOY_RMD = 1, VP_TOY_SMD = 2 };
/* per-trial results: Phi, reached (0/1), first step with z <= r_product (-1:
 * none), final x and y, ratchet minimum (NaN for other kinds), polar angle at
 * the first step with z <= r_gate (NaN: none) */
enum { VP_TOY_PHI = 0, VP_TOY_REACHED, VP_TOY_T_REACH, VP_TOY_X, VP_TOY_Y, VP_TOY_ZMIN,
       VP_TOY_THETA_GATE, VP_TOY_COUNT };

/* Run n_trials independent toy trials, one GPU thread each.  p: HOST.
 * kind_dev, k_dev, seed_dev: DEVICE [n_trials] (kind, bias constant, Philox
 * key); out_dev: DEVICE [n_trials][VP_TOY_COUNT] FP64; path_dev: DEVICE
 * [n_trials][n_steps/path_stride + 1][2] FP32 (x, y at steps 0, stride, ...)
 * or NULL.  Allocates nothing; asynchronous on hip_stream.  VP_ERR_ARG for
 * n_trials <= 0, n_steps < 0, non-positive mass, dt or kT, negative gamma, or
 * a path buffer without path_stride > 0. */
vp_status vp_toy_trials(const vp_toy_params *p, int32_t n_trials, const int32_t *kind_dev,
                        const double *k_dev, const uint64_t *seed_dev, double *out_dev, float *path_dev,
                        void *hip_stream);

/* Variational selection over toy results (HOST [n][VP_TOY_COUNT], e.g. copied
 * from vp_toy_trials): least finite Phi among reached trials whose eligible
 * flag (HOST [n] or NULL) is set, ties to the lowest index; VP_ERR_NOPATH and
 * *best = -1 when none qualifies. */
vp_status vp_toy_select(const double *out_host, int32_t n, const uint8_t *eligible, int32_t *best,
                        double *best_phi);

const char *vp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VP_H */
