// Host-side launchers of the vp kernels (one translation unit per kernel group).
#pragma once
#include "vp_internal.h"

namespace vp {

enum { INT_FINISH = 1, INT_START = 2, INT_INIT = 4 };

// binning + permutation + lists; mode 0: trajectory (device decides), 1: from x_user
void launch_rebuild(vp_system *s, Work &W, int mode, const float *x_user, hipStream_t st);
void launch_debug_pairs(vp_system *s, Work &W, int rep, int2 *out, unsigned long long cap,
                        unsigned long long *counter, hipStream_t st);
void launch_forces(vp_system *s, Work &W, hipStream_t st);  // pair + bonded
void launch_pair_forces(vp_system *s, Work &W, hipStream_t st);  // k_forces launches only
void launch_bonded(vp_system *s, Work &W, hipStream_t st);  // adds the bonded forces
// one tile shape (index into kForceShapes) over a list of blocks (NULL: all nblk blocks)
void launch_forces_shape(vp_system *s, Work &W, int shape, const int32_t *blist, int nblk,
                         hipStream_t st);
// energy and virial partials per block into W.epart; gated: only on steps whose
// count after the step in progress is a multiple of s->opt.nst_out
void launch_energies(vp_system *s, Work &W, bool gated, hipStream_t st);
size_t energy_lds_bytes(const vp_system *s);
hipError_t prepare_energies(const vp_system *s);
// energy record of every replica into s->records (gated: on record steps only;
// otherwise the step just completed is recorded unconditionally)
void launch_record(vp_system *s, bool gated, hipStream_t st);
// RMSD of every replica's solute from its X_f into s->rmsd
void launch_rmsd(vp_system *s, hipStream_t st);
// first-formation steps of the native contacts at the current step counter
void launch_contact_form(vp_system *s, hipStream_t st);
// LDS of the similarity kernel for lists of up to max_contacts contacts
hipError_t prepare_similarity(int max_contacts);
// concordant ordered contact pairs of the replica pairs pr [npairs] into out
void launch_similarity(vp_system *s, const int2 *pr, int npairs, int max_contacts, unsigned long long *out,
                       hipStream_t st);
// toy-model trials (one thread each)
void launch_toy(const vp_toy_params &p, int n, const int32_t *kind, const double *k, const uint64_t *seed,
                double *out, float *path, hipStream_t st);
void launch_cv(vp_system *s, Work &W, int inc_step, hipStream_t st, bool tan);
// derivatives along the tangents in W.tx (both directions)
void launch_tangent_forces(vp_system *s, Work &W, hipStream_t st);
size_t tangent_lds_bytes(const vp_system *s);
hipError_t prepare_tangent(const vp_system *s);
// total force derivative along user-order directions dx_user [2][users][3] (eval context)
void launch_force_dir(vp_system *s, Work &W, const float *dx_user, double t, float *out,
                      hipStream_t st);
void launch_force_out(vp_system *s, Work &W, double t, float *f_user, double *e_out,
                      hipStream_t st);
void launch_integrate(vp_system *s, int mode, hipStream_t st);  // tangents too when s->tangent
void launch_init_state(vp_system *s, const int32_t *xq_user, const float *v_user,
                       const uint8_t *has_v, hipStream_t st);
void launch_native_map(const float *xf, int ns, int min_sep, float r0, float rs, float rc,
                       float *out, hipStream_t st);
// the same map per 64 x 64 tile in diagonal order (k_cv_pairs reads it above the diagonal)
void launch_cv_skew(const float *cmap, int ns, float *skew, hipStream_t st);
// reads `bytes` of device memory (autotuning: evicts the last-level cache between timed launches)
void launch_touch(const void *p, size_t bytes, int *sink, hipStream_t st);
size_t force_lds_bytes(const vp_system *s);
hipError_t prepare_forces(const vp_system *s);  // dynamic LDS above 64 KB
void launch_gather_state(vp_system *s, float *x_out, float *v_out, hipStream_t st);
void launch_kinetic(vp_system *s, double *out, hipStream_t st);  // per-tile partials
// exact state in user order (device FP64 buffers; xt, vt may be NULL)
void launch_export_state(vp_system *s, double *x, double *v, double *xt, double *vt, hipStream_t st);
void launch_debug_noise(uint64_t seed, uint32_t atom0, uint32_t step, uint32_t tag, int n,
                        float *out, hipStream_t st);

// the evaluation of vp_forces into the buffers of an evaluation context W
vp_status enqueue_forces(vp_system *s, Work &W, const float *x_dev, float *f_dev, double *energy_dev,
                         double t, hipStream_t st);
// sets the message of vp_last_error and returns st
vp_status set_error(vp_status st, const std::string &msg);

}  // namespace vp
