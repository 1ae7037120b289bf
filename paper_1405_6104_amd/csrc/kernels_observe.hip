// Observables of the trajectories: energy records on output steps and the
// RMSD of each replica's solute from its product structure X_f.
//
// k_record   one thread per replica: the energy and virial partials that the
//            gated energy kernels left for the step just completed, the
//            kinetic energy partials of the integrator, Phi so far and the
//            status, as one record in the replica's ring of records.
// k_rmsd     one workgroup per replica: centroids, correlation matrix
//            S_ab = sum_i (x_i - x_c)_a (y_i - y_c)_b and the sums of squares in
//            FP64 (fixed-order block sums), then the least-squares rotation's
//            residual from the singular values of S (Kabsch): the largest trace
//            of R S over proper rotations R is s1 + s2 + sign(det S) s3, so
//            RMSD^2 = (sum |x_c|^2 + sum |y_c|^2 - 2 (s1 + s2 + sign(det S) s3)) / n.
//            The singular values come from a Jacobi eigen-decomposition of S^T S.
#include "vp_device.h"
#include "vp_launch.h"

namespace vp {

template <bool GATED>
__global__ void k_record(const RepInfo *__restrict__ info, RepState *__restrict__ state, Work W,
                         const long long *__restrict__ step, int nst_out, int cap,
                         double *__restrict__ records) {
  const long long n = *step;
  if (GATED && n % nst_out != 0) return;
  const int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  const RepInfo &R = info[r];
  RepState &S = state[r];
  double rec[VP_REC_COUNT];
  energy_columns(R, W, r, S.z0, S.z_m, (double)n * R.dt, rec);
  rec[VP_E_STATUS] = (double)S.status;
  rec[VP_REC_STEP] = (double)n;
  double ke = 0.0;
  for (int t = R.tile0; t < R.tile0 + R.ntiles; ++t) ke += W.ke_tile[t];
  rec[VP_REC_KE] = ke;
  rec[VP_REC_PHI] = S.status ? INFINITY : (S.phi_acc - 0.5 * S.s_last) * R.dt / (4.0 * R.kT);
  double *o = records + ((size_t)r * cap + (size_t)(S.n_records % cap)) * VP_REC_COUNT;
  for (int k = 0; k < VP_REC_COUNT; ++k) o[k] = rec[k];
  S.n_records += 1;
}

// cyclic Jacobi eigen-decomposition of a symmetric 3 x 3 matrix (values only)
__device__ void sym3_eigenvalues(double a[3][3], double lam[3]) {
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-34 * diag) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double kp = a[k][p], kq = a[k][q];
          a[k][p] = c * kp - s * kq;
          a[k][q] = s * kp + c * kq;
        }
        for (int k = 0; k < 3; ++k) {
          const double pk = a[p][k], qk = a[q][k];
          a[p][k] = c * pk - s * qk;
          a[q][k] = s * pk + c * qk;
        }
      }
  }
  for (int k = 0; k < 3; ++k) lam[k] = a[k][k];
}

__global__ __launch_bounds__(kCvBlock) void k_rmsd(const RepInfo *__restrict__ info, Work W,
                                                   const double *__restrict__ xf,
                                                   double *__restrict__ out) {
  __shared__ double s_red[kCvBlock / 64];
  __shared__ double s_c[6];
  const int r = blockIdx.x;
  const RepInfo &R = info[r];
  const int tid = threadIdx.x, ns = R.ns;
  if (R.xf_off < 0 || ns < 1) {
    if (tid == 0) out[r] = NAN;
    return;
  }
  const double *y = xf + 3 * (size_t)R.xf_off;
  auto pos = [&](int a, double x[3]) {  // unwrapped solute position in nm
    const int4 q = W.xq[W.inv[R.uoff + a]];
    x[0] = (double)q.x * kInvQ;
    x[1] = (double)q.y * kInvQ;
    x[2] = (double)q.z * kInvQ;
  };
  double c[6] = {0, 0, 0, 0, 0, 0};
  for (int a = tid; a < ns; a += kCvBlock) {
    double x[3];
    pos(a, x);
    for (int k = 0; k < 3; ++k) {
      c[k] += x[k];
      c[3 + k] += y[3 * a + k];
    }
  }
  for (int k = 0; k < 6; ++k) {
    const double v = block_sum<kCvBlock>(c[k], s_red);
    if (tid == 0) s_c[k] = v / ns;
  }
  __syncthreads();
  double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // S (row-major), then sum |x_c|^2 + |y_c|^2
  for (int a = tid; a < ns; a += kCvBlock) {
    double p[3], q[3];
    pos(a, p);
    for (int k = 0; k < 3; ++k) {
      p[k] -= s_c[k];
      q[k] = y[3 * a + k] - s_c[3 + k];
    }
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) m[3 * u + v] += p[u] * q[v];
    m[9] += p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  }
  double tot[10];
  for (int k = 0; k < 10; ++k) tot[k] = block_sum<kCvBlock>(m[k], s_red);
  if (tid != 0) return;
  double A[3][3];  // S^T S
  for (int u = 0; u < 3; ++u)
    for (int v = 0; v < 3; ++v) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += tot[3 * k + u] * tot[3 * k + v];
      A[u][v] = acc;
    }
  double lam[3];
  sym3_eigenvalues(A, lam);
  double sv[3];
  for (int k = 0; k < 3; ++k) sv[k] = sqrt(lam[k] > 0.0 ? lam[k] : 0.0);
  int lo = 0;  // the smallest singular value takes the sign of det S
  for (int k = 1; k < 3; ++k)
    if (sv[k] < sv[lo]) lo = k;
  const double det = tot[0] * (tot[4] * tot[8] - tot[5] * tot[7]) -
                     tot[1] * (tot[3] * tot[8] - tot[5] * tot[6]) +
                     tot[2] * (tot[3] * tot[7] - tot[4] * tot[6]);
  double tr = 0.0;
  for (int k = 0; k < 3; ++k) tr += (k == lo && det < 0.0) ? -sv[k] : sv[k];
  const double msd = (tot[9] - 2.0 * tr) / ns;
  out[r] = sqrt(msd > 0.0 ? msd : 0.0);
}

void launch_record(vp_system *s, bool gated, hipStream_t st) {
  const int nout = s->opt.nst_out > 0 ? s->opt.nst_out : 1;
  if (gated)
    hipLaunchKernelGGL(k_record<true>, dim3(s->R), dim3(64), 0, st, s->info, s->state, s->traj, s->step,
                       nout, s->out_cap, s->records);
  else
    hipLaunchKernelGGL(k_record<false>, dim3(s->R), dim3(64), 0, st, s->info, s->state, s->traj, s->step,
                       nout, s->out_cap, s->records);
}

void launch_rmsd(vp_system *s, hipStream_t st) {
  hipLaunchKernelGGL(k_rmsd, dim3(s->R), dim3(kCvBlock), 0, st, s->info, s->traj, s->xf, s->rmsd);
}

}  // namespace vp

namespace vp {

// First-formation step of every native contact not formed yet: formed when
// the squared integer distance of its two (unwrapped, same-molecule) atoms
// is at most (r0 in grid units)^2.  One thread per (contact, replica).
__global__ __launch_bounds__(256) void k_contact_form(const RepInfo *__restrict__ info, Work W,
                                                      const int2 *__restrict__ cpairs,
                                                      int32_t *__restrict__ t_form,
                                                      const long long *__restrict__ step) {
  const RepInfo &R = info[blockIdx.y];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= R.n_contacts) return;
  int32_t *tf = t_form + R.tf_off + k;
  if (*tf >= 0) return;
  const int2 pq = cpairs[R.cp_off + k];
  const int4 a = W.xq[W.inv[R.uoff + pq.x]], b = W.xq[W.inv[R.uoff + pq.y]];
  const long long dx = (long long)b.x - a.x, dy = (long long)b.y - a.y, dz = (long long)b.z - a.z;
  const unsigned long long d2 = (unsigned long long)(dx * dx) + (unsigned long long)(dy * dy) +
                                (unsigned long long)(dz * dz);
  if (d2 <= (unsigned long long)R.r0q2) *tf = (int32_t)*step;
}

// Concordant ordered contact pairs of two replicas with the same native
// contacts: count of (i, j), i != j, whose order entries M_ij (1, 0, 1/2 for
// formed before, after, together) agree; contacts not formed yet take the
// same, latest step.  One workgroup per replica pair; formation steps in LDS.
__global__ __launch_bounds__(256) void k_similarity(const RepInfo *__restrict__ info,
                                                    const int32_t *__restrict__ t_form,
                                                    const int2 *__restrict__ pr, int npairs,
                                                    unsigned long long *__restrict__ out) {
  extern __shared__ int32_t s_t[];  // [2][nc]
  __shared__ unsigned long long s_red[4];
  const int q = blockIdx.x;
  if (q >= npairs) return;
  const RepInfo &A = info[pr[q].x], &B = info[pr[q].y];
  const int nc = A.n_contacts;
  int32_t *ta = s_t, *tb = s_t + nc;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const int32_t a = t_form[A.tf_off + i], b = t_form[B.tf_off + i];
    ta[i] = a < 0 ? 0x7fffffff : a;
    tb[i] = b < 0 ? 0x7fffffff : b;
  }
  __syncthreads();
  unsigned long long same = 0;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const int32_t ai = ta[i], bi = tb[i];
    for (int j = 0; j < nc; ++j) {
      const int32_t aj = ta[j], bj = tb[j];
      const int ma = (ai < aj) ? 2 : (ai > aj ? 0 : 1);
      const int mb = (bi < bj) ? 2 : (bi > bj ? 0 : 1);
      same += (ma == mb && j != i) ? 1ull : 0ull;
    }
  }
  for (int o = 32; o > 0; o >>= 1) same += __shfl_xor(same, o, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = same;
  __syncthreads();
  if (threadIdx.x == 0) out[q] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

void launch_contact_form(vp_system *s, hipStream_t st) {
  const int nb = (s->max_contacts + 255) / 256;
  if (nb == 0) return;
  hipLaunchKernelGGL(k_contact_form, dim3(nb, s->R), dim3(256), 0, st, s->info, s->traj, s->cpairs, s->t_form,
                     s->step);
}

hipError_t prepare_similarity(int max_contacts) {
  return hipFuncSetAttribute((const void *)k_similarity, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(int32_t) * 2 * (size_t)max_contacts));
}

void launch_similarity(vp_system *s, const int2 *pr, int npairs, int max_contacts, unsigned long long *out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_similarity, dim3(npairs), dim3(256), sizeof(int32_t) * 2 * (size_t)max_contacts, st,
                     s->info, s->t_form, pr, npairs, out);
}

}  // namespace vp
