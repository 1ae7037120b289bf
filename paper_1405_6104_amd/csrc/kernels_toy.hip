// Trial paths of the toy model (supplement, "Illustrative Application in a
// Toy Model"): one point particle per thread on the 2-D surface
//   U(x,y) = w^2 r^4 - A1 s1^2/(r^2+s1^2)^2 + A2 s2^2/(r^2+s2^2)^2
//            - A3 s3^2/((x-xm)^2+(y-ym)^2+s3^2)^2,   r^2 = x^2 + y^2,
// integrated with the BAOAB splitting of the Langevin equation (as for the
// atomistic trials), under no bias, the ratchet of Eq. VR on z = r, or the
// steering force -K z grad z, accumulating the functional of Eq.
// VMDcondition (trapezoid rule, 1/(4 kT) prefactor).  Everything is FP64 with
// products and sums rounded separately (no fused multiply-add), so that a
// trial follows the reference arithmetic closely.  The trials are
// independent: a launch holds all of them and each thread keeps its particle
// in registers for the whole run.
#include <hip/hip_runtime.h>

#include "vp_device.h"
#include "vp_launch.h"

namespace vp {

// Two standard normals (Box-Muller, FP64) from Philox4x32-10 words of
// counter (0, step, tag, 0) under the trial's key.
__device__ __forceinline__ void normal2(uint64_t seed, uint32_t step, uint32_t tag, double &g0, double &g1) {
  const uint4 w = philox4x32_10(make_uint4(0u, step, tag, 0u), (uint32_t)seed, (uint32_t)(seed >> 32));
  const double u0 = (double)word_to_uniform(w.x), u1 = (double)word_to_uniform(w.y);
  const double rho = sqrt(-2.0 * log(u0));
  const double ang = 6.283185307179586 * u1;
  g0 = rho * cos(ang);
  g1 = rho * sin(ang);
}

__global__ __launch_bounds__(64) void k_toy(const vp_toy_params p, int n_trials,
                                            const int32_t *__restrict__ kind,
                                            const double *__restrict__ kbias,
                                            const uint64_t *__restrict__ seed,
                                            double *__restrict__ out, float *__restrict__ path) {
#pragma clang fp contract(off)
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_trials) return;
  const int kd = kind[t];
  const double K = kbias[t];
  const uint64_t key = seed[t];
  const double a1 = p.A1 * p.s1 * p.s1, a2 = p.A2 * p.s2 * p.s2, a3 = p.A3 * p.s3 * p.s3;
  const double s1q = p.s1 * p.s1, s2q = p.s2 * p.s2, s3q = p.s3 * p.s3, w2 = p.w * p.w;
  const double gm = p.gamma * p.mass;
  // force (potential + bias) at (x, y) with ratchet minimum zm; S = |F_bias|^2/(gamma m)
  auto force = [&](double x, double y, double zm, double &fx, double &fy) -> double {
    const double r2 = x * x + y * y;
    const double d1 = r2 + s1q, d2 = r2 + s2q;
    const double ex = x - p.xm, ey = y - p.ym;
    const double d3 = ex * ex + ey * ey + s3q;
    const double g = 2.0 * w2 * r2 + 2.0 * a1 / (d1 * d1 * d1) - 2.0 * a2 / (d2 * d2 * d2);
    const double h = 2.0 * a3 / (d3 * d3 * d3);
    fx = -(g * 2.0 * x + h * 2.0 * ex);
    fy = -(g * 2.0 * y + h * 2.0 * ey);
    double bx = 0.0, by = 0.0;
    if (kd == VP_TOY_RMD) {
      const double z = sqrt(r2);
      if (z > zm && z > 0.0) {
        const double c = -0.5 * K * (z - zm) / z;
        bx = c * x;
        by = c * y;
      }
    } else if (kd == VP_TOY_SMD) {
      bx = -K * x;
      by = -K * y;
    }
    fx += bx;
    fy += by;
    return (bx * bx + by * by) / gm;
  };
  double x = p.x0, y = p.y0, g0, g1;
  normal2(key, 0u, 1u, g0, g1);  // Maxwell velocities
  const double sd0 = sqrt(p.kT / p.mass);
  double vx = sd0 * g0, vy = sd0 * g1;
  const double dt = p.dt, m = p.mass;
  const double c1 = exp(-p.gamma * dt);
  const double sv = sqrt((1.0 - c1 * c1) * p.kT / m);
  double z = sqrt(x * x + y * y), zm = z;
  double fx, fy;
  double S = force(x, y, zm, fx, fy);
  double acc = 0.5 * S, s_last = S;
  long long t_reach = z <= p.r_product ? 0 : -1;
  double theta = z <= p.r_gate ? atan2(y, x) : NAN;
  const int stride = p.path_stride;
  const int nsamp = stride > 0 ? p.n_steps / stride + 1 : 0;
  if (path) {
    path[(size_t)t * nsamp * 2] = (float)x;
    path[(size_t)t * nsamp * 2 + 1] = (float)y;
  }
  for (int n = 0; n < p.n_steps; ++n) {
    normal2(key, (uint32_t)n, 2u, g0, g1);
    vx += 0.5 * dt * fx / m;
    vy += 0.5 * dt * fy / m;
    x += 0.5 * dt * vx;
    y += 0.5 * dt * vy;
    vx = c1 * vx + sv * g0;
    vy = c1 * vy + sv * g1;
    x += 0.5 * dt * vx;
    y += 0.5 * dt * vy;
    z = sqrt(x * x + y * y);
    if (kd == VP_TOY_RMD && z < zm) zm = z;  // before the force (Eq. VR)
    S = force(x, y, zm, fx, fy);
    vx += 0.5 * dt * fx / m;
    vy += 0.5 * dt * fy / m;
    acc += S;
    s_last = S;
    if (t_reach < 0 && z <= p.r_product) t_reach = n + 1;
    if (theta != theta && z <= p.r_gate) theta = atan2(y, x);
    if (path && (n + 1) % stride == 0) {
      const size_t k = (size_t)t * nsamp + (size_t)((n + 1) / stride);
      path[2 * k] = (float)x;
      path[2 * k + 1] = (float)y;
    }
  }
  double *o = out + (size_t)t * VP_TOY_COUNT;
  o[VP_TOY_PHI] = (acc - 0.5 * s_last) * dt / (4.0 * p.kT);
  o[VP_TOY_REACHED] = t_reach >= 0 ? 1.0 : 0.0;
  o[VP_TOY_T_REACH] = (double)t_reach;
  o[VP_TOY_X] = x;
  o[VP_TOY_Y] = y;
  o[VP_TOY_ZMIN] = kd == VP_TOY_RMD ? zm : NAN;
  o[VP_TOY_THETA_GATE] = theta;
}

void launch_toy(const vp_toy_params &p, int n, const int32_t *kind, const double *k, const uint64_t *seed,
                double *out, float *path, hipStream_t st) {
  hipLaunchKernelGGL(k_toy, dim3((n + 63) / 64), dim3(64), 0, st, p, n, kind, k, seed, out, path);
}

}  // namespace vp
