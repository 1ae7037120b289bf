// BAOAB splitting of the Langevin equations (Eq. Lang) with Philox noise, and
// the running functional of every replica.
//
// One step n -> n+1 is split over two launches so that the forces of the new
// positions sit between them:
//   START:   v += dt/2 F_n/m; x += dt/2 v; v = c1 v + sigma_v g(seed, atom, n);
//            x += dt/2 v                            (then list, forces, CV)
//   FINISH:  v += dt/2 F_{n+1}/m; Phi_acc += S_{n+1}
// where F includes the bias c * dz/dx on solute atoms (c from bias_coef) and
// S = c^2 sum_i |dz/dx_i|^2/(gamma_i m_i) = sum_i |F_i^bias|^2/(gamma_i m_i).
// A FINISH and the next START are fused into one launch inside a block of
// steps.  INIT evaluates S_0 at creation (Phi_acc = S_0/2: trapezoid weight).
// A replica whose status has a flag (unstable, or a pair list that overflowed)
// is frozen.  On record steps (nst_out > 0 divides the completed step) FINISH
// also leaves each tile's kinetic energy of the completed velocities in
// ke_tile for the energy record.
#include "vp_device.h"
#include "vp_launch.h"

namespace vp {

enum { MODE_FINISH = 1, MODE_START = 2, MODE_INIT = 4 };

// With TAN, the same steps carry the tangents xi_p = dx/dtheta_p and
// eta_p = dv/dtheta_p (theta = (bias_k, ramp_rate), the noise held fixed):
//   B: eta += dt/2 dF_p/m;  A: xi += dt/2 eta;  O: eta = c1 eta;  A: xi += dt/2 eta,
// where dF_p = -H_U xi_p + (dc/dz dz_p + dc/dtheta_p) g + c (d g)[xi_p] on
// solute atoms, and the derivative of Phi accumulates
//   dS_p = 2 c dc_p G + c^2 dG_p   (trapezoid weights as for Phi).
template <int MODE, bool TAN>
__global__ __launch_bounds__(kBlock) void k_integrate(const RepInfo *__restrict__ info,
                                                      RepState *__restrict__ state, Work W,
                                                      const int32_t *__restrict__ tile_rep,
                                                      const int32_t *__restrict__ tile_first,
                                                      int ntiles,
                                                      const long long *__restrict__ step,
                                                      const double *__restrict__ mass0, int nst_out) {
  __shared__ float s_max[kBlock / 64];
  __shared__ double s_red[kBlock / 64];
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  RepState &S = state[r];
  const int p = tile_first[tile] + threadIdx.x;
  const int slot = R.off + p;
  const long long n = *step;
  const double t = (double)n * R.dt;
  double z, G, zr, ub;
  {
    z = 0.0;
    G = 0.0;
    for (int b = 0; b < R.cv_blocks; ++b) {
      z += W.zpart[(size_t)r * kMaxCvBlocks + b];
      G += W.gpart[(size_t)r * kMaxCvBlocks + b];
    }
  }
  const bool init = (MODE & MODE_INIT) != 0;
  const double c = bias_coef(R, z, S.z0, S.z_m, t, init, zr, ub);
  double cd[2] = {0.0, 0.0};  // total dc/dtheta_p
  if (TAN) {
    double dcdz, dcdth[2];
    bias_coef_deriv(R, z, S.z0, t, init, dcdz, dcdth);
    double zd[2] = {0.0, 0.0}, gd[2] = {0.0, 0.0};
    for (int b = 0; b < R.cv_blocks; ++b)
      for (int d = 0; d < 2; ++d) {
        zd[d] += W.tzpart[((size_t)r * kMaxCvBlocks + b) * 2 + d];
        gd[d] += W.tgpart[((size_t)r * kMaxCvBlocks + b) * 2 + d];
      }
    for (int d = 0; d < 2; ++d) cd[d] = dcdz * zd[d] + dcdth[d];
    if (p == 0 && (MODE & (MODE_INIT | MODE_FINISH)) && !S.status) {
      for (int d = 0; d < 2; ++d) {
        const double sd = 2.0 * c * cd[d] * G + c * c * gd[d];
        S.pd_acc[d] = init ? 0.5 * sd : S.pd_acc[d] + sd;
        S.pd_last[d] = sd;
      }
    }
  }
  if (p == 0 && (MODE & (MODE_INIT | MODE_FINISH))) {
    const double Sn = c * c * G;
    if (init) {
      S.z0 = z;
      S.z_m = z;
      S.phi_acc = 0.5 * Sn;
    } else {
      S.phi_acc += Sn;
      if (R.bias == VP_BIAS_RMD_CONTACT && z < S.z_m) S.z_m = z;
    }
    S.s_last = Sn;
    S.z_last = z;
    S.zref_last = zr;
  }
  if (init) return;
  float disp = 0.0f;
  const bool rec = (MODE & MODE_FINISH) && nst_out > 0 && n % nst_out == 0;  // uniform
  double ke = 0.0;
  const int status = S.status;
  if (rec && p < R.n && status) {  // a frozen replica keeps its velocities
    const float4 v = W.vel[slot];
    ke = 0.5 * mass0[R.uoff + W.orig[slot]] * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
  }
  if (p < R.n && !status) {
    const int a = W.orig[slot];
    double f0 = from_fix(W.F[slot]), f1 = from_fix(W.F[W.fstride + slot]),
           f2 = from_fix(W.F[2 * W.fstride + slot]);
    if (a < R.ns && c != 0.0) {
      const float4 g = W.g[R.sol_off + a];
      f0 += c * g.x;
      f1 += c * g.y;
      f2 += c * g.z;
    }
    const bool bad = !(fabs(f0) <= kForceLimit && fabs(f1) <= kForceLimit && fabs(f2) <= kForceLimit);
    if (bad) {
      atomicOr(&S.status, VP_REPLICA_UNSTABLE);
    } else {
      const float4 ig = W.integ[slot];  // 1/m, c1, sigma_v
      const float hdt = 0.5f * (float)R.dt;
      const float kx = hdt * ig.x * (float)f0, ky = hdt * ig.x * (float)f1, kz = hdt * ig.x * (float)f2;
      float4 v = W.vel[slot];
      if (MODE & MODE_FINISH) {
        v.x += kx;
        v.y += ky;
        v.z += kz;
        if (rec) ke = 0.5 * mass0[R.uoff + a] * ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
      }
      if (MODE & MODE_START) {
        // positions are fixed point (unit 2^-22 nm): each drift is rounded once
        int4 x = W.xq[slot];
        const float hq = hdt * kQf;
        v.x += kx;
        v.y += ky;
        v.z += kz;
        x.x += __float2int_rn(hq * v.x);
        x.y += __float2int_rn(hq * v.y);
        x.z += __float2int_rn(hq * v.z);
        const float3 g = noise3(R.seed, (uint32_t)a, (uint32_t)n, 0u);
        v.x = ig.y * v.x + ig.z * g.x;
        v.y = ig.y * v.y + ig.z * g.y;
        v.z = ig.y * v.z + ig.z * g.z;
        x.x += __float2int_rn(hq * v.x);
        x.y += __float2int_rn(hq * v.y);
        x.z += __float2int_rn(hq * v.z);
        W.xq[slot] = x;
        const int4 x0 = W.xref[slot];
        const float ex = (float)(x.x - x0.x) * kInvQf, ey = (float)(x.y - x0.y) * kInvQf,
                    ez = (float)(x.z - x0.z) * kInvQf;
        disp = sqrtf(ex * ex + ey * ey + ez * ez);
      }
      W.vel[slot] = v;
      if (TAN) {
        for (int d = 0; d < 2; ++d) {
          const float4 h = W.tf[d * W.fstride + slot];
          double q0 = h.x, q1 = h.y, q2 = h.z;
          if (a < R.ns) {
            const float4 g = W.g[R.sol_off + a];
            const float4 dg = W.tg[d * W.solstride + R.sol_off + a];
            q0 += cd[d] * g.x + c * dg.x;
            q1 += cd[d] * g.y + c * dg.y;
            q2 += cd[d] * g.z + c * dg.z;
          }
          const float hx = hdt * ig.x * (float)q0, hy = hdt * ig.x * (float)q1, hz = hdt * ig.x * (float)q2;
          float4 e = W.tv[d * W.fstride + slot];
          if (MODE & MODE_FINISH) {
            e.x += hx;
            e.y += hy;
            e.z += hz;
          }
          if (MODE & MODE_START) {
            float4 xt = W.tx[d * W.fstride + slot];
            e.x += hx;
            e.y += hy;
            e.z += hz;
            xt.x += hdt * e.x;
            xt.y += hdt * e.y;
            xt.z += hdt * e.z;
            e.x *= ig.y;
            e.y *= ig.y;
            e.z *= ig.y;
            xt.x += hdt * e.x;
            xt.y += hdt * e.y;
            xt.z += hdt * e.z;
            W.tx[d * W.fstride + slot] = xt;
          }
          W.tv[d * W.fstride + slot] = e;
        }
      }
    }
  }
  if (rec) {
    const double k = block_sum<kBlock>(ke, s_red);
    if (threadIdx.x == 0) W.ke_tile[tile] = k;
  }
  if (MODE & MODE_START) {
    disp = wave_max(disp);
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = disp;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = s_max[0];
      for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, s_max[w]);
      if (m > 0.0f) atomicMax(&S.maxdisp_bits, __float_as_uint(m));
    }
  }
}

// Initial state in user order -> identity slots; positions already in fixed
// point; velocities from v0 or from the Maxwell-Boltzmann distribution
// (noise tag 1 at step 0).
__global__ __launch_bounds__(kBlock) void k_init_state(const RepInfo *__restrict__ info, Work W,
                                                       const int32_t *__restrict__ tile_rep,
                                                       const int32_t *__restrict__ tile_first,
                                                       int ntiles, const int32_t *__restrict__ type0,
                                                       const float4 *__restrict__ integ0,
                                                       const double *__restrict__ mass0,
                                                       const int32_t *__restrict__ xq_user,
                                                       const float *__restrict__ v_user,
                                                       const uint8_t *__restrict__ has_v) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  const int slot = R.off + p;
  if (p >= R.npad) return;
  if (W.tx) {
    for (int d = 0; d < 2; ++d) {
      W.tx[d * W.fstride + slot] = make_float4(0.f, 0.f, 0.f, 0.f);
      W.tv[d * W.fstride + slot] = make_float4(0.f, 0.f, 0.f, 0.f);
      W.tf[d * W.fstride + slot] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  if (p >= R.n) {
    W.xq[slot] = make_int4(0, 0, 0, R.ntypes);
    W.vel[slot] = make_float4(0.f, 0.f, 0.f, 0.f);
    W.orig[slot] = -1;
    W.wrap[slot] = 0;
    W.integ[slot] = make_float4(0.f, 0.f, 0.f, 0.f);
    W.nbcnt[slot] = 0;
    W.nblj[slot] = 0;
    return;
  }
  const int u = R.uoff + p;
  const int32_t *xu = xq_user + 3ll * u;
  W.xq[slot] = make_int4(xu[0], xu[1], xu[2], type0[u]);
  W.xref[slot] = W.xq[slot];
  W.orig[slot] = p;
  W.wrap[slot] = 0;
  W.inv[u] = slot;
  W.integ[slot] = integ0[u];
  if (has_v[r]) {
    const float *vu = v_user + 3ll * u;
    W.vel[slot] = make_float4(vu[0], vu[1], vu[2], 0.f);
  } else {
    const float3 g = noise3(R.seed, (uint32_t)p, 0u, 1u);
    const float sd = (float)sqrt(R.kT / mass0[u]);
    W.vel[slot] = make_float4(sd * g.x, sd * g.y, sd * g.z, 0.f);
  }
}

// Positions and velocities in user order.
__global__ __launch_bounds__(kBlock) void k_gather_state(const RepInfo *__restrict__ info, Work W,
                                                         const int32_t *__restrict__ tile_rep,
                                                         const int32_t *__restrict__ tile_first,
                                                         int ntiles, float *__restrict__ x_out,
                                                         float *__restrict__ v_out) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  if (p >= R.n) return;
  const int slot = R.off + p;
  const int u = R.uoff + W.orig[slot];
  const int4 x = W.xq[slot];
  const float4 v = W.vel[slot];
  if (x_out) {
    x_out[3ll * u] = (float)((double)x.x * kInvQ);
    x_out[3ll * u + 1] = (float)((double)x.y * kInvQ);
    x_out[3ll * u + 2] = (float)((double)x.z * kInvQ);
  }
  if (v_out) {
    v_out[3ll * u] = v.x;
    v_out[3ll * u + 1] = v.y;
    v_out[3ll * u + 2] = v.z;
  }
}

// Exact trajectory state in user order, FP64: positions (grid values),
// velocities and, when derivatives are on, the tangents [2][users][3].
__global__ __launch_bounds__(kBlock) void k_export_state(const RepInfo *__restrict__ info, Work W,
                                                         const int32_t *__restrict__ tile_rep,
                                                         const int32_t *__restrict__ tile_first,
                                                         int ntiles, int64_t users,
                                                         double *__restrict__ x_out,
                                                         double *__restrict__ v_out,
                                                         double *__restrict__ xt_out,
                                                         double *__restrict__ vt_out) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  if (p >= R.n) return;
  const int slot = R.off + p;
  const int64_t u = R.uoff + W.orig[slot];
  const int4 x = W.xq[slot];
  const float4 v = W.vel[slot];
  x_out[3 * u] = (double)x.x * kInvQ;
  x_out[3 * u + 1] = (double)x.y * kInvQ;
  x_out[3 * u + 2] = (double)x.z * kInvQ;
  v_out[3 * u] = v.x;
  v_out[3 * u + 1] = v.y;
  v_out[3 * u + 2] = v.z;
  if (xt_out && W.tx)
    for (int d = 0; d < 2; ++d) {
      const float4 a = W.tx[d * W.fstride + slot], b = W.tv[d * W.fstride + slot];
      double *xo = xt_out + (size_t)d * 3 * users + 3 * u, *vo = vt_out + (size_t)d * 3 * users + 3 * u;
      xo[0] = a.x;
      xo[1] = a.y;
      xo[2] = a.z;
      vo[0] = b.x;
      vo[1] = b.y;
      vo[2] = b.z;
    }
}

// Kinetic energy partials per tile (fixed-order reduction on the host).
__global__ __launch_bounds__(kBlock) void k_kinetic(const RepInfo *__restrict__ info, Work W,
                                                    const int32_t *__restrict__ tile_rep,
                                                    const int32_t *__restrict__ tile_first,
                                                    int ntiles, const double *__restrict__ mass0,
                                                    double *__restrict__ out) {
  __shared__ double s_red[kBlock / 64];
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  double ke = 0.0;
  if (p < R.n) {
    const int slot = R.off + p;
    const float4 v = W.vel[slot];
    ke = 0.5 * mass0[R.uoff + W.orig[slot]] *
         ((double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z);
  }
  const double s = block_sum<kBlock>(ke, s_red);
  if (threadIdx.x == 0) out[tile] = s;
}

__global__ void k_debug_noise(uint64_t seed, uint32_t atom0, uint32_t step, uint32_t tag, int n,
                              float *__restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float u0;
  const float3 g = noise3(seed, atom0 + (uint32_t)k, step, tag, &u0);
  out[4 * k] = g.x;
  out[4 * k + 1] = g.y;
  out[4 * k + 2] = g.z;
  out[4 * k + 3] = u0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int xcd_grid(int nb) { return 8 * ((nb + 7) / 8); }

template <bool TAN>
static void launch_integrate_t(vp_system *s, int mode, hipStream_t st) {
  dim3 g(xcd_grid(s->n_tiles)), b(kBlock);
  Work &W = s->traj;
  const int nout = s->opt.nst_out;
  switch (mode) {
    case MODE_START:
      hipLaunchKernelGGL((k_integrate<MODE_START, TAN>), g, b, 0, st, s->info, s->state, W,
                         s->tile_rep, s->tile_first, s->n_tiles, s->step, s->mass0, nout);
      break;
    case MODE_FINISH:
      hipLaunchKernelGGL((k_integrate<MODE_FINISH, TAN>), g, b, 0, st, s->info, s->state, W,
                         s->tile_rep, s->tile_first, s->n_tiles, s->step, s->mass0, nout);
      break;
    case MODE_FINISH | MODE_START:
      hipLaunchKernelGGL((k_integrate<MODE_FINISH | MODE_START, TAN>), g, b, 0, st, s->info,
                         s->state, W, s->tile_rep, s->tile_first, s->n_tiles, s->step, s->mass0, nout);
      break;
    default:
      hipLaunchKernelGGL((k_integrate<MODE_INIT, TAN>), g, b, 0, st, s->info, s->state, W,
                         s->tile_rep, s->tile_first, s->n_tiles, s->step, s->mass0, nout);
  }
}

void launch_integrate(vp_system *s, int mode, hipStream_t st) {
  if (s->tangent)
    launch_integrate_t<true>(s, mode, st);
  else
    launch_integrate_t<false>(s, mode, st);
}

void launch_init_state(vp_system *s, const int32_t *xq_user, const float *v_user,
                       const uint8_t *has_v, hipStream_t st) {
  hipLaunchKernelGGL(k_init_state, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                     s->traj, s->tile_rep, s->tile_first, s->n_tiles, s->type0, s->integ0,
                     s->mass0, xq_user, v_user, has_v);
}

void launch_gather_state(vp_system *s, float *x_out, float *v_out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_state, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                     s->traj, s->tile_rep, s->tile_first, s->n_tiles, x_out, v_out);
}

void launch_export_state(vp_system *s, double *x, double *v, double *xt, double *vt, hipStream_t st) {
  hipLaunchKernelGGL(k_export_state, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info, s->traj,
                     s->tile_rep, s->tile_first, s->n_tiles, (int64_t)s->n_users, x, v, xt, vt);
}

void launch_kinetic(vp_system *s, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_kinetic, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info, s->traj,
                     s->tile_rep, s->tile_first, s->n_tiles, s->mass0, out);
}

void launch_debug_noise(uint64_t seed, uint32_t atom0, uint32_t step, uint32_t tag, int n,
                        float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_debug_noise, dim3((n + 255) / 256), dim3(256), 0, st, seed, atom0, step, tag,
                     n, out);
}

}  // namespace vp
