// Forces of the potential U(X,Y) and the collective variable of the bias.
//
// k_forces: one thread per atom of the cell-sorted state.  The thread walks
// its full Verlet list (both members of every pair hold it, so no atomics and
// no cross-lane reductions are needed), evaluates potential-shifted LJ with
// Lorentz-Berthelot mixing plus reaction-field Coulomb in FP32 for members
// inside r_cut, adds the bonded terms it owns in FP64, and stores the total
// as 64-bit fixed point.  The list order is fixed by the deterministic sort,
// so the result does not depend on scheduling.
//
// k_cv: collective variable z and dz/dx of the solute (contact map: several
// workgroups per replica, each owning a range of solute rows; radius of
// gyration, constant force and no bias: one workgroup), with per-workgroup
// FP64 partial sums of z and of sum_i |dz/dx_i|^2/(gamma_i m_i) that the
// consumers reduce in a fixed order.
#include "vp_device.h"
#include "vp_launch.h"

namespace vp {

template <bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_forces(const RepInfo *__restrict__ info, Work W,
                                                   const int32_t *__restrict__ tile_rep,
                                                   const int32_t *__restrict__ tile_first,
                                                   int ntiles,
                                                   const int32_t *__restrict__ bt_start,
                                                   const BTerm *__restrict__ bterms) {
  __shared__ double s_red[kBlock / 64];
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  const int slot = R.off + p;
  const bool active = p < R.n;
  double elj = 0.0, erf = 0.0, ebond = 0.0, eangle = 0.0;
  long long fxs = 0, fys = 0, fzs = 0;
  if (active) {
    const float4 xi = W.xq[slot];
    const float2 pi = W.prm[slot];
    const int a = W.orig[slot];
    const float qi = (float)kCoulomb * xi.w;
    const float se24 = 24.0f * pi.y;
    const float sgi = pi.x;
    const float rc2 = R.rc2, krf2 = R.krf2;
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    const int cnt = W.nbcnt[slot];
    const uint16_t *lst = W.nblist + R.list_off + p;
    const float4 *xqr = W.xq + R.off;
    const float2 *prr = W.prm + R.off;
    const int npad = R.npad;
    for (int k = 0; k < cnt; ++k) {
      const int j = lst[(int64_t)k * npad];
      const float4 xj = xqr[j];
      const float2 pj = prr[j];
      float dx, dy, dz;
      const float r2 = pair_r2(xi, xj, R, dx, dy, dz);
      if (r2 < rc2) {
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r2inv = rinv * rinv;
        const float sg = sgi + pj.x;
        const float sr2 = sg * sg * r2inv;
        const float sr6 = sr2 * sr2 * sr2;
        const float e24 = se24 * pj.y;
        const float flj = e24 * sr6 * __builtin_fmaf(2.0f, sr6, -1.0f) * r2inv;
        const float qq = qi * xj.w;
        const float fc = qq * __builtin_fmaf(rinv, r2inv, -krf2);
        const float fs = flj + fc;
        fx = __builtin_fmaf(-fs, dx, fx);
        fy = __builtin_fmaf(-fs, dy, fy);
        fz = __builtin_fmaf(-fs, dz, fz);
        if (ENERGY) {
          const double sgd = (double)sg;
          const double s2c = sgd * sgd / (R.rc * R.rc);
          const double s6c = s2c * s2c * s2c;
          const double e4 = (double)e24 * (1.0 / 6.0);
          elj += e4 * ((double)sr6 * sr6 - sr6) - e4 * (s6c * s6c - s6c);
          erf += (double)qq * ((double)rinv + R.krf * (double)r2 - R.krf * R.rc * R.rc - 1.0 / R.rc);
        }
      }
    }
    // bonded terms owned by this atom (FP64)
    double bx = 0.0, by = 0.0, bz = 0.0;
    const int ga = R.uoff + a;
    const int t0 = bt_start[ga], t1 = bt_start[ga + 1];
    for (int t = t0; t < t1; ++t) {
      const BTerm T = bterms[t];
      if (T.kind == 0) {
        const float4 xb = W.xq[W.inv[R.uoff + T.a]];
        const double d0 = (double)xb.x - xi.x, d1 = (double)xb.y - xi.y, d2 = (double)xb.z - xi.z;
        const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double g = T.k * (rr - T.r0) / rr;
        bx += g * d0;
        by += g * d1;
        bz += g * d2;
        if (ENERGY) ebond += 0.25 * T.k * (rr - T.r0) * (rr - T.r0);  // owned by both atoms
      } else {
        // angle end--vertex--end; this atom is an end (kind 1) or the vertex (kind 2)
        float4 pa, pc, pb;
        if (T.kind == 1) {
          pa = xi;
          pc = W.xq[W.inv[R.uoff + T.a]];
          pb = W.xq[W.inv[R.uoff + T.b]];
        } else {
          pa = W.xq[W.inv[R.uoff + T.a]];
          pc = xi;
          pb = W.xq[W.inv[R.uoff + T.b]];
        }
        const double u0 = (double)pa.x - pc.x, u1 = (double)pa.y - pc.y, u2 = (double)pa.z - pc.z;
        const double w0 = (double)pb.x - pc.x, w1 = (double)pb.y - pc.y, w2 = (double)pb.z - pc.z;
        const double uu = u0 * u0 + u1 * u1 + u2 * u2, ww = w0 * w0 + w1 * w1 + w2 * w2;
        const double uw = u0 * w0 + u1 * w1 + u2 * w2;
        const double nn = sqrt(uu * ww);
        double cs = uw / nn;
        cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
        const double th = acos(cs);
        double sn = sqrt(1.0 - cs * cs);
        sn = sn < 1e-12 ? 1e-12 : sn;
        const double dv = T.k * (th - T.r0) / sn;
        if (T.kind == 1) {
          bx += dv * (w0 / nn - cs * u0 / uu);
          by += dv * (w1 / nn - cs * u1 / uu);
          bz += dv * (w2 / nn - cs * u2 / uu);
        } else {
          bx -= dv * (w0 / nn - cs * u0 / uu + u0 / nn - cs * w0 / ww);
          by -= dv * (w1 / nn - cs * u1 / uu + u1 / nn - cs * w1 / ww);
          bz -= dv * (w2 / nn - cs * u2 / uu + u2 / nn - cs * w2 / ww);
        }
        if (ENERGY) eangle += (0.5 / 3.0) * T.k * (th - T.r0) * (th - T.r0);  // owned by 3 atoms
      }
    }
    fxs = to_fix((double)fx + bx);
    fys = to_fix((double)fy + by);
    fzs = to_fix((double)fz + bz);
  }
  if (p < R.npad) {
    W.F[slot] = fxs;
    W.F[W.fstride + slot] = fys;
    W.F[2 * W.fstride + slot] = fzs;
  }
  if (ENERGY) {
    double v0 = block_sum<kBlock>(0.5 * elj, s_red);
    double v1 = block_sum<kBlock>(0.5 * erf, s_red);
    double v2 = block_sum<kBlock>(ebond, s_red);
    double v3 = block_sum<kBlock>(eangle, s_red);
    if (threadIdx.x == 0) {
      W.epart[4 * (size_t)tile + 0] = v0;
      W.epart[4 * (size_t)tile + 1] = v1;
      W.epart[4 * (size_t)tile + 2] = v2;
      W.epart[4 * (size_t)tile + 3] = v3;
    }
  }
}

// ---------------------------------------------------------------------------
// collective variable of the bias
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCvBlock) void k_cv(const RepInfo *__restrict__ info, Work W,
                                                 const float *__restrict__ cmap,
                                                 const double *__restrict__ igm0,
                                                 const double *__restrict__ mass0,
                                                 const float4 *__restrict__ cforce, int inc_step,
                                                 long long *__restrict__ step) {
  extern __shared__ float4 s_x[];  // solute positions of this replica
  __shared__ double s_red[kCvBlock / 64];
  __shared__ double s_cm[5];
  const int r = blockIdx.y, b = blockIdx.x;
  const RepInfo &R = info[r];
  const int tid = threadIdx.x;
  const int ns = R.ns;
  const bool contact = (R.bias == VP_BIAS_CONTACT || R.bias == VP_BIAS_RMD_CONTACT);
  if (b < R.cv_blocks) {
    double zacc = 0.0, gq = 0.0;
    if (contact) {
      for (int a = tid; a < ns; a += kCvBlock) s_x[a] = W.xq[W.inv[R.uoff + a]];
      __syncthreads();
      const int i = b * kCvBlock + tid;
      if (i < ns) {
        const float4 xi = s_x[i];
        const float *cf = cmap + R.cmap_off + i;
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        const int msep = R.min_sep;
        for (int j = 0; j < ns; ++j) {
          if (abs(j - i) <= msep) continue;
          const float4 xj = s_x[j];
          const float dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
          const float rr = sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
          float dc;
          const float c = contact_value(rr, R.cr0, R.crs, R.crc, dc);
          const float diff = c - cf[(int64_t)j * ns];
          if (j > i) zacc += (double)diff * (double)diff;
          const float coef = 2.0f * diff * dc / rr;  // dz/dr_ij / r_ij
          gx = __builtin_fmaf(-coef, dx, gx);
          gy = __builtin_fmaf(-coef, dy, gy);
          gz = __builtin_fmaf(-coef, dz, gz);
        }
        W.g[R.sol_off + i] = make_float4(gx, gy, gz, 0.0f);
        gq = ((double)gx * gx + (double)gy * gy + (double)gz * gz) * igm0[R.uoff + i];
      }
    } else if (R.bias == VP_BIAS_RG) {
      // mass-weighted radius of gyration on unwrapped coordinates
      double m = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
      for (int a = tid; a < ns; a += kCvBlock) {
        const float4 x = W.xq[W.inv[R.uoff + a]];
        s_x[a] = x;
        const double ma = mass0[R.uoff + a];
        m += ma;
        cx += ma * x.x;
        cy += ma * x.y;
        cz += ma * x.z;
      }
      double M = block_sum<kCvBlock>(m, s_red);
      double X = block_sum<kCvBlock>(cx, s_red);
      double Y = block_sum<kCvBlock>(cy, s_red);
      double Z = block_sum<kCvBlock>(cz, s_red);
      if (tid == 0) {
        s_cm[0] = X / M;
        s_cm[1] = Y / M;
        s_cm[2] = Z / M;
        s_cm[4] = M;
      }
      __syncthreads();
      M = s_cm[4];  // block_sum leaves the total in thread 0 only
      double q = 0.0;
      for (int a = tid; a < ns; a += kCvBlock) {
        const float4 x = s_x[a];
        const double d0 = x.x - s_cm[0], d1 = x.y - s_cm[1], d2 = x.z - s_cm[2];
        q += mass0[R.uoff + a] * (d0 * d0 + d1 * d1 + d2 * d2);
      }
      double Q = block_sum<kCvBlock>(q, s_red);
      if (tid == 0) s_cm[3] = sqrt(Q / M);  // Rg
      __syncthreads();
      const double rg = s_cm[3];
      for (int a = tid; a < ns; a += kCvBlock) {
        const float4 x = s_x[a];
        const double w = mass0[R.uoff + a] / (M * rg);
        const double g0 = w * (x.x - s_cm[0]), g1 = w * (x.y - s_cm[1]), g2 = w * (x.z - s_cm[2]);
        W.g[R.sol_off + a] = make_float4((float)g0, (float)g1, (float)g2, 0.0f);
        gq += (g0 * g0 + g1 * g1 + g2 * g2) * igm0[R.uoff + a];
      }
      zacc = (tid == 0) ? rg : 0.0;
    } else if (R.bias == VP_BIAS_CONST) {
      for (int a = tid; a < ns; a += kCvBlock) {
        const float4 f = cforce[R.sol_off + a];
        W.g[R.sol_off + a] = f;
        gq += ((double)f.x * f.x + (double)f.y * f.y + (double)f.z * f.z) * igm0[R.uoff + a];
      }
    }
    const double zs = block_sum<kCvBlock>(zacc, s_red);
    const double gs = block_sum<kCvBlock>(gq, s_red);
    if (tid == 0) {
      W.zpart[(size_t)r * kMaxCvBlocks + b] = zs;
      W.gpart[(size_t)r * kMaxCvBlocks + b] = gs;
    }
  }
  if (inc_step && r == 0 && b == 0 && tid == 0) *step += 1;
}

// replica scalars from the CV partials (fixed order)
__device__ __forceinline__ void cv_sums(const RepInfo &R, const Work &W, int r, double &z,
                                        double &G) {
  z = 0.0;
  G = 0.0;
  for (int b = 0; b < R.cv_blocks; ++b) {
    z += W.zpart[(size_t)r * kMaxCvBlocks + b];
    G += W.gpart[(size_t)r * kMaxCvBlocks + b];
  }
}

// vp_forces output: total force (fixed point + bias) in user order.
__global__ __launch_bounds__(kBlock) void k_force_out(const RepInfo *__restrict__ info,
                                                      const RepState *__restrict__ state, Work W,
                                                      const int32_t *__restrict__ tile_rep,
                                                      const int32_t *__restrict__ tile_first,
                                                      int ntiles, double t,
                                                      float *__restrict__ f_user) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  if (p >= R.n) return;
  const int slot = R.off + p;
  double z, G, zr, ub;
  cv_sums(R, W, r, z, G);
  const RepState &S = state[r];
  const double c = bias_coef(R, z, S.z0, S.z_m, t, false, zr, ub);
  const int a = W.orig[slot];
  double f0 = from_fix(W.F[slot]), f1 = from_fix(W.F[W.fstride + slot]),
         f2 = from_fix(W.F[2 * W.fstride + slot]);
  if (a < R.ns && c != 0.0) {
    const float4 g = W.g[R.sol_off + a];
    f0 += c * g.x;
    f1 += c * g.y;
    f2 += c * g.z;
  }
  float *o = f_user + 3ll * (R.uoff + a);
  o[0] = (float)f0;
  o[1] = (float)f1;
  o[2] = (float)f2;
}

// energy columns: LJ, RF, bond, angle, bias, z, z_ref, S
__global__ void k_energy_out(const RepInfo *__restrict__ info, const RepState *__restrict__ state,
                             Work W, double t, double *__restrict__ e_out) {
  const int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  const RepInfo &R = info[r];
  double e[4] = {0, 0, 0, 0};
  for (int tt = R.tile0; tt < R.tile0 + R.ntiles; ++tt)
    for (int k = 0; k < 4; ++k) e[k] += W.epart[4 * (size_t)tt + k];
  double z, G, zr, ub;
  cv_sums(R, W, r, z, G);
  const RepState &S = state[r];
  const double c = bias_coef(R, z, S.z0, S.z_m, t, false, zr, ub);
  double *o = e_out + 8 * (size_t)r;
  o[0] = e[0];
  o[1] = e[1];
  o[2] = e[2];
  o[3] = e[3];
  o[4] = ub;
  o[5] = (R.bias == VP_BIAS_CONST || R.bias == VP_BIAS_NONE) ? 0.0 : z;
  o[6] = zr;
  o[7] = c * c * G;
}

// native contact map of the product X_f: cmap[i][j] = C~(|xf_j - xf_i|) for
// |i - j| > min_sep, else 0 (symmetric, so a row read by lane i is coalesced)
__global__ void k_native_map(const float *__restrict__ xf, int ns, int min_sep, float r0, float rs,
                             float rc, float *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)ns * ns) return;
  const int i = (int)(k / ns), j = (int)(k % ns);
  float v = 0.0f;
  if (abs(i - j) > min_sep) {
    const float dx = xf[3 * j] - xf[3 * i], dy = xf[3 * j + 1] - xf[3 * i + 1],
                dz = xf[3 * j + 2] - xf[3 * i + 2];
    const float rr = sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
    float dc;
    v = contact_value(rr, r0, rs, rc, dc);
  }
  out[k] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_native_map(const float *xf, int ns, int min_sep, float r0, float rs, float rc,
                       float *out, hipStream_t st) {
  int64_t n = (int64_t)ns * ns;
  hipLaunchKernelGGL(k_native_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xf, ns,
                     min_sep, r0, rs, rc, out);
}

static inline int xcd_grid(int nb) { return 8 * ((nb + 7) / 8); }

void launch_forces(vp_system *s, Work &W, bool energy, hipStream_t st) {
  if (energy)
    hipLaunchKernelGGL(k_forces<true>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       W, s->tile_rep, s->tile_first, s->n_tiles, s->bt_start, s->bterms);
  else
    hipLaunchKernelGGL(k_forces<false>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       W, s->tile_rep, s->tile_first, s->n_tiles, s->bt_start, s->bterms);
}

void launch_cv(vp_system *s, Work &W, int inc_step, hipStream_t st) {
  int gx = 1, nsmax = 1;
  for (const RepInfo &R : s->info_h) {
    gx = R.cv_blocks > gx ? R.cv_blocks : gx;
    nsmax = R.ns > nsmax ? R.ns : nsmax;
  }
  size_t lds = sizeof(float4) * (size_t)nsmax;
  hipLaunchKernelGGL(k_cv, dim3(gx, s->R), dim3(kCvBlock), lds, st, s->info, W, s->cmap, s->igm0,
                     s->mass0, s->cforce, inc_step, s->step);
}

void launch_force_out(vp_system *s, Work &W, double t, float *f_user, double *e_out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_force_out, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                     s->state, W, s->tile_rep, s->tile_first, s->n_tiles, t, f_user);
  if (e_out)
    hipLaunchKernelGGL(k_energy_out, dim3(s->R), dim3(64), 0, st, s->info, s->state, W, t, e_out);
}

}  // namespace vp
