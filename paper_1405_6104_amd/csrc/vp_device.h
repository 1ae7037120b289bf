// Device helpers shared by the vp kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vp_internal.h"

namespace vp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter = (atom, step,
// tag, 0), key = 64-bit trajectory seed.  Ten rounds; the key advances by the
// two Weyl constants after every round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    uint32_t lo0 = m0 * c.x, hi0 = __umulhi(m0, c.x);
    uint32_t lo1 = m1 * c.z, hi1 = __umulhi(m1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Uniform in (0,1) from a 32-bit word: ((w >> 9) + 1/2) 2^-23, exact in FP32.
__device__ __forceinline__ float word_to_uniform(uint32_t w) {
  return ((float)(w >> 9) + 0.5f) * 1.1920928955078125e-7f;
}

// Three standard normals by Box-Muller: (g0, g1) from (u0, u1), g2 from (u2, u3).
__device__ __forceinline__ float3 noise3(uint64_t seed, uint32_t atom, uint32_t step, uint32_t tag,
                                         float *u0_out = nullptr) {
  uint4 w = philox4x32_10(make_uint4(atom, step, tag, 0u), (uint32_t)seed, (uint32_t)(seed >> 32));
  float u0 = word_to_uniform(w.x), u1 = word_to_uniform(w.y);
  float u2 = word_to_uniform(w.z), u3 = word_to_uniform(w.w);
  float rho = sqrtf(-2.0f * logf(u0));
  float s1, c1, s3, c3;
  sincospif(2.0f * u1, &s1, &c1);
  sincospif(2.0f * u3, &s3, &c3);
  if (u0_out) *u0_out = u0;
  return make_float3(rho * c1, rho * s1, sqrtf(-2.0f * logf(u2)) * c3);
}

// ---------------------------------------------------------------------------
// Pair membership on fixed-point coordinates (unit 2^-22 nm).  The integer
// difference of two images is exact; its single rounding to FP32 and the
// FMA chain below are the exact operation order the CPU test oracle uses:
//   d = fl(Xj - Xi - n Lq);  r2 = fma(dz, dz, fma(dy, dy, fl(dx * dx))).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ long long floordiv(long long a, long long b) {
  long long q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ float qr2(float dx, float dy, float dz) {
  float sq = dx * dx;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, sq));
}

// minimum image of an integer displacement (exact for |d| < L/2 + list radius)
__device__ __forceinline__ int qimage(int d, int Lq) {
  int n = (int)__builtin_rintf((float)d / (float)Lq);
  return d - n * Lq;
}

// ---------------------------------------------------------------------------
// Contact value of the collective variable: C = (1+u+u^2)/(1+u+u^2+u^3+u^4),
// u = (r/r0)^2 (the smooth form of (1-(r/r0)^6)/(1-(r/r0)^10)), times a
// quintic switch from 1 at rs to 0 at rc.  Returns C*S and d(C*S)/dr.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float contact_value(float r, float r0, float rs, float rc, float &dcdr) {
  float ir0 = 1.0f / r0;
  float u = (r * ir0) * (r * ir0);
  float u2 = u * u;
  float num = 1.0f + u + u2;
  float den = num + u2 * u + u2 * u2;
  float iden = 1.0f / den;
  float c = num * iden;
  float dnum = 1.0f + 2.0f * u;
  float dden = dnum + 3.0f * u2 + 4.0f * u2 * u;
  float dc = (dnum - c * dden) * iden * (2.0f * r * ir0 * ir0);
  float sw = 1.0f, dsw = 0.0f;
  if (r >= rc) {
    sw = 0.0f;
  } else if (r > rs) {
    float w = 1.0f / (rc - rs);
    float t = (r - rs) * w;
    sw = 1.0f - t * t * t * (10.0f - 15.0f * t + 6.0f * t * t);
    dsw = -30.0f * t * t * (1.0f - t) * (1.0f - t) * w;
  }
  dcdr = dc * sw + c * dsw;
  return c * sw;
}

// ---------------------------------------------------------------------------
// Fixed-point forces: round(F * 2^32) in int64, clamped to +-2^62.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long to_fix(double f) {
  double s = f * kFixScale;
  if (!(s > -4.6e18)) s = (s != s) ? 4.6e18 : -4.6e18;  // NaN marks as huge
  if (s > 4.6e18) s = 4.6e18;
  return __double2ll_rn(s);
}
__device__ __forceinline__ double from_fix(long long v) { return (double)v * (1.0 / kFixScale); }

// ---------------------------------------------------------------------------
// wave64 reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide FP64 sum in a fixed order (wave sums, then waves in order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < NT / 64; ++k) s += lds[k];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// Bias of one replica at time t, given z and its gradient direction: returns
// the coefficient c with F_i^bias = c * dz/dx_i, the reference (or ratchet
// minimum) zr and the bias energy.  INIT evaluates at t = 0 with z(X_0) = z.
//   harmonic: c = -k (z - zr),  zr = z_t + (z_0 - z_t) max(0, 1 - rho t);
//   ratchet (Eq. VR): zm = min(z_m, z), c = -(k/2)(z - zm) if z > zm else 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bias_coef(const RepInfo &R, double z, double z0, double zm_prev,
                                            double t, bool init, double &zr, double &ub) {
  ub = 0.0;
  zr = 0.0;
  if (R.bias == VP_BIAS_CONST) {  // z = sum_i F0_i . x_i, U_b = -z, F^bias = grad z
    ub = -z;
    return 1.0;
  }
  if (R.bias == VP_BIAS_RG || R.bias == VP_BIAS_CONTACT) {
    double zz0 = init ? z : z0;
    double w = 1.0 - R.ramp_rate * t;
    w = w < 0.0 ? 0.0 : w;
    zr = R.z_target + (zz0 - R.z_target) * w;
    ub = 0.5 * R.bias_k * (z - zr) * (z - zr);
    return -R.bias_k * (z - zr);
  }
  if (R.bias == VP_BIAS_RMD_CONTACT) {
    double zm = init ? z : (zm_prev < z ? zm_prev : z);
    zr = zm;
    if (z > zm) {
      ub = 0.25 * R.bias_k * (z - zm) * (z - zm);
      return -0.5 * R.bias_k * (z - zm);
    }
    return 0.0;
  }
  return 0.0;
}

// Derivatives of the bias coefficient c of bias_coef for the harmonic kinds:
// dc/dz and the explicit dc/dtheta_p, theta = (bias_k, ramp_rate), with
//   c = -k (z - z_ref),  z_ref = z_t + (z_0 - z_t) max(0, 1 - rho t),
// so dc/dk = -(z - z_ref) and dc/drho = -k (z_0 - z_t) t while the ramp runs.
// Other kinds: zero (constant force) -- the ratchet is not differentiated.
__device__ __forceinline__ void bias_coef_deriv(const RepInfo &R, double z, double z0, double t,
                                                bool init, double &dcdz, double dcdth[2]) {
  dcdz = 0.0;
  dcdth[0] = dcdth[1] = 0.0;
  if (R.bias == VP_BIAS_RG || R.bias == VP_BIAS_CONTACT) {
    const double zz0 = init ? z : z0;
    const double w = 1.0 - R.ramp_rate * t;
    const double zr = R.z_target + (zz0 - R.z_target) * (w < 0.0 ? 0.0 : w);
    dcdz = -R.bias_k;
    dcdth[0] = -(z - zr);
    dcdth[1] = w < 0.0 ? 0.0 : -R.bias_k * (zz0 - R.z_target) * t;
  }
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

// Energy columns VP_E_LJ .. VP_E_WZZ of replica r from the per-block partials
// (added in block order) and the CV partials, at time t with the ramp start
// z0 and ratchet minimum zm.
__device__ __forceinline__ void energy_columns(const RepInfo &R, const Work &W, int r, double z0,
                                               double zm, double t, double *o) {
  double e[4] = {0, 0, 0, 0}, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int bb = R.blk0; bb < R.blk0 + R.npad / kBlk; ++bb) {
    const double *p = W.epart + kEp * (size_t)bb;
    for (int k = 0; k < 4; ++k) e[k] += p[k];
    for (int k = 0; k < 9; ++k) w[k] += p[kEpPairW + k] + p[kEpBondW + k];
  }
  double z, G, zr, ub;
  cv_sums(R, W, r, z, G);
  const double c = bias_coef(R, z, z0, zm, t, false, zr, ub);
  o[VP_E_LJ] = e[0];
  o[VP_E_RF] = e[1];
  o[VP_E_BOND] = e[2];
  o[VP_E_ANGLE] = e[3];
  o[VP_E_BIAS] = ub;
  o[VP_E_Z] = R.bias == VP_BIAS_NONE ? 0.0 : z;
  o[VP_E_ZREF] = zr;
  o[VP_E_S] = c * c * G;
  o[VP_E_TOTAL] = e[0] + e[1] + e[2] + e[3] + ub;
  for (int k = 0; k < 9; ++k) o[VP_E_WXX + k] = w[k];
}

// Value and one directional derivative (forward-mode differentiation of the
// FP64 bonded terms along a tangent).
struct dual1 {
  double v, d;
};
__device__ __forceinline__ dual1 operator+(dual1 a, dual1 b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dual1 operator-(dual1 a, dual1 b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dual1 operator*(dual1 a, dual1 b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ dual1 operator*(double s, dual1 a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ dual1 operator/(dual1 a, dual1 b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ dual1 dsqrt(dual1 a) {
  const double r = sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}

// Map a launch-order workgroup index to a tile (or block) so that consecutive tiles of one
// replica run on the same XCD (blocks are dealt round-robin over 8 XCDs).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int nx = 8;
  int per = (nb + nx - 1) / nx;
  int x = b % nx, k = b / nx;
  int t = x * per + k;
  return t < nb ? t : -1;
}

}  // namespace vp
