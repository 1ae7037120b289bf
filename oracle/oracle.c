/* FP64 CPU oracle — test infrastructure only (see oracle.h).
 *
 * Build: plain C99, -O2 -ffp-contract=off, single-threaded.  Everything is
 * FP64 except the pair-membership predicate, which is defined on fixed-point
 * coordinates (unit 2^-22 nm) with one FP32 rounding of the exact integer
 * separation, so that pair *sets* can be compared exactly with the GPU.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define COULOMB_F 138.935458 /* kJ mol^-1 nm e^-2 */
#define TWO_PI 6.283185307179586476925286766559
#define FORCE_LIMIT 1.0e6 /* kJ/mol/nm: above this a replica is unstable */
#define ORA_QSCALE 4194304.0 /* 2^22: fixed-point coordinates of the pair predicate */

struct ora_ctx {
  ora_sys s;
  /* exclusions as sorted per-atom lists (CSR) */
  int32_t *ex_start, *ex_list;
  /* native contact map C~(X_f) for solute pairs, dense [ns][ns] */
  double *cmap_f;
  /* fixed-point geometry of the pair predicate (unit 2^-22 nm) */
  int64_t Lq[3];
  float rc2_q;
  /* reaction-field constants */
  double krf, crf;
  /* scratch */
  double *f_tmp, *fb_tmp, *grad_tmp;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies on a      */
/* 4-word counter with a 2-word key bumped by Weyl constants between rounds.  */
/* Parity pinned by the published known-answer vectors.                      */
/* ------------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Noise stream: key = 64-bit replica seed, counter = (atom, step, tag, 0).
 * Each word w gives the uniform ((w >> 9) + 1/2) * 2^-23, exactly
 * representable in FP32 and strictly inside (0, 1). */
void ora_uniforms(uint64_t seed, uint32_t atom, uint32_t step, uint32_t tag, double u[4]) {
  uint32_t ctr[4] = {atom, step, tag, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  ora_philox4x32_10(ctr, key, w);
  for (int k = 0; k < 4; ++k) u[k] = ((double)(w[k] >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Box-Muller in FP64 on the exact uniforms: (g0, g1) from (u0, u1), g2 from
 * (u2, u3).  White noise of the Langevin equation (Eq. Lang). */
void ora_normals(uint64_t seed, uint32_t atom, uint32_t step, uint32_t tag, double g[3]) {
  double u[4];
  ora_uniforms(seed, atom, step, tag, u);
  double rho = sqrt(-2.0 * log(u[0]));
  g[0] = rho * cos(TWO_PI * u[1]);
  g[1] = rho * sin(TWO_PI * u[1]);
  g[2] = sqrt(-2.0 * log(u[2])) * cos(TWO_PI * u[3]);
}

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Smoothly truncated contact value (supplement, "Collective coordinate"):
 * C(r) = (1 - (r/r0)^6) / (1 - (r/r0)^10), evaluated in the equivalent form
 * (1+u+u^2)/(1+u+u^2+u^3+u^4) with u = (r/r0)^2, which is finite at r = r0
 * (value 3/5), times a quintic switch S(r) that is 1 below rs and 0 above rc.
 * Returns C*S and its r-derivative. */
double ora_contact_value(double r, double r0, double rs, double rc, double *dcdr) {
  double u = (r / r0) * (r / r0);
  double num = 1.0 + u + u * u;
  double den = num + u * u * u + u * u * u * u;
  double c = num / den;
  double dnum = 1.0 + 2.0 * u;
  double dden = dnum + 3.0 * u * u + 4.0 * u * u * u;
  double dcdu = (dnum * den - num * dden) / (den * den);
  double dc = dcdu * 2.0 * r / (r0 * r0);
  double sw = 1.0, dsw = 0.0;
  if (r >= rc) {
    sw = 0.0;
  } else if (r > rs) {
    double t = (r - rs) / (rc - rs);
    sw = 1.0 - t * t * t * (10.0 - 15.0 * t + 6.0 * t * t);
    dsw = -30.0 * t * t * (1.0 - t) * (1.0 - t) / (rc - rs);
  }
  if (dcdr) *dcdr = dc * sw + c * dsw;
  return c * sw;
}

ora_ctx *ora_create(const ora_sys *s) {
  ora_ctx *c = (ora_ctx *)calloc(1, sizeof(ora_ctx));
  if (!c) return NULL;
  c->s = *s;
  int n = s->n_atoms;
  /* exclusions: both directions, sorted */
  int32_t *cnt = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  for (int e = 0; e < s->n_excl; ++e) {
    cnt[s->excl[2 * e]]++;
    cnt[s->excl[2 * e + 1]]++;
  }
  c->ex_start = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  for (int i = 0; i < n; ++i) c->ex_start[i + 1] = c->ex_start[i] + cnt[i];
  c->ex_list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c->ex_start[n] + 1));
  memset(cnt, 0, sizeof(int32_t) * ((size_t)n + 1));
  for (int e = 0; e < s->n_excl; ++e) {
    int a = s->excl[2 * e], b = s->excl[2 * e + 1];
    c->ex_list[c->ex_start[a] + cnt[a]++] = b;
    c->ex_list[c->ex_start[b] + cnt[b]++] = a;
  }
  for (int i = 0; i < n; ++i)
    qsort(c->ex_list + c->ex_start[i], (size_t)(c->ex_start[i + 1] - c->ex_start[i]),
          sizeof(int32_t), cmp_i32);
  free(cnt);
  for (int a = 0; a < 3; ++a) c->Lq[a] = llrint(s->box[a] * ORA_QSCALE);
  {
    double rq = s->r_cut * ORA_QSCALE;
    c->rc2_q = (float)(rq * rq);
  }
  double rc = s->r_cut;
  c->krf = (s->eps_rf - 1.0) / ((2.0 * s->eps_rf + 1.0) * rc * rc * rc);
  c->crf = 1.0 / rc + c->krf * rc * rc;
  int ns = s->n_solute;
  if ((s->bias == ORA_BIAS_CONTACT || s->bias == ORA_BIAS_RMD_CONTACT) && s->x_final && ns > 0) {
    c->cmap_f = (double *)calloc((size_t)ns * ns, sizeof(double));
    for (int i = 0; i < ns; ++i)
      for (int j = 0; j < ns; ++j) {
        if (abs(i - j) <= s->contact_min_sep) continue;
        double d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          d[a] = s->x_final[3 * j + a] - s->x_final[3 * i + a];
          r2 += d[a] * d[a];
        }
        c->cmap_f[(size_t)i * ns + j] =
            ora_contact_value(sqrt(r2), s->contact_r0, s->contact_rs, s->contact_rc, NULL);
      }
  }
  c->f_tmp = (double *)calloc((size_t)3 * n, sizeof(double));
  c->fb_tmp = (double *)calloc((size_t)3 * n, sizeof(double));
  c->grad_tmp = (double *)calloc((size_t)3 * (ns > 0 ? ns : 1), sizeof(double));
  return c;
}

void ora_destroy(ora_ctx *c) {
  if (!c) return;
  free(c->ex_start);
  free(c->ex_list);
  free(c->cmap_f);
  free(c->f_tmp);
  free(c->fb_tmp);
  free(c->grad_tmp);
  free(c);
}

static int excluded(const ora_ctx *c, int i, int j) {
  for (int k = c->ex_start[i]; k < c->ex_start[i + 1]; ++k)
    if (c->ex_list[k] == j) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Pair membership on fixed-point coordinates (unit q = 2^-22 nm):           */
/*   X = round(x / q) (nearest, ties to even), Lq = round(L / q);            */
/*   D = Xj - Xi - n Lq with n the nearest integer to (Xj - Xi) / Lq;        */
/*   d = fl32(D);  r2 = fma(dz, dz, fma(dy, dy, fl32(dx * dx)));             */
/*   in <=> r2 < fl32((rc / q)^2).                                           */
/* Inside the cutoff the image n is unique, so the set does not depend on    */
/* how n is found.  The FP64 separation used for the force is                */
/* (xj - xi) - n L in FP64.                                                  */
/* ------------------------------------------------------------------------ */
static int64_t nearest_int_div(int64_t d, int64_t L) {
  /* floor((2d + L) / (2L)) */
  int64_t num = 2 * d + L, den = 2 * L;
  int64_t q = num / den;
  if ((num % den != 0) && ((num < 0) != (den < 0))) q -= 1;
  return q;
}

static int pair_in(const ora_ctx *c, const double *x, int i, int j, double d[3]) {
  float dp[3];
  for (int a = 0; a < 3; ++a) {
    int64_t xi = llrint(x[3 * i + a] * ORA_QSCALE), xj = llrint(x[3 * j + a] * ORA_QSCALE);
    int64_t D = xj - xi;
    int64_t n = nearest_int_div(D, c->Lq[a]);
    dp[a] = (float)(D - n * c->Lq[a]);
    d[a] = (x[3 * j + a] - x[3 * i + a]) - (double)n * c->s.box[a];
  }
  float sq = dp[0] * dp[0];
  float r2 = fmaf(dp[2], dp[2], fmaf(dp[1], dp[1], sq));
  return r2 < c->rc2_q;
}

/* Brute force: every unordered pair, definition of the interaction set. */
static int64_t pairs_brute(const ora_ctx *c, const double *x, int32_t *out, int64_t cap,
                           void (*visit)(ora_ctx *, int, int, const double *, void *), void *arg) {
  int n = c->s.n_atoms;
  int64_t np = 0;
  double d[3];
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      if (!pair_in(c, x, i, j, d)) continue;
      if (excluded(c, i, j)) continue;
      if (visit) visit((ora_ctx *)c, i, j, d, arg);
      if (out && np < cap) {
        out[2 * np] = i;
        out[2 * np + 1] = j;
      }
      ++np;
    }
  return np;
}

/* Cell list (cells of side >= rc, FP64 wrapped coordinates); visits the same
 * set as the brute force because the predicate is the same. */
static int64_t pairs_cells(const ora_ctx *c, const double *x, int32_t *out, int64_t cap,
                           void (*visit)(ora_ctx *, int, int, const double *, void *), void *arg) {
  int n = c->s.n_atoms;
  int nc[3];
  for (int a = 0; a < 3; ++a) {
    nc[a] = (int)floor(c->s.box[a] / (c->s.r_cut * (1.0 + 1e-5)));
    if (nc[a] < 1) nc[a] = 1;
  }
  int ncell = nc[0] * nc[1] * nc[2];
  int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
  int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  for (int k = 0; k < ncell; ++k) head[k] = -1;
  for (int i = n - 1; i >= 0; --i) {
    int ci[3];
    for (int a = 0; a < 3; ++a) {
      double L = c->s.box[a];
      double w = x[3 * i + a] - floor(x[3 * i + a] / L) * L;
      int k = (int)floor(w * nc[a] / L);
      if (k < 0) k = 0;
      if (k >= nc[a]) k = nc[a] - 1;
      ci[a] = k;
    }
    int id = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
    cell[i] = id;
    next[i] = head[id];
    head[id] = i;
  }
  int64_t np = 0;
  double d[3];
  for (int cz = 0; cz < nc[2]; ++cz)
    for (int cy = 0; cy < nc[1]; ++cy)
      for (int cx = 0; cx < nc[0]; ++cx) {
        int home = (cz * nc[1] + cy) * nc[0] + cx;
        /* distinct neighbour cells (a box with < 3 cells per side wraps) */
        int nb[27], nnb = 0;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int ox = ((cx + dx) % nc[0] + nc[0]) % nc[0];
              int oy = ((cy + dy) % nc[1] + nc[1]) % nc[1];
              int oz = ((cz + dz) % nc[2] + nc[2]) % nc[2];
              int id = (oz * nc[1] + oy) * nc[0] + ox;
              int dup = 0;
              for (int k = 0; k < nnb; ++k) dup |= (nb[k] == id);
              if (!dup) nb[nnb++] = id;
            }
        for (int i = head[home]; i >= 0; i = next[i])
          for (int k = 0; k < nnb; ++k)
            for (int j = head[nb[k]]; j >= 0; j = next[j]) {
              if (j <= i) continue;
              if (!pair_in(c, x, i, j, d)) continue;
              if (excluded(c, i, j)) continue;
              if (visit) visit((ora_ctx *)c, i, j, d, arg);
              if (out && np < cap) {
                out[2 * np] = i;
                out[2 * np + 1] = j;
              }
              ++np;
            }
      }
  free(head);
  free(next);
  free(cell);
  return np;
}

int64_t ora_pairs(const ora_ctx *c, const double *x, int32_t use_cells, int32_t *out, int64_t cap) {
  return use_cells ? pairs_cells(c, x, out, cap, NULL, NULL) : pairs_brute(c, x, out, cap, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Potential U(X,Y) of Eq. Lang: potential-shifted LJ with Lorentz-Berthelot */
/* mixing + reaction-field Coulomb for non-excluded pairs inside rc,        */
/* harmonic bonds and angles.                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  double *f;
  double e_lj, e_rf;
  double vir[9]; /* sum over pairs of d_a F_b, d = x_j - x_i, F the force on j */
} nb_acc;

static void nb_visit(ora_ctx *c, int i, int j, const double *d, void *arg) {
  nb_acc *acc = (nb_acc *)arg;
  const ora_sys *s = &c->s;
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double r = sqrt(r2);
  double sig = 0.5 * (s->sigma[i] + s->sigma[j]);
  double eps = sqrt(s->epsilon[i] * s->epsilon[j]);
  double fscal = 0.0; /* -(dV/dr)/r */
  if (eps > 0.0) {
    double sr2 = sig * sig / r2;
    double sr6 = sr2 * sr2 * sr2;
    double src2 = sig * sig / (s->r_cut * s->r_cut);
    double src6 = src2 * src2 * src2;
    acc->e_lj += 4.0 * eps * (sr6 * sr6 - sr6) - 4.0 * eps * (src6 * src6 - src6);
    fscal += 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / r2;
  }
  double qq = COULOMB_F * s->charge[i] * s->charge[j];
  if (qq != 0.0) {
    acc->e_rf += qq * (1.0 / r + c->krf * r2 - c->crf);
    fscal += qq * (1.0 / (r2 * r) - 2.0 * c->krf);
  }
  for (int a = 0; a < 3; ++a) {
    acc->f[3 * i + a] -= fscal * d[a];
    acc->f[3 * j + a] += fscal * d[a];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) acc->vir[3 * a + b] += d[a] * (fscal * d[b]);
}

/* Bonds and angles; vir accumulates, per term, the separation of each moved
 * atom from the term's reference atom (i for a bond, the vertex for an angle)
 * times the force on it. */
static void bonded(const ora_ctx *c, const double *x, double *f, double *e_bond, double *e_angle,
                   double *vir) {
  const ora_sys *s = &c->s;
  double eb = 0.0, ea = 0.0;
  for (int b = 0; b < s->n_bonds; ++b) {
    int i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
    double d[3], r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      d[a] = x[3 * j + a] - x[3 * i + a];
      r2 += d[a] * d[a];
    }
    double r = sqrt(r2);
    double dr = r - s->bond_r0[b];
    eb += 0.5 * s->bond_k[b] * dr * dr;
    double g = s->bond_k[b] * dr / r; /* dV/dr / r */
    for (int a = 0; a < 3; ++a) {
      f[3 * i + a] += g * d[a];
      f[3 * j + a] -= g * d[a];
    }
    for (int a = 0; a < 3; ++a)
      for (int e = 0; e < 3; ++e) vir[3 * a + e] += d[a] * (-g * d[e]);
  }
  for (int k = 0; k < s->n_angles; ++k) {
    int ia = s->angles[3 * k], ic = s->angles[3 * k + 1], ib = s->angles[3 * k + 2];
    double u[3], w[3], uu = 0.0, ww = 0.0, uw = 0.0;
    for (int a = 0; a < 3; ++a) {
      u[a] = x[3 * ia + a] - x[3 * ic + a];
      w[a] = x[3 * ib + a] - x[3 * ic + a];
      uu += u[a] * u[a];
      ww += w[a] * w[a];
      uw += u[a] * w[a];
    }
    double nu = sqrt(uu), nw = sqrt(ww);
    double cs = uw / (nu * nw);
    if (cs > 1.0) cs = 1.0;
    if (cs < -1.0) cs = -1.0;
    double th = acos(cs);
    double sn = sqrt(1.0 - cs * cs);
    if (sn < 1e-12) sn = 1e-12;
    double dth = th - s->angle_theta0[k];
    ea += 0.5 * s->angle_k[k] * dth * dth;
    double dv = s->angle_k[k] * dth; /* dV/dtheta */
    double fu[3], fw[3];
    /* dtheta/du = -(w/(|u||w|) - cos u/|u|^2)/sin */
    for (int a = 0; a < 3; ++a) {
      double dcu = w[a] / (nu * nw) - cs * u[a] / uu;
      double dcw = u[a] / (nu * nw) - cs * w[a] / ww;
      double fa = dv / sn * dcu;
      double fb = dv / sn * dcw;
      f[3 * ia + a] += fa;
      f[3 * ib + a] += fb;
      f[3 * ic + a] -= fa + fb;
      fu[a] = fa;
      fw[a] = fb;
    }
    for (int a = 0; a < 3; ++a)
      for (int e = 0; e < 3; ++e) vir[3 * a + e] += u[a] * fu[e] + w[a] * fw[e];
  }
  *e_bond = eb;
  *e_angle = ea;
}

/* ------------------------------------------------------------------------ */
/* Collective variables (solute only, unwrapped coordinates, no periodic     */
/* images: the solute is one connected molecule).                            */
/*   RG:      mass-weighted radius of gyration.                              */
/*   CONTACT: z = sum_{i<j, j-i > min_sep} (C~_ij(X) - C~_ij(X_f))^2         */
/*            (supplement, "Collective coordinate"; unordered pairs).         */
/* Returns z and writes dz/dx_i for solute atoms.                             */
/* ------------------------------------------------------------------------ */
double ora_cv(const ora_ctx *c, const double *x, double *grad) {
  const ora_sys *s = &c->s;
  int ns = s->n_solute;
  if (grad) memset(grad, 0, sizeof(double) * 3 * (size_t)ns);
  if (s->bias == ORA_BIAS_RG) {
    double M = 0.0, cm[3] = {0, 0, 0};
    for (int i = 0; i < ns; ++i) {
      M += s->mass[i];
      for (int a = 0; a < 3; ++a) cm[a] += s->mass[i] * x[3 * i + a];
    }
    for (int a = 0; a < 3; ++a) cm[a] /= M;
    double acc = 0.0;
    for (int i = 0; i < ns; ++i)
      for (int a = 0; a < 3; ++a) {
        double d = x[3 * i + a] - cm[a];
        acc += s->mass[i] * d * d;
      }
    double rg = sqrt(acc / M);
    if (grad && rg > 0.0)
      for (int i = 0; i < ns; ++i)
        for (int a = 0; a < 3; ++a) grad[3 * i + a] = s->mass[i] * (x[3 * i + a] - cm[a]) / (M * rg);
    return rg;
  }
  if ((s->bias == ORA_BIAS_CONTACT || s->bias == ORA_BIAS_RMD_CONTACT) && c->cmap_f) {
    double z = 0.0;
    for (int i = 0; i < ns; ++i)
      for (int j = i + s->contact_min_sep + 1; j < ns; ++j) {
        double d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          d[a] = x[3 * j + a] - x[3 * i + a];
          r2 += d[a] * d[a];
        }
        double r = sqrt(r2), dc;
        double cij = ora_contact_value(r, s->contact_r0, s->contact_rs, s->contact_rc, &dc);
        double diff = cij - c->cmap_f[(size_t)i * ns + j];
        z += diff * diff;
        if (grad) {
          double g = 2.0 * diff * dc / r; /* dz/dr / r */
          for (int a = 0; a < 3; ++a) {
            grad[3 * j + a] += g * d[a];
            grad[3 * i + a] -= g * d[a];
          }
        }
      }
    return z;
  }
  return 0.0;
}

/* Reference of the harmonic bias, ramped linearly from z(X_0) to z_target
 * at rate rho (1/ps) and held there. */
static double z_ref(const ora_sys *s, double z0, double t) {
  double w = 1.0 - s->ramp_rate * t;
  if (w < 0.0) w = 0.0;
  return s->z_target + (z0 - s->z_target) * w;
}

/* Bias force on solute atoms (text after Eq. Lang; Eq. VR for the ratchet).
 * Returns S = sum_i |F_i^bias|^2 / (gamma_i m_i), the integrand of the
 * variational functional (Eq. VMDcondition). */
static double bias_force(ora_ctx *c, const double *x, double t, double z0, double z_m,
                         double *fb, double *terms) {
  const ora_sys *s = &c->s;
  int ns = s->n_solute;
  memset(fb, 0, sizeof(double) * 3 * (size_t)s->n_atoms);
  double z = 0.0, zr = 0.0, ub = 0.0;
  if (s->bias == ORA_BIAS_CONST && s->const_force) {
    /* constant force F0 on each solute atom: the gradient of -sum_i F0_i . x_i
     * (z is taken as that projection, so U_b = -z) */
    for (int i = 0; i < 3 * ns; ++i) {
      fb[i] = s->const_force[i];
      z += s->const_force[i] * x[i];
    }
    ub = -z;
  } else if (s->bias == ORA_BIAS_RG || s->bias == ORA_BIAS_CONTACT) {
    z = ora_cv(c, x, c->grad_tmp);
    zr = z_ref(s, z0, t);
    double k = s->bias_k;
    ub = 0.5 * k * (z - zr) * (z - zr);
    for (int i = 0; i < 3 * ns; ++i) fb[i] = -k * (z - zr) * c->grad_tmp[i];
  } else if (s->bias == ORA_BIAS_RMD_CONTACT) {
    z = ora_cv(c, x, c->grad_tmp);
    double zm = z_m < z ? z_m : z; /* running minimum, updated first */
    zr = zm;
    if (z > zm) {
      double k = s->bias_k;
      ub = 0.25 * k * (z - zm) * (z - zm);
      for (int i = 0; i < 3 * ns; ++i) fb[i] = -0.5 * k * (z - zm) * c->grad_tmp[i];
    }
  }
  double S = 0.0;
  for (int i = 0; i < ns; ++i) {
    double f2 = fb[3 * i] * fb[3 * i] + fb[3 * i + 1] * fb[3 * i + 1] + fb[3 * i + 2] * fb[3 * i + 2];
    S += f2 / (s->gamma[i] * s->mass[i]);
  }
  if (terms) {
    terms[ORA_E_BIAS] = ub;
    terms[ORA_Z] = z;
    terms[ORA_ZREF] = zr;
    terms[ORA_S] = S;
  }
  return S;
}

/* Total force F = -grad U + F^bias at time t.  f, fbias: [n][3] (fbias may be
 * NULL).  terms: [ORA_N_TERMS] (may be NULL).  Returns 1 if any force is
 * non-finite or above the instability limit. */
int ora_forces(ora_ctx *c, const double *x, double t, const ora_state *st, int32_t use_cells,
               double *f, double *fbias, double *terms) {
  const ora_sys *s = &c->s;
  int n = s->n_atoms;
  double tl[ORA_N_TERMS];
  memset(tl, 0, sizeof(tl));
  memset(f, 0, sizeof(double) * 3 * (size_t)n);
  nb_acc acc = {f, 0.0, 0.0, {0.0}};
  if (use_cells)
    pairs_cells(c, x, NULL, 0, nb_visit, &acc);
  else
    pairs_brute(c, x, NULL, 0, nb_visit, &acc);
  tl[ORA_E_LJ] = acc.e_lj;
  tl[ORA_E_RF] = acc.e_rf;
  for (int k = 0; k < 9; ++k) tl[ORA_VIR + k] = acc.vir[k];
  bonded(c, x, f, &tl[ORA_E_BOND], &tl[ORA_E_ANGLE], &tl[ORA_VIR]);
  double z0 = st ? st->z0 : 0.0;
  double zm = st ? st->z_m : DBL_MAX;
  bias_force(c, x, t, z0, zm, c->fb_tmp, tl);
  tl[ORA_U_TOTAL] = tl[ORA_E_LJ] + tl[ORA_E_RF] + tl[ORA_E_BOND] + tl[ORA_E_ANGLE] + tl[ORA_E_BIAS];
  int bad = 0;
  for (int i = 0; i < 3 * n; ++i) {
    f[i] += c->fb_tmp[i];
    if (!isfinite(f[i]) || fabs(f[i]) > FORCE_LIMIT) bad = 1;
  }
  if (fbias) memcpy(fbias, c->fb_tmp, sizeof(double) * 3 * (size_t)n);
  if (terms) memcpy(terms, tl, sizeof(tl));
  return bad;
}

/* ------------------------------------------------------------------------ */
/* Trajectories: BAOAB splitting of Eq. Lang with white noise of variance    */
/* 2 m gamma kT per unit time (the weight 1/(4 kT gamma m) of Eq. StrVMD).    */
/* Step n -> n+1:  v += dt/2 F_n/m;  x += dt/2 v;                             */
/*                 v = c1 v + sqrt((1-c1^2) kT/m) g(n);  x += dt/2 v;         */
/*                 F_{n+1} = F(x_{n+1}, t_{n+1});  v += dt/2 F_{n+1}/m.       */
/* Functional (Eq. VMDcondition, prefactor of Eq. StrVMD), trapezoid in time: */
/*   Phi = dt/(4 kT) * sum_n w_n S_n,  w_0 = w_N = 1/2, else 1.                */
/* ------------------------------------------------------------------------ */
void ora_maxwell(const ora_ctx *c, double *v) {
  const ora_sys *s = &c->s;
  for (int i = 0; i < s->n_atoms; ++i) {
    double g[3];
    ora_normals(s->seed, (uint32_t)i, 0u, 1u, g);
    double sd = sqrt(s->kT / s->mass[i]);
    for (int a = 0; a < 3; ++a) v[3 * i + a] = sd * g[a];
  }
}

int ora_init(ora_ctx *c, const double *x0, ora_state *st) {
  memset(st, 0, sizeof(*st));
  st->z0 = ora_cv(c, x0, NULL);
  st->z_m = st->z0;
  double terms[ORA_N_TERMS];
  int bad = ora_forces(c, x0, 0.0, st, 1, c->f_tmp, NULL, terms);
  st->phi_acc = 0.5 * terms[ORA_S];
  st->s_last = terms[ORA_S];
  st->z_last = terms[ORA_Z];
  st->status = bad;
  return bad;
}

int ora_run(ora_ctx *c, double *x, double *v, ora_state *st, int32_t nsteps, int32_t use_cells,
            double *traj) {
  const ora_sys *s = &c->s;
  int n = s->n_atoms;
  double dt = s->dt;
  double *f = c->f_tmp;
  double terms[ORA_N_TERMS];
  if (st->status) return st->status;
  if (ora_forces(c, x, (double)st->step * dt, st, use_cells, f, NULL, terms)) {
    st->status = 1;
    return 1;
  }
  for (int it = 0; it < nsteps; ++it) {
    uint32_t step = (uint32_t)st->step;
    for (int i = 0; i < n; ++i) {
      double m = s->mass[i];
      double c1 = exp(-s->gamma[i] * dt);
      double sd = sqrt((1.0 - c1 * c1) * s->kT / m);
      double g[3];
      ora_normals(s->seed, (uint32_t)i, step, 0u, g);
      for (int a = 0; a < 3; ++a) {
        double vv = v[3 * i + a] + 0.5 * dt * f[3 * i + a] / m;
        double xx = x[3 * i + a] + 0.5 * dt * vv;
        vv = c1 * vv + sd * g[a];
        xx = xx + 0.5 * dt * vv;
        v[3 * i + a] = vv;
        x[3 * i + a] = xx;
      }
    }
    st->step += 1;
    /* ratchet minimum is updated before the force at the new step */
    int bad = ora_forces(c, x, (double)st->step * dt, st, use_cells, f, NULL, terms);
    if (s->bias == ORA_BIAS_RMD_CONTACT && terms[ORA_Z] < st->z_m) st->z_m = terms[ORA_Z];
    for (int i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) v[3 * i + a] += 0.5 * dt * f[3 * i + a] / s->mass[i];
    st->phi_acc += terms[ORA_S];
    st->s_last = terms[ORA_S];
    st->z_last = terms[ORA_Z];
    if (traj) memcpy(traj + (size_t)it * 3 * n, x, sizeof(double) * 3 * (size_t)n);
    if (bad) {
      st->status = 1;
      return 1;
    }
  }
  return 0;
}

double ora_phi(const ora_ctx *c, const ora_state *st) {
  if (st->status) return INFINITY;
  return (st->phi_acc - 0.5 * st->s_last) * c->s.dt / (4.0 * c->s.kT);
}

/* ------------------------------------------------------------------------ */
/* RMSD to the product after the optimal rigid superposition (the folding     */
/* criterion of the main text: final RMSD to the native structure).          */
/* Both structures are centred; the rotation that brings the centred X onto  */
/* the centred X_f is found by the quaternion method of Horn (J. Opt. Soc.   */
/* Am. A 4, 629 (1987)): the unit quaternion is the eigenvector of the       */
/* largest eigenvalue of a symmetric 4x4 matrix built from the correlation    */
/* matrix S_ab = sum_i x_ia y_ib.  The rotation is then applied and the mean  */
/* squared distance summed directly.                                          */
/* ------------------------------------------------------------------------ */
/* cyclic Jacobi rotations of a symmetric n x n matrix (n <= 4): a becomes
 * diagonal (its eigenvalues), v collects the eigenvectors as columns */
static void jacobi_eigen(int n, double a[4][4], double v[4][4]) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, scale = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i != j) off += a[i][j] * a[i][j];
        scale += a[i][j] * a[i][j];
      }
    if (off <= 1e-32 * scale || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (a[p][q] == 0.0) continue;
        /* rotation angle that zeroes a[p][q] */
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) { /* columns p, q */
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = cs * akp - sn * akq;
          a[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) { /* rows p, q */
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = cs * apk - sn * aqk;
          a[q][k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = cs * vkp - sn * vkq;
          v[k][q] = sn * vkp + cs * vkq;
        }
      }
  }
}

double ora_rmsd(const ora_ctx *c, const double *x) {
  const ora_sys *s = &c->s;
  int ns = s->n_solute;
  if (!s->x_final || ns <= 0) return NAN;
  double cx[3] = {0, 0, 0}, cy[3] = {0, 0, 0};
  for (int i = 0; i < ns; ++i)
    for (int a = 0; a < 3; ++a) {
      cx[a] += x[3 * i + a];
      cy[a] += s->x_final[3 * i + a];
    }
  for (int a = 0; a < 3; ++a) {
    cx[a] /= ns;
    cy[a] /= ns;
  }
  double S[3][3] = {{0}};
  for (int i = 0; i < ns; ++i)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        S[a][b] += (x[3 * i + a] - cx[a]) * (s->x_final[3 * i + b] - cy[b]);
  double N[4][4] = {
      {S[0][0] + S[1][1] + S[2][2], S[1][2] - S[2][1], S[2][0] - S[0][2], S[0][1] - S[1][0]},
      {S[1][2] - S[2][1], S[0][0] - S[1][1] - S[2][2], S[0][1] + S[1][0], S[2][0] + S[0][2]},
      {S[2][0] - S[0][2], S[0][1] + S[1][0], -S[0][0] + S[1][1] - S[2][2], S[1][2] + S[2][1]},
      {S[0][1] - S[1][0], S[2][0] + S[0][2], S[1][2] + S[2][1], -S[0][0] - S[1][1] + S[2][2]}};
  double V[4][4];
  jacobi_eigen(4, N, V);
  int m = 0;
  for (int k = 1; k < 4; ++k)
    if (N[k][k] > N[m][m]) m = k;
  double q0 = V[0][m], q1 = V[1][m], q2 = V[2][m], q3 = V[3][m];
  double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  q0 /= qn; q1 /= qn; q2 /= qn; q3 /= qn;
  double R[3][3] = {
      {q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3, 2.0 * (q1 * q2 - q0 * q3), 2.0 * (q1 * q3 + q0 * q2)},
      {2.0 * (q1 * q2 + q0 * q3), q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3, 2.0 * (q2 * q3 - q0 * q1)},
      {2.0 * (q1 * q3 - q0 * q2), 2.0 * (q2 * q3 + q0 * q1), q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3}};
  double acc = 0.0;
  for (int i = 0; i < ns; ++i) {
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = x[3 * i + a] - cx[a];
    for (int a = 0; a < 3; ++a) {
      double r = R[a][0] * p[0] + R[a][1] * p[1] + R[a][2] * p[2];
      double d = r - (s->x_final[3 * i + a] - cy[a]);
      acc += d * d;
    }
  }
  return sqrt(acc / ns);
}

/* Product reached: a stable trajectory with |z(X_T) - z_target| <= reach_tol
 * and, when reach_rmsd is finite, an RMSD to X_f of at most reach_rmsd (the
 * folding criterion of the main text, RMSD < 2 A). */
int ora_reached(const ora_ctx *c, const ora_state *st, const double *x) {
  if (st->status) return 0;
  if (!(fabs(st->z_last - c->s.z_target) <= c->s.reach_tol)) return 0;
  if (isfinite(c->s.reach_rmsd)) {
    if (!x) return 0;
    double r = ora_rmsd(c, x);
    if (!(r <= c->s.reach_rmsd)) return 0;
  }
  return 1;
}

/* Variational selection (Eq. VMDcondition and the folding-event criterion):
 * least Phi over trials that reached the product, are eligible and finite;
 * ties go to the lowest index.  Returns 0, or -1 if no trial qualifies. */
int ora_select(int32_t n, const double *phi, const uint8_t *reached, const uint8_t *eligible,
               int32_t *best, double *best_phi) {
  int32_t b = -1;
  double bp = INFINITY;
  for (int32_t r = 0; r < n; ++r) {
    if (reached && !reached[r]) continue;
    if (eligible && !eligible[r]) continue;
    if (!isfinite(phi[r])) continue;
    if (b < 0 || phi[r] < bp) {
      b = r;
      bp = phi[r];
    }
  }
  *best = b;
  *best_phi = bp;
  return b < 0 ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Pathwise derivative of the functional with respect to the bias           */
/* parameters theta = (bias_k, ramp_rate), the noise held fixed.            */
/*                                                                          */
/* Every quantity is carried as a dual number: its value and its            */
/* derivatives along two directions (direction 0: bias_k, direction 1:      */
/* ramp_rate).  Evaluating the same potential, collective variable, bias,   */
/* BAOAB step and functional on dual numbers applies the chain rule         */
/* mechanically, so the derivative parts are d/dtheta of exactly the        */
/* computation above.  The pair set is fixed by the values (a pair moving   */
/* across the cutoff is a measure-zero event for the derivative).           */
/* Parity pinned by central differences of the plain computation.           */
/* ------------------------------------------------------------------------ */
typedef struct {
  double v, d[2];
} dual2;

static dual2 dn(double v) {
  dual2 r = {v, {0.0, 0.0}};
  return r;
}
static dual2 dadd(dual2 a, dual2 b) {
  dual2 r = {a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1]}};
  return r;
}
static dual2 dsub(dual2 a, dual2 b) {
  dual2 r = {a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1]}};
  return r;
}
static dual2 dmul(dual2 a, dual2 b) {
  dual2 r = {a.v * b.v, {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1]}};
  return r;
}
static dual2 dscale(double s, dual2 a) {
  dual2 r = {s * a.v, {s * a.d[0], s * a.d[1]}};
  return r;
}
static dual2 ddiv(dual2 a, dual2 b) {
  dual2 r;
  r.v = a.v / b.v;
  for (int k = 0; k < 2; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r;
}
static dual2 dsqrt(dual2 a) {
  dual2 r;
  r.v = sqrt(a.v);
  for (int k = 0; k < 2; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}
/* acos with the derivative -1/sin, sin bounded below as in the angle force */
static dual2 dacos(dual2 a, double sn) {
  dual2 r;
  r.v = acos(a.v);
  for (int k = 0; k < 2; ++k) r.d[k] = -a.d[k] / sn;
  return r;
}

typedef struct {
  const dual2 *X;
  dual2 *F;
} nb_dual_acc;

/* pair force of the potential on dual positions: the separation's value is
 * the minimum-image one found by the pair search, its derivative that of
 * x_j - x_i (the image shift is a constant) */
static void nb_visit_dual(ora_ctx *c, int i, int j, const double *dv, void *arg) {
  nb_dual_acc *acc = (nb_dual_acc *)arg;
  const ora_sys *s = &c->s;
  dual2 d[3];
  for (int a = 0; a < 3; ++a) {
    d[a].v = dv[a];
    for (int k = 0; k < 2; ++k) d[a].d[k] = acc->X[3 * j + a].d[k] - acc->X[3 * i + a].d[k];
  }
  dual2 r2 = dadd(dadd(dmul(d[0], d[0]), dmul(d[1], d[1])), dmul(d[2], d[2]));
  dual2 r = dsqrt(r2);
  double sig = 0.5 * (s->sigma[i] + s->sigma[j]);
  double eps = sqrt(s->epsilon[i] * s->epsilon[j]);
  dual2 fscal = dn(0.0);
  if (eps > 0.0) {
    dual2 sr2 = ddiv(dn(sig * sig), r2);
    dual2 sr6 = dmul(dmul(sr2, sr2), sr2);
    dual2 lj = dsub(dscale(2.0, dmul(sr6, sr6)), sr6);
    fscal = dadd(fscal, ddiv(dscale(24.0 * eps, lj), r2));
  }
  double qq = COULOMB_F * s->charge[i] * s->charge[j];
  if (qq != 0.0) {
    dual2 inv3 = ddiv(dn(1.0), dmul(r2, r));
    fscal = dadd(fscal, dscale(qq, dsub(inv3, dn(2.0 * c->krf))));
  }
  for (int a = 0; a < 3; ++a) {
    dual2 fa = dmul(fscal, d[a]);
    acc->F[3 * i + a] = dsub(acc->F[3 * i + a], fa);
    acc->F[3 * j + a] = dadd(acc->F[3 * j + a], fa);
  }
}

static void bonded_dual(const ora_ctx *c, const dual2 *X, dual2 *F) {
  const ora_sys *s = &c->s;
  for (int b = 0; b < s->n_bonds; ++b) {
    int i = s->bonds[2 * b], j = s->bonds[2 * b + 1];
    dual2 d[3], r2 = dn(0.0);
    for (int a = 0; a < 3; ++a) {
      d[a] = dsub(X[3 * j + a], X[3 * i + a]);
      r2 = dadd(r2, dmul(d[a], d[a]));
    }
    dual2 r = dsqrt(r2);
    dual2 g = ddiv(dscale(s->bond_k[b], dsub(r, dn(s->bond_r0[b]))), r);
    for (int a = 0; a < 3; ++a) {
      F[3 * i + a] = dadd(F[3 * i + a], dmul(g, d[a]));
      F[3 * j + a] = dsub(F[3 * j + a], dmul(g, d[a]));
    }
  }
  for (int k = 0; k < s->n_angles; ++k) {
    int ia = s->angles[3 * k], ic = s->angles[3 * k + 1], ib = s->angles[3 * k + 2];
    dual2 u[3], w[3], uu = dn(0.0), ww = dn(0.0), uw = dn(0.0);
    for (int a = 0; a < 3; ++a) {
      u[a] = dsub(X[3 * ia + a], X[3 * ic + a]);
      w[a] = dsub(X[3 * ib + a], X[3 * ic + a]);
      uu = dadd(uu, dmul(u[a], u[a]));
      ww = dadd(ww, dmul(w[a], w[a]));
      uw = dadd(uw, dmul(u[a], w[a]));
    }
    dual2 nuw = dmul(dsqrt(uu), dsqrt(ww));
    dual2 cs = ddiv(uw, nuw);
    if (cs.v > 1.0) cs = dn(1.0);
    if (cs.v < -1.0) cs = dn(-1.0);
    double snv = sqrt(1.0 - cs.v * cs.v);
    if (snv < 1e-12) snv = 1e-12;
    dual2 sn = snv > 1e-12 ? dsqrt(dsub(dn(1.0), dmul(cs, cs))) : dn(1e-12);
    dual2 th = dacos(cs, snv);
    dual2 dvs = ddiv(dscale(s->angle_k[k], dsub(th, dn(s->angle_theta0[k]))), sn);
    for (int a = 0; a < 3; ++a) {
      dual2 dcu = dsub(ddiv(w[a], nuw), ddiv(dmul(cs, u[a]), uu));
      dual2 dcw = dsub(ddiv(u[a], nuw), ddiv(dmul(cs, w[a]), ww));
      dual2 fa = dmul(dvs, dcu), fb = dmul(dvs, dcw);
      F[3 * ia + a] = dadd(F[3 * ia + a], fa);
      F[3 * ib + a] = dadd(F[3 * ib + a], fb);
      F[3 * ic + a] = dsub(F[3 * ic + a], dadd(fa, fb));
    }
  }
}

/* contact value and its r-derivative on a dual distance */
static dual2 contact_dual(dual2 r, double r0, double rs, double rc, dual2 *dcdr) {
  dual2 u = dmul(dscale(1.0 / r0, r), dscale(1.0 / r0, r));
  dual2 u2 = dmul(u, u);
  dual2 num = dadd(dadd(dn(1.0), u), u2);
  dual2 den = dadd(dadd(num, dmul(u2, u)), dmul(u2, u2));
  dual2 cv = ddiv(num, den);
  dual2 dnum = dadd(dn(1.0), dscale(2.0, u));
  dual2 dden = dadd(dadd(dnum, dscale(3.0, u2)), dscale(4.0, dmul(u2, u)));
  dual2 dcdu = ddiv(dsub(dmul(dnum, den), dmul(num, dden)), dmul(den, den));
  dual2 dc = dmul(dcdu, dscale(2.0 / (r0 * r0), r));
  dual2 sw = dn(1.0), dsw = dn(0.0);
  if (r.v >= rc) {
    sw = dn(0.0);
  } else if (r.v > rs) {
    dual2 t = dscale(1.0 / (rc - rs), dsub(r, dn(rs)));
    dual2 t2 = dmul(t, t), t3 = dmul(t2, t);
    dual2 poly = dadd(dsub(dn(10.0), dscale(15.0, t)), dscale(6.0, t2));
    sw = dsub(dn(1.0), dmul(t3, poly));
    dual2 omt = dsub(dn(1.0), t);
    dsw = dscale(-30.0 / (rc - rs), dmul(t2, dmul(omt, omt)));
  }
  *dcdr = dadd(dmul(dc, sw), dmul(cv, dsw));
  return dmul(cv, sw);
}

/* collective variable and its gradient on dual positions (as ora_cv) */
static dual2 cv_dual(const ora_ctx *c, const dual2 *X, dual2 *G) {
  const ora_sys *s = &c->s;
  int ns = s->n_solute;
  for (int i = 0; i < 3 * ns; ++i) G[i] = dn(0.0);
  if (s->bias == ORA_BIAS_RG) {
    double M = 0.0;
    dual2 cm[3] = {dn(0.0), dn(0.0), dn(0.0)};
    for (int i = 0; i < ns; ++i) {
      M += s->mass[i];
      for (int a = 0; a < 3; ++a) cm[a] = dadd(cm[a], dscale(s->mass[i], X[3 * i + a]));
    }
    for (int a = 0; a < 3; ++a) cm[a] = dscale(1.0 / M, cm[a]);
    dual2 acc = dn(0.0);
    for (int i = 0; i < ns; ++i)
      for (int a = 0; a < 3; ++a) {
        dual2 d = dsub(X[3 * i + a], cm[a]);
        acc = dadd(acc, dscale(s->mass[i], dmul(d, d)));
      }
    dual2 rg = dsqrt(dscale(1.0 / M, acc));
    for (int i = 0; i < ns; ++i)
      for (int a = 0; a < 3; ++a)
        G[3 * i + a] = ddiv(dscale(s->mass[i], dsub(X[3 * i + a], cm[a])), dscale(M, rg));
    return rg;
  }
  dual2 z = dn(0.0);
  if (s->bias == ORA_BIAS_CONTACT || s->bias == ORA_BIAS_RMD_CONTACT) {
    for (int i = 0; i < ns; ++i)
      for (int j = i + s->contact_min_sep + 1; j < ns; ++j) {
        dual2 d[3], r2 = dn(0.0);
        for (int a = 0; a < 3; ++a) {
          d[a] = dsub(X[3 * j + a], X[3 * i + a]);
          r2 = dadd(r2, dmul(d[a], d[a]));
        }
        dual2 r = dsqrt(r2), dc;
        dual2 cij = contact_dual(r, s->contact_r0, s->contact_rs, s->contact_rc, &dc);
        dual2 diff = dsub(cij, dn(c->cmap_f[(size_t)i * ns + j]));
        z = dadd(z, dmul(diff, diff));
        dual2 g = ddiv(dscale(2.0, dmul(diff, dc)), r);
        for (int a = 0; a < 3; ++a) {
          G[3 * j + a] = dadd(G[3 * j + a], dmul(g, d[a]));
          G[3 * i + a] = dsub(G[3 * i + a], dmul(g, d[a]));
        }
      }
  }
  return z;
}

/* total force and functional integrand on dual positions; theta != 0 seeds
 * the bias parameters (direction 0: bias_k, direction 1: ramp_rate).
 * Returns 1 if a force is non-finite or above the limit, -1 for the ratchet
 * bias (its running minimum makes the pathwise derivative undefined here). */
static int forces_dual(ora_ctx *c, const dual2 *X, int theta, double t, double z0, int use_cells,
                       dual2 *F, dual2 *S) {
  const ora_sys *s = &c->s;
  int n = s->n_atoms, ns = s->n_solute;
  if (s->bias == ORA_BIAS_RMD_CONTACT) return -1;
  double *xv = (double *)malloc(sizeof(double) * 3 * (size_t)n);
  dual2 *G = (dual2 *)malloc(sizeof(dual2) * 3 * (size_t)(ns > 0 ? ns : 1));
  for (int i = 0; i < 3 * n; ++i) {
    xv[i] = X[i].v;
    F[i] = dn(0.0);
  }
  nb_dual_acc acc = {X, F};
  if (use_cells)
    pairs_cells(c, xv, NULL, 0, nb_visit_dual, &acc);
  else
    pairs_brute(c, xv, NULL, 0, nb_visit_dual, &acc);
  bonded_dual(c, X, F);
  dual2 k = dn(s->bias_k), rho = dn(s->ramp_rate);
  if (theta) {
    k.d[0] = 1.0;
    rho.d[1] = 1.0;
  }
  dual2 Sd = dn(0.0);
  if (s->bias == ORA_BIAS_RG || s->bias == ORA_BIAS_CONTACT) {
    dual2 z = cv_dual(c, X, G);
    dual2 w = dsub(dn(1.0), dscale(t, rho));
    if (w.v < 0.0) w = dn(0.0);
    dual2 zr = dadd(dn(s->z_target), dscale(z0 - s->z_target, w));
    dual2 cb = dscale(-1.0, dmul(k, dsub(z, zr)));
    for (int i = 0; i < ns; ++i) {
      dual2 f2 = dn(0.0);
      for (int a = 0; a < 3; ++a) {
        dual2 fb = dmul(cb, G[3 * i + a]);
        F[3 * i + a] = dadd(F[3 * i + a], fb);
        f2 = dadd(f2, dmul(fb, fb));
      }
      Sd = dadd(Sd, dscale(1.0 / (s->gamma[i] * s->mass[i]), f2));
    }
  } else if (s->bias == ORA_BIAS_CONST && s->const_force) {
    for (int i = 0; i < ns; ++i) {
      double f2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        F[3 * i + a] = dadd(F[3 * i + a], dn(s->const_force[3 * i + a]));
        f2 += s->const_force[3 * i + a] * s->const_force[3 * i + a];
      }
      Sd = dadd(Sd, dn(f2 / (s->gamma[i] * s->mass[i])));
    }
  }
  *S = Sd;
  int bad = 0;
  for (int i = 0; i < 3 * n; ++i)
    if (!isfinite(F[i].v) || fabs(F[i].v) > FORCE_LIMIT) bad = 1;
  free(xv);
  free(G);
  return bad;
}

int ora_forces_dir(ora_ctx *c, const double *x, const double *dx, int32_t theta, double t,
                   const ora_state *st, int32_t use_cells, double *f, double *fdot, double *S,
                   double *Sdot) {
  int n = c->s.n_atoms;
  dual2 *X = (dual2 *)malloc(sizeof(dual2) * 3 * (size_t)n);
  dual2 *F = (dual2 *)malloc(sizeof(dual2) * 3 * (size_t)n);
  for (int i = 0; i < 3 * n; ++i) {
    X[i] = dn(x[i]);
    if (dx)
      for (int k = 0; k < 2; ++k) X[i].d[k] = dx[(size_t)k * 3 * n + i];
  }
  dual2 Sd;
  int bad = forces_dual(c, X, theta, t, st ? st->z0 : 0.0, use_cells, F, &Sd);
  for (int i = 0; i < 3 * n; ++i) {
    if (f) f[i] = F[i].v;
    if (fdot)
      for (int k = 0; k < 2; ++k) fdot[(size_t)k * 3 * n + i] = F[i].d[k];
  }
  if (S) *S = Sd.v;
  if (Sdot) {
    Sdot[0] = Sd.d[0];
    Sdot[1] = Sd.d[1];
  }
  free(X);
  free(F);
  return bad;
}

int ora_init_tangent(ora_ctx *c, const double *x0, const ora_state *st, double *pd) {
  double Sd[2], S;
  int bad = ora_forces_dir(c, x0, NULL, 1, 0.0, st, 1, NULL, NULL, &S, Sd);
  for (int k = 0; k < 2; ++k) {
    pd[k] = 0.5 * Sd[k];
    pd[2 + k] = Sd[k];
  }
  return bad;
}

int ora_run_tangent(ora_ctx *c, double *x, double *v, ora_state *st, double *xt, double *vt,
                    double *pd, int32_t nsteps, int32_t use_cells) {
  const ora_sys *s = &c->s;
  int n = s->n_atoms;
  double dt = s->dt;
  if (st->status) return st->status;
  if (s->bias == ORA_BIAS_RMD_CONTACT) return -1;
  size_t m = 3 * (size_t)n;
  dual2 *X = (dual2 *)malloc(sizeof(dual2) * m);
  dual2 *V = (dual2 *)malloc(sizeof(dual2) * m);
  dual2 *F = (dual2 *)malloc(sizeof(dual2) * m);
  for (size_t i = 0; i < m; ++i) {
    X[i] = dn(x[i]);
    V[i] = dn(v[i]);
    for (int k = 0; k < 2; ++k) {
      X[i].d[k] = xt[k * m + i];
      V[i].d[k] = vt[k * m + i];
    }
  }
  dual2 S;
  int bad = forces_dual(c, X, 1, (double)st->step * dt, st->z0, use_cells, F, &S);
  for (int it = 0; it < nsteps && !bad; ++it) {
    uint32_t step = (uint32_t)st->step;
    for (int i = 0; i < n; ++i) {
      double mi = s->mass[i];
      double c1 = exp(-s->gamma[i] * dt);
      double sd = sqrt((1.0 - c1 * c1) * s->kT / mi);
      double g[3];
      ora_normals(s->seed, (uint32_t)i, step, 0u, g);
      for (int a = 0; a < 3; ++a) {
        size_t q = 3 * (size_t)i + a;
        dual2 vv = dadd(V[q], dscale(0.5 * dt / mi, F[q]));
        dual2 xx = dadd(X[q], dscale(0.5 * dt, vv));
        vv = dadd(dscale(c1, vv), dn(sd * g[a]));
        xx = dadd(xx, dscale(0.5 * dt, vv));
        V[q] = vv;
        X[q] = xx;
      }
    }
    st->step += 1;
    bad = forces_dual(c, X, 1, (double)st->step * dt, st->z0, use_cells, F, &S);
    for (size_t q = 0; q < m; ++q) V[q] = dadd(V[q], dscale(0.5 * dt / s->mass[q / 3], F[q]));
    st->phi_acc += S.v;
    st->s_last = S.v;
    for (int k = 0; k < 2; ++k) {
      pd[k] += S.d[k];
      pd[2 + k] = S.d[k];
    }
  }
  for (size_t i = 0; i < m; ++i) {
    x[i] = X[i].v;
    v[i] = V[i].v;
    for (int k = 0; k < 2; ++k) {
      xt[k * m + i] = X[i].d[k];
      vt[k * m + i] = V[i].d[k];
    }
  }
  free(X);
  free(V);
  free(F);
  if (bad) st->status = 1;
  return bad;
}

void ora_phi_grad(const ora_ctx *c, const ora_state *st, const double *pd, double *out) {
  for (int k = 0; k < 2; ++k)
    out[k] = st->status ? NAN : (pd[k] - 0.5 * pd[2 + k]) * c->s.dt / (4.0 * c->s.kT);
}

/* ------------------------------------------------------------------------ */
/* Toy model (supplement, "Illustrative Application in a Toy Model").        */
/* ------------------------------------------------------------------------ */
double ora_toy_potential(const ora_toy_params *p, double x, double y, double *gx, double *gy) {
  double r2 = x * x + y * y;
  double d1 = r2 + p->s1 * p->s1, d2 = r2 + p->s2 * p->s2;
  double dxm = x - p->xm, dym = y - p->ym;
  double d3 = dxm * dxm + dym * dym + p->s3 * p->s3;
  double a1 = p->A1 * p->s1 * p->s1, a2 = p->A2 * p->s2 * p->s2, a3 = p->A3 * p->s3 * p->s3;
  double u = p->w * p->w * r2 * r2 - a1 / (d1 * d1) + a2 / (d2 * d2) - a3 / (d3 * d3);
  /* d/dr2 of each radial term, then chain rule: d(r2)/dx = 2x */
  double dr2 = 2.0 * p->w * p->w * r2 + 2.0 * a1 / (d1 * d1 * d1) - 2.0 * a2 / (d2 * d2 * d2);
  double dd3 = 2.0 * a3 / (d3 * d3 * d3); /* d/d(d3) of -a3/d3^2 */
  if (gx) *gx = dr2 * 2.0 * x + dd3 * 2.0 * dxm;
  if (gy) *gy = dr2 * 2.0 * y + dd3 * 2.0 * dym;
  return u;
}

/* bias force on the particle for z = |(x, y)|: returns S = |F|^2/(gamma m) */
static double toy_bias(const ora_toy_params *p, int32_t kind, double k, double x, double y, double zm,
                       double *fx, double *fy) {
  double z = sqrt(x * x + y * y);
  *fx = 0.0;
  *fy = 0.0;
  if (kind == ORA_TOY_RMD && z > zm && z > 0.0) {
    /* Eq. VR: -(k/2)(z - z_m) grad z, grad z = (x, y)/z */
    double c = -0.5 * k * (z - zm) / z;
    *fx = c * x;
    *fy = c * y;
  } else if (kind == ORA_TOY_SMD) {
    /* steered MD toward the bottom of the funnel: -K z grad z = -K (x, y) */
    *fx = -k * x;
    *fy = -k * y;
  }
  return (*fx * *fx + *fy * *fy) / (p->gamma * p->mass);
}

void ora_toy_run(const ora_toy_params *p, int32_t kind, double k_bias, uint64_t seed, double *out,
                 double *path) {
  double x = p->x0, y = p->y0, vx, vy;
  double g[3];
  ora_normals(seed, 0u, 0u, 1u, g); /* Maxwell velocities: tag 1 at step 0 */
  double sd0 = sqrt(p->kT / p->mass);
  vx = sd0 * g[0];
  vy = sd0 * g[1];
  double dt = p->dt, m = p->mass;
  double c1 = exp(-p->gamma * dt);
  double sv = sqrt((1.0 - c1 * c1) * p->kT / m);
  double zm = sqrt(x * x + y * y); /* running minimum: z(X_0) */
  double ux, uy, bx, by;
  ora_toy_potential(p, x, y, &ux, &uy);
  double S = toy_bias(p, kind, k_bias, x, y, zm, &bx, &by);
  double fx = -ux + bx, fy = -uy + by;
  double acc = 0.5 * S, s_last = S;
  long long t_reach = -1;
  double theta = NAN;
  double z = zm;
  if (z <= p->r_product) t_reach = 0;
  if (z <= p->r_gate) theta = atan2(y, x);
  if (path) {
    path[0] = x;
    path[1] = y;
  }
  for (int32_t n = 0; n < p->n_steps; ++n) {
    ora_normals(seed, 0u, (uint32_t)n, 2u, g);
    vx += 0.5 * dt * fx / m;
    vy += 0.5 * dt * fy / m;
    x += 0.5 * dt * vx;
    y += 0.5 * dt * vy;
    vx = c1 * vx + sv * g[0];
    vy = c1 * vy + sv * g[1];
    x += 0.5 * dt * vx;
    y += 0.5 * dt * vy;
    z = sqrt(x * x + y * y);
    if (kind == ORA_TOY_RMD && z < zm) zm = z; /* updated before the force (Eq. VR) */
    ora_toy_potential(p, x, y, &ux, &uy);
    S = toy_bias(p, kind, k_bias, x, y, zm, &bx, &by);
    fx = -ux + bx;
    fy = -uy + by;
    vx += 0.5 * dt * fx / m;
    vy += 0.5 * dt * fy / m;
    acc += S;
    s_last = S;
    if (t_reach < 0 && z <= p->r_product) t_reach = n + 1;
    if (isnan(theta) && z <= p->r_gate) theta = atan2(y, x);
    if (path) {
      path[2 * (n + 1)] = x;
      path[2 * (n + 1) + 1] = y;
    }
  }
  out[ORA_TOY_PHI] = (acc - 0.5 * s_last) * dt / (4.0 * p->kT);
  out[ORA_TOY_REACHED] = t_reach >= 0 ? 1.0 : 0.0;
  out[ORA_TOY_T_REACH] = (double)t_reach;
  out[ORA_TOY_X] = x;
  out[ORA_TOY_Y] = y;
  out[ORA_TOY_ZMIN] = kind == ORA_TOY_RMD ? zm : NAN;
  out[ORA_TOY_THETA_GATE] = theta;
}

/* ------------------------------------------------------------------------ */
/* Path similarity (main text, mechanism analysis): the fraction of ordered  */
/* contact pairs whose formation order is the same in both trajectories.     */
/* ------------------------------------------------------------------------ */
static double order_entry(const int64_t *t, int i, int j) {
  if (t[i] < t[j]) return 1.0;
  if (t[i] > t[j]) return 0.0;
  return 0.5;
}

double ora_path_similarity(int32_t nc, const int64_t *ta, const int64_t *tb) {
  if (nc < 2) return NAN;
  int64_t same = 0;
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) {
      if (i == j) continue;
      if (order_entry(ta, i, j) == order_entry(tb, i, j)) ++same;
    }
  return (double)same / ((double)nc * (double)(nc - 1));
}

/* squared distance of atoms i, j of x in squared grid units (exact integers) */
static int64_t grid_d2(const double *x, int i, int j) {
  int64_t s = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t d = llrint(x[3 * j + a] * ORA_QSCALE) - llrint(x[3 * i + a] * ORA_QSCALE);
    s += d * d;
  }
  return s;
}

int64_t ora_native_contacts(const ora_ctx *c, int32_t *pairs, int64_t cap) {
  const ora_sys *s = &c->s;
  if (!s->x_final) return 0;
  int64_t r0 = llrint(s->contact_r0 * ORA_QSCALE), n = 0;
  for (int i = 0; i < s->n_solute; ++i)
    for (int j = i + s->contact_min_sep + 1; j < s->n_solute; ++j) {
      if (grid_d2(s->x_final, i, j) > r0 * r0) continue;
      if (pairs && n < cap) {
        pairs[2 * n] = i;
        pairs[2 * n + 1] = j;
      }
      ++n;
    }
  return n;
}

void ora_contacts_formed(const ora_ctx *c, const double *x, const int32_t *pairs, int64_t nc,
                         uint8_t *formed) {
  int64_t r0 = llrint(c->s.contact_r0 * ORA_QSCALE);
  for (int64_t k = 0; k < nc; ++k) formed[k] = grid_d2(x, pairs[2 * k], pairs[2 * k + 1]) <= r0 * r0;
}
