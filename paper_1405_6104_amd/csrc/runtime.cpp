// Host runtime of the vp C ABI: validation, device layout, uploads, the step
// schedule (direct launches or replayed hipGraphs), the functional and the
// variational selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <string>
#include <vector>

#include "vp_internal.h"
#include "vp_launch.h"

using namespace vp;

namespace {

thread_local std::string g_err;

vp_status fail(vp_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIPCHECK(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(VP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// Device memory through the caller's allocator (vp_options.dev_alloc) when
// one is given, else hipMalloc.
void *raw_alloc(const vp_system *s, size_t bytes) {
  if (s->opt.dev_alloc) return s->opt.dev_alloc(bytes, s->opt.alloc_ctx);
  void *q = nullptr;
  return hipMalloc(&q, bytes) == hipSuccess ? q : nullptr;
}

void raw_free(const vp_system *s, void *q) {
  if (!q) return;
  if (s->opt.dev_free)
    s->opt.dev_free(q, s->opt.alloc_ctx);
  else
    (void)hipFree(q);
}

template <class T>
vp_status dalloc(vp_system *s, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  void *q = raw_alloc(s, sizeof(T) * count);
  if (!q) return fail(VP_ERR_NOMEM, "device allocation failed: " + std::to_string(sizeof(T) * count) + " bytes");
  s->allocations.push_back(q);
  s->device_bytes += (int64_t)(sizeof(T) * count);
  *p = (T *)q;
  return VP_OK;
}

// A temporary device buffer of a diagnostic call, released on scope exit.
struct TmpBuf {
  const vp_system *s;
  void *p = nullptr;
  TmpBuf(const vp_system *sys, size_t bytes) : s(sys) { p = raw_alloc(sys, bytes ? bytes : 1); }
  ~TmpBuf() { raw_free(s, p); }
  TmpBuf(const TmpBuf &) = delete;
  TmpBuf &operator=(const TmpBuf &) = delete;
};

// Ordering of the calls of one system across streams: an asynchronous call
// first waits for the previous call's work if that went to another stream,
// and records the system's event after its own work.
hipError_t begin_async(vp_system *s, hipStream_t st) {
  if (s->done_valid && st != s->last_stream) return hipStreamWaitEvent(st, s->done, 0);
  return hipSuccess;
}

hipError_t end_async(vp_system *s, hipStream_t st) {
  hipError_t e = hipEventRecord(s->done, st);
  s->done_valid = e == hipSuccess;
  s->last_stream = st;
  return e;
}

// Waits for all work of the system's calls.
hipError_t sync_system(vp_system *s) {
  if (s->done_valid) return hipEventSynchronize(s->done);
  return hipSuccess;
}

template <class T>
vp_status upload(vp_system *s, T **p, const std::vector<T> &h) {
  vp_status st = dalloc(s, p, h.size());
  if (st != VP_OK) return st;
  if (!h.empty()) HIPCHECK(hipMemcpy(*p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return VP_OK;
}

#define TRY(expr)                     \
  do {                                \
    vp_status s_ = (expr);            \
    if (s_ != VP_OK) return s_;       \
  } while (0)

vp_status validate(const vp_replica_desc &d, int r, bool tangent) {
  auto bad = [&](const std::string &m) { return fail(VP_ERR_ARG, "replica " + std::to_string(r) + ": " + m); };
  if (d.n_atoms <= 0 || d.n_atoms > 65536) return bad("n_atoms must be in [1, 65536]");
  if (d.n_solute < 0 || d.n_solute > d.n_atoms) return bad("n_solute out of range");
  if (!d.mass || !d.gamma || !d.charge || !d.sigma || !d.epsilon || !d.x0)
    return bad("NULL per-atom array");
  for (int a = 0; a < 3; ++a)
    if (!(d.box[a] > 0) || !(d.box[a] <= 30.0)) return bad("box edges must lie in (0, 30] nm");
  if (!(d.r_cut > 0)) return bad("r_cut must be positive");
  for (int a = 0; a < 3; ++a)
    if (!(d.r_cut < 0.5 * d.box[a])) return bad("r_cut must be below half the box");
  if (!(d.dt > 0) || !(d.kT > 0)) return bad("dt and kT must be positive");
  for (int i = 0; i < d.n_atoms; ++i) {
    if (!(d.mass[i] > 0)) return bad("masses must be positive");
    if (!(d.gamma[i] >= 0)) return bad("frictions must be non-negative");
    if (i < d.n_solute && d.bias != VP_BIAS_NONE && !(d.gamma[i] > 0))
      return bad("solute frictions must be positive (the functional divides by gamma m)");
    if (!(d.sigma[i] >= 0) || !(d.epsilon[i] >= 0)) return bad("sigma and epsilon must be >= 0");
  }
  if (d.n_bonds < 0 || (d.n_bonds > 0 && (!d.bonds || !d.bond_k || !d.bond_r0))) return bad("bond arrays");
  for (int b = 0; b < d.n_bonds; ++b)
    for (int k = 0; k < 2; ++k)
      if (d.bonds[2 * b + k] < 0 || d.bonds[2 * b + k] >= d.n_atoms) return bad("bond index out of range");
  for (int b = 0; b < d.n_bonds; ++b)
    if (d.bonds[2 * b] == d.bonds[2 * b + 1]) return bad("a bond joins an atom to itself");
  if (d.n_angles < 0 || (d.n_angles > 0 && (!d.angles || !d.angle_k || !d.angle_theta0)))
    return bad("angle arrays");
  for (int b = 0; b < d.n_angles; ++b)
    for (int k = 0; k < 3; ++k)
      if (d.angles[3 * b + k] < 0 || d.angles[3 * b + k] >= d.n_atoms) return bad("angle index out of range");
  for (int b = 0; b < d.n_angles; ++b) {
    const int32_t *q = d.angles + 3 * b;
    if (q[0] == q[1] || q[1] == q[2] || q[0] == q[2]) return bad("an angle names one atom twice");
  }
  if (d.n_excl < 0 || (d.n_excl > 0 && !d.excl)) return bad("exclusion array");
  for (int b = 0; b < d.n_excl; ++b)
    for (int k = 0; k < 2; ++k)
      if (d.excl[2 * b + k] < 0 || d.excl[2 * b + k] >= d.n_atoms) return bad("excluded index out of range");
  if (d.bias < VP_BIAS_NONE || d.bias > VP_BIAS_RMD_CONTACT) return bad("unknown bias kind");
  if (tangent && d.bias == VP_BIAS_RMD_CONTACT)
    return bad("derivatives are not available for the ratchet bias (its running minimum is not differentiable)");
  if ((d.bias == VP_BIAS_CONTACT || d.bias == VP_BIAS_RMD_CONTACT)) {
    if (!d.x_final) return bad("contact-map bias needs x_final");
    if (d.n_solute > kMaxCvBlocks * kCvTile) return bad("too many solute atoms for the contact map");
    if (!(d.contact_r0 > 0) || !(d.contact_rc > d.contact_rs) || d.contact_min_sep < 0)
      return bad("contact parameters");
  }
  if (d.bias == VP_BIAS_CONST && !d.const_force) return bad("constant bias needs const_force");
  if (d.bias != VP_BIAS_NONE && d.n_solute < 1) return bad("a bias needs at least one solute atom");
  if (d.bias == VP_BIAS_RG || d.bias == VP_BIAS_CONTACT || d.bias == VP_BIAS_RMD_CONTACT)
    if (!(d.bias_k >= 0) || !(d.ramp_rate >= 0)) return bad("bias_k and ramp_rate must be >= 0");
  if (d.bias == VP_BIAS_RG && d.n_solute > kMaxSoluteLds)
    return bad("the radius-of-gyration bias takes at most 4096 solute atoms");
  if (std::isnan(d.reach_tol) || std::isnan(d.reach_rmsd)) return bad("reach_tol and reach_rmsd must not be NaN");
  if (std::isfinite(d.reach_rmsd) && (!d.x_final || d.n_solute < 1))
    return bad("an RMSD criterion (finite reach_rmsd) needs x_final");
  return VP_OK;
}

}  // namespace

static vp_status alloc_work(vp_system *s, Work &W, bool traj) {
  size_t S = (size_t)s->n_slots, U = (size_t)s->n_users, R = (size_t)s->R, B = (size_t)s->n_blocks;
  TRY(dalloc(s, &W.xq, S));
  if (traj) {
    TRY(dalloc(s, &W.vel, S));
    TRY(dalloc(s, &W.xref, S));
  }
  TRY(dalloc(s, &W.integ, S));
  TRY(dalloc(s, &W.orig, S));
  TRY(dalloc(s, &W.wrap, S));
  TRY(dalloc(s, &W.inv, U));
  TRY(dalloc(s, &W.F, 3 * S));
  W.fstride = (int64_t)S;
  TRY(dalloc(s, &W.nbcnt, S));
  TRY(dalloc(s, &W.nblj, S));
  TRY(dalloc(s, &W.nblist, (size_t)s->list_elems));
  TRY(dalloc(s, &W.stage_n, B));
  TRY(dalloc(s, &W.bctr, B));
  W.stage_stride = s->stage_cap_max;
  TRY(dalloc(s, &W.stage, B * (size_t)W.stage_stride));
  TRY(dalloc(s, &W.cell_start, (size_t)s->n_cells));
  TRY(dalloc(s, &W.cell_slots, S));
  TRY(dalloc(s, &W.cell_of, S));
  TRY(dalloc(s, &W.g, (size_t)std::max<int64_t>(1, s->n_solute_total)));
  TRY(dalloc(s, &W.gtile, (size_t)std::max<int64_t>(1, s->n_cv_tiles) * kCvTile));
  TRY(dalloc(s, &W.ztile, (size_t)std::max<int64_t>(1, s->n_cv_tiles)));
  TRY(dalloc(s, &W.zpart, R * kMaxCvBlocks));
  TRY(dalloc(s, &W.gpart, R * kMaxCvBlocks));
  TRY(dalloc(s, &W.epart, (size_t)kEp * B));
  TRY(dalloc(s, &W.flags, R));
  if (traj) TRY(dalloc(s, &W.ke_tile, (size_t)s->n_tiles));
  if (s->tangent) {
    const size_t CT = (size_t)std::max<int64_t>(1, s->n_cv_tiles) * kCvTile;
    const size_t NS = (size_t)std::max<int64_t>(1, s->n_solute_total);
    W.cvstride = (int64_t)CT;
    W.solstride = (int64_t)NS;
    TRY(dalloc(s, &W.tx, 2 * S));
    TRY(dalloc(s, &W.tv, 2 * S));
    TRY(dalloc(s, &W.tf, 2 * S));
    TRY(dalloc(s, &W.tg, 2 * NS));
    TRY(dalloc(s, &W.tgtile, 2 * CT));
    TRY(dalloc(s, &W.tzpart, 2 * R * kMaxCvBlocks));
    TRY(dalloc(s, &W.tgpart, 2 * R * kMaxCvBlocks));
    HIPCHECK(hipMemset(W.tx, 0, sizeof(float4) * 2 * S));
    HIPCHECK(hipMemset(W.tv, 0, sizeof(float4) * 2 * S));
    HIPCHECK(hipMemset(W.tf, 0, sizeof(float4) * 2 * S));
    HIPCHECK(hipMemset(W.tg, 0, sizeof(float4) * 2 * NS));
    HIPCHECK(hipMemset(W.tgtile, 0, sizeof(float4) * 2 * CT));
    HIPCHECK(hipMemset(W.tzpart, 0, sizeof(double) * 2 * R * kMaxCvBlocks));
    HIPCHECK(hipMemset(W.tgpart, 0, sizeof(double) * 2 * R * kMaxCvBlocks));
  }
  HIPCHECK(hipMemset(W.nbcnt, 0, sizeof(int32_t) * S));
  HIPCHECK(hipMemset(W.nblj, 0, sizeof(int32_t) * S));
  HIPCHECK(hipMemset(W.stage_n, 0, sizeof(int32_t) * B));
  HIPCHECK(hipMemset(W.orig, 0xff, sizeof(int32_t) * S));
  HIPCHECK(hipMemset(W.wrap, 0, sizeof(int32_t) * S));
  HIPCHECK(hipMemset(W.zpart, 0, sizeof(double) * R * kMaxCvBlocks));
  HIPCHECK(hipMemset(W.gpart, 0, sizeof(double) * R * kMaxCvBlocks));
  HIPCHECK(hipMemset(W.epart, 0, sizeof(double) * kEp * B));
  HIPCHECK(hipMemset(W.flags, 0, sizeof(int32_t) * R));
  if (traj) HIPCHECK(hipMemset(W.ke_tile, 0, sizeof(double) * (size_t)s->n_tiles));
  HIPCHECK(hipMemset(W.F, 0, sizeof(long long) * 3 * S));
  return VP_OK;
}

static void free_all(vp_system *s) {
  for (hipEvent_t e : s->ev_before) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->ev_after) (void)hipEventDestroy(e);
  s->ev_before.clear();
  s->ev_after.clear();
  for (auto &g : s->graphs) {
    (void)hipGraphExecDestroy(g.exec);
  }
  s->graphs.clear();
  for (void *p : s->allocations) raw_free(s, p);
  s->allocations.clear();
  s->device_bytes = 0;
}

// distinct (charge, sigma, epsilon) classes of a replica (its type-table size)
static int count_types(const vp_replica_desc &d) {
  std::set<std::tuple<double, double, double>> cls;
  for (int i = 0; i < d.n_atoms; ++i) cls.emplace(d.charge[i], d.sigma[i], d.epsilon[i]);
  return (int)cls.size();
}

// Staged neighbourhood a 64-atom block may need: atoms within rl of a compact
// block (side ~0.93 (64/rho)^(1/3)), with a margin for the blocks that turn
// from one column into the next (every atom within rl of a quarter's box is
// staged).
static int stage_estimate(double rl, double rho) {
  const double a = 0.93 * std::cbrt(kBlk / rho);
  const double vst = a * a * a + 6.0 * a * a * rl + 3.0 * M_PI * a * rl * rl + 4.0 / 3.0 * M_PI * rl * rl * rl;
  return (int)std::ceil(1.5 * vst * rho + 128);
}

// Pair-list buffer and rebuild interval of one replica.  Given values are used
// as they are.  By default:
//  - the skin may be at most the largest of 0.14, 0.13, ... nm whose staged
//    neighbourhood fits the force kernel's LDS and whose list radius stays
//    below half the box;
//  - the interval is the largest power of two (up to 32) in which a fast atom
//    (5 sigma of the Maxwell speed of the lightest atom, the onset of the
//    displacement rebuilds measured in water at 300 K) moves less than half of
//    that maximal skin, and the skin is then just large enough for that
//    interval (rounded up to 0.01 nm).
// Powers of two keep the rebuild steps of replicas with different intervals
// aligned (every rebuild step of a replica with interval 2k is one of a
// replica with interval k), so rebuilds share launches; a rebuild still
// happens earlier whenever an atom has moved half the skin.
static void list_params(const vp_replica_desc &d, const vp_options &o, int ntypes_max, double *skin,
                        int *nstlist) {
  const double rho = d.n_atoms / (d.box[0] * d.box[1] * d.box[2]);
  const double half = 0.5 * std::min({d.box[0], d.box[1], d.box[2]});
  double cap = o.skin;
  if (!(cap > 0)) {
    const long long budget = (long long)kMaxLds / (long long)sizeof(int4) - (ntypes_max + 1) - kStageDummies;
    cap = 0.14;
    while (cap > 0.025 && (stage_estimate(d.r_cut + cap, rho) > std::min<long long>(budget, kMaxStage) ||
                           !(d.r_cut + cap < half)))
      cap -= 0.01;
  }
  double mmin = d.mass[0];
  for (int i = 1; i < d.n_atoms; ++i) mmin = std::min(mmin, d.mass[i]);
  const double step_disp = 5.0 * std::sqrt(d.kT / mmin) * d.dt;  // nm per step of a fast atom
  int nst = o.nstlist;
  if (nst <= 0) {
    nst = 1;
    while (nst < 32 && 2 * nst * step_disp <= 0.49 * cap) nst *= 2;
  }
  *nstlist = nst;
  if (o.skin > 0) {
    *skin = o.skin;
  } else {
    const double need = std::ceil(nst * step_disp / 0.49 * 100.0 - 1e-9) / 100.0;
    *skin = std::max(0.02, std::min(cap, need));
  }
}

// Native contacts of every replica that gives X_f (one list per distinct
// X_f, min_sep and r0): solute pairs i < j, j - i > min_sep, whose squared
// distance on the 2^-22 nm grid is at most (r0 on that grid)^2, exactly in
// integers; the formation steps start at -1.
static vp_status native_contacts(vp_system *s, const vp_replica_desc *reps) {
  std::vector<int2> pairs;
  struct Key {
    const double *xf;
    int ns, sep;
    double r0;
    int off, n;
  };
  std::vector<Key> seen;
  int64_t tf = 0;
  for (int r = 0; r < s->R; ++r) {
    const vp_replica_desc &d = reps[r];
    RepInfo &R = s->info_h[r];
    R.n_contacts = 0;
    R.cp_off = 0;
    R.tf_off = (int32_t)tf;
    const int64_t r0q = std::llrint(d.contact_r0 * kQ);
    R.r0q2 = r0q * r0q;
    if (!d.x_final || d.n_solute < 2 || !(d.contact_r0 > 0)) continue;
    int found = -1;
    for (size_t k = 0; k < seen.size(); ++k)
      if (seen[k].ns == d.n_solute && seen[k].sep == d.contact_min_sep && seen[k].r0 == d.contact_r0 &&
          std::memcmp(seen[k].xf, d.x_final, sizeof(double) * 3 * (size_t)d.n_solute) == 0)
        found = (int)k;
    if (found < 0) {
      Key k{d.x_final, d.n_solute, d.contact_min_sep, d.contact_r0, (int)pairs.size(), 0};
      std::vector<int64_t> q(3 * (size_t)d.n_solute);
      for (size_t i = 0; i < q.size(); ++i) q[i] = std::llrint(d.x_final[i] * kQ);
      for (int i = 0; i < d.n_solute; ++i)
        for (int j = i + std::max(0, d.contact_min_sep) + 1; j < d.n_solute; ++j) {
          int64_t d2 = 0;
          for (int a = 0; a < 3; ++a) {
            const int64_t e = q[3 * j + a] - q[3 * i + a];
            d2 += e * e;
          }
          if (d2 <= R.r0q2) pairs.push_back(make_int2(i, j));
        }
      k.n = (int)pairs.size() - k.off;
      seen.push_back(k);
      found = (int)seen.size() - 1;
    }
    R.cp_off = seen[found].off;
    R.n_contacts = seen[found].n;
    tf += R.n_contacts;
    s->max_contacts = std::max(s->max_contacts, R.n_contacts);
  }
  TRY(upload(s, &s->cpairs, pairs));
  TRY(dalloc(s, &s->t_form, (size_t)std::max<int64_t>(1, tf)));
  HIPCHECK(hipMemset(s->t_form, 0xff, sizeof(int32_t) * (size_t)std::max<int64_t>(1, tf)));
  HIPCHECK(hipMemcpy(s->info, s->info_h.data(), sizeof(RepInfo) * s->R, hipMemcpyHostToDevice));
  return VP_OK;
}

static vp_status build(vp_system *s, const vp_replica_desc *reps, int32_t n_reps) {
  const vp_options &o = s->opt;
  int ntypes_all = 0;
  for (int r = 0; r < n_reps; ++r) ntypes_all = std::max(ntypes_all, count_types(reps[r]));
  s->R = n_reps;
  s->info_h.resize(n_reps);
  int64_t off = 0, uoff = 0, cell0 = 0, list_off = 0, sol_off = 0, cv_tiles = 0, xf_rows = 0;
  int32_t tile0 = 0, type_off = 0;
  std::vector<int32_t> tile_rep, tile_first;
  std::vector<float4> types;
  std::vector<int32_t> type0;
  struct MapKey {
    const double *xf;
    int ns, sep;
    double r0, rs, rc;
  };
  std::vector<MapKey> maps;
  std::vector<int64_t> map_off, skew_off;
  int64_t cmap_total = 0, skew_total = 0;
  int stage_cap_max = 0, ntypes_max = 0;
  const double cell_target = 0.45;  // nm: fine cells of the candidate search
  const double col_target = 0.8;    // nm: xy columns of the sort order
  for (int r = 0; r < n_reps; ++r) {
    const vp_replica_desc &d = reps[r];
    RepInfo &R = s->info_h[r];
    std::memset(&R, 0, sizeof(R));
    R.n = d.n_atoms;
    R.ns = d.n_solute;
    R.npad = (d.n_atoms + kTile - 1) / kTile * kTile;
    R.off = (int32_t)off;
    R.uoff = (int32_t)uoff;
    R.tile0 = tile0;
    R.ntiles = R.npad / kTile;
    R.blk0 = tile0 * (kTile / kBlk);
    for (int t = 0; t < R.ntiles; ++t) {
      tile_rep.push_back(r);
      tile_first.push_back(t * kTile);
    }
    R.bias = d.bias;
    R.min_sep = d.contact_min_sep;
    double skin = 0.0;
    int nstlist = 1;
    list_params(d, o, ntypes_all, &skin, &nstlist);
    const double rl = d.r_cut + skin;
    if (!(rl < 0.5 * std::min({d.box[0], d.box[1], d.box[2]})))
      return fail(VP_ERR_ARG, "replica " + std::to_string(r) + ": r_cut + skin must be below half the box");
    for (int a = 0; a < 3; ++a) {
      int nc = (int)std::floor(d.box[a] / cell_target);
      R.nc[a] = std::max(1, std::min(nc, 16));
      R.Lq[a] = (int32_t)std::llrint(d.box[a] * kQ);
      R.Ld[a] = d.box[a];
    }
    R.ncell = R.nc[0] * R.nc[1] * R.nc[2];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k <= R.nc[a]; ++k)
        R.cedge[a][k] = (int32_t)(((int64_t)k * R.Lq[a]) / R.nc[a]);
    R.cell0 = (int32_t)cell0;
    for (int a = 0; a < 2; ++a) R.ncol[a] = std::max(1, std::min(16, (int)std::floor(d.box[a] / col_target)));
    R.nzb = std::max(1, std::min(64, kMaxCells / (R.ncol[0] * R.ncol[1])));
    const double vol = d.box[0] * d.box[1] * d.box[2];
    const double rho = d.n_atoms / vol;
    const double expect = 4.0 / 3.0 * M_PI * rl * rl * rl * rho;
    int maxnb = o.max_neighbors > 0 ? o.max_neighbors : (int)std::ceil(1.5 * expect + 64);
    if (o.max_neighbors <= 0 && r < (int)s->maxnb_override.size() && s->maxnb_override[r] > 0)
      maxnb = s->maxnb_override[r];
    maxnb = std::min(maxnb, d.n_atoms + 8);
    maxnb = ((maxnb + 7) / 8 * 8 + 8 + 8 * kListGroup - 1) / (8 * kListGroup) * (8 * kListGroup);
    R.maxnb = maxnb;
    int cap = std::min(kMaxStage, std::min(stage_estimate(rl, rho), d.n_atoms * 27 + 8));
    R.stage_cap = cap;
    stage_cap_max = std::max(stage_cap_max, cap);
    R.list_off = list_off;
    R.sol_off = (int32_t)sol_off;
    R.nstlist = nstlist;
    R.skin = skin;
    const double rcq = d.r_cut * kQ, rlq = rl * kQ;
    R.rc2q = (float)(rcq * rcq);
    R.rl2q = (float)(rlq * rlq);
    R.rlq = (int32_t)std::ceil(rlq);
    R.rc = d.r_cut;
    R.krf = (d.eps_rf - 1.0) / ((2.0 * d.eps_rf + 1.0) * d.r_cut * d.r_cut * d.r_cut);
    R.crf = 1.0 / d.r_cut + R.krf * d.r_cut * d.r_cut;
    R.krf2q = (float)(2.0 * R.krf / (kQ * kQ * kQ));
    R.half_skin_margin = (float)(0.5 * skin * 0.98);
    R.cr0 = (float)d.contact_r0;
    R.crs = (float)d.contact_rs;
    R.crc = (float)d.contact_rc;
    R.bias_k = d.bias_k;
    R.ramp_rate = d.ramp_rate;
    R.z_target = d.z_target;
    R.kT = d.kT;
    R.dt = d.dt;
    R.reach_tol = d.reach_tol;
    R.reach_rmsd = d.reach_rmsd;
    R.xf_off = -1;
    if (d.x_final && d.n_solute > 0) {
      R.xf_off = (int32_t)xf_rows;
      xf_rows += d.n_solute;
    }
    R.seed = d.seed;
    // (charge, sigma, epsilon) classes of this replica, those with epsilon > 0
    // first (in order of first appearance within each group); the last entry
    // is inert
    {
      std::map<std::tuple<double, double, double>, int> cls;
      std::vector<int> first;  // an atom of each class, by first appearance
      std::vector<int> cl(d.n_atoms);
      for (int i = 0; i < d.n_atoms; ++i) {
        auto key = std::make_tuple(d.charge[i], d.sigma[i], d.epsilon[i]);
        auto it = cls.find(key);
        if (it == cls.end()) {
          cl[i] = (int)first.size();
          cls.emplace(key, cl[i]);
          first.push_back(i);
        } else {
          cl[i] = it->second;
        }
      }
      if ((int)first.size() >= kMaxTypes)
        return fail(VP_ERR_ARG, "replica " + std::to_string(r) + ": more than 1023 distinct (charge, sigma, epsilon)");
      std::vector<int> renum(first.size());
      std::vector<float4> tab;
      for (int pass = 0; pass < 2; ++pass)
        for (size_t c = 0; c < first.size(); ++c) {
          const int i = first[c];
          if ((d.epsilon[i] > 0.0) != (pass == 0)) continue;
          renum[c] = (int)tab.size();
          tab.push_back(make_float4((float)(d.charge[i] * std::sqrt(kCoulomb) * kQ * std::sqrt(kQ)),
                                    (float)(0.5 * d.sigma[i] * kQ),
                                    (float)(std::sqrt(24.0 * d.epsilon[i]) * kQ), 0.0f));
          if (pass == 0) R.nlj_types = (int32_t)tab.size();
        }
      for (int i = 0; i < d.n_atoms; ++i) type0.push_back(renum[cl[i]]);
      R.ntypes = (int32_t)tab.size();
      R.type_off = type_off;
      tab.push_back(make_float4(0.f, 0.f, 0.f, 0.f));
      types.insert(types.end(), tab.begin(), tab.end());
      type_off += (int32_t)tab.size();
      ntypes_max = std::max(ntypes_max, R.ntypes);
    }
    const bool contact = d.bias == VP_BIAS_CONTACT || d.bias == VP_BIAS_RMD_CONTACT;
    R.cv_blocks = contact ? std::max(1, (d.n_solute + kCvTile - 1) / kCvTile) : 1;
    R.cvt_off = cv_tiles;
    if (contact) cv_tiles += (int64_t)R.cv_blocks * R.cv_blocks;
    R.cinv_r02 = (float)(1.0 / (d.contact_r0 * d.contact_r0));
    R.cinv_w = (float)(1.0 / (d.contact_rc - d.contact_rs));
    R.crs2 = (float)(d.contact_rs * d.contact_rs);
    R.crc2 = (float)(d.contact_rc * d.contact_rc);
    R.cmap_off = 0;
    R.cskew_off = 0;
    if (contact) {
      int found = -1;
      for (size_t m = 0; m < maps.size(); ++m) {
        const MapKey &k = maps[m];
        if (k.ns == d.n_solute && k.sep == d.contact_min_sep && k.r0 == d.contact_r0 &&
            k.rs == d.contact_rs && k.rc == d.contact_rc &&
            std::memcmp(k.xf, d.x_final, sizeof(double) * 3 * d.n_solute) == 0) {
          found = (int)m;
          break;
        }
      }
      if (found < 0) {
        maps.push_back({d.x_final, d.n_solute, d.contact_min_sep, d.contact_r0, d.contact_rs, d.contact_rc});
        map_off.push_back(cmap_total);
        cmap_total += (int64_t)d.n_solute * d.n_solute;
        skew_off.push_back(skew_total);
        skew_total += (int64_t)R.cv_blocks * R.cv_blocks * kCvTile * kCvTile;
        found = (int)maps.size() - 1;
      }
      R.cmap_off = map_off[found];
      R.cskew_off = skew_off[found];
    }
    off += R.npad;
    uoff += R.n;
    cell0 += R.ncell + 1;
    list_off += (int64_t)maxnb * R.npad;
    sol_off += R.ns;
    tile0 += R.ntiles;
  }
  s->n_slots = off;
  s->n_users = uoff;
  s->n_cells = cell0;
  s->list_elems = list_off;
  s->n_solute_total = sol_off;
  s->n_cv_tiles = cv_tiles;
  s->n_tiles = tile0;
  s->n_blocks = tile0 * (kTile / kBlk);
  s->ntypes_max = ntypes_max;
  {
    // Staging capacity: every block may use the LDS that still lets two
    // force workgroups share a CU (up to the staging array's size), and never
    // less than the estimate above; a block whose candidates would overflow
    // it is built again in exact mode.
    const long long budget = (long long)kMaxLds / (long long)sizeof(int4) - (ntypes_max + 1) - kStageDummies;
    stage_cap_max = 0;
    for (int r = 0; r < n_reps; ++r) {
      RepInfo &R = s->info_h[r];
      long long want = std::min<long long>({(long long)kMaxStage, budget, 27ll * R.n + 8});
      if (o.stage_cap > 0) {
        want = std::min<long long>(want, o.stage_cap);  // diagnostic: exact-mode builds
      } else if (want < R.stage_cap) {
        return fail(VP_ERR_ARG, "replica " + std::to_string(r) + ": its neighbourhoods need " +
                                    std::to_string(R.stage_cap) + " staged atoms; the force kernel's LDS holds " +
                                    std::to_string(want));
      }
      R.stage_cap = (int32_t)want;
      stage_cap_max = std::max(stage_cap_max, R.stage_cap);
    }
    s->stage_cap_max = stage_cap_max;
    size_t need = force_lds_bytes(s);
    if (need > (size_t)kMaxLds)
      return fail(VP_ERR_ARG, "force kernel would need " + std::to_string(need) +
                                  " bytes of LDS per workgroup (limit " + std::to_string(kMaxLds) + ")");
    HIPCHECK(prepare_forces(s));
    HIPCHECK(prepare_energies(s));
    if (s->tangent) {
      const size_t tneed = tangent_lds_bytes(s);
      if (tneed > (size_t)kMaxLdsTangent)
        return fail(VP_ERR_ARG, "tangent force kernel would need " + std::to_string(tneed) +
                                    " bytes of LDS per workgroup (limit " +
                                    std::to_string(kMaxLdsTangent) + ")");
      HIPCHECK(prepare_tangent(s));
    }
  }

  // ---------------- constant per-atom data (user order)
  const size_t U = (size_t)s->n_users;
  std::vector<float4> integ0(U);
  std::vector<double> igm0(U), mass0(U);
  std::vector<int32_t> xh(3 * U);
  std::vector<float> vh(3 * U, 0.0f);
  std::vector<uint8_t> has_v(n_reps, 0);
  std::vector<std::vector<BTerm>> terms(U);
  std::vector<std::vector<int32_t>> excl(U);
  std::vector<float4> cforce(std::max<int64_t>(1, s->n_solute_total), make_float4(0, 0, 0, 0));
  std::vector<double> xf_h(3 * (size_t)std::max<int64_t>(1, xf_rows), 0.0);
  for (int r = 0; r < n_reps; ++r) {
    const vp_replica_desc &d = reps[r];
    const RepInfo &R = s->info_h[r];
    for (int i = 0; i < d.n_atoms; ++i) {
      size_t u = (size_t)R.uoff + i;
      double c1 = std::exp(-d.gamma[i] * d.dt);
      double sv = std::sqrt((1.0 - c1 * c1) * d.kT / d.mass[i]);
      integ0[u] = make_float4((float)(1.0 / d.mass[i]), (float)c1, (float)sv, 0.0f);
      igm0[u] = d.gamma[i] > 0 ? 1.0 / (d.gamma[i] * d.mass[i]) : 0.0;
      mass0[u] = d.mass[i];
      for (int a = 0; a < 3; ++a) {
        double xq = d.x0[3 * i + a] * kQ;
        if (!(std::fabs(xq) < 1.0e9))
          return fail(VP_ERR_ARG, "replica " + std::to_string(r) + ": coordinates must lie within 238 nm of the origin");
        xh[3 * u + a] = (int32_t)std::llrint(xq);
        if (d.v0) vh[3 * u + a] = (float)d.v0[3 * i + a];
      }
    }
    has_v[r] = d.v0 ? 1 : 0;
    for (int b = 0; b < d.n_bonds; ++b) {
      int i = d.bonds[2 * b], j = d.bonds[2 * b + 1];
      terms[R.uoff + i].push_back({0, j, 0, b, d.bond_k[b], d.bond_r0[b]});
      terms[R.uoff + j].push_back({0, i, 0, b, d.bond_k[b], d.bond_r0[b]});
    }
    for (int b = 0; b < d.n_angles; ++b) {
      int i = d.angles[3 * b], c = d.angles[3 * b + 1], j = d.angles[3 * b + 2];
      const int ord = d.n_bonds + b;
      terms[R.uoff + i].push_back({1, c, j, ord, d.angle_k[b], d.angle_theta0[b]});
      terms[R.uoff + j].push_back({1, c, i, ord, d.angle_k[b], d.angle_theta0[b]});
      terms[R.uoff + c].push_back({2, i, j, ord, d.angle_k[b], d.angle_theta0[b]});
    }
    for (int e = 0; e < d.n_excl; ++e) {
      int i = d.excl[2 * e], j = d.excl[2 * e + 1];
      if (i == j) continue;
      excl[R.uoff + i].push_back(j);
      excl[R.uoff + j].push_back(i);
    }
    if (R.xf_off >= 0)
      std::memcpy(&xf_h[3 * (size_t)R.xf_off], d.x_final, sizeof(double) * 3 * (size_t)d.n_solute);
    if (d.bias == VP_BIAS_CONST)
      for (int i = 0; i < d.n_solute; ++i)
        cforce[R.sol_off + i] = make_float4((float)d.const_force[3 * i], (float)d.const_force[3 * i + 1],
                                            (float)d.const_force[3 * i + 2], 0.0f);
  }
  std::vector<int32_t> bt_start(U + 1, 0), ex_start(U + 1, 0), ex_list;
  std::vector<BTerm> bterms;
  for (size_t u = 0; u < U; ++u) {
    bt_start[u] = (int32_t)bterms.size();
    bterms.insert(bterms.end(), terms[u].begin(), terms[u].end());
    std::sort(excl[u].begin(), excl[u].end());
    excl[u].erase(std::unique(excl[u].begin(), excl[u].end()), excl[u].end());
    ex_start[u] = (int32_t)ex_list.size();
    ex_list.insert(ex_list.end(), excl[u].begin(), excl[u].end());
  }
  bt_start[U] = (int32_t)bterms.size();
  ex_start[U] = (int32_t)ex_list.size();
  // Three-atom sites (water molecules): atoms i, i+1, i+2 of a replica that
  // exclude each other and nothing else, the last two without LJ parameters.
  // The list build names such a site by one entry (role 1: its first atom,
  // role 2: the other two); every other atom is listed on its own (role 0).
  std::vector<int32_t> role0(U, 0);
  for (int r = 0; r < n_reps; ++r) {
    const vp_replica_desc &d = reps[r];
    const size_t u0 = (size_t)s->info_h[r].uoff;
    auto only = [&](size_t v, int32_t p, int32_t q) {
      return excl[v].size() == 2 && excl[v][0] == p && excl[v][1] == q;
    };
    for (int i = 0; i + 2 < d.n_atoms;) {
      const size_t u = u0 + (size_t)i;
      if (only(u, i + 1, i + 2) && only(u + 1, i, i + 2) && only(u + 2, i, i + 1) && d.epsilon[i + 1] == 0.0 &&
          d.epsilon[i + 2] == 0.0) {
        role0[u] = 1;
        role0[u + 1] = 2;
        role0[u + 2] = 2;
        i += 3;
      } else {
        ++i;
      }
    }
  }

  // Force-only bonded tables.  Bonded groups: three consecutive atoms i, i+1,
  // i+2 of a replica, each with terms only among the three and at most
  // kGroupTerms terms in all (water molecules); each group's terms are
  // evaluated once.  Every other atom with terms keeps its own term list,
  // partners renumbered to global user indices.
  std::vector<BGroup> bgroups;
  std::vector<int32_t> bf_atoms, bf_start;
  std::vector<BTerm> bf_terms;
  for (int r = 0; r < n_reps; ++r) {
    const vp_replica_desc &d = reps[r];
    const int32_t uoff = s->info_h[r].uoff;
    auto inside = [&](int i, int v) { return v >= i && v < i + 3; };
    auto closed = [&](int i) {  // every term of atoms i..i+2 lies among them
      if (i + 2 >= d.n_atoms) return false;
      for (int m = 0; m < 3; ++m)
        for (const BTerm &T : terms[(size_t)uoff + i + m])
          if (!inside(i, T.a) || (T.kind != 0 && !inside(i, T.b))) return false;
      return true;
    };
    for (int i = 0; i < d.n_atoms;) {
      if (closed(i)) {
        // the group's distinct terms (by their place in the description), in order
        std::vector<const BTerm *> tl;
        for (int m = 0; m < 3; ++m)
          for (const BTerm &T : terms[(size_t)uoff + i + m])
            if (std::none_of(tl.begin(), tl.end(), [&](const BTerm *x) { return x->order == T.order; }))
              tl.push_back(&T);
        std::sort(tl.begin(), tl.end(), [](const BTerm *x, const BTerm *y) { return x->order < y->order; });
        if (!tl.empty() && (int)tl.size() <= kGroupTerms) {
          BGroup G{};
          G.ga = uoff + i;
          for (int t = 0; t < kGroupTerms; ++t) {
            if (t < (int)tl.size()) {
              const int ord = tl[t]->order;
              if (ord < d.n_bonds) {  // bond i--j as the description names it
                G.code[t] = 0 | (d.bonds[2 * ord] - i) << 4 | (d.bonds[2 * ord + 1] - i) << 12;
              } else {  // angle i--c--j as the description names it
                const int q = ord - d.n_bonds;
                G.code[t] = 1 | (d.angles[3 * q] - i) << 4 | (d.angles[3 * q + 1] - i) << 8 |
                            (d.angles[3 * q + 2] - i) << 12;
              }
              G.k[t] = tl[t]->k;
              G.r0[t] = tl[t]->r0;
            } else {
              G.code[t] = 0 | 0 << 4 | 1 << 12;  // bond 0--1 with k = 0
            }
          }
          bgroups.push_back(G);
          i += 3;
          continue;
        }
      }
      const size_t u = (size_t)uoff + i;
      if (!terms[u].empty()) {
        bf_atoms.push_back((int32_t)u);
        bf_start.push_back((int32_t)bf_terms.size());
        for (BTerm T : terms[u]) {
          T.a += uoff;
          if (T.kind != 0) T.b += uoff;
          bf_terms.push_back(T);
        }
      }
      ++i;
    }
  }
  bf_start.push_back((int32_t)bf_terms.size());
  s->n_bgroups = (int32_t)bgroups.size();
  s->n_bf_atoms = (int32_t)bf_atoms.size();

  // ---------------- device allocations and uploads
  TRY(upload(s, &s->info, s->info_h));
  std::vector<RepState> st(n_reps);
  for (auto &x : st) {
    std::memset(&x, 0, sizeof(x));
    x.force_rebuild = 1;
  }
  TRY(upload(s, &s->state, st));
  TRY(upload(s, &s->tile_rep, tile_rep));
  TRY(upload(s, &s->tile_first, tile_first));
  TRY(upload(s, &s->type0, type0));
  TRY(upload(s, &s->types, types));
  TRY(upload(s, &s->integ0, integ0));
  TRY(upload(s, &s->igm0, igm0));
  TRY(upload(s, &s->mass0, mass0));
  TRY(upload(s, &s->bt_start, bt_start));
  TRY(upload(s, &s->bterms, bterms));
  TRY(upload(s, &s->bgroups, bgroups));
  TRY(upload(s, &s->bf_atoms, bf_atoms));
  TRY(upload(s, &s->bf_start, bf_start));
  TRY(upload(s, &s->bf_terms, bf_terms));
  TRY(upload(s, &s->ex_start, ex_start));
  TRY(upload(s, &s->ex_list, ex_list));
  TRY(upload(s, &s->role0, role0));
  TRY(upload(s, &s->cforce, cforce));
  TRY(upload(s, &s->xf, xf_h));
  if (o.contact_order) TRY(native_contacts(s, reps));
  TRY(dalloc(s, &s->rmsd, (size_t)n_reps));
  if (o.nst_out > 0) {
    s->out_cap = o.out_capacity > 0 ? o.out_capacity : 1024;
    TRY(dalloc(s, &s->records, (size_t)n_reps * s->out_cap * VP_REC_COUNT));
  }
  TRY(dalloc(s, &s->cmap, (size_t)std::max<int64_t>(1, cmap_total)));
  for (size_t m = 0; m < maps.size(); ++m) {
    const MapKey &k = maps[m];
    std::vector<float> xf(3 * (size_t)k.ns);
    for (int i = 0; i < 3 * k.ns; ++i) xf[i] = (float)k.xf[i];
    float *dxf = nullptr;
    TRY(dalloc(s, &dxf, xf.size()));
    HIPCHECK(hipMemcpy(dxf, xf.data(), sizeof(float) * xf.size(), hipMemcpyHostToDevice));
    launch_native_map(dxf, k.ns, k.sep, (float)k.r0, (float)k.rs, (float)k.rc, s->cmap + map_off[m], 0);
  }
  TRY(dalloc(s, &s->cskew, (size_t)std::max<int64_t>(1, skew_total)));
  for (size_t m = 0; m < maps.size(); ++m)
    launch_cv_skew(s->cmap + map_off[m], maps[m].ns, s->cskew + skew_off[m], 0);
  const size_t S = (size_t)s->n_slots;
  TRY(dalloc(s, &s->xq_t, S));
  TRY(dalloc(s, &s->vel_t, S));
  TRY(dalloc(s, &s->orig_t, S));
  TRY(dalloc(s, &s->wrap_t, S));
  TRY(dalloc(s, &s->cellid_t, S));
  TRY(dalloc(s, &s->zkey_t, S));
  TRY(dalloc(s, &s->fcell_t, S));
  TRY(dalloc(s, &s->bucket_t, S));
  TRY(dalloc(s, &s->bko_t, S));
  TRY(dalloc(s, &s->cellpos_t, S));
  TRY(dalloc(s, &s->cellx_t, S));
  TRY(dalloc(s, &s->celljw_t, S));
  TRY(dalloc(s, &s->inv_t, U));
  if (s->tangent) {
    TRY(dalloc(s, &s->tx_t, 2 * S));
    TRY(dalloc(s, &s->tv_t, 2 * S));
  }
  TRY(dalloc(s, &s->step, 1));
  HIPCHECK(hipMemset(s->step, 0, sizeof(long long)));
  TRY(alloc_work(s, s->traj, true));

  // ---------------- initial state, list, forces, S_0
  int32_t *dx = nullptr;
  float *dv = nullptr;
  uint8_t *dhv = nullptr;
  TRY(dalloc(s, &dx, xh.size()));
  TRY(dalloc(s, &dv, vh.size()));
  TRY(dalloc(s, &dhv, has_v.size()));
  HIPCHECK(hipMemcpy(dx, xh.data(), sizeof(int32_t) * xh.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dv, vh.data(), sizeof(float) * vh.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dhv, has_v.data(), has_v.size(), hipMemcpyHostToDevice));
  launch_init_state(s, dx, dv, dhv, 0);
  launch_rebuild(s, s->traj, 0, nullptr, 0);
  launch_forces(s, s->traj, 0);
  launch_cv(s, s->traj, 0, 0, s->tangent);
  launch_integrate(s, INT_INIT, 0);
  if (o.nst_out > 0) {  // the record of step 0
    launch_energies(s, s->traj, false, 0);
    launch_kinetic(s, s->traj.ke_tile, 0);
    launch_record(s, false, 0);
  }
  if (o.contact_order) launch_contact_form(s, 0);  // contacts formed in X_0
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipDeviceSynchronize());
  return VP_OK;
}

// ---------------- tile shapes per size bucket
static_assert(kNumForceShapes == VP_FORCE_SHAPES, "shape count of the ABI");

static void make_buckets(vp_system *s) {
  s->buckets.clear();
  for (int r = 0; r < s->R; ++r) {
    const RepInfo &R = s->info_h[r];
    const double rc = R.rc;
    int lg = 0;
    while ((2ll << lg) <= (long long)R.n) ++lg;
    vp_system::TileBucket *b = nullptr;
    for (auto &x : s->buckets)
      if (x.r_cut == rc && x.log2n == lg) b = &x;
    if (!b) {
      s->buckets.push_back({rc, lg, 0, {}, s->force_shape, {0.0}});
      b = &s->buckets.back();
    }
    b->nrep += 1;
    for (int k = 0; k < R.ntiles * (kTile / kBlk); ++k) b->blocks.push_back(R.blk0 + k);
  }
}

// The timed launches leave pair forces only in the trajectory's force arrays:
// recompute the full forces of the current state (the same values as before,
// whatever the tile shape).
static vp_status restore_forces(vp_system *s) {
  launch_forces(s, s->traj, 0);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipDeviceSynchronize());
  return VP_OK;
}

// Shortest of `reps` timed executions of the launches `plan`.
static vp_status time_plan(vp_system *s, const std::vector<vp_system::ForceLaunch> &plan, int reps,
                           double *ms) {
  hipEvent_t a, b;
  HIPCHECK(hipEventCreate(&a));
  HIPCHECK(hipEventCreate(&b));
  double best = 1e30;
  hipError_t e = hipSuccess;
  for (int k = 0; k < reps && e == hipSuccess; ++k) {
    e = hipEventRecord(a, 0);
    for (const auto &g : plan) launch_forces_shape(s, s->traj, g.shape, g.blist, g.nblk, 0);
    if (e == hipSuccess) e = hipEventRecord(b, 0);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (t < best) best = t;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fail(VP_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
  *ms = best;
  return VP_OK;
}

// The best launch time of each plan, the plans taken in turn over `rounds`
// rounds (one untimed launch of each first), so that a clock still settling
// favours none of them; before each timed launch a 256 MiB read evicts the
// last-level cache, as the other kernels of a step do between two force
// launches of a trajectory.
static vp_status time_plans(vp_system *s, const std::vector<std::vector<vp_system::ForceLaunch>> &plans,
                            int rounds, std::vector<double> &ms) {
  constexpr size_t kFlush = size_t(256) << 20;
  TmpBuf flush(s, kFlush), sink(s, sizeof(int));
  ms.assign(plans.size(), 1e30);
  for (const auto &plan : plans)
    for (const auto &g : plan) launch_forces_shape(s, s->traj, g.shape, g.blist, g.nblk, 0);
  for (int k = 0; k < rounds; ++k)
    for (size_t i = 0; i < plans.size(); ++i) {
      if (flush.p && sink.p) launch_touch(flush.p, kFlush, (int *)sink.p, 0);
      double t = 0.0;
      TRY(time_plan(s, plans[i], 1, &t));
      ms[i] = std::min(ms[i], t);
    }
  HIPCHECK(hipDeviceSynchronize());  // the temporary buffers are released on return
  return VP_OK;
}

// One force launch per shape that some bucket uses, over those buckets' blocks.
static vp_status split_plan(vp_system *s, std::vector<vp_system::ForceLaunch> &plan) {
  plan.clear();
  for (int k = 0; k < kNumForceShapes; ++k) {
    std::vector<int32_t> blocks;
    for (const auto &b : s->buckets)
      if (b.shape == k) blocks.insert(blocks.end(), b.blocks.begin(), b.blocks.end());
    if (blocks.empty()) continue;
    std::sort(blocks.begin(), blocks.end());
    int32_t *p = nullptr;
    TRY(upload(s, &p, blocks));
    plan.push_back({k, p, (int)blocks.size()});
  }
  return VP_OK;
}

// Times every shape on every bucket's blocks, groups the buckets by their
// fastest shape into one launch per shape, and keeps that split plan only if it
// beats the fastest single shape over all blocks.  The forces do not depend on
// the shape, so the choice affects time only.
static vp_status autotune(vp_system *s) {
  constexpr int kReps = 5;
  std::vector<const int32_t *> dev(s->buckets.size());
  for (size_t i = 0; i < s->buckets.size(); ++i) {
    auto &b = s->buckets[i];
    int32_t *p = nullptr;
    TRY(upload(s, &p, b.blocks));
    dev[i] = p;
    std::vector<std::vector<vp_system::ForceLaunch>> plans;
    for (int k = 0; k < kNumForceShapes; ++k) plans.push_back({{k, p, (int)b.blocks.size()}});
    std::vector<double> t;
    TRY(time_plans(s, plans, kReps, t));
    int best = 0;
    for (int k = 0; k < kNumForceShapes; ++k) {
      b.ms[k] = t[k];
      if (t[k] < t[best]) best = k;
    }
    b.shape = best;
  }
  std::vector<vp_system::ForceLaunch> split;
  TRY(split_plan(s, split));
  if (split.size() == 1) {  // one shape everywhere: a plain launch over all blocks
    s->force_shape = split[0].shape;
    s->force_plan.clear();
    s->plan_split = false;
    return restore_forces(s);
  }
  std::vector<std::vector<vp_system::ForceLaunch>> plans{split};
  for (int k = 0; k < kNumForceShapes; ++k) plans.push_back({{k, nullptr, s->n_blocks}});
  std::vector<double> t;
  TRY(time_plans(s, plans, kReps, t));
  const double t_split = t[0];
  double t_one = 1e30;
  int one = 0;
  for (int k = 0; k < kNumForceShapes; ++k)
    if (t[1 + k] < t_one) {
      t_one = t[1 + k];
      one = k;
    }
  if (t_split < t_one) {
    s->force_plan = split;
    s->plan_split = true;
  } else {
    s->force_shape = one;
    s->force_plan.clear();
    s->plan_split = false;
    for (auto &b : s->buckets) b.shape = one;
  }
  return restore_forces(s);
}

extern "C" vp_status vp_debug_set_tiles(vp_system *s, const int32_t *shapes, int32_t n) {
  if (!s || !shapes) return fail(VP_ERR_ARG, "NULL argument");
  if (n != (int32_t)s->buckets.size()) return fail(VP_ERR_ARG, "one shape per size bucket expected");
  for (int i = 0; i < n; ++i)
    if (shapes[i] < 0 || shapes[i] >= kNumForceShapes) return fail(VP_ERR_ARG, "unknown force shape");
  HIPCHECK(hipDeviceSynchronize());
  for (auto &g : s->graphs) (void)hipGraphExecDestroy(g.exec);  // they hold the old launches
  s->graphs.clear();
  for (int i = 0; i < n; ++i) s->buckets[i].shape = shapes[i];
  TRY(split_plan(s, s->force_plan));
  s->plan_split = true;
  return VP_OK;
}

extern "C" vp_status vp_tile_buckets(vp_system *s, vp_tile_bucket *out, int32_t cap,
                                     int32_t *n_buckets, int32_t *split) {
  if (!s || !n_buckets || cap < 0 || (cap > 0 && !out)) return fail(VP_ERR_ARG, "invalid argument");
  *n_buckets = (int32_t)s->buckets.size();
  if (split) *split = s->plan_split ? 1 : 0;
  for (int i = 0; i < (int)s->buckets.size() && i < cap; ++i) {
    const auto &b = s->buckets[i];
    vp_tile_bucket &o = out[i];
    o.r_cut = b.r_cut;
    o.log2_atoms = b.log2n;
    o.n_replicas = b.nrep;
    o.n_blocks = (int32_t)b.blocks.size();
    o.shape = b.shape;
    o.waves = kForceShapes[b.shape].parts;
    o.entries = kForceShapes[b.shape].unroll;
    for (int k = 0; k < kNumForceShapes; ++k) o.ms[k] = b.ms[k];
  }
  return VP_OK;
}

extern "C" vp_status vp_system_create(const vp_replica_desc *reps, int32_t n_reps,
                                      const vp_options *opt, vp_system **out) {
  if (!out) return fail(VP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!reps) return fail(VP_ERR_ARG, "reps is NULL");
  if (n_reps <= 0) return fail(VP_ERR_ARG, "n_reps must be positive");
  int64_t total = 0;
  for (int r = 0; r < n_reps; ++r) {
    vp_status st = validate(reps[r], r, opt && opt->tangent != 0);
    if (st != VP_OK) return st;
    total += reps[r].n_atoms;
  }
  if (total > ((int64_t)1 << 31) - (int64_t)kTile * n_reps) return fail(VP_ERR_ARG, "batch too large");
  if (opt && (opt->force_shape < 0 || opt->force_shape >= kNumForceShapes))
    return fail(VP_ERR_ARG, "unknown force_shape");
  if (opt && (opt->nst_out < 0 || opt->out_capacity < 0 || opt->stage_cap < 0))
    return fail(VP_ERR_ARG, "nst_out, out_capacity and stage_cap must be >= 0");
  if (opt && ((opt->dev_alloc == nullptr) != (opt->dev_free == nullptr)))
    return fail(VP_ERR_ARG, "dev_alloc and dev_free go together");
  vp_system *s = new (std::nothrow) vp_system();
  if (!s) return fail(VP_ERR_NOMEM, "host allocation failed");
  vp_options o{};
  if (opt) o = *opt;
  if (o.steps_per_graph <= 0) o.steps_per_graph = 20;
  if (!opt) o.use_graph = 1;
  s->opt = o;
  s->tangent = o.tangent != 0;
  s->force_shape = o.force_shape;
  if (hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
    delete s;
    return fail(VP_ERR_HIP, "hipEventCreate failed");
  }
  vp_status st = build(s, reps, n_reps);
  // List capacity: sized from the mean density, then checked against the
  // first build; a replica whose longest list uses more than 80% of it (local
  // density well above the mean) is built again with 1.3x that length.
  for (int attempt = 0; st == VP_OK && o.max_neighbors <= 0 && attempt < 3; ++attempt) {
    std::vector<RepState> rs(n_reps);
    if (hipMemcpy(rs.data(), s->state, sizeof(RepState) * n_reps, hipMemcpyDeviceToHost) != hipSuccess) {
      st = fail(VP_ERR_HIP, "reading the first list build");
      break;
    }
    std::vector<int32_t> grow(n_reps, 0);
    bool any = false;
    for (int r = 0; r < n_reps; ++r)
      if (rs[r].list_max > (int)(0.8 * s->info_h[r].maxnb)) {
        grow[r] = ((int)std::ceil(1.3 * rs[r].list_max) + 16 + 7) / 8 * 8;
        any = true;
      }
    if (!any) break;
    std::vector<int32_t> keep = s->maxnb_override;
    keep.resize(n_reps, 0);
    for (int r = 0; r < n_reps; ++r)
      if (grow[r] > 0) keep[r] = std::max(keep[r], grow[r]);
    free_all(s);
    s->graphs.clear();
    s->eval_ready = false;
    s->traj = Work{};
    s->eval = Work{};
    s->maxnb_override = keep;
    st = build(s, reps, n_reps);
  }
  if (st == VP_OK) {
    make_buckets(s);
    if (o.autotune) st = autotune(s);
  }
  if (st != VP_OK) {
    std::string msg = g_err;
    (void)hipDeviceSynchronize();
    free_all(s);
    (void)hipEventDestroy(s->done);
    delete s;
    g_err = msg;
    return st;
  }
  *out = s;
  return VP_OK;
}

extern "C" vp_status vp_system_destroy(vp_system *s) {
  if (!s) return VP_OK;
  (void)hipDeviceSynchronize();
  free_all(s);
  (void)hipEventDestroy(s->done);
  delete s;
  return VP_OK;
}

// one block of steps: START ... FINISH, with FINISH|START fused inside; with
// energy records, the gated energy kernels after the forces of every step and
// the gated record kernel after every FINISH
static void enqueue_block(vp_system *s, int steps, hipStream_t st) {
  const bool timing = s->timing;
  const bool rec = s->opt.nst_out > 0;
  for (int k = 0; k < steps; ++k) {
    launch_integrate(s, k == 0 ? INT_START : (INT_FINISH | INT_START), st);
    if (rec && k > 0) launch_record(s, true, st);
    launch_rebuild(s, s->traj, 0, nullptr, st);
    if (timing) (void)hipEventRecord(s->ev_before[k], st);
    launch_pair_forces(s, s->traj, st);
    if (timing) (void)hipEventRecord(s->ev_after[k], st);
    launch_bonded(s, s->traj, st);
    if (rec) launch_energies(s, s->traj, true, st);
    if (s->tangent) launch_tangent_forces(s, s->traj, st);
    launch_cv(s, s->traj, 1, st, s->tangent);
    if (s->opt.contact_order) launch_contact_form(s, st);
  }
  launch_integrate(s, INT_FINISH, st);
  if (rec) launch_record(s, true, st);
}

static vp_status collect_timing(vp_system *s, int steps) {
  HIPCHECK(hipEventSynchronize(s->ev_after[steps - 1]));
  for (int k = 0; k < steps; ++k) {
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, s->ev_before[k], s->ev_after[k]));
    s->timing_ms += ms;
    s->timing_count += 1;
  }
  return VP_OK;
}

static vp_status graph_for(vp_system *s, int steps, hipGraphExec_t *exec) {
  for (auto &g : s->graphs)
    if (g.steps == steps) {
      *exec = g.exec;
      return VP_OK;
    }
  hipStream_t cs;
  HIPCHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph;
  HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  enqueue_block(s, steps, cs);
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(VP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  hipGraphExec_t ex;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return fail(VP_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  s->graphs.push_back({steps, nullptr, ex});
  *exec = ex;
  return VP_OK;
}

extern "C" vp_status vp_step_batch(vp_system *s, int32_t n_steps, void *hip_stream) {
  if (!s) return fail(VP_ERR_ARG, "system is NULL");
  if (n_steps < 0) return fail(VP_ERR_ARG, "n_steps must be >= 0");
  hipStream_t st = (hipStream_t)hip_stream;
  if (n_steps == 0) return VP_OK;
  HIPCHECK(begin_async(s, st));
  const int B = s->opt.steps_per_graph;
  int left = n_steps;
  while (left > 0) {
    int k = std::min(left, B);
    if (s->opt.use_graph && !s->timing) {
      hipGraphExec_t ex;
      TRY(graph_for(s, k, &ex));
      HIPCHECK(hipGraphLaunch(ex, st));
    } else {
      enqueue_block(s, k, st);
      HIPCHECK(hipGetLastError());
    }
    if (s->timing) TRY(collect_timing(s, k));
    left -= k;
  }
  s->host_step += n_steps;
  HIPCHECK(end_async(s, st));
  return VP_OK;
}

static vp_status fetch_state(vp_system *s, std::vector<RepState> &st) {
  HIPCHECK(sync_system(s));
  HIPCHECK(hipGetLastError());
  st.resize(s->R);
  HIPCHECK(hipMemcpy(st.data(), s->state, sizeof(RepState) * s->R, hipMemcpyDeviceToHost));
  return VP_OK;
}

// RMSD of every replica from its X_f (NaN without one); after fetch_state.
static vp_status fetch_rmsd(vp_system *s, std::vector<double> &rmsd) {
  launch_rmsd(s, 0);
  HIPCHECK(hipGetLastError());
  rmsd.resize(s->R);
  HIPCHECK(hipMemcpy(rmsd.data(), s->rmsd, sizeof(double) * s->R, hipMemcpyDeviceToHost));
  return VP_OK;
}

// A flagged replica (unstable, or a pair list that overflowed) has no finite functional.
static double phi_of(const RepInfo &R, const RepState &S) {
  if (S.status) return INFINITY;
  return (S.phi_acc - 0.5 * S.s_last) * R.dt / (4.0 * R.kT);
}

// The product criterion of vp_select_path.
static bool reached_of(const RepInfo &R, const RepState &S, double rmsd) {
  if (S.status) return false;
  if (!(std::fabs(S.z_last - R.z_target) <= R.reach_tol)) return false;
  if (std::isfinite(R.reach_rmsd) && !(rmsd <= R.reach_rmsd)) return false;
  return true;
}

extern "C" vp_status vp_functional(vp_system *s, double *phi_host, double *dphi_dtheta_host) {
  if (!s || !phi_host) return fail(VP_ERR_ARG, "NULL argument");
  if (dphi_dtheta_host && !s->tangent)
    return fail(VP_ERR_STATE, "the functional gradient needs derivatives enabled at creation (vp_options.tangent)");
  std::vector<RepState> st;
  TRY(fetch_state(s, st));
  for (int r = 0; r < s->R; ++r) {
    const RepInfo &R = s->info_h[r];
    phi_host[r] = phi_of(R, st[r]);
    if (dphi_dtheta_host)
      for (int d = 0; d < 2; ++d)
        dphi_dtheta_host[2 * r + d] = st[r].status
                                          ? NAN
                                          : (st[r].pd_acc[d] - 0.5 * st[r].pd_last[d]) * R.dt / (4.0 * R.kT);
  }
  return VP_OK;
}

extern "C" vp_status vp_debug_trajectory_state(vp_system *s, double *x_host, double *v_host,
                                               double *xt_host, double *vt_host, double *pd_host) {
  if (!s || !x_host || !v_host) return fail(VP_ERR_ARG, "NULL argument");
  if ((xt_host || vt_host || pd_host) && !s->tangent)
    return fail(VP_ERR_STATE, "derivatives were not enabled at creation (vp_options.tangent)");
  if ((xt_host == nullptr) != (vt_host == nullptr)) return fail(VP_ERR_ARG, "xt and vt go together");
  HIPCHECK(sync_system(s));
  const size_t n3 = 3 * (size_t)s->n_users;
  TmpBuf buf(s, sizeof(double) * n3 * 6);
  if (!buf.p) return fail(VP_ERR_NOMEM, "device allocation failed");
  double *d = (double *)buf.p;
  launch_export_state(s, d, d + n3, xt_host ? d + 2 * n3 : nullptr, xt_host ? d + 4 * n3 : nullptr, 0);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(x_host, d, sizeof(double) * n3, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(v_host, d + n3, sizeof(double) * n3, hipMemcpyDeviceToHost);
  if (e == hipSuccess && xt_host) e = hipMemcpy(xt_host, d + 2 * n3, sizeof(double) * 2 * n3, hipMemcpyDeviceToHost);
  if (e == hipSuccess && vt_host) e = hipMemcpy(vt_host, d + 4 * n3, sizeof(double) * 2 * n3, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(VP_ERR_HIP, hipGetErrorString(e));
  if (pd_host) {
    std::vector<RepState> st;
    TRY(fetch_state(s, st));
    for (int r = 0; r < s->R; ++r)
      for (int k = 0; k < 2; ++k) {
        pd_host[4 * r + k] = st[r].pd_acc[k];
        pd_host[4 * r + 2 + k] = st[r].pd_last[k];
      }
  }
  return VP_OK;
}

extern "C" vp_status vp_debug_force_dir(vp_system *s, const float *x_dev, const float *dx_dev,
                                        float *out_dev, double t, void *hip_stream) {
  if (!s || !x_dev || !dx_dev || !out_dev) return fail(VP_ERR_ARG, "NULL argument");
  if (!s->tangent) return fail(VP_ERR_STATE, "derivatives were not enabled at creation (vp_options.tangent)");
  hipStream_t st = (hipStream_t)hip_stream;
  if (!s->eval_ready) {
    HIPCHECK(hipDeviceSynchronize());
    TRY(alloc_work(s, s->eval, false));
    s->eval_ready = true;
  }
  HIPCHECK(begin_async(s, st));
  launch_rebuild(s, s->eval, 1, x_dev, st);
  launch_forces(s, s->eval, st);
  launch_cv(s, s->eval, 0, st, false);
  launch_force_dir(s, s->eval, dx_dev, t, out_dev, st);
  HIPCHECK(hipGetLastError());
  HIPCHECK(end_async(s, st));
  return VP_OK;
}

extern "C" vp_status vp_select_path(vp_system *s, const uint8_t *eligible, int32_t *best,
                                    double *best_phi) {
  if (!s || !best || !best_phi) return fail(VP_ERR_ARG, "NULL argument");
  *best = -1;
  *best_phi = INFINITY;
  std::vector<RepState> st;
  TRY(fetch_state(s, st));
  std::vector<double> rmsd;
  TRY(fetch_rmsd(s, rmsd));
  for (int r = 0; r < s->R; ++r) {
    const RepInfo &R = s->info_h[r];
    double phi = phi_of(R, st[r]);
    if (!reached_of(R, st[r], rmsd[r]) || (eligible && !eligible[r]) || !std::isfinite(phi)) continue;
    if (*best < 0 || phi < *best_phi) {
      *best = r;
      *best_phi = phi;
    }
  }
  if (*best < 0) return fail(VP_ERR_NOPATH, "no replica reached the product with a finite functional");
  return VP_OK;
}

namespace vp {

vp_status set_error(vp_status st, const std::string &msg) { return fail(st, msg); }

// The evaluation of vp_forces into the buffers of W (an evaluation context
// that the call's kernels fill before they read it), ordered after the
// system's previous calls.
vp_status enqueue_forces(vp_system *s, Work &W, const float *x_dev, float *f_dev, double *energy_dev,
                         double t, hipStream_t st) {
  HIPCHECK(begin_async(s, st));
  launch_rebuild(s, W, 1, x_dev, st);
  launch_forces(s, W, st);
  if (energy_dev) launch_energies(s, W, false, st);
  launch_cv(s, W, 0, st, false);
  launch_force_out(s, W, t, f_dev, energy_dev, st);
  HIPCHECK(hipGetLastError());
  HIPCHECK(end_async(s, st));
  return VP_OK;
}

}  // namespace vp

extern "C" vp_status vp_forces(vp_system *s, const float *x_dev, float *f_dev, double *energy_dev,
                               double t, void *hip_stream) {
  if (!s || !x_dev || !f_dev) return fail(VP_ERR_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  if (!s->eval_ready) {
    HIPCHECK(sync_system(s));
    TRY(alloc_work(s, s->eval, false));
    s->eval_ready = true;
  }
  return enqueue_forces(s, s->eval, x_dev, f_dev, energy_dev, t, st);
}

extern "C" vp_status vp_get_state(vp_system *s, float *x_dev, float *v_dev, void *hip_stream) {
  if (!s) return fail(VP_ERR_ARG, "NULL system");
  hipStream_t st = (hipStream_t)hip_stream;
  HIPCHECK(begin_async(s, st));
  launch_gather_state(s, x_dev, v_dev, st);
  HIPCHECK(hipGetLastError());
  HIPCHECK(end_async(s, st));
  return VP_OK;
}

extern "C" vp_status vp_observables(vp_system *s, double *obs) {
  if (!s || !obs) return fail(VP_ERR_ARG, "NULL argument");
  std::vector<RepState> st;
  TRY(fetch_state(s, st));
  long long step = 0;
  HIPCHECK(hipMemcpy(&step, s->step, sizeof(step), hipMemcpyDeviceToHost));
  std::vector<double> rmsd;
  TRY(fetch_rmsd(s, rmsd));
  std::vector<int32_t> eflags(s->R, 0);
  if (s->eval_ready)
    HIPCHECK(hipMemcpy(eflags.data(), s->eval.flags, sizeof(int32_t) * s->R, hipMemcpyDeviceToHost));
  TmpBuf kebuf(s, sizeof(double) * (size_t)s->n_tiles);
  if (!kebuf.p) return fail(VP_ERR_NOMEM, "device allocation failed");
  double *ke = (double *)kebuf.p;
  launch_kinetic(s, ke, 0);
  std::vector<double> keh(s->n_tiles);
  hipError_t e = hipMemcpy(keh.data(), ke, sizeof(double) * keh.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(VP_ERR_HIP, hipGetErrorString(e));
  for (int r = 0; r < s->R; ++r) {
    const RepInfo &R = s->info_h[r];
    double k = 0.0;
    for (int t = R.tile0; t < R.tile0 + R.ntiles; ++t) k += keh[t];
    double *o = obs + (size_t)r * VP_OBS_COUNT;
    o[VP_OBS_STEP] = (double)step;
    o[VP_OBS_Z] = st[r].z_last;
    o[VP_OBS_ZREF] = st[r].zref_last;
    o[VP_OBS_ZMIN] = st[r].z_m;
    o[VP_OBS_PHI] = phi_of(R, st[r]);
    o[VP_OBS_STATUS] = st[r].status;
    o[VP_OBS_REBUILDS] = st[r].rebuilds;
    o[VP_OBS_KE] = k;
    o[VP_OBS_STAGE_MAX] = st[r].stage_max;
    o[VP_OBS_STAGE_CAP] = R.stage_cap;
    o[VP_OBS_LIST_MAX] = st[r].list_max;
    o[VP_OBS_LIST_CAP] = R.maxnb;
    o[VP_OBS_EXACT_BUILDS] = st[r].exact_builds;
    o[VP_OBS_SKIN] = R.skin;
    o[VP_OBS_NSTLIST] = R.nstlist;
    o[VP_OBS_RMSD] = rmsd[r];
    o[VP_OBS_REACHED] = reached_of(R, st[r], rmsd[r]) ? 1.0 : 0.0;
    o[VP_OBS_EVAL_STATUS] = (eflags[r] & VP_REPLICA_LIST_OVERFLOW) ? (double)VP_REPLICA_LIST_OVERFLOW : 0.0;
  }
  return VP_OK;
}

extern "C" vp_status vp_energy_records(vp_system *s, double *out_host, int32_t cap, int32_t *n_records) {
  if (!s || !n_records || cap < 0) return fail(VP_ERR_ARG, "invalid argument");
  if (s->opt.nst_out <= 0) return fail(VP_ERR_STATE, "the system records no energies (vp_options.nst_out = 0)");
  std::vector<RepState> st;
  TRY(fetch_state(s, st));
  const int written = st[0].n_records;  // the same in every replica
  const int held = std::min(written, s->out_cap);
  *n_records = held;
  if (!out_host || cap == 0 || held == 0) return VP_OK;
  std::vector<double> all((size_t)s->R * s->out_cap * VP_REC_COUNT);
  HIPCHECK(hipMemcpy(all.data(), s->records, sizeof(double) * all.size(), hipMemcpyDeviceToHost));
  const int take = std::min(cap, held);
  for (int r = 0; r < s->R; ++r)
    for (int k = 0; k < take; ++k) {
      // oldest held record first: index written - held + k in the ring
      const int slot = (written - held + k) % s->out_cap;
      std::memcpy(out_host + ((size_t)r * take + k) * VP_REC_COUNT,
                  &all[((size_t)r * s->out_cap + slot) * VP_REC_COUNT], sizeof(double) * VP_REC_COUNT);
    }
  return VP_OK;
}

extern "C" vp_status vp_contact_order(vp_system *s, int32_t rep, int32_t *pairs_host, int64_t *steps_host,
                                      int32_t cap, int32_t *n_contacts) {
  if (!s || !n_contacts || cap < 0) return fail(VP_ERR_ARG, "invalid argument");
  if (rep < 0 || rep >= s->R) return fail(VP_ERR_ARG, "replica index out of range");
  if (!s->opt.contact_order) return fail(VP_ERR_STATE, "contact order was not enabled at creation (vp_options.contact_order)");
  const RepInfo &R = s->info_h[rep];
  *n_contacts = R.n_contacts;
  const int take = std::min(cap, R.n_contacts);
  if (take == 0) return VP_OK;
  HIPCHECK(sync_system(s));
  if (pairs_host)
    HIPCHECK(hipMemcpy(pairs_host, s->cpairs + R.cp_off, sizeof(int2) * (size_t)take, hipMemcpyDeviceToHost));
  if (steps_host) {
    std::vector<int32_t> t(take);
    HIPCHECK(hipMemcpy(t.data(), s->t_form + R.tf_off, sizeof(int32_t) * (size_t)take, hipMemcpyDeviceToHost));
    for (int k = 0; k < take; ++k) steps_host[k] = t[k];
  }
  return VP_OK;
}

extern "C" vp_status vp_path_similarity(vp_system *s, double *sim_host) {
  if (!s || !sim_host) return fail(VP_ERR_ARG, "NULL argument");
  if (!s->opt.contact_order) return fail(VP_ERR_STATE, "contact order was not enabled at creation (vp_options.contact_order)");
  const int R = s->R;
  std::vector<int2> pr;
  for (int a = 0; a < R; ++a)
    for (int b = a + 1; b < R; ++b) {
      const RepInfo &A = s->info_h[a], &B = s->info_h[b];
      if (A.n_contacts >= 2 && A.cp_off == B.cp_off && A.n_contacts == B.n_contacts) pr.push_back(make_int2(a, b));
    }
  for (int a = 0; a < R; ++a)
    for (int b = 0; b < R; ++b) sim_host[(size_t)a * R + b] = (a == b && s->info_h[a].n_contacts >= 2) ? 1.0 : NAN;
  if (pr.empty()) return VP_OK;
  if ((size_t)s->max_contacts * 2 * sizeof(int32_t) > 160 * 1024)
    return fail(VP_ERR_ARG, "too many native contacts for the similarity kernel's LDS (at most 20480)");
  HIPCHECK(sync_system(s));
  HIPCHECK(prepare_similarity(s->max_contacts));
  TmpBuf pbuf(s, sizeof(int2) * pr.size()), cbuf(s, sizeof(unsigned long long) * pr.size());
  if (!pbuf.p || !cbuf.p) return fail(VP_ERR_NOMEM, "device allocation failed");
  HIPCHECK(hipMemcpy(pbuf.p, pr.data(), sizeof(int2) * pr.size(), hipMemcpyHostToDevice));
  launch_similarity(s, (const int2 *)pbuf.p, (int)pr.size(), s->max_contacts, (unsigned long long *)cbuf.p, 0);
  HIPCHECK(hipGetLastError());
  std::vector<unsigned long long> same(pr.size());
  HIPCHECK(hipMemcpy(same.data(), cbuf.p, sizeof(unsigned long long) * same.size(), hipMemcpyDeviceToHost));
  for (size_t q = 0; q < pr.size(); ++q) {
    const double nc = (double)s->info_h[pr[q].x].n_contacts;
    const double v = (double)same[q] / (nc * (nc - 1.0));
    sim_host[(size_t)pr[q].x * R + pr[q].y] = v;
    sim_host[(size_t)pr[q].y * R + pr[q].x] = v;
  }
  return VP_OK;
}

extern "C" vp_status vp_toy_trials(const vp_toy_params *p, int32_t n_trials, const int32_t *kind_dev,
                                   const double *k_dev, const uint64_t *seed_dev, double *out_dev,
                                   float *path_dev, void *hip_stream) {
  if (!p || !kind_dev || !k_dev || !seed_dev || !out_dev) return fail(VP_ERR_ARG, "NULL argument");
  if (n_trials <= 0) return fail(VP_ERR_ARG, "n_trials must be positive");
  if (p->n_steps < 0) return fail(VP_ERR_ARG, "n_steps must be >= 0");
  if (!(p->mass > 0) || !(p->dt > 0) || !(p->kT > 0) || !(p->gamma >= 0))
    return fail(VP_ERR_ARG, "mass, dt and kT must be positive and gamma non-negative");
  if (path_dev && p->path_stride <= 0) return fail(VP_ERR_ARG, "a path buffer needs path_stride > 0");
  launch_toy(*p, n_trials, kind_dev, k_dev, seed_dev, out_dev, path_dev, (hipStream_t)hip_stream);
  HIPCHECK(hipGetLastError());
  return VP_OK;
}

extern "C" vp_status vp_toy_select(const double *out_host, int32_t n, const uint8_t *eligible, int32_t *best,
                                   double *best_phi) {
  if (!out_host || !best || !best_phi || n < 0) return fail(VP_ERR_ARG, "invalid argument");
  *best = -1;
  *best_phi = INFINITY;
  for (int r = 0; r < n; ++r) {
    const double *o = out_host + (size_t)r * VP_TOY_COUNT;
    if (!(o[VP_TOY_REACHED] != 0.0) || (eligible && !eligible[r]) || !std::isfinite(o[VP_TOY_PHI])) continue;
    if (*best < 0 || o[VP_TOY_PHI] < *best_phi) {
      *best = r;
      *best_phi = o[VP_TOY_PHI];
    }
  }
  if (*best < 0) return fail(VP_ERR_NOPATH, "no toy trial reached the product with a finite functional");
  return VP_OK;
}

extern "C" vp_status vp_device_bytes(const vp_system *s, int64_t *bytes) {
  if (!s || !bytes) return fail(VP_ERR_ARG, "NULL argument");
  *bytes = s->device_bytes;
  return VP_OK;
}

extern "C" vp_status vp_set_timing(vp_system *s, int32_t on) {
  if (!s) return fail(VP_ERR_ARG, "NULL system");
  while (on && (int)s->ev_before.size() < s->opt.steps_per_graph) {
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    s->ev_before.push_back(a);
    s->ev_after.push_back(b);
  }
  s->timing = on != 0;
  return VP_OK;
}

extern "C" vp_status vp_kernel_timing(vp_system *s, double *avg_ms, int64_t *count, int32_t reset) {
  if (!s) return fail(VP_ERR_ARG, "NULL system");
  if (avg_ms) *avg_ms = s->timing_count ? s->timing_ms / (double)s->timing_count : 0.0;
  if (count) *count = s->timing_count;
  if (reset) {
    s->timing_ms = 0.0;
    s->timing_count = 0;
  }
  return VP_OK;
}

extern "C" vp_status vp_pair_count(vp_system *s, int32_t rep, int64_t *count) {
  return vp_debug_pairs(s, rep, nullptr, 0, count);
}

extern "C" vp_status vp_sizes(const vp_system *s, int64_t *n_atoms_total, int32_t *n_reps) {
  if (!s) return fail(VP_ERR_ARG, "NULL system");
  if (n_atoms_total) *n_atoms_total = s->n_users;
  if (n_reps) *n_reps = s->R;
  return VP_OK;
}

extern "C" vp_status vp_debug_pairs(vp_system *s, int32_t rep, int32_t *pairs_host, int64_t cap,
                                    int64_t *count) {
  if (!s || !count || (cap > 0 && !pairs_host)) return fail(VP_ERR_ARG, "NULL argument");
  if (rep < 0 || rep >= s->R) return fail(VP_ERR_ARG, "replica index out of range");
  HIPCHECK(sync_system(s));
  TmpBuf dbuf(s, sizeof(int2) * (size_t)std::max<int64_t>(1, cap));
  TmpBuf cbuf(s, sizeof(unsigned long long));
  if (!dbuf.p || !cbuf.p) return fail(VP_ERR_NOMEM, "device allocation failed");
  int2 *d = (int2 *)dbuf.p;
  unsigned long long *cnt = (unsigned long long *)cbuf.p;
  HIPCHECK(hipMemset(cnt, 0, sizeof(unsigned long long)));
  launch_debug_pairs(s, s->traj, rep, d, (unsigned long long)cap, cnt, 0);
  unsigned long long c = 0;
  hipError_t e = hipMemcpy(&c, cnt, sizeof(c), hipMemcpyDeviceToHost);
  if (e == hipSuccess && cap > 0)
    e = hipMemcpy(pairs_host, d, sizeof(int2) * (size_t)std::min<int64_t>(cap, (int64_t)c),
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(VP_ERR_HIP, hipGetErrorString(e));
  *count = (int64_t)c;
  return VP_OK;
}

extern "C" vp_status vp_debug_noise(uint64_t seed, uint32_t atom0, uint32_t step, uint32_t tag,
                                    int32_t n, float *out_dev, void *hip_stream) {
  if (!out_dev || n < 0) return fail(VP_ERR_ARG, "bad argument");
  if (n == 0) return VP_OK;
  launch_debug_noise(seed, atom0, step, tag, n, out_dev, (hipStream_t)hip_stream);
  HIPCHECK(hipGetLastError());
  return VP_OK;
}

extern "C" const char *vp_last_error(void) { return g_err.c_str(); }
