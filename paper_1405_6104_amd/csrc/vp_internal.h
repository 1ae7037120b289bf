// Internal declarations of the vp library (gfx950).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/vp.h"

namespace vp {

constexpr int kBlock = 256;          // threads per workgroup of the per-atom kernels
constexpr int kTile = 256;           // slots per tile (a tile never crosses replicas)
constexpr int kBlk = 64;             // atoms per neighbourhood block (one wave)
// Pair lists of a block: entry k of lane l is element k % 8 of row k / 8 of
// that lane, a row being 16 bytes (eight 16-bit staging indices).  Row c of
// lane l is the uint4 at list_row(c, l): rows are grouped by kListGroup per
// lane, so that a lane's consecutive rows share one 64-byte segment (the
// list build stores each lane's rows at the lane's own pace, and a segment
// filled by one lane in a short time combines in the cache before it reaches
// memory), while row c of all 64 lanes is still one load instruction of the
// force kernel.  List capacities are multiples of 8 kListGroup entries.
constexpr int kListGroup = 4;
__host__ __device__ inline int64_t list_row(int c, int lane) {
  return ((int64_t)(c / kListGroup) * kBlk + lane) * kListGroup + (c % kListGroup);
}
// A lane's list is two streams of rows.  Partners with Lennard-Jones
// parameters (epsilon > 0) fill rows 0, 1, ... upward; the others (charge-only
// atoms such as hydrogens) fill rows rowcap - 1, rowcap - 2, ... downward.
// Chunk c of the list (its c-th row in evaluation order) is row c of the
// first stream for c < nlj, else the (c - nlj)-th row from the top.
__host__ __device__ inline int chunk_row(int c, int nlj, int rowcap) {
  return c < nlj ? c : rowcap - 1 - (c - nlj);
}
constexpr int kParts = 8;            // waves sharing one block in the force kernel
constexpr int kForceThreads = kParts * kBlk;
constexpr int kMaxForceParts = 16;   // largest number of waves per block among the force tile shapes
constexpr int kLogicalParts = 16;    // force partial sums per atom: list chunk c goes to c mod 16
constexpr int kNumForceShapes = 4;
struct ForceShape {
  int parts, unroll;  // waves per 64-atom block, list entries per batch of LDS reads
};
extern const ForceShape kForceShapes[kNumForceShapes];
constexpr int kBinThreads = 1024;    // workgroup of the binning kernel
constexpr int kMaxCells = 4096;      // cells per replica held in LDS by the binning kernel
constexpr int kMaxStage = 8191;      // staged neighbourhood atoms per block (16-bit list entries; LDS decides)
constexpr int kMaxLds = 81920;       // LDS bytes per force workgroup (two share a 160 KB CU)
constexpr int kMaxLdsTangent = 163840;  // LDS bytes per workgroup of the tangent force kernel
constexpr int kMaxCols = 256;        // xy columns per replica (sort order)
constexpr int kMaxTypes = 1024;      // (charge, sigma, epsilon) classes per replica
constexpr int kCvBlock = 256;        // workgroup of the single-workgroup CV kinds (Rg, constant)
constexpr int kCvTile = 64;          // solute rows (and columns) of one contact-map tile
constexpr int kMaxCvBlocks = 256;    // row tiles per replica => at most 16384 solute atoms
constexpr int kMaxSoluteLds = 4096;  // solute positions staged in LDS by the Rg kernel
constexpr double kFixScale = 4294967296.0;  // 2^32: fixed-point force unit
constexpr double kForceLimit = 1.0e6;       // kJ/mol/nm: above this a replica is unstable
constexpr double kCoulomb = 138.935458;
// 2^22: coordinate unit is 2^-22 nm.  A coordinate relative to a point within
// 4 nm (a block's staged neighbourhood around its centre) is an integer below
// 2^24 and so exact in FP32, and the difference of two such values is an
// exact FP32 subtraction.
constexpr double kQ = 4194304.0;
constexpr float kQf = 4194304.0f;
constexpr float kInvQf = 2.384185791015625e-7f;  // 2^-22
constexpr double kInvQ = 2.384185791015625e-7;
constexpr int kDummyCoord = 1 << 30;  // staged position of the list padding entry
// Staged places after a block's capacity that hold the inert padding entry:
// three, so that padding read as a three-atom site stays inert.
constexpr int kStageDummies = 3;
// energy partials per 64-atom block: LJ, RF, bond, angle, pair virial [9],
// bonded virial [9] (each written by one kernel), two unused
constexpr int kEp = 24;
constexpr int kEpPairW = 4, kEpBondW = 13;

// Constant per-replica data (device copy in an array indexed by replica).
struct RepInfo {
  int32_t n, ns, npad, off;     // atoms, solute atoms, padded slots, first slot
  int32_t uoff;                 // first user-order index
  int32_t tile0, ntiles;        // tiles [tile0, tile0+ntiles)
  int32_t blk0;                 // first neighbourhood block
  int32_t bias, min_sep;
  int32_t nc[3], ncell, cell0;  // fine cell grid (candidate search) and offset into the cell arrays
  int32_t ncol[2];              // xy columns of the sort order
  int32_t nzb;                  // z slabs per column in the sort's buckets
  int32_t cedge[3][17];         // fine-cell edges floor(k Lq / nc), k = 0..nc
  int32_t Lq[3];                // box edges in coordinate units
  int32_t maxnb;                // per-atom list capacity (multiple of 8)
  int32_t stage_cap;            // staged atoms per block (<= kMaxStage)
  int32_t ntypes, type_off;     // type table (ntypes + 1 entries, last is inert)
  int32_t nlj_types;            // types [0, nlj_types) have epsilon > 0, the others none
  int64_t list_off;             // first element of this replica's list storage
  int64_t cmap_off;             // first element of the native contact map (FP32 [ns][ns])
  int64_t cskew_off;            // first element of its copy in tile-diagonal order (64 x 64 per tile)
  int32_t cv_blocks;            // contact map: row tiles (ceil(ns / 64)); other kinds: 1
  int64_t cvt_off;              // first entry of this replica's contact-map tile partials
  float cinv_r02, cinv_w;       // contact map: 1/r0^2, 1/(r_c - r_s) (nm)
  float crs2, crc2;             // r_s^2, r_c^2 (nm^2)
  int32_t sol_off;              // first index in per-solute arrays
  int32_t nstlist;              // lists are rebuilt when (step + 1) % nstlist == 0
  float rc2q, rl2q;             // (rc/q)^2 and (rl/q)^2 in FP32
  float krf2q;                  // 2 k_rf q^3 (RF term in coordinate units)
  float half_skin_margin;       // displacement (nm) that forces a rebuild
  double skin;                  // pair-list buffer (nm)
  float cr0, crs, crc;          // contact r0, switch start, switch end (nm)
  int32_t rlq;                  // list radius in coordinate units
  double Ld[3];
  double rc, krf, crf;
  double bias_k, ramp_rate, z_target;
  double kT, dt, reach_tol;
  double reach_rmsd;            // +inf: no RMSD criterion
  int32_t xf_off;               // first row of this replica's X_f in the FP64 copy, -1 without
  int32_t n_contacts;           // native contacts (contact order on), else 0
  int32_t cp_off;               // first pair of its native-contact list (shared by equal maps)
  int32_t tf_off;               // first entry of its formation steps
  int64_t r0q2;                 // (contact r0 in grid units)^2
  uint64_t seed;
};

// Mutable per-replica state (device).
struct RepState {
  double phi_acc;    // sum_n w_n S_n, w_0 = 1/2
  double s_last;     // S at the latest step
  double z0;         // z(X_0)
  double z_m;        // ratchet running minimum
  double z_last, zref_last;
  int64_t last_build;
  uint32_t maxdisp_bits;  // float bits of the largest displacement since the last build
  int32_t status;
  int32_t rebuild;        // 1 when this step rebuilds the pair list
  int32_t force_rebuild;
  int32_t rebuilds;
  int32_t stage_max;     // largest staged neighbourhood of a block so far
  int32_t list_max;      // longest per-atom list so far (entries needed, before any clamp)
  int32_t exact_builds;  // blocks built again in exact mode (staging capacity reached)
  int32_t n_records;     // energy records written
  // derivative of the functional with respect to (bias_k, ramp_rate)
  double pd_acc[2];   // sum_n w_n dS_n/dtheta, w_0 = 1/2
  double pd_last[2];  // dS/dtheta at the latest step
};

// One bonded contribution evaluated by the atom that owns it.
struct BTerm {
  int32_t kind;  // 0: bond to a; 1: angle end (vertex a, other end b); 2: angle vertex (ends a, b)
  int32_t a, b;
  int32_t order;  // host only: the term's place in the description (bonds, then angles)
  double k, r0;
};

// A bonded group: three consecutive atoms of a replica whose bonds and angles
// all lie among themselves (a water molecule), at most kGroupTerms of them,
// evaluated once by one thread.  Term t: code[t] = kind | i << 4 | c << 8 |
// j << 12 with local atom indices 0..2 (kind 0: bond i--j; kind 1: angle
// i--c--j, vertex c); unused terms are bonds 0--1 with k = 0.  Terms are in
// the description's order, so each atom sums its forces in the order its
// own term list holds them.
constexpr int kGroupTerms = 3;
struct alignas(16) BGroup {
  int32_t ga;                  // global user index of the first atom
  int32_t code[kGroupTerms];
  double k[kGroupTerms], r0[kGroupTerms];
};

// Device buffers of one evaluation context (trajectory or vp_forces).
struct Work {
  int4 *xq = nullptr;       // [slots] x, y, z (unwrapped, units of 2^-22 nm), type
  float4 *vel = nullptr;    // [slots] vx, vy, vz, 0
  float4 *integ = nullptr;  // [slots] 1/m, c1, sigma_v, 0
  int32_t *orig = nullptr;  // [slots] replica-local user index or -1
  int32_t *wrap = nullptr;  // [slots] periodic image of the atom at the last build (packed)
  int4 *xref = nullptr;     // [slots] positions at the last list build
  int32_t *inv = nullptr;   // [users] global slot of each atom
  long long *F = nullptr;   // [3][slots] fixed-point forces (without bias), SoA
  int64_t fstride = 0;      // slots: distance between the x, y and z planes of F
  int32_t *nbcnt = nullptr;     // [slots] list length (multiple of 8)
  int32_t *nblj = nullptr;      // [slots] rows of the list's first stream (LJ partners, chunk_row)
  uint16_t *nblist = nullptr;   // per block: maxnb/8 rows of 8 staged indices per lane, at list_row
  int32_t *stage_n = nullptr;   // [blocks]
  int4 *bctr = nullptr;         // [blocks] centre of the block's box at the last build (wrapped frame)
  uint32_t *stage = nullptr;    // [blocks][stage_stride] slot | image shifts
  int64_t stage_stride = 0;     // staging entries per block (largest capacity)
  int32_t *cell_start = nullptr;  // [sum ncell + R] fine-cell CSR offsets (replica-local)
  int32_t *cell_slots = nullptr;  // [slots] slots of each fine cell, ascending
  int32_t *cell_of = nullptr;     // [slots] fine cell of each new slot
  float4 *g = nullptr;            // [solute total] dz/dx (xyz) of each solute atom
  float4 *gtile = nullptr;        // contact map: dz/dx partials per (column tile, row tile, row)
  double *ztile = nullptr;        // contact map: z partials per (row tile, column tile)
  double *zpart = nullptr;        // [R][kMaxCvBlocks]
  double *gpart = nullptr;        // [R][kMaxCvBlocks] sum |g|^2/(gamma m)
  double *epart = nullptr;        // [blocks][kEp] energy and virial partials
  double *ke_tile = nullptr;      // [tiles] kinetic energy partials (energy records)
  int32_t *flags = nullptr;       // [R] rebuild flag for the eval context
  // tangents along (bias_k, ramp_rate) when derivatives are on: [2][slots]
  // (index p * fstride + slot), xyz used
  int64_t cvstride = 0;     // entries per direction of tgtile (cv tiles * 64)
  int64_t solstride = 0;    // entries per direction of tg (solute total)
  float4 *tx = nullptr;     // dx/dtheta_p
  float4 *tv = nullptr;     // dv/dtheta_p
  float4 *tf = nullptr;     // -H_U dx/dtheta_p (potential part of the tangent force)
  float4 *tg = nullptr;     // [2][solute total] (d grad z)[dx/dtheta_p]
  float4 *tgtile = nullptr; // [2][cv tiles * 64] partials of tg per column tile
  double *tzpart = nullptr; // [R][kMaxCvBlocks][2] parts of dz/dtheta_p = grad z . dx/dtheta_p
  double *tgpart = nullptr; // [R][kMaxCvBlocks][2] parts of sum_i 2 g_i . tg_i / (gamma_i m_i)
};

// packed periodic image (3 x 10-bit signed)
__host__ __device__ inline int32_t pack_wrap(int kx, int ky, int kz) {
  return ((kx & 1023)) | ((ky & 1023) << 10) | ((kz & 1023) << 20);
}
__host__ __device__ inline int unpack_wrap(int32_t w, int d) {
  int v = (w >> (10 * d)) & 1023;
  return v >= 512 ? v - 1024 : v;
}

}  // namespace vp

struct vp_system {
  int32_t R = 0;
  int64_t n_users = 0;   // sum of atoms
  int64_t n_slots = 0;   // sum of padded atoms
  int32_t n_tiles = 0;
  int32_t n_blocks = 0;
  int64_t n_cells = 0;
  int64_t list_elems = 0;
  int64_t n_solute_total = 0;
  int64_t n_cv_tiles = 0;  // sum over contact-map replicas of (row tiles)^2
  int32_t stage_cap_max = 0, ntypes_max = 0;
  vp_options opt{};
  std::vector<vp::RepInfo> info_h;
  vp::RepInfo *info = nullptr;    // device
  vp::RepState *state = nullptr;  // device
  int32_t *tile_rep = nullptr;    // [tiles] replica of each tile
  int32_t *tile_first = nullptr;  // [tiles] first slot of each tile
  // constant per-atom data in user order
  int32_t *type0 = nullptr;  // [users] type of each atom
  float4 *types = nullptr;   // type tables: (q sqrt(f) 2^33, sigma/2 2^22, sqrt(24 eps) 2^22, 0)
  float4 *integ0 = nullptr;  // [users]
  double *igm0 = nullptr;    // [users] 1/(gamma m) (solute entries used)
  double *mass0 = nullptr;   // [users] masses
  int32_t *bt_start = nullptr;  // [users + 1]
  vp::BTerm *bterms = nullptr;  // partners as replica-local user indices
  // force-only bonded tables: the groups, then the other atoms with terms
  // (global user indices, partners global too)
  vp::BGroup *bgroups = nullptr;
  int32_t n_bgroups = 0;
  int32_t *bf_atoms = nullptr;   // [n_bf_atoms]
  int32_t *bf_start = nullptr;   // [n_bf_atoms + 1]
  vp::BTerm *bf_terms = nullptr;
  int32_t n_bf_atoms = 0;
  int32_t *ex_start = nullptr;  // [users + 1]
  int32_t *ex_list = nullptr;   // replica-local user indices
  int32_t *role0 = nullptr;     // [users] 0: listed alone, 1: first atom of a three-atom site, 2: other site atom
  float *cmap = nullptr;        // native contact maps, [ns][ns] per distinct map
  float *cskew = nullptr;       // the same maps per tile in diagonal order: [tile][k][lane] = C~f(row lane, column (lane + k) mod 64)
  float4 *cforce = nullptr;     // [solute total] constant bias force
  double *xf = nullptr;         // [solute rows][3] FP64 X_f of the replicas that give one
  double *rmsd = nullptr;       // [R] RMSD to X_f (vp_select_path, vp_observables)
  double *records = nullptr;    // [R][out_cap][VP_REC_COUNT] energy records
  int32_t out_cap = 0;
  int2 *cpairs = nullptr;       // native-contact pairs (replica-local user indices) per distinct map
  int32_t *t_form = nullptr;    // [sum of contacts] first-formation step, -1 = not yet
  int32_t max_contacts = 0;
  // scratch shared by both contexts (list rebuild)
  int4 *xq_t = nullptr;
  float4 *vel_t = nullptr;
  int32_t *orig_t = nullptr;
  int32_t *wrap_t = nullptr;
  int32_t *cellid_t = nullptr;  // [slots] sort bucket (column, z slab) of each old slot
  int32_t *zkey_t = nullptr;    // [slots] serpentine z key of each old slot
  int32_t *fcell_t = nullptr;   // [slots] fine cell of each old slot
  int32_t *bucket_t = nullptr;  // [slots] old slots grouped by column / new slots by cell
  int2 *bko_t = nullptr;        // [slots] (z key, user index) in bucket order
  int32_t *cellpos_t = nullptr; // [slots] position of each new slot in fine-cell order
  float4 *tx_t = nullptr;       // [2][slots] tangents in the new order (rebuild)
  float4 *tv_t = nullptr;
  int4 *cellx_t = nullptr;      // [slots] fine-cell order: wrapped x, y, z and user index
  int2 *celljw_t = nullptr;     // [slots] fine-cell order: slot (| LJ class << 31 | site role << 29) and packed image
  int32_t *inv_t = nullptr;     // [users] global slot of each atom in the new order (rebuild)
  long long *step = nullptr;  // device step counter
  vp::Work traj, eval;
  bool eval_ready = false;
  bool tangent = false;  // derivatives of the functional are propagated
  int force_shape = 0;   // index into kForceShapes used by the force launches
  // size buckets (cutoff, floor(log2 n)) with their blocks and tile shapes
  struct TileBucket {
    double r_cut;
    int log2n, nrep;
    std::vector<int32_t> blocks;
    int shape;
    double ms[vp::kNumForceShapes];
  };
  std::vector<TileBucket> buckets;
  // force launches of one step: empty = one launch of force_shape over every block
  struct ForceLaunch {
    int shape;
    const int32_t *blist;  // device
    int nblk;
  };
  std::vector<ForceLaunch> force_plan;
  bool plan_split = false;
  std::vector<int32_t> maxnb_override;  // per-replica list capacity set after a first build
  struct GraphEntry {
    int32_t steps;
    hipStream_t stream;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int64_t host_step = 0;
  hipStream_t last_stream = nullptr;
  hipEvent_t done = nullptr;  // recorded at the end of every asynchronous call
  bool done_valid = false;
  bool timing = false;
  std::vector<hipEvent_t> ev_before, ev_after;
  double timing_ms = 0.0;
  int64_t timing_count = 0;
  std::vector<void *> allocations;
  int64_t device_bytes = 0;
};
