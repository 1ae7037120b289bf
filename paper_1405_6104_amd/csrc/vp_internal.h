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
constexpr int kBinThreads = 1024;    // workgroup of the binning kernel
constexpr int kMaxCells = 4096;      // cells per replica held in LDS by the binning kernel
constexpr int kCvBlock = 256;        // solute atoms per contact-map workgroup
constexpr int kMaxCvBlocks = 64;     // => at most 16384 solute atoms
constexpr int kMaxSoluteLds = 8192;  // solute positions staged in LDS (float4, dynamic)
constexpr double kFixScale = 4294967296.0;  // 2^32: fixed-point force unit
constexpr double kForceLimit = 1.0e6;       // kJ/mol/nm: above this a replica is unstable
constexpr double kCoulomb = 138.935458;

// Constant per-replica data (device copy in an array indexed by replica).
struct RepInfo {
  int32_t n, ns, npad, off;     // atoms, solute atoms, padded slots, first slot
  int32_t uoff;                 // first user-order index
  int32_t tile0, ntiles;        // tiles [tile0, tile0+ntiles)
  int32_t bias, min_sep;
  int32_t nc[3], ncell, cell0;  // cell grid and offset into the cell arrays
  int32_t maxnb;                // per-atom list capacity
  int64_t list_off;             // first element of this replica's list block
  int64_t cmap_off;             // first element of the native contact map (FP32 [ns][ns])
  int32_t cv_blocks;            // contact-map workgroups used by this replica
  int32_t sol_off;              // first index in per-solute arrays
  int32_t nstlist_max;
  float L[3], invL[3];
  float rc2, rl2, krf2, crf;    // cutoff^2, list radius^2, 2*k_rf, c_rf
  float half_skin_margin;       // displacement that forces a rebuild
  float cr0, crs, crc;          // contact r0, switch start, switch end
  double Ld[3];
  double rc, krf;
  double bias_k, ramp_rate, z_target;
  double kT, dt, reach_tol;
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
  int32_t pad;
};

// One bonded contribution evaluated by the atom that owns it.
struct BTerm {
  int32_t kind;  // 0: bond to a; 1: angle end (vertex a, other end b); 2: angle vertex (ends a, b)
  int32_t a, b;
  int32_t pad;
  double k, r0;
};

// Device buffers of one evaluation context (trajectory or vp_forces).
struct Work {
  float4 *xq = nullptr;     // [slots] x, y, z (unwrapped), charge
  float4 *vel = nullptr;    // [slots] vx, vy, vz, 0
  float2 *prm = nullptr;    // [slots] sigma/2, sqrt(eps)
  float4 *integ = nullptr;  // [slots] 1/m, c1, sigma_v, 0
  int32_t *orig = nullptr;  // [slots] replica-local user index or -1
  float4 *xref = nullptr;   // [slots] positions at the last list build
  int32_t *inv = nullptr;   // [users] global slot of each atom
  long long *F = nullptr;   // [3][slots] fixed-point forces (without bias), SoA
  int64_t fstride = 0;      // slots: distance between the x, y and z planes of F
  int32_t *nbcnt = nullptr;     // [slots]
  uint16_t *nblist = nullptr;   // per replica [maxnb][npad]
  int32_t *cell_start = nullptr;  // [sum ncell + R]
  int32_t *cell_of = nullptr;     // [slots] cell of each new slot
  float4 *g = nullptr;            // [solute total] dz/dx (xyz) of each solute atom
  double *zpart = nullptr;        // [R][kMaxCvBlocks]
  double *gpart = nullptr;        // [R][kMaxCvBlocks] sum |g|^2/(gamma m)
  double *epart = nullptr;        // [tiles][4] energy partials (LJ, RF, bond, angle)
  int32_t *flags = nullptr;       // [R] rebuild flag for the eval context
};

struct Timing;

}  // namespace vp

struct vp_system {
  int32_t R = 0;
  int64_t n_users = 0;   // sum of atoms
  int64_t n_slots = 0;   // sum of padded atoms
  int32_t n_tiles = 0;
  int64_t n_cells = 0;
  int64_t list_elems = 0;
  int64_t n_solute_total = 0;
  vp_options opt{};
  std::vector<vp::RepInfo> info_h;
  vp::RepInfo *info = nullptr;    // device
  vp::RepState *state = nullptr;  // device
  int32_t *tile_rep = nullptr;    // [tiles] replica of each tile (XCD-aware order)
  int32_t *tile_first = nullptr;  // [tiles] first slot of each tile
  // constant per-atom data in user order
  float4 *q0 = nullptr;      // [users] charge in .w (xyz unused)
  float2 *prm0 = nullptr;    // [users]
  float4 *integ0 = nullptr;  // [users]
  double *igm0 = nullptr;    // [users] 1/(gamma m) (solute entries used)
  double *mass0 = nullptr;   // [users] masses
  int32_t *bt_start = nullptr;  // [users + 1]
  vp::BTerm *bterms = nullptr;
  int32_t *ex_start = nullptr;  // [users + 1]
  int32_t *ex_list = nullptr;   // replica-local user indices
  float *cmap = nullptr;        // native contact maps, [ns][ns] per distinct map
  float4 *cforce = nullptr;     // [solute total] constant bias force
  // scratch shared by both contexts (list rebuild)
  float4 *xq_t = nullptr;
  float4 *vel_t = nullptr;
  int32_t *orig_t = nullptr;
  int32_t *src_t = nullptr;
  int32_t *cellid_t = nullptr;
  int32_t *bucket_t = nullptr;
  int32_t *borig_t = nullptr;
  long long *step = nullptr;  // device step counter
  vp::Work traj, eval;
  bool eval_ready = false;
  // graphs keyed by (steps, first-block) shape
  struct GraphEntry {
    int32_t steps;
    hipStream_t stream;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  bool started = false;       // a step has begun since the last finishing half-kick
  int64_t host_step = 0;
  hipStream_t last_stream = nullptr;
  // force-kernel timing: one event pair per step of a block, reused per replay
  bool timing = false;
  std::vector<hipEvent_t> ev_before, ev_after;
  double timing_ms = 0.0;
  int64_t timing_count = 0;
  std::vector<void *> allocations;
};
