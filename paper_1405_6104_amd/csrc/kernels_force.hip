// Forces of the potential U(X,Y) and the collective variable of the bias.
//
// k_forces: one workgroup (PARTS waves) per block of 64 atoms.  The block's
// neighbourhood (every atom its lists name, with its periodic image applied
// as an exact integer shift) is staged in LDS as (x, y, z, LDS address of
// its type-table row), followed by the replica's (charge, sigma, epsilon)
// type table.  Wave w walks the list chunks (rows of eight 16-bit LDS
// indices) w, w + PARTS, ... of the 64 atoms' full lists, so every pair is
// read from LDS instead of gathered from memory and no image arithmetic is
// left in the pair loop.  A list holds the partners with Lennard-Jones
// parameters first; a chunk in which no lane with LJ parameters still has
// such partners runs the reaction-field term alone.  Potential-shifted LJ
// (Lorentz-Berthelot) + reaction-field Coulomb in FP32 on integer-exact
// separations; chunk c feeds partial sum c mod 16, the 16 sums are added in
// index order (one wave per force component) and stored as 64-bit fixed
// point.  Both members of a pair evaluate it (no atomics), and the list order
// is fixed by the deterministic sort, so results do not depend on
// scheduling.  Bonded terms are added by k_bonded_forces (one thread per
// water-like group of three atoms or per other atom with terms).
//
// k_cv_pairs / k_cv_reduce / k_cv: collective variable z and dz/dx of the
// solute (contact map: one wave per 64 x 64 tile of solute pairs, then one
// wave per row tile; radius of gyration, constant force and no bias: one
// workgroup), with FP64 partial sums of z and of
// sum_i |dz/dx_i|^2/(gamma_i m_i) per row tile that the consumers reduce in a
// fixed order.
#include "vp_device.h"
#include "vp_launch.h"

namespace vp {
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const f4v lds_f4;
typedef __attribute__((address_space(3))) const float lds_f1;
__device__ __forceinline__ const lds_f4 *lds_row(int a) { return (const lds_f4 *)(size_t)a; }
__device__ __forceinline__ const lds_f1 *lds_word(int a) { return (const lds_f1 *)(size_t)a; }

// Copies a block's staged neighbourhood into LDS: entry s (slot | 3 x 5-bit
// image shift) becomes that atom's position shifted by the image, with the
// LDS byte address of its type-table row (trow + 16 type) in place of the
// type, so a pair reads the row without an address computation.  Each thread keeps kStageBatch entries in flight (their codes, then
// their positions) so that the gathers cost two memory latencies per batch
// rather than two per entry.
constexpr int kStageBatch = 8;
template <int NT>
__device__ __forceinline__ void stage_neighbourhood(const uint32_t *__restrict__ stg, int nst,
                                                    const int4 *__restrict__ xr, int Lx, int Ly, int Lz,
                                                    int trow, int tid, int4 *__restrict__ st) {
  for (int s0 = 0; s0 < nst; s0 += NT * kStageBatch) {
    // loads past the end read the last entry again (no branch between the
    // loads, so they stay in flight together); only the stores are guarded
    uint32_t e[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) e[k] = stg[min(s0 + k * NT + tid, nst - 1)];
    int4 xj[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) xj[k] = xr[e[k] & 0xffffu];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      const int s = s0 + k * NT + tid;
      const int sx = (int)((e[k] >> 16) & 31) - 16, sy = (int)((e[k] >> 21) & 31) - 16,
                sz = (int)((e[k] >> 26) & 31) - 16;
      if (s < nst)
        st[s] = make_int4(xj[k].x + sx * Lx, xj[k].y + sy * Ly, xj[k].z + sz * Lz, trow + 16 * xj[k].w);
    }
  }
}

// The same staging for the pair kernel, with the coordinates stored as FP32
// values relative to the block centre c (bit patterns in the int4): every
// such coordinate is an integer below 2^24 grid units (the list build checks
// it), so it is exact, and so is the FP32 difference of two of them.
template <int NT>
__device__ __forceinline__ void stage_neighbourhood_rel(const uint32_t *__restrict__ stg, int nst,
                                                        const int4 *__restrict__ xr, int Lx, int Ly, int Lz,
                                                        int trow, int tid, int4 *__restrict__ st, int4 c) {
  for (int s0 = 0; s0 < nst; s0 += NT * kStageBatch) {
    uint32_t e[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) e[k] = stg[min(s0 + k * NT + tid, nst - 1)];
    int4 xj[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) xj[k] = xr[e[k] & 0xffffu];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k) {
      const int s = s0 + k * NT + tid;
      const int sx = (int)((e[k] >> 16) & 31) - 16, sy = (int)((e[k] >> 21) & 31) - 16,
                sz = (int)((e[k] >> 26) & 31) - 16;
      if (s < nst)
        st[s] = make_int4(__float_as_int((float)(xj[k].x + sx * Lx - c.x)),
                          __float_as_int((float)(xj[k].y + sy * Ly - c.y)),
                          __float_as_int((float)(xj[k].z + sz * Lz - c.z)), trow + 16 * xj[k].w);
    }
  }
}

// One pair with the LJ + reaction-field evaluation: the force scalar over
// one 1/r^2, the cutoff applied by a select (no divergent branch).
__device__ __forceinline__ void pair_full(const int4 sj, const f4v tj, const float4 ti, float wx, float wy,
                                          float wz, float rc2, float krf2, float &fx, float &fy, float &fz) {
  const float dx = __int_as_float(sj.x) - wx, dy = __int_as_float(sj.y) - wy, dz = __int_as_float(sj.z) - wz;
  const float r2 = qr2(dx, dy, dz);
  const bool in = r2 < rc2;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r2inv = rinv * rinv;
  const float sg = ti.y + tj.y;
  const float sr2 = sg * sg * r2inv;
  const float sr6 = sr2 * sr2 * sr2;
  const float ee = ti.z * tj.z;
  const float c6 = ee * sr6 * __builtin_fmaf(2.0f, sr6, -1.0f);
  const float qq = ti.x * tj.x;
  const float cq = qq * __builtin_fmaf(rinv, r2inv, -krf2);
  const float fs = in ? __builtin_fmaf(c6, r2inv, cq) : 0.0f;
  fx = __builtin_fmaf(-fs, dx, fx);
  fy = __builtin_fmaf(-fs, dy, fy);
  fz = __builtin_fmaf(-fs, dz, fz);
}

// One list chunk (8 single-atom entries of one atom's list) evaluated against
// the staged neighbourhood: LJ + reaction-field forces accumulated in the
// chunk's order into (fx, fy, fz).  UNROLL entries share one batch of LDS
// reads.
template <int UNROLL>
__device__ __forceinline__ void eval_chunk(const uint4 e, const int4 *__restrict__ st, const float4 ti, float wx,
                                           float wy, float wz, float rc2, float krf2, float &fx, float &fy,
                                           float &fz) {
  const uint32_t w[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
  for (int h = 0; h < 8; h += UNROLL) {
    int4 sj[UNROLL];
#pragma unroll
    for (int v = 0; v < UNROLL; ++v) {
      const int u = h + v;
      sj[v] = st[(w[u >> 1] >> (16 * (u & 1))) & 0xffffu];
    }
    f4v tj[UNROLL];
#pragma unroll
    for (int v = 0; v < UNROLL; ++v) tj[v] = *lds_row(sj[v].w);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) pair_full(sj[u], tj[u], ti, wx, wy, wz, rc2, krf2, fx, fy, fz);
  }
}

// One chunk of site entries: each entry names a three-atom site staged at
// three consecutive places (its first atom, then two atoms without LJ
// parameters).  The first atom takes the LJ + reaction-field evaluation,
// the other two the reaction-field term alone, read with their charge only
// (for them the LJ factor of the full evaluation is an exact zero, so the
// result has the same bits).  Two sites share one batch of LDS reads.
__device__ __forceinline__ void pair_rf(const int4 sj, const float qj, const float qi, float wx, float wy,
                                        float wz, float rc2, float krf2, float &fx, float &fy, float &fz) {
  const float dx = __int_as_float(sj.x) - wx, dy = __int_as_float(sj.y) - wy, dz = __int_as_float(sj.z) - wz;
  const float r2 = qr2(dx, dy, dz);
  const bool in = r2 < rc2;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float r2inv = rinv * rinv;
  const float qq = qi * qj;
  const float cq = qq * __builtin_fmaf(rinv, r2inv, -krf2);
  const float fs = in ? cq : 0.0f;
  fx = __builtin_fmaf(-fs, dx, fx);
  fy = __builtin_fmaf(-fs, dy, fy);
  fz = __builtin_fmaf(-fs, dz, fz);
}
__device__ __forceinline__ void eval_chunk_sites(const uint4 e, const int4 *__restrict__ st, const float4 ti,
                                                 float wx, float wy, float wz, float rc2, float krf2, float &fx,
                                                 float &fy, float &fz) {
  const uint32_t w[4] = {e.x, e.y, e.z, e.w};
  constexpr int SB = 2;  // sites per batch of LDS reads
#pragma unroll
  for (int h = 0; h < 8; h += SB) {
    int4 sj[SB][3];
#pragma unroll
    for (int v = 0; v < SB; ++v) {
      const int u = h + v;
      const int L = (w[u >> 1] >> (16 * (u & 1))) & 0xffffu;
      sj[v][0] = st[L];
      sj[v][1] = st[L + 1];
      sj[v][2] = st[L + 2];
    }
    f4v t0[SB];
    float q1[SB], q2[SB];
#pragma unroll
    for (int v = 0; v < SB; ++v) {
      t0[v] = *lds_row(sj[v][0].w);
      q1[v] = *lds_word(sj[v][1].w);
      q2[v] = *lds_word(sj[v][2].w);
    }
#pragma unroll
    for (int v = 0; v < SB; ++v) {
      pair_full(sj[v][0], t0[v], ti, wx, wy, wz, rc2, krf2, fx, fy, fz);
      pair_rf(sj[v][1], q1[v], ti.x, wx, wy, wz, rc2, krf2, fx, fy, fz);
      pair_rf(sj[v][2], q2[v], ti.x, wx, wy, wz, rc2, krf2, fx, fy, fz);
    }
  }
}

// Tile shape: PARTS waves share one block's staged neighbourhood and UNROLL
// list entries share one batch of LDS reads; MINW asks the compiler for
// registers that let MINW waves share a SIMD.  blist (or NULL for all blocks)
// selects the blocks of one launch.
//
// The result does not depend on the shape: chunk c of an atom's list is summed
// into logical accumulator c mod kLogicalParts (each wave holds
// kLogicalParts / PARTS of them, in chunk order), and the accumulators are
// added in index order at the end.  Every shape therefore performs the same
// FP32 operations in the same order, and the forces agree bit for bit
// whichever shape a launch uses.
template <int PARTS, int UNROLL, int MINW>
__global__ __launch_bounds__(64 * PARTS) __attribute__((amdgpu_waves_per_eu(MINW))) void k_forces(const RepInfo *__restrict__ info, Work W,
                                                       const int32_t *__restrict__ tile_rep,
                                                       const int32_t *__restrict__ tile_first,
                                                       const int32_t *__restrict__ blist, int nblk,
                                                       const float4 *__restrict__ types,
                                                       int stage_slots) {
  constexpr int NT = 64 * PARTS;
  constexpr int SETS = kLogicalParts / PARTS;
  static_assert(kLogicalParts % PARTS == 0, "PARTS must divide the logical accumulator count");
  extern __shared__ int4 lds[];
  int4 *st = lds;                                              // [stage_slots] staged atoms
  float4 *tab = reinterpret_cast<float4 *>(lds + stage_slots);  // the replica's type table
  // after the pair loop the staging area holds the logical partial sums:
  // forces [3][kLogicalParts][64] FP32
  float *red = reinterpret_cast<float *>(lds);
  const int bt = xcd_tile(blockIdx.x, nblk);
  if (bt < 0) return;
  const int b = blist ? blist[bt] : bt;
  const int tile = b / (kTile / kBlk);
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p0 = tile_first[tile] + (b % (kTile / kBlk)) * kBlk;
  const int tid = threadIdx.x;
  if (p0 >= R.n) {
    if (tid < kBlk) {
      const int slot = R.off + p0 + tid;
      W.F[slot] = 0;
      W.F[W.fstride + slot] = 0;
      W.F[2 * W.fstride + slot] = 0;
    }
    return;
  }
  const int Lx = R.Lq[0], Ly = R.Lq[1], Lz = R.Lq[2];
  // ---- stage the neighbourhood and the type table
  const int trow = (int)(size_t)(const lds_f4 *)tab;  // LDS byte address of the type table
  const int4 bc = W.bctr[b];
  stage_neighbourhood_rel<NT>(W.stage + (int64_t)b * W.stage_stride, W.stage_n[b], W.xq + R.off, Lx, Ly, Lz,
                              trow, tid, st, bc);
  if (tid < kStageDummies) {
    const int far = __float_as_int((float)kDummyCoord);
    st[R.stage_cap + tid] = make_int4(far, far, far, trow + 16 * R.ntypes);
  }
  for (int t = tid; t <= R.ntypes; t += NT) tab[t] = types[R.type_off + t];
  __syncthreads();

  const int lane = tid & (kBlk - 1), part = tid / kBlk;
  const int p = p0 + lane;
  const int slot = R.off + p;
  const bool active = p < R.n;
  float fx[SETS], fy[SETS], fz[SETS];
#pragma unroll
  for (int k = 0; k < SETS; ++k) fx[k] = fy[k] = fz[k] = 0.0f;
  int4 xi = make_int4(0, 0, 0, 0);
  if (active) {
    xi = W.xq[slot];
    const int wr = W.wrap[slot];
    // the lane's atom relative to the block centre (exact in FP32)
    const float wx = (float)(xi.x - unpack_wrap(wr, 0) * Lx - bc.x);
    const float wy = (float)(xi.y - unpack_wrap(wr, 1) * Ly - bc.y);
    const float wz = (float)(xi.z - unpack_wrap(wr, 2) * Lz - bc.z);
    const float4 ti = tab[xi.w];
    const float rc2 = R.rc2q, krf2 = R.krf2q;
    const int nch = W.nbcnt[slot] >> 3, nlj = W.nblj[slot], rowcap = R.maxnb >> 3;
    const uint4 *lp = reinterpret_cast<const uint4 *>(W.nblist + R.list_off + (int64_t)(b - R.blk0) * R.maxnb * kBlk);
    uint4 e = lp[list_row(chunk_row(min(part, max(nch - 1, 0)), nlj, rowcap), lane)];
    // this wave takes chunks part, part + PARTS, ...: its k-th chunk of every
    // group of SETS feeds set k, which is logical accumulator k PARTS + part.
    // A lane's chunk c < nlj holds single atoms, a later one sites; a chunk
    // step runs each kind for the lanes that hold it.
    for (int c0 = part; c0 < nch; c0 += PARTS * SETS) {
#pragma unroll
      for (int k = 0; k < SETS; ++k) {
        const int c = c0 + k * PARTS;
        if (c < nch) {
          // the next chunk's indices are fetched while this one is evaluated
          // (the last chunk is fetched again rather than reading past the list)
          const uint4 en = lp[list_row(chunk_row(min(c + PARTS, nch - 1), nlj, rowcap), lane)];
          const bool single = c < nlj;
          if (single) eval_chunk<UNROLL>(e, st, ti, wx, wy, wz, rc2, krf2, fx[k], fy[k], fz[k]);
          else eval_chunk_sites(e, st, ti, wx, wy, wz, rc2, krf2, fx[k], fy[k], fz[k]);
          e = en;
        }
      }
    }
  }
  // ---- fixed-order sum of the logical partial sums, bonded terms, store
  __syncthreads();  // every wave is done with the staged neighbourhood
#pragma unroll
  for (int k = 0; k < SETS; ++k) {
    const int q = k * PARTS + part;  // logical accumulator held in set k
    red[(0 * kLogicalParts + q) * kBlk + lane] = fx[k];
    red[(1 * kLogicalParts + q) * kBlk + lane] = fy[k];
    red[(2 * kLogicalParts + q) * kBlk + lane] = fz[k];
  }
  __syncthreads();
  // wave d (d < 3) sums component d of the block's 64 atoms
  static_assert(PARTS >= 3, "one wave per force component");
  if (part < 3) {
    long long v = 0;
    if (active) {
      const float *rd = red + part * kLogicalParts * kBlk + lane;
      float sum = rd[0];
#pragma unroll 5
      for (int q = 1; q < kLogicalParts; ++q) sum += rd[q * kBlk];
      v = to_fix((double)sum * kInvQ);
    }
    W.F[part * W.fstride + slot] = v;
  }
}

// Energies and virial of the pair terms (for vp_forces and the energy records
// of trajectories), one workgroup of kParts waves per 64-atom block over the
// same lists and staging as k_forces: per list entry, in FP64 from the FP32
// quantities of the force kernel, the shifted LJ and reaction-field energies
// and the virial (1/2) fs q^2 d (x) d (each pair sits in both atoms' lists;
// with F_j = fs q d the pair's r (x) F_j is fs q^2 d (x) d, symmetric).  The
// waves' partials are added in wave order and over the block's lanes in a
// fixed butterfly, into W.epart[b][0, 1] and [b][kEpPairW .. +9).  GATED: returns
// at once unless the step being completed (*step + 1) is a multiple of nst_out.
template <bool GATED>
__global__ __launch_bounds__(kForceThreads) void k_pair_energy(const RepInfo *__restrict__ info, Work W,
                                                               const int32_t *__restrict__ tile_rep,
                                                               const int32_t *__restrict__ tile_first,
                                                               int nblk, const float4 *__restrict__ types,
                                                               int stage_slots,
                                                               const long long *__restrict__ step,
                                                               int nst_out) {
  if (GATED && (*step + 1) % nst_out != 0) return;
  extern __shared__ int4 lds[];
  int4 *st = lds;
  float4 *tab = reinterpret_cast<float4 *>(lds + stage_slots);
  double *red = reinterpret_cast<double *>(lds);  // [8 values][kParts][64] after the loop
  const int b = xcd_tile(blockIdx.x, nblk);
  if (b < 0) return;
  const int tile = b / (kTile / kBlk);
  const RepInfo &R = info[tile_rep[tile]];
  const int p0 = tile_first[tile] + (b % (kTile / kBlk)) * kBlk;
  const int tid = threadIdx.x;
  if (p0 >= R.n) {
    if (tid < 2) W.epart[kEp * (size_t)b + tid] = 0.0;
    if (tid < 9) W.epart[kEp * (size_t)b + kEpPairW + tid] = 0.0;
    return;
  }
  const int Lx = R.Lq[0], Ly = R.Lq[1], Lz = R.Lq[2];
  const int trow = (int)sizeof(int4) * stage_slots;
  stage_neighbourhood<kForceThreads>(W.stage + (int64_t)b * W.stage_stride, W.stage_n[b], W.xq + R.off, Lx,
                                     Ly, Lz, trow, tid, st);
  if (tid < kStageDummies) st[R.stage_cap + tid] = make_int4(kDummyCoord, kDummyCoord, kDummyCoord, trow + 16 * R.ntypes);
  for (int t = tid; t <= R.ntypes; t += kForceThreads) tab[t] = types[R.type_off + t];
  __syncthreads();
  const int lane = tid & (kBlk - 1), part = tid / kBlk;
  const int p = p0 + lane;
  const int slot = R.off + p;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // LJ, RF, W xx yy zz xy xz yz
  if (p < R.n) {
    const int4 xi = W.xq[slot];
    const int wr = W.wrap[slot];
    const int wx = xi.x - unpack_wrap(wr, 0) * Lx, wy = xi.y - unpack_wrap(wr, 1) * Ly,
              wz = xi.z - unpack_wrap(wr, 2) * Lz;
    const float4 ti = tab[xi.w];
    const float rc2 = R.rc2q, krf2 = R.krf2q;
    const int nent = W.nbcnt[slot], nlj = W.nblj[slot], rowcap = R.maxnb >> 3;
    const uint16_t *lp = W.nblist + R.list_off + (int64_t)(b - R.blk0) * R.maxnb * kBlk;
    // entry k names one atom (chunks below nlj) or a three-atom site
    for (int k = part; k < nent; k += kParts) {
      const int L0 = lp[list_row(chunk_row(k >> 3, nlj, rowcap), lane) * 8 + (k & 7)];
      const int na = (k >> 3) < nlj ? 1 : 3;
      for (int m = 0; m < na; ++m) {
      const int L = L0 + m;
      const int4 sj = st[L];
      const float4 tj = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(lds) + sj.w);
      const float dx = (float)(sj.x - wx), dy = (float)(sj.y - wy), dz = (float)(sj.z - wz);
      const float r2 = qr2(dx, dy, dz);
      if (!(r2 < rc2)) continue;
      // the force kernel's FP32 quantities
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float r2inv = rinv * rinv;
      const float sg = ti.y + tj.y;
      const float sr2 = sg * sg * r2inv;
      const float sr6 = sr2 * sr2 * sr2;
      const float ee = ti.z * tj.z;
      const float c6 = ee * sr6 * __builtin_fmaf(2.0f, sr6, -1.0f);
      const float qq = ti.x * tj.x;
      const float cq = qq * __builtin_fmaf(rinv, r2inv, -krf2);
      const float fs = __builtin_fmaf(c6, r2inv, cq);
      // ee = 24 eps 2^44, qq = f q q 2^66 (see the type table)
      const double e4 = (double)ee * (1.0 / 6.0) * (kInvQ * kInvQ);
      const double s2c = (double)sg * sg / ((double)rc2);
      const double s6c = s2c * s2c * s2c;
      acc[0] += e4 * ((double)sr6 * sr6 - sr6) - e4 * (s6c * s6c - s6c);
      const double fqq = (double)qq * (kInvQ * kInvQ * kInvQ);
      acc[1] += fqq * ((double)rinv * kQ + R.krf * (double)r2 * (kInvQ * kInvQ) - R.crf);
      const double w = 0.5 * (double)fs * (kInvQ * kInvQ);
      const double ddx = dx, ddy = dy, ddz = dz;
      acc[2] += w * ddx * ddx;
      acc[3] += w * ddy * ddy;
      acc[4] += w * ddz * ddz;
      acc[5] += w * ddx * ddy;
      acc[6] += w * ddx * ddz;
      acc[7] += w * ddy * ddz;
      }
    }
  }
  __syncthreads();  // the staged neighbourhood is no longer read
#pragma unroll
  for (int v = 0; v < 8; ++v) red[(v * kParts + part) * kBlk + lane] = acc[v];
  __syncthreads();
  if (part != 0) return;
  double sum[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    double a = 0.0;
    for (int q = 0; q < kParts; ++q) a += red[(v * kParts + q) * kBlk + lane];
    sum[v] = wave_sum(a);
  }
  if (lane == 0) {
    // each pair sits in both atoms' lists: half of every energy
    double *e = W.epart + kEp * (size_t)b;
    e[0] = 0.5 * sum[0];
    e[1] = 0.5 * sum[1];
    double *wv = e + kEpPairW;
    wv[0] = sum[2]; wv[1] = sum[5]; wv[2] = sum[6];
    wv[3] = sum[5]; wv[4] = sum[3]; wv[5] = sum[7];
    wv[6] = sum[6]; wv[7] = sum[7]; wv[8] = sum[4];
  }
}

// One bonded term of an atom at xi: a bond to the atom at p1, or an angle with
// vertex p1 and other end p2 (kind 1) or with ends p1 and p2 (kind 2).
template <bool ENERGY>
__device__ __forceinline__ void bonded_term(const BTerm &T, const int4 xi, const int4 p1, const int4 p2,
                                            double &bx, double &by, double &bz, double &ebond,
                                            double &eangle) {
  if (T.kind == 0) {
    const int4 xb = p1;
    const double d0 = (double)(xb.x - xi.x) * kInvQ, d1 = (double)(xb.y - xi.y) * kInvQ,
                 d2 = (double)(xb.z - xi.z) * kInvQ;
    const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double g = T.k * (rr - T.r0) / rr;
    bx += g * d0;
    by += g * d1;
    bz += g * d2;
    if (ENERGY) ebond += 0.25 * T.k * (rr - T.r0) * (rr - T.r0);  // owned by both atoms
  } else {
    // angle end--vertex--end; this atom is an end (kind 1) or the vertex (kind 2)
    int4 pa, pc, pb;
    if (T.kind == 1) {
      pa = xi;
      pc = p1;
      pb = p2;
    } else {
      pa = p1;
      pc = xi;
      pb = p2;
    }
    const double u0 = (double)(pa.x - pc.x) * kInvQ, u1 = (double)(pa.y - pc.y) * kInvQ,
                 u2 = (double)(pa.z - pc.z) * kInvQ;
    const double w0 = (double)(pb.x - pc.x) * kInvQ, w1 = (double)(pb.y - pc.y) * kInvQ,
                 w2 = (double)(pb.z - pc.z) * kInvQ;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2, ww = w0 * w0 + w1 * w1 + w2 * w2;
    const double uw = u0 * w0 + u1 * w1 + u2 * w2;
    // three reciprocals instead of a division per force component
    const double inn = 1.0 / sqrt(uu * ww), iuu = 1.0 / uu, iww = 1.0 / ww;
    double cs = uw * inn;
    cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
    const double th = acos(cs);
    double sn = sqrt(1.0 - cs * cs);
    sn = sn < 1e-12 ? 1e-12 : sn;
    const double dv = T.k * (th - T.r0) / sn;
    // gradient of theta at the end a (ga) and at the end b (gb); the vertex
    // takes -(ga + gb); a select rather than a branch keeps the wave together
    const double ga0 = w0 * inn - cs * u0 * iuu, ga1 = w1 * inn - cs * u1 * iuu, ga2 = w2 * inn - cs * u2 * iuu;
    const double gb0 = u0 * inn - cs * w0 * iww, gb1 = u1 * inn - cs * w1 * iww, gb2 = u2 * inn - cs * w2 * iww;
    const bool end = T.kind == 1;
    bx += dv * (end ? ga0 : -(ga0 + gb0));
    by += dv * (end ? ga1 : -(ga1 + gb1));
    bz += dv * (end ? ga2 : -(ga2 + gb2));
    if (ENERGY) eangle += (0.5 / 3.0) * T.k * (th - T.r0) * (th - T.r0);  // owned by 3 atoms
  }
}

// Terms gathered per pass of a per-atom bonded loop: their records, partner
// slots and partner positions are each loaded together, so an atom's terms
// cost three dependent loads per pass instead of three per term.
constexpr int kBondBatch = 4;

// Threads per workgroup of k_bonded_forces.
constexpr int kBondedThreads = 256;

// The force of one bonded group's term on its three atoms (f[3 m + k] for
// atom m, component k), with the arithmetic of bonded_term: a bond as its
// first atom evaluates it (its partner takes the negated force), an angle as
// its first end evaluates it (the vertex takes -(ga + gb), the other end gb).
// Local indices pick values by selects, so nothing is indexed at run time.
__device__ __forceinline__ void group_term(int code, double k, double r0, const int4 p0, const int4 p1,
                                           const int4 p2, double (&f)[9]) {
  const int kind = code & 15, li = (code >> 4) & 15, lc = (code >> 8) & 15, lj = (code >> 12) & 15;
  auto pick = [&](int m, int a0, int a1, int a2) { return m == 0 ? a0 : (m == 1 ? a1 : a2); };
  const int ix = pick(li, p0.x, p1.x, p2.x), iy = pick(li, p0.y, p1.y, p2.y), iz = pick(li, p0.z, p1.z, p2.z);
  const int jx = pick(lj, p0.x, p1.x, p2.x), jy = pick(lj, p0.y, p1.y, p2.y), jz = pick(lj, p0.z, p1.z, p2.z);
  if (kind == 0) {
    const double d0 = (double)(jx - ix) * kInvQ, d1 = (double)(jy - iy) * kInvQ, d2 = (double)(jz - iz) * kInvQ;
    const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double g = k * (rr - r0) / rr;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double c = m == li ? g : (m == lj ? -g : 0.0);
      f[3 * m] = __builtin_fma(c, d0, f[3 * m]);
      f[3 * m + 1] = __builtin_fma(c, d1, f[3 * m + 1]);
      f[3 * m + 2] = __builtin_fma(c, d2, f[3 * m + 2]);
    }
  } else {
    const int cx = pick(lc, p0.x, p1.x, p2.x), cy = pick(lc, p0.y, p1.y, p2.y), cz = pick(lc, p0.z, p1.z, p2.z);
    const double u0 = (double)(ix - cx) * kInvQ, u1 = (double)(iy - cy) * kInvQ, u2 = (double)(iz - cz) * kInvQ;
    const double w0 = (double)(jx - cx) * kInvQ, w1 = (double)(jy - cy) * kInvQ, w2 = (double)(jz - cz) * kInvQ;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2, ww = w0 * w0 + w1 * w1 + w2 * w2;
    const double uw = u0 * w0 + u1 * w1 + u2 * w2;
    const double inn = 1.0 / sqrt(uu * ww), iuu = 1.0 / uu, iww = 1.0 / ww;
    double cs = uw * inn;
    cs = cs > 1.0 ? 1.0 : (cs < -1.0 ? -1.0 : cs);
    const double th = acos(cs);
    double sn = sqrt(1.0 - cs * cs);
    sn = sn < 1e-12 ? 1e-12 : sn;
    const double dv = k * (th - r0) / sn;
    const double ga0 = w0 * inn - cs * u0 * iuu, ga1 = w1 * inn - cs * u1 * iuu, ga2 = w2 * inn - cs * u2 * iuu;
    const double gb0 = u0 * inn - cs * w0 * iww, gb1 = u1 * inn - cs * w1 * iww, gb2 = u2 * inn - cs * w2 * iww;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const bool a = m == li, bb = m == lj;
      f[3 * m] = __builtin_fma(dv, a ? ga0 : (bb ? gb0 : -(ga0 + gb0)), f[3 * m]);
      f[3 * m + 1] = __builtin_fma(dv, a ? ga1 : (bb ? gb1 : -(ga1 + gb1)), f[3 * m + 1]);
      f[3 * m + 2] = __builtin_fma(dv, a ? ga2 : (bb ? gb2 : -(ga2 + gb2)), f[3 * m + 2]);
    }
  }
}

// Bonded forces (harmonic bonds and angles, FP64 on the exact integer
// separations) added to the fixed-point forces the pair kernel stored.  The
// first nwa workgroups (after the XCD deal) take the atoms outside bonded
// groups that have terms, one atom per thread, which evaluates every term it
// belongs to (an angle by its two ends and its vertex), kBondBatch terms per
// pass; the next nwg take the bonded groups, one group per thread, whose
// terms are evaluated once and whose three atoms' forces it stores.  Every
// atom's force is thus written by one thread, and each atom sums its terms in
// the order of its own term list, as the energy kernel below does.  Both
// ranges are dealt to the XCDs in contiguous pieces (atoms and groups are in
// replica order), so each XCD's L2 holds the forces and positions of a few
// replicas; the atoms' longer dependent chains start first.
__global__ __launch_bounds__(kBondedThreads) void k_bonded_forces(Work W, const int32_t *__restrict__ atoms,
                                                                  const int32_t *__restrict__ start,
                                                                  const BTerm *__restrict__ terms, int na,
                                                                  int nwa, const BGroup *__restrict__ groups,
                                                                  int ng, int nwg) {
  const int nba = 8 * ((nwa + 7) / 8);
  if ((int)blockIdx.x >= nba) {
    const int wg = xcd_tile((int)blockIdx.x - nba, nwg);
    if (wg < 0) return;
    const int t = wg * kBondedThreads + threadIdx.x;
    if (t >= ng) return;
    const BGroup G = groups[t];
    const int s0 = W.inv[G.ga], s1 = W.inv[G.ga + 1], s2 = W.inv[G.ga + 2];
    const int4 p0 = W.xq[s0], p1 = W.xq[s1], p2 = W.xq[s2];
    // the pair forces these terms are added to, loaded with the positions
    const int64_t fs = W.fstride;
    const int64_t at[9] = {s0, fs + s0, 2 * fs + s0, s1, fs + s1, 2 * fs + s1, s2, fs + s2, 2 * fs + s2};
    long long fp[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) fp[q] = W.F[at[q]];
    double f[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kGroupTerms; ++q) group_term(G.code[q], G.k[q], G.r0[q], p0, p1, p2, f);
#pragma unroll
    for (int q = 0; q < 9; ++q) W.F[at[q]] = fp[q] + to_fix(f[q]);
    return;
  }
  const int wg = xcd_tile((int)blockIdx.x, nwa);
  if (wg < 0) return;
  const int k = wg * kBondedThreads + threadIdx.x;
  if (k >= na) return;
  const int ga = atoms[k];
  const int slot = W.inv[ga];
  const int4 xi = W.xq[slot];
  const long long f0 = W.F[slot], f1 = W.F[W.fstride + slot], f2 = W.F[2 * W.fstride + slot];
  double bx = 0.0, by = 0.0, bz = 0.0, ebond = 0.0, eangle = 0.0;
  const int t0 = start[k], t1 = start[k + 1];
  for (int u0 = t0; u0 < t1; u0 += kBondBatch) {
    BTerm T[kBondBatch];
#pragma unroll
    for (int u = 0; u < kBondBatch; ++u) T[u] = terms[min(u0 + u, t1 - 1)];
    int q1[kBondBatch], q2[kBondBatch];
#pragma unroll
    for (int u = 0; u < kBondBatch; ++u) {
      q1[u] = W.inv[T[u].a];
      q2[u] = W.inv[T[u].kind == 0 ? T[u].a : T[u].b];
    }
    int4 x1[kBondBatch], x2[kBondBatch];
#pragma unroll
    for (int u = 0; u < kBondBatch; ++u) {
      x1[u] = W.xq[q1[u]];
      x2[u] = W.xq[q2[u]];
    }
#pragma unroll
    for (int u = 0; u < kBondBatch; ++u)
      if (u0 + u < t1) bonded_term<false>(T[u], xi, x1[u], x2[u], bx, by, bz, ebond, eangle);
  }
  W.F[slot] = f0 + to_fix(bx);
  W.F[W.fstride + slot] = f1 + to_fix(by);
  W.F[2 * W.fstride + slot] = f2 + to_fix(bz);
}

// Bonded energies and virial (no forces), one thread per atom: every atom
// evaluates the terms it belongs to; the block's bond and angle energies and
// the virial sum_i x_i (x) F_i^bonded go to W.epart[b][2, 3] and
// [b][kEpBondW .. +9) (each term's forces sum to zero, so this equals the sum
// over terms of (x_i - x_ref) (x) F_i).  Threads take atoms in their original
// order (block b, lane l: atom 64 b + l of the replica), so the term ranges
// and records are read coalesced and the atom's slot comes from one lookup.
// GATED: as in k_pair_energy.
template <bool GATED>
__global__ __launch_bounds__(kBlk) void k_bonded_energy(const RepInfo *__restrict__ info, Work W,
                                                        const int32_t *__restrict__ tile_rep,
                                                        const int32_t *__restrict__ tile_first, int nblk,
                                                        const int32_t *__restrict__ bt_start,
                                                        const BTerm *__restrict__ bterms,
                                                        const long long *__restrict__ step, int nst_out) {
  if (GATED && (*step + 1) % nst_out != 0) return;
  const int b = xcd_tile(blockIdx.x, nblk);
  if (b < 0) return;
  const int tile = b / (kTile / kBlk);
  const RepInfo &R = info[tile_rep[tile]];
  const int p0 = tile_first[tile] + (b % (kTile / kBlk)) * kBlk;
  if (p0 >= R.n) {  // padding block
    if (threadIdx.x < 2) W.epart[kEp * (size_t)b + 2 + threadIdx.x] = 0.0;
    if (threadIdx.x < 9) W.epart[kEp * (size_t)b + kEpBondW + threadIdx.x] = 0.0;
    return;
  }
  const int lane = threadIdx.x;
  const int a = p0 + lane;  // the atom's index in the replica's original order
  const bool active = a < R.n;
  double ebond = 0.0, eangle = 0.0;
  double vir[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (active) {
    const int ga = R.uoff + a;
    const int slot = W.inv[ga];
    const int4 xi = W.xq[slot];
    double bx = 0.0, by = 0.0, bz = 0.0;
    const int t0 = bt_start[ga], t1 = bt_start[ga + 1];
    for (int t = t0; t < t1; t += kBondBatch) {
      BTerm T[kBondBatch];
#pragma unroll
      for (int u = 0; u < kBondBatch; ++u) T[u] = bterms[min(t + u, t1 - 1)];
      int s1[kBondBatch], s2[kBondBatch];
#pragma unroll
      for (int u = 0; u < kBondBatch; ++u) {
        s1[u] = W.inv[R.uoff + T[u].a];
        s2[u] = W.inv[R.uoff + (T[u].kind == 0 ? T[u].a : T[u].b)];
      }
      int4 p1[kBondBatch], p2[kBondBatch];
#pragma unroll
      for (int u = 0; u < kBondBatch; ++u) {
        p1[u] = W.xq[s1[u]];
        p2[u] = W.xq[s2[u]];
      }
#pragma unroll
      for (int u = 0; u < kBondBatch; ++u)
        if (t + u < t1) bonded_term<true>(T[u], xi, p1[u], p2[u], bx, by, bz, ebond, eangle);
    }
    const double x[3] = {(double)xi.x * kInvQ, (double)xi.y * kInvQ, (double)xi.z * kInvQ};
    const double f[3] = {bx, by, bz};
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) vir[3 * u + v] = x[u] * f[v];
  }
  const double v2 = wave_sum(ebond), v3 = wave_sum(eangle);
  double w[9];
  for (int k = 0; k < 9; ++k) w[k] = wave_sum(vir[k]);
  if (lane == 0) {
    double *e = W.epart + kEp * (size_t)b;
    e[2] = v2;
    e[3] = v3;
    for (int k = 0; k < 9; ++k) e[kEpBondW + k] = w[k];
  }
}

// Directional derivative of the potential force along a tangent dx/dtheta_p
// (one direction p per launch): -H_U . xi, the Hessian-vector product that
// carries the pathwise derivative of a trajectory.  Same blocks, lists and
// staging as k_forces; the staged neighbourhood carries its tangents too.
// For a pair, F_i = -f(s) d with s = r^2 and d = x_j - x_i, so
//   dF_i = -f(s) delta - 2 f'(s) (d . delta) d,   delta = xi_j - xi_i,
// with f the LJ + reaction-field force scalar of k_forces; the bonded terms
// are differentiated in FP64 (dual numbers for the angle).  The pair set is
// the force kernel's (exact cutoff).
__global__ __launch_bounds__(kForceThreads) void k_tangent_forces(
    const RepInfo *__restrict__ info, Work W, const int32_t *__restrict__ tile_rep,
    const int32_t *__restrict__ tile_first, int nblk, const float4 *__restrict__ types, int stage_slots,
    int dir) {
  extern __shared__ int4 lds[];
  int4 *st = lds;                                                     // staged atoms
  float4 *sxi = reinterpret_cast<float4 *>(lds + stage_slots);        // their tangents
  float4 *tab = reinterpret_cast<float4 *>(lds + 2 * stage_slots);    // type table
  float *red = reinterpret_cast<float *>(lds);
  const int b = xcd_tile(blockIdx.x, nblk);
  if (b < 0) return;
  const int tile = b / (kTile / kBlk);
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p0 = tile_first[tile] + (b % (kTile / kBlk)) * kBlk;
  const int tid = threadIdx.x;
  const float4 *txp = W.tx + (size_t)dir * W.fstride;
  float4 *tfp = W.tf + (size_t)dir * W.fstride;
  if (p0 >= R.n) {
    if (tid < kBlk) tfp[R.off + p0 + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const int Lx = R.Lq[0], Ly = R.Lq[1], Lz = R.Lq[2];
  const int nst = W.stage_n[b];
  const uint32_t *stg = W.stage + (int64_t)b * W.stage_stride;
  const int4 *xr = W.xq + R.off;
  const int trow = (int)sizeof(int4) * 2 * stage_slots;  // LDS byte address of the type table
  stage_neighbourhood<kForceThreads>(stg, nst, xr, Lx, Ly, Lz, trow, tid, st);
  for (int q0 = 0; q0 < nst; q0 += kForceThreads * kStageBatch) {
    // the staged atoms' tangents, kStageBatch loads in flight per thread
    float4 t[kStageBatch];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k)
      t[k] = txp[R.off + (stg[min(q0 + k * kForceThreads + tid, nst - 1)] & 0xffffu)];
#pragma unroll
    for (int k = 0; k < kStageBatch; ++k)
      if (q0 + k * kForceThreads + tid < nst) sxi[q0 + k * kForceThreads + tid] = t[k];
  }
  if (tid < kStageDummies) {
    st[R.stage_cap + tid] = make_int4(kDummyCoord, kDummyCoord, kDummyCoord, trow + 16 * R.ntypes);
    sxi[R.stage_cap + tid] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int t = tid; t <= R.ntypes; t += kForceThreads) tab[t] = types[R.type_off + t];
  __syncthreads();

  const int lane = tid & (kBlk - 1), part = tid / kBlk;
  const int p = p0 + lane;
  const int slot = R.off + p;
  const bool active = p < R.n;
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  int4 xi = make_int4(0, 0, 0, 0);
  float4 ti4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (active) {
    xi = W.xq[slot];
    ti4 = txp[slot];
    const int wr = W.wrap[slot];
    const int wx = xi.x - unpack_wrap(wr, 0) * Lx, wy = xi.y - unpack_wrap(wr, 1) * Ly,
              wz = xi.z - unpack_wrap(wr, 2) * Lz;
    const float4 ti = tab[xi.w];
    const float rc2 = R.rc2q, krf2 = R.krf2q;
    const int nch = W.nbcnt[slot] >> 3, nlj = W.nblj[slot], rowcap = R.maxnb >> 3;
    const uint4 *lp = reinterpret_cast<const uint4 *>(W.nblist + R.list_off + (int64_t)(b - R.blk0) * R.maxnb * kBlk);
    for (int c = part; c < nch; c += kParts) {
      const uint4 e = lp[list_row(chunk_row(c, nlj, rowcap), lane)];
      const uint32_t w[4] = {e.x, e.y, e.z, e.w};
      // an entry names one atom (chunks below nlj) or a three-atom site
      const int na = c < nlj ? 1 : 3;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int L0 = (int)((w[u >> 1] >> (16 * (u & 1))) & 0xffffu);
        for (int m = 0; m < na; ++m) {
        const int L = L0 + m;
        const int4 sj = st[L];
        const float4 tj = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(lds) + sj.w);
        const float4 xj = sxi[L];
        const float dx = (float)(sj.x - wx), dy = (float)(sj.y - wy), dz = (float)(sj.z - wz);
        const float r2 = qr2(dx, dy, dz);
        const bool in = r2 < rc2;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r2inv = rinv * rinv;
        const float sg = ti.y + tj.y;
        const float sr2 = sg * sg * r2inv;
        const float sr6 = sr2 * sr2 * sr2;
        const float ee = ti.z * tj.z;
        const float qq = ti.x * tj.x;
        // f(s) and f'(s) in the units of k_forces (coordinates in 2^-22 nm)
        const float fs = ee * sr6 * __builtin_fmaf(2.0f, sr6, -1.0f) * r2inv +
                         qq * __builtin_fmaf(rinv, r2inv, -krf2);
        const float fsp = r2inv * r2inv *
                          (ee * sr6 * __builtin_fmaf(-14.0f, sr6, 4.0f) - 1.5f * qq * rinv);
        const float ddx = (xj.x - ti4.x) * kQf, ddy = (xj.y - ti4.y) * kQf, ddz = (xj.z - ti4.z) * kQf;
        const float dot = __builtin_fmaf(dz, ddz, __builtin_fmaf(dy, ddy, dx * ddx));
        const float a = in ? fs : 0.0f, bq = in ? 2.0f * fsp * dot : 0.0f;
        gx = __builtin_fmaf(-a, ddx, __builtin_fmaf(-bq, dx, gx));
        gy = __builtin_fmaf(-a, ddy, __builtin_fmaf(-bq, dy, gy));
        gz = __builtin_fmaf(-a, ddz, __builtin_fmaf(-bq, dz, gz));
        }
      }
    }
  }
  __syncthreads();
  red[tid] = gx;
  red[kForceThreads + tid] = gy;
  red[2 * kForceThreads + tid] = gz;
  __syncthreads();
  if (part != 0 || !active) return;
  float sx = red[lane], sy = red[kForceThreads + lane], sz = red[2 * kForceThreads + lane];
#pragma unroll
  for (int q = 1; q < kParts; ++q) {
    sx += red[q * kBlk + lane];
    sy += red[kForceThreads + q * kBlk + lane];
    sz += red[2 * kForceThreads + q * kBlk + lane];
  }
  tfp[slot] = make_float4((float)((double)sx * kInvQ), (float)((double)sy * kInvQ),
                          (float)((double)sz * kInvQ), 0.0f);
}

// Bonded part of the tangent forces (one direction per launch): the FP64
// bonds and angles of each atom differentiated along the tangent on dual
// numbers, one thread per atom, added to the pair part k_tangent_forces
// stored (separate so that its dependent gathers and FP64 chains run over the
// whole chip instead of on one wave of each pair block).
__global__ __launch_bounds__(kBlk) void k_tangent_bonded(const RepInfo *__restrict__ info, Work W,
                                                         const int32_t *__restrict__ tile_rep,
                                                         const int32_t *__restrict__ tile_first, int nblk,
                                                         const int32_t *__restrict__ bt_start,
                                                         const BTerm *__restrict__ bterms, int dir) {
  const int b = xcd_tile(blockIdx.x, nblk);
  if (b < 0) return;
  const int tile = b / (kTile / kBlk);
  const RepInfo &R = info[tile_rep[tile]];
  // atoms in their original order, as in k_bonded_energy
  const int a = tile_first[tile] + (b % (kTile / kBlk)) * kBlk + (int)threadIdx.x;
  if (a >= R.n) return;
  const int slot = W.inv[R.uoff + a];
  const float4 *txp = W.tx + (size_t)dir * W.fstride;
  float4 *tfp = W.tf + (size_t)dir * W.fstride;
  double bx = 0.0, by = 0.0, bz = 0.0;
  const int t0 = bt_start[R.uoff + a], t1 = bt_start[R.uoff + a + 1];
  // an atom's position and tangent as three dual numbers (one gather each)
  auto load = [&](int atom, dual1 out[3]) {
    const int sl = W.inv[R.uoff + atom];
    const int4 xa = W.xq[sl];
    const float4 ta = txp[sl];
    out[0] = {(double)xa.x * kInvQ, (double)ta.x};
    out[1] = {(double)xa.y * kInvQ, (double)ta.y};
    out[2] = {(double)xa.z * kInvQ, (double)ta.z};
  };
  dual1 self[3];
  load(a, self);
  for (int t = t0; t < t1; ++t) {
    const BTerm T = bterms[t];
    dual1 A[3], B[3];
    load(T.a, A);
    if (T.kind != 0) load(T.b, B);
    if (T.kind == 0) {
      dual1 d[3] = {A[0] - self[0], A[1] - self[1], A[2] - self[2]};
      const dual1 rr = dsqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const dual1 g = (T.k * (rr - dual1{T.r0, 0.0})) / rr;
      bx += (g * d[0]).d;
      by += (g * d[1]).d;
      bz += (g * d[2]).d;
    } else {
      const dual1 *pa = T.kind == 1 ? self : A, *pc = T.kind == 1 ? A : self;
      const dual1 *pb = B;
      dual1 u[3], v[3];
      for (int k = 0; k < 3; ++k) {
        u[k] = pa[k] - pc[k];
        v[k] = pb[k] - pc[k];
      }
      const dual1 uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const dual1 vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      const dual1 uv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
      // reciprocals formed once (dual divisions cost two FP64 divisions each)
      const dual1 one = {1.0, 0.0};
      const dual1 inn = one / dsqrt(uu * vv), iuu = one / uu, ivv = one / vv;
      dual1 cs = uv * inn;
      if (cs.v > 1.0) cs = {1.0, 0.0};
      if (cs.v < -1.0) cs = {-1.0, 0.0};
      const double snv = sqrt(1.0 - cs.v * cs.v);
      const dual1 sn = snv > 1e-12 ? dsqrt(dual1{1.0, 0.0} - cs * cs) : dual1{1e-12, 0.0};
      const dual1 th = {acos(cs.v), -cs.d / (snv > 1e-12 ? snv : 1e-12)};
      const dual1 dv = (T.k * (th - dual1{T.r0, 0.0})) / sn;
      // end a: dv e1; vertex: -dv (e1 + e2) (a select, so the wave stays together)
      double f[3];
      for (int k = 0; k < 3; ++k) {
        const dual1 e1 = v[k] * inn - (cs * u[k]) * iuu;
        const dual1 e2 = u[k] * inn - (cs * v[k]) * ivv;
        const double fe = (dv * e1).d, fv = -(dv * (e1 + e2)).d;
        f[k] = T.kind == 1 ? fe : fv;
      }
      bx += f[0];
      by += f[1];
      bz += f[2];
    }
  }
  if (t1 > t0) {
    float4 g = tfp[slot];
    g.x = (float)((double)g.x + bx);
    g.y = (float)((double)g.y + by);
    g.z = (float)((double)g.z + bz);
    tfp[slot] = g;
  }
}


// ---------------------------------------------------------------------------
// collective variable of the bias
// ---------------------------------------------------------------------------

// The switched contact function C~ = C(u) sw(r), u = (r/r0)^2, and (dC~/dr)/r
// at squared distance r2 (nm^2), in FP32.
__device__ __forceinline__ void contact_tilde(float r2, float ir02, float iw, float rs, float rs2, float rc2,
                                              float &ct, float &dct_r) {
  const float rinv = __builtin_amdgcn_rsqf(r2);
  // C(u) and dC/du
  const float u = r2 * ir02, u2 = u * u;
  const float num = 1.0f + u + u2;
  const float den = num + u2 * u + u2 * u2;
  const float iden = __builtin_amdgcn_rcpf(den);
  const float c = num * iden;
  const float dnum = __builtin_fmaf(2.0f, u, 1.0f);
  const float dden = dnum + u2 * __builtin_fmaf(4.0f, u, 3.0f);
  const float dcdu = (dnum - c * dden) * iden;
  // quintic switch on r
  const float rr = r2 * rinv;
  const float t = (rr - rs) * iw;
  const float t2 = t * t;
  const float swp = 1.0f - t2 * t * __builtin_fmaf(t, __builtin_fmaf(6.0f, t, -15.0f), 10.0f);
  const float dswp = -30.0f * t2 * (1.0f - t) * (1.0f - t) * iw;
  const bool inner = r2 <= rs2, outer = r2 >= rc2;
  const float sw = inner ? 1.0f : (outer ? 0.0f : swp);
  const float dsw = (inner || outer) ? 0.0f : dswp;
  ct = c * sw;
  dct_r = 2.0f * ir02 * dcdu * sw + c * dsw * rinv;
}

// Contact-map CV (supplement, "Collective coordinate"), one wave per tile of
// 64 rows i x 64 columns j of one replica's solute:
//   z = sum_{i<j, j-i>min_sep} (C~(r_ij) - C~f_ij)^2,
//   dz/dx_i = -sum_j 2 (C~(r_ij) - C~f_ij) (dC~/dr)/r (x_j - x_i),
// with C = (1+u+u^2)/(1+u+u^2+u^3+u^4), u = (r/r0)^2, times a quintic switch
// from 1 at r_s to 0 at r_c.  Only the tiles on and above the diagonal are
// launched, those above it first, two waves per tile, each wave taking half of
// the tile's 64 column steps; the two halves are added in wave order.  A tile
// above the diagonal evaluates each of its pairs once and stores the row sums
// and the column sums (as the partials the mirrored tile below the diagonal
// would give); a diagonal tile visits both orderings of each pair, each
// contributing to its own row's gradient, and z takes its pairs j > i.  The
// column-tile partials are reduced in a fixed order by k_cv_reduce.
constexpr int kCvHalf = kCvTile / 2;  // column steps per wave
__global__ __launch_bounds__(2 * kCvTile) void k_cv_pairs(const RepInfo *__restrict__ info, Work W,
                                                          const float *__restrict__ cmap,
                                                          const float *__restrict__ cskew) {
  __shared__ int4 s_x[kCvTile];
  __shared__ float4 s_g[2][kCvTile];  // wave 1's row and column sums
  __shared__ double s_z;
  const int r = blockIdx.y;
  const RepInfo &R = info[r];
  if (R.bias != VP_BIAS_CONTACT && R.bias != VP_BIAS_RMD_CONTACT) return;
  const int nt = R.cv_blocks, noff = nt * (nt - 1) / 2;
  if ((int)blockIdx.x >= noff + nt) return;
  int it, jc;
  if ((int)blockIdx.x < noff) {  // the b-th tile above the diagonal, row tiles in order
    int b = blockIdx.x;
    it = 0;
    while (b >= nt - 1 - it) {
      b -= nt - 1 - it;
      ++it;
    }
    jc = it + 1 + b;
  } else {
    it = jc = (int)blockIdx.x - noff;
  }
  const int lane = threadIdx.x & (kCvTile - 1), wv = threadIdx.x / kCvTile, ns = R.ns;
  const int i = it * kCvTile + lane;
  const int j0 = jc * kCvTile, jn = min(kCvTile, ns - j0);
  if (wv == 0) s_x[lane] = lane < jn ? W.xq[W.inv[R.uoff + j0 + lane]] : make_int4(0, 0, 0, 0);
  const bool row = i < ns;
  const int4 xi = row ? W.xq[W.inv[R.uoff + i]] : make_int4(0, 0, 0, 0);
  __syncthreads();
  const float ir02 = R.cinv_r02, iw = R.cinv_w, rs = R.crs, rs2 = R.crs2, rc2 = R.crc2;
  const int msep = R.min_sep;
  float gx = 0.0f, gy = 0.0f, gz = 0.0f, hx = 0.0f, hy = 0.0f, hz = 0.0f;
  double zacc = 0.0;
  const int k0 = wv * kCvHalf;
  if (jc > it) {
    // Every pair once: at step k lane l takes column (l + k) mod 64, adds the
    // pair's gradient to its row (i) and to a column sum (j, opposite sign);
    // the column sums move one lane down after each step.  The reference
    // values come from the map's copy in the same diagonal order (one
    // coalesced load per step).
    const float *sk = cskew + R.cskew_off + ((int64_t)it * nt + jc) * kCvTile * kCvTile + lane;
    const int nxt = (lane + 1) & (kCvTile - 1);
    for (int k = k0; k < k0 + kCvHalf; ++k) {
      const int c = (lane + k) & (kCvTile - 1);
      const int j = j0 + c;
      const int4 xj = s_x[c];
      const float dx = (float)(xj.x - xi.x) * kInvQf, dy = (float)(xj.y - xi.y) * kInvQf,
                  dz = (float)(xj.z - xi.z) * kInvQf;
      const float r2 = qr2(dx, dy, dz);
      const bool valid = row && c < jn && j - i > msep;
      const float cref = sk[k * kCvTile];
      if (__ballot(valid && r2 < rc2) != 0ull) {
        float ct, dct_r;
        contact_tilde(r2, ir02, iw, rs, rs2, rc2, ct, dct_r);
        const float diff = ct - cref;
        const float coef = valid ? 2.0f * diff * dct_r : 0.0f;
        gx = __builtin_fmaf(-coef, dx, gx);
        gy = __builtin_fmaf(-coef, dy, gy);
        gz = __builtin_fmaf(-coef, dz, gz);
        hx = __builtin_fmaf(coef, dx, hx);
        hy = __builtin_fmaf(coef, dy, hy);
        hz = __builtin_fmaf(coef, dz, hz);
        if (valid) zacc += (double)diff * (double)diff;
      } else if (valid) {
        // every pair of this step is beyond the switch: C~ is 0 there
        zacc += (double)cref * (double)cref;
      }
      hx = __shfl(hx, nxt, kCvTile);
      hy = __shfl(hy, nxt, kCvTile);
      hz = __shfl(hz, nxt, kCvTile);
    }
    // after its 32 steps wave 1's lane l holds column l's sum, wave 0's
    // column (l + 32) mod 64's: move those by half a wave
    if (wv == 0) {
      const int half = (lane + kCvHalf) & (kCvTile - 1);
      hx = __shfl(hx, half, kCvTile);
      hy = __shfl(hy, half, kCvTile);
      hz = __shfl(hz, half, kCvTile);
    }
  } else {
    // diagonal tile: both orderings of each pair, each adding to its own row
    const float *cf = cmap + R.cmap_off + (int64_t)j0 * ns + (row ? i : 0);
    for (int k = k0; k < min(jn, k0 + kCvHalf); ++k) {
      const int j = j0 + k;
      const int4 xj = s_x[k];
      const float dx = (float)(xj.x - xi.x) * kInvQf, dy = (float)(xj.y - xi.y) * kInvQf,
                  dz = (float)(xj.z - xi.z) * kInvQf;
      const float r2 = qr2(dx, dy, dz);
      const bool valid = row && abs(j - i) > msep;
      const float cref = cf[(int64_t)k * ns];
      if (__ballot(row && r2 < rc2) == 0ull) {
        // every row of the tile is beyond the switch: C~ and its derivative
        // are exactly 0 there, so the gradient gains nothing and z only the
        // reference term (the same bits as the full evaluation below)
        const float diff = 0.0f - cref;
        if (valid && j > i) zacc += (double)diff * (double)diff;
        continue;
      }
      float ct, dct_r;
      contact_tilde(r2, ir02, iw, rs, rs2, rc2, ct, dct_r);
      const float diff = ct - cref;
      const float coef = valid ? 2.0f * diff * dct_r : 0.0f;
      gx = __builtin_fmaf(-coef, dx, gx);
      gy = __builtin_fmaf(-coef, dy, gy);
      gz = __builtin_fmaf(-coef, dz, gz);
      if (valid && j > i) zacc += (double)diff * (double)diff;
    }
  }
  const double zs = wave_sum(zacc);
  if (wv == 1) {
    s_g[0][lane] = make_float4(gx, gy, gz, 0.0f);
    s_g[1][lane] = make_float4(hx, hy, hz, 0.0f);
    if (lane == 0) s_z = zs;
  }
  __syncthreads();
  if (wv == 1) return;
  const float4 g1 = s_g[0][lane];
  W.gtile[(R.cvt_off + (int64_t)jc * nt + it) * kCvTile + lane] =
      make_float4(gx + g1.x, gy + g1.y, gz + g1.z, 0.0f);
  if (jc > it) {
    const float4 h1 = s_g[1][lane];
    W.gtile[(R.cvt_off + (int64_t)it * nt + jc) * kCvTile + lane] =
        make_float4(hx + h1.x, hy + h1.y, hz + h1.z, 0.0f);
  }
  if (lane == 0) {
    W.ztile[R.cvt_off + (int64_t)it * nt + jc] = zs + s_z;
    if (jc > it) W.ztile[R.cvt_off + (int64_t)jc * nt + it] = 0.0;  // the mirrored tile's share
  }
}

// Tangent of the contact-map gradient, one wave per 64 x 64 tile as in
// k_cv_pairs: for both directions p,
//   d(dz/dx_i)[xi] = -sum_j 2 [ (phi'^2 + diff phi'') rdot e
//                               + diff phi' (delta - e rdot) / r ],
// with phi = C~(r), e = (x_j - x_i)/r, delta = xi_j - xi_i, rdot = e . delta.
__global__ __launch_bounds__(kCvTile) void k_cv_tangent_pairs(const RepInfo *__restrict__ info,
                                                              Work W,
                                                              const float *__restrict__ cmap) {
  __shared__ int4 s_x[kCvTile];
  __shared__ float4 s_t[2][kCvTile];
  const int r = blockIdx.y;
  const RepInfo &R = info[r];
  if (R.bias != VP_BIAS_CONTACT && R.bias != VP_BIAS_RMD_CONTACT) return;
  const int nt = R.cv_blocks;
  if ((int)blockIdx.x >= nt * nt) return;
  const int it = blockIdx.x / nt, jc = blockIdx.x % nt;
  const int lane = threadIdx.x, ns = R.ns;
  const int i = it * kCvTile + lane;
  const int j0 = jc * kCvTile, jn = min(kCvTile, ns - j0);
  if (lane < jn) {
    const int sl = W.inv[R.uoff + j0 + lane];
    s_x[lane] = W.xq[sl];
    s_t[0][lane] = W.tx[sl];
    s_t[1][lane] = W.tx[W.fstride + sl];
  }
  const bool row = i < ns;
  int4 xi = make_int4(0, 0, 0, 0);
  float4 t0 = make_float4(0.f, 0.f, 0.f, 0.f), t1 = t0;
  if (row) {
    const int sl = W.inv[R.uoff + i];
    xi = W.xq[sl];
    t0 = W.tx[sl];
    t1 = W.tx[W.fstride + sl];
  }
  __syncthreads();
  const float *cf = cmap + R.cmap_off + (int64_t)j0 * ns + (row ? i : 0);
  const float ir02 = R.cinv_r02, iw = R.cinv_w, rs = R.crs, rs2 = R.crs2, rc2 = R.crc2;
  const int msep = R.min_sep;
  float ax = 0.f, ay = 0.f, az = 0.f, bx = 0.f, by = 0.f, bz = 0.f;
  for (int k = 0; k < jn; ++k) {
    const int j = j0 + k;
    const int4 xj = s_x[k];
    const float dx = (float)(xj.x - xi.x) * kInvQf, dy = (float)(xj.y - xi.y) * kInvQf,
                dz = (float)(xj.z - xi.z) * kInvQf;
    const float r2 = qr2(dx, dy, dz);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rr = r2 * rinv;
    // C(u), C'(u), C''(u)
    const float u = r2 * ir02, u2 = u * u;
    const float num = 1.0f + u + u2;
    const float den = num + u2 * u + u2 * u2;
    const float iden = __builtin_amdgcn_rcpf(den);
    const float c = num * iden;
    const float dnum = __builtin_fmaf(2.0f, u, 1.0f);
    const float dden = dnum + u2 * __builtin_fmaf(4.0f, u, 3.0f);
    const float d2den = 2.0f + u * __builtin_fmaf(12.0f, u, 6.0f);
    const float c1 = (dnum - c * dden) * iden;
    const float c2 = (2.0f - 2.0f * c1 * dden - c * d2den) * iden;
    // r-derivatives of C: u_r = 2 r / r0^2, u_rr = 2 / r0^2
    const float ur = 2.0f * rr * ir02;
    const float cr = c1 * ur, crr = c2 * ur * ur + c1 * 2.0f * ir02;
    // quintic switch and its r-derivatives
    const float t = (rr - rs) * iw;
    const float omt = 1.0f - t;
    const float swp = 1.0f - t * t * t * __builtin_fmaf(t, __builtin_fmaf(6.0f, t, -15.0f), 10.0f);
    const float dswp = -30.0f * t * t * omt * omt * iw;
    const float d2swp = -60.0f * t * omt * (1.0f - 2.0f * t) * iw * iw;
    const bool inner = r2 <= rs2, outer = r2 >= rc2;
    const float sw = inner ? 1.0f : (outer ? 0.0f : swp);
    const float sr = (inner || outer) ? 0.0f : dswp;
    const float srr = (inner || outer) ? 0.0f : d2swp;
    const float ph = c * sw, ph1 = cr * sw + c * sr, ph2 = crr * sw + 2.0f * cr * sr + c * srr;
    const bool valid = row && abs(j - i) > msep;
    const float diff = ph - cf[(int64_t)k * ns];
    const float A = valid ? ph1 * ph1 + diff * ph2 : 0.0f;
    const float B = valid ? diff * ph1 * rinv : 0.0f;
    // unit vector only for contributing pairs (i == j would give 0 * inf)
    const float ri = valid ? rinv : 0.0f;
    const float ex = dx * ri, ey = dy * ri, ez = dz * ri;
    {
      const float4 tj = s_t[0][k];
      const float hx = tj.x - t0.x, hy = tj.y - t0.y, hz = tj.z - t0.z;
      const float rd = __builtin_fmaf(ez, hz, __builtin_fmaf(ey, hy, ex * hx));
      const float q = 2.0f * (A - B) * rd;  // coefficient of e
      ax = __builtin_fmaf(-q, ex, __builtin_fmaf(-2.0f * B, hx, ax));
      ay = __builtin_fmaf(-q, ey, __builtin_fmaf(-2.0f * B, hy, ay));
      az = __builtin_fmaf(-q, ez, __builtin_fmaf(-2.0f * B, hz, az));
    }
    {
      const float4 tj = s_t[1][k];
      const float hx = tj.x - t1.x, hy = tj.y - t1.y, hz = tj.z - t1.z;
      const float rd = __builtin_fmaf(ez, hz, __builtin_fmaf(ey, hy, ex * hx));
      const float q = 2.0f * (A - B) * rd;
      bx = __builtin_fmaf(-q, ex, __builtin_fmaf(-2.0f * B, hx, bx));
      by = __builtin_fmaf(-q, ey, __builtin_fmaf(-2.0f * B, hy, by));
      bz = __builtin_fmaf(-q, ez, __builtin_fmaf(-2.0f * B, hz, bz));
    }
  }
  const int64_t o = (R.cvt_off + (int64_t)jc * nt + it) * kCvTile + lane;
  W.tgtile[o] = make_float4(ax, ay, az, 0.0f);
  W.tgtile[W.cvstride + o] = make_float4(bx, by, bz, 0.0f);
}

// Row tile it of a contact-map replica: dz/dx_i summed over the column tiles
// in order, sum_i |dz/dx_i|^2/(gamma_i m_i) and the tile's part of z.
// With TAN, also the tangents: (d grad z)[xi_p] summed over the column tiles,
// dz/dtheta_p = sum_i g_i . xi_p,i and sum_i 2 g_i . (d g_i)[xi_p] / (gamma_i m_i).
// When every replica carries a contact-map bias k_cv is not launched, and this
// kernel advances the step counter instead (inc_step; no block reads it).
template <bool TAN>
__global__ __launch_bounds__(kCvTile) void k_cv_reduce(const RepInfo *__restrict__ info, Work W,
                                                       const double *__restrict__ igm0, int inc_step,
                                                       long long *__restrict__ step) {
  if (inc_step && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *step += 1;
  const int r = blockIdx.y;
  const RepInfo &R = info[r];
  if (R.bias != VP_BIAS_CONTACT && R.bias != VP_BIAS_RMD_CONTACT) return;
  const int nt = R.cv_blocks, it = blockIdx.x;
  if (it >= nt) return;
  const int lane = threadIdx.x, i = it * kCvTile + lane;
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
  for (int jc = 0; jc < nt; ++jc) {
    const float4 g = W.gtile[(R.cvt_off + (int64_t)jc * nt + it) * kCvTile + lane];
    gx += g.x;
    gy += g.y;
    gz += g.z;
  }
  double gq = 0.0;
  if (i < R.ns) {
    W.g[R.sol_off + i] = make_float4(gx, gy, gz, 0.0f);
    gq = ((double)gx * gx + (double)gy * gy + (double)gz * gz) * igm0[R.uoff + i];
  }
  const double gs = wave_sum(gq);
  if (lane == 0) {
    double z = 0.0;
    for (int jc = 0; jc < nt; ++jc) z += W.ztile[R.cvt_off + (int64_t)it * nt + jc];
    W.zpart[(size_t)r * kMaxCvBlocks + it] = z;
    W.gpart[(size_t)r * kMaxCvBlocks + it] = gs;
  }
  if (TAN) {
    for (int d = 0; d < 2; ++d) {
      float hx = 0.0f, hy = 0.0f, hz = 0.0f;
      for (int jc = 0; jc < nt; ++jc) {
        const float4 h = W.tgtile[d * W.cvstride + (R.cvt_off + (int64_t)jc * nt + it) * kCvTile + lane];
        hx += h.x;
        hy += h.y;
        hz += h.z;
      }
      double zd = 0.0, gd = 0.0;
      if (i < R.ns) {
        W.tg[d * W.solstride + R.sol_off + i] = make_float4(hx, hy, hz, 0.0f);
        const float4 t = W.tx[d * W.fstride + W.inv[R.uoff + i]];
        zd = (double)gx * t.x + (double)gy * t.y + (double)gz * t.z;
        gd = 2.0 * ((double)gx * hx + (double)gy * hy + (double)gz * hz) * igm0[R.uoff + i];
      }
      zd = wave_sum(zd);
      gd = wave_sum(gd);
      if (lane == 0) {
        W.tzpart[((size_t)r * kMaxCvBlocks + it) * 2 + d] = zd;
        W.tgpart[((size_t)r * kMaxCvBlocks + it) * 2 + d] = gd;
      }
    }
  }
}

// The other CV kinds, one workgroup per replica: radius of gyration (FP64 on
// unwrapped coordinates), constant force; also advances the step counter.
// With tan != 0, also the tangents of the radius of gyration (g_i =
// m_i (x_i - X_cm) / (M Rg)): dz = sum_i g_i . xi_i and
// (d g_i)[xi] = m_i (xi_i - Xi_cm) / (M Rg) - g_i dz / Rg; zero for the other
// kinds handled here.
__global__ __launch_bounds__(kCvBlock) void k_cv(const RepInfo *__restrict__ info, Work W,
                                                 const double *__restrict__ igm0,
                                                 const double *__restrict__ mass0,
                                                 const float4 *__restrict__ cforce, int inc_step,
                                                 long long *__restrict__ step, int tan) {
  extern __shared__ int4 s_x[];  // solute positions of this replica
  __shared__ double s_red[kCvBlock / 64];
  __shared__ double s_cm[5];
  const int r = blockIdx.x;
  const RepInfo &R = info[r];
  const int tid = threadIdx.x;
  const int ns = R.ns;
  if (R.bias == VP_BIAS_RG || R.bias == VP_BIAS_CONST || R.bias == VP_BIAS_NONE) {
    double zacc = 0.0, gq = 0.0;
    if (R.bias == VP_BIAS_RG) {
      // mass-weighted radius of gyration on unwrapped coordinates (FP64)
      double m = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
      for (int a = tid; a < ns; a += kCvBlock) {
        const int4 x = W.xq[W.inv[R.uoff + a]];
        s_x[a] = x;
        const double ma = mass0[R.uoff + a];
        m += ma;
        cx += ma * (double)x.x * kInvQ;
        cy += ma * (double)x.y * kInvQ;
        cz += ma * (double)x.z * kInvQ;
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
        const int4 x = s_x[a];
        const double d0 = (double)x.x * kInvQ - s_cm[0], d1 = (double)x.y * kInvQ - s_cm[1],
                     d2 = (double)x.z * kInvQ - s_cm[2];
        q += mass0[R.uoff + a] * (d0 * d0 + d1 * d1 + d2 * d2);
      }
      double Q = block_sum<kCvBlock>(q, s_red);
      if (tid == 0) s_cm[3] = sqrt(Q / M);  // Rg
      __syncthreads();
      const double rg = s_cm[3];
      for (int a = tid; a < ns; a += kCvBlock) {
        const int4 x = s_x[a];
        const double w = mass0[R.uoff + a] / (M * rg);
        const double g0 = w * ((double)x.x * kInvQ - s_cm[0]), g1 = w * ((double)x.y * kInvQ - s_cm[1]),
                     g2 = w * ((double)x.z * kInvQ - s_cm[2]);
        W.g[R.sol_off + a] = make_float4((float)g0, (float)g1, (float)g2, 0.0f);
        gq += (g0 * g0 + g1 * g1 + g2 * g2) * igm0[R.uoff + a];
      }
      zacc = (tid == 0) ? rg : 0.0;
      if (tan) {
        for (int d = 0; d < 2; ++d) {
          // centre of mass of the tangent and dz = sum_i g_i . xi_i
          double tm[3] = {0.0, 0.0, 0.0}, zd = 0.0;
          for (int a = tid; a < ns; a += kCvBlock) {
            const float4 t = W.tx[d * W.fstride + W.inv[R.uoff + a]];
            const double ma = mass0[R.uoff + a];
            tm[0] += ma * t.x;
            tm[1] += ma * t.y;
            tm[2] += ma * t.z;
            const float4 g = W.g[R.sol_off + a];
            zd += (double)g.x * t.x + (double)g.y * t.y + (double)g.z * t.z;
          }
          const double TX = block_sum<kCvBlock>(tm[0], s_red), TY = block_sum<kCvBlock>(tm[1], s_red),
                       TZ = block_sum<kCvBlock>(tm[2], s_red), ZD = block_sum<kCvBlock>(zd, s_red);
          if (tid == 0) {
            s_cm[0] = TX / M;
            s_cm[1] = TY / M;
            s_cm[2] = TZ / M;
            s_cm[3] = ZD;
          }
          __syncthreads();
          const double tcx = s_cm[0], tcy = s_cm[1], tcz = s_cm[2], zdot = s_cm[3];
          double gd = 0.0;
          for (int a = tid; a < ns; a += kCvBlock) {
            const float4 t = W.tx[d * W.fstride + W.inv[R.uoff + a]];
            const float4 g = W.g[R.sol_off + a];
            const double w = mass0[R.uoff + a] / (M * rg);
            const double h0 = w * ((double)t.x - tcx) - (double)g.x * zdot / rg;
            const double h1 = w * ((double)t.y - tcy) - (double)g.y * zdot / rg;
            const double h2 = w * ((double)t.z - tcz) - (double)g.z * zdot / rg;
            W.tg[d * W.solstride + R.sol_off + a] = make_float4((float)h0, (float)h1, (float)h2, 0.0f);
            gd += 2.0 * ((double)g.x * h0 + (double)g.y * h1 + (double)g.z * h2) * igm0[R.uoff + a];
          }
          const double GD = block_sum<kCvBlock>(gd, s_red);
          if (tid == 0) {
            W.tzpart[(size_t)r * kMaxCvBlocks * 2 + d] = zdot;
            W.tgpart[(size_t)r * kMaxCvBlocks * 2 + d] = GD;
          }
          __syncthreads();
        }
      }
    } else if (R.bias == VP_BIAS_CONST) {
      // F0 = grad z with z = sum_i F0_i . x_i (U_b = -z)
      for (int a = tid; a < ns; a += kCvBlock) {
        const float4 f = cforce[R.sol_off + a];
        W.g[R.sol_off + a] = f;
        gq += ((double)f.x * f.x + (double)f.y * f.y + (double)f.z * f.z) * igm0[R.uoff + a];
        const int4 x = W.xq[W.inv[R.uoff + a]];
        zacc += (double)f.x * ((double)x.x * kInvQ) + (double)f.y * ((double)x.y * kInvQ) +
                (double)f.z * ((double)x.z * kInvQ);
      }
    }
    const double zs = block_sum<kCvBlock>(zacc, s_red);
    const double gs = block_sum<kCvBlock>(gq, s_red);
    if (tid == 0) {
      W.zpart[(size_t)r * kMaxCvBlocks] = zs;
      W.gpart[(size_t)r * kMaxCvBlocks] = gs;
      if (tan && R.bias != VP_BIAS_RG)
        for (int d = 0; d < 2; ++d) {
          W.tzpart[(size_t)r * kMaxCvBlocks * 2 + d] = 0.0;
          W.tgpart[(size_t)r * kMaxCvBlocks * 2 + d] = 0.0;
        }
    }
    if (tan && R.bias == VP_BIAS_CONST)
      for (int a = tid; a < ns; a += kCvBlock)
        for (int d = 0; d < 2; ++d) W.tg[d * W.solstride + R.sol_off + a] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if (inc_step && r == 0 && tid == 0) *step += 1;
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
  if (W.flags[r] & VP_REPLICA_LIST_OVERFLOW) f0 = f1 = f2 = NAN;  // pairs were left out
  float *o = f_user + 3ll * (R.uoff + a);
  o[0] = (float)f0;
  o[1] = (float)f1;
  o[2] = (float)f2;
}

// Directional derivative of the total force along the two tangents held in
// W.tx, the parameters fixed: out [2][users][3] =
//   -H_U xi_p + (dc/dz dz_p) g + c (d g)[xi_p]   (bias terms on solute atoms).
__global__ __launch_bounds__(kBlock) void k_force_dir_out(const RepInfo *__restrict__ info,
                                                          const RepState *__restrict__ state, Work W,
                                                          const int32_t *__restrict__ tile_rep,
                                                          const int32_t *__restrict__ tile_first,
                                                          int ntiles, double t, int64_t users,
                                                          float *__restrict__ out) {
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
  double dcdz, dcdth[2];
  bias_coef_deriv(R, z, S.z0, t, false, dcdz, dcdth);
  const int a = W.orig[slot];
  for (int d = 0; d < 2; ++d) {
    double zd = 0.0;
    for (int b = 0; b < R.cv_blocks; ++b) zd += W.tzpart[((size_t)r * kMaxCvBlocks + b) * 2 + d];
    const float4 h = W.tf[d * W.fstride + slot];
    double f0 = h.x, f1 = h.y, f2 = h.z;
    if (a < R.ns) {
      const float4 g = W.g[R.sol_off + a];
      const float4 dg = W.tg[d * W.solstride + R.sol_off + a];
      const double cd = dcdz * zd;
      f0 += cd * g.x + c * dg.x;
      f1 += cd * g.y + c * dg.y;
      f2 += cd * g.z + c * dg.z;
    }
    float *o = out + (size_t)d * 3 * users + 3ll * (R.uoff + a);
    o[0] = (float)f0;
    o[1] = (float)f1;
    o[2] = (float)f2;
  }
}

// Tangent directions given in user order ([2][users][3] FP32) into slot order.
__global__ __launch_bounds__(kBlock) void k_scatter_dirs(const RepInfo *__restrict__ info, Work W,
                                                         const int32_t *__restrict__ tile_rep,
                                                         const int32_t *__restrict__ tile_first,
                                                         int ntiles, int64_t users,
                                                         const float *__restrict__ dx) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  const int p = tile_first[tile] + threadIdx.x;
  const int slot = R.off + p;
  for (int d = 0; d < 2; ++d) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p < R.n) {
      const float *u = dx + (size_t)d * 3 * users + 3ll * (R.uoff + W.orig[slot]);
      v = make_float4(u[0], u[1], u[2], 0.0f);
    }
    W.tx[d * W.fstride + slot] = v;
  }
}

// vp_forces energy table: the VP_E_* columns of every replica
__global__ void k_energy_out(const RepInfo *__restrict__ info, const RepState *__restrict__ state,
                             Work W, double t, double *__restrict__ e_out) {
  const int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  const RepInfo &R = info[r];
  double *o = e_out + VP_E_COUNT * (size_t)r;
  energy_columns(R, W, r, state[r].z0, state[r].z_m, t, o);
  o[VP_E_STATUS] = (W.flags[r] & VP_REPLICA_LIST_OVERFLOW) ? (double)VP_REPLICA_LIST_OVERFLOW : 0.0;
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
    const float rr = sqrtf(qr2(dx, dy, dz));
    float dc;
    v = contact_value(rr, r0, rs, rc, dc);
  }
  out[k] = v;
}

// A contact map's copy per 64 x 64 tile in diagonal order:
// skew[tile][k][l] = C~f(row 64 it + l, column 64 jc + (l + k) mod 64), zero
// outside the map; one wave per tile.
__global__ __launch_bounds__(kCvTile) void k_cv_skew(const float *__restrict__ cmap, int ns,
                                                     float *__restrict__ skew) {
  const int nt = (ns + kCvTile - 1) / kCvTile;
  const int it = blockIdx.x / nt, jc = blockIdx.x % nt, l = threadIdx.x;
  const int i = it * kCvTile + l;
  float *o = skew + (int64_t)blockIdx.x * kCvTile * kCvTile + l;
  for (int k = 0; k < kCvTile; ++k) {
    const int j = jc * kCvTile + ((l + k) & (kCvTile - 1));
    o[k * kCvTile] = (i < ns && j < ns) ? cmap[(int64_t)j * ns + i] : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int xcd_grid(int nb) { return 8 * ((nb + 7) / 8); }

size_t force_lds_bytes(const vp_system *s) {
  size_t stage = sizeof(int4) * ((size_t)(s->stage_cap_max + kStageDummies) + (size_t)(s->ntypes_max + 1));
  // logical partial sums: forces FP32 [3][kLogicalParts][64]
  size_t red = sizeof(float) * 3 * kLogicalParts * kBlk;
  return stage > red ? stage : red;
}

size_t energy_lds_bytes(const vp_system *s) {
  size_t stage = sizeof(int4) * ((size_t)(s->stage_cap_max + kStageDummies) + (size_t)(s->ntypes_max + 1));
  size_t red = sizeof(double) * 8 * kParts * kBlk;  // [8 values][kParts][64] FP64
  return stage > red ? stage : red;
}

// the tile shapes the force kernel is built for: (waves per block, entries per batch)
const ForceShape kForceShapes[kNumForceShapes] = {{8, 4}, {8, 2}, {4, 4}, {16, 2}};

template <int P, int U, int M>
static hipError_t set_lds(int lds) {
  return hipFuncSetAttribute((const void *)k_forces<P, U, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds);
}

hipError_t prepare_forces(const vp_system *s) {
  const int lds = (int)force_lds_bytes(s);
  hipError_t e = hipSuccess;
  for (hipError_t x : {set_lds<8, 4, 1>(lds), set_lds<8, 2, 1>(lds), set_lds<4, 4, 1>(lds),
                       set_lds<16, 2, 1>(lds)})
    if (x != hipSuccess) e = x;
  return e;
}

hipError_t prepare_energies(const vp_system *s) {
  const int lds = (int)energy_lds_bytes(s);
  hipError_t e = hipFuncSetAttribute((const void *)k_pair_energy<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipError_t e2 = hipFuncSetAttribute((const void *)k_pair_energy<true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  return e != hipSuccess ? e : e2;
}

void launch_native_map(const float *xf, int ns, int min_sep, float r0, float rs, float rc,
                       float *out, hipStream_t st) {
  int64_t n = (int64_t)ns * ns;
  hipLaunchKernelGGL(k_native_map, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xf, ns,
                     min_sep, r0, rs, rc, out);
}

// Reads a buffer (n int4 values) so that the last-level cache no longer holds
// what the launch before it read; the sum is stored only if it takes a value
// the data never gives in practice, so the loads are not removed.
__global__ __launch_bounds__(256) void k_touch(const int4 *__restrict__ p, int64_t n, int *__restrict__ sink) {
  int acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int4 v = p[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x5eed1e55) *sink = acc;
}

void launch_touch(const void *p, size_t bytes, int *sink, hipStream_t st) {
  hipLaunchKernelGGL(k_touch, dim3(2048), dim3(256), 0, st, (const int4 *)p, (int64_t)(bytes / sizeof(int4)), sink);
}

void launch_cv_skew(const float *cmap, int ns, float *skew, hipStream_t st) {
  const int nt = (ns + kCvTile - 1) / kCvTile;
  hipLaunchKernelGGL(k_cv_skew, dim3(nt * nt), dim3(kCvTile), 0, st, cmap, ns, skew);
}

template <int P, int U, int M>
static void launch_forces_t(vp_system *s, Work &W, const int32_t *blist, int nblk, hipStream_t st) {
  hipLaunchKernelGGL((k_forces<P, U, M>), dim3(xcd_grid(nblk)), dim3(64 * P), force_lds_bytes(s), st,
                     s->info, W, s->tile_rep, s->tile_first, blist, nblk, s->types, s->stage_cap_max + kStageDummies);
}

void launch_forces_shape(vp_system *s, Work &W, int shape, const int32_t *blist, int nblk, hipStream_t st) {
  switch (shape) {
    case 0: launch_forces_t<8, 4, 1>(s, W, blist, nblk, st); break;
    case 1: launch_forces_t<8, 2, 1>(s, W, blist, nblk, st); break;
    case 2: launch_forces_t<4, 4, 1>(s, W, blist, nblk, st); break;
    default: launch_forces_t<16, 2, 1>(s, W, blist, nblk, st); break;
  }
}

void launch_pair_forces(vp_system *s, Work &W, hipStream_t st) {
  if (s->force_plan.empty()) {
    launch_forces_shape(s, W, s->force_shape, nullptr, s->n_blocks, st);
    return;
  }
  for (const auto &g : s->force_plan) launch_forces_shape(s, W, g.shape, g.blist, g.nblk, st);
}

void launch_bonded(vp_system *s, Work &W, hipStream_t st) {
  const int nwa = (s->n_bf_atoms + kBondedThreads - 1) / kBondedThreads;
  const int nwg = (s->n_bgroups + kBondedThreads - 1) / kBondedThreads;
  if (nwa + nwg == 0) return;
  hipLaunchKernelGGL(k_bonded_forces, dim3(xcd_grid(nwa) + xcd_grid(nwg)), dim3(kBondedThreads), 0, st, W,
                     s->bf_atoms, s->bf_start, s->bf_terms, s->n_bf_atoms, nwa, s->bgroups, s->n_bgroups, nwg);
}

void launch_forces(vp_system *s, Work &W, hipStream_t st) {
  launch_pair_forces(s, W, st);
  launch_bonded(s, W, st);
}

void launch_energies(vp_system *s, Work &W, bool gated, hipStream_t st) {
  const size_t lds = energy_lds_bytes(s);
  const int nout = s->opt.nst_out > 0 ? s->opt.nst_out : 1;
  if (gated) {
    hipLaunchKernelGGL(k_pair_energy<true>, dim3(xcd_grid(s->n_blocks)), dim3(kForceThreads), lds, st,
                       s->info, W, s->tile_rep, s->tile_first, s->n_blocks, s->types, s->stage_cap_max + kStageDummies,
                       s->step, nout);
    hipLaunchKernelGGL((k_bonded_energy<true>), dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info, W,
                       s->tile_rep, s->tile_first, s->n_blocks, s->bt_start, s->bterms, s->step, nout);
  } else {
    hipLaunchKernelGGL(k_pair_energy<false>, dim3(xcd_grid(s->n_blocks)), dim3(kForceThreads), lds, st,
                       s->info, W, s->tile_rep, s->tile_first, s->n_blocks, s->types, s->stage_cap_max + kStageDummies,
                       s->step, nout);
    hipLaunchKernelGGL((k_bonded_energy<false>), dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info, W,
                       s->tile_rep, s->tile_first, s->n_blocks, s->bt_start, s->bterms, s->step, nout);
  }
}

void launch_cv(vp_system *s, Work &W, int inc_step, hipStream_t st, bool tan) {
  int nt = 0, nsmax = 1;
  bool any_single = false, any_other = false;
  for (const RepInfo &R : s->info_h) {
    if (R.bias == VP_BIAS_CONTACT || R.bias == VP_BIAS_RMD_CONTACT) {
      nt = R.cv_blocks > nt ? R.cv_blocks : nt;
    } else {
      any_other = true;
      any_single = any_single || R.bias == VP_BIAS_RG;
      if (R.bias == VP_BIAS_RG) nsmax = R.ns > nsmax ? R.ns : nsmax;
    }
  }
  // k_cv handles the other kinds and advances the step counter; with contact
  // maps alone, k_cv_reduce advances it and k_cv is not needed
  const int reduce_inc = any_other ? 0 : inc_step;
  if (nt > 0) {
    hipLaunchKernelGGL(k_cv_pairs, dim3(nt * (nt + 1) / 2, s->R), dim3(2 * kCvTile), 0, st, s->info, W, s->cmap,
                       s->cskew);
    if (tan) {
      hipLaunchKernelGGL(k_cv_tangent_pairs, dim3(nt * nt, s->R), dim3(kCvTile), 0, st, s->info, W,
                         s->cmap);
      hipLaunchKernelGGL(k_cv_reduce<true>, dim3(nt, s->R), dim3(kCvTile), 0, st, s->info, W, s->igm0,
                         reduce_inc, s->step);
    } else {
      hipLaunchKernelGGL(k_cv_reduce<false>, dim3(nt, s->R), dim3(kCvTile), 0, st, s->info, W, s->igm0,
                         reduce_inc, s->step);
    }
  }
  if (!any_other && nt > 0) return;
  size_t lds = any_single ? sizeof(int4) * (size_t)nsmax : 0;
  hipLaunchKernelGGL(k_cv, dim3(s->R), dim3(kCvBlock), lds, st, s->info, W, s->igm0, s->mass0,
                     s->cforce, inc_step, s->step, tan ? 1 : 0);
}

size_t tangent_lds_bytes(const vp_system *s) {
  size_t stage = 2 * sizeof(int4) * (size_t)(s->stage_cap_max + kStageDummies) + sizeof(int4) * (size_t)(s->ntypes_max + 1);
  size_t red = sizeof(float) * 3 * kForceThreads;
  return stage > red ? stage : red;
}

hipError_t prepare_tangent(const vp_system *s) {
  return hipFuncSetAttribute((const void *)k_tangent_forces, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)tangent_lds_bytes(s));
}

void launch_tangent_forces(vp_system *s, Work &W, hipStream_t st) {
  const size_t lds = tangent_lds_bytes(s);
  for (int d = 0; d < 2; ++d) {
    hipLaunchKernelGGL(k_tangent_forces, dim3(xcd_grid(s->n_blocks)), dim3(kForceThreads), lds, st,
                       s->info, W, s->tile_rep, s->tile_first, s->n_blocks, s->types, s->stage_cap_max + kStageDummies, d);
    hipLaunchKernelGGL(k_tangent_bonded, dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info, W,
                       s->tile_rep, s->tile_first, s->n_blocks, s->bt_start, s->bterms, d);
  }
}

void launch_force_dir(vp_system *s, Work &W, const float *dx_user, double t, float *out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_dirs, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info, W,
                     s->tile_rep, s->tile_first, s->n_tiles, (int64_t)s->n_users, dx_user);
  launch_tangent_forces(s, W, st);
  launch_cv(s, W, 0, st, true);
  hipLaunchKernelGGL(k_force_dir_out, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                     s->state, W, s->tile_rep, s->tile_first, s->n_tiles, t, (int64_t)s->n_users, out);
}

void launch_force_out(vp_system *s, Work &W, double t, float *f_user, double *e_out,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_force_out, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                     s->state, W, s->tile_rep, s->tile_first, s->n_tiles, t, f_user);
  if (e_out)
    hipLaunchKernelGGL(k_energy_out, dim3(s->R), dim3(64), 0, st, s->info, s->state, W, t, e_out);
}

}  // namespace vp
