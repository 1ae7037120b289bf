// Cell binning, deterministic spatial sort and per-block neighbourhood lists.
//
// Coordinates are 32-bit fixed point (unit 2^-22 nm), so image shifts by the
// box edge are exact integer additions.  The trajectory state is kept sorted
// along serpentine xy columns, z inside a column, so 64 consecutive slots form
// a compact block.  A rebuild (creation, every step whose count n + 1 is a
// multiple of nstlist -- the same steps in every replica, so that rebuilding
// replicas share launches -- or a largest displacement since the last build
// reaching half the skin) is decided on the device, so the kernels of a
// captured step graph run every step and return at once for replicas that
// keep their lists.
//
//   k_bin      one workgroup per replica: periodic image, column and fine cell
//              of every atom, counting sorts whose in-bucket order is fixed by
//              keys (independent of the order of atomic operations);
//   k_permute  gathers positions/velocities into the new order;
//   k_list     one wave per block of 64 atoms: scans the cells (and their
//              periodic images) within the list radius of the block's
//              bounding box; every candidate that lies within r_cut + skin of
//              at least one block atom is appended to the block's staging
//              list (slot + image shift), and each such atom's list receives
//              the candidate's staging index.  The force kernel stages the
//              listed atoms in LDS with their shifts applied.
#include <type_traits>

#include "vp_device.h"
#include "vp_launch.h"

namespace vp {

__device__ __forceinline__ void cell_of_q(int X, int Lq, int nc, int &k, int &c) {
  long long kk = floordiv((long long)X, (long long)Lq);
  long long w = (long long)X - kk * Lq;
  long long cc = (w * nc) / Lq;
  k = (int)kk;
  c = (int)(cc < 0 ? 0 : (cc >= nc ? nc - 1 : cc));
}

// Exclusive scan of cnt[0, count) into start[0, count] (start[count] = total)
// by a 1024-thread workgroup, 4 entries per thread (count <= 4096).
__device__ __forceinline__ void block_scan(const int *cnt, int *start, int count, int total,
                                           int *wsum) {
  const int tid = threadIdx.x;
  int base = tid * 4, loc[4], sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int c = base + k;
    loc[k] = (c < count) ? cnt[c] : 0;
    sum += loc[k];
  }
  int incl = sum;
  const int lane = tid & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[tid >> 6] = incl;
  __syncthreads();
  int wpre = 0;
  for (int w = 0; w < (tid >> 6); ++w) wpre += wsum[w];
  int ex = wpre + incl - sum;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int c = base + k;
    if (c < count) {
      start[c] = ex;
      ex += loc[k];
    }
  }
  if (tid == 0) start[count] = total;
  __syncthreads();
}

// Sort order: xy columns (~0.8 nm) visited in a serpentine, atoms of a column
// by z (ascending in even, descending in odd columns) and then by user index,
// so consecutive slots are spatial neighbours and 64 of them form a compact
// block.  The sort is a counting sort over (column, z slab) buckets, whose
// order agrees with the z key, followed by a rank by (z key, user index)
// inside each bucket (a few atoms).  A second index lists the slots of every
// fine cell (~0.45 nm) in ascending order for the candidate search of the
// list build.  Both orders are fixed by keys, not by the order of atomic
// operations.
// MODE 0: trajectory (old sorted order, device decides whether to rebuild);
// MODE 1: evaluation from user-order FP32 positions x_user (always rebuilds).
template <int MODE>
__global__ __launch_bounds__(kBinThreads) void k_bin(const RepInfo *__restrict__ info,
                                                     RepState *__restrict__ state, Work W,
                                                     const float *__restrict__ x_user,
                                                     int32_t *__restrict__ bkt_t,
                                                     int32_t *__restrict__ zkey_t,
                                                     int32_t *__restrict__ fcell_t,
                                                     int32_t *__restrict__ bucket_t,
                                                     int2 *__restrict__ bko_t,
                                                     int32_t *__restrict__ orig_t,
                                                     int32_t *__restrict__ cellpos_t,
                                                     const long long *__restrict__ step) {
  const int r = blockIdx.x;
  const RepInfo R = info[r];
  __shared__ int s_cnt[kMaxCells];
  __shared__ int s_start[kMaxCells + 1];
  __shared__ int s_need;
  __shared__ int s_wsum[kBinThreads / 64];
  const int tid = threadIdx.x;
  if (tid == 0) {
    int need = 1;
    if (MODE == 0) {
      RepState &S = state[r];
      long long n = *step;
      float md = __uint_as_float(S.maxdisp_bits);
      need = S.force_rebuild || (md >= R.half_skin_margin) || ((n + 1) % R.nstlist == 0);
      S.rebuild = need;
      S.maxdisp_bits = 0u;
      if (need) {
        S.last_build = n;
        S.force_rebuild = 0;
        S.rebuilds += 1;
      }
    } else {
      W.flags[r] = 1;
    }
    s_need = need;
  }
  const int nzb = R.nzb;
  const int nbk = R.ncol[0] * R.ncol[1] * nzb;  // <= kMaxCells (checked at creation)
  for (int c = tid; c < nbk; c += kBinThreads) s_cnt[c] = 0;
  __syncthreads();
  if (!s_need) return;
  const int off = R.off;
  // ---- keys of every atom (old slot order)
#pragma unroll 4
  for (int p = tid; p < R.n; p += kBinThreads) {
    int X, Y, Z;
    if (MODE == 0) {
      int4 v = W.xq[off + p];
      X = v.x; Y = v.y; Z = v.z;
    } else {
      const float *u = x_user + 3ll * (R.uoff + p);
      X = (int)__builtin_rintf(u[0] * kQf);
      Y = (int)__builtin_rintf(u[1] * kQf);
      Z = (int)__builtin_rintf(u[2] * kQf);
    }
    const long long wx = (long long)X - floordiv(X, R.Lq[0]) * R.Lq[0];
    const long long wy = (long long)Y - floordiv(Y, R.Lq[1]) * R.Lq[1];
    const long long wz = (long long)Z - floordiv(Z, R.Lq[2]) * R.Lq[2];
    int cx = (int)((wx * R.ncol[0]) / R.Lq[0]), cy = (int)((wy * R.ncol[1]) / R.Lq[1]);
    cx = min(cx, R.ncol[0] - 1);
    cy = min(cy, R.ncol[1] - 1);
    const int col = cy * R.ncol[0] + ((cy & 1) ? R.ncol[0] - 1 - cx : cx);
    // z key: ascending z in even columns, descending in odd ones; the slab
    // index is a nondecreasing function of the key
    const long long zk = (col & 1) ? (long long)R.Lq[2] - 1 - wz : wz;
    const int zb = min(nzb - 1, (int)((zk * nzb) / R.Lq[2]));
    int fx = (int)((wx * R.nc[0]) / R.Lq[0]), fy = (int)((wy * R.nc[1]) / R.Lq[1]),
        fz = (int)((wz * R.nc[2]) / R.Lq[2]);
    fx = min(fx, R.nc[0] - 1);
    fy = min(fy, R.nc[1] - 1);
    fz = min(fz, R.nc[2] - 1);
    const int bk = col * nzb + zb;
    bkt_t[off + p] = bk;
    zkey_t[off + p] = (col & 1) ? -(int)wz : (int)wz;
    fcell_t[off + p] = (fz * R.nc[1] + fy) * R.nc[0] + fx;
    atomicAdd(&s_cnt[bk], 1);
  }
  __syncthreads();
  block_scan(s_cnt, s_start, nbk, R.n, s_wsum);
  for (int c = tid; c < nbk; c += kBinThreads) s_cnt[c] = s_start[c];
  __syncthreads();
  for (int p = tid; p < R.n; p += kBinThreads) {
    const int bk = bkt_t[off + p];
    const int pos = atomicAdd(&s_cnt[bk], 1);
    bucket_t[off + pos] = p;
    bko_t[off + pos] = make_int2(zkey_t[off + p], (MODE == 0) ? W.orig[off + p] : p);
  }
  __syncthreads();
  // ---- rank inside a bucket by (z key, user index)
  for (int s = tid; s < R.n; s += kBinThreads) {
    const int p = bucket_t[off + s];
    const int bk = bkt_t[off + p];
    const int2 me = bko_t[off + s];
    auto before = [&](int2 o) { return (o.x < me.x || (o.x == me.x && o.y < me.y)) ? 1 : 0; };
    // the bucket's entries are independent loads: four in flight at a time
    int rank = 0, q = s_start[bk];
    const int qe = s_start[bk + 1];
    for (; q + 4 <= qe; q += 4) {
      const int2 o0 = bko_t[off + q], o1 = bko_t[off + q + 1], o2 = bko_t[off + q + 2], o3 = bko_t[off + q + 3];
      rank += before(o0) + before(o1) + before(o2) + before(o3);
    }
    for (; q < qe; ++q) rank += before(bko_t[off + q]);
    const int ns = s_start[bk] + rank;
    orig_t[off + ns] = me.y;
    W.cell_of[off + ns] = fcell_t[off + p];
  }
  __syncthreads();
  // ---- fine-cell index of the new slots
  for (int c = tid; c < R.ncell; c += kBinThreads) s_cnt[c] = 0;
  __syncthreads();
  for (int s = tid; s < R.n; s += kBinThreads) atomicAdd(&s_cnt[W.cell_of[off + s]], 1);
  __syncthreads();
  block_scan(s_cnt, s_start, R.ncell, R.n, s_wsum);
  for (int c = tid; c <= R.ncell; c += kBinThreads) W.cell_start[R.cell0 + c] = s_start[c];
  for (int c = tid; c < R.ncell; c += kBinThreads) s_cnt[c] = s_start[c];
  __syncthreads();
  for (int s = tid; s < R.n; s += kBinThreads) {
    const int pos = atomicAdd(&s_cnt[W.cell_of[off + s]], 1);
    bucket_t[off + pos] = s;
  }
  __syncthreads();
  for (int q = tid; q < R.n; q += kBinThreads) {
    const int s = bucket_t[off + q];
    const int c = W.cell_of[off + s];
    int rank = 0, t = s_start[c];
    const int te = s_start[c + 1];
    for (; t + 4 <= te; t += 4) {
      const int b0 = bucket_t[off + t], b1 = bucket_t[off + t + 1], b2 = bucket_t[off + t + 2],
                b3 = bucket_t[off + t + 3];
      rank += (b0 < s) + (b1 < s) + (b2 < s) + (b3 < s);
    }
    for (; t < te; ++t) rank += (bucket_t[off + t] < s);
    W.cell_slots[off + s_start[c] + rank] = s;
    cellpos_t[off + s] = s_start[c] + rank;
  }
}

// New slot -> source (old slot through the old inverse map, or user index);
// also records the atom's periodic image at this build, writes its wrapped
// position, user index, slot (with its Lennard-Jones class and site role) and
// image in fine-cell order, and its new slot by user index.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_permute(const RepInfo *__restrict__ info,
                                                    const RepState *__restrict__ state, Work W,
                                                    const int32_t *__restrict__ tile_rep,
                                                    const int32_t *__restrict__ tile_first,
                                                    int ntiles, const float *__restrict__ x_user,
                                                    const int32_t *__restrict__ type0,
                                                    const int32_t *__restrict__ role0,
                                                    const int32_t *__restrict__ orig_t,
                                                    int4 *__restrict__ xq_t,
                                                    float4 *__restrict__ vel_t,
                                                    int32_t *__restrict__ wrap_t,
                                                    const int32_t *__restrict__ cellpos_t,
                                                    int4 *__restrict__ cellx_t,
                                                    int2 *__restrict__ celljw_t,
                                                    float4 *__restrict__ tx_t,
                                                    float4 *__restrict__ tv_t,
                                                    int32_t *__restrict__ inv_t) {
  int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  if (MODE == 0 ? !state[r].rebuild : !W.flags[r]) return;
  int p = tile_first[tile] + threadIdx.x;
  if (p >= R.n) return;
  int slot = R.off + p;
  int a = orig_t[slot];
  int4 x;
  if (MODE == 0) {
    int old = W.inv[R.uoff + a];
    x = W.xq[old];
    vel_t[slot] = W.vel[old];
    if (W.tx)  // tangents follow their atoms
      for (int d = 0; d < 2; ++d) {
        tx_t[d * W.fstride + slot] = W.tx[d * W.fstride + old];
        tv_t[d * W.fstride + slot] = W.tv[d * W.fstride + old];
      }
  } else {
    const float *u = x_user + 3ll * (R.uoff + a);
    x = make_int4((int)__builtin_rintf(u[0] * kQf), (int)__builtin_rintf(u[1] * kQf),
                  (int)__builtin_rintf(u[2] * kQf), type0[R.uoff + a]);
  }
  xq_t[slot] = x;
  int kx = (int)floordiv(x.x, R.Lq[0]), ky = (int)floordiv(x.y, R.Lq[1]),
      kz = (int)floordiv(x.z, R.Lq[2]);
  const int wr = pack_wrap(kx, ky, kz);
  wrap_t[slot] = wr;
  // the same atom in fine-cell order (wrapped position) for the candidate search
  const int q = R.off + cellpos_t[slot];
  cellx_t[q] = make_int4(x.x - kx * R.Lq[0], x.y - ky * R.Lq[1], x.z - kz * R.Lq[2], a);
  // the sign bit marks an atom with Lennard-Jones parameters, bits 29-30 its
  // site role
  celljw_t[q] = make_int2(p | (x.w < R.nlj_types ? (int)0x80000000u : 0) | (role0[R.uoff + a] << 29), wr);
  inv_t[R.uoff + a] = slot;
}

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
// minimum / maximum over the 16 lanes of a quarter wave
__device__ __forceinline__ int quarter_min_i(int v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int quarter_max_i(int v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// A lane's list entries are collected in LDS, one buffer of twelve entries
// per stream (partners with Lennard-Jones parameters, charge-only partners:
// chunk_row), by one
// 16-bit store per entry at a running address.  When a buffer holds eight or
// more entries, the first eight are copied as one 16-byte row of its stream
// (upward from row 0, or downward from the last row), and the rest move to
// the front.  Rows past the list's capacity are not stored (entries are still
// counted: the overflow is flagged).  Twelve entries let a batch of up to
// four appends run with one check for a full row after it.
constexpr int kBufLen = 12;
constexpr int kBufStride = 2 * kBufLen;  // bytes between lanes' buffers
typedef __attribute__((address_space(3))) uint16_t lds_u16;  // 32-bit LDS addresses
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ lds_u16 *lds16(uint32_t a) { return (lds_u16 *)(size_t)a; }
__device__ __forceinline__ lds_u32 *lds32(uint32_t a) { return (lds_u32 *)(size_t)a; }
// the buffer's addresses are kept as plain 32-bit integers, so that an append
// is a store and an add of 0 or 2
struct ListBuf {
  uint32_t base;  // LDS byte address of the lane's entries (4-byte aligned)
  uint32_t wa;    // LDS byte address of the next free entry
  uint4 *list;    // the block's list rows
  int lane;
  int rowcap;     // rows per lane
  int rows;       // rows copied out, stored or not
  bool down;      // rows fill the list from its last row downward

  __device__ __forceinline__ void flush() {
    const uint4 r = make_uint4(*lds32(base), *lds32(base + 4), *lds32(base + 8), *lds32(base + 12));
    if (rows < rowcap) list[list_row(down ? rowcap - 1 - rows : rows, lane)] = r;
    ++rows;
    const uint32_t t0 = *lds32(base + 16), t1 = *lds32(base + 20);
    *lds32(base) = t0;
    *lds32(base + 4) = t1;
    wa -= 16;
  }
  __device__ __forceinline__ void append(uint32_t e) {
    *lds16(wa) = (uint16_t)e;
    wa += 2;
    if (wa == base + 16) flush();
  }
  __device__ __forceinline__ bool row_full() const { return wa >= base + 16; }
  __device__ __forceinline__ int count() const { return 8 * rows + (int)(wa - base) / 2; }
};

// Staged candidates tested together per step of the list kernel's inner loop
// (kBlk is a multiple, so reads stay inside the 64-entry batch buffer).
constexpr int kListBatch = 4;
// Quantised coordinates of the list test: 14-bit signed values, inert |q|^2,
// and the replica size below which user indices fit the fast test's 16 bits.
constexpr int kQMax = 8191;
constexpr int kQInert = 1200000000;  // > 3 kQMax^2 + 4 kQMax^2 + any threshold, < 2^31 - 4 kQMax^2
constexpr int kMaxFastAtoms = 65535;
// Largest distance (squared, coordinate units) between the first atom of a
// three-atom site and its other atoms: 0.25 nm; a larger one flags the replica.
constexpr float kSiteMax2 = (float)(0.25 * kQ * 0.25 * kQ);
constexpr long long kSiteMaxQ = (long long)(0.25 * kQ) + 1;
typedef short short2v __attribute__((ext_vector_type(2)));
// Runs of cells listed per row group of the list kernel's search.
constexpr int kMaxRuns = 2 * kBlk;
static_assert(kBlk % kListBatch == 0, "batch must divide the candidate buffer");

// One wave per block of 64 sorted atoms.  The cells that can hold a neighbour
// of the block (fine cells within the list radius of the block's bounding
// box, with their periodic images) are visited row by row; the cells of one
// row that share an image are consecutive, so their atoms form one range of
// the fine-cell ordered copy of the positions.  Each range is read 64
// candidates at a time (one coalesced load per lane): every lane applies the
// cell's image to its candidate and keeps it if it lies within the list
// radius of the bounding box of one of the block's quarters (16 atoms).
// Every kept candidate receives the next staging index (its slot | image
// shift is stored) and its position is compacted into LDS; then each lane
// tests the batch against its own atom, with no communication between lanes,
// and appends the staging indices of the candidates within the list radius
// (exclusions removed) to its list.  This test runs in FP32 on coordinates
// relative to the block's corner, with the radius enlarged by a bound on the
// rounding (a few hundred grid units at most): the list is a superset
// of the exact list radius, and the force kernel applies the exact cutoff.
template <int MODE>
// Register budget for seven waves per SIMD (measured: a full rebuild of the
// 64 x 12,560 batch takes 1.89 ms at seven waves with a few spilled
// registers, 2.26 ms at the four that the unconstrained allocation allows,
// 2.20 ms at eight with more spills): the candidate loop is latency-bound,
// so more waves in flight beat spill-free code.
__global__ __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(5))) void k_list(const RepInfo *__restrict__ info,
                                               RepState *__restrict__ state, Work W,
                                               const int32_t *__restrict__ tile_rep,
                                               const int32_t *__restrict__ tile_first, int nblk,
                                               const int4 *__restrict__ xq_t,
                                               const float4 *__restrict__ vel_t,
                                               const int32_t *__restrict__ orig_t,
                                               const int32_t *__restrict__ wrap_t,
                                               const int4 *__restrict__ cellx_t,
                                               const int2 *__restrict__ celljw_t,
                                               const int32_t *__restrict__ ex_start,
                                               const int32_t *__restrict__ ex_list,
                                               const float4 *__restrict__ integ0,
                                               const float4 *__restrict__ tx_t,
                                               const float4 *__restrict__ tv_t,
                                               const int32_t *__restrict__ inv_t) {
  // kept candidates: quantised position q (x | y << 16, z | user index << 16,
  // |q|^2) and user index
  __shared__ __align__(16) int32_t s_qxy[kBlk], s_qzu[kBlk], s_qc2[kBlk], s_uid[kBlk];
  // kept sites: the same records for each of their three atoms
  __shared__ __align__(16) int32_t s_sxy[3][kBlk], s_szu[3][kBlk], s_sc2[3][kBlk];
  // each lane's list entries not yet stored: first stream (LJ partners)
  // [0, kBlk), second stream (charge-only partners) [kBlk, 2 kBlk)
  __shared__ __align__(16) uint8_t s_buf[2 * kBlk * kBufStride];
  __shared__ int s_cidx[3][18];  // fine-cell edges of the replica
  __shared__ int s_rq0[kMaxRuns];       // runs of a row group: first slot in fine-cell order,
  __shared__ int s_rimg[kMaxRuns];      // image (packed),
  __shared__ int s_rpre[kMaxRuns + 1];  // number of candidates before the run
  const int b = xcd_tile(blockIdx.x, nblk);
  if (b < 0) return;
  const int tile = b / (kTile / kBlk);
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  if (MODE == 0 ? !state[r].rebuild : !W.flags[r]) return;
  const int lane = threadIdx.x;
  const int p0 = tile_first[tile] + (b % (kTile / kBlk)) * kBlk;
  const int p = p0 + lane;
  const int slot = R.off + p;
  const bool active = p < R.n;
  if (p0 >= R.n) {
    W.nbcnt[slot] = 0;
    W.nblj[slot] = 0;
    if (lane == 0) W.stage_n[b] = 0;
    return;
  }
  const int off = R.off;
  const int Lx = R.Lq[0], Ly = R.Lq[1], Lz = R.Lq[2];
  const int ncx = R.nc[0], ncy = R.nc[1], ncz = R.nc[2];
  if (lane < 3 * 17) s_cidx[lane / 17][lane % 17] = R.cedge[lane / 17][lane % 17];
  s_qxy[lane] = 0;  // every record ever read holds bounded values
  s_qzu[lane] = 0;
  // the lane's atom; an inactive lane sits far away and never matches
  int4 xi = make_int4(0, 0, 0, 0);
  int wx = kDummyCoord, wy = kDummyCoord, wz = kDummyCoord, a = -(1 << 20), e0 = 0, e1 = 0;
  // exclusions of the lane's atom: user-index offsets in [-32, 31] as a bit
  // mask (offset 0 is the atom itself), any others checked against the list
  uint64_t exm = 0;
  bool exfar = false;
  bool exrun = true;
  int exlo = 0, excnt = 0;
  int bx0 = 0, bx1 = 0, by0 = 0, by1 = 0, bz0 = 0, bz1 = 0;
  // quarter boxes in LDS (x0, x1, y0, y1 | z0, z1, has an atom): read once per
  // candidate batch rather than held in scalar registers across the cell loops
  __shared__ int4 s_qb[4][2];
  {
    int ax = 0, ay = 0, az = 0;
    if (active) {
      xi = xq_t[slot];
      const int wr = wrap_t[slot];
      ax = wx = xi.x - unpack_wrap(wr, 0) * Lx;
      ay = wy = xi.y - unpack_wrap(wr, 1) * Ly;
      az = wz = xi.z - unpack_wrap(wr, 2) * Lz;
      a = orig_t[slot];
      e0 = ex_start[R.uoff + a];
      e1 = ex_start[R.uoff + a + 1];
      exm = 1ull << 32;
      for (int e = e0; e < e1; ++e) {
        const int d = ex_list[e] - a;
        if (d >= -32 && d < 32) exm |= 1ull << (d + 32);
        else exfar = true;
      }
      // the atom and its exclusions as one run of user indices [exlo, exlo +
      // excnt) when they form one (the three atoms of a water molecule)
      int mn = a, mx = a;
      for (int e = e0; e < e1; ++e) {
        mn = min(mn, ex_list[e]);
        mx = max(mx, ex_list[e]);
      }
      exrun = mx - mn == e1 - e0;
      exlo = mn;
      excnt = e1 - e0 + 1;
    }
    // bounding box of the block (wrapped frame)
    const int big = 0x7fffffff;
    bx0 = wave_min_i(active ? ax : big);
    bx1 = wave_max_i(active ? ax : -big);
    by0 = wave_min_i(active ? ay : big);
    by1 = wave_max_i(active ? ay : -big);
    bz0 = wave_min_i(active ? az : big);
    bz1 = wave_max_i(active ? az : -big);
    // bounding boxes of the four quarters (16 consecutive atoms each)
    const int qx0 = quarter_min_i(active ? ax : big), qx1 = quarter_max_i(active ? ax : -big);
    const int qy0 = quarter_min_i(active ? ay : big), qy1 = quarter_max_i(active ? ay : -big);
    const int qz0 = quarter_min_i(active ? az : big), qz1 = quarter_max_i(active ? az : -big);
    const bool qact = __ballot(active) & (0xffffull << (lane & 48));
    if ((lane & 15) == 0) {
      s_qb[lane >> 4][0] = make_int4(qx0, qx1, qy0, qy1);
      s_qb[lane >> 4][1] = make_int4(qz0, qz1, qact ? 1 : 0, 0);
    }
  }
  // the fast test takes user indices modulo 2^16 and needs them below 2^15
  const bool anyfar = __ballot(exfar) != 0ull || R.n > kMaxFastAtoms;
  // for every atom of the block the atom and its exclusions form one run of
  // user indices: the fast test checks the candidate's user index against
  // the run instead of the window (exclusion lists hold distinct atoms other
  // than the atom itself, so max - min = count means a run)
  const bool few = __ballot(!exrun) == 0ull;
  const long long rl = R.rlq;
  // cell ranges (unfolded: u = image * nc + cell)
  const int ux0 = (int)floordiv(((long long)bx0 - rl) * ncx, Lx);
  const int ux1 = (int)floordiv(((long long)bx1 + rl) * ncx, Lx);
  const int uy0 = (int)floordiv(((long long)by0 - rl) * ncy, Ly);
  const int uy1 = (int)floordiv(((long long)by1 + rl) * ncy, Ly);
  const int uz0 = (int)floordiv(((long long)bz0 - rl) * ncz, Lz);
  const int uz1 = (int)floordiv(((long long)bz1 + rl) * ncz, Lz);
  const double rl2d = (double)rl * (double)rl;
  const float rl2 = R.rl2q;
  // The candidate test runs in integers.  Coordinates relative to the block's
  // centre are divided by 2^qs (floor) and clamped to [-8191, 8191], with qs
  // the smallest shift that keeps every kept candidate (within rl of the
  // block box) and every block atom inside that range; then
  //   |qc - qa|^2 = |qc|^2 - 2 qc.qa + |qa|^2
  // is exact in 32 bits, |qc|^2 is formed once per kept candidate, and a test
  // is two signed 16-bit dot products against the lane's threshold
  // T - |qa|^2.  Flooring moves each component of a separation by less than
  // one unit, so a pair at distance d has |qc - qa| < d / 2^qs + sqrt(3): with
  // T = ceil((rl / 2^qs + sqrt(3))^2) every candidate within the list radius
  // passes (the list is a superset of the exact list, larger by ~0.1% at the
  // usual block size, and the force kernel applies the exact cutoff).
  const int ox = bx0 + (bx1 - bx0) / 2, oy = by0 + (by1 - by0) / 2, oz = bz0 + (bz1 - bz0) / 2;
  int qs = 0;
  // every coordinate of a staged atom lies within half of the block centre
  // (kept sites' atoms within two site offsets beyond the list radius)
  const long long half = (long long)max(bx1 - bx0, max(by1 - by0, bz1 - bz0)) / 2 + 1 + rl + 64 +
                         (anyfar ? 0ll : 2ll * kSiteMaxQ);
  while ((half >> qs) > (long long)kQMax - 1) ++qs;
  const int qthr = (int)ceil(((double)rl / (double)(1ll << qs) + 1.7320508075688772) *
                             ((double)rl / (double)(1ll << qs) + 1.7320508075688772) + 1e-6);
  short2v m2axy = {0, 0}, m2az0 = {0, 0};
  int thr = 0;  // inactive lanes: no candidate passes (|qc|^2 >= 0)
  if (active) {
    const int qax = (wx - ox) >> qs, qay = (wy - oy) >> qs, qaz = (wz - oz) >> qs;
    m2axy = short2v{(short)(-2 * qax), (short)(-2 * qay)};
    m2az0 = short2v{(short)(-2 * qaz), 0};
    thr = qthr - (qax * qax + qay * qay + qaz * qaz);
  }
  // candidate record (qxy, qzu, |qc|^2) passes the lane's test
  auto near = [&](int qxy, int qzu, int qc2) {
    const int t = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, qxy), m2axy, qc2, false);
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, qzu), m2az0, t, false) < thr;
  };
  // exclusion window: for a candidate of user index oj, bit oj - a + 32 of exm
  // is moved to bit 63 by a left shift of a + 31 - oj (in range iff that
  // shift is below 64)
  const int exs = a + 31;
  const int lb = b - R.blk0;
  uint16_t *lst = W.nblist + R.list_off + (int64_t)lb * R.maxnb * kBlk;
  uint32_t *stg = W.stage + (int64_t)b * W.stage_stride;
  const int cap = R.stage_cap;
  const int *cstart = W.cell_start + R.cell0;
  int nst = 0;
  const uint32_t bufl = (uint32_t)(size_t)(lds_u16 *)(s_buf + lane * kBufStride);
  const uint32_t bufr = (uint32_t)(size_t)(lds_u16 *)(s_buf + (kBlk + lane) * kBufStride);
  const int rowcap = R.maxnb >> 3;
  ListBuf lbl{bufl, bufl, reinterpret_cast<uint4 *>(lst), lane, rowcap, 0, false};
  ListBuf lbr{bufr, bufr, reinterpret_cast<uint4 *>(lst), lane, rowcap, 0, true};

  // The force kernel stages positions relative to the block centre in FP32,
  // exact while every coordinate stays below 2^24 grid units from it (with
  // 0.1 nm of room for the motion until the next build, which half the skin
  // bounds); a block beyond that flags its replica.
  bool bad = half + (long long)(0.1 * kQ) >= (1ll << 24);
  __syncthreads();  // cell edges in LDS
  // Fast mode stages every candidate kept by the quarter boxes.  If that
  // would exceed the block's staging capacity, the block is built again in
  // exact mode, which stages only candidates within the list radius of at
  // least one atom (a ballot per candidate; rare).
  // The rows of the search, (uz, uy) with uz outermost, are taken in groups.
  // One lane per row finds the cells of its row that pass the gap test (the
  // gap along x first falls, then grows, so they are consecutive) and splits
  // them at image boundaries into runs, each a range of the fine-cell order.
  // The group's runs are listed in LDS in row order and their candidates are
  // read 64 at a time across run boundaries, so every load but the group's
  // last is full.  The candidates come in the order of a sequential scan of
  // rows and cells.
  const int ny = uy1 - uy0 + 1, nrows = (uz1 - uz0 + 1) * ny;
  const int nimg = (int)(floordiv(ux1, ncx) - floordiv(ux0, ncx)) + 1;  // runs per row at most
  const int gsize = nimg <= kMaxRuns ? min(kBlk, kMaxRuns / nimg) : 0;
  if (gsize == 0) bad = true;  // a list radius of more than a hundred box edges
  bool exact = false;
  for (int mode = 0; mode < 2; ++mode) {
    exact = mode == 1;
    // site mode: the fast test with three-atom sites listed by one entry
    const bool sm = !exact && !anyfar;
    nst = 0;
    lbl.wa = lbl.base;
    lbl.rows = 0;
    lbr.wa = lbr.base;
    lbr.rows = 0;
    bool full = false;
    for (int g0 = 0; gsize > 0 && g0 < nrows && !full; g0 += gsize) {
      // ---- runs of the group's rows
      int nr = 0, ua = 0, ub = 0, rowcell = 0, iyr = 0, izr = 0;
      if (lane < gsize && g0 + lane < nrows) {
        const int row = g0 + lane;
        const int uz = uz0 + row / ny, uy = uy0 + row % ny;
        izr = (int)floordiv(uz, ncz);
        iyr = (int)floordiv(uy, ncy);
        const int cz = uz - izr * ncz, cy = uy - iyr * ncy;
        rowcell = (cz * ncy + cy) * ncx;
        // gaps between the row's slabs and the block box (coordinate units)
        const long long zl = (long long)izr * Lz + s_cidx[2][cz], zh = (long long)izr * Lz + s_cidx[2][cz + 1];
        const double gz = (double)max(0ll, max(zl - bz1, (long long)bz0 - zh));
        const long long yl = (long long)iyr * Ly + s_cidx[1][cy], yh = (long long)iyr * Ly + s_cidx[1][cy + 1];
        const double gy = (double)max(0ll, max(yl - by1, (long long)by0 - yh));
        const double gyz = gz * gz + gy * gy;
        if (gyz <= rl2d) {
          int ix = (int)floordiv(ux0, ncx), cx = ux0 - ix * ncx;
          bool found = false;
          for (int ux = ux0; ux <= ux1; ++ux) {
            const long long xl = (long long)ix * Lx + s_cidx[0][cx], xh = (long long)ix * Lx + s_cidx[0][cx + 1];
            const double gx = (double)max(0ll, max(xl - bx1, (long long)bx0 - xh));
            if (gyz + gx * gx <= rl2d) {
              if (!found) ua = ux;
              ub = ux;
              found = true;
            }
            if (++cx == ncx) {
              cx = 0;
              ++ix;
            }
          }
          if (found) nr = (int)(floordiv(ub, ncx) - floordiv(ua, ncx)) + 1;
        }
      }
      int roff = nr;  // inclusive scan of the run counts
#pragma unroll
      for (int o = 1; o < kBlk; o <<= 1) {
        const int t = __shfl_up(roff, o, kBlk);
        if (lane >= o) roff += t;
      }
      const int nruns = __shfl(roff, kBlk - 1, kBlk);
      roff -= nr;
      for (int k = 0; k < nr; ++k) {
        const int im = (int)floordiv(ua, ncx) + k;
        const int lo = max(ua, im * ncx), hi = min(ub, im * ncx + ncx - 1);
        const int c0 = rowcell + lo - im * ncx;
        const int qs = cstart[c0];
        s_rq0[roff + k] = qs;
        s_rpre[roff + k] = cstart[c0 + hi - lo + 1] - qs;  // length, replaced by its prefix below
        s_rimg[roff + k] = pack_wrap(im, iyr, izr);
      }
      __syncthreads();
      int total = 0;
      {
        // exclusive prefix of the run lengths, two runs per lane; entries past
        // the last run hold the total
        const int l0 = 2 * lane < nruns ? s_rpre[2 * lane] : 0;
        const int l1 = 2 * lane + 1 < nruns ? s_rpre[2 * lane + 1] : 0;
        int incl = l0 + l1;
#pragma unroll
        for (int o = 1; o < kBlk; o <<= 1) {
          const int t = __shfl_up(incl, o, kBlk);
          if (lane >= o) incl += t;
        }
        total = __shfl(incl, kBlk - 1, kBlk);
        const int ex = incl - l0 - l1;
        s_rpre[2 * lane] = ex;
        s_rpre[2 * lane + 1] = ex + l0;
        if (lane == kBlk - 1) s_rpre[kMaxRuns] = total;
      }
      __syncthreads();
      int rc = 0;  // run of the first candidate of the next load (uniform)
      for (int t0 = 0; t0 < total && !full; t0 += kBlk) {
        const int t = t0 + lane;
        const bool valid = t < total;
        int run = rc;
        if (valid)
          while (s_rpre[run + 1] <= t) ++run;
        rc = __shfl(run, kBlk - 1, kBlk);  // lane 63 is valid whenever another load follows
        // ---- load 64 candidates, keep those near one of the quarter boxes.
        // In site mode the first atom of a three-atom site stands for the
        // site (its other atoms are not candidates): it is kept if within the
        // list radius plus its larger member offset of a quarter box, and
        // its three atoms are staged together with its image shift.
        bool keep = false, site = false;
        int3 cq = make_int3(0, 0, 0), cm1 = cq, cm2 = cq;
        uint32_t code = 0u, code1 = 0u, code2 = 0u;
        int uid = 0;
        if (valid) {
          const int q = s_rq0[run] + (t - s_rpre[run]);
          const int img = s_rimg[run];
          const int six = unpack_wrap(img, 0), siy = unpack_wrap(img, 1), siz = unpack_wrap(img, 2);
          const int4 cxq = cellx_t[off + q];
          const int2 jw = celljw_t[off + q];
          const int px = cxq.x + six * Lx, py = cxq.y + siy * Ly, pz = cxq.z + siz * Lz;
          const int role = (jw.x >> 29) & 3;
          site = sm && role == 1;
          float krl2 = rl2;
          int3 d1 = make_int3(0, 0, 0), d2 = d1;
          int sl1 = 0, sl2 = 0;
          if (site) {
            const int4 xh = xq_t[off + (jw.x & 0xffff)];
            sl1 = inv_t[R.uoff + cxq.w + 1];
            sl2 = inv_t[R.uoff + cxq.w + 2];
            const int4 x1 = xq_t[sl1], x2 = xq_t[sl2];
            d1 = make_int3(x1.x - xh.x, x1.y - xh.y, x1.z - xh.z);
            d2 = make_int3(x2.x - xh.x, x2.y - xh.y, x2.z - xh.z);
            const float m2 = fmaxf(qr2((float)d1.x, (float)d1.y, (float)d1.z), qr2((float)d2.x, (float)d2.y, (float)d2.z));
            if (!(m2 <= kSiteMax2)) bad = true;  // a site torn apart: the replica is flagged
            // rounding of the two squares and the root is far below the unit added
            const float kr = (float)R.rlq + __builtin_sqrtf(fminf(m2, kSiteMax2)) + 2.0f;
            krl2 = kr * kr;
          }
          // kept if within the list radius of a quarter box; a box distance
          // never exceeds an atom distance, also after rounding
          if (!(sm && role == 2)) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const int4 q0 = s_qb[g][0], q1 = s_qb[g][1];
              const float gxq = (float)max(0, max(q0.x - px, px - q0.y));
              const float gyq = (float)max(0, max(q0.z - py, py - q0.w));
              const float gzq = (float)max(0, max(q1.x - pz, pz - q1.y));
              keep = keep || (q1.z != 0 && qr2(gxq, gyq, gzq) < krl2);
            }
          }
          const int sx = six - unpack_wrap(jw.y, 0), sy = siy - unpack_wrap(jw.y, 1),
                    sz = siz - unpack_wrap(jw.y, 2);
          if (keep && (sx < -16 || sx > 15 || sy < -16 || sy > 15 || sz < -16 || sz > 15)) {
            bad = true;  // shift not representable: the replica is flagged
            keep = false;
          }
          uid = cxq.w;
          auto record = [&](int x, int y, int z) {
            const int qx = min(max((x - ox) >> qs, -kQMax), kQMax), qy = min(max((y - oy) >> qs, -kQMax), kQMax),
                      qz = min(max((z - oz) >> qs, -kQMax), kQMax);
            return make_int3((int)(((uint32_t)qx & 0xffffu) | ((uint32_t)qy << 16)),
                             (int)(((uint32_t)qz & 0xffffu) | ((uint32_t)uid << 16)), qx * qx + qy * qy + qz * qz);
          };
          cq = record(px, py, pz);
          const uint32_t shift = ((uint32_t)((sx + 16) & 31) << 16) | ((uint32_t)((sy + 16) & 31) << 21) |
                                 ((uint32_t)((sz + 16) & 31) << 26);
          code = ((uint32_t)jw.x & 0xffffu) | shift;
          if (site) {
            cm1 = record(px + d1.x, py + d1.y, pz + d1.z);
            cm2 = record(px + d2.x, py + d2.y, pz + d2.z);
            code1 = ((uint32_t)(sl1 - off) & 0xffffu) | shift;
            code2 = ((uint32_t)(sl2 - off) & 0xffffu) | shift;
          }
        }
        // kept single atoms take places [0, n1) of the load's records and
        // staging, kept sites places [0, ns3) of the site records and three
        // staging places each after the single atoms (each group in lane
        // order)
        const uint64_t km = __ballot(keep), kms = __ballot(keep && site);
        const uint64_t below = (1ull << lane) - 1ull;
        const int nk = __popcll(km), ns3 = __popcll(kms), n1 = nk - ns3;
        const int at = site ? __popcll(kms & below) : __popcll(km & ~kms & below);
        if (!exact && nst + n1 + 3 * ns3 > cap) {
          full = true;  // uniform: the block is redone in exact mode
          break;
        }
        if (keep && !site) {
          s_qxy[at] = cq.x;
          s_qzu[at] = cq.y;
          s_qc2[at] = cq.z;
          s_uid[at] = uid;
        }
        if (keep && site) {
          s_sxy[0][at] = cq.x;
          s_szu[0][at] = cq.y;
          s_sc2[0][at] = cq.z;
          s_sxy[1][at] = cm1.x;
          s_szu[1][at] = cm1.y;
          s_sc2[1][at] = cm1.z;
          s_sxy[2][at] = cm2.x;
          s_szu[2][at] = cm2.y;
          s_sc2[2][at] = cm2.z;
        }
        // the fast test reads whole batches: entries up to the next
        // multiple of the batch are made inert (|qc|^2 beyond any test)
        if (lane >= n1 && lane < ((n1 + kListBatch - 1) & ~(kListBatch - 1))) s_qc2[lane] = kQInert;
        if (lane >= ns3 && lane < ((ns3 + kListBatch - 1) & ~(kListBatch - 1))) {
          s_sc2[0][lane] = kQInert;
          s_sc2[1][lane] = kQInert;
          s_sc2[2][lane] = kQInert;
        }
        if (!exact && keep) {  // every kept candidate is staged
          if (!site) {
            stg[nst + at] = code;
          } else {
            stg[nst + n1 + 3 * at] = code;
            stg[nst + n1 + 3 * at + 1] = code1;
            stg[nst + n1 + 3 * at + 2] = code2;
          }
        }
        __syncthreads();
        if (!exact) {
          // ---- every staged candidate against the lane's own atom
          if (!anyfar) {
            // kListBatch candidates read and tested together (their LDS
            // reads overlap), then appended in order with one check for a
            // completed row per batch (a batch adds at most four entries).
            auto test_singles = [&](ListBuf &buf, int hi, auto few_tag) {
              constexpr bool FEW = decltype(few_tag)::value;
              for (int k0 = 0; k0 < hi; k0 += kListBatch) {
                static_assert(kListBatch == 4, "one 16-byte read per record field and batch");
                const int4 qxy = *reinterpret_cast<const int4 *>(&s_qxy[k0]);
                const int4 qzu = *reinterpret_cast<const int4 *>(&s_qzu[k0]);
                const int4 qc2 = *reinterpret_cast<const int4 *>(&s_qc2[k0]);
                const int rxy[kListBatch] = {qxy.x, qxy.y, qxy.z, qxy.w};
                const int rzu[kListBatch] = {qzu.x, qzu.y, qzu.z, qzu.w};
                const int rc2[kListBatch] = {qc2.x, qc2.y, qc2.z, qc2.w};
#pragma unroll
                for (int u = 0; u < kListBatch; ++u) {
                  bool exw;
                  if constexpr (FEW) {
                    exw = (uint32_t)((int)((uint32_t)rzu[u] >> 16) - exlo) < (uint32_t)excnt;
                  } else {
                    const uint32_t sh = (uint32_t)(exs - (int)((uint32_t)rzu[u] >> 16));
                    exw = sh < 64u && (int32_t)(uint32_t)((exm << (sh & 63u)) >> 32) < 0;
                  }
                  const bool in = near(rxy[u], rzu[u], rc2[u]) && !exw;
                  // stored by every lane: an entry that is not kept is
                  // overwritten by the next one appended (or left past the end)
                  *lds16(buf.wa) = (uint16_t)(nst + k0 + u);
                  buf.wa += in ? 2u : 0u;
                }
                static_assert(kListBatch <= kBufLen - 8, "a batch must fit behind seven entries");
                if (buf.row_full()) buf.flush();
              }
            };
            // single atoms go to the first stream
            if (few) test_singles(lbl, n1, std::true_type{});
            else test_singles(lbl, n1, std::false_type{});
            // sites go to the second: listed when one of their three atoms
            // is within the list radius, unless the lane's atom is one of
            // them (a site's atoms exclude each other and nothing else)
            constexpr int SB = 2;  // sites per batch of LDS reads
            for (int k0 = 0; k0 < ns3; k0 += SB) {
              int2 rxy[3], rzu[3], rc2[3];
#pragma unroll
              for (int m = 0; m < 3; ++m) {
                rxy[m] = *reinterpret_cast<const int2 *>(&s_sxy[m][k0]);
                rzu[m] = *reinterpret_cast<const int2 *>(&s_szu[m][k0]);
                rc2[m] = *reinterpret_cast<const int2 *>(&s_sc2[m][k0]);
              }
#pragma unroll
              for (int u = 0; u < SB; ++u) {
                const int zu0 = u ? rzu[0].y : rzu[0].x;
                const bool mine = (uint32_t)(a - (int)((uint32_t)zu0 >> 16)) < 3u;
                bool in = false;
#pragma unroll
                for (int m = 0; m < 3; ++m)
                  in = in || near(u ? rxy[m].y : rxy[m].x, u ? rzu[m].y : rzu[m].x, u ? rc2[m].y : rc2[m].x);
                *lds16(lbr.wa) = (uint16_t)(nst + n1 + 3 * (k0 + u));
                lbr.wa += in && !mine ? 2u : 0u;
              }
              if (lbr.row_full()) lbr.flush();
            }
          } else {
            for (int k = 0; k < nk; ++k) {
              const int oj = s_uid[k];
              const uint32_t sh = (uint32_t)(exs - oj);
              const bool win = sh < 64u;
              bool in = near(s_qxy[k], s_qzu[k], s_qc2[k]) && !(win && (int32_t)(uint32_t)((exm << (sh & 63u)) >> 32) < 0);
              if (in && !win && exfar)
                for (int e = e0; e < e1; ++e) in = in && (ex_list[e] != oj);
              if (in) lbl.append((uint32_t)(nst + k));
            }
          }
          nst += n1 + 3 * ns3;
        } else {
          // ---- exact mode (single atoms only): a candidate is staged only
          // if some atom needs it
          const int nst0 = nst;
          uint64_t acc = 0ull;
          for (int k = 0; k < nk; ++k) {
            const int oj = s_uid[k];
            const uint32_t sh = (uint32_t)(exs - oj);
            const bool win = sh < 64u;
            bool in = near(s_qxy[k], s_qzu[k], s_qc2[k]) && !(win && (int32_t)(uint32_t)((exm << (sh & 63u)) >> 32) < 0);
            if (in && !win && exfar)
              for (int e = e0; e < e1; ++e) in = in && (ex_list[e] != oj);
            if (__ballot(in)) {
              if (nst < cap) {
                if (in) lbl.append((uint32_t)nst);
                acc |= 1ull << k;
                ++nst;
              } else {
                bad = true;  // staging full even in exact mode: the replica is flagged
              }
            }
          }
          if (keep && ((acc >> at) & 1ull)) stg[nst0 + __popcll(acc & ((1ull << at) - 1ull))] = code;
        }
        __syncthreads();
      }
    }
    if (!full) break;
  }
  // pad the last row of each stream with the inert staging entry (index cap)
  if (active) {
    while (lbl.wa != lbl.base) lbl.append((uint32_t)cap);
    while (lbr.wa != lbr.base) lbr.append((uint32_t)cap);
  }
  // longest list before any clamp (the capacity check at creation reads it)
  int nlj = lbl.rows, nrf = lbr.rows;
  const int cneed = wave_max_i(active ? 8 * (nlj + nrf) : 0);
  if (nlj + nrf > rowcap - 1) {
    // overflow: the replica is flagged; the rows read stay inside the list
    // and were all written by this build (the two streams may have
    // overwritten each other's rows, with staging indices of this build)
    bad = true;
    nlj = min(nlj, rowcap - 1);
    nrf = min(nrf, rowcap - 1 - nlj);
  }
  W.nbcnt[slot] = active ? 8 * (nlj + nrf) : 0;
  W.nblj[slot] = active ? nlj : 0;
  if (lane == 0) {
    W.stage_n[b] = nst;
    W.bctr[b] = make_int4(ox, oy, oz, 0);
  }
  if (__ballot(bad) && lane == 0) {
    if (MODE == 0) atomicOr(&state[r].status, VP_REPLICA_LIST_OVERFLOW);
    else atomicOr(&W.flags[r], 2);
  }
  if (MODE == 0 && lane == 0) {
    atomicMax(&state[r].stage_max, nst);
    atomicMax(&state[r].list_max, cneed);
    if (exact) atomicAdd(&state[r].exact_builds, 1);
  }
  if (!active) return;
  // the new order becomes the state
  W.xq[slot] = xi;
  if (MODE == 0) {
    W.vel[slot] = vel_t[slot];
    W.xref[slot] = xi;
    if (W.tx)
      for (int d = 0; d < 2; ++d) {
        W.tx[d * W.fstride + slot] = tx_t[d * W.fstride + slot];
        W.tv[d * W.fstride + slot] = tv_t[d * W.fstride + slot];
      }
  }
  W.orig[slot] = a;
  W.wrap[slot] = wrap_t[slot];
  W.integ[slot] = integ0[R.uoff + a];
  W.inv[R.uoff + a] = slot;
}

// List entries whose current separation passes the force kernel's predicate,
// as (user i, user j) with i < j.
__global__ __launch_bounds__(kBlk) void k_debug_pairs(const RepInfo *__restrict__ info, Work W,
                                                      const int32_t *__restrict__ tile_rep,
                                                      const int32_t *__restrict__ tile_first,
                                                      int rep, int2 *__restrict__ out,
                                                      unsigned long long cap,
                                                      unsigned long long *__restrict__ counter) {
  const RepInfo &R = info[rep];
  const int b = R.blk0 + blockIdx.x;
  const int tile = b / (kTile / kBlk);
  const int p = tile_first[tile] + (b % (kTile / kBlk)) * kBlk + threadIdx.x;
  if (p >= R.n) return;
  const int slot = R.off + p;
  const int4 xi = W.xq[slot];
  const int wr = W.wrap[slot];
  const int wx = xi.x - unpack_wrap(wr, 0) * R.Lq[0], wy = xi.y - unpack_wrap(wr, 1) * R.Lq[1],
            wz = xi.z - unpack_wrap(wr, 2) * R.Lq[2];
  const int a = W.orig[slot];
  const int cnt = W.nbcnt[slot], nlj = W.nblj[slot], rowcap = R.maxnb >> 3;
  const uint16_t *lst = W.nblist + R.list_off + (int64_t)(b - R.blk0) * R.maxnb * kBlk;
  const uint32_t *stg = W.stage + (int64_t)b * W.stage_stride;
  const int nst = W.stage_n[b];
  for (int k = 0; k < cnt; ++k) {
    const int L0 = lst[list_row(chunk_row(k >> 3, nlj, rowcap), threadIdx.x) * 8 + (k & 7)];
    // an entry names one atom (chunks below nlj) or a three-atom site
    const int na = (k >> 3) < nlj ? 1 : 3;
    for (int m = 0; m < na; ++m) {
    const int L = L0 + m;
    if (L >= nst) continue;
    const uint32_t e = stg[L];
    const int j = (int)(e & 0xffffu);
    const int sx = (int)((e >> 16) & 31) - 16, sy = (int)((e >> 21) & 31) - 16,
              sz = (int)((e >> 26) & 31) - 16;
    const int4 xj = W.xq[R.off + j];
    const float dx = (float)(xj.x + sx * R.Lq[0] - wx), dy = (float)(xj.y + sy * R.Lq[1] - wy),
                dz = (float)(xj.z + sz * R.Lq[2] - wz);
    const int bj = W.orig[R.off + j];
    if (bj <= a) continue;
    if (qr2(dx, dy, dz) < R.rc2q) {
      unsigned long long idx = atomicAdd(counter, 1ull);
      if (idx < cap) out[idx] = make_int2(a, bj);
    }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int xcd_grid(int nb) { return 8 * ((nb + 7) / 8); }

void launch_rebuild(vp_system *s, Work &W, int mode, const float *x_user, hipStream_t st) {
  if (mode == 0) {
    hipLaunchKernelGGL(k_bin<0>, dim3(s->R), dim3(kBinThreads), 0, st, s->info, s->state, W,
                       x_user, s->cellid_t, s->zkey_t, s->fcell_t, s->bucket_t, s->bko_t,
                       s->orig_t, s->cellpos_t, s->step);
    hipLaunchKernelGGL(k_permute<0>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, x_user, s->type0, s->role0,
                       s->orig_t, s->xq_t, s->vel_t, s->wrap_t, s->cellpos_t, s->cellx_t,
                       s->celljw_t, s->tx_t, s->tv_t, s->inv_t);
    hipLaunchKernelGGL(k_list<0>, dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_blocks, s->xq_t, s->vel_t,
                       s->orig_t, s->wrap_t, s->cellx_t, s->celljw_t, s->ex_start, s->ex_list,
                       s->integ0, s->tx_t, s->tv_t, s->inv_t);
  } else {
    hipLaunchKernelGGL(k_bin<1>, dim3(s->R), dim3(kBinThreads), 0, st, s->info, s->state, W,
                       x_user, s->cellid_t, s->zkey_t, s->fcell_t, s->bucket_t, s->bko_t,
                       s->orig_t, s->cellpos_t, s->step);
    hipLaunchKernelGGL(k_permute<1>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, x_user, s->type0, s->role0,
                       s->orig_t, s->xq_t, s->vel_t, s->wrap_t, s->cellpos_t, s->cellx_t,
                       s->celljw_t, s->tx_t, s->tv_t, s->inv_t);
    hipLaunchKernelGGL(k_list<1>, dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_blocks, s->xq_t, s->vel_t,
                       s->orig_t, s->wrap_t, s->cellx_t, s->celljw_t, s->ex_start, s->ex_list,
                       s->integ0, s->tx_t, s->tv_t, s->inv_t);
  }
}

void launch_debug_pairs(vp_system *s, Work &W, int rep, int2 *out, unsigned long long cap,
                        unsigned long long *counter, hipStream_t st) {
  const RepInfo &R = s->info_h[rep];
  hipLaunchKernelGGL(k_debug_pairs, dim3(R.npad / kBlk), dim3(kBlk), 0, st, s->info, W,
                     s->tile_rep, s->tile_first, rep, out, cap, counter);
}

}  // namespace vp
