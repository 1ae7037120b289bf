// Cell binning, deterministic spatial sort and per-block neighbourhood lists.
//
// Coordinates are 32-bit fixed point (unit 2^-24 nm), so image shifts by the
// box edge are exact integer additions.  The trajectory state is kept sorted
// along serpentine xy columns, z inside a column, so 64 consecutive slots form
// a compact block.  A rebuild (first step, largest displacement since the last
// build reaching half the skin, or nstlist_max steps) is decided on the
// device, so the kernels of a captured step graph run every step and return
// at once for replicas that keep their lists.
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
// block.  A second index lists the slots of every fine cell (~0.45 nm) in
// ascending order for the candidate search of the list build.  Both orders
// are fixed by keys, not by the order of atomic operations.
// MODE 0: trajectory (old sorted order, device decides whether to rebuild);
// MODE 1: evaluation from user-order FP32 positions x_user (always rebuilds).
template <int MODE>
__global__ __launch_bounds__(kBinThreads) void k_bin(const RepInfo *__restrict__ info,
                                                     RepState *__restrict__ state, Work W,
                                                     const float *__restrict__ x_user,
                                                     int32_t *__restrict__ colid_t,
                                                     int32_t *__restrict__ zkey_t,
                                                     int32_t *__restrict__ fcell_t,
                                                     int32_t *__restrict__ bucket_t,
                                                     int32_t *__restrict__ bkey_t,
                                                     int32_t *__restrict__ borig_t,
                                                     int32_t *__restrict__ orig_t,
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
      need = S.force_rebuild || (md >= R.half_skin_margin) || (n - S.last_build >= R.nstlist_max);
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
  const int ncols = R.ncol[0] * R.ncol[1];
  for (int c = tid; c < ncols; c += kBinThreads) s_cnt[c] = 0;
  __syncthreads();
  if (!s_need) return;
  const int off = R.off;
  // ---- keys of every atom (old slot order)
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
    int fx = (int)((wx * R.nc[0]) / R.Lq[0]), fy = (int)((wy * R.nc[1]) / R.Lq[1]),
        fz = (int)((wz * R.nc[2]) / R.Lq[2]);
    fx = min(fx, R.nc[0] - 1);
    fy = min(fy, R.nc[1] - 1);
    fz = min(fz, R.nc[2] - 1);
    colid_t[off + p] = col;
    zkey_t[off + p] = (col & 1) ? -(int)wz : (int)wz;
    fcell_t[off + p] = (fz * R.nc[1] + fy) * R.nc[0] + fx;
    atomicAdd(&s_cnt[col], 1);
  }
  __syncthreads();
  block_scan(s_cnt, s_start, ncols, R.n, s_wsum);
  for (int c = tid; c < ncols; c += kBinThreads) s_cnt[c] = s_start[c];
  __syncthreads();
  for (int p = tid; p < R.n; p += kBinThreads) {
    const int col = colid_t[off + p];
    const int pos = atomicAdd(&s_cnt[col], 1);
    bucket_t[off + pos] = p;
    bkey_t[off + pos] = zkey_t[off + p];
    borig_t[off + pos] = (MODE == 0) ? W.orig[off + p] : p;
  }
  __syncthreads();
  // ---- rank inside a column by (z key, user index)
  for (int s = tid; s < R.n; s += kBinThreads) {
    const int p = bucket_t[off + s];
    const int col = colid_t[off + p];
    const int key = bkey_t[off + s], me = borig_t[off + s];
    int rank = 0;
    for (int q = s_start[col]; q < s_start[col + 1]; ++q) {
      const int kq = bkey_t[off + q];
      rank += (kq < key) || (kq == key && borig_t[off + q] < me);
    }
    const int ns = s_start[col] + rank;
    orig_t[off + ns] = me;
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
    int rank = 0;
    for (int t = s_start[c]; t < s_start[c + 1]; ++t) rank += (bucket_t[off + t] < s);
    W.cell_slots[off + s_start[c] + rank] = s;
  }
}

// New slot -> source (old slot through the old inverse map, or user index);
// also records the atom's periodic image at this build.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_permute(const RepInfo *__restrict__ info,
                                                    const RepState *__restrict__ state, Work W,
                                                    const int32_t *__restrict__ tile_rep,
                                                    const int32_t *__restrict__ tile_first,
                                                    int ntiles, const float *__restrict__ x_user,
                                                    const int32_t *__restrict__ type0,
                                                    const int32_t *__restrict__ orig_t,
                                                    int4 *__restrict__ xq_t,
                                                    float4 *__restrict__ vel_t,
                                                    int32_t *__restrict__ wrap_t) {
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
  } else {
    const float *u = x_user + 3ll * (R.uoff + a);
    x = make_int4((int)__builtin_rintf(u[0] * kQf), (int)__builtin_rintf(u[1] * kQf),
                  (int)__builtin_rintf(u[2] * kQf), type0[R.uoff + a]);
  }
  xq_t[slot] = x;
  int kx = (int)floordiv(x.x, R.Lq[0]), ky = (int)floordiv(x.y, R.Lq[1]),
      kz = (int)floordiv(x.z, R.Lq[2]);
  wrap_t[slot] = pack_wrap(kx, ky, kz);
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

template <int MODE>
__global__ __launch_bounds__(kBlk) void k_list(const RepInfo *__restrict__ info,
                                               RepState *__restrict__ state, Work W,
                                               const int32_t *__restrict__ tile_rep,
                                               const int32_t *__restrict__ tile_first, int nblk,
                                               const int4 *__restrict__ xq_t,
                                               const float4 *__restrict__ vel_t,
                                               const int32_t *__restrict__ orig_t,
                                               const int32_t *__restrict__ wrap_t,
                                               const int32_t *__restrict__ ex_start,
                                               const int32_t *__restrict__ ex_list,
                                               const float4 *__restrict__ integ0) {
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
    if (lane == 0) W.stage_n[b] = 0;
    return;
  }
  const int Lx = R.Lq[0], Ly = R.Lq[1], Lz = R.Lq[2];
  int4 xi = make_int4(0, 0, 0, 0);
  int wx = 0, wy = 0, wz = 0, a = -1, e0 = 0, e1 = 0;
  if (active) {
    xi = xq_t[slot];
    const int wr = wrap_t[slot];
    wx = xi.x - unpack_wrap(wr, 0) * Lx;
    wy = xi.y - unpack_wrap(wr, 1) * Ly;
    wz = xi.z - unpack_wrap(wr, 2) * Lz;
    a = orig_t[slot];
    e0 = ex_start[R.uoff + a];
    e1 = ex_start[R.uoff + a + 1];
  }
  // bounding box of the block (wrapped frame)
  const int big = 0x7fffffff;
  const int bx0 = wave_min_i(active ? wx : big), bx1 = wave_max_i(active ? wx : -big);
  const int by0 = wave_min_i(active ? wy : big), by1 = wave_max_i(active ? wy : -big);
  const int bz0 = wave_min_i(active ? wz : big), bz1 = wave_max_i(active ? wz : -big);
  const long long rl = R.rlq;
  const int ux0 = (int)floordiv(((long long)bx0 - rl) * R.nc[0], Lx);
  const int ux1 = (int)floordiv(((long long)bx1 + rl) * R.nc[0], Lx);
  const int uy0 = (int)floordiv(((long long)by0 - rl) * R.nc[1], Ly);
  const int uy1 = (int)floordiv(((long long)by1 + rl) * R.nc[1], Ly);
  const int uz0 = (int)floordiv(((long long)bz0 - rl) * R.nc[2], Lz);
  const int uz1 = (int)floordiv(((long long)bz1 + rl) * R.nc[2], Lz);
  const double rl2d = (double)rl * (double)rl;
  const int lb = b - R.blk0;
  uint16_t *lst = W.nblist + R.list_off + (int64_t)lb * R.maxnb * kBlk;
  uint32_t *stg = W.stage + (int64_t)b * kMaxStage;
  const int cap = R.stage_cap, maxnb = R.maxnb;
  int nst = 0, cnt = 0;
  bool bad = false;
  for (int uz = uz0; uz <= uz1; ++uz) {
    const int iz = (int)floordiv(uz, R.nc[2]);
    const int cz = uz - iz * R.nc[2];
    // gap between the cell's slab and the block box along z (coordinate units)
    const long long zl = floordiv((long long)uz * Lz, R.nc[2]), zh = floordiv((long long)(uz + 1) * Lz, R.nc[2]);
    const double gz = (double)max(0ll, max(zl - bz1, (long long)bz0 - zh));
    for (int uy = uy0; uy <= uy1; ++uy) {
      const int iy = (int)floordiv(uy, R.nc[1]);
      const int cy = uy - iy * R.nc[1];
      const long long yl = floordiv((long long)uy * Ly, R.nc[1]), yh = floordiv((long long)(uy + 1) * Ly, R.nc[1]);
      const double gy = (double)max(0ll, max(yl - by1, (long long)by0 - yh));
      if (gz * gz + gy * gy > rl2d) continue;
      for (int ux = ux0; ux <= ux1; ++ux) {
        const int ix = (int)floordiv(ux, R.nc[0]);
        const int cx = ux - ix * R.nc[0];
        const long long xl = floordiv((long long)ux * Lx, R.nc[0]), xh = floordiv((long long)(ux + 1) * Lx, R.nc[0]);
        const double gx = (double)max(0ll, max(xl - bx1, (long long)bx0 - xh));
        if (gz * gz + gy * gy + gx * gx > rl2d) continue;
        const int cell = (cz * R.nc[1] + cy) * R.nc[0] + cx;
        const int q0 = W.cell_start[R.cell0 + cell], q1 = W.cell_start[R.cell0 + cell + 1];
        const bool self_image = (ix == 0 && iy == 0 && iz == 0);
        for (int q = q0; q < q1; ++q) {
          const int j = W.cell_slots[R.off + q];
          const int4 xj = xq_t[R.off + j];
          const int wj = wrap_t[R.off + j];
          const int sx = ix - unpack_wrap(wj, 0), sy = iy - unpack_wrap(wj, 1),
                    sz = iz - unpack_wrap(wj, 2);
          const int px = xj.x + sx * Lx, py = xj.y + sy * Ly, pz = xj.z + sz * Lz;
          const float dx = (float)(px - wx), dy = (float)(py - wy), dz = (float)(pz - wz);
          bool in = active && (qr2(dx, dy, dz) < R.rl2q) && !(self_image && j == p);
          if (in) {
            const int oj = orig_t[R.off + j];
            for (int e = e0; e < e1; ++e) in = in && (ex_list[e] != oj);
          }
          if (__ballot(in)) {
            if (nst < cap) {
              if (lane == 0)
                stg[nst] = (uint32_t)j | ((uint32_t)((sx + 16) & 31) << 16) |
                           ((uint32_t)((sy + 16) & 31) << 21) | ((uint32_t)((sz + 16) & 31) << 26);
              if (in) {
                if (cnt < maxnb) lst[(((cnt >> 3) * kBlk) + lane) * 8 + (cnt & 7)] = (uint16_t)nst;
                ++cnt;  // entries past maxnb are counted only to flag the overflow
              }
              ++nst;
            } else {
              bad = true;  // staging full: the candidate is dropped and the replica flagged
            }
            bad = bad || (sx < -16 || sx > 15 || sy < -16 || sy > 15 || sz < -16 || sz > 15);
          }
        }
      }
    }
  }
  if (cnt > maxnb - 8) {
    bad = true;
    cnt = maxnb - 8;
  }
  if (active) {
    // pad to a multiple of 8 with the inert staging entry (index cap)
    while (cnt & 7) {
      lst[(((cnt >> 3) * kBlk) + lane) * 8 + (cnt & 7)] = (uint16_t)cap;
      ++cnt;
    }
  }
  W.nbcnt[slot] = active ? cnt : 0;
  if (lane == 0) W.stage_n[b] = nst;
  if (__ballot(bad) && lane == 0) {
    if (MODE == 0) atomicOr(&state[r].status, VP_REPLICA_LIST_OVERFLOW);
    else atomicOr(&W.flags[r], 2);
  }
  if (!active) return;
  // the new order becomes the state
  W.xq[slot] = xi;
  if (MODE == 0) {
    W.vel[slot] = vel_t[slot];
    W.xref[slot] = xi;
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
  const int cnt = W.nbcnt[slot];
  const uint16_t *lst = W.nblist + R.list_off + (int64_t)(b - R.blk0) * R.maxnb * kBlk;
  const uint32_t *stg = W.stage + (int64_t)b * kMaxStage;
  const int nst = W.stage_n[b];
  for (int k = 0; k < cnt; ++k) {
    const int L = lst[(((k >> 3) * kBlk) + threadIdx.x) * 8 + (k & 7)];
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int xcd_grid(int nb) { return 8 * ((nb + 7) / 8); }

void launch_rebuild(vp_system *s, Work &W, int mode, const float *x_user, hipStream_t st) {
  if (mode == 0) {
    hipLaunchKernelGGL(k_bin<0>, dim3(s->R), dim3(kBinThreads), 0, st, s->info, s->state, W,
                       x_user, s->cellid_t, s->zkey_t, s->fcell_t, s->bucket_t, s->bkey_t,
                       s->borig_t, s->orig_t, s->step);
    hipLaunchKernelGGL(k_permute<0>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, x_user, s->type0,
                       s->orig_t, s->xq_t, s->vel_t, s->wrap_t);
    hipLaunchKernelGGL(k_list<0>, dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_blocks, s->xq_t, s->vel_t,
                       s->orig_t, s->wrap_t, s->ex_start, s->ex_list, s->integ0);
  } else {
    hipLaunchKernelGGL(k_bin<1>, dim3(s->R), dim3(kBinThreads), 0, st, s->info, s->state, W,
                       x_user, s->cellid_t, s->zkey_t, s->fcell_t, s->bucket_t, s->bkey_t,
                       s->borig_t, s->orig_t, s->step);
    hipLaunchKernelGGL(k_permute<1>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, x_user, s->type0,
                       s->orig_t, s->xq_t, s->vel_t, s->wrap_t);
    hipLaunchKernelGGL(k_list<1>, dim3(xcd_grid(s->n_blocks)), dim3(kBlk), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_blocks, s->xq_t, s->vel_t,
                       s->orig_t, s->wrap_t, s->ex_start, s->ex_list, s->integ0);
  }
}

void launch_debug_pairs(vp_system *s, Work &W, int rep, int2 *out, unsigned long long cap,
                        unsigned long long *counter, hipStream_t st) {
  const RepInfo &R = s->info_h[rep];
  hipLaunchKernelGGL(k_debug_pairs, dim3(R.npad / kBlk), dim3(kBlk), 0, st, s->info, W,
                     s->tile_rep, s->tile_first, rep, out, cap, counter);
}

}  // namespace vp
