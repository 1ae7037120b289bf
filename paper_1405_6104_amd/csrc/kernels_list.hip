// Cell binning, deterministic spatial sort and per-atom Verlet lists.
//
// The trajectory state is kept in cell-sorted order per replica.  A rebuild
// (first step, displacement beyond half the skin, or nstlist_max steps) is
// decided on the device, so the kernels of a captured step graph run every
// step and return at once for replicas that keep their list.
//
//   k_bin      one workgroup per replica: cell of every atom (FP64 wrap),
//              counting sort with the within-cell order fixed by the atom's
//              user index (so the sort does not depend on atomic order);
//   k_permute  gathers positions/velocities into the new order;
//   k_list     one thread per atom: scans the distinct cells of its 27-cell
//              stencil in a fixed order and keeps every non-excluded atom
//              within r_cut + skin (16-bit replica-local slot indices, stored
//              [k][slot] so that a wave reads consecutive addresses), then
//              copies its own slot back into the state arrays.
#include "vp_device.h"
#include "vp_launch.h"

namespace vp {

__device__ __forceinline__ int cell_coord(float x, double L, int nc) {
  double xd = (double)x;
  double w = xd - floor(xd / L) * L;
  int k = (int)floor(w * (double)nc / L);
  return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// MODE 0: trajectory (old sorted order, device decides whether to rebuild);
// MODE 1: evaluation from user-order positions x_user (always rebuilds).
template <int MODE>
__global__ __launch_bounds__(kBinThreads) void k_bin(const RepInfo *__restrict__ info,
                                                     RepState *__restrict__ state, Work W,
                                                     const float *__restrict__ x_user,
                                                     const float4 *__restrict__ q0,
                                                     int32_t *__restrict__ cellid_t,
                                                     int32_t *__restrict__ bucket_t,
                                                     int32_t *__restrict__ borig_t,
                                                     int32_t *__restrict__ orig_t,
                                                     int32_t *__restrict__ cell_of,
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
  for (int c = tid; c < R.ncell; c += kBinThreads) s_cnt[c] = 0;
  __syncthreads();
  if (!s_need) return;
  const int off = R.off;
  // cell of each atom in its current (old) position
  for (int p = tid; p < R.n; p += kBinThreads) {
    float x, y, z;
    if (MODE == 0) {
      float4 v = W.xq[off + p];
      x = v.x; y = v.y; z = v.z;
    } else {
      const float *u = x_user + 3ll * (R.uoff + p);
      x = u[0]; y = u[1]; z = u[2];
    }
    int cx = cell_coord(x, R.Ld[0], R.nc[0]);
    int cy = cell_coord(y, R.Ld[1], R.nc[1]);
    int cz = cell_coord(z, R.Ld[2], R.nc[2]);
    int c = (cz * R.nc[1] + cy) * R.nc[0] + cx;
    cellid_t[off + p] = c;
    atomicAdd(&s_cnt[c], 1);
  }
  __syncthreads();
  // exclusive scan of the cell counts (4 cells per thread, then the waves)
  {
    int base = tid * 4, loc[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int c = base + k;
      loc[k] = (c < R.ncell) ? s_cnt[c] : 0;
      sum += loc[k];
    }
    int incl = sum;
    int lane = tid & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (lane == 63) s_wsum[tid >> 6] = incl;
    __syncthreads();
    int wpre = 0;
    for (int w = 0; w < (tid >> 6); ++w) wpre += s_wsum[w];
    int ex = wpre + incl - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int c = base + k;
      if (c < R.ncell) {
        s_start[c] = ex;
        ex += loc[k];
      }
    }
    if (tid == 0) s_start[R.ncell] = R.n;
  }
  __syncthreads();
  for (int c = tid; c <= R.ncell; c += kBinThreads) W.cell_start[R.cell0 + c] = s_start[c];
  for (int c = tid; c < R.ncell; c += kBinThreads) s_cnt[c] = s_start[c];
  __syncthreads();
  // unordered scatter into cell buckets
  for (int p = tid; p < R.n; p += kBinThreads) {
    int c = cellid_t[off + p];
    int pos = atomicAdd(&s_cnt[c], 1);
    bucket_t[off + pos] = p;
    borig_t[off + pos] = (MODE == 0) ? W.orig[off + p] : p;
  }
  __syncthreads();
  // within a cell, order by user index: rank = #members with a smaller index
  for (int s = tid; s < R.n; s += kBinThreads) {
    int c = cellid_t[off + bucket_t[off + s]];
    int me = borig_t[off + s];
    int rank = 0;
    for (int q = s_start[c]; q < s_start[c + 1]; ++q) rank += (borig_t[off + q] < me);
    int ns = s_start[c] + rank;
    orig_t[off + ns] = me;
    cell_of[off + ns] = c;
  }
}

// New slot -> source: old slot (trajectory) found through the old inverse
// map, or the user index (evaluation).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_permute(const RepInfo *__restrict__ info,
                                                    const RepState *__restrict__ state, Work W,
                                                    const int32_t *__restrict__ tile_rep,
                                                    const int32_t *__restrict__ tile_first,
                                                    int ntiles, const float *__restrict__ x_user,
                                                    const float4 *__restrict__ q0,
                                                    const int32_t *__restrict__ orig_t,
                                                    float4 *__restrict__ xq_t,
                                                    float4 *__restrict__ vel_t) {
  int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  if (MODE == 0 ? !state[r].rebuild : !W.flags[r]) return;
  int p = tile_first[tile] + threadIdx.x;
  if (p >= R.n) return;
  int slot = R.off + p;
  int a = orig_t[slot];
  if (MODE == 0) {
    int old = W.inv[R.uoff + a];
    xq_t[slot] = W.xq[old];
    vel_t[slot] = W.vel[old];
  } else {
    const float *u = x_user + 3ll * (R.uoff + a);
    xq_t[slot] = make_float4(u[0], u[1], u[2], q0[R.uoff + a].w);
  }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_list(const RepInfo *__restrict__ info,
                                                 RepState *__restrict__ state, Work W,
                                                 const int32_t *__restrict__ tile_rep,
                                                 const int32_t *__restrict__ tile_first, int ntiles,
                                                 const float4 *__restrict__ xq_t,
                                                 const float4 *__restrict__ vel_t,
                                                 const int32_t *__restrict__ orig_t,
                                                 const int32_t *__restrict__ cell_of,
                                                 const int32_t *__restrict__ ex_start,
                                                 const int32_t *__restrict__ ex_list,
                                                 const float2 *__restrict__ prm0,
                                                 const float4 *__restrict__ integ0) {
  int tile = xcd_tile(blockIdx.x, ntiles);
  if (tile < 0) return;
  const int r = tile_rep[tile];
  const RepInfo &R = info[r];
  if (MODE == 0 ? !state[r].rebuild : !W.flags[r]) return;
  int p = tile_first[tile] + threadIdx.x;
  if (p >= R.npad) return;
  int slot = R.off + p;
  if (p >= R.n) {
    W.nbcnt[slot] = 0;
    return;
  }
  const int a = orig_t[slot];
  const float4 xi = xq_t[slot];
  const int c = cell_of[slot];
  const int cx = c % R.nc[0], cy = (c / R.nc[0]) % R.nc[1], cz = c / (R.nc[0] * R.nc[1]);
  const int e0 = ex_start[R.uoff + a], e1 = ex_start[R.uoff + a + 1];
  uint16_t *out = W.nblist + R.list_off + p;
  const int npad = R.npad, maxnb = R.maxnb;
  int cnt = 0;
  const int nz = R.nc[2] >= 3 ? 3 : R.nc[2];
  const int ny = R.nc[1] >= 3 ? 3 : R.nc[1];
  const int nx = R.nc[0] >= 3 ? 3 : R.nc[0];
  for (int iz = 0; iz < nz; ++iz) {
    int oz = (R.nc[2] >= 3) ? (cz + iz - 1 + R.nc[2]) % R.nc[2] : (cz + iz) % R.nc[2];
    for (int iy = 0; iy < ny; ++iy) {
      int oy = (R.nc[1] >= 3) ? (cy + iy - 1 + R.nc[1]) % R.nc[1] : (cy + iy) % R.nc[1];
      for (int ix = 0; ix < nx; ++ix) {
        int ox = (R.nc[0] >= 3) ? (cx + ix - 1 + R.nc[0]) % R.nc[0] : (cx + ix) % R.nc[0];
        int nb = (oz * R.nc[1] + oy) * R.nc[0] + ox;
        int j0 = W.cell_start[R.cell0 + nb], j1 = W.cell_start[R.cell0 + nb + 1];
        for (int j = j0; j < j1; ++j) {
          if (j == p) continue;
          float dx, dy, dz;
          float r2 = pair_r2(xi, xq_t[R.off + j], R, dx, dy, dz);
          if (!(r2 < R.rl2)) continue;
          int oj = orig_t[R.off + j];
          bool ex = false;
          for (int e = e0; e < e1; ++e) ex |= (ex_list[e] == oj);
          if (ex) continue;
          if (cnt < maxnb) out[(int64_t)cnt * npad] = (uint16_t)j;
          ++cnt;
        }
      }
    }
  }
  if (cnt > maxnb) {
    if (MODE == 0) atomicOr(&state[r].status, VP_REPLICA_LIST_OVERFLOW);
    cnt = maxnb;
  }
  W.nbcnt[slot] = cnt;
  // the new order becomes the state
  W.xq[slot] = xi;
  if (MODE == 0) {
    W.vel[slot] = vel_t[slot];
    W.xref[slot] = xi;
  }
  W.orig[slot] = a;
  W.prm[slot] = prm0[R.uoff + a];
  W.integ[slot] = integ0[R.uoff + a];
  W.inv[R.uoff + a] = slot;
}

// List entries whose current separation passes the force kernel's predicate,
// as (user i, user j) with i < j.
__global__ __launch_bounds__(kBlock) void k_debug_pairs(const RepInfo *__restrict__ info, Work W,
                                                        int rep, int2 *__restrict__ out,
                                                        unsigned long long cap,
                                                        unsigned long long *__restrict__ counter) {
  const RepInfo &R = info[rep];
  int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= R.n) return;
  int slot = R.off + p;
  float4 xi = W.xq[slot];
  int a = W.orig[slot];
  int cnt = W.nbcnt[slot];
  for (int k = 0; k < cnt; ++k) {
    int j = W.nblist[R.list_off + (int64_t)k * R.npad + p];
    int b = W.orig[R.off + j];
    if (b <= a) continue;
    float dx, dy, dz;
    float r2 = pair_r2(xi, W.xq[R.off + j], R, dx, dy, dz);
    if (r2 < R.rc2) {
      unsigned long long idx = atomicAdd(counter, 1ull);
      if (idx < cap) out[idx] = make_int2(a, b);
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
                       x_user, s->q0, s->cellid_t, s->bucket_t, s->borig_t, s->orig_t,
                       W.cell_of, s->step);
    hipLaunchKernelGGL(k_permute<0>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, x_user, s->q0,
                       s->orig_t, s->xq_t, s->vel_t);
    hipLaunchKernelGGL(k_list<0>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, s->xq_t, s->vel_t,
                       s->orig_t, W.cell_of, s->ex_start, s->ex_list, s->prm0, s->integ0);
  } else {
    hipLaunchKernelGGL(k_bin<1>, dim3(s->R), dim3(kBinThreads), 0, st, s->info, s->state, W,
                       x_user, s->q0, s->cellid_t, s->bucket_t, s->borig_t, s->orig_t,
                       W.cell_of, s->step);
    hipLaunchKernelGGL(k_permute<1>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, x_user, s->q0,
                       s->orig_t, s->xq_t, s->vel_t);
    hipLaunchKernelGGL(k_list<1>, dim3(xcd_grid(s->n_tiles)), dim3(kBlock), 0, st, s->info,
                       s->state, W, s->tile_rep, s->tile_first, s->n_tiles, s->xq_t, s->vel_t,
                       s->orig_t, W.cell_of, s->ex_start, s->ex_list, s->prm0, s->integ0);
  }
}

void launch_debug_pairs(vp_system *s, Work &W, int rep, int2 *out, unsigned long long cap,
                        unsigned long long *counter, hipStream_t st) {
  int n = s->info_h[rep].n;
  hipLaunchKernelGGL(k_debug_pairs, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, s->info,
                     W, rep, out, cap, counter);
}

}  // namespace vp
