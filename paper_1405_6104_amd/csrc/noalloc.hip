// vp_forces_noalloc: vp_forces with its evaluation context in a static device
// array instead of memory the library allocates, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The evaluation context (positions in sorted fixed-point order, pair lists,
// staged neighbourhoods, cell index, fixed-point forces, collective-variable
// and energy partials, status flags) of one call is laid out in `scratch`,
// 256-byte aligned piece by piece.  Every piece the call's kernels read is
// written earlier in the same call (the rebuild writes the cell index, the
// lists, the staging and the sorted positions of every slot it later reads and
// sets the status flags; the force, collective-variable and energy kernels
// write every partial their consumers add up), so nothing has to start at
// zero and the contents a previous call left behind are never read.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <string>

#include "vp_internal.h"
#include "vp_launch.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address (it is a host-side stand-in): the device address comes
// from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The current device's copy of the scratch array, looked up once per device.
vp_status scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return vp::set_error(VP_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return vp::set_error(VP_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return vp::set_error(VP_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return VP_OK;
}

// Places the evaluation context of system s at base (or only measures it when
// base is NULL); returns the bytes it spans.
size_t layout(const vp_system *s, unsigned char *base, vp::Work &W) {
  using namespace vp;
  const size_t S = (size_t)s->n_slots, U = (size_t)s->n_users, R = (size_t)s->R, B = (size_t)s->n_blocks;
  const size_t NS = (size_t)(s->n_solute_total > 0 ? s->n_solute_total : 1);
  const size_t CT = (size_t)(s->n_cv_tiles > 0 ? s->n_cv_tiles : 1);
  size_t off = 0;
  auto take = [&](auto **p, size_t count) {
    using T = typename std::remove_pointer<typename std::remove_pointer<decltype(p)>::type>::type;
    *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += (sizeof(T) * (count ? count : 1) + 255) / 256 * 256;
  };
  W = Work{};
  take(&W.xq, S);
  take(&W.integ, S);
  take(&W.orig, S);
  take(&W.wrap, S);
  take(&W.inv, U);
  take(&W.F, 3 * S);
  W.fstride = (int64_t)S;
  take(&W.nbcnt, S);
  take(&W.nblj, S);
  take(&W.nblist, (size_t)s->list_elems);
  take(&W.stage_n, B);
  take(&W.bctr, B);
  W.stage_stride = s->stage_cap_max;
  take(&W.stage, B * (size_t)W.stage_stride);
  take(&W.cell_start, (size_t)s->n_cells);
  take(&W.cell_slots, S);
  take(&W.cell_of, S);
  take(&W.g, NS);
  take(&W.gtile, CT * kCvTile);
  take(&W.ztile, CT);
  take(&W.zpart, R * kMaxCvBlocks);
  take(&W.gpart, R * kMaxCvBlocks);
  take(&W.epart, (size_t)kEp * B);
  take(&W.flags, R);
  return off;
}

}  // namespace

extern "C" vp_status vp_forces_noalloc(vp_system *s, const float *x_dev, float *f_dev, double *energy_dev,
                                       double t, void *hip_stream) {
  if (!s || !x_dev || !f_dev) return vp::set_error(VP_ERR_ARG, "NULL argument");
  vp::Work W;
  const size_t need = layout(s, nullptr, W);
  if (need > kScratchBytes)
    return vp::set_error(VP_ERR_ARG, "vp_forces_noalloc: this system's evaluation context needs " +
                                         std::to_string(need) + " bytes; the static scratch holds " +
                                         std::to_string(kScratchBytes) + " bytes (use vp_forces)");
  void *p = nullptr;
  vp_status st = scratch_address(&p);
  if (st != VP_OK) return st;
  layout(s, static_cast<unsigned char *>(p), W);
  return vp::enqueue_forces(s, W, x_dev, f_dev, energy_dev, t, (hipStream_t)hip_stream);
}
