// fdtd_debye.hip -- fused one-step pass of grids with Debye media (gfx950).
//
// The fused tile of fdtd_tile.h with its Debye switch on: the owner of each
// E node also advances that node's pole currents, in place (they are
// node-local, so one thread per node and step touches them).  The field sets
// ping-pong as in the plain fused pass.  Compared with the split pass (H over
// the grid, then E), E and H are read once per step instead of twice, and
// one launch does the whole step.  The Debye terms go through debye_load and
// debye_apply, as in the split pass, so the two agree bit for bit.
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"
#include "fdtd_tile.h"

namespace mi355fdtd {

// Prefetch distance of the Debye tiles (planes).
constexpr int DPF = 2;

// Dynamic LDS (FP32, 1-byte classes): the pole factors of every class, then
// the per-class flags.
template <typename T, typename CI>
constexpr bool dlds() { return sizeof(CI) == 1 && sizeof(T) == 4; }
template <typename T, typename CI>
size_t dlds_bytes(int ncls) {
  return dlds<T, CI>() ? (size_t)ncls * (D_STRIDE * sizeof(T) + 1) : 0;
}

template <typename T, typename CI, bool PML>
__global__ __launch_bounds__(512) void k_fused_debye(GridView<T> g, DebyeView<T> d, int step, int kz, int ntx,
                                                     int nty) {
  step = gstep(g, step);
  __shared__ FusedSmem<T, 64, 8> sm;
  extern __shared__ __align__(16) unsigned char dsm[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_x = tile % ntx, rest = tile / ntx;
  const int k0 = (rest / nty) * kz;
  fused_tile<T, CI, PML, 64, 8, 7, true, DPF>(g, sm, tile_x * 64, (rest % nty) * 8, k0, min(k0 + kz, g.nz), step, &d,
                                         (T*)dsm, dsm + (size_t)g.ncls * D_STRIDE * sizeof(T));
}

// Tile list of a grid with a CPML, grouped by the slabs a tile reaches (as
// for the plain fused lists: AX masks the CPML axes compiled in).
template <typename T, typename CI, int TX, int AX>
__global__ __launch_bounds__(TX * 8) void k_fused_list_debye(GridView<T> g, DebyeView<T> d,
                                                            const int4* __restrict__ tiles, int step) {
  step = gstep(g, step);
  __shared__ FusedSmem<T, TX, 8> sm;
  extern __shared__ __align__(16) unsigned char dsm[];
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  fused_tile<T, CI, true, TX, 8, AX, true, DPF>(g, sm, t.x, t.y, t.z, t.w, step, &d, (T*)dsm,
                                           dsm + (size_t)g.ncls * D_STRIDE * sizeof(T));
}

template <typename T, typename CI>
hipError_t debye_lists(const GridView<T>& g, const DebyeView<T>& d, int step, const int4* tiles, const int* counts,
                       hipStream_t st, hipStream_t st2) {
  if (sizeof(CI) == 1 && g.ncls > 256) return hipErrorInvalidValue;
  constexpr bool D = sizeof(T) == 8;
  const size_t dyn = dlds_bytes<T, CI>(g.ncls);
  const int4* t = tiles;
  if (counts[0] > 0)
    hipLaunchKernelGGL((k_fused_list_debye<T, CI, 64, D ? 7 : 4>), dim3((unsigned)counts[0]), dim3(512), dyn, st, g,
                       d, t, step);
  t += counts[0];
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_fused_list_debye<T, CI, 32, D ? 7 : 5>), dim3((unsigned)counts[1]), dim3(256), dyn, st2,
                       g, d, t, step);
  t += counts[1];
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_fused_list_debye<T, CI, 64, D ? 7 : 6>), dim3((unsigned)counts[2]), dim3(512), dyn, st2,
                       g, d, t, step);
  t += counts[2];
  if (counts[3] > 0)
    hipLaunchKernelGGL((k_fused_list_debye<T, CI, 32, 7>), dim3((unsigned)counts[3]), dim3(256), dyn, st2, g, d, t,
                       step);
  return hipGetLastError();
}

template <typename T, typename CI>
hipError_t debye_fused(const GridView<T>& g, const DebyeView<T>& d, int step, int kz, hipStream_t st) {
  const int ntx = (g.nx + 63) / 64, nty = (g.ny + 7) / 8, ntz = (g.nz + kz - 1) / kz;
  const long long nb = (long long)ntx * nty * ntz;
  if (nb > 0x7fffffff || (sizeof(CI) == 1 && g.ncls > 256)) return hipErrorInvalidValue;
  const size_t dyn = dlds_bytes<T, CI>(g.ncls);
  if (g.npml > 0)
    hipLaunchKernelGGL((k_fused_debye<T, CI, true>), dim3((unsigned)nb), dim3(512), dyn, st, g, d, step, kz, ntx,
                       nty);
  else
    hipLaunchKernelGGL((k_fused_debye<T, CI, false>), dim3((unsigned)nb), dim3(512), dyn, st, g, d, step, kz, ntx,
                       nty);
  return hipGetLastError();
}

template <typename T>
hipError_t debye_any(const GridView<T>& g, const DebyeView<T>& d, int cls16, int step, int tile_z, const int4* tiles,
                     const int* counts, hipStream_t st, hipStream_t st2) {
  if (tiles)
    return cls16 ? debye_lists<T, uint16_t>(g, d, step, tiles, counts, st, st2)
                 : debye_lists<T, uint8_t>(g, d, step, tiles, counts, st, st2);
  const int kz = tile_z > 0 ? tile_z : 32;
  return cls16 ? debye_fused<T, uint16_t>(g, d, step, kz, st) : debye_fused<T, uint8_t>(g, d, step, kz, st);
}

int launch_fused_debye(int prec, const void* view, const void* dview, int cls16, int step, int tile_z,
                       const void* tiles, const int* counts, void* stream, void* stream2) {
  hipStream_t st = (hipStream_t)stream, st2 = (hipStream_t)stream2;
  const int4* t = (const int4*)tiles;
  hipError_t e;
  if (prec == 64)
    e = debye_any<double>(*(const GridView<double>*)view, *(const DebyeView<double>*)dview, cls16, step, tile_z, t,
                          counts, st, st2);
  else
    e = debye_any<float>(*(const GridView<float>*)view, *(const DebyeView<float>*)dview, cls16, step, tile_z, t,
                         counts, st, st2);
  return (int)e;
}

}  // namespace mi355fdtd
