// fdtd_kernels.hip -- HIP kernels of the Yee FDTD step for gfx950.
//
// Layout (all device memory lives in the caller's workspace): each field
// component is an nx*ny*nz array, x fastest, holding the component owned by
// node (i, j, k).  Values on the upper walls (index n along an axis) are not
// stored: they are the zero tangential E of a perfect conductor or the zero
// normal H next to it, so reads past the last node return 0.  Each node
// carries a 1- or 2-byte coefficient class id; the class table holds the 9
// coefficients of the node's six components.
//
// Variants:
//   split  two passes (H over the grid, then E), in place;
//   fused  one pass per step over x-y tiles marching up z; each block
//          recomputes the H it needs on a one-node low-side halo; reads one
//          field set and writes the other;
//   tb2    one pass per two steps (temporal blocking): 60 x TY output tiles
//          in 64 x (TY+4) regions, four stages per plane;
// each also as tile lists grouped by the CPML slabs the tiles reach, and
// batched over many grids.  All evaluate every component through h_core /
// e_core of fdtd_tile.h (with the arithmetic of yee_update.h) and are compiled with FP
// contraction off, so they agree bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fdtd_dev.h"
#include "fdtd_tile.h"
#include "yee_update.h"

namespace mi355fdtd {

// ---------------------------------------------------------------------------
// split variant: two in-place passes
// ---------------------------------------------------------------------------

template <typename T, typename CI, bool PML, int NB>
__global__ __launch_bounds__(NB) void k_h_split(GridView<T> g) {
  // node of the xy plane, x fastest.  On small planes (NB 256) each XCD takes
  // a contiguous band of the plane, so a block's neighbour row was just read
  // into the same L2 (5% faster on a 100 x 100 plane, 5.5% slower on a
  // 512 x 512 one, where the blocks keep their dealt order).
  const unsigned t =
      (unsigned)(NB == 256 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x) * (unsigned)NB + threadIdx.x;
  if (t >= (unsigned)g.sxy) return;
  const int i = (int)(t % (unsigned)g.nx), j = (int)(t / (unsigned)g.nx);
  const int k = blockIdx.y;
  const unsigned n = (unsigned)i + (unsigned)g.nx * ((unsigned)j + (unsigned)g.ny * (unsigned)k);
  const T* cf = g.ctab + (int)ldg((const CI*)g.cls, n) * K_STRIDE;
  const T ex = ldg(g.fi[0], n), ey = ldg(g.fi[1], n), ez = ldg(g.fi[2], n);
  const T ex_j = (j + 1 < g.ny) ? ldg(g.fi[0], n + (unsigned)g.nx) : T(0);
  const T ex_k = (k + 1 < g.nz) ? ldg(g.fi[0], n + (unsigned)g.sxy) : T(0);
  const T ey_i = (i + 1 < g.nx) ? ldg(g.fi[1], n + 1) : T(0);
  const T ey_k = (k + 1 < g.nz) ? ldg(g.fi[1], n + (unsigned)g.sxy) : T(0);
  const T ez_i = (i + 1 < g.nx) ? ldg(g.fi[2], n + 1) : T(0);
  const T ez_j = (j + 1 < g.ny) ? ldg(g.fi[2], n + (unsigned)g.nx) : T(0);
  const T hold[3] = {ldg(g.fi[3], n), ldg(g.fi[4], n), ldg(g.fi[5], n)};
  T h[3];
  h_point<T, PML>(g, i, j, k, cf, ex, ey, ez, ex_j, ex_k, ey_i, ey_k, ez_i, ez_j, hold, true, h);
  stg(g.fo[3], n, h[0]);
  stg(g.fo[4], n, h[1]);
  stg(g.fo[5], n, h[2]);
}

template <typename T, typename CI, bool PML, int NB>
__global__ __launch_bounds__(NB) void k_e_split(GridView<T> g, int step) {
  step = gstep(g, step);
  // node of the xy plane, x fastest.  On small planes (NB 256) each XCD takes
  // a contiguous band of the plane, so a block's neighbour row was just read
  // into the same L2 (5% faster on a 100 x 100 plane, 5.5% slower on a
  // 512 x 512 one, where the blocks keep their dealt order).
  const unsigned t =
      (unsigned)(NB == 256 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x) * (unsigned)NB + threadIdx.x;
  if (t >= (unsigned)g.sxy) return;
  const int i = (int)(t % (unsigned)g.nx), j = (int)(t / (unsigned)g.nx);
  const int k = blockIdx.y;
  const unsigned n = (unsigned)i + (unsigned)g.nx * ((unsigned)j + (unsigned)g.ny * (unsigned)k);
  const T* cf = g.ctab + (int)ldg((const CI*)g.cls, n) * K_STRIDE;
  const T hx = ldg(g.fi[3], n), hy = ldg(g.fi[4], n), hz = ldg(g.fi[5], n);
  const T hx_j = (j > 0) ? ldg(g.fi[3], n - (unsigned)g.nx) : T(0);
  const T hx_k = (k > 0) ? ldg(g.fi[3], n - (unsigned)g.sxy) : T(0);
  const T hy_i = (i > 0) ? ldg(g.fi[4], n - 1) : T(0);
  const T hy_k = (k > 0) ? ldg(g.fi[4], n - (unsigned)g.sxy) : T(0);
  const T hz_i = (i > 0) ? ldg(g.fi[5], n - 1) : T(0);
  const T hz_j = (j > 0) ? ldg(g.fi[5], n - (unsigned)g.nx) : T(0);
  const T eold[3] = {ldg(g.fi[0], n), ldg(g.fi[1], n), ldg(g.fi[2], n)};
  T e[3];
  const SrcRange sr = src_node(g, i, j, k);
  e_point<T, PML>(g, i, j, k, n, cf, hx, hy, hz, hx_j, hx_k, hy_i, hy_k, hz_i, hz_j, eold, step, e, sr.lo, sr.hi);
  stg(g.fo[0], n, e[0]);
  stg(g.fo[1], n, e[1]);
  stg(g.fo[2], n, e[2]);
}

// Split E update in Debye media: the plain update, then the pole currents.
// Nodes whose class has no pole term (air, walls, wire edges) skip them, so
// their J stays 0 without traffic.
template <typename T, typename CI, bool PML, int NB>
__global__ __launch_bounds__(NB) void k_e_split_debye(GridView<T> g, DebyeView<T> d, int step) {
  step = gstep(g, step);
  // node of the xy plane, x fastest.  On small planes (NB 256) each XCD takes
  // a contiguous band of the plane, so a block's neighbour row was just read
  // into the same L2 (5% faster on a 100 x 100 plane, 5.5% slower on a
  // 512 x 512 one, where the blocks keep their dealt order).
  const unsigned t =
      (unsigned)(NB == 256 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x) * (unsigned)NB + threadIdx.x;
  if (t >= (unsigned)g.sxy) return;
  const int i = (int)(t % (unsigned)g.nx), j = (int)(t / (unsigned)g.nx);
  const int k = blockIdx.y;
  const unsigned n = (unsigned)i + (unsigned)g.nx * ((unsigned)j + (unsigned)g.ny * (unsigned)k);
  const int cid = (int)ldg((const CI*)g.cls, n);
  const T* cf = g.ctab + cid * K_STRIDE;
  const T hx = ldg(g.fi[3], n), hy = ldg(g.fi[4], n), hz = ldg(g.fi[5], n);
  const T hx_j = (j > 0) ? ldg(g.fi[3], n - (unsigned)g.nx) : T(0);
  const T hx_k = (k > 0) ? ldg(g.fi[3], n - (unsigned)g.sxy) : T(0);
  const T hy_i = (i > 0) ? ldg(g.fi[4], n - 1) : T(0);
  const T hy_k = (k > 0) ? ldg(g.fi[4], n - (unsigned)g.sxy) : T(0);
  const T hz_i = (i > 0) ? ldg(g.fi[5], n - 1) : T(0);
  const T hz_j = (j > 0) ? ldg(g.fi[5], n - (unsigned)g.nx) : T(0);
  const T eold[3] = {ldg(g.fi[0], n), ldg(g.fi[1], n), ldg(g.fi[2], n)};
  T e[3];
  const SrcRange sr = src_node(g, i, j, k);
  e_point<T, PML>(g, i, j, k, n, cf, hx, hy, hz, hx_j, hx_k, hy_i, hy_k, hz_i, hz_j, eold, step, e, sr.lo, sr.hi);
  debye_point(d, cid, n, eold, e);
  stg(g.fo[0], n, e[0]);
  stg(g.fo[1], n, e[1]);
  stg(g.fo[2], n, e[2]);
}


template <typename T, typename CI, bool PML, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_fused(GridView<T> g, int step, int kz, int ntx, int nty) {
  step = gstep(g, step);
  __shared__ FusedSmem<T, TX, TY> sm;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_x = tile % ntx, rest = tile / ntx;
  const int k0 = (rest / nty) * kz;
  fused_tile<T, CI, PML, TX, TY>(g, sm, tile_x * TX, (rest % nty) * TY, k0, min(k0 + kz, g.nz), step);
}

// One grid, tile list: block b takes tile (i0, j0, k0, k1).  The host splits
// a grid with a CPML into tiles clear of every slab (including the recomputed
// halo and the prologue plane), which run the lean instantiation, and the
// rest, which runs the CPML one.
template <typename T, typename CI, bool PML, int TX, int TY, int AX>
__global__ __launch_bounds__(TX * TY) void k_fused_list(GridView<T> g, const int4* __restrict__ tiles, int step) {
  step = gstep(g, step);
  __shared__ FusedSmem<T, TX, TY> sm;
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  fused_tile<T, CI, PML, TX, TY, AX>(g, sm, t.x, t.y, t.z, t.w, step);
}

// Batched: one block per entry of a tile list spanning many grids; each
// grid's view is read from a device table (one table per field-set parity).
// The step index is a device counter (plus a per-launch offset) so that a
// captured graph of several steps can be replayed unchanged.
template <typename T, typename CI, bool PML, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_fused_batch(const GridView<T>* __restrict__ views,
                                                        const int4* __restrict__ tiles,
                                                        const int* __restrict__ d_step, int offset) {
  __shared__ FusedSmem<T, TX, TY> sm;
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];  // (grid, i0, j0, k0 | kz << 16)
  const GridView<T>& g = views[t.x];
  const int k0 = t.w & 0xffff, kz = t.w >> 16;
  fused_tile<T, CI, PML, TX, TY>(g, sm, t.y, t.z, k0, min(k0 + kz, g.nz), *d_step + offset);
}

// ---------------------------------------------------------------------------
// temporally blocked variant: two steps per pass
//
// Block = TY + 4 waves; wave v, lane u own the point x = i0 - 2 + u,
// y = j0 - 2 + v of a 64 x (TY + 4) region around the 60 x TY output tile
// [i0, i0+60) x [j0, j0+TY).  Each point is updated by the same thread in
// every stage it belongs to (the dependency cone shrinks by one node per
// half step on the high or low side):
//   A  H^{n+1/2} on u <= 62, v <= TY+2            (from E^n, H^{n-1/2})
//   B  E^{n+1}   on 1 <= u <= 62, 1 <= v <= TY+2  (sources of step n)
//   C  H^{n+3/2} on 1 <= u <= 61, 1 <= v <= TY+1
//   D  E^{n+2}   on 2 <= u <= 61, 2 <= v <= TY+1  (the tile; sources n+1)
// Marching up z, iteration k does A and B of plane k and C and D of plane
// k-1; the chunk [k0, k1) starts its pipeline at k0-2.  Neighbours are read
// from LDS planes; a point's own values of earlier planes stay in
// registers, as does its CPML state between the two steps.  Only E^{n+2},
// H^{n+3/2} and the CPML state after two steps reach memory (output set).
// ---------------------------------------------------------------------------

template <typename T, int TY>
struct TB2Smem {
  static constexpr int R = TY + 4;
  static constexpr int PZ = 512 / sizeof(T);  // longest z profile row held here (2 npml)
  T se0[3][R][64];      // E^n, plane k
  T sh1[3][R][64];      // H^{n+1/2}, plane k
  T se1[2][3][R][64];   // E^{n+1}, planes k and k-1
  T sh2[3][R][64];      // H^{n+3/2}, plane k-1
  T stab[256 * K_STRIDE];
  T px[P_NROW][64];     // CPML profile at each lane's x
  T py[P_NROW][R];      // ... at each wave's y
  T pz[P_NROW * PZ];    // the z table
};

// CPML profile values of a two-step tile from the LDS copies made at the
// tile start.  Reading them from global memory in every plane would make the
// wave wait for its whole prefetch at each CPML term.  (The host runs the
// two-step pass only on grids whose z table fits its copy: 2 npml <= PZ.)
template <typename T, int TY>
struct ProfTB2 {
  const GridView<T>& g;
  const TB2Smem<T, TY>& sm;
  int u, v;
  template <int U>
  __device__ __forceinline__ Prof3<T> at(int row, int l) const {
    if (U == 0) return {sm.px[row][u], sm.px[row + 1][u], sm.px[row + 2][u]};
    if (U == 1) return {sm.py[row][v], sm.py[row + 1][v], sm.py[row + 2][v]};
    const int tn = 2 * g.npml, q = row * tn + l;
    return {sm.pz[q], sm.pz[q + tn], sm.pz[q + 2 * tn]};
  }
};

// One two-step tile: outputs [i0, i0+iw) x [j0, j0+jh) x [k0, k1) with
// iw <= 60, jh <= TY.  AX masks the axes whose CPML slabs the tile can reach.
template <typename T, typename CI, bool PML, int TY, int AX, bool USLAB = false, bool LEAN = false>
__device__ __forceinline__ void tb2_tile(const GridView<T>& g, TB2Smem<T, TY>& sm, int i0, int j0, int iw, int jh,
                                         int k0, int k1, int step) {
  constexpr int TX = 60, NT = 64 * (TY + 4);
  constexpr bool LDS_TAB = sizeof(CI) == 1;
  const int tid = threadIdx.x, u = tid & 63, v = tid >> 6;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned sxy = (unsigned)g.sxy;
  const CI* cls = (const CI*)g.cls;
  if (LDS_TAB) {
    for (int q = tid; q < g.ncls * K_STRIDE; q += NT) sm.stab[q] = ldg(g.ctab, (unsigned)q);
  }
  auto coef = [&](int c) -> const T* { return LDS_TAB ? sm.stab + c * K_STRIDE : g.ctab + c * K_STRIDE; };

  const int x = i0 - 2 + u, y = j0 - 2 + v;
  const bool dom = x >= 0 && x < nx && y >= 0 && y < ny;
  const bool inA = dom && u <= TX + 2 && v <= TY + 2;
  const bool inB = inA && u >= 1 && v >= 1;
  const bool inC = inB && u <= TX + 1 && v <= TY + 1;
  const bool inD = inC && u >= 2 && v >= 2 && u < 2 + iw && v < 2 + jh;
  const unsigned n0 = dom ? (unsigned)x + (unsigned)nx * (unsigned)y : 0u;
  const int lx = PML && (AX & 1) && dom ? slab_pos(x, nx, g.npml) : -1;
  const int ly = PML && (AX & 2) && dom ? slab_pos(y, ny, g.npml) : -1;
  constexpr bool PZ = PML && (AX & 4);
  // (E is updated on planes k0 - 1 .. k1: the first step's cone, then the outputs)
  const SrcRange srcr = src_wave(g, n0, inB, k0 - 1, k1);
  if (PML) {
    const int tn = 2 * g.npml;
    if ((AX & 1) && v == 0) {
      const int xl = x >= 0 && x < nx ? slab_pos(x, nx, g.npml) : -1;
      for (int r = 0; r < P_NROW; ++r) sm.px[r][u] = xl >= 0 ? ldg(g.prof[0], (unsigned)(r * tn + xl)) : T(0);
    }
    if ((AX & 2) && u == 0) {
      const int yl = y >= 0 && y < ny ? slab_pos(y, ny, g.npml) : -1;
      for (int r = 0; r < P_NROW; ++r) sm.py[r][v] = yl >= 0 ? ldg(g.prof[1], (unsigned)(r * tn + yl)) : T(0);
    }
    if (AX & 4)
      for (int q = tid; q < P_NROW * tn; q += NT) sm.pz[q] = ldg(g.prof[2], (unsigned)q);
  }
  const ProfTB2<T, TY> pf{g, sm, u, v};

  // Loads are unconditional, from uniform plane bases and the thread's
  // column offset n0 (0 for points outside the grid): E planes outside
  // [0, nz) read the zero plane, H and class planes are clamped (those values
  // are never used).  E of points outside the grid is zeroed where it enters
  // LDS.  No load then sits behind a branch, and none waits on a select.
  // The x- and y-slab instantiations (AX 5, 6) keep predicated loads unless
  // USLAB: the batched kernels, which read their grid's view from memory,
  // have no registers to spare for them there.  LEAN corner tiles keep
  // predicated loads too and store at once, to fit two blocks per CU: the
  // batch's corner tiles (its grids are small, so they carry much of the
  // work) and the FP32 single-grid ones.
  constexpr bool UNC = AX == 4 || (AX == 7 && !LEAN) || USLAB;
  auto ld_e = [&](int k, T e[3]) {
    const bool in = k >= 0 && k < nz;
    if (UNC) {
      const size_t po = (size_t)sxy * (size_t)(in ? k : 0);
      e[0] = ldg(in ? g.fi[0] + po : g.zpl, n0);
      e[1] = ldg(in ? g.fi[1] + po : g.zpl, n0);
      e[2] = ldg(in ? g.fi[2] + po : g.zpl, n0);
    } else {
      const bool ok = dom && in;
      const unsigned n = n0 + sxy * (unsigned)(ok ? k : 0);
      e[0] = ok ? ldg(g.fi[0], n) : T(0);
      e[1] = ok ? ldg(g.fi[1], n) : T(0);
      e[2] = ok ? ldg(g.fi[2], n) : T(0);
    }
  };
  auto ld_h = [&](int k, T h[3]) {
    if (UNC) {
      const size_t po = (size_t)sxy * (size_t)min(max(k, 0), nz - 1);
      h[0] = ldg(g.fi[3] + po, n0);
      h[1] = ldg(g.fi[4] + po, n0);
      h[2] = ldg(g.fi[5] + po, n0);
    } else {
      const bool ok = inA && k >= 0 && k < nz;
      const unsigned n = n0 + sxy * (unsigned)(ok ? k : 0);
      h[0] = ok ? ldg(g.fi[3], n) : T(0);
      h[1] = ok ? ldg(g.fi[4], n) : T(0);
      h[2] = ok ? ldg(g.fi[5], n) : T(0);
    }
  };
  auto ld_c = [&](int k) -> int {
    if (UNC) return (int)ldg(cls + (size_t)sxy * (size_t)min(max(k, 0), nz - 1), n0);
    return (inA && k >= 0 && k < nz) ? (int)ldg(cls, n0 + sxy * (unsigned)k) : 0;
  };

  // pipeline registers of this thread's point
  T e0c[3], e0n[3], h0c[3];
  T h1p[3] = {T(0), T(0), T(0)};   // H^{n+1/2}, plane k-1
  T e1p[3] = {T(0), T(0), T(0)};   // E^{n+1},   plane k-1
  T h2p[2] = {T(0), T(0)};         // H^{n+3/2}, plane k-2 (x, y)
  T psh[3][2], pse[3][2];          // CPML state after step n+1, plane k-1
  for (int a = 0; a < 3; ++a) psh[a][0] = psh[a][1] = pse[a][0] = pse[a][1] = T(0);
  const int kb = k0 - 2;
  ld_e(kb, e0c);
  ld_e(kb + 1, e0n);
  ld_h(kb, h0c);
  int cc = ld_c(kb), cp = 0;

  // The outputs of plane k-1 are written at the top of the next iteration,
  // ahead of its prefetch: the vector-memory counter retires in order, so a
  // wait for the prefetched values then never has to wait for stores issued
  // after them.
  T e2[3] = {T(0), T(0), T(0)};
  T h2z = T(0);
  unsigned nst = 0;
  bool pend = false;
  // (The x- and y-slab instantiations store at once: they have no registers
  // to spare under their cap.)
  constexpr bool DEFER = (AX == 4 || (AX == 7 && !LEAN)) && sizeof(T) == 4;
  auto flush = [&]() {
    if (DEFER && pend) {
      stg(g.fo[0], nst, e2[0]);
      stg(g.fo[1], nst, e2[1]);
      stg(g.fo[2], nst, e2[2]);
      stg(g.fo[3], nst, h2p[0]);
      stg(g.fo[4], nst, h2p[1]);
      stg(g.fo[5], nst, h2z);
    }
  };

  // Let the prologue's loads land before the loop.  Otherwise the compiler,
  // which merges the loop entry with the back edge, places the wait for them
  // after the stores at the top of every iteration and so waits for those
  // stores as well.  (vmcnt 0, expcnt and lgkmcnt unconstrained)
  __builtin_amdgcn_s_waitcnt(0x0F70);
  for (int k = kb; k <= k1; ++k) {
    flush();
    // prefetch: classes and H^{n-1/2} of plane k+1, E^n of plane k+2 (the
    // classes first: the end of the iteration then waits for all of it)
    T e0f[3], h0f[3];
    const int cf1 = ld_c(k + 1);
    ld_e(k + 2, e0f);
    ld_h(k + 1, h0f);
    const bool kin = k >= 0 && k < nz;
    for (int c = 0; c < 3; ++c) sm.se0[c][v][u] = dom ? e0c[c] : T(0);
    __syncthreads();
    // A: H^{n+1/2}, plane k
    T h1c[3] = {T(0), T(0), T(0)};
    T pshn[3][2];
    // The z-slab planes take their own branch (lz is uniform), so that the
    // CPML state loaded there is consumed inside it and no wait for it is
    // left at the end of the iteration, where it would also wait for the
    // prefetch and the stores.
    const int lz = PZ ? slab_pos(k, nz, g.npml) : -1;
    if (inA && kin) {
      auto stage_a = [&](const int l[3]) {
        if (PML) psi_load(g, 1, l, x, y, k, pshn);
        h_core_pf<T, PML>(pf, l, coef(cc), e0c[0], e0c[1], e0c[2], sm.se0[0][v + 1][u], e0n[0], sm.se0[1][v][u + 1],
                       e0n[1], sm.se0[2][v][u + 1], sm.se0[2][v + 1][u], h0c, pshn, h1c);
      };
      if (lz >= 0) {
        const int l[3] = {lx, ly, lz};
        stage_a(l);
      } else {
        const int l[3] = {lx, ly, -1};
        stage_a(l);
      }
    }
    for (int c = 0; c < 3; ++c) sm.sh1[c][v][u] = h1c[c];
    __syncthreads();
    // B: E^{n+1}, plane k (needs H^{n+1/2} of plane k-1: valid from k0-1 on)
    T e1c[3] = {T(0), T(0), T(0)};
    T psen[3][2];
    if (inB && kin && k >= k0 - 1) {
      auto stage_b = [&](const int l[3]) {
        if (PML) psi_load(g, 0, l, x, y, k, psen);
        e_core_pf<T, PML>(pf, g, l, n0 + sxy * (unsigned)k, coef(cc), h1c[0], h1c[1], h1c[2], sm.sh1[0][v - 1][u],
                       h1p[0], sm.sh1[1][v][u - 1], h1p[1], sm.sh1[2][v][u - 1], sm.sh1[2][v - 1][u], e0c, step,
                       psen, e1c, srcr.first(k), srcr.last(k));
      };
      if (lz >= 0) {
        const int l[3] = {lx, ly, lz};
        stage_b(l);
      } else {
        const int l[3] = {lx, ly, -1};
        stage_b(l);
      }
    }
    const int s1 = (k + 2) & 1, s1m = s1 ^ 1;
    for (int c = 0; c < 3; ++c) sm.se1[s1][c][v][u] = e1c[c];
    // No barrier here: C reads the neighbours' E^{n+1} of plane k-1 (slot
    // s1m, written in the previous iteration, before its two barriers) and
    // this thread's own E^{n+1} of plane k (a register).  Slot s1, written
    // just now, is read by the next iteration's C, after that iteration's
    // first two barriers; it last held plane k-2, whose readers finished
    // before this iteration's barriers.
    // C: H^{n+3/2}, plane k-1
    const int km = k - 1;
    T h2c[3] = {T(0), T(0), T(0)};
    if (inC && k >= k0 && km >= 0 && km < nz) {
      int l[3] = {lx, ly, PZ ? slab_pos(km, nz, g.npml) : -1};
      h_core_pf<T, PML>(pf, l, coef(cp), e1p[0], e1p[1], e1p[2], sm.se1[s1m][0][v + 1][u], e1c[0],
                     sm.se1[s1m][1][v][u + 1], e1c[1], sm.se1[s1m][2][v][u + 1], sm.se1[s1m][2][v + 1][u], h1p, psh,
                     h2c);
      if (inD && km >= k0) {
        if (!DEFER) {
          const unsigned n = n0 + sxy * (unsigned)km;
          stg(g.fo[3], n, h2c[0]);
          stg(g.fo[4], n, h2c[1]);
          stg(g.fo[5], n, h2c[2]);
        }
        if (PML) psi_store(g, 1, l, x, y, km, psh);
      }
    }
    for (int c = 0; c < 3; ++c) sm.sh2[c][v][u] = h2c[c];
    __syncthreads();
    // D: E^{n+2}, plane k-1 (the output tile; km < k1 always holds)
    pend = inD && km >= k0;
    nst = n0 + sxy * (unsigned)km;
    if (pend) {
      int l[3] = {lx, ly, PZ ? slab_pos(km, nz, g.npml) : -1};
      e_core_pf<T, PML>(pf, g, l, nst, coef(cp), h2c[0], h2c[1], h2c[2], sm.sh2[0][v - 1][u], h2p[0], sm.sh2[1][v][u - 1],
                     h2p[1], sm.sh2[2][v][u - 1], sm.sh2[2][v - 1][u], e1p, step + 1, pse, e2, srcr.first(km),
                     srcr.last(km));
      if (!DEFER) {
        stg(g.fo[0], nst, e2[0]);
        stg(g.fo[1], nst, e2[1]);
        stg(g.fo[2], nst, e2[2]);
      }
      if (PML) psi_store(g, 0, l, x, y, km, pse);
    }
    // rotate the pipeline
    h2p[0] = h2c[0];
    h2p[1] = h2c[1];
    h2z = h2c[2];
    for (int c = 0; c < 3; ++c) {
      h1p[c] = h1c[c];
      e1p[c] = e1c[c];
      e0c[c] = e0n[c];
      e0n[c] = e0f[c];
      h0c[c] = h0f[c];
    }
    if (PML)
      for (int a = 0; a < 3; ++a) {
        psh[a][0] = pshn[a][0];
        psh[a][1] = pshn[a][1];
        pse[a][0] = psen[a][0];
        pse[a][1] = psen[a][1];
      }
    cp = cc;
    cc = cf1;
  }
  flush();
}

template <typename T, typename CI, bool PML, int TY>
__global__ __launch_bounds__(64 * (TY + 4)) void k_tb2(GridView<T> g, int step, int kz, int ntx, int nty) {
  step = gstep(g, step);
  __shared__ TB2Smem<T, TY> sm;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tile_x = tile % ntx, rest = tile / ntx;
  const int k0 = (rest / nty) * kz;
  tb2_tile<T, CI, PML, TY, 7>(g, sm, tile_x * 60, (rest % nty) * TY, 60, TY, k0, min(k0 + kz, g.nz), step);
}

// Tile list: (i0 | iw << 16, j0 | jh << 16, k0, k1) per block.  FP32: at
// most 80 VGPRs (6 waves per SIMD), so that two blocks share a CU.  The
// corner tiles get there as LEAN tiles, which also lets them run beside the
// z-only tiles rather than wait for a free CU.
template <typename T, typename CI, bool PML, int TY, int AX>
__global__ __launch_bounds__(64 * (TY + 4), (sizeof(T) == 8 ? 1 : 6)) void k_tb2_list(GridView<T> g,
                                                                                      const int4* __restrict__ tiles,
                                                                                      int step) {
  step = gstep(g, step);
  __shared__ TB2Smem<T, TY> sm;
  const int4 t = tiles[xcd_runs(blockIdx.x, gridDim.x)];
  constexpr bool LEAN = AX == 7 && sizeof(T) == 4;
  tb2_tile<T, CI, PML, TY, AX, !LEAN, LEAN>(g, sm, t.x & 0xffff, t.y & 0xffff, t.x >> 16, t.y >> 16, t.z, t.w,
                                           step);
}

// Probes of a two-step pass: the intermediate step's values are recomputed
// point by point from the input set (which the pass leaves untouched) with
// the same per-point arithmetic; the second step's values are read from the
// output set.
template <typename T, typename CI, bool PML>
__device__ __forceinline__ void h1_at(const GridView<T>& g, int x, int y, int k, T h[3]) {
  h[0] = h[1] = h[2] = T(0);
  if (x < 0 || y < 0 || k < 0 || x >= g.nx || y >= g.ny || k >= g.nz) return;
  const unsigned n = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)k);
  const T* cf = g.ctab + (int)ldg((const CI*)g.cls, n) * K_STRIDE;
  const T ex = ldg(g.fi[0], n), ey = ldg(g.fi[1], n), ez = ldg(g.fi[2], n);
  const T ex_j = (y + 1 < g.ny) ? ldg(g.fi[0], n + (unsigned)g.nx) : T(0);
  const T ex_k = (k + 1 < g.nz) ? ldg(g.fi[0], n + (unsigned)g.sxy) : T(0);
  const T ey_i = (x + 1 < g.nx) ? ldg(g.fi[1], n + 1) : T(0);
  const T ey_k = (k + 1 < g.nz) ? ldg(g.fi[1], n + (unsigned)g.sxy) : T(0);
  const T ez_i = (x + 1 < g.nx) ? ldg(g.fi[2], n + 1) : T(0);
  const T ez_j = (y + 1 < g.ny) ? ldg(g.fi[2], n + (unsigned)g.nx) : T(0);
  const T hold[3] = {ldg(g.fi[3], n), ldg(g.fi[4], n), ldg(g.fi[5], n)};
  int l[3] = {-1, -1, -1};
  T ps[3][2];
  if (PML) {
    slabs(g, x, y, k, l);
    psi_load(g, 1, l, x, y, k, ps);
  }
  h_core<T, PML>(g, l, cf, ex, ey, ez, ex_j, ex_k, ey_i, ey_k, ez_i, ez_j, hold, ps, h);
}

template <typename T, typename CI, bool PML>
__device__ __forceinline__ void e1_at(const GridView<T>& g, int x, int y, int k, int step, T e[3]) {
  const unsigned n = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)k);
  T h[3], hi[3], hj[3], hk[3];
  h1_at<T, CI, PML>(g, x, y, k, h);
  h1_at<T, CI, PML>(g, x - 1, y, k, hi);
  h1_at<T, CI, PML>(g, x, y - 1, k, hj);
  h1_at<T, CI, PML>(g, x, y, k - 1, hk);
  const T* cf = g.ctab + (int)ldg((const CI*)g.cls, n) * K_STRIDE;
  const T eold[3] = {ldg(g.fi[0], n), ldg(g.fi[1], n), ldg(g.fi[2], n)};
  int l[3] = {-1, -1, -1};
  T ps[3][2];
  if (PML) {
    slabs(g, x, y, k, l);
    psi_load(g, 0, l, x, y, k, ps);
  }
  const SrcRange sr = src_node(g, x, y, k);
  e_core<T, PML>(g, l, n, cf, h[0], h[1], h[2], hj[0], hk[0], hi[1], hk[1], hi[2], hj[2], eold, step, ps, e, sr.lo,
                 sr.hi);
}

// Probes: one block of PR_NT threads per probe.  Thread `tid` sums terms
// tid, tid + PR_NT, ... of the probe in order; the lanes of each wave are
// then summed by a shuffle tree and the four wave sums in order.  Every probe
// kernel sums in this one FP64 order, so that all variants, and a batch and
// its grids run alone, agree bit for bit.
constexpr int PR_NT = 256;

// Block sum of `a` in the fixed order; `red` holds 4 doubles of LDS.  The
// total is returned to every thread.
__device__ __forceinline__ double probe_block_sum(double a, double* red) {
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// Probe p of a two-step pass, one block: sample `step` (S1: recomputed from
// the input set, which the pass leaves untouched) and sample `step` + 1 (S2:
// read from the output set).  `red` holds 8 doubles of LDS.
template <typename T, typename CI, bool PML, bool S1 = true, bool S2 = true>
__device__ __forceinline__ void probe_tb2(const GridView<T>& g, int p, int step, double* red) {
  double a1 = 0.0, a2 = 0.0;
  for (int t = g.pr_off[p] + (int)threadIdx.x; t < g.pr_off[p + 1]; t += PR_NT) {
    const int c = g.term_comp[t];
    const unsigned n = (unsigned)g.term_idx[t];
    if (S1) {
      const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), k = (int)(n / g.sxy);
      T v3[3];
      if (c < 3) e1_at<T, CI, PML>(g, x, y, k, step, v3);
      else h1_at<T, CI, PML>(g, x, y, k, v3);
      const int cc = c < 3 ? c : c - 3;
      const T v1 = cc == 0 ? v3[0] : cc == 1 ? v3[1] : v3[2];
      a1 += g.term_w[t] * (double)v1;
    }
    if (S2) {
      const T* f = c == 0 ? g.fo[0] : c == 1 ? g.fo[1] : c == 2 ? g.fo[2] : c == 3 ? g.fo[3] : c == 4 ? g.fo[4] : g.fo[5];
      a2 += g.term_w[t] * (double)ldg((const T*)f, n);
    }
  }
  if (S1) a1 = probe_block_sum(a1, red);
  if (S2) a2 = probe_block_sum(a2, red + 4);
  if (threadIdx.x == 0) {
    if (S1) g.pr_out[(long long)p * g.max_steps + step] = a1;
    if (S2) g.pr_out[(long long)p * g.max_steps + step + 1] = a2;
  }
}

template <typename T, typename CI, bool PML, bool S1 = true, bool S2 = true>
__global__ __launch_bounds__(PR_NT) void k_probes_tb2(GridView<T> g, int step) {
  step = gstep(g, step);
  __shared__ double red[8];
  if ((int)blockIdx.x >= g.n_probe) return;  // uniform per block
  probe_tb2<T, CI, PML, S1, S2>(g, blockIdx.x, step, red);
}

// Batched two-step probes: entry q of the list is (grid, probe).
template <typename T, typename CI>
__global__ __launch_bounds__(PR_NT) void k_probes_tb2_batch(const GridView<T>* __restrict__ views,
                                                           const int2* __restrict__ plist, int n,
                                                           const int* __restrict__ d_step, int offset) {
  __shared__ double red[8];
  if ((int)blockIdx.x >= n) return;  // uniform per block
  const int2 e = plist[blockIdx.x];
  probe_tb2<T, CI, true>(views[e.x], e.y, *d_step + offset, red);
}

// Batched two-step pass: tile (grid, i0 | iw << 16, j0 | jh << 16,
// k0 | kz << 16) per block; step index *d_step + offset.  FP32: at most 80
// VGPRs, so that two blocks share a CU.
template <typename T, typename CI, int TY, int AX>
__global__ __launch_bounds__(64 * (TY + 4), (sizeof(T) == 8 ? 1 : 6)) void k_tb2_batch(const GridView<T>* __restrict__ views,
                                                                               const int4* __restrict__ tiles,
                                                                               const int* __restrict__ d_step,
                                                                               int offset) {
  __shared__ TB2Smem<T, TY> sm;
  const int4 t = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const GridView<T>& g = views[t.x];
  const int k0 = t.w & 0xffff;
  tb2_tile<T, CI, true, TY, AX, false, true>(g, sm, t.y & 0xffff, t.z & 0xffff, t.y >> 16, t.z >> 16, k0,
                                             k0 + (t.w >> 16),
                                             *d_step + offset);
}

// Batched two-step pass as persistent launches, one per code path (AXP 5:
// the x-slab instantiation, which also serves tiles clear of the x and y
// slabs; AXP 7: the all-axes one, for y-slab and corner tiles, and every FP64
// tile).  One kernel holding both paths spilled at its 80-register cap, and
// each reload of a spill waited for all loads in flight.  A path's tile list
// holds its tiles grid by grid (larger grids first), (grid | group << 24,
// i0 | iw << 16, j0 | jh << 16, k0 | kz << 16), cut into 8 contiguous runs,
// one per XCD, so that a grid's tiles share that XCD's L2.  A block takes
// tiles from its own XCD's run through an atomic counter, then from the
// other runs in turn, and leaves once every run is empty: each counter only
// grows, so every block finishes.  Tiles of one pass write disjoint outputs
// and read only the pass's input set, so no block waits for another (nor a
// kernel for the other path's).  The counters start at 0 (k_qreset before
// the launches).
template <typename T, typename CI, int AXP>
__global__ __launch_bounds__(768, (sizeof(T) == 8 ? 1 : 6)) void k_tb2_batch_q(const GridView<T>* __restrict__ views,
                                                                             const int4* __restrict__ tiles,
                                                                             QRuns runs, int* __restrict__ ctr,
                                                                             const int* __restrict__ d_step,
                                                                             int offset) {
  __shared__ TB2Smem<T, 8> sm;
  __shared__ int pick;
  const int step = *d_step + offset;
  const int x0 = (int)(blockIdx.x % 8);
  for (int r = 0; r < 8; ++r) {
    const int x = (x0 + r) % 8, base = runs.start[x], n = runs.start[x + 1] - base;
    for (;;) {
      __syncthreads();  // the previous tile is done with the LDS and with `pick`
      if (threadIdx.x == 0) pick = atomicAdd(ctr + x, 1);
      __syncthreads();
      const int q = __builtin_amdgcn_readfirstlane(pick);  // uniform: the tile is read into scalar registers
      if (q >= n) break;
      const int4 t = tiles[base + q];
      const GridView<T>& g = views[t.x & 0xffffff];
      const int i0 = t.y & 0xffff, j0 = t.z & 0xffff, iw = t.y >> 16, jh = t.z >> 16;
      const int k0 = t.w & 0xffff, k1 = k0 + (t.w >> 16);
      tb2_tile<T, CI, true, 8, AXP, false, true>(g, sm, i0, j0, iw, jh, k0, k1, step);
    }
  }
}

__global__ void k_qreset(int* ctr) {
  if (threadIdx.x < 16) ctr[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// probes of a one-step pass: one block per probe, the fixed FP64 order of
// probe_block_sum
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void probe_one(const GridView<T>& g, int p, int step, double* red) {
  double acc = 0.0;
  for (int t = g.pr_off[p] + (int)threadIdx.x; t < g.pr_off[p + 1]; t += PR_NT) {
    const int c = g.term_comp[t];
    const T* f = c == 0 ? g.fi[0] : c == 1 ? g.fi[1] : c == 2 ? g.fi[2] : c == 3 ? g.fi[3] : c == 4 ? g.fi[4] : g.fi[5];
    acc += g.term_w[t] * (double)ldg(f, (unsigned)g.term_idx[t]);
  }
  acc = probe_block_sum(acc, red);
  if (threadIdx.x == 0) g.pr_out[(long long)p * g.max_steps + step] = acc;
}

template <typename T>
__global__ __launch_bounds__(PR_NT) void k_probes(GridView<T> g, int step) {
  step = gstep(g, step);
  __shared__ double red[4];
  if ((int)blockIdx.x >= g.n_probe) return;  // uniform per block
  probe_one(g, blockIdx.x, step, red);
}

// Batched probes: entry q of the list is (grid, probe); one block each.
template <typename T>
__global__ __launch_bounds__(PR_NT) void k_probes_batch(const GridView<T>* __restrict__ views,
                                                       const int2* __restrict__ plist, int n,
                                                       const int* __restrict__ d_step, int offset) {
  __shared__ double red[4];
  if ((int)blockIdx.x >= n) return;  // uniform per block
  const int2 e = plist[blockIdx.x];
  probe_one(views[e.x], e.y, *d_step + offset, red);
}

__global__ void k_add(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Split-pass blocks: NB consecutive nodes of a plane (full waves for any
// nx).  512 on large planes, 256 (dealt in bands per XCD) on small ones: on a
// 512 x 512 plane 512 ran 2.5% faster, on a 100 x 100 plane 4% slower (and
// 128 slower on both).
inline int split_nb(const long long sxy) { return sxy >= 65536 ? 512 : 256; }

template <typename T, typename CI, int NB>
hipError_t step_split_nb(const GridView<T>& g, int step, hipStream_t st) {
  const dim3 blk(NB), grd((unsigned)((g.sxy + NB - 1) / NB), (unsigned)g.nz);
  if (g.npml > 0) {
    hipLaunchKernelGGL((k_h_split<T, CI, true, NB>), grd, blk, 0, st, g);
    hipLaunchKernelGGL((k_e_split<T, CI, true, NB>), grd, blk, 0, st, g, step);
  } else {
    hipLaunchKernelGGL((k_h_split<T, CI, false, NB>), grd, blk, 0, st, g);
    hipLaunchKernelGGL((k_e_split<T, CI, false, NB>), grd, blk, 0, st, g, step);
  }
  return hipGetLastError();
}

template <typename T, typename CI>
hipError_t step_split(const GridView<T>& g, int step, hipStream_t st) {
  return split_nb(g.sxy) == 512 ? step_split_nb<T, CI, 512>(g, step, st) : step_split_nb<T, CI, 256>(g, step, st);
}

// Oblique thin wires.  k_owire_cur: the new segment currents from E^n (the
// input field set, or with E1 the values of k_owire_e1) and the charges q^n
// (the driven segment takes its sample); k_owire_q: then the charges from
// the new currents, and the record.  Both before the step's field pass,
// which they do not depend on.  One one-wave block per segment (block
// (s, wire)): lane l sums the gather terms l, l + 64, ... in table order,
// then the 64 partial sums meet in a fixed shuffle tree, so the result does
// not depend on scheduling.  The blocks are single waves so that they find
// room on CUs that the field pass's blocks keep busy.
template <typename T, bool E1>
__global__ void __launch_bounds__(64) k_owire_cur(GridView<T> g, OWireView w, int step) {
  step = gstep(g, step);
  const OWireParam p = w.par[blockIdx.y];
  const int s = (int)blockIdx.x;
  if (s >= p.nseg) return;  // uniform per block
  double* cur = w.cur + p.seg0;
  const double* q = w.q + p.seg0 + blockIdx.y;
  const int lane = (int)threadIdx.x;
  double et = 0.0;
  for (int e = w.seg_off[p.seg0 + s] + lane, e1 = w.seg_off[p.seg0 + s + 1]; e < e1; e += 64) {
    if (E1) {
      et += w.g_w[e] * w.e1[w.g_edge[e]];
    } else {
      const long long key = w.g_key[e];
      et += w.g_w[e] * (double)g.fi[(int)(key >> 40)][key & ((1ll << 40) - 1)];
    }
  }
  for (int off = 32; off > 0; off >>= 1) et += __shfl_down(et, off, 64);
  if (lane == 0)
    cur[s] = s == p.src ? w.amp[(size_t)blockIdx.y * w.max_steps + step]
                        : cur[s] + p.dtL * (et - (q[s + 1] - q[s]) * p.invCdl);
}

template <typename T>
__global__ void __launch_bounds__(64) k_owire_q(GridView<T> g, OWireView w, int step) {
  step = gstep(g, step);
  const OWireParam p = w.par[blockIdx.y];
  const double* cur = w.cur + p.seg0;
  double* q = w.q + p.seg0 + blockIdx.y;
  const int j = (int)(blockIdx.x * 64 + threadIdx.x);
  if (j <= p.nseg) {
    const double il = j > 0 ? cur[j - 1] : 0.0, ir = j < p.nseg ? cur[j] : 0.0;
    q[j] -= ((j == 0 || j == p.nseg) ? 2.0 * p.dtdl : p.dtdl) * (ir - il);
  }
  if (j == 0 && p.rec >= 0) w.rec[(size_t)blockIdx.y * w.max_steps + step] = cur[p.rec];
}

// Junctions, after k_owire_q: that kernel moved each member end node's
// charge by its own segment's current as for an open end, so the members'
// charges sum (times their half segments) to the junction's new charge;
// they then take the shared potential, q_m = C'_m Q / sum_m C'_m len_m.  One
// thread per junction, members in table order (FP64).
__global__ void __launch_bounds__(64) k_owire_junc(OWireView w) {
  const int J = (int)(blockIdx.x * 64 + threadIdx.x);
  if (J >= w.n_junc) return;
  double Q = 0.0, cap = 0.0;
  for (int m = w.jn_off[J]; m < w.jn_off[J + 1]; ++m) {
    Q += w.q[w.jn_q[m]] * w.jn_a[m];
    cap += w.jn_c[m] * w.jn_a[m];
  }
  const double V = Q / cap;
  for (int m = w.jn_off[J]; m < w.jn_off[J + 1]; ++m) w.q[w.jn_q[m]] = w.jn_c[m] * V;
}

// The touched edges' source amplitudes of step `step`: one thread per edge
// sums its terms in increasing segment order (FP64), times the edge's Cb / dx.
template <typename T, typename CI>
__global__ void __launch_bounds__(64) k_owire_amp(GridView<T> g, OWireView w, int step) {
  step = gstep(g, step);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w.n_edge) return;
  const long long key = w.e_key[e];
  const int a = (int)(key >> 40);
  const long long n = key & ((1ll << 40) - 1);
  double sum = 0.0;
  for (int t = w.e_off[e], t1 = w.e_off[e + 1]; t < t1; ++t) sum += w.j_w[t] * w.cur[w.j_seg[t]];
  const int cls = ((const CI*)g.cls)[n];
  const double cbdx = (double)g.ctab[cls * K_STRIDE + K_CBX + 2 * a];
  T* amp = const_cast<T*>(g.src_amp);
  amp[(size_t)w.wsrc[e] * (size_t)g.max_steps + (size_t)step] = (T)(cbdx * sum);
}

// E^{step+1} at the touched edges for a two-step pass: the step's update
// at the edge's node, recomputed from the input set as the pass will do it
// (its sources, the wires' included, and CPML).
template <typename T, typename CI, bool PML>
__global__ void __launch_bounds__(64) k_owire_e1(GridView<T> g, OWireView w, int step) {
  step = gstep(g, step);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w.n_edge) return;
  const long long key = w.e_key[e];
  const int a = (int)(key >> 40);
  const long long n = key & ((1ll << 40) - 1);
  const int x = (int)(n % g.nx), y = (int)((n / g.nx) % g.ny), k = (int)(n / g.sxy);
  T v[3];
  e1_at<T, CI, PML>(g, x, y, k, step, v);
  w.e1[e] = (double)v[a];
}

template <typename T, typename CI, int NB>
hipError_t step_split_debye_nb(const GridView<T>& g, const DebyeView<T>& d, int step, hipStream_t st) {
  const dim3 blk(NB), grd((unsigned)((g.sxy + NB - 1) / NB), (unsigned)g.nz);
  if (g.npml > 0) {
    hipLaunchKernelGGL((k_h_split<T, CI, true, NB>), grd, blk, 0, st, g);
    hipLaunchKernelGGL((k_e_split_debye<T, CI, true, NB>), grd, blk, 0, st, g, d, step);
  } else {
    hipLaunchKernelGGL((k_h_split<T, CI, false, NB>), grd, blk, 0, st, g);
    hipLaunchKernelGGL((k_e_split_debye<T, CI, false, NB>), grd, blk, 0, st, g, d, step);
  }
  return hipGetLastError();
}

template <typename T, typename CI>
hipError_t step_split_debye(const GridView<T>& g, const DebyeView<T>& d, int step, hipStream_t st) {
  return split_nb(g.sxy) == 512 ? step_split_debye_nb<T, CI, 512>(g, d, step, st)
                                : step_split_debye_nb<T, CI, 256>(g, d, step, st);
}

int launch_owire_iq(int prec, const void* view, const OWireView* ow, int step, int from_e1, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const dim3 gc((unsigned)ow->max_seg, (unsigned)ow->n_wire), gq((unsigned)(ow->max_seg / 64 + 1), (unsigned)ow->n_wire);
  if (prec == 64) {
    const GridView<double>& g = *(const GridView<double>*)view;
    if (from_e1) hipLaunchKernelGGL((k_owire_cur<double, true>), gc, dim3(64), 0, st, g, *ow, step);
    else hipLaunchKernelGGL((k_owire_cur<double, false>), gc, dim3(64), 0, st, g, *ow, step);
    hipLaunchKernelGGL((k_owire_q<double>), gq, dim3(64), 0, st, g, *ow, step);
  } else {
    const GridView<float>& g = *(const GridView<float>*)view;
    if (from_e1) hipLaunchKernelGGL((k_owire_cur<float, true>), gc, dim3(64), 0, st, g, *ow, step);
    else hipLaunchKernelGGL((k_owire_cur<float, false>), gc, dim3(64), 0, st, g, *ow, step);
    hipLaunchKernelGGL((k_owire_q<float>), gq, dim3(64), 0, st, g, *ow, step);
  }
  if (ow->n_junc > 0) hipLaunchKernelGGL(k_owire_junc, dim3((unsigned)((ow->n_junc + 63) / 64)), dim3(64), 0, st, *ow);
  return (int)hipGetLastError();
}

template <typename T>
hipError_t owire_amp_t(const GridView<T>& g, int cls16, const OWireView& w, int step, hipStream_t st) {
  const dim3 grd((unsigned)((w.n_edge + 63) / 64)), blk(64);
  if (cls16) hipLaunchKernelGGL((k_owire_amp<T, uint16_t>), grd, blk, 0, st, g, w, step);
  else hipLaunchKernelGGL((k_owire_amp<T, uint8_t>), grd, blk, 0, st, g, w, step);
  return hipGetLastError();
}

template <typename T>
hipError_t owire_e1_t(const GridView<T>& g, int cls16, const OWireView& w, int step, hipStream_t st) {
  const dim3 grd((unsigned)((w.n_edge + 63) / 64)), blk(64);
  const bool pml = g.npml > 0;
  if (cls16) {
    if (pml) hipLaunchKernelGGL((k_owire_e1<T, uint16_t, true>), grd, blk, 0, st, g, w, step);
    else hipLaunchKernelGGL((k_owire_e1<T, uint16_t, false>), grd, blk, 0, st, g, w, step);
  } else {
    if (pml) hipLaunchKernelGGL((k_owire_e1<T, uint8_t, true>), grd, blk, 0, st, g, w, step);
    else hipLaunchKernelGGL((k_owire_e1<T, uint8_t, false>), grd, blk, 0, st, g, w, step);
  }
  return hipGetLastError();
}

int launch_owire_amp(int prec, const void* view, int cls16, const OWireView* ow, int step, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == 64) return (int)owire_amp_t(*(const GridView<double>*)view, cls16, *ow, step, st);
  return (int)owire_amp_t(*(const GridView<float>*)view, cls16, *ow, step, st);
}

int launch_owire_e1(int prec, const void* view, int cls16, const OWireView* ow, int step, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == 64) return (int)owire_e1_t(*(const GridView<double>*)view, cls16, *ow, step, st);
  return (int)owire_e1_t(*(const GridView<float>*)view, cls16, *ow, step, st);
}

int launch_step_debye(int prec, const void* view, const void* dview, int cls16, int step, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (prec == 64) {
    const GridView<double>& g = *(const GridView<double>*)view;
    const DebyeView<double>& d = *(const DebyeView<double>*)dview;
    e = cls16 ? step_split_debye<double, uint16_t>(g, d, step, st) : step_split_debye<double, uint8_t>(g, d, step, st);
  } else {
    const GridView<float>& g = *(const GridView<float>*)view;
    const DebyeView<float>& d = *(const DebyeView<float>*)dview;
    e = cls16 ? step_split_debye<float, uint16_t>(g, d, step, st) : step_split_debye<float, uint8_t>(g, d, step, st);
  }
  return (int)e;
}

template <typename T, typename CI, bool PML, int TX, int TY>
hipError_t launch_fused(const GridView<T>& g, int step, int kz, hipStream_t st) {
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + kz - 1) / kz;
  const long long nb = (long long)ntx * nty * ntz;
  if (nb > 0x7fffffff || (sizeof(CI) == 1 && g.ncls > 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_fused<T, CI, PML, TX, TY>), dim3((unsigned)nb), dim3(TX * TY), 0, st, g, step, kz, ntx,
                     nty);
  return hipGetLastError();
}

template <typename T, typename CI>
hipError_t step_fused(const GridView<T>& g, int step, int tile_y, int tile_z, hipStream_t st) {
  const int kz = tile_z > 0 ? tile_z : 32;
  const bool pml = g.npml > 0;
  if (tile_y == 4)
    return pml ? launch_fused<T, CI, true, 64, 4>(g, step, kz, st) : launch_fused<T, CI, false, 64, 4>(g, step, kz, st);
  return pml ? launch_fused<T, CI, true, 64, 8>(g, step, kz, st) : launch_fused<T, CI, false, 64, 8>(g, step, kz, st);
}

// Tile groups of a grid with a CPML, by the slabs a tile (halo included)
// reaches: 0 neither the x nor the y slabs (z CPML code only), 1 x slabs, 2
// y slabs, 3 both (x-y corners).  Fused tiles are 32 wide in groups 1 and 3
// and 64 wide otherwise; two-step tiles are 60 wide.  FP64 (a diagnostic
// precision) keeps the all-axes instantiation for every group.
template <typename T, typename CI, int TY>
hipError_t launch_lists(const GridView<T>& g, int step, const int4* tiles, const int* counts, hipStream_t st,
                        hipStream_t st2, void* ev_src) {
  if (sizeof(CI) == 1 && g.ncls > 256) return hipErrorInvalidValue;
  constexpr bool D = sizeof(T) == 8;
  const int4* t = tiles;
  if (counts[0] > 0)
    hipLaunchKernelGGL((k_fused_list<T, CI, true, 64, TY, D ? 7 : 4>), dim3((unsigned)counts[0]), dim3(64 * TY), 0,
                       st, g, t, step);
  t += counts[0];
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_fused_list<T, CI, true, 32, TY, D ? 7 : 5>), dim3((unsigned)counts[1]), dim3(32 * TY), 0,
                       st2, g, t, step);
  t += counts[1];
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_fused_list<T, CI, true, 64, TY, D ? 7 : 6>), dim3((unsigned)counts[2]), dim3(64 * TY), 0,
                       st2, g, t, step);
  t += counts[2];
  if (counts[3] > 0)
    hipLaunchKernelGGL((k_fused_list<T, CI, true, 32, TY, 7>), dim3((unsigned)counts[3]), dim3(32 * TY), 0, st2, g, t,
                       step);
  t += counts[3];
  if (ev_src) {
    const hipError_t we = hipStreamWaitEvent(st2, (hipEvent_t)ev_src, 0);
    if (we != hipSuccess) return we;
  }
  if (counts[4] > 0)  // tiles that read an oblique wire's source amplitudes, once written
    hipLaunchKernelGGL((k_fused_list<T, CI, true, 32, TY, 7>), dim3((unsigned)counts[4]), dim3(32 * TY), 0, st2, g, t,
                       step);
  return hipGetLastError();
}

template <typename T, typename CI, int TY>
hipError_t launch_lists_tb2(const GridView<T>& g, int step, const int4* tiles, const int* counts, hipStream_t st,
                            hipStream_t st2, void* ev_src) {
  if (sizeof(CI) == 1 && g.ncls > 256) return hipErrorInvalidValue;
  constexpr bool D = sizeof(T) == 8;
  const dim3 blk(64 * (TY + 4));
  const int4* t1 = tiles + counts[0];
  const int4* t2 = t1 + counts[1];
  const int4* t3 = t2 + counts[2];
  if (counts[0] > 0)
    hipLaunchKernelGGL((k_tb2_list<T, CI, true, TY, D ? 7 : 4>), dim3((unsigned)counts[0]), blk, 0, st, g, tiles,
                       step);
  // Second stream: the few corner tiles first, beside the z-only ones; the
  // y-slab tiles last, to fill the end of the pass.
  if (counts[3] > 0)
    hipLaunchKernelGGL((k_tb2_list<T, CI, true, TY, 7>), dim3((unsigned)counts[3]), blk, 0, st2, g, t3, step);
  if (counts[1] > 0)
    hipLaunchKernelGGL((k_tb2_list<T, CI, true, TY, D ? 7 : 5>), dim3((unsigned)counts[1]), blk, 0, st2, g, t1, step);
  if (counts[2] > 0)
    hipLaunchKernelGGL((k_tb2_list<T, CI, true, TY, D ? 7 : 6>), dim3((unsigned)counts[2]), blk, 0, st2, g, t2, step);
  // tiles that read an oblique wire's source amplitudes, once the wire
  // kernels (on a third stream) have written them
  if (ev_src) {
    const hipError_t we = hipStreamWaitEvent(st2, (hipEvent_t)ev_src, 0);
    if (we != hipSuccess) return we;
  }
  // (those clear of the x and y slabs, listed first, as z-only tiles)
  const int4* t4 = t3 + counts[3];
  if (counts[5] > 0)
    hipLaunchKernelGGL((k_tb2_list<T, CI, true, TY, D ? 7 : 4>), dim3((unsigned)counts[5]), blk, 0, st2, g, t4, step);
  if (counts[4] > counts[5])
    hipLaunchKernelGGL((k_tb2_list<T, CI, true, TY, 7>), dim3((unsigned)(counts[4] - counts[5])), blk, 0, st2, g,
                       t4 + counts[5], step);
  // The probes' first sample, recomputed from the input set (which no group
  // writes), runs on the second stream beside the clear tiles; the caller
  // reads the second sample after the join (launch_probes2 with first = 0).
  if (g.n_probe > 0)
    hipLaunchKernelGGL((k_probes_tb2<T, CI, true, true, false>), dim3((unsigned)g.n_probe), dim3(PR_NT), 0, st2, g,
                       step);
  return hipGetLastError();
}

template <typename T>
hipError_t lists_any(const GridView<T>& g, int cls16, int variant, int step, int ty, const int4* tiles,
                     const int* counts, hipStream_t st, hipStream_t st2, void* ev) {
  if (variant == 3) {
    if (ty == 4)
      return cls16 ? launch_lists_tb2<T, uint16_t, 4>(g, step, tiles, counts, st, st2, ev)
                   : launch_lists_tb2<T, uint8_t, 4>(g, step, tiles, counts, st, st2, ev);
    if (ty == 12)
      return cls16 ? launch_lists_tb2<T, uint16_t, 12>(g, step, tiles, counts, st, st2, ev)
                   : launch_lists_tb2<T, uint8_t, 12>(g, step, tiles, counts, st, st2, ev);
    return cls16 ? launch_lists_tb2<T, uint16_t, 8>(g, step, tiles, counts, st, st2, ev)
                 : launch_lists_tb2<T, uint8_t, 8>(g, step, tiles, counts, st, st2, ev);
  }
  if (ty == 4)
    return cls16 ? launch_lists<T, uint16_t, 4>(g, step, tiles, counts, st, st2, ev)
                 : launch_lists<T, uint8_t, 4>(g, step, tiles, counts, st, st2, ev);
  return cls16 ? launch_lists<T, uint16_t, 8>(g, step, tiles, counts, st, st2, ev)
               : launch_lists<T, uint8_t, 8>(g, step, tiles, counts, st, st2, ev);
}

template <typename T, typename CI, bool PML, int TY>
hipError_t launch_tb2(const GridView<T>& g, int step, int kz, hipStream_t st) {
  const int ntx = (g.nx + 59) / 60, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + kz - 1) / kz;
  const long long nb = (long long)ntx * nty * ntz;
  if (nb > 0x7fffffff || (sizeof(CI) == 1 && g.ncls > 256)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_tb2<T, CI, PML, TY>), dim3((unsigned)nb), dim3(64 * (TY + 4)), 0, st, g, step, kz, ntx,
                     nty);
  return hipGetLastError();
}

template <typename T, typename CI>
hipError_t step_tb2(const GridView<T>& g, int step, int tile_y, int tile_z, hipStream_t st) {
  const int kz = tile_z > 0 ? tile_z : 64;
  const bool pml = g.npml > 0;
  if (tile_y == 4)
    return pml ? launch_tb2<T, CI, true, 4>(g, step, kz, st) : launch_tb2<T, CI, false, 4>(g, step, kz, st);
  if (tile_y == 12)
    return pml ? launch_tb2<T, CI, true, 12>(g, step, kz, st) : launch_tb2<T, CI, false, 12>(g, step, kz, st);
  return pml ? launch_tb2<T, CI, true, 8>(g, step, kz, st) : launch_tb2<T, CI, false, 8>(g, step, kz, st);
}

template <typename T>
hipError_t step_any(const GridView<T>& g, int cls16, int variant, int step, int tile_y, int tile_z,
                    hipStream_t st) {
  if (variant == 3)
    return cls16 ? step_tb2<T, uint16_t>(g, step, tile_y, tile_z, st)
                 : step_tb2<T, uint8_t>(g, step, tile_y, tile_z, st);
  if (variant == 2)
    return cls16 ? step_fused<T, uint16_t>(g, step, tile_y, tile_z, st)
                 : step_fused<T, uint8_t>(g, step, tile_y, tile_z, st);
  return cls16 ? step_split<T, uint16_t>(g, step, st) : step_split<T, uint8_t>(g, step, st);
}

int launch_lists_step(int prec, const void* view, int cls16, int variant, int step, int tile_y, const void* tiles,
                      const int* counts, void* stream, void* stream2, void* ev_src) {
  hipStream_t st = (hipStream_t)stream, st2 = (hipStream_t)stream2;
  const int4* t = (const int4*)tiles;
  const int ty = tile_y == 4 ? 4 : (tile_y == 12 && variant == 3) ? 12 : 8;
  hipError_t e = prec == 64 ? lists_any<double>(*(const GridView<double>*)view, cls16, variant, step, ty, t, counts,
                                                st, st2, ev_src)
                            : lists_any<float>(*(const GridView<float>*)view, cls16, variant, step, ty, t, counts,
                                               st, st2, ev_src);
  return (int)e;
}

int launch_step(int prec, const void* view, int cls16, int variant, int step, int tile_y, int tile_z,
                void* stream) {
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (prec == 64)
    e = step_any<double>(*(const GridView<double>*)view, cls16, variant, step, tile_y, tile_z, st);
  else
    e = step_any<float>(*(const GridView<float>*)view, cls16, variant, step, tile_y, tile_z, st);
  return (int)e;
}

template <typename T>
hipError_t probes_any(const GridView<T>& g, int step, hipStream_t st) {
  if (g.n_probe <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_probes<T>), dim3((unsigned)g.n_probe), dim3(PR_NT), 0, st, g, step);
  return hipGetLastError();
}

template <typename T>
hipError_t probes2_any(const GridView<T>& g, int cls16, int step, bool first, hipStream_t st) {
  if (g.n_probe <= 0) return hipSuccess;
  const dim3 grd((unsigned)g.n_probe), blk(PR_NT);
  const bool pml = g.npml > 0;
  if (!first) {  // the second sample only (two-step tile lists, which have a CPML)
    if (cls16) hipLaunchKernelGGL((k_probes_tb2<T, uint16_t, true, false, true>), grd, blk, 0, st, g, step);
    else hipLaunchKernelGGL((k_probes_tb2<T, uint8_t, true, false, true>), grd, blk, 0, st, g, step);
  } else if (cls16) {
    if (pml) hipLaunchKernelGGL((k_probes_tb2<T, uint16_t, true>), grd, blk, 0, st, g, step);
    else hipLaunchKernelGGL((k_probes_tb2<T, uint16_t, false>), grd, blk, 0, st, g, step);
  } else {
    if (pml) hipLaunchKernelGGL((k_probes_tb2<T, uint8_t, true>), grd, blk, 0, st, g, step);
    else hipLaunchKernelGGL((k_probes_tb2<T, uint8_t, false>), grd, blk, 0, st, g, step);
  }
  return hipGetLastError();
}

int launch_probes2(int prec, const void* view, int cls16, int step, int first, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == 64) return (int)probes2_any<double>(*(const GridView<double>*)view, cls16, step, first != 0, st);
  return (int)probes2_any<float>(*(const GridView<float>*)view, cls16, step, first != 0, st);
}

int launch_probes(int prec, const void* view, int step, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (prec == 64) return (int)probes_any<double>(*(const GridView<double>*)view, step, st);
  return (int)probes_any<float>(*(const GridView<float>*)view, step, st);
}

template <typename T, typename CI, bool PML>
hipError_t batch_step_t(const void* views, const void* tiles, int n_tiles, int tx, int ty, const int* d_step,
                        int offset, hipStream_t st) {
  const GridView<T>* v = (const GridView<T>*)views;
  const int4* t = (const int4*)tiles;
  if (tx == 32 && ty == 8)
    hipLaunchKernelGGL((k_fused_batch<T, CI, PML, 32, 8>), dim3(n_tiles), dim3(256), 0, st, v, t, d_step, offset);
  else if (tx == 32 && ty == 16)
    hipLaunchKernelGGL((k_fused_batch<T, CI, PML, 32, 16>), dim3(n_tiles), dim3(512), 0, st, v, t, d_step, offset);
  else if (tx == 64 && ty == 8)
    hipLaunchKernelGGL((k_fused_batch<T, CI, PML, 64, 8>), dim3(n_tiles), dim3(512), 0, st, v, t, d_step, offset);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int launch_batch_step(int prec, int cls16, int pml, const void* views, const void* tiles, int n_tiles, int tx,
                      int ty, const int* d_step, int offset, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n_tiles <= 0) return 0;
  hipError_t e;
  if (prec == 64) {
    if (cls16) e = pml ? batch_step_t<double, uint16_t, true>(views, tiles, n_tiles, tx, ty, d_step, offset, st)
                       : batch_step_t<double, uint16_t, false>(views, tiles, n_tiles, tx, ty, d_step, offset, st);
    else e = pml ? batch_step_t<double, uint8_t, true>(views, tiles, n_tiles, tx, ty, d_step, offset, st)
                 : batch_step_t<double, uint8_t, false>(views, tiles, n_tiles, tx, ty, d_step, offset, st);
  } else {
    if (cls16) e = pml ? batch_step_t<float, uint16_t, true>(views, tiles, n_tiles, tx, ty, d_step, offset, st)
                       : batch_step_t<float, uint16_t, false>(views, tiles, n_tiles, tx, ty, d_step, offset, st);
    else e = pml ? batch_step_t<float, uint8_t, true>(views, tiles, n_tiles, tx, ty, d_step, offset, st)
                 : batch_step_t<float, uint8_t, false>(views, tiles, n_tiles, tx, ty, d_step, offset, st);
  }
  return (int)e;
}

int launch_batch_probes(int prec, const void* views, const void* plist, int n, const int* d_step, int offset,
                        void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n <= 0) return 0;
  const dim3 grd((unsigned)n), blk(PR_NT);
  if (prec == 64)
    hipLaunchKernelGGL((k_probes_batch<double>), grd, blk, 0, st, (const GridView<double>*)views,
                       (const int2*)plist, n, d_step, offset);
  else
    hipLaunchKernelGGL((k_probes_batch<float>), grd, blk, 0, st, (const GridView<float>*)views,
                       (const int2*)plist, n, d_step, offset);
  return (int)hipGetLastError();
}

// Probes of both steps of a batched two-step pass (one block per (grid,
// probe) pair).
int batch_probes_tb2(int prec, int cls16, const void* views, const void* plist, int n_probes, const int* d_step,
                     int offset, hipStream_t st) {
  if (n_probes <= 0) return 0;
  const dim3 grd((unsigned)n_probes), blk(PR_NT);
  if (prec == 64) {
    if (cls16)
      hipLaunchKernelGGL((k_probes_tb2_batch<double, uint16_t>), grd, blk, 0, st, (const GridView<double>*)views,
                         (const int2*)plist, n_probes, d_step, offset);
    else
      hipLaunchKernelGGL((k_probes_tb2_batch<double, uint8_t>), grd, blk, 0, st, (const GridView<double>*)views,
                         (const int2*)plist, n_probes, d_step, offset);
  } else {
    if (cls16)
      hipLaunchKernelGGL((k_probes_tb2_batch<float, uint16_t>), grd, blk, 0, st, (const GridView<float>*)views,
                         (const int2*)plist, n_probes, d_step, offset);
    else
      hipLaunchKernelGGL((k_probes_tb2_batch<float, uint8_t>), grd, blk, 0, st, (const GridView<float>*)views,
                         (const int2*)plist, n_probes, d_step, offset);
  }
  return (int)hipGetLastError();
}

// Group q of the pass's tile list runs the instantiation for the slabs its
// tiles reach (FP64: the all-axes one).
template <typename T, typename CI>
hipError_t batch_group_t(int q, const void* views, const int4* t, int count, const int* d_step, int offset,
                         hipStream_t st) {
  constexpr bool D = sizeof(T) == 8;
  const GridView<T>* v = (const GridView<T>*)views;
  const dim3 blk(64 * 12), grd((unsigned)count);
  if (q == 0) hipLaunchKernelGGL((k_tb2_batch<T, CI, 8, D ? 7 : 4>), grd, blk, 0, st, v, t, d_step, offset);
  if (q == 1) hipLaunchKernelGGL((k_tb2_batch<T, CI, 8, D ? 7 : 5>), grd, blk, 0, st, v, t, d_step, offset);
  if (q == 2) hipLaunchKernelGGL((k_tb2_batch<T, CI, 8, D ? 7 : 6>), grd, blk, 0, st, v, t, d_step, offset);
  if (q == 3) hipLaunchKernelGGL((k_tb2_batch<T, CI, 8, 7>), grd, blk, 0, st, v, t, d_step, offset);
  return hipGetLastError();
}

template <typename T, typename CI>
hipError_t batch_queue_t(const void* views, const int4* tiles_a, const QRuns& runs_a, int blocks_a,
                         const int4* tiles_b, const QRuns& runs_b, int blocks_b, int* ctr, const int* d_step,
                         int offset, hipStream_t st, hipStream_t st2, hipEvent_t ev_fork, hipEvent_t ev_join) {
  const GridView<T>* v = (const GridView<T>*)views;
  hipLaunchKernelGGL(k_qreset, dim3(1), dim3(64), 0, st, ctr);
  // the all-axes path (slower per cell) on the second stream, launched
  // first: both launches fill the device, so the x-slab path's blocks start
  // as the all-axes ones drain and fill the end of the pass
  const bool fork = blocks_a > 0 && blocks_b > 0;
  hipError_t e = hipSuccess;
  if (fork) {
    e = hipEventRecord(ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st2, ev_fork, 0);
    if (e != hipSuccess) return e;
  }
  if (blocks_b > 0)
    hipLaunchKernelGGL((k_tb2_batch_q<T, CI, 7>), dim3((unsigned)blocks_b), dim3(768), 0, fork ? st2 : st, v,
                       tiles_b, runs_b, ctr + 8, d_step, offset);
  if (blocks_a > 0)
    hipLaunchKernelGGL((k_tb2_batch_q<T, CI, 5>), dim3((unsigned)blocks_a), dim3(768), 0, st, v, tiles_a, runs_a, ctr,
                       d_step, offset);
  if (fork) {
    e = hipEventRecord(ev_join, st2);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev_join, 0);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

template <typename T, typename CI, int AXP>
int queue_blocks_t() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tb2_batch_q<T, CI, AXP>, 768, 0) != hipSuccess) return 0;
  return cus * std::max(per, 1);
}

int batch_queue_blocks(int prec, int cls16, int axp) {
  if (prec == 64) {
    if (axp == 5) return cls16 ? queue_blocks_t<double, uint16_t, 5>() : queue_blocks_t<double, uint8_t, 5>();
    return cls16 ? queue_blocks_t<double, uint16_t, 7>() : queue_blocks_t<double, uint8_t, 7>();
  }
  if (axp == 5) return cls16 ? queue_blocks_t<float, uint16_t, 5>() : queue_blocks_t<float, uint8_t, 5>();
  return cls16 ? queue_blocks_t<float, uint16_t, 7>() : queue_blocks_t<float, uint8_t, 7>();
}

int launch_batch_pass_queue(int prec, int cls16, const void* views, const void* tiles_a, const QRuns* runs_a,
                            int blocks_a, const void* tiles_b, const QRuns* runs_b, int blocks_b, int* ctr,
                            const void* plist, int n_probes, const int* d_step, int offset, void* stream,
                            void* stream2, void* ev_fork, void* ev_join) {
  hipStream_t st = (hipStream_t)stream, st2 = (hipStream_t)stream2;
  hipEvent_t ef = (hipEvent_t)ev_fork, ej = (hipEvent_t)ev_join;
  const int4 *ta = (const int4*)tiles_a, *tb = (const int4*)tiles_b;
  hipError_t e;
  if (prec == 64)
    e = cls16 ? batch_queue_t<double, uint16_t>(views, ta, *runs_a, blocks_a, tb, *runs_b, blocks_b, ctr, d_step,
                                                offset, st, st2, ef, ej)
              : batch_queue_t<double, uint8_t>(views, ta, *runs_a, blocks_a, tb, *runs_b, blocks_b, ctr, d_step,
                                               offset, st, st2, ef, ej);
  else
    e = cls16 ? batch_queue_t<float, uint16_t>(views, ta, *runs_a, blocks_a, tb, *runs_b, blocks_b, ctr, d_step,
                                               offset, st, st2, ef, ej)
              : batch_queue_t<float, uint8_t>(views, ta, *runs_a, blocks_a, tb, *runs_b, blocks_b, ctr, d_step,
                                              offset, st, st2, ef, ej);
  if (e != hipSuccess) return (int)e;
  return batch_probes_tb2(prec, cls16, views, plist, n_probes, d_step, offset, st);
}

int launch_batch_pass_tb2(int prec, int cls16, const void* views, const void* tiles, const int* counts,
                          const void* plist, int n_probes, const int* d_step, int offset, void* stream,
                          void* stream2, void* ev_fork, void* ev_join) {
  hipStream_t st = (hipStream_t)stream, st2 = (hipStream_t)stream2;
  hipError_t e = hipSuccess;
  // group 1 on the second stream beside the others, when both are there
  const bool fork = st2 && counts[1] > 0 && counts[0] + counts[2] + counts[3] > 0;
  if (fork) {
    e = hipEventRecord((hipEvent_t)ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st2, (hipEvent_t)ev_fork, 0);
  }
  const int4* t = (const int4*)tiles;
  for (int q = 0; q < 4 && e == hipSuccess; t += counts[q], ++q) {
    if (counts[q] <= 0) continue;
    hipStream_t s = fork && q == 1 ? st2 : st;
    if (prec == 64)
      e = cls16 ? batch_group_t<double, uint16_t>(q, views, t, counts[q], d_step, offset, s)
                : batch_group_t<double, uint8_t>(q, views, t, counts[q], d_step, offset, s);
    else
      e = cls16 ? batch_group_t<float, uint16_t>(q, views, t, counts[q], d_step, offset, s)
                : batch_group_t<float, uint8_t>(q, views, t, counts[q], d_step, offset, s);
  }
  if (fork && e == hipSuccess) {
    e = hipEventRecord((hipEvent_t)ev_join, st2);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, (hipEvent_t)ev_join, 0);
  }
  if (e != hipSuccess) return (int)e;
  return batch_probes_tb2(prec, cls16, views, plist, n_probes, d_step, offset, st);
}

__global__ void k_set(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

int launch_set(int* d, int v, void* stream) {
  hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, (hipStream_t)stream, d, v);
  return (int)hipGetLastError();
}

int launch_add(int* d, int v, void* stream) {
  hipLaunchKernelGGL(k_add, dim3(1), dim3(64), 0, (hipStream_t)stream, d, v);
  return (int)hipGetLastError();
}

}  // namespace mi355fdtd
