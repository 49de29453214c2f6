// fdtd_tile.h -- device-side building blocks of the Yee FDTD kernels shared
// by the kernel translation units: per-point H and E updates with CPML, the
// source test of a column, and the fused one-step tile.
#pragma once
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"
#include "yee_update.h"

namespace mi355fdtd {

// ---------------------------------------------------------------------------
// per-point updates shared by all variants
// ---------------------------------------------------------------------------

// Slab-local CPML positions of node (x, y, k) along each axis (-1 outside).
// AX masks the axes whose slabs the caller can reach (bit 0 x, 1 y, 2 z); the
// other positions are the constant -1, which removes their CPML code.
template <typename T, int AX = 7>
__device__ __forceinline__ void slabs(const GridView<T>& g, int x, int y, int k, int l[3]) {
  l[0] = (AX & 1) ? slab_pos(x, g.nx, g.npml) : -1;
  l[1] = (AX & 2) ? slab_pos(y, g.ny, g.npml) : -1;
  l[2] = (AX & 4) ? slab_pos(k, g.nz, g.npml) : -1;
}

// The step a single-grid kernel works on: its argument, plus the device
// counter when the launch is replayed from a captured graph.
template <typename T>
__device__ __forceinline__ int gstep(const GridView<T>& g, int step) {
  return g.dstep ? *g.dstep + step : step;
}

// CPML state of one node: ps[axis][q], q = 0 for the component along
// axis+1, q = 1 for axis+2; kind 0 = E-type, 1 = H-type.
template <typename T>
__device__ __forceinline__ void psi_load(const GridView<T>& g, int kind, const int l[3], int x, int y, int k,
                                         T ps[3][2]) {
  for (int u = 0; u < 3; ++u) {
    ps[u][0] = ps[u][1] = T(0);
    if (l[u] >= 0) {
      const unsigned q = psi_index(u, l[u], x, y, k, g.nx, g.ny, g.npml) + (unsigned)(2 * kind) * g.pel[u];
      ps[u][0] = ldg(g.pib[u], q);
      ps[u][1] = ldg(g.pib[u], q + g.pel[u]);
    }
  }
}
template <typename T>
__device__ __forceinline__ void psi_store(const GridView<T>& g, int kind, const int l[3], int x, int y, int k,
                                          const T ps[3][2]) {
  for (int u = 0; u < 3; ++u) {
    if (l[u] >= 0) {
      const unsigned q = psi_index(u, l[u], x, y, k, g.nx, g.ny, g.npml) + (unsigned)(2 * kind) * g.pel[u];
      stg(g.pob[u], q, ps[u][0]);
      stg(g.pob[u], q + g.pel[u], ps[u][1]);
    }
  }
}

// CPML profile values (b - 1, c, 1/kappa) of one axis at slab position l;
// `row` is P_BE or P_BH.  ProfG reads the grid's tables in global memory.
template <typename T>
struct Prof3 {
  T b, c, k;
};
template <typename T>
struct ProfG {
  const GridView<T>& g;
  template <int U>
  __device__ __forceinline__ Prof3<T> at(int row, int l) const {
    const int tn = 2 * g.npml;
    const unsigned q = (unsigned)(row * tn + l);
    return {ldg(g.prof[U], q), ldg(g.prof[U], q + tn), ldg(g.prof[U], q + 2 * tn)};
  }
};

// H^{n+1/2} of one node from E^n at the node (ex, ey, ez), at x+1 (ey_i,
// ez_i), y+1 (ex_j, ez_j) and k+1 (ex_k, ey_k); ps is the node's H-type CPML
// state, advanced in place.
template <typename T, bool PML, typename PF>
__device__ __forceinline__ void h_core_pf(const PF& pf, const int l[3], const T* cf, T ex, T ey, T ez, T ex_j,
                                          T ex_k, T ey_i, T ey_k, T ez_i, T ez_j, const T hold[3], T ps[3][2],
                                          T hnew[3]) {
  T a_hx = ey_k - ey, b_hx = ez_j - ez;  // Hx: dEy/dz - dEz/dy
  T a_hy = ez_i - ez, b_hy = ex_k - ex;  // Hy: dEz/dx - dEx/dz
  T a_hz = ex_j - ex, b_hz = ey_i - ey;  // Hz: dEx/dy - dEy/dx
  if (PML) {
    if (l[0] >= 0) {  // Hy (dEz/dx), Hz (dEy/dx)
      const Prof3<T> q = pf.template at<0>(P_BH, l[0]);
      a_hy = pml_step(a_hy, ps[0][0], q.b, q.c, q.k);
      b_hz = pml_step(b_hz, ps[0][1], q.b, q.c, q.k);
    }
    if (l[1] >= 0) {  // Hz (dEx/dy), Hx (dEz/dy)
      const Prof3<T> q = pf.template at<1>(P_BH, l[1]);
      a_hz = pml_step(a_hz, ps[1][0], q.b, q.c, q.k);
      b_hx = pml_step(b_hx, ps[1][1], q.b, q.c, q.k);
    }
    if (l[2] >= 0) {  // Hx (dEy/dz), Hy (dEx/dz)
      const Prof3<T> q = pf.template at<2>(P_BH, l[2]);
      a_hx = pml_step(a_hx, ps[2][0], q.b, q.c, q.k);
      b_hy = pml_step(b_hy, ps[2][1], q.b, q.c, q.k);
    }
  }
  hnew[0] = h_new(hold[0], cf[K_DBX], a_hx, b_hx);
  hnew[1] = h_new(hold[1], cf[K_DBY], a_hy, b_hy);
  hnew[2] = h_new(hold[2], cf[K_DBZ], a_hz, b_hz);
}

// E^{n+1} of node n from H^{n+1/2} at the node (hx, hy, hz), at x-1 (hy_i,
// hz_i), y-1 (hx_j, hz_j) and k-1 (hx_k, hy_k), then the sources of `step`;
// ps is the node's E-type CPML state, advanced in place.
template <typename T, bool PML, typename PF>
__device__ __forceinline__ void e_core_pf(const PF& pf, const GridView<T>& g, const int l[3], unsigned n,
                                          const T* cf, T hx, T hy, T hz, T hx_j, T hx_k, T hy_i, T hy_k, T hz_i,
                                          T hz_j, const T eold[3], int step, T ps[3][2], T enew[3], int slo,
                                          int shi) {
  T a_ex = hz - hz_j, b_ex = hy - hy_k;  // Ex: dHz/dy - dHy/dz
  T a_ey = hx - hx_k, b_ey = hz - hz_i;  // Ey: dHx/dz - dHz/dx
  T a_ez = hy - hy_i, b_ez = hx - hx_j;  // Ez: dHy/dx - dHx/dy
  if (PML) {
    if (l[0] >= 0) {  // Ey (dHz/dx), Ez (dHy/dx)
      const Prof3<T> q = pf.template at<0>(P_BE, l[0]);
      b_ey = pml_step(b_ey, ps[0][0], q.b, q.c, q.k);
      a_ez = pml_step(a_ez, ps[0][1], q.b, q.c, q.k);
    }
    if (l[1] >= 0) {  // Ez (dHx/dy), Ex (dHz/dy)
      const Prof3<T> q = pf.template at<1>(P_BE, l[1]);
      b_ez = pml_step(b_ez, ps[1][0], q.b, q.c, q.k);
      a_ex = pml_step(a_ex, ps[1][1], q.b, q.c, q.k);
    }
    if (l[2] >= 0) {  // Ex (dHy/dz), Ey (dHx/dz)
      const Prof3<T> q = pf.template at<2>(P_BE, l[2]);
      b_ex = pml_step(b_ex, ps[2][0], q.b, q.c, q.k);
      a_ey = pml_step(a_ey, ps[2][1], q.b, q.c, q.k);
    }
  }
  enew[0] = e_new(eold[0], cf[K_CAX], cf[K_CBX], a_ex, b_ex);
  enew[1] = e_new(eold[1], cf[K_CAY], cf[K_CBY], a_ey, b_ey);
  enew[2] = e_new(eold[2], cf[K_CAZ], cf[K_CBZ], a_ez, b_ez);
  // ideal current sources: E -= Cb I / dx^2 (precomputed per step), from the
  // entries [slo, shi) of the source list (empty where none can apply).  The
  // tile kernels pass a range that is uniform across the wave, so that the
  // scan reads the list with scalar loads.
  for (int s = slo; s < shi; ++s) {
    if ((unsigned)ldg(g.src_idx, (unsigned)s) != n) continue;
    const T v = ldg(g.src_amp, (unsigned)s * (unsigned)g.max_steps + (unsigned)step);
    const int comp = ldg(g.src_comp, (unsigned)s);
    enew[0] = comp == 0 ? enew[0] - v : enew[0];
    enew[1] = comp == 1 ? enew[1] - v : enew[1];
    enew[2] = comp == 2 ? enew[2] - v : enew[2];
  }
}

template <typename T, bool PML>
__device__ __forceinline__ void h_core(const GridView<T>& g, const int l[3], const T* cf, T ex, T ey, T ez,
                                       T ex_j, T ex_k, T ey_i, T ey_k, T ez_i, T ez_j, const T hold[3],
                                       T ps[3][2], T hnew[3]) {
  h_core_pf<T, PML>(ProfG<T>{g}, l, cf, ex, ey, ez, ex_j, ex_k, ey_i, ey_k, ez_i, ez_j, hold, ps, hnew);
}
template <typename T, bool PML>
__device__ __forceinline__ void e_core(const GridView<T>& g, const int l[3], unsigned n, const T* cf, T hx, T hy,
                                       T hz, T hx_j, T hx_k, T hy_i, T hy_k, T hz_i, T hz_j, const T eold[3],
                                       int step, T ps[3][2], T enew[3], int slo, int shi) {
  e_core_pf<T, PML>(ProfG<T>{g}, g, l, n, cf, hx, hy, hz, hx_j, hx_k, hy_i, hy_k, hz_i, hz_j, eold, step, ps, enew,
                    slo, shi);
}

// Sources of column n0 (= x + nx*y) as a range [lo, hi) of the grouped
// source list with their planes [klo, khi]; empty (lo = hi = 0, no planes)
// if the column holds none, if !on, or if they all lie outside planes
// [ka, kb].
struct SrcRange {
  int lo, hi, klo, khi;
  // the range to scan for plane k
  __device__ __forceinline__ int first(int k) const { return k >= klo && k <= khi ? lo : 0; }
  __device__ __forceinline__ int last(int k) const { return k >= klo && k <= khi ? hi : 0; }
};
template <typename T>
__device__ __forceinline__ SrcRange src_column(const GridView<T>& g, unsigned n0, bool on, int ka, int kb) {
  SrcRange r{0, 0, 1, 0};
  const int f = on ? ldg(g.src_first, n0) : -1;
  if (f >= 0) {
    const int kr = ldg(g.src_kr, n0), kl = kr & 0xffff, kh = (int)((unsigned)kr >> 16);
    if (kb >= kl && ka <= kh) r = SrcRange{f & 0xfffff, (f & 0xfffff) + (f >> 20), kl, kh};
  }
  return r;
}
// The same over a whole wave: the union of its lanes' ranges (contiguous in
// the list when the lanes' columns are, as along one row), uniform across
// the wave.  The tile kernels evaluate it once per tile, so that the
// per-plane scan reads the list with scalar loads, and waves with no source
// skip it.  Every lane of the wave must call it.
template <typename T>
__device__ __forceinline__ SrcRange src_wave(const GridView<T>& g, unsigned n0, bool on, int ka, int kb) {
  const SrcRange c = src_column(g, n0, on, ka, kb);
  const bool has = c.hi > c.lo;
  int lo = has ? c.lo : 0x7fffffff, hi = has ? c.hi : 0, klo = has ? c.klo : 0x7fffffff, khi = has ? c.khi : -1;
  for (int m = 1; m < 64; m <<= 1) {
    lo = min(lo, __shfl_xor(lo, m, 64));
    hi = max(hi, __shfl_xor(hi, m, 64));
    klo = min(klo, __shfl_xor(klo, m, 64));
    khi = max(khi, __shfl_xor(khi, m, 64));
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  hi = __builtin_amdgcn_readfirstlane(hi);
  if (hi <= lo) return SrcRange{0, 0, 1, 0};
  return SrcRange{lo, hi, __builtin_amdgcn_readfirstlane(klo), __builtin_amdgcn_readfirstlane(khi)};
}
// For one node (x, y, k): its column's range if it covers plane k.
template <typename T>
__device__ __forceinline__ SrcRange src_node(const GridView<T>& g, int x, int y, int k) {
  return src_column(g, (unsigned)x + (unsigned)g.nx * (unsigned)y, true, k, k);
}

// One-step wrappers: CPML state from the input set, written (optionally for
// H) to the output set.
template <typename T, bool PML, int AX = 7>
__device__ __forceinline__ void h_point(const GridView<T>& g, int x, int y, int k, const T* cf, T ex, T ey,
                                        T ez, T ex_j, T ex_k, T ey_i, T ey_k, T ez_i, T ez_j, const T hold[3],
                                        bool store_psi, T hnew[3]) {
  int l[3] = {-1, -1, -1};
  T ps[3][2];
  if (PML) {
    slabs<T, AX>(g, x, y, k, l);
    psi_load(g, 1, l, x, y, k, ps);
  }
  h_core<T, PML>(g, l, cf, ex, ey, ez, ex_j, ex_k, ey_i, ey_k, ez_i, ez_j, hold, ps, hnew);
  if (PML && store_psi) psi_store(g, 1, l, x, y, k, ps);
}

template <typename T, bool PML, int AX = 7>
__device__ __forceinline__ void e_point(const GridView<T>& g, int x, int y, int k, unsigned n, const T* cf,
                                        T hx, T hy, T hz, T hx_j, T hx_k, T hy_i, T hy_k, T hz_i, T hz_j,
                                        const T eold[3], int step, T enew[3], int slo, int shi) {
  int l[3] = {-1, -1, -1};
  T ps[3][2];
  if (PML) {
    slabs<T, AX>(g, x, y, k, l);
    psi_load(g, 0, l, x, y, k, ps);
  }
  e_core<T, PML>(g, l, n, cf, hx, hy, hz, hx_j, hx_k, hy_i, hy_k, hz_i, hz_j, eold, step, ps, enew, slo, shi);
  if (PML) psi_store(g, 0, l, x, y, k, ps);
}

// Pole currents of a Debye node (index n) after its plain E update:
// subtract sum_p gam_p J_p^n from the new E, then advance each J_p with the
// change of E.  debye_load fetches J^n without branches (poles beyond npole
// read an aliased array and count as 0); debye_apply does the arithmetic
// with the class's pole factors dt (in global memory, or in LDS with
// LDS = true).  Nodes whose class has no pole term skip both, so their J
// stays 0 without traffic.  Every variant goes through these two, so they
// agree bit for bit.
// (the values loaded for p >= npole are masked where they are used, so that
// no wait on a load in flight is needed before then)
template <typename T>
__device__ __forceinline__ void debye_load(const DebyeView<T>& d, unsigned n, T jo[3][D_MAXPOLE]) {
  for (int a = 0; a < 3; ++a)
    for (int p = 0; p < D_MAXPOLE; ++p) jo[a][p] = ldg(d.j[a * D_MAXPOLE + p], n);
}
template <typename T, bool LDS = false>
__device__ __forceinline__ void debye_apply(const DebyeView<T>& d, const T* dt, unsigned n, const T eold[3], T e[3],
                                            const T jo[3][D_MAXPOLE]) {
  auto f = [&](int q) -> T { return LDS ? dt[q] : ldg(dt, (unsigned)q); };
  for (int a = 0; a < 3; ++a) {
    T sum = T(0);
    for (int p = 0; p < D_MAXPOLE; ++p) sum += f(a * 2 * D_MAXPOLE + 2 * p + 1) * (p < d.npole ? jo[a][p] : T(0));
    e[a] -= sum;
    const T de = e[a] - eold[a];
    for (int p = 0; p < D_MAXPOLE; ++p)
      if (p < d.npole) stg(d.j[a * D_MAXPOLE + p], n, d.kp[p] * jo[a][p] + f(a * 2 * D_MAXPOLE + 2 * p) * de);
  }
}
template <typename T>
__device__ __forceinline__ void debye_point(const DebyeView<T>& d, int cid, unsigned n, const T eold[3], T e[3]) {
  if (!ldg(d.dflag, (unsigned)cid)) return;
  T jo[3][D_MAXPOLE];
  debye_load(d, n, jo);
  debye_apply(d, d.dtab + cid * D_STRIDE, n, eold, e, jo);
}

// ---------------------------------------------------------------------------
// fused variant
//
// Block = TY waves owning the x-y tile [i0, i0+64) x [j0, j0+TY) over the
// z-chunk [k0, k1); thread (tx, ty) owns column (i0+tx, j0+ty) and keeps its
// own E and H in registers.  LDS holds only what neighbours need: E^n of
// planes k and k+1 on the region [i0-1, i0+64] x [j0-1, j0+TY] (2-plane
// ring) and H^{n+1/2} of plane k on [i0-1, i0+63] x [j0-1, j0+TY-1].  The
// low-side H halo (row j0-1, column i0-1) is recomputed by the first
// threads with the owners' arithmetic; the E halo is loaded by the last
// threads.  Loads for plane k+1 are issued before plane k is computed.
// Per plane: stage E(k+1) -> barrier -> H(k) -> barrier -> E(k).
// ---------------------------------------------------------------------------

// Block b of nb (dealt to the 8 XCDs round robin) takes list entry
// xcd_runs(b, nb): each XCD gets runs of XCD_RUN consecutive entries, interleaved
// with the other XCDs' runs.  Neighbouring tiles then share an L2 while every
// XCD's reads stay spread over the whole grid.  Blocks past the last full
// round of runs keep their own index, so the map is one to one.  On the
// 512 x 512 x 384 two-step pass (Mcell-updates/s, same process), runs of 9
// gave 112.3k, 4 112.1k, 2 110.7k, 1 (plain order) 107.8k, 18 111.9k,
// 36 110.5k, 72 107.6k, and one run per XCD (xcd_tile) 106.0k.
constexpr int XCD_RUN = 9;
__device__ __forceinline__ int xcd_runs(int b, int nb) {
  const int nf = nb / (8 * XCD_RUN) * (8 * XCD_RUN);
  if (b >= nf) return b;
  const int x = b & 7, t = b >> 3, g = t / XCD_RUN;
  return (g * 8 + x) * XCD_RUN + (t - g * XCD_RUN);
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run
// of tiles so that neighbouring tiles share that XCD's L2 for their halos.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, t = b / 8;
  return x * q + (x < r ? x : r) + t;
}

template <typename T>
__device__ __forceinline__ void load3(const GridView<T>& g, bool ok, unsigned n, T v[3]) {
  v[0] = ok ? ldg(g.fi[0], n) : T(0);
  v[1] = ok ? ldg(g.fi[1], n) : T(0);
  v[2] = ok ? ldg(g.fi[2], n) : T(0);
}
template <typename T>
__device__ __forceinline__ void load3h(const GridView<T>& g, bool ok, unsigned n, T v[3]) {
  v[0] = ok ? ldg(g.fi[3], n) : T(0);
  v[1] = ok ? ldg(g.fi[4], n) : T(0);
  v[2] = ok ? ldg(g.fi[5], n) : T(0);
}

template <typename T, int TX, int TY>
struct FusedSmem {
  static constexpr int EW = TX + 2, EH = TY + 2, HW = TX + 1, HH = TY + 1;
  T se[2][3][EH][EW];
  T sh[3][HH][HW];
  T stab[256 * K_STRIDE];
};

// One tile [i0, i0+TX) x [j0, j0+TY) x [k0, k1) of one grid, one step.
// DB: the grid has Debye media; each own E node also advances its pole
// currents (node-local, in place: one thread per node per step).  J^n of
// plane k+1 is fetched at the end of plane k's iteration, so that its
// latency hides behind the next plane's staging and H stage; the class that
// decides whether to fetch it is read a plane earlier than the one the H and
// E stages use, so that the fetch waits on no load of the current plane.
// With 1-byte classes in FP32 the pole factors and flags sit in LDS (sdt:
// ncls * D_STRIDE values, sdf: ncls bytes, both supplied by the kernel).
// PF: prefetch distance in planes (1 or 2): plane k's iteration issues the
// loads of H and classes of plane k + PF and of E of plane k + 1 + PF; with
// 2 the loads have a whole iteration more to arrive, for one more set of
// registers.
template <typename T, typename CI, bool PML, int TX, int TY, int AX = 7, bool DB = false, int PF = 1>
__device__ __forceinline__ void fused_tile(const GridView<T>& g, FusedSmem<T, TX, TY>& sm, int i0, int j0,
                                           int k0, int k1, int step, const DebyeView<T>* dv = nullptr,
                                           T* sdt = nullptr, unsigned char* sdf = nullptr) {
  constexpr int NT = TX * TY, EW = TX + 2, EH = TY + 2, HW = TX + 1;
  constexpr int NHE = 2 * EW + 2 * TY;  // E halo points
  constexpr int NHH = HW + TY;          // H halo points
  static_assert(NHE <= NT && NHH <= NT, "tile too small for its halo");
  constexpr bool LDS_TAB = sizeof(CI) == 1;
  auto& se = sm.se;
  auto& sh = sm.sh;
  T* stab = sm.stab;

  if (k0 >= k1) return;  // uniform per block, before any barrier
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const unsigned sxy = (unsigned)g.sxy;
  const CI* cls = (const CI*)g.cls;

  if (LDS_TAB) {
    for (int q = tid; q < g.ncls * K_STRIDE; q += NT) stab[q] = ldg(g.ctab, (unsigned)q);
  }
  auto coef = [&](int c) -> const T* { return LDS_TAB ? stab + c * K_STRIDE : g.ctab + c * K_STRIDE; };
  constexpr bool DLDS = DB && sizeof(CI) == 1 && sizeof(T) == 4;
  if (DLDS) {
    for (int q = tid; q < g.ncls * D_STRIDE; q += NT) sdt[q] = ldg(dv->dtab, (unsigned)q);
    for (int q = tid; q < g.ncls; q += NT) sdf[q] = ldg(dv->dflag, (unsigned)q);
  }
  auto dflag = [&](int c) -> bool { return DLDS ? sdf[c] != 0 : ldg(dv->dflag, (unsigned)c) != 0; };

  // own column
  const int i = i0 + tx, j = j0 + ty;
  const bool own = i < nx && j < ny;
  const unsigned n0 = own ? (unsigned)i + (unsigned)nx * (unsigned)j : 0u;  // + sxy * k
  const SrcRange srcr = src_wave(g, n0, own, k0, k1 - 1);
  // E halo point (threads NT-NHE .. NT-1)
  int er = 0, ec = 0;
  bool eh = false;
  {
    const int h = tid - (NT - NHE);
    if (h >= 0) {
      eh = true;
      if (h < EW) { er = 0; ec = h; }
      else if (h < 2 * EW) { er = EH - 1; ec = h - EW; }
      else if (h < 2 * EW + TY) { er = h - 2 * EW + 1; ec = 0; }
      else { er = h - 2 * EW - TY + 1; ec = EW - 1; }
    }
  }
  const int ex_x = i0 - 1 + ec, ex_y = j0 - 1 + er;
  const bool eh_in = eh && ex_x >= 0 && ex_x < nx && ex_y >= 0 && ex_y < ny;
  const unsigned en0 = eh_in ? (unsigned)ex_x + (unsigned)nx * (unsigned)ex_y : 0u;
  // H halo point (threads 0 .. NHH-1): row j0-1 (c = 0..64) then column i0-1
  const bool hh = tid < NHH;
  const int hr = tid < HW ? 0 : tid - HW + 1, hc = tid < HW ? tid : 0;
  const int hx_x = i0 - 1 + hc, hx_y = j0 - 1 + hr;
  const bool hh_in = hh && hx_x >= 0 && hx_x < nx && hx_y >= 0 && hx_y < ny;
  const unsigned hn0 = hh_in ? (unsigned)hx_x + (unsigned)nx * (unsigned)hx_y : 0u;

  // ---- prologue: H^{n+1/2} of plane k0-1 at the own column (needed as H(k-1))
  static_assert(PF == 1 || PF == 2, "prefetch distance 1 or 2");
  T ecur[3], enext[3], xe_next[3], hold[3], xh_old[3], hm[2] = {T(0), T(0)};
  int cls_cur = 0, xcls_cur = 0;
  // PF 2: E of plane k+2, H and classes of plane k+1, already in flight
  T e2[3], xe2[3], h2[3], xh2[3];
  int c2 = 0, xc2 = 0;
  {
    const int kb = k0 - 1;
    T eb[3], xeb[3], xe0[3], hb[3];
    load3(g, own && kb >= 0, n0 + sxy * (unsigned)(kb), eb);
    load3(g, eh_in && kb >= 0, en0 + sxy * (unsigned)(kb), xeb);
    load3(g, own, n0 + sxy * (unsigned)(k0), ecur);
    load3(g, eh_in, en0 + sxy * (unsigned)(k0), xe0);
    load3h(g, own && kb >= 0, n0 + sxy * (unsigned)(kb), hb);
    const int cb = (own && kb >= 0) ? (int)ldg(cls, n0 + sxy * (unsigned)kb) : 0;
    const int sb = (kb + 2) & 1, s0 = k0 & 1;
    for (int c = 0; c < 3; ++c) {
      se[sb][c][ty + 1][tx + 1] = eb[c];
      se[s0][c][ty + 1][tx + 1] = ecur[c];
      if (eh) {
        se[sb][c][er][ec] = xeb[c];
        se[s0][c][er][ec] = xe0[c];
      }
    }
    __syncthreads();
    if (own && kb >= 0) {
      T h[3];
      h_point<T, PML, AX>(g, i, j, kb, coef(cb), eb[0], eb[1], eb[2], se[sb][0][ty + 2][tx + 1], ecur[0],
                      se[sb][1][ty + 1][tx + 2], ecur[1], se[sb][2][ty + 1][tx + 2], se[sb][2][ty + 2][tx + 1],
                      hb, false, h);
      hm[0] = h[0];
      hm[1] = h[1];
    }
    // plane k0 inputs and plane k0+1 E
    load3h(g, own, n0 + sxy * (unsigned)(k0), hold);
    load3h(g, hh_in, hn0 + sxy * (unsigned)(k0), xh_old);
    cls_cur = own ? (int)ldg(cls, n0 + sxy * (unsigned)k0) : 0;
    xcls_cur = hh_in ? (int)ldg(cls, hn0 + sxy * (unsigned)k0) : 0;
    const bool nxt = k0 + 1 < nz;
    load3(g, own && nxt, n0 + sxy * (unsigned)(k0 + 1), enext);
    load3(g, eh_in && nxt, en0 + sxy * (unsigned)(k0 + 1), xe_next);
    if (PF == 2) {
      const bool e2ok = k0 + 2 < nz, h2ok = k0 + 1 < k1;
      load3(g, own && e2ok, n0 + sxy * (unsigned)(k0 + 2), e2);
      load3(g, eh_in && e2ok, en0 + sxy * (unsigned)(k0 + 2), xe2);
      load3h(g, own && h2ok, n0 + sxy * (unsigned)(k0 + 1), h2);
      load3h(g, hh_in && h2ok, hn0 + sxy * (unsigned)(k0 + 1), xh2);
      c2 = (own && h2ok) ? (int)ldg(cls, n0 + sxy * (unsigned)(k0 + 1)) : 0;
      xc2 = (hh_in && h2ok) ? (int)ldg(cls, hn0 + sxy * (unsigned)(k0 + 1)) : 0;
    }
    __syncthreads();  // plane kb's LDS slot is rewritten below
  }
  T jcur[3][D_MAXPOLE];
  bool dcur = false;
  int dcls1 = 0;  // PF 1: class of plane k + 1, read one plane ahead of cpf
  if (DB) {
    dcur = own && dflag(cls_cur);
    if (dcur) debye_load(*dv, n0 + sxy * (unsigned)k0, jcur);
    if (PF == 1) dcls1 = (own && k0 + 1 < k1) ? (int)ldg(cls, n0 + sxy * (unsigned)(k0 + 1)) : 0;
  }

  for (int k = k0; k < k1; ++k) {
    const int s = k & 1, s1 = s ^ 1;
    // (a) stage E(k+1)
    for (int c = 0; c < 3; ++c) {
      se[s1][c][ty + 1][tx + 1] = enext[c];
      if (eh) se[s1][c][er][ec] = xe_next[c];
    }
    // (b) prefetch the inputs of plane k+PF and E(k+1+PF)
    T epf[3], xepf[3], hpf[3], xhpf[3];
    const int kh = k + PF, ke = k + 1 + PF;
    const bool n1 = kh < k1, n2 = ke < nz;
    load3(g, own && n2, n0 + sxy * (unsigned)ke, epf);
    load3(g, eh_in && n2, en0 + sxy * (unsigned)ke, xepf);
    load3h(g, own && n1, n0 + sxy * (unsigned)kh, hpf);
    load3h(g, hh_in && n1, hn0 + sxy * (unsigned)kh, xhpf);
    const int cpf = (own && n1) ? (int)ldg(cls, n0 + sxy * (unsigned)kh) : 0;
    const int xcpf = (hh_in && n1) ? (int)ldg(cls, hn0 + sxy * (unsigned)kh) : 0;
    const int dcls2 = (DB && PF == 1 && own && k + 2 < k1) ? (int)ldg(cls, n0 + sxy * (unsigned)(k + 2)) : 0;
    __syncthreads();
    // (c) H(k): own column, then the low-side halo point
    T hown[3] = {T(0), T(0), T(0)};
    if (own) {
      h_point<T, PML, AX>(g, i, j, k, coef(cls_cur), ecur[0], ecur[1], ecur[2], se[s][0][ty + 2][tx + 1], enext[0],
                      se[s][1][ty + 1][tx + 2], enext[1], se[s][2][ty + 1][tx + 2], se[s][2][ty + 2][tx + 1],
                      hold, true, hown);
      const unsigned n = n0 + sxy * (unsigned)k;
      stg(g.fo[3], n, hown[0]);
      stg(g.fo[4], n, hown[1]);
      stg(g.fo[5], n, hown[2]);
    }
    sh[0][ty + 1][tx + 1] = hown[0];
    sh[1][ty + 1][tx + 1] = hown[1];
    sh[2][ty + 1][tx + 1] = hown[2];
    if (hh) {
      T hx3[3] = {T(0), T(0), T(0)};
      if (hh_in) {
        h_point<T, PML, AX>(g, hx_x, hx_y, k, coef(xcls_cur), se[s][0][hr][hc], se[s][1][hr][hc], se[s][2][hr][hc],
                        se[s][0][hr + 1][hc], se[s1][0][hr][hc], se[s][1][hr][hc + 1], se[s1][1][hr][hc],
                        se[s][2][hr][hc + 1], se[s][2][hr + 1][hc], xh_old, false, hx3);
      }
      sh[0][hr][hc] = hx3[0];
      sh[1][hr][hc] = hx3[1];
      sh[2][hr][hc] = hx3[2];
    }
    __syncthreads();
    // (d) E(k) at the own column
    if (own) {
      const unsigned n = n0 + sxy * (unsigned)k;
      T e[3];
      e_point<T, PML, AX>(g, i, j, k, n, coef(cls_cur), hown[0], hown[1], hown[2], sh[0][ty][tx + 1], hm[0],
                      sh[1][ty + 1][tx], hm[1], sh[2][ty + 1][tx], sh[2][ty][tx + 1], ecur, step, e,
                      srcr.first(k), srcr.last(k));
      if (DB && dcur) {
        if (DLDS) debye_apply<T, true>(*dv, sdt + cls_cur * D_STRIDE, n, ecur, e, jcur);
        else debye_apply<T, false>(*dv, dv->dtab + cls_cur * D_STRIDE, n, ecur, e, jcur);
      }
      stg(g.fo[0], n, e[0]);
      stg(g.fo[1], n, e[1]);
      stg(g.fo[2], n, e[2]);
    }
    // rotate the pipeline
    hm[0] = hown[0];
    hm[1] = hown[1];
    for (int c = 0; c < 3; ++c) {
      ecur[c] = enext[c];
      if (PF == 2) {
        enext[c] = e2[c];
        e2[c] = epf[c];
        xe_next[c] = xe2[c];
        xe2[c] = xepf[c];
        hold[c] = h2[c];
        h2[c] = hpf[c];
        xh_old[c] = xh2[c];
        xh2[c] = xhpf[c];
      } else {
        enext[c] = epf[c];
        xe_next[c] = xepf[c];
        hold[c] = hpf[c];
        xh_old[c] = xhpf[c];
      }
    }
    if (PF == 2) {
      cls_cur = c2;
      c2 = cpf;
      xcls_cur = xc2;
      xc2 = xcpf;
    } else {
      cls_cur = cpf;
      xcls_cur = xcpf;
    }
    if (DB) {  // J^n of the next plane (PF 2: its class came a plane ago)
      dcur = own && k + 1 < k1 && dflag(PF == 2 ? cls_cur : dcls1);
      if (dcur) debye_load(*dv, n0 + sxy * (unsigned)(k + 1), jcur);
      dcls1 = dcls2;
    }
  }
}

}  // namespace mi355fdtd
