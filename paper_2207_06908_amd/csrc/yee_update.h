// yee_update.h -- per-element arithmetic of the Yee update, shared by every
// kernel variant so that all variants produce bit-identical fields.
//
// Section 2.1 of the paper: the H update of eq. 5 and the E update of eq. 4
// (semi-implicit or literal loss factor folded into ca / cb), the other
// components by cyclic permutation; Section 2.2: inside the CPML each
// derivative term d of axis u becomes d / kappa_u + psi with
// psi <- b_u psi + c_u d (recursive convolution).  Differences are raw (not
// divided by dx): 1/dx is folded into cb and db, and psi is stored times dx.
#pragma once
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"

namespace mi355fdtd {

// One CPML-stretched derivative term.  `prof` is the axis table, `l` the
// slab-local position, `row` P_BE (E position) or P_BH (H position).  The
// table holds b - 1, so the recursion psi <- b psi + c d is evaluated as
// psi + ((b - 1) psi + c d), which keeps FP32 accurate where b is near 1.
template <typename T>
__device__ __forceinline__ T pml_step(T d, T& psi, T bm1, T c, T ik) {
  psi = psi + fma(bm1, psi, c * d);
  return fma(d, ik, psi);
}
template <typename T>
__device__ __forceinline__ T pml_term(T d, T& psi, const T* prof, int l, int two_np, int row) {
  return pml_step(d, psi, prof[(row + 0) * two_np + l], prof[(row + 1) * two_np + l], prof[(row + 2) * two_np + l]);
}

// Slab-local position of node index `pos` along an axis of n cells, or -1.
__device__ __forceinline__ int slab_pos(int pos, int n, int np) {
  if (pos < np) return pos;
  if (pos >= n - np) return pos - n + 2 * np;
  return -1;
}

// Index of node (i, j, k) inside the psi slab of axis u at local position l
// (every array the kernels touch is below 4 GiB; the host checks).
__device__ __forceinline__ unsigned psi_index(int u, int l, int i, int j, int k, int nx, int ny, int np) {
  const unsigned t = 2u * np;
  if (u == 0) return (unsigned)l + t * ((unsigned)j + (unsigned)ny * (unsigned)k);
  if (u == 1) return (unsigned)i + (unsigned)nx * ((unsigned)l + t * (unsigned)k);
  return (unsigned)i + (unsigned)nx * ((unsigned)j + (unsigned)ny * (unsigned)l);
}

// Element access through a uniform base pointer and a 32-bit byte offset, so
// that loads and stores use the scalar-base + vector-offset address form.
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned idx) {
  // every array read this way lives in global memory; saying so keeps the
  // access a global (not generic) one where the pointer itself was read from
  // memory, e.g. a batched grid's view
  typedef __attribute__((address_space(1))) const T GT;
  return *(GT*)((const __attribute__((address_space(1))) char*)base + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T* base, unsigned idx, T v) {
  typedef __attribute__((address_space(1))) T GT;
  *(GT*)((__attribute__((address_space(1))) char*)base + idx * (unsigned)sizeof(T)) = v;
}

// H update of one node from raw E differences.
//   Hx += db_x ((Ey[k+1] - Ey) - (Ez[j+1] - Ez))
//   Hy += db_y ((Ez[i+1] - Ez) - (Ex[k+1] - Ex))
//   Hz += db_z ((Ex[j+1] - Ex) - (Ey[i+1] - Ey))
template <typename T>
__device__ __forceinline__ T h_new(T h, T db, T t_plus, T t_minus) {
  return fma(db, t_plus - t_minus, h);
}

// E update of one node from raw H differences, with cam1 = ca - 1:
//   Ex = Ex + ((ca_x - 1) Ex + cb_x ((Hz - Hz[j-1]) - (Hy - Hy[k-1])))
//   Ey = Ey + ((ca_y - 1) Ey + cb_y ((Hx - Hx[k-1]) - (Hz - Hz[i-1])))
//   Ez = Ez + ((ca_z - 1) Ez + cb_z ((Hy - Hy[i-1]) - (Hx - Hx[j-1])))
// i.e. ca E + cb curl, written so that a loss factor close to 1 keeps its
// full precision in FP32.
template <typename T>
__device__ __forceinline__ T e_new(T e, T cam1, T cb, T t_plus, T t_minus) {
  return e + fma(cam1, e, cb * (t_plus - t_minus));
}

}  // namespace mi355fdtd
