// Device helpers shared by the kernel sources of the PSWF fast Ewald pipeline: vector and
// complex types, system lookup in prefix tables, packed cells, grid coordinates, the window
// support offsets and the tile walk of the particle kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace pswfe {
namespace {


template <class T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <class T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <class C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <class C> __device__ __forceinline__ C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }

// Global-address-space view of a device pointer taken from a descriptor: loads through it
// compile to global_load (the compiler cannot infer the address space of a pointer read from
// memory, and flat loads also count against the LDS wait counter).
template <class T>
using global_ptr = const __attribute__((address_space(1))) T*;
template <class T>
using global_mut_ptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ global_ptr<T> as_global(const T* p) {
  return (global_ptr<T>)p;
}
template <class T>
__device__ __forceinline__ global_mut_ptr<T> as_global_mut(T* p) {
  return (global_mut_ptr<T>)p;
}

// Loads and stores of two-element vectors (float2, double2) in global memory through the
// compiler's native vector type (the HIP vector classes cannot be accessed through a
// global-address-space pointer).
template <class V>
__device__ __forceinline__ V gload(const V* p) {
  using E = std::remove_cv_t<std::remove_reference_t<decltype(V{}.x)>>;
  typedef E N __attribute__((ext_vector_type(2)));
  const N n = *((const __attribute__((address_space(1))) N*)p);
  return V{n.x, n.y};
}
template <class V>
__device__ __forceinline__ void gstore(V* p, const V& v) {
  using E = std::remove_cv_t<std::remove_reference_t<decltype(V{}.x)>>;
  typedef E N __attribute__((ext_vector_type(2)));
  N n;
  n.x = v.x;
  n.y = v.y;
  *((__attribute__((address_space(1))) N*)p) = n;
}

// Atomic adds into device (HBM) memory; the result is not used, so the non-returning global
// form is emitted.
__device__ __forceinline__ void atomic_add_global(float* p, float v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f32((__attribute__((address_space(1))) float*)p, v);
}
__device__ __forceinline__ void atomic_add_global(double* p, double v) {
  (void)__builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double*)p, v);
}

// System owning global item i: the largest s < nsys with prefix[s] <= i (prefix is
// non-decreasing with prefix[0] = 0; an empty system repeats its successor's start and is
// skipped).
template <class I>
__device__ __forceinline__ int find_sys(const I* __restrict__ prefix, int nsys, I i) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// The same search restricted to [lo, hi] (a range known to hold i's system).
template <class I>
__device__ __forceinline__ int find_sys_in(const I* __restrict__ prefix, int lo, int hi, I i) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Cell coordinates (each < m <= 512) packed into 10-bit fields.
__device__ __forceinline__ int pack_cell(int cx, int cy, int cz) { return cx | (cy << 10) | (cz << 20); }
__device__ __forceinline__ int cell_x(int c) { return c & 1023; }
__device__ __forceinline__ int cell_y(int c) { return (c >> 10) & 1023; }
__device__ __forceinline__ int cell_z(int c) { return c >> 20; }

// Grid coordinate of x: cell c in [0, m) and fractional offset f with x/h = c + f (mod m).
// The product x * (1/h) uses 1/h split into two words (ih_hi + ih_lo) and the exact product
// error from an FMA, so f keeps the working precision's relative accuracy instead of losing
// log2(m) bits to the integer part. Non-finite inputs map to cell 0 so every index derived
// from the result stays inside the grid. Contraction is off here: fusing the rounded product
// p into (p - floor(p)) would count its rounding error twice.
template <class T>
__device__ __forceinline__ int grid_coord(T x, T ih_hi, T ih_lo, T L, int m, T& f) {
#pragma clang fp contract(off)
  T xr = x;
  if (!(xr >= T(0) && xr < L)) {
    xr = x - L * floor(x / L);
    if (!(xr >= T(0) && xr < L)) xr = T(0);
  }
  const T p = xr * ih_hi;
  const T lo = fma(xr, ih_lo, fma(xr, ih_hi, -p));
  const T fl = floor(p);
  int c = static_cast<int>(fl);
  T fr = (p - fl) + lo;
  if (fr < T(0)) {
    fr += T(1);
    c -= 1;
  } else if (fr >= T(1)) {
    fr -= T(1);
    c += 1;
  }
  if (c < 0) c += m;
  if (c >= m) c -= m;
  if (!(fr >= T(0) && fr <= T(1))) fr = T(0);
  f = fr;
  return c;
}

// ------------------------------------------------------------------------------------
// Window evaluation. For a particle at x/h = c + f (cell c, 0 <= f < 1) the support is the
// P consecutive points starting at floor(c + f - P/2) + 1 = a + 1 - ceil(P/2), with the anchor
// a = c for even P and the nearest grid point a = c + [f >= 1/2] (mod m) for odd P; point j sits
// at offset u_j = g + (P-1)/2 - j with g = f - 1/2 (even P) or f - [f >= 1/2] (odd P), g in
// [-1/2, 1/2), and its window value phi_1(2 u_j / P) is the polynomial `coef[j]` evaluated at g
// (Horner). Binning sorts particles by the tile of their anchor and stores (g, anchor), so the
// support starts at o = a - T0 from the tile's halo origin T0 + 1 - ceil(P/2), with o in
// [0, B - 1]: the halo block has edge S = B + P - 1.
// ------------------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ int support_anchor(int c, T f, int P, int m, T& g) {
  if (P % 2 == 0) {
    g = f - T(0.5);
    return c;
  }
  const int hh = f >= T(0.5) ? 1 : 0;
  g = f - static_cast<T>(hh);
  const int a = c + hh;
  return a >= m ? a - m : a;
}

// Periodic image of a grid index a in [-m, 3m) (the range of every halo index: a tile origin
// is below m, tile edge and half support are at most m).
__device__ __forceinline__ int fold_index(int a, int m) {
  a += a < 0 ? m : 0;
  a -= a >= m ? m : 0;
  a -= a >= m ? m : 0;
  return a;
}

// Walks the S^3 points of a tile's LDS block (x fastest) with a stride of one workgroup:
// load(k, lds_index, grid_index) for up to K points per thread, then use(...)
// for the same points, so K independent memory accesses are in flight before their results
// are needed. The (x, y, z) offsets advance by the stride's digits instead of being divided
// out of the flat index.
template <int K, class Load, class Use>
__device__ __forceinline__ void walk_tile(int S, int m, int my, int mz, int Ox, int Oy, int Oz, Load&& load,
                                          Use&& use) {
  const int S2 = S * S, S3 = S2 * S;
  const int nt = blockDim.x;
  const int sz = nt / S2, sy = (nt - sz * S2) / S, sx = nt - sz * S2 - sy * S;
  const int t = threadIdx.x;
  int iz = t / S2, iy = (t - iz * S2) / S, ix = t - iz * S2 - iy * S;
  for (int base = t; base < S3; base += nt * K) {
    int li[K];
    int64_t gi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      li[k] = base + nt * k;
      gi[k] = (static_cast<int64_t>(fold_index(Oz + iz, mz)) * my + fold_index(Oy + iy, my)) * m + fold_index(Ox + ix, m);
      ix += sx;
      if (ix >= S) {
        ix -= S;
        ++iy;
      }
      iy += sy;
      if (iy >= S) {
        iy -= S;
        ++iz;
      }
      iz += sz;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (li[k] < S3) load(k, li[k], gi[k]);
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (li[k] < S3) use(k, li[k], gi[k]);
  }
}

}  // namespace
}  // namespace pswfe
