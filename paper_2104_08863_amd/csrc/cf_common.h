// Shared device/host helpers for the chanflow HIP kernels: a plain complex
// type and the handful of operations the transforms and solves need.
//
// Everything here is usable from host code as well, so the per-thread math of
// the kernels can be exercised on the CPU.
#pragma once

#include <cstddef>
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define CF_HD __host__ __device__ __forceinline__
#else
#define CF_HD inline
#endif

namespace cf {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T> CF_HD cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T> CF_HD cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> CF_HD cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> CF_HD cx<T> operator*(cx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T> CF_HD cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
template <typename T> CF_HD cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename T> CF_HD cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
// multiply by -i (forward sign) or +i (inverse sign)
template <bool INV, typename T> CF_HD cx<T> mul_mi(cx<T> a) {
  return INV ? mk(-a.im, a.re) : mk(a.im, -a.re);
}

// Reciprocal: on the device the hardware estimate refined by Newton steps
// (error about one ulp, no IEEE division sequence); on the host 1/x.
CF_HD double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
CF_HD float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  float r = __builtin_amdgcn_rcpf(x);
  float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
#else
  return 1.0f / x;
#endif
}

template <typename T> CF_HD T cf_max(T a, T b) { return a > b ? a : b; }
template <typename T> CF_HD T cf_min(T a, T b) { return a < b ? a : b; }

// A load and a store of a value that a kernel touches once: non-temporal when
// NT (streamed past the caches; the launches choose it for fields larger than
// the XCDs' L2s together), plain otherwise.
#if defined(__HIPCC__)
template <bool NT, typename T>
__device__ __forceinline__ T ld_once(const T* a) {
  if constexpr (NT) return __builtin_nontemporal_load(a);
  else return *a;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_once(T v, T* a) {
  if constexpr (NT) __builtin_nontemporal_store(v, a);
  else *a = v;
}
template <bool NT, typename T>
__device__ __forceinline__ cx<T> ld_once(const cx<T>* a) {
  if constexpr (NT) {
    const T* p = reinterpret_cast<const T*>(a);
    return mk(__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + 1));
  } else {
    return *a;
  }
}
template <bool NT, typename T>
__device__ __forceinline__ void st_once(cx<T> v, cx<T>* a) {
  if constexpr (NT) {
    T* p = reinterpret_cast<T*>(a);
    __builtin_nontemporal_store(v.re, p);
    __builtin_nontemporal_store(v.im, p + 1);
  } else {
    *a = v;
  }
}
#endif
// Data size from which the kernels that touch their arrays once (the
// corrections, the z transforms, the wall-normal solve, the fused RK2 pass's
// output) take non-temporal loads and stores: the 8 XCDs' L2s together
// (32 MiB).  Smaller arrays stay cached for the next kernel (streamed, the
// 64^3 time loop was 2-4 % slower).
constexpr long kStreamBytes = 32L << 20;

// Work order for the 8 XCDs, each with its own L2.  The hardware deals
// blocks round-robin (block b to XCD b mod 8); for a grid made of groups of n
// consecutive work items (n a multiple of 8), block b is given the item that
// puts XCD x on the contiguous run [x n/8, (x+1) n/8) of every group, so items
// beside each other, which read each other's edge cells, do so from one L2.
// With n the whole grid each XCD gets one run.  A permutation of the grid
// either way (identity when n is not a multiple of 8).
CF_HD int xcd_slab_block(int b, int n) {
  if (n & 7) return b;
  const int x = b & 7, s = b >> 3, per = n >> 3;
  return (s / per) * n + x * per + s % per;
}

// Modes of the partitioned solve.  kWhole: every partition of a line in one
// block.  The two slab modes split the same computation at the point where a
// partition needs data from the others (the paper's exchange across
// processes): kSlabLocal runs the local solves of the partitions [pa, pb) and
// writes their interface rows; kSlabFinish reads every partition's interface
// rows, solves the reduced system, redoes the local solves of [pa, pb) and
// writes their corrected rows.
enum YMode { kWhole = 0, kSlabLocal = 1, kSlabFinish = 2 };

}  // namespace cf
