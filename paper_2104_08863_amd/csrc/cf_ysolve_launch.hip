// Launch of the wall-normal line solves.
#include "cf_internal.h"
#include "cf_ysolve_kernels.h"

namespace cf {

// Rows per partition compiled for both precisions, and the longer partitions
// compiled for FP32 only (in FP64 their rows no longer fit the registers).
#define CF_FOR_EACH_M(X) X(1) X(2) X(3) X(4) X(6) X(8) X(12) X(16)
#define CF_FOR_EACH_M_FP32(X) X(24) X(32)

bool ysolve_m_compiled(int m, bool fp64) {
  switch (m) {
#define CF_CASE(M) case M:
    CF_FOR_EACH_M(CF_CASE)
    return true;
    CF_FOR_EACH_M_FP32(CF_CASE)
    return !fp64;
#undef CF_CASE
    default:
      return false;
  }
}

// Default lines per block: about 256 threads per block with 8 to 16 lines (to
// 32 for the FP32-only partitions of more than 16 rows), and at least one
// wave.  Those FP32 partitions take at least 16 lines, so that each row of a
// block is a 128-byte run of consecutive lines, up to 512 threads.  Measured
// on MI355X for the default partitionings of the workload grids this is the
// fastest block or within 2 % of it (P = 32 partitions of 24 rows on
// 2048x768x2048: 7.0 ms per launch at 16 lines against 7.4 at 8); other shapes
// can be chosen by measurement.
int ysolve_default_lb(int P, int M) {
  const int hi = M > 16 ? 32 : 16;
  int lb = 256 / P;
  if (M > 16 && lb < 16) lb = 16 * P <= 512 ? 16 : 512 / P;
  lb = lb < 8 ? 8 : (lb > hi ? hi : lb);
  if (lb * P < 64) lb = (64 + P - 1) / P;
  return lb;
}

template <typename T, int M, int MODE, bool DROP>
static hipError_t ysolve_go(long blocks, const int* blist, const YArgs& ya, int threads, const cx<T>* fin,
                            cx<T>* pout, const T* a, const T* c, const T* kx2, const T* kz2, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  const int nyp = ya.P * M;  // rows of the partitions (padded past ny)
  const size_t lds = MODE == kSlabLocal ? sizeof(T) * 2 * (size_t)nyp : ysolve_lds_bytes<T>(nyp, ya.P, ya.LB, DROP);
  if constexpr (MODE == kWhole) {
    // the slab passes read their right-hand side twice: only the one-pass
    // solve streams it
    if ((long)ya.nlines * ya.ny * (long)sizeof(cx<T>) >= kStreamBytes) {
      hipLaunchKernelGGL((k_ysolve<T, M, MODE, DROP, true>), dim3(blocks), dim3(threads), lds, s, fin, pout, a, c,
                         kx2, kz2, blist, ya);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_ysolve<T, M, MODE, DROP, false>), dim3(blocks), dim3(threads), lds, s, fin, pout, a, c, kx2,
                     kz2, blist, ya);
  return hipGetLastError();
}

template <typename T, int M>
static hipError_t ysolve_m(const YLaunch& y, const YArgs& ya, int threads, const cx<T>* fin, cx<T>* pout, const T* a,
                           const T* c, const T* kx2, const T* kz2, hipStream_t s) {
  const long all = (y.nlines + ya.LB - 1) / ya.LB;
  if (y.mode == kSlabLocal) return ysolve_go<T, M, kSlabLocal, false>(all, nullptr, ya, threads, fin, pout, a, c,
                                                                      kx2, kz2, s);
  // blocks whose lines all allow the drop take the dropped reduced system, the
  // others the exact one (two launches over the plan's block lists; without
  // lists every block is exact)
  const long ne = y.blocks_exact ? y.n_exact : all;
  hipError_t e;
  if (y.mode == kSlabFinish) {
    e = ysolve_go<T, M, kSlabFinish, false>(ne, y.blocks_exact, ya, threads, fin, pout, a, c, kx2, kz2, s);
    if (e == hipSuccess && y.blocks_drop)
      e = ysolve_go<T, M, kSlabFinish, true>(y.n_drop, y.blocks_drop, ya, threads, fin, pout, a, c, kx2, kz2, s);
  } else {
    e = ysolve_go<T, M, kWhole, false>(ne, y.blocks_exact, ya, threads, fin, pout, a, c, kx2, kz2, s);
    if (e == hipSuccess && y.blocks_drop)
      e = ysolve_go<T, M, kWhole, true>(y.n_drop, y.blocks_drop, ya, threads, fin, pout, a, c, kx2, kz2, s);
  }
  return e;
}

template <typename T>
hipError_t launch_ysolve(const YLaunch& y, const cx<T>* fin, cx<T>* pout, const T* a, const T* c,
                         const T* kx2, const T* kz2, hipStream_t s) {
  YArgs ya;
  ya.ny = y.ny;
  ya.nz = y.nz;
  ya.nkx = y.nkx;
  ya.P = y.P;
  ya.LB = y.LB > 0 ? y.LB : ysolve_default_lb(y.P, y.M);
  ya.nlines = y.nlines;
  ya.skip_kx = y.skip_kx;
  ya.skip_kz = y.skip_kz;
  ya.pa = y.mode == kWhole ? 0 : y.pa;
  ya.pb = y.mode == kWhole ? y.P : y.pb;
  ya.iface = y.iface;
  ya.G = y.G > 0 ? y.G : y.P;
  if (y.mode != kWhole && (ya.pa < 0 || ya.pb > y.P || ya.pa >= ya.pb || y.iface == nullptr))
    return hipErrorInvalidValue;
  if (y.P % ya.G != 0) return hipErrorInvalidValue;
  // A local-mode block holds the threads of its slab's partitions only and no
  // interface data, so it takes more lines (about 256 threads) and only the
  // coefficient rows in LDS.
  if (y.mode == kSlabLocal) {
    const int np = ya.pb - ya.pa;
    while (2 * ya.LB * np <= 256) ya.LB *= 2;
  }
  const int threads = ya.LB * (y.mode == kSlabLocal ? ya.pb - ya.pa : y.P);
  switch (y.M) {
#define CF_CASE(M) \
  case M:          \
    return ysolve_m<T, M>(y, ya, threads, fin, pout, a, c, kx2, kz2, s);
    CF_FOR_EACH_M(CF_CASE)
#undef CF_CASE
    default:
      break;
  }
  if constexpr (std::is_same<T, float>::value) {
    switch (y.M) {
#define CF_CASE(M) \
  case M:          \
    return ysolve_m<T, M>(y, ya, threads, fin, pout, a, c, kx2, kz2, s);
      CF_FOR_EACH_M_FP32(CF_CASE)
#undef CF_CASE
      default:
        break;
    }
  }
  return hipErrorInvalidValue;
}

// Dynamic LDS needed by a y-solve launch over P partitions of nyp / P rows
// (checked by the plan against the device limit).
size_t ysolve_lds_needed(int nyp, int P, int LB, bool fp64) {
  return fp64 ? ysolve_lds_bytes<double>(nyp, P, LB, true) : ysolve_lds_bytes<float>(nyp, P, LB, true);
}

template <typename T>
hipError_t launch_special_lines(const cx<T>* fin, cx<T>* pout, const double* a, const double* den,
                                const double* cp, const double* dy, const int* lines, int n_lines,
                                int ny, int nz, const double* psum, int nzb, int* numflag, hipStream_t s) {
  if (n_lines <= 0) return hipSuccess;
  const int th = 256;
  const size_t lds = sizeof(double) * (5 * (size_t)ny + 3 * th);
  hipLaunchKernelGGL((k_special_lines<T>), dim3(n_lines), dim3(th), lds, s, fin, pout, a, den, cp, dy, lines,
                     ny, nz, psum, nzb, numflag);
  return hipGetLastError();
}

#define CF_INST(T)                                                                                  \
  template hipError_t launch_ysolve<T>(const YLaunch&, const cx<T>*, cx<T>*, const T*, const T*,   \
                                       const T*, const T*, hipStream_t);                           \
  template hipError_t launch_special_lines<T>(const cx<T>*, cx<T>*, const double*, const double*, \
                                              const double*, const double*, const int*, int, int, int, \
                                              const double*, int, int*, hipStream_t);
CF_INST(double)
CF_INST(float)
#undef CF_INST

}  // namespace cf
