// Launch of the adjoint (transpose) kernels of the projection step.
#include "cf_adjoint_kernels.h"
#include "cf_internal.h"

namespace cf {

// Tile of the transposed stencil (six LDS fields x three planes) and chunks of
// 32 planes.  FP64: 32 x 8 columns (51 KB of LDS, three blocks per CU; 64 x 8
// and 32 x 16 were slower, 32-plane chunks 2 % faster than 64 and 16).  FP32:
// 64 x 8 columns, 36 % faster than 32 x 8 and ahead of 64 x 16, 128 x 4,
// 128 x 8 and 32 x 16 on 512x384x512 (half the LDS per value lets the wider
// tile keep its occupancy while cutting the halo share).
template <typename T>
struct AdjTile {
  static constexpr int TX = 32, TZ = 8;
};
template <>
struct AdjTile<float> {
  static constexpr int TX = 64, TZ = 8;
};
constexpr int ADJ_CY = 32;

template <typename T>
hipError_t launch_rhs_adjoint(const T* u, const T* v, const T* w, const T* au, const T* av, const T* aw,
                              const T* bu, const T* bv, const T* bw, T c1, T c2, const AdjGeo<T>& g, T nu, T s,
                              int add, T* gu, T* gv, T* gw, hipStream_t st) {
  constexpr int ADJ_TX = AdjTile<T>::TX, ADJ_TZ = AdjTile<T>::TZ;
  AdjPtrs P{u, v, w, au, av, aw, bu, bv, bw, gu, gv, gw};
  const long blocks = (long)((g.g.nx + ADJ_TX - 1) / ADJ_TX) * ((g.g.nz + ADJ_TZ - 1) / ADJ_TZ) *
                      ((g.g.ny + ADJ_CY - 1) / ADJ_CY);
  const dim3 grid(blocks), block(ADJ_TX * ADJ_TZ);
  const bool nt = (long)g.g.nx * g.g.ny * g.g.nz * (long)sizeof(T) >= kStreamBytes;
#define CF_ADJ_GO(HASB, ADD)                                                                                     \
  if (nt)                                                                                                        \
    hipLaunchKernelGGL((k_rhs_adjoint<T, ADJ_TX, ADJ_TZ, ADJ_CY, HASB, ADD, true>), grid, block, 0, st, P, c1, c2, \
                       g, nu, s);                                                                                \
  else                                                                                                           \
    hipLaunchKernelGGL((k_rhs_adjoint<T, ADJ_TX, ADJ_TZ, ADJ_CY, HASB, ADD, false>), grid, block, 0, st, P, c1,   \
                       c2, g, nu, s)
  if (bu != nullptr && add) {
    CF_ADJ_GO(true, true);
  } else if (bu != nullptr) {
    CF_ADJ_GO(true, false);
  } else if (add) {
    CF_ADJ_GO(false, true);
  } else {
    CF_ADJ_GO(false, false);
  }
#undef CF_ADJ_GO
  return hipGetLastError();
}

template <typename T>
hipError_t launch_correct_w(const T* gu, const T* gv, const T* gw, T* ou, T* ov, T* ow, const double* phi,
                            const AdjGeo<T>& g, hipStream_t st) {
  const long n = (long)g.g.nx * g.g.ny * g.g.nz;
  const int th = 256;
  const long blocks = (n + th - 1) / th;
  if (n * (long)sizeof(T) >= kStreamBytes)
    hipLaunchKernelGGL((k_correct_w<T, true>), dim3(blocks), dim3(th), 0, st, gu, gv, gw, ou, ov, ow, phi, g);
  else
    hipLaunchKernelGGL((k_correct_w<T, false>), dim3(blocks), dim3(th), 0, st, gu, gv, gw, ou, ov, ow, phi, g);
  return hipGetLastError();
}

#define CF_INST(T)                                                                                         \
  template hipError_t launch_rhs_adjoint<T>(const T*, const T*, const T*, const T*, const T*, const T*,    \
                                            const T*, const T*, const T*, T, T, const AdjGeo<T>&, T, T, int, \
                                            T*, T*, T*, hipStream_t);                                      \
  template hipError_t launch_correct_w<T>(const T*, const T*, const T*, T*, T*, T*, const double*,         \
                                          const AdjGeo<T>&, hipStream_t);
CF_INST(double)
CF_INST(float)
#undef CF_INST

}  // namespace cf
