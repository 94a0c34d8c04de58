// Launch of the RK2 momentum stages, the pressure-gradient correction and the
// plane statistics.
#include "cf_internal.h"
#include "cf_rk_fused.h"
#include "cf_step_kernels.h"

namespace cf {

// Split-stage tile: 64 x 8 columns, chunks of 32 planes.
constexpr int RK_TX = 64, RK_TZ = 8, RK_CY = 32;

template <typename T>
hipError_t launch_rk_stage(int stage, const T* u, const T* v, const T* w, const T* u0, const T* v0,
                           const T* w0, T* uo, T* vo, T* wo, const Geo<T>& g, T dt, T nu, T fx,
                           hipStream_t s) {
  const long blocks = (long)((g.nx + RK_TX - 1) / RK_TX) * ((g.nz + RK_TZ - 1) / RK_TZ) *
                      ((g.ny + RK_CY - 1) / RK_CY);
  const dim3 th(RK_TX * RK_TZ);
  const bool nt = (long)g.nx * g.ny * g.nz * (long)sizeof(T) >= kStreamBytes;
#define CF_RK_GO(ST, NT)                                                                                         \
  hipLaunchKernelGGL((k_rk_stage<T, ST, RK_TX, RK_TZ, RK_CY, NT>), dim3(blocks), th, 0, s, u, v, w, u0, v0, w0, \
                     uo, vo, wo, g, dt, nu, fx)
  if (stage == 1) {
    if (nt) CF_RK_GO(1, true);
    else CF_RK_GO(1, false);
  } else {
    if (nt) CF_RK_GO(2, true);
    else CF_RK_GO(2, false);
  }
#undef CF_RK_GO
  return hipGetLastError();
}

// Fused RK2 tile.  FP64: 64 x 16 columns, one block of 16 waves per CU (stage 1
// on the 66 x 18 grown tile, whose 164 outer cells keep 3 of the 16 waves busy
// for one more stencil pass).  FP32: 64 x 8 columns, two blocks per CU (half
// the LDS per value; 6 % faster than 64 x 16 on a 512x384x512 mixed step,
// 64 x 4 was 15 % slower).  Chunks of 128 planes; shorter chunks (32, then 8
// planes) when that leaves fewer than two blocks per CU, as on small grids.
template <typename T>
struct RkfTile {
  static constexpr int TX = 64, TZ = 16;
};
template <>
struct RkfTile<float> {
  static constexpr int TX = 64, TZ = 8;
};

template <typename T>
hipError_t launch_rk2_fused(const T* u, const T* v, const T* w, T* uo, T* vo, T* wo, const Geo<T>& g, T dt, T nu,
                            T fx, hipStream_t s) {
  constexpr int RKF_TX = RkfTile<T>::TX, RKF_TZ = RkfTile<T>::TZ;
  const long cols = (long)((g.nx + RKF_TX - 1) / RKF_TX) * ((g.nz + RKF_TZ - 1) / RKF_TZ);
  auto blocks = [&](int cy) { return cols * ((g.ny + cy - 1) / cy); };
  const dim3 th(RKF_TX * RKF_TZ);
  const bool nt = (long)g.nx * g.ny * g.nz * (long)sizeof(T) >= kStreamBytes;
#define CF_RKF_GO(CY, NT)                                                                                          \
  hipLaunchKernelGGL((k_rk2_fused<T, RKF_TX, RKF_TZ, CY, NT>), dim3(blocks(CY)), th, 0, s, u, v, w, uo, vo, wo, g, \
                     dt, nu, fx)
  if (blocks(128) >= 512) {
    if (nt) CF_RKF_GO(128, true);
    else CF_RKF_GO(128, false);
  } else if (blocks(32) >= 512) {
    if (nt) CF_RKF_GO(32, true);
    else CF_RKF_GO(32, false);
  } else {
    if (nt) CF_RKF_GO(8, true);
    else CF_RKF_GO(8, false);
  }
#undef CF_RKF_GO
  return hipGetLastError();
}

template <typename T>
hipError_t launch_correct(T* u, T* v, T* w, const double* p, const Geo<T>& g, T dt, hipStream_t s) {
  const long n = (long)g.nx * g.ny * g.nz;
  const int th = 256;
  const long blocks = (n + th - 1) / th;
  if (n * (long)sizeof(T) >= kStreamBytes)
    hipLaunchKernelGGL((k_correct<T, true>), dim3(blocks), dim3(th), 0, s, u, v, w, p, g, dt);
  else
    hipLaunchKernelGGL((k_correct<T, false>), dim3(blocks), dim3(th), 0, s, u, v, w, p, g, dt);
  return hipGetLastError();
}

// st[j*6 + f] (+)= scale * sum over the nch chunks of plane j, in chunk order.
__global__ void __launch_bounds__(256)
k_stats_gather(const double* __restrict__ part, double* __restrict__ st, int ny, int nch, double scale,
               int accumulate) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ny * 6) return;
  const int j = t / 6, f = t % 6;
  double x = 0.0;
  for (int c = 0; c < nch; ++c) x += part[((long)j * nch + c) * 6 + f];
  x *= scale;
  st[t] = accumulate ? st[t] + x : x;
}

// Chunks per plane of the fused correction + statistics: about 32768 blocks in
// all, at least 1024 points per chunk.
int correct_stats_chunks(int nx, int ny, int nz) {
  const int nxz = nx * nz;
  int nch = (32768 + ny - 1) / ny;
  if (nch > nxz / 1024) nch = nxz / 1024;
  return nch < 1 ? 1 : nch;
}

template <typename T>
hipError_t launch_correct_stats(T* u, T* v, T* w, const double* p, const Geo<T>& g, T dt, double* part, int nch,
                                double* st, int accumulate, hipStream_t s) {
  if ((long)g.nx * g.ny * g.nz * (long)sizeof(T) >= kStreamBytes)
    hipLaunchKernelGGL((k_correct_stats<T, 256, true>), dim3((long)g.ny * nch), dim3(256), 0, s, u, v, w, p, g, dt,
                       part, nch);
  else
    hipLaunchKernelGGL((k_correct_stats<T, 256, false>), dim3((long)g.ny * nch), dim3(256), 0, s, u, v, w, p, g, dt,
                       part, nch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = g.ny * 6;
  hipLaunchKernelGGL(k_stats_gather, dim3((n + 255) / 256), dim3(256), 0, s, part, st, g.ny, nch,
                     1.0 / double(g.nx * g.nz), accumulate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plane_stats(const T* u, const T* v, const T* w, double* st, const Geo<T>& g, int accumulate,
                              hipStream_t s) {
  const int nxz = g.nx * g.nz;
  hipLaunchKernelGGL((k_plane_stats<T, 1024>), dim3(g.ny), dim3(1024), 0, s, u, v, w, st, nxz, 1.0 / double(nxz),
                     accumulate);
  return hipGetLastError();
}

#define CF_INST(T)                                                                                     \
  template hipError_t launch_rk_stage<T>(int, const T*, const T*, const T*, const T*, const T*,        \
                                         const T*, T*, T*, T*, const Geo<T>&, T, T, T, hipStream_t); \
  template hipError_t launch_rk2_fused<T>(const T*, const T*, const T*, T*, T*, T*, const Geo<T>&, T, T, T, \
                                          hipStream_t);                                                   \
  template hipError_t launch_plane_stats<T>(const T*, const T*, const T*, double*, const Geo<T>&, int, \
                                            hipStream_t);                                            \
  template hipError_t launch_correct<T>(T*, T*, T*, const double*, const Geo<T>&, T, hipStream_t);          \
  template hipError_t launch_correct_stats<T>(T*, T*, T*, const double*, const Geo<T>&, T, double*, int,    \
                                              double*, int, hipStream_t);
CF_INST(double)
CF_INST(float)
#undef CF_INST

}  // namespace cf
