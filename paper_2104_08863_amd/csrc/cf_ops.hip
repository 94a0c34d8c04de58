// Pointwise staggered-grid operators that are not fused into a transform.
#include "cf_internal.h"

namespace cf {

// f = scale * [(u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy_j + (w_k - w_{k-1})/dz]
// with v = 0 on both walls (the stored top-wall plane is not read).
__global__ void k_divergence(const double* __restrict__ u, const double* __restrict__ v,
                             const double* __restrict__ w, double* __restrict__ f,
                             const double* __restrict__ rdy, double rdx, double rdz, double scale,
                             int nx, int ny, int nz) {
  const long n = (long)nx * ny * nz;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int i = int(id % nx);
  const long jk = id / nx;
  const int k = int(jk % nz);
  const int j = int(jk / nz);
  const long plane = (long)nx * nz;
  const int im = (i == 0) ? nx - 1 : i - 1;
  const int km = (k == 0) ? nz - 1 : k - 1;
  const double vj = (j == ny - 1) ? 0.0 : v[id];
  const double vjm = (j == 0) ? 0.0 : v[id - plane];
  const double du = (u[id] - u[id - i + im]) * rdx;
  const double dv = (vj - vjm) * rdy[j];
  const double dw = (w[id] - w[id + (long)(km - k) * nx]) * rdz;
  f[id] = (du + dv + dw) * scale;
}

hipError_t launch_divergence(const double* u, const double* v, const double* w, double* f,
                             const double* rdy, double rdx, double rdz, double scale, int nx, int ny,
                             int nz, hipStream_t s) {
  const long n = (long)nx * ny * nz;
  const int th = 256;
  const long blocks = (n + th - 1) / th;
  hipLaunchKernelGGL(k_divergence, dim3(blocks), dim3(th), 0, s, u, v, w, f, rdy, rdx, rdz, scale, nx, ny, nz);
  return hipGetLastError();
}

}  // namespace cf
