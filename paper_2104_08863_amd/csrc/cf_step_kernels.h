// Momentum right-hand side, RK2 stages and pressure-gradient correction of the
// projection step (Section 2, Eq. (3)-(6) and Eq. (4)).
//
//   R(u) = -N(u) + nu lap(u) + fx e_x,  N(u) = div(u u) in flux form on the
//   staggered grid (linear interpolation; y-interpolation to a face weighted by
//   the two cell heights), lap with the no-slip ghost mirrored about the wall
//   (wall distance half a cell), v = 0 on both walls.
//   stage 1: ub = u + dt R(u)
//   stage 2: us = (u + ub)/2 + dt/2 R(ub)   (= u + dt/2 [R(u) + R(ub)])
//   correction: u1 = us - dt G p
//
// One thread per grid point evaluates all three components at its (i, j, k);
// neighbour values come through the caches.  Fields are (ny, nz, nx), x
// fastest; v[ny-1] is the top wall (read as 0, written as 0).
#pragma once

#include "cf_common.h"

namespace cf {

template <typename T>
struct Geo {
  const T* rdy;   // 1/dy_j, ny
  const T* rdyc;  // 1/dyc_{j+1/2}, ny-1
  const T* wl;    // dy_{j+1}/(dy_j+dy_{j+1}), ny-1: weight of the lower cell
  const T* wu;    // dy_j/(dy_j+dy_{j+1}), ny-1: weight of the upper cell
  T rdx, rdz, rdx2, rdz2;
  int nx, ny, nz;
};

template <typename T>
struct RhsOut {
  T ru, rv, rw;
};

template <typename T>
__device__ __forceinline__ RhsOut<T> momentum_rhs(const T* __restrict__ u, const T* __restrict__ v,
                                                  const T* __restrict__ w, const Geo<T>& g, int i,
                                                  int j, int k, T nu, T fx) {
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ip = (i + 1 == nx) ? 0 : i + 1, im = (i == 0) ? nx - 1 : i - 1;
  const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
  const long pl = (long)nz * nx;
  const long r0 = ((long)j * nz + k) * nx;         // row (j, k)
  const long rkp = ((long)j * nz + kp) * nx;       // row (j, k+1)
  const long rkm = ((long)j * nz + km) * nx;       // row (j, k-1)
  const bool top = (j == ny - 1), bot = (j == 0);
  const T h = T(0.5);
  // ---- values
  const T u0 = u[r0 + i], uip = u[r0 + ip], uim = u[r0 + im];
  const T ukp = u[rkp + i], ukm = u[rkm + i], ukpm = u[rkp + im];
  const T w0 = w[r0 + i], wip = w[r0 + ip], wim = w[r0 + im];
  const T wkp = w[rkp + i], wkm = w[rkm + i], wkmp = w[rkm + ip];
  const T v0 = top ? T(0) : v[r0 + i];
  const T vip = top ? T(0) : v[r0 + ip], vim = top ? T(0) : v[r0 + im];
  const T vkp = top ? T(0) : v[rkp + i], vkm = top ? T(0) : v[rkm + i];
  T uj1 = T(0), uj1m = T(0), wj1 = T(0), wj1m = T(0), vj1 = T(0);
  if (!top) {
    uj1 = u[r0 + pl + i];
    uj1m = u[r0 + pl + im];
    wj1 = w[r0 + pl + i];
    wj1m = w[rkm + pl + i];
    vj1 = (j + 1 == ny - 1) ? T(0) : v[r0 + pl + i];
  }
  T ujm = T(0), wjm = T(0), vjm = T(0), vjmip = T(0), vjmkp = T(0);
  if (!bot) {
    ujm = u[r0 - pl + i];
    wjm = w[r0 - pl + i];
    vjm = v[r0 - pl + i];
    vjmip = v[r0 - pl + ip];
    vjmkp = v[rkp - pl + i];
  }
  const T rdy = g.rdy[j];
  // ---- edge products (flux form)
  // x-y edges at face j+1 (u interpolated in y, v in x), at i and i-1
  T exy_i = T(0), exy_im = T(0), eyz_k = T(0), eyz_km = T(0);
  if (!top) {
    const T a = g.wl[j], b = g.wu[j];
    exy_i = (u0 * a + uj1 * b) * (h * (v0 + vip));
    exy_im = (uim * a + uj1m * b) * (h * (vim + v0));
    eyz_k = (w0 * a + wj1 * b) * (h * (v0 + vkp));
    eyz_km = (wkm * a + wj1m * b) * (h * (vkm + v0));
  }
  T exy_b = T(0), eyz_b = T(0);  // face j (bottom of cell j) at (k, i)
  if (!bot) {
    const T a = g.wl[j - 1], b = g.wu[j - 1];
    exy_b = (ujm * a + u0 * b) * (h * (vjm + vjmip));
    eyz_b = (wjm * a + w0 * b) * (h * (vjm + vjmkp));
  }
  // x-z edges at (i+1/2, k+1/2) and neighbours
  const T exz = (h * (u0 + ukp)) * (h * (w0 + wip));
  const T exz_km = (h * (ukm + u0)) * (h * (wkm + wkmp));
  const T exz_im = (h * (uim + ukpm)) * (h * (wim + w0));
  // ---- x-momentum
  const T ucp = h * (uip + u0), ucm = h * (u0 + uim);
  T nxu = (ucp * ucp - ucm * ucm) * g.rdx + (exy_i - exy_b) * rdy + (exz - exz_km) * g.rdz;
  T lu = (uip - T(2) * u0 + uim) * g.rdx2 + (ukp - T(2) * u0 + ukm) * g.rdz2;
  {
    const T ft = top ? -T(2) * u0 * g.rdy[ny - 1] : (uj1 - u0) * g.rdyc[j];
    const T fb = bot ? T(2) * u0 * g.rdy[0] : (u0 - ujm) * g.rdyc[j - 1];
    lu += (ft - fb) * rdy;
  }
  // ---- z-momentum
  const T cwp = h * (wkp + w0), cwm = h * (w0 + wkm);
  T nzw = (exz - exz_im) * g.rdx + (eyz_k - eyz_b) * rdy + (cwp * cwp - cwm * cwm) * g.rdz;
  T lw = (wip - T(2) * w0 + wim) * g.rdx2 + (wkp - T(2) * w0 + wkm) * g.rdz2;
  {
    const T ft = top ? -T(2) * w0 * g.rdy[ny - 1] : (wj1 - w0) * g.rdyc[j];
    const T fb = bot ? T(2) * w0 * g.rdy[0] : (w0 - wjm) * g.rdyc[j - 1];
    lw += (ft - fb) * rdy;
  }
  // ---- y-momentum (interior faces only)
  T rv = T(0);
  if (!top) {
    const T ct = h * (vj1 + v0), cb = h * (v0 + vjm);
    const T nyv = (exy_i - exy_im) * g.rdx + (ct * ct - cb * cb) * g.rdyc[j] + (eyz_k - eyz_km) * g.rdz;
    T lv = (vip - T(2) * v0 + vim) * g.rdx2 + (vkp - T(2) * v0 + vkm) * g.rdz2;
    lv += ((vj1 - v0) * g.rdy[j + 1] - (v0 - vjm) * rdy) * g.rdyc[j];
    rv = -nyv + nu * lv;
  }
  RhsOut<T> o;
  o.ru = -nxu + nu * lu + fx;
  o.rv = rv;
  o.rw = -nzw + nu * lw;
  return o;
}

// STAGE 1: out = f + dt R(f).  STAGE 2: out = (f0 + f)/2 + dt/2 R(f).
template <typename T, int STAGE>
__global__ void __launch_bounds__(256)
k_rk_stage(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
           const T* u0, const T* v0, const T* w0, T* uo, T* vo, T* wo, Geo<T> g, T dt, T nu, T fx) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int i = int(id % g.nx);
  const long jk = id / g.nx;
  const int k = int(jk % g.nz);
  const int j = int(jk / g.nz);
  const RhsOut<T> r = momentum_rhs<T>(u, v, w, g, i, j, k, nu, fx);
  const bool top = (j == g.ny - 1);
  if (STAGE == 1) {
    uo[id] = u[id] + dt * r.ru;
    vo[id] = top ? T(0) : v[id] + dt * r.rv;
    wo[id] = w[id] + dt * r.rw;
  } else {
    const T h = T(0.5), hd = T(0.5) * dt;
    const T a = u0[id], b = top ? T(0) : v0[id], c = w0[id];
    uo[id] = h * (a + u[id]) + hd * r.ru;
    vo[id] = top ? T(0) : h * (b + v[id]) + hd * r.rv;
    wo[id] = h * (c + w[id]) + hd * r.rw;
  }
}

// u1 = us - dt G p (in place on the velocity arrays); the top-wall v plane is 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_correct(T* u, T* v, T* w, const double* __restrict__ p, Geo<T> g, T dt) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int i = int(id % g.nx);
  const long jk = id / g.nx;
  const int k = int(jk % g.nz);
  const int j = int(jk / g.nz);
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const long row = jk * g.nx;
  const double p0 = p[id];
  const T gx = T(p[row + ip] - p0) * g.rdx;
  const T gz = T(p[((long)j * g.nz + kp) * g.nx + i] - p0) * g.rdz;
  u[id] = u[id] - dt * gx;
  w[id] = w[id] - dt * gz;
  if (j == g.ny - 1) {
    v[id] = T(0);
  } else {
    const T gy = T(p[id + (long)g.nz * g.nx] - p0) * g.rdyc[j];
    v[id] = v[id] - dt * gy;
  }
}

}  // namespace cf
