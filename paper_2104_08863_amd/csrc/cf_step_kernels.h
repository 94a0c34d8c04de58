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
// The RK stages march in y over LDS-resident planes (2.5D tiling, see
// k_rk_stage); the correction is pointwise.  Fields are (ny, nz, nx), x
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

// The wall-normal metric rows a y-chunk touches (jb .. jb + n - 1 of 1/dy,
// 1/dyc, wl and wu, zero where a table has no entry), staged in LDS once per
// block, plus 1/dy of the two wall cells held in registers.  The marching
// stencils read them from here so that no per-plane global load shares the
// in-order vector-memory counter with the next plane's prefetch: a wait for
// such a load would also wait for the prefetch and serialise the pipeline.
template <typename T>
struct YTab {
  const T* s;  // 4 x n values in LDS
  int n, jb;
  T rdy_bot, rdy_top;
  __device__ __forceinline__ T rdy(int j) const { return s[j - jb]; }
  __device__ __forceinline__ T rdyc(int j) const { return s[n + j - jb]; }
  __device__ __forceinline__ T wl(int j) const { return s[2 * n + j - jb]; }
  __device__ __forceinline__ T wu(int j) const { return s[3 * n + j - jb]; }
};

// Block-cooperative fill of a YTab over rows jb .. jb + n - 1; the caller
// synchronises before the first read.
template <typename T>
__device__ __forceinline__ YTab<T> ytab_fill(T* s, int n, int jb, const Geo<T>& g) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int jj = jb + t;
    const bool in = jj >= 0 && jj < g.ny - 1;
    s[t] = (jj >= 0 && jj < g.ny) ? g.rdy[jj] : T(0);
    s[n + t] = in ? g.rdyc[jj] : T(0);
    s[2 * n + t] = in ? g.wl[jj] : T(0);
    s[3 * n + t] = in ? g.wu[jj] : T(0);
  }
  return YTab<T>{s, n, jb, g.rdy[0], g.rdy[g.ny - 1]};
}

template <typename T>
struct RhsOut {
  T ru, rv, rw;
};

// R at point (i, j, k) from an accessor A with A.u(dj, dk, di) etc. returning
// the neighbour values (dj, dk, di in {-1, 0, 1}); A returns 0 for v on the
// top wall and for planes outside [0, ny).
template <typename T>
struct FaceFlux {
  T exy, eyz;  // x-y and y-z edge products at the upper face of the cell
};

// `below`: the edge products at the lower face (j) when have_below (they are
// the upper-face products of plane j-1); `above` receives those of face j+1.
template <typename T, class Acc>
__device__ __forceinline__ RhsOut<T> momentum_rhs(const Acc& A, const Geo<T>& g, const YTab<T>& Y, int j, T nu,
                                                  T fx, bool have_below, FaceFlux<T> below, FaceFlux<T>& above) {
  const int ny = g.ny;
  const bool top = (j == ny - 1), bot = (j == 0);
  const T h = T(0.5);
  const T u0 = A.u(0, 0, 0), uip = A.u(0, 0, 1), uim = A.u(0, 0, -1);
  const T ukp = A.u(0, 1, 0), ukm = A.u(0, -1, 0), ukpm = A.u(0, 1, -1);
  const T w0 = A.w(0, 0, 0), wip = A.w(0, 0, 1), wim = A.w(0, 0, -1);
  const T wkp = A.w(0, 1, 0), wkm = A.w(0, -1, 0), wkmp = A.w(0, -1, 1);
  const T v0 = A.v(0, 0, 0), vip = A.v(0, 0, 1), vim = A.v(0, 0, -1);
  const T vkp = A.v(0, 1, 0), vkm = A.v(0, -1, 0);
  const T uj1 = A.u(1, 0, 0), uj1m = A.u(1, 0, -1), wj1 = A.w(1, 0, 0), wj1m = A.w(1, -1, 0);
  const T vj1 = A.v(1, 0, 0);
  const T ujm = A.u(-1, 0, 0), wjm = A.w(-1, 0, 0), vjm = A.v(-1, 0, 0);
  const T rdy = Y.rdy(j);
  // x-y and y-z edge products at face j+1 (u, w interpolated in y, v in x or z)
  T exy_i = T(0), exy_im = T(0), eyz_k = T(0), eyz_km = T(0);
  if (!top) {
    const T a = Y.wl(j), b = Y.wu(j);
    exy_i = (u0 * a + uj1 * b) * (h * (v0 + vip));
    exy_im = (uim * a + uj1m * b) * (h * (vim + v0));
    eyz_k = (w0 * a + wj1 * b) * (h * (v0 + vkp));
    eyz_km = (wkm * a + wj1m * b) * (h * (vkm + v0));
  }
  T exy_b = T(0), eyz_b = T(0);  // face j (bottom of cell j)
  if (have_below) {
    exy_b = below.exy;
    eyz_b = below.eyz;
  } else if (!bot) {
    const T a = Y.wl(j - 1), b = Y.wu(j - 1);
    exy_b = (ujm * a + u0 * b) * (h * (vjm + A.v(-1, 0, 1)));
    eyz_b = (wjm * a + w0 * b) * (h * (vjm + A.v(-1, 1, 0)));
  }
  above.exy = exy_i;
  above.eyz = eyz_k;
  // x-z edge products at (i+1/2, k+1/2) and the neighbours
  const T exz = (h * (u0 + ukp)) * (h * (w0 + wip));
  const T exz_km = (h * (ukm + u0)) * (h * (wkm + wkmp));
  const T exz_im = (h * (uim + ukpm)) * (h * (wim + w0));
  // x-momentum
  const T ucp = h * (uip + u0), ucm = h * (u0 + uim);
  const T nxu = (ucp * ucp - ucm * ucm) * g.rdx + (exy_i - exy_b) * rdy + (exz - exz_km) * g.rdz;
  T lu = (uip - T(2) * u0 + uim) * g.rdx2 + (ukp - T(2) * u0 + ukm) * g.rdz2;
  {
    const T ft = top ? -T(2) * u0 * Y.rdy_top : (uj1 - u0) * Y.rdyc(j);
    const T fb = bot ? T(2) * u0 * Y.rdy_bot : (u0 - ujm) * Y.rdyc(j - 1);
    lu += (ft - fb) * rdy;
  }
  // z-momentum
  const T cwp = h * (wkp + w0), cwm = h * (w0 + wkm);
  const T nzw = (exz - exz_im) * g.rdx + (eyz_k - eyz_b) * rdy + (cwp * cwp - cwm * cwm) * g.rdz;
  T lw = (wip - T(2) * w0 + wim) * g.rdx2 + (wkp - T(2) * w0 + wkm) * g.rdz2;
  {
    const T ft = top ? -T(2) * w0 * Y.rdy_top : (wj1 - w0) * Y.rdyc(j);
    const T fb = bot ? T(2) * w0 * Y.rdy_bot : (w0 - wjm) * Y.rdyc(j - 1);
    lw += (ft - fb) * rdy;
  }
  // y-momentum (interior faces only)
  T rv = T(0);
  if (!top) {
    const T ct = h * (vj1 + v0), cb = h * (v0 + vjm);
    const T nyv = (exy_i - exy_im) * g.rdx + (ct * ct - cb * cb) * Y.rdyc(j) + (eyz_k - eyz_km) * g.rdz;
    T lv = (vip - T(2) * v0 + vim) * g.rdx2 + (vkp - T(2) * v0 + vkm) * g.rdz2;
    lv += ((vj1 - v0) * Y.rdy(j + 1) - (v0 - vjm) * rdy) * Y.rdyc(j);
    rv = -nyv + nu * lv;
  }
  RhsOut<T> o;
  o.ru = -nxu + nu * lu + fx;
  o.rv = rv;
  o.rw = -nzw + nu * lw;
  return o;
}

// 2.5D tiling: a block owns TX x TZ columns (x, z) and marches over a chunk of
// CY planes in y, keeping three consecutive planes of u, v, w (with a one-cell
// halo in x and z, periodic wrap) in LDS; every field value is read from
// global memory once per plane step plus the halo.
template <int TX, int TZ, int CY>
struct RkTile {
  static constexpr int SX = TX + 2, SZ = TZ + 2, PLANE = SX * SZ, THREADS = TX * TZ;
};

template <typename T, int TX, int TZ>
struct LdsAcc {
  const T* su;  // three plane slots of u, each PLANE values
  const T* sv;
  const T* sw;
  int sm, s0, sp;  // slot offsets of planes j-1, j, j+1
  int base;        // (tz+1)*SX + tx+1
  static constexpr int SX = TX + 2;
  __device__ __forceinline__ int off(int dj, int dk, int di) const {
    return (dj < 0 ? sm : (dj > 0 ? sp : s0)) + base + dk * SX + di;
  }
  __device__ __forceinline__ T u(int dj, int dk, int di) const { return su[off(dj, dk, di)]; }
  __device__ __forceinline__ T v(int dj, int dk, int di) const { return sv[off(dj, dk, di)]; }
  __device__ __forceinline__ T w(int dj, int dk, int di) const { return sw[off(dj, dk, di)]; }
};

// STAGE 1: out = f + dt R(f).  STAGE 2: out = (f0 + f)/2 + dt/2 R(f).
// Plane j+2 is fetched into registers while plane j is computed from LDS.
// Each XCD takes a contiguous run of every y-chunk's tiles (xcd_slab_block):
// the FP32 stage on 2048x768x2048 runs in 17.2 ms instead of 22.0.
// NT: outputs, written once, stored non-temporally for large fields (FP64
// stage 1 on 1024x256x512: 1.37-1.43 -> 1.30 ms).
template <typename T, int STAGE, int TX, int TZ, int CY, bool NT>
__global__ void __launch_bounds__(TX * TZ)
k_rk_stage(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w,
           const T* u0, const T* v0, const T* w0, T* uo, T* vo, T* wo, Geo<T> g, T dt, T nu, T fx) {
  using Tl = RkTile<TX, TZ, CY>;
  constexpr int PER = (Tl::PLANE + Tl::THREADS - 1) / Tl::THREADS;  // tile values per thread
  __shared__ T su[3 * Tl::PLANE], sv[3 * Tl::PLANE], sw[3 * Tl::PLANE];
  __shared__ T sy[4 * (CY + 2)];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ntx = (nx + TX - 1) / TX, ntz = (nz + TZ - 1) / TZ;
  int b = xcd_slab_block(blockIdx.x, ntx * ntz);
  const int bx = b % ntx;
  b /= ntx;
  const int bz = b % ntz;
  const int by = b / ntz;
  const int i0 = bx * TX, k0 = bz * TZ;
  const int j0 = by * CY, j1 = (j0 + CY < ny) ? j0 + CY : ny;
  const int tx = threadIdx.x % TX, tz = threadIdx.x / TX;
  const int i = i0 + tx, k = k0 + tz;
  const bool mine = (i < nx) && (k < nz);
  const long plane = (long)nx * nz;
  // in-plane offsets of this thread's tile values (periodic wrap); -1 = none
  int toff[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = threadIdx.x + q * Tl::THREADS;
    const int zz = idx / Tl::SX, xx = idx % Tl::SX;
    int gi = (i0 + xx - 1) % nx;
    if (gi < 0) gi += nx;
    int gk = (k0 + zz - 1) % nz;
    if (gk < 0) gk += nz;
    toff[q] = (idx < Tl::PLANE) ? gk * nx + gi : -1;
  }
  T ru[PER], rv[PER], rw[PER];
#define CF_RK_FETCH(jj)                                          \
  _Pragma("unroll") for (int q = 0; q < PER; ++q) {             \
    ru[q] = rv[q] = rw[q] = T(0);                               \
    if (toff[q] >= 0 && (jj) >= 0 && (jj) < ny) {               \
      const long o = (long)(jj) * plane + toff[q];              \
      ru[q] = u[o];                                             \
      rw[q] = w[o];                                             \
      if ((jj) < ny - 1) rv[q] = v[o];                          \
    }                                                           \
  }
#define CF_RK_STORE(s)                                           \
  _Pragma("unroll") for (int q = 0; q < PER; ++q) {             \
    if (toff[q] >= 0) {                                         \
      const int idx = threadIdx.x + q * Tl::THREADS;            \
      su[(s) * Tl::PLANE + idx] = ru[q];                        \
      sv[(s) * Tl::PLANE + idx] = rv[q];                        \
      sw[(s) * Tl::PLANE + idx] = rw[q];                        \
    }                                                           \
  }
  const long pid = (long)k * nx + i;  // this thread's in-plane offset
  CF_RK_FETCH(j0 - 1)
  CF_RK_STORE((j0 + 2) % 3)
  CF_RK_FETCH(j0)
  CF_RK_STORE(j0 % 3)
  CF_RK_FETCH(j0 + 1)
  T a0 = T(0), b0 = T(0), c0 = T(0);
  if (STAGE == 2 && mine) {
    a0 = u0[(long)j0 * plane + pid];
    b0 = (j0 < ny - 1) ? v0[(long)j0 * plane + pid] : T(0);
    c0 = w0[(long)j0 * plane + pid];
  }
  LdsAcc<T, TX, TZ> A{su, sv, sw, 0, 0, 0, (tz + 1) * Tl::SX + tx + 1};
  const YTab<T> Y = ytab_fill(sy, CY + 2, j0 - 1, g);
  FaceFlux<T> carry{T(0), T(0)};
  bool have = false;
  for (int j = j0; j < j1; ++j) {
    CF_RK_STORE((j + 1) % 3)
    __syncthreads();
    CF_RK_FETCH(j + 2)
    T a1 = T(0), b1 = T(0), c1 = T(0);
    if (STAGE == 2 && mine && j + 1 < j1) {
      a1 = u0[(long)(j + 1) * plane + pid];
      b1 = (j + 1 < ny - 1) ? v0[(long)(j + 1) * plane + pid] : T(0);
      c1 = w0[(long)(j + 1) * plane + pid];
    }
    A.sm = ((j + 2) % 3) * Tl::PLANE;
    A.s0 = (j % 3) * Tl::PLANE;
    A.sp = ((j + 1) % 3) * Tl::PLANE;
    if (mine) {
      FaceFlux<T> up;
      const RhsOut<T> r = momentum_rhs<T>(A, g, Y, j, nu, fx, have, carry, up);
      carry = up;
      have = true;
      const long id = (long)j * plane + pid;
      const bool top = (j == ny - 1);
      const T uc = A.u(0, 0, 0), vc = A.v(0, 0, 0), wc = A.w(0, 0, 0);
      if (STAGE == 1) {
        st_once<NT>(uc + dt * r.ru, &uo[id]);
        st_once<NT>(top ? T(0) : vc + dt * r.rv, &vo[id]);
        st_once<NT>(wc + dt * r.rw, &wo[id]);
      } else {
        const T hh = T(0.5), hd = T(0.5) * dt;
        st_once<NT>(hh * (a0 + uc) + hd * r.ru, &uo[id]);
        st_once<NT>(top ? T(0) : hh * (b0 + vc) + hd * r.rv, &vo[id]);
        st_once<NT>(hh * (c0 + wc) + hd * r.rw, &wo[id]);
      }
    }
    a0 = a1;
    b0 = b1;
    c0 = c1;
    __syncthreads();
  }
#undef CF_RK_FETCH
#undef CF_RK_STORE
}

// u1 = us - dt G p at point id = (j, k, i), row = (j nz + k) nx (in place; the
// top-wall v plane is 0); returns the corrected values.  Each velocity value
// is read and written once, non-temporally when NT (the FP64 correction on
// 1024x256x512 runs 5 % faster than with plain loads and stores); p, whose
// values neighbouring points share, is read through the caches.
template <bool NT, typename T>
__device__ __forceinline__ void correct_point(T* u, T* v, T* w, const double* __restrict__ p, const Geo<T>& g,
                                              T dt, long id, long row, int i, int k, int j, T& cu, T& cv, T& cw) {
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const double p0 = p[id];
  const T gx = T(p[row + ip] - p0) * g.rdx;
  const T gz = T(p[((long)j * g.nz + kp) * g.nx + i] - p0) * g.rdz;
  cu = ld_once<NT>(&u[id]) - dt * gx;
  st_once<NT>(cu, &u[id]);
  cw = ld_once<NT>(&w[id]) - dt * gz;
  st_once<NT>(cw, &w[id]);
  if (j == g.ny - 1) {
    cv = T(0);
  } else {
    const T gy = T(p[id + (long)g.nz * g.nx] - p0) * g.rdyc[j];
    cv = ld_once<NT>(&v[id]) - dt * gy;
  }
  st_once<NT>(cv, &v[id]);
}

// u1 = us - dt G p (in place on the velocity arrays); the top-wall v plane is 0.
// One thread per point; the neighbours of p come through the caches.
template <typename T, bool NT>
__global__ void __launch_bounds__(256)
k_correct(T* u, T* v, T* w, const double* __restrict__ p, Geo<T> g, T dt) {
  const long n = (long)g.nx * g.ny * g.nz;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int i = int(id % g.nx);
  const long jk = id / g.nx;
  const int k = int(jk % g.nz);
  const int j = int(jk / g.nz);
  T cu, cv, cw;
  correct_point<NT, T>(u, v, w, p, g, dt, id, jk * g.nx, i, k, j, cu, cv, cw);
}

// Block reduction of six FP64 per-thread sums in a fixed order (wave shuffles,
// then the waves in order); thread f < 6 returns sum f.
template <int TH>
__device__ __forceinline__ double block_sum6(const double (&sm)[6], double (&red)[6][TH / 64]) {
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    double x = sm[f];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d, 64);
    if ((threadIdx.x & 63) == 0) red[f][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  double x = 0.0;
  if (threadIdx.x < 6)
    for (int k = 0; k < TH / 64; ++k) x += red[threadIdx.x][k];
  return x;
}

// The correction of k_correct (same per-point arithmetic) fused with the
// plane statistics of the corrected fields: block b corrects chunk b % nch of
// plane b / nch and writes the six FP64 sums of that chunk (u, v, w and their
// squares; fixed order: strided per-thread sums, then block_sum6) to
// part[b * 6 + f].  k_stats_gather adds the chunks of each plane in order.
template <typename T, int TH, bool NT>
__global__ void __launch_bounds__(TH)
k_correct_stats(T* __restrict__ u, T* __restrict__ v, T* __restrict__ w, const double* __restrict__ p, Geo<T> g,
                T dt, double* __restrict__ part, int nch) {
  __shared__ double red[6][TH / 64];
  const int nxz = g.nx * g.nz;
  const int j = blockIdx.x / nch, c = blockIdx.x % nch;
  const int len = (nxz + nch - 1) / nch;
  const int e0 = c * len, e1 = (e0 + len < nxz) ? e0 + len : nxz;
  const long o = (long)j * nxz;
  double sm[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int e = e0 + threadIdx.x; e < e1; e += TH) {
    const int i = e % g.nx, k = e / g.nx;
    T cu, cv, cw;
    correct_point<NT, T>(u, v, w, p, g, dt, o + e, o + e - i, i, k, j, cu, cv, cw);
    const double a = double(cu), b = double(cv), d = double(cw);
    sm[0] += a;
    sm[1] += b;
    sm[2] += d;
    sm[3] += a * a;
    sm[4] += b * b;
    sm[5] += d * d;
  }
  const double x = block_sum6<TH>(sm, red);
  if (threadIdx.x < 6) part[(long)blockIdx.x * 6 + threadIdx.x] = x;
}

// Plane statistics of a velocity field: for every y-plane j the means over the
// x-z plane of u, v, w and of their squares, summed in FP64.  One block per
// plane and a fixed reduction order (strided per-thread sums, wave shuffles,
// then the waves in order), so the result is bitwise repeatable.  st[j*6 + c]
// receives (or, with accumulate, gains) the means.
template <typename T, int TH>
__global__ void __launch_bounds__(TH)
k_plane_stats(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w, double* __restrict__ st,
              int nxz, double scale, int accumulate) {
  __shared__ double red[6][TH / 64];
  const long o = (long)blockIdx.x * nxz;
  double sm[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int e = threadIdx.x; e < nxz; e += TH) {
    const double a = double(u[o + e]), b = double(v[o + e]), c = double(w[o + e]);
    sm[0] += a;
    sm[1] += b;
    sm[2] += c;
    sm[3] += a * a;
    sm[4] += b * b;
    sm[5] += c * c;
  }
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    double x = sm[f];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_down(x, d, 64);
    if ((threadIdx.x & 63) == 0) red[f][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double x = 0.0;
    for (int k = 0; k < TH / 64; ++k) x += red[threadIdx.x][k];
    x *= scale;
    double* d = st + (long)blockIdx.x * 6 + threadIdx.x;
    *d = accumulate ? *d + x : x;
  }
}

}  // namespace cf
