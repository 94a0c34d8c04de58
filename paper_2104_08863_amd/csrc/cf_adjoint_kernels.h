// Transposes for the adjoint of the projection step (Euclidean gradients).
//
// Momentum RHS.  R(u) = -N(u) + nu lap(u) + fx e_x with the flux-form
// N(u) = [Dx(uc^2) + Dy(Exy) + Dz(Exz), Dx(Exy) + Dyc(vc^2) + Dz(Eyz),
//         Dx(Exz) + Dy(Eyz) + Dz(wc^2)] built from
//   uc = (u_i + u_{i-1})/2,  vc = (v_j + v_{j-1})/2,  wc = (w_k + w_{k-1})/2,
//   Exy = Iy(u) Ax(v),  Exz = Az(u) Ax(w),  Eyz = Iy(w) Az(v),
//   Iy(q)_j = q_j wl_j + q_{j+1} wu_j (face j+1),  Ax(q)_i = (q_i + q_{i+1})/2,
//   Az(q)_k = (q_k + q_{k+1})/2.
// Its Jacobian transpose applied to an adjoint field lam is gathered at every
// velocity point: each edge product E contributes mu * dE/du, where mu is the
// transpose of the two differences that consume E (for Exy: Dy^T lam_u +
// Dx^T lam_v), and each centre square c^2 contributes 2 c (D^T lam).  The
// Laplacian is self-adjoint in the face-volume inner product, so its transpose
// is the same flux stencil applied to lam / W with the outer 1/W dropped
// (W = dy_j for u, w and dyc_j for v).  v on the top wall is not a variable.
//
// Projection.  P = I - G L^+ D is self-adjoint in the face-volume inner
// product, so P^T g = g - W G L^+ D (g / W): the forward solve applied to
// g / W (k_divergence-style source with row weights, SrcDivW) and a weighted
// correction (k_correct_w).
#pragma once

#include "cf_common.h"
#include "cf_step_kernels.h"

namespace cf {

template <typename T>
struct AdjGeo {
  Geo<T> g;
  const T* dy;    // dy_j
  const T* dyc;   // dyc_{j+1/2}
  const T* rdyc;  // 1/dyc
};

// J_R(u)^T lam at point (i, j, k) from an accessor with relative offsets:
// A.U(dj, dk, di) etc. for the state and A.LU(...) for lam; A returns 0 outside
// [0, ny) and for v / lam_v on the top wall.
template <typename T>
struct AdjOut {
  T gu, gv, gw;
};

// Lower-face terms of plane j that equal upper-face terms of plane j-1: the
// x-y and y-z edge factors mu * A(v) at face j (before the wl/wu weight) and
// the centre term vc * xi_y at centre j.
template <typename T>
struct AdjCarry {
  T exy, eyz, cy;
};

template <typename T, class Acc>
__device__ __forceinline__ AdjOut<T> rhs_adjoint_point(const Acc& A, const AdjGeo<T>& G, const YTab<T>& Y, int j,
                                                       T nu, bool have, AdjCarry<T> below, AdjCarry<T>& above) {
  const Geo<T>& g = G.g;
  const int ny = g.ny;
  const T h = T(0.5);
  const T rdx = g.rdx, rdz = g.rdz;
  const bool top = (j == ny - 1), bot = (j == 0);
  const T ry0 = Y.rdy(j);
  const T ryp = top ? T(0) : Y.rdy(j + 1);
  const T rym = bot ? T(0) : Y.rdy(j - 1);
  AdjOut<T> o;
  // ---------------- u point (i+1/2, j, k)
  {
    const T uc0 = h * (A.U(0, 0, 0) + A.U(0, 0, -1));
    const T uc1 = h * (A.U(0, 0, 1) + A.U(0, 0, 0));
    const T xi0 = (A.LU(0, 0, -1) - A.LU(0, 0, 0)) * rdx;
    const T xi1 = (A.LU(0, 0, 0) - A.LU(0, 0, 1)) * rdx;
    T acc = uc0 * xi0 + uc1 * xi1;
    above.exy = T(0);
    if (!top) {
      const T mu = A.LU(0, 0, 0) * ry0 - A.LU(1, 0, 0) * ryp + (A.LV(0, 0, 0) - A.LV(0, 0, 1)) * rdx;
      above.exy = mu * (h * (A.V(0, 0, 0) + A.V(0, 0, 1)));
      acc += above.exy * Y.wl(j);
    }
    if (!bot) {
      T e;
      if (have) {
        e = below.exy;
      } else {
        const T mu = A.LU(-1, 0, 0) * rym - A.LU(0, 0, 0) * ry0 + (A.LV(-1, 0, 0) - A.LV(-1, 0, 1)) * rdx;
        e = mu * (h * (A.V(-1, 0, 0) + A.V(-1, 0, 1)));
      }
      acc += e * Y.wu(j - 1);
    }
    {
      const T mk0 = (A.LU(0, 0, 0) - A.LU(0, 1, 0)) * rdz + (A.LW(0, 0, 0) - A.LW(0, 0, 1)) * rdx;
      const T mk1 = (A.LU(0, -1, 0) - A.LU(0, 0, 0)) * rdz + (A.LW(0, -1, 0) - A.LW(0, -1, 1)) * rdx;
      acc += h * (mk0 * (h * (A.W(0, 0, 0) + A.W(0, 0, 1))) + mk1 * (h * (A.W(0, -1, 0) + A.W(0, -1, 1))));
    }
    const T l0 = A.LU(0, 0, 0);
    T lap = (A.LU(0, 0, 1) - T(2) * l0 + A.LU(0, 0, -1)) * g.rdx2 + (A.LU(0, 1, 0) - T(2) * l0 + A.LU(0, -1, 0)) * g.rdz2;
    const T q0 = l0 * ry0;
    const T ft = top ? -T(2) * q0 * Y.rdy_top : (A.LU(1, 0, 0) * ryp - q0) * Y.rdyc(j);
    const T fb = bot ? T(2) * q0 * Y.rdy_bot : (q0 - A.LU(-1, 0, 0) * rym) * Y.rdyc(j - 1);
    lap += ft - fb;
    o.gu = -acc + nu * lap;
  }
  // ---------------- w point (i, j, k+1/2)
  {
    const T wc0 = h * (A.W(0, 0, 0) + A.W(0, -1, 0));
    const T wc1 = h * (A.W(0, 1, 0) + A.W(0, 0, 0));
    const T xi0 = (A.LW(0, -1, 0) - A.LW(0, 0, 0)) * rdz;
    const T xi1 = (A.LW(0, 0, 0) - A.LW(0, 1, 0)) * rdz;
    T acc = wc0 * xi0 + wc1 * xi1;
    {
      const T m0 = (A.LU(0, 0, 0) - A.LU(0, 1, 0)) * rdz + (A.LW(0, 0, 0) - A.LW(0, 0, 1)) * rdx;
      const T m1 = (A.LU(0, 0, -1) - A.LU(0, 1, -1)) * rdz + (A.LW(0, 0, -1) - A.LW(0, 0, 0)) * rdx;
      acc += h * (m0 * (h * (A.U(0, 0, 0) + A.U(0, 1, 0))) + m1 * (h * (A.U(0, 0, -1) + A.U(0, 1, -1))));
    }
    above.eyz = T(0);
    if (!top) {
      const T mu = (A.LV(0, 0, 0) - A.LV(0, 1, 0)) * rdz + A.LW(0, 0, 0) * ry0 - A.LW(1, 0, 0) * ryp;
      above.eyz = mu * (h * (A.V(0, 0, 0) + A.V(0, 1, 0)));
      acc += above.eyz * Y.wl(j);
    }
    if (!bot) {
      T e;
      if (have) {
        e = below.eyz;
      } else {
        const T mu = (A.LV(-1, 0, 0) - A.LV(-1, 1, 0)) * rdz + A.LW(-1, 0, 0) * rym - A.LW(0, 0, 0) * ry0;
        e = mu * (h * (A.V(-1, 0, 0) + A.V(-1, 1, 0)));
      }
      acc += e * Y.wu(j - 1);
    }
    const T l0 = A.LW(0, 0, 0);
    T lap = (A.LW(0, 0, 1) - T(2) * l0 + A.LW(0, 0, -1)) * g.rdx2 + (A.LW(0, 1, 0) - T(2) * l0 + A.LW(0, -1, 0)) * g.rdz2;
    const T q0 = l0 * ry0;
    const T ft = top ? -T(2) * q0 * Y.rdy_top : (A.LW(1, 0, 0) * ryp - q0) * Y.rdyc(j);
    const T fb = bot ? T(2) * q0 * Y.rdy_bot : (q0 - A.LW(-1, 0, 0) * rym) * Y.rdyc(j - 1);
    lap += ft - fb;
    o.gw = -acc + nu * lap;
  }
  // ---------------- v point (i, face j+1, k), interior faces only
  o.gv = T(0);
  above.cy = T(0);
  if (!top) {
    const T rc0 = Y.rdyc(j);
    const T rcm = bot ? T(0) : Y.rdyc(j - 1);
    const T rcp = (j + 1 < ny - 1) ? Y.rdyc(j + 1) : T(0);
    T c0;
    if (have) {
      c0 = below.cy;
    } else {
      const T vc0 = h * (A.V(0, 0, 0) + A.V(-1, 0, 0));
      c0 = vc0 * (A.LV(-1, 0, 0) * rcm - A.LV(0, 0, 0) * rc0);
    }
    const T vc1 = h * (A.V(1, 0, 0) + A.V(0, 0, 0));
    above.cy = vc1 * (A.LV(0, 0, 0) * rc0 - A.LV(1, 0, 0) * rcp);
    T acc = c0 + above.cy;
    const T a = Y.wl(j), b = Y.wu(j);
    {
      const T m0 = A.LU(0, 0, 0) * ry0 - A.LU(1, 0, 0) * ryp + (A.LV(0, 0, 0) - A.LV(0, 0, 1)) * rdx;
      const T m1 = A.LU(0, 0, -1) * ry0 - A.LU(1, 0, -1) * ryp + (A.LV(0, 0, -1) - A.LV(0, 0, 0)) * rdx;
      acc += h * (m0 * (A.U(0, 0, 0) * a + A.U(1, 0, 0) * b) + m1 * (A.U(0, 0, -1) * a + A.U(1, 0, -1) * b));
    }
    {
      const T m0 = (A.LV(0, 0, 0) - A.LV(0, 1, 0)) * rdz + A.LW(0, 0, 0) * ry0 - A.LW(1, 0, 0) * ryp;
      const T m1 = (A.LV(0, -1, 0) - A.LV(0, 0, 0)) * rdz + A.LW(0, -1, 0) * ry0 - A.LW(1, -1, 0) * ryp;
      acc += h * (m0 * (A.W(0, 0, 0) * a + A.W(1, 0, 0) * b) + m1 * (A.W(0, -1, 0) * a + A.W(1, -1, 0) * b));
    }
    const T l0 = A.LV(0, 0, 0);
    T lap = (A.LV(0, 0, 1) - T(2) * l0 + A.LV(0, 0, -1)) * g.rdx2 + (A.LV(0, 1, 0) - T(2) * l0 + A.LV(0, -1, 0)) * g.rdz2;
    const T q0 = l0 * rc0;
    const T qp = A.LV(1, 0, 0) * rcp;
    const T qm = A.LV(-1, 0, 0) * rcm;
    lap += (qp - q0) * ryp - (q0 - qm) * ry0;
    o.gv = -acc + nu * lap;
  }
  return o;
}

// LDS accessor: six fields (u, v, w, lam_u, lam_v, lam_w), three plane slots each.
template <typename T, int TX, int TZ>
struct AdjLdsAcc {
  const T* s;      // 6 fields x 3 slots x PLANE
  int sm, s0, sp;  // slot offsets (in elements) of planes j-1, j, j+1 within a field
  int base;
  static constexpr int SX = TX + 2, PLANE = (TX + 2) * (TZ + 2);
  __device__ __forceinline__ int off(int f, int dj, int dk, int di) const {
    return f * 3 * PLANE + (dj < 0 ? sm : (dj > 0 ? sp : s0)) + base + dk * SX + di;
  }
  __device__ __forceinline__ T U(int dj, int dk, int di) const { return s[off(0, dj, dk, di)]; }
  __device__ __forceinline__ T V(int dj, int dk, int di) const { return s[off(1, dj, dk, di)]; }
  __device__ __forceinline__ T W(int dj, int dk, int di) const { return s[off(2, dj, dk, di)]; }
  __device__ __forceinline__ T LU(int dj, int dk, int di) const { return s[off(3, dj, dk, di)]; }
  __device__ __forceinline__ T LV(int dj, int dk, int di) const { return s[off(4, dj, dk, di)]; }
  __device__ __forceinline__ T LW(int dj, int dk, int di) const { return s[off(5, dj, dk, di)]; }
};

struct AdjPtrs {
  const void *u, *v, *w, *au, *av, *aw, *bu, *bv, *bw;
  void *gu, *gv, *gw;
};

// out = s * J_R(state)^T lam (+ A + B when ADD), lam = c1 A (+ c2 B when HASB).
// 2.5D tiling as in k_rk_stage: a TX x TZ column tile marches over CY planes
// keeping three planes of the six fields in LDS, the raw values of plane j+2
// fetched into registers while plane j is computed.  lam is formed only when a
// plane moves from registers to LDS, and every global load is unconditional
// (clamped address, masked on the move), so the compiler's waits never cover
// a load still in flight for a later plane.  Each thread fetches its own cell
// first (a wave reads aligned x runs), so the A + B term of the ADD output is
// taken from that fetch (two planes kept in registers) instead of a second
// load.  Each XCD takes a contiguous run of every y-chunk's tiles
// (xcd_slab_block; one run over the whole grid is as fast in FP32 and 12 %
// slower in FP64): the two launches of one adjoint step take 70.8 ms instead
// of 82.8 on 2048x768x2048 in FP32, 5.7 instead of 6.5 on 1024x256x512 in FP64.
// NT: outputs, written once, stored non-temporally for large fields (the
// two launches of an FP32 adjoint step on 2048x768x2048: 72-74 -> 71.5 ms).
template <typename T, int TX, int TZ, int CY, bool HASB, bool ADD, bool NT>
__global__ void __launch_bounds__(TX * TZ)
k_rhs_adjoint(AdjPtrs P, T c1, T c2, AdjGeo<T> G, T nu, T s) {
  constexpr int SX = TX + 2, SZ = TZ + 2, PLANE = SX * SZ, TH = TX * TZ;
  constexpr int NHALO = PLANE - TH;                // 2 SX + 2 TZ ring cells
  constexpr int PER = 1 + (NHALO + TH - 1) / TH;  // own cell first, then ring cells
  constexpr int NF = HASB ? 9 : 6;  // raw fields fetched per tile value
  __shared__ T sm[6 * 3 * PLANE];
  __shared__ T sy[4 * (CY + 2)];
  const T* src[9] = {static_cast<const T*>(P.u),  static_cast<const T*>(P.v),  static_cast<const T*>(P.w),
                     static_cast<const T*>(P.au), static_cast<const T*>(P.av), static_cast<const T*>(P.aw),
                     static_cast<const T*>(P.bu), static_cast<const T*>(P.bv), static_cast<const T*>(P.bw)};
  const Geo<T>& g = G.g;
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
  // tile cells of this thread: q = 0 its own cell (tz+1, tx+1), q >= 1 the
  // ring cells (top row, bottom row, left column, right column)
  int toff[PER], cidx[PER];
  bool tin[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    int zz, xx;
    if (q == 0) {
      zz = tz + 1;
      xx = tx + 1;
      tin[q] = true;
    } else {
      const int h = threadIdx.x + (q - 1) * TH;
      tin[q] = h < NHALO;
      if (h < SX) {
        zz = 0, xx = h;
      } else if (h < 2 * SX) {
        zz = SZ - 1, xx = h - SX;
      } else if (h < 2 * SX + TZ) {
        zz = 1 + h - 2 * SX, xx = 0;
      } else {
        zz = 1 + (h - 2 * SX - TZ) % TZ, xx = SX - 1;
      }
    }
    int gi = (i0 + xx - 1) % nx;
    if (gi < 0) gi += nx;
    int gk = (k0 + zz - 1) % nz;
    if (gk < 0) gk += nz;
    toff[q] = tin[q] ? gk * nx + gi : 0;
    cidx[q] = zz * SX + xx;
  }
  T r[NF][PER];
#define CF_ADJ_FETCH(jj)                                                        \
  {                                                                            \
    const long b_ = (long)min(max((jj), 0), ny - 1) * plane;                   \
    _Pragma("unroll") for (int q = 0; q < PER; ++q) {                          \
      _Pragma("unroll") for (int f = 0; f < NF; ++f) r[f][q] = src[f][b_ + toff[q]]; \
    }                                                                          \
  }
#define CF_ADJ_STORE(jj)                                                        \
  {                                                                            \
    const int sl_ = (((jj) % 3) + 3) % 3;                                      \
    const bool pin_ = (jj) >= 0 && (jj) < ny, vin_ = (jj) >= 0 && (jj) < ny - 1; \
    _Pragma("unroll") for (int q = 0; q < PER; ++q) {                          \
      if (tin[q]) {                                                            \
        const int idx = sl_ * PLANE + cidx[q];                                 \
        _Pragma("unroll") for (int f = 0; f < 3; ++f) {                        \
          const bool in_ = (f == 1) ? vin_ : pin_;                             \
          const T lam_ = HASB ? c1 * r[3 + f][q] + c2 * r[(6 + f) % NF][q] : c1 * r[3 + f][q]; \
          sm[f * 3 * PLANE + idx] = in_ ? r[f][q] : T(0);                      \
          sm[(3 + f) * 3 * PLANE + idx] = in_ ? lam_ : T(0);                   \
        }                                                                      \
      }                                                                        \
    }                                                                          \
    if (ADD) {                                                                 \
      _Pragma("unroll") for (int f = 0; f < 3; ++f) {                          \
        const T ps_ = HASB ? r[3 + f][0] + r[(6 + f) % NF][0] : r[3 + f][0];   \
        if ((jj) & 1) ps1[f] = ps_; else ps0[f] = ps_;                         \
      }                                                                        \
    }                                                                          \
  }
  const long pid = (long)k * nx + i;
  // A (+ B) at the own cell of planes with even / odd index, kept from the
  // move of the plane into LDS for the ADD output
  T ps0[3] = {T(0), T(0), T(0)}, ps1[3] = {T(0), T(0), T(0)};
  CF_ADJ_FETCH(j0 - 1)
  CF_ADJ_STORE(j0 - 1)
  CF_ADJ_FETCH(j0)
  CF_ADJ_STORE(j0)
  CF_ADJ_FETCH(j0 + 1)
  AdjLdsAcc<T, TX, TZ> A{sm, 0, 0, 0, (tz + 1) * SX + tx + 1};
  T* gu = static_cast<T*>(P.gu);
  T* gv = static_cast<T*>(P.gv);
  T* gw = static_cast<T*>(P.gw);
  const YTab<T> Y = ytab_fill(sy, CY + 2, j0 - 1, g);
  AdjCarry<T> carry{T(0), T(0), T(0)};
  bool have = false;
  for (int j = j0; j < j1; ++j) {
    CF_ADJ_STORE(j + 1)
    __syncthreads();
    CF_ADJ_FETCH(j + 2)
    A.sm = ((j + 2) % 3) * PLANE;
    A.s0 = (j % 3) * PLANE;
    A.sp = ((j + 1) % 3) * PLANE;
    AdjCarry<T> up;
    const AdjOut<T> o = rhs_adjoint_point<T>(A, G, Y, j, nu, have, carry, up);
    carry = up;
    have = true;
    T ou = s * o.gu, ov = s * o.gv, ow = s * o.gw;
    if (ADD) {
      ou += (j & 1) ? ps1[0] : ps0[0];
      ov += (j & 1) ? ps1[1] : ps0[1];
      ow += (j & 1) ? ps1[2] : ps0[2];
    }
    if (mine) {
      const long id = (long)j * plane + pid;
      st_once<NT>(ou, &gu[id]);
      st_once<NT>((j == ny - 1) ? T(0) : ov, &gv[id]);
      st_once<NT>(ow, &gw[id]);
    }
    __syncthreads();
  }
#undef CF_ADJ_FETCH
#undef CF_ADJ_STORE
}

// g* = g - W G phi (weighted correction of the projection transpose);
// W = dy_j for u and w, dyc_j for v (so the v part is g - (phi_{j+1} - phi_j)).
template <typename T, bool NT>
__global__ void __launch_bounds__(256)
k_correct_w(const T* __restrict__ gu, const T* __restrict__ gv, const T* __restrict__ gw, T* ou, T* ov, T* ow,
            const double* __restrict__ phi, AdjGeo<T> G) {
  const Geo<T>& g = G.g;
  const long n = (long)g.nx * g.ny * g.nz;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int i = int(id % g.nx);
  const long jk = id / g.nx;
  const int k = int(jk % g.nz);
  const int j = int(jk / g.nz);
  const int ip = (i + 1 == g.nx) ? 0 : i + 1;
  const int kp = (k + 1 == g.nz) ? 0 : k + 1;
  const double p0 = phi[id];
  const T dyj = G.dy[j];
  // g and g* are touched once (streamed when NT, as in the forward correction)
  st_once<NT>(ld_once<NT>(&gu[id]) - dyj * (T(phi[jk * g.nx + ip] - p0) * g.rdx), &ou[id]);
  st_once<NT>(ld_once<NT>(&gw[id]) - dyj * (T(phi[((long)j * g.nz + kp) * g.nx + i] - p0) * g.rdz), &ow[id]);
  st_once<NT>((j == g.ny - 1) ? T(0) : ld_once<NT>(&gv[id]) - T(phi[id + (long)g.nz * g.nx] - p0), &ov[id]);
}

}  // namespace cf
