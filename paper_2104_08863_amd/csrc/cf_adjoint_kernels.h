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

// Global-memory accessor with periodic x, z and the wall rules; lam is formed
// as c1 * A + c2 * B on the fly.
template <typename T>
struct AdjAcc {
  const T *u, *v, *w;
  const T *au, *av, *aw, *bu, *bv, *bw;
  T c1, c2;
  int nx, ny, nz;
  __device__ __forceinline__ long at(int j, int k, int i) const {
    k = (k < 0) ? k + nz : (k >= nz ? k - nz : k);
    i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
    return ((long)j * nz + k) * nx + i;
  }
  __device__ __forceinline__ bool yin(int j) const { return j >= 0 && j < ny; }
  __device__ __forceinline__ bool vin(int j) const { return j >= 0 && j < ny - 1; }
  __device__ __forceinline__ T U(int j, int k, int i) const { return yin(j) ? u[at(j, k, i)] : T(0); }
  __device__ __forceinline__ T V(int j, int k, int i) const { return vin(j) ? v[at(j, k, i)] : T(0); }
  __device__ __forceinline__ T W(int j, int k, int i) const { return yin(j) ? w[at(j, k, i)] : T(0); }
  __device__ __forceinline__ T lam(const T* a, const T* b, long o) const {
    return b ? c1 * a[o] + c2 * b[o] : c1 * a[o];
  }
  __device__ __forceinline__ T LU(int j, int k, int i) const { return yin(j) ? lam(au, bu, at(j, k, i)) : T(0); }
  __device__ __forceinline__ T LV(int j, int k, int i) const { return vin(j) ? lam(av, bv, at(j, k, i)) : T(0); }
  __device__ __forceinline__ T LW(int j, int k, int i) const { return yin(j) ? lam(aw, bw, at(j, k, i)) : T(0); }
};

// out = s * J_R(u)^T lam (+ A + B when add), lam = c1 A + c2 B.
template <typename T>
__global__ void __launch_bounds__(256)
k_rhs_adjoint(AdjAcc<T> X, AdjGeo<T> G, T nu, T s, int add, T* __restrict__ gu, T* __restrict__ gv,
              T* __restrict__ gw) {
  const Geo<T>& g = G.g;
  const long n = (long)g.nx * g.ny * g.nz;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const int i = int(id % g.nx);
  const long jk = id / g.nx;
  const int k = int(jk % g.nz);
  const int j = int(jk / g.nz);
  const int ny = g.ny;
  const T h = T(0.5);
  const T rdx = g.rdx, rdz = g.rdz;
  const bool top = (j == ny - 1), bot = (j == 0);
  auto rdyv = [&](int jj) { return (jj >= 0 && jj < ny) ? g.rdy[jj] : T(0); };

  // ---------------- u point (i+1/2, j, k)
  T nu_u;
  {
    // (1) centre squares along x
    const T uc0 = h * (X.U(j, k, i) + X.U(j, k, i - 1));
    const T uc1 = h * (X.U(j, k, i + 1) + X.U(j, k, i));
    const T xi0 = (X.LU(j, k, i - 1) - X.LU(j, k, i)) * rdx;
    const T xi1 = (X.LU(j, k, i) - X.LU(j, k, i + 1)) * rdx;
    T acc = uc0 * xi0 + uc1 * xi1;
    // (2) x-y edges at faces j+1 (weight wl_j) and j (weight wu_{j-1})
    if (!top) {
      const T mu = X.LU(j, k, i) * g.rdy[j] - X.LU(j + 1, k, i) * g.rdy[j + 1] +
                   (X.LV(j, k, i) - X.LV(j, k, i + 1)) * rdx;
      acc += mu * (h * (X.V(j, k, i) + X.V(j, k, i + 1))) * g.wl[j];
    }
    if (!bot) {
      const T mu = X.LU(j - 1, k, i) * g.rdy[j - 1] - X.LU(j, k, i) * g.rdy[j] +
                   (X.LV(j - 1, k, i) - X.LV(j - 1, k, i + 1)) * rdx;
      acc += mu * (h * (X.V(j - 1, k, i) + X.V(j - 1, k, i + 1))) * g.wu[j - 1];
    }
    // (3) x-z edges at k+1/2 and k-1/2
    {
      const T mk0 = (X.LU(j, k, i) - X.LU(j, k + 1, i)) * rdz + (X.LW(j, k, i) - X.LW(j, k, i + 1)) * rdx;
      const T mk1 = (X.LU(j, k - 1, i) - X.LU(j, k, i)) * rdz + (X.LW(j, k - 1, i) - X.LW(j, k - 1, i + 1)) * rdx;
      acc += h * (mk0 * (h * (X.W(j, k, i) + X.W(j, k, i + 1))) + mk1 * (h * (X.W(j, k - 1, i) + X.W(j, k - 1, i + 1))));
    }
    // Laplacian transpose
    const T l0 = X.LU(j, k, i);
    T lap = (X.LU(j, k, i + 1) - T(2) * l0 + X.LU(j, k, i - 1)) * g.rdx2 +
            (X.LU(j, k + 1, i) - T(2) * l0 + X.LU(j, k - 1, i)) * g.rdz2;
    const T q0 = l0 * g.rdy[j];
    const T ft = top ? -T(2) * q0 * g.rdy[ny - 1] : (X.LU(j + 1, k, i) * rdyv(j + 1) - q0) * g.rdyc[j];
    const T fb = bot ? T(2) * q0 * g.rdy[0] : (q0 - X.LU(j - 1, k, i) * rdyv(j - 1)) * g.rdyc[j - 1];
    lap += ft - fb;
    nu_u = -acc + nu * lap;
  }
  // ---------------- w point (i, j, k+1/2)
  T nu_w;
  {
    // (6) centre squares along z
    const T wc0 = h * (X.W(j, k, i) + X.W(j, k - 1, i));
    const T wc1 = h * (X.W(j, k + 1, i) + X.W(j, k, i));
    const T xi0 = (X.LW(j, k - 1, i) - X.LW(j, k, i)) * rdz;
    const T xi1 = (X.LW(j, k, i) - X.LW(j, k + 1, i)) * rdz;
    T acc = wc0 * xi0 + wc1 * xi1;
    // (3) x-z edges at i+1/2 and i-1/2
    {
      const T m0 = (X.LU(j, k, i) - X.LU(j, k + 1, i)) * rdz + (X.LW(j, k, i) - X.LW(j, k, i + 1)) * rdx;
      const T m1 = (X.LU(j, k, i - 1) - X.LU(j, k + 1, i - 1)) * rdz + (X.LW(j, k, i - 1) - X.LW(j, k, i)) * rdx;
      acc += h * (m0 * (h * (X.U(j, k, i) + X.U(j, k + 1, i))) + m1 * (h * (X.U(j, k, i - 1) + X.U(j, k + 1, i - 1))));
    }
    // (4) y-z edges at faces j+1 and j
    if (!top) {
      const T mu = (X.LV(j, k, i) - X.LV(j, k + 1, i)) * rdz + X.LW(j, k, i) * g.rdy[j] -
                   X.LW(j + 1, k, i) * g.rdy[j + 1];
      acc += mu * (h * (X.V(j, k, i) + X.V(j, k + 1, i))) * g.wl[j];
    }
    if (!bot) {
      const T mu = (X.LV(j - 1, k, i) - X.LV(j - 1, k + 1, i)) * rdz + X.LW(j - 1, k, i) * g.rdy[j - 1] -
                   X.LW(j, k, i) * g.rdy[j];
      acc += mu * (h * (X.V(j - 1, k, i) + X.V(j - 1, k + 1, i))) * g.wu[j - 1];
    }
    const T l0 = X.LW(j, k, i);
    T lap = (X.LW(j, k, i + 1) - T(2) * l0 + X.LW(j, k, i - 1)) * g.rdx2 +
            (X.LW(j, k + 1, i) - T(2) * l0 + X.LW(j, k - 1, i)) * g.rdz2;
    const T q0 = l0 * g.rdy[j];
    const T ft = top ? -T(2) * q0 * g.rdy[ny - 1] : (X.LW(j + 1, k, i) * rdyv(j + 1) - q0) * g.rdyc[j];
    const T fb = bot ? T(2) * q0 * g.rdy[0] : (q0 - X.LW(j - 1, k, i) * rdyv(j - 1)) * g.rdyc[j - 1];
    lap += ft - fb;
    nu_w = -acc + nu * lap;
  }
  // ---------------- v point (i, face j+1, k), interior faces only
  T nu_v = T(0);
  if (!top) {
    // (5) centre squares along y: centres j and j+1
    const T vc0 = h * (X.V(j, k, i) + X.V(j - 1, k, i));
    const T vc1 = h * (X.V(j + 1, k, i) + X.V(j, k, i));
    const T xi0 = (bot ? T(0) : X.LV(j - 1, k, i) * G.rdyc[j - 1]) - X.LV(j, k, i) * G.rdyc[j];
    const T xi1 = X.LV(j, k, i) * G.rdyc[j] - ((j + 1 < ny - 1) ? X.LV(j + 1, k, i) * G.rdyc[j + 1] : T(0));
    T acc = vc0 * xi0 + vc1 * xi1;
    // (2) x-y edges at i+1/2 and i-1/2 (face j+1)
    {
      const T a = g.wl[j], b = g.wu[j];
      const T m0 = X.LU(j, k, i) * g.rdy[j] - X.LU(j + 1, k, i) * g.rdy[j + 1] + (X.LV(j, k, i) - X.LV(j, k, i + 1)) * rdx;
      const T m1 = X.LU(j, k, i - 1) * g.rdy[j] - X.LU(j + 1, k, i - 1) * g.rdy[j + 1] +
                   (X.LV(j, k, i - 1) - X.LV(j, k, i)) * rdx;
      acc += h * (m0 * (X.U(j, k, i) * a + X.U(j + 1, k, i) * b) + m1 * (X.U(j, k, i - 1) * a + X.U(j + 1, k, i - 1) * b));
    }
    // (4) y-z edges at k+1/2 and k-1/2 (face j+1)
    {
      const T a = g.wl[j], b = g.wu[j];
      const T m0 = (X.LV(j, k, i) - X.LV(j, k + 1, i)) * rdz + X.LW(j, k, i) * g.rdy[j] - X.LW(j + 1, k, i) * g.rdy[j + 1];
      const T m1 = (X.LV(j, k - 1, i) - X.LV(j, k, i)) * rdz + X.LW(j, k - 1, i) * g.rdy[j] -
                   X.LW(j + 1, k - 1, i) * g.rdy[j + 1];
      acc += h * (m0 * (X.W(j, k, i) * a + X.W(j + 1, k, i) * b) + m1 * (X.W(j, k - 1, i) * a + X.W(j + 1, k - 1, i) * b));
    }
    const T l0 = X.LV(j, k, i);
    T lap = (X.LV(j, k, i + 1) - T(2) * l0 + X.LV(j, k, i - 1)) * g.rdx2 +
            (X.LV(j, k + 1, i) - T(2) * l0 + X.LV(j, k - 1, i)) * g.rdz2;
    const T q0 = l0 * G.rdyc[j];
    const T qp = (j + 1 < ny - 1) ? X.LV(j + 1, k, i) * G.rdyc[j + 1] : T(0);
    const T qm = bot ? T(0) : X.LV(j - 1, k, i) * G.rdyc[j - 1];
    lap += (qp - q0) * g.rdy[j + 1] - (q0 - qm) * g.rdy[j];
    nu_v = -acc + nu * lap;
  }
  T ou = s * nu_u, ov = s * nu_v, ow = s * nu_w;
  if (add) {
    ou += X.au[id] + (X.bu ? X.bu[id] : T(0));
    ow += X.aw[id] + (X.bw ? X.bw[id] : T(0));
    ov += top ? T(0) : X.av[id] + (X.bv ? X.bv[id] : T(0));
  }
  gu[id] = ou;
  gv[id] = top ? T(0) : ov;
  gw[id] = ow;
}

// g* = g - W G phi (weighted correction of the projection transpose);
// W = dy_j for u and w, dyc_j for v (so the v part is g - (phi_{j+1} - phi_j)).
template <typename T>
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
  ou[id] = gu[id] - dyj * (T(phi[jk * g.nx + ip] - p0) * g.rdx);
  ow[id] = gw[id] - dyj * (T(phi[((long)j * g.nz + kp) * g.nx + i] - p0) * g.rdz);
  ov[id] = (j == g.ny - 1) ? T(0) : gv[id] - T(phi[id + (long)g.nz * g.nx] - p0);
}

}  // namespace cf
