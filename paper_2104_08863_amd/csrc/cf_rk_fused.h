// Both stages of the RK2 (Heun) momentum update in one marching pass.
//
// ub = u + dt R(u) and u2 = (u + ub)/2 + dt/2 R(ub) are computed plane by
// plane: while a block marches up its y-chunk, stage 1 runs one plane ahead
// of stage 2 on the tile grown by one cell in x and z (the cells stage 2's
// stencil reads), and ub lives only in LDS.  The pass reads u, v, w once and
// writes u2 once, instead of the two passes of the split stages (read u, write
// ub; read ub and u, write u2).  The stencil arithmetic is the same function as
// in the split stages.
//
// Both stages use the edge products carried up from the plane below and the
// plane-below values of the thread's own column from registers, so the input
// ring keeps two planes (j, j+1).  Stage 2 runs two planes behind stage 1 (the
// ub ring keeps three planes), so within one barrier interval the two stages
// are independent and their LDS reads and arithmetic interleave.  The first
// planes of a chunk get the carries from a short prologue over the two planes
// below it.
#pragma once

#include "cf_step_kernels.h"

namespace cf {

// x-y and y-z edge products at the upper face of plane j (face j+1): the
// expressions momentum_rhs uses for its carried products.  Zero at and above
// the top wall and below the bottom wall.
template <typename T, class Acc>
__device__ __forceinline__ FaceFlux<T> upper_face_flux(const Acc& A, const YTab<T>& Y, int j, int ny) {
  FaceFlux<T> f{T(0), T(0)};
  if (j >= 0 && j < ny - 1) {
    const T h = T(0.5);
    const T a = Y.wl(j), b = Y.wu(j);
    const T v0 = A.v(0, 0, 0);
    f.exy = (A.u(0, 0, 0) * a + A.u(1, 0, 0) * b) * (h * (v0 + A.v(0, 0, 1)));
    f.eyz = (A.w(0, 0, 0) * a + A.w(1, 0, 0) * b) * (h * (v0 + A.v(0, 1, 0)));
  }
  return f;
}

// Two-plane LDS ring (planes j and j+1, row stride SXX) with the thread's own
// column at plane j-1 held in registers.  Off-column values of plane j-1 are
// never requested: the stencil is always called with its lower-face products
// carried.
template <typename T, int SXX>
struct Ring2Acc {
  const T* su;
  const T* sv;
  const T* sw;
  int s0, sp;  // slot offsets of planes j and j+1
  int base;    // this point within a slot
  T um, vm, wm;
  __device__ __forceinline__ int off(int dj, int dk, int di) const { return (dj > 0 ? sp : s0) + base + dk * SXX + di; }
  __device__ __forceinline__ T u(int dj, int dk, int di) const { return dj < 0 ? um : su[off(dj, dk, di)]; }
  __device__ __forceinline__ T v(int dj, int dk, int di) const { return dj < 0 ? vm : sv[off(dj, dk, di)]; }
  __device__ __forceinline__ T w(int dj, int dk, int di) const { return dj < 0 ? wm : sw[off(dj, dk, di)]; }
};

// Per-column marching state of one stencil point: the values of the plane
// below and the edge products at the lower face of the current plane.
template <typename T>
struct ColState {
  T um, vm, wm;
  FaceFlux<T> c;
};

// Stage 1 at plane j for one point of the grown tile: reads u at planes j and
// j+1 from the ring (slot offsets s0, sp; point offset ubase), writes ub of
// plane j into the ub ring at boff (zero outside 0 <= j < ny, v zero on the
// top wall) and advances the column state.
template <typename T, int UX>
__device__ __forceinline__ void rk_stage1_point(const T* su, const T* sv, const T* sw, T* bu, T* bv, T* bw, int s0,
                                                int sp, int ubase, int boff, ColState<T>& st, const Geo<T>& g,
                                                const YTab<T>& Y, int j, T dt, T nu, T fx) {
  const int ny = g.ny;
  const Ring2Acc<T, UX> A{su, sv, sw, s0, sp, ubase, st.um, st.vm, st.wm};
  const T uc = A.u(0, 0, 0), vc = A.v(0, 0, 0), wc = A.w(0, 0, 0);
  T ou = T(0), ov = T(0), ow = T(0);
  FaceFlux<T> up{T(0), T(0)};
  if (j >= 0 && j < ny) {
    const RhsOut<T> r = momentum_rhs<T>(A, g, Y, j, nu, fx, true, st.c, up);
    ou = uc + dt * r.ru;
    ov = (j == ny - 1) ? T(0) : vc + dt * r.rv;
    ow = wc + dt * r.rw;
  }
  st.c = up;
  st.um = uc;
  st.vm = vc;
  st.wm = wc;
  bu[boff] = ou;
  bv[boff] = ov;
  bw[boff] = ow;
}

template <int TX, int TZ>
struct RkFusedTile {
  static constexpr int TH = TX * TZ;
  static constexpr int EX = TX + 2, EZ = TZ + 2, EPL = EX * EZ;  // grown tile (stage 1)
  static constexpr int UX = TX + 4, UZ = TZ + 4, UPL = UX * UZ;  // input tile
  static constexpr int NRING = 2 * EX + 2 * TZ;                  // grown-tile cells outside the block's own
  static constexpr int PER = (UPL + TH - 1) / TH;                // input values per thread per plane
};

// At least four waves per SIMD: the register cap this sets (128 VGPRs, some
// spilled in FP64) costs less than the latency hiding fewer waves would lose.
// The tile index is remapped (xcd_slab_block over the whole grid) so that each
// XCD walks one contiguous run of tiles and neighbouring tiles share the halo
// lines in one L2 (runs within each y-chunk instead: within 1.5 %, either way).
// NT: the outputs, written once, are streamed (non-temporal) for large fields
// (the FP64 pass on 1024x256x512: about 2 % faster).
template <typename T, int TX, int TZ, int CY, bool NT>
__global__ void __launch_bounds__(TX * TZ, 4)
k_rk2_fused(const T* __restrict__ u, const T* __restrict__ v, const T* __restrict__ w, T* uo, T* vo, T* wo,
            Geo<T> g, T dt, T nu, T fx) {
  using Tl = RkFusedTile<TX, TZ>;
  constexpr int TH = Tl::TH, EX = Tl::EX, EPL = Tl::EPL, UX = Tl::UX, UPL = Tl::UPL, PER = Tl::PER;
  static_assert(Tl::NRING <= TH, "the grown tile's outer cells must fit one pass of the block");
  __shared__ T su[2 * UPL], sv[2 * UPL], sw[2 * UPL];
  __shared__ T bu[3 * EPL], bv[3 * EPL], bw[3 * EPL];
  __shared__ T sy[4 * (CY + 4)];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ntx = (nx + TX - 1) / TX, ntz = (nz + TZ - 1) / TZ;
  int b = xcd_slab_block(blockIdx.x, gridDim.x);
  const int bx = b % ntx;
  b /= ntx;
  const int bz = b % ntz;
  const int by = b / ntz;
  const int i0 = bx * TX, k0 = bz * TZ;
  const int j0 = by * CY, j1 = (j0 + CY < ny) ? j0 + CY : ny;
  const int t = threadIdx.x;
  const int tx = t % TX, tz = t / TX;
  const int i = i0 + tx, k = k0 + tz;
  const bool mine = (i < nx) && (k < nz);
  const long plane = (long)nx * nz;
  // input tile: two-cell halo, periodic wrap
  int toff[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int idx = t + q * TH;
    const int zz = idx / UX, xx = idx % UX;
    int gi = (i0 + xx - 2) % nx;
    if (gi < 0) gi += nx;
    int gk = (k0 + zz - 2) % nz;
    if (gk < 0) gk += nz;
    toff[q] = (idx < UPL) ? gk * nx + gi : -1;
  }
  T ru[PER], rv[PER], rw[PER];
#define CF_RKF_FETCH(jj)                                         \
  _Pragma("unroll") for (int q = 0; q < PER; ++q) {             \
    ru[q] = rv[q] = rw[q] = T(0);                               \
    if (toff[q] >= 0 && (jj) >= 0 && (jj) < ny) {               \
      const long o = (long)(jj) * plane + toff[q];              \
      ru[q] = u[o];                                             \
      rw[q] = w[o];                                             \
      if ((jj) < ny - 1) rv[q] = v[o];                          \
    }                                                           \
  }
#define CF_RKF_STORE(jj)                                         \
  _Pragma("unroll") for (int q = 0; q < PER; ++q) {             \
    if (toff[q] >= 0) {                                         \
      const int idx = ((jj) & 1) * UPL + t + q * TH;            \
      su[idx] = ru[q];                                          \
      sv[idx] = rv[q];                                          \
      sw[idx] = rw[q];                                          \
    }                                                           \
  }
  // point A: the block's own cell (tx, tz); point B (t < NRING): one cell of
  // the grown tile's outer ring
  const int ubA = (tz + 2) * UX + tx + 2, eA = (tz + 1) * EX + tx + 1;
  const bool hasB = t < Tl::NRING;
  int exB, ezB;
  if (t < EX) {
    exB = t, ezB = 0;
  } else if (t < 2 * EX) {
    exB = t - EX, ezB = Tl::EZ - 1;
  } else if (t < 2 * EX + TZ) {
    exB = 0, ezB = 1 + t - 2 * EX;
  } else {
    exB = EX - 1, ezB = 1 + (t - 2 * EX - TZ) % TZ;
  }
  const int ubB = (ezB + 1) * UX + exB + 1, eB = ezB * EX + exB;
#define CF_US(jj) (((jj) & 1) * UPL)
#define CF_BS(jj) ((((jj) + 3) % 3) * EPL)

  CF_RKF_FETCH(j0 - 2)
  CF_RKF_STORE(j0 - 2)
  CF_RKF_FETCH(j0 - 1)
  CF_RKF_STORE(j0 - 1)
  const YTab<T> Y = ytab_fill(sy, CY + 4, j0 - 2, g);
  __syncthreads();
  // stage-1 carries at face j0-1 and the columns at plane j0-2
  ColState<T> sA, sB;
  {
    const Ring2Acc<T, UX> A{su, sv, sw, CF_US(j0 - 2), CF_US(j0 - 1), ubA, T(0), T(0), T(0)};
    sA.c = upper_face_flux<T>(A, Y, j0 - 2, ny);
    sA.um = A.u(0, 0, 0);
    sA.vm = A.v(0, 0, 0);
    sA.wm = A.w(0, 0, 0);
    const Ring2Acc<T, UX> B{su, sv, sw, CF_US(j0 - 2), CF_US(j0 - 1), ubB, T(0), T(0), T(0)};
    sB.c = upper_face_flux<T>(B, Y, j0 - 2, ny);
    sB.um = B.u(0, 0, 0);
    sB.vm = B.v(0, 0, 0);
    sB.wm = B.w(0, 0, 0);
  }
  CF_RKF_FETCH(j0)
  __syncthreads();
  CF_RKF_STORE(j0)
  __syncthreads();
  CF_RKF_FETCH(j0 + 1)
  rk_stage1_point<T, UX>(su, sv, sw, bu, bv, bw, CF_US(j0 - 1), CF_US(j0), ubA, CF_BS(j0 - 1) + eA, sA, g, Y, j0 - 1,
                         dt, nu, fx);
  if (hasB)
    rk_stage1_point<T, UX>(su, sv, sw, bu, bv, bw, CF_US(j0 - 1), CF_US(j0), ubB, CF_BS(j0 - 1) + eB, sB, g, Y,
                           j0 - 1, dt, nu, fx);
  __syncthreads();
  CF_RKF_STORE(j0 + 1)
  __syncthreads();
  CF_RKF_FETCH(j0 + 2)
  rk_stage1_point<T, UX>(su, sv, sw, bu, bv, bw, CF_US(j0), CF_US(j0 + 1), ubA, CF_BS(j0) + eA, sA, g, Y, j0, dt, nu,
                         fx);
  if (hasB)
    rk_stage1_point<T, UX>(su, sv, sw, bu, bv, bw, CF_US(j0), CF_US(j0 + 1), ubB, CF_BS(j0) + eB, sB, g, Y, j0, dt,
                           nu, fx);
  __syncthreads();
  // stage-2 carries at face j0 and the own column of ub at plane j0-1
  ColState<T> s2;
  {
    const Ring2Acc<T, EX> A{bu, bv, bw, CF_BS(j0 - 1), CF_BS(j0), eA, T(0), T(0), T(0)};
    s2.c = upper_face_flux<T>(A, Y, j0 - 1, ny);
    s2.um = A.u(0, 0, 0);
    s2.vm = A.v(0, 0, 0);
    s2.wm = A.w(0, 0, 0);
  }
  const T hh = T(0.5), hd = T(0.5) * dt;
  // iteration s: stage 1 at plane s+1 and stage 2 at plane s-1, independent of
  // each other within the barrier interval (three ub planes in LDS)
  T p0u = T(0), p0v = T(0), p0w = T(0);
  for (int s = j0; s <= j1; ++s) {
    CF_RKF_STORE(s + 2)
    __syncthreads();
    CF_RKF_FETCH(s + 3)
    const T c0u = sA.um, c0v = sA.vm, c0w = sA.wm;  // u, v, w of this cell at plane s
    if (s + 1 <= j1) {
      rk_stage1_point<T, UX>(su, sv, sw, bu, bv, bw, CF_US(s + 1), CF_US(s + 2), ubA, CF_BS(s + 1) + eA, sA, g, Y,
                             s + 1, dt, nu, fx);
      if (hasB)
        rk_stage1_point<T, UX>(su, sv, sw, bu, bv, bw, CF_US(s + 1), CF_US(s + 2), ubB, CF_BS(s + 1) + eB, sB, g,
                               Y, s + 1, dt, nu, fx);
    }
    if (s > j0) {
      const int q = s - 1;
      const Ring2Acc<T, EX> B{bu, bv, bw, CF_BS(q), CF_BS(q + 1), eA, s2.um, s2.vm, s2.wm};
      const T uc = B.u(0, 0, 0), vc = B.v(0, 0, 0), wc = B.w(0, 0, 0);
      FaceFlux<T> up;
      const RhsOut<T> r = momentum_rhs<T>(B, g, Y, q, nu, fx, true, s2.c, up);
      s2.c = up;
      s2.um = uc;
      s2.vm = vc;
      s2.wm = wc;
      if (mine) {
        const long id = (long)q * plane + (long)k * nx + i;
        st_once<NT>(hh * (p0u + uc) + hd * r.ru, &uo[id]);
        st_once<NT>((q == ny - 1) ? T(0) : hh * (p0v + vc) + hd * r.rv, &vo[id]);
        st_once<NT>(hh * (p0w + wc) + hd * r.rw, &wo[id]);
      }
    }
    p0u = c0u;
    p0v = c0v;
    p0w = c0w;
    __syncthreads();
  }
#undef CF_RKF_FETCH
#undef CF_RKF_STORE
#undef CF_US
#undef CF_BS
}

}  // namespace cf
