// Batched LDS Stockham FFT kernels for the periodic directions.
//
// Two spectral layouts, both with z fastest (every z-line contiguous):
//   A = [ny][nx/2+1][nz]  (x-side: the real transforms read and write it)
//   B = [nx/2+1][ny][nz]  (y-side: a wall-normal line is a column of one
//                          contiguous kx-slab)
//   * k_fft_z     : complex transform of every z-line, moving it from one
//                   layout to the other (line (o, i) of an [no][ni] array of
//                   lines goes to line (i, o)).
//   * k_r2c_x     : real transform of K consecutive x-rows (fixed j, rows
//                   k0..k0+K-1) through a half-length complex transform,
//                   written transposed into the spectral layout (for every kx
//                   a contiguous run of K values of kz).
//   * k_c2r_x     : the inverse, reading the transposed tile.
// Data enter the first radix pass straight from global memory and leave the
// last pass straight to global memory (or to LDS where the real<->half-complex
// step needs partner elements); intermediate passes exchange through LDS.
#pragma once

#include "cf_fft.h"

namespace cf {

template <int N>
struct FftT {
  static constexpr RadixPlan P = make_radix_plan(N);
  static constexpr int E = P.e;
  static constexpr int TPL = N / E;
  static constexpr int R0 = P.r[0];
  static constexpr int RL = P.r[P.np - 1];
};

// LDS position of element e of a line: one pad slot after every 16 elements.
// The exchange after a first radix-16 pass writes element b*16 + r from thread
// b, a stride of 16 elements that would put every lane of a quarter-wave on
// the same LDS banks; the pad turns it into a stride of 17.
CF_HD constexpr int lpad(int e) { return e + (e >> 4); }
constexpr int lpad_len(int n) { return n + (n >> 4); }

// Runs passes PASS..np-1 on the registers x (pass PASS input order on entry,
// last-pass output order on exit).  sl: this line's LDS (N slots).  Every
// thread of the block must call this (it contains block barriers).
template <int N, bool INV, typename T, int PASS>
__device__ __forceinline__ void fft_passes(cx<T>* x, int t, cx<T>* sl, const cx<T>* __restrict__ tw) {
  constexpr RadixPlan P = make_radix_plan(N);
  constexpr int E = P.e;
  constexpr int TPL = N / E;
  constexpr int R = P.r[PASS];
  constexpr int NS = plan_ns(N, PASS);
  if constexpr (PASS > 0) {
    constexpr int RP = P.r[PASS - 1];
    constexpr int NSP = plan_ns(N, PASS - 1);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E / RP; ++q) {
      const int b = t + q * TPL;
#pragma unroll
      for (int r = 0; r < RP; ++r) sl[lpad(st_out(RP, NSP, b, r))] = x[q * RP + r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
      const int b = t + q * TPL;
#pragma unroll
      for (int r = 0; r < R; ++r) x[q * R + r] = sl[lpad(st_in(N, R, b, r))];
    }
  }
#pragma unroll
  for (int q = 0; q < E / R; ++q) pass_group<N, R, NS, INV>(x + q * R, t + q * TPL, tw);
  if constexpr (PASS + 1 < P.np) fft_passes<N, INV, T, PASS + 1>(x, t, sl, tw);
}

constexpr int pow2_floor(int n) {
  int p = 1;
  while (2 * p <= n) p *= 2;
  return p;
}

constexpr int lds_lines(int n, int tpl, int esize, int budget) {
  int l = 256 / tpl;
  if (l < 1) l = 1;
  while (l > 1 && l * n * esize > budget) l /= 2;
  return l;
}

// ---------------------------------------------------------------- z (contiguous lines)
// Lines per block: about 256 threads, within 64 KB of LDS (against 32 KB: the
// FP32 2048- and 1536-point and FP64 512-point transforms 2-8 % faster).
template <typename T, int N>
struct ZCfg {
  static constexpr int LPB = lds_lines(lpad_len(N), FftT<N>::TPL, int(sizeof(cx<T>)), 65536);
  static constexpr int THREADS = LPB * FftT<N>::TPL;
};

// NT: lines read and written once, streamed (non-temporal) for large spectra:
// the FP64 512-point transforms on 1024x256x512 take 380 instead of 411-434 us.
template <typename T, int N, bool INV, bool NT>
__global__ void __launch_bounds__((ZCfg<T, N>::THREADS))
k_fft_z(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, const cx<T>* __restrict__ tw, int no,
        int ni) {
  using F = FftT<N>;
  constexpr int LPB = ZCfg<T, N>::LPB;
  __shared__ cx<T> lds[LPB * lpad_len(N)];
  const int tl = threadIdx.x % F::TPL;
  const int lb = threadIdx.x / F::TPL;
  const long nlines = (long)no * ni;
  const long line = (long)blockIdx.x * LPB + lb;
  const bool ok = line < nlines;
  const long lo = ok ? line : 0;
  const cx<T>* g = src + lo * N;
  cx<T>* o = dst + ((lo % ni) * no + lo / ni) * N;
  cx<T> x[F::E];
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) x[q * F::R0 + r] = ok ? ld_once<NT>(&g[st_in(N, F::R0, b, r)]) : mk(T(0), T(0));
  }
  fft_passes<N, INV, T, 0>(x, tl, lds + lb * lpad_len(N), tw);
  if (ok) {
#pragma unroll
    for (int q = 0; q < F::E / F::RL; ++q) {
      const int b = tl + q * F::TPL;
#pragma unroll
      for (int r = 0; r < F::RL; ++r) st_once<NT>(x[q * F::RL + r], &o[b + r * (N / F::RL)]);
    }
  }
}

// ---------------------------------------------------------------- x (real rows, transposed spectrum)
template <typename T, int NH>
struct XCfg {
  // FP32 blocks keep their twiddle tables (the length-NH table of the passes
  // and the NH+1 post-processing factors) in LDS: their many small cached loads
  // inside the barrier-separated passes cost more than the LDS (the FP32 tile
  // leaves room for them; in FP64 they would halve the blocks per CU).
  static constexpr bool kLdsTw = sizeof(T) == 4;
  static constexpr int TWB = kLdsTw ? (2 * NH + 1) * int(sizeof(cx<T>)) : 0;
  // rows per block: aim for 128-byte runs of kz in the transposed spectrum
  static constexpr int KWANT = int(128 / sizeof(cx<T>));
  static constexpr int S = lpad(NH) + 1;  // LDS row stride (holds kx = 0..NH at lpad(kx))
  static constexpr int kfit(int k) {
    return (k > 1 && (k * S * int(sizeof(cx<T>)) > (kLdsTw ? 159744 - TWB : 147456) || k * FftT<NH>::TPL > 1024))
               ? kfit(k / 2)
               : k;
  }
  static constexpr int K = kfit(KWANT);
  static constexpr int THREADS = K * FftT<NH>::TPL;
};

// The twiddle tables of an x-transform block: copied to LDS when XCfg says so
// (the caller synchronises before the first use), else the global tables.
template <typename T, int NH>
struct XTw {
  __device__ __forceinline__ static void stage(cx<T>* stw, cx<T>* stwp, const cx<T>*& tw, const cx<T>*& twp) {
    if constexpr (XCfg<T, NH>::kLdsTw) {
      for (int q = threadIdx.x; q <= NH; q += XCfg<T, NH>::THREADS) {
        if (q < NH) stw[q] = tw[q];
        stwp[q] = twp[q];
      }
      tw = stw;
      twp = stwp;
    }
  }
};

// Row sources for the forward real transform: element pair (x_{2m}, x_{2m+1})
// of row (j, k).
// Sources whose kPSum is true also give the FP64 sum over their rows of the
// pressure they read (psum_pair); k_r2c_x adds it up per block into psum.
template <typename T, typename Tin>
struct SrcPlain {
  static constexpr bool kPSum = false;
  const Tin* __restrict__ f;
  int nx, nz;
  __device__ __forceinline__ cx<T> pair(int j, int k, int m) const {
    const cx<Tin>* row = reinterpret_cast<const cx<Tin>*>(f + ((long)j * nz + k) * nx);
    cx<Tin> v = row[m];
    return mk(T(v.re), T(v.im));
  }
};

// Divergence of a staggered velocity field times `scale` (Eq. (7) right-hand
// side), produced on the fly: f_i = [(u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy_j
// + (w_k - w_{k-1})/dz] * scale with v = 0 on both walls.
template <typename T, typename Ts>
struct SrcDiv {
  static constexpr bool kPSum = false;
  const Ts* __restrict__ u;
  const Ts* __restrict__ v;
  const Ts* __restrict__ w;
  const double* __restrict__ rdy;
  double rdx, rdz, scale;
  int nx, ny, nz;
  __device__ __forceinline__ cx<T> pair(int j, int k, int m) const {
    const long row = ((long)j * nz + k) * nx;
    const long plane = (long)nz * nx;
    const int km = (k == 0) ? nz - 1 : k - 1;
    const long rowm = ((long)j * nz + km) * nx;
    const int i0 = 2 * m, i1 = 2 * m + 1, im = (m == 0) ? nx - 1 : 2 * m - 1;
    const cx<Ts> up = reinterpret_cast<const cx<Ts>*>(u + row)[m];
    const double uim = double(u[row + im]);
    const cx<Ts> wp = reinterpret_cast<const cx<Ts>*>(w + row)[m];
    const cx<Ts> wmp = reinterpret_cast<const cx<Ts>*>(w + rowm)[m];
    double v0 = 0.0, v1 = 0.0, vm0 = 0.0, vm1 = 0.0;
    if (j < ny - 1) {
      const cx<Ts> vp = reinterpret_cast<const cx<Ts>*>(v + row)[m];
      v0 = double(vp.re);
      v1 = double(vp.im);
    }
    if (j > 0) {
      const cx<Ts> vmp = reinterpret_cast<const cx<Ts>*>(v + row - plane)[m];
      vm0 = double(vmp.re);
      vm1 = double(vmp.im);
    }
    const double r = rdy[j];
    const double f0 = ((double(up.re) - uim) * rdx + (v0 - vm0) * r + (double(wp.re) - double(wmp.re)) * rdz) * scale;
    const double f1 = ((double(up.im) - double(up.re)) * rdx + (v1 - vm1) * r +
                       (double(wp.im) - double(wmp.im)) * rdz) * scale;
    (void)i0;
    (void)i1;
    return mk(T(f0), T(f1));
  }
};

// Divergence of the face field (g_u / dy_j, g_v / dyc_j, g_w / dy_j): the right-
// hand side of the transposed projection (g / W with the face weights W).
template <typename T, typename Ts>
struct SrcDivW {
  static constexpr bool kPSum = false;
  const Ts* __restrict__ u;
  const Ts* __restrict__ v;
  const Ts* __restrict__ w;
  const double* __restrict__ rdy;
  const double* __restrict__ rdyc;
  double rdx, rdz;
  int nx, ny, nz;
  __device__ __forceinline__ cx<T> pair(int j, int k, int m) const {
    const long row = ((long)j * nz + k) * nx;
    const long plane = (long)nz * nx;
    const int km = (k == 0) ? nz - 1 : k - 1;
    const long rowm = ((long)j * nz + km) * nx;
    const int im = (m == 0) ? nx - 1 : 2 * m - 1;
    const double ry = rdy[j];
    const cx<Ts> up = reinterpret_cast<const cx<Ts>*>(u + row)[m];
    const double uim = double(u[row + im]);
    const cx<Ts> wp = reinterpret_cast<const cx<Ts>*>(w + row)[m];
    const cx<Ts> wmp = reinterpret_cast<const cx<Ts>*>(w + rowm)[m];
    double v0 = 0.0, v1 = 0.0, vm0 = 0.0, vm1 = 0.0;
    if (j < ny - 1) {
      const cx<Ts> vp = reinterpret_cast<const cx<Ts>*>(v + row)[m];
      v0 = double(vp.re) * rdyc[j];
      v1 = double(vp.im) * rdyc[j];
    }
    if (j > 0) {
      const cx<Ts> vmp = reinterpret_cast<const cx<Ts>*>(v + row - plane)[m];
      vm0 = double(vmp.re) * rdyc[j - 1];
      vm1 = double(vmp.im) * rdyc[j - 1];
    }
    const double f0 = ((double(up.re) - uim) * ry * rdx + (v0 - vm0) * ry + (double(wp.re) - double(wmp.re)) * ry * rdz);
    const double f1 = ((double(up.im) - double(up.re)) * ry * rdx + (v1 - vm1) * ry +
                       (double(wp.im) - double(wmp.im)) * ry * rdz);
    return mk(T(f0), T(f1));
  }
};

// FP64 residual of the Poisson equation, r = f - L_h p (7-point staggered
// Laplacian, no flux through the walls: a_0 = c_{ny-1} = 0), rounded to T.
// The right-hand side f comes from an inner source evaluated in FP64 (a plain
// array, a divergence, or a weighted divergence).  The residual cannot see a
// constant in p, so the kernel also sums p (FP64, per block of rows) into
// psum: the correction solve uses it to restore the gauge mean_W(p) = 0 that
// the FP32 transforms of the previous solve leave off by their rounding.
// Tp = float: every row of the FP64 array p holds that row's nx values as
// FP32 in its first half (the FP32 solve's output before the first correction
// is added; see DstRows32), read exactly as FP64.
template <typename T, typename In, typename Tp = double>
struct SrcResidual {
  static constexpr bool kPSum = true;
  In in;
  const double* __restrict__ p;
  const double* __restrict__ a;
  const double* __restrict__ c;
  double rdx2, rdz2;
  int nx, ny, nz;
  double* __restrict__ psum;  // [blocks of k_r2c_x]: the block's sum of p
  // values 2m, 2m+1 and value i of the row starting at FP64 offset row
  __device__ __forceinline__ cx<double> pv2(long row, int m) const {
    const cx<Tp> v = reinterpret_cast<const cx<Tp>*>(reinterpret_cast<const Tp*>(p + row))[m];
    return mk(double(v.re), double(v.im));
  }
  __device__ __forceinline__ double pv1(long row, int i) const {
    return double(reinterpret_cast<const Tp*>(p + row)[i]);
  }
  __device__ __forceinline__ double psum_pair(int j, int k, int m) const {
    const cx<double> pc = pv2(((long)j * nz + k) * nx, m);
    return pc.re + pc.im;
  }
  __device__ __forceinline__ cx<T> pair(int j, int k, int m) const {
    const long plane = (long)nz * nx;
    const long row = ((long)j * nz + k) * nx;
    const int kp = (k + 1 == nz) ? 0 : k + 1, km = (k == 0) ? nz - 1 : k - 1;
    const long rowp = ((long)j * nz + kp) * nx, rowm = ((long)j * nz + km) * nx;
    const int i0 = 2 * m, i1 = 2 * m + 1;
    const int im = (m == 0) ? nx - 1 : i0 - 1, ip = (i1 + 1 == nx) ? 0 : i1 + 1;
    const cx<double> fd = in.pair(j, k, m);
    const cx<double> pc = pv2(row, m);
    const double pim = pv1(row, im), pip = pv1(row, ip);
    const cx<double> pkp = pv2(rowp, m);
    const cx<double> pkm = pv2(rowm, m);
    double l0 = (pc.im - 2.0 * pc.re + pim) * rdx2 + (pkp.re - 2.0 * pc.re + pkm.re) * rdz2;
    double l1 = (pip - 2.0 * pc.im + pc.re) * rdx2 + (pkp.im - 2.0 * pc.im + pkm.im) * rdz2;
    if (j + 1 < ny) {
      const cx<double> q = pv2(row + plane, m);
      l0 += c[j] * (q.re - pc.re);
      l1 += c[j] * (q.im - pc.im);
    }
    if (j > 0) {
      const cx<double> q = pv2(row - plane, m);
      l0 += a[j] * (q.re - pc.re);
      l1 += a[j] * (q.im - pc.im);
    }
    return mk(T(fd.re - l0), T(fd.im - l1));
  }
};

template <typename T, int NH, typename Src>
__global__ void __launch_bounds__((XCfg<T, NH>::THREADS))
k_r2c_x(Src src, cx<T>* __restrict__ spec, const cx<T>* tw, const cx<T>* twp, int ny, int nz) {
  using F = FftT<NH>;
  constexpr int K = XCfg<T, NH>::K;
  constexpr int S = XCfg<T, NH>::S;
  constexpr int NKX = NH + 1;
  constexpr int NTW = XCfg<T, NH>::kLdsTw ? NH + 1 : 1;
  __shared__ cx<T> lds[K * S];
  __shared__ cx<T> stw[NTW], stwp[NTW];
  XTw<T, NH>::stage(stw, stwp, tw, twp);
  if constexpr (XCfg<T, NH>::kLdsTw) __syncthreads();
  // ny * nzb row blocks (nzb blocks of K rows per y-plane), each XCD on a
  // contiguous run of every plane's blocks: the z-neighbour rows that the
  // divergence and residual sources read across block edges are mostly in the
  // same L2 (the mixed 2048x512x1536 solve's residual transform: 9.8 -> 8.7 ms)
  const int nzb = (nz + K - 1) / K;
  const int lb = xcd_slab_block(blockIdx.x, nzb);
  const int j = lb / nzb;
  const int k0 = (lb % nzb) * K;
  const int tl = threadIdx.x % F::TPL;
  const int rr = threadIdx.x / F::TPL;
  const int k = k0 + rr;
  const bool ok = k < nz;
  cx<T> x[F::E];
  double psum = 0.0;
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      x[q * F::R0 + r] = ok ? src.pair(j, k, st_in(NH, F::R0, b, r)) : mk(T(0), T(0));
      if constexpr (Src::kPSum) psum += ok ? src.psum_pair(j, k, st_in(NH, F::R0, b, r)) : 0.0;
    }
  }
  cx<T>* sl = lds + rr * S;
  fft_passes<NH, false, T, 0>(x, tl, sl, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::E / F::RL; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::RL; ++r) sl[lpad(b + r * (NH / F::RL))] = x[q * F::RL + r];
  }
  __syncthreads();
  const long plane = (long)j * NKX;
  constexpr int TH = XCfg<T, NH>::THREADS;
  constexpr int ITEMS = NKX * K;
#pragma unroll
  for (int it = 0; it < (ITEMS + TH - 1) / TH; ++it) {
    const int idx = threadIdx.x + it * TH;
    const int r = idx % K;
    const int kx = idx / K;
    if (idx < ITEMS && k0 + r < nz) {
      const cx<T>* row = lds + r * S;
      cx<T> X = r2c_post(row[lpad(kx == NH ? 0 : kx)], row[lpad(kx == 0 ? 0 : NH - kx)], twp[kx]);
      spec[(plane + kx) * nz + k0 + r] = X;
    }
  }
  if constexpr (Src::kPSum) {
    // block sum of p in a fixed order (the LDS tile is free again: TH <= K*S
    // complex slots hold TH doubles)
    double* red = reinterpret_cast<double*>(lds);
    __syncthreads();
    red[threadIdx.x] = psum;
    __syncthreads();
    constexpr int P2 = pow2_floor(TH);
    for (int h = P2; h > 0; h >>= 1) {
      if (threadIdx.x < h && threadIdx.x + h < TH) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) src.psum[lb] = red[0];
  }
}

// Row sinks for the inverse real transform: receives (x_{2m}, x_{2m+1}) of row
// (j, k), already scaled.
template <typename T, typename Tout>
struct DstPlain {
  static constexpr bool kPre = false;
  Tout* __restrict__ p;
  int nx, nz;
  __device__ __forceinline__ void put(int j, int k, int m, cx<T> v) const {
    cx<Tout>* row = reinterpret_cast<cx<Tout>*>(p + ((long)j * nz + k) * nx);
    row[m] = mk(Tout(v.re), Tout(v.im));
  }
};

// FP32 output packed into FP64 rows: row (j, k) of the FP64 array p receives
// its nx values as FP32 in the first half of its own bytes.  An FP32 solve
// that a refinement will correct stores its result this way: the values are
// exactly those the FP64 store would hold, at half the bytes written here and
// read by the residual and the accumulation that follow.
template <typename T>
struct DstRows32 {
  static constexpr bool kPre = false;
  double* __restrict__ p;
  int nx, nz;
  __device__ __forceinline__ void put(int j, int k, int m, cx<T> v) const {
    float* row = reinterpret_cast<float*>(p + ((long)j * nz + k) * nx);
    reinterpret_cast<cx<float>*>(row)[m] = mk(float(v.re), float(v.im));
  }
};

// p += correction (iterative refinement: the correction solve adds to p).
template <typename T>
struct DstAccum {
  static constexpr bool kPre = false;
  double* __restrict__ p;
  int nx, nz;
  __device__ __forceinline__ void put(int j, int k, int m, cx<T> v) const {
    cx<double>* row = reinterpret_cast<cx<double>*>(p + ((long)j * nz + k) * nx);
    cx<double> o = row[m];
    o.re += double(v.re);
    o.im += double(v.im);
    row[m] = o;
  }
};

// p = p32 + correction, p32 packed into the same FP64 rows (DstRows32).  The
// row's FP32 values are read before the FP64 values are written over them:
// k_c2r_x loads them (pre) before its first barrier and writes after its
// last; a block owns its rows, so no other block touches those bytes.
struct DstAccumRows32 {
  static constexpr bool kPre = true;
  double* __restrict__ p;
  int nx, nz;
  __device__ __forceinline__ cx<float> pre(int j, int k, int m) const {
    const float* row = reinterpret_cast<const float*>(p + ((long)j * nz + k) * nx);
    return reinterpret_cast<const cx<float>*>(row)[m];
  }
  __device__ __forceinline__ void put(int j, int k, int m, cx<float> v, cx<float> old) const {
    cx<double>* row = reinterpret_cast<cx<double>*>(p + ((long)j * nz + k) * nx);
    row[m] = mk(double(old.re) + double(v.re), double(old.im) + double(v.im));
  }
};

template <typename T, int NH, typename Dst>
__global__ void __launch_bounds__((XCfg<T, NH>::THREADS))
k_c2r_x(const cx<T>* __restrict__ spec, Dst dst, const cx<T>* tw, const cx<T>* twp, int ny, int nz, T scale) {
  using F = FftT<NH>;
  constexpr int K = XCfg<T, NH>::K;
  constexpr int S = XCfg<T, NH>::S;
  constexpr int NKX = NH + 1;
  constexpr int NTW = XCfg<T, NH>::kLdsTw ? NH + 1 : 1;
  __shared__ cx<T> lds[K * S];
  __shared__ cx<T> stw[NTW], stwp[NTW];
  XTw<T, NH>::stage(stw, stwp, tw, twp);  // first read after the barrier below
  const int nzb = (nz + K - 1) / K;
  const int j = blockIdx.x / nzb;
  const int k0 = (blockIdx.x % nzb) * K;
  const long plane = (long)j * NKX;
  const int tl = threadIdx.x % F::TPL;
  const int rr = threadIdx.x / F::TPL;
  const int k = k0 + rr;
  // the sink's old row values (DstAccumRows32), in the order of the output loop
  cx<float> pre[Dst::kPre ? F::E : 1];
  if constexpr (Dst::kPre) {
#pragma unroll
    for (int q = 0; q < F::E / F::RL; ++q) {
      const int b = tl + q * F::TPL;
#pragma unroll
      for (int r = 0; r < F::RL; ++r)
        pre[q * F::RL + r] = (k < nz) ? dst.pre(j, k, b + r * (NH / F::RL)) : mk(0.f, 0.f);
    }
  }
  {
    constexpr int TH = XCfg<T, NH>::THREADS;
    constexpr int ITEMS = NKX * K;
    constexpr int IT = (ITEMS + TH - 1) / TH;
    cx<T> v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * TH;
      const int r = idx % K;
      const int kx = idx / K;
      v[it] = (idx < ITEMS && k0 + r < nz) ? spec[(plane + kx) * nz + k0 + r] : mk(T(0), T(0));
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = threadIdx.x + it * TH;
      if (idx < ITEMS) lds[(idx % K) * S + lpad(idx / K)] = v[it];
    }
  }
  if constexpr (Dst::kPre) {
    // every old value has arrived before the barrier (the block overwrites
    // these bytes after later barriers)
#pragma unroll
    for (int e = 0; e < F::E; ++e) asm volatile("" : : "v"(pre[e].re), "v"(pre[e].im));
  }
  __syncthreads();
  cx<T>* sl = lds + rr * S;
  cx<T> x[F::E];
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) {
      const int m = st_in(NH, F::R0, b, r);
      cx<T> a = sl[lpad(m)], bb = sl[lpad(NH - m)];
      if (m == 0) {
        a.im = T(0);
        bb.im = T(0);
      }
      x[q * F::R0 + r] = c2r_pre(a, bb, twp[m]);
    }
  }
  fft_passes<NH, true, T, 0>(x, tl, sl, tw);
  if (k < nz) {
#pragma unroll
    for (int q = 0; q < F::E / F::RL; ++q) {
      const int b = tl + q * F::TPL;
#pragma unroll
      for (int r = 0; r < F::RL; ++r) {
        if constexpr (Dst::kPre)
          dst.put(j, k, b + r * (NH / F::RL), x[q * F::RL + r] * scale, pre[q * F::RL + r]);
        else
          dst.put(j, k, b + r * (NH / F::RL), x[q * F::RL + r] * scale);
      }
    }
  }
}

}  // namespace cf
