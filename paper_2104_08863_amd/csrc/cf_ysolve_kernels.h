// Wall-normal solves of the spectral lines (Section 2.1, Eq. (9) corrected;
// Section 2.2 PDD).  Spectral layout [ny][nx/2+1][nz]; line l = kx*nz + kz,
// row stride (nx/2+1)*nz.
//
// k_ysolve: a block owns LB consecutive lines (consecutive kz, so every row
// access of the block is a contiguous run of LB complex values); each line is
// cut into P partitions of M rows and thread (q, i) = (tid % LB, tid / LB)
// solves partition i of line q in registers (Eq. (20)).  Interfaces go through
// LDS; the reduced system is either the dropped 2x2 form (all lines of the
// block above the plan's k^2 threshold) or the exact block system solved by
// cyclic reduction.  Lines flagged special (the kx = kz = 0 line, and in mixed
// precision the lowest-wavenumber set) are not written here.
//
// k_special_lines: FP64 Thomas along whole lines, one thread per line, with
// the gauge handling of the singular kx = kz = 0 line.
#pragma once

#include "cf_pdd.h"

namespace cf {

struct YArgs {
  int ny, nz, nkx;
  int P;        // partitions per line
  int LB;       // lines per block
  long nlines;  // nkx * nz
  int skip_kx;  // lines with kx < skip_kx and min(kz, nz-kz) < skip_kz are special
  int skip_kz;
};

__device__ __forceinline__ bool is_special(int kx, int kz, int nz, int skip_kx, int skip_kz) {
  const int kzs = kz < nz - kz ? kz : nz - kz;
  return (kx == 0 && kz == 0) || (kx < skip_kx && kzs < skip_kz);
}

// Dynamic LDS layout: a[ny], c[ny] (T), then per (partition, line):
//   interface data: x1, xm (cx), v1, vm, w1, wm (T)  -> arrays [P][LB]
//   reduced rows zrow<T> [P][LB], results y1, y2 (cx) [P][LB]
template <typename T>
__host__ __device__ constexpr size_t ysolve_lds_bytes(int ny, int P, int LB) {
  return sizeof(T) * 2 * ny + (sizeof(cx<T>) * 4 + sizeof(T) * 4 + sizeof(zrow<T>)) * size_t(P) * LB;
}

template <typename T, int M>
__global__ void __launch_bounds__(512)
k_ysolve(const cx<T>* fin, cx<T>* pout, const T* __restrict__ acoef,
         const T* __restrict__ ccoef, const T* __restrict__ kx2, const T* __restrict__ kz2, T k2drop,
         YArgs ya) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int LB = ya.LB, P = ya.P, ny = ya.ny;
  T* sa = reinterpret_cast<T*>(smem);
  T* sc = sa + ny;
  cx<T>* s_x1 = reinterpret_cast<cx<T>*>(sc + ny);
  cx<T>* s_xm = s_x1 + P * LB;
  cx<T>* s_y1 = s_xm + P * LB;
  cx<T>* s_y2 = s_y1 + P * LB;
  T* s_v1 = reinterpret_cast<T*>(s_y2 + P * LB);
  T* s_vm = s_v1 + P * LB;
  T* s_w1 = s_vm + P * LB;
  T* s_wm = s_w1 + P * LB;
  zrow<T>* s_z = reinterpret_cast<zrow<T>*>(s_wm + P * LB);

  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    sa[j] = acoef[j];
    sc[j] = ccoef[j];
  }
  const int q = threadIdx.x % LB;
  const int i = threadIdx.x / LB;
  const long line = (long)blockIdx.x * LB + q;
  const bool ok = line < ya.nlines;
  const int kx = ok ? int(line / ya.nz) : 0;
  const int kz = ok ? int(line % ya.nz) : 1;
  const T k2 = ok ? kx2[kx] + kz2[kz] : T(1);
  const long rs = (long)ya.nkx * ya.nz;
  const int j0 = i * M;
  const long base = (ok ? line : 0) + (long)j0 * rs;

  cx<T> d[M];
  T v[M], w[M];
#pragma unroll
  for (int s = 0; s < M; ++s) d[s] = ok ? fin[base + s * rs] : mk(T(0), T(0));
  __syncthreads();  // coefficients staged
  pdd_local<M, T>(sa + j0, sc + j0, k2, d, v, w);

  const int me = i * LB + q;
  s_x1[me] = d[0];
  s_xm[me] = d[M - 1];
  s_v1[me] = v[0];
  s_vm[me] = v[M - 1];
  s_w1[me] = w[0];
  s_wm[me] = w[M - 1];
  // drop the corner terms only when every line of the block allows it
  const int all_drop = __syncthreads_and((!ok) || k2 >= k2drop);
  const int Q = P - 1;
  cx<T> y1 = mk(T(0), T(0)), y2 = mk(T(0), T(0));
  if (all_drop) {
    if (i < Q) {
      const int nx_ = (i + 1) * LB + q;
      pdd_cramer(s_wm[me], s_v1[nx_], s_xm[me], s_x1[nx_], y1, y2);
    }
  } else {
    zrow<T> z;
    if (i < Q) {
      const int nx_ = (i + 1) * LB + q;
      z = zrow_make(s_vm[me], s_wm[me], s_v1[nx_], s_w1[nx_], s_xm[me], s_x1[nx_]);
    }
    for (int st = 1; st < Q; st *= 2) {
      if (i < Q) s_z[me] = z;
      __syncthreads();
      if (i < Q) {
        const bool hl = i - st >= 0, hh = i + st < Q;
        z = zrow_reduce(z, &s_z[(hl ? i - st : i) * LB + q], hl, &s_z[(hh ? i + st : i) * LB + q], hh);
      }
      __syncthreads();
    }
    if (i < Q) zrow_finish(z, y1, y2);
  }
  if (i < Q) {
    s_y1[me] = y1;
    s_y2[me] = y2;
  }
  __syncthreads();
  const cx<T> y1p = (i > 0) ? s_y1[(i - 1) * LB + q] : mk(T(0), T(0));
  const cx<T> y2m = (i < Q) ? y2 : mk(T(0), T(0));
  pdd_correct<M, T>(d, v, w, y1p, y2m);
  if (ok && !is_special(kx, kz, ya.nz, ya.skip_kx, ya.skip_kz)) {
#pragma unroll
    for (int s = 0; s < M; ++s) pout[base + s * rs] = d[s];
  }
}

// FP64 Thomas on whole lines, one thread per line.  lines[]: line indices;
// scratch: 3 * ny doubles per line (eliminated upper coefficient and the two
// parts of the eliminated right-hand side, then of the solution).  The k^2 = 0
// line is made compatible (dy-weighted mean of the RHS removed), solved with
// its top unknown pinned to zero, and shifted to zero dy-weighted mean.  Reads
// of fin all precede writes of pout, so the two may alias.
template <typename T>
__global__ void k_special_lines(const cx<T>* fin, cx<T>* pout,
                                const double* __restrict__ a, const double* __restrict__ c,
                                const double* __restrict__ dy, const double* __restrict__ kx2,
                                const double* __restrict__ kz2, const int* __restrict__ lines,
                                int n_lines, double* __restrict__ scratch, int ny, int nz, int nkx) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_lines) return;
  const long line = lines[l];
  const int kx = int(line / nz), kz = int(line % nz);
  const double k2 = kx2[kx] + kz2[kz];
  const long rs = (long)nkx * nz;
  double* cp = scratch + (long)l * 3 * ny;
  double* xr = cp + ny;
  double* xi = xr + ny;
  const bool mean_line = (kx == 0 && kz == 0);
  double sw = 0.0;
  for (int j = 0; j < ny; ++j) sw += dy[j];
  double mr = 0.0, mi = 0.0;
  if (mean_line) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < ny; ++j) {
      const cx<T> f = fin[line + j * rs];
      sr += dy[j] * double(f.re);
      si += dy[j] * double(f.im);
    }
    mr = sr / sw;
    mi = si / sw;
  }
  const int n = mean_line ? ny - 1 : ny;
  for (int j = 0; j < n; ++j) {
    const cx<T> f = fin[line + j * rs];
    const double fr = double(f.re) - mr, fi = double(f.im) - mi;
    const double b = -(a[j] + c[j]) - k2;
    const double cj = (j == n - 1) ? 0.0 : c[j];
    if (j == 0) {
      cp[j] = cj / b;
      xr[j] = fr / b;
      xi[j] = fi / b;
    } else {
      const double den = b - a[j] * cp[j - 1];
      cp[j] = cj / den;
      xr[j] = (fr - a[j] * xr[j - 1]) / den;
      xi[j] = (fi - a[j] * xi[j - 1]) / den;
    }
  }
  for (int j = n - 2; j >= 0; --j) {
    xr[j] = xr[j] - cp[j] * xr[j + 1];
    xi[j] = xi[j] - cp[j] * xi[j + 1];
  }
  double or_ = 0.0, oi = 0.0;
  if (mean_line) {
    xr[ny - 1] = 0.0;
    xi[ny - 1] = 0.0;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < ny; ++j) {
      sr += dy[j] * xr[j];
      si += dy[j] * xi[j];
    }
    or_ = sr / sw;
    oi = si / sw;
  }
  for (int j = 0; j < ny; ++j) pout[line + j * rs] = mk(T(xr[j] - or_), T(xi[j] - oi));
}

}  // namespace cf
