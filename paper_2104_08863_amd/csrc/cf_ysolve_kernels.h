// Wall-normal solves of the spectral lines (Section 2.1, Eq. (9) corrected;
// Section 2.2 PDD).  Spectral layout B = [nx/2+1][ny][nz]: line l = kx*nz + kz
// starts at kx*ny*nz + kz and has row stride nz, so a block of consecutive
// lines stays inside one contiguous kx-slab.
//
// k_ysolve: a block owns LB consecutive lines (consecutive kz, so every row
// access of the block is a contiguous run of LB complex values); each line is
// cut into P partitions of M rows and thread (q, i) = (tid % LB, tid / LB)
// solves partition i of line q in registers (Eq. (20)).  Interfaces go through
// LDS; the reduced system is either the dropped 2x2 form (all lines of the
// block above the plan's k^2 threshold) or the exact block system solved by
// cyclic reduction.  Lines flagged special (the kx = kz = 0 line, and in mixed
// precision the lowest-wavenumber set) are not written here.  The slab modes
// (YMode) split this kernel at the interface exchange: the interface rows go
// through a global buffer instead of LDS.
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
  int pa, pb;   // slab modes: the partitions [pa, pb) of one y-slab
  void* iface;  // slab modes: interface rows [P][8][nlines] (x1 re/im, xm re/im, v1, vm, w1, wm)
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

template <typename T, int M, int MODE>
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
  const zrow_soa<T> s_z{s_wm + P * LB, P * LB};

  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    sa[j] = acoef[j];
    sc[j] = ccoef[j];
  }
  const int q = threadIdx.x % LB;
  // partition of this thread (a local-mode block has threads for [pa, pb) only)
  const int i = threadIdx.x / LB + (MODE == kSlabLocal ? ya.pa : 0);
  const bool own = (MODE == kWhole) || (i >= ya.pa && i < ya.pb);
  const long line = (long)blockIdx.x * LB + q;
  const bool ok = line < ya.nlines;
  const int kx = ok ? int(line / ya.nz) : 0;
  const int kz = ok ? int(line % ya.nz) : 1;
  const T k2 = ok ? kx2[kx] + kz2[kz] : T(1);
  const long rs = ya.nz;
  const int j0 = i * M;
  const long base = (long)kx * ny * ya.nz + kz + (long)j0 * rs;

  cx<T> d[M];
  T v[M], w[M];
#pragma unroll
  for (int s = 0; s < M; ++s) d[s] = (ok && own) ? fin[base + s * rs] : mk(T(0), T(0));
  __syncthreads();  // coefficients staged
  if (own) pdd_local<M, T>(sa + j0, sc + j0, k2, d, v, w);

  T* ifc = static_cast<T*>(ya.iface);
  const long nl = ya.nlines;
  if (MODE == kSlabLocal) {
    if (ok) {
      T* r = ifc + (long)i * 8 * nl + line;
      r[0 * nl] = d[0].re;
      r[1 * nl] = d[0].im;
      r[2 * nl] = d[M - 1].re;
      r[3 * nl] = d[M - 1].im;
      r[4 * nl] = v[0];
      r[5 * nl] = v[M - 1];
      r[6 * nl] = w[0];
      r[7 * nl] = w[M - 1];
    }
    return;
  }
  const int me = i * LB + q;
  if (MODE == kWhole) {
    s_x1[me] = d[0];
    s_xm[me] = d[M - 1];
    s_v1[me] = v[0];
    s_vm[me] = v[M - 1];
    s_w1[me] = w[0];
    s_wm[me] = w[M - 1];
  } else {
    // every partition's rows as the local passes wrote them (bitwise equal to
    // this thread's own recomputed values for i in [pa, pb))
    const T* r = ifc + (long)i * 8 * nl + (ok ? line : 0);
    s_x1[me] = mk(r[0 * nl], r[1 * nl]);
    s_xm[me] = mk(r[2 * nl], r[3 * nl]);
    s_v1[me] = r[4 * nl];
    s_vm[me] = r[5 * nl];
    s_w1[me] = r[6 * nl];
    s_wm[me] = r[7 * nl];
  }
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
      if (i < Q) s_z.put(me, z);
      __syncthreads();
      if (i < Q) {
        const bool hl = i - st >= 0, hh = i + st < Q;
        const zrow<T> lo = s_z.get((hl ? i - st : i) * LB + q);
        const zrow<T> hi = s_z.get((hh ? i + st : i) * LB + q);
        z = zrow_reduce(z, &lo, hl, &hi, hh);
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
  if (ok && own && !is_special(kx, kz, ya.nz, ya.skip_kx, ya.skip_kz)) {
#pragma unroll
    for (int s = 0; s < M; ++s) pout[base + s * rs] = d[s];
  }
}

// FP64 Thomas on whole lines, one block per line.  The elimination factors
// of each listed line (den_j = b_j - a_j cp_{j-1}, cp_j = c_j / den_j, with the
// top row left out for the k^2 = 0 line) come from the plan.  The k^2 = 0
// line is made compatible (dy-weighted mean of the RHS removed), solved with
// its top unknown pinned to zero, and shifted to zero dy-weighted mean.  The
// line is staged in LDS; reads of fin all precede writes of pout, so the two
// may alias.  The sweeps follow the textbook operation order without
// contraction, like the reference definition.
template <typename T>
__global__ void __launch_bounds__(256)
k_special_lines(const cx<T>* fin, cx<T>* pout, const double* __restrict__ a,
                const double* __restrict__ den, const double* __restrict__ cpt,
                const double* __restrict__ dy, const int* __restrict__ lines, int ny, int nz) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) double sm[];
  double* fr = sm;
  double* fi = fr + ny;
  double* sa = fi + ny;
  double* sd = sa + ny;
  double* sc = sd + ny;
  double* red = sc + ny;  // 3 * blockDim doubles
  const int l = blockIdx.x;
  const long line = lines[l];
  const int kx = int(line / nz), kz = int(line % nz);
  const long base = (long)kx * ny * nz + kz;
  const bool mean_line = (kx == 0 && kz == 0);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int j = tid; j < ny; j += nt) {
    const cx<T> f = fin[base + (long)j * nz];
    fr[j] = double(f.re);
    fi[j] = double(f.im);
    sa[j] = a[j];
    sd[j] = den[(long)l * ny + j];
    sc[j] = cpt[(long)l * ny + j];
  }
  __syncthreads();
  // dy-weighted means (block reduction), used by the k^2 = 0 line only
  auto wmean = [&](double& mr, double& mi) {
    double r = 0.0, im = 0.0, w = 0.0;
    for (int j = tid; j < ny; j += nt) {
      r += dy[j] * fr[j];
      im += dy[j] * fi[j];
      w += dy[j];
    }
    red[tid] = r;
    red[nt + tid] = im;
    red[2 * nt + tid] = w;
    __syncthreads();
    for (int h = nt / 2; h > 0; h /= 2) {
      if (tid < h) {
        red[tid] += red[tid + h];
        red[nt + tid] += red[nt + tid + h];
        red[2 * nt + tid] += red[2 * nt + tid + h];
      }
      __syncthreads();
    }
    mr = red[0] / red[2 * nt];
    mi = red[nt] / red[2 * nt];
    __syncthreads();
  };
  if (mean_line) {
    double mr, mi;
    wmean(mr, mi);
    for (int j = tid; j < ny; j += nt) {
      fr[j] = fr[j] - mr;
      fi[j] = fi[j] - mi;
    }
    __syncthreads();
  }
  const int n = mean_line ? ny - 1 : ny;
  if (tid == 0) {
    // sweeps in chunks of 8 rows whose operands are read before the chain
    constexpr int C = 8;
    double xr = fr[0] / sd[0], xi = fi[0] / sd[0];
    fr[0] = xr;
    fi[0] = xi;
    for (int j0 = 1; j0 < n; j0 += C) {
      double ar[C], br[C], bi[C], dr[C];
#pragma unroll
      for (int u = 0; u < C; ++u) {
        const int j = j0 + u < n ? j0 + u : n - 1;
        ar[u] = sa[j];
        br[u] = fr[j];
        bi[u] = fi[j];
        dr[u] = sd[j];
      }
#pragma unroll
      for (int u = 0; u < C; ++u) {
        if (j0 + u < n) {
          const double tr = ar[u] * xr, ti = ar[u] * xi;
          xr = (br[u] - tr) / dr[u];
          xi = (bi[u] - ti) / dr[u];
          fr[j0 + u] = xr;
          fi[j0 + u] = xi;
        }
      }
    }
    for (int j0 = n - 2; j0 >= 0; j0 -= C) {
      double cr[C], br[C], bi[C];
#pragma unroll
      for (int u = 0; u < C; ++u) {
        const int j = j0 - u >= 0 ? j0 - u : 0;
        cr[u] = sc[j];
        br[u] = fr[j];
        bi[u] = fi[j];
      }
#pragma unroll
      for (int u = 0; u < C; ++u) {
        if (j0 - u >= 0) {
          const double tr = cr[u] * xr, ti = cr[u] * xi;
          xr = br[u] - tr;
          xi = bi[u] - ti;
          fr[j0 - u] = xr;
          fi[j0 - u] = xi;
        }
      }
    }
    if (mean_line) {
      fr[ny - 1] = 0.0;
      fi[ny - 1] = 0.0;
    }
  }
  __syncthreads();
  double orr = 0.0, oi = 0.0;
  if (mean_line) wmean(orr, oi);
  for (int j = tid; j < ny; j += nt) pout[base + (long)j * nz] = mk(T(fr[j] - orr), T(fi[j] - oi));
}

}  // namespace cf
