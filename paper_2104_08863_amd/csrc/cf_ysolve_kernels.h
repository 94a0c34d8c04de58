// Wall-normal solves of the spectral lines (Section 2.1, Eq. (9) corrected;
// Section 2.2 PDD).  Spectral layout B = [nx/2+1][ny][nz]: line l = kx*nz + kz
// starts at kx*ny*nz + kz and has row stride nz, so a block of consecutive
// lines stays inside one contiguous kx-slab.
//
// k_ysolve: a block owns LB consecutive lines (consecutive kz, so every row
// access of the block is a contiguous run of LB complex values); each line is
// cut into P partitions of M rows and thread (q, i) = (tid % LB, tid / LB)
// solves partition i of line q in registers (Eq. (20)).  Interfaces go through
// LDS.  For blocks whose lines all lie above the plan's k^2 threshold (the
// plan launches them separately) the reduced system is solved as an outer PDD of G partitions, each a group of
// P/G consecutive inner partitions: inside a group the inner interfaces are
// solved exactly (cyclic reduction, carrying the group's spike columns along),
// and the G-1 outer interfaces take the dropped 2x2 form of step 4 (for G = P
// this is the plain dropped PDD).  Otherwise the whole reduced system is
// solved exactly by cyclic reduction.  Lines flagged special (the kx = kz = 0 line, and in mixed
// precision the lowest-wavenumber set) are not written here.  The slab modes
// (YMode) split this kernel at the interface exchange: the interface rows go
// through a global buffer instead of LDS.
//
// k_special_lines: FP64 Thomas along whole lines, one block per line, with
// the gauge handling of the singular kx = kz = 0 line and its check for
// non-finite values.
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
  int G;        // outer partitions of the dropped reduced system (divides P)
};

__device__ __forceinline__ bool is_special(int kx, int kz, int nz, int skip_kx, int skip_kz) {
  const int kzs = kz < nz - kz ? kz : nz - kz;
  return (kx == 0 && kz == 0) || (kx < skip_kx && kzs < skip_kz);
}

// Dynamic LDS layout: a[nyp], c[nyp] (T; nyp = P*M rows, see k_ysolve), then
// per (partition, line):
//   interface data: x1, xm (cx), v1, vm, w1, wm (T)  -> arrays [P][LB]
//   results y1, y2 (cx) [P][LB]
//   reduced rows zrow<T> [P][LB] (16 planes), or in the dropped form zrow3<T>
//   (20 planes), where once the rows are reduced this region holds the spike results y1v, y2v, y1w, y2w (T) [P][LB] and, per
//   outer partition g and line, the group's end values xg_m, xg_1 (cx), wg_m,
//   vg_1 (T) and the outer interface results Y1, Y2 (cx)
template <typename T>
__host__ __device__ constexpr size_t ysolve_lds_bytes(int nyp, int P, int LB, bool drop) {
  return sizeof(T) * 2 * nyp +
         (sizeof(cx<T>) * 4 + sizeof(T) * 4 + (drop ? sizeof(zrow3<T>) : sizeof(zrow<T>))) * size_t(P) * LB;
}

// DROP: every line of the block lies above the plan's k^2 threshold (the
// launch covers only such blocks) and the reduced system takes the dropped
// form; otherwise it is solved exactly.  blist (nullable): the blocks of the
// launch, as indices of LB-line blocks (identity when null).
// The P partitions of M rows cover nyp = P*M >= ny rows: rows j >= ny (fewer
// than M, all in the last partition) are padding with a = c = 0 in the
// coefficient tables and a zero right-hand side.  The wall row ny-1 has c = 0,
// so they are decoupled from the line (each solves -k^2 x = 0); they are never
// loaded or stored.
// The FP32 24-row instance is held to 128 VGPRs (four waves per SIMD, two
// 512-thread blocks per CU; the dropped form then spills 16 registers): 5 %
// faster on 2048x768x2048 than at its natural 153 VGPRs and one block per CU.
// The 32-row instance spills 46 at that cap and is 20 % slower; held to 168
// (three waves per SIMD, one register spilled) instead of its natural 169 it
// is 2-3 % faster on 2048x512x1536.
// NT: the right-hand side is read and the solution written once, streamed
// (non-temporal) for large spectra in the one-pass mode: on 2048x768x2048
// (FP32, 24-row partitions) the solve takes 11.5 instead of 13.5 ms.
template <typename T, int M, int MODE, bool DROP, bool NT = false>
__global__ void __launch_bounds__(512, sizeof(T) != 4 ? 1 : M == 24 ? 4 : M == 32 ? 3 : 1)
k_ysolve(const cx<T>* fin, cx<T>* pout, const T* __restrict__ acoef,
         const T* __restrict__ ccoef, const T* __restrict__ kx2, const T* __restrict__ kz2,
         const int* __restrict__ blist, YArgs ya) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int LB = ya.LB, P = ya.P, ny = ya.ny, nyp = P * M;
  T* sa = reinterpret_cast<T*>(smem);
  T* sc = sa + nyp;
  cx<T>* s_x1 = reinterpret_cast<cx<T>*>(sc + nyp);
  cx<T>* s_xm = s_x1 + P * LB;
  cx<T>* s_y1 = s_xm + P * LB;
  cx<T>* s_y2 = s_y1 + P * LB;
  T* s_v1 = reinterpret_cast<T*>(s_y2 + P * LB);
  T* s_vm = s_v1 + P * LB;
  T* s_w1 = s_vm + P * LB;
  T* s_wm = s_w1 + P * LB;
  T* s_red = s_wm + P * LB;  // reduced rows: 16 planes (exact) or 20 (dropped) of P * LB values

  for (int j = threadIdx.x; j < nyp; j += blockDim.x) {
    sa[j] = acoef[j];
    sc[j] = ccoef[j];
  }
  const int q = threadIdx.x % LB;
  // partition of this thread (a local-mode block has threads for [pa, pb) only)
  const int i = threadIdx.x / LB + (MODE == kSlabLocal ? ya.pa : 0);
  const bool own = (MODE == kWhole) || (i >= ya.pa && i < ya.pb);
  const long blk = blist ? (long)blist[blockIdx.x] : (long)blockIdx.x;
  const long line = blk * LB + q;
  const bool ok = line < ya.nlines;
  const int kx = ok ? int(line / ya.nz) : 0;
  const int kz = ok ? int(line % ya.nz) : 1;
  const T k2 = ok ? kx2[kx] + kz2[kz] : T(1);
  const long rs = ya.nz;
  const int j0 = i * M;
  const long base = (long)kx * ny * ya.nz + kz + (long)j0 * rs;

  cx<T> d[M];
  T v0 = T(0), vM = T(0), w0 = T(0), wM = T(0);  // end values of the spike columns
#pragma unroll
  for (int s = 0; s < M; ++s) d[s] = (ok && own && j0 + s < ny) ? ld_once<NT>(&fin[base + s * rs]) : mk(T(0), T(0));
  __syncthreads();  // coefficients staged
  if (own) {
    T v[M], w[M];
    pdd_local<M, T>(sa + j0, sc + j0, k2, d, v, w);
    v0 = v[0];
    vM = v[M - 1];
    w0 = w[0];
    wM = w[M - 1];
  }

  T* ifc = static_cast<T*>(ya.iface);
  const long nl = ya.nlines;
  if (MODE == kSlabLocal) {
    if (ok) {
      T* r = ifc + (long)i * 8 * nl + line;
      r[0 * nl] = d[0].re;
      r[1 * nl] = d[0].im;
      r[2 * nl] = d[M - 1].re;
      r[3 * nl] = d[M - 1].im;
      r[4 * nl] = v0;
      r[5 * nl] = vM;
      r[6 * nl] = w0;
      r[7 * nl] = wM;
    }
    return;
  }
  const int me = i * LB + q;
  if (MODE == kWhole) {
    s_x1[me] = d[0];
    s_xm[me] = d[M - 1];
    s_v1[me] = v0;
    s_vm[me] = vM;
    s_w1[me] = w0;
    s_wm[me] = wM;
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
  __syncthreads();  // interface data staged
  const int Q = P - 1;
  cx<T> y1p = mk(T(0), T(0)), y2n = mk(T(0), T(0));  // interface values entering step 5
  if constexpr (DROP) {
    // Outer PDD over G groups of Pg inner partitions.  Group g = i / Pg,
    // inner interfaces sf..sl-1 (sf, sl: its first and last partition).
    const int Pg = P / ya.G, g = i / Pg, sf = g * Pg, sl = sf + Pg - 1;
    const bool has_if = i < sl;
    const zrow3_soa<T> s_z3{s_red, P * LB};
    // (1) inner reduced system of the group with three right-hand sides: the
    // partitions' xt (the group's solution), and for the group's spike
    // columns the first partition's v (at interface sf) and the last
    // partition's w (at interface sl - 1)
    zrow3<T> z;
    if (has_if) {
      const int nx_ = (i + 1) * LB + q;
      z.z = zrow_make(s_vm[me], s_wm[me], s_v1[nx_], s_w1[nx_], s_xm[me], s_x1[nx_]);
      z.rv0 = (i == sf) ? s_vm[me] : T(0);
      z.rv1 = T(0);
      z.rw0 = T(0);
      z.rw1 = (i + 1 == sl) ? s_w1[nx_] : T(0);
    }
    for (int st = 1; st < Pg - 1; st *= 2) {
      if (has_if) s_z3.put(me, z);
      __syncthreads();
      if (has_if) {
        const bool hl = i - st >= sf, hh = i + st < sl;
        const zrow3<T> lo = s_z3.get((hl ? i - st : i) * LB + q);
        const zrow3<T> hi = s_z3.get((hh ? i + st : i) * LB + q);
        z = zrow3_reduce(z, &lo, hl, &hi, hh);
      }
      __syncthreads();
    }
    cx<T> y1 = mk(T(0), T(0)), y2 = mk(T(0), T(0));
    T y1v = T(0), y2v = T(0), y1w = T(0), y2w = T(0);
    if (has_if) zrow3_finish(z, y1, y2, y1v, y2v, y1w, y2w);
    // the reduced rows are dead: reuse their region
    T* s_y1v = s_red;
    T* s_y2v = s_y1v + P * LB;
    T* s_y1w = s_y2v + P * LB;
    T* s_y2w = s_y1w + P * LB;
    cx<T>* s_gxm = reinterpret_cast<cx<T>*>(s_y2w + P * LB);  // [G][LB] each
    cx<T>* s_gx1 = s_gxm + ya.G * LB;
    cx<T>* s_gY1 = s_gx1 + ya.G * LB;
    cx<T>* s_gY2 = s_gY1 + ya.G * LB;
    T* s_gwm = reinterpret_cast<T*>(s_gY2 + ya.G * LB);
    T* s_gv1 = s_gwm + ya.G * LB;
    __syncthreads();
    if (has_if) {
      s_y1[me] = y1;
      s_y2[me] = y2;
      s_y1v[me] = y1v;
      s_y2v[me] = y2v;
      s_y1w[me] = y1w;
      s_y2w[me] = y2w;
    }
    __syncthreads();
    // (2) the group's end values: x and w at its last row, x and v at its first
    const int gme = g * LB + q;
    const bool prev_in = i > sf;
    const int pme = (i - 1) * LB + q;
    if (i == sl) {
      const cx<T> yp = prev_in ? s_y1[pme] : mk(T(0), T(0));
      const T ywp = prev_in ? s_y1w[pme] : T(0);
      s_gxm[gme] = s_xm[me] - yp * s_vm[me];
      s_gwm[gme] = s_wm[me] - s_vm[me] * ywp;
    }
    if (i == sf) {
      s_gx1[gme] = s_x1[me] - y2 * s_w1[me];
      s_gv1[gme] = s_v1[me] - s_w1[me] * y2v;
    }
    __syncthreads();
    // (3) step 4 on the outer interfaces (corner terms dropped)
    if (i == sl && g + 1 < ya.G) {
      cx<T> Y1, Y2;
      pdd_cramer(s_gwm[gme], s_gv1[gme + LB], s_gxm[gme], s_gx1[gme + LB], Y1, Y2);
      s_gY1[gme] = Y1;
      s_gY2[gme] = Y2;
    }
    __syncthreads();
    // (4) step 5 with effective interface values of this partition:
    // x = xt - v y1eff - w y2eff with
    //   y1eff = y1^{i-1} + ([i == sf] - y1v^{i-1}) Y1^{g-1} - y1w^{i-1} Y2^g,
    //   y2eff = y2^i - y2v^i Y1^{g-1} + ([i == sl] - y2w^i) Y2^g
    const cx<T> Y1p = g > 0 ? s_gY1[gme - LB] : mk(T(0), T(0));
    const cx<T> Y2n = g + 1 < ya.G ? s_gY2[gme] : mk(T(0), T(0));
    const cx<T> y1i = prev_in ? s_y1[pme] : mk(T(0), T(0));
    const T y1vi = prev_in ? s_y1v[pme] : T(0);
    const T y1wi = prev_in ? s_y1w[pme] : T(0);
    y1p = y1i + Y1p * ((i == sf ? T(1) : T(0)) - y1vi) - Y2n * y1wi;
    y2n = y2 - Y1p * y2v + Y2n * ((i == sl ? T(1) : T(0)) - y2w);
  } else {
    const zrow_soa<T> s_z{s_red, P * LB};
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
    cx<T> y1 = mk(T(0), T(0)), y2 = mk(T(0), T(0));
    if (i < Q) zrow_finish(z, y1, y2);
    if (i < Q) {
      s_y1[me] = y1;
      s_y2[me] = y2;
    }
    __syncthreads();
    y1p = (i > 0) ? s_y1[(i - 1) * LB + q] : mk(T(0), T(0));
    y2n = (i < Q) ? y2 : mk(T(0), T(0));
  }
  {
    T v[M], w[M];
    pdd_spikes<M, T>(sa + j0, sc + j0, k2, v, w);
    pdd_correct<M, T>(d, v, w, y1p, y2n);
  }
  if (ok && own && !is_special(kx, kz, ya.nz, ya.skip_kx, ya.skip_kz)) {
#pragma unroll
    for (int s = 0; s < M; ++s)
      if (j0 + s < ny) st_once<NT>(d[s], &pout[base + s * rs]);
  }
}

// FP64 Thomas on whole lines, one block per line.  The elimination factors
// of each listed line (den_j = b_j - a_j cp_{j-1}, cp_j = c_j / den_j, with the
// top row left out for the k^2 = 0 line) come from the plan.  The k^2 = 0
// line is made compatible (dy-weighted mean of the RHS removed), solved with
// its top unknown pinned to zero, and shifted to zero dy-weighted mean (or,
// for a correction solve given the block sums psum of the pressure it
// corrects, to the weighted mean -sum_j dy_j sum(p_j) / sum_j dy_j, the line
// value of the constant -mean_W(p)).  The
// line is staged in LDS; reads of fin all precede writes of pout, so the two
// may alias.  The sweeps follow the textbook operation order without
// contraction, like the reference definition.
template <typename T>
__global__ void __launch_bounds__(256)
k_special_lines(const cx<T>* fin, cx<T>* pout, const double* __restrict__ a,
                const double* __restrict__ den, const double* __restrict__ cpt,
                const double* __restrict__ dy, const int* __restrict__ lines, int ny, int nz,
                const double* __restrict__ psum, int nzb, int* __restrict__ numflag) {
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
  // A non-finite value anywhere in a plane of the right-hand side reaches that
  // plane's row of the kx = kz = 0 line (the sum over the plane): flag it for
  // cf_plan_numeric_status.
  if (mean_line && numflag) {
    bool bad = false;
    for (int j = tid; j < ny; j += nt) bad = bad || !__builtin_isfinite(fr[j]) || !__builtin_isfinite(fi[j]);
    if (bad) *numflag = 1;
  }
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
  if (mean_line && psum) {
    // -sum_j dy_j sum_b psum[j][b] / sum_j dy_j, summed in a fixed order
    double sp = 0.0, w = 0.0;
    for (int j = tid; j < ny; j += nt) {
      double rowsum = 0.0;
      for (int b = 0; b < nzb; ++b) rowsum += psum[(long)j * nzb + b];
      sp += dy[j] * rowsum;
      w += dy[j];
    }
    red[tid] = sp;
    red[nt + tid] = w;
    __syncthreads();
    for (int h = nt / 2; h > 0; h /= 2) {
      if (tid < h) {
        red[tid] += red[tid + h];
        red[nt + tid] += red[nt + tid + h];
      }
      __syncthreads();
    }
    orr += red[0] / red[nt];
  }
  for (int j = tid; j < ny; j += nt) pout[base + (long)j * nz] = mk(T(fr[j] - orr), T(fi[j] - oi));
}

}  // namespace cf
