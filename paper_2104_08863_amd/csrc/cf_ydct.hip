// Wall-normal solve for uniform y grids by a transform along y (the fully
// spectral variant that Section 2.1 notes for uniform spacing).
//
// With uniform spacing the staggered second difference with no flux through
// the walls is diagonalised by the DCT-II, F_m = sum_j f_j cos(pi m (2j+1) / 2N)
// (N = ny), with eigenvalues -(2 sin(pi m / 2N) / dy)^2; so each (kx, kz) line
// is transformed, divided by mu_m = -(2 sin(pi m / 2N) / dy)^2 - k^2 and
// transformed back with the DCT-III, p_j = P_0 / N + (2/N) sum_{m>0} P_m
// cos(pi m (2j+1) / 2N).  mu_0 = 0 only on the kx = kz = 0 line: its P_0 is set
// to 0 (zero-mean gauge; the mean of f is dropped, as in the tridiagonal path).
//
// Both transforms are N-point complex FFTs (Makhoul's reordering), which holds
// for complex lines because every step is complex-linear:
//   forward   v_n = f_2n, v_(N-1-n) = f_(2n+1);  V = FFT(v);
//             F_m = (w_m V_m + conj(w_m) V_(N-m)) / 2,   w_m = exp(-i pi m / 2N)
//   inverse   Q_m = conj(w_m) (P_m - i P_(N-m)),  P_N = 0;  q = IFFT(Q) / N;
//             p_2n = q_n, p_(2n+1) = q_(N-1-n).
// A thread owns the pair (m, N-m), which is all that the steps between the
// two FFTs couple.
#include "cf_fft_kernels.h"
#include "cf_internal.h"

namespace cf {

template <typename T, int N>
struct YdctCfg {
  // lines per block: about 64 threads' worth of lines, 8 to 64 (8 measured
  // fastest of 4, 8, 16 for N = 128, 256 in FP64: more blocks per CU), fewer
  // where LDS would exceed 72 KB
  static constexpr int pick(int l) {
    return (l > 1 && (l * lpad_len(N) * int(sizeof(cx<T>)) > 73728 || l * FftT<N>::TPL > 1024)) ? pick(l / 2) : l;
  }
  static constexpr int want = (64 / FftT<N>::TPL < 8) ? 8 : (64 / FftT<N>::TPL > 64 ? 64 : 64 / FftT<N>::TPL);
  static constexpr int LB = pick(want);
  static constexpr int THREADS = LB * FftT<N>::TPL;
};

// LDS slot of row j of a line in the reordered sequence v.
template <int N>
__device__ __forceinline__ int mk_pos(int j) {
  return (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
}

// Lines (kx, kz0 .. kz0+LB-1) of layout B (nkx, ny, nz) per block; in place
// allowed (a block reads its lines completely before writing them).
template <typename T, int N>
__global__ void __launch_bounds__((YdctCfg<T, N>::THREADS))
k_ydct(const cx<T>* fin, cx<T>* pout, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ wq,
       const T* __restrict__ lam, const T* __restrict__ kx2, const T* __restrict__ kz2, int nz) {
  using F = FftT<N>;
  constexpr int LB = YdctCfg<T, N>::LB;
  constexpr int TH = YdctCfg<T, N>::THREADS;
  constexpr int S = lpad_len(N);
  constexpr int NPAIR = N / 2 + 1;  // pairs (m, N-m), m = 0..N/2
  __shared__ cx<T> lds[LB * S];
  const int nzb = (nz + LB - 1) / LB;
  const int kx = blockIdx.x / nzb;
  const int kz0 = (blockIdx.x % nzb) * LB;
  const long base = (long)kx * N * nz + kz0;
  {
    // all loads of the thread in flight before the first LDS store
    constexpr int PT = N * LB / TH;
    cx<T> ld[PT];
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int idx = threadIdx.x + r * TH, q = idx % LB, j = idx / LB;
      ld[r] = (kz0 + q < nz) ? fin[base + (long)j * nz + q] : mk(T(0), T(0));
    }
#pragma unroll
    for (int r = 0; r < PT; ++r) {
      const int idx = threadIdx.x + r * TH, q = idx % LB, j = idx / LB;
      lds[q * S + lpad(mk_pos<N>(j))] = ld[r];
    }
  }
  __syncthreads();
  const int tl = threadIdx.x % F::TPL, qq = threadIdx.x / F::TPL;
  cx<T>* sl = lds + qq * S;
  cx<T> x[F::E];
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) x[q * F::R0 + r] = sl[lpad(st_in(N, F::R0, b, r))];
  }
  fft_passes<N, false, T, 0>(x, tl, sl, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::E / F::RL; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::RL; ++r) sl[lpad(b + r * (N / F::RL))] = x[q * F::RL + r];
  }
  __syncthreads();
  // pairs (m, N-m): DCT-II coefficients, division, DCT-III input
  const int kz = kz0 + qq;
  const T k2 = (kz < nz) ? kx2[kx] + kz2[kz] : T(1);
  const T rn = T(1) / T(N);
  cx<T> qa[(NPAIR + F::TPL - 1) / F::TPL], qb[(NPAIR + F::TPL - 1) / F::TPL];
#pragma unroll
  for (int c = 0; c < (NPAIR + F::TPL - 1) / F::TPL; ++c) {
    const int m = tl + c * F::TPL;
    if (m < NPAIR) {
      const int mb = (N - m) % N;  // partner index (m = 0 and m = N/2 pair with themselves)
      const cx<T> va = sl[lpad(m)], vb = sl[lpad(mb)];
      const cx<T> wa = wq[m], wb = wq[mb];
      const cx<T> fa = (cmul(wa, va) + cmul(conj(wa), vb)) * T(0.5);
      const cx<T> fb = (cmul(wb, vb) + cmul(conj(wb), va)) * T(0.5);
      const T ma = lam[m] - k2, mbv = lam[m == 0 ? 0 : N - m] - k2;
      const cx<T> pa = (ma == T(0)) ? mk(T(0), T(0)) : fa * (rn / ma);
      const cx<T> pb = (mbv == T(0)) ? mk(T(0), T(0)) : fb * (rn / mbv);
      // Q_m = conj(w_m) (P_m - i P_(N-m)); P_N = 0 for m = 0
      const cx<T> pm = (m == 0) ? mk(T(0), T(0)) : pb;
      qa[c] = cmul(conj(wa), mk(pa.re + pm.im, pa.im - pm.re));
      qb[c] = cmul(conj(wb), mk(pb.re + pa.im, pb.im - pa.re));
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < (NPAIR + F::TPL - 1) / F::TPL; ++c) {
    const int m = tl + c * F::TPL;
    if (m < NPAIR) {
      sl[lpad(m)] = qa[c];
      if (m != 0 && m != N / 2) sl[lpad(N - m)] = qb[c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) x[q * F::R0 + r] = sl[lpad(st_in(N, F::R0, b, r))];
  }
  fft_passes<N, true, T, 0>(x, tl, sl, tw);
  __syncthreads();
  // q_n -> rows: p_2n = q_n, p_(2n+1) = q_(N-1-n), i.e. q_m lands on row
  // 2m (m < N/2) or 2(N-1-m)+1
#pragma unroll
  for (int q = 0; q < F::E / F::RL; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::RL; ++r) {
      const int m = b + r * (N / F::RL);
      const int row = (m < N / 2) ? 2 * m : 2 * (N - 1 - m) + 1;
      sl[lpad(row)] = x[q * F::RL + r];
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int idx = threadIdx.x; idx < N * LB; idx += TH) {
    const int q = idx % LB, j = idx / LB;
    if (kz0 + q < nz) pout[base + (long)j * nz + q] = lds[q * S + lpad(j)];
  }
}

template <typename T, int N>
static hipError_t ydct_n(const cx<T>* fin, cx<T>* pout, const cx<T>* tw, const cx<T>* wq, const T* lam,
                         const T* kx2, const T* kz2, int nz, int nkx, hipStream_t s) {
  using C = YdctCfg<T, N>;
  const long blocks = (long)nkx * ((nz + C::LB - 1) / C::LB);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_ydct<T, N>), dim3(blocks), dim3(C::THREADS), 0, s, fin, pout, tw, wq, lam, kx2, kz2, nz);
  return hipGetLastError();
}

#define CF_FOR_EACH_YDCT_LEN(X)                                                                         \
  X(2) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) \
  X(1024) X(1536) X(2048)

bool ydct_len_compiled(int n) {
  switch (n) {
#define CF_CASE(N) case N:
    CF_FOR_EACH_YDCT_LEN(CF_CASE)
#undef CF_CASE
    return true;
    default:
      return false;
  }
}

template <typename T>
hipError_t launch_ydct(const cx<T>* fin, cx<T>* pout, const cx<T>* tw, const cx<T>* wq, const T* lam,
                       const T* kx2, const T* kz2, int ny, int nz, int nkx, hipStream_t s) {
  switch (ny) {
#define CF_CASE(N) \
  case N:          \
    return ydct_n<T, N>(fin, pout, tw, wq, lam, kx2, kz2, nz, nkx, s);
    CF_FOR_EACH_YDCT_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_ydct<double>(const cx<double>*, cx<double>*, const cx<double>*, const cx<double>*,
                                        const double*, const double*, const double*, int, int, int, hipStream_t);

}  // namespace cf
