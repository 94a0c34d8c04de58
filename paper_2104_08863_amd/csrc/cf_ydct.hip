// Wall-normal solve for uniform y grids by a transform along y (the fully
// spectral variant that Section 2.1 notes for uniform spacing).
//
// With uniform spacing the staggered second difference with no flux through
// the walls, on ny points, is the periodic second difference on the 2ny-point
// even extension (p_{2ny-1-j} = p_j): both give p_1 - p_0 at the bottom row.
// So each (kx, kz) line is solved by the FFT of its even extension (a DCT-II of
// the line, up to twiddles), a division by the periodic eigenvalue
//   mu_m = -(2 sin(pi m / 2ny) / dy)^2 - k^2,      mu_m = mu_{2ny-m},
// and the inverse FFT scaled by 1/(2ny), keeping rows 0..ny-1.  The spectrum of
// an even extension is again even, so the inverse is again one.  mu_0 = 0 only
// on the kx = kz = 0 line: its m = 0 coefficient is set to 0 (zero-mean gauge,
// and the mean of f is dropped, as in the tridiagonal path).
#include "cf_fft_kernels.h"
#include "cf_internal.h"

namespace cf {

template <typename T, int N2>
struct YdctCfg {
  // lines per block: enough threads per block, LDS within 72 KB
  static constexpr int pick(int l) {
    return (l > 1 && (l * lpad_len(N2) * int(sizeof(cx<T>)) > 73728 || l * FftT<N2>::TPL > 1024)) ? pick(l / 2) : l;
  }
  static constexpr int want = (256 / FftT<N2>::TPL < 8) ? 8 : (256 / FftT<N2>::TPL > 64 ? 64 : 256 / FftT<N2>::TPL);
  static constexpr int LB = pick(want);
  static constexpr int THREADS = LB * FftT<N2>::TPL;
};

// Lines (kx, kz0 .. kz0+LB-1) of layout B (nkx, ny, nz) per block; in place
// allowed (a block reads its lines completely before writing them).
template <typename T, int N2>
__global__ void __launch_bounds__((YdctCfg<T, N2>::THREADS))
k_ydct(const cx<T>* fin, cx<T>* pout, const cx<T>* __restrict__ tw, const T* __restrict__ lam,
       const T* __restrict__ kx2, const T* __restrict__ kz2, int ny, int nz) {
  using F = FftT<N2>;
  constexpr int LB = YdctCfg<T, N2>::LB;
  constexpr int TH = YdctCfg<T, N2>::THREADS;
  constexpr int S = lpad_len(N2);
  __shared__ cx<T> lds[LB * S];
  const int nzb = (nz + LB - 1) / LB;
  const int kx = blockIdx.x / nzb;
  const int kz0 = (blockIdx.x % nzb) * LB;
  const long base = (long)kx * ny * nz + kz0;
  // the lines and their mirror images, read along kz (coalesced)
  for (int idx = threadIdx.x; idx < ny * LB; idx += TH) {
    const int q = idx % LB, j = idx / LB;
    const cx<T> val = (kz0 + q < nz) ? fin[base + (long)j * nz + q] : mk(T(0), T(0));
    lds[q * S + lpad(j)] = val;
    lds[q * S + lpad(N2 - 1 - j)] = val;
  }
  __syncthreads();
  const int tl = threadIdx.x % F::TPL, qq = threadIdx.x / F::TPL;
  cx<T>* sl = lds + qq * S;
  cx<T> x[F::E];
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) x[q * F::R0 + r] = sl[lpad(st_in(N2, F::R0, b, r))];
  }
  fft_passes<N2, false, T, 0>(x, tl, sl, tw);
  // divide by the eigenvalue; the inverse transform's 1/N2 folded in
  const int kz = kz0 + qq;
  const T k2 = (kz < nz) ? kx2[kx] + kz2[kz] : T(1);
#pragma unroll
  for (int q = 0; q < F::E / F::RL; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::RL; ++r) {
      const int m = b + r * (N2 / F::RL);
      const T mu = lam[m <= N2 / 2 ? m : N2 - m] - k2;
      const T sc = (mu == T(0)) ? T(0) : T(1) / (mu * T(N2));
      x[q * F::RL + r] = x[q * F::RL + r] * sc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::E / F::RL; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::RL; ++r) sl[lpad(b + r * (N2 / F::RL))] = x[q * F::RL + r];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::E / F::R0; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::R0; ++r) x[q * F::R0 + r] = sl[lpad(st_in(N2, F::R0, b, r))];
  }
  fft_passes<N2, true, T, 0>(x, tl, sl, tw);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < F::E / F::RL; ++q) {
    const int b = tl + q * F::TPL;
#pragma unroll
    for (int r = 0; r < F::RL; ++r) sl[lpad(b + r * (N2 / F::RL))] = x[q * F::RL + r];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < ny * LB; idx += TH) {
    const int q = idx % LB, j = idx / LB;
    if (kz0 + q < nz) pout[base + (long)j * nz + q] = lds[q * S + lpad(j)];
  }
}

template <typename T, int N2>
static hipError_t ydct_n(const cx<T>* fin, cx<T>* pout, const cx<T>* tw, const T* lam, const T* kx2, const T* kz2,
                         int ny, int nz, int nkx, hipStream_t s) {
  using C = YdctCfg<T, N2>;
  const long blocks = (long)nkx * ((nz + C::LB - 1) / C::LB);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_ydct<T, N2>), dim3(blocks), dim3(C::THREADS), 0, s, fin, pout, tw, lam, kx2, kz2, ny, nz);
  return hipGetLastError();
}

bool ydct_len_compiled(int n2) {
  switch (n2) {
    case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128:
    case 192: case 256: case 384: case 512: case 768: case 1024: case 1536: case 2048:
      return true;
    default:
      return false;
  }
}

template <typename T>
hipError_t launch_ydct(const cx<T>* fin, cx<T>* pout, const cx<T>* tw, const T* lam, const T* kx2, const T* kz2,
                       int ny, int nz, int nkx, hipStream_t s) {
  switch (2 * ny) {
#define CF_CASE(N) \
  case N:          \
    return ydct_n<T, N>(fin, pout, tw, lam, kx2, kz2, ny, nz, nkx, s);
    CF_CASE(4) CF_CASE(6) CF_CASE(8) CF_CASE(12) CF_CASE(16) CF_CASE(24) CF_CASE(32) CF_CASE(48) CF_CASE(64)
    CF_CASE(96) CF_CASE(128) CF_CASE(192) CF_CASE(256) CF_CASE(384) CF_CASE(512) CF_CASE(768) CF_CASE(1024)
    CF_CASE(1536) CF_CASE(2048)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_ydct<double>(const cx<double>*, cx<double>*, const cx<double>*, const double*,
                                        const double*, const double*, int, int, int, hipStream_t);

}  // namespace cf
