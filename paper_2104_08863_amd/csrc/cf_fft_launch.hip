// Length dispatch and launch of the periodic-direction transforms.
#include "cf_fft_kernels.h"
#include "cf_internal.h"

namespace cf {

#define CF_FOR_EACH_LEN(X) \
  X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
  X(384) X(512) X(768) X(1024) X(1536) X(2048)

bool fft_len_compiled(int n) {
  switch (n) {
#define CF_CASE(N) case N:
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    return true;
    default:
      return false;
  }
}

template <typename T, int N>
static hipError_t fft_z_n(bool inv, const cx<T>* src, cx<T>* dst, const cx<T>* tw, int no, int ni,
                          hipStream_t s) {
  using C = ZCfg<T, N>;
  const long blocks = ((long)no * ni + C::LPB - 1) / C::LPB;
  if (blocks <= 0) return hipSuccess;
  const bool nt = (long)no * ni * N * (long)sizeof(cx<T>) >= kStreamBytes;
  if (inv && nt)
    hipLaunchKernelGGL((k_fft_z<T, N, true, true>), dim3(blocks), dim3(C::THREADS), 0, s, src, dst, tw, no, ni);
  else if (inv)
    hipLaunchKernelGGL((k_fft_z<T, N, true, false>), dim3(blocks), dim3(C::THREADS), 0, s, src, dst, tw, no, ni);
  else if (nt)
    hipLaunchKernelGGL((k_fft_z<T, N, false, true>), dim3(blocks), dim3(C::THREADS), 0, s, src, dst, tw, no, ni);
  else
    hipLaunchKernelGGL((k_fft_z<T, N, false, false>), dim3(blocks), dim3(C::THREADS), 0, s, src, dst, tw, no, ni);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_z(int n, bool inv, const cx<T>* src, cx<T>* dst, const cx<T>* tw, int no, int ni,
                        hipStream_t s) {
  switch (n) {
#define CF_CASE(N) \
  case N:          \
    return fft_z_n<T, N>(inv, src, dst, tw, no, ni, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, int NH, typename Src>
static hipError_t r2c_n(Src src, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny, int nz,
                        hipStream_t s) {
  using C = XCfg<T, NH>;
  const long blocks = (long)ny * ((nz + C::K - 1) / C::K);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_r2c_x<T, NH, Src>), dim3(blocks), dim3(C::THREADS), 0, s, src, spec, tw, twp,
                     ny, nz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_r2c_plain(int nh, const double* f, cx<T>* spec, const cx<T>* tw, const cx<T>* twp,
                            int ny, int nz, hipStream_t s) {
  SrcPlain<T, double> src{f, 2 * nh, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return r2c_n<T, N>(src, spec, tw, twp, ny, nz, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_r2c_div(int nh, const double* u, const double* v, const double* w, const double* rdy,
                          double rdx, double rdz, double scale, cx<T>* spec, const cx<T>* tw,
                          const cx<T>* twp, int ny, int nz, hipStream_t s) {
  SrcDiv<T, double> src{u, v, w, rdy, rdx, rdz, scale, 2 * nh, ny, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return r2c_n<T, N>(src, spec, tw, twp, ny, nz, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
int r2c_rows(int nh) {
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return XCfg<T, N>::K;
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return 0;
  }
}
template int r2c_rows<double>(int);
template int r2c_rows<float>(int);

template <typename T, typename Tp, typename In>
static hipError_t r2c_resid_n(int nh, In in, const double* p, const double* a, const double* c, double rdx,
                              double rdz, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny, int nz,
                              double* psum, hipStream_t s) {
  SrcResidual<T, In, Tp> src{in, p, a, c, rdx * rdx, rdz * rdz, 2 * nh, ny, nz, psum};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return r2c_n<T, N>(src, spec, tw, twp, ny, nz, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, typename In>
static hipError_t r2c_resid_any(int nh, In in, const double* p, bool p32, const double* a, const double* c,
                                double rdx, double rdz, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny,
                                int nz, double* psum, hipStream_t s) {
  if (p32) return r2c_resid_n<T, float>(nh, in, p, a, c, rdx, rdz, spec, tw, twp, ny, nz, psum, s);
  return r2c_resid_n<T, double>(nh, in, p, a, c, rdx, rdz, spec, tw, twp, ny, nz, psum, s);
}

template <typename T, typename Ts>
hipError_t launch_r2c_resid(int kind, int nh, const double* f, const Ts* u, const Ts* v, const Ts* w,
                            double scale, const double* p, bool p32, const double* a, const double* c,
                            const double* rdy, const double* rdyc, double rdx, double rdz, cx<T>* spec,
                            const cx<T>* tw, const cx<T>* twp, int ny, int nz, double* psum, hipStream_t s) {
  const int nx = 2 * nh;
  if (kind == 0)
    return r2c_resid_any<T>(nh, SrcPlain<double, double>{f, nx, nz}, p, p32, a, c, rdx, rdz, spec, tw, twp, ny, nz,
                            psum, s);
  if (kind == 1)
    return r2c_resid_any<T>(nh, SrcDiv<double, Ts>{u, v, w, rdy, rdx, rdz, scale, nx, ny, nz}, p, p32, a, c, rdx,
                            rdz, spec, tw, twp, ny, nz, psum, s);
  return r2c_resid_any<T>(nh, SrcDivW<double, Ts>{u, v, w, rdy, rdyc, rdx, rdz, nx, ny, nz}, p, p32, a, c, rdx,
                          rdz, spec, tw, twp, ny, nz, psum, s);
}

template <typename T, typename Ts>
hipError_t launch_r2c_div_t(int nh, const Ts* u, const Ts* v, const Ts* w, const double* rdy, double rdx,
                            double rdz, double scale, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny,
                            int nz, hipStream_t s) {
  SrcDiv<T, Ts> src{u, v, w, rdy, rdx, rdz, scale, 2 * nh, ny, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return r2c_n<T, N>(src, spec, tw, twp, ny, nz, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, int NH, typename Dst>
static hipError_t c2r_n(const cx<T>* spec, Dst dst, const cx<T>* tw, const cx<T>* twp, int ny, int nz,
                        T scale, hipStream_t s) {
  using C = XCfg<T, NH>;
  const long blocks = (long)ny * ((nz + C::K - 1) / C::K);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_c2r_x<T, NH, Dst>), dim3(blocks), dim3(C::THREADS), 0, s, spec, dst, tw, twp,
                     ny, nz, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_c2r_plain(int nh, const cx<T>* spec, double* p, const cx<T>* tw, const cx<T>* twp,
                            int ny, int nz, T scale, hipStream_t s) {
  DstPlain<T, double> dst{p, 2 * nh, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return c2r_n<T, N>(spec, dst, tw, twp, ny, nz, scale, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, typename Ts>
hipError_t launch_r2c_divw(int nh, const Ts* u, const Ts* v, const Ts* w, const double* rdy, const double* rdyc,
                           double rdx, double rdz, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny,
                           int nz, hipStream_t s) {
  SrcDivW<T, Ts> src{u, v, w, rdy, rdyc, rdx, rdz, 2 * nh, ny, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return r2c_n<T, N>(src, spec, tw, twp, ny, nz, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}
template hipError_t launch_r2c_divw<double, double>(int, const double*, const double*, const double*,
                                                    const double*, const double*, double, double, cx<double>*,
                                                    const cx<double>*, const cx<double>*, int, int, hipStream_t);

template <typename T>
hipError_t launch_c2r_accum(int nh, const cx<T>* spec, double* p, const cx<T>* tw, const cx<T>* twp, int ny,
                            int nz, T scale, bool p32, hipStream_t s) {
  if (p32) {
    if constexpr (std::is_same<T, float>::value) {
      DstAccumRows32 dst{p, 2 * nh, nz};
      switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return c2r_n<T, N>(spec, dst, tw, twp, ny, nz, scale, s);
        CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
        default:
          return hipErrorInvalidValue;
      }
    }
    return hipErrorInvalidValue;
  }
  DstAccum<T> dst{p, 2 * nh, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return c2r_n<T, N>(spec, dst, tw, twp, ny, nz, scale, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_c2r_rows32(int nh, const cx<T>* spec, double* p, const cx<T>* tw, const cx<T>* twp, int ny,
                             int nz, T scale, hipStream_t s) {
  DstRows32<T> dst{p, 2 * nh, nz};
  switch (nh) {
#define CF_CASE(N) \
  case N:          \
    return c2r_n<T, N>(spec, dst, tw, twp, ny, nz, scale, s);
    CF_FOR_EACH_LEN(CF_CASE)
#undef CF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_r2c_resid<float, float>(int, int, const double*, const float*, const float*,
                                                   const float*, double, const double*, bool, const double*,
                                                   const double*, const double*, const double*, double, double,
                                                   cx<float>*, const cx<float>*, const cx<float>*, int, int,
                                                   double*, hipStream_t);
template hipError_t launch_r2c_divw<float, float>(int, const float*, const float*, const float*, const double*,
                                                  const double*, double, double, cx<float>*, const cx<float>*,
                                                  const cx<float>*, int, int, hipStream_t);
template hipError_t launch_r2c_div_t<float, float>(int, const float*, const float*, const float*,
                                                   const double*, double, double, double, cx<float>*,
                                                   const cx<float>*, const cx<float>*, int, int, hipStream_t);
template hipError_t launch_c2r_accum<float>(int, const cx<float>*, double*, const cx<float>*,
                                            const cx<float>*, int, int, float, bool, hipStream_t);
template hipError_t launch_c2r_rows32<float>(int, const cx<float>*, double*, const cx<float>*,
                                             const cx<float>*, int, int, float, hipStream_t);

#define CF_INST(T)                                                                                   \
  template hipError_t launch_fft_z<T>(int, bool, const cx<T>*, cx<T>*, const cx<T>*, int, int, hipStream_t); \
  template hipError_t launch_r2c_plain<T>(int, const double*, cx<T>*, const cx<T>*, const cx<T>*, int, \
                                          int, hipStream_t);                                         \
  template hipError_t launch_c2r_plain<T>(int, const cx<T>*, double*, const cx<T>*, const cx<T>*, int, \
                                          int, T, hipStream_t);                                      \
  template hipError_t launch_r2c_div<T>(int, const double*, const double*, const double*, const double*, \
                                        double, double, double, cx<T>*, const cx<T>*, const cx<T>*,  \
                                        int, int, hipStream_t);
CF_INST(double)
CF_INST(float)
#undef CF_INST

}  // namespace cf
