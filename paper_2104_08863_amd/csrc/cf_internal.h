// Internal launch interface between the plan/ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "cf_common.h"

namespace cf {

// Transform lengths with compiled kernels: 2^a and 3*2^a from 2 to 2048.
bool fft_len_compiled(int n);

// Complex transform of the no*ni z-lines of src (line (o, i) at (o*ni + i)*n),
// written to line (i, o) of dst; src and dst must not overlap.
template <typename T>
hipError_t launch_fft_z(int n, bool inv, const cx<T>* src, cx<T>* dst, const cx<T>* tw, int no, int ni,
                        hipStream_t s);

// Forward real transform of rows of a plain array (Tin = double, stored as
// (ny, nz, nx)) into the transposed spectrum.
template <typename T>
hipError_t launch_r2c_plain(int nh, const double* f, cx<T>* spec, const cx<T>* tw, const cx<T>* twp,
                            int ny, int nz, hipStream_t s);

// Divergence of (u, v, w) times `scale`, fused into the forward real transform.
template <typename T>
hipError_t launch_r2c_div(int nh, const double* u, const double* v, const double* w,
                          const double* rdy, double rdx, double rdz, double scale, cx<T>* spec,
                          const cx<T>* tw, const cx<T>* twp, int ny, int nz, hipStream_t s);

// Forward real transform of the FP64 residual f - L_h p with f = the array f
// (kind 0), scale * D(u, v, w) (kind 1) or D(u / W, v / W, w / W) (kind 2).
// psum: one double per block, the block's FP64 sum of p; block (j, b) covers
// rows k = b*K .. b*K+K-1 of plane j and is entry j * ceil(nz/K) + b, with K =
// r2c_rows<T>(nh).  p32: p holds FP32 rows packed into its FP64 rows (as
// launch_c2r_rows32 writes them).
template <typename T, typename Ts>
hipError_t launch_r2c_resid(int kind, int nh, const double* f, const Ts* u, const Ts* v, const Ts* w,
                            double scale, const double* p, bool p32, const double* a, const double* c,
                            const double* rdy, const double* rdyc, double rdx, double rdz, cx<T>* spec,
                            const cx<T>* tw, const cx<T>* twp, int ny, int nz, double* psum, hipStream_t s);
// Rows per block of the x transforms of half-length nh.
template <typename T>
int r2c_rows(int nh);

// Divergence fused into the forward real transform, velocity type Ts.
template <typename T, typename Ts>
hipError_t launch_r2c_div_t(int nh, const Ts* u, const Ts* v, const Ts* w, const double* rdy, double rdx,
                            double rdz, double scale, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny,
                            int nz, hipStream_t s);

// Forward real transform of D(g / W) (transposed projection right-hand side).
template <typename T, typename Ts>
hipError_t launch_r2c_divw(int nh, const Ts* u, const Ts* v, const Ts* w, const double* rdy, const double* rdyc,
                           double rdx, double rdz, cx<T>* spec, const cx<T>* tw, const cx<T>* twp, int ny,
                           int nz, hipStream_t s);

template <typename T>
struct AdjGeo;

// out = s * J_R(state)^T lam (+ A + B when add), lam = c1 A + c2 B (B may be null).
template <typename T>
hipError_t launch_rhs_adjoint(const T* u, const T* v, const T* w, const T* au, const T* av, const T* aw,
                              const T* bu, const T* bv, const T* bw, T c1, T c2, const AdjGeo<T>& g, T nu, T s,
                              int add, T* gu, T* gv, T* gw, hipStream_t st);

// g* = g - W G phi.
template <typename T>
hipError_t launch_correct_w(const T* gu, const T* gv, const T* gw, T* ou, T* ov, T* ow, const double* phi,
                            const AdjGeo<T>& g, hipStream_t st);

// Inverse real transform added into p (refinement correction).  p32 (FP32
// only): p holds FP32 rows packed into its FP64 rows; the result is FP64.
template <typename T>
hipError_t launch_c2r_accum(int nh, const cx<T>* spec, double* p, const cx<T>* tw, const cx<T>* twp, int ny,
                            int nz, T scale, bool p32, hipStream_t s);

// Inverse real transform stored as FP32 into the first half of each FP64 row
// of p (a solve whose result a refinement pass corrects next).
template <typename T>
hipError_t launch_c2r_rows32(int nh, const cx<T>* spec, double* p, const cx<T>* tw, const cx<T>* twp, int ny,
                             int nz, T scale, hipStream_t s);

template <typename T>
hipError_t launch_c2r_plain(int nh, const cx<T>* spec, double* p, const cx<T>* tw, const cx<T>* twp,
                            int ny, int nz, T scale, hipStream_t s);

struct YLaunch {
  int ny, nz, nkx, P, M;
  int LB;  // lines per block (threads per block = LB * P <= 512)
  long nlines;
  int skip_kx, skip_kz;
  int mode = 0;            // YMode: whole lines, or one y-slab's local / finishing pass
  int pa = 0, pb = 0;      // slab modes: partitions [pa, pb)
  void* iface = nullptr;   // slab modes: interface rows [P][8][nlines] of the plan's precision
  int G = 0;               // outer partitions of the dropped reduced system (0: P)
  // LB-line blocks solved with the exact (blocks_exact: null = all blocks) and
  // the dropped reduced system (blocks_drop: null = none); device arrays
  const int* blocks_exact = nullptr;
  long n_exact = 0;
  const int* blocks_drop = nullptr;
  long n_drop = 0;
};

// Default lines per block of the partitioned solve for P partitions.
int ysolve_default_lb(int P, int M);
// Dynamic LDS of one partitioned-solve block.
size_t ysolve_lds_needed(int nyp, int P, int LB, bool fp64);

template <typename T>
hipError_t launch_ysolve(const YLaunch& y, const cx<T>* fin, cx<T>* pout, const T* a, const T* c,
                         const T* kx2, const T* kz2, hipStream_t s);

// Whole-line FP64 Thomas on the listed lines of layout B, with per-line
// elimination factors den, cp ([n_lines][ny]) prepared by the plan.  psum
// (nullable): [ny][nzb] block sums of a pressure p; when given, the kx = kz = 0
// line is gauged to the dy-weighted mean -mean_W(p) * nx * nz instead of 0, so
// that adding the solution to p makes mean_W vanish.  numflag (nullable): set
// to 1 when the kx = kz = 0 line of fin holds a non-finite value.
template <typename T>
hipError_t launch_special_lines(const cx<T>* fin, cx<T>* pout, const double* a, const double* den,
                                const double* cp, const double* dy, const int* lines, int n_lines,
                                int ny, int nz, const double* psum, int nzb, int* numflag, hipStream_t s);

bool ysolve_m_compiled(int m, bool fp64);

template <typename T>
struct Geo;

// RK2 stages of the momentum equation: stage 1 out = f + dt R(f); stage 2
// out = (f0 + f)/2 + dt/2 R(f).
template <typename T>
hipError_t launch_rk_stage(int stage, const T* u, const T* v, const T* w, const T* u0, const T* v0,
                           const T* w0, T* uo, T* vo, T* wo, const Geo<T>& g, T dt, T nu, T fx,
                           hipStream_t s);

// u1 = us - dt G p in place.
// Both RK2 stages in one pass: uo = (u + ub)/2 + dt/2 R(ub), ub = u + dt R(u).
template <typename T>
hipError_t launch_rk2_fused(const T* u, const T* v, const T* w, T* uo, T* vo, T* wo, const Geo<T>& g, T dt, T nu,
                            T fx, hipStream_t s);
// Per-plane means of u, v, w and their squares into st (ny, 6), or added to it.
template <typename T>
hipError_t launch_plane_stats(const T* u, const T* v, const T* w, double* st, const Geo<T>& g, int accumulate,
                              hipStream_t s);
// The correction of launch_correct fused with the plane statistics of the
// corrected fields into st (ny, 6) (or added to it); part: scratch of
// ny * nch * 6 doubles, nch = correct_stats_chunks(nx, ny, nz).
int correct_stats_chunks(int nx, int ny, int nz);
template <typename T>
hipError_t launch_correct_stats(T* u, T* v, T* w, const double* p, const Geo<T>& g, T dt, double* part, int nch,
                                double* st, int accumulate, hipStream_t s);
// Uniform-y wall-normal solve by a DCT-II / DCT-III pair along y (N-point
// FFTs, N = ny even); in place allowed.  tw: FFT twiddles of length ny;
// wq: exp(-i pi m / 2ny), m < ny; lam: -(2 sin(pi m / 2ny) / dy)^2, m <= ny.
bool ydct_len_compiled(int n);
template <typename T>
hipError_t launch_ydct(const cx<T>* fin, cx<T>* pout, const cx<T>* tw, const cx<T>* wq, const T* lam,
                       const T* kx2, const T* kz2, int ny, int nz, int nkx, hipStream_t s);
template <typename T>
hipError_t launch_correct(T* u, T* v, T* w, const double* p, const Geo<T>& g, T dt, hipStream_t s);

// Plain divergence (test hook): f = scale * D(u, v, w).
hipError_t launch_divergence(const double* u, const double* v, const double* w, double* f,
                             const double* rdy, double rdx, double rdz, double scale, int nx,
                             int ny, int nz, hipStream_t s);

}  // namespace cf
