// Plan creation and the C ABI of chanflow (see include/chanflow.h).
//
// The plan turns the problem statement of Section 2 into device tables: the
// wall-normal coefficients of the staggered Laplacian, the modified
// wavenumbers of Eq. (9) (eigenvalues of the periodic second difference), the
// twiddle tables of the transforms, the PDD partitioning of Section 2.2 with
// the k^2 threshold above which the corner terms of Eq. (21) are negligible,
// and the list of lines solved by whole-line FP64 Thomas.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/chanflow.h"
#include "cf_fft.h"
#include "cf_internal.h"
#include "cf_pdd.h"
#include "cf_adjoint_kernels.h"
#include "cf_step_kernels.h"

using cf::cx;

// Interface rows of cf_solve_spectral_slabs_noalloc: a fixed device array (each
// device the library runs on holds its own copy until the process ends), so
// that entry point allocates nothing.  Host code must not pass this name to a
// kernel or a copy: it is a host-side stand-in; the device address of each
// device's copy is taken once per device at plan creation (scratch_ptr below).
constexpr size_t kSlabScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kSlabScratchBytes];

namespace {

thread_local std::string g_last_error;

cf_status fail(cf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

cf_status dev_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return CF_ERR_DEVICE;
}

#define CF_HIP_RET(x)                              \
  do {                                             \
    hipError_t _e = (x);                           \
    if (_e != hipSuccess) return dev_fail(_e, #x); \
  } while (0)

// exp(-2 pi i m / n) from the exactly reduced ratio m/n.
cx<double> unit_root(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long double t = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
  return cf::mk((double)cosl(t), (double)-sinl(t));
}

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

// Device address of `scratch` per device, looked up with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

struct cf_plan {
  int nx, ny, nz, nkx, nh;
  double lx, lz, dx, dz;
  cf_options opt;
  int device;
  int P, M;
  int LB;  // lines per block of the partitioned solve
  int G;   // outer partitions of the dropped reduced system
  double k2drop;
  long long n_drop;     // lines above the drop threshold
  long long n_dropped;  // lines in blocks wholly above it (dropped by the kernel)
  // LB-line blocks of the partitioned solve taking the exact and the dropped
  // reduced system (host lists; the device copy d_blocks holds the exact list
  // then the dropped one)
  std::vector<int> blocks_exact, blocks_drop;
  int* d_blocks = nullptr;
  // partition counts and block shapes timed at creation (CF_PLAN_TUNE_PARTS)
  struct TuneRow {
    int P, LB;
    double us;
  };
  std::vector<TuneRow> tune;
  std::vector<double> yf, dy, dyc, a, c, kx2, kz2;
  std::vector<int> special;
  std::vector<DevBuf> allocs;
  size_t bytes = 0;
  // device tables (FP64 and FP32 copies)
  double *d_a = nullptr, *d_c = nullptr, *d_dy = nullptr, *d_rdy = nullptr, *d_kx2 = nullptr,
         *d_kz2 = nullptr, *d_rdyc = nullptr, *d_wl = nullptr, *d_wu = nullptr;
  float *s_rdy = nullptr, *s_rdyc = nullptr, *s_wl = nullptr, *s_wu = nullptr;
  float *s_a = nullptr, *s_c = nullptr, *s_kx2 = nullptr, *s_kz2 = nullptr;
  cx<double>*tw_z64 = nullptr, *tw_x64 = nullptr, *twp64 = nullptr;
  // uniform-y transform solve (CF_PLAN_Y_DCT): FFT twiddles of length ny, the
  // DCT twiddles exp(-i pi m / 2ny) and the y eigenvalues
  // -(2 sin(pi m / 2ny) / dy)^2, m = 0..ny
  cx<double>* tw_y64 = nullptr;
  cx<double>* d_wqy = nullptr;
  double* d_lamy = nullptr;
  cx<float>*tw_z32 = nullptr, *tw_x32 = nullptr, *twp32 = nullptr;
  int* d_special = nullptr;
  double* d_special_den = nullptr;  // [n_special][ny] elimination pivots
  double* d_special_cp = nullptr;   // [n_special][ny] eliminated upper coefficients
  // spectral workspaces of the bulk precision: layout A (ny, nkx, nz) on the
  // x side, layout B (nkx, ny, nz) on the wall-normal side
  void* specA = nullptr;
  void* specB = nullptr;
  // projection-step workspace: RK stage-1 fields (state precision) and pressure
  void *ub = nullptr, *vb = nullptr, *wb = nullptr;
  double* pws = nullptr;
  // step plans: per-chunk sums of the fused correction + plane statistics
  double* d_stat_part = nullptr;
  int stat_nch = 1;
  double* fws = nullptr;  // mixed precision: copy of f when p aliases it
  // mixed precision: FP64 block sums of p from the residual transform (gauge
  // of the correction solves), [ny][psum_nzb]
  double* d_psum = nullptr;
  int psum_nzb = 0;
  // set by the kx = kz = 0 line solve when its right-hand side holds a
  // non-finite value; read and cleared by cf_plan_numeric_status
  int* d_numflag = nullptr;
  // adjoint workspace: projected gradient g* and gb (state precision)
  void *gsu = nullptr, *gsv = nullptr, *gsw = nullptr, *gbu = nullptr, *gbv = nullptr, *gbw = nullptr;
  double *d_dyc = nullptr;
  float *s_dy = nullptr, *s_dyc = nullptr;
  cf::AdjGeo<double> a64{};
  cf::AdjGeo<float> a32{};
  cf::Geo<double> g64{};
  cf::Geo<float> g32{};

  bool mixed() const { return opt.precision == CF_MIXED; }
  // side stream for the whole-line solves, which overlap the PDD kernel
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // stream on which step sequences are recorded into HIP graphs and replayed
  // (capture needs a stream other than the legacy default one)
  hipStream_t gstream = nullptr;
  hipEvent_t ev_gin = nullptr, ev_gout = nullptr;
  // recorded loop steps, reused while the arrays and parameters repeat
  struct GraphEntry {
    void* a[3];
    void* b[3];
    double* p;
    double* acc;
    double dt, nu, fx;
    hipGraphExec_t exec;
    unsigned long long last_use;
  };
  std::vector<GraphEntry> graphs;
  unsigned long long graph_clock = 0;
  // per-kernel event timing
  bool timing = false;
  std::vector<hipEvent_t> events;  // created on demand, reused after each harvest
  size_t ev_used = 0;
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double acc_ms[CF_K_COUNT] = {0};
  long long acc_n[CF_K_COUNT] = {0};
};

namespace {

template <typename T>
cf_status dalloc(cf_plan* pl, T** out, size_t count) {
  void* p = nullptr;
  const size_t nb = std::max<size_t>(count * sizeof(T), 256);
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(CF_ERR_NOMEM, "hipMalloc of " + std::to_string(nb) + " bytes failed");
  }
  pl->allocs.push_back(DevBuf{p, nb});
  pl->bytes += nb;
  *out = static_cast<T*>(p);
  return CF_OK;
}

template <typename T>
cf_status upload(cf_plan* pl, T** out, const std::vector<T>& h) {
  cf_status s = dalloc(pl, out, h.size());
  if (s != CF_OK) return s;
  hipError_t e = hipMemcpy(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return dev_fail(e, "hipMemcpy (plan tables)");
  return CF_OK;
}

void free_all(cf_plan* pl) {
  if (!pl->allocs.empty() || !pl->events.empty()) (void)hipDeviceSynchronize();
  for (auto& b : pl->allocs) (void)hipFree(b.p);
  pl->allocs.clear();
  for (hipEvent_t e : pl->events) (void)hipEventDestroy(e);
  pl->events.clear();
  pl->pending.clear();
  if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
  if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
  if (pl->aux) (void)hipStreamDestroy(pl->aux);
  for (auto& g : pl->graphs) (void)hipGraphExecDestroy(g.exec);
  pl->graphs.clear();
  if (pl->ev_gin) (void)hipEventDestroy(pl->ev_gin);
  if (pl->ev_gout) (void)hipEventDestroy(pl->ev_gout);
  if (pl->gstream) (void)hipStreamDestroy(pl->gstream);
  pl->ev_fork = pl->ev_join = pl->ev_gin = pl->ev_gout = nullptr;
  pl->aux = pl->gstream = nullptr;
}

hipError_t next_event(cf_plan* pl, hipEvent_t* ev) {
  if (pl->ev_used == pl->events.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pl->events.push_back(e);
  }
  *ev = pl->events[pl->ev_used++];
  return hipSuccess;
}

// Launch through `launch` (returning hipError_t), bracketed by events when the
// plan's timing is on.
template <class F>
cf_status timed(cf_plan* pl, int cls, hipStream_t s, const char* what, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (pl->timing) {
    hipError_t r = next_event(pl, &a);
    if (r == hipSuccess) r = next_event(pl, &b);
    if (r == hipSuccess) r = hipEventRecord(a, s);
    if (r != hipSuccess) return dev_fail(r, "timing event");
  }
  hipError_t e = launch();
  if (e != hipSuccess) return dev_fail(e, what);
  if (pl->timing) {
    hipError_t r = hipEventRecord(b, s);
    if (r != hipSuccess) return dev_fail(r, "timing event");
    pl->pending.push_back(cf_plan::Pending{cls, a, b});
  }
  return CF_OK;
}

cf_status harvest(cf_plan* pl) {
  for (auto& p : pl->pending) {
    hipError_t r = hipEventSynchronize(p.b);
    if (r != hipSuccess) return dev_fail(r, "hipEventSynchronize");
    float ms = 0.f;
    r = hipEventElapsedTime(&ms, p.a, p.b);
    if (r != hipSuccess) return dev_fail(r, "hipEventElapsedTime");
    pl->acc_ms[p.cls] += ms;
    pl->acc_n[p.cls] += 1;
  }
  pl->pending.clear();
  pl->ev_used = 0;
  return CF_OK;
}

// Largest corner term of Eq. (21) over the interior partitions of the outer
// (G-partition) PDD, for one k^2: partition g of ny/G rows solves A_g v =
// a_first e_1 and A_g w = c_last e_last (Thomas, FP64), and the corner terms are
// v at its last row and w at its first.
double corner_delta(const cf_plan* pl, double k2) {
  const int G = pl->G, Mg = pl->P * pl->M / G;  // interior groups hold no padding rows
  double delta = 0.0;
  std::vector<double> cp(Mg), v(Mg), w(Mg);
  for (int g = 1; g + 1 < G; ++g) {
    const double* ar = pl->a.data() + g * Mg;
    const double* cr = pl->c.data() + g * Mg;
    // forward elimination of the block (its first a and last c left out)
    double den_last = 0.0;
    for (int s = 0; s < Mg; ++s) {
      const double b = -(ar[s] + cr[s]) - k2;
      const double den = (s == 0) ? b : b - ar[s] * cp[s - 1];
      cp[s] = (s == Mg - 1) ? 0.0 : cr[s] / den;
      v[s] = (s == 0) ? ar[0] / den : -(ar[s] * v[s - 1]) / den;
      if (s == Mg - 1) den_last = den;
    }
    w[Mg - 1] = cr[Mg - 1] / den_last;
    for (int s = Mg - 2; s >= 0; --s) {
      v[s] = v[s] - cp[s] * v[s + 1];
      w[s] = -(cp[s] * w[s + 1]);
    }
    delta = std::max(delta, std::max(std::fabs(v[Mg - 1]), std::fabs(w[0])));
  }
  return delta;
}

// Default outer partitions of the dropped reduced system: four groups when
// four divide P (the corner terms then span a quarter of the channel, long
// enough on the stretched workload grids for most wavenumbers), else P.
int auto_drop_parts(int P) { return (P % 4 == 0) ? 4 : P; }

// Zero rows after the wall-normal coefficient tables: more than any
// partitioning pads (fewer than the largest compiled row count, 32).
constexpr int kPadRows = 32;

// Rows per partition when ny is split into P parts: M = ceil(ny/P); when P
// does not divide ny the last partition is completed by P*M - ny < M padding
// rows (a = c = 0 in the line solve's tables, zero right-hand side; below the
// wall row, whose c is 0, they are decoupled from the line).
int part_rows(int ny, int P) { return (ny + P - 1) / P; }

// Partitioning of the wall-normal lines into P parts of M = part_rows(ny, P)
// rows (Section 2.2), the outer partitions G of the dropped reduced system,
// and the drop threshold that goes with them: the smallest k^2 whose G-level
// corner terms are all <= drop_tol (the corner terms fall monotonically with
// k^2).
void set_partitions(cf_plan* pl, int P, int LB) {
  pl->P = P;
  pl->M = part_rows(pl->ny, P);
  pl->LB = LB;
  pl->G = (pl->opt.drop_parts > 0 && P % pl->opt.drop_parts == 0) ? pl->opt.drop_parts : auto_drop_parts(P);
  double kmax = 0.0;
  for (double v : pl->kx2) kmax = std::max(kmax, v);
  double kzm = 0.0;
  for (double v : pl->kz2) kzm = std::max(kzm, v);
  kmax += kzm;
  const double tol = pl->opt.drop_tol;
  if (pl->G <= 2) {
    pl->k2drop = 0.0;
  } else if (corner_delta(pl, kmax) > tol) {
    pl->k2drop = INFINITY;
  } else {
    double lo = 0.0, hi = kmax;
    if (corner_delta(pl, 0.0) <= tol) hi = 0.0;
    for (int it = 0; it < 200 && hi > 0.0 && (hi - lo) > 1e-12 * hi; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (corner_delta(pl, mid) <= tol) hi = mid; else lo = mid;
    }
    pl->k2drop = hi;
  }
  pl->n_drop = 0;
  for (int kx = 0; kx < pl->nkx; ++kx)
    for (int kz = 0; kz < pl->nz; ++kz)
      if (pl->kx2[kx] + pl->kz2[kz] >= pl->k2drop) ++pl->n_drop;
  // a block of LB consecutive lines drops the corner terms only when all of
  // its lines qualify
  const long nl = (long)pl->nkx * pl->nz;
  pl->n_dropped = 0;
  pl->blocks_exact.clear();
  pl->blocks_drop.clear();
  for (long b0 = 0; b0 < nl; b0 += LB) {
    const long b1 = std::min(nl, b0 + LB);
    bool all = true;
    for (long l = b0; l < b1 && all; ++l) all = pl->kx2[l / pl->nz] + pl->kz2[l % pl->nz] >= pl->k2drop;
    if (all) {
      pl->n_dropped += b1 - b0;
      pl->blocks_drop.push_back(int(b0 / LB));
    } else {
      pl->blocks_exact.push_back(int(b0 / LB));
    }
  }
}

// Copies the block lists of set_partitions to the device (synchronously).
cf_status upload_blocks(cf_plan* pl) {
  if (!pl->d_blocks) return CF_OK;
  const size_t ne = pl->blocks_exact.size(), nd = pl->blocks_drop.size();
  if (ne) CF_HIP_RET(hipMemcpy(pl->d_blocks, pl->blocks_exact.data(), ne * sizeof(int), hipMemcpyHostToDevice));
  if (nd) CF_HIP_RET(hipMemcpy(pl->d_blocks + ne, pl->blocks_drop.data(), nd * sizeof(int), hipMemcpyHostToDevice));
  return CF_OK;
}

// P parts of part_rows(ny, P) rows with a compiled row count, P <= 64, every
// part holding at least one row of the line.
bool parts_ok(int ny, int P, bool fp64) {
  if (P < 1 || P > 64) return false;
  const int M = part_rows(ny, P);
  return cf::ysolve_m_compiled(M, fp64) && (P - 1) * M < ny;
}

int auto_parts(int ny, bool fp64) {
  // fewest partitions with a compiled row count (at most 16 rows in FP64, 32 in
  // FP32) that divide ny, preferring powers of two; if none divides ny, the
  // partitioning with the fewest padding rows (then the fewest partitions)
  for (int P = 1; P <= 64; P *= 2)
    if (ny % P == 0 && parts_ok(ny, P, fp64)) return P;
  for (int P = 1; P <= 64; ++P)
    if (ny % P == 0 && parts_ok(ny, P, fp64)) return P;
  int best = 0;
  for (int P = 1; P <= 64; ++P)
    if (parts_ok(ny, P, fp64) && (best == 0 || P * part_rows(ny, P) < best * part_rows(ny, best))) best = P;
  return best;
}

cf_status check_plan(const cf_plan* pl) {
  if (!pl) return fail(CF_ERR_ARG, "plan is NULL");
  return CF_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Whether the byte ranges [a, a + na) and [b, b + nb) share a byte.
bool bytes_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + nb && y < x + na;
}

// CF_ERR_ARG when output `out` (nout bytes) overlaps input `in` (nin bytes),
// unless same_ok and out is in itself.
cf_status check_disjoint(const void* out, size_t nout, const void* in, size_t nin, bool same_ok, const char* what) {
  if (same_ok && out == in) return CF_OK;
  if (bytes_overlap(out, nout, in, nin)) return fail(CF_ERR_ARG, what);
  return CF_OK;
}

// Bytes of a physical field and of a spectrum of the plan.
size_t field_bytes(const cf_plan* pl, size_t esize) { return (size_t)pl->nx * pl->ny * pl->nz * esize; }
size_t spec_bytes(const cf_plan* pl) {
  return (size_t)pl->nkx * pl->ny * pl->nz * (pl->mixed() ? sizeof(cx<float>) : sizeof(cx<double>));
}

cf_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(CF_ERR_ARG, std::string(name) + " is NULL");
  if (!aligned16(p)) return fail(CF_ERR_ARG, std::string(name) + " is not 16-byte aligned");
  return CF_OK;
}

#define CF_TRY(x)                     \
  do {                                \
    cf_status _s = (x);               \
    if (_s != CF_OK) return _s;       \
  } while (0)
#define CF_HIP(x, what)                          \
  do {                                           \
    hipError_t _e = (x);                         \
    if (_e != hipSuccess) return dev_fail(_e, what); \
  } while (0)

// ---------------------------------------------------------------- pipelines
template <typename T>
struct Tabs;
template <>
struct Tabs<double> {
  static const double* a(const cf_plan* p) { return p->d_a; }
  static const double* c(const cf_plan* p) { return p->d_c; }
  static const double* kx2(const cf_plan* p) { return p->d_kx2; }
  static const double* kz2(const cf_plan* p) { return p->d_kz2; }
  static const cx<double>* twz(const cf_plan* p) { return p->tw_z64; }
  static const cx<double>* twx(const cf_plan* p) { return p->tw_x64; }
  static const cx<double>* twp(const cf_plan* p) { return p->twp64; }
};
template <>
struct Tabs<float> {
  static const float* a(const cf_plan* p) { return p->s_a; }
  static const float* c(const cf_plan* p) { return p->s_c; }
  static const float* kx2(const cf_plan* p) { return p->s_kx2; }
  static const float* kz2(const cf_plan* p) { return p->s_kz2; }
  static const cx<float>* twz(const cf_plan* p) { return p->tw_z32; }
  static const cx<float>* twx(const cf_plan* p) { return p->tw_x32; }
  static const cx<float>* twp(const cf_plan* p) { return p->twp32; }
};

// f (physical) -> spectrum in layout B
template <typename T>
const cf::AdjGeo<T>& adj_geo(const cf_plan* pl);
template <>
const cf::AdjGeo<double>& adj_geo<double>(const cf_plan* pl) { return pl->a64; }
template <>
const cf::AdjGeo<float>& adj_geo<float>(const cf_plan* pl) { return pl->a32; }

template <typename T>
cf_status forward_t(cf_plan* pl, const double* f, cx<T>* outB, hipStream_t s) {
  using TB = Tabs<T>;
  cx<T>* A = static_cast<cx<T>*>(pl->specA);
  CF_TRY(timed(pl, CF_K_R2C_X, s, "r2c launch", [&] {
    return cf::launch_r2c_plain<T>(pl->nh, f, A, TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, s);
  }));
  CF_TRY(timed(pl, CF_K_FFT_Z_FWD, s, "z fft launch", [&] {
    return cf::launch_fft_z<T>(pl->nz, false, A, outB, TB::twz(pl), pl->ny, pl->nkx, s);
  }));
  return CF_OK;
}

// scale * D(u, v, w) -> spectrum in layout B (divergence fused into the x transform)
template <typename T>
cf_status forward_div_t(cf_plan* pl, const double* u, const double* v, const double* w, double scale,
                        cx<T>* outB, hipStream_t s) {
  using TB = Tabs<T>;
  cx<T>* A = static_cast<cx<T>*>(pl->specA);
  CF_TRY(timed(pl, CF_K_R2C_X, s, "r2c+div launch", [&] {
    return cf::launch_r2c_div<T>(pl->nh, u, v, w, pl->d_rdy, 1.0 / pl->dx, 1.0 / pl->dz, scale, A,
                                 TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, s);
  }));
  CF_TRY(timed(pl, CF_K_FFT_Z_FWD, s, "z fft launch", [&] {
    return cf::launch_fft_z<T>(pl->nz, false, A, outB, TB::twz(pl), pl->ny, pl->nkx, s);
  }));
  return CF_OK;
}

// spectrum in layout B -> p (physical), scaled by 1/(nx nz); inB is not modified
template <typename T>
cf_status inverse_t(cf_plan* pl, const cx<T>* inB, double* p, hipStream_t s) {
  using TB = Tabs<T>;
  cx<T>* A = static_cast<cx<T>*>(pl->specA);
  CF_TRY(timed(pl, CF_K_FFT_Z_INV, s, "z ifft launch", [&] {
    return cf::launch_fft_z<T>(pl->nz, true, inB, A, TB::twz(pl), pl->nkx, pl->ny, s);
  }));
  const T scale = T(1.0 / ((double)pl->nx * (double)pl->nz));
  CF_TRY(timed(pl, CF_K_C2R_X, s, "c2r launch", [&] {
    return cf::launch_c2r_plain<T>(pl->nh, A, p, TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, scale, s);
  }));
  return CF_OK;
}

// One launch of the partitioned line solve with the plan's partitioning (whole
// lines, or one slab's local or finishing pass over partitions [pa, pb)).
template <typename T>
hipError_t pdd_launch(const cf_plan* pl, const cx<T>* fin, cx<T>* pout, hipStream_t s, int mode = cf::kWhole,
                      int pa = 0, int pb = 0, void* iface = nullptr) {
  using TB = Tabs<T>;
  cf::YLaunch y;
  y.ny = pl->ny;
  y.nz = pl->nz;
  y.nkx = pl->nkx;
  y.P = pl->P;
  y.M = pl->M;
  y.LB = pl->LB;
  y.nlines = (long)pl->nkx * pl->nz;
  y.skip_kx = pl->mixed() ? pl->opt.fp64_kx : 0;
  y.skip_kz = pl->mixed() ? pl->opt.fp64_kz : 0;
  y.mode = mode;
  y.pa = pa;
  y.pb = pb;
  y.iface = iface;
  y.G = pl->G;
  if (pl->d_blocks) {
    y.blocks_exact = pl->d_blocks;
    y.n_exact = (long)pl->blocks_exact.size();
    y.blocks_drop = pl->blocks_drop.empty() ? nullptr : pl->d_blocks + pl->blocks_exact.size();
    y.n_drop = (long)pl->blocks_drop.size();
  }
  return cf::launch_ysolve<T>(y, fin, pout, TB::a(pl), TB::c(pl), TB::kx2(pl), TB::kz2(pl), s);
}

// The partitioned solve as n_slabs y-slabs: every slab's local pass, then the
// whole-line FP64 solves of the special lines on the side stream next to every
// slab's finishing pass (they touch only the special lines, which the
// finishing passes do not write).
template <typename T>
cf_status slabs_t(cf_plan* pl, int n_slabs, const cx<T>* fin, cx<T>* pout, void* iface, hipStream_t s) {
  const int per = pl->P / n_slabs;
  for (int g = 0; g < n_slabs; ++g)
    CF_TRY(timed(pl, CF_K_SLAB_LOCAL, s, "slab local launch", [&] {
      return pdd_launch<T>(pl, fin, pout, s, cf::kSlabLocal, g * per, (g + 1) * per, iface);
    }));
  CF_HIP(hipEventRecord(pl->ev_fork, s), "hipEventRecord");
  CF_HIP(hipStreamWaitEvent(pl->aux, pl->ev_fork, 0), "hipStreamWaitEvent");
  CF_TRY(timed(pl, CF_K_SPECIAL, pl->aux, "special-line launch", [&] {
    return cf::launch_special_lines<T>(fin, pout, pl->d_a, pl->d_special_den, pl->d_special_cp, pl->d_dy,
                                       pl->d_special, (int)pl->special.size(), pl->ny, pl->nz, nullptr, 0,
                                       pl->d_numflag, pl->aux);
  }));
  CF_HIP(hipEventRecord(pl->ev_join, pl->aux), "hipEventRecord");
  for (int g = 0; g < n_slabs; ++g)
    CF_TRY(timed(pl, CF_K_SLAB_FINISH, s, "slab finish launch", [&] {
      return pdd_launch<T>(pl, fin, pout, s, cf::kSlabFinish, g * per, (g + 1) * per, iface);
    }));
  CF_HIP(hipStreamWaitEvent(s, pl->ev_join, 0), "hipStreamWaitEvent");
  return CF_OK;
}

// psum (nullable): block sums of the pressure a correction solve adds to (see
// launch_special_lines).
template <typename T>
cf_status solve_t(cf_plan* pl, const cx<T>* fin, cx<T>* pout, hipStream_t s, const double* psum = nullptr) {
  if constexpr (std::is_same<T, double>::value) {
    if (pl->opt.flags & CF_PLAN_Y_DCT)
      return timed(pl, CF_K_YSOLVE, s, "y-transform solve launch", [&] {
        return cf::launch_ydct<double>(fin, pout, pl->tw_y64, pl->d_wqy, pl->d_lamy, pl->d_kx2, pl->d_kz2, pl->ny,
                                       pl->nz, pl->nkx, s);
      });
  }
  // The whole-line solves run on the side stream next to the PDD kernel: they
  // read and write only the special lines, which the PDD kernel reads but does
  // not write (lines are independent there, so the values it reads for them
  // are discarded).
  CF_HIP(hipEventRecord(pl->ev_fork, s), "hipEventRecord");
  CF_HIP(hipStreamWaitEvent(pl->aux, pl->ev_fork, 0), "hipStreamWaitEvent");
  CF_TRY(timed(pl, CF_K_SPECIAL, pl->aux, "special-line launch", [&] {
    return cf::launch_special_lines<T>(fin, pout, pl->d_a, pl->d_special_den, pl->d_special_cp, pl->d_dy,
                                       pl->d_special, (int)pl->special.size(), pl->ny, pl->nz, psum,
                                       psum ? pl->psum_nzb : 0, pl->d_numflag, pl->aux);
  }));
  CF_HIP(hipEventRecord(pl->ev_join, pl->aux), "hipEventRecord");
  CF_TRY(timed(pl, CF_K_YSOLVE, s, "y-solve launch", [&] {
    return pdd_launch<T>(pl, fin, pout, s);
  }));
  CF_HIP(hipStreamWaitEvent(s, pl->ev_join, 0), "hipStreamWaitEvent");
  return CF_OK;
}

template <typename T>
cf_status poisson_t(cf_plan* pl, const double* f, double* p, hipStream_t s) {
  cx<T>* B = static_cast<cx<T>*>(pl->specB);
  CF_TRY(forward_t<T>(pl, f, B, s));
  CF_TRY(solve_t<T>(pl, B, B, s));
  CF_TRY(inverse_t<T>(pl, B, p, s));
  return CF_OK;
}

// Right-hand side of a mixed-precision solve: an FP64 array f (kind 0),
// scale * D(u, v, w) (kind 1) or D(u / W, v / W, w / W) (kind 2, the
// transposed projection), with float velocities.
struct MixedRhs {
  int kind;
  const double* f;
  const float *u, *v, *w;
  double scale;
};

// Mixed-precision Poisson solve: p0 = S32(f), then refine_passes times
// p += S32(f - L_h p) with the residual formed in FP64.  S32 runs the transforms
// and the bulk PDD in FP32 and the FP64 line set in FP64.  p0 comes out of an
// FP32 transform, so when a refinement follows it is stored as FP32, packed
// into the first half of each FP64 row of p (the same values at half the
// bytes); the residual reads it from there and the first correction writes
// the FP64 sum over it.
cf_status poisson_mixed(cf_plan* pl, MixedRhs rhs, double* p, hipStream_t s) {
  using TB = Tabs<float>;
  cx<float>* A = static_cast<cx<float>*>(pl->specA);
  cx<float>* B = static_cast<cx<float>*>(pl->specB);
  if (rhs.kind == 0 && rhs.f == p && pl->opt.refine_passes > 0) {
    CF_HIP(hipMemcpyAsync(pl->fws, rhs.f, sizeof(double) * (size_t)pl->nx * pl->ny * pl->nz,
                          hipMemcpyDeviceToDevice, s),
           "hipMemcpyAsync");
    rhs.f = pl->fws;
  }
  if (rhs.kind == 0) {
    CF_TRY(forward_t<float>(pl, rhs.f, B, s));
  } else {
    CF_TRY(timed(pl, CF_K_R2C_X, s, "r2c+div launch", [&] {
      if (rhs.kind == 1)
        return cf::launch_r2c_div_t<float, float>(pl->nh, rhs.u, rhs.v, rhs.w, pl->d_rdy, 1.0 / pl->dx,
                                                  1.0 / pl->dz, rhs.scale, A, TB::twx(pl), TB::twp(pl), pl->ny,
                                                  pl->nz, s);
      return cf::launch_r2c_divw<float, float>(pl->nh, rhs.u, rhs.v, rhs.w, pl->d_rdy, pl->d_rdyc, 1.0 / pl->dx,
                                               1.0 / pl->dz, A, TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, s);
    }));
    CF_TRY(timed(pl, CF_K_FFT_Z_FWD, s, "z fft launch", [&] {
      return cf::launch_fft_z<float>(pl->nz, false, A, B, TB::twz(pl), pl->ny, pl->nkx, s);
    }));
  }
  CF_TRY(solve_t<float>(pl, B, B, s));
  const float scl = float(1.0 / ((double)pl->nx * (double)pl->nz));
  const bool p32 = pl->opt.refine_passes > 0;
  if (p32) {
    CF_TRY(timed(pl, CF_K_FFT_Z_INV, s, "z ifft launch", [&] {
      return cf::launch_fft_z<float>(pl->nz, true, B, A, TB::twz(pl), pl->nkx, pl->ny, s);
    }));
    CF_TRY(timed(pl, CF_K_C2R_X, s, "c2r launch", [&] {
      return cf::launch_c2r_rows32<float>(pl->nh, A, p, TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, scl, s);
    }));
  } else {
    CF_TRY(inverse_t<float>(pl, B, p, s));
  }
  for (int it = 0; it < pl->opt.refine_passes; ++it) {
    const bool in32 = p32 && it == 0;  // p still holds the packed FP32 rows
    CF_TRY(timed(pl, CF_K_R2C_X, s, "residual r2c launch", [&] {
      return cf::launch_r2c_resid<float, float>(rhs.kind, pl->nh, rhs.f, rhs.u, rhs.v, rhs.w, rhs.scale, p, in32,
                                                pl->d_a, pl->d_c, pl->d_rdy, pl->d_rdyc, 1.0 / pl->dx, 1.0 / pl->dz,
                                                A, TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, pl->d_psum, s);
    }));
    CF_TRY(timed(pl, CF_K_FFT_Z_FWD, s, "z fft launch", [&] {
      return cf::launch_fft_z<float>(pl->nz, false, A, B, TB::twz(pl), pl->ny, pl->nkx, s);
    }));
    // the correction's mean line carries -mean_W(p): the residual is blind to
    // a constant in p, and the FP32 transforms of the previous solve leave
    // mean_W(p) off zero by their rounding
    CF_TRY(solve_t<float>(pl, B, B, s, pl->d_psum));
    CF_TRY(timed(pl, CF_K_FFT_Z_INV, s, "z ifft launch", [&] {
      return cf::launch_fft_z<float>(pl->nz, true, B, A, TB::twz(pl), pl->nkx, pl->ny, s);
    }));
    CF_TRY(timed(pl, CF_K_C2R_X, s, "c2r accumulate launch", [&] {
      return cf::launch_c2r_accum<float>(pl->nh, A, p, TB::twx(pl), TB::twp(pl), pl->ny, pl->nz, scl, in32, s);
    }));
  }
  return CF_OK;
}

// The RK2 momentum update u1 = (u + ub)/2 + dt/2 R(ub), ub = u + dt R(u).  One
// fused pass when the outputs are separate arrays; when an output overlaps an
// input (in-place step) the fused pass would read cells other blocks already
// overwrote, so the two stages run as separate passes through the stage-1
// workspace (stage 2 reads the old field only at the cell it writes).
template <typename T>
cf_status rk2_t(cf_plan* pl, const T* u, const T* v, const T* w, T* u1, T* v1, T* w1, const cf::Geo<T>& g, T dt,
                T nu, T fx, hipStream_t s) {
  const uintptr_t bytes = (uintptr_t)pl->nx * pl->ny * pl->nz * sizeof(T);
  const T* in[3] = {u, v, w};
  const T* out[3] = {u1, v1, w1};
  bool overlap = false;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const uintptr_t x = reinterpret_cast<uintptr_t>(in[a]), y = reinterpret_cast<uintptr_t>(out[b]);
      overlap = overlap || (x < y + bytes && y < x + bytes);
    }
  if (!overlap)
    return timed(pl, CF_K_RK_FUSED, s, "fused rk2",
                 [&] { return cf::launch_rk2_fused<T>(u, v, w, u1, v1, w1, g, dt, nu, fx, s); });
  T* ub = static_cast<T*>(pl->ub);
  T* vb = static_cast<T*>(pl->vb);
  T* wb = static_cast<T*>(pl->wb);
  CF_TRY(timed(pl, CF_K_RK1, s, "rk stage 1", [&] {
    return cf::launch_rk_stage<T>(1, u, v, w, nullptr, nullptr, nullptr, ub, vb, wb, g, dt, nu, fx, s);
  }));
  return timed(pl, CF_K_RK2, s, "rk stage 2",
               [&] { return cf::launch_rk_stage<T>(2, ub, vb, wb, u, v, w, u1, v1, w1, g, dt, nu, fx, s); });
}

// One mixed-precision projection step (FP32 velocity state, FP64 pressure).
// acc (optional): the plane statistics of the new state are added into it by
// the correction pass.
cf_status step_mixed(cf_plan* pl, const float* u, const float* v, const float* w, float* u1, float* v1,
                     float* w1, double* p, double dt, double nu, double fx, hipStream_t s, double* acc = nullptr) {
  double* pp = p ? p : pl->pws;
  const float fdt = float(dt), fnu = float(nu), ffx = float(fx);
  CF_TRY(rk2_t<float>(pl, u, v, w, u1, v1, w1, pl->g32, fdt, fnu, ffx, s));
  CF_TRY(poisson_mixed(pl, MixedRhs{1, nullptr, u1, v1, w1, 1.0 / dt}, pp, s));
  CF_TRY(timed(pl, CF_K_CORRECT, s, "correction", [&] {
    return acc ? cf::launch_correct_stats<float>(u1, v1, w1, pp, pl->g32, fdt, pl->d_stat_part, pl->stat_nch, acc, 1, s)
               : cf::launch_correct<float>(u1, v1, w1, pp, pl->g32, fdt, s);
  }));
  return CF_OK;
}

// One FP64 projection step.
cf_status step64(cf_plan* pl, const double* u, const double* v, const double* w, double* u1, double* v1,
                 double* w1, double* p, double dt, double nu, double fx, hipStream_t s, double* acc = nullptr) {
  double* pp = p ? p : pl->pws;
  CF_TRY(rk2_t<double>(pl, u, v, w, u1, v1, w1, pl->g64, dt, nu, fx, s));
  cx<double>* B = static_cast<cx<double>*>(pl->specB);
  CF_TRY(forward_div_t<double>(pl, u1, v1, w1, 1.0 / dt, B, s));
  CF_TRY(solve_t<double>(pl, B, B, s));
  CF_TRY(inverse_t<double>(pl, B, pp, s));
  CF_TRY(timed(pl, CF_K_CORRECT, s, "correction", [&] {
    return acc ? cf::launch_correct_stats<double>(u1, v1, w1, pp, pl->g64, dt, pl->d_stat_part, pl->stat_nch, acc, 1, s)
               : cf::launch_correct<double>(u1, v1, w1, pp, pl->g64, dt, s);
  }));
  return CF_OK;
}

// Adjoint of one projection step, state type T.  The transposed projection
// runs first: its spectral workspace shares memory with the stage-1 fields,
// which are recomputed afterwards; the pressure workspace shares memory with gb.
template <typename T>
cf_status step_adjoint_t(cf_plan* pl, const T* u, const T* v, const T* w, const T* g1u, const T* g1v,
                         const T* g1w, T* gu, T* gv, T* gw, double dt, double nu, double fx, hipStream_t s) {
  T* ub = static_cast<T*>(pl->ub);
  T* vb = static_cast<T*>(pl->vb);
  T* wb = static_cast<T*>(pl->wb);
  T* su = static_cast<T*>(pl->gsu);
  T* sv = static_cast<T*>(pl->gsv);
  T* sw = static_cast<T*>(pl->gsw);
  T* bu = static_cast<T*>(pl->gbu);
  T* bv = static_cast<T*>(pl->gbv);
  T* bw = static_cast<T*>(pl->gbw);
  const T tdt = T(dt), tnu = T(nu), tfx = T(fx);
  // g* = g1 - W G L^+ D (g1 / W)
  if constexpr (std::is_same<T, double>::value) {
    cx<double>* A = static_cast<cx<double>*>(pl->specA);
    cx<double>* B = static_cast<cx<double>*>(pl->specB);
    CF_TRY(timed(pl, CF_K_R2C_X, s, "r2c+weighted div launch", [&] {
      return cf::launch_r2c_divw<double, double>(pl->nh, g1u, g1v, g1w, pl->d_rdy, pl->d_rdyc, 1.0 / pl->dx,
                                                 1.0 / pl->dz, A, pl->tw_x64, pl->twp64, pl->ny, pl->nz, s);
    }));
    CF_TRY(timed(pl, CF_K_FFT_Z_FWD, s, "z fft launch", [&] {
      return cf::launch_fft_z<double>(pl->nz, false, A, B, pl->tw_z64, pl->ny, pl->nkx, s);
    }));
    CF_TRY(solve_t<double>(pl, B, B, s));
    CF_TRY(inverse_t<double>(pl, B, pl->pws, s));
  } else {
    CF_TRY(poisson_mixed(pl, MixedRhs{2, nullptr, g1u, g1v, g1w, 1.0}, pl->pws, s));
  }
  const cf::AdjGeo<T>& ag = adj_geo<T>(pl);
  CF_TRY(timed(pl, CF_K_ADJ_CORRECT, s, "weighted correction", [&] {
    return cf::launch_correct_w<T>(g1u, g1v, g1w, su, sv, sw, pl->pws, ag, s);
  }));
  // recompute the stage-1 field (overwrites the spectral workspace)
  CF_TRY(timed(pl, CF_K_RK1, s, "rk stage 1", [&] {
    return cf::launch_rk_stage<T>(1, u, v, w, nullptr, nullptr, nullptr, ub, vb, wb, ag.g, tdt, tnu, tfx, s);
  }));
  // gb = dt/2 J_R(ub)^T g*   (overwrites the pressure workspace)
  CF_TRY(timed(pl, CF_K_ADJ_RHS, s, "rhs adjoint", [&] {
    return cf::launch_rhs_adjoint<T>(ub, vb, wb, su, sv, sw, nullptr, nullptr, nullptr, T(1), T(0), ag, tnu,
                                     T(0.5) * tdt, 0, bu, bv, bw, s);
  }));
  // g = g* + gb + J_R(u)^T (dt/2 g* + dt gb)
  CF_TRY(timed(pl, CF_K_ADJ_RHS, s, "rhs adjoint", [&] {
    return cf::launch_rhs_adjoint<T>(u, v, w, su, sv, sw, bu, bv, bw, T(0.5) * tdt, tdt, ag, tnu, T(1), 1, gu, gv,
                                     gw, s);
  }));
  return CF_OK;
}

// Elimination factors of one whole-line solve, in the operation order of the
// textbook Thomas algorithm (no contraction).
void special_factors(const cf_plan* pl, int line, double* den, double* cp) {
#pragma clang fp contract(off)
  const int ny = pl->ny, nz = pl->nz;
  const int kx = line / nz, kz = line % nz;
  const double k2 = pl->kx2[kx] + pl->kz2[kz];
  const bool mean_line = (line == 0);
  const int n = mean_line ? ny - 1 : ny;
  double cprev = 0.0;
  for (int j = 0; j < ny; ++j) {
    if (j >= n) {
      den[j] = 1.0;
      cp[j] = 0.0;
      continue;
    }
    const double b = -(pl->a[j] + pl->c[j]) - k2;
    const double t = pl->a[j] * cprev;
    const double d = (j == 0) ? b : b - t;
    const double cj = (j == n - 1) ? 0.0 : pl->c[j];
    den[j] = d;
    cp[j] = cj / d;
    cprev = cp[j];
  }
}

// Partition count and block shape by measurement (the count and placement
// question of Section 2.2, answered on the device): every P with ny = P*M for
// a compiled M, P <= 64 (if there is none, every padded partitioning that
// parts_ok admits), and every block of LB lines with 64 <= LB*P <= 512
// threads that fits in LDS, is timed over five launches of the partitioned
// solve (in place, on zeros in the plan's spectral workspace, on the plan's
// capture stream, after two warm-up launches); the fastest is kept and the drop
// threshold follows its P.
cf_status tune_partitions(cf_plan* pl, size_t lds_max) {
  const bool fp64 = !pl->mixed();
  hipStream_t s = pl->gstream;
  const size_t nspec = (size_t)pl->ny * pl->nkx * pl->nz;
  CF_HIP(hipMemsetAsync(pl->specB, 0, nspec * (fp64 ? sizeof(cx<double>) : sizeof(cx<float>)), s),
         "hipMemsetAsync");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto done = [&](cf_status st) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st;
  };
  if (e != hipSuccess) return done(dev_fail(e, "hipEventCreate"));
  constexpr int kWarm = 2, kRuns = 5;
  pl->tune.clear();
  size_t best = 0;
  // the partition counts that divide ny, or the padded ones when none does
  bool any_exact = false;
  for (int P = 1; P <= 64; ++P) any_exact = any_exact || (pl->ny % P == 0 && parts_ok(pl->ny, P, fp64));
  for (int P = 1; P <= 64; ++P) {
    if (!parts_ok(pl->ny, P, fp64) || (any_exact && pl->ny % P != 0)) continue;
    for (int LB = 4; LB <= 256; LB *= 2) {
      if (LB * P < 64 || LB * P > 512 || cf::ysolve_lds_needed(P * part_rows(pl->ny, P), P, LB, fp64) > lds_max)
        continue;
      set_partitions(pl, P, LB);
      if (upload_blocks(pl) != CF_OK) return done(CF_ERR_DEVICE);
      for (int r = 0; r < kWarm + kRuns && e == hipSuccess; ++r) {
        if (r == kWarm) e = hipEventRecord(e0, s);
        if (e != hipSuccess) break;
        e = fp64 ? pdd_launch<double>(pl, static_cast<cx<double>*>(pl->specB), static_cast<cx<double>*>(pl->specB), s)
                 : pdd_launch<float>(pl, static_cast<cx<float>*>(pl->specB), static_cast<cx<float>*>(pl->specB), s);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) return done(dev_fail(e, "partition timing"));
      pl->tune.push_back({P, LB, 1e3 * (double)ms / kRuns});
      if (pl->tune.back().us < pl->tune[best].us) best = pl->tune.size() - 1;
    }
  }
  if (pl->tune.empty()) return done(fail(CF_ERR_UNSUPPORTED, "no partitioning fits"));
  set_partitions(pl, pl->tune[best].P, pl->tune[best].LB);
  return done(upload_blocks(pl));
}

}  // namespace

// ============================================================================
extern "C" {

void cf_options_default(cf_options* opt) {
  if (!opt) return;
  opt->precision = CF_FP64;
  opt->n_parts = 0;
  opt->drop_tol = -1.0;
  opt->fp64_kx = 4;
  opt->fp64_kz = 4;
  opt->refine_passes = 1;
  opt->flags = 0;
  opt->lines_per_block = 0;
  opt->drop_parts = 0;
}

const char* cf_status_string(cf_status s) {
  switch (s) {
    case CF_OK: return "ok";
    case CF_ERR_ARG: return "invalid argument";
    case CF_ERR_UNSUPPORTED: return "unsupported size";
    case CF_ERR_NOMEM: return "out of device memory";
    case CF_ERR_DEVICE: return "device error";
    case CF_ERR_NUMERIC: return "non-finite values";
  }
  return "unknown status";
}

const char* cf_last_error(void) { return g_last_error.c_str(); }

cf_status cf_plan_create(cf_plan** out, int nx, int ny, int nz, double lx, double lz,
                         const double* y_faces, const cf_options* opt_in) {
  g_last_error.clear();
  if (!out) return fail(CF_ERR_ARG, "out is NULL");
  *out = nullptr;
  cf_options opt;
  cf_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.precision != CF_FP64 && opt.precision != CF_MIXED) return fail(CF_ERR_ARG, "precision must be CF_FP64 or CF_MIXED");
  if (nx < 4 || nx % 2 != 0) return fail(CF_ERR_ARG, "nx must be even and >= 4");
  if (nz < 2) return fail(CF_ERR_ARG, "nz must be >= 2");
  if (ny < 2) return fail(CF_ERR_ARG, "ny must be >= 2");
  if (!(lx > 0.0) || !(lz > 0.0) || !std::isfinite(lx) || !std::isfinite(lz)) return fail(CF_ERR_ARG, "lx, lz must be finite and > 0");
  if (!y_faces) return fail(CF_ERR_ARG, "y_faces is NULL");
  for (int j = 0; j <= ny; ++j)
    if (!std::isfinite(y_faces[j])) return fail(CF_ERR_ARG, "y_faces holds a non-finite value");
  for (int j = 0; j < ny; ++j)
    if (!(y_faces[j + 1] > y_faces[j])) return fail(CF_ERR_ARG, "y_faces must be strictly increasing");
  if (!cf::fft_len_compiled(nx / 2)) return fail(CF_ERR_UNSUPPORTED, "nx/2 must be 2^a or 3*2^a in [2, 2048]");
  if (!cf::fft_len_compiled(nz)) return fail(CF_ERR_UNSUPPORTED, "nz must be 2^a or 3*2^a in [2, 2048]");
  const bool tune = (opt.flags & CF_PLAN_TUNE_PARTS) != 0;
  if (tune && (opt.n_parts != 0 || opt.lines_per_block != 0 || (opt.flags & CF_PLAN_Y_DCT)))
    return fail(CF_ERR_ARG, "CF_PLAN_TUNE_PARTS needs n_parts = 0, lines_per_block = 0 and the partitioned solve");
  int P = opt.n_parts;
  const bool fp64 = opt.precision == CF_FP64;
  if (P == 0) P = auto_parts(ny, fp64);
  if (P == 0 || !parts_ok(ny, P, fp64))
    return fail(CF_ERR_UNSUPPORTED,
                fp64 ? "ny needs P <= 64 partitions of M = ceil(ny/P) rows, M in {1,2,3,4,6,8,12,16}, "
                       "(P-1)*M < ny"
                     : "ny needs P <= 64 partitions of M = ceil(ny/P) rows, M in {1,2,3,4,6,8,12,16,24,32}, "
                       "(P-1)*M < ny");
  if (opt.lines_per_block < 0 || opt.lines_per_block * P > 512)
    return fail(CF_ERR_ARG, "lines_per_block must be >= 0 with lines_per_block * n_parts <= 512");
  if (opt.drop_parts < 0 || (opt.drop_parts > 0 && (tune || P % opt.drop_parts != 0)))
    return fail(CF_ERR_ARG, "drop_parts must be 0 or divide n_parts (and be 0 with CF_PLAN_TUNE_PARTS)");
  const int LB = opt.lines_per_block > 0 ? opt.lines_per_block : cf::ysolve_default_lb(P, part_rows(ny, P));
  if (opt.precision == CF_MIXED) {
    if (opt.fp64_kx < 1 || opt.fp64_kz < 1) return fail(CF_ERR_ARG, "fp64_kx and fp64_kz must be >= 1");
    if (opt.refine_passes < 0 || opt.refine_passes > 8) return fail(CF_ERR_ARG, "refine_passes must be in [0, 8]");
  }
  if (opt.drop_tol < 0) opt.drop_tol = (opt.precision == CF_MIXED) ? 1e-7 : 1e-15;
  if (opt.flags & CF_PLAN_Y_DCT) {
    if (opt.precision != CF_FP64) return fail(CF_ERR_UNSUPPORTED, "the y-transform solve is FP64 only");
    if (ny % 2 != 0 || !cf::ydct_len_compiled(ny))
      return fail(CF_ERR_UNSUPPORTED, "the y-transform solve needs an even ny = 2^a or 3*2^a <= 2048");
    const double d0 = y_faces[1] - y_faces[0];
    for (int j = 0; j < ny; ++j)
      if (std::fabs((y_faces[j + 1] - y_faces[j]) - d0) > 1e-12 * d0)
        return fail(CF_ERR_ARG, "the y-transform solve needs uniform y faces");
  }

  cf_plan* pl = new cf_plan();
  pl->nx = nx;
  pl->ny = ny;
  pl->nz = nz;
  pl->nh = nx / 2;
  pl->nkx = nx / 2 + 1;
  pl->lx = lx;
  pl->lz = lz;
  pl->dx = lx / nx;
  pl->dz = lz / nz;
  pl->opt = opt;
  pl->P = P;
  pl->M = part_rows(ny, P);
  pl->yf.assign(y_faces, y_faces + ny + 1);
  pl->dy.resize(ny);
  for (int j = 0; j < ny; ++j) pl->dy[j] = pl->yf[j + 1] - pl->yf[j];
  std::vector<double> yc(ny);
  for (int j = 0; j < ny; ++j) yc[j] = 0.5 * (pl->yf[j] + pl->yf[j + 1]);
  pl->dyc.resize(ny - 1);
  for (int j = 0; j + 1 < ny; ++j) pl->dyc[j] = yc[j + 1] - yc[j];
  // wall-normal rows of L_h = D o G (no flux through the walls), followed by
  // zeros for the padding rows of any partitioning (fewer than 32)
  pl->a.assign(ny + kPadRows, 0.0);
  pl->c.assign(ny + kPadRows, 0.0);
  for (int j = 1; j < ny; ++j) pl->a[j] = 1.0 / (pl->dy[j] * pl->dyc[j - 1]);
  for (int j = 0; j + 1 < ny; ++j) pl->c[j] = 1.0 / (pl->dy[j] * pl->dyc[j]);
  // modified wavenumbers: -(2 sin(pi k/n)/d)^2 are the eigenvalues of the periodic second difference
  pl->kx2.resize(pl->nkx);
  pl->kz2.resize(nz);
  for (int k = 0; k < pl->nkx; ++k) {
    const double sn = std::sin(M_PI * (double)k / (double)nx);
    pl->kx2[k] = (2.0 * sn / pl->dx) * (2.0 * sn / pl->dx);
  }
  for (int k = 0; k < nz; ++k) {
    const double sn = std::sin(M_PI * (double)k / (double)nz);
    pl->kz2[k] = (2.0 * sn / pl->dz) * (2.0 * sn / pl->dz);
  }
  set_partitions(pl, P, LB);
  // special lines: kx = kz = 0 always; the FP64 low set in mixed precision
  pl->special.push_back(0);
  if (opt.precision == CF_MIXED) {
    for (int kx = 0; kx < std::min(opt.fp64_kx, pl->nkx); ++kx)
      for (int kz = 0; kz < nz; ++kz) {
        const int kzs = std::min(kz, nz - kz);
        if ((kx == 0 && kz == 0) || kzs >= opt.fp64_kz) continue;
        pl->special.push_back(kx * nz + kz);
      }
  }

  // device side
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) {
    delete pl;
    return dev_fail(e, "hipGetDevice");
  }
  int lds_max = 0;
  e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, pl->device);
  if (e != hipSuccess) {
    delete pl;
    return dev_fail(e, "hipDeviceGetAttribute");
  }
  // the static interface-row array of this device (plan creation is the
  // library's set-up call; the device is current here)
  e = scratch_lookup(pl->device);
  if (e != hipSuccess) {
    delete pl;
    return dev_fail(e, "hipGetSymbolAddress (interface-row scratch)");
  }
  const size_t lds_need = cf::ysolve_lds_needed(P * pl->M, P, LB, opt.precision == CF_FP64);
  if (lds_need > (size_t)lds_max) {
    delete pl;
    return fail(CF_ERR_UNSUPPORTED, "partitioning needs " + std::to_string(lds_need) + " bytes of LDS per block");
  }
  auto bail = [&](cf_status s) {
    free_all(pl);
    delete pl;
    return s;
  };
  std::vector<double> rdy(ny);
  for (int j = 0; j < ny; ++j) rdy[j] = 1.0 / pl->dy[j];
  cf_status st;
  e = hipStreamCreateWithFlags(&pl->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->gstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_gin, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_gout, hipEventDisableTiming);
  if (e != hipSuccess) return bail(dev_fail(e, "stream/event creation"));
  if ((st = upload(pl, &pl->d_a, pl->a)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->d_c, pl->c)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->d_dy, pl->dy)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->d_rdy, rdy)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->d_kx2, pl->kx2)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->d_kz2, pl->kz2)) != CF_OK) return bail(st);
  auto tof = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
  if ((st = upload(pl, &pl->s_a, tof(pl->a))) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->s_c, tof(pl->c))) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->s_kx2, tof(pl->kx2))) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->s_kz2, tof(pl->kz2))) != CF_OK) return bail(st);
  std::vector<cx<double>> twz(nz), twx(pl->nh), twp(pl->nh + 1);
  for (int m = 0; m < nz; ++m) twz[m] = unit_root(m, nz);
  for (int m = 0; m < pl->nh; ++m) twx[m] = unit_root(m, pl->nh);
  for (int m = 0; m <= pl->nh; ++m) twp[m] = unit_root(m, nx);
  auto tofc = [](const std::vector<cx<double>>& v) {
    std::vector<cx<float>> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = cf::mk((float)v[i].re, (float)v[i].im);
    return o;
  };
  if ((st = upload(pl, &pl->tw_z64, twz)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->tw_x64, twx)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->twp64, twp)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->tw_z32, tofc(twz))) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->tw_x32, tofc(twx))) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->twp32, tofc(twp))) != CF_OK) return bail(st);
  if (opt.flags & CF_PLAN_Y_DCT) {
    std::vector<cx<double>> twy(ny), wqy(ny);
    for (int m = 0; m < ny; ++m) twy[m] = unit_root(m, ny);
    for (int m = 0; m < ny; ++m) wqy[m] = unit_root(m, 4 * ny);
    // dy as the mean spacing (the faces are uniform to 1e-12)
    const double dyu = (pl->yf[ny] - pl->yf[0]) / ny;
    std::vector<double> lamy(ny + 1);
    for (int m = 0; m <= ny; ++m) {
      const double sn = std::sin(M_PI * (double)m / (double)(2 * ny));
      lamy[m] = -(2.0 * sn / dyu) * (2.0 * sn / dyu);
    }
    if ((st = upload(pl, &pl->tw_y64, twy)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->d_wqy, wqy)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->d_lamy, lamy)) != CF_OK) return bail(st);
  }
  {
    std::vector<double> rdyc(std::max(ny - 1, 1)), wl(std::max(ny - 1, 1)), wu(std::max(ny - 1, 1));
    for (int j = 0; j + 1 < ny; ++j) {
      rdyc[j] = 1.0 / pl->dyc[j];
      wl[j] = pl->dy[j + 1] / (pl->dy[j] + pl->dy[j + 1]);
      wu[j] = pl->dy[j] / (pl->dy[j] + pl->dy[j + 1]);
    }
    if ((st = upload(pl, &pl->d_rdyc, rdyc)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->d_wl, wl)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->d_wu, wu)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->s_rdy, tof(rdy))) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->s_rdyc, tof(rdyc))) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->s_wl, tof(wl))) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->s_wu, tof(wu))) != CF_OK) return bail(st);
    const double rdx = 1.0 / pl->dx, rdz = 1.0 / pl->dz;
    pl->g64 = cf::Geo<double>{pl->d_rdy, pl->d_rdyc, pl->d_wl, pl->d_wu, rdx, rdz, rdx * rdx, rdz * rdz, nx, ny, nz};
    pl->g32 = cf::Geo<float>{pl->s_rdy, pl->s_rdyc, pl->s_wl, pl->s_wu, (float)rdx, (float)rdz,
                             (float)(rdx * rdx), (float)(rdz * rdz), nx, ny, nz};
    std::vector<double> dyc(std::max(ny - 1, 1), 1.0);
    for (int j = 0; j + 1 < ny; ++j) dyc[j] = pl->dyc[j];
    if ((st = upload(pl, &pl->d_dyc, dyc)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->s_dy, tof(pl->dy))) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->s_dyc, tof(dyc))) != CF_OK) return bail(st);
    pl->a64 = cf::AdjGeo<double>{pl->g64, pl->d_dy, pl->d_dyc, pl->d_rdyc};
    pl->a32 = cf::AdjGeo<float>{pl->g32, pl->s_dy, pl->s_dyc, pl->s_rdyc};
  }
  // Workspace.  Step plans: the stage-1 fields and the two spectral buffers
  // share one block (the stage-1 fields are dead while the pressure is solved);
  // adjoint plans: the pressure shares the block of gb.  The FP64 copy of f a
  // mixed solve needs when p aliases f is the pressure workspace of step plans.
  const size_t npts = (size_t)nx * ny * nz;
  const size_t es = (opt.precision == CF_FP64) ? sizeof(double) : sizeof(float);
  const size_t ecs = 2 * es;
  const size_t nspec = (size_t)ny * pl->nkx * nz;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t field_b = al(npts * es), spec_b = al(nspec * ecs);
  if (opt.flags & CF_PLAN_STEP) {
    unsigned char* blk = nullptr;
    if ((st = dalloc(pl, &blk, std::max(3 * field_b, 2 * spec_b))) != CF_OK) return bail(st);
    pl->ub = blk;
    pl->vb = blk + field_b;
    pl->wb = blk + 2 * field_b;
    pl->specA = blk;
    pl->specB = blk + spec_b;
    if (opt.flags & CF_PLAN_ADJOINT) {
      unsigned char *gs = nullptr, *gb = nullptr;
      if ((st = dalloc(pl, &gs, 3 * field_b)) != CF_OK) return bail(st);
      if ((st = dalloc(pl, &gb, std::max(3 * field_b, al(npts * sizeof(double))))) != CF_OK) return bail(st);
      pl->gsu = gs;
      pl->gsv = gs + field_b;
      pl->gsw = gs + 2 * field_b;
      pl->gbu = gb;
      pl->gbv = gb + field_b;
      pl->gbw = gb + 2 * field_b;
      pl->pws = reinterpret_cast<double*>(gb);
    } else {
      if ((st = dalloc(pl, &pl->pws, npts)) != CF_OK) return bail(st);
    }
    pl->fws = pl->pws;
    pl->stat_nch = cf::correct_stats_chunks(nx, ny, nz);
    if ((st = dalloc(pl, &pl->d_stat_part, (size_t)ny * pl->stat_nch * 6)) != CF_OK) return bail(st);
  } else {
    unsigned char *a = nullptr, *b = nullptr;
    if ((st = dalloc(pl, &a, spec_b)) != CF_OK) return bail(st);
    if ((st = dalloc(pl, &b, spec_b)) != CF_OK) return bail(st);
    pl->specA = a;
    pl->specB = b;
    if (opt.precision == CF_MIXED && opt.refine_passes > 0) {
      if ((st = dalloc(pl, &pl->fws, npts)) != CF_OK) return bail(st);
    }
  }
  if (opt.precision == CF_MIXED && opt.refine_passes > 0) {
    const int K = cf::r2c_rows<float>(pl->nh);
    pl->psum_nzb = (nz + K - 1) / K;
    if ((st = dalloc(pl, &pl->d_psum, (size_t)ny * pl->psum_nzb)) != CF_OK) return bail(st);
  }
  if ((st = upload(pl, &pl->d_numflag, std::vector<int>(1, 0))) != CF_OK) return bail(st);
  // block lists of the partitioned solve (room for one line per block, the
  // most any lines_per_block can need)
  if ((st = dalloc(pl, &pl->d_blocks, (size_t)pl->nkx * nz)) != CF_OK) return bail(st);
  if ((st = upload_blocks(pl)) != CF_OK) return bail(st);
  if ((st = upload(pl, &pl->d_special, pl->special)) != CF_OK) return bail(st);
  {
    std::vector<double> den(pl->special.size() * (size_t)ny), cpv(den.size());
    for (size_t l = 0; l < pl->special.size(); ++l)
      special_factors(pl, pl->special[l], den.data() + l * ny, cpv.data() + l * ny);
    if ((st = upload(pl, &pl->d_special_den, den)) != CF_OK) return bail(st);
    if ((st = upload(pl, &pl->d_special_cp, cpv)) != CF_OK) return bail(st);
  }
  if (tune && (st = tune_partitions(pl, (size_t)lds_max)) != CF_OK) return bail(st);
  *out = pl;
  return CF_OK;
}

void cf_plan_destroy(cf_plan* plan) {
  if (!plan) return;
  free_all(plan);
  delete plan;
}

cf_status cf_plan_query(const cf_plan* pl, cf_plan_info* info) {
  CF_TRY(check_plan(pl));
  if (!info) return fail(CF_ERR_ARG, "info is NULL");
  info->nx = pl->nx;
  info->ny = pl->ny;
  info->nz = pl->nz;
  info->precision = pl->opt.precision;
  info->n_parts = pl->P;
  info->rows_per_part = pl->M;
  info->n_lines = (long long)pl->nkx * pl->nz;
  info->n_drop_lines = pl->n_drop;
  info->n_special = (long long)pl->special.size();
  info->k2_threshold = pl->k2drop;
  info->workspace_bytes = pl->bytes;
  info->lines_per_block = pl->LB;
  info->slab_iface_bytes = (size_t)pl->P * 8 * (size_t)pl->nkx * pl->nz * (pl->mixed() ? sizeof(float) : sizeof(double));
  info->drop_parts = pl->G;
  info->n_dropped_lines = pl->n_dropped;
  return CF_OK;
}

cf_status cf_plan_tuning(const cf_plan* pl, int cap, int* count, int* parts, int* lbs, double* us) {
  CF_TRY(check_plan(pl));
  if (!count) return fail(CF_ERR_ARG, "count is NULL");
  if (cap < 0) return fail(CF_ERR_ARG, "cap must be >= 0");
  if (cap > 0 && (!parts || !lbs || !us)) return fail(CF_ERR_ARG, "output arrays are NULL");
  *count = (int)pl->tune.size();
  for (int q = 0; q < cap && q < *count; ++q) {
    parts[q] = pl->tune[q].P;
    lbs[q] = pl->tune[q].LB;
    us[q] = pl->tune[q].us;
  }
  return CF_OK;
}

cf_status cf_forward_spectral(cf_plan* pl, const double* f, void* fhat, void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(f, "f"));
  CF_TRY(check_ptr(fhat, "fhat"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed()) return forward_t<float>(pl, f, static_cast<cx<float>*>(fhat), s);
  return forward_t<double>(pl, f, static_cast<cx<double>*>(fhat), s);
}

cf_status cf_inverse_spectral(cf_plan* pl, const void* phat, double* p, void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(phat, "phat"));
  CF_TRY(check_ptr(p, "p"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed()) return inverse_t<float>(pl, static_cast<const cx<float>*>(phat), p, s);
  return inverse_t<double>(pl, static_cast<const cx<double>*>(phat), p, s);
}

cf_status cf_solve_spectral(cf_plan* pl, const void* fhat, void* phat, void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(fhat, "fhat"));
  CF_TRY(check_ptr(phat, "phat"));
  CF_TRY(check_disjoint(phat, spec_bytes(pl), fhat, spec_bytes(pl), true, "phat must be fhat itself or not overlap it"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed())
    return solve_t<float>(pl, static_cast<const cx<float>*>(fhat), static_cast<cx<float>*>(phat), s);
  return solve_t<double>(pl, static_cast<const cx<double>*>(fhat), static_cast<cx<double>*>(phat), s);
}

cf_status cf_solve_spectral_slabs(cf_plan* pl, int n_slabs, const void* fhat, void* phat, void* iface,
                                  void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(fhat, "fhat"));
  CF_TRY(check_ptr(phat, "phat"));
  CF_TRY(check_disjoint(phat, spec_bytes(pl), fhat, spec_bytes(pl), true, "phat must be fhat itself or not overlap it"));
  CF_TRY(check_ptr(iface, "iface"));
  if (pl->opt.flags & CF_PLAN_Y_DCT) return fail(CF_ERR_ARG, "the y-transform solve has no partitions");
  if (n_slabs < 1 || pl->P % n_slabs != 0)
    return fail(CF_ERR_ARG, "n_slabs must divide the plan's partition count " + std::to_string(pl->P));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed())
    return slabs_t<float>(pl, n_slabs, static_cast<const cx<float>*>(fhat), static_cast<cx<float>*>(phat), iface, s);
  return slabs_t<double>(pl, n_slabs, static_cast<const cx<double>*>(fhat), static_cast<cx<double>*>(phat), iface, s);
}

cf_status cf_solve_spectral_slabs_noalloc(cf_plan* pl, int n_slabs, const void* fhat, void* phat, void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(fhat, "fhat"));
  CF_TRY(check_ptr(phat, "phat"));
  CF_TRY(check_disjoint(phat, spec_bytes(pl), fhat, spec_bytes(pl), true, "phat must be fhat itself or not overlap it"));
  if (pl->opt.flags & CF_PLAN_Y_DCT) return fail(CF_ERR_ARG, "the y-transform solve has no partitions");
  if (n_slabs < 1 || pl->P % n_slabs != 0)
    return fail(CF_ERR_ARG, "n_slabs must divide the plan's partition count " + std::to_string(pl->P));
  const size_t need = (size_t)pl->P * 8 * (size_t)pl->nkx * pl->nz * (pl->mixed() ? sizeof(float) : sizeof(double));
  if (need > kSlabScratchBytes)
    return fail(CF_ERR_ARG, "the plan's interface rows need " + std::to_string(need) + " bytes, more than the " +
                                std::to_string(kSlabScratchBytes) + "-byte static scratch");
  void* iface = scratch_ptr(pl->device);
  if (!iface) return fail(CF_ERR_DEVICE, "no interface-row scratch for the plan's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // no per-kernel timing here: recording it may create events
  const bool timing = pl->timing;
  pl->timing = false;
  const cf_status st =
      pl->mixed() ? slabs_t<float>(pl, n_slabs, static_cast<const cx<float>*>(fhat), static_cast<cx<float>*>(phat), iface, s)
                  : slabs_t<double>(pl, n_slabs, static_cast<const cx<double>*>(fhat), static_cast<cx<double>*>(phat),
                                    iface, s);
  pl->timing = timing;
  return st;
}

cf_status cf_poisson_solve(cf_plan* pl, const double* f, double* p, void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(f, "f"));
  CF_TRY(check_ptr(p, "p"));
  {
    // p is f itself or disjoint from it: a mixed solve reads f again after
    // writing p (the residual), so a partial overlap would read overwritten f
    const uintptr_t bytes = (uintptr_t)pl->nx * pl->ny * pl->nz * sizeof(double);
    const uintptr_t a = reinterpret_cast<uintptr_t>(f), b = reinterpret_cast<uintptr_t>(p);
    if (a != b && a < b + bytes && b < a + bytes) return fail(CF_ERR_ARG, "p must be f itself or not overlap it");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed()) return poisson_mixed(pl, MixedRhs{0, f, nullptr, nullptr, nullptr, 1.0}, p, s);
  return poisson_t<double>(pl, f, p, s);
}

cf_status cf_divergence(cf_plan* pl, const double* u, const double* v, const double* w, double* f,
                        double scale, void* stream) {
  CF_TRY(check_plan(pl));
  CF_TRY(check_ptr(u, "u"));
  CF_TRY(check_ptr(v, "v"));
  CF_TRY(check_ptr(w, "w"));
  CF_TRY(check_ptr(f, "f"));
  if (!std::isfinite(scale)) return fail(CF_ERR_ARG, "scale must be finite");
  for (const double* q : {u, v, w})
    CF_TRY(check_disjoint(f, field_bytes(pl, sizeof(double)), q, field_bytes(pl, sizeof(double)), false,
                          "f must not overlap u, v or w"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  return timed(pl, CF_K_DIVERGENCE, s, "divergence launch", [&] {
    return cf::launch_divergence(u, v, w, f, pl->d_rdy, 1.0 / pl->dx, 1.0 / pl->dz, scale, pl->nx, pl->ny,
                                 pl->nz, s);
  });
}

cf_status cf_projection_step(cf_plan* pl, const void* u, const void* v, const void* w, void* u1, void* v1,
                             void* w1, double* p, double dt, double nu, double fx, void* stream) {
  CF_TRY(check_plan(pl));
  if (!(pl->opt.flags & CF_PLAN_STEP)) return fail(CF_ERR_ARG, "plan was created without CF_PLAN_STEP");
  CF_TRY(check_ptr(u, "u"));
  CF_TRY(check_ptr(v, "v"));
  CF_TRY(check_ptr(w, "w"));
  CF_TRY(check_ptr(u1, "u1"));
  CF_TRY(check_ptr(v1, "v1"));
  CF_TRY(check_ptr(w1, "w1"));
  if (p) CF_TRY(check_ptr(p, "p"));
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CF_ERR_ARG, "dt must be finite and > 0");
  if (!(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(fx)) return fail(CF_ERR_ARG, "nu >= 0 and fx must be finite");
  {
    // the outputs are written while the others are still read: u1, v1, w1
    // pairwise disjoint, and p disjoint from all six velocity arrays
    const size_t nb = (size_t)pl->nx * pl->ny * pl->nz * (pl->mixed() ? sizeof(float) : sizeof(double));
    const void* outs[3] = {u1, v1, w1};
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b)
        if (bytes_overlap(outs[a], nb, outs[b], nb)) return fail(CF_ERR_ARG, "u1, v1, w1 must not overlap");
    if (p) {
      const size_t pb = (size_t)pl->nx * pl->ny * pl->nz * sizeof(double);
      const void* vel[6] = {u, v, w, u1, v1, w1};
      for (const void* q : vel)
        if (bytes_overlap(p, pb, q, nb)) return fail(CF_ERR_ARG, "p must not overlap the velocity arrays");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed())
    return step_mixed(pl, static_cast<const float*>(u), static_cast<const float*>(v), static_cast<const float*>(w),
                      static_cast<float*>(u1), static_cast<float*>(v1), static_cast<float*>(w1), p, dt, nu, fx, s);
  return step64(pl, static_cast<const double*>(u), static_cast<const double*>(v), static_cast<const double*>(w),
                static_cast<double*>(u1), static_cast<double*>(v1), static_cast<double*>(w1), p, dt, nu, fx, s);
}

cf_status cf_rk2_predictor(cf_plan* pl, const void* u, const void* v, const void* w, void* us, void* vs, void* ws,
                           double dt, double nu, double fx, void* stream) {
  CF_TRY(check_plan(pl));
  if (!(pl->opt.flags & CF_PLAN_STEP)) return fail(CF_ERR_ARG, "plan was created without CF_PLAN_STEP");
  const void* ptrs[6] = {u, v, w, us, vs, ws};
  const char* names[6] = {"u", "v", "w", "us", "vs", "ws"};
  for (int q = 0; q < 6; ++q) CF_TRY(check_ptr(ptrs[q], names[q]));
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CF_ERR_ARG, "dt must be finite and > 0");
  if (!(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(fx)) return fail(CF_ERR_ARG, "nu >= 0 and fx must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed())
    return rk2_t<float>(pl, static_cast<const float*>(u), static_cast<const float*>(v), static_cast<const float*>(w),
                        static_cast<float*>(us), static_cast<float*>(vs), static_cast<float*>(ws), pl->g32, float(dt),
                        float(nu), float(fx), s);
  return rk2_t<double>(pl, static_cast<const double*>(u), static_cast<const double*>(v),
                       static_cast<const double*>(w), static_cast<double*>(us), static_cast<double*>(vs),
                       static_cast<double*>(ws), pl->g64, dt, nu, fx, s);
}

cf_status cf_plane_stats(cf_plan* pl, const void* u, const void* v, const void* w, double* stats, void* stream) {
  CF_TRY(check_plan(pl));
  const void* ptrs[4] = {u, v, w, stats};
  const char* names[4] = {"u", "v", "w", "stats"};
  for (int q = 0; q < 4; ++q) CF_TRY(check_ptr(ptrs[q], names[q]));
  const size_t es = pl->mixed() ? sizeof(float) : sizeof(double);
  for (int q = 0; q < 3; ++q)
    CF_TRY(check_disjoint(stats, (size_t)pl->ny * 6 * sizeof(double), ptrs[q], field_bytes(pl, es), false,
                          "stats must not overlap u, v or w"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = pl->mixed() ? cf::launch_plane_stats<float>(static_cast<const float*>(u), static_cast<const float*>(v),
                                                             static_cast<const float*>(w), stats, pl->g32, 0, s)
                             : cf::launch_plane_stats<double>(static_cast<const double*>(u),
                                                              static_cast<const double*>(v),
                                                              static_cast<const double*>(w), stats, pl->g64, 0, s);
  if (e != hipSuccess) return dev_fail(e, "plane statistics launch");
  return CF_OK;
}

namespace {

// One step of the time loop from state a to state b (never the same arrays);
// with acc, the correction pass also adds the plane statistics of b into acc.
cf_status loop_step(cf_plan* pl, void* const a[3], void* const b[3], double* p, double dt, double nu, double fx,
                    double* acc, hipStream_t s) {
  if (pl->mixed())
    return step_mixed(pl, static_cast<const float*>(a[0]), static_cast<const float*>(a[1]),
                      static_cast<const float*>(a[2]), static_cast<float*>(b[0]), static_cast<float*>(b[1]),
                      static_cast<float*>(b[2]), p, dt, nu, fx, s, acc);
  return step64(pl, static_cast<const double*>(a[0]), static_cast<const double*>(a[1]),
                static_cast<const double*>(a[2]), static_cast<double*>(b[0]), static_cast<double*>(b[1]),
                static_cast<double*>(b[2]), p, dt, nu, fx, s, acc);
}

// Records loop_step into an executable graph on the plan's capture stream.
cf_status record_step(cf_plan* pl, void* const a[3], void* const b[3], double* p, double dt, double nu, double fx,
                      double* acc, hipGraphExec_t* out) {
  hipStream_t g = pl->gstream;
  CF_HIP(hipStreamBeginCapture(g, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  const cf_status st = loop_step(pl, a, b, p, dt, nu, fx, acc, g);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(g, &graph);
  if (st != CF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return dev_fail(e, "hipStreamEndCapture");
  const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return dev_fail(ei, "hipGraphInstantiate");
  return CF_OK;
}

}  // namespace

cf_status cf_run_steps(cf_plan* pl, void* u, void* v, void* w, void* u2, void* v2, void* w2, int nsteps, double dt,
                       double nu, double fx, int stats_every, double* stats_acc, double* p, int use_graph,
                       void* stream) {
  CF_TRY(check_plan(pl));
  if (!(pl->opt.flags & CF_PLAN_STEP)) return fail(CF_ERR_ARG, "plan was created without CF_PLAN_STEP");
  void* const A[3] = {u, v, w};
  void* const B[3] = {u2, v2, w2};
  const char* na[3] = {"u", "v", "w"};
  const char* nb[3] = {"u2", "v2", "w2"};
  for (int q = 0; q < 3; ++q) {
    CF_TRY(check_ptr(A[q], na[q]));
    CF_TRY(check_ptr(B[q], nb[q]));
  }
  const uintptr_t bytes = (uintptr_t)pl->nx * pl->ny * pl->nz * (pl->mixed() ? sizeof(float) : sizeof(double));
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const uintptr_t x = reinterpret_cast<uintptr_t>(A[a]), y = reinterpret_cast<uintptr_t>(B[b]);
      if (x < y + bytes && y < x + bytes) return fail(CF_ERR_ARG, "the two state sets must not overlap");
    }
  if (nsteps < 0) return fail(CF_ERR_ARG, "nsteps must be >= 0");
  if (stats_every < 0) return fail(CF_ERR_ARG, "stats_every must be >= 0");
  if (stats_every > 0) CF_TRY(check_ptr(stats_acc, "stats_acc"));
  if (p) CF_TRY(check_ptr(p, "p"));
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CF_ERR_ARG, "dt must be finite and > 0");
  if (!(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(fx)) return fail(CF_ERR_ARG, "nu >= 0 and fx must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto acc_at = [&](int step) -> double* { return (stats_every > 0 && (step + 1) % stats_every == 0) ? stats_acc : nullptr; };
  if (!use_graph) {
    for (int k = 0; k < nsteps; ++k) CF_TRY(loop_step(pl, (k & 1) ? B : A, (k & 1) ? A : B, p, dt, nu, fx, acc_at(k), s));
    return CF_OK;
  }
  if (nsteps == 0) return CF_OK;
  // One recorded step per (parity, statistics or not), found in or added to
  // the plan's cache (at most kMaxGraphs entries; the least recently used one
  // is dropped after the capture stream has drained).  Per-launch event timing
  // is not recorded into graphs.
  constexpr size_t kMaxGraphs = 8;
  auto find = [&](void* const* a, void* const* b, double* acc) -> hipGraphExec_t {
    for (auto& g : pl->graphs)
      if (g.a[0] == a[0] && g.a[1] == a[1] && g.a[2] == a[2] && g.b[0] == b[0] && g.b[1] == b[1] &&
          g.b[2] == b[2] && g.p == p && g.acc == acc && g.dt == dt && g.nu == nu && g.fx == fx) {
        g.last_use = ++pl->graph_clock;
        return g.exec;
      }
    return nullptr;
  };
  hipGraphExec_t ex[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  for (int k = 0; k < nsteps && k < 2 * (stats_every > 0 ? stats_every : 1); ++k) {
    const int par = k & 1, ws = acc_at(k) ? 1 : 0;
    if (ex[par][ws]) continue;
    void* const* a = par ? B : A;
    void* const* b = par ? A : B;
    double* acc = ws ? stats_acc : nullptr;
    ex[par][ws] = find(a, b, acc);
    if (ex[par][ws]) continue;
    if (pl->graphs.size() >= kMaxGraphs) {
      CF_HIP(hipStreamSynchronize(pl->gstream), "hipStreamSynchronize");
      size_t old = 0;
      for (size_t q = 1; q < pl->graphs.size(); ++q)
        if (pl->graphs[q].last_use < pl->graphs[old].last_use) old = q;
      bool in_use = false;
      for (auto& row : ex)
        for (hipGraphExec_t g : row) in_use = in_use || g == pl->graphs[old].exec;
      if (!in_use) {
        (void)hipGraphExecDestroy(pl->graphs[old].exec);
        pl->graphs.erase(pl->graphs.begin() + old);
      }
    }
    const bool timing = pl->timing;
    pl->timing = false;
    hipGraphExec_t g = nullptr;
    const cf_status st = record_step(pl, a, b, p, dt, nu, fx, acc, &g);
    pl->timing = timing;
    CF_TRY(st);
    cf_plan::GraphEntry en;
    for (int q = 0; q < 3; ++q) {
      en.a[q] = a[q];
      en.b[q] = b[q];
    }
    en.p = p;
    en.acc = acc;
    en.dt = dt;
    en.nu = nu;
    en.fx = fx;
    en.exec = g;
    en.last_use = ++pl->graph_clock;
    pl->graphs.push_back(en);
    ex[par][ws] = g;
  }
  hipError_t e = hipEventRecord(pl->ev_gin, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(pl->gstream, pl->ev_gin, 0);
  for (int k = 0; k < nsteps && e == hipSuccess; ++k) e = hipGraphLaunch(ex[k & 1][acc_at(k) ? 1 : 0], pl->gstream);
  if (e == hipSuccess) e = hipEventRecord(pl->ev_gout, pl->gstream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, pl->ev_gout, 0);
  if (e != hipSuccess) return dev_fail(e, "graph replay");
  return CF_OK;
}

cf_status cf_projection_step_adjoint(cf_plan* pl, const void* u, const void* v, const void* w,
                                     const void* gu1, const void* gv1, const void* gw1, void* gu, void* gv,
                                     void* gw, double dt, double nu, double fx, void* stream) {
  CF_TRY(check_plan(pl));
  if (!(pl->opt.flags & CF_PLAN_STEP) || !(pl->opt.flags & CF_PLAN_ADJOINT))
    return fail(CF_ERR_ARG, "plan was created without CF_PLAN_STEP | CF_PLAN_ADJOINT");
  const void* ptrs[9] = {u, v, w, gu1, gv1, gw1, gu, gv, gw};
  const char* names[9] = {"u", "v", "w", "gu1", "gv1", "gw1", "gu", "gv", "gw"};
  for (int q = 0; q < 9; ++q) CF_TRY(check_ptr(ptrs[q], names[q]));
  // the last transposed-stencil pass writes g while it reads the step input's
  // neighbourhoods, so no byte of an output may lie in an input array
  const uintptr_t fbytes = (uintptr_t)pl->nx * pl->ny * pl->nz * (pl->mixed() ? sizeof(float) : sizeof(double));
  for (int q = 6; q < 9; ++q)
    for (int r = 0; r < 3; ++r) {
      const uintptr_t x = reinterpret_cast<uintptr_t>(ptrs[q]), y = reinterpret_cast<uintptr_t>(ptrs[r]);
      if (x < y + fbytes && y < x + fbytes)
        return fail(CF_ERR_ARG, "the gradient output must not overlap the step input");
    }
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CF_ERR_ARG, "dt must be finite and > 0");
  if (!(nu >= 0.0) || !std::isfinite(nu) || !std::isfinite(fx)) return fail(CF_ERR_ARG, "nu >= 0 and fx must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed())
    return step_adjoint_t<float>(pl, static_cast<const float*>(u), static_cast<const float*>(v),
                                 static_cast<const float*>(w), static_cast<const float*>(gu1),
                                 static_cast<const float*>(gv1), static_cast<const float*>(gw1),
                                 static_cast<float*>(gu), static_cast<float*>(gv), static_cast<float*>(gw), dt, nu, fx, s);
  return step_adjoint_t<double>(pl, static_cast<const double*>(u), static_cast<const double*>(v),
                                static_cast<const double*>(w), static_cast<const double*>(gu1),
                                static_cast<const double*>(gv1), static_cast<const double*>(gw1),
                                static_cast<double*>(gu), static_cast<double*>(gv), static_cast<double*>(gw), dt, nu, fx, s);
}

cf_status cf_rhs_adjoint(cf_plan* pl, const void* u, const void* v, const void* w, const void* lu, const void* lv,
                         const void* lw, void* gu, void* gv, void* gw, double nu, void* stream) {
  CF_TRY(check_plan(pl));
  const void* ptrs[9] = {u, v, w, lu, lv, lw, gu, gv, gw};
  const char* names[9] = {"u", "v", "w", "lu", "lv", "lw", "gu", "gv", "gw"};
  for (int q = 0; q < 9; ++q) CF_TRY(check_ptr(ptrs[q], names[q]));
  {
    // the stencil reads neighbours of every output cell: outputs disjoint from
    // the inputs and from each other
    const size_t nb = field_bytes(pl, pl->mixed() ? sizeof(float) : sizeof(double));
    for (int o = 6; o < 9; ++o)
      for (int q = 0; q < 9; ++q)
        if (q != o) CF_TRY(check_disjoint(ptrs[o], nb, ptrs[q], nb, false, "gu, gv, gw must not overlap each other or the inputs"));
  }
  if (!(nu >= 0.0) || !std::isfinite(nu)) return fail(CF_ERR_ARG, "nu must be finite and >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (pl->mixed())
    return timed(pl, CF_K_ADJ_RHS, s, "rhs adjoint", [&] {
      return cf::launch_rhs_adjoint<float>(
          static_cast<const float*>(u), static_cast<const float*>(v), static_cast<const float*>(w),
          static_cast<const float*>(lu), static_cast<const float*>(lv), static_cast<const float*>(lw), nullptr, nullptr,
          nullptr, 1.0f, 0.0f, pl->a32, (float)nu, 1.0f, 0, static_cast<float*>(gu), static_cast<float*>(gv),
          static_cast<float*>(gw), s);
    });
  return timed(pl, CF_K_ADJ_RHS, s, "rhs adjoint", [&] {
    return cf::launch_rhs_adjoint<double>(
        static_cast<const double*>(u), static_cast<const double*>(v), static_cast<const double*>(w),
        static_cast<const double*>(lu), static_cast<const double*>(lv), static_cast<const double*>(lw), nullptr,
        nullptr, nullptr, 1.0, 0.0, pl->a64, nu, 1.0, 0, static_cast<double*>(gu), static_cast<double*>(gv),
        static_cast<double*>(gw), s);
  });
}

cf_status cf_plan_numeric_status(cf_plan* pl, void* stream) {
  CF_TRY(check_plan(pl));
  hipStream_t s = static_cast<hipStream_t>(stream);
  CF_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  CF_HIP(hipStreamSynchronize(pl->aux), "hipStreamSynchronize");
  int flag = 0;
  CF_HIP(hipMemcpy(&flag, pl->d_numflag, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy (numeric flag)");
  if (!flag) return CF_OK;
  const int zero = 0;
  CF_HIP(hipMemcpy(pl->d_numflag, &zero, sizeof(int), hipMemcpyHostToDevice), "hipMemcpy (numeric flag)");
  return fail(CF_ERR_NUMERIC, "a right-hand side of a pressure solve held a non-finite value");
}

cf_status cf_plan_set_timing(cf_plan* pl, int enable) {
  CF_TRY(check_plan(pl));
  if (!enable) CF_TRY(harvest(pl));
  pl->timing = enable != 0;
  return CF_OK;
}

cf_status cf_plan_reset_timing(cf_plan* pl) {
  CF_TRY(check_plan(pl));
  CF_TRY(harvest(pl));
  for (int k = 0; k < CF_K_COUNT; ++k) {
    pl->acc_ms[k] = 0.0;
    pl->acc_n[k] = 0;
  }
  return CF_OK;
}

cf_status cf_plan_get_timing(cf_plan* pl, int kernel, double* total_ms, long long* launches) {
  CF_TRY(check_plan(pl));
  if (kernel < 0 || kernel >= CF_K_COUNT) return fail(CF_ERR_ARG, "kernel class out of range");
  if (!total_ms || !launches) return fail(CF_ERR_ARG, "output pointer is NULL");
  CF_TRY(harvest(pl));
  *total_ms = pl->acc_ms[kernel];
  *launches = pl->acc_n[kernel];
  return CF_OK;
}

const char* cf_kernel_name(int k) {
  static const char* names[CF_K_COUNT] = {"r2c_x",     "fft_z_fwd", "ysolve",      "special_lines",
                                          "fft_z_inv", "c2r_x",     "divergence",  "rk_stage1",
                                          "rk_stage2", "correct",   "rhs_adjoint", "correct_weighted",
                                          "rk2_fused", "slab_local", "slab_finish"};
  return (k >= 0 && k < CF_K_COUNT) ? names[k] : "unknown";
}

}  // extern "C"
