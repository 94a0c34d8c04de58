// Host emulation of the per-thread math of the transform and line-solve
// kernels, built with a plain C++ compiler.  It runs the same Stockham index
// rules, butterflies, real<->half-complex steps and PDD partition/reduced-system
// code as the device kernels (all taken from the shared headers), visiting the
// threads of a line one after another, so the arithmetic of the kernels can be
// checked on a machine without a GPU.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cf_fft.h"
#include "cf_pdd.h"

using cf::cx;
using cf::mk;

namespace {

template <typename T>
std::vector<cx<T>> roots(int n) {
  std::vector<cx<T>> w(n);
  for (int m = 0; m < n; ++m) {
    const long double t = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
    w[m] = mk((T)(double)cosl(t), (T)(double)-sinl(t));
  }
  return w;
}

template <int N, bool INV, typename T, int PASS>
void emul_passes(std::vector<cx<T>>& buf, const cx<T>* tw) {
  constexpr cf::RadixPlan P = cf::make_radix_plan(N);
  constexpr int E = P.e;
  constexpr int TPL = N / E;
  constexpr int R = P.r[PASS];
  constexpr int NS = cf::plan_ns(N, PASS);
  std::vector<cx<T>> nxt(N);
  for (int t = 0; t < TPL; ++t)
    for (int q = 0; q < E / R; ++q) {
      const int b = t + q * TPL;
      cx<T> x[R];
      for (int r = 0; r < R; ++r) x[r] = buf[cf::st_in(N, R, b, r)];
      cf::pass_group<N, R, NS, INV>(x, b, tw);
      for (int r = 0; r < R; ++r) nxt[cf::st_out(R, NS, b, r)] = x[r];
    }
  buf.swap(nxt);
  if constexpr (PASS + 1 < P.np) emul_passes<N, INV, T, PASS + 1>(buf, tw);
}

template <typename T>
bool emul_fft(int n, bool inv, std::vector<cx<T>>& buf) {
  const std::vector<cx<T>> tw = roots<T>(n);
  switch (n) {
#define CF_CASE(NN)                                          \
  case NN:                                                   \
    if (inv) emul_passes<NN, true, T, 0>(buf, tw.data());    \
    else emul_passes<NN, false, T, 0>(buf, tw.data());       \
    return true;
    CF_CASE(2) CF_CASE(3) CF_CASE(4) CF_CASE(6) CF_CASE(8) CF_CASE(12) CF_CASE(16) CF_CASE(24)
    CF_CASE(32) CF_CASE(48) CF_CASE(64) CF_CASE(96) CF_CASE(128) CF_CASE(192) CF_CASE(256)
    CF_CASE(384) CF_CASE(512) CF_CASE(768) CF_CASE(1024) CF_CASE(1536) CF_CASE(2048)
#undef CF_CASE
    default:
      return false;
  }
}

template <typename T>
int fft_c2c(int n, int inv, const double* in, double* out) {
  std::vector<cx<T>> b(n);
  for (int i = 0; i < n; ++i) b[i] = mk((T)in[2 * i], (T)in[2 * i + 1]);
  if (!emul_fft<T>(n, inv != 0, b)) return 1;
  for (int i = 0; i < n; ++i) {
    out[2 * i] = b[i].re;
    out[2 * i + 1] = b[i].im;
  }
  return 0;
}

template <typename T>
int rfft(int nx, const double* x, double* X) {
  const int h = nx / 2;
  std::vector<cx<T>> z(h);
  for (int m = 0; m < h; ++m) z[m] = mk((T)x[2 * m], (T)x[2 * m + 1]);
  if (!emul_fft<T>(h, false, z)) return 1;
  const std::vector<cx<T>> w = roots<T>(nx);
  for (int k = 0; k <= h; ++k) {
    cx<T> v = cf::r2c_post(z[k == h ? 0 : k], z[k == 0 ? 0 : h - k], w[k]);
    X[2 * k] = v.re;
    X[2 * k + 1] = v.im;
  }
  return 0;
}

template <typename T>
int irfft(int nx, const double* X, double* x) {
  const int h = nx / 2;
  const std::vector<cx<T>> w = roots<T>(nx);
  std::vector<cx<T>> z(h);
  for (int m = 0; m < h; ++m) {
    cx<T> a = mk((T)X[2 * m], (T)X[2 * m + 1]);
    cx<T> b = mk((T)X[2 * (h - m)], (T)X[2 * (h - m) + 1]);
    if (m == 0) {
      a.im = T(0);
      b.im = T(0);
    }
    z[m] = cf::c2r_pre(a, b, w[m]);
  }
  if (!emul_fft<T>(h, true, z)) return 1;
  const T s = T(1.0 / nx);
  for (int m = 0; m < h; ++m) {
    x[2 * m] = z[m].re * s;
    x[2 * m + 1] = z[m].im * s;
  }
  return 0;
}

template <int M, typename T>
void pdd_line_m(int P, const T* a, const T* c, T k2, int exact, std::vector<cx<T>>& d) {
  std::vector<std::vector<T>> v(P, std::vector<T>(M)), w(P, std::vector<T>(M));
  for (int i = 0; i < P; ++i) cf::pdd_local<M, T>(a + i * M, c + i * M, k2, d.data() + i * M, v[i].data(), w[i].data());
  const int Q = P - 1;
  std::vector<cx<T>> y1(P, mk(T(0), T(0))), y2(P, mk(T(0), T(0)));
  if (!exact) {
    for (int i = 0; i < Q; ++i)
      cf::pdd_cramer(w[i][M - 1], v[i + 1][0], d[i * M + M - 1], d[(i + 1) * M], y1[i], y2[i]);
  } else if (Q > 0) {
    std::vector<cf::zrow<T>> z(Q), zn(Q);
    for (int i = 0; i < Q; ++i)
      z[i] = cf::zrow_make(v[i][M - 1], w[i][M - 1], v[i + 1][0], w[i + 1][0], d[i * M + M - 1], d[(i + 1) * M]);
    for (int st = 1; st < Q; st *= 2) {
      for (int i = 0; i < Q; ++i) {
        const bool hl = i - st >= 0, hh = i + st < Q;
        zn[i] = cf::zrow_reduce(z[i], &z[hl ? i - st : i], hl, &z[hh ? i + st : i], hh);
      }
      z.swap(zn);
    }
    for (int i = 0; i < Q; ++i) cf::zrow_finish(z[i], y1[i], y2[i]);
  }
  for (int i = 0; i < P; ++i) {
    const cx<T> yp = i > 0 ? y1[i - 1] : mk(T(0), T(0));
    const cx<T> yn = i < Q ? y2[i] : mk(T(0), T(0));
    cf::pdd_correct<M, T>(d.data() + i * M, v[i].data(), w[i].data(), yp, yn);
  }
}

// The dropped reduced system as an outer PDD of G groups of Pg = P/G inner
// partitions, in the order of the y kernel: inner interfaces of each group by
// cyclic reduction with the three right-hand sides, the groups' end values, the
// dropped 2x2 step on the outer interfaces, and the correction with the
// effective interface values.
template <int M, typename T>
void pdd_line_grouped_m(int P, int G, const T* a, const T* c, T k2, std::vector<cx<T>>& d) {
  std::vector<std::vector<T>> v(P, std::vector<T>(M)), w(P, std::vector<T>(M));
  for (int i = 0; i < P; ++i) cf::pdd_local<M, T>(a + i * M, c + i * M, k2, d.data() + i * M, v[i].data(), w[i].data());
  const int Pg = P / G;
  const cx<T> z0 = mk(T(0), T(0));
  std::vector<cx<T>> y1(P, z0), y2(P, z0);
  std::vector<T> y1v(P, T(0)), y2v(P, T(0)), y1w(P, T(0)), y2w(P, T(0));
  for (int g = 0; g < G; ++g) {
    const int sf = g * Pg, sl = sf + Pg - 1;
    std::vector<cf::zrow3<T>> z(P), zn(P);
    for (int i = sf; i < sl; ++i) {
      z[i].z = cf::zrow_make(v[i][M - 1], w[i][M - 1], v[i + 1][0], w[i + 1][0], d[i * M + M - 1], d[(i + 1) * M]);
      z[i].rv0 = (i == sf) ? v[i][M - 1] : T(0);
      z[i].rv1 = T(0);
      z[i].rw0 = T(0);
      z[i].rw1 = (i + 1 == sl) ? w[i + 1][0] : T(0);
    }
    for (int st = 1; st < Pg - 1; st *= 2) {
      for (int i = sf; i < sl; ++i) {
        const bool hl = i - st >= sf, hh = i + st < sl;
        zn[i] = cf::zrow3_reduce(z[i], &z[hl ? i - st : i], hl, &z[hh ? i + st : i], hh);
      }
      for (int i = sf; i < sl; ++i) z[i] = zn[i];
    }
    for (int i = sf; i < sl; ++i) cf::zrow3_finish(z[i], y1[i], y2[i], y1v[i], y2v[i], y1w[i], y2w[i]);
  }
  std::vector<cx<T>> gxm(G), gx1(G), Y1(G, z0), Y2(G, z0);
  std::vector<T> gwm(G), gv1(G);
  for (int g = 0; g < G; ++g) {
    const int sf = g * Pg, sl = sf + Pg - 1;
    const cx<T> y1p = sl > sf ? y1[sl - 1] : z0;
    const T y1wp = sl > sf ? y1w[sl - 1] : T(0);
    gxm[g] = d[sl * M + M - 1] - y1p * v[sl][M - 1];
    gwm[g] = w[sl][M - 1] - v[sl][M - 1] * y1wp;
    gx1[g] = d[sf * M] - y2[sf] * w[sf][0];
    gv1[g] = v[sf][0] - w[sf][0] * y2v[sf];
  }
  for (int g = 0; g + 1 < G; ++g) cf::pdd_cramer(gwm[g], gv1[g + 1], gxm[g], gx1[g + 1], Y1[g], Y2[g]);
  for (int i = 0; i < P; ++i) {
    const int g = i / Pg, sf = g * Pg, sl = sf + Pg - 1;
    const cx<T> Y1p = g > 0 ? Y1[g - 1] : z0;
    const cx<T> Y2n = g + 1 < G ? Y2[g] : z0;
    const bool prev_in = i > sf;
    const cx<T> y1i = prev_in ? y1[i - 1] : z0;
    const T y1vi = prev_in ? y1v[i - 1] : T(0), y1wi = prev_in ? y1w[i - 1] : T(0);
    const cx<T> y1eff = y1i + Y1p * ((i == sf ? T(1) : T(0)) - y1vi) - Y2n * y1wi;
    const cx<T> y2eff = y2[i] - Y1p * y2v[i] + Y2n * ((i == sl ? T(1) : T(0)) - y2w[i]);
    cf::pdd_correct<M, T>(d.data() + i * M, v[i].data(), w[i].data(), y1eff, y2eff);
  }
}

// Both line emulations split the ny rows into P partitions of M = ceil(ny/P)
// rows like the plan: the rows past ny complete the last partition with
// a = c = 0 and a zero right-hand side.
template <typename T>
int pdd_line_grouped(int ny, int P, int G, const double* a, const double* c, double k2, const double* din,
                     double* xout) {
  if (P < 1 || G < 1 || P % G) return 1;
  const int M = (ny + P - 1) / P;
  if ((P - 1) * M >= ny) return 1;
  std::vector<T> at(P * M, T(0)), ct(P * M, T(0));
  std::copy(a, a + ny, at.begin());
  std::copy(c, c + ny, ct.begin());
  std::vector<cx<T>> d(P * M, mk(T(0), T(0)));
  for (int j = 0; j < ny; ++j) d[j] = mk((T)din[2 * j], (T)din[2 * j + 1]);
  switch (M) {
#define CF_CASE(MM)                                                         \
  case MM:                                                                  \
    pdd_line_grouped_m<MM, T>(P, G, at.data(), ct.data(), (T)k2, d);        \
    break;
    CF_CASE(1) CF_CASE(2) CF_CASE(3) CF_CASE(4) CF_CASE(6) CF_CASE(8) CF_CASE(12) CF_CASE(16)
#undef CF_CASE
    default:
      return 2;
  }
  for (int j = 0; j < ny; ++j) {
    xout[2 * j] = d[j].re;
    xout[2 * j + 1] = d[j].im;
  }
  return 0;
}

template <typename T>
int pdd_line(int ny, int P, const double* a, const double* c, double k2, int exact, const double* din,
             double* xout) {
  if (P < 1) return 1;
  const int M = (ny + P - 1) / P;
  if ((P - 1) * M >= ny) return 1;
  std::vector<T> at(P * M, T(0)), ct(P * M, T(0));
  std::copy(a, a + ny, at.begin());
  std::copy(c, c + ny, ct.begin());
  std::vector<cx<T>> d(P * M, mk(T(0), T(0)));
  for (int j = 0; j < ny; ++j) d[j] = mk((T)din[2 * j], (T)din[2 * j + 1]);
  switch (M) {
#define CF_CASE(MM)                                                     \
  case MM:                                                              \
    pdd_line_m<MM, T>(P, at.data(), ct.data(), (T)k2, exact, d);        \
    break;
    CF_CASE(1) CF_CASE(2) CF_CASE(3) CF_CASE(4) CF_CASE(6) CF_CASE(8) CF_CASE(12) CF_CASE(16)
#undef CF_CASE
    default:
      return 2;
  }
  for (int j = 0; j < ny; ++j) {
    xout[2 * j] = d[j].re;
    xout[2 * j + 1] = d[j].im;
  }
  return 0;
}

}  // namespace

extern "C" {

// Complex transform of length n (interleaved re/im), forward (inv = 0, sign -1,
// unnormalised) or inverse (sign +1, unnormalised), in FP64 or FP32 arithmetic.
int cfh_fft_c2c(int n, int inv, int fp32, const double* in, double* out) {
  return fp32 ? fft_c2c<float>(n, inv, in, out) : fft_c2c<double>(n, inv, in, out);
}

// Real transform of length nx through the half-length complex transform:
// X[0..nx/2] (interleaved), unnormalised.
int cfh_rfft(int nx, int fp32, const double* x, double* X) {
  return fp32 ? rfft<float>(nx, x, X) : rfft<double>(nx, x, X);
}

// Inverse of cfh_rfft, normalised by 1/nx.
int cfh_irfft(int nx, int fp32, const double* X, double* x) {
  return fp32 ? irfft<float>(nx, X, x) : irfft<double>(nx, X, x);
}

// One wall-normal line through the PDD solve of the y kernel: P partitions,
// exact (cyclic reduction) or dropped (2x2 Cramer) reduced system.
int cfh_pdd_line(int ny, int P, const double* a, const double* c, double k2, int exact, int fp32,
                 const double* d, double* x) {
  return fp32 ? pdd_line<float>(ny, P, a, c, k2, exact, d, x) : pdd_line<double>(ny, P, a, c, k2, exact, d, x);
}

// The same line with the dropped reduced system taken as an outer PDD of G
// groups of P/G partitions (exact inside each group).
int cfh_pdd_line_grouped(int ny, int P, int G, const double* a, const double* c, double k2, int fp32,
                         const double* d, double* x) {
  return fp32 ? pdd_line_grouped<float>(ny, P, G, a, c, k2, d, x) : pdd_line_grouped<double>(ny, P, G, a, c, k2, d, x);
}

// The work item that block b of a launch takes (groups of n items, each XCD
// on a contiguous run of every group): the index map of the row-block and
// stencil-tile launches.
int cfh_xcd_slab_block(int b, int n) { return cf::xcd_slab_block(b, n); }

}
