// Per-thread math of the Stockham radix FFTs used in the periodic directions
// (Section 2.1, Eq. (9): a real DFT along x, a complex DFT along z).
//
// A length-N transform (N = 2^a or 3 * 2^a) is a sequence of radix-R passes.
// Pass with radix R at sub-transform length NS (the product of the radices of
// the earlier passes) maps, for every butterfly b in [0, N/R):
//     inputs   x_r = in[b + r N/R],                     r = 0..R-1
//     twiddle  x_r *= w_{NS R}^{(b mod NS) r}           (w_M = exp(-2 pi i / M))
//     DFT_R over r
//     outputs  out[(b div NS) NS R + (b mod NS) + r NS] = y_r
// which leaves the result in natural order after the last pass (Stockham
// autosort).  A thread owns E = lcm(radices) elements and runs E/R butterflies
// b = t + q T (q < E/R, T = N/E threads per line) in every pass.
//
// The index rules and butterflies here are shared by the device kernels and
// by a host emulation used in the CPU tests.
#pragma once

#include "cf_common.h"

namespace cf {

struct RadixPlan {
  int np;      // number of passes
  int r[16];   // radix of each pass
  int e;       // elements per thread
};

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }

// Radices for N = 2^a (greedy 16s, then one smaller power of two) or
// N = 3 * 2^a (8s, one smaller power of two, then a radix-3 pass).
constexpr RadixPlan make_radix_plan(int n) {
  RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, 1};
  int m = n;
  bool three = (m % 3 == 0);
  if (three) m /= 3;
  if (!three) {
    while (m >= 16) { p.r[p.np++] = 16; m /= 16; }
    if (m > 1) p.r[p.np++] = m;
  } else {
    while (m >= 8) { p.r[p.np++] = 8; m /= 8; }
    if (m > 1) p.r[p.np++] = m;
    p.r[p.np++] = 3;
  }
  int e = 1;
  for (int i = 0; i < p.np; ++i) e = clcm(e, p.r[i]);
  p.e = e;
  return p;
}

// Sub-transform length before pass `pass`.
constexpr int plan_ns(int n, int pass) {
  RadixPlan p = make_radix_plan(n);
  int ns = 1;
  for (int i = 0; i < pass; ++i) ns *= p.r[i];
  return ns;
}

constexpr bool fft_len_supported(int n) {
  if (n < 2 || n > 4096) return false;
  int m = n;
  if (m % 3 == 0) m /= 3;
  return (m & (m - 1)) == 0 && m >= 1 && (n % 9 != 0);
}

CF_HD int st_in(int n, int r_radix, int b, int r) { return b + r * (n / r_radix); }
CF_HD int st_out(int r_radix, int ns, int b, int r) { return (b / ns) * ns * r_radix + (b % ns) + r * ns; }
CF_HD int st_tw(int n, int r_radix, int ns, int b, int r) { return (b % ns) * r * (n / (ns * r_radix)); }

// ---------------------------------------------------------------- butterflies
template <bool INV, typename T> CF_HD void bfly2(cx<T>* x) {
  cx<T> a = x[0], b = x[1];
  x[0] = a + b;
  x[1] = a - b;
}

template <bool INV, typename T> CF_HD void bfly3(cx<T>* x) {
  const T h = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
  cx<T> t = x[1] + x[2];
  cx<T> s = mul_mi<INV>((x[1] - x[2]) * h);
  cx<T> m = x[0] - t * T(0.5);
  x[0] = x[0] + t;
  x[1] = m + s;
  x[2] = m - s;
}

template <bool INV, typename T> CF_HD void bfly4(cx<T>* x) {
  cx<T> t0 = x[0] + x[2], t1 = x[0] - x[2];
  cx<T> t2 = x[1] + x[3], t3 = mul_mi<INV>(x[1] - x[3]);
  x[0] = t0 + t2;
  x[2] = t0 - t2;
  x[1] = t1 + t3;
  x[3] = t1 - t3;
}

// multiply by w_8^k (forward sign) for k = 1, 3
template <bool INV, typename T> CF_HD cx<T> w8_1(cx<T> a) {
  const T r = T(0.70710678118654752440084436210485);
  return INV ? mk((a.re - a.im) * r, (a.re + a.im) * r) : mk((a.re + a.im) * r, (a.im - a.re) * r);
}
template <bool INV, typename T> CF_HD cx<T> w8_3(cx<T> a) {
  const T r = T(0.70710678118654752440084436210485);
  return INV ? mk(-(a.re + a.im) * r, (a.re - a.im) * r) : mk((a.im - a.re) * r, -(a.re + a.im) * r);
}

template <bool INV, typename T> CF_HD void bfly8(cx<T>* x) {
  cx<T> e[4] = {x[0], x[2], x[4], x[6]};
  cx<T> o[4] = {x[1], x[3], x[5], x[7]};
  bfly4<INV>(e);
  bfly4<INV>(o);
  o[1] = w8_1<INV>(o[1]);
  o[2] = mul_mi<INV>(o[2]);
  o[3] = w8_3<INV>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = e[k] + o[k];
    x[k + 4] = e[k] - o[k];
  }
}

template <bool INV, typename T> CF_HD void bfly16(cx<T>* x) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = x[2 * k];
    o[k] = x[2 * k + 1];
  }
  bfly8<INV>(e);
  bfly8<INV>(o);
  const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
  const T sg = INV ? T(1) : T(-1);
  o[1] = cmul(o[1], mk(c1, sg * s1));
  o[2] = w8_1<INV>(o[2]);
  o[3] = cmul(o[3], mk(s1, sg * c1));
  o[4] = mul_mi<INV>(o[4]);
  o[5] = cmul(o[5], mk(-s1, sg * c1));
  o[6] = w8_3<INV>(o[6]);
  o[7] = cmul(o[7], mk(-c1, sg * s1));
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = e[k] + o[k];
    x[k + 8] = e[k] - o[k];
  }
}

template <int R, bool INV, typename T> CF_HD void bfly(cx<T>* x) {
  if constexpr (R == 2) bfly2<INV>(x);
  else if constexpr (R == 3) bfly3<INV>(x);
  else if constexpr (R == 4) bfly4<INV>(x);
  else if constexpr (R == 8) bfly8<INV>(x);
  else if constexpr (R == 16) bfly16<INV>(x);
}

// Twiddle and butterfly of one radix-R group; tw is the length-N table of
// w_N^m (forward sign), conjugated for the inverse.
template <int N, int R, int NS, bool INV, typename T>
CF_HD void pass_group(cx<T>* x, int b, const cx<T>* tw) {
  if constexpr (NS > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cx<T> w = tw[st_tw(N, R, NS, b, r)];
      x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
    }
  }
  bfly<R, INV>(x);
}

// ---------------------------------------------------------------- real <-> half-complex
// Forward real transform of length 2H from the length-H complex transform Z of
// z_m = x_{2m} + i x_{2m+1}:  X_k = 1/2 [(A + B) - i w^k (A - B)],
// A = Z_k, B = conj(Z_{H-k}) (Z_H = Z_0), w = exp(-2 pi i/(2H)), k = 0..H.
template <typename T> CF_HD cx<T> r2c_post(cx<T> zk, cx<T> zhk, cx<T> wk) {
  cx<T> A = zk, B = conj(zhk);
  cx<T> s = A + B, d = A - B;
  cx<T> t = mul_mi<false>(cmul(wk, d));
  return (s + t) * T(0.5);
}

// Inverse: from X_k, X_{H-k} (k = 0..H-1) build 2 Z_k = (A + B) + i conj(w^k)(A - B),
// A = X_k, B = conj(X_{H-k}); at k = 0 only the real parts of X_0 and X_H enter.
template <typename T> CF_HD cx<T> c2r_pre(cx<T> xk, cx<T> xhk, cx<T> wk) {
  cx<T> A = xk, B = conj(xhk);
  cx<T> s = A + B, d = A - B;
  cx<T> t = mul_mi<true>(cmulc(d, wk));
  return s + t;
}

}  // namespace cf
