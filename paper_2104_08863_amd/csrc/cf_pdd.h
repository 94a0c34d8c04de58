// Per-thread math of the PDD partitioned tridiagonal solve (Section 2.2,
// Eq. (10)-(21) and the five steps that follow them).
//
// A wall-normal line of ny rows, a_j p_{j-1} + b_j p_j + c_j p_{j+1} = d_j with
// b_j = -(a_j + c_j) - k^2, is cut into P partitions of M rows.  Partition i
// solves, with its own diagonal block A_i (Eq. (20)),
//     A_i [xt, v, w] = [d^i, a_1^i e_1, c_M^i e_M]
// by one forward elimination shared by the three right-hand sides.  The
// interfaces i = 0..P-2 then satisfy the reduced system Z y = E^T xt of
// Eq. (21), unknowns y1^i = x_M^i and y2^i = x_1^{i+1}:
//     y1^i + v_M^i y1^{i-1} + w_M^i y2^i         = xt_M^i
//     y2^i + v_1^{i+1} y1^i + w_1^{i+1} y2^{i+1} = xt_1^{i+1}
// i.e. a 2x2-block tridiagonal system with diagonal block D_i = [[1, w_M^i],
// [v_1^{i+1}, 1]], lower block L_i = [[v_M^i, 0], [0, 0]] and upper block
// U_i = [[0, 0], [0, w_1^{i+1}]].  Dropping the corner terms v_M^i, w_1^{i+1}
// leaves the independent 2x2 blocks of step 4 (Cramer's rule); keeping them
// gives the exact solution, obtained here by block cyclic reduction across the
// interfaces.  Step 5: x^i = xt^i - v^i y1^{i-1} - w^i y2^i.
#pragma once

#include "cf_common.h"

namespace cf {

template <typename T>
struct m22 {
  T a, b, c, d;  // [[a, b], [c, d]]
};

template <typename T> CF_HD m22<T> m22_mul(m22<T> x, m22<T> y) {
  return m22<T>{x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d,
                x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
template <typename T> CF_HD m22<T> m22_add(m22<T> x, m22<T> y) {
  return m22<T>{x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d};
}
template <typename T> CF_HD m22<T> m22_inv(m22<T> x) {
  T r = rcp(x.a * x.d - x.b * x.c);
  return m22<T>{x.d * r, -x.b * r, -x.c * r, x.a * r};
}
template <typename T> CF_HD m22<T> m22_neg(m22<T> x) { return m22<T>{-x.a, -x.b, -x.c, -x.d}; }
template <typename T> CF_HD void m22_mv(m22<T> m, cx<T> u0, cx<T> u1, cx<T>& o0, cx<T>& o1) {
  o0 = u0 * m.a + u1 * m.b;
  o1 = u0 * m.c + u1 * m.d;
}

// One row of the reduced system, owned by the thread of the partition below
// the interface.
template <typename T>
struct zrow {
  m22<T> L, D, U;
  cx<T> r0, r1;
};

// Structure-of-arrays storage of reduced-system rows (16 planes of n values),
// so that neighbouring lanes touch neighbouring addresses.
template <typename T>
struct zrow_soa {
  T* base;
  int n;
  CF_HD void put(int k, const zrow<T>& z) const {
    T* p = base + k;
    const T v[16] = {z.L.a, z.L.b, z.L.c, z.L.d, z.D.a, z.D.b, z.D.c, z.D.d,
                     z.U.a, z.U.b, z.U.c, z.U.d, z.r0.re, z.r0.im, z.r1.re, z.r1.im};
#pragma unroll
    for (int f = 0; f < 16; ++f) p[f * n] = v[f];
  }
  CF_HD zrow<T> get(int k) const {
    const T* p = base + k;
    zrow<T> z;
    z.L = m22<T>{p[0 * n], p[1 * n], p[2 * n], p[3 * n]};
    z.D = m22<T>{p[4 * n], p[5 * n], p[6 * n], p[7 * n]};
    z.U = m22<T>{p[8 * n], p[9 * n], p[10 * n], p[11 * n]};
    z.r0 = mk(p[12 * n], p[13 * n]);
    z.r1 = mk(p[14 * n], p[15 * n]);
    return z;
  }
};

// Local solves of one partition (Eq. (20)): arow[s] = a_{j0+s}, crow[s] =
// c_{j0+s} (s = 0..M-1).  On entry d holds the right-hand side; on exit d
// holds xt, and v, w the two spike columns.
template <int M, typename T>
CF_HD void pdd_local(const T* arow, const T* crow, T k2, cx<T>* d, T* v, T* w) {
  T cp[M];
  T rlast = T(0);
#pragma unroll
  for (int s = 0; s < M; ++s) {
    T as = arow[s], cs = crow[s];
    T bs = -(as + cs) - k2;
    T cin = (s == M - 1) ? T(0) : cs;
    T den = (s == 0) ? bs : bs - as * cp[s - 1];
    T rden = rcp(den);
    cp[s] = cin * rden;
    if (s == 0) {
      d[0] = d[0] * rden;
      v[0] = as * rden;
    } else {
      d[s] = (d[s] - d[s - 1] * as) * rden;
      v[s] = -(as * v[s - 1]) * rden;
    }
    if (s == M - 1) rlast = rden;
  }
  w[M - 1] = crow[M - 1] * rlast;
#pragma unroll
  for (int s = M - 2; s >= 0; --s) {
    d[s] = d[s] - d[s + 1] * cp[s];
    v[s] = v[s] - cp[s] * v[s + 1];
    w[s] = -(cp[s] * w[s + 1]);
  }
}

// The spike columns v, w of pdd_local alone (the same operations in the same
// order, so bitwise the same values): the y kernel keeps only their end values
// through the reduced solve and rebuilds them for step 5, which frees the
// registers of 2M values while the reduced system is solved.
template <int M, typename T>
CF_HD void pdd_spikes(const T* arow, const T* crow, T k2, T* v, T* w) {
  T cp[M];
  T rlast = T(0);
#pragma unroll
  for (int s = 0; s < M; ++s) {
    T as = arow[s], cs = crow[s];
    T bs = -(as + cs) - k2;
    T cin = (s == M - 1) ? T(0) : cs;
    T den = (s == 0) ? bs : bs - as * cp[s - 1];
    T rden = rcp(den);
    cp[s] = cin * rden;
    v[s] = (s == 0) ? as * rden : -(as * v[s - 1]) * rden;
    if (s == M - 1) rlast = rden;
  }
  w[M - 1] = crow[M - 1] * rlast;
#pragma unroll
  for (int s = M - 2; s >= 0; --s) {
    v[s] = v[s] - cp[s] * v[s + 1];
    w[s] = -(cp[s] * w[s + 1]);
  }
}

// Step 4 with the corner terms dropped: Cramer's rule on D_i.
template <typename T>
CF_HD void pdd_cramer(T wm, T v1n, cx<T> xm, cx<T> x1n, cx<T>& y1, cx<T>& y2) {
  T rdet = rcp(T(1) - wm * v1n);
  y1 = (xm - x1n * wm) * rdet;
  y2 = (x1n - xm * v1n) * rdet;
}

template <typename T>
CF_HD zrow<T> zrow_make(T vm, T wm, T v1n, T w1n, cx<T> xm, cx<T> x1n) {
  zrow<T> z;
  z.L = m22<T>{vm, T(0), T(0), T(0)};
  z.D = m22<T>{T(1), wm, v1n, T(1)};
  z.U = m22<T>{T(0), T(0), T(0), w1n};
  z.r0 = xm;
  z.r1 = x1n;
  return z;
}

// One cyclic-reduction step: eliminate the couplings of row `me` to rows *lo
// and *hi (has_lo / has_hi false at the ends of the interface range).
template <typename T>
CF_HD zrow<T> zrow_reduce(const zrow<T>& me, const zrow<T>* lo, bool has_lo,
                          const zrow<T>* hi, bool has_hi) {
  zrow<T> o;
  o.D = me.D;
  o.r0 = me.r0;
  o.r1 = me.r1;
  o.L = m22<T>{T(0), T(0), T(0), T(0)};
  o.U = m22<T>{T(0), T(0), T(0), T(0)};
  if (has_lo) {
    const m22<T> al = m22_neg(m22_mul(me.L, m22_inv(lo->D)));
    o.L = m22_mul(al, lo->L);
    o.D = m22_add(o.D, m22_mul(al, lo->U));
    cx<T> t0, t1;
    m22_mv(al, lo->r0, lo->r1, t0, t1);
    o.r0 = o.r0 + t0;
    o.r1 = o.r1 + t1;
  }
  if (has_hi) {
    const m22<T> be = m22_neg(m22_mul(me.U, m22_inv(hi->D)));
    o.U = m22_mul(be, hi->U);
    o.D = m22_add(o.D, m22_mul(be, hi->L));
    cx<T> t0, t1;
    m22_mv(be, hi->r0, hi->r1, t0, t1);
    o.r0 = o.r0 + t0;
    o.r1 = o.r1 + t1;
  }
  return o;
}

template <typename T>
CF_HD void zrow_finish(const zrow<T>& z, cx<T>& y1, cx<T>& y2) {
  m22_mv(m22_inv(z.D), z.r0, z.r1, y1, y2);
}

// Reduced-system rows carrying two more (real) right-hand sides next to the
// complex one: the two-level solve (a group of consecutive partitions solved
// exactly as one partition of an outer PDD) needs, besides the group's own
// solution, its two spike columns, whose partition-level right-hand sides are
// the first partition's v and the last partition's w.  The matrix part is
// reduced once for all three.
template <typename T>
struct zrow3 {
  zrow<T> z;
  T rv0, rv1, rw0, rw1;
};

// SoA storage of zrow3 (20 planes of n values; planes 0..15 as zrow_soa).
template <typename T>
struct zrow3_soa {
  T* base;
  int n;
  CF_HD void put(int k, const zrow3<T>& z) const {
    zrow_soa<T>{base, n}.put(k, z.z);
    T* p = base + 16 * n + k;
    p[0] = z.rv0;
    p[n] = z.rv1;
    p[2 * n] = z.rw0;
    p[3 * n] = z.rw1;
  }
  CF_HD zrow3<T> get(int k) const {
    zrow3<T> z;
    z.z = zrow_soa<T>{base, n}.get(k);
    const T* p = base + 16 * n + k;
    z.rv0 = p[0];
    z.rv1 = p[n];
    z.rw0 = p[2 * n];
    z.rw1 = p[3 * n];
    return z;
  }
};

template <typename T>
CF_HD void m22_mvr(m22<T> m, T u0, T u1, T& o0, T& o1) {
  o0 = m.a * u0 + m.b * u1;
  o1 = m.c * u0 + m.d * u1;
}

// zrow_reduce with the two real right-hand sides carried along.
template <typename T>
CF_HD zrow3<T> zrow3_reduce(const zrow3<T>& me, const zrow3<T>* lo, bool has_lo, const zrow3<T>* hi,
                            bool has_hi) {
  zrow3<T> o;
  o.z.D = me.z.D;
  o.z.r0 = me.z.r0;
  o.z.r1 = me.z.r1;
  o.rv0 = me.rv0;
  o.rv1 = me.rv1;
  o.rw0 = me.rw0;
  o.rw1 = me.rw1;
  o.z.L = m22<T>{T(0), T(0), T(0), T(0)};
  o.z.U = m22<T>{T(0), T(0), T(0), T(0)};
  if (has_lo) {
    const m22<T> al = m22_neg(m22_mul(me.z.L, m22_inv(lo->z.D)));
    o.z.L = m22_mul(al, lo->z.L);
    o.z.D = m22_add(o.z.D, m22_mul(al, lo->z.U));
    cx<T> t0, t1;
    m22_mv(al, lo->z.r0, lo->z.r1, t0, t1);
    o.z.r0 = o.z.r0 + t0;
    o.z.r1 = o.z.r1 + t1;
    T s0, s1;
    m22_mvr(al, lo->rv0, lo->rv1, s0, s1);
    o.rv0 += s0;
    o.rv1 += s1;
    m22_mvr(al, lo->rw0, lo->rw1, s0, s1);
    o.rw0 += s0;
    o.rw1 += s1;
  }
  if (has_hi) {
    const m22<T> be = m22_neg(m22_mul(me.z.U, m22_inv(hi->z.D)));
    o.z.U = m22_mul(be, hi->z.U);
    o.z.D = m22_add(o.z.D, m22_mul(be, hi->z.L));
    cx<T> t0, t1;
    m22_mv(be, hi->z.r0, hi->z.r1, t0, t1);
    o.z.r0 = o.z.r0 + t0;
    o.z.r1 = o.z.r1 + t1;
    T s0, s1;
    m22_mvr(be, hi->rv0, hi->rv1, s0, s1);
    o.rv0 += s0;
    o.rv1 += s1;
    m22_mvr(be, hi->rw0, hi->rw1, s0, s1);
    o.rw0 += s0;
    o.rw1 += s1;
  }
  return o;
}

template <typename T>
CF_HD void zrow3_finish(const zrow3<T>& z, cx<T>& y1, cx<T>& y2, T& y1v, T& y2v, T& y1w, T& y2w) {
  const m22<T> inv = m22_inv(z.z.D);
  m22_mv(inv, z.z.r0, z.z.r1, y1, y2);
  m22_mvr(inv, z.rv0, z.rv1, y1v, y2v);
  m22_mvr(inv, z.rw0, z.rw1, y1w, y2w);
}

// Step 5.
template <int M, typename T>
CF_HD void pdd_correct(cx<T>* x, const T* v, const T* w, cx<T> y1prev, cx<T> y2) {
#pragma unroll
  for (int s = 0; s < M; ++s) x[s] = x[s] - y1prev * v[s] - y2 * w[s];
}

}  // namespace cf
