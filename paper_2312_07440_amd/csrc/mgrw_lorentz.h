// Lorentz and Dirac building blocks of tree-level helicity amplitudes.
//
// Conventions: metric (+,-,-,-); chiral gamma matrices
//   gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]],  sigma^mu = (1, s),
//   sigmabar^mu = (1, -s), upper two spinor components left-handed.
// A slashed vector a = gamma^mu a_mu therefore has the blocks
//   a.sigma    = [[a0 - a3, -(a1 - i a2)], [-(a1 + i a2), a0 + a3]]  (upper right)
//   a.sigmabar = [[a0 + a3,   a1 - i a2 ], [  a1 + i a2 , a0 - a3]]  (lower left)
//
// Everything is a template on the real type T (float, double, or a host-side
// counting type) so that the same source runs on the GPU, runs on the host
// for generator validation, and yields exact operation counts.  External gluon
// polarisations have a vanishing time component in the frame of the supplied
// momenta; they are carried by a distinct vector type whose time component is
// the empty type `zero`, so that helpers specialise at compile time and no
// arithmetic on that zero is executed or counted.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MGRW_HD __host__ __device__ __forceinline__
#else
#define MGRW_HD inline
#endif

// Scheduling fence between independent groups of a generated program: keeps
// the device scheduler from interleaving groups (and so from growing the
// live register set); no effect on the host.
#if defined(__HIP_DEVICE_COMPILE__)
#define MGRW_SCHED_BARRIER() __builtin_amdgcn_sched_barrier(0)
#else
#define MGRW_SCHED_BARRIER() ((void)0)
#endif

namespace mgrw {

struct zero {};

template <typename T>
struct cx {
    T re, im;
};

// --- complex arithmetic (negation is a source modifier on the GPU: free) ---
template <typename T> MGRW_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> MGRW_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> MGRW_HD cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> MGRW_HD cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> MGRW_HD cx<T> operator*(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> MGRW_HD cx<T> operator*(T s, cx<T> a) { return {a.re * s, a.im * s}; }
template <typename T> MGRW_HD cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// i * a and -i * a (no arithmetic)
template <typename T> MGRW_HD cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }
template <typename T> MGRW_HD cx<T> times_mi(cx<T> a) { return {a.im, -a.re}; }
// acc + a * b and acc - a * b with each real product added to the running sum
// on its own, so that every product feeds an addition and the device compiler
// fuses the pair (two fused multiply-adds per component instead of a complex
// product and a separate addition).  Same operations and counts as
// `acc + a * b`; only the rounding of the intermediate sums differs.
template <typename T> MGRW_HD cx<T> cmad(cx<T> a, cx<T> b, cx<T> acc) {
    return {(acc.re + a.re * b.re) - a.im * b.im, (acc.im + a.re * b.im) + a.im * b.re};
}
template <typename T> MGRW_HD cx<T> cmsb(cx<T> a, cx<T> b, cx<T> acc) {
    return {(acc.re - a.re * b.re) + a.im * b.im, (acc.im - a.re * b.im) - a.im * b.re};
}

// --- the empty zero ---
template <typename T> MGRW_HD cx<T> operator+(cx<T> a, zero) { return a; }
template <typename T> MGRW_HD cx<T> operator+(zero, cx<T> a) { return a; }
template <typename T> MGRW_HD cx<T> operator-(cx<T> a, zero) { return a; }
template <typename T> MGRW_HD cx<T> operator-(zero, cx<T> a) { return -a; }
template <typename T> MGRW_HD zero operator*(cx<T>, zero) { return {}; }
template <typename T> MGRW_HD zero operator*(zero, cx<T>) { return {}; }
template <typename T> MGRW_HD zero operator*(zero, T) { return {}; }
template <typename T> MGRW_HD zero operator*(T, zero) { return {}; }
MGRW_HD zero operator+(zero, zero) { return {}; }
MGRW_HD zero operator-(zero, zero) { return {}; }
MGRW_HD zero operator-(zero) { return {}; }
MGRW_HD zero operator*(zero, zero) { return {}; }
template <typename T> MGRW_HD cx<T> cmad(cx<T> a, cx<T> b, zero) { return a * b; }
template <typename T> MGRW_HD cx<T> cmsb(cx<T> a, cx<T> b, zero) { return -(a * b); }
template <typename T, typename Acc> MGRW_HD Acc cmad(zero, cx<T>, Acc acc) { return acc; }
template <typename T, typename Acc> MGRW_HD Acc cmsb(zero, cx<T>, Acc acc) { return acc; }

// --- four-vectors ---
template <typename T>
struct r4 {                    // real four-vector (momenta), upper index
    T t, x, y, z;
};
template <typename T, typename Tt = cx<T>>
struct v4 {                    // complex four-vector, upper index; Tt = zero for external gluons
    Tt t;
    cx<T> x, y, z;
};
template <typename T> using pol4 = v4<T, zero>;

// Momentum combinations of a three-gluon vertex whose gluon lines carry the
// incoming momenta P1, P2: d = P1 - P2, b = P1 + 2 P2, c = P2 + 2 P1.  They
// depend on the event only, so they are formed once per event (in double)
// rather than once per helicity and point.
template <typename T>
struct vvv_mom {
    r4<T> d, b, c;
};
// A top-line momentum q in light-cone form: qp = q0 + q3, qm = q0 - q3, and
// q1, q2 (again formed once per event).
template <typename T>
struct lc4 {
    T qp, qm, qx, qy;
};

template <typename T> MGRW_HD r4<T> operator+(r4<T> a, r4<T> b) { return {a.t + b.t, a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T> MGRW_HD r4<T> operator-(r4<T> a, r4<T> b) { return {a.t - b.t, a.x - b.x, a.y - b.y, a.z - b.z}; }

// The vertex and propagator momenta formed in the program, from the
// gluon-set momenta P1, P2 and a top-line momentum q.
template <typename T>
MGRW_HD vvv_mom<T> vvv_mom_of(const r4<T>& P1, const r4<T>& P2) {
    return {P1 - P2,
            {P1.t + (P2.t + P2.t), P1.x + (P2.x + P2.x), P1.y + (P2.y + P2.y), P1.z + (P2.z + P2.z)},
            {P2.t + (P1.t + P1.t), P2.x + (P1.x + P1.x), P2.y + (P1.y + P1.y), P2.z + (P1.z + P1.z)}};
}
template <typename T>
MGRW_HD lc4<T> lc4_of(const r4<T>& q) {
    return {q.t + q.z, q.t - q.z, q.x, q.y};
}

// Minkowski products
template <typename T, typename A, typename B>
MGRW_HD cx<T> dot(const v4<T, A>& a, const v4<T, B>& b) {
    return cmsb(a.z, b.z, cmsb(a.y, b.y, cmsb(a.x, b.x, a.t * b.t)));
}
template <typename T, typename A>
MGRW_HD cx<T> dot(const v4<T, A>& a, const r4<T>& p) {
    return ((a.t * p.t - a.x * p.x) - a.y * p.y) - a.z * p.z;
}

template <typename T, typename A>
MGRW_HD v4<T> scale(const v4<T, A>& a, cx<T> s) {
    return {a.t * s, a.x * s, a.y * s, a.z * s};
}

// --- spinors: four complex components ---
template <typename T>
struct sp {
    cx<T> c0, c1, c2, c3;
};

// ---------------------------------------------------------------- vertices

// Three-gluon vertex with the propagator of the combined line (Feynman gauge):
// off-shell current of two gluon currents J1, J2 carrying incoming momenta P1,
// P2.  Returns  coup * [(J1.J2)(P1-P2) + (J1.(P1+2P2)) J2 - (J2.(2P1+P2)) J1],
// where coup = g / (P1+P2)^2 (the colour factor and the constant phase are
// applied by the caller); V holds the three momentum combinations.
template <typename T, typename A, typename B>
MGRW_HD v4<T> vvv(const v4<T, A>& J1, const v4<T, B>& J2, const vvv_mom<T>& V, T coup) {
    const r4<T>& d = V.d;
    cx<T> j12 = dot(J1, J2) * coup;
    cx<T> j1b = dot(J1, V.b) * coup;
    cx<T> j2c = dot(J2, V.c) * coup;
    v4<T> r;
    r.t = cmsb(J1.t, j2c, cmad(J2.t, j1b, j12 * d.t));
    r.x = cmsb(J1.x, j2c, cmad(J2.x, j1b, j12 * d.x));
    r.y = cmsb(J1.y, j2c, cmad(J2.y, j1b, j12 * d.y));
    r.z = cmsb(J1.z, j2c, cmad(J2.z, j1b, j12 * d.z));
    return r;
}
// The same with the coupling and propagator already in V (V scaled by coup).
template <typename T, typename A, typename B>
MGRW_HD v4<T> vvv(const v4<T, A>& J1, const v4<T, B>& J2, const vvv_mom<T>& V) {
    const r4<T>& d = V.d;
    cx<T> j12 = dot(J1, J2);
    cx<T> j1b = dot(J1, V.b);
    cx<T> j2c = dot(J2, V.c);
    v4<T> r;
    r.t = cmsb(J1.t, j2c, cmad(J2.t, j1b, j12 * d.t));
    r.x = cmsb(J1.x, j2c, cmad(J2.x, j1b, j12 * d.x));
    r.y = cmsb(J1.y, j2c, cmad(J2.y, j1b, j12 * d.y));
    r.z = cmsb(J1.z, j2c, cmad(J2.z, j1b, j12 * d.z));
    return r;
}

// A three-gluon vertex closed on the current K (the t tbar current of a root
// closure): K . vvv(J1, J2, V) contracted term by term,
//   (J1.J2)(K.d) + (K.J2)(J1.b) - (K.J1)(J2.c),
// so that K.J1 and K.J2 are shared between the closures of J1 and J2 with
// other partners.
template <typename T, typename A, typename B>
MGRW_HD cx<T> vvv_close(const v4<T>& K, const v4<T, A>& J1, const v4<T, B>& J2, const vvv_mom<T>& V) {
    return cmsb(dot(K, J1), dot(J2, V.c), cmad(dot(K, J2), dot(J1, V.b), dot(J1, J2) * dot(K, V.d)));
}

// Four-gluon vertex with propagator: the three colour structures
//   A = J2 (J1.J3) - J3 (J1.J2)   (colour [1,[2,3]])
//   B = J1 (J2.J3) - J3 (J1.J2)   (colour [2,[1,3]])
//   C = J1 (J2.J3) - J2 (J1.J3)   (colour [3,[1,2]])
// each times coup = g^2 / P^2.  A piece built only from external gluons keeps
// a vanishing time component (its type is deduced).
template <typename V1, typename V2, typename V3>
struct vvvv_out {
    V1 A;
    V2 B;
    V3 C;
};

template <typename T, typename A, typename B, typename C>
MGRW_HD auto vvvv(const v4<T, A>& J1, const v4<T, B>& J2, const v4<T, C>& J3, T coup) {
    cx<T> d12 = dot(J1, J2) * coup, d13 = dot(J1, J3) * coup, d23 = dot(J2, J3) * coup;
    using TA = decltype(J2.t * d13 - J3.t * d12);
    using TB = decltype(J1.t * d23 - J3.t * d12);
    using TC = decltype(J1.t * d23 - J2.t * d13);
    vvvv_out<v4<T, TA>, v4<T, TB>, v4<T, TC>> o;
    o.A.t = cmsb(J3.t, d12, J2.t * d13);
    o.A.x = cmsb(J3.x, d12, J2.x * d13);
    o.A.y = cmsb(J3.y, d12, J2.y * d13);
    o.A.z = cmsb(J3.z, d12, J2.z * d13);
    o.B.t = cmsb(J3.t, d12, J1.t * d23);
    o.B.x = cmsb(J3.x, d12, J1.x * d23);
    o.B.y = cmsb(J3.y, d12, J1.y * d23);
    o.B.z = cmsb(J3.z, d12, J1.z * d23);
    o.C.t = cmsb(J2.t, d13, J1.t * d23);
    o.C.x = cmsb(J2.x, d13, J1.x * d23);
    o.C.y = cmsb(J2.y, d13, J1.y * d23);
    o.C.z = cmsb(J2.z, d13, J1.z * d23);
    return o;
}

// The three four-gluon structures closed on the current K (unit coupling):
// K.A = (K.J2)(J1.J3) - (K.J3)(J1.J2), K.B = (K.J1)(J2.J3) - (K.J3)(J1.J2),
// K.C = (K.J1)(J2.J3) - (K.J2)(J1.J3).
template <typename T>
struct vvvv_closed {
    cx<T> A, B, C;
};
template <typename T, typename A, typename B, typename C>
MGRW_HD vvvv_closed<T> vvvv_close(const v4<T>& K, const v4<T, A>& J1, const v4<T, B>& J2, const v4<T, C>& J3) {
    const cx<T> d12 = dot(J1, J2), d13 = dot(J1, J3), d23 = dot(J2, J3);
    const cx<T> k1 = dot(K, J1), k2 = dot(K, J2), k3 = dot(K, J3);
    return {cmsb(k3, d12, k2 * d13), cmsb(k3, d12, k1 * d23), cmsb(k2, d13, k1 * d23)};
}

// Row spinor times a slashed complex vector: (a . Jslash).
template <typename T, typename A>
MGRW_HD sp<T> row_slash(const sp<T>& a, const v4<T, A>& J) {
    cx<T> jp = J.t + J.z;           // J0 + J3
    cx<T> jm = J.t - J.z;           // J0 - J3
    cx<T> jt = J.x + times_i(J.y);  // J1 + i J2
    cx<T> js = J.x - times_i(J.y);  // J1 - i J2
    sp<T> b;
    b.c0 = cmad(a.c3, jt, a.c2 * jp);
    b.c1 = cmad(a.c3, jm, a.c2 * js);
    b.c2 = cmsb(a.c1, jt, a.c0 * jm);
    b.c3 = cmsb(a.c0, js, a.c1 * jp);
    return b;
}

// Slashed complex vector times a column spinor: (Jslash . v).
template <typename T, typename A>
MGRW_HD sp<T> slash_col(const v4<T, A>& J, const sp<T>& v) {
    cx<T> jp = J.t + J.z, jm = J.t - J.z;
    cx<T> jt = J.x + times_i(J.y), js = J.x - times_i(J.y);
    sp<T> b;
    b.c0 = cmsb(js, v.c3, jm * v.c2);
    b.c1 = cmsb(jt, v.c2, jp * v.c3);
    b.c2 = cmad(js, v.c1, jp * v.c0);
    b.c3 = cmad(jm, v.c1, jt * v.c0);
    return b;
}

// Row spinor times (qslash + m) for a real momentum q (and q, m already
// scaled by the propagator's denominator where the caller wants it).
template <typename T>
MGRW_HD sp<T> row_prop(const sp<T>& b, const lc4<T>& q, T m) {
    const T qp = q.qp, qm = q.qm;
    cx<T> qt = {q.qx, q.qy}, qs = {q.qx, -q.qy};   // q1 + i q2, q1 - i q2
    sp<T> c;
    c.c0 = cmad(b.c3, qt, b.c0 * m + b.c2 * qp);
    c.c1 = cmad(b.c2, qs, b.c1 * m) + b.c3 * qm;
    c.c2 = cmsb(b.c1, qt, b.c2 * m + b.c0 * qm);
    c.c3 = cmsb(b.c0, qs, b.c3 * m + b.c1 * qp);
    return c;
}
// (qslash + m) times a column spinor, as row_prop.
template <typename T>
MGRW_HD sp<T> prop_col(const lc4<T>& q, T m, const sp<T>& v) {
    const T qp = q.qp, qm = q.qm;
    cx<T> qt = {q.qx, q.qy}, qs = {q.qx, -q.qy};
    sp<T> c;
    c.c0 = cmsb(v.c3, qs, v.c0 * m + v.c2 * qm);
    c.c1 = cmsb(v.c2, qt, v.c1 * m + v.c3 * qp);
    c.c2 = cmad(v.c1, qs, v.c2 * m + v.c0 * qp);
    c.c3 = cmad(v.c0, qt, v.c3 * m) + v.c1 * qm;
    return c;
}

// The same times a real factor.
template <typename T>
MGRW_HD sp<T> row_prop(const sp<T>& b, const lc4<T>& q, T m, T f) {
    const sp<T> c = row_prop(b, q, m);
    return {c.c0 * f, c.c1 * f, c.c2 * f, c.c3 * f};
}
template <typename T>
MGRW_HD sp<T> prop_col(const lc4<T>& q, T m, const sp<T>& v, T f) {
    const sp<T> c = prop_col(q, m, v);
    return {c.c0 * f, c.c1 * f, c.c2 * f, c.c3 * f};
}

template <typename T>
MGRW_HD cx<T> row_col(const sp<T>& a, const sp<T>& b) {
    return cmad(a.c3, b.c3, cmad(a.c2, b.c2, cmad(a.c1, b.c1, a.c0 * b.c0)));
}

// Top-gluon vertex followed by the top propagator, on the row (outgoing-top)
// side:  coup * a . Jslash . (qslash + m), coup = g kappa / (q^2 - m^2).
template <typename T, typename A>
MGRW_HD sp<T> ffv_row(const sp<T>& a, const v4<T, A>& J, const lc4<T>& q, T m, T coup) {
    return row_prop(row_slash(a, J), q, m, coup);
}

// Top-gluon vertex followed by the top propagator on the column (antitop)
// side: coup * (qslash + m) . Jslash . v.
template <typename T, typename A>
MGRW_HD sp<T> ffv_col(const v4<T, A>& J, const sp<T>& v, const lc4<T>& q, T m, T coup) {
    return prop_col(q, m, slash_col(J, v), coup);
}

template <typename T, typename A>
MGRW_HD sp<T> ffv_row(const sp<T>& a, const v4<T, A>& J, const r4<T>& q, T m, T coup) {
    return ffv_row(a, J, lc4_of(q), m, coup);
}
// Unit coupling, with q and m already divided by q^2 - m^2.
template <typename T, typename A>
MGRW_HD sp<T> ffv_row(const sp<T>& a, const v4<T, A>& J, const lc4<T>& q, T m) {
    return row_prop(row_slash(a, J), q, m);
}
template <typename T, typename A>
MGRW_HD sp<T> ffv_col(const v4<T, A>& J, const sp<T>& v, const lc4<T>& q, T m) {
    return prop_col(q, m, slash_col(J, v));
}
template <typename T, typename A>
MGRW_HD sp<T> ffv_col(const v4<T, A>& J, const sp<T>& v, const r4<T>& q, T m, T coup) {
    return ffv_col(J, v, lc4_of(q), m, coup);
}

// Closing vertex: coup * a . Jslash . v, coup = g kappa.
template <typename T, typename A>
MGRW_HD cx<T> ffv_amp(const sp<T>& a, const v4<T, A>& J, const sp<T>& v, T coup) {
    return row_col(row_slash(a, J), v) * coup;
}
// The same closure associated as a . (Jslash . v): it then shares Jslash . v
// with the column current that continues through this vertex.
template <typename T, typename A>
MGRW_HD cx<T> ffv_amp_col(const sp<T>& a, const v4<T, A>& J, const sp<T>& v, T coup) {
    return row_col(a, slash_col(J, v)) * coup;
}

// psibar gamma^mu psi' for row spinor a and column spinor b (complex vector).
template <typename T>
MGRW_HD v4<T> vector_current(const sp<T>& a, const sp<T>& b) {
    // upper-right block sigma^mu = (1, s), lower-left sigmabar^mu = (1, -s)
    v4<T> j;
    j.t = cmad(a.c3, b.c1, cmad(a.c2, b.c0, cmad(a.c1, b.c3, a.c0 * b.c2)));
    j.x = cmsb(a.c3, b.c0, cmsb(a.c2, b.c1, cmad(a.c1, b.c2, a.c0 * b.c3)));
    j.y = times_i(cmsb(a.c3, b.c0, cmad(a.c2, b.c1, cmsb(a.c0, b.c3, a.c1 * b.c2))));
    j.z = cmad(a.c3, b.c1, cmsb(a.c2, b.c0, cmsb(a.c1, b.c3, a.c0 * b.c2)));
    return j;
}

// The t tbar current f * (ubar gamma^mu v): the off-shell gluon emitted by the
// top line with no other attachment (f carries g kappa and 1/P^2).
template <typename T>
MGRW_HD v4<T> tt_current(const sp<T>& ub, const sp<T>& v, T f) {
    v4<T> j = vector_current(ub, v);
    return {j.t * f, j.x * f, j.y * f, j.z * f};
}

// ------------------------------------------------ external wavefunctions

// Helicity-independent pieces of a gluon's polarisation vectors in the frame
// of the given momentum: e1 = (0, cos t cos f, cos t sin f, -sin t) and
// e2 = (0, -sin f, cos f, 0), pre-scaled by 1/sqrt(2).
template <typename T>
struct gluon_basis {
    T e1x, e1y, e1z, e2x, e2y;
};

// eps(k, lam) = (-lam e1 - i e2)/sqrt2; the conjugate for an outgoing gluon.
template <typename T>
MGRW_HD pol4<T> gluon_pol(const gluon_basis<T>& g, int lam, bool outgoing) {
    T s = lam > 0 ? T(-1) : T(1);          // -lam
    pol4<T> e;
    // imaginary part -e2 (incoming) or +e2 (outgoing): a sign choice, no arithmetic
    T e2x = outgoing ? g.e2x : -g.e2x;
    T e2y = outgoing ? g.e2y : -g.e2y;
    e.x = {s > T(0) ? g.e1x : -g.e1x, e2x};
    e.y = {s > T(0) ? g.e1y : -g.e1y, e2y};
    e.z = {s > T(0) ? g.e1z : -g.e1z, T(0)};
    return e;
}

// Helicity-independent pieces of a massive spinor: the two-component
// helicity eigenstates chi_+ and chi_- of p-hat, and w_pm = sqrt(E pm |p|).
template <typename T>
struct fermion_basis {
    cx<T> cp0, cp1, cm0, cm1;   // chi_+, chi_-
    T wp, wm;                   // sqrt(E + |p|), sqrt(E - |p|)
};

// ubar(p, lam) for an outgoing fermion: u = (w_{-lam} chi_lam, w_lam chi_lam),
// ubar = u^dagger gamma^0 = (conj(u2), conj(u3), conj(u0), conj(u1)).
template <typename T>
MGRW_HD sp<T> ubar_out(const fermion_basis<T>& f, int lam) {
    cx<T> c0 = lam > 0 ? f.cp0 : f.cm0;
    cx<T> c1 = lam > 0 ? f.cp1 : f.cm1;
    T up = lam > 0 ? f.wm : f.wp;       // w_{-lam}
    T lo = lam > 0 ? f.wp : f.wm;       // w_lam
    return {conj(c0) * lo, conj(c1) * lo, conj(c0) * up, conj(c1) * up};
}

// v(p, lam) for an outgoing antifermion: (-lam w_lam chi_{-lam}, lam w_{-lam} chi_{-lam}).
template <typename T>
MGRW_HD sp<T> v_out(const fermion_basis<T>& f, int lam) {
    cx<T> c0 = lam > 0 ? f.cm0 : f.cp0;
    cx<T> c1 = lam > 0 ? f.cm1 : f.cp1;
    T a = lam > 0 ? -f.wp : f.wm;       // -lam w_lam
    T b = lam > 0 ? f.wm : -f.wp;       // lam w_{-lam}
    return {c0 * a, c1 * a, c0 * b, c1 * b};
}

// Build the polarisation basis of a massless gluon from its momentum (double
// precision in, rounded to T once).
template <typename T, typename P>
MGRW_HD gluon_basis<T> make_gluon_basis(const P& k) {
    double kt = sqrt(k[1] * k[1] + k[2] * k[2]);
    double ka = sqrt(kt * kt + k[3] * k[3]);
    double ct = k[3] / ka, st = kt / ka;
    double cf = 1.0, sf = 0.0;
    if (kt > 0.0) {
        cf = k[1] / kt;
        sf = k[2] / kt;
    }
    const double r = 0.70710678118654752440;
    return {T(ct * cf * r), T(ct * sf * r), T(-st * r), T(-sf * r), T(cf * r)};
}

// Build the spinor basis of a fermion of mass m and momentum p.  |p| + pz is
// formed as pT^2 / (|p| - pz) when pz < 0 to avoid cancellation; on shell
// sqrt(E - |p|) = m / sqrt(E + |p|).
template <typename T, typename P>
MGRW_HD fermion_basis<T> make_fermion_basis(const P& p, double m) {
    double pt2 = p[1] * p[1] + p[2] * p[2];
    double pa = sqrt(pt2 + p[3] * p[3]);
    double d = p[3] >= 0.0 ? pa + p[3] : pt2 / (pa - p[3]);
    fermion_basis<T> f;
    if (d <= 0.0) {   // along -z
        f.cp0 = {T(0), T(0)};
        f.cp1 = {T(1), T(0)};
        f.cm0 = {T(-1), T(0)};
        f.cm1 = {T(0), T(0)};
    } else {
        double nrm = 1.0 / sqrt(2.0 * pa * d);
        f.cp0 = {T(d * nrm), T(0)};
        f.cp1 = {T(p[1] * nrm), T(p[2] * nrm)};
        f.cm0 = {T(-p[1] * nrm), T(p[2] * nrm)};
        f.cm1 = {T(d * nrm), T(0)};
    }
    double wp = sqrt(p[0] + pa);
    f.wp = T(wp);
    f.wm = T(m / wp);
    return f;
}

}  // namespace mgrw
