// Per-event evaluation of |M|^2 at a list of parameter points.
//
// The same templates run in the GPU kernels (one event per lane) and in the
// host validation build.  Structure per event (Sec. 3.2, steps 3-7 of the
// reweighting procedure, with the parameter loop inside the event so the
// momenta are read once):
//   helicity-independent kinematics and propagator denominators (double);
//   external-wavefunction bases (double, rounded to T once);
//   for each parameter point: for each helicity: external wavefunctions,
//   diagram chains -> colour-flow amplitudes J (T), colour sum (T),
//   accumulated over helicities in double; normalised.
#pragma once

#include "mgrw_lorentz.h"

namespace mgrw {

// Couplings of one QCD parameter point, derived on the host from alpha_s and
// kappa: g, g^2 and g*kappa.
struct qcd_point {
    double gs, gs2, gk;
};

// |M|^2 of one event at one parameter point: the full amplitude program for
// every helicity configuration, colour-summed, accumulated in double.
// k and b are the event's kinematics and wavefunction bases, held in
// registers or in LDS.  On the GPU a compiler-level memory barrier at the top
// of each helicity iteration keeps their loads inside the loop instead of
// letting them be hoisted into registers for the whole loop.
template <class Proc, typename T, typename KN, typename BS>
MGRW_HD double point_me(const KN& k, const BS& b, const qcd_point& pt) {
    const auto c = Proc::template couplings<T>(pt.gs, pt.gs2, pt.gk);
    double acc = 0.0;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll 1
#endif
    for (int h = 0; h < Proc::NHEL; ++h) {
#if defined(__HIP_DEVICE_COMPILE__)
        __asm__ volatile("" ::: "memory");
#endif
        typename Proc::template ext<T> w;
        Proc::template external<T>(b, h, w);
        cx<T> J[Proc::K];
        Proc::amplitude(w, k, c, J);
        acc += double(Proc::colour_sum(J));
    }
    return acc * Proc::point_norm(pt.gs);
}

// ------------------------------------------------ kappa-polynomial form
//
// Every diagram of g g -> t tbar + n g carries g^NG kappa^k, k its number of
// top-gluon vertices, so J(g, kappa) = g^NG sum_k kappa^k J_k with J_k from one
// evaluation at unit couplings, and
//   |M|^2(g, kappa) = NORM g^(2 NG) sum_{a<=b} (2 - delta_ab) kappa^(a+b+2) B_ab,
//   B_ab = sum_h Re(J_a^+ CF J_b)            (a, b = 0..NG-1 for powers 1..NG).
// Exact: the same diagrams as the plain program, evaluated once for any
// number of parameter points.

template <typename T>
struct kpoly_acc { using type = T; };
template <>
struct kpoly_acc<float> { using type = double; };

template <class Proc>
constexpr int kpoly_pairs() {
    return Proc::NG * (Proc::NG + 1) / 2;
}

// Add the colour products of one helicity configuration's kappa-power
// amplitudes J[NG K] to B (pair (a <= b) at b(b+1)/2 + a).
template <class Proc, typename T>
MGRW_HD void kpoly_colour(const cx<T>* J, double* B) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
    for (int pb = 0; pb < Proc::NG; ++pb) {
        // The terms of different kappa powers cancel strongly against each
        // other (no single power is gauge invariant), so the colour products
        // of float amplitudes are accumulated in double.
        using TA = typename kpoly_acc<T>::type;
        if (pb == 0) {
            // B_00 alone: the symmetric quadratic form, half the products of
            // CF J_0 followed by a dot product
            cx<TA> Jd[Proc::K];
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
            for (int i = 0; i < Proc::K; ++i) Jd[i] = {TA(J[i].re), TA(J[i].im)};
            B[0] += double(Proc::template colour_sum<TA>(Jd));
            continue;
        }
        cx<TA> Z[Proc::K];
        Proc::template colour_matvec<TA, T>(J + pb * Proc::K, Z);
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
        for (int pa = 0; pa <= pb; ++pa)
            B[pb * (pb + 1) / 2 + pa] += double(Proc::template re_dot<TA, T>(J + pa * Proc::K, Z));
    }
}

// Add one helicity configuration's B_ab.
// w: storage for the external wavefunctions (registers or an LDS slot).
template <class Proc, typename T, typename KN, typename BS, typename EXT>
MGRW_HD void kpoly_helicity(const KN& k, const BS& b, int h, double* B, EXT& w) {
    typename Proc::template coup<T> c = {T(1), T(1), T(1)};
    Proc::template external<T>(b, h, w);
    cx<T> J[Proc::NG * Proc::K];
    Proc::amplitude_kpoly(w, k, c, J);
    kpoly_colour<Proc, T>(J, B);
}

template <class Proc, typename T, typename KN, typename BS>
MGRW_HD void kpoly_helicity(const KN& k, const BS& b, int h, double* B) {
    typename Proc::template ext<T> w;
    kpoly_helicity<Proc, T>(k, b, h, B, w);
}

// |M|^2 at couplings (gs, kappa) from the helicity-summed B.
template <class Proc>
MGRW_HD double kpoly_me(const double* B, double gs, double kappa) {
    double kp[2 * Proc::NG + 1];
    kp[0] = 1.0;
    for (int i = 1; i <= 2 * Proc::NG; ++i) kp[i] = kp[i - 1] * kappa;
    double s = 0.0;
    for (int pb = 0; pb < Proc::NG; ++pb)
        for (int pa = 0; pa <= pb; ++pa) s += (pa == pb ? 1.0 : 2.0) * kp[pa + pb + 2] * B[pb * (pb + 1) / 2 + pa];
    double g2n = 1.0;
    for (int i = 0; i < Proc::NG; ++i) g2n *= gs * gs;
    return s * g2n * Proc::NORM;
}

// Helicity-independent state of one event held by value (host build, and the
// FP64 kernels): kinematics with double-precision propagator denominators,
// and the external-wavefunction bases.
template <class Proc, typename T>
struct qcd_event {
    typename Proc::template kin<T> k;
    typename Proc::template basis<T> b;

    template <typename P>
    MGRW_HD void setup(const P& p, double mt) {
        Proc::kinematics(p, mt, k);
        Proc::external_basis(p, mt, b);
    }

    MGRW_HD double me(const qcd_point& pt) const { return point_me<Proc, T>(k, b, pt); }
};

// ------------------------------------------------------ e+ e- -> mu+ mu-

// One electroweak parameter point, derived on the host: e^2 and the Z coupling
// squared g_Z^2 = e^2/(sw^2 cw^2), chiral couplings, and the Z pole.
struct ew_point {
    double e2, gz2, gl, gr, mz2, mzwz;
};

template <typename T>
MGRW_HD sp<T> u_in(const fermion_basis<T>& f, int lam) {
    cx<T> c0 = lam > 0 ? f.cp0 : f.cm0;
    cx<T> c1 = lam > 0 ? f.cp1 : f.cm1;
    T up = lam > 0 ? f.wm : f.wp;
    T lo = lam > 0 ? f.wp : f.wm;
    return {c0 * up, c1 * up, c0 * lo, c1 * lo};
}

template <typename T>
MGRW_HD sp<T> vbar_in(const fermion_basis<T>& f, int lam) {
    sp<T> v = v_out(f, lam);
    return {conj(v.c2), conj(v.c3), conj(v.c0), conj(v.c1)};
}

// Spin-averaged |M|^2 of e+(p0) e-(p1) -> mu+(p2) mu-(p3), gamma + Z in the s
// channel.  With vertices -i e Q gamma^mu and -i g_Z gamma^mu (gL PL + gR PR)
// and propagators -i g/s, -i g/(s - MZ^2 + i MZ GZ), a configuration with
// electron chirality i and muon chirality j has
//   M = (jout . jin) [e^2/s + g_Z^2 g_i g_j /(s - MZ^2 + i MZ GZ)]
// up to a phase.  For massless fermions the 12 configurations with equal
// helicities on a fermion line vanish identically and are not evaluated.
struct ee_mumu_event {
    cx<double> cc[2][2];   // jout . jin per (electron, muon) chirality L/R
    double s;

    template <typename P>
    MGRW_HD void setup(const P& p) {
        fermion_basis<double> f0 = make_fermion_basis<double>(p[0], 0.0);
        fermion_basis<double> f1 = make_fermion_basis<double>(p[1], 0.0);
        fermion_basis<double> f2 = make_fermion_basis<double>(p[2], 0.0);
        fermion_basis<double> f3 = make_fermion_basis<double>(p[3], 0.0);
        double q0 = p[0][0] + p[1][0], q1 = p[0][1] + p[1][1], q2 = p[0][2] + p[1][2], q3 = p[0][3] + p[1][3];
        s = ((q0 - q3) * (q0 + q3) - q1 * q1) - q2 * q2;
        // (e+, e-) helicities (+,-) form a left-handed current, (-,+) right-handed
        for (int i = 0; i < 2; ++i) {
            int le = i == 0 ? -1 : 1;
            v4<double> jin = vector_current(vbar_in(f0, -le), u_in(f1, le));
            for (int j = 0; j < 2; ++j) {
                int lm = j == 0 ? -1 : 1;
                v4<double> jout = vector_current(ubar_out(f3, lm), v_out(f2, -lm));
                cc[i][j] = dot(jout, jin);
            }
        }
    }

    MGRW_HD double me(const ew_point& c) const {
        double dr = s - c.mz2, di = c.mzwz, dd = 1.0 / (dr * dr + di * di);
        cx<double> iz = {dr * dd, -di * dd};          // 1/(s - MZ^2 + i MZ GZ)
        double acc = 0.0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double gi = i == 0 ? c.gl : c.gr, gj = j == 0 ? c.gl : c.gr;
                cx<double> f = iz * (c.gz2 * gi * gj);
                f.re = f.re + c.e2 / s;
                cx<double> a = cc[i][j] * f;
                acc += a.re * a.re + a.im * a.im;
            }
        return 0.25 * acc;
    }
};

}  // namespace mgrw
