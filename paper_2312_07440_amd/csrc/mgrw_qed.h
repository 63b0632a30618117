// e+ e- -> n photons in massless QED: the process timed in the paper's own
// reweighting experiment (Sec. 3.3, Table 1).
//
// Particles: e+(p0) e-(p1) -> photons p2 .. p_{n+1}.  The n! Feynman diagrams
// attach the photons to the electron line in every order.  For a massless
// electron the vector coupling preserves chirality, so along the line only
// one two-component (Weyl) half of the Dirac spinor is non-zero, and only the
// 2^(n+1) helicity configurations with opposite e+ and e- labels survive; the
// others vanish identically and are not evaluated.
//
// In the chiral representation, starting from u(p1, lam) = sqrt(2E1) chi_lam
// (right-handed for lam = +1), a vertex -i e Q eps*-slash maps the spinor to
// the other chirality with the 2x2 matrix -s eps*.sigma (eps^0 = 0 in the
// frame of the event; s = lam), a propagator i qslash / q^2 maps it back with
// (q^0 + s q.sigma) / q^2, and the line ends on vbar(p0, -lam), i.e. on
// -sqrt(2E0) chi_lam(p0)^dagger.  All diagrams share the phase i^(2n-1), which
// drops out of |M|^2.
//
// The diagram sum is built as a recursion over subsets S of the photons
// (Berends-Giele style): R_0 = chi_lam(p1) and
//   R_S = P(q_S) sum_{i in S} V_i R_{S \ i},  q_S = p1 - sum_{i in S} k_i,
// so R_S sums the |S|! orderings of S; the amplitude is
//   M = -sqrt(4 E0 E1) chi_lam(p0)^dagger sum_i V_i R_{all \ i}.
#pragma once

#include "mgrw_lorentz.h"

namespace mgrw {

template <typename T>
struct wspin {   // two-component spinor
    cx<T> a, b;
};

template <int NA>
struct ee_photons {
    static constexpr int NEXT = NA + 2;
    static constexpr int NHEL = 1 << (NA + 2);      // all helicity configurations
    static constexpr int NLIVE = 1 << (NA + 1);     // those with opposite e+ e- labels
    static constexpr int NSUB = (1 << NA) - 1;      // proper subsets 1 .. 2^NA - 2 (index = mask)
    static constexpr int NDIAG = [] {
        int f = 1;
        for (int i = 2; i <= NA; ++i) f *= i;
        return f;
    }();
    // spin average 1/4, identical photons 1/n!
    static constexpr double NORM = 1.0 / (4.0 * NDIAG);

    // Helicity-independent data of one event.
    template <typename T>
    struct event {
        T P[NSUB][4];             // q_S / q_S^2 for subset mask S (index 0 unused)
        T e1[NA][3], e2[NA][3];   // photon polarisation basis, spatial parts
        cx<T> chi1[2][2];         // chi_{+1}, chi_{-1} of the e- direction
        cx<T> chi0[2][2];         // the same for the e+ direction
        double flux;              // 4 E0 E1 = |sqrt(2E0) sqrt(2E1)|^2
    };

    // Two-component helicity eigenstate chi_lam(p-hat) (lam = +-1).
    static MGRW_HD void chi(const double (&p)[4], int lam, double* re, double* im) {
        const double pa = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        const double d = pa + p[3];
        if (d <= 0.0) {   // along -z
            re[0] = lam > 0 ? 0.0 : -1.0;
            re[1] = lam > 0 ? 1.0 : 0.0;
            im[0] = im[1] = 0.0;
            return;
        }
        const double r = 1.0 / sqrt(2.0 * pa * d);
        if (lam > 0) {
            re[0] = d * r;
            im[0] = 0.0;
            re[1] = p[1] * r;
            im[1] = p[2] * r;
        } else {
            re[0] = -p[1] * r;
            im[0] = p[2] * r;
            re[1] = d * r;
            im[1] = 0.0;
        }
    }

    template <typename T, typename P>
    static MGRW_HD void setup(const P& p, event<T>& ev) {
        for (int mask = 1; mask < NSUB; ++mask) {
            double q[4];
            for (int m = 0; m < 4; ++m) q[m] = p[1][m];
            for (int i = 0; i < NA; ++i)
                if (mask >> i & 1)
                    for (int m = 0; m < 4; ++m) q[m] -= p[2 + i][m];
            const double iq2 = 1.0 / (((q[0] * q[0] - q[1] * q[1]) - q[2] * q[2]) - q[3] * q[3]);
            for (int m = 0; m < 4; ++m) ev.P[mask][m] = T(q[m] * iq2);
        }
        for (int m = 0; m < 4; ++m) ev.P[0][m] = T(0);
        for (int i = 0; i < NA; ++i) {
            const double* k = p[2 + i];
            const double kt = sqrt(k[1] * k[1] + k[2] * k[2]);
            const double ka = sqrt(kt * kt + k[3] * k[3]);
            const double ct = k[3] / ka, st = kt / ka;
            const double cf = kt > 0.0 ? k[1] / kt : 1.0, sf = kt > 0.0 ? k[2] / kt : 0.0;
            ev.e1[i][0] = T(ct * cf);
            ev.e1[i][1] = T(ct * sf);
            ev.e1[i][2] = T(-st);
            ev.e2[i][0] = T(-sf);
            ev.e2[i][1] = T(cf);
            ev.e2[i][2] = T(0);
        }
        for (int l = 0; l < 2; ++l) {
            double re[2], im[2];
            const double p1[4] = {p[1][0], p[1][1], p[1][2], p[1][3]};
            const double p0[4] = {p[0][0], p[0][1], p[0][2], p[0][3]};
            chi(p1, l == 0 ? 1 : -1, re, im);
            for (int c = 0; c < 2; ++c) ev.chi1[l][c] = {T(re[c]), T(im[c])};
            chi(p0, l == 0 ? 1 : -1, re, im);
            for (int c = 0; c < 2; ++c) ev.chi0[l][c] = {T(re[c]), T(im[c])};
        }
        ev.flux = 4.0 * p[0][0] * p[1][0];
    }

    // Amplitude (up to the common phase, without the flux factor) of live
    // configuration h: bit NA gives the e- label (1: +1), bit i < NA the
    // helicity of photon i (1: +1); the e+ label is the opposite of the e-
    // one.  e: the electromagnetic coupling at every vertex.  The helicity
    // signs enter as factors +-1, which the compiler folds into the products.
    template <typename T, typename EV>
    static MGRW_HD cx<T> amplitude(const EV& ev, int h, T e) {
        const int lam = (h >> NA) & 1 ? 1 : -1;
        const T s = T(lam);
        const int li = lam > 0 ? 0 : 1;
        // vertex matrices V_i = -s e eps*.sigma = [[va, vb], [vc, -va]],
        // eps* = (-l e1 + i e2)/sqrt2 for photon helicity l
        cx<T> va[NA], vb[NA], vc[NA];
        const T r2 = T(0.70710678118654752440);
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
        for (int i = 0; i < NA; ++i) {
            const T l = (h >> i) & 1 ? T(1) : T(-1);
            const T f = -s * e * r2;
            const cx<T> ex = {-l * ev.e1[i][0] * f, ev.e2[i][0] * f};
            const cx<T> ey = {-l * ev.e1[i][1] * f, ev.e2[i][1] * f};
            const cx<T> ez = {-l * ev.e1[i][2] * f, ev.e2[i][2] * f};
            va[i] = ez;
            vb[i] = {ex.re + ey.im, ex.im - ey.re};   // ex - i ey
            vc[i] = {ex.re - ey.im, ex.im + ey.re};   // ex + i ey
        }
        wspin<T> R[NSUB];
        R[0] = {ev.chi1[li][0], ev.chi1[li][1]};
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
        // Each product is added to its running sum on its own (cmad/cmsb:
        // fused multiply-adds); the first term of a sum starts it.
        for (int mask = 1; mask < NSUB; ++mask) {
            cx<T> ua, ub;
            bool first = true;   // a constant in every unrolled step
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
            for (int i = 0; i < NA; ++i) {
                if (!(mask >> i & 1)) continue;
                const wspin<T>& x = R[mask & ~(1 << i)];
                ua = cmad(vb[i], x.b, first ? va[i] * x.a : cmad(va[i], x.a, ua));
                ub = cmsb(va[i], x.b, first ? vc[i] * x.a : cmad(vc[i], x.a, ub));
                first = false;
            }
            // P(q) = [[A + sZ, s(X - iY)], [s(X + iY), A - sZ]] with (A, X, Y, Z) = q / q^2
            const T A = ev.P[mask][0], X = s * ev.P[mask][1], Y = s * ev.P[mask][2], Z = s * ev.P[mask][3];
            const cx<T> xmy = {X, -Y}, xpy = {X, Y};
            R[mask] = {cmad(xmy, ub, (A + Z) * ua), cmad(xpy, ua, (A - Z) * ub)};
        }
        cx<T> ta = va[0] * R[NSUB & ~1].a, tb = vc[0] * R[NSUB & ~1].a;
        ta = cmad(vb[0], R[NSUB & ~1].b, ta);
        tb = cmsb(va[0], R[NSUB & ~1].b, tb);
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
        for (int i = 1; i < NA; ++i) {
            const wspin<T>& x = R[NSUB & ~(1 << i)];
            ta = cmad(vb[i], x.b, cmad(va[i], x.a, ta));
            tb = cmsb(va[i], x.b, cmad(vc[i], x.a, tb));
        }
        // -chi_lam(p0)^dagger (ta, tb)
        return -cmad(conj(ev.chi0[li][1]), tb, conj(ev.chi0[li][0]) * ta);
    }
};

using ee_5a = ee_photons<5>;

}  // namespace mgrw
