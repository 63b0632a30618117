// Host build of the per-event amplitude programs -- used by the tests only.
//
// Two uses, neither on the product path (the Python binding never loads this
// library):
//  * run the generated programs on the CPU in double precision so that the
//    generator can be validated without a GPU;
//  * count the floating-point operations of one helicity program exactly, by
//    instantiating the same templates with a counting scalar type.
#include <cstdint>
#include <cstring>

#include "mgrw_event.h"
#include "mgrw_qed.h"
#include "gen/gg_tt.inc"
#include "gen/gg_ttg.inc"
#include "gen/gg_ttgg.inc"
#include "gen/gg_ttggg.inc"

namespace {

struct cfloat {
    double v;
    static thread_local long long n_add, n_mul;
    cfloat() = default;
    constexpr cfloat(double x) : v(x) {}
    explicit operator double() const { return v; }
};
thread_local long long cfloat::n_add = 0;
thread_local long long cfloat::n_mul = 0;

inline cfloat operator+(cfloat a, cfloat b) { ++cfloat::n_add; return {a.v + b.v}; }
inline cfloat operator-(cfloat a, cfloat b) { ++cfloat::n_add; return {a.v - b.v}; }
inline cfloat operator*(cfloat a, cfloat b) { ++cfloat::n_mul; return {a.v * b.v}; }
inline cfloat operator-(cfloat a) { return {-a.v}; }
inline bool operator>(cfloat a, cfloat b) { return a.v > b.v; }

template <class Proc, typename T>
void me_events(const double* mom, int64_t n, double mt, const mgrw::qcd_point* pts, int npts, double* me) {
    for (int64_t e = 0; e < n; ++e) {
        double p[Proc::NEXT][4];
        for (int i = 0; i < Proc::NEXT; ++i)
            for (int m = 0; m < 4; ++m) p[i][m] = mom[(int64_t(i) * 4 + m) * n + e];
        mgrw::qcd_event<Proc, T> ev;
        ev.setup(p, mt);
        for (int k = 0; k < npts; ++k) me[int64_t(k) * n + e] = ev.me(pts[k]);
    }
}

template <class Proc, typename T>
void me_events_kpoly(const double* mom, int64_t n, double mt, const mgrw::qcd_point* pts, int npts, double* me) {
    for (int64_t e = 0; e < n; ++e) {
        double p[Proc::NEXT][4];
        for (int i = 0; i < Proc::NEXT; ++i)
            for (int m = 0; m < 4; ++m) p[i][m] = mom[(int64_t(i) * 4 + m) * n + e];
        mgrw::qcd_event<Proc, T> ev;
        ev.setup(p, mt);
        double B[mgrw::kpoly_pairs<Proc>()] = {};
        for (int h = 0; h < Proc::NHEL; ++h) mgrw::kpoly_helicity<Proc, T>(ev.k, ev.b, h, B);
        for (int k = 0; k < npts; ++k) me[int64_t(k) * n + e] = mgrw::kpoly_me<Proc>(B, pts[k].gs, pts[k].gk / pts[k].gs);
    }
}

// |M|^2 through the double-precision cut of a split program: every (chunk,
// flow range) function adds its terms to its range of J, then the colour sum.
template <class Proc, int Q>
void fr_all(const typename Proc::template ext<double>& w, const typename Proc::template kin<double>& k,
            const typename Proc::template coup<double>& c, mgrw::cx<double>* J) {
    if constexpr (Q < Proc::NCHUNK64 * Proc::NFR) {
        constexpr int C = Q / Proc::NFR, R = Q % Proc::NFR;
        Proc::template amplitude_fr<C, R, double>(w, k, c, J + R * Proc::KR);
        fr_all<Proc, Q + 1>(w, k, c, J);
    }
}

template <class Proc>
void me_events_split(const double* mom, int64_t n, double mt, const mgrw::qcd_point* pts, int npts, double* me) {
    for (int64_t e = 0; e < n; ++e) {
        double p[Proc::NEXT][4];
        for (int i = 0; i < Proc::NEXT; ++i)
            for (int m = 0; m < 4; ++m) p[i][m] = mom[(int64_t(i) * 4 + m) * n + e];
        mgrw::qcd_event<Proc, double> ev;
        ev.setup(p, mt);
        for (int kp = 0; kp < npts; ++kp) {
            const auto c = Proc::template couplings<double>(pts[kp].gs, pts[kp].gs2, pts[kp].gk);
            double acc = 0.0;
            for (int h = 0; h < Proc::NHEL; ++h) {
                typename Proc::template ext<double> w;
                Proc::template external<double>(ev.b, h, w);
                mgrw::cx<double> J[Proc::K];
                for (int f = 0; f < Proc::K; ++f) J[f] = {0.0, 0.0};
                fr_all<Proc, 0>(w, ev.k, c, J);
                acc += Proc::colour_sum(J);
            }
            me[int64_t(kp) * n + e] = acc * Proc::point_norm(pts[kp].gs);
        }
    }
}

// add + mul of one helicity of the kappa-polynomial evaluation
template <class Proc>
long long count_kpoly() {
    double p[Proc::NEXT][4];
    for (int i = 0; i < Proc::NEXT; ++i)
        for (int m = 0; m < 4; ++m) p[i][m] = 1.0 + i + 0.25 * m;
    typename Proc::template kin<cfloat> k;
    Proc::kinematics(p, 173.0, k);
    typename Proc::template basis<cfloat> b;
    Proc::external_basis(p, 173.0, b);
    double B[mgrw::kpoly_pairs<Proc>()] = {};
    cfloat::n_add = cfloat::n_mul = 0;
    mgrw::kpoly_helicity<Proc, cfloat>(k, b, 5, B);
    return cfloat::n_add + cfloat::n_mul;
}

// counts[0..1]: add, mul of one helicity program (external wavefunctions,
// diagram chains and colour sum); counts[2..3]: the colour sum alone;
// counts[4..5]: external wavefunctions alone.
template <class Proc>
void count_ops(long long* counts) {
    double p[Proc::NEXT][4];
    for (int i = 0; i < Proc::NEXT; ++i)
        for (int m = 0; m < 4; ++m) p[i][m] = 1.0 + i + 0.25 * m;
    typename Proc::template kin<cfloat> k;
    Proc::kinematics(p, 173.0, k);
    typename Proc::template basis<cfloat> b;
    Proc::external_basis(p, 173.0, b);
    typename Proc::template coup<cfloat> c = {cfloat(1.0), cfloat(1.0), cfloat(1.0)};
    typename Proc::template ext<cfloat> w;
    mgrw::cx<cfloat> J[Proc::K];
    cfloat::n_add = cfloat::n_mul = 0;
    Proc::external(b, 5, w);
    counts[4] = cfloat::n_add;
    counts[5] = cfloat::n_mul;
    Proc::amplitude(w, k, c, J);
    long long a0 = cfloat::n_add, m0 = cfloat::n_mul;
    (void)Proc::colour_sum(J);
    counts[2] = cfloat::n_add - a0;
    counts[3] = cfloat::n_mul - m0;
    counts[0] = cfloat::n_add;
    counts[1] = cfloat::n_mul;
}

}  // namespace

extern "C" {

int mgrw_host_qcd_me(int ng, const double* mom, int64_t n, double mt, const double* pts_gs_gk, int npts,
                     double* me) {
    if (npts < 1 || npts > 64 || n < 0) return -1;
    mgrw::qcd_point pts[64];
    for (int k = 0; k < npts; ++k) {
        double gs = pts_gs_gk[2 * k], kap = pts_gs_gk[2 * k + 1];
        pts[k] = {gs, gs * gs, gs * kap};
    }
    switch (ng) {
        case 2: me_events<mgrw::gg_tt, double>(mom, n, mt, pts, npts, me); return 0;
        case 3: me_events<mgrw::gg_ttg, double>(mom, n, mt, pts, npts, me); return 0;
        case 4: me_events<mgrw::gg_ttgg, double>(mom, n, mt, pts, npts, me); return 0;
        case 5: me_events<mgrw::gg_ttggg, double>(mom, n, mt, pts, npts, me); return 0;
        default: return -2;
    }
}

int mgrw_host_qcd_me_kpoly(int ng, const double* mom, int64_t n, double mt, const double* pts_gs_gk, int npts,
                           double* me) {
    if (npts < 1 || npts > 64 || n < 0) return -1;
    mgrw::qcd_point pts[64];
    for (int k = 0; k < npts; ++k) {
        double gs = pts_gs_gk[2 * k], kap = pts_gs_gk[2 * k + 1];
        pts[k] = {gs, gs * gs, gs * kap};
    }
    switch (ng) {
        case 2: me_events_kpoly<mgrw::gg_tt, double>(mom, n, mt, pts, npts, me); return 0;
        case 3: me_events_kpoly<mgrw::gg_ttg, double>(mom, n, mt, pts, npts, me); return 0;
        case 4: me_events_kpoly<mgrw::gg_ttgg, double>(mom, n, mt, pts, npts, me); return 0;
        default: return -2;
    }
}

// g g -> t tbar g g g through its double-precision (chunk, flow range) cut.
int mgrw_host_qcd_me_split(int ng, const double* mom, int64_t n, double mt, const double* pts_gs_gk, int npts,
                           double* me) {
    if (npts < 1 || npts > 64 || n < 0) return -1;
    if (ng != 5) return -2;
    mgrw::qcd_point pts[64];
    for (int k = 0; k < npts; ++k) {
        double gs = pts_gs_gk[2 * k], kap = pts_gs_gk[2 * k + 1];
        pts[k] = {gs, gs * gs, gs * kap};
    }
    me_events_split<mgrw::gg_ttggg>(mom, n, mt, pts, npts, me);
    return 0;
}

long long mgrw_host_kpoly_flops(int ng) {
    switch (ng) {
        case 2: return count_kpoly<mgrw::gg_tt>();
        case 3: return count_kpoly<mgrw::gg_ttg>();
        case 4: return count_kpoly<mgrw::gg_ttgg>();
        default: return -1;
    }
}

// e+ e- -> 5 photons, |M|^2 for every alpha in alphas; mom SoA [7][4][n].
int mgrw_host_ee5a_me(const double* mom, int64_t n, const double* alphas, int npts, double* me) {
    using Proc = mgrw::ee_5a;
    if (n < 0 || npts < 1) return -1;
    for (int64_t e = 0; e < n; ++e) {
        double p[Proc::NEXT][4];
        for (int i = 0; i < Proc::NEXT; ++i)
            for (int m = 0; m < 4; ++m) p[i][m] = mom[(int64_t(i) * 4 + m) * n + e];
        Proc::event<double> ev;
        Proc::setup(p, ev);
        for (int k = 0; k < npts; ++k) {
            const double ec = std::sqrt(4.0 * M_PI * alphas[k]);
            double acc = 0.0;
            for (int h = 0; h < Proc::NLIVE; ++h) {
                mgrw::cx<double> a = Proc::amplitude<double>(ev, h, ec);
                acc += a.re * a.re + a.im * a.im;
            }
            me[int64_t(k) * n + e] = acc * ev.flux * Proc::NORM;
        }
    }
    return 0;
}

// add + mul of one live helicity configuration of e+ e- -> 5 photons
long long mgrw_host_ee5a_flops() {
    using Proc = mgrw::ee_5a;
    double p[Proc::NEXT][4];
    for (int i = 0; i < Proc::NEXT; ++i)
        for (int m = 0; m < 4; ++m) p[i][m] = 1.0 + i + 0.25 * m;
    Proc::event<cfloat> ev;
    Proc::setup(p, ev);
    cfloat::n_add = cfloat::n_mul = 0;
    mgrw::cx<cfloat> a = Proc::amplitude<cfloat>(ev, 37, cfloat(0.3));
    (void)a;
    return cfloat::n_add + cfloat::n_mul + 3;   // + |a|^2
}

int mgrw_host_qcd_flops(int ng, long long* counts) {
    switch (ng) {
        case 2: count_ops<mgrw::gg_tt>(counts); return 0;
        case 3: count_ops<mgrw::gg_ttg>(counts); return 0;
        case 4: count_ops<mgrw::gg_ttgg>(counts); return 0;
        case 5: count_ops<mgrw::gg_ttggg>(counts); return 0;
        default: return -2;
    }
}

int mgrw_host_ee_mumu_me(const double* mom, int64_t n, const double* pts6, int npts, double* me) {
    if (npts < 1 || npts > 64 || n < 0) return -1;
    mgrw::ew_point pts[64];
    for (int k = 0; k < npts; ++k)
        pts[k] = {pts6[6 * k], pts6[6 * k + 1], pts6[6 * k + 2], pts6[6 * k + 3], pts6[6 * k + 4], pts6[6 * k + 5]};
    for (int64_t e = 0; e < n; ++e) {
        double p[4][4];
        for (int i = 0; i < 4; ++i)
            for (int m = 0; m < 4; ++m) p[i][m] = mom[(int64_t(i) * 4 + m) * n + e];
        mgrw::ee_mumu_event ev;
        ev.setup(p);
        for (int k = 0; k < npts; ++k) me[int64_t(k) * n + e] = ev.me(pts[k]);
    }
    return 0;
}

}  // extern "C"
