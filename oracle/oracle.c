/*
 * Reference oracle for leading-order event reweighting -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the CPU baseline of the benchmark may
 * load this library.  It shares no code with the HIP path.
 *
 * What it computes (all in the scalar type R: double, or __float128 when built
 * with -DORC_QUAD as an outlier referee):
 *
 *  - the squared matrix element |M|^2 of an event, spin-averaged over the
 *    incoming partons, colour-averaged, summed over all outgoing helicities and
 *    colours, with the symmetry factor of identical outgoing gluons (Sec. 2.1,
 *    eq. (1) names |M|^2 as the amplitude factor of the event weight);
 *  - |M|^2 of e+ e- -> n photons (massless QED, all n! diagrams written out);
 *  - the reweighted weight W' = W |M'|^2 / |M|^2 (Sec. 2.2, eq. (3)), quiet NaN
 *    where |M|^2 = 0 (the validity condition stated with eq. (3)).
 *
 * The amplitudes are tree-level helicity amplitudes built from the Feynman
 * rules (Sec. 3.1: amplitudes are helicity amplitudes).  The paper does not fix
 * conventions; the ones used here are textbook:
 *   metric (+,-,-,-); chiral gamma matrices; helicity spinors and transverse
 *   gluon polarisations with vanishing time component in the frame of the
 *   supplied momenta; Feynman gauge; Peskin-Schroeder vertices
 *   (i g kappa gamma^mu T^a for the top-gluon vertex, g f^abc [...] for three
 *   gluons, -i g^2 [f f (g g - g g) + ...] for four gluons, -i g/p^2 and
 *   i(pslash+m)/(p^2-m^2) propagators).  kappa multiplies every top-top-gluon
 *   vertex and nothing else.
 *
 * QCD processes g g -> t tbar + (ng-2) g are computed by a colour-dressed
 * recursion over subsets of gluons (Berends-Giele style: every tree diagram is
 * produced exactly once, each off-shell current summing all sub-diagrams of its
 * subset).  Colour is kept symbolically: a current is a map from ordered words
 * of gluon labels (the product T^{a_w1} ... T^{a_wk}) to Lorentz objects; the
 * structure constants enter through  sum_a T^a f^{abc} = -i [T^b, T^c].  The
 * amplitude is M = sum_w (T^{a_w1}..T^{a_wn})_{i_t j_tbar} J_w, and
 * sum_colours |M|^2 = sum_{w,w'} conj(J_w) CF_{w w'} J_{w'} with the colour
 * matrix CF supplied by the caller (exact rationals, computed by the oracle's
 * Fierz recursion).
 *
 * This code is deliberately plain: explicit 4x4 complex matrices, no fusion,
 * no precomputation beyond the external wavefunctions.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_QUAD
#include <quadmath.h>
typedef __float128 R;
typedef __complex128 C;
#define RSQRT(x) sqrtq(x)
#define RABS(x) fabsq(x)
#define CRE(z) crealq(z)
#define CIM(z) cimagq(z)
#define CONJ(z) conjq(z)
#define API(name) orcq_##name
#define PI_R M_PIq
#define I_C ((C)(__extension__ 1.0i))
#else
#include <complex.h>
typedef double R;
typedef double complex C;
#define RSQRT(x) sqrt(x)
#define RABS(x) fabs(x)
#define CRE(z) creal(z)
#define CIM(z) cimag(z)
#define CONJ(z) conj(z)
#define API(name) orc_##name
#define PI_R 3.14159265358979323846264338327950288
#define I_C ((C)_Complex_I)
#endif

/* ---------------------------------------------------------------- Dirac algebra */

typedef struct { C m[4][4]; } M4;
typedef struct { C c[4]; } S4;      /* spinor (column or row, by context) */
typedef struct { C c[4]; } V4;      /* complex Lorentz vector, upper index */

static const R METRIC[4] = {1, -1, -1, -1};

/* gamma^mu in the chiral representation:
 *   gamma^0 = [[0, 1], [1, 0]],  gamma^k = [[0, sigma^k], [-sigma^k, 0]],
 *   gamma^5 = diag(-1, -1, 1, 1)  (upper components left-handed). */
static M4 gamma_mu(int mu) {
    M4 g;
    memset(&g, 0, sizeof g);
    C s[4][2][2];
    memset(s, 0, sizeof s);
    s[0][0][0] = 1; s[0][1][1] = 1;                 /* identity */
    s[1][0][1] = 1; s[1][1][0] = 1;                 /* sigma_x */
    s[2][0][1] = -I_C; s[2][1][0] = I_C;            /* sigma_y */
    s[3][0][0] = 1; s[3][1][1] = -1;                /* sigma_z */
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            if (mu == 0) {
                g.m[a][2 + b] = s[0][a][b];
                g.m[2 + a][b] = s[0][a][b];
            } else {
                g.m[a][2 + b] = s[mu][a][b];
                g.m[2 + a][b] = -s[mu][a][b];
            }
        }
    return g;
}

static M4 gamma5(void) {
    M4 g;
    memset(&g, 0, sizeof g);
    g.m[0][0] = -1; g.m[1][1] = -1; g.m[2][2] = 1; g.m[3][3] = 1;
    return g;
}

static M4 m4_zero(void) { M4 z; memset(&z, 0, sizeof z); return z; }
static M4 m4_unit(void) { M4 u = m4_zero(); for (int i = 0; i < 4; ++i) u.m[i][i] = 1; return u; }

static M4 m4_add(M4 a, M4 b, C cb) {
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) a.m[i][j] += cb * b.m[i][j];
    return a;
}

static M4 m4_mul(M4 a, M4 b) {
    M4 r = m4_zero();
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) r.m[i][j] += a.m[i][k] * b.m[k][j];
    return r;
}

/* aslash = gamma^mu a_mu = sum_mu g_{mu mu} gamma^mu a^mu  (a complex) */
static M4 slash_c(const C a[4]) {
    M4 r = m4_zero();
    for (int mu = 0; mu < 4; ++mu) r = m4_add(r, gamma_mu(mu), METRIC[mu] * a[mu]);
    return r;
}

static M4 slash_r(const R a[4]) {
    C c[4];
    for (int mu = 0; mu < 4; ++mu) c[mu] = a[mu];
    return slash_c(c);
}

static S4 row_times(S4 row, M4 m) {        /* (row . m)_j = sum_i row_i m_ij */
    S4 r;
    for (int j = 0; j < 4; ++j) {
        r.c[j] = 0;
        for (int i = 0; i < 4; ++i) r.c[j] += row.c[i] * m.m[i][j];
    }
    return r;
}

static S4 times_col(M4 m, S4 col) {
    S4 r;
    for (int i = 0; i < 4; ++i) {
        r.c[i] = 0;
        for (int j = 0; j < 4; ++j) r.c[i] += m.m[i][j] * col.c[j];
    }
    return r;
}

static C row_col(S4 row, S4 col) {
    C s = 0;
    for (int i = 0; i < 4; ++i) s += row.c[i] * col.c[i];
    return s;
}

static S4 bar(S4 col) {                      /* psibar = psi^dagger gamma^0 */
    M4 g0 = gamma_mu(0);
    S4 r;
    for (int j = 0; j < 4; ++j) {
        r.c[j] = 0;
        for (int i = 0; i < 4; ++i) r.c[j] += CONJ(col.c[i]) * g0.m[i][j];
    }
    return r;
}

/* Minkowski products */
static C dot_cc(const C a[4], const C b[4]) {
    C s = 0;
    for (int mu = 0; mu < 4; ++mu) s += METRIC[mu] * a[mu] * b[mu];
    return s;
}
static C dot_cr(const C a[4], const R b[4]) {
    C s = 0;
    for (int mu = 0; mu < 4; ++mu) s += METRIC[mu] * a[mu] * b[mu];
    return s;
}
static R dot_rr(const R a[4], const R b[4]) {
    R s = 0;
    for (int mu = 0; mu < 4; ++mu) s += METRIC[mu] * a[mu] * b[mu];
    return s;
}

/* ---------------------------------------------------- external wavefunctions */

/* Two-component helicity eigenstates chi_lambda(p-hat) of sigma.p-hat. */
static void chi(const R p[4], int lam, C out[2]) {
    R pa = RSQRT(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    R d = pa + p[3];
    if (d <= 0) {                             /* p along -z */
        if (lam > 0) { out[0] = 0; out[1] = 1; }
        else { out[0] = -1; out[1] = 0; }
        return;
    }
    R nrm = RSQRT(2 * pa * d);
    if (lam > 0) { out[0] = d / nrm; out[1] = (p[1] + I_C * p[2]) / nrm; }
    else { out[0] = (-p[1] + I_C * p[2]) / nrm; out[1] = d / nrm; }
}

/* u(p, lam) = (w_{-lam} chi_lam, w_lam chi_lam),  w_pm = sqrt(E pm |p|); for an
 * on-shell particle w_- = sqrt(E - |p|) = m / sqrt(E + |p|), which is used so
 * that massless spinors are exactly chiral. */
static S4 spinor_u(const R p[4], R m, int lam) {
    R pa = RSQRT(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    R wp = RSQRT(p[0] + pa), wm = m / wp;
    C x[2];
    chi(p, lam, x);
    R up = lam > 0 ? wm : wp;                 /* w_{-lam} */
    R lo = lam > 0 ? wp : wm;                 /* w_{lam} */
    S4 s = {{up * x[0], up * x[1], lo * x[0], lo * x[1]}};
    return s;
}

/* v(p, lam) = (-lam w_lam chi_{-lam}, lam w_{-lam} chi_{-lam}) */
static S4 spinor_v(const R p[4], R m, int lam) {
    R pa = RSQRT(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    R wp = RSQRT(p[0] + pa), wm = m / wp;
    C x[2];
    chi(p, -lam, x);
    R wl = lam > 0 ? wp : wm;                 /* w_lam */
    R wml = lam > 0 ? wm : wp;                /* w_{-lam} */
    S4 s = {{-lam * wl * x[0], -lam * wl * x[1], lam * wml * x[0], lam * wml * x[1]}};
    return s;
}

/* eps^mu(k, lam) = (-lam e1 - i e2)/sqrt2 with e1 = (0, cos t cos f, cos t sin f,
 * -sin t), e2 = (0, -sin f, cos f, 0); the conjugate for an outgoing gluon. */
static V4 polvec(const R k[4], int lam, int outgoing) {
    R kt = RSQRT(k[1] * k[1] + k[2] * k[2]);
    R ka = RSQRT(kt * kt + k[3] * k[3]);
    R ct = k[3] / ka, st = kt / ka;
    R cf = 1, sf = 0;
    if (kt > 0) { cf = k[1] / kt; sf = k[2] / kt; }
    R e1[4] = {0, ct * cf, ct * sf, -st};
    R e2[4] = {0, -sf, cf, 0};
    V4 e;
    R is2 = 1 / RSQRT((R)2);
    for (int mu = 0; mu < 4; ++mu) {
        C v = (-lam * e1[mu] - I_C * e2[mu]) * is2;
        e.c[mu] = outgoing ? CONJ(v) : v;
    }
    return e;
}

/* -------------------------------------------------------- e+ e- -> mu+ mu- */

typedef struct { double alpha, sw2, mz, wz; } orc_ew_point;
typedef struct { double alphas, mt, kappa; } orc_qcd_point;

/* Helicity amplitude for e+(p1) e-(p2) -> mu+(p3) mu-(p4) via photon and Z in
 * the s channel; hel[i] = +-1 in particle order. */
static C ee_mumu_amp(const R p[4][4], const int hel[4], const orc_ew_point *pt) {
    R e = RSQRT(4 * PI_R * (R)pt->alpha);
    R sw2 = pt->sw2, cw2 = 1 - sw2;
    R gz = e / RSQRT(sw2 * cw2);
    R gl = -0.5 + sw2, gr = sw2;              /* charged lepton: T3 - Q sw2, -Q sw2 */
    R Q = -1;
    M4 g5 = gamma5(), one = m4_unit();
    M4 PL = m4_add(one, g5, -1), PR = m4_add(one, g5, 1);
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) { PL.m[i][j] *= 0.5; PR.m[i][j] *= 0.5; }
    M4 chir = m4_add(m4_add(m4_zero(), PL, gl), PR, gr);  /* gL PL + gR PR */

    S4 vb1 = bar(spinor_v(p[0], 0, hel[0]));  /* incoming e+ */
    S4 u2 = spinor_u(p[1], 0, hel[1]);        /* incoming e- */
    S4 v3 = spinor_v(p[2], 0, hel[2]);        /* outgoing mu+ */
    S4 ub4 = bar(spinor_u(p[3], 0, hel[3]));  /* outgoing mu- */

    R q[4];
    for (int mu = 0; mu < 4; ++mu) q[mu] = p[0][mu] + p[1][mu];
    R s = dot_rr(q, q);
    C dz = s - (R)pt->mz * (R)pt->mz + I_C * (R)pt->mz * (R)pt->wz;

    C amp = 0;
    for (int mu = 0; mu < 4; ++mu) {
        M4 gm = gamma_mu(mu);
        /* photon: vertices -i e Q gamma, propagator -i g_{mu nu}/s */
        C jin_a = row_col(vb1, times_col(gm, u2)) * (-I_C * e * Q);
        C jout_a = row_col(ub4, times_col(gm, v3)) * (-I_C * e * Q);
        /* Z: vertices -i gz gamma (gL PL + gR PR), propagator -i g_{mu nu}/dz */
        M4 gmz = m4_mul(gm, chir);
        C jin_z = row_col(vb1, times_col(gmz, u2)) * (-I_C * gz);
        C jout_z = row_col(ub4, times_col(gmz, v3)) * (-I_C * gz);
        amp += METRIC[mu] * (jout_a * jin_a * (-I_C / s) + jout_z * jin_z * (-I_C / dz));
    }
    return amp;                               /* i M; |i M|^2 = |M|^2 */
}

/* ----------------------------------------------- g g -> t tbar + n gluons */

#define MAXG 5
#define MAXW 120

static const int FACT[7] = {1, 1, 2, 6, 24, 120, 720};

static int popc(unsigned m) { int c = 0; while (m) { c += m & 1; m >>= 1; } return c; }

/* Rank of an ordered word over the elements of its set, in the lexicographic
 * order of permutations of the sorted elements (Lehmer code). */
static int word_rank(const int *w, int len) {
    int r = 0;
    for (int i = 0; i < len; ++i) {
        int smaller = 0;
        for (int j = i + 1; j < len; ++j) smaller += w[j] < w[i];
        r += smaller * FACT[len - 1 - i];
    }
    return r;
}

/* Inverse: the rank-th permutation of the sorted elements of mask m. */
static void word_unrank(unsigned m, int rank, int *w) {
    int elem[MAXG], n = 0;
    for (int i = 0; i < MAXG; ++i) if (m >> i & 1) elem[n++] = i;
    for (int i = 0; i < n; ++i) {
        int f = FACT[n - 1 - i], k = rank / f;
        rank %= f;
        w[i] = elem[k];
        for (int j = k; j < n - 1 - i; ++j) elem[j] = elem[j + 1];
    }
}

typedef struct {
    int ng;                    /* number of gluons */
    R P[1 << MAXG][4];         /* incoming momentum of each gluon subset */
    V4 eps[MAXG];              /* external gluon vectors for this helicity */
    R pt[4], pbt[4];           /* outgoing t, tbar momenta */
    S4 ubar_t, v_tb;
    R gs, kappa, mt;
    /* currents, per subset, per word */
    V4 gcur[1 << MAXG][MAXW];
    S4 qcur[1 << MAXG][MAXW];  /* row spinors on the t side */
} qcd_ws;

static void v4_axpy(V4 *y, C a, V4 x) { for (int mu = 0; mu < 4; ++mu) y->c[mu] += a * x.c[mu]; }
static void s4_axpy(S4 *y, C a, S4 x) { for (int i = 0; i < 4; ++i) y->c[i] += a * x.c[i]; }

/* Concatenate words; return rank of the concatenation within its set. */
static int cat_rank2(unsigned m1, int r1, unsigned m2, int r2) {
    int w[MAXG], n1 = popc(m1), n2 = popc(m2);
    word_unrank(m1, r1, w);
    word_unrank(m2, r2, w + n1);
    return word_rank(w, n1 + n2);
}

/* rank of the word formed by three sub-words in the given order */
static int cat_rank3(const unsigned *m, const int *r, int a, int b, int c) {
    int w[MAXG], n = 0;
    int idx[3] = {a, b, c};
    for (int k = 0; k < 3; ++k) {
        word_unrank(m[idx[k]], r[idx[k]], w + n);
        n += popc(m[idx[k]]);
    }
    return word_rank(w, n);
}

/* Three-gluon vertex with the propagator left out: for currents J1 (momentum
 * P1 incoming) and J2 (P2 incoming), the Lorentz part of
 * f^{abc}[g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu + g^{rho mu}(q-k)^nu] J1_nu J2_rho
 * with k = -(P1+P2), p = P1, q = P2, index mu raised. */
static V4 vvv(V4 J1, const R P1[4], V4 J2, const R P2[4]) {
    R a[4], b[4], d[4];
    for (int mu = 0; mu < 4; ++mu) {
        a[mu] = P1[mu] - P2[mu];
        b[mu] = P1[mu] + 2 * P2[mu];
        d[mu] = 2 * P1[mu] + P2[mu];
    }
    C j12 = dot_cc(J1.c, J2.c), j1b = dot_cr(J1.c, b), j2d = dot_cr(J2.c, d);
    V4 r;
    for (int mu = 0; mu < 4; ++mu) r.c[mu] = j12 * a[mu] + j1b * J2.c[mu] - j2d * J1.c[mu];
    return r;
}

static void gluon_currents(qcd_ws *ws) {
    int ng = ws->ng;
    unsigned full = (1u << ng) - 1;
    for (int i = 0; i < ng; ++i) ws->gcur[1u << i][0] = ws->eps[i];
    for (int size = 2; size <= ng; ++size) {
        for (unsigned S = 1; S <= full; ++S) {
            if (popc(S) != size) continue;
            int nw = FACT[size];
            for (int w = 0; w < nw; ++w) memset(&ws->gcur[S][w], 0, sizeof(V4));
            R P2 = dot_rr(ws->P[S], ws->P[S]);
            /* three-gluon vertex: (-i/P^2) g (-i) [J1, J2] -> coefficient -g/P^2 */
            C f3 = -ws->gs / P2;
            unsigned low = S & (~S + 1);
            for (unsigned S1 = S; S1; S1 = (S1 - 1) & S) {
                if (!(S1 & low) || S1 == S) continue;
                unsigned S2 = S ^ S1;
                for (int r1 = 0; r1 < FACT[popc(S1)]; ++r1)
                    for (int r2 = 0; r2 < FACT[popc(S2)]; ++r2) {
                        V4 v = vvv(ws->gcur[S1][r1], ws->P[S1], ws->gcur[S2][r2], ws->P[S2]);
                        v4_axpy(&ws->gcur[S][cat_rank2(S1, r1, S2, r2)], f3, v);
                        v4_axpy(&ws->gcur[S][cat_rank2(S2, r2, S1, r1)], -f3, v);
                    }
            }
            /* four-gluon vertex: (-i/P^2)(-i g^2)(-1)[.,[.,.]] -> coefficient +g^2/P^2 */
            C f4 = ws->gs * ws->gs / P2;
            for (unsigned S1 = S; S1; S1 = (S1 - 1) & S) {
                if (!(S1 & low) || S1 == S) continue;
                unsigned rest = S ^ S1;
                unsigned low2 = rest & (~rest + 1);
                for (unsigned S2 = rest; S2; S2 = (S2 - 1) & rest) {
                    if (!(S2 & low2) || S2 == rest) continue;
                    unsigned S3 = rest ^ S2;
                    unsigned m[3] = {S1, S2, S3};
                    int r[3];
                    for (r[0] = 0; r[0] < FACT[popc(S1)]; ++r[0])
                        for (r[1] = 0; r[1] < FACT[popc(S2)]; ++r[1])
                            for (r[2] = 0; r[2] < FACT[popc(S3)]; ++r[2]) {
                                V4 J1 = ws->gcur[S1][r[0]], J2 = ws->gcur[S2][r[1]], J3 = ws->gcur[S3][r[2]];
                                C d12 = dot_cc(J1.c, J2.c), d13 = dot_cc(J1.c, J3.c), d23 = dot_cc(J2.c, J3.c);
                                V4 LA, LB, LC;
                                for (int mu = 0; mu < 4; ++mu) {
                                    LA.c[mu] = J2.c[mu] * d13 - J3.c[mu] * d12;
                                    LB.c[mu] = J1.c[mu] * d23 - J3.c[mu] * d12;
                                    LC.c[mu] = J1.c[mu] * d23 - J2.c[mu] * d13;
                                }
                                /* [1,[2,3]] = 123 - 132 - 231 + 321 */
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 0, 1, 2)], f4, LA);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 0, 2, 1)], -f4, LA);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 1, 2, 0)], -f4, LA);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 2, 1, 0)], f4, LA);
                                /* [2,[1,3]] = 213 - 231 - 132 + 312 */
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 1, 0, 2)], f4, LB);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 1, 2, 0)], -f4, LB);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 0, 2, 1)], -f4, LB);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 2, 0, 1)], f4, LB);
                                /* [3,[1,2]] = 312 - 321 - 123 + 213 */
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 2, 0, 1)], f4, LC);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 2, 1, 0)], -f4, LC);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 0, 1, 2)], -f4, LC);
                                v4_axpy(&ws->gcur[S][cat_rank3(m, r, 1, 0, 2)], f4, LC);
                            }
                }
            }
        }
    }
}

/* Top line, built from the outgoing top: qcur[S] = ubar(t) [vertices with the
 * gluons of S attached in word order, each followed by its propagator].  The
 * fermion momentum after attaching S is q = p_t - P(S). Then the amplitude. */
static void top_line(qcd_ws *ws, C *J) {
    int ng = ws->ng;
    unsigned full = (1u << ng) - 1;
    C vtx = I_C * ws->gs * ws->kappa;          /* i g kappa gamma^mu T^a */
    ws->qcur[0][0] = ws->ubar_t;
    for (int size = 1; size < ng; ++size) {
        for (unsigned S = 1; S < full; ++S) {
            if (popc(S) != size) continue;
            for (int w = 0; w < FACT[size]; ++w) memset(&ws->qcur[S][w], 0, sizeof(S4));
            R q[4];
            for (int mu = 0; mu < 4; ++mu) q[mu] = ws->pt[mu] - ws->P[S][mu];
            M4 prop = slash_r(q);
            for (int i = 0; i < 4; ++i) prop.m[i][i] += ws->mt;
            C pf = I_C / (dot_rr(q, q) - ws->mt * ws->mt);   /* i (qslash + m)/(q^2 - m^2) */
            for (unsigned S1 = S; S1; S1 = (S1 - 1) & S) {
                unsigned S0 = S ^ S1;               /* attached before S1 */
                for (int r0 = 0; r0 < FACT[popc(S0)]; ++r0)
                    for (int r1 = 0; r1 < FACT[popc(S1)]; ++r1) {
                        M4 js = slash_c(ws->gcur[S1][r1].c);
                        S4 t = row_times(row_times(ws->qcur[S0][r0], js), prop);
                        s4_axpy(&ws->qcur[S][cat_rank2(S0, r0, S1, r1)], vtx * pf, t);
                    }
            }
        }
    }
    for (int w = 0; w < FACT[ng]; ++w) J[w] = 0;
    for (unsigned S1 = full; S1; S1 = (S1 - 1) & full) {
        unsigned S0 = full ^ S1;
        for (int r0 = 0; r0 < FACT[popc(S0)]; ++r0)
            for (int r1 = 0; r1 < FACT[popc(S1)]; ++r1) {
                M4 js = slash_c(ws->gcur[S1][r1].c);
                C a = row_col(row_times(ws->qcur[S0][r0], js), ws->v_tb);
                J[cat_rank2(S0, r0, S1, r1)] += vtx * a;
            }
    }
}

/* Particle order: g(0) g(1) t(2) tbar(3) g(4) ...; gluon i <-> particle
 * gl[i] = {0, 1, 4, 5, 6}. gauge_leg >= 0 replaces that gluon's polarisation by
 * its momentum (Ward identity checks). */
static const int GLUON_PARTICLE[MAXG] = {0, 1, 4, 5, 6};

static void qcd_flows(qcd_ws *ws, int ng, const R p[][4], const int *hel,
                      const orc_qcd_point *pt, int gauge_leg, C *J) {
    ws->ng = ng;
    ws->gs = RSQRT(4 * PI_R * (R)pt->alphas);
    ws->kappa = pt->kappa;
    ws->mt = pt->mt;
    R kin[MAXG][4];
    for (int i = 0; i < ng; ++i) {
        int ip = GLUON_PARTICLE[i];
        R sgn = ip < 2 ? 1 : -1;              /* incoming momentum into the diagram */
        for (int mu = 0; mu < 4; ++mu) kin[i][mu] = sgn * p[ip][mu];
        if (i == gauge_leg) {
            for (int mu = 0; mu < 4; ++mu) ws->eps[i].c[mu] = p[ip][mu];
        } else {
            ws->eps[i] = polvec(p[ip], hel[ip], ip >= 2);
        }
    }
    for (unsigned S = 0; S < (1u << ng); ++S)
        for (int mu = 0; mu < 4; ++mu) {
            R s = 0;
            for (int i = 0; i < ng; ++i) if (S >> i & 1) s += kin[i][mu];
            ws->P[S][mu] = s;
        }
    for (int mu = 0; mu < 4; ++mu) { ws->pt[mu] = p[2][mu]; ws->pbt[mu] = p[3][mu]; }
    ws->ubar_t = bar(spinor_u(p[2], ws->mt, hel[2]));
    ws->v_tb = spinor_v(p[3], ws->mt, hel[3]);
    gluon_currents(ws);
    top_line(ws, J);
}

static R colour_sum(int K, const C *J, const double *cf) {
    R s = 0;
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) s += (R)cf[a * K + b] * CRE(CONJ(J[a]) * J[b]);
    return s;
}

/* ------------------------------------------------------------------ exports */

/* Single-event colour-ordered amplitudes J_w (K = ng! words, lexicographic
 * order of permutations of the gluon labels 0..ng-1) for one helicity. */
int API(qcd_flows)(int ng, const double *mom_aos, const int *hel, const orc_qcd_point *pt,
                   int gauge_leg, double *J_out) {
    if (ng < 2 || ng > MAXG) return -1;
    int next = ng + 2;
    R p[7][4];
    for (int i = 0; i < next; ++i) for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom_aos[i * 4 + mu];
    qcd_ws *ws = (qcd_ws *)malloc(sizeof(qcd_ws));
    if (!ws) return -2;
    C J[MAXW];
    qcd_flows(ws, ng, (const R(*)[4])p, hel, pt, gauge_leg, J);
    for (int w = 0; w < FACT[ng]; ++w) { J_out[2 * w] = (double)CRE(J[w]); J_out[2 * w + 1] = (double)CIM(J[w]); }
    free(ws);
    return 0;
}

/* |M|^2 of g g -> t tbar + (ng-2) g for every event and parameter point.
 * mom: SoA [ng+2][4][n]; me: [npts][n]; cf: [K][K] colour matrix. */
/* Threads of the OpenMP loops (timing of the oracle only). */
void API(set_threads)(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int API(max_threads)(void) { return omp_get_max_threads(); }

int API(qcd_me)(int ng, const double *mom, int64_t n, const orc_qcd_point *pts, int npts,
                const double *cf, double *me) {
    if (ng < 2 || ng > MAXG || n < 0 || npts < 1) return -1;
    int next = ng + 2, K = FACT[ng], nhel = 1 << next;
    R norm = (R)1 / (4 * 64 * FACT[ng - 2]);  /* spins, gluon colours, identical gluons */
    int fail = 0;
#pragma omp parallel
    {
        qcd_ws *ws = (qcd_ws *)malloc(sizeof(qcd_ws));
        if (!ws) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t e = 0; e < n; ++e) {
            if (!ws) continue;
            R p[7][4];
            for (int i = 0; i < next; ++i)
                for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom[((int64_t)i * 4 + mu) * n + e];
            for (int k = 0; k < npts; ++k) {
                R acc = 0;
                for (int h = 0; h < nhel; ++h) {
                    int hel[7];
                    for (int i = 0; i < next; ++i) hel[i] = (h >> (next - 1 - i) & 1) ? 1 : -1;
                    C J[MAXW];
                    qcd_flows(ws, ng, (const R(*)[4])p, hel, &pts[k], -1, J);
                    acc += colour_sum(K, J, cf);
                }
                me[(int64_t)k * n + e] = (double)(acc * norm);
            }
        }
        free(ws);
    }
    return fail ? -2 : 0;
}

/* |M|^2 of e+ e- -> mu+ mu-, all 16 helicities summed, averaged over 4. */
int API(ee_mumu_me)(const double *mom, int64_t n, const orc_ew_point *pts, int npts, double *me) {
    if (n < 0 || npts < 1) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        R p[4][4];
        for (int i = 0; i < 4; ++i)
            for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom[((int64_t)i * 4 + mu) * n + e];
        for (int k = 0; k < npts; ++k) {
            R acc = 0;
            for (int h = 0; h < 16; ++h) {
                int hel[4];
                for (int i = 0; i < 4; ++i) hel[i] = (h >> (3 - i) & 1) ? 1 : -1;
                C a = ee_mumu_amp((const R(*)[4])p, hel, &pts[k]);
                acc += CRE(a * CONJ(a));
            }
            me[(int64_t)k * n + e] = (double)(acc / 4);
        }
    }
    return 0;
}

/* Single helicity amplitude of e+ e- -> mu+ mu- (for per-helicity checks). */
int API(ee_mumu_amp)(const double *mom_aos, const int *hel, const orc_ew_point *pt, double *out) {
    R p[4][4];
    for (int i = 0; i < 4; ++i) for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom_aos[i * 4 + mu];
    C a = ee_mumu_amp((const R(*)[4])p, hel, pt);
    out[0] = (double)CRE(a);
    out[1] = (double)CIM(a);
    return 0;
}

/* ------------------------------------------------ e+ e- -> n photons (QED)
 *
 * e+(p0) e-(p1) -> gamma(p2) ... gamma(p_{n+1}) with a massless electron.
 * Each of the n! Feynman diagrams attaches the photons to the electron line in
 * one order s_1 .. s_n (counted from the electron end):
 *   M_s = vbar(p0) V_{s_n} S(q_{n-1}) V_{s_{n-1}} ... V_{s_2} S(q_1) V_{s_1} u(p1),
 *   q_j = p1 - k_{s_1} - ... - k_{s_j},  V_i = -i e Q eps_i*-slash (Q = -1),
 *   S(q) = i qslash / q^2,
 * and M is the sum over all n! orders, each written out as its own product.
 * gauge_leg >= 0 replaces that photon's polarisation by its momentum (the
 * Ward identity makes the amplitude vanish). */

#define MAXA 6

static int next_perm(int *a, int n) {          /* lexicographic successor */
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

static C ee_photons_amp(int na, const R p[][4], const int *hel, R e, int gauge_leg) {
    S4 vb = bar(spinor_v(p[0], 0, hel[0]));     /* incoming e+ */
    S4 u = spinor_u(p[1], 0, hel[1]);           /* incoming e- */
    const R Q = -1;
    M4 V[MAXA];
    for (int i = 0; i < na; ++i) {
        C eps[4];
        if (i == gauge_leg) {
            for (int mu = 0; mu < 4; ++mu) eps[mu] = p[2 + i][mu];
        } else {
            V4 ev = polvec(p[2 + i], hel[2 + i], 1);
            for (int mu = 0; mu < 4; ++mu) eps[mu] = ev.c[mu];
        }
        M4 sl = slash_c(eps);
        V[i] = m4_add(m4_zero(), sl, -I_C * e * Q);
    }
    int perm[MAXA];
    for (int i = 0; i < na; ++i) perm[i] = i;
    C amp = 0;
    do {
        S4 psi = u;
        R q[4];
        for (int mu = 0; mu < 4; ++mu) q[mu] = p[1][mu];
        for (int j = 0; j < na; ++j) {
            psi = times_col(V[perm[j]], psi);
            if (j + 1 < na) {
                for (int mu = 0; mu < 4; ++mu) q[mu] -= p[2 + perm[j]][mu];
                M4 prop = m4_add(m4_zero(), slash_r(q), I_C / dot_rr(q, q));
                psi = times_col(prop, psi);
            }
        }
        amp += row_col(vb, psi);
    } while (next_perm(perm, na));
    return amp;
}

/* |M|^2 of e+ e- -> na photons for every event and every alpha: all 2^(na+2)
 * helicity configurations summed, averaged over the 4 initial spins, divided
 * by na! for the identical photons.  mom: [na+2][4][n] (SoA). */
int API(ee_photons_me)(int na, const double *mom, int64_t n, const double *alpha, int npts, double *me) {
    if (na < 1 || na > MAXA || n < 0 || npts < 1) return -1;
    const int next = na + 2;
    R fact = 1;
    for (int i = 2; i <= na; ++i) fact *= i;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ev = 0; ev < n; ++ev) {
        R p[MAXA + 2][4];
        for (int i = 0; i < next; ++i)
            for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom[((int64_t)i * 4 + mu) * n + ev];
        for (int k = 0; k < npts; ++k) {
            R e = RSQRT(4 * PI_R * (R)alpha[k]);
            R acc = 0;
            for (int h = 0; h < (1 << next); ++h) {
                int hel[MAXA + 2];
                for (int i = 0; i < next; ++i) hel[i] = (h >> (next - 1 - i) & 1) ? 1 : -1;
                C a = ee_photons_amp(na, (const R(*)[4])p, hel, e, -1);
                acc += CRE(a * CONJ(a));
            }
            me[(int64_t)k * n + ev] = (double)(acc / 4 / fact);
        }
    }
    return 0;
}

/* One helicity amplitude (hel[i] = +-1 in particle order), out = (re, im). */
int API(ee_photons_amp)(int na, const double *mom_aos, const int *hel, double alpha, int gauge_leg,
                        double *out) {
    if (na < 1 || na > MAXA) return -1;
    R p[MAXA + 2][4];
    for (int i = 0; i < na + 2; ++i) for (int mu = 0; mu < 4; ++mu) p[i][mu] = mom_aos[i * 4 + mu];
    C a = ee_photons_amp(na, (const R(*)[4])p, hel, RSQRT(4 * PI_R * (R)alpha), gauge_leg);
    out[0] = (double)CRE(a);
    out[1] = (double)CIM(a);
    return 0;
}

/* Eq. (3): W'_k = W * me[k] / me[0] for k = 1..npts-1; NaN where me[0] = 0.
 * w_in may be NULL (W = 1). w_out: [npts-1][n]. */
int API(reweight)(const double *me, int npts, int64_t n, const double *w_in, double *w_out) {
    if (npts < 1 || n < 0) return -1;
    for (int k = 1; k < npts; ++k)
        for (int64_t e = 0; e < n; ++e) {
            double w = w_in ? w_in[e] : 1.0;
            double m0 = me[e];
            w_out[(int64_t)(k - 1) * n + e] = m0 != 0.0 ? w * (me[(int64_t)k * n + e] / m0) : NAN;
        }
    return 0;
}

/* External wavefunctions, exported for the spinor/polarisation pins.
 * kind: 0 u, 1 v, 2 ubar, 3 vbar, 4 eps (incoming), 5 eps* (outgoing). */
int API(wavefunction)(int kind, const double *p_in, double m, int lam, double *out) {
    R p[4];
    for (int mu = 0; mu < 4; ++mu) p[mu] = p_in[mu];
    C c[4];
    if (kind <= 3) {
        S4 s = (kind == 0 || kind == 2) ? spinor_u(p, m, lam) : spinor_v(p, m, lam);
        if (kind >= 2) s = bar(s);
        for (int i = 0; i < 4; ++i) c[i] = s.c[i];
    } else if (kind <= 5) {
        V4 e = polvec(p, lam, kind == 5);
        for (int i = 0; i < 4; ++i) c[i] = e.c[i];
    } else {
        return -1;
    }
    for (int i = 0; i < 4; ++i) { out[2 * i] = (double)CRE(c[i]); out[2 * i + 1] = (double)CIM(c[i]); }
    return 0;
}
