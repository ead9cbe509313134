/*
 * qed_oracle.c -- plain FP64 CPU oracle of the spin- and polarization-resolved
 * strong-field QED particle step of arXiv 2511.08929 (Qian et al.).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Written directly from
 * the paper's formulas, in the paper's order, for a reader to check by eye.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *  R1  Basis: khat = p/|p|; eps = unit(-q (E + v x B) perpendicular to khat) with q = -1
 *      for electrons and photons, +1 for positrons; beta = khat x eps (right-handed).
 *      The printed spectra are non-negative for every pure state only in this
 *      handedness; the orientation makes electrons polarize against the rest-frame B.
 *      For photons (NBW) the electron-line convention rests on the crossing symmetry of
 *      the outgoing-electron term; beyond positivity that orientation is parity unpinned.
 *  R2  Last term of G3 (NBW appendix, Bessel form) taken with a plus sign, as in the
 *      Airy form of the same equation.
 *  R3  Both branches of the spin-up/down inverse-CDF selection in the NLC section print
 *      the up table; the first branch is read as the down table (as in the NBW section).
 *  R4  Rate prefactor alpha m c^2 / (sqrt(3) pi hbar gamma) (the Sokolov-Ternov
 *      equation's prefactor lacks the 1/pi); in 1/omega_r units: alpha/(sqrt3 pi eps_r gamma).
 *  R5  Per-step probability W dt > 1 is clamped: the event always happens and the
 *      down/up (or -/+) branch uses r1 < a/P, which keeps the mixture exact.
 *  R6  The no-transition update of the non-transition section can leave |s| > 1 at
 *      finite dt; the result is renormalised to unit length and counted.
 *  R7  Pair-spin thresholds of the NBW section are read as cumulative sums of
 *      G(down,down), G(down,up), G(up,down), G(up,up) over 4 w0 (first arrow positron).
 *  R8  Photon-polarization collapse picks +/- Xi (the section writes s_f where xi is meant).
 *  R9  T-BMT with the standard E-term coefficient (a + 1/(gamma+1)); Cayley rotation with
 *      the Boris mid-step gamma, so that g = 2 keeps the spin-momentum angle.
 *  R10 Optical-depth decision (the alternative of the decision-making overview): tau grows by
 *      the spin-weighted W dt each step, in FP64; emission when tau >= tau*, with tau* =
 *      -ln(1 - u) drawn from Philox channel 4 (53-bit words 0,1 when no target is set yet,
 *      words 2,3 after an emission, when tau restarts at 0).  The up/down branch is then
 *      r1 < a/P with the step's r1; without emission the no-transition update is the same as
 *      with the per-step draw, applied only while W dt < 1 (otherwise skipped and counted).
 *  R11 Field-dependent g (loop appendix): the Scorer-function term of the one-loop
 *      self-energy is taken as the anomalous moment a(chi) of the T-BMT equation, with
 *      a(chi)/a(0) = 2 pi int_0^inf du/(1+u)^3 z Gi(z), z = (u/chi)^(2/3) (the standard one-loop
 *      form; the appendix's own prefactors are garbled).  chi is taken at the Boris mid step
 *      (momentum (u- + u+)/2, energy gamma-), and the ratio is tabulated like the rates: ln of it
 *      at 64 nodes per decade of chi from 1e-7 to 1e4, 4-point Lagrange in ln chi; 1 below,
 *      the chi^(-2/3) law above.
 *  R12 Sub-cycling (the decision-making section requires W dt << 1 and flags the accuracy of
 *      the per-step draw as the weak point): after the push a lepton takes m sub-steps of the
 *      whole QED part, m the smallest power of two with W_s dt / m <= 0.1 (at most 16), W_s dt
 *      at the state after the push; the sub-steps run in 16 rounds over the set (a lepton takes
 *      one in every 16/m-th round), with the Philox channels of round r offset by 16 r and r in
 *      the photon id, each round's photons appended after the previous round's.
 */
#include "qed_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ALPHA 7.2973525693e-3
#define ORC_PI 3.14159265358979323846
#define BESSEL_XMAX 700.0
#define NLC_NU_LO (-60.0)

/* ====================================================================== */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its definition. */
/* ====================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u01_53(uint32_t hi, uint32_t lo)
{
    uint64_t m = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
    return ((double)m + 0.5) * 0x1p-53;
}

double orc_u01_24(uint32_t hi)
{
    return (double)(2u * (hi >> 9) + 1u) * 0x1p-24;
}

static void philox_block(uint64_t seed, uint64_t id, int64_t step, uint32_t channel, uint32_t w[4])
{
    uint32_t c[4] = {(uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step, channel};
    uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(c, k, w);
}

/* two uniforms (pairs of words 0,1 and 2,3) from one Philox block */
static void uniforms2(const orc_params *prm, uint64_t id, uint32_t channel, double *ra, double *rb)
{
    uint32_t w[4];
    philox_block(prm->seed, id, prm->step, channel + 16u * (uint32_t)prm->sub_round, w);
    if (prm->u24) { *ra = orc_u01_24(w[0]); *rb = orc_u01_24(w[2]); }
    else          { *ra = orc_u01_53(w[0], w[1]); *rb = orc_u01_53(w[2], w[3]); }
}

/* ====================================================================== */
/* Modified Bessel functions K_{1/3}, K_{2/3} and IntK_{1/3}(x) = int_x^inf K_{1/3}. */
/* Small x: the textbook ascending series K_nu = pi/(2 sin nu pi) (I_-nu - I_nu).    */
/* Otherwise: K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt and                   */
/*            IntK_1/3(x) = int_0^inf exp(-x cosh t) cosh(t/3)/cosh(t) dt,           */
/* by composite 20-point Gauss-Legendre quadrature in t.                              */
/* ====================================================================== */
#define NGL 20
static double gl_x[NGL], gl_w[NGL];

__attribute__((constructor)) static void gl_init(void)
{
    const int n = NGL;
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-17) break;
        }
        /* one more evaluation at the converged node for the weight */
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1.0);
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* sum_k (x/2)^(2k+mu) / (k! Gamma(k+mu+1)) and its integral from 0 to x */
static void bessel_i_series(double x, double mu, double *I, double *intI)
{
    double h = 0.5 * x, h2 = h * h;
    double term = pow(h, mu) / tgamma(mu + 1.0);
    double sum = 0.0, isum = 0.0;
    for (int k = 0; k < 60; ++k) {
        sum += term;
        isum += 2.0 * term * h / (2.0 * k + mu + 1.0);
        if (term < 1e-19 * sum) break;
        term *= h2 / ((k + 1.0) * (k + 1.0 + mu));
    }
    *I = sum;
    *intI = isum;
}

void orc_bessel3(double x, double out[3])
{
    if (!(x < BESSEL_XMAX)) { out[0] = out[1] = out[2] = 0.0; return; }
    if (x < 0.1) {
        double a, ia, b, ib, c, ic, d, id;
        bessel_i_series(x, -1.0 / 3.0, &a, &ia);
        bessel_i_series(x, 1.0 / 3.0, &b, &ib);
        bessel_i_series(x, -2.0 / 3.0, &c, &ic);
        bessel_i_series(x, 2.0 / 3.0, &d, &id);
        double f13 = ORC_PI / (2.0 * sin(ORC_PI / 3.0));
        double f23 = ORC_PI / (2.0 * sin(2.0 * ORC_PI / 3.0));
        out[0] = f13 * (a - b);
        out[1] = f23 * (c - d);
        out[2] = ORC_PI / sqrt(3.0) - f13 * (ia - ib);
        return;
    }
    double T = acosh(1.0 + 800.0 / x);
    double width = fmin(1.0, 1.0 / sqrt(x));
    int np = (int)ceil(T / width);
    double ex = exp(-x);
    double k13 = 0.0, k23 = 0.0, ik = 0.0;
    for (int j = 0; j < np; ++j) {
        double a = j * width, b = (j + 1) * width;
        double mid = 0.5 * (a + b), half = 0.5 * (b - a);
        double s13 = 0.0, s23 = 0.0, sik = 0.0;
        for (int i = 0; i < NGL; ++i) {
            double t = mid + half * gl_x[i];
            double sh = sinh(0.5 * t);
            double e = ex * exp(-2.0 * x * sh * sh);   /* exp(-x cosh t), cosh t - 1 = 2 sinh^2(t/2) */
            double z = exp(t / 3.0), zi = 1.0 / z;
            double c1 = 0.5 * (z + zi);                       /* cosh(t/3)  */
            double c2 = 0.5 * (z * z + zi * zi);              /* cosh(2t/3) */
            double ch = 1.0 + 2.0 * sh * sh;                  /* cosh(t)    */
            s13 += gl_w[i] * e * c1;
            s23 += gl_w[i] * e * c2;
            sik += gl_w[i] * e * c1 / ch;
        }
        k13 += half * s13;
        k23 += half * s23;
        ik += half * sik;
    }
    out[0] = k13; out[1] = k23; out[2] = ik;
}

/* ====================================================================== */
/* Spectra (appendix, Bessel forms).  Components are taken in the basis    */
/* (eps, beta, khat): index 0 = eps, 1 = beta, 2 = khat.                   */
/* lam = photon / lepton momentum ratio (NLC) or positron / photon (NBW).  */
/* ====================================================================== */
typedef struct { double lam, oml, K13, K23, IK; } spec_pt;

/* NLC quantities at lam for given chi: u = lam/(1-lam), u' = 2u/(3 chi) */
static spec_pt nlc_point(double chi, double lam, double oml)
{
    spec_pt s; double B[3];
    s.lam = lam; s.oml = oml;
    double u = lam / oml;
    orc_bessel3(2.0 * u / (3.0 * chi), B);
    s.K13 = B[0]; s.K23 = B[1]; s.IK = B[2];
    return s;
}

/* NBW quantities: u~ = 1/lam + 1/(1-lam), u~' = 2 u~ /(3 chi) */
static spec_pt nbw_point(double chi, double lam, double oml)
{
    spec_pt s; double B[3];
    s.lam = lam; s.oml = oml;
    double ut = 1.0 / lam + 1.0 / oml;
    orc_bessel3(2.0 * ut / (3.0 * chi), B);
    s.K13 = B[0]; s.K23 = B[1]; s.IK = B[2];
    return s;
}

/* w = -IntK + kappa K23 + lam (s_i . beta) K13  (NLC appendix, eq. for w) */
static double nlc_w_pt(const spec_pt *q, double sb)
{
    double kappa = 1.0 / q->oml + q->oml;
    return -q->IK + kappa * q->K23 + q->lam * sb * q->K13;
}

/* g = u K13 beta + (-IntK + 2 K23) s_i + lam u (-IntK + K23)(s_i . k) k */
static void nlc_g_pt(const spec_pt *q, const double si[3], double g[3])
{
    double u = q->lam / q->oml;
    double c = -q->IK + 2.0 * q->K23;
    g[0] = c * si[0];
    g[1] = u * q->K13 + c * si[1];
    g[2] = c * si[2] + q->lam * u * (-q->IK + q->K23) * si[2];
}

/* F0 and F = (F1, F2, F3) for initial spin a = s_i and final spin b = s_f (NLC appendix) */
static void nlc_F_pt(const spec_pt *q, const double a[3], const double b[3], double F[4])
{
    double lam = q->lam, oml = q->oml, u = lam / oml;
    double kap = 1.0 / oml + oml, kapt = 1.0 / oml - oml;
    double I = q->IK, K1 = q->K13, K2 = q->K23;
    double g[3];
    nlc_g_pt(q, a, g);
    F[0] = nlc_w_pt(q, a[1]) + b[0] * g[0] + b[1] * g[1] + b[2] * g[2];
    /* (s_f x s_i) . khat and (s_f x s_i) . eps in the right-handed (eps, beta, khat) basis */
    double cross_k = b[0] * a[1] - b[1] * a[0];
    double cross_e = b[1] * a[2] - b[2] * a[1];
    F[1] = -K1 * (u * a[0] + lam * b[0])
           - 0.5 * lam * u * I * (b[0] * a[1] + b[1] * a[0])
           + 0.5 * kapt * K2 * cross_k;
    F[2] = 0.5 * kapt * K1 * cross_e
           - (lam * I - kapt * K2) * a[2]
           - (u * I - kapt * K2) * b[2]
           + 0.5 * lam * u * K1 * (b[2] * a[1] + b[1] * a[2]);
    F[3] = K2 + (u * a[1] + lam * b[1]) * K1
           - 0.5 * lam * u * I * (b[0] * a[0] - b[1] * a[1])
           + 0.5 * kap * K2 * (b[0] * a[0] + b[1] * a[1] + b[2] * a[2])
           - 0.5 * lam * u * K2 * b[2] * a[2];
}

/* G0 and G = (G1, G2, G3) for electron spin e = s_e and positron spin p = s_p (NBW appendix;
   last term of G3 with a plus sign, reading R2) */
static void nbw_G_pt(const spec_pt *q, const double e[3], const double p[3], double G[4])
{
    double lam = q->lam, oml = q->oml;
    double ut = 1.0 / lam + 1.0 / oml;
    double rho = oml / lam + lam / oml, rhot = oml / lam - lam / oml;
    double I = q->IK, K1 = q->K13, K2 = q->K23;
    double pe = p[0] * e[0] + p[1] * e[1] + p[2] * e[2];
    double cross_k = p[0] * e[1] - p[1] * e[0];     /* (s_p x s_e) . khat */
    double cross_e = p[1] * e[2] - p[2] * e[1];     /* (s_p x s_e) . eps  */
    G[0] = I + rho * K2 + e[1] * K1 / oml - p[1] * K1 / lam
           + (I - 2.0 * K2) * pe
           + (rho * I - (rho - 2.0) * K2) * p[2] * e[2];
    G[1] = K1 * (e[0] / lam - p[0] / oml)
           - 0.5 * ut * I * (p[0] * e[1] + p[1] * e[0])
           + 0.5 * rhot * K2 * cross_k;
    G[2] = -0.5 * ut * K1 * cross_e
           + (I / oml + rhot * K2) * e[2]
           + (I / lam - rhot * K2) * p[2]
           - 0.5 * rhot * K1 * (p[2] * e[1] + p[1] * e[2]);
    G[3] = -K2 + (-e[1] / lam + p[1] / oml) * K1
           - 0.5 * ut * I * (p[0] * e[0] - p[1] * e[1])
           + 0.5 * rho * K2 * pe
           + (1.0 - 0.5 * rho) * K2 * p[2] * e[2];
}

/* w0, j_e, j_p (NBW appendix): marginals of G over the other lepton's spin */
static void nbw_j_pt(const spec_pt *q, const double xi[3], double *w0, double je[3], double jp[3])
{
    double lam = q->lam, oml = q->oml;
    double rho = oml / lam + lam / oml, rhot = oml / lam - lam / oml;
    double I = q->IK, K1 = q->K13, K2 = q->K23;
    *w0 = I + rho * K2 - xi[2] * K2;
    je[0] = xi[0] * K1 / lam;
    je[1] = (1.0 / oml - xi[2] / lam) * K1;
    je[2] = xi[1] * (I / oml + rhot * K2);
    jp[0] = -xi[0] * K1 / oml;
    jp[1] = (-1.0 / lam + xi[2] / oml) * K1;
    jp[2] = xi[1] * (I / lam - rhot * K2);
}

double orc_nlc_w(double chi, double lam, double sb)
{
    spec_pt q = nlc_point(chi, lam, 1.0 - lam);
    return nlc_w_pt(&q, sb);
}
void orc_nlc_g(double chi, double lam, const double si[3], double g[3])
{
    spec_pt q = nlc_point(chi, lam, 1.0 - lam);
    nlc_g_pt(&q, si, g);
}
void orc_nlc_F(double chi, double lam, const double si[3], const double sf[3], double F[4])
{
    spec_pt q = nlc_point(chi, lam, 1.0 - lam);
    nlc_F_pt(&q, si, sf, F);
}
void orc_nbw_G(double chi, double lam, const double se[3], const double sp[3], double G[4])
{
    spec_pt q = nbw_point(chi, lam, 1.0 - lam);
    nbw_G_pt(&q, se, sp, G);
}
void orc_nbw_j(double chi, double lam, const double xi[3], double *w0, double je[3], double jp[3])
{
    spec_pt q = nbw_point(chi, lam, 1.0 - lam);
    nbw_j_pt(&q, xi, w0, je, jp);
}

/* ====================================================================== */
/* Exact rates and inverse CDFs.  The spectrum is integrated in            */
/* nu = ln(lam/(1-lam)), where dlam = lam (1-lam) dnu; the density in nu   */
/* is smooth and decays at both ends.  NLC below nu = -60 uses the leading */
/* small-lam law int_0^lam w = 3 Gamma(2/3) (3 chi)^(2/3) lam^(1/3)        */
/* - (pi/sqrt3) lam (relative remainder < 1e-26 there).                    */
/* ====================================================================== */
static void lam_from_nu(double nu, double *lam, double *oml)
{
    *lam = 1.0 / (1.0 + exp(-nu));
    *oml = 1.0 / (1.0 + exp(nu));
}

double orc_density_nu(int ch, double chi, double nu)
{
    double lam, oml;
    lam_from_nu(nu, &lam, &oml);
    if (ch < 2) {
        spec_pt q = nlc_point(chi, lam, oml);
        return nlc_w_pt(&q, ch == 1 ? 1.0 : -1.0) * lam * oml;
    } else {
        spec_pt q = nbw_point(chi, lam, oml);
        double rho = oml / lam + lam / oml;
        double w0 = q.IK + rho * q.K23 - (ch == 3 ? 1.0 : -1.0) * q.K23;
        return w0 * lam * oml;
    }
}

static double nlc_tail(double chi, double lam)
{
    double A = 3.0 * tgamma(2.0 / 3.0) * pow(3.0 * chi, 2.0 / 3.0);
    return A * cbrt(lam) - ORC_PI / sqrt(3.0) * lam;
}

typedef struct {
    int ch; double chi;
    int np; double a0, b_end;
    double *edge_nu;        /* panel boundaries, np + 1 */
    double *left, *right;   /* cumulative integrals at panel edges */
    double tail, total;
} cdf_ctx;

static double gl_panel(int ch, double chi, double a, double b)
{
    double mid = 0.5 * (a + b), half = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < NGL; ++i) s += gl_w[i] * orc_density_nu(ch, chi, mid + half * gl_x[i]);
    return half * s;
}

/* Integration range in nu and the local decay rate |d u'/d nu| of the density's e^{-u'} factor.
   The range stops where u' exceeds its smallest value by 80 (the mass beyond is < e^-80 of
   the total); panel widths keep |d u'/d nu| * width <= 2 so every panel is smooth. */
static void nu_range(int ch, double chi, double *a, double *b)
{
    if (ch < 2) {
        /* u' = 2 e^nu / (3 chi) */
        *a = NLC_NU_LO;
        *b = log(1.5 * chi * 80.0);
    } else {
        /* u~' = 4 (1 + cosh nu) / (3 chi), smallest 8 / (3 chi) at nu = 0 */
        double c = 1.0 + 0.75 * chi * 80.0;
        double m = acosh(c);
        *a = -m; *b = m;
    }
}

static double decay_rate(int ch, double chi, double nu)
{
    if (ch < 2) return 2.0 * exp(nu) / (3.0 * chi);
    return 4.0 * fabs(sinh(nu)) / (3.0 * chi);
}

static void cdf_build(cdf_ctx *C, int ch, double chi)
{
    C->ch = ch; C->chi = chi;
    nu_range(ch, chi, &C->a0, &C->b_end);
    int cap = 64;
    C->edge_nu = (double *)malloc(sizeof(double) * cap);
    C->np = 0;
    double a = C->a0;
    C->edge_nu[0] = a;
    while (a < C->b_end) {
        double w = 1.0;
        while (w > 1.0 / 1024.0 && w * fmax(decay_rate(ch, chi, a), decay_rate(ch, chi, a + w)) > 2.0) w *= 0.5;
        double b = fmin(a + w, C->b_end);
        if (C->np + 2 > cap) { cap *= 2; C->edge_nu = (double *)realloc(C->edge_nu, sizeof(double) * cap); }
        C->edge_nu[++C->np] = b;
        a = b;
    }
    C->left = (double *)malloc(sizeof(double) * (C->np + 1));
    C->right = (double *)malloc(sizeof(double) * (C->np + 1));
    double *pint = (double *)malloc(sizeof(double) * C->np);
    for (int k = 0; k < C->np; ++k) pint[k] = gl_panel(ch, chi, C->edge_nu[k], C->edge_nu[k + 1]);
    C->tail = 0.0;
    if (ch < 2) { double l, o; lam_from_nu(C->a0, &l, &o); C->tail = nlc_tail(chi, l); }
    C->left[0] = C->tail;
    for (int k = 0; k < C->np; ++k) C->left[k + 1] = C->left[k] + pint[k];
    C->right[C->np] = 0.0;
    for (int k = C->np - 1; k >= 0; --k) C->right[k] = C->right[k + 1] + pint[k];
    C->total = C->tail + C->right[0];
    free(pint);
}

static void cdf_free(cdf_ctx *C) { free(C->edge_nu); free(C->left); free(C->right); }

static double edge(const cdf_ctx *C, int k) { return C->edge_nu[k]; }

/* panel containing nu (a0 <= nu < b_end) */
static int panel_of(const cdf_ctx *C, double nu)
{
    int lo = 0, hi = C->np;
    while (hi - lo > 1) { int m = (lo + hi) / 2; if (C->edge_nu[m] <= nu) lo = m; else hi = m; }
    return lo;
}

/* integral of the density over [a, b] inside one panel */
static double partial(const cdf_ctx *C, double a, double b)
{
    if (b <= a) return 0.0;
    return gl_panel(C->ch, C->chi, a, b);
}

double orc_rate_integral(int ch, double chi)
{
    cdf_ctx C;
    cdf_build(&C, ch, chi);
    double t = C.total;
    cdf_free(&C);
    return t;
}

double orc_cdf(int ch, double chi, double lam)
{
    cdf_ctx C;
    cdf_build(&C, ch, chi);
    double nu = log(lam) - log1p(-lam), r;
    if (nu <= C.a0) r = (ch < 2) ? nlc_tail(chi, lam) / C.total : 0.0;
    else if (nu >= C.b_end) r = 1.0;
    else {
        int k = panel_of(&C, nu);
        r = (C.left[k] + partial(&C, edge(&C, k), nu)) / C.total;
    }
    cdf_free(&C);
    return r;
}

double orc_ccdf(int ch, double chi, double lam)
{
    cdf_ctx C;
    cdf_build(&C, ch, chi);
    double nu = log(lam) - log1p(-lam), r;
    if (nu >= C.b_end) r = 0.0;
    else if (nu <= C.a0) r = 1.0 - ((ch < 2) ? nlc_tail(chi, lam) / C.total : 0.0);
    else {
        int k = panel_of(&C, nu);
        r = (C.right[k + 1] + partial(&C, nu, edge(&C, k + 1))) / C.total;
    }
    cdf_free(&C);
    return r;
}

/* Solve ln(cum(nu)) = ln(target) on [lo, hi] by safeguarded Newton (bisection fallback).
   side = +1: cum(nu) = base + int_lo^nu f;  side = -1: cum(nu) = base + int_nu^hi f. */
static double solve_panel(const cdf_ctx *C, int side, double base, double lo, double hi, double target)
{
    double a = lo, b = hi;
    double ca = (side > 0) ? base : base + partial(C, lo, hi);
    double cb = (side > 0) ? base + partial(C, lo, hi) : base;
    /* initial guess: linear in log cumulative */
    double la = log(fmax(ca, 1e-300)), lb = log(fmax(cb, 1e-300)), lt = log(target);
    double nu = (lb != la) ? a + (b - a) * (lt - la) / (lb - la) : 0.5 * (a + b);
    if (!(nu > a && nu < b)) nu = 0.5 * (a + b);
    for (int it = 0; it < 100; ++it) {
        double cum = (side > 0) ? base + partial(C, lo, nu) : base + partial(C, nu, hi);
        double g = log(cum) - lt;
        /* bracket update: cum increases with nu for side > 0, decreases for side < 0 */
        if ((side > 0) == (g > 0)) b = nu; else a = nu;
        double f = orc_density_nu(C->ch, C->chi, nu);
        double step = (f > 0.0) ? g * cum / (side > 0 ? f : -f) : 0.0;
        if (fabs(g) < 1e-15) {          /* converged to rounding: take the last Newton step */
            if (nu - step > a && nu - step < b) nu -= step;
            break;
        }
        double nn = nu - step;
        if (!(f > 0.0) || !(nn > a && nn < b)) nn = 0.5 * (a + b);
        double tol = 2e-16 * fmax(1.0, fabs(nu));
        if (fabs(nn - nu) <= tol || (b - a) <= tol) { nu = nn; break; }
        nu = nn;
    }
    return nu;
}

static double icdf_ctx(const cdf_ctx *C, double rho)
{
    if (rho <= 0.0) {
        double r = 1.0 / (1.0 + exp(-rho));
        double target = r * C->total;
        if (C->ch < 2 && target <= C->tail) {
            /* invert A y - B y^3 = target with y = lam^(1/3) */
            double A = 3.0 * tgamma(2.0 / 3.0) * pow(3.0 * C->chi, 2.0 / 3.0), Bc = ORC_PI / sqrt(3.0);
            double y = target / A;
            for (int it = 0; it < 4; ++it) y -= (A * y - Bc * y * y * y - target) / (A - 3.0 * Bc * y * y);
            double lam = y * y * y;
            return 3.0 * log(y) - log1p(-lam);
        }
        int lo = 0, hi = C->np;      /* find k with left[k] <= target < left[k+1] */
        while (hi - lo > 1) { int m = (lo + hi) / 2; if (C->left[m] <= target) lo = m; else hi = m; }
        return solve_panel(C, +1, C->left[lo], edge(C, lo), edge(C, lo + 1), target);
    } else {
        double q = 1.0 / (1.0 + exp(rho));
        double target = q * C->total;
        int lo = 0, hi = C->np;      /* find k with right[k+1] <= target < right[k] */
        while (hi - lo > 1) { int m = (lo + hi) / 2; if (C->right[m] > target) lo = m; else hi = m; }
        return solve_panel(C, -1, C->right[lo + 1], edge(C, lo), edge(C, lo + 1), target);
    }
}

double orc_icdf_nu(int ch, double chi, double rho)
{
    cdf_ctx C;
    cdf_build(&C, ch, chi);
    double nu = icdf_ctx(&C, rho);
    cdf_free(&C);
    return nu;
}

/* ====================================================================== */
/* Tables of the specified grid and their 4-point Lagrange interpolation.  */
/* ====================================================================== */
static int nchi_of(const orc_table_spec *s, int ch) { return s->n_chi[ch < 2 ? 0 : 1]; }

static void alloc_tables(orc_tables *T, const orc_table_spec *spec)
{
    T->spec = *spec;
    int64_t r = 0, v = 0;
    for (int c = 0; c < 4; ++c) {
        T->off_rate[c] = r; T->off_nu[c] = v;
        r += nchi_of(spec, c);
        v += (int64_t)nchi_of(spec, c) * spec->n_rho;
    }
    T->lnrate = (double *)calloc(r, sizeof(double));
    T->nu = (double *)calloc(v, sizeof(double));
    T->lngfac = (double *)calloc(ORC_GF_N, sizeof(double));
}

static void gfac_build(orc_tables *T, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
#endif
    for (int i = 0; i < ORC_GF_N; ++i) T->lngfac[i] = log(orc_gfactor_ratio(exp(ORC_GF_LNCHI0 + i * ORC_GF_DLNCHI)));
}

/* The pair rows hold ln W + 8/(3 chi): at small chi the pair rate falls as exp(-8/(3 chi)) (the
   Erber law), a curvature in ln chi that 4-point interpolation follows poorly (5e-5 in ln W on
   32 nodes per decade) while the difference is smooth (1e-8).  The lookup subtracts it again. */
static double rate_offset(int ch, double chi) { return ch >= 2 ? (8.0 / 3.0) / chi : 0.0; }

int orc_tables_build(orc_tables *T, const orc_table_spec *spec, int nthreads)
{
    alloc_tables(T, spec);
    int nchi0 = spec->n_chi[0], nchi1 = spec->n_chi[1];
    int ntask = 2 * nchi0 + 2 * nchi1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int task = 0; task < ntask; ++task) {
        int ch, i;
        if (task < 2 * nchi0) { ch = task / nchi0; i = task % nchi0; }
        else { int t2 = task - 2 * nchi0; ch = 2 + t2 / nchi1; i = t2 % nchi1; }
        int g = ch < 2 ? 0 : 1;
        double chi = exp(spec->lnchi0[g] + i * spec->dlnchi[g]);
        cdf_ctx C;
        cdf_build(&C, ch, chi);
        T->lnrate[T->off_rate[ch] + i] = log(C.total) + rate_offset(ch, chi);
        double *row = T->nu + T->off_nu[ch] + (int64_t)i * spec->n_rho;
        for (int j = 0; j < spec->n_rho; ++j) row[j] = icdf_ctx(&C, spec->rho0 + j * spec->drho);
        cdf_free(&C);
    }
    gfac_build(T, nthreads);
    return 0;
}

int orc_tables_load(orc_tables *T, const orc_table_spec *spec, const double *lnrate, const double *nu,
                    const double *lngfac)
{
    alloc_tables(T, spec);
    int64_t nr = T->off_rate[3] + nchi_of(spec, 3);
    int64_t nv = T->off_nu[3] + (int64_t)nchi_of(spec, 3) * spec->n_rho;
    memcpy(T->lnrate, lnrate, sizeof(double) * nr);
    memcpy(T->nu, nu, sizeof(double) * nv);
    if (lngfac) memcpy(T->lngfac, lngfac, sizeof(double) * ORC_GF_N);
    else gfac_build(T, 0);
    return 0;
}

void orc_tables_free(orc_tables *T)
{
    free(T->lnrate); free(T->nu); free(T->lngfac);
    T->lnrate = T->nu = T->lngfac = NULL;
}

/* 4-point Lagrange weights on nodes v0 + i h (i = 0..n-1), one-sided at the ends */
static void lagrange4(double v, double v0, double h, int n, int *i0, double L[4])
{
    double s = (v - v0) / h;
    if (s < 0.0) s = 0.0;
    if (s > n - 1) s = n - 1;
    int i = (int)floor(s) - 1;
    if (i < 0) i = 0;
    if (i > n - 4) i = n - 4;
    double t = s - i;
    L[0] = -(t - 1.0) * (t - 2.0) * (t - 3.0) / 6.0;
    L[1] = t * (t - 2.0) * (t - 3.0) / 2.0;
    L[2] = -t * (t - 1.0) * (t - 3.0) / 2.0;
    L[3] = t * (t - 1.0) * (t - 2.0) / 6.0;
    *i0 = i;
}

double orc_table_lnrate(const orc_tables *T, int ch, double lnchi)
{
    int g = ch < 2 ? 0 : 1, i0;
    double L[4];
    lagrange4(lnchi, T->spec.lnchi0[g], T->spec.dlnchi[g], T->spec.n_chi[g], &i0, L);
    const double *r = T->lnrate + T->off_rate[ch] + i0;
    return L[0] * r[0] + L[1] * r[1] + L[2] * r[2] + L[3] * r[3] - rate_offset(ch, exp(lnchi));
}

double orc_table_nu(const orc_tables *T, int ch, double lnchi, double rho)
{
    int g = ch < 2 ? 0 : 1, i0, j0;
    double Lc[4], Lr[4];
    lagrange4(lnchi, T->spec.lnchi0[g], T->spec.dlnchi[g], T->spec.n_chi[g], &i0, Lc);
    lagrange4(rho, T->spec.rho0, T->spec.drho, T->spec.n_rho, &j0, Lr);
    double acc = 0.0;
    for (int a = 0; a < 4; ++a) {
        const double *row = T->nu + T->off_nu[ch] + (int64_t)(i0 + a) * T->spec.n_rho + j0;
        acc += Lc[a] * (Lr[0] * row[0] + Lr[1] * row[1] + Lr[2] * row[2] + Lr[3] * row[3]);
    }
    return acc;
}

/* ====================================================================== */
/* Field-dependent anomalous magnetic moment (loop appendix).  The Scorer-  */
/* function term of the one-loop self-energy rotates the spin like an      */
/* anomalous moment a(chi) that falls from Schwinger's alpha/(2 pi) at     */
/* chi -> 0; written through the Airy-Scorer integral of the appendix,     */
/*   a(chi) = alpha int_0^inf du/(1+u)^3 z Gi(z),  z = (u/chi)^(2/3),     */
/* i.e. a(chi)/a(0) = 2 pi int_0^inf du/(1+u)^3 z Gi(z).                   */
/* ====================================================================== */
/* Gi(z) for z >= 0.  From Ai + i Gi = (1/pi) int_0^inf exp(i(z t + t^3/3)) dt, turned onto the ray
   t = exp(i pi/6) s (the arc at infinity vanishes in that sector):
     Gi(z) = (1/pi) int_0^inf exp(-s^3/3 - z s/2) sin((sqrt3/2) z s + pi/6) ds,
   by 20-point Gauss-Legendre panels of width at most 1/(1+z) up to where the exponent reaches -45.
   For z > 20 the large-argument expansion Gi = (1/(pi z)) sum_k (3k)!/(k! (3 z^3)^k), ten terms
   (remainder below 1e-18 relative there). */
double orc_scorer_gi(double z)
{
    if (z > 20.0) {
        double x = 1.0 / (3.0 * z * z * z), term = 1.0, sum = 1.0;
        for (int k = 1; k <= 10; ++k) {
            term *= (3.0 * k) * (3.0 * k - 1.0) * (3.0 * k - 2.0) / k * x;   /* (3k)!/k! x^k */
            sum += term;
        }
        return sum / (ORC_PI * z);
    }
    double send = 0.0;                      /* root of s^3/3 + z s/2 = 45 by bisection */
    {
        double lo = 0.0, hi = 10.0;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid * mid * mid / 3.0 + 0.5 * z * mid < 45.0) lo = mid; else hi = mid;
        }
        send = hi;
    }
    double wmax = 1.0 / (1.0 + z);
    int np = (int)ceil(send / wmax);
    double w = send / np, acc = 0.0;
    for (int k = 0; k < np; ++k) {
        double mid = (k + 0.5) * w, half = 0.5 * w, ps = 0.0;
        for (int i = 0; i < NGL; ++i) {
            double s = mid + half * gl_x[i];
            ps += gl_w[i] * exp(-s * s * s / 3.0 - 0.5 * z * s) * sin(0.5 * sqrt(3.0) * z * s + ORC_PI / 6.0);
        }
        acc += half * ps;
    }
    return acc / ORC_PI;
}

/* a(chi)/a(0) = 2 pi int dv e^v/(1+e^v)^3 z Gi(z), u = e^v, z = exp(2 (v - ln chi)/3), by the
   trapezoidal rule in v with step 0.2 on [min(ln chi, 0) - 40, 25].  The integrand is analytic in
   |Im v| < pi/2 and decays exponentially at both ends (as e^(5v/3) and e^(-2v)), so the rule's
   error is of order exp(-pi^2/0.2), far below rounding. */
double orc_gfactor_ratio(double chi)
{
    if (!(chi > 0.0)) return 1.0;
    double lc = log(chi), vlo = (lc < 0.0 ? lc : 0.0) - 40.0, vhi = 25.0, h = 0.2, acc = 0.0;
    int n = (int)ceil((vhi - vlo) / h);
    for (int k = 0; k <= n; ++k) {
        double v = vlo + k * h, u = exp(v), z = exp(2.0 * (v - lc) / 3.0);
        double f = u / ((1.0 + u) * (1.0 + u) * (1.0 + u)) * z * orc_scorer_gi(z);
        acc += (k == 0 || k == n) ? 0.5 * f : f;
    }
    return 2.0 * ORC_PI * h * acc;
}

/* Table: 4-point Lagrange in ln chi of ln(a/a(0)) on the nodes ORC_GF_LNCHI0 + i ORC_GF_DLNCHI.
   Below the first node (chi < 1e-7, where 1 - a/a(0) < 2e-12) the ratio is 1; beyond the last
   (chi > 1e4) it follows the large-chi law a ~ chi^(-2/3) from the last node. */
double orc_table_gfac(const orc_tables *T, double chi)
{
    if (!(chi > 0.0)) return 1.0;
    double lc = log(chi);
    if (lc < ORC_GF_LNCHI0) return 1.0;
    double lnlast = ORC_GF_LNCHI0 + (ORC_GF_N - 1) * ORC_GF_DLNCHI;
    if (lc > lnlast) return exp(T->lngfac[ORC_GF_N - 1] - (2.0 / 3.0) * (lc - lnlast));
    int i0;
    double L[4];
    lagrange4(lc, ORC_GF_LNCHI0, ORC_GF_DLNCHI, ORC_GF_N, &i0, L);
    const double *g = T->lngfac + i0;
    return exp(L[0] * g[0] + L[1] * g[1] + L[2] * g[2] + L[3] * g[3]);
}

/* ====================================================================== */
/* Fields                                                                  */
/* ====================================================================== */
void orc_fields_eval(const orc_fields *f, const double x[3], double t, double E[3], double B[3])
{
    for (int i = 0; i < 3; ++i) { E[i] = f->E0[i]; B[i] = f->B0[i]; }
    if (f->kind == ORC_FIELD_PLANE_LP) {
        /* linearly polarized plane wave travelling along -x: phase t + x, E along y, B = -x^ x E */
        double phi = t + x[0], g = 1.0;
        if (f->phase_len > 0.0) {
            if (phi < 0.0 || phi > f->phase_len) g = 0.0;
            else { double sn = sin(ORC_PI * phi / f->phase_len); g = sn * sn; }
        }
        double ey = f->a0 * g * cos(phi);
        E[1] += ey;
        B[2] += -ey;
    } else if (f->kind == ORC_FIELD_ROTATING_E) {
        /* uniform electric field of magnitude a0 rotating in the (x, y) plane at the laser
           frequency (polarized-cascade section: the 0-D rotating-field setup) */
        E[0] += f->a0 * cos(t);
        E[1] += f->a0 * sin(t);
    } else if (f->kind == ORC_FIELD_GRID2D) {
        /* bilinear interpolation between the four nodes around (x, y), periodic grid */
        double u = (x[0] - f->x0) / f->dx, v = (x[1] - f->y0) / f->dy;
        double iu = floor(u), iv = floor(v);
        double ax = u - iu, ay = v - iv;
        long i0 = ((long)fmod(iu, (double)f->nx) + f->nx) % f->nx, j0 = ((long)fmod(iv, (double)f->ny) + f->ny) % f->ny;
        long i1 = (i0 + 1) % f->nx, j1 = (j0 + 1) % f->ny;
        double w00 = (1 - ax) * (1 - ay), w10 = ax * (1 - ay), w01 = (1 - ax) * ay, w11 = ax * ay;
        for (int c = 0; c < 6; ++c) {
            const float *g = f->grid[c];
            double val = w00 * g[j0 * f->nx + i0] + w10 * g[j0 * f->nx + i1] + w01 * g[j1 * f->nx + i0]
                       + w11 * g[j1 * f->nx + i1];
            if (c < 3) E[c] += val; else B[c - 3] += val;
        }
    }
}

/* ====================================================================== */
/* Vector helpers                                                          */
/* ====================================================================== */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Inputs that are not finite (NaN or infinity) are not stepped: a lepton keeps its state, a
   photon is removed, and each is counted; a step in a non-finite field is cut short. */
static int finite3(const double v[3]) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }
static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Rest-frame basis of the method (reading R1) and the quantum parameter chi
   = eps_r sqrt((p0 E + p x B)^2 - (p.E)^2), p0 = gamma for leptons, |k| for photons. */
double orc_basis(int charge, double eps_r, const double E[3], const double B[3],
                 const double p[3], double e[3], double b[3], double k[3])
{
    double pn = sqrt(dot3(p, p));
    double p0 = (charge == 0) ? pn : sqrt(1.0 + pn * pn);
    double pxB[3], F[3];
    cross3(p, B, pxB);
    for (int i = 0; i < 3; ++i) F[i] = p0 * E[i] + pxB[i];
    double pE = dot3(p, E);
    double rad = dot3(F, F) - pE * pE;
    double chi = eps_r * sqrt(rad > 0.0 ? rad : 0.0);
    for (int i = 0; i < 3; ++i) k[i] = p[i] / pn;
    /* transverse force direction: (E + v x B) perpendicular to khat */
    double f[3], fk;
    for (int i = 0; i < 3; ++i) f[i] = F[i] / p0;
    fk = dot3(f, k);
    for (int i = 0; i < 3; ++i) f[i] -= fk * k[i];
    double fn = sqrt(dot3(f, f));
    double sgn = (charge > 0) ? -1.0 : 1.0;   /* -q with q = -1 for e- and photons */
    if (fn > 0.0) for (int i = 0; i < 3; ++i) e[i] = sgn * f[i] / fn;
    else { e[0] = e[1] = e[2] = 0.0; }
    cross3(k, e, b);
    return (fn > 0.0) ? chi : 0.0;
}

/* Stokes (xi1 diagonal, xi2 circular, xi3 linear along eps) -> P-vector (photon section) */
void orc_stokes_to_P(const double xi[3], const double e[3], const double b[3], const double k[3], double P[3])
{
    double d = sqrt(dot3(xi, xi));
    if (!(d > 0.0)) { P[0] = P[1] = P[2] = 0.0; return; }
    double x1 = xi[0] / d, x2 = xi[1] / d, x3 = xi[2] / d;
    double dth = 0.5 * atan2(x1, x3);
    double tr = sqrt(fmax(0.0, 1.0 - x2 * x2));
    double pe = tr * cos(dth), pb = tr * sin(dth), pk = x2;
    for (int i = 0; i < 3; ++i) P[i] = d * (pe * e[i] + pb * b[i] + pk * k[i]);
}

void orc_P_to_stokes(const double P[3], const double e[3], const double b[3], const double k[3], double xi[3])
{
    double d = sqrt(dot3(P, P));
    if (!(d > 0.0)) { xi[0] = xi[1] = xi[2] = 0.0; return; }
    double p1 = dot3(P, e) / d, p2 = dot3(P, b) / d, pk = dot3(P, k) / d;
    double rr = p1 * p1 + p2 * p2;
    if (rr > 0.0) {
        double r = sqrt(rr);
        xi[0] = d * 2.0 * p1 * p2 / r;
        xi[2] = d * (p1 * p1 - p2 * p2) / r;
    } else { xi[0] = xi[2] = 0.0; }
    xi[1] = d * pk;
}

/* ====================================================================== */
/* Lorentz push (Boris) and T-BMT spin rotation (reading R9)               */
/* ====================================================================== */
static void cayley(double v[3], const double t[3])
{
    double tt = dot3(t, t), s[3], vp[3], c[3];
    for (int i = 0; i < 3; ++i) s[i] = 2.0 * t[i] / (1.0 + tt);
    cross3(v, t, c);
    for (int i = 0; i < 3; ++i) vp[i] = v[i] + c[i];
    cross3(vp, s, c);
    for (int i = 0; i < 3; ++i) v[i] += c[i];
}

void orc_push_one(int q, double a_e, const double E[3], const double B[3], double dt,
                  uint32_t flags, const orc_tables *T, double eps_r, double p[3], double s[3], double x[3])
{
    double um[3], up[3], t[3];
    for (int i = 0; i < 3; ++i) um[i] = p[i] + 0.5 * q * dt * E[i];
    double gm = sqrt(1.0 + dot3(um, um));
    for (int i = 0; i < 3; ++i) t[i] = 0.5 * q * dt * B[i] / gm;
    for (int i = 0; i < 3; ++i) up[i] = um[i];
    cayley(up, t);
    if (flags & ORC_F_TBMT) {
        double be[3], bxE[3], Om[3], ts[3];
        for (int i = 0; i < 3; ++i) be[i] = 0.5 * (um[i] + up[i]) / gm;
        cross3(be, E, bxE);
        double bB = dot3(be, B);
        if (flags & ORC_F_GCHI) {
            /* chi at the mid step: momentum u = (u- + u+)/2, energy gamma- */
            double u[3], uxB[3], F[3];
            for (int i = 0; i < 3; ++i) u[i] = 0.5 * (um[i] + up[i]);
            cross3(u, B, uxB);
            for (int i = 0; i < 3; ++i) F[i] = gm * E[i] + uxB[i];
            double uE = dot3(u, E), rad = dot3(F, F) - uE * uE;
            a_e *= orc_table_gfac(T, eps_r * sqrt(rad > 0.0 ? rad : 0.0));
        }
        for (int i = 0; i < 3; ++i)
            Om[i] = -q * ((a_e + 1.0 / gm) * B[i] - (a_e * gm / (gm + 1.0)) * bB * be[i]
                          - (a_e + 1.0 / (gm + 1.0)) * bxE[i]);
        for (int i = 0; i < 3; ++i) ts[i] = -0.5 * Om[i] * dt;
        cayley(s, ts);
    }
    for (int i = 0; i < 3; ++i) p[i] = up[i] + 0.5 * q * dt * E[i];
    double g = sqrt(1.0 + dot3(p, p));
    for (int i = 0; i < 3; ++i) x[i] += p[i] / g * dt;
}

/* ====================================================================== */
/* The QED part of the lepton step (NLC section, flow chart of the NLC     */
/* algorithm; non-transition section for non-emitters)                     */
/* ====================================================================== */
static int near_tie(double r, double thr, double tol)
{
    return fabs(r - thr) <= tol * fabs(thr);
}

static uint64_t lepton_id(int species, int64_t index) { return ((uint64_t)species << 62) | (uint64_t)index; }

/* 2^63 | species << 61 | (sub-cycling round << 33 | parent index mod 2^33) << 24 | step mod 2^24 */
static uint64_t photon_id(int species, int64_t index, int64_t step, int round)
{
    return (1ull << 63) | ((uint64_t)species << 61) | ((uint64_t)(round & 15) << 57)
           | (((uint64_t)index & ((1ull << 33) - 1)) << 24) | ((uint64_t)step & 0xFFFFFFull);
}

/* no-transition spin update (non-transition section), renormalised if it leaves |s| > 1 (R6) */
static void no_emission_update(double s[3], const double bh[3], double Wbar, double dW, double dt, double P,
                               orc_counters *ctr)
{
    double den = 1.0 - P;
    for (int i = 0; i < 3; ++i) s[i] = (s[i] * (1.0 - Wbar * dt) - dW * dt * bh[i]) / den;
    double n2 = dot3(s, s);
    if (n2 > 1.0) {
        double n = sqrt(n2);
        for (int i = 0; i < 3; ++i) s[i] /= n;
        if (n2 > 1.0 + 1e-12) ctr->n_norm_clamped++;
    }
}

/* Conditioning of the collapse axes of the last orc_lepton_qed_one / orc_photon_qed_one call on
   this thread (diagnostics for the comparisons; the step never reads them): the norm of the vector
   of each component's sum of absolute terms -- the scale that rounding the terms works on -- over
   the norm of the vector the axis is taken from. */
static _Thread_local double g_cond_spin, g_cond_pol, g_cond_pe, g_cond_pp;

static double norm3(double x, double y, double z) { return sqrt(x * x + y * y + z * z); }

/* rounding scale of g (terms of nlc_g_pt in absolute value) */
static double nlc_g_scale(const spec_pt *q, const double si[3])
{
    double u = q->lam / q->oml, c = q->IK + 2.0 * q->K23;
    return norm3(c * fabs(si[0]), u * q->K13 + c * fabs(si[1]),
                 c * fabs(si[2]) + q->lam * u * (q->IK + q->K23) * fabs(si[2]));
}

/* rounding scale of F = (F1, F2, F3) (terms of nlc_F_pt in absolute value) */
static double nlc_F_scale(const spec_pt *q, const double a[3], const double b[3])
{
    double lam = q->lam, oml = q->oml, u = lam / oml;
    double kap = 1.0 / oml + oml, kapt = fabs(1.0 / oml - oml);
    double I = q->IK, K1 = q->K13, K2 = q->K23;
    double A[3] = {fabs(a[0]), fabs(a[1]), fabs(a[2])}, B[3] = {fabs(b[0]), fabs(b[1]), fabs(b[2])};
    double f1 = K1 * (u * A[0] + lam * B[0]) + 0.5 * lam * u * I * (B[0] * A[1] + B[1] * A[0])
                + 0.5 * kapt * K2 * (B[0] * A[1] + B[1] * A[0]);
    double f2 = 0.5 * kapt * K1 * (B[1] * A[2] + B[2] * A[1]) + (lam * I + kapt * K2) * A[2]
                + (u * I + kapt * K2) * B[2] + 0.5 * lam * u * K1 * (B[2] * A[1] + B[1] * A[2]);
    double f3 = K2 + (u * A[1] + lam * B[1]) * K1 + 0.5 * lam * u * I * (B[0] * A[0] + B[1] * A[1])
                + 0.5 * kap * K2 * (B[0] * A[0] + B[1] * A[1] + B[2] * A[2]) + 0.5 * lam * u * K2 * B[2] * A[2];
    return norm3(f1, f2, f3);
}

/* rounding scales of j_e and j_p (terms of nbw_j_pt in absolute value) */
static void nbw_j_scale(const spec_pt *q, const double xi[3], double *se, double *sp)
{
    double lam = q->lam, oml = q->oml;
    double rhot = fabs(oml / lam - lam / oml);
    double I = q->IK, K1 = q->K13, K2 = q->K23;
    *se = norm3(fabs(xi[0]) * K1 / lam, (1.0 / oml + fabs(xi[2]) / lam) * K1, fabs(xi[1]) * (I / oml + rhot * K2));
    *sp = norm3(fabs(xi[0]) * K1 / oml, (1.0 / lam + fabs(xi[2]) / oml) * K1, fabs(xi[1]) * (I / lam + rhot * K2));
}

/* returns 1 if a photon was emitted (k_out, P_out, id_out valid), 0 otherwise;
   bit 1 of the return value flags a near tie of one of the decisions.  tau2 = {tau, tau*}
   of the lepton, updated in place, with ORC_F_TAU (may be NULL otherwise). */
int orc_lepton_qed_one(const orc_tables *T, const orc_params *prm, int species, int64_t index,
                       const double E[3], const double B[3], const double x[3],
                       double p[3], double s[3], double k_out[3], double P_out[3],
                       uint64_t *id_out, double tau2[2], orc_counters *ctr)
{
    (void)x;
    uint32_t fl = prm->flags;
    int near = 0;
    if (!(fl & ORC_F_EMIT)) return 0;
    int q = species == 0 ? -1 : 1;
    double eh[3], bh[3], kh[3];
    double chi = orc_basis(q, prm->eps_r, E, B, p, eh, bh, kh);
    if (!(chi >= prm->chi_e_min)) return 0;
    if (chi > prm->chi_e_max) { chi = prm->chi_e_max; ctr->n_chi_clamped++; }
    double gamma = sqrt(1.0 + dot3(p, p));
    double Ce = ORC_ALPHA / (sqrt(3.0) * ORC_PI * prm->eps_r * gamma);
    double lnchi = log(chi);
    double Wdn = Ce * exp(orc_table_lnrate(T, 0, lnchi));
    double Wup = Ce * exp(orc_table_lnrate(T, 1, lnchi));
    double sb = dot3(s, bh);
    double dt = prm->dt;
    double a = Wdn * 0.5 * (1.0 - sb) * dt;
    double b = Wup * 0.5 * (1.0 + sb) * dt;
    double P = a + b;
    uint64_t id = lepton_id(species, index);
    double r1, r2;
    uniforms2(prm, id, 0, &r1, &r2);
    double Wbar = 0.5 * (Wup + Wdn), dW = 0.5 * (Wup - Wdn);
    double thr;
    double lam, oml;
    if (fl & ORC_F_REJECT) {
        /* rejection sampling (spectrum-sampling section): the candidate lambda = r1^3 is accepted
           with probability 3 r1^2 dW/dlambda dt, dW/dlambda = Ce w(lambda, s_beta) the spectrum of
           the initial spin state summed over the final states; integrated over r1 this is W_s dt */
        lam = r1 * r1 * r1;
        oml = (1.0 - r1) * (1.0 + r1 + r1 * r1);
        spec_pt q0 = nlc_point(chi, lam, oml);
        double A = 3.0 * r1 * r1 * Ce * nlc_w_pt(&q0, sb) * dt;
        if (A > 1.0) ctr->n_prob_clamped++;
        if (near_tie(r2, A, prm->near_tol)) near = 1;
        if (!(r2 < A)) {
            if (fl & ORC_F_NOEMIT) {
                if (P < 1.0) no_emission_update(s, bh, Wbar, dW, dt, P, ctr);
                else ctr->n_prob_clamped++;
            }
            return near << 1;
        }
        goto emission;
    }
    if ((fl & ORC_F_TAU) && tau2) {
        /* optical depth (R10) */
        uint32_t w4[4];
        philox_block(prm->seed, id, prm->step, 4u, w4);
        double target = tau2[1];
        if (!(target > 0.0)) target = -log1p(-orc_u01_53(w4[0], w4[1]));
        double tn = tau2[0] + P;
        if (near_tie(tn, target, prm->near_tol)) near = 1;
        if (!(tn >= target)) {
            tau2[0] = tn;
            tau2[1] = target;
            if (fl & ORC_F_NOEMIT) {
                if (P < 1.0) no_emission_update(s, bh, Wbar, dW, dt, P, ctr);
                else ctr->n_prob_clamped++;
            }
            return near << 1;
        }
        tau2[0] = 0.0;
        tau2[1] = -log1p(-orc_u01_53(w4[2], w4[3]));
        thr = a / P;
    } else {
        /* per-step draw */
        if (P <= 1.0 && near_tie(r1, P, prm->near_tol)) near = 1;
        if (P <= 1.0 && !(r1 < P)) {
            if (fl & ORC_F_NOEMIT) no_emission_update(s, bh, Wbar, dW, dt, P, ctr);
            return near << 1;
        }
        if (P > 1.0) ctr->n_prob_clamped++;
        /* branch: down table iff r1 < a (or r1 < a/P when the probability is clamped) */
        thr = (P <= 1.0) ? a : a / P;
    }
    if (near_tie(r1, thr, prm->near_tol)) near = 1;
    int up = !(r1 < thr);
    double rho = log(r2) - log1p(-r2);
    double nu = orc_table_nu(T, up ? 1 : 0, lnchi, rho);
    lam_from_nu(nu, &lam, &oml);
emission:
    for (int i = 0; i < 3; ++i) k_out[i] = lam * p[i];
    double r3, r4;
    uniforms2(prm, id, 1, &r3, &r4);
    /* spin and Stokes components in the emission basis */
    double si[3] = {dot3(s, eh), sb, dot3(s, kh)};
    spec_pt qp = nlc_point(chi, lam, oml);
    double w = nlc_w_pt(&qp, si[1]);
    double g[3];
    nlc_g_pt(&qp, si, g);
    double sf[3] = {si[0], si[1], si[2]};
    g_cond_spin = 1.0;
    g_cond_pol = 1.0;
    if (fl & ORC_F_SPIN) {
        if (fl & ORC_F_MEAN) { for (int i = 0; i < 3; ++i) sf[i] = g[i] / w; }
        else {
            double gn = sqrt(dot3(g, g));
            g_cond_spin = gn > 0.0 ? nlc_g_scale(&qp, si) / gn : HUGE_VAL;
            double S[3];
            if (gn > 0.0) for (int i = 0; i < 3; ++i) S[i] = g[i] / gn;
            else { S[0] = 0.0; S[1] = 1.0; S[2] = 0.0; }
            double thr3 = (w - gn) / (2.0 * w);
            if (near_tie(r3, thr3, prm->near_tol)) near = 1;
            double sg = (r3 < thr3) ? -1.0 : 1.0;
            for (int i = 0; i < 3; ++i) sf[i] = sg * S[i];
        }
    }
    double xi[3] = {0.0, 0.0, 0.0};
    if (fl & ORC_F_PHOTON_POL) {
        double F[4];
        if (fl & ORC_F_MEAN) {
            double z[3] = {0.0, 0.0, 0.0};
            nlc_F_pt(&qp, si, z, F);
            for (int i = 0; i < 3; ++i) xi[i] = F[i + 1] / w;
        } else {
            nlc_F_pt(&qp, si, sf, F);
            double Fn = sqrt(F[1] * F[1] + F[2] * F[2] + F[3] * F[3]);
            if (Fn > 0.0) {
                g_cond_pol = nlc_F_scale(&qp, si, sf) * (1.0 + g_cond_spin) / Fn;
                double thr4 = (F[0] - Fn) / (2.0 * F[0]);
                if (near_tie(r4, thr4, prm->near_tol)) near = 1;
                double sg = (r4 < thr4) ? -1.0 : 1.0;
                for (int i = 0; i < 3; ++i) xi[i] = sg * F[i + 1] / Fn;
            }
        }
    }
    orc_stokes_to_P(xi, eh, bh, kh, P_out);
    if (fl & ORC_F_RECOIL) for (int i = 0; i < 3; ++i) p[i] *= oml;
    if (fl & ORC_F_SPIN) for (int i = 0; i < 3; ++i) s[i] = sf[0] * eh[i] + sf[1] * bh[i] + sf[2] * kh[i];
    *id_out = photon_id(species, index, prm->step, prm->sub_round);
    ctr->n_emit++;
    return 1 | (near << 1);
}

/* ====================================================================== */
/* The photon step (NBW section, flow chart of the NBW algorithm).         */
/* Returns 1 on pair creation (pe, se, pp, sp valid), 0 otherwise; P is    */
/* updated in place on survival; bit 1 flags a near tie.                   */
/* ====================================================================== */
int orc_photon_qed_one(const orc_tables *T, const orc_params *prm, uint64_t id,
                       const double E[3], const double B[3], const double k[3], double P[3],
                       double pe[3], double se[3], double pp[3], double sp[3], orc_counters *ctr)
{
    uint32_t fl = prm->flags;
    int near = 0;
    if (!(fl & ORC_F_PAIR)) return 0;
    double eh[3], bh[3], kh[3];
    double chi = orc_basis(0, prm->eps_r, E, B, k, eh, bh, kh);
    if (!(chi >= prm->chi_g_min)) return 0;
    if (chi > prm->chi_g_max) { chi = prm->chi_g_max; ctr->n_chi_clamped++; }
    double k0 = sqrt(dot3(k, k));
    double Cg = ORC_ALPHA / (sqrt(3.0) * ORC_PI * prm->eps_r * k0);
    double lnchi = log(chi);
    double Wm = Cg * exp(orc_table_lnrate(T, 2, lnchi));
    double Wp = Cg * exp(orc_table_lnrate(T, 3, lnchi));
    double xi[3] = {0.0, 0.0, 0.0};
    if (finite3(P)) orc_P_to_stokes(P, eh, bh, kh, xi);
    else ctr->n_nonfinite++;                   /* a non-finite P-vector is stepped as unpolarized */
    double dt = prm->dt;
    double a = Wm * 0.5 * (1.0 - xi[2]) * dt;
    double b = Wp * 0.5 * (1.0 + xi[2]) * dt;
    double Pr = a + b;
    double r1, r2;
    uniforms2(prm, id, 2, &r1, &r2);
    if (Pr <= 1.0 && near_tie(r1, Pr, prm->near_tol)) near = 1;
    if (Pr <= 1.0 && !(r1 < Pr)) {
        if (fl & ORC_F_NOPAIR) {
            double Wbar = 0.5 * (Wp + Wm), dW = 0.5 * (Wp - Wm);
            double den = 1.0 - Pr;
            double xn[3] = {xi[0] * (1.0 - Wbar * dt) / den, xi[1] * (1.0 - Wbar * dt) / den,
                            (xi[2] * (1.0 - Wbar * dt) - dW * dt) / den};
            double n2 = dot3(xn, xn);
            if (n2 > 1.0) {
                double n = sqrt(n2);
                for (int i = 0; i < 3; ++i) xn[i] /= n;
                if (n2 > 1.0 + 1e-12) ctr->n_norm_clamped++;
            }
            orc_stokes_to_P(xn, eh, bh, kh, P);
        }
        return near << 1;
    }
    if (Pr > 1.0) ctr->n_prob_clamped++;
    double thr = (Pr <= 1.0) ? a : a / Pr;
    if (near_tie(r1, thr, prm->near_tol)) near = 1;
    int plus = !(r1 < thr);
    double rho = log(r2) - log1p(-r2);
    double nu = orc_table_nu(T, plus ? 3 : 2, lnchi, rho);
    double lam, oml;
    lam_from_nu(nu, &lam, &oml);
    for (int i = 0; i < 3; ++i) { pp[i] = lam * k[i]; pe[i] = oml * k[i]; }
    double e_c[3] = {0.0, 0.0, 0.0}, p_c[3] = {0.0, 0.0, 0.0};
    g_cond_pe = 1.0;
    g_cond_pp = 1.0;
    if (fl & ORC_F_PAIR_SPIN) {
        spec_pt qp = nbw_point(chi, lam, oml);
        double w0, je[3], jp[3];
        nbw_j_pt(&qp, xi, &w0, je, jp);
        if (fl & ORC_F_MEAN) {
            for (int i = 0; i < 3; ++i) { e_c[i] = je[i] / w0; p_c[i] = jp[i] / w0; }
        } else {
            double r3, r3b;
            uniforms2(prm, id, 3, &r3, &r3b);
            double Se[3], Sp[3];
            double jen = sqrt(dot3(je, je)), jpn = sqrt(dot3(jp, jp));
            double sce, scp;
            nbw_j_scale(&qp, xi, &sce, &scp);
            g_cond_pe = jen > 0.0 ? sce / jen : HUGE_VAL;
            g_cond_pp = jpn > 0.0 ? scp / jpn : HUGE_VAL;
            for (int i = 0; i < 3; ++i) {
                Se[i] = jen > 0.0 ? je[i] / jen : (i == 1 ? 1.0 : 0.0);
                Sp[i] = jpn > 0.0 ? jp[i] / jpn : (i == 1 ? 1.0 : 0.0);
            }
            /* outcomes (positron, electron) = (dn,dn), (dn,up), (up,dn), (up,up) */
            static const double sgp[4] = {-1.0, -1.0, 1.0, 1.0}, sge[4] = {-1.0, 1.0, -1.0, 1.0};
            double cum = 0.0;
            int pick = 3;
            for (int o = 0; o < 4; ++o) {
                double ev[3], pv[3], G[4];
                for (int i = 0; i < 3; ++i) { ev[i] = sge[o] * Se[i]; pv[i] = sgp[o] * Sp[i]; }
                nbw_G_pt(&qp, ev, pv, G);
                cum += (G[0] + xi[0] * G[1] + xi[1] * G[2] + xi[2] * G[3]) / (4.0 * w0);
                if (o < 3) {
                    if (near_tie(r3, cum, prm->near_tol)) near = 1;
                    if (r3 < cum) { pick = o; break; }
                }
            }
            for (int i = 0; i < 3; ++i) { e_c[i] = sge[pick] * Se[i]; p_c[i] = sgp[pick] * Sp[i]; }
        }
    }
    for (int i = 0; i < 3; ++i) {
        se[i] = e_c[0] * eh[i] + e_c[1] * bh[i] + e_c[2] * kh[i];
        sp[i] = p_c[0] * eh[i] + p_c[1] * bh[i] + p_c[2] * kh[i];
    }
    ctr->n_pair++;
    return 1 | (near << 1);
}

/* ====================================================================== */
/* Array-level steps: per-particle work in parallel, appends in index order */
/* ====================================================================== */
static double getx(double *const x[3], int i, int64_t j) { return x[i] ? x[i][j] : 0.0; }

static void add_counters(orc_counters *d, const orc_counters *s)
{
    d->n_emit += s->n_emit; d->n_pair += s->n_pair; d->n_prob_clamped += s->n_prob_clamped;
    d->n_chi_clamped += s->n_chi_clamped; d->n_norm_clamped += s->n_norm_clamped;
    d->n_capacity_overflow += s->n_capacity_overflow; d->n_retired += s->n_retired;
    d->n_near_threshold += s->n_near_threshold;
    d->n_lepton_steps += s->n_lepton_steps; d->n_photon_steps += s->n_photon_steps;
    d->n_nonfinite += s->n_nonfinite;
}

/* append the photons of one pass over the leptons in lepton index order */
static void append_photons(const orc_params *prm, const orc_leptons *L, orc_photons *G, int64_t n,
                           const char *emitted, const double *kb, const uint64_t *ib, const double *cb,
                           orc_counters *tot)
{
    for (int64_t j = 0; j < n; ++j) {
        if (!emitted[j]) continue;
        if (G->n >= G->cap) { tot->n_capacity_overflow++; continue; }
        int64_t m = G->n++;
        const double *kk = kb + 6 * j, *PP = kb + 6 * j + 3;
        double k0 = sqrt(kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2]);
        if (k0 < prm->k_retire) {
            G->id[m] = 0;
            for (int i = 0; i < 3; ++i) { if (G->x[i]) G->x[i][m] = 0.0; G->k[i][m] = 0.0; G->P[i][m] = 0.0; }
            if (G->cond) G->cond[m] = 0.0;
            tot->n_retired++;
            continue;
        }
        G->id[m] = ib[j];
        if (G->cond) G->cond[m] = cb[j];
        for (int i = 0; i < 3; ++i) {
            if (G->x[i]) G->x[i][m] = getx(L->x, i, j);
            G->k[i][m] = kk[i];
            G->P[i][m] = PP[i];
        }
        if (G->near) G->near[m] = 0;
    }
}

/* The spin-weighted emission probability W_s dt of the decision (NLC section) at the lepton's
   current state, 0 where the step does no QED; sets *near when it lies within near_tol of a
   sub-cycling boundary ORC_SUB_WDT 2^k. */
static double lepton_wdt(const orc_tables *T, const orc_params *prm, int species, const double E[3],
                         const double B[3], const double p[3], const double s[3], int *near)
{
    double eh[3], bh[3], kh[3];
    double chi = orc_basis(species == 0 ? -1 : 1, prm->eps_r, E, B, p, eh, bh, kh);
    if (!(chi >= prm->chi_e_min)) return 0.0;
    if (chi > prm->chi_e_max) chi = prm->chi_e_max;
    double gamma = sqrt(1.0 + dot3(p, p));
    double Ce = ORC_ALPHA / (sqrt(3.0) * ORC_PI * prm->eps_r * gamma);
    double lnchi = log(chi);
    double sb = dot3(s, bh);
    double a = Ce * exp(orc_table_lnrate(T, 0, lnchi)) * 0.5 * (1.0 - sb) * prm->dt;
    double b = Ce * exp(orc_table_lnrate(T, 1, lnchi)) * 0.5 * (1.0 + sb) * prm->dt;
    double P = a + b;
    for (int m = 1; m < ORC_SUB_ROUNDS; m *= 2)
        if (near_tie(P, ORC_SUB_WDT * m, prm->near_tol)) *near = 1;
    return P;
}

/* Per-particle sub-cycling of the lepton step where the per-step draw would need W dt << 1
   (decision-making section).  After the push, each lepton takes m sub-steps of dt/m, m the
   smallest power of two with W_s dt / m <= ORC_SUB_WDT, at most ORC_SUB_ROUNDS, W_s dt taken at
   the state after the push.  The sub-steps run in ORC_SUB_ROUNDS rounds over the whole set: in
   round r a lepton with m sub-steps takes one (the whole QED part with the fields at t + dt:
   decision with its current chi and spin, emission with recoil and collapses, or the
   no-transition update over dt/m) when r is a multiple of ORC_SUB_ROUNDS/m.  Each round's
   photons are appended in lepton index order after the previous round's. */
static int lepton_step_subcycled(const orc_tables *T, const orc_params *prm, const orc_fields *f,
                                 orc_leptons *L, orc_photons *G, orc_counters *ctr, int nthreads)
{
    int64_t n = L->n;
    int q = L->species == 0 ? -1 : 1;
    int *msub = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    char *near = (char *)calloc(n > 0 ? n : 1, 1);
    char *emitted = (char *)calloc(n > 0 ? n : 1, 1);
    double *kb = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    uint64_t *ib = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    double *cb = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    orc_counters tot = {0};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    /* the push, and the number of sub-steps */
#pragma omp parallel
    {
        orc_counters loc = {0};
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            loc.n_lepton_steps++;
            double x[3] = {getx(L->x, 0, j), getx(L->x, 1, j), getx(L->x, 2, j)};
            double p[3] = {L->p[0][j], L->p[1][j], L->p[2][j]};
            double s[3] = {L->s[0][j], L->s[1][j], L->s[2][j]};
            double E[3], B[3];
            msub[j] = 0;                                  /* 0: no sub-step in any round */
            if (!(finite3(x) && finite3(p) && finite3(s))) { loc.n_nonfinite++; continue; }
            if (prm->flags & ORC_F_PUSH) {
                orc_fields_eval(f, x, prm->t, E, B);
                if (!(finite3(E) && finite3(B))) { loc.n_nonfinite++; continue; }
                orc_push_one(q, prm->a_e, E, B, prm->dt, prm->flags, T, prm->eps_r, p, s, x);
            }
            int m = 1;
            if (prm->flags & ORC_F_EMIT) {
                orc_fields_eval(f, x, prm->t + prm->dt, E, B);
                if (!(finite3(E) && finite3(B))) {
                    loc.n_nonfinite++;
                    m = 0;
                    goto store;
                }
                int nr = 0;
                double P = lepton_wdt(T, prm, L->species, E, B, p, s, &nr);
                while (m < ORC_SUB_ROUNDS && P > ORC_SUB_WDT * m) m *= 2;
                near[j] = (char)nr;
            }
        store:
            msub[j] = m;
            for (int i = 0; i < 3; ++i) {
                if (L->x[i]) L->x[i][j] = x[i];
                L->p[i][j] = p[i];
                L->s[i][j] = s[i];
            }
        }
#pragma omp critical
        add_counters(&tot, &loc);
    }
    /* the rounds */
    for (int r = 0; r < ORC_SUB_ROUNDS && (prm->flags & ORC_F_EMIT); ++r) {
#pragma omp parallel
        {
            orc_counters loc = {0};
#pragma omp for schedule(static)
            for (int64_t j = 0; j < n; ++j) {
                emitted[j] = 0;
                if (msub[j] == 0 || r % (ORC_SUB_ROUNDS / msub[j]) != 0) continue;
                orc_params sub = *prm;
                sub.dt = prm->dt / msub[j];
                sub.sub_round = r;
                double x[3] = {getx(L->x, 0, j), getx(L->x, 1, j), getx(L->x, 2, j)};
                double p[3] = {L->p[0][j], L->p[1][j], L->p[2][j]};
                double s[3] = {L->s[0][j], L->s[1][j], L->s[2][j]};
                double E[3], B[3];
                orc_fields_eval(f, x, prm->t + prm->dt, E, B);
                int64_t idx = L->index ? L->index[j] : j;
                int res = orc_lepton_qed_one(T, &sub, L->species, idx, E, B, x, p, s, kb + 6 * j, kb + 6 * j + 3,
                                             ib + j, NULL, &loc);
                emitted[j] = (char)(res & 1);
                if (res & 1) {
                    cb[j] = g_cond_pol;
                    if (L->cond && g_cond_spin > L->cond[j]) L->cond[j] = g_cond_spin;
                }
                if (res & 2) near[j] = 1;
                for (int i = 0; i < 3; ++i) {
                    L->p[i][j] = p[i];
                    L->s[i][j] = s[i];
                }
            }
#pragma omp critical
            add_counters(&tot, &loc);
        }
        append_photons(prm, L, G, n, emitted, kb, ib, cb, &tot);
    }
    for (int64_t j = 0; j < n; ++j) {
        if (near[j]) tot.n_near_threshold++;
        if (L->near) L->near[j] = (uint8_t)near[j];
    }
    add_counters(ctr, &tot);
    free(msub); free(near); free(emitted); free(kb); free(ib); free(cb);
    return 0;
}

int orc_lepton_step(const orc_tables *T, const orc_params *prm, const orc_fields *f,
                    orc_leptons *L, orc_photons *G, orc_counters *ctr, int nthreads)
{
    if (prm->flags & ORC_F_SUB) return lepton_step_subcycled(T, prm, f, L, G, ctr, nthreads);
    int64_t n = L->n;
    int q = L->species == 0 ? -1 : 1;
    char *emitted = (char *)calloc(n > 0 ? n : 1, 1);
    double *kb = (double *)malloc(sizeof(double) * 6 * (n > 0 ? n : 1));
    uint64_t *ib = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    double *cb = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    orc_counters tot = {0};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        orc_counters loc = {0};
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            loc.n_lepton_steps++;
            double x[3] = {getx(L->x, 0, j), getx(L->x, 1, j), getx(L->x, 2, j)};
            double p[3] = {L->p[0][j], L->p[1][j], L->p[2][j]};
            double s[3] = {L->s[0][j], L->s[1][j], L->s[2][j]};
            double E[3], B[3];
            if (L->near) L->near[j] = 0;
            if (!(finite3(x) && finite3(p) && finite3(s))) { loc.n_nonfinite++; continue; }
            if (prm->flags & ORC_F_PUSH) {
                orc_fields_eval(f, x, prm->t, E, B);
                if (!(finite3(E) && finite3(B))) { loc.n_nonfinite++; continue; }
                orc_push_one(q, prm->a_e, E, B, prm->dt, prm->flags, T, prm->eps_r, p, s, x);
            }
            if (prm->flags & ORC_F_EMIT) {
                orc_fields_eval(f, x, prm->t + prm->dt, E, B);
                if (!(finite3(E) && finite3(B))) {
                    loc.n_nonfinite++;
                    for (int i = 0; i < 3; ++i) {
                        if (L->x[i]) L->x[i][j] = x[i];
                        L->p[i][j] = p[i];
                        L->s[i][j] = s[i];
                    }
                    continue;
                }
            } else {
                orc_fields_eval(f, x, prm->t + prm->dt, E, B);
            }
            int64_t idx = L->index ? L->index[j] : j;
            double tau2[2] = {L->tau ? L->tau[j] : 0.0, L->tau_target ? L->tau_target[j] : 0.0};
            int mode_b = (prm->flags & ORC_F_TAU) && L->tau && L->tau_target;
            int r = orc_lepton_qed_one(T, prm, L->species, idx, E, B, x, p, s, kb + 6 * j, kb + 6 * j + 3,
                                       ib + j, mode_b ? tau2 : NULL, &loc);
            if (mode_b) { L->tau[j] = tau2[0]; L->tau_target[j] = tau2[1]; }
            emitted[j] = (char)(r & 1);
            if (r & 1) {
                cb[j] = g_cond_pol;
                if (L->cond && g_cond_spin > L->cond[j]) L->cond[j] = g_cond_spin;
            }
            if (r & 2) loc.n_near_threshold++;
            if (L->near) L->near[j] = (uint8_t)((r >> 1) & 1);
            for (int i = 0; i < 3; ++i) {
                if (L->x[i]) L->x[i][j] = x[i];
                L->p[i][j] = p[i];
                L->s[i][j] = s[i];
            }
        }
#pragma omp critical
        add_counters(&tot, &loc);
    }
    append_photons(prm, L, G, n, emitted, kb, ib, cb, &tot);
    add_counters(ctr, &tot);
    free(emitted); free(kb); free(ib); free(cb);
    return 0;
}

int orc_photon_step(const orc_tables *T, const orc_params *prm, const orc_fields *f,
                    orc_photons *G, orc_leptons *Le, orc_leptons *Lp, orc_counters *ctr, int nthreads)
{
    int64_t n = G->n_prev;
    char *pair = (char *)calloc(n > 0 ? n : 1, 1);
    double *ob = (double *)malloc(sizeof(double) * 14 * (n > 0 ? n : 1));
    orc_counters tot = {0};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        orc_counters loc = {0};
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            if (G->id[j] == 0) continue;
            double k[3] = {G->k[0][j], G->k[1][j], G->k[2][j]};
            double k0 = sqrt(dot3(k, k));
            double x0[3] = {getx(G->x, 0, j), getx(G->x, 1, j), getx(G->x, 2, j)};
            if (!(finite3(k) && finite3(x0) && (k[0] != 0.0 || k[1] != 0.0 || k[2] != 0.0))) {
                G->id[j] = 0;
                loc.n_nonfinite++;
                continue;
            }
            double x[3];
            for (int i = 0; i < 3; ++i) {
                x[i] = getx(G->x, i, j) + k[i] / k0 * prm->dt;
                if (G->x[i]) G->x[i][j] = x[i];
            }
            loc.n_photon_steps++;
            int behind = f->kind == ORC_FIELD_PLANE_LP && f->phase_len > 0.0 &&
                         prm->t + prm->dt + x[0] > f->phase_len;
            if (k0 < prm->k_retire || behind) { G->id[j] = 0; loc.n_retired++; continue; }
            double E[3], B[3];
            orc_fields_eval(f, x, prm->t + prm->dt, E, B);
            if ((prm->flags & ORC_F_PAIR) && !(finite3(E) && finite3(B))) { loc.n_nonfinite++; continue; }
            double P[3] = {G->P[0][j], G->P[1][j], G->P[2][j]};
            double *o = ob + 14 * j;
            int r = orc_photon_qed_one(T, prm, G->id[j], E, B, k, P, o, o + 3, o + 6, o + 9, &loc);
            if (r & 1) { o[12] = g_cond_pe; o[13] = g_cond_pp; }
            if (r & 2) loc.n_near_threshold++;
            if (G->near) G->near[j] = (uint8_t)((r >> 1) & 1);
            if (r & 1) { pair[j] = 1; G->id[j] = 0; }
            else for (int i = 0; i < 3; ++i) G->P[i][j] = P[i];
        }
#pragma omp critical
        add_counters(&tot, &loc);
    }
    for (int64_t j = 0; j < n; ++j) {
        if (!pair[j]) continue;
        const double *o = ob + 14 * j;
        if (Le->n >= Le->cap || Lp->n >= Lp->cap) { tot.n_capacity_overflow++; continue; }
        int64_t me = Le->n++, mp = Lp->n++;
        if (Le->cond) Le->cond[me] = o[12];
        if (Lp->cond) Lp->cond[mp] = o[13];
        if (Le->index) Le->index[me] = me;
        if (Lp->index) Lp->index[mp] = mp;
        /* new leptons start with no optical depth and no target (drawn at their first step) */
        if (Le->tau) Le->tau[me] = 0.0;
        if (Le->tau_target) Le->tau_target[me] = 0.0;
        if (Lp->tau) Lp->tau[mp] = 0.0;
        if (Lp->tau_target) Lp->tau_target[mp] = 0.0;
        for (int i = 0; i < 3; ++i) {
            double xv = getx(G->x, i, j);
            if (Le->x[i]) Le->x[i][me] = xv;
            if (Lp->x[i]) Lp->x[i][mp] = xv;
            Le->p[i][me] = o[i]; Le->s[i][me] = o[3 + i];
            Lp->p[i][mp] = o[6 + i]; Lp->s[i][mp] = o[9 + i];
        }
    }
    G->n_prev = G->n;
    add_counters(ctr, &tot);
    free(pair); free(ob);
    return 0;
}

void orc_compact(orc_photons *G)
{
    int64_t m = 0;
    for (int64_t j = 0; j < G->n; ++j) {
        if (G->id[j] == 0) continue;
        if (m != j) {
            G->id[m] = G->id[j];
            if (G->cond) G->cond[m] = G->cond[j];
            for (int i = 0; i < 3; ++i) {
                if (G->x[i]) G->x[i][m] = G->x[i][j];
                G->k[i][m] = G->k[i][j];
                G->P[i][m] = G->P[i][j];
            }
        }
        ++m;
    }
    G->n = m;
    G->n_prev = m;
}
