/*
 * qed_oracle.h -- plain FP64 CPU oracle of the spin- and polarization-resolved
 * strong-field QED particle step (nonlinear Compton emission for e-/e+ and
 * nonlinear Breit-Wheeler pair production for photons) of Qian, Seipt, Vranic,
 * Grismayer, Ridgers and Thomas, "A Fully Spin and Polarization Resolved Strong
 * Field QED Algorithm for Particle-in-Cell Codes" (arXiv 2511.08929).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or constant generator with the HIP library.
 *
 * Units: time in 1/omega_r, length in c/omega_r, momenta in m c, fields in
 * m c omega_r / e, eps_r = hbar omega_r / (m c^2).  Spin and photon polarization
 * vectors are lab-frame 3-vectors.  All arithmetic is IEEE double.
 */
#ifndef QED_ORACLE_H
#define QED_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- counter-based random numbers (Philox4x32-10) ---------------- */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01_53(uint32_t hi, uint32_t lo);   /* (m + 1/2) 2^-53, m from 27 + 26 bits */
double orc_u01_24(uint32_t hi);                /* (2 (hi >> 9) + 1) 2^-24, exact in float */

/* ---------------- special functions ---------------- */
/* out = { K_{1/3}(x), K_{2/3}(x), IntK_{1/3}(x) = int_x^inf K_{1/3} }; 0 for x >= 700 */
void orc_bessel3(double x, double out[3]);

/* ---------------- spectra (basis components: 0 = eps, 1 = beta, 2 = k) ---------------- */
double orc_nlc_w(double chi, double lam, double sb);
void   orc_nlc_g(double chi, double lam, const double si[3], double g[3]);
void   orc_nlc_F(double chi, double lam, const double si[3], const double sf[3], double F[4]);
void   orc_nbw_G(double chi, double lam, const double se[3], const double sp[3], double G[4]);
void   orc_nbw_j(double chi, double lam, const double xi[3], double *w0, double je[3], double jp[3]);

/* ---------------- exact rates, CDFs and inverse CDFs ---------------- */
/* channel: 0 = NLC spin-down (s_beta=-1), 1 = NLC spin-up (+1),
            2 = NBW xi3=-1, 3 = NBW xi3=+1 */
double orc_density_nu(int channel, double chi, double nu);      /* spectrum * lam(1-lam) */
double orc_rate_integral(int channel, double chi);              /* int_0^1 spectrum dlam */
double orc_cdf(int channel, double chi, double lam);            /* exact, by quadrature */
double orc_ccdf(int channel, double chi, double lam);           /* 1 - cdf, computed directly */
double orc_icdf_nu(int channel, double chi, double rho);        /* logit(lam) at logit(r)=rho */

/* ---------------- tables of the specified grid ---------------- */
typedef struct {
    int    n_chi[2];        /* 0 = NLC, 1 = NBW */
    double lnchi0[2];       /* ln chi of node 0 */
    double dlnchi[2];       /* node spacing in ln chi */
    int    n_rho;
    double rho0, drho;      /* rho node j = rho0 + j drho */
} orc_table_spec;

typedef struct {
    orc_table_spec spec;
    double *lnrate;         /* [4][n_chi(channel)] : ln int spectrum, + 8/(3 chi) in the pair rows */
    double *nu;             /* [4][n_chi(channel)][n_rho] */
    int64_t off_rate[4], off_nu[4];
    double *lngfac;         /* [ORC_GF_N]: ln(a(chi)/a(0)) at ln chi = ORC_GF_LNCHI0 + i ORC_GF_DLNCHI */
} orc_tables;

int    orc_tables_build(orc_tables *T, const orc_table_spec *spec, int nthreads);
void   orc_tables_free(orc_tables *T);
/* lngfac may be NULL: the g-factor table is then built here */
int    orc_tables_load(orc_tables *T, const orc_table_spec *spec, const double *lnrate, const double *nu,
                       const double *lngfac);
double orc_table_lnrate(const orc_tables *T, int channel, double lnchi);
double orc_table_nu(const orc_tables *T, int channel, double lnchi, double rho);

/* ---------------- fields ---------------- */
enum { ORC_FIELD_UNIFORM = 0, ORC_FIELD_PLANE_LP = 1, ORC_FIELD_GRID2D = 2, ORC_FIELD_ROTATING_E = 3 };
typedef struct {
    int    kind;
    double E0[3], B0[3];    /* uniform */
    double a0;              /* plane wave amplitude */
    double phase_len;       /* sin^2 envelope length in phase (0 = no envelope) */
    /* static 2-D grid (x, y), periodic: six node arrays Ex, Ey, Ez, Bx, By, Bz of nx * ny floats,
       node (i, j) at (x0 + i dx, y0 + j dy), index j * nx + i; bilinear interpolation */
    const float *grid[6];
    int    nx, ny;
    double dx, dy, x0, y0;
} orc_fields;
void orc_fields_eval(const orc_fields *f, const double x[3], double t, double E[3], double B[3]);

/* ---------------- particle state ---------------- */
enum {
    ORC_F_PUSH = 1u << 0, ORC_F_TBMT = 1u << 1, ORC_F_EMIT = 1u << 2, ORC_F_RECOIL = 1u << 3,
    ORC_F_SPIN = 1u << 4, ORC_F_NOEMIT = 1u << 5, ORC_F_PHOTON_POL = 1u << 6, ORC_F_MEAN = 1u << 7,
    ORC_F_PAIR = 1u << 8, ORC_F_NOPAIR = 1u << 9, ORC_F_PAIR_SPIN = 1u << 10,
    ORC_F_TAU = 1u << 11,    /* emission decided by the optical depth instead of the per-step draw */
    ORC_F_REJECT = 1u << 12, /* emission decided and lambda sampled together by rejection from the
                                spin-resolved spectrum with candidates lambda = r1^3 (spectrum-sampling
                                section), instead of the draw against W dt and the inverse CDF */
    ORC_F_GCHI = 1u << 13,   /* T-BMT with the field-dependent anomalous moment a_e a(chi)/a(0)
                                (loop appendix) instead of the constant a_e */
    ORC_F_SUB = 1u << 14     /* per-particle sub-cycling of the lepton QED part where W dt is large:
                                m = the smallest power of two with W_s dt / m <= ORC_SUB_WDT (at most
                                ORC_SUB_ROUNDS) sub-steps of dt/m, taken in ORC_SUB_ROUNDS rounds */
};
#define ORC_SUB_ROUNDS 16
#define ORC_SUB_WDT 0.1

typedef struct {
    double   t, dt, a_e, eps_r;
    double   chi_e_min, chi_e_max, chi_g_min, chi_g_max;
    double   k_retire;      /* photons with |k| below this are never stored / stepped */
    double   near_tol;      /* relative distance to a threshold that counts as a near tie */
    int64_t  step;
    uint64_t seed;
    uint32_t flags;
    int      u24;           /* 1: uniforms from the 24-bit map (single-precision path) */
    int      sub_round;     /* sub-cycling round of this call (0 otherwise): Philox channels of the
                               lepton step are offset by 16 sub_round, and the photon id carries it */
} orc_params;

typedef struct {
    int64_t n, cap;
    int     species;        /* 0 = e-, 1 = e+ */
    double *x[3], *p[3], *s[3];   /* x[i] may be NULL: coordinate not tracked (taken as 0) */
    uint8_t *near;          /* optional: set to 1 when a decision of this particle was a near tie */
    int64_t *index;         /* optional: index that names particle j in its full set (default j) */
    double  *tau, *tau_target;  /* optical depth and its target (ORC_F_TAU only); target 0 = not drawn */
    double  *cond;          /* optional diagnostic, no effect on the step: the conditioning of the
                               collapse axes behind the particle's spin, i.e. how many times the
                               unit roundoff the axis direction can be off: the norm of the sums of
                               the absolute terms of g over |g| (NLC appendix: s_f = +-g/|g|), the
                               largest over its emissions so far; the same of j over |j| for a
                               lepton made by a pair (NBW appendix); 0 with no collapse */
} orc_leptons;

typedef struct {
    int64_t   n, cap, n_prev;
    double   *x[3], *k[3], *P[3];
    uint64_t *id;           /* 0 = dead slot */
    uint8_t  *near;         /* optional, as for leptons */
    double   *cond;         /* optional diagnostic, as for leptons: of the Stokes collapse
                               xi = +-F/|F| at the photon's birth, the norm of the sums of the
                               absolute terms of F over |F|, times 1 + the parent's spin-axis
                               conditioning (F is taken at the collapsed s_f); 1 without it */
} orc_photons;

typedef struct {
    int64_t n_emit, n_pair, n_prob_clamped, n_chi_clamped, n_norm_clamped,
            n_capacity_overflow, n_retired, n_near_threshold, n_lepton_steps, n_photon_steps,
            n_nonfinite;    /* particle-steps not taken for a NaN or infinity in the inputs (see the steps) */
} orc_counters;

/* Lorentz (Boris) push + T-BMT rotation + position advance for one lepton.  With ORC_F_GCHI the
   anomalous moment is a_e times the tabulated a(chi)/a(0) at the mid-step chi (T and eps_r
   needed then; otherwise T may be NULL). */
void orc_push_one(int charge, double a_e, const double E[3], const double B[3], double dt,
                  uint32_t flags, const orc_tables *T, double eps_r, double p[3], double s[3], double x[3]);

/* Field-dependent anomalous moment (loop appendix). */
double orc_scorer_gi(double z);              /* Scorer function Gi(z), z >= 0 */
double orc_gfactor_ratio(double chi);        /* a(chi)/a(0) by direct quadrature */
double orc_table_gfac(const orc_tables *T, double chi);   /* the same from the table */
#define ORC_GF_N 705                         /* chi from 1e-7 to 1e4, 64 nodes per decade */
#define ORC_GF_LNCHI0 (-16.11809565095832)   /* ln 1e-7 */
#define ORC_GF_DLNCHI (0.03597789207803197)  /* ln 10 / 64 */

/* One whole lepton step (push with fields at t, QED with fields at t+dt) over L. */
int orc_lepton_step(const orc_tables *T, const orc_params *prm, const orc_fields *f,
                    orc_leptons *L, orc_photons *G, orc_counters *ctr, int nthreads);
/* One photon step over photons [0, G->n_prev); afterwards n_prev = n.  A photon is retired
   (dead slot) when |k| < k_retire or, for the plane-wave field with an envelope, when its
   phase t + x is past the pulse's trailing end (the phase of a photon never decreases). */
int orc_photon_step(const orc_tables *T, const orc_params *prm, const orc_fields *f,
                    orc_photons *G, orc_leptons *Le, orc_leptons *Lp, orc_counters *ctr,
                    int nthreads);
/* Order-preserving removal of dead photons (id == 0). */
void orc_compact(orc_photons *G);

/* QED-only steps on one particle at given fields (used by the per-particle tests). */
int orc_lepton_qed_one(const orc_tables *T, const orc_params *prm, int species, int64_t index,
                       const double E[3], const double B[3], const double x[3],
                       double p[3], double s[3], double k_out[3], double P_out[3],
                       uint64_t *id_out, double tau2[2], orc_counters *ctr);
int orc_photon_qed_one(const orc_tables *T, const orc_params *prm, uint64_t id,
                       const double E[3], const double B[3], const double k[3], double P[3],
                       double pe[3], double se[3], double pp[3], double sp[3], orc_counters *ctr);

/* Stokes <-> P-vector in a given right-handed basis (eps, beta, khat). */
void orc_stokes_to_P(const double xi[3], const double e[3], const double b[3], const double k[3],
                     double P[3]);
void orc_P_to_stokes(const double P[3], const double e[3], const double b[3], const double k[3],
                     double xi[3]);
/* lepton (charge -1/+1) or photon (charge 0 -> electron convention) basis; returns chi */
double orc_basis(int charge, double eps_r, const double E[3], const double B[3],
                 const double p[3], double e[3], double b[3], double k[3]);

#ifdef __cplusplus
}
#endif
#endif
