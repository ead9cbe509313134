// qs_tables.hip -- GPU construction of the rate and inverse-CDF tables (qed_init_tables).
//
// The NLC section tabulates the emission rate and the inverse CDF of the photon spectrum only
// for the initial spin along / against the rest-frame B (s_beta = +1 / -1); the NBW section
// does the same for photons with xi3 = +1 / -1.  Each table entry is computed here by
// quadrature of the spectrum in nu = ln(lam/(1-lam)) (dlam = lam (1-lam) dnu), where the
// integrand is smooth and decays at both ends:
//   rate   ln int_0^1 w dlam;
//   ICDF   nu(rho) with CDF(lam(nu)) = r, rho = ln(r/(1-r)), solved by Newton's method on
//          ln(cumulative) with a bisection safeguard, from the left for r <= 1/2 and on the
//          complementary CDF from the right for r > 1/2 so both tails keep full precision.
// Below nu = -60 the NLC spectrum follows its small-lambda law
//   int_0^lam w = 3 Gamma(2/3) (3 chi)^(2/3) lam^(1/3) - (pi/sqrt 3) lam   (relative remainder < 1e-26).
// Quadrature: 12-point Gauss-Legendre panels in nu, at most 1/2 wide and narrow enough that
// the density's exponential factor e^{-u'} changes by at most e per panel (the density is
// analytic in the strip |Im nu| < pi/2, so each panel is exact to rounding); the range ends
// where u' exceeds its minimum by 90.  Bessel functions by the trapezoidal rule of qs_device.hpp.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "qs_internal.hpp"

namespace {

constexpr int kNQ = 12;
constexpr double kNuLo = -60.0;
constexpr int kMaxPanels = 512;

struct GL12 { double x[kNQ], w[kNQ]; };

struct BuildArgs {
    int n_chi[2];
    double lnchi0[2], dlnchi[2];
    int n_rho;
    double rho0, drho;
    int off_rate[4];
    int64_t off_nu[4];
};

// Legendre nodes and weights on [-1, 1] by Newton's method on P_n (host)
GL12 legendre_nodes()
{
    GL12 g;
    const int n = kNQ;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double dp = 1.0;
        for (int it = 0; it < 50; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        g.x[i] = x;
        g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

__device__ __forceinline__ double kPi_over_sqrt3() { return qs::kPi / sqrt(3.0); }

// trapezoid node tables of qs_device.hpp (host, FP64 libm): per node cosh t - 1, cosh(t/3),
// cosh(2t/3), cosh(t/3)/cosh t at t = j h
void fill_nodes(std::vector<double> &n64, std::vector<float> &n32)
{
    n64.assign(4 * qs::kBn64Nodes, 0.0);
    for (int k = 0; k < qs::kBn64Levels; ++k) {
        const int off = k == 0 ? 0 : qs::kBn64N0 + (k - 1) * qs::kBn64N, nn = k == 0 ? qs::kBn64N0 : qs::kBn64N;
        const double h = 0.2 / (double)(1 << k);
        for (int j = 0; j < nn; ++j) {
            const double t = j * h, sh = sinh(0.5 * t);
            const double chm1 = 2.0 * sh * sh, c1 = cosh(t / 3.0);
            double *q = &n64[4 * (off + j)];
            q[0] = chm1; q[1] = c1; q[2] = cosh(2.0 * t / 3.0); q[3] = c1 / (1.0 + chm1);
        }
    }
    n32.assign(4 * qs::kBn32Nodes, 0.0f);
    const double *h32 = qs::kBn32H;
    for (int k = 0; k < qs::kBn32Levels; ++k) {
        const int off = k == 0 ? 0 : qs::kBn32N0 + (k - 1) * qs::kBn32N, nn = k == 0 ? qs::kBn32N0 : qs::kBn32N;
        for (int j = 0; j < nn; ++j) {
            const double t = j * h32[k], sh = sinh(0.5 * t);
            const double chm1 = 2.0 * sh * sh, c1 = cosh(t / 3.0);
            float *q = &n32[4 * (off + j)];
            q[0] = (float)fmin(chm1, 1e38); q[1] = (float)c1; q[2] = (float)cosh(2.0 * t / 3.0);
            q[3] = (float)(c1 / (1.0 + chm1));
        }
    }
}

// spectrum density in nu for channel ch (un-normalized): w lam (1-lam)
__device__ double density(int ch, double chi, double nu, const double *bn)
{
    const double lam = 1.0 / (1.0 + exp(-nu)), oml = 1.0 / (1.0 + exp(nu));
    if (ch < 2) {
        const double up = 2.0 * exp(nu) / (3.0 * chi);
        if (!(up < 700.0)) return 0.0;
        const qs::Bessel3 b = qs::bessel3_scaled(up, bn);
        const double kap = 1.0 / oml + oml;
        const double w = -b.ik + kap * b.k23 + (ch == 1 ? lam : -lam) * b.k13;
        return exp(-up) * w * lam * oml;
    } else {
        const double ut = 1.0 / lam + 1.0 / oml;
        const double up = 2.0 * ut / (3.0 * chi);
        if (!(up < 700.0)) return 0.0;
        const qs::Bessel3 b = qs::bessel3_scaled(up, bn);
        const double rho = oml / lam + lam / oml;
        const double w0 = b.ik + rho * b.k23 - (ch == 3 ? 1.0 : -1.0) * b.k23;
        return exp(-up) * w0 * lam * oml;
    }
}

__device__ double gl_integral(const GL12 &g, int ch, double chi, double a, double b, const double *bn)
{
    if (!(b > a)) return 0.0;
    const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    double s = 0.0;
    for (int i = 0; i < kNQ; ++i) s += g.w[i] * density(ch, chi, mid + half * g.x[i], bn);
    return half * s;
}

// Newton on ln(cum(nu)) - ln(target) inside [lo, hi].
// side > 0: cum = base + int_lo^nu f (increasing); side < 0: cum = base + int_nu^hi f (decreasing).
__device__ double solve_root(const GL12 &g, int ch, double chi, int side, double base, double pint,
                             double lo, double hi, double target, const double *bn)
{
    const double c_lo = side > 0 ? base : base + pint;
    const double c_hi = side > 0 ? base + pint : base;
    const double lt = log(target);
    const double l_lo = log(fmax(c_lo, 1e-300)), l_hi = log(fmax(c_hi, 1e-300));
    double a = lo, b = hi;
    double nu = (l_hi != l_lo) ? lo + (hi - lo) * (lt - l_lo) / (l_hi - l_lo) : 0.5 * (lo + hi);
    if (!(nu > a && nu < b)) nu = 0.5 * (a + b);
    for (int it = 0; it < 80; ++it) {
        const double cum = side > 0 ? base + gl_integral(g, ch, chi, lo, nu, bn) : base + gl_integral(g, ch, chi, nu, hi, bn);
        const double r = log(cum) - lt;
        const double f = density(ch, chi, nu, bn);
        const double step = f > 0.0 ? r * cum / (side > 0 ? f : -f) : 0.0;
        if (fabs(r) < 1e-15) {
            if (nu - step > a && nu - step < b) nu -= step;
            break;
        }
        if ((side > 0) == (r > 0.0)) b = nu; else a = nu;
        double nn = nu - step;
        if (!(f > 0.0) || !(nn > a && nn < b)) nn = 0.5 * (a + b);
        if (fabs(nn - nu) <= 2e-16 * fmax(1.0, fabs(nu)) || (b - a) <= 2e-16 * fmax(1.0, fabs(nu))) {
            nu = nn;
            break;
        }
        nu = nn;
    }
    return nu;
}

// decay rate |d u'/d nu| of the density's e^{-u'} factor: NLC u' = 2 e^nu/(3 chi),
// NBW u~' = 4 (1 + cosh nu)/(3 chi)
__device__ __forceinline__ double decay(int ch, double chi, double nu)
{
    return ch < 2 ? 2.0 * exp(nu) / (3.0 * chi) : 4.0 * fabs(sinh(nu)) / (3.0 * chi);
}

__global__ void __launch_bounds__(256) k_build_tables(BuildArgs A, GL12 g, double *lnrate, double *nu_out,
                                                      const double *bn)
{
    __shared__ double pint[kMaxPanels], left[kMaxPanels + 1], right[kMaxPanels + 1], edge[kMaxPanels + 1];
    __shared__ double s_total, s_tail;
    __shared__ int s_np;
    int task = blockIdx.x, ch, i;
    if (task < 2 * A.n_chi[0]) { ch = task / A.n_chi[0]; i = task % A.n_chi[0]; }
    else { const int t2 = task - 2 * A.n_chi[0]; ch = 2 + t2 / A.n_chi[1]; i = t2 % A.n_chi[1]; }
    const int grp = ch < 2 ? 0 : 1;
    const double chi = exp(A.lnchi0[grp] + i * A.dlnchi[grp]);
    // range: up to where u' exceeds its minimum by 90 (the mass beyond is < e^-90 of the total)
    double a0, b1;
    if (ch < 2) { a0 = kNuLo; b1 = log(1.5 * chi * 90.0); }
    else {
        const double m = acosh(1.0 + 0.75 * chi * 90.0);
        a0 = -m; b1 = m;
    }
    // panels no wider than 1/2 with |d u'/d nu| * width <= 1 (built by one thread)
    if (threadIdx.x == 0) {
        int np = 0;
        double a = a0;
        edge[0] = a;
        while (a < b1 && np < kMaxPanels) {
            double w = 0.5;
            while (w > 1.0 / 4096.0 && w * fmax(decay(ch, chi, a), decay(ch, chi, a + w)) > 1.0) w *= 0.5;
            const double b = np == kMaxPanels - 1 ? b1 : fmin(a + w, b1);
            edge[++np] = b;
            a = b;
        }
        s_np = np;
    }
    __syncthreads();
    int np = s_np;
    for (int p = threadIdx.x; p < np; p += blockDim.x) pint[p] = gl_integral(g, ch, chi, edge[p], edge[p + 1], bn);
    __syncthreads();
    if (threadIdx.x == 0) {
        double tail = 0.0;
        if (ch < 2) {
            const double lam0 = 1.0 / (1.0 + exp(-a0));
            tail = 3.0 * tgamma(2.0 / 3.0) * pow(3.0 * chi, 2.0 / 3.0) * cbrt(lam0) - kPi_over_sqrt3() * lam0;
        }
        left[0] = tail;
        for (int p = 0; p < np; ++p) left[p + 1] = left[p] + pint[p];
        right[np] = 0.0;
        for (int p = np - 1; p >= 0; --p) right[p] = right[p + 1] + pint[p];
        s_total = tail + right[0];
        s_tail = tail;
        s_np = np;
        // pair rows: ln W + 8/(3 chi), the Erber exponent taken out so the rows are smooth in ln chi
        lnrate[A.off_rate[ch] + i] = log(s_total) + (ch >= 2 ? qs::kErber / chi : 0.0);
    }
    __syncthreads();
    const double total = s_total, tail = s_tail;
    np = s_np;
    double *row = nu_out + A.off_nu[ch] + (int64_t)i * A.n_rho;
    for (int j = threadIdx.x; j < A.n_rho; j += blockDim.x) {
        const double rho = A.rho0 + j * A.drho;
        double nu;
        if (rho <= 0.0) {
            const double target = total / (1.0 + exp(-rho));
            if (ch < 2 && target <= tail) {
                const double Ac = 3.0 * tgamma(2.0 / 3.0) * pow(3.0 * chi, 2.0 / 3.0), Bc = kPi_over_sqrt3();
                double y = target / Ac;
                for (int it = 0; it < 4; ++it) y -= (Ac * y - Bc * y * y * y - target) / (Ac - 3.0 * Bc * y * y);
                nu = 3.0 * log(y) - log1p(-y * y * y);
            } else {
                int lo = 0, hi = np;
                while (hi - lo > 1) { const int m = (lo + hi) >> 1; if (left[m] <= target) lo = m; else hi = m; }
                nu = solve_root(g, ch, chi, +1, left[lo], pint[lo], edge[lo], edge[lo + 1], target, bn);
            }
        } else {
            const double target = total / (1.0 + exp(rho));
            int lo = 0, hi = np;
            while (hi - lo > 1) { const int m = (lo + hi) >> 1; if (right[m] > target) lo = m; else hi = m; }
            nu = solve_root(g, ch, chi, -1, right[lo + 1], pint[lo], edge[lo], edge[lo + 1], target, bn);
        }
        row[j] = nu;
    }
}

// ---------------------------------------------------------------- field-dependent g (loop appendix)
// Scorer function Gi(z), z >= 0.  For z <= 16 the ray form of Ai + i Gi = (1/pi) int_0^inf
// exp(i(z t + t^3/3)) dt at t = exp(i pi/6) s,
//   Gi(z) = (1/pi) int_0^inf exp(-s^3/3 - z s/2) sin((sqrt3/2) z s + pi/6) ds,
// by the trapezoidal rule in w = ln s with step 1/20 (the integrand is analytic for |Im w| < pi/6,
// so the rule's error is of order exp(-pi^2/(3 h)) = e^-66), from w = -45 until the exponent
// passes -50.  For z > 16 the large-argument series (1/(pi z)) sum_k (3k)!/(k! (3 z^3)^k), summed
// until a term falls below 1e-18 of the sum (its smallest term there is far below that).
__device__ double scorer_gi(double z)
{
    if (z > 16.0) {
        const double x = 1.0 / (3.0 * z * z * z);
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < 40; ++k) {
            term *= (3.0 * k) * (3.0 * k - 1.0) * (3.0 * k - 2.0) / k * x;
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        return sum / (qs::kPi * z);
    }
    const double h = 0.05, c = 0.5 * sqrt(3.0) * z;
    double acc = 0.0;
    for (int k = 0; k < 1000; ++k) {
        const double s = exp(-45.0 + k * h), ex = s * s * s / 3.0 + 0.5 * z * s;
        if (ex > 50.0) break;
        acc += s * exp(-ex) * sin(c * s + qs::kPi / 6.0);
    }
    return acc * h / qs::kPi;
}

// One block per node: a(chi)/a(0) = 2 pi int_0^1 (1 - lam) z Gi(z) dlam, z = (lam/((1-lam) chi))^(2/3),
// in nu = ln(lam/(1-lam)) (dlam = lam (1-lam) dnu), by 12-point Gauss-Legendre panels at most 1/2
// wide on [min(ln chi, 0) - 40, 25] (the integrand falls as e^(5 nu/3) and e^(-2 nu) at the ends
// and is analytic within pi/2 of the real axis).  Threads take the points in a fixed order and
// the block sums them by a fixed tree, so the table is the same on every build.
__global__ void __launch_bounds__(256) k_build_gfac(GL12 g, double *lng)
{
    __shared__ double part[256];
    const int node = blockIdx.x;
    const double lc = qs::kGfLnChi0 + node * qs::kGfDlnChi;
    const double a = (lc < 0.0 ? lc : 0.0) - 40.0, b = 25.0;
    const int np = (int)ceil((b - a) / 0.5);
    const double w = (b - a) / np;
    double acc = 0.0;
    for (int k = threadIdx.x; k < np * kNQ; k += blockDim.x) {
        const int pnl = k / kNQ, q = k % kNQ;
        const double nu = a + (pnl + 0.5) * w + 0.5 * w * g.x[q];
        const double u = exp(nu), z = exp(2.0 * (nu - lc) / 3.0);
        acc += g.w[q] * u / ((1.0 + u) * (1.0 + u) * (1.0 + u)) * z * scorer_gi(z);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) lng[node] = log(2.0 * qs::kPi * 0.5 * w * part[0]);
}

__global__ void k_to_float(const double *src, float *dst, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

}  // namespace

static thread_local char g_last_error[256];

qed_status qs_fail(hipError_t e, const char *where)
{
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
    return QED_ERR_HIP;
}

qed_status qs_reject(qed_status st, const char *msg)
{
    snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
    return st;
}

extern "C" const char *qed_last_error(void) { return g_last_error; }

extern "C" qed_status qed_init_tables(const qed_table_params *params, qed_stream stream, qed_tables *out)
{
    if (!params || !out) return QED_ERR_INVALID;
    const qed_table_grid &G = params->grid;
    if (G.n_chi[0] < 4 || G.n_chi[1] < 4 || G.n_rho < 4 || !(G.dlnchi[0] > 0) || !(G.dlnchi[1] > 0) ||
        !(G.drho > 0))
        return QED_ERR_INVALID;
    if (params->precision != QED_F64 && params->precision != QED_F32) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    qed_tables T = (qed_tables)calloc(1, sizeof(qed_tables_s));
    if (!T) return QED_ERR_INVALID;
    T->params = *params;
    BuildArgs A;
    int r = 0;
    int64_t v = 0;
    for (int c = 0; c < 4; ++c) {
        const int n = G.n_chi[c < 2 ? 0 : 1];
        A.off_rate[c] = r;
        A.off_nu[c] = v;
        T->dev.off_rate[c] = r;
        T->dev.off_nu[c] = v;
        r += n;
        v += (int64_t)n * G.n_rho;
    }
    for (int k = 0; k < 2; ++k) {
        A.n_chi[k] = G.n_chi[k];
        A.lnchi0[k] = G.lnchi0[k];
        A.dlnchi[k] = G.dlnchi[k];
    }
    A.n_rho = G.n_rho;
    A.rho0 = G.rho0;
    A.drho = G.drho;
    T->n_rate = r;
    T->n_nu = v;
    std::vector<double> n64;
    std::vector<float> n32;
    fill_nodes(n64, n32);
    hipError_t e = hipMalloc(&T->d_lnrate, sizeof(double) * r);
    if (e == hipSuccess) e = hipMalloc(&T->d_lnrate32, sizeof(float) * r);
    if (e == hipSuccess) e = hipMalloc(&T->d_nu, sizeof(double) * v);
    if (e == hipSuccess) e = hipMalloc(&T->d_bn64, sizeof(double) * n64.size());
    if (e == hipSuccess) e = hipMalloc(&T->d_bn32, sizeof(float) * n32.size());
    if (e == hipSuccess) e = hipMalloc(&T->d_lng, sizeof(double) * qs::kGfN);
    if (e == hipSuccess) e = hipMalloc(&T->d_lng32, sizeof(float) * qs::kGfN);
    if (e == hipSuccess) e = hipMemcpyAsync(T->d_bn64, n64.data(), sizeof(double) * n64.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(T->d_bn32, n32.data(), sizeof(float) * n32.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        qed_free_tables(T);
        return qs_fail(e, "hipMalloc / upload (tables)");
    }
    const GL12 g = legendre_nodes();
    const int ntask = 2 * G.n_chi[0] + 2 * G.n_chi[1];
    QS_LAUNCH(K_TABLES, k_build_tables, dim3(ntask), dim3(256), 0, st, A, g, T->d_lnrate, T->d_nu,
              (const double *)T->d_bn64);
    QS_LAUNCH(K_TABLES, k_to_float, dim3((r + 255) / 256), dim3(256), 0, st, T->d_lnrate, T->d_lnrate32, r);
    QS_LAUNCH(K_TABLES, k_build_gfac, dim3(qs::kGfN), dim3(256), 0, st, g, T->d_lng);
    QS_LAUNCH(K_TABLES, k_to_float, dim3((qs::kGfN + 255) / 256), dim3(256), 0, st, (const double *)T->d_lng,
              T->d_lng32, qs::kGfN);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        qed_free_tables(T);
        return qs_fail(e, "table build kernels");
    }
    TablesDev &D = T->dev;
    for (int k = 0; k < 2; ++k) {
        D.n_chi[k] = G.n_chi[k];
        D.lnchi0[k] = G.lnchi0[k];
        D.dlnchi[k] = G.dlnchi[k];
    }
    D.n_rho = G.n_rho;
    D.rho0 = G.rho0;
    D.drho = G.drho;
    D.lnrate = T->d_lnrate;
    D.lnrate32 = T->d_lnrate32;
    D.nu = T->d_nu;
    D.bn64 = T->d_bn64;
    D.bn32 = T->d_bn32;
    D.lng = T->d_lng;
    D.lng32 = T->d_lng32;
    *out = T;
    return QED_OK;
}

extern "C" qed_status qed_free_tables(qed_tables T)
{
    if (!T) return QED_OK;
    if (T->d_lnrate) (void)hipFree(T->d_lnrate);
    if (T->d_lnrate32) (void)hipFree(T->d_lnrate32);
    if (T->d_nu) (void)hipFree(T->d_nu);
    if (T->d_bn64) (void)hipFree(T->d_bn64);
    if (T->d_bn32) (void)hipFree(T->d_bn32);
    if (T->d_lng) (void)hipFree(T->d_lng);
    if (T->d_lng32) (void)hipFree(T->d_lng32);
    free(T);
    return QED_OK;
}

extern "C" qed_status qed_tables_download(qed_tables T, double *lnrate, int64_t *n_lnrate, double *nu, int64_t *n_nu)
{
    if (!T) return QED_ERR_INVALID;
    if (n_lnrate) *n_lnrate = T->n_rate;
    if (n_nu) *n_nu = T->n_nu;
    if (lnrate) QS_CHECK(hipMemcpy(lnrate, T->d_lnrate, sizeof(double) * T->n_rate, hipMemcpyDeviceToHost));
    if (nu) QS_CHECK(hipMemcpy(nu, T->d_nu, sizeof(double) * T->n_nu, hipMemcpyDeviceToHost));
    return QED_OK;
}

extern "C" qed_status qed_tables_download_gfac(qed_tables T, double *lngfac, int64_t *n)
{
    if (!T) return QED_ERR_INVALID;
    if (n) *n = qs::kGfN;
    if (lngfac) QS_CHECK(hipMemcpy(lngfac, T->d_lng, sizeof(double) * qs::kGfN, hipMemcpyDeviceToHost));
    return QED_OK;
}
