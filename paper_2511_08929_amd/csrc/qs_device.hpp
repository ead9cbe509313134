// qs_device.hpp -- device math of the spin- and polarization-resolved QED step (gfx950).
//
// Precision policy: particle state and bulk arithmetic in R (float or double); FP64 islands
// for chi (cancellation in p0 E + p x B for co-propagating geometry), for the inverse-CDF
// interpolation and lambda = 1/(1+exp(-nu)) (small-photon-energy tail), and for the Bessel
// functions K_1/3, K_2/3, IntK_1/3 of the emitters.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

constexpr double kAlpha = 7.2973525693e-3;
constexpr double kPi = 3.14159265358979323846;
// exponent of the low-chi pair rate, W ~ exp(-kErber / chi_gamma): the pair rows of the rate table
// hold ln W + kErber / chi
constexpr double kErber = 8.0 / 3.0;

// physics switches (values of the C ABI enum)
enum : uint32_t {
    F_PUSH = 1u << 0, F_TBMT = 1u << 1, F_EMIT = 1u << 2, F_RECOIL = 1u << 3, F_SPIN = 1u << 4,
    F_NOEMIT = 1u << 5, F_PHOTON_POL = 1u << 6, F_MEAN = 1u << 7, F_PAIR = 1u << 8,
    F_NOPAIR = 1u << 9, F_PAIR_SPIN = 1u << 10, F_TAU = 1u << 11, F_REJECT = 1u << 12, F_GCHI = 1u << 13,
    F_SUB = 1u << 14
};

// Sub-cycling of the lepton step: a lepton takes 2^k <= kSubRounds sub-steps, the smallest with
// W_s dt / 2^k <= kSubWdt, one in every kSubRounds / 2^k-th of kSubRounds rounds.
constexpr int kSubRounds = 16;
constexpr int kSubLog2Max = 4;
constexpr double kSubWdt = 0.1;

// Field-dependent anomalous moment (loop appendix): table of ln(a(chi)/a(0)) at 64 nodes per
// decade of chi from 1e-7 to 1e4 (node i at ln chi = kGfLnChi0 + i kGfDlnChi).
constexpr int kGfN = 705;
constexpr double kGfLnChi0 = -16.11809565095832;   // ln 1e-7
constexpr double kGfDlnChi = 0.03597789207803197;  // ln 10 / 64

// ------------------------------------------------------------------ small vectors
// A renormalization of |s| or |xi| is counted when the excess over 1 of the squared norm is
// above rounding noise of the precision: 1e-12 in FP64, 1e-6 (about 8 ulp) in FP32.
template <class R> __device__ __forceinline__ constexpr R norm_count_tol();
template <> __device__ __forceinline__ constexpr double norm_count_tol<double>() { return 1e-12; }
template <> __device__ __forceinline__ constexpr float norm_count_tol<float>() { return 1e-6f; }

template <class R> struct V3 { R x, y, z; };

template <class R> __device__ __forceinline__ V3<R> v3(R a, R b, R c) { return V3<R>{a, b, c}; }
template <class R> __device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator*(R s, V3<R> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class R> __device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class R> __device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class D, class S> __device__ __forceinline__ V3<D> cvt(V3<S> a) { return {(D)a.x, (D)a.y, (D)a.z}; }

// Single precision uses the hardware approximations (about 1 ulp): v_rsq, v_sqrt, v_rcp, v_exp
// (base 2) and v_log (base 2).  Double precision uses the correctly rounded library forms.
__device__ __forceinline__ float rsqrt_r(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double rsqrt_r(double v) { return 1.0 / sqrt(v); }
__device__ __forceinline__ float sqrt_r(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double sqrt_r(double v) { return sqrt(v); }
__device__ __forceinline__ float rcp_r(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp_r(double v) { return 1.0 / v; }
__device__ __forceinline__ float exp_r(float v) { return __builtin_amdgcn_exp2f(v * 1.44269504088896341f); }
__device__ __forceinline__ double exp_r(double v) { return exp(v); }
__device__ __forceinline__ float log_r(float v) { return __builtin_amdgcn_logf(v) * 0.693147180559945309f; }
__device__ __forceinline__ double log_r(double v) { return log(v); }
// num / den of two FP64 values, rounded to R: exact division in FP64, v_rcp in FP32
template <class R> __device__ __forceinline__ R ratio_r(double num, double den);
template <> __device__ __forceinline__ double ratio_r<double>(double num, double den) { return num / den; }
template <> __device__ __forceinline__ float ratio_r<float>(double num, double den) { return (float)num * rcp_r((float)den); }

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): 10 rounds of two 32x32 -> 64 multiplies with
// Weyl-sequence key bumps.
// PIN: the key (the step's seed, the same for every lane of a wave, so its first lane is exact)
// is taken into scalar registers and hidden from the optimizer, so that the round keys are formed
// by scalar adds at each call instead of once ahead of a loop; kept there, they outnumber the
// scalar registers of the photon pass, whose hot loop then reloaded each from a vector lane.
template <bool PIN = false> __device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
    if constexpr (PIN) {
        k0 = __builtin_amdgcn_readfirstlane(k0);
        k1 = __builtin_amdgcn_readfirstlane(k1);
        asm volatile("" : "+s"(k0), "+s"(k1));
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product per multiplier gives both halves
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x, m1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(m1 >> 32) ^ c.y ^ k0, (uint32_t)m1, (uint32_t)(m0 >> 32) ^ c.w ^ k1, (uint32_t)m0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

template <bool PIN = false>
__device__ __forceinline__ uint4 philox_block(uint64_t seed, uint64_t id, int64_t step, uint32_t channel)
{
    return philox4x32_10<PIN>(make_uint4((uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step, channel),
                         (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in (0,1): m = 27 high bits of hi : 26 high bits of lo, u = (m + 1/2) 2^-53
__device__ __forceinline__ double u01_53(uint32_t hi, uint32_t lo)
{
    const uint64_t m = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
    return ((double)m + 0.5) * 0x1p-53;
}
// 24-bit uniform in (0,1), exactly representable in float: (2 (hi >> 9) + 1) 2^-24
__device__ __forceinline__ float u01_24(uint32_t hi) { return (float)(2u * (hi >> 9) + 1u) * 0x1p-24f; }

template <class R> struct Unif;
template <> struct Unif<double> {
    static __device__ __forceinline__ void two(uint4 w, double &a, double &b) { a = u01_53(w.x, w.y); b = u01_53(w.z, w.w); }
};
template <> struct Unif<float> {
    static __device__ __forceinline__ void two(uint4 w, float &a, float &b) { a = u01_24(w.x); b = u01_24(w.z); }
};

__device__ __forceinline__ uint64_t lepton_id(int species, int64_t index) { return ((uint64_t)species << 62) | (uint64_t)index; }
// 2^63 | species << 61 | (sub-cycling round << 33 | parent index mod 2^33) << 24 | step mod 2^24
__device__ __forceinline__ uint64_t photon_id(int species, int64_t index, int64_t step, int round)
{
    return (1ull << 63) | ((uint64_t)species << 61) | ((uint64_t)(round & 15) << 57) |
           (((uint64_t)index & ((1ull << 33) - 1)) << 24) | ((uint64_t)step & 0xFFFFFFull);
}

// ------------------------------------------------------------------ Bessel functions
// K_nu(x) = int_0^inf e^{-x cosh t} cosh(nu t) dt, IntK_1/3(x) = int_0^inf e^{-x cosh t} cosh(t/3)/cosh(t) dt,
// by the trapezoidal rule in t, which converges geometrically for these integrands (analytic in
// the strip |Im t| < pi/2): error ~ e^{-pi^2/h} for step h, and e^{-2 pi^2/(h^2 x)} for large x
// where the integrand is a Gaussian of width 1/sqrt(x), hence h = min(h0, c/sqrt(x)).  The
// node values cosh t - 1, cosh(t/3), cosh(2t/3), cosh(t/3)/cosh t are tabulated once per step
// size (qed_init_tables), so a node costs one exponential.  Values are returned scaled by e^{+x}.
//
// FP64 tables: h = 0.2 / 2^k, k = 0..4 (x <= 9, 36, 144, 576, 2304), 1024 nodes at k = 0 and 64
// above, 4 doubles per node; terms stop below e^{-44} of the first.  FP32 tables: h = 0.4, 0.1,
// 0.025 (x <= 6.25, 100, 1600), 256 and 64 nodes, one float4 per node; terms stop below e^{-22}.
constexpr int kBn64Levels = 5, kBn64N0 = 1024, kBn64N = 64;
constexpr int kBn32Levels = 3, kBn32N0 = 256, kBn32N = 64;
constexpr int kBn64Nodes = kBn64N0 + (kBn64Levels - 1) * kBn64N;
constexpr int kBn32Nodes = kBn32N0 + (kBn32Levels - 1) * kBn32N;
constexpr double kBn32H[kBn32Levels] = {0.4, 0.1, 0.025};

struct Bessel3 { double k13, k23, ik; };

__device__ inline Bessel3 bessel3_scaled(double x, const double *nodes)
{
    Bessel3 o{0.0, 0.0, 0.0};
    if (!(x < 700.0)) return o;
    const int k = x <= 9.0 ? 0 : (x <= 36.0 ? 1 : (x <= 144.0 ? 2 : (x <= 576.0 ? 3 : 4)));
    const double h = 0.2 / (double)(1 << k);
    const int off = k == 0 ? 0 : kBn64N0 + (k - 1) * kBn64N, nn = k == 0 ? kBn64N0 : kBn64N;
    const double2 *q = reinterpret_cast<const double2 *>(nodes) + 2 * off;
    double s13 = 0.5, s23 = 0.5, sik = 0.5;     // t = 0 node, half weight
    // nodes in groups of four: the group's loads are issued together, the sums run node by node
    // in the same order (and stop at the same node) as a plain loop
    for (int j0 = 1; j0 < nn; j0 += 4) {
        double2 a[4], b[4];                           // (cosh t - 1, cosh t/3), (cosh 2t/3, cosh t/3 / cosh t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = j0 + u < nn ? j0 + u : nn - 1;
            a[u] = q[2 * j];
            b[u] = q[2 * j + 1];
        }
        bool done = false;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (j0 + u >= nn) {
                done = true;
                break;
            }
            const double e = exp(-x * a[u].x);
            s13 += e * a[u].y;
            s23 += e * b[u].x;
            sik += e * b[u].y;
            if (x * a[u].x > 44.0 && x * (1.0 + a[u].x) > 44.0) {
                done = true;
                break;
            }
        }
        if (done) break;
    }
    o.k13 = h * s13;
    o.k23 = h * s23;
    o.ik = h * sik;
    return o;
}

// Below x = 1 in FP64: the ascending series K_nu = (pi / (2 sin nu pi)) (I_-nu - I_nu), with
// I_mu = sum_k (x/2)^(2k+mu) / (k! Gamma(k+mu+1)) and IntK_1/3(x) = pi/sqrt3 - int_0^x K_1/3 from the
// term-wise integrals 2 (x/2)^(2k+mu+1) / ((2k+mu+1) k! Gamma(k+mu+1)), each of the three divided
// by pi/sqrt3 (sin(pi/3) = sin(2 pi/3)).  Eleven terms: on (0, 1] the three functions and their
// ratios are within 4e-15 relative of their values to 30 digits, where the trapezoid sum needs
// 23 to 70 nodes with an exponential each (the collapse of most emissions is at small x).
template <int M3> __device__ __forceinline__ void small_series64(double h, double lh, double rg, double &s, double &j)
{
    constexpr double mu = (double)M3 / 3.0;          // mu = M3 / 3
    const double h2 = h * h;
    double t = rg * exp(mu * lh);                    // (x/2)^mu / Gamma(mu + 1)
    s = t;
    j = t * h * (2.0 / (mu + 1.0));
#pragma unroll
    for (int k = 1; k < 11; ++k) {
        t *= h2 * (1.0 / ((double)k * ((double)k + mu)));
        s += t;
        j += t * h * (2.0 / (2.0 * (double)k + mu + 1.0));
    }
}

__device__ __forceinline__ void bessel_small64(double x, double &k13, double &k23, double &ik)
{
    const double h = 0.5 * x, lh = log(h);
    double sm2, jm2, sm1, jm1, sp1, jp1, sp2, jp2;
    small_series64<-2>(h, lh, 1.0 / 2.678938534707747634, sm2, jm2);      // 1 / Gamma(1/3)
    small_series64<-1>(h, lh, 1.0 / 1.354117939426400417, sm1, jm1);      // 1 / Gamma(2/3)
    small_series64<1>(h, lh, 1.0 / 0.8929795115692492112, sp1, jp1);      // 1 / Gamma(4/3)
    small_series64<2>(h, lh, 1.0 / 0.9027452929509336113, sp2, jp2);      // 1 / Gamma(5/3)
    k13 = sm1 - sp1;
    k23 = sm2 - sp2;
    ik = 1.0 - (jm1 - jp1);
}

// Ratios K_1/3 / K_2/3 and IntK_1/3 / K_2/3 at x: all the spin and polarization collapse needs.
template <class R> __device__ __forceinline__ void bessel_ratios(double x, const void *nodes, R &K1, R &I);

template <> __device__ __forceinline__ void bessel_ratios<double>(double x, const void *nodes, double &K1, double &I)
{
    if (x < 1.0) {
        double k13, k23, ik;
        bessel_small64(fmax(x, 1e-300), k13, k23, ik);
        K1 = k13 / k23;
        I = ik / k23;
        return;
    }
    const Bessel3 b = bessel3_scaled(x, (const double *)nodes);
    K1 = b.k13 / b.k23;
    I = b.ik / b.k23;
}

// FP32 trapezoid sums of e^{x} K_1/3, e^{x} K_2/3 and e^{x} IntK_1/3 without the step h of
// their level (lvl)
__device__ __forceinline__ void bessel_sums32(float x, const void *nodes, float &s13, float &s23, float &sik, int &lvl)
{
    const int k = x <= 6.25f ? 0 : (x <= 100.0f ? 1 : 2);
    const int off = k == 0 ? 0 : kBn32N0 + (k - 1) * kBn32N, nn = k == 0 ? kBn32N0 : kBn32N;
    const float4 *q = reinterpret_cast<const float4 *>(nodes) + off;
    s13 = 0.5f; s23 = 0.5f; sik = 0.5f;
    lvl = k;
    // nodes in groups of four, as in the double precision sum
    for (int j0 = 1; j0 < nn; j0 += 4) {
        float4 a[4];                                    // cosh t - 1, cosh t/3, cosh 2t/3, ratio
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = q[j0 + u < nn ? j0 + u : nn - 1];
        bool done = false;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (j0 + u >= nn) {
                done = true;
                break;
            }
            const float e = exp_r(-x * a[u].x);
            s13 += e * a[u].y;
            s23 += e * a[u].z;
            sik += e * a[u].w;
            if (x * a[u].x > 22.0f && x * (1.0f + a[u].x) > 22.0f) {
                done = true;
                break;
            }
        }
        if (done) break;
    }
}

// Small x (below 1/2) in FP32: the ascending series K_nu = (pi / (2 sin nu pi)) (I_-nu - I_nu) with
// I_mu = sum_k (x/2)^(2k+mu) / (k! Gamma(k+mu+1)) (sin(pi/3) = sin(2 pi/3), so one factor pi/sqrt3
// for both orders), and IntK_1/3(x) = pi/sqrt3 - int_0^x K_1/3 from the term-wise integrals
// 2 (x/2)^(2k+mu+1) / ((2k+mu+1) k! Gamma(k+mu+1)); the common factor pi/sqrt3 cancels in the
// ratios.  Seven terms: the eighth is below 1e-9 of the first at x = 1/2.
template <int M3> struct SmallSeries {                 // mu = M3 / 3
    static __device__ __forceinline__ void sum(float h, float lh, float rg, float &s, float &j)
    {
        constexpr float mu = (float)M3 / 3.0f;
        const float h2 = h * h;
        float t = rg * exp_r(mu * lh);                  // (x/2)^mu / Gamma(mu + 1)
        s = t;
        j = t * h * (2.0f / (mu + 1.0f));
#pragma unroll
        for (int k = 1; k < 7; ++k) {
            t *= h2 * (1.0f / ((float)k * ((float)k + mu)));
            s += t;
            j += t * h * (2.0f / (2.0f * (float)k + mu + 1.0f));
        }
    }
};

// K_1/3, K_2/3 and IntK_1/3 at x < 1/2, each divided by pi/sqrt3
__device__ __forceinline__ void bessel_small32(float x, float &k13, float &k23, float &ik)
{
    const float h = 0.5f * x, lh = log_r(h);
    float sm2, jm2, sm1, jm1, sp1, jp1, sp2, jp2;
    SmallSeries<-2>::sum(h, lh, 1.0f / 2.678938534707747f, sm2, jm2);      // 1 / Gamma(1/3)
    SmallSeries<-1>::sum(h, lh, 1.0f / 1.3541179394264005f, sm1, jm1);     // 1 / Gamma(2/3)
    SmallSeries<1>::sum(h, lh, 1.0f / 0.8929795115692492f, sp1, jp1);      // 1 / Gamma(4/3)
    SmallSeries<2>::sum(h, lh, 1.0f / 0.9027452929509336f, sp2, jp2);      // 1 / Gamma(5/3)
    k13 = sm1 - sp1;
    k23 = sm2 - sp2;
    ik = 1.0f - (jm1 - jp1);
}

__device__ __forceinline__ void bessel_ratios_small32(float x, float &K1, float &I)
{
    float k13, k23, ik;
    bessel_small32(x, k13, k23, ik);
    K1 = k13 / k23;
    I = ik / k23;
}

template <> __device__ __forceinline__ void bessel_ratios<float>(double xd, const void *nodes, float &K1, float &I)
{
    const float x = fmaxf((float)xd, 1e-30f);
    if (x < 0.5f) {
        bessel_ratios_small32(x, K1, I);
        return;
    }
    float s13, s23, sik;
    int lvl;
    bessel_sums32(x, nodes, s13, s23, sik, lvl);
    K1 = s13 / s23;       // the step h cancels in the ratios
    I = sik / s23;
}

// K_1/3, K_2/3 and IntK_1/3 at x themselves (the rejection step needs the spectrum's size)
template <class R> __device__ __forceinline__ void bessel_abs(double x, const void *nodes, R &K13, R &K23, R &IK);

template <> __device__ __forceinline__ void bessel_abs<double>(double x, const void *nodes, double &K13, double &K23,
                                                               double &IK)
{
    if (x < 1.0) {
        constexpr double c = 1.813799364234217851;  // pi / sqrt3
        bessel_small64(fmax(x, 1e-300), K13, K23, IK);
        K13 *= c;
        K23 *= c;
        IK *= c;
        return;
    }
    const Bessel3 b = bessel3_scaled(x, (const double *)nodes);
    const double e = x < 700.0 ? exp(-x) : 0.0;
    K13 = b.k13 * e;
    K23 = b.k23 * e;
    IK = b.ik * e;
}

template <> __device__ __forceinline__ void bessel_abs<float>(double xd, const void *nodes, float &K13, float &K23,
                                                              float &IK)
{
    const float x = fmaxf((float)xd, 1e-30f);
    if (x < 0.5f) {
        constexpr float c = 1.8137993642342178f;    // pi / sqrt3
        bessel_small32(x, K13, K23, IK);
        K13 *= c;
        K23 *= c;
        IK *= c;
        return;
    }
    float s13, s23, sik;
    int lvl;
    bessel_sums32(x, nodes, s13, s23, sik, lvl);
    const float h = (float)(lvl == 0 ? kBn32H[0] : (lvl == 1 ? kBn32H[1] : kBn32H[2]));
    const float f = h * exp_r(-x);
    K13 = s13 * f;
    K23 = s23 * f;
    IK = sik * f;
}

// ------------------------------------------------------------------ fields
struct FieldDev {
    int kind;
    double E0[3], B0[3];
    double a0, phase_len;
    double inv_phase_len;      // 1 / phase_len (0 without envelope)
    const float *g[6];         // grid: Ex, Ey, Ez, Bx, By, Bz node arrays [ny][nx]
    const float4 *gn;          // or NULL: the same nodes interleaved, two float4 per node
                               // (Ex, Ey, Ez, Bx), (By, Bz, 0, 0), so a corner is one 32-byte read
    int nx, ny;
    double gx0, gy0, inv_dx, inv_dy, inv_nx, inv_ny;
};

// Bilinear interpolation on the periodic grid: cell index and fractions from FP64 coordinates
// (the index wraps with an FP64 floor, exact for |index| < 2^52), weights in R.
template <class R> __device__ __forceinline__ void add_grid(const FieldDev &f, double x, double y, V3<R> &E, V3<R> &B)
{
    const double u = (x - f.gx0) * f.inv_dx, v = (y - f.gy0) * f.inv_dy;
    const double fu = floor(u), fv = floor(v);
    const R ax = (R)(u - fu), ay = (R)(v - fv);
    int i0 = (int)(fu - (double)f.nx * floor(fu * f.inv_nx));
    int j0 = (int)(fv - (double)f.ny * floor(fv * f.inv_ny));
    i0 = i0 >= f.nx ? i0 - f.nx : (i0 < 0 ? i0 + f.nx : i0);
    j0 = j0 >= f.ny ? j0 - f.ny : (j0 < 0 ? j0 + f.ny : j0);
    const int i1 = i0 + 1 == f.nx ? 0 : i0 + 1, j1 = j0 + 1 == f.ny ? 0 : j0 + 1;
    const int64_t a = (int64_t)j0 * f.nx, b = (int64_t)j1 * f.nx;
    const R w00 = ((R)1 - ax) * ((R)1 - ay), w10 = ax * ((R)1 - ay), w01 = ((R)1 - ax) * ay, w11 = ax * ay;
    R val[6];
    if (f.gn) {
        // the same sums over the interleaved copy (same values, same order: equal bit for bit)
        const float4 *q = f.gn;
        const float4 c00 = q[2 * (a + i0)], c10 = q[2 * (a + i1)], c01 = q[2 * (b + i0)], c11 = q[2 * (b + i1)];
        const float4 d00 = q[2 * (a + i0) + 1], d10 = q[2 * (a + i1) + 1], d01 = q[2 * (b + i0) + 1],
                     d11 = q[2 * (b + i1) + 1];
        val[0] = w00 * (R)c00.x + w10 * (R)c10.x + w01 * (R)c01.x + w11 * (R)c11.x;
        val[1] = w00 * (R)c00.y + w10 * (R)c10.y + w01 * (R)c01.y + w11 * (R)c11.y;
        val[2] = w00 * (R)c00.z + w10 * (R)c10.z + w01 * (R)c01.z + w11 * (R)c11.z;
        val[3] = w00 * (R)c00.w + w10 * (R)c10.w + w01 * (R)c01.w + w11 * (R)c11.w;
        val[4] = w00 * (R)d00.x + w10 * (R)d10.x + w01 * (R)d01.x + w11 * (R)d11.x;
        val[5] = w00 * (R)d00.y + w10 * (R)d10.y + w01 * (R)d01.y + w11 * (R)d11.y;
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float *g = f.g[c];
            val[c] = w00 * (R)g[a + i0] + w10 * (R)g[a + i1] + w01 * (R)g[b + i0] + w11 * (R)g[b + i1];
        }
    }
    E.x += val[0]; E.y += val[1]; E.z += val[2];
    B.x += val[3]; B.y += val[4]; B.z += val[5];
}

// E and B at position (x, y) (the plane wave depends on x only, the grid on x and y) and time t.
// Field-model variants of the kernels (each keeps only the registers its models need):
// kFldPlain: uniform and plane wave; kFldRotating: also the rotating field; kFldGeneral: also the
// grid (and, in the lepton pass, the field-dependent g).
enum : int { kFldPlain = 0, kFldRotating = 1, kFldGeneral = 2 };

template <class R, int FLD> struct FieldEval;

template <int FLD> struct FieldEval<double, FLD> {
static __device__ __forceinline__ void eval(const FieldDev &f, double x0, double y0, double t, V3<double> &E,
                                            V3<double> &B)
{
    E = {f.E0[0], f.E0[1], f.E0[2]};
    B = {f.B0[0], f.B0[1], f.B0[2]};
    if (f.kind == 1) {
        const double phi = t + x0;
        double g = 1.0;
        if (f.phase_len > 0.0) {
            if (phi < 0.0 || phi > f.phase_len) return;      // outside the pulse
            const double sn = sin(kPi * phi * f.inv_phase_len);
            g = sn * sn;
        }
        const double ey = f.a0 * g * cos(phi);
        E.y += ey;
        B.z -= ey;
    } else if (FLD >= kFldRotating && f.kind == 3) {
        E.x += f.a0 * cos(t);
        E.y += f.a0 * sin(t);
    } else if (FLD == kFldGeneral && f.kind == 2) {
        add_grid<double>(f, x0, y0, E, B);
    }
}
};

// single precision: the phase is formed and reduced to revolutions in FP64; the sine and
// cosine of the reduced argument use the hardware instructions (|argument| <= 1 revolution)
template <int FLD> struct FieldEval<float, FLD> {
static __device__ __forceinline__ void eval(const FieldDev &f, double x0, double y0, double t, V3<float> &E,
                                            V3<float> &B)
{
    E = {(float)f.E0[0], (float)f.E0[1], (float)f.E0[2]};
    B = {(float)f.B0[0], (float)f.B0[1], (float)f.B0[2]};
    if (f.kind == 1) {
        const double phi = t + x0;
        float g = 1.0f;
        if (f.phase_len > 0.0) {
            if (phi < 0.0 || phi > f.phase_len) return;
            const float a = (float)(phi * f.inv_phase_len);          // in [0, 1]: half a revolution of sin(pi a)
            const float sn = __builtin_amdgcn_sinf(0.5f * a);         // sin(2 pi r), r in revolutions
            g = sn * sn;
        }
        const double rev = phi * (0.5 / kPi);
        const float red = (float)(rev - rint(rev));                    // in [-1/2, 1/2] revolutions
        const float ey = (float)f.a0 * g * __builtin_amdgcn_cosf(red);
        E.y += ey;
        B.z -= ey;
    } else if (FLD >= kFldRotating && f.kind == 3) {
        const double rev = t * (0.5 / kPi);
        const float red = (float)(rev - rint(rev));
        E.x += (float)f.a0 * __builtin_amdgcn_cosf(red);
        E.y += (float)f.a0 * __builtin_amdgcn_sinf(red);
    } else if (FLD == kFldGeneral && f.kind == 2) {
        add_grid<float>(f, x0, y0, E, B);
    }
}
};

// FLD: the field-model variant (kFldPlain, kFldRotating, kFldGeneral)
template <class R, int FLD = kFldGeneral>
__device__ __forceinline__ void eval_fields(const FieldDev &f, double x0, double y0, double t, V3<R> &E, V3<R> &B)
{
    FieldEval<R, FLD>::eval(f, x0, y0, t, E, B);
}

// ------------------------------------------------------------------ push (Boris + T-BMT)
// Cayley rotation v <- v + (v + v x t) x 2t/(1+t^2): exact rotation by 2 atan|t| about t.
template <class R> __device__ __forceinline__ V3<R> cayley(V3<R> v, V3<R> t)
{
    const R f = (R)2 / ((R)1 + dot(t, t));
    const V3<R> vp = v + cross(v, t);
    return v + cross(vp, f * t);
}

// ------------------------------------------------------------------ table interpolation
// 4-point Lagrange weights on nodes v0 + i h, i = 0..n-1 (one-sided at the ends).
template <class R> __device__ __forceinline__ int lagrange4(R v, R v0, R h, int n, R L[4])
{
    R s = (v - v0) / h;
    s = s < (R)0 ? (R)0 : s;
    s = s > (R)(n - 1) ? (R)(n - 1) : s;
    int i = (int)floor(s) - 1;
    i = i < 0 ? 0 : (i > n - 4 ? n - 4 : i);
    const R t = s - (R)i;
    const R a = t - (R)1, b = t - (R)2, c = t - (R)3;
    L[0] = -(a * b * c) / (R)6;
    L[1] = (t * b * c) / (R)2;
    L[2] = -(t * a * c) / (R)2;
    L[3] = (t * a * b) / (R)6;
    return i;
}

// a(chi)/a(0) from the table: 4-point Lagrange in ln chi of its logarithm; 1 below the first
// node (chi < 1e-7), the chi^(-2/3) law from the last node above chi = 1e4.
template <class R> __device__ __forceinline__ R gfac_ratio(const R *lng, R chi)
{
    if (!(chi > (R)0)) return (R)1;
    const R lc = log_r(chi);
    if (lc < (R)kGfLnChi0) return (R)1;
    const R lnlast = (R)(kGfLnChi0 + (kGfN - 1) * kGfDlnChi);
    if (lc > lnlast) return exp_r(lng[kGfN - 1] - (R)(2.0 / 3.0) * (lc - lnlast));
    R L[4];
    const int i = lagrange4(lc, (R)kGfLnChi0, (R)kGfDlnChi, kGfN, L);
    return exp_r(L[0] * lng[i] + L[1] * lng[i + 1] + L[2] * lng[i + 2] + L[3] * lng[i + 3]);
}

// Boris momentum update with fields at the old position; T-BMT with the standard E-term
// coefficient a + 1/(gamma+1), the Boris mid-step gamma and beta = (u- + u+)/(2 gamma);
// returns the displacement p/gamma dt with the new momentum.  With a g-factor table `lng` the
// anomalous moment is a_e a(chi)/a(0), chi at the mid step (momentum (u- + u+)/2, energy gamma-).
template <class R>
__device__ __forceinline__ V3<R> push(int q, R a_e, V3<R> E, V3<R> B, R dt, bool tbmt, V3<R> &p, V3<R> &s,
                                      const R *lng = nullptr, R eps_r = (R)0)
{
    const R hq = (R)0.5 * (R)q * dt;
    const V3<R> um = p + hq * E;
    const R gm = sqrt_r((R)1 + dot(um, um));
    const V3<R> up = cayley(um, (hq / gm) * B);
    if (tbmt) {
        const V3<R> be = ((R)0.5 / gm) * (um + up);
        const V3<R> bxE = cross(be, E);
        const R bB = dot(be, B);
        if (lng) {
            const V3<R> u = (R)0.5 * (um + up);
            const V3<R> F = gm * E + cross(u, B);
            const R uE = dot(u, E), rad = dot(F, F) - uE * uE;
            a_e *= gfac_ratio<R>(lng, eps_r * sqrt_r(rad > (R)0 ? rad : (R)0));
        }
        const V3<R> Om = (R)(-q) * ((a_e + (R)1 / gm) * B - (a_e * gm / (gm + (R)1) * bB) * be -
                                    (a_e + (R)1 / (gm + (R)1)) * bxE);
        s = cayley(s, ((R)(-0.5) * dt) * Om);
    }
    p = up + hq * E;
    const R g = sqrt_r((R)1 + dot(p, p));
    return (dt / g) * p;
}

// ------------------------------------------------------------------ basis and chi
// chi = eps_r sqrt((p0 E + p x B)^2 - (p.E)^2) in FP64 (p0 = gamma for leptons, |k| for photons);
// khat = p/|p|; eps = unit(sgn (E + v x B) perpendicular to khat), sgn = -q (q = -1 for e-
// and photons, +1 for e+); beta = khat x eps (right-handed triad).  chi = 0 when the
// transverse force vanishes.
template <class R> struct Basis { V3<R> e, b, k; };

template <class R>
__device__ __forceinline__ double basis_chi(int charge, double eps_r, V3<R> p, double p0, V3<R> E, V3<R> B, Basis<R> &out)
{
    // FP64: the cancellation-prone F = p0 E + p x B and the invariant (p0 E + p x B)^2 - (p.E)^2
    const V3<double> pd = cvt<double>(p), Ed = cvt<double>(E), Bd = cvt<double>(B);
    const V3<double> F = p0 * Ed + cross(pd, Bd);
    const double pE = dot(pd, Ed);
    const double rad = dot(F, F) - pE * pE;
    // directions in R: khat, the part of F transverse to khat, eps, beta
    out.k = rsqrt_r(dot(p, p)) * p;
    const V3<double> kd = cvt<double>(out.k);
    const V3<double> Ft = F - dot(F, kd) * kd;
    const double ft2 = dot(Ft, Ft);
    if (!(ft2 > 0.0)) {
        out.e = {0, 0, 0};
        out.b = {0, 0, 0};
        return 0.0;
    }
    const R sgn = charge > 0 ? (R)-1 : (R)1;
    out.e = (sgn * rsqrt_r((R)ft2)) * cvt<R>(Ft);
    out.b = cross(out.k, out.e);
    return eps_r * (double)sqrt_r((R)(rad > 0.0 ? rad : 0.0));
}

// ------------------------------------------------------------------ P-vector <-> Stokes
// Encode xi (emission-basis Stokes, xi3 linear along eps, xi2 circular) as P = d [sqrt(1-xi2^2)
// (cos dth eps + sin dth beta) + xi2 k], dth = atan2(xi1, xi3)/2, for unit xi scaled by d = |xi|.
template <class R> __device__ __forceinline__ V3<R> stokes_to_P(R x1, R x2, R x3, const Basis<R> &bs)
{
    const R d = sqrt_r(x1 * x1 + x2 * x2 + x3 * x3);
    if (!(d > (R)0)) return {0, 0, 0};
    // transverse part: length sqrt(x1^2 + x3^2), at half the Stokes angle 2 dth = atan2(x1, x3),
    // from the half-angle formulas (cos dth >= 0 on the principal branch); the cancelling
    // square root is avoided by dividing by the larger of the two
    const R tr = sqrt_r(x1 * x1 + x3 * x3);
    R c = (R)1, sn = (R)0;
    if (tr > (R)0) {
        const R cth = x3 / tr, sth = x1 / tr;
        if (cth >= (R)0) {
            c = sqrt_r((R)0.5 * ((R)1 + cth));
            sn = sth / ((R)2 * c);
        } else {
            sn = sqrt_r((R)0.5 * ((R)1 - cth));
            sn = sth < (R)0 ? -sn : sn;
            c = sth / ((R)2 * sn);
        }
    }
    return (tr * c) * bs.e + (tr * sn) * bs.b + x2 * bs.k;
}

// A P-vector with a NaN or infinity decodes as unpolarized (all Stokes parameters 0); the
// return value is false then.
template <class R> __device__ __forceinline__ bool P_to_stokes(V3<R> P, const Basis<R> &bs, R &x1, R &x2, R &x3)
{
    const R d2 = dot(P, P);
    const bool fin = __builtin_isfinite(d2);
    if (!(d2 > (R)0) || !fin) { x1 = x2 = x3 = 0; return fin; }
    const R d = sqrt_r(d2), id = (R)1 / d;
    const R p1 = dot(P, bs.e) * id, p2 = dot(P, bs.b) * id, pk = dot(P, bs.k) * id;
    const R rr = p1 * p1 + p2 * p2;
    if (rr > (R)0) {
        const R ir = rsqrt_r(rr);
        x1 = d * (R)2 * p1 * p2 * ir;
        x3 = d * (p1 * p1 - p2 * p2) * ir;
    } else {
        x1 = x3 = 0;
    }
    x2 = d * pk;
    return true;
}

// ------------------------------------------------------------------ spectra
// Bessel values normalized by K_2/3 (ratios are all the collapse needs):
// K1 = K_1/3/K_2/3, I = IntK_1/3/K_2/3 at u' (NLC) or u~' (NBW).
template <class R> struct SpecPt { R lam, oml, u, K1, I; };

// NLC (appendix, Bessel forms), a = s_i and b = s_f in (eps, beta, k) components.
// w = -I + kappa K2 + lam a_beta K1; g = u K1 beta + (-I + 2 K2) a + lam u (-I + K2) a_k k.
template <class R> __device__ __forceinline__ R nlc_w(const SpecPt<R> &q, R ab)
{
    const R kap = (R)1 / q.oml + q.oml;
    return -q.I + kap + q.lam * ab * q.K1;
}
template <class R> __device__ __forceinline__ V3<R> nlc_g(const SpecPt<R> &q, V3<R> a)
{
    const R c = -q.I + (R)2;
    return {c * a.x, q.u * q.K1 + c * a.y, c * a.z + q.lam * q.u * (-q.I + (R)1) * a.z};
}
// F = (F1, F2, F3) for initial a and final b (diagonal, circular, linear-along-eps components)
template <class R> __device__ __forceinline__ V3<R> nlc_F(const SpecPt<R> &q, V3<R> a, V3<R> b)
{
    const R lam = q.lam, u = q.u, I = q.I, K1 = q.K1;
    const R kap = (R)1 / q.oml + q.oml, kapt = (R)1 / q.oml - q.oml;
    const R ck = b.x * a.y - b.y * a.x;           // (s_f x s_i) . k
    const R ce = b.y * a.z - b.z * a.y;           // (s_f x s_i) . eps
    const R hlu = (R)0.5 * lam * u;
    V3<R> F;
    F.x = -K1 * (u * a.x + lam * b.x) - hlu * I * (b.x * a.y + b.y * a.x) + (R)0.5 * kapt * ck;
    F.y = (R)0.5 * kapt * K1 * ce - (lam * I - kapt) * a.z - (u * I - kapt) * b.z + hlu * K1 * (b.z * a.y + b.y * a.z);
    F.z = (R)1 + (u * a.y + lam * b.y) * K1 - hlu * I * (b.x * a.x - b.y * a.y) + (R)0.5 * kap * dot(b, a) - hlu * b.z * a.z;
    return F;
}

// NBW (appendix, Bessel forms) with the plus sign of the last term of G3 (as in its Airy form);
// e = s_e, p = s_p components; returns G0 and G = (G1, G2, G3).
template <class R> __device__ __forceinline__ R nbw_G(const SpecPt<R> &q, V3<R> e, V3<R> p, V3<R> &G)
{
    const R lam = q.lam, oml = q.oml, I = q.I, K1 = q.K1;
    const R il = (R)1 / lam, io = (R)1 / oml;
    const R ut = il + io, rho = oml * il + lam * io, rhot = oml * il - lam * io;
    const R pe = dot(p, e);
    const R ck = p.x * e.y - p.y * e.x;           // (s_p x s_e) . k
    const R ce = p.y * e.z - p.z * e.y;           // (s_p x s_e) . eps
    const R G0 = I + rho + e.y * K1 * io - p.y * K1 * il + (I - (R)2) * pe + (rho * I - (rho - (R)2)) * p.z * e.z;
    G.x = K1 * (e.x * il - p.x * io) - (R)0.5 * ut * I * (p.x * e.y + p.y * e.x) + (R)0.5 * rhot * ck;
    G.y = -(R)0.5 * ut * K1 * ce + (I * io + rhot) * e.z + (I * il - rhot) * p.z - (R)0.5 * rhot * K1 * (p.z * e.y + p.y * e.z);
    G.z = -(R)1 + (-e.y * il + p.y * io) * K1 - (R)0.5 * ut * I * (p.x * e.x - p.y * e.y) + (R)0.5 * rho * pe +
          ((R)1 - (R)0.5 * rho) * p.z * e.z;
    return G0;
}
// w0 and the spin vectors j_e, j_p (marginals of G over the other lepton's spin)
template <class R> __device__ __forceinline__ R nbw_j(const SpecPt<R> &q, V3<R> xi, V3<R> &je, V3<R> &jp)
{
    const R lam = q.lam, oml = q.oml, I = q.I, K1 = q.K1;
    const R il = (R)1 / lam, io = (R)1 / oml;
    const R rho = oml * il + lam * io, rhot = oml * il - lam * io;
    je = {xi.x * K1 * il, (io - xi.z * il) * K1, xi.y * (I * io + rhot)};
    jp = {-xi.x * K1 * io, (-il + xi.z * io) * K1, xi.y * (I * il - rhot)};
    return I + rho - xi.z;
}

}  // namespace qs
