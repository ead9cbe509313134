// qs_pass.hpp -- device views of the particle sets, the decision parts of the two channels and
// the per-particle bodies of the streaming and processing passes, shared by the per-species
// entry points (qs_step.hip) and the merged multi-instance step (qs_plan.hip).
#pragma once
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "qs_internal.hpp"

namespace qs {

constexpr int kBlock = 256;
constexpr int kMaxGrid = 2048;                               // 256 CUs x 8 resident blocks

template <class R> struct LepDev {
    int64_t cap;
    int64_t *count;
    int species;
    R *x[3], *p[3], *s[3];
    double *tau, *tau_t;       // optical depth and its target (FP64 in both precisions), or NULL
    uint8_t *msub;             // log2 of the sub-steps of this time step (sub-cycling only)
    uint32_t *sub;             // merged step with sub-cycling: per slot of a lepton with a photon this
                               // step, (log2 of its sub-steps << 16) | (bit r: a photon in round r);
                               // NULL: no sub-cycling
    R *stage;                  // ... and per slot kSubRounds x (k, P-vector) of the photons its
                               // sub-steps made, for the processing pass to place
};

template <class R> struct PhoDev {
    int64_t cap;
    int64_t *count, *count_prev;
    R *x[3], *k[3], *P[3];
    uint64_t *id;
};

struct StepDev {
    double t, dt, a_e, eps_r, chi_e_min, chi_e_max, chi_g_min, chi_g_max, k_retire;
    double Kc;                 // alpha / (sqrt3 pi eps_r): rate prefactor times gamma (or |k|)
    int64_t step;
    uint64_t seed;
    uint32_t flags;
    int sub_round;             // sub-cycling round (Philox channels + 16 sub_round; photon ids)
    const int64_t *clock;      // optional device step offset (replayable launches)
};

// step index and time of this launch: params.step + *clock and params.t + *clock dt
__device__ __forceinline__ StepDev localize(StepDev S)
{
    if (S.clock) {
        const int64_t off = *S.clock;
        S.step += off;
        S.t += (double)off * S.dt;
    }
    return S;
}

enum { C_EMIT = 0, C_PAIR, C_PROB, C_CHI, C_NORM, C_OVER, C_RETIRED, C_LSTEP, C_GSTEP, C_GQED, C_NONFIN, kNCtr };

struct WS {
    uint64_t *mask;      // [2][nchunks]: transition, branch (up / plus)
    uint32_t *bcnt;      // [kMaxGrid]: transitions per block of the streaming pass
    int64_t *book;       // [8]: base0, total, base1, n_fit, n processed, block range
    uint32_t *bctr;      // [kMaxGrid][kNCtr]: per-block counts of the streaming pass
    uint32_t *idx;       // [max particles]
    uint8_t *msub;       // [max particles]: log2 of each lepton's sub-steps (sub-cycling)
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline WS carve(void *ws, int64_t cap, int64_t *nchunks_out)
{
    const int64_t nch = cdiv(cap > 0 ? cap : 1, 64);
    char *b = (char *)ws;
    WS w;
    w.mask = (uint64_t *)b; b += align256(sizeof(uint64_t) * 2 * nch);
    w.bcnt = (uint32_t *)b; b += align256(sizeof(uint32_t) * kMaxGrid);
    w.book = (int64_t *)b;  b += align256(sizeof(int64_t) * 8);
    w.bctr = (uint32_t *)b; b += align256(sizeof(uint32_t) * kMaxGrid * kNCtr);
    w.idx = (uint32_t *)b; b += align256(sizeof(uint32_t) * (cap > 0 ? cap : 1));
    w.msub = (uint8_t *)b;
    *nchunks_out = nch;
    return w;
}

// ------------------------------------------------------------------ device helpers
template <class R> __device__ __forceinline__ const R *rate_src(const TablesDev &T);
template <> __device__ __forceinline__ const double *rate_src<double>(const TablesDev &T) { return T.lnrate; }
template <> __device__ __forceinline__ const float *rate_src<float>(const TablesDev &T) { return T.lnrate32; }

// the g-factor table of the push when the step asks for the field-dependent anomalous moment
// (compiled into the general variants only), else NULL
template <class R, int FLD> __device__ __forceinline__ const R *gfac_src(const TablesDev &T, uint32_t flags)
{
    if (FLD != kFldGeneral || !(flags & F_GCHI)) return nullptr;
    if constexpr (sizeof(R) == 8) return (const R *)T.lng;
    else return (const R *)T.lng32;
}

template <class R> __device__ __forceinline__ const void *bn_of(const TablesDev &T)
{
    return sizeof(R) == 8 ? (const void *)T.bn64 : (const void *)T.bn32;
}

// stage the two rate rows of one process (NLC: channels 0,1; NBW: 2,3) into LDS
template <class R> __device__ __forceinline__ int stage_rates(const TablesDev &T, int grp, R *lds)
{
    const int n = T.n_chi[grp];
    const R *src = rate_src<R>(T) + T.off_rate[2 * grp];
    for (int j = threadIdx.x; j < 2 * n; j += blockDim.x) lds[j] = src[j];
    __syncthreads();
    return n;
}

template <class R> __device__ __forceinline__ R rate_lookup(const R *row, R lnchi, R x0, R h, int n)
{
    R L[4];
    const int i = lagrange4(lnchi, x0, h, n, L);
    return L[0] * row[i] + L[1] * row[i + 1] + L[2] * row[i + 2] + L[3] * row[i + 3];
}

// inverse CDF (FP64 island): nu at (ln chi, rho) for channel ch
__device__ __forceinline__ double icdf_nu(const TablesDev &T, int ch, double lnchi, double rho)
{
    const int grp = ch < 2 ? 0 : 1;
    double Lc[4], Lr[4];
    const int i0 = lagrange4(lnchi, T.lnchi0[grp], T.dlnchi[grp], T.n_chi[grp], Lc);
    const int j0 = lagrange4(rho, T.rho0, T.drho, T.n_rho, Lr);
    const double *base = T.nu + T.off_nu[ch] + (int64_t)i0 * T.n_rho + j0;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double *r = base + (int64_t)a * T.n_rho;
        acc += Lc[a] * (Lr[0] * r[0] + Lr[1] * r[1] + Lr[2] * r[2] + Lr[3] * r[3]);
    }
    return acc;
}

template <class R> __device__ __forceinline__ V3<R> ld3(R *const a[3], int64_t i)
{
    return {a[0][i], a[1][i], a[2][i]};
}
template <class R> __device__ __forceinline__ void st3(R *const a[3], int64_t i, V3<R> v)
{
    a[0][i] = v.x;
    a[1][i] = v.y;
    a[2][i] = v.z;
}
template <class R> __device__ __forceinline__ V3<R> ldx(R *const a[3], int64_t i)
{
    return {a[0] ? a[0][i] : (R)0, a[1] ? a[1][i] : (R)0, a[2] ? a[2][i] : (R)0};
}
template <class R> __device__ __forceinline__ void stx(R *const a[3], int64_t i, V3<R> v)
{
    if (a[0]) a[0][i] = v.x;
    if (a[1]) a[1][i] = v.y;
    if (a[2]) a[2][i] = v.z;
}

// Contiguous partition of [0, n) over the grid of a streaming pass: block b owns
// [b B, (b+1) B) with B a multiple of 64, so each 64-particle mask word belongs to one block and
// the per-block transition counts are the scan input in particle order.
__host__ __device__ __forceinline__ int64_t block_len(int64_t n, int64_t nblk)
{
    return ((cdiv(n, nblk > 0 ? nblk : 1) + 63) / 64) * 64;
}

// Block totals of the per-thread counts v[0..kNCtr) and of the transition count v[kNCtr]:
// on return tot[c] holds the block's sum (shared, valid after the barrier inside).
__device__ __forceinline__ void block_sum(unsigned (&v)[kNCtr + 1], unsigned (&tot)[kNCtr + 1])
{
    __shared__ unsigned red[kBlock / 64][kNCtr + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c <= kNCtr; ++c) {
        unsigned t = v[c];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) red[wid][c] = t;
    }
    __syncthreads();
    if (threadIdx.x <= kNCtr) {
        unsigned t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w][threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
}

// Reduce over the block (of kBlock threads, every one of which calls this), one atomic per
// block.  Atomics on one address are performed one after the other: with one per wave, the
// hundreds of waves of a processing launch spent several microseconds queued on the counter.
__device__ __forceinline__ void block_add(unsigned long long *ctr, int slot, unsigned v)
{
    __shared__ unsigned part[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += part[w];
        if (t) atomicAdd(ctr + slot, (unsigned long long)t);
    }
}

// Non-finite inputs (NaN or infinity in a particle's state or in the fields it sees) are not
// stepped: such a lepton keeps its stored state, such a photon becomes a dead slot, and each is
// counted in n_nonfinite; the step writes no NaN of its own.  Analytic field models with finite
// parameters (checked on the host) give finite fields, so only interpolated grid values are
// checked per particle (the general field variant).
// One test on a sum: an infinite or NaN component makes the sum non-finite, and a finite sum of
// finite components needs magnitudes beyond a ninth of the type's range to overflow (which then
// counts as non-finite too).
template <class R> __device__ __forceinline__ bool finite_sum(R a) { return __builtin_isfinite(a); }
template <class R> __device__ __forceinline__ bool finite3(V3<R> v) { return finite_sum(v.x + v.y + v.z); }

template <class R> __device__ __forceinline__ bool zero_field(V3<R> E, V3<R> B)
{
    return E.x == (R)0 && E.y == (R)0 && E.z == (R)0 && B.x == (R)0 && B.y == (R)0 && B.z == (R)0;
}

// ------------------------------------------------------------------ lepton QED: decision part
// Everything up to and including the emit / no-emit decision (NLC section: chi_e, beta, the
// spin-weighted rate W = W_up (1+s.beta)/2 + W_down (1-s.beta)/2, the draw r1 < W dt).
template <class R> struct LDecide {
    double chi;        // clamped for lookups
    Basis<R> bs;
    R Ce, Wdn, Wup, a, P, r1, r2;
    bool active;       // chi >= chi_min
    bool clamped_chi;
};

// The part that depends on the momentum and the fields only: chi_e, the emission basis and the
// two rates (d.active false outside the pulse or below chi_min).  A sub-cycled lepton keeps it
// through its sub-steps until an emission changes its momentum.
template <class R>
__device__ __forceinline__ void lepton_geom(const StepDev &S, const TablesDev &T, const R *lds, int species, V3<R> p,
                                            V3<R> E, V3<R> B, LDecide<R> &d)
{
    d.clamped_chi = false;
    if (zero_field(E, B)) {           // outside the pulse: no QED, skip the FP64 island
        d.active = false;
        d.chi = 0.0;
        return;
    }
    const int q = species == 0 ? -1 : 1;
    const double gam = sqrt(1.0 + dot(cvt<double>(p), cvt<double>(p)));
    d.chi = basis_chi(q, S.eps_r, p, gam, E, B, d.bs);
    d.active = d.chi >= S.chi_e_min;
    d.clamped_chi = d.chi > S.chi_e_max;
    if (d.clamped_chi) d.chi = S.chi_e_max;
    if (!d.active) return;
    const int n = T.n_chi[0];
    const R lnchi = log_r((R)d.chi);
    const R x0 = (R)T.lnchi0[0], h = (R)T.dlnchi[0];
    const R Ce = ratio_r<R>(S.Kc, gam);
    d.Ce = Ce;
    d.Wdn = Ce * exp_r(rate_lookup(lds, lnchi, x0, h, n));
    d.Wup = Ce * exp_r(rate_lookup(lds + n, lnchi, x0, h, n));
}

// The part that depends on the spin and the draw of this step (and sub-cycling round): the
// branch weights a = W_down (1 - s.beta)/2 dt, P = a + W_up (1 + s.beta)/2 dt and r1, r2.
template <class R>
__device__ __forceinline__ void lepton_draw(const StepDev &S, int species, int64_t index, V3<R> s, LDecide<R> &d)
{
    if (!d.active) return;
    const R sb = dot(s, d.bs.b);
    const R dt = (R)S.dt;
    d.a = d.Wdn * (R)0.5 * ((R)1 - sb) * dt;
    const R b = d.Wup * (R)0.5 * ((R)1 + sb) * dt;
    d.P = d.a + b;
    const uint4 w = philox_block(S.seed, lepton_id(species, index), S.step, 16u * (uint32_t)S.sub_round);
    Unif<R>::two(w, d.r1, d.r2);
}

template <class R>
__device__ __forceinline__ LDecide<R> lepton_decide(const StepDev &S, const TablesDev &T, const R *lds, int species,
                                                    int64_t index, V3<R> p, V3<R> s, V3<R> E, V3<R> B)
{
    LDecide<R> d;
    lepton_geom<R>(S, T, lds, species, p, E, B, d);
    lepton_draw<R>(S, species, index, s, d);
    return d;
}

// ------------------------------------------------------------------ photons: decision part
template <class R> struct PDecide {
    double chi;
    Basis<R> bs;
    R Wm, Wp, a, P, r1, r2, x1, x2, x3;
    bool active, clamped_chi;
    bool nonfinite;    // the P-vector is not finite: the photon is stepped as unpolarized
};

// PIN: the draw's key pinned to scalar registers (philox4x32_10), in the photon pass's loop only
template <class R, bool PIN = false>
__device__ __forceinline__ PDecide<R> photon_decide(const StepDev &S, const TablesDev &T, const R *lds, uint64_t id,
                                                    V3<R> k, double k0, V3<R> P, V3<R> E, V3<R> B)
{
    PDecide<R> d;
    d.clamped_chi = false;
    d.nonfinite = false;
    if (zero_field(E, B)) {
        d.active = false;
        d.chi = 0.0;
        return d;
    }
    d.chi = basis_chi(0, S.eps_r, k, k0, E, B, d.bs);
    d.active = d.chi >= S.chi_g_min;
    d.clamped_chi = d.chi > S.chi_g_max;
    if (d.clamped_chi) d.chi = S.chi_g_max;
    if (!d.active) return d;
    const int n = T.n_chi[1];
    const R lnchi = log_r((R)d.chi);
    const R x0 = (R)T.lnchi0[1], h = (R)T.dlnchi[1];
    const R Cg = ratio_r<R>(S.Kc, k0);
    const R erb = (R)kErber / (R)d.chi;                  // the rows hold ln W + 8/(3 chi)
    d.Wm = Cg * exp_r(rate_lookup(lds, lnchi, x0, h, n) - erb);
    d.Wp = Cg * exp_r(rate_lookup(lds + n, lnchi, x0, h, n) - erb);
    d.nonfinite = !P_to_stokes(P, d.bs, d.x1, d.x2, d.x3);
    const R dt = (R)S.dt;
    d.a = d.Wm * (R)0.5 * ((R)1 - d.x3) * dt;
    const R b = d.Wp * (R)0.5 * ((R)1 + d.x3) * dt;
    d.P = d.a + b;
    Unif<R>::two(philox_block<PIN>(S.seed, id, S.step, 2u), d.r1, d.r2);
    return d;
}

// Photons whose FP32 bound eps_r k0 (|E| + |B|) >= |F_perp| eps_r = chi cannot reach chi_min skip
// the QED part.  The bound carries a relative margin far above FP32 rounding, so every photon
// with chi >= chi_min (FP64) is a candidate.
template <class R> __device__ __forceinline__ bool photon_candidate(const StepDev &S, R k0, V3<R> E, V3<R> B)
{
    const R bound = (R)S.eps_r * k0 * (sqrt_r(dot(E, E)) + sqrt_r(dot(B, B)));
    return bound * (R)1.001 >= (R)S.chi_g_min;
}


// ------------------------------------------------------------------ per-particle work
// The bodies below are shared by the per-species entry points and the merged step.

// The emission of a lepton whose decision d (taken at its state p, s) chose the spin branch `up`
// (NLC section): lambda from the selected inverse CDF (or the accepted rejection candidate), the
// photon's momentum k and P-vector from the Stokes collapse, and the lepton's recoil and spin
// collapse, in p and s.  nu_in: nu from the learned inverse CDF instead of the table.  PHOTON =
// false leaves out the photon's Stokes collapse and P-vector (k and Pv unset), which the lepton's
// own state does not depend on.
template <class R, bool PHOTON = true>
__device__ __forceinline__ void emit_core(const StepDev &S, const TablesDev &T, const LDecide<R> &d, int species,
                                          int64_t i, bool up, V3<R> &p, V3<R> &s, V3<R> &k, V3<R> &Pv,
                                          const float *nu_in = nullptr)
{
    const double r2 = (double)d.r2;
    const double rho = log(r2) - log1p(-r2);
    double lam_d, oml_d;
    if (S.flags & F_REJECT) {                     // the candidate the streaming pass accepted
        const double r1 = (double)d.r1;
        lam_d = r1 * r1 * r1;
        oml_d = (1.0 - r1) * (1.0 + r1 + r1 * r1);
    } else {
        const double nu = nu_in ? (double)*nu_in : icdf_nu(T, up ? 1 : 0, log(d.chi), rho);
        lam_d = 1.0 / (1.0 + exp(-nu));
        oml_d = 1.0 / (1.0 + exp(nu));
    }
    const double u_d = lam_d / oml_d;
    k = (R)lam_d * p;
    R r3, r4;
    Unif<R>::two(philox_block(S.seed, lepton_id(species, i), S.step, 1u + 16u * (uint32_t)S.sub_round), r3, r4);
    SpecPt<R> qp;
    qp.lam = (R)lam_d; qp.oml = (R)oml_d; qp.u = (R)u_d;
    bessel_ratios<R>(2.0 * u_d / (3.0 * d.chi), bn_of<R>(T), qp.K1, qp.I);
    const V3<R> si = {dot(s, d.bs.e), dot(s, d.bs.b), dot(s, d.bs.k)};
    const R w = nlc_w(qp, si.y);
    const V3<R> g = nlc_g(qp, si);
    V3<R> sf = si;
    if (S.flags & F_SPIN) {
        if (S.flags & F_MEAN) sf = ((R)1 / w) * g;
        else {
            const R gn = sqrt_r(dot(g, g));
            const V3<R> Sq = gn > (R)0 ? ((R)1 / gn) * g : v3<R>(0, 1, 0);
            const R thr3 = (w - gn) / ((R)2 * w);
            sf = (r3 < thr3 ? (R)-1 : (R)1) * Sq;
        }
    }
    V3<R> xi = {0, 0, 0};
    if (PHOTON && (S.flags & F_PHOTON_POL)) {
        if (S.flags & F_MEAN) xi = ((R)1 / w) * nlc_F(qp, si, v3<R>(0, 0, 0));
        else {
            const V3<R> Fv = nlc_F(qp, si, sf);
            const R F0 = w + dot(sf, g);
            const R Fn = sqrt_r(dot(Fv, Fv));
            if (Fn > (R)0) {
                const R thr4 = (F0 - Fn) / ((R)2 * F0);
                xi = ((r4 < thr4 ? (R)-1 : (R)1) / Fn) * Fv;
            }
        }
    }
    if (PHOTON) Pv = stokes_to_P(xi.x, xi.y, xi.z, d.bs);
    if (S.flags & F_RECOIL) p = (R)oml_d * p;
    if (S.flags & F_SPIN) s = sf.x * d.bs.e + sf.y * d.bs.b + sf.z * d.bs.k;
}

// The emitted photon into slot `slot`: a dead slot (id 0) below the retirement energy, counted
template <class R>
__device__ __forceinline__ void store_photon(const PhoDev<R> &G, const StepDev &S, int species, int64_t i, int64_t slot,
                                             V3<R> x, V3<R> k, V3<R> Pv, unsigned &c_ret)
{
    if (sqrt(dot(cvt<double>(k), cvt<double>(k))) < S.k_retire) {
        G.id[slot] = 0;
        ++c_ret;
    } else {
        G.id[slot] = photon_id(species, i, S.step, S.sub_round);
        stx(G.x, slot, x);
        st3(G.k, slot, k);
        st3(G.P, slot, Pv);
    }
}

struct LCount {
    unsigned prob = 0, chi = 0, norm = 0, step = 0, trans = 0, nonfin = 0;
    unsigned rnd[kSubRounds] = {};          // merged step with sub-cycling: photons per round
};

// No-transition spin update over dt 2^-msh (non-transition section), renormalized where rounding
// pushed |s| past 1
template <class R>
__device__ __forceinline__ void noemit_spin(const StepDev &S, const LDecide<R> &d, int msh, V3<R> &s, unsigned &norm)
{
    const R dt = ldexp((R)S.dt, -msh);
    const R Wbar = (R)0.5 * (d.Wup + d.Wdn), dW = (R)0.5 * (d.Wup - d.Wdn);
    const R inv = (R)1 / ((R)1 - d.P);
    s = inv * (((R)1 - Wbar * dt) * s - (dW * dt) * d.bs.b);
    const R n2 = dot(s, s);
    if (n2 > (R)1) {
        s = rsqrt_r(n2) * s;
        norm += n2 > (R)1 + norm_count_tol<R>();
    }
}

// One sub-step of a sub-cycled lepton in the merged step (decision-making section): the decision
// d of round S.sub_round (taken at the current p, s) with W dt scaled by 2^-msh (exact), then the
// emission (true; photon in k, Pv; p, s recoiled and collapsed) or the no-transition update over
// dt 2^-msh.  With c, the counts lepton_item keeps (chi clamps, P > 1, renormalizations).
// substep_decide is the part up to the choice (the no-transition update included; true: an
// emission follows), substep_emit the emission with the d it left.
template <class R>
__device__ __forceinline__ bool substep_decide(const StepDev &S, int msh, LDecide<R> &d, V3<R> &s, LCount *c)
{
    if (!d.active) return false;
    d.a = ldexp(d.a, -msh);
    d.P = ldexp(d.P, -msh);
    if (c) c->chi += d.clamped_chi;
    if (d.P <= (R)1 && !(d.r1 < d.P)) {
        unsigned nrm = 0;
        if (S.flags & F_NOEMIT) noemit_spin<R>(S, d, msh, s, nrm);
        if (c) c->norm += nrm;
        return false;
    }
    return true;
}

template <class R, bool PHOTON = true>
__device__ __forceinline__ void substep_emit(const StepDev &S, const TablesDev &T, const LDecide<R> &d, int species,
                                             int64_t i, V3<R> &p, V3<R> &s, V3<R> &k, V3<R> &Pv, LCount *c)
{
    if (c) c->prob += d.P > (R)1;
    const R thr = d.P <= (R)1 ? d.a : d.a / d.P;
    emit_core<R, PHOTON>(S, T, d, species, i, !(d.r1 < thr), p, s, k, Pv);
}

template <class R, bool PHOTON = true>
__device__ __forceinline__ bool lepton_substep(const StepDev &S, const TablesDev &T, int species, int64_t i, int msh,
                                               LDecide<R> d, V3<R> &p, V3<R> &s, V3<R> &k, V3<R> &Pv, LCount *c)
{
    if (!substep_decide<R>(S, msh, d, s, c)) return false;
    substep_emit<R, PHOTON>(S, T, d, species, i, p, s, k, Pv, c);
    return true;
}

// Main pass, one lepton: Boris push and T-BMT rotation with the fields at t, the fields at
// t + dt, chi and the decision (NLC section); a non-emitter gets the no-transition spin update
// (non-transition section).  Stores x, p, s.  DEC: decision variants compiled in (bit 0: the
// optical-depth decision, bit 1: rejection sampling, bit 2: sub-cycling; the variant with none
// needs the fewest registers); the step's flags choose among the compiled ones.
// Sub-cycling (bit 2) runs the QED part in kSubRounds launches (S.sub_round): round 0 pushes and
// sets the lepton's sub-steps 2^k from W_s dt; a lepton takes its sub-steps of dt/2^k in the
// rounds that are multiples of kSubRounds/2^k and leaves its state alone in the others.
template <class R, int DEC, int FLD>
__device__ __forceinline__ void lepton_item(const LepDev<R> &L, const FieldDev &F, const StepDev &S, const TablesDev &T,
                                            const R *lds, int64_t i, V3<R> x, V3<R> p, V3<R> s, bool &emit, bool &up,
                                            LCount &c)
{
    const int q = L.species == 0 ? -1 : 1;
    int msh = 0;                                  // log2 of the sub-steps (sub-cycling)
    if constexpr ((DEC & 4) != 0) {
        if (S.sub_round > 0) {
            msh = L.msub[i];
            if ((S.sub_round & ((kSubRounds >> msh) - 1)) != 0) return;     // not this lepton's round
        } else {
            ++c.step;
            L.msub[i] = 0;
        }
    } else {
        ++c.step;
    }
    // a non-finite lepton is neither pushed nor stepped (stored back as it is); a non-finite grid
    // field at t stops the step there, one at t + dt leaves the push without the QED part
    bool go = finite_sum(x.x + x.y + x.z + p.x + p.y + p.z + s.x + s.y + s.z);
    c.nonfin += !go;
    V3<R> E, B;
    if (go && (S.flags & F_PUSH)) {
        eval_fields<R, FLD>(F, (double)x.x, (double)x.y, S.t, E, B);
        if (FLD == kFldGeneral && !finite_sum(E.x + E.y + E.z + B.x + B.y + B.z)) {
            ++c.nonfin;
            go = false;
        } else {
            x = x + push<R>(q, (R)S.a_e, E, B, (R)S.dt, (S.flags & F_TBMT) != 0, p, s, gfac_src<R, FLD>(T, S.flags),
                            (R)S.eps_r);
        }
    }
    if (go && (S.flags & F_EMIT)) {
        eval_fields<R, FLD>(F, (double)x.x, (double)x.y, S.t + S.dt, E, B);
        if (FLD == kFldGeneral && !finite_sum(E.x + E.y + E.z + B.x + B.y + B.z)) {
            ++c.nonfin;
            go = false;
        }
    }
    if (go && (S.flags & F_EMIT)) {
        LDecide<R> d = lepton_decide<R>(S, T, lds, L.species, i, p, s, E, B);
        if constexpr ((DEC & 8) != 0) {
            // merged step with sub-cycling: a lepton with more than one sub-step is only flagged
            // here (no transition, branch bit set: a combination no decision produces) with its
            // sub-step count; its state after the push is stored below, and the plan's sub-step
            // launch runs its sub-steps
            if (L.sub && d.active) {
                int m = 0;
                while (m < kSubLog2Max && d.P > (R)kSubWdt * (R)(1 << m)) ++m;
                if (m > 0) {
                    L.sub[i] = (unsigned)m << 16;
                    up = true;
                    d.active = false;                 // the plain path below is skipped
                }
            }
        }
        if constexpr ((DEC & 4) != 0) {
            if (d.active) {
                if (S.sub_round == 0) {
                    while (msh < kSubLog2Max && d.P > (R)kSubWdt * (R)(1 << msh)) ++msh;
                    L.msub[i] = (uint8_t)msh;
                }
                d.a = ldexp(d.a, -msh);               // W dt / 2^k, exact
                d.P = ldexp(d.P, -msh);
            }
        }
        if (d.active) {
            c.chi += d.clamped_chi;
            bool noemit_update = false;
            if ((DEC & 1) && (S.flags & F_TAU) && L.tau) {
                // optical depth in FP64: tau += W dt; emission at tau >= tau*, tau* = -ln(1 - u)
                // from channel 4 (words 0,1 if no target is set yet, words 2,3 after an emission)
                const uint4 w4 = philox_block(S.seed, lepton_id(L.species, i), S.step, 4u);
                double target = L.tau_t[i];
                if (!(target > 0.0)) target = -log1p(-u01_53(w4.x, w4.y));
                const double tn = L.tau[i] + (double)d.P;
                if (tn >= target) {
                    L.tau[i] = 0.0;
                    L.tau_t[i] = -log1p(-u01_53(w4.z, w4.w));
                    emit = true;
                    up = !(d.r1 < d.a / d.P);
                } else {
                    L.tau[i] = tn;
                    L.tau_t[i] = target;
                    if (d.P < (R)1) noemit_update = true;
                    else if (S.flags & F_NOEMIT) ++c.prob;
                }
            } else if ((DEC & 2) && (S.flags & F_REJECT)) {
                // rejection (spectrum-sampling section): candidate lambda = r1^3, accepted when
                // r2 < 3 r1^2 dW/dlambda dt with the spectrum of the lepton's spin state
                const double r1 = (double)d.r1;
                const double lam = r1 * r1 * r1, oml = (1.0 - r1) * (1.0 + r1 + r1 * r1);
                R K13, K23, IK;
                bessel_abs<R>(2.0 * (lam / oml) / (3.0 * d.chi), bn_of<R>(T), K13, K23, IK);
                const R kappa = (R)(1.0 / oml + oml);
                const R w = -IK + kappa * K23 + (R)lam * dot(s, d.bs.b) * K13;
                const R A = (R)(3.0 * r1 * r1) * d.Ce * w * (R)S.dt;
                c.prob += A > (R)1;
                if (d.r2 < A) {
                    emit = true;
                } else if (d.P < (R)1) {
                    noemit_update = true;
                } else if (S.flags & F_NOEMIT) {
                    ++c.prob;
                }
            } else if (d.P <= (R)1 && !(d.r1 < d.P)) {
                noemit_update = true;
            } else {
                emit = true;
                c.prob += d.P > (R)1;
                const R thr = d.P <= (R)1 ? d.a : d.a / d.P;
                up = !(d.r1 < thr);
                if constexpr ((DEC & 8) != 0) {
                    if (L.sub) {                      // one sub-step: its photon is in round 0
                        L.sub[i] = 1u;
                        ++c.rnd[0];
                    }
                }
            }
            if (noemit_update && (S.flags & F_NOEMIT)) noemit_spin<R>(S, d, msh, s, c.norm);
        }
    }
    stx(L.x, i, x);
    st3(L.p, i, p);
    st3(L.s, i, s);
}

// Main pass over the lepton range [start, end) (start a multiple of 64): the wave's decisions
// and branch choices go to mask[w] and mask[nchunks + w] of its 64-particle word w.
template <class R, int DEC, int FLD>
__device__ __forceinline__ void lepton_range(const LepDev<R> &L, const FieldDev &F, const StepDev &S, const TablesDev &T,
                                             const R *lds, int64_t start, int64_t end, uint64_t *mask, int64_t nchunks,
                                             LCount &c)
{
    const int lane = threadIdx.x & 63;
    if constexpr ((DEC & 4) != 0) {
        if (S.sub_round > 0) {
            // a later sub-cycling round: only the leptons with a sub-step in it load their state
            for (int64_t base = start + (threadIdx.x & ~63); base < end; base += blockDim.x) {
                const int64_t i = base + lane;
                bool emit = false, up = false;
                if (i < end && (S.sub_round & ((kSubRounds >> L.msub[i]) - 1)) == 0)
                    lepton_item<R, DEC, FLD>(L, F, S, T, lds, i, ldx(L.x, i), ld3(L.p, i), ld3(L.s, i), emit, up, c);
                const uint64_t m = __ballot(emit), mu = __ballot(up);
                if (lane == 0) {
                    mask[base >> 6] = m;
                    mask[nchunks + (base >> 6)] = mu;
                    c.trans += __popcll(m);
                }
            }
            return;
        }
    }
    // the next particle's x, p, s are loaded before this one is worked on
    V3<R> xn = {0, 0, 0}, pn = {0, 0, 0}, sn = {0, 0, 0};
    {
        const int64_t i = start + (threadIdx.x & ~63) + lane;
        if (i < end) { xn = ldx(L.x, i); pn = ld3(L.p, i); sn = ld3(L.s, i); }
    }
    for (int64_t base = start + (threadIdx.x & ~63); base < end; base += blockDim.x) {
        const int64_t i = base + lane;
        const V3<R> x = xn, p = pn, s = sn;
        const int64_t inext = i + blockDim.x;
        if (inext < end) { xn = ldx(L.x, inext); pn = ld3(L.p, inext); sn = ld3(L.s, inext); }
        bool emit = false, up = false;
        if (i < end) lepton_item<R, DEC, FLD>(L, F, S, T, lds, i, x, p, s, emit, up, c);
        const uint64_t m = __ballot(emit), mu = __ballot(up);
        if (lane == 0) {
            mask[base >> 6] = m;
            mask[nchunks + (base >> 6)] = mu;
            c.trans += __popcll(m);
        }
    }
}

// Emitter processing (NLC section, after the decision): lambda from the selected inverse CDF,
// recoil, spin collapse, Stokes collapse, P-vector; the photon goes to slot `slot` (< 0: no room).
// With x_out set, only the inputs of the inverse CDF (ln chi, rho, channel sign) are written there;
// with nu_in set, nu is taken from it instead of the table (learned inverse CDF).
template <class R, int FLD>
__device__ __forceinline__ void emit_item(const LepDev<R> &L, const PhoDev<R> &G, const FieldDev &F, const StepDev &S,
                                          const TablesDev &T, const R *lds, int64_t i, bool up, int64_t slot,
                                          unsigned &c_ret, const float *nu_in = nullptr, float *x_out = nullptr)
{
    const V3<R> x = ldx(L.x, i);
    V3<R> p = ld3(L.p, i), s = ld3(L.s, i);
    V3<R> E, B;
    eval_fields<R, FLD>(F, (double)x.x, (double)x.y, S.t + S.dt, E, B);
    const LDecide<R> d = lepton_decide<R>(S, T, lds, L.species, i, p, s, E, B);
    if (x_out) {
        const double r2 = (double)d.r2;
        x_out[0] = (float)log(d.chi);
        x_out[1] = (float)(log(r2) - log1p(-r2));
        x_out[2] = up ? 1.0f : -1.0f;
        return;
    }
    V3<R> k, Pv;
    emit_core<R>(S, T, d, L.species, i, up, p, s, k, Pv, nu_in);
    st3(L.p, i, p);
    st3(L.s, i, s);
    if (slot >= 0) store_photon<R>(G, S, L.species, i, slot, x, k, Pv, c_ret);
}

struct GCount { unsigned chi = 0, norm = 0, ret = 0, prob = 0, step = 0, qed = 0, trans = 0, nonfin = 0; };

// Photon streaming pass, one tile of at most kPhoTile slots starting at `tile` (a multiple of 64).
// Phase 1 (every slot): advance x, retire, evaluate the fields, queue the chi candidates in LDS.
// Phase 2 (queued slots only, so the QED part runs on full waves): chi in FP64, rates, draw,
// no-pair update, and the transition bits, OR-ed into the tile's mask words in LDS and stored
// once: decisions at mask[w], branch (plus) at mask[nchunks + w].
constexpr int kPhoTile = 1024;

// What the queue keeps of a candidate for phase 2's fields (QK): its x, from which phase 2
// evaluates the plane-wave or rotating field again at little cost (plain and rotating variants);
// its x and y (the general variant in FP64); or, in single precision, the E and B phase 1
// evaluated, so that phase 2 gathers no grid corners again (same values; the 16 KB more of LDS
// per block still leave the general variant its three blocks per compute unit, which the 48 KB
// more in FP64 would not).
enum : int { kQueueX = 0, kQueueXY = 1, kQueueEB = 2 };
template <class R, int FLD> constexpr int queue_kind()
{
    return FLD != kFldGeneral ? kQueueX : (sizeof(R) == 4 ? kQueueEB : kQueueXY);
}

template <class R, int TILE = kPhoTile, int QK = kQueueX> struct PhoQueue {
    uint32_t idx[TILE];
    uint64_t id[TILE];
    R x[QK == kQueueEB ? 1 : TILE], y[QK == kQueueXY ? TILE : 1];
    R eb[QK == kQueueEB ? 6 : 1][QK == kQueueEB ? TILE : 1];   // Ex, Ey, Ez, Bx, By, Bz
    R k[3][TILE];                  // the candidates' momenta, read once in phase 1
    unsigned long long bits[2][TILE / 64];
    uint32_t n;
};

// A tile's phase-1 inputs per thread (slots tile + 64-slot group of its wave + u kBlock + lane)
template <class R, int TILE> struct TileIn {
    uint64_t id[TILE / kBlock];
    V3<R> k[TILE / kBlock], x[TILE / kBlock];
};

// The reads of id, k and x of the tile [tile, tend) (non-temporal: the pass streams the store once)
template <class R, int TILE>
__device__ __forceinline__ void photon_tile_load(const PhoDev<R> &G, int64_t tile, int64_t tend, TileIn<R, TILE> &in)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < TILE / kBlock; ++u) {
        const int64_t i = tile + (threadIdx.x & ~63) + (int64_t)u * kBlock + lane;
        in.id[u] = 0;
        if (i < tend) {
            in.id[u] = __builtin_nontemporal_load(&G.id[i]);
            in.k[u] = {__builtin_nontemporal_load(&G.k[0][i]), __builtin_nontemporal_load(&G.k[1][i]),
                       __builtin_nontemporal_load(&G.k[2][i])};
            in.x[u] = {G.x[0] ? __builtin_nontemporal_load(&G.x[0][i]) : (R)0,
                       G.x[1] ? __builtin_nontemporal_load(&G.x[1][i]) : (R)0,
                       G.x[2] ? __builtin_nontemporal_load(&G.x[2][i]) : (R)0};
        }
    }
}

// PREF: the tile's inputs are in *pre already (photon_tile_load), and once phase 1 has used them
// the next tile's [next, next_end) (next >= 0) are loaded into it, so that their reads are in
// flight during phase 2; otherwise the tile loads its own.
template <class R, int FLD, int TILE = kPhoTile, bool PREF = false>
__device__ __forceinline__ void photon_tile(const PhoDev<R> &G, const FieldDev &F, const StepDev &S, const TablesDev &T,
                                            const R *lds, PhoQueue<R, TILE, queue_kind<R, FLD>()> &Q, int64_t tile,
                                            int64_t tend,
                                            uint64_t *mask, int64_t nchunks, GCount &c, TileIn<R, TILE> *pre = nullptr,
                                            int64_t next = -1, int64_t next_end = -1)
{
    const int lane = threadIdx.x & 63;
    const bool qed = (S.flags & F_PAIR) != 0;
    if (threadIdx.x < TILE / 64) { Q.bits[0][threadIdx.x] = 0ull; Q.bits[1][threadIdx.x] = 0ull; }
    if (threadIdx.x == 0) Q.n = 0;
    __syncthreads();
    // the slots of this thread: all loads first (id, k and x do not wait for each other), then the
    // work; a dead slot (id 0) loads values it never uses.  The pass streams through the photon
    // store once per step, so these reads and the position write are non-temporal: they do not
    // push the lepton arrays and tables out of the caches (the sparse P-vector accesses of phase
    // 2 stay ordinary: non-temporal partial writes cost more there)
    constexpr int kPer = TILE / kBlock;
    TileIn<R, TILE> own;
    if constexpr (!PREF) photon_tile_load<R, TILE>(G, tile, tend, own);
    TileIn<R, TILE> &in = PREF ? *pre : own;
    const uint64_t *idv = in.id;
    const V3<R> *kv = in.k, *xv = in.x;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t base = tile + (threadIdx.x & ~63) + (int64_t)u * kBlock;
        if (base >= tend) break;                      // wave-uniform
        const int64_t i = base + lane;
        constexpr int QK = queue_kind<R, FLD>();
        bool cand = false;
        R xq = (R)0, yq = (R)0;
        V3<R> Eq = {}, Bq = {};
        if (idv[u] != 0) {
            const V3<R> k = kv[u];
            const R k0r = sqrt_r(dot(k, k));
            V3<R> x = xv[u];
            x = x + ((R)S.dt / k0r) * k;
            // removed: k = 0 or a NaN or infinity in k or x (then the moved x is not finite), or
            // |k| beyond the type's range
            const bool fin = finite_sum(x.x + x.y + x.z) && finite_sum(k0r);
            if (fin) {
                ++c.step;
                if (G.x[0]) __builtin_nontemporal_store(x.x, &G.x[0][i]);
                if (G.x[1]) __builtin_nontemporal_store(x.y, &G.x[1][i]);
                if (G.x[2]) __builtin_nontemporal_store(x.z, &G.x[2][i]);
            }
            // retirement: too soft to ever reach chi_min, or behind the trailing edge of the
            // plane-wave pulse (the phase t + x of a photon never decreases)
            const bool behind = F.kind == 1 && F.phase_len > 0.0 && S.t + S.dt + (double)x.x > F.phase_len;
            if (!fin) {
                G.id[i] = 0;
                ++c.nonfin;
            } else if ((double)k0r < S.k_retire || behind) {
                G.id[i] = 0;
                ++c.ret;
            } else if (qed) {
                V3<R> E, Bf;
                eval_fields<R, FLD>(F, (double)x.x, (double)x.y, S.t + S.dt, E, Bf);
                if (FLD != kFldGeneral || (finite3(E) && finite3(Bf))) cand = photon_candidate<R>(S, k0r, E, Bf);
                else ++c.nonfin;                          // no QED in a non-finite grid field
                xq = x.x;
                yq = x.y;
                Eq = E;
                Bq = Bf;
            }
        }
        const uint64_t m = __ballot(cand);
        uint32_t wbase = 0;
        if (lane == 0 && m) wbase = atomicAdd(&Q.n, (uint32_t)__popcll(m));
        wbase = __shfl(wbase, 0);
        if (cand) {
            const uint32_t r = wbase + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            Q.idx[r] = (uint32_t)(i - tile);
            Q.id[r] = idv[u];
            if constexpr (QK == kQueueEB) {
                Q.eb[0][r] = Eq.x; Q.eb[1][r] = Eq.y; Q.eb[2][r] = Eq.z;
                Q.eb[3][r] = Bq.x; Q.eb[4][r] = Bq.y; Q.eb[5][r] = Bq.z;
            } else {
                Q.x[r] = xq;
                if constexpr (QK == kQueueXY) Q.y[r] = yq;
            }
            Q.k[0][r] = kv[u].x;
            Q.k[1][r] = kv[u].y;
            Q.k[2][r] = kv[u].z;
        }
    }
    __syncthreads();
    if constexpr (PREF) {
        if (next >= 0) photon_tile_load<R, TILE>(G, next, next_end, in);   // phase 1 is done with it
    }
    const uint32_t nq = Q.n;
    for (uint32_t j = threadIdx.x; j < nq; j += blockDim.x) {
        const uint32_t o = Q.idx[j];
        const int64_t i = tile + o;
        const V3<R> P = ld3(G.P, i);                  // the one global load of phase 2
        const uint64_t id = Q.id[j];
        const V3<R> k = {Q.k[0][j], Q.k[1][j], Q.k[2][j]};
        const double k0 = (double)sqrt_r(dot(k, k));
        V3<R> E, Bf;
        if constexpr (queue_kind<R, FLD>() == kQueueEB) {
            E = {Q.eb[0][j], Q.eb[1][j], Q.eb[2][j]};
            Bf = {Q.eb[3][j], Q.eb[4][j], Q.eb[5][j]};
        } else {
            eval_fields<R, FLD>(F, (double)Q.x[j], queue_kind<R, FLD>() == kQueueXY ? (double)Q.y[j] : 0.0, S.t + S.dt,
                                E, Bf);
        }
        const PDecide<R> d = photon_decide<R, true>(S, T, lds, id, k, k0, P, E, Bf);
        if (!d.active) continue;
        c.nonfin += d.nonfinite;
        ++c.qed;
        c.chi += d.clamped_chi;
        if (d.P <= (R)1 && !(d.r1 < d.P)) {
            if (S.flags & F_NOPAIR) {
                const R dt = (R)S.dt;
                const R Wbar = (R)0.5 * (d.Wp + d.Wm), dW = (R)0.5 * (d.Wp - d.Wm);
                const R inv = (R)1 / ((R)1 - d.P);
                const R f = ((R)1 - Wbar * dt) * inv;
                V3<R> xn = {d.x1 * f, d.x2 * f, (d.x3 * ((R)1 - Wbar * dt) - dW * dt) * inv};
                const R n2 = dot(xn, xn);
                if (n2 > (R)1) {
                    xn = rsqrt_r(n2) * xn;
                    c.norm += n2 > (R)1 + norm_count_tol<R>();
                }
                st3(G.P, i, stokes_to_P(xn.x, xn.y, xn.z, d.bs));
            }
        } else {
            c.prob += d.P > (R)1;
            const R thr = d.P <= (R)1 ? d.a : d.a / d.P;
            const unsigned long long bit = 1ull << (o & 63);
            atomicOr(&Q.bits[0][o >> 6], bit);
            if (!(d.r1 < thr)) atomicOr(&Q.bits[1][o >> 6], bit);
        }
    }
    __syncthreads();
    const int nw = (int)cdiv(tend - tile, 64);
    if (threadIdx.x < nw) {
        const uint64_t m = Q.bits[0][threadIdx.x];
        mask[(tile >> 6) + threadIdx.x] = m;
        mask[nchunks + (tile >> 6) + threadIdx.x] = Q.bits[1][threadIdx.x];
        c.trans += __popcll(m);
    }
    __syncthreads();
}

// Pair processing (NBW section, after the decision): lambda~ from the selected inverse CDF,
// momenta, correlated spins; the pair goes to slots se (electrons) and sp (positrons) when
// se >= 0; the photon becomes a dead slot.
template <class R, int FLD>
__device__ __forceinline__ void pair_item(const PhoDev<R> &G, const LepDev<R> &Le, const LepDev<R> &Lp, const FieldDev &F,
                                          const StepDev &S, const TablesDev &T, const R *lds, int64_t i, bool plus,
                                          int64_t se, int64_t sp, const float *nu_in = nullptr, float *x_out = nullptr)
{
    const uint64_t id = G.id[i];
    const V3<R> k = ld3(G.k, i), x = ldx(G.x, i), P = ld3(G.P, i);
    const double k0 = (double)sqrt_r(dot(k, k));
    V3<R> E, B;
    eval_fields<R, FLD>(F, (double)x.x, (double)x.y, S.t + S.dt, E, B);
    const PDecide<R> d = photon_decide<R>(S, T, lds, id, k, k0, P, E, B);
    const double r2 = (double)d.r2;
    const double rho = log(r2) - log1p(-r2);
    if (x_out) {
        x_out[0] = (float)log(d.chi);
        x_out[1] = (float)rho;
        x_out[2] = plus ? 1.0f : -1.0f;
        return;
    }
    const double nu = nu_in ? (double)*nu_in : icdf_nu(T, plus ? 3 : 2, log(d.chi), rho);
    const double lam_d = 1.0 / (1.0 + exp(-nu)), oml_d = 1.0 / (1.0 + exp(nu));
    const V3<R> pp = (R)lam_d * k, pe = (R)oml_d * k;
    V3<R> ec = {0, 0, 0}, pc = {0, 0, 0};
    if (S.flags & F_PAIR_SPIN) {
        SpecPt<R> qp;
        qp.lam = (R)lam_d; qp.oml = (R)oml_d; qp.u = (R)0;
        bessel_ratios<R>(2.0 * (1.0 / lam_d + 1.0 / oml_d) / (3.0 * d.chi), bn_of<R>(T), qp.K1, qp.I);
        const V3<R> xi = {d.x1, d.x2, d.x3};
        V3<R> je, jp;
        const R w0 = nbw_j(qp, xi, je, jp);
        if (S.flags & F_MEAN) {
            ec = ((R)1 / w0) * je;
            pc = ((R)1 / w0) * jp;
        } else {
            R r3, r3b;
            Unif<R>::two(philox_block(S.seed, id, S.step, 3u), r3, r3b);
            const R jen = sqrt_r(dot(je, je)), jpn = sqrt_r(dot(jp, jp));
            const V3<R> Se = jen > (R)0 ? ((R)1 / jen) * je : v3<R>(0, 1, 0);
            const V3<R> Sp = jpn > (R)0 ? ((R)1 / jpn) * jp : v3<R>(0, 1, 0);
            // outcomes (positron, electron): (down,down), (down,up), (up,down), (up,up)
            const R inv4 = (R)1 / ((R)4 * w0);
            R cum = 0;
            int pick = 3;
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                const R spn = o < 2 ? (R)-1 : (R)1, sen = (o & 1) ? (R)1 : (R)-1;
                V3<R> Gv;
                const R G0 = nbw_G(qp, sen * Se, spn * Sp, Gv);
                cum += (G0 + dot(xi, Gv)) * inv4;
                if (pick == 3 && r3 < cum) pick = o;
            }
            const R spn = pick < 2 ? (R)-1 : (R)1, sen = (pick & 1) ? (R)1 : (R)-1;
            ec = sen * Se;
            pc = spn * Sp;
        }
    }
    G.id[i] = 0;
    if (se >= 0) {
        // new leptons start with no optical depth and no target (drawn at their first step)
        if (Le.tau) { Le.tau[se] = 0.0; Le.tau_t[se] = 0.0; }
        if (Lp.tau) { Lp.tau[sp] = 0.0; Lp.tau_t[sp] = 0.0; }
        const V3<R> se_lab = ec.x * d.bs.e + ec.y * d.bs.b + ec.z * d.bs.k;
        const V3<R> sp_lab = pc.x * d.bs.e + pc.y * d.bs.b + pc.z * d.bs.k;
        stx(Le.x, se, x);
        st3(Le.p, se, pe);
        st3(Le.s, se, se_lab);
        stx(Lp.x, sp, x);
        st3(Lp.p, sp, pp);
        st3(Lp.s, sp, sp_lab);
    }
}

// ------------------------------------------------------------------ host-side views
template <class R> LepDev<R> lep_dev(const qed_leptons *L)
{
    LepDev<R> d;
    d.cap = L->capacity;
    d.count = L->d_count;
    d.species = L->species;
    for (int c = 0; c < 3; ++c) {
        d.x[c] = (R *)L->x[c];
        d.p[c] = (R *)L->p[c];
        d.s[c] = (R *)L->s[c];
    }
    d.tau = L->tau;
    d.tau_t = L->tau_target;
    d.msub = nullptr;
    d.sub = nullptr;
    d.stage = nullptr;
    return d;
}

template <class R> PhoDev<R> pho_dev(const qed_photons *G)
{
    PhoDev<R> d;
    if (!G) {                     // emission disabled: a view with no room, never written
        memset(&d, 0, sizeof(d));
        return d;
    }
    d.cap = G->capacity;
    d.count = G->d_count;
    d.count_prev = G->d_count_prev;
    for (int c = 0; c < 3; ++c) {
        d.x[c] = (R *)G->x[c];
        d.k[c] = (R *)G->k[c];
        d.P[c] = (R *)G->P[c];
    }
    d.id = G->id;
    return d;
}

inline FieldDev field_dev(const qed_fields *f)
{
    FieldDev d;
    memset(&d, 0, sizeof(d));
    d.kind = f->kind;
    for (int c = 0; c < 3; ++c) {
        d.E0[c] = f->E0[c];
        d.B0[c] = f->B0[c];
    }
    d.a0 = f->a0;
    d.phase_len = f->phase_len;
    d.inv_phase_len = f->phase_len > 0.0 ? 1.0 / f->phase_len : 0.0;
    if (f->kind == QED_FIELD_GRID2D) {
        for (int c = 0; c < 6; ++c) d.g[c] = f->grid[c];
        d.nx = f->nx; d.ny = f->ny;
        d.gx0 = f->x0; d.gy0 = f->y0;
        d.inv_dx = 1.0 / f->dx; d.inv_dy = 1.0 / f->dy;
        d.inv_nx = 1.0 / f->nx; d.inv_ny = 1.0 / f->ny;
    }
    return d;
}

inline StepDev step_dev(const qed_step_params *p)
{
    StepDev s;
    s.t = p->t; s.dt = p->dt; s.a_e = p->a_e; s.eps_r = p->eps_r;
    s.chi_e_min = p->chi_e_min; s.chi_e_max = p->chi_e_max; s.chi_g_min = p->chi_g_min; s.chi_g_max = p->chi_g_max;
    s.k_retire = p->k_retire;
    s.Kc = kAlpha / (sqrt(3.0) * kPi * p->eps_r);
    s.step = p->step; s.seed = p->seed; s.flags = p->flags;
    s.sub_round = 0;
    s.clock = p->d_clock;
    return s;
}

inline int grid_for(int64_t n)
{
    const int64_t g = cdiv(n > 0 ? n : 1, kBlock);
    return (int)(g < kMaxGrid ? g : kMaxGrid);
}


inline bool leptons_ok(const qed_leptons *L)
{
    if (!L || !L->d_count || L->capacity < 0 || L->capacity >= (int64_t)1 << 32) return false;
    if (L->species != 0 && L->species != 1) return false;
    for (int c = 0; c < 3; ++c)
        if (!L->p[c] || !L->s[c]) return false;
    return true;
}

// the optical-depth decision needs both FP64 arrays
inline bool tau_ok(const qed_leptons *L, uint32_t flags)
{
    return !(flags & QED_OPTICAL_DEPTH) || (L->tau && L->tau_target);
}

inline bool photons_ok(const qed_photons *G)
{
    if (!G || !G->d_count || !G->d_count_prev || !G->id || G->capacity < 0 || G->capacity >= (int64_t)1 << 32) return false;
    for (int c = 0; c < 3; ++c)
        if (!G->k[c] || !G->P[c]) return false;
    return true;
}

// the field-model variant a field needs (the variants are nested: general > rotating > plain)
inline int field_variant(const qed_fields *f)
{
    return f->kind == QED_FIELD_GRID2D ? kFldGeneral : f->kind == QED_FIELD_ROTATING_E ? kFldRotating : kFldPlain;
}

// the lepton pass's variant: the field's, or the general one for the field-dependent g
inline int lepton_variant(const qed_fields *f, uint32_t flags)
{
    return (flags & QED_G_CHI) ? (int)kFldGeneral : field_variant(f);
}

// field parameters must be finite and far below the FP32 range (so every analytic field value is
// finite in both precisions)
inline bool field_param_ok(double v) { return v == v && v < 1e30 && v > -1e30; }

inline bool fields_ok(const qed_fields *f)
{
    if (!f) return false;
    for (int c = 0; c < 3; ++c)
        if (!field_param_ok(f->E0[c]) || !field_param_ok(f->B0[c])) return false;
    if (!field_param_ok(f->a0) || !field_param_ok(f->phase_len)) return false;
    if (f->kind == QED_FIELD_UNIFORM || f->kind == QED_FIELD_PLANE_LP) return true;
    if (f->kind == QED_FIELD_ROTATING_E) return f->a0 == f->a0;
    if (f->kind != QED_FIELD_GRID2D) return false;
    for (int c = 0; c < 6; ++c)
        if (!f->grid[c]) return false;
    return f->nx >= 2 && f->ny >= 2 && f->dx > 0.0 && f->dy > 0.0 && field_param_ok(f->dx) && field_param_ok(f->dy) &&
           field_param_ok(f->x0) && field_param_ok(f->y0);
}

}  // namespace qs
