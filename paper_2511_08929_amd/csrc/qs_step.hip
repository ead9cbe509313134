// qs_step.hip -- the per-particle QED step on gfx950: qed_push_spin, qed_emit, qed_pair,
// qed_compact.
//
// Each transition step runs as
//   main     one streaming pass over the particle SoA (coalesced loads/stores, rate tables in
//            LDS): push, chi, basis, rates, Philox draw, decision, no-transition update; the
//            wave's 64 decisions and branch choices are ballot'ed into two 64-bit mask words;
//   reduce   per-block popcount sums of the mask words;
//   book     one block: total, append bases, capacity clamp, counters, device-side counts;
//   expand   per-block prefix + block scan of the mask popcounts -> dense, ascending list of
//            the transitioning particles' indices;
//   process  one thread per transitioning particle (dense, no divergence from the ~97 % that
//            do not transition): inverse-CDF sampling, Bessel functions, spin / Stokes collapse,
//            appends at base + rank.
// Everything is keyed on device-resident counts, so a step enqueues without host sync.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "qs_internal.hpp"

namespace {
using namespace qs;

constexpr int kBlock = 256;
constexpr int kMaxGrid = 2048;                               // 256 CUs x 8 resident blocks

template <class R> struct LepDev {
    int64_t cap;
    int64_t *count;
    int species;
    R *x[3], *p[3], *s[3];
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

enum { C_EMIT = 0, C_PAIR, C_PROB, C_CHI, C_NORM, C_OVER, C_RETIRED, C_LSTEP, C_GSTEP, C_GQED, kNCtr };

struct WS {
    uint64_t *mask;      // [2][nchunks]: transition, branch (up / plus)
    uint32_t *bcnt;      // [kMaxGrid]: transitions per block of the streaming pass
    int64_t *book;       // [8]: base0, total, base1, n_fit, n processed, block range
    uint32_t *bctr;      // [kMaxGrid][kNCtr]: per-block counts of the streaming pass
    uint32_t *idx;       // [max particles]
};

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

WS carve(void *ws, int64_t cap, int64_t *nchunks_out)
{
    const int64_t nch = cdiv(cap > 0 ? cap : 1, 64);
    char *b = (char *)ws;
    WS w;
    w.mask = (uint64_t *)b; b += align256(sizeof(uint64_t) * 2 * nch);
    w.bcnt = (uint32_t *)b; b += align256(sizeof(uint32_t) * kMaxGrid);
    w.book = (int64_t *)b;  b += align256(sizeof(int64_t) * 8);
    w.bctr = (uint32_t *)b; b += align256(sizeof(uint32_t) * kMaxGrid * kNCtr);
    w.idx = (uint32_t *)b;
    *nchunks_out = nch;
    return w;
}

// ------------------------------------------------------------------ device helpers
template <class R> __device__ __forceinline__ const R *rate_src(const TablesDev &T);
template <> __device__ __forceinline__ const double *rate_src<double>(const TablesDev &T) { return T.lnrate; }
template <> __device__ __forceinline__ const float *rate_src<float>(const TablesDev &T) { return T.lnrate32; }

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

// per-block totals of the streaming pass's counts and of its transitions, written (not
// atomically added) to the workspace; the bookkeeping kernel reduces them
__device__ __forceinline__ void block_counts(uint32_t *bctr, uint32_t *bcnt, const unsigned (&v)[kNCtr], unsigned ntrans)
{
    __shared__ unsigned red[kBlock / 64][kNCtr + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kNCtr; ++c) {
        unsigned t = v[c];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) red[wid][c] = t;
    }
    if (lane == 0) red[wid][kNCtr] = ntrans;      // lane 0 holds its wave's transition count
    __syncthreads();
    if (threadIdx.x <= kNCtr) {
        unsigned t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w][threadIdx.x];
        if (threadIdx.x < kNCtr) bctr[blockIdx.x * kNCtr + threadIdx.x] = t;
        else bcnt[blockIdx.x] = t;
    }
}

__device__ __forceinline__ void wave_add(unsigned long long *ctr, int slot, unsigned v)
{
    // reduce over the wave, one atomic per wave
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr + slot, (unsigned long long)v);
}

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
    R Wdn, Wup, a, P, r1, r2;
    bool active;       // chi >= chi_min
    bool clamped_chi;
};

template <class R>
__device__ __forceinline__ LDecide<R> lepton_decide(const StepDev &S, const TablesDev &T, const R *lds, int species,
                                                    int64_t index, V3<R> p, V3<R> s, V3<R> E, V3<R> B)
{
    LDecide<R> d;
    d.clamped_chi = false;
    if (zero_field(E, B)) {           // outside the pulse: no QED, skip the FP64 island
        d.active = false;
        d.chi = 0.0;
        return d;
    }
    const int q = species == 0 ? -1 : 1;
    const double gam = sqrt(1.0 + dot(cvt<double>(p), cvt<double>(p)));
    d.chi = basis_chi(q, S.eps_r, p, gam, E, B, d.bs);
    d.active = d.chi >= S.chi_e_min;
    d.clamped_chi = d.chi > S.chi_e_max;
    if (d.clamped_chi) d.chi = S.chi_e_max;
    if (!d.active) return d;
    const int n = T.n_chi[0];
    const R lnchi = log_r((R)d.chi);
    const R x0 = (R)T.lnchi0[0], h = (R)T.dlnchi[0];
    const R Ce = ratio_r<R>(S.Kc, gam);
    d.Wdn = Ce * exp_r(rate_lookup(lds, lnchi, x0, h, n));
    d.Wup = Ce * exp_r(rate_lookup(lds + n, lnchi, x0, h, n));
    const R sb = dot(s, d.bs.b);
    const R dt = (R)S.dt;
    d.a = d.Wdn * (R)0.5 * ((R)1 - sb) * dt;
    const R b = d.Wup * (R)0.5 * ((R)1 + sb) * dt;
    d.P = d.a + b;
    const uint4 w = philox_block(S.seed, lepton_id(species, index), S.step, 0u);
    Unif<R>::two(w, d.r1, d.r2);
    return d;
}

// ------------------------------------------------------------------ kernels: leptons
template <class R>
__global__ void __launch_bounds__(kBlock) k_push(LepDev<R> L, FieldDev F, StepDev S0)
{
    const StepDev S = localize(S0);
    const int64_t n = *L.count;
    const int q = L.species == 0 ? -1 : 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        V3<R> x = ldx(L.x, i), p = ld3(L.p, i), s = ld3(L.s, i);
        V3<R> E, B;
        eval_fields<R>(F, (double)x.x, S.t, E, B);
        const V3<R> d = push<R>(q, (R)S.a_e, E, B, (R)S.dt, (S.flags & F_TBMT) != 0, p, s);
        stx(L.x, i, x + d);
        st3(L.p, i, p);
        st3(L.s, i, s);
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_lepton_main(LepDev<R> L, FieldDev F, StepDev S0, TablesDev T,
                                                        uint64_t *mask, int64_t nchunks, uint32_t *bctr, uint32_t *bcnt)
{
    const StepDev S = localize(S0);
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    stage_rates<R>(T, 0, lds);
    const int64_t n = *L.count;
    const int64_t B = block_len(n, gridDim.x);
    const int64_t start = (int64_t)blockIdx.x * B, end = start + B < n ? start + B : n;
    const int q = L.species == 0 ? -1 : 1;
    const int lane = threadIdx.x & 63;
    unsigned c_prob = 0, c_chi = 0, c_norm = 0, c_step = 0, ntrans = 0;
    for (int64_t base = start + (threadIdx.x & ~63); base < end; base += blockDim.x) {
        const int64_t i = base + lane;
        bool emit = false, up = false;
        if (i < end) {
            ++c_step;
            V3<R> x = ldx(L.x, i), p = ld3(L.p, i), s = ld3(L.s, i);
            V3<R> E, B;
            if (S.flags & F_PUSH) {
                eval_fields<R>(F, (double)x.x, S.t, E, B);
                x = x + push<R>(q, (R)S.a_e, E, B, (R)S.dt, (S.flags & F_TBMT) != 0, p, s);
            }
            if (S.flags & F_EMIT) {
                eval_fields<R>(F, (double)x.x, S.t + S.dt, E, B);
                const LDecide<R> d = lepton_decide<R>(S, T, lds, L.species, i, p, s, E, B);
                if (d.active) {
                    c_chi += d.clamped_chi;
                    if (d.P <= (R)1 && !(d.r1 < d.P)) {
                        if (S.flags & F_NOEMIT) {
                            const R dt = (R)S.dt;
                            const R Wbar = (R)0.5 * (d.Wup + d.Wdn), dW = (R)0.5 * (d.Wup - d.Wdn);
                            const R inv = (R)1 / ((R)1 - d.P);
                            s = inv * (((R)1 - Wbar * dt) * s - (dW * dt) * d.bs.b);
                            const R n2 = dot(s, s);
                            if (n2 > (R)1) {
                                s = rsqrt_r(n2) * s;
                                c_norm += n2 > (R)1 + norm_count_tol<R>();
                            }
                        }
                    } else {
                        emit = true;
                        c_prob += d.P > (R)1;
                        const R thr = d.P <= (R)1 ? d.a : d.a / d.P;
                        up = !(d.r1 < thr);
                    }
                }
            }
            stx(L.x, i, x);
            st3(L.p, i, p);
            st3(L.s, i, s);
        }
        const uint64_t m = __ballot(emit), mu = __ballot(up);
        if (lane == 0) {
            mask[base >> 6] = m;
            mask[nchunks + (base >> 6)] = mu;
            ntrans += __popcll(m);
        }
    }
    unsigned v[kNCtr] = {};
    v[C_PROB] = c_prob; v[C_CHI] = c_chi; v[C_NORM] = c_norm; v[C_LSTEP] = c_step;
    block_counts(bctr, bcnt, v, ntrans);
}

// emitter processing: lambda from the selected inverse CDF, recoil, spin collapse, Stokes
// collapse, P-vector, photon append (NLC section, steps after the decision)
template <class R>
__global__ void __launch_bounds__(kBlock) k_emit_process(LepDev<R> L, PhoDev<R> G, FieldDev F, StepDev S0, TablesDev T,
                                                         const uint64_t *mask, int64_t nchunks, const uint32_t *idx,
                                                         const int64_t *book, unsigned long long *ctr)
{
    const StepDev S = localize(S0);
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    stage_rates<R>(T, 0, lds);
    const int64_t total = book[1], gbase = book[0], nfit = book[3];
    unsigned c_ret = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[j];
        const V3<R> x = ldx(L.x, i);
        V3<R> p = ld3(L.p, i), s = ld3(L.s, i);
        V3<R> E, B;
        eval_fields<R>(F, (double)x.x, S.t + S.dt, E, B);
        const LDecide<R> d = lepton_decide<R>(S, T, lds, L.species, i, p, s, E, B);
        const bool up = (mask[nchunks + (i >> 6)] >> (i & 63)) & 1ull;
        const double r2 = (double)d.r2;
        const double rho = log(r2) - log1p(-r2);
        const double nu = icdf_nu(T, up ? 1 : 0, log(d.chi), rho);
        const double lam_d = 1.0 / (1.0 + exp(-nu)), oml_d = 1.0 / (1.0 + exp(nu));
        const double u_d = lam_d / oml_d;
        const V3<R> k = (R)lam_d * p;
        R r3, r4;
        Unif<R>::two(philox_block(S.seed, lepton_id(L.species, i), S.step, 1u), r3, r4);
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
        if (S.flags & F_PHOTON_POL) {
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
        const V3<R> Pv = stokes_to_P(xi.x, xi.y, xi.z, d.bs);
        if (S.flags & F_RECOIL) p = (R)oml_d * p;
        if (S.flags & F_SPIN) s = sf.x * d.bs.e + sf.y * d.bs.b + sf.z * d.bs.k;
        st3(L.p, i, p);
        st3(L.s, i, s);
        if (j < nfit) {
            const int64_t m = gbase + j;
            if (sqrt(dot(cvt<double>(k), cvt<double>(k))) < S.k_retire) {
                G.id[m] = 0;
                ++c_ret;
            } else {
                G.id[m] = photon_id(L.species, i, S.step);
                stx(G.x, m, x);
                st3(G.k, m, k);
                st3(G.P, m, Pv);
            }
        }
    }
    wave_add(ctr, C_RETIRED, c_ret);
}

// ------------------------------------------------------------------ kernels: photons
template <class R> struct PDecide {
    double chi;
    Basis<R> bs;
    R Wm, Wp, a, P, r1, r2, x1, x2, x3;
    bool active, clamped_chi;
};

template <class R>
__device__ __forceinline__ PDecide<R> photon_decide(const StepDev &S, const TablesDev &T, const R *lds, uint64_t id,
                                                    V3<R> k, double k0, V3<R> P, V3<R> E, V3<R> B)
{
    PDecide<R> d;
    d.clamped_chi = false;
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
    d.Wm = Cg * exp_r(rate_lookup(lds, lnchi, x0, h, n));
    d.Wp = Cg * exp_r(rate_lookup(lds + n, lnchi, x0, h, n));
    P_to_stokes(P, d.bs, d.x1, d.x2, d.x3);
    const R dt = (R)S.dt;
    d.a = d.Wm * (R)0.5 * ((R)1 - d.x3) * dt;
    const R b = d.Wp * (R)0.5 * ((R)1 + d.x3) * dt;
    d.P = d.a + b;
    Unif<R>::two(philox_block(S.seed, id, S.step, 2u), d.r1, d.r2);
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

// Photon streaming pass.  The block walks its contiguous range in tiles of kPhoTile slots.
// Phase 1 (every slot): advance x, retire, evaluate the fields, queue the candidates in LDS.
// Phase 2 (queued slots only, all lanes busy): chi in FP64, rates, draw, no-pair update, and
// the transition bits, OR-ed into the tile's mask words in LDS and stored once per tile.
constexpr int kPhoTile = 1024;

template <class R>
__global__ void __launch_bounds__(kBlock) k_photon_main(PhoDev<R> G, FieldDev F, StepDev S0, TablesDev T, uint64_t *mask,
                                                        int64_t nchunks, uint32_t *bctr, uint32_t *bcnt)
{
    const StepDev S = localize(S0);
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    __shared__ uint32_t q_idx[kPhoTile];
    __shared__ R q_x[kPhoTile];
    __shared__ unsigned long long q_bits[2][kPhoTile / 64];
    __shared__ uint32_t q_n;
    stage_rates<R>(T, 1, lds);
    const int64_t n = *G.count_prev;
    const int64_t B = block_len(n, gridDim.x);
    const int64_t start = (int64_t)blockIdx.x * B, end = start + B < n ? start + B : n;
    const int lane = threadIdx.x & 63;
    const bool qed = (S.flags & F_PAIR) != 0;
    unsigned c_chi = 0, c_norm = 0, c_ret = 0, c_prob = 0, c_step = 0, c_qed = 0, ntrans = 0;
    for (int64_t tile = start; tile < end; tile += kPhoTile) {
        const int64_t tend = tile + kPhoTile < end ? tile + kPhoTile : end;
        if (threadIdx.x < kPhoTile / 64) { q_bits[0][threadIdx.x] = 0ull; q_bits[1][threadIdx.x] = 0ull; }
        if (threadIdx.x == 0) q_n = 0;
        __syncthreads();
        // phase 1
        for (int64_t base = tile + (threadIdx.x & ~63); base < tend; base += blockDim.x) {
            const int64_t i = base + lane;
            bool cand = false;
            R xq = (R)0;
            if (i < tend) {
                const uint64_t id = G.id[i];
                if (id != 0) {
                    ++c_step;
                    const V3<R> k = ld3(G.k, i);
                    const R k0r = sqrt_r(dot(k, k));
                    V3<R> x = ldx(G.x, i);
                    x = x + ((R)S.dt / k0r) * k;
                    stx(G.x, i, x);
                    // retirement: too soft to ever reach chi_min, or behind the trailing edge of the
                    // plane-wave pulse (the phase t + x of a photon never decreases)
                    const bool behind = F.kind == 1 && F.phase_len > 0.0 && S.t + S.dt + (double)x.x > F.phase_len;
                    if ((double)k0r < S.k_retire || behind) {
                        G.id[i] = 0;
                        ++c_ret;
                    } else if (qed) {
                        V3<R> E, Bf;
                        eval_fields<R>(F, (double)x.x, S.t + S.dt, E, Bf);
                        cand = photon_candidate<R>(S, k0r, E, Bf);
                        xq = x.x;
                    }
                }
            }
            const uint64_t m = __ballot(cand);
            uint32_t wbase = 0;
            if (lane == 0 && m) wbase = atomicAdd(&q_n, (uint32_t)__popcll(m));
            wbase = __shfl(wbase, 0);
            if (cand) {
                const uint32_t r = wbase + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                q_idx[r] = (uint32_t)(i - tile);
                q_x[r] = xq;
            }
        }
        __syncthreads();
        // phase 2
        const uint32_t nq = q_n;
        for (uint32_t j = threadIdx.x; j < nq; j += blockDim.x) {
            const uint32_t o = q_idx[j];
            const int64_t i = tile + o;
            const uint64_t id = G.id[i];
            const V3<R> k = ld3(G.k, i);
            const double k0 = (double)sqrt_r(dot(k, k));
            V3<R> E, Bf;
            eval_fields<R>(F, (double)q_x[j], S.t + S.dt, E, Bf);
            const V3<R> P = ld3(G.P, i);
            const PDecide<R> d = photon_decide<R>(S, T, lds, id, k, k0, P, E, Bf);
            if (!d.active) continue;
            ++c_qed;
            c_chi += d.clamped_chi;
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
                        c_norm += n2 > (R)1 + norm_count_tol<R>();
                    }
                    st3(G.P, i, stokes_to_P(xn.x, xn.y, xn.z, d.bs));
                }
            } else {
                c_prob += d.P > (R)1;
                const R thr = d.P <= (R)1 ? d.a : d.a / d.P;
                const unsigned long long bit = 1ull << (o & 63);
                atomicOr(&q_bits[0][o >> 6], bit);
                if (!(d.r1 < thr)) atomicOr(&q_bits[1][o >> 6], bit);
            }
        }
        __syncthreads();
        const int nw = (int)cdiv(tend - tile, 64);
        if (threadIdx.x < nw) {
            const uint64_t m = q_bits[0][threadIdx.x];
            mask[(tile >> 6) + threadIdx.x] = m;
            mask[nchunks + (tile >> 6) + threadIdx.x] = q_bits[1][threadIdx.x];
            ntrans += __popcll(m);
        }
        __syncthreads();
    }
    unsigned v[kNCtr] = {};
    v[C_PROB] = c_prob; v[C_CHI] = c_chi; v[C_NORM] = c_norm; v[C_RETIRED] = c_ret; v[C_GSTEP] = c_step;
    v[C_GQED] = c_qed;
    // block_counts takes lane 0's transition count per wave: reduce the tile-word counts first
    for (int o = 32; o > 0; o >>= 1) ntrans += __shfl_xor(ntrans, o);
    block_counts(bctr, bcnt, v, ntrans);
}

// pair processing: lambda~ from the selected inverse CDF, momenta, correlated spins
// (NBW section), appends at base + rank in both lepton sets, decayed photon -> dead slot
template <class R>
__global__ void __launch_bounds__(kBlock) k_pair_process(PhoDev<R> G, LepDev<R> Le, LepDev<R> Lp, FieldDev F, StepDev S0,
                                                         TablesDev T, const uint64_t *mask, int64_t nchunks,
                                                         const uint32_t *idx, const int64_t *book)
{
    const StepDev S = localize(S0);
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    stage_rates<R>(T, 1, lds);
    // photons born later in this step wait for the next one: the next pair step covers all stored now
    if (blockIdx.x == 0 && threadIdx.x == 0) *G.count_prev = *G.count;
    const int64_t total = book[1], be = book[0], bp = book[2], nfit = book[3];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[j];
        const uint64_t id = G.id[i];
        const V3<R> k = ld3(G.k, i), x = ldx(G.x, i), P = ld3(G.P, i);
        const double k0 = (double)sqrt_r(dot(k, k));
        V3<R> E, B;
        eval_fields<R>(F, (double)x.x, S.t + S.dt, E, B);
        const PDecide<R> d = photon_decide<R>(S, T, lds, id, k, k0, P, E, B);
        const bool plus = (mask[nchunks + (i >> 6)] >> (i & 63)) & 1ull;
        const double r2 = (double)d.r2;
        const double nu = icdf_nu(T, plus ? 3 : 2, log(d.chi), log(r2) - log1p(-r2));
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
                    const R sp = o < 2 ? (R)-1 : (R)1, se = (o & 1) ? (R)1 : (R)-1;
                    V3<R> Gv;
                    const R G0 = nbw_G(qp, se * Se, sp * Sp, Gv);
                    cum += (G0 + dot(xi, Gv)) * inv4;
                    if (pick == 3 && r3 < cum) pick = o;
                }
                const R sp = pick < 2 ? (R)-1 : (R)1, se = (pick & 1) ? (R)1 : (R)-1;
                ec = se * Se;
                pc = sp * Sp;
            }
        }
        G.id[i] = 0;
        if (j < nfit) {
            const V3<R> se_lab = ec.x * d.bs.e + ec.y * d.bs.b + ec.z * d.bs.k;
            const V3<R> sp_lab = pc.x * d.bs.e + pc.y * d.bs.b + pc.z * d.bs.k;
            stx(Le.x, be + j, x);
            st3(Le.p, be + j, pe);
            st3(Le.s, be + j, se_lab);
            stx(Lp.x, bp + j, x);
            st3(Lp.p, bp + j, pp);
            st3(Lp.s, bp + j, sp_lab);
        }
    }
}

// ------------------------------------------------------------------ kernels: scan / compaction
// Scan + bookkeeping + expansion in one launch over the streaming pass's grid.
// Block b sums the transition counts of the blocks before it (its rank offset) and writes the
// ascending indices of the transitioning particles of the range it owned in the streaming pass.
// Block 0 also does the bookkeeping: total, append bases, capacity clamp, device counts:
//   mode 0  photon append (emission)      cnt0 = photons
//   mode 1  pair append to two lepton sets (cnt0 = electrons, cnt1 = positrons)
//   mode 2  compaction (cnt_prev = survivors; the photon count is set by the copy-back)
// and every 32nd block adds the streaming pass's per-block counters of 32 blocks to ctr.
// `count` is the particle count the streaming pass used; it is not modified here.
__global__ void __launch_bounds__(kBlock) k_expand(const uint64_t *mask, const uint32_t *bcnt, const int64_t *count,
                                                   int64_t *book, int mode, int64_t *cnt0, int64_t cap0, int64_t *cnt1,
                                                   int64_t cap1, int64_t *cnt_prev, unsigned long long *ctr,
                                                   const uint32_t *bctr, uint32_t *idx)
{
    __shared__ uint32_t wtot[kBlock / 64];
    __shared__ unsigned long long wc[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nblk = gridDim.x, b = blockIdx.x;
    const int64_t n = *count;
    // rank offset of this block and (block 0) the total
    uint32_t pre = 0, all = 0;
    for (int k = threadIdx.x; k < nblk; k += kBlock) {
        const uint32_t v = bcnt[k];
        all += v;
        if (k < b) pre += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        pre += __shfl_xor(pre, o);
        all += __shfl_xor(all, o);
    }
    if (lane == 0) { wtot[wid] = pre; wc[wid] = all; }
    __syncthreads();
    uint32_t rank0 = 0, total = 0;
    for (int w = 0; w < kBlock / 64; ++w) { rank0 += wtot[w]; total += (uint32_t)wc[w]; }
    __syncthreads();
    // counters of the streaming pass: in blocks b = 0, 32, 64, ..., thread c adds counter c of 32 blocks
    if (ctr && bctr && (b & 31) == 0 && threadIdx.x < kNCtr) {
        const int hi = b + 32 < nblk ? b + 32 : nblk;
        unsigned long long t = 0;
        for (int k = b; k < hi; ++k) t += bctr[k * kNCtr + threadIdx.x];
        if (t) atomicAdd(ctr + threadIdx.x, t);
    }
    if (b == 0 && threadIdx.x == 0) {
        if (mode == 0) {
            const int64_t base = cnt0 ? *cnt0 : 0;
            const int64_t room = cnt0 && cap0 - base > 0 ? cap0 - base : 0;
            const int64_t nfit = (int64_t)total < room ? (int64_t)total : room;
            book[0] = base; book[1] = total; book[2] = 0; book[3] = nfit;
            if (cnt0) *cnt0 = base + nfit;
            if (ctr) {
                atomicAdd(ctr + C_EMIT, (unsigned long long)total);
                if (total > nfit) atomicAdd(ctr + C_OVER, (unsigned long long)(total - nfit));
            }
        } else if (mode == 1) {
            const int64_t be = *cnt0, bp = *cnt1;
            int64_t room = cap0 - be < cap1 - bp ? cap0 - be : cap1 - bp;
            room = room > 0 ? room : 0;
            const int64_t nfit = (int64_t)total < room ? (int64_t)total : room;
            book[0] = be; book[1] = total; book[2] = bp; book[3] = nfit;
            *cnt0 = be + nfit;
            *cnt1 = bp + nfit;
            if (ctr) {
                atomicAdd(ctr + C_PAIR, (unsigned long long)total);
                if (total > nfit) atomicAdd(ctr + C_OVER, (unsigned long long)(total - nfit));
            }
        } else {
            book[0] = 0; book[1] = total; book[2] = 0; book[3] = total;
            if (cnt_prev) *cnt_prev = (int64_t)total;
        }
    }
    // expansion of this block's mask words
    const int64_t B = block_len(n, nblk);
    const int64_t start = (int64_t)b * B;
    if (start >= n) return;
    const int64_t end = start + B < n ? start + B : n;
    const int64_t c0 = start >> 6, c1 = cdiv(end, 64);
    for (int64_t tile = c0; tile < c1; tile += kBlock) {
        const int64_t c = tile + threadIdx.x;
        const uint64_t m = c < c1 ? mask[c] : 0ull;
        const uint32_t pc = __popcll(m);
        uint32_t incl = pc;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wtot[wid] = incl;
        __syncthreads();
        uint32_t woff = 0, ttot = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            if (w < wid) woff += wtot[w];
            ttot += wtot[w];
        }
        uint32_t rank = rank0 + woff + incl - pc;
        uint64_t bits = m;
        while (bits) {
            const int bit = __ffsll((long long)bits) - 1;
            idx[rank++] = (uint32_t)(c * 64 + bit);
            bits &= bits - 1;
        }
        rank0 += ttot;
        __syncthreads();
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_alive_mask(PhoDev<R> G, uint64_t *mask, uint32_t *bcnt)
{
    __shared__ unsigned red[kBlock / 64];
    const int64_t n = *G.count;
    const int64_t B = block_len(n, gridDim.x);
    const int64_t start = (int64_t)blockIdx.x * B, end = start + B < n ? start + B : n;
    unsigned ntrans = 0;
    for (int64_t base = start + (threadIdx.x & ~63); base < end; base += blockDim.x) {
        const int64_t i = base + (threadIdx.x & 63);
        const bool alive = i < end && G.id[i] != 0;
        const uint64_t m = __ballot(alive);
        if ((threadIdx.x & 63) == 0) {
            mask[base >> 6] = m;
            ntrans += __popcll(m);
        }
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ntrans;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[w];
        bcnt[blockIdx.x] = t;
    }
}

template <class R> struct PhoStage {
    R *x[3], *k[3], *P[3];
    uint64_t *id;
};

template <class R>
__global__ void __launch_bounds__(kBlock) k_gather(PhoDev<R> G, PhoStage<R> T, const uint32_t *idx, const int64_t *book)
{
    const int64_t total = book[1];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[j];
        T.id[j] = G.id[i];
        for (int c = 0; c < 3; ++c) {
            if (G.x[c]) T.x[c][j] = G.x[c][i];
            T.k[c][j] = G.k[c][i];
            T.P[c][j] = G.P[c][i];
        }
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_scatter_back(PhoDev<R> G, PhoStage<R> T, const int64_t *book)
{
    const int64_t total = book[1];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (int64_t)gridDim.x * blockDim.x) {
        G.id[j] = T.id[j];
        for (int c = 0; c < 3; ++c) {
            if (G.x[c]) G.x[c][j] = T.x[c][j];
            G.k[c][j] = T.k[c][j];
            G.P[c][j] = T.P[c][j];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *G.count = total;
}

// ------------------------------------------------------------------ host side
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

FieldDev field_dev(const qed_fields *f)
{
    FieldDev d;
    d.kind = f->kind;
    for (int c = 0; c < 3; ++c) {
        d.E0[c] = f->E0[c];
        d.B0[c] = f->B0[c];
    }
    d.a0 = f->a0;
    d.phase_len = f->phase_len;
    d.inv_phase_len = f->phase_len > 0.0 ? 1.0 / f->phase_len : 0.0;
    return d;
}

StepDev step_dev(const qed_step_params *p)
{
    StepDev s;
    s.t = p->t; s.dt = p->dt; s.a_e = p->a_e; s.eps_r = p->eps_r;
    s.chi_e_min = p->chi_e_min; s.chi_e_max = p->chi_e_max; s.chi_g_min = p->chi_g_min; s.chi_g_max = p->chi_g_max;
    s.k_retire = p->k_retire;
    s.Kc = kAlpha / (sqrt(3.0) * kPi * p->eps_r);
    s.step = p->step; s.seed = p->seed; s.flags = p->flags;
    s.clock = p->d_clock;
    return s;
}

int grid_for(int64_t n)
{
    const int64_t g = cdiv(n > 0 ? n : 1, kBlock);
    return (int)(g < kMaxGrid ? g : kMaxGrid);
}


bool leptons_ok(const qed_leptons *L)
{
    if (!L || !L->d_count || L->capacity < 0 || L->capacity >= (int64_t)1 << 32) return false;
    if (L->species != 0 && L->species != 1) return false;
    for (int c = 0; c < 3; ++c)
        if (!L->p[c] || !L->s[c]) return false;
    return true;
}

bool photons_ok(const qed_photons *G)
{
    if (!G || !G->d_count || !G->d_count_prev || !G->id || G->capacity < 0 || G->capacity >= (int64_t)1 << 32) return false;
    for (int c = 0; c < 3; ++c)
        if (!G->k[c] || !G->P[c]) return false;
    return true;
}

bool fields_ok(const qed_fields *f) { return f && (f->kind == QED_FIELD_UNIFORM || f->kind == QED_FIELD_PLANE_LP); }

template <class R>
qed_status emit_impl(qed_tables T, const qed_leptons *L, const qed_fields *f, const qed_step_params *p,
                     const qed_photons *G, qed_counters *ctr, void *ws, size_t ws_bytes, hipStream_t st)
{
    int64_t nch;
    const WS w = carve(ws, L->capacity, &nch);
    const LepDev<R> ld = lep_dev<R>(L);
    const FieldDev fd = field_dev(f);
    const StepDev sd = step_dev(p);
    unsigned long long *c = (unsigned long long *)ctr;
    const size_t lds_nlc = sizeof(R) * 2 * T->dev.n_chi[0];
    const int g = grid_for(L->capacity);
    QS_LAUNCH(K_LEPTON_MAIN, k_lepton_main<R>, dim3(g), dim3(kBlock), lds_nlc, st, ld, fd, sd, T->dev, w.mask, nch, w.bctr,
              w.bcnt);
    const PhoDev<R> gd = pho_dev<R>((p->flags & QED_EMIT) ? G : nullptr);
    QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask, (const uint32_t *)w.bcnt,
              (const int64_t *)L->d_count, w.book, 0, gd.count, gd.cap, (int64_t *)nullptr, (int64_t)0,
              (int64_t *)nullptr, c, (const uint32_t *)w.bctr, w.idx);
    QS_LAUNCH(K_EMIT_PROCESS, k_emit_process<R>, dim3(g), dim3(kBlock), lds_nlc, st, ld, gd, fd, sd, T->dev, w.mask, nch, w.idx,
                       w.book, c);
    return qs_launch_status(__func__);
}

template <class R>
qed_status pair_impl(qed_tables T, const qed_photons *G, const qed_fields *f, const qed_step_params *p,
                     const qed_leptons *Le, const qed_leptons *Lp, qed_counters *ctr, void *ws, size_t ws_bytes,
                     hipStream_t st)
{
    int64_t nch;
    const WS w = carve(ws, G->capacity, &nch);
    const PhoDev<R> gd = pho_dev<R>(G);
    const FieldDev fd = field_dev(f);
    const StepDev sd = step_dev(p);
    unsigned long long *c = (unsigned long long *)ctr;
    const size_t lds_nbw = sizeof(R) * 2 * T->dev.n_chi[1];
    const int g = grid_for(G->capacity);
    QS_LAUNCH(K_PHOTON_MAIN, k_photon_main<R>, dim3(g), dim3(kBlock), lds_nbw, st, gd, fd, sd, T->dev, w.mask, nch, w.bctr,
              w.bcnt);
    QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask, (const uint32_t *)w.bcnt,
              (const int64_t *)G->d_count_prev, w.book, 1, Le->d_count, Le->capacity, Lp->d_count, Lp->capacity,
              (int64_t *)nullptr, c, (const uint32_t *)w.bctr, w.idx);
    QS_LAUNCH(K_PAIR_PROCESS, k_pair_process<R>, dim3(g), dim3(kBlock), lds_nbw, st, gd, lep_dev<R>(Le), lep_dev<R>(Lp), fd, sd,
                       T->dev, w.mask, nch, w.idx, w.book);
    return qs_launch_status(__func__);
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" size_t qed_workspace_size(int64_t max_particles)
{
    const int64_t cap = max_particles > 0 ? max_particles : 1;
    const int64_t nch = cdiv(cap, 64);
    return align256(sizeof(uint64_t) * 2 * nch) + align256(sizeof(uint32_t) * kMaxGrid) +
           align256(sizeof(int64_t) * 8) + align256(sizeof(uint32_t) * kMaxGrid * kNCtr) + align256(sizeof(uint32_t) * cap);
}

extern "C" qed_status qed_push_spin(const qed_leptons *L, const qed_fields *f, const qed_step_params *p, qed_tables T,
                                    qed_stream stream)
{
    if (!T || !leptons_ok(L) || !p || !fields_ok(f)) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    const FieldDev fd = field_dev(f);
    const StepDev sd = step_dev(p);
    const int g = grid_for(L->capacity);
    if (T->params.precision == QED_F64)
        QS_LAUNCH(K_PUSH, k_push<double>, dim3(g), dim3(kBlock), 0, st, lep_dev<double>(L), fd, sd);
    else
        QS_LAUNCH(K_PUSH, k_push<float>, dim3(g), dim3(kBlock), 0, st, lep_dev<float>(L), fd, sd);
    return qs_launch_status(__func__);
}

extern "C" qed_status qed_emit(qed_tables T, const qed_leptons *L, const qed_fields *f, const qed_step_params *p,
                               const qed_photons *G, qed_counters *ctr, void *ws, size_t ws_bytes, qed_stream stream)
{
    if (!T || !leptons_ok(L) || !p || !fields_ok(f) || !ctr || !ws) return QED_ERR_INVALID;
    if ((p->flags & QED_EMIT) && !photons_ok(G)) return QED_ERR_INVALID;
    if (!(p->dt > 0.0) || !(p->eps_r > 0.0)) return QED_ERR_INVALID;
    if (ws_bytes < qed_workspace_size(L->capacity)) return QED_ERR_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    if (T->params.precision == QED_F64) return emit_impl<double>(T, L, f, p, G, ctr, ws, ws_bytes, st);
    return emit_impl<float>(T, L, f, p, G, ctr, ws, ws_bytes, st);
}

extern "C" qed_status qed_pair(qed_tables T, const qed_photons *G, const qed_fields *f, const qed_step_params *p,
                               const qed_leptons *Le, const qed_leptons *Lp, qed_counters *ctr, void *ws, size_t ws_bytes,
                               qed_stream stream)
{
    if (!T || !photons_ok(G) || !p || !fields_ok(f) || !ctr || !ws) return QED_ERR_INVALID;
    if (!leptons_ok(Le) || !leptons_ok(Lp) || Le->species != 0 || Lp->species != 1) return QED_ERR_INVALID;
    if (!(p->dt > 0.0) || !(p->eps_r > 0.0)) return QED_ERR_INVALID;
    if (ws_bytes < qed_workspace_size(G->capacity)) return QED_ERR_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    if (T->params.precision == QED_F64) return pair_impl<double>(T, G, f, p, Le, Lp, ctr, ws, ws_bytes, st);
    return pair_impl<float>(T, G, f, p, Le, Lp, ctr, ws, ws_bytes, st);
}

__global__ void k_clock_advance(int64_t *clock) { *clock += 1; }

extern "C" qed_status qed_clock_advance(int64_t *d_clock, qed_stream stream)
{
    if (!d_clock) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    QS_LAUNCH(K_SET_PREV, k_clock_advance, dim3(1), dim3(1), 0, st, d_clock);
    return qs_launch_status(__func__);
}

extern "C" size_t qed_compact_workspace_size(const qed_photons *G, qed_precision prec)
{
    if (!G) return 0;
    const size_t es = prec == QED_F64 ? sizeof(double) : sizeof(float);
    int ncomp = 6;
    for (int c = 0; c < 3; ++c) ncomp += G->x[c] != nullptr;
    return qed_workspace_size(G->capacity) + ncomp * align256(es * (G->capacity > 0 ? G->capacity : 1)) +
           align256(sizeof(uint64_t) * (G->capacity > 0 ? G->capacity : 1));
}

template <class R> static qed_status compact_impl(const qed_photons *G, void *ws, hipStream_t st)
{
    int64_t nch;
    const WS w = carve(ws, G->capacity, &nch);
    char *b = (char *)ws + qed_workspace_size(G->capacity);
    const int64_t cap = G->capacity > 0 ? G->capacity : 1;
    PhoStage<R> S;
    for (int c = 0; c < 3; ++c) {
        S.x[c] = nullptr;
        if (G->x[c]) { S.x[c] = (R *)b; b += align256(sizeof(R) * cap); }
    }
    for (int c = 0; c < 3; ++c) { S.k[c] = (R *)b; b += align256(sizeof(R) * cap); }
    for (int c = 0; c < 3; ++c) { S.P[c] = (R *)b; b += align256(sizeof(R) * cap); }
    S.id = (uint64_t *)b;
    const PhoDev<R> gd = pho_dev<R>(G);
    const int g = grid_for(G->capacity);
    QS_LAUNCH(K_ALIVE_MASK, k_alive_mask<R>, dim3(g), dim3(kBlock), 0, st, gd, w.mask, w.bcnt);
    QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask, (const uint32_t *)w.bcnt,
              (const int64_t *)G->d_count, w.book, 2, (int64_t *)nullptr, (int64_t)0, (int64_t *)nullptr, (int64_t)0,
              G->d_count_prev, (unsigned long long *)nullptr, (const uint32_t *)nullptr, w.idx);
    QS_LAUNCH(K_GATHER, k_gather<R>, dim3(g), dim3(kBlock), 0, st, gd, S, w.idx, w.book);
    QS_LAUNCH(K_SCATTER_BACK, k_scatter_back<R>, dim3(g), dim3(kBlock), 0, st, gd, S, w.book);
    return qs_launch_status(__func__);
}

extern "C" qed_status qed_compact(const qed_photons *G, qed_precision prec, void *ws, size_t ws_bytes, qed_stream stream)
{
    if (!photons_ok(G) || !ws) return QED_ERR_INVALID;
    if (prec != QED_F64 && prec != QED_F32) return QED_ERR_INVALID;
    if (ws_bytes < qed_compact_workspace_size(G, prec)) return QED_ERR_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    if (prec == QED_F64) return compact_impl<double>(G, ws, st);
    return compact_impl<float>(G, ws, st);
}
