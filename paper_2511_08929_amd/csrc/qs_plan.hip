// qs_plan.hip -- one whole step (NLC for electrons and positrons, NBW for photons) of any number
// of independent instances in three launches: qed_plan_create / qed_plan_step / qed_plan_destroy.
//
// A plan splits every particle set of every instance into a contiguous range of blocks of one
// block index space ("segments": the electrons and positrons of every instance, then the photons
// of every instance).
//   main     block b streams its share of its segment (lepton push + decision + no-emission
//            update, or the two-phase photon pass) and writes its transition count and event
//            counts (plain stores); leptons and photons are two launches, each with its own
//            register allocation; the first lepton block of an instance also stores the
//            instance's counts and clock at the start of the step;
//   process  each block covers a group of main blocks of one segment: it sums the transition
//            counts it needs (its rank offset in its set, the totals of its instance's sets),
//            derives the append bases from the stored counts, expands its own mask words into
//            an ordered list in LDS and processes its transitions, writing photons (or pairs)
//            at the instance's base + the rank; the first block of an instance stores the new
//            counts and clock, and every 16th block of a set adds event counts to the counters.
// With a learned inverse CDF the processing launch also runs the network on the transitions of
// each block (inputs and outputs stay in LDS).
// No block waits for another and no fence orders blocks: every hand-over is a launch boundary
// on the stream.  (On this chip the L2 is per XCD, so a device-scope release or acquire fence
// inside a kernel writes back or invalidates a whole L2.)
// The appends keep the order of the per-species calls: photons of electrons, then of
// positrons, in emitter order; pairs in photon order.  So a plan step gives the same particles,
// bit for bit, as qed_emit(electrons), qed_emit(positrons), qed_pair, qed_clock_advance.
#include <algorithm>
#include <vector>

#include "qs_mlp.hpp"

namespace {
using namespace qs;

template <class R> struct InstDev {
    LepDev<R> E, P;
    PhoDev<R> G;
    FieldDev F;
    StepDev S;
    unsigned long long *ctr;
    int se, sp, sg;            // segment indices (-1: set not stepped)
};

struct SegDev {
    int kind;                  // 0 electrons, 1 positrons, 2 photons
    int inst;
    int b0, nb;                // block range of the streaming pass
    int pb0, npb;              // block range of the processing pass (one block per `group` streaming blocks)
    int64_t mask_off, nchunks; // decision plane at mask + mask_off, branch plane nchunks words later
};

// a processing block's view of its set's bookkeeping
struct SegBook {
    int64_t n_main;            // particles the main pass covered
    int64_t base, base2;       // append base (photons; pairs: electrons, positrons)
    int64_t total, nfit;       // transitions, of which stored
};

// An instance's counts and step clock at the start of a step (written by the lepton streaming
// pass, read by the processing pass that does the bookkeeping itself)
struct Snap {
    int64_t ne, np, gb, ng, clock;
};

// Streaming block ranges [b0, b1) of an instance's electron, positron and photon sets (empty
// ranges for sets that are not stepped)
struct InstSeg {
    int e0, e1, p0, p1, g0, g1;
};

struct PlanDev {
    const SegDev *seg;
    int nseg, nblk, ninst;
    int group;                 // streaming blocks per processing block
    uint64_t *mask;
    uint32_t *bcnt;            // [nblk]
    uint32_t *bctr;            // [nblk][kNCtr] event counts of each main block
    const int *bseg, *binst;   // [nblk] segment and instance of each streaming block
    const int4 *pbd;           // [npb] processing block: segment, streaming blocks [mb0, mb1), instance
    const InstSeg *iseg;       // [ninst]
    Snap *snap;                // [ninst]
    MlpDev mlp[2];             // learned inverse CDF of NLC and NBW, used where mlp_on is set
    int mlp_on[2];
    uint32_t *bsub;            // [lepton streaming blocks][kSubRounds] photons per sub-cycling round
};

// The streaming pass runs as two launches with their own register allocation: PHO = 0 over the
// lepton segments (blocks [0, nblk_lep)), PHO = 1 over the photon segments (the rest).  Waves per
// SIMD in FP32: three for the photon pass of the general field variant (which spills at four),
// four otherwise.  PV, the photon pass's launch variant (a tuning dimension of the plan): 0 tiles
// of 1024 slots; 1 tiles of 512 (half the LDS queue); 2 tiles of 1024 at three waves per SIMD
// (up to 168 registers) with the next tile's reads issued before the current tile's phase 2,
// which needs the room (at four waves the reads held through phase 2 spill).
template <int PV> constexpr int pho_tile() { return PV == 1 ? 512 : kPhoTile; }

template <class R, int PHO, int DEC, int FLD, int PV = 0>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? ((PHO == 1 && (FLD == kFldGeneral || PV == 2)) ? 3 : 4) : 1,
                                   PV == 2 ? 3 : 8)))
k_plan_main(const InstDev<R> *inst, PlanDev P, TablesDev T, int b_first)
{
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    constexpr int TILE = pho_tile<PV>();
    __shared__ PhoQueue<R, TILE, queue_kind<R, FLD>()> Q;
    __shared__ unsigned tot[kNCtr + 1];
    const int b = b_first + blockIdx.x;
    const int sj = P.bseg[b];
    const SegDev sg = P.seg[sj];
    // local copies of the instance's views: the particle stores below may not alias them, so
    // they stay in registers instead of being re-read from global memory after every store
    const InstDev<R> *Ip = inst + P.binst[b];
    const StepDev S = localize(Ip->S);
    const FieldDev F = Ip->F;
    uint64_t *mask = P.mask + sg.mask_off;
    unsigned v[kNCtr + 1] = {};
    if (!PHO) {
        const LepDev<R> L = sg.kind == 0 ? Ip->E : Ip->P;
        if (sg.kind == 0 && b == sg.b0 && threadIdx.x == 0) {
            Snap sn;
            sn.ne = *Ip->E.count;
            sn.np = Ip->sp >= 0 ? *Ip->P.count : 0;
            sn.gb = Ip->G.count != nullptr ? *Ip->G.count : 0;
            sn.ng = Ip->sg >= 0 ? *Ip->G.count_prev : 0;
            sn.clock = Ip->S.clock ? *Ip->S.clock : 0;
            P.snap[P.binst[b]] = sn;
        }
        stage_rates<R>(T, 0, lds);
        const int64_t n = *L.count;
        const int64_t B = block_len(n, sg.nb);
        const int64_t start = (int64_t)(b - sg.b0) * B, end = start + B < n ? start + B : n;
        LCount c;
        lepton_range<R, DEC, FLD>(L, F, S, T, lds, start, end, mask, sg.nchunks, c);
        v[C_PROB] = c.prob; v[C_CHI] = c.chi; v[C_NORM] = c.norm; v[C_LSTEP] = c.step; v[C_NONFIN] = c.nonfin;
        v[kNCtr] = c.trans;
        if constexpr ((DEC & 8) != 0) {
            if (L.sub) {
                // sub-cycling: the block's photons per round, and its photons in all (not its
                // transitions) as the count the processing pass ranks and books
                __shared__ unsigned rsum[kSubRounds][kBlock / 64];
                unsigned ph = 0;
#pragma unroll
                for (int r = 0; r < kSubRounds; ++r) {
                    unsigned t = c.rnd[r];
                    ph += t;
                    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
                    if ((threadIdx.x & 63) == 0) rsum[r][threadIdx.x >> 6] = t;
                }
                v[kNCtr] = ph;
                __syncthreads();
                if (threadIdx.x < kSubRounds) {
                    unsigned t = 0;
#pragma unroll
                    for (int w = 0; w < kBlock / 64; ++w) t += rsum[threadIdx.x][w];
                    P.bsub[(int64_t)b * kSubRounds + threadIdx.x] = t;
                }
            }
        }
    } else {
        const PhoDev<R> G = Ip->G;
        stage_rates<R>(T, 1, lds);
        const int64_t n = *G.count_prev;
        const int64_t B = block_len(n, sg.nb);
        const int64_t start = (int64_t)(b - sg.b0) * B, end = start + B < n ? start + B : n;
        GCount c;
        if constexpr (PV == 2) {                      // the next tile's reads issued early
            TileIn<R, TILE> in;
            if (start < end) photon_tile_load<R, TILE>(G, start, start + TILE < end ? start + TILE : end, in);
            for (int64_t tile = start; tile < end; tile += TILE) {
                const int64_t nt = tile + TILE;
                photon_tile<R, FLD, TILE, true>(G, F, S, T, lds, Q, tile, nt < end ? nt : end, mask, sg.nchunks, c, &in,
                                                nt < end ? nt : -1, nt + TILE < end ? nt + TILE : end);
            }
        } else {
            for (int64_t tile = start; tile < end; tile += TILE)
                photon_tile<R, FLD, TILE>(G, F, S, T, lds, Q, tile, tile + TILE < end ? tile + TILE : end, mask,
                                          sg.nchunks, c);
        }
        v[C_PROB] = c.prob; v[C_CHI] = c.chi; v[C_NORM] = c.norm; v[C_RETIRED] = c.ret; v[C_GSTEP] = c.step;
        v[C_GQED] = c.qed; v[C_NONFIN] = c.nonfin; v[kNCtr] = c.trans;
    }
    block_sum(v, tot);
    if (threadIdx.x < kNCtr) P.bctr[(int64_t)b * kNCtr + threadIdx.x] = tot[threadIdx.x];
    else if (threadIdx.x == kNCtr) P.bcnt[b] = tot[kNCtr];
}

constexpr int kExpandWords = kBlock; // mask words expanded per round of the process pass, one per thread (16384 slots)
constexpr int kStage = kSubRounds * 6;  // per lepton slot with sub-cycling: k and P-vector of each round's photon

// The set bits of the mask words [c0, c1) (word c0 + t given as m by thread t, 0 past c1) as
// positions 64 (word - c0) + bit in slot order, into list; returns their number.  Block-wide.
__device__ __forceinline__ uint32_t mask_list(uint64_t m, uint16_t *list, uint32_t *wtot, uint32_t *nlist)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t pc = __popcll(m);
    uint32_t incl = pc;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wid] = incl;
    __syncthreads();
    uint32_t pos = incl - pc;
    for (int w = 0; w < wid; ++w) pos += wtot[w];
    uint64_t bits = m;
    while (bits) {
        const int bit = __ffsll((long long)bits) - 1;
        list[pos++] = (uint16_t)(threadIdx.x * 64 + bit);
        bits &= bits - 1;
    }
    if (threadIdx.x == kBlock - 1) *nlist = pos;
    __syncthreads();
    return *nlist;
}

// Sub-cycled leptons of the merged step (QED_SUBCYCLE), `split` blocks per lepton streaming block
// (each over an equal share of its mask words: kBlock slots at most, unless the launch would exceed
// its cap on blocks), between the streaming and
// the processing launches.  A block gathers the leptons of its share that the streaming pass
// flagged (branch bit without a transition), runs all sub-steps of each on full waves, and books
// their photons per round: the rounds with a photon in the lepton's sub-step word, its transition
// bit if it has one, and its photon counts per round and in all and its event counts added
// atomically to the streaming block's (the order of the photons comes from the processing pass's
// ranks, not from these sums).  Every lepton is finished here (its state after
// the sub-steps stored), and the momentum and P-vector of each photon its sub-steps make are kept
// in its slot's staging entries, which the processing pass copies to the photons' places.
// Its waves hold long dependent chains (the sub-steps of one lepton run one after the other), so it
// is held to two waves per SIMD in FP64 (one otherwise) and three in FP32.
template <class R, int FLD>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2)))
k_plan_sub(const InstDev<R> *inst, PlanDev P, TablesDev T, int split)
{
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    __shared__ uint16_t list[kExpandWords * 64];
    __shared__ uint32_t nlist, wtot[kBlock / 64];
    __shared__ unsigned red[kSubRounds + 3][kBlock / 64];
    const int b = blockIdx.x / split, q = blockIdx.x - b * split;
    const SegDev sg = P.seg[P.bseg[b]];
    const InstDev<R> *Ip = inst + P.binst[b];
    const LepDev<R> L = sg.kind == 0 ? Ip->E : Ip->P;
    if (!L.sub) return;                                // block-uniform: this set does not sub-cycle
    const StepDev S = localize(Ip->S);
    const FieldDev F = Ip->F;
    uint64_t *mask = P.mask + sg.mask_off;
    const int64_t n = *L.count;
    const int64_t B = block_len(n, sg.nb);
    const int64_t start = (int64_t)(b - sg.b0) * B, end = start + B < n ? start + B : n;
    // this block's share of the streaming block's mask words: [w0, w1)
    const int64_t wl = cdiv(end, 64), wq = cdiv(B >> 6, split);
    const int64_t w0 = (start >> 6) + q * wq < wl ? (start >> 6) + q * wq : wl;
    const int64_t w1 = w0 + wq < wl ? w0 + wq : wl;
    LCount c;
    bool staged = false;                               // block-uniform: the rate rows are in LDS
    for (int64_t c0 = w0; c0 < w1; c0 += kExpandWords) {
        const int64_t c1 = c0 + kExpandWords < w1 ? c0 + kExpandWords : w1;
        const int64_t cw = c0 + threadIdx.x;
        const uint32_t nl = mask_list(cw < c1 ? mask[sg.nchunks + cw] & ~mask[cw] : 0ull, list, wtot, &nlist);
        if (nl && !staged) {
            stage_rates<R>(T, 0, lds);
            staged = true;
        }
        for (uint32_t j = threadIdx.x; j < nl; j += kBlock) {
            const int64_t i = c0 * 64 + list[j];
            const V3<R> x = ldx(L.x, i);
            V3<R> p = ld3(L.p, i), s = ld3(L.s, i);
            V3<R> E, Bf;
            eval_fields<R, FLD>(F, (double)x.x, (double)x.y, S.t + S.dt, E, Bf);
            const int m = min((int)(L.sub[i] >> 16), kSubLog2Max);    // the loop's stride stays >= 1
            unsigned em = 0;
            // chi, the basis and the rates hold until an emission changes the momentum.  Each lane
            // runs its no-emission sub-steps up to its next emission, then the lanes that reached
            // one emit together: a wave runs the emission code once per emission of its busiest
            // lepton, not once per sub-step in which some lepton emits.
            LDecide<R> g;
            lepton_geom<R>(S, T, lds, L.species, p, E, Bf, g);
            const int stride = kSubRounds >> m;
            int r = 0;
            while (r < kSubRounds) {
                LDecide<R> d;
                bool emit = false;
                for (; r < kSubRounds; r += stride) {
                    StepDev Sr = S;
                    Sr.sub_round = r;
                    d = g;
                    lepton_draw<R>(Sr, L.species, i, s, d);
                    if (substep_decide<R>(Sr, m, d, s, &c)) {
                        emit = true;
                        break;
                    }
                }
                if (!emit) break;
                StepDev Sr = S;
                Sr.sub_round = r;
                V3<R> k, Pv;
                substep_emit<R>(Sr, T, d, L.species, i, p, s, k, Pv, &c);
                em |= 1u << r;
                R *st = L.stage + ((int64_t)i * kSubRounds + r) * 6;
                st[0] = k.x; st[1] = k.y; st[2] = k.z;
                st[3] = Pv.x; st[4] = Pv.y; st[5] = Pv.z;
                lepton_geom<R>(S, T, lds, L.species, p, E, Bf, g);
                r += stride;
            }
#pragma unroll
            for (int r = 0; r < kSubRounds; ++r) c.rnd[r] += (em >> r) & 1u;
            if (em) {
                L.sub[i] = ((unsigned)m << 16) | em;
                atomicOr(reinterpret_cast<unsigned long long *>(mask + (i >> 6)), 1ull << (i & 63));
            }
            st3(L.p, i, p);
            st3(L.s, i, s);
        }
        __syncthreads();
    }
    if (!staged) return;                               // no flagged lepton in this share: nothing to add
    // the block's bookkeeping, added to its streaming block's entries (the other blocks of the
    // streaming block add theirs)
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k2 = 0; k2 < kSubRounds + 3; ++k2) {
        unsigned t = k2 < kSubRounds ? c.rnd[k2] : (k2 == kSubRounds ? c.chi : (k2 == kSubRounds + 1 ? c.prob : c.norm));
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) red[k2][wid] = t;
    }
    __syncthreads();
    __shared__ unsigned tot[kSubRounds + 3];
    if (threadIdx.x < kSubRounds + 3) {
        unsigned t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += red[threadIdx.x][w];
        tot[threadIdx.x] = t;
        uint32_t *dst = threadIdx.x < kSubRounds ? P.bsub + (int64_t)b * kSubRounds + threadIdx.x
                        : P.bctr + (int64_t)b * kNCtr + (threadIdx.x == kSubRounds ? C_CHI : threadIdx.x == kSubRounds + 1 ? C_PROB : C_NORM);
        if (t) atomicAdd(dst, t);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned ph = 0;
        for (int r = 0; r < kSubRounds; ++r) ph += tot[r];
        if (ph) atomicAdd(P.bcnt + b, ph);
    }
}

constexpr int kAggGroups = 16;   // processing blocks per event-count aggregation (fused bookkeeping)

// Sums of a[0..3] over the block (every thread gets them); red: LDS.  Synchronizes.
__device__ __forceinline__ void block_totals4(unsigned long long (&a)[4], unsigned long long (*red)[kBlock / 64])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        for (int o = 32; o > 0; o >>= 1) a[k] += __shfl_xor(a[k], o);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = a[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = 0;
        for (int w = 0; w < kBlock / 64; ++w) a[k] += red[k][w];
    }
}

// LDS of the learned inverse CDF in the processing pass: per wave the forward pass's rows, per
// thread one transition's raw inputs and nu
template <bool SUR> struct SurLds {
    MlpFwdWave wv[kBlock / 64];
    float xin[kBlock][3];
    float nu[kBlock];
};
template <> struct SurLds<false> {
    int unused;
};

// One launch over the processing blocks of every set (lepton sets first, then photons); the
// channel follows the block's set.  No bookkeeping launch precedes it: each block sums the
// transition counts it needs (its rank offset inside its set, the totals of its instance's
// sets) and derives its append base from the counts at the start of the step; the first block
// of an instance's electron set stores the new counts, the counters and the next clock (no block
// of this launch reads them), and every kAggGroups-th block of a set adds the event counts of its
// streaming blocks to the instance's counters.
// SUR: a process with a learned inverse CDF (P.mlp_on) handles its transitions in rounds of one
// per thread: each thread writes its transition's network inputs to LDS, the waves run the
// network on the round's rows (16 per forward pass), and each thread finishes its transition
// with its nu (coarse table + network), or with the table inverse CDF where the tables judged
// the network out of bound.
// SUB: lepton sets with sub-cycling (their LepDev::sub set) place each lepton's photons round by
// round: all of a set's round-r photons, in lepton order, before its round-r+1 photons, as the
// per-species calls do.  The sub-step launch ran the sub-steps, counted each block's photons per
// round and kept them; here each photon is copied to its round's offset plus its rank, and a
// lepton the streaming pass chose to emit in its one step (round 0) is processed as usual.
template <class R, int FLD, bool SUR, bool SUB = false>
__global__ void __launch_bounds__(kBlock) k_plan_process(const InstDev<R> *inst, PlanDev P, TablesDev T, int b_first)
{
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    __shared__ uint16_t list[kExpandWords * 64];
    __shared__ uint32_t nlist, wtot[kBlock / 64];
    __shared__ unsigned long long red[4][kBlock / 64];
    __shared__ SurLds<SUR> sl;
    // this block covers the streaming blocks [mb0, mb1) of one segment: a contiguous slot range
    const int4 pd = P.pbd[b_first + blockIdx.x];
    const int sj = pd.x, mb0 = pd.y, mb1 = pd.z;
    const SegDev sg = P.seg[sj];
    const InstDev<R> *Ip = inst + pd.w;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // transitions of this block's streaming blocks: one load per lane, a wave sum
    uint32_t mine = 0;
    for (int b = mb0 + lane; b < mb1; b += 64) mine += P.bcnt[b];
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
    const bool lead = sg.kind == 0 && mb0 == sg.b0;
    const bool agg = ((mb0 - sg.b0) / P.group) % kAggGroups == 0;
    if (mine == 0 && !lead && !agg) return;           // block-uniform
    const InstSeg is = P.iseg[pd.w];
    const Snap sn = P.snap[pd.w];
    if (agg && threadIdx.x < 64) {
        const int bend = mb0 + kAggGroups * P.group < sg.b0 + sg.nb ? mb0 + kAggGroups * P.group : sg.b0 + sg.nb;
        unsigned long long v[kNCtr] = {};
        for (int b = mb0 + lane; b < bend; b += 64)
#pragma unroll
            for (int c = 0; c < kNCtr; ++c) v[c] += P.bctr[(int64_t)b * kNCtr + c];
        // every sum first (independent shuffle chains), then the atomics through one pointer read
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int c = 0; c < kNCtr; ++c) v[c] += __shfl_xor(v[c], o);
        if (lane == 0) {
            unsigned long long *ctr = Ip->ctr;
#pragma unroll
            for (int c = 0; c < kNCtr; ++c)
                if (v[c]) atomicAdd(ctr + c, v[c]);
        }
    }
    // transition counts: rank offset inside the set, totals of the sets this block needs;
    // every load first (independent), then the sums
    const bool ne_ = sg.kind != 2 || lead, np_ = sg.kind == 1 || lead, ng_ = sg.kind == 2 || lead;
    unsigned long long a[4] = {0, 0, 0, 0};
    auto range_sum = [&](int lo, int hi) -> unsigned long long {
        unsigned long long t = 0;
#pragma unroll 4
        for (int b = lo + (int)threadIdx.x; b < hi; b += kBlock) t += P.bcnt[b];
        return t;
    };
    a[0] = range_sum(sg.b0, mb0);
    if (ne_) a[1] = range_sum(is.e0, is.e1);
    if (np_) a[2] = range_sum(is.p0, is.p1);
    if (ng_) a[3] = range_sum(is.g0, is.g1);
    block_totals4(a, red);
    int64_t rank0 = (int64_t)a[0];
    const int64_t te = (int64_t)a[1], tp = (int64_t)a[2], tg = (int64_t)a[3];
    // append bases and capacity clamps from the counts at the start of the step
    const bool has_g = Ip->G.count != nullptr, pair = Ip->sg >= 0;
    const int64_t room_g = has_g && Ip->G.cap - sn.gb > 0 ? Ip->G.cap - sn.gb : 0;
    const int64_t nfe = te < room_g ? te : room_g;
    const int64_t nfp = tp < room_g - nfe ? tp : room_g - nfe;
    int64_t room_p = Ip->E.cap - sn.ne < Ip->P.cap - sn.np ? Ip->E.cap - sn.ne : Ip->P.cap - sn.np;
    room_p = room_p > 0 ? room_p : 0;
    const int64_t nfg = tg < room_p ? tg : room_p;
    SegBook bk;
    if (sg.kind == 0) bk = SegBook{sn.ne, sn.gb, 0, te, nfe};
    else if (sg.kind == 1) bk = SegBook{sn.np, sn.gb + nfe, 0, tp, nfp};
    else bk = SegBook{sn.ng, sn.ne, sn.np, tg, nfg};
    if (lead && threadIdx.x == 0) {
        unsigned long long *ctr = Ip->ctr;
        int64_t over = 0;
        if (has_g) {
            const int64_t gnew = sn.gb + nfe + nfp;
            *Ip->G.count = gnew;
            over += (te - nfe) + (tp - nfp);
            if (te + tp) atomicAdd(ctr + C_EMIT, (unsigned long long)(te + tp));
            // photons born in this step wait for the next one
            if (pair) *Ip->G.count_prev = gnew;
        }
        if (pair) {
            *Ip->E.count = sn.ne + nfg;
            *Ip->P.count = sn.np + nfg;
            over += tg - nfg;
            if (tg) atomicAdd(ctr + C_PAIR, (unsigned long long)tg);
        }
        if (over) atomicAdd(ctr + C_OVER, (unsigned long long)over);
        if (Ip->S.clock) *const_cast<int64_t *>(Ip->S.clock) = sn.clock + 1;
    }
    if (mine == 0) return;                             // block-uniform
    StepDev S = Ip->S;
    S.step += sn.clock;
    S.t += (double)sn.clock * S.dt;
    const FieldDev F = Ip->F;
    const int PHO = sg.kind == 2;
    // single precision: the Bessel quadrature nodes (6 KB) join the rate rows in LDS, so the
    // node-by-node sums of the emitters and pairs read LDS instead of L2
    __shared__ float4 bnodes[sizeof(R) == 4 ? kBn32Nodes : 1];
    TablesDev Tl = T;
    if (sizeof(R) == 4) {
        const float4 *src = reinterpret_cast<const float4 *>(T.bn32);
        for (int j = threadIdx.x; j < kBn32Nodes; j += kBlock) bnodes[j] = src[j];
        Tl.bn32 = reinterpret_cast<const float *>(bnodes);
    }
    stage_rates<R>(T, PHO, lds);                      // (its barrier also covers the nodes)
    const uint64_t *mask = P.mask + sg.mask_off;
    const int64_t n = bk.n_main;
    const int64_t B = block_len(n, sg.nb);
    const int64_t start = (int64_t)(mb0 - sg.b0) * B;
    const int64_t end = (int64_t)(mb1 - sg.b0) * B < n ? (int64_t)(mb1 - sg.b0) * B : n;
    const bool net = SUR && P.mlp_on[PHO];
    unsigned c_ret = 0;
    // sub-cycling: this block's first photon of each round, and per entry of a round of the list
    // its rank among the round's photons of that round of entries
    __shared__ unsigned long long sub_off[SUB ? kSubRounds : 1];
    __shared__ unsigned sub_wt[SUB ? kSubRounds : 1][kBlock / 64];
    __shared__ unsigned sub_pos[SUB ? kSubRounds : 1][SUB ? kBlock : 1];
    bool subm = false;
    if constexpr (SUB) {
        subm = !PHO && (sg.kind == 0 ? Ip->E.sub : Ip->P.sub) != nullptr;        // block-uniform
        if (subm) {
            // per round: the set's photons (all its streaming blocks) and those of the blocks before
            // this one, summed block-wide
            __shared__ unsigned red32[2 * kSubRounds][kBlock / 64];
            unsigned tot[kSubRounds] = {}, pre[kSubRounds] = {};
            for (int bb = sg.b0 + (int)threadIdx.x; bb < sg.b0 + sg.nb; bb += kBlock) {
                const uint4 *q = reinterpret_cast<const uint4 *>(P.bsub + (int64_t)bb * kSubRounds);
#pragma unroll
                for (int u = 0; u < kSubRounds / 4; ++u) {
                    const uint4 vv = q[u];
                    tot[4 * u] += vv.x; tot[4 * u + 1] += vv.y; tot[4 * u + 2] += vv.z; tot[4 * u + 3] += vv.w;
                    if (bb < mb0) {
                        pre[4 * u] += vv.x; pre[4 * u + 1] += vv.y; pre[4 * u + 2] += vv.z; pre[4 * u + 3] += vv.w;
                    }
                }
            }
#pragma unroll
            for (int k2 = 0; k2 < 2 * kSubRounds; ++k2) {
                unsigned t = k2 < kSubRounds ? tot[k2] : pre[k2 - kSubRounds];
                for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
                if (lane == 0) red32[k2][wid] = t;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                unsigned long long run = 0;
                for (int r = 0; r < kSubRounds; ++r) {
                    unsigned long long tr = 0, pr = 0;
                    for (int w = 0; w < kBlock / 64; ++w) {
                        tr += red32[r][w];
                        pr += red32[kSubRounds + r][w];
                    }
                    sub_off[r] = run + pr;
                    run += tr;
                }
            }
            __syncthreads();
        }
    }
    for (int64_t c0 = start >> 6; c0 < cdiv(end, 64); c0 += kExpandWords) {
        const int64_t c1 = c0 + kExpandWords < cdiv(end, 64) ? c0 + kExpandWords : cdiv(end, 64);
        // one mask word per thread; positions by a block-wide exclusive scan of the popcounts
        const int64_t c = c0 + threadIdx.x;
        const uint64_t m = c < c1 ? mask[c] : 0ull;
        const uint32_t pc = __popcll(m);
        uint32_t incl = pc;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wtot[wid] = incl;
        __syncthreads();
        uint32_t pos = incl - pc;
        for (int w = 0; w < wid; ++w) pos += wtot[w];
        uint64_t bits = m;
        while (bits) {
            const int bit = __ffsll((long long)bits) - 1;
            list[pos++] = (uint16_t)(threadIdx.x * 64 + bit);
            bits &= bits - 1;
        }
        if (threadIdx.x == kBlock - 1) nlist = pos;
        __syncthreads();
        const uint32_t nl = nlist;
        // transition j of this round: emitter (photon into slot base + rank) or decaying photon
        auto item = [&](uint32_t j, const float *nu_in, float *x_out) {
            const int64_t i = c0 * 64 + list[j];
            const int64_t r = rank0 + j;
            const bool br = (mask[sg.nchunks + (i >> 6)] >> (i & 63)) & 1ull;
            if (!PHO)
                emit_item<R, FLD>(sg.kind == 0 ? Ip->E : Ip->P, Ip->G, F, S, Tl, lds, i, br, r < bk.nfit ? bk.base + r : -1,
                                   c_ret, nu_in, x_out);
            else
                pair_item<R, FLD>(Ip->G, Ip->E, Ip->P, F, S, Tl, lds, i, br, r < bk.nfit ? bk.base + r : -1, bk.base2 + r,
                                   nu_in, x_out);
        };
        if (net) {
            if constexpr (SUR) {
                const MlpDev &M = P.mlp[PHO];
                for (uint32_t j0 = 0; j0 < nl; j0 += kBlock) {
                    const uint32_t j = j0 + threadIdx.x;
                    const int rows = nl - j0 < (uint32_t)kBlock ? (int)(nl - j0) : kBlock;
                    if (j < nl) item(j, nullptr, sl.xin[threadIdx.x]);
                    __syncthreads();
                    // every wave runs the same number of forward passes (they synchronize the block)
                    const int calls = (int)cdiv(cdiv(rows, 16), kBlock / 64);
                    MlpFwdWave &W = sl.wv[wid];
                    for (int k = 0; k < calls; ++k) {
                        const int row = (k * (kBlock / 64) + wid) * 16 + (lane & 15);
                        if (lane < 16) {
                            float xo[3] = {0.0f, 0.0f, 1.0f};
                            if (row < rows) mlp_normalize(M, sl.xin[row], xo);
                            W.x[lane][0] = xo[0]; W.x[lane][1] = xo[1]; W.x[lane][2] = xo[2];
                        }
                        __syncthreads();
                        const float y = mlp_forward(M, W);
                        if (lane < 16 && row < rows) sl.nu[row] = mlp_base(M, sl.xin[row]) + M.out_s * y;
                        __syncthreads();
                    }
                    // in a cell the tables judged the network out of bound, the table inverse CDF
                    if (j < nl) item(j, mlp_masked(M, sl.xin[threadIdx.x]) ? nullptr : &sl.nu[threadIdx.x], nullptr);
                    __syncthreads();
                }
            }
        } else if (SUB && subm) {
            if constexpr (SUB) {
                const LepDev<R> &Ls = sg.kind == 0 ? Ip->E : Ip->P;
                const uint64_t below = (1ull << lane) - 1ull;
                for (uint32_t j0 = 0; j0 < nl; j0 += kBlock) {
                    const uint32_t j = j0 + threadIdx.x;
                    const int64_t i = c0 * 64 + (j < nl ? list[j] : 0);
                    const uint32_t wsub = j < nl ? Ls.sub[i] : 0u;
#pragma unroll
                    for (int r = 0; r < kSubRounds; ++r) {
                        const uint64_t bm = __ballot((wsub >> r) & 1u);
                        if (lane == 0) sub_wt[r][wid] = (unsigned)__popcll(bm);
                        sub_pos[r][threadIdx.x] = (unsigned)__popcll(bm & below);
                    }
                    __syncthreads();
                    if (j < nl) {
#pragma unroll
                        for (int r = 0; r < kSubRounds; ++r)
                            for (int w = 0; w < wid; ++w) sub_pos[r][threadIdx.x] += sub_wt[r][w];
                        if ((wsub >> 16) != 0) {
                            // sub-cycled: the sub-step launch finished the lepton and kept the
                            // momentum and P-vector of each of its photons
                            const V3<R> x = ldx(Ls.x, i);
                            for (int r = 0; r < kSubRounds; ++r)
                                if ((wsub >> r) & 1u) {
                                    const int64_t q = (int64_t)(sub_off[r] + sub_pos[r][threadIdx.x]);
                                    if (q < bk.nfit) {
                                        const R *st = Ls.stage + ((int64_t)i * kSubRounds + r) * 6;
                                        StepDev Sr = S;
                                        Sr.sub_round = r;
                                        store_photon<R>(Ip->G, Sr, Ls.species, i, bk.base + q, x, v3<R>(st[0], st[1], st[2]),
                                                        v3<R>(st[3], st[4], st[5]), c_ret);
                                    }
                                }
                        } else {
                            // one step (the emission the streaming pass decided, its branch in the
                            // mask as in the plain path): its photon is in round 0
                            const int64_t q = (int64_t)(sub_off[0] + sub_pos[0][threadIdx.x]);
                            const bool br = (mask[sg.nchunks + (i >> 6)] >> (i & 63)) & 1ull;
                            emit_item<R, FLD>(Ls, Ip->G, F, S, Tl, lds, i, br, q < bk.nfit ? bk.base + q : -1, c_ret);
                        }
                    }
                    __syncthreads();
                    if (threadIdx.x < kSubRounds) {
                        unsigned t = 0;
                        for (int w = 0; w < kBlock / 64; ++w) t += sub_wt[threadIdx.x][w];
                        sub_off[threadIdx.x] += t;
                    }
                    __syncthreads();
                }
            }
        } else {
            for (uint32_t j = threadIdx.x; j < nl; j += blockDim.x) item(j, nullptr, nullptr);
        }
        rank0 += nl;
        __syncthreads();
    }
    block_add(Ip->ctr, C_RETIRED, c_ret);
}

}  // namespace

struct qed_plan_s {
    qed_tables T;
    int ninst, nseg, nblk, nblk_lep, npb, npb_lep, group;
    void *d_inst;
    SegDev *d_seg;
    uint64_t *d_mask;
    uint32_t *d_bcnt;
    uint32_t *d_bsub;          // sub-cycling: photons per round of each lepton streaming block
    uint32_t *d_sub;           // sub-cycling: the sub-step word of every slot of those lepton sets
    void *d_stage;             // ... and the photons of each slot's sub-steps (kStage values of R)
    int sub;                   // some instance sub-cycles
    int sub_split;             // sub-step blocks per lepton streaming block (kBlock slots or fewer each)
    hipStream_t side;          // sub-cycling: the sub-step launch runs here, beside the photon pass
    hipEvent_t fork, join;
    uint32_t *d_bctr;
    int *d_bseg, *d_binst;
    int4 *d_pbd;
    InstSeg *d_iseg;
    Snap *d_snap;
    qed_surrogate sur[2];      // learned inverse CDF per process (NULL: tables)
    FieldDev *h_grid;          // [ninst] host copy of each instance's fields (grid instances only)
    float4 **h_gn;             // [ninst] the plan's interleaved copy of that grid, or NULL
    int dec;                   // decision variants needed (bit 0: optical depth, bit 1: rejection)
    int fv;                    // field-model variant the instances need (the largest of field_variant)
    int pv;                    // photon pass launch variant (single precision, plain fields)
    int flep;                  // the lepton pass's (the largest of lepton_variant)
    size_t lds;
};

namespace {

template <class R> InstDev<R> inst_dev(const qed_instance *in)
{
    InstDev<R> d;
    memset(&d, 0, sizeof(d));
    d.E = lep_dev<R>(&in->electrons);
    d.P = lep_dev<R>(&in->positrons);
    d.G = pho_dev<R>((in->params.flags & (QED_EMIT | QED_PAIR)) ? &in->photons : nullptr);
    d.F = field_dev(&in->fields);
    d.S = step_dev(&in->params);
    d.ctr = (unsigned long long *)in->d_counters;
    d.se = d.sp = d.sg = -1;
    return d;
}

void plan_free(qed_plan p)
{
    if (!p) return;
    (void)hipFree(p->d_inst);
    (void)hipFree(p->d_seg);
    (void)hipFree(p->d_mask);
    (void)hipFree(p->d_bcnt);
    (void)hipFree(p->d_bsub);
    (void)hipFree(p->d_sub);
    (void)hipFree(p->d_stage);
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->join) (void)hipEventDestroy(p->join);
    if (p->side) (void)hipStreamDestroy(p->side);
    (void)hipFree(p->d_bctr);
    (void)hipFree(p->d_bseg);
    (void)hipFree(p->d_binst);
    (void)hipFree(p->d_pbd);
    (void)hipFree(p->d_iseg);
    (void)hipFree(p->d_snap);
    if (p->h_gn)
        for (int i = 0; i < p->ninst; ++i)
            if (p->h_gn[i]) (void)hipFree(p->h_gn[i]);
    free(p->h_gn);
    free(p->h_grid);
    delete p;
}

// the caller's six grid arrays, interleaved two float4 per node (the plan's copy of the step)
__global__ void __launch_bounds__(kBlock) k_pack_grid(FieldDev f, float4 *gn)
{
    const int64_t n = (int64_t)f.nx * f.ny;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        gn[2 * i] = make_float4(f.g[0][i], f.g[1][i], f.g[2][i], f.g[3][i]);
        gn[2 * i + 1] = make_float4(f.g[4][i], f.g[5][i], 0.0f, 0.0f);
    }
}

// Default cap on the blocks of one set: one resident round of the photon streaming kernel on
// this device (compute units x blocks per compute unit at its register and LDS use), so that a
// set's blocks all run at once instead of in a ragged second round.
template <class R> int resident_blocks(size_t lds, int pv)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kMaxGrid;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return kMaxGrid;
    hipError_t e;
    if (pv == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_plan_main<R, 1, 0, kFldPlain, 1>, kBlock, lds);
    else if (pv == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_plan_main<R, 1, 0, kFldPlain, 2>, kBlock, lds);

    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_plan_main<R, 1, 0, kFldPlain>, kBlock, lds);
    if (e != hipSuccess || per_cu <= 0) return kMaxGrid;
    return cus * per_cu;
}

template <class R>
qed_status plan_create(qed_tables T, int n, const qed_instance *in, int ppb, int maxb, int group, int pv,
                       qed_surrogate s_nlc, qed_surrogate s_nbw, qed_plan *out)
{
    const size_t lds = sizeof(R) * 2 * (T->dev.n_chi[0] > T->dev.n_chi[1] ? T->dev.n_chi[0] : T->dev.n_chi[1]);
    if (sizeof(R) != 4) pv = 0;                        // the variants are compiled in single precision
    if (maxb <= 0) maxb = resident_blocks<R>(lds, pv);
    std::vector<InstDev<R>> inst(n);
    std::vector<SegDev> seg;
    int64_t nblk = 0, mask_words = 0;
    int64_t npb = 0;
    auto add = [&](int kind, int i, int64_t cap) {
        SegDev s;
        s.kind = kind;
        s.inst = i;
        const int64_t want = cdiv(cap > 0 ? cap : 1, ppb);
        s.nb = (int)(want < maxb ? want : maxb);
        s.b0 = (int)nblk;
        s.npb = (int)cdiv(s.nb, group);
        s.pb0 = (int)npb;
        npb += s.npb;
        s.nchunks = cdiv(cap > 0 ? cap : 1, 64);
        s.mask_off = mask_words;
        nblk += s.nb;
        mask_words += 2 * s.nchunks;
        seg.push_back(s);
        return (int)seg.size() - 1;
    };
    // lepton segments of every instance first (first launch), then the photon segments
    for (int i = 0; i < n; ++i) {
        inst[i] = inst_dev<R>(&in[i]);
        inst[i].se = add(0, i, in[i].electrons.capacity);
        if (in[i].params.flags & QED_PAIR) inst[i].sp = add(1, i, in[i].positrons.capacity);
    }
    const int64_t nblk_lep = nblk, npb_lep = npb;
    for (int i = 0; i < n; ++i)
        if (in[i].params.flags & QED_PAIR) inst[i].sg = add(2, i, in[i].photons.capacity);
    if (nblk > (1 << 24)) return QED_ERR_INVALID;
    qed_plan p = new qed_plan_s();
    memset(p, 0, sizeof(*p));
    p->T = T;
    p->ninst = n;
    p->nseg = (int)seg.size();
    p->nblk = (int)nblk;
    p->nblk_lep = (int)nblk_lep;
    p->npb = (int)npb;
    p->npb_lep = (int)npb_lep;
    p->group = group;
    p->lds = lds;
    p->pv = pv;
    hipError_t e = hipMalloc(&p->d_inst, sizeof(InstDev<R>) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_seg, sizeof(SegDev) * seg.size());
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_mask, sizeof(uint64_t) * mask_words);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_bcnt, sizeof(uint32_t) * nblk);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_bctr, sizeof(uint32_t) * kNCtr * nblk);
    p->sur[0] = s_nlc;
    p->sur[1] = s_nbw;
    p->dec = 0;
    p->fv = kFldPlain;
    p->flep = kFldPlain;
    for (int i = 0; i < n; ++i) {
        if (in[i].params.flags & QED_OPTICAL_DEPTH) p->dec |= 1;
        if (in[i].params.flags & QED_REJECTION) p->dec |= 2;
        if (in[i].params.flags & QED_SUBCYCLE) p->sub = 1;
        p->fv = std::max(p->fv, field_variant(&in[i].fields));
        p->flep = std::max(p->flep, lepton_variant(&in[i].fields, in[i].params.flags));
    }
    // sub-cycling: a word per slot of each sub-cycled lepton set, and per-round block counts
    if (p->sub && e == hipSuccess) {
        int64_t words = 0;
        for (int i = 0; i < n; ++i)
            if (in[i].params.flags & QED_SUBCYCLE)
                words += in[i].electrons.capacity + ((in[i].params.flags & QED_PAIR) ? in[i].positrons.capacity : 0);
        e = hipMalloc((void **)&p->d_sub, sizeof(uint32_t) * (words > 0 ? words : 1));
        if (e == hipSuccess) e = hipMalloc(&p->d_stage, sizeof(R) * kStage * (words > 0 ? words : 1));
        if (e == hipSuccess) e = hipMalloc((void **)&p->d_bsub, sizeof(uint32_t) * kSubRounds * (nblk_lep > 0 ? nblk_lep : 1));
        // a streaming block's slots are split over sub-step blocks of kBlock slots at most, so each
        // thread takes the sub-steps of one flagged lepton and small sets still spread over the chip;
        // at most kSubGrid blocks in all (large sets: a few rounds of slots per block instead of
        // hundreds of thousands of blocks that mostly find no flagged lepton)
        constexpr int64_t kSubGrid = 8192;
        int64_t bmax = 64;
        for (const SegDev &sgm : seg)
            if (sgm.kind != 2) bmax = std::max<int64_t>(bmax, block_len(sgm.nchunks * 64, sgm.nb));
        p->sub_split = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(bmax, kBlock), kSubGrid / std::max<int64_t>(1, nblk_lep)));
        // default priority, like every stream of the library
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join, hipEventDisableTiming);
        uint32_t *at = p->d_sub;
        R *st = (R *)p->d_stage;
        for (int i = 0; i < n && e == hipSuccess; ++i)
            if (in[i].params.flags & QED_SUBCYCLE) {
                inst[i].E.sub = at;
                inst[i].E.stage = st;
                at += in[i].electrons.capacity;
                st += kStage * in[i].electrons.capacity;
                if (in[i].params.flags & QED_PAIR) {
                    inst[i].P.sub = at;
                    inst[i].P.stage = st;
                    at += in[i].positrons.capacity;
                    st += kStage * in[i].positrons.capacity;
                }
            }
    }
    // grid fields: the plan keeps a node-interleaved copy, refreshed from the caller's arrays at
    // the start of every step, so an interpolation reads four 32-byte corners instead of 24 scalars
    p->h_grid = (FieldDev *)calloc(n, sizeof(FieldDev));
    p->h_gn = (float4 **)calloc(n, sizeof(float4 *));
    if (!p->h_grid || !p->h_gn) e = hipErrorOutOfMemory;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        if (in[i].fields.kind != QED_FIELD_GRID2D) continue;
        p->h_grid[i] = inst[i].F;
        e = hipMalloc((void **)&p->h_gn[i], sizeof(float4) * 2 * (size_t)in[i].fields.nx * (size_t)in[i].fields.ny);
        inst[i].F.gn = p->h_gn[i];
    }
    if (e == hipSuccess) e = hipMemcpy(p->d_inst, inst.data(), sizeof(InstDev<R>) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_seg, seg.data(), sizeof(SegDev) * seg.size(), hipMemcpyHostToDevice);
    // block -> segment (and instance) tables: one load instead of a search over the segments
    std::vector<int> bseg(nblk), binst(nblk);
    std::vector<int4> pbd(npb > 0 ? npb : 1);
    for (int sj = 0; sj < (int)seg.size(); ++sj) {
        const SegDev &sg = seg[sj];
        for (int b = sg.b0; b < sg.b0 + sg.nb; ++b) {
            bseg[b] = sj;
            binst[b] = sg.inst;
        }
        for (int pb = sg.pb0; pb < sg.pb0 + sg.npb; ++pb) {
            const int mb0 = sg.b0 + (pb - sg.pb0) * group;
            const int mb1 = mb0 + group < sg.b0 + sg.nb ? mb0 + group : sg.b0 + sg.nb;
            pbd[pb] = make_int4(sj, mb0, mb1, sg.inst);
        }
    }
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_bseg, sizeof(int) * nblk);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_binst, sizeof(int) * nblk);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_pbd, sizeof(int4) * pbd.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_bseg, bseg.data(), sizeof(int) * nblk, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_binst, binst.data(), sizeof(int) * nblk, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_pbd, pbd.data(), sizeof(int4) * pbd.size(), hipMemcpyHostToDevice);
    std::vector<InstSeg> iseg(n);
    for (int i = 0; i < n; ++i) {
        auto range = [&](int sj, int &b0, int &b1) {
            b0 = sj >= 0 ? seg[sj].b0 : 0;
            b1 = sj >= 0 ? seg[sj].b0 + seg[sj].nb : 0;
        };
        range(inst[i].se, iseg[i].e0, iseg[i].e1);
        range(inst[i].sp, iseg[i].p0, iseg[i].p1);
        range(inst[i].sg, iseg[i].g0, iseg[i].g1);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_iseg, sizeof(InstSeg) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_snap, sizeof(Snap) * n);
    if (e == hipSuccess) e = hipMemcpy(p->d_iseg, iseg.data(), sizeof(InstSeg) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        plan_free(p);
        return qs_fail(e, "qed_plan_create");
    }
    *out = p;
    return QED_OK;
}

template <class R> qed_status plan_step(qed_plan p, hipStream_t st)
{
    PlanDev P;
    P.seg = p->d_seg;
    P.nseg = p->nseg;
    P.nblk = p->nblk;
    P.group = p->group;
    P.ninst = p->ninst;
    P.mask = p->d_mask;
    P.bcnt = p->d_bcnt;
    P.bctr = p->d_bctr;
    P.bseg = p->d_bseg;
    P.binst = p->d_binst;
    P.pbd = p->d_pbd;
    P.iseg = p->d_iseg;
    P.snap = p->d_snap;
    P.bsub = p->d_bsub;
    memset(P.mlp, 0, sizeof(P.mlp));
    P.mlp_on[0] = P.mlp_on[1] = 0;
    const InstDev<R> *inst = (const InstDev<R> *)p->d_inst;
    for (int i = 0; i < p->ninst; ++i)
        if (p->h_gn[i]) {
            const int64_t nn = (int64_t)p->h_grid[i].nx * p->h_grid[i].ny;
            const int gb = (int)std::min<int64_t>(cdiv(nn, kBlock), 4096);
            QS_LAUNCH(K_GRID_PACK, k_pack_grid, dim3(gb), dim3(kBlock), 0, st, p->h_grid[i], p->h_gn[i]);
        }
    if (p->nblk_lep > 0) {
        if (p->sub && p->flep == kFldGeneral)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 8, kFldGeneral>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st, inst, P,
                      p->T->dev, 0);
        else if (p->sub && p->flep == kFldRotating)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 8, kFldRotating>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st, inst,
                      P, p->T->dev, 0);
        else if (p->sub)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 8, kFldPlain>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st, inst, P,
                      p->T->dev, 0);
        else if (p->dec == 3)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 3, kFldGeneral>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st, inst, P,
                      p->T->dev, 0);
        else if (p->dec == 2)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 2, kFldGeneral>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st, inst, P,
                      p->T->dev, 0);
        else if (p->dec == 1)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 1, kFldGeneral>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st, inst, P,
                      p->T->dev, 0);
        else if (p->flep == kFldGeneral)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 0, kFldGeneral>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st,
                      inst, P, p->T->dev, 0);
        else if (p->flep == kFldRotating)
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 0, kFldRotating>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st,
                      inst, P, p->T->dev, 0);
        else
            QS_LAUNCH(K_PLAN_LEPTON, (k_plan_main<R, 0, 0, kFldPlain>), dim3(p->nblk_lep), dim3(kBlock), p->lds, st,
                      inst, P, p->T->dev, 0);
    }
    // sub-cycling: the sub-step launch (latency-bound: long chains on few waves) on the side stream,
    // beside the photon pass, which does not touch the leptons; joined before the processing
    const bool fork = p->sub && p->nblk_lep > 0;
    if (fork) {
        QS_CHECK(hipEventRecord(p->fork, st));
        QS_CHECK(hipStreamWaitEvent(p->side, p->fork, 0));
        auto sk = p->fv == kFldGeneral ? k_plan_sub<R, kFldGeneral> : p->fv == kFldRotating ? k_plan_sub<R, kFldRotating>
                                                                                            : k_plan_sub<R, kFldPlain>;
        QS_LAUNCH(K_PLAN_SUB, sk, dim3(p->nblk_lep * p->sub_split), dim3(kBlock), p->lds, p->side, inst, P, p->T->dev,
                  p->sub_split);
        QS_CHECK(hipEventRecord(p->join, p->side));
    }
    if (p->nblk > p->nblk_lep) {
        if (p->fv == kFldGeneral)
            QS_LAUNCH(K_PLAN_PHOTON, (k_plan_main<R, 1, 0, kFldGeneral>), dim3(p->nblk - p->nblk_lep), dim3(kBlock), p->lds,
                      st, inst, P, p->T->dev, p->nblk_lep);
        else if (p->fv == kFldRotating)
            QS_LAUNCH(K_PLAN_PHOTON, (k_plan_main<R, 1, 0, kFldRotating>), dim3(p->nblk - p->nblk_lep), dim3(kBlock),
                      p->lds, st, inst, P, p->T->dev, p->nblk_lep);
        else if (p->pv == 1)
            QS_LAUNCH(K_PLAN_PHOTON, (k_plan_main<R, 1, 0, kFldPlain, 1>), dim3(p->nblk - p->nblk_lep), dim3(kBlock),
                      p->lds, st, inst, P, p->T->dev, p->nblk_lep);
        else if (p->pv == 2)
            QS_LAUNCH(K_PLAN_PHOTON, (k_plan_main<R, 1, 0, kFldPlain, 2>), dim3(p->nblk - p->nblk_lep), dim3(kBlock),
                      p->lds, st, inst, P, p->T->dev, p->nblk_lep);

        else
            QS_LAUNCH(K_PLAN_PHOTON, (k_plan_main<R, 1, 0, kFldPlain>), dim3(p->nblk - p->nblk_lep), dim3(kBlock), p->lds,
                      st, inst, P, p->T->dev, p->nblk_lep);
    }
    if (fork) QS_CHECK(hipStreamWaitEvent(st, p->join, 0));
    // processing, with the bookkeeping; a process with a learned inverse CDF evaluates it in the
    // same launch (single precision only)
    const bool sl = p->sur[0] != nullptr, sb = p->sur[1] != nullptr;
    if (p->npb > 0) {
        if constexpr (sizeof(R) == 4) {
            if (sl || sb) {
                if (sl) P.mlp[0] = qs_surrogate_view(p->sur[0]);
                if (sb) P.mlp[1] = qs_surrogate_view(p->sur[1]);
                P.mlp_on[0] = sl;
                P.mlp_on[1] = sb;
                auto proc = p->fv == kFldGeneral    ? k_plan_process<R, kFldGeneral, true>
                            : p->fv == kFldRotating ? k_plan_process<R, kFldRotating, true>
                                                    : k_plan_process<R, kFldPlain, true>;
                QS_LAUNCH(K_PLAN_PROCESS, proc, dim3(p->npb), dim3(kBlock), p->lds, st, inst, P, p->T->dev, 0);
                return qs_launch_status("qed_plan_step");
            }
        }
        if (p->sub) {
            auto proc = p->fv == kFldGeneral    ? k_plan_process<R, kFldGeneral, false, true>
                        : p->fv == kFldRotating ? k_plan_process<R, kFldRotating, false, true>
                                                : k_plan_process<R, kFldPlain, false, true>;
            QS_LAUNCH(K_PLAN_PROCESS, proc, dim3(p->npb), dim3(kBlock), p->lds, st, inst, P, p->T->dev, 0);
            return qs_launch_status("qed_plan_step");
        }
        auto proc = p->fv == kFldGeneral    ? k_plan_process<R, kFldGeneral, false>
                    : p->fv == kFldRotating ? k_plan_process<R, kFldRotating, false>
                                            : k_plan_process<R, kFldPlain, false>;
        QS_LAUNCH(K_PLAN_PROCESS, proc, dim3(p->npb), dim3(kBlock), p->lds, st, inst, P, p->T->dev, 0);
    }
    return qs_launch_status("qed_plan_step");
}

bool instance_ok(const qed_instance *in)
{
    const uint32_t fl = in->params.flags;
    if (!leptons_ok(&in->electrons) || in->electrons.species != 0 || !tau_ok(&in->electrons, fl)) return false;
    if ((fl & QED_REJECTION) && (fl & QED_OPTICAL_DEPTH)) return false;
    if ((fl & QED_SUBCYCLE) && (fl & (QED_REJECTION | QED_OPTICAL_DEPTH))) return false;
    if (!fields_ok(&in->fields) || !in->d_counters || !in->params.d_clock) return false;
    if (!(in->params.dt > 0.0) || !(in->params.eps_r > 0.0)) return false;
    if ((fl & (QED_EMIT | QED_PAIR)) && !photons_ok(&in->photons)) return false;
    if ((fl & QED_PAIR) && (!leptons_ok(&in->positrons) || in->positrons.species != 1 || !tau_ok(&in->positrons, fl)))
        return false;
    return true;
}

}  // namespace

extern "C" qed_status qed_plan_create(qed_tables T, int n_instances, const qed_instance *instances,
                                      const qed_plan_config *config, qed_plan *out)
{
    if (!T || !out || n_instances <= 0 || !instances) return QED_ERR_INVALID;
    *out = nullptr;
    for (int i = 0; i < n_instances; ++i)
        if (!instance_ok(&instances[i])) return QED_ERR_INVALID;
    const int ppb = config && config->particles_per_block > 0 ? config->particles_per_block : kBlock;
    const int maxb = config && config->max_blocks_per_set > 0 ? config->max_blocks_per_set : 0;   // 0: one resident round
    const int group = config && config->process_group > 0 ? config->process_group : 4;
    const int pv = config ? config->photon_variant : 0;
    if (pv < 0 || pv > 2) return QED_ERR_INVALID;
    qed_surrogate sn = config ? config->icdf_nlc : nullptr, sb = config ? config->icdf_nbw : nullptr;
    // the networks are trained for 24-bit uniforms (single precision) on these tables' ranges
    if ((sn || sb) && T->params.precision != QED_F32) return QED_ERR_UNSUPPORTED;
    if (sn && (qs_surrogate_process(sn) != 0 || qs_surrogate_tables(sn) != T)) return QED_ERR_INVALID;
    if (sb && (qs_surrogate_process(sb) != 1 || qs_surrogate_tables(sb) != T)) return QED_ERR_INVALID;
    if (sn || sb)
        for (int i = 0; i < n_instances; ++i)
            if (instances[i].params.flags & QED_SUBCYCLE) return QED_ERR_UNSUPPORTED;   // tables only
    qs_clear_error();
    if (T->params.precision == QED_F64)
        return plan_create<double>(T, n_instances, instances, ppb, maxb, group, pv, sn, sb, out);
    return plan_create<float>(T, n_instances, instances, ppb, maxb, group, pv, sn, sb, out);
}

extern "C" qed_status qed_plan_step(qed_plan plan, qed_stream stream)
{
    if (!plan) return QED_ERR_INVALID;
    qs_clear_error();
    if (plan->T->params.precision == QED_F64) return plan_step<double>(plan, (hipStream_t)stream);
    return plan_step<float>(plan, (hipStream_t)stream);
}

extern "C" int64_t qed_plan_blocks(qed_plan plan) { return plan ? plan->nblk : 0; }

extern "C" qed_status qed_plan_destroy(qed_plan plan)
{
    if (plan) {
        (void)hipDeviceSynchronize();
        plan_free(plan);
    }
    return QED_OK;
}
