// qs_step.hip -- the per-species entry points qed_push_spin, qed_emit, qed_pair, and the photon
// compaction qed_compact.
//
// Each transition step runs as
//   main     one streaming pass over the particle SoA (coalesced loads/stores, rate tables in
//            LDS): push, chi, basis, rates, Philox draw, decision, no-transition update; the
//            wave's 64 decisions and branch choices are ballot'ed into two 64-bit mask words,
//            each block writes its transition and event counts;
//   expand   per-block prefix of the block counts (block 0 also does the bookkeeping: total,
//            append bases, capacity clamp, counters, device counts) and expansion of the block's
//            mask words into a dense, ascending list of the transitioning particles;
//   process  one thread per transitioning particle: inverse-CDF sampling, Bessel functions,
//            spin / Stokes collapse, appends at base + rank.
// Everything is keyed on device-resident counts, so a step enqueues without host sync.  The
// per-particle bodies are shared with the merged step (qs_plan.hip) through qs_pass.hpp.
#include <mutex>

#include "qs_pass.hpp"

namespace {
using namespace qs;

// ------------------------------------------------------------------ kernels: leptons
template <class R>
__global__ void __launch_bounds__(kBlock) k_push(LepDev<R> L, FieldDev F, StepDev S0, TablesDev T)
{
    const StepDev S = localize(S0);
    const int64_t n = *L.count;
    const int q = L.species == 0 ? -1 : 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        V3<R> x = ldx(L.x, i), p = ld3(L.p, i), s = ld3(L.s, i);
        V3<R> E, B;
        if (!(finite3(x) && finite3(p) && finite3(s))) continue;      // non-finite: left as stored
        eval_fields<R, kFldGeneral>(F, (double)x.x, (double)x.y, S.t, E, B);
        if (!(finite3(E) && finite3(B))) continue;                      // (grid values)
        const V3<R> d = push<R>(q, (R)S.a_e, E, B, (R)S.dt, (S.flags & F_TBMT) != 0, p, s,
                                gfac_src<R, kFldGeneral>(T, S.flags), (R)S.eps_r);
        stx(L.x, i, x + d);
        st3(L.p, i, p);
        st3(L.s, i, s);
    }
}

template <class R, int DEC, int FLD>
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
    LCount c;
    lepton_range<R, DEC, FLD>(L, F, S, T, lds, start, end, mask, nchunks, c);
    unsigned v[kNCtr + 1] = {};
    v[C_PROB] = c.prob; v[C_CHI] = c.chi; v[C_NORM] = c.norm; v[C_LSTEP] = c.step; v[C_NONFIN] = c.nonfin;
        v[kNCtr] = c.trans;
    __shared__ unsigned tot[kNCtr + 1];
    block_sum(v, tot);
    if (threadIdx.x < kNCtr) bctr[blockIdx.x * kNCtr + threadIdx.x] = tot[threadIdx.x];
    else if (threadIdx.x == kNCtr) bcnt[blockIdx.x] = tot[kNCtr];
}

template <class R, int FLD>
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
        const bool up = (mask[nchunks + (i >> 6)] >> (i & 63)) & 1ull;
        emit_item<R, FLD>(L, G, F, S, T, lds, i, up, j < nfit ? gbase + j : -1, c_ret);
    }
    block_add(ctr, C_RETIRED, c_ret);
}

// ------------------------------------------------------------------ kernels: photons
template <class R, int FLD>
__global__ void __launch_bounds__(kBlock) k_photon_main(PhoDev<R> G, FieldDev F, StepDev S0, TablesDev T, uint64_t *mask,
                                                        int64_t nchunks, uint32_t *bctr, uint32_t *bcnt)
{
    const StepDev S = localize(S0);
    extern __shared__ unsigned char smem_raw[];
    R *lds = reinterpret_cast<R *>(smem_raw);
    __shared__ PhoQueue<R, kPhoTile, queue_kind<R, FLD>()> Q;
    stage_rates<R>(T, 1, lds);
    const int64_t n = *G.count_prev;
    const int64_t B = block_len(n, gridDim.x);
    const int64_t start = (int64_t)blockIdx.x * B, end = start + B < n ? start + B : n;
    GCount c;
    for (int64_t tile = start; tile < end; tile += kPhoTile)
        photon_tile<R, FLD>(G, F, S, T, lds, Q, tile, tile + kPhoTile < end ? tile + kPhoTile : end, mask, nchunks, c);
    unsigned v[kNCtr + 1] = {};
    v[C_PROB] = c.prob; v[C_CHI] = c.chi; v[C_NORM] = c.norm; v[C_RETIRED] = c.ret; v[C_GSTEP] = c.step;
    v[C_GQED] = c.qed; v[C_NONFIN] = c.nonfin; v[kNCtr] = c.trans;
    __shared__ unsigned tot[kNCtr + 1];
    block_sum(v, tot);
    if (threadIdx.x < kNCtr) bctr[blockIdx.x * kNCtr + threadIdx.x] = tot[threadIdx.x];
    else if (threadIdx.x == kNCtr) bcnt[blockIdx.x] = tot[kNCtr];
}

template <class R, int FLD>
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
        const bool plus = (mask[nchunks + (i >> 6)] >> (i & 63)) & 1ull;
        pair_item<R, FLD>(G, Le, Lp, F, S, T, lds, i, plus, j < nfit ? be + j : -1, bp + j);
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

// The survivors are copied in rounds of at most kCompactChunk ranks through a staging buffer of
// that size: round [r0, r0 + len) gathers the survivors of ranks r0.. (at slots idx[r] >= r) and
// writes them back to slots r0..  Later rounds read slots idx[r] >= r >= r0 + len only, which
// this round does not write, so the stream order of the rounds makes the copy exact.
constexpr int64_t kCompactChunk = int64_t(1) << 26;

template <class R>
__global__ void __launch_bounds__(kBlock) k_gather(PhoDev<R> G, PhoStage<R> T, const uint32_t *idx, const int64_t *book,
                                                   int64_t r0, int64_t len)
{
    const int64_t hi = book[1] < r0 + len ? book[1] : r0 + len;
    for (int64_t j = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < hi; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[j], t = j - r0;
        T.id[t] = G.id[i];
        for (int c = 0; c < 3; ++c) {
            if (G.x[c]) T.x[c][t] = G.x[c][i];
            T.k[c][t] = G.k[c][i];
            T.P[c][t] = G.P[c][i];
        }
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_scatter_back(PhoDev<R> G, PhoStage<R> T, const int64_t *book, int64_t r0,
                                                         int64_t len)
{
    const int64_t total = book[1];
    const int64_t hi = total < r0 + len ? total : r0 + len;
    for (int64_t j = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < hi; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = j - r0;
        G.id[j] = T.id[t];
        for (int c = 0; c < 3; ++c) {
            if (G.x[c]) G.x[c][j] = T.x[c][t];
            G.k[c][j] = T.k[c][t];
            G.P[c][j] = T.P[c][t];
        }
    }
    if (r0 == 0 && blockIdx.x == 0 && threadIdx.x == 0) *G.count = total;
}

// ------------------------------------------------------------------ host side
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
    const int fv = lepton_variant(f, p->flags);
    if (p->flags & QED_SUBCYCLE) {
        // the QED part in kSubRounds rounds of streaming pass, expansion and processing; the push
        // only in round 0; each round appends its photons after the previous round's
        LepDev<R> ls = ld;
        ls.msub = w.msub;
        const PhoDev<R> gs = pho_dev<R>((p->flags & QED_EMIT) ? G : nullptr);
        for (int r = 0; r < kSubRounds; ++r) {
            StepDev sr = sd;
            sr.sub_round = r;
            if (r > 0) sr.flags &= ~(uint32_t)QED_PUSH;
            QS_LAUNCH(K_LEPTON_MAIN, (k_lepton_main<R, 4, kFldGeneral>), dim3(g), dim3(kBlock), lds_nlc, st, ls, fd, sr, T->dev,
                      w.mask, nch, w.bctr, w.bcnt);
            QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask,
                      (const uint32_t *)w.bcnt, (const int64_t *)L->d_count, w.book, 0, gs.count, gs.cap,
                      (int64_t *)nullptr, (int64_t)0, (int64_t *)nullptr, c, (const uint32_t *)w.bctr, w.idx);
            QS_LAUNCH(K_EMIT_PROCESS, (k_emit_process<R, kFldGeneral>), dim3(g), dim3(kBlock), lds_nlc, st, ls, gs, fd, sr,
                      T->dev, w.mask, nch, w.idx, w.book, c);
        }
        return qs_launch_status(__func__);
    }
    if (p->flags & QED_OPTICAL_DEPTH)
        QS_LAUNCH(K_LEPTON_MAIN, (k_lepton_main<R, 1, kFldGeneral>), dim3(g), dim3(kBlock), lds_nlc, st, ld, fd, sd, T->dev,
                  w.mask, nch, w.bctr, w.bcnt);
    else if (p->flags & QED_REJECTION)
        QS_LAUNCH(K_LEPTON_MAIN, (k_lepton_main<R, 2, kFldGeneral>), dim3(g), dim3(kBlock), lds_nlc, st, ld, fd, sd, T->dev,
                  w.mask, nch, w.bctr, w.bcnt);
    else if (fv == kFldGeneral)
        QS_LAUNCH(K_LEPTON_MAIN, (k_lepton_main<R, 0, kFldGeneral>), dim3(g), dim3(kBlock), lds_nlc, st, ld, fd, sd,
                  T->dev, w.mask, nch, w.bctr, w.bcnt);
    else if (fv == kFldRotating)
        QS_LAUNCH(K_LEPTON_MAIN, (k_lepton_main<R, 0, kFldRotating>), dim3(g), dim3(kBlock), lds_nlc, st, ld, fd, sd,
                  T->dev, w.mask, nch, w.bctr, w.bcnt);
    else
        QS_LAUNCH(K_LEPTON_MAIN, (k_lepton_main<R, 0, kFldPlain>), dim3(g), dim3(kBlock), lds_nlc, st, ld, fd, sd,
                  T->dev, w.mask, nch, w.bctr, w.bcnt);
    const PhoDev<R> gd = pho_dev<R>((p->flags & QED_EMIT) ? G : nullptr);
    QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask, (const uint32_t *)w.bcnt,
              (const int64_t *)L->d_count, w.book, 0, gd.count, gd.cap, (int64_t *)nullptr, (int64_t)0,
              (int64_t *)nullptr, c, (const uint32_t *)w.bctr, w.idx);
    QS_LAUNCH(K_EMIT_PROCESS, (k_emit_process<R, kFldGeneral>), dim3(g), dim3(kBlock), lds_nlc, st, ld, gd, fd, sd, T->dev, w.mask,
              nch, w.idx, w.book, c);
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
    const int fv = field_variant(f);
    if (fv == kFldGeneral)
        QS_LAUNCH(K_PHOTON_MAIN, (k_photon_main<R, kFldGeneral>), dim3(g), dim3(kBlock), lds_nbw, st, gd, fd, sd, T->dev,
                  w.mask, nch, w.bctr, w.bcnt);
    else if (fv == kFldRotating)
        QS_LAUNCH(K_PHOTON_MAIN, (k_photon_main<R, kFldRotating>), dim3(g), dim3(kBlock), lds_nbw, st, gd, fd, sd, T->dev,
                  w.mask, nch, w.bctr, w.bcnt);
    else
        QS_LAUNCH(K_PHOTON_MAIN, (k_photon_main<R, kFldPlain>), dim3(g), dim3(kBlock), lds_nbw, st, gd, fd, sd, T->dev,
                  w.mask, nch, w.bctr, w.bcnt);
    QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask, (const uint32_t *)w.bcnt,
              (const int64_t *)G->d_count_prev, w.book, 1, Le->d_count, Le->capacity, Lp->d_count, Lp->capacity,
              (int64_t *)nullptr, c, (const uint32_t *)w.bctr, w.idx);
    QS_LAUNCH(K_PAIR_PROCESS, (k_pair_process<R, kFldGeneral>), dim3(g), dim3(kBlock), lds_nbw, st, gd, lep_dev<R>(Le),
              lep_dev<R>(Lp), fd, sd, T->dev, w.mask, nch, w.idx, w.book);
    return qs_launch_status(__func__);
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" size_t qed_workspace_size(int64_t max_particles)
{
    const int64_t cap = max_particles > 0 ? max_particles : 1;
    const int64_t nch = cdiv(cap, 64);
    return align256(sizeof(uint64_t) * 2 * nch) + align256(sizeof(uint32_t) * kMaxGrid) +
           align256(sizeof(int64_t) * 8) + align256(sizeof(uint32_t) * kMaxGrid * kNCtr) + align256(sizeof(uint32_t) * cap) +
           align256(sizeof(uint8_t) * cap);
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
        QS_LAUNCH(K_PUSH, k_push<double>, dim3(g), dim3(kBlock), 0, st, lep_dev<double>(L), fd, sd, T->dev);
    else
        QS_LAUNCH(K_PUSH, k_push<float>, dim3(g), dim3(kBlock), 0, st, lep_dev<float>(L), fd, sd, T->dev);
    return qs_launch_status(__func__);
}

extern "C" qed_status qed_emit(qed_tables T, const qed_leptons *L, const qed_fields *f, const qed_step_params *p,
                               const qed_photons *G, qed_counters *ctr, void *ws, size_t ws_bytes, qed_stream stream)
{
    if (!T || !leptons_ok(L) || !p || !fields_ok(f) || !ctr || !ws) return QED_ERR_INVALID;
    if ((p->flags & QED_EMIT) && !photons_ok(G)) return QED_ERR_INVALID;
    if (!tau_ok(L, p->flags)) return QED_ERR_INVALID;
    if ((p->flags & QED_REJECTION) && (p->flags & QED_OPTICAL_DEPTH)) return QED_ERR_INVALID;
    if ((p->flags & QED_SUBCYCLE) && (p->flags & (QED_REJECTION | QED_OPTICAL_DEPTH))) return QED_ERR_INVALID;
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
    if (!tau_ok(Le, p->flags) || !tau_ok(Lp, p->flags)) return QED_ERR_INVALID;
    if (!(p->dt > 0.0) || !(p->eps_r > 0.0)) return QED_ERR_INVALID;
    if (ws_bytes < qed_workspace_size(G->capacity)) return QED_ERR_CAPACITY;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    if (T->params.precision == QED_F64) return pair_impl<double>(T, G, f, p, Le, Lp, ctr, ws, ws_bytes, st);
    return pair_impl<float>(T, G, f, p, Le, Lp, ctr, ws, ws_bytes, st);
}

// ------------------------------------------------------------------ qed_emit without allocation
// The workspace of qed_emit_noalloc is this file-scope device array, one copy per GPU, held until
// the process ends.  Host code never passes `scratch` itself to a kernel (in host code the name
// stands for a host-side shadow, not a device address): the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current and kept per device.
static __device__ __align__(256) unsigned char scratch[QED_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// the device address of this device's `scratch` (NULL on failure, with the error recorded)
void *scratch_ptr(qed_status &st)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        st = qs_fail(e, "qed_emit_noalloc: hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        st = qs_reject(QED_ERR_UNSUPPORTED, "qed_emit_noalloc: device index beyond the library's table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            st = qs_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "qed_emit_noalloc: hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" qed_status qed_emit_noalloc(qed_tables T, const qed_leptons *L, const qed_fields *f, const qed_step_params *p,
                                       const qed_photons *G, qed_counters *ctr, qed_stream stream)
{
    if (!T || !leptons_ok(L) || !p || !fields_ok(f) || !ctr) return QED_ERR_INVALID;
    if (L->capacity > QED_NOALLOC_MAX_LEPTONS || qed_workspace_size(L->capacity) > sizeof(scratch)) {
        char msg[160];
        snprintf(msg, sizeof(msg), "qed_emit_noalloc: lepton capacity %lld exceeds the static scratch maximum of %lld",
                 (long long)L->capacity, (long long)QED_NOALLOC_MAX_LEPTONS);
        return qs_reject(QED_ERR_CAPACITY, msg);
    }
    qed_status st = QED_OK;
    void *ws = scratch_ptr(st);
    if (!ws) return st;
    // every word of the scratch that a step reads is written earlier in the same step (masks and
    // per-block counts by the streaming pass, the bookkeeping and index list by the expansion,
    // sub-step counts in round 0), so nothing needs clearing between calls
    return qed_emit(T, L, f, p, G, ctr, ws, sizeof(scratch), stream);
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
    const int64_t stage = G->capacity < kCompactChunk ? (G->capacity > 0 ? G->capacity : 1) : kCompactChunk;
    return qed_workspace_size(G->capacity) + ncomp * align256(es * stage) + align256(sizeof(uint64_t) * stage);
}

template <class R> static qed_status compact_impl(const qed_photons *G, void *ws, hipStream_t st)
{
    int64_t nch;
    const WS w = carve(ws, G->capacity, &nch);
    char *b = (char *)ws + qed_workspace_size(G->capacity);
    const int64_t cap = G->capacity > 0 ? G->capacity : 1;
    const int64_t stage = cap < kCompactChunk ? cap : kCompactChunk;
    PhoStage<R> S;
    for (int c = 0; c < 3; ++c) {
        S.x[c] = nullptr;
        if (G->x[c]) { S.x[c] = (R *)b; b += align256(sizeof(R) * stage); }
    }
    for (int c = 0; c < 3; ++c) { S.k[c] = (R *)b; b += align256(sizeof(R) * stage); }
    for (int c = 0; c < 3; ++c) { S.P[c] = (R *)b; b += align256(sizeof(R) * stage); }
    S.id = (uint64_t *)b;
    const PhoDev<R> gd = pho_dev<R>(G);
    const int g = grid_for(G->capacity);
    QS_LAUNCH(K_ALIVE_MASK, k_alive_mask<R>, dim3(g), dim3(kBlock), 0, st, gd, w.mask, w.bcnt);
    QS_LAUNCH(K_MASK_EXPAND, k_expand, dim3(g), dim3(kBlock), 0, st, (const uint64_t *)w.mask, (const uint32_t *)w.bcnt,
              (const int64_t *)G->d_count, w.book, 2, (int64_t *)nullptr, (int64_t)0, (int64_t *)nullptr, (int64_t)0,
              G->d_count_prev, (unsigned long long *)nullptr, (const uint32_t *)nullptr, w.idx);
    const int gs = grid_for(stage);
    for (int64_t r0 = 0; r0 < cap; r0 += stage) {
        QS_LAUNCH(K_GATHER, k_gather<R>, dim3(gs), dim3(kBlock), 0, st, gd, S, w.idx, w.book, r0, stage);
        QS_LAUNCH(K_SCATTER_BACK, k_scatter_back<R>, dim3(gs), dim3(kBlock), 0, st, gd, S, w.book, r0, stage);
    }
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
