// qs_mlp.hip -- training and evaluation of the learned inverse CDF (qed_surrogate_*).
//
// Training data come from the library's own inverse-CDF tables (FP64 interpolation, the same
// lookup the table path uses): every step draws fresh samples (ln chi, rho, c) from Philox
// channel 6 (ln chi uniform; rho half uniform, half distributed as in the sampling) and fits
// the residual y = (nu - base)/out_s over the coarse table by mean squared error with Adam.  The
// fine tables stay the fallback and the judge: qed_surrogate_judge samples every coarse cell
// against them and marks the cells where the network's error exceeds the given bound.
//   k_mlp_base   the coarse table: the fine tables' nu at the coarse nodes, in FP32
//   k_mlp_grad   forward + backward of 16-row tiles per wave on the matrix cores; parameter
//                gradients summed per block in LDS, written per block
//   k_mlp_adam   sums the block gradients, Adam update of the FP32 master, BF16 copy
//   k_mlp_image  BF16 copy of W2..W4 rearranged as MFMA B operands
//   k_mlp_eval   nu for given (ln chi, rho, c): as the step uses it, the network without the
//                fallback, or the coarse table alone
//   k_mlp_judge  largest |nu_net - nu_table| over K x K points of every coarse cell
#include <math.h>
#include <stdint.h>

#include <vector>

#include "qs_mlp.hpp"

namespace {
using namespace qs;
using namespace qs::mlp;

// the network fits (nu - base)/out_s, out_s = kResidualMargin times the coarse table's largest
// judged error, so that its output spans about [-1, 1]
constexpr float kResidualMargin = 1.25f;
constexpr double kBaseChiPerDecade = 4.0;   // coarse ln chi nodes per decade (at least)
constexpr double kBaseRho = 20.0;           // coarse rho nodes on [-20, 20] ...
constexpr double kBaseDrho = 1.0;           // ... every 1

constexpr int kMlpBlock = 256;          // 4 waves
constexpr int kGradGrid = 256;          // blocks of a training step
constexpr int kAcc = kNP + 1;           // per-block record: gradient, then the summed squared error
constexpr float kRho24 = 16.635532f;    // ln(2^24 - 1/2): the largest |rho| of a 24-bit uniform

// normalized inputs (u, v, c) and target y of sample `id` of training step `step`
__device__ inline void draw_sample(const MlpDev &M, const TablesDev &T, int proc, uint64_t seed, uint64_t id,
                                   int64_t step, float xo[3], float &yo)
{
    // ln chi uniform over the table range; rho half the time uniform over its range, half the time
    // rho = logit(r) of a uniform r, as in the sampling itself
    const uint4 w = philox_block(seed, id, step, 6u);
    const float u = 2.0f * u01_24(w.x) - 1.0f;
    const float c = (w.z & 1u) ? 1.0f : -1.0f;
    const float xr[3] = {M.in_m + M.in_h * u, 0.0f, c};
    const double r = (double)u01_24(w.y);
    const double rho = (w.z & 2u) ? log(r) - log1p(-r) : (double)M.rho_s * (2.0 * r - 1.0);
    float xs[3] = {xr[0], (float)rho, c};
    const double nu = icdf_nu(T, 2 * proc + (c > 0.0f ? 1 : 0), (double)xs[0], (double)xs[1]);
    mlp_normalize(M, xs, xo);
    yo = (float)((nu - (double)mlp_base(M, xs)) / (double)M.out_s);
}

// the coarse table: nu of the fine tables at node (c, i, j), one thread per node
__global__ void k_mlp_base(MlpDev M, TablesDev T, int proc, float *base)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * M.bnx * M.bny) return;
    const int c = e / (M.bnx * M.bny), i = (e / M.bny) % M.bnx, j = e % M.bny;
    base[e] = (float)icdf_nu(T, 2 * proc + c, (double)M.bx0 + (double)M.bhx * i, (double)M.by0 + (double)M.bhy * j);
}


// One training step's gradients.  xs/ys given (n samples: raw ln chi, rho, c and the target of
// the network output y): the gradient of sum_i (y(x_i) - ys_i)^2 over them; otherwise samples
// drawn from the tables with the residual over the coarse table as target.
__global__ void __launch_bounds__(kMlpBlock) k_mlp_grad(MlpDev M, TablesDev T, int proc, const float *xs, const float *ys,
                                                        int64_t n, uint64_t seed, int64_t step, int tiles_per_wave,
                                                        float *acc_out)
{
    __shared__ float G[kAcc];
    __shared__ MlpWave Wv[kMlpBlock / 64];
    __shared__ float yt[kMlpBlock / 64][16];
    __shared__ int ok[kMlpBlock / 64][16];
    for (int i = threadIdx.x; i < kAcc; i += blockDim.x) G[i] = 0.0f;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15;
    MlpWave &W = Wv[w];
    __syncthreads();
    for (int t = 0; t < tiles_per_wave; ++t) {
        const int64_t tile = ((int64_t)blockIdx.x * (kMlpBlock / 64) + w) * tiles_per_wave + t;
        if (l < 16) {
            const int64_t id = tile * 16 + l;
            float xo[3] = {0.0f, 0.0f, 1.0f}, yo = 0.0f;
            int valid = 1;
            if (xs) {
                valid = id < n;
                if (valid) {
                    mlp_normalize(M, xs + 3 * id, xo);
                    yo = ys[id];
                }
            } else {
                draw_sample(M, T, proc, seed, (uint64_t)id, step, xo, yo);
            }
            W.x[l][0] = xo[0]; W.x[l][1] = xo[1]; W.x[l][2] = xo[2];
            yt[w][l] = yo;
            ok[w][l] = valid;
        }
        __syncthreads();
        const float y = mlp_forward(M, W);
        const float e = ok[w][r] ? y - yt[w][r] : 0.0f;
        if (l < 16) {
            const float s = row_sum16(e * e);
            if (l == 0) atomicAdd(&G[kNP], s);
        }
        mlp_backward(M, W, 2.0f * e, G);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kAcc; i += blockDim.x) acc_out[(int64_t)blockIdx.x * kAcc + i] = G[i];
}

// sum of the block records (gradient and squared error) into out[kAcc]
__global__ void k_mlp_sum(const float *acc, int nblk, float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kAcc) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += acc[(int64_t)b * kAcc + i];
    out[i] = s;
}

// Adam (Kingma and Ba) on the mean gradient; loss[step] = mean squared error of the batch
__global__ void k_mlp_adam(float *p, float *m1, float *m2, const float *acc, int nblk, float inv_count, float lr, int t,
                           unsigned short *wt, float *loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kNP) return;
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += acc[(int64_t)b * kAcc + i];
    g *= inv_count;
    if (i == kNP) {
        if (loss) loss[0] = g;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float a = b1 * m1[i] + (1.0f - b1) * g, v = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    const float ah = a / (1.0f - powf(b1, (float)t)), vh = v / (1.0f - powf(b2, (float)t));
    const float x = p[i] - lr * ah / (sqrtf(vh) + eps);
    p[i] = x;
    wt[i] = f2bf(x);
}

__global__ void k_mlp_to_bf16(const float *p, unsigned short *wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNP) wt[i] = f2bf(p[i]);
}

// img[(L-2)*512 + (kc*4 + nb)*64 + lane][j] = W_L[k = kc*32 + 8(lane/16) + j][n = nb*16 + lane%16]
__global__ void k_mlp_image(const unsigned short *wt, s16x8 *img)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kImg) return;
    const int L = 2 + e / 512, kcnb = (e % 512) / 64, lane = e % 64;
    const int kc = kcnb / 4, nb = kcnb % 4;
    s16x8 v;
    for (int j = 0; j < 8; ++j)
        v[j] = (short)wt[kW(L) + (kc * 32 + 8 * (lane / 16) + j) * kH + nb * 16 + (lane % 16)];
    img[e] = v;
}

// nu for n samples given as raw (ln chi, rho, c); every wave takes 16-row tiles, block-uniformly.
// mode: QED_SURROGATE_AS_USED (the table inverse CDF in marked cells), QED_SURROGATE_NETWORK
// (base + network everywhere) or QED_SURROGATE_BASE (the coarse table alone)
__global__ void __launch_bounds__(kMlpBlock) k_mlp_eval(MlpDev M, TablesDev T, int proc, int mode, const float *xs,
                                                        int64_t n, float *nu)
{
    __shared__ MlpFwdWave Wv[kMlpBlock / 64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    MlpFwdWave &W = Wv[w];
    const int64_t ntiles = cdiv(n, 16);
    for (int64_t t0 = (int64_t)blockIdx.x * (kMlpBlock / 64); t0 < ntiles; t0 += (int64_t)gridDim.x * (kMlpBlock / 64)) {
        const int64_t tile = t0 + w;
        const int64_t id = tile * 16 + (l & 15);
        if (l < 16) {
            float xo[3] = {0.0f, 0.0f, 1.0f};
            if (id < n) mlp_normalize(M, xs + 3 * id, xo);
            W.x[l][0] = xo[0]; W.x[l][1] = xo[1]; W.x[l][2] = xo[2];
        }
        __syncthreads();
        const float y = mlp_forward(M, W);
        if (l < 16 && id < n) {
            const float *xr = xs + 3 * id;
            float v;
            if (mode == QED_SURROGATE_AS_USED && mlp_masked(M, xr))
                v = (float)icdf_nu(T, 2 * proc + (xr[2] > 0.0f ? 1 : 0), (double)xr[0], (double)xr[1]);
            else
                v = mlp_base(M, xr) + (mode == QED_SURROGATE_BASE ? 0.0f : M.out_s * y);
            nu[id] = v;
        }
        __syncthreads();
    }
}

// Largest |base + network - table| (base_only: |base - table|) over K x K points of every coarse
// cell (points at the centres of a K x K subdivision; cells, or points, outside |rho| <= ln 2^24
// are not sampled): sample e = cell * K^2 + point; errors as float bits, atomicMax (non-negative
// floats order as integers).
__global__ void __launch_bounds__(kMlpBlock) k_mlp_judge(MlpDev M, TablesDev T, int proc, int K, int64_t n,
                                                         int base_only, unsigned *cell_err)
{
    __shared__ MlpFwdWave Wv[kMlpBlock / 64];
    __shared__ float xr[kMlpBlock / 64][16][3];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    MlpFwdWave &W = Wv[w];
    const int ncy = M.bny - 1, ncx = M.bnx - 1;
    const int64_t ntiles = cdiv(n, 16);
    for (int64_t t0 = (int64_t)blockIdx.x * (kMlpBlock / 64); t0 < ntiles; t0 += (int64_t)gridDim.x * (kMlpBlock / 64)) {
        const int64_t e = (t0 + w) * 16 + (l & 15);
        const int64_t cell = e / (K * K);
        const int pt = (int)(e % (K * K));
        if (l < 16) {
            const int j = (int)(cell % ncy), i = (int)((cell / ncy) % ncx), c = (int)(cell / ((int64_t)ncy * ncx));
            xr[w][l][0] = M.bx0 + M.bhx * ((float)i + ((float)(pt / K) + 0.5f) / (float)K);
            xr[w][l][1] = M.by0 + M.bhy * ((float)j + ((float)(pt % K) + 0.5f) / (float)K);
            xr[w][l][2] = c ? 1.0f : -1.0f;
            float xo[3];
            mlp_normalize(M, xr[w][l], xo);
            W.x[l][0] = xo[0]; W.x[l][1] = xo[1]; W.x[l][2] = xo[2];
        }
        __syncthreads();
        const float y = base_only ? 0.0f : mlp_forward(M, W);       // base_only: block-uniform
        if (l < 16 && e < n && fabsf(xr[w][l][1]) <= kRho24) {
            const float *x = xr[w][l];
            const double tab = icdf_nu(T, 2 * proc + (x[2] > 0.0f ? 1 : 0), (double)x[0], (double)x[1]);
            const float err = (float)fabs((double)(mlp_base(M, x) + M.out_s * y) - tab);
            atomicMax(cell_err + cell, __float_as_uint(err));
        }
        __syncthreads();
    }
}

}  // namespace

struct qed_surrogate_s {
    qed_tables T;
    int proc;
    uint64_t seed;
    int64_t steps_done;
    float *p, *m1, *m2, *acc, *loss_tmp;
    unsigned short *wt;
    s16x8 *img;
    float *base;                 // coarse table [2][bnx][bny]
    uint32_t *mask;              // judged cells (bit per cell)
    unsigned *cell_err;          // largest sampled error per cell of the last judgement (float bits)
    float in_m, in_h, rho_s, out_s;
    float bx0, bhx, by0, bhy;
    int bnx, bny;
    int64_t n_masked;
    float bound;                 // of the last judgement (0: never judged)
};

namespace {
int64_t n_cells(const qed_surrogate_s *s) { return 2 * (int64_t)(s->bnx - 1) * (s->bny - 1); }

MlpDev mlp_dev(const qed_surrogate_s *s)
{
    MlpDev M;
    M.p = s->p;
    M.wt = s->wt;
    M.img = s->img;
    M.base = s->base;
    M.mask = s->mask;
    M.in_m = s->in_m; M.in_h = s->in_h; M.rho_s = s->rho_s; M.out_s = s->out_s;
    M.bx0 = s->bx0; M.bhx = s->bhx; M.by0 = s->by0; M.bhy = s->bhy;
    M.bnx = s->bnx; M.bny = s->bny;
    return M;
}

qed_status refresh_bf16(qed_surrogate s, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kNP + 255) / 256), dim3(256), 0, st, (const float *)s->p, s->wt);
    hipLaunchKernelGGL(k_mlp_image, dim3((kImg + 255) / 256), dim3(256), 0, st, (const unsigned short *)s->wt, s->img);
    return qs_launch_status("surrogate parameters");
}

hipError_t clear_judgement(qed_surrogate s, hipStream_t st)
{
    s->n_masked = 0;
    s->bound = 0.0f;
    return hipMemsetAsync(s->mask, 0, sizeof(uint32_t) * ((n_cells(s) + 31) / 32), st);
}

void surrogate_free(qed_surrogate s)
{
    if (!s) return;
    (void)hipFree(s->p); (void)hipFree(s->m1); (void)hipFree(s->m2); (void)hipFree(s->acc);
    (void)hipFree(s->loss_tmp); (void)hipFree(s->wt); (void)hipFree(s->img);
    (void)hipFree(s->base); (void)hipFree(s->mask); (void)hipFree(s->cell_err);
    delete s;
}
}  // namespace

// device view for the step kernels (qs_plan.hip)
MlpDev qs_surrogate_view(const qed_surrogate_s *s) { return mlp_dev(s); }
int qs_surrogate_process(const qed_surrogate_s *s) { return s->proc; }
const qed_tables_s *qs_surrogate_tables(const qed_surrogate_s *s) { return s->T; }

extern "C" int64_t qed_surrogate_n_params(void) { return kNP; }

extern "C" qed_status qed_surrogate_create(qed_tables T, int process, uint64_t seed, qed_surrogate *out)
{
    if (!T || !out || (process != 0 && process != 1)) return QED_ERR_INVALID;
    *out = nullptr;
    qs_clear_error();
    qed_surrogate s = new qed_surrogate_s();
    memset(s, 0, sizeof(*s));
    s->T = T;
    s->proc = process;
    s->seed = seed;
    const qed_table_grid &g = T->params.grid;
    const double lo = g.lnchi0[process], hi = g.lnchi0[process] + (g.n_chi[process] - 1) * g.dlnchi[process];
    s->in_m = (float)(0.5 * (lo + hi));
    s->in_h = (float)(0.5 * (hi - lo));
    s->rho_s = 17.0f;        // 24-bit uniforms: |rho| <= ln(2^24) = 16.64
    s->out_s = 1.0f;         // set below from the coarse table's error
    // coarse grid: the fine table's ln chi range in steps of at most ln(10)/kBaseChiPerDecade;
    // rho nodes every kBaseDrho from -kBaseRho to kBaseRho (the stencils of |rho| <= 16.64 stay
    // inside it)
    s->bnx = (int)ceil((hi - lo) / (log(10.0) / kBaseChiPerDecade) - 1e-9) + 1;
    s->bx0 = (float)lo;
    s->bhx = (float)((hi - lo) / (s->bnx - 1));
    s->bny = (int)lround(2.0 * kBaseRho / kBaseDrho) + 1;
    s->by0 = (float)-kBaseRho;
    s->bhy = (float)kBaseDrho;
    // He-style initialization from Philox channel 7 (uniform with the variance 2 / fan_in)
    std::vector<float> p(kNP, 0.0f);
    auto fill = [&](int off, int fan_in, int count) {
        const float a = sqrtf(6.0f / (float)fan_in);
        uint32_t w[4];
        for (int i = 0; i < count; i += 4) {
            // host Philox: same definition as the device one
            uint32_t c0 = (uint32_t)(off + i), c1 = 0u, c2 = 0u, c3 = 7u, k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
            for (int rr = 0; rr < 10; ++rr) {
                const uint64_t m0 = (uint64_t)0xD2511F53u * c0, m1 = (uint64_t)0xCD9E8D57u * c2;
                const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
                c0 = n0; c1 = (uint32_t)m1; c2 = n2; c3 = (uint32_t)m0;
                k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
            }
            w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
            for (int j = 0; j < 4 && i + j < count; ++j)
                p[off + i + j] = a * (2.0f * ((float)(w[j] >> 8) + 0.5f) * 0x1p-24f - 1.0f);
        }
    };
    fill(kW1, 3, 3 * kH);
    for (int L = 2; L <= 4; ++L) fill(kW(L), kH, kH * kH);
    fill(kW5, kH, kH);
    hipError_t e = hipMalloc((void **)&s->p, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMalloc((void **)&s->m1, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMalloc((void **)&s->m2, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMalloc((void **)&s->acc, sizeof(float) * kAcc * kGradGrid);
    if (e == hipSuccess) e = hipMalloc((void **)&s->loss_tmp, sizeof(float) * kAcc);
    if (e == hipSuccess) e = hipMalloc((void **)&s->wt, sizeof(unsigned short) * kNP);
    if (e == hipSuccess) e = hipMalloc((void **)&s->img, sizeof(s16x8) * kImg);
    if (e == hipSuccess) e = hipMalloc((void **)&s->base, sizeof(float) * 2 * s->bnx * s->bny);
    if (e == hipSuccess) e = hipMalloc((void **)&s->mask, sizeof(uint32_t) * ((n_cells(s) + 31) / 32));
    if (e == hipSuccess) e = hipMalloc((void **)&s->cell_err, sizeof(unsigned) * n_cells(s));
    if (e == hipSuccess) e = hipMemset(s->mask, 0, sizeof(uint32_t) * ((n_cells(s) + 31) / 32));
    if (e == hipSuccess) e = hipMemset(s->cell_err, 0, sizeof(unsigned) * n_cells(s));
    if (e == hipSuccess) e = hipMemcpy(s->p, p.data(), sizeof(float) * kNP, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->m1, 0, sizeof(float) * kNP);
    if (e == hipSuccess) e = hipMemset(s->m2, 0, sizeof(float) * kNP);
    if (e != hipSuccess) {
        surrogate_free(s);
        return qs_fail(e, "qed_surrogate_create");
    }
    qed_status st = refresh_bf16(s, nullptr);
    if (st == QED_OK) {
        const int nb = 2 * s->bnx * s->bny;
        hipLaunchKernelGGL(k_mlp_base, dim3((nb + 255) / 256), dim3(256), 0, nullptr, mlp_dev(s), T->dev, process, s->base);
        st = qs_launch_status("qed_surrogate_create");
    }
    if (st == QED_OK) {      // the residual scale: the coarse table's largest error, 8 x 8 points per cell
        const int K = 8;
        const int64_t n = n_cells(s) * K * K, blocks = cdiv(cdiv(n, 16), kMlpBlock / 64);
        hipLaunchKernelGGL(k_mlp_judge, dim3((int)(blocks < 4096 ? blocks : 4096)), dim3(kMlpBlock), 0, nullptr,
                           mlp_dev(s), T->dev, process, K, n, 1, s->cell_err);
        std::vector<unsigned> bits(n_cells(s));
        st = qs_launch_status("qed_surrogate_create");
        if (st == QED_OK && (e = hipMemcpy(bits.data(), s->cell_err, sizeof(unsigned) * bits.size(),
                                           hipMemcpyDeviceToHost)) != hipSuccess)
            st = qs_fail(e, "qed_surrogate_create");
        float mx = 0.0f;
        for (unsigned b : bits) {
            float v;
            memcpy(&v, &b, 4);
            mx = v > mx ? v : mx;
        }
        s->out_s = mx > 0.0f ? kResidualMargin * mx : 1.0f;
        if (st == QED_OK && (e = hipMemset(s->cell_err, 0, sizeof(unsigned) * n_cells(s))) != hipSuccess)
            st = qs_fail(e, "qed_surrogate_create");
    }
    if (st == QED_OK && (e = hipDeviceSynchronize()) != hipSuccess) st = qs_fail(e, "qed_surrogate_create");
    if (st != QED_OK) {
        surrogate_free(s);
        return st;
    }
    *out = s;
    return QED_OK;
}

extern "C" qed_status qed_surrogate_norm(qed_surrogate s, float *out4)
{
    if (!s || !out4) return QED_ERR_INVALID;
    out4[0] = s->in_m; out4[1] = s->in_h; out4[2] = s->rho_s; out4[3] = s->out_s;
    return QED_OK;
}

extern "C" qed_status qed_surrogate_train(qed_surrogate s, int steps, int tiles_per_wave, float lr, float *d_loss,
                                          qed_stream stream)
{
    if (!s || steps < 0 || tiles_per_wave <= 0 || !(lr > 0.0f)) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    QS_CHECK(clear_judgement(s, st));
    const MlpDev M = mlp_dev(s);
    const float inv = 1.0f / (float)((int64_t)kGradGrid * (kMlpBlock / 64) * tiles_per_wave * 16);
    for (int k = 0; k < steps; ++k) {
        const int64_t t = ++s->steps_done;
        hipLaunchKernelGGL(k_mlp_grad, dim3(kGradGrid), dim3(kMlpBlock), 0, st, M, s->T->dev, s->proc, (const float *)nullptr,
                           (const float *)nullptr, (int64_t)0, s->seed, t, tiles_per_wave, s->acc);
        hipLaunchKernelGGL(k_mlp_adam, dim3((kAcc + 255) / 256), dim3(256), 0, st, s->p, s->m1, s->m2, (const float *)s->acc,
                           kGradGrid, inv, lr, (int)t, s->wt, d_loss ? d_loss + k : (float *)nullptr);
        hipLaunchKernelGGL(k_mlp_image, dim3((kImg + 255) / 256), dim3(256), 0, st, (const unsigned short *)s->wt, s->img);
    }
    return qs_launch_status("qed_surrogate_train");
}

extern "C" qed_status qed_surrogate_gradient(qed_surrogate s, const float *d_x, const float *d_nu, int64_t n,
                                             float *d_grad, qed_stream stream)
{
    if (!s || !d_x || !d_nu || !d_grad || n <= 0) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    const int64_t tiles = cdiv(n, 16);
    const int64_t blocks = cdiv(tiles, kMlpBlock / 64);
    if (blocks > kGradGrid) return QED_ERR_CAPACITY;
    hipLaunchKernelGGL(k_mlp_grad, dim3((int)blocks), dim3(kMlpBlock), 0, st, mlp_dev(s), s->T->dev, s->proc, d_x, d_nu, n,
                       s->seed, (int64_t)0, 1, s->acc);
    hipLaunchKernelGGL(k_mlp_sum, dim3((kAcc + 255) / 256), dim3(256), 0, st, (const float *)s->acc, (int)blocks, d_grad);
    return qs_launch_status("qed_surrogate_gradient");
}

extern "C" qed_status qed_surrogate_eval(qed_surrogate s, const float *d_x, int64_t n, int mode, float *d_nu,
                                         qed_stream stream)
{
    if (!s || !d_x || !d_nu || n < 0 || mode < QED_SURROGATE_AS_USED || mode > QED_SURROGATE_BASE) return QED_ERR_INVALID;
    if (n == 0) return QED_OK;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    const int64_t blocks = cdiv(cdiv(n, 16), kMlpBlock / 64);
    hipLaunchKernelGGL(k_mlp_eval, dim3((int)(blocks < 4096 ? blocks : 4096)), dim3(kMlpBlock), 0, st, mlp_dev(s),
                       s->T->dev, s->proc, mode, d_x, n, d_nu);
    return qs_launch_status("qed_surrogate_eval");
}

extern "C" qed_status qed_surrogate_judge(qed_surrogate s, float bound, int points_per_axis, float *cell_err,
                                          int64_t *n_masked, qed_stream stream)
{
    if (!s || !(bound >= 0.0f) || points_per_axis < 1 || points_per_axis > 64) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    const int64_t nc = n_cells(s), n = nc * points_per_axis * points_per_axis;
    QS_CHECK(hipMemsetAsync(s->cell_err, 0, sizeof(unsigned) * nc, st));
    const int64_t blocks = cdiv(cdiv(n, 16), kMlpBlock / 64);
    hipLaunchKernelGGL(k_mlp_judge, dim3((int)(blocks < 4096 ? blocks : 4096)), dim3(kMlpBlock), 0, st, mlp_dev(s),
                       s->T->dev, s->proc, points_per_axis, n, 0, s->cell_err);
    qed_status r = qs_launch_status("qed_surrogate_judge");
    if (r != QED_OK) return r;
    std::vector<unsigned> bits(nc);
    QS_CHECK(hipMemcpyAsync(bits.data(), s->cell_err, sizeof(unsigned) * nc, hipMemcpyDeviceToHost, st));
    QS_CHECK(hipStreamSynchronize(st));
    std::vector<uint32_t> mask((nc + 31) / 32, 0u);
    int64_t m = 0;
    for (int64_t c = 0; c < nc; ++c) {
        float v;
        memcpy(&v, &bits[c], 4);
        if (cell_err) cell_err[c] = v;
        if (v > bound) {
            mask[c >> 5] |= 1u << (c & 31);
            ++m;
        }
    }
    QS_CHECK(hipMemcpyAsync(s->mask, mask.data(), sizeof(uint32_t) * mask.size(), hipMemcpyHostToDevice, st));
    QS_CHECK(hipStreamSynchronize(st));
    s->n_masked = m;
    s->bound = bound;
    if (n_masked) *n_masked = m;
    return QED_OK;
}

extern "C" qed_status qed_surrogate_get_info(qed_surrogate s, qed_surrogate_info *out)
{
    if (!s || !out) return QED_ERR_INVALID;
    out->process = s->proc;
    out->n_params = kNP;
    out->in_m = s->in_m; out->in_h = s->in_h; out->rho_s = s->rho_s; out->out_s = s->out_s;
    out->base_lnchi0 = s->bx0; out->base_dlnchi = s->bhx; out->base_n_chi = s->bnx;
    out->base_rho0 = s->by0; out->base_drho = s->bhy; out->base_n_rho = s->bny;
    out->n_cells = n_cells(s);
    out->n_masked = s->n_masked;
    out->bound = s->bound;
    out->bytes_network = (int64_t)kNP * 2;
    out->bytes_base = (int64_t)2 * s->bnx * s->bny * 4;
    out->bytes_mask = (int64_t)((n_cells(s) + 31) / 32) * 4;
    return QED_OK;
}

extern "C" qed_status qed_surrogate_get_params(qed_surrogate s, float *d_params, qed_stream stream)
{
    if (!s || !d_params) return QED_ERR_INVALID;
    qs_clear_error();
    QS_CHECK(hipMemcpyAsync(d_params, s->p, sizeof(float) * kNP, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return QED_OK;
}

extern "C" qed_status qed_surrogate_set_params(qed_surrogate s, const float *d_params, qed_stream stream)
{
    if (!s || !d_params) return QED_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    qs_clear_error();
    QS_CHECK(hipMemcpyAsync(s->p, d_params, sizeof(float) * kNP, hipMemcpyDeviceToDevice, st));
    QS_CHECK(clear_judgement(s, st));
    return refresh_bf16(s, st);
}

extern "C" qed_status qed_surrogate_destroy(qed_surrogate s)
{
    if (s) {
        (void)hipDeviceSynchronize();
        surrogate_free(s);
    }
    return QED_OK;
}
