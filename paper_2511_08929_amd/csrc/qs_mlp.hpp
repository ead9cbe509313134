// qs_mlp.hpp -- the learned inverse CDF: nu(ln chi, rho, c) = base(ln chi, rho, c) + out_s y, with
// base a coarse FP32 table of nu (4-point Lagrange in ln chi and rho, a few nodes per decade and
// per unit of rho) and y a multilayer perceptron with inputs u = (ln chi - m)/h, v = rho/rho_s and
// the channel c = -1 / +1 (spin down / up for NLC, xi3 = -1 / +1 for NBW), four hidden layers of
// 64 SiLU units and one linear output.  It stands in for the two fine inverse-CDF tables of one
// process (NLCS and NBW implementation sections tabulate only these two channels).  The fine
// tables judge it: every cell of the coarse grid whose largest sampled error exceeds a stated
// bound is marked, and in a marked cell the table inverse CDF is used instead.
//
// Precision: weights and activations enter the three 64x64 layers as BF16 on the matrix cores
// (v_mfma_f32_16x16x32_bf16, two per 16 x 16 output block), accumulation and everything else in
// FP32.
//
// A wave evaluates 16 samples (rows) at a time.  MFMA operand layouts (16x16x32): lane l holds
//   A[m = l%16][k = 8(l/16) + j],  B[k = 8(l/16) + j][n = l%16]  (j < 8),
//   D[m = 4(l/16) + j][n = l%16]  (j < 4);
// the weight-gradient products (K = the 16 rows of a tile) use the 16x16x16 form, whose lane l
// holds A[m = l%16][k = 4(l/16) + j] and B[k = 4(l/16) + j][n = l%16] (j < 4), D as above.
// Activations pass between layers through LDS (the D layout of one layer is transposed with
// respect to the A layout of the next).  All waves of a block call these functions the same
// number of times: they synchronize the block.
#pragma once
#include "qs_pass.hpp"

namespace qs {
namespace mlp {
constexpr int kH = 64;
constexpr int kW1 = 0;                       // W1[j][k], j = input 0..2, k = unit
constexpr int kB1 = 3 * kH;
constexpr int kL2 = 4 * kH;
constexpr int kLayer = kH * kH + kH;
__host__ __device__ constexpr int kW(int l) { return kL2 + (l - 2) * kLayer; }   // W_l[k][n], l = 2, 3, 4
__host__ __device__ constexpr int kB(int l) { return kW(l) + kH * kH; }
constexpr int kW5 = kL2 + 3 * kLayer;
constexpr int kB5 = kW5 + kH;
constexpr int kNP = kB5 + 1;                 // 12801 parameters
constexpr int kImg = 3 * 8 * 64;             // bf16x8 entries of the B-operand image of W2..W4
}  // namespace mlp

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// D += A B over K = 32 (16 x 16 output), operands as BF16 bit patterns
__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 d)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), d, 0, 0,
                                                   0);
}

__host__ __device__ inline unsigned short f2bf(float f)    // round to nearest even (finite f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

struct MlpDev {
    const float *p;              // FP32 master parameters [kNP] (training only)
    const unsigned short *wt;    // BF16 copy of every parameter [kNP] (layouts as in p)
    const s16x8 *img;            // W2..W4 as B operands: img[(l-2)*512 + (kc*4 + nb)*64 + lane]
    const float *base;           // coarse nu nodes [2 channels][bnx][bny]
    const uint32_t *mask;        // judged cells, bit (c (bnx-1) + i) (bny-1) + j: table inverse CDF
                                 // there (NULL: no cell marked)
    float in_m, in_h, rho_s, out_s;
    float bx0, bhx, by0, bhy;    // coarse grid: ln chi = bx0 + i bhx, rho = by0 + j bhy
    int bnx, bny;
};

// coarse cell of raw inputs (ln chi, rho, c): the node interval of each axis, clamped to the grid
__device__ __forceinline__ int mlp_cell(const MlpDev &M, const float *xr)
{
    int i = (int)floorf((xr[0] - M.bx0) / M.bhx), j = (int)floorf((xr[1] - M.by0) / M.bhy);
    i = i < 0 ? 0 : (i > M.bnx - 2 ? M.bnx - 2 : i);
    j = j < 0 ? 0 : (j > M.bny - 2 ? M.bny - 2 : j);
    return ((xr[2] > 0.0f ? 1 : 0) * (M.bnx - 1) + i) * (M.bny - 1) + j;
}

__device__ __forceinline__ bool mlp_masked(const MlpDev &M, const float *xr)
{
    if (!M.mask) return false;
    const int b = mlp_cell(M, xr);
    return (M.mask[b >> 5] >> (b & 31)) & 1u;
}

// coarse-table nu at raw inputs (the lookup of the fine tables, in FP32 on the coarse nodes)
__device__ __forceinline__ float mlp_base(const MlpDev &M, const float *xr)
{
    float Lx[4], Ly[4];
    const int i0 = lagrange4(xr[0], M.bx0, M.bhx, M.bnx, Lx);
    const int j0 = lagrange4(xr[1], M.by0, M.bhy, M.bny, Ly);
    const float *b = M.base + ((int64_t)(xr[2] > 0.0f ? 1 : 0) * M.bnx + i0) * M.bny + j0;
    float acc = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const float *r = b + a * M.bny;
        acc += Lx[a] * (Ly[0] * r[0] + Ly[1] * r[1] + Ly[2] * r[2] + Ly[3] * r[3]);
    }
    return acc;
}

struct MlpWave {
    float z[4][16][mlp::kH];     // pre-activations of the hidden layers
    float dz[16][mlp::kH];       // backward: gradient of the loss w.r.t. the current z
    float x[16][3];              // normalized inputs u, v, c
};

// What the forward pass alone needs of a wave's LDS: one pre-activation buffer, reused by every
// layer (a wave reads a layer's buffer into registers before it writes the next layer's).
struct MlpFwdWave {
    float z[1][16][mlp::kH];
    float x[16][3];
};

// pre-activations of hidden layer k (0..3)
__device__ __forceinline__ float (*zbuf(MlpWave &W, int k))[mlp::kH] { return W.z[k]; }
__device__ __forceinline__ float (*zbuf(MlpFwdWave &W, int))[mlp::kH] { return W.z[0]; }

// network inputs from the raw ones (ln chi, rho, channel sign)
__device__ __forceinline__ void mlp_normalize(const MlpDev &M, const float *xr, float xo[3])
{
    xo[0] = (xr[0] - M.in_m) / M.in_h;
    xo[1] = xr[1] / M.rho_s;
    xo[2] = xr[2] > 0.0f ? 1.0f : -1.0f;
}

__device__ __forceinline__ float silu_f(float z) { return z * rcp_r(1.0f + exp_r(-z)); }
__device__ __forceinline__ float dsilu_f(float z)
{
    const float s = rcp_r(1.0f + exp_r(-z));
    return s * (1.0f + z * (1.0f - s));
}

// Forward pass of the 16 rows in W.x; returns y of row l%16 in every lane.  With an MlpWave it
// leaves the pre-activations of every layer in W.z (for the backward pass).
template <class WV> __device__ inline float mlp_forward(const MlpDev &M, WV &W)
{
    using namespace mlp;
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const unsigned short *wt = M.wt;
    s16x8 a[2];                      // A operand: activations of row r, units kc*32 + 8q + j
    const float x0 = W.x[r][0], x1 = W.x[r][1], x2 = W.x[r][2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kc * 32 + 8 * q + j;
            const float z = bf2f(wt[kB1 + k]) + bf2f(wt[kW1 + k]) * x0 + bf2f(wt[kW1 + kH + k]) * x1 +
                            bf2f(wt[kW1 + 2 * kH + k]) * x2;
            zbuf(W, 0)[r][k] = z;
            a[kc][j] = (short)f2bf(silu_f(z));
        }
    }
    for (int L = 2; L <= 4; ++L) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const float bias = bf2f(wt[kB(L) + nb * 16 + r]);
            f32x4 acc = {bias, bias, bias, bias};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) acc = mfma32(a[kc], M.img[(L - 2) * 512 + (kc * 4 + nb) * 64 + l], acc);
#pragma unroll
            for (int j = 0; j < 4; ++j) zbuf(W, L - 1)[4 * q + j][nb * 16 + r] = acc[j];
        }
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
#pragma unroll
            for (int j = 0; j < 8; ++j) a[kc][j] = (short)f2bf(silu_f(zbuf(W, L - 1)[r][kc * 32 + 8 * q + j]));
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int k = 16 * q + j;
        s += bf2f(wt[kW5 + k]) * silu_f(zbuf(W, 3)[r][k]);
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s + bf2f(wt[kB5]);
}

// sum over the 16 rows held by lanes q*16 .. q*16+15 (same q), result in every one of them
__device__ __forceinline__ float row_sum16(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Backward pass after mlp_forward on the same W: dy = dLoss/dy of row l%16 (every lane of the
// row holds it, 0 for padding rows).  Adds the parameter gradients to G[kNP] (LDS) atomically.
__device__ inline void mlp_backward(const MlpDev &M, MlpWave &W, float dy, float *G)
{
    using namespace mlp;
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const unsigned short *wt = M.wt;
    // output layer
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const int k = 16 * q + j;
        const float z = W.z[3][r][k];
        const float g = row_sum16(dy * silu_f(z));
        if (r == 0) atomicAdd(&G[kW5 + k], g);
        W.dz[r][k] = dy * bf2f(wt[kW5 + k]) * dsilu_f(z);
    }
    if (l < 16) {
        const float g = row_sum16(dy);
        if (l == 0) atomicAdd(&G[kB5], g);
    }
    __syncthreads();
    for (int L = 4; L >= 2; --L) {
        // dW_L[k][n] += sum_i h[i][k] dz[i][n]   (M = k, N = n, K = the 16 rows)
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            bf16x4 ha;
#pragma unroll
            for (int j = 0; j < 4; ++j) ha[j] = (short)f2bf(silu_f(W.z[L - 2][4 * q + j][mb * 16 + r]));
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                bf16x4 db;
#pragma unroll
                for (int j = 0; j < 4; ++j) db[j] = (short)f2bf(W.dz[4 * q + j][nb * 16 + r]);
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ha, db, acc, 0, 0, 0);
#pragma unroll
                for (int j = 0; j < 4; ++j) atomicAdd(&G[kW(L) + (mb * 16 + 4 * q + j) * kH + nb * 16 + r], acc[j]);
            }
        }
        {   // db_L[n]: lane n sums its column over the rows
            float s = 0.0f;
#pragma unroll 4
            for (int i = 0; i < 16; ++i) s += W.dz[i][l];
            atomicAdd(&G[kB(L) + l], s);
        }
        // dh[i][k] = sum_n dz[i][n] W_L[k][n]   (M = i, N = k, K = n)
        f32x4 dh[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) dh[nb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            s16x8 da;
#pragma unroll
            for (int j = 0; j < 8; ++j) da[j] = (short)f2bf(W.dz[r][kc * 32 + 8 * q + j]);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                s16x8 wb;
                const unsigned short *row = wt + kW(L) + (nb * 16 + r) * kH + kc * 32 + 8 * q;
#pragma unroll
                for (int j = 0; j < 8; ++j) wb[j] = (short)row[j];
                dh[nb] = mfma32(da, wb, dh[nb]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 4 * q + j, k = nb * 16 + r;
                W.dz[i][k] = dh[nb][j] * dsilu_f(W.z[L - 2][i][k]);
            }
        __syncthreads();
    }
    // first layer: lane k
    float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gb = 0.0f;
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        const float d = W.dz[i][l];
        g0 += d * W.x[i][0];
        g1 += d * W.x[i][1];
        g2 += d * W.x[i][2];
        gb += d;
    }
    atomicAdd(&G[kW1 + l], g0);
    atomicAdd(&G[kW1 + kH + l], g1);
    atomicAdd(&G[kW1 + 2 * kH + l], g2);
    atomicAdd(&G[kB1 + l], gb);
    __syncthreads();
}

}  // namespace qs

// for the step kernels (defined in qs_mlp.hip)
qs::MlpDev qs_surrogate_view(const qed_surrogate_s *s);
int qs_surrogate_process(const qed_surrogate_s *s);
const qed_tables_s *qs_surrogate_tables(const qed_surrogate_s *s);
