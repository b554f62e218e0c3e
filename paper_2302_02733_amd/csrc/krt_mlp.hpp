// Surrogate of the kappa coefficients: an MLP 4 -> 64 -> 64 -> 64 -> 8 with
// SiLU activations that maps (kappa, w, X, cos theta) to the eight
// dimensionless integrals (as standardised log10 values).
//
// Definition (training and inference compute this function):
//   features  x = ((kappa - 5.5)/2.5, (log10 w - 0.75)/1.25, (log10 X - 2.5)/4.5, cos theta)
//   h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), h3 = silu(W3 h2 + b3),
//   z = W4 h3 + b4,
//   log10 I_k = sum_j c_kj m_j(x) + mu_k + sd_k z_k,  silu(t) = t / (1 + e^-t),
// with every weight matrix rounded to bfloat16 (nearest even) and FP32
// biases; m_j are the 20 monomials of degree <= 3 in (x0, x1, x2), in the
// order 1, x0, x1, x2, x0x0, x0x1, x0x2, x1x1, x1x2, x2x2, x0x0x0, x0x0x1,
// x0x0x2, x0x1x1, x0x1x2, x0x2x2, x1x1x1, x1x1x2, x1x2x2, x2x2x2.  The cubic
// baseline c is the least-squares fit of log10 I on the training set (it
// takes out the integrals' many-decade trends), mu and sd the mean and
// spread of what it leaves, which the network learns.  Loss: the mean over
// samples and outputs of (z_k - t_k)^2, t = (log10 I - baseline - mu) / sd.
// Domain: kappa in [3, 8], w in [10^-0.5, 10^2], X in [1e-2, 1e7]; outside it
// the exact integrator is used.
//
// Training (FP32 vector ALU): per block 32 samples, forward and backward
// through LDS-resident activations, per-block gradient partials, then one
// kernel that sums them in a fixed order and takes an Adam step on the FP32
// master weights.
// Inference (bf16 MFMA): a wave evaluates the network for its 64 lanes with
// v_mfma_f32_32x32x16_bf16, rays along N (two 32-ray tiles), hidden units
// along M; activations enter the MFMA as hi + lo bfloat16 pairs (two MFMAs,
// exact products, FP32 accumulation), so only the weights carry bfloat16
// rounding.  The K order of each layer's packed weights follows the lane
// layout of the previous layer's accumulators, so no data moves between
// lanes between layers.
#pragma once

#include "krt_device.hpp"

namespace krt {

constexpr int kMlpIn = 4, kMlpH = 64, kMlpOut = 8;
constexpr int kOffW1 = 0;                           // [64][4]
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;     // 256
constexpr int kOffW2 = kOffB1 + kMlpH;              // [64][64]
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH * kMlpH;
constexpr int kOffW4 = kOffB3 + kMlpH;              // [8][64]
constexpr int kOffB4 = kOffW4 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOffB4 + kMlpOut;        // 9160

constexpr double kKapMin = 3.0, kKapMax = 8.0, kWMin = 0.31622776601683794, kWMax = 1e2, kXMin = 1e-2, kXMax = 1e7;
constexpr int kPolyTerms = 20;
constexpr int kNormLen = 16 + 8 * kPolyTerms;   // mu[8], sd[8], c[8][20]

KRT_HD bool mlp_in_domain(double kap, double w, double X) {
    return kap >= kKapMin && kap <= kKapMax && w >= kWMin && w <= kWMax && X >= kXMin && X <= kXMax;
}

KRT_HD void mlp_features(double kap, double w, double X, double cth, float f[4]) {
    f[0] = (float)((kap - 5.5) * 0.4);
    f[1] = (float)((log10(w) - 0.75) * 0.8);
    f[2] = (float)((log10(X) - 2.5) * (1.0 / 4.5));
    f[3] = (float)cth;
}

// The 20 monomials of degree <= 3 in (x0, x1, x2), in the documented order.
template <class T>
KRT_HD void mlp_monomials(T a, T b, T c, T m[kPolyTerms]) {
    m[0] = T(1);
    m[1] = a; m[2] = b; m[3] = c;
    m[4] = a * a; m[5] = a * b; m[6] = a * c; m[7] = b * b; m[8] = b * c; m[9] = c * c;
    m[10] = a * a * a; m[11] = a * a * b; m[12] = a * a * c; m[13] = a * b * b; m[14] = a * b * c;
    m[15] = a * c * c; m[16] = b * b * b; m[17] = b * b * c; m[18] = b * c * c; m[19] = c * c * c;
}

// Round to bfloat16, nearest even (finite inputs), returned as float.
KRT_HD float bf16_round(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    return __builtin_bit_cast(float, u);
}

KRT_HD float silu_f(float z) { return z / (1.0f + expf(-z)); }
KRT_HD float silu_grad(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// Training: one block of 256 threads per 32 samples.  Thread (u = lane,
// group = wave) owns hidden unit u for samples 8 group .. 8 group + 7 in the
// forward pass.  Activations H and SiLU slopes G of the three hidden layers
// and two gradient buffers live in LDS as [64][33] (padded rows: lanes that
// walk the unit index hit distinct banks); the weights are staged in LDS
// rounded to bfloat16, W2 and W3 with padded rows.
// ---------------------------------------------------------------------------
constexpr int kTrainTile = 32;
constexpr int kLd = kTrainTile + 1;
constexpr int kLdW = kMlpH + 1;

struct MlpTrainArgs {
    const float* P;       // master parameters [kMlpParams]
    const float* feat;    // [n][4]
    const float* targ;    // [n][8] standardised log10 integrals
    int64_t n;            // samples in the set
    int64_t first;        // first position of this batch in the (permuted) order
    int64_t count;        // samples in the batch
    uint64_t perm_a, perm_c;  // position -> sample: (a p + c) mod n (n a power of two), or identity
    int permute;
    float inv_norm;       // 1 / (8 * batch size) of the loss
    float* gpart;         // [gridDim.x][kMlpParams]
    double* lpart;        // [gridDim.x] sums of squared errors
};

__device__ __forceinline__ int64_t mlp_sample(const MlpTrainArgs& A, int64_t pos) {
    if (!A.permute) return pos;
    return (int64_t)((A.perm_a * (uint64_t)pos + A.perm_c) & (uint64_t)(A.n - 1));
}

__global__ __launch_bounds__(256) void mlp_train_tile(MlpTrainArgs A) {
    __shared__ float sW1[kMlpH * 5], sB1[kMlpH], sW2[kMlpH * kLdW], sB2[kMlpH], sW3[kMlpH * kLdW], sB3[kMlpH];
    __shared__ float sW4[kMlpOut * kMlpH], sB4[kMlpOut];
    __shared__ float sX[kTrainTile][4], sT[kTrainTile][8], sY[kMlpOut][kTrainTile];
    __shared__ float sH[3][kMlpH * kLd], sG[3][kMlpH * kLd], sDa[kMlpH * kLd], sDb[kMlpH * kLd];
    __shared__ double sL[256];
    const int t = threadIdx.x;
    const int u = t & 63, grp = t >> 6;
    for (int k = t; k < kMlpH * kMlpH; k += 256) {
        const int r = k >> 6, c = k & 63;
        sW2[r * kLdW + c] = bf16_round(A.P[kOffW2 + k]);
        sW3[r * kLdW + c] = bf16_round(A.P[kOffW3 + k]);
    }
    for (int k = t; k < kMlpH * 4; k += 256) sW1[(k >> 2) * 5 + (k & 3)] = bf16_round(A.P[kOffW1 + k]);
    for (int k = t; k < kMlpOut * kMlpH; k += 256) sW4[k] = bf16_round(A.P[kOffW4 + k]);
    if (t < kMlpH) {
        sB1[t] = A.P[kOffB1 + t];
        sB2[t] = A.P[kOffB2 + t];
        sB3[t] = A.P[kOffB3 + t];
    }
    if (t < kMlpOut) sB4[t] = A.P[kOffB4 + t];
    const int64_t base = A.first + (int64_t)blockIdx.x * kTrainTile;
    const int64_t end = A.first + A.count;
    if (t < kTrainTile * 4) {
        const int s = t >> 2;
        sX[s][t & 3] = (base + s < end) ? A.feat[mlp_sample(A, base + s) * 4 + (t & 3)] : 0.0f;
    }
    {
        const int s = t >> 3;
        sT[s][t & 7] = (base + s < end) ? A.targ[mlp_sample(A, base + s) * 8 + (t & 7)] : 0.0f;
    }
    __syncthreads();
    const int s0 = grp * 8;
    float acc[16];
    // layer 1
    for (int q = 0; q < 8; ++q) {
        float z = sB1[u];
        for (int k = 0; k < 4; ++k) z += sW1[u * 5 + k] * sX[s0 + q][k];
        sH[0][u * kLd + s0 + q] = silu_f(z);
        sG[0][u * kLd + s0 + q] = silu_grad(z);
    }
    __syncthreads();
    // layers 2 and 3
    for (int L = 1; L <= 2; ++L) {
        const float* W = L == 1 ? sW2 : sW3;
        const float* Bv = L == 1 ? sB2 : sB3;
        for (int q = 0; q < 8; ++q) acc[q] = Bv[u];
        for (int k = 0; k < kMlpH; ++k) {
            const float wv = W[u * kLdW + k];
            for (int q = 0; q < 8; ++q) acc[q] += wv * sH[L - 1][k * kLd + s0 + q];
        }
        for (int q = 0; q < 8; ++q) {
            sH[L][u * kLd + s0 + q] = silu_f(acc[q]);
            sG[L][u * kLd + s0 + q] = silu_grad(acc[q]);
        }
        __syncthreads();
    }
    // output layer and loss: thread -> (output o, sample s)
    double lsum = 0.0;
    {
        const int o = t >> 5, s = t & 31;
        float z = sB4[o];
        for (int j = 0; j < kMlpH; ++j) z += sW4[o * kMlpH + j] * sH[2][j * kLd + s];
        const float d = (base + s < end) ? z - sT[s][o] : 0.0f;
        lsum = (double)d * (double)d;
        sY[o][s] = 2.0f * d * A.inv_norm;   // dL/dz
    }
    sL[t] = lsum;
    __syncthreads();
    float* g = A.gpart + (size_t)blockIdx.x * kMlpParams;
    // output layer: dW4[o][j] = sum_s dY[o][s] h3[j][s], db4
    for (int k = t; k < kMlpOut * kMlpH; k += 256) {
        const int o = k >> 6, j = k & 63;
        float s = 0.0f;
        for (int q = 0; q < kTrainTile; ++q) s += sY[o][q] * sH[2][j * kLd + q];
        g[kOffW4 + k] = s;
    }
    if (t < kMlpOut) {
        float s = 0.0f;
        for (int q = 0; q < kTrainTile; ++q) s += sY[t][q];
        g[kOffB4 + t] = s;
    }
    // dZ3 = G3 (W4^T dY) -> sDa
    for (int q = 0; q < 8; ++q) {
        float s = 0.0f;
        for (int o = 0; o < kMlpOut; ++o) s += sW4[o * kMlpH + u] * sY[o][s0 + q];
        sDa[u * kLd + s0 + q] = s * sG[2][u * kLd + s0 + q];
    }
    __syncthreads();
    // hidden layers, top down
    float* dz = sDa;
    float* dzn = sDb;
    for (int L = 2; L >= 1; --L) {
        const float* W = L == 2 ? sW3 : sW2;
        const int offw = L == 2 ? kOffW3 : kOffW2, offb = L == 2 ? kOffB3 : kOffB2;
        // dW[h = u][k = 16 grp + q] = sum_s dZ[h][s] H_(L-1)[k][s]
        for (int q = 0; q < 16; ++q) acc[q] = 0.0f;
        for (int s = 0; s < kTrainTile; ++s) {
            const float d = dz[u * kLd + s];
            for (int q = 0; q < 16; ++q) acc[q] += d * sH[L - 1][(16 * grp + q) * kLd + s];
        }
        for (int q = 0; q < 16; ++q) g[offw + u * kMlpH + 16 * grp + q] = acc[q];
        if (grp == 0) {
            float s = 0.0f;
            for (int q = 0; q < kTrainTile; ++q) s += dz[u * kLd + q];
            g[offb + u] = s;
        }
        // dZ_(L-1)[k = u][s] = G_(L-1)[k][s] sum_h W[h][k] dZ[h][s]
        for (int q = 0; q < 8; ++q) acc[q] = 0.0f;
        for (int h = 0; h < kMlpH; ++h) {
            const float wv = W[h * kLdW + u];
            for (int q = 0; q < 8; ++q) acc[q] += wv * dz[h * kLd + s0 + q];
        }
        for (int q = 0; q < 8; ++q) dzn[u * kLd + s0 + q] = acc[q] * sG[L - 1][u * kLd + s0 + q];
        __syncthreads();
        float* tmp = dz;
        dz = dzn;
        dzn = tmp;
    }
    // first layer: dW1[h][k] = sum_s dZ1[h][s] x[s][k], db1
    {
        const int h = t >> 2, k = t & 3;
        float s = 0.0f;
        for (int q = 0; q < kTrainTile; ++q) s += dz[h * kLd + q] * sX[q][k];
        g[kOffW1 + h * 4 + k] = s;
        if (k == 0) {
            float b = 0.0f;
            for (int q = 0; q < kTrainTile; ++q) b += dz[h * kLd + q];
            g[kOffB1 + h] = b;
        }
    }
    // loss partial
    for (int st = 128; st >= 1; st >>= 1) {
        if (t < st) sL[t] += sL[t + st];
        __syncthreads();
    }
    if (t == 0) A.lpart[blockIdx.x] = sL[0];
}

// Sum of the per-block partials (fixed order), then either the raw gradient
// (grad != null) or an Adam step on P with moments m, v.
struct MlpStepArgs {
    float* P;
    float* m;
    float* v;
    const float* gpart;
    int nparts;
    float* grad;         // gradient output (no step) or null
    float lr, beta1, beta2, eps, bc1, bc2;   // bc = 1 - beta^step
};

__global__ void mlp_adam(MlpStepArgs S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    float gsum = 0.0f;
    for (int b = 0; b < S.nparts; ++b) gsum += S.gpart[(size_t)b * kMlpParams + i];
    if (S.grad) {
        S.grad[i] = gsum;
        return;
    }
    const float m = S.beta1 * S.m[i] + (1.0f - S.beta1) * gsum;
    const float v = S.beta2 * S.v[i] + (1.0f - S.beta2) * gsum * gsum;
    S.m[i] = m;
    S.v[i] = v;
    S.P[i] -= S.lr * (m / S.bc1) / (sqrtf(v / S.bc2) + S.eps);
}

__global__ void mlp_loss_sum(const double* lpart, int n, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += lpart[k];
        out[0] = s;
    }
}

// Features and standardised targets of a training set: in [n][4] (kappa, w,
// X, cos theta), integrals [n][8]; norm = (mu[8], sd[8]).
__global__ void mlp_prepare(int64_t n, const double* in, const double* integ, const double* norm, float* feat,
                            float* targ) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float* f = feat + k * 4;
    mlp_features(in[k * 4], in[k * 4 + 1], in[k * 4 + 2], in[k * 4 + 3], f);
    double m[kPolyTerms];
    mlp_monomials<double>(f[0], f[1], f[2], m);
    for (int o = 0; o < 8; ++o) {
        double base = 0.0;
        for (int j = 0; j < kPolyTerms; ++j) base += norm[16 + o * kPolyTerms + j] * m[j];
        targ[k * 8 + o] = (float)((log10(integ[k * 8 + o]) - base - norm[o]) / norm[8 + o]);
    }
}

// Sums for the least-squares baseline, per block: M^T M (20 x 20), M^T y
// (20 x 8) and y^T y (8) over the block's samples, y = log10 of the
// integrals, M the monomials of the FP32 features (out: [gridDim.x][628]).
constexpr int kFitLen = kPolyTerms * kPolyTerms + kPolyTerms * 8 + 8;

__global__ __launch_bounds__(256) void mlp_fit_sums(int64_t n, const double* in, const double* integ,
                                                   double* out) {
    __shared__ double sM[256][kPolyTerms + 1];
    __shared__ double sY[256][9];
    const int t = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};   // entries q = t + 256 r of the sums
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t k = base + t;
        if (k < n) {
            float f[4];
            mlp_features(in[k * 4], in[k * 4 + 1], in[k * 4 + 2], in[k * 4 + 3], f);
            double m[kPolyTerms];
            mlp_monomials<double>(f[0], f[1], f[2], m);
            for (int j = 0; j < kPolyTerms; ++j) sM[t][j] = m[j];
            for (int o = 0; o < 8; ++o) sY[t][o] = log10(integ[k * 8 + o]);
        } else {
            for (int j = 0; j < kPolyTerms; ++j) sM[t][j] = 0.0;
            for (int o = 0; o < 8; ++o) sY[t][o] = 0.0;
        }
        __syncthreads();
        for (int r = 0; r < 3; ++r) {
            const int q = t + 256 * r;
            if (q >= kFitLen) break;
            double sum = 0.0;
            if (q < kPolyTerms * kPolyTerms) {
                const int i = q / kPolyTerms, j = q % kPolyTerms;
                for (int s = 0; s < 256; ++s) sum += sM[s][i] * sM[s][j];
            } else if (q < kPolyTerms * kPolyTerms + kPolyTerms * 8) {
                const int i = (q - kPolyTerms * kPolyTerms) / 8, o = (q - kPolyTerms * kPolyTerms) % 8;
                for (int s = 0; s < 256; ++s) sum += sM[s][i] * sY[s][o];
            } else {
                const int o = q - kPolyTerms * kPolyTerms - kPolyTerms * 8;
                for (int s = 0; s < 256; ++s) sum += sY[s][o] * sY[s][o];
            }
            acc[r] += sum;
        }
        __syncthreads();
    }
    for (int r = 0; r < 3; ++r) {
        const int q = t + 256 * r;
        if (q < kFitLen) out[(size_t)blockIdx.x * kFitLen + q] = acc[r];
    }
}

// ---------------------------------------------------------------------------
// Inference on MFMA.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Packed network: A-operand fragments (64 lanes x 8 bfloat16 = 1 KiB each)
// for W1 (2 M tiles x 1 K step), W2 and W3 (2 x 4), W4 (1 x 4, rows >= 8
// zero), then FP32 biases.
constexpr int kFragW1 = 0, kFragW2 = 2, kFragW3 = 10, kFragW4 = 18, kFrags = 22;
struct MlpPacked {
    bf16x8 frag[kFrags][64];
    float b1[64], b2[64], b3[64], b4[8];
    float mu[8], sd[8];
    float poly[8][kPolyTerms];
};
// The packed network as read from LDS.
typedef __attribute__((address_space(3))) const MlpPacked LdsMlp;

// Hidden unit fed to B-operand position (K step ks, lane half hf, element e):
// the unit held by that lane's accumulator of the previous layer, register
// v = 4 i + (e & 3) of M tile mt, with 4 mt + i = 2 ks + (e >> 2).
KRT_HD int mlp_kunit(int ks, int hf, int e) {
    const int idx = 2 * ks + (e >> 2);
    return 32 * (idx >> 2) + 8 * (idx & 3) + 4 * hf + (e & 3);
}

__global__ void mlp_pack(const float* P, const double* norm, MlpPacked* out) {
    const int t = threadIdx.x;   // one block of 64 x 4 threads
    const int lane = t & 63;
    for (int f = t >> 6; f < kFrags; f += 4) {
        bf16x8 v;
        for (int e = 0; e < 8; ++e) {
            float w = 0.0f;
            const int hf = lane >> 5, r = lane & 31;
            if (f < kFragW2) {
                const int row = 32 * f + r, k = 8 * hf + e;
                w = k < 4 ? P[kOffW1 + row * 4 + k] : 0.0f;
            } else if (f < kFragW4) {
                const int L = f < kFragW3 ? 0 : 1;
                const int fi = f - (L ? kFragW3 : kFragW2);
                const int mt = fi / 4, ks = fi % 4;
                w = P[(L ? kOffW3 : kOffW2) + (32 * mt + r) * kMlpH + mlp_kunit(ks, hf, e)];
            } else {
                const int ks = f - kFragW4;
                w = r < kMlpOut ? P[kOffW4 + r * kMlpH + mlp_kunit(ks, hf, e)] : 0.0f;
            }
            v[e] = (__bf16)bf16_round(w);
        }
        out->frag[f][lane] = v;
    }
    for (int k = t; k < 64; k += 256) {
        out->b1[k] = P[kOffB1 + k];
        out->b2[k] = P[kOffB2 + k];
        out->b3[k] = P[kOffB3 + k];
    }
    if (t < 8) {
        out->b4[t] = P[kOffB4 + t];
        out->mu[t] = (float)norm[t];
        out->sd[t] = (float)norm[8 + t];
    }
    for (int k = t; k < 8 * kPolyTerms; k += 256) out->poly[k / kPolyTerms][k % kPolyTerms] = (float)norm[16 + k];
}

__device__ __forceinline__ float silu_fast(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// hi + lo bfloat16 split of 8 floats, two at a time: hi = x rounded to the
// nearest bfloat16 (ties to even: one hardware conversion per pair), lo = the
// remainder x - hi (exact in FP32) rounded the same way.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split8(const float x[8], bf16x8& hi, bf16x8& lo) {
    for (int q = 0; q < 4; ++q) {
        const f32x2 v = {x[2 * q], x[2 * q + 1]};
        const bf16x2 h = __builtin_convertvector(v, bf16x2);
        const uint32_t u = __builtin_bit_cast(uint32_t, h);
        const f32x2 r = {v.x - __builtin_bit_cast(float, u << 16), v.y - __builtin_bit_cast(float, u & 0xFFFF0000u)};
        const bf16x2 l = __builtin_convertvector(r, bf16x2);
        hi[2 * q] = h.x;
        hi[2 * q + 1] = h.y;
        lo[2 * q] = l.x;
        lo[2 * q + 1] = l.y;
    }
}

// Bias in accumulator layout: register v of M tile mt holds row
// 32 mt + 8 (v / 4) + 4 hf + v % 4.
template <class P>
__device__ __forceinline__ void bias_init(P b, int mt, int hf, f32x16& acc) {
    for (int v = 0; v < 16; ++v) acc[v] = b[32 * mt + 8 * (v >> 2) + 4 * hf + (v & 3)];
}

// One 32-ray tile: x = this lane's feature row for the tile (zeros in the
// upper half-wave); returns in z[0..3] the outputs 4 hf .. 4 hf + 3 of ray
// (lane & 31) of the tile.  Must be called by all 64 lanes together.
__device__ __forceinline__ void mlp_tile(LdsMlp* __restrict__ W, const float x[8], float z[4]) {
    const int lane = threadIdx.x & 63, hf = lane >> 5;
    f32x16 acc[2];
    bf16x8 bh[4], bl[4];
    split8(x, bh[0], bl[0]);
    for (int mt = 0; mt < 2; ++mt) {
        bias_init(W->b1, mt, hf, acc[mt]);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W->frag[kFragW1 + mt][lane], bh[0], acc[mt], 0, 0, 0);
        acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W->frag[kFragW1 + mt][lane], bl[0], acc[mt], 0, 0, 0);
    }
    for (int L = 0; L < 2; ++L) {
        // activations -> B fragments (K order of mlp_kunit)
        for (int ks = 0; ks < 4; ++ks) {
            float a[8];
            for (int e = 0; e < 8; ++e) {
                const int idx = 2 * ks + (e >> 2);
                a[e] = silu_fast(acc[idx >> 2][4 * (idx & 3) + (e & 3)]);
            }
            split8(a, bh[ks], bl[ks]);
        }
        const int fw = L ? kFragW3 : kFragW2;
        const auto b = L ? W->b3 : W->b2;
        for (int mt = 0; mt < 2; ++mt) {
            bias_init(b, mt, hf, acc[mt]);
            for (int ks = 0; ks < 4; ++ks) {
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W->frag[fw + 4 * mt + ks][lane], bh[ks], acc[mt],
                                                                   0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W->frag[fw + 4 * mt + ks][lane], bl[ks], acc[mt],
                                                                   0, 0, 0);
            }
        }
    }
    for (int ks = 0; ks < 4; ++ks) {
        float a[8];
        for (int e = 0; e < 8; ++e) {
            const int idx = 2 * ks + (e >> 2);
            a[e] = silu_fast(acc[idx >> 2][4 * (idx & 3) + (e & 3)]);
        }
        split8(a, bh[ks], bl[ks]);
    }
    f32x16 o;
    for (int v = 0; v < 16; ++v) o[v] = 0.0f;
    for (int v = 0; v < 4; ++v) o[v] = W->b4[4 * hf + v];
    for (int ks = 0; ks < 4; ++ks) {
        o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W->frag[kFragW4 + ks][lane], bh[ks], o, 0, 0, 0);
        o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(W->frag[kFragW4 + ks][lane], bl[ks], o, 0, 0, 0);
    }
    for (int v = 0; v < 4; ++v) z[v] = o[v];
}

// 10^y for an output of the network (y in FP32): 2^e = 2^k 2^(e - k) with
// e = y log2 10 formed in FP64, k = rint(e), 2^(e - k) by the hardware's FP32
// exp2; relative error about 1e-7, as y itself carries.
__device__ __forceinline__ double exp10_out(float y) {
    const double e = (double)y * 3.321928094887362;
    const double k = __builtin_rint(e);
    return __builtin_ldexp((double)__builtin_amdgcn_exp2f((float)(e - k)), (int)k);
}

// The network for the 64 lanes of a wave: W = the packed network staged in
// LDS (its fragments are read through an LDS address), f = this lane's
// features; on return out[8] = the eight integrals of this lane (log10
// destandardised and exponentiated).  Must be called by all 64 lanes together.
__device__ __forceinline__ void mlp_wave(const MlpPacked* __restrict__ W, const float f[4], double out[8]) {
    const int lane = threadIdx.x & 63, hf = lane >> 5;
    float zt[2][4];
    for (int nt = 0; nt < 2; ++nt) {
        // B rows 0..3 of ray (lane & 31) + 32 nt live in the lower half-wave
        float x[8];
        for (int k = 0; k < 4; ++k) {
            const float mine = f[k];
            const float other = __shfl_xor(mine, 32);
            const float v = (nt == 0) ? mine : other;
            x[k] = hf == 0 ? v : 0.0f;
        }
        for (int k = 4; k < 8; ++k) x[k] = 0.0f;
        // the weights are read again for each tile: an address the compiler
        // cannot see through keeps it from holding all 22 fragments (88
        // registers) from the first tile into the second
        LdsMlp* Wt = (LdsMlp*)W;
        asm volatile("" : "+v"(Wt));
        mlp_tile(Wt, x, zt[nt]);
    }
    // ray R = lane sits in tile hf at column lane & 31: this lane holds its
    // outputs 4 hf .. 4 hf + 3, the partner lane (lane ^ 32) the other four,
    // in the partner's accumulators of tile hf (= 1 - the partner's half)
    float z[8];
    for (int v = 0; v < 4; ++v) {
        const float own = zt[hf][v];
        const float partner = __shfl_xor(zt[1 - hf][v], 32);
        z[4 * hf + v] = own;
        z[4 * (1 - hf) + v] = partner;
    }
    float m[kPolyTerms];
    mlp_monomials<float>(f[0], f[1], f[2], m);
    for (int o = 0; o < 8; ++o) {
        float base = 0.0f;
        for (int j = 0; j < kPolyTerms; ++j) base += W->poly[o][j] * m[j];
        out[o] = exp10_out(base + W->mu[o] + W->sd[o] * z[o]);
    }
}

// Test hook / batch evaluation: in [n][4] (kappa, w, X, cos theta) -> out [n][8].
__global__ __launch_bounds__(256) void hook_mlp_eval(const MlpPacked* __restrict__ Wg, int64_t n, const double* in,
                                                    double* out) {
    __shared__ MlpPacked W;
    {
        const int4* src = reinterpret_cast<const int4*>(Wg);
        int4* dst = reinterpret_cast<int4*>(&W);
        for (int k = threadIdx.x; k < (int)(sizeof(MlpPacked) / 16); k += blockDim.x) dst[k] = src[k];
    }
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (k < n) mlp_features(in[k * 4], in[k * 4 + 1], in[k * 4 + 2], in[k * 4 + 3], f);
    double o[8];
    mlp_wave(&W, f, o);
    if (k < n)
        for (int q = 0; q < 8; ++q) out[k * 8 + q] = o[q];
}

}  // namespace krt
