// Learned codec selector: an 8 -> 64 -> 64 -> 35 ReLU network over the
// per-block features, trained on the GPU with softmax cross-entropy against
// the exhaustive choice and Adam.  (The paper picks one codec offline from
// measured tables, experimental-performance section; a per-block learned
// choice is this project's extension.)
//
// Rounding points (same as the CPU oracle): weights rounded to fp16 from the
// fp32 master copy; fp16 inputs; h = fp16(relu(W x + b)) with fp32
// accumulation and fp32 bias; fp32 logits.  The backward pass is fp32 and
// straight-through at the roundings.
//
// One workgroup of 256 threads handles 64 samples; per-workgroup gradient
// partials are reduced by a second kernel in a fixed order (deterministic).
#include "common.hpp"
#include "mlp_mfma.hpp"

namespace bfsc {

constexpr int kChunk = 64;
constexpr int kThreads = 256;

struct MlpArgs {
    const uint16_t *X;
    const uint8_t *y;     // NULL: forward only
    uint32_t n;
    const float *params;
    const _Float16 *w16;
    float *logits;        // forward only: [n][35]
    float *partial;       // [nchunks][kNParams]
    float *partial_loss;  // [nchunks]
};

__device__ __forceinline__ float h16(float x) { return (float)(_Float16)x; }

__global__ __launch_bounds__(kThreads) void k_mlp(MlpArgs a) {
    __shared__ float sx[kChunk][kIn];
    __shared__ float sz1[kChunk][kH + 1];
    __shared__ float sh1[kChunk][kH + 1];
    __shared__ float sz2[kChunk][kH + 1];
    __shared__ float sh2[kChunk][kH + 1];
    __shared__ float sg3[kChunk][kOut + 1];
    __shared__ float s_loss[kChunk];
    const uint32_t tid = threadIdx.x;
    const uint32_t c = blockIdx.x;
    const uint32_t s0 = c * kChunk;
    const uint32_t ns = min((uint32_t)kChunk, a.n - s0);
    const bool train = a.y != nullptr;
    const float invN = 1.0f / (float)a.n;

    for (uint32_t o = tid; o < kChunk * kIn; o += kThreads) {
        const uint32_t s = o / kIn, i = o % kIn;
        sx[s][i] = s < ns ? (float)__builtin_bit_cast(_Float16, a.X[(uint64_t)(s0 + s) * kIn + i]) : 0.0f;
    }
    __syncthreads();
    for (uint32_t o = tid; o < kChunk * kH; o += kThreads) {
        const uint32_t s = o / kH, u = o % kH;
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < kIn; ++i) acc += (float)a.w16[kW1 + u * kIn + i] * sx[s][i];
        const float z = acc + a.params[kB1 + u];
        sz1[s][u] = z;
        sh1[s][u] = h16(fmaxf(z, 0.0f));
    }
    __syncthreads();
    for (uint32_t o = tid; o < kChunk * kH; o += kThreads) {
        const uint32_t s = o / kH, u = o % kH;
        float acc = 0.0f;
        for (int i = 0; i < kH; ++i) acc += (float)a.w16[kW2 + u * kH + i] * sh1[s][i];
        const float z = acc + a.params[kB2 + u];
        sz2[s][u] = z;
        sh2[s][u] = h16(fmaxf(z, 0.0f));
    }
    __syncthreads();
    for (uint32_t o = tid; o < kChunk * kOut; o += kThreads) {
        const uint32_t s = o / kOut, k = o % kOut;
        float acc = 0.0f;
        for (int i = 0; i < kH; ++i) acc += (float)a.w16[kW3 + k * kH + i] * sh2[s][i];
        const float z = acc + a.params[kB3 + k];
        sg3[s][k] = z;
        if (!train && s < ns) a.logits[(uint64_t)(s0 + s) * kOut + k] = z;
    }
    if (!train) return;
    __syncthreads();
    // softmax cross-entropy: g3 = (p - onehot) / N
    if (tid < kChunk) {
        const uint32_t s = tid;
        float loss = 0.0f;
        if (s < ns) {
            float mx = sg3[s][0];
            for (int k = 1; k < kOut; ++k) mx = fmaxf(mx, sg3[s][k]);
            float sum = 0.0f;
            for (int k = 0; k < kOut; ++k) sum += expf(sg3[s][k] - mx);
            const uint32_t ys = a.y[s0 + s];
            loss = -(sg3[s][ys] - mx - logf(sum)) * invN;
            for (int k = 0; k < kOut; ++k) {
                const float p = expf(sg3[s][k] - mx) / sum;
                sg3[s][k] = (p - (k == (int)ys ? 1.0f : 0.0f)) * invN;
            }
        } else {
            for (int k = 0; k < kOut; ++k) sg3[s][k] = 0.0f;
        }
        s_loss[s] = loss;
    }
    __syncthreads();
    float *part = a.partial + (uint64_t)c * kNParams;
    // dW3, db3
    for (uint32_t o = tid; o < kOut * kH + kOut; o += kThreads) {
        float acc = 0.0f;
        if (o < kOut * kH) {
            const uint32_t k = o / kH, i = o % kH;
            for (int s = 0; s < kChunk; ++s) acc += sg3[s][k] * sh2[s][i];
            part[kW3 + o] = acc;
        } else {
            const uint32_t k = o - kOut * kH;
            for (int s = 0; s < kChunk; ++s) acc += sg3[s][k];
            part[kB3 + k] = acc;
        }
    }
    // d2 = (g3 W3h) * [z2 > 0], in place of z2
    for (uint32_t o = tid; o < kChunk * kH; o += kThreads) {
        const uint32_t s = o / kH, i = o % kH;
        float acc = 0.0f;
        for (int k = 0; k < kOut; ++k) acc += sg3[s][k] * (float)a.w16[kW3 + k * kH + i];
        sz2[s][i] = sz2[s][i] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // dW2, db2
    for (uint32_t o = tid; o < kH * kH + kH; o += kThreads) {
        float acc = 0.0f;
        if (o < kH * kH) {
            const uint32_t u = o / kH, i = o % kH;
            for (int s = 0; s < kChunk; ++s) acc += sz2[s][u] * sh1[s][i];
            part[kW2 + o] = acc;
        } else {
            const uint32_t u = o - kH * kH;
            for (int s = 0; s < kChunk; ++s) acc += sz2[s][u];
            part[kB2 + u] = acc;
        }
    }
    // d1 = (d2 W2h) * [z1 > 0], in place of z1
    for (uint32_t o = tid; o < kChunk * kH; o += kThreads) {
        const uint32_t s = o / kH, i = o % kH;
        float acc = 0.0f;
        for (int u = 0; u < kH; ++u) acc += sz2[s][u] * (float)a.w16[kW2 + u * kH + i];
        sz1[s][i] = sz1[s][i] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    for (uint32_t o = tid; o < kH * kIn + kH; o += kThreads) {
        float acc = 0.0f;
        if (o < kH * kIn) {
            const uint32_t u = o / kIn, i = o % kIn;
            for (int s = 0; s < kChunk; ++s) acc += sz1[s][u] * sx[s][i];
            part[kW1 + o] = acc;
        } else {
            const uint32_t u = o - kH * kIn;
            for (int s = 0; s < kChunk; ++s) acc += sz1[s][u];
            part[kB1 + u] = acc;
        }
    }
    if (tid == 0) {
        float l = 0.0f;
        for (int s = 0; s < kChunk; ++s) l += s_loss[s];
        a.partial_loss[c] = l;
    }
}

// Fixed-order reduction of the per-workgroup partials.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float *partial, const float *partial_loss,
                                                    uint32_t nchunks, float *grads, float *loss) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint32_t)kNParams) {
        float acc = 0.0f;
        for (uint32_t c = 0; c < nchunks; ++c) acc += partial[(uint64_t)c * kNParams + i];
        grads[i] = acc;
    }
    if (i == 0 && loss) {
        float l = 0.0f;
        for (uint32_t c = 0; c < nchunks; ++c) l += partial_loss[c];
        *loss = l;
    }
}

__global__ __launch_bounds__(256) void k_adam(float *params, float *m, float *v, _Float16 *w16,
                                              const float *grads, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)kNParams) return;
    const float g = grads[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float p = params[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    params[i] = p;
    w16[i] = (_Float16)p;
}

__global__ __launch_bounds__(256) void k_round16(const float *params, _Float16 *w16) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint32_t)kNParams) w16[i] = (_Float16)params[i];
}

size_t mlp_ws_bytes(uint32_t n) {
    const size_t nch = (n + kChunk - 1) / kChunk;
    return align256(nch * kNParams * 4) + align256(nch * 4) + 256;
}

static void mlp_ws(void *ws, uint32_t n, float **partial, float **ploss) {
    const size_t nch = (n + kChunk - 1) / kChunk;
    char *b = (char *)ws;
    *partial = (float *)b;
    *ploss = (float *)(b + align256(nch * kNParams * 4));
}

// The fp16 weights in MFMA A-operand lane order, and the fp32 biases (one
// thread per tile lane).  Tile (t, s) of a layer with M outputs and K inputs
// holds, in lane l, W[16t + l mod 16][16s + 4(l/16) + j] for j = 0..3, zero
// outside the matrix.
__global__ void k_mlp_pack_mfma(const _Float16 *w16, const float *params, MlpMfma *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMfmaTiles * 64) {
        const uint32_t tile = i / 64, lane = i % 64;
        uint32_t t, sk, M, K, base;
        if (tile < kMfmaT2) {
            t = tile, sk = 0, M = kH, K = kIn, base = kW1;
        } else if (tile < kMfmaT3) {
            t = (tile - kMfmaT2) / 4, sk = (tile - kMfmaT2) % 4, M = kH, K = kH, base = kW2;
        } else {
            t = (tile - kMfmaT3) / 4, sk = (tile - kMfmaT3) % 4, M = kOut, K = kH, base = kW3;
        }
        const uint32_t m = 16 * t + lane % 16;
        half4_t v;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t k = 16 * sk + 4 * (lane / 16) + j;
            v[j] = (m < M && k < K) ? w16[base + m * K + k] : (_Float16)0.0f;
        }
        out->w[tile][lane] = v;
    }
    if (i < kMfmaBias) {
        float b = 0.0f;
        if (i < 64) b = params[kB1 + i];
        else if (i < 128) b = params[kB2 + i - 64];
        else if (i - 128 < (uint32_t)kOut) b = params[kB3 + i - 128];
        out->b[i] = b;
    }
}

static int launch_mlp_pack(bfsc_ctx *ctx, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack_mfma, dim3((kMfmaTiles * 64 + 255) / 256), dim3(256), 0, s,
                       ctx->mlp_w16, ctx->mlp_params, (MlpMfma *)ctx->mlp_mfma);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_round16(bfsc_ctx *ctx, hipStream_t s) {
    hipLaunchKernelGGL(k_round16, dim3((kNParams + 255) / 256), dim3(256), 0, s, ctx->mlp_params,
                       ctx->mlp_w16);
    if (hipGetLastError() != hipSuccess) return BFSC_E_HIP;
    return launch_mlp_pack(ctx, s);
}

// Inference on the matrix cores: every wave takes 16 samples at a time.
__global__ __launch_bounds__(256) void k_mlp_infer(const MlpMfma *Wg, const uint16_t *X, uint32_t n,
                                                   float *logits, uint8_t *cls) {
    __shared__ MlpMfma W;
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    mlp_mfma_stage(&W, Wg, tid, 256);
    __syncthreads();
    const uint32_t groups = (n + 15) / 16;
    for (uint32_t g = blockIdx.x * 4 + w; g < groups; g += gridDim.x * 4) {
        const uint32_t smp = g * 16 + (lane & 15);
        half4_t x = {(_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f, (_Float16)0.0f};
        if (lane < 32 && smp < n) x = *(const half4_t *)(X + (uint64_t)smp * kIn + (lane >> 4) * 4);
        float4_t z[3];
        mlp16(W, x, lane, z);
        if (logits && smp < n) {
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t c = 16u * t + (lane >> 4) * 4 + j;
                    if (c < (uint32_t)kOut) logits[(uint64_t)smp * kOut + c] = z[t][j];
                }
        }
        const uint32_t best = mlp16_argmax(z, lane);
        if (cls && lane < 16 && smp < n) cls[smp] = (uint8_t)best;
    }
}

int launch_mlp_infer(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, uint8_t *cls,
                     hipStream_t s) {
    if (n == 0) return BFSC_OK;
    uint64_t groups = (n + 15) / 16, grid = (groups + 3) / 4;
    if (grid > (uint64_t)ctx->n_cu * 8) grid = (uint64_t)ctx->n_cu * 8;
    hipLaunchKernelGGL(k_mlp_infer, dim3((uint32_t)grid), dim3(256), 0, s,
                       (const MlpMfma *)ctx->mlp_mfma, X, n, logits, cls);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_mlp_forward(bfsc_ctx *ctx, const uint16_t *X, uint32_t n, float *logits, hipStream_t s) {
    if (n == 0) return BFSC_OK;
    MlpArgs a;
    a.X = X;
    a.y = nullptr;
    a.n = n;
    a.params = ctx->mlp_params;
    a.w16 = ctx->mlp_w16;
    a.logits = logits;
    a.partial = nullptr;
    a.partial_loss = nullptr;
    const uint32_t nch = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_mlp, dim3(nch), dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_mlp_grad(bfsc_ctx *ctx, const uint16_t *X, const uint8_t *y, uint32_t n, float *grads,
                    float *loss, void *ws, hipStream_t s) {
    if (n == 0) return BFSC_E_INVAL;
    MlpArgs a;
    a.X = X;
    a.y = y;
    a.n = n;
    a.params = ctx->mlp_params;
    a.w16 = ctx->mlp_w16;
    a.logits = nullptr;
    mlp_ws(ws, n, &a.partial, &a.partial_loss);
    const uint32_t nch = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_mlp, dim3(nch), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParams + 255) / 256), dim3(256), 0, s, a.partial,
                       a.partial_loss, nch, grads, loss);
    return hipGetLastError() == hipSuccess ? BFSC_OK : BFSC_E_HIP;
}

int launch_adam(bfsc_ctx *ctx, const float *grads, const bfsc_adam *opt, hipStream_t s) {
    ctx->adam_t += 1;
    const double t = (double)ctx->adam_t;
    const float c1 = (float)(1.0 / (1.0 - pow((double)opt->beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)opt->beta2, t)));
    hipLaunchKernelGGL(k_adam, dim3((kNParams + 255) / 256), dim3(256), 0, s, ctx->mlp_params,
                       ctx->adam_m, ctx->adam_v, ctx->mlp_w16, grads, opt->lr, opt->beta1,
                       opt->beta2, opt->eps, c1, c2);
    if (hipGetLastError() != hipSuccess) return BFSC_E_HIP;
    return launch_mlp_pack(ctx, s);
}

}  // namespace bfsc
