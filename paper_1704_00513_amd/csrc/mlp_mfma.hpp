// Inference of the 8-64-64-35 codec selector on the matrix cores.
//
// The network is the only dense contraction of the path.  The layers are
// evaluated transposed, Z^T = W3 relu(W2 relu(W1 X^T)), with
// v_mfma_f32_16x16x16_f16 (fp16 operands, fp32 accumulation) on 16 samples at
// a time: M = output units, K = input units, N = 16 samples.  With that
// orientation a layer's result tile (lane l: rows 4(l/16)+j, column l mod 16)
// is already laid out as the next layer's B operand (lane l: k = 4(l/16)+j,
// n = l mod 16), so activations never leave registers.  The weights are
// stored once, fp16 and in the A-operand lane order, so every MFMA reads its
// operand with one 8-byte load per lane.
//
// Rounding points follow the selector's definition: fp16 weights (RNE of the
// fp32 master), fp16 features, fp32 accumulation plus fp32 bias, ReLU, RNE to
// fp16 for the hidden activations, fp32 logits.  Only the order of the fp32
// additions inside a dot product differs from a sequential sum.
#pragma once

#include "common.hpp"

namespace bfsc {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// A-operand tiles: layer 1 (4 tiles of 16 units x 16 features, features 8..15
// zero), layer 2 (4 x 4 tiles), layer 3 (3 x 4 tiles, classes 35..47 zero).
constexpr uint32_t kMfmaT1 = 0, kMfmaT2 = 4, kMfmaT3 = 20, kMfmaTiles = 32;
constexpr uint32_t kMfmaBias = 64 + 64 + 48;  // b1 | b2 | b3 (zero past class 34)

struct MlpMfma {
    half4_t w[kMfmaTiles][64];
    float b[kMfmaBias];
};
static_assert(sizeof(MlpMfma) % 16 == 0, "staged with 16-byte copies");

// Copies the operand tiles into LDS (the whole workgroup; a barrier follows).
__device__ __forceinline__ void mlp_mfma_stage(MlpMfma *dst, const MlpMfma *src, uint32_t tid,
                                               uint32_t nthr) {
    const uint4 *s = (const uint4 *)src;
    uint4 *d = (uint4 *)dst;
    for (uint32_t i = tid; i < sizeof(MlpMfma) / 16; i += nthr) d[i] = s[i];
}

__device__ __forceinline__ half4_t relu_f16(float4_t c) {
    half4_t h;
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = (_Float16)fmaxf(c[j], 0.0f);
    return h;
}

// Logits of the 16 samples whose features the wave holds in x (lane l:
// features 4(l/16) .. 4(l/16)+3 of sample l mod 16, zero on lanes 32..63).
// Lane l receives in z[t][j] the logit of class 16t + 4(l/16) + j of sample
// l mod 16.
__device__ __forceinline__ void mlp16(const MlpMfma &W, half4_t x, uint32_t lane, float4_t z[3]) {
    const uint32_t q4 = (lane >> 4) * 4;
    half4_t h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float4_t c = *(const float4_t *)&W.b[16 * t + q4];
        c = __builtin_amdgcn_mfma_f32_16x16x16f16(W.w[kMfmaT1 + t][lane], x, c, 0, 0, 0);
        h1[t] = relu_f16(c);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float4_t c = *(const float4_t *)&W.b[64 + 16 * t + q4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            c = __builtin_amdgcn_mfma_f32_16x16x16f16(W.w[kMfmaT2 + 4 * t + s][lane], h1[s], c, 0, 0, 0);
        h2[t] = relu_f16(c);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        float4_t c = *(const float4_t *)&W.b[128 + 16 * t + q4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            c = __builtin_amdgcn_mfma_f32_16x16x16f16(W.w[kMfmaT3 + 4 * t + s][lane], h2[s], c, 0, 0, 0);
        z[t] = c;
    }
}

// Predicted class of sample lane mod 16: the largest logit, the lowest class
// on ties, 255 when any of its logits is NaN.  All four lanes of a sample
// return the same value.  A lane visits its classes in increasing order, so
// inside the lane a later class wins only by a strictly larger logit; the
// first one (class 4(l/16) < 35) starts the scan, so a lane whose logits
// are all -inf still names its lowest class.  Written without branches:
// short-circuit tests would put exec-mask handling around every logit.
__device__ __forceinline__ uint32_t mlp16_argmax(const float4_t z[3], uint32_t lane) {
    const uint32_t q4 = (lane >> 4) * 4;
    float best = z[0][0];
    uint32_t bi = q4;
    bool nan = best != best;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
#pragma unroll
        for (int j = (t == 0 ? 1 : 0); j < 4; ++j) {
            const uint32_t c = 16u * t + q4 + j;
            const float v = z[t][j];
            const bool valid = c < (uint32_t)kOut;
            nan |= valid & (v != v);
            const bool take = valid & (v > best);
            best = take ? v : best;
            bi = take ? c : bi;
        }
    }
#pragma unroll
    for (int d = 16; d <= 32; d <<= 1) {
        const float ob = __builtin_bit_cast(float, shfl_xor(__builtin_bit_cast(uint32_t, best), d));
        const uint32_t oi = shfl_xor(bi, d);
        nan |= shfl_xor((uint32_t)nan, d) != 0u;
        const bool take = (ob > best) | ((ob == best) & (oi < bi));
        best = take ? ob : best;
        bi = take ? oi : bi;
    }
    return nan ? 255u : bi;
}

}  // namespace bfsc
