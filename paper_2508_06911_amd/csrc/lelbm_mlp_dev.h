// Device-side pieces of the warm-start network shared by the training
// kernels and the per-step inference/harvesting: BF16 conversion, the MFMA
// wrapper, weight fragments, the wavefront forward pass, and the scaling of
// features and targets.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "lelbm_internal.h"

namespace lelbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                        // round to nearest even
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = (short)f2bf(a); r[1] = (short)f2bf(b); r[2] = (short)f2bf(c); r[3] = (short)f2bf(d);
    return r;
}
__device__ inline bf16x4 pack4(const f32x4 &v) { return pack4(v[0], v[1], v[2], v[3]); }

__device__ inline f32x4 mfma(const bf16x4 &a, const bf16x4 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Two K-tiles of 16 in one gfx950 16x16x32 BF16 MFMA: lane group g holds
// the four k of tile 0 and the four k of tile 1 that it holds in the
// 16x16x16 form, in both operands, so every product pairs the same k and
// the sum runs over all 32.
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ inline f32x4 mfma2(const bf16x4 &a0, const bf16x4 &a1, const bf16x4 &b0, const bf16x4 &b1,
                              const f32x4 &c) {
    const bf16x8s a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const bf16x8s b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// A fragment of W^T (tile mt of outputs, kt of inputs) from a row-major
// [nin][nout] BF16 weight matrix: lane l holds W[16kt+4(l/16)+i][16mt+l%16].
__device__ inline bf16x4 frag_wT(const unsigned short *W, int nout, int mt, int kt, int lane) {
    const int k0 = 16 * kt + 4 * (lane >> 4), m = 16 * mt + (lane & 15);
    bf16x4 r;
#pragma unroll
    for (int i = 0; i < 4; i++) r[i] = (short)W[(k0 + i) * nout + m];
    return r;
}
// A fragment of W (tile mt of inputs, kt of outputs): lane l holds
// W[16mt+l%16][16kt+4(l/16)+i] (four consecutive entries of one row).
__device__ inline bf16x4 frag_w(const unsigned short *W, int nout, int mt, int kt, int lane) {
    const int m = 16 * mt + (lane & 15), k0 = 16 * kt + 4 * (lane >> 4);
    bf16x4 r;
#pragma unroll
    for (int i = 0; i < 4; i++) r[i] = (short)W[m * nout + k0 + i];
    return r;
}

// Forward pass of one wavefront.  xs: LDS [64][16] BF16 inputs (sample-major).
// Outputs the BF16 hidden activations (B-operand layout, kept for the
// backward pass) and the FP32 outputs y[nt] (lane: outputs 4(l/16)..+3 of
// sample 16nt+l%16).
// xrow(r) points to the MLP_IN BF16 inputs of sample r.
template <class XRow>
__device__ inline void mlp_forward_wave_rows(const unsigned short *Wb, const float *bias, XRow xrow,
                                             bf16x4 (&h1)[4][4], bf16x4 (&h2)[4][4], f32x4 (&y)[4], int lane) {
    const unsigned short *W1 = Wb + MLP_OFF_W1, *W2 = Wb + MLP_OFF_W2, *W3 = Wb + MLP_OFF_W3;
    const float *b1 = bias + MLP_OFF_B1, *b2 = bias + MLP_OFF_B2, *b3 = bias + MLP_OFF_B3;
    const int r4 = 4 * (lane >> 4);
    bf16x4 xb[4];
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        const unsigned short *p = xrow(16 * nt + (lane & 15)) + r4;
#pragma unroll
        for (int i = 0; i < 4; i++) xb[nt][i] = (short)p[i];
    }
    // layer 1: 16 -> 64
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        bf16x4 a = frag_wT(W1, MLP_H, mt, 0, lane);
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            f32x4 d = mfma(a, xb[nt], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int i = 0; i < 4; i++) d[i] = fmaxf(d[i] + b1[16 * mt + r4 + i], 0.f);
            h1[mt][nt] = pack4(d);
        }
    }
    // layer 2: 64 -> 64
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        f32x4 d[4];
#pragma unroll
        for (int nt = 0; nt < 4; nt++) d[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt += 2) {
            const bf16x4 a0 = frag_wT(W2, MLP_H, mt, kt, lane), a1 = frag_wT(W2, MLP_H, mt, kt + 1, lane);
#pragma unroll
            for (int nt = 0; nt < 4; nt++) d[nt] = mfma2(a0, a1, h1[kt][nt], h1[kt + 1][nt], d[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
#pragma unroll
            for (int i = 0; i < 4; i++) d[nt][i] = fmaxf(d[nt][i] + b2[16 * mt + r4 + i], 0.f);
            h2[mt][nt] = pack4(d[nt]);
        }
    }
    // layer 3: 64 -> 16 (linear)
#pragma unroll
    for (int nt = 0; nt < 4; nt++) y[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; kt += 2) {
        const bf16x4 a0 = frag_wT(W3, MLP_OUT, 0, kt, lane), a1 = frag_wT(W3, MLP_OUT, 0, kt + 1, lane);
#pragma unroll
        for (int nt = 0; nt < 4; nt++) y[nt] = mfma2(a0, a1, h2[kt][nt], h2[kt + 1][nt], y[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) y[nt][i] += b3[r4 + i];
}

// Inputs of the 64 samples contiguous in xs ([64][MLP_IN]).
__device__ inline void mlp_forward_wave(const unsigned short *Wb, const float *bias, const unsigned short *xs,
                                        bf16x4 (&h1)[4][4], bf16x4 (&h2)[4][4], f32x4 (&y)[4], int lane) {
    mlp_forward_wave_rows(Wb, bias, [&](int r) { return xs + r * MLP_IN; }, h1, h2, y, lane);
}

// Standardisation constants of the network (64 floats): input means and
// inverse standard deviations, output means and standard deviations.  The
// network itself sees standardised inputs and predicts standardised outputs.
__device__ inline float norm_in(const float *nm, int k, float x) { return (x - nm[k]) * nm[16 + k]; }
__device__ inline float denorm_out(const float *nm, int k, float y) { return nm[32 + k] + nm[48 + k] * y; }

// Features of one 2D cell (16): normalised post-collision targets (second
// and third fluon moments, phonon zeroth and first), offset of the bulk
// velocity from its nearest lattice point, and the stencil resolution.
__device__ inline void mlp_features(const double *mf, const double *mg, double ux, double uy, double RT, int R,
                                    float *x) {
    const double sq = sqrt(RT), is = 1.0 / sq, i3 = is * is * is;
    x[0] = (float)(mf[3] / RT - 1.0);
    x[1] = (float)(mf[4] / RT);
    x[2] = (float)(mf[5] / RT - 1.0);
    x[3] = (float)(mf[6] * i3);
    x[4] = (float)(mf[7] * i3);
    x[5] = (float)(mf[8] * i3);
    x[6] = (float)(mf[9] * i3);
    x[7] = (float)(mg[0] - 1.0);
    x[8] = (float)(mg[1] * is);
    x[9] = (float)(mg[2] * is);
    x[10] = (float)(ux - floor(ux + 0.5));
    x[11] = (float)(uy - floor(uy + 0.5));
    x[12] = (float)is;
    x[13] = (float)((R + 0.5) * is * 0.25 - 1.0);
    x[14] = (float)(0.25 * log(RT));
    x[15] = 0.f;
}

// Scaled multipliers relative to Eq. (IID13): out_j = lambda_j RT^(k_j/2)
// minus the IID13 value, fluon j = 0..9 then phonon j = 0..5.
__device__ inline double iid13_scaled(int j, double RT) {
    if (j == 0) return -1.0 + log(2.0 * M_PI * RT);
    if (j == 3 || j == 5) return 0.5;
    return 0.0;
}
__device__ inline int basis_order2(int j) { return j == 0 ? 0 : (j < 3 ? 1 : (j < 6 ? 2 : 3)); }

}  // namespace lelbm
