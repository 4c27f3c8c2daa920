// Warm-start network of the entropic reconstruction: a 16-64-64-16 ReLU MLP
// that maps normalised post-collision moments and stencil geometry of a cell
// to its Lagrange multipliers (relative to the guess of Eq. IID13, in units
// scaled by RT^(k/2)).  Forward, backward and Adam kernels are hand-written
// for gfx950 with BF16 MFMA (v_mfma_f32_16x16x16_bf16) and FP32 accumulation.
//
// Every layer is computed in transposed form, H_out^T = W^T H_in^T: the
// weights are the A operand and the activations the B operand, so the MFMA
// result layout of one layer (lane l holds rows 4*(l/16)..+3 of column l%16)
// is exactly the B-operand layout of the next layer.  One wavefront handles
// 64 samples (four 16-sample column tiles).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lelbm_internal.h"
#include "lelbm_mlp_dev.h"

namespace lelbm {

// Stores a B-layout tile set (rows = features, cols = samples) transposed
// into LDS as [feature][64 samples] BF16.
template <int NT_ROWS>
__device__ inline void store_fs(unsigned short *dst, const bf16x4 (&v)[NT_ROWS][4], int lane) {
    const int r4 = 4 * (lane >> 4), c = lane & 15;
#pragma unroll
    for (int mt = 0; mt < NT_ROWS; mt++)
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) dst[(16 * mt + r4 + i) * 64 + 16 * nt + c] = (unsigned short)v[mt][nt][i];
}

// Weight gradient G[nin][nout] = sum_s A^T[in][s] B^T[out][s] over the 64
// samples of the wave, from LDS [in][64] and [out][64] BF16 arrays; added to
// g (FP32, row-major [nin][nout]).
template <int MT, int NTO>
__device__ inline void weight_grad(const unsigned short *aT, const unsigned short *bT, float *g, int nout,
                                   int lane) {
    const int r4 = 4 * (lane >> 4), c = lane & 15;
#pragma unroll
    for (int mt = 0; mt < MT; mt++) {
#pragma unroll
        for (int nt = 0; nt < NTO; nt++) {
            f32x4 d = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 4; kt += 2) {
                bf16x4 a[2], b[2];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const unsigned short *pa = aT + (16 * mt + c) * 64 + 16 * (kt + h) + r4;
                    const unsigned short *pb = bT + (16 * nt + c) * 64 + 16 * (kt + h) + r4;
#pragma unroll
                    for (int i = 0; i < 4; i++) { a[h][i] = (short)pa[i]; b[h][i] = (short)pb[i]; }
                }
                d = mfma2(a[0], a[1], b[0], b[1], d);
            }
            // d: rows = in 16mt + r4 + i, col = out 16nt + c
#pragma unroll
            for (int i = 0; i < 4; i++) g[(16 * mt + r4 + i) * nout + 16 * nt + c] = d[i];
        }
    }
}

// Sum over the 16 lanes of a row group (the 16 samples of a column tile).
__device__ inline float sum16(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// Counter-based sample index (SplitMix64 finaliser of seed, step and slot).
__device__ inline unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Forward + backward of one 64-sample wavefront per workgroup.  pairs: n x 32
// FP32 (16 inputs, 16 targets).  Samples are drawn with replacement by the
// counter-based generator (seed, step); with draw == 0 the wave takes the
// consecutive samples 64*blockIdx.x.. (gradient checks).  Writes the wave's
// gradient (loss = mean over samples and outputs of the squared error) to
// partial[blockIdx.x][MLP_NPARAM] and its loss sum to lossp[blockIdx.x].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_mlp_fwdbwd(const unsigned short *Wb, const float *bias, const float *nm,
                                                   const float *pairs, long long n, long long nsamp, int draw,
                                                   unsigned long long seed, unsigned long long step, float *partial,
                                                   float *lossp) {
    __shared__ unsigned short xs[64 * MLP_IN];       // [sample][in]
    __shared__ float ts[64 * MLP_OUT];               // [sample][out]
    __shared__ unsigned short bufA[64 * 64], bufB[64 * 64];
    const int lane = threadIdx.x;
    const int r4 = 4 * (lane >> 4), c = lane & 15;
    long long idx;
    if (draw) idx = (long long)(mix64(seed ^ mix64(step * 1048583ull + blockIdx.x * 64ull + lane)) % (unsigned long long)n);
    else idx = (long long)blockIdx.x * 64 + lane;
    const bool valid = idx < n && ((long long)blockIdx.x * 64 + lane) < nsamp;
    const float *pr = pairs + (valid ? idx : 0) * 32;
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) xs[lane * MLP_IN + k] = valid ? f2bf(norm_in(nm, k, pr[k])) : 0;
#pragma unroll
    for (int k = 0; k < MLP_OUT; k++) ts[lane * MLP_OUT + k] = valid ? (pr[16 + k] - nm[32 + k]) / nm[48 + k] : 0.f;
    __syncthreads();
    bf16x4 h1[4][4], h2[4][4];
    f32x4 y[4];
    mlp_forward_wave(Wb, bias, xs, h1, h2, y, lane);
    // dL/dy = 2 (y - t) / (nsamp * 16); invalid samples contribute nothing
    const float sc = 2.0f / ((float)nsamp * MLP_OUT);
    bf16x4 dy[1][4];
    float lsum = 0.f, db3[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        const int smp = 16 * nt + c;
        const bool ok = ((long long)blockIdx.x * 64 + smp) < nsamp &&
                        (draw ? true : ((long long)blockIdx.x * 64 + smp) < n);
        f32x4 g;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float e = ok ? y[nt][i] - ts[smp * MLP_OUT + r4 + i] : 0.f;
            lsum += e * e;
            g[i] = sc * e;
            db3[i] += g[i];
        }
        dy[0][nt] = pack4(g);
    }
    float *gp = partial + (long long)blockIdx.x * MLP_NPARAM;
    // bias gradient of layer 3
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float v = sum16(db3[i]);
        if (c == 0) gp[MLP_OFF_B3 + r4 + i] = v;
    }
    // dW3 = H2 dY  (H2^T [64][s], dY^T [16][s])
    store_fs<4>(bufA, h2, lane);
    store_fs<1>(bufB, dy, lane);
    __syncthreads();
    weight_grad<4, 1>(bufA, bufB, gp + MLP_OFF_W3, MLP_OUT, lane);
    __syncthreads();
    // dH2^T = W3 dY^T, masked by ReLU'(H2)
    const unsigned short *W2 = Wb + MLP_OFF_W2, *W3 = Wb + MLP_OFF_W3;
    bf16x4 dh2[4][4];
    float db2[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        bf16x4 a = frag_w(W3, MLP_OUT, mt, 0, lane);
#pragma unroll
        for (int i = 0; i < 4; i++) db2[mt][i] = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            f32x4 d = mfma(a, dy[0][nt], f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int i = 0; i < 4; i++) {
                if (bf2f((unsigned short)h2[mt][nt][i]) <= 0.f) d[i] = 0.f;
                db2[mt][i] += d[i];
            }
            dh2[mt][nt] = pack4(d);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float v = sum16(db2[mt][i]);
            if (c == 0) gp[MLP_OFF_B2 + 16 * mt + r4 + i] = v;
        }
    // dW2 = H1 dH2
    store_fs<4>(bufA, h1, lane);
    store_fs<4>(bufB, dh2, lane);
    __syncthreads();
    weight_grad<4, 4>(bufA, bufB, gp + MLP_OFF_W2, MLP_H, lane);
    __syncthreads();
    // dH1^T = W2 dH2^T, masked by ReLU'(H1)
    bf16x4 dh1[4][4];
    float db1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        f32x4 d[4];
#pragma unroll
        for (int nt = 0; nt < 4; nt++) d[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; kt += 2) {
            const bf16x4 a0 = frag_w(W2, MLP_H, mt, kt, lane), a1 = frag_w(W2, MLP_H, mt, kt + 1, lane);
#pragma unroll
            for (int nt = 0; nt < 4; nt++) d[nt] = mfma2(a0, a1, dh2[kt][nt], dh2[kt + 1][nt], d[nt]);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) db1[mt][i] = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                if (bf2f((unsigned short)h1[mt][nt][i]) <= 0.f) d[nt][i] = 0.f;
                db1[mt][i] += d[nt][i];
            }
            dh1[mt][nt] = pack4(d[nt]);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            float v = sum16(db1[mt][i]);
            if (c == 0) gp[MLP_OFF_B1 + 16 * mt + r4 + i] = v;
        }
    // dW1 = X dH1  (X^T [16][s])
    for (int k = 0; k < MLP_IN; k++) bufA[k * 64 + lane] = xs[lane * MLP_IN + k];
    store_fs<4>(bufB, dh1, lane);
    __syncthreads();
    weight_grad<1, 4>(bufA, bufB, gp + MLP_OFF_W1, MLP_H, lane);
    // loss
    float l = lsum;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == 0) lossp[blockIdx.x] = l;
}

// Sums the per-wave gradients in a fixed order and applies one Adam update
// to the FP32 master parameters; refreshes the BF16 weights.
__global__ void __launch_bounds__(256) k_mlp_adam(const float *partial, int nparts, float *params, float *m1,
                                                  float *m2, unsigned short *Wb, float lr, float b1, float b2,
                                                  float eps, int t, int apply, float *grad_out) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    float g = 0.f;
    for (int i = 0; i < nparts; i++) g += partial[(long long)i * MLP_NPARAM + p];
    if (grad_out) grad_out[p] = g;
    if (!apply) return;
    float a = b1 * m1[p] + (1.f - b1) * g;
    float v = b2 * m2[p] + (1.f - b2) * g * g;
    m1[p] = a;
    m2[p] = v;
    float ah = a / (1.f - powf(b1, (float)t)), vh = v / (1.f - powf(b2, (float)t));
    float w = params[p] - lr * ah / (sqrtf(vh) + eps);
    params[p] = w;
    Wb[p] = f2bf(w);
}

__global__ void k_mlp_to_bf16(const float *params, unsigned short *Wb) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAM) Wb[p] = f2bf(params[p]);
}

// Inference for n samples (x: n x 16 FP32 rows with stride xs_stride floats),
// y: n x 16 FP32.  One wavefront per 64 samples.
__global__ void __launch_bounds__(64) k_mlp_forward(const unsigned short *Wb, const float *bias, const float *nm,
                                                    const float *x, long long xstride, long long n, float *y) {
    __shared__ unsigned short xs[64 * MLP_IN];
    __shared__ float ys[64 * MLP_OUT];
    const int lane = threadIdx.x;
    long long s = (long long)blockIdx.x * 64 + lane;
#pragma unroll
    for (int k = 0; k < MLP_IN; k++) xs[lane * MLP_IN + k] = s < n ? f2bf(norm_in(nm, k, x[s * xstride + k])) : 0;
    __syncthreads();
    bf16x4 h1[4][4], h2[4][4];
    f32x4 out[4];
    mlp_forward_wave(Wb, bias, xs, h1, h2, out, lane);
    const int r4 = 4 * (lane >> 4), c = lane & 15;
#pragma unroll
    for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) ys[(16 * nt + c) * MLP_OUT + r4 + i] = out[nt][i];
    __syncthreads();
    if (s < n)
#pragma unroll
        for (int k = 0; k < MLP_OUT; k++) y[s * MLP_OUT + k] = denorm_out(nm, k, ys[lane * MLP_OUT + k]);
}

// Column means and standard deviations of n pairs (32 columns), two passes in
// a fixed order (one workgroup per column).  Columns with a standard
// deviation below 1e-12 get unit scale.
__global__ void __launch_bounds__(256) k_mlp_norm_fit(const float *pairs, long long n, float *nm) {
    __shared__ double sh[256];
    const int col = blockIdx.x;
    double a = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) a += pairs[i * 32 + col];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double mean = sh[0] / (double)n;
    __syncthreads();
    a = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) {
        double d = pairs[i * 32 + col] - mean;
        a += d * d;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double sd = sqrt(sh[0] / (double)n);
        if (!(sd > 1e-12)) sd = 1.0;
        if (col < 16) { nm[col] = (float)mean; nm[16 + col] = (float)(1.0 / sd); }
        else { nm[32 + col - 16] = (float)mean; nm[48 + col - 16] = (float)sd; }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_mlp_norm_fit(const float *pairs, long long n, float *nm, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_norm_fit, dim3(32), dim3(256), 0, s, pairs, n, nm);
    return hipGetLastError();
}

hipError_t launch_mlp_fwdbwd(const unsigned short *Wb, const float *bias, const float *nm, const float *pairs,
                             long long n, long long nsamp, int draw, unsigned long long seed, unsigned long long step,
                             float *partial, float *lossp, hipStream_t s) {
    int nw = (int)((nsamp + 63) / 64);
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(nw), dim3(64), 0, s, Wb, bias, nm, pairs, n, nsamp, draw, seed, step,
                       partial, lossp);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(const float *partial, int nparts, float *params, float *m1, float *m2, unsigned short *Wb,
                           float lr, int t, int apply, float *grad_out, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, partial, nparts, params, m1, m2,
                       Wb, lr, 0.9f, 0.999f, 1e-8f, t, apply, grad_out);
    return hipGetLastError();
}

hipError_t launch_mlp_to_bf16(const float *params, unsigned short *Wb, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_to_bf16, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, params, Wb);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const unsigned short *Wb, const float *bias, const float *nm, const float *x,
                              long long xstride, long long n, float *y, hipStream_t s) {
    int nw = (int)((n + 63) / 64);
    if (nw == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(nw), dim3(64), 0, s, Wb, bias, nm, x, xstride, n, y);
    return hipGetLastError();
}

}  // namespace lelbm
