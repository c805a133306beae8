// Warm-start network for the local spectral problems (section 4.2): a small fully
// convolutional network maps the permeability of omega_i = K1 u K2 to a block of
// initial vectors for the Rayleigh-Ritz solve of the face's pencil.
//
//   input   X[h][w] = log10(kappa) / 3 on the cells of omega_i, rows h across E_i
//           (H = 2 x block depth), columns w along E_i (W = J, in the order of the
//           pencil's fine-face index);
//   layers  four 3x3 convolutions, zero padding, channels 1 -> 16 -> 16 -> 16 -> 8,
//           ReLU after the first three;
//   output  the first 8 DCT-II vectors of length W (unit norm; zero beyond W) plus
//           the mean over the rows: the network learns a correction to the start
//           that is exact for a homogeneous medium.
//
// Parameters: one flat FP32 array, per layer the weights [cout][cin][3][3] and
// then the biases [cout].  Training minimises, per sample, sum_c |y_c/|y_c| - s_c v_c|^2
// over the first k channels (v_c: the eigenvectors of the k largest mu of the
// pencil, s_c = sign(y_c . v_c)), averaged over the batch, with Adam.
//
// Kernels: one workgroup of 256 threads per sample.  The forward pass keeps both
// activation buffers (16 channels, padded by one cell) and the current layer's
// weights in LDS; each thread computes all output channels of two positions, with
// the weights read as float4 broadcasts.  The backward pass reloads each layer's
// input from the saved activations and propagates the output gradient through LDS;
// per-sample gradients are summed by the Adam kernel (no atomics, fixed order).
#include "common.h"

namespace {

constexpr int C = 16, KOUT = 8, NT = 256;
constexpr int WL0 = 0, BL0 = WL0 + C * 9, WL1 = BL0 + C, BL1 = WL1 + C * C * 9, WL2 = BL1 + C, BL2 = WL2 + C * C * 9,
              WL3 = BL2 + C, BL3 = WL3 + KOUT * C * 9, NPARAM = BL3 + KOUT;
constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f, ADAM_EPS = 1e-8f, NORM_EPS = 1e-12f;

struct Shape {
    int H, W, PW, plane, HW;
};
__host__ __device__ inline Shape shape(int H, int W) { return Shape{H, W, W + 2, (H + 2) * (W + 2), H * W}; }
__device__ inline int padpos(const Shape& S, int p) { return (p / S.W + 1) * S.PW + p % S.W + 1; }
__device__ inline int tapoff(const Shape& S, int t) { return (t / 3 - 1) * S.PW + (t % 3 - 1); }

// out = conv3x3(in) + b (ReLU optional) on the interior of padded LDS planes.
// wt: LDS [CIN][9][COUT] (the layer's weights transposed for float4 reads).
template <int CIN, int COUT>
__device__ void conv_layer(const Shape& S, const float* in, float* out, const float* __restrict__ wg,
                           const float* __restrict__ bg, float* wt, float* bs, bool relu) {
    const int tid = threadIdx.x;
    for (int e = tid; e < COUT * CIN * 9; e += NT) {
        const int co = e / (CIN * 9), r = e % (CIN * 9);
        wt[r * COUT + co] = wg[e];
    }
    for (int e = tid; e < COUT; e += NT) bs[e] = bg[e];
    __syncthreads();
    for (int p0 = tid; p0 < S.HW; p0 += 2 * NT) {
        const int p1 = p0 + NT;
        const bool two = p1 < S.HW;
        const int q0 = padpos(S, p0), q1 = two ? padpos(S, p1) : q0;
        float a0[COUT], a1[COUT];
#pragma unroll
        for (int co = 0; co < COUT; ++co) a0[co] = a1[co] = bs[co];
        for (int ci = 0; ci < CIN; ++ci) {
            const float* ip = in + ci * S.plane;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int off = tapoff(S, t);
                const float x0 = ip[q0 + off], x1 = ip[q1 + off];
                const float4* wv = reinterpret_cast<const float4*>(wt + (ci * 9 + t) * COUT);
#pragma unroll
                for (int q = 0; q < COUT / 4; ++q) {
                    const float4 w4 = wv[q];
                    a0[4 * q + 0] += w4.x * x0;
                    a0[4 * q + 1] += w4.y * x0;
                    a0[4 * q + 2] += w4.z * x0;
                    a0[4 * q + 3] += w4.w * x0;
                    a1[4 * q + 0] += w4.x * x1;
                    a1[4 * q + 1] += w4.y * x1;
                    a1[4 * q + 2] += w4.z * x1;
                    a1[4 * q + 3] += w4.w * x1;
                }
            }
        }
#pragma unroll
        for (int co = 0; co < COUT; ++co) {
            out[co * S.plane + q0] = relu ? fmaxf(a0[co], 0.f) : a0[co];
            if (two) out[co * S.plane + q1] = relu ? fmaxf(a1[co], 0.f) : a1[co];
        }
    }
    __syncthreads();
}

__device__ void store_act(const Shape& S, const float* buf, float* dst) {
    for (int e = threadIdx.x; e < C * S.HW; e += NT) {
        const int ch = e / S.HW, p = e % S.HW;
        dst[e] = buf[ch * S.plane + padpos(S, p)];
    }
}

// Forward pass of n samples X [n][H][W] -> Y [n][8][W]; act (optional) receives the
// post-ReLU activations of the first three layers [n][3][16][H][W].
__global__ void __launch_bounds__(NT) k_cnn_fwd(const float* __restrict__ prm, const float* __restrict__ X, int H,
                                                int W, float* __restrict__ Y, float* __restrict__ act) {
    extern __shared__ float sm[];
    const Shape S = shape(H, W);
    float* A = sm;
    float* B = A + C * S.plane;
    float* wt = B + C * S.plane;
    float* bs = wt + C * C * 9;
    const long long s = blockIdx.x;
    const int tid = threadIdx.x;
    for (int e = tid; e < 2 * C * S.plane; e += NT) sm[e] = 0.f;
    __syncthreads();
    for (int p = tid; p < S.HW; p += NT) A[padpos(S, p)] = X[s * S.HW + p];
    __syncthreads();
    float* as = act ? act + s * 3 * C * S.HW : nullptr;
    conv_layer<1, C>(S, A, B, prm + WL0, prm + BL0, wt, bs, true);
    if (as) store_act(S, B, as);
    conv_layer<C, C>(S, B, A, prm + WL1, prm + BL1, wt, bs, true);
    if (as) store_act(S, A, as + C * S.HW);
    conv_layer<C, C>(S, A, B, prm + WL2, prm + BL2, wt, bs, true);
    if (as) store_act(S, B, as + 2 * C * S.HW);
    conv_layer<C, KOUT>(S, B, A, prm + WL3, prm + BL3, wt, bs, false);
    for (int e = tid; e < KOUT * W; e += NT) {
        const int c = e / W, w = e % W;
        float sum = 0.f;
        for (int h = 0; h < H; ++h) sum += A[c * S.plane + (h + 1) * S.PW + w + 1];
        const double d = c < W ? cos(M_PI * (w + 0.5) * c / W) * sqrt((c == 0 ? 1.0 : 2.0) / W) : 0.0;
        Y[s * KOUT * W + e] = sum / H + (float)d;
    }
}

// Weight and bias gradients of one layer from the output gradient G and the layer
// input A (both padded LDS planes), written to the sample's gradient row.
template <int CIN, int COUT>
__device__ void layer_wgrad(const Shape& S, const float* G, const float* A, float* __restrict__ gw,
                            float* __restrict__ gb) {
    for (int e = threadIdx.x; e < COUT * CIN * 9 + COUT; e += NT) {
        float acc = 0.f;
        if (e < COUT * CIN * 9) {
            const int co = e / (CIN * 9), r = e % (CIN * 9), ci = r / 9, t = r % 9;
            const float* g = G + co * S.plane;
            const float* a = A + ci * S.plane + tapoff(S, t);
            for (int p = 0; p < S.HW; ++p) {
                const int q = padpos(S, p);
                acc += g[q] * a[q];
            }
            gw[e] = acc;
        } else {
            const int co = e - COUT * CIN * 9;
            const float* g = G + co * S.plane;
            for (int p = 0; p < S.HW; ++p) acc += g[padpos(S, p)];
            gb[co] = acc;
        }
    }
}

// In place on A: A[ci] <- (sum_co,t w[co][ci][t] G[co][. - off(t)]) * (A[ci] > 0), i.e.
// the gradient w.r.t. the previous layer's pre-activation (A holds its ReLU output).
// wt: LDS [COUT][9][CIN].
template <int CIN, int COUT>
__device__ void layer_dgrad(const Shape& S, const float* G, float* A, const float* __restrict__ wg, float* wt) {
    const int tid = threadIdx.x;
    for (int e = tid; e < COUT * CIN * 9; e += NT) {
        const int co = e / (CIN * 9), r = e % (CIN * 9), ci = r / 9, t = r % 9;
        wt[(co * 9 + t) * CIN + ci] = wg[e];
    }
    __syncthreads();
    for (int p = tid; p < S.HW; p += NT) {
        const int q = padpos(S, p);
        float ga[CIN];
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) ga[ci] = 0.f;
        for (int co = 0; co < COUT; ++co) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const float g = G[co * S.plane + q - tapoff(S, t)];
                const float4* wv = reinterpret_cast<const float4*>(wt + (co * 9 + t) * CIN);
#pragma unroll
                for (int k = 0; k < CIN / 4; ++k) {
                    const float4 w4 = wv[k];
                    ga[4 * k + 0] += w4.x * g;
                    ga[4 * k + 1] += w4.y * g;
                    ga[4 * k + 2] += w4.z * g;
                    ga[4 * k + 3] += w4.w * g;
                }
            }
        }
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) {
            float* a = A + ci * S.plane + q;
            *a = (*a > 0.f) ? ga[ci] : 0.f;
        }
    }
    __syncthreads();
}

__device__ void load_plane(const Shape& S, const float* __restrict__ src, int nch, float* dst) {
    for (int e = threadIdx.x; e < nch * S.HW; e += NT) {
        const int ch = e / S.HW, p = e % S.HW;
        dst[ch * S.plane + padpos(S, p)] = src[e];
    }
}

// Loss of each sample and the gradient of every parameter, per sample:
// grad [n][NPARAM], loss [n].  V: targets [n][8][W] (the first k rows used).
__global__ void __launch_bounds__(NT) k_cnn_bwd(const float* __restrict__ prm, const float* __restrict__ X,
                                                const float* __restrict__ act, const float* __restrict__ Y,
                                                const float* __restrict__ V, int H, int W, int k,
                                                float* __restrict__ grad, float* __restrict__ loss) {
    extern __shared__ float sm[];
    const Shape S = shape(H, W);
    float* Gb = sm;
    float* Ab = Gb + C * S.plane;
    float* wt = Ab + C * S.plane;
    float* gy = wt + C * C * 9;   // [KOUT][64]
    float* lc = gy + KOUT * 64;   // [KOUT]
    const long long s = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int e = tid; e < 2 * C * S.plane; e += NT) sm[e] = 0.f;
    // dL/dy per channel (one wavefront per channel, lane = position along E)
    for (int c = wv; c < KOUT; c += NT / 64) {
        float g = 0.f, L = 0.f;
        if (c < k) {
            const float y = lane < W ? Y[(s * KOUT + c) * W + lane] : 0.f;
            const float v = lane < W ? V[(s * KOUT + c) * W + lane] : 0.f;
            const float nrm = sqrtf(wave_sum(y * y) + NORM_EPS);
            const float u = y / nrm;
            const float sg = wave_sum(u * v) >= 0.f ? 1.f : -1.f;
            const float d = u - sg * v;
            L = wave_sum(d * d);
            g = (2.f / nrm) * (d - u * wave_sum(u * d));
        }
        if (lane < W) gy[c * 64 + lane] = g;
        if (lane == 0) lc[c] = L;
    }
    __syncthreads();
    if (tid == 0) {
        float L = 0.f;
        for (int c = 0; c < k; ++c) L += lc[c];
        loss[s] = L;
    }
    // through the mean over rows: dL/dz3[c][h][w] = gy[c][w] / H
    for (int e = tid; e < KOUT * S.HW; e += NT) {
        const int c = e / S.HW, p = e % S.HW;
        Gb[c * S.plane + padpos(S, p)] = gy[c * 64 + p % W] / H;
    }
    const float* as = act + s * 3 * C * S.HW;
    float* gs = grad + s * NPARAM;
    // layer 3 (16 -> 8)
    load_plane(S, as + 2 * C * S.HW, C, Ab);
    __syncthreads();
    layer_wgrad<C, KOUT>(S, Gb, Ab, gs + WL3, gs + BL3);
    __syncthreads();
    layer_dgrad<C, KOUT>(S, Gb, Ab, prm + WL3, wt);
    // layer 2 (16 -> 16): output gradient now in Ab
    load_plane(S, as + C * S.HW, C, Gb);
    __syncthreads();
    layer_wgrad<C, C>(S, Ab, Gb, gs + WL2, gs + BL2);
    __syncthreads();
    layer_dgrad<C, C>(S, Ab, Gb, prm + WL2, wt);
    // layer 1 (16 -> 16): output gradient in Gb
    load_plane(S, as, C, Ab);
    __syncthreads();
    layer_wgrad<C, C>(S, Gb, Ab, gs + WL1, gs + BL1);
    __syncthreads();
    layer_dgrad<C, C>(S, Gb, Ab, prm + WL1, wt);
    // layer 0 (1 -> 16): output gradient in Ab, input X
    load_plane(S, X + s * S.HW, 1, Gb);
    __syncthreads();
    layer_wgrad<1, C>(S, Ab, Gb, gs + WL0, gs + BL0);
}

// Adam on the batch-mean gradient (per-sample rows summed in a fixed order).
__global__ void k_cnn_adam(const float* __restrict__ grad, int n, float* __restrict__ prm, float* __restrict__ m,
                           float* __restrict__ v, float lr, float bc1, float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float g = 0.f;
    for (int s = 0; s < n; ++s) g += grad[(long long)s * NPARAM + p];
    g /= n;
    const float mm = ADAM_B1 * m[p] + (1.f - ADAM_B1) * g;
    const float vv = ADAM_B2 * v[p] + (1.f - ADAM_B2) * g * g;
    m[p] = mm;
    v[p] = vv;
    prm[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + ADAM_EPS);
}

// Network inputs of the interior coarse faces (square blocks b x b): x-faces first
// (rows along x over K(I-1,J) and K(I,J), columns along y), then y-faces (rows along y
// over K(I,J-1) and K(I,J), columns along x).  kinv: kappa^{-1} per cell.
__global__ void k_cnn_windows(const double* __restrict__ kinv, int nx, int Nx, int b, int nex, int ne,
                              float* __restrict__ X) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int hw = 2 * b * b;
    if (e >= (long long)ne * hw) return;
    const int fid = (int)(e / hw), r = (int)(e % hw), h = r / b, w = r % b;
    long long cell;
    if (fid < nex) {
        const int J = fid / (Nx - 1), I = fid % (Nx - 1) + 1;
        cell = (long long)(J * b + w) * nx + (I - 1) * b + h;
    } else {
        const int f = fid - nex, J = f / Nx + 1, I = f % Nx;
        cell = (long long)((J - 1) * b + h) * nx + I * b + w;
    }
    X[e] = (float)(-log10(kinv[cell]) / 3.0);
}

// ------------------------------------------------------------------ BF16 inference
// The same forward pass (no saved activations) on the matrix cores: one workgroup
// per sample; activations in LDS as BF16 with the 16 channels innermost
// ([H+2][W+2][16], zero ring).  A tile is 16 consecutive positions of one row (the
// columns past W repeat column W - 1 and their outputs are dropped).  Each tile
// computes D = Wt X^T (rows: output channels, k: input channels or taps, columns:
// positions): layer 0 (one input channel) in FP32 as three v_mfma_f32_16x16x4_f32
// (k: the 9 taps, padded to 12 with zero weights), layers 1-3 as one
// v_mfma_f32_16x16x16_bf16 per tap, FP32 accumulation.  Operand layout of both
// instructions: lane l holds A[l%16][kq(l/16) + e] and B[kq(l/16) + e][l%16] (e < q,
// q = 1 or 4 elements per lane); result item j of lane l is D[4(l/16) + j][l%16], so
// a lane ends with 4 consecutive channels of one position (one 8-byte store).
typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ inline unsigned short f2bf(float x) {  // round to nearest even
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// The tile's outputs of this lane (channels 4 kg .. 4 kg + 3 at column w0 + col): bias
// and ReLU to the next activation plane, or the raw values to yout [H W][KOUT].
template <int COUT, bool HIDDEN>
__device__ inline void tile_out(const Shape& S, int h, int w0, int col, int kg, const f4_t& acc, const float* bias4,
                                unsigned short* __restrict__ out, float* __restrict__ yout) {
    const int w = w0 + col;
    if (w >= S.W || 4 * kg >= COUT) return;
    if (HIDDEN) {
        unsigned short v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = f2bf(fmaxf(acc[j] + bias4[j], 0.f));
        *reinterpret_cast<uint2*>(out + ((h + 1) * S.PW + w + 1) * C + 4 * kg) =
            make_uint2(v[0] | ((unsigned)v[1] << 16), v[2] | ((unsigned)v[3] << 16));
    } else {
        *reinterpret_cast<float4*>(yout + (h * S.W + w) * KOUT + 4 * kg) =
            make_float4(acc[0] + bias4[0], acc[1] + bias4[1], acc[2] + bias4[2], acc[3] + bias4[3]);
    }
}

// layer 0: xin (padded FP32 plane) -> out (BF16, 16 channels), FP32 matrix cores
__device__ void conv0_mfma(const Shape& S, const float* __restrict__ xin, unsigned short* __restrict__ out,
                           const float* __restrict__ wg, const float* __restrict__ bg) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    float bw[3], bias4[4];
    int toff[3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const int t = 4 * kk + kg;
        bw[kk] = t < 9 ? wg[col * 9 + t] : 0.f;  // A[cout = col][tap t]
        toff[kk] = t < 9 ? tapoff(S, t) : 0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) bias4[j] = bg[4 * kg + j];
    const int nch = (S.W + 15) >> 4, ntiles = S.H * nch;
    for (int tile = wave; tile < ntiles; tile += NT / 64) {
        const int h = tile / nch, w0 = (tile - h * nch) * 16;
        const int q = (h + 1) * S.PW + min(w0 + col, S.W - 1) + 1;
        f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(bw[kk], xin[q + toff[kk]], acc, 0, 0, 0);
        tile_out<C, true>(S, h, w0, col, kg, acc, bias4, out, nullptr);
    }
    __syncthreads();
}

template <int COUT, bool HIDDEN>
__device__ void conv_mfma(const Shape& S, const unsigned short* __restrict__ in, unsigned short* __restrict__ out,
                          float* __restrict__ yout, const float* __restrict__ wg, const float* __restrict__ bg) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kg = lane >> 4;
    bf4_t wfr[9];  // A[cout = col][cin = 4 kg + e] of each tap
    int toff[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        toff[t] = tapoff(S, t) * C;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ci = 4 * kg + e;
            wfr[t][e] = (short)f2bf(col < COUT ? wg[(col * C + ci) * 9 + t] : 0.f);
        }
    }
    float bias4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bias4[j] = 4 * kg + j < COUT ? bg[4 * kg + j] : 0.f;
    const int nch = (S.W + 15) >> 4, ntiles = S.H * nch;
    for (int tile = wave; tile < ntiles; tile += NT / 64) {
        const int h = tile / nch, w0 = (tile - h * nch) * 16;
        const int base = ((h + 1) * S.PW + min(w0 + col, S.W - 1) + 1) * C + 4 * kg;
        f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const bf4_t x = *reinterpret_cast<const bf4_t*>(in + base + toff[t]);  // B[cin][position col]
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wfr[t], x, acc, 0, 0, 0);
        }
        tile_out<COUT, HIDDEN>(S, h, w0, col, kg, acc, bias4, out, yout);
    }
    __syncthreads();
}

__global__ void __launch_bounds__(NT) k_cnn_infer_bf16(const float* __restrict__ prm, const float* __restrict__ X,
                                                       int H, int W, float* __restrict__ Y) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Shape S = shape(H, W);
    unsigned short* A0 = reinterpret_cast<unsigned short*>(smem_raw);  // [plane][16] BF16
    unsigned short* A1 = A0 + (size_t)S.plane * C;
    float* xin = reinterpret_cast<float*>(A1 + (size_t)S.plane * C);    // padded input plane
    float* yout = reinterpret_cast<float*>(A1);                         // [HW][8], over A1 after layer 2
    const long long s = blockIdx.x;
    const int tid = threadIdx.x;
    uint4* z = reinterpret_cast<uint4*>(smem_raw);
    const int nz = (int)((2 * (size_t)S.plane * C * sizeof(unsigned short) + (size_t)S.plane * sizeof(float) + 15) / 16);
    for (int e = tid; e < nz; e += NT) z[e] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    for (int p = tid; p < S.HW; p += NT) xin[padpos(S, p)] = X[s * S.HW + p];
    __syncthreads();
    conv0_mfma(S, xin, A0, prm + WL0, prm + BL0);
    conv_mfma<C, true>(S, A0, A1, nullptr, prm + WL1, prm + BL1);
    conv_mfma<C, true>(S, A1, A0, nullptr, prm + WL2, prm + BL2);
    conv_mfma<KOUT, false>(S, A0, nullptr, yout, prm + WL3, prm + BL3);
    for (int e = tid; e < KOUT * W; e += NT) {
        const int c = e / W, w = e % W;
        float sum = 0.f;
        for (int h = 0; h < H; ++h) sum += yout[(h * W + w) * KOUT + c];
        const double d = c < W ? cos(M_PI * (w + 0.5) * c / W) * sqrt((c == 0 ? 1.0 : 2.0) / W) : 0.0;
        Y[s * KOUT * W + e] = sum / H + (float)d;
    }
}

size_t infer_lds(int H, int W) {  // both activation buffers and the input plane, in 16-byte units
    const size_t plane = (size_t)shape(H, W).plane;
    return (2 * plane * C * sizeof(unsigned short) + plane * sizeof(float) + 15) / 16 * 16;
}

size_t fwd_lds(int H, int W) { return sizeof(float) * (2 * C * shape(H, W).plane + C * C * 9 + C); }
size_t bwd_lds(int H, int W) { return sizeof(float) * (2 * C * shape(H, W).plane + C * C * 9 + KOUT * 64 + KOUT); }

void allow_cnn_lds() {
    static bool done = false;
    if (done) return;
    const int big = 160 * 1024;
    (void)hipFuncSetAttribute((const void*)k_cnn_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute((const void*)k_cnn_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipGetLastError();
    done = true;
}

}  // namespace

namespace tgms {

int cnn_nparams() { return NPARAM; }
int cnn_kout() { return KOUT; }

// H, W within the kernels' LDS layout: H, W in [1, 64], H * W <= 512.
bool cnn_shape_ok(int H, int W) { return H >= 1 && W >= 1 && H <= 64 && W <= 64 && H * W <= 512; }

size_t cnn_train_workspace(long long n, int H, int W) {
    return (size_t)n * (3 * C * (size_t)H * W + KOUT * (size_t)W + NPARAM + 1);
}

void cnn_forward(hipStream_t st, const float* prm, const float* X, long long n, int H, int W, float* Y, float* act) {
    allow_cnn_lds();
    hipLaunchKernelGGL(k_cnn_fwd, dim3((unsigned)n), dim3(NT), fwd_lds(H, W), st, prm, X, H, W, Y, act);
    LAUNCH_OK();
}

double cnn_train_step(hipStream_t st, float* prm, float* m, float* v, int t, float lr, const float* X, const float* V,
                      long long n, int H, int W, int k, float* work) {
    allow_cnn_lds();
    float* act = work;
    float* Y = act + n * 3 * C * H * W;
    float* grad = Y + n * KOUT * W;
    float* loss = grad + n * NPARAM;
    hipLaunchKernelGGL(k_cnn_fwd, dim3((unsigned)n), dim3(NT), fwd_lds(H, W), st, (const float*)prm, X, H, W, Y, act);
    LAUNCH_OK();
    hipLaunchKernelGGL(k_cnn_bwd, dim3((unsigned)n), dim3(NT), bwd_lds(H, W), st, (const float*)prm, X,
                       (const float*)act, (const float*)Y, V, H, W, k, grad, loss);
    LAUNCH_OK();
    const float bc1 = (float)(1.0 - std::pow((double)ADAM_B1, t)), bc2 = (float)(1.0 - std::pow((double)ADAM_B2, t));
    hipLaunchKernelGGL(k_cnn_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, (const float*)grad, (int)n, prm, m, v,
                       lr, bc1, bc2);
    LAUNCH_OK();
    std::vector<float> lh((size_t)n);
    HIP_OK(hipMemcpyAsync(lh.data(), loss, sizeof(float) * n, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    double L = 0.0;
    for (float x : lh) L += x;
    return L / n;
}

void cnn_infer_bf16(hipStream_t st, const float* prm, const float* X, long long n, int H, int W, float* Y) {
    hipLaunchKernelGGL(k_cnn_infer_bf16, dim3((unsigned)n), dim3(NT), infer_lds(H, W), st, prm, X, H, W, Y);
    LAUNCH_OK();
}

void cnn_windows(tgms_ctx* c, float* X) {
    const long long tot = (long long)c->ne * 2 * c->bx * c->bx;
    hipLaunchKernelGGL(k_cnn_windows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream,
                       (const double*)c->kinv, c->nx, c->Nx, c->bx, c->nex, c->ne, X);
    LAUNCH_OK();
}

}  // namespace tgms
