// mlp.hip -- the small MLP of the learned flux correction on CDNA4 matrix cores.
//
// Network: 32 inputs -> H -> H -> H (SiLU) -> 8 outputs, parameters as one flat vector
// W1[H][32], b1[H], W2[H][H], b2[H], W3[H][H], b3[H], W4[8][H], b4[8] (weights row-major, output first).
// The products run on v_mfma_f32_16x16x32_bf16: BF16 operands (weights from a BF16 copy of the FP32
// master parameters, activations rounded to BF16), FP32 accumulation; biases, SiLU and every reduction
// stay in FP32. A second mode evaluates the same products with FP32 FMAs (used to check gradients
// against a float64 reference to FP32 accuracy).
//
// MFMA 16x16x32 operand layout (wave of 64 lanes, lane l, q = l / 16, r = l % 16):
//   A (16 x 32, rows m, cols k): lane holds A[r][8q .. 8q+7]
//   B (32 x 16, rows k, cols n): lane holds B[8q .. 8q+7][r]
//   C/D (16 x 16):               lane holds D[4q .. 4q+3][r]
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <type_traits>

#include "bmhd_internal.h"

namespace bmhd {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int MLP_IN = 32;
constexpr int MLP_OUT = 8;

struct MlpView {
    int H;
    long off_w[4], off_b[4];
    int nin[4], nout[4];
};

__host__ __device__ inline MlpView mlp_view(int H) {
    MlpView v;
    v.H = H;
    const int in[4] = {MLP_IN, H, H, H}, out[4] = {H, H, H, MLP_OUT};
    long o = 0;
    for (int l = 0; l < 4; ++l) {
        v.nin[l] = in[l];
        v.nout[l] = out[l];
        v.off_w[l] = o;
        o += long(out[l]) * in[l];
        v.off_b[l] = o;
        o += out[l];
    }
    return v;
}

__host__ __device__ inline long mlp_params(int H) {
    return long(H) * MLP_IN + H + 2L * (long(H) * H + H) + long(MLP_OUT) * H + MLP_OUT;
}

// z * sigmoid(z) with the hardware exponential and reciprocal (no IEEE division sequence)
__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------------------------------------------
// fused forward: one wave per tile of 16 samples, activations of the tile in LDS (BF16 for the
// MFMA mode, FP32 for the FP32 mode), weights read from L2.

template <int H, bool MFMA>
struct FwdLds {
    using T = typename std::conditional<MFMA, __bf16, float>::type;
    static constexpr int PAD = MFMA ? 8 : 1;  // row padding against bank conflicts
    static constexpr int LD = H + PAD;
};

template <int H, bool MFMA>
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ P, const __bf16 *__restrict__ Pb, int n,
                                                     const float *__restrict__ X, float *__restrict__ Y,
                                                     float *__restrict__ Zsave) {
    using L = FwdLds<H, MFMA>;
    using T = typename L::T;
    __shared__ T act[4][16 * L::LD];
    const MlpView V = mlp_view(H);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
    const int tile = blockIdx.x * 4 + wave;
    const int s0 = tile * 16;  // waves past the end still take part in the barriers
    T *a = act[wave];
    // stage the 16 x 32 input tile (rows beyond n are zero)
    for (int e = lane; e < 16 * MLP_IN; e += 64) {
        const int m = e / MLP_IN, k = e % MLP_IN;
        const float x = (s0 + m < n) ? X[size_t(s0 + m) * MLP_IN + k] : 0.0f;
        a[m * L::LD + k] = T(x);
    }
    __syncthreads();
    for (int l = 0; l < 4; ++l) {
        const int nin = V.nin[l], nout = V.nout[l];
        const int ntile = (nout + 15) / 16;
        float outv[H / 16][4];
        for (int nt = 0; nt < ntile; ++nt) {
            const int o = nt * 16 + r;  // output column this lane's B operand and results belong to
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            if constexpr (MFMA) {
                // accumulate onto the bias, as the inference kernel does (equal results bit for bit)
                const float b0 = (o < nout) ? P[V.off_b[l] + o] : 0.0f;
                acc = f32x4{b0, b0, b0, b0};
                for (int k0 = 0; k0 < nin; k0 += 32) {
                    bf16x8 av, bv;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        av[j] = a[r * L::LD + k0 + 8 * q + j];
                        bv[j] = (o < nout) ? Pb[V.off_w[l] + long(o) * nin + k0 + 8 * q + j] : __bf16(0.0f);
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
                }
            } else {
                // same output layout, plain FP32 products
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = 4 * q + i;
                    float s = 0.f;
                    if (o < nout)
                        for (int k = 0; k < nin; ++k) s = fmaf(float(a[m * L::LD + k]), P[V.off_w[l] + long(o) * nin + k], s);
                    acc[i] = s;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) outv[nt][i] = acc[i];
        }
        __syncthreads();  // every lane has read this layer's input
        for (int nt = 0; nt < ntile; ++nt) {
            const int o = nt * 16 + r;
            if (o >= nout) continue;
            const float bias = MFMA ? 0.0f : P[V.off_b[l] + o];  // MFMA: already in the products
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 4 * q + i;
                const float z = MFMA ? outv[nt][i] : outv[nt][i] + bias;
                if (s0 + m >= n) continue;
                if (l < 3) {
                    if (Zsave) Zsave[(size_t(l) * n + s0 + m) * H + o] = z;
                    a[m * L::LD + o] = T(silu(z));
                } else {
                    Y[size_t(s0 + m) * MLP_OUT + o] = z;
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------------
// inference (BF16 products, no saved pre-activations): a persistent grid of one workgroup per CU keeps
// every BF16 weight in LDS (rows padded by 8 elements against bank conflicts; the 8-row output layer
// padded to 16 zero rows; 84.2 KB for H = 128) and each wave streams tiles of 16 samples through the four
// layers with the activations in registers (each layer's products become the next layer's operands by
// lane swaps, chunk_operand below).

// per workgroup: three wavefronts per SIMD (162 VGPRs), two 16-sample tiles each per iteration, so that
// each weight fragment read from LDS feeds two products. Measured per launch on the 128^3 learned stage:
// activations through a private LDS tile per wave, one tile, sixteen wavefronts 0.81 ms; activations in
// registers, one tile, sixteen wavefronts (103 VGPRs) 0.76 ms; two tiles, twelve wavefronts 0.75 ms;
// two tiles, sixteen wavefronts (128 VGPRs, 112 bytes of spills) 0.87 ms.
constexpr int MLP_INFER_WAVES = 12;
constexpr int MLP_INFER_TILES = 2;

template <int H>
struct InferLds {
    static constexpr int L1 = MLP_IN + 8;  // padded row of the first layer (32 inputs)
    static constexpr int LH = H + 8;       // padded row of the H-input layers
    static constexpr int W1 = 0;
    static constexpr int W2 = W1 + H * L1;
    static constexpr int W3 = W2 + H * LH;
    static constexpr int W4 = W3 + H * LH;
    static constexpr int NWE = W4 + 16 * LH;
};

// The 32-wide input chunk c of the next layer as an MFMA B operand (lane (q, r): act[sample r][32c + 8q ..
// 32c + 8q + 7]) from this layer's products, where lane (q, r) holds outputs 16 nt + 4q .. + 3 of sample r:
// lo = its four (BF16) of nt = 2c, hi = its four of nt = 2c + 1. Lane row q (16 lanes) needs the pieces of
// rows 2(q mod 2) and 2(q mod 2) + 1 of nt = 2c + q / 2; one 32-lane and one 16-lane swap per dword move
// them there, in registers (gfx950 lane swaps: the first exchanges a's upper half with b's lower half,
// the second a's odd rows with b's even rows).
__device__ __forceinline__ bf16x8 chunk_operand(bf16x4 lo, bf16x4 hi) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const u32x2 a = __builtin_bit_cast(u32x2, lo), b = __builtin_bit_cast(u32x2, hi);
    u32x4 t;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const auto h = __builtin_amdgcn_permlane32_swap(a[d], b[d], false, false);
        const auto w = __builtin_amdgcn_permlane16_swap(h[0], h[1], false, false);
        t[d] = w[0];      // outputs 8q .. 8q + 3 of the chunk
        t[2 + d] = w[1];  // outputs 8q + 4 .. 8q + 7
    }
    return __builtin_bit_cast(bf16x8, t);
}

// X holds FP32 inputs (rounded to BF16 here) or inputs already rounded to BF16 by their producer.
template <int H, int NW, int TP, typename TX>
__global__ void __launch_bounds__(64 * NW) k_mlp_infer(const float *__restrict__ P, const __bf16 *__restrict__ Pb,
                                                       int n, const TX *__restrict__ X, float *__restrict__ Y) {
    using Z = InferLds<H>;
    constexpr int NT = H / 16, NC = H / 32;
    __shared__ __attribute__((aligned(16))) __bf16 sw[Z::NWE];
    __shared__ float sb[3 * H + 16];
    const MlpView V = mlp_view(H);
    // stage the weights (16-byte moves) and biases
    const int ldl[4] = {Z::L1, Z::LH, Z::LH, Z::LH}, basel[4] = {Z::W1, Z::W2, Z::W3, Z::W4};
    for (int l = 0; l < 4; ++l) {
        const int nin = V.nin[l], nout = V.nout[l], rows = l == 3 ? 16 : nout, per = nin / 8;
        for (int c = threadIdx.x; c < rows * per; c += blockDim.x) {
            const int row = c / per, c8 = c % per;
            bf16x8 v;
            if (row < nout) v = *reinterpret_cast<const bf16x8 *>(Pb + V.off_w[l] + long(row) * nin + 8 * c8);
            else
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = __bf16(0.0f);
            *reinterpret_cast<bf16x8 *>(sw + basel[l] + row * ldl[l] + 8 * c8) = v;
        }
        for (int o = threadIdx.x; o < rows; o += blockDim.x) sb[l * H + o] = o < nout ? P[V.off_b[l] + o] : 0.0f;
    }
    __syncthreads();
    // Products are formed transposed, D[out][sample] = W x act^T: the weight tile is the A operand (lane
    // holds W[o][8q .. 8q+7]), the activation chunk the B operand (lane holds act[sample r][8q .. 8q+7]),
    // so lane (q, r) ends with outputs 4q .. 4q+3 of sample r, which chunk_operand turns into the next
    // layer's B operands without leaving registers. A wavefront carries TP tiles of 16 samples at once, so
    // each weight fragment read from LDS feeds TP products.
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
    const int ntiles = (n + 15) / 16;
    for (int t0 = (blockIdx.x * NW + wave) * TP; t0 < ntiles; t0 += gridDim.x * NW * TP) {
        // the biases are read from LDS in each tile, where they are used: hoisted out of the loop they
        // would hold 100 registers (no instruction is emitted for this)
        asm volatile("" ::: "memory");
        bf16x8 act[TP][NC];  // this layer's input chunks (the first layer's 32 inputs: chunk 0)
#pragma unroll
        for (int p = 0; p < TP; ++p) {
            const int smp = (t0 + p) * 16 + r;
            bf16x8 v;
            if (smp < n) {
                if constexpr (std::is_same<TX, __bf16>::value) {
                    v = *reinterpret_cast<const bf16x8 *>(X + size_t(smp) * MLP_IN + 8 * q);
                } else {
                    const float4 x0 = *reinterpret_cast<const float4 *>(X + size_t(smp) * MLP_IN + 8 * q);
                    const float4 x1 = *reinterpret_cast<const float4 *>(X + size_t(smp) * MLP_IN + 8 * q + 4);
                    v[0] = __bf16(x0.x); v[1] = __bf16(x0.y); v[2] = __bf16(x0.z); v[3] = __bf16(x0.w);
                    v[4] = __bf16(x1.x); v[5] = __bf16(x1.y); v[6] = __bf16(x1.z); v[7] = __bf16(x1.w);
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = __bf16(0.0f);
            }
            act[p][0] = v;
        }
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int nc = l == 0 ? MLP_IN / 32 : NC, ld = l == 0 ? Z::L1 : Z::LH, wb = l == 0 ? Z::W1 : (l == 1 ? Z::W2 : Z::W3);
            f32x4 acc[TP][NT];
            // the products accumulate onto the bias (no separate add in the epilogue)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const float4 bias = *reinterpret_cast<const float4 *>(sb + l * H + 16 * nt + 4 * q);
#pragma unroll
                for (int p = 0; p < TP; ++p) acc[p][nt] = f32x4{bias.x, bias.y, bias.z, bias.w};
            }
#pragma unroll
            for (int c = 0; c < nc; ++c) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(sw + wb + (16 * nt + r) * ld + 32 * c + 8 * q);
#pragma unroll
                    for (int p = 0; p < TP; ++p)
                        acc[p][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, act[p][c], acc[p][nt], 0, 0, 0);
                }
            }
#pragma unroll
            for (int p = 0; p < TP; ++p)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    bf16x4 lo, hi;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        lo[i] = __bf16(silu(acc[p][2 * c][i]));
                        hi[i] = __bf16(silu(acc[p][2 * c + 1][i]));
                    }
                    act[p][c] = chunk_operand(lo, hi);
                }
        }
        f32x4 out[TP];
        {
            // output rows 8..15 of the product are padding with zero bias
            const float4 bias = *reinterpret_cast<const float4 *>(sb + 3 * H + 4 * q);
#pragma unroll
            for (int p = 0; p < TP; ++p) out[p] = f32x4{bias.x, bias.y, bias.z, bias.w};
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(sw + Z::W4 + r * Z::LH + 32 * c + 8 * q);
#pragma unroll
            for (int p = 0; p < TP; ++p) out[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, act[p][c], out[p], 0, 0, 0);
        }
#pragma unroll
        for (int p = 0; p < TP; ++p) {
            const int s0 = (t0 + p) * 16;
            if (q < 2 && s0 + r < n) {
                const float4 y = make_float4(out[p][0], out[p][1], out[p][2], out[p][3]);
                *reinterpret_cast<float4 *>(Y + size_t(s0 + r) * MLP_OUT + 4 * q) = y;
            }
        }
    }
}

// ------------------------------------------------------------------------------------------------
// generic product for the backward pass: C[M x N] = A[M x K] B[K x N] (+ C when ACC), element (m, k)
// of A at A[m * am + k * ak], element (k, n) of B at B[k * bk + n * bn]; rows/cols/k beyond the sizes
// read as 0. One workgroup of four waves per 32 x 32 tile of C, each wave one 16 x 16 quarter. For every
// 32-wide slice of K the workgroup stages the A and B tiles in LDS, loading along whichever axis of each
// operand is contiguous in memory (so a wave's loads are coalesced whatever the transposition), and each
// wave then forms its quarter from LDS: one MFMA per slice, or (FP32 reference mode) one FMA chain per
// output in ascending k.
constexpr int GT = 32;  // tile edge and K slice of k_gemm

template <bool MFMA, bool ACC>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float *__restrict__ A, long am, long ak,
                                              const float *__restrict__ B, long bk, long bn, float *__restrict__ C,
                                              long ldc) {
    __shared__ float sA[GT][GT + 1];  // [m][k]
    __shared__ float sB[GT][GT + 1];  // [k][n]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, r = lane & 15;
    const int tiles_n = (N + GT - 1) / GT;
    const int m0 = int(blockIdx.x) / tiles_n * GT, n0 = int(blockIdx.x) % tiles_n * GT;
    const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
    const bool a_k_fast = ak == 1, b_n_fast = bn == 1;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += GT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int fast = tid & 31, slow = (tid >> 5) + 8 * i;
            const int ta = a_k_fast ? slow : fast, ka = a_k_fast ? fast : slow;  // A tile row m, column k
            const int gm = m0 + ta, gka = k0 + ka;
            sA[ta][ka] = (gm < M && gka < K) ? A[gm * am + gka * ak] : 0.0f;
            const int tb = b_n_fast ? fast : slow, kb = b_n_fast ? slow : fast;  // B tile column n, row k
            const int gn = n0 + tb, gkb = k0 + kb;
            sB[kb][tb] = (gn < N && gkb < K) ? B[gkb * bk + gn * bn] : 0.0f;
        }
        __syncthreads();
        if constexpr (MFMA) {
            bf16x8 av, bv;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                av[j] = __bf16(sA[wm + r][8 * q + j]);
                bv[j] = __bf16(sB[8 * q + j][wn + r]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        } else {
            const int kend = K - k0 < GT ? K - k0 : GT;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                for (int kk = 0; kk < kend; ++kk) acc[i] = fmaf(sA[wm + 4 * q + i][kk], sB[kk][wn + r], acc[i]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm + 4 * q + i, n = n0 + wn + r;
        if (m < M && n < N) {
            float *c = C + m * ldc + n;
            *c = ACC ? *c + acc[i] : acc[i];
        }
    }
}

// dY = 2 (Y - T) / (8 n); also the per-sample squared error (for the loss)
__global__ void k_loss_grad(int n, const float *__restrict__ Y, const float *__restrict__ Tt, float *__restrict__ dY,
                            float *__restrict__ sqerr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * MLP_OUT) return;
    const float d = Y[i] - Tt[i];
    dY[i] = 2.0f * d / (8.0f * float(n));
    sqerr[i] = d * d;
}

// dZ = dA * silu'(Z), elementwise over n x H
__global__ void k_silu_back(long count, const float *__restrict__ dA, const float *__restrict__ Z, float *__restrict__ dZ) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) dZ[i] = dA[i] * silu_grad(Z[i]);
}

// A = silu(Z), elementwise
__global__ void k_silu(long count, const float *__restrict__ Z, float *__restrict__ A) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) A[i] = silu(Z[i]);
}

// column sums of G[n][cols] into out[cols]: one workgroup of 1,024 threads per 64 columns; thread (c, p)
// sums the rows p, p + 16, ... of column c in ascending order (a wave reads 64 neighbouring columns of
// one row), then the 16 partial sums of a column are added pairwise in LDS (fixed tree: deterministic)
constexpr int CS_PHASES = 16;

__global__ void __launch_bounds__(1024) k_colsum(int n, int cols, const float *__restrict__ G, float *__restrict__ out) {
    __shared__ float part[CS_PHASES][64];
    const int tx = threadIdx.x & 63, p = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + tx;
    float s = 0.f;
    if (c < cols)
        for (int i = p; i < n; i += CS_PHASES) s += G[size_t(i) * cols + c];
    part[p][tx] = s;
    __syncthreads();
#pragma unroll
    for (int h = CS_PHASES / 2; h > 0; h >>= 1) {
        if (p < h) part[p][tx] += part[p + h][tx];
        __syncthreads();
    }
    if (p == 0 && c < cols) out[c] = part[0][tx];
}

// Adam on the FP32 master vector; refreshes the BF16 copy
__global__ void k_adam(long np, float *__restrict__ p, __bf16 *__restrict__ pb, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = __bf16(pi);
}

__global__ void k_to_bf16(long np, const float *__restrict__ p, __bf16 *__restrict__ pb) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < np) pb[i] = __bf16(p[i]);
}

// Scratch of bmhd_mlp_backward_noalloc, laid out like bmhd_mlp_backward's d_work (dY in the first n x 16
// floats, then two [n][H] gradient buffers); every element the backward pass reads it has written first. Every device the library runs on holds its own
// copy until the process ends. Host code never passes `scratch` itself to a kernel: it passes the
// device address hipGetSymbolAddress returns for the current device.
constexpr size_t MLP_SCRATCH_FLOATS = size_t(8) << 20;  // 32 MiB
static __device__ __align__(256) float scratch[MLP_SCRATCH_FLOATS];

}  // namespace bmhd

// ================================================================================================
// C ABI

using namespace bmhd;

namespace {
thread_local std::string m_err;
int32_t mfail(int32_t code, const char *msg) {
    m_err = msg;
    return code;
}
int32_t mcheck(const char *what) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return BMHD_OK;
    m_err = std::string(what) + ": " + hipGetErrorString(e);
    return BMHD_EHIP;
}
unsigned blocks_for(long n, int t) { return unsigned((n + t - 1) / t); }

template <bool MFMA>
void gemm(int M, int N, int K, const float *A, long am, long ak, const float *B, long bk, long bn, float *C, long ldc,
          bool acc, hipStream_t s) {
    const unsigned tiles = unsigned((M + GT - 1) / GT) * unsigned((N + GT - 1) / GT);
    if (tiles == 0) return;
    if (acc) k_gemm<MFMA, true><<<tiles, 256, 0, s>>>(M, N, K, A, am, ak, B, bk, bn, C, ldc);
    else k_gemm<MFMA, false><<<tiles, 256, 0, s>>>(M, N, K, A, am, ak, B, bk, bn, C, ldc);
}

// BF16 inference: persistent, one workgroup per CU
template <int H, typename TX>
int32_t infer_h(const float *P, const uint16_t *Pb, int n, const TX *X, float *Y, hipStream_t s) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    const unsigned tiles = unsigned((n + 15) / 16);
    const unsigned per = MLP_INFER_WAVES * MLP_INFER_TILES;
    const unsigned g = tiles < per * unsigned(cus) ? blocks_for(tiles, int(per)) : unsigned(cus);
    k_mlp_infer<H, MLP_INFER_WAVES, MLP_INFER_TILES, TX><<<g, 64 * MLP_INFER_WAVES, 0, s>>>(
        P, reinterpret_cast<const __bf16 *>(Pb), n, X, Y);
    return mcheck("mlp inference");
}

template <int H>
int32_t forward_h(const float *P, const uint16_t *Pb, int n, const float *X, float *Y, float *Z, int mode, hipStream_t s) {
    const unsigned grid = blocks_for((n + 15) / 16, 4);
    const __bf16 *pb = reinterpret_cast<const __bf16 *>(Pb);
    if (mode == 0 && !Z) return infer_h<H, float>(P, Pb, n, X, Y, s);
    if (mode == 0) k_mlp_forward<H, true><<<grid, 256, 0, s>>>(P, pb, n, X, Y, Z);
    else k_mlp_forward<H, false><<<grid, 256, 0, s>>>(P, pb, n, X, Y, Z);
    return mcheck("mlp forward");
}

// Device address of `scratch` on the current device, looked up once per device (with that device
// current) and kept: the symbol's host-side name is not a device address.
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_dev[MAX_DEVICES] = {};

int32_t scratch_address(float **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return mfail(BMHD_EHIP, "mlp_backward_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= MAX_DEVICES) return mfail(BMHD_EUNSUPPORTED, "mlp_backward_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mfail(BMHD_EHIP, (std::string("mlp_backward_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e)).c_str());
        scratch_dev[dev] = static_cast<float *>(p);
    }
    *out = scratch_dev[dev];
    return BMHD_OK;
}

// Backward pass on a caller-supplied work area (bmhd_mlp_work_bytes(hidden, n) bytes); arguments checked
// by the caller.
int32_t backward_impl(const float *d_params, int32_t hidden, int32_t n, const float *d_x, const float *d_t,
                      const float *d_save, const float *d_y, float *d_grad, float *d_sqerr, float *d_work,
                      int32_t mode, void *stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int H = hidden;
    const MlpView V = mlp_view(H);
    float *dY = d_work;                                  // [n][8]
    float *bufA = d_work + size_t(n) * 16;               // [n][H]
    float *bufB = bufA + size_t(n) * H;                  // [n][H]
    const bool mf = mode == 0;
    auto G = [&](int M, int N, int K, const float *A, long am, long ak, const float *B, long bk, long bn, float *C,
                 long ldc) {
        if (mf) gemm<true>(M, N, K, A, am, ak, B, bk, bn, C, ldc, false, s);
        else gemm<false>(M, N, K, A, am, ak, B, bk, bn, C, ldc, false, s);
    };
    k_loss_grad<<<blocks_for(long(n) * 8, 256), 256, 0, s>>>(n, d_y, d_t, dY, d_sqerr);
    // layer 4: dW4[o][i] = sum_n dY[n][o] A3[n][i], db4 = sum_n dY, dA3 = dY W4
    float *A3 = bufB;
    k_silu<<<blocks_for(long(n) * H, 256), 256, 0, s>>>(long(n) * H, d_save + size_t(2) * n * H, A3);
    G(8, H, n, dY, 1, 8, A3, H, 1, d_grad + V.off_w[3], H);
    k_colsum<<<1, 1024, 0, s>>>(n, 8, dY, d_grad + V.off_b[3]);
    float *dA = bufA, *other = bufB;
    G(n, H, 8, dY, 8, 1, d_params + V.off_w[3], H, 1, dA, H);
    // hidden layers 3, 2, 1 (index l = 2, 1, 0)
    for (int l = 2; l >= 0; --l) {
        const float *Z = d_save + size_t(l) * n * H;
        float *dZ = dA;  // in place: dZ overwrites dA
        k_silu_back<<<blocks_for(long(n) * H, 256), 256, 0, s>>>(long(n) * H, dA, Z, dZ);
        const int nin = V.nin[l];
        if (l > 0) {
            float *Ain = other;
            k_silu<<<blocks_for(long(n) * H, 256), 256, 0, s>>>(long(n) * H, d_save + size_t(l - 1) * n * H, Ain);
            G(H, nin, n, dZ, 1, H, Ain, H, 1, d_grad + V.off_w[l], nin);
        } else {
            G(H, nin, n, dZ, 1, H, d_x, MLP_IN, 1, d_grad + V.off_w[l], nin);
        }
        k_colsum<<<blocks_for(H, 64), 1024, 0, s>>>(n, H, dZ, d_grad + V.off_b[l]);
        if (l > 0) {
            // dA_{l-1}[n][i] = sum_o dZ[n][o] W_l[o][i], into the buffer the inputs no longer need
            G(n, nin, H, dZ, H, 1, d_params + V.off_w[l], nin, 1, other, nin);
            float *t = dA;
            dA = other;
            other = t;
        }
    }
    return mcheck("mlp backward");
}
}  // namespace

namespace bmhd {
int32_t mlp_infer_bf16_inputs(
const float *d_params, const uint16_t *d_params_bf16, int32_t hidden, int32_t n,
                              const uint16_t *d_x, float *d_y, void *stream, std::string &err) {
    if (!d_params || !d_params_bf16 || !d_x || !d_y || n < 0 || (reinterpret_cast<uintptr_t>(d_x) & 15u)) {
        err = "mlp inference: null or misaligned buffers";
        return BMHD_EINVAL;
    }
    if (n == 0) return BMHD_OK;
    const __bf16 *x = reinterpret_cast<const __bf16 *>(d_x);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t rc;
    switch (hidden) {
        case 32: rc = infer_h<32, __bf16>(d_params, d_params_bf16, n, x, d_y, s); break;
        case 64: rc = infer_h<64, __bf16>(d_params, d_params_bf16, n, x, d_y, s); break;
        case 128: rc = infer_h<128, __bf16>(d_params, d_params_bf16, n, x, d_y, s); break;
        default: err = "mlp inference: hidden must be 32, 64 or 128"; return BMHD_EUNSUPPORTED;
    }
    if (rc) err = m_err;
    return rc;
}
}  // namespace bmhd

extern "C" {

const char *bmhd_mlp_last_error(void) { return m_err.c_str(); }

int64_t bmhd_mlp_n_params(int32_t hidden) { return mlp_params(hidden); }

size_t bmhd_mlp_work_bytes(int32_t hidden, int32_t n) {
    // dY, squared errors [n][8]; two [n][H] gradient buffers
    return sizeof(float) * (size_t(n) * 16 + 2 * size_t(n) * hidden);
}

int32_t bmhd_mlp_forward(const float *d_params, const uint16_t *d_params_bf16, int32_t hidden, int32_t n,
                         const float *d_x, float *d_y, float *d_save, int32_t mode, void *stream) {
    if (!d_params || !d_params_bf16 || !d_x || !d_y || n < 0 || (mode != 0 && mode != 1))
        return mfail(BMHD_EINVAL, "mlp_forward: bad arguments");
    if (n == 0) return BMHD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch (hidden) {
        case 32: return forward_h<32>(d_params, d_params_bf16, n, d_x, d_y, d_save, mode, s);
        case 64: return forward_h<64>(d_params, d_params_bf16, n, d_x, d_y, d_save, mode, s);
        case 128: return forward_h<128>(d_params, d_params_bf16, n, d_x, d_y, d_save, mode, s);
        default: return mfail(BMHD_EUNSUPPORTED, "mlp_forward: hidden must be 32, 64 or 128");
    }
}

int32_t bmhd_mlp_backward(const float *d_params, int32_t hidden, int32_t n, const float *d_x, const float *d_t,
                          const float *d_save, const float *d_y, float *d_grad, float *d_sqerr, float *d_work,
                          int32_t mode, void *stream) {
    if (!d_params || !d_x || !d_t || !d_save || !d_y || !d_grad || !d_sqerr || !d_work || n <= 0 ||
        (mode != 0 && mode != 1))
        return mfail(BMHD_EINVAL, "mlp_backward: bad arguments");
    if (hidden != 32 && hidden != 64 && hidden != 128) return mfail(BMHD_EUNSUPPORTED, "hidden must be 32, 64 or 128");
    return backward_impl(d_params, hidden, n, d_x, d_t, d_save, d_y, d_grad, d_sqerr, d_work, mode, stream);
}

int32_t bmhd_mlp_backward_noalloc(const float *d_params, int32_t hidden, int32_t n, const float *d_x,
                                  const float *d_t, const float *d_save, const float *d_y, float *d_grad,
                                  float *d_sqerr, int32_t mode, void *stream) {
    if (!d_params || !d_x || !d_t || !d_save || !d_y || !d_grad || !d_sqerr || n <= 0 || (mode != 0 && mode != 1))
        return mfail(BMHD_EINVAL, "mlp_backward_noalloc: bad arguments");
    if (hidden != 32 && hidden != 64 && hidden != 128) return mfail(BMHD_EUNSUPPORTED, "hidden must be 32, 64 or 128");
    const size_t need = bmhd_mlp_work_bytes(hidden, n) / sizeof(float);
    if (need > MLP_SCRATCH_FLOATS) {
        const size_t max_n = MLP_SCRATCH_FLOATS / (16 + 2 * size_t(hidden));
        return mfail(BMHD_EINVAL, ("mlp_backward_noalloc: n = " + std::to_string(n) + " exceeds the static scratch (" +
                                   std::to_string(max_n) + " samples at hidden " + std::to_string(hidden) + ")").c_str());
    }
    float *work = nullptr;
    if (int32_t rc = scratch_address(&work)) return rc;
    return backward_impl(d_params, hidden, n, d_x, d_t, d_save, d_y, d_grad, d_sqerr, work, mode, stream);
}

int32_t bmhd_mlp_adam(float *d_params, uint16_t *d_params_bf16, float *d_m, float *d_v, const float *d_grad,
                      int64_t n_params, float lr, float b1, float b2, float eps, int32_t t, void *stream) {
    if (!d_params || !d_params_bf16 || !d_m || !d_v || !d_grad || n_params <= 0 || t < 1)
        return mfail(BMHD_EINVAL, "mlp_adam: bad arguments");
    const float c1 = 1.0f - powf(b1, float(t)), c2 = 1.0f - powf(b2, float(t));
    k_adam<<<blocks_for(n_params, 256), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        n_params, d_params, reinterpret_cast<__bf16 *>(d_params_bf16), d_m, d_v, d_grad, lr, b1, b2, eps, c1, c2);
    return mcheck("mlp adam");
}

int32_t bmhd_mlp_to_bf16(const float *d_params, uint16_t *d_params_bf16, int64_t n_params, void *stream) {
    if (!d_params || !d_params_bf16 || n_params <= 0) return mfail(BMHD_EINVAL, "mlp_to_bf16: bad arguments");
    k_to_bf16<<<blocks_for(n_params, 256), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
        n_params, d_params, reinterpret_cast<__bf16 *>(d_params_bf16));
    return mcheck("mlp to bf16");
}

}  // extern "C"
