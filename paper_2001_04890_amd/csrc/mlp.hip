// Learned Davidson preconditioner: kernels of the per-coefficient MLP (HIP, gfx950).
//
// Network (one MLP shared by all psi coefficients, 16 features per coefficient, see k_mlp_features):
//   h1 = relu(x W1 + b1)   W1 16 x 256
//   h2 = relu(h1 W2 + b2)  W2 256 x 256
//   m  = h2 . w3 + b3
// and the correction of Davidson's method becomes t_i = t_diag_i (1 + m_i), with t_diag the
// diagonal correction r / (theta - D) (Sections 2.1, 2.2.1). A network with w3 = b3 = 0 is exactly
// the diagonal preconditioner.
//
// Precision. The master parameters are FP32 (Adam state too). Inference and training use BF16
// copies of W1 and W2 on the matrix cores with FP32 accumulation (k_mlp_fwd_mfma); a debug mode runs
// the same network from the FP32 parameters on the vector units (k_mlp_fwd_f32).
//
// MFMA forward. One wavefront owns 64 rows (4 row tiles of 16). Both layers are computed transposed,
// H^T = W^T X^T, so the rows of the data are the N dimension of v_mfma_f32_16x16x32_bf16: after
// layer 1 lane l holds units 16u + 4(l/16) + v (v = 0..3) of row l%16 of every row tile, which is
// the B-operand layout of layer 2 once layer 2's reduction index is permuted the same way
// (slot s of lane group g in k-step q <-> unit 32q + 16(s/4) + 4g + s%4). W1 and W2 are stored
// pre-permuted (k_mlp_pack) so every A fragment is one 16-byte load, and layer 1's output never
// leaves the registers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.h"

namespace dmrg {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// float -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t pack2(float a, float b) {
    return (uint32_t)f32_to_bf16_bits(a) | ((uint32_t)f32_to_bf16_bits(b) << 16);
}

__device__ __forceinline__ f32x4 mfma_bf16(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}

unsigned grid_of(int64_t n, int per) {
    int64_t b = (n + per - 1) / per;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// ------------------------------------------------------------------ features
// Per chunk of one psi block: sum r^2 and u^2 (deterministic tree reduction).
__global__ __launch_bounds__(256) void k_mlp_block_sums(const MlpChunk* __restrict__ chunks, const double* __restrict__ r,
                                                        const double* __restrict__ u, double* __restrict__ part) {
    __shared__ double s0[256], s1[256];
    const MlpChunk C = chunks[blockIdx.x];
    double sr = 0.0, su = 0.0;
    for (int64_t i = C.begin + threadIdx.x; i < C.end; i += blockDim.x) {
        sr += r[i] * r[i];
        su += u[i] * u[i];
    }
    s0[threadIdx.x] = sr;
    s1[threadIdx.x] = su;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// Features of every coefficient of one chunk (layout in mlp.h).
__global__ __launch_bounds__(256) void k_mlp_features(const MlpChunk* __restrict__ chunks,
                                                      const MlpBlockInfo* __restrict__ blocks,
                                                      const double* __restrict__ part, const double* __restrict__ r,
                                                      const double* __restrict__ t, const double* __restrict__ u,
                                                      const double* __restrict__ d, double theta, MlpScales sc,
                                                      float* __restrict__ feat) {
    const MlpChunk C = chunks[blockIdx.x];
    const MlpBlockInfo B = blocks[C.block];
    double sr = 0.0, su = 0.0;
    for (int k = B.chunk_begin; k < B.chunk_end; ++k) {
        sr += part[2 * k];
        su += part[2 * k + 1];
    }
    const double cnt = (double)B.m_a * (double)B.m_d;
    const float f12 = (float)asinh(sqrt(sr / cnt) * sc.inv_r);
    const float f13 = (float)asinh(sqrt(su / cnt) * sc.inv_u);
    float oh[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        oh[k] = B.b == k ? 1.f : 0.f;
        oh[4 + k] = B.c == k ? 1.f : 0.f;
    }
    for (int64_t i = C.begin + threadIdx.x; i < C.end; i += blockDim.x) {
        float4* f = reinterpret_cast<float4*>(feat + i * kMlpIn);
        f[0] = make_float4((float)asinh(r[i] * sc.inv_r), (float)asinh(t[i] * sc.inv_t), (float)asinh(u[i] * sc.inv_u),
                           (float)asinh((d[i] - theta) * sc.inv_dt));
        f[1] = make_float4(oh[0], oh[1], oh[2], oh[3]);
        f[2] = make_float4(oh[4], oh[5], oh[6], oh[7]);
        f[3] = make_float4(f12, f13, B.lma, B.lmd);
    }
}

// out[k][:] = in[idx[k]][:] (cols floats per row)
__global__ void k_mlp_gather(const float* __restrict__ in, const int64_t* __restrict__ idx, int64_t n, int cols,
                             float* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n * cols; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = k / cols, c = k - row * cols;
        out[k] = in[idx[row] * cols + c];
    }
}

// Training pairs of one recorded iteration at sampled coefficients i = idx[k]: a = sa t_i, b = sb v_i,
// weight w.
__global__ void k_mlp_pairs(const double* __restrict__ t, const double* __restrict__ v, const int64_t* __restrict__ idx,
                            int64_t n, double sa, double sb, float w, float* __restrict__ aux) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[k];
        aux[3 * k] = (float)(sa * t[i]);
        aux[3 * k + 1] = (float)(sb * v[i]);
        aux[3 * k + 2] = w;
    }
}

// ------------------------------------------------------------------ weights
// BF16 copies: W1p / W2p in the MFMA fragment order described at the top, w2 row-major.
__global__ void k_mlp_pack(const float* __restrict__ p, uint16_t* __restrict__ w1p, uint16_t* __restrict__ w2p,
                           uint16_t* __restrict__ w2) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < kMlpHidden * kMlpHidden) {
        // W2p[((o*8 + q)*64 + l)*8 + s] = W2[32q + 16(s/4) + 4(l/16) + s%4][16o + l%16]
        const int s = (int)(e & 7), l = (int)((e >> 3) & 63), q = (int)((e >> 9) & 7), o = (int)(e >> 12);
        const int g = l >> 4, c = l & 15;
        const int kin = 32 * q + 16 * (s >> 2) + 4 * g + (s & 3);
        w2p[e] = f32_to_bf16_bits(p[kOffW2 + kin * kMlpHidden + 16 * o + c]);
        w2[e] = f32_to_bf16_bits(p[kOffW2 + e]);
    }
    if (e < 16 * 64 * 8) {
        // W1p[(u*64 + l)*8 + s] = W1[8(l/16) + s][16u + l%16] for l/16 < 2, else 0 (K padded to 32)
        const int s = (int)(e & 7), l = (int)((e >> 3) & 63), uu = (int)(e >> 9);
        const int g = l >> 4, c = l & 15;
        w1p[e] = g < 2 ? f32_to_bf16_bits(p[(8 * g + s) * kMlpHidden + 16 * uu + c]) : (uint16_t)0;
    }
}

// ------------------------------------------------------------------ forward (BF16, matrix cores)
template <bool TRAIN>
__global__ __launch_bounds__(64) void k_mlp_fwd_mfma(const MlpDev W, const float* __restrict__ feat, int64_t n,
                                                     float* __restrict__ out, float* __restrict__ h1o,
                                                     float* __restrict__ h2o, double* __restrict__ t_apply) {
    const int l = threadIdx.x, g = l >> 4, c = l & 15;
    const int64_t row0 = (int64_t)blockIdx.x * 64;
    // layer-1 B operand (X^T, K padded to 32): lane holds X[row][8g .. 8g+7] for g < 2
    u32x4 xb[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int64_t row = row0 + 16 * rt + c;
        xb[rt] = u32x4{0u, 0u, 0u, 0u};
        if (g < 2 && row < n) {
            const float4* src = reinterpret_cast<const float4*>(feat + row * kMlpIn + 8 * g);
            const float4 a = src[0], b = src[1];
            xb[rt] = u32x4{pack2(a.x, a.y), pack2(a.z, a.w), pack2(b.x, b.y), pack2(b.z, b.w)};
        }
    }
    const u32x4* w1p = reinterpret_cast<const u32x4*>(W.w1p);
    const u32x4* w2p = reinterpret_cast<const u32x4*>(W.w2p);
    const float4* b1v = reinterpret_cast<const float4*>(W.p + kOffB1);
    const float4* b2v = reinterpret_cast<const float4*>(W.p + kOffB2);
    const float4* w3v = reinterpret_cast<const float4*>(W.p + kOffW3);
    // layer 1 -> h1 as BF16 pairs: h1p[u][rt] = units 16u + 4g + {0,1 | 2,3} of row 16rt + c
    uint32_t h1p[16][4][2];
#pragma unroll
    for (int uu = 0; uu < 16; ++uu) {
        const u32x4 a = w1p[uu * 64 + l];
        const float4 bb = b1v[4 * uu + g];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            f32x4 acc = mfma_bf16(a, xb[rt], f32x4{0.f, 0.f, 0.f, 0.f});
            const float h0 = fmaxf(acc[0] + bb.x, 0.f), h1 = fmaxf(acc[1] + bb.y, 0.f);
            const float h2 = fmaxf(acc[2] + bb.z, 0.f), h3 = fmaxf(acc[3] + bb.w, 0.f);
            h1p[uu][rt][0] = pack2(h0, h1);
            h1p[uu][rt][1] = pack2(h2, h3);
            if (TRAIN) {
                const int64_t row = row0 + 16 * rt + c;
                if (row < n) *reinterpret_cast<float4*>(h1o + row * kMlpHidden + 16 * uu + 4 * g) = make_float4(h0, h1, h2, h3);
            }
        }
    }
    // layer 2 and the output dot product
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int o = 0; o < 16; ++o) {
        f32x4 acc[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const u32x4 a = w2p[(o * 8 + q) * 64 + l];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const u32x4 b = u32x4{h1p[2 * q][rt][0], h1p[2 * q][rt][1], h1p[2 * q + 1][rt][0], h1p[2 * q + 1][rt][1]};
                acc[rt] = mfma_bf16(a, b, acc[rt]);
            }
        }
        const float4 bb = b2v[4 * o + g];
        const float4 ww = w3v[4 * o + g];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const float h0 = fmaxf(acc[rt][0] + bb.x, 0.f), h1 = fmaxf(acc[rt][1] + bb.y, 0.f);
            const float h2 = fmaxf(acc[rt][2] + bb.z, 0.f), h3 = fmaxf(acc[rt][3] + bb.w, 0.f);
            part[rt] += h0 * ww.x + h1 * ww.y + h2 * ww.z + h3 * ww.w;
            if (TRAIN) {
                const int64_t row = row0 + 16 * rt + c;
                if (row < n) *reinterpret_cast<float4*>(h2o + row * kMlpHidden + 16 * o + 4 * g) = make_float4(h0, h1, h2, h3);
            }
        }
    }
    const float b3 = W.p[kOffB3];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        float v = part[rt];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int64_t row = row0 + 16 * rt + c;
        if (g == 0 && row < n) {
            const float m = v + b3;
            if (out) out[row] = m;
            if (t_apply) t_apply[row] *= 1.0 + (double)m;
        }
    }
}

// ------------------------------------------------------------------ forward (FP32 debug mode)
// 64 rows per workgroup of 256 threads; thread j owns hidden unit j of both layers.
constexpr int kRows = 64;

template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_fwd_f32(const MlpDev W, const float* __restrict__ feat, int64_t n,
                                                     float* __restrict__ out, float* __restrict__ h1o,
                                                     float* __restrict__ h2o, double* __restrict__ t_apply) {
    __shared__ float X[kRows][kMlpIn + 1];
    __shared__ float H1[kRows][kMlpHidden + 1];
    __shared__ float R[kRows][4];
    const int j = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * kRows;
    for (int e = j; e < kRows * kMlpIn; e += blockDim.x) {
        const int r = e / kMlpIn, c = e % kMlpIn;
        X[r][c] = row0 + r < n ? feat[(row0 + r) * kMlpIn + c] : 0.f;
    }
    float w1[kMlpIn];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) w1[k] = W.p[k * kMlpHidden + j];
    const float b1 = W.p[kOffB1 + j], b2 = W.p[kOffB2 + j], w3 = W.p[kOffW3 + j];
    __syncthreads();
    for (int r = 0; r < kRows; ++r) {
        float z = b1;
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) z += X[r][k] * w1[k];
        const float h = fmaxf(z, 0.f);
        H1[r][j] = h;
        if (TRAIN && row0 + r < n) h1o[(row0 + r) * kMlpHidden + j] = h;
    }
    __syncthreads();
    const int wave = j >> 6, lane = j & 63;
    for (int r = 0; r < kRows; ++r) {
        float z = b2;
        for (int k = 0; k < kMlpHidden; ++k) z += H1[r][k] * W.p[kOffW2 + k * kMlpHidden + j];
        const float h = fmaxf(z, 0.f);
        if (TRAIN && row0 + r < n) h2o[(row0 + r) * kMlpHidden + j] = h;
        float v = h * w3;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) R[r][wave] = v;
    }
    __syncthreads();
    if (j < kRows && row0 + j < n) {
        const float m = W.p[kOffB3] + R[j][0] + R[j][1] + R[j][2] + R[j][3];
        if (out) out[row0 + j] = m;
        if (t_apply) t_apply[row0 + j] *= 1.0 + (double)m;
    }
}

// ------------------------------------------------------------------ backward
// loss = (1/B) sum_r w_r (a_r (1 + m_r) - b_r)^2 over the B rows of the minibatch.
// Per row: g = dloss/dm, d2 = g w3 [h2 > 0], d1 = (d2 W2^T) [h1 > 0]; thread j owns unit j.
__global__ __launch_bounds__(256) void k_mlp_backward(const MlpDev W, const float* __restrict__ aux,
                                                      const float* __restrict__ m, const float* __restrict__ h1,
                                                      const float* __restrict__ h2, int64_t n, float inv_b,
                                                      float* __restrict__ g_out, float* __restrict__ d1,
                                                      float* __restrict__ d2, float* __restrict__ loss_part) {
    __shared__ float D2[kRows][kMlpHidden + 1];
    __shared__ float G[kRows];
    __shared__ float Lp[kRows];
    const int j = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * kRows;
    if (j < kRows) {
        float gg = 0.f, ll = 0.f;
        if (row0 + j < n) {
            const float a = aux[3 * (row0 + j)], b = aux[3 * (row0 + j) + 1], w = aux[3 * (row0 + j) + 2];
            const float e = a * (1.f + m[row0 + j]) - b;
            gg = 2.f * inv_b * w * a * e;
            ll = inv_b * w * e * e;
            g_out[row0 + j] = gg;
        }
        G[j] = gg;
        Lp[j] = ll;
    }
    const float w3 = W.p[kOffW3 + j];
    __syncthreads();
    for (int r = 0; r < kRows; ++r) {
        const int64_t row = row0 + r;
        float v = 0.f;
        if (row < n) {
            v = h2[row * kMlpHidden + j] > 0.f ? G[r] * w3 : 0.f;
            d2[row * kMlpHidden + j] = v;
        }
        D2[r][j] = v;
    }
    __syncthreads();
    for (int r = 0; r < kRows; ++r) {
        const int64_t row = row0 + r;
        if (row >= n) break;
        float s = 0.f;
        if (W.fp32) {
            for (int q = 0; q < kMlpHidden; ++q) s += D2[r][q] * W.p[kOffW2 + j * kMlpHidden + q];
        } else {
            for (int q = 0; q < kMlpHidden; ++q) s += D2[r][q] * bf16_bits_to_f32(W.w2[j * kMlpHidden + q]);
        }
        d1[row * kMlpHidden + j] = h1[row * kMlpHidden + j] > 0.f ? s : 0.f;
    }
    if (j == 0) {
        float s = 0.f;
        for (int r = 0; r < kRows; ++r) s += Lp[r];
        loss_part[blockIdx.x] = s;
    }
}

// Parameter gradients, each a sum over the minibatch rows in row order:
//   dW1[k][j] = sum_r x[r][k] d1[r][j], db1 = sum d1, dW2[k][j] = sum_r h1[r][k] d2[r][j], db2 = sum d2,
//   dw3[j] = sum_r g[r] h2[r][j], db3 = sum g.
__global__ void k_mlp_wgrad(const float* __restrict__ x, const float* __restrict__ h1, const float* __restrict__ h2,
                            const float* __restrict__ d1, const float* __restrict__ d2, const float* __restrict__ g,
                            int64_t n, float* __restrict__ grad) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float s = 0.f;
    if (p < kOffB1) {
        const int k = (int)(p / kMlpHidden), jj = (int)(p % kMlpHidden);
        for (int64_t r = 0; r < n; ++r) s += x[r * kMlpIn + k] * d1[r * kMlpHidden + jj];
    } else if (p < kOffW2) {
        const int jj = (int)(p - kOffB1);
        for (int64_t r = 0; r < n; ++r) s += d1[r * kMlpHidden + jj];
    } else if (p < kOffB2) {
        const int k = (int)((p - kOffW2) / kMlpHidden), jj = (int)((p - kOffW2) % kMlpHidden);
        for (int64_t r = 0; r < n; ++r) s += h1[r * kMlpHidden + k] * d2[r * kMlpHidden + jj];
    } else if (p < kOffW3) {
        const int jj = (int)(p - kOffB2);
        for (int64_t r = 0; r < n; ++r) s += d2[r * kMlpHidden + jj];
    } else if (p < kOffB3) {
        const int jj = (int)(p - kOffW3);
        for (int64_t r = 0; r < n; ++r) s += g[r] * h2[r * kMlpHidden + jj];
    } else {
        for (int64_t r = 0; r < n; ++r) s += g[r];
    }
    grad[p] = s;
}

// Adam (bias-corrected moments) on the FP32 parameters.
__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ m1,
                           float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= kMlpParams) return;
    const float gg = grad[i];
    const float a = b1 * m1[i] + (1.f - b1) * gg;
    const float v = b2 * m2[i] + (1.f - b2) * gg * gg;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// out[0] = sum of the per-workgroup partial losses (fixed order)
__global__ void k_mlp_sum(const float* __restrict__ v, int n, float* __restrict__ out) {
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += v[i];
        out[0] = s;
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_mlp_features(const MlpChunk* chunks, int n_chunks, const MlpBlockInfo* blocks, double* part,
                               const double* r, const double* t, const double* u, const double* d, double theta,
                               const MlpScales& sc, float* feat, hipStream_t s) {
    if (n_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_block_sums, dim3(n_chunks), dim3(256), 0, s, chunks, r, u, part);
    hipLaunchKernelGGL(k_mlp_features, dim3(n_chunks), dim3(256), 0, s, chunks, blocks, part, r, t, u, d, theta, sc,
                       feat);
    return hipGetLastError();
}

hipError_t launch_mlp_gather(const float* in, const int64_t* idx, int64_t n, int cols, float* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_gather, dim3(grid_of(n * cols, 256)), dim3(256), 0, s, in, idx, n, cols, out);
    return hipGetLastError();
}

hipError_t launch_mlp_pairs(const double* t, const double* v, const int64_t* idx, int64_t n, double sa, double sb,
                            float w, float* aux, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_pairs, dim3(grid_of(n, 256)), dim3(256), 0, s, t, v, idx, n, sa, sb, w, aux);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float* p, uint16_t* w1p, uint16_t* w2p, uint16_t* w2, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_pack, dim3(kMlpHidden * kMlpHidden / 256), dim3(256), 0, s, p, w1p, w2p, w2);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev& W, const float* feat, int64_t n, float* out, float* h1, float* h2,
                              double* t_apply, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const bool train = h1 != nullptr;
    if (W.fp32) {
        const unsigned nb = (unsigned)((n + kRows - 1) / kRows);
        if (train)
            hipLaunchKernelGGL(k_mlp_fwd_f32<true>, dim3(nb), dim3(256), 0, s, W, feat, n, out, h1, h2, t_apply);
        else
            hipLaunchKernelGGL(k_mlp_fwd_f32<false>, dim3(nb), dim3(256), 0, s, W, feat, n, out, h1, h2, t_apply);
    } else {
        const unsigned nb = (unsigned)((n + 63) / 64);
        if (train)
            hipLaunchKernelGGL(k_mlp_fwd_mfma<true>, dim3(nb), dim3(64), 0, s, W, feat, n, out, h1, h2, t_apply);
        else
            hipLaunchKernelGGL(k_mlp_fwd_mfma<false>, dim3(nb), dim3(64), 0, s, W, feat, n, out, h1, h2, t_apply);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpDev& W, const float* aux, const float* m, const float* h1, const float* h2,
                               int64_t n, float* g, float* d1, float* d2, float* loss_part, float* loss,
                               hipStream_t s) {
    const unsigned nb = (unsigned)((n + kRows - 1) / kRows);
    if (nb == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(256), 0, s, W, aux, m, h1, h2, n, 1.f / (float)n, g, d1, d2,
                       loss_part);
    hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(64), 0, s, loss_part, (int)nb, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_wgrad(const float* x, const float* h1, const float* h2, const float* d1, const float* d2,
                            const float* g, int64_t n, float* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, x, h1, h2, d1, d2, g, n, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, const float* grad, float* m1, float* m2, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, grad, m1, m2, lr, b1, b2, 1e-8f,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace dmrg

namespace dmrg {

// Sums of squares of r, u, t and D - theta (FP64, fixed-order reduction): part[4 * block + k], then
// out[k] = sum over blocks.
__global__ __launch_bounds__(256) void k_mlp_norms(const double* __restrict__ r, const double* __restrict__ u,
                                                   const double* __restrict__ t, const double* __restrict__ d,
                                                   double theta, int64_t n, double* __restrict__ part) {
    __shared__ double red[4][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double dd = d[i] - theta;
        s[0] += r[i] * r[i];
        s[1] += u[i] * u[i];
        s[2] += t[i] * t[i];
        s[3] += dd * dd;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = s[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        part[4 * blockIdx.x + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
    }
}

__global__ void k_mlp_norms_finish(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[4 * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Loss of rows (a, b, w) at outputs m (NULL: m = 0, the diagonal preconditioner): part[block] =
// sum of w (a (1 + m) - b)^2 over the block's rows (FP64, fixed order).
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ aux, const float* __restrict__ m, int64_t n,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double mm = m ? (double)m[i] : 0.0;
        const double e = (double)aux[3 * i] * (1.0 + mm) - (double)aux[3 * i + 1];
        s += (double)aux[3 * i + 2] * e * e;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_mlp_sum_f64(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        out[0] = s;
    }
}

int mlp_reduce_blocks(int64_t n) {
    int64_t b = (n + 4095) / 4096;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

hipError_t launch_mlp_norms(const double* r, const double* u, const double* t, const double* d, double theta,
                            int64_t n, double* part, double* out, hipStream_t s) {
    const int nb = mlp_reduce_blocks(n);
    hipLaunchKernelGGL(k_mlp_norms, dim3(nb), dim3(256), 0, s, r, u, t, d, theta, n, part);
    hipLaunchKernelGGL(k_mlp_norms_finish, dim3(1), dim3(64), 0, s, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float* aux, const float* m, int64_t n, double* part, double* out, hipStream_t s) {
    const int nb = mlp_reduce_blocks(n);
    hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, s, aux, m, n, part);
    hipLaunchKernelGGL(k_mlp_sum_f64, dim3(1), dim3(64), 0, s, part, nb, out);
    return hipGetLastError();
}

}  // namespace dmrg
