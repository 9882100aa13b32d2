// HIP kernels of libdmrg for gfx950 (CDNA4): the two-site H.psi sector GEMMs of Eq. dgemm
// (Section 2.2.1) on MFMA, operator pre-summation (Section 2.2.3), BF16 hi/lo splitting, diag(H)
// and the FP64 vector kernels of Davidson's method.
//
// Sector-GEMM kernels. One wavefront owns a 32 x 32 tile of a target psi block and loops over all
// tasks writing to that block (owner computes, no atomics, fixed order => deterministic). A task
// adds f * A . X . B^T. The product is chained through registers: for each 16-wide chunk j of the
// source columns, T'^T = X(:, j)^T A(rows, :)^T is formed by MFMA; the MFMA output layout of T'^T
// (lane l holds column l%16 and four rows) is exactly the A-operand layout of the second MFMA
// Y += T' B(cols, j)^T when the reduction index of instruction v is taken as the row of T'^T held in
// result slot v, so the intermediate never leaves the registers. MFMA lane layouts (checked on the
// device): operands -- lane l holds A[l%16][k-group l/16] and B[k-group l/16][l%16]; results --
// v_mfma_f64_16x16x4f64: lane l holds D[l/16 + 4v][l%16]; v_mfma_f32_16x16x32_bf16: lane l holds
// D[4*(l/16) + v][l%16], v = 0..3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dmrg {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

constexpr int TP = 2;   // 16-row tiles per wavefront
constexpr int TQ = 2;   // 16-col tiles per wavefront

__device__ __forceinline__ int ldo(int m) { return (m + kLd - 1) / kLd * kLd; }

// ------------------------------------------------------------------ pre-summation / transposition
__global__ void k_presum(const PresumBlock* __restrict__ blocks, const PresumTerm* __restrict__ terms,
                         double* __restrict__ pool) {
    const PresumBlock b = blocks[blockIdx.x];
    const int ld = ldo(b.cols);
    const int n = b.rows * b.cols;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int i = e / b.cols, j = e - (e / b.cols) * b.cols;
        double acc = 0.0;
        for (int t = b.t_begin; t < b.t_end; ++t) {
            const PresumTerm T = terms[t];
            const double v = T.trans ? pool[T.src_off + (int64_t)j * T.src_ld + i]
                                     : pool[T.src_off + (int64_t)i * T.src_ld + j];
            acc += T.coeff * v;
        }
        pool[b.out_off + (int64_t)i * ld + j] = acc;
    }
}

hipError_t launch_presum(const PresumBlock* blocks, int n_blocks, const PresumTerm* terms, double* pool,
                         hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_presum, dim3(n_blocks), dim3(256), 0, s, blocks, terms, pool);
    return hipGetLastError();
}

// ------------------------------------------------------------------ BF16 hi/lo split
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
// hi = bf16(fp32(x)), lo = bf16(fp32(x - hi))
__device__ __forceinline__ void split2(double x, unsigned short& hi, unsigned short& lo) {
    hi = f32_to_bf16_rne((float)x);
    lo = f32_to_bf16_rne((float)(x - (double)bf16_to_f32(hi)));
}
__device__ __forceinline__ void split2f(float x, unsigned short& hi, unsigned short& lo) {
    hi = f32_to_bf16_rne(x);
    lo = f32_to_bf16_rne(x - bf16_to_f32(hi));
}

__global__ void k_split(const double* __restrict__ x, int64_t n, unsigned short* __restrict__ hi,
                        unsigned short* __restrict__ lo) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        unsigned short h, l;
        split2(x[i], h, l);
        hi[i] = h;
        lo[i] = l;
    }
}

hipError_t launch_split(const double* pool, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_split, dim3((unsigned)blocks), dim3(256), 0, s, pool, n, hi, lo);
    return hipGetLastError();
}

// ------------------------------------------------------------------ FP64 sector GEMMs
__global__ __launch_bounds__(64) void k_hpsi_f64(const Unit* __restrict__ units, const Task* __restrict__ tasks,
                                                 const double* __restrict__ pool, const double* __restrict__ xall,
                                                 double* __restrict__ yall, int64_t n_coeff) {
    const Unit U = units[blockIdx.x];
    const double* __restrict__ x = xall + (int64_t)blockIdx.y * n_coeff;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    const int lane = threadIdx.x;
    const int li = lane & 15, g = lane >> 4;
    f64x4 acc[TP][TQ];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};

    for (int t = U.t_begin; t < U.t_end; ++t) {
        const Task T = tasks[t];
        const double* __restrict__ X = x + T.x_off;
        const int ma = T.m_a, md = T.m_d;
        const double f = T.f;
        if (T.a_off < 0 && T.b_off < 0) {
            // Y += f X (same block shape)
#pragma unroll
            for (int p = 0; p < TP; ++p)
#pragma unroll
                for (int q = 0; q < TQ; ++q)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = U.r0 + 16 * p + g + 4 * v, col = U.c0 + 16 * q + li;
                        if (row < ma && col < md) acc[p][q][v] += f * X[(int64_t)row * md + col];
                    }
        } else if (T.b_off < 0) {
            // Y += f A X : rows of Y from A, columns from X (m_d' = m_d)
            const double* __restrict__ A = pool + T.a_off;
            const int lda = ldo(ma);
            for (int k0 = 0; k0 < ma; k0 += 4) {
                const int k = k0 + g;
                double av[TP], bv[TQ];
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int row = U.r0 + 16 * p + li;
                    av[p] = (row < U.m_ap && k < ma) ? f * A[(int64_t)row * lda + k] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int col = U.c0 + 16 * q + li;
                    bv[q] = (k < ma && col < md) ? X[(int64_t)k * md + col] : 0.0;
                }
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int q = 0; q < TQ; ++q)
                        acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
            }
        } else if (T.a_off < 0) {
            // Y += f X B^T (m_a' = m_a)
            const double* __restrict__ B = pool + T.b_off;
            const int ldb = ldo(md);
            for (int k0 = 0; k0 < md; k0 += 4) {
                const int k = k0 + g;
                double av[TP], bv[TQ];
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int row = U.r0 + 16 * p + li;
                    av[p] = (row < ma && k < md) ? X[(int64_t)row * md + k] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int col = U.c0 + 16 * q + li;
                    bv[q] = (col < U.m_dp && k < md) ? f * B[(int64_t)col * ldb + k] : 0.0;
                }
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int q = 0; q < TQ; ++q)
                        acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
            }
        } else {
            // Y += f A X B^T, chained through registers over 16-column chunks of X
            const double* __restrict__ A = pool + T.a_off;
            const double* __restrict__ B = pool + T.b_off;
            const int lda = ldo(ma), ldb = ldo(md);
            for (int j0 = 0; j0 < md; j0 += 16) {
                f64x4 tt[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) tt[p] = f64x4{0.0, 0.0, 0.0, 0.0};
                const int jx = j0 + li;
                for (int k0 = 0; k0 < ma; k0 += 4) {
                    const int k = k0 + g;
                    const double xa = (k < ma && jx < md) ? X[(int64_t)k * md + jx] : 0.0;
#pragma unroll
                    for (int p = 0; p < TP; ++p) {
                        const int row = U.r0 + 16 * p + li;
                        const double ab = (row < U.m_ap && k < ma) ? A[(int64_t)row * lda + k] : 0.0;
                        tt[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, ab, tt[p], 0, 0, 0);
                    }
                }
                // tt[p][v] = T'[row = r0 + 16p + li][j = j0 + g + 4v]
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = j0 + g + 4 * v;
                    double bb[TQ];
#pragma unroll
                    for (int q = 0; q < TQ; ++q) {
                        const int col = U.c0 + 16 * q + li;
                        bb[q] = (col < U.m_dp && j < md) ? f * B[(int64_t)col * ldb + j] : 0.0;
                    }
#pragma unroll
                    for (int p = 0; p < TP; ++p)
#pragma unroll
                        for (int q = 0; q < TQ; ++q)
                            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(tt[p][v], bb[q], acc[p][q], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = U.r0 + 16 * p + g + 4 * v, col = U.c0 + 16 * q + li;
                if (row < U.m_ap && col < U.m_dp) y[U.y_off + (int64_t)row * U.m_dp + col] = acc[p][q][v];
            }
}

hipError_t launch_hpsi_f64(const Unit* units, int n_units, const Task* tasks, const double* pool, const double* x,
                           double* y, int64_t n_coeff, int nvec, hipStream_t s) {
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hpsi_f64, dim3(n_units, nvec), dim3(64), 0, s, units, tasks, pool, x, y, n_coeff);
    return hipGetLastError();
}

// ------------------------------------------------------------------ split-BF16 sector GEMMs
// Operands as BF16 hi/lo pairs; each product a.b is hi.hi + hi.lo + lo.hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation inside a task; task results are added in FP64.
__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mma3(u16x8 ah, u16x8 al, u16x8 bh, u16x8 bl, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bh), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bl), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al), as_bf(bh), c, 0, 0, 0);
    return c;
}

// 8 consecutive bf16 of a pool row starting at column k (masked beyond `lim`); 16-byte aligned.
__device__ __forceinline__ void load8(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t base,
                                      int k, int lim, bool ok, u16x8& h, u16x8& l) {
    if (ok && k + 8 <= lim + 7 && k < lim) {
        // rows are padded with zeros up to ld (multiple of 8), so a full 8-vector read stays in the row
        h = *reinterpret_cast<const u16x8*>(hi + base + k);
        l = *reinterpret_cast<const u16x8*>(lo + base + k);
    } else {
        h = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        l = h;
    }
}
__device__ __forceinline__ void load4(const uint16_t* __restrict__ hi, const uint16_t* __restrict__ lo, int64_t base,
                                      int k, int lim, bool ok, u16x4& h, u16x4& l) {
    if (ok && k < lim) {
        h = *reinterpret_cast<const u16x4*>(hi + base + k);
        l = *reinterpret_cast<const u16x4*>(lo + base + k);
    } else {
        h = u16x4{0, 0, 0, 0};
        l = h;
    }
}

__global__ __launch_bounds__(64) void k_hpsi_split(const Unit* __restrict__ units, const Task* __restrict__ tasks,
                                                   const uint16_t* __restrict__ phi, const uint16_t* __restrict__ plo,
                                                   const double* __restrict__ xall, double* __restrict__ yall,
                                                   int64_t n_coeff) {
    const Unit U = units[blockIdx.x];
    const double* __restrict__ x = xall + (int64_t)blockIdx.y * n_coeff;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    const int lane = threadIdx.x;
    const int li = lane & 15, g = lane >> 4;
    double acc[TP][TQ][4];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[p][q][v] = 0.0;

    for (int t = U.t_begin; t < U.t_end; ++t) {
        const Task T = tasks[t];
        const double* __restrict__ X = x + T.x_off;
        const int ma = T.m_a, md = T.m_d;
        const double f = T.f;
        f32x4 c32[TP][TQ];
#pragma unroll
        for (int p = 0; p < TP; ++p)
#pragma unroll
            for (int q = 0; q < TQ; ++q) c32[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (T.a_off < 0 && T.b_off < 0) {
#pragma unroll
            for (int p = 0; p < TP; ++p)
#pragma unroll
                for (int q = 0; q < TQ; ++q)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = U.r0 + 16 * p + 4 * g + v, col = U.c0 + 16 * q + li;
                        if (row < ma && col < md) acc[p][q][v] += f * X[(int64_t)row * md + col];
                    }
            continue;
        } else if (T.b_off < 0) {
            // Y += f A X: A-operand rows of A (8 consecutive k), B-operand X (split on the fly)
            const int lda = ldo(ma);
            for (int k0 = 0; k0 < ma; k0 += 32) {
                const int kb = k0 + 8 * g;
                u16x8 ah[TP], al[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int row = U.r0 + 16 * p + li;
                    load8(phi, plo, T.a_off + (int64_t)row * lda, kb, ma, row < U.m_ap, ah[p], al[p]);
                }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int col = U.c0 + 16 * q + li;
                    u16x8 bh, bl;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = kb + u;
                        const double xv = (k < ma && col < md) ? X[(int64_t)k * md + col] : 0.0;
                        unsigned short h, l;
                        split2(xv, h, l);
                        bh[u] = h;
                        bl[u] = l;
                    }
#pragma unroll
                    for (int p = 0; p < TP; ++p) c32[p][q] = mma3(ah[p], al[p], bh, bl, c32[p][q]);
                }
            }
        } else if (T.a_off < 0) {
            // Y += f X B^T: A-operand rows of X (split), B-operand rows of B (8 consecutive k)
            const int ldb = ldo(md);
            for (int k0 = 0; k0 < md; k0 += 32) {
                const int kb = k0 + 8 * g;
                u16x8 xh[TP], xl[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int row = U.r0 + 16 * p + li;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int k = kb + u;
                        const double xv = (row < ma && k < md) ? X[(int64_t)row * md + k] : 0.0;
                        unsigned short h, l;
                        split2(xv, h, l);
                        xh[p][u] = h;
                        xl[p][u] = l;
                    }
                }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int col = U.c0 + 16 * q + li;
                    u16x8 bh, bl;
                    load8(phi, plo, T.b_off + (int64_t)col * ldb, kb, md, col < U.m_dp, bh, bl);
#pragma unroll
                    for (int p = 0; p < TP; ++p) c32[p][q] = mma3(xh[p], xl[p], bh, bl, c32[p][q]);
                }
            }
        } else {
            const int lda = ldo(ma), ldb = ldo(md);
            for (int j0 = 0; j0 < md; j0 += 32) {
                // GEMM1: T'^T for two 16-column chunks (j0 .. j0+15 and j0+16 .. j0+31)
                f32x4 tt[2][TP];
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int p = 0; p < TP; ++p) tt[h2][p] = f32x4{0.f, 0.f, 0.f, 0.f};
                for (int k0 = 0; k0 < ma; k0 += 32) {
                    const int kb = k0 + 8 * g;
                    u16x8 ah[TP], al[TP];
#pragma unroll
                    for (int p = 0; p < TP; ++p) {
                        const int row = U.r0 + 16 * p + li;
                        load8(phi, plo, T.a_off + (int64_t)row * lda, kb, ma, row < U.m_ap, ah[p], al[p]);
                    }
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int jx = j0 + 16 * h2 + li;
                        u16x8 xh, xl;
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int k = kb + u;
                            const double xv = (k < ma && jx < md) ? X[(int64_t)k * md + jx] : 0.0;
                            unsigned short hh, ll;
                            split2(xv, hh, ll);
                            xh[u] = hh;
                            xl[u] = ll;
                        }
#pragma unroll
                        for (int p = 0; p < TP; ++p) tt[h2][p] = mma3(xh, xl, ah[p], al[p], tt[h2][p]);
                    }
                }
                // tt[h2][p][v] = T'[row = r0+16p+li][j = j0 + 16 h2 + 4g + v]; k-position 8g+u <->
                // j = j0 + 4g + u (u < 4), j0 + 16 + 4g + (u - 4) (u >= 4)
                u16x8 th[TP], tl[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float v = (float)f * tt[u >> 2][p][u & 3];
                        unsigned short hh, ll;
                        split2f(v, hh, ll);
                        th[p][u] = hh;
                        tl[p][u] = ll;
                    }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int col = U.c0 + 16 * q + li;
                    const bool okc = col < U.m_dp;
                    const int64_t base = T.b_off + (int64_t)col * ldb;
                    u16x4 bh0, bl0, bh1, bl1;
                    load4(phi, plo, base, j0 + 4 * g, md, okc, bh0, bl0);
                    load4(phi, plo, base, j0 + 16 + 4 * g, md, okc, bh1, bl1);
                    u16x8 bh = u16x8{bh0[0], bh0[1], bh0[2], bh0[3], bh1[0], bh1[1], bh1[2], bh1[3]};
                    u16x8 bl = u16x8{bl0[0], bl0[1], bl0[2], bl0[3], bl1[0], bl1[1], bl1[2], bl1[3]};
#pragma unroll
                    for (int p = 0; p < TP; ++p) c32[p][q] = mma3(th[p], tl[p], bh, bl, c32[p][q]);
                }
            }
            // f already applied to T'
#pragma unroll
            for (int p = 0; p < TP; ++p)
#pragma unroll
                for (int q = 0; q < TQ; ++q)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[p][q][v] += (double)c32[p][q][v];
            continue;
        }
#pragma unroll
        for (int p = 0; p < TP; ++p)
#pragma unroll
            for (int q = 0; q < TQ; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[p][q][v] += f * (double)c32[p][q][v];
    }
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = U.r0 + 16 * p + 4 * g + v, col = U.c0 + 16 * q + li;
                if (row < U.m_ap && col < U.m_dp) y[U.y_off + (int64_t)row * U.m_dp + col] = acc[p][q][v];
            }
}

hipError_t launch_hpsi_split(const Unit* units, int n_units, const Task* tasks, const uint16_t* hi, const uint16_t* lo,
                             const double* x, double* y, int64_t n_coeff, int nvec, hipStream_t s) {
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hpsi_split, dim3(n_units, nvec), dim3(64), 0, s, units, tasks, hi, lo, x, y, n_coeff);
    return hipGetLastError();
}

// ------------------------------------------------------------------ diag(H)
__global__ void k_diag(const DiagBlock* __restrict__ blocks, const DiagTask* __restrict__ tasks,
                       const double* __restrict__ pool, double* __restrict__ d) {
    const DiagBlock b = blocks[blockIdx.x];
    const int lda = ldo(b.m_a), ldb = ldo(b.m_d);
    const int n = b.m_a * b.m_d;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int i = e / b.m_d, j = e - (e / b.m_d) * b.m_d;
        double acc = 0.0;
        for (int t = b.t_begin; t < b.t_end; ++t) {
            const DiagTask T = tasks[t];
            const double a = T.a_off < 0 ? 1.0 : pool[T.a_off + (int64_t)i * lda + i];
            const double c = T.b_off < 0 ? 1.0 : pool[T.b_off + (int64_t)j * ldb + j];
            acc += T.f * a * c;
        }
        d[b.off + e] = acc;
    }
}

hipError_t launch_diag(const DiagBlock* blocks, int n_blocks, const DiagTask* tasks, const double* pool, double* d,
                       hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag, dim3(n_blocks), dim3(256), 0, s, blocks, tasks, pool, d);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Davidson vector kernels (FP64)
int multidot_parts(int64_t n) {
    int64_t p = (n + 8191) / 8192;
    if (p < 1) p = 1;
    if (p > 1024) p = 1024;
    return (int)p;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial[j * n_part + block] = sum over the block's chunk of V[j] . w   (fixed order)
__global__ void k_multidot(const double* __restrict__ V, int nv, int64_t n, const double* __restrict__ w,
                           double* __restrict__ partial, int n_part) {
    __shared__ double red[4];
    const int64_t chunk = (n + n_part - 1) / n_part;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int j = 0; j < nv; ++j) {
        const double* __restrict__ v = V + (int64_t)j * n;
        double s = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += v[i] * w[i];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partial[(int64_t)j * n_part + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
    }
}

__global__ void k_multidot_finish(const double* __restrict__ partial, int n_part, int nv, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    double s = 0.0;
    for (int b = 0; b < n_part; ++b) s += partial[(int64_t)j * n_part + b];
    out[j] = s;
}

hipError_t launch_multidot(const double* V, int nv, int64_t n, const double* w, double* partial, int n_part,
                           double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_multidot, dim3(n_part), dim3(256), 0, s, V, nv, n, w, partial, n_part);
    hipLaunchKernelGGL(k_multidot_finish, dim3((nv + 63) / 64), dim3(64), 0, s, partial, n_part, nv, out);
    return hipGetLastError();
}

// out = beta * out + sum_j coef[j] V[j]   (coefficients passed by value)
__global__ void k_combine(const double* __restrict__ V, int nv, int64_t n, const Coefs coef,
                          double* __restrict__ out, double beta) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = beta == 0.0 ? 0.0 : beta * out[i];
        for (int j = 0; j < nv; ++j) s += coef.c[j] * V[(int64_t)j * n + i];
        out[i] = s;
    }
}

hipError_t launch_combine(const double* V, int nv, int64_t n, const Coefs& coef, double* out, double beta,
                          hipStream_t s) {
    if (nv > kMaxCombine) return hipErrorInvalidValue;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(256), 0, s, V, nv, n, coef, out, beta);
    return hipGetLastError();
}

// t = r / (theta - d), |theta - d| floored at 1e-8 with its sign kept
__global__ void k_precond(const double* __restrict__ r, const double* __restrict__ d, double theta,
                          double* __restrict__ t, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double den = theta - d[i];
        if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
        t[i] = r[i] / den;
    }
}

hipError_t launch_precond(const double* r, const double* d, double theta, double* t, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_precond, dim3((unsigned)blocks), dim3(256), 0, s, r, d, theta, t, n);
    return hipGetLastError();
}

__global__ void k_scale(double* __restrict__ x, double a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= a;
}

hipError_t launch_scale(double* x, double a, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, s, x, a, n);
    return hipGetLastError();
}

}  // namespace dmrg
