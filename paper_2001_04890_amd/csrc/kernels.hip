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

// Register budget per tile class: two wavefronts per SIMD where that fits without spills.
constexpr int min_waves_f64(int tp, int tq) { return tp * tq <= 8 ? 2 : 1; }
constexpr int min_waves_split(int tp, int tq) { return tp * tq <= 12 ? 2 : 1; }

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

// ------------------------------------------------------------------ input packing (Eq. wf_sec blocks)
// xp: FP64, every block pa x pd row-major (zero padding). Split path: BF16 hi/lo of the same block
// row-major (xr) and transposed (xt, pd x pa).
__global__ void k_pack(const PackBlock* __restrict__ packs, const double* __restrict__ xall, int64_t n_coeff,
                       int64_t psize, double* __restrict__ xpall, uint16_t* __restrict__ xrh, uint16_t* __restrict__ xrl,
                       uint16_t* __restrict__ xth, uint16_t* __restrict__ xtl, int split) {
    const PackBlock P = packs[blockIdx.x];
    const double* __restrict__ x = xall + (int64_t)blockIdx.y * n_coeff + P.src_off;
    const int64_t vo = (int64_t)blockIdx.y * psize + P.dst_off;
    const int n = P.pa * P.pd;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int i = e / P.pd, j = e - (e / P.pd) * P.pd;
        const double v = (i < P.m_a && j < P.m_d) ? x[(int64_t)i * P.m_d + j] : 0.0;
        xpall[vo + e] = v;
        if (split) {
            unsigned short h, l;
            split2(v, h, l);
            xrh[vo + e] = h;
            xrl[vo + e] = l;
            const int64_t t = vo + (int64_t)j * P.pa + i;
            xth[t] = h;
            xtl[t] = l;
        }
    }
}

// ------------------------------------------------------------------ tile store (direct or partial tile)
template <int TP, int TQ, class Acc>
__device__ __forceinline__ void store_tile(const Item& I, double* __restrict__ y, double* __restrict__ part,
                                           const Acc& acc, int li, int g, bool f64_layout) {
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = 16 * p + (f64_layout ? g + 4 * v : 4 * g + v);
                const int cc = 16 * q + li;
                const int row = I.r0 + rr, col = I.c0 + cc;
                if (I.part_off < 0) {
                    if (row < I.m_ap && col < I.m_dp) y[I.y_off + (int64_t)row * I.m_dp + col] += acc[p][q][v];
                } else {
                    part[I.part_off + rr * (16 * TQ) + cc] = acc[p][q][v];
                }
            }
}

// y_tile += sum of its partial tiles, in item order
__global__ void k_reduce(const Reduce* __restrict__ red, const double* __restrict__ partall, double* __restrict__ yall,
                         int64_t n_coeff, int64_t part_stride, const int32_t* __restrict__ active) {
    const Reduce R = red[blockIdx.x];
    if (active && active[R.part] != kPartActive) return;
    const double* __restrict__ part = partall + (int64_t)blockIdx.y * part_stride + R.part_off;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    const int n = R.tm * R.tn;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int rr = e / R.tn, cc = e - (e / R.tn) * R.tn;
        const int row = R.r0 + rr, col = R.c0 + cc;
        if (row >= R.m_ap || col >= R.m_dp) continue;
        double s = 0.0;
        for (int k = 0; k < R.n_parts; ++k) s += part[(int64_t)k * n + e];
        y[R.y_off + (int64_t)row * R.m_dp + col] += s;
    }
}

__device__ __forceinline__ f64x4 ld4(const double* p) { return *reinterpret_cast<const f64x4*>(p); }

// ------------------------------------------------------------------ FP64 sector GEMMs
// Operands are read without masks from the padded pool and the packed input. The reduction index of
// GEMM1 is permuted (instruction v takes k = k0 + 4g + v in lane group g) so that A rows are read
// as 32-byte vectors; GEMM1's X operand uses columns j0 + pl(li), pl(r) = 4 (r % 4) + r / 4, so that
// result slot v of lane group g holds column j0 + 4g + v and B rows are read as 32-byte vectors too.
template <int TP, int TQ>
__global__ __launch_bounds__(64, min_waves_f64(TP, TQ)) void k_hpsi_f64(const Item* __restrict__ items, const Task* __restrict__ tasks,
                                                 const double* __restrict__ pool, const double* __restrict__ xpall,
                                                 double* __restrict__ yall, double* __restrict__ partall,
                                                 int64_t n_coeff, int64_t psize, int64_t slot_stride,
                                                 const int32_t* __restrict__ active) {
    const Item I = items[blockIdx.x];
    if (active && active[I.part] != kPartActive) return;
    const double* __restrict__ xp = xpall + (int64_t)blockIdx.y * psize;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    double* __restrict__ part = partall + (int64_t)blockIdx.y * slot_stride;
    const int lane = threadIdx.x;
    const int li = lane & 15, g = lane >> 4;
    const int pl = 4 * (li & 3) + (li >> 2);
    f64x4 acc[TP][TQ];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q) acc[p][q] = f64x4{0.0, 0.0, 0.0, 0.0};

    Task Tn = tasks[I.t_begin];   // descriptor of the next task, loaded one task ahead
    for (int t = I.t_begin; t < I.t_end; ++t) {
        const Task T = Tn;
        if (t + 1 < I.t_end) Tn = tasks[t + 1];
        const double* __restrict__ X = xp + T.x_off;
        const int pa = T.pa, pd = T.pd;
        const double f = T.f;
        if (T.a_off < 0 && T.b_off < 0) {
#pragma unroll
            for (int p = 0; p < TP; ++p)
#pragma unroll
                for (int q = 0; q < TQ; ++q)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[p][q][v] += f * X[(I.r0 + 16 * p + g + 4 * v) * pd + I.c0 + 16 * q + li];
        } else if (T.b_off < 0) {
            // Y += f A X (right identity)
            const double* __restrict__ A = pool + T.a_off;
            for (int k0 = 0; k0 < T.ka; k0 += 16) {
                f64x4 a4[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) a4[p] = f * ld4(A + (I.r0 + 16 * p + li) * pa + k0 + 4 * g);
                double xv[4][TQ];
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int q = 0; q < TQ; ++q) xv[v][q] = X[(k0 + 4 * g + v) * pd + I.c0 + 16 * q + li];
                // consecutive MFMAs accumulate into the same registers (the fast path of the matrix core)
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int q = 0; q < TQ; ++q)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[p][v], xv[v][q], acc[p][q], 0, 0, 0);
            }
        } else if (T.a_off < 0) {
            // Y += f X B^T (left identity)
            const double* __restrict__ B = pool + T.b_off;
            for (int k0 = 0; k0 < T.kd; k0 += 16) {
                f64x4 x4[TP], b4[TQ];
#pragma unroll
                for (int p = 0; p < TP; ++p) x4[p] = f * ld4(X + (I.r0 + 16 * p + li) * pd + k0 + 4 * g);
#pragma unroll
                for (int q = 0; q < TQ; ++q) b4[q] = ld4(B + (I.c0 + 16 * q + li) * pd + k0 + 4 * g);
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int q = 0; q < TQ; ++q)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(x4[p][v], b4[q][v], acc[p][q], 0, 0, 0);
            }
        } else {
            // Y += f A X B^T, chained through registers over 16-column chunks of X
            const double* __restrict__ A = pool + T.a_off;
            const double* __restrict__ B = pool + T.b_off;
            for (int j0 = 0; j0 < T.kd; j0 += 16) {
                f64x4 tt[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) tt[p] = f64x4{0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < T.ka; k0 += 16) {
                    f64x4 a4[TP];
#pragma unroll
                    for (int p = 0; p < TP; ++p) a4[p] = ld4(A + (I.r0 + 16 * p + li) * pa + k0 + 4 * g);
                    double xv[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) xv[v] = X[(k0 + 4 * g + v) * pd + j0 + pl];
#pragma unroll
                    for (int p = 0; p < TP; ++p)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            tt[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[v], a4[p][v], tt[p], 0, 0, 0);
                }
                // tt[p][v] = T'[r0 + 16p + li][j0 + 4g + v]
                f64x4 b4[TQ];
#pragma unroll
                for (int q = 0; q < TQ; ++q) b4[q] = ld4(B + (I.c0 + 16 * q + li) * pd + j0 + 4 * g);
#pragma unroll
                for (int p = 0; p < TP; ++p) tt[p] *= f;
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int q = 0; q < TQ; ++q)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(tt[p][v], b4[q][v], acc[p][q], 0, 0, 0);
            }
        }
    }
    store_tile<TP, TQ>(I, y, part, acc, li, g, true);
}

__global__ void k_zero(double* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 0.0;
}

static hipError_t launch_pack(const HpsiPlan& plan, const double* x, int64_t n_coeff, int nvec, int split,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(plan.n_packs, nvec), dim3(256), 0, s, plan.packs, x, n_coeff, plan.packed_size,
                       plan.xp, plan.xr_hi, plan.xr_lo, plan.xt_hi, plan.xt_lo, split);
    return hipGetLastError();
}

// y = 0, then phase by phase: the item launches of every tile class, then the phase's reductions
template <class F>
static hipError_t run_phases(const HpsiPlan& plan, double* y, int64_t n_coeff, int nvec, hipStream_t s, F&& launch_one,
                             bool zero_y, const int32_t* active) {
    int64_t n = n_coeff * nvec, blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (zero_y) hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, y, n);
    for (int ph = 0; ph < plan.n_phases; ++ph) {
        const HpsiPhase& P = plan.phases[ph];
        for (int l = P.launch_begin; l < P.launch_end; ++l) {
            const HpsiLaunch& L = plan.launches[l];
            launch_one(L.cls, L.item_begin, L.item_count);
        }
        const int nr = P.reduce_end - P.reduce_begin;
        if (nr > 0)
            hipLaunchKernelGGL(k_reduce, dim3(nr, nvec), dim3(256), 0, s, plan.reduces + P.reduce_begin, plan.partial,
                               y, n_coeff, plan.partial_size, active);
    }
    return hipGetLastError();
}

#define DMRG_CLASS_SWITCH(KERNEL, ...)                                                                 \
    switch (c) {                                                                                       \
        case 0: hipLaunchKernelGGL((KERNEL<1, 1>), __VA_ARGS__); break;                                \
        case 1: hipLaunchKernelGGL((KERNEL<1, 2>), __VA_ARGS__); break;                                \
        case 2: hipLaunchKernelGGL((KERNEL<1, 3>), __VA_ARGS__); break;                                \
        case 3: hipLaunchKernelGGL((KERNEL<1, 4>), __VA_ARGS__); break;                                \
        case 4: hipLaunchKernelGGL((KERNEL<1, 5>), __VA_ARGS__); break;                                \
        case 5: hipLaunchKernelGGL((KERNEL<1, 6>), __VA_ARGS__); break;                                \
        case 6: hipLaunchKernelGGL((KERNEL<1, 7>), __VA_ARGS__); break;                                \
        case 7: hipLaunchKernelGGL((KERNEL<1, 8>), __VA_ARGS__); break;                                \
        case 8: hipLaunchKernelGGL((KERNEL<2, 1>), __VA_ARGS__); break;                                \
        case 9: hipLaunchKernelGGL((KERNEL<2, 2>), __VA_ARGS__); break;                                \
        case 10: hipLaunchKernelGGL((KERNEL<2, 3>), __VA_ARGS__); break;                               \
        case 11: hipLaunchKernelGGL((KERNEL<2, 4>), __VA_ARGS__); break;                               \
        case 12: hipLaunchKernelGGL((KERNEL<2, 5>), __VA_ARGS__); break;                               \
        case 13: hipLaunchKernelGGL((KERNEL<2, 6>), __VA_ARGS__); break;                               \
        case 14: hipLaunchKernelGGL((KERNEL<2, 7>), __VA_ARGS__); break;                               \
        default: hipLaunchKernelGGL((KERNEL<2, 8>), __VA_ARGS__); break;                               \
    }

hipError_t launch_hpsi_f64(const HpsiPlan& plan, const double* pool, const double* x, double* y, int64_t n_coeff,
                           int nvec, hipStream_t s, const int32_t* active) {
    // the packed input feeds only this plan's items (the other FP64 kernels pack their own)
    bool any = false;
    for (int ph = 0; ph < plan.n_phases && !any; ++ph)
        for (int l = plan.phases[ph].launch_begin; l < plan.phases[ph].launch_end; ++l)
            any = any || plan.launches[l].item_count > 0;
    if (any) {
        hipError_t e = launch_pack(plan, x, n_coeff, nvec, 0, s);
        if (e != hipSuccess) return e;
    }
    const int64_t ss = plan.partial_size;
    return run_phases(plan, y, n_coeff, nvec, s, [&](int c, int b, int n) {
        DMRG_CLASS_SWITCH(k_hpsi_f64, dim3(n, nvec), dim3(64), 0, s, plan.items + b, plan.tasks, pool, plan.xp, y,
                          plan.partial, n_coeff, plan.packed_size, ss, active)
    }, true, active);
}

// ------------------------------------------------------------------ split-BF16 sector GEMMs
// Operands as BF16 hi/lo pairs; each product a.b is hi.hi + hi.lo + lo.hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation inside a task; task results are added in FP64.
// All operand reads are 16-byte vectors: pool rows, packed X rows and packed X^T rows. GEMM1's X^T
// operand row li of chunk h (h = 0, 1) is column j0 + 8 (li / 4) + 4 h + li % 4, which puts column
// j0 + 8g + u into k-position 8g + u of GEMM2 (u = 4h + v).
__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mma3(u16x8 ah, u16x8 al, u16x8 bh, u16x8 bl, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bh), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bl), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al), as_bf(bh), c, 0, 0, 0);
    return c;
}
__device__ __forceinline__ u16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }

template <int TP, int TQ>
__global__ __launch_bounds__(64, min_waves_split(TP, TQ)) void k_hpsi_split(const Item* __restrict__ items, const Task* __restrict__ tasks,
                                                   const uint16_t* __restrict__ phi, const uint16_t* __restrict__ plo,
                                                   const double* __restrict__ xpall, const uint16_t* __restrict__ xrh,
                                                   const uint16_t* __restrict__ xrl, const uint16_t* __restrict__ xth,
                                                   const uint16_t* __restrict__ xtl, double* __restrict__ yall,
                                                   double* __restrict__ partall, int64_t n_coeff, int64_t psize,
                                                   int64_t slot_stride, const int32_t* __restrict__ active) {
    const Item I = items[blockIdx.x];
    if (active && active[I.part] != kPartActive) return;
    const int64_t vo = (int64_t)blockIdx.y * psize;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    double* __restrict__ part = partall + (int64_t)blockIdx.y * slot_stride;
    const int lane = threadIdx.x;
    const int li = lane & 15, g = lane >> 4;
    double acc[TP][TQ][4];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < TQ; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[p][q][v] = 0.0;

    Task Tn = tasks[I.t_begin];   // descriptor of the next task, loaded one task ahead
    for (int t = I.t_begin; t < I.t_end; ++t) {
        const Task T = Tn;
        if (t + 1 < I.t_end) Tn = tasks[t + 1];
        const int pa = T.pa, pd = T.pd;
        const int64_t xo = vo + T.x_off;
        const double f = T.f;
        if (T.a_off < 0 && T.b_off < 0) {
            const double* __restrict__ X = xpall + xo;
#pragma unroll
            for (int p = 0; p < TP; ++p)
#pragma unroll
                for (int q = 0; q < TQ; ++q)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[p][q][v] += f * X[(I.r0 + 16 * p + 4 * g + v) * pd + I.c0 + 16 * q + li];
            continue;
        }
        f32x4 c32[TP][TQ];
#pragma unroll
        for (int p = 0; p < TP; ++p)
#pragma unroll
            for (int q = 0; q < TQ; ++q) c32[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        double scale = f;
        if (T.b_off < 0) {
            // Y += f A X: A-operand rows of A, B-operand columns of X (rows of X^T)
            const int64_t ab = T.a_off;
            for (int k0 = 0; k0 < pa; k0 += 32) {
                u16x8 ah[TP], al[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int64_t o = ab + (I.r0 + 16 * p + li) * pa + k0 + 8 * g;
                    ah[p] = ld8(phi + o);
                    al[p] = ld8(plo + o);
                }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int64_t o = xo + (I.c0 + 16 * q + li) * pa + k0 + 8 * g;
                    const u16x8 bh = ld8(xth + o), bl = ld8(xtl + o);
#pragma unroll
                    for (int p = 0; p < TP; ++p) c32[p][q] = mma3(ah[p], al[p], bh, bl, c32[p][q]);
                }
            }
        } else if (T.a_off < 0) {
            // Y += f X B^T: A-operand rows of X, B-operand rows of B
            const int64_t bb = T.b_off;
            for (int k0 = 0; k0 < pd; k0 += 32) {
                u16x8 xh[TP], xl[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p) {
                    const int64_t o = xo + (I.r0 + 16 * p + li) * pd + k0 + 8 * g;
                    xh[p] = ld8(xrh + o);
                    xl[p] = ld8(xrl + o);
                }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int64_t o = bb + (I.c0 + 16 * q + li) * pd + k0 + 8 * g;
                    const u16x8 bh = ld8(phi + o), bl = ld8(plo + o);
#pragma unroll
                    for (int p = 0; p < TP; ++p) c32[p][q] = mma3(xh[p], xl[p], bh, bl, c32[p][q]);
                }
            }
        } else {
            const int64_t ab = T.a_off, bb = T.b_off;
            const int jl = 8 * (li >> 2) + (li & 3);
            for (int j0 = 0; j0 < pd; j0 += 32) {
                f32x4 tt[2][TP];
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int p = 0; p < TP; ++p) tt[h2][p] = f32x4{0.f, 0.f, 0.f, 0.f};
                for (int k0 = 0; k0 < pa; k0 += 32) {
                    u16x8 ah[TP], al[TP];
#pragma unroll
                    for (int p = 0; p < TP; ++p) {
                        const int64_t o = ab + (I.r0 + 16 * p + li) * pa + k0 + 8 * g;
                        ah[p] = ld8(phi + o);
                        al[p] = ld8(plo + o);
                    }
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int64_t o = xo + (int64_t)(j0 + jl + 4 * h2) * pa + k0 + 8 * g;
                        const u16x8 xh = ld8(xth + o), xl = ld8(xtl + o);
#pragma unroll
                        for (int p = 0; p < TP; ++p) tt[h2][p] = mma3(xh, xl, ah[p], al[p], tt[h2][p]);
                    }
                }
                // tt[h][p][v] = T'[r0 + 16p + li][j0 + 8g + 4h + v]
                u16x8 th[TP], tl[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        unsigned short hh, ll;
                        split2f((float)f * tt[u >> 2][p][u & 3], hh, ll);
                        th[p][u] = hh;
                        tl[p][u] = ll;
                    }
#pragma unroll
                for (int q = 0; q < TQ; ++q) {
                    const int64_t o = bb + (I.c0 + 16 * q + li) * pd + j0 + 8 * g;
                    const u16x8 bh = ld8(phi + o), bl = ld8(plo + o);
#pragma unroll
                    for (int p = 0; p < TP; ++p) c32[p][q] = mma3(th[p], tl[p], bh, bl, c32[p][q]);
                }
            }
            scale = 1.0;   // f already applied to T'
        }
#pragma unroll
        for (int p = 0; p < TP; ++p)
#pragma unroll
            for (int q = 0; q < TQ; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[p][q][v] += scale * (double)c32[p][q][v];
    }
    store_tile<TP, TQ>(I, y, part, acc, li, g, false);
}

static hipError_t hpsi_split_impl(const HpsiPlan& plan, const uint16_t* hi, const uint16_t* lo, const double* x,
                                  double* y, int64_t n_coeff, int nvec, hipStream_t s, bool zero_y,
                                  const int32_t* active) {
    hipError_t e = launch_pack(plan, x, n_coeff, nvec, 1, s);
    if (e != hipSuccess) return e;
    const int64_t ss = plan.partial_size;
    return run_phases(plan, y, n_coeff, nvec, s, [&](int c, int b, int n) {
        DMRG_CLASS_SWITCH(k_hpsi_split, dim3(n, nvec), dim3(64), 0, s, plan.items + b, plan.tasks, hi, lo, plan.xp,
                          plan.xr_hi, plan.xr_lo, plan.xt_hi, plan.xt_lo, y, plan.partial, n_coeff, plan.packed_size, ss,
                          active)
    }, zero_y, active);
}

hipError_t launch_hpsi_split(const HpsiPlan& plan, const uint16_t* hi, const uint16_t* lo, const double* x, double* y,
                             int64_t n_coeff, int nvec, hipStream_t s, const int32_t* active) {
    return hpsi_split_impl(plan, hi, lo, x, y, n_coeff, nvec, s, true, active);
}

hipError_t launch_hpsi_split_acc(const HpsiPlan& plan, const uint16_t* hi, const uint16_t* lo, const double* x,
                                 double* y, int64_t n_coeff, int nvec, hipStream_t s, const int32_t* active) {
    if (plan.n_phases == 0) return hipSuccess;
    return hpsi_split_impl(plan, hi, lo, x, y, n_coeff, nvec, s, false, active);
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
// Dot products V[j] . w: the vector is cut into n_part chunks of kDotChunk elements; workgroup (b, g)
// forms the partial sums of chunk b for vectors 8 g .. 8 g + 7 (w read once per element for all 8),
// then one wavefront per vector adds the n_part partials. Fixed partition and order: deterministic.
constexpr int kDotChunk = 1024;
constexpr int kDotVecs = 8;

int multidot_parts(int64_t n) {
    int64_t p = (n + kDotChunk - 1) / kDotChunk;
    return (int)(p < 1 ? 1 : p);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// partial[j * n_part + b] = sum over chunk b of V[j] . w
__global__ __launch_bounds__(256) void k_multidot(const double* __restrict__ V, int nv, int64_t n,
                                                  const double* __restrict__ w, double* __restrict__ partial,
                                                  int n_part) {
    __shared__ double red[4][kDotVecs];
    const int64_t lo = (int64_t)blockIdx.x * kDotChunk;
    const int64_t hi = lo + kDotChunk < n ? lo + kDotChunk : n;
    const int j0 = blockIdx.y * kDotVecs;
    const int nj = nv - j0 < kDotVecs ? nv - j0 : kDotVecs;
    double acc[kDotVecs];
#pragma unroll
    for (int j = 0; j < kDotVecs; ++j) acc[j] = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < kDotVecs; ++j)
            if (j < nj) acc[j] += V[(int64_t)(j0 + j) * n + i] * wi;
    }
#pragma unroll
    for (int j = 0; j < kDotVecs; ++j) {
        const double v = wave_sum(acc[j]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nj)
        partial[(int64_t)(j0 + threadIdx.x) * n_part + blockIdx.x] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// out[j] = sum_b partial[j * n_part + b]; one wavefront per vector
__global__ void k_multidot_finish(const double* __restrict__ partial, int n_part, double* __restrict__ out) {
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < n_part; b += 64) s += partial[(int64_t)j * n_part + b];
    s = wave_sum(s);
    if (threadIdx.x == 0) out[j] = s;
}

hipError_t launch_multidot(const double* V, int nv, int64_t n, const double* w, double* partial, int n_part,
                           double* out, hipStream_t s) {
    if (nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_multidot, dim3(n_part, (nv + kDotVecs - 1) / kDotVecs), dim3(256), 0, s, V, nv, n, w,
                       partial, n_part);
    hipLaunchKernelGGL(k_multidot_finish, dim3(nv), dim3(64), 0, s, partial, n_part, out);
    return hipGetLastError();
}

// out -= sum_j c[j] V[j] with the coefficients in device memory (Gram-Schmidt step)
__global__ void k_project_out(const double* __restrict__ V, int nv, int64_t n, const double* __restrict__ c,
                              double* __restrict__ out) {
    __shared__ double cs[kMaxCombine];
    for (int j = threadIdx.x; j < nv; j += blockDim.x) cs[j] = c[j];
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < nv; ++j) s += cs[j] * V[(int64_t)j * n + i];
        out[i] -= s;
    }
}

hipError_t launch_project_out(const double* V, int nv, int64_t n, const double* c, double* out, hipStream_t s) {
    if (nv > kMaxCombine) return hipErrorInvalidValue;
    if (nv <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_project_out, dim3((unsigned)blocks), dim3(256), 0, s, V, nv, n, c, out);
    return hipGetLastError();
}

// x *= 1 / sqrt(*nrm2) (left unchanged when *nrm2 is not positive)
__global__ void k_scale_dev(double* __restrict__ x, const double* __restrict__ nrm2, int64_t n) {
    const double q = *nrm2;
    if (!(q > 0.0)) return;
    const double a = 1.0 / sqrt(q);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= a;
}

hipError_t launch_scale_dev(double* x, const double* nrm2, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_scale_dev, dim3((unsigned)blocks), dim3(256), 0, s, x, nrm2, n);
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

// ------------------------------------------------------------------ reduced density matrix
// rho^L = psi psi^T per enlarged-left sector (Section 2.1), FP64, one workgroup per item; each
// thread owns output elements and sums over the column groups and columns in a fixed order.
__global__ void k_rdm_left(const RdmItem* __restrict__ items, const int64_t* __restrict__ gblk,
                           const int32_t* __restrict__ cdmd, const double* __restrict__ psi,
                           double* __restrict__ rho) {
    const RdmItem it = items[blockIdx.x];
    const int n = it.ma * it.ma2;
    for (int e = (int)threadIdx.x; e < n; e += (int)blockDim.x) {
        const int l = e / it.ma2, l2 = e - (e / it.ma2) * it.ma2;
        double acc = 0.0;
        for (int k = 0; k < it.n_cd; ++k) {
            const int md = cdmd[it.cd + k];
            const double* x = psi + gblk[it.g + k] + (int64_t)l * md;
            const double* y = psi + gblk[it.g2 + k] + (int64_t)l2 * md;
            for (int r = 0; r < md; ++r) acc = fma(x[r], y[r], acc);
        }
        rho[it.rho_off + (int64_t)l * it.ld + l2] = acc;
    }
}

hipError_t launch_rdm_left(const RdmItem* items, int n_items, const int64_t* gblk, const int32_t* cdmd,
                           const double* psi, double* rho, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rdm_left, dim3((unsigned)n_items), dim3(256), 0, s, items, gblk, cdmd, psi, rho);
    return hipGetLastError();
}

// rho^R = psi^T psi per enlarged-right sector: element (r, r2) sums X_k[l][r] X2_k[l][r2] over the
// sector's row groups k and their rows l (columns r of blocks with ma columns, r2 of blocks with ma2).
__global__ void k_rdm_right(const RdmItem* __restrict__ items, const int64_t* __restrict__ gblk,
                            const int32_t* __restrict__ rows, const double* __restrict__ psi,
                            double* __restrict__ rho) {
    const RdmItem it = items[blockIdx.x];
    const int n = it.ma * it.ma2;
    for (int e = (int)threadIdx.x; e < n; e += (int)blockDim.x) {
        const int r = e / it.ma2, r2 = e - (e / it.ma2) * it.ma2;
        double acc = 0.0;
        for (int k = 0; k < it.n_cd; ++k) {
            const int ml = rows[it.cd + k];
            const double* x = psi + gblk[it.g + k] + r;
            const double* y = psi + gblk[it.g2 + k] + r2;
            for (int l = 0; l < ml; ++l) acc = fma(x[(int64_t)l * it.ma], y[(int64_t)l * it.ma2], acc);
        }
        rho[it.rho_off + (int64_t)r * it.ld + r2] = acc;
    }
}

hipError_t launch_rdm_right(const RdmItem* items, int n_items, const int64_t* gblk, const int32_t* cdmd,
                            const double* psi, double* rho, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rdm_right, dim3((unsigned)n_items), dim3(256), 0, s, items, gblk, cdmd, psi, rho);
    return hipGetLastError();
}

// ------------------------------------------------------------------ renormalized operator blocks
// Eq. renorm_mat, FP64, one workgroup per sector block and pass; each thread owns output elements and
// sums in a fixed order.
__global__ void k_renorm_t(const RenormItem* __restrict__ items, const double* __restrict__ A,
                           const double* __restrict__ O, double* __restrict__ T, int chunk) {
    const RenormItem it = items[blockIdx.x];
    const int n = it.rows * it.k_in;
    const int e0 = (int)blockIdx.y * chunk, e1 = min(n, e0 + chunk);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += (int)blockDim.x) {
        const int r = e / it.k_in, j = e - (e / it.k_in) * it.k_in;
        const double* a = A + it.a_off + (int64_t)r * it.cols;
        const double* o = O + it.oi_off + j;                    // column j of O_in, stride k_in
        double acc = 0.0;
        for (int c = 0; c < it.cols; ++c) acc = fma(a[c], o[(int64_t)c * it.k_in], acc);
        T[it.t_off + e] = acc;
    }
}

__global__ void k_renorm_out(const RenormItem* __restrict__ items, const double* __restrict__ O,
                             const double* __restrict__ T, double* __restrict__ out, int chunk) {
    const RenormItem it = items[blockIdx.x];
    const int n = it.k_out * it.k_in;
    const int e0 = (int)blockIdx.y * chunk, e1 = min(n, e0 + chunk);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += (int)blockDim.x) {
        const int i = e / it.k_in, j = e - (e / it.k_in) * it.k_in;
        const double* o = O + it.oo_off + i;                    // column i of O_out, stride k_out
        const double* t = T + it.t_off + j;                     // column j of T, stride k_in
        double acc = 0.0;
        for (int r = 0; r < it.rows; ++r) acc = fma(o[(int64_t)r * it.k_out], t[(int64_t)r * it.k_in], acc);
        out[it.out_off + e] = acc;
    }
}

// Output elements of one item are cut into chunks of at least 1024 (grid.y <= 65535), so that a few
// large sector blocks still spread over the chip; max_t / max_out: most elements of one item per pass.
hipError_t launch_renormalize(const RenormItem* items, int n_items, int64_t max_t, int64_t max_out, const double* A,
                              const double* O, double* T, double* out, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    auto grid = [&](int64_t most, int& chunk) {
        int64_t c = std::max<int64_t>(1024, (most + 65534) / 65535);
        c = (c + 255) / 256 * 256;
        chunk = (int)c;
        return dim3((unsigned)n_items, (unsigned)std::max<int64_t>(1, (most + c - 1) / c));
    };
    int ct = 0, co = 0;
    const dim3 gt = grid(max_t, ct), go = grid(max_out, co);
    hipLaunchKernelGGL(k_renorm_t, gt, dim3(256), 0, s, items, A, O, T, ct);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_renorm_out, go, dim3(256), 0, s, items, O, T, out, co);
    return hipGetLastError();
}

}  // namespace dmrg
