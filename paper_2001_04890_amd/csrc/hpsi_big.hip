// Split-BF16 sector GEMMs of Eq. dgemm (Section 2.2.1) for large sector blocks (gfx950).
//
// A task Y += f A X B^T whose blocks are larger than the 96-wide LDS stages of hpsi_lds.hip runs as
// two GEMM passes over 128 x 128 workgroup tiles (4 wavefronts, 64 x 64 each):
//   pass 1  T'^T = X^T A^T   per task; P = X^T fragments (row order of k_pack_xt), Q = A rows; the
//                             result is scaled by f, re-split into hi/lo and stored as T tiles in the
//                             A-operand layout of pass 2 (the MFMA result layout of T'^T is exactly
//                             that layout, so no shuffle is needed)
//   pass 2  Y += sum_tasks T B^T   per target tile; K runs over every task of the item and its
//                             32-column chunks; P = T fragments, Q = B rows
// Each stage holds 16 tiles (32 KB) of both operands for one 32-wide k step, copied with
// global_load_lds_dwordx4 one stage ahead (two stages, 64 KB: two workgroups per CU). Tiles outside
// the operands are not copied; they only feed output positions that are never stored.
// Precision as in hpsi_lds.hip: hi.hi + hi.lo + lo.hi products with FP32 accumulation; pass 2 adds
// its FP32 sums into the FP64 output every kFlushBig tasks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dmrg {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr int kStageTiles = 16;
constexpr int kStageU16 = kStageTiles * kTileU16;
constexpr int kFlushBig = 8;

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(unsigned short h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }
__device__ __forceinline__ bf16x8 as_bf(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ f32x4 mma3(u16x8 ah, u16x8 al, u16x8 bh, u16x8 bl, f32x4 c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bh), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bl), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al), as_bf(bh), c, 0, 0, 0);
    return c;
}
__device__ __forceinline__ u16x8 lds8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Copy the 16 tiles of one stage: tile i (0..15) from (i < 8 ? p_base : q_base) + src[i] (u16
// offset, < 0: not present) to stage + i * kTileU16. 32 half-tile copies of 1 KB, 8 per wavefront.
__device__ __forceinline__ void copy_stage(const uint16_t* __restrict__ p_base, const uint16_t* __restrict__ q_base,
                                           const int64_t (&src)[kStageTiles], uint16_t* stage, int wave, int lane) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int h = wave * 8 + k, tile = h >> 1, part = h & 1;
        const uint16_t* base = tile < 8 ? p_base : q_base;
        if (src[tile] >= 0)
            __builtin_amdgcn_global_load_lds((const void*)(base + src[tile] + part * 512 + lane * 8),
                                             (lds_ptr_t)(stage + tile * kTileU16 + part * 512), 16, 0, 0);
    }
}

}  // namespace

// ------------------------------------------------------------------ pass 1: T = f A X per task
// One workgroup runs the groups [ranges[blockIdx.x], ranges[blockIdx.x + 1]) (each: one task's 8 row
// tiles x 4 column chunks) as one pipeline of k steps; at the end of a group its T tiles are stored.
__global__ __launch_bounds__(256) void k_big_t(const BigT1* __restrict__ work, const int32_t* __restrict__ ranges,
                                               const uint16_t* __restrict__ pool_t, const uint16_t* __restrict__ xt,
                                               uint16_t* __restrict__ tbuf, const int32_t* __restrict__ mask) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kStageU16];
    const int g_begin = uni(ranges[blockIdx.x]), g_end = uni(ranges[blockIdx.x + 1]);
    if (mask && mask[work[g_begin].part] != kPartActive) return;   // a workgroup's groups share one part
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wj = wave & 1, wr = wave >> 1;   // wave: chunks jb + 2 wj + {0,1}, row tiles rb + 4 wr + {0..3}
    struct G { int64_t x, a, t; float f; int pa32, pd32, nrt, rb, jb; };
    auto load_g = [&](int i) {
        const BigT1* wp = work + i;
        G d;
        d.x = uni64(wp->xt); d.a = uni64(wp->a); d.t = uni64(wp->t);
        d.f = (float)__builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, wp->f)));
        d.pa32 = uni(wp->pa32); d.pd32 = uni(wp->pd32); d.nrt = uni(wp->nrt); d.rb = uni(wp->rb); d.jb = uni(wp->jb);
        return d;
    };
    // stage (group, kt): tiles 0..7 = X^T (chunk jb + i/2, half i%2, kt), tiles 8..15 = A (row tile rb + i, kt)
    auto sources = [&](const G d, int kt, int64_t (&src)[kStageTiles]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int jc = d.jb + (i >> 1), h2 = i & 1;
            src[i] = jc < d.pd32 ? d.x + (int64_t)((jc * 2 + h2) * d.pa32 + kt) * kTileU16 : -1;
            const int rt = d.rb + i;
            src[8 + i] = rt < d.nrt ? d.a + (int64_t)(rt * d.pa32 + kt) * kTileU16 : -1;
        }
    };
    f32x4 acc[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[a][b][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto store = [&](const G d) {
        int ln = lane;   // opaque copy: keep the store addresses out of the main loop
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int jc = d.jb + 2 * wj + jj, rt = d.rb + 4 * wr + rr;
                if (jc < d.pd32 && rt < d.nrt) {
                    // acc[jj][h2][rr][v] = T'[row 16 rt + li][col 32 jc + 8 g + 4 h2 + v]
                    u16x8 th, tl;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float v = d.f * acc[jj][u >> 2][rr][u & 3];
                        const unsigned short hh = bf16_rne(v);
                        th[u] = hh;
                        tl[u] = bf16_rne(v - bf16_f32(hh));
                    }
                    uint16_t* dst = tbuf + d.t + (int64_t)(rt * d.pd32 + jc) * kTileU16 + ln * 8;
                    *reinterpret_cast<u16x8*>(dst) = th;
                    *reinterpret_cast<u16x8*>(dst + 512) = tl;
                }
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) acc[jj][h2][rr] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
    };

    int gi = g_begin, kt = 0;
    G cur = load_g(gi);
    {
        int64_t src[kStageTiles];
        sources(cur, 0, src);
        copy_stage(xt, pool_t, src, lds, wave, lane);
    }
    wait_vm();
    __syncthreads();
    int st = 0;
    for (;;) {
        int ngi = gi, nkt = kt + 1;
        if (nkt == cur.pa32) { ngi = gi + 1; nkt = 0; }
        const bool has_next = ngi < g_end;
        G nxt = cur;
        if (has_next) {
            if (ngi != gi) nxt = load_g(ngi);
            int64_t src[kStageTiles];
            sources(nxt, nkt, src);
            copy_stage(xt, pool_t, src, lds + (st ^ 1) * kStageU16, wave, lane);
        }
        const uint16_t* sp = lds + st * kStageU16 + lane * 8;
        u16x8 ph[2][2], pl[2][2], qh[4], ql[4];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const uint16_t* t = sp + ((2 * wj + jj) * 2 + h2) * kTileU16;
                ph[jj][h2] = lds8(t);
                pl[jj][h2] = lds8(t + 512);
            }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const uint16_t* t = sp + (8 + 4 * wr + rr) * kTileU16;
            qh[rr] = lds8(t);
            ql[rr] = lds8(t + 512);
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
                    acc[jj][h2][rr] = mma3(ph[jj][h2], pl[jj][h2], qh[rr], ql[rr], acc[jj][h2][rr]);
        if (ngi != gi) store(cur);        // last k step of the group
        wait_vm();
        __syncthreads();
        if (!has_next) break;
        gi = ngi; kt = nkt; cur = nxt;
        st ^= 1;
    }
}

// ------------------------------------------------------------------ pass 2: Y += sum T B^T per tile
__global__ __launch_bounds__(256) void k_big_y(const Item* __restrict__ items, const BigT2* __restrict__ tasks,
                                               const uint16_t* __restrict__ pool_t,
                                               const uint16_t* __restrict__ tbuf, double* __restrict__ y,
                                               double* __restrict__ part, const int32_t* __restrict__ mask) {
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kStageU16];
    const Item* ip = items + blockIdx.x;
    if (mask && mask[ip->part] != kPartActive) return;
    const int64_t y_off = uni64(ip->y_off), part_off = uni64(ip->part_off);
    const int m_ap = uni(ip->m_ap), m_dp = uni(ip->m_dp), r0 = uni(ip->r0), c0 = uni(ip->c0);
    const int t_begin = uni(ip->t_begin), t_end = uni(ip->t_end);
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wr = wave >> 1, wq = wave & 1;   // wave: row tiles rb + 4 wr + {0..3}, col tiles qb + 4 wq + {0..3}
    const int rb = r0 >> 4, qb = c0 >> 4;
    const int nrt = (m_ap + 15) >> 4, nq = (m_dp + 15) >> 4;
    const int tn = 16 * min(8, nq - qb);       // partial tile: rows [r0, r0 + 128), cols [c0, c0 + tn)

    // stage (task t, chunk jc): tiles 0..7 = T (row tile rb + i, jc), tiles 8..15 = B (col tile qb + i, jc)
    auto sources = [&](int64_t t_t, int64_t t_b, int pd32, int jc, int64_t (&src)[kStageTiles]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int rt = rb + i;
            src[i] = rt < nrt ? t_t + (int64_t)(rt * pd32 + jc) * kTileU16 : -1;
            const int q = qb + i;
            src[8 + i] = q < nq ? t_b + (int64_t)(q * pd32 + jc) * kTileU16 : -1;
        }
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    bool first_flush = true;
    auto flush = [&]() {
        // output addresses are recomputed here from an opaque copy of the lane id: hoisted out of the
        // main loop they would hold 64 address pairs in registers for the whole kernel
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const int fli = ln & 15, fg = ln >> 4;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int rt = rb + 4 * wr + rr, q = qb + 4 * wq + qq;
                if (rt < nrt && q < nq) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * rt + 4 * fg + v, col = 16 * q + fli;
                        if (part_off < 0) {
                            if (row < m_ap && col < m_dp) y[y_off + (int64_t)row * m_dp + col] += (double)acc[rr][qq][v];
                        } else {
                            double* d = part + part_off + (int64_t)(row - r0) * tn + (col - c0);
                            *d = first_flush ? (double)acc[rr][qq][v] : *d + (double)acc[rr][qq][v];
                        }
                    }
                    asm volatile("" ::: "memory");
                }
                acc[rr][qq] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        first_flush = false;
    };

    int t = t_begin, jc = 0;
    int64_t T_t = uni64(tasks[t].t), T_b = uni64(tasks[t].b);
    int T_pd = uni(tasks[t].pd32);
    {
        int64_t src[kStageTiles];
        sources(T_t, T_b, T_pd, 0, src);
        copy_stage(tbuf, pool_t, src, lds, wave, lane);
    }
    wait_vm();
    __syncthreads();
    int st = 0, since_flush = 0;
    for (;;) {
        // next stage
        int nt = t, njc = jc + 1;
        if (njc == T_pd) { nt = t + 1; njc = 0; }
        const bool has_next = nt < t_end;
        int64_t N_t = T_t, N_b = T_b;
        int N_pd = T_pd;
        if (has_next) {
            if (nt != t) { N_t = uni64(tasks[nt].t); N_b = uni64(tasks[nt].b); N_pd = uni(tasks[nt].pd32); }
            int64_t src[kStageTiles];
            sources(N_t, N_b, N_pd, njc, src);
            copy_stage(tbuf, pool_t, src, lds + (st ^ 1) * kStageU16, wave, lane);
        }
        const uint16_t* sp = lds + st * kStageU16 + lane * 8;
        u16x8 ph[4], pl[4], qh[4], ql[4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const uint16_t* p = sp + (4 * wr + rr) * kTileU16;
            ph[rr] = lds8(p);
            pl[rr] = lds8(p + 512);
        }
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const uint16_t* p = sp + (8 + 4 * wq + qq) * kTileU16;
            qh[qq] = lds8(p);
            ql[qq] = lds8(p + 512);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) acc[rr][qq] = mma3(ph[rr], pl[rr], qh[qq], ql[qq], acc[rr][qq]);
        if (nt != t || !has_next) {                 // task boundary
            if (++since_flush == kFlushBig || !has_next) { since_flush = 0; flush(); }
        }
        wait_vm();
        __syncthreads();
        if (!has_next) break;
        t = nt; jc = njc; T_t = N_t; T_b = N_b; T_pd = N_pd;
        st ^= 1;
    }
}

__global__ void k_reduce_big(const Reduce* __restrict__ red, const double* __restrict__ part, double* __restrict__ y,
                             const int32_t* __restrict__ mask) {
    const Reduce R = red[blockIdx.x];
    if (mask && mask[R.part] != kPartActive) return;
    const int n = R.tm * R.tn;
    const int e = blockIdx.y * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int rr = e / R.tn, cc = e - (e / R.tn) * R.tn;
    const int row = R.r0 + rr, col = R.c0 + cc;
    if (row >= R.m_ap || col >= R.m_dp) return;
    double s = 0.0;
    for (int k = 0; k < R.n_parts; ++k) s += part[R.part_off + (int64_t)k * n + e];
    y[R.y_off + (int64_t)row * R.m_dp + col] += s;
}

hipError_t launch_hpsi_big(const BigPlan& P, const uint16_t* pool_t, const uint16_t* xt, double* y, hipStream_t s,
                           const int32_t* active) {
    for (int c = 0; c < P.n_chunks; ++c) {
        const BigChunk& C = P.chunks[c];
        if (C.t1_end > C.t1_begin)
            hipLaunchKernelGGL(k_big_t, dim3(C.t1_end - C.t1_begin), dim3(256), 0, s, P.t1, P.t1_ranges + C.t1_begin,
                               pool_t, xt, P.tbuf, active);
        if (C.item_end > C.item_begin)
            hipLaunchKernelGGL(k_big_y, dim3(C.item_end - C.item_begin), dim3(256), 0, s, P.items + C.item_begin, P.t2,
                               pool_t, P.tbuf, y, P.partial, active);
        if (C.red_end > C.red_begin)
            hipLaunchKernelGGL(k_reduce_big, dim3(C.red_end - C.red_begin, P.red_chunks), dim3(256), 0, s,
                               P.reduces + C.red_begin, P.partial, y, active);
    }
    return hipGetLastError();
}

}  // namespace dmrg
