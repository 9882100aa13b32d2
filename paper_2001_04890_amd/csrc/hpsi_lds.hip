// LDS-staged split-BF16 sector GEMMs of Eq. dgemm (Section 2.2.1) for gfx950.
//
// One workgroup of NW compute wavefronts (kLdsWaves, or six of one row tile each for targets of
// 65..96 rows) owns a whole row block of a target psi block (every column) and loops over the
// target's tasks Y += f * A . X . B^T, sorted by source block. Wave w owns row tiles
// [TP w, TP w + TP) of the block; an optional extra wavefront only touches the cache lines of the
// task after next. Per task:
//   GEMM1  T'^T = X^T . A(rows)^T       A-operand: X^T fragments from LDS, B-operand: A rows held in
//                                       registers (loaded straight from the tiled pool)
//   GEMM2  Y   += T' . B^T              A-operand: T' (the MFMA result layout of GEMM1 is the
//                                       A-operand layout of GEMM2), B-operand: B fragments from LDS
// X^T (shared by the run of tasks with the same source) and B (per task) are copied into LDS with
// global_load_lds_dwordx4 one task ahead (two stages), so the copy of task k+1 and the A-fragment
// loads of task k+1 (branch-free: the compiler must not have to wait for them before task k's
// MFMAs) overlap the MFMAs of task k. Operands are stored pre-tiled in fragment order
// (internal.h), which makes every copy a contiguous 1 KB per wave instruction and every LDS read a
// conflict-free ds_read_b128 at lane * 16 bytes.
//
// Precision: each product a.b is a_hi b_hi + a_hi b_lo + a_lo b_hi on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation; T' is scaled by f and re-split; task results are accumulated in FP32 over at
// most kFlush tasks and then added into FP64 accumulators.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dmrg {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kFlush = 8;   // tasks accumulated in FP32 before the FP64 update

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
__device__ __forceinline__ u16x8 gld8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }
__device__ __forceinline__ u16x8 lds8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Copy n16 16-byte chunks (a multiple of 64) from global src to LDS dst, spread over the workgroup's
// waves; each wave instruction moves 64 consecutive chunks (lane i -> dst + 16 i).
template <int NW = kLdsWaves>
__device__ __forceinline__ void copy_to_lds(const uint16_t* __restrict__ src, uint16_t* dst, int n16, int wave,
                                            int lane) {
    for (int c = wave * 64; c < n16; c += NW * 64)
        __builtin_amdgcn_global_load_lds((const void*)(src + (int64_t)(c + lane) * 8), (lds_ptr_t)(dst + c * 8), 16,
                                         0, 0);
}

__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wave-uniform values in scalar registers (descriptors must not round-trip through scratch memory:
// a scratch reload waits on vmcnt and would drain the copies of the next task).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float unif(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Task descriptor held in scalar registers.
struct TD { int64_t x, a, b; float f; int pa32, pd32; };
__device__ __forceinline__ TD load_td(const LTask* __restrict__ p) {
    TD d;
    d.x = uni64(p->x_off);
    d.a = uni64(p->a_off);
    d.b = uni64(p->b_off);
    d.f = unif(p->f);
    d.pa32 = uni(p->pa32);
    d.pd32 = uni(p->pd32);
    return d;
}
struct ID { int64_t y_off, part_off; int m_ap, m_dp, r0, c0, t_begin, t_end; };
__device__ __forceinline__ ID load_item(const Item* __restrict__ p) {
    ID d;
    d.y_off = uni64(p->y_off);
    d.part_off = uni64(p->part_off);
    d.m_ap = uni(p->m_ap);
    d.m_dp = uni(p->m_dp);
    d.r0 = uni(p->r0);
    d.c0 = uni(p->c0);
    d.t_begin = uni(p->t_begin);
    d.t_end = uni(p->t_end);
    return d;
}

}  // namespace

// ------------------------------------------------------------------ operator pool -> tiled hi/lo
__global__ void k_split_tiled(const double* __restrict__ pool, const PoolBlock* __restrict__ blocks,
                              uint16_t* __restrict__ tiled) {
    const PoolBlock B = blocks[blockIdx.x];
    const int ld = B.k32 * 32;
    const int n = B.r16 * B.k32 * 64;   // lane slots
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int tile = e >> 6, lane = e & 63;
        const int rt = tile / B.k32, kt = tile - (tile / B.k32) * B.k32;
        const int row = rt * 16 + (lane & 15), col = kt * 32 + 8 * (lane >> 4);
        const double* src = pool + B.off + (int64_t)row * ld + col;
        u16x8 h, l;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double x = src[u];
            const unsigned short hh = bf16_rne((float)x);
            h[u] = hh;
            l[u] = bf16_rne((float)(x - (double)bf16_f32(hh)));
        }
        uint16_t* dst = tiled + 2 * B.off + (int64_t)tile * kTileU16 + lane * 8;
        *reinterpret_cast<u16x8*>(dst) = h;
        *reinterpret_cast<u16x8*>(dst + 512) = l;
    }
}

hipError_t launch_split_tiled(const double* pool, const PoolBlock* blocks, int n_blocks, uint16_t* tiled,
                              hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_tiled, dim3(n_blocks), dim3(256), 0, s, pool, blocks, tiled);
    return hipGetLastError();
}

// ------------------------------------------------------------------ psi -> tiled X^T (per matvec)
// Source block X (m_a x m_d, row-major in the caller's vector) -> X^T tiles: 32-row chunk jc of X^T
// (rows j = columns of X), half h2, k tile kt: lane l = (li, g) holds X^T[j][k] with
// j = 32 jc + 8 (li / 4) + li % 4 + 4 h2, k = 32 kt + 8 g + u. With this row order the GEMM1 result
// lane layout is the GEMM2 A-operand layout (see the kernel).
__global__ void k_pack_xt(const PackBlock* __restrict__ packs, const double* __restrict__ xall, int64_t n_coeff,
                          int64_t xt_size, uint16_t* __restrict__ xtall) {
    const PackBlock P = packs[blockIdx.x];
    const double* __restrict__ x = xall + (int64_t)blockIdx.y * n_coeff + P.src_off;
    uint16_t* __restrict__ xt = xtall + (int64_t)blockIdx.y * xt_size + 2 * P.dst_off;
    const int pa32 = P.pa / 32, pd32 = P.pd / 32;
    const int n = pd32 * 2 * pa32 * 64;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int tile = e >> 6, lane = e & 63;
        const int kt = tile % pa32, jh = tile / pa32;
        const int jc = jh >> 1, h2 = jh & 1;
        const int li = lane & 15, g = lane >> 4;
        const int j = 32 * jc + 8 * (li >> 2) + (li & 3) + 4 * h2;
        const int k0 = 32 * kt + 8 * g;
        u16x8 h, l;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            const double v = (j < P.m_d && k < P.m_a) ? x[(int64_t)k * P.m_d + j] : 0.0;
            const unsigned short hh = bf16_rne((float)v);
            h[u] = hh;
            l[u] = bf16_rne((float)(v - (double)bf16_f32(hh)));
        }
        uint16_t* dst = xt + (int64_t)tile * kTileU16 + lane * 8;
        *reinterpret_cast<u16x8*>(dst) = h;
        *reinterpret_cast<u16x8*>(dst + 512) = l;
    }
}

// ------------------------------------------------------------------ the sector-GEMM kernel
// S: largest padded dimension of the class (LDS stage size), TP: row tiles per wave. The item's
// column tile count tq = ceil((m_d' - c0) / 16) <= S / 16 is a runtime bound of unrolled loops.
// PF = 1: one more wavefront per workgroup touches, during task t, the cache lines of the operands
// of task t+2 (X^T if its source changes, B, and the workgroup's A rows) with loads into a scratch
// LDS word that nobody reads; it never waits for them, so the LDS copies of task t+2, issued by the
// compute waves one task later, find their lines in L2.
// NW compute wavefronts (16 TP rows each): kLdsWaves, or 3 for the (96, 2) class with a prefetch
// wavefront, whose targets have at most 96 rows, so the workgroup stays at four wavefronts.
// CW = 1 (with PF = 0): the extra wavefront is a copy wavefront instead, which issues every LDS copy
// of the item one task ahead, so the compute wavefronts never wait for copies in flight (the compiler
// makes the first LDS read after a global-to-LDS copy wait for it, per wavefront).
template <int S, int TP, int PF, int NW = kLdsWaves, int CW = 0>
__global__ __launch_bounds__(NW * 64 + PF * 64 + CW * 64) void k_hpsi_lds(const Item* __restrict__ items,
                                                             const LTask* __restrict__ tasks,
                                                             const uint16_t* __restrict__ pool_t,
                                                             const uint16_t* __restrict__ xtall,
                                                             double* __restrict__ yall, double* __restrict__ partall,
                                                             int64_t n_coeff, int64_t xt_size, int64_t slot_stride,
                                                             const int32_t* __restrict__ mask) {
    if (mask && mask[items[blockIdx.x].part] != kPartActive) return;   // whole workgroup, before any barrier
    constexpr int KS = S / 32;          // max k tiles (and j chunks) of a source
    constexpr int QS = S / 16;          // max column tiles of the target
    constexpr int XS = KS * 2 * KS * kTileU16;
    constexpr int BS = QS * KS * kTileU16;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * XS + 2 * BS + PF * 128];   // + touch target

    const ID I = load_item(items + blockIdx.x);
    const uint16_t* __restrict__ xt = xtall + (int64_t)blockIdx.y * xt_size;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    double* __restrict__ part = partall + (int64_t)blockIdx.y * slot_stride;
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int li = lane & 15, g = lane >> 4;
    const int nrt = (I.m_ap + 15) >> 4;                 // row tiles of the target block
    const int rt0 = (I.r0 >> 4) + wave * TP;            // this wave's first row tile
    const int qt0 = I.c0 >> 4;
    const int tq = min(QS, ((I.m_dp - I.c0) + 15) >> 4);
    const bool active = rt0 < nrt;

    if constexpr (PF == 1) {
        if (wave == NW) {
            const int rtw0 = I.r0 >> 4;
            const int nrow = min(NW * TP, nrt - rtw0);            // row tiles of the workgroup
            auto touch = [&](const TD P, bool with_x) {
                const int nxl = with_x ? P.pd32 * P.pa32 * 32 : 0;                 // 128-byte lines
                const int nbl = tq * P.pd32 * 16;
                const int n = nxl + nbl + nrow * P.pa32 * 16;
                const uint16_t* xb = xt + P.x;
                const uint16_t* bb = pool_t + P.b + (int64_t)qt0 * P.pd32 * kTileU16;
                const uint16_t* ab = pool_t + P.a + (int64_t)rtw0 * P.pa32 * kTileU16;
                for (int l0 = 0; l0 < n; l0 += 64) {
                    const int l = min(l0 + lane, n - 1);
                    const uint16_t* src = l < nxl ? xb + (int64_t)l * 64
                                        : l < nxl + nbl ? bb + (int64_t)(l - nxl) * 64
                                                        : ab + (int64_t)(l - nxl - nbl) * 64;
                    __builtin_amdgcn_global_load_lds((const void*)src, (lds_ptr_t)(lds + 2 * XS + 2 * BS), 4, 0, 0);
                }
            };
            // one barrier before the loop and one per task, as the compute waves
            int t = I.t_begin;
            TD Pp = load_td(tasks + t);
            if (t + 1 < I.t_end) {
                const TD P1 = load_td(tasks + t + 1);
                touch(P1, P1.x != Pp.x);
                Pp = P1;
            }
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            for (; t < I.t_end; ++t) {
                if (t + 2 < I.t_end) {
                    const TD P2 = load_td(tasks + t + 2);
                    touch(P2, P2.x != Pp.x);
                    Pp = P2;
                }
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_barrier();
            }
            wait_vm();   // the touches land in LDS: all of them before the wave ends
            return;
        }
    }

    f32x4 c32[TP][QS];
    double acc[TP][QS][4];
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            c32[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[p][q][v] = 0.0;
        }

    u16x8 ah[TP][KS], al[TP][KS];
    // Branch-free: a fragment outside the block (k tile >= pa32, or a row tile past the target) is
    // loaded from tile (0, 0) of the same block instead and never used for a stored result (the
    // GEMMs skip k tiles >= pa32; rows past the target are not stored). A conditional load merged
    // with a zero fragment would make the compiler wait for the load right away, which would
    // serialize this prefetch of the next task with the current task's GEMMs.
    auto load_a = [&](const TD T, u16x8 (&h)[TP][KS], u16x8 (&l)[TP][KS]) {
#pragma unroll
        for (int p = 0; p < TP; ++p)
#pragma unroll
            for (int kt = 0; kt < KS; ++kt) {
                const bool in = kt < T.pa32 && rt0 + p < nrt;
                const int64_t tile = in ? (int64_t)((rt0 + p) * T.pa32 + kt) : 0;
                const uint16_t* src = pool_t + T.a + tile * kTileU16 + lane * 8;
                h[p][kt] = gld8(src);
                l[p][kt] = gld8(src + 512);
            }
    };
    auto stage = [&](const TD T, int st, int xsl, bool load_x) {
        if (load_x) copy_to_lds<NW>(xt + T.x, lds + xsl * XS, T.pd32 * T.pa32 * 256, wave, lane);
        copy_to_lds<NW>(pool_t + T.b + (int64_t)qt0 * T.pd32 * kTileU16, lds + 2 * XS + st * BS, tq * T.pd32 * 128,
                    wave, lane);
    };

    static_assert(CW == 0 || PF == 0, "the extra wavefront copies or prefetches, not both");
    // per-task barrier: without a copy wavefront each wave waits for its own copies first; with one,
    // the compute waves only read LDS (their reads are consumed before the barrier) and the copy
    // wave waits for its copies
    auto task_barrier = [&]() {
        if constexpr (CW == 0) {
            wait_vm();
            __syncthreads();
        } else {
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        }
    };
    int t = I.t_begin;
    TD T = load_td(tasks + t);
    int st = 0, xsl = 0;
    int64_t xcur = T.x;
    TD Tn = t + 1 < I.t_end ? load_td(tasks + t + 1) : T;   // descriptors are read one task ahead of use
    if constexpr (CW == 1) {
        if (wave == NW) {
            auto stage1 = [&](const TD P, int st1, int xsl1, bool load_x) {
                if (load_x) copy_to_lds<1>(xt + P.x, lds + xsl1 * XS, P.pd32 * P.pa32 * 256, 0, lane);
                copy_to_lds<1>(pool_t + P.b + (int64_t)qt0 * P.pd32 * kTileU16, lds + 2 * XS + st1 * BS,
                               tq * P.pd32 * 128, 0, lane);
            };
            stage1(T, 0, 0, true);
            wait_vm();
            task_barrier();
            for (; t + 1 < I.t_end; ++t) {
                const bool nx = Tn.x != xcur;
                if (nx) xsl ^= 1;
                stage1(Tn, st ^ 1, xsl, nx);          // that stage was last read before the previous barrier
                wait_vm();
                task_barrier();
                st ^= 1;
                xcur = Tn.x;
                Tn = t + 2 < I.t_end ? load_td(tasks + t + 2) : Tn;
            }
            task_barrier();                           // the compute waves' barrier after their last task
            return;
        }
    }
    if constexpr (CW == 0) stage(T, 0, 0, true);
    load_a(T, ah, al);
    if constexpr (CW == 0) wait_vm();
    task_barrier();
    int since_flush = 0;
    for (;;) {
        const bool has_next = t + 1 < I.t_end;
        const TD Tnn = t + 2 < I.t_end ? load_td(tasks + t + 2) : Tn;
        int xsl_n = xsl;
        u16x8 nh[TP][KS], nl[TP][KS];
        if (has_next) {
            const bool nx = Tn.x != xcur;
            if (nx) xsl_n ^= 1;
            if constexpr (CW == 0) stage(Tn, st ^ 1, xsl_n, nx);
            load_a(Tn, nh, nl);
        }
        if (active) {
            const uint16_t* xs = lds + xsl * XS;
            const uint16_t* bs = lds + 2 * XS + st * BS;
            const float f = T.f;
            for (int jc = 0; jc < T.pd32; ++jc) {
                f32x4 tt[2][TP];
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                    for (int p = 0; p < TP; ++p) tt[h2][p] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < KS; ++kt) {
                    if (kt < T.pa32) {
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2) {
                            const uint16_t* tl = xs + ((jc * 2 + h2) * T.pa32 + kt) * kTileU16 + lane * 8;
                            const u16x8 xh = lds8(tl), xl = lds8(tl + 512);
#pragma unroll
                            for (int p = 0; p < TP; ++p) tt[h2][p] = mma3(xh, xl, ah[p][kt], al[p][kt], tt[h2][p]);
                        }
                    }
                }
                // tt[h2][p][v] = T'[row 16 (rt0 + p) + li][col 32 jc + 8 g + 4 h2 + v] (unscaled)
                u16x8 th[TP], tlo[TP];
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float v = f * tt[u >> 2][p][u & 3];
                        const unsigned short hh = bf16_rne(v);
                        th[p][u] = hh;
                        tlo[p][u] = bf16_rne(v - bf16_f32(hh));
                    }
#pragma unroll
                for (int q = 0; q < QS; ++q) {
                    if (q < tq) {
                        const uint16_t* tl = bs + (q * T.pd32 + jc) * kTileU16 + lane * 8;
                        const u16x8 bh = lds8(tl), bl = lds8(tl + 512);
#pragma unroll
                        for (int p = 0; p < TP; ++p) c32[p][q] = mma3(th[p], tlo[p], bh, bl, c32[p][q]);
                    }
                }
            }
            if (++since_flush == kFlush || !has_next) {
                since_flush = 0;
#pragma unroll
                for (int p = 0; p < TP; ++p)
#pragma unroll
                    for (int q = 0; q < QS; ++q) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[p][q][v] += (double)c32[p][q][v];
                        c32[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        task_barrier();
        if (!has_next) break;
        ++t;
        T = Tn;
        Tn = Tnn;
        st ^= 1;
        xsl = xsl_n;
        xcur = T.x;
#pragma unroll
        for (int p = 0; p < TP; ++p)
#pragma unroll
            for (int kt = 0; kt < KS; ++kt) {
                ah[p][kt] = nh[p][kt];
                al[p][kt] = nl[p][kt];
            }
    }
    if (!active) return;
    // store: lane (li, g) holds Y[16 (rt0 + p) + 4 g + v][16 (qt0 + q) + li]
    const int tn = 16 * tq;
#pragma unroll
    for (int p = 0; p < TP; ++p)
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            if (q >= tq || rt0 + p >= nrt) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * (rt0 + p) + 4 * g + v, col = 16 * (qt0 + q) + li;
                if (I.part_off < 0) {
                    if (row < I.m_ap && col < I.m_dp) y[I.y_off + (int64_t)row * I.m_dp + col] += acc[p][q][v];
                } else {
                    part[I.part_off + (int64_t)(row - I.r0) * tn + (col - I.c0)] = acc[p][q][v];
                }
            }
        }
}

// ------------------------------------------------------------------ task-mode kernel (small sources)
// For tasks whose source block fits one 32 x 32 tile (pa32 = pd32 = 1). One wavefront owns a row
// block of NR row tiles (every column, tq <= NQ column tiles) of a target and runs its tasks in
// order with every operand fragment read straight from global memory (1 KB coalesced per wave
// instruction); the fragments of task t+1 are loaded while task t computes, and many independent
// wavefronts per CU hide the remaining latency. Results are accumulated in FP32 over kFlushT tasks
// and added into the FP64 output (y, or the item's partial tile) by read-modify-write: the item
// is the only writer of those elements in its launch.
constexpr int kFlushT = 32;

template <int NR, int NQ>
__global__ __launch_bounds__(64) void k_hpsi_small(const Item* __restrict__ items, const LTask* __restrict__ tasks,
                                                   const uint16_t* __restrict__ pool_t,
                                                   const uint16_t* __restrict__ xtall, double* __restrict__ yall,
                                                   double* __restrict__ partall, int64_t n_coeff, int64_t xt_size,
                                                   int64_t slot_stride, const int32_t* __restrict__ mask) {
    if (mask && mask[items[blockIdx.x].part] != kPartActive) return;
    const ID I = load_item(items + blockIdx.x);
    const uint16_t* __restrict__ xt = xtall + (int64_t)blockIdx.y * xt_size;
    double* __restrict__ y = yall + (int64_t)blockIdx.y * n_coeff;
    double* __restrict__ part = partall + (int64_t)blockIdx.y * slot_stride;
    const int lane = threadIdx.x & 63;
    const int rt0 = I.r0 >> 4, qt0 = I.c0 >> 4;
    const int nr = min(NR, ((I.m_ap + 15) >> 4) - rt0);
    const int tq = min(NQ, ((I.m_dp - I.c0) + 15) >> 4);
    const int tn = 16 * tq;

    // operand fragments of one task: A rows, X^T (two halves), B rows; hi and lo
    u16x8 ah[NR], al[NR], xh[2], xl[2], bh[NQ], bl[NQ];
    u16x8 nah[NR], nal[NR], nxh[2], nxl[2], nbh[NQ], nbl[NQ];
    // Branch-free loads (a conditional load merged with a zero or kept fragment makes the compiler
    // wait for it at once, serializing the prefetch of task t+1 with task t): row tiles past the
    // target and column tiles past tq read the block's first tile instead and are never stored; the
    // X^T fragments are re-read even when the source is unchanged (a cache hit).
    auto load = [&](const TD T, u16x8 (&fah)[NR], u16x8 (&fal)[NR], u16x8 (&fxh)[2], u16x8 (&fxl)[2],
                    u16x8 (&fbh)[NQ], u16x8 (&fbl)[NQ]) {
#pragma unroll
        for (int p = 0; p < NR; ++p) {
            const uint16_t* src = pool_t + T.a + (int64_t)(p < nr ? rt0 + p : rt0) * kTileU16 + lane * 8;
            fah[p] = gld8(src);
            fal[p] = gld8(src + 512);
        }
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            const uint16_t* src = xt + T.x + h2 * kTileU16 + lane * 8;
            fxh[h2] = gld8(src);
            fxl[h2] = gld8(src + 512);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const uint16_t* src = pool_t + T.b + (int64_t)(q < tq ? qt0 + q : qt0) * kTileU16 + lane * 8;
            fbh[q] = gld8(src);
            fbl[q] = gld8(src + 512);
        }
    };

    f32x4 c32[NR][NQ];
#pragma unroll
    for (int p = 0; p < NR; ++p)
#pragma unroll
        for (int q = 0; q < NQ; ++q) c32[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    bool first_flush = true;
    auto flush = [&]() {
        // addresses from an opaque copy of the lane id, so they are not hoisted into the main loop
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const int fli = ln & 15, fg = ln >> 4;
#pragma unroll
        for (int p = 0; p < NR; ++p)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (p < nr && q < tq) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * (rt0 + p) + 4 * fg + v, col = 16 * (qt0 + q) + fli;
                        if (I.part_off < 0) {
                            if (row < I.m_ap && col < I.m_dp)
                                y[I.y_off + (int64_t)row * I.m_dp + col] += (double)c32[p][q][v];
                        } else {
                            double* d = part + I.part_off + (int64_t)(row - I.r0) * tn + (col - I.c0);
                            *d = first_flush ? (double)c32[p][q][v] : *d + (double)c32[p][q][v];
                        }
                    }
                    // keep the read-modify-writes of one tile together (bounded register use)
                    asm volatile("" ::: "memory");
                }
                c32[p][q] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        first_flush = false;
    };

    int t = I.t_begin;
    TD T = load_td(tasks + t);
    TD Tn = t + 1 < I.t_end ? load_td(tasks + t + 1) : T;
    load(T, ah, al, xh, xl, bh, bl);
    // nothing outstanding at the loop head: the first task's fragments are complete here, and each
    // iteration's prefetch completes at its end (the copies into the current-task registers), so the
    // compiler's wait analysis lets this task's GEMMs run while the next task's loads are in flight
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0) expcnt(7) lgkmcnt(15)
    int since_flush = 0;
    for (;;) {
        const bool has_next = t + 1 < I.t_end;
        const TD Tnn = t + 2 < I.t_end ? load_td(tasks + t + 2) : Tn;
        if (has_next) load(Tn, nah, nal, nxh, nxl, nbh, nbl);
        // GEMM1: T'^T (32 x 16 per row tile) = X^T A(rows)^T, one k step (K = 32)
        f32x4 tt[2][NR];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
            for (int p = 0; p < NR; ++p)
                tt[h2][p] = mma3(xh[h2], xl[h2], ah[p], al[p], f32x4{0.f, 0.f, 0.f, 0.f});
        u16x8 th[NR], tlo[NR];
        const float f = T.f;
#pragma unroll
        for (int p = 0; p < NR; ++p)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float v = f * tt[u >> 2][p][u & 3];
                const unsigned short hh = bf16_rne(v);
                th[p][u] = hh;
                tlo[p][u] = bf16_rne(v - bf16_f32(hh));
            }
        // GEMM2: Y += T' B^T
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q < tq) {
#pragma unroll
                for (int p = 0; p < NR; ++p) c32[p][q] = mma3(th[p], tlo[p], bh[q], bl[q], c32[p][q]);
            }
        }
        if (++since_flush == kFlushT || !has_next) {
            since_flush = 0;
            flush();
        }
        if (!has_next) break;
        ++t;
        T = Tn;
        Tn = Tnn;
#pragma unroll
        for (int p = 0; p < NR; ++p) { ah[p] = nah[p]; al[p] = nal[p]; }
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) { xh[h2] = nxh[h2]; xl[h2] = nxl[h2]; }
#pragma unroll
        for (int q = 0; q < NQ; ++q) { bh[q] = nbh[q]; bl[q] = nbl[q]; }
    }
}

// y_tile += sum of its partial tiles, in item order; block (record, 256-element chunk), one element
// per thread
__global__ void k_reduce_lds(const Reduce* __restrict__ red, const double* __restrict__ partall,
                             double* __restrict__ yall, int64_t n_coeff, int64_t part_stride,
                             const int32_t* __restrict__ mask) {
    const Reduce R = red[blockIdx.x];
    if (mask && mask[R.part] != kPartActive) return;
    const int n = R.tm * R.tn;
    const int e = blockIdx.z * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int rr = e / R.tn, cc = e - (e / R.tn) * R.tn;
    const int row = R.r0 + rr, col = R.c0 + cc;
    if (row >= R.m_ap || col >= R.m_dp) return;
    const double* __restrict__ part = partall + (int64_t)blockIdx.y * part_stride + R.part_off;
    double s = 0.0;
    for (int k = 0; k < R.n_parts; ++k) s += part[(int64_t)k * n + e];
    yall[(int64_t)blockIdx.y * n_coeff + R.y_off + (int64_t)row * R.m_dp + col] += s;
}

hipError_t launch_reduce_partials(const Reduce* reduces, int n, int chunks, const double* partial, double* y,
                                  hipStream_t s, const int32_t* active) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_lds, dim3(n, 1, chunks), dim3(256), 0, s, reduces, partial, y, (int64_t)0, (int64_t)0,
                       active);
    return hipGetLastError();
}

__global__ void k_zero_lds(double* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 0.0;
}

hipError_t launch_hpsi_lds(const LdsPlan& P, const uint16_t* pool_t, const double* x, double* y, int64_t n_coeff,
                           int nvec, bool zero_y, hipStream_t s, const int32_t* active) {
    if (zero_y) {
        int64_t n = n_coeff * nvec, blocks = (n + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_zero_lds, dim3((unsigned)blocks), dim3(256), 0, s, y, n);
    }
    if (P.n_packs == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_pack_xt, dim3(P.n_packs, nvec), dim3(256), 0, s, P.packs, x, n_coeff, P.xt_size, P.xt);
    const int64_t ss = P.partial_size;
    for (int c = 0; c < kLdsClasses; ++c) {
        const int b = P.cls_begin[c], n = P.cls_begin[c + 1] - b;
        if (n <= 0) continue;
        const dim3 grid(n, nvec), block(kLdsWaves * 64), block_pf(kLdsWaves * 64 + 64);
        const bool cw = (P.copy_wave_mask >> c) & 1;     // a copy wavefront (replaces the prefetch one)
        const bool pf = !cw && ((P.prefetch_mask >> c) & 1);
        const bool w6 = (P.six_wave_mask >> c) & 1;      // (S, 2) classes as six one-row-tile wavefronts
        const dim3 block6(6 * 64), block6_pf(7 * 64);
        if (cw) {
#define DMRG_LDS_CW(S_, TP_, NW_)                                                                          \
    hipLaunchKernelGGL((k_hpsi_lds<S_, TP_, 0, NW_, 1>), grid, dim3((NW_ + 1) * 64), 0, s, P.items + b, P.tasks, \
                       pool_t, P.xt, y, P.partial, n_coeff, P.xt_size, ss, active)
            switch (c) {
                case 0: DMRG_LDS_CW(64, 1, kLdsWaves); break;
                case 1:
                    if (w6) DMRG_LDS_CW(64, 1, 6);
                    else DMRG_LDS_CW(64, 2, kLdsWaves);
                    break;
                case 2: DMRG_LDS_CW(96, 1, kLdsWaves); break;
                default:
                    if (w6) DMRG_LDS_CW(96, 1, 6);
                    else DMRG_LDS_CW(96, 2, kLdsWaves);
                    break;
            }
#undef DMRG_LDS_CW
            continue;
        }
        switch (c) {
            case 0:
                if (pf) hipLaunchKernelGGL((k_hpsi_lds<64, 1, 1>), grid, block_pf, 0, s, P.items + b, P.tasks, pool_t,
                                           P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else hipLaunchKernelGGL((k_hpsi_lds<64, 1, 0>), grid, block, 0, s, P.items + b, P.tasks, pool_t, P.xt,
                                        y, P.partial, n_coeff, P.xt_size, ss, active);
                break;
            case 1:
                if (w6) hipLaunchKernelGGL((k_hpsi_lds<64, 1, 0, 6>), grid, block6, 0, s, P.items + b, P.tasks, pool_t,
                                           P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else if (pf) hipLaunchKernelGGL((k_hpsi_lds<64, 2, 1>), grid, block_pf, 0, s, P.items + b, P.tasks,
                                                pool_t, P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else hipLaunchKernelGGL((k_hpsi_lds<64, 2, 0>), grid, block, 0, s, P.items + b, P.tasks, pool_t, P.xt,
                                        y, P.partial, n_coeff, P.xt_size, ss, active);
                break;
            case 2:
                if (pf) hipLaunchKernelGGL((k_hpsi_lds<96, 1, 1>), grid, block_pf, 0, s, P.items + b, P.tasks, pool_t,
                                           P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else hipLaunchKernelGGL((k_hpsi_lds<96, 1, 0>), grid, block, 0, s, P.items + b, P.tasks, pool_t, P.xt,
                                        y, P.partial, n_coeff, P.xt_size, ss, active);
                break;
            default:   // with prefetch: 3 compute wavefronts (targets of at most 96 rows) + the prefetch one
                if (w6 && pf) hipLaunchKernelGGL((k_hpsi_lds<96, 1, 1, 6>), grid, block6_pf, 0, s, P.items + b,
                                                 P.tasks, pool_t, P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else if (w6) hipLaunchKernelGGL((k_hpsi_lds<96, 1, 0, 6>), grid, block6, 0, s, P.items + b, P.tasks,
                                                pool_t, P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else if (pf) hipLaunchKernelGGL((k_hpsi_lds<96, 2, 1, 3>), grid, block, 0, s, P.items + b, P.tasks,
                                                pool_t, P.xt, y, P.partial, n_coeff, P.xt_size, ss, active);
                else hipLaunchKernelGGL((k_hpsi_lds<96, 2, 0>), grid, block, 0, s, P.items + b, P.tasks, pool_t, P.xt,
                                        y, P.partial, n_coeff, P.xt_size, ss, active);
                break;
        }
    }
    for (int c = 0; c < kSmallClasses; ++c) {
        const int b = P.small_begin[c], n = P.small_begin[c + 1] - b;
        if (n <= 0) continue;
        const dim3 grid(n, nvec), block(64);
#define DMRG_SMALL(NR, NQ) hipLaunchKernelGGL((k_hpsi_small<NR, NQ>), grid, block, 0, s, P.items + b, P.tasks, pool_t, \
                                              P.xt, y, P.partial, n_coeff, P.xt_size, ss, active)
        switch (c) {
            case 0: DMRG_SMALL(1, 2); break;
            case 1: DMRG_SMALL(2, 2); break;
            default: DMRG_SMALL(1, 4); break;
        }
#undef DMRG_SMALL
    }
    // one launch per record kind: the records of one launch touch disjoint parts of y
    for (int k = 0; k < kReduceKinds; ++k) {
        const int nr = P.red_begin[k + 1] - P.red_begin[k];
        if (nr > 0)
            hipLaunchKernelGGL(k_reduce_lds, dim3(nr, nvec, P.red_chunks[k]), dim3(256), 0, s, P.reduces + P.red_begin[k],
                               P.partial, y, n_coeff, P.partial_size, active);
    }
    return hipGetLastError();
}

}  // namespace dmrg
