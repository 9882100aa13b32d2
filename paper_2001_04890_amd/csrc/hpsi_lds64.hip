// LDS-staged FP64 sector GEMMs of Eq. dgemm (Section 2.2.1) for gfx950, on v_mfma_f64_16x16x4f64
// with FP64 accumulation.
//
// One workgroup of W wavefronts (6 or 7) owns a whole target psi block of at most 16 W x 16 W (every
// row and column) and loops over a range of its tasks Y += f * A . X . B^T (sorted by source block); wave w
// owns row tile w (waves past the target's rows only help with the copies). The tasks are cut into
// steps, one per 16-wide column tile jc of the source (the tiles that hold data), and per step:
//   GEMM1  T'(w, jc)^T = X^T(jc, :) . A(w, :)^T   A-operand: the X^T slice from LDS; B-operand: the
//                                                  wave's A row tile, held in registers for the
//                                                  whole task (read straight from the tiled pool)
//   GEMM2  Y(w, :)   += f T'(w, jc) . B(:, jc)^T  A-operand: T' (the MFMA result layout of GEMM1 is
//                                                  the tile format, i.e. the A-operand layout of
//                                                  GEMM2); B-operand: the B slice from LDS
// The step's X^T slice (at most KT tiles) and B slice (at most QT tiles) are copied into one of two
// LDS slots with global_load_lds_dwordx4 (2 KB tiles, 1 KB per wave instruction), issued before the
// previous step computes; every operand read is a contiguous 32 bytes per lane. All wavefronts share
// each staged slice, so a task reads its X and B blocks once per workgroup rather than once per
// output tile. The compiler cannot tell which LDS such a copy writes and makes the step's first LDS
// read wait for the copies in flight, so the latency is hidden across workgroups rather than inside
// one: a slot is (KT + QT) tiles, at most 24 KB, and two to four workgroups share a CU (measured:
// staging through registers instead, which removes that wait, is slower at these sizes, as the extra
// registers cost a workgroup per CU). The A rows of the next task are read during the last step's
// GEMM2.
// Consecutive MFMAs accumulate into the same registers, the fast path of the matrix core.
//
// Tile format (internal.h, hpsi_big64.hip): a 16 x 16 tile holds M[16 rt + li][16 kt + 4 v + g] in
// lane (li, g) = (l % 16, l / 16), value v.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dmrg {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr int kTileD = 256;   // doubles per 16 x 16 tile

__device__ __forceinline__ f64x4 ld4g(const double* p) { return *reinterpret_cast<const f64x4*>(p); }
__device__ __forceinline__ f64x4 ld4s(const double* p) { return *reinterpret_cast<const f64x4*>(p); }
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double unid(double v) {
    return __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, v)));
}

// Task descriptor in scalar registers (offsets in doubles; pa16 / pd16: tile strides of the source's
// rows / columns; ka16 / kd16: the tiles of them that hold data).
struct TD { int64_t x, a, b; double f; int pa16, pd16, ka16, kd16; };
__device__ __forceinline__ TD load_td(const LTask64* __restrict__ p) {
    TD d;
    d.x = uni64(p->x_off);
    d.a = uni64(p->a_off);
    d.b = uni64(p->b_off);
    d.f = unid(p->f);
    d.pa16 = uni(p->pa16);
    d.pd16 = uni(p->pd16);
    d.ka16 = uni(p->ka16);
    d.kd16 = uni(p->kd16);
    return d;
}

}  // namespace

// KT: most k tiles (source rows in 16-wide tiles) of the item's tasks; QT: most column tiles of the
// target; W: wavefronts, at least the target's row tiles; MINW: wavefronts per SIMD the register
// allocation must allow (4 holds the 7-wavefront class to 128 VGPRs, so that two of its workgroups
// share a CU, at the price of a few spilled registers).
// NS: LDS slots; 3 (with the copy wavefront) puts the copies two steps ahead of the compute
// wavefronts instead of one, for classes whose steps are short against the copy latency.
template <int KT, int QT, int W, int MINW, int CW, int NS = 2>
__global__ __launch_bounds__((W + CW) * 64, MINW) void k_hpsi_lds64(const Item* __restrict__ items,
                                                                const LTask64* __restrict__ tasks,
                                                                const double* __restrict__ pool_t,
                                                                const double* __restrict__ xt,
                                                                double* __restrict__ y, double* __restrict__ part,
                                                                const int32_t* __restrict__ mask) {
    if (mask && mask[items[blockIdx.x].part] != kPartActive) return;   // whole workgroup, before any barrier
    static_assert(NS == 2 || (NS == 3 && CW == 1), "three slots need the copy wavefront");
    constexpr int SLOT = (KT + QT) * kTileD;   // doubles of one slot: X^T slice, then B slice
    __shared__ __attribute__((aligned(16))) double lds[NS * SLOT];

    const Item I = items[blockIdx.x];
    const int64_t y_off = uni64(I.y_off), part_off = uni64(I.part_off);
    const int m_ap = uni(I.m_ap), m_dp = uni(I.m_dp);
    const int t_begin = uni(I.t_begin), t_end = uni(I.t_end);
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int li = lane & 15, g = lane >> 4;
    const int nrt = (m_ap + 15) >> 4;
    const int tq = min(QT, (m_dp + 15) >> 4);
    const bool active = wave < nrt;

    f64x4 acc[QT];
#pragma unroll
    for (int q = 0; q < QT; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};

    // the wave's A row tile of a task: tiles (wave, kt); outside the source (kt >= ka16) or past the
    // target the block's first tile is read instead and never used (branch-free, so the loads stay
    // in flight)
    auto load_a = [&](const TD& T, f64x4 (&ar)[KT]) {
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
            const bool in = kt < T.ka16 && active;
            const int64_t tile = in ? (int64_t)wave * T.pa16 + kt : 0;
            ar[kt] = ld4g(pool_t + T.a + tile * kTileD + lane * 4);
        }
    };
    // copy the operands of step (T, jc) into a slot: X^T tiles (jc, kt < ka16), contiguous in the
    // tiled X^T, then B tiles (q < tq, jc), one per target column tile; half tiles h0, h0 + hs, ...
    // nfix > 0: exactly nfix copy instructions (the last copy repeated: the same bytes to the same
    // place), so that a wait for all but the newest nfix copies waits for every earlier step
    auto stage = [&](const TD& T, int jc, int slot, int h0, int hs, int nfix = 0) {
        double* d = lds + slot * SLOT;
        const double* xs = xt + T.x + (int64_t)jc * T.pa16 * kTileD;
        const int nx = 2 * T.ka16, n = nx + 2 * tq;
        const int nend = nfix > 0 ? nfix : n;
        for (int h0i = h0; h0i < nend; h0i += hs) {
            const int h = h0i < n ? h0i : n - 1;
            const double* src;
            double* dst;
            if (h < nx) {
                src = xs + h * 128;
                dst = d + h * 128;
            } else {
                const int q = (h - nx) >> 1, half = (h - nx) & 1;
                src = pool_t + T.b + ((int64_t)q * T.pd16 + jc) * kTileD + half * 128;
                dst = d + (KT + q) * kTileD + half * 128;
            }
            __builtin_amdgcn_global_load_lds((const void*)(src + lane * 2), (lds_ptr_t)dst, 16, 0, 0);
        }
    };
    auto next_slot = [](int sl) { return sl + 1 == NS ? 0 : sl + 1; };

    // barrier of the step loop: CW = 0, every wave copies (waits for its copies, then the barrier);
    // CW = 1, the compute waves only read LDS (whose values the MFMAs have consumed by then), so a
    // bare barrier, while the copy wave waits for its copies before it
    auto step_barrier = [&]() {
        if constexpr (CW == 0) {
            wait_vm();
            __syncthreads();
        } else {
            asm volatile("" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        }
    };
    int t = t_begin, jc = 0, slot = 0;
    TD T = load_td(tasks + t);
    if constexpr (CW == 1 && NS == 3) {
        if (wave == W) {
            // the copy wavefront, two steps ahead: while the compute wavefronts run step s it issues the
            // copies of step s + 2 (exactly kCopies instructions per step) and then waits for those of
            // step s + 1 (every copy but the newest kCopies), before the barrier that starts step s + 1
            constexpr int kCopies = 2 * (KT + QT);
            static_assert(kCopies < 64, "vmcnt holds at most 63");
            constexpr int kWait = (kCopies & 15) | (7 << 4) | (15 << 8) | (((kCopies >> 4) & 3) << 14);
            struct Step { int t, jc; TD T; bool ok; };
            auto advance = [&](Step& c) {
                if (!c.ok) return;
                if (c.jc + 1 < c.T.kd16) {
                    ++c.jc;
                } else if (c.t + 1 < t_end) {
                    ++c.t;
                    c.jc = 0;
                    c.T = load_td(tasks + c.t);
                } else {
                    c.ok = false;
                }
            };
            Step s1{t, 0, T, true};               // the step after the compute waves' current one
            stage(s1.T, 0, 0, 0, 1, kCopies);
            advance(s1);
            int sl = 1;                            // slot of step s1
            if (s1.ok) {
                stage(s1.T, s1.jc, sl, 0, 1, kCopies);
                asm volatile("" ::: "memory");
                __builtin_amdgcn_s_waitcnt(kWait);
                asm volatile("" ::: "memory");
            } else {
                wait_vm();
            }
            step_barrier();
            while (s1.ok) {
                Step s2 = s1;
                advance(s2);
                const int sl2 = next_slot(sl);
                if (s2.ok) {
                    stage(s2.T, s2.jc, sl2, 0, 1, kCopies);   // slot read by the compute waves before the last barrier
                    asm volatile("" ::: "memory");
                    __builtin_amdgcn_s_waitcnt(kWait);
                    asm volatile("" ::: "memory");
                } else {
                    wait_vm();
                }
                step_barrier();
                s1 = s2;
                sl = sl2;
            }
            step_barrier();                           // the compute waves' barrier after their last step
            return;
        }
    }
    if constexpr (CW == 1 && NS == 2) {
        if (wave == W) {
            // the copy wavefront: every copy of the item, one step ahead of the compute wavefronts,
            // which then never wait for a copy in flight (the wait before an LDS read that the
            // compiler puts after a global-to-LDS copy is per wavefront)
            stage(T, 0, 0, 0, 1);
            wait_vm();
            step_barrier();
            for (;;) {
                const bool more_cols = jc + 1 < T.kd16;
                const bool new_task = !more_cols && t + 1 < t_end;
                if (!more_cols && !new_task) break;
                const TD Tn = new_task ? load_td(tasks + t + 1) : T;
                stage(Tn, more_cols ? jc + 1 : 0, slot ^ 1, 0, 1);   // last read before the previous barrier
                wait_vm();
                step_barrier();
                if (more_cols) {
                    ++jc;
                } else {
                    ++t;
                    jc = 0;
                    T = Tn;
                }
                slot ^= 1;
            }
            step_barrier();                           // the compute waves' barrier after their last step
            return;
        }
    }
    f64x4 ar[KT];
    if constexpr (CW == 0) stage(T, 0, 0, wave, W);
    load_a(T, ar);
    if constexpr (CW == 0) wait_vm();
    step_barrier();
    for (;;) {
        const bool more_cols = jc + 1 < T.kd16;
        const bool new_task = !more_cols && t + 1 < t_end;
        const bool has_next = more_cols || new_task;
        TD Tn = T;
        if (new_task) Tn = load_td(tasks + t + 1);
        if constexpr (CW == 0)
            if (has_next) stage(Tn, more_cols ? jc + 1 : 0, next_slot(slot), wave, W);   // last read before the previous barrier
        const double* xs = lds + slot * SLOT;
        const double* bs = xs + KT * kTileD;
        f64x4 tt = f64x4{0.0, 0.0, 0.0, 0.0};
        if (active) {
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                if (kt < T.ka16) {
                    const f64x4 xv = ld4s(xs + kt * kTileD + lane * 4);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        tt = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[v], ar[kt][v], tt, 0, 0, 0);
                }
            }
        }
        // tt[v] = T'[16 wave + li][16 jc + 4 v + g] (unscaled); the A rows are free now
        if (new_task) load_a(Tn, ar);
        if (active) {
            tt *= T.f;
#pragma unroll
            for (int q = 0; q < QT; ++q) {
                if (q < tq) {
                    const f64x4 bv = ld4s(bs + q * kTileD + lane * 4);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(tt[v], bv[v], acc[q], 0, 0, 0);
                }
            }
        }
        step_barrier();
        if (!has_next) break;
        if (more_cols) {
            ++jc;
        } else {
            ++t;
            jc = 0;
            T = Tn;
        }
        slot = next_slot(slot);
    }
    if (!active) return;
    // store: lane (li, g) holds Y[16 wave + g + 4 v][16 q + li]
    const int tn = 16 * tq;
#pragma unroll
    for (int q = 0; q < QT; ++q) {
        if (q >= tq) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * wave + g + 4 * v, col = 16 * q + li;
            if (part_off < 0) {
                if (row < m_ap && col < m_dp) y[y_off + (int64_t)row * m_dp + col] += acc[q][v];
            } else {
                part[part_off + (int64_t)row * tn + col] = acc[q][v];
            }
        }
    }
}

hipError_t launch_hpsi_lds64(const LdsPlan64& P, const double* pool_t, const double* xt, double* y, hipStream_t s,
                             const int32_t* active) {
    if (P.n_items == 0) return hipSuccess;
    for (int c = 0; c < kLds64Classes; ++c) {
        const int b = P.cls_begin[c], n = P.cls_begin[c + 1] - b;
        if (n <= 0) continue;
        const dim3 grid(n);
#define DMRG_L64C(KT_, QT_, W_, MINW_, CW_, NS_)                                                          \
    hipLaunchKernelGGL((k_hpsi_lds64<KT_, QT_, W_, MINW_, CW_, NS_>), grid, dim3((W_ + CW_) * 64), 0, s,     \
                       P.items + b, P.tasks, pool_t, xt, y, P.partial, active)
#define DMRG_L64(KT_, QT_, W_, MINW_)                                                   \
    do {                                                                                \
        if (P.copy_wave && KT_ == 2 && P.three_slots) DMRG_L64C(KT_, QT_, W_, MINW_, 1, 3); \
        else if (P.copy_wave) DMRG_L64C(KT_, QT_, W_, MINW_, 1, 2);                     \
        else DMRG_L64C(KT_, QT_, W_, MINW_, 0, 2);                                      \
    } while (0)
        switch (c) {
            case 0: DMRG_L64(2, 3, 6, 1); break;
            case 1: DMRG_L64(2, 6, 6, 1); break;
            case 2: DMRG_L64(6, 3, 6, 1); break;
            case 3: DMRG_L64(6, 6, 6, 1); break;
            default:
                if (P.w7_min_waves == 4) DMRG_L64(7, 7, 7, 4);
                else DMRG_L64(7, 7, 7, 1);
                break;
        }
#undef DMRG_L64C
#undef DMRG_L64
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || P.n_reduces <= 0) return e;
    return launch_reduce_partials(P.reduces, P.n_reduces, P.red_chunks, P.partial, y, s, active);
}

}  // namespace dmrg
