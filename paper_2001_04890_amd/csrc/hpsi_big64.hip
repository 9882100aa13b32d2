// FP64 sector GEMMs of Eq. dgemm (Section 2.2.1) for large sector blocks (gfx950), the FP64
// counterpart of hpsi_big.hip: pass 1 T'^T = X^T A^T per task, pass 2 Y += sum_tasks T B^T per
// 128 x 128 target tile, on v_mfma_f64_16x16x4f64.
//
// FP64 tile format (16 rows x 16 k, 2 KB): lane l = (li, g) = (l % 16, l / 16) holds the 4 doubles
// M[16 rt + li][16 kt + 4 v + g], v = 0..3. Value v is the lane's operand of the v-th 16x16x4 MFMA
// over that tile (A operand M[i = li][k = g], or B operand M^T[k = g][n = li]). The MFMA result layout
// (lane holds D[g + 4 v][li]) of a 16 x 16 tile of T'^T = X^T A^T is exactly this tile format for T
// (rows r = li, k = j = 4 v + g), so pass 1 stores its accumulators as T tiles without a shuffle.
// Stages hold 16 tiles (32 KB) of both operands for one 16-wide k tile, copied with
// global_load_lds_dwordx4 one stage ahead (two stages). Accumulation is FP64 throughout.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dmrg {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr int kTileD = 256;                  // doubles per tile
constexpr int kStageTiles = 16;
constexpr int kStageD = kStageTiles * kTileD;

__device__ __forceinline__ f64x4 lds4(const double* p) { return *reinterpret_cast<const f64x4*>(p); }
__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Copy the 16 tiles of one stage (tile i from (i < 8 ? p_base : q_base) + src[i] doubles, < 0: absent)
// to stage + i * kTileD: 32 half-tile copies of 1 KB, 8 per wavefront.
__device__ __forceinline__ void copy_stage(const double* __restrict__ p_base, const double* __restrict__ q_base,
                                           const int64_t (&src)[kStageTiles], double* stage, int wave, int lane) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int h = wave * 8 + k, tile = h >> 1, part = h & 1;
        const double* base = tile < 8 ? p_base : q_base;
        if (src[tile] >= 0)
            __builtin_amdgcn_global_load_lds((const void*)(base + src[tile] + part * 128 + lane * 2),
                                             (lds_ptr_t)(stage + tile * kTileD + part * 128), 16, 0, 0);
    }
}

}  // namespace

// ------------------------------------------------------------------ tiled FP64 operands
// pool block (rows r16 * 16 x cols k32 * 32, row-major, ld = k32 * 32) -> tiles (rt, kt), kt < 2 k32
__global__ void k_tile_f64(const double* __restrict__ pool, const PoolBlock* __restrict__ blocks,
                           double* __restrict__ tiled) {
    const PoolBlock B = blocks[blockIdx.x];
    const int ld = B.k32 * 32, k16 = 2 * B.k32;
    const int n = B.r16 * k16 * 64;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int tile = e >> 6, lane = e & 63;
        const int rt = tile / k16, kt = tile - (tile / k16) * k16;
        const int row = rt * 16 + (lane & 15), col0 = kt * 16 + (lane >> 4);
        const double* src = pool + B.off + (int64_t)row * ld + col0;
        f64x4 v = {src[0], src[4], src[8], src[12]};
        *reinterpret_cast<f64x4*>(tiled + B.off + (int64_t)tile * kTileD + lane * 4) = v;
    }
}

hipError_t launch_tile_f64(const double* pool, const PoolBlock* blocks, int n_blocks, double* tiled, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_f64, dim3(n_blocks), dim3(256), 0, s, pool, blocks, tiled);
    return hipGetLastError();
}

// psi block X (m_a x m_d) -> tiled X^T (rows j < pd, k < pa), at 2 * dst_off / 2 = dst_off doubles
__global__ void k_pack_xt64(const PackBlock* __restrict__ packs, const double* __restrict__ x, double* __restrict__ xt) {
    const PackBlock P = packs[blockIdx.x];
    const int k16 = P.pa / 16;
    const int n = (P.pd / 16) * k16 * 64;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int tile = e >> 6, lane = e & 63;
        const int jt = tile / k16, kt = tile - (tile / k16) * k16;
        const int j = jt * 16 + (lane & 15), k0 = kt * 16 + (lane >> 4);
        f64x4 v;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u;
            v[u] = (j < P.m_d && k < P.m_a) ? x[P.src_off + (int64_t)k * P.m_d + j] : 0.0;
        }
        *reinterpret_cast<f64x4*>(xt + P.dst_off + (int64_t)tile * kTileD + lane * 4) = v;
    }
}

// ------------------------------------------------------------------ pass 1: T = f A X per task
// Group: one task, T rows [16 rb, 16 rb + 128) (8 row tiles), T columns [16 jb, 16 jb + 128) (8 j
// tiles); BigT1.pa32 / pd32 hold the source's 16-wide k tiles here (the tile strides) and ka / kd the
// ones that hold data: the k loop stops at ka, and T tiles past kd are neither copied nor stored.
// Wave (wj, wr): j tiles jb + 4 wj + {0..3}, row tiles rb + 4 wr + {0..3}: 16 accumulator tiles.
__global__ __launch_bounds__(256) void k_big64_t(const BigT1* __restrict__ work, const int32_t* __restrict__ ranges,
                                                 const double* __restrict__ pool_t, const double* __restrict__ xt,
                                                 double* __restrict__ tbuf, const int32_t* __restrict__ mask) {
    __shared__ __attribute__((aligned(16))) double lds[2 * kStageD];
    const int g_begin = uni(ranges[blockIdx.x]), g_end = uni(ranges[blockIdx.x + 1]);
    if (mask && mask[work[g_begin].part] != kPartActive) return;   // a workgroup's groups share one part
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wj = wave & 1, wr = wave >> 1;
    struct G { int64_t x, a, t; double f; int pa, pd, nrt, rb, jb, ka, kd; };
    auto load_g = [&](int i) {
        const BigT1* wp = work + i;
        G d;
        d.x = uni64(wp->xt); d.a = uni64(wp->a); d.t = uni64(wp->t);
        d.f = __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, wp->f)));
        d.pa = uni(wp->pa32); d.pd = uni(wp->pd32); d.nrt = uni(wp->nrt); d.rb = uni(wp->rb); d.jb = uni(wp->jb);
        d.ka = uni(wp->ka); d.kd = uni(wp->kd);
        return d;
    };
    auto sources = [&](const G d, int kt, int64_t (&src)[kStageTiles]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int jt = d.jb + i;
            src[i] = jt < d.kd ? d.x + (int64_t)(jt * d.pa + kt) * kTileD : -1;
            const int rt = d.rb + i;
            src[8 + i] = rt < d.nrt ? d.a + (int64_t)(rt * d.pa + kt) * kTileD : -1;
        }
    };
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
    auto store = [&](const G d) {
        int ln = lane;   // opaque copy: keep the store addresses out of the main loop
        asm volatile("" : "+v"(ln));
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int jt = d.jb + 4 * wj + jj, rt = d.rb + 4 * wr + rr;
                if (jt < d.kd && rt < d.nrt) {
                    // acc[jj][rr][v] = T'^T[j 16 jt + g + 4 v][r 16 rt + li] = T tile (rt, jt), lane value v
                    f64x4 v = acc[jj][rr] * d.f;
                    *reinterpret_cast<f64x4*>(tbuf + d.t + (int64_t)(rt * d.pd + jt) * kTileD + ln * 4) = v;
                }
                acc[jj][rr] = f64x4{0.0, 0.0, 0.0, 0.0};
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
        if (nkt == cur.ka) { ngi = gi + 1; nkt = 0; }
        const bool has_next = ngi < g_end;
        G nxt = cur;
        if (has_next) {
            if (ngi != gi) nxt = load_g(ngi);
            int64_t src[kStageTiles];
            sources(nxt, nkt, src);
            copy_stage(xt, pool_t, src, lds + (st ^ 1) * kStageD, wave, lane);
        }
        const double* sp = lds + st * kStageD + lane * 4;
        f64x4 p[4], q[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) p[jj] = lds4(sp + (4 * wj + jj) * kTileD);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) q[rr] = lds4(sp + (8 + 4 * wr + rr) * kTileD);
        // consecutive MFMAs accumulate into the same registers (the fast path of the matrix core); every
        // tile runs (skipping those outside the block costs this kernel its second workgroup per CU)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[jj][rr] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[jj][v], q[rr][v], acc[jj][rr], 0, 0, 0);
        if (ngi != gi) store(cur);
        wait_vm();
        __syncthreads();
        if (!has_next) break;
        gi = ngi; kt = nkt; cur = nxt;
        st ^= 1;
    }
}

// ------------------------------------------------------------------ pass 2: Y += sum T B^T per tile
// The k loop runs over the T tiles that hold data (BigT2.kd); a wave runs the MFMAs of its output
// tiles inside the target only.
__global__ __launch_bounds__(256) void k_big64_y(const Item* __restrict__ items, const BigT2* __restrict__ tasks,
                                                 const double* __restrict__ pool_t, const double* __restrict__ tbuf,
                                                 double* __restrict__ y, double* __restrict__ part,
                                                 const int32_t* __restrict__ mask) {
    __shared__ __attribute__((aligned(16))) double lds[2 * kStageD];
    const Item* ip = items + blockIdx.x;
    if (mask && mask[ip->part] != kPartActive) return;
    const int64_t y_off = uni64(ip->y_off), part_off = uni64(ip->part_off);
    const int m_ap = uni(ip->m_ap), m_dp = uni(ip->m_dp), r0 = uni(ip->r0), c0 = uni(ip->c0);
    const int t_begin = uni(ip->t_begin), t_end = uni(ip->t_end);
    const int wave = uni(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wr = wave >> 1, wq = wave & 1;
    const int rb = r0 >> 4, qb = c0 >> 4;
    const int nrt = (m_ap + 15) >> 4, nq = (m_dp + 15) >> 4;
    const int tn = 16 * min(8, nq - qb);

    auto sources = [&](int64_t t_t, int64_t t_b, int pd, int jt, int64_t (&src)[kStageTiles]) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int rt = rb + i;
            src[i] = rt < nrt ? t_t + (int64_t)(rt * pd + jt) * kTileD : -1;
            const int q = qb + i;
            src[8 + i] = q < nq ? t_b + (int64_t)(q * pd + jt) * kTileD : -1;
        }
    };
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
            asm volatile("" : "+a"(acc[a][b]));   // accumulators live in AGPRs across the loop
        }

    // this wave's output tiles inside the target (wave-uniform counts)
    const int nr = min(4, max(0, nrt - rb - 4 * wr)), nqw = min(4, max(0, nq - qb - 4 * wq));
    int t = t_begin, jt = 0;
    int64_t T_t = uni64(tasks[t].t), T_b = uni64(tasks[t].b);
    int T_pd = uni(tasks[t].pd32), T_kd = uni(tasks[t].kd);
    {
        int64_t src[kStageTiles];
        sources(T_t, T_b, T_pd, 0, src);
        copy_stage(tbuf, pool_t, src, lds, wave, lane);
    }
    wait_vm();
    __syncthreads();
    int st = 0;
    for (;;) {
        int nt = t, njt = jt + 1;
        if (njt == T_kd) { nt = t + 1; njt = 0; }
        const bool has_next = nt < t_end;
        int64_t N_t = T_t, N_b = T_b;
        int N_pd = T_pd, N_kd = T_kd;
        if (has_next) {
            if (nt != t) {
                N_t = uni64(tasks[nt].t); N_b = uni64(tasks[nt].b);
                N_pd = uni(tasks[nt].pd32); N_kd = uni(tasks[nt].kd);
            }
            int64_t src[kStageTiles];
            sources(N_t, N_b, N_pd, njt, src);
            copy_stage(tbuf, pool_t, src, lds + (st ^ 1) * kStageD, wave, lane);
        }
        const double* sp = lds + st * kStageD + lane * 4;
        f64x4 p[4], q[4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) p[rr] = lds4(sp + (4 * wr + rr) * kTileD);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) q[qq] = lds4(sp + (8 + 4 * wq + qq) * kTileD);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int qq = 0; qq < 4; ++qq)
                if (rr < nr && qq < nqw) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[rr][qq] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[rr][v], q[qq][v], acc[rr][qq], 0, 0, 0);
                }
        wait_vm();
        __syncthreads();
        if (!has_next) break;
        t = nt; jt = njt; T_t = N_t; T_b = N_b; T_pd = N_pd; T_kd = N_kd;
        st ^= 1;
    }
    // pin the accumulators to AGPRs at the loop exit (else the allocator copies them to VGPRs on every
    // iteration, for the epilogue's sake)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) asm volatile("" : "+a"(acc[rr][qq]));
    // acc[rr][qq][v] = Y[16 rt + g + 4 v][16 q + li]
    int ln = lane;   // opaque copy: keep the store addresses out of the main loop
    asm volatile("" : "+v"(ln));
    const int li = ln & 15, g = ln >> 4;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int rt = rb + 4 * wr + rr, q = qb + 4 * wq + qq;
            if (rt >= nrt || q >= nq) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rt + g + 4 * v, col = 16 * q + li;
                if (part_off < 0) {
                    if (row < m_ap && col < m_dp) y[y_off + (int64_t)row * m_dp + col] += acc[rr][qq][v];
                } else {
                    part[part_off + (int64_t)(row - r0) * tn + (col - c0)] = acc[rr][qq][v];
                }
            }
            if (qq == 3) asm volatile("" ::: "memory");   // at most 16 read-modify-writes of y in flight
        }
}

__global__ void k_reduce_big64(const Reduce* __restrict__ red, const double* __restrict__ part, double* __restrict__ y,
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

hipError_t launch_pack_xt64(const PackBlock* packs, int n_packs, const double* x, double* xt, hipStream_t s) {
    if (n_packs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_xt64, dim3(n_packs), dim3(256), 0, s, packs, x, xt);
    return hipGetLastError();
}

hipError_t launch_hpsi_big64(const BigPlan& P, const double* pool_t, const PackBlock* packs, int n_packs,
                             const double* x, double* xt, double* y, hipStream_t s, const int32_t* active) {
    if (P.n_chunks == 0) return hipSuccess;
    if (packs && n_packs > 0) hipLaunchKernelGGL(k_pack_xt64, dim3(n_packs), dim3(256), 0, s, packs, x, xt);
    const double* tb = reinterpret_cast<const double*>(P.tbuf);
    for (int c = 0; c < P.n_chunks; ++c) {
        const BigChunk& C = P.chunks[c];
        if (C.t1_end > C.t1_begin)
            hipLaunchKernelGGL(k_big64_t, dim3(C.t1_end - C.t1_begin), dim3(256), 0, s, P.t1, P.t1_ranges + C.t1_begin,
                               pool_t, xt, reinterpret_cast<double*>(P.tbuf), active);
        if (C.item_end > C.item_begin)
            hipLaunchKernelGGL(k_big64_y, dim3(C.item_end - C.item_begin), dim3(256), 0, s, P.items + C.item_begin, P.t2,
                               pool_t, tb, y, P.partial, active);
        if (C.red_end > C.red_begin)
            hipLaunchKernelGGL(k_reduce_big64, dim3(C.red_end - C.red_begin, P.red_chunks), dim3(256), 0, s,
                               P.reduces + C.red_begin, P.partial, y, active);
    }
    return hipGetLastError();
}

}  // namespace dmrg
