// Kernels that grow a block by one site and renormalize it (Section 2.1: the operators of the
// enlarged block, Eq. renorm_mat; Section 2.2.2: the renormalization tasks; Section 2.2.3: the
// pre-summed operators they use). FP64 throughout.
//
// A grown operator is a sum of pieces Z (x) E_{s's}: Z a (pre-summed) operator of the old block, E
// an elementary site matrix. Its renormalized sector block (q_out, q_in) is
//     sum over items  coef * O_out^T Z O_in,
// O_out / O_in the rows of the renormalization matrix that belong to the pair (old sector, site
// state) of the item. Pass 1 forms T = Z O_in per item, pass 2 sums coef * O_out^T T per output
// block in item order (deterministic, no atomics); items with Z = identity skip pass 1.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "grow.h"

namespace dmrg {

namespace {

// dst block b (rows x cols, compact) = sum_t coeff_t * src_t (or its transpose; src_off < 0: the
// identity, for terms of square blocks that keep the sector)
__global__ void k_grow_presum(const PresumBlock* __restrict__ blocks, const PresumTerm* __restrict__ terms,
                              const double* __restrict__ src, double* __restrict__ dst, int chunk) {
    const PresumBlock b = blocks[blockIdx.x];
    const int n = b.rows * b.cols;
    const int e0 = (int)blockIdx.y * chunk, e1 = min(n, e0 + chunk);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += (int)blockDim.x) {
        const int i = e / b.cols, j = e - i * b.cols;
        double acc = 0.0;
        for (int t = b.t_begin; t < b.t_end; ++t) {
            const PresumTerm T = terms[t];
            const double v = T.src_off < 0 ? (i == j ? 1.0 : 0.0)        // the identity (square blocks)
                           : T.trans ? src[T.src_off + (int64_t)j * T.src_ld + i]
                                     : src[T.src_off + (int64_t)i * T.src_ld + j];
            acc = fma(T.coeff, v, acc);
        }
        dst[b.out_off + e] = acc;
    }
}

// pass 1: T[t_off + r * k_i + j] = sum_c Z[r][c] O_in[c][j]
__global__ void k_grow_t(const GrowItem* __restrict__ items, const int32_t* __restrict__ t_items,
                         const double* __restrict__ data, const double* __restrict__ zbuf,
                         const double* __restrict__ O, double* __restrict__ T, int chunk) {
    const GrowItem it = items[t_items[blockIdx.x]];
    const int n = it.m_out * it.k_i;
    const int e0 = (int)blockIdx.y * chunk, e1 = min(n, e0 + chunk);
    const double* __restrict__ Z = (it.z_buf ? zbuf : data) + it.z_off;
    const double* __restrict__ oi = O + it.oi_off;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += (int)blockDim.x) {
        const int r = e / it.k_i, j = e - r * it.k_i;
        double acc = 0.0;
        if (it.z_tr) {
            for (int c = 0; c < it.m_in; ++c) acc = fma(Z[(int64_t)c * it.z_ld + r], oi[(int64_t)c * it.k_i + j], acc);
        } else {
            const double* zr = Z + (int64_t)r * it.z_ld;
            for (int c = 0; c < it.m_in; ++c) acc = fma(zr[c], oi[(int64_t)c * it.k_i + j], acc);
        }
        T[it.t_off + e] = acc;
    }
}

// pass 2: out[i][j] = sum over the block's items of coef * sum_r O_out[r][i] T[r][j]
__global__ void k_grow_out(const GrowOut* __restrict__ outs, const GrowItem* __restrict__ items,
                           const double* __restrict__ O, const double* __restrict__ T, double* __restrict__ out,
                           int chunk) {
    const GrowOut b = outs[blockIdx.x];
    const int n = b.k_o * b.k_i;
    const int e0 = (int)blockIdx.y * chunk, e1 = min(n, e0 + chunk);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += (int)blockDim.x) {
        const int i = e / b.k_i, j = e - i * b.k_i;
        double acc = 0.0;
        for (int k = b.i_begin; k < b.i_end; ++k) {
            const GrowItem it = items[k];
            // identity Z: T is O_in itself (m_in = m_out rows)
            const double* __restrict__ t = it.z_off < 0 ? O + it.oi_off : T + it.t_off;
            const double* __restrict__ oo = O + it.oo_off + i;
            double s = 0.0;
            for (int r = 0; r < it.m_out; ++r) s = fma(oo[(int64_t)r * it.k_o], t[(int64_t)r * it.k_i + j], s);
            acc = fma(it.coef, s, acc);
        }
        out[b.out_off + e] = acc;
    }
}

dim3 chunked(int64_t n_groups, int64_t most, int& chunk) {
    int64_t c = std::max<int64_t>(1024, (most + 65534) / 65535);
    c = (c + 255) / 256 * 256;
    chunk = (int)c;
    return dim3((unsigned)n_groups, (unsigned)std::max<int64_t>(1, (most + c - 1) / c));
}

}  // namespace

hipError_t launch_grow_presum(const PresumBlock* blocks, int n_blocks, int64_t max_elems, const PresumTerm* terms,
                              const double* src, double* dst, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    int chunk = 0;
    const dim3 g = chunked(n_blocks, max_elems, chunk);
    hipLaunchKernelGGL(k_grow_presum, g, dim3(256), 0, s, blocks, terms, src, dst, chunk);
    return hipGetLastError();
}

hipError_t launch_grow_renorm(const GrowItem* items, const int32_t* t_items, int n_t_items, int64_t max_t,
                              const GrowOut* outs, int n_outs, int64_t max_out, const double* data, const double* zbuf,
                              const double* O, double* T, double* out, hipStream_t s) {
    int chunk = 0;
    if (n_t_items > 0) {
        const dim3 g = chunked(n_t_items, max_t, chunk);
        hipLaunchKernelGGL(k_grow_t, g, dim3(256), 0, s, items, t_items, data, zbuf, O, T, chunk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_outs <= 0) return hipSuccess;
    const dim3 g = chunked(n_outs, max_out, chunk);
    hipLaunchKernelGGL(k_grow_out, g, dim3(256), 0, s, outs, items, O, T, out, chunk);
    return hipGetLastError();
}

}  // namespace dmrg
