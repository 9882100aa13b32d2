// Growth and renormalization of a block by one site (Section 2.1, Eq. renorm_mat; Section 2.2.2):
// device work lists and kernels (grow.hip) and the host driver (grow.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dmrg {

// One renormalization contribution coef * O_out^T Z O_in to an output sector block.
struct GrowItem {
    int64_t z_off;     // Z (m_out x m_in, leading dimension z_ld) in the operator data or the pre-sum
                       // buffer; < 0: Z is the identity (m_in = m_out)
    int64_t t_off;     // T = Z O_in (m_out x k_i, compact) in the T buffer (items with Z != identity)
    int64_t oo_off;    // first of the m_out rows of O that belong to the item's (sector, site) pair,
                       // row-major with k_o columns (the kept states of the output bra sector)
    int64_t oi_off;    // the same for the m_in rows of the ket side, k_i columns
    double  coef;
    int32_t z_ld, z_tr, z_buf;   // z_tr: Z is stored transposed; z_buf: 1 = pre-sum buffer
    int32_t m_out, m_in, k_o, k_i;
    int32_t pad;
};
// One output sector block (k_o x k_i, row-major at out_off) and its items [i_begin, i_end).
struct GrowOut {
    int64_t out_off;
    int32_t k_o, k_i, i_begin, i_end;
};

// dst[block] = sum of coefficient * (source, its transpose, or the identity when src_off < 0), compact
// row-major outputs.
hipError_t launch_grow_presum(const PresumBlock* blocks, int n_blocks, int64_t max_elems, const PresumTerm* terms,
                              const double* src, double* dst, hipStream_t s);
// Pass 1 over the items listed in t_items (those with Z != identity), then pass 2 over the outputs.
hipError_t launch_grow_renorm(const GrowItem* items, const int32_t* t_items, int n_t_items, int64_t max_t,
                              const GrowOut* outs, int n_outs, int64_t max_out, const double* data, const double* zbuf,
                              const double* O, double* T, double* out, hipStream_t s);

}  // namespace dmrg
