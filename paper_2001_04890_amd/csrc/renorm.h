// Host-side helpers of the renormalization entry points (renorm_host.cpp, noalloc.cpp).
#pragma once
#include <cstdint>
#include <vector>

#include "internal.h"

namespace dmrg {

// Work list of Eq. renorm_mat per sector block (out = O_out^T A O_in, two passes through T = A O_in):
// one item per block that keeps states on both sides, T offsets packed one after another.
struct RenormWork {
    std::vector<RenormItem> items;
    int64_t t_len = 0, max_t = 0, max_out = 0;
};

// Checks every argument of dmrg_renormalize_blocks against the buffer lengths (throws Error with the
// entry point's status codes) and builds its work list; nothing touches the device.
RenormWork renorm_work(int32_t n_sec, const int32_t* dims, const int32_t* kept, const int64_t* o_off, const double* O,
                       int64_t o_len, int32_t n_blk, const int32_t* sec_out, const int32_t* sec_in,
                       const int64_t* a_off, const double* A, int64_t a_len, const int64_t* out_off, double* out,
                       int64_t out_len);

}  // namespace dmrg
