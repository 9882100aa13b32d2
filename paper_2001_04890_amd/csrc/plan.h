// Launch plans of the two-site H.psi (Eq. dgemm, Section 2.2.1): the handle's task list cut into
// work items for every kernel path, with the ordered reductions of cut items, the part tags of
// merged handles and the tiled operator copies that the kernels read (plan.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "host_common.h"
#include "hop.h"

namespace dmrg {

// Device allocation owned by the handle (freed with it), counted in its device bytes.
template <class T>
T* dev_alloc(dmrg_hop& H, size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    HIPCHK(hipMalloc(&p, n * sizeof(T)));
    H.allocations.push_back(p);
    H.dev_bytes += (int64_t)(n * sizeof(T));
    return static_cast<T*>(p);
}

// (Re)builds every launch plan of the handle from its task list and tuning settings; drops its
// cached graphs and the previous plans' allocations.
void build_plan(dmrg_hop& H, hipStream_t s);
// Destroys the handle's cached H.psi graphs.
void drop_graphs(dmrg_hop& H);
// True when some target block (or one of its sources) is wider than the split LDS stages.
bool needs_fallback(const dmrg_hop& H);
// Tiled split-BF16 copy of the handle's operator pool (and identity blocks).
void make_tiled_split(dmrg_hop& H, hipStream_t s);

}  // namespace dmrg
