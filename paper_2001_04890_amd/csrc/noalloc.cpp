// dmrg_renormalize_blocks_noalloc: Eq. renorm_mat per sector block (the work of
// dmrg_renormalize_blocks, same kernels and summation order) for callers that cannot allocate device
// memory. Its work list and the intermediate T = A O_in live in one fixed device array, `scratch`,
// of kScratchBytes per GPU, held until the process ends.
//
// `scratch` is a device symbol: its name in host code is a host-side stand-in, not a device address.
// The first call on a device (with that device current) asks the runtime for the array's device
// address once and keeps it per device; kernels, copies and offsets only ever use that address.
// Nothing in this file calls hipMalloc / hipFree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "host_common.h"
#include "internal.h"
#include "renorm.h"

namespace {

using dmrg::Error;

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up once per device.
unsigned char* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) throw Error(DMRG_ERR_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(DMRG_ERR_DEVICE, "no device address for the scratch array");
        g_scratch_ptr[device] = p;
    }
    return static_cast<unsigned char*>(g_scratch_ptr[device]);
}

}  // namespace

extern "C" dmrg_status dmrg_renormalize_blocks_noalloc(int32_t device, int32_t n_sec, const int32_t* dims,
                                                       const int32_t* kept, const int64_t* o_off, const double* O,
                                                       int64_t o_len, int32_t n_blk, const int32_t* sec_out,
                                                       const int32_t* sec_in, const int64_t* a_off, const double* A,
                                                       int64_t a_len, const int64_t* out_off, double* out,
                                                       int64_t out_len, void* stream) {
    dmrg::clear_error();
    try {
        const dmrg::RenormWork wk = dmrg::renorm_work(n_sec, dims, kept, o_off, O, o_len, n_blk, sec_out, sec_in,
                                                      a_off, A, a_len, out_off, out, out_len);
        if (wk.items.empty()) return DMRG_OK;
        // [items | pad to 256 B | T]: every byte the kernels read is written first (items by the copy,
        // T by the first pass), so nothing is cleared
        const size_t items_bytes = wk.items.size() * sizeof(dmrg::RenormItem);
        const size_t t_at = (items_bytes + kAlign - 1) / kAlign * kAlign;
        if ((uint64_t)wk.t_len > (kScratchBytes - std::min(kScratchBytes, t_at)) / sizeof(double))
            throw Error(DMRG_ERR_NOMEM, "work list + intermediate (" + std::to_string(t_at + wk.t_len * sizeof(double)) +
                                            " bytes) exceed the fixed scratch of " +
                                            std::to_string(kScratchBytes) + " bytes");
        HIPCHK(hipSetDevice(device));
        unsigned char* base = scratch_on(device);
        hipStream_t s = (hipStream_t)stream;
        auto* d_items = reinterpret_cast<dmrg::RenormItem*>(base);
        auto* d_t = reinterpret_cast<double*>(base + t_at);
        try {
            HIPCHK(hipMemcpyAsync(d_items, wk.items.data(), items_bytes, hipMemcpyHostToDevice, s));
            HIPCHK(dmrg::launch_renormalize(d_items, (int)wk.items.size(), wk.max_t, wk.max_out, A, O, d_t, out, s));
            HIPCHK(hipStreamSynchronize(s));   // the host work list is read by the copy until here
        } catch (...) {
            (void)hipStreamSynchronize(s);
            throw;
        }
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}
