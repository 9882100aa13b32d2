// Device-side data structures shared by the host driver (host.cpp) and the HIP kernels
// (kernels.hip). Plain structs, no HIP types, so host-only builds can include it.
#pragma once
#include <stdint.h>

namespace dmrg {

// One sector-GEMM contribution to an output psi block (Eq. dgemm, Section 2.2.1):
//   Y_target += f * A . X_source . B^T
// A (m_a' x m_a) and B (m_d' x m_d) live in the operator pool, row-major with leading dimension
// ld(m) = round_up(m, kLd). a_off / b_off < 0 mean identity.
struct Task {
    int64_t x_off;   // element offset of the source block in x
    int64_t a_off;   // pool offset of A, or -1
    int64_t b_off;   // pool offset of B, or -1
    double  f;
    int32_t m_a;     // source rows
    int32_t m_d;     // source cols
};

// One output tile owned by one wavefront: rows [r0, r0 + TM) x cols [c0, c0 + TN) of a target block.
struct Unit {
    int64_t y_off;
    int32_t m_ap, m_dp;
    int32_t r0, c0;
    int32_t t_begin, t_end;
};

// Pre-summed / transposed operator block (Section 2.2.3): out = sum_k coeff_k * src_k (or src_k^T).
struct PresumBlock {
    int64_t out_off;
    int32_t rows, cols;
    int32_t t_begin, t_end;
};
struct PresumTerm {
    int64_t src_off;
    int32_t src_ld;
    int32_t trans;
    double  coeff;
};

// Diagonal contribution of a task that maps a block onto itself: D += f diag(A) diag(B)^T.
struct DiagTask {
    int64_t a_off, b_off;   // -1 for identity
    double  f;
};
struct DiagBlock {
    int64_t off;
    int32_t m_a, m_d;
    int32_t t_begin, t_end;
};

constexpr int kLd = 8;     // leading-dimension alignment of pool blocks (64 B in FP64, 16 B in BF16)
inline int32_t ld_of(int32_t m) { return (m + kLd - 1) / kLd * kLd; }

}  // namespace dmrg

#ifndef DMRG_HOST_ONLY
#include <hip/hip_runtime.h>
namespace dmrg {
// Launchers (kernels.hip). All asynchronous on `s`.
hipError_t launch_presum(const PresumBlock* blocks, int n_blocks, const PresumTerm* terms,
                         double* pool, hipStream_t s);
hipError_t launch_split(const double* pool, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t s);
hipError_t launch_hpsi_f64(const Unit* units, int n_units, const Task* tasks, const double* pool,
                           const double* x, double* y, int64_t n_coeff, int nvec, hipStream_t s);
hipError_t launch_hpsi_split(const Unit* units, int n_units, const Task* tasks, const uint16_t* hi,
                             const uint16_t* lo, const double* x, double* y, int64_t n_coeff,
                             int nvec, hipStream_t s);
hipError_t launch_diag(const DiagBlock* blocks, int n_blocks, const DiagTask* tasks,
                       const double* pool, double* d, hipStream_t s);
// Davidson vector kernels (FP64).
hipError_t launch_multidot(const double* V, int nv, int64_t n, const double* w, double* partial,
                           int n_part, double* out, hipStream_t s);
constexpr int kMaxCombine = 72;
struct Coefs { double c[kMaxCombine]; };
hipError_t launch_combine(const double* V, int nv, int64_t n, const Coefs& coef, double* out,
                          double beta, hipStream_t s);
hipError_t launch_precond(const double* r, const double* d, double theta, double* t, int64_t n,
                          hipStream_t s);
hipError_t launch_scale(double* x, double a, int64_t n, hipStream_t s);
int multidot_parts(int64_t n);
}  // namespace dmrg
#endif
