// Batched, device-resident Davidson (Sections 2.1, 2.2.1: Davidson's method for the lowest eigenpair
// of each two-site problem) over the parts of a merged handle: device kernels (davidson_batch.hip)
// and the host driver (davidson_batch.cpp).
//
// Layout: every basis vector is one full-length vector of the merged handle (n coefficients, the
// parts' segments at their first_coeff offsets), so column j of V holds the j-th basis vector of
// every part. Reductions run over a table of chunks, each inside one part, summed per part in chunk
// order (deterministic). Per part p the device holds its status, its Rayleigh-Ritz matrix G_p
// (K x K), its Ritz value and coefficient vector, and a row of dot products (kDotSlots).
// Parts that have left the active set (converged, stalled, non-finite) are skipped by every kernel
// below except bcopy with all_parts: their vectors and dot products keep stale values, and their
// Ritz pair stays that of the iteration at which they left.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmrg {

struct BChunk { int64_t begin, end; int32_t part, pad; };

// dot-product row of one part: [0, K) basis dots, then these slots
constexpr int kSlotNorm1 = 0;   // offsets past K
constexpr int kSlotNorm2 = 1;
constexpr int kSlotResid = 2;
constexpr int kSlotExtra = 3;
constexpr int kDotTail = 4;

// part status
constexpr int kActive = 1;
constexpr int kConverged = 0;
constexpr int kStalled = 2;     // the correction lay in the subspace (no new direction)
constexpr int kNonFinite = 3;

struct BatchDev {
    const BChunk* chunks;      // n_chunks
    int n_chunks;
    const int32_t* part_chunk; // n_parts + 1: first chunk of each part
    int n_parts;
    int64_t n;                 // coefficients of the merged handle
    int K;                     // max_sub
    double* partial;           // n_chunks x (K + kDotTail)
    double* dots;              // n_parts x (K + kDotTail)
    double* G;                 // n_parts x K x K
    double* s;                 // n_parts x K: Ritz coefficients (lowest eigenvector of G)
    double* ms;                // n_parts x K: -theta s
    double* y1;                // n_parts x K: second restart vector
    double* theta;             // n_parts
    double* rnorm;             // n_parts
    int32_t* status;           // n_parts
    int32_t* iters;            // n_parts: iterations while active
    double* Qp;                // n_parts x K x K: eigenvectors of the last Rayleigh-Ritz step (ld K)
    int32_t* qk;               // n_parts: their size (0: none, the next step starts cold)
};

// dots[p][slot + j] = <V[j], x> over part p, j < nv (nv <= K + kDotTail - slot), active parts
hipError_t bdots(const BatchDev& B, const double* V, int nv, const double* x, int slot, hipStream_t s);
// out = beta out + sum_j coef[p][j] V[j] on the active parts (coef rows of length K)
hipError_t bcombine(const BatchDev& B, const double* V, int nv, const double* coef, double* out, double beta,
                    hipStream_t s);
// x -= sum_j dots[p][j] V[j], j < nv, on the active parts
hipError_t bproject(const BatchDev& B, const double* V, int nv, double* x, hipStream_t s);
// x /= sqrt(dots[p][K + slot]) where positive, on the active parts
hipError_t bscale(const BatchDev& B, double* x, int slot, hipStream_t s);
// t = r / (theta_p - d) on the active parts
hipError_t bprecond(const BatchDev& B, const double* r, const double* d, double* t, hipStream_t s);
// dst = src on the parts whose status is active (all parts: all_parts)
hipError_t bcopy(const BatchDev& B, const double* src, double* dst, bool all_parts, hipStream_t s);
// Rayleigh-Ritz of the k x k leading block of G_p (active parts): theta, s, ms; warm-started from
// the previous step's eigenvectors when G grew by one row and column since
hipError_t brr(const BatchDev& B, int k, hipStream_t s);
// residual check: rnorm = sqrt(dots[K + kSlotResid]); converged below tol; counts the iteration
hipError_t bcheck(const BatchDev& B, double tol, hipStream_t s);
// new column k of G from dots[0..k] (active parts); a part whose new vector had no norm stalls
hipError_t bgcol(const BatchDev& B, int k, hipStream_t s);
// restart coefficients from s and dots[0..K) = V^T u_prev: y1, and G <- [s y1]^T G [s y1]
hipError_t brestart(const BatchDev& B, hipStream_t s);
// status <- active for every part (and the iteration counts <- 0)
hipError_t bactivate(const BatchDev& B, bool reset_iters, hipStream_t s);

}  // namespace dmrg
