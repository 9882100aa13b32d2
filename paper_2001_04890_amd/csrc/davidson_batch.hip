// Kernels of the batched, device-resident Davidson (Sections 2.1, 2.2.1): per-part reductions,
// vector updates and the Rayleigh-Ritz step of every part on the device, so that a whole Davidson
// iteration is a fixed launch sequence (capturable as one hipGraph) with no host synchronization.
//
// Reductions: each workgroup sums its chunk (one part's coefficients) in a fixed order into a partial
// row; a second kernel adds a part's partial rows in chunk order. Element-wise kernels walk the chunk
// table too, so every workgroup knows its part. The Rayleigh-Ritz step is cyclic Jacobi on the
// symmetric k x k matrix (k <= 64) of each part in one workgroup: rounds of disjoint rotations in the
// round-robin order (every pair once per sweep), each round updating rows, then columns, then the
// eigenvector matrix in parallel, until the off-diagonal Frobenius norm is below 1e-15 of the whole.
#include <hip/hip_runtime.h>

#include <cmath>

#include "batch.h"

namespace dmrg {

namespace {

constexpr int kDotGroup = 8;       // basis vectors per reduction workgroup
constexpr int kRR = 64;            // largest subspace of the Rayleigh-Ritz kernel

__device__ __forceinline__ int status_of(const BatchDev& B, int p) { return B.status[p]; }

__global__ __launch_bounds__(256) void k_bdots(BatchDev B, const double* __restrict__ V, int nv,
                                               const double* __restrict__ x, int slot) {
    const BChunk c = B.chunks[blockIdx.x];
    if (status_of(B, c.part) != kActive) return;
    const int j0 = blockIdx.y * kDotGroup;
    const int nj = min(kDotGroup, nv - j0);
    double acc[kDotGroup];
#pragma unroll
    for (int j = 0; j < kDotGroup; ++j) acc[j] = 0.0;
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        const double xi = x[i];
#pragma unroll
        for (int j = 0; j < kDotGroup; ++j)
            if (j < nj) acc[j] = fma(V[(int64_t)(j0 + j) * B.n + i], xi, acc[j]);
    }
    // butterfly sums inside each wavefront, then the four wavefronts' sums in a fixed order
    __shared__ double red[4][kDotGroup];
#pragma unroll
    for (int j = 0; j < kDotGroup; ++j) {
        double v = acc[j];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][j] = v;
    }
    __syncthreads();
    const int ld = B.K + kDotTail;
    if ((int)threadIdx.x < nj)
        B.partial[(int64_t)blockIdx.x * ld + slot + j0 + threadIdx.x] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// one workgroup per (part, dot product): thread t adds the partials of chunks c0 + t, c0 + t + 256, ...
// in order, then a fixed tree adds the 256 sums (deterministic for a given chunk table)
__global__ __launch_bounds__(256) void k_bdots_finish(BatchDev B, int slot) {
    const int p = blockIdx.x, j = blockIdx.y;
    if (status_of(B, p) != kActive) return;
    const int ld = B.K + kDotTail;
    const int c0 = B.part_chunk[p], c1 = B.part_chunk[p + 1];
    double sum = 0.0;
    for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) sum += B.partial[(int64_t)c * ld + slot + j];
    __shared__ double red[256];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) B.dots[(int64_t)p * ld + slot + j] = red[0];
}

__global__ __launch_bounds__(256) void k_bcombine(BatchDev B, const double* __restrict__ V, int nv,
                                                  const double* __restrict__ coef, double* __restrict__ out,
                                                  double beta) {
    const BChunk c = B.chunks[blockIdx.x];
    if (status_of(B, c.part) != kActive) return;
    // the coefficients are uniform over the workgroup: scalar loads, no LDS in the dependency chain
    const double* __restrict__ cf = coef + (int64_t)__builtin_amdgcn_readfirstlane(c.part) * B.K;
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        double v = beta != 0.0 ? beta * out[i] : 0.0;
        for (int j = 0; j < nv; ++j) v = fma(cf[j], V[(int64_t)j * B.n + i], v);
        out[i] = v;
    }
}

__global__ __launch_bounds__(256) void k_bproject(BatchDev B, const double* __restrict__ V, int nv,
                                                  double* __restrict__ x) {
    const BChunk c = B.chunks[blockIdx.x];
    if (status_of(B, c.part) != kActive) return;
    const int ld = B.K + kDotTail;
    const double* __restrict__ cf = B.dots + (int64_t)__builtin_amdgcn_readfirstlane(c.part) * ld;
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        double v = x[i];
        for (int j = 0; j < nv; ++j) v = fma(-cf[j], V[(int64_t)j * B.n + i], v);
        x[i] = v;
    }
}

__global__ __launch_bounds__(256) void k_bscale(BatchDev B, double* __restrict__ x, int slot) {
    const BChunk c = B.chunks[blockIdx.x];
    if (status_of(B, c.part) != kActive) return;
    const double nn = B.dots[(int64_t)c.part * (B.K + kDotTail) + B.K + slot];
    if (!(nn > 0.0)) return;
    const double f = 1.0 / sqrt(nn);
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) x[i] *= f;
}

__global__ __launch_bounds__(256) void k_bprecond(BatchDev B, const double* __restrict__ r,
                                                  const double* __restrict__ d, double* __restrict__ t) {
    const BChunk c = B.chunks[blockIdx.x];
    if (status_of(B, c.part) != kActive) return;
    const double th = B.theta[c.part];
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        double den = th - d[i];
        if (fabs(den) < 1e-8) den = den < 0.0 ? -1e-8 : 1e-8;
        t[i] = r[i] / den;
    }
}

__global__ __launch_bounds__(256) void k_bcopy(BatchDev B, const double* __restrict__ src, double* __restrict__ dst,
                                               int all_parts) {
    const BChunk c = B.chunks[blockIdx.x];
    if (!all_parts && status_of(B, c.part) != kActive) return;
    for (int64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) dst[i] = src[i];
}

// one workgroup of 64 threads per part. Warm start: when the part's previous Rayleigh-Ritz step
// diagonalized the leading (k-1) x (k-1) block of this G (Qp, qk = k - 1), the Jacobi sweeps start
// from A = Q^T G Q with Q = diag(Qp, 1), which is diagonal but for the new row and column, and
// accumulate onto that Q; any orthogonal start gives the same eigenpairs, only in fewer sweeps.
__global__ __launch_bounds__(64) void k_brr(BatchDev B, int k) {
    const int p = blockIdx.x;
    if (status_of(B, p) != kActive) return;
    __shared__ double A[kRR][kRR + 1];
    __shared__ double Q[kRR][kRR + 1];
    __shared__ double T[kRR][kRR + 1];
    __shared__ double cs[kRR / 2], sn[kRR / 2];
    __shared__ int pa[kRR / 2], pb[kRR / 2];
    __shared__ double red[64];
    const int tid = threadIdx.x;
    const double* G = B.G + (int64_t)p * B.K * B.K;
    double* Qp = B.Qp + (int64_t)p * B.K * B.K;
    const bool warm = k >= 2 && B.qk[p] == k - 1;
    for (int e = tid; e < k * k; e += 64) {
        const int i = e / k, j = e - (e / k) * k;
        A[i][j] = 0.5 * (G[(int64_t)i * B.K + j] + G[(int64_t)j * B.K + i]);
        Q[i][j] = warm && i < k - 1 && j < k - 1 ? Qp[(int64_t)i * B.K + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    if (warm) {
        for (int e = tid; e < k * k; e += 64) {   // T = A Q
            const int i = e / k, j = e - (e / k) * k;
            double v = 0.0;
            for (int l = 0; l < k; ++l) v = fma(A[i][l], Q[l][j], v);
            T[i][j] = v;
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += 64) {   // A = Q^T T
            const int i = e / k, j = e - (e / k) * k;
            double v = 0.0;
            for (int l = 0; l < k; ++l) v = fma(Q[l][i], T[l][j], v);
            A[i][j] = v;
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += 64) {   // symmetric to the last bit
            const int i = e / k, j = e - (e / k) * k;
            if (i < j) {
                const double m = 0.5 * (A[i][j] + A[j][i]);
                A[i][j] = m;
                A[j][i] = m;
            }
        }
        __syncthreads();
    }
    const int kk = k + (k & 1);              // even count; index k is a dummy when k is odd
    const int np = kk / 2;
    for (int sweep = 0; sweep < 60 && k > 1; ++sweep) {
        // convergence: off-diagonal norm against the whole
        double off = 0.0, all = 0.0;
        for (int e = tid; e < k * k; e += 64) {
            const int i = e / k, j = e - (e / k) * k;
            const double v = A[i][j] * A[i][j];
            all += v;
            if (i != j) off += v;
        }
        red[tid] = off;
        __syncthreads();
        for (int w = 32; w > 0; w >>= 1) { if (tid < w) red[tid] += red[tid + w]; __syncthreads(); }
        const double off_sum = red[0];
        __syncthreads();
        red[tid] = all;
        __syncthreads();
        for (int w = 32; w > 0; w >>= 1) { if (tid < w) red[tid] += red[tid + w]; __syncthreads(); }
        const double all_sum = red[0];
        __syncthreads();
        if (off_sum <= 1e-30 * all_sum) break;
        for (int r = 0; r < kk - 1; ++r) {
            if (tid < np) {
                // round-robin: position 0 fixed, the others rotate by r
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (kk - 1); };
                int a = player(tid), b = player(kk - 1 - tid);
                if (a > b) { const int t = a; a = b; b = t; }
                double c = 1.0, s = 0.0;
                if (b < k && A[a][b] != 0.0) {
                    const double tau = (A[b][b] - A[a][a]) / (2.0 * A[a][b]);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                pa[tid] = a;
                pb[tid] = b < k ? b : -1;
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            // rows a, b <- J^T rows
            for (int e = tid; e < np * k; e += 64) {
                const int i = e / k, j = e - (e / k) * k;
                const int a = pa[i], b = pb[i];
                if (b < 0) continue;
                const double c = cs[i], s = sn[i], x = A[a][j], y = A[b][j];
                A[a][j] = c * x - s * y;
                A[b][j] = s * x + c * y;
            }
            __syncthreads();
            // columns a, b <- columns J, and the eigenvector matrix likewise
            for (int e = tid; e < np * k; e += 64) {
                const int i = e / k, j = e - (e / k) * k;
                const int a = pa[i], b = pb[i];
                if (b < 0) continue;
                const double c = cs[i], s = sn[i];
                const double x = A[j][a], y = A[j][b];
                A[j][a] = c * x - s * y;
                A[j][b] = s * x + c * y;
                const double u = Q[j][a], v = Q[j][b];
                Q[j][a] = c * u - s * v;
                Q[j][b] = s * u + c * v;
            }
            __syncthreads();
        }
    }
    __shared__ int imin;
    if (tid == 0) {
        int m = 0;
        for (int i = 1; i < k; ++i) if (A[i][i] < A[m][m]) m = i;
        imin = m;
        B.theta[p] = A[m][m];
    }
    __syncthreads();
    const double th = A[imin][imin];
    for (int j = tid; j < B.K; j += 64) {
        const double v = j < k ? Q[j][imin] : 0.0;
        B.s[(int64_t)p * B.K + j] = v;
        B.ms[(int64_t)p * B.K + j] = -th * v;
    }
    for (int e = tid; e < k * k; e += 64) {
        const int i = e / k, j = e - (e / k) * k;
        Qp[(int64_t)i * B.K + j] = Q[i][j];
    }
    if (tid == 0) B.qk[p] = k;
}

__global__ void k_bcheck(BatchDev B, double tol) {
    const int ld = B.K + kDotTail;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < B.n_parts; p += gridDim.x * blockDim.x) {
        if (B.status[p] != kActive) continue;
        const double rn = sqrt(B.dots[(int64_t)p * ld + B.K + kSlotResid]);
        B.rnorm[p] = rn;
        B.iters[p] += 1;
        if (!isfinite(rn) || !isfinite(B.theta[p])) B.status[p] = kNonFinite;
        else if (rn <= tol) B.status[p] = kConverged;
    }
}

__global__ void k_bgcol(BatchDev B, int k) {
    const int ld = B.K + kDotTail;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < B.n_parts; p += gridDim.x * blockDim.x) {
        if (B.status[p] != kActive) continue;
        const double* d = B.dots + (int64_t)p * ld;
        const double nt = sqrt(d[B.K + kSlotNorm1]);
        if (!isfinite(nt) || !isfinite(d[B.K + kSlotNorm2])) { B.status[p] = kNonFinite; continue; }
        if (k > 0 && nt < 1e-14) { B.status[p] = kStalled; continue; }   // no new direction
        double* G = B.G + (int64_t)p * B.K * B.K;
        for (int i = 0; i <= k; ++i) {
            G[(int64_t)i * B.K + k] = d[i];
            G[(int64_t)k * B.K + i] = d[i];
        }
    }
}

// restart coefficients of one part (one workgroup of 64): y1 from V^T u_prev (in dots), made
// orthonormal to s; a unit vector orthogonal to s instead when u_prev ~ u; G <- [s y1]^T G [s y1]
__global__ __launch_bounds__(64) void k_brestart(BatchDev B) {
    const int p = blockIdx.x;
    if (status_of(B, p) != kActive) return;
    const int K = B.K, tid = threadIdx.x;
    __shared__ double sv[kRR], y[kRR], red[64];
    const double* d = B.dots + (int64_t)p * (K + kDotTail);
    for (int j = tid; j < kRR; j += 64) {
        sv[j] = j < K ? B.s[(int64_t)p * K + j] : 0.0;
        y[j] = j < K ? d[j] : 0.0;
    }
    __syncthreads();
    auto dot = [&](const double* a, const double* b) {
        double v = 0.0;
        for (int j = tid; j < K; j += 64) v += a[j] * b[j];
        red[tid] = v;
        __syncthreads();
        for (int w = 32; w > 0; w >>= 1) { if (tid < w) red[tid] += red[tid + w]; __syncthreads(); }
        const double r = red[0];
        __syncthreads();
        return r;
    };
    for (int pass = 0; pass < 2; ++pass) {
        const double c = dot(y, sv);
        for (int j = tid; j < K; j += 64) y[j] -= c * sv[j];
        __syncthreads();
    }
    double nn = sqrt(dot(y, y));
    if (!(nn > 1e-6)) {
        // u_prev ~ u: the unit vector of the smallest |s_j|, made orthogonal to s
        __shared__ int jm;
        if (tid == 0) {
            int m = 0;
            for (int j = 1; j < K; ++j) if (fabs(sv[j]) < fabs(sv[m])) m = j;
            jm = m;
        }
        __syncthreads();
        for (int j = tid; j < K; j += 64) y[j] = j == jm ? 1.0 : 0.0;
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            const double c = dot(y, sv);
            for (int j = tid; j < K; j += 64) y[j] -= c * sv[j];
            __syncthreads();
        }
        nn = sqrt(dot(y, y));
    }
    for (int j = tid; j < K; j += 64) y[j] /= nn;
    __syncthreads();
    // G s and G y, then the 2 x 2 block
    double* G = B.G + (int64_t)p * K * K;
    __shared__ double gs[kRR], gy[kRR];
    for (int i = tid; i < K; i += 64) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < K; ++j) {
            const double g = G[(int64_t)i * K + j];
            a += g * sv[j];
            b += g * y[j];
        }
        gs[i] = a;
        gy[i] = b;
    }
    __syncthreads();
    const double g00 = dot(sv, gs), g01 = dot(sv, gy), g11 = dot(y, gy);
    for (int j = tid; j < K; j += 64) B.y1[(int64_t)p * K + j] = y[j];
    if (tid == 0) {
        B.qk[p] = 0;   // G is replaced: the next Rayleigh-Ritz step starts cold
        G[0] = g00;
        G[1] = g01;
        G[K] = g01;
        G[K + 1] = g11;
    }
}

__global__ void k_bactivate(BatchDev B, int reset_iters) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < B.n_parts; p += gridDim.x * blockDim.x) {
        B.status[p] = kActive;
        B.qk[p] = 0;
        if (reset_iters) B.iters[p] = 0;
    }
}

}  // namespace

hipError_t bdots(const BatchDev& B, const double* V, int nv, const double* x, int slot, hipStream_t s) {
    if (nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bdots, dim3(B.n_chunks, (nv + kDotGroup - 1) / kDotGroup), dim3(256), 0, s, B, V, nv, x,
                       slot);
    hipLaunchKernelGGL(k_bdots_finish, dim3(B.n_parts, nv), dim3(256), 0, s, B, slot);
    return hipGetLastError();
}
hipError_t bcombine(const BatchDev& B, const double* V, int nv, const double* coef, double* out, double beta,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_bcombine, dim3(B.n_chunks), dim3(256), 0, s, B, V, nv, coef, out, beta);
    return hipGetLastError();
}
hipError_t bproject(const BatchDev& B, const double* V, int nv, double* x, hipStream_t s) {
    if (nv <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bproject, dim3(B.n_chunks), dim3(256), 0, s, B, V, nv, x);
    return hipGetLastError();
}
hipError_t bscale(const BatchDev& B, double* x, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_bscale, dim3(B.n_chunks), dim3(256), 0, s, B, x, slot);
    return hipGetLastError();
}
hipError_t bprecond(const BatchDev& B, const double* r, const double* d, double* t, hipStream_t s) {
    hipLaunchKernelGGL(k_bprecond, dim3(B.n_chunks), dim3(256), 0, s, B, r, d, t);
    return hipGetLastError();
}
hipError_t bcopy(const BatchDev& B, const double* src, double* dst, bool all_parts, hipStream_t s) {
    hipLaunchKernelGGL(k_bcopy, dim3(B.n_chunks), dim3(256), 0, s, B, src, dst, all_parts ? 1 : 0);
    return hipGetLastError();
}
hipError_t brr(const BatchDev& B, int k, hipStream_t s) {
    if (k < 1 || k > kRR || k > B.K) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_brr, dim3(B.n_parts), dim3(64), 0, s, B, k);
    return hipGetLastError();
}
hipError_t bcheck(const BatchDev& B, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_bcheck, dim3((B.n_parts + 255) / 256), dim3(256), 0, s, B, tol);
    return hipGetLastError();
}
hipError_t bgcol(const BatchDev& B, int k, hipStream_t s) {
    if (k < 0 || k >= B.K) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bgcol, dim3((B.n_parts + 255) / 256), dim3(256), 0, s, B, k);
    return hipGetLastError();
}
hipError_t brestart(const BatchDev& B, hipStream_t s) {
    if (B.K > kRR) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_brestart, dim3(B.n_parts), dim3(64), 0, s, B);
    return hipGetLastError();
}
hipError_t bactivate(const BatchDev& B, bool reset_iters, hipStream_t s) {
    hipLaunchKernelGGL(k_bactivate, dim3((B.n_parts + 255) / 256), dim3(256), 0, s, B, reset_iters ? 1 : 0);
    return hipGetLastError();
}

}  // namespace dmrg
