// Symmetric eigensolver (host, FP64), written from the textbook method (Golub and Van Loan, "Matrix
// Computations", Sections 8.3.1-8.3.3):
//  1. Householder tridiagonalization A = Q T Q^T: step k reflects column k below the diagonal onto
//     its first entry and applies the reflector to the trailing block as a symmetric rank-2 update.
//  2. Q^T is accumulated as H_{n-3} ... H_1 H_0, each reflector applied to the rows of the trailing
//     block (contiguous row operations).
//  3. The implicit symmetric QR step with the Wilkinson shift chases a bulge down each unreduced
//     block of T; off-diagonal entries below eps (|d_i| + |d_i+1|) (or below eps^2 ||A||) deflate.
//  4. Every Givens rotation R of step 3 turns T into R T R^T, so the eigenvector matrix becomes
//     Q R^T, i.e. rows k, k+1 of Q^T are rotated. The rotations do not feed back into T, so they
//     are buffered and applied in order to column slices of Q^T, one slice per host thread.
#include "eigen.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <thread>

#include "host_common.h"

namespace dmrg {
namespace {

// Rotations (k, c, s) of the QR sweeps, applied to rows k, k+1 of zt (n x n, row-major) in order,
// restricted to columns [c0, c1).
void apply_rotations(double* zt, int n, const int32_t* rk, const double* rc, const double* rs, size_t nrot, int c0,
                     int c1) {
    for (size_t r = 0; r < nrot; ++r) {
        double* x = zt + (size_t)rk[r] * n;
        double* y = x + n;
        const double c = rc[r], s = rs[r];
        for (int j = c0; j < c1; ++j) {
            const double xj = x[j], yj = y[j];
            x[j] = c * xj + s * yj;
            y[j] = c * yj - s * xj;
        }
    }
}

void apply_rotations_mt(double* zt, int n, const std::vector<int32_t>& rk, const std::vector<double>& rc,
                        const std::vector<double>& rs, int threads) {
    const size_t nrot = rk.size();
    if (nrot == 0) return;
    constexpr int kSlice = 64;                            // columns per slice (n rows x 512 B)
    const int n_slices = (n + kSlice - 1) / kSlice;
    const int nt = std::max(1, std::min(threads, n_slices));
    auto work = [&](int t) {
        for (int sl = t; sl < n_slices; sl += nt)
            apply_rotations(zt, n, rk.data(), rc.data(), rs.data(), nrot, sl * kSlice, std::min(n, (sl + 1) * kSlice));
    };
    if (nt == 1) { work(0); return; }
    std::vector<std::thread> pool;
    try {
        for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    } catch (...) {
        // thread creation failed: the slices of the threads that did not start run here
        for (auto& th : pool) th.join();
        for (int t = (int)pool.size() + 1; t < nt; ++t) work(t);
        work(0);
        return;
    }
    work(0);
    for (auto& th : pool) th.join();
}

}  // namespace

void sym_eigen(int n, const double* a, std::vector<double>& evals, std::vector<double>& vecs_t, int threads) {
    evals.assign(n, 0.0);
    vecs_t.assign((size_t)n * n, 0.0);
    if (n <= 0) return;
    const double eps = std::numeric_limits<double>::epsilon();
    // full symmetric working copy from the lower triangle
    std::vector<double> W((size_t)n * n);
    double fro = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            const double v = a[(size_t)i * n + j];
            if (!std::isfinite(v)) throw Error(DMRG_ERR_NAN, "non-finite matrix element in the eigensolver");
            W[(size_t)i * n + j] = W[(size_t)j * n + i] = v;
            fro += (i == j ? 1.0 : 2.0) * v * v;
        }
    fro = std::sqrt(fro);
    std::vector<double> d(n, 0.0), e(std::max(1, n - 1), 0.0), beta(std::max(1, n), 0.0);
    std::vector<double> p(n), w(n);
    // 1. tridiagonalization; the reflector of step k (v with v_0 = 1) is kept in row k right of the
    //    diagonal, which is no longer needed
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double* x = &W[(size_t)k * n + k + 1];            // = column k below the diagonal
        double sigma = 0.0;
        for (int j = 1; j < m; ++j) sigma += x[j] * x[j];
        d[k] = W[(size_t)k * n + k];
        if (sigma == 0.0) {                               // already reduced: no reflection
            e[k] = x[0];
            beta[k] = 0.0;
            continue;
        }
        const double x0 = x[0];
        const double mu = std::sqrt(x0 * x0 + sigma);
        const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
        const double b = 2.0 * v0 * v0 / (sigma + v0 * v0);
        x[0] = 1.0;
        for (int j = 1; j < m; ++j) x[j] /= v0;
        beta[k] = b;
        e[k] = mu;                                        // (I - b v v^T) x = ||x|| e_1
        // p = b A22 v, w = p - (b/2)(p.v) v, A22 -= v w^T + w v^T
        double pv = 0.0;
        for (int i = 0; i < m; ++i) {
            const double* row = &W[(size_t)(k + 1 + i) * n + k + 1];
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * x[j];
            p[i] = b * s;
            pv += p[i] * x[i];
        }
        const double K = 0.5 * b * pv;
        for (int i = 0; i < m; ++i) w[i] = p[i] - K * x[i];
        for (int i = 0; i < m; ++i) {
            double* row = &W[(size_t)(k + 1 + i) * n + k + 1];
            const double vi = x[i], wi = w[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * x[j];
        }
    }
    if (n >= 2) {
        d[n - 2] = W[(size_t)(n - 2) * n + n - 2];
        e[n - 2] = W[(size_t)(n - 1) * n + n - 2];
    }
    d[n - 1] = W[(size_t)(n - 1) * n + n - 1];
    // 2. Q^T = H_{n-3} ... H_0, built right to left: X <- X H_k touches rows and columns > k only
    double* zt = vecs_t.data();
    for (int i = 0; i < n; ++i) zt[(size_t)i * n + i] = 1.0;
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const int m = n - k - 1;
        const double* v = &W[(size_t)k * n + k + 1];
        for (int i = k + 1; i < n; ++i) {
            double* row = zt + (size_t)i * n + k + 1;
            double t = 0.0;
            for (int j = 0; j < m; ++j) t += row[j] * v[j];
            t *= beta[k];
            if (t != 0.0)
                for (int j = 0; j < m; ++j) row[j] -= t * v[j];
        }
    }
    W.clear();
    W.shrink_to_fit();
    // 3. implicit QR with Wilkinson shifts; 4. rotations buffered and applied to Q^T
    std::vector<int32_t> rk;
    std::vector<double> rc, rs;
    const size_t kBuf = (size_t)1 << 20;
    rk.reserve(std::min(kBuf, (size_t)n * n));
    rc.reserve(rk.capacity());
    rs.reserve(rk.capacity());
    auto flush = [&]() {
        apply_rotations_mt(zt, n, rk, rc, rs, threads);
        rk.clear();
        rc.clear();
        rs.clear();
    };
    const double small = eps * eps * fro;
    int hi = n - 1;
    int64_t steps = 0;
    while (hi > 0) {
        for (int i = 0; i < hi; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1])) || std::fabs(e[i]) <= small) e[i] = 0.0;
        while (hi > 0 && e[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        if (++steps > 30 * (int64_t)n) throw Error(DMRG_ERR_NAN, "symmetric QR iteration did not converge");
        // Wilkinson shift from the trailing 2 x 2 of the block
        const double bb = e[hi - 1];
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double den = delta + std::copysign(std::hypot(delta, bb), delta);
        const double mu = den != 0.0 ? d[hi] - bb * bb / den : d[hi];
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r != 0.0 ? x / r : 1.0, s = r != 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;
            // 2 x 2 block [d_k e_k; e_k d_k+1] -> R B R^T with R = [c s; -s c]
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            if (k + 1 < hi) {
                z = s * e[k + 1];                         // bulge at (k, k+2)
                e[k + 1] *= c;
                x = e[k];
            }
            rk.push_back(k);
            rc.push_back(c);
            rs.push_back(s);
        }
        if (rk.size() >= kBuf) flush();
    }
    flush();
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(d[i])) throw Error(DMRG_ERR_NAN, "non-finite eigenvalue");
    // ascending order, rows permuted alike
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
    bool sorted = true;
    for (int i = 0; i < n; ++i) sorted &= order[i] == i;
    if (sorted) {
        evals = d;
        return;
    }
    std::vector<double> out((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        evals[i] = d[order[i]];
        std::copy(zt + (size_t)order[i] * n, zt + (size_t)(order[i] + 1) * n, out.begin() + (size_t)i * n);
    }
    vecs_t.swap(out);
}

}  // namespace dmrg
