// Learned Davidson preconditioner: definitions shared by the MLP kernels (mlp.hip), the MLP host
// driver (mlp_host.cpp) and the Davidson driver (host.cpp). The network is described in mlp.hip.
#pragma once
#include <stdint.h>

namespace dmrg {

constexpr int kMlpIn = 16;
constexpr int kMlpHidden = 256;
constexpr int kOffB1 = kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden;
constexpr int kMlpParams = kOffB3 + 1;
constexpr int64_t kMlpChunk = 16384;   // coefficients per feature workgroup

// Features of coefficient i of psi block (a, b, c, d) (FP64 arithmetic, stored as FP32):
//   0 asinh(r_i s_r)   1 asinh(t_i s_t)   2 asinh(u_i s_u)   3 asinh((D_i - theta) s_D)
//   4..7 one-hot b     8..11 one-hot c
//   12 asinh(rms_block(r) s_r)   13 asinh(rms_block(u) s_u)   14 ln(m_a) / 8   15 ln(m_d) / 8
// with r the residual, u the Ritz vector, t = r / (theta - D) the diagonal correction, D = diag(H),
// s_x = sqrt(n) / ||x|| the reciprocal RMS over the whole vector (0 for a zero vector).
struct MlpBlockInfo {
    int64_t off;
    int32_t m_a, m_d;
    int32_t b, c;
    int32_t chunk_begin, chunk_end;   // chunks covering this block
    float lma, lmd;                   // ln(m_a) / 8, ln(m_d) / 8
};

struct MlpChunk {
    int64_t begin, end;   // coefficient range, inside one block
    int32_t block;
    int32_t pad;
};

struct MlpScales {
    double inv_r, inv_t, inv_u, inv_dt;
};

// Device view of the network weights.
struct MlpDev {
    const float* p;          // FP32 parameters [W1 (16 x 256), b1, W2 (256 x 256), b2, w3, b3]
    const uint16_t* w1p;     // BF16 W1 in MFMA fragment order (K padded to 32)
    const uint16_t* w2p;     // BF16 W2 in MFMA fragment order
    const uint16_t* w2;      // BF16 W2, row-major
    int fp32;                // 1: FP32 debug mode (vector-unit kernels on the FP32 parameters)
};

}  // namespace dmrg

#ifndef DMRG_HOST_ONLY
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/dmrg.h"

namespace dmrg {
hipError_t launch_mlp_features(const MlpChunk* chunks, int n_chunks, const MlpBlockInfo* blocks, double* part,
                               const double* r, const double* t, const double* u, const double* d, double theta,
                               const MlpScales& sc, float* feat, hipStream_t s);
hipError_t launch_mlp_gather(const float* in, const int64_t* idx, int64_t n, int cols, float* out, hipStream_t s);
hipError_t launch_mlp_pairs(const double* t, const double* v, const int64_t* idx, int64_t n, double sa, double sb,
                            float w, float* aux, hipStream_t s);
hipError_t launch_mlp_pack(const float* p, uint16_t* w1p, uint16_t* w2p, uint16_t* w2, hipStream_t s);
// out (FP32, may be NULL) = m; if t_apply is not NULL, t_apply[i] *= 1 + m_i. h1/h2 non-NULL: training
// forward that keeps the hidden activations (FP32, n x 256 each).
hipError_t launch_mlp_forward(const MlpDev& W, const float* feat, int64_t n, float* out, float* h1, float* h2,
                              double* t_apply, hipStream_t s);
hipError_t launch_mlp_backward(const MlpDev& W, const float* aux, const float* m, const float* h1, const float* h2,
                               int64_t n, float* g, float* d1, float* d2, float* loss_part, float* loss,
                               hipStream_t s);
hipError_t launch_mlp_wgrad(const float* x, const float* h1, const float* h2, const float* d1, const float* d2,
                            const float* g, int64_t n, float* grad, hipStream_t s);
hipError_t launch_mlp_adam(float* p, const float* grad, float* m1, float* m2, float lr, int step, hipStream_t s);
// out[0..3] = sum of squares of r, u, t and D - theta; part: 4 * mlp_reduce_blocks(n) doubles
hipError_t launch_mlp_norms(const double* r, const double* u, const double* t, const double* d, double theta,
                            int64_t n, double* part, double* out, hipStream_t s);
// out[0] = sum of w (a (1 + m) - b)^2 over n rows (m NULL: m = 0); part: mlp_reduce_blocks(n) doubles
hipError_t launch_mlp_loss(const float* aux, const float* m, int64_t n, double* part, double* out, hipStream_t s);
int mlp_reduce_blocks(int64_t n);

// What the preconditioner needs to know about one H.psi handle.
struct MlpProblem {
    int64_t n = 0;
    const double* diag = nullptr;                 // device, diag(H)
    std::vector<int64_t> off;                     // per psi block
    std::vector<int32_t> m_a, m_d, b, c;
};

// Per-Davidson-solve state of the learned preconditioner and of the training-pair recorder
// (mlp_host.cpp). Methods throw dmrg::Error.
class MlpSession {
public:
    // net: apply this network to every correction (NULL: diagonal). rec: record training pairs into
    // dataset `slot` of this network (NULL: no recording), rows_per_iter sampled coefficients per
    // recorded iteration, sampling seed `seed`, psi_star the converged eigenvector of the same
    // solve (device, normalized).
    MlpSession(const dmrg_mlp* net, dmrg_mlp* rec, int slot, int rows_per_iter, uint64_t seed, const double* psi_star,
               const MlpProblem& prob, hipStream_t s);
    ~MlpSession();
    MlpSession(const MlpSession&) = delete;
    MlpSession& operator=(const MlpSession&) = delete;
    // t holds the diagonal correction of (r, theta) on entry and V (k orthonormal vectors) the
    // subspace t is about to be orthogonalized against; records a training pair and/or (apply_net)
    // applies the network to t.
    void correction(const double* r, const double* u, double* t, double theta, const double* V, int k,
                    bool apply_net = true);
    int64_t rows_recorded() const { return rows_; }

private:
    struct Impl;
    Impl* impl_;
    int64_t rows_ = 0;
};

// Feature vectors of every coefficient of a handle (features above; t = r / (theta - D) is written
// too). feat: n x 16 FP32, device.
void mlp_features(const MlpProblem& prob, const double* r, const double* u, double theta, double* t, float* feat,
                  hipStream_t s);

// host.cpp: the handle's layout and diagonal, and Davidson with a training-pair recorder.
MlpProblem mlp_problem_of(const dmrg_hop* H);
struct MlpRecord {
    dmrg_mlp* mlp;
    int slot;
    int rows_per_iter;
    uint64_t seed;
    const double* psi_star;   // device, converged eigenvector of the same solve
    int64_t rows_added = 0;
};
dmrg_status davidson_run(dmrg_hop* H, double* psi, const dmrg_dav_opts* o, dmrg_dav_result* res, void* stream,
                         MlpRecord* rec);
}  // namespace dmrg
#endif
