// Host driver of the learned Davidson preconditioner: network handle, features of a Davidson
// iteration, the training-pair recorder, minibatch Adam training and the dmrg_mlp_* C-ABI.
// Kernels and the network are in mlp.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/dmrg.h"
#include "host_common.h"
#include "internal.h"
#include "mlp.h"

using dmrg::Error;

namespace {

// splitmix64 (Steele, Lea, Flood 2014): x += 0x9e3779b97f4a7c15, then two xor-shift-multiply rounds.
struct SplitMix64 {
    uint64_t x;
    explicit SplitMix64(uint64_t seed) : x(seed) {}
    uint64_t next() {
        uint64_t z = (x += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }          // [0, 1)
    int64_t below(int64_t n) { return (int64_t)((next() >> 11) % (uint64_t)n); }
};

template <class T>
T* dev_alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw Error(DMRG_ERR_NOMEM, "device allocation failed (learned preconditioner)");
    return (T*)p;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() { if (p) (void)hipFree(p); p = nullptr; bytes = 0; }
    // grow (contents are not kept)
    template <class T> T* ensure(size_t n) {
        if (n * sizeof(T) > bytes) {
            release();
            p = dev_alloc<T>(n);
            bytes = n * sizeof(T);
        }
        return (T*)p;
    }
    template <class T> T* get() const { return (T*)p; }
};

constexpr int64_t kMaxBatch = int64_t(1) << 20;

}  // namespace

struct dmrg_mlp {
    int device = 0;
    int fp32 = 0;
    int step = 0;
    float* p = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    float* grad = nullptr;
    uint16_t* w1p = nullptr;
    uint16_t* w2p = nullptr;
    uint16_t* w2 = nullptr;
    struct Set {
        DevBuf feat, aux;
        int64_t rows = 0, cap = 0;
    } set[2];
    // minibatch work space
    DevBuf idx, xb, ab, m, h1, h2, g, d1, d2, lpart, loss, red;
    std::vector<void*> owned;
    dmrg::MlpDev dev() const { return dmrg::MlpDev{p, w1p, w2p, w2, fp32}; }
    ~dmrg_mlp() { for (void* q : owned) (void)hipFree(q); }
};

namespace dmrg {
namespace {

void ensure_batch(dmrg_mlp* M, int64_t n) {
    if (n < 1 || n > kMaxBatch) throw Error(DMRG_ERR_ARG, "minibatch size out of range (1 .. 2^20)");
    M->xb.ensure<float>((size_t)n * kMlpIn);
    M->ab.ensure<float>((size_t)n * 3);
    M->m.ensure<float>(n);
    M->h1.ensure<float>((size_t)n * kMlpHidden);
    M->h2.ensure<float>((size_t)n * kMlpHidden);
    M->g.ensure<float>(n);
    M->d1.ensure<float>((size_t)n * kMlpHidden);
    M->d2.ensure<float>((size_t)n * kMlpHidden);
    M->lpart.ensure<float>(n / 64 + 1);
}

// forward (training), backward, parameter gradient into grad, loss into loss; Adam step if lr > 0
void grad_step(dmrg_mlp* M, const float* x, const float* aux, int64_t n, float lr, float* grad, float* loss, hipStream_t s) {
    ensure_batch(M, n);
    const MlpDev W = M->dev();
    HIPCHK(launch_mlp_forward(W, x, n, M->m.get<float>(), M->h1.get<float>(), M->h2.get<float>(), nullptr, s));
    HIPCHK(launch_mlp_backward(W, aux, M->m.get<float>(), M->h1.get<float>(), M->h2.get<float>(), n, M->g.get<float>(),
                               M->d1.get<float>(), M->d2.get<float>(), M->lpart.get<float>(), loss, s));
    HIPCHK(launch_mlp_wgrad(x, M->h1.get<float>(), M->h2.get<float>(), M->d1.get<float>(), M->d2.get<float>(),
                            M->g.get<float>(), n, grad, s));
    if (lr > 0.f) {
        ++M->step;
        HIPCHK(launch_mlp_adam(M->p, grad, M->m1, M->m2, lr, M->step, s));
        HIPCHK(launch_mlp_pack(M->p, M->w1p, M->w2p, M->w2, s));
    }
}

// append rows (device feat rows x 16, aux rows x 3) to a dataset slot
void append_rows(dmrg_mlp* M, int slot, const float* feat, const float* aux, int64_t rows, hipStream_t s) {
    auto& S = M->set[slot];
    if (rows == 0) return;
    if (S.rows + rows > S.cap) {
        int64_t cap = std::max<int64_t>(S.rows + rows, 2 * S.cap);
        float* nf = dev_alloc<float>((size_t)cap * kMlpIn);
        float* na = dev_alloc<float>((size_t)cap * 3);
        if (S.rows) {
            HIPCHK(hipMemcpyAsync(nf, S.feat.p, (size_t)S.rows * kMlpIn * sizeof(float), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(na, S.aux.p, (size_t)S.rows * 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        S.feat.release();
        S.aux.release();
        S.feat.p = nf; S.feat.bytes = (size_t)cap * kMlpIn * sizeof(float);
        S.aux.p = na;  S.aux.bytes = (size_t)cap * 3 * sizeof(float);
        S.cap = cap;
    }
    HIPCHK(hipMemcpyAsync(S.feat.get<float>() + S.rows * kMlpIn, feat, (size_t)rows * kMlpIn * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(S.aux.get<float>() + S.rows * 3, aux, (size_t)rows * 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
    S.rows += rows;
}

}  // namespace

// ---------------------------------------------------------------- features of one iteration
struct FeatureState {
    const MlpProblem& prob;
    MlpBlockInfo* d_blocks = nullptr;
    MlpChunk* d_chunks = nullptr;
    int n_chunks = 0;
    double* d_part = nullptr;      // 2 per chunk
    double* d_red = nullptr;       // norms partials + 4 results
    std::vector<void*> owned;
    explicit FeatureState(const MlpProblem& p, hipStream_t s) : prob(p) {
        const int nb = (int)p.off.size();
        std::vector<MlpBlockInfo> blocks(nb);
        std::vector<MlpChunk> chunks;
        for (int k = 0; k < nb; ++k) {
            MlpBlockInfo& B = blocks[k];
            B.off = p.off[k];
            B.m_a = p.m_a[k];
            B.m_d = p.m_d[k];
            B.b = p.b[k];
            B.c = p.c[k];
            B.lma = (float)(std::log((double)B.m_a) / 8.0);
            B.lmd = (float)(std::log((double)B.m_d) / 8.0);
            B.chunk_begin = (int)chunks.size();
            const int64_t size = (int64_t)B.m_a * B.m_d;
            for (int64_t o = 0; o < size; o += kMlpChunk)
                chunks.push_back(MlpChunk{B.off + o, B.off + std::min(size, o + kMlpChunk), k, 0});
            B.chunk_end = (int)chunks.size();
        }
        n_chunks = (int)chunks.size();
        d_blocks = dev_alloc<MlpBlockInfo>(nb);
        owned.push_back(d_blocks);
        d_chunks = dev_alloc<MlpChunk>(n_chunks);
        owned.push_back(d_chunks);
        d_part = dev_alloc<double>((size_t)2 * n_chunks);
        owned.push_back(d_part);
        d_red = dev_alloc<double>((size_t)4 * mlp_reduce_blocks(p.n) + 4);
        owned.push_back(d_red);
        if (nb) HIPCHK(hipMemcpy(d_blocks, blocks.data(), nb * sizeof(MlpBlockInfo), hipMemcpyHostToDevice));
        if (n_chunks) HIPCHK(hipMemcpy(d_chunks, chunks.data(), n_chunks * sizeof(MlpChunk), hipMemcpyHostToDevice));
        (void)s;
    }
    ~FeatureState() { for (void* q : owned) (void)hipFree(q); }
    // t = r / (theta - D) must already be in t. Returns ||t||.
    double compute(const double* r, const double* u, const double* t, double theta, float* feat, hipStream_t s) {
        const int64_t n = prob.n;
        const int nb = mlp_reduce_blocks(n);
        double* out = d_red + 4 * nb;
        HIPCHK(launch_mlp_norms(r, u, t, prob.diag, theta, n, d_red, out, s));
        double h[4];
        HIPCHK(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double sq = std::sqrt((double)n);
        auto inv = [&](double ss) { return ss > 0.0 ? sq / std::sqrt(ss) : 0.0; };
        MlpScales sc{inv(h[0]), inv(h[2]), inv(h[1]), inv(h[3])};
        HIPCHK(launch_mlp_features(d_chunks, n_chunks, d_blocks, d_part, r, t, u, prob.diag, theta, sc, feat, s));
        return std::sqrt(h[2]);
    }
};

void mlp_features(const MlpProblem& prob, const double* r, const double* u, double theta, double* t, float* feat,
                  hipStream_t s) {
    FeatureState F(prob, s);
    HIPCHK(launch_precond(r, prob.diag, theta, t, prob.n, s));
    F.compute(r, u, t, theta, feat, s);
    HIPCHK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- Davidson session
struct MlpSession::Impl {
    const dmrg_mlp* net;
    dmrg_mlp* rec;
    int slot, rows_per_iter;
    SplitMix64 rng;
    const double* psi_star;
    MlpProblem prob;
    hipStream_t s;
    FeatureState feats;
    std::vector<void*> owned;
    float* feat = nullptr;          // n x 16
    // recorder work space
    double* target = nullptr;       // n
    double* dots = nullptr;         // kMaxCombine + 1
    double* part = nullptr;
    int np = 0;
    int64_t* idx = nullptr;         // rows_per_iter
    float* rows = nullptr;          // rows_per_iter x 16
    float* aux = nullptr;           // rows_per_iter x 3
    template <class T> T* alloc(size_t n) { T* q = dev_alloc<T>(n); owned.push_back(q); return q; }
    Impl(const dmrg_mlp* n_, dmrg_mlp* r_, int sl, int rpi, uint64_t seed, const double* ps, const MlpProblem& p,
         hipStream_t st)
        : net(n_), rec(r_), slot(sl), rows_per_iter(rpi), rng(seed), psi_star(ps), prob(p), s(st), feats(prob, st) {
        try {
            feat = alloc<float>((size_t)prob.n * kMlpIn);
            if (rec) {
                if (!psi_star) throw Error(DMRG_ERR_ARG, "recording needs the converged eigenvector");
                const int64_t nr = std::min<int64_t>(rows_per_iter, prob.n);
                target = alloc<double>(prob.n);
                dots = alloc<double>(kMaxCombine + 1);
                np = multidot_parts(prob.n);
                part = alloc<double>((size_t)np * (kMaxCombine + 1));
                idx = alloc<int64_t>(nr);
                rows = alloc<float>((size_t)nr * kMlpIn);
                aux = alloc<float>((size_t)nr * 3);
            }
        } catch (...) {
            for (void* q : owned) (void)hipFree(q);
            throw;
        }
    }
    ~Impl() { for (void* q : owned) (void)hipFree(q); }
    std::vector<double> dot(const double* V, int k, const double* x) {
        std::vector<double> h(k);
        HIPCHK(launch_multidot(V, k, prob.n, x, part, np, dots, s));
        HIPCHK(hipMemcpyAsync(h.data(), dots, k * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return h;
    }
};

MlpSession::MlpSession(const dmrg_mlp* net, dmrg_mlp* rec, int slot, int rows_per_iter, uint64_t seed,
                       const double* psi_star, const MlpProblem& prob, hipStream_t s)
    : impl_(new Impl(net, rec, slot, rows_per_iter, seed, psi_star, prob, s)) {}

MlpSession::~MlpSession() { delete impl_; }

void MlpSession::correction(const double* r, const double* u, double* t, double theta, const double* V, int k,
                            bool apply_net) {
    Impl& I = *impl_;
    const int64_t n = I.prob.n;
    I.feats.compute(r, u, t, theta, I.feat, I.s);
    if (I.rec) {
        // target: the part of psi* outside span(V) (classical Gram-Schmidt, twice); with it the next
        // Rayleigh-Ritz step would be exact
        HIPCHK(hipMemcpyAsync(I.target, I.psi_star, n * sizeof(double), hipMemcpyDeviceToDevice, I.s));
        for (int pass = 0; pass < 2 && k > 0; ++pass) {
            std::vector<double> c = I.dot(V, k, I.target);
            Coefs cf{};
            for (int j = 0; j < k; ++j) cf.c[j] = -c[j];
            HIPCHK(launch_combine(V, k, n, cf, I.target, 1.0, I.s));
        }
        const double dd = I.dot(I.target, 1, I.target)[0];
        const double td = I.dot(t, 1, I.target)[0];
        const double tt = I.dot(t, 1, t)[0];
        if (std::sqrt(dd) >= 1e-7 && tt > 0.0 && std::isfinite(td)) {
            const int64_t nr = std::min<int64_t>(I.rows_per_iter, n);
            std::vector<int64_t> h(nr);
            if (nr == n) for (int64_t q = 0; q < n; ++q) h[q] = q;
            else for (auto& v : h) v = I.rng.below(n);
            HIPCHK(hipStreamSynchronize(I.s));    // the previous iteration's gathers are done with idx
            HIPCHK(hipMemcpy(I.idx, h.data(), nr * sizeof(int64_t), hipMemcpyHostToDevice));
            HIPCHK(launch_mlp_gather(I.feat, I.idx, nr, kMlpIn, I.rows, I.s));
            // both sides at unit RMS; the target's sign taken so that it points along t
            const double sa = std::sqrt((double)n / tt);
            const double sb = (td < 0.0 ? -1.0 : 1.0) * std::sqrt((double)n / dd);
            HIPCHK(launch_mlp_pairs(t, I.target, I.idx, nr, sa, sb, 1.0f, I.aux, I.s));
            append_rows(I.rec, I.slot, I.rows, I.aux, nr, I.s);
            rows_ += nr;
        }
    }
    if (I.net && apply_net) HIPCHK(launch_mlp_forward(I.net->dev(), I.feat, n, nullptr, nullptr, nullptr, t, I.s));
}

}  // namespace dmrg

// ====================================================================== C-ABI

extern "C" dmrg_status dmrg_mlp_create(int32_t device, uint64_t seed, dmrg_mlp** out) {
    dmrg::clear_error();
    dmrg_mlp* M = nullptr;
    try {
        if (!out) throw Error(DMRG_ERR_ARG, "NULL argument");
        int nd = 0;
        HIPCHK(hipGetDeviceCount(&nd));
        if (device < 0 || device >= nd) throw Error(DMRG_ERR_ARG, "device index out of range");
        HIPCHK(hipSetDevice(device));
        M = new dmrg_mlp();
        M->device = device;
        auto own = [&](auto* q) { M->owned.push_back((void*)q); return q; };
        M->p = own(dev_alloc<float>(dmrg::kMlpParams));
        M->m1 = own(dev_alloc<float>(dmrg::kMlpParams));
        M->m2 = own(dev_alloc<float>(dmrg::kMlpParams));
        M->grad = own(dev_alloc<float>(dmrg::kMlpParams));
        M->w1p = own(dev_alloc<uint16_t>(16 * 64 * 8));
        M->w2p = own(dev_alloc<uint16_t>(dmrg::kMlpHidden * dmrg::kMlpHidden));
        M->w2 = own(dev_alloc<uint16_t>(dmrg::kMlpHidden * dmrg::kMlpHidden));
        std::vector<float> h(dmrg::kMlpParams, 0.f);
        SplitMix64 rng(seed);
        const double a1 = std::sqrt(6.0 / dmrg::kMlpIn), a2 = std::sqrt(6.0 / dmrg::kMlpHidden);
        for (int i = 0; i < dmrg::kOffB1; ++i) h[i] = (float)((2.0 * rng.uniform() - 1.0) * a1);
        for (int i = 0; i < dmrg::kMlpHidden * dmrg::kMlpHidden; ++i) h[dmrg::kOffW2 + i] = (float)((2.0 * rng.uniform() - 1.0) * a2);
        dmrg_status st = dmrg_mlp_params(M, nullptr, h.data());
        if (st != DMRG_OK) { delete M; return st; }
        *out = M;
        return DMRG_OK;
    } catch (const Error& e) {
        delete M;
        return dmrg::record_error(e);
    }
}

extern "C" void dmrg_mlp_free(dmrg_mlp* mlp) {
    if (!mlp) return;
    (void)hipSetDevice(mlp->device);
    (void)hipDeviceSynchronize();
    delete mlp;
}

extern "C" dmrg_status dmrg_mlp_params(dmrg_mlp* M, float* get, const float* set) {
    dmrg::clear_error();
    try {
        if (!M) throw Error(DMRG_ERR_ARG, "NULL handle");
        HIPCHK(hipSetDevice(M->device));
        HIPCHK(hipDeviceSynchronize());
        if (get) HIPCHK(hipMemcpy(get, M->p, dmrg::kMlpParams * sizeof(float), hipMemcpyDeviceToHost));
        if (set) {
            for (int i = 0; i < dmrg::kMlpParams; ++i)
                if (!std::isfinite(set[i])) throw Error(DMRG_ERR_NAN, "non-finite parameter");
            HIPCHK(hipMemcpy(M->p, set, dmrg::kMlpParams * sizeof(float), hipMemcpyHostToDevice));
            HIPCHK(hipMemset(M->m1, 0, dmrg::kMlpParams * sizeof(float)));
            HIPCHK(hipMemset(M->m2, 0, dmrg::kMlpParams * sizeof(float)));
            M->step = 0;
            HIPCHK(dmrg::launch_mlp_pack(M->p, M->w1p, M->w2p, M->w2, 0));
            HIPCHK(hipDeviceSynchronize());
        }
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

extern "C" dmrg_status dmrg_mlp_set_fp32(dmrg_mlp* M, int32_t fp32) {
    dmrg::clear_error();
    if (!M) return dmrg::record_error(Error(DMRG_ERR_ARG, "NULL handle"));
    if (fp32 != 0 && fp32 != 1) return dmrg::record_error(Error(DMRG_ERR_ARG, "fp32 must be 0 or 1"));
    M->fp32 = fp32;
    return DMRG_OK;
}

extern "C" dmrg_status dmrg_mlp_features(dmrg_hop* hop, const double* r, const double* u, double theta, float* feat,
                                         double* t, void* stream) {
    dmrg::clear_error();
    try {
        if (!hop || !r || !u || !feat || !t) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (!std::isfinite(theta)) throw Error(DMRG_ERR_NAN, "theta is not finite");
        dmrg::MlpProblem prob = dmrg::mlp_problem_of(hop);
        dmrg::mlp_features(prob, r, u, theta, t, feat, (hipStream_t)stream);
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

extern "C" dmrg_status dmrg_mlp_forward(const dmrg_mlp* M, const float* feat, int64_t n, float* m, void* stream) {
    dmrg::clear_error();
    try {
        if (!M || (n > 0 && (!feat || !m))) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (n < 0) throw Error(DMRG_ERR_ARG, "negative row count");
        HIPCHK(hipSetDevice(M->device));
        HIPCHK(dmrg::launch_mlp_forward(M->dev(), feat, n, m, nullptr, nullptr, nullptr, (hipStream_t)stream));
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

extern "C" dmrg_status dmrg_mlp_grad(dmrg_mlp* M, const float* feat, const float* pairs, int64_t n, float lr, float* grad,
                                     float* loss, void* stream) {
    dmrg::clear_error();
    try {
        if (!M || !feat || !pairs || !grad || !loss) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (!(lr >= 0.f) || !std::isfinite(lr)) throw Error(DMRG_ERR_ARG, "learning rate must be finite and >= 0");
        HIPCHK(hipSetDevice(M->device));
        dmrg::grad_step(M, feat, pairs, n, lr, grad, loss, (hipStream_t)stream);
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

extern "C" dmrg_status dmrg_mlp_collect(dmrg_mlp* M, dmrg_hop* hop, double* psi, const dmrg_dav_opts* opts,
                                        int32_t slot, int32_t rows_per_iter, uint64_t seed, dmrg_dav_result* result,
                                        int64_t* n_rows, void* stream) {
    dmrg::clear_error();
    if (!M || !hop) return dmrg::record_error(Error(DMRG_ERR_ARG, "NULL handle"));
    if (slot != 0 && slot != 1) return dmrg::record_error(Error(DMRG_ERR_ARG, "slot must be 0 or 1"));
    if (rows_per_iter < 1) return dmrg::record_error(Error(DMRG_ERR_ARG, "rows_per_iter must be >= 1"));
    if (!psi || !opts || !result) return dmrg::record_error(Error(DMRG_ERR_ARG, "NULL argument"));
    // solve once for psi*, then again from the same start vector (the solver is deterministic, so
    // it takes the same steps) recording the pairs of every iteration
    double* psi0 = nullptr;
    double* star = nullptr;
    dmrg_status st = DMRG_OK;
    try {
        HIPCHK(hipSetDevice(M->device));
        int64_t n = 0;
        if (dmrg_hop_layout(hop, &n, nullptr, nullptr, nullptr, nullptr) != DMRG_OK)
            throw Error(DMRG_ERR_ARG, "bad handle");
        hipStream_t s = (hipStream_t)stream;
        psi0 = dev_alloc<double>(n);
        star = dev_alloc<double>(n);
        HIPCHK(hipMemcpyAsync(psi0, psi, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = dmrg::davidson_run(hop, psi, opts, result, stream, nullptr);
        if (st == DMRG_OK) {
            HIPCHK(hipMemcpyAsync(star, psi, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(psi, psi0, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            dmrg::MlpRecord rec{M, slot, rows_per_iter, seed, star};
            st = dmrg::davidson_run(hop, psi, opts, result, stream, &rec);
        }
    } catch (const Error& e) {
        st = dmrg::record_error(e);
    }
    if (psi0) (void)hipFree(psi0);
    if (star) (void)hipFree(star);
    if (n_rows) *n_rows = M->set[slot].rows;
    return st;
}

extern "C" dmrg_status dmrg_mlp_dataset(const dmrg_mlp* M, int32_t slot, int64_t row0, int64_t rows, float* feat,
                                        float* pairs, int64_t* total_rows, void* stream) {
    dmrg::clear_error();
    try {
        if (!M) throw Error(DMRG_ERR_ARG, "NULL handle");
        if (slot != 0 && slot != 1) throw Error(DMRG_ERR_ARG, "slot must be 0 or 1");
        const auto& S = M->set[slot];
        if (total_rows) *total_rows = S.rows;
        if (rows == 0 || (!feat && !pairs)) return DMRG_OK;
        if (row0 < 0 || rows < 0 || row0 + rows > S.rows) throw Error(DMRG_ERR_ARG, "row range outside the dataset");
        HIPCHK(hipSetDevice(M->device));
        hipStream_t s = (hipStream_t)stream;
        if (feat)
            HIPCHK(hipMemcpyAsync(feat, S.feat.get<float>() + row0 * dmrg::kMlpIn, (size_t)rows * dmrg::kMlpIn * sizeof(float),
                                  hipMemcpyDefault, s));
        if (pairs)
            HIPCHK(hipMemcpyAsync(pairs, S.aux.get<float>() + row0 * 3, (size_t)rows * 3 * sizeof(float), hipMemcpyDefault, s));
        HIPCHK(hipStreamSynchronize(s));
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

extern "C" dmrg_status dmrg_mlp_train(dmrg_mlp* M, int32_t steps, int32_t batch, float lr, uint64_t seed, float* losses,
                                      void* stream) {
    dmrg::clear_error();
    try {
        if (!M) throw Error(DMRG_ERR_ARG, "NULL handle");
        if (steps < 0 || batch < 1 || batch > kMaxBatch) throw Error(DMRG_ERR_ARG, "bad steps or batch size");
        if (!(lr > 0.f) || !std::isfinite(lr)) throw Error(DMRG_ERR_ARG, "learning rate must be finite and > 0");
        const int64_t rows = M->set[0].rows;
        if (rows == 0) throw Error(DMRG_ERR_ARG, "training set is empty");
        HIPCHK(hipSetDevice(M->device));
        hipStream_t s = (hipStream_t)stream;
        dmrg::ensure_batch(M, batch);
        const int chunk = 256;
        int64_t* d_idx = M->idx.ensure<int64_t>((size_t)chunk * batch);
        float* d_loss = M->loss.ensure<float>((size_t)std::max(steps, 1));
        SplitMix64 rng(seed);
        std::vector<int64_t> h_idx((size_t)chunk * batch);
        for (int s0 = 0; s0 < steps; s0 += chunk) {
            const int ns = std::min(chunk, steps - s0);
            for (size_t k = 0; k < (size_t)ns * batch; ++k) h_idx[k] = rng.below(rows);
            HIPCHK(hipStreamSynchronize(s));   // the previous chunk's gathers are done with d_idx
            HIPCHK(hipMemcpy(d_idx, h_idx.data(), (size_t)ns * batch * sizeof(int64_t), hipMemcpyHostToDevice));
            for (int k = 0; k < ns; ++k) {
                const int64_t* idx = d_idx + (size_t)k * batch;
                HIPCHK(dmrg::launch_mlp_gather(M->set[0].feat.get<float>(), idx, batch, dmrg::kMlpIn, M->xb.get<float>(), s));
                HIPCHK(dmrg::launch_mlp_gather(M->set[0].aux.get<float>(), idx, batch, 3, M->ab.get<float>(), s));
                dmrg::grad_step(M, M->xb.get<float>(), M->ab.get<float>(), batch, lr, M->grad, d_loss + s0 + k, s);
            }
        }
        HIPCHK(hipStreamSynchronize(s));
        if (losses && steps > 0) HIPCHK(hipMemcpy(losses, d_loss, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost));
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

extern "C" dmrg_status dmrg_mlp_eval(dmrg_mlp* M, int32_t slot, double* loss, double* loss_diag, void* stream) {
    dmrg::clear_error();
    try {
        if (!M) throw Error(DMRG_ERR_ARG, "NULL handle");
        if (slot != 0 && slot != 1) throw Error(DMRG_ERR_ARG, "slot must be 0 or 1");
        const int64_t rows = M->set[slot].rows;
        if (rows == 0) throw Error(DMRG_ERR_ARG, "dataset slot is empty");
        HIPCHK(hipSetDevice(M->device));
        hipStream_t s = (hipStream_t)stream;
        const int64_t chunk = 65536;
        float* m = M->m.ensure<float>(chunk);
        double* red = M->red.ensure<double>((size_t)dmrg::mlp_reduce_blocks(chunk) + 2);
        double tot = 0.0, tot_diag = 0.0;
        for (int64_t r0 = 0; r0 < rows; r0 += chunk) {
            const int64_t nr = std::min(chunk, rows - r0);
            const float* x = M->set[slot].feat.get<float>() + r0 * dmrg::kMlpIn;
            const float* a = M->set[slot].aux.get<float>() + r0 * 3;
            double h[2];
            HIPCHK(dmrg::launch_mlp_forward(M->dev(), x, nr, m, nullptr, nullptr, nullptr, s));
            HIPCHK(dmrg::launch_mlp_loss(a, m, nr, red + 2, red, s));
            HIPCHK(dmrg::launch_mlp_loss(a, nullptr, nr, red + 2, red + 1, s));
            HIPCHK(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            tot += h[0];
            tot_diag += h[1];
        }
        if (loss) *loss = tot / (double)rows;
        if (loss_diag) *loss_diag = tot_diag / (double)rows;
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}
