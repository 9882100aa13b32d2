// Batched, device-resident Davidson (Sections 2.1, 2.2.1) over the parts of a merged handle: the
// host only enqueues fixed launch sequences (one per subspace size, optionally captured as hipGraphs)
// and reads the parts' status every few iterations. The arithmetic is that of dmrg_davidson: basis
// V with W = H V, Rayleigh-Ritz on G = V^T W, Ritz vector u = V s, residual r = W s - theta u,
// diagonal correction, Gram-Schmidt twice with normalization twice, restart at max_sub to
// {u, u_prev}; here per part, with the Rayleigh-Ritz step on the device (davidson_batch.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <vector>

#include "batch.h"
#include "hop.h"

namespace {

using dmrg::Error;

constexpr int64_t kChunk = 1024;     // reduction chunk (coefficients): four per thread of a 256-wide workgroup
constexpr int kCheckEvery = 4;       // iterations between status reads

struct Dev {
    std::vector<void*> allocs;
    ~Dev() { for (void* p : allocs) (void)hipFree(p); }
    template <class T> T* get(size_t n, hipStream_t s) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
            throw Error(DMRG_ERR_NOMEM, "device allocation failed (batched Davidson work space)");
        allocs.push_back(p);
        HIPCHK(hipMemsetAsync(p, 0, std::max<size_t>(n, 1) * sizeof(T), s));   // not inside a graph
        return static_cast<T*>(p);
    }
};

// The parts' status array doubles as the part mask of the merged H.psi launches (see kPartActive),
// so that parts that have converged cost no H.psi work; the handle drops it on every exit.
static_assert(dmrg::kActive == dmrg::kPartActive, "part status and part mask use one active value");
struct MaskGuard {
    dmrg_hop* H;
    ~MaskGuard() { H->d_active = nullptr; }
};

struct Graphs {
    std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> g;
    ~Graphs() { clear(); }
    void clear() {
        for (auto& kv : g) {
            (void)hipGraphExecDestroy(kv.second.second);
            (void)hipGraphDestroy(kv.second.first);
        }
        g.clear();
    }
};

}  // namespace

extern "C" dmrg_status dmrg_davidson_batch(dmrg_hop* H, double* psi, const dmrg_dav_opts* o,
                                           dmrg_dav_batch_result* res, void* stream) {
    dmrg::clear_error();
    hipStream_t cap = nullptr;
    try {
        if (!H || !psi || !o || !res) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (H->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle has no device state");
        if (H->trimmed) throw Error(DMRG_ERR_UNSUPPORTED, "handle was trimmed (dmrg_hop_trim)");
        if (o->max_sub < 3 || o->max_sub > 64 || o->max_iter < 1 || !(o->tol > 0)) throw Error(DMRG_ERR_ARG, "bad Davidson options");
        if (o->use_graph != 0 && o->use_graph != 1) throw Error(DMRG_ERR_ARG, "use_graph must be 0 or 1");
        if (o->precond != DMRG_PRECOND_DIAG) throw Error(DMRG_ERR_UNSUPPORTED, "the batched Davidson uses the diagonal preconditioner");
        if (o->precision != DMRG_PREC_FP64 && o->precision != DMRG_PREC_SPLIT2) throw Error(DMRG_ERR_ARG, "unknown precision");
        if (o->precision == DMRG_PREC_SPLIT2 && !H->has_split) throw Error(DMRG_ERR_UNSUPPORTED, "handle built without split operators");
        const int P = H->n_parts;
        if (res->capacity > 0 && res->capacity < P) throw Error(DMRG_ERR_ARG, "result arrays shorter than the number of parts");
        HIPCHK(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)stream;
        const double t0 = dmrg::now_seconds();
        const int64_t n = H->n_coeff;
        const int K = o->max_sub;
        // chunk table: every chunk inside one part
        std::vector<dmrg::BChunk> chunks;
        std::vector<int32_t> part_chunk(P + 1, 0);
        for (int p = 0; p < P; ++p) {
            part_chunk[p] = (int32_t)chunks.size();
            const int64_t b = H->part_coeff[p], e = H->part_coeff[p + 1];
            if (e <= b) throw Error(DMRG_ERR_ARG, "empty part");
            for (int64_t c = b; c < e; c += kChunk) chunks.push_back({c, std::min(e, c + kChunk), p, 0});
        }
        part_chunk[P] = (int32_t)chunks.size();
        Dev d;
        dmrg::BatchDev B{};
        const int ld = K + dmrg::kDotTail;
        auto* d_chunks = d.get<dmrg::BChunk>(chunks.size(), s);
        auto* d_pc = d.get<int32_t>(P + 1, s);
        HIPCHK(hipMemcpyAsync(d_chunks, chunks.data(), chunks.size() * sizeof(chunks[0]), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_pc, part_chunk.data(), (P + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
        B.chunks = d_chunks;
        B.n_chunks = (int)chunks.size();
        B.part_chunk = d_pc;
        B.n_parts = P;
        B.n = n;
        B.K = K;
        B.partial = d.get<double>(chunks.size() * (size_t)ld, s);
        B.dots = d.get<double>((size_t)P * ld, s);
        B.G = d.get<double>((size_t)P * K * K, s);
        B.s = d.get<double>((size_t)P * K, s);
        B.ms = d.get<double>((size_t)P * K, s);
        B.y1 = d.get<double>((size_t)P * K, s);
        B.theta = d.get<double>(P, s);
        B.rnorm = d.get<double>(P, s);
        B.status = d.get<int32_t>(P, s);
        B.iters = d.get<int32_t>(P, s);
        B.Qp = d.get<double>((size_t)P * K * K, s);
        B.qk = d.get<int32_t>(P, s);
        double* V = d.get<double>((size_t)K * n, s);
        double* W = d.get<double>((size_t)K * n, s);
        double* u = d.get<double>(n, s);
        double* r = d.get<double>(n, s);
        double* t = d.get<double>(n, s);
        double* prev = d.get<double>(n, s);
        double* S = d.get<double>((size_t)4 * n, s);
        HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        MaskGuard mask_guard{H};
        const char* mk = std::getenv("DMRG_BATCH_PART_MASK");   // "0": every part's H.psi work runs to the end
        if (!(mk && mk[0] == '0') && P <= 32767) H->d_active = B.status;   // pass-1 groups hold 16-bit part numbers
        int matvecs = 0, n_graphs = 0;
        int prec = o->precision;
        auto matvec = [&](const double* x, double* y, hipStream_t st) {
            dmrg::hpsi_enqueue(H, x, y, 1, prec, st);
        };
        auto orth_norm = [&](double* x, int k, hipStream_t st) {
            for (int rep = 0; rep < 2; ++rep) {
                for (int pass = 0; pass < 2 && k > 0; ++pass) {
                    HIPCHK(dmrg::bdots(B, V, k, x, 0, st));
                    HIPCHK(dmrg::bproject(B, V, k, x, st));
                }
                const int slot = rep == 0 ? dmrg::kSlotNorm1 : dmrg::kSlotNorm2;
                HIPCHK(dmrg::bdots(B, x, 1, x, K + slot, st));
                HIPCHK(dmrg::bscale(B, x, slot, st));
            }
        };
        // one iteration at subspace size k (the restart at k == K included)
        auto iteration = [&](int k, double tol, hipStream_t st) {
            HIPCHK(dmrg::brr(B, k, st));
            HIPCHK(dmrg::bcombine(B, V, k, B.s, u, 0.0, st));
            HIPCHK(dmrg::bcombine(B, W, k, B.s, r, 0.0, st));
            HIPCHK(dmrg::bcombine(B, V, k, B.ms, r, 1.0, st));
            HIPCHK(dmrg::bdots(B, r, 1, r, K + dmrg::kSlotResid, st));
            HIPCHK(dmrg::bcheck(B, tol, st));
            HIPCHK(dmrg::bprecond(B, r, H->d_diag, t, st));
            int kk = k;
            if (k == K) {
                HIPCHK(dmrg::bdots(B, V, K, prev, 0, st));
                HIPCHK(dmrg::brestart(B, st));
                HIPCHK(dmrg::bcombine(B, V, K, B.s, S, 0.0, st));
                HIPCHK(dmrg::bcombine(B, V, K, B.y1, S + n, 0.0, st));
                HIPCHK(dmrg::bcombine(B, W, K, B.s, S + 2 * n, 0.0, st));
                HIPCHK(dmrg::bcombine(B, W, K, B.y1, S + 3 * n, 0.0, st));
                HIPCHK(dmrg::bcopy(B, S, V, false, st));
                HIPCHK(dmrg::bcopy(B, S + n, V + n, false, st));
                HIPCHK(dmrg::bcopy(B, S + 2 * n, W, false, st));
                HIPCHK(dmrg::bcopy(B, S + 3 * n, W + n, false, st));
                kk = 2;
            }
            HIPCHK(dmrg::bcopy(B, u, prev, false, st));
            double* vk = V + (size_t)kk * n;
            HIPCHK(dmrg::bcopy(B, t, vk, false, st));
            orth_norm(vk, kk, st);
            matvec(vk, W + (size_t)kk * n, st);
            HIPCHK(dmrg::bdots(B, V, kk + 1, W + (size_t)kk * n, 0, st));
            HIPCHK(dmrg::bgcol(B, kk, st));
            return kk + 1;
        };
        std::vector<int32_t> st_h(P);
        auto any_active = [&]() {
            HIPCHK(hipMemcpyAsync(st_h.data(), B.status, P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int v : st_h) if (v == dmrg::kActive) return true;
            return false;
        };
        struct Phase { int prec; double tol; };
        std::vector<Phase> phases;
        if (o->precision == DMRG_PREC_SPLIT2 && o->fp64_polish)
            phases = {{DMRG_PREC_SPLIT2, std::max(o->split_tol, o->tol)}, {DMRG_PREC_FP64, o->tol}};
        else
            phases = {{o->precision, o->tol}};
        int it_total = 0;
        for (size_t ph = 0; ph < phases.size(); ++ph) {
            prec = phases[ph].prec;
            const double tol = phases[ph].tol;
            // start: V0 = psi (first phase) or the Ritz vectors, normalized per part; W0 = H V0
            HIPCHK(dmrg::bactivate(B, ph == 0, s));
            HIPCHK(dmrg::bcopy(B, ph == 0 ? psi : u, V, true, s));
            orth_norm(V, 0, s);
            {
                // every part's start vector must have a norm
                std::vector<double> dh((size_t)P * ld);
                HIPCHK(hipMemcpyAsync(dh.data(), B.dots, dh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                for (int p = 0; p < P; ++p) {
                    const double nn = dh[(size_t)p * ld + K + dmrg::kSlotNorm1];
                    if (!std::isfinite(nn)) throw Error(DMRG_ERR_NAN, "non-finite start vector");
                    if (!(nn > 0.0)) throw Error(DMRG_ERR_ARG, "a part's start vector is zero");
                }
            }
            matvec(V, W, s);
            ++matvecs;
            HIPCHK(dmrg::bdots(B, V, 1, W, 0, s));
            HIPCHK(dmrg::bgcol(B, 0, s));
            Graphs graphs;
            int k = 1;
            bool active = true;
            for (int it = 0; it < o->max_iter && active; ++it) {
                const int key = k;
                int next = 0;
                if (o->use_graph) {
                    auto f = graphs.g.find(key);
                    if (f == graphs.g.end()) {
                        hipGraph_t g = nullptr;
                        hipGraphExec_t e = nullptr;
                        HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
                        try {
                            next = iteration(k, tol, cap);
                        } catch (...) {
                            hipGraph_t junk = nullptr;
                            (void)hipStreamEndCapture(cap, &junk);
                            if (junk) (void)hipGraphDestroy(junk);
                            throw;
                        }
                        HIPCHK(hipStreamEndCapture(cap, &g));
                        HIPCHK(hipGraphInstantiate(&e, g, nullptr, nullptr, 0));
                        f = graphs.g.emplace(key, std::make_pair(g, e)).first;
                        ++n_graphs;
                    } else {
                        next = k == K ? 3 : k + 1;
                    }
                    HIPCHK(hipGraphLaunch(f->second.second, s));
                } else {
                    next = iteration(k, tol, s);
                }
                ++matvecs;
                ++it_total;
                k = next;
                if ((it + 1) % kCheckEvery == 0 || it + 1 == o->max_iter) active = any_active();
            }
        }
        HIPCHK(dmrg::bcopy(B, u, psi, true, s));
        std::vector<double> th(P), rn(P);
        std::vector<int32_t> its(P);
        HIPCHK(hipMemcpyAsync(th.data(), B.theta, P * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(rn.data(), B.rnorm, P * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(its.data(), B.iters, P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(st_h.data(), B.status, P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        (void)hipStreamDestroy(cap);
        cap = nullptr;
        int n_conv = 0;
        bool nonfinite = false;
        for (int p = 0; p < P; ++p) {
            const int code = st_h[p] == dmrg::kConverged ? 0 : st_h[p] == dmrg::kStalled ? 2 : 1;
            if (st_h[p] == dmrg::kNonFinite) nonfinite = true;
            n_conv += code == 0;
            if (res->capacity >= P) {
                if (res->energy) res->energy[p] = th[p];
                if (res->resid) res->resid[p] = rn[p];
                if (res->iters) res->iters[p] = its[p];
                if (res->status) res->status[p] = code;
            }
        }
        res->n_parts = P;
        res->n_converged = n_conv;
        res->matvecs = matvecs;
        res->graphs = n_graphs;
        res->t_total = dmrg::now_seconds() - t0;
        (void)it_total;
        if (nonfinite) throw Error(DMRG_ERR_NAN, "non-finite residual in the batched Davidson");
        if (n_conv < P) { dmrg::last_error() = "batched Davidson: not every part converged"; return DMRG_NOT_CONVERGED; }
        return DMRG_OK;
    } catch (const Error& e) {
        if (cap) (void)hipStreamDestroy(cap);
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        if (cap) (void)hipStreamDestroy(cap);
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    } catch (const std::exception& e) {   // nothing else may cross the C boundary
        if (cap) (void)hipStreamDestroy(cap);
        dmrg::last_error() = e.what();
        return DMRG_ERR_ARG;
    }
}
