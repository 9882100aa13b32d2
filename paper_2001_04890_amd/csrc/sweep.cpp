// Two-site DMRG sweeps (Section 2.1): warm-up right blocks grown from the vacuum, then forward and
// backward sweeps that solve the two-site problem at every bond (dmrg_build_blocks + dmrg_davidson)
// and renormalize the growing block with the M leading eigenvectors of its reduced density matrix
// (dmrg_renormalize). Blocks live on the host between bonds (the dmrg_block form of
// dmrg_build_blocks); every computational step runs in the library's device kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "hop.h"

namespace {

using dmrg::Error;

// splitmix64: a counter-based generator (Steele, Lea, Flood 2014) for start vectors and warm-up bases
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {                                      // Box-Muller
        const double u = uniform(), v = uniform();
        return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
    }
};

// A block with no orbitals: the vacuum, one sector (0, 0) of dimension 1, and every operator the
// bond's H.psi and growth ask for (all zero: they sum over the block's orbitals).
struct Vacuum {
    int32_t qn[2] = {0, 0}, dim[1] = {1};
    std::vector<dmrg_op> ops;
    double data[1] = {0.0};
    dmrg_block b{};
    Vacuum(bool right, int L) {
        auto add = [&](int k, int i0, int i1) { ops.push_back(dmrg_op{k, i0, i1, 0, nullptr, nullptr, nullptr}); };
        add(DMRG_OP_H, -1, -1);
        const int n = 2 * L;
        if (!right) {
            for (int W = 0; W < n; ++W) add(DMRG_OP_S, W, -1);
        } else {
            for (int P = 0; P < n; ++P) add(DMRG_OP_U, P, -1);
            for (int P = 0; P < n; ++P) for (int Q = P + 1; Q < n; ++Q) add(DMRG_OP_P, P, Q);
            for (int X = 0; X < n; ++X) for (int Y = X; Y < n; ++Y) add(DMRG_OP_Q, X, Y);
        }
        b = dmrg_block{1, qn, dim, (int32_t)ops.size(), ops.data(), data, 1};
    }
};

struct BlockPtr {
    dmrg_block* p = nullptr;
    BlockPtr() = default;
    explicit BlockPtr(dmrg_block* q) : p(q) {}
    BlockPtr(const BlockPtr&) = delete;
    BlockPtr& operator=(const BlockPtr&) = delete;
    BlockPtr(BlockPtr&& o) noexcept : p(o.p) { o.p = nullptr; }
    BlockPtr& operator=(BlockPtr&& o) noexcept { reset(o.p); o.p = nullptr; return *this; }
    void reset(dmrg_block* q = nullptr) { if (p) dmrg_block_free(p); p = q; }
    ~BlockPtr() { reset(); }
};

struct HopPtr {
    dmrg_hop* p = nullptr;
    void reset(dmrg_hop* q = nullptr) { if (p) dmrg_hop_free(p); p = q; }
    ~HopPtr() { reset(); }
};

struct DevVec {
    double* p = nullptr;
    ~DevVec() { if (p) (void)hipFree(p); }
};

void check(dmrg_status st) {
    if (st < 0) throw Error(st, dmrg::last_error());
}

// Kept states per enlarged sector for a warm-up block of `k` orbitals: a Gaussian weight around the
// filling N k / L (width sqrt(k) / 2 + 1) times the sector size, water-filled up to m states under
// the sector caps.
std::vector<int> warmup_kept(const std::vector<int32_t>& qn, const std::vector<int32_t>& dims, int k, int L, int na,
                             int nb, int m) {
    const size_t n = dims.size();
    std::vector<int> kept(n, 0);
    int64_t total = 0;
    for (int d : dims) total += d;
    if (total <= m) {
        for (size_t i = 0; i < n; ++i) kept[i] = dims[i];
        return kept;
    }
    const double ca = (double)na * k / L, cb = (double)nb * k / L, sg = std::sqrt((double)k) / 2.0 + 1.0;
    std::vector<double> w(n);
    for (size_t i = 0; i < n; ++i) {
        const double da = qn[2 * i] - ca, db = qn[2 * i + 1] - cb;
        w[i] = dims[i] * std::exp(-(da * da + db * db) / (2.0 * sg * sg));
    }
    int left = m;
    for (int round = 0; round < 64 && left > 0; ++round) {
        double ws = 0.0;
        for (size_t i = 0; i < n; ++i) if (kept[i] < dims[i]) ws += w[i];
        if (ws <= 0.0) break;
        int added = 0;
        for (size_t i = 0; i < n && left > 0; ++i) {
            if (kept[i] >= dims[i]) continue;
            int a = (int)std::floor(left * w[i] / ws);
            a = std::min({a, dims[i] - kept[i], left - added});
            kept[i] += a;
            added += a;
        }
        left -= added;
        if (added == 0) {                                 // hand out the rest one by one, heaviest first
            std::vector<size_t> order(n);
            for (size_t i = 0; i < n; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return w[x] > w[y]; });
            for (size_t i : order) if (left > 0 && kept[i] < dims[i]) { ++kept[i]; --left; }
            if (left > 0) break;
        }
    }
    return kept;
}

// Random orthonormal columns (classical Gram-Schmidt twice on Gaussian vectors), d x k row-major.
void random_columns(SplitMix& g, int d, int k, std::vector<double>& out) {
    std::vector<double> Q((size_t)d * k);
    for (int c = 0; c < k; ++c) {
        std::vector<double> v(d);
        for (double& x : v) x = g.normal();
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j < c; ++j) {
                double dot = 0.0;
                for (int r = 0; r < d; ++r) dot += Q[(size_t)r * k + j] * v[r];
                for (int r = 0; r < d; ++r) v[r] -= dot * Q[(size_t)r * k + j];
            }
        double nrm = 0.0;
        for (double x : v) nrm += x * x;
        nrm = std::sqrt(nrm);
        for (int r = 0; r < d; ++r) Q[(size_t)r * k + c] = v[r] / nrm;
    }
    out.insert(out.end(), Q.begin(), Q.end());
}

}  // namespace

extern "C" dmrg_status dmrg_sweep(const dmrg_problem* p, const dmrg_sweep_opts* o, dmrg_sweep_result* res) {
    dmrg::clear_error();
    try {
        if (!p || !o || !res || !p->h || !p->eri) throw Error(DMRG_ERR_ARG, "NULL argument");
        const int L = p->n_orb;
        if (L < 2) throw Error(DMRG_ERR_ARG, "need n_orb >= 2");
        if (o->n_sweeps < 1 || !o->m_per_sweep || o->m_warmup < 1) throw Error(DMRG_ERR_ARG, "bad sweep schedule");
        for (int k = 0; k < o->n_sweeps; ++k)
            if (o->m_per_sweep[k] < 1) throw Error(DMRG_ERR_ARG, "bond dimensions must be >= 1");
        res->left_block = res->right_block = nullptr;
        if (o->keep_site < 0 || (o->keep_site > 0 && o->keep_site > L - 3))
            throw Error(DMRG_ERR_ARG, "keep_site must be 0 (none) or 1 .. n_orb - 3");
        if (o->mlp && (o->mlp_from_sweep < 0 || o->mlp_from_sweep >= o->n_sweeps))
            throw Error(DMRG_ERR_ARG, "mlp_from_sweep must be 0 .. n_sweeps - 1");
        const double t0 = dmrg::now_seconds();
        hipStream_t s = (hipStream_t)o->stream;
        HIPCHK(hipSetDevice(o->device));
        SplitMix g{o->seed};
        dmrg_build_opts bo{};
        bo.device = o->device;
        bo.want_split = o->precision == DMRG_PREC_SPLIT2 ? 1 : 0;
        bo.stream = o->stream;
        dmrg_dav_opts dav{};
        dav.tol = o->tol;
        dav.max_iter = o->max_iter;
        dav.max_sub = o->max_sub;
        dav.precision = o->precision;
        dav.fp64_polish = o->fp64_polish;
        dav.split_tol = o->split_tol;
        dav.precond = DMRG_PRECOND_DIAG;
        Vacuum vac_left(false, L), vac_right(true, L);
        // right[k]: the right block of the last k orbitals (L - k .. L - 1); left[k]: orbitals 0 .. k-1
        std::vector<BlockPtr> right(L), left(L);
        auto right_of = [&](int k) -> const dmrg_block* { return k == 0 ? &vac_right.b : right[k].p; };
        auto left_of = [&](int k) -> const dmrg_block* { return k == 0 ? &vac_left.b : left[k].p; };
        // warm-up: grow the right blocks from the vacuum, keeping m_warmup random states per step
        for (int k = 0; k + 2 < L; ++k) {
            dmrg_problem q = *p;
            q.site = L - k - 2;                  // the block of the last k orbitals is the right block of bond (L-k-2, L-k-1)
            int32_t nq = 0;
            check(dmrg_block_grow_layout(right_of(k), 1, &nq, nullptr, nullptr));
            std::vector<int32_t> qn(2 * nq), dims(nq);
            check(dmrg_block_grow_layout(right_of(k), 1, &nq, qn.data(), dims.data()));
            const std::vector<int> kept = warmup_kept(qn, dims, k + 1, L, p->n_alpha, p->n_beta, o->m_warmup);
            std::vector<int32_t> kp(kept.begin(), kept.end());
            std::vector<double> O;
            for (int i = 0; i < nq; ++i) random_columns(g, dims[i], kept[i], O);
            dmrg_block* nb = nullptr;
            check(dmrg_block_grow(&q, right_of(k), 1, kp.data(), O.data(), &bo, &nb));
            right[k + 1].reset(nb);
            if (o->verbose) std::fprintf(stderr, "[dmrg_sweep] warm-up right block of %d orbitals\n", k + 1);
        }
        int n_solves = 0;
        double best = INFINITY;
        HopPtr hop;
        DevVec psi, psi2;
        int64_t psi_n = 0;
        for (int i = 0; i < res->capacity; ++i) {
            if (res->energies_alt) res->energies_alt[i] = std::nan("");
            if (res->iters_alt) res->iters_alt[i] = -1;
        }
        auto solve = [&](int site, int sweep, int m) {
            dmrg_problem q = *p;
            q.site = site;
            hop.reset();
            dmrg_hop* hp = nullptr;
            check(dmrg_build_blocks(&q, left_of(site), right_of(L - site - 2), &bo, &hp));
            hop.reset(hp);
            int64_t n = 0;
            check(dmrg_hop_layout(hop.p, &n, nullptr, nullptr, nullptr, nullptr));
            if (n > psi_n) {
                for (DevVec* v : {&psi, &psi2}) {
                    if (v->p) (void)hipFree(v->p);
                    v->p = nullptr;
                    if (hipMalloc(&v->p, (size_t)n * sizeof(double)) != hipSuccess)
                        throw Error(DMRG_ERR_NOMEM, "device allocation failed (sweep vector)");
                }
                psi_n = n;
            }
            std::vector<double> x((size_t)n);
            for (double& v : x) v = g.normal();
            HIPCHK(hipMemcpyAsync(psi.p, x.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
            dmrg_dav_result r{};
            const bool learned = o->mlp && sweep >= o->mlp_from_sweep;
            const bool shadow = learned && o->mlp_shadow;
            if (shadow) {
                // the learned solve on the same problem from the same start vector; the sweep goes on
                // with the diagonal one below
                HIPCHK(hipMemcpyAsync(psi2.p, x.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
                dmrg_dav_opts d2 = dav;
                d2.precond = DMRG_PRECOND_MLP;
                d2.mlp = o->mlp;
                dmrg_dav_result r2{};
                check(dmrg_davidson(hop.p, psi2.p, &d2, &r2, s));
                if (n_solves < res->capacity) {
                    if (res->energies_alt) res->energies_alt[n_solves] = r2.energy;
                    if (res->iters_alt) res->iters_alt[n_solves] = r2.iters;
                }
            }
            dav.precond = learned && !shadow ? DMRG_PRECOND_MLP : DMRG_PRECOND_DIAG;
            dav.mlp = learned && !shadow ? o->mlp : nullptr;
            const dmrg_status st = dmrg_davidson(hop.p, psi.p, &dav, &r, s);
            check(st);
            if (n_solves < res->capacity) {
                if (res->energies) res->energies[n_solves] = r.energy;
                if (res->iters) res->iters[n_solves] = r.iters;
                if (res->sites) res->sites[n_solves] = site;
            }
            if (o->verbose)
                std::fprintf(stderr, "[dmrg_sweep] sweep %d bond (%d,%d) M %d: E %.12f resid %.2e iters %d%s\n", sweep,
                             site, site + 1, m, r.energy, r.resid, r.iters, st == DMRG_NOT_CONVERGED ? " (not converged)" : "");
            best = std::min(best, r.energy);
            ++n_solves;
            res->energy = r.energy;
            if (st == DMRG_NOT_CONVERGED) ++res->n_not_converged;
        };
        auto record_disc = [&](double d) {
            if (n_solves - 1 < res->capacity && res->discarded) res->discarded[n_solves - 1] = d;
        };
        res->n_not_converged = 0;
        res->energy = INFINITY;
        for (int sw = 0; sw < o->n_sweeps; ++sw) {
            const int m = o->m_per_sweep[sw];
            // forward: bonds 0 .. L-2, growing the left block
            // (after the first sweep the backward sweep's last solve, at bond (0, 1), has grown the left block)
            for (int site = (sw == 0 ? 0 : 1); site <= L - 2; ++site) {
                solve(site, sw, m);
                if (site < L - 2) {
                    dmrg_block* nb = nullptr;
                    double disc = 0.0;
                    check(dmrg_renormalize(hop.p, psi.p, 0, m, &nb, &disc, s));
                    left[site + 1].reset(nb);
                    record_disc(disc);
                }
            }
            // backward: bonds L-3 .. 0 (the last forward solve at L-2 grows the right block first)
            {
                dmrg_block* nb = nullptr;
                double disc = 0.0;
                check(dmrg_renormalize(hop.p, psi.p, 1, m, &nb, &disc, s));
                right[1].reset(nb);
                record_disc(disc);
            }
            for (int site = L - 3; site >= 0; --site) {
                solve(site, sw, m);
                dmrg_block* nb = nullptr;
                double disc = 0.0;
                if (site > 0) {
                    check(dmrg_renormalize(hop.p, psi.p, 1, m, &nb, &disc, s));
                    right[L - site - 1].reset(nb);
                } else if (sw + 1 < o->n_sweeps) {
                    // bond (0, 1) starts the next forward sweep: grow the left block with the next M
                    check(dmrg_renormalize(hop.p, psi.p, 0, o->m_per_sweep[sw + 1], &nb, &disc, s));
                    left[1].reset(nb);
                }
                record_disc(disc);
            }
        }
        hop.reset();
        HIPCHK(hipStreamSynchronize(s));
        if (o->keep_site > 0) {
            // left[keep_site]: last grown in the final forward pass; right[L - keep_site - 2]: in the
            // final backward pass, before its solve at this bond
            res->left_block = left[o->keep_site].p;
            left[o->keep_site].p = nullptr;
            res->right_block = right[L - o->keep_site - 2].p;
            right[L - o->keep_site - 2].p = nullptr;
        }
        res->n_solves = n_solves;
        res->best_energy = best;
        res->seconds = dmrg::now_seconds() - t0;
        return res->n_not_converged ? DMRG_NOT_CONVERGED : DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    } catch (const std::exception& e) {   // nothing else may cross the C boundary
        dmrg::last_error() = e.what();
        return DMRG_ERR_ARG;
    }
}
