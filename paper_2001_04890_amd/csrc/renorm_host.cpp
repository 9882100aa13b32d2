// Density matrices, truncation and renormalization (Section 2.1: Eq. renorm, Eq. renorm_mat; Section
// 2.2.2): rho^L / rho^R of the enlarged blocks on the GPU, the M-state cut on the host, and
// O^T A O per sector block on the GPU.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "eigen.h"
#include "hop.h"
#include "renorm.h"

using dmrg::BlockIn;
using dmrg::Error;
using dmrg::kSiteQn;
using dmrg::RenormItem;
using dmrg::RenormWork;
using dmrg::EnlargedLayout;

dmrg::EnlargedLayout dmrg::enlarged_layout(const BlockIn& B, bool right) {
    std::map<std::pair<int, int>, std::vector<std::array<int, 3>>> groups;
    std::map<std::pair<int, int>, int> dims;
    auto add = [&](int x, int y, int sec, int site) {
        const std::pair<int, int> q{B.qa[sec] + kSiteQn[site][0], B.qb[sec] + kSiteQn[site][1]};
        int& d = dims[q];
        groups[q].push_back({x, y, d});
        d += B.dim[sec];
    };
    if (!right) {
        for (int a = 0; a < B.n_sec; ++a)
            if (B.dim[a] > 0)
                for (int b = 0; b < 4; ++b) add(a, b, a, b);
    } else {
        for (int c = 0; c < 4; ++c)
            for (int d = 0; d < B.n_sec; ++d)
                if (B.dim[d] > 0) add(c, d, d, c);
    }
    EnlargedLayout R;
    R.off.push_back(0);
    for (auto& kv : groups) {
        const int d = dims[kv.first];
        R.qn.push_back(kv.first);
        R.dim.push_back(d);
        R.off.push_back(R.off.back() + (int64_t)d * d);
        R.groups.push_back(kv.second);
    }
    return R;
}

// ---------------------------------------------------------------- reduced density matrices
namespace {
// psi read as the matrix psi_{(l s_l),(s_r r)} (Section 2.1): rows are the enlarged left block,
// columns the enlarged right block, both in the layout of dmrg::enlarged_layout.
using RdmLayout = dmrg::EnlargedLayout;

RdmLayout rdm_layout(const dmrg_hop& H, bool right) {
    if (H.n_parts != 1) throw Error(DMRG_ERR_UNSUPPORTED, "merged handle: density matrices are per problem");
    return dmrg::enlarged_layout(right ? H.right : H.left, right);
}

// psi blocks of one group, in the order of the other side's groups: left group (a, b) -> blocks
// (a, b, c, d) for c = 0..3; right group (c, d) -> blocks (a, b, c, d) for (a, b) in (a, b) order.
std::vector<int> rdm_group_blocks(const dmrg_hop& H, bool right, int x, int y) {
    std::vector<int> ids;
    if (!right) {
        for (int c = 0; c < 4; ++c) {
            const int id = H.blk_index[(x * 4 + y) * 4 + c];
            if (id >= 0) ids.push_back(id);
        }
    } else {
        for (int a = 0; a < H.left.n_sec; ++a)
            for (int b = 0; b < 4; ++b) {
                const int id = H.blk_index[(a * 4 + b) * 4 + x];
                if (id >= 0 && H.blk[id][3] == y) ids.push_back(id);
            }
    }
    return ids;
}

dmrg_status rdm_layout_entry(const dmrg_hop* H, bool right, int32_t* n_sec, int32_t* qn, int32_t* dims,
                             int64_t* offsets) {
    dmrg::clear_error();
    try {
        if (!H || !n_sec) throw Error(DMRG_ERR_ARG, "NULL argument");
        const RdmLayout R = rdm_layout(*H, right);
        *n_sec = (int32_t)R.dim.size();
        for (size_t i = 0; i < R.dim.size(); ++i) {
            if (qn) { qn[2 * i] = R.qn[i].first; qn[2 * i + 1] = R.qn[i].second; }
            if (dims) dims[i] = R.dim[i];
        }
        if (offsets)
            for (size_t i = 0; i < R.off.size(); ++i) offsets[i] = R.off[i];
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    }
}

dmrg_status rdm_entry(dmrg_hop* H, bool right, const double* psi, double* rho, int64_t rho_len, void* stream) {
    dmrg::clear_error();
    try {
        if (!H || !psi || !rho) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (H->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle has no device state");
        const RdmLayout R = rdm_layout(*H, right);
        if (rho_len != R.off.back()) throw Error(DMRG_ERR_SHAPE, "rho_len must be the sum of dim_q^2 of the sectors");
        // per group: its psi blocks; within a sector every group has the same inner dimensions
        // (m_d on the left side, m_a on the right), checked here
        std::vector<dmrg::RdmItem> items;
        std::vector<int64_t> gblk;
        std::vector<int32_t> inner;
        const BlockIn& B = right ? H->right : H->left;
        for (size_t qi = 0; qi < R.dim.size(); ++qi) {
            const auto& G = R.groups[qi];
            const int in0 = (int)inner.size();
            std::vector<int> g0(G.size());
            int n_in = -1;
            for (size_t k = 0; k < G.size(); ++k) {
                g0[k] = (int)gblk.size();
                const std::vector<int> ids = rdm_group_blocks(*H, right, G[k][0], G[k][1]);
                if (k > 0 && (int)ids.size() != n_in)
                    throw Error(DMRG_ERR_ARG, "internal: groups of a sector meet different blocks");
                for (size_t t = 0; t < ids.size(); ++t) {
                    const int m = right ? H->blk_ma[ids[t]] : H->blk_md[ids[t]];
                    if (k == 0) inner.push_back(m);
                    else if (inner[in0 + t] != m) throw Error(DMRG_ERR_ARG, "internal: groups of a sector meet different blocks");
                    gblk.push_back(H->blk_off[ids[t]]);
                }
                n_in = (int)ids.size();
            }
            for (size_t k = 0; k < G.size(); ++k)
                for (size_t k2 = 0; k2 < G.size(); ++k2) {
                    dmrg::RdmItem it{};
                    it.rho_off = R.off[qi] + (int64_t)G[k][2] * R.dim[qi] + G[k2][2];
                    it.ld = R.dim[qi];
                    it.ma = B.dim[right ? G[k][1] : G[k][0]];
                    it.ma2 = B.dim[right ? G[k2][1] : G[k2][0]];
                    it.g = g0[k];
                    it.g2 = g0[k2];
                    it.cd = in0;
                    it.n_cd = n_in;
                    items.push_back(it);
                }
        }
        if (items.size() > (size_t)INT32_MAX) throw Error(DMRG_ERR_UNSUPPORTED, "too many density-matrix items");
        HIPCHK(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)stream;
        void *d_items = nullptr, *d_g = nullptr, *d_c = nullptr;
        auto release = [&]() {
            if (d_items) (void)hipFree(d_items);
            if (d_g) (void)hipFree(d_g);
            if (d_c) (void)hipFree(d_c);
        };
        try {
            HIPCHK(hipMalloc(&d_items, std::max<size_t>(1, items.size()) * sizeof(dmrg::RdmItem)));
            HIPCHK(hipMalloc(&d_g, std::max<size_t>(1, gblk.size()) * sizeof(int64_t)));
            HIPCHK(hipMalloc(&d_c, std::max<size_t>(1, inner.size()) * sizeof(int32_t)));
            if (!items.empty())
                HIPCHK(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(dmrg::RdmItem), hipMemcpyHostToDevice, s));
            if (!gblk.empty())
                HIPCHK(hipMemcpyAsync(d_g, gblk.data(), gblk.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
            if (!inner.empty())
                HIPCHK(hipMemcpyAsync(d_c, inner.data(), inner.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
            const auto* di = static_cast<const dmrg::RdmItem*>(d_items);
            const auto* dg = static_cast<const int64_t*>(d_g);
            const auto* dc = static_cast<const int32_t*>(d_c);
            if (right) HIPCHK(dmrg::launch_rdm_right(di, (int)items.size(), dg, dc, psi, rho, s));
            else HIPCHK(dmrg::launch_rdm_left(di, (int)items.size(), dg, dc, psi, rho, s));
            HIPCHK(hipStreamSynchronize(s));   // the host work lists and scratch end here
        } catch (...) {
            (void)hipStreamSynchronize(s);
            release();
            throw;
        }
        release();
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}
}  // namespace

extern "C" dmrg_status dmrg_rdm_left_layout(const dmrg_hop* H, int32_t* n_sec, int32_t* qn, int32_t* dims,
                                            int64_t* offsets) {
    return rdm_layout_entry(H, false, n_sec, qn, dims, offsets);
}

extern "C" dmrg_status dmrg_rdm_left(dmrg_hop* H, const double* psi, double* rho, int64_t rho_len, void* stream) {
    return rdm_entry(H, false, psi, rho, rho_len, stream);
}

extern "C" dmrg_status dmrg_rdm_right_layout(const dmrg_hop* H, int32_t* n_sec, int32_t* qn, int32_t* dims,
                                             int64_t* offsets) {
    return rdm_layout_entry(H, true, n_sec, qn, dims, offsets);
}

extern "C" dmrg_status dmrg_rdm_right(dmrg_hop* H, const double* psi, double* rho, int64_t rho_len, void* stream) {
    return rdm_entry(H, true, psi, rho, rho_len, stream);
}

extern "C" dmrg_status dmrg_truncate(const double* rho, int32_t n_sec, const int32_t* dims, const int64_t* offsets,
                                     int32_t M, int32_t* kept, double* evals, double* vecs, double* discarded) {
    dmrg::clear_error();
    try {
        if (!rho || !dims || !offsets || !kept || !evals || !vecs || !discarded) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (n_sec < 0 || M < 0) throw Error(DMRG_ERR_ARG, "n_sec and M must be >= 0");
        int64_t pos = 0;
        std::vector<int64_t> eoff(n_sec + 1, 0);
        for (int i = 0; i < n_sec; ++i) {
            if (dims[i] < 0 || offsets[i] != pos) throw Error(DMRG_ERR_SHAPE, "offsets must be the prefix sums of dims^2");
            pos += (int64_t)dims[i] * dims[i];
            eoff[i + 1] = eoff[i] + dims[i];
        }
        for (int64_t k = 0; k < pos; ++k)
            if (!std::isfinite(rho[k])) throw Error(DMRG_ERR_NAN, "non-finite density matrix element");
        // one sector: eigenpairs in descending eigenvalue order, each vector's largest-magnitude
        // component positive, written to the sector's own parts of evals and vecs
        std::vector<double> trace(n_sec, 0.0);
        auto solve = [&](int i) {
            const int n = dims[i];
            std::vector<double> A(rho + offsets[i], rho + offsets[i] + (int64_t)n * n), ev, vt;
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < r; ++c)              // symmetrize: the input is psi psi^T up to rounding
                    A[(size_t)r * n + c] = 0.5 * (A[(size_t)r * n + c] + A[(size_t)c * n + r]);
            for (int r = 0; r < n; ++r) trace[i] += A[(size_t)r * n + r];
            dmrg::sym_eigen(n, A.data(), ev, vt, 1);     // ascending, eigenvectors as rows
            double* out = vecs + offsets[i];
            for (int k = 0; k < n; ++k) {
                const double* v = vt.data() + (size_t)(n - 1 - k) * n;
                int big = 0;
                for (int r = 1; r < n; ++r)
                    if (std::fabs(v[r]) > std::fabs(v[big])) big = r;
                const double sg = v[big] < 0.0 ? -1.0 : 1.0;
                for (int r = 0; r < n; ++r) out[(size_t)r * n + k] = sg * v[r];
                evals[eoff[i] + k] = ev[n - 1 - k];
            }
        };
        // sectors are independent: a few host threads take them largest first; the first error (in
        // sector order) is reported
        std::vector<int> todo(n_sec);
        for (int i = 0; i < n_sec; ++i) todo[i] = i;
        std::stable_sort(todo.begin(), todo.end(), [&](int x, int y) { return dims[x] > dims[y]; });
        std::vector<dmrg_status> st(n_sec, DMRG_OK);
        std::vector<std::string> msg(n_sec);
        std::atomic<int> next{0};
        auto worker = [&]() {
            for (int t = next++; t < n_sec; t = next++) {
                const int i = todo[t];
                try {
                    solve(i);
                } catch (const Error& e) {
                    st[i] = e.code;
                    msg[i] = e.what();
                } catch (const std::bad_alloc&) {
                    st[i] = DMRG_ERR_NOMEM;
                    msg[i] = "host allocation failed";
                }
            }
        };
        const int n_thr = std::max(1, std::min({n_sec, 16, (int)std::thread::hardware_concurrency()}));
        std::vector<std::thread> pool;
        try {
            for (int k = 1; k < n_thr; ++k) pool.emplace_back(worker);
        } catch (...) {
            // no more threads: the ones started and this thread drain the shared queue
        }
        worker();
        for (auto& th : pool) th.join();
        for (int i = 0; i < n_sec; ++i)
            if (st[i] != DMRG_OK) throw Error(st[i], msg[i]);
        // the M largest eigenvalues over all sectors, ties in (sector, position) order
        struct Cand { double w; int sec, pos; };
        std::vector<Cand> cand;
        cand.reserve((size_t)eoff[n_sec]);
        double tr = 0.0;
        for (int i = 0; i < n_sec; ++i) {
            tr += trace[i];
            kept[i] = 0;
            for (int k = 0; k < dims[i]; ++k) cand.push_back({evals[eoff[i] + k], i, k});
        }
        std::stable_sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
            if (x.w != y.w) return x.w > y.w;
            if (x.sec != y.sec) return x.sec < y.sec;
            return x.pos < y.pos;
        });
        double sum = 0.0;
        const size_t take = std::min(cand.size(), (size_t)M);
        for (size_t k = 0; k < take; ++k) { ++kept[cand[k].sec]; sum += cand[k].w; }
        *discarded = tr - sum;
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}

dmrg::RenormWork dmrg::renorm_work(int32_t n_sec, const int32_t* dims, const int32_t* kept, const int64_t* o_off,
                                   const double* O, int64_t o_len, int32_t n_blk, const int32_t* sec_out,
                                   const int32_t* sec_in, const int64_t* a_off, const double* A, int64_t a_len,
                                   const int64_t* out_off, double* out, int64_t out_len) {
    RenormWork w;
    if (n_sec < 0 || n_blk < 0) throw Error(DMRG_ERR_ARG, "n_sec and n_blk must be >= 0");
    if (n_blk == 0) return w;
    if (!dims || !kept || !o_off || !O || !sec_out || !sec_in || !a_off || !A || !out_off || !out)
        throw Error(DMRG_ERR_ARG, "NULL argument");
    for (int s = 0; s < n_sec; ++s) {
        if (dims[s] < 0 || kept[s] < 0 || kept[s] > dims[s]) throw Error(DMRG_ERR_ARG, "need 0 <= kept <= dims");
        if (o_off[s] < 0 || o_off[s] + (int64_t)dims[s] * kept[s] > o_len)
            throw Error(DMRG_ERR_SHAPE, "renormalization matrix outside O");
    }
    for (int b = 0; b < n_blk; ++b) {
        const int so = sec_out[b], si = sec_in[b];
        if (so < 0 || so >= n_sec || si < 0 || si >= n_sec) throw Error(DMRG_ERR_ARG, "sector index out of range");
        const int64_t rows = dims[so], cols = dims[si], ko = kept[so], ki = kept[si];
        if (a_off[b] < 0 || a_off[b] + rows * cols > a_len) throw Error(DMRG_ERR_SHAPE, "operator block outside A");
        if (out_off[b] < 0 || out_off[b] + ko * ki > out_len) throw Error(DMRG_ERR_SHAPE, "output block outside out");
        if (rows * ki >= INT32_MAX || ko * ki >= INT32_MAX) throw Error(DMRG_ERR_UNSUPPORTED, "sector block too large");
        if (ko == 0 || ki == 0) continue;                  // nothing kept on one side: empty block
        RenormItem it{};
        it.a_off = a_off[b];
        it.t_off = w.t_len;
        it.out_off = out_off[b];
        it.oo_off = o_off[so];
        it.oi_off = o_off[si];
        it.rows = (int32_t)rows;
        it.cols = (int32_t)cols;
        it.k_out = (int32_t)ko;
        it.k_in = (int32_t)ki;
        w.items.push_back(it);
        w.t_len += rows * ki;
        w.max_t = std::max(w.max_t, rows * ki);
        w.max_out = std::max(w.max_out, ko * ki);
    }
    if (w.items.size() > (size_t)INT32_MAX) throw Error(DMRG_ERR_UNSUPPORTED, "too many blocks");
    return w;
}

extern "C" dmrg_status dmrg_renormalize_blocks(int32_t device, int32_t n_sec, const int32_t* dims, const int32_t* kept,
                                               const int64_t* o_off, const double* O, int64_t o_len, int32_t n_blk,
                                               const int32_t* sec_out, const int32_t* sec_in, const int64_t* a_off,
                                               const double* A, int64_t a_len, const int64_t* out_off, double* out,
                                               int64_t out_len, void* stream) {
    dmrg::clear_error();
    try {
        const dmrg::RenormWork wk = dmrg::renorm_work(n_sec, dims, kept, o_off, O, o_len, n_blk, sec_out, sec_in,
                                                      a_off, A, a_len, out_off, out, out_len);
        const auto& items = wk.items;
        if (items.empty()) return DMRG_OK;
        HIPCHK(hipSetDevice(device));
        hipStream_t s = (hipStream_t)stream;
        void *d_items = nullptr, *d_t = nullptr;
        try {
            HIPCHK(hipMalloc(&d_items, items.size() * sizeof(dmrg::RenormItem)));
            HIPCHK(hipMalloc(&d_t, (size_t)std::max<int64_t>(1, wk.t_len) * sizeof(double)));
            HIPCHK(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(dmrg::RenormItem), hipMemcpyHostToDevice, s));
            HIPCHK(dmrg::launch_renormalize(static_cast<const dmrg::RenormItem*>(d_items), (int)items.size(), wk.max_t,
                                            wk.max_out, A, O, static_cast<double*>(d_t), out, s));
            HIPCHK(hipStreamSynchronize(s));   // the work list and T end here
        } catch (...) {
            (void)hipStreamSynchronize(s);
            if (d_items) (void)hipFree(d_items);
            if (d_t) (void)hipFree(d_t);
            throw;
        }
        (void)hipFree(d_items);
        (void)hipFree(d_t);
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}


// ---------------------------------------------------------------- growth and renormalization
namespace {

void check_side(int32_t side) {
    if (side != 0 && side != 1) throw Error(DMRG_ERR_ARG, "side must be 0 (left block) or 1 (right block)");
}

}  // namespace

extern "C" dmrg_status dmrg_block_grow_layout(const dmrg_block* block, int32_t side, int32_t* n_sec, int32_t* qn,
                                              int32_t* dims) {
    dmrg::clear_error();
    try {
        if (!n_sec) throw Error(DMRG_ERR_ARG, "NULL argument");
        check_side(side);
        const BlockIn B = dmrg::import_block(block, side == 0 ? "left" : "right");
        const EnlargedLayout E = dmrg::enlarged_layout(B, side == 1);
        *n_sec = (int32_t)E.dim.size();
        for (size_t i = 0; i < E.dim.size(); ++i) {
            if (qn) { qn[2 * i] = E.qn[i].first; qn[2 * i + 1] = E.qn[i].second; }
            if (dims) dims[i] = E.dim[i];
        }
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}

extern "C" dmrg_status dmrg_block_grow(const dmrg_problem* p, const dmrg_block* block, int32_t side,
                                       const int32_t* kept, const double* O, const dmrg_build_opts* opts,
                                       dmrg_block** out) {
    dmrg::clear_error();
    if (!out) { dmrg::last_error() = "out is NULL"; return DMRG_ERR_ARG; }
    *out = nullptr;
    try {
        if (!p || !p->h || !p->eri) throw Error(DMRG_ERR_ARG, "problem or its integrals are NULL");
        if (p->n_orb < 2 || p->site < 0 || p->site > p->n_orb - 2)
            throw Error(DMRG_ERR_ARG, "need n_orb >= 2 and 0 <= site <= n_orb - 2");
        check_side(side);
        if ((kept == nullptr) != (O == nullptr)) throw Error(DMRG_ERR_ARG, "kept and O must both be given or both NULL");
        const int dev = opts ? opts->device : 0;
        if (dev < 0) throw Error(DMRG_ERR_UNSUPPORTED, "block growth runs on a device");
        hipStream_t s = (hipStream_t)(opts ? opts->stream : nullptr);
        const int64_t L = p->n_orb;
        std::vector<double> h(p->h, p->h + L * L), eri(p->eri, p->eri + L * L * L * L);
        for (double v : h) if (!std::isfinite(v)) throw Error(DMRG_ERR_NAN, "non-finite one-electron integral");
        for (double v : eri) if (!std::isfinite(v)) throw Error(DMRG_ERR_NAN, "non-finite two-electron integral");
        const BlockIn B = dmrg::import_block(block, side == 0 ? "left" : "right");
        const EnlargedLayout E = dmrg::enlarged_layout(B, side == 1);
        std::vector<int> k(E.dim.size());
        std::vector<double> Ov;
        if (kept) {
            int64_t len = 0;
            for (size_t q = 0; q < E.dim.size(); ++q) {
                k[q] = kept[q];
                if (k[q] < 0 || k[q] > E.dim[q]) throw Error(DMRG_ERR_ARG, "need 0 <= kept <= enlarged sector dimension");
                len += (int64_t)E.dim[q] * k[q];
            }
            Ov.assign(O, O + len);
            for (double v : Ov) if (!std::isfinite(v)) throw Error(DMRG_ERR_NAN, "non-finite renormalization matrix");
        } else {
            for (size_t q = 0; q < E.dim.size(); ++q) {        // keep everything: O = identity
                k[q] = E.dim[q];
                const size_t o = Ov.size();
                Ov.resize(o + (size_t)E.dim[q] * E.dim[q], 0.0);
                for (int i = 0; i < E.dim[q]; ++i) Ov[o + (size_t)i * E.dim[q] + i] = 1.0;
            }
        }
        HIPCHK(hipSetDevice(dev));
        // the block's data as given (compact sector blocks at the caller's offsets)
        std::vector<int64_t> off((size_t)B.ops.size() * B.n_sec, -1);
        for (size_t o = 0; o < B.ops.size(); ++o)
            for (int si = 0; si < B.n_sec; ++si) off[o * B.n_sec + si] = B.ops[o].off_of_in[si];
        void* d_data = nullptr;
        if (hipMalloc(&d_data, (size_t)std::max<int64_t>(1, B.n_data) * sizeof(double)) != hipSuccess)
            throw Error(DMRG_ERR_NOMEM, "device allocation failed (block data)");
        try {
            if (B.n_data > 0)
                HIPCHK(hipMemcpyAsync(d_data, B.data, (size_t)B.n_data * sizeof(double), hipMemcpyHostToDevice, s));
            dmrg::Integrals I{(int)L, h.data(), eri.data()};
            const int site = side == 0 ? p->site : p->site + 1;
            *out = dmrg::grow_block(B, side == 1, site, I, static_cast<const double*>(d_data), B.n_data, off, false, k, Ov,
                                    dev, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(d_data);
            throw;
        }
        (void)hipFree(d_data);
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}

extern "C" dmrg_status dmrg_renormalize(dmrg_hop* H, const double* psi, int32_t dir, int32_t m_max, dmrg_block** out,
                                        double* discarded, void* stream) {
    dmrg::clear_error();
    if (!out) { dmrg::last_error() = "out is NULL"; return DMRG_ERR_ARG; }
    *out = nullptr;
    try {
        if (!H || !psi) throw Error(DMRG_ERR_ARG, "NULL argument");
        check_side(dir);
        if (m_max < 1) throw Error(DMRG_ERR_ARG, "m_max must be >= 1");
        if (H->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle has no device state");
        if (H->n_parts != 1) throw Error(DMRG_ERR_UNSUPPORTED, "merged handle: renormalization is per problem");
        const bool right = dir == 1;
        const RdmLayout R = rdm_layout(*H, right);
        hipStream_t s = (hipStream_t)stream;
        HIPCHK(hipSetDevice(H->device));
        // 1. rho of the enlarged block (device), then the M-state cut (host)
        std::vector<double> rho((size_t)R.off.back());
        {
            void* d_rho = nullptr;
            if (hipMalloc(&d_rho, std::max<size_t>(1, rho.size()) * sizeof(double)) != hipSuccess)
                throw Error(DMRG_ERR_NOMEM, "device allocation failed (density matrix)");
            dmrg_status st = rdm_entry(H, right, psi, static_cast<double*>(d_rho), R.off.back(), stream);
            if (st == DMRG_OK && !rho.empty() &&
                hipMemcpy(rho.data(), d_rho, rho.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
                st = dmrg::record_error(Error(DMRG_ERR_DEVICE, "density matrix copy failed"));
            (void)hipFree(d_rho);
            if (st != DMRG_OK) return st;
        }
        const int nq = (int)R.dim.size();
        std::vector<int32_t> dims(R.dim.begin(), R.dim.end()), kept(nq);
        std::vector<double> evals;
        for (int d : R.dim) evals.resize(evals.size() + d);
        std::vector<double> vecs(rho.size());
        double disc = 0.0;
        dmrg_status st = dmrg_truncate(rho.data(), nq, dims.data(), R.off.data(), m_max, kept.data(), evals.data(),
                                       vecs.data(), &disc);
        if (st != DMRG_OK) return st;
        // 2. O: the kept leading columns of each sector's eigenvectors, packed dims x kept
        std::vector<int> k(kept.begin(), kept.end());
        std::vector<double> Ov;
        for (int q = 0; q < nq; ++q) {
            const int d = R.dim[q];
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < kept[q]; ++c) Ov.push_back(vecs[(size_t)R.off[q] + (size_t)r * d + c]);
        }
        // 3. the grown block's operators from the handle's device copy of the old block, Eq. renorm_mat
        const BlockIn& B = right ? H->right : H->left;
        dmrg::Integrals I{H->L, H->h.data(), H->eri.data()};
        const int site = right ? H->site + 1 : H->site;
        if (H->trimmed) throw Error(DMRG_ERR_UNSUPPORTED, "handle was trimmed (dmrg_hop_trim)");
        *out = dmrg::grow_block(B, right, site, I, H->d_pool, H->pool_size, H->op_pool_off[right ? 1 : 0], true, k, Ov,
                                H->device, s);
        if (discarded) *discarded = disc;
        return DMRG_OK;
    } catch (const Error& e) {
        return dmrg::record_error(e);
    } catch (const std::bad_alloc&) {
        dmrg::last_error() = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}
