// Host driver of libdmrg: block import, psi sector layout (Eq. wf_sec), the operator-combination
// list of the two-site H.psi (Section 2.2.1), pre-summation plans (Section 2.2.3), the
// owner-computes task list for Eq. dgemm, device residency and the C-ABI entry points (the launch
// plans built from the task list are in plan.cpp).
//
// Term generator. With L = left block (normal operators), S = the two sites s1 s2 and R = right
// block (complementary operators), H is split by two nested cut identities:
//   cut 1, L | (S R):  H = H_L + H_SR + sum_{W in SR} [S^L_W c_W + h.c.] + sum_{P in L} [c+_P U^SR_P
//                      + h.c.] + sum_{P<Q in L} [A_PQ P^SR_PQ + h.c.] + sum_{X,Y in L} B_XY Q^SR_XY
//   cut 2, S | R:      H_SR = H_S + H_R + the same five cross families with S as the normal side,
// and every complementary operator of (S R) is split into its S-only, R-only and mixed parts
// (e.g. P^SR_PQ = P^R_PQ + sum_{zw in S} w_PQzw c_z c_w + sum_{y in S, Z in R} (w_PQyZ - w_PQZy)
// c_y c_Z). Mixed sums over block indices are folded into pre-summed left-block operators
// (integrals contracted inside one block: Section 2.1 footnote, Section 2.2.3), so every
// combination alpha is (left matrix) x (16x16 two-site matrix) x (right matrix), Section 2.2.1.
// The matrix of an operator product O_L O_S O_R on |l>|s1 s2>|r> is
// (O_L P_L^{p(O_L)}) x (O_S P_S^{p(O_R)}) x O_R with P the ket parity; the Hermitian conjugate of a
// combination is the transpose of each of its three matrices.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dmrg.h"
#include "host_common.h"
#include "internal.h"
#include "hop.h"
#include "mlp.h"
#include "plan.h"

namespace {

thread_local std::string g_err;

using dmrg::Error;

using dmrg::M16;
using dmrg::kSiteQn;
using dmrg::OpIn;
using dmrg::BlockIn;
using dmrg::Term;
using dmrg::MatDef;
using dmrg::Alpha;
using dmrg::kind_name;
using dmrg::import_block;
using dmrg::build_plan;
using dmrg::dev_alloc;
using dmrg::drop_graphs;
using dmrg::make_tiled_split;
using dmrg::needs_fallback;

M16 zero16() { M16 m; m.fill(0.0); return m; }
M16 eye16() { M16 m = zero16(); for (int i = 0; i < 16; ++i) m[i * 17] = 1.0; return m; }
M16 mul(const M16& a, const M16& b) {
    M16 c = zero16();
    for (int i = 0; i < 16; ++i)
        for (int k = 0; k < 16; ++k) {
            double v = a[i * 16 + k];
            if (v == 0.0) continue;
            for (int j = 0; j < 16; ++j) c[i * 16 + j] += v * b[k * 16 + j];
        }
    return c;
}
M16 tr16(const M16& a) { M16 c; for (int i = 0; i < 16; ++i) for (int j = 0; j < 16; ++j) c[j * 16 + i] = a[i * 16 + j]; return c; }
void axpy16(M16& y, double a, const M16& x) { for (int i = 0; i < 256; ++i) y[i] += a * x[i]; }
bool nonzero16(const M16& a) { for (double v : a) if (v != 0.0) return true; return false; }

// Two-site Jordan-Wigner fermion matrices. Site mode y: 0 = s1 alpha, 1 = s1 beta, 2 = s2 alpha,
// 3 = s2 beta. Site basis (0, up, dn, updn), |updn> = c+_up c+_dn |0>:
//   c+_up = E10 + E32, c+_dn = E20 - E31; on s2 the s1 parity diag(1,-1,-1,1) is applied.
M16 site_cd(int y) {
    double a[16] = {0};
    if (y % 2 == 0) { a[1 * 4 + 0] = 1; a[3 * 4 + 2] = 1; }
    else            { a[2 * 4 + 0] = 1; a[3 * 4 + 1] = -1; }
    const double par[4] = {1, -1, -1, 1};
    M16 m = zero16();
    for (int bp = 0; bp < 4; ++bp)
        for (int b = 0; b < 4; ++b)
            for (int cp = 0; cp < 4; ++cp)
                for (int c = 0; c < 4; ++c) {
                    double v;
                    if (y < 2) v = a[bp * 4 + b] * (cp == c ? 1.0 : 0.0);
                    else v = (bp == b ? par[b] : 0.0) * a[cp * 4 + c];
                    m[(bp * 4 + cp) * 16 + (b * 4 + c)] = v;
                }
    return m;
}
M16 site_c(int y) { return tr16(site_cd(y)); }
M16 site_parity() {
    const double par[4] = {1, -1, -1, 1};
    M16 m = zero16();
    for (int b = 0; b < 4; ++b) for (int c = 0; c < 4; ++c) m[(b * 4 + c) * 17] = par[b] * par[c];
    return m;
}


}  // namespace

namespace dmrg {

const char* kind_name(int k) {
    static const char* n[] = {"H", "C", "A", "B", "S", "U", "P", "Q"};
    return (k >= 0 && k < 8) ? n[k] : "?";
}

BlockIn import_block(const dmrg_block* b, const char* side) {
    if (!b) throw Error(DMRG_ERR_ARG, std::string(side) + " block is NULL");
    BlockIn B;
    if (b->n_sec <= 0 || !b->qn || !b->dim) throw Error(DMRG_ERR_ARG, std::string(side) + " block has no sectors");
    B.n_sec = b->n_sec;
    std::map<std::pair<int, int>, int> seen;
    for (int i = 0; i < b->n_sec; ++i) {
        B.qa.push_back(b->qn[2 * i]);
        B.qb.push_back(b->qn[2 * i + 1]);
        B.dim.push_back(b->dim[i]);
        if (b->dim[i] < 0) throw Error(DMRG_ERR_SHAPE, std::string(side) + " block: negative sector dimension");
        if (!seen.emplace(std::make_pair(b->qn[2 * i], b->qn[2 * i + 1]), i).second)
            throw Error(DMRG_ERR_ARG, std::string(side) + " block: duplicate sector quantum numbers");
    }
    B.data = b->data;
    B.n_data = b->n_data;
    if (b->n_ops < 0 || (b->n_ops > 0 && !b->ops)) throw Error(DMRG_ERR_ARG, std::string(side) + " block: bad op list");
    for (int k = 0; k < b->n_ops; ++k) {
        const dmrg_op& o = b->ops[k];
        OpIn op;
        op.kind = o.kind; op.i0 = o.i0; op.i1 = o.i1;
        if (o.kind < 0 || o.kind > 7) throw Error(DMRG_ERR_ARG, "unknown operator kind");
        op.out_of_in.assign(B.n_sec, -1);
        op.off_of_in.assign(B.n_sec, -1);
        for (int j = 0; j < o.n_blk; ++j) {
            int so = o.sec_out[j], si = o.sec_in[j];
            int64_t off = o.off[j];
            if (so < 0 || so >= B.n_sec || si < 0 || si >= B.n_sec)
                throw Error(DMRG_ERR_SHAPE, std::string(side) + " block: sector index out of range");
            if (op.out_of_in[si] >= 0)
                throw Error(DMRG_ERR_SHAPE, std::string(side) + " block: two blocks with the same ket sector");
            int64_t sz = (int64_t)B.dim[so] * B.dim[si];
            if (off < 0 || off + sz > B.n_data)
                throw Error(DMRG_ERR_SHAPE, std::string(side) + " block: data offset out of range");
            op.out_of_in[si] = so;
            op.off_of_in[si] = off;
        }
        if (!B.index.emplace(std::array<int, 3>{o.kind, o.i0, o.i1}, k).second)
            throw Error(DMRG_ERR_ARG, std::string(side) + " block: duplicate operator");
        B.ops.push_back(std::move(op));
    }
    if (B.n_data > 0 && !B.data) throw Error(DMRG_ERR_ARG, std::string(side) + " block: data is NULL");
    for (int64_t i = 0; i < B.n_data; ++i)
        if (!std::isfinite(B.data[i])) throw Error(DMRG_ERR_NAN, std::string(side) + " block: non-finite operator entry");
    return B;
}

}  // namespace dmrg

namespace {

using dmrg::Integrals;

struct Builder {
    dmrg_hop& H;
    Integrals I;
    Builder(dmrg_hop& h) : H(h) { I.L = h.L; I.h = h.h.data(); I.eri = h.eri.data(); }

    BlockIn& side(int s) { return s == 0 ? H.left : H.right; }

    // stored operator (with B/Q transposition fallback); throws if absent
    std::pair<int, bool> op(int s, int kind, int i0, int i1 = -1) {
        BlockIn& B = side(s);
        int k = B.find(kind, i0, i1);
        if (k >= 0) return {k, false};
        if (kind == DMRG_OP_B || kind == DMRG_OP_Q) {
            k = B.find(kind, i1, i0);
            if (k >= 0) return {k, true};
        }
        if (H.share) return {-1, false};   // share mode: the combinations using it are left out
        char buf[160];
        std::snprintf(buf, sizeof buf, "%s block lacks operator %s(%d,%d)", s == 0 ? "left" : "right",
                      kind_name(kind), i0, i1);
        throw Error(DMRG_ERR_ARG, buf);
    }

    int mat(int s, std::pair<int, bool> o) {
        if (o.first < 0) return -2;            // absent operator (share mode)
        auto key = std::make_tuple(s, o.first, o.second);
        auto it = H.mat_cache.find(key);
        if (it != H.mat_cache.end()) return it->second;
        MatDef m;
        m.side = s;
        m.terms.push_back({1.0, o.first, o.second});
        H.mats.push_back(m);
        int id = (int)H.mats.size() - 1;
        H.mat_cache[key] = id;
        return id;
    }
    int presum(int s, const std::vector<Term>& terms) {
        // share mode: a summand whose operator the blocks do not supply (op < 0) belongs to another
        // device's share and is left out; the combination keeps its supplied summands
        std::vector<Term> nz;
        for (const Term& t : terms) if (t.c != 0.0 && t.op >= 0) nz.push_back(t);
        if (nz.empty()) return -2;   // identically zero, or no summand supplied
        if (nz.size() == 1 && nz[0].c == 1.0) return mat(s, {nz[0].op, nz[0].tr});
        MatDef m;
        m.side = s;
        m.terms = nz;
        H.mats.push_back(m);
        return (int)H.mats.size() - 1;
    }
    int transpose(int id) {
        if (id < 0) return id;
        if (H.mats[id].transpose_id >= 0) return H.mats[id].transpose_id;
        int tid;
        if (H.mats[id].terms.size() == 1 && H.mats[id].terms[0].c == 1.0) {
            tid = mat(H.mats[id].side, {H.mats[id].terms[0].op, !H.mats[id].terms[0].tr});
        } else {
            MatDef m;
            m.side = H.mats[id].side;
            for (const Term& t : H.mats[id].terms) m.terms.push_back({t.c, t.op, !t.tr});
            H.mats.push_back(m);
            tid = (int)H.mats.size() - 1;
        }
        H.mats[id].transpose_id = tid;
        H.mats[tid].transpose_id = id;
        return tid;
    }

    void emit(int family, int lm, bool lodd, const M16& S, int rm, bool hc) {
        if (lm == -2 || rm == -2 || !nonzero16(S)) return;
        H.alphas.push_back({1.0, lm, lodd ? 1 : 0, S, rm, family});
        if (hc) H.alphas.push_back({1.0, transpose(lm), lodd ? 2 : 0, tr16(S), transpose(rm), -family});
    }

    void generate() {
        const int site = H.site, L = H.L;
        const int nL = 2 * site;                 // left spin-orbitals 0 .. nL-1
        const int G0 = 2 * site;                 // site mode y -> spin-orbital G0 + y
        const int R0 = 2 * (site + 2), R1 = 2 * L;
        M16 cd[4], c[4];
        for (int y = 0; y < 4; ++y) { cd[y] = site_cd(y); c[y] = site_c(y); }
        const M16 PS = site_parity(), I16 = eye16();
        auto G = [&](int y) { return G0 + y; };
        enum { LEFT = 0, RIGHT = 1 };

        // F1, F3: block Hamiltonians
        emit(1, mat(LEFT, op(LEFT, DMRG_OP_H, -1, -1)), false, I16, -1, false);
        emit(3, -1, false, I16, mat(RIGHT, op(RIGHT, DMRG_OP_H, -1, -1)), false);
        // F2: two-site Hamiltonian
        {
            M16 HS = zero16();
            for (int y = 0; y < 4; ++y)
                for (int z = 0; z < 4; ++z) {
                    double v = I.t(G(y), G(z));
                    if (v != 0.0) axpy16(HS, v, mul(cd[y], c[z]));
                }
            for (int p = 0; p < 4; ++p) for (int q = 0; q < 4; ++q)
                for (int r = 0; r < 4; ++r) for (int s = 0; s < 4; ++s) {
                    double v = I.w(G(p), G(q), G(r), G(s));
                    if (v != 0.0) axpy16(HS, 0.5 * v, mul(mul(cd[p], cd[q]), mul(c[r], c[s])));
                }
            emit(2, -1, false, HS, -1, false);
        }
        // F4: S^L_W c_W, W in the sites (S^L_W completed with its one-body part)
        for (int y = 0; y < 4; ++y) {
            int W = G(y);
            std::vector<Term> t;
            auto s = op(LEFT, DMRG_OP_S, W);
            t.push_back({1.0, s.first, s.second});
            for (int P = 0; P < nL; ++P) { auto o = op(LEFT, DMRG_OP_C, P); t.push_back({I.t(P, W), o.first, o.second}); }
            emit(4, presum(LEFT, t), true, c[y], -1, true);
        }
        // F5: S^L_W c_W, W in the right block
        for (int W = R0; W < R1; ++W) {
            std::vector<Term> t;
            auto s = op(LEFT, DMRG_OP_S, W);
            t.push_back({1.0, s.first, s.second});
            for (int P = 0; P < nL; ++P) { auto o = op(LEFT, DMRG_OP_C, P); t.push_back({I.t(P, W), o.first, o.second}); }
            auto cw = op(RIGHT, DMRG_OP_C, W);
            emit(5, presum(LEFT, t), true, PS, mat(RIGHT, {cw.first, !cw.second}), true);
        }
        for (int P = 0; P < nL; ++P) {
            int cP = mat(LEFT, op(LEFT, DMRG_OP_C, P));
            // F6: c+_P U^R_P
            emit(6, cP, true, PS, mat(RIGHT, op(RIGHT, DMRG_OP_U, P)), true);
            // F7: c+_P U^S_P
            M16 US = zero16();
            for (int q = 0; q < 4; ++q) for (int z = 0; z < 4; ++z) for (int x = 0; x < 4; ++x) {
                double v = I.w(P, G(q), G(z), G(x));
                if (v != 0.0) axpy16(US, v, mul(mul(cd[q], c[z]), c[x]));
            }
            emit(7, cP, true, US, -1, true);
            // F8: c+_P c+_q P^R_Pq ; F9: c+_P c_y Q^R_Py
            for (int q = 0; q < 4; ++q) emit(8, cP, true, cd[q], mat(RIGHT, op(RIGHT, DMRG_OP_P, P, G(q))), true);
            for (int y = 0; y < 4; ++y) emit(9, cP, true, c[y], mat(RIGHT, op(RIGHT, DMRG_OP_Q, P, G(y))), true);
        }
        // F10: [sum_P (w_PqyZ - w_PqZy) c+_P] c+_q c_y c_Z, Z in R
        for (int Z = R0; Z < R1; ++Z) {
            auto cz = op(RIGHT, DMRG_OP_C, Z);
            int cZ = mat(RIGHT, {cz.first, !cz.second});
            for (int q = 0; q < 4; ++q) for (int y = 0; y < 4; ++y) {
                std::vector<Term> t;
                for (int P = 0; P < nL; ++P) {
                    auto o = op(LEFT, DMRG_OP_C, P);
                    t.push_back({I.w(P, G(q), G(y), Z) - I.w(P, G(q), Z, G(y)), o.first, o.second});
                }
                emit(10, presum(LEFT, t), true, mul(mul(cd[q], c[y]), PS), cZ, true);
            }
        }
        // F11: [sum_P (w_PQzw - w_PQwz) c+_P] c_z c_w c+_Q, Q in R, z < w
        for (int Q = R0; Q < R1; ++Q) {
            int cQ = mat(RIGHT, op(RIGHT, DMRG_OP_C, Q));
            for (int z = 0; z < 4; ++z) for (int x = z + 1; x < 4; ++x) {
                std::vector<Term> t;
                for (int P = 0; P < nL; ++P) {
                    auto o = op(LEFT, DMRG_OP_C, P);
                    t.push_back({I.w(P, Q, G(z), G(x)) - I.w(P, Q, G(x), G(z)), o.first, o.second});
                }
                emit(11, presum(LEFT, t), true, mul(mul(c[z], c[x]), PS), cQ, true);
            }
        }
        // F12: A_PQ P^R_PQ
        for (int P = 0; P < nL; ++P)
            for (int Q = P + 1; Q < nL; ++Q)
                emit(12, mat(LEFT, op(LEFT, DMRG_OP_A, P, Q)), false, I16, mat(RIGHT, op(RIGHT, DMRG_OP_P, P, Q)), true);
        // F13: [sum_{P<Q} (w_PQzw - w_PQwz) A_PQ] c_z c_w
        for (int z = 0; z < 4; ++z) for (int x = z + 1; x < 4; ++x) {
            std::vector<Term> t;
            for (int P = 0; P < nL; ++P) for (int Q = P + 1; Q < nL; ++Q) {
                auto o = op(LEFT, DMRG_OP_A, P, Q);
                t.push_back({I.w(P, Q, G(z), G(x)) - I.w(P, Q, G(x), G(z)), o.first, o.second});
            }
            emit(13, presum(LEFT, t), false, mul(c[z], c[x]), -1, true);
        }
        // F14: [sum_{P<Q} (w_PQyZ - w_PQZy) A_PQ] c_y c_Z
        for (int y = 0; y < 4; ++y) for (int Z = R0; Z < R1; ++Z) {
            std::vector<Term> t;
            for (int P = 0; P < nL; ++P) for (int Q = P + 1; Q < nL; ++Q) {
                auto o = op(LEFT, DMRG_OP_A, P, Q);
                t.push_back({I.w(P, Q, G(y), Z) - I.w(P, Q, Z, G(y)), o.first, o.second});
            }
            auto cz = op(RIGHT, DMRG_OP_C, Z);
            emit(14, presum(LEFT, t), false, mul(c[y], PS), mat(RIGHT, {cz.first, !cz.second}), true);
        }
        // F15: B_XY Q^R_XY
        for (int X = 0; X < nL; ++X)
            for (int Y = 0; Y < nL; ++Y)
                emit(15, mat(LEFT, op(LEFT, DMRG_OP_B, X, Y)), false, I16, mat(RIGHT, op(RIGHT, DMRG_OP_Q, X, Y)), false);
        // F16, F17, F18: the site and mixed parts of Q^SR_XY
        auto bsum = [&](auto coef) {
            std::vector<Term> t;
            for (int X = 0; X < nL; ++X) for (int Y = 0; Y < nL; ++Y) {
                auto o = op(LEFT, DMRG_OP_B, X, Y);
                t.push_back({coef(X, Y), o.first, o.second});
            }
            return presum(LEFT, t);
        };
        for (int z = 0; z < 4; ++z) for (int x = 0; x < 4; ++x) {
            int lm = bsum([&](int X, int Y) { return I.w(X, G(z), G(x), Y) - I.w(X, G(z), Y, G(x)); });
            emit(16, lm, false, mul(cd[z], c[x]), -1, false);
        }
        for (int z = 0; z < 4; ++z) for (int W = R0; W < R1; ++W) {
            int lm = bsum([&](int X, int Y) { return I.w(X, G(z), W, Y) - I.w(X, G(z), Y, W); });
            auto cw = op(RIGHT, DMRG_OP_C, W);
            emit(17, lm, false, mul(cd[z], PS), mat(RIGHT, {cw.first, !cw.second}), false);
        }
        for (int x = 0; x < 4; ++x) for (int Z = R0; Z < R1; ++Z) {
            int lm = bsum([&](int X, int Y) { return -(I.w(X, Z, G(x), Y) - I.w(X, Z, Y, G(x))); });
            emit(18, lm, false, mul(c[x], PS), mat(RIGHT, op(RIGHT, DMRG_OP_C, Z)), false);
        }
        // F19: S^S_W c_W, W in R
        for (int W = R0; W < R1; ++W) {
            M16 SS = zero16();
            for (int p = 0; p < 4; ++p) {
                double v = I.t(G(p), W);
                if (v != 0.0) axpy16(SS, v, cd[p]);
            }
            for (int p = 0; p < 4; ++p) for (int q = 0; q < 4; ++q) for (int r = 0; r < 4; ++r) {
                double v = I.w(G(p), G(q), G(r), W);
                if (v != 0.0) axpy16(SS, v, mul(mul(cd[p], cd[q]), c[r]));
            }
            auto cw = op(RIGHT, DMRG_OP_C, W);
            emit(19, -1, false, mul(SS, PS), mat(RIGHT, {cw.first, !cw.second}), true);
        }
        // F20 .. F22: site operators times right complementary operators with site indices
        for (int p = 0; p < 4; ++p) emit(20, -1, false, mul(cd[p], PS), mat(RIGHT, op(RIGHT, DMRG_OP_U, G(p))), true);
        for (int p = 0; p < 4; ++p) for (int q = p + 1; q < 4; ++q)
            emit(21, -1, false, mul(cd[p], cd[q]), mat(RIGHT, op(RIGHT, DMRG_OP_P, G(p), G(q))), true);
        for (int x = 0; x < 4; ++x) for (int y = 0; y < 4; ++y)
            emit(22, -1, false, mul(cd[x], c[y]), mat(RIGHT, op(RIGHT, DMRG_OP_Q, G(x), G(y))), false);
    }
};

void build_layout(dmrg_hop& H) {
    const BlockIn &Lb = H.left, &Rb = H.right;
    std::map<std::pair<int, int>, int> ridx;
    for (int d = 0; d < Rb.n_sec; ++d) ridx[{Rb.qa[d], Rb.qb[d]}] = d;
    H.blk_index.assign((size_t)Lb.n_sec * 16, -1);
    int64_t off = 0;
    for (int a = 0; a < Lb.n_sec; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                int qa = H.na - Lb.qa[a] - kSiteQn[b][0] - kSiteQn[c][0];
                int qb = H.nb - Lb.qb[a] - kSiteQn[b][1] - kSiteQn[c][1];
                auto it = ridx.find({qa, qb});
                if (it == ridx.end()) continue;
                int d = it->second;
                int ma = Lb.dim[a], md = Rb.dim[d];
                if (ma == 0 || md == 0) continue;
                H.blk_index[(a * 4 + b) * 4 + c] = (int)H.blk.size();
                H.blk.push_back({a, b, c, d});
                H.blk_ma.push_back(ma);
                H.blk_md.push_back(md);
                H.blk_off.push_back(off);
                off += (int64_t)ma * md;
            }
    H.n_coeff = off;
    if (H.blk.empty()) throw Error(DMRG_ERR_SHAPE, "no psi sector satisfies the electron-number constraints");
}

// Sector map of a matrix definition (all terms must change the quantum numbers alike).
void mat_sectors(dmrg_hop& H, MatDef& m) {
    BlockIn& B = m.side == 0 ? H.left : H.right;
    m.out_of_in.assign(B.n_sec, -1);
    for (const Term& t : m.terms) {
        const OpIn& o = B.ops[t.op];
        for (int s = 0; s < B.n_sec; ++s) {
            int si, so;
            if (!t.tr) { si = s; so = o.out_of_in[s]; }
            else { so = s; si = o.out_of_in[s]; }
            if (so < 0 || si < 0) continue;
            if (m.out_of_in[si] >= 0 && m.out_of_in[si] != so)
                throw Error(DMRG_ERR_ARG, "pre-sum mixes operators with different sector changes");
            m.out_of_in[si] = so;
        }
    }
    m.bytes = 0.0;
    for (int si = 0; si < B.n_sec; ++si)
        if (m.out_of_in[si] >= 0) m.bytes += 8.0 * dmrg::rows_of(B.dim[m.out_of_in[si]]) * dmrg::ld_of(B.dim[si]);
}

void build_tasks(dmrg_hop& H) {
    for (MatDef& m : H.mats) mat_sectors(H, m);
    struct Key { int i, j, lm, rm; bool operator==(const Key& o) const { return i == o.i && j == o.j && lm == o.lm && rm == o.rm; } };
    struct KH { size_t operator()(const Key& k) const {
        uint64_t a = ((uint64_t)(uint32_t)k.i << 32) | (uint32_t)k.j;
        uint64_t b = ((uint64_t)(uint32_t)k.lm << 32) | (uint32_t)k.rm;
        return std::hash<uint64_t>()(a * 0x9E3779B97F4A7C15ULL ^ b); } };
    std::unordered_map<Key, double, KH> acc;
    acc.reserve(1 << 20);
    const BlockIn &Lb = H.left, &Rb = H.right;
    for (const Alpha& al : H.alphas) {
        const MatDef* lm = al.lmat >= 0 ? &H.mats[al.lmat] : nullptr;
        const MatDef* rm = al.rmat >= 0 ? &H.mats[al.rmat] : nullptr;
        for (size_t i = 0; i < H.blk.size(); ++i) {
            int a = H.blk[i][0], b = H.blk[i][1], c = H.blk[i][2], d = H.blk[i][3];
            int ap = lm ? lm->out_of_in[a] : a;
            if (ap < 0) continue;
            int dp = rm ? rm->out_of_in[d] : d;
            if (dp < 0) continue;
            double par = 1.0;
            if (al.lpar == 1) par = ((Lb.qa[a] + Lb.qb[a]) & 1) ? -1.0 : 1.0;
            if (al.lpar == 2) par = ((Lb.qa[ap] + Lb.qb[ap]) & 1) ? -1.0 : 1.0;
            int col = b * 4 + c;
            for (int row = 0; row < 16; ++row) {
                double s = al.S[row * 16 + col];
                if (s == 0.0) continue;
                int bp = row / 4, cp = row % 4;
                int j = H.blk_index[(ap * 4 + bp) * 4 + cp];
                if (j < 0 || H.blk[j][3] != dp)
                    throw Error(DMRG_ERR_ARG, "operator combination leaves the electron-number sector "
                                              "(inconsistent block quantum numbers)");
                acc[{(int)i, j, al.lmat, al.rmat}] += al.coeff * s * par;
            }
        }
    }
    H.tasks.clear();
    H.tasks.reserve(acc.size());
    for (auto& kv : acc)
        if (kv.second != 0.0) H.tasks.push_back({kv.first.i, kv.first.j, kv.first.lm, kv.first.rm, kv.second});
    std::sort(H.tasks.begin(), H.tasks.end(), [](const dmrg_hop::HTask& x, const dmrg_hop::HTask& y) {
        if (x.j != y.j) return x.j < y.j;
        if (x.i != y.i) return x.i < y.i;
        if (x.lm != y.lm) return x.lm < y.lm;
        return x.rm < y.rm;
    });
    (void)Rb;
    // algorithmic flops / bytes
    double fl = 0.0;
    for (const auto& t : H.tasks) {
        double ma = H.blk_ma[t.i], md = H.blk_md[t.i], mj = H.blk_ma[t.j], nj = H.blk_md[t.j];
        if (t.lm < 0 && t.rm < 0) continue;
        if (t.lm < 0) fl += 2.0 * ma * md * nj;
        else if (t.rm < 0) fl += 2.0 * mj * ma * md;
        else fl += 2.0 * std::min(mj * ma * md + mj * md * nj, ma * md * nj + mj * ma * nj);
    }
    H.flops = fl;
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void upload(dmrg_hop& H, const dmrg_build_opts* opts) {
    hipStream_t s = (hipStream_t)(opts ? opts->stream : nullptr);
    HIPCHK(hipSetDevice(H.device));
    // DMRG_BUILD_TRACE=1: synchronize after each phase and print its wall time
    const char* bt = std::getenv("DMRG_BUILD_TRACE");
    const bool btrace = bt && bt[0] == '1';
    double bt0 = now();
    auto phase = [&](const char* name) {
        if (!btrace) return;
        HIPCHK(hipStreamSynchronize(s));
        const double t = now();
        std::fprintf(stderr, "[dmrg build] %-28s %8.3f s\n", name, t - bt0);
        bt0 = t;
    };
    // 1. pool layout: every stored block of both sides (padded rows), then derived matrices
    std::vector<int64_t> base_off[2];
    int64_t pool = 0;
    H.pool_blocks.clear();
    auto reserve = [&](int rows, int cols) {
        int64_t o = pool;
        H.pool_blocks.push_back({o, dmrg::rows_of(rows) / 16, dmrg::ld_of(cols) / 32});
        pool += (int64_t)dmrg::rows_of(rows) * dmrg::ld_of(cols);
        pool = (pool + 31) / 32 * 32;
        return o;
    };
    for (int sd = 0; sd < 2; ++sd) {
        BlockIn& B = sd == 0 ? H.left : H.right;
        base_off[sd].assign(B.ops.size() * (size_t)B.n_sec, -1);
        for (size_t k = 0; k < B.ops.size(); ++k)
            for (int si = 0; si < B.n_sec; ++si) {
                int so = B.ops[k].out_of_in[si];
                if (so < 0) continue;
                base_off[sd][k * B.n_sec + si] = reserve(B.dim[so], B.dim[si]);
            }
    }
    H.op_pool_off[0] = base_off[0];
    H.op_pool_off[1] = base_off[1];
    // which matrices are used by tasks
    std::vector<char> used(H.mats.size(), 0);
    for (const auto& t : H.tasks) { if (t.lm >= 0) used[t.lm] = 1; if (t.rm >= 0) used[t.rm] = 1; }
    std::vector<dmrg::PresumBlock> pblocks;
    std::vector<dmrg::PresumTerm> pterms;
    for (size_t m = 0; m < H.mats.size(); ++m) {
        MatDef& M = H.mats[m];
        BlockIn& B = M.side == 0 ? H.left : H.right;
        M.pool_of_in.assign(B.n_sec, -1);
        if (!used[m]) continue;
        bool direct = M.terms.size() == 1 && M.terms[0].c == 1.0 && !M.terms[0].tr;
        for (int si = 0; si < B.n_sec; ++si) {
            int so = M.out_of_in[si];
            if (so < 0) continue;
            if (direct) { M.pool_of_in[si] = base_off[M.side][(size_t)M.terms[0].op * B.n_sec + si]; continue; }
            int64_t o = reserve(B.dim[so], B.dim[si]);
            M.pool_of_in[si] = o;
            dmrg::PresumBlock pb{o, B.dim[so], B.dim[si], (int32_t)pterms.size(), 0};
            for (const Term& t : M.terms) {
                int src_in = t.tr ? so : si;          // stored block is (src_out <- src_in)
                const OpIn& op = B.ops[t.op];
                if (op.out_of_in[src_in] < 0) continue;
                int src_out = op.out_of_in[src_in];
                pterms.push_back({base_off[M.side][(size_t)t.op * B.n_sec + src_in], dmrg::ld_of(B.dim[src_in]),
                                  t.tr ? 1 : 0, t.c});
                (void)src_out;
            }
            pb.t_end = (int32_t)pterms.size();
            pblocks.push_back(pb);
        }
    }
    H.pool_size = pool;
    double need = pool * 8.0 * (H.has_split ? 1.5 : 1.0);
    if (opts && opts->mem_budget_bytes > 0 && need > (double)opts->mem_budget_bytes)
        throw Error(DMRG_ERR_NOMEM, "operator pool exceeds the memory budget");
    H.d_pool = dev_alloc<double>(H, pool);
    HIPCHK(hipMemsetAsync(H.d_pool, 0, pool * sizeof(double), s));
    phase("pool layout + alloc");
    // 2. stored blocks, padded, host -> device: packed on the host into the pool layout inside pinned
    //    staging chunks (two, alternating, ~256 MB or one block if larger), one copy per chunk
    {
        struct Src { int64_t off; const double* src; int rows, cols; };
        std::vector<Src> blocks;
        for (int sd = 0; sd < 2; ++sd) {
            BlockIn& B = sd == 0 ? H.left : H.right;
            for (size_t k = 0; k < B.ops.size(); ++k)
                for (int si = 0; si < B.n_sec; ++si) {
                    int so = B.ops[k].out_of_in[si];
                    if (so < 0) continue;
                    int rows = B.dim[so], cols = B.dim[si];
                    if (rows == 0 || cols == 0) continue;
                    blocks.push_back({base_off[sd][k * B.n_sec + si], B.data + B.ops[k].off_of_in[si], rows, cols});
                }
        }
        std::sort(blocks.begin(), blocks.end(), [](const Src& a, const Src& b) { return a.off < b.off; });
        auto extent = [](const Src& b) { return (int64_t)dmrg::rows_of(b.rows) * dmrg::ld_of(b.cols); };
        int64_t cap = (int64_t)32 << 20;                       // doubles per staging chunk
        for (const Src& b : blocks) cap = std::max(cap, extent(b));
        if (!blocks.empty()) cap = std::min(cap, std::max(blocks.back().off + extent(blocks.back()), (int64_t)1));
        double* stage[2] = {nullptr, nullptr};
        hipEvent_t done[2] = {nullptr, nullptr};
        bool used[2] = {false, false};
        try {
            for (int b = 0; b < 2 && !blocks.empty(); ++b) {
                HIPCHK(hipHostMalloc((void**)&stage[b], (size_t)cap * sizeof(double), hipHostMallocDefault));
                HIPCHK(hipEventCreateWithFlags(&done[b], hipEventDisableTiming));
            }
            size_t i = 0;
            for (int slot = 0; i < blocks.size(); slot ^= 1) {
                const int64_t c0 = blocks[i].off;
                size_t e = i;
                while (e < blocks.size() && blocks[e].off + extent(blocks[e]) - c0 <= cap) ++e;
                const int64_t len = blocks[e - 1].off + extent(blocks[e - 1]) - c0;
                if (used[slot]) HIPCHK(hipEventSynchronize(done[slot]));   // the copy out of this buffer is done
                double* st = stage[slot];
                std::memset(st, 0, (size_t)len * sizeof(double));
                for (size_t q = i; q < e; ++q) {
                    const Src& b = blocks[q];
                    const int ld = dmrg::ld_of(b.cols);
                    for (int r = 0; r < b.rows; ++r)
                        std::memcpy(st + (b.off - c0) + (int64_t)r * ld, b.src + (int64_t)r * b.cols,
                                    (size_t)b.cols * sizeof(double));
                }
                HIPCHK(hipMemcpyAsync(H.d_pool + c0, st, (size_t)len * sizeof(double), hipMemcpyHostToDevice, s));
                HIPCHK(hipEventRecord(done[slot], s));
                used[slot] = true;
                i = e;
            }
            HIPCHK(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipStreamSynchronize(s);
            for (int b = 0; b < 2; ++b) {
                if (stage[b]) (void)hipHostFree(stage[b]);
                if (done[b]) (void)hipEventDestroy(done[b]);
            }
            throw;
        }
        for (int b = 0; b < 2; ++b) {
            if (stage[b]) (void)hipHostFree(stage[b]);
            if (done[b]) (void)hipEventDestroy(done[b]);
        }
    }
    phase("operator upload");
    // 3. pre-summed and transposed matrices on the GPU (Section 2.2.3)
    if (!pblocks.empty()) {
        dmrg::PresumBlock* d_pb = dev_alloc<dmrg::PresumBlock>(H, pblocks.size());
        dmrg::PresumTerm* d_pt = dev_alloc<dmrg::PresumTerm>(H, pterms.size());
        HIPCHK(hipMemcpyAsync(d_pb, pblocks.data(), pblocks.size() * sizeof(pblocks[0]), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_pt, pterms.data(), pterms.size() * sizeof(pterms[0]), hipMemcpyHostToDevice, s));
        HIPCHK(dmrg::launch_presum(d_pb, (int)pblocks.size(), d_pt, H.d_pool, s));
    }
    phase("pre-summation");
    // 4. split copies: tiled hi/lo for the LDS-staged kernel; row-major hi/lo only when some target
    //    needs the one-wave kernel
    if (H.has_split) {
        make_tiled_split(H, s);
        if (!H.tune_big && needs_fallback(H)) {
            H.d_hi = dev_alloc<uint16_t>(H, pool);
            H.d_lo = dev_alloc<uint16_t>(H, pool);
            HIPCHK(dmrg::launch_split(H.d_pool, pool, H.d_hi, H.d_lo, s));
        }
    }
    phase("split tiling");
    // 5. packed input layout, work items and launch plan
    build_plan(H, s);
    phase("launch plans");
    // 7. diag(H): tasks mapping a block onto itself (host staging vectors live until the final sync)
    std::vector<dmrg::DiagBlock> db;
    std::vector<dmrg::DiagTask> dt;
    {
        size_t k = 0;
        for (size_t j = 0; j < H.blk.size(); ++j) {
            int32_t tb = (int32_t)dt.size();
            while (k < H.tasks.size() && H.tasks[k].j == (int)j) {
                const auto& ht = H.tasks[k];
                if (ht.i == (int)j) {
                    int64_t ao = ht.lm >= 0 ? H.mats[ht.lm].pool_of_in[H.blk[j][0]] : -1;
                    int64_t bo = ht.rm >= 0 ? H.mats[ht.rm].pool_of_in[H.blk[j][3]] : -1;
                    dt.push_back({ao, bo, ht.f});
                }
                ++k;
            }
            db.push_back({H.blk_off[j], H.blk_ma[j], H.blk_md[j], tb, (int32_t)dt.size()});
        }
        H.d_diag = dev_alloc<double>(H, H.n_coeff);
        dmrg::DiagBlock* d_db = dev_alloc<dmrg::DiagBlock>(H, db.size());
        dmrg::DiagTask* d_dt = dev_alloc<dmrg::DiagTask>(H, dt.size());
        HIPCHK(hipMemcpyAsync(d_db, db.data(), db.size() * sizeof(db[0]), hipMemcpyHostToDevice, s));
        if (!dt.empty()) HIPCHK(hipMemcpyAsync(d_dt, dt.data(), dt.size() * sizeof(dt[0]), hipMemcpyHostToDevice, s));
        HIPCHK(dmrg::launch_diag(d_db, (int)db.size(), d_dt, H.d_pool, H.d_diag, s));
    }
    // bytes: distinct operator blocks used + x read + y write
    double by = 16.0 * H.n_coeff;
    std::vector<char> seen_blk;
    {
        std::map<int64_t, int64_t> distinct;
        for (const auto& ht : H.tasks) {
            if (ht.lm >= 0) { int a = H.blk[ht.i][0]; int so = H.mats[ht.lm].out_of_in[a];
                distinct[H.mats[ht.lm].pool_of_in[a]] = (int64_t)H.left.dim[so] * H.left.dim[a]; }
            if (ht.rm >= 0) { int d = H.blk[ht.i][3]; int so = H.mats[ht.rm].out_of_in[d];
                distinct[H.mats[ht.rm].pool_of_in[d]] = (int64_t)H.right.dim[so] * H.right.dim[d]; }
        }
        for (auto& kv : distinct) by += 8.0 * kv.second;
    }
    H.bytes = by;
    HIPCHK(hipStreamSynchronize(s));
    phase("diag(H) + byte count");
    if (btrace) std::fprintf(stderr, "[dmrg build] device memory: %.1f MB data + %.1f MB plans\n", H.dev_bytes * 1e-6,
                             H.plan_bytes * 1e-6);
}

dmrg_status fail(const Error& e) { g_err = e.what(); return e.code; }

}  // namespace

namespace dmrg {
dmrg_status record_error(const Error& e) { return fail(e); }
std::string& last_error() { return g_err; }
void clear_error() { g_err.clear(); }
double now_seconds() { return now(); }
}  // namespace dmrg

// ====================================================================== C-ABI

extern "C" const char* dmrg_last_error(void) { return g_err.c_str(); }
extern "C" const char* dmrg_version(void) { return "libdmrg 0.1 (gfx950)"; }

extern "C" dmrg_status dmrg_build_blocks(const dmrg_problem* p, const dmrg_block* left,
                                         const dmrg_block* right, const dmrg_build_opts* opts,
                                         dmrg_hop** out) {
    g_err.clear();
    if (!out) { g_err = "out is NULL"; return DMRG_ERR_ARG; }
    *out = nullptr;
    dmrg_hop* H = new (std::nothrow) dmrg_hop;
    if (!H) { g_err = "host allocation failed"; return DMRG_ERR_NOMEM; }
    try {
        if (!p || !p->h || !p->eri) throw Error(DMRG_ERR_ARG, "problem or its integrals are NULL");
        if (p->n_orb < 2 || p->site < 0 || p->site > p->n_orb - 2)
            throw Error(DMRG_ERR_ARG, "need n_orb >= 2 and 0 <= site <= n_orb - 2");
        if (p->n_alpha < 0 || p->n_beta < 0 || p->n_alpha > p->n_orb || p->n_beta > p->n_orb)
            throw Error(DMRG_ERR_ARG, "electron numbers out of range");
        H->L = p->n_orb; H->na = p->n_alpha; H->nb = p->n_beta; H->site = p->site;
        int64_t L = H->L;
        H->h.assign(p->h, p->h + L * L);
        H->eri.assign(p->eri, p->eri + L * L * L * L);
        for (double v : H->h) if (!std::isfinite(v)) throw Error(DMRG_ERR_NAN, "non-finite one-electron integral");
        for (double v : H->eri) if (!std::isfinite(v)) throw Error(DMRG_ERR_NAN, "non-finite two-electron integral");
        H->left = import_block(left, "left");
        H->right = import_block(right, "right");
        H->share = opts && opts->share != 0;
        build_layout(*H);
        Builder(*H).generate();
        build_tasks(*H);
        H->n_alpha = (int64_t)H->alphas.size();
        H->part_coeff = {0, H->n_coeff};
        int dev = opts ? opts->device : 0;
        if (const char* e = std::getenv("DMRG_MAX_TQ")) H->tune_max_tq = std::max(1, std::min(8, std::atoi(e)));
        if (const char* e = std::getenv("DMRG_ITEMS")) H->tune_items = std::max(256, std::atoi(e));
        if (const char* e = std::getenv("DMRG_ORDER")) H->tune_order = std::max(0, std::min(2, std::atoi(e)));
        if (const char* e = std::getenv("DMRG_PHASES")) H->tune_phases = std::max(0, std::atoi(e));
        if (const char* e = std::getenv("DMRG_LDS_ITEMS")) H->tune_lds_items = std::max(64, std::atoi(e));
        if (const char* e = std::getenv("DMRG_SMALL_MODE")) H->tune_small_mode = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_SMALL_NR")) H->tune_small_nr = std::max(1, std::min(2, std::atoi(e)));
        if (const char* e = std::getenv("DMRG_LDS_ORDER")) H->tune_lds_order = std::max(0, std::min(2, std::atoi(e)));
        if (const char* e = std::getenv("DMRG_LDS_SPLIT64")) H->tune_lds_split64 = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS_PF")) H->tune_lds_pf = std::atoi(e) & 0xF;
        if (const char* e = std::getenv("DMRG_LDS_W6")) H->tune_lds_w6 = std::atoi(e) & 0xA;
        if (const char* e = std::getenv("DMRG_BIG")) H->tune_big = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_BIG64")) H->tune_big64 = std::max(0, std::min(2, std::atoi(e)));
        if (const char* e = std::getenv("DMRG_LDS64")) H->tune_lds64 = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS64_ITEMS")) H->tune_lds64_items = std::max(64, std::atoi(e));
        if (const char* e = std::getenv("DMRG_LDS64_SMALL")) H->tune_lds64_small = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS64_W7")) H->tune_lds64_w7 = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS64_CW")) H->tune_lds64_cw = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS64_NS3")) H->tune_lds64_ns3 = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS64_TASK_ROUTE")) H->tune_lds64_task_route = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_LDS_CW")) H->tune_lds_cw = std::atoi(e) & 0xF;
        if (const char* e = std::getenv("DMRG_SPLIT_TASK_ROUTE")) H->tune_split_task_route = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_PART_ITEMS")) H->tune_part_items = std::atoi(e) != 0;
        if (const char* e = std::getenv("DMRG_VEC_STEP")) H->vec_step = std::max(1, std::min(dmrg::kPartialVecs, std::atoi(e)));
        if (const char* e = std::getenv("DMRG_BIG_STAGES")) H->tune_big_stages = std::max(4, std::atoi(e));
        if (const char* e = std::getenv("DMRG_BIG_STAGES1")) H->tune_big_stages1 = std::max(4, std::atoi(e));
        if (const char* e = std::getenv("DMRG_BIG_TBUDGET_MB")) H->tune_big_tbudget_mb = std::max(16, std::atoi(e));
        if (const char* e = std::getenv("DMRG_LDS_TASK_ORDER")) H->tune_lds_task_order = std::atoi(e) == 1 ? 1 : 0;
        if (const char* e = std::getenv("DMRG_SMALL_NQ")) H->tune_small_nq = std::max(2, std::min(6, std::atoi(e))) / 2 * 2;
        H->has_split = opts && opts->want_split;
        if (dev >= 0) {
            int ndev = 0;
            HIPCHK(hipGetDeviceCount(&ndev));
            if (dev >= ndev) throw Error(DMRG_ERR_ARG, "device ordinal out of range");
            H->device = dev;
            upload(*H, opts);
        } else {
            // host-only build: derive matrix sectors for the statistics; no device state
            H->bytes = 16.0 * H->n_coeff;
        }
        *out = H;
        return DMRG_OK;
    } catch (const Error& e) {
        dmrg_status st = fail(e);
        dmrg_hop_free(H);
        return st;
    } catch (const std::bad_alloc&) {
        dmrg_hop_free(H);
        g_err = "host allocation failed";
        return DMRG_ERR_NOMEM;
    } catch (const std::exception& e) {
        dmrg_hop_free(H);
        g_err = e.what();
        return DMRG_ERR_ARG;
    }
}

extern "C" void dmrg_hop_free(dmrg_hop* H) {
    if (!H) return;
    if (H->device >= 0) {
        (void)hipSetDevice(H->device);
        drop_graphs(*H);
        if (H->cap_stream) (void)hipStreamDestroy(H->cap_stream);
        for (void* p : H->allocations) (void)hipFree(p);
        for (void* p : H->plan_allocations) (void)hipFree(p);
    }
    delete H;
}

extern "C" dmrg_status dmrg_hop_layout(const dmrg_hop* H, int64_t* n_coeff, int32_t* n_blocks,
                                       int32_t* abcd, int32_t* dims, int64_t* offsets) {
    g_err.clear();
    if (!H) { g_err = "hop is NULL"; return DMRG_ERR_ARG; }
    if (n_coeff) *n_coeff = H->n_coeff;
    if (n_blocks) *n_blocks = (int32_t)H->blk.size();
    for (size_t i = 0; i < H->blk.size(); ++i) {
        if (abcd) for (int k = 0; k < 4; ++k) abcd[4 * i + k] = H->blk[i][k];
        if (dims) { dims[2 * i] = H->blk_ma[i]; dims[2 * i + 1] = H->blk_md[i]; }
        if (offsets) offsets[i] = H->blk_off[i];
    }
    return DMRG_OK;
}

extern "C" dmrg_status dmrg_hop_stats(const dmrg_hop* H, double* flops, double* bytes, int64_t* n_alpha,
                                      int64_t* n_tasks) {
    g_err.clear();
    if (!H) { g_err = "hop is NULL"; return DMRG_ERR_ARG; }
    if (flops) *flops = H->flops;
    if (bytes) *bytes = H->bytes;
    if (n_alpha) *n_alpha = H->n_alpha;
    if (n_tasks) *n_tasks = (int64_t)H->tasks.size();
    return DMRG_OK;
}

extern "C" dmrg_status dmrg_hop_export_tasks(const dmrg_hop* H, int64_t* n_tasks, int32_t* quads, double* f,
                                             int64_t* n_terms, int32_t* term_int, double* term_coeff) {
    g_err.clear();
    if (!H) { g_err = "hop is NULL"; return DMRG_ERR_ARG; }
    if (n_tasks) *n_tasks = (int64_t)H->tasks.size();
    for (size_t k = 0; k < H->tasks.size(); ++k) {
        const auto& t = H->tasks[k];
        if (quads) { quads[4 * k] = t.i; quads[4 * k + 1] = t.j; quads[4 * k + 2] = t.lm; quads[4 * k + 3] = t.rm; }
        if (f) f[k] = t.f;
    }
    int64_t nt = 0;
    for (size_t m = 0; m < H->mats.size(); ++m)
        for (const Term& t : H->mats[m].terms) {
            if (term_int) {
                term_int[4 * nt] = (int32_t)m;
                term_int[4 * nt + 1] = H->mats[m].side;
                term_int[4 * nt + 2] = t.op;
                term_int[4 * nt + 3] = t.tr ? 1 : 0;
            }
            if (term_coeff) term_coeff[nt] = t.c;
            ++nt;
        }
    if (n_terms) *n_terms = nt;
    return DMRG_OK;
}

namespace {

void check_hpsi_args(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision) {
    if (!H) throw Error(DMRG_ERR_ARG, "hop is NULL");
    if (H->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle has no device state");
    if (H->trimmed) throw Error(DMRG_ERR_UNSUPPORTED, "handle was trimmed (dmrg_hop_trim): it can only be combined");
    if (!x || !y || nvec < 1) throw Error(DMRG_ERR_ARG, "bad x/y/nvec");
    int64_t n = H->n_coeff * nvec;
    if (!(x + n <= y || y + n <= x)) throw Error(DMRG_ERR_ALIAS, "x and y overlap");
    if (precision != DMRG_PREC_FP64 && precision != DMRG_PREC_SPLIT2) throw Error(DMRG_ERR_ARG, "unknown precision");
    if (precision == DMRG_PREC_SPLIT2 && !H->has_split)
        throw Error(DMRG_ERR_UNSUPPORTED, "handle built without split operators");
}

// The launch sequence of one H.psi (no host synchronization, so it can be captured).
void enqueue_hpsi(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision, hipStream_t s) {
    const int step = H->vec_step;   // packed-input and partial buffers hold this many vectors
    const int32_t* act = H->d_active;
    for (int v0 = 0; v0 < nvec; v0 += step) {
        const int nv = std::min(step, nvec - v0);
        const double* xv = x + (int64_t)v0 * H->n_coeff;
        double* yv = y + (int64_t)v0 * H->n_coeff;
        if (precision == DMRG_PREC_FP64) {
            // zeroes y, then the one-wave targets
            HIPCHK(dmrg::launch_hpsi_f64(H->plan, H->d_pool, xv, yv, H->n_coeff, nv, s, act));
            const bool lds = H->lplan64.n_items > 0, big = H->bplan64.n_chunks > 0;
            for (int v = 0; v < nv && (lds || big); ++v) {
                const double* x1 = xv + (int64_t)v * H->n_coeff;
                double* y1 = yv + (int64_t)v * H->n_coeff;
                HIPCHK(dmrg::launch_pack_xt64(H->plan.packs, H->plan.n_packs, x1, H->xt64, s));
                if (lds) HIPCHK(dmrg::launch_hpsi_lds64(H->lplan64, H->d_tiled64, H->xt64, y1, s, act));
                if (big) HIPCHK(dmrg::launch_hpsi_big64(H->bplan64, H->d_tiled64, nullptr, 0, x1, H->xt64, y1, s, act));
            }
        } else {
            HIPCHK(dmrg::launch_hpsi_lds(H->lplan, H->d_tiled, xv, yv, H->n_coeff, nv, true, s, act));
            for (int v = 0; v < nv && H->bplan.n_chunks > 0; ++v)
                HIPCHK(dmrg::launch_hpsi_big(H->bplan, H->d_tiled, H->lplan.xt + (int64_t)v * H->lplan.xt_size,
                                             yv + (int64_t)v * H->n_coeff, s, act));
            if (H->n_fallback_targets > 0)
                HIPCHK(dmrg::launch_hpsi_split_acc(H->plan_fb, H->d_hi, H->d_lo, xv, yv, H->n_coeff, nv, s, act));
        }
    }
}

// Replay (capturing on first use) the hipGraph of the launch sequence for (x, y, nvec, precision).
void launch_hpsi_graph(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision, hipStream_t s) {
    for (const auto& g : H->graphs)
        if (g.x == x && g.y == y && g.nvec == nvec && g.prec == precision) {
            HIPCHK(hipGraphLaunch(g.exec, s));
            return;
        }
    // capture only records the launches (nothing runs on the capture stream); the graph is then
    // launched on s, after the work already queued there
    if (!H->cap_stream) HIPCHK(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
    dmrg_hop::GraphEntry g{x, y, nvec, precision, nullptr, nullptr};
    HIPCHK(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_hpsi(H, x, y, nvec, precision, H->cap_stream);
    } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(H->cap_stream, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        throw;
    }
    HIPCHK(hipStreamEndCapture(H->cap_stream, &g.graph));
    HIPCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    H->graphs.push_back(g);
    HIPCHK(hipGraphLaunch(g.exec, s));
}

}  // namespace

void dmrg::hpsi_enqueue(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision, hipStream_t s) {
    check_hpsi_args(H, x, y, nvec, precision);
    enqueue_hpsi(H, x, y, nvec, precision, s);
}

extern "C" dmrg_status dmrg_hpsi(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision,
                                 void* stream) {
    g_err.clear();
    try {
        check_hpsi_args(H, x, y, nvec, precision);
        HIPCHK(hipSetDevice(H->device));
        enqueue_hpsi(H, x, y, nvec, precision, (hipStream_t)stream);
        return DMRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

extern "C" dmrg_status dmrg_hpsi_batched(dmrg_hop* const* hops, int32_t n, const double* const* x, double* const* y,
                                         int32_t precision, void* stream) {
    g_err.clear();
    try {
        if (n < 0 || (n > 0 && (!hops || !x || !y))) throw Error(DMRG_ERR_ARG, "NULL argument or n < 0");
        for (int32_t i = 0; i < n; ++i) {
            check_hpsi_args(hops[i], x[i], y[i], 1, precision);
            if (hops[i]->device != hops[0]->device) throw Error(DMRG_ERR_ARG, "handles on different devices");
        }
        // no output may overlap another problem's input or output (each pair is checked above)
        for (int32_t i = 0; i < n; ++i)
            for (int32_t j = 0; j < n; ++j) {
                if (i == j) continue;
                const double* yi = y[i];
                const int64_t ni = hops[i]->n_coeff, nj = hops[j]->n_coeff;
                const bool over_x = yi < x[j] + nj && x[j] < yi + ni;
                const bool over_y = yi < y[j] + nj && y[j] < yi + ni;
                if (over_x || over_y) throw Error(DMRG_ERR_ALIAS, "an output overlaps another problem's vector");
            }
        if (n == 0) return DMRG_OK;
        HIPCHK(hipSetDevice(hops[0]->device));
        for (int32_t i = 0; i < n; ++i) enqueue_hpsi(hops[i], x[i], y[i], 1, precision, (hipStream_t)stream);
        return DMRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

extern "C" dmrg_status dmrg_hpsi_graph(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision,
                                       void* stream) {
    g_err.clear();
    try {
        check_hpsi_args(H, x, y, nvec, precision);
        HIPCHK(hipSetDevice(H->device));
        launch_hpsi_graph(H, x, y, nvec, precision, (hipStream_t)stream);
        return DMRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

extern "C" dmrg_status dmrg_hop_diagonal(dmrg_hop* H, double* d, void* stream) {
    g_err.clear();
    try {
        if (!H || !d) throw Error(DMRG_ERR_ARG, "NULL argument");
        if (H->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle has no device state");
        HIPCHK(hipSetDevice(H->device));
        HIPCHK(hipMemcpyAsync(d, H->d_diag, H->n_coeff * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
        return DMRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

// ---------------------------------------------------------------- batching and tuning
extern "C" dmrg_status dmrg_hop_combine(dmrg_hop* const* hops, int32_t n, void* stream, dmrg_hop** out) {
    g_err.clear();
    if (!out) { g_err = "out is NULL"; return DMRG_ERR_ARG; }
    *out = nullptr;
    dmrg_hop* C = new (std::nothrow) dmrg_hop;
    if (!C) { g_err = "host allocation failed"; return DMRG_ERR_NOMEM; }
    try {
        if (!hops || n < 1) throw Error(DMRG_ERR_ARG, "need at least one handle");
        for (int k = 0; k < n; ++k) {
            if (!hops[k]) throw Error(DMRG_ERR_ARG, "NULL handle in the batch");
            if (hops[k]->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle in the batch");
            if (hops[k]->device != hops[0]->device) throw Error(DMRG_ERR_ARG, "handles on different devices");
        }
        hipStream_t s = (hipStream_t)stream;
        C->device = hops[0]->device;
        HIPCHK(hipSetDevice(C->device));
        C->has_split = true;
        for (int k = 0; k < n; ++k) C->has_split = C->has_split && hops[k]->has_split;
        C->tune_max_tq = hops[0]->tune_max_tq;
        C->tune_items = hops[0]->tune_items;
        C->tune_order = hops[0]->tune_order;
        C->tune_phases = 1;
        C->n_parts = n;
        C->part_coeff.assign(1, 0);
        for (int k = 0; k < n; ++k) {
            const dmrg_hop& h = *hops[k];
            const int blk_base = (int)C->blk.size(), mat_base = (int)C->mats.size();
            const int64_t coeff_base = C->n_coeff, pool_base = C->pool_size;
            for (size_t i = 0; i < h.blk.size(); ++i) {
                C->blk.push_back(h.blk[i]);
                C->blk_ma.push_back(h.blk_ma[i]);
                C->blk_md.push_back(h.blk_md[i]);
                C->blk_off.push_back(h.blk_off[i] + coeff_base);
            }
            for (const MatDef& m : h.mats) {
                MatDef c = m;
                for (auto& o : c.pool_of_in) if (o >= 0) o += pool_base;
                c.transpose_id = -1;
                C->mats.push_back(std::move(c));
            }
            for (const auto& t : h.tasks)
                C->tasks.push_back({t.i + blk_base, t.j + blk_base, t.lm >= 0 ? t.lm + mat_base : -1,
                                    t.rm >= 0 ? t.rm + mat_base : -1, t.f});
            for (const auto& pb : h.pool_blocks) C->pool_blocks.push_back({pb.off + pool_base, pb.r16, pb.k32});
            C->n_coeff += h.n_coeff;
            C->pool_size += h.pool_size;
            C->flops += h.flops;
            C->bytes += h.bytes;
            C->n_alpha += h.n_alpha;
            C->part_coeff.push_back(C->n_coeff);
        }
        C->d_pool = dev_alloc<double>(*C, C->pool_size);
        C->d_diag = dev_alloc<double>(*C, C->n_coeff);
        int64_t pb = 0, cb = 0;
        for (int k = 0; k < n; ++k) {
            const dmrg_hop& h = *hops[k];
            HIPCHK(hipMemcpyAsync(C->d_pool + pb, h.d_pool, h.pool_size * sizeof(double), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(C->d_diag + cb, h.d_diag, h.n_coeff * sizeof(double), hipMemcpyDeviceToDevice, s));
            pb += h.pool_size;
            cb += h.n_coeff;
        }
        if (C->has_split) {
            C->tune_big = hops[0]->tune_big;
            make_tiled_split(*C, s);
            if (!C->tune_big && needs_fallback(*C)) {
                C->d_hi = dev_alloc<uint16_t>(*C, C->pool_size);
                C->d_lo = dev_alloc<uint16_t>(*C, C->pool_size);
                HIPCHK(dmrg::launch_split(C->d_pool, C->pool_size, C->d_hi, C->d_lo, s));
            }
        }
        C->tune_big64 = hops[0]->tune_big64;
        C->tune_lds64 = hops[0]->tune_lds64;
        C->tune_lds64_items = hops[0]->tune_lds64_items;
        C->tune_lds64_small = hops[0]->tune_lds64_small;
        C->tune_lds64_w7 = hops[0]->tune_lds64_w7;
        C->tune_lds64_cw = hops[0]->tune_lds64_cw;
        C->tune_lds64_ns3 = hops[0]->tune_lds64_ns3;
        C->tune_lds64_task_route = hops[0]->tune_lds64_task_route;
        C->tune_split_task_route = hops[0]->tune_split_task_route;
        C->tune_part_items = hops[0]->tune_part_items;
        C->vec_step = hops[0]->vec_step;
        C->tune_lds_pf = hops[0]->tune_lds_pf;
        C->tune_lds_w6 = hops[0]->tune_lds_w6;
        C->tune_lds_cw = hops[0]->tune_lds_cw;
        build_plan(*C, s);
        *out = C;
        return DMRG_OK;
    } catch (const Error& e) {
        dmrg_status st = fail(e);
        dmrg_hop_free(C);
        return st;
    } catch (const std::bad_alloc&) {
        dmrg_hop_free(C);
        g_err = "host allocation failed";
        return DMRG_ERR_NOMEM;
    }
}

extern "C" dmrg_status dmrg_hop_parts(const dmrg_hop* H, int32_t* n_parts, int64_t* first_coeff) {
    g_err.clear();
    if (!H) { g_err = "hop is NULL"; return DMRG_ERR_ARG; }
    if (n_parts) *n_parts = H->n_parts;
    if (first_coeff) for (size_t k = 0; k < H->part_coeff.size(); ++k) first_coeff[k] = H->part_coeff[k];
    return DMRG_OK;
}

// Autotuner: times the H.psi launch plan for candidate (widest tile, work items, launch order)
// settings on the device and keeps the fastest.
// Release everything of a handle that only H.psi needs (launch plans, graphs, tiled operator
// copies), keeping the FP64 pool, diag(H) and the host description, which dmrg_hop_combine reads.
extern "C" dmrg_status dmrg_hop_trim(dmrg_hop* H) {
    g_err.clear();
    try {
        if (!H) throw Error(DMRG_ERR_ARG, "hop is NULL");
        if (H->device < 0 || H->trimmed) return DMRG_OK;
        HIPCHK(hipSetDevice(H->device));
        HIPCHK(hipDeviceSynchronize());   // no kernel of this handle may still be reading what is freed
        drop_graphs(*H);
        for (void* p : H->plan_allocations) (void)hipFree(p);
        H->plan_allocations.clear();
        H->plan_bytes = 0;
        H->plan = dmrg::HpsiPlan{};
        H->plan_fb = dmrg::HpsiPlan{};
        H->lplan = dmrg::LdsPlan{};
        H->bplan = dmrg::BigPlan{};
        H->bplan64 = dmrg::BigPlan{};
        H->lplan64 = dmrg::LdsPlan64{};
        H->launches.clear(); H->phases.clear(); H->launches_fb.clear(); H->phases_fb.clear();
        H->big_chunks.clear(); H->big_chunks64.clear();
        H->n_fallback_targets = 0;
        H->xt64 = nullptr;
        auto release = [&](void* p, int64_t bytes) {
            if (!p) return;
            auto it = std::find(H->allocations.begin(), H->allocations.end(), p);
            if (it != H->allocations.end()) H->allocations.erase(it);
            (void)hipFree(p);
            H->dev_bytes -= bytes;
        };
        release(H->d_tiled, H->tiled_size * (int64_t)sizeof(uint16_t));
        release(H->d_tiled64, H->tiled64_size * (int64_t)sizeof(double));
        release(H->d_hi, H->pool_size * (int64_t)sizeof(uint16_t));
        release(H->d_lo, H->pool_size * (int64_t)sizeof(uint16_t));
        H->d_tiled = nullptr; H->d_tiled64 = nullptr; H->d_hi = nullptr; H->d_lo = nullptr;
        H->tiled_size = H->tiled64_size = 0;
        H->trimmed = true;
        return DMRG_OK;
    } catch (const Error& e) {
        return fail(e);
    }
}

extern "C" dmrg_status dmrg_hop_autotune(dmrg_hop* H, int32_t precision, int32_t reps, void* stream,
                                         int32_t* chosen, double* best_ms) {
    g_err.clear();
    void* xy = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        if (!H) throw Error(DMRG_ERR_ARG, "hop is NULL");
        if (H->device < 0) throw Error(DMRG_ERR_UNSUPPORTED, "host-only handle has no device state");
        if (H->trimmed) throw Error(DMRG_ERR_UNSUPPORTED, "handle was trimmed (dmrg_hop_trim)");
        if (precision != DMRG_PREC_FP64 && precision != DMRG_PREC_SPLIT2) throw Error(DMRG_ERR_ARG, "unknown precision");
        if (precision == DMRG_PREC_SPLIT2 && !H->has_split)
            throw Error(DMRG_ERR_UNSUPPORTED, "handle built without split operators");
        if (reps < 1) reps = 3;
        HIPCHK(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)stream;
        HIPCHK(hipMalloc(&xy, 2 * H->n_coeff * sizeof(double)));
        double* x = (double*)xy;
        double* y = x + H->n_coeff;
        HIPCHK(hipMemsetAsync(x, 0, H->n_coeff * sizeof(double), s));
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        // The plan's settings, each with its candidate values (the current value is measured first).
        // Split: LDS item count and launch order, the task-mode tile (row tiles x column tiles per
        // wavefront: 1 x 2 / 2 x 2 / 1 x 4), the 64-wide stage classes, the six-wavefront (S, 2)
        // classes, the copy and prefetch wavefronts. FP64: the LDS-staged kernel's item count, copy
        // wavefront, single-tile sources and 7-wavefront register cap, the two-pass routing of large
        // targets, and the one-wavefront kernel's tile width, item count and launch order.
        struct Knob { int* field; std::vector<int> cand; };
        std::vector<Knob> knobs;
        int small_shape = H->tune_small_nq > 2 ? 2 : H->tune_small_nr > 1 ? 1 : 0;
        const bool split = precision == DMRG_PREC_SPLIT2;
        if (split) {
            knobs.push_back({&H->tune_lds_items, {4096, 8192, 16384, 32768, 65536}});
            knobs.push_back({&H->tune_lds_order, H->n_parts > 1 ? std::vector<int>{0, 1, 2} : std::vector<int>{0, 1}});
            knobs.push_back({&small_shape, {0, 1, 2}});
            knobs.push_back({&H->tune_lds_split64, {1, 0}});
            knobs.push_back({&H->tune_lds_w6, {0x8, 0, 0xA}});
            knobs.push_back({&H->tune_lds_cw, {0, 0xF}});
            knobs.push_back({&H->tune_lds_pf, {0x4, 0}});
        } else {
            const bool lds64 = H->tune_lds64 != 0;
            knobs.push_back({&H->tune_lds64_items, lds64 ? std::vector<int>{8192, 16384, 32768, 65536} : std::vector<int>{}});
            knobs.push_back({&H->tune_lds64_cw, lds64 ? std::vector<int>{1, 0} : std::vector<int>{}});
            knobs.push_back({&H->tune_lds64_small, lds64 ? std::vector<int>{1, 0} : std::vector<int>{}});
            knobs.push_back({&H->tune_lds64_w7, lds64 ? std::vector<int>{1, 0} : std::vector<int>{}});
            knobs.push_back({&H->tune_big64, {1, 2}});
            knobs.push_back({&H->tune_max_tq, {2, 4, 8}});
            knobs.push_back({&H->tune_items, {8192, 32768, 65536}});
            knobs.push_back({&H->tune_order, {0, 2}});
        }
        const char* tr = std::getenv("DMRG_AUTOTUNE_TRACE");
        const bool trace = tr && tr[0] == '1';
        auto measure = [&]() {
            H->tune_small_nr = small_shape == 1 ? 2 : 1;
            H->tune_small_nq = small_shape == 2 ? 4 : 2;
            const double tb = now();
            build_plan(*H, s);
            const double t_build = now() - tb;
            dmrg_status st = dmrg_hpsi(H, x, y, 1, precision, stream);   // warm-up
            if (st != DMRG_OK) throw Error(st, g_err);
            double best = INFINITY;
            for (int r = 0; r < reps; ++r) {
                HIPCHK(hipEventRecord(e0, s));
                st = dmrg_hpsi(H, x, y, 1, precision, stream);
                if (st != DMRG_OK) throw Error(st, g_err);
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                best = std::min(best, (double)ms);
            }
            if (trace) {
                std::fprintf(stderr, "[dmrg autotune] precision %d:", precision);
                for (const Knob& k : knobs) std::fprintf(stderr, " %d", *k.field);
                std::fprintf(stderr, " -> %.3f ms (plan built in %.2f s)\n", best, t_build);
            }
            return best;
        };
        // one pass of coordinate descent: each setting in turn takes its fastest candidate, the
        // others held at their best values so far
        double best = measure();
        for (Knob& k : knobs) {
            const int keep = *k.field;
            int arg = keep;
            for (int v : k.cand) {
                if (v == keep) continue;
                *k.field = v;
                const double t = measure();
                if (t < best) { best = t; arg = v; }
            }
            *k.field = arg;
        }
        const double final_ms = measure();
        if (chosen)
            for (int i = 0; i < DMRG_AUTOTUNE_KNOBS; ++i) chosen[i] = i < (int)knobs.size() ? *knobs[i].field : 0;
        if (best_ms) *best_ms = std::min(best, final_ms);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(xy);
        return DMRG_OK;
    } catch (const Error& e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (xy) (void)hipFree(xy);
        return fail(e);
    }
}

