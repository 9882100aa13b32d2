// Growth of a block by one site and its renormalization (Section 2.1: "complete operator
// intermediates" of the enlarged block, the truncation by the M leading eigenvectors of rho, Eq.
// renorm and Eq. renorm_mat; Section 2.2.2: renormalization tasks; Section 2.2.3: pre-summed
// operators).
//
// Term generator. Every operator of the enlarged block is written, from its definition, as a sum of
// products (old-block operator) x (site operator), with the old-block factor always a single stored
// operator (or the identity) so that truncated blocks stay projections of the exact operators:
//  * left growth, X' = X + s (X normal, Jordan-Wigner order X before s): a product O_X O_s with O_s
//    of parity p is the matrix (O_X P_X^p) (x) O_s, P_X the parity of X's ket sector. The grown H
//    follows the cut identity X | s: H_X + h_s + sum_W [S^X_W c_W + h.c.] + sum_P [c+_P U^s_P + h.c.]
//    + sum_{P<Q} [A_PQ P^s_PQ + h.c.] + sum_XY B_XY Q^s_XY, with the site-side complementary
//    operators as 4 x 4 matrices; C, A, B, S of X' split the same way (e.g. S'_W gets
//    (w_PQrW - w_QPrW) A_PQ P_X (x) c_r and (w_yXRW - w_XyRW) B_XR P_X (x) c+_y).
//  * right growth, Y' = s + Y (Y complementary, s before Y): O_s O_Y is (O_s P_s^p) (x) O_Y with p the
//    parity of O_Y, so the parity folds into the 4 x 4 site matrix. U', P', Q' of Y' take the stored
//    U, P, Q of Y where every index but the site's is summed inside Y (e.g. the two terms of U'_P with
//    one site index among the annihilators add up to c_t (x) Q^Y_Pt), and pre-summed C of Y (sums of
//    w over one Y index) where a site operator takes the place of a summed index.
// Each site matrix is cut into elementary matrices E_{s's}; the old-block factors of one (s', s) are
// pre-summed into one matrix Z, so a grown operator is sum_{s's} (Z_{s's} P^p) (x) E_{s's}. Its
// renormalized sector blocks are sums of coef * O_out^T Z O_in over (piece, old sector) items
// (grow.hip).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "grow.h"
#include "hop.h"

namespace dmrg {
namespace {

// ---------------------------------------------------------------- 4 x 4 site matrices
using M4 = std::array<double, 16>;   // index s' * 4 + s, basis (0, up, down, updown)

M4 zero4() { M4 m; m.fill(0.0); return m; }
M4 eye4() { M4 m = zero4(); for (int i = 0; i < 4; ++i) m[i * 5] = 1.0; return m; }
M4 mul4(const M4& a, const M4& b) {
    M4 c = zero4();
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j) c[i * 4 + j] += a[i * 4 + k] * b[k * 4 + j];
    return c;
}
M4 tr4(const M4& a) { M4 c; for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) c[j * 4 + i] = a[i * 4 + j]; return c; }
void axpy4(M4& y, double a, const M4& x) { for (int i = 0; i < 16; ++i) y[i] += a * x[i]; }
// c+ of site mode y (0 = up, 1 = down), |updown> = c+_up c+_down |0>
M4 cd4(int y) {
    M4 m = zero4();
    if (y == 0) { m[1 * 4 + 0] = 1.0; m[3 * 4 + 2] = 1.0; }
    else        { m[2 * 4 + 0] = 1.0; m[3 * 4 + 1] = -1.0; }
    return m;
}
M4 c4(int y) { return tr4(cd4(y)); }
M4 par4() { M4 m = zero4(); m[0] = 1.0; m[5] = -1.0; m[10] = -1.0; m[15] = 1.0; return m; }
const int kSiteN[4] = {0, 1, 1, 2};
bool odd_elem(int k) { return ((kSiteN[k / 4] - kSiteN[k % 4]) & 1) != 0; }

// ---------------------------------------------------------------- grown-operator definitions
struct XT { double c; int op; bool tr; };           // op -1: identity of the old block
struct GrownDef {
    int kind, i0, i1;
    std::map<int, std::vector<XT>> piece;           // key s' * 4 + s
};

class Gen {
public:
    Gen(const BlockIn& B, bool right, int site, const Integrals& I)
        : B(B), right(right), site(site), I(I), empty(right ? site + 1 >= I.L : site == 0) {}
    std::vector<GrownDef> defs;

    void generate() { if (right) gen_right(); else gen_left(); }

private:
    const BlockIn& B;
    bool right;
    int site;
    const Integrals& I;
    const bool empty;                             // the old block has no orbitals (the vacuum)

    XT ref(double c, int kind, int i0, int i1 = -1, bool tr = false) {
        int k = B.find(kind, i0, i1);
        if (k >= 0) return {c, k, tr};
        if (kind == DMRG_OP_B || kind == DMRG_OP_Q) {
            k = B.find(kind, i1, i0);
            if (k >= 0) return {c, k, !tr};
        }
        if (empty) return {0.0, -2, false};      // operators of an empty block vanish
        char buf[160];
        std::snprintf(buf, sizeof buf, "%s block lacks operator %s(%d,%d)", right ? "right" : "left", kind_name(kind),
                      i0, i1);
        throw Error(DMRG_ERR_ARG, buf);
    }
    static XT ident(double c = 1.0) { return {c, -1, false}; }

    GrownDef& def(int kind, int i0 = -1, int i1 = -1) {
        defs.push_back(GrownDef{kind, i0, i1, {}});
        return defs.back();
    }
    // g += sum over xs of (x_c * X * P^p) (x) M, p the parity of each elementary piece (left growth:
    // on X's ket sector; right growth: already inside M)
    void emit(GrownDef& g, const std::vector<XT>& xs, const M4& m) {
        for (int k = 0; k < 16; ++k) {
            if (m[k] == 0.0) continue;
            auto& v = g.piece[k];
            for (const XT& x : xs)
                if (x.op != -2 && x.c != 0.0) v.push_back({x.c * m[k], x.op, x.tr});
        }
    }
    // the transposed term (Hermitian conjugate). Left growth: (X P_X^p)^T = P_X^p X^T, which is
    // -X^T P_X for odd X and odd p.
    void emit_hc(GrownDef& g, const std::vector<XT>& xs, const M4& m, bool x_odd) {
        std::vector<XT> t;
        for (const XT& x : xs) t.push_back({x.c, x.op, x.op >= 0 ? !x.tr : false});
        const M4 mt = tr4(m);
        if (!right && x_odd) {
            M4 even = zero4(), odd = zero4();
            for (int k = 0; k < 16; ++k) (odd_elem(k) ? odd : even)[k] = mt[k];
            emit(g, t, even);
            for (XT& x : t) x.c = -x.c;
            emit(g, t, odd);
        } else {
            emit(g, t, mt);
        }
    }

    M4 site_h(int G0) const {
        M4 hs = zero4();
        M4 cd[2] = {cd4(0), cd4(1)}, c[2] = {c4(0), c4(1)};
        for (int y = 0; y < 2; ++y)
            for (int z = 0; z < 2; ++z)
                if (double v = I.t(G0 + y, G0 + z)) axpy4(hs, v, mul4(cd[y], c[z]));
        for (int p = 0; p < 2; ++p) for (int q = 0; q < 2; ++q) for (int r = 0; r < 2; ++r) for (int s = 0; s < 2; ++s)
            if (double v = I.w(G0 + p, G0 + q, G0 + r, G0 + s))
                axpy4(hs, 0.5 * v, mul4(mul4(cd[p], cd[q]), mul4(c[r], c[s])));
        return hs;
    }

    void gen_left() {
        const int nX = 2 * site, G0 = 2 * site, L2 = 2 * I.L;
        const M4 I4 = eye4();
        M4 cd[2] = {cd4(0), cd4(1)}, c[2] = {c4(0), c4(1)};
        // H' = H_X + h_s + cross terms of the cut X | s
        {
            GrownDef& g = def(DMRG_OP_H);
            emit(g, {ref(1.0, DMRG_OP_H, -1, -1)}, I4);
            emit(g, {ident()}, site_h(G0));
            for (int y = 0; y < 2; ++y) {                           // S^X_W c_W + h.c., W on the site
                std::vector<XT> xs{ref(1.0, DMRG_OP_S, G0 + y)};
                for (int P = 0; P < nX; ++P) xs.push_back(ref(I.t(P, G0 + y), DMRG_OP_C, P));
                emit(g, xs, c[y]);
                emit_hc(g, xs, c[y], true);
            }
            for (int P = 0; P < nX; ++P) {                          // c+_P U^s_P + h.c.
                M4 us = zero4();
                for (int q = 0; q < 2; ++q) for (int z = 0; z < 2; ++z) for (int x = 0; x < 2; ++x)
                    if (double v = I.w(P, G0 + q, G0 + z, G0 + x)) axpy4(us, v, mul4(mul4(cd[q], c[z]), c[x]));
                const std::vector<XT> xs{ref(1.0, DMRG_OP_C, P)};
                emit(g, xs, us);
                emit_hc(g, xs, us, true);
            }
            for (int P = 0; P < nX; ++P)                            // A_PQ P^s_PQ + h.c.
                for (int Q = P + 1; Q < nX; ++Q) {
                    M4 ps = zero4();
                    for (int z = 0; z < 2; ++z) for (int x = 0; x < 2; ++x)
                        if (double v = I.w(P, Q, G0 + z, G0 + x)) axpy4(ps, v, mul4(c[z], c[x]));
                    const std::vector<XT> xs{ref(1.0, DMRG_OP_A, P, Q)};
                    emit(g, xs, ps);
                    emit_hc(g, xs, ps, false);
                }
            for (int X = 0; X < nX; ++X)                            // B_XY Q^s_XY
                for (int Y = 0; Y < nX; ++Y) {
                    M4 qs = zero4();
                    for (int z = 0; z < 2; ++z) for (int x = 0; x < 2; ++x)
                        if (double v = I.w(X, G0 + z, G0 + x, Y) - I.w(X, G0 + z, Y, G0 + x)) axpy4(qs, v, mul4(cd[z], c[x]));
                    emit(g, {ref(1.0, DMRG_OP_B, X, Y)}, qs);
                }
        }
        // C'
        for (int P = 0; P < nX; ++P) emit(def(DMRG_OP_C, P), {ref(1.0, DMRG_OP_C, P)}, I4);
        for (int y = 0; y < 2; ++y) emit(def(DMRG_OP_C, G0 + y), {ident()}, cd[y]);
        // A'_PQ, P < Q
        for (int P = 0; P < nX + 2; ++P)
            for (int Q = P + 1; Q < nX + 2; ++Q) {
                GrownDef& g = def(DMRG_OP_A, P, Q);
                if (Q < nX) emit(g, {ref(1.0, DMRG_OP_A, P, Q)}, I4);
                else if (P < nX) emit(g, {ref(1.0, DMRG_OP_C, P)}, cd[Q - G0]);
                else emit(g, {ident()}, mul4(cd[P - G0], cd[Q - G0]));
            }
        // B'_PQ, P <= Q (B'_QP = B'_PQ^T)
        for (int P = 0; P < nX + 2; ++P)
            for (int Q = P; Q < nX + 2; ++Q) {
                GrownDef& g = def(DMRG_OP_B, P, Q);
                if (Q < nX) emit(g, {ref(1.0, DMRG_OP_B, P, Q)}, I4);
                else if (P < nX) emit(g, {ref(1.0, DMRG_OP_C, P)}, c[Q - G0]);
                else emit(g, {ident()}, mul4(cd[P - G0], c[Q - G0]));
            }
        // S'_W for W right of X' (three-index part)
        for (int W = G0 + 2; W < L2; ++W) {
            GrownDef& g = def(DMRG_OP_S, W);
            emit(g, {ref(1.0, DMRG_OP_S, W)}, I4);
            for (int r = 0; r < 2; ++r) {                           // c+_P c+_Q c_r, P, Q in X
                std::vector<XT> xs;
                for (int P = 0; P < nX; ++P)
                    for (int Q = P + 1; Q < nX; ++Q) xs.push_back(ref(I.w(P, Q, G0 + r, W) - I.w(Q, P, G0 + r, W), DMRG_OP_A, P, Q));
                emit(g, xs, c[r]);
            }
            for (int y = 0; y < 2; ++y) {                           // one creator on the site, X's B
                std::vector<XT> xs;
                for (int X = 0; X < nX; ++X)
                    for (int R = 0; R < nX; ++R)
                        xs.push_back(ref(I.w(G0 + y, X, R, W) - I.w(X, G0 + y, R, W), DMRG_OP_B, X, R));
                emit(g, xs, cd[y]);
            }
            for (int y = 0; y < 2; ++y)                             // c+_P (x) c+_y c_z
                for (int z = 0; z < 2; ++z) {
                    std::vector<XT> xs;
                    for (int P = 0; P < nX; ++P)
                        xs.push_back(ref(I.w(P, G0 + y, G0 + z, W) - I.w(G0 + y, P, G0 + z, W), DMRG_OP_C, P));
                    emit(g, xs, mul4(cd[y], c[z]));
                }
            for (int p = 0; p < 2; ++p)                             // c_R (x) c+_p c+_q
                for (int q = 0; q < 2; ++q) {
                    if (p == q) continue;
                    std::vector<XT> xs;
                    for (int R = 0; R < nX; ++R) xs.push_back(ref(I.w(G0 + p, G0 + q, R, W), DMRG_OP_C, R, -1, true));
                    emit(g, xs, mul4(cd[p], cd[q]));
                }
            M4 s3 = zero4();                                        // all three on the site
            for (int p = 0; p < 2; ++p) for (int q = 0; q < 2; ++q) for (int r = 0; r < 2; ++r)
                if (double v = I.w(G0 + p, G0 + q, G0 + r, W)) axpy4(s3, v, mul4(mul4(cd[p], cd[q]), c[r]));
            emit(g, {ident()}, s3);
        }
    }

    void gen_right() {
        const int G0 = 2 * site, Y0 = 2 * (site + 1), L2 = 2 * I.L;
        const M4 I4 = eye4(), P4 = par4();
        M4 cd[2] = {cd4(0), cd4(1)}, c[2] = {c4(0), c4(1)};
        // H' = h_s + H_Y + cross terms of the cut s | Y
        {
            GrownDef& g = def(DMRG_OP_H);
            emit(g, {ref(1.0, DMRG_OP_H, -1, -1)}, I4);
            emit(g, {ident()}, site_h(G0));
            for (int W = Y0; W < L2; ++W) {                         // S^s_W c_W + h.c.
                M4 ss = zero4();
                for (int y = 0; y < 2; ++y) if (double v = I.t(G0 + y, W)) axpy4(ss, v, cd[y]);
                for (int p = 0; p < 2; ++p) for (int q = 0; q < 2; ++q) for (int r = 0; r < 2; ++r)
                    if (double v = I.w(G0 + p, G0 + q, G0 + r, W)) axpy4(ss, v, mul4(mul4(cd[p], cd[q]), c[r]));
                const M4 m = mul4(ss, P4);
                const std::vector<XT> xs{ref(1.0, DMRG_OP_C, W, -1, true)};
                emit(g, xs, m);
                emit_hc(g, xs, m, true);
            }
            for (int p = 0; p < 2; ++p) {                           // c+_p U^Y_p + h.c.
                const M4 m = mul4(cd[p], P4);
                const std::vector<XT> xs{ref(1.0, DMRG_OP_U, G0 + p)};
                emit(g, xs, m);
                emit_hc(g, xs, m, true);
            }
            {                                                       // A_{up,down} P^Y + h.c.
                const M4 m = mul4(cd[0], cd[1]);
                const std::vector<XT> xs{ref(1.0, DMRG_OP_P, G0, G0 + 1)};
                emit(g, xs, m);
                emit_hc(g, xs, m, false);
            }
            for (int x = 0; x < 2; ++x)                             // B_xy Q^Y_xy
                for (int y = 0; y < 2; ++y) emit(g, {ref(1.0, DMRG_OP_Q, G0 + x, G0 + y)}, mul4(cd[x], c[y]));
        }
        // C'
        for (int y = 0; y < 2; ++y) emit(def(DMRG_OP_C, G0 + y), {ident()}, cd[y]);
        for (int Z = Y0; Z < L2; ++Z) emit(def(DMRG_OP_C, Z), {ref(1.0, DMRG_OP_C, Z)}, P4);
        // U'_P, P outside Y'
        for (int P = 0; P < G0; ++P) {
            GrownDef& g = def(DMRG_OP_U, P);
            emit(g, {ref(1.0, DMRG_OP_U, P)}, P4);
            for (int q = 0; q < 2; ++q) emit(g, {ref(1.0, DMRG_OP_P, P, G0 + q)}, cd[q]);
            for (int t = 0; t < 2; ++t) emit(g, {ref(1.0, DMRG_OP_Q, P, G0 + t)}, c[t]);
            for (int q = 0; q < 2; ++q)
                for (int z = 0; z < 2; ++z) {
                    std::vector<XT> xs;
                    for (int V = Y0; V < L2; ++V)
                        xs.push_back(ref(I.w(P, G0 + q, G0 + z, V) - I.w(P, G0 + q, V, G0 + z), DMRG_OP_C, V, -1, true));
                    emit(g, xs, mul4(mul4(cd[q], c[z]), P4));
                }
            for (int z = 0; z < 2; ++z)
                for (int x = 0; x < 2; ++x) {
                    if (z == x) continue;
                    std::vector<XT> xs;
                    for (int Q = Y0; Q < L2; ++Q) xs.push_back(ref(I.w(P, Q, G0 + z, G0 + x), DMRG_OP_C, Q));
                    emit(g, xs, mul4(mul4(c[z], c[x]), P4));
                }
            M4 u3 = zero4();
            for (int q = 0; q < 2; ++q) for (int z = 0; z < 2; ++z) for (int x = 0; x < 2; ++x)
                if (double v = I.w(P, G0 + q, G0 + z, G0 + x)) axpy4(u3, v, mul4(mul4(cd[q], c[z]), c[x]));
            emit(g, {ident()}, u3);
        }
        // P'_PQ, P < Q outside Y'
        for (int P = 0; P < G0; ++P)
            for (int Q = P + 1; Q < G0; ++Q) {
                GrownDef& g = def(DMRG_OP_P, P, Q);
                emit(g, {ref(1.0, DMRG_OP_P, P, Q)}, I4);
                for (int t = 0; t < 2; ++t) {
                    std::vector<XT> xs;
                    for (int V = Y0; V < L2; ++V)
                        xs.push_back(ref(I.w(P, Q, G0 + t, V) - I.w(P, Q, V, G0 + t), DMRG_OP_C, V, -1, true));
                    emit(g, xs, mul4(c[t], P4));
                }
                M4 p2 = zero4();
                for (int z = 0; z < 2; ++z) for (int x = 0; x < 2; ++x)
                    if (double v = I.w(P, Q, G0 + z, G0 + x)) axpy4(p2, v, mul4(c[z], c[x]));
                emit(g, {ident()}, p2);
            }
        // Q'_XY, X <= Y outside Y' (Q'_YX = Q'_XY^T)
        for (int X = 0; X < G0; ++X)
            for (int Y = X; Y < G0; ++Y) {
                GrownDef& g = def(DMRG_OP_Q, X, Y);
                emit(g, {ref(1.0, DMRG_OP_Q, X, Y)}, I4);
                for (int t = 0; t < 2; ++t) {
                    std::vector<XT> a, b;
                    for (int V = Y0; V < L2; ++V) {
                        a.push_back(ref(I.w(X, G0 + t, V, Y) - I.w(X, G0 + t, Y, V), DMRG_OP_C, V, -1, true));
                        b.push_back(ref(-(I.w(X, V, G0 + t, Y) - I.w(X, V, Y, G0 + t)), DMRG_OP_C, V));
                    }
                    emit(g, a, mul4(cd[t], P4));
                    emit(g, b, mul4(c[t], P4));
                }
                M4 q2 = zero4();
                for (int z = 0; z < 2; ++z) for (int x = 0; x < 2; ++x)
                    if (double v = I.w(X, G0 + z, G0 + x, Y) - I.w(X, G0 + z, Y, G0 + x)) axpy4(q2, v, mul4(cd[z], c[x]));
                emit(g, {ident()}, q2);
            }
    }
};

// ---------------------------------------------------------------- Z matrices and their sectors
struct ZDef {
    std::vector<XT> terms;      // merged, non-zero
    double coef = 1.0;          // direct reference / identity: the scalar; pre-sum: 1
    int presum = -1;            // index into the pre-sum list, or -1 (direct / identity)
    std::vector<int> out_of_in; // old-block sector map
};

// Bra sector of a (possibly transposed) stored operator for ket sector x.
int op_out(const BlockIn& B, int op, bool tr, int x) {
    const OpIn& o = B.ops[op];
    if (!tr) return o.out_of_in[x];
    for (int s = 0; s < B.n_sec; ++s)
        if (o.out_of_in[s] == x) return s;
    return -1;
}

struct OwnedBlock {
    dmrg_block b{};
    std::vector<int32_t> qn, dim;
    std::vector<dmrg_op> ops;
    std::vector<std::vector<int32_t>> so, si;
    std::vector<std::vector<int64_t>> off;
    std::vector<double> data;
};
std::mutex g_blocks_mu;
std::unordered_map<const dmrg_block*, OwnedBlock*> g_blocks;

struct DevFree {
    std::vector<void*> p;
    ~DevFree() { for (void* q : p) (void)hipFree(q); }
    template <class T> T* alloc(size_t n) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess)
            throw Error(DMRG_ERR_NOMEM, "device allocation failed (block growth)");
        p.push_back(q);
        return static_cast<T*>(q);
    }
};

// Device -> host copy through two pinned 32 MB staging buffers: the DMA of chunk k + 1 overlaps the
// host copy of chunk k (a pageable destination would be copied at a fraction of the link speed).
void download(double* dst, const double* src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    constexpr int64_t kChunk = (int64_t)4 << 20;        // doubles
    const int64_t cs = std::min(n, kChunk);
    double* stage[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto release = [&]() {
        for (int b = 0; b < 2; ++b) {
            if (stage[b]) (void)hipHostFree(stage[b]);
            if (ev[b]) (void)hipEventDestroy(ev[b]);
        }
    };
    try {
        for (int b = 0; b < 2; ++b) {
            HIPCHK(hipHostMalloc((void**)&stage[b], (size_t)cs * sizeof(double), hipHostMallocDefault));
            HIPCHK(hipEventCreateWithFlags(&ev[b], hipEventDisableTiming));
        }
        const int64_t nch = (n + cs - 1) / cs;
        auto issue = [&](int64_t c) {
            const int64_t o = c * cs, len = std::min(cs, n - o);
            HIPCHK(hipMemcpyAsync(stage[c & 1], src + o, (size_t)len * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(ev[c & 1], s));
        };
        issue(0);
        for (int64_t c = 0; c < nch; ++c) {
            if (c + 1 < nch) issue(c + 1);
            HIPCHK(hipEventSynchronize(ev[c & 1]));
            const int64_t o = c * cs, len = std::min(cs, n - o);
            std::memcpy(dst + o, stage[c & 1], (size_t)len * sizeof(double));
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        release();
        throw;
    }
    release();
}

template <class T>
T* upload(DevFree& mem, const std::vector<T>& v, hipStream_t s) {
    T* d = mem.alloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

}  // namespace

// Grow block B (operators on the device: data + op_off[op * n_sec + ket sector], leading dimension
// ld_of(cols) when `padded`, else cols) by one site and renormalize with O (host, per enlarged
// sector of enlarged_layout(B, right): dims x kept row-major, concatenated; kept[q] columns).
dmrg_block* grow_block(const BlockIn& B, bool right, int site, const Integrals& I, const double* data,
                       int64_t data_len, const std::vector<int64_t>& op_off, bool padded, const std::vector<int>& kept,
                       const std::vector<double>& O, int device, hipStream_t s) {
    const EnlargedLayout E = enlarged_layout(B, right);
    const int nq = (int)E.dim.size();
    if ((int)kept.size() != nq) throw Error(DMRG_ERR_SHAPE, "kept must list one count per enlarged sector");
    std::vector<int64_t> ooff(nq + 1, 0);
    for (int q = 0; q < nq; ++q) {
        if (kept[q] < 0 || kept[q] > E.dim[q]) throw Error(DMRG_ERR_ARG, "need 0 <= kept <= enlarged sector dimension");
        ooff[q + 1] = ooff[q] + (int64_t)E.dim[q] * kept[q];
    }
    if ((int64_t)O.size() != ooff[nq]) throw Error(DMRG_ERR_SHAPE, "O has the wrong length for kept");
    // new sectors: the enlarged sectors that keep states
    std::vector<int> new_index(nq, -1);
    auto* ob = new OwnedBlock;
    std::unique_ptr<OwnedBlock> owned(ob);
    for (int q = 0; q < nq; ++q)
        if (kept[q] > 0) {
            new_index[q] = (int)ob->dim.size();
            ob->qn.push_back(E.qn[q].first);
            ob->qn.push_back(E.qn[q].second);
            ob->dim.push_back(kept[q]);
        }
    if (ob->dim.empty()) throw Error(DMRG_ERR_ARG, "the renormalization keeps no state");
    // (old sector, site state) -> (enlarged sector, first row)
    std::vector<std::pair<int, int>> rowmap((size_t)B.n_sec * 4, {-1, -1});
    for (int q = 0; q < nq; ++q)
        for (const auto& gr : E.groups[q]) {
            const int x = right ? gr[1] : gr[0], st = right ? gr[0] : gr[1];
            rowmap[(size_t)x * 4 + st] = {q, gr[2]};
        }
    // term generation
    Gen gen(B, right, site, I);
    gen.generate();
    // Z matrices: direct references and pre-sums (deduplicated)
    std::vector<ZDef> zs;
    std::map<std::vector<std::tuple<int, bool, double>>, int> zcache;
    struct PieceRef { int key, z; };
    std::vector<std::vector<PieceRef>> pieces(gen.defs.size());
    std::vector<PresumBlock> pblocks;
    std::vector<PresumTerm> pterms;
    int64_t zlen = 0, zmax = 0;
    auto ld = [&](int cols) { return padded ? dmrg::ld_of(cols) : cols; };
    for (size_t g = 0; g < gen.defs.size(); ++g) {
        for (auto& kv : gen.defs[g].piece) {
            std::map<std::pair<int, bool>, double> merged;
            for (const XT& x : kv.second) merged[{x.op, x.op >= 0 && x.tr}] += x.c;
            std::vector<std::tuple<int, bool, double>> key;
            for (auto& m : merged)
                if (m.second != 0.0) key.emplace_back(m.first.first, m.first.second, m.second);
            if (key.empty()) continue;
            int zid;
            auto it = zcache.find(key);
            if (it != zcache.end()) {
                zid = it->second;
            } else {
                ZDef z;
                for (auto& k : key) z.terms.push_back({std::get<2>(k), std::get<0>(k), std::get<1>(k)});
                z.out_of_in.assign(B.n_sec, -1);
                for (const XT& t : z.terms)
                    for (int x = 0; x < B.n_sec; ++x) {
                        const int xp = t.op < 0 ? x : op_out(B, t.op, t.tr, x);
                        if (xp < 0) continue;
                        if (z.out_of_in[x] >= 0 && z.out_of_in[x] != xp)
                            throw Error(DMRG_ERR_ARG, "internal: pre-sum mixes operators with different sector changes");
                        z.out_of_in[x] = xp;
                    }
                if (z.terms.size() == 1) {
                    z.coef = z.terms[0].c;
                } else {
                    z.presum = 1;
                }
                zid = (int)zs.size();
                zs.push_back(std::move(z));
                zcache.emplace(key, zid);
            }
            pieces[g].push_back({kv.first, zid});
        }
    }
    // pre-sum blocks (compact) for every used sector of every pre-summed Z
    std::vector<std::vector<int64_t>> zoff(zs.size());
    for (size_t z = 0; z < zs.size(); ++z) {
        if (zs[z].presum < 0) continue;
        zoff[z].assign(B.n_sec, -1);
        for (int x = 0; x < B.n_sec; ++x) {
            const int xp = zs[z].out_of_in[x];
            if (xp < 0 || B.dim[x] == 0 || B.dim[xp] == 0) continue;
            PresumBlock pb{};
            pb.out_off = zlen;
            pb.rows = B.dim[xp];
            pb.cols = B.dim[x];
            pb.t_begin = (int32_t)pterms.size();
            for (const XT& t : zs[z].terms) {
                if (t.op < 0) {                                  // identity (x = xp)
                    PresumTerm pt{};
                    pt.src_off = -1;
                    pt.coeff = t.c;
                    pterms.push_back(pt);
                    continue;
                }
                // stored block of the term that maps x -> xp: (op, ket x) or, transposed, (op, ket xp)
                const int src_in = t.tr ? xp : x;
                const int src_out = t.tr ? x : xp;
                if (B.ops[t.op].out_of_in[src_in] != src_out) continue;
                PresumTerm pt{};
                pt.src_off = op_off[(size_t)t.op * B.n_sec + src_in];
                pt.src_ld = ld(B.dim[src_in]);
                pt.trans = t.tr ? 1 : 0;
                pt.coeff = t.c;
                pterms.push_back(pt);
            }
            pb.t_end = (int32_t)pterms.size();
            pblocks.push_back(pb);
            zoff[z][x] = zlen;
            zlen += (int64_t)pb.rows * pb.cols;
            zmax = std::max<int64_t>(zmax, (int64_t)pb.rows * pb.cols);
        }
    }
    // renormalization items, grouped by output block (grown op, ket sector) in op order
    std::vector<GrowItem> items;
    std::vector<GrowOut> outs;
    std::vector<int32_t> t_items;
    int64_t t_len = 0, max_t = 0, max_out = 0, out_len = 0;
    ob->ops.resize(gen.defs.size());
    ob->so.resize(gen.defs.size());
    ob->si.resize(gen.defs.size());
    ob->off.resize(gen.defs.size());
    for (size_t g = 0; g < gen.defs.size(); ++g) {
        // items per enlarged ket sector
        std::map<int, std::vector<GrowItem>> by_in;
        std::map<int, int> out_of;
        for (const PieceRef& pr : pieces[g]) {
            const int sp = pr.key / 4, st = pr.key % 4;
            const ZDef& z = zs[pr.z];
            const bool par = !right && odd_elem(pr.key);
            for (int x = 0; x < B.n_sec; ++x) {
                const int xp = z.out_of_in[x];
                if (xp < 0 || B.dim[x] == 0 || B.dim[xp] == 0) continue;
                const auto ri = rowmap[(size_t)x * 4 + st], ro = rowmap[(size_t)xp * 4 + sp];
                if (ri.first < 0 || ro.first < 0) throw Error(DMRG_ERR_ARG, "internal: enlarged basis lacks a pair");
                const int qi = ri.first, qo = ro.first;
                if (kept[qi] == 0 || kept[qo] == 0) continue;
                auto oq = out_of.find(qi);
                if (oq != out_of.end() && oq->second != qo)
                    throw Error(DMRG_ERR_ARG, "internal: grown operator with two sector changes");
                out_of[qi] = qo;
                GrowItem it{};
                double coef = z.coef;
                if (par && ((B.qa[x] + B.qb[x]) & 1)) coef = -coef;
                it.coef = coef;
                it.m_out = B.dim[xp];
                it.m_in = B.dim[x];
                it.k_o = kept[qo];
                it.k_i = kept[qi];
                it.oo_off = ooff[qo] + (int64_t)ro.second * kept[qo];
                it.oi_off = ooff[qi] + (int64_t)ri.second * kept[qi];
                if (z.presum >= 0) {
                    it.z_off = zoff[pr.z][x];
                    it.z_ld = B.dim[x];
                    it.z_tr = 0;
                    it.z_buf = 1;
                } else if (z.terms[0].op < 0) {
                    it.z_off = -1;
                } else {
                    const XT& t = z.terms[0];
                    const int src_in = t.tr ? xp : x;
                    it.z_off = op_off[(size_t)t.op * B.n_sec + src_in];
                    it.z_ld = ld(B.dim[src_in]);
                    it.z_tr = t.tr ? 1 : 0;
                    it.z_buf = 0;
                }
                by_in[qi].push_back(it);
            }
        }
        const GrownDef& d = gen.defs[g];
        dmrg_op& op = ob->ops[g];
        op.kind = d.kind;
        op.i0 = d.i0;
        op.i1 = d.i1;
        for (auto& kv : by_in) {
            const int qi = kv.first, qo = out_of[qi];
            GrowOut o{};
            o.out_off = out_len;
            o.k_o = kept[qo];
            o.k_i = kept[qi];
            o.i_begin = (int32_t)items.size();
            for (GrowItem& it : kv.second) {
                if (it.z_off >= 0) {
                    it.t_off = t_len;
                    t_items.push_back((int32_t)items.size());
                    t_len += (int64_t)it.m_out * it.k_i;
                    max_t = std::max<int64_t>(max_t, (int64_t)it.m_out * it.k_i);
                }
                items.push_back(it);
            }
            o.i_end = (int32_t)items.size();
            outs.push_back(o);
            ob->so[g].push_back(new_index[qo]);
            ob->si[g].push_back(new_index[qi]);
            ob->off[g].push_back(out_len);
            out_len += (int64_t)o.k_o * o.k_i;
            max_out = std::max<int64_t>(max_out, (int64_t)o.k_o * o.k_i);
        }
    }
    if (items.size() > (size_t)INT32_MAX || outs.size() > (size_t)INT32_MAX || pblocks.size() > (size_t)INT32_MAX)
        throw Error(DMRG_ERR_UNSUPPORTED, "too many renormalization items");
    // every device access of the three kernels stays inside its buffer (checked before any launch)
    auto inside = [](int64_t off, int64_t rows, int64_t ld, int64_t cols, int64_t len) {
        return rows == 0 || cols == 0 || (off >= 0 && ld >= cols && off + (rows - 1) * ld + cols <= len);
    };
    for (const PresumBlock& pb : pblocks) {
        if (!inside(pb.out_off, pb.rows, pb.cols, pb.cols, zlen)) throw Error(DMRG_ERR_SHAPE, "internal: pre-sum output");
        for (int k = pb.t_begin; k < pb.t_end; ++k) {
            const PresumTerm& pt = pterms[k];
            if (pt.src_off < 0) {
                if (pb.rows != pb.cols) throw Error(DMRG_ERR_SHAPE, "internal: identity term of a non-square block");
                continue;
            }
            const bool ok = pt.trans ? inside(pt.src_off, pb.cols, pt.src_ld, pb.rows, data_len)
                                     : inside(pt.src_off, pb.rows, pt.src_ld, pb.cols, data_len);
            if (!ok) throw Error(DMRG_ERR_SHAPE, "internal: pre-sum source outside the operator data");
        }
    }
    const int64_t olen = (int64_t)O.size();
    for (const GrowOut& o : outs) {
        if (!inside(o.out_off, o.k_o, o.k_i, o.k_i, out_len)) throw Error(DMRG_ERR_SHAPE, "internal: output block");
        for (int k = o.i_begin; k < o.i_end; ++k) {
            const GrowItem& it = items[k];
            if (it.k_o != o.k_o || it.k_i != o.k_i) throw Error(DMRG_ERR_SHAPE, "internal: item shape");
            if (!inside(it.oo_off, it.m_out, it.k_o, it.k_o, olen) || !inside(it.oi_off, it.m_in, it.k_i, it.k_i, olen))
                throw Error(DMRG_ERR_SHAPE, "internal: rows of O outside O");
            if (it.z_off < 0) {
                if (it.m_in != it.m_out) throw Error(DMRG_ERR_SHAPE, "internal: identity item of a non-square block");
                continue;
            }
            if (!inside(it.t_off, it.m_out, it.k_i, it.k_i, t_len)) throw Error(DMRG_ERR_SHAPE, "internal: T block");
            const bool ok = it.z_buf ? inside(it.z_off, it.m_out, it.z_ld, it.m_in, zlen)
                          : it.z_tr ? inside(it.z_off, it.m_in, it.z_ld, it.m_out, data_len)
                                    : inside(it.z_off, it.m_out, it.z_ld, it.m_in, data_len);
            if (!ok) throw Error(DMRG_ERR_SHAPE, "internal: Z block outside its buffer");
        }
    }
    for (int32_t k : t_items)
        if (k < 0 || k >= (int32_t)items.size() || items[k].z_off < 0) throw Error(DMRG_ERR_SHAPE, "internal: pass-1 list");
    // device work (DMRG_GROW_TRACE=1: synchronize after each phase and print its wall time)
    const char* gt = std::getenv("DMRG_GROW_TRACE");
    const bool trace = gt && gt[0] == '1';
    double tp = now_seconds();
    auto phase = [&](const char* what) {
        if (!trace) return;
        HIPCHK(hipStreamSynchronize(s));
        const double t = now_seconds();
        std::fprintf(stderr, "[dmrg grow] %-34s %9.3f ms\n", what, (t - tp) * 1e3);
        tp = t;
    };
    if (trace)
        std::fprintf(stderr, "[dmrg grow] %zu operators, %zu pre-sum blocks (%lld elements, %zu terms), %zu items "
                     "(%zu with T, %lld T elements), %zu output blocks (%lld elements)\n", gen.defs.size(),
                     pblocks.size(), (long long)zlen, pterms.size(), items.size(), t_items.size(), (long long)t_len,
                     outs.size(), (long long)out_len);
    phase("host term list and work lists");
    HIPCHK(hipSetDevice(device));
    {
        DevFree mem;
        double* d_z = mem.alloc<double>((size_t)zlen);
        double* d_o = upload(mem, O, s);
        double* d_t = mem.alloc<double>((size_t)t_len);
        double* d_out = mem.alloc<double>((size_t)out_len);
        const PresumBlock* d_pb = upload(mem, pblocks, s);
        const PresumTerm* d_pt = upload(mem, pterms, s);
        const GrowItem* d_items = upload(mem, items, s);
        const int32_t* d_ti = upload(mem, t_items, s);
        const GrowOut* d_outs = upload(mem, outs, s);
        try {
            phase("uploads");
            HIPCHK(launch_grow_presum(d_pb, (int)pblocks.size(), zmax, d_pt, data, d_z, s));
            phase("pre-sums");
            HIPCHK(launch_grow_renorm(d_items, d_ti, (int)t_items.size(), max_t, d_outs, (int)outs.size(), max_out, data,
                                      d_z, d_o, d_t, d_out, s));
            phase("O^T Z O (two passes)");
            ob->data.resize((size_t)out_len);
            download(ob->data.data(), d_out, out_len, s);
            phase("download");
        } catch (...) {
            (void)hipStreamSynchronize(s);
            throw;
        }
    }
    // the C description of the new block
    for (size_t g = 0; g < ob->ops.size(); ++g) {
        dmrg_op& op = ob->ops[g];
        op.n_blk = (int32_t)ob->so[g].size();
        op.sec_out = ob->so[g].data();
        op.sec_in = ob->si[g].data();
        op.off = ob->off[g].data();
    }
    ob->b.n_sec = (int32_t)ob->dim.size();
    ob->b.qn = ob->qn.data();
    ob->b.dim = ob->dim.data();
    ob->b.n_ops = (int32_t)ob->ops.size();
    ob->b.ops = ob->ops.data();
    ob->b.data = ob->data.data();
    ob->b.n_data = (int64_t)ob->data.size();
    dmrg_block* res = &ob->b;
    {
        std::lock_guard<std::mutex> lock(g_blocks_mu);
        g_blocks[res] = ob;
    }
    owned.release();
    return res;
}

}  // namespace dmrg

extern "C" void dmrg_block_free(dmrg_block* b) {
    if (!b) return;
    dmrg::OwnedBlock* ob = nullptr;
    {
        std::lock_guard<std::mutex> lock(dmrg::g_blocks_mu);
        auto it = dmrg::g_blocks.find(b);
        if (it == dmrg::g_blocks.end()) return;           // not a library-created block: nothing to do
        ob = it->second;
        dmrg::g_blocks.erase(it);
    }
    delete ob;
}
