// Launch planning of the two-site H.psi (Eq. dgemm, Section 2.2.1): the owner-computes task list of
// a handle cut into balanced work items for each kernel path -- FP64 one-wavefront tiles, the FP64
// LDS-staged kernel, the split LDS-staged row-mode and task-mode kernels, the two-pass large-block
// path in both precisions -- with ordered reductions of the partial tiles of cut items (no atomics),
// part tags for the part masks of merged handles, and the tiled operator copies these kernels read.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dmrg.h"
#include "host_common.h"
#include "internal.h"
#include "hop.h"
#include "plan.h"

namespace dmrg {

namespace {


// Merged problem (dmrg_hop_combine) that holds coefficient `off`.
int32_t part_of(const dmrg_hop& H, int64_t off) {
    return (int32_t)(std::upper_bound(H.part_coeff.begin(), H.part_coeff.end(), off) - H.part_coeff.begin()) - 1;
}
// Tag work records (items, reductions) with the merged problem of their target, for part masks.
template <class R>
void tag_parts(const dmrg_hop& H, std::vector<R>& recs) {
    for (auto& r : recs) r.part = H.n_parts > 1 ? part_of(H, r.y_off) : 0;
}

// Cost caps of work items. A plan cuts the task list of a tile into items of at most `cap` cost
// units, with cap = total / (target item count). A merged handle sets the cap of each problem from
// that problem's own total (tune_part_items), as its own handle would: when a part mask leaves only
// a few problems running, their items are as fine as in their own plans and still fill the GPU.
struct CostCaps {
    const dmrg_hop& H;
    std::vector<double> total;
    explicit CostCaps(const dmrg_hop& h) : H(h), total(h.n_parts > 1 && h.tune_part_items ? h.n_parts : 1, 0.0) {}
    size_t slot(int j) const { return total.size() > 1 ? (size_t)part_of(H, H.blk_off[j]) : 0; }
    void add(int j, double c) { total[slot(j)] += c; }
    double cap(int j, int items, double floor) const {
        return std::max(total[slot(j)] / std::max(1, items), floor);
    }
};

template <class T>
T* plan_alloc(dmrg_hop& H, size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    HIPCHK(hipMalloc(&p, n * sizeof(T)));
    H.plan_allocations.push_back(p);
    H.plan_bytes += (int64_t)(n * sizeof(T));
    return static_cast<T*>(p);
}

// Bytes of a matrix definition as stored in the pool (all its sector blocks, padded).
double mat_bytes(const dmrg_hop& H, int m) { return m < 0 ? 0.0 : H.mats[m].bytes; }

// Launch plan of H.psi: packed input layout, phases, work items, reductions (see internal.h).
//  * Phases: the distinct (left matrix, right matrix) pairs are sorted by (right, left) and cut into
//    groups of about kCacheBudget bytes of operators, so that the operators of one phase stay in
//    the last-level cache while all target tiles are updated.
//  * Items: in each phase every output tile (16 or 32 rows x up to 16 * tune_max_tq columns) gets
//    the phase's tasks of its target block, cut into chunks of bounded MFMA cost (about
//    tune_items items per matvec); a tile split over several chunks writes partial tiles that the
//    phase's reduction adds in order.
void build_plan_core(dmrg_hop& H, hipStream_t s, const std::vector<char>* only, bool split_bufs, dmrg::HpsiPlan& plan,
                     std::vector<dmrg::HpsiLaunch>& launches_out, std::vector<dmrg::HpsiPhase>& phases_out,
                     const std::vector<char>* task_only = nullptr) {
    // tasks of this plan: those of the targets in `only` (all without it) that `task_only` keeps
    auto keep = [&](size_t t) {
        return (!only || (*only)[H.tasks[t].j]) && (!task_only || (*task_only)[t]);
    };
    constexpr double kCacheBudget = 96.0 * 1024 * 1024;
    // packed input layout: every psi block padded to multiples of 32 in both directions
    std::vector<dmrg::PackBlock> packs;
    std::vector<int64_t> pk_off(H.blk.size());
    int64_t psize = 0;
    for (size_t i = 0; i < H.blk.size(); ++i) {
        int pa = dmrg::ld_of(H.blk_ma[i]), pd = dmrg::ld_of(H.blk_md[i]);
        pk_off[i] = psize;
        packs.push_back({H.blk_off[i], psize, H.blk_ma[i], H.blk_md[i], pa, pd});
        psize += (int64_t)pa * pd;
    }
    // phases over (left, right) matrix pairs
    std::map<std::pair<int, int>, int> pair_phase;
    {
        std::vector<std::pair<int, int>> pairs;
        for (size_t t = 0; t < H.tasks.size(); ++t)
            if (keep(t)) pairs.push_back({H.tasks[t].rm, H.tasks[t].lm});
        std::sort(pairs.begin(), pairs.end());
        pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
        std::vector<double> pb(pairs.size());
        double total = 0.0;
        for (size_t k = 0; k < pairs.size(); ++k) { pb[k] = mat_bytes(H, pairs[k].first) + mat_bytes(H, pairs[k].second); total += pb[k]; }
        int np = H.tune_phases > 0 ? H.tune_phases : std::max(1, (int)std::ceil(total / kCacheBudget));
        np = std::min<int>(np, std::max<size_t>(1, pairs.size()));
        double cum = 0.0;
        for (size_t k = 0; k < pairs.size(); ++k) {
            int ph = std::min(np - 1, (int)(np * (cum + 0.5 * pb[k]) / std::max(total, 1.0)));
            pair_phase[{pairs[k].second, pairs[k].first}] = ph;
            cum += pb[k];
        }
        plan.n_phases = np;
    }
    const int np = plan.n_phases;
    // device tasks, grouped per target block and phase (stable: source order kept inside)
    std::vector<dmrg::Task> dtasks;
    dtasks.reserve(H.tasks.size());
    // trange[j * np + ph] = task range of target j in phase ph
    std::vector<std::pair<int32_t, int32_t>> trange(H.blk.size() * np, {0, 0});
    auto r16 = [](int m) { return (m + 15) / 16 * 16; };
    {
        size_t t = 0;
        std::vector<std::vector<size_t>> by_phase(np);
        for (size_t j = 0; j < H.blk.size(); ++j) {
            for (auto& v : by_phase) v.clear();
            while (t < H.tasks.size() && H.tasks[t].j == (int)j) {
                if (keep(t)) by_phase[pair_phase[{H.tasks[t].lm, H.tasks[t].rm}]].push_back(t);
                ++t;
            }
            for (int ph = 0; ph < np; ++ph) {
                int32_t tb = (int32_t)dtasks.size();
                for (size_t k : by_phase[ph]) {
                    const auto& ht = H.tasks[k];
                    int64_t ao = ht.lm >= 0 ? H.mats[ht.lm].pool_of_in[H.blk[ht.i][0]] : -1;
                    int64_t bo = ht.rm >= 0 ? H.mats[ht.rm].pool_of_in[H.blk[ht.i][3]] : -1;
                    const int ma = H.blk_ma[ht.i], md = H.blk_md[ht.i];
                    dtasks.push_back({pk_off[ht.i], ao, bo, ht.f, dmrg::ld_of(ma), dmrg::ld_of(md), r16(ma), r16(md)});
                }
                trange[j * np + ph] = {tb, (int32_t)dtasks.size()};
            }
        }
    }
    auto task_cost = [&](const dmrg::Task& T, int tp, int tq) -> double {
        double c = 8.0;                                   // per-task overhead
        if (T.a_off < 0 && T.b_off < 0) return c + 1.0;
        if (T.b_off < 0) return c + (double)(T.ka / 4) * tp * tq;
        if (T.a_off < 0) return c + (double)(T.kd / 4) * tp * tq;
        return c + (double)(T.kd / 16) * (tp * (T.ka / 4) + 4.0 * tp * tq);
    };
    struct Tile { int j, r0, c0, tp, tq; };
    std::vector<Tile> tiles;
    double max_task = 0.0;
    CostCaps caps(H);
    const int tile_cols = 16 * H.tune_max_tq;
    for (size_t j = 0; j < H.blk.size(); ++j) {
        if (only && !(*only)[j]) continue;
        if (trange[j * np].first == trange[j * np + np - 1].second) continue;   // no task kept
        int mj = H.blk_ma[j], nj = H.blk_md[j];
        for (int r0 = 0; r0 < mj; r0 += dmrg::kTileRows)
            for (int c0 = 0; c0 < nj; c0 += tile_cols) {
                int tp = mj - r0 <= 16 ? 1 : 2;
                int tq = (std::min(tile_cols, nj - c0) + 15) / 16;
                for (int32_t t = trange[j * np].first; t < trange[j * np + np - 1].second; ++t) {
                    double tc = task_cost(dtasks[t], tp, tq);
                    caps.add((int)j, tc);
                    max_task = std::max(max_task, tc);
                }
                tiles.push_back({(int)j, r0, c0, tp, tq});
            }
    }
    std::vector<dmrg::Item> all_items;
    std::vector<dmrg::Reduce> all_red;
    launches_out.clear();
    phases_out.clear();
    int64_t part_max = 0;
    for (int ph = 0; ph < np; ++ph) {
        std::vector<dmrg::Item> items;
        std::vector<double> icost;
        std::vector<int> iclass, igroup;
        std::vector<dmrg::Reduce> reduces;
        int64_t part_size = 0;
        for (const Tile& T : tiles) {
            const int j = T.j;
            const auto tr = trange[j * np + ph];
            if (tr.first == tr.second) continue;
            std::vector<std::pair<int32_t, int32_t>> chunks;
            std::vector<double> ccost;
            int32_t b = tr.first;
            double c = 0.0;
            const double cmax = std::max(caps.cap(j, H.tune_items, 256.0), max_task);
            for (int32_t t = tr.first; t < tr.second; ++t) {
                double tc = task_cost(dtasks[t], T.tp, T.tq);
                if (c + tc > cmax && t > b) { chunks.push_back({b, t}); ccost.push_back(c); b = t; c = 0.0; }
                c += tc;
            }
            chunks.push_back({b, tr.second});
            ccost.push_back(c);
            const int cls = (T.tp - 1) * 8 + (T.tq - 1);
            const int tm = 16 * T.tp, tn = 16 * T.tq;
            const int grp = H.blk[j][0];                     // target left sector: shares left operators
            if (chunks.size() == 1) {
                items.push_back({H.blk_off[j], -1, H.blk_ma[j], H.blk_md[j], T.r0, T.c0, chunks[0].first, chunks[0].second});
                icost.push_back(ccost[0]);
                iclass.push_back(cls);
                igroup.push_back(grp);
            } else {
                reduces.push_back({H.blk_off[j], part_size, H.blk_ma[j], H.blk_md[j], T.r0, T.c0, tm, tn,
                                   (int32_t)chunks.size(), 0});
                for (size_t k = 0; k < chunks.size(); ++k) {
                    items.push_back({H.blk_off[j], part_size, H.blk_ma[j], H.blk_md[j], T.r0, T.c0, chunks[k].first,
                                     chunks[k].second});
                    part_size += (int64_t)tm * tn;
                    icost.push_back(ccost[k]);
                    iclass.push_back(cls);
                    igroup.push_back(grp);
                }
            }
        }
        part_max = std::max(part_max, part_size);
        // Launch order inside a tile class. 0: heaviest first. 1: target order. 2: XCD-aware -- items
        // whose targets share the left sector (hence the left operators) are placed at positions of
        // the same residue mod 8, i.e. on the same XCD and its L2, groups balanced over the 8 XCDs.
        std::vector<int> perm(items.size());
        for (size_t i = 0; i < perm.size(); ++i) perm[i] = (int)i;
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
            if (iclass[a] != iclass[b]) return iclass[a] < iclass[b];
            if (H.tune_order == 0) return icost[a] > icost[b];
            if (H.tune_order == 2 && igroup[a] != igroup[b]) return igroup[a] < igroup[b];
            return false;
        });
        if (H.tune_order == 2) {
            const int nx = 8;
            std::vector<int> out;
            out.reserve(perm.size());
            size_t c0 = 0;
            while (c0 < perm.size()) {
                size_t c1 = c0;
                while (c1 < perm.size() && iclass[perm[c1]] == iclass[perm[c0]]) ++c1;
                std::map<int, std::vector<int>> grp;
                std::map<int, double> gcost;
                for (size_t i = c0; i < c1; ++i) { grp[igroup[perm[i]]].push_back(perm[i]); gcost[igroup[perm[i]]] += icost[perm[i]]; }
                std::vector<std::pair<double, int>> order;
                for (auto& kv : gcost) order.push_back({-kv.second, kv.first});
                std::sort(order.begin(), order.end());
                std::vector<double> load(nx, 0.0);
                std::vector<std::vector<int>> lane(nx);
                for (auto& og : order) {
                    int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                    load[x] -= og.first;
                    for (int it : grp[og.second]) lane[x].push_back(it);
                }
                std::vector<size_t> pos(nx, 0);
                size_t left = c1 - c0;
                for (size_t p = 0; left > 0; ++p) {
                    int x = (int)(p % nx);
                    if (pos[x] < lane[x].size()) { out.push_back(lane[x][pos[x]++]); --left; }
                    else {
                        int best = -1;
                        size_t rem = 0;
                        for (int y = 0; y < nx; ++y) if (lane[y].size() - pos[y] > rem) { rem = lane[y].size() - pos[y]; best = y; }
                        out.push_back(lane[best][pos[best]++]);
                        --left;
                    }
                }
                c0 = c1;
            }
            perm = out;
        }
        dmrg::HpsiPhase P;
        P.launch_begin = (int)launches_out.size();
        const int base = (int)all_items.size();
        for (size_t i = 0; i < perm.size(); ++i) {
            all_items.push_back(items[perm[i]]);
            const int cls = iclass[perm[i]];
            if (launches_out.size() == (size_t)P.launch_begin || launches_out.back().cls != cls)
                launches_out.push_back({cls, base + (int)i, 0});
            launches_out.back().item_count++;
        }
        P.launch_end = (int)launches_out.size();
        P.reduce_begin = (int)all_red.size();
        for (const auto& r : reduces) all_red.push_back(r);
        P.reduce_end = (int)all_red.size();
        phases_out.push_back(P);
    }
    if (!only) H.n_items = (int)all_items.size();
    H.n_dev_tasks = (int64_t)dtasks.size();
    if (const char* e = std::getenv("DMRG_PLAN_TRACE"))
        if (e[0] == '1')
            std::fprintf(stderr, "[dmrg plan] phases %d items %zu launches %zu reduces %zu partial %.1f MB packed %.1f MB\n",
                         np, all_items.size(), H.launches.size(), all_red.size(), part_max * 8e-6, psize * 8e-6);
    tag_parts(H, all_items);
    tag_parts(H, all_red);
    dmrg::Item* d_items = plan_alloc<dmrg::Item>(H, all_items.size());
    dmrg::Task* d_tasks = plan_alloc<dmrg::Task>(H, dtasks.size());
    dmrg::Reduce* d_red = plan_alloc<dmrg::Reduce>(H, all_red.size());
    dmrg::PackBlock* d_packs = plan_alloc<dmrg::PackBlock>(H, packs.size());
    HIPCHK(hipMemcpyAsync(d_items, all_items.data(), all_items.size() * sizeof(all_items[0]), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_tasks, dtasks.data(), dtasks.size() * sizeof(dtasks[0]), hipMemcpyHostToDevice, s));
    if (!all_red.empty())
        HIPCHK(hipMemcpyAsync(d_red, all_red.data(), all_red.size() * sizeof(all_red[0]), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_packs, packs.data(), packs.size() * sizeof(packs[0]), hipMemcpyHostToDevice, s));
    if (!only) H.d_tasks = d_tasks;
    plan.items = d_items;
    plan.reduces = d_red;
    plan.tasks = d_tasks;
    plan.partial = plan_alloc<double>(H, (size_t)std::max<int64_t>(part_max, 1) * H.vec_step);
    plan.partial_size = part_max;
    plan.launches = launches_out.data();
    plan.phases = phases_out.data();
    plan.packs = d_packs;
    plan.n_packs = (int)packs.size();
    plan.packed_size = psize;
    plan.xp = plan_alloc<double>(H, (size_t)psize * H.vec_step);
    if (split_bufs) {
        plan.xr_hi = plan_alloc<uint16_t>(H, (size_t)psize * H.vec_step);
        plan.xr_lo = plan_alloc<uint16_t>(H, (size_t)psize * H.vec_step);
        plan.xt_hi = plan_alloc<uint16_t>(H, (size_t)psize * H.vec_step);
        plan.xt_lo = plan_alloc<uint16_t>(H, (size_t)psize * H.vec_step);
    }
    HIPCHK(hipStreamSynchronize(s));
}

// Launch plan of the split kernels of hpsi_lds.hip. The tasks of every target block whose own and
// sources' padded dimensions are at most 96 are divided into small tasks (source one 32 x 32 tile)
// for the task-mode kernel and the others for the LDS-staged row-mode kernel; both lists keep the
// source order. Row-mode items cover the whole target (all rows and columns), task-mode items a row
// block of one or two row tiles; each list is cut into items of bounded cost, and a target row block
// covered by several items of one kind gets partial tiles that a reduction adds in item order.
// Targets with larger blocks (own, or every source with tune_split_task_route = 0) are flagged in
// `fallback`, and with them the tasks in `fb_task`: those the other paths (two-pass or one-wave) run.
// With tune_split_task_route, a target within the stages keeps its tasks whose source fits them too
// and only those with a larger source fall back, so one target can take both paths (each adds into y).
void build_lds_plan(dmrg_hop& H, hipStream_t s, std::vector<char>& fallback, std::vector<char>& fb_task) {
    const size_t nb = H.blk.size();
    fallback.assign(nb, 0);
    fb_task.assign(H.tasks.size(), 0);
    std::vector<int64_t> pk_off(nb);
    std::vector<dmrg::PackBlock> packs;
    int64_t psize = 0;
    for (size_t i = 0; i < nb; ++i) {
        int pa = dmrg::ld_of(H.blk_ma[i]), pd = dmrg::ld_of(H.blk_md[i]);
        pk_off[i] = psize;
        packs.push_back({H.blk_off[i], psize, H.blk_ma[i], H.blk_md[i], pa, pd});
        psize += (int64_t)pa * pd;
    }
    auto ident = [&](int p) -> int64_t {
        int k = p / 32 - 1;
        if (k < 0 || k >= (int)H.ident_off.size()) throw Error(DMRG_ERR_ARG, "internal: no tiled identity block");
        return H.ident_off[k];
    };
    // one run of tasks of one kernel kind for one target row block
    struct Run { int j, kind, cls, r0, c0, nr, tq; int32_t tb, te; };
    std::vector<dmrg::LTask> lt;
    lt.reserve(H.tasks.size());
    std::vector<Run> runs;
    auto row_cost = [](const dmrg::LTask& L, int tp, int tq, bool new_src) {
        return 3.0 * L.pd32 * (2.0 * L.pa32 * tp + tq * tp) + 24.0 + (new_src ? 2.0 * L.pd32 * L.pa32 : 0.0);
    };
    auto small_cost = [](int nr, int tq) { return 3.0 * (2.0 * nr + nr * tq) + 24.0; };
    CostCaps caps(H);
    size_t k = 0;
    for (size_t j = 0; j < nb; ++j) {
        size_t kb = k;
        while (k < H.tasks.size() && H.tasks[k].j == (int)j) ++k;
        if (k == kb) continue;
        const int own = std::max(dmrg::ld_of(H.blk_ma[j]), dmrg::ld_of(H.blk_md[j]));
        auto src_dim = [&](size_t t) {
            const int i = H.tasks[t].i;
            return std::max(dmrg::ld_of(H.blk_ma[i]), dmrg::ld_of(H.blk_md[i]));
        };
        int smax = own;
        for (size_t t = kb; t < k; ++t) smax = std::max(smax, src_dim(t));
        if (own > 96 || (smax > 96 && !H.tune_split_task_route)) {
            fallback[j] = 1;
            for (size_t t = kb; t < k; ++t) fb_task[t] = 1;
            continue;
        }
        if (smax > 96) {                              // per-task routing: the larger sources fall back
            fallback[j] = 1;
            for (size_t t = kb; t < k; ++t) fb_task[t] = src_dim(t) > 96;
        }
        const int nrt = dmrg::rows_of(H.blk_ma[j]) / 16, tq = dmrg::rows_of(H.blk_md[j]) / 16;
        std::vector<dmrg::LTask> big, small;
        int big_s = 32;
        std::vector<size_t> order;
        for (size_t t = kb; t < k; ++t)
            if (!fb_task[t]) order.push_back(t);
        if (H.tune_lds_task_order == 1)   // operator-pair order (same across targets) instead of source order
            std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
                const auto &a = H.tasks[x], &b = H.tasks[y];
                if (a.lm != b.lm) return a.lm < b.lm;
                return a.rm < b.rm;
            });
        for (size_t t : order) {
            const auto& ht = H.tasks[t];
            const int a = H.blk[ht.i][0], d = H.blk[ht.i][3];
            const int pa = dmrg::ld_of(H.blk_ma[ht.i]), pd = dmrg::ld_of(H.blk_md[ht.i]);
            dmrg::LTask L;
            L.x_off = 2 * pk_off[ht.i];
            L.a_off = ht.lm >= 0 ? 2 * H.mats[ht.lm].pool_of_in[a] : ident(pa);
            L.b_off = ht.rm >= 0 ? 2 * H.mats[ht.rm].pool_of_in[d] : ident(pd);
            L.f = (float)ht.f;
            L.pa32 = (int16_t)(pa / 32);
            L.pd32 = (int16_t)(pd / 32);
            if (L.pa32 == 1 && L.pd32 == 1 && H.tune_small_mode) small.push_back(L);
            else { big.push_back(L); big_s = std::max({big_s, pa, pd}); }
        }
        (void)big_s;
        if (!big.empty()) {
            // tasks that fit 64-wide stages (source and target columns <= 64) -> S = 64 run, rest -> S = 96
            const int tp = nrt > dmrg::kLdsWaves ? 2 : 1;
            std::vector<dmrg::LTask> b64, b96;
            for (const auto& L : big)
                (L.pa32 <= 2 && L.pd32 <= 2 && tq <= 4 && H.tune_lds_split64 ? b64 : b96).push_back(L);
            for (int S : {64, 96}) {
                const auto& v = S == 64 ? b64 : b96;
                if (v.empty()) continue;
                Run R{(int)j, S == 64 ? 0 : 1, (S == 64 ? 0 : 2) + (tp - 1), 0, 0, nrt, tq, (int32_t)lt.size(), 0};
                int64_t px = -1;
                for (const auto& L : v) {
                    lt.push_back(L);
                    caps.add((int)j, row_cost(L, tp, tq, L.x_off != px));
                    px = L.x_off;
                }
                R.te = (int32_t)lt.size();
                runs.push_back(R);
            }
        }
        if (!small.empty()) {
            const int tb = (int32_t)lt.size();
            for (const auto& L : small) lt.push_back(L);
            const int te = (int32_t)lt.size();
            // classes (1,2) (2,2) (1,4); targets wider than 4 column tiles get column blocks
            const int NQ = tq <= 2 && H.tune_small_nq <= 2 ? 2 : 4;
            const int NR = NQ == 2 && nrt > 1 && H.tune_small_nr > 1 ? 2 : 1;
            const int cls = NQ == 4 ? 2 : NR - 1;
            for (int r = 0; r < nrt; r += NR)
                for (int c = 0; c < tq; c += NQ) {
                    const int nr = std::min(NR, nrt - r), nq = std::min(NQ, tq - c);
                    runs.push_back({(int)j, 2, cls, 16 * r, 16 * c, nr, nq, tb, te});
                    caps.add((int)j, (te - tb) * small_cost(nr, nq));
                }
        }
    }
    H.lplan = dmrg::LdsPlan{};
    struct It { dmrg::Item item; double cost; int kind, cls; };
    std::vector<It> its;
    std::vector<dmrg::Reduce> reds_k[dmrg::kReduceKinds];
    int64_t part = 0;
    for (const Run& R : runs) {
        const int tp = R.kind < 2 && R.nr > dmrg::kLdsWaves ? 2 : 1;
        std::vector<std::pair<int32_t, int32_t>> chunks;
        std::vector<double> ccost;
        int32_t b = R.tb;
        double c = 0.0;
        int64_t px = -1;
        const double cmax = caps.cap(R.j, H.tune_lds_items, 600.0);
        for (int32_t t = R.tb; t < R.te; ++t) {
            const double tc = R.kind < 2 ? row_cost(lt[t], tp, R.tq, lt[t].x_off != px || t == b) : small_cost(R.nr, R.tq);
            px = lt[t].x_off;
            if (c + tc > cmax && t > b) { chunks.push_back({b, t}); ccost.push_back(c); b = t; c = 0.0; }
            c += tc;
        }
        chunks.push_back({b, R.te});
        ccost.push_back(c);
        const int j = R.j;
        const int tm = 16 * R.nr, tn = 16 * R.tq;
        if (chunks.size() == 1) {
            its.push_back({{H.blk_off[j], -1, H.blk_ma[j], H.blk_md[j], R.r0, R.c0, chunks[0].first, chunks[0].second},
                           ccost[0], R.kind, R.cls});
        } else {
            reds_k[R.kind].push_back({H.blk_off[j], part, H.blk_ma[j], H.blk_md[j], R.r0, R.c0, tm, tn,
                                      (int32_t)chunks.size(), 0});
            for (size_t q = 0; q < chunks.size(); ++q) {
                its.push_back({{H.blk_off[j], part, H.blk_ma[j], H.blk_md[j], R.r0, R.c0, chunks[q].first,
                                chunks[q].second},
                               ccost[q], R.kind, R.cls});
                part += (int64_t)tm * tn;
            }
        }
    }
    // launch order: row-mode classes, then task-mode classes; heaviest item first inside a class
    for (It& x : its) x.kind = x.kind < 2 ? 0 : 1;
    std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) {
        if (a.kind != b.kind) return a.kind < b.kind;
        if (a.cls != b.cls) return a.cls < b.cls;
        return a.cost > b.cost;
    });
    if (H.tune_lds_order == 2 && H.n_parts > 1) {
        // merged problems: inside a class, the items of one problem stay together (heaviest first),
        // so that the workgroups running at one time share that problem's operators in the caches
        auto part_of = [&](int64_t y_off) {
            return (int)(std::upper_bound(H.part_coeff.begin(), H.part_coeff.end(), y_off) - H.part_coeff.begin());
        };
        std::stable_sort(its.begin(), its.end(), [&](const It& a, const It& b) {
            if (a.kind != b.kind) return a.kind < b.kind;
            if (a.cls != b.cls) return a.cls < b.cls;
            const int pa = part_of(a.item.y_off), pb = part_of(b.item.y_off);
            if (pa != pb) return pa < pb;
            return a.cost > b.cost;
        });
    }
    if (H.tune_lds_order == 1) {
        // XCD-aware: workgroups are dealt to the 8 XCDs round-robin, so items at positions of one
        // residue mod 8 share an L2. Items of targets with the same left sector (which read the same
        // left operator blocks) are kept on one XCD; sectors are balanced over the XCDs by cost.
        constexpr int nx = 8;
        size_t c0 = 0;
        std::vector<It> out;
        out.reserve(its.size());
        while (c0 < its.size()) {
            size_t c1 = c0;
            while (c1 < its.size() && its[c1].kind == its[c0].kind && its[c1].cls == its[c0].cls) ++c1;
            std::map<int, std::vector<size_t>> grp;
            std::map<int, double> gcost;
            for (size_t i = c0; i < c1; ++i) {
                const int a = H.blk[std::lower_bound(H.blk_off.begin(), H.blk_off.end(), its[i].item.y_off) -
                                    H.blk_off.begin()][0];
                grp[a].push_back(i);
                gcost[a] += its[i].cost;
            }
            std::vector<std::pair<double, int>> gorder;
            for (auto& kv : gcost) gorder.push_back({-kv.second, kv.first});
            std::sort(gorder.begin(), gorder.end());
            std::vector<double> load(nx, 0.0);
            std::vector<std::vector<size_t>> lane(nx);
            for (auto& og : gorder) {
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[x] -= og.first;
                for (size_t i : grp[og.second]) lane[x].push_back(i);
            }
            std::vector<size_t> pos(nx, 0);
            for (size_t left = c1 - c0, p = 0; left > 0; ++p) {
                int x = (int)(p % nx);
                if (pos[x] >= lane[x].size()) {
                    size_t rem = 0;
                    for (int y2 = 0; y2 < nx; ++y2)
                        if (lane[y2].size() - pos[y2] > rem) { rem = lane[y2].size() - pos[y2]; x = y2; }
                }
                out.push_back(its[lane[x][pos[x]++]]);
                --left;
            }
            c0 = c1;
        }
        its.swap(out);
    }
    std::vector<dmrg::Item> items;
    items.reserve(its.size());
    int cnt_row[dmrg::kLdsClasses] = {0}, cnt_small[dmrg::kSmallClasses] = {0};
    for (const It& x : its) {
        items.push_back(x.item);
        if (x.kind == 0) cnt_row[x.cls]++; else cnt_small[x.cls]++;
    }
    H.lplan.cls_begin[0] = 0;
    for (int c = 0; c < dmrg::kLdsClasses; ++c) H.lplan.cls_begin[c + 1] = H.lplan.cls_begin[c] + cnt_row[c];
    H.lplan.small_begin[0] = H.lplan.cls_begin[dmrg::kLdsClasses];
    for (int c = 0; c < dmrg::kSmallClasses; ++c) H.lplan.small_begin[c + 1] = H.lplan.small_begin[c] + cnt_small[c];
    H.n_fallback_targets = 0;
    for (char f : fallback) H.n_fallback_targets += f;
    std::vector<dmrg::Reduce> reds;
    H.lplan.red_begin[0] = 0;
    for (int kk = 0; kk < dmrg::kReduceKinds; ++kk) {
        int mx = 1;
        for (const auto& r : reds_k[kk]) mx = std::max(mx, r.tm * r.tn);
        H.lplan.red_chunks[kk] = (mx + 255) / 256;
        reds.insert(reds.end(), reds_k[kk].begin(), reds_k[kk].end());
        H.lplan.red_begin[kk + 1] = (int)reds.size();
    }
    tag_parts(H, items);
    tag_parts(H, reds);
    dmrg::Item* d_items = plan_alloc<dmrg::Item>(H, items.size());
    dmrg::LTask* d_lt = plan_alloc<dmrg::LTask>(H, lt.size());
    dmrg::Reduce* d_red = plan_alloc<dmrg::Reduce>(H, reds.size());
    dmrg::PackBlock* d_packs = plan_alloc<dmrg::PackBlock>(H, packs.size());
    if (!items.empty())
        HIPCHK(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(items[0]), hipMemcpyHostToDevice, s));
    if (!lt.empty()) HIPCHK(hipMemcpyAsync(d_lt, lt.data(), lt.size() * sizeof(lt[0]), hipMemcpyHostToDevice, s));
    if (!reds.empty()) HIPCHK(hipMemcpyAsync(d_red, reds.data(), reds.size() * sizeof(reds[0]), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_packs, packs.data(), packs.size() * sizeof(packs[0]), hipMemcpyHostToDevice, s));
    H.lplan.items = d_items;
    H.lplan.tasks = d_lt;
    H.lplan.reduces = d_red;

    H.lplan.partial_size = part;
    H.lplan.partial = plan_alloc<double>(H, (size_t)std::max<int64_t>(part, 1) * H.vec_step);
    H.lplan.packs = d_packs;
    H.lplan.n_packs = (int)packs.size();
    H.lplan.xt_size = 2 * psize;
    H.lplan.xt = plan_alloc<uint16_t>(H, (size_t)2 * psize * H.vec_step);
    H.lplan.prefetch_mask = H.tune_lds_pf;
    H.lplan.six_wave_mask = H.tune_lds_w6;
    H.lplan.copy_wave_mask = H.tune_lds_cw;
    if (const char* e = std::getenv("DMRG_PLAN_TRACE"))
        if (e[0] == '1') {
            std::fprintf(stderr, "[dmrg lds plan] items %zu row classes", items.size());
            for (int c = 0; c < dmrg::kLdsClasses; ++c) std::fprintf(stderr, " %d", cnt_row[c]);
            std::fprintf(stderr, " small classes");
            for (int c = 0; c < dmrg::kSmallClasses; ++c) std::fprintf(stderr, " %d", cnt_small[c]);
            std::fprintf(stderr, " reduces %zu partial %.1f MB fallback %d\n", reds.size(), part * 8e-6,
                         H.n_fallback_targets);
        }
    HIPCHK(hipStreamSynchronize(s));
}

// Launch plan of the two-pass large-block path for the targets flagged in `big`, split (hpsi_big.hip,
// fp64 = false: 16 x 32 hi/lo tiles, u16 offsets) or FP64 (hpsi_big64.hip: 16 x 16 tiles, offsets
// in doubles). Targets are grouped into chunks whose T buffers (one per task: target rows x source
// columns, tiled) stay below the T budget; per chunk, pass 1 has one group per (task, 8 row tiles,
// 128 T columns), consecutive groups packed into workgroups of about tune_big_stages1 k steps, and
// pass 2 one item per (target, 8 row tiles, 8 column tiles, task range), the task lists cut into
// items of about tune_big_stages k steps whose partial tiles a reduction adds in order.
void build_big_plan(dmrg_hop& H, hipStream_t s, const std::vector<char>& big, bool fp64,
                    const std::vector<char>* task_keep = nullptr) {
    auto kept = [&](size_t k) { return !task_keep || (*task_keep)[k]; };
    const int unit = fp64 ? 16 : 32;                 // k-tile width
    const int64_t esc = fp64 ? 1 : 2;                // tiled-array elements per pool element
    const int64_t tile_el = fp64 ? 256 : dmrg::kTileU16;
    const int64_t kBigTBudget = (int64_t)H.tune_big_tbudget_mb << (fp64 ? 18 : 19);   // T elements per chunk
    dmrg::BigPlan& plan = fp64 ? H.bplan64 : H.bplan;
    std::vector<dmrg::BigChunk>& chunks = fp64 ? H.big_chunks64 : H.big_chunks;
    const std::vector<int64_t>& ident_tab = fp64 ? H.ident64_off : H.ident_off;
    plan = dmrg::BigPlan{};
    chunks.clear();
    const size_t nb = H.blk.size();
    std::vector<int64_t> pk_off(nb);
    {
        int64_t ps = 0;
        for (size_t i = 0; i < nb; ++i) { pk_off[i] = ps; ps += (int64_t)dmrg::ld_of(H.blk_ma[i]) * dmrg::ld_of(H.blk_md[i]); }
    }
    auto ident = [&](int p) -> int64_t {
        const int k = p / 32 - 1;
        if (k < 0 || k >= (int)ident_tab.size()) return -1;
        return ident_tab[k];
    };
    std::vector<dmrg::BigT1> t1;
    std::vector<dmrg::BigT2> t2;
    std::vector<dmrg::Item> items;
    std::vector<dmrg::Reduce> reds;
    int64_t part_max = 0, tbuf_max = 0;
    int red_max = 1;
    // per target: its task range in H.tasks
    std::vector<std::pair<size_t, size_t>> trange(nb, {0, 0});
    for (size_t k = 0; k < H.tasks.size();) {
        size_t e = k;
        while (e < H.tasks.size() && H.tasks[e].j == H.tasks[k].j) ++e;
        trange[H.tasks[k].j] = {k, e};
        k = e;
    }
    dmrg::BigChunk cur{0, 0, 0, 0, 0, 0};
    int64_t tsize = 0, part = 0;
    std::vector<int32_t> t1_ranges;
    int32_t g_first = 0;
    std::vector<int> chunk_targets;
    auto close_chunk = [&]() {
        if (chunk_targets.empty()) return;
        // pass-1 workgroups: consecutive groups of the chunk with about tune_big_stages1 k steps each
        cur.t1_begin = (int)t1_ranges.size();
        {
            int c = 0;
            t1_ranges.push_back(g_first);
            for (int32_t gidx = g_first; gidx < (int32_t)t1.size(); ++gidx) {
                // a workgroup's groups belong to one merged problem (part masks skip whole workgroups)
                if (c >= H.tune_big_stages1 || (gidx > g_first && t1[gidx].part != t1[gidx - 1].part)) {
                    t1_ranges.push_back(gidx);
                    c = 0;
                }
                c += t1[gidx].pa32;
            }
            cur.t1_end = (int)t1_ranges.size();   // workgroups [t1_begin, t1_end); ranges has one more entry
            t1_ranges.push_back((int32_t)t1.size());
        }
        g_first = (int32_t)t1.size();
        cur.item_begin = (int)items.size();
        cur.red_begin = (int)reds.size();
        part = 0;
        for (int j : chunk_targets) {
            const int nrt = dmrg::rows_of(H.blk_ma[j]) / 16, nq = dmrg::rows_of(H.blk_md[j]) / 16;
            const int32_t b0 = H.big_t2_range[j].first, b1 = H.big_t2_range[j].second;
            for (int rb = 0; rb < nrt; rb += 8)
                for (int qb = 0; qb < nq; qb += 8) {
                    const int tn = 16 * std::min(8, nq - qb);
                    std::vector<std::pair<int32_t, int32_t>> cuts;
                    int32_t b = b0;
                    int c = 0;
                    for (int32_t t = b0; t < b1; ++t) {
                        if (c >= H.tune_big_stages && t > b) { cuts.push_back({b, t}); b = t; c = 0; }
                        c += t2[t].pd32;
                    }
                    cuts.push_back({b, b1});
                    if (cuts.size() == 1) {
                        items.push_back({H.blk_off[j], -1, H.blk_ma[j], H.blk_md[j], 16 * rb, 16 * qb, cuts[0].first,
                                         cuts[0].second});
                    } else {
                        reds.push_back({H.blk_off[j], part, H.blk_ma[j], H.blk_md[j], 16 * rb, 16 * qb, 128, tn,
                                        (int32_t)cuts.size(), 0});
                        red_max = std::max(red_max, 128 * tn);
                        for (auto& cp : cuts) {
                            items.push_back({H.blk_off[j], part, H.blk_ma[j], H.blk_md[j], 16 * rb, 16 * qb, cp.first,
                                             cp.second});
                            part += (int64_t)128 * tn;
                        }
                    }
                }
        }
        cur.item_end = (int)items.size();
        cur.red_end = (int)reds.size();
        part_max = std::max(part_max, part);
        tbuf_max = std::max(tbuf_max, tsize);
        chunks.push_back(cur);
        cur = dmrg::BigChunk{0, 0, 0, 0, 0, 0};
        chunk_targets.clear();
        tsize = 0;
    };
    H.big_t2_range.assign(nb, {0, 0});
    for (size_t j = 0; j < nb; ++j) {
        if (!big[j]) continue;
        const int nrt = dmrg::rows_of(H.blk_ma[j]) / 16;
        int64_t need = 0;
        for (size_t k = trange[j].first; k < trange[j].second; ++k)
            if (kept(k)) need += (int64_t)nrt * (dmrg::ld_of(H.blk_md[H.tasks[k].i]) / unit) * tile_el;
        if (need == 0) continue;                  // every task of the target runs elsewhere
        if (tsize > 0 && tsize + need > kBigTBudget) close_chunk();
        const int32_t b0 = (int32_t)t2.size();
        const size_t g_t1 = t1.size();
        const int32_t part_j = H.n_parts > 1 ? part_of(H, H.blk_off[j]) : 0;
        for (size_t k = trange[j].first; k < trange[j].second; ++k) {
            if (!kept(k)) continue;
            const auto& ht = H.tasks[k];
            const int a = H.blk[ht.i][0], d = H.blk[ht.i][3];
            const int pa = dmrg::ld_of(H.blk_ma[ht.i]), pd = dmrg::ld_of(H.blk_md[ht.i]);
            const int64_t a_off = ht.lm >= 0 ? esc * H.mats[ht.lm].pool_of_in[a] : ident(pa);
            const int64_t b_off = ht.rm >= 0 ? esc * H.mats[ht.rm].pool_of_in[d] : ident(pd);
            if (a_off < 0 || b_off < 0) throw Error(DMRG_ERR_ARG, "internal: no tiled identity block");
            const int64_t t_off = tsize;
            tsize += (int64_t)nrt * (pd / unit) * tile_el;
            const int ka = (H.blk_ma[ht.i] + unit - 1) / unit, kd = (H.blk_md[ht.i] + unit - 1) / unit;
            for (int rb = 0; rb < nrt; rb += 8)
                for (int jb = 0; jb < kd; jb += 128 / unit)
                    t1.push_back({esc * pk_off[ht.i], a_off, t_off, ht.f, (int16_t)(pa / unit),
                                  (int16_t)(pd / unit), (int16_t)nrt, (int16_t)rb, (int16_t)jb, 0, (int16_t)ka,
                                  (int16_t)kd});
            t2.push_back({t_off, b_off, pd / unit, kd});
        }
        H.big_t2_range[j] = {b0, (int32_t)t2.size()};
        for (size_t g = g_t1; g < t1.size(); ++g) t1[g].part = (int16_t)part_j;
        chunk_targets.push_back((int)j);
    }
    close_chunk();
    if (t1.empty()) return;
    dmrg::BigT1* d_t1 = plan_alloc<dmrg::BigT1>(H, t1.size());
    int32_t* d_t1r = plan_alloc<int32_t>(H, t1_ranges.size());
    HIPCHK(hipMemcpyAsync(d_t1r, t1_ranges.data(), t1_ranges.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    plan.t1_ranges = d_t1r;
    dmrg::BigT2* d_t2 = plan_alloc<dmrg::BigT2>(H, t2.size());
    tag_parts(H, items);
    tag_parts(H, reds);
    dmrg::Item* d_items = plan_alloc<dmrg::Item>(H, items.size());
    dmrg::Reduce* d_red = plan_alloc<dmrg::Reduce>(H, reds.size());
    HIPCHK(hipMemcpyAsync(d_t1, t1.data(), t1.size() * sizeof(t1[0]), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_t2, t2.data(), t2.size() * sizeof(t2[0]), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(items[0]), hipMemcpyHostToDevice, s));
    if (!reds.empty()) HIPCHK(hipMemcpyAsync(d_red, reds.data(), reds.size() * sizeof(reds[0]), hipMemcpyHostToDevice, s));
    plan.t1 = d_t1;
    plan.t2 = d_t2;
    plan.items = d_items;
    plan.reduces = d_red;
    plan.chunks = chunks.data();
    plan.n_chunks = (int)chunks.size();
    plan.red_chunks = (red_max + 255) / 256;
    const size_t tbytes = (size_t)std::max<int64_t>(tbuf_max, 1) * (fp64 ? sizeof(double) : sizeof(uint16_t));
    plan.tbuf = plan_alloc<uint16_t>(H, tbytes / sizeof(uint16_t));
    plan.partial = plan_alloc<double>(H, (size_t)std::max<int64_t>(part_max, 1));
    plan.partial_size = part_max;
    if (const char* e = std::getenv("DMRG_PLAN_TRACE"))
        if (e[0] == '1')
            std::fprintf(stderr, "[dmrg big plan%s] chunks %zu pass-1 groups %zu pass-2 items %zu reduces %zu T %.1f MB "
                         "partial %.1f MB\n", fp64 ? " fp64" : "", chunks.size(), t1.size(), items.size(), reds.size(),
                         tbytes * 1e-6, part_max * 8e-6);
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace

void drop_graphs(dmrg_hop& H) {
    for (auto& g : H.graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    H.graphs.clear();
}

namespace {

// Targets whose own or some source's dimension exceeds `limit` (the 96-wide LDS stages of the split
// kernel; 112 for the FP64 LDS-staged kernel).
std::vector<char> large_targets(const dmrg_hop& H, int limit = 96) {
    std::vector<int> smax(H.blk.size(), 0);
    for (size_t j = 0; j < H.blk.size(); ++j) smax[j] = std::max(H.blk_ma[j], H.blk_md[j]);
    for (const auto& t : H.tasks) smax[t.j] = std::max({smax[t.j], H.blk_ma[t.i], H.blk_md[t.i]});
    std::vector<char> big(H.blk.size(), 0);
    for (size_t j = 0; j < H.blk.size(); ++j) big[j] = smax[j] > limit;
    return big;
}

// Targets of the FP64 H.psi that take the two-pass path. The one-wavefront kernel has no size limit,
// so this is a cost choice: per target, the MFMA work each path executes (padded to its tiles; the
// one-wavefront kernel recomputes A.X for every 128-column output tile) divided by the fraction of
// the FP64 MFMA rate it sustains (measured: two-pass ~0.65 of peak on its padded work, one-wavefront
// ~0.3). mode 2: every target above the 96-wide LDS stages (as the split path).
// Tasks already taken by the FP64 LDS-staged kernel (lds_task) are left out of the comparison.
std::vector<char> fp64_big_targets(const dmrg_hop& H, int mode, const std::vector<char>* lds_task) {
    // with the LDS-staged kernel on, targets within its 112 x 112 tiles are its own
    std::vector<char> big = large_targets(H, H.tune_lds64 ? 16 * dmrg::kLds64MaxTiles : 96);
    if (mode == 2) return big;
    auto up = [](double m, double q) { return std::ceil(m / q) * q; };
    std::vector<double> c_big(H.blk.size(), 0.0), c_one(H.blk.size(), 0.0);
    for (size_t k = 0; k < H.tasks.size(); ++k) {
        const auto& t = H.tasks[k];
        if (!big[t.j] || (lds_task && !lds_task->empty() && (*lds_task)[k])) continue;
        const double ma = H.blk_ma[t.i], md = H.blk_md[t.i], mj = H.blk_ma[t.j], nj = H.blk_md[t.j];
        const double r16 = up(mj, 16), nrt = r16 / 16, nq = up(nj, 16) / 16;
        const double ka = up(ma, 16), kd = up(md, 16);
        // two-pass: pass 1 (8 x 8 tiles of 16 per group, k over the source rows holding data), pass 2
        // (the output tiles inside the target, k over the T tiles holding data)
        c_big[t.j] += (2.0 * up(nrt, 8) * 16 * up(kd / 16, 8) * 16 * ka + 2.0 * r16 * up(nj, 16) * kd) / 0.65;
        // one wavefront per 32 x 128 tile: A.X per column tile, then (A.X).B^T
        const double ncol = std::ceil(nj / 128.0);
        c_one[t.j] += (2.0 * up(mj, 32) * up(ma, 16) * up(md, 16) * ncol + 2.0 * up(mj, 32) * up(md, 16) * up(nj, 16)) / 0.3;
    }
    for (size_t j = 0; j < big.size(); ++j) big[j] = big[j] && c_big[j] < c_one[j];
    return big;
}

// FP64 tiled copy of the whole pool (16 x 16 tiles of hpsi_big64.hip, same offsets as the pool)
// followed by FP64 tiled identity blocks of sizes 32, 64, ... up to the widest padded block, which
// stand in for identity factors. Made once, on the first plan that routes targets to the FP64
// large-block path.
void make_tiled_f64(dmrg_hop& H, hipStream_t s) {
    if (H.d_tiled64) return;
    const int64_t n = H.pool_size;
    int pmax = 96;
    for (size_t i = 0; i < H.blk.size(); ++i)
        pmax = std::max({pmax, dmrg::ld_of(H.blk_ma[i]), dmrg::ld_of(H.blk_md[i])});
    std::vector<double> id;
    H.ident64_off.assign(pmax / 32, -1);
    for (int k = 0; k < pmax / 32; ++k) {
        const int p = 32 * (k + 1), k16 = p / 16;
        H.ident64_off[k] = n + (int64_t)id.size();
        const size_t base = id.size();
        id.resize(base + (size_t)p * p, 0.0);
        for (int i = 0; i < p; ++i) {
            // element (i, i): tile (i / 16, i / 16), lane (i % 16) + 16 ((i % 16) % 4), value (i % 16) / 4
            const int t = i / 16, c = i % 16, lane = c + 16 * (c % 4), v = c / 4;
            id[base + (size_t)(t * k16 + t) * 256 + lane * 4 + v] = 1.0;
        }
    }
    H.tiled64_size = n + (int64_t)id.size();
    H.d_tiled64 = dev_alloc<double>(H, H.tiled64_size);
    dmrg::PoolBlock* d_pb = dev_alloc<dmrg::PoolBlock>(H, H.pool_blocks.size());
    HIPCHK(hipMemcpyAsync(d_pb, H.pool_blocks.data(), H.pool_blocks.size() * sizeof(dmrg::PoolBlock),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(H.d_tiled64 + n, id.data(), id.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(dmrg::launch_tile_f64(H.d_pool, d_pb, (int)H.pool_blocks.size(), H.d_tiled64, s));
    HIPCHK(hipStreamSynchronize(s));   // the staging vector goes out of scope
}

// Launch plan of the FP64 LDS-staged kernel (hpsi_lds64.hip) for the target blocks whose own and
// sources' padded dimensions are at most 96 (targets flagged in `large` are skipped, and so are tasks
// whose source is a single 32 x 32 tile unless tune_lds64_small; `lds` marks the tasks taken). A
// target's tasks (source order) go to the KT = 2 classes when the source has at most 32 rows, else to
// KT = 6; each run is cut into items of bounded cost (the MFMA instructions of one wavefront plus a
// per-step and per-task overhead), and a target covered by several items gets partial tiles that a
// reduction adds in item order. The packed input has the geometry of the other FP64 plans (every psi
// block padded to multiples of 32).
void build_lds64_plan(dmrg_hop& H, hipStream_t s, const std::vector<char>& large, std::vector<char>& lds) {
    const size_t nb = H.blk.size();
    lds.assign(H.tasks.size(), 0);
    std::vector<int64_t> pk_off(nb);
    int64_t psize = 0;
    for (size_t i = 0; i < nb; ++i) {
        pk_off[i] = psize;
        psize += (int64_t)dmrg::ld_of(H.blk_ma[i]) * dmrg::ld_of(H.blk_md[i]);
    }
    auto ident = [&](int p) -> int64_t {
        const int k = p / 32 - 1;
        if (k < 0 || k >= (int)H.ident64_off.size() || H.ident64_off[k] < 0)
            throw Error(DMRG_ERR_ARG, "internal: no FP64 tiled identity block");
        return H.ident64_off[k];
    };
    // every operand block the kernel reads must be a pool block of the task's shape (rows in 16-row
    // tiles, at least the rows read; columns exactly the source's padded dimension) or an identity block
    std::unordered_map<int64_t, std::pair<int, int>> shape;   // offset -> (row tiles, 16-wide k tiles)
    for (const auto& pb : H.pool_blocks) shape[pb.off] = {pb.r16, 2 * pb.k32};
    for (size_t q = 0; q < H.ident64_off.size(); ++q)
        if (H.ident64_off[q] >= 0) shape[H.ident64_off[q]] = {2 * (int)(q + 1), 2 * (int)(q + 1)};
    auto check = [&](int64_t off, int rows16, int k16) {
        auto it = shape.find(off);
        if (it == shape.end() || it->second.first < rows16 || it->second.second != k16)
            throw Error(DMRG_ERR_ARG, "internal: FP64 LDS task operand does not match its pool block");
    };
    // MFMA instructions of one wavefront (per source column tile: GEMM1 over ka16 k tiles, GEMM2 over
    // tq column tiles) + per-step and per-task overhead
    auto cost = [](const dmrg::LTask64& L, int tq) { return L.kd16 * (4.0 * (L.ka16 + tq) + 6.0) + 4.0; };
    struct Run { int j, cls, tq; int32_t tb, te; };
    std::vector<dmrg::LTask64> lt;
    lt.reserve(H.tasks.size());
    std::vector<Run> runs;
    CostCaps caps(H);
    size_t k = 0;
    for (size_t j = 0; j < nb; ++j) {
        const size_t kb = k;
        while (k < H.tasks.size() && H.tasks[k].j == (int)j) ++k;
        if (k == kb || large[j]) continue;
        const int nrt = dmrg::rows_of(H.blk_ma[j]) / 16, tq = dmrg::rows_of(H.blk_md[j]) / 16;
        constexpr int kMax = dmrg::kLds64MaxTiles;
        if (nrt > kMax || tq > kMax) throw Error(DMRG_ERR_ARG, "internal: FP64 LDS target beyond 112 x 112");
        const bool wide = nrt > 6 || tq > 6;      // the (7, 7, 7) class takes every task of the target
        const int qcls = tq <= 3 ? 0 : 1;
        std::vector<dmrg::LTask64> v2, v6, v7;
        for (size_t t = kb; t < k; ++t) {
            const auto& ht = H.tasks[t];
            const int a = H.blk[ht.i][0], d = H.blk[ht.i][3];
            const int pa = dmrg::ld_of(H.blk_ma[ht.i]), pd = dmrg::ld_of(H.blk_md[ht.i]);
            if (!H.tune_lds64_small && pa <= 32 && pd <= 32) continue;   // single-tile source: one-wave kernel
            if (std::max(H.blk_ma[ht.i], H.blk_md[ht.i]) > 16 * kMax) continue;   // source above the tiles: other paths
            lds[t] = 1;
            dmrg::LTask64 L;
            L.x_off = pk_off[ht.i];
            L.a_off = ht.lm >= 0 ? H.mats[ht.lm].pool_of_in[a] : ident(pa);
            L.b_off = ht.rm >= 0 ? H.mats[ht.rm].pool_of_in[d] : ident(pd);
            if (L.a_off < 0 || L.b_off < 0) throw Error(DMRG_ERR_ARG, "internal: operator block missing from the pool");
            L.f = ht.f;
            L.pa16 = (int16_t)(pa / 16);
            L.pd16 = (int16_t)(pd / 16);
            L.ka16 = (int16_t)((H.blk_ma[ht.i] + 15) / 16);
            L.kd16 = (int16_t)((H.blk_md[ht.i] + 15) / 16);
            if (L.ka16 > kMax || L.kd16 > kMax || L.x_off + (int64_t)pa * pd > psize)
                throw Error(DMRG_ERR_ARG, "internal: FP64 LDS task beyond 112-wide sources");
            check(L.a_off, nrt, L.pa16);
            check(L.b_off, tq, L.pd16);
            (wide || L.ka16 > 6 ? v7 : L.ka16 <= 2 ? v2 : v6).push_back(L);
        }
        for (int kc : {0, 1, 2}) {
            const auto& v = kc == 0 ? v2 : kc == 1 ? v6 : v7;
            if (v.empty()) continue;
            Run R{(int)j, kc == 2 ? 4 : 2 * kc + qcls, tq, (int32_t)lt.size(), 0};
            for (const auto& L : v) {
                lt.push_back(L);
                caps.add((int)j, cost(L, tq));
            }
            R.te = (int32_t)lt.size();
            runs.push_back(R);
        }
    }
    H.lplan64 = dmrg::LdsPlan64{};
    struct It { dmrg::Item item; double cost; int cls; };
    std::vector<It> its;
    std::vector<dmrg::Reduce> reds;
    int64_t part = 0;
    int most = 1;
    // the runs of one target (one per stage size) are consecutive; all their chunks share one
    // reduction record, so that no two records of the one reduction launch add into the same tile
    for (size_t r0 = 0, r1; r0 < runs.size(); r0 = r1) {
        r1 = r0;
        while (r1 < runs.size() && runs[r1].j == runs[r0].j) ++r1;
        struct Chunk { int32_t b, e; double cost; int cls; };
        std::vector<Chunk> chunks;
        for (size_t r = r0; r < r1; ++r) {
            const Run& R = runs[r];
            int32_t b = R.tb;
            double c = 0.0;
            const double cmax = caps.cap(R.j, H.tune_lds64_items, 200.0);
            for (int32_t t = R.tb; t < R.te; ++t) {
                const double tc = cost(lt[t], R.tq);
                if (c + tc > cmax && t > b) { chunks.push_back({b, t, c, R.cls}); b = t; c = 0.0; }
                c += tc;
            }
            chunks.push_back({b, R.te, c, R.cls});
        }
        const int j = runs[r0].j, tm = dmrg::rows_of(H.blk_ma[j]), tn = 16 * runs[r0].tq;
        if (chunks.size() == 1) {
            const Chunk& q = chunks[0];
            its.push_back({{H.blk_off[j], -1, H.blk_ma[j], H.blk_md[j], 0, 0, q.b, q.e}, q.cost, q.cls});
            continue;
        }
        reds.push_back({H.blk_off[j], part, H.blk_ma[j], H.blk_md[j], 0, 0, tm, tn, (int32_t)chunks.size(), 0});
        most = std::max(most, tm * tn);
        for (const Chunk& q : chunks) {
            its.push_back({{H.blk_off[j], part, H.blk_ma[j], H.blk_md[j], 0, 0, q.b, q.e}, q.cost, q.cls});
            part += (int64_t)tm * tn;
        }
    }
    // launch order: class, then heaviest item first
    std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) {
        if (a.cls != b.cls) return a.cls < b.cls;
        return a.cost > b.cost;
    });
    std::vector<dmrg::Item> items;
    items.reserve(its.size());
    int cnt[dmrg::kLds64Classes] = {0};
    for (const It& x : its) { items.push_back(x.item); cnt[x.cls]++; }
    for (int c = 0; c < dmrg::kLds64Classes; ++c) H.lplan64.cls_begin[c + 1] = H.lplan64.cls_begin[c] + cnt[c];
    tag_parts(H, items);
    tag_parts(H, reds);
    dmrg::Item* d_items = plan_alloc<dmrg::Item>(H, items.size());
    dmrg::LTask64* d_lt = plan_alloc<dmrg::LTask64>(H, lt.size());
    dmrg::Reduce* d_red = plan_alloc<dmrg::Reduce>(H, reds.size());
    if (!items.empty())
        HIPCHK(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(items[0]), hipMemcpyHostToDevice, s));
    if (!lt.empty()) HIPCHK(hipMemcpyAsync(d_lt, lt.data(), lt.size() * sizeof(lt[0]), hipMemcpyHostToDevice, s));
    if (!reds.empty()) HIPCHK(hipMemcpyAsync(d_red, reds.data(), reds.size() * sizeof(reds[0]), hipMemcpyHostToDevice, s));
    H.lplan64.items = d_items;
    H.lplan64.tasks = d_lt;
    H.lplan64.reduces = d_red;
    H.lplan64.n_reduces = (int)reds.size();
    H.lplan64.red_chunks = (most + 255) / 256;
    H.lplan64.partial = plan_alloc<double>(H, (size_t)std::max<int64_t>(part, 1));
    H.lplan64.partial_size = part;
    H.lplan64.n_items = (int)items.size();
    H.lplan64.w7_min_waves = H.tune_lds64_w7 ? 4 : 1;
    H.lplan64.copy_wave = H.tune_lds64_cw;
    H.lplan64.three_slots = H.tune_lds64_ns3;
    if (const char* e = std::getenv("DMRG_PLAN_TRACE"))
        if (e[0] == '1') {
            std::fprintf(stderr, "[dmrg lds64 plan] items %zu classes", items.size());
            for (int c = 0; c < dmrg::kLds64Classes; ++c) std::fprintf(stderr, " %d", cnt[c]);
            std::fprintf(stderr, " reduces %zu partial %.1f MB\n", reds.size(), part * 8e-6);
        }
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace

// Every launch plan of the handle: FP64 (all targets) and, with split operators, the LDS-staged
// plan plus the plans for the targets it does not cover.
void build_plan(dmrg_hop& H, hipStream_t s) {
    drop_graphs(H);
    for (void* p : H.plan_allocations) (void)hipFree(p);
    H.plan_allocations.clear();
    H.plan_bytes = 0;
    // FP64: targets within the 96-wide LDS stages take the LDS-staged kernel; larger ones the
    // two-pass path where it is cheaper, the one-wave kernel otherwise
    H.bplan64 = dmrg::BigPlan{};
    H.big_chunks64.clear();
    H.lplan64 = dmrg::LdsPlan64{};
    H.xt64 = nullptr;
    const size_t nb = H.blk.size();
    std::vector<char> big64(nb, 0), lds64;   // targets of the two-pass path; tasks of the LDS kernel
    bool any_big = false, any_lds = false;
    if (H.tune_lds64) {
        // the LDS-staged kernel takes the targets within its 112 x 112 tiles: with task routing every
        // task of such a target whose source fits too, otherwise only targets whose sources all fit
        make_tiled_f64(H, s);
        std::vector<char> lds_large = large_targets(H, 16 * dmrg::kLds64MaxTiles);
        if (H.tune_lds64_task_route)
            for (size_t j = 0; j < nb; ++j) lds_large[j] = std::max(H.blk_ma[j], H.blk_md[j]) > 16 * dmrg::kLds64MaxTiles;
        build_lds64_plan(H, s, lds_large, lds64);
        for (char b : lds64) any_lds |= b != 0;
    }
    if (H.tune_big64) {
        big64 = fp64_big_targets(H, H.tune_big64, &lds64);
        for (char b : big64) any_big |= b != 0;
    }
    if (any_big) make_tiled_f64(H, s);
    if (any_big || any_lds) {
        std::vector<char> rest(nb), rest_tasks(H.tasks.size(), 1);
        for (size_t j = 0; j < nb; ++j) rest[j] = !big64[j];
        for (size_t t = 0; t < lds64.size(); ++t) rest_tasks[t] = !lds64[t];
        build_plan_core(H, s, &rest, false, H.plan, H.launches, H.phases, &rest_tasks);
        if (any_big) build_big_plan(H, s, big64, true, &rest_tasks);
        H.xt64 = plan_alloc<double>(H, (size_t)std::max<int64_t>(H.plan.packed_size, 1));
    } else {
        build_plan_core(H, s, nullptr, false, H.plan, H.launches, H.phases);
    }
    H.plan_fb = dmrg::HpsiPlan{};
    H.launches_fb.clear();
    H.phases_fb.clear();
    H.n_fallback_targets = 0;
    if (!H.has_split) return;
    std::vector<char> fb, fb_task;
    build_lds_plan(H, s, fb, fb_task);
    H.bplan = dmrg::BigPlan{};
    if (H.n_fallback_targets > 0) {
        if (H.tune_big) {
            build_big_plan(H, s, fb, false, &fb_task);
            H.n_fallback_targets = 0;
        } else {
            if (!H.d_hi) throw Error(DMRG_ERR_ARG, "internal: row-major split operators missing");
            build_plan_core(H, s, &fb, true, H.plan_fb, H.launches_fb, H.phases_fb, &fb_task);
        }
    }
}


// True when some target block (or one of its sources) has a padded dimension above the LDS stage
// size of the LDS-staged split kernel.
bool needs_fallback(const dmrg_hop& H) {
    for (char b : large_targets(H)) if (b) return true;
    return false;
}


// Tiled hi/lo copy of the whole FP64 pool (internal.h) followed by tiled identity blocks of sizes
// 32, 64, ... up to the widest padded block (hi = 1 on the diagonal, lo = 0), which stand in for
// identity factors.
void make_tiled_split(dmrg_hop& H, hipStream_t s) {
    int64_t n = 2 * H.pool_size;
    int pmax = 96;
    for (size_t i = 0; i < H.blk.size(); ++i)
        pmax = std::max({pmax, dmrg::ld_of(H.blk_ma[i]), dmrg::ld_of(H.blk_md[i])});
    std::vector<uint16_t> id;
    H.ident_off.assign(pmax / 32, -1);
    for (int k = 0; k < pmax / 32; ++k) {
        const int p = 32 * (k + 1), r16 = p / 16, k32 = p / 32;
        H.ident_off[k] = n + (int64_t)id.size();
        const size_t base = id.size();
        id.resize(base + (size_t)r16 * k32 * dmrg::kTileU16, 0);
        for (int i = 0; i < p; ++i) {
            const int rt = i / 16, kt = i / 32, lane = (i % 16) + 16 * ((i % 32) / 8), u = i % 8;
            id[base + (size_t)(rt * k32 + kt) * dmrg::kTileU16 + lane * 8 + u] = 0x3F80;   // bf16 1.0
        }
    }
    H.tiled_size = n + (int64_t)id.size();
    H.d_tiled = dev_alloc<uint16_t>(H, H.tiled_size);
    dmrg::PoolBlock* d_pb = dev_alloc<dmrg::PoolBlock>(H, H.pool_blocks.size());
    HIPCHK(hipMemcpyAsync(d_pb, H.pool_blocks.data(), H.pool_blocks.size() * sizeof(dmrg::PoolBlock),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(H.d_tiled + n, id.data(), id.size() * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    HIPCHK(dmrg::launch_split_tiled(H.d_pool, d_pb, (int)H.pool_blocks.size(), H.d_tiled, s));
    HIPCHK(hipStreamSynchronize(s));   // the staging vector goes out of scope
}


}  // namespace dmrg
