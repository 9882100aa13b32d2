// The H.psi handle (struct dmrg_hop) and the host-side types it is made of, shared by the host
// translation units of libdmrg: host.cpp (term generator, task list, launch plans, H.psi),
// renorm_host.cpp (density matrices, truncation, renormalization), davidson.cpp, sweep.cpp.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dmrg.h"
#include "host_common.h"
#include "internal.h"

namespace dmrg {

using M16 = std::array<double, 256>;   // two-site operator, index (b'*4+c') * 16 + (b*4+c)

// (n_alpha, n_beta) of the site states (0, up, down, updown).
constexpr int kSiteQn[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};

// ---------------------------------------------------------------- imported blocks
struct OpIn {
    int kind, i0, i1;
    std::vector<int> out_of_in;       // per ket sector: bra sector or -1
    std::vector<int64_t> off_of_in;   // host element offset of the block
};
struct BlockIn {
    int n_sec = 0;
    std::vector<int> qa, qb, dim;
    std::vector<OpIn> ops;
    std::map<std::array<int, 3>, int> index;
    const double* data = nullptr;
    int64_t n_data = 0;
    int find(int kind, int i0, int i1) const {
        auto it = index.find({kind, i0, i1});
        return it == index.end() ? -1 : it->second;
    }
};

// Name of an operator kind ("H", "C", ...).
const char* kind_name(int k);
// Validated copy of a caller's block description (throws Error).
BlockIn import_block(const dmrg_block* b, const char* side);

// ---------------------------------------------------------------- matrices and combinations
struct Term { double c; int op; bool tr; };
struct MatDef {
    int side;                       // 0 left, 1 right
    std::vector<Term> terms;        // matrix = sum c * op (or op^T)
    int transpose_id = -1;          // cache
    // materialized:
    std::vector<int> out_of_in;
    std::vector<int64_t> pool_of_in;
    double bytes = 0.0;             // padded pool bytes of all its sector blocks
};

struct Alpha {
    double coeff;
    int lmat;       // -1 identity
    int lpar;       // 0 none, 1 (-1)^{n(ket sector)}, 2 (-1)^{n(bra sector)}
    M16 S;
    int rmat;       // -1 identity
    int family;
};

// Spin-orbital integrals (reading of Eq. H2q: v_pqrs = (ps|qr)/2).
struct Integrals {
    int L;
    const double* h;
    const double* eri;
    double t(int P, int Q) const {
        if ((P & 1) != (Q & 1)) return 0.0;
        return h[(P >> 1) * L + (Q >> 1)];
    }
    double w(int P, int Q, int R, int S) const {
        if ((P & 1) != (S & 1) || (Q & 1) != (R & 1)) return 0.0;
        int p = P >> 1, q = Q >> 1, r = R >> 1, s = S >> 1;
        return eri[(((int64_t)p * L + s) * L + q) * L + r];
    }
};

// Basis of an enlarged block (block + one site), the rows of rho and of the renormalization matrix
// O of Eq. renorm: sectors q ascending in (n_alpha, n_beta); left side: pairs (a, s) in (a, s) order
// with q = qn(a) + qn(s), right side: pairs (s, d) in (s, d) order with q = qn(s) + qn(d); each pair
// contributes the dim states of its block sector consecutively (pairs of empty sectors are left
// out). groups[i] holds (x, y, first row) with (x, y) = (a, s) or (s, d).
struct EnlargedLayout {
    std::vector<std::pair<int, int>> qn;
    std::vector<int> dim;
    std::vector<int64_t> off;                                  // n_sec + 1: dense dim x dim blocks
    std::vector<std::vector<std::array<int, 3>>> groups;
};
EnlargedLayout enlarged_layout(const BlockIn& B, bool right);

// Block B (left: orbitals [0, site); right: orbitals (site, L)) grown by orbital `site` and
// renormalized by O (Eq. renorm_mat): B's operators on the device at data + op_off[op * n_sec + ket
// sector] (data_len doubles; leading dimension ld_of(columns) when `padded`, else the column count;
// every access is checked against data_len before launch); O on the host,
// per sector of enlarged_layout(B, right) a dim x kept row-major matrix, concatenated. Returns a
// library-owned block (free with dmrg_block_free). Synchronizes `s`.
dmrg_block* grow_block(const BlockIn& B, bool right, int site, const Integrals& I, const double* data,
                       int64_t data_len, const std::vector<int64_t>& op_off, bool padded, const std::vector<int>& kept,
                       const std::vector<double>& O, int device, hipStream_t s);

// The launch sequence of one H.psi on stream s (arguments checked; no host synchronization, so it can
// be captured into a graph).
void hpsi_enqueue(dmrg_hop* H, const double* x, double* y, int32_t nvec, int32_t precision, hipStream_t s);

}  // namespace dmrg

struct dmrg_hop {
    using BlockIn = dmrg::BlockIn;
    using MatDef = dmrg::MatDef;
    using Alpha = dmrg::Alpha;
    int L = 0, na = 0, nb = 0, site = 0;
    BlockIn left, right;
    std::vector<double> h, eri;
    // layout
    std::vector<std::array<int, 4>> blk;     // (a, b, c, d)
    std::vector<int> blk_ma, blk_md;
    std::vector<int64_t> blk_off;
    std::vector<int> blk_index;              // [(a*4+b)*4+c] -> block id or -1
    int64_t n_coeff = 0;
    // terms
    std::vector<MatDef> mats;
    std::map<std::tuple<int, int, bool>, int> mat_cache;
    std::vector<Alpha> alphas;
    // tasks
    struct HTask { int i, j, lm, rm; double f; };
    std::vector<HTask> tasks;
    double flops = 0.0, bytes = 0.0;
    // device
    int device = -1;
    bool has_split = false;
    int64_t pool_size = 0;
    double* d_pool = nullptr;
    uint16_t* d_hi = nullptr;
    uint16_t* d_lo = nullptr;
    dmrg::Task* d_tasks = nullptr;
    dmrg::HpsiPlan plan{};
    std::vector<dmrg::HpsiLaunch> launches;
    std::vector<dmrg::HpsiPhase> phases;
    // split path: LDS-staged kernel over tiled operands, plus the one-wave kernel (row-major hi/lo
    // operands, plan_fb) for targets whose blocks exceed the LDS stage size
    std::vector<dmrg::PoolBlock> pool_blocks;   // every block of the FP64 pool (for the tiled split)
    uint16_t* d_tiled = nullptr;                // tiled hi/lo operators + identity blocks
    int64_t tiled_size = 0;
    std::vector<int64_t> ident_off;             // tiled identity block of size 32 (k + 1), k = 0, 1, ...
    dmrg::LdsPlan lplan{};
    dmrg::HpsiPlan plan_fb{};
    std::vector<dmrg::HpsiLaunch> launches_fb;
    std::vector<dmrg::HpsiPhase> phases_fb;
    int n_fallback_targets = 0;
    int tune_lds_items = 16384;                 // target number of LDS work items per H.psi
    int tune_small_mode = 1;                    // 1: single-tile sources run in the task-mode kernel
    int tune_small_nr = 2;                      // task mode: most row tiles per wavefront (1 or 2)
    // hipGraphs of the H.psi launch sequence, one per (x, y, nvec, precision); dropped when a plan is rebuilt
    struct GraphEntry { const double* x; double* y; int nvec, prec; hipGraph_t graph; hipGraphExec_t exec; };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;           // capture stream (default priority)
    bool share = false;                         // build only the combinations whose operators are supplied
    int tune_lds_order = 0;                     // 0: heaviest item first; 1: XCD-aware by left sector;
                                                // 2: merged handle, each problem's items together
    int tune_lds_task_order = 0;                // 0: tasks by source; 1: by operator pair
    int tune_lds_split64 = 1;                   // 1: tasks fitting 64-wide stages run in the S = 64 classes
    int tune_lds_pf = 0x4;                      // row-mode classes with a prefetch wavefront (bit mask)
    int tune_lds_w6 = 0x8;                      // (S, 2) row-mode classes run as six one-row-tile wavefronts
    int tune_lds_cw = 0;                        // row-mode classes with a copy wavefront (bit mask; measured
                                                // slower for the split kernels, whose tasks are short)
    int tune_big = 1;                           // 1: targets above the LDS stages take the two-pass GEMM path
    int tune_big_stages = 64;                   // pass-2 item size in 32-wide k steps
    int tune_big_stages1 = 16;                  // pass-1 workgroup size in 32-wide k steps
    int tune_big_tbudget_mb = 1024;             // T buffer of one chunk of large targets (MB)
    dmrg::BigPlan bplan{};
    std::vector<dmrg::BigChunk> big_chunks;
    std::vector<std::pair<int32_t, int32_t>> big_t2_range;
    int tune_small_nq = 2;                      // task mode: least column-tile bound (2, 4 or 6)
    int tune_part_items = 1;                    // merged handles: 1 item cost caps per merged problem (from
                                                // its own total), 0 one cap from the whole handle's total
    int tune_split_task_route = 1;              // 1: a target within the split LDS stages keeps its tasks
                                                // with sources that fit them; 0: any larger source sends
                                                // the whole target to the two-pass path
    // FP64 two-pass path (hpsi_big64.hip) for the same large targets
    int tune_big64 = 1;                         // FP64 two-pass path: 0 off, 1 where cheaper, 2 every target above 96
    double* d_tiled64 = nullptr;                // FP64 tiled operators + identity blocks (made on first use)
    int64_t tiled64_size = 0;
    std::vector<int64_t> ident64_off;           // FP64 tiled identity block of size 32 (k + 1)
    dmrg::BigPlan bplan64{};
    std::vector<dmrg::BigChunk> big_chunks64;
    double* xt64 = nullptr;                     // FP64 tiled X^T of one vector (plan allocation)
    // FP64 LDS-staged kernel (hpsi_lds64.hip) for the targets within the 96-wide stages
    int tune_lds64 = 1;                         // 0: those targets take the one-wave kernel
    int tune_lds64_items = 32768;               // target number of its work items per H.psi
    int tune_lds64_small = 1;                   // 1: it also takes tasks whose source is one 32 x 32 tile
                                                // (0: those run in the one-wave kernel)
    int tune_lds64_w7 = 1;                      // 1: its 7-wavefront class held to 128 VGPRs (two per CU)
    int tune_lds64_cw = 1;                      // 1: a copy wavefront per workgroup issues every LDS copy
    int tune_lds64_ns3 = 0;                     // 1: its KT = 2 classes keep three LDS slots (copies two steps
                                                // ahead; measured no faster at L = 24, M = 1024)
    int tune_lds64_task_route = 0;              // 1: a target within its tiles keeps the tasks whose source fits
                                                // them (larger sources: two-pass or one-wave path); 0: a
                                                // target with any larger source leaves it entirely
    dmrg::LdsPlan64 lplan64{};
    std::vector<void*> plan_allocations;   // freed when the plan is rebuilt
    int64_t dev_bytes = 0, plan_bytes = 0; // device memory held (handle lifetime / current plan)
    int vec_step = 1;                      // vectors per launch sequence (packed-input and partial buffers)
    bool trimmed = false;                  // dmrg_hop_trim: plans and derived operator copies released
    int64_t n_alpha = 0;
    int n_parts = 1;                       // problems merged into this handle (dmrg_hop_combine)
    std::vector<int64_t> part_coeff;       // first coefficient of each merged problem (+ end)
    const int32_t* d_active = nullptr;     // device part mask of every H.psi launch (null: all parts); set only
                                           // inside dmrg_davidson_batch, whose part status array it is
    int n_items = 0;
    int64_t n_dev_tasks = 0;
    int tune_max_tq = 8;       // widest output tile, in 16-column MFMA tiles (1..8)
    int tune_items = 32768;    // target number of work items per H.psi launch
    int tune_order = 2;        // item launch order (see build_plan)
    int tune_phases = 1;       // 0: from the operator footprint and kCacheBudget
    double* d_diag = nullptr;
    std::vector<void*> allocations;
    // pool offset of every stored operator sector block, per side: [op * n_sec + ket sector] or -1
    // (row-major, leading dimension ld_of(columns)); used to grow and renormalize the blocks
    std::vector<int64_t> op_pool_off[2];
};
