// Device-side data structures shared by the host driver (host.cpp) and the HIP kernels
// (kernels.hip). Plain structs, no HIP types, so host-only builds can include it.
//
// Padded layouts. Every operator block in the pool is stored row-major with its rows padded to a
// multiple of 16 and its leading dimension (columns) padded to a multiple of 32, zero-filled.
// Before each H.psi the input vector is packed into the same kind of layout (rows and columns of
// every psi block padded to multiples of 32). MFMA tiles therefore never need bounds masks.
#pragma once
#include <stdint.h>

namespace dmrg {

constexpr int kRowPad = 16;    // row padding of pool blocks (MFMA tile height)
constexpr int kLd = 32;        // leading-dimension padding of pool blocks and packed psi blocks
inline int32_t ld_of(int32_t m) { return (m + kLd - 1) / kLd * kLd; }
inline int32_t rows_of(int32_t m) { return (m + kRowPad - 1) / kRowPad * kRowPad; }

// One sector-GEMM contribution to an output psi block (Eq. dgemm, Section 2.2.1):
//   Y_target += f * A . X_source . B^T
// A (m_a' x m_a) and B (m_d' x m_d) live in the operator pool (padded layout); a_off / b_off < 0
// mean identity. X is read from the packed input (pa x pd, row-major, ld = pd; and for the split
// path also its transpose, ld = pa).
struct Task {
    int64_t x_off;   // element offset of the packed source block
    int64_t a_off;   // pool offset of A, or -1
    int64_t b_off;   // pool offset of B, or -1
    double  f;
    int32_t pa;      // source rows padded to 32 (leading dimension of A and of the packed X^T)
    int32_t pd;      // source cols padded to 32 (leading dimension of B and of the packed X)
    int32_t ka;      // source rows padded to 16 (FP64 reduction bound over m_a)
    int32_t kd;      // source cols padded to 16 (FP64 reduction bound over m_d)
};

// One wavefront's work: a contiguous range of the tasks writing one output tile of a target block
// (rows [r0, r0 + 16*TP) x cols [c0, c0 + 16*TQ)). slot < 0: the item owns the whole tile and stores
// it into y; otherwise it stores a partial tile into partial slot `slot` and a reduction item adds
// the slots of the tile in a fixed order (deterministic, no atomics).
struct Item {
    int64_t y_off;
    int64_t part_off;        // < 0: store into y; else offset of this item's partial tile (tm x tn)
    int32_t m_ap, m_dp;
    int32_t r0, c0;
    int32_t t_begin, t_end;
    int32_t part = 0;        // merged problem of the target (dmrg_hop_combine), see kPartActive
    int32_t pad = 0;
};
constexpr int kTileRows = 32;                  // max rows of a tile (TP <= 2)
constexpr int kPartialVecs = 4;                // vectors per launch

struct Reduce {
    int64_t y_off;
    int64_t part_off;        // first partial tile; the tile's n_parts partials follow contiguously
    int32_t m_ap, m_dp;
    int32_t r0, c0;
    int32_t tm, tn;          // tile extent
    int32_t n_parts;
    int32_t part;            // merged problem of the target
};
// Part mask of a merged handle: launchers take an optional device array with one entry per merged
// problem; the records (items, reductions, pass-1 groups) of a problem whose entry is not
// kPartActive are skipped, which leaves its part of y unspecified. A null mask runs every record.
constexpr int32_t kPartActive = 1;

// ---------------------------------------------------------------- tiled split-BF16 operands
// Split-BF16 operands of the LDS-staged sector-GEMM kernel are stored pre-tiled in MFMA fragment
// order: a matrix with R rows (padded to 16) and K columns (padded to 32) is cut into 16 x 32 tiles,
// tile (rt, kt) at ((rt * K/32) + kt) * kTileU16 elements, row-major over tiles. Inside a tile the
// 64 lanes' 8-element fragments are contiguous (hi: lane * 8 + u, lo: 512 + lane * 8 + u) with lane
// l = (row % 16) + 16 * ((col % 32) / 8), u = col % 8 -- the operand layout of
// v_mfma_f32_16x16x32_bf16. A pool block of rows_of(R) x ld_of(K) doubles at pool offset o occupies
// exactly the u16 range [2 o, 2 o + 2 rows_of(R) ld_of(K)) of the tiled array.
constexpr int kTileU16 = 1024;
struct PoolBlock { int64_t off; int32_t r16, k32; };

// Task of the LDS-staged split kernel: Y_tile += f * A . X . B^T with every factor present (identity
// factors point at tiled identity blocks). Offsets are u16 offsets into the tiled arrays.
struct LTask {
    int64_t x_off;   // tiled X^T of the source block (see k_pack_xt)
    int64_t a_off;   // tiled A block (rows = target rows, K = source rows)
    int64_t b_off;   // tiled B block (rows = target cols, K = source cols)
    float   f;
    int16_t pa32;    // source rows padded to 32, in units of 32
    int16_t pd32;    // source cols padded to 32, in units of 32
};

// Packing of one psi block into the padded input layout.
struct PackBlock {
    int64_t src_off;         // offset in the caller's x (m_a x m_d, row-major)
    int64_t dst_off;         // offset in the packed buffers
    int32_t m_a, m_d;
    int32_t pa, pd;
};

// Pre-summed / transposed operator block (Section 2.2.3): out = sum_k coeff_k * src_k (or src_k^T).
struct PresumBlock {
    int64_t out_off;
    int32_t rows, cols;
    int32_t t_begin, t_end;
};
struct PresumTerm {
    int64_t src_off;
    int32_t src_ld;
    int32_t trans;
    double  coeff;
};

// Diagonal contribution of a task that maps a block onto itself: D += f diag(A) diag(B)^T.
struct DiagTask {
    int64_t a_off, b_off;   // -1 for identity
    double  f;
};
struct DiagBlock {
    int64_t off;
    int32_t m_a, m_d;
    int32_t t_begin, t_end;
};

}  // namespace dmrg

#ifndef DMRG_HOST_ONLY
#include <hip/hip_runtime.h>
namespace dmrg {
// H.psi launch plan. Work items are grouped by phase (a subset of the operator combinations whose
// operators fit in the last-level cache) and, inside a phase, by tile class
// c = (TP - 1) * 8 + (TQ - 1), TP in 1..2, TQ in 1..8. y is zeroed first; every item and every
// reduction then adds its tile into y (each tile has one owner per phase, phases run in order).
constexpr int kClasses = 16;
struct HpsiLaunch { int cls, item_begin, item_count; };
struct HpsiPhase { int launch_begin, launch_end, reduce_begin, reduce_end; };
struct HpsiPlan {
    const Item* items;            // device
    const Reduce* reduces;        // device
    const Task* tasks;            // device
    double* partial;              // device, partial_size * kPartialVecs doubles
    int64_t partial_size;         // elements of the partial tiles of one vector (largest phase)
    const HpsiLaunch* launches;   // host
    const HpsiPhase* phases;      // host
    int n_phases;
    const PackBlock* packs;       // device
    int n_packs;
    int64_t packed_size;          // elements of one packed vector
    double* xp;                   // packed FP64 input, kPartialVecs vectors
    uint16_t* xr_hi;              // packed BF16 split input, row-major
    uint16_t* xr_lo;
    uint16_t* xt_hi;              // packed BF16 split input, transposed
    uint16_t* xt_lo;
};

// Launch plan of the LDS-staged split kernel (hpsi_lds.hip). Items (internal.h Item) cover whole
// target row blocks; launch class = (S, TP): S = largest padded dimension (32, 64 or 96) sizing the
// LDS stages, TP = row tiles per wave; each class is one launch of kLdsWaves-wave workgroups.
// Tasks whose source is a single 32 x 32 tile run in the task-mode kernel (one wavefront per target
// block of NR row tiles and at most NQ column tiles), classes (NR, NQ) = (1,2) (2,2) (1,4), launched
// after the row-mode classes; items[small_begin[c] .. small_begin[c+1]).
// Row-mode classes (S, TP) = (64,1) (64,2) (96,1) (96,2): a target's tasks whose source and target
// fit 64-wide stages run in the S = 64 classes (64 KB of LDS, several workgroups per CU), the other
// big-source tasks in the S = 96 classes.
constexpr int kLdsWaves = 4;
constexpr int kLdsClasses = 4;
constexpr int kSmallClasses = 3;
constexpr int kReduceKinds = 3;         // partial tiles of S = 64 runs, S = 96 runs, task-mode runs
struct LdsPlan {
    const Item* items = nullptr;        // device
    const LTask* tasks = nullptr;       // device
    const Reduce* reduces = nullptr;    // device, grouped by kind; one reduction launch per kind
                                        // (records of one kind cover disjoint parts of y)
    int red_begin[kReduceKinds + 1] = {0, 0, 0, 0};
    int red_chunks[kReduceKinds] = {1, 1, 1};   // 256-element chunks of the largest tile per kind
    int cls_begin[kLdsClasses + 1] = {0, 0, 0, 0, 0};   // item ranges per class
    int small_begin[kSmallClasses + 1] = {0, 0, 0, 0};
    double* partial = nullptr;          // device, partial_size * kPartialVecs doubles
    int64_t partial_size = 0;
    const PackBlock* packs = nullptr;   // device (same packing geometry as HpsiPlan)
    int n_packs = 0;
    int64_t xt_size = 0;                // u16 elements of one tiled X^T vector (2 * packed_size)
    uint16_t* xt = nullptr;             // device, xt_size * kPartialVecs
    int prefetch_mask = 0x4;            // row-mode classes (bit c) whose workgroups get a cache-line
                                        // prefetch wavefront: (96,1) (one workgroup per CU anyway);
                                        // the S = 64 classes would lose their second workgroup per
                                        // CU (measured slower); (96,2) runs 3 compute wavefronts then
    int copy_wave_mask = 0;             // row-mode classes (bit c) with a copy wavefront that issues every
                                        // LDS copy (no prefetch wavefront then)
    int six_wave_mask = 0x8;            // (S, 2) classes (bits 1, 3) run as six wavefronts of one row
                                        // tile each (targets of 65..96 rows) instead of four of two:
                                        // (96,2), whose one workgroup per CU then has two wavefronts on
                                        // two of the SIMDs (measured faster; (64,2) is not)
};

// Launch plan of the FP64 LDS-staged kernel (hpsi_lds64.hip): items (internal.h Item; r0 = c0 = 0)
// each cover a whole target block of at most 112 x 112 and a range of its tasks, over the FP64 tiled
// pool (identity factors point at its identity blocks) and the tiled FP64 X^T of the packed input
// (offsets in doubles). Launch classes (KT, QT, W): c = 2 (KT == 6) + (QT == 6) for targets of at most
// 96 x 96 and sources of at most 96 rows (W = 6; KT = 2 when every task of the item has at most 32
// source rows, else 6; QT = 3 for targets of at most 48 columns, else 6), c = 4 (7, 7, 7) for the
// rest (a target or a source of 97 .. 112 rows or columns).
constexpr int kLds64Classes = 5;
constexpr int kLds64MaxTiles = 7;       // target rows / columns and source rows, in 16-wide tiles
struct LTask64 {
    int64_t x_off, a_off, b_off;
    double  f;
    int16_t pa16, pd16;      // source rows / columns padded to 32, in 16-wide tiles (tile strides)
    int16_t ka16, kd16;      // source rows / columns padded to 16: the k tiles and j tiles that hold
                             // data (the others are zero padding and are skipped)
};
struct LdsPlan64 {
    const Item* items = nullptr;        // device
    const LTask64* tasks = nullptr;     // device
    const Reduce* reduces = nullptr;    // device; one record per target cut into several items (its
    int n_reduces = 0;                  // items of both stage sizes), so one launch adds them all
    int red_chunks = 1;                 // 256-element chunks of the largest partial tile
    int cls_begin[kLds64Classes + 1] = {0, 0, 0, 0, 0, 0};
    double* partial = nullptr;          // device, partial tiles of one vector
    int64_t partial_size = 0;
    int n_items = 0;
    int w7_min_waves = 1;               // 4: the (7, 7, 7) class held to 128 VGPRs (two workgroups per CU)
    int copy_wave = 1;                  // 1: one more wavefront per workgroup issues every LDS copy
    int three_slots = 0;                // with the copy wavefront: the KT = 2 classes stage two steps ahead
};
// y (one vector) += the plan's targets of f A X B^T; xt = that vector's tiled FP64 X^T
// (launch_pack_xt64 with the FP64 packing geometry)
hipError_t launch_hpsi_lds64(const LdsPlan64& P, const double* pool_t, const double* xt, double* y, hipStream_t s,
                             const int32_t* active = nullptr);
// tiled FP64 X^T of every psi block (hpsi_big64.hip)
hipError_t launch_pack_xt64(const PackBlock* packs, int n_packs, const double* x, double* xt, hipStream_t s);
// y (one vector) += the partial tiles of each record, in order (hpsi_lds.hip)
hipError_t launch_reduce_partials(const Reduce* reduces, int n, int chunks, const double* partial, double* y,
                                  hipStream_t s, const int32_t* active = nullptr);

// ---------------------------------------------------------------- large blocks (hpsi_big.hip)
// Targets whose blocks (or sources) exceed the 96-wide LDS stages take two passes per chunk of
// targets: pass 1 writes T = f A X of every task into a tiled hi/lo buffer (tile (rt, jc) of the
// task's T at t_off + (rt * pd32 + jc) * kTileU16, in the A-operand fragment layout of pass 2),
// pass 2 accumulates Y += sum_tasks T B^T per 128 x 128 output tile.
// FP64 form (hpsi_big64.hip): 16 x 16 FP64 tiles, offsets in doubles, pa32 / pd32 / jb counted in
// 16-wide tiles.
struct BigT1 {             // pass-1 group: one task, rows [16 rb, 16 rb + 128), T^T rows [32 jb, 32 jb + 128)
    int64_t xt, a, t;      // tiled X^T of the source, tiled A, output T (u16 offsets)
    double f;
    int16_t pa32, pd32;    // source rows / cols in 32-element k tiles
    int16_t nrt;           // row tiles of the target block
    int16_t rb, jb;        // first row tile, first 32-column chunk
    int16_t part;          // merged problem of the target (masks use part < 32768)
    int16_t ka, kd;        // source rows / cols holding data, in k tiles (FP64 form: the k loop of
                           // pass 1 and the T tiles it writes stop there)
};
struct BigT2 {             // pass-2 task: T of the task and its B block
    int64_t t, b;
    int32_t pd32;
    int32_t kd;            // T tiles holding data along k (FP64 form: the k loop of pass 2 stops there)
};
// Chunk c: pass-1 workgroups [t1_begin, t1_end) (workgroup w runs groups t1_ranges[w] ..
// t1_ranges[w + 1] - 1), pass-2 items [item_begin, item_end), reductions [red_begin, red_end).
struct BigChunk { int t1_begin, t1_end, item_begin, item_end, red_begin, red_end; };
struct BigPlan {                    // split or FP64 form (see BigT1)
    const BigT1* t1 = nullptr;      // device
    const int32_t* t1_ranges = nullptr;   // device, one entry per pass-1 workgroup plus one
    const BigT2* t2 = nullptr;      // device
    const Item* items = nullptr;    // device: pass-2 items (r0 = 16 rb, c0 = 16 qb, task range in t2)
    const Reduce* reduces = nullptr;
    const BigChunk* chunks = nullptr;   // host
    int n_chunks = 0;
    int red_chunks = 1;             // 256-element chunks of the largest partial tile
    uint16_t* tbuf = nullptr;       // device, largest chunk's T (one vector at a time; doubles in the FP64 form)
    double* partial = nullptr;      // device, partial tiles of the largest chunk
    int64_t partial_size = 0;
};

// Launchers (kernels.hip). All asynchronous on `s`.
hipError_t launch_presum(const PresumBlock* blocks, int n_blocks, const PresumTerm* terms,
                         double* pool, hipStream_t s);
hipError_t launch_split(const double* pool, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t s);
hipError_t launch_hpsi_f64(const HpsiPlan& plan, const double* pool, const double* x, double* y,
                           int64_t n_coeff, int nvec, hipStream_t s, const int32_t* active = nullptr);
hipError_t launch_hpsi_split(const HpsiPlan& plan, const uint16_t* hi, const uint16_t* lo, const double* x,
                             double* y, int64_t n_coeff, int nvec, hipStream_t s, const int32_t* active = nullptr);
hipError_t launch_diag(const DiagBlock* blocks, int n_blocks, const DiagTask* tasks,
                       const double* pool, double* d, hipStream_t s);
// Davidson vector kernels (FP64).
hipError_t launch_multidot(const double* V, int nv, int64_t n, const double* w, double* partial,
                           int n_part, double* out, hipStream_t s);
constexpr int kMaxCombine = 72;
struct Coefs { double c[kMaxCombine]; };
hipError_t launch_combine(const double* V, int nv, int64_t n, const Coefs& coef, double* out,
                          double beta, hipStream_t s);
hipError_t launch_precond(const double* r, const double* d, double theta, double* t, int64_t n,
                          hipStream_t s);
hipError_t launch_scale(double* x, double a, int64_t n, hipStream_t s);
int multidot_parts(int64_t n);
// out -= sum_j c[j] V[j], c in device memory; x *= 1 / sqrt(*nrm2) with *nrm2 in device memory.
hipError_t launch_project_out(const double* V, int nv, int64_t n, const double* c, double* out, hipStream_t s);
hipError_t launch_scale_dev(double* x, const double* nrm2, int64_t n, hipStream_t s);

// Reduced density matrix of the enlarged left block (Section 2.1), one item per (sector, row group,
// row group): rho[rho_off + l * ld + l2] = sum over the sector's n_cd column groups k of
// sum_r X_{g,k}[l][r] X_{g2,k}[l2][r], with X_{g,k} the psi block at gblk[g + k] (row-major, m_d =
// cdmd[cd + k] columns), l < ma, l2 < ma2. Every element of rho is written by exactly one item.
struct RdmItem {
    int64_t rho_off;
    int32_t ld, ma, ma2, g, g2, cd, n_cd, pad;
};
hipError_t launch_rdm_left(const RdmItem* items, int n_items, const int64_t* gblk, const int32_t* cdmd,
                           const double* psi, double* rho, hipStream_t s);
// rho^R = psi^T psi with the same items: here ma, ma2 are the column counts of the two psi blocks of
// each term (their m_d), cdmd[cd + k] the k-th row count (m_a), and the sum runs over rows.
hipError_t launch_rdm_right(const RdmItem* items, int n_items, const int64_t* gblk, const int32_t* cdmd,
                            const double* psi, double* rho, hipStream_t s);

// Eq. renorm_mat per sector block, out = O_out^T A O_in, in two passes over the same items:
// pass 1 T = A O_in (rows_a x k_in, at t_off), pass 2 out = O_out^T T (k_out x k_in, at out_off).
// A is rows_a x cols_a (= O_out rows x O_in rows), row-major; O matrices are row-major (rows x k).
struct RenormItem {
    int64_t a_off, t_off, out_off, oo_off, oi_off;
    int32_t rows, cols, k_out, k_in;
};
hipError_t launch_renormalize(const RenormItem* items, int n_items, int64_t max_t, int64_t max_out, const double* A,
                              const double* O, double* T, double* out, hipStream_t s);
// Tiled split-BF16 kernels (hpsi_lds.hip).
hipError_t launch_split_tiled(const double* pool, const PoolBlock* blocks, int n_blocks, uint16_t* tiled, hipStream_t s);
// y (+)= H x over the LDS plan's targets; zero_y: clear y first (else accumulate into it).
hipError_t launch_hpsi_lds(const LdsPlan& plan, const uint16_t* pool_t, const double* x, double* y, int64_t n_coeff,
                           int nvec, bool zero_y, hipStream_t s, const int32_t* active = nullptr);
// Large-block split path (hpsi_big.hip) for one vector: y += the large targets' part of H x;
// xt = that vector's tiled X^T (packed by launch_hpsi_lds).
hipError_t launch_hpsi_big(const BigPlan& plan, const uint16_t* pool_t, const uint16_t* xt, double* y,
                           hipStream_t s, const int32_t* active = nullptr);
// FP64 large-block path (hpsi_big64.hip) for one vector: y += the large targets' part of H x, over the
// FP64 tiled pool; packs x into xt (FP64 tiled X^T, packed_size doubles) first unless packs is null
// (xt already holds it).
hipError_t launch_tile_f64(const double* pool, const PoolBlock* blocks, int n_blocks, double* tiled, hipStream_t s);
hipError_t launch_hpsi_big64(const BigPlan& plan, const double* pool_t, const PackBlock* packs, int n_packs,
                             const double* x, double* xt, double* y, hipStream_t s, const int32_t* active = nullptr);
// Old-kernel split path over a plan without clearing y first.
hipError_t launch_hpsi_split_acc(const HpsiPlan& plan, const uint16_t* hi, const uint16_t* lo, const double* x,
                                 double* y, int64_t n_coeff, int nvec, hipStream_t s,
                                 const int32_t* active = nullptr);
}  // namespace dmrg
#endif
