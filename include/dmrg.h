/*
 * dmrg.h -- C-ABI of libdmrg.so: the two-site QC-DMRG Davidson matrix-vector product H.psi on one
 * AMD Instinct MI355X (gfx950), after Brabec et al., "Massively parallel quantum chemical density
 * matrix renormalization group method" (Section 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Orbitals are 0-based, p = 0 .. L-1, ordered along the DMRG lattice. Spin-orbital id P = 2p + s,
 *    s = 0 (alpha) or 1 (beta). Fermionic (Jordan-Wigner) order is ascending P.
 *  - Hamiltonian (Eq. H2q, Section 2.1) with chemist integrals (pq|rs):
 *        H = sum t_PQ c+_P c_Q + 1/2 sum w_PQRS c+_P c+_Q c_R c_S,
 *        t_PQ = h_pq d(sP,sQ),  w_PQRS = (ps|qr) d(sP,sS) d(sQ,sR)      (i.e. v_pqrs = (ps|qr)/2).
 *  - Bond with left site s1 = `site` and right site s2 = site+1; left block = orbitals [0, site),
 *    right block = orbitals [site+2, L). The left block carries the "normal" operator set and the
 *    right block the "complementary" (pre-summed) set, see dmrg_op_kind.
 *  - Site basis (0, up, down, updown) with |updown> = c+_up c+_down |0>.
 *  - Symmetry sectors are (n_alpha, n_beta) pairs (U(1) x U(1), Section 2.1). Operator sector blocks
 *    are dense row-major <l'|O|l> of shape dim[sec_out] x dim[sec_in] (the operator class of
 *    Section 2.2: a sector table plus dense sector tensors).
 *  - psi layout (Eq. wf_sec): blocks (a, b, c, d) with a = left sector, b, c = site states, d = right
 *    sector, present iff the (n_alpha, n_beta) of the four parts add up to the targets; ordered by
 *    (a, b, c) lexicographically; each block row-major m_a x m_d, contiguous, no padding.
 *  - Status codes: 0 ok, >0 warning, <0 error; dmrg_last_error() gives a thread-local message.
 *    No C++ exception crosses the ABI. HIP runtime failures map to DMRG_ERR_DEVICE.
 *  - Ownership: inputs are caller-owned and only read during the call (the library copies what it
 *    keeps). Handles created by the library are released with the matching _free call.
 *  - Device vectors passed to dmrg_hpsi / dmrg_davidson are caller-owned device pointers on the
 *    handle's device; work is ordered on the given stream (0 = the handle's default stream).
 */
#ifndef DMRG_H
#define DMRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmrg_status;
#define DMRG_OK                 0
#define DMRG_NOT_CONVERGED      1
#define DMRG_ERR_ARG          (-1)
#define DMRG_ERR_SHAPE        (-2)
#define DMRG_ERR_NOMEM        (-3)
#define DMRG_ERR_DEVICE       (-4)
#define DMRG_ERR_NAN          (-5)
#define DMRG_ERR_ALIAS        (-6)
#define DMRG_ERR_UNSUPPORTED  (-7)

/* Last error message of the calling thread (never NULL; "" after success). */
const char* dmrg_last_error(void);

/* Library version string. */
const char* dmrg_version(void);

/* Problem definition: integrals (Eq. H2q), electron numbers (Section 2.1, sector constraints of
 * Eq. wf_sec) and the bond. Host pointers, read during dmrg_build_blocks only. */
typedef struct {
    int32_t n_orb;          /* L >= 2 */
    int32_t n_alpha;        /* N_alpha */
    int32_t n_beta;         /* N_beta */
    int32_t site;           /* s1 (0-based), 0 <= site <= L-2 */
    const double* h;        /* L*L row-major, symmetric */
    const double* eri;      /* L^4 row-major chemist (pq|rs), 8-fold symmetric */
} dmrg_problem;

/* Operator kinds of a block (indices are global spin-orbital ids).
 * Left ("normal") block X:
 *   H                 block Hamiltonian
 *   C  (P)            c+_P, P in X
 *   A  (P<Q)          c+_P c+_Q
 *   B  (P,Q)          c+_P c_Q, every ordered pair (B_QP may be omitted if B_PQ is given: then
 *                     B_QP = B_PQ^T is used)
 *   S  (W)            sum_{P,Q,R in X} w_PQRW c+_P c+_Q c_R for every W to the right of X
 *                     (three-index part only; the one-body part is added by the library)
 * Right ("complementary") block Y; "outside" = every spin-orbital to the left of Y:
 *   H, C (Z in Y)
 *   U  (P)            sum_{Q,Z,W in Y} w_PQZW c+_Q c_Z c_W, P outside
 *   P  (P<Q)          sum_{Z,W in Y} w_PQZW c_Z c_W, P<Q outside
 *   Q  (X,Y')         sum_{Z,W in Y} (w_XZWY' - w_XZY'W) c+_Z c_W, every ordered outside pair
 *                     (Q_Y'X may be omitted: then Q_Y'X = Q_XY'^T is used)
 * These are the complete operator intermediates of Section 2.1 (every stored operator must be the
 * projection of the exact operator onto the block basis for H.psi to equal P H P psi). */
typedef enum {
    DMRG_OP_H = 0, DMRG_OP_C = 1, DMRG_OP_A = 2, DMRG_OP_B = 3,
    DMRG_OP_S = 4, DMRG_OP_U = 5, DMRG_OP_P = 6, DMRG_OP_Q = 7
} dmrg_op_kind;

typedef struct {
    int32_t kind;           /* dmrg_op_kind */
    int32_t i0, i1;         /* spin-orbital ids, -1 if unused */
    int32_t n_blk;          /* number of stored sector blocks */
    const int32_t* sec_out; /* n_blk bra-side sector indices */
    const int32_t* sec_in;  /* n_blk ket-side sector indices (at most one block per sec_in) */
    const int64_t* off;     /* n_blk element offsets into dmrg_block.data */
} dmrg_op;

typedef struct {
    int32_t n_sec;
    const int32_t* qn;      /* 2*n_sec: (n_alpha, n_beta) per sector, distinct */
    const int32_t* dim;     /* n_sec: sector dimensions (>= 0) */
    int32_t n_ops;
    const dmrg_op* ops;
    const double* data;     /* host FP64 sector blocks, row-major */
    int64_t n_data;
} dmrg_block;

typedef struct dmrg_hop dmrg_hop;   /* opaque: device-resident operators, task lists, layout, diag */

#define DMRG_PREC_FP64    0         /* FP64 MFMA (v_mfma_f64_16x16x4) */
#define DMRG_PREC_SPLIT2  1         /* BF16 hi/lo split, 3 BF16 MFMA products, FP32 accumulation */

typedef struct {
    int32_t device;          /* HIP device ordinal; -1 = host-only build (term and task lists only,
                                no device memory; dmrg_hpsi then returns DMRG_ERR_UNSUPPORTED) */
    int32_t want_split;      /* 1: also prepare BF16 hi/lo operator copies (DMRG_PREC_SPLIT2) */
    int64_t mem_budget_bytes;/* 0 = no limit; exceeding it returns DMRG_ERR_NOMEM */
    void*   stream;          /* hipStream_t for the build; 0 = legacy default stream */
    int32_t share;           /* 0: every operator of the sets below must be supplied (missing ->
                                DMRG_ERR_ARG). 1: one device's share of the sum over operator
                                combinations (the paper's distribution of the combinations over
                                processes, Section 2.2.1), defined term by term: H.psi is the sum of
                                the Hamiltonian terms (left operator) x (site part) x (right operator)
                                whose left and right block operators are both supplied (identity
                                counts as supplied); a pre-summed left operator keeps its supplied
                                summands. Shares of disjoint operator pairs add up to the full sum
                                (terms without block operators belong to every share) */
} dmrg_build_opts;

/* Build the H.psi operator of one bond, once per bond and before Davidson starts (the pre-generated
 * task list of Section 2.2.1): psi sector layout (Eq. wf_sec), the list of operator
 * combinations alpha (the sum over alpha of the H.Phi equation, Section 2.2.1), on-the-fly
 * pre-summed left-block operators (Section 2.2.3) formed on the GPU, the owner-computes task list
 * for Eq. dgemm, and diag(H). `left` must carry the normal operator set and `right` the
 * complementary set described above; a missing operator returns DMRG_ERR_ARG naming it.
 * On success *out receives a handle owned by the caller (free with dmrg_hop_free). */
dmrg_status dmrg_build_blocks(const dmrg_problem* problem, const dmrg_block* left,
                              const dmrg_block* right, const dmrg_build_opts* opts, dmrg_hop** out);

void dmrg_hop_free(dmrg_hop* hop);

/* psi layout (Eq. wf_sec). Pass NULL arrays to query the counts only.
 *   abcd    4*n_blocks sector indices (a, b, c, d);   dims 2*n_blocks (m_a, m_d);
 *   offsets n_blocks element offsets. */
dmrg_status dmrg_hop_layout(const dmrg_hop* hop, int64_t* n_coeff, int32_t* n_blocks,
                            int32_t* abcd, int32_t* dims, int64_t* offsets);

/* Algorithmic work of one H.psi: flops = sum over tasks of 2 * MACs of the cheaper association of
 * A.X.B^T (identity factors skipped); bytes = one read of every distinct operator block used + one
 * read of x + one write of y (FP64). n_alpha = operator combinations, n_tasks = sector GEMM tasks. */
dmrg_status dmrg_hop_stats(const dmrg_hop* hop, double* flops, double* bytes, int64_t* n_alpha,
                           int64_t* n_tasks);

/* y = H x for `nvec` vectors stored one after another (stride n_coeff). Device pointers, FP64,
 * x and y must not overlap (DMRG_ERR_ALIAS). precision: DMRG_PREC_FP64 or DMRG_PREC_SPLIT2 (the
 * latter needs want_split at build). Deterministic: each output tile is owned by one wavefront and
 * accumulated in a fixed order (no atomics). Asynchronous on `stream`. */
dmrg_status dmrg_hpsi(dmrg_hop* hop, const double* x, double* y, int32_t nvec, int32_t precision,
                      void* stream);

/* Same result as dmrg_hpsi, through a hipGraph of the whole launch sequence: the first call for a
 * given (x, y, nvec, precision) captures the sequence (on a private stream of default priority)
 * and instantiates it, then launches it on `stream`; later calls with the same
 * arguments replay it on `stream` with one launch. The handle keeps at most one graph per argument
 * tuple until it is freed or its launch plan is rebuilt (dmrg_hop_autotune). Buffers x and y must
 * stay allocated while their graph may be replayed. Callers for whom launch overhead matters (many
 * small H.psi, the Davidson loop with use_graph = 1) use this form. */
dmrg_status dmrg_hpsi_graph(dmrg_hop* hop, const double* x, double* y, int32_t nvec, int32_t precision,
                            void* stream);

/* diag(H) (FP64) into a device buffer of n_coeff doubles. */
dmrg_status dmrg_hop_diagonal(dmrg_hop* hop, double* d, void* stream);

/* Reduced density matrix of the enlarged left block, rho^L = psi psi^T (Section 2.1, the matrix whose
 * M leading eigenvectors form the renormalization matrix of Eq. renorm), with psi read as the matrix
 * psi_{(l s_l), (s_r r)}. U(1) x U(1) makes rho^L block diagonal in the enlarged-left quantum number
 * q = qn(a) + qn(s_l).
 *
 * dmrg_rdm_left_layout: the sectors, in ascending (n_alpha, n_beta). *n_sec receives their number;
 * qn (2 * n_sec int32: n_alpha, n_beta), dims (n_sec) and offsets (n_sec + 1 int64, offsets of the
 * dense blocks, offsets[n_sec] = sum of dims^2) are filled when not NULL (call once with NULL to size
 * them). Rows of sector q: the pairs (a, s_l) with qn(a) + qn(s_l) = q in (a, s_l) order, each with
 * the dim(a) states of left sector a, including pairs that no psi block reaches (zero rows). Works on
 * host-only handles; a merged handle (dmrg_hop_combine) returns DMRG_ERR_UNSUPPORTED.
 *
 * dmrg_rdm_left: rho (device, rho_len doubles, rho_len = offsets[n_sec]) receives every sector's
 * dim x dim block, row-major, at its offset; psi is a device vector of n_coeff doubles in the handle's
 * layout. FP64, each element summed in a fixed order (deterministic). Synchronizes `stream` before
 * returning (it allocates and frees small device work lists). Errors: DMRG_ERR_ARG (NULL),
 * DMRG_ERR_SHAPE (rho_len), DMRG_ERR_UNSUPPORTED (host-only or merged handle), DMRG_ERR_DEVICE. */
dmrg_status dmrg_rdm_left_layout(const dmrg_hop* hop, int32_t* n_sec, int32_t* qn, int32_t* dims,
                                 int64_t* offsets);
dmrg_status dmrg_rdm_left(dmrg_hop* hop, const double* psi, double* rho, int64_t rho_len, void* stream);

/* The same for the enlarged right block (backward sweeps): rho^R = psi^T psi, block diagonal in the
 * enlarged-right quantum number q = qn(s_r) + qn(d), sectors ascending. Rows of sector q: the pairs
 * (s_r, d) in (s_r, d) order, each with the dim(d) states of right sector d, including pairs that no
 * psi block reaches. Arguments, layout of rho, determinism, synchronization and errors as above. */
dmrg_status dmrg_rdm_right_layout(const dmrg_hop* hop, int32_t* n_sec, int32_t* qn, int32_t* dims,
                                  int64_t* offsets);
dmrg_status dmrg_rdm_right(dmrg_hop* hop, const double* psi, double* rho, int64_t rho_len, void* stream);

/* The truncation of Section 2.1: the M eigenvectors of a block-diagonal density matrix with the
 * largest eigenvalues (they form the renormalization matrix of Eq. renorm). Host routine, FP64: each
 * sector by Householder tridiagonalization and the implicit symmetric QR iteration with Wilkinson
 * shifts; sectors are solved on up to 16 host threads (results do not depend on their number).
 * rho (host, read only): n_sec symmetric dims[i] x dims[i] row-major blocks at offsets[i], the prefix
 * sums of dims^2 (the layout of dmrg_rdm_left_layout). Outputs, all host, caller-allocated:
 * evals (sum of dims doubles: per sector, in sector order, its eigenvalues in descending order);
 * vecs (offsets[n_sec] doubles: per sector a row-major dims x dims matrix whose column k is the
 * eigenvector of the k-th largest eigenvalue, its largest-magnitude component positive); kept (n_sec
 * int32: how many leading columns of each sector are kept); discarded (1 double: trace minus the kept
 * eigenvalues). The M largest eigenvalues are taken over all sectors together, ties in (sector,
 * position) order; M = 0 keeps nothing, M >= sum of dims keeps everything. Only the projector onto
 * the kept columns is unique (when the cut falls between distinct eigenvalues). Errors: DMRG_ERR_ARG
 * (NULL, negative n_sec or M), DMRG_ERR_SHAPE (offsets), DMRG_ERR_NAN (non-finite input, no
 * convergence). */
dmrg_status dmrg_truncate(const double* rho, int32_t n_sec, const int32_t* dims, const int64_t* offsets, int32_t M,
                          int32_t* kept, double* evals, double* vecs, double* discarded);

/* Eq. renorm_mat per sector block: out_b = O[sec_out[b]]^T A_b O[sec_in[b]] for n_blk operator blocks
 * given in an enlarged (untruncated) basis of n_sec sectors. FP64 on `device`, two passes (T = A O_in,
 * then O_out^T T), each element summed in a fixed order.
 * Host arrays: dims, kept (n_sec: sector dimension, kept states, 0 <= kept <= dims), o_off (n_sec:
 * offset of sector s's renormalization matrix in O), sec_out, sec_in (n_blk sector indices), a_off,
 * out_off (n_blk offsets). Device arrays: O (o_len doubles; sector s at o_off[s], row-major dims[s] x
 * kept[s], columns = kept eigenvectors, e.g. the leading columns of dmrg_truncate's vecs), A (a_len;
 * block b at a_off[b], row-major dims[sec_out] x dims[sec_in]), out (out_len; block b at out_off[b],
 * row-major kept[sec_out] x kept[sec_in]; blocks must not overlap each other, A or O). Blocks with
 * nothing kept on a side are empty and skipped. Every index and extent is checked against the
 * lengths before launch. Synchronizes `stream` before returning (allocates and frees the
 * intermediate T). Errors: DMRG_ERR_ARG (NULL, negative counts, sector index, kept > dims),
 * DMRG_ERR_SHAPE (a block outside its buffer), DMRG_ERR_UNSUPPORTED (block above 2^31 elements),
 * DMRG_ERR_DEVICE. */
dmrg_status dmrg_renormalize_blocks(int32_t device, int32_t n_sec, const int32_t* dims, const int32_t* kept,
                                    const int64_t* o_off, const double* O, int64_t o_len, int32_t n_blk,
                                    const int32_t* sec_out, const int32_t* sec_in, const int64_t* a_off,
                                    const double* A, int64_t a_len, const int64_t* out_off, double* out,
                                    int64_t out_len, void* stream);

/* dmrg_renormalize_blocks for callers that cannot allocate device memory (code under stream
 * capture, serving loops, harnesses that forbid hipMalloc): same arguments, checks, kernels and
 * results (bit for bit), but the work list and the intermediate T = A O_in live in a fixed device
 * array of 64 MiB per GPU inside the library (held until the process ends) instead of fresh
 * allocations; the call allocates nothing. Limit: 256-byte-rounded work list (40 B per block that
 * keeps states on both sides) + 8 B x sum over those blocks of rows(sec_out) x kept(sec_in) must fit
 * in 64 MiB, else DMRG_ERR_NOMEM (nothing is launched). Every call on one GPU shares that GPU's
 * array: calls that overlap in time on the same GPU (other host threads or streams) race and must
 * be serialized by the caller. Synchronizes `stream` before returning. */
dmrg_status dmrg_renormalize_blocks_noalloc(int32_t device, int32_t n_sec, const int32_t* dims, const int32_t* kept,
                                            const int64_t* o_off, const double* O, int64_t o_len, int32_t n_blk,
                                            const int32_t* sec_out, const int32_t* sec_in, const int64_t* a_off,
                                            const double* A, int64_t a_len, const int64_t* out_off, double* out,
                                            int64_t out_len, void* stream);

/* ---------------------------------------------------------------------------------------------
 * Growth and renormalization of a block (Section 2.1: the operators of the enlarged block, its
 * truncation by the M eigenvectors of rho with the largest eigenvalues, Eq. renorm, Eq. renorm_mat;
 * Section 2.2.2).
 * side 0 grows the left block of the bond (site, site+1): orbitals [0, site) + orbital `site` become
 * the left block of the bond (site+1, site+2), with the normal set H, C (P in the block), A (P < Q),
 * B (P <= Q only: B_QP = B_PQ^T), S (W >= 2(site+1)). side 1 grows the right block: orbital site+1 +
 * orbitals [site+2, L) become the right block of the bond (site-1, site), with the complementary set
 * H, C (Z in the block), U (P < 2(site+1)), P (P < Q < 2(site+1)), Q (X <= Y < 2(site+1) only: Q_YX =
 * Q_XY^T). Every grown operator is formed from its definition with single stored operators of the
 * old block (pre-summed over old-block indices where the definition sums them), so operators that are
 * projections of the exact ones stay so. The basis of the enlarged block is the one of
 * dmrg_rdm_left_layout / dmrg_rdm_right_layout: sectors ascending, left pairs (a, s) in (a, s) order,
 * right pairs (s, d) in (s, d) order. The new block's sectors are the enlarged sectors that keep
 * states, ascending; its states in sector q are the kept columns of O_q in order.
 * The returned block is owned by the library (host arrays, valid until dmrg_block_free) and can be
 * passed to dmrg_build_blocks and grown again. FP64, on the GPU (pre-sums and O^T Z O per sector
 * block); synchronizes the stream.
 * ------------------------------------------------------------------------------------------- */

/* Sectors of the enlarged block (block + site) that `block` grows into: *n_sec, and when not NULL qn
 * (2 * n_sec) and dims (n_sec). Host only. */
dmrg_status dmrg_block_grow_layout(const dmrg_block* block, int32_t side, int32_t* n_sec, int32_t* qn,
                                   int32_t* dims);

/* Grow `block` (host data, as for dmrg_build_blocks) by one site at the bond of `problem` (its site
 * field) and renormalize it with the caller's O: kept (host, n_sec of dmrg_block_grow_layout: states
 * kept per enlarged sector, 0 <= kept <= dims) and O (host, per enlarged sector a dims x kept
 * row-major matrix whose columns span the kept states, concatenated in sector order). kept = O = NULL
 * keeps every state (exact growth). Runs on opts->device / opts->stream. *out receives a
 * library-owned block. Errors: DMRG_ERR_ARG (missing operator of the old block, bad side or kept),
 * DMRG_ERR_NAN, DMRG_ERR_NOMEM, DMRG_ERR_DEVICE. */
dmrg_status dmrg_block_grow(const dmrg_problem* problem, const dmrg_block* block, int32_t side, const int32_t* kept,
                            const double* O, const dmrg_build_opts* opts, dmrg_block** out);

/* One renormalization step of the sweep for the handle's bond: rho of the enlarged block from the
 * device vector psi (dir 0: rho^L = psi psi^T, growing the left block; dir 1: rho^R = psi^T psi,
 * growing the right block), its M-state cut with M = m_max (dmrg_truncate: the m_max largest
 * eigenvalues over all sectors), and the grown block's operators renormalized with those eigenvectors
 * (Eq. renorm_mat), using the handle's device copy of the old block. *out receives a library-owned
 * block; *discarded (may be NULL) the discarded weight (trace of rho minus the kept eigenvalues).
 * Works on handles built with a device (not merged ones). Synchronizes `stream`. */
dmrg_status dmrg_renormalize(dmrg_hop* hop, const double* psi, int32_t dir, int32_t m_max, dmrg_block** out,
                             double* discarded, void* stream);

/* Release a block returned by dmrg_block_grow / dmrg_renormalize (NULL and blocks the library did not
 * create are ignored). */
void dmrg_block_free(dmrg_block* block);

/* Davidson's method for the lowest eigenpair (Sections 2.1, 2.2.1). FP64 basis, Gram-Schmidt
 * (classical, applied twice), Rayleigh-Ritz and energies; the matvec runs in `precision`.
 * With precision = SPLIT2 and fp64_polish = 1 the solve switches to FP64 matvecs (restarting from the
 * current Ritz vector) once the split residual falls below split_tol, or is below 30 split_tol and has
 * made no new minimum (by 1%) for 10 iterations, and finishes at tol. The correction vector comes from
 * the diagonal preconditioner or from a learned network (precond, mlp). */
typedef struct dmrg_mlp dmrg_mlp;   /* opaque: learned preconditioner (weights, Adam state, datasets) */
typedef struct {
    double  tol;             /* ||r||_2 convergence threshold on the normalized Ritz vector */
    int32_t max_iter;        /* iterations (matvecs beyond the first) */
    int32_t max_sub;         /* subspace size before restart (2 .. 64) */
    int32_t precision;       /* DMRG_PREC_* for the matvec */
    int32_t fp64_polish;     /* see above */
    double  split_tol;       /* residual at which split precision hands over to FP64 (e.g. 1e-5) */
    int32_t use_graph;       /* 1: matvecs through dmrg_hpsi_graph (one graph per basis slot), 0: dmrg_hpsi */
    int32_t precond;         /* DMRG_PRECOND_DIAG or DMRG_PRECOND_MLP */
    const struct dmrg_mlp* mlp;   /* network for DMRG_PRECOND_MLP (same device as the handle) */
} dmrg_dav_opts;

#define DMRG_PRECOND_DIAG 0  /* t = r / (theta - D), D = diag(H), |theta - D| floored at 1e-8 */
#define DMRG_PRECOND_MLP  1  /* t = r / (theta - D) * (1 + m), m from the learned network below, until
                                the diagonal rule takes over (see precond_fallback_iter) */

typedef struct {
    double  energy;          /* lowest Ritz value */
    double  resid;           /* final ||r||_2 */
    int32_t iters;           /* iterations performed */
    int32_t matvecs;         /* total H.psi applications */
    int32_t matvecs_split;   /* of which in split precision */
    double  t_total;         /* seconds, wall */
    double  t_hpsi;          /* seconds spent in H.psi (device time, HIP events) */
    int32_t precond_fallback_iter; /* DMRG_PRECOND_MLP: iteration from which the diagonal correction
                                      replaced the network (the residual made no new minimum, by 1%,
                                      for 20 iterations, or did not halve within 10 iterations under
                                      the network); -1 if the network ran to the end */
} dmrg_dav_result;

/* psi: device pointer, n_coeff doubles: in = start vector (need not be normalized, must be
 * non-zero), out = Ritz vector (normalized). Returns DMRG_NOT_CONVERGED (with the best pair filled
 * in) when max_iter is reached, DMRG_ERR_NAN when the start vector or a matvec is not finite.
 * Synchronizes the stream before returning. */
dmrg_status dmrg_davidson(dmrg_hop* hop, double* psi, const dmrg_dav_opts* opts,
                          dmrg_dav_result* result, void* stream);

/* Batching: merge several built handles (same device) into one handle whose psi is the
 * concatenation of the inputs' psi vectors (in the given order) and whose H is the direct sum, so a
 * single dmrg_hpsi call computes all problems in one launch sequence whose work items are balanced
 * over the whole batch (the task list of Section 2.2.1, merged across problems). The inputs stay
 * valid and independent; the new handle owns copies of their device operators. Davidson on a
 * combined handle solves the direct-sum problem (its lowest eigenpair over all parts). */
dmrg_status dmrg_hop_combine(dmrg_hop* const* hops, int32_t n, void* stream, dmrg_hop** out);

/* Batched H.psi of independent problems (the task lists of Section 2.2.1, one per problem):
 * y[i] = H_i x[i] for i < n, one vector per handle (device pointers of hops[i]'s n_coeff doubles),
 * every handle on one device, enqueued in order on `stream` without host synchronization. The
 * launch sequences stay those of the individual handles; for one launch sequence over a common pool
 * of work items (and one graph launch), merge the handles once with dmrg_hop_combine and call
 * dmrg_hpsi / dmrg_hpsi_graph on the merged handle with the vectors concatenated. Errors:
 * DMRG_ERR_ARG (NULL pointers, n < 0, handles on different devices, bad precision),
 * DMRG_ERR_ALIAS (x[i] and y[i] overlap, or an output overlaps another problem's vector), and those
 * of dmrg_hpsi; nothing is launched unless every argument is valid. */
dmrg_status dmrg_hpsi_batched(dmrg_hop* const* hops, int32_t n, const double* const* x, double* const* y,
                              int32_t precision, void* stream);

/* Release the parts of a built handle that only its own H.psi uses — launch plans, cached graphs,
 * the tiled split and tiled FP64 operator copies — keeping the FP64 operator pool, diag(H) and the
 * host-side description that dmrg_hop_combine reads: for callers that merge many handles and need
 * the memory for the merged one. Waits for all work on the device (hipDeviceSynchronize) before
 * freeing. Afterwards the handle can be combined, queried (layout, stats, parts, diagonal) and
 * freed; dmrg_hpsi, dmrg_hpsi_graph, dmrg_davidson and dmrg_hop_autotune return
 * DMRG_ERR_UNSUPPORTED. Trimming a trimmed or host-only handle does nothing. */
dmrg_status dmrg_hop_trim(dmrg_hop* hop);

/* Number of merged problems and their first coefficient offsets (n_parts + 1 entries, the last is
 * n_coeff). A handle from dmrg_build_blocks has one part. */
dmrg_status dmrg_hop_parts(const dmrg_hop* hop, int32_t* n_parts, int64_t* first_coeff);

/* Davidson for the lowest eigenpair of every part of a merged handle (dmrg_hop_combine; a plain
 * handle is one part), all parts in lockstep with the whole iteration on the device (Sections 2.1,
 * 2.2.1 for the method): the merged H.psi, per-part dot products, Gram-Schmidt (twice) and norms, the
 * Rayleigh-Ritz step of every part (cyclic Jacobi on its k x k matrix in one workgroup), Ritz vector,
 * residual, diagonal preconditioner, and the restart at max_sub (to the Ritz vector and the previous
 * one), so no host synchronization is needed inside an iteration. With opts->use_graph = 1 the launch
 * sequence of each subspace size is captured once as a hipGraph and replayed (the graphs live for the
 * call); 0 launches the same sequence directly (same results bit for bit). The host reads the parts'
 * status every 4 iterations and stops when none is active. Parts that have stopped cost no further
 * work: their H.psi records and vector chunks are skipped (environment DMRG_BATCH_PART_MASK=0 runs
 * their H.psi work to the end, with the same results). A part stops when its residual norm is
 * <= tol, or when its correction lies in its subspace (stalled). psi (device, n_coeff doubles): in,
 * the start vectors (each part's segment nonzero), out, the Ritz vectors. Split precision with
 * fp64_polish runs every part to max(split_tol, tol) with split matvecs, then restarts every part in
 * FP64 from its Ritz vector. opts->precond must be DMRG_PRECOND_DIAG; max_sub 3 .. 64. Per-part
 * results go into the caller's arrays (capacity >= n_parts, NULL to skip); status: 0 converged, 1 not
 * converged in max_iter, 2 stalled. Returns DMRG_NOT_CONVERGED when some part did not converge,
 * DMRG_ERR_NAN on a non-finite residual, errors as dmrg_davidson. Synchronizes the stream. */
typedef struct {
    int32_t  capacity;
    double*  energy;
    double*  resid;
    int32_t* iters;
    int32_t* status;
    int32_t  n_parts;
    int32_t  n_converged;
    int32_t  matvecs;       /* merged H.psi launches */
    int32_t  graphs;        /* iteration graphs captured */
    double   t_total;       /* wall time of the call */
} dmrg_dav_batch_result;
dmrg_status dmrg_davidson_batch(dmrg_hop* hop, double* psi, const dmrg_dav_opts* opts, dmrg_dav_batch_result* result,
                                void* stream);

/* Autotuner of the H.psi launch plan for `precision`: one pass of coordinate descent over the
 * plan's settings, each taking in turn its fastest candidate value with the others held at their
 * best so far; every candidate is timed on the device (the fastest of `reps` calls after one
 * warm-up) and the plan is rebuilt with the winners. Settings, in the order of `chosen`:
 * split: LDS work items (4k .. 64k; per merged problem on a merged handle), launch order (heaviest
 * first / XCD-aware by left sector / each merged problem's items together), task-mode tile shape
 * (0: 1 x 2, 1: 2 x 2, 2: 1 x 4 row x column MFMA tiles per wavefront), 64-wide stage classes (1 on),
 * six-wavefront (S, 2) classes (bit mask 0x8 / 0 / 0xA), copy-wavefront classes (0 / 0xF), prefetch
 * wavefront (0x4 / 0), 0. FP64: LDS-staged kernel work items (8k .. 64k), its copy wavefront (1/0),
 * single-tile sources in it (1/0), its 7-wavefront register cap (1/0), two-pass routing of large
 * targets (1 where cheaper, 2 all), one-wavefront tile width (2, 4, 8 tiles of 16 columns), its work
 * items (8k, 32k, 64k) and launch order (0 heaviest first, 2 cache-aware). chosen
 * (DMRG_AUTOTUNE_KNOBS ints) and best_ms (milliseconds of the chosen plan) may be NULL. Drops the
 * handle's cached graphs. Synchronizes `stream`. */
#define DMRG_AUTOTUNE_KNOBS 8
dmrg_status dmrg_hop_autotune(dmrg_hop* hop, int32_t precision, int32_t reps, void* stream,
                              int32_t* chosen, double* best_ms);

/* Host-logic introspection (used by the CPU tests of the term generator): the task list as
 * (source block, target block, left matrix id, right matrix id) quadruples with scalars f, and the
 * definition of every matrix id as a list of (matrix id, side 0=left/1=right, op index into the
 * block's op array, transposed 0/1, coefficient) entries -- i.e. matrix = sum coeff * op(^T).
 * Matrix id -1 is the identity. Pass NULL arrays to query the counts. */
dmrg_status dmrg_hop_export_tasks(const dmrg_hop* hop, int64_t* n_tasks, int32_t* quads, double* f,
                                  int64_t* n_terms, int32_t* term_int, double* term_coeff);

/* ---------------------------------------------------------------------------------------------
 * Two-site DMRG sweeps (Section 2.1). Warm-up: the right blocks of the last 1 .. L-2 orbitals are
 * grown from the vacuum (dmrg_block_grow), each step keeping at most m_warmup states of the enlarged
 * block (every state while they fit; else a seeded random orthonormal basis per sector, with the kept
 * counts spread over the sectors near the filling N k / L of the block's k orbitals). Sweep j (of
 * n_sweeps, bond dimension m_per_sweep[j]): forward over the bonds (0, 1) .. (L-2, L-1) -- Davidson
 * for the lowest eigenpair (seeded random start vector), then dmrg_renormalize of the left block --
 * and backward over (L-3, L-2) .. (0, 1), renormalizing the right block (the solve at (L-2, L-1)
 * and, between sweeps, at (0, 1) serves both directions). Each solve builds its H.psi with
 * dmrg_build_blocks from the current blocks, so every step runs on the GPU; blocks are kept in host
 * memory between bonds.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    int32_t        n_sweeps;       /* >= 1 */
    const int32_t* m_per_sweep;    /* n_sweeps bond dimensions (M of each sweep, >= 1) */
    int32_t        m_warmup;       /* states kept per warm-up growth step (>= 1) */
    double         tol;            /* Davidson residual tolerance per bond */
    int32_t        max_iter;       /* Davidson iterations per bond */
    int32_t        max_sub;        /* Davidson subspace size (2 .. 64) */
    int32_t        precision;      /* DMRG_PREC_* of the matvec */
    int32_t        fp64_polish;    /* see dmrg_dav_opts */
    double         split_tol;
    uint64_t       seed;           /* warm-up bases and start vectors (splitmix64 stream) */
    int32_t        device;
    void*          stream;
    int32_t        verbose;        /* 1: one line per solve on stderr */
    int32_t        keep_site;      /* 1 .. n_orb - 3: hand the blocks of the bond (keep_site, keep_site+1)
                                      after the last sweep back in the result; 0: none */
    const struct dmrg_mlp* mlp;    /* learned preconditioner (DMRG_PRECOND_MLP, with its diagonal judge)
                                      for the solves of sweeps mlp_from_sweep .. n_sweeps - 1; NULL: the
                                      diagonal preconditioner everywhere (warm-up has no solves) */
    int32_t        mlp_from_sweep; /* 0 .. n_sweeps - 1 */
    int32_t        mlp_shadow;     /* 1: in those sweeps every bond is solved twice from the same start
                                      vector, with the diagonal preconditioner (the sweep goes on with
                                      this solve) and with the network (results in energies_alt /
                                      iters_alt): a comparison on identical two-site problems */
} dmrg_sweep_opts;

typedef struct {
    int32_t  capacity;             /* length of the caller's arrays below (they may be NULL) */
    double*  energies;             /* per Davidson solve, in order: lowest Ritz value */
    double*  discarded;            /* discarded weight of the renormalization after that solve (0 if none) */
    int32_t* iters;                /* Davidson iterations */
    int32_t* sites;                /* left site of the solve's bond */
    int32_t  n_solves;             /* solves performed (2L - 3 in the first sweep, 2L - 4 in each later one) */
    int32_t  n_not_converged;      /* solves that reached max_iter */
    double   energy;               /* energy of the last solve */
    double   best_energy;          /* lowest energy of any solve */
    double   seconds;              /* wall time */
    dmrg_block* left_block;        /* keep_site > 0: the left block (orbitals 0 .. keep_site - 1) and */
    dmrg_block* right_block;       /* the right block (keep_site + 2 .. n_orb - 1) of that bond as the
                                      last sweep left them (left from its forward pass, right from its
                                      backward pass: the pair the last solve at that bond used); owned
                                      by the caller (dmrg_block_free); NULL otherwise or on error */
    double*  energies_alt;         /* mlp_shadow: per solve, the learned solve's Ritz value (NaN where */
    int32_t* iters_alt;            /* none ran) and iterations (-1); may be NULL */
} dmrg_sweep_result;

/* Run the warm-up and n_sweeps sweeps for `problem` (its site field is ignored). Returns
 * DMRG_NOT_CONVERGED when some Davidson solve reached max_iter (the sweep goes on with its best
 * pair), errors as the calls it makes; keep_site outside 0 .. n_orb - 3, or mlp_from_sweep outside
 * 0 .. n_sweeps - 1 with an mlp, is DMRG_ERR_ARG. */
dmrg_status dmrg_sweep(const dmrg_problem* problem, const dmrg_sweep_opts* opts, dmrg_sweep_result* result);

/* ---------------------------------------------------------------------------------------------
 * Learned Davidson preconditioner (an addition to the method of the paper, which uses Davidson's
 * diagonal preconditioner). One MLP is shared by all psi coefficients:
 *     x_i (16 features) -> relu(256) -> relu(256) -> m_i,   t_i = r_i / (theta - D_i) * (1 + m_i),
 * so a network whose output layer is zero is exactly the diagonal preconditioner. Features of
 * coefficient i of psi block (a, b, c, d), with s_x = sqrt(n) / ||x|| (0 for x = 0):
 *     asinh(r_i s_r), asinh(t_i s_t), asinh(u_i s_u), asinh((D_i - theta) s_D), one-hot b (4),
 *     one-hot c (4), asinh(rms_block(r) s_r), asinh(rms_block(u) s_u), ln(m_a)/8, ln(m_d)/8
 * (r residual, u Ritz vector, t = r / (theta - D) the diagonal correction, D = diag(H)).
 * Parameters (FP32, DMRG_MLP_PARAMS floats): W1 (16 x 256, row = input), b1 (256), W2 (256 x 256,
 * row = input), b2 (256), w3 (256), b3 (1). Inference and training run hand-written kernels: the
 * forward on the matrix cores with BF16 copies of W1, W2 and FP32 accumulation; set_fp32 selects an
 * FP32 debug mode on the vector units.
 * Training pairs come from converged solves (dmrg_mlp_collect). For each iteration, with V the
 * subspace that the correction t is about to be orthogonalized against and psi the solve's final
 * eigenvector, the ideal correction is P psi = psi - V V^T psi (appending it makes the subspace
 * contain psi). Davidson only uses the direction of t, so per sampled coefficient the pair is t and
 * P psi at unit RMS, P psi turned to point along t:
 *     a = t_i sqrt(n) / ||t||,  b = sign(<t, P psi>) (P psi)_i sqrt(n) / ||P psi||,
 * and the loss of a minibatch of B rows is (1/B) sum w (a (1 + m) - b)^2 with weight w = 1 (for
 * m = 0 its mean over one iteration is 2 (1 - cos(t, P psi))). Iterations with ||P psi|| < 1e-7
 * give no rows.
 * ------------------------------------------------------------------------------------------- */
#define DMRG_MLP_IN      16
#define DMRG_MLP_HIDDEN  256
#define DMRG_MLP_PARAMS  (16 * 256 + 256 + 256 * 256 + 256 + 256 + 1)

/* New network on `device`: W1, W2 uniform in +-sqrt(6 / fan_in) from a splitmix64 stream of `seed`,
 * biases, w3 and b3 zero (so it starts as the diagonal preconditioner). */
dmrg_status dmrg_mlp_create(int32_t device, uint64_t seed, dmrg_mlp** out);
void dmrg_mlp_free(dmrg_mlp* mlp);

/* Copy the FP32 parameters out to `get` and/or in from `set` (host arrays of DMRG_MLP_PARAMS floats,
 * either may be NULL; get happens first). Setting parameters resets the Adam state. */
dmrg_status dmrg_mlp_params(dmrg_mlp* mlp, float* get, const float* set);

/* 1: FP32 debug mode (forward, backward and inference from the FP32 parameters on the vector
 * units); 0 (default): BF16 weights on the matrix cores, FP32 accumulation. */
dmrg_status dmrg_mlp_set_fp32(dmrg_mlp* mlp, int32_t fp32);

/* Features of every coefficient for residual r, Ritz vector u and Ritz value theta of handle `hop`
 * (device pointers, n_coeff doubles each): feat (device, n_coeff x 16 FP32, row-major) and the
 * diagonal correction t (device, n_coeff doubles). */
dmrg_status dmrg_mlp_features(dmrg_hop* hop, const double* r, const double* u, double theta, float* feat,
                              double* t, void* stream);

/* m (device, n FP32) = network output for n feature rows (device, n x 16 FP32). */
dmrg_status dmrg_mlp_forward(const dmrg_mlp* mlp, const float* feat, int64_t n, float* m, void* stream);

/* Loss and gradient of a minibatch (device arrays): feat n x 16, pairs n x 3 (a, b, w). grad
 * (device, DMRG_MLP_PARAMS FP32) and loss (device, 1 FP32). With lr > 0 one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected) is then taken with learning rate lr. 1 <= n <= 2^20. */
dmrg_status dmrg_mlp_grad(dmrg_mlp* mlp, const float* feat, const float* pairs, int64_t n, float lr, float* grad,
                          float* loss, void* stream);

/* Run dmrg_davidson on `hop` from psi (device, in: start vector, out: eigenvector) with `opts`
 * (its precond and mlp fields are honoured) twice: once to find psi, then again from the same start
 * vector (the solver is deterministic) recording the training pairs of every iteration into dataset
 * `slot` (0 = training, 1 = validation) of `mlp`: rows_per_iter coefficients sampled uniformly with
 * replacement (splitmix64 stream of `seed`), or all coefficients when rows_per_iter >= n_coeff.
 * Rows are appended to what the slot already holds; n_rows (may be NULL) receives the slot's new
 * size. Nothing is recorded when the first solve does not converge. Returns the Davidson status,
 * result describes the second solve. */
dmrg_status dmrg_mlp_collect(dmrg_mlp* mlp, dmrg_hop* hop, double* psi, const dmrg_dav_opts* opts, int32_t slot,
                             int32_t rows_per_iter, uint64_t seed, dmrg_dav_result* result, int64_t* n_rows,
                             void* stream);

/* Dataset slot contents: total_rows (may be NULL) receives the slot's size; rows [row0, row0+rows)
 * are copied into feat (rows x 16) and pairs (rows x 3 as a, b, w), caller-owned host or device
 * buffers (either may be NULL). Synchronizes `stream`. */
dmrg_status dmrg_mlp_dataset(const dmrg_mlp* mlp, int32_t slot, int64_t row0, int64_t rows, float* feat,
                             float* pairs, int64_t* total_rows, void* stream);

/* `steps` Adam steps on minibatches of `batch` rows drawn uniformly with replacement from slot 0
 * (splitmix64 stream of `seed`); losses (host, `steps` floats, may be NULL) receives each step's
 * minibatch loss. Synchronizes `stream`. */
dmrg_status dmrg_mlp_train(dmrg_mlp* mlp, int32_t steps, int32_t batch, float lr, uint64_t seed, float* losses,
                           void* stream);

/* Mean loss of the current network over every row of dataset `slot` (no update), and the loss of
 * the diagonal preconditioner (m = 0) on the same rows; either output may be NULL. */
dmrg_status dmrg_mlp_eval(dmrg_mlp* mlp, int32_t slot, double* loss, double* loss_diag, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DMRG_H */
