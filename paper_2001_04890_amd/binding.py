"""ctypes binding of include/dmrg.h (argument marshalling only)."""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libdmrg.so")

# torch's bundled HIP runtime must be the one in the process (libdmrg resolves libamdhip64.so.7
# by SONAME, so importing torch first makes both share a single runtime).
try:
    import torch  # noqa: F401
except ImportError:  # CPU-only environments without torch can still load the library
    torch = None

if not os.path.exists(lib_path):
    raise ImportError(f"{lib_path} is missing: build it with `python paper_2001_04890_amd/build.py` "
                      "(there is no CPU fallback)")
lib = C.CDLL(lib_path)

DMRG_OK = 0
DMRG_NOT_CONVERGED = 1
PREC_FP64 = 0
PREC_SPLIT2 = 1

# dmrg_hop_autotune: settings reported in `chosen`, in order (DMRG_AUTOTUNE_KNOBS entries)
AUTOTUNE_KNOBS = 8
_AUTOTUNE_SPLIT = ("lds_items", "lds_order", "small_shape", "split64", "six_wave", "copy_wave", "prefetch")
_AUTOTUNE_FP64 = ("lds64_items", "lds64_copy_wave", "lds64_small", "lds64_w7_cap", "big64", "max_tq", "items",
                  "order")
_KIND = {"H": 0, "C": 1, "A": 2, "B": 3, "S": 4, "U": 5, "P": 6, "Q": 7}

i32p = C.POINTER(C.c_int32)
i64p = C.POINTER(C.c_int64)
f64p = C.POINTER(C.c_double)


class Problem(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32), ("site", C.c_int32),
                ("h", f64p), ("eri", f64p)]


class OpDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32), ("n_blk", C.c_int32),
                ("sec_out", i32p), ("sec_in", i32p), ("off", i64p)]


class BlockDesc(C.Structure):
    _fields_ = [("n_sec", C.c_int32), ("qn", i32p), ("dim", i32p), ("n_ops", C.c_int32),
                ("ops", C.POINTER(OpDesc)), ("data", f64p), ("n_data", C.c_int64)]


class BuildOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("want_split", C.c_int32), ("mem_budget_bytes", C.c_int64),
                ("stream", C.c_void_p), ("share", C.c_int32)]


class DavOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("max_sub", C.c_int32), ("precision", C.c_int32),
                ("fp64_polish", C.c_int32), ("split_tol", C.c_double), ("use_graph", C.c_int32),
                ("precond", C.c_int32), ("mlp", C.c_void_p)]


class DavResult(C.Structure):
    _fields_ = [("energy", C.c_double), ("resid", C.c_double), ("iters", C.c_int32), ("matvecs", C.c_int32),
                ("matvecs_split", C.c_int32), ("t_total", C.c_double), ("t_hpsi", C.c_double),
                ("precond_fallback_iter", C.c_int32)]


class DavBatchResult(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("energy", f64p), ("resid", f64p), ("iters", i32p), ("status", i32p),
                ("n_parts", C.c_int32), ("n_converged", C.c_int32), ("matvecs", C.c_int32), ("graphs", C.c_int32),
                ("t_total", C.c_double)]


class SweepOpts(C.Structure):
    _fields_ = [("n_sweeps", C.c_int32), ("m_per_sweep", i32p), ("m_warmup", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("max_sub", C.c_int32), ("precision", C.c_int32), ("fp64_polish", C.c_int32),
                ("split_tol", C.c_double), ("seed", C.c_uint64), ("device", C.c_int32), ("stream", C.c_void_p),
                ("verbose", C.c_int32), ("keep_site", C.c_int32), ("mlp", C.c_void_p), ("mlp_from_sweep", C.c_int32),
                ("mlp_shadow", C.c_int32)]


class SweepResult(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("energies", f64p), ("discarded", f64p), ("iters", i32p), ("sites", i32p),
                ("n_solves", C.c_int32), ("n_not_converged", C.c_int32), ("energy", C.c_double),
                ("best_energy", C.c_double), ("seconds", C.c_double), ("left_block", C.POINTER(BlockDesc)),
                ("right_block", C.POINTER(BlockDesc)), ("energies_alt", f64p), ("iters_alt", i32p)]


lib.dmrg_last_error.restype = C.c_char_p
lib.dmrg_version.restype = C.c_char_p
lib.dmrg_build_blocks.argtypes = [C.POINTER(Problem), C.POINTER(BlockDesc), C.POINTER(BlockDesc),
                                  C.POINTER(BuildOpts), C.POINTER(C.c_void_p)]
lib.dmrg_build_blocks.restype = C.c_int32
lib.dmrg_hop_free.argtypes = [C.c_void_p]
lib.dmrg_hop_free.restype = None
lib.dmrg_hop_layout.argtypes = [C.c_void_p, i64p, i32p, i32p, i32p, i64p]
lib.dmrg_hop_layout.restype = C.c_int32
lib.dmrg_hop_stats.argtypes = [C.c_void_p, f64p, f64p, i64p, i64p]
lib.dmrg_hop_stats.restype = C.c_int32
lib.dmrg_hpsi.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
lib.dmrg_hpsi_batched.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                  C.c_int32, C.c_void_p]
lib.dmrg_hpsi_batched.restype = C.c_int32
lib.dmrg_hpsi.restype = C.c_int32
lib.dmrg_hpsi_graph.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
lib.dmrg_hpsi_graph.restype = C.c_int32
lib.dmrg_hop_diagonal.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
lib.dmrg_hop_diagonal.restype = C.c_int32
lib.dmrg_rdm_left_layout.argtypes = [C.c_void_p, i32p, i32p, i32p, i64p]
lib.dmrg_rdm_left_layout.restype = C.c_int32
lib.dmrg_rdm_left.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
lib.dmrg_rdm_left.restype = C.c_int32
lib.dmrg_rdm_right_layout.argtypes = [C.c_void_p, i32p, i32p, i32p, i64p]
lib.dmrg_rdm_right_layout.restype = C.c_int32
lib.dmrg_rdm_right.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
lib.dmrg_rdm_right.restype = C.c_int32
lib.dmrg_truncate.argtypes = [f64p, C.c_int32, i32p, i64p, C.c_int32, i32p, f64p, f64p, f64p]
lib.dmrg_truncate.restype = C.c_int32
lib.dmrg_renormalize_blocks.argtypes = [C.c_int32, C.c_int32, i32p, i32p, i64p, C.c_void_p, C.c_int64, C.c_int32,
                                        i32p, i32p, i64p, C.c_void_p, C.c_int64, i64p, C.c_void_p, C.c_int64,
                                        C.c_void_p]
lib.dmrg_renormalize_blocks.restype = C.c_int32
lib.dmrg_renormalize_blocks_noalloc.argtypes = lib.dmrg_renormalize_blocks.argtypes
lib.dmrg_renormalize_blocks_noalloc.restype = C.c_int32
lib.dmrg_block_grow_layout.argtypes = [C.POINTER(BlockDesc), C.c_int32, i32p, i32p, i32p]
lib.dmrg_block_grow_layout.restype = C.c_int32
lib.dmrg_block_grow.argtypes = [C.POINTER(Problem), C.POINTER(BlockDesc), C.c_int32, i32p, f64p, C.POINTER(BuildOpts),
                                C.POINTER(C.POINTER(BlockDesc))]
lib.dmrg_block_grow.restype = C.c_int32
lib.dmrg_renormalize.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.POINTER(BlockDesc)),
                                 f64p, C.c_void_p]
lib.dmrg_renormalize.restype = C.c_int32
lib.dmrg_block_free.argtypes = [C.POINTER(BlockDesc)]
lib.dmrg_block_free.restype = None
lib.dmrg_sweep.argtypes = [C.POINTER(Problem), C.POINTER(SweepOpts), C.POINTER(SweepResult)]
lib.dmrg_sweep.restype = C.c_int32
lib.dmrg_davidson.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(DavOpts), C.POINTER(DavResult), C.c_void_p]
lib.dmrg_davidson.restype = C.c_int32
lib.dmrg_davidson_batch.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(DavOpts), C.POINTER(DavBatchResult), C.c_void_p]
lib.dmrg_davidson_batch.restype = C.c_int32
lib.dmrg_hop_export_tasks.argtypes = [C.c_void_p, i64p, i32p, f64p, i64p, i32p, f64p]
lib.dmrg_hop_export_tasks.restype = C.c_int32
lib.dmrg_hop_combine.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
lib.dmrg_hop_combine.restype = C.c_int32
lib.dmrg_hop_trim.argtypes = [C.c_void_p]
lib.dmrg_hop_trim.restype = C.c_int32
lib.dmrg_hop_parts.argtypes = [C.c_void_p, i32p, i64p]
lib.dmrg_hop_parts.restype = C.c_int32
lib.dmrg_hop_autotune.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, i32p, f64p]
lib.dmrg_hop_autotune.restype = C.c_int32
lib.dmrg_mlp_create.argtypes = [C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]
lib.dmrg_mlp_create.restype = C.c_int32
lib.dmrg_mlp_free.argtypes = [C.c_void_p]
lib.dmrg_mlp_free.restype = None
lib.dmrg_mlp_params.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
lib.dmrg_mlp_params.restype = C.c_int32
lib.dmrg_mlp_set_fp32.argtypes = [C.c_void_p, C.c_int32]
lib.dmrg_mlp_set_fp32.restype = C.c_int32
lib.dmrg_mlp_features.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                  C.c_void_p]
lib.dmrg_mlp_features.restype = C.c_int32
lib.dmrg_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
lib.dmrg_mlp_forward.restype = C.c_int32
lib.dmrg_mlp_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p,
                              C.c_void_p]
lib.dmrg_mlp_grad.restype = C.c_int32
lib.dmrg_mlp_collect.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(DavOpts), C.c_int32, C.c_int32,
                                 C.c_uint64, C.POINTER(DavResult), i64p, C.c_void_p]
lib.dmrg_mlp_collect.restype = C.c_int32
lib.dmrg_mlp_dataset.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, i64p,
                                 C.c_void_p]
lib.dmrg_mlp_dataset.restype = C.c_int32
lib.dmrg_mlp_train.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_uint64, C.c_void_p, C.c_void_p]
lib.dmrg_mlp_train.restype = C.c_int32
lib.dmrg_mlp_eval.argtypes = [C.c_void_p, C.c_int32, f64p, f64p, C.c_void_p]
lib.dmrg_mlp_eval.restype = C.c_int32

PRECOND_DIAG = 0
PRECOND_MLP = 1
MLP_IN = 16
MLP_HIDDEN = 256
MLP_PARAMS = 16 * 256 + 256 + 256 * 256 + 256 + 256 + 1


def version():
    return lib.dmrg_version().decode()


class DmrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libdmrg status {status}: {msg}")
        self.status = status


def _check(st, allow=(DMRG_OK,)):
    if st not in allow:
        raise DmrgError(st, lib.dmrg_last_error().decode())
    return st


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def truncate(rho, dims, M):
    """dmrg_truncate on host arrays: rho (flat, sector blocks dims[i]^2 in order), dims, M.
    Returns (kept (n_sec,), evals list of descending arrays, vecs list of (d, d) arrays, discarded)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    off = np.concatenate([[0], np.cumsum(dims.astype(np.int64) ** 2)]).astype(np.int64)
    kept = np.zeros(dims.size, dtype=np.int32)
    evals = np.zeros(int(dims.sum()), dtype=np.float64)
    vecs = np.zeros(int(off[-1]), dtype=np.float64)
    disc = np.zeros(1, dtype=np.float64)
    _check(lib.dmrg_truncate(_ptr(rho, C.c_double), int(dims.size), _ptr(dims, C.c_int32), _ptr(off, C.c_int64),
                             int(M), _ptr(kept, C.c_int32), _ptr(evals, C.c_double), _ptr(vecs, C.c_double),
                             _ptr(disc, C.c_double)))
    e0 = np.concatenate([[0], np.cumsum(dims)])
    return (kept, [evals[e0[i]:e0[i + 1]] for i in range(dims.size)],
            [vecs[off[i]:off[i + 1]].reshape(dims[i], dims[i]) for i in range(dims.size)], float(disc[0]))


def _device_f64(t, device, what):
    """The C-ABI reads 8-byte doubles from device memory: refuse tensors of another dtype or device."""
    if torch is not None and isinstance(t, torch.Tensor):
        if t.dtype != torch.float64:
            raise TypeError(f"{what} must be float64, got {t.dtype}")
        if t.device.type != "cuda" or (device is not None and t.device.index != device):
            raise ValueError(f"{what} must be on cuda:{device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def renormalize_blocks(dims, kept, o_off, O, sec_out, sec_in, a_off, A, out_off, out, device=0, stream=None,
                       noalloc=False):
    """dmrg_renormalize_blocks (or, with noalloc, dmrg_renormalize_blocks_noalloc): index arrays on the
    host (numpy), O, A, out device tensors (float64)."""
    dims, kept = np.ascontiguousarray(dims, dtype=np.int32), np.ascontiguousarray(kept, dtype=np.int32)
    o_off = np.ascontiguousarray(o_off, dtype=np.int64)
    sec_out, sec_in = np.ascontiguousarray(sec_out, dtype=np.int32), np.ascontiguousarray(sec_in, dtype=np.int32)
    a_off, out_off = np.ascontiguousarray(a_off, dtype=np.int64), np.ascontiguousarray(out_off, dtype=np.int64)
    for t, what in ((O, "O"), (A, "A"), (out, "out")):
        _device_f64(t, device, what)
    fn = lib.dmrg_renormalize_blocks_noalloc if noalloc else lib.dmrg_renormalize_blocks
    _check(fn(int(device), int(dims.size), _ptr(dims, C.c_int32), _ptr(kept, C.c_int32),
              _ptr(o_off, C.c_int64), C.c_void_p(O.data_ptr()), int(O.numel()),
              int(sec_out.size), _ptr(sec_out, C.c_int32), _ptr(sec_in, C.c_int32),
              _ptr(a_off, C.c_int64), C.c_void_p(A.data_ptr()), int(A.numel()),
              _ptr(out_off, C.c_int64), C.c_void_p(out.data_ptr()), int(out.numel()),
              _stream_ptr(stream)))


_KIND_NAME = {v: k for k, v in _KIND.items()}


def _take_block(ptr, side, orbitals):
    """Copy a library-owned dmrg_block into a dmrg_inputs Block and release it."""
    from dmrg_inputs.blocks import Block, Op
    try:
        d = ptr.contents
        n_sec = d.n_sec
        qn = np.array([d.qn[i] for i in range(2 * n_sec)], dtype=np.int32).reshape(-1, 2)
        dim = np.array([d.dim[i] for i in range(n_sec)], dtype=np.int32)
        data = np.ctypeslib.as_array(d.data, shape=(max(1, d.n_data),))[:d.n_data].copy() if d.n_data else np.zeros(0)
        ops = []
        for k in range(d.n_ops):
            o = d.ops[k]
            blocks = {}
            for j in range(o.n_blk):
                so, si, off = o.sec_out[j], o.sec_in[j], o.off[j]
                r, c = int(dim[so]), int(dim[si])
                blocks[(so, si)] = data[off:off + r * c].reshape(r, c).copy()
            ops.append(Op(_KIND_NAME[o.kind], o.i0, o.i1, blocks))
        return Block(side=side, orbitals=tuple(orbitals), qn=qn, dim=dim, ops=ops)
    finally:
        lib.dmrg_block_free(ptr)


def block_grow_layout(block, side):
    """Enlarged sectors (qn (n, 2), dims (n,)) that ``block`` grows into (dmrg_block_grow_layout)."""
    m = _BlockMarshal(block)
    n = C.c_int32()
    _check(lib.dmrg_block_grow_layout(C.byref(m.desc), int(side), C.byref(n), None, None))
    qn = np.zeros(2 * n.value, dtype=np.int32)
    dims = np.zeros(n.value, dtype=np.int32)
    _check(lib.dmrg_block_grow_layout(C.byref(m.desc), int(side), C.byref(n), _ptr(qn, C.c_int32),
                                      _ptr(dims, C.c_int32)))
    return qn.reshape(-1, 2), dims


def block_grow(h, eri, n_alpha, n_beta, site, block, side, kept=None, O=None, device=0, stream=None):
    """dmrg_block_grow: ``block`` grown by one site at the bond (site, site+1) and renormalized by O
    (a list of per-enlarged-sector (dims, kept) arrays, or None to keep every state). Returns a Block."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    L = h.shape[0]
    prob = Problem(L, n_alpha, n_beta, site, _ptr(h, C.c_double), _ptr(eri, C.c_double))
    m = _BlockMarshal(block)
    opts = BuildOpts(device, 0, 0, _stream_ptr(stream), 0)
    kp = op = None
    if O is not None:
        kk = np.ascontiguousarray([o.shape[1] for o in O], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(o, dtype=np.float64).ravel() for o in O] + [np.zeros(0)]))
        kp, op = _ptr(kk, C.c_int32), _ptr(flat, C.c_double)
    out = C.POINTER(BlockDesc)()
    _check(lib.dmrg_block_grow(C.byref(prob), C.byref(m.desc), int(side), kp, op, C.byref(opts), C.byref(out)))
    orbitals = range(0, site + 1) if side == 0 else range(site + 1, L)
    return _take_block(out, "left" if side == 0 else "right", orbitals)


def sweep(h, eri, n_alpha, n_beta, m_per_sweep, m_warmup=None, tol=1e-8, max_iter=300, max_sub=24,
          precision=PREC_FP64, fp64_polish=False, split_tol=1e-5, seed=0, device=0, stream=None, verbose=False,
          keep_site=0, mlp=None, mlp_from_sweep=0, mlp_shadow=False):
    """dmrg_sweep: warm-up plus len(m_per_sweep) two-site sweeps. Returns a dict with the per-solve
    energies, discarded weights, iterations and bond sites, and the run's summary fields; with
    keep_site > 0 also "left" and "right", the blocks of the bond (keep_site, keep_site + 1) after the
    last sweep (dmrg_inputs Blocks). mlp: a learned preconditioner (Mlp) for the solves of sweeps
    mlp_from_sweep and later; mlp_shadow: those bonds are solved with both preconditioners on the same
    problem, the sweep continuing with the diagonal solve ("energies_alt", "iters_alt": the learned ones)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    L = h.shape[0]
    ms = np.ascontiguousarray(m_per_sweep, dtype=np.int32)
    prob = Problem(L, n_alpha, n_beta, 0, _ptr(h, C.c_double), _ptr(eri, C.c_double))
    opts = SweepOpts(int(ms.size), _ptr(ms, C.c_int32), int(m_warmup if m_warmup else ms[0]), tol, max_iter, max_sub,
                     precision, 1 if fp64_polish else 0, split_tol, seed, device, _stream_ptr(stream),
                     1 if verbose else 0, int(keep_site), mlp._h.value if mlp is not None else None,
                     int(mlp_from_sweep), 1 if mlp_shadow else 0)
    cap = int(ms.size) * (2 * L) + 2
    e = np.zeros(cap)
    d = np.zeros(cap)
    it = np.zeros(cap, dtype=np.int32)
    si = np.zeros(cap, dtype=np.int32)
    ea = np.zeros(cap)
    ia = np.zeros(cap, dtype=np.int32)
    res = SweepResult(cap, _ptr(e, C.c_double), _ptr(d, C.c_double), _ptr(it, C.c_int32), _ptr(si, C.c_int32))
    res.energies_alt = _ptr(ea, C.c_double)
    res.iters_alt = _ptr(ia, C.c_int32)
    st = _check(lib.dmrg_sweep(C.byref(prob), C.byref(opts), C.byref(res)), allow=(DMRG_OK, DMRG_NOT_CONVERGED))
    n = res.n_solves
    out = dict(energies=e[:n], discarded=d[:n], iters=it[:n], sites=si[:n], energy=res.energy,
               best_energy=res.best_energy, seconds=res.seconds, n_not_converged=res.n_not_converged,
               converged=st == DMRG_OK, energies_alt=ea[:n], iters_alt=ia[:n])
    if keep_site > 0:
        out["left"] = _take_block(res.left_block, "left", range(0, keep_site))
        out["right"] = _take_block(res.right_block, "right", range(keep_site + 2, L))
    return out


class _BlockMarshal:
    """Keeps the numpy arrays behind a BlockDesc alive."""

    def __init__(self, block):
        data, table = block.flatten()
        self.data = np.ascontiguousarray(data, dtype=np.float64)
        self.qn = np.ascontiguousarray(block.qn, dtype=np.int32).ravel()
        self.dim = np.ascontiguousarray(block.dim, dtype=np.int32)
        self.keep = []
        ops = (OpDesc * max(1, len(block.ops)))()
        for k, (op, rows) in enumerate(zip(block.ops, table)):
            so = np.array([r[0] for r in rows], dtype=np.int32)
            si = np.array([r[1] for r in rows], dtype=np.int32)
            off = np.array([r[2] for r in rows], dtype=np.int64)
            self.keep += [so, si, off]
            ops[k] = OpDesc(_KIND[op.kind], op.i0, op.i1, len(rows), _ptr(so, C.c_int32), _ptr(si, C.c_int32),
                            _ptr(off, C.c_int64))
        self.ops = ops
        self.desc = BlockDesc(block.n_sec, _ptr(self.qn, C.c_int32), _ptr(self.dim, C.c_int32), len(block.ops),
                              ops, _ptr(self.data, C.c_double), self.data.size)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Hop:
    """Handle of one bond's H.psi operator (dmrg_build_blocks), or of several merged ones."""

    @staticmethod
    def hpsi_batched(hops, xs, ys, precision=PREC_FP64, stream=None):
        """dmrg_hpsi_batched: ys[i] = H_i xs[i] for device tensors (one vector per handle), in one call."""
        n = len(hops)
        assert len(xs) == n and len(ys) == n
        for h, x, y in zip(hops, xs, ys):
            _device_f64(x, h.device, "x")
            _device_f64(y, h.device, "y")
            assert x.numel() == h.n_coeff and y.numel() == h.n_coeff
        hp = (C.c_void_p * max(n, 1))(*[h._h.value for h in hops])
        xp = (C.c_void_p * max(n, 1))(*[x.data_ptr() for x in xs])
        yp = (C.c_void_p * max(n, 1))(*[y.data_ptr() for y in ys])
        _check(lib.dmrg_hpsi_batched(hp, n, xp, yp, precision, _stream_ptr(stream)))

    @classmethod
    def combine(cls, hops, stream=None):
        """One handle computing all problems of ``hops`` in one launch sequence (dmrg_hop_combine)."""
        arr = (C.c_void_p * len(hops))(*[h._h.value for h in hops])
        handle = C.c_void_p()
        _check(lib.dmrg_hop_combine(arr, len(hops), _stream_ptr(stream), C.byref(handle)))
        self = cls.__new__(cls)
        self._h = handle
        self.device = hops[0].device
        self._load_layout()
        return self

    def __init__(self, h, eri, left, right, n_alpha, n_beta, site, device=0, want_split=False,
                 mem_budget_bytes=0, stream=None, share=False):
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        prob = Problem(h.shape[0], n_alpha, n_beta, site, _ptr(h, C.c_double), _ptr(eri, C.c_double))
        lm, rm = _BlockMarshal(left), _BlockMarshal(right)
        opts = BuildOpts(device, 1 if want_split else 0, mem_budget_bytes, _stream_ptr(stream), 1 if share else 0)
        handle = C.c_void_p()
        _check(lib.dmrg_build_blocks(C.byref(prob), C.byref(lm.desc), C.byref(rm.desc), C.byref(opts),
                                     C.byref(handle)))
        self._h = handle
        self.device = device
        self.site = site
        self.L = h.shape[0]
        self._load_layout()

    def _load_layout(self):
        handle = self._h
        n = C.c_int64()
        nb = C.c_int32()
        _check(lib.dmrg_hop_layout(handle, C.byref(n), C.byref(nb), None, None, None))
        self.n_coeff = n.value
        self.n_blocks = nb.value
        abcd = np.zeros(4 * self.n_blocks, dtype=np.int32)
        dims = np.zeros(2 * self.n_blocks, dtype=np.int32)
        offs = np.zeros(self.n_blocks, dtype=np.int64)
        _check(lib.dmrg_hop_layout(handle, None, None, _ptr(abcd, C.c_int32), _ptr(dims, C.c_int32),
                                   _ptr(offs, C.c_int64)))
        self.abcd = abcd.reshape(-1, 4)
        self.dims = dims.reshape(-1, 2)
        self.offsets = offs
        npart = C.c_int32()
        _check(lib.dmrg_hop_parts(handle, C.byref(npart), None))
        first = np.zeros(npart.value + 1, dtype=np.int64)
        _check(lib.dmrg_hop_parts(handle, None, _ptr(first, C.c_int64)))
        self.part_coeff = first

    def trim(self):
        """Release plans and tiled operator copies; the handle can then only be combined or queried."""
        _check(lib.dmrg_hop_trim(self._h))

    def autotune(self, precision=PREC_SPLIT2, reps=3, stream=None):
        """Pick the fastest H.psi launch plan (dmrg_hop_autotune); returns the chosen settings by name
        and the chosen plan's time ("ms")."""
        ch = np.zeros(AUTOTUNE_KNOBS, dtype=np.int32)
        ms = C.c_double()
        _check(lib.dmrg_hop_autotune(self._h, precision, reps, _stream_ptr(stream), _ptr(ch, C.c_int32),
                                     C.byref(ms)))
        names = _AUTOTUNE_SPLIT if precision == PREC_SPLIT2 else _AUTOTUNE_FP64
        out = {n: int(v) for n, v in zip(names, ch)}
        out["ms"] = ms.value
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.dmrg_hop_free(h)
            self._h = None

    def stats(self):
        fl, by = C.c_double(), C.c_double()
        na, nt = C.c_int64(), C.c_int64()
        _check(lib.dmrg_hop_stats(self._h, C.byref(fl), C.byref(by), C.byref(na), C.byref(nt)))
        return dict(flops=fl.value, bytes=by.value, n_alpha=na.value, n_tasks=nt.value)

    def hpsi(self, x, y, precision=PREC_FP64, stream=None):
        """y = H x for device tensors (torch, float64) of shape (n,) or (nvec, n)."""
        nvec = 1 if x.dim() == 1 else x.shape[0]
        _device_f64(x, self.device, "x")
        _device_f64(y, self.device, "y")
        assert x.numel() == nvec * self.n_coeff and y.numel() == x.numel()
        _check(lib.dmrg_hpsi(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nvec, precision,
                             _stream_ptr(stream)))

    def hpsi_graph(self, x, y, precision=PREC_FP64, stream=None):
        """Same as hpsi, replaying a cached hipGraph of the launch sequence for these buffers."""
        nvec = 1 if x.dim() == 1 else x.shape[0]
        _device_f64(x, self.device, "x")
        _device_f64(y, self.device, "y")
        assert x.numel() == nvec * self.n_coeff and y.numel() == x.numel()
        _check(lib.dmrg_hpsi_graph(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nvec, precision,
                                   _stream_ptr(stream)))

    def diagonal(self, d, stream=None):
        _device_f64(d, self.device, "d")
        assert d.numel() == self.n_coeff
        _check(lib.dmrg_hop_diagonal(self._h, C.c_void_p(d.data_ptr()), _stream_ptr(stream)))

    def _rdm_layout(self, fn):
        n = C.c_int32(0)
        _check(fn(self._h, C.byref(n), None, None, None))
        qn = np.zeros(2 * n.value, dtype=np.int32)
        dims = np.zeros(n.value, dtype=np.int32)
        off = np.zeros(n.value + 1, dtype=np.int64)
        _check(fn(self._h, C.byref(n), _ptr(qn, C.c_int32), _ptr(dims, C.c_int32), _ptr(off, C.c_int64)))
        return qn.reshape(-1, 2), dims, off

    def _rdm(self, fn, psi, rho, stream):
        _device_f64(psi, self.device, "psi")
        _device_f64(rho, self.device, "rho")
        assert psi.numel() == self.n_coeff
        _check(fn(self._h, C.c_void_p(psi.data_ptr()), C.c_void_p(rho.data_ptr()), int(rho.numel()),
                  _stream_ptr(stream)))

    def rdm_left_layout(self):
        """Sectors of rho^L: (qn (n, 2), dims (n,), offsets (n + 1,)) from dmrg_rdm_left_layout."""
        return self._rdm_layout(lib.dmrg_rdm_left_layout)

    def rdm_left(self, psi, rho, stream=None):
        """rho^L = psi psi^T per sector (dmrg_rdm_left) into the device buffer rho."""
        self._rdm(lib.dmrg_rdm_left, psi, rho, stream)

    def rdm_right_layout(self):
        """Sectors of rho^R (dmrg_rdm_right_layout)."""
        return self._rdm_layout(lib.dmrg_rdm_right_layout)

    def rdm_right(self, psi, rho, stream=None):
        """rho^R = psi^T psi per sector (dmrg_rdm_right) into the device buffer rho."""
        self._rdm(lib.dmrg_rdm_right, psi, rho, stream)

    def renormalize(self, psi, direction, m_max, stream=None, keep=True):
        """dmrg_renormalize: rho from psi, the m_max-state cut and the grown block's renormalized
        operators. direction 0 grows the left block, 1 the right block. Returns (Block, discarded);
        keep=False releases the library's block right away and returns (None, discarded)."""
        _device_f64(psi, self.device, "psi")
        assert psi.numel() == self.n_coeff
        out = C.POINTER(BlockDesc)()
        disc = C.c_double()
        _check(lib.dmrg_renormalize(self._h, C.c_void_p(psi.data_ptr()), int(direction), int(m_max), C.byref(out),
                                    C.byref(disc), _stream_ptr(stream)))
        if not keep:
            lib.dmrg_block_free(out)
            return None, disc.value
        orbitals = range(0, self.site + 1) if direction == 0 else range(self.site + 1, self.L)
        return _take_block(out, "left" if direction == 0 else "right", orbitals), disc.value

    def davidson(self, psi, tol=1e-8, max_iter=200, max_sub=24, precision=PREC_FP64, fp64_polish=False,
                 split_tol=1e-5, mlp=None, stream=None, use_graph=False):
        """In-place Davidson on the device vector psi; returns a dict of the result fields.
        ``mlp``: a Mlp network to use as the preconditioner (default: the diagonal one).
        ``use_graph``: run the matvecs through cached hipGraphs (dmrg_hpsi_graph)."""
        _device_f64(psi, self.device, "psi")
        assert psi.numel() == self.n_coeff
        o = _dav_opts(tol, max_iter, max_sub, precision, fp64_polish, split_tol, mlp, use_graph)
        r = DavResult()
        st = _check(lib.dmrg_davidson(self._h, C.c_void_p(psi.data_ptr()), C.byref(o), C.byref(r),
                                      _stream_ptr(stream)), allow=(DMRG_OK, DMRG_NOT_CONVERGED))
        return _dav_result(r, st)

    def davidson_batch(self, psi, tol=1e-8, max_iter=200, max_sub=24, precision=PREC_FP64, fp64_polish=False,
                       split_tol=1e-5, use_graph=True, stream=None):
        """dmrg_davidson_batch: every part of this (merged) handle solved in lockstep on the device; psi
        (device, n_coeff doubles) in: start vectors, out: Ritz vectors. Returns per-part arrays
        (energy, resid, iters, status: 0 converged, 1 not converged, 2 stalled) and the run's counts."""
        _device_f64(psi, self.device, "psi")
        assert psi.numel() == self.n_coeff
        P = len(self.part_coeff) - 1
        o = _dav_opts(tol, max_iter, max_sub, precision, fp64_polish, split_tol, None, use_graph)
        e, rr = np.zeros(P), np.zeros(P)
        it, stt = np.zeros(P, dtype=np.int32), np.zeros(P, dtype=np.int32)
        r = DavBatchResult(P, _ptr(e, C.c_double), _ptr(rr, C.c_double), _ptr(it, C.c_int32), _ptr(stt, C.c_int32))
        st = _check(lib.dmrg_davidson_batch(self._h, C.c_void_p(psi.data_ptr()), C.byref(o), C.byref(r),
                                            _stream_ptr(stream)), allow=(DMRG_OK, DMRG_NOT_CONVERGED))
        return dict(energy=e, resid=rr, iters=it, status=stt, n_converged=r.n_converged, matvecs=r.matvecs,
                    graphs=r.graphs, t_total=r.t_total, converged=st == DMRG_OK)

    def export_tasks(self):
        """Host-side task list and matrix definitions (introspection of the term generator)."""
        nt, nterm = C.c_int64(), C.c_int64()
        _check(lib.dmrg_hop_export_tasks(self._h, C.byref(nt), None, None, C.byref(nterm), None, None))
        quads = np.zeros(4 * nt.value, dtype=np.int32)
        f = np.zeros(nt.value)
        ti = np.zeros(4 * nterm.value, dtype=np.int32)
        tc = np.zeros(nterm.value)
        _check(lib.dmrg_hop_export_tasks(self._h, None, _ptr(quads, C.c_int32), _ptr(f, C.c_double), None,
                                         _ptr(ti, C.c_int32), _ptr(tc, C.c_double)))
        return quads.reshape(-1, 4), f, ti.reshape(-1, 4), tc


def _dav_opts(tol, max_iter, max_sub, precision, fp64_polish, split_tol, mlp, use_graph=False):
    return DavOpts(tol, max_iter, max_sub, precision, 1 if fp64_polish else 0, split_tol, 1 if use_graph else 0,
                   PRECOND_MLP if mlp is not None else PRECOND_DIAG, mlp._h.value if mlp is not None else None)


def _dav_result(r, st):
    return dict(energy=r.energy, resid=r.resid, iters=r.iters, matvecs=r.matvecs, matvecs_split=r.matvecs_split,
                t_total=r.t_total, t_hpsi=r.t_hpsi, precond_fallback_iter=r.precond_fallback_iter,
                converged=st == DMRG_OK)


class Mlp:
    """Learned Davidson preconditioner (dmrg_mlp_*): network, Adam state and two datasets."""

    def __init__(self, device=0, seed=0):
        handle = C.c_void_p()
        _check(lib.dmrg_mlp_create(device, seed, C.byref(handle)))
        self._h = handle
        self.device = device

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.dmrg_mlp_free(h)
            self._h = None

    def get_params(self):
        p = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib.dmrg_mlp_params(self._h, p.ctypes.data, None))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == MLP_PARAMS
        _check(lib.dmrg_mlp_params(self._h, None, p.ctypes.data))

    def set_fp32(self, on):
        _check(lib.dmrg_mlp_set_fp32(self._h, 1 if on else 0))

    @staticmethod
    def features(hop, r, u, theta, feat, t, stream=None):
        """Features (n x 16 float32) and diagonal correction t of (r, u, theta) on hop's layout."""
        assert feat.numel() == hop.n_coeff * MLP_IN and t.numel() == hop.n_coeff
        _check(lib.dmrg_mlp_features(hop._h, C.c_void_p(r.data_ptr()), C.c_void_p(u.data_ptr()), float(theta),
                                     C.c_void_p(feat.data_ptr()), C.c_void_p(t.data_ptr()), _stream_ptr(stream)))

    def forward(self, feat, out, stream=None):
        n = feat.numel() // MLP_IN
        assert out.numel() == n and feat.is_contiguous() and out.is_contiguous()
        _check(lib.dmrg_mlp_forward(self._h, C.c_void_p(feat.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)))

    def grad(self, feat, pairs, grad, loss, lr=0.0, stream=None):
        """Loss and parameter gradient of a minibatch; with lr > 0 also one Adam step."""
        n = feat.numel() // MLP_IN
        assert pairs.numel() == 3 * n and grad.numel() == MLP_PARAMS and loss.numel() >= 1
        _check(lib.dmrg_mlp_grad(self._h, C.c_void_p(feat.data_ptr()), C.c_void_p(pairs.data_ptr()), n, lr,
                                 C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()), _stream_ptr(stream)))

    def collect(self, hop, psi, slot=0, rows_per_iter=4096, seed=0, tol=1e-10, max_iter=300, max_sub=24,
                precision=PREC_FP64, fp64_polish=False, split_tol=1e-5, use_mlp=False, stream=None):
        """Davidson on hop from psi, recording training pairs into dataset ``slot``."""
        o = _dav_opts(tol, max_iter, max_sub, precision, fp64_polish, split_tol, self if use_mlp else None)
        r = DavResult()
        rows = C.c_int64()
        st = _check(lib.dmrg_mlp_collect(self._h, hop._h, C.c_void_p(psi.data_ptr()), C.byref(o), slot,
                                         rows_per_iter, seed, C.byref(r), C.byref(rows), _stream_ptr(stream)),
                    allow=(DMRG_OK, DMRG_NOT_CONVERGED))
        out = _dav_result(r, st)
        out["rows"] = rows.value
        return out

    def dataset_rows(self, slot=0):
        rows = C.c_int64()
        _check(lib.dmrg_mlp_dataset(self._h, slot, 0, 0, None, None, C.byref(rows), None))
        return rows.value

    def dataset(self, slot=0, row0=0, rows=None):
        """Copy of dataset rows as numpy arrays (features n x 16, pairs n x 3)."""
        total = self.dataset_rows(slot)
        rows = total - row0 if rows is None else rows
        feat = np.zeros((rows, MLP_IN), dtype=np.float32)
        pairs = np.zeros((rows, 3), dtype=np.float32)
        _check(lib.dmrg_mlp_dataset(self._h, slot, row0, rows, feat.ctypes.data, pairs.ctypes.data, None, None))
        return feat, pairs

    def train(self, steps, batch=4096, lr=1e-3, seed=0, stream=None):
        losses = np.zeros(max(steps, 1), dtype=np.float32)
        _check(lib.dmrg_mlp_train(self._h, steps, batch, lr, seed, losses.ctypes.data, _stream_ptr(stream)))
        return losses[:steps]

    def eval(self, slot=1, stream=None):
        """(mean loss of the network, mean loss of the diagonal preconditioner) over dataset ``slot``."""
        a, b = C.c_double(), C.c_double()
        _check(lib.dmrg_mlp_eval(self._h, slot, C.byref(a), C.byref(b), _stream_ptr(stream)))
        return a.value, b.value
