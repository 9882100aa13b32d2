"""dmrg_renormalize_blocks_noalloc (the entry point that allocates no device memory) against
dmrg_renormalize_blocks, through the C-ABI: the same kernels in the same order, so the outputs must be
equal bit for bit, on two calls in a row (the second smaller, reusing the fixed scratch that still
holds the first call's contents), plus its size limit and argument checks.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
lib_mod = pytest.importorskip("paper_2001_04890_amd")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def make_case(rng, dims, kept):
    Os = [np.linalg.qr(rng.normal(size=(d, d)))[0][:, :k] if d else np.zeros((0, 0)) for d, k in zip(dims, kept)]
    n = len(dims)
    blocks = [(so, si, rng.normal(size=(dims[so], dims[si]))) for so in range(n) for si in range(n)
              if (so + 2 * si) % 3 != 1]
    o_off = np.concatenate([[0], np.cumsum([d * k for d, k in zip(dims, kept)])]).astype(np.int64)
    O = np.concatenate([o.ravel() for o in Os] + [np.zeros(1)])
    a_off = np.concatenate([[0], np.cumsum([A.size for _, _, A in blocks])]).astype(np.int64)
    A = np.concatenate([A.ravel() for _, _, A in blocks])
    sizes = [kept[so] * kept[si] for so, si, _ in blocks]
    out_off = np.concatenate([[0], np.cumsum([s + 2 for s in sizes])]).astype(np.int64)
    ref = [Os[so].T @ A_ @ Os[si] for so, si, A_ in blocks]
    return dict(dims=dims, kept=kept, o_off=o_off[:-1], O=torch.as_tensor(O, device=DEV),
                sec_out=[b[0] for b in blocks], sec_in=[b[1] for b in blocks], a_off=a_off[:-1],
                A=torch.as_tensor(A, device=DEV), out_off=out_off[:-1]), int(out_off[-1]), sizes, ref


def run(args, out_len, noalloc):
    out = torch.full((out_len,), float("nan"), dtype=torch.float64, device=DEV)
    lib_mod.renormalize_blocks(**args, out=out, noalloc=noalloc)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_against_numpy(got, args, sizes, ref):
    scale = max(float(np.abs(r).max(initial=0.0)) for r in ref) or 1.0
    for b, (sz, r) in enumerate(zip(sizes, ref)):
        o = int(args["out_off"][b])
        if sz:
            assert np.abs(got[o:o + sz].reshape(r.shape) - r).max() < 1e-12 * scale * 10
        assert np.all(np.isnan(got[o + sz:o + sz + 2]))


def test_noalloc_equals_allocating_entry_point_twice():
    rng = np.random.default_rng(31)
    # first call: sectors of 1 .. 260 states (several 256-element chunks, ragged), second call smaller
    for step, (dims, kept) in enumerate((([1, 17, 64, 130, 260, 90], [1, 5, 64, 33, 120, 0]),
                                         ([9, 40, 3], [4, 40, 2]))):
        args, out_len, sizes, ref = make_case(rng, dims, kept)
        print(f"[noalloc] call {step}: dims {dims} kept {kept}, {len(sizes)} blocks", flush=True)
        want = run(args, out_len, noalloc=False)
        got = run(args, out_len, noalloc=True)
        assert np.array_equal(got, want, equal_nan=True)
        check_against_numpy(got, args, sizes, ref)


def test_noalloc_rejects_work_beyond_its_scratch():
    rng = np.random.default_rng(32)
    # one 3000 x 3000 block keeping 3000 states: T alone is 72 MB > 64 MiB
    d = 3000
    O = torch.as_tensor(rng.normal(size=d * d), device=DEV)
    A = torch.as_tensor(rng.normal(size=d * d), device=DEV)
    out = torch.zeros(d * d, dtype=torch.float64, device=DEV)
    args = dict(dims=[d], kept=[d], o_off=[0], O=O, sec_out=[0], sec_in=[0], a_off=[0], A=A, out_off=[0], out=out)
    with pytest.raises(lib_mod.DmrgError) as e:
        lib_mod.renormalize_blocks(**args, noalloc=True)
    assert e.value.status == -3 and "scratch" in str(e.value)
    assert float(out.abs().max()) == 0.0                      # nothing was launched
    # the same arguments with a block that fits still work afterwards
    small = dict(args, dims=[40], kept=[30])
    got = torch.full((900,), float("nan"), dtype=torch.float64, device=DEV)
    lib_mod.renormalize_blocks(**{**small, "out": got}, noalloc=True)
    Om = O[:1200].cpu().numpy().reshape(40, 30)
    Am = A[:1600].cpu().numpy().reshape(40, 40)
    assert np.abs(got.cpu().numpy().reshape(30, 30) - Om.T @ Am @ Om).max() < 1e-10


def test_noalloc_argument_errors_match():
    rng = np.random.default_rng(33)
    args, out_len, sizes, ref = make_case(rng, [5, 7], [3, 7])
    out = torch.zeros(out_len, dtype=torch.float64, device=DEV)
    for noalloc in (False, True):
        with pytest.raises(lib_mod.DmrgError) as e:
            lib_mod.renormalize_blocks(**{**args, "kept": [6, 7]}, out=out, noalloc=noalloc)
        assert e.value.status == -1
        with pytest.raises(lib_mod.DmrgError) as e:
            lib_mod.renormalize_blocks(**args, out=out[:out_len - 3], noalloc=noalloc)
        assert e.value.status == -2
