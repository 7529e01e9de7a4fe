"""The allocation-free solve (ifmm_solve_noalloc) against ifmm_solve (collected last on purpose).

Both run the same kernels in the same order, ifmm_solve with its own work
vector (and a captured graph), ifmm_solve_noalloc with the library's fixed
per-device array, so the solutions must agree bit for bit.  Two calls in a
row, the second on a smaller problem with fewer right-hand sides, check that
the shared array is cleared where it must be."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _factored(shape, N, seed, leaf):
    from paper_1905_10602_amd import IFMM
    kw = {"jitter": 0.05} if shape == "ellipsoid" else {}
    pts = synth.geometry_points(shape, N, seed, **kw)
    return IFMM(pts, 1e-6, 3, diag=synth.laplace_self_term(N), leaf_max=leaf).factor()


def _noalloc(h, B):
    """B: (k, N) contiguous device tensor (column-major N x k); returns X like it."""
    import torch
    from paper_1905_10602_amd.ifmm import _check, _ptr, load_library
    X = torch.full_like(B, float("nan"))
    _check(load_library().ifmm_solve_noalloc(h._h, _ptr(B), _ptr(X), B.shape[0], h.N))
    torch.cuda.synchronize()
    return X


def _reference(h, B):
    import torch
    from paper_1905_10602_amd.ifmm import _check, _ptr, load_library
    X = torch.empty_like(B)
    _check(load_library().ifmm_solve(h._h, _ptr(B), _ptr(X), B.shape[0], h.N, 1))
    return X


def test_noalloc_solve_equals_solve_twice_then_smaller():
    import torch
    from paper_1905_10602_amd import IfmmError
    from paper_1905_10602_amd.ifmm import _check, _ptr, load_library
    lib = load_library()
    assert lib.ifmm_solve_noalloc_max_bytes() == 256 << 20
    cases = [("ellipsoid", 3000, 7, 32, 4), ("sphere", 1500, 3, 24, 2)]
    for shape, N, seed, leaf, k in cases:
        print(f"case noalloc {shape} N={N} nrhs={k}", flush=True)
        h = _factored(shape, N, seed, leaf)
        b = synth.uniform_rhs(N, k, 40 + seed)
        B = torch.from_numpy(np.ascontiguousarray(b.T)).cuda()
        ref = _reference(h, B).cpu().numpy()
        got = _noalloc(h, B).cpu().numpy()
        assert np.array_equal(got, ref)
        xo = h.solve(b)  # host path, for a residual-free sanity check of the layout
        assert np.array_equal(got.T, xo)
    # a request beyond the fixed array is refused before any device work
    with pytest.raises(IfmmError) as e:
        _check(lib.ifmm_solve_noalloc(h._h, _ptr(B), _ptr(B), 1 << 20, h.N))
    assert e.value.status == "IFMM_EINVAL" and "bytes" in str(e.value)
