"""rac_permutation_noalloc (the allocation-free partition draw) through the C ABI,
against rac_permutation (the allocating entry point) and the oracle: bit for
bit, on two calls in a row (the second smaller, so stale scratch contents of
the first call must not leak into it), plus the size limit."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from paper_1907_01995_amd import racmb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _noalloc(lib, seed, inst, it, n, out):
    code = lib.rac_permutation_noalloc(seed, inst, it, n, C.c_void_p(out.data_ptr()),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return code


def test_noalloc_permutation_matches_allocating_entry_point():
    lib = racmb.load()
    out = torch.full((racmb.NOALLOC_MAX_N,), -1, dtype=torch.int32, device="cuda")
    cases = [(7, 3, 11, 100000), (7, 3, 12, 4097), (123456789, 0, 0, racmb.NOALLOC_MAX_N), (5, 9, 2, 1000),
             (5, 9, 3, 1), (2**63 + 5, 255, 4999, 65537)]
    for seed, inst, it, n in cases:
        print("noalloc case", seed, inst, it, n, flush=True)
        out.fill_(-1)
        assert _noalloc(lib, seed, inst, it, n, out) == racmb.RAC_OK
        got = out[:n].cpu().numpy()
        ref = racmb.permutation(seed, inst, it, n).cpu().numpy()
        assert np.array_equal(got, ref)
        assert np.all(out[n:].cpu().numpy() == -1)       # nothing written past n
        if n <= 100000:
            assert np.array_equal(got, O.permutation(seed, inst, it, n))


def test_noalloc_permutation_rejects_sizes_beyond_the_scratch():
    lib = racmb.load()
    out = torch.empty(4, dtype=torch.int32, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.rac_permutation_noalloc(1, 0, 0, racmb.NOALLOC_MAX_N + 1, C.c_void_p(out.data_ptr()), st) == \
        racmb.RAC_ERR_ARG
    assert lib.rac_permutation_noalloc(1, 0, 0, 0, C.c_void_p(out.data_ptr()), st) == racmb.RAC_ERR_ARG
    assert lib.rac_permutation_noalloc(1, 0, -1, 4, C.c_void_p(out.data_ptr()), st) == racmb.RAC_ERR_ARG
    assert lib.rac_permutation_noalloc(1, 0, 0, 4, None, st) == racmb.RAC_ERR_ARG
