"""dmpt_response_static (the responses with the library's own device scratch,
for callers that cannot allocate) against dmpt_response with a caller
workspace: the same kernels and partial layout, so the results must be
identical bit for bit.  Two calls in a row, the second with a smaller input
(the scratch keeps the first call's contents).  Sizes beyond the 4 MiB
scratch are refused before any device call (tests/test_abi.py)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call_static(lib, chi, h1):
    import torch
    k, p, n = chi.shape[0], h1.shape[0], chi.shape[-1]
    out = (C.c_double * (k * p))()
    st = lib.dmpt_response_static(C.c_void_p(chi.data_ptr()), k, C.c_void_p(h1.data_ptr()), p, n, out,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, np.array(out[:]).reshape(k, p)


def test_static_response_matches_workspace_response(gpu):
    import torch

    import paper_2409_17033_amd as dm
    lib = dm.load()
    rng = np.random.default_rng(7)
    for n, k, p in [(1000, 3, 9), (257, 2, 3)]:          # second call smaller
        chi = torch.from_numpy(rng.normal(size=(k, n, n)).astype(np.float32)).to(gpu)
        h1 = torch.from_numpy(rng.normal(size=(p, n, n)).astype(np.float32)).to(gpu)
        st, got = _call_static(lib, chi, h1)
        assert st == 0, dm._lib.last_error()
        ref = dm.response(chi, h1)
        print(f"n={n} k={k} p={p}: max |static - workspace| = {np.max(np.abs(got - ref)):.3e}")
        assert np.array_equal(got, ref)
        exact = np.einsum("kij,pij->kp", chi.double().cpu().numpy(), h1.double().cpu().numpy())
        assert np.allclose(got, exact, rtol=1e-12, atol=1e-9 * n)
