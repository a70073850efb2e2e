"""bkwd_true_residual_noalloc (the entry point for callers that cannot
allocate) against bkwd_true_residual, through the C ABI, on two calls in a
row: a 16^3 x 32 lattice with 12 columns (two-stage reduction of 1023
partial records), then a smaller 4^4 lattice with 3 columns, which reuses
the same static device array."""
import ctypes

import numpy as np
import pytest

import synthetic as S
from oracle import dirac, solvers
from tests.gpu_util import lattice, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(lat, B, X):
    from paper_0903_4936_amd import bkwd
    L = B.shape[-1]
    out = (ctypes.c_double * L)()
    code = bkwd.lib().bkwd_true_residual_noalloc(lat._h, L, ctypes.c_void_p(B.data_ptr()),
                                                 ctypes.c_void_p(X.data_ptr()), out, None)
    assert code == bkwd.OK, bkwd.last_error()
    return np.array(out[:L])


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_workspace_entry(order):
    import torch
    cases = [((16, 16, 16, 32), 12, 0.135), ((4, 4, 4, 4), 3, 0.125)]
    for dims, L, kappa in cases:
        U = S.gauge_links(dims, 0.3, 17)
        B = S.gaussian_sources(dims, L, 18)
        # an approximate solution, so that the residual is far above rounding level
        X = 0.9 * B + 1e-3 * S.gaussian_sources(dims, L, 19)
        lat = lattice(U, kappa, 1.6)
        Bd, Xd = to_dev(B), to_dev(X)
        ref = lat.true_residual(Bd, Xd)
        got = _noalloc(lat, Bd, Xd)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(got)) and got.shape == (L,)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max(), (dims, got, ref)
        if dims == (4, 4, 4, 4):
            N = 12 * S.volume(dims)
            oracle = solvers.true_residual(dirac.as_matrix_operator(U, kappa, 1.6), B.reshape(N, L),
                                           X.reshape(N, L))
            assert np.allclose(got, oracle, rtol=1e-12, atol=0)


def test_noalloc_rejects_bad_arguments():
    from paper_0903_4936_amd import bkwd
    dims = (4, 4, 2, 2)
    lat = lattice(S.gauge_links(dims, 0.4, 5), 0.125, 1.0)
    B = to_dev(S.gaussian_sources(dims, 2, 6))
    out = (ctypes.c_double * 65)()
    lib = bkwd.lib()
    assert lib.bkwd_true_residual_noalloc(lat._h, 65, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                          out, None) == bkwd.EINVAL
    assert lib.bkwd_true_residual_noalloc(lat._h, 2, None, ctypes.c_void_p(B.data_ptr()), out,
                                          None) == bkwd.EINVAL
    assert lib.bkwd_true_residual_noalloc(None, 2, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                          out, None) == bkwd.EINVAL
