"""acch_residual_noalloc (the entry point that allocates nothing: a static device
array holds its reduction scratch) against acch_residual on the same inputs, through
the C ABI, on two calls in a row, the second on a smaller grid."""
import ctypes

import numpy as np
import pytest

from acch_inputs import perturbed_pair

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2007_04560_amd as pkg  # noqa: E402
from paper_2007_04560_amd import Solver  # noqa: E402


def _vec(u, v):
    return torch.as_tensor(np.ascontiguousarray(np.concatenate([u.ravel(), v.ravel()]))).cuda()


def _case(shape, bc, seed, dt):
    lib = pkg.load_library()
    u1, v1, u0, v0 = perturbed_pair(shape, seed, amp=0.03)
    X, Xn = _vec(u1, v1), _vec(u0, v0)
    kw = dict(bc=bc, alpha=4.0, beta=2.0, gamma=0.005, rho=0.001, sub=(2, 2), overlap=1)
    with Solver(u0, v0, **kw) as s:
        F_ref, f2_ref, bad_ref = s.residual(X, Xn, dt)
        torch.cuda.synchronize()
        F_ref = F_ref.clone()
    p = pkg.make_params(shape, **kw)
    p.stream = torch.cuda.current_stream().cuda_stream
    F = torch.full_like(X, float("nan"))
    f2, bad = ctypes.c_double(), ctypes.c_int()
    rc = lib.acch_residual_noalloc(ctypes.byref(p), X.data_ptr(), Xn.data_ptr(), dt, F.data_ptr(),
                                   ctypes.byref(f2), ctypes.byref(bad))
    assert rc == 0, lib.acch_last_error()
    # the same kernels on the same inputs: identical values, bit for bit
    assert torch.equal(F, F_ref)
    assert f2.value == f2_ref and bad.value == bad_ref


def test_noalloc_residual_matches_the_context_entry_point_twice():
    _case((96, 130), "neumann", 5, 3e-3)      # 17 x 12 tiles
    _case((37, 29), "periodic", 6, 2e-3)      # smaller grid: fewer partials than the first call


def test_noalloc_rejects_grids_beyond_the_scratch():
    lib = pkg.load_library()
    p = pkg.make_params((4096, 4100), bc="neumann")
    F = torch.empty(1, dtype=torch.float64, device="cuda")
    rc = lib.acch_residual_noalloc(ctypes.byref(p), F.data_ptr(), F.data_ptr(), 1e-3, F.data_ptr(), None, None)
    assert rc == 1   # ACCH_EINVAL
