"""The allocation-free variant of the diagnostics against the allocating entry point.

dgns_diagnostics_noalloc runs the same kernels as dgns_diagnostics with its partial sums
in the library's static device workspace and writes the eight diagnostics to a device
array without synchronising; two calls in a row, the second on a smaller mesh, must give
exactly (bitwise) what dgns_diagnostics returns, and a mesh beyond the workspace's
capacity must be rejected before anything is launched.
"""
import ctypes
import math

import pytest
import torch

from tests.gpu_cases import announce, make_pair, tgv_input

pytestmark = pytest.mark.gpu


def _noalloc(lib):
    return lib.dgns_diagnostics_noalloc


@pytest.mark.parametrize("with_L", [True, False])
def test_noalloc_diagnostics_match_the_allocating_entry_point(with_L):
    from paper_1806_03095_amd import binding
    for n, k, nq in (((6, 5, 4), 3, 6), ((3, 2, 2), 2, 4)):          # the second call on fewer cells
        announce("no-alloc diagnostics n=%s k=%d nq=%d with_L=%s" % (n, k, nq, with_L))
        oop, gop = make_pair(n, k, nq)
        U = tgv_input(oop, seed=3).to("cuda").contiguous()
        L = gop.apply(U) if with_L else None
        host = (ctypes.c_double * 8)()
        Lp = ctypes.c_void_p(L.data_ptr()) if with_L else None
        assert gop.lib.dgns_diagnostics(gop.h, ctypes.c_void_p(U.data_ptr()), Lp, host) == binding.OK
        dev = torch.full((8,), 12345.0, dtype=torch.float64, device="cuda")
        rc = _noalloc(gop.lib)(gop.h, ctypes.c_void_p(U.data_ptr()), Lp, ctypes.c_void_p(dev.data_ptr()))
        assert rc == binding.OK, gop.lib.dgns_last_error()
        torch.cuda.synchronize()
        got = dev.cpu().tolist()
        want = list(host)
        for i in range(8):
            if i == 2 and not with_L:
                assert math.isnan(got[i]) and math.isnan(want[i])
            else:
                assert got[i] == want[i], (i, got, want)
        gop.close()


def test_noalloc_diagnostics_reject_a_mesh_beyond_the_workspace():
    from paper_1806_03095_amd import binding
    announce("no-alloc diagnostics: 65x64x64 cells rejected")
    oop_n = (65, 64, 64)
    from paper_1806_03095_amd import Operator
    gop = Operator(1, 2, oop_n, (0.0,) * 3, (1.0,) * 3, mu=1e-3, lam=1e-3)
    U = torch.ones(gop.shape, dtype=torch.float64, device="cuda")
    dev = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    rc = _noalloc(gop.lib)(gop.h, ctypes.c_void_p(U.data_ptr()), None, ctypes.c_void_p(dev.data_ptr()))
    assert rc == binding.EINVAL
    assert b"at most" in gop.lib.dgns_last_error()
    torch.cuda.synchronize()
    assert dev.cpu().tolist() == [7.0] * 8
    gop.close()
