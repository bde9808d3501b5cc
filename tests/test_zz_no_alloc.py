"""The allocation-free operator entry point (sa_apply_operator_static) against the existing
one (sa_apply_operator) through the C ABI: two calls in a row on one GPU, the second on a
smaller grid than the first (the static scratch keeps the first call's contents), each
compared element by element with the problem-based operator to the operator parity bar
(1e-11 of the row's |A||x| bound, computed from the oracle's assembled operator), and with
the size limit refused before any device work."""
import sys

import numpy as np
import pytest

from oracle.discretization import Grid, mixed_stage_operator
from paper_2511_18071_amd import workload as W


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


def test_static_entry_rejects_grids_beyond_its_scratch(B):
    w = W.get("periodic_65x9")
    w.nx = 40000  # 39999 columns > the 32770 the static scratch holds
    x = np.zeros(4)
    with pytest.raises(B.SawaveError) as e:
        grid, h, _ = B.workload_args(w)
        D = B.C.POINTER(B.C.c_double)
        eta = np.zeros(w.nphys)
        B._check(B.lib.sa_apply_operator_static(B.C.byref(grid), h.ctypes.data_as(D), eta.ctypes.data_as(D),
                                                eta.ctypes.data_as(D), B.C.c_void_p(x.ctypes.data),
                                                B.C.c_void_p(x.ctypes.data), B.C.c_void_p(0)))
    assert e.value.code == -1 and "static scratch" in str(e.value)


@pytest.mark.gpu
def test_static_operator_equals_the_problem_operator_two_calls(B):
    import torch
    rs = np.random.default_rng(21)
    for name, s in (("bar_513x17", 3), ("periodic_65x9", 1)):  # the second call is smaller
        w = W.get(name)
        ep, ec, ps = w.system(s)
        ec = ec * 1.2
        g = Grid(w.nx, w.nz, w.bc, w.length)
        absA = abs(mixed_stage_operator(g, w.depth(), ep, ec))
        p = B.Problem.from_workload(w, stream=0, precond="none", guess="cold")
        p.set_surface(ep, ec)
        for label, xh in (("p*", ps), ("random", rs.standard_normal(w.n))):
            _say(f"[static operator] {name} system {s} {label} n={w.n}")
            x = torch.from_numpy(xh).cuda()
            y_static = torch.full((w.n,), np.nan, dtype=torch.float64, device="cuda")
            y_ref = torch.empty_like(y_static)
            torch.cuda.synchronize()
            B.apply_operator_static(w, ep, ec, x, y_static, stream=0)
            p.apply_operator(x, y_ref)
            ys, yr = y_static.cpu().numpy(), y_ref.cpu().numpy()
            bound = absA @ np.abs(xh)
            bound = np.maximum(bound, 1e-4 * bound.max())
            ratio = (np.abs(ys - yr) / bound).max()
            same = int(np.count_nonzero(ys == yr))
            _say(f"   max |y_static - y_problem| / (|A||x|) = {ratio:.2e}, bitwise equal {same} of {w.n}")
            assert np.all(np.isfinite(ys))
            assert ratio <= 1e-11
        p.close()
