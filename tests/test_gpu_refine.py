"""GPU parity of the mixed-precision path (FP32 inner GMRES, FP64 refinement) through the C ABI.

Inputs are seeded and synthetic (paper_2511_18071_amd.workload); b = A p* is formed by the
oracle. Tolerances follow from FP32 arithmetic (unit roundoff u = 2^-24):

* FP32 operator: |y_gpu - y_oracle|_i <= 1e-5 max((|A||x|)_i, 1e-4 max_j (|A||x|)_j): each
  row sums ~100 rounded products of rounded coefficients (bound ~100 u = 6e-6 relative to
  |A||x|), the oracle is exact FP64;
* FP32 V-cycle: max(1e-5, 8 kappa(M_c) u) max|z| against the FP64 oracle V-cycle (the
  coarsest explicit inverse is rounded to FP32, which limits it to kappa(M_c) u);
* refinement solves: every solve converged (status 0) with relative residual <= rtol = 1e-10,
  recomputed on the CPU with the oracle's FP64 operator; solution within 1e-7 relative of the
  oracle's own refinement sequence (both are converged to 1e-10; decisions are not compared,
  the two sides round differently in FP32).
"""
import sys

import numpy as np
import pytest

from oracle import precond as opc
from oracle.discretization import Grid, mixed_stage_operator
from oracle.sequence import Simulation
from paper_2511_18071_amd import workload as W

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_2511_18071_amd import binding
    return binding


def _workload(name):
    if name == "walls_131x9":  # ragged last operator tile
        w = W.get("bar_65x9")
        w.nx = 131
        return w
    return W.get(name)


@pytest.mark.parametrize("name", ["periodic_65x9", "bar_65x9", "walls_131x9", "bar_513x17"])
def test_operator_f32_parity(B, name):
    w = _workload(name)
    _say(f"[operator f32] {name} n={w.n}")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    p = B.Problem.from_workload(w, stream=0, precision="fp32_ir")
    rs = np.random.default_rng(4)
    worst = 0.0
    for s in (1, 4):
        ep, ec, ps = w.system(s)
        A = mixed_stage_operator(g, w.depth(), ep, ec)
        p.set_surface(ep, ec)
        for x in (ps, rs.standard_normal(w.n)):
            x32 = x.astype(np.float32)
            y = p.apply_operator_f32(x32).astype(np.float64)
            ref = A @ x32.astype(np.float64)
            bound = abs(A) @ np.abs(x32.astype(np.float64))
            bound = np.maximum(bound, 1e-4 * bound.max())
            ratio = (np.abs(y - ref) / bound).max()
            worst = max(worst, ratio)
            _say(f"   system {s}: max err/(|A||x|) {ratio:.3e}")
    p.close()
    assert worst <= 1e-5, worst


@pytest.mark.parametrize("name,cmax", [("periodic_65x9", 40), ("bar_65x9", 50), ("bar_513x17", 700),
                                       ("periodic_65x9", 700), ("periodic_257x33", 200)])
def test_precond_f32_parity(B, name, cmax):
    w = W.get(name)
    _say(f"[precond f32] {name} coarse_max={cmax}")
    g = Grid(w.nx, w.nz, w.bc, w.length)
    minv = opc.make(g, w.depth(), "mg", 1, w.nu2, coarse_max=cmax)  # the workload's V(1, nu2)
    kappa = np.linalg.cond(minv.levels[-1]["m"].toarray())
    tol = max(1e-5, 8.0 * kappa * U32)
    p = B.Problem.from_workload(w, stream=0, precision="fp32_ir", coarse_max=cmax)
    v = np.random.default_rng(6).standard_normal(w.n).astype(np.float32)
    z = p.apply_precond_f32(v).astype(np.float64)
    ref = minv(v.astype(np.float64))
    err = np.abs(z - ref).max() / np.abs(ref).max()
    _say(f"   rel err {err:.3e} (tol {tol:.1e}, kappa(M_c) {kappa:.2e})")
    p.close()
    assert err <= tol


@pytest.mark.parametrize("name,nsys,kw", [("periodic_65x9", 10, {}), ("bar_65x9", 10, dict(coarse_max=50)),
                                          ("bar_513x17", 8, {}), ("periodic_65x9", 5, dict(guess="cold"))])
def test_refinement_sequence(B, name, nsys, kw):
    w = W.get(name)
    rtol = 1e-10
    _say(f"[refine] {name} nsys={nsys} {kw}")
    ora = Simulation.from_workload(w, rtol=rtol, precision="fp32_ir", **kw)
    p = B.Problem.from_workload(w, stream=0, rtol=rtol, precision="fp32_ir", **kw)
    for s in range(nsys):
        ep, ec, ps = w.system(s)
        A = ora.operator(ep, ec)
        b = A @ ps
        ro = ora.solve(ep, ec, b)
        p.set_surface(ep, ec)
        p.push_rhs(b)
        info = p.solve()
        x = p.solution()
        rel_cpu = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        dx = np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x)
        err_star = np.linalg.norm(x - ps) / np.linalg.norm(ps)
        _say(f"   sys {s:2d}: gpu it={info.iters} ref={info.refinements} ck={info.checks} rank={info.rank} "
             f"r0={info.relres0:.2e} r={info.relres:.2e} (cpu {rel_cpu:.2e}) | oracle it={ro.info.iters} "
             f"ref={ro.info.refinements} ck={ro.info.checks} | dx={dx:.2e} |x-p*|={err_star:.2e}")
        assert info.status == 0
        assert info.relres <= rtol and rel_cpu <= 1.01 * rtol
        assert dx <= 1e-7
    p.close()
