"""The C-ABI library loads and exports what include/sawave.h declares (no GPU work here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import rng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sawave.h")


@pytest.fixture(scope="module")
def binding():
    from paper_2511_18071_amd import binding
    return binding


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sa_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sa_create", "sa_set_surface", "sa_push_rhs", "sa_solve", "sa_get_solution", "sa_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(binding):
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options(binding):
    o = binding.default_options()
    assert (o.restart, o.max_restarts, o.rtol, o.precond, o.guess, o.k, o.r) == (30, 200, 1e-8, 2, 2, 8, 0.9)
    assert o.omega == 0.5 and o.tau_drop == 1e-7


def test_sketch_draws_bitwise_equal_to_oracle_stream(binding):
    for seed in (0, 7, 2**63 + 12345):
        for index in (0, 1, 17, 100000):
            lib_draws = binding.sketch_draws(seed, index, 16)
            ref = np.array(rng.omega(seed, index, 16))
            assert np.array_equal(lib_draws, ref), (seed, index)


def test_argument_errors_need_no_gpu(binding):
    with pytest.raises(binding.SawaveError) as e:
        binding.Problem(65, 3, "periodic", 1.0, np.ones(64))  # nz too small
    assert e.value.code == -1
    with pytest.raises(binding.SawaveError) as e:
        binding.Problem(65, 9, "periodic", 1.0, -np.ones(64))  # non-positive depth
    assert e.value.code == -2
    with pytest.raises(binding.SawaveError):
        binding.Problem(65, 9, "periodic", 1.0, np.ones(64), k=17)
    with pytest.raises(binding.SawaveError):
        binding.Problem(65, 9, "periodic", 1.0, np.ones(64), restart=0)


def test_ctypes_struct_layout(binding):
    # field offsets follow the C rules for the declared order (int32 then double gets padded)
    assert binding.SaGrid.length.offset == 16
    assert ctypes.sizeof(binding.SaSolveInfo) == 6 * 4 + 2 * 8
    assert binding.SaOptions.rtol.offset == 8


def test_refinement_option_errors_need_no_gpu(binding):
    for bad in (dict(rtol_inner=0.0), dict(rtol_inner=1.5), dict(max_refine=0)):
        with pytest.raises(binding.SawaveError) as e:
            binding.Problem(65, 9, "periodic", 1.0, np.ones(64), precision="fp32_ir", **bad)
        assert e.value.code == -1, bad
    with pytest.raises(binding.SawaveError):
        binding.Problem(65, 9, "periodic", 1.0, np.ones(64), precision=7)


def test_footprint_needs_no_gpu(binding):
    from paper_2511_18071_amd import workload as W
    w = W.get("bar_513x17")
    f64 = binding.footprint(w)
    f32 = binding.footprint(w, precision="fp32_ir")
    cold = binding.footprint(w, guess="cold")
    n = w.n
    # at least the Krylov basis (m + 1 vectors) and the two sketch buffers
    assert f64 >= 8 * n * (w.restart + 1 + 2 * w.k)
    assert f32 >= f64 + 4 * n * (w.restart + 1)   # plus the FP32 basis
    assert cold <= f64 - 8 * n * 2 * w.k + 4096   # no sketch
    with pytest.raises(binding.SawaveError):
        binding.footprint(w, k=99)


def test_server_option_errors_need_no_gpu(binding):
    for bad in (dict(max_inflight=0), dict(max_inflight=17), dict(max_batch=-1), dict(unknowns_per_workgroup=0)):
        with pytest.raises(binding.SawaveError) as e:
            binding.Server(**bad)
        assert e.value.code == -1, bad


def test_footprint_of_every_preconditioner_on_the_large_grid(binding):
    # the LDS sizing of the coarsest solve applies to the V-cycle only
    from paper_2511_18071_amd import workload as W
    w = W.get("periodic_16385x33")
    for pc in ("none", "line", "mg"):
        assert binding.footprint(w, precond=pc, cluster=64) > 8 * w.n * (w.restart + 1)


def test_library_hierarchy_rule_matches_the_serving_grid_rule(binding):
    """The grid sizes the serving mix picks are the ones sa_create accepts: the dry run that
    computes a footprint builds the hierarchy and refuses a coarsest grid above 4096 unknowns
    (no GPU needed)."""
    from paper_2511_18071_amd import workload as W
    cases = [(4097, 33, "periodic"), (4096, 33, "periodic"), (1985, 33, "periodic"), (4065, 33, "periodic"),
             (961, 33, "periodic"),
             (4097, 9, "walls"), (4098, 9, "walls"), (1025, 17, "walls"), (1031, 17, "walls")]
    for nx, nz, bc in cases:
        if bc == "periodic":
            w = W._stream("t", nx, nz, 2.0, 1, 4, 0.05, 1, 2, 30, 8, 0.9)
        else:
            w = W._bar("t", nx, nz, 1, 2, 30, 8, 0.9, scale=(nx - 1) / 512.0, a0=0.01)
        fits = W.hierarchy_fits(nx, nz, bc)
        try:
            binding.footprint(w)
            ok = True
        except binding.SawaveError:
            ok = False
        assert ok == fits, (nx, nz, bc, fits)
