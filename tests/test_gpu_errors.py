"""Failure paths of the C ABI on the GPU, forced from the host: calls out of
the documented order (HFE_ESTATE), invalid solver parameters (HFE_EINVAL), a
load increment whose stress overflows (HFE_ENUMERIC, the context keeps its
previous state), and an increment that ends at i_NR,max (HFE_NOT_CONVERGED:
Algorithm 2 commits the damage history only on convergence). Every kernel
runs to its normal end; only host-side checks and finite arithmetic are
involved."""
import numpy as np
import pytest

from synthetic import workload
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu

ESTATE, EINVAL, ENUMERIC = -5, -1, -4


def _solver(w):
    from paper_2207_10657_amd import Solver
    return Solver(w.shape, w.element)


def test_calls_out_of_order_return_estate():
    require_gpu()
    announce("errors: order of calls")
    from paper_2207_10657_amd.hfe import HfeError
    w = workload("c1_3d8", steps=1)
    s = _solver(w)
    with pytest.raises(HfeError) as e:
        s.solve_increment()              # no load step yet
    assert e.value.status == ESTATE
    with pytest.raises(HfeError) as e:
        s.apply_load_step(w.load_path[0])   # no microstructure / materials
    assert e.value.status == ESTATE
    with pytest.raises(HfeError) as e:
        s.set_material(0, w.materials[0])   # no microstructure
    assert e.value.status == ESTATE
    s.set_microstructure(w.phase, len(w.materials))
    s.set_material(0, w.materials[0])
    with pytest.raises(HfeError) as e:
        s.apply_load_step(w.load_path[0])   # phase 1 has no material yet
    assert e.value.status == ESTATE
    s.set_material(1, w.materials[1])
    s.apply_load_step(w.load_path[0])
    with pytest.raises(HfeError) as e:
        s.set_material(0, w.materials[0])   # materials are fixed once loading started
    assert e.value.status == ESTATE
    assert s.solve_increment()["converged"]


@pytest.mark.parametrize("bad", [{"precision": 7}, {"cg_stall": -1}, {"restart": float("nan")}])
def test_invalid_solver_parameters_return_einval(bad):
    require_gpu()
    announce("errors: parameters", bad)
    from paper_2207_10657_amd.hfe import HfeError
    w = workload("c1_3d8", steps=1)
    s = _solver(w)
    s.setup(w.phase, w.materials)
    s.apply_load_step(w.load_path[0])
    with pytest.raises(HfeError) as e:
        s.solve_increment(bad)
    assert e.value.status == EINVAL
    assert s.solve_increment()["converged"]


def test_overflowing_increment_returns_enumeric_and_keeps_the_state():
    """A strain increment of 1e300 overflows the stress: HFE_ENUMERIC, and the
    context goes on from the state before that call exactly as a context
    that never saw it (bit for bit)."""
    require_gpu()
    announce("errors: non-finite stress")
    from paper_2207_10657_amd.hfe import HfeError
    w = workload("c1_3d8", steps=3)
    a, b = _solver(w), _solver(w)
    for s in (a, b):
        s.setup(w.phase, w.materials)
        s.apply_load_step(w.load_path[0])
        assert s.solve_increment()["converged"]
    big = np.zeros((3, 3))
    big[0, 0] = 1e300
    with pytest.raises(HfeError) as e:
        a.apply_load_step(big)
    print("[errors] after the overflowing increment: %s; E_xx %.3e; sigma_xx %.6e / %.6e"
          % (e.value, a.get_state()["E"][0, 0], a.homogenized_stress()[0, 0],
             b.homogenized_stress()[0, 0]), flush=True)
    assert e.value.status == ENUMERIC
    np.testing.assert_array_equal(a.get_state()["E"], b.get_state()["E"])
    np.testing.assert_array_equal(a.homogenized_stress(), b.homogenized_stress())
    for s in (a, b):
        s.apply_load_step(w.load_path[1])
        assert s.solve_increment()["converged"]
    np.testing.assert_array_equal(a.displacement(), b.displacement())
    np.testing.assert_array_equal(a.homogenized_stress(), b.homogenized_stress())
    with pytest.raises(HfeError) as e:
        u = a.displacement()
        u[0, 0, 0, 0] = np.nan
        a.set_displacement(u)
    assert e.value.status == EINVAL


def test_unconverged_increment_does_not_commit_the_history():
    """An increment into the damage regime stopped after one Newton
    iteration ends HFE_NOT_CONVERGED; the committed history (kappa_hist) is
    the one before the increment, bit for bit, and solving the same increment
    again to convergence then commits it."""
    require_gpu()
    announce("errors: not converged")
    w = workload("c1_3d16", steps=3)
    s = _solver(w)
    s.setup(w.phase, w.materials)
    for n in range(2):
        s.apply_load_step(w.load_path[n])
        assert s.solve_increment({"i_nr_max": 2000})["converged"]
    kappa0 = s.field(4)
    s.apply_load_step(w.load_path[2])
    rep = s.solve_increment({"i_nr_max": 1})
    assert not rep["converged"] and rep["newton_iters"] == 1
    np.testing.assert_array_equal(s.field(4), kappa0)
    rep = s.solve_increment({"i_nr_max": 2000})
    assert rep["converged"]
    k1 = s.field(4)
    assert np.all(k1 >= kappa0) and np.any(k1 > kappa0)
