"""GPU checks of the batched solve and of the launch-shape autotuner.

Launch shapes change which block computes a value, not the arithmetic of
that value (every FFT value and every nodal sum of the Hessian is formed in
the same order whatever the shape), so the Green's operator and K d must be
bit-identical under every shape the tuner may pick. A batch of solvers on
their own streams must give, per solver, the bits of the same solve run
alone."""
import numpy as np
import pytest

from synthetic import workload
from tests.gpu_util import require_gpu, announce

pytestmark = pytest.mark.gpu


def _shapes(solver):
    from paper_2207_10657_amd import hfe
    lib = hfe.load_library()
    out = []
    for pt in (256, 512, 1024):
        for pc, pth in ((4, 64), (4, 128), (8, 64), (8, 128), (8, 256), (16, 128), (16, 256), (32, 256)):
            for bs in range(4):
                try:
                    solver.set_tuning(plane_threads=pt, pencil_cols=pc, pencil_threads=pth,
                                      plane_threads32=pt, pencil_cols32=pc, pencil_threads32=pth,
                                      brick_shape=bs, brick_shape32=bs)
                except hfe.HfeError:
                    continue
                out.append((pt, pc, pth, bs))
    return out


@pytest.mark.parametrize("shape", [(16, 12, 8), (32, 32, 32)])
def test_every_launch_shape_gives_the_same_bits(shape):
    torch = require_gpu()
    announce("launch shapes", shape)
    from paper_2207_10657_amd import Solver
    w = workload("c1_3d16")
    rng = np.random.default_rng(3)
    phase = (rng.random(shape) < 0.3).astype(np.uint8)
    s = Solver(shape, "q1")
    s.setup(phase, w.materials)
    E = np.zeros((3, 3))
    E[0, 0] = 1.5e-3
    s.apply_load_step(E)
    s.set_displacement(4e-4 * rng.normal(size=(3,) + shape))
    d = torch.tensor(rng.normal(size=(3,) + shape), device="cuda")
    d32 = d.float()
    ref = None
    shapes = _shapes(s)
    assert len(shapes) >= 8
    for sh in shapes:
        pt, pc, pth, bs = sh
        s.set_tuning(plane_threads=pt, pencil_cols=pc, pencil_threads=pth, plane_threads32=pt,
                     pencil_cols32=pc, pencil_threads32=pth, brick_shape=bs, brick_shape32=bs)
        g = s.apply_green(d).cpu().numpy()
        k = s.apply_stiffness(d).cpu().numpy()
        h32 = s.apply_projected_hessian_f32(d32)[0].cpu().numpy()
        if ref is None:
            ref = (g, k, h32)
            continue
        np.testing.assert_array_equal(g, ref[0], err_msg=str(sh))
        np.testing.assert_array_equal(k, ref[1], err_msg=str(sh))
        np.testing.assert_array_equal(h32, ref[2], err_msg=str(sh))
    tuned = s.autotune()
    announce("autotuned", shape, tuned)
    np.testing.assert_array_equal(s.apply_green(d).cpu().numpy(), ref[0])
    np.testing.assert_array_equal(s.apply_stiffness(d).cpu().numpy(), ref[1])


def _load_cases(mag):
    cases = []
    for (i, j) in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)):
        dE = np.zeros((3, 3))
        dE[i, j] = dE[j, i] = mag
        cases.append(dE)
    return cases


def test_batch_of_six_load_cases_matches_single_solves():
    """The six unit macroscopic load cases of one cell, two increments each,
    solved as a batch and one by one."""
    require_gpu()
    announce("batch of 6 load cases, 16^3")
    from paper_2207_10657_amd import Solver, solve_batch
    w = workload("c1_3d16")
    cases = _load_cases(2e-4)
    batch = [Solver(w.shape, "q1", own_stream=True) for _ in cases]
    for s in batch:
        s.setup(w.phase, w.materials)
    for step in range(2):
        for s, dE in zip(batch, cases):
            s.apply_load_step(dE)
        reps = solve_batch(batch)
        announce("batch step", step, [(r["newton_iters"], r["cg_iters"]) for r in reps])
    for n, (sb, dE) in enumerate(zip(batch, cases)):
        s = Solver(w.shape, "q1")
        s.setup(w.phase, w.materials)
        for step in range(2):
            s.apply_load_step(dE)
            s.solve_increment()
        np.testing.assert_array_equal(sb.homogenized_stress(), s.homogenized_stress(), err_msg=str(n))
        np.testing.assert_array_equal(sb.get_state()["u"], s.get_state()["u"], err_msg=str(n))
        s.close()
