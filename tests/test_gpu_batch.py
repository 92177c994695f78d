"""GPU checks of the batched solve and of the launch-shape autotuner.

Launch shapes change which block computes a value, not the arithmetic of
that value: every FFT value and every nodal sum of the Hessian is formed in
the same order whatever the shape, the Hessian's sums are formed per
canonical 8x4x4 tile of nodes, and the fused inverse FFT pass sums runs of 64
values. So the Green's operator, K d and a whole Newton solve must be
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
            for bs in range(13):
                try:
                    solver.set_tuning(plane_threads=pt, pencil_cols=pc, pencil_threads=pth,
                                      plane_threads32=pt, pencil_cols32=pc, pencil_threads32=pth,
                                      brick_shape=bs, brick_shape32=bs)
                except hfe.HfeError:
                    continue
                out.append((pt, pc, pth, bs))
    return out


@pytest.mark.parametrize("shape", [(16, 12, 8), (32, 32, 32), (24, 16, 16)])
def test_every_launch_shape_gives_the_same_bits(shape):
    """(16, 12, 8): bricks only (no column divides ny = 12); (32, 32, 32):
    bricks and every marching column; (24, 16, 16): columns whose last block
    marches fewer layers (24 is not a multiple of 16 or 32)."""
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


def _spread_tunings(solver):
    """Every Hessian shape the grid allows, each with other FFT launch shapes,
    and every plane block size with the 8x8x8 brick."""
    combos = _shapes(solver)
    by_shape = {}
    for sh in combos:
        by_shape.setdefault(sh[3], []).append(sh)
    picked = []
    for j, bs in enumerate(sorted(by_shape)):
        lst = by_shape[bs]
        picked.append(lst[(7 * j + 3) % len(lst)])
    for pt in (256, 512, 1024):
        for sh in combos:
            if sh[0] == pt and sh[3] == 1 and sh not in picked:
                picked.append(sh)
                break
    return picked


@pytest.mark.parametrize("shape,precision,control", [
    ((32, 32, 24), "fp64", False),   # bricks and every column, columns cut along z
    ((24, 12, 6), "fp64", False),    # ragged bricks, tiles cut by the grid
    ((32, 32, 24), "mixed", False),
    ((16, 16, 12), "fp64", True),    # mean-stress control: the Hessian's tail rows
])
def test_every_launch_shape_gives_the_same_solve(shape, precision, control):
    """A softening increment (Newton with Steihaug CG, its decisions taken on
    the reductions of the Hessian and of the fused FFT passes) solved under
    many launch shapes: the Newton log, the CG residual trace, the state and
    the stress have the same bits under every shape."""
    torch = require_gpu()
    announce("same solve under every launch shape", shape, precision, control)
    from paper_2207_10657_amd import Solver
    w = workload("c1_3d16")
    rng = np.random.default_rng(11)
    phase = (rng.random(shape) < 0.3).astype(np.uint8)
    s = Solver(shape, "q1")
    s.setup(phase, w.materials)
    if control:
        free = np.zeros((3, 3), dtype=bool)
        free[1, 1] = free[2, 2] = True
        s.set_mean_stress_control(free)
    ck = s.get_state()
    u0 = 3e-4 * rng.normal(size=(3,) + shape)
    E0 = np.zeros((3, 3))
    E0[0, 0] = 1.2e-3
    dE = np.zeros((3, 3))
    dE[0, 0] = 2e-4
    params = {"i_nr_max": 4, "precision": precision}
    ref = None
    tunings = _spread_tunings(s)
    assert len(tunings) >= 6
    for sh in tunings:
        pt, pc, pth, bs = sh
        s.set_tuning(plane_threads=pt, pencil_cols=pc, pencil_threads=pth, plane_threads32=pt,
                     pencil_cols32=pc, pencil_threads32=pth, brick_shape=bs, brick_shape32=bs)
        s.set_state(u0, ck["kappa_hist"], E0, ck["R"], ck["Rmax"])
        s.apply_load_step(dE)
        rep = s.solve_increment(params)
        st = s.get_state()
        log = s.newton_log()
        out = (np.array([[float(r[k]) for k in sorted(r)] for r in log]), s.cg_trace(), st["u"],
               st["kappa_hist"], st["E"], s.homogenized_stress())
        if ref is None:
            ref = out
            assert rep["cg_iters"] > 20 and len(log) >= 2, rep
            continue
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(np.asarray(a), np.asarray(b), err_msg=str(sh))


def test_autotune_between_load_steps_changes_no_result():
    """The autotuner times CG iterations of a probe solve at the current
    state (its FP64 FFT shapes): tuning between two load steps must leave
    every later result as it is, bit for bit, against the same steps solved
    without tuning."""
    require_gpu()
    announce("autotune between load steps", (16, 16, 16))
    from paper_2207_10657_amd import Solver
    w = workload("c1_3d16", steps=4)
    runs = []
    for tune in (False, True):
        s = Solver(w.shape, "q1")
        s.setup(w.phase, w.materials)
        out = []
        for n, dE in enumerate(w.load_path):
            if tune and n == 2:
                s.autotune()
            s.apply_load_step(dE)
            s.solve_increment()
            log = s.newton_log()
            st = s.get_state()
            out.append((np.array([[float(r[k]) for k in sorted(r)] for r in log]), s.cg_trace(),
                        st["u"], st["kappa_hist"], s.homogenized_stress()))
        s.close()
        runs.append(out)
    for n, (a, b) in enumerate(zip(*runs)):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(np.asarray(x), np.asarray(y), err_msg="step %d" % n)


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


def test_batch_of_uneven_cells_matches_single_solves():
    """Cells of uneven sizes (8^3, 12^3, 16^3, 24^3 of the workload recipe, an
    uneven brick fit at 12^3 and 24^3), each under its own unit load case,
    solved as one batch and one by one: the same bits."""
    require_gpu()
    announce("batch of uneven cells")
    from paper_2207_10657_amd import Solver, solve_batch
    cases = _load_cases(2e-4)
    cells = []
    for k, n in enumerate((8, 12, 16, 24)):
        w = workload("c1_3d%d" % n)
        cells.append((w, cases[k]))
    batch = [Solver(w.shape, "q1", own_stream=True) for w, _ in cells]
    for s, (w, _) in zip(batch, cells):
        s.setup(w.phase, w.materials)
    for step in range(2):
        for s, (_, dE) in zip(batch, cells):
            s.apply_load_step(dE)
        reps = solve_batch(batch)
        announce("uneven batch step", step, [(r["newton_iters"], r["cg_iters"]) for r in reps])
    for n, (sb, (w, dE)) in enumerate(zip(batch, cells)):
        s = Solver(w.shape, "q1")
        s.setup(w.phase, w.materials)
        for step in range(2):
            s.apply_load_step(dE)
            s.solve_increment()
        np.testing.assert_array_equal(sb.homogenized_stress(), s.homogenized_stress(), err_msg=str(n))
        np.testing.assert_array_equal(sb.get_state()["u"], s.get_state()["u"], err_msg=str(n))
        s.close()


def test_batch_of_uneven_cells_against_the_oracle():
    """A batch of cells of uneven sizes (8^3, 12^3, 16^3 and a 8x12x16 box of
    the workload recipe), each under its own unit load case, two increments
    solved with hfe_solve_batch, each cell against its own oracle: the same
    Newton decisions and the homogenized stress at 1e-10 of the load scale,
    the damage at 1e-10 (Sec. 3.3's stiffness cells, strain control)."""
    require_gpu()
    announce("batch of uneven cells vs the oracle")
    from oracle.solver import CellSolver
    from paper_2207_10657_amd import Solver, solve_batch
    from synthetic import inclusion_microstructure
    cases = _load_cases(2e-4)
    w16 = workload("c1_3d16")
    shapes = [(8, 8, 8), (12, 12, 12), (16, 16, 16), (8, 12, 16)]
    cells = []
    for k, shape in enumerate(shapes):
        n = max(shape)
        phase = inclusion_microstructure(shape, 4.0 * n / 64, 8.0 * n / 64, 0.25, 31 + k)[0]
        cells.append((shape, phase, cases[(2 * k + 1) % 6]))
    batch = [Solver(sh, "q1", own_stream=True) for sh, _, _ in cells]
    oracles = [CellSolver(ph, w16.materials, "q1") for _, ph, _ in cells]
    for s, (_, ph, _) in zip(batch, cells):
        s.setup(ph, w16.materials)
    for step in range(2):
        for s, o, (_, _, dE) in zip(batch, oracles, cells):
            s.apply_load_step(dE)
            o.apply_load_step(dE)
        reps = solve_batch(batch)
        for k, (s, o, r) in enumerate(zip(batch, oracles, reps)):
            ro = o.solve_increment()
            assert [x["flag"] for x in s.newton_log()] == ro["flags"], (step, k)
            assert [x["cg_iters"] for x in s.newton_log()] == ro["cg_per_newton"], (step, k)
            assert r["converged"] == ro["converged"]
            lam, mu = 10.0 * 0.3 / (1.3 * 0.4), 10.0 / 2.6
            scale = np.linalg.norm(lam * np.trace(o.E) * np.eye(3) + 2 * mu * o.E)
            dS = np.linalg.norm(s.homogenized_stress() - o.homogenized_stress()) / scale
            dd = float(np.abs(s.damage() - o.damage()).max())
            print("[batch] cell %s step %d: Newton %d, |dSigma|/scale %.2e, damage %.2e"
                  % (cells[k][0], step, r["newton_iters"], dS, dd), flush=True)
            assert dS < 1e-10 and dd < 1e-10, (step, k, dS, dd)


@pytest.mark.parametrize("n", [48, 96])
def test_projected_hessian_48_and_96_against_the_displacement_oracle(n):
    """The cell sizes of uneven batches with radix-3 FFT lengths (48 = 16 x 3,
    96 = 32 x 3): one projected-Hessian application at a softening state
    against the displacement-space oracle (oracle/uspace.py, itself pinned to
    the strain-space projector), element by element at 1e-12."""
    torch = require_gpu()
    announce("projected hessian vs displacement oracle", n)
    from oracle import material
    from oracle.uspace import UOperator
    from paper_2207_10657_amd import Solver
    from tests.gpu_util import max_err
    w = workload("c1_3d%d" % n)
    rng = np.random.default_rng(12)
    u = 4e-4 * rng.normal(size=(3,) + w.shape)
    E = np.zeros((3, 3))
    E[0, 0] = 2e-3
    s = Solver(w.shape, "q1")
    s.setup(w.phase, w.materials)
    s.apply_load_step(E)
    s.set_displacement(u)
    d = rng.normal(size=(3,) + w.shape)
    dt = torch.tensor(d, device="cuda")
    out = s.apply_projected_hessian(dt)[0].cpu().numpy()
    kh = material.MaterialField(w.phase, w.materials, 8).initial_history()
    op = UOperator(w.phase, w.materials, "q1", E, u, kh)
    ref = op.apply(d)
    err = max_err(out, ref)
    print("[batch] %d^3 projected Hessian vs displacement oracle: max err %.2e" % (n, err),
          flush=True)
    if err >= 1e-12:
        # which stage: K d, or the Green's operator applied to the GPU's K d
        Kd = s.apply_stiffness(dt).cpu().numpy()
        GKd = s.apply_green(torch.tensor(Kd, device="cuda")).cpu().numpy()
        out2 = s.apply_projected_hessian(dt)[0].cpu().numpy()
        Kd_ref = op.stiffness(d)
        ref1 = UOperator(w.phase, w.materials, "q1", E, u, kh, workers=1).apply(d)
        bad = np.argwhere(np.abs(out - ref) > 1e-6 * np.abs(ref).max())
        print("[batch]   K d %.2e, green(K d) %.2e, a second application %.2e, the oracle on "
              "one thread vs its first result %.2e; %d bad values, z %s, y %s, x %s"
              % (max_err(Kd, Kd_ref), max_err(GKd, op.green(Kd)), max_err(out2, ref),
                 max_err(ref1, ref), len(bad), np.unique(bad[:, 1])[:12],
                 np.unique(bad[:, 2])[:12], np.unique(bad[:, 3])[:12]), flush=True)
    s.close()
    assert err < 1e-12


# ---- effective stiffness (six unit load cases as one batch) -------------------

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
TIGHT = {"eta_eq": 1e-12, "eta_nr": 1e-14, "eta_cg": 1e-10}


def _unit_case(J, strain):
    i, j = VOIGT[J]
    dE = np.zeros((3, 3))
    e = strain if i == j else 0.5 * strain
    dE[i, j] = dE[j, i] = e
    return dE


def _oracle_stiffness(phase, materials, strain, kappa_hist=None):
    from oracle.solver import CellSolver
    C = np.zeros((6, 6))
    for J in range(6):
        o = CellSolver(phase, materials, "q1")
        if kappa_hist is not None:
            o.kappa_hist = kappa_hist.copy()
        o.apply_load_step(_unit_case(J, strain))
        assert o.solve_increment(TIGHT)["converged"]
        S = o.homogenized_stress()
        C[:, J] = [S[i, j] for i, j in VOIGT]
    return C / strain


def _gpu_stiffness(shape, phase, materials, strain, kappa_hist=None):
    from paper_2207_10657_amd import Solver, effective_stiffness
    sv = [Solver(shape, "q1", own_stream=True) for _ in range(6)]
    for s in sv:
        s.setup(phase, materials)
        if kappa_hist is not None:
            s.set_state(np.zeros((3,) + shape), kappa_hist, np.zeros((3, 3)), 0.0, 0.0)
    C, reps = effective_stiffness(sv, strain, TIGHT)
    assert all(r["converged"] for r in reps)
    for s in sv:
        s.close()
    return C


def test_effective_stiffness_of_a_laminate():
    """Backus averages of a layered cell (layers normal to x), exact for the
    voxel-aligned laminate."""
    require_gpu()
    announce("effective stiffness, laminate")
    from synthetic import laminate_microstructure
    shape = (8, 8, 16)
    layers = np.array([0, 0, 1, 1, 1, 0, 1, 0] * 2, dtype=np.uint8)
    phase = laminate_microstructure(shape, layers)
    m1 = {"kind": "elastic", "E": 1.0, "nu": 0.3}
    m2 = {"kind": "elastic", "E": 7.0, "nu": 0.2}
    C = _gpu_stiffness(shape, phase, [m1, m2], 1e-4)
    f = np.array([np.mean(layers == 0), np.mean(layers == 1)])
    lam = np.array([m["E"] * m["nu"] / ((1 + m["nu"]) * (1 - 2 * m["nu"])) for m in (m1, m2)])
    mu = np.array([m["E"] / (2 * (1 + m["nu"])) for m in (m1, m2)])
    M = lam + 2 * mu
    avg = lambda x: float(np.sum(f * x))
    Cnn = 1.0 / avg(1.0 / M)
    Cnt = avg(lam / M) * Cnn
    Ctt = avg(M - lam ** 2 / M) + avg(lam / M) ** 2 * Cnn
    Ctt2 = avg(lam - lam ** 2 / M) + avg(lam / M) ** 2 * Cnn
    ref = np.zeros((6, 6))
    ref[0, 0] = Cnn
    ref[0, 1] = ref[1, 0] = ref[0, 2] = ref[2, 0] = Cnt
    ref[1, 1] = ref[2, 2] = Ctt
    ref[1, 2] = ref[2, 1] = Ctt2
    ref[3, 3] = avg(mu)                    # yz: shear within the layers
    ref[4, 4] = ref[5, 5] = 1.0 / avg(1.0 / mu)   # xz, xy: shear across the layers
    err = np.abs(C - ref).max() / np.abs(ref).max()
    print("[stiffness] laminate: max |C - Backus| / max|C| = %.2e" % err, flush=True)
    assert err < 1e-9


def test_effective_and_damaged_secant_stiffness_against_oracle():
    """An inclusion cell (8^3): the initial stiffness, then the secant
    stiffness of a damaged cell (a frozen history between kappa0 and kappaf:
    small loads unload) against the oracle's six solves."""
    require_gpu()
    announce("effective stiffness vs oracle, 8^3")
    w = workload("c1_3d16")
    shape = (8, 8, 8)
    phase = np.ascontiguousarray(w.phase[:8, :8, :8])
    C0 = _gpu_stiffness(shape, phase, w.materials, 1e-5)
    R0 = _oracle_stiffness(phase, w.materials, 1e-5)
    e0 = np.abs(C0 - R0).max() / np.abs(R0).max()
    sym = np.abs(C0 - C0.T).max() / np.abs(C0).max()
    # a damaged history: kappa_hist between kappa0 and kappaf on the matrix points
    rng = np.random.default_rng(11)
    k0, kf = w.materials[0]["kappa0"], w.materials[0]["kappaf"]
    kh = np.where((phase == 0)[..., None], k0 + (kf - k0) * rng.random(shape + (8,)), 0.0)
    C1 = _gpu_stiffness(shape, phase, w.materials, 1e-6, kh)
    R1 = _oracle_stiffness(phase, w.materials, 1e-6, kh)
    e1 = np.abs(C1 - R1).max() / np.abs(R1).max()
    print("[stiffness] 8^3 inclusion cell: initial vs oracle %.2e (asym %.1e); damaged secant vs "
          "oracle %.2e; C11 %.4f -> %.4f" % (e0, sym, e1, C0[0, 0], C1[0, 0]), flush=True)
    assert e0 < 1e-9 and e1 < 1e-9 and sym < 1e-8
    assert C1[0, 0] < C0[0, 0]
