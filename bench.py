"""Benchmark: projected-Hessian throughput and time per load step on one GPU.

Workload: the 3D periodic cell of 64^3 voxels (trilinear hexahedra, 8 Gauss
points per voxel) with random non-overlapping spherical inclusions (radius 4-8
voxels, volume fraction 0.25, E = 10) in a damaging matrix (E = 1, nu = 0.3,
energy-norm damage with linear softening, kappa0 = 1e-3, kappaf = 5e-3),
loaded in 30 equal uniaxial macro-strain steps to 0.6%, FP64 trust-region +
Steihaug-CG solver at tolerance 1e-8. Inputs are synthetic and seeded.

One step = one load increment (apply_load_step + solve_increment), which runs
every stage of the hot path. `--warmup W` increments run untimed, then `--steps
K` increments are timed. The headline value is
    Gvoxel-matvec/s = N_voxels x (projected-Hessian applications) / s / 1e9
over the timed increments (whole-solver throughput, inputs resident in HBM).

The JSON line also carries the roofline of the dominant kernel (algorithmic
bytes per launch over its average duration, timed with HIP events on the
library's stream during the timed region) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The metric is the time per load step at a 1e-8 residual, so every timed
# increment runs until it converges. The library's default of 50 Newton
# iterations (the parity tests' setting) stops the damage-onset increments of
# this path early, at r_eq ~ 0.1; with this cap every one of them converges.
NEWTON_CAP = 2000
SOLVE = {"i_nr_max": NEWTON_CAP}
# Stated bound on the homogenized-stress difference of a mixed-precision load
# step from the FP64 step solved from the same state (relative to |Sigma|).
# Both stop at the same FP64 residual tolerance; the difference is that of two
# inexact Newton paths through a softening increment.
MIXED_SIGMA_BOUND = 1e-5
# window of the CG stall exit in the variant runs
STALL_WINDOW = 100


# The least a projected-Hessian matvec's element pass (gradient, tangent,
# divergence) must move per voxel, FP64: the direction in (24 B), the state it
# linearises about when the tangent is recomputed from it, i.e. the nodal
# displacement (24 B) and the history at the 8 points (64 B), the phase
# (1 B), and K d out (24 B). The roofline of the Hessian is quoted against it.
HESSIAN_MIN_BYTES_PER_VOXEL = 24 + 24 + 64 + 1 + 24


def algorithmic_bytes(name, shape, n_soft=0.0):
    """Bytes per launch that each kernel must move at minimum (3D Q1, FP64, or
    FP32 for the kernels of the mixed-precision CG, names ending in _f32).
    n_soft: softening points of the state; at each, the element kernels move
    the six FP64 components of the rank-one softening factor w."""
    nz, ny, nx = shape
    N = nx * ny * nz
    f32 = name.endswith("_f32")
    base = name[:-4] if f32 else name
    r = 4 if f32 else 8                        # bytes per real
    spec = 6.0 * r * (nx // 2 + 1) / nx         # 3 half-spectrum fields, B / voxel
    per_vox = {
        # d, a at 8 points, phase, soft mask, K d
        "stiffness": 3 * r + 8 * r + 1 + 1 + 3 * r,
        # 3 real fields in, 3 half spectra out (and back)
        "fft_plane_fwd": 3 * r + spec,
        "fft_pencil_green": 2 * spec,
        "fft_plane_inv": spec + 3 * r,
        # fused CG passes: + z, d, g in and z, g out / + y, g in and y out
        "fft_plane_fwd_cg": 3 * r + spec + 15 * r,
        "fft_plane_inv_cg": spec + 9 * r,
        # u, kappa_hist, phase in; a, soft mask and D^T sigma out
        "residual": 24 + 64 + 1 + 64 + 1 + 24,
        # u, z, kappa_hist, a, phase, soft mask in; sums only
        "trial": 24 + 24 + 64 + 64 + 1 + 1,
    }
    if base not in per_vox or (f32 and base in ("residual", "trial")):
        return None
    soft = 48.0 * n_soft if base in ("stiffness", "residual", "trial") else 0.0
    return per_vox[base] * N + soft


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_matvec):
    """Time the oracle's projected Hessian in displacement coordinates
    (oracle/uspace.py: the same operator as the GPU's, validated against the
    strain-space projector) on every host core: slabs on a thread pool and
    threaded FFTs. State: E_xx = 2e-3 and a random fluctuation (three
    quarters of the points softening)."""
    from oracle import material
    from oracle.uspace import UOperator
    rng = np.random.default_rng(0)
    E = np.zeros((3, 3))
    E[0, 0] = 2e-3
    u = 4e-4 * rng.normal(size=(3,) + w.shape)
    kh = material.MaterialField(w.phase, w.materials, 8).initial_history()
    cores = os.cpu_count() or 1
    op = UOperator(w.phase, w.materials, "q1", E, u, kh, workers=cores)
    d = rng.normal(size=(3,) + w.shape)
    op.apply(d)
    t0 = time.perf_counter()
    for _ in range(n_matvec):
        op.apply(d)
    dt = time.perf_counter() - t0
    return {"value": w.nvox * n_matvec / dt / 1e9, "unit": "Gvoxel-matvec/s",
            "cores": cores, "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "%d projected-Hessian applications of the FP64 displacement-space oracle "
                      "(numpy, %d threads, scipy.fft with %d workers) at %d^3 on a softening "
                      "state, %.1f s" % (n_matvec, cores, cores, w.shape[0], dt)}


COPY_BYTES = 1 << 28


def unit_load_cases(mag):
    """The six macroscopic strain increments xx, yy, zz, xy, xz, yz of size mag."""
    cases = []
    for (i, j) in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)):
        dE = np.zeros((3, 3))
        dE[i, j] = dE[j, i] = mag
        cases.append(dE)
    return cases


def warm_start_bench(n=16, train_seeds=tuple(range(101, 149)), test_seed=201, steps=6,
                     epochs=20):
    """Learned warm start on cells of the workload recipe at n^3: increments
    of `train_seeds` cells train the encoder-decoder (hand-written BF16
    kernels), then
    a held-out cell is solved `steps` increments with the plain guess (the
    previous fluctuation), the extrapolated previous increment, and the
    network's prediction. Per guess: Newton and CG iterations, time."""
    import torch
    from paper_2207_10657_amd import Solver
    from paper_2207_10657_amd.warmstart import WarmStart
    from synthetic import inclusion_microstructure, workload
    w = workload("c1_3d%d" % n)
    dE = w.load_path[0]
    scale = float(np.linalg.norm(dE)) * n

    def cell(seed):
        return inclusion_microstructure((n, n, n), 4.0 * n / 64, 8.0 * n / 64, 0.25, seed)[0]

    def run(phase, guess=None, ws=None, record=None, params=None):
        s = Solver(phase.shape, "q1")
        s.setup(phase, w.materials)
        u_prev = np.zeros((3,) + phase.shape)
        du_prev = None
        newton = cg = conv = taken = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.apply_load_step(dE)
            if guess == "extrapolate" and du_prev is not None:
                s.set_displacement(u_prev + du_prev)
            elif guess == "learned" and du_prev is not None:
                taken += int(ws.warm_start(s, phase, u_prev, du_prev, scale))
            r = s.solve_increment(params)
            newton += r["newton_iters"]
            cg += r["cg_iters"]
            conv += int(r["converged"])
            u = s.get_state()["u"]
            if record is not None and du_prev is not None and r["converged"]:
                record.record(phase, s.damage(), du_prev, u - u_prev, scale)
            du_prev, u_prev = u - u_prev, u
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        out = {"newton_iters": newton, "cg_iters": cg, "converged_steps": conv,
               "ms_per_step": dt / steps * 1e3}
        if guess == "learned":
            out["learned_guess_taken"] = taken   # else the previous fluctuation (lower r_eq)
        return out

    ws = WarmStart(seed=0)
    t0 = time.perf_counter()
    for seed in train_seeds:
        run(cell(seed), record=ws)
    t1 = time.perf_counter()
    losses = ws.train(epochs)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    phase = cell(test_seed)
    # held-out increments to convergence (1e-8), as the timed steps of the main line
    out = {g or "previous": run(phase, g, ws, params=SOLVE)
           for g in (None, "extrapolate", "learned")}
    return {"grid": n, "train_cells": len(train_seeds), "samples": len(ws.samples),
            "epochs": epochs, "data_s": t1 - t0, "train_s": t2 - t1,
            "loss_first_last": [float(np.mean(losses[:10])), float(np.mean(losses[-10:]))],
            "held_out_steps": steps, "guesses": out}


def warm_start_scaled_bench(n=64, train_seeds=tuple(range(4000, 4050)),
                            test_seeds=tuple(range(4050, 4055)), steps=6, epochs=8, log=None):
    """The learned warm start at the scale of its configuration: cells of the
    workload recipe at n^3 (radii 4-8 voxels, vf 0.25, one cell per seed),
    the uniaxial increments of the recipe, each solved to the 1e-8 residual.
    The 4-level network widening 16, 32, 64, 64 channels takes 18 input
    channels (phase, damage, previous increment, current strain, macroscopic
    increment) recorded at the start of each increment; its target is the
    increment the solve reached. Trained on the increments of `train_seeds`,
    evaluated on `test_seeds` with the plain guess (the previous
    fluctuation), the extrapolated previous increment, and the learned guess
    (kept only where it lowers r_eq): Newton and CG iterations, ms per step."""
    import torch
    from paper_2207_10657_amd import Solver
    from paper_2207_10657_amd.warmstart import WarmStart
    from synthetic import inclusion_microstructure, workload
    w = workload("c1_3d%d" % n)
    dE = w.load_path[0]
    scale = float(np.linalg.norm(dE)) * n
    shape = (n, n, n)
    ws = WarmStart(seed=0, full=True)

    def cell(seed):
        return inclusion_microstructure(shape, 4.0 * n / 64, 8.0 * n / 64, 0.25, seed)[0]

    def run(phase, guess=None, record=False):
        s = Solver(shape, "q1")
        s.setup(phase, w.materials)
        u_prev = np.zeros((3,) + shape)
        du_prev = None
        newton = cg = conv = taken = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.apply_load_step(dE)
            f = None
            if record and du_prev is not None:
                f = ws.state_features(s, phase, u_prev, du_prev, scale, dE)
            if guess == "extrapolate" and du_prev is not None:
                s.set_displacement(u_prev + du_prev)
            elif guess == "learned" and du_prev is not None:
                taken += int(ws.warm_start(s, phase, u_prev, du_prev, scale, dE))
            r = s.solve_increment(SOLVE)
            newton += r["newton_iters"]
            cg += r["cg_iters"]
            conv += int(r["converged"])
            u = s.get_state()["u"]
            if f is not None and r["converged"]:
                ws.record_sample(f, du_prev, u - u_prev, scale, shape)
            du_prev, u_prev = u - u_prev, u
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        out = {"newton_iters": newton, "cg_iters": cg, "converged_steps": conv,
               "ms_per_step": dt / steps * 1e3}
        if guess == "learned":
            out["learned_guess_taken"] = taken
        return out

    t0 = time.perf_counter()
    for k, seed in enumerate(train_seeds):
        run(cell(seed), record=True)
        if log and (k + 1) % 10 == 0:
            log("scaled warm start: %d training cells solved, %d samples" % (k + 1, len(ws.samples)))
    t1 = time.perf_counter()
    losses = ws.train(epochs)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if log:
        log("scaled warm start: trained, loss %.3e -> %.3e"
            % (float(np.mean(losses[:20])), float(np.mean(losses[-20:]))))
    guesses = {}
    for g in (None, "extrapolate", "learned"):
        per = [run(cell(seed), g) for seed in test_seeds]
        agg = {k: sum(p[k] for p in per) for k in ("newton_iters", "cg_iters", "converged_steps")}
        agg["ms_per_step"] = float(np.mean([p["ms_per_step"] for p in per]))
        if g == "learned":
            agg["learned_guess_taken"] = sum(p["learned_guess_taken"] for p in per)
        guesses[g or "previous"] = agg
        if log:
            log("scaled warm start: %s guess done" % (g or "previous"))
    return {"grid": n, "levels": 4, "widths": list(ws.net.widths), "in_channels": 18,
            "train_cells": len(train_seeds), "test_cells": len(test_seeds),
            "increments_per_cell": steps, "samples": len(ws.samples), "epochs": epochs,
            "data_s": t1 - t0, "train_s": t2 - t1,
            "loss_first_last": [float(np.mean(losses[:20])), float(np.mean(losses[-20:]))],
            "guesses": guesses}


def batch_bench(w, steps):
    """The six unit load cases of the cell, `steps` increments each after one
    untimed increment: solved one cell after the other, then as one batch
    (one solver per case on its own stream, hfe_solve_batch), from the same
    states. Each solver's launch shapes come from the autotuner."""
    import torch
    from paper_2207_10657_amd import Solver, solve_batch
    cases = unit_load_cases(float(w.load_path[0][0, 0]))
    solvers = [Solver(w.shape, w.element, own_stream=True) for _ in cases]
    tuned = None
    for s, dE in zip(solvers, cases):
        s.setup(w.phase, w.materials)
        s.apply_load_step(dE)
        tuned = s.autotune()
    solve_batch(solvers)
    cks = [s.get_state() for s in solvers]

    def run(batched):
        mv = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for s, dE in zip(solvers, cases):
                s.apply_load_step(dE)
            if batched:
                reps = solve_batch(solvers)
            else:
                reps = [s.solve_increment() for s in solvers]
            mv += sum(r["matvecs"] for r in reps)
        torch.cuda.synchronize()
        return mv, time.perf_counter() - t0

    mv_seq, dt_seq = run(False)
    out_seq = [s.homogenized_stress() for s in solvers]
    for s, ck in zip(solvers, cks):
        s.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
    mv_bat, dt_bat = run(True)
    same = all(np.array_equal(a, s.homogenized_stress()) for a, s in zip(out_seq, solvers))
    for s in solvers:
        s.close()
    return {"cases": 6, "steps_timed": steps,
            "sequential": {"value": w.nvox * mv_seq / dt_seq / 1e9, "ms": dt_seq * 1e3,
                           "matvecs": mv_seq},
            "batched": {"value": w.nvox * mv_bat / dt_bat / 1e9, "ms": dt_bat * 1e3,
                        "matvecs": mv_bat},
            "unit": "Gvoxel-matvec/s", "speedup": dt_seq / dt_bat,
            "same_results_as_sequential": bool(same and mv_seq == mv_bat),
            "autotuned_launch": tuned}

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def population_batch_bench(n_cells=64, sizes=(32, 48, 64, 96), strain=1e-4, seed=2207,
                           log=None):
    """A population of cells of uneven sizes, each under the six unit load
    cases: n_cells cells of the 3D recipe (vf 0.25, radii 4-8 voxels scaled
    with the grid, microstructure seed 3000 + i), sizes drawn uniformly from
    `sizes` by `seed`; per cell the increment `strain` along each Voigt
    direction (xx, yy, zz, yz, xz, xy; engineering shears) from the fresh
    state, 6 n_cells solves, and the cell's effective stiffness
    C_IJ = Sigma_I / strain_J. Six contexts per size (each on its own stream)
    serve all cells of that size. Batched: one cell per size at a time, its
    6 solves and those of the other sizes' cells in one hfe_solve_batch call
    (up to 6 len(sizes) solves); sequential: the same solves one context at
    a time. Times count the solves only (not setup), and both runs must give
    the same bits."""
    import torch
    from paper_2207_10657_amd import Solver, solve_batch
    from synthetic import inclusion_microstructure, MATRIX_DAMAGE, INCLUSION_ELASTIC
    mats = [dict(MATRIX_DAMAGE), dict(INCLUSION_ELASTIC)]
    draw = np.random.default_rng(seed).integers(0, len(sizes), n_cells)
    cells = [(sizes[k], 3000 + i) for i, k in enumerate(draw)]
    pool = {n: [Solver((n, n, n), "q1", own_stream=True) for _ in range(6)] for n in sizes}
    cases = []
    for (i, j) in VOIGT:
        dE = np.zeros((3, 3))
        dE[i, j] = dE[j, i] = strain if i == j else strain / 2
        cases.append(dE)

    def phase_of(n, sd):
        return inclusion_microstructure((n, n, n), 4.0 * n / 64, 8.0 * n / 64, 0.25, sd)[0]

    def prepare(group):
        for n, sd in group:
            ph = phase_of(n, sd)
            for s, dE in zip(pool[n], cases):
                s.setup(ph, mats)
                s.apply_load_step(dE)

    def stiffness_of(n):
        C = np.zeros((6, 6))
        for J, s in enumerate(pool[n]):
            S = s.homogenized_stress()
            for I, (i, j) in enumerate(VOIGT):
                C[I, J] = S[i, j] / strain
        return C

    def run(batched):
        by_size = {n: [c for c in cells if c[0] == n] for n in sizes}
        rounds = []
        while any(by_size.values()):
            rounds.append([by_size[n].pop(0) for n in sizes if by_size[n]])
        if not batched:
            rounds = [[c] for r in rounds for c in r]
        secs, vm, conv, Cs = 0.0, 0.0, 0, {}
        for r in rounds:
            prepare(r)
            solvers = [s for n, _ in r for s in pool[n]]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = solve_batch(solvers) if batched else [s.solve_increment() for s in solvers]
            torch.cuda.synchronize()
            secs += time.perf_counter() - t0
            vm += sum(rep["matvecs"] * int(np.prod(s.shape)) for rep, s in zip(reps, solvers))
            conv += sum(int(rep["converged"]) for rep in reps)
            for n, sd in r:
                Cs[sd] = stiffness_of(n)
            if log:
                log("population %s: %d cells done" % ("batch" if batched else "one by one",
                                                      len(Cs)))
        return secs, vm, conv, Cs

    dt_seq, vm_seq, conv_seq, C_seq = run(False)
    dt_bat, vm_bat, conv_bat, C_bat = run(True)
    for ss in pool.values():
        for s in ss:
            s.close()
    same = all(np.array_equal(C_seq[k], C_bat[k]) for k in C_seq)
    per_size = {}
    for n in sizes:
        Cn = [C_bat[sd] for m, sd in cells if m == n]
        if Cn:
            per_size["%d^3" % n] = {"cells": len(Cn),
                                    "C11_mean": float(np.mean([C[0, 0] for C in Cn])),
                                    "C44_mean": float(np.mean([C[3, 3] for C in Cn])),
                                    "C11_spread": float(np.std([C[0, 0] for C in Cn]))}
    return {"cells": n_cells, "sizes": list(sizes), "solves": 6 * n_cells,
            "converged": conv_bat,
            "sequential": {"value": vm_seq / dt_seq / 1e9, "ms": dt_seq * 1e3,
                           "converged": conv_seq},
            "batched": {"value": vm_bat / dt_bat / 1e9, "ms": dt_bat * 1e3},
            "unit": "Gvoxel-matvec/s", "speedup": dt_seq / dt_bat,
            "same_results_as_sequential": bool(same and vm_seq == vm_bat),
            "effective_stiffness": per_size,
            "note": "increment %.0e from the fresh cell along each Voigt direction; C from the "
                    "homogenized stress; solve time only (context setup excluded); launch "
                    "shapes at the library's defaults" % strain}


# Counter summaries written by `--pmc-summary` (one per grid); read back for
# roofline.traffic.
def traffic_file(grid):
    return os.path.join(ROOT, "profiles", "hbm_traffic_%dcubed.md" % grid)
CSRC = os.path.join(ROOT, "paper_2207_10657_amd", "csrc")
# sources each timed kernel is compiled from: a counter reading is void once
# any of them has changed
KERNEL_SOURCES = {
    "stiffness": ["k_element.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
    "stiffness_f32": ["k_element.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
    "trial": ["k_element.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
    "residual": ["k_element.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
    "fft_plane_fwd": ["k_fft.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
    "fft_pencil_green": ["k_fft.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
    "fft_plane_inv": ["k_fft.hip", "hfe_internal.h", "hfe_reduce.h", "hfe_cg.h"],
}
# device kernel name (as rocprofv3 prints it) -> timed kernel; the probe runs
# the Hessian and the plain FFT passes, the solver the CG-fused ones
PMC_KERNELS = [("k_hessian<double,", "stiffness"), ("k_hessian_col<double,", "stiffness_col"),
               ("k_brick<0,", "residual"),
               ("k_plane<0,double>", "fft_plane_fwd"), ("k_pencil<0,double>", "fft_pencil_green"),
               ("k_plane<1,double>", "fft_plane_inv"), ("copyBuffer", "copy")]
PROBE_REPS = 5
LBFGS_STEPS = 2
PROBE_STEPS = 2
# Hessian launch shapes by tuning index: bricks of nodes (x, y, z), and
# marching columns of CX x CY nodes over BZ node layers (cx, cy, bz)
BRICKS = {0: (8, 8, 4), 1: (8, 8, 8), 2: (16, 8, 4), 3: (16, 4, 4), 4: (8, 4, 4)}
COLUMNS = {5: (16, 16, 16), 6: (16, 16, 8), 7: (16, 8, 16), 8: (16, 8, 8), 9: (8, 8, 8),
           10: (8, 8, 16), 11: (16, 8, 32), 12: (16, 16, 32)}


def progress(what):
    """One line on stderr per finished section (stdout carries only the JSON
    line)."""
    print("[bench] %s" % what, file=sys.stderr, flush=True)


def tensile_bench(W=6, K=4, grid=64):
    """The paper's own damage law (Appendix A, tensile masking) in the setting
    of its ASR example on the 64^3 cell: cement paste and aggregates under that
    law, gel sites expanding at zero macroscopic strain (workload asr_3d64).
    W untimed increments (elastic), then K timed ones from the onset of
    cracking; launch shapes autotuned at the first timed state. The Hessian
    runs its non-symmetric variant (a second per-point factor)."""
    import torch
    from paper_2207_10657_amd import Solver
    from synthetic import workload
    w = workload("asr_3d%d" % grid)
    s = Solver(w.shape, w.element)
    s.setup(w.phase, w.materials)

    def load(n):
        s.set_eigenstrain(w.eig_phase, w.eig_path[n])
        s.apply_load_step(w.load_path[n])

    for n in range(W):
        load(n)
        s.solve_increment(SOLVE)
    tuning = s.autotune()
    ck = s.get_state()
    per = []

    def steps():
        mv = 0
        per.clear()
        for n in range(W, W + K):
            load(n)
            r = s.solve_increment(SOLVE)
            mv += r["matvecs"]
            per.append({k: r[k] for k in ("newton_iters", "rejected", "cg_iters", "r_eq", "converged")})
        return mv

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv = steps()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
    s.set_profiling(True)
    steps()
    torch.cuda.synchronize()
    st = s.kernel_stats()
    soft = s.soft_points()[1]
    s.set_profiling(False)
    hc, hms = st.get("stiffness", (0, 0.0))
    return {"workload": "asr_3d%d" % grid, "value": w.nvox * mv / dt / 1e9,
            "unit": "Gvoxel-matvec/s", "ms_per_step": dt / K * 1e3, "steps_timed": [W, W + K - 1],
            "matvecs": mv, "converged_steps": sum(int(p["converged"]) for p in per),
            "per_step": list(per), "hessian_us_per_launch": hms / max(hc, 1) * 1e3,
            "softening_points_mean": soft, "launch_shapes": tuning,
            "note": "paste and aggregates under the tensile-masking law, gel eigenstrain growing "
                    "1e-4 per increment at zero macroscopic strain; increments that reach the "
                    "Newton limit (50) end unconverged, as the oracle does on such increments"}


def hessian_scaling(grids=(64, 128), launches=50):
    """The FP64 Hessian (K d, the dominant kernel) on the cells of the
    workload recipe, timed inside projected-Hessian applications, at two
    states: the damage onset of the load path (load
    steps 0 and 1 solved under the library's default Newton limit, step 2
    applied) and a heavily softening one (E_xx = 2e-3 plus a random
    fluctuation, history at kappa0). Per state: the event-timed duration per
    launch at the autotuned shape, the softening points, and the roofline
    against HESSIAN_MIN_BYTES_PER_VOXEL. The 64^3 working set stays in the
    256 MB Infinity Cache; the 128^3 one streams from HBM."""
    import torch
    from paper_2207_10657_amd import Solver
    from synthetic import workload
    out = {}
    for n in grids:
        w = workload("c1_3d%d" % n)
        s = Solver(w.shape, w.element)
        s.setup(w.phase, w.materials)
        kh0 = s.get_state()["kappa_hist"]
        rng = np.random.default_rng(5)
        d = torch.tensor(rng.normal(size=(3,) + w.shape), device="cuda")

        def timed(state):
            # the Hessian inside projected-Hessian applications: between two
            # of its launches the Green's operator runs, as in the CG loop and
            # in the counter probe, so it does not find its inputs left in the
            # Infinity Cache by itself
            tuning = s.autotune()
            out = s.new_nodal()
            for _ in range(5):
                s.apply_projected_hessian(d, out)
            s.set_profiling(True)
            for _ in range(launches):
                s.apply_projected_hessian(d, out)
            torch.cuda.synchronize()
            c, ms = s.kernel_stats()["stiffness"]
            s.set_profiling(False)
            us = ms / c * 1e3
            alg = HESSIAN_MIN_BYTES_PER_VOXEL * w.nvox
            return {"state": state, "us_per_launch": us, "softening_points": s.soft_points()[0],
                    "algorithmic_bytes": alg, "achieved_GBs": alg / us / 1e3,
                    "frac": alg / us / 1e3 / HBM_PEAK_GBS, "hessian_shape": tuning["brick_shape"],
                    "launch_shapes": tuning}

        res = {}
        for k in range(PROBE_STEPS):
            s.apply_load_step(w.load_path[k])
            s.solve_increment()
        s.apply_load_step(w.load_path[PROBE_STEPS])
        res["onset"] = timed("load steps 0-1 solved (i_NR,max 50), step 2 applied")
        E = np.zeros((3, 3))
        E[0, 0] = 2e-3
        s.set_state(4e-4 * rng.normal(size=(3,) + w.shape), kh0, E, 0.0, 0.0)
        res["softening"] = timed("E_xx = 2e-3 plus a random fluctuation")
        out["%d^3" % n] = res
        s.close()
    return out


def hessian_label(shape_index):
    """Counter label of a Hessian launch shape: the brick, or the column (the
    layers per block are a launch argument, not part of the kernel's name)."""
    if shape_index in BRICKS:
        return "stiffness:%dx%dx%d" % BRICKS[shape_index]
    return "stiffness:col%dx%d" % COLUMNS[shape_index][:2]


def sources_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def read_pmc(path):
    """Per-dispatch counter values from rocprofv3 counter_collection CSVs."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % path)
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                name = row.get("Kernel_Name", "").replace(" ", "")
                label = next((lab for key, lab in PMC_KERNELS if key in name), None)
                if label == "stiffness":
                    # one entry per brick shape: k_hessian<double,BX,BY,BZ,FULL>
                    dims = name.split("k_hessian<double,", 1)[1].split(">", 1)[0].split(",")[:3]
                    label = "stiffness:" + "x".join(dims)
                elif label == "stiffness_col":
                    # one entry per column: k_hessian_col<double,CX,CY,NS>
                    dims = name.split("k_hessian_col<double,", 1)[1].split(">", 1)[0].split(",")[:2]
                    label = "stiffness:col" + "x".join(dims)
                if label is not None:
                    rows.append((int(row["Dispatch_Id"]), label, float(row["Counter_Value"])))
    out = {}
    for _, label, v in sorted(rows):
        out.setdefault(label, []).append(v)
    # the probe's own dispatches are the last PROBE_REPS of each kernel (the
    # autotuner and the load step launch the same kernels before them)
    return {k: v[-PROBE_REPS:] for k, v in out.items()}


# which launch-shape fields a kernel's traffic depends on
SHAPE_KEYS = {"stiffness": ("brick_shape",), "stiffness_f32": ("brick_shape32",),
              "residual": (), "trial": (),
              "fft_plane_fwd": ("plane_threads",), "fft_plane_inv": ("plane_threads",),
              "fft_pencil_green": ("pencil_cols", "pencil_threads")}


def pmc_summary(fetch_dir, write_dir, grid, tuning=None):
    """Markdown summary of a FETCH_SIZE and a WRITE_SIZE pass over `--probe`.

    Both counters are in KiB per dispatch. The copy kernel moves COPY_BYTES in
    and COPY_BYTES out, which fixes one scale factor per counter."""
    fetch, write = read_pmc(fetch_dir), read_pmc(write_dir)
    tuning = dict(tuning or {})
    soft_points = float(tuning.pop("soft_points", 0.0))
    if "copy" not in fetch or "copy" not in write:
        raise SystemExit("the calibration copy is missing from the counter runs")
    # the calibration copies are the last copy dispatches of the probe
    kf = COPY_BYTES / (1024.0 * np.median(fetch["copy"]))
    kw = COPY_BYTES / (1024.0 * np.median(write["copy"]))
    shape = (grid, grid, grid)
    rows, table = [], {}
    labels = sorted({hessian_label(k) for k in list(BRICKS) + list(COLUMNS)})
    labels += ["residual", "fft_plane_fwd", "fft_pencil_green", "fft_plane_inv"]
    for label in labels:
        if label not in fetch or label not in write:
            continue
        base = label.split(":")[0]
        fb = float(np.median(fetch[label])) * 1024.0 * kf
        wb = float(np.median(write[label])) * 1024.0 * kw
        alg = algorithmic_bytes(base, shape, soft_points)
        keys = () if base == "stiffness" else SHAPE_KEYS[base]   # the brick is in the label
        table[label] = {"fetch_bytes": fb, "write_bytes": wb, "dispatches": len(fetch[label]),
                        "algorithmic_bytes": alg, "sources": sources_digest(base),
                        "launch": {k: tuning[k] for k in keys} if tuning else None}
        rows.append("| %s | %d | %.2f | %.2f | %.2f | %.2f |" % (
            label, len(fetch[label]), fb / 1e6, wb / 1e6, (fb + wb) / 1e6,
            (fb + wb) / alg if alg else float("nan")))
    lines = [
        "| kernel | dispatches | fetch MB | write MB | HBM MB / launch | / algorithmic |",
        "|---|---|---|---|---|---|"] + rows + [
        "",
        "Calibration (copy of %d bytes): FETCH_SIZE x %.3f, WRITE_SIZE x %.3f." % (COPY_BYTES, kf, kw),
        "State: %d softening points (%.1f %% of the points); the element kernels' algorithmic "
        "bytes include 48 B for each." % (soft_points, 100.0 * soft_points / (8.0 * grid ** 3)),
        "",
        "```json",
        json.dumps({"grid": grid, "fetch_scale": kf, "write_scale": kw, "soft_points": soft_points,
                    "kernels": table}, indent=1),
        "```"]
    return "\n".join(lines)


def load_traffic(kernel, shape, tuning):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if there is none for this grid and launch shape or the kernel's
    sources changed."""
    try:
        with open(traffic_file(shape[0])) as fh:
            text = fh.read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if kernel == "stiffness":
        label, keys = hessian_label(tuning["brick_shape"]), ()
    else:
        label, keys = kernel, SHAPE_KEYS.get(kernel, ())
    k = blob.get("kernels", {}).get(label)
    if not k or tuple([blob.get("grid")] * 3) != tuple(shape):
        return None
    if k.get("sources") != sources_digest(kernel):
        return None
    if k.get("launch") != {key: tuning[key] for key in keys}:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


def probe(n, tuning_out=None, tuning_in=None):
    """Kernels for counter passes (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE).

    The damage-onset state of the workload recipe at n^3 that
    hessian_scaling times (the first PROBE_STEPS load increments solved
    under the library's default Newton limit, the next one applied), the
    autotuner (the launch shapes the benchmark uses), then, for every Hessian
    brick shape,
    PROBE_REPS projected-Hessian applications at that state, and PROBE_REPS
    device-to-device copies of COPY_BYTES (the copy kernel calibrates the
    counters: it reads and writes exactly COPY_BYTES per launch)."""
    import torch
    from paper_2207_10657_amd import Solver
    from paper_2207_10657_amd.hfe import HfeError
    from synthetic import workload
    w = workload("c1_3d%d" % n)
    s = Solver(w.shape, w.element)
    s.setup(w.phase, w.materials)
    for k in range(PROBE_STEPS):
        s.apply_load_step(w.load_path[k])
        s.solve_increment()
    s.apply_load_step(w.load_path[PROBE_STEPS])
    if tuning_in:
        with open(tuning_in) as fh:
            t = json.load(fh)
        t.pop("soft_points", None)
        s.set_tuning(**t)
        tuned = s.tuning()
    else:
        tuned = s.autotune()
    soft = s.soft_points()[0]
    print("probe launch shapes:", tuned, "softening points:", soft, flush=True)
    if tuning_out:
        with open(tuning_out, "w") as fh:
            json.dump(dict(tuned, soft_points=soft), fh)
    rng = np.random.default_rng(0)
    d = torch.tensor(rng.normal(size=(3,) + w.shape), device="cuda")
    # every Hessian kernel once (FFT shapes as tuned): the bricks, and per
    # column width the tuned shape or else the first with that width
    shapes, cols = list(sorted(BRICKS)), {}
    for k in sorted(COLUMNS):
        key = COLUMNS[k][:2]
        if key not in cols or k == tuned["brick_shape"]:
            cols[key] = k
    shapes += sorted(cols.values())
    for shape_index in shapes:
        try:
            s.set_tuning(brick_shape=shape_index)
        except HfeError:
            continue          # a column that does not divide this grid
        for _ in range(PROBE_REPS):
            s.apply_projected_hessian(d)
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(PROBE_REPS):
        b.copy_(a)
    torch.cuda.synchronize()
    print("probe done: %d^3, copy %d bytes" % (n, COPY_BYTES), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-matvecs", type=int, default=100,
                    help="oracle applications timed for cpu_baseline (about 10 s on 16 cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the same steps")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the six-load-case batch run")
    ap.add_argument("--no-lbfgs", action="store_true",
                    help="skip the L-BFGS run of the first timed load steps")
    ap.add_argument("--no-scaling", action="store_true",
                    help="skip the Hessian-alone line at 64^3 and 128^3")
    ap.add_argument("--no-tensile", action="store_true",
                    help="skip the tensile-masking law (Appendix A) line")
    ap.add_argument("--tuning", metavar="FILE",
                    help="launch shapes (JSON, as config.launch_shapes of a bench line) for the "
                         "timed steps instead of the autotuner's choice, e.g. to profile the "
                         "shapes an unprofiled run chose")
    ap.add_argument("--warm-start-64", action="store_true",
                    help="also run the learned warm start at its configured scale: 64^3 cells, "
                         "the 4-level widening network, 50 training and 5 held-out cells "
                         "(minutes)")
    ap.add_argument("--stall-study", action="store_true",
                    help="also run the timed steps with the CG stall exit in both precisions "
                         "(minutes: the exit leaves Newton steps unconverged)")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the learned warm-start run (16^3 cells)")
    ap.add_argument("--probe", action="store_true",
                    help="short run for hardware-counter passes: after one load step, a few "
                         "projected-Hessian applications and a calibration copy of known size")
    ap.add_argument("--grid", type=int, default=64,
                    help="cell size N of the workload recipe at N^3 (the main line and --probe; "
                         "the default 64 is the benchmark configuration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc runs of --probe "
                         "(FETCH_SIZE, then WRITE_SIZE; csv output)")
    ap.add_argument("--probe-tuning", metavar="FILE",
                    help="--probe: write the launch shapes it used; --pmc-summary: read them")
    ap.add_argument("--probe-set-tuning", metavar="FILE",
                    help="--probe: use these launch shapes instead of autotuning")
    args = ap.parse_args()
    if args.pmc_summary:
        tuning = None
        if args.probe_tuning:
            with open(args.probe_tuning) as fh:
                tuning = json.load(fh)
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.grid, tuning))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver is single-GPU (a batch of cells "
              "would shard across GPUs with no communication); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2207_10657_amd import Solver
    from synthetic import workload

    if args.probe:
        probe(args.grid, args.probe_tuning, args.probe_set_tuning)
        return
    w = workload("c1_3d%d" % args.grid)
    W, K = args.warmup, args.steps
    if W + K > len(w.load_path):
        K = len(w.load_path) - W
    s = Solver(w.shape, w.element)
    s.setup(w.phase, w.materials)
    for n in range(W):
        s.apply_load_step(w.load_path[n])
        s.solve_increment(SOLVE)
    # launch shapes for this grid and state, chosen by measurement (setup)
    if args.tuning:
        with open(args.tuning) as fh:
            t = json.load(fh)
        t = t.get("config", {}).get("launch_shapes", t)
        s.set_tuning(**{k: int(v) for k, v in t.items() if k != "soft_points"})
        tuning = s.tuning()
    else:
        tuning = s.autotune()
    ck = s.get_state()

    detail, sigmas, step_s, states, damages = [], [], [], [], []

    def record(rep):
        return {k: rep[k] for k in ("newton_iters", "rejected", "cg_iters", "restarts",
                                    "boundary_exits", "negcurv_exits", "stall_exits", "r_eq",
                                    "R", "converged")}

    def timed_steps(params=SOLVE, keep_states=False):
        matvecs = newton = cg = converged = 0
        detail.clear()
        sigmas.clear()
        step_s.clear()
        for n in range(W, W + K):
            if keep_states:
                states.append(s.get_state())
            ts = time.perf_counter()
            s.apply_load_step(w.load_path[n])
            rep = s.solve_increment(params)
            step_s.append(time.perf_counter() - ts)     # the solve ends with a synchronisation
            matvecs += rep["matvecs"]
            newton += rep["newton_iters"]
            cg += rep["cg_iters"]
            converged += int(rep["converged"])
            detail.append(record(rep))
            sigmas.append(s.homogenized_stress())
            if keep_states:
                damages.append(s.damage())
                progress("replay step %d: Newton %d, CG %d" % (n, rep["newton_iters"], rep["cg_iters"]))
        return matvecs, newton, cg, converged

    def from_states(params, label):
        """Each timed load step once more, each from the FP64 state before it
        (restarts are bit-exact): per step its time and result, and the
        homogenized stress against the FP64 step from the same state."""
        per, errs, ddmg, mv, secs = [], [], [], 0, 0.0
        for j, st in enumerate(states):
            s.set_state(st["u"], st["kappa_hist"], st["E"], st["R"], st["Rmax"])
            torch.cuda.synchronize()
            ts = time.perf_counter()
            s.apply_load_step(w.load_path[W + j])
            rep = s.solve_increment(params)
            secs += time.perf_counter() - ts
            mv += rep["matvecs"]
            per.append(record(rep))
            S = s.homogenized_stress()
            errs.append(float(np.linalg.norm(S - sig64[j]) / max(np.linalg.norm(sig64[j]), 1e-300)))
            ddmg.append(float(np.abs(s.damage() - damages[j]).max()))
            progress("%s step %d: Newton %d, CG %d, %.2f s, stress error %.1e"
                     % (label, W + j, rep["newton_iters"], rep["cg_iters"],
                        time.perf_counter() - ts, errs[-1]))
        unconverged = sum(1 for p in per if not p["converged"])
        return {"value": w.nvox * mv / secs / 1e9, "unit": "Gvoxel-matvec/s",
                "ms_per_step": secs / len(states) * 1e3,
                "speedup_per_step_vs_fp64": sum(fp64_step_s) / secs,
                "matvecs": mv, "newton_iters": sum(p["newton_iters"] for p in per),
                "cg_iters": sum(p["cg_iters"] for p in per),
                "stall_exits": sum(p["stall_exits"] for p in per),
                "converged_steps": sum(int(p["converged"]) for p in per),
                "unconverged_steps": unconverged,
                "sigma_rel_err_vs_fp64_same_state": errs,
                "sigma_rel_err_max": max(errs) if errs else None,
                "damage_max_diff_vs_fp64_same_state": ddmg,
                "per_step": per}

    progress("setup and autotuning done")
    # timed region: CG iterations replayed from captured HIP graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs, newton, cg, converged = timed_steps()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_detail = list(detail)
    sig64 = list(sigmas)
    fp64_step_s = list(step_s)
    # the same steps under the library's default limit of 50 Newton iterations
    # (the damage-onset increments end there unconverged), for comparison
    s.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
    torch.cuda.synchronize()
    t50 = time.perf_counter()
    capped = timed_steps({})
    torch.cuda.synchronize()
    dt50 = time.perf_counter() - t50
    # the same steps again from the same state (restart is bit-exact), every
    # kernel launch bracketed by HIP events on the library's stream; the state
    # before each step is kept for the runs below
    s.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
    s.set_profiling(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    replay = timed_steps(keep_states=True)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    stats = s.kernel_stats()
    soft_mean = s.soft_points()[1]       # softening points, mean over the Hessian launches
    s.set_profiling(False)
    if replay[0] != matvecs:
        print("warning: event-timed replay differs from the timed run", replay, matvecs,
              file=sys.stderr)

    # each timed step once more from the FP64 state before it: with the
    # mixed-precision CG (FP32 Hessian, FFT and CG vectors; FP64 residual,
    # trial, energy ratio and history), and with the stall exit of the CG
    # (cg_stall = STALL_WINDOW) in both precisions
    mixed = stall = None
    progress("timed steps, 50-iteration comparison and event-timed replay done")
    if not args.no_mixed:
        mixed = from_states(dict(SOLVE, precision="mixed"), "mixed")
        s.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
        s.set_profiling(True)
        for j, st in enumerate(states[:2]):
            s.set_state(st["u"], st["kappa_hist"], st["E"], st["R"], st["Rmax"])
            s.apply_load_step(w.load_path[W + j])
            s.solve_increment(dict(SOLVE, precision="mixed"))
        torch.cuda.synchronize()
        stats32 = s.kernel_stats()
        s.set_profiling(False)
        mixed["kernels_ms_first_two_steps"] = {k: {"launches": c, "total_ms": m}
                                               for k, (c, m) in stats32.items() if c}
        mixed["note"] = ("each step from the FP64 state before it; the stress error is against "
                         "the FP64 solve of the same step from the same state (the FP64 path is "
                         "checked against the oracle); bound %.0e" % MIXED_SIGMA_BOUND)
        mixed["within_bound"] = bool(mixed["sigma_rel_err_max"] <= MIXED_SIGMA_BOUND)
        # a step over the bound where both solves meet the FP64 equilibrium
        # test (the mixed path evaluates residual and r_eq in FP64) ended at
        # two equilibria of the same softening increment
        over = []
        for j, e in enumerate(mixed["sigma_rel_err_vs_fp64_same_state"]):
            if e > MIXED_SIGMA_BOUND:
                over.append({"step": W + j, "sigma_rel_err": e,
                             "damage_max_diff": mixed["damage_max_diff_vs_fp64_same_state"][j],
                             "r_eq_mixed": mixed["per_step"][j]["r_eq"],
                             "r_eq_fp64": step_detail[j]["r_eq"],
                             "both_converged": bool(mixed["per_step"][j]["converged"]
                                                    and step_detail[j]["converged"])})
        mixed["steps_over_bound"] = over
        if args.stall_study:
            stall = {"window": STALL_WINDOW,
                     "fp64": from_states(dict(SOLVE, cg_stall=STALL_WINDOW), "fp64 stall"),
                     "mixed": from_states(dict(SOLVE, precision="mixed", cg_stall=STALL_WINDOW),
                                          "mixed stall"),
                     "note": "the CG returns its iterate once its residual has not halved in "
                             "`window` iterations (an exit this library adds to Algorithm 1; "
                             "off by default); each step from the FP64 state before it"}
        progress("mixed precision done")

    # the paper's quasi-Newton remark: the first LBFGS_STEPS timed increments
    # from the same checkpoint by L-BFGS on the approximate energy increment
    lbfgs = None
    if not args.no_lbfgs:
        s.set_state(ck["u"], ck["kappa_hist"], ck["E"], ck["R"], ck["Rmax"])
        per = []
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for n in range(W, W + min(LBFGS_STEPS, K)):
            s.apply_load_step(w.load_path[n])
            r = s.solve_increment_lbfgs()
            per.append({k: r[k] for k in ("iters", "trials", "pairs_skipped", "resets", "r_eq",
                                          "converged", "time_ms")})
        torch.cuda.synchronize()
        dtl = time.perf_counter() - t3
        lbfgs = {"steps": len(per), "ms_per_step": dtl / max(len(per), 1) * 1e3,
                 "per_step": per,
                 "newton_ms_per_step": dt / K * 1e3,
                 "note": "m = 5, Armijo on the approximate energy increment; same checkpoint "
                         "as the timed Newton steps"}

    # dominant kernel: largest total time in the timed region. The Hessian's
    # roofline counts HESSIAN_MIN_BYTES_PER_VOXEL; the bytes this library's
    # layout reads (cached tangent, softening factors) are given beside it.
    kern = max(stats.items(), key=lambda kv: kv[1][1])
    kname, (kcount, kms) = kern
    avg_s = kms / max(kcount, 1) / 1e3
    model = algorithmic_bytes(kname, w.shape, soft_mean)
    alg = HESSIAN_MIN_BYTES_PER_VOXEL * w.nvox if kname == "stiffness" else model
    roof = None
    if alg is not None and avg_s > 0:
        achieved = alg / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": load_traffic(kname, w.shape, tuning),
                "kernel": kname, "algorithmic_bytes": alg,
                "layout_bytes_model": model,
                "softening_points_mean": soft_mean,
                "avg_launch_us": avg_s * 1e6, "launches": kcount,
                "hessian_shape": tuning["brick_shape"]}
    value = w.nvox * matvecs / dt / 1e9
    out = {
        "metric": "projected-Hessian Gvoxel-matvec/s (% HBM peak); time/load step at 1e-8 resid",
        "value": value,
        "unit": "Gvoxel-matvec/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D %d^3 Q1 inclusion cell (vf 0.25, seed %d), damage matrix, "
                               "uniaxial 30 x 2e-4 load path, FP64 TR+Steihaug tol 1e-8"
                               % (args.grid, 3 if args.grid == 128 else 1),
                   "load_steps_timed": [W, W + K - 1], "i_nr_max": NEWTON_CAP,
                   "matvecs": matvecs,
                   "newton_iters": newton, "cg_iters": cg, "converged_steps": converged,
                   "per_step": step_detail, "launch_shapes": tuning},
        "roofline": roof,
        "kernel_timing": "HIP events around every launch in a replay of the timed steps from the "
                         "same checkpoint (kernel-by-kernel launches, %.1f ms/step)" % (dt_prof / K * 1e3),
        "kernels_ms": {k: {"launches": c, "total_ms": m} for k, (c, m) in stats.items() if c},
        "newton_limit_50": {"ms_per_step": dt50 / K * 1e3, "matvecs": capped[0],
                            "newton_iters": capped[1], "cg_iters": capped[2],
                            "converged_steps": capped[3],
                            "value": w.nvox * capped[0] / dt50 / 1e9,
                            "note": "the same steps with the library's default i_NR,max = 50: "
                                    "a time per 50 Newton iterations where a step does not "
                                    "converge"},
        "mixed_precision": mixed,
        "cg_stall_exit": stall if stall is not None else "not run (bench.py --stall-study)",
        "lbfgs": lbfgs,
    }
    if not args.no_batch:
        out["batch_six_load_cases"] = batch_bench(w, 2)
        out["batch_population"] = population_batch_bench(log=progress)
        progress("batches done")
    if not args.no_tensile:
        out["tensile_law"] = tensile_bench()
        progress("tensile-masking law done")
    if not args.no_scaling:
        hs = hessian_scaling()
        out["hessian_scaling"] = hs
        # the Hessian streaming from HBM: the 128^3 cell at its damage onset
        on = hs.get("128^3", {}).get("onset")
        if on:
            out["roofline_128"] = {
                "bound": "hbm", "achieved": on["achieved_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": on["frac"],
                "traffic": load_traffic("stiffness", (128, 128, 128), on["launch_shapes"]),
                "kernel": "stiffness", "algorithmic_bytes": on["algorithmic_bytes"],
                "avg_launch_us": on["us_per_launch"], "softening_points": on["softening_points"],
                "state": "128^3 cell of the recipe (seed 3), " + on["state"],
                "hessian_shape": on["hessian_shape"]}
        progress("Hessian scaling done")
    if not args.no_warm_start:
        out["warm_start"] = warm_start_bench()
        progress("warm start done")
    if args.warm_start_64:
        out["warm_start_64"] = warm_start_scaled_bench(log=progress)
        progress("scaled warm start done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_matvecs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
