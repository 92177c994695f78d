"""Seeded two-phase microstructures on periodic voxel grids.

Arrays are indexed ``[z, y, x]`` in 3D and ``[y, x]`` in 2D (x fastest in
memory), which is the layout the C-ABI expects for the phase map. Phase 0 is
the matrix, phase 1 the inclusions.

Recipe (stand-in for the paper's random aggregate microstructures, Sec. 3.3,
which are not available): draw a centre uniformly in the periodic cell and a
radius uniformly in ``[r_min, r_max]``; accept the inclusion only if its
minimum-image centre distance to every accepted inclusion is at least the sum
of the two radii (no overlap); mark every voxel whose centre ``x + 1/2`` lies
within the radius (minimum image); stop as soon as the marked fraction reaches
the target volume fraction.
"""
import numpy as np


def _min_image(delta, n):
    """Shortest periodic difference per axis (``delta`` in voxel units)."""
    return delta - n * np.round(delta / n)


def inclusion_microstructure(shape, r_min, r_max, vf, seed, max_rejects=100000):
    """Random non-overlapping circular (2D) / spherical (3D) inclusions.

    ``shape`` is ``(ny, nx)`` or ``(nz, ny, nx)``. Returns ``(phase, info)``
    with ``phase`` a uint8 array of that shape and ``info`` a dict holding the
    accepted inclusions and the achieved volume fraction.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if dim not in (2, 3):
        raise ValueError("shape must be 2D or 3D")
    rng = np.random.default_rng(seed)
    # per-axis sizes in (x, y[, z]) order
    n_xyz = np.array(shape[::-1], dtype=np.float64)
    # voxel centres, per axis, in (x, y, z) order
    axes = [np.arange(n, dtype=np.float64) + 0.5 for n in shape[::-1]]
    centres_grid = np.meshgrid(*axes[::-1], indexing="ij")  # [z,y,x] arrays
    centres_grid = centres_grid[::-1]                        # now x, y, z order
    phase = np.zeros(shape, dtype=np.uint8)
    accepted = []
    rejects = 0
    target = vf * phase.size
    while np.count_nonzero(phase) < target:
        c = rng.uniform(0.0, 1.0, size=dim) * n_xyz
        r = rng.uniform(r_min, r_max)
        ok = True
        for (c2, r2) in accepted:
            dist = np.linalg.norm(_min_image(c - c2, n_xyz))
            if dist < r + r2:
                ok = False
                break
        if not ok:
            rejects += 1
            if rejects > max_rejects:
                raise RuntimeError("inclusion placement gave up after %d rejections"
                                   % max_rejects)
            continue
        accepted.append((c, r))
        d2 = np.zeros(shape, dtype=np.float64)
        for m in range(dim):
            d2 += _min_image(centres_grid[m] - c[m], n_xyz[m]) ** 2
        phase[d2 <= r * r] = 1
    info = {"inclusions": [(tuple(c), float(r)) for c, r in accepted],
            "vf": float(np.count_nonzero(phase)) / phase.size,
            "rejects": rejects}
    return phase, info


def laminate_microstructure(shape, layers_x):
    """Layers normal to x: ``layers_x[i]`` is the phase of voxel column ``x=i``.

    Interfaces are grid-aligned, so the FE effective stiffness of the laminate
    equals the classical laminate means exactly.
    """
    shape = tuple(int(s) for s in shape)
    layers_x = np.asarray(layers_x, dtype=np.uint8)
    if layers_x.shape != (shape[-1],):
        raise ValueError("one phase id per x column expected")
    return np.broadcast_to(layers_x, shape).copy()
