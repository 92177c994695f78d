"""Named synthetic workloads: grid, element, microstructure, materials, loads.

Materials: a damaging matrix (E=1, nu=0.3, isotropic damage driven by the
energy-norm equivalent strain, linear softening between kappa0=1e-3 and
kappaf=5e-3) with stiff linear-elastic inclusions (E=10, nu=0.3). Loads are
strain controlled: equal increments of the macroscopic strain component
``E_xx``, every other component held at zero.
"""
from dataclasses import dataclass, field
import numpy as np

from .microstructure import inclusion_microstructure

# material records: plain dicts so both sides can read them without sharing code
MATRIX_DAMAGE = {"kind": "damage", "E": 1.0, "nu": 0.3, "kappa0": 1e-3, "kappaf": 5e-3}
INCLUSION_ELASTIC = {"kind": "elastic", "E": 10.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}
# the tensile-masking law (the paper's Appendix A) with the matrix's threshold
# and softening: relative softening slope alpha = kappa0 / (kappaf - kappa0) = 0.25
MATRIX_TENSILE = {"kind": "tensile", "E": 1.0, "nu": 0.3, "kappa0": 1e-3, "kappaf": 5e-3}
# the ASR example's phases (the paper's table of material properties, moduli
# divided by the cement paste's 12 GPa): paste and aggregates damage in
# tension with kappa0 = f_t / E; the softening end kappaf = 10 kappa0 stands in
# for the paper's fracture-energy regularisation, which needs its mesh size
ASR_PASTE = {"kind": "tensile", "E": 1.0, "nu": 0.3, "kappa0": 2.5e-4, "kappaf": 2.5e-3}
ASR_AGGREGATE = {"kind": "tensile", "E": 59.0 / 12.0, "nu": 0.3, "kappa0": 10.0 / 59e3,
                 "kappaf": 100.0 / 59e3}
ASR_GEL = {"kind": "elastic", "E": 11.0 / 12.0, "nu": 0.18, "kappa0": 0.0, "kappaf": 0.0}


def uniaxial_load_path(dim, total, steps):
    """``steps`` equal increments of ``E_xx`` summing to ``total``.

    Returns an array ``(steps, 3, 3)`` of macroscopic strain increments (the
    3x3 form is used for 2D plane strain as well; only the in-plane block is
    read there).
    """
    inc = np.zeros((steps, 3, 3))
    inc[:, 0, 0] = total / steps
    return inc


@dataclass
class Workload:
    name: str
    dim: int
    shape: tuple          # (ny, nx) or (nz, ny, nx)
    element: str          # "p1pair" (2D, two linear triangles per pixel) or "q1" (3D)
    phase: np.ndarray
    materials: list       # indexed by phase id
    load_path: np.ndarray  # (steps, 3, 3)
    info: dict = field(default_factory=dict)
    eig_phase: int = -1          # phase whose eigenstrain grows along the path (or -1)
    eig_path: np.ndarray = None  # (steps, 3, 3): that phase's eigenstrain at each step

    @property
    def nvox(self):
        return int(np.prod(self.shape))

    @property
    def nq(self):
        return 2 if self.element == "p1pair" else 8


def workload(name, steps=None):
    """Build one of the named workloads.

    ``c0_2d32``   2D plane strain 32x32, circles r 3..5 px, vf 0.3, seed 0,
                  20 steps of E_xx to 0.5%.
    ``c1_3d64``   3D 64^3, spheres r 4..8 vox, vf 0.25, seed 1,
                  30 steps of E_xx to 0.6%.
    ``c1_3dN``    (N in 8..128) the same recipe on an N^3 grid with radii
                  scaled by N/64 (small parity and large bandwidth cases),
                  seed 3 for N=128, else seed 1.
    ``gel_3dN``   the c1_3dN cell with expanding sites: the inclusion voxels
                  whose centres lie within half a radius (at least one voxel
                  diagonal) of an inclusion centre form an elastic phase 2
                  whose isotropic eigenstrain grows by 2.5e-4 per step, at zero
                  macroscopic strain (20 steps).
    ``asr_3dN``   the gel_3dN geometry with the ASR example's phases: cement
                  paste and aggregates under the tensile-masking law, gel
                  sites expanding by 1e-4 per step (20 steps).
    ``steps`` truncates the load path (the increment size is kept).
    """
    if name.startswith("asr_3d"):
        base = workload("gel_3d" + name[len("asr_3d"):], steps)
        nsteps = len(base.eig_path)
        eig = np.array([(k + 1) * 1e-4 * np.eye(3) for k in range(nsteps)])
        return Workload(name=name, dim=3, shape=base.shape, element="q1", phase=base.phase,
                        materials=[dict(ASR_PASTE), dict(ASR_AGGREGATE), dict(ASR_GEL)],
                        load_path=base.load_path, info=base.info, eig_phase=2, eig_path=eig)
    if name.startswith("gel_3d"):
        n = int(name[len("gel_3d"):])
        base = workload("c1_3d%d" % n)
        shape = np.array(base.shape[::-1], dtype=np.float64)          # (nx, ny, nz)
        grid = np.stack(np.meshgrid(*[np.arange(k) + 0.5 for k in base.shape[::-1]],
                                    indexing="ij"), axis=-1)           # voxel centres (x, y, z)
        core = np.zeros(base.shape[::-1], dtype=bool)
        for centre, r in base.info["inclusions"]:
            d = grid - np.asarray(centre, dtype=np.float64)
            d -= shape * np.round(d / shape)                          # minimum image
            core |= np.sqrt(np.sum(d * d, axis=-1)) <= max(0.5 * r, 0.87)
        core = core.transpose(2, 1, 0) & (base.phase == 1)            # back to (z, y, x)
        phase = base.phase.copy()
        phase[core] = 2
        nsteps = 20 if steps is None else steps
        eig = np.array([(k + 1) * 2.5e-4 * np.eye(3) for k in range(nsteps)])
        gel = dict(INCLUSION_ELASTIC)
        return Workload(name=name, dim=3, shape=base.shape, element="q1", phase=phase,
                        materials=[dict(MATRIX_DAMAGE), dict(INCLUSION_ELASTIC), gel],
                        load_path=np.zeros((nsteps, 3, 3)), info=dict(base.info, gel_voxels=int(core.sum())),
                        eig_phase=2, eig_path=eig)
    if name == "c0_2d32":
        shape, (rmin, rmax), vf, seed = (32, 32), (3.0, 5.0), 0.3, 0
        total, nsteps, element = 5e-3, 20, "p1pair"
    elif name.startswith("c1_3d"):
        n = int(name[len("c1_3d"):])
        scale = n / 64.0
        shape, (rmin, rmax), vf = (n, n, n), (4.0 * scale, 8.0 * scale), 0.25
        seed = 3 if n == 128 else 1
        total, nsteps, element = 6e-3, 30, "q1"
    else:
        raise KeyError(name)
    phase, info = inclusion_microstructure(shape, rmin, rmax, vf, seed)
    path = uniaxial_load_path(len(shape), total, nsteps)
    if steps is not None:
        path = path[:steps]
    return Workload(name=name, dim=len(shape), shape=shape, element=element,
                    phase=phase, materials=[dict(MATRIX_DAMAGE), dict(INCLUSION_ELASTIC)],
                    load_path=path, info=info)
