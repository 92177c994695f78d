"""Linear finite elements on a periodic grid of unit voxels (oracle).

The paper builds its projector from the derivative of a linear FE
discretisation evaluated at quadrature points (Sec. 2.1, after eq.
proj_Fourier_2). Two element types are used:

* ``q1``     trilinear hexahedron per voxel, 2x2x2 Gauss points
             (xi = 1/2 -+ 1/(2 sqrt 3)), quadrature index q = qx + 2 qy + 4 qz;
* ``p1pair`` two linear triangles per pixel, one point each:
             T1 = corners (0,0),(1,0),(0,1);  T2 = corners (1,1),(0,1),(1,0).

Nodes sit at voxel corners; element ``e`` at integer position ``x`` uses the
nodes ``x + o_a`` with ``o_a`` in {0,1}^d, local index a = ax + 2 ay (+ 4 az).
Fields are numpy arrays indexed ``[z, y, x]`` (3D) or ``[y, x]`` (2D).

Pinned by: closed-form FE Laplacian symbols (``test_oracle_fe``), a dense
brute-force D assembled element by element, and the Fourier identity
DFT(D u) = Dhat * DFT(u).
"""
import itertools
import numpy as np

GAUSS_1D = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))


def offsets(dim):
    """Local node offsets o_a, a = ax + 2 ay (+ 4 az), as (x, y[, z]) tuples."""
    return [tuple((a >> m) & 1 for m in range(dim)) for a in range(2 ** dim)]


def _lin(o, t):
    """1D linear shape function of the node at offset o in {0,1}, at t."""
    return t if o == 1 else 1.0 - t


def _dlin(o):
    return 1.0 if o == 1 else -1.0


def shape_gradients(element):
    """B[q, a, j] = dN_a/dx_j at quadrature point q (unit voxel)."""
    if element == "q1":
        dim = 3
        offs = offsets(3)
        pts = [tuple(GAUSS_1D[(q >> m) & 1] for m in range(3)) for q in range(8)]
        B = np.zeros((8, 8, 3))
        for q, xi in enumerate(pts):
            for a, o in enumerate(offs):
                for j in range(dim):
                    val = _dlin(o[j])
                    for m in range(dim):
                        if m != j:
                            val *= _lin(o[m], xi[m])
                    B[q, a, j] = val
        return B
    if element == "p1pair":
        # barycentric gradients of the two triangles, written per pixel corner
        B = np.zeros((2, 4, 2))
        corner = {o: a for a, o in enumerate(offsets(2))}
        # T1: N = 1-x-y at (0,0), x at (1,0), y at (0,1)
        B[0, corner[(0, 0)]] = (-1.0, -1.0)
        B[0, corner[(1, 0)]] = (1.0, 0.0)
        B[0, corner[(0, 1)]] = (0.0, 1.0)
        # T2: N = x+y-1 at (1,1), 1-x at (0,1), 1-y at (1,0)
        B[1, corner[(1, 1)]] = (1.0, 1.0)
        B[1, corner[(0, 1)]] = (-1.0, 0.0)
        B[1, corner[(1, 0)]] = (0.0, -1.0)
        return B
    raise ValueError(element)


def element_dim(element):
    return 3 if element == "q1" else 2


def _shift(field, o):
    """field(x + o) for a periodic array indexed [z, y, x] / [y, x]."""
    dim = len(o)
    out = field
    for m in range(dim):
        if o[m]:
            axis = field.ndim - 1 - m          # x is the last axis
            out = np.roll(out, -o[m], axis=axis)
    return out


def _unshift(field, o):
    """field(x - o)."""
    dim = len(o)
    out = field
    for m in range(dim):
        if o[m]:
            axis = field.ndim - 1 - m
            out = np.roll(out, o[m], axis=axis)
    return out


def gradient(u, element):
    """Full displacement gradient at quadrature points.

    ``u`` has shape (d, *grid). Returns H of shape (*grid, nq, d, d) with
    H[..., q, i, j] = sum_a B[q, a, j] u_i(x + o_a).
    """
    B = shape_gradients(element)
    dim = element_dim(element)
    nq = B.shape[0]
    grid = u.shape[1:]
    H = np.zeros(grid + (nq, dim, dim))
    for a, o in enumerate(offsets(dim)):
        us = np.stack([_shift(u[i], o) for i in range(dim)], axis=-1)  # (*grid, d)
        for q in range(nq):
            H[..., q, :, :] += us[..., :, None] * B[q, a][None, :]
    return H


def divergence(tau, element):
    """Adjoint of ``gradient`` under the plain sum over points and components.

    ``tau`` has shape (*grid, nq, d, d). Returns f of shape (d, *grid) with
    f_i(x) = sum_a sum_q sum_j B[q, a, j] tau_{q,ij}(x - o_a).
    """
    B = shape_gradients(element)
    dim = element_dim(element)
    nq = B.shape[0]
    grid = tau.shape[:-3]
    f = np.zeros((dim,) + grid)
    for a, o in enumerate(offsets(dim)):
        # contribution of element e to its node a:  sum_q sum_j B tau
        contrib = np.einsum("...qij,qj->...i", tau, B[:, a, :])
        for i in range(dim):
            f[i] += _unshift(contrib[..., i], o)
    return f


def wave_angles(grid):
    """theta_m = 2 pi k_m / N_m on the full DFT grid, as arrays in [z,y,x] layout.

    Returns a list (theta_x, theta_y[, theta_z]) of broadcastable arrays.
    """
    dim = len(grid)
    thetas = []
    for m in range(dim):
        n = grid[dim - 1 - m]
        k = np.arange(n)
        shape = [1] * dim
        shape[dim - 1 - m] = n
        thetas.append((2.0 * np.pi * k / n).reshape(shape))
    return thetas


def fourier_symbol(grid, element):
    """Dhat[..., q, j](k) = sum_a B[q, a, j] exp(+i theta . o_a).

    With the unscaled forward DFT xhat(k) = sum_x x(x) exp(-i theta . x), this
    is the multiplier of the gradient: DFT((D u)_{q,j}) = Dhat_{qj} * DFT(u).
    """
    B = shape_gradients(element)
    dim = element_dim(element)
    nq = B.shape[0]
    thetas = wave_angles(grid)
    Dh = np.zeros(tuple(grid) + (nq, dim), dtype=np.complex128)
    for a, o in enumerate(offsets(dim)):
        phase = np.ones(tuple(grid), dtype=np.complex128)
        for m in range(dim):
            if o[m]:
                phase = phase * np.exp(1j * thetas[m])
        Dh += phase[..., None, None] * B[:, a, :]
    return Dh


def all_points(grid):
    """Iterate over integer grid positions in (x, y[, z]) order (tests only)."""
    ranges = [range(n) for n in grid[::-1]]
    return itertools.product(*ranges)
