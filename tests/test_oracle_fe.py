"""Pins of the oracle's finite-element operators (Sec. 2.1: the derivative
operator of a linear FE discretisation evaluated at quadrature points).

Each check rests on something other than the oracle's own formulas:
linear-field exactness of the shape functions, an element-by-element dense
assembly written with explicit loops, the adjoint identity, a naive O(N^2)
DFT, and the textbook Fourier symbols of the FE Laplacian.
"""
import itertools

import numpy as np
import pytest

from oracle import fe

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.mark.parametrize("element", ["q1", "p1pair"])
def test_shape_gradients_reproduce_linear_fields(element):
    # u(x) = A x sampled at the element's corner nodes must give grad u = A at
    # every quadrature point (linear completeness of Q1 and P1 elements).
    dim = fe.element_dim(element)
    B = fe.shape_gradients(element)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(dim, dim))
    offs = fe.offsets(dim)
    for q in range(B.shape[0]):
        H = np.zeros((dim, dim))
        for a, o in enumerate(offs):
            H += np.outer(A @ np.array(o, float), B[q, a])
        np.testing.assert_allclose(H, A, rtol=0, atol=1e-14)
    # constants have zero gradient
    np.testing.assert_allclose(B.sum(axis=1), 0.0, atol=1e-15)


def test_q1_gauss_points_and_p1_areas():
    # Q1: the derivative along x at a Gauss point is the y,z interpolation of
    # the x-differences with weights 1/2 -+ 1/(2 sqrt 3).
    B = fe.shape_gradients("q1")
    g0 = 0.5 - 0.5 / np.sqrt(3.0)
    # qp 0 = (g0,g0,g0); node 1 = (1,0,0): dN/dx = (1-g0)^2
    assert abs(B[0, 1, 0] - (1 - g0) ** 2) < 1e-15
    # P1 pair: each triangle has area 1/2, gradient of the corner-(0,0) hat in
    # T1 is (-1,-1)
    Bp = fe.shape_gradients("p1pair")
    np.testing.assert_allclose(Bp[0, 0], (-1.0, -1.0))


def _dense_gradient_matrix(grid, element):
    """Dense matrix of u -> (D u) assembled with explicit loops over elements.

    Written independently of fe.gradient: nodal index and element index are
    computed here from integer coordinates.
    """
    dim = fe.element_dim(element)
    B = fe.shape_gradients(element)
    nq = B.shape[0]
    shape = tuple(grid)               # [z,y,x] / [y,x]
    n = int(np.prod(shape))
    nxyz = shape[::-1]

    def lin(c):                       # c in (x, y[, z]) order, periodic
        idx = 0
        for m in reversed(range(dim)):
            idx = idx * nxyz[m] + (c[m] % nxyz[m])
        return idx

    M = np.zeros((n * nq * dim * dim, dim * n))
    for e in itertools.product(*[range(s) for s in nxyz]):
        ei = lin(e)
        for q in range(nq):
            for a, o in enumerate(fe.offsets(dim)):
                node = lin(tuple(e[m] + o[m] for m in range(dim)))
                for i in range(dim):
                    for j in range(dim):
                        row = ((ei * nq + q) * dim + i) * dim + j
                        M[row, i * n + node] += B[q, a, j]
    return M


@pytest.mark.parametrize("element,grid", [("q1", (3, 2, 4)), ("p1pair", (3, 5))])
def test_gradient_matches_dense_assembly(element, grid):
    dim = fe.element_dim(element)
    rng = np.random.default_rng(1)
    u = rng.normal(size=(dim,) + grid)
    M = _dense_gradient_matrix(grid, element)
    H = fe.gradient(u, element)
    np.testing.assert_allclose(H.reshape(-1), M @ u.reshape(-1), rtol=0, atol=1e-13)


@pytest.mark.parametrize("element,grid", [("q1", (4, 3, 5)), ("p1pair", (6, 4))])
def test_divergence_is_adjoint(element, grid):
    dim = fe.element_dim(element)
    nq = fe.shape_gradients(element).shape[0]
    rng = np.random.default_rng(2)
    u = rng.normal(size=(dim,) + grid)
    tau = rng.normal(size=grid + (nq, dim, dim))
    lhs = np.sum(fe.gradient(u, element) * tau)
    rhs = np.sum(u * fe.divergence(tau, element))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _naive_dft(f, axes_shape):
    """O(N^2) DFT over the leading grid axes, unscaled, e^{-i theta.x}."""
    grid = axes_shape
    dim = len(grid)
    out = np.zeros(f.shape, dtype=np.complex128)
    pts = list(itertools.product(*[range(s) for s in grid]))
    for k in pts:
        acc = 0.0
        for x in pts:
            ph = sum(2.0 * np.pi * k[m] * x[m] / grid[m] for m in range(dim))
            acc = acc + f[x] * np.exp(-1j * ph)
        out[k] = acc
    return out


@pytest.mark.parametrize("element,grid", [("q1", (2, 3, 4)), ("p1pair", (3, 4))])
def test_fourier_symbol_against_naive_dft(element, grid):
    # DFT((D u)_{q,i,j})(k) = Dhat_{q j}(k) * DFT(u_i)(k)
    dim = fe.element_dim(element)
    rng = np.random.default_rng(3)
    u = rng.normal(size=(dim,) + grid)
    H = fe.gradient(u, element)
    Hh = _naive_dft(H, grid)
    uh = np.stack([_naive_dft(u[i], grid) for i in range(dim)], axis=0)
    Dh = fe.fourier_symbol(grid, element)
    pred = np.einsum("...qj,i...->...qij", Dh, uh)
    np.testing.assert_allclose(Hh, pred, rtol=0, atol=1e-12)


def test_green_symbol_closed_forms():
    # Sum over points and directions of |Dhat|^2 is the Fourier symbol of the
    # FE stiffness of the Laplacian (unweighted sum = nq x the integral):
    # Q1: 8 sum_j (2 - 2 cos t_j) prod_{m != j} (2 + cos t_m)/3 (1D stiffness
    # times 1D consistent mass), P1 split: 2 sum_j (2 - 2 cos t_j) (5-point).
    for grid in [(4, 5, 6), (7, 3, 8)]:
        Dh = fe.fourier_symbol(grid, "q1")
        S = np.sum(np.abs(Dh) ** 2, axis=(-2, -1))
        th = fe.wave_angles(grid)
        ref = 0.0
        for j in range(3):
            t = 2.0 - 2.0 * np.cos(th[j])
            for m in range(3):
                if m != j:
                    t = t * (2.0 + np.cos(th[m])) / 3.0
            ref = ref + t
        np.testing.assert_allclose(S, 8.0 * ref, rtol=1e-13, atol=1e-14)
    for grid in [(5, 7), (8, 8)]:
        Dh = fe.fourier_symbol(grid, "p1pair")
        S = np.sum(np.abs(Dh) ** 2, axis=(-2, -1))
        th = fe.wave_angles(grid)
        ref = 2.0 * sum(2.0 - 2.0 * np.cos(t) for t in th)
        np.testing.assert_allclose(S, ref + 0.0 * S, rtol=1e-13, atol=1e-14)
