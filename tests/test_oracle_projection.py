"""Pins of the oracle's compatibility projector (Sec. 2.1, eq. projection,
eq. conv_to_fourier, eq. proj_operator with ghat(0) = 0).

The projector must be the orthogonal projection onto the compatible fields
(gradients of periodic displacements): checked against a dense
D pinv(D^T D) D^T built from explicitly assembled D, and through its
defining properties.
"""
import numpy as np
import pytest

from oracle import fe
from oracle.projection import Projector
from tests.test_oracle_fe import _dense_gradient_matrix

CASES = [("q1", (2, 3, 2)), ("p1pair", (3, 4)), ("p1pair", (4, 4))]


def _shape(grid, element):
    dim = fe.element_dim(element)
    nq = fe.shape_gradients(element).shape[0]
    return tuple(grid) + (nq, dim, dim)


@pytest.mark.parametrize("element,grid", CASES)
def test_projector_equals_dense_pinv(element, grid):
    D = _dense_gradient_matrix(grid, element)
    Gd = D @ np.linalg.pinv(D.T @ D) @ D.T
    P = Projector(grid, element)
    shp = _shape(grid, element)
    n = int(np.prod(shp))
    cols = []
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        cols.append(P(e.reshape(shp)).reshape(-1))
    Gf = np.stack(cols, axis=1)
    np.testing.assert_allclose(Gf, Gd, rtol=0, atol=1e-12)
    # eigenvalues of an orthogonal projector are 0 or 1
    ev = np.linalg.eigvalsh(0.5 * (Gf + Gf.T))
    assert np.all(np.minimum(np.abs(ev), np.abs(ev - 1.0)) < 1e-10)


@pytest.mark.parametrize("element,grid", [("q1", (4, 6, 5)), ("p1pair", (8, 6))])
def test_projector_properties(element, grid):
    P = Projector(grid, element)
    dim = fe.element_dim(element)
    rng = np.random.default_rng(4)
    shp = _shape(grid, element)
    X = rng.normal(size=shp)
    Y = rng.normal(size=shp)
    GX = P(X)
    # idempotent
    np.testing.assert_allclose(P(GX), GX, rtol=0, atol=1e-12)
    # self-adjoint
    assert abs(np.sum(P(X) * Y) - np.sum(X * P(Y))) < 1e-10
    # reproduces gradients of periodic fields
    u = rng.normal(size=(dim,) + tuple(grid))
    Du = fe.gradient(u, element)
    np.testing.assert_allclose(P(Du), Du, rtol=0, atol=1e-12)
    # annihilates constants (ghat(0) = 0): a uniform macroscopic strain is not
    # a fluctuation
    C = np.broadcast_to(rng.normal(size=(dim, dim)), shp).copy()
    np.testing.assert_allclose(P(C), 0.0, atol=1e-12)
    # the compatible part has zero mean
    assert np.max(np.abs(GX.mean(axis=tuple(range(dim))))) < 1e-13
