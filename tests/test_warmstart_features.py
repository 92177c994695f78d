"""Host-side input features of the scaled learned warm start (no GPU)."""
import numpy as np

from paper_2207_10657_amd.warmstart import features_full, strain_channels


def test_strain_channels_of_simple_fields():
    """A constant displacement gives the macroscopic strain E. A field
    u_x(x) gives at every element centre the difference of u_x across the
    element in xx, and nothing in the other channels."""
    rng = np.random.default_rng(1)
    n = (4, 5, 6)                                    # nz, ny, nx
    E = rng.normal(size=(3, 3))
    E = 0.5 * (E + E.T)
    u = np.ones((3,) + n) * rng.normal(size=(3, 1, 1, 1))
    S = strain_channels(u, E)
    for k, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))):
        assert np.allclose(S[k], E[i, j], atol=1e-15)
    x = np.arange(n[2])
    ux = np.sin(2 * np.pi * x / n[2])
    u = np.zeros((3,) + n)
    u[0] = ux[None, None, :]
    S = strain_channels(u, np.zeros((3, 3)))
    ref = np.roll(ux, -1) - ux
    assert np.allclose(S[0], ref[None, None, :], atol=1e-15)
    assert np.abs(S[1:]).max() < 1e-15


def test_full_features_layout():
    rng = np.random.default_rng(2)
    n = (4, 4, 4)
    phase = (rng.random(n) < 0.3).astype(np.uint8)
    damage = rng.random(n + (8,)) * 0.5
    du = rng.normal(size=(3,) + n)
    u = rng.normal(size=(3,) + n)
    E = np.diag([1e-3, 0.0, 0.0])
    dE = np.diag([2e-4, 0.0, 0.0])
    f = features_full(phase, damage, du, 0.5, u, E, dE)
    assert f.shape == (18,) + n and f.dtype == np.float32
    assert np.array_equal(f[0], (phase == 0).astype(np.float32))
    assert np.allclose(f[12], 1.0) and np.allclose(f[13:18], 0.0)
