"""Pins of the oracle's damage law (stress, consistent tangent, stored energy).

The law is the isotropic energy-norm damage of the benchmark workloads; its
tangent is the Hessian of eq. graient_and_hessian and its stress the gradient.
Pins: central finite differences (stress -> tangent, energy -> stress), the
textbook isotropic elastic responses (uniaxial stress, plane strain), and the
defining property of linear softening: the equivalent stress E (1-d) kappa
falls on a straight line from (kappa0, E kappa0) to (kappaf, 0).
"""
import numpy as np
import pytest

from oracle import material

MATS = [{"kind": "damage", "E": 1.0, "nu": 0.3, "kappa0": 1e-3, "kappaf": 5e-3},
        {"kind": "elastic", "E": 10.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}]


def _field(phase_val, dim, npts=6):
    shape = (npts,) * 1 + (1,) * (dim - 1)
    return material.MaterialField(np.full(shape, phase_val, dtype=np.uint8), MATS, 1)


@pytest.mark.parametrize("dim", [2, 3])
def test_uniaxial_and_plane_strain_elastic(dim):
    mf = _field(1, dim)
    E, nu, e = 10.0, 0.3, 1e-4
    H = np.zeros(mf.grid + (1, dim, dim))
    if dim == 3:
        # uniaxial stress: eps = diag(e, -nu e, -nu e) -> sigma = diag(E e, 0, 0)
        H[..., 0, 0, 0] = e
        H[..., 0, 1, 1] = -nu * e
        H[..., 0, 2, 2] = -nu * e
        st = material.evaluate(mf, H, mf.initial_history())
        ref = np.zeros((3, 3))
        ref[0, 0] = E * e
        np.testing.assert_allclose(st["sigma"][0, 0, 0, 0], ref, atol=1e-18)
    else:
        # plane strain uniaxial strain: sigma_xx = E(1-nu)/((1+nu)(1-2nu)) e,
        # sigma_yy = sigma_zz = E nu/((1+nu)(1-2nu)) e
        H[..., 0, 0, 0] = e
        st = material.evaluate(mf, H, mf.initial_history())
        c = E / ((1 + nu) * (1 - 2 * nu))
        np.testing.assert_allclose(st["sigma"][0, 0, 0, 0, 0], c * (1 - nu) * e, rtol=1e-14)
        np.testing.assert_allclose(st["sigma"][0, 0, 0, 1, 1], c * nu * e, rtol=1e-14)
        np.testing.assert_allclose(st["sigma_zz"][0, 0, 0], c * nu * e, rtol=1e-14)
    # shear: sigma_xy = 2 mu eps_xy, mu = E / (2 (1 + nu))
    H2 = np.zeros_like(H)
    H2[..., 0, 0, 1] = 2e-4                  # eps_xy = 1e-4, skew part ignored
    st = material.evaluate(mf, H2, mf.initial_history())
    mu = E / (2 * (1 + nu))
    np.testing.assert_allclose(st["sigma"][(0,) * dim + (0, 0, 1)], 2 * mu * 1e-4, rtol=1e-14)


def test_linear_softening_line():
    # homogeneous uniaxial-stress-like states of the damage phase: the
    # equivalent stress sigma_eq = E (1 - d) kappa is linear between kappa0
    # and kappaf, and d is clamped to [0, 1]
    k0, kf, E = 1e-3, 5e-3, 1.0
    kap = np.array([0.5e-3, 1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 7e-3])
    d = material.damage_of_kappa(kap, k0, kf)
    seq = E * (1 - d) * kap
    line = np.where(kap <= k0, E * kap, np.maximum(E * k0 * (kf - kap) / (kf - k0), 0.0))
    np.testing.assert_allclose(seq, line, rtol=1e-13, atol=1e-18)
    assert d[0] == 0.0 and d[1] == 0.0 and d[-2] == 1.0 and d[-1] == 1.0


def _random_state(dim, scale, rng, npts=5):
    mf = material.MaterialField(np.zeros((npts,) * dim, dtype=np.uint8), MATS, 2)
    H = scale * rng.normal(size=mf.grid + (2, dim, dim))
    return mf, H


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("regime", ["elastic", "softening", "unloading", "stiff"])
def test_tangent_is_derivative_of_stress(dim, regime):
    rng = np.random.default_rng(10 + dim)
    if regime == "stiff":
        mf = material.MaterialField(np.ones((4,) * dim, dtype=np.uint8), MATS, 2)
        H = 1e-3 * rng.normal(size=mf.grid + (2, dim, dim))
        kh = mf.initial_history()
    else:
        scale = {"elastic": 2e-4, "softening": 2.0e-3, "unloading": 2.0e-3}[regime]
        mf, H = _random_state(dim, scale, rng)
        kh = mf.initial_history()
        if regime == "unloading":
            st0 = material.evaluate(mf, H, kh)
            kh = 1.5 * st0["kappa_t"]          # every point below its history
    st = material.evaluate(mf, H, kh)
    if regime == "softening":
        assert np.mean(st["cprime"] > 0) > 0.5
    V = rng.normal(size=H.shape) * np.abs(H).max()
    h = 1e-6
    sp = material.evaluate(mf, H + h * V, kh)["sigma"]
    sm = material.evaluate(mf, H - h * V, kh)["sigma"]
    fd = (sp - sm) / (2 * h)
    an = material.apply_tangent(mf, st, V)
    err = np.max(np.abs(fd - an)) / np.max(np.abs(an))
    assert err < 1e-6, err
    # the tangent is symmetric: <W, B V> = <V, B W>
    W = rng.normal(size=H.shape)
    a = np.sum(W * material.apply_tangent(mf, st, V))
    b = np.sum(V * material.apply_tangent(mf, st, W))
    assert abs(a - b) <= 1e-12 * max(abs(a), 1e-30)


@pytest.mark.parametrize("dim", [2, 3])
def test_stress_is_derivative_of_energy(dim):
    rng = np.random.default_rng(20 + dim)
    mf, H = _random_state(dim, 2e-3, rng)
    kh = mf.initial_history()
    st = material.evaluate(mf, H, kh)
    V = rng.normal(size=H.shape) * 1e-3
    h = 1e-5
    fd = (material.energy(mf, H + h * V, kh) - material.energy(mf, H - h * V, kh)) / (2 * h)
    an = np.sum(st["sigma"] * V)
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_history_commit_is_monotone():
    rng = np.random.default_rng(5)
    mf, H = _random_state(3, 2e-3, rng)
    kh = mf.initial_history()
    st = material.evaluate(mf, H, kh)
    kh2 = material.committed_history(mf, st, kh)
    assert np.all(kh2 >= kh)
    st2 = material.evaluate(mf, 0.1 * H, kh2)      # unloading keeps damage
    np.testing.assert_allclose(st2["d"], st["d"], rtol=0, atol=1e-15)
    assert not np.any(st2["loading"])
