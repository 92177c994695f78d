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


# ---- tensile-masking law (Appendix A) ------------------------------------

TMATS = [{"kind": "tensile", "E": 1.0, "nu": 0.25, "kappa0": 1e-3,
          "kappaf": material.kappa_alpha(1e-3, 0.25)},
         {"kind": "elastic", "E": 10.0, "nu": 0.3, "kappa0": 0.0, "kappaf": 0.0}]


def _rotation(rng):
    Q, R = np.linalg.qr(rng.normal(size=(3, 3)))
    return Q * np.sign(np.diag(R))


def test_tensile_part_of_diagonal_and_rotated_strains():
    # diag(3, -1, 2) e-3: the tensile part keeps the positive entries; a
    # rotation of the strain rotates its tensile part, kappa is invariant
    rng = np.random.default_rng(31)
    eps = np.diag([3e-3, -1e-3, 2e-3])
    et = material.tensile_part(eps)
    np.testing.assert_allclose(et, np.diag([3e-3, 0.0, 2e-3]), atol=1e-18)
    for _ in range(4):
        Q = _rotation(rng)
        etr = material.tensile_part(Q @ eps @ Q.T)
        np.testing.assert_allclose(etr, Q @ et @ Q.T, atol=1e-17)
        assert abs(np.linalg.norm(etr) - np.sqrt(13.0) * 1e-3) < 1e-17


@pytest.mark.parametrize("dim", [2, 3])
def test_tensile_part_is_the_projection_on_the_psd_cone(dim):
    # the positive part P of a symmetric eps is the nearest positive
    # semidefinite matrix: P >= 0, P - eps >= 0 and P (P - eps) = 0
    rng = np.random.default_rng(32 + dim)
    for _ in range(20):
        A = rng.normal(size=(dim, dim))
        eps = 1e-3 * (A + A.T)
        P = material.tensile_part(eps)
        tol = 1e-14 * np.linalg.norm(eps)
        assert np.linalg.eigvalsh(P).min() > -tol
        assert np.linalg.eigvalsh(P - eps).min() > -tol
        np.testing.assert_allclose(P @ (P - eps), 0.0, atol=1e-19)
        np.testing.assert_allclose(P, P.T, atol=0)


def test_alpha_form_of_the_damage_variable():
    # D = (kappa - k0)(1 + alpha)/kappa, clamped to [0, 1], for the kf the
    # tensile phase is given
    k0, alpha = 1e-3, 0.25
    kf = material.kappa_alpha(k0, alpha)
    kap = np.array([0.5e-3, 1e-3, 1.5e-3, 3e-3, 4.9e-3, kf, 7e-3])
    D = np.clip((kap - k0) * (1 + alpha) / kap, 0.0, 1.0)
    np.testing.assert_allclose(material.damage_of_kappa(kap, k0, kf), D, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("dim", [2, 3])
def test_tensile_law_uniaxial_and_compression(dim):
    mf = material.MaterialField(np.zeros((4,) + (1,) * (dim - 1), dtype=np.uint8), TMATS, 1)
    kh = mf.initial_history()
    H = np.zeros(mf.grid + (1, dim, dim))
    e = 2.5e-3
    H[..., 0, 0, 0] = e
    H[..., 0, 1, 1] = -0.25 * e
    if dim == 3:
        H[..., 0, 2, 2] = -0.25 * e
    st = material.evaluate(mf, H, kh)
    # one positive principal strain: kappa = e, d = d(e)
    np.testing.assert_allclose(st["kappa_t"], e, rtol=1e-15)
    np.testing.assert_allclose(st["d"], (e - 1e-3) * 1.25 / e, rtol=1e-13)
    # any compression (negative definite strain) leaves the phase elastic
    rng = np.random.default_rng(41)
    A = rng.normal(size=mf.grid + (1, dim, dim))
    Hc = -5e-2 * (np.einsum("...ik,...jk->...ij", A, A) + 0.1 * np.eye(dim))
    stc = material.evaluate(mf, Hc, kh)
    assert np.all(stc["kappa_t"] == 0.0) and np.all(stc["d"] == 0.0)
    assert not np.any(stc["loading"])
    lam, mu = material.lame(1.0, 0.25)
    ref = lam * np.trace(Hc, axis1=-2, axis2=-1)[..., None, None] * np.eye(dim) + 2 * mu * Hc
    np.testing.assert_allclose(stc["sigma"], ref, rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("regime", ["softening", "unloading"])
def test_tensile_tangent_is_derivative_of_stress(dim, regime):
    rng = np.random.default_rng(50 + dim)
    mf = material.MaterialField(np.zeros((5,) * dim, dtype=np.uint8), TMATS, 2)
    A = rng.normal(size=mf.grid + (2, dim, dim))
    # strains with principal values of both signs, mostly past the threshold
    H = 1.5e-3 * A + 1e-3 * np.eye(dim)
    kh = mf.initial_history()
    if regime == "unloading":
        kh = 1.5 * material.evaluate(mf, H, kh)["kappa_t"] + 1e-3
    st = material.evaluate(mf, H, kh)
    if regime == "softening":
        assert np.mean(st["cprime"] > 0) > 0.5
        assert np.mean(np.any(np.linalg.eigvalsh(st["eps"]) < 0, axis=-1)) > 0.3
    else:
        assert not np.any(st["cprime"] > 0)
    V = rng.normal(size=H.shape) * np.abs(H).max()
    h = 1e-7
    sp = material.evaluate(mf, H + h * V, kh)["sigma"]
    sm = material.evaluate(mf, H - h * V, kh)["sigma"]
    fd = (sp - sm) / (2 * h)
    an = material.apply_tangent(mf, st, V)
    err = np.max(np.abs(fd - an)) / np.max(np.abs(an))
    assert err < 1e-6, err
    if regime == "softening":
        # the rank-one update couples C:eps with eps_t: not symmetric
        W = rng.normal(size=H.shape)
        a = np.sum(W * material.apply_tangent(mf, st, V))
        b = np.sum(V * material.apply_tangent(mf, st, W))
        assert abs(a - b) > 1e-6 * abs(a)


def test_tensile_law_has_no_energy():
    mf = material.MaterialField(np.zeros((2, 2, 2), dtype=np.uint8), TMATS, 1)
    with pytest.raises(ValueError):
        material.energy(mf, np.zeros(mf.grid + (1, 3, 3)), mf.initial_history())
