"""Isotropic damage laws at the quadrature points (oracle).

Two damage laws share the bilinear softening d(kappa) and the frozen history
kappa_hist of a load step:

    sigma = (1 - d) C : eps,      eps = sym(H),
    d(kappa) = kf/kappa * (kappa - k0)/(kf - k0), clamped to [0, 1],

with C isotropic (Lame constants from E, nu; plane strain in 2D, eps_zz = 0).
They differ in the equivalent strain kappa_t:

* kind 'damage' (the energy norm of the benchmark workloads):
  kappa_t = sqrt(eps : C : eps / E);
* kind 'tensile' (the tensile-masking law of Appendix A): kappa_t = |eps_t|,
  the Frobenius norm of the tensile part eps_t = M eps M, where the masking
  matrix M = sum_i H(e_i) q_i (x) q_i keeps the eigenvectors q_i of eps with
  positive eigenvalues e_i (eqs. strain_measure,
  stress_contributions_maksing_matrices, Mask_matrices_t); so
  eps_t = sum_i max(e_i, 0) q_i (x) q_i. The appendix writes the damage as
  D = (kappa - k0)(1 + alpha)/kappa (eq. our_model_damage_variable), alpha
  the relative softening slope: the same d(kappa) with kf = k0 (1 + alpha)/alpha.

A phase may carry an eigenstrain eps_eig, added to the strain before the law
is evaluated (Algorithm 2: eps_eval = eps + eps_eig), so eps above is
sym(H) + eps_eig. A point is loading iff kappa_t > kappa_hist (strict); then
d = d(kappa_t), else d = d(kappa_hist).

The paper's Newton linearisation (eq. project_stress_linear) and energy
Hessian (eq. graient_and_hessian) use the consistent tangent, a rank-one
update of the secant stiffness:

    dsigma = a C : sym(dH) - c' (n : dH) s,    s = C : eps, a = 1 - d,

while loading with 0 < d < 1 (else c' = 0), where d kappa_t / d eps = n c'/d'
with d' = d d/d kappa at kappa_t:

* energy norm: n = s, c' = d'(kappa_t) / (E kappa_t) (symmetric tangent);
* tensile masking: n = eps_t, c' = d'(kappa_t) / kappa_t. The derivative of
  kappa_t^2 = sum_i max(e_i, 0)^2 needs only the eigenvalue derivatives
  d e_i / d eps = q_i (x) q_i, so it is 2 eps_t: no eigenvector derivative
  and no division by eigenvalue gaps enter (the singularity that the
  appendix removes with the masking matrix). The tangent is not symmetric,
  and the law has no stored energy.

The exact stored energy of the energy-norm law for a frozen history (used
only to pin the FAIEF estimate of eq. incr_energy_func) is w = F(kappa_t)
while loading, else F(kappa_hist) + (1 - d(kappa_hist)) E (kappa_t^2 -
kappa_hist^2) / 2, with F(kappa) = int_0^kappa E k (1 - d(k)) dk.

Pinned by: central finite differences of the stress (tangent) and of the
energy (stress), the small-strain elastic limit, uniaxial-stress compliance,
and for the tensile law the closed forms of diagonal strains, rotation
invariance, the absence of damage under compression and the alpha form of
the damage variable (``tests/test_oracle_material.py``).
"""
import numpy as np


def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def damage_of_kappa(kappa, k0, kf):
    """d(kappa) clamped to [0, 1]; kappa must be > 0 where k0 > 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        d = kf / kappa * (kappa - k0) / (kf - k0)
    return np.clip(np.nan_to_num(d, nan=0.0), 0.0, 1.0)


class MaterialField:
    """Per-quadrature-point material parameters from a phase map.

    ``phase`` has the grid shape, ``materials[p]`` is a dict with keys kind
    ('elastic' | 'damage' | 'tensile'), E, nu, kappa0, kappaf. Arrays have
    shape (*grid, nq).
    """

    def __init__(self, phase, materials, nq):
        phase = np.asarray(phase)
        self.grid = phase.shape
        self.nq = nq
        self.dim = phase.ndim

        def per_qp(key, conv=float):
            table = np.array([conv(m[key]) for m in materials])
            return np.repeat(table[phase][..., None], nq, axis=-1)

        self.E = per_qp("E")
        nu = per_qp("nu")
        self.lam, self.mu = lame(self.E, nu)
        self.damage = per_qp("kind", conv=lambda k: 1.0 if k in ("damage", "tensile")
                             else 0.0) > 0.5
        self.tensile = per_qp("kind", conv=lambda k: 1.0 if k == "tensile" else 0.0) > 0.5
        self.k0 = np.where(self.damage, per_qp("kappa0"), 0.0)
        self.kf = np.where(self.damage, per_qp("kappaf"), 1.0)
        self.phase = phase
        self.eig_table = np.zeros((len(materials), self.dim, self.dim))
        for p, m in enumerate(materials):
            if m.get("eig") is not None:
                self.set_eigenstrain(p, m["eig"])
        self._update_eig()

    def set_eigenstrain(self, p, eig):
        """Eigenstrain of phase p (3x3, symmetric; the in-plane block in 2D)."""
        e = np.asarray(eig, dtype=np.float64).reshape(3, 3)
        self.eig_table[p] = 0.5 * (e + e.T)[:self.dim, :self.dim]
        self._update_eig()

    def _update_eig(self):
        self.eig = np.repeat(self.eig_table[self.phase][..., None, :, :], self.nq, axis=-3)

    def initial_history(self):
        """kappa_hist := kappa0 on damage points (no damage yet), 0 elsewhere."""
        return np.where(self.damage, self.k0, 0.0)


def sym(H):
    return 0.5 * (H + np.swapaxes(H, -1, -2))


def _c_contract(mat, eps):
    """C : eps for the in-plane (2D) or full (3D) strain."""
    dim = eps.shape[-1]
    tr = np.trace(eps, axis1=-2, axis2=-1)
    return mat.lam[..., None, None] * tr[..., None, None] * np.eye(dim) \
        + 2.0 * mat.mu[..., None, None] * eps


def kappa_alpha(k0, alpha):
    """kf of the bilinear d(kappa) that equals the appendix's
    D = (kappa - k0)(1 + alpha)/kappa (eq. our_model_damage_variable)."""
    return k0 * (1.0 + alpha) / alpha


def tensile_part(eps):
    """eps_t = M eps M = sum_i max(e_i, 0) q_i (x) q_i over the eigenpairs of
    the symmetric eps (eqs. stress_contributions_maksing_matrices and
    Mask_matrices_t). In 2D the plane-strain eps_zz = 0 adds a zero
    eigenvalue, which has no tensile part."""
    e, Q = np.linalg.eigh(eps)
    return np.einsum("...ik,...k,...jk->...ij", Q, np.maximum(e, 0.0), Q)


def evaluate(mat, H, kappa_hist):
    """Stress and tangent data at the full-gradient field H (*grid, nq, d, d);
    the law sees eps = sym(H) + eps_eig."""
    eps = sym(H) + mat.eig
    s = _c_contract(mat, eps)
    ecs = np.sum(eps * s, axis=(-2, -1))
    k_energy = np.sqrt(np.maximum(ecs, 0.0) / mat.E)
    if np.any(mat.tensile):
        eps_t = tensile_part(eps)
        k_tens = np.sqrt(np.sum(eps_t * eps_t, axis=(-2, -1)))
        kappa_t = np.where(mat.tensile, k_tens, k_energy)
        n = np.where(mat.tensile[..., None, None], eps_t, s)
    else:
        kappa_t = k_energy
        n = s
    loading = mat.damage & (kappa_t > kappa_hist)
    kappa_eff = np.where(loading, kappa_t, kappa_hist)
    d = np.where(mat.damage, damage_of_kappa(np.where(mat.damage, kappa_eff, 1.0),
                                             mat.k0, mat.kf), 0.0)
    a = 1.0 - d
    softening = loading & (d > 0.0) & (d < 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        dprime = mat.kf * mat.k0 / ((mat.kf - mat.k0) * kappa_t ** 2)
        scale = np.where(mat.tensile, 1.0, mat.E)
        cprime = np.where(softening, dprime / (scale * kappa_t), 0.0)
    sigma = a[..., None, None] * s
    tr = np.trace(eps, axis1=-2, axis2=-1)
    sigma_zz = a * mat.lam * tr if H.shape[-1] == 2 else None
    return {"eps": eps, "s": s, "n": n, "sigma": sigma, "a": a, "cprime": cprime,
            "kappa_t": kappa_t, "loading": loading, "d": d, "sigma_zz": sigma_zz}


def apply_tangent(mat, state, dH):
    """dsigma = a C : sym(dH) - c' (n : dH) s at every quadrature point."""
    deps = sym(dH)
    out = state["a"][..., None, None] * _c_contract(mat, deps)
    nde = np.sum(state["n"] * deps, axis=(-2, -1))
    out -= (state["cprime"] * nde)[..., None, None] * state["s"]
    return out


def _F(mat, kappa):
    """int_0^kappa E k (1 - d(k)) dk for the damage law (elastic: E kappa^2/2)."""
    E, k0, kf = mat.E, mat.k0, mat.kf
    el = 0.5 * E * kappa ** 2
    k = np.minimum(kappa, kf)
    soft = 0.5 * E * k0 ** 2 + E * (0.5 * (k ** 2 - k0 ** 2)
                                    - kf / (kf - k0) * 0.5 * (k - k0) ** 2)
    dmg = np.where(kappa <= k0, el, soft)
    return np.where(mat.damage, dmg, el)


def energy(mat, H, kappa_hist):
    """Exact stored energy W = sum over points of w (frozen history); the
    energy-norm law only (the tensile law has no potential)."""
    if np.any(mat.tensile):
        raise ValueError("the tensile-masking law has no stored energy")
    st = evaluate(mat, H, kappa_hist)
    kt = st["kappa_t"]
    a_h = 1.0 - np.where(mat.damage,
                         damage_of_kappa(np.where(mat.damage, kappa_hist, 1.0),
                                         mat.k0, mat.kf), 0.0)
    unload = _F(mat, kappa_hist) + 0.5 * a_h * mat.E * (kt ** 2 - kappa_hist ** 2)
    w = np.where(mat.damage & ~(kt > kappa_hist), unload, _F(mat, kt))
    return float(np.sum(w))


def committed_history(mat, state, kappa_hist):
    """kappa_hist <- max(kappa_hist, kappa_t) on damage points."""
    return np.where(mat.damage, np.maximum(kappa_hist, state["kappa_t"]), kappa_hist)
