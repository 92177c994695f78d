"""Periodic 1D damage-spring system of Sec. 3.1 (oracle, test infrastructure).

Three nodes on a ring joined by springs k1 (node 0 to 1), k2 (1 to 2) and the
damage spring k0 (2 back to 0 across the period). Springs k1 = k2 = k are
elastic; k0 follows k until the elongation reaches gamma_0 and then softens
with tangent alpha k (eq. K_mat). Reading of the figure-only parts: the
softening branch ends where the force reaches zero (a fully broken spring
carries no force), and a mean stretch x_bar per spring is prescribed.

In the paper's strain-space setting the unknowns are the three elongations
gamma = x_bar + fluctuation, the fluctuation has zero sum (it is the
difference of periodic nodal displacements), so the compatibility projector
is G = I - 1 1^T / 3, the "stress" is the spring force vector and the tangent
is diagonal. The same Steihaug and FAIEF trust-region steps as the cell
solver are applied. The true energy is known here, so the standard ratio of
eq. rho can be used as well (the paper's comparison of Sec. 3.1).

Pinned by: the eigenvalues [0, 3k, (2 alpha + 1) k] of eq. K_mat, and a
brute-force scan of the energy over the two free degrees of freedom
(``tests/test_oracle_solver.py``).
"""
import math
import numpy as np

from .solver import steihaug, faief_ratio, tr_update, BOUNDARY, NEGCURV


class SpringRing:
    def __init__(self, k=1.0, gamma0=0.1, alpha=-1.0, x_bar=0.11):
        self.k, self.g0, self.alpha, self.x_bar = k, gamma0, alpha, x_bar
        # end of the softening branch (zero force), infinite for alpha >= 0
        self.g_end = gamma0 - gamma0 / alpha if alpha < 0.0 else math.inf

    # -- damage spring k0 (loading only, as in one monotonic solve) --------
    def _f0(self, g):
        k, g0, a = self.k, self.g0, self.alpha
        if g <= g0:
            return k * g
        if g >= self.g_end:
            return 0.0
        return k * g0 + a * k * (g - g0)

    def _t0(self, g):
        if g <= self.g0:
            return self.k
        if g >= self.g_end:
            return 0.0
        return self.alpha * self.k

    def _w0(self, g):
        k, g0, a = self.k, self.g0, self.alpha
        if g <= g0:
            return 0.5 * k * g * g
        ge = min(g, self.g_end)
        w = 0.5 * k * g0 * g0 + k * g0 * (ge - g0) + 0.5 * a * k * (ge - g0) ** 2
        return w

    # -- strain-space quantities --------------------------------------------
    def stress(self, gam):
        """Spring forces (k gamma_1, k gamma_2, f_0(gamma_0)) as an array."""
        return np.array([self.k * gam[0], self.k * gam[1], self._f0(gam[2])])

    def tangent(self, gam):
        return np.array([self.k, self.k, self._t0(gam[2])])

    def energy(self, gam):
        return 0.5 * self.k * (gam[0] ** 2 + gam[1] ** 2) + self._w0(gam[2])

    @staticmethod
    def project(v):
        """G v = v - mean(v): zero-sum (compatible) part."""
        return v - np.mean(v)

    def nodal_stiffness(self, gam):
        """Stiffness in nodal displacements (u0, u1, u2) (eq. K_mat form)."""
        k1 = k2 = self.k
        k0 = self._t0(gam[2])
        # spring 1: u1 - u0, spring 2: u2 - u1, spring 0: u0 - u2
        K = np.zeros((3, 3))
        for (i, j, kk) in ((0, 1, k1), (1, 2, k2), (2, 0, k0)):
            K[i, i] += kk
            K[j, j] += kk
            K[i, j] -= kk
            K[j, i] -= kk
        return K

    def solve(self, R0=0.01, Rmax=1.0, eta=1e-10, eta_up=0.15, i_max=200,
              standard=False):
        """Trust-region Newton with the FAIEF ratio (or the true-energy ratio).

        Returns (gamma, info). ``standard=True`` uses eq. rho with the exact
        energy instead of eq. rho_bar.
        """
        gam = np.full(3, self.x_bar)
        R = R0
        info = {"iters": 0, "accepted": 0, "rejected": 0, "path": [gam.copy()]}
        for it in range(i_max):
            sig = self.stress(gam)
            g = self.project(sig)
            if math.sqrt(float(g @ g)) <= eta:
                break
            tan = self.tangent(gam)

            def A(v):
                return self.project(tan * self.project(v))

            p, flag, _ = steihaug(A, g, R, 1e-12, 50)
            info["iters"] = it + 1
            sp = float(sig @ p)
            pBp = float(p @ (tan * p))
            sig_t = self.stress(gam + p)
            dm, dW, rho = faief_ratio(sp, pBp, float(sig_t @ p))
            if standard:
                dW_true = self.energy(gam + p) - self.energy(gam)
                rho = dW_true / dm if dm < 0.0 else -math.inf
            on_b = flag in (BOUNDARY, NEGCURV)
            R = tr_update(rho, R, Rmax, on_b)
            if rho > eta_up:
                gam = gam + p
                info["accepted"] += 1
                info["path"].append(gam.copy())
            else:
                info["rejected"] += 1
        return gam, info
