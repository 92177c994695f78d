"""Projected Hessian in displacement coordinates on all host cores (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.1 relates the projection scheme to the FE problem: every compatible
field is the FE gradient D u of a nodal field u, and the projector of eq.
proj_operator is G = D (D^T D)^+ D^T. The projected Hessian of eq.
project_stress_linear applied to a compatible direction D d is therefore

    G : B : (D d) = D w,    w = L^+ (D^T B D d),    L = D^T D,

where L^+ is diagonal in Fourier space with the symbol 1 / S(k),
S(k) = sum_{q,j} |Dhat_qj(k)|^2 (the denominator of eq. proj_operator), set
to 0 at k = 0. S is written here in closed form, the textbook symbol of the
element's FE Laplacian (theta_j = 2 pi k_j / n_j):

    Q1, 2x2x2 Gauss points:  8 sum_j (2 - 2 cos theta_j) prod_{m != j} (2 + cos theta_m) / 3
    P1 pair of triangles:    2 sum_j (2 - 2 cos theta_j)

Three nodal FFTs replace the 9 nq point-component FFTs of projection.py, which
this module is validated against (tests/test_oracle_uspace.py).

The grid is split into slabs of element layers along its first axis (z in
3D, y in 2D), evaluated on a thread pool (numpy's array loops release the
GIL), with BLAS held to one thread meanwhile (its own thread pool is not safe
under concurrent callers); the nodal sums of the slabs are added in slab
order, so the result does not depend on the number of threads. FFTs run on scipy.fft with
`workers` threads. This is the oracle the CPU baseline times on every host
core.
"""
import os
from concurrent.futures import ThreadPoolExecutor

from threadpoolctl import threadpool_limits

import numpy as np
import scipy.fft as sfft

from . import fe, material


def laplacian_symbol(grid, element):
    """S(k) on the full DFT grid ([z, y, x] or [y, x] layout), closed form."""
    th = fe.wave_angles(grid)
    dim = len(grid)
    S = np.zeros(tuple(grid))
    if element == "q1":
        for j in range(dim):
            t = 2.0 - 2.0 * np.cos(th[j])
            for m in range(dim):
                if m != j:
                    t = t * (2.0 + np.cos(th[m])) / 3.0
            S = S + 8.0 * t
    elif element == "p1pair":
        for j in range(dim):
            S = S + 2.0 * (2.0 - 2.0 * np.cos(th[j]))
    else:
        raise ValueError(element)
    return S


class UOperator:
    """The projected Hessian at a fixed state (E, u, kappa_hist) in
    displacement coordinates: apply(d) = L^+ D^T B D d, so that
    D apply(d) = G : B : (D d)."""

    def __init__(self, phase, materials, element, E, u, kappa_hist, workers=None, slabs=None):
        self.phase = np.asarray(phase)
        self.grid = self.phase.shape
        self.element = element
        self.dim = fe.element_dim(element)
        self.nq = fe.shape_gradients(element).shape[0]
        self.workers = int(workers or os.cpu_count() or 1)
        n0 = self.grid[0]
        ns = max(1, min(int(slabs or self.workers), n0))
        cuts = np.linspace(0, n0, ns + 1).round().astype(int)
        self.slabs = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
        kh = np.asarray(kappa_hist)
        Em = np.asarray(E, dtype=np.float64)[:self.dim, :self.dim]
        self._mf = []
        self._st = []
        # one BLAS thread per slab: a threaded BLAS called from several
        # threads at once can return wrong products
        with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(self.workers) as pool:
            def evaluate(sl):
                z0, z1 = sl
                mf = material.MaterialField(self.phase[z0:z1], materials, self.nq)
                H = self._gradient(u, z0, z1) + Em
                return mf, material.evaluate(mf, H, kh[z0:z1])
            for mf, st in pool.map(evaluate, self.slabs):
                self._mf.append(mf)
                self._st.append(st)
        S = laplacian_symbol(self.grid, element)
        half = S[..., : self.grid[-1] // 2 + 1]
        inv = np.zeros_like(half)
        nz = half != 0.0
        inv[nz] = 1.0 / half[nz]
        inv.flat[0] = 0.0
        self._inv_half = inv
        self._axes = tuple(range(1, self.dim + 1))

    def _gradient(self, v, z0, z1):
        """D v at the element layers z0..z1-1 (their nodes z0..z1, wrapped)."""
        idx = np.arange(z0, z1 + 1) % self.grid[0]
        ext = np.take(v, idx, axis=1)
        return fe.gradient(ext, self.element)[: z1 - z0]

    def _divergence(self, tau):
        """D^T of the slab's point tensors: nodal sums at its node layers
        z0..z1 (the last one shared with the next slab). Element e adds
        sum_{q,j} B[q,a,j] tau_{q,ij}(e) to its corner node e + o_a."""
        pad = np.zeros((1,) + tau.shape[1:])
        t = np.concatenate([tau, pad], axis=0)
        B = fe.shape_gradients(self.element)
        C = np.tensordot(t, B, axes=([-3, -1], [0, 2]))        # (*slab, i, a)
        f = np.zeros((self.dim,) + t.shape[:-3])
        for a, o in enumerate(fe.offsets(self.dim)):
            for i in range(self.dim):
                f[i] += fe._unshift(C[..., i, a], o)
        return f

    def stiffness(self, d):
        """K d = D^T B D d."""
        d = np.asarray(d, dtype=np.float64)

        def slab(k):
            z0, z1 = self.slabs[k]
            tau = material.apply_tangent(self._mf[k], self._st[k], self._gradient(d, z0, z1))
            return self._divergence(tau)

        with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(self.workers) as pool:
            parts = list(pool.map(slab, range(len(self.slabs))))
        f = np.zeros_like(d)
        n0 = self.grid[0]
        for (z0, z1), fx in zip(self.slabs, parts):
            f[:, z0:z1] += fx[:, : z1 - z0]
            f[:, z1 % n0] += fx[:, z1 - z0]
        return f

    def green(self, f):
        """L^+ f (the k = 0 mode removed)."""
        fh = sfft.rfftn(f, axes=self._axes, workers=self.workers)
        fh *= self._inv_half[None]
        return sfft.irfftn(fh, s=self.grid, axes=self._axes, workers=self.workers)

    def apply(self, d):
        """w = L^+ K d; D w is the projected Hessian G : B : (D d)."""
        return self.green(self.stiffness(d))
