"""Compatibility projector G of the FE-projection scheme (oracle).

Sec. 2.1: G maps any field of second-order tensors at the quadrature points to
its compatible part (eq. projection); it is block diagonal in the wave vector
(eq. conv_to_fourier) and built from the derivative operator Dhat as
ghat = Dhat (x) Dhat^* / (Dhat . Dhat^*) (eq. proj_operator), zero at k = 0.

Reading of the small-strain form (the paper defers it to cited work): G acts
on the full displacement gradient, G_{ijkl} = delta_ik ghat_jl, where the
"derivative" index j runs over (quadrature point, direction) pairs. Applied to
a field X[..., q, i, j] this is, per wave vector k and displacement component i,

    (G X)hat_{i,(q,j)} = Dhat_{qj} * sum_{q',l} conj(Dhat_{q'l}) Xhat_{i,(q',l)}
                         / sum_{q',l} |Dhat_{q'l}|^2 .

Pinned by: a dense D pinv(D^T D) D^T on tiny grids, idempotence, self-adjointness,
exact reproduction of gradients, annihilation of constants
(``tests/test_oracle_projection.py``).
"""
import numpy as np

from . import fe


class Projector:
    def __init__(self, grid, element):
        self.grid = tuple(grid)
        self.element = element
        self.dim = fe.element_dim(element)
        self.Dh = fe.fourier_symbol(self.grid, element)          # (*grid, nq, d)
        self.S = np.sum(np.abs(self.Dh) ** 2, axis=(-2, -1))      # (*grid,)
        # the derivative of a constant vanishes: k = 0 is the only zero mode,
        # and the projector is defined as 0 there (ghat(0) = 0)
        self.zero = np.zeros(self.S.shape, dtype=bool)
        self.zero.flat[0] = True
        if np.min(self.S[~self.zero], initial=np.inf) <= 1e-12:
            raise ValueError("derivative symbol vanishes away from k = 0")
        self.invS = np.where(self.zero, 0.0, 1.0 / np.where(self.zero, 1.0, self.S))
        self.axes = tuple(range(self.dim))

    def __call__(self, X):
        """G X for X of shape (*grid, nq, d, d); returns the same shape."""
        Xh = np.fft.fftn(X, axes=self.axes)
        # t_i(k) = sum_{q,j} conj(Dhat_{qj}) Xhat_{q,i,j}
        t = np.einsum("...qj,...qij->...i", np.conj(self.Dh), Xh)
        t *= self.invS[..., None]
        Yh = np.einsum("...qj,...i->...qij", self.Dh, t)
        Y = np.fft.ifftn(Yh, axes=self.axes)
        return Y.real
