"""Order-zero prolate spheroidal wave function psi_0^c (paper, Appendix A.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper defines psi_0^c as the eigenfunction, for the eigenvalue of largest
modulus, of the operator  phi -> int_{-1}^{1} phi(t) exp(i c x t) dt  on
L^2[-1,1] (eq. psidefinit), normalised to unit L^2 norm.  The eigenvalues of
that operator cluster in modulus for large c, so the eigenvector is computed
from the classical Sturm-Liouville operator that commutes with it,

    L psi = -((1 - x^2) psi')' + c^2 x^2 psi ,

whose eigenvalues are well separated (the reference the paper cites for PSWF
properties, Osipov-Rokhlin-Xiao, uses this route).  psi_0 is even, so it is
expanded in normalised even Legendre polynomials  Pbar_n = sqrt(n+1/2) P_n,
which turns L into a symmetric tridiagonal matrix.  The result is pinned in
tests against the paper's own integral eigen-equation and against SciPy's
independent prolate routines.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.linalg import eigh_tridiagonal
from scipy.optimize import brentq


class PSWF:
    """psi_0^c for one bandwidth c, with the derived constants of Sec. 3.1.

    Attributes
    ----------
    c       bandwidth parameter.
    coef    Legendre-series coefficients (standard P_n basis) of psi on [-1,1].
    lam0    eigenvalue of eq. psidefinit (real, positive for n = 0).
    C0      int_0^1 psi(x) dx  (definition below eq. decomposition).
    psi0    psi(0).
    """

    def __init__(self, c: float, nterms: int | None = None):
        c = float(c)
        if c <= 0:
            raise ValueError("c must be positive")
        self.c = c
        K = nterms if nterms is not None else int(1.5 * c) + 40
        n = 2.0 * np.arange(K)                      # even degrees 0, 2, 4, ...
        diag = n * (n + 1) + c * c * (2 * n * (n + 1) - 1) / ((2 * n + 3) * (2 * n - 1))
        nn = n[:-1]
        off = c * c * (nn + 2) * (nn + 1) / ((2 * nn + 3) * np.sqrt((2 * nn + 1) * (2 * nn + 5)))
        _, vec = eigh_tridiagonal(diag, off, select="i", select_range=(0, 0))
        beta = vec[:, 0]
        # expand into the standard Legendre basis: Pbar_n = sqrt(n + 1/2) P_n
        coef = np.zeros(2 * K - 1)
        coef[0::2] = beta * np.sqrt(n + 0.5)
        if npleg.legval(0.0, coef) < 0:             # sign convention: psi(0) > 0
            coef = -coef
        self.coef = coef
        self.dcoef = npleg.legder(coef)
        self.icoef = npleg.legint(coef, lbnd=0.0)   # antiderivative, zero at 0
        self.psi0 = float(npleg.legval(0.0, coef))
        self.C0 = float(npleg.legval(1.0, self.icoef))
        # eigenvalue of eq. psidefinit as the Rayleigh quotient of the integral
        # operator (psi has unit L^2 norm), by Gauss-Legendre quadrature
        t, w = np.polynomial.legendre.leggauss(int(2 * c) + 80)
        pt = npleg.legval(t, coef)
        self.lam0 = float(np.einsum("i,ij,j->", w * pt, np.cos(c * np.outer(t, t)), w * pt))
        self._qt, self._qw, self._qpsi = t, w, pt

    # -- psi and its derivative on [-1, 1] (extension beyond, see psi_ext) ----
    def psi(self, x):
        """psi_0^c(x) for |x| <= 1 from the Legendre series."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self.coef)

    def dpsi(self, x):
        """d psi_0^c / dx for |x| <= 1."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self.dcoef)

    def int_psi(self, x):
        """int_0^x psi_0^c(t) dt for |x| <= 1."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self.icoef)

    def psi_ext(self, x):
        """psi_0^c(x) for any real x.

        Inside [-1, 1] this is the series.  Outside, psi is continued by the
        eigen-equation itself (eq. psidefinit), (1/lam0) int psi(t) cos(cxt) dt,
        which is also the exact Fourier transform of the compactly supported
        psi used in the window transform (eq. pswf_fourier) beyond its band.
        """
        x = np.asarray(x, dtype=np.float64)
        out = np.empty_like(x)
        inside = np.abs(x) <= 1.0
        out[inside] = self.psi(x[inside])
        xo = x[~inside]
        if xo.size:
            ph = np.cos(self.c * np.multiply.outer(xo, self._qt))
            out[~inside] = ph @ (self._qw * self._qpsi) / self.lam0
        return out

    def dpsi_ext(self, x):
        """d/dx of psi_ext (series inside, differentiated eigen-equation outside)."""
        x = np.asarray(x, dtype=np.float64)
        out = np.empty_like(x)
        inside = np.abs(x) <= 1.0
        out[inside] = self.dpsi(x[inside])
        xo = x[~inside]
        if xo.size:
            ph = -self.c * np.sin(self.c * np.multiply.outer(xo, self._qt)) * self._qt
            out[~inside] = ph @ (self._qw * self._qpsi) / self.lam0
        return out


@functools.lru_cache(maxsize=64)
def pswf(c: float) -> PSWF:
    """Cached PSWF object for bandwidth c."""
    return PSWF(float(c))


def c_from_tol(delta: float) -> float:
    """Bandwidth c such that psi_0^c(1) = Delta, read as psi(1)/psi(0) = Delta.

    Parameter rule of Sec. 5.1; the normalisation the rule is stated in is
    not given, and the ratio to psi(0) is the reading used throughout.
    """
    if not (1e-14 <= delta < 1.0):
        raise ValueError("Delta must lie in [1e-14, 1)")

    def f(c):
        p = PSWF(c)
        return np.log(float(p.psi(1.0)) / p.psi0) - np.log(delta)

    return float(brentq(f, 0.05, 36.0, xtol=1e-13, rtol=1e-14))
