"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on the same FP32-rounded inputs with the same parameters."""
import numpy as np

from oracle import esp_grid
from oracle.pswf import c_from_tol


def paper_params(h, tol, coupling="iso", rc=0.9, sigma=1.07):
    """Analytic parameters computed on the oracle side (Sec. 5.1 rule and the
    grid rule), passed to the library as explicit parameters."""
    delta = tol / 5 if coupling == "flex" else tol
    c = c_from_tol(delta)
    P = int(np.ceil(-np.log10(delta) - 1e-9)) + 1

    def smooth(m):
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        return m == 1
    M = []
    for d in range(3):
        m = max(int(np.ceil(sigma * np.linalg.norm(h[:, d]) * c / (np.pi * rc) - 1e-9)), P)
        while not smooth(m):
            m += 1
        M.append(m)
    return dict(c_split=c, c_spread=c, P=P, M=tuple(M), rc=rc)


def as_inputs(r, q, precision):
    dt = np.float32 if precision == "fp32" else np.float64
    r = np.ascontiguousarray(r, dtype=dt)
    q = np.ascontiguousarray(q, dtype=dt)
    return r, q, r.astype(np.float64), q.astype(np.float64)


def oracle(h, r64, q64, prm, forces=True):
    return esp_grid.esp_grid(h, r64, q64, esp_grid.GridParams(prm["c_split"], prm["c_spread"], prm["P"],
                                                              tuple(prm["M"]), prm["rc"]), forces=forces)


def w6(W):
    return np.array([W[0, 0], W[1, 1], W[2, 2], W[0, 1], W[0, 2], W[1, 2]])


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def tensor_rel(out7, W):
    """Relative error of the six virial components (Frobenius norm of the
    symmetric tensor, off-diagonals counted twice)."""
    ref = w6(W)
    wt = np.array([1, 1, 1, 2, 2, 2.0])
    return float(np.sqrt(np.sum(wt * (out7[1:] - ref) ** 2) / np.sum(wt * ref ** 2)))


# Parity bars.  FP32: the stated bound for pressure and RMS force (1e-5
# relative).  FP64: the same kernels in double precision; the bar allows for
# the polynomial window fit (relative error <= 1e-3 Delta) and the Chebyshev
# kernel fit (1e-13).
TOL = {"fp32": 1e-5, "fp64": 1e-9}
