"""DST-I diagonalisation of the lattice Laplacian and the C^T A C solve (FP64 oracle).

Sec. 3.2.1 (eqs. (30)-(31)): C^T C = S Lambda S^T with S the type-I discrete sine
transform, and C^T A C = C^T C (I + alpha C^T C).  With A = I/dt - L/2 (Sec. 2.2) the
solve used by the predictor (eq. (16)) and the corrector (eq. (20)) is

    (C^T A C)^{-1} r = dt * S2 diag(1 / (lam (1 + alpha lam))) S2 r,

S2 = S (x) S the 2-D transform.  The oracle applies S as a dense orthonormal
matrix (naive O(n^3) products, no FFT).
"""
import numpy as np


def sine_matrix(n):
    """Orthonormal DST-I of size n-1: S[j-1, k-1] = sqrt(2/n) sin(pi j k / n)."""
    j = np.arange(1, n)
    return np.sqrt(2.0 / n) * np.sin(np.pi * np.outer(j, j) / n)


def eigenvalues_1d(n):
    k = np.arange(1, n)
    return 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2


def eigenvalues(n):
    """lam[l-1, k-1] = 4 sin^2(pi k / 2n) + 4 sin^2(pi l / 2n): eigenvalues of C^T C."""
    lam = eigenvalues_1d(n)
    return lam[:, None] + lam[None, :]


def dst2(x):
    """2-D orthonormal DST-I of an (n-1, n-1) array (self-inverse)."""
    s = sine_matrix(x.shape[0] + 1)
    return s @ x @ s


def solve_cac(rhs, alpha):
    """[C^T C (I + alpha C^T C)]^{-1} rhs with homogeneous Dirichlet values.

    Multiply by dt for (C^T A C)^{-1}.
    """
    n = rhs.shape[0] + 1
    s = sine_matrix(n)
    lam = eigenvalues(n)
    return s @ ((s @ rhs @ s) / (lam * (1.0 + alpha * lam))) @ s


def solve_poisson(rhs):
    """(C^T C)^{-1} rhs with homogeneous Dirichlet values."""
    n = rhs.shape[0] + 1
    s = sine_matrix(n)
    return s @ ((s @ rhs @ s) / eigenvalues(n)) @ s
