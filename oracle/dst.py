"""DST-I diagonalisation of the lattice Laplacian and the C^T A C solve (FP64 oracle).

Sec. 3.2.1 (eqs. (30)-(31)): C^T C = S Lambda S^T with S the type-I discrete sine
transform, and C^T A C = C^T C (I + alpha C^T C).  With A = I/dt - L/2 (Sec. 2.2) the
solve used by the predictor (eq. (16)) and the corrector (eq. (20)) is

    (C^T A C)^{-1} r = dt * S2 diag(1 / (lam (1 + alpha lam))) S2 r,

S2 = S_y (x) S_x the 2-D transform (one sine matrix per axis; the same one on square
levels), lam = lam_x + lam_y.  In double precision the oracle applies S as a dense
orthonormal matrix (naive O(n^3) products, no FFT).

Extended precision (arrays of ``numpy.longdouble``, the x87 80-bit format with a 64-bit
significand): every function here follows the dtype of its input.  The products with S are
then done by a library primitive, the orthonormal type-I DST of ``scipy.fft`` (pocketfft,
which computes in the input's precision), because a dense long-double product of size
1023 takes about 12 s; it is pinned against the dense long-double S.
"""
import numpy as np
import scipy.fft


PI_TEXT = "3.14159265358979323846264338327950288419716939937510"


def _pi(dtype):
    return np.pi if dtype == np.float64 else np.asarray(PI_TEXT, dtype=np.longdouble).astype(dtype)[()]


def sine_matrix(n, dtype=np.float64):
    """Orthonormal DST-I of size n-1: S[j-1, k-1] = sqrt(2/n) sin(pi j k / n).

    The integer j k is first reduced modulo 2n (sin has period 2 pi), so that the rounding
    of pi is not multiplied by j k / n, up to n, in the angle."""
    j = np.arange(1, n)
    two = np.asarray(2, dtype=dtype)
    m = np.outer(j, j) % (2 * n)
    return np.sqrt(two / n) * np.sin(_pi(dtype) * m.astype(dtype) / n)


def eigenvalues_1d(n, dtype=np.float64):
    k = np.arange(1, n).astype(dtype)
    return 4 * np.sin(_pi(dtype) * k / (2 * n)) ** 2


def eigenvalues(n, dtype=np.float64, ny=None):
    """lam[l-1, k-1] = 4 sin^2(pi k / 2n) + 4 sin^2(pi l / 2 ny): eigenvalues of C^T C on a
    level of n cells along x and ny (default n) along y; rows are the y modes."""
    ny = n if ny is None else ny
    return eigenvalues_1d(ny, dtype)[:, None] + eigenvalues_1d(n, dtype)[None, :]


def dst2(x):
    """2-D orthonormal DST-I of an (ny-1, nx-1) array (self-inverse): S_y x S_x."""
    if x.dtype != np.float64:
        return scipy.fft.dst(scipy.fft.dst(x, type=1, norm="ortho", axis=0), type=1, norm="ortho",
                             axis=1)
    return sine_matrix(x.shape[0] + 1) @ x @ sine_matrix(x.shape[1] + 1)


def solve_cac(rhs, alpha):
    """[C^T C (I + alpha C^T C)]^{-1} rhs with homogeneous Dirichlet values.

    Multiply by dt for (C^T A C)^{-1}.
    """
    ny, nx = rhs.shape[0] + 1, rhs.shape[1] + 1
    lam = eigenvalues(nx, rhs.dtype, ny)
    if rhs.dtype != np.float64:
        return dst2(dst2(rhs) / (lam * (1 + alpha * lam)))
    sy, sx = sine_matrix(ny), sine_matrix(nx)
    return sy @ ((sy @ rhs @ sx) / (lam * (1.0 + alpha * lam))) @ sx


def solve_poisson(rhs):
    """(C^T C)^{-1} rhs with homogeneous Dirichlet values."""
    ny, nx = rhs.shape[0] + 1, rhs.shape[1] + 1
    if rhs.dtype != np.float64:
        return dst2(dst2(rhs) / eigenvalues(nx, rhs.dtype, ny))
    sy, sx = sine_matrix(ny), sine_matrix(nx)
    return sy @ ((sy @ rhs @ sx) / eigenvalues(nx, np.float64, ny)) @ sx
