"""Discrete Fourier transform on a periodic voxel grid.

Fields live on voxel centres of the periodic cell Y = [0, Lx) x [0, Ly) x [0, Lz)
and are stored as arrays (..., nz, ny, nx) with x fastest. The transform is

    f^(k) = sum_x f(x) exp(-2 pi i sum_j k_j x_j / n_j),

its inverse carries 1 / (nx ny nz). The frequency of index k_j is
xi_j = 2 pi k_j / L_j with k_j in {-floor(n_j/2), ..., ceil(n_j/2) - 1}
(Moulinec-Suquet trigonometric collocation, cited in Sec. 5.4).

Nyquist reading (the paper is silent): for even n_j, the index k_j = -n_j/2
gets xi_j := 0. Operators built from the direction n = xi / |xi| then stay
orthogonal projectors and map real fields to real fields.
"""
import numpy as np
import scipy.fft

# threads of the library FFT (scipy's pocketfft, the same transform as
# numpy.fft); the CPU baseline sets it to the host's core count
WORKERS = 1


def integer_frequencies(n):
    """Signed integer frequency of each FFT index along an axis of n points."""
    idx = np.arange(n)
    k = np.where(idx < (n + 1) // 2, idx, idx - n)
    return k


def frequency_vectors(shape_zyx, lengths_xyz=(1.0, 1.0, 1.0)):
    """xi = (xi_x, xi_y, xi_z), each of shape (nz, ny, nx), Nyquist entries zeroed."""
    nz, ny, nx = shape_zyx
    out = []
    for n, L, axis in ((nx, lengths_xyz[0], 2), (ny, lengths_xyz[1], 1), (nz, lengths_xyz[2], 0)):
        k = integer_frequencies(n).astype(np.float64)
        if n % 2 == 0:
            k[n // 2] = 0.0          # Nyquist reading
        xi = 2.0 * np.pi * k / L
        shape = [1, 1, 1]
        shape[axis] = n
        out.append(np.broadcast_to(xi.reshape(shape), (nz, ny, nx)))
    return np.stack(out)


def directions(shape_zyx, lengths_xyz=(1.0, 1.0, 1.0)):
    """Unit directions n = xi / |xi| (3, nz, ny, nx); zero where xi = 0."""
    xi = frequency_vectors(shape_zyx, lengths_xyz)
    mag = np.sqrt((xi * xi).sum(axis=0))
    safe = np.where(mag > 0.0, mag, 1.0)
    return np.where(mag > 0.0, xi / safe, 0.0)


def dft_direct(f):
    """Direct triple sum of the forward transform over the last three axes.
    O(n^6): tiny grids only."""
    f = np.asarray(f, dtype=np.complex128)
    nz, ny, nx = f.shape[-3:]
    out = np.zeros_like(f)
    z = np.arange(nz)
    y = np.arange(ny)
    x = np.arange(nx)
    for kz in range(nz):
        ez = np.exp(-2j * np.pi * kz * z / nz)
        for ky in range(ny):
            ey = np.exp(-2j * np.pi * ky * y / ny)
            for kx in range(nx):
                ex = np.exp(-2j * np.pi * kx * x / nx)
                w = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
                out[..., kz, ky, kx] = (f * w).sum(axis=(-3, -2, -1))
    return out


def fft3(f):
    """Forward transform over the last three axes (library FFT)."""
    return scipy.fft.fftn(f, axes=(-3, -2, -1), workers=WORKERS)


def ifft3(F):
    """Inverse transform over the last three axes, real part (input Hermitian)."""
    return scipy.fft.ifftn(F, axes=(-3, -2, -1), workers=WORKERS).real


def rotated_wavevectors(shape_zyx, lengths_xyz=(1.0, 1.0, 1.0)):
    """Modified wave vectors of the rotated finite-difference scheme (Willot's
    discretization, the paper's "staggered grid" citation in Sec. 5.2):
    with theta_j = 2 pi k_j / n_j and h_j = L_j / n_j,

        k_j = (exp(i theta_j) - 1) / h_j * prod_{l != j} (1 + exp(i theta_l)) / 2,

    the Fourier symbol of the difference along j of a corner displacement,
    averaged over the 4 cell edges parallel to j. Complex (3, nz, ny, nx)."""
    nz, ny, nx = shape_zyx
    e = []
    h = []
    for n, L, axis in ((nx, lengths_xyz[0], 2), (ny, lengths_xyz[1], 1), (nz, lengths_xyz[2], 0)):
        shape = [1, 1, 1]
        shape[axis] = n
        e.append(np.exp(2j * np.pi * np.arange(n) / n).reshape(shape))
        h.append(L / n)
    k = []
    for j in range(3):
        term = (e[j] - 1.0) / h[j]
        for l in range(3):
            if l != j:
                term = term * (1.0 + e[l]) / 2.0
        k.append(np.broadcast_to(term, (nz, ny, nx)))
    return np.stack(k)


def rotated_directions(shape_zyx, lengths_xyz=(1.0, 1.0, 1.0)):
    """Complex unit vectors n = k / |k| of the rotated scheme (|k|^2 = sum_j
    |k_j|^2); zero where k = 0: the mean, and the modes with k_j = 0 for every
    j (a Nyquist index on two axes), which the scheme cannot see. "Zero" means
    |k| below 1e-12 of the largest possible |k|, sqrt(sum_j (2 / h_j)^2)."""
    nz, ny, nx = shape_zyx
    k = rotated_wavevectors(shape_zyx, lengths_xyz)
    mag = np.sqrt((np.abs(k) ** 2).sum(axis=0))
    kmax = np.sqrt(sum((2.0 * n / L) ** 2 for n, L in zip((nx, ny, nz), lengths_xyz)))
    safe = np.where(mag > 1e-300, mag, 1.0)
    return np.where(mag > 1e-12 * kmax, k / safe, 0.0)
