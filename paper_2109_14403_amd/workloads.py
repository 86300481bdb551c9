"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module holds inputs only: material parameter tables, phase-id voxel
images and macroscopic load histories. It contains none of the solver's or
the constitutive laws' arithmetic; derived moduli (bulk/shear moduli,
relaxation times, shift factors, ...) are computed separately by each
consumer.

Conventions
-----------
* Voxel images are ``uint8`` arrays of shape ``(nz, ny, nx)`` (x fastest),
  holding a phase id per voxel.
* Strain tensors are given by their components in the order
  (11, 22, 33, 23, 13, 12), tensorial shear (not engineering shear).
* Units: MPa, s, K, m. Heat capacities in MPa/K (1 MPa/K = 1e6 J/(m^3 K)),
  conductivities in W/(m K), temperature gradients in K/m.

Material tables follow the paper's Table "Material parameters of the E-glass
fibers" (Sec. 4) and Table "Material parameters of the PA66" (Sec. 4). The
paper never states the stress-free reference temperature of the free energy;
293.15 K (the initial temperature of its virtual experiments, Sec. 5.4) is
used for the paper's materials.

Random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# material tables (inputs)
# --------------------------------------------------------------------------

THERMOELASTIC = "thermoelastic"
PA66 = "pa66"


def e_glass(theta0: float = 293.15) -> dict:
    """E-glass fibre parameters (paper Sec. 4, E-glass table)."""
    return dict(kind=THERMOELASTIC, E=72.0e3, nu=0.26, c0=2.1, alpha0=9.0e-6,
                kappa0=0.93, theta0=theta0)


def pa66(theta0: float = 293.15) -> dict:
    """PA66 matrix parameters (paper Sec. 4, PA66 table), N = 12 Maxwell branches."""
    return dict(
        kind=PA66, E=1.5e3, nu=0.42, c0=1.9, alpha0=70.0e-6, kappa0=0.27, theta0=theta0,
        E_i=[265.0, 262.0, 248.0, 231.0, 211.0, 190.0, 170.0, 92.0, 78.0, 65.0, 54.0, 48.0],
        log10_tau_i=[-4.22, -3.42, -2.63, -1.84, -1.05, -0.26, 0.53, 1.32, 2.12, 2.91, 3.70, 4.49],
        C1=26.21, C2=446.31, theta_ref=298.15,
        sigma_y0=15.5, k_h=103.0, n_h=0.32, eta0=74.0, m=2.0,
        beta1=0.011, beta2=0.07,
    )


def small_sphere_matrix() -> dict:
    """Linear thermoelastic matrix of the 16^3 centred-sphere workload."""
    return dict(kind=THERMOELASTIC, E=3.0e3, nu=0.35, c0=1.9, alpha0=6.0e-5,
                kappa0=0.2, theta0=293.0)


def small_sphere_inclusion() -> dict:
    """Linear thermoelastic inclusion of the 16^3 centred-sphere workload."""
    return dict(kind=THERMOELASTIC, E=70.0e3, nu=0.22, c0=2.1, alpha0=5.0e-6,
                kappa0=1.0, theta0=293.0)


# --------------------------------------------------------------------------
# voxel images
# --------------------------------------------------------------------------

def _centres(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) + 0.5


def centred_sphere(n: int = 16, radius: float = 5.8) -> np.ndarray:
    """Phase 1 where the voxel centre lies within ``radius`` of the cell centre."""
    c = _centres(n) - n / 2.0
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return ((x * x + y * y + z * z) <= radius * radius).astype(np.uint8)


def laminate(n: tuple[int, int, int], layer_bounds: list[int], axis: int = 0) -> np.ndarray:
    """Layered image: phase alternates 0/1 at the given voxel indices along ``axis``
    (0 = x, 1 = y, 2 = z). ``layer_bounds`` are the starting indices of phase-1 runs
    and phase-0 runs alternately, e.g. [4, 12] -> phase 1 on [4, 12)."""
    nx, ny, nz = n
    size = (nx, ny, nz)[axis]
    prof = np.zeros(size, dtype=np.uint8)
    b = list(layer_bounds) + [size]
    for j in range(0, len(layer_bounds), 2):
        prof[b[j]:b[j + 1]] = 1
    img = np.zeros((nz, ny, nx), dtype=np.uint8)
    if axis == 0:
        img[:] = prof[None, None, :]
    elif axis == 1:
        img[:] = prof[None, :, None]
    else:
        img[:] = prof[:, None, None]
    return img


def _periodic_ball(img: np.ndarray, centre: np.ndarray, radius: float) -> None:
    nz, ny, nx = img.shape
    lo = np.floor(centre - radius - 1).astype(int)
    hi = np.ceil(centre + radius + 1).astype(int)
    zs = np.arange(lo[2], hi[2] + 1)
    ys = np.arange(lo[1], hi[1] + 1)
    xs = np.arange(lo[0], hi[0] + 1)
    dz = (zs + 0.5 - centre[2])[:, None, None]
    dy = (ys + 0.5 - centre[1])[None, :, None]
    dx = (xs + 0.5 - centre[0])[None, None, :]
    inside = (dx * dx + dy * dy + dz * dz) <= radius * radius
    iz, iy, ix = np.nonzero(inside)
    img[zs[iz] % nz, ys[iy] % ny, xs[ix] % nx] = 1


def rsa_spheres(n: int, seed: int, radius_range: tuple[float, float],
                target_fraction: float, gap: float = 0.0, max_attempts: int = 200000,
                fixed_radius: float | None = None) -> tuple[np.ndarray, dict]:
    """Random sequential addition of non-overlapping spheres in a periodic cube.

    Centres uniform in [0, n)^3, radii uniform in ``radius_range`` (or fixed),
    minimum-image distance between centres >= r1 + r2 + gap. Spheres are added
    until the voxel fraction of phase 1 reaches ``target_fraction``.
    Returns the image and a record (achieved fraction, count, jammed flag).
    """
    rng = np.random.default_rng(seed)
    img = np.zeros((n, n, n), dtype=np.uint8)
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    attempts = 0
    frac = 0.0
    while frac < target_fraction and attempts < max_attempts:
        attempts += 1
        c = rng.uniform(0.0, n, size=3)
        r = fixed_radius if fixed_radius is not None else rng.uniform(*radius_range)
        if len(radii):
            d = centres - c
            d -= n * np.round(d / n)
            dist = np.sqrt((d * d).sum(axis=1))
            if np.any(dist < radii + r + gap):
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        _periodic_ball(img, c, r)
        frac = img.mean()
    rec = dict(fraction=float(frac), count=int(len(radii)), attempts=attempts,
               jammed=bool(frac < target_fraction))
    return img, rec


def _cylinder_columns(cx, cy, u, direction, length, radius, n):
    """Voxel columns of a cylinder lying in the x-y plane, axis through
    (cx, cy, z0 + u) along ``direction``: returns (xs, ys, lo, hi) so that voxel
    (x, y, z0 + dz) is inside for lo <= dz <= hi (voxel centres at +0.5)."""
    half = 0.5 * length
    ext = np.abs(direction[:2]) * half + radius + 1.0
    xs = np.arange(int(np.floor(cx - ext[0])), int(np.ceil(cx + ext[0])) + 1)
    ys = np.arange(int(np.floor(cy - ext[1])), int(np.ceil(cy + ext[1])) + 1)
    X, Y = np.meshgrid(xs + 0.5 - cx, ys + 0.5 - cy, indexing="xy")
    along = X * direction[0] + Y * direction[1]
    perp2 = (X - along * direction[0]) ** 2 + (Y - along * direction[1]) ** 2
    ok = (np.abs(along) <= half) & (perp2 <= radius * radius)
    # remaining z half-extent for voxel centres dz + 0.5 - u
    hz = np.sqrt(np.maximum(radius * radius - perp2, 0.0))
    lo = np.ceil(u - 0.5 - hz).astype(int)
    hi = np.floor(u - 0.5 + hz).astype(int)
    ok &= hi >= lo
    iy, ix = np.nonzero(ok)
    return (xs[ix] % n), (ys[iy] % n), lo[iy, ix], hi[iy, ix]


def rsa_fibres(n: int, seed: int, diameter: float, length: float,
               target_fraction: float, max_attempts: int = 200000) -> tuple[np.ndarray, dict]:
    """Random sequential addition of straight, non-overlapping cylinders in a
    periodic cube.

    Each candidate draws an axis angle phi ~ U[0, pi) in the x-y plane
    (planar isotropic orientation) and a centre (x, y) ~ U[0, n)^2 plus a
    sub-voxel z offset; among all z levels where its voxels are free it takes
    one uniformly at random (a candidate with no free level is rejected).
    Fibres never share voxels. Candidates are added until the voxel fraction
    reaches ``target_fraction``; the record says whether the sequence jammed.
    """
    rng = np.random.default_rng(seed)
    occ = np.zeros((n, n, n), dtype=bool)        # [y, x, z]: z contiguous per column
    radius = 0.5 * diameter
    attempts = 0
    count = 0
    filled = 0
    target = target_fraction * n ** 3
    while filled < target and attempts < max_attempts:
        attempts += 1
        phi = rng.uniform(0.0, math.pi)
        d = np.array([math.cos(phi), math.sin(phi), 0.0])
        cx, cy, u = rng.uniform(0.0, n), rng.uniform(0.0, n), rng.uniform(0.0, 1.0)
        xs, ys, lo, hi = _cylinder_columns(cx, cy, u, d, length, radius, n)
        cols = occ[ys, xs]                                   # (ncol, n)
        # blocked[z0]: some column j is occupied at z0 + dz for lo_j <= dz <= hi_j
        blocked = np.zeros(n, dtype=bool)
        for a, b in set(zip(lo.tolist(), hi.tolist())):
            v = cols[(lo == a) & (hi == b)].any(axis=0)
            for dz in range(a, b + 1):
                blocked |= np.roll(v, -dz)
        free = np.nonzero(~blocked)[0]
        if free.size == 0:
            continue
        z0 = int(free[rng.integers(free.size)])
        for dz in range(int(lo.min()), int(hi.max()) + 1):
            sel = (lo <= dz) & (dz <= hi)
            occ[ys[sel], xs[sel], (z0 + dz) % n] = True
            filled += int(sel.sum())
        count += 1
    img = np.ascontiguousarray(occ.transpose(2, 0, 1)).astype(np.uint8)
    frac = float(img.mean())
    rec = dict(fraction=frac, count=count, attempts=attempts, jammed=bool(frac < target_fraction))
    return img, rec

# --------------------------------------------------------------------------
# load histories
# --------------------------------------------------------------------------

@dataclass
class LoadStep:
    strain: np.ndarray          # (6,) components (11,22,33,23,13,12)
    theta: float                # K
    grad: np.ndarray            # (3,) K/m
    dt: float                   # s


def _tensor(e11=0.0, e22=0.0, e33=0.0, e23=0.0, e13=0.0, e12=0.0) -> np.ndarray:
    return np.array([e11, e22, e33, e23, e13, e12], dtype=np.float64)


def history_small_sphere(n_steps: int = 10) -> list[LoadStep]:
    """Uniaxial macro strain to 1 % in 10 steps with a 293 -> 393 K ramp."""
    return [LoadStep(_tensor(e11=0.001 * k), 293.0 + 10.0 * k, np.array([1.0, 0.0, 0.0]), 2.0)
            for k in range(1, n_steps + 1)]


def history_shear_tension(n_steps: int = 20) -> list[LoadStep]:
    """Mixed tension/shear to 2 % under a cyclic 293.15-373.15 K temperature."""
    out = []
    for k in range(1, n_steps + 1):
        s = k / 20.0
        out.append(LoadStep(_tensor(e11=0.02 * s, e12=0.01 * s),
                            333.15 - 40.0 * math.cos(2.0 * math.pi * k / 10.0),
                            np.array([1.0, 0.0, 0.0]), 2.0))
    return out


def history_fibre_tension(n_steps: int = 50) -> list[LoadStep]:
    """Uniaxial e1 extension to 2 % with a 293.15 -> 333.15 K ramp, dt = 0.8 s."""
    return [LoadStep(_tensor(e11=0.02 * k / 50.0), 293.15 + 40.0 * k / 50.0,
                     np.array([1.0, 0.0, 0.0]), 0.8) for k in range(1, n_steps + 1)]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    phases: np.ndarray
    laws: list
    history: list
    record: dict = field(default_factory=dict)


def small_sphere_workload() -> Workload:
    """16^3 centred sphere (840 voxels, c = 0.2051), linear thermoelastic phases."""
    img = centred_sphere(16, 5.8)
    return Workload("sphere16_thermoelastic", img,
                    [small_sphere_matrix(), small_sphere_inclusion()],
                    history_small_sphere(), dict(fraction=float(img.mean())))


def sphere_composite_workload(n: int = 64, seed: int = 2) -> Workload:
    """RSA spheres (radius 4-6 voxels at n = 64, scaled with n) at >= 25 %,
    PA66 matrix and E-glass inclusions."""
    scale = n / 64.0
    img, rec = rsa_spheres(n, seed, (4.0 * scale, 6.0 * scale), 0.25)
    return Workload(f"spheres{n}_pa66_glass", img, [pa66(), e_glass()],
                    history_shear_tension(), rec)


def fibre_composite_workload(n: int = 256, seed: int = 3) -> Workload:
    """Planar-isotropic short fibres (diameter 6, aspect ratio 20 at n = 256,
    scaled with n) at >= 20 %, PA66 matrix and E-glass fibres."""
    scale = n / 256.0
    img, rec = rsa_fibres(n, seed, 6.0 * scale, 120.0 * scale, 0.20)
    return Workload(f"fibres{n}_pa66_glass", img, [pa66(), e_glass()],
                    history_fibre_tension(), rec)


def batch_problem(index: int, seed: int = 4, sizes=(24, 32, 48), n_steps: int = 5):
    """One microproblem of the batched workload: grid size drawn from ``sizes``,
    RSA spheres with fraction ~ U[0.10, 0.30] and radius (n/8) U[0.8, 1.2], and a
    random proportional strain/temperature history of ``n_steps`` increments."""
    rng = np.random.default_rng([seed, index])
    n = int(sizes[rng.integers(len(sizes))])
    frac = rng.uniform(0.10, 0.30)
    radius = (n / 8.0) * rng.uniform(0.8, 1.2)
    img, rec = rsa_spheres(n, int(rng.integers(2**31)), (radius, radius), frac)
    direction = rng.normal(size=6)
    direction /= np.linalg.norm(direction)
    amp = rng.uniform(0.0, 0.015)
    # direction is uniform on the unit sphere of normalized Mandel vectors
    sq2 = math.sqrt(2.0)
    e_full = amp * np.array([direction[0], direction[1], direction[2],
                             direction[3] / sq2, direction[4] / sq2, direction[5] / sq2])
    d_theta = rng.uniform(0.0, 80.0)
    dt = math.exp(rng.uniform(math.log(0.006), math.log(6.0)))
    grad = rng.normal(size=3)
    hist = [LoadStep(e_full * k / n_steps, 293.15 + d_theta * k / n_steps, grad.copy(), dt)
            for k in range(1, n_steps + 1)]
    rec.update(n=n, target=frac, radius=radius)
    return Workload(f"batch{index}_n{n}", img, [pa66(), e_glass()], hist, rec)


# --------------------------------------------------------------------------
# surrogate workload: one fixed microstructure, many Gauss-point histories
# --------------------------------------------------------------------------
SQ2 = math.sqrt(2.0)
_MANDEL_W = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


def surrogate_microstructure(n: int = 32, seed: int = 5):
    """The fixed n^3 RSA sphere microstructure of the surrogate (radius n/8,
    fraction >= 0.20; PA66 matrix id 0, E-glass spheres id 1)."""
    return rsa_spheres(n, seed, (n / 8.0, n / 8.0), 0.20)


def surrogate_histories(count: int, seed: int, steps: int = 5) -> dict:
    """Proportional strain / temperature histories of the batch recipe: strain
    direction uniform on the unit 6-sphere (Mandel) times U[0, 0.015],
    Delta T ~ U[0, 80] K, dt ~ logU[0.006, 6] s per history, grad theta
    ~ N(0, 1) K/m per history. Returns strain [count, steps, 6] (components),
    theta [count, steps], dt [count], grad [count, 3]."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(count, 6))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    amp = rng.uniform(0.0, 0.015, size=count)
    e_full = amp[:, None] * d / _MANDEL_W[None, :]
    dT = rng.uniform(0.0, 80.0, size=count)
    dt = np.exp(rng.uniform(math.log(0.006), math.log(6.0), size=count))
    grad = rng.normal(size=(count, 3))
    k = np.arange(1, steps + 1) / steps
    strain = e_full[:, None, :] * k[None, :, None]
    theta = 293.15 + dT[:, None] * k[None, :]
    return dict(strain=strain, theta=theta, dt=dt, grad=grad)
