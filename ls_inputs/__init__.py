"""Seeded synthetic inputs for the two-level Lippmann-Schwinger solver.

This module only draws inputs: media m(x) sampled on the grid, incident plane
waves u_I sampled on the grid, and random complex vectors.  It holds none of
the solver's arithmetic, so both the CPU oracle and the GPU path (and their
tests and the benchmark) can use it without sharing any method code.

Grid convention (Section 2 of the paper): collocation points
x_{i,j} = (h*i, h*j) for 1 <= i, j <= n.  Arrays are stored 0-based as
a[j, i] with the x index fastest (the row-by-row global ordering of
Section 3.2), so a[j, i] is the sample at (h*(i+1), h*(j+1)).

The paper's media (its Fig. 3 and the plasma profile) are pictures only; the
generators below are synthetic stand-ins with the same character (smooth,
compactly supported or decaying perturbations of contrast ~0.1-0.3).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid_coords",
    "gaussian_disk_medium",
    "gaussian_bumps_medium",
    "gaussian_random_field_medium",
    "smooth_bump_medium",
    "disk_medium",
    "plane_wave",
    "random_complex",
    "CONFIGS",
    "config_inputs",
    "fno_param_sizes",
    "fno_initial_parameters",
    "fno_sample_recipe",
]


def grid_coords(n: int, h: float | None = None):
    """Return (X, Z), each [n, n] with X[j, i] = h*(i+1), Z[j, i] = h*(j+1)."""
    if h is None:
        h = 1.0 / n
    x = h * (np.arange(n) + 1.0)
    Z, X = np.meshgrid(x, x, indexing="ij")
    return X, Z


def gaussian_disk_medium(n: int, amp=0.2, width=0.08, radius=0.3, centre=(0.5, 0.5)):
    """Single Gaussian bump truncated to a disk (the small CPU-sized case)."""
    X, Z = grid_coords(n)
    r2 = (X - centre[0]) ** 2 + (Z - centre[1]) ** 2
    m = amp * np.exp(-r2 / (2.0 * width**2))
    m[r2 > radius**2] = 0.0
    return m


def gaussian_bumps_medium(n: int, seed: int, nbumps: int = 8):
    """Sum of Gaussian bumps; returns (m, theta).

    Draw order with numpy.random.default_rng(seed): centres U[0.2,0.8]^2
    (nbumps x 2, columns x then z), widths U[0.03,0.1] (nbumps), amplitudes
    U[-0.3,0.3] (nbumps), then one incidence angle U[0, 2*pi).
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, size=(nbumps, 2))
    widths = rng.uniform(0.03, 0.1, size=nbumps)
    amps = rng.uniform(-0.3, 0.3, size=nbumps)
    theta = float(rng.uniform(0.0, 2.0 * np.pi))
    X, Z = grid_coords(n)
    m = np.zeros((n, n))
    for (cx, cz), w, a in zip(centres, widths, amps):
        m += a * np.exp(-((X - cx) ** 2 + (Z - cz) ** 2) / (2.0 * w * w))
    return m, theta


def gaussian_random_field_medium(n: int, seed: int, corr_len=0.05, std=0.15,
                                 r_in=0.35, r_out=0.45):
    """Smooth Gaussian random field with compact support.

    White noise (default_rng(seed).standard_normal((n, n))) filtered in
    Fourier space by exp(-|k|^2 corr_len^2 / 2), rescaled to empirical
    standard deviation `std`, times a radial cut-off that is 1 for
    r <= r_in and falls to 0 at r_out with a cubic smoothstep.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n))
    h = 1.0 / n
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
    KZ, KX = np.meshgrid(k, k, indexing="ij")
    filt = np.exp(-(KX**2 + KZ**2) * corr_len**2 / 2.0)
    field = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
    field *= std / field.std()
    X, Z = grid_coords(n)
    r = np.sqrt((X - 0.5) ** 2 + (Z - 0.5) ** 2)
    tau = np.clip((r - r_in) / (r_out - r_in), 0.0, 1.0)
    cut = 1.0 - 3.0 * tau**2 + 2.0 * tau**3
    return field * cut


def smooth_bump_medium(n: int, amp: float, width: float = 0.15, centre=(0.5, 0.5)):
    """One smooth Gaussian perturbation amp * exp(-|x - centre|^2 / (2 width^2)):
    a focusing (amp > 0) or defocusing (amp < 0) medium, the stand-in for the
    positive and negative smooth perturbations the paper's Section 5.1
    compares (shown there only as a picture)."""
    X, Z = grid_coords(n)
    r2 = (X - centre[0]) ** 2 + (Z - centre[1]) ** 2
    return amp * np.exp(-r2 / (2.0 * width**2))


def disk_medium(n: int, contrast: float, radius: float, centre=(0.5, 0.5)):
    """Homogeneous disk: m = contrast inside |x - centre| <= radius."""
    X, Z = grid_coords(n)
    r2 = (X - centre[0]) ** 2 + (Z - centre[1]) ** 2
    return np.where(r2 <= radius**2, float(contrast), 0.0)


def plane_wave(n: int, omega: float, theta: float, h: float | None = None):
    """Incident plane wave u_I = exp(i*omega*(x cos(theta) + z sin(theta)))
    sampled on the grid, [n, n] complex128."""
    if h is None:
        h = 1.0 / n
    X, Z = grid_coords(n, h)
    return np.exp(1j * omega * (X * np.cos(theta) + Z * np.sin(theta)))


def random_complex(shape, seed: int):
    """Standard complex normal samples, complex128."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# Workloads: (name, n, omega, slabs, medium recipe).  omega = 2*pi*f keeps
# ~10 points per wavelength on the unit square with h = 1/n.
CONFIGS = {
    "c1_64_gauss_disk": dict(n=64, omega=2 * np.pi * 6, slabs=4),
    "c2_1024_bumps": dict(n=1024, omega=2 * np.pi * 100, slabs=16),
    "c3_2048_grf": dict(n=2048, omega=2 * np.pi * 200, slabs=32),
}


def config_inputs(name: str):
    """Return dict(n, h, omega, slabs, m, uI, theta) for a named workload."""
    cfg = dict(CONFIGS[name])
    n = cfg["n"]
    if name.startswith("c1"):
        m = gaussian_disk_medium(n)
        theta = 0.0
    elif name.startswith("c2"):
        m, theta = gaussian_bumps_medium(n, seed=0)
    elif name.startswith("c3"):
        m = gaussian_random_field_medium(n, seed=0)
        theta = 0.0
    else:
        raise KeyError(name)
    cfg.update(h=1.0 / n, m=m, theta=theta, uI=plane_wave(n, cfg["omega"], theta))
    return cfg


# ---------------------------------------------------------------- learned part
# Flat parameter vector of the Fourier-neural-operator preconditioner, in
# order: lift weight [W][5], lift bias [W]; per Fourier layer l: spectral
# weights real part [2M][M][W][W], imaginary part [2M][M][W][W], pointwise
# weight [W][W], bias [W]; projection 1 weight [Hd][W], bias [Hd];
# projection 2 weight [2][Hd], bias [2].
def fno_param_sizes(width=32, modes=16, layers=4, hidden=128):
    """(kind, fan_in, size) of each block of the flat vector, in order."""
    sizes = [("affine", 5, width * 5), ("bias", 5, width)]
    for _ in range(layers):
        sizes += [("spectral", width, 2 * modes * modes * width * width),
                  ("spectral", width, 2 * modes * modes * width * width),
                  ("affine", width, width * width), ("bias", width, width)]
    sizes += [("affine", width, hidden * width), ("bias", width, hidden),
              ("last", hidden, 2 * hidden), ("lastbias", hidden, 2)]
    return sizes


def fno_initial_parameters(seed: int, width=32, modes=16, layers=4, hidden=128):
    """Seeded initial weights, float64: affine maps and biases uniform in
    +-1/sqrt(fan_in), spectral weights uniform in [0, 1) / width^2, and the
    last projection scaled by 1e-2 (the network starts close to z = r)."""
    rng = np.random.default_rng(seed)
    parts = []
    for kind, fan_in, size in fno_param_sizes(width, modes, layers, hidden):
        if kind == "spectral":
            parts.append(rng.random(size) / width**2)
        else:
            a = 1.0 / np.sqrt(fan_in)
            scale = 1e-2 if kind.startswith("last") else 1.0
            parts.append(scale * rng.uniform(-a, a, size))
    return np.concatenate(parts)


def fno_sample_recipe(seed: int, n: int = 256):
    """One training / test sample of the learned preconditioner: a Gaussian
    random field medium (seed) and an incident angle theta ~ U[0, 2 pi) drawn
    from the same seed.  Returns (m, theta)."""
    m = gaussian_random_field_medium(n, seed=seed)
    theta = float(np.random.default_rng(10_000_000 + seed).uniform(0.0, 2 * np.pi))
    return m, theta
