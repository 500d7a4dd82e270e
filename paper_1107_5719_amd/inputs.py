"""Seeded synthetic media for the 3D scattering solve.

This module is the only code that the HIP path's tests and the CPU oracle's tests share.  It builds
*inputs* only -- opacity chi, thermalisation parameter epsilon and Planck function B on an
``(nz, ny, nx)`` grid (x fastest, k = 0 is the bottom layer) -- and holds none of the arithmetic of
the method itself (no formal solution, no Lambda operator, no operator splitting).

The workloads stand in for the paper's parameterised slab test ("Test case setup": a plane-parallel
slab with periodic x,y, a power-law continuum optical depth spanning many decades, an isothermal
source, coherent isotropic scattering with a constant epsilon).  The paper's own atmosphere needs its
earlier papers and physical units; here the medium is a synthetic stratified atmosphere with the same
structure: unit voxels, chi falling exponentially with height over about seven decades, a seeded
perturbation on chi, uniform epsilon and a given B profile.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Workload", "WORKLOADS", "stratified_profile", "paper_slab_profile", "make_medium", "random_medium",
           "diffusion_medium", "wavelength_batch",
           "emergent_target"]


@dataclass(frozen=True)
class Workload:
    """One named synthetic workload: grid, angle set, medium recipe and stopping rule."""

    name: str
    nx: int
    ny: int
    nz: int
    n_theta: int
    n_phi: int
    tau_total: float          # vertical optical depth of the unperturbed column
    eps: float                # uniform thermalisation parameter
    b_profile: str            # "const" (B = b_value) or "linear_10_1" (10 at the bottom, 1 at the top)
    noise: str                # "iid" (i.i.d. log-normal) or "grf" (Gaussian random field, periodic in x,y)
    sigma: float              # standard deviation of log(chi) perturbation
    seed: int
    tol: float = 1e-8         # outer stopping threshold on max_v |dJ_v| / |J_v|
    corr_len: float = 4.0     # correlation length in voxels ("grf" only)
    b_value: float = 1.0
    I_top: float = 0.0        # incoming intensity at the outer (top) boundary
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_dir(self):
        return self.n_theta * self.n_phi

    @property
    def n_vox(self):
        return self.nx * self.ny * self.nz


# The three plain-method / precision-form workloads.  Sizes and angle counts follow the benchmark
# configurations; the stratification scale is H = nz / (7 ln 10) so that chi spans about seven
# decades between the bottom and the top voxel.
WORKLOADS = {
    "strat17": Workload("strat17", 17, 17, 17, 8, 8, tau_total=1e3, eps=1e-2, b_profile="const",
                        noise="iid", sigma=0.05, seed=1, tol=1e-8),
    "grf65": Workload("grf65", 65, 65, 65, 16, 16, tau_total=1e4, eps=1e-4, b_profile="linear_10_1",
                      noise="grf", sigma=0.2, seed=2, tol=1e-8),
    "strat129": Workload("strat129", 129, 129, 129, 16, 16, tau_total=1e3, eps=1e-6, b_profile="const",
                         noise="iid", sigma=0.05, seed=3, tol=1e-8),
    # the paper's timing grids ("Timing results": 65^3 and 129^2 x 193 voxels) with its slab
    # ("Test case setup": continuum optical depth a power law from 1e-4 at the outer boundary to 1e8 at
    # the inner one, isothermal, eps = 1e-2); plane-parallel in structure, so no perturbation
    "slab65": Workload("slab65", 65, 65, 65, 16, 16, tau_total=1e8, eps=1e-2, b_profile="const",
                       noise="none", sigma=0.0, seed=0, tol=1e-8, extra={"profile": "paper_slab"}),
    "slab193": Workload("slab193", 129, 129, 193, 16, 16, tau_total=1e8, eps=1e-2, b_profile="const",
                        noise="none", sigma=0.0, seed=0, tol=1e-8, extra={"profile": "paper_slab"}),
    # differentiation workload: gradients of a loss on the emergent light through the converged solution
    "strat65adj": Workload("strat65adj", 65, 65, 65, 8, 8, tau_total=1e3, eps=1e-2, b_profile="const",
                           noise="iid", sigma=0.05, seed=5, tol=1e-14),
}


def stratified_profile(nz: int, tau_total: float, decades: float = 7.0) -> np.ndarray:
    """chi_k = chi0 * exp(-(k + 1/2) / H) with H = nz / (decades * ln 10) and sum_k chi_k = tau_total."""
    H = nz / (decades * math.log(10.0))
    zc = np.arange(nz, dtype=np.float64) + 0.5
    prof = np.exp(-zc / H)
    return prof * (tau_total / prof.sum())


def paper_slab_profile(nz: int, tau_min: float = 1e-4, tau_max: float = 1e8) -> np.ndarray:
    """The paper's slab: the continuum optical depth at height z (unit voxels, z = nz outside) is the
    power law tau(z) = tau_min (tau_max / tau_min)^((nz - z) / nz), so layer k has the opacity
    chi_k = tau(k) - tau(k + 1) (its optical thickness); tau(nz) = tau_min is the optical depth of the
    medium above the grid, which carries no opacity here."""
    z = np.arange(nz + 1, dtype=np.float64)
    tau = tau_min * (tau_max / tau_min) ** ((nz - z) / nz)
    return tau[:-1] - tau[1:]


def _grf(rng: np.random.Generator, nz: int, ny: int, nx: int, corr_len: float) -> np.ndarray:
    """Unit-variance Gaussian random field with covariance exp(-r^2 / (2 l^2)).

    Periodic in x,y (FFT on the true grid); z is generated on a box padded by 3 l on each side and
    cropped, so the top and bottom are not correlated with each other."""
    pad = int(math.ceil(3.0 * corr_len))
    nzp = nz + 2 * pad
    white = rng.standard_normal((nzp, ny, nx))
    kz = np.fft.fftfreq(nzp) * 2.0 * math.pi
    ky = np.fft.fftfreq(ny) * 2.0 * math.pi
    kx = np.fft.fftfreq(nx) * 2.0 * math.pi
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    amp = np.exp(-0.25 * corr_len ** 2 * k2)        # square root of the Gaussian spectral density
    field_ = np.real(np.fft.ifftn(np.fft.fftn(white) * amp))[pad:pad + nz]
    field_ -= field_.mean()
    return field_ / field_.std()


def make_medium(w: Workload | str):
    """Return dict(chi, eps, B) as C-contiguous float64 arrays of shape (nz, ny, nx)."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    rng = np.random.Generator(np.random.PCG64(w.seed))
    if w.extra.get("profile") == "paper_slab":
        prof = paper_slab_profile(w.nz)
    else:
        prof = stratified_profile(w.nz, w.tau_total)
    if w.noise == "iid":
        g = rng.standard_normal(w.shape)
    elif w.noise == "grf":
        g = _grf(rng, w.nz, w.ny, w.nx, w.corr_len)
    elif w.noise == "none":
        g = np.zeros(w.shape)
    else:
        raise ValueError(f"unknown noise model {w.noise!r}")
    chi = prof[:, None, None] * np.exp(w.sigma * g)
    eps = np.full(w.shape, w.eps)
    if w.b_profile == "const":
        B = np.full(w.shape, w.b_value)
    elif w.b_profile == "linear_10_1":
        k = np.arange(w.nz, dtype=np.float64)
        B = np.broadcast_to((10.0 - 9.0 * k / (w.nz - 1))[:, None, None], w.shape).copy()
    else:
        raise ValueError(f"unknown B profile {w.b_profile!r}")
    return {"chi": np.ascontiguousarray(chi), "eps": np.ascontiguousarray(eps),
            "B": np.ascontiguousarray(B)}


def diffusion_medium(nx: int, ny: int, nz: int, seed: int, chi_range=(1e-2, 3.0), eps_range=(0.05, 0.5)):
    """Small random medium for the LTE-diffusion inner condition, which assumes an optically thick
    bottom and B varying slowly with depth: as random_medium, but the two bottom layers have
    chi >= 1 and B falls linearly from 1.5 (bottom) to 1 (top) with a 5 % perturbation."""
    m = random_medium(nx, ny, nz, seed, chi_range=chi_range, eps_range=eps_range)
    m["chi"][:2] = np.maximum(m["chi"][:2], 1.0)
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    prof = 1.5 - 0.5 * np.arange(nz) / max(nz - 1, 1)
    m["B"] = prof[:, None, None] * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, (nz, ny, nx)))
    return m


def random_medium(nx: int, ny: int, nz: int, seed: int, chi_range=(1e-2, 1e2),
                  eps_range=(1e-3, 1.0), b_range=(0.5, 2.0)):
    """Small fully heterogeneous medium for parity tests: log-uniform chi and eps, uniform B."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)
    lo, hi = np.log(chi_range[0]), np.log(chi_range[1])
    chi = np.exp(rng.uniform(lo, hi, shape))
    elo, ehi = np.log(eps_range[0]), np.log(eps_range[1])
    eps = np.exp(rng.uniform(elo, ehi, shape))
    B = rng.uniform(b_range[0], b_range[1], shape)
    return {"chi": chi, "eps": eps, "B": B}


def wavelength_batch(n: int = 64, sizes=(33, 65, 97), n_theta: int = 8, n_phi: int = 8, seed0: int = 1000,
                     chi0_range=(1e-2, 1e2), eps_range=(1e-6, 1e-1), sigma: float = 0.05,
                     decades: float = 7.0):
    """Many wavelengths of one stratified atmosphere, each on a grid of its own.

    Wavelength l uses the generator seeded with seed0 + l: it draws the grid edge N uniformly from
    ``sizes`` (an N^3 grid), the opacity chi0 at the bottom plane log-uniformly from chi0_range and
    a uniform epsilon log-uniformly from eps_range; then chi_k = chi0 exp(-(k + 1/2) / H) with
    H = N / (decades ln 10) (the same fall-off over the column as the single-wavelength workloads),
    times an i.i.d. log-normal perturbation of standard deviation sigma per voxel; B = 1.

    Returns a list of dicts: grid (nx, ny, nz, n_theta, n_phi) and medium (chi, eps, B), plus the
    drawn chi0 and eps."""
    out = []
    for lam in range(n):
        rng = np.random.Generator(np.random.PCG64(seed0 + lam))
        N = int(sizes[int(rng.integers(len(sizes)))])
        chi0 = float(np.exp(rng.uniform(np.log(chi0_range[0]), np.log(chi0_range[1]))))
        eps = float(np.exp(rng.uniform(np.log(eps_range[0]), np.log(eps_range[1]))))
        H = N / (decades * math.log(10.0))
        prof = chi0 * np.exp(-(np.arange(N, dtype=np.float64) + 0.5) / H)
        chi = prof[:, None, None] * np.exp(sigma * rng.standard_normal((N, N, N)))
        out.append({
            "grid": {"nx": N, "ny": N, "nz": N, "n_theta": n_theta, "n_phi": n_phi},
            "chi": np.ascontiguousarray(chi), "eps": np.full((N, N, N), eps), "B": np.ones((N, N, N)),
            "chi0": chi0, "eps_value": eps,
        })
    return out


def emergent_target(n_up: int, ny: int, nx: int, seed: int, lo: float = 0.2, hi: float = 0.8):
    """Seeded target T for a loss sum (I_em - T)^2 on the emergent top intensities
    ([n_up, ny, nx], uniform in [lo, hi])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, (n_up, ny, nx))
