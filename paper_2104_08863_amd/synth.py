"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the bench.

This module holds input recipes only: the wall-normal grid, seeded velocity
fields and right-hand sides, and the named workloads.  It contains none of the
solver's arithmetic (no divergence, no transform, no tridiagonal solve), so the
oracle and the HIP path can both consume it without sharing any method code.

Array convention everywhere: C-order (ny, nz, nx), x fastest.  ``v[j]`` sits on
the wall-normal face ``y_faces[j+1]``; ``v[ny-1]`` is the top wall and is zero.

Workloads: the channel grids of the paper's validation runs (Section 5,
Table 3) scaled to one GPU, with the wall-normal clustering of Section 2
(non-uniform grid clustered toward both walls).
"""
from __future__ import annotations

import dataclasses
import numpy as np


# ----------------------------------------------------------------------------
# Wall-normal grids
# ----------------------------------------------------------------------------
def tanh_faces(ny: int, gamma: float) -> np.ndarray:
    """Faces of a tanh-clustered grid on [-1, 1]: y_j = tanh(g(2j/ny-1))/tanh(g).

    The paper (Section 5, Table 3) gives only the resulting wall spacings; this
    mapping reproduces the printed dy+ ranges of the L550/L1000/L2000 cases
    (checked in the tests against a fixture holding the table's values).
    """
    if ny < 2:
        raise ValueError("ny must be >= 2")
    j = np.arange(ny + 1, dtype=np.float64)
    if gamma == 0.0:
        return -1.0 + 2.0 * j / ny
    y = np.tanh(gamma * (2.0 * j / ny - 1.0)) / np.tanh(gamma)
    y[0], y[-1] = -1.0, 1.0
    return y


def uniform_faces(ny: int) -> np.ndarray:
    j = np.arange(ny + 1, dtype=np.float64)
    return -1.0 + 2.0 * j / ny


# ----------------------------------------------------------------------------
# Named workloads (shapes from Table 3 scaled to one GPU)
# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    gamma: float
    nu: float = 1.0 / 550.0
    dt: float = 1.0
    fx: float = 0.0
    what: str = ""

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz

    def y_faces(self) -> np.ndarray:
        return tanh_faces(self.ny, self.gamma)


PI = np.pi
WORKLOADS = {
    # 64^3 plain FP64 Poisson solve, box 2pi x pi, tanh factor 2.0
    "poisson64": Workload("poisson64", 64, 64, 64, 2 * PI, PI, 2.0, dt=1.0,
                          what="FP64 Poisson solve, RHS = divergence of U[-1,1] field"),
    # Re_tau=550-shaped FP64 projection step, 4pi x 2pi, tanh 2.5
    "step550": Workload("step550", 1024, 256, 512, 4 * PI, 2 * PI, 2.5,
                        nu=1.0 / 550.0, dt=4e-5, fx=3.0 / 550.0,
                        what="FP64 projection step, perturbed Poiseuille"),
    # Re_tau=1000-shaped mixed-precision Poisson solve
    "mixed1000": Workload("mixed1000", 2048, 512, 1536, 4 * PI, 2 * PI, 2.6,
                          what="mixed-precision Poisson solve, k^-5/3 divergent field"),
    # differentiable rollout grid
    "rollout256": Workload("rollout256", 256, 128, 256, 2 * PI, PI, 2.0,
                           nu=1.0 / 550.0, dt=1e-3, fx=3.0 / 550.0,
                           what="8-step FP64 rollout, forward + adjoint"),
    # Re_tau=2000-shaped mixed-precision forward + adjoint step
    "adj2000": Workload("adj2000", 2048, 768, 2048, 2 * PI, PI, 3.0,
                        nu=1.0 / 2000.0, dt=3e-6, fx=3.0 / 2000.0,
                        what="mixed-precision forward + adjoint step"),
}


# ----------------------------------------------------------------------------
# Seeded fields
# ----------------------------------------------------------------------------
def uniform_rhs(nx: int, ny: int, nz: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(ny, nz, nx))


def uniform_velocity(nx: int, ny: int, nz: int, seed: int = 0):
    """u, v, w ~ U[-1, 1] (seeded PCG64), top-wall v plane zero."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(ny, nz, nx))
    v = rng.uniform(-1.0, 1.0, size=(ny, nz, nx))
    w = rng.uniform(-1.0, 1.0, size=(ny, nz, nx))
    v[ny - 1] = 0.0
    return u, v, w


def perturbed_poiseuille(nx: int, ny: int, nz: int, y_faces: np.ndarray,
                         seed: int = 0, amp: float = 0.1, dtype=np.float64):
    """Laminar profile U = 1.5 (1 - y^2) at cell centres plus i.i.d. N(0, amp^2)
    on every velocity unknown (outer units: half height 1, bulk velocity 1);
    the top-wall v plane is zero."""
    rng = np.random.default_rng(seed)
    yc = 0.5 * (y_faces[1:] + y_faces[:-1])
    u = rng.standard_normal(size=(ny, nz, nx)).astype(dtype) * dtype(amp)
    u += (1.5 * (1.0 - yc * yc)).astype(dtype)[:, None, None]
    v = rng.standard_normal(size=(ny, nz, nx)).astype(dtype) * dtype(amp)
    w = rng.standard_normal(size=(ny, nz, nx)).astype(dtype) * dtype(amp)
    v[ny - 1] = 0.0
    return u, v, w


def powerlaw_velocity(nx: int, ny: int, nz: int, seed: int = 0,
                      exponent: float = -4.0 / 3.0):
    """Random divergent field whose horizontal amplitude decays as
    max(k, 1)^exponent (shell-summed 2D energy ~ k^-5/3 for -4/3), random
    phases, white in y, independent per component, unit RMS, top-wall v zero."""
    rng = np.random.default_rng(seed)
    kx = np.arange(nx // 2 + 1, dtype=np.float64)
    kz = np.fft.fftfreq(nz, d=1.0 / nz)
    kk = np.sqrt(kx[None, :] ** 2 + kz[:, None] ** 2)
    amp = np.maximum(kk, 1.0) ** exponent
    out = []
    for _ in range(3):
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nz, nx // 2 + 1))
        spec = amp[None] * np.exp(1j * ph)
        f = np.fft.irfft2(spec, s=(nz, nx), axes=(1, 2))
        f /= np.sqrt(np.mean(f * f))
        out.append(f)
    out[1][ny - 1] = 0.0
    return tuple(out)


def powerlaw_velocity_device(nx: int, ny: int, nz: int, seed: int = 0, device="cuda",
                             exponent: float = -4.0 / 3.0):
    """The recipe of powerlaw_velocity generated on a device with a seeded
    torch generator (for grids too large to synthesise on the host): amplitude
    max(k, 1)^exponent in (kx, kz), uniform random phases, white in y,
    independent per component, unit RMS, top-wall v zero.  Same distribution,
    different random stream from the numpy version."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    kx = torch.arange(nx // 2 + 1, dtype=torch.float64, device=device)
    kz = torch.fft.fftfreq(nz, d=1.0 / nz, dtype=torch.float64, device=device)
    amp = torch.clamp(torch.sqrt(kx[None, :] ** 2 + kz[:, None] ** 2), min=1.0) ** exponent
    out = []
    for _ in range(3):
        ph = torch.rand(ny, nz, nx // 2 + 1, dtype=torch.float64, device=device, generator=gen) * (2.0 * np.pi)
        spec = torch.polar(amp.expand(ny, nz, nx // 2 + 1), ph)
        del ph
        f = torch.fft.irfft2(spec, s=(nz, nx), dim=(1, 2))
        del spec
        f /= torch.sqrt(torch.mean(f * f))
        out.append(f)
    out[1][ny - 1] = 0.0
    return tuple(out)


def random_directions(nx: int, ny: int, nz: int, seed: int):
    """N(0,1) perturbation of every free velocity unknown (top-wall v zero)."""
    rng = np.random.default_rng(seed)
    du = rng.standard_normal(size=(ny, nz, nx))
    dv = rng.standard_normal(size=(ny, nz, nx))
    dw = rng.standard_normal(size=(ny, nz, nx))
    dv[ny - 1] = 0.0
    return du, dv, dw
