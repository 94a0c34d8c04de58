"""Plain FP64 CPU oracle for the FFT + tridiagonal pressure-Poisson projection method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module:
only the tests, the package smoke check and the bench's CPU-baseline leg use it.
It shares no code with the HIP path (it is written in plain PyTorch CPU ops,
complex128/float64, so that autograd of this forward also serves as the oracle
gradient for the hand-written adjoint).

What it computes, following the paper (arXiv 2104.08863):
  * Section 2, Eq. (1)-(7): projection method, explicit RK2 (Heun, Eq. (5)-(6)),
    pressure Poisson equation for grad p from div u*/dt, velocity update Eq. (4);
  * Section 2.1, Eq. (8)-(9): transform the two periodic directions (x: real
    FFT, z: complex FFT) so every wavenumber pair leaves one tridiagonal system
    along the wall-normal direction y; solve it, transform back;
  * Section 2.2, Eq. (10)-(21): the PDD partitioned tridiagonal solve (local
    Thomas solves, reduced system Z with or without the small corner terms,
    correction) -- kept here as the approximation the GPU drop path reproduces;
    the plain Thomas solve is the exact definition used for the pressure.

Readings where the paper is silent or garbled:
  * y is wall-normal, z spanwise (Section 5 naming);
  * Eq. (9): the middle coefficient is -2 (the printed +2 is a sign garble);
  * steps (6) and (8) of Section 3.2 are inverse transforms;
  * the non-uniform wall-normal stencil is L_h = D o G on the staggered grid;
  * gauge of the singular kx=kz=0 line: the RHS is first made compatible by
    removing its dy-weighted mean, the last unknown is pinned to zero, and the
    dy-weighted mean of the result is removed;
  * momentum RHS: divergence (flux) form with linear interpolation, Laplacian
    with the no-slip ghost mirrored about the wall (parity of this part is
    pinned by conservation, Galilean and convergence properties, not by
    values printed in the paper);
  * per-plane statistics: plain means over the x-z plane of the stored
    (staggered) u, v, w and their squares.

Array layout: physical (ny, nz, nx); spectrum (ny, nz, nx//2+1).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

F64 = torch.float64
C128 = torch.complex128


# ----------------------------------------------------------------------------
# Geometry (Section 2: uniform in x and z, stretched in y; staggered, Fig. 2)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Box:
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    y_faces: np.ndarray  # (ny+1,) strictly increasing

    def __post_init__(self):
        yf = np.asarray(self.y_faces, dtype=np.float64)
        assert yf.shape == (self.ny + 1,)
        self.y_faces = yf
        self.dx = self.lx / self.nx
        self.dz = self.lz / self.nz
        self.dy_np = yf[1:] - yf[:-1]                     # cell heights, (ny,)
        yc = 0.5 * (yf[1:] + yf[:-1])
        self.dyc_np = yc[1:] - yc[:-1]                     # centre spacing at face j+1, (ny-1,)
        self.dy = torch.tensor(self.dy_np, dtype=F64)
        self.dyc = torch.tensor(self.dyc_np, dtype=F64)
        self.nkx = self.nx // 2 + 1


def y_coefficients(box: Box):
    """Rows of the wall-normal operator (L_h restricted to y):
    (L p)_j = a_j p_{j-1} - (a_j + c_j) p_j + c_j p_{j+1},
    a_j = 1/(dy_j dyc_{j-1/2}) (zero at the bottom wall row),
    c_j = 1/(dy_j dyc_{j+1/2}) (zero at the top wall row)."""
    ny = box.ny
    a = np.zeros(ny)
    c = np.zeros(ny)
    a[1:] = 1.0 / (box.dy_np[1:] * box.dyc_np)
    c[:-1] = 1.0 / (box.dy_np[:-1] * box.dyc_np)
    return torch.tensor(a, dtype=F64), torch.tensor(c, dtype=F64)


def modified_wavenumbers(box: Box):
    """Eigenvalues of the periodic second difference under the DFT (Eq. (9)'s
    lambda_i, lambda_j): lambda(k)/d^2 = -(2 sin(pi k / n)/d)^2.  Returns
    k2[kz, kx] = (2 sin(pi kx/nx)/dx)^2 + (2 sin(pi kz/nz)/dz)^2 >= 0."""
    kx = np.arange(box.nkx, dtype=np.float64)
    kz = np.arange(box.nz, dtype=np.float64)
    sx = (2.0 * np.sin(np.pi * kx / box.nx) / box.dx) ** 2
    sz = (2.0 * np.sin(np.pi * kz / box.nz) / box.dz) ** 2
    return torch.tensor(sz[:, None] + sx[None, :], dtype=F64)


def mean_w(q: torch.Tensor, box: Box) -> torch.Tensor:
    """Volume-weighted mean of a cell-centred field: sum dy_j q / (nx nz sum dy)."""
    return (q * box.dy[:, None, None]).sum() / (box.nx * box.nz * box.dy.sum())


# ----------------------------------------------------------------------------
# Transforms (Eq. (9): real DFT in x, complex DFT in z; inverse as in the text
# after Eq. (9), normalised once by 1/(nx nz))
# ----------------------------------------------------------------------------
def forward_transform(f: torch.Tensor) -> torch.Tensor:
    return torch.fft.fft(torch.fft.rfft(f, dim=2), dim=1)


def inverse_transform(fh: torch.Tensor, nx: int) -> torch.Tensor:
    return torch.fft.irfft(torch.fft.ifft(fh, dim=1), n=nx, dim=2)


# ----------------------------------------------------------------------------
# Thomas algorithm (Section 2.1: O(n) elimination along the wall-normal lines)
# ----------------------------------------------------------------------------
def thomas(a, b, c, d):
    """Solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j, j = 0..n-1, along dim 0.
    a, b, c, d broadcast against each other over the trailing (line) dims;
    a_0 and c_{n-1} are ignored."""
    n = d.shape[0]
    cp = [None] * n
    dp = [None] * n
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for j in range(1, n):
        den = b[j] - a[j] * cp[j - 1]
        cp[j] = c[j] / den
        dp[j] = (d[j] - a[j] * dp[j - 1]) / den
    x = [None] * n
    x[n - 1] = dp[n - 1]
    for j in range(n - 2, -1, -1):
        x[j] = dp[j] - cp[j] * x[j + 1]
    return torch.stack(x, dim=0)


def solve_spectral(fh: torch.Tensor, box: Box) -> torch.Tensor:
    """Solve every (kx, kz) line of Eq. (9) (corrected) along y.

    fh: (ny, nz, nkx) complex, the unnormalised forward transform of f.
    Lines with (kx, kz) != (0, 0): Thomas on a_j p_{j-1} + (-a_j-c_j-k^2) p_j +
    c_j p_{j+1} = fh_j.  Line (0, 0): compatibility projection (remove the
    dy-weighted mean of the RHS), pin the top unknown to zero, Thomas on the
    remaining ny-1 rows, then remove the dy-weighted mean of the result."""
    ny, nz, nkx = fh.shape
    a, c = y_coefficients(box)
    k2 = modified_wavenumbers(box)
    k2 = k2.clone()
    k2[0, 0] = 1.0  # placeholder; the (0,0) line is replaced below
    b = -(a + c)[:, None, None] - k2[None]
    ph = thomas(a[:, None, None], b, c[:, None, None], fh)
    ph = ph.clone()
    ph[:, 0, 0] = solve_mean_line(fh[:, 0, 0], box)
    return ph


def solve_mean_line(f0: torch.Tensor, box: Box) -> torch.Tensor:
    """The kx = kz = 0 line (singular Neumann operator) with the gauge of the
    reading above."""
    ny = box.ny
    a, c = y_coefficients(box)
    dy = box.dy.to(f0.dtype)
    g = f0 - (dy * f0).sum() / dy.sum()
    b = -(a + c)
    x = thomas(a[: ny - 1], b[: ny - 1], c[: ny - 1], g[: ny - 1])
    x = torch.cat([x, torch.zeros(1, dtype=x.dtype)])
    return x - (dy * x).sum() / dy.sum()


def poisson(f: torch.Tensor, box: Box) -> torch.Tensor:
    """p with L_h p = f - mean_W(f) and mean_W(p) = 0 (FFT x,z + Thomas y)."""
    return inverse_transform(solve_spectral(forward_transform(f), box), box.nx)


# ----------------------------------------------------------------------------
# Staggered operators (Fig. 2; second-order centred differences)
# ----------------------------------------------------------------------------
def _ym1(q):
    """q_{j-1} along y with a zero plane below j = 0."""
    return torch.cat([torch.zeros_like(q[:1]), q[:-1]], dim=0)


def _wall_v(v):
    """v with its top-wall plane forced to zero (the stored plane is ignored)."""
    return torch.cat([v[:-1], torch.zeros_like(v[:1])], dim=0)


def divergence(u, v, w, box: Box):
    """D: faces -> centres.  (u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy_j + (w_k - w_{k-1})/dz
    with v = 0 on both walls."""
    vv = _wall_v(v)
    return ((u - torch.roll(u, 1, 2)) / box.dx
            + (vv - _ym1(vv)) / box.dy[:, None, None]
            + (w - torch.roll(w, 1, 1)) / box.dz)


def gradient(p, box: Box):
    """G: centres -> faces.  The v component exists on interior faces only;
    the top-wall plane is zero."""
    gu = (torch.roll(p, -1, 2) - p) / box.dx
    gv = (p[1:] - p[:-1]) / box.dyc[:, None, None]
    gv = torch.cat([gv, torch.zeros_like(p[:1])], dim=0)
    gw = (torch.roll(p, -1, 1) - p) / box.dz
    return gu, gv, gw


def laplacian_p(p, box: Box):
    """L_h = D o G (7-point, non-uniform in y, Neumann walls)."""
    return divergence(*gradient(p, box), box)


# ----------------------------------------------------------------------------
# Momentum right-hand side R(u) = -N(u) + nu lap(u) + fx e_x (Eq. (3), (5), (6))
# ----------------------------------------------------------------------------
def _lap_xz(q, box):
    return ((torch.roll(q, -1, 2) - 2 * q + torch.roll(q, 1, 2)) / box.dx ** 2
            + (torch.roll(q, -1, 1) - 2 * q + torch.roll(q, 1, 1)) / box.dz ** 2)


def _lap_y_centre(q, box):
    """Wall-normal part for a cell-centred-in-y component (u or w), no-slip
    ghost q_{-1} = -q_0, q_{ny} = -q_{ny-1} at distance dy of the wall cell."""
    dy = box.dy[:, None, None]
    dyc = box.dyc[:, None, None]
    inner = (q[1:] - q[:-1]) / dyc                       # flux at faces 1..ny-1
    bot = 2.0 * q[:1] / box.dy[0]                          # (q_0 - q_{-1}) / dy_0
    top = -2.0 * q[-1:] / box.dy[-1]                       # (q_{ny} - q_{ny-1}) / dy_{ny-1}
    flux = torch.cat([bot, inner, top], dim=0)             # faces 0..ny
    return (flux[1:] - flux[:-1]) / dy


def _lap_y_face(v, box):
    """Wall-normal part for v on interior faces j = 0..ny-2 (v = 0 on walls);
    the top-wall plane of the result is zero."""
    vv = _wall_v(v)
    dy = box.dy[:, None, None]
    vm = _ym1(vv)
    # flux at centre j: (v_j - v_{j-1}) / dy_j, j = 0..ny-1
    flux = (vv - vm) / dy
    dyc = box.dyc[:, None, None]
    out = (flux[1:] - flux[:-1]) / dyc                     # faces j = 0..ny-2
    return torch.cat([out, torch.zeros_like(v[:1])], dim=0)


def _interp_y_to_face(q, box):
    """Linear interpolation of a centre-in-y quantity to interior faces j+1,
    j = 0..ny-2, weighted by distance: (q_j dy_{j+1} + q_{j+1} dy_j)/(dy_j+dy_{j+1})."""
    dy = box.dy
    wl = (dy[1:] / (dy[:-1] + dy[1:]))[:, None, None]
    wu = (dy[:-1] / (dy[:-1] + dy[1:]))[:, None, None]
    return q[:-1] * wl + q[1:] * wu


def advection(u, v, w, box: Box):
    """N(u) = div(u u) in flux form with linear interpolation (conservative)."""
    dx, dz = box.dx, box.dz
    dy = box.dy[:, None, None]
    dyc = box.dyc[:, None, None]
    vv = _wall_v(v)
    zero_plane = torch.zeros_like(u[:1])
    # centre squares
    uc = 0.5 * (u + torch.roll(u, 1, 2))
    wc = 0.5 * (w + torch.roll(w, 1, 1))
    vc = 0.5 * (vv + _ym1(vv))
    # edge products
    exy = _interp_y_to_face(u, box) * (0.5 * (vv[:-1] + torch.roll(vv[:-1], -1, 2)))
    exy = torch.cat([exy, zero_plane], dim=0)              # top-wall edge: v = 0
    eyz = _interp_y_to_face(w, box) * (0.5 * (vv[:-1] + torch.roll(vv[:-1], -1, 1)))
    eyz = torch.cat([eyz, zero_plane], dim=0)
    exz = (0.5 * (u + torch.roll(u, -1, 1))) * (0.5 * (w + torch.roll(w, -1, 2)))
    # x-momentum at (i+1/2, j, k)
    nx_ = ((torch.roll(uc * uc, -1, 2) - uc * uc) / dx
           + (exy - _ym1(exy)) / dy
           + (exz - torch.roll(exz, 1, 1)) / dz)
    # y-momentum at (i, j+1 face, k), j = 0..ny-2
    vv2 = vc * vc
    ny_ = ((exy - torch.roll(exy, 1, 2)) / dx
           + torch.cat([(vv2[1:] - vv2[:-1]) / dyc, zero_plane], dim=0)
           + (eyz - torch.roll(eyz, 1, 1)) / dz)
    ny_ = torch.cat([ny_[:-1], zero_plane], dim=0)
    # z-momentum at (i, j, k+1/2)
    nz_ = ((exz - torch.roll(exz, 1, 2)) / dx
           + (eyz - _ym1(eyz)) / dy
           + (torch.roll(wc * wc, -1, 1) - wc * wc) / dz)
    return nx_, ny_, nz_


def laplacian_vel(u, v, w, box: Box):
    lu = _lap_xz(u, box) + _lap_y_centre(u, box)
    lv = _lap_xz(_wall_v(v), box) + _lap_y_face(v, box)
    lv = torch.cat([lv[:-1], torch.zeros_like(v[:1])], dim=0)
    lw = _lap_xz(w, box) + _lap_y_centre(w, box)
    return lu, lv, lw


def momentum_rhs(u, v, w, box: Box, nu: float, fx: float):
    nxu, nyv, nzw = advection(u, v, w, box)
    lu, lv, lw = laplacian_vel(u, v, w, box)
    return (-nxu + nu * lu + fx, -nyv + nu * lv, -nzw + nu * lw)


# ----------------------------------------------------------------------------
# One projection step (Eq. (4)-(7), RK2 of Eq. (5)-(6), one pressure solve)
# ----------------------------------------------------------------------------
def rk2_predictor(u, v, w, box: Box, dt: float, nu: float, fx: float):
    """Heun predictor of Eq. (5)-(6): ub = u + dt R(u),
    u* = u + dt/2 (R(u) + R(ub)); v is zero on the top wall."""
    v = _wall_v(v)
    r0 = momentum_rhs(u, v, w, box, nu, fx)
    ub = u + dt * r0[0]
    vb = _wall_v(v + dt * r0[1])
    wb = w + dt * r0[2]
    r1 = momentum_rhs(ub, vb, wb, box, nu, fx)
    us = u + 0.5 * dt * (r0[0] + r1[0])
    vs = _wall_v(v + 0.5 * dt * (r0[1] + r1[1]))
    ws = w + 0.5 * dt * (r0[2] + r1[2])
    return us, vs, ws


def projection_step(u, v, w, box: Box, dt: float, nu: float, fx: float,
                    return_pressure: bool = False):
    us, vs, ws = rk2_predictor(u, v, w, box, dt, nu, fx)
    p = poisson(divergence(us, vs, ws, box) / dt, box)
    gu, gv, gw = gradient(p, box)
    out = (us - dt * gu, vs - dt * gv, ws - dt * gw)
    if return_pressure:
        return out + (p,)
    return out



def plane_stats(u, v, w):
    """Per-plane means over the x-z plane of the stored u, v, w and of their
    squares (the averages of a channel-flow run, Section 5): (ny, 6)."""
    cols = [u, v, w, u * u, v * v, w * w]
    return torch.stack([c.mean(dim=(1, 2)) for c in cols], dim=1)

def rollout(u, v, w, box: Box, nsteps: int, dt: float, nu: float, fx: float):
    for _ in range(nsteps):
        u, v, w = projection_step(u, v, w, box, dt, nu, fx)
    return u, v, w


def rollout_loss_and_grad(u0, v0, w0, box: Box, nsteps: int, dt: float,
                          nu: float, fx: float):
    """loss = 0.5 sum(u^2 + v^2 + w^2) after nsteps; gradient by autograd of
    this plain forward (the oracle gradient for the hand-written adjoint)."""
    u = u0.detach().clone().requires_grad_(True)
    v = v0.detach().clone().requires_grad_(True)
    w = w0.detach().clone().requires_grad_(True)
    a, b, c = rollout(u, v, w, box, nsteps, dt, nu, fx)
    loss = 0.5 * ((a * a).sum() + (b * b).sum() + (c * c).sum())
    gu, gv, gw = torch.autograd.grad(loss, (u, v, w))
    return loss.detach(), gu, gv, gw


# ----------------------------------------------------------------------------
# PDD partitioned tridiagonal solve (Section 2.2, Eq. (10)-(21), steps 1-5)
# ----------------------------------------------------------------------------
def _partition_solves(a, b, c, d, p):
    """Eq. (20): for each partition i, A_i [xt, v, w] = [d^i, a_1^i e_1, c_m^i e_m]
    where A_i is the diagonal block (its own first a and last c left out).
    a, c: (n,) real; b: (n, L) real; d: (n, L) complex.  Returns lists."""
    n = d.shape[0]
    m = n // p
    xt, vs, ws = [], [], []
    for i in range(p):
        r0, r1 = i * m, (i + 1) * m
        ai = a[r0:r1].clone()
        ci = c[r0:r1].clone()
        a_first = ai[0].item()
        c_last = ci[-1].item()
        ai[0] = 0.0
        ci[-1] = 0.0
        bi = b[r0:r1]
        L = b.shape[1]
        e1 = torch.zeros(m, L, dtype=F64)
        em = torch.zeros(m, L, dtype=F64)
        e1[0] = a_first if i > 0 else 0.0
        em[-1] = c_last if i < p - 1 else 0.0
        xt.append(thomas(ai[:, None], bi, ci[:, None], d[r0:r1]))
        vs.append(thomas(ai[:, None], bi, ci[:, None], e1))
        ws.append(thomas(ai[:, None], bi, ci[:, None], em))
    return xt, vs, ws


def pdd_solve(a, b, c, d, p: int, drop: bool):
    """PDD solve of the lines (a_j, b_j(line), c_j; d_j(line)) split into p
    partitions of m = n/p rows.  drop=True: the reduced system Z of Eq. (21)
    loses the corner terms v_m^i, w_1^i and decouples into 2x2 blocks solved by
    Cramer's rule (step 4).  drop=False: the full Z is solved (exact SMW)."""
    n, L = d.shape
    assert n % p == 0
    if p == 1:
        return thomas(a[:, None], b, c[:, None], d)
    xt, vs, ws = _partition_solves(a, b, c, d, p)
    q = p - 1
    if drop:
        y1 = []
        y2 = []
        for i in range(q):
            wm = ws[i][-1]
            v1 = vs[i + 1][0]
            r1 = xt[i][-1]
            r2 = xt[i + 1][0]
            det = 1.0 - wm * v1
            y1.append((r1 - wm * r2) / det)
            y2.append((r2 - v1 * r1) / det)
    else:
        # unknowns ordered (y1^1, y2^1, y1^2, y2^2, ...), y1^i = x_m^i, y2^i = x_1^{i+1}
        Z = torch.zeros(L, 2 * q, 2 * q, dtype=F64)
        rhs = torch.zeros(L, 2 * q, dtype=C128)
        for i in range(q):
            r, s = 2 * i, 2 * i + 1
            Z[:, r, r] = 1.0
            Z[:, s, s] = 1.0
            Z[:, r, s] = ws[i][-1]              # w_m^i  * y2^i
            Z[:, s, r] = vs[i + 1][0]           # v_1^{i+1} * y1^i
            if i > 0:
                Z[:, r, r - 2] = vs[i][-1]      # v_m^i * y1^{i-1}
            if i < q - 1:
                Z[:, s, s + 2] = ws[i + 1][0]   # w_1^{i+1} * y2^{i+1}
            rhs[:, r] = xt[i][-1]
            rhs[:, s] = xt[i + 1][0]
        y = torch.linalg.solve(Z.to(C128), rhs.unsqueeze(-1)).squeeze(-1)
        y1 = [y[:, 2 * i] for i in range(q)]
        y2 = [y[:, 2 * i + 1] for i in range(q)]
    out = []
    for i in range(p):
        x = xt[i]
        if i > 0:
            x = x - vs[i] * y1[i - 1][None]
        if i < p - 1:
            x = x - ws[i] * y2[i][None]
        out.append(x)
    return torch.cat(out, dim=0)


def pdd_indicator(a, b, c, p: int):
    """delta = max over interior partitions of max(|v_m^i|, |w_1^i|): the size
    of the corner terms the drop discards (Eq. (21) framed entries).
    b: (n, L).  Returns (L,) float64; zero when p <= 2."""
    n, L = b.shape
    if p <= 2:
        return torch.zeros(L, dtype=F64)
    d = torch.zeros(n, L, dtype=C128)
    _, vs, ws = _partition_solves(a, b, c, d, p)
    delta = torch.zeros(L, dtype=F64)
    for i in range(1, p - 1):
        delta = torch.maximum(delta, vs[i][-1].abs())
        delta = torch.maximum(delta, ws[i][0].abs())
    return delta


def line_coefficients(box: Box):
    """(a, c, k2) with k2 of shape (nz, nkx); b = -(a + c) - k2."""
    a, c = y_coefficients(box)
    return a, c, modified_wavenumbers(box)


def set_threads(n: int | None = None) -> int:
    if n is not None:
        torch.set_num_threads(n)
    return torch.get_num_threads()


__all__ = [
    "Box", "y_coefficients", "modified_wavenumbers", "mean_w", "forward_transform",
    "inverse_transform", "thomas", "solve_spectral", "solve_mean_line", "poisson",
    "divergence", "gradient", "laplacian_p", "advection", "laplacian_vel",
    "momentum_rhs", "rk2_predictor", "projection_step", "plane_stats", "rollout", "rollout_loss_and_grad",
    "pdd_solve", "pdd_indicator", "line_coefficients", "set_threads",
]

