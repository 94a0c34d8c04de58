"""GPU parity of the Poisson path (HIP kernels through the C ABI) against the
FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2104_08863_amd import synth

pytestmark = pytest.mark.gpu

# (nx, ny, nz, gamma, n_parts): config sizes, several tiles, ragged tails,
# radix-3 lengths and non-power-of-two partition counts
CASES = [
    (64, 64, 64, 2.0, 0),
    (64, 64, 64, 2.0, 4),
    (48, 24, 12, 2.0, 0),
    (96, 36, 24, 2.5, 3),
    (16, 8, 6, 1.0, 0),
    (128, 128, 96, 2.0, 8),
    (256, 96, 48, 2.5, 6),
    (32, 16, 2, 2.0, 1),
    # long x rows: 8 (FP64) rows per x-transform block, a ragged last block in z
    (2048, 8, 12, 2.0, 0),
    (4096, 8, 6, 1.5, 0),
    # P not dividing ny: the last partition padded (130 = 11*12 - 2 automatic,
    # 97 = 13*8 - 7 automatic, 8 = 3*3 - 1, 250 = 16*16 - 6)
    (64, 130, 32, 2.5, 0),
    (48, 97, 24, 2.0, 0),
    (32, 8, 16, 2.0, 3),
    (64, 250, 16, 2.5, 16),
]


def dev():
    return torch.device("cuda", 0)


def plan_for(nx, ny, nz, gamma, n_parts=0, precision="fp64", lx=2 * np.pi, lz=np.pi, **kw):
    from paper_2104_08863_amd.api import Plan
    yf = synth.tanh_faces(ny, gamma)
    return Plan(nx, ny, nz, lx, lz, yf, precision=precision, n_parts=n_parts, **kw), \
        O.Box(nx, ny, nz, lx, lz, yf)


def rel(a, b):
    return (np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("nx,ny,nz,gamma,parts", CASES)
def test_forward_and_inverse_transforms(nx, ny, nz, gamma, parts):
    pl, box = plan_for(nx, ny, nz, gamma, parts)
    f = synth.uniform_rhs(nx, ny, nz, seed=1)
    fg = torch.tensor(f, device=dev())
    fh = pl.forward_spectral(fg)
    ref = O.forward_transform(torch.tensor(f)).permute(2, 0, 1).numpy()   # (nkx, ny, nz)
    got = fh.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    back = pl.inverse_spectral(fh).cpu().numpy()
    assert torch.equal(fh.cpu(), torch.tensor(got))   # input spectrum left intact
    assert np.abs(back - f).max() <= 1e-14 * max(1.0, np.log2(nx * nz))


@pytest.mark.parametrize("nx,ny,nz,gamma,parts", CASES)
def test_solve_spectral_per_mode(nx, ny, nz, gamma, parts):
    pl, box = plan_for(nx, ny, nz, gamma, parts)
    rng = np.random.default_rng(2)
    fh = rng.standard_normal((nx // 2 + 1, ny, nz)) + 1j * rng.standard_normal((nx // 2 + 1, ny, nz))
    fh[0, :, 0].imag = 0.0
    fg = torch.tensor(fh, device=dev())
    ph = pl.solve_spectral(fg).cpu().numpy()
    ref = O.solve_spectral(torch.tensor(fh).permute(1, 2, 0), box).permute(2, 0, 1).numpy()
    err = np.abs(ph - ref).max(axis=1) / np.abs(ref).max(axis=1)      # per (kx, kz) line
    assert err.max() <= 1e-11, f"worst line {np.unravel_index(err.argmax(), err.shape)}: {err.max():.3e}"
    # in place
    ph2 = pl.solve_spectral(fg, out=fg).cpu().numpy()
    assert np.array_equal(ph2, ph)


def _dropped_lines(info, k2, nz):
    """Lines (kx, kz) the kernel drops: blocks of lines_per_block consecutive
    lines (line = kx * nz + kz) lying wholly above the plan's threshold."""
    flat = k2.reshape(-1)                         # (nkx * nz,), line order
    lb = info["lines_per_block"]
    ok = np.zeros(flat.size, dtype=bool)
    for b0 in range(0, flat.size, lb):
        blk = flat[b0:b0 + lb]
        ok[b0:b0 + lb] = bool((blk >= info["k2_threshold"]).all())
    return ok


def test_drop_path_matches_oracle_pdd():
    """A plan with four partitions and a loose tolerance drops the corner terms
    on high-wavenumber lines.  The kernel decides per block of consecutive
    lines: a block drops only if all its lines may.  The lines it drops (as
    many as the plan reports) equal the oracle's dropped PDD, and differ from
    the exact solve by no more than a small multiple of their corner terms
    delta; every other line equals the exact solve."""
    nx, ny, nz = 64, 64, 64
    pl, box = plan_for(nx, ny, nz, 2.0, n_parts=4, drop_tol=1e-5)
    info = pl.info()
    assert info["drop_parts"] == 4
    assert 0 < info["n_drop_lines"] < info["n_lines"]
    rng = np.random.default_rng(4)
    fh = rng.standard_normal((nx // 2 + 1, ny, nz)) + 1j * rng.standard_normal((nx // 2 + 1, ny, nz))
    ph = pl.solve_spectral(torch.tensor(fh, device=dev())).cpu().numpy()      # (nkx, ny, nz)
    a, c, k2 = O.line_coefficients(box)
    k2 = k2.numpy().T.copy()                                                  # (nkx, nz)
    drop = _dropped_lines(info, k2, nz).reshape(k2.shape)
    assert drop.sum() == info["n_dropped_lines"] > 0
    # the singular kx = kz = 0 line (never in a dropping block) takes its gauge
    mean = O.solve_mean_line(torch.tensor(fh[0, :, 0]), box).numpy()
    assert np.abs(ph[0, :, 0] - mean).max() <= 1e-11 * np.abs(mean).max()
    for want_drop in (True, False):
        sel = np.argwhere(drop == want_drop)
        sel = sel[(sel[:, 0] > 0) | (sel[:, 1] > 0)]
        b = -(a + c)[:, None] - torch.tensor(k2[sel[:, 0], sel[:, 1]])[None, :]
        d = torch.tensor(np.ascontiguousarray(fh[sel[:, 0], :, sel[:, 1]].T))  # (ny, lines)
        got = ph[sel[:, 0], :, sel[:, 1]].T
        ref_exact = O.thomas(a[:, None], b, c[:, None], d).numpy()
        scale = np.abs(ref_exact).max(0)
        e_exact = np.abs(got - ref_exact).max(0) / scale
        if want_drop:
            ref_drop = O.pdd_solve(a, b, c, d, 4, drop=True).numpy()
            assert (np.abs(got - ref_drop).max(0) / scale).max() <= 1e-11
            delta = O.pdd_indicator(a, b, c, 4).numpy()
            assert (delta <= 1e-5).all()
            assert (e_exact <= 50 * delta + 1e-11).all()
            assert e_exact.max() > 1e-11          # the drop is visible on some lines
        else:
            assert e_exact.max() <= 1e-11


def test_grouped_drop_on_the_step_grid():
    """The 1024x256x512 step grid at the default drop tolerance (1e-15): the
    dropped reduced system is an outer PDD of 4 groups of 4 partitions (64 rows
    each), whose corner terms fall below 1e-15 for most wavenumbers, so most
    lines take the dropped 2x2 step.  Every line matches the exact solve
    (Thomas) to 1e-11, and sampled dropped lines match the oracle's dropped PDD
    of the same 4 partitions; with drop_tol = 0 nothing is dropped and the
    result agrees."""
    wl = synth.WORKLOADS["step550"]
    pl, box = plan_for(wl.nx, wl.ny, wl.nz, wl.gamma, lx=wl.lx, lz=wl.lz)
    info = pl.info()
    assert info["n_parts"] == 16 and info["drop_parts"] == 4
    assert info["n_dropped_lines"] > 0.9 * info["n_lines"]
    print(f"step grid: {info['n_drop_lines']} lines above k2 = {info['k2_threshold']:.1f}, "
          f"{info['n_dropped_lines']} of {info['n_lines']} dropped")
    rng = np.random.default_rng(8)
    shape = (pl.nkx, wl.ny, wl.nz)
    fh = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    fh[0, :, 0].imag = 0.0
    fg = torch.tensor(fh, device=dev())
    ph = pl.solve_spectral(fg).cpu().numpy()
    ref = O.solve_spectral(torch.tensor(fh).permute(1, 2, 0), box).permute(2, 0, 1).numpy()
    err = np.abs(ph - ref).max(axis=1) / np.abs(ref).max(axis=1)
    print(f"step grid, dropped reduced system: worst line error vs Thomas {err.max():.3e}")
    assert err.max() <= 1e-11
    a, c, k2 = O.line_coefficients(box)
    k2 = k2.numpy().T.copy()
    drop = _dropped_lines(info, k2, wl.nz).reshape(k2.shape)
    assert drop.sum() == info["n_dropped_lines"]
    sel = np.argwhere(drop)[rng.choice(int(drop.sum()), 256, replace=False)]
    b = -(a + c)[:, None] - torch.tensor(k2[sel[:, 0], sel[:, 1]])[None, :]
    d = torch.tensor(np.ascontiguousarray(fh[sel[:, 0], :, sel[:, 1]].T))
    ref_drop = O.pdd_solve(a, b, c, d, 4, drop=True).numpy()
    got = ph[sel[:, 0], :, sel[:, 1]].T
    assert (np.abs(got - ref_drop).max(0) / np.abs(ref_drop).max(0)).max() <= 1e-11
    assert (O.pdd_indicator(a, b, c, 4).numpy() <= 1e-15).all()
    exact, _ = plan_for(wl.nx, wl.ny, wl.nz, wl.gamma, lx=wl.lx, lz=wl.lz, drop_tol=0.0)
    assert exact.info()["n_dropped_lines"] == 0
    pe = exact.solve_spectral(fg).cpu().numpy()
    assert (np.abs(pe - ref).max(axis=1) / np.abs(ref).max(axis=1)).max() <= 1e-11


@pytest.mark.parametrize("nx,ny,nz,gamma,parts", CASES)
def test_poisson_solve_matches_oracle(nx, ny, nz, gamma, parts):
    pl, box = plan_for(nx, ny, nz, gamma, parts)
    u, v, w = synth.uniform_velocity(nx, ny, nz, seed=0)
    ug, vg, wg = (torch.tensor(q, device=dev()) for q in (u, v, w))
    fg = pl.divergence(ug, vg, wg)
    f_ref = O.divergence(*(torch.tensor(q) for q in (u, v, w)), box)
    assert (fg.cpu() - f_ref).abs().max() <= 1e-12 * f_ref.abs().max()
    pg = pl.poisson_solve(fg).cpu().numpy()
    p_ref = O.poisson(f_ref, box).numpy()
    assert rel(pg, p_ref) <= 1e-12
    # aliasing p = f is allowed
    pg2 = pl.poisson_solve(fg, out=fg).cpu().numpy()
    assert np.array_equal(pg2, pg)


@pytest.mark.parametrize("ny,precision", [(1024, "fp64"), (1023, "fp64"), (2048, "mixed"), (2047, "mixed")])
def test_largest_wall_normal_sizes(ny, precision):
    """The largest ny each precision takes (64 partitions of 16 rows in FP64,
    of 32 in mixed precision), and one row fewer (the last partition padded),
    on a thin x-z grid: the Poisson solve against the oracle.  The bounds grow
    with ny because the conditioning of the lowest wall-normal modes does: in
    FP64 5e-12 instead of the 1e-12 of ny <= 256 (per line, two correct FP64
    solvers differ by about 2e-11 at ny = 1024 and k^2 = 0.25; measured field
    rel-L2 1.9e-12); in mixed precision one refinement pass reaches 1.3e-6 at
    ny = 2048 (bound 3e-6) and a second pass brings it below 1e-6."""
    nx, nz = 8, 6
    mk = lambda **kw: plan_for(nx, ny, nz, 2.0, precision=precision, **kw)  # noqa: E731
    pl, box = mk()
    info = pl.info()
    assert info["n_parts"] == 64 and info["rows_per_part"] == (16 if precision == "fp64" else 32)
    f = synth.uniform_rhs(nx, ny, nz, seed=7)
    ref = O.poisson(torch.tensor(f), box).numpy()
    e1 = rel(pl.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy(), ref)
    if precision == "fp64":
        assert e1 <= 5e-12
    else:
        e2 = rel(mk(refine_passes=2)[0].poisson_solve(torch.tensor(f, device=dev())).cpu().numpy(), ref)
        print(f"mixed ny={ny}: rel-L2 one pass {e1:.3e}, two passes {e2:.3e}")
        assert e1 <= 3e-6 and e2 <= 1e-6 and e2 < e1


def test_poisson_64cubed_config_and_determinism():
    wl = synth.WORKLOADS["poisson64"]
    pl, box = plan_for(wl.nx, wl.ny, wl.nz, wl.gamma, lx=wl.lx, lz=wl.lz)
    f = synth.uniform_rhs(wl.nx, wl.ny, wl.nz, seed=0)
    fg = torch.tensor(f, device=dev())
    p1 = pl.poisson_solve(fg)
    p2 = pl.poisson_solve(fg)
    assert torch.equal(p1, p2)
    p_ref = O.poisson(torch.tensor(f), box).numpy()
    assert rel(p1.cpu().numpy(), p_ref) <= 1e-12
    # gauge and residual
    pc = torch.tensor(p1.cpu().numpy())
    assert abs(O.mean_w(pc, box).item()) < 1e-14
    r = O.laplacian_p(pc, box) - (torch.tensor(f) - O.mean_w(torch.tensor(f), box))
    assert r.abs().max() <= 1e-10 * torch.tensor(f).abs().max()


def test_empty_stream_and_plan_reuse():
    """Two plans live at once and alternate on the same stream."""
    pa, ba = plan_for(32, 16, 8, 2.0)
    pb, bb = plan_for(64, 32, 24, 2.5)
    for _ in range(2):
        for pl, box in ((pa, ba), (pb, bb)):
            f = synth.uniform_rhs(box.nx, box.ny, box.nz, seed=5)
            p = pl.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy()
            assert rel(p, O.poisson(torch.tensor(f), box).numpy()) <= 1e-12


def test_bad_tensor_arguments_rejected():
    pl, box = plan_for(32, 16, 8, 2.0)
    f = torch.zeros(16, 8, 32, dtype=torch.float64, device=dev())
    with pytest.raises(TypeError):
        pl.poisson_solve(f.float())
    with pytest.raises(ValueError):
        pl.poisson_solve(f[:, :, :16])
    with pytest.raises(ValueError):
        pl.poisson_solve(f.transpose(1, 2).contiguous().transpose(1, 2))


def test_overlapping_outputs_of_other_entry_points_rejected():
    """The divergence's output inside a velocity array, a spectral solve's
    output overlapping its input at another offset, and plane statistics
    written into the field they average are refused (CF_ERR_ARG)."""
    from paper_2104_08863_amd._lib import ChanflowError
    nx, ny, nz = 32, 16, 8
    pl, box = plan_for(nx, ny, nz, 2.0)
    u, v, w = (torch.tensor(q, device=dev()) for q in synth.uniform_velocity(nx, ny, nz, seed=1))
    with pytest.raises(ChanflowError):
        pl.divergence(u, v, w, out=v)
    fh = pl.forward_spectral(pl.divergence(u, v, w))
    n = fh.numel()
    buf = torch.zeros(2 * n, dtype=fh.dtype, device=dev())
    buf[:n].copy_(fh.reshape(-1))
    a = buf[:n].view(fh.shape)
    with pytest.raises(ChanflowError):
        pl.solve_spectral(a, out=buf[1:n + 1].view(fh.shape))
    assert torch.equal(pl.solve_spectral(a, out=a), pl.solve_spectral(fh))   # in place is fine
    with pytest.raises(ChanflowError):
        pl.plane_stats(u, v, w, out=u.view(-1)[:ny * 6].view(ny, 6))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_partially_overlapping_output_rejected(precision):
    """p may be f itself, but an output that overlaps f at another offset is
    refused before anything runs (a mixed solve reads f again after writing
    p), and f is left untouched."""
    from paper_2104_08863_amd._lib import ChanflowError
    nx, ny, nz = 32, 16, 8
    pl, box = plan_for(nx, ny, nz, 2.0, precision=precision)
    n = nx * ny * nz
    buf = torch.zeros(2 * n, dtype=torch.float64, device=dev())
    f = buf[:n].view(ny, nz, nx)
    f.copy_(torch.tensor(synth.uniform_rhs(nx, ny, nz, seed=5), device=dev()))
    keep = f.clone()
    for off in (2, n // 2, n - 2):
        with pytest.raises(ChanflowError):
            pl.poisson_solve(f, out=buf[off:off + n].view(ny, nz, nx))
    assert torch.equal(f, keep)
    p = pl.poisson_solve(f, out=buf[n:].view(ny, nz, nx))   # disjoint: fine
    q = pl.poisson_solve(f.clone())
    assert torch.equal(p, q)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_non_finite_right_hand_side_is_reported(precision):
    """A NaN or an infinity anywhere in f reaches the kx = kz = 0 line of its
    plane; the solve flags it and cf_plan_numeric_status returns CF_ERR_NUMERIC
    once (the flag is cleared), while clean solves report nothing."""
    pl, box = plan_for(32, 16, 24, 2.0, precision=precision)
    f = torch.tensor(synth.uniform_rhs(32, 16, 24, seed=4), device=dev())
    pl.poisson_solve(f)
    assert pl.numeric_status()
    for j, k, i, bad in [(7, 3, 11, float("nan")), (15, 23, 31, float("inf")), (0, 0, 0, -float("inf"))]:
        g = f.clone()
        g[j, k, i] = bad
        pl.poisson_solve(g)
        assert not pl.numeric_status(), (j, k, i, bad)
        assert pl.numeric_status()      # cleared by the read
    pl.poisson_solve(f)
    assert pl.numeric_status()
