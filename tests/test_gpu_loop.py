"""The time loop (cf_run_steps, eager and replayed from HIP graphs) and the
plane statistics (cf_plane_stats) against single steps and the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2104_08863_amd import synth

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda", 0)


def setup(nx, ny, nz, gamma, precision="fp64"):
    from paper_2104_08863_amd.api import Plan
    yf = synth.tanh_faces(ny, gamma)
    pl = Plan(nx, ny, nz, 2 * np.pi, np.pi, yf, precision=precision, step=True)
    return pl, O.Box(nx, ny, nz, 2 * np.pi, np.pi, yf)


def state(pl, box, seed, dtype=torch.float64):
    return [torch.tensor(q, device=dev()).to(dtype)
            for q in synth.perturbed_poiseuille(pl.nx, pl.ny, pl.nz, box.y_faces, seed=seed)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_plane_stats_matches_oracle(precision):
    pl, box = setup(96, 70, 24, 2.0, precision)
    u, v, w = state(pl, box, 1, pl.state_dtype)
    got = pl.plane_stats(u, v, w)
    ref = O.plane_stats(*(t.cpu().double() for t in (u, v, w)))
    assert float((got.cpu() - ref).abs().max() / ref.abs().max()) <= 1e-14
    assert torch.equal(got, pl.plane_stats(u, v, w))   # fixed reduction order


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_run_steps_equals_single_steps_and_accumulates_stats(precision):
    pl, box = setup(64, 48, 32, 2.0, precision)
    dt, nu = 1e-3, 1 / 550
    u, v, w = state(pl, box, 2, pl.state_dtype)
    ref = [t.clone() for t in (u, v, w)]
    ref_stats = torch.zeros(pl.ny, 6, dtype=torch.float64, device=dev())
    for k in range(5):
        ref = list(pl.projection_step(*ref, dt, nu, 3 * nu))
        if (k + 1) % 2 == 0:
            ref_stats += O.plane_stats(*(t.cpu().double() for t in ref)).to(dev())
    a = [t.clone() for t in (u, v, w)]
    work = tuple(torch.empty_like(t) for t in a)
    stats = torch.zeros(pl.ny, 6, dtype=torch.float64, device=dev())
    out = pl.run_steps(*a, 5, dt, nu, 3 * nu, work=work, stats_every=2, stats=stats)
    assert all(x.data_ptr() == y.data_ptr() for x, y in zip(out, work))   # odd count ends in work
    for x, y in zip(out, ref):
        assert torch.equal(x, y)
    assert float((stats - ref_stats).abs().max() / ref_stats.abs().max()) <= 1e-14


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager(precision):
    """The graph mode gives the eager result bitwise; the call is repeated with
    eager work and synchronisation between, and every repetition is checked."""
    pl, box = setup(64, 48, 32, 2.5, precision)
    dt, nu = 1e-3, 1 / 550
    u, v, w = state(pl, box, 3, pl.state_dtype)
    e = [t.clone() for t in (u, v, w)]
    ew = tuple(torch.empty_like(t) for t in e)
    es = torch.zeros(pl.ny, 6, dtype=torch.float64, device=dev())
    eager = pl.run_steps(*e, 4, dt, nu, 3 * nu, work=ew, stats_every=3, stats=es)
    for rep in range(3):
        g = [t.clone() for t in (u, v, w)]
        gw = tuple(torch.empty_like(t) for t in g)
        gs = torch.zeros(pl.ny, 6, dtype=torch.float64, device=dev())
        got = pl.run_steps(*g, 4, dt, nu, 3 * nu, work=gw, stats_every=3, stats=gs, use_graph=True)
        torch.cuda.synchronize()
        for x, y in zip(got, eager):
            assert torch.equal(x, y), f"repetition {rep}"
        assert torch.equal(gs, es), f"repetition {rep}"
        # eager work between the repetitions
        pl.projection_step(*(t.clone() for t in (u, v, w)), dt, nu, 3 * nu)
        torch.cuda.synchronize()
    # odd step count, no statistics
    g = [t.clone() for t in (u, v, w)]
    gw = tuple(torch.empty_like(t) for t in g)
    got = pl.run_steps(*g, 3, dt, nu, 3 * nu, work=gw, use_graph=True)
    e = [t.clone() for t in (u, v, w)]
    want = pl.run_steps(*e, 3, dt, nu, 3 * nu, work=tuple(torch.empty_like(t) for t in e))
    for x, y in zip(got, want):
        assert torch.equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nsteps", [1, 2, 5])
@pytest.mark.parametrize("use_graph", [False, True])
def test_loop_without_stats_equals_single_steps(precision, nsteps, use_graph):
    """Without statistics, eager and from graphs: the states and the last
    pressure equal those of single projection steps bitwise (ragged tile
    edges: 96 x 70 x 24)."""
    pl, box = setup(96, 70, 24, 2.0, precision)
    dt, nu = 1e-3, 1 / 550
    u, v, w = state(pl, box, 6, pl.state_dtype)
    ref = [t.clone() for t in (u, v, w)]
    p_ref = torch.empty(pl.ny, pl.nz, pl.nx, dtype=torch.float64, device=dev())
    for _ in range(nsteps):
        ref = list(pl.projection_step(*ref, dt, nu, 3 * nu, p=p_ref))
    a = [t.clone() for t in (u, v, w)]
    p = torch.empty_like(p_ref)
    out = pl.run_steps(*a, nsteps, dt, nu, 3 * nu, p=p, use_graph=use_graph)
    torch.cuda.synchronize()
    for x, y, n in zip(out, ref, "uvw"):
        assert torch.equal(x, y), n
    assert torch.equal(p, p_ref)


def test_run_steps_rejects_overlapping_state_sets():
    from paper_2104_08863_amd._lib import ChanflowError
    pl, box = setup(32, 16, 24, 2.0)
    u, v, w = state(pl, box, 4)
    with pytest.raises(ChanflowError):
        pl.run_steps(u, v, w, 2, 1e-3, 1 / 550, 3 / 550, work=(v, u, w))
    with pytest.raises(ChanflowError):
        pl.run_steps(u, v, w, -1, 1e-3, 1 / 550, 3 / 550)


def test_graph_cache_eviction_and_pressure_output():
    """More distinct (arrays, parameters) sets than the plan keeps recorded
    steps for: entries are dropped and re-recorded, results stay equal to the
    eager loop; the optional pressure output receives the last step's p."""
    pl, box = setup(32, 16, 24, 2.0)
    dt, nu = 1e-3, 1 / 550
    u, v, w = state(pl, box, 5)
    for rep in range(2):
        for k in range(6):                       # 6 parameter sets x 2 parities > 8 entries
            g = [t.clone() for t in (u, v, w)]
            gw = tuple(torch.empty_like(t) for t in g)
            got = pl.run_steps(*g, 2, dt * (1 + 0.1 * k), nu, 3 * nu, work=gw, use_graph=True)
            e = [t.clone() for t in (u, v, w)]
            want = pl.run_steps(*e, 2, dt * (1 + 0.1 * k), nu, 3 * nu, work=tuple(torch.empty_like(t) for t in e))
            for x, y in zip(got, want):
                assert torch.equal(x, y), f"rep {rep} set {k}"
    p = torch.empty_like(u)
    a = [t.clone() for t in (u, v, w)]
    out = pl.run_steps(*a, 3, dt, nu, 3 * nu, p=p)
    b = [t.clone() for t in (u, v, w)]
    for _ in range(2):
        b = list(pl.projection_step(*b, dt, nu, 3 * nu))
    p_ref = torch.empty_like(u)
    b = pl.projection_step(*b, dt, nu, 3 * nu, p=p_ref)
    assert torch.equal(p, p_ref)
    for x, y in zip(out, b):
        assert torch.equal(x, y)
