"""Partition count and block shape chosen by measurement (CF_PLAN_TUNE_PARTS):
the candidates timed are exactly the admissible ones, the plan keeps the
fastest, and the tuned plan solves to the same bar against the FP64 oracle and
bitwise like a plan given that partitioning explicitly."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2104_08863_amd import synth

pytestmark = pytest.mark.gpu

M_SET = (1, 2, 3, 4, 6, 8, 12, 16)
M_SET_FP32 = M_SET + (24, 32)   # mixed precision also compiles longer partitions


def dev():
    return torch.device("cuda", 0)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def admissible(ny, mixed=False):
    """(P, lines per block) candidates: P partitions that divide ny into a
    compiled row count; if none does, P partitions of ceil(ny/P) compiled rows
    with every partition holding a row of the line (the last one padded)."""
    ms = M_SET_FP32 if mixed else M_SET
    ps = [P for P in range(1, 65) if ny % P == 0 and ny // P in ms]
    if not ps:
        ps = [P for P in range(1, 65) if -(-ny // P) in ms and (P - 1) * -(-ny // P) < ny]
    return {(P, lb) for P in ps for lb in (4, 8, 16, 32, 64, 128, 256) if 64 <= lb * P <= 512}


def make(nx, ny, nz, gamma, **kw):
    from paper_2104_08863_amd.api import Plan
    yf = synth.tanh_faces(ny, gamma)
    return Plan(nx, ny, nz, 2 * np.pi, np.pi, yf, **kw), O.Box(nx, ny, nz, 2 * np.pi, np.pi, yf)


@pytest.mark.parametrize("nx,ny,nz,gamma", [(128, 96, 64, 2.0), (64, 256, 48, 2.5), (96, 36, 24, 2.5)])
def test_tuned_partitioning_fp64(nx, ny, nz, gamma):
    pl, box = make(nx, ny, nz, gamma, tune_parts=True)
    rows = pl.partition_timings()
    got = {(P, lb) for P, lb, _ in rows}
    assert len(rows) == len(got)
    assert got <= admissible(ny) and len(got) >= 2
    assert all(us > 0 for _, _, us in rows)
    info = pl.info()
    best = min(rows, key=lambda r: r[2])
    assert (info["n_parts"], info["lines_per_block"]) == best[:2]
    assert info["rows_per_part"] * info["n_parts"] == ny   # a partitioning that divides ny exists
    f = synth.uniform_rhs(nx, ny, nz, seed=3)
    p = pl.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy()
    p_ref = O.poisson(torch.tensor(f), box).numpy()
    assert rel(p, p_ref) <= 1e-12
    same, _ = make(nx, ny, nz, gamma, n_parts=best[0], lines_per_block=best[1])
    assert same.partition_timings() == []
    q = same.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy()
    assert np.array_equal(p, q)


def test_tuned_partitioning_padded():
    """ny = 130 has no partitioning into a compiled row count: the candidates
    are the padded ones (M = ceil(130/P)), and the tuned plan meets the
    oracle."""
    nx, ny, nz = 64, 130, 32
    pl, box = make(nx, ny, nz, 2.5, tune_parts=True)
    rows = pl.partition_timings()
    got = {(P, lb) for P, lb, _ in rows}
    assert got <= admissible(ny) and len(got) >= 2
    info = pl.info()
    assert (info["n_parts"], info["lines_per_block"]) == min(rows, key=lambda r: r[2])[:2]
    M, Pn = info["rows_per_part"], info["n_parts"]
    assert (Pn - 1) * M < ny < Pn * M
    f = synth.uniform_rhs(nx, ny, nz, seed=6)
    p = pl.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy()
    assert rel(p, O.poisson(torch.tensor(f), box).numpy()) <= 1e-12


@pytest.mark.parametrize("lb", [4, 8, 16, 32])
def test_explicit_lines_per_block(lb):
    """Any block shape gives the oracle's solution (the block only decides,
    for lines above the drop threshold, whether the corner terms are dropped)."""
    nx, ny, nz = 64, 128, 48
    pl, box = make(nx, ny, nz, 2.0, n_parts=16, lines_per_block=lb)
    assert pl.info()["lines_per_block"] == lb
    f = synth.uniform_rhs(nx, ny, nz, seed=4)
    p = pl.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy()
    assert rel(p, O.poisson(torch.tensor(f), box).numpy()) <= 1e-12


def test_tuned_partitioning_mixed():
    nx, ny, nz = 128, 192, 96
    pl, box = make(nx, ny, nz, 2.0, precision="mixed", tune_parts=True)
    rows = pl.partition_timings()
    got = {(P, lb) for P, lb, _ in rows}
    assert got <= admissible(ny, mixed=True)
    assert any(ny // P > 16 for P, _ in got)      # the FP32-only 24- and 32-row partitions are candidates
    info = pl.info()
    assert (info["n_parts"], info["lines_per_block"]) == min(rows, key=lambda r: r[2])[:2]
    f = synth.uniform_rhs(nx, ny, nz, seed=5)
    p = pl.poisson_solve(torch.tensor(f, device=dev())).cpu().numpy()
    assert rel(p, O.poisson(torch.tensor(f), box).numpy()) <= 1e-6


def test_tuning_rejects_conflicting_options():
    from paper_2104_08863_amd._lib import ChanflowError
    with pytest.raises(ChanflowError):
        make(64, 64, 32, 2.0, tune_parts=True, n_parts=4)
    with pytest.raises(ChanflowError):
        make(64, 64, 32, 2.0, tune_parts=True, lines_per_block=16)
    with pytest.raises(ChanflowError):
        make(64, 64, 32, 2.0, n_parts=16, lines_per_block=64)     # 1024 threads
