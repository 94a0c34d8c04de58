"""The kernels' per-thread math (Stockham passes, real<->half-complex steps,
PDD partition and reduced-system solves), run on the CPU through the host
build of the same headers, against numpy's FFT and the FP64 oracle."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_2104_08863_amd import _lib as L
from paper_2104_08863_amd import synth

LENS = [2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048]


def P(a):
    return C.c_void_p(a.ctypes.data)


@pytest.fixture(scope="module")
def H():
    return L.hostlib()


@pytest.mark.parametrize("n", LENS)
@pytest.mark.parametrize("fp32", [0, 1])
def test_c2c_matches_numpy(H, n, fp32):
    rng = np.random.default_rng(n)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    zi = np.ascontiguousarray(np.stack([z.real, z.imag], -1).reshape(-1))
    out = np.zeros(2 * n)
    tol = 3e-6 if fp32 else 1e-14
    for inv, ref in ((0, np.fft.fft(z)), (1, np.fft.ifft(z) * n)):
        assert H.cfh_fft_c2c(n, inv, fp32, P(zi), P(out)) == 0
        got = out[0::2] + 1j * out[1::2]
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max() * max(1.0, np.log2(n))


@pytest.mark.parametrize("nx", [4, 6, 8, 12, 24, 64, 96, 256, 1024, 3072, 4096])
@pytest.mark.parametrize("fp32", [0, 1])
def test_real_transform_pair(H, nx, fp32):
    rng = np.random.default_rng(nx)
    x = rng.standard_normal(nx)
    X = np.zeros(2 * (nx // 2 + 1))
    assert H.cfh_rfft(nx, fp32, P(x), P(X)) == 0
    ref = np.fft.rfft(x)
    got = X[0::2] + 1j * X[1::2]
    tol = 3e-6 if fp32 else 1e-14
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max() * np.log2(nx)
    # inverse: feed the exact spectrum with junk imaginary parts on DC/Nyquist
    R = np.stack([ref.real, ref.imag], -1).reshape(-1).copy()
    R[1] = 5.0
    R[-1] = -3.0
    back = np.zeros(nx)
    assert H.cfh_irfft(nx, fp32, P(R), P(back)) == 0
    assert np.abs(back - x).max() <= tol * 10 * np.abs(x).max()


def _line_system(ny, gamma, k2):
    box = O.Box(8, ny, 8, 2 * np.pi, np.pi, synth.tanh_faces(ny, gamma))
    a, c = O.y_coefficients(box)
    return a.numpy().copy(), c.numpy().copy()


@pytest.mark.parametrize("ny,Pn", [(16, 1), (24, 2), (64, 4), (64, 16), (256, 16), (48, 4), (96, 8),
                                   (768, 64), (36, 3), (60, 5), (16, 16)])
@pytest.mark.parametrize("k2", [0.25, 7.0, 3000.0])
def test_pdd_exact_matches_thomas(H, ny, Pn, k2):
    a, c = _line_system(ny, 2.5, k2)
    rng = np.random.default_rng(ny + Pn)
    d = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    di = np.ascontiguousarray(np.stack([d.real, d.imag], -1).reshape(-1))
    x = np.zeros(2 * ny)
    assert H.cfh_pdd_line(ny, Pn, P(a), P(c), k2, 1, 0, P(di), P(x)) == 0
    got = x[0::2] + 1j * x[1::2]
    b = -(a + c) - k2
    ref = O.thomas(torch.tensor(a), torch.tensor(b), torch.tensor(c), torch.tensor(d)).numpy()
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("ny,Pn", [(130, 11), (97, 13), (250, 16), (7, 2), (1000, 63), (61, 8)])
@pytest.mark.parametrize("k2", [0.25, 7.0, 3000.0])
def test_padded_partitions_match_thomas(H, ny, Pn, k2):
    """ny not a multiple of P: partitions of M = ceil(ny/P) rows, the last one
    completed by zero rows (a = c = 0, zero right-hand side) past the wall row.
    The exact PDD (cyclic reduction of the reduced system) and the one-group
    grouped form both reproduce Thomas on the ny real rows (to a bound that
    grows with ny: the low-k^2 lines' conditioning, the same with and without
    padding, e.g. 1.4e-11 relative at ny = 1000 and 2.3e-11 at ny = 1008 = 63*16
    for k^2 = 0.25)."""
    tol = max(1e-11, 5e-14 * ny)
    a, c = _line_system(ny, 2.5, k2)
    rng = np.random.default_rng(ny * Pn)
    d = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    di = np.ascontiguousarray(np.stack([d.real, d.imag], -1).reshape(-1))
    b = -(a + c) - k2
    ref = O.thomas(torch.tensor(a), torch.tensor(b), torch.tensor(c), torch.tensor(d)).numpy()
    x = np.zeros(2 * ny)
    assert H.cfh_pdd_line(ny, Pn, P(a), P(c), k2, 1, 0, P(di), P(x)) == 0
    got = x[0::2] + 1j * x[1::2]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    x[:] = 0
    assert H.cfh_pdd_line_grouped(ny, Pn, 1, P(a), P(c), k2, 0, P(di), P(x)) == 0
    got = x[0::2] + 1j * x[1::2]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()


@pytest.mark.parametrize("ny,Pn", [(17, 16), (100, 64), (5, 4)])
def test_partitionings_with_an_empty_part_are_rejected(H, ny, Pn):
    """(P-1) * ceil(ny/P) >= ny leaves the last partition without a row of the
    line (only padding): such a partitioning is refused."""
    a, c = _line_system(max(ny, 2), 2.5, 1.0)
    di = np.zeros(2 * ny)
    x = np.zeros(2 * ny)
    assert H.cfh_pdd_line(ny, Pn, P(a), P(c), 1.0, 1, 0, P(di), P(x)) == 1


@pytest.mark.parametrize("ny,Pn", [(64, 4), (256, 16), (96, 8)])
def test_pdd_drop_matches_oracle_pdd(H, ny, Pn):
    a, c = _line_system(ny, 2.0, 0)
    rng = np.random.default_rng(3)
    for k2 in (1.0, 50.0, 5e4):
        d = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
        di = np.ascontiguousarray(np.stack([d.real, d.imag], -1).reshape(-1))
        x = np.zeros(2 * ny)
        assert H.cfh_pdd_line(ny, Pn, P(a), P(c), k2, 0, 0, P(di), P(x)) == 0
        got = x[0::2] + 1j * x[1::2]
        b = torch.tensor(-(a + c) - k2)[:, None]
        ref = O.pdd_solve(torch.tensor(a), b, torch.tensor(c), torch.tensor(d)[:, None], Pn,
                          drop=True)[:, 0].numpy()
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_pdd_fp32_close_to_thomas_at_high_k(H):
    ny, Pn, k2 = 256, 16, 2e4
    a, c = _line_system(ny, 2.5, k2)
    rng = np.random.default_rng(9)
    d = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    di = np.ascontiguousarray(np.stack([d.real, d.imag], -1).reshape(-1))
    x = np.zeros(2 * ny)
    assert H.cfh_pdd_line(ny, Pn, P(a), P(c), k2, 1, 1, P(di), P(x)) == 0
    got = x[0::2] + 1j * x[1::2]
    b = -(a + c) - k2
    ref = O.thomas(torch.tensor(a), torch.tensor(b), torch.tensor(c), torch.tensor(d)).numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("ny,Pn,G", [(256, 16, 4), (256, 16, 2), (256, 16, 16), (128, 8, 4), (192, 12, 3),
                                     (96, 8, 8), (64, 4, 1)])
def test_grouped_drop_matches_oracle_pdd_of_the_groups(H, ny, Pn, G):
    """The y kernel's dropped reduced system taken as an outer PDD of G groups
    of Pn/G partitions (exact inside each group) is the paper's dropped PDD
    with G partitions: it matches the oracle's pdd_solve(p=G, drop=True) at
    every k^2, low wavenumbers (where the drop is far from exact) included,
    and Thomas where the G-level corner terms are below round-off."""
    a, c = _line_system(ny, 2.5, 0)
    rng = np.random.default_rng(ny + Pn + G)
    for k2 in (0.3, 30.0, 3e3, 5e4):
        d = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
        di = np.ascontiguousarray(np.stack([d.real, d.imag], -1).reshape(-1))
        x = np.zeros(2 * ny)
        assert H.cfh_pdd_line_grouped(ny, Pn, G, P(a), P(c), k2, 0, P(di), P(x)) == 0
        got = x[0::2] + 1j * x[1::2]
        b = torch.tensor(-(a + c) - k2)[:, None]
        ref = O.pdd_solve(torch.tensor(a), b, torch.tensor(c), torch.tensor(d)[:, None], G,
                          drop=True)[:, 0].numpy()
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), k2
        delta = float(O.pdd_indicator(torch.tensor(a), b, torch.tensor(c), G)[0])
        th = O.thomas(torch.tensor(a), b[:, 0], torch.tensor(c), torch.tensor(d)).numpy()
        if delta < 1e-15:
            assert np.abs(got - th).max() <= 1e-11 * np.abs(th).max(), k2


@pytest.mark.parametrize("n,groups", [(8, 1), (64, 3), (2048, 8), (8192, 2), (24, 5), (12, 4), (7, 3)])
def test_xcd_work_order_is_a_permutation_in_runs(H, n, groups):
    """The block -> work item map of the row-block and stencil-tile launches:
    a permutation of the grid; for n a multiple of 8 the blocks one XCD
    receives (b mod 8 = x) take, in launch order, the contiguous run
    [x n/8, (x+1) n/8) of each group of n items in turn; otherwise the identity."""
    nb = n * groups
    got = [H.cfh_xcd_slab_block(b, n) for b in range(nb)]
    assert sorted(got) == list(range(nb))
    if n % 8:
        assert got == list(range(nb))
        return
    per = n // 8
    for x in range(8):
        items = got[x::8]
        assert items == [g * n + x * per + s for g in range(groups) for s in range(per)]
