"""Pins of the oracle's Lambda* (the 27-point band of Lambda, built along the lines).

Lambda is pinned by brute force: column u of Lambda is the mean intensity of a unit source in voxel
u alone with no boundary light.  Lambda* must equal that band exactly, including on grids so small
that shallow lines wrap around inside one layer.  Independently of the oracle, Lambda obeys
reciprocity chi_v Lambda_vu = chi_u Lambda_uv (lines for Omega and -Omega coincide and the weights
are symmetric), is non-negative, and its rows sum to J(S = 1) < 1; Lambda*_vv tends to 1 in very
thick voxels.
"""
import numpy as np
import pytest

from paper_1107_5719_amd.inputs import random_medium


def _band_from_dense(Lam, shape):
    nz, ny, nx = shape
    V = nx * ny * nz
    out = np.zeros((27, V))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                v = (k * ny + j) * nx + i
                for dk in (-1, 0, 1):
                    if not 0 <= k + dk < nz:
                        continue
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            o = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1)
                            u = ((k + dk) * ny + (j + dj) % ny) * nx + (i + di) % nx
                            out[o, v] = Lam[v, u]
    return out


@pytest.mark.parametrize("shape,nt,nph,seed", [((5, 5, 5), 8, 8, 1), ((7, 5, 6), 8, 8, 2),
                                                ((4, 3, 3), 16, 16, 3), ((5, 4, 3), 2, 4, 4)])
def test_lstar_equals_bruteforce_band(orc, shape, nt, nph, seed):
    nz, ny, nx = shape
    m = random_medium(nx, ny, nz, seed=seed, chi_range=(1e-2, 1e1))
    Lam = orc.lambda_bruteforce(m["chi"], nt, nph)
    L = orc.lstar(m["chi"], nt, nph).reshape(27, -1)
    ref = _band_from_dense(Lam, shape)
    assert np.max(np.abs(L - ref)) < 1e-12


def test_reciprocity_and_structure(orc):
    m = random_medium(5, 5, 6, seed=5, chi_range=(1e-3, 1e2))
    chi = m["chi"].ravel()
    Lam = orc.lambda_bruteforce(m["chi"], 8, 8)
    R = chi[:, None] * Lam
    assert np.max(np.abs(R - R.T)) < 1e-12 * np.max(np.abs(R))
    assert Lam.min() >= 0.0
    rows = Lam.sum(1)
    J1 = orc.formal_solution(m["chi"], np.ones_like(m["chi"]), 8, 8).ravel()
    assert np.max(np.abs(rows - J1)) < 1e-13
    assert rows.max() < 1.0
    L = orc.lstar(m["chi"], 8, 8).reshape(27, -1)
    assert L.min() >= 0.0
    assert np.all(L.sum(0) <= rows + 1e-15)
    # reciprocity inside the band: o and its mirror 26 - o
    nz, ny, nx = m["chi"].shape
    for o in range(27):
        dk, dj, di = o // 9 - 1, (o // 3) % 3 - 1, o % 3 - 1
        for v in range(chi.size):
            k, j, i = v // (nx * ny), (v // nx) % ny, v % nx
            if not 0 <= k + dk < nz:
                continue
            u = ((k + dk) * ny + (j + dj) % ny) * nx + (i + di) % nx
            assert abs(chi[v] * L[o, v] - chi[u] * L[26 - o, u]) <= 1e-12 * chi[v] * L[o, v] + 1e-300


def test_thick_voxels_diagonal_tends_to_one(orc):
    chi = np.full((5, 5, 5), 1e4)
    L = orc.lstar(chi, 8, 8).reshape(27, -1)
    assert L[13].min() > 0.999
    # very thin medium: almost nothing is absorbed, Lambda* is tiny
    L0 = orc.lstar(np.full((5, 5, 5), 1e-6), 8, 8).reshape(27, -1)
    assert L0.sum(0).max() < 1e-4
