"""Pins of the oracle's angle set and line geometry against facts that do not come from the oracle.

Quadrature: Gauss-Legendre nodes/weights equal numpy's ``leggauss``; the direction weights reproduce
the exact angular moments of the unit sphere.  Geometry: every line crosses a layer with path length
1/|mu|; every voxel receives exactly 1/|mu| of path per direction; the horizontal displacement per
layer is tan(theta)(cos phi, sin phi); the mean number of segments per voxel and angle is
1 + tan(theta)(|cos phi| + |sin phi|) on average over layers.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32])
def test_gauss_legendre_matches_numpy(orc, n):
    x, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-15
    assert np.max(np.abs(w - wr)) < 1e-14


@pytest.mark.parametrize("nt,nph", [(2, 4), (8, 8), (16, 16), (6, 12)])
def test_quadrature_moments(orc, nt, nph):
    mu, ox, oy, W = orc.quadrature(nt, nph)
    assert abs(W.sum() - 1.0) < 1e-15
    # sphere moments: <mu^2m> = 1/(2m+1), exact for 2m <= 2 nt - 1
    for m in range(0, nt):
        assert abs((W * mu ** (2 * m)).sum() - 1.0 / (2 * m + 1)) < 1e-14
        assert abs((W * mu ** (2 * m + 1)).sum()) < 1e-15
    # isotropy in the plane: <ox> = <oy> = <ox oy> = 0, <ox^2> = <oy^2> = 1/3
    for q in (ox, oy, ox * oy, ox * mu, oy * mu):
        assert abs((W * q).sum()) < 1e-15
    assert abs((W * ox * ox).sum() - 1 / 3) < 1e-15
    assert abs((W * oy * oy).sum() - 1 / 3) < 1e-15
    # unit vectors; half offset in phi keeps every direction off the grid axes
    assert np.max(np.abs(mu ** 2 + ox ** 2 + oy ** 2 - 1)) < 1e-15
    assert np.min(np.abs(ox)) > 1e-3 and np.min(np.abs(oy)) > 1e-3
    # the direction set is closed under Omega -> -Omega, x -> -x, y -> -y and x <-> y
    dirs = np.stack([ox, oy, mu], 1)
    for T in (np.diag([-1, -1, -1]), np.diag([-1, 1, 1]), np.diag([1, -1, 1]),
              np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])):
        img = dirs @ T.T
        dist = np.min(np.linalg.norm(img[:, None, :] - dirs[None, :, :], axis=2), axis=1)
        assert np.max(dist) < 1e-14


@pytest.mark.parametrize("nt,nph,shape", [(8, 8, (5, 6, 7)), (16, 16, (3, 4, 5))])
def test_segment_lengths_and_voxel_path(orc, nt, nph, shape):
    nz, ny, nx = shape
    mu, ox, oy, W = orc.quadrature(nt, nph)
    for d in range(nt * nph):
        path = np.zeros(nx * ny * nz)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    v, ln = orc.trace_layer(nx, ny, nz, nt, nph, d, i, j, k)
                    assert abs(ln.sum() - 1.0 / abs(mu[d])) < 1e-13
                    assert np.all(v // (nx * ny) == k)
                    np.add.at(path, v, ln)
        # one line of the translated lattice crosses every voxel cross-section at every height
        assert np.max(np.abs(path * abs(mu[d]) - 1.0)) < 1e-12


def test_segments_follow_the_line(orc):
    """Consecutive segments are face neighbours, and the layer path starts and ends in the voxels
    that contain x(z) = i + 1/2 + (z - nz) tan(theta) cos(phi) (likewise y) at its two ends."""
    nx = ny = nz = 9
    nt, nph = 16, 16
    mu, ox, oy, W = orc.quadrature(nt, nph)
    rng = np.random.default_rng(0)
    for d in range(nt * nph):
        tx, ty = ox[d] / mu[d], oy[d] / mu[d]
        for _ in range(4):
            i, j, k = (int(a) for a in rng.integers(0, 9, 3))
            v, ln = orc.trace_layer(nx, ny, nz, nt, nph, d, i, j, k)
            iv, jv = v % nx, (v // nx) % ny
            za, zb = (k + 1, k) if mu[d] < 0 else (k, k + 1)
            # evaluate a hair inside the layer to stay off exact faces
            fa, fb = 1e-9, 1 - 1e-9
            xa = i + 0.5 + (za + fa * (zb - za) - nz) * tx
            ya = j + 0.5 + (za + fa * (zb - za) - nz) * ty
            xb = i + 0.5 + (za + fb * (zb - za) - nz) * tx
            yb = j + 0.5 + (za + fb * (zb - za) - nz) * ty
            assert (int(np.floor(xa)) % nx, int(np.floor(ya)) % ny) == (iv[0], jv[0])
            assert (int(np.floor(xb)) % nx, int(np.floor(yb)) % ny) == (iv[-1], jv[-1])
            step = (np.diff(iv) % nx != 0).astype(int) + (np.diff(jv) % ny != 0).astype(int)
            assert np.all(step <= 1)
            assert len(v) - 1 <= int(np.ceil(abs(tx))) + int(np.ceil(abs(ty)))


@pytest.mark.parametrize("nt,nph,expect", [(8, 8, 3.62), (16, 16, 4.05)])
def test_mean_segments_per_voxel_angle(orc, nt, nph, expect):
    mu, ox, oy, W = orc.quadrature(nt, nph)
    formula = np.mean(1 + (np.abs(ox) + np.abs(oy)) / np.abs(mu))
    assert abs(formula - expect) < 0.005
    N = 33
    tot = 0
    for d in range(nt * nph):
        for k in range(N):
            v, _ = orc.trace_layer(N, N, N, nt, nph, d, 0, 0, k)
            tot += len(v)
    assert abs(tot / (nt * nph * N) - formula) / formula < 0.01
