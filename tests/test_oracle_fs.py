"""Pins of the oracle's formal solution (FS) and mean intensity J.

Each pin is a fact fixed by the transfer equation, not by the oracle's own code:
  * equilibrium: S = c everywhere with boundary light c gives I = c, hence J = c, for any chi;
  * escape: constant S, no incident light, horizontally homogeneous layers: the top-plane
    intensity is S (1 - exp(-tau / mu));
  * plane-parallel reduction: a horizontally homogeneous grid gives the 1D solution, and the 1D
    solver reproduces the closed-form layer average of S (1 - exp(-t / |mu|));
  * a hand-derived geometry (tan(theta) = sqrt(2) at phi = 45 deg + n 90 deg moves each line by one
    voxel diagonally per layer, half a layer path in each of two voxels);
  * translation, mirror and x<->y symmetry, and linearity in S.
"""
import numpy as np
import pytest

from paper_1107_5719_amd.inputs import random_medium


def test_equilibrium_any_medium(orc):
    m = random_medium(5, 6, 7, seed=11, chi_range=(1e-4, 1e4))
    c = 2.75
    S = np.full(m["chi"].shape, c)
    J, Iem = orc.formal_solution(m["chi"], S, 8, 8, I_top=c, I_bot=np.full((6, 5), c),
                                 want_emergent=True)
    assert np.max(np.abs(J / c - 1)) < 1e-14
    assert np.max(np.abs(Iem / c - 1)) < 1e-14


def test_escape_constant_source(orc):
    rng = np.random.default_rng(5)
    nz, ny, nx = 7, 4, 5
    chi_k = np.exp(rng.uniform(np.log(1e-3), np.log(3.0), nz))
    chi = np.broadcast_to(chi_k[:, None, None], (nz, ny, nx)).copy()
    S0 = 1.7
    J, Iem = orc.formal_solution(chi, np.full(chi.shape, S0), 16, 16, want_emergent=True)
    mu = orc.quadrature(16, 16)[0]
    mu_up = mu[mu > 0]
    expect = S0 * (1 - np.exp(-chi_k.sum() / mu_up))
    got = Iem.reshape(len(mu_up), -1)
    assert np.max(np.abs(got / expect[:, None] - 1)) < 1e-13


def test_escape_heterogeneous_line(orc):
    """Heterogeneous chi: the top-plane intensity of an upward line is S (1 - exp(-tau_path)) with
    tau_path the optical length summed over that line's segments."""
    m = random_medium(5, 5, 6, seed=12, chi_range=(1e-3, 1.0))
    chi = m["chi"]
    nz, ny, nx = chi.shape
    S0 = 0.8
    _, Iem = orc.formal_solution(chi, np.full(chi.shape, S0), 8, 8, want_emergent=True)
    mu = orc.quadrature(8, 8)[0]
    up = np.nonzero(mu > 0)[0]
    for d in up[::7]:
        q = int(d - up[0])
        for (i, j) in ((0, 0), (3, 1), (4, 4)):
            tau = 0.0
            for k in range(nz):
                v, ln = orc.trace_layer(nx, ny, nz, 8, 8, int(d), i, j, k)
                tau += float(np.sum(chi.ravel()[v] * ln))
            assert abs(Iem[q, j, i] / (S0 * -np.expm1(-tau)) - 1) < 1e-13


def _pp_closed_form_constant_S(dtau, S0, n_theta, orc):
    """Layer averages of I = S0 (1 - exp(-t / |mu|)), t the optical depth from the side the light
    comes from, averaged over each layer -- written with explicit exponentials."""
    x, w = orc.gauss_legendre(n_theta)
    edges = np.concatenate([[0.0], np.cumsum(dtau)])   # from the bottom
    total = edges[-1]
    J = np.zeros(len(dtau))
    for mu_a, w_a in zip(x, w):
        amu = abs(mu_a)
        if mu_a > 0:  # coming from the bottom: t = depth above the bottom
            ta, tb = edges[:-1], edges[1:]
        else:         # coming from the top
            ta, tb = total - edges[1:], total - edges[:-1]
        avg = S0 * (1 - amu * (np.exp(-ta / amu) - np.exp(-tb / amu)) / (tb - ta))
        J += 0.5 * w_a * avg
    return J


def test_pp1d_closed_form(orc):
    rng = np.random.default_rng(3)
    dtau = np.exp(rng.uniform(np.log(1e-3), np.log(5.0), 12))
    J = orc.pp1d(dtau, np.full(12, 2.0), 16)
    ref = _pp_closed_form_constant_S(dtau, 2.0, 16, orc)
    assert np.max(np.abs(J / ref - 1)) < 1e-12


@pytest.mark.parametrize("nt,nph,shape", [(8, 8, (9, 4, 5)), (16, 16, (6, 3, 3))])
def test_horizontally_homogeneous_is_plane_parallel(orc, nt, nph, shape):
    nz, ny, nx = shape
    rng = np.random.default_rng(9)
    chi_k = np.exp(rng.uniform(np.log(1e-4), np.log(30.0), nz))
    S_k = rng.uniform(0.2, 3.0, nz)
    chi = np.broadcast_to(chi_k[:, None, None], shape).copy()
    S = np.broadcast_to(S_k[:, None, None], shape).copy()
    J = orc.formal_solution(chi, S, nt, nph, I_top=0.3, I_bot=np.full((ny, nx), 1.9))
    J1 = orc.pp1d(chi_k, S_k, nt, I_top=0.3, I_bot=1.9)
    assert np.max(np.abs(J / J1[:, None, None] - 1)) < 1e-12


def test_hand_derived_unit_drift_geometry(orc):
    """n_theta = 2, n_phi = 4: mu = +-1/sqrt(3), tan(theta) = sqrt(2), phi = 45, 135, 225, 315 deg,
    so a line moves by exactly one voxel in x and in y per layer.  A line at a voxel centre on a
    layer face spends half of its layer path (length sqrt(3)/2) in the voxel below that centre and
    half in the diagonal neighbour it moves to.  Expected J from that picture alone."""
    nz, ny, nx = 4, 5, 6
    m = random_medium(nx, ny, nz, seed=21, chi_range=(0.05, 5.0))
    chi, S = m["chi"], m["B"]
    I_top, I_bot = 0.4, m["eps"][0] * 3.0
    J = orc.formal_solution(chi, S, 2, 4, I_top=I_top, I_bot=I_bot)
    mu_n = 1 / np.sqrt(3.0)
    half = 0.5 / mu_n
    Jref = np.zeros(chi.shape)
    for mu_s in (-1, 1):
        for phi in np.deg2rad([45, 135, 225, 315]):
            sx = int(np.sign(np.cos(phi))) * mu_s   # column step per unit of height
            sy = int(np.sign(np.sin(phi))) * mu_s
            acc = np.zeros(chi.shape)
            for j in range(ny):
                for i in range(nx):
                    if mu_s < 0:
                        I = I_top
                        layers = range(nz - 1, -1, -1)
                    else:
                        # the line is at column (i - nz sx, j - nz sy) on the bottom plane
                        I = I_bot[(j - nz * sy) % ny, (i - nz * sx) % nx]
                        layers = range(nz)
                    for k in layers:
                        # column on the layer face where the line enters, then the one it exits at
                        z_in, z_out = (k + 1, k) if mu_s < 0 else (k, k + 1)
                        cols = [((i + (z_in - nz) * sx) % nx, (j + (z_in - nz) * sy) % ny),
                                ((i + (z_out - nz) * sx) % nx, (j + (z_out - nz) * sy) % ny)]
                        for (ci, cj) in cols:
                            t = chi[k, cj, ci] * half
                            s = S[k, cj, ci]
                            # exact: integral of chi I ds = s t + (I - s)(1 - e^-t)
                            acc[k, cj, ci] += s * t + (I - s) * (1 - np.exp(-t))
                            I = s + (I - s) * np.exp(-t)
            Jref += 0.125 * mu_n / chi * acc    # W = w_a / (2 n_phi) = 1 / 8
    assert np.max(np.abs(J / Jref - 1)) < 1e-12


def test_translation_mirror_swap(orc):
    m = random_medium(6, 6, 5, seed=31)
    chi, S = m["chi"], m["B"]
    Ib = m["eps"][0] * 2
    J = orc.formal_solution(chi, S, 8, 8, I_top=0.2, I_bot=Ib)
    # integer shift (2, 3) in (x, y)
    Js = orc.formal_solution(np.roll(chi, (3, 2), (1, 2)), np.roll(S, (3, 2), (1, 2)), 8, 8, I_top=0.2,
                             I_bot=np.roll(Ib, (3, 2), (0, 1)))
    assert np.max(np.abs(Js / np.roll(J, (3, 2), (1, 2)) - 1)) < 1e-13
    # mirror in x, mirror in y, swap x <-> y
    for f in (lambda a: a[..., ::-1], lambda a: a[..., ::-1, :], lambda a: np.swapaxes(a, -1, -2)):
        Jm = orc.formal_solution(np.ascontiguousarray(f(chi)), np.ascontiguousarray(f(S)), 8, 8,
                                 I_top=0.2, I_bot=np.ascontiguousarray(f(Ib)))
        assert np.max(np.abs(Jm / f(J) - 1)) < 1e-13


def test_linearity_zero_boundary(orc):
    m = random_medium(5, 4, 6, seed=41)
    rng = np.random.default_rng(1)
    S1, S2 = rng.uniform(0, 1, m["chi"].shape), rng.uniform(-1, 1, m["chi"].shape)
    a, b = 0.7, -2.3
    J12 = orc.formal_solution(m["chi"], a * S1 + b * S2, 8, 8)
    J1 = orc.formal_solution(m["chi"], S1, 8, 8)
    J2 = orc.formal_solution(m["chi"], S2, 8, 8)
    assert np.max(np.abs(J12 - (a * J1 + b * J2))) < 1e-13 * np.max(np.abs(J12))


def test_threads_do_not_change_result_beyond_rounding(orc):
    m = random_medium(7, 5, 6, seed=51)
    J1 = orc.formal_solution(m["chi"], m["B"], 8, 8, n_threads=1)
    J4 = orc.formal_solution(m["chi"], m["B"], 8, 8, n_threads=4)
    assert np.max(np.abs(J4 / J1 - 1)) < 1e-14


def test_lte_diffusion_boundary_pins(orc):
    """The LTE-diffusion inner condition I = B_0 + mu (B_0 - B_1) / ((chi_0 + chi_1) / 2):
    * with isothermal B it is the B condition, exactly;
    * through an almost transparent slab the emergent light of every upward line is that boundary
      light of the column the line enters;
    * for a horizontally homogeneous slab the 3D formal solution equals the 1D plane-parallel one
      with the same boundary (a separate code path with no 3D geometry)."""
    nz, ny, nx = 4, 5, 6
    rng = np.random.default_rng(7)
    chi = np.exp(rng.uniform(np.log(0.05), np.log(3.0), (nz, ny, nx)))
    eps = rng.uniform(0.1, 0.9, (nz, ny, nx))
    B1 = np.full((nz, ny, nx), 1.7)
    assert np.array_equal(orc.dense_os_solution(chi, eps, B1, 4, 4, bottom_from_B="diffusion"),
                          orc.dense_os_solution(chi, eps, B1, 4, 4, bottom_from_B=True))
    # almost transparent: I_em = B_0 + mu slope of the entry column
    B = rng.uniform(0.5, 2.0, (nz, ny, nx))
    chi_t = np.full((nz, ny, nx), 1e-13)
    slope = orc.diffusion_slope(chi_t * 0 + 1.0, B)       # any slope field will do
    _, Iem = orc.formal_solution(chi_t, np.zeros_like(B), 4, 8, I_bot=B[0], I_slope=slope,
                                 want_emergent=True)
    mu, ox, oy, _ = orc.quadrature(4, 8)
    for q, d in enumerate(range(16, 32)):
        for j in range(ny):
            for i in range(nx):
                v, _ = orc.trace_layer(nx, ny, nz, 4, 8, d, i, j, 0)
                c = v[0]
                assert abs(Iem[q, j, i] - (B[0].ravel()[c] + mu[d] * slope.ravel()[c])) < 1e-10
    # horizontally homogeneous: 3D = 1D with the same boundary
    chi_k = np.array([2.5, 0.8, 0.3, 0.05])
    B_k = np.array([3.0, 2.2, 1.5, 1.0])
    S_k = np.array([2.0, 1.5, 1.1, 0.6])
    chi3 = np.broadcast_to(chi_k[:, None, None], (nz, ny, nx)).copy()
    B3 = np.broadcast_to(B_k[:, None, None], (nz, ny, nx)).copy()
    S3 = np.broadcast_to(S_k[:, None, None], (nz, ny, nx)).copy()
    sl = orc.diffusion_slope(chi3, B3)
    J3 = orc.formal_solution(chi3, S3, 8, 8, I_top=0.2, I_bot=B3[0], I_slope=sl)
    J1 = orc.pp1d(chi_k, S_k, 8, I_top=0.2, I_bot=B_k[0], I_slope=(B_k[0] - B_k[1]) / (0.5 * (chi_k[0] + chi_k[1])))
    np.testing.assert_allclose(J3, np.broadcast_to(J1[:, None, None], J3.shape), rtol=1e-13)


def test_lte_diffusion_slope_pinned_by_optical_depth(orc):
    """The gradient of the LTE-diffusion condition, pinned by two facts that do not restate its formula.

    * Definition: with B a linear function a + s tau of the optical depth tau measured inwards from
      the top (tau of a voxel centre = the opacity of all voxels above it plus half its own), the
      condition's dB/dtau is s in every column, for any opacities.
    * Transfer: for S = B = a + s tau (eps = 1) in a semi-infinite medium the emergent intensity is
      exactly a + s mu.  A finite slab closed by the diffusion condition emits that value up to the
      discretisation (piecewise-constant S; the condition sits half a voxel below the bottom centre),
      so its error falls in proportion to the layer thickness under refinement; closed by I = B_0 or
      by the slope with the wrong sign, the error stays at the order of s mu e^{-tau/mu}."""
    rng = np.random.default_rng(3)
    nz, ny, nx = 5, 4, 6
    chi = np.exp(rng.uniform(np.log(0.01), np.log(50.0), (nz, ny, nx)))
    a, s = 1.3, 0.45
    tau_c = np.cumsum(chi[::-1], axis=0)[::-1] - 0.5 * chi
    B = a + s * tau_c
    np.testing.assert_allclose(orc.diffusion_slope(chi, B), s, rtol=1e-10)
    mu = orc.quadrature(8, 8)[0]
    exact = a + s * mu[mu > 0]
    tau_b = 2.0
    errs = {"diffusion": [], "B": [], "negative": []}
    for N in (16, 32, 64, 128):
        chi_k = np.full(N, tau_b / N)
        B_k = a + s * (np.cumsum(chi_k[::-1])[::-1] - 0.5 * chi_k)
        chi3 = np.broadcast_to(chi_k[:, None, None], (N, 3, 3)).copy()
        B3 = np.broadcast_to(B_k[:, None, None], (N, 3, 3)).copy()
        sl = orc.diffusion_slope(chi3, B3)
        for name, slope in (("diffusion", sl), ("B", None), ("negative", -sl)):
            _, Iem = orc.formal_solution(chi3, B3, 8, 8, I_bot=B3[0], I_slope=slope, want_emergent=True)
            errs[name].append(float(np.max(np.abs(Iem[:, 1, 1] - exact))))
    e = errs["diffusion"]
    for coarse, fine in zip(e, e[1:]):
        assert 1.8 < coarse / fine < 2.2, e
    assert e[-1] < 0.01 * errs["B"][-1]
    assert min(errs["B"]) > 0.05 and min(errs["negative"]) > 0.1, errs
