"""Pins of the oracle's derivative machinery (complex step), which the GPU adjoint is checked against.

* The complex formal solution reduces to the real one for real inputs.
* Its complex-step derivatives equal central finite differences of the real formal solution.
* For a horizontally homogeneous slab, the derivative of an emergent intensity with respect to one
  layer's opacity has a closed form from the 1D recurrence I_{k+1} = S_k + (I_k - S_k) e^{-chi_k/mu}.
* The gradient of the converged loss equals central finite differences of the converged loss.
"""
import numpy as np
import pytest

from paper_1107_5719_amd.inputs import random_medium


def test_fs_complex_real_part_is_the_formal_solution(orc):
    m = random_medium(5, 4, 6, seed=21, chi_range=(1e-3, 1e2))
    S = np.random.default_rng(1).uniform(0.2, 2.0, m["chi"].shape)
    J, Iem = orc.formal_solution(m["chi"], S, 4, 8, I_top=0.3, I_bot=m["B"][0], want_emergent=True)
    Jc, Iemc = orc.fs_complex(m["chi"], S, 4, 8, I_top=0.3, I_bot=m["B"][0], want_emergent=True)
    assert np.max(np.abs(Jc.real - J) / J) < 1e-14
    assert np.max(np.abs(Iemc.real - Iem) / Iem) < 1e-14
    assert not Jc.imag.any() and not Iemc.imag.any()


def test_fs_complex_derivatives_match_finite_differences(orc):
    m = random_medium(4, 5, 4, seed=22, chi_range=(1e-2, 5.0))
    chi = m["chi"]
    S = np.random.default_rng(2).uniform(0.2, 2.0, chi.shape)
    h = 1e-30
    rng = np.random.default_rng(5)
    for v in rng.choice(chi.size, 5, replace=False):
        idx = np.unravel_index(v, chi.shape)
        for which in ("chi", "S"):
            c = chi.astype(complex)
            s = S.astype(complex)
            (c if which == "chi" else s)[idx] += 1j * h
            Jc, Ec = orc.fs_complex(c, s, 4, 4, I_top=0.1, I_bot=m["B"][0], want_emergent=True)
            base = chi if which == "chi" else S
            step = 1e-6 * base[idx]
            out = []
            for sign in (1.0, -1.0):
                a = base.copy()
                a[idx] += sign * step
                args = (a, S) if which == "chi" else (chi, a)
                out.append(orc.formal_solution(*args, 4, 4, I_top=0.1, I_bot=m["B"][0], want_emergent=True))
            dJ = (out[0][0] - out[1][0]) / (2 * step)
            dE = (out[0][1] - out[1][1]) / (2 * step)
            np.testing.assert_allclose(Jc.imag / h, dJ, rtol=0, atol=1e-6 * np.abs(dJ).max())
            np.testing.assert_allclose(Ec.imag / h, dE, rtol=0, atol=1e-6 * np.abs(dE).max())


@pytest.mark.parametrize("nt,nph", [(2, 4), (4, 8)])
def test_layer_opacity_derivative_of_emergent_light_closed_form(orc, nt, nph):
    """Horizontally homogeneous 4-layer slab: moving every voxel of layer k by i h gives the
    derivative with respect to the layer opacity; along an upward line of direction cosine mu the
    emergent intensity is the 1D recurrence, so dI_em/dchi_k = -(I_k - S_k) e^{-chi_k/mu}/mu times the
    transmission of the layers above."""
    nz, ny, nx = 4, 5, 6
    chi_k = np.array([2.0, 0.7, 0.3, 0.05])
    S_k = np.array([1.5, 1.2, 0.8, 0.4])
    I_bot = 2.0
    chi = np.broadcast_to(chi_k[:, None, None], (nz, ny, nx)).copy()
    S = np.broadcast_to(S_k[:, None, None], (nz, ny, nx)).copy()
    mu, _, _, _ = orc.quadrature(nt, nph)
    n_down = nt * nph // 2
    h = 1e-30
    for k in range(nz):
        c = chi.astype(complex)
        c[k] += 1j * h
        _, E = orc.fs_complex(c, S, nt, nph, I_bot=np.full((ny, nx), I_bot), want_emergent=True)
        for q, d in enumerate(range(n_down, nt * nph)):
            m_ = mu[d]
            I = I_bot
            for kk in range(k):
                I = S_k[kk] + (I - S_k[kk]) * np.exp(-chi_k[kk] / m_)
            dI = -(I - S_k[k]) * np.exp(-chi_k[k] / m_) / m_
            for kk in range(k + 1, nz):
                dI *= np.exp(-chi_k[kk] / m_)
            np.testing.assert_allclose(E[q].imag / h, dI, rtol=1e-12)


def test_loss_gradient_matches_finite_differences(orc):
    m = random_medium(4, 5, 3, seed=23, chi_range=(1e-2, 3.0), eps_range=(0.05, 0.5))
    nt, nph = 2, 4
    T = np.random.default_rng(3).uniform(0.5, 1.5, (nt * nph // 2, 5, 4))
    gchi, geps = orc.loss_gradient_cs(m["chi"], m["eps"], m["B"], T, nt, nph, I_top=0.2)
    rng = np.random.default_rng(0)
    for v in rng.choice(m["chi"].size, 4, replace=False):
        idx = np.unravel_index(v, m["chi"].shape)
        for name, g in (("chi", gchi), ("eps", geps)):
            step = 1e-5 * m[name][idx]
            L = []
            for sign in (1.0, -1.0):
                p = dict(m)
                p[name] = m[name].copy()
                p[name][idx] += sign * step
                L.append(orc.emergent_loss(p["chi"], p["eps"], p["B"], T, nt, nph, I_top=0.2)[0])
            fd = (L[0] - L[1]) / (2 * step)
            assert abs(g[idx] - fd) <= 1e-6 * abs(fd) + 1e-9 * np.abs(g).max(), (name, idx, g[idx], fd)


def test_loss_gradient_with_lte_diffusion_boundary_matches_fd(orc):
    """With the LTE-diffusion inner condition the bottom light depends on chi of the two bottom
    layers; the complex-step gradient carries that dependence (checked on bottom-layer voxels)."""
    m = random_medium(4, 4, 3, seed=29, chi_range=(0.05, 2.0), eps_range=(0.05, 0.5))
    nt, nph = 2, 4
    T = np.random.default_rng(4).uniform(0.5, 1.5, (nt * nph // 2, 4, 4))
    gchi, geps = orc.loss_gradient_cs(m["chi"], m["eps"], m["B"], T, nt, nph, bottom_from_B="diffusion")
    for idx in ((0, 1, 2), (1, 3, 0), (2, 0, 1)):
        step = 1e-5 * m["chi"][idx]
        L = []
        for sign in (1.0, -1.0):
            c = m["chi"].copy()
            c[idx] += sign * step
            L.append(orc.emergent_loss(c, m["eps"], m["B"], T, nt, nph, bottom_from_B="diffusion")[0])
        fd = (L[0] - L[1]) / (2 * step)
        assert abs(gchi[idx] - fd) <= 1e-6 * abs(fd) + 1e-9 * np.abs(gchi).max(), (idx, gchi[idx], fd)
