"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle, element by element.

Bar (FP64 path): |x_gpu - x_oracle| <= 1e-10 |x_oracle| (+ a tiny absolute floor for entries that
are exactly zero), on J_fs, the top-plane intensities, Lambda*, every OS iterate, and the converged
J.  The oracle never sees anything the GPU produced: both sides get the same seeded media.
"""
import numpy as np
import pytest

from lstar_bar import close_lstar
from paper_1107_5719_amd.inputs import WORKLOADS, diffusion_medium, make_medium, random_medium

pytestmark = pytest.mark.gpu

RTOL = 1e-10


@pytest.fixture(scope="module")
def R():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.zeros(1, device="cuda")
    from paper_1107_5719_amd import rt3d

    return rt3d


def _close(a, b, rtol=RTOL, floor=1e-300):
    err = np.abs(a - b)
    lim = rtol * np.abs(b) + floor
    bad = err > lim
    assert not bad.any(), f"{bad.sum()} of {bad.size} off; worst rel {np.max(err / (np.abs(b) + floor)):.3e}"


def _medium_case(name):
    if name in WORKLOADS:
        w = WORKLOADS[name]
        m = make_medium(w)
        return m, w.n_theta, w.n_phi, w.I_top
    raise KeyError(name)


FS_CASES = [
    # (shape (nz, ny, nx), n_theta, n_phi, seed, I_top, bottom_bc)
    ((5, 5, 5), 8, 8, 1, 0.3, 0),
    ((11, 7, 9), 16, 16, 2, 0.0, 0),     # non-cubic, odd sizes
    ((3, 3, 3), 16, 16, 3, 0.7, 0),      # minimum grid: shallow lines wrap many times per layer
    ((7, 5, 6), 8, 8, 4, 0.0, 1),        # zero light at the bottom
    ((4, 40, 33), 16, 16, 5, 0.1, 0),    # several bands per direction and a ragged last band
    ((6, 9, 131), 8, 8, 6, 0.0, 0),      # rows longer than two wavefronts
    ((6, 5, 7), 2, 4, 7, 0.2, 0),        # smallest angle set; every line runs through voxel edges
    ((5, 8, 6), 8, 4, 8, 0.0, 0),        # n_phi = 4 with steep and shallow directions
    ((6, 7, 5), 8, 8, 9, 0.1, 2),        # LTE-diffusion inner condition
    ((3, 4, 256), 16, 16, 10, 0.0, 0),   # wide rows, 16 x 16 angles in the 48 KB LDS budget
    ((3, 4, 300), 16, 16, 11, 0.0, 0),   # about the widest in the 48 KB budget
    ((4, 5, 520), 16, 16, 12, 0.2, 0),   # one row per band in the wide LDS budget
    ((3, 4, 1024), 16, 16, 13, 0.1, 0),  # the widest grid: a whole workgroup per row
    ((3, 5, 600), 32, 32, 14, 0.0, 0),   # 32 x 32 angles: the largest row spread, wide LDS budget
    ((5, 6, 4), 8, 8, 15, 0.2, 0),       # nx = 4: a move of the B lines by two columns is half a row
]


@pytest.mark.parametrize("case", FS_CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}" for c in FS_CASES])
def test_formal_solution_parity(R, orc, case):
    shape, nt, nph, seed, I_top, bbc = case
    nz, ny, nx = shape
    m = (diffusion_medium(nx, ny, nz, seed=seed, chi_range=(1e-4, 1e2)) if bbc == 2 else
         random_medium(nx, ny, nz, seed=seed, chi_range=(1e-4, 1e2)))
    S = np.random.default_rng(seed).uniform(0.1, 3.0, shape)
    J_orc, Iem_orc = orc.formal_solution(m["chi"], S, nt, nph, I_top=I_top,
                                         I_bot=(m["B"][0] if bbc != 1 else None), want_emergent=True,
                                         I_slope=(orc.diffusion_slope(m["chi"], m["B"]) if bbc == 2 else None))
    with R.Solver(nx, ny, nz, nt, nph, I_top=I_top, bottom_bc=bbc) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        J = s.formal_solution(S)
        Iem = s.emergent_top()
    _close(J, J_orc)
    _close(Iem, Iem_orc)


def test_formal_solution_source_from_J_and_device_pointers(R, orc):
    import torch

    nz, ny, nx = 6, 7, 8
    m = random_medium(nx, ny, nz, seed=7)
    J0 = np.random.default_rng(7).uniform(0.5, 2.0, (nz, ny, nx))
    S = m["eps"] * m["B"] + (1 - m["eps"]) * J0
    J_orc = orc.formal_solution(m["chi"], S, 8, 8, I_bot=m["B"][0])
    dev = {k: torch.from_numpy(v).cuda() for k, v in m.items()}
    with R.Solver(nx, ny, nz, 8, 8) as s:
        s.set_medium(dev["chi"], dev["eps"], dev["B"])
        s.set_J(torch.from_numpy(J0).cuda())
        out = torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda")
        s.formal_solution(None, out)
        torch.cuda.synchronize()
        _close(out.cpu().numpy(), J_orc)
        _close(s.get_J(), J0, rtol=0.0, floor=0.0)


LSTAR_CASES = [((5, 5, 5), 8, 8, 1), ((7, 5, 6), 16, 16, 2), ((3, 4, 3), 16, 16, 3), ((9, 12, 11), 8, 8, 4)]


@pytest.mark.parametrize("case", LSTAR_CASES, ids=[str(c[0]) + f"-{c[1]}" for c in LSTAR_CASES])
def test_lstar_parity(R, orc, case):
    shape, nt, nph, seed = case
    nz, ny, nx = shape
    m = random_medium(nx, ny, nz, seed=seed, chi_range=(1e-3, 1e2))
    L_orc = orc.lstar(m["chi"], nt, nph)
    with R.Solver(nx, ny, nz, nt, nph) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        s.build_lstar()
        L = s.get_lstar()
    close_lstar(L, L_orc, m["chi"], nt)


def test_lstar_and_fs_parity_strat17(R, orc):
    m, nt, nph, I_top = _medium_case("strat17")
    nz, ny, nx = m["chi"].shape
    L_orc = orc.lstar(m["chi"], nt, nph)
    S = m["eps"] * m["B"] + (1 - m["eps"]) * m["B"]
    J_orc = orc.formal_solution(m["chi"], S, nt, nph, I_top=I_top, I_bot=m["B"][0])
    with R.Solver(nx, ny, nz, nt, nph, I_top=I_top) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        J = s.formal_solution(None)
        s.build_lstar()
        L = s.get_lstar()
    _close(J, J_orc)
    close_lstar(L, L_orc, m["chi"], nt)


@pytest.mark.parametrize("M", [1, 2, 7])
def test_os_iterates_parity(R, orc, M):
    """The same outer iteration on both sides: every iterate and every convergence measure."""
    nz, ny, nx = 6, 5, 7
    m = random_medium(nx, ny, nz, seed=11, chi_range=(1e-2, 1e2), eps_range=(1e-3, 1.0))
    L = orc.lstar(m["chi"], 8, 8)
    J_orc = m["B"].copy()
    with R.Solver(nx, ny, nz, 8, 8, I_top=0.2) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        for it in range(6):
            c = s.os_step(M)
            J_orc, c_orc = orc.os_step(m["chi"], m["eps"], m["B"], L, J_orc, 8, 8, M=M, I_top=0.2)
            _close(s.get_J(), J_orc)
            assert abs(c - c_orc) <= 1e-6 * c_orc + 1e-14, (it, c, c_orc)


def test_converged_equals_dense_solution(R, orc):
    nz, ny, nx = 5, 5, 5
    m = random_medium(nx, ny, nz, seed=12, chi_range=(1e-2, 1e1), eps_range=(1e-2, 1.0))
    Jd = orc.dense_os_solution(m["chi"], m["eps"], m["B"], 8, 8, I_top=0.1)
    with R.Solver(nx, ny, nz, 8, 8, I_top=0.1) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        st, it, c = s.solve(1e-14, 500, 50)
        assert st == R.RT3D_OK
        _close(s.get_J(), Jd)


def test_solve_parity_strat17(R, orc):
    """17^3 x 64 angles, eps = 1e-2, stop at max rel dJ < 1e-8: same iteration count and J."""
    w = WORKLOADS["strat17"]
    m = make_medium(w)
    M = 20
    J_orc, it_orc, c_orc, ok = orc.solve(m["chi"], m["eps"], m["B"], w.n_theta, w.n_phi, tol=w.tol,
                                         max_iter=500, M=M, I_top=w.I_top)
    assert ok
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        st, it, c = s.solve(w.tol, 500, M)
        assert st == R.RT3D_OK
        assert it == it_orc
        _close(s.get_J(), J_orc)


def test_fs_and_os_step_parity_grf65(R, orc):
    """65^3 x 256 angles: J_fs, Lambda* and one OS step against the oracle."""
    w = WORKLOADS["grf65"]
    m = make_medium(w)
    M = 4
    S = m["eps"] * m["B"] + (1 - m["eps"]) * m["B"]
    J_fs_orc = orc.formal_solution(m["chi"], S, w.n_theta, w.n_phi, I_top=w.I_top, I_bot=m["B"][0])
    L_orc = orc.lstar(m["chi"], w.n_theta, w.n_phi)
    J1_orc, c_orc = orc.os_step(m["chi"], m["eps"], m["B"], L_orc, m["B"], w.n_theta, w.n_phi, M=M,
                                I_top=w.I_top)
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        _close(s.formal_solution(None), J_fs_orc)
        s.build_lstar()
        close_lstar(s.get_lstar(), L_orc, m["chi"], w.n_theta)
        c = s.os_step(M)
        _close(s.get_J(), J1_orc)
        assert abs(c - c_orc) <= 1e-8 * c_orc


def test_fs_parity_strat129(R, orc):
    """129^3 x 256 angles (the benchmark workload, launched exactly as the benchmark launches it):
    every voxel of J_fs against the oracle."""
    w = WORKLOADS["strat129"]
    m = make_medium(w)
    S = m["eps"] * m["B"] + (1 - m["eps"]) * m["B"]
    J_orc = orc.formal_solution(m["chi"], S, w.n_theta, w.n_phi, I_top=w.I_top, I_bot=m["B"][0])
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi, I_top=w.I_top) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        J = s.formal_solution(None)
    _close(J, J_orc)


def test_paper_slab_grids_parity(R, orc):
    """The paper's slab (continuum optical depth 1e-4 .. 1e8, isothermal, eps = 1e-2) on its two timing
    grids: at 65^3 x 256 J_fs, Lambda* and one OS step; at 129^2 x 193 x 256 every voxel of J_fs for a
    seeded source (the slab has no horizontal structure, the source does)."""
    w = WORKLOADS["slab65"]
    m = make_medium(w)
    L_orc = orc.lstar(m["chi"], w.n_theta, w.n_phi)
    J1_orc, c_orc = orc.os_step(m["chi"], m["eps"], m["B"], L_orc, m["B"], w.n_theta, w.n_phi, M=4)
    S = np.random.default_rng(65).uniform(0.5, 1.5, w.shape)
    J_fs_orc = orc.formal_solution(m["chi"], S, w.n_theta, w.n_phi, I_bot=m["B"][0])
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        _close(s.formal_solution(S), J_fs_orc)
        s.build_lstar()
        close_lstar(s.get_lstar(), L_orc, m["chi"], w.n_theta)
        c = s.os_step(4)
        _close(s.get_J(), J1_orc)
        assert abs(c - c_orc) <= 1e-8 * c_orc
    w = WORKLOADS["slab193"]
    m = make_medium(w)
    S = np.random.default_rng(193).uniform(0.5, 1.5, w.shape)
    J_orc = orc.formal_solution(m["chi"], S, w.n_theta, w.n_phi, I_bot=m["B"][0])
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        J = s.formal_solution(S)
    _close(J, J_orc)


def test_solve_parity_lte_diffusion(R, orc):
    """A converged solve with the LTE-diffusion inner condition (B varying with depth, so the
    condition differs from I = B) against the oracle's: same iteration count, J within 1e-10."""
    nz, ny, nx = 6, 5, 7
    m = diffusion_medium(nx, ny, nz, seed=31, chi_range=(0.05, 5.0), eps_range=(0.01, 0.3))
    J_orc, it_o, c_o, ok = orc.solve(m["chi"], m["eps"], m["B"], 8, 8, 1e-10, 3000, 6,
                                     bottom_from_B="diffusion")
    assert ok
    J_dense = orc.dense_os_solution(m["chi"], m["eps"], m["B"], 8, 8, bottom_from_B="diffusion")
    with R.Solver(nx, ny, nz, 8, 8, bottom_bc=2) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        st, it, c = s.solve(1e-10, 3000, 6)
        J = s.get_J()
    assert st == R.RT3D_OK and it == it_o
    _close(J, J_orc)
    np.testing.assert_allclose(J, J_dense, rtol=1e-8)


def test_error_paths(R):
    import torch

    nz, ny, nx = 4, 4, 4
    m = random_medium(nx, ny, nz, seed=13)
    with R.Solver(nx, ny, nz, 8, 8) as s:
        with pytest.raises(R.Rt3dError) as e:
            s.formal_solution(None)
        assert e.value.status == R.RT3D_ERR_STATE
        with pytest.raises(R.Rt3dError) as e:
            s.get_lstar()
        assert e.value.status == R.RT3D_ERR_STATE
        bad = m["chi"].copy()
        bad[1, 2, 3] = np.nan
        with pytest.raises(R.Rt3dError) as e:
            s.set_medium(bad, m["eps"], m["B"])
        assert e.value.status == R.RT3D_ERR_ARG
        dev = {k: torch.from_numpy(v).cuda() for k, v in m.items()}
        dev_bad_eps = dev["eps"].clone()
        dev_bad_eps[0, 0, 0] = 0.0
        with pytest.raises(R.Rt3dError) as e:
            s.set_medium(dev["chi"], dev_bad_eps, dev["B"])
        assert e.value.status == R.RT3D_ERR_ARG
        s.set_medium(dev["chi"], dev["eps"], dev["B"])
        with pytest.raises(R.Rt3dError) as e:
            s.os_step(0)
        assert e.value.status == R.RT3D_ERR_ARG
        st, it, c = s.solve(1e-30, 2, 3)
        assert st == R.RT3D_ERR_NOT_CONVERGED and it == 2 and np.isfinite(c)
        Jbad = np.ones((nz, ny, nx))
        Jbad[0, 1, 1] = np.inf
        with pytest.raises(R.Rt3dError) as e:
            s.set_J(Jbad)
        assert e.value.status == R.RT3D_ERR_ARG


def test_determinism_and_resume(R):
    """Two runs are bitwise identical, and 3 + 3 steps through get_J / set_J in a fresh context equal
    6 straight steps bitwise (the kernels use no atomics in any floating-point sum)."""
    w = WORKLOADS["strat17"]
    m = make_medium(w)
    runs = []
    for _ in range(2):
        with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi) as s:
            s.set_medium(m["chi"], m["eps"], m["B"])
            for _ in range(6):
                s.os_step(5)
            runs.append(s.get_J())
    assert np.array_equal(runs[0], runs[1])
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        for _ in range(3):
            s.os_step(5)
        J3 = s.get_J()
    with R.Solver(w.nx, w.ny, w.nz, w.n_theta, w.n_phi) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        s.set_J(J3)
        for _ in range(3):
            s.os_step(5)
        assert np.array_equal(s.get_J(), runs[0])


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_sweep"])
def test_jacobi_grid_layouts_agree_bitwise(R, precision, monkeypatch):
    """Every launch layout of the Jacobi sweep (one block per plane chunk, padded, XCD-grouped, 2D
    tiles, columns of 1, 2 or 4 voxels marched in z, in either order of the column layers, odd layers
    walked bottom up or top down) computes each voxel's sum in the same order, so OS steps agree
    bitwise; the grid (nz = 10, not a multiple of the column height 4; 37 x 9 columns, a ragged last
    chunk) also checks the column form's ends.  The layout is read from RT3D_JACOBI_XCD,
    RT3D_JACOBI_ALTERNATE, RT3D_JACOBI_COLUMN and RT3D_JACOBI_WALK when a context is created."""
    m = random_medium(37, 9, 10, seed=77, chi_range=(1e-3, 3e1), eps_range=(1e-4, 0.3))
    out = {}
    # (layout, alternate, column height, walk): layouts 0..3 ignore the rest; column height 0 is the
    # size rule (1 on this grid); walk -1 is the default rule (top-down odd layers for float
    # coefficients in columns of 4, which the FP32-sweep form stores)
    layouts = ((0, 1, 0, -1), (1, 1, 0, -1), (2, 1, 0, -1), (3, 1, 0, -1), (4, 1, 0, -1), (4, 0, 0, -1),
               (4, 1, 2, -1), (4, 1, 4, -1), (4, 0, 4, -1), (4, 1, 4, 1), (4, 0, 4, 1), (4, 1, 4, 0),
               (4, 1, 2, 1))
    for layout in layouts:
        monkeypatch.setenv("RT3D_JACOBI_XCD", str(layout[0]))
        monkeypatch.setenv("RT3D_JACOBI_ALTERNATE", str(layout[1]))
        monkeypatch.setenv("RT3D_JACOBI_COLUMN", str(layout[2]))
        monkeypatch.setenv("RT3D_JACOBI_WALK", str(layout[3]))
        with R.Solver(37, 9, 10, 4, 8, precision=precision) as s:
            s.set_medium(m["chi"], m["eps"], m["B"])
            cs = [s.os_step(7) for _ in range(3)]
            st = s.stats()
            if layout[0] == 4 and layout[2] == 4:
                want = layout[3] == 1 or (layout[3] == -1 and st["coef_storage"] == "fp32")
                assert st["jacobi_alt_walk"] == int(want), layout
            out[layout] = (s.get_J(), cs)
    for layout in layouts[1:]:
        assert np.array_equal(out[layout][0], out[layouts[0]][0]), f"layout {layout}"
        assert out[layout][1] == out[layouts[0]][1]


def test_formal_solution_parity_extreme_optical_depths(R, orc):
    """Segment optical depths from ~1e-10 to ~1e6 (chi log-uniform over 16 decades): the float64
    exponential's reduction, table and clamp at both ends, against the oracle's libm expm1."""
    nz, ny, nx = 6, 7, 9
    rng = np.random.default_rng(31)
    chi = np.exp(rng.uniform(np.log(1e-10), np.log(1e6), (nz, ny, nx)))
    S = rng.uniform(0.1, 3.0, (nz, ny, nx))
    B = rng.uniform(0.5, 2.0, (nz, ny, nx))
    J_orc, Iem_orc = orc.formal_solution(chi, S, 8, 8, I_top=0.2, I_bot=B[0], want_emergent=True)
    with R.Solver(nx, ny, nz, 8, 8, I_top=0.2) as s:
        s.set_medium(chi, np.full_like(chi, 0.5), B)
        J = s.formal_solution(S)
        Iem = s.emergent_top()
    _close(J, J_orc)
    _close(Iem, Iem_orc)


def test_sampled_timing_counts(R):
    """Timing mode 2 (the benchmark's): per OS step one timed source, sweep and reduction launch and
    the M - 2 intermediate Jacobi sweeps as one group; mode 1 times every launch; results unchanged."""
    m = random_medium(9, 8, 7, seed=51)
    J = {}
    for mode in (0, 1, 2):
        with R.Solver(9, 8, 7, 4, 8) as s:
            s.set_medium(m["chi"], m["eps"], m["B"])
            s.build_lstar()
            s.set_timing(mode)
            for _ in range(3):
                s.os_step(6)
            st = s.stats()
            J[mode] = s.get_J()
        k = st["kernels"]
        assert st["timing"] == mode
        assert k["sweep"]["launches"] == 3 and k["jacobi"]["launches"] == 18
        if mode == 1:
            assert k["sweep"]["timed"] == 3 and k["jacobi"]["timed"] == 18
        elif mode == 2:
            assert k["sweep"]["timed"] == 3 and k["reduce"]["timed"] == 3 and k["jacobi"]["timed"] == 3 * 4
            assert k["jacobi"]["total_ms"] > 0
        else:
            assert k["sweep"]["timed"] == 0 and k["jacobi"]["total_ms"] == 0
    assert np.array_equal(J[0], J[1]) and np.array_equal(J[0], J[2])


def test_stats_report_the_sweep_plan(R):
    """rt3d_get_stats names the sweep plan's largest window and a sweep workgroup's LDS: within the
    48 KB budget for a grid whose bands fit it, in the wide budget (one workgroup per CU) for one
    that needs it; float32 sweeps take half the bytes."""
    with R.Solver(300, 4, 3, 16, 16) as s:
        st = s.stats()
        assert 0 < st["sweep_lds_bytes"] <= 48 * 1024 and st["max_window_rows"] > 0
    with R.Solver(520, 5, 4, 16, 16) as s:
        assert 48 * 1024 < s.stats()["sweep_lds_bytes"] <= 156 * 1024
    with R.Solver(520, 5, 4, 16, 16, precision=R.RT3D_FP32_SWEEP) as s:
        assert s.stats()["sweep_lds_bytes"] <= 78 * 1024
