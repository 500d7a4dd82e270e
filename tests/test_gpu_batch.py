"""GPU tests of the batched form (many problems, one launch per kernel, graph-replayed iteration).

The batch runs the single-problem arithmetic with device-side control, so its results are compared
*bitwise* with single contexts of the same sweep shape (formal solutions, whole solves with and
without Ng, FP64 and FP32 forms, iteration counts and stop states); one member is also compared with
the FP64 oracle at the parity bar (rel 1e-10).  The autotuner is checked for a working cache.
"""
import json

import numpy as np
import pytest

from paper_1107_5719_amd.inputs import diffusion_medium, random_medium, wavelength_batch

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


def _members(seed=0):
    """Ragged members: different sizes, angle sets, boundary light and media."""
    out = []
    specs = [((6, 7, 9), 4, 8, 0.2, 0), ((9, 12, 10), 8, 8, 0.0, 2), ((5, 5, 5), 4, 4, 0.0, 1),
             ((8, 33, 20), 8, 16, 0.1, 0)]
    for i, (shape, nt, nph, I_top, bbc) in enumerate(specs):
        nz, ny, nx = shape
        make = diffusion_medium if bbc == 2 else random_medium
        m = make(nx, ny, nz, seed=100 + seed + i, chi_range=(1e-3, 3e1), eps_range=(1e-3, 0.5))
        out.append({"grid": {"nx": nx, "ny": ny, "nz": nz, "n_theta": nt, "n_phi": nph, "I_top": I_top,
                             "bottom_bc": bbc}, "chi": m["chi"], "eps": m["eps"], "B": m["B"]})
    return out


def _single(R, g, precision, shape=0):
    s = R.Solver(g["nx"], g["ny"], g["nz"], g["n_theta"], g["n_phi"], I_top=g.get("I_top", 0.0),
                 bottom_bc=g.get("bottom_bc", 0), precision=precision)
    s.set_sweep_shape(shape)
    return s


# sweep shapes the batched tests run: the default one and 256 x 2, which the autotuner picks for the
# benchmark's 64-wavelength batch (each shape is its own kernel instantiation)
SHAPES = [0, 5]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"shape{x}" for x in SHAPES])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_sweep"])
def test_batch_formal_solution_bitwise(R, precision, shape):
    mem = _members()
    with R.Batch([m["grid"] for m in mem], precision=precision, sweep_shape=shape) as b:
        for i, m in enumerate(mem):
            b.set_medium(i, m["chi"], m["eps"], m["B"])
            b.set_J(i, m["B"] * 0.5 + 0.25)
        b.formal_solution()
        got = [b.get_Jfs(i) for i in range(len(mem))]
    for i, m in enumerate(mem):
        with _single(R, m["grid"], precision, shape) as s:
            s.set_medium(m["chi"], m["eps"], m["B"])
            s.set_J(m["B"] * 0.5 + 0.25)
            ref = s.formal_solution()
        assert np.array_equal(got[i], ref), f"member {i}: max diff {np.max(np.abs(got[i] - ref))}"


@pytest.mark.parametrize("shape", SHAPES, ids=[f"shape{x}" for x in SHAPES])
@pytest.mark.parametrize("precision,ng", [(0, (0, 0)), (0, (2, 4)), (1, (0, 0)), (1, (3, 6)), (0, "aa5"),
                                          (1, "aa3")],
                         ids=["fp64", "fp64-ng2", "fp32", "fp32-ng3", "fp64-aa5", "fp32-aa3"])
def test_batch_solve_bitwise(R, precision, ng, shape):
    """Every member of the batched solve takes bitwise the steps of solving it alone (Ng, or Anderson
    mixing with the window kept per member on the device)."""
    mem = _members(seed=7)
    tol, max_iter, M = 1e-9, 300, 6

    def accelerate(x):
        if isinstance(ng, str):
            x.set_anderson(int(ng[2:]))
        elif ng[0]:
            x.set_acceleration(*ng)

    with R.Batch([m["grid"] for m in mem], precision=precision, sweep_shape=shape) as b:
        for i, m in enumerate(mem):
            b.set_medium(i, m["chi"], m["eps"], m["B"])
        accelerate(b)
        st, iters, cs, states = b.solve(tol, max_iter, M, poll_every=3)
        Jb = [b.get_J(i) for i in range(len(mem))]
    assert st == R.RT3D_OK
    assert (states == R.RT3D_MEMBER_CONVERGED).all()
    for i, m in enumerate(mem):
        with _single(R, m["grid"], precision, shape) as s:
            s.set_medium(m["chi"], m["eps"], m["B"])
            accelerate(s)
            st1, it1, c1 = s.solve(tol, max_iter, M)
            J1 = s.get_J()
        assert st1 == R.RT3D_OK
        assert iters[i] == it1, f"member {i}: {iters[i]} vs {it1} iterations"
        assert cs[i] == c1
        assert np.array_equal(Jb[i], J1), f"member {i}: max diff {np.max(np.abs(Jb[i] - J1))}"


def test_batch_acceleration_setters_replace_each_other(R):
    """Ng and Anderson settings replace each other on the batch as on a context (each frees the
    other's member buffers): switching back and forth, or off, solves like a batch that was set so
    from the start."""
    mem = _members(seed=11)
    grids = [m["grid"] for m in mem]

    def solve(setup):
        with R.Batch(grids) as b:
            for i, m in enumerate(mem):
                b.set_medium(i, m["chi"], m["eps"], m["B"])
            setup(b)
            st, iters, cs, states = b.solve(1e-9, 400, 5, poll_every=4)
            assert st == R.RT3D_OK
            return iters.copy(), [b.get_J(i) for i in range(len(mem))]

    plain = solve(lambda b: None)
    ng = solve(lambda b: b.set_acceleration(3, 6))
    aa = solve(lambda b: b.set_anderson(4))
    for want, setup in ((plain, lambda b: (b.set_anderson(4), b.set_acceleration(0, 0))),
                        (plain, lambda b: (b.set_acceleration(3, 6), b.set_anderson(0))),
                        (ng, lambda b: (b.set_anderson(4), b.set_acceleration(3, 6))),
                        (aa, lambda b: (b.set_acceleration(3, 6), b.set_anderson(4)))):
        got = solve(setup)
        assert np.array_equal(got[0], want[0])
        for a, c in zip(got[1], want[1]):
            assert np.array_equal(a, c)
    with R.Batch(grids) as b:
        with pytest.raises(R.Rt3dError):
            b.set_anderson(9)


def test_batch_poll_interval_does_not_change_iterates(R):
    mem = _members(seed=3)
    res = []
    for poll in (1, 5):
        with R.Batch([m["grid"] for m in mem]) as b:
            for i, m in enumerate(mem):
                b.set_medium(i, m["chi"], m["eps"], m["B"])
            b.set_acceleration(2, 4)
            st, iters, cs, states = b.solve(1e-9, 300, 5, poll_every=poll)
            stats = b.stats()
            res.append((iters.copy(), [b.get_J(i) for i in range(len(mem))]))
        assert stats["replays"] >= iters.max()
        assert stats["polls"] >= 1
    assert np.array_equal(res[0][0], res[1][0])
    for a, c in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, c)


def test_batch_member_matches_oracle(R, orc):
    """A member of a ragged batch against the FP64 oracle's converged solution."""
    mem = wavelength_batch(n=3, sizes=(9, 13), n_theta=4, n_phi=8, eps_range=(1e-3, 1e-1))
    tol = 1e-12
    with R.Batch([m["grid"] for m in mem]) as b:
        for i, m in enumerate(mem):
            b.set_medium(i, m["chi"], m["eps"], m["B"])
        st, iters, cs, states = b.solve(tol, 2000, 10, poll_every=8)
        Jb = [b.get_J(i) for i in range(len(mem))]
    assert st == R.RT3D_OK
    for i, m in enumerate(mem):
        g = m["grid"]
        J_orc, it_o, c_o, ok = orc.solve(m["chi"], m["eps"], m["B"], g["n_theta"], g["n_phi"], tol, 2000, 10)
        assert ok
        assert it_o == iters[i], f"member {i}: {iters[i]} vs oracle {it_o} iterations"
        err = np.max(np.abs(Jb[i] - J_orc) / np.abs(J_orc))
        assert err <= RTOL, f"member {i}: rel err {err:.3e}"


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_sweep"])
def test_batch_real_size_members_match_oracle(R, orc, precision):
    """Members of the benchmark's many-wavelength workload (its first three wavelengths, 64 angles: a
    33^3, a 65^3 and a 97^3 grid with their drawn chi0 and eps), batched with the benchmark's settings (sweep shape 256 x 2, M = 8,
    Ng order 3 every 6 steps) for a fixed number of iterations: the 33^3 member against the oracle's
    iterate after the same steps (FP64 form 1e-10, FP32-sweep form 1e-5)."""
    allm = wavelength_batch(3)          # the workload's first three wavelengths: 33^3, 97^3, 65^3
    pick = sorted(allm, key=lambda m: m["grid"]["nx"])
    assert [m["grid"]["nx"] for m in pick] == [33, 65, 97]
    steps, M = 12, 8
    with R.Batch([m["grid"] for m in pick], precision=precision, sweep_shape=5) as b:
        for i, m in enumerate(pick):
            b.set_medium(i, m["chi"], m["eps"], m["B"])
        b.set_acceleration(3, 6)
        st, iters, cs, states = b.solve(1e-300, steps, M, poll_every=4, check=False)
        J33 = b.get_J(0)
    assert (iters == steps).all() and (states == R.RT3D_MEMBER_MAX_ITER).all()
    m, g = pick[0], pick[0]["grid"]
    J_orc, it_o, c_o, ok = orc.solve_ng(m["chi"], m["eps"], m["B"], g["n_theta"], g["n_phi"], 1e-300, steps, M,
                                        3, 6)
    assert it_o == steps
    err = np.max(np.abs(J33 - J_orc) / np.abs(J_orc))
    bar = RTOL if precision == 0 else 1e-5
    assert err <= bar, f"33^3 member after {steps} steps: rel err {err:.3e} (eps {m['eps'].flat[0]:.2e})"
    print(f"33^3 member (eps {m['eps'].flat[0]:.3e}): max rel error {err:.3e} after {steps} steps")


def test_batch_stop_states_and_errors(R):
    mem = _members(seed=11)
    grids = [m["grid"] for m in mem]
    with R.Batch(grids) as b:
        assert len(b) == len(mem) and R.rt3d_batch_size(b.b) == len(mem)
        with pytest.raises(R.Rt3dError) as e:
            b.solve(1e-8, 10, 4)
        assert e.value.status == R.RT3D_ERR_STATE          # no medium yet
        with pytest.raises(R.Rt3dError) as e:
            b.set_medium(len(mem), mem[0]["chi"], mem[0]["eps"], mem[0]["B"])
        assert e.value.status == R.RT3D_ERR_ARG
        bad = mem[1]["chi"].copy()
        bad[0, 0, 0] = -1.0
        with pytest.raises(R.Rt3dError) as e:
            b.set_medium(1, bad, mem[1]["eps"], mem[1]["B"])
        assert e.value.status == R.RT3D_ERR_ARG and "member 1" in str(e.value)
        for i, m in enumerate(mem):
            b.set_medium(i, m["chi"], m["eps"], m["B"])
        for args in [(0.0, 10, 4, 1), (1e-8, 0, 4, 1), (1e-8, 10, 0, 1), (1e-8, 10, 4, 0)]:
            with pytest.raises(R.Rt3dError) as e:
                b.solve(*args)
            assert e.value.status == R.RT3D_ERR_ARG
        st, iters, cs, states = b.solve(1e-14, 3, 2, poll_every=2, check=False)
        assert st == R.RT3D_ERR_NOT_CONVERGED
        assert (states == R.RT3D_MEMBER_MAX_ITER).all() and (iters == 3).all()
        assert np.isfinite(cs).all()
        # resuming continues from the stored iterate, exactly as a single context does
        st2, iters2, cs2, _ = b.solve(1e-14, 2, 2, check=False)
        J_b = b.get_J(0)
        with pytest.raises(R.Rt3dError) as e:
            b.set_sweep_shape(99)
        assert e.value.status == R.RT3D_ERR_ARG
    with _single(R, grids[0], 0) as s:
        s.set_medium(mem[0]["chi"], mem[0]["eps"], mem[0]["B"])
        s.solve(1e-14, 3, 2)
        s.solve(1e-14, 2, 2)
        assert np.array_equal(s.get_J(), J_b)
    with pytest.raises(R.Rt3dError):
        R.Batch([])
    with pytest.raises(R.Rt3dError) as e:
        R.Batch([dict(grids[0], n_phi=6)])
    assert "member 0" in str(e.value)
    # a member wider than the sweep's LDS allows (nx > 832 at 32 x 32 angles) names itself
    with pytest.raises(R.Rt3dError) as e:
        R.Batch([grids[0], dict(nx=833, ny=4, nz=3, n_theta=32, n_phi=32)])
    assert e.value.status == R.RT3D_ERR_ARG and "member 1" in str(e.value) and "LDS" in str(e.value)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32_sweep"])
def test_set_sweep_shape_changes_only_rounding(R, orc, precision):
    """Every sweep shape gives J_fs within rounding of every other (float64: 1e-13; float32 sweeps:
    1e-6, each shape's float32 window sums split differently across bands) and of the oracle."""
    m = random_medium(14, 11, 9, seed=5, chi_range=(1e-3, 1e1))
    S = m["eps"] * m["B"] + (1 - m["eps"]) * m["B"]
    J_orc = orc.formal_solution(m["chi"], S, 8, 8, I_bot=m["B"][0])
    J = {}
    for shape in range(len(R.rt3d_sweep_shapes())):
        with R.Solver(14, 11, 9, 8, 8, precision=precision) as s:
            s.set_medium(m["chi"], m["eps"], m["B"])
            s.set_sweep_shape(shape)
            assert s.stats()["sweep_shape"] == shape
            J[shape] = s.formal_solution()
    rtol = 1e-13 if precision == 0 else 1e-6
    for shape, x in J.items():
        np.testing.assert_allclose(x, J[0], rtol=rtol, atol=0)
        np.testing.assert_allclose(x, J_orc, rtol=1e-10 if precision == 0 else 1e-5, atol=0)


def test_autotune_cache(R, tmp_path):
    path = tmp_path / "tune.json"
    m = random_medium(17, 17, 17, seed=9)
    with R.Solver(17, 17, 17, 4, 8) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        shape, ms = s.autotune(str(path), repeats=2)
        assert 0 <= shape < len(ms) and ms[shape] > 0 and ms[shape] == ms[ms > 0].min()
        assert s.stats()["sweep_shape"] == shape
    data = json.loads(path.read_text())
    (key, entry), = data.items()
    assert "17x17x17|4x8" in key and "fp64" in key and entry["shape"] == shape
    with R.Solver(17, 17, 17, 4, 8) as s:
        s.set_medium(m["chi"], m["eps"], m["B"])
        shape2, ms2 = s.autotune(str(path), repeats=2)
        assert shape2 == shape and (ms2 == -1).all()
    mem = _members()
    with R.Batch([x["grid"] for x in mem]) as b:
        for i, x in enumerate(mem):
            b.set_medium(i, x["chi"], x["eps"], x["B"])
        bshape, bms = b.autotune(str(path), repeats=2)
        assert b.stats()["sweep_shape"] == bshape and bms[bshape] > 0
        b.solve(1e-8, 200, 4)
    data = json.loads(path.read_text())
    assert len(data) == 2 and any("|batch|" in k for k in data)
