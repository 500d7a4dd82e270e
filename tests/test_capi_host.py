"""Host-only checks of the C ABI (no GPU needed): the library loads and exports every symbol that
include/rt3d.h declares; its own angle set and segment tables agree with the oracle's independent
ones; argument validation rejects bad descriptors and media before any device work."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def R():
    from paper_1107_5719_amd import rt3d

    return rt3d


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            decl = r"^(?:int|void|const char)\s*\*?\s*(rt3d_[A-Za-z_0-9]+)\s*\("
            names |= set(re.findall(decl, txt, flags=re.M))
    return names


def test_every_declared_symbol_is_exported(R):
    decl = _declared_symbols()
    assert len(decl) >= 18
    lib = R.library()
    for name in sorted(decl):
        assert hasattr(lib, name), name
    assert decl == set(R.EXPORTED)


@pytest.mark.parametrize("nt,nph", [(2, 4), (8, 8), (16, 16), (4, 12)])
def test_quadrature_matches_oracle(R, orc, nt, nph):
    lib_q = R.rt3d_quadrature(nt, nph)
    orc_q = orc.quadrature(nt, nph)
    for a, b in zip(lib_q, orc_q):
        assert np.max(np.abs(a - b)) < 1e-15


def _merge_same_voxel(v, l, sliver=1e-12):
    """Drop rounding-sized pieces (a line through a voxel edge touches the side voxels in a point;
    rounding decides whether a 1e-15 piece appears there) and join consecutive pieces inside one voxel
    (the exact integral over a voxel does not depend on how its path is split)."""
    mv, ml = [], []
    for a, b in zip(v, l):
        if b <= sliver:
            continue
        if mv and mv[-1] == a:
            ml[-1] += b
        else:
            mv.append(int(a))
            ml.append(float(b))
    return np.array(mv), np.array(ml)


@pytest.mark.parametrize("shape,nt,nph", [((5, 6, 7), 8, 8), ((4, 3, 5), 16, 16), ((6, 9, 9), 16, 16),
                                          ((5, 6, 7), 2, 4), ((5, 5, 5), 8, 4)])
def test_segment_tables_match_oracle_lines(R, orc, shape, nt, nph):
    """The library's one table per (direction, layer), translated to line (i,j), equals the oracle's
    own tracing of that line (n_phi = 4: every line runs through voxel edges)."""
    nz, ny, nx = shape
    desc = R._desc(nx, ny, nz, nt, nph)
    rng = np.random.default_rng(0)
    for d in range(nt * nph):
        for k in range(nz):
            di, dj, ln = R.rt3d_segment_table(desc, d, k)
            assert abs(ln.sum() * abs(orc.quadrature(nt, nph)[0][d]) - 1) < 1e-13
            for _ in range(3):
                i, j = int(rng.integers(nx)), int(rng.integers(ny))
                v, l = _merge_same_voxel(*orc.trace_layer(nx, ny, nz, nt, nph, d, i, j, k))
                vv, ll = _merge_same_voxel((k * ny + (j + dj) % ny) * nx + (i + di) % nx, ln)
                assert np.array_equal(v, vv)
                assert np.max(np.abs(l - ll)) < 1e-12


@pytest.mark.parametrize("nt,nph", [(2, 4), (8, 4), (8, 8), (4, 12)])
def test_mirrored_directions_share_tables(R, nt, nph):
    """Directions mirrored in x (phi -> pi - phi) have the same tables with negated columns, which is
    what lets one sweep workgroup carry both (n_phi = 4 included, where lines pass through edges)."""
    nz, ny, nx = 6, 5, 7
    desc = R._desc(nx, ny, nz, nt, nph)
    mu, ox, oy, _ = R.rt3d_quadrature(nt, nph)
    for a in range(nt):
        for b in range(nph):
            d = a * nph + b
            dm = [e for e in range(a * nph, (a + 1) * nph) if ox[e] == -ox[d] and oy[e] == oy[d]]
            assert len(dm) == 1
            for k in range(nz):
                di, dj, ln = R.rt3d_segment_table(desc, d, k)
                di2, dj2, ln2 = R.rt3d_segment_table(desc, dm[0], k)
                assert np.array_equal(di, -di2) and np.array_equal(dj, dj2) and np.array_equal(ln, ln2)
                assert (ln > 1e-9).all()


def test_deposits_are_a_bijection_per_segment(R):
    """For a fixed (direction, layer, segment index) the map line -> voxel is a bijection of the
    layer, which is what lets the sweep deposit without atomics."""
    nx, ny, nz = 7, 5, 4
    desc = R._desc(nx, ny, nz, 16, 16)
    for d in range(256):
        for k in range(nz):
            di, dj, _ = R.rt3d_segment_table(desc, d, k)
            for s in range(len(di)):
                jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
                vox = ((jj + dj[s]) % ny) * nx + (ii + di[s]) % nx
                assert len(np.unique(vox)) == nx * ny


def test_validation_reports_the_sweep_size_limits(R):
    """A grid wider than the sweep kernel's budgets (whole x-rows per workgroup; a deposit window of
    rows + row spread and two exchange rows per line row in 156 KB of LDS) is rejected on the host, by
    rt3d_validate and by rt3d_create before any device allocation, with the reason in
    rt3d_last_error(NULL).  Below that the widths of wide grids (300 and 520 at 16 x 16 angles) are
    accepted."""
    for nx in (257, 300, 520):
        assert R.rt3d_validate(R._desc(nx, 5, 4, 16, 16)) == R.RT3D_OK
    for nt, nph, nmax in ((16, 16, 1024), (24, 24, 1024), (32, 32, 832), (48, 48, 587), (8, 8, 1024), (2, 4, 1024)):
        assert R.rt3d_validate(R._desc(nmax, 4, 3, nt, nph)) == R.RT3D_OK
        assert R.rt3d_last_error(None) == ""
        assert R.rt3d_validate(R._desc(nmax + 1, 4, 3, nt, nph)) == R.RT3D_ERR_ARG
        msg = R.rt3d_last_error(None)
        assert ("LDS" in msg) or ("lines" in msg), msg
        with pytest.raises(R.Rt3dError) as e:
            R.rt3d_create(R._desc(nmax + 1, 4, 3, nt, nph), R.RT3D_FP64, 0)
        assert e.value.status == R.RT3D_ERR_ARG and msg in str(e.value)
    assert R.rt3d_validate(R._desc(2, 5, 5, 8, 8)) == R.RT3D_ERR_ARG
    assert "nx, ny, nz" in R.rt3d_last_error(None)


def test_failed_batch_creation_names_the_member(R):
    """rt3d_batch_create validates every member descriptor on the host, before any device work; the
    reason of the failure, naming the member, is in rt3d_batch_last_error(NULL)."""
    good, bad = R._desc(5, 5, 5, 8, 8), R._desc(5, 5, 5, 8, 6)
    with pytest.raises(R.Rt3dError) as e:
        R.rt3d_batch_create([good, bad], R.RT3D_FP64, 0)
    assert e.value.status == R.RT3D_ERR_ARG
    assert "member 1" in str(e.value) and "n_phi" in str(e.value)
    assert R.rt3d_batch_last_error(None).startswith("member 1")
    with pytest.raises(R.Rt3dError) as e:
        R.rt3d_batch_create([good], R.RT3D_FP64, 99)
    assert "sweep shape" in str(e.value)


def test_validation_rejects_bad_input(R):
    good = R._desc(5, 5, 5, 8, 8)
    assert R.rt3d_validate(good) == R.RT3D_OK
    for bad in (R._desc(2, 5, 5, 8, 8), R._desc(5, 5, 2, 8, 8), R._desc(5, 5, 5, 7, 8),
                R._desc(5, 5, 5, 0, 8), R._desc(5, 5, 5, 8, 6), R._desc(5, 5, 5, 8, 8, I_top=-1.0),
                R._desc(5, 5, 5, 8, 8, I_top=math.inf), R._desc(5, 5, 5, 8, 8, bottom_bc=3)):
        assert R.rt3d_validate(bad) == R.RT3D_ERR_ARG
        with pytest.raises(R.Rt3dError) as e:
            R.rt3d_create(bad, R.RT3D_FP64, 0)
        assert e.value.status == R.RT3D_ERR_ARG
    with pytest.raises(R.Rt3dError):
        R.rt3d_create(good, 7, 0)
    shape = (5, 5, 5)
    chi, eps, B = np.ones(shape), np.full(shape, 0.5), np.ones(shape)
    assert R.rt3d_validate(good, chi, eps, B) == R.RT3D_OK
    for name, val in (("chi", 0.0), ("chi", -1.0), ("chi", np.nan), ("chi", np.inf), ("eps", 0.0),
                      ("eps", 1.5), ("eps", np.nan), ("B", np.nan), ("B", -np.inf)):
        m = {"chi": chi.copy(), "eps": eps.copy(), "B": B.copy()}
        m[name][2, 1, 3] = val
        assert R.rt3d_validate(good, m["chi"], m["eps"], m["B"]) == R.RT3D_ERR_ARG, (name, val)
    assert R.rt3d_status_str(R.RT3D_ERR_NOT_CONVERGED) == "not converged"
    assert R.rt3d_status_str(R.RT3D_ERR_NONFINITE) == "non-finite value"
