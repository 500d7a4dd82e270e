"""The Lambda* parity bar shared by the GPU parity tests (a helper module, not a test file)."""
import numpy as np


def close_lstar(L, L_ref, chi, n_theta, rtol=1e-10, rel_above=1e-30):
    """Lambda* parity, two bars.  (1) Every entry within rtol of its voxel row's scale: |dL[o, v]| <=
    rtol * max_o' |L_ref[o', v]| (the row scale is what enters the operator-splitting sum).  (2) Every
    entry above rel_above of that scale (and above 1e-290, clear of subnormals) within a relative
    bound of its own: rtol plus the exponent rounding of two independent geometries.  Segment lengths
    are differences of crossing heights of size up to nz divided by |mu|, so each side rounds them to
    about eps nz / |mu|; an entry's exponent sums the optical depths of at most four segments in the
    3 x 3 x 3 block, so the two sides' exponents differ by at most 8 eps nz chi_max / mu_min, chi_max
    the largest opacity of the block (e.g. 2.7e-9 for the 65^3 Gaussian-random-field medium's
    thickest voxels, below 1e-10 for the small test media)."""
    scale = np.max(np.abs(L_ref), axis=0, keepdims=True)
    err = np.abs(L - L_ref)
    bad = err > rtol * scale + 1e-300
    assert not bad.any(), f"{bad.sum()} of {bad.size} off; worst {np.max(err / (scale + 1e-300)):.3e}"
    nz = chi.shape[0]
    mu_min = np.min(np.abs(np.polynomial.legendre.leggauss(n_theta)[0]))
    cmax = chi.copy()
    for ax in range(3):
        lo = np.concatenate([cmax.take([0], axis=ax), cmax], axis=ax) if ax == 0 else np.roll(cmax, 1, axis=ax)
        hi = np.concatenate([cmax, cmax.take([-1], axis=ax)], axis=ax) if ax == 0 else np.roll(cmax, -1, axis=ax)
        if ax == 0:
            lo, hi = lo[:-1], hi[1:]
        cmax = np.maximum(cmax, np.maximum(lo, hi))
    tol = rtol + 8 * np.finfo(float).eps * nz * cmax / mu_min
    tol = np.broadcast_to(tol, L_ref.shape)
    big = (np.abs(L_ref) >= rel_above * scale) & (np.abs(L_ref) > 1e-290)
    rel = err[big] / np.abs(L_ref[big])
    off = rel > tol[big]
    assert big.sum() > 0 and not off.any(), (
        f"{int(off.sum())} of {int(big.sum())} entries above {rel_above:g} of their row off; "
        f"worst rel {rel.max():.3e} against a bound of {tol[big][np.argmax(rel)]:.3e}")
