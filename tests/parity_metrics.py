"""Error measures of the GPU-versus-oracle parity tests.

Field-wide relative 2-norms hide errors confined to modes that are small
next to the field's largest one (the top kx or kz column, the Hermitian
n_x = 0 column, one member tile).  `mode_errors` therefore judges every
(member, n_x, n_z) on its own y-profile:

    err_k = ||a_k - b_k||_y / max(||b_k||_y, floor * max_k ||b_k||_y)

with floor = 1e-12, and reports the largest.  FP64 arithmetic leaves every
mode an absolute error of a few hundred roundings of the field's largest
mode (transforms and products mix all modes), so a mode far below the
largest one cannot be held to a relative bar; `mode_check` bounds each
mode's error by  rel_bar * ||b_k||_y + abs_bar * max_k ||b_k||_y  instead,
where abs_bar = 1e-13 (about 500 FP64 roundings).  A slip confined to one
mode moves that mode by its own size, far above either term.
"""

import numpy as np

MODE_FLOOR = 1e-12
ABS_BAR = 1e-13


def rel(a, b):
    """Relative 2-norm over every element."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def _ynorm(a):
    return np.sqrt(np.sum(np.abs(a) ** 2, axis=-1))


def mode_errors(a, b, floor=MODE_FLOOR):
    """Largest per-(member, n_x, n_z) relative error over y of state-layout
    arrays (E, Nx/2, Nz-1, N); each mode normalised by its own norm, floored
    at `floor` of the largest mode norm.  Returns (max error, its index)."""
    na = _ynorm(a - b)
    nb = _ynorm(b)
    top = nb.max()
    if top == 0.0:
        return float(na.max()), None
    r = na / np.maximum(nb, floor * top)
    idx = np.unravel_index(np.argmax(r), r.shape)
    return float(r[idx]), tuple(int(i) for i in idx)


def mode_check(a, b, rel_bar, abs_bar=ABS_BAR):
    """Worst ratio err_k / (rel_bar ||b_k|| + abs_bar max ||b_k||) over modes
    (<= 1 passes) and the mode attaining it."""
    na = _ynorm(a - b)
    nb = _ynorm(b)
    top = nb.max()
    allow = rel_bar * nb + abs_bar * (top if top > 0 else 1.0)
    r = na / allow
    idx = np.unravel_index(np.argmax(r), r.shape)
    return float(r[idx]), tuple(int(i) for i in idx)


def profile_check(a, b, rel_bar, abs_bar=ABS_BAR):
    """Per-member version of mode_check for (E, Ny) mean profiles."""
    na = np.sqrt(np.sum((a - b) ** 2, axis=-1))
    nb = np.sqrt(np.sum(b ** 2, axis=-1))
    top = nb.max()
    allow = rel_bar * nb + abs_bar * (top if top > 0 else 1.0)
    r = na / allow
    return float(r.max()), int(np.argmax(r))


def hermitian_defect(a):
    """max |f(0, n_z) - conj f(0, -n_z)| over the stored n_x = 0 column of a
    state-layout array (E, Nx/2, Nz-1, N), relative to max |f|."""
    nz_count = a.shape[2]
    P = (nz_count + 1) // 2
    iz = np.arange(nz_count)
    nz = np.where(iz < P, iz, iz - nz_count)
    mirror = (-nz) % nz_count
    col = a[:, 0]
    d = np.abs(col - np.conj(col[:, mirror])).max()
    top = np.abs(a).max()
    return float(d / (top if top > 0 else 1.0))


def state_report(got, ref_state, lam, rel_bar):
    """Field-wide relative errors, per-mode errors (floor 1e-12) and the
    mode_check / profile_check ratios of a (v, eta, U, W) state against the
    oracle's; lam is the laminar profile subtracted from U."""
    v, eta, U, W = got
    rv, reta, rU, rW = ref_state
    out = {
        "v": rel(v, rv), "eta": rel(eta, reta), "U-Ulam": rel(U - lam, rU - lam),
        "W": rel(W, rW) if np.any(rW) else float(np.abs(W).max()),
        "v/mode": mode_errors(v, rv)[0], "eta/mode": mode_errors(eta, reta)[0],
        "v/check": mode_check(v, rv, rel_bar)[0], "eta/check": mode_check(eta, reta, rel_bar)[0],
        "U/check": profile_check(U - lam, rU - lam, rel_bar)[0],
        "herm v": hermitian_defect(v), "herm eta": hermitian_defect(eta),
    }
    if np.any(rW):
        out["W/check"] = profile_check(W, rW, rel_bar)[0]
    return out


def assert_state(report, rel_bar):
    """Field-wide errors <= rel_bar, every mode within mode_check's bound,
    and the n_x = 0 column Hermitian to round-off."""
    for k in ("v", "eta", "U-Ulam", "W"):
        assert report[k] <= rel_bar, (k, report[k])
    for k in ("v/check", "eta/check", "U/check", "W/check"):
        if k in report:
            assert report[k] <= 1.0, (k, report[k])
    for k in ("herm v", "herm eta"):
        assert report[k] <= 1e-15, (k, report[k])
