"""Shared checks of GPU factors against the oracle (the A19 reading of the
1e-10 bar).

* Pivot sequences (perm, ipiv) bit-exact, on screened inputs: every top-two
  pivot gap >= 1e-5 in the oracle and no pivot at rounding level.
* Y within 1e-10 relative (Frobenius).
* L columns and U rows j whose predicted rounding u rho_j kappa^2 is at most
  1e-12 (u the FP64 unit roundoff) within ``tol`` relative, per column / row;
  every column and row on well-conditioned inputs.  The growth of step j of
  an LU is |d_0| / |d_j| over its U diagonal d; column j of L = L_y L~ and row
  j of U carry the rounding of both LUs and of every earlier step, so rho_j is
  the running maximum, over steps 0..j, of the larger of the two LUs' growth.
  kappa = kappa(L_y): the device forms B = L_y^+ P A through the normal
  equations, whose forward error grows like u kappa^2, where the oracle's
  Householder QR grows like u kappa, and B feeds every column of L~ and U.
* Everything else through the product, ||L_g U_g - L_o U_o||_F <= tol ||A||_F,
  formed in full, or on a sample of its entries when m n is too large.
* rlu_info's min_gap_* against the oracle's top-two gaps.
"""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def growth(diag):
    d = np.abs(diag)
    return d[0] / np.where(d > 0, d, np.inf)


U_ROUND = 2.0 ** -53
PREDICTED_MAX = 1e-12          # columns / rows held to the per-column bar: u rho_j kappa^2 <= this


def factor_growth(o):
    """Running maximum over steps 0..j of both LUs' growth (see above)."""
    return np.maximum.accumulate(np.maximum(growth(np.diag(o.Uy)), growth(np.diag(o.U))))


def check_gaps(info, o, tol=1e-6):
    """rlu_info's pivot screening against the oracle's top-two gaps.  The
    gaps are ratios of candidates that carry the rounding of the Schur
    complements they come from (growth up to 1e9 on screened inputs), so they
    agree to about 1e-7 at worst, not to the last bit."""
    for key in ("min_gap_y", "min_gap_b"):
        og, gg = getattr(o, key), info[key]
        if np.isinf(og):
            assert np.isinf(gg), (key, gg)
        else:
            assert abs(gg - og) <= tol, (key, gg, og)


def product_diff(Lg, Ug, Lo, Uo, a_fro, sample=None, seed=0):
    """||L_g U_g - L_o U_o||_F / ||A||_F; with ``sample`` = (rows, cols), on
    that many random rows and columns, scaled to the whole matrix."""
    m, n = Lg.shape[0], Ug.shape[1]
    if sample is None:
        return np.linalg.norm(Lg @ Ug - Lo @ Uo) / a_fro
    rng = np.random.default_rng(seed)
    I = np.sort(rng.choice(m, size=min(m, sample[0]), replace=False))
    J = np.sort(rng.choice(n, size=min(n, sample[1]), replace=False))
    d = Lg[I] @ Ug[:, J] - Lo[I] @ Uo[:, J]
    return np.linalg.norm(d) * np.sqrt((m * n) / (len(I) * len(J))) / a_fro


def compare_factors(A_fro, g, o, check_all_columns=False, tol=1e-10, sample=None, B=True):
    """g: rlu.Factorization (device), o: oracle Result.  ``A_fro``: ||A||_F
    (or the dense A itself); ``tol`` is the bar of the L columns, U rows and
    the product (Y stays at 1e-10)."""
    if not np.isscalar(A_fro):
        A_fro = np.linalg.norm(A_fro)
    np.testing.assert_array_equal(g.perm_r.cpu().numpy(), o.perm_r)
    np.testing.assert_array_equal(g.perm_c.cpu().numpy(), o.perm_c)
    np.testing.assert_array_equal(g.ipiv_r.cpu().numpy(), o.ipiv_r)
    np.testing.assert_array_equal(g.ipiv_c.cpu().numpy(), o.ipiv_c)
    Lg, Ug = g.L.cpu().numpy(), g.U.cpu().numpy()
    if g.Y is not None:
        assert rel_fro(g.Y.cpu().numpy(), o.Y) <= 1e-10
    if B and g.B is not None and check_all_columns:
        assert rel_fro(g.B.cpu().numpy(), o.B) <= tol
    kappa = np.linalg.cond(o.Ly)
    pred = U_ROUND * factor_growth(o) * kappa ** 2
    held = np.ones_like(pred, dtype=bool) if check_all_columns else pred <= PREDICTED_MAX
    worst = 0.0     # largest error per unit of prediction over the columns held (printed: the bar's margin)
    for j in np.flatnonzero(held):
        el, eu = rel_fro(Lg[:, j], o.L[:, j]), rel_fro(Ug[j], o.U[j])
        worst = max(worst, max(el, eu) / pred[j])
        assert el <= tol, (j, el, pred[j])
        assert eu <= tol, (j, eu, pred[j])
    print(f"per-column parity: kappa(L_y) {kappa:.3g}, {int(held.sum())} of {len(pred)} columns held, "
          f"max error / (u rho kappa^2) = {worst:.3g}")
    assert product_diff(Lg, Ug, o.L, o.U, A_fro, sample) <= tol
    check_gaps(g.info_dict(), o)


def screened(o):
    """Pivot choices robust to rounding: every top-two gap >= 1e-5, and no pivot
    down at rounding level (growth rho_j <= 1e9, so u * rho_j <= 1e-7)."""
    if o.min_gap_y < 1e-5 or o.min_gap_b < 1e-5:
        return False
    return growth(np.diag(o.Uy)).max() <= 1e9 and growth(np.diag(o.U)).max() <= 1e9


def screened_factor(A, k, l, s, seed, tries=20, csr=None, **kw):
    from oracle import rlu as R
    for sd in range(seed, seed + tries):
        o = R.rlu(A, R.Params(k, l, s, sd, **kw), csr=csr)
        if screened(o):
            return sd, o
    raise RuntimeError("no screened seed")
