"""Test helpers for comparing Fiedler vectors element by element.

lambda23() gives the two smallest nonzero eigenvalues of a small connected
dual graph's Laplacian from a library routine (numpy's dense eigvalsh, or
scipy's shift-invert Lanczos above a few thousand rows), so that a vector
comparison can use the spectral gap.  The Laplacian is assembled here from
the oracle's CSR as D - A (Sec. 4 of the paper).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla


def laplacian(rp, col, w):
    n = len(rp) - 1
    A = sp.csr_matrix((np.asarray(w, dtype=np.float64), np.asarray(col), np.asarray(rp)),
                      shape=(n, n))
    return (sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A).tocsc()


def lambda23(orc, ids, graph="weighted"):
    """(lambda_2, lambda_3) of a connected mesh's dual-graph Laplacian."""
    rp, col, w = orc.dual_graph(ids, graph=graph)
    L = laplacian(rp, col, w)
    if L.shape[0] <= 3000:
        ev = np.linalg.eigvalsh(L.toarray())[:3]
    else:
        ev = np.sort(sla.eigsh(L, k=3, sigma=-1e-3, which="LM", return_eigenvectors=False))
    assert abs(ev[0]) < 1e-8 * max(1.0, ev[2]) and ev[1] > 1e-8, ev  # connected
    return float(ev[1]), float(ev[2])


def assert_fiedler_close(y, oy, res, ores, gap):
    """Element-wise agreement of two unit Fiedler vectors of a simple pair.

    A unit vector whose Rayleigh residual is r lies within an angle of
    asin(r / gap) of the eigenvector (Davis-Kahan sin-theta bound, gap = the
    distance from the Rayleigh quotient to the rest of the spectrum, here
    lambda_3 - lambda_2 up to rounding), so after aligning the signs
    max_i |y_i - oy_i| <= ||y - oy|| <= (r + r_oracle) / gap to first order.
    """
    y = np.asarray(y, dtype=np.float64)
    oy = np.asarray(oy, dtype=np.float64)
    if float(y @ oy) < 0:
        y = -y
    bound = 1.05 * (res + ores) / gap + 1e-13
    d = float(np.max(np.abs(y - oy)))
    assert d <= bound, f"max |y - oy| = {d:.3e} above the gap bound {bound:.3e}"
    return d, bound
