"""Placement of adjoint lattices (test helper).

The GPU library keeps dJ/dx_i(x) at site x + c_i of plane i (the site where
population i of x arrives in the next streaming), i.e. nu = S lam with
nu_i(y) = lam_i(y - c_i).  These helpers convert between that placement and
plain per-site arrays (19, ny, nx), with the plane velocities of the D2Q9 and
D2Q5 lattices (Sec. 3 velocity lists: f_0..f_8, then the five vectors for the
x and for the y component of g).
"""
import numpy as np

CX = (0, 1, 0, -1, 0, 1, -1, -1, 1) + (0, 1, 0, -1, 0) * 2
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1) + (0, 0, 1, 0, -1) * 2


def streamed(lam):
    """nu_i(y) = lam_i(y - c_i), periodic over the last two axes (y, x)."""
    lam = np.asarray(lam)
    return np.stack([np.roll(lam[i], (CY[i], CX[i]), axis=(-2, -1)) for i in range(19)])


def unstreamed(nu):
    """lam_i(x) = nu_i(x + c_i): the inverse of streamed()."""
    nu = np.asarray(nu)
    return np.stack([np.roll(nu[i], (-CY[i], -CX[i]), axis=(-2, -1)) for i in range(19)])
