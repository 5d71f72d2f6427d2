"""Wall-unit bookkeeping for one-point statistics (host logic, no GPU).

Paper: Sec. 4, Table "stats": box sizes and grid spacings in wall units,
x+ = Re_tau x for lengths scaled by the half width h, with Re_tau = h u_tau / nu.
Streamwise/spanwise spacings are the box length over the number of +- Fourier
components kept after de-aliasing; the wall-normal spacing is that of the
Chebyshev-Gauss-Lobatto grid next to the wall and at the centreline.
"""

import math


def wall_units(re_tau, Lx, Lz, nx_components, nz_components, My):
    dy_wall = 1.0 - math.cos(math.pi / (My - 1))
    # spacing of the two nodes closest to y = 0
    ys = sorted(-math.cos(math.pi * j / (My - 1)) for j in range(My))
    mid = min(range(My - 1), key=lambda j: abs(ys[j] + ys[j + 1]))
    dy_centre = ys[mid + 1] - ys[mid]
    if My % 2 == 1:
        centre = My // 2
        dy_centre = ys[centre + 1] - ys[centre]
    return {
        "Lx+": re_tau * Lx, "Ly+": re_tau * 2.0, "Lz+": re_tau * Lz,
        "dx+": re_tau * Lx / nx_components, "dz+": re_tau * Lz / nz_components,
        "dywall+": re_tau * dy_wall, "dycentre+": re_tau * dy_centre,
    }


def re_tau_from_wall_shear(Re, dUdy_wall):
    """Re_tau = Re sqrt(tau_w) with tau_w = |dU/dy|_wall / Re (nu = 1/Re, h = 1)."""
    return Re * math.sqrt(abs(dUdy_wall) / Re)
