"""Oracle: fan-beam scanner geometry (Section II-A, Table I and Eq. 2).

Test infrastructure only: the product never imports this package.

Rows of A are ordered view-major: row i = view * n_bins + bin, so M is the
number of detectors times the number of views (Section II-A, Eq. 1).
"""
import math
import numpy as np


def projection_angles_deg(v, schedule=1):
    """Projection angles Theta_1..Theta_v in degrees.

    schedule 1 follows Eq. 2: the views are split into quarters at floor(v/4),
    floor(v/2) and floor(3v/4); inside each quarter the angle advances by
    360/v, and at the start of quarters 2, 3 and 4 the schedule jumps by an
    extra +0.5, -0.75 and -0.25 degrees.  The printed equation is ambiguous
    about where each quarter restarts; the reading taken here continues every
    quarter from the last angle of the previous one (so Theta_i =
    Theta_{q_end} + shift + (360/v)(i - q_end)).  schedule 0 is the plain
    uniform schedule (360/v)(i - 1).
    """
    step = 360.0 / v
    theta = np.empty(v)
    if schedule == 0:
        for i in range(1, v + 1):
            theta[i - 1] = step * (i - 1)
        return theta
    q1, q2, q3 = v // 4, v // 2, (3 * v) // 4
    for i in range(1, v + 1):
        if i <= q1:
            t = step * (i - 1)
        elif i <= q2:
            t = theta[q1 - 1] + 0.5 + step * (i - q1)
        elif i <= q3:
            t = theta[q2 - 1] - 0.75 + step * (i - q2)
        else:
            t = theta[q3 - 1] - 0.25 + step * (i - q3)
        theta[i - 1] = t
    return theta


def ray_endpoints(geom):
    """Source points and detector-bin centres of every ray, both (M, 2) arrays.

    The source sits on the circle of radius src_iso_cm at angle Theta; the flat
    detector is perpendicular to the central ray at distance src_det_cm from the
    source; its n_bins equal bins span the fan, so bin b's centre lies at
    offset (b - (n_bins-1)/2) * pitch along the detector, pitch =
    2 * src_det_cm * tan(fan/2) / n_bins.
    """
    v, nb = geom["n_views"], geom["n_bins"]
    R, sdd = geom["src_iso_cm"], geom["src_det_cm"]
    half = math.radians(geom["fan_deg"]) / 2.0
    pitch = 2.0 * sdd * math.tan(half) / nb
    th = np.radians(projection_angles_deg(v, geom.get("angle_schedule", 1)))
    src = np.empty((v * nb, 2))
    dst = np.empty((v * nb, 2))
    for view in range(v):
        c, s = math.cos(th[view]), math.sin(th[view])
        sx, sy = R * c, R * s
        dcx, dcy = sx - sdd * c, sy - sdd * s          # detector centre
        ax, ay = -s, c                                  # detector axis
        for b in range(nb):
            u = (b - (nb - 1) / 2.0) * pitch
            i = view * nb + b
            src[i] = (sx, sy)
            dst[i] = (dcx + u * ax, dcy + u * ay)
    return src, dst


def image_grid(geom):
    """(x0, y0, delta): lower-left corner of the square image and pixel pitch."""
    L = geom["fov_side_cm"]
    return -L / 2.0, -L / 2.0, L / geom["side"]


def sizes(geom):
    """(M, N): rays x pixels."""
    return geom["n_views"] * geom["n_bins"], geom["side"] * geom["side"]
