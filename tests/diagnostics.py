"""Post-processing used by the tests (not part of the method or the GPU path).

Contact-angle measurement (Sec. III A): the interface phi = 1/2 is located at
sub-cell precision by linear interpolation along grid lines, fitted with an
algebraic least-squares sphere (or, in the paper's literal variant, a circle in
a vertical section, Eq. (56)), and the angle follows from the fitted centre
height above the wall position z_w (Eq. (57)): theta = pi - acos((z0 - z_w)/R).
"""
import numpy as np


def interface_points(phi3, level=0.5, zmin=1.0):
    """Sub-cell crossings of `level` along x, y and z grid lines.
    phi3 is indexed [z, y, x]; returns an (n, 3) array of (x, y, z)."""
    pts = []
    nz, ny, nx = phi3.shape
    for axis in range(3):
        a = phi3
        b = np.roll(phi3, -1, axis=axis)
        s = (a - level) * (b - level) < 0
        # do not interpolate across the periodic seam
        idx = [slice(None)] * 3
        idx[axis] = -1
        s[tuple(idx)] = False
        zz, yy, xx = np.nonzero(s)
        t = (level - a[s]) / (b[s] - a[s])
        p = np.stack([xx, yy, zz], axis=1).astype(float)
        p[:, 2 - axis] += t
        pts.append(p)
    p = np.concatenate(pts)
    return p[p[:, 2] >= zmin]


def fit_sphere(p):
    """Algebraic least squares: |x|^2 = 2 c.x + (R^2 - |c|^2)."""
    A = np.column_stack([2 * p, np.ones(len(p))])
    b = (p ** 2).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    c = sol[:3]
    R = np.sqrt(sol[3] + c @ c)
    return c, R


def fit_circle(p2):
    A = np.column_stack([2 * p2, np.ones(len(p2))])
    b = (p2 ** 2).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    c = sol[:2]
    return c, np.sqrt(sol[2] + c @ c)


def contact_angle_sphere(phi, shape, z_w=0.5, zmin=None):
    """Angle (degrees) of a sessile droplet on the bottom wall from a sphere fit."""
    nx, ny, nz = shape
    phi3 = np.asarray(phi, dtype=np.float64).reshape(nz, ny, nx).copy()
    phi3[0] = phi3[1]  # exclude the ghost layer from the crossings
    p = interface_points(phi3, zmin=(z_w + 1.0) if zmin is None else zmin)
    p = p[p[:, 2] < nz / 2 + 0.0]  # bottom droplet only
    c, R = fit_sphere(p)
    arg = np.clip((c[2] - z_w) / R, -1.0, 1.0)
    return float(np.degrees(np.pi - np.arccos(arg))), c, R


def contact_angle_section(phi, shape, y_plane, z_w=0.5, eps_fit=0.1):
    """Paper-literal variant: points with |phi - 1/2| < eps_fit in the vertical
    plane y = y_plane, circle fit, Eq. (57)."""
    nx, ny, nz = shape
    phi3 = np.asarray(phi).reshape(nz, ny, nx)
    sec = phi3[:, y_plane, :]
    zz, xx = np.nonzero(np.abs(sec - 0.5) < eps_fit)
    keep = zz >= 1
    c, R = fit_circle(np.column_stack([xx[keep], zz[keep]]).astype(float))
    arg = np.clip((c[1] - z_w) / R, -1.0, 1.0)
    return float(np.degrees(np.pi - np.arccos(arg)))


def wetted_radius(phi, shape, z_layer=1):
    """r = sqrt(sum of phi over the first fluid layer / pi)."""
    nx, ny, nz = shape
    return float(np.sqrt(np.asarray(phi).reshape(nz, ny, nx)[z_layer].sum() / np.pi))


def liquid_floor(phi, shape, level=0.5):
    """Lowest fluid layer z >= 1 that holds a node with phi > level on the
    central column region, or nz when there is none (a drop that left the
    bottom wall has floor > 1)."""
    nx, ny, nz = shape
    phi3 = np.asarray(phi).reshape(nz, ny, nx)
    for z in range(1, nz // 2):
        if (phi3[z] > level).any():
            return int(z)
    return int(nz)
