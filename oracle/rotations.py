"""Rotations, cubic symmetry and disorientation in FP64 (oracle; test only).

Conventions (the paper defers frame conventions to a cited reference that is
not reproduced in it, so these are the readings used everywhere):

* A quaternion q = (w, x, y, z) with w >= 0 encodes the rotation matrix
  R(q) acting on column vectors (right-handed, active).
* An orientation R maps a direction d in the detector frame to the crystal
  direction c = R d.  Crystal symmetry S acts on crystal directions, so R and
  S R describe the same orientation.
* The disorientation between two orientations is the smallest rotation
  angle among all symmetry-equivalent misorientations (section "SO(3)
  Spacing", the disorientation equation, with the 24 proper cubic
  operators).  That equation is garbled in the text (a minimum over
  matrices, operators on both sides); the reading used is the minimum of the
  rotation angle, and one-sided operators suffice for a single phase since
  the angle is invariant under conjugation.
"""

import numpy as np

SQ = np.sqrt(0.5)


def quat_normalise(q):
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    return np.where(q[..., :1] < 0, -q, q)


def quat_to_matrix(q):
    """Rotation matrix of unit quaternion(s) q = (w, x, y, z), shape (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def matrix_to_quat(r):
    """Unit quaternion (w >= 0) of rotation matrix r (Shepperd's method)."""
    r = np.asarray(r, dtype=np.float64)
    flat = r.reshape(-1, 3, 3)
    out = np.empty((flat.shape[0], 4))
    for n, m in enumerate(flat):
        tr = m[0, 0] + m[1, 1] + m[2, 2]
        cand = np.array([tr, m[0, 0], m[1, 1], m[2, 2]])
        k = int(np.argmax(cand))
        if k == 0:
            s = 2.0 * np.sqrt(1.0 + tr)
            q = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif k == 1:
            s = 2.0 * np.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2])
            q = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif k == 2:
            s = 2.0 * np.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2])
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = 2.0 * np.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1])
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
        out[n] = q
    return quat_normalise(out).reshape(r.shape[:-2] + (4,))


def axis_angle_matrix(axis, angle):
    """Active right-handed rotation by `angle` (rad) about unit `axis` (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * k + (1 - np.cos(angle)) * (k @ k)


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def rotation_angle(m):
    """Rotation angle (rad) of rotation matrix m: acos(clamp((tr m - 1) / 2))."""
    tr = np.trace(m, axis1=-2, axis2=-1)
    return np.arccos(np.clip((tr - 1.0) / 2.0, -1.0, 1.0))


def cubic_operators():
    """The 24 proper rotations of the cubic point group 432 as matrices.

    Identity; 180 deg about <100> (3) and +-90 deg about <100> (6); +-120 deg
    about <111> (8); 180 deg about <110> (6).  Built from axes and angles, not
    from a quaternion table.
    """
    ops = [np.eye(3)]
    for ax in np.eye(3):
        ops.append(axis_angle_matrix(ax, np.pi))
        ops.append(axis_angle_matrix(ax, np.pi / 2))
        ops.append(axis_angle_matrix(ax, -np.pi / 2))
    for sx in (1, -1):
        for sy in (1, -1):
            ax = np.array([1.0, sx, sy])
            ops.append(axis_angle_matrix(ax, 2 * np.pi / 3))
            ops.append(axis_angle_matrix(ax, -2 * np.pi / 3))
    for ax in ([1, 1, 0], [1, -1, 0], [1, 0, 1], [1, 0, -1], [0, 1, 1], [0, 1, -1]):
        ops.append(axis_angle_matrix(ax, np.pi))
    ops = np.array(ops)
    ops[np.abs(ops) < 1e-15] = 0.0
    return ops


def misorientation_angle(ra, rb):
    """Rotation angle of R_a^T R_b (no symmetry)."""
    return rotation_angle(np.swapaxes(ra, -1, -2) @ rb)


def disorientation(ra, rb, ops=None):
    """Disorientation angle (rad): min over cubic S of angle(R_a^T S R_b)."""
    ops = cubic_operators() if ops is None else ops
    ra = np.asarray(ra, dtype=np.float64)
    rb = np.asarray(rb, dtype=np.float64)
    # broadcast (..., 1, 3, 3) against (24, 3, 3)
    m = np.swapaxes(ra, -1, -2)[..., None, :, :] @ ops @ rb[..., None, :, :]
    return rotation_angle(m).min(axis=-1)


def disorientation_q(qa, qb):
    return disorientation(quat_to_matrix(qa), quat_to_matrix(qb))


def fz_representative(r, ops=None):
    """Symmetry-equivalent S R with the smallest rotation angle (the cubic
    fundamental-zone representative); ties go to the lowest operator index."""
    ops = cubic_operators() if ops is None else ops
    cand = ops @ np.asarray(r, dtype=np.float64)
    ang = rotation_angle(cand)
    return cand[int(np.argmin(ang))]
