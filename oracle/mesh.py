"""Uniform n x n Cartesian mesh of [0,1]^2: elements, interior faces, trace DoFs.

Test infrastructure only (see oracle/__init__.py).

The paper partitions the unit square into N x N squares (Sec. 5) and keeps the
trace unknowns on the interior skeleton Gamma_h^o (Sec. 3, eqs. eq_h1-eq_h3);
boundary traces carry the projected Dirichlet data.  Its matvec names index
maps Map0..Map3 (Sec. 8, Alg. algo_mv) without fixing an order; the order used
here is a convention of this project:

  element (i, j), e = i + n j, K = [i h, (i+1) h] x [j h, (j+1) h]
  vertical interior face between (i-1, j) and (i, j):   f = (i-1) + (n-1) j
  horizontal interior face between (i, j-1) and (i, j): f = n(n-1) + i + n(j-1)
  trace DoF  f (p+1) + a, a = GLL node index along increasing y (vertical)
             or increasing x (horizontal)
  local faces of an element: 0 left, 1 right, 2 bottom, 3 top
  boundary faces: numbered separately, bottom, right, top, left, each by
             increasing coordinate, index nb in [0, 4n)
"""
import numpy as np

LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3


def n_faces(n):
    """Number of interior faces 2 n (n - 1)."""
    return 2 * n * (n - 1)


def n_trace_dofs(n, p):
    return n_faces(n) * (p + 1)


def element_faces(n, i, j):
    """Interior face index of the 4 local faces of element (i, j), or -1 on the boundary."""
    nv = n * (n - 1)
    left = (i - 1) + (n - 1) * j if i >= 1 else -1
    right = i + (n - 1) * j if i <= n - 2 else -1
    bottom = nv + i + n * (j - 1) if j >= 1 else -1
    top = nv + i + n * j if j <= n - 2 else -1
    return [left, right, bottom, top]


def element_boundary_faces(n, i, j):
    """Boundary face index (bottom, right, top, left ordering) of local faces, or -1."""
    out = [-1, -1, -1, -1]
    if j == 0:
        out[BOTTOM] = i
    if i == n - 1:
        out[RIGHT] = n + j
    if j == n - 1:
        out[TOP] = 2 * n + i
    if i == 0:
        out[LEFT] = 3 * n + j
    return out


def face_elements(n, f):
    """(lo, hi) element indices of interior face f and its orientation ('v' or 'h').

    lo is the left (vertical face) or bottom (horizontal face) element."""
    nv = n * (n - 1)
    if f < nv:
        j, im1 = divmod(f, n - 1)
        i = im1 + 1
        return (i - 1) + n * j, i + n * j, 'v'
    g = f - nv
    jm1, i = divmod(g, n)
    j = jm1 + 1
    return i + n * (j - 1), i + n * j, 'h'


def face_local_index(n, f):
    """Local face index of f in its lo and hi element."""
    _, _, o = face_elements(n, f)
    return (RIGHT, LEFT) if o == 'v' else (TOP, BOTTOM)


def element_dof_map(n, p):
    """dofs[e, lf*(p+1)+a] = global trace DoF of local trace DoF, or -1 on the boundary."""
    P = p + 1
    out = -np.ones((n * n, 4 * P), dtype=np.int64)
    for j in range(n):
        for i in range(n):
            e = i + n * j
            for lf, f in enumerate(element_faces(n, i, j)):
                if f >= 0:
                    out[e, lf * P:(lf + 1) * P] = f * P + np.arange(P)
    return out


def element_bdry_map(n, p):
    """bd[e, lf*(p+1)+a] = boundary trace DoF index (nb*(p+1)+a), or -1 if interior."""
    P = p + 1
    out = -np.ones((n * n, 4 * P), dtype=np.int64)
    for j in range(n):
        for i in range(n):
            e = i + n * j
            for lf, nb in enumerate(element_boundary_faces(n, i, j)):
                if nb >= 0:
                    out[e, lf * P:(lf + 1) * P] = nb * P + np.arange(P)
    return out


def face_midpoint_and_direction(n, f):
    """Midpoint of interior face f and its unit tangent (direction of increasing node index)."""
    h = 1.0 / n
    lo, hi, o = face_elements(n, f)
    i, j = hi % n, hi // n
    if o == 'v':
        return np.array([i * h, (j + 0.5) * h]), np.array([0.0, 1.0])
    return np.array([(i + 0.5) * h, j * h]), np.array([1.0, 0.0])


def boundary_face_geometry(n, nb):
    """Start point and unit tangent of boundary face nb (nodes in increasing coordinate)."""
    h = 1.0 / n
    side, t = divmod(nb, n)
    if side == 0:   # bottom, y = 0
        return np.array([t * h, 0.0]), np.array([1.0, 0.0])
    if side == 1:   # right, x = 1
        return np.array([1.0, t * h]), np.array([0.0, 1.0])
    if side == 2:   # top, y = 1
        return np.array([t * h, 1.0]), np.array([1.0, 0.0])
    return np.array([0.0, t * h]), np.array([0.0, 1.0])  # left, x = 0
