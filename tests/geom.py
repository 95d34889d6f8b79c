"""Small hand-built geometry for the closed-form tests (no rendering
arithmetic here: only vertex lists and poses)."""
import numpy as np

IDENT_POSE = np.array([0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1], np.float32)


def pose_at(x, y, z, R=None):
    R = np.eye(3) if R is None else np.asarray(R, np.float64)
    return np.concatenate([[x, y, z], R.ravel()]).astype(np.float32)


def quad(a, b, c, d):
    """Two triangles (a, b, c), (a, c, d)."""
    pos = np.array([a, b, c, d], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    return pos, idx


def merge(*meshes):
    """Concatenate (pos, idx[, col]) meshes."""
    P, I, Cs = [], [], []
    base = 0
    for m in meshes:
        pos, idx = m[0], m[1]
        col = m[2] if len(m) > 2 else np.full((len(pos), 3), 255, np.uint8)
        P.append(np.asarray(pos, np.float32))
        I.append(np.asarray(idx, np.uint32) + base)
        Cs.append(np.asarray(col, np.uint8))
        base += len(pos)
    return np.concatenate(P), np.concatenate(I), np.concatenate(Cs)


def unit_cube(x0, x1, y0, y1, z0, z1, front_first=True):
    """Closed cube as 12 triangles; the +z face (z = z1) comes first so its
    two triangles have ids 0 and 1.  The front face is split along the
    diagonal from (x0, y1) to (x1, y0), i.e. from the top-left to the
    bottom-right corner as seen from +z."""
    v = np.array([[x, y, z] for z in (z0, z1) for y in (y0, y1) for x in (x0, x1)], np.float32)
    # index = 4*zi + 2*yi + xi
    def q(a, b, c, d):
        return [[a, b, c], [a, c, d]]
    front = q(6, 7, 5, 4)             # z1: (x0,y1) (x1,y1) (x1,y0) (x0,y0)
    back = q(2, 3, 1, 0)
    left = q(0, 4, 6, 2)
    right = q(1, 3, 7, 5)
    bottom = q(0, 1, 5, 4)
    top = q(2, 6, 7, 3)
    faces = front + back + left + right + bottom + top
    return v, np.array(faces, np.uint32)
