"""Crystal geometry and tensor algebra for the oracle (test infrastructure).

Sec. 2.1: FCC crystals with 12 slip systems (normals in {111}, directions in
<110>), cubic anisotropic elasticity; eq. nye1: 12 edge and 6 screw GND
families.  Orientation: unit quaternion (w, x, y, z) whose rotation takes
crystal-frame vectors to the sample frame.
"""
import itertools
import numpy as np

SQ2 = np.sqrt(2.0)
# Mandel order of a symmetric 3x3 tensor: 11, 22, 33, 23, 13, 12
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
WEIGHT = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


def quat_to_rot(q):
    """Rotation matrix of unit quaternion(s) q = (w, x, y, z); v_sample = R v_crystal."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(q, -1, 0)
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def cubic_stiffness(C11, C12, C44):
    """Fourth-order cubic stiffness in the crystal frame (3x3x3x3)."""
    d = np.eye(3)
    C = (C12 * np.einsum("ij,kl->ijkl", d, d)
         + C44 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    aniso = C11 - C12 - 2.0 * C44
    for a in range(3):
        C[a, a, a, a] += aniso
    return C


def rotate4(C, R):
    """C'_ijkl = R_ia R_jb R_kc R_ld C_abcd."""
    return np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, C)


def fcc_slip_systems():
    """The 12 FCC systems as unit (s, n) pairs, s in <110>, n in {111}, s.n = 0.

    Enumerated rather than tabulated: the 4 plane normals up to sign and the 6
    <110> directions up to sign, kept where orthogonal.
    """
    normals = [np.array(v, dtype=float) for v in [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)]]
    dirs = screw_directions()
    s_list, n_list = [], []
    for nrm in normals:
        nrm = nrm / np.linalg.norm(nrm)
        for s in dirs:
            if abs(s @ nrm) < 1e-12:
                s_list.append(s)
                n_list.append(nrm)
    s = np.array(s_list)
    n = np.array(n_list)
    assert s.shape == (12, 3)
    return s, n


def screw_directions():
    """The 6 <110> unit directions (one of each +/- pair)."""
    out = []
    for v in itertools.product((-1, 0, 1), repeat=3):
        v = np.array(v, dtype=float)
        if np.count_nonzero(v) != 2:
            continue
        # keep one representative of each +/- pair: first non-zero component positive
        if v[np.nonzero(v)[0][0]] < 0:
            continue
        out.append(v / np.linalg.norm(v))
    assert len(out) == 6
    return np.array(out)


def to_mandel2(T):
    """Symmetric tensor(s) (...,3,3) -> Mandel vector(s) (...,6)."""
    T = 0.5 * (T + np.swapaxes(T, -1, -2))
    return np.stack([WEIGHT[a] * T[..., i, j] for a, (i, j) in enumerate(PAIRS)], axis=-1)


def from_mandel2(v):
    """Mandel vector(s) (...,6) -> symmetric tensor(s) (...,3,3)."""
    T = np.empty(v.shape[:-1] + (3, 3))
    for a, (i, j) in enumerate(PAIRS):
        T[..., i, j] = v[..., a] / WEIGHT[a]
        T[..., j, i] = v[..., a] / WEIGHT[a]
    return T


def to_mandel4(C):
    """Minor-symmetric fourth-order tensor(s) (...,3,3,3,3) -> Mandel matrix (...,6,6)."""
    M = np.empty(C.shape[:-4] + (6, 6))
    for a, (i, j) in enumerate(PAIRS):
        for b, (k, l) in enumerate(PAIRS):
            M[..., a, b] = WEIGHT[a] * WEIGHT[b] * C[..., i, j, k, l]
    return M


def from_mandel4(M):
    """Mandel matrix (...,6,6) -> fourth-order tensor with both minor symmetries."""
    C = np.empty(M.shape[:-2] + (3, 3, 3, 3))
    for a, (i, j) in enumerate(PAIRS):
        for b, (k, l) in enumerate(PAIRS):
            val = M[..., a, b] / (WEIGHT[a] * WEIGHT[b])
            for (p, q) in {(i, j), (j, i)}:
                for (r, s) in {(k, l), (l, k)}:
                    C[..., p, q, r, s] = val
    return C


def gnd_matrix():
    """9x18 matrix whose columns are vec(b (x) t) of the FCC GND families (eq. nye1):
    12 edge dislocations (t = s x n) and 6 screw dislocations (t = s), crystal frame,
    row-major vec of the 3x3 dyad."""
    s, n = fcc_slip_systems()
    cols = []
    for a in range(12):
        t = np.cross(s[a], n[a])
        cols.append(np.outer(s[a], t).ravel())
    for d in screw_directions():
        cols.append(np.outer(d, d).ravel())
    return np.array(cols).T
