"""Periodic voxel microstructures: grain maps, orientations and notches.

Every array that describes the voxel grid is returned *flat with x fastest*:
voxel (i, j, k) sits at index ``i + N1*(j + N2*k)``.  Voxel centres are at
``(i + 1/2, j + 1/2, k + 1/2)`` in voxel units; distances use the minimum image
of the periodic box.
"""
import numpy as np
from scipy.spatial import cKDTree


def _voxel_centres(n):
    n1, n2, n3 = n
    i = np.arange(n1) + 0.5
    j = np.arange(n2) + 0.5
    k = np.arange(n3) + 0.5
    # x fastest: meshgrid with indexing "ij" over (k, j, i) then reverse columns
    kk, jj, ii = np.meshgrid(k, j, i, indexing="ij")
    return np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)


def periodic_voronoi(n, seeds):
    """Grain id of every voxel: the nearest seed under the periodic minimum image.

    ``n`` = (N1, N2, N3); ``seeds`` (G, 3) in voxel units inside the box.
    Returns int32 array of N1*N2*N3 ids, x fastest.
    """
    n = tuple(int(v) for v in n)
    box = np.array(n, dtype=np.float64)
    tree = cKDTree(np.mod(seeds, box), boxsize=box)
    _, idx = tree.query(_voxel_centres(n), k=1)
    return idx.astype(np.int32)


def periodic_laguerre(n, seeds, weights, k_candidates=32):
    """Power-diagram (Laguerre) grain map: argmin over seeds of d^2 - w (periodic).

    Exact: the ``k_candidates`` Euclidean-nearest seeds are scanned, and every
    voxel for which a farther seed could still win (its distance^2 minus the
    largest weight below the best power distance found) is resolved by brute
    force over all seeds.
    """
    n = tuple(int(v) for v in n)
    box = np.array(n, dtype=np.float64)
    seeds = np.mod(seeds, box)
    weights = np.asarray(weights, dtype=np.float64)
    pts = _voxel_centres(n)
    g = len(seeds)
    kc = min(k_candidates + 1, g)
    tree = cKDTree(seeds, boxsize=box)
    d, idx = tree.query(pts, k=kc)
    if kc == 1:
        d = d[:, None]
        idx = idx[:, None]
    use = kc - 1 if kc < g else kc
    pw = d[:, :use] ** 2 - weights[idx[:, :use]]
    best = np.argmin(pw, axis=1)
    best_pw = pw[np.arange(len(pts)), best]
    best_id = idx[np.arange(len(pts)), best]
    if kc < g:
        bound = d[:, kc - 1] ** 2 - weights.max()
        bad = np.nonzero(bound <= best_pw)[0]
    else:
        bad = np.arange(len(pts))
    out = best_id.astype(np.int64)
    for s in range(0, len(bad), 16384):
        sel = bad[s:s + 16384]
        dx = np.abs(pts[sel, None, :] - seeds[None, :, :])
        dx = np.minimum(dx, box - dx)
        p = (dx ** 2).sum(axis=2) - weights[None, :]
        out[sel] = np.argmin(p, axis=1)
    return out.astype(np.int32)


def lognormal_laguerre_weights(n, n_grains, sigma, rng):
    """Laguerre weights w_i = r_i^2 with r_i the equivalent-sphere radius of a
    log-normal target volume V_i ~ LogNormal(0, sigma), volumes normalised to the box."""
    v = rng.lognormal(mean=0.0, sigma=sigma, size=n_grains)
    v = v / v.sum() * float(np.prod(n))
    r = (3.0 * v / (4.0 * np.pi)) ** (1.0 / 3.0)
    return r ** 2


def shoemake_quaternions(count, rng):
    """Uniformly distributed unit quaternions (w, x, y, z), Shoemake's subgroup method."""
    u = rng.random((count, 3))
    a = np.sqrt(1.0 - u[:, 0])
    b = np.sqrt(u[:, 0])
    t1 = 2.0 * np.pi * u[:, 1]
    t2 = 2.0 * np.pi * u[:, 2]
    q = np.stack([b * np.cos(t2), a * np.sin(t1), a * np.cos(t1), b * np.sin(t2)], axis=1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def notch_mask(n, width_x=2, width_y=2):
    """Through-thickness notch: voxels with i in the central ``width_x`` columns and
    j in the central ``width_y`` rows, for every k.  Flat, x fastest, float 0/1."""
    n1, n2, n3 = n
    i0 = n1 // 2 - width_x // 2
    j0 = n2 // 2 - width_y // 2
    m = np.zeros((n3, n2, n1))
    m[:, j0:j0 + width_y, i0:i0 + width_x] = 1.0
    return m.ravel()
