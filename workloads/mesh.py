"""Periodic and bounded tetrahedral meshes of the cube [-1,1]^3.

Each of the n^3 hexahedra of side h = 2/n is cut into six tetrahedra by the
Kuhn (Freudenthal) split: for every permutation p of the three axes the
tetrahedron is {o, o + h e_p0, o + h (e_p0 + e_p1), o + h (e_p0 + e_p1 + e_p2)}.
Every hexahedron uses the same main diagonal, so the split is translation
invariant and therefore conforming, also across the periodic wrap.

Outputs
-------
EToV : int64 [K][4]    periodic vertex ids (lattice index taken mod n per axis)
VXYZ : float64 [K][4][3] unwrapped vertex coordinates of each element, all
                         inside [-1,1]^3; the affine map of element k sends
                         reference vertex i to VXYZ[k][i]
Elements are ordered hexahedron-major (x fastest), six per hexahedron.
Vertices are ordered so that every element has positive orientation.
"""
import itertools

import numpy as np

_PERMS = list(itertools.permutations(range(3)))


def _orient(p):
    """Sign of the determinant of (e_p0, e_p1, e_p2)."""
    return np.linalg.det(np.eye(3)[list(p)])


def kuhn_periodic_mesh(n, shuffle_seed=None):
    """Build the 6 n^3-element periodic Kuhn mesh.

    shuffle_seed: if given, each element's four vertices are relabelled by a
    random even permutation (orientation kept positive).  The geometry is the
    same; only the local vertex order, hence the face orientations between
    neighbours, changes.  Used to exercise every face-to-face permutation.
    """
    h = 2.0 / n
    K = 6 * n ** 3
    # hexahedron origins, x fastest: index = i + n (j + n k)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    org = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=-1)            # [n^3][3]
    tets = np.zeros((6, 4, 3), dtype=np.int64)
    for t, p in enumerate(_PERMS):
        cur = np.zeros(3, dtype=np.int64)
        pts = [cur.copy()]
        for ax in p:
            cur[ax] += 1
            pts.append(cur.copy())
        if _orient(p) < 0:
            pts[2], pts[3] = pts[3], pts[2]
        tets[t] = np.array(pts)
    lat = (org[:, None, None, :] + tets[None, :, :, :]).reshape(K, 4, 3)
    if shuffle_seed is not None:
        rng = np.random.default_rng(shuffle_seed)
        even = np.array([q for q in itertools.permutations(range(4))
                         if np.linalg.det(np.eye(4)[list(q)]) > 0])
        choice = rng.integers(0, len(even), size=K)
        lat = np.take_along_axis(lat, even[choice][:, :, None], axis=1)
    wrapped = lat % n
    EToV = wrapped[..., 0] + n * (wrapped[..., 1] + n * wrapped[..., 2])
    VXYZ = -1.0 + h * lat.astype(np.float64)
    return EToV.astype(np.int64), VXYZ


def kuhn_box_mesh(n, shuffle_seed=None):
    """The same 6 n^3 Kuhn tetrahedra of [-1,1]^3 without the periodic wrap:
    vertex ids index the (n+1)^3 lattice, so the faces on the box boundary
    have no partner.  Element order and shapes as kuhn_periodic_mesh."""
    _, VXYZ = kuhn_periodic_mesh(n, shuffle_seed=shuffle_seed)
    h = 2.0 / n
    lat = np.rint((VXYZ + 1.0) / h).astype(np.int64)
    EToV = lat[..., 0] + (n + 1) * (lat[..., 1] + (n + 1) * lat[..., 2])
    return EToV.astype(np.int64), VXYZ


def hex_translation_permutation(n, shift):
    """Element permutation induced by translating the mesh by whole hexahedra.

    Returns perm with element e of the mesh moved by shift=(dx,dy,dz) hexes
    landing on element perm[e].  Only valid for the unshuffled mesh.
    """
    dx, dy, dz = shift
    perm = np.empty(6 * n ** 3, dtype=np.int64)
    for k in range(n):
        for j in range(n):
            for i in range(n):
                src = i + n * (j + n * k)
                dst = ((i + dx) % n) + n * (((j + dy) % n) + n * ((k + dz) % n))
                for t in range(6):
                    perm[6 * src + t] = 6 * dst + t
    return perm
