"""Affine geometry and face matching of a periodic tetrahedral mesh (oracle).

Implements the mesh conventions of Sec. 2: elements K_j, the skeleton of
faces, the outward normal n^- of an element and n^+ = -n^- of its neighbour.
Faces are matched purely by the physical coordinates of their vertices,
wrapped into the periodic box [-1,1)^3 (periodic meshes) or as they are
(bounded meshes, where a face without a partner is a boundary face of the
skeleton, the set of boundary faces of Sec. 2); the GPU library instead
matches faces topologically from vertex ids.
"""
import numpy as np

from .reference import FACE_VERTS, REF_VERTS

_GRID = 1e9          # coordinates are compared on a 1e-9 lattice after wrapping
_PERIOD = 2.0


def _wrap_key(x):
    """Integer key of a point modulo the periodic box."""
    k = np.rint((x + 1.0) * _GRID).astype(np.int64)
    return tuple(int(v) for v in np.mod(k, int(_PERIOD * _GRID)))


def _plain_key(x):
    """Integer key of a point (no periodic wrap)."""
    k = np.rint((x + 1.0) * _GRID).astype(np.int64)
    return tuple(int(v) for v in k)


class Mesh:
    def __init__(self, VXYZ, periodic=True):
        X = np.asarray(VXYZ, dtype=np.float64)
        self.K = X.shape[0]
        self.X = X
        # x = X0 + A (rhat + 1), A columns = (X_i - X_0)/2 for i = 1,2,3.
        self.A = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]],
                          axis=-1) / 2.0
        self.J = np.linalg.det(self.A)
        if np.any(self.J <= 0.0):
            raise ValueError("element with non-positive Jacobian")
        # rk_x[k][i][j] = d r_i / d x_j
        self.rk_x = np.linalg.inv(self.A)
        self.volume = self.J * (4.0 / 3.0)
        self.periodic = bool(periodic)
        self._faces()
        self._match()

    def to_physical(self, k, rhat):
        return self.X[k, 0] + (np.asarray(rhat) + 1.0) @ self.A[k].T

    def to_reference(self, k, x):
        return (np.asarray(x) - self.X[k, 0]) @ self.rk_x[k].T - 1.0

    def _faces(self):
        K = self.K
        self.normal = np.zeros((K, 4, 3))
        self.area = np.zeros((K, 4))
        for f, (ia, ib, ic) in enumerate(FACE_VERTS):
            opp = ({0, 1, 2, 3} - {ia, ib, ic}).pop()
            cr = np.cross(self.X[:, ib] - self.X[:, ia], self.X[:, ic] - self.X[:, ia])
            nrm = np.linalg.norm(cr, axis=1)
            n = cr / nrm[:, None]
            inward = np.einsum('kd,kd->k', n, self.X[:, opp] - self.X[:, ia]) > 0
            n[inward] *= -1.0
            self.normal[:, f] = n
            self.area[:, f] = 0.5 * nrm
        # inradius r = 3 |K| / |dK|
        self.inradius = 3.0 * self.volume / self.area.sum(axis=1)

    def _match(self):
        """Find, for every (element, face), the neighbour element and the
        neighbour's local vertex numbers of our face's three vertices."""
        K = self.K
        key_of = _wrap_key if self.periodic else _plain_key
        vkey = [[key_of(self.X[k, i]) for i in range(4)] for k in range(K)]
        table = {}
        for k in range(K):
            for f, tri in enumerate(FACE_VERTS):
                key = tuple(sorted(vkey[k][i] for i in tri))
                table.setdefault(key, []).append((k, f))
        self.nbr = np.full((K, 4), -1, dtype=np.int64)
        self.nbr_face = np.full((K, 4), -1, dtype=np.int64)
        # nbr_verts[k][f] = neighbour-local vertex numbers matching FACE_VERTS[f]
        self.nbr_verts = np.full((K, 4, 3), -1, dtype=np.int64)
        self.boundary = np.zeros((K, 4), dtype=bool)
        for key, lst in table.items():
            if len(lst) == 1 and not self.periodic:
                k1, f1 = lst[0]
                self.boundary[k1, f1] = True
                continue
            if len(lst) != 2:
                raise ValueError("face without exactly one partner (mesh not periodic "
                                 "or not conforming)")
            (k1, f1), (k2, f2) = lst
            for (ka, fa), (kb, fb) in (((k1, f1), (k2, f2)), ((k2, f2), (k1, f1))):
                self.nbr[ka, fa] = kb
                self.nbr_face[ka, fa] = fb
                for m, iv in enumerate(FACE_VERTS[fa]):
                    jv = [j for j in range(4) if vkey[kb][j] == vkey[ka][iv]]
                    assert len(jv) == 1
                    self.nbr_verts[ka, fa, m] = jv[0]

    def check_face_points(self, bary):
        """Max distance (mod period) between a face-rule point placed on our
        face and the same barycentric point placed on the neighbour's matched
        vertices, mapped to physical space.  Zero for a consistent matching."""
        err = 0.0
        for f, tri in enumerate(FACE_VERTS):
            inner = ~self.boundary[:, f]
            own = np.einsum('pm,kmd->kpd', bary, self.X[inner][:, list(tri)])
            nb = self.nbr[inner, f]
            nv = self.nbr_verts[inner, f]
            Xn = np.take_along_axis(self.X[nb], nv[:, :, None], axis=1)   # [K][3][3]
            other = np.einsum('pm,kmd->kpd', bary, Xn)
            d = other - own
            if self.periodic:
                d = d - _PERIOD * np.rint(d / _PERIOD)
            if d.size:
                err = max(err, float(np.abs(d).max()))
        return err

    def locate(self, x, tol=1e-12):
        """Owning element of a point: all barycentric coordinates >= -tol;
        ties (points on shared faces, edges or vertices) go to the lowest
        element index.  Returns (element, reference coordinates)."""
        x = np.asarray(x, dtype=np.float64)
        rh = np.einsum('kij,kj->ki', self.rk_x, x[None, :] - self.X[:, 0]) - 1.0
        lam = np.stack([-(rh.sum(axis=1) + 1.0) / 2.0, (rh[:, 0] + 1) / 2,
                        (rh[:, 1] + 1) / 2, (rh[:, 2] + 1) / 2], axis=1)
        inside = np.all(lam >= -tol, axis=1)
        idx = np.nonzero(inside)[0]
        if len(idx) == 0:
            raise ValueError("point outside the mesh")
        k = int(idx[0])
        return k, rh[k]


__all__ = ["Mesh", "REF_VERTS"]
