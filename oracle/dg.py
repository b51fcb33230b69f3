"""Semi-discrete upwind DG operator for velocity-strain elastodynamics (oracle).

Unknowns per element: q = (v_x, v_y, v_z, e_xx, e_yy, e_zz, e_yz, e_xz, e_xy),
tensor (not engineering) shear strains, each a polynomial of degree N stored
as orthonormal modal coefficients c[K][9][Np].

PDE (an instance of the first-order system of Sec. 2, eq. LPDE, with C = 0):
    rho dv/dt = div(sigma) + f,    de/dt = sym(grad v),
    sigma = lambda tr(e) I + 2 mu e.

Weak form on element K with test functions psi (Sec. 2, eq. HDGlocal after
integrating the volume term by parts back to strong form):
    (rho dv/dt, w)_Q = (div sigma_h, w) + <T* - T^-, w>_dK + f-term
    (de/dt, psi)     = (sym grad v, psi) + <sym(n (x) (v* - v^-)), psi>_dK
where sigma_h is the L2 projection (under the quadrature Q_N) of
lambda_q tr(e_q) I + 2 mu_q e_q computed at the quadrature points, and
(rho ., .)_Q is the quadrature-defined mass with the sampled density.

Interface state (T*, v*).  The upwind HDG flux F^.n = F(u).n + |A|(u - u^)
(Sec. 2, eq. RiemannFluxBoth) with the trace u^ eliminated by the single-
valued flux condition (Sec. 2, eq. HDGeqn; Sec. 3, eq. iHDGtrace with equal
iterates) is, for continuous coefficients, 1/2 A (u^- + u^+) + 1/2 |A| (u^- - u^+).
The paper assumes A_k continuous; with element-wise material the exact
Riemann solution per characteristic mode is used instead (normal mode with
the P impedance Z_p, tangential modes with the S impedance Z_s):
    T* = (Z^+ T^- + Z^- T^+ + Z^- Z^+ [v]) / (Z^- + Z^+)
    v* = (Z^- v^- + Z^+ v^+ + [T]) / (Z^- + Z^+)
with [a] = a^+ - a^-, T = sigma_h n and n the outward normal of K.  For
Z^- = Z^+ this is exactly the eliminated HDG flux above.  Impedances use the
quadrature-weighted element means of rho, lambda, mu.
"""
import numpy as np

from .mesh import Mesh
from .reference import FACE_VERTS, Reference

VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def _full(s6):
    """Voigt-ordered symmetric components [..., 6, X] -> [..., 3, 3, X]."""
    out = np.empty(s6.shape[:-2] + (3, 3) + s6.shape[-1:], dtype=s6.dtype)
    for m, (i, j) in enumerate(VOIGT):
        out[..., i, j, :] = s6[..., m, :]
        out[..., j, i, :] = s6[..., m, :]
    return out


def _voigt_sym(g):
    """sym part of a [..., 3, 3, X] tensor -> Voigt [..., 6, X]."""
    return np.stack([0.5 * (g[..., i, j, :] + g[..., j, i, :]) for (i, j) in VOIGT],
                    axis=-2)


def _apply(op, x):
    """Apply a matrix op[m][n] to the last axis of x[..., n] -> [..., m]."""
    shp = x.shape
    return (np.ascontiguousarray(x).reshape(-1, shp[-1]) @ op.T).reshape(shp[:-1] + (op.shape[0],))


def _double_dot(e6, s6):
    """e:s for Voigt-ordered symmetric tensors along axis -2."""
    w = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    return np.einsum('m,...mx,...mx->...x', w, e6, s6)


class Elastic:
    """The oracle operator L(q) for one mesh, degree and material."""

    def __init__(self, N, VXYZ, rho_q, lam_q, mu_q, flux="upwind", boundary=None, mass="exact"):
        if flux not in ("upwind", "central"):
            raise ValueError(flux)
        if mass not in ("exact", "wadg"):
            raise ValueError(mass)
        self.mass = mass
        if boundary not in (None, "free", "absorbing"):
            raise ValueError(boundary)
        self.flux = flux
        self.bc = boundary
        self.ref = Reference(N)
        self.mesh = Mesh(VXYZ, periodic=boundary is None)
        R, M = self.ref, self.mesh
        self.N, self.Np, self.Nq, self.K = N, R.Np, R.Nq, M.K
        if M.check_face_points(R.face_bary) > 1e-12:
            raise ValueError("inconsistent face matching")
        # real FP64 normally; complex values are accepted so that derivatives
        # can be taken by the complex-step method
        dt_ = np.result_type(np.asarray(rho_q).dtype, np.asarray(lam_q).dtype,
                             np.asarray(mu_q).dtype, np.float64)
        self.rho_q = np.asarray(rho_q, dtype=dt_).reshape(self.K, self.Nq)
        self.lam_q = np.asarray(lam_q, dtype=dt_).reshape(self.K, self.Nq)
        self.mu_q = np.asarray(mu_q, dtype=dt_).reshape(self.K, self.Nq)
        if min(self.rho_q.real.min(), self.mu_q.real.min()) <= 0 or self.lam_q.real.min() < 0:
            raise ValueError("material must satisfy rho, mu > 0, lambda >= 0")
        w = R.wq
        # Density-weighted mass M_rho[k] = J_k (rho psi_m, psi_n)_Q, i.e.
        # J_k Psi^T diag(w rho_k) Psi, formed in element chunks as products.
        self.Mrho = np.empty((self.K, self.Np, self.Np), dtype=dt_)
        for k0 in range(0, self.K, 4096):
            k1 = min(k0 + 4096, self.K)
            wr = (w[None, :] * self.rho_q[k0:k1])[:, :, None] * R.Psi_q[None, :, :]   # [k][q][n]
            self.Mrho[k0:k1] = M.J[k0:k1, None, None] * (R.Psi_q.T[None, :, :] @ wr)
        if mass == "exact":
            self.Mrho_inv = np.linalg.inv(self.Mrho)
        else:
            # weight-adjusted approximation M_rho^-1 ~ M^-1 M_{1/rho} M^-1; with the
            # orthonormal modes M = J I and M_{1/rho} = J Psi^T diag(w / rho) Psi,
            # so it is J^-1 Psi^T diag(w / rho) Psi
            self.Mrho_inv = np.empty_like(self.Mrho)
            for k0 in range(0, self.K, 4096):
                k1 = min(k0 + 4096, self.K)
                wr = (w[None, :] / self.rho_q[k0:k1])[:, :, None] * R.Psi_q[None, :, :]
                self.Mrho_inv[k0:k1] = (R.Psi_q.T[None, :, :] @ wr) / M.J[k0:k1, None, None]
        # the velocity mass the scheme inverts (M_rho, or the inverse of its
        # weight-adjusted approximation): the energy that the flux dissipates
        self.Mvel = self.Mrho if mass == "exact" else np.linalg.inv(self.Mrho_inv)
        wsum = w.sum()
        self.rho_bar = self.rho_q @ w / wsum
        self.lam_bar = self.lam_q @ w / wsum
        self.mu_bar = self.mu_q @ w / wsum
        self.Zp = np.sqrt(self.rho_bar * (self.lam_bar + 2.0 * self.mu_bar))
        self.Zs = np.sqrt(self.rho_bar * self.mu_bar)
        # Face evaluation tables.
        self.own_psi = np.stack([R.face_psi(FACE_VERTS[f]) for f in range(4)])  # [4][P][Np]
        # neighbour face tables of the interior faces (boundary faces: -1)
        trip = M.nbr_verts.reshape(-1, 3)
        inner = ~M.boundary.reshape(-1)
        keys = sorted({tuple(int(v) for v in t) for t in trip[inner]})
        self.combo_keys = keys
        self.combo_psi = np.stack([R.face_psi(k) for k in keys])                # [C][P][Np]
        lut = {k: i for i, k in enumerate(keys)}
        self.combo = np.array([lut[tuple(int(v) for v in t)] if ok else -1 for t, ok in zip(trip, inner)],
                              dtype=np.int64).reshape(self.K, 4)
        self.source = None

    # ---------------------------------------------------------------- helpers
    def project_q(self, fq):
        """L2_Q projection of values at Q_N points [K][F][Nq] -> modal."""
        return self.ref.project_q(fq)

    def to_q(self, c):
        return self.ref.to_q(c)

    def sigma_h(self, c, elems):
        """sigma_h = P_q(lambda_q tr(e_q) I + 2 mu_q e_q), Voigt modal [E][6][Np]."""
        R = self.ref
        eq = _apply(R.Psi_q, c[:, 3:9])                             # [E][6][Nq]
        tr = eq[:, 0] + eq[:, 1] + eq[:, 2]
        sq = 2.0 * self.mu_q[elems][:, None, :] * eq
        sq[:, 0:3] += (self.lam_q[elems] * tr)[:, None, :]
        return _apply(R.Psi_q.T, sq * R.wq)

    def grad(self, u, elems):
        """Physical gradient of modal fields u [E][F][Np] -> [E][F][3][Np]."""
        dr = [_apply(Dk, u) for Dk in self.ref.D]                  # d/dr, d/ds, d/dt
        rx = self.mesh.rk_x[elems]                                  # [E][i][j] = dr_i/dx_j
        return np.stack([sum(rx[:, i, j][:, None, None] * dr[i] for i in range(3))
                         for j in range(3)], axis=2)

    def _riemann(self, vm, Tm, vp, Tp, n, zpm, zpp, zsm, zsp):
        """Interface (T*, v*) from both sides' traces; arrays [..., 3]."""
        if self.flux == "central":
            return 0.5 * (Tm + Tp), 0.5 * (vm + vp)
        dv = vp - vm
        dT = Tp - Tm

        def split(a):
            an = np.sum(a * n, axis=-1, keepdims=True)
            return an, a - an * n

        Tmn, Tmt = split(Tm)
        Tpn, Tpt = split(Tp)
        vmn, vmt = split(vm)
        vpn, vpt = split(vp)
        dvn, dvt = split(dv)
        dTn, dTt = split(dT)
        Tsn = (zpp * Tmn + zpm * Tpn + zpm * zpp * dvn) / (zpm + zpp)
        vsn = (zpm * vmn + zpp * vpn + dTn) / (zpm + zpp)
        Tst = (zsp * Tmt + zsm * Tpt + zsm * zsp * dvt) / (zsm + zsp)
        vst = (zsm * vmt + zsp * vpt + dTt) / (zsm + zsp)
        return Tsn * n + Tst, vsn * n + vst

    def face_traces(self, c, s, pos, elems):
        """Own and neighbour traces of v and T at the face-rule points.

        Returns vm, Tm, vp, Tp with shape [E][4][P][3], using sigma_h
        (s, indexed through pos) of the element and its neighbours."""
        M = self.mesh
        E = len(elems)
        P = self.ref.Nfq
        dt_ = np.result_type(c.dtype, s.dtype)
        vm = np.empty((E, 4, P, 3), dtype=dt_)
        Tm = np.empty((E, 4, P, 3), dtype=dt_)
        vp = np.empty((E, 4, P, 3), dtype=dt_)
        Tp = np.empty((E, 4, P, 3), dtype=dt_)
        n = M.normal[elems]                                     # [E][4][3]
        for f in range(4):
            psi = self.own_psi[f]
            vm[:, f] = np.swapaxes(_apply(psi, c[elems, 0:3]), 1, 2)
            sig = _full(_apply(psi, s[pos[elems]]))                 # [E][3][3][P]
            Tm[:, f] = np.einsum('kijp,kj->kpi', sig, n[:, f])
            nb = M.nbr[elems, f]
            cid = self.combo[elems, f]
            # boundary faces: the exterior state of the boundary condition
            # (traction-free mirror v+ = v-, T+ = -T-; absorbing: zero)
            bd = cid < 0
            if np.any(bd):
                if self.bc == "free":
                    vp[bd, f] = vm[bd, f]
                    Tp[bd, f] = -Tm[bd, f]
                else:
                    vp[bd, f] = 0.0
                    Tp[bd, f] = 0.0
            for ci in np.unique(cid[~bd]):
                sel = np.nonzero(cid == ci)[0]
                psin = self.combo_psi[ci]
                kb = nb[sel]
                vp[sel, f] = np.swapaxes(_apply(psin, c[kb, 0:3]), 1, 2)
                sgn = _full(_apply(psin, s[pos[kb]]))
                Tp[sel, f] = np.einsum('kijp,kj->kpi', sgn, n[sel, f])
        return vm, Tm, vp, Tp

    # ------------------------------------------------------------- operator
    def set_source(self, xs, direction, amp=1.0):
        """Point force amp * d * delta(x - xs); returns the owning element."""
        k, rh = self.mesh.locate(xs)
        phi = self.ref.basis.eval(rh[None, :])[0]
        self.source = (k, self.Mrho_inv[k] @ phi, np.asarray(direction, float) * amp)
        return k

    def rhs(self, c, src_value=0.0, elems=None):
        """L(c) (+ src_value * source term) on all elements or a subset.

        c: modal state [K][9][Np]; returns [E][9][Np] for elems (default all).
        """
        M = self.mesh
        if elems is None:
            elems = np.arange(self.K)
        elems = np.asarray(elems, dtype=np.int64)
        nbs = M.nbr[elems].ravel()
        U = np.unique(np.concatenate([elems, nbs[nbs >= 0]]))
        pos = np.full(self.K, -1, dtype=np.int64)
        pos[U] = np.arange(len(U))
        s = self.sigma_h(c[U], U)                                # [U][6][Np]
        sE = s[pos[elems]]
        # Volume terms, exact for P_N on affine elements.
        gs = self.grad(sE, elems)                                 # [E][6][3][Np]
        gs_full = _full(np.moveaxis(gs, 2, 1))                    # [E][3dir][3][3][Np]
        div = np.einsum('kjijn->kin', gs_full)                    # sum_j d_j sigma_ij
        gv = self.grad(c[elems, 0:3], elems)                      # [E][3 comp][3 dir][Np]
        symg = _voigt_sym(gv)                                     # [E][6][Np]
        # Face terms.
        vm, Tm, vp, Tp = self.face_traces(c, s, pos, elems)
        n = M.normal[elems][:, :, None, :]                        # [E][4][1][3]
        # impedances across a boundary face: the element's own
        nb = np.where(M.boundary[elems], elems[:, None], M.nbr[elems])
        zpm = self.Zp[elems][:, None, None, None]
        zsm = self.Zs[elems][:, None, None, None]
        zpp = self.Zp[nb][:, :, None, None]
        zsp = self.Zs[nb][:, :, None, None]
        Ts, vs = self._riemann(vm, Tm, vp, Tp, n, zpm, zpp, zsm, zsp)
        dv = Ts - Tm                                               # velocity correction
        w = vs - vm
        de = np.stack([0.5 * (n[..., i] * w[..., j] + n[..., j] * w[..., i])
                       for (i, j) in VOIGT], axis=-1)              # [E][4][P][6]
        wts = M.area[elems][:, :, None] * self.ref.face_w[None, None, :]   # [E][4][P]
        bv = sum(_apply(self.own_psi[f].T, np.swapaxes(wts[:, f, :, None] * dv[:, f], 1, 2))
                 for f in range(4))
        be = sum(_apply(self.own_psi[f].T, np.swapaxes(wts[:, f, :, None] * de[:, f], 1, 2))
                 for f in range(4))
        J = M.J[elems]
        out = np.empty((len(elems), 9, self.Np), dtype=np.result_type(c.dtype, s.dtype, self.Mrho_inv.dtype))
        rv = J[:, None, None] * div + bv                           # [E][3][Np]
        out[:, 0:3] = np.swapaxes(self.Mrho_inv[elems] @ np.swapaxes(rv, 1, 2), 1, 2)
        out[:, 3:9] = symg + be / J[:, None, None]
        if self.source is not None and src_value != 0.0:
            ks, svec, d = self.source
            hit = np.nonzero(elems == ks)[0]
            for h in hit:
                out[h, 0:3] += src_value * d[:, None] * svec[None, :]
        return out

    # ---------------------------------------------------------- diagnostics
    def energy(self, c):
        """E = 1/2 (rho v, v)_Q + 1/2 sum_K J sum_q w e_q : sigma_q."""
        R, M = self.ref, self.mesh
        ev = 0.5 * np.einsum('kcm,kmn,kcn->', c[:, 0:3], self.Mrho, c[:, 0:3])
        eq = np.einsum('qm,kfm->kfq', R.Psi_q, c[:, 3:9])
        tr = eq[:, 0] + eq[:, 1] + eq[:, 2]
        sq = 2.0 * self.mu_q[:, None, :] * eq
        sq[:, 0:3] += (self.lam_q * tr)[:, None, :]
        ee = 0.5 * np.einsum('k,q,kq->', M.J, R.wq, _double_dot(eq, sq))
        return float(ev + ee)

    def energy_rate(self, c, cdot):
        """dE/dt along the direction cdot (the semi-discrete energy rate), with
        the kinetic energy in the velocity mass the scheme inverts."""
        R, M = self.ref, self.mesh
        rv = np.einsum('kcm,kmn,kcn->', cdot[:, 0:3], self.Mvel, c[:, 0:3])
        eq = np.einsum('qm,kfm->kfq', R.Psi_q, c[:, 3:9])
        edq = np.einsum('qm,kfm->kfq', R.Psi_q, cdot[:, 3:9])
        tr = eq[:, 0] + eq[:, 1] + eq[:, 2]
        sq = 2.0 * self.mu_q[:, None, :] * eq
        sq[:, 0:3] += (self.lam_q * tr)[:, None, :]
        re = np.einsum('k,q,kq->', M.J, R.wq, _double_dot(edq, sq))
        return float(rv + re)

    def face_dissipation(self, c):
        """Closed form of the energy rate under the interface states above:
        each interior face point contributes -([T]^2 + Z^- Z^+ [v]^2)/(Z^- + Z^+)
        per mode (normal with Z_p, tangential with Z_s), integrated over faces.

        A boundary face adds the element's surface term v-.T* + v*.T- - v-.T-
        with the boundary's exterior state: traction-free (T* = 0,
        v* = v- - T-/Z per mode) gives -T^2/Z per mode; absorbing (zero
        exterior: T* = (T- - Z v-)/2, v* = (v- - T-/Z)/2) gives
        -(Z v^2 + T^2/Z)/2 per mode."""
        M = self.mesh
        elems = np.arange(self.K)
        pos = elems
        s = self.sigma_h(c, elems)
        vm, Tm, vp, Tp = self.face_traces(c, s, pos, elems)
        n = M.normal[:, :, None, :]
        nb = M.nbr
        zpm = self.Zp[:, None, None]
        zsm = self.Zs[:, None, None]
        zpp = self.Zp[nb][:, :, None]
        zsp = self.Zs[nb][:, :, None]
        dv = vp - vm
        dT = Tp - Tm
        dvn = np.sum(dv * n, axis=-1)
        dTn = np.sum(dT * n, axis=-1)
        dvt = dv - dvn[..., None] * n
        dTt = dT - dTn[..., None] * n
        dens = ((dTn ** 2 + zpm * zpp * dvn ** 2) / (zpm + zpp)
                + (np.sum(dTt ** 2, -1) + zsm * zsp * np.sum(dvt ** 2, -1)) / (zsm + zsp))
        wts = M.area[:, :, None] * self.ref.face_w[None, None, :]
        inner = ~M.boundary[:, :, None]
        # every interior face is visited from both sides
        total = -0.5 * np.sum(wts * dens * inner)
        if np.any(M.boundary):
            Tmn = np.sum(Tm * n, axis=-1)
            Tmt = Tm - Tmn[..., None] * n
            vmn = np.sum(vm * n, axis=-1)
            vmt = vm - vmn[..., None] * n
            if self.bc == "free":
                bdens = Tmn ** 2 / zpm + np.sum(Tmt ** 2, -1) / zsm
            else:
                bdens = 0.5 * (zpm * vmn ** 2 + Tmn ** 2 / zpm + zsm * np.sum(vmt ** 2, -1)
                               + np.sum(Tmt ** 2, -1) / zsm)
            total -= np.sum(wts * bdens * M.boundary[:, :, None])
        return float(total)

    def momentum(self, c):
        """Total momentum sum_K (rho v, 1)_Q."""
        R, M = self.ref, self.mesh
        vq = np.einsum('qm,kcm->kcq', R.Psi_q, c[:, 0:3])
        return np.einsum('k,q,kq,kcq->c', M.J, R.wq, self.rho_q, vq)

    def eval_points(self, c, pts):
        """Field values at physical points (owner by the lowest-index rule)."""
        out = []
        for x in np.atleast_2d(pts):
            k, rh = self.mesh.locate(x)
            out.append(self.ref.basis.eval(rh[None, :])[0] @ c[k].T)
        return np.array(out)

    def locate(self, x):
        return self.mesh.locate(x)

    def l2_q(self, fq):
        """Quadrature L2 norm over the mesh of values [K][F][Nq]."""
        return float(np.sqrt(np.einsum('k,q,kfq->', self.mesh.J, self.ref.wq, fq ** 2)))
