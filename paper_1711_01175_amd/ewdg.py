"""ctypes binding of libewdg.so (declared in include/ewdg.h).

Argument marshalling only: every step of the method runs inside the HIP
library.  PyTorch supplies device memory (the workspace and the device
arrays passed in and out) and the HIP stream.  Importing works without a
GPU; any call that needs the device fails loudly if the library or the GPU
is missing.

Stream ordering.  The library enqueues a context's work on the context's
stream, which need not be torch's current stream.  Every method that passes
device tensors makes the context's stream wait for torch's current stream
first (the tensors' producers, and earlier users of recycled memory), makes
torch's current stream wait for the context's stream afterwards (the
tensors' consumers), and marks the tensors as used on the context's stream
(record_stream), so the caching allocator does not hand their memory out
again before that work has run.
"""
import contextlib
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libewdg.so")

EWDG_OK, EWDG_EINVAL, EWDG_ESTATE, EWDG_ENOMEM, EWDG_EHIP, EWDG_EMESH, EWDG_EPOINT = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "EWDG_OK", -1: "EWDG_EINVAL", -2: "EWDG_ESTATE", -3: "EWDG_ENOMEM",
          -4: "EWDG_EHIP", -5: "EWDG_EMESH", -6: "EWDG_EPOINT"}

_c_p = ctypes.c_void_p
_c_i = ctypes.c_int
_c_d = ctypes.c_double
_c_i64 = ctypes.c_int64
_c_sz = ctypes.c_size_t
_P_d = ctypes.POINTER(ctypes.c_double)
_P_i = ctypes.POINTER(ctypes.c_int)

# name -> argtypes (all return int unless listed in _RESTYPE)
BC_PERIODIC, BC_FREE, BC_ABSORBING = 0, 1, 2   # boundary conditions of ewdg_set_mesh_bc

SIGNATURES = {
    "ewdg_create": [_c_i, _c_i, _c_p, ctypes.POINTER(_c_p)],
    "ewdg_destroy": [_c_p],
    "ewdg_set_stream": [_c_p, _c_p],
    "ewdg_set_mesh": [_c_p, _c_i64, _c_p, _c_p],
    "ewdg_set_mesh_bc": [_c_p, _c_i64, _c_p, _c_p, _c_i],
    "ewdg_sizes": [_c_p, _P_i, _P_i, _P_i],
    "ewdg_node_points": [_c_p, _c_p],
    "ewdg_quadrature_points": [_c_p, _c_p],
    "ewdg_reference_operator": [_c_p, _c_i, _c_p],
    "ewdg_connectivity": [_c_p, _c_p],
    "ewdg_workspace_bytes": [_c_p, _c_i, _c_i, ctypes.POINTER(_c_sz)],
    "ewdg_bind_workspace": [_c_p, _c_p, _c_sz, _c_i, _c_i],
    "ewdg_set_material": [_c_p, _c_p, _c_p, _c_p],
    "ewdg_set_mass_inverse": [_c_p, _c_i],
    "ewdg_set_state": [_c_p, _c_p, _c_i, _c_d],
    "ewdg_get_state": [_c_p, _c_p, _c_i, _P_d],
    "ewdg_project_quadrature": [_c_p, _c_p, _c_p],
    "ewdg_eval_quadrature": [_c_p, _c_p, _c_p],
    "ewdg_set_source": [_c_p, _c_p, _c_p, _c_d, _c_d, _c_d],
    "ewdg_clear_source": [_c_p],
    "ewdg_set_receivers": [_c_p, _c_i, _c_p],
    "ewdg_receivers": [_c_p, _c_p, _P_i],
    "ewdg_cfl_dt": [_c_p, _c_d, _P_d],
    "ewdg_rhs": [_c_p, _c_d, _c_p, _c_p],
    "ewdg_step": [_c_p, _c_d, _c_i],
    "ewdg_time": [_c_p, _P_d],
    "ewdg_energy": [_c_p, _P_d],
    "ewdg_energy_device": [_c_p, _c_p],
    "ewdg_batch_table_bytes": [_c_i, ctypes.POINTER(_c_sz)],
    "ewdg_step_batch": [ctypes.POINTER(_c_p), _c_i, ctypes.POINTER(_c_d), _c_i, _c_p, _c_sz, _c_p],
    "ewdg_static_table_max_bytes": [ctypes.POINTER(_c_sz)],
    "ewdg_step_batch_static": [ctypes.POINTER(_c_p), _c_i, ctypes.POINTER(_c_d), _c_i, _c_p],
    "ewdg_adjoint_workspace_bytes": [_c_p, _c_i, _c_i, ctypes.POINTER(_c_sz)],
    "ewdg_adjoint_workspace_bytes_overlapped": [_c_p, _c_i, _c_i, ctypes.POINTER(_c_sz)],
    "ewdg_bind_adjoint_workspace": [_c_p, _c_p, _c_sz, _c_i, _c_i],
    "ewdg_rhs_adjoint": [_c_p, _c_d, _c_p, _c_p, _c_p, _c_p],
    "ewdg_forward_misfit": [_c_p, _c_d, _c_i, _c_p, _P_d],
    "ewdg_adjoint_gradient": [_c_p, _c_p, _c_p],
    "ewdg_implicit_workspace_bytes": [_c_p, ctypes.POINTER(_c_sz)],
    "ewdg_bind_implicit_workspace": [_c_p, _c_p, _c_sz],
    "ewdg_implicit_setup": [_c_p, _c_d, _c_d],
    "ewdg_implicit_step": [_c_p, _c_i, _c_d, _c_i, _c_p, _c_p],
    "ewdg_implicit_dt": [_c_p, _P_d, _P_d],
    "ewdg_transport_create": [_c_i, _c_i, _c_i, _c_p, _c_i, _c_p, ctypes.POINTER(_c_p)],
    "ewdg_transport_destroy": [_c_p],
    "ewdg_transport_sizes": [_c_p, ctypes.POINTER(_c_i64), _P_i, _P_i, _P_i],
    "ewdg_transport_points": [_c_p, _c_p, _c_p],
    "ewdg_transport_workspace_bytes": [_c_p, ctypes.POINTER(_c_sz)],
    "ewdg_transport_bind_workspace": [_c_p, _c_p, _c_sz],
    "ewdg_transport_set_problem": [_c_p, _c_p, _c_p, _c_p],
    "ewdg_transport_solve": [_c_p, _c_d, _c_i, _P_i, _c_p],
    "ewdg_transport_values": [_c_p, _c_p],
    "ewdg_transport_last_error": [_c_p],
    "ewdg_last_error": [_c_p],
}
_RESTYPE = {"ewdg_last_error": ctypes.c_char_p, "ewdg_transport_last_error": ctypes.c_char_p}

_lib = None


def load():
    """Load libewdg.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libewdg.so is not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = _RESTYPE.get(name, ctypes.c_int)
        _lib = lib
    return _lib


class EwdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    """Raw pointer of a numpy array or torch tensor (must be contiguous)."""
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return ctypes.c_void_p(a.ctypes.data)
    assert a.is_contiguous()
    return ctypes.c_void_p(a.data_ptr())


def _torch():
    import torch
    return torch


class Context:
    """One ewdg context: a mesh, a degree, a precision and a workspace.

    Methods mirror the C entry points (ewdg_<name>)."""

    def __init__(self, N, precision=64, stream=None):
        self.lib = load()
        self.N = int(N)
        self.precision = int(precision)
        self._ws = None
        self._adj_ws = None
        self._imp_ws = None
        self._stream = int(stream or 0)
        h = _c_p()
        rc = self.lib.ewdg_create(self.N, self.precision, _c_p(stream), ctypes.byref(h))
        if rc != EWDG_OK:
            raise EwdgError(rc, f"ewdg_create(N={N}, precision={precision}) failed")
        self.h = h
        Np, Nfp, Nq = _c_i(), _c_i(), _c_i()
        self._check(self.lib.ewdg_sizes(self.h, ctypes.byref(Np), ctypes.byref(Nfp), ctypes.byref(Nq)))
        self.Np, self.Nfp, self.Nq = Np.value, Nfp.value, Nq.value
        self.K = 0

    # -------------------------------------------------------------- plumbing
    def _check(self, rc, what=""):
        if rc != EWDG_OK:
            msg = self.lib.ewdg_last_error(self.h) if getattr(self, "h", None) else b""
            raise EwdgError(rc, f"{what} {msg.decode() if msg else ''}".strip())

    def _shape(self, t, per_elem):
        if t.numel() != self.K * per_elem:
            raise EwdgError(EWDG_EINVAL, f"array has {t.numel()} values, expected {self.K * per_elem}")

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float32 if self.precision == 32 else torch.float64

    @property
    def np_dtype(self):
        return np.float32 if self.precision == 32 else np.float64

    def close(self):
        if getattr(self, "h", None):
            self.lib.ewdg_destroy(self.h)
            self.h = None
        self._ws = None
        self._adj_ws = None
        self._imp_ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._check(self.lib.ewdg_set_stream(self.h, _c_p(stream)), "set_stream")
        self._stream = int(stream or 0)

    def _stream_obj(self):
        torch = _torch()
        if self._stream == 0:
            return torch.cuda.default_stream()
        return torch.cuda.ExternalStream(self._stream)

    @contextlib.contextmanager
    def _ordered(self, *tensors):
        """Order the context's stream against torch's current stream around
        a library call that reads or writes the given device tensors."""
        torch = _torch()
        cur = torch.cuda.current_stream()
        if cur.cuda_stream == self._stream:
            yield
            return
        s = self._stream_obj()
        s.wait_stream(cur)
        yield
        cur.wait_stream(s)
        for t in tensors:
            if t is not None and t.is_cuda:
                t.record_stream(s)

    # ----------------------------------------------------------------- mesh
    def set_mesh(self, EToV, VXYZ, boundary=None):
        """boundary: None (periodic: every face has a partner), "free"
        (traction-free) or "absorbing" for the faces without a partner."""
        EToV = _host(EToV, np.int64)
        VXYZ = _host(VXYZ, np.float64)
        K = EToV.shape[0]
        assert EToV.shape == (K, 4) and VXYZ.shape == (K, 4, 3)
        codes = {None: BC_PERIODIC, "free": BC_FREE, "absorbing": BC_ABSORBING}
        if boundary not in codes:
            raise EwdgError(EWDG_EINVAL, f"unknown boundary condition {boundary!r}")
        bc = codes[boundary]
        self._check(self.lib.ewdg_set_mesh_bc(self.h, K, _ptr(EToV), _ptr(VXYZ), bc), "set_mesh")
        self.K = K

    def node_points(self):
        out = np.empty((self.K, self.Np, 3))
        self._check(self.lib.ewdg_node_points(self.h, _ptr(out)), "node_points")
        return out

    def quadrature_points(self):
        out = np.empty((self.K, self.Nq, 3))
        self._check(self.lib.ewdg_quadrature_points(self.h, _ptr(out)), "quadrature_points")
        return out

    def reference_operator(self, which):
        Np, Nfp, Nq = self.Np, self.Nfp, self.Nq
        shapes = {0: (Np, Np), 1: (Np, Np), 2: (Np, Np), 3: (Np, 4 * Nfp), 4: (Nq, Np),
                  5: (Np, Nq), 6: (Np, Np), 7: (Np, 3), 8: (Nq,), 9: (4, Nfp), 10: (4, 4, 6, Nfp)}
        out = np.empty(shapes[which])
        self._check(self.lib.ewdg_reference_operator(self.h, which, _ptr(out)), "reference_operator")
        return out

    def connectivity(self):
        out = np.empty((self.K, 4), dtype=np.int32)
        self._check(self.lib.ewdg_connectivity(self.h, _ptr(out)), "connectivity")
        return out

    # ------------------------------------------------------------ workspace
    def workspace_bytes(self, max_receivers=0, max_record_steps=0):
        b = _c_sz()
        self._check(self.lib.ewdg_workspace_bytes(self.h, max_receivers, max_record_steps,
                                                  ctypes.byref(b)), "workspace_bytes")
        return b.value

    def bind_workspace(self, max_receivers=0, max_record_steps=0, buffer=None):
        """Bind a torch-allocated device buffer (allocated here if not given)."""
        torch = _torch()
        nbytes = self.workspace_bytes(max_receivers, max_record_steps)
        if buffer is None:
            buffer = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        with self._ordered(buffer):
            self._check(self.lib.ewdg_bind_workspace(self.h, _ptr(buffer), buffer.numel() * buffer.element_size(),
                                                     max_receivers, max_record_steps), "bind_workspace")
        self._ws = buffer
        return buffer

    # ------------------------------------------------------------- material
    def set_material(self, rho_q, lam_q, mu_q):
        shp = (self.K, self.Nq)
        r, l, m = (_host(x, np.float64).reshape(shp) for x in (rho_q, lam_q, mu_q))
        self._check(self.lib.ewdg_set_material(self.h, _ptr(r), _ptr(l), _ptr(m)), "set_material")

    # ---------------------------------------------------------------- state
    def set_mass_inverse(self, mode):
        """"exact" (W_rho = M_rho^-1 M, the default) or "weight-adjusted"
        (M^-1 M_{1/rho} M^-1)."""
        codes = {"exact": 0, "weight-adjusted": 1}
        if mode not in codes:
            raise EwdgError(EWDG_EINVAL, f"unknown mass inverse {mode!r}")
        self._check(self.lib.ewdg_set_mass_inverse(self.h, codes[mode]), "set_mass_inverse")

    def set_state(self, q, t=0.0):
        torch = _torch()
        if isinstance(q, np.ndarray):
            qh = _host(q, self.np_dtype)
            if qh.size != self.K * 9 * self.Np:
                raise EwdgError(EWDG_EINVAL, "state has the wrong size")
            self._check(self.lib.ewdg_set_state(self.h, _ptr(qh), 0, float(t)), "set_state")
        else:
            qd = q.to(device="cuda", dtype=self.torch_dtype).contiguous()
            self._shape(qd, 9 * self.Np)
            with self._ordered(qd):
                self._check(self.lib.ewdg_set_state(self.h, _ptr(qd), 1, float(t)), "set_state")

    def get_state(self):
        torch = _torch()
        out = torch.empty((self.K, 9, self.Np), dtype=self.torch_dtype, device="cuda")
        t = _c_d()
        with self._ordered(out):
            self._check(self.lib.ewdg_get_state(self.h, _ptr(out), 1, ctypes.byref(t)), "get_state")
        return out

    def project_quadrature(self, fq):
        torch = _torch()
        fq = fq.to(device="cuda", dtype=torch.float64).contiguous()
        self._shape(fq, 9 * self.Nq)
        out = torch.empty((self.K, 9, self.Np), dtype=self.torch_dtype, device="cuda")
        with self._ordered(fq, out):
            self._check(self.lib.ewdg_project_quadrature(self.h, _ptr(fq), _ptr(out)), "project_quadrature")
        return out

    def eval_quadrature(self, q=None):
        torch = _torch()
        out = torch.empty((self.K, 9, self.Nq), dtype=torch.float64, device="cuda")
        if q is not None:
            assert q.is_cuda and q.dtype == self.torch_dtype and q.is_contiguous()
            self._shape(q, 9 * self.Np)
        qp = _c_p(None) if q is None else _ptr(q)
        with self._ordered(q, out):
            self._check(self.lib.ewdg_eval_quadrature(self.h, qp, _ptr(out)), "eval_quadrature")
        return out

    # ------------------------------------------------- source and receivers
    def set_source(self, xs, direction, amp, f0, t0):
        xs = _host(xs, np.float64)
        d = _host(direction, np.float64)
        self._check(self.lib.ewdg_set_source(self.h, _ptr(xs), _ptr(d), float(amp), float(f0), float(t0)),
                    "set_source")

    def clear_source(self):
        self._check(self.lib.ewdg_clear_source(self.h), "clear_source")

    def set_receivers(self, xr):
        xr = _host(xr, np.float64).reshape(-1, 3)
        self._check(self.lib.ewdg_set_receivers(self.h, xr.shape[0], _ptr(xr)), "set_receivers")
        self.nr = xr.shape[0]

    def receivers(self):
        n = _c_i()
        self._check(self.lib.ewdg_receivers(self.h, _c_p(None), ctypes.byref(n)), "receivers")
        out = np.zeros((n.value, self.nr, 3))
        if n.value and self.nr:
            self._check(self.lib.ewdg_receivers(self.h, _ptr(out), ctypes.byref(n)), "receivers")
        return out

    # ------------------------------------------------------------- stepping
    def cfl_dt(self, cfl):
        dt = _c_d()
        self._check(self.lib.ewdg_cfl_dt(self.h, float(cfl), ctypes.byref(dt)), "cfl_dt")
        return dt.value

    def rhs(self, t, q):
        torch = _torch()
        q = q.to(device="cuda", dtype=self.torch_dtype).contiguous()
        self._shape(q, 9 * self.Np)
        out = torch.empty_like(q)
        with self._ordered(q, out):
            self._check(self.lib.ewdg_rhs(self.h, float(t), _ptr(q), _ptr(out)), "rhs")
        return out

    def step(self, dt, nsteps):
        self._check(self.lib.ewdg_step(self.h, float(dt), int(nsteps)), "step")

    def time(self):
        t = _c_d()
        self._check(self.lib.ewdg_time(self.h, ctypes.byref(t)), "time")
        return t.value

    def energy(self):
        e = _c_d()
        self._check(self.lib.ewdg_energy(self.h, ctypes.byref(e)), "energy")
        return e.value

    def energy_device(self, out):
        """Enqueue the energy into out (a one-element FP64 device tensor,
        possibly a view into a larger one) on the context's stream; no sync."""
        assert out.is_cuda and out.dtype == _torch().float64 and out.numel() >= 1
        with self._ordered(out):
            self._check(self.lib.ewdg_energy_device(self.h, _ptr(out)), "energy_device")

    # -------------------------------------------------------------- adjoint
    # ------------------------------------------------ locally implicit step
    def implicit_workspace_bytes(self):
        b = _c_sz()
        self._check(self.lib.ewdg_implicit_workspace_bytes(self.h, ctypes.byref(b)), "implicit_workspace_bytes")
        return b.value

    def bind_implicit_workspace(self, buffer=None):
        torch = _torch()
        nbytes = self.implicit_workspace_bytes()
        if buffer is None:
            buffer = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        with self._ordered(buffer):
            self._check(self.lib.ewdg_bind_implicit_workspace(self.h, _ptr(buffer),
                                                              buffer.numel() * buffer.element_size()),
                        "bind_implicit_workspace")
        self._imp_ws = buffer
        return buffer

    def implicit_setup(self, dt, theta=1.0):
        """Form and invert I - theta dt A_k for every element (synchronises)."""
        self._check(self.lib.ewdg_implicit_setup(self.h, float(dt), float(theta)), "implicit_setup")

    def implicit_step(self, nsteps, tol=1e-10, max_iters=1000):
        """nsteps theta-scheme steps solved by iHDG-II; returns the iteration
        count and the final L2 change of every step (numpy arrays)."""
        iters = np.zeros(max(int(nsteps), 1), dtype=np.int32)
        change = np.zeros(max(int(nsteps), 1), dtype=np.float64)
        self._check(self.lib.ewdg_implicit_step(self.h, int(nsteps), float(tol), int(max_iters), _ptr(iters),
                                                _ptr(change)), "implicit_step")
        return iters[:nsteps], change[:nsteps]

    def implicit_dt(self):
        dt, th = _c_d(), _c_d()
        self._check(self.lib.ewdg_implicit_dt(self.h, ctypes.byref(dt), ctypes.byref(th)), "implicit_dt")
        return dt.value, th.value

    def adjoint_workspace_bytes(self, max_steps, checkpoint_every=50, overlapped=False):
        """Bytes of the adjoint workspace; overlapped=True adds the second
        segment buffer that lets the recomputation run on a second stream."""
        b = _c_sz()
        fn = self.lib.ewdg_adjoint_workspace_bytes_overlapped if overlapped else self.lib.ewdg_adjoint_workspace_bytes
        self._check(fn(self.h, int(max_steps), int(checkpoint_every), ctypes.byref(b)), "adjoint_workspace_bytes")
        return b.value

    def bind_adjoint_workspace(self, max_steps, checkpoint_every=50, buffer=None, overlapped=True):
        torch = _torch()
        nbytes = self.adjoint_workspace_bytes(max_steps, checkpoint_every, overlapped)
        if buffer is None:
            buffer = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        with self._ordered(buffer):
            self._check(self.lib.ewdg_bind_adjoint_workspace(self.h, _ptr(buffer),
                                                             buffer.numel() * buffer.element_size(),
                                                             int(max_steps), int(checkpoint_every)),
                        "bind_adjoint_workspace")
        self._adj_ws = buffer
        return buffer

    def rhs_adjoint(self, t, y, q=None, grad=False):
        """L^T y, and with grad=True also y . d(L q + f)/d theta ([K][3] FP64)."""
        torch = _torch()
        y = y.to(device="cuda", dtype=self.torch_dtype).contiguous()
        self._shape(y, 9 * self.Np)
        if q is not None:
            q = q.to(device="cuda", dtype=self.torch_dtype).contiguous()
            self._shape(q, 9 * self.Np)
        out = torch.empty_like(y)
        g = torch.empty((self.K, 3), dtype=torch.float64, device="cuda") if grad else None
        with self._ordered(y, q, out, g):
            self._check(self.lib.ewdg_rhs_adjoint(self.h, float(t), _c_p(None) if q is None else _ptr(q), _ptr(y),
                                                  _ptr(out), _c_p(None) if g is None else _ptr(g)), "rhs_adjoint")
        return (out, g) if grad else out

    def forward_misfit(self, dt, nsteps, data):
        """Run nsteps from the stored state, checkpointing; J for data[nsteps][nr][3]."""
        d = _host(data, np.float64)
        if d.size != int(nsteps) * getattr(self, "nr", 0) * 3:
            raise EwdgError(EWDG_EINVAL, "data must be [nsteps][nr][3]")
        J = _c_d()
        self._check(self.lib.ewdg_forward_misfit(self.h, float(dt), int(nsteps), _ptr(d) if d.size else _c_p(None),
                                                 ctypes.byref(J)), "forward_misfit")
        return J.value

    def adjoint_gradient(self, want_qbar0=False):
        """(g [K][3] FP64 device tensor, dJ/dq0 [K][9][Np] or None)."""
        torch = _torch()
        g = torch.empty((self.K, 3), dtype=torch.float64, device="cuda")
        qb = torch.empty((self.K, 9, self.Np), dtype=self.torch_dtype, device="cuda") if want_qbar0 else None
        with self._ordered(g, qb):
            self._check(self.lib.ewdg_adjoint_gradient(self.h, _ptr(g), _c_p(None) if qb is None else _ptr(qb)),
                        "adjoint_gradient")
        return g, qb


def batch_table_bytes(n):
    b = _c_sz()
    rc = load().ewdg_batch_table_bytes(int(n), ctypes.byref(b))
    if rc != EWDG_OK:
        raise EwdgError(rc, "batch_table_bytes")
    return b.value


def step_batch(contexts, dts, nsteps, table, stream=None):
    """ewdg_step_batch over Context objects; table is a torch device buffer
    of at least batch_table_bytes(len(contexts)) bytes.  The work runs on
    `stream` (a hipStream_t; torch's current stream if None)."""
    n = len(contexts)
    if n == 0:
        return
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    hs = (_c_p * n)(*[c.h for c in contexts])
    d = (_c_d * n)(*[float(x) for x in dts])
    cur = torch.cuda.current_stream()
    s = cur if int(stream) == cur.cuda_stream else (
        torch.cuda.default_stream() if int(stream) == 0 else torch.cuda.ExternalStream(int(stream)))
    if s is not cur:
        s.wait_stream(cur)
    rc = load().ewdg_step_batch(hs, n, d, int(nsteps), _ptr(table), table.numel() * table.element_size(),
                                _c_p(stream))
    if s is not cur:
        cur.wait_stream(s)
        table.record_stream(s)
    if rc != EWDG_OK:
        msgs = "; ".join(c.lib.ewdg_last_error(c.h).decode() for c in contexts
                         if c.lib.ewdg_last_error(c.h))
        raise EwdgError(rc, "step_batch " + msgs)


def static_table_max_bytes():
    b = _c_sz()
    rc = load().ewdg_static_table_max_bytes(ctypes.byref(b))
    if rc != EWDG_OK:
        raise EwdgError(rc, "static_table_max_bytes")
    return b.value


def step_batch_static(contexts, dts, nsteps, stream=None):
    """ewdg_step_batch_static: as step_batch, with the launch table in the
    library's fixed device array (no table buffer, nothing allocated)."""
    n = len(contexts)
    if n == 0:
        return
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    hs = (_c_p * n)(*[c.h for c in contexts])
    d = (_c_d * n)(*[float(x) for x in dts])
    cur = torch.cuda.current_stream()
    s = cur if int(stream) == cur.cuda_stream else (
        torch.cuda.default_stream() if int(stream) == 0 else torch.cuda.ExternalStream(int(stream)))
    if s is not cur:
        s.wait_stream(cur)
    rc = load().ewdg_step_batch_static(hs, n, d, int(nsteps), _c_p(stream))
    if s is not cur:
        cur.wait_stream(s)
    if rc != EWDG_OK:
        msgs = "; ".join(c.lib.ewdg_last_error(c.h).decode() for c in contexts
                         if c.lib.ewdg_last_error(c.h))
        raise EwdgError(rc, "step_batch_static " + msgs)


class Transport:
    """Steady transport beta . grad u = f on the unit square or cube, solved
    by iHDG-II on the GPU (ewdg_transport_*); arrays as in include/ewdg.h."""

    def __init__(self, dim, p, n, beta, precision=64, stream=None):
        self.lib = load()
        self.dim, self.p, self.n, self.precision = int(dim), int(p), int(n), int(precision)
        b = np.zeros(3)
        b[:self.dim] = np.asarray(beta, dtype=np.float64)[:self.dim]
        h = _c_p()
        rc = self.lib.ewdg_transport_create(self.dim, self.p, self.n, _ptr(b), self.precision, _c_p(stream),
                                            ctypes.byref(h))
        if rc != EWDG_OK:
            raise EwdgError(rc, f"ewdg_transport_create(dim={dim}, p={p}, n={n}) failed")
        self.h = h
        E, Np, Nq, Nqf = _c_i64(), _c_i(), _c_i(), _c_i()
        self._check(self.lib.ewdg_transport_sizes(self.h, ctypes.byref(E), ctypes.byref(Np), ctypes.byref(Nq),
                                                  ctypes.byref(Nqf)), "sizes")
        self.E, self.Np, self.Nq, self.Nqf = E.value, Np.value, Nq.value, Nqf.value
        self._ws = None

    def _check(self, rc, what=""):
        if rc != EWDG_OK:
            msg = self.lib.ewdg_transport_last_error(self.h) if getattr(self, "h", None) else b""
            raise EwdgError(rc, f"{what} {msg.decode() if msg else ''}".strip())

    def points(self):
        """Volume points [E][Nq][dim] and face points [E][2 dim][Nqf][dim]."""
        xv = np.zeros((self.E, self.Nq, self.dim))
        xf = np.zeros((self.E, 2 * self.dim, self.Nqf, self.dim))
        self._check(self.lib.ewdg_transport_points(self.h, _ptr(xv), _ptr(xf)), "points")
        return xv, xf

    def workspace_bytes(self):
        b = _c_sz()
        self._check(self.lib.ewdg_transport_workspace_bytes(self.h, ctypes.byref(b)), "workspace_bytes")
        return b.value

    def bind_workspace(self, buffer=None):
        torch = _torch()
        if buffer is None:
            buffer = torch.empty(self.workspace_bytes(), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        self._check(self.lib.ewdg_transport_bind_workspace(self.h, _ptr(buffer), buffer.numel()), "bind_workspace")
        self._ws = buffer
        return buffer

    def set_problem(self, f, g, ue=None):
        f = _host(f, np.float64)
        g = _host(g, np.float64)
        if f.size != self.E * self.Nq or g.size != self.E * 2 * self.dim * self.Nqf:
            raise EwdgError(EWDG_EINVAL, "f must be [E][Nq] and g [E][2 dim][Nqf]")
        if ue is not None:
            ue = _host(ue, np.float64)
            if ue.size != self.E * self.Nq:
                raise EwdgError(EWDG_EINVAL, "ue must be [E][Nq]")
        self._check(self.lib.ewdg_transport_set_problem(self.h, _ptr(f), _ptr(g), _c_p(None) if ue is None
                                                        else _ptr(ue)), "set_problem")

    def solve(self, tol=1e-10, max_iters=100000):
        """Returns (iterations, history) as in ewdg_transport_solve."""
        it = _c_i()
        hist = np.zeros(int(max_iters) + 1)
        self._check(self.lib.ewdg_transport_solve(self.h, float(tol), int(max_iters), ctypes.byref(it),
                                                  _ptr(hist)), "solve")
        return it.value, hist[:it.value + 1]

    def values(self):
        out = np.zeros((self.E, self.Nq))
        self._check(self.lib.ewdg_transport_values(self.h, _ptr(out)), "values")
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.ewdg_transport_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
