"""GPU discrete adjoint through the C ABI.

Checks, in FP64 unless stated:
  * L^T against L: dot-product identity <L x, y> = <x, L^T y> for every
    degree, and L^T y entry by entry against <L e_j, y> on whole elements;
  * FP32 L^T y against FP64;
  * the parameter term y . d(L q + f)/d theta against central differences
    of the forward operator;
  * the misfit gradient of a recorded LSRK run against the oracle's
    complex-step derivative of its own discrete misfit, and dJ/dq0 against
    central differences;
  * MisfitFn (torch.autograd.Function) and the 1/theta chain rule.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

from helpers import oracle_case

pytestmark = pytest.mark.gpu

SRC = dict(xs=[0.05, -0.10, 0.15], direction=[0.2, -0.3, 0.9], amp=1.7, f0=5.0, t0=0.2)


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _ctx(N, prec, EToV, VXYZ, mat, max_rec=0, max_steps=1, every=1):
    import paper_1711_01175_amd as P
    c = P.Context(N, prec)
    c.set_mesh(EToV, VXYZ)
    c.bind_workspace(max_rec, max_steps if max_rec else 0)
    c.set_material(*mat)
    c.bind_adjoint_workspace(max_steps, every)
    return c


def _report(name, **kw):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


def _dot(a, b):
    return float((a.double() * b.double()).sum())


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_rhs_adjoint_dot_product(N):
    torch = _torch()
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=N, jump_seed=200 + N)
    c = _ctx(N, 64, EToV, VXYZ, mat)
    g = torch.Generator(device="cuda").manual_seed(N)
    for trial in range(3):
        x = torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda", generator=g)
        y = torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda", generator=g)
        Lx = c.rhs(0.0, x)
        LTy = c.rhs_adjoint(0.0, y)
        a, b = _dot(Lx, y), _dot(x, LTy)
        scale = float(Lx.norm() * y.norm())
        _report("dot", N=N, trial=trial, lhs=a, rhs=b, rel=abs(a - b) / scale)
        assert abs(a - b) <= 1e-13 * scale


@pytest.mark.parametrize("N", [1, 2, 3])
def test_rhs_adjoint_entries(N):
    """(L^T y)_j = <L e_j, y> for every unknown j of three elements."""
    torch = _torch()
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=N, jump_seed=300 + N)
    c = _ctx(N, 64, EToV, VXYZ, mat)
    y = torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(7))
    LTy = c.rhs_adjoint(0.0, y).cpu()
    e = torch.zeros((c.K, 9, c.Np), dtype=torch.float64, device="cuda")
    worst = 0.0
    for k in (0, 77, c.K - 1):
        for f in range(9):
            for i in range(c.Np):
                e.zero_()
                e[k, f, i] = 1.0
                col = _dot(c.rhs(0.0, e), y)
                worst = max(worst, abs(col - float(LTy[k, f, i])) / max(1.0, abs(col)))
    _report("entries", N=N, worst=worst)
    assert worst <= 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_rhs_adjoint_fp32_vs_fp64(N):
    torch = _torch()
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=N, jump_seed=400 + N)
    c64 = _ctx(N, 64, EToV, VXYZ, mat)
    c32 = _ctx(N, 32, EToV, VXYZ, mat)
    y = torch.randn((c64.K, 9, c64.Np), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(N))
    q = torch.randn((c64.K, 9, c64.Np), dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(100 + N))
    a64, g64 = c64.rhs_adjoint(0.1, y, q, grad=True)
    a32, g32 = c32.rhs_adjoint(0.1, y.float(), q.float(), grad=True)
    err = float((a32.double() - a64).norm() / a64.norm())
    gerr = float((g32 - g64).norm() / g64.norm())
    _report("fp32", N=N, LTy_rel_l2=err, g_rel_l2=gerr)
    assert err <= 1e-5 and gerr <= 1e-5


@pytest.mark.parametrize("N", [2, 4])
def test_parameter_gradient_vs_central_differences(N):
    """g = y . d(L q + f)/d theta_e against (F(1+h) - F(1-h)) / 2h with
    F(theta) = y . (L(theta) q + f(theta)), source included."""
    torch = _torch()
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=N, jump_seed=500 + N)
    c = _ctx(N, 64, EToV, VXYZ, mat)
    c.set_source(SRC["xs"], SRC["direction"], SRC["amp"], SRC["f0"], SRC["t0"])
    gen = torch.Generator(device="cuda").manual_seed(N)
    q = torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda", generator=gen)
    y = torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda", generator=gen)
    t = 0.21
    _, g = c.rhs_adjoint(t, y, q, grad=True)
    g = g.cpu().numpy()
    src_elem = op.mesh.locate(np.array(SRC["xs"]))[0]
    nb = c.connectivity()[src_elem, 0] >> 5
    h = 1e-6
    worst = 0.0
    for e in sorted({int(src_elem), int(nb), 0, 101}):
        for k in range(3):
            vals = []
            for s in (1 + h, 1 - h):
                m = [x.copy() for x in mat]
                m[k][e] *= s
                c.set_material(*m)
                vals.append(_dot(c.rhs(t, q), y))
            fd = (vals[0] - vals[1]) / (2 * h)
            worst = max(worst, abs(fd - g[e, k]))
            _report("param", N=N, e=e, k=k, adjoint=float(g[e, k]), fd=fd)
    scale = np.abs(g).max()
    _report("param", N=N, worst=worst, scale=float(scale))
    assert worst <= 1e-6 * scale


def _misfit_case(N=2, n=3, nsteps=15):
    from oracle import adjoint, timestep
    op, EToV, VXYZ, xyz, mat = oracle_case(N, n, shuffle_seed=1, jump_seed=3)
    src = timestep.Source(np.array(SRC["xs"]), np.array(SRC["direction"]), SRC["amp"], SRC["f0"], SRC["t0"])
    rec = np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, -0.6]])
    dt = timestep.cfl_dt(op, 0.5)
    c0 = np.zeros((op.K, 9, op.Np))
    _, tr = adjoint.misfit(N, VXYZ, *mat, c0, dt, nsteps, src, rec, np.zeros((nsteps, 2, 3)), t0=0.1)
    data = 0.7 * tr[::-1]
    return N, op, EToV, VXYZ, mat, src, rec, dt, nsteps, data


def test_misfit_gradient_vs_oracle_complex_step():
    """Recorded run with checkpoints every 4 of 15 steps (ragged last
    segment): J and dJ/dtheta against the oracle's complex step."""
    _torch()
    from oracle import adjoint
    N, op, EToV, VXYZ, mat, src, rec, dt, nsteps, data = _misfit_case()
    elems = [0, 17, int(op.mesh.locate(src.xs)[0]), 140]
    Jo, _ = adjoint.misfit(N, VXYZ, *mat, np.zeros((op.K, 9, op.Np)), dt, nsteps, src, rec, data, t0=0.1)
    go = adjoint.complex_step_gradient(N, VXYZ, *mat, np.zeros((op.K, 9, op.Np)), dt, nsteps, src, rec, data,
                                       elems, t0=0.1)
    c = _ctx(N, 64, EToV, VXYZ, mat, max_rec=2, max_steps=nsteps, every=4)
    c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
    c.set_receivers(rec)
    import torch
    c.set_state(torch.zeros((c.K, 9, c.Np), dtype=torch.float64, device="cuda"), 0.1)
    J = c.forward_misfit(dt, nsteps, data)
    g, _ = c.adjoint_gradient()
    g = g.cpu().numpy()[elems]
    jerr = abs(J - Jo) / abs(Jo)
    gerr = np.abs(g - go).max() / np.abs(go).max()
    _report("misfit", J=J, J_oracle=Jo, J_rel=jerr, g_rel_max=gerr)
    assert jerr <= 1e-12
    assert gerr <= 1e-9


def test_overlapped_sweep_is_bitwise_single_buffer_sweep():
    """The reverse sweep with the second segment buffer (next segment
    recomputed on a second stream) gives the same bits as the single-buffer
    sweep: 15 steps in segments of 4 (ragged last), FP32 and FP64."""
    torch = _torch()
    import paper_1711_01175_amd as P
    N, op, EToV, VXYZ, mat, src, rec, dt, nsteps, data = _misfit_case()
    for prec in (32, 64):
        out = {}
        for overlapped in (False, True):
            c = P.Context(N, prec)
            c.set_mesh(EToV, VXYZ)
            c.bind_workspace(2, nsteps)
            c.set_material(*mat)
            ws = c.bind_adjoint_workspace(nsteps, 4, overlapped=overlapped)
            assert ws.numel() == c.adjoint_workspace_bytes(nsteps, 4, overlapped)
            c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
            c.set_receivers(rec)
            gen = torch.Generator(device="cuda").manual_seed(5)
            q0 = 0.1 * torch.randn((c.K, 9, c.Np), dtype=c.torch_dtype, device="cuda", generator=gen)
            c.set_state(q0, 0.1)
            J = c.forward_misfit(dt, nsteps, data)
            g, qbar = c.adjoint_gradient(want_qbar0=True)
            out[overlapped] = (J, g.cpu().numpy(), qbar.cpu().numpy())
            c.close()
        _report("overlap", prec=prec, J=out[True][0], g_max=float(np.abs(out[True][1]).max()))
        assert out[True][0] == out[False][0]
        assert np.array_equal(out[True][1], out[False][1])
        assert np.array_equal(out[True][2], out[False][2])


@pytest.mark.parametrize("N,n,nsteps", [(2, 3, 15), (5, 3, 10)])
def test_initial_state_gradient_vs_central_differences(N, n, nsteps):
    """dJ/dq0 from the reverse sweep against central differences (J is
    quadratic in q0).  N=5 in FP64 runs the LDS-staged pass B (its
    matrix-core tile does not fit in LDS), N=2 the matrix-core one."""
    torch = _torch()
    N, op, EToV, VXYZ, mat, src, rec, dt, nsteps, data = _misfit_case(N, n, nsteps)
    c = _ctx(N, 64, EToV, VXYZ, mat, max_rec=2, max_steps=nsteps, every=6)
    c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
    c.set_receivers(rec)
    gen = torch.Generator(device="cuda").manual_seed(11)
    q0 = 0.1 * torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda", generator=gen)
    d = torch.randn((c.K, 9, c.Np), dtype=torch.float64, device="cuda", generator=gen)
    c.set_state(q0, 0.1)
    c.forward_misfit(dt, nsteps, data)
    _, qbar = c.adjoint_gradient(want_qbar0=True)
    h = 1e-3
    Js = []
    for s in (h, -h):
        c.set_state(q0 + s * d, 0.1)
        Js.append(c.forward_misfit(dt, nsteps, data))
    fd = (Js[0] - Js[1]) / (2 * h)
    ad = _dot(qbar, d)
    _report("dJ/dq0", N=N, adjoint=ad, fd=fd, rel=abs(ad - fd) / abs(fd))
    assert abs(ad - fd) <= 1e-10 * abs(fd)


def test_misfitfn_autograd_chain_rule():
    torch = _torch()
    from paper_1711_01175_amd.adjoint import MisfitFn, MisfitProblem
    N, op, EToV, VXYZ, mat, src, rec, dt, nsteps, data = _misfit_case()
    p = MisfitProblem(N, EToV, VXYZ, *mat, (src.xs, src.direction, src.amp, src.f0, src.t0), rec, data, dt,
                      nsteps, precision=64, checkpoint_every=5, t0=0.1)
    theta0 = 1.0 + 0.05 * np.random.default_rng(2).standard_normal((op.K, 3))
    theta = torch.tensor(theta0, dtype=torch.float64, device="cuda", requires_grad=True)
    J = MisfitFn.apply(theta, p)
    J.backward()
    gt = theta.grad.cpu().numpy()
    e = int(op.mesh.locate(src.xs)[0])
    h = 1e-6
    worst = 0.0
    for k in range(3):
        vals = []
        for s in (h, -h):
            th = theta0.copy()
            th[e, k] += s
            vals.append(p.misfit(th))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst = max(worst, abs(fd - gt[e, k]) / np.abs(gt[e]).max())
        _report("autograd", k=k, adjoint=float(gt[e, k]), fd=fd)
    assert worst <= 1e-7
    assert float(J.detach()) > 0
    p.close()
