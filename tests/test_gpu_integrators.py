"""Parity of the other time integrators (six-stage SDIRK4 with its explicit
first stage, backward Euler, BDF2 with its backward-Euler start, explicit
ERK2) through the C ABI with the oracle's steppers.  Implicit steps: the
same Newton and GMRES counts per stage and 1e-12 relative per variable in
the state (as for SDIRK2/3); explicit steps: 1e-12 relative (residual evaluations and
vector updates only)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from oracle import solver as OS
from tests.gpu_util import assert_step, setup


def _ctx(cfg, mesh, **over):
    from paper_2002_04222_amd import Context
    return Context(mesh, cfg, **over)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _run(ctx, stepper, du, uo, dts, tol):
    for dt in dts:
        st = ctx.sdirk_step(du, dt)
        uo, sto = stepper.step(uo, dt)
        assert st["stages"] == len(sto)
        assert st["newton_its"] == [s.newton_its for s in sto]
        assert st["gmres_its"] == [s.gmres_its for s in sto]
        print(f"  dt {dt}: newton {st['newton_its']}", flush=True)
        assert_step(_host(du), uo, f"{type(stepper).__name__} dt {dt}", tol)
    return uo


@pytest.mark.parametrize("scheme", ["sdirk4", "beuler", "bdf2"])
def test_implicit_integrators_2d(scheme):
    _case(f"implicit step 2D 4x3 P=2 {scheme}")
    cfg, mesh, disc = setup(2, (4, 3), 2, Ma=0.3, Re=40.0, scheme=scheme)
    ctx = _ctx(cfg, mesh)
    u0 = W.random_state(mesh.n_elem, 2, 2, seed=41)
    stepper = OS.make_stepper(disc, OS.SolverOpts(scheme=scheme))
    # BDF2: a backward-Euler start, two BDF2 steps, a dt change (backward
    # Euler again, with a rebuilt preconditioner), then BDF2 at the new dt
    _run(ctx, stepper, _dev(u0), u0, [0.1, 0.1, 0.1, 0.05, 0.05], 1e-12)


def test_sdirk4_3d_and_refresh():
    _case("sdirk4 3D 3^3 P=2")
    cfg, mesh, disc = setup(3, (3, 3, 3), 2, Ma=0.3, Re=40.0, scheme="sdirk4")
    ctx = _ctx(cfg, mesh)
    u0 = W.random_state(mesh.n_elem, 3, 2, seed=43)
    stepper = OS.make_stepper(disc, OS.SolverOpts(scheme="sdirk4"))
    _run(ctx, stepper, _dev(u0), u0, [0.15, 0.15], 1e-12)


def test_erk2_explicit_steps():
    _case("erk2 2D 4x3 P=3 and 3D 3^3 P=2")
    for dim, cells, P in ((2, (4, 3), 3), (3, (3, 3, 3), 2)):
        cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0, scheme="erk2")
        ctx = _ctx(cfg, mesh)
        u0 = W.random_state(mesh.n_elem, dim, P, seed=45)
        stepper = OS.make_stepper(disc, OS.SolverOpts(scheme="erk2"))
        du = _dev(u0)
        for k in range(3):
            st = ctx.sdirk_step(du, 1e-3)
            assert st["pc_built"] == 0 and st["newton_its"] == [0, 0] and st["residual_evals"] == 2
        uo = u0
        for k in range(3):
            uo, _ = stepper.step(uo, 1e-3)
        assert_step(_host(du), uo, f"erk2 dim {dim}")


def test_bdf2_reset_history_restarts_with_backward_euler():
    _case("bdf2 reset history")
    cfg, mesh, disc = setup(2, (4, 3), 2, Ma=0.3, Re=40.0, scheme="bdf2")
    ctx = _ctx(cfg, mesh)
    u0 = W.random_state(mesh.n_elem, 2, 2, seed=47)
    du = _dev(u0)
    ctx.sdirk_step(du, 0.1)
    ctx.sdirk_step(du, 0.1)
    ctx.reset_history()
    u1 = _host(du)
    # after the reset the next step is backward Euler from u1, like a fresh stepper's first step
    stepper = OS.make_stepper(disc, OS.SolverOpts(scheme="bdf2"))
    st = ctx.sdirk_step(du, 0.1)
    uo, sto = stepper.step(u1, 0.1)
    assert st["newton_its"] == [s.newton_its for s in sto]
    assert_step(_host(du), uo, "bdf2 after reset")


@pytest.mark.parametrize("dim,cells,P,scheme", [(2, (4, 3), 3, "sdirk3"), (3, (3, 3, 3), 2, "sdirk2")])
def test_cgs2_gmres_steps(dim, cells, P, scheme):
    """GMRES with classical Gram-Schmidt applied twice: the same counts as the
    oracle's CGS2 GMRES and its state to 1e-12 per variable."""
    _case(f"cgs2 {dim}D {cells} P={P} {scheme}")
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0, scheme=scheme)
    ctx = _ctx(cfg, mesh, ortho="cgs2")
    u0 = W.random_state(mesh.n_elem, dim, P, seed=47)
    stepper = OS.make_stepper(disc, OS.SolverOpts(scheme=scheme, ortho="cgs2"))
    _run(ctx, stepper, _dev(u0), u0, [0.1, 0.1], 1e-12)
