"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances: residual and stage residual 1e-12 relative per variable (FP64
with a different summation order); the Jacobian-free matvec 1e-6 (the
forward difference amplifies rounding by ~1/sqrt(eps_hat)); preconditioner
blocks and apply 1e-6 (forward-difference face Jacobians, Eq. 31); SDIRK
steps 1e-12 relative per variable in the state (Newton contracts early
differences; both runs take identical Newton and GMRES counts)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from oracle import solver as OS
from oracle.dg import initial_state
from tests.gpu_util import assert_step, rel_err_per_var, setup


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


RES_CASES = [
    (2, (3, 2), 1, 0, 0), (2, (3, 2), 2, 0, 0), (2, (4, 3), 3, 0, 0), (2, (2, 3), 4, 0, 0), (2, (3, 3), 5, 0, 0),
    (2, (3, 2), 2, 1, 0), (2, (3, 2), 2, 2, 0), (2, (3, 2), 2, 0, 1),
    (3, (2, 2, 3), 1, 0, 0), (3, (2, 3, 2), 2, 0, 0), (3, (3, 2, 2), 3, 0, 0), (3, (2, 2, 2), 4, 0, 0),
    (3, (2, 2, 3), 3, 1, 0), (3, (2, 2, 3), 2, 0, 1),
]


@pytest.mark.parametrize("dim,cells,P,mode,riemann", RES_CASES)
def test_residual_parity(dim, cells, P, mode, riemann):
    _case(f"residual dim={dim} cells={cells} P={P} mode={mode} riemann={riemann}")
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0, flux_mode=mode, riemann=riemann)
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, dim, P, seed=100 + P)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    Rg = _host(R)
    Ro = disc.residual(u)
    assert rel_err_per_var(Rg, Ro) <= 1e-12
    # conservation: element sums of the mode-0 component of M R cancel
    detJ = disc.detJ[:, None]
    tot = (Rg[:, :, 0] * detJ).sum(0)
    assert np.all(np.abs(tot) <= 1e-13 * np.abs(Rg[:, :, 0] * detJ).sum(0) + 1e-300)


@pytest.mark.parametrize("dim,cells,P", [(2, (3, 2), 3), (3, (2, 2, 3), 2)])
def test_residual_parity_sutherland(dim, cells, P):
    """Sutherland's viscosity law (visc_law 1): a state whose temperature
    varies by a few percent, so mu(T) varies over the mesh."""
    _case(f"residual Sutherland dim={dim} cells={cells} P={P}")
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0, visc_law=1)
    assert disc.gas.visc_law == 1
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, dim, P, seed=150 + P, amp=0.1)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    assert rel_err_per_var(_host(R), disc.residual(u)) <= 1e-12


def test_precond_and_step_parity_sutherland():
    _case("precond + SDIRK2 steps Sutherland 2D P=2")
    cfg, mesh, disc = setup(2, (4, 3), 2, Ma=0.3, Re=40.0, visc_law=1, scheme="sdirk2")
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, 2, 2, seed=161, amp=0.1)
    ctx.precond_build(_dev(u), 0.1)
    pc = OS.BRJ(disc, u, 0.1)
    nb = disc.nv * disc.ref.nm
    out = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
    ctx.precond_diag_inverse(out)
    assert np.abs(_host(out) - pc.Dinv).max() <= 1e-6 * np.abs(pc.Dinv).max()
    ctx2 = _ctx(cfg, mesh)
    du = _dev(u)
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme="sdirk2"))
    uo = u
    for k in range(2):
        st = ctx2.sdirk_step(du, 0.1)
        uo, sto = stepper.step(uo, 0.1)
        assert st["newton_its"] == [s.newton_its for s in sto]
        assert st["gmres_its"] == [s.gmres_its for s in sto]
        assert_step(_host(du), uo, f"Sutherland SDIRK2 step {k}")


def test_residual_parity_nonuniform_sizes():
    _case("residual non-uniform element sizes")
    cfg, mesh, disc = setup(2, (4, 3), 2, Ma=0.3, Re=40.0)
    rng = np.random.default_rng(0)
    # stretch columns/rows while keeping a conforming grid
    hx = rng.uniform(0.5, 1.5, 4)
    hy = rng.uniform(0.5, 1.5, 3)
    ix = np.arange(mesh.n_elem) % 4
    iy = np.arange(mesh.n_elem) // 4
    mesh.elem_h[:, 0] = hx[ix]
    mesh.elem_h[:, 1] = hy[iy]
    from oracle.dg import make_disc
    disc = make_disc(cfg, mesh)
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, 2, 2, seed=7)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    assert rel_err_per_var(_host(R), disc.residual(u)) <= 1e-12


def test_stage_residual_and_matvec_parity():
    _case("stage residual + matvec 3D P=2")
    cfg, mesh, disc = setup(3, (2, 3, 2), 2, Ma=0.3, Re=40.0)
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, 3, 2, seed=11)
    S = 0.999 * u
    dt_a = 0.05
    du, dS = _dev(u), _dev(S)
    N = ctx.empty()
    ctx.stage_residual(du, dS, dt_a, N)
    No = disc.stage_residual(u, S, dt_a)
    Ng = _host(N)
    assert np.abs(Ng - No).max() <= 1e-12 * np.abs(No).max()
    v = W.random_vector(mesh.n_elem, 3, 2, seed=12)
    eps = OS.jfnk_eps(u)
    Jv = ctx.empty()
    # both sides take the same stored N(u) (the oracle's) and eps
    ctx.jfnk_matvec(du, _dev(No), dS, dt_a, _dev(v), eps, Jv)
    Jo = OS.jfnk_matvec(disc, u, No, S, dt_a, v, eps)
    assert np.linalg.norm(_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)
    # eps <= 0 selects Eq. 26 on the device
    ctx.jfnk_matvec(du, _dev(No), dS, dt_a, _dev(v), 0.0, Jv)
    assert np.linalg.norm(_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)


# 3D P = 2 and 4 have odd block sizes (135, 625): FP64 blocks stored with
# padding rows (columns of whole cache lines: 144, 640 rows)
@pytest.mark.parametrize("dim,cells,P", [(2, (3, 3), 2), (3, (2, 2, 3), 1), (3, (2, 2, 2), 3), (3, (2, 1, 1), 4),
                                         (2, (2, 2), 1), (3, (3, 2, 2), 2)])
def test_precond_parity(dim, cells, P):
    _case(f"precond build/apply dim={dim} P={P}")
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0)
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, dim, P, seed=21)
    dt_a = 0.1
    ctx.precond_build(_dev(u), dt_a)
    pc = OS.BRJ(disc, u, dt_a)
    nb = disc.nv * disc.ref.nm
    out = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
    ctx.precond_diag_inverse(out)
    Dg = _host(out)
    assert np.abs(Dg - pc.Dinv).max() <= 1e-6 * np.abs(pc.Dinv).max()
    q = W.random_vector(mesh.n_elem, dim, P, seed=22)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    assert np.abs(_host(o) - ref).max() <= 1e-6 * np.abs(ref).max()


# block sizes 320 (3D P = 3), 135 (3D P = 2: padded to 136 rows in FP32
# and BF16) and 36 (2D P = 2: padded to 40 rows in BF16)
@pytest.mark.parametrize("dim,cells,P", [(3, (2, 2, 2), 3), (3, (2, 2, 3), 2), (2, (3, 3), 2)])
@pytest.mark.parametrize("prec,tol", [("f32", 1e-4), ("bf16", 3e-2)])
def test_precond_reduced_precision(prec, tol, dim, cells, P):
    _case(f"precond {prec} dim={dim} P={P}")
    cfg, mesh, disc = setup(dim, cells, P, Ma=0.3, Re=40.0, pc_precision=prec)
    ctx = _ctx(cfg, mesh)
    u = W.random_state(mesh.n_elem, dim, P, seed=23)
    ctx.precond_build(_dev(u), 0.1)
    pc = OS.BRJ(disc, u, 0.1)
    nb = disc.nv * disc.ref.nm
    out = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
    ctx.precond_diag_inverse(out)
    assert np.abs(_host(out) - pc.Dinv).max() <= tol * np.abs(pc.Dinv).max()
    q = W.random_vector(mesh.n_elem, dim, P, seed=24)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    assert np.abs(_host(o) - ref).max() <= tol * np.abs(ref).max()


def test_gmres_and_newton_parity():
    _case("gmres + newton 2D P=2")
    cfg, mesh, disc = setup(2, (4, 4), 2, Ma=0.3, Re=40.0)
    ctx = _ctx(cfg, mesh)
    un = W.random_state(mesh.n_elem, 2, 2, seed=31)
    dt_a = 0.05
    ctx.precond_build(_dev(un), dt_a)
    pc = OS.BRJ(disc, un, dt_a)
    No = disc.stage_residual(un, un, dt_a)
    eps = OS.jfnk_eps(un)
    x = ctx.empty()
    its = ctx.gmres(_dev(un), _dev(No), _dev(un), dt_a, eps, _dev(-No), x)
    mv = lambda q: OS.jfnk_matvec(disc, un, No, un, dt_a, q, eps)
    xo, itso, ok, _ = OS.gmres(mv, pc.apply, -No, cfg.gmres_restart, cfg.gmres_rtol, cfg.gmres_max)
    assert its == itso
    assert np.abs(_host(x) - xo).max() <= 1e-6 * np.abs(xo).max()
    du = _dev(un)
    nit, git = ctx.newton(_dev(un), dt_a, du)
    uo, st = OS.newton_solve(disc, un, dt_a, pc, OS.SolverOpts())
    assert nit == st.newton_its and git == st.gmres_its
    assert_step(_host(du), uo, "newton 2D P=2")


def test_project_tgv_parity():
    _case("project tgv")
    cfg = W.config(1)
    mesh = cfg.mesh()
    from oracle.dg import make_disc
    disc = make_disc(cfg, mesh)
    ctx = _ctx(cfg, mesh)
    noise = W.noise(disc.shape, cfg.seed)
    u = ctx.empty()
    ctx.project_tgv(_dev(noise), cfg.noise_amp, u)
    uo = initial_state(disc, noise, cfg.noise_amp)
    assert rel_err_per_var(_host(u), uo) <= 1e-13


@pytest.mark.parametrize("P,cells", [(4, (3, 3)), (5, (3, 2))])
def test_sdirk_step_parity_high_order_2d(P, cells):
    """2D P = 4 and 5 (the batching workload's upper orders): two SDIRK2
    steps with identical counts and 1e-12 per variable."""
    _case(f"sdirk2 steps 2D P={P} cells={cells}")
    cfg, mesh, disc = setup(2, cells, P, Ma=0.3, Re=40.0, scheme="sdirk2")
    ctx = _ctx(cfg, mesh)
    u0 = W.random_state(mesh.n_elem, 2, P, seed=45)
    du = _dev(u0)
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme="sdirk2"))
    uo = u0
    for k in range(2):
        st = ctx.sdirk_step(du, 0.05)
        uo, sto = stepper.step(uo, 0.05)
        assert st["newton_its"] == [s.newton_its for s in sto]
        assert st["gmres_its"] == [s.gmres_its for s in sto]
        assert_step(_host(du), uo, f"2D P={P} SDIRK2 step {k}")


@pytest.mark.parametrize("scheme", ["sdirk2", "sdirk3"])
def test_sdirk_step_parity_small(scheme):
    _case(f"sdirk step small {scheme}")
    cfg, mesh, disc = setup(2, (4, 3), 2, Ma=0.3, Re=40.0, scheme=scheme)
    ctx = _ctx(cfg, mesh)
    u0 = W.random_state(mesh.n_elem, 2, 2, seed=41)
    du = _dev(u0)
    dt = 0.1
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme=scheme))
    uo = u0
    for k in range(2):
        st = ctx.sdirk_step(du, dt)
        uo, sto = stepper.step(uo, dt)
        assert st["newton_its"] == [s.newton_its for s in sto]
        assert st["gmres_its"] == [s.gmres_its for s in sto]
        assert_step(_host(du), uo, f"{scheme} 4x3 P=2 step {k}")


def test_sdirk_step_parity_tgv2d_workload():
    """The 2D Taylor-Green workload: 8x8 P=2, Re 100, Ma 0.1, SDIRK2 at CFL 20."""
    _case("sdirk step tgv2d 8x8 P=2")
    cfg = W.config(1)
    mesh = cfg.mesh()
    from oracle.dg import make_disc
    disc = make_disc(cfg, mesh)
    ctx = _ctx(cfg, mesh)
    noise = W.noise(disc.shape, cfg.seed)
    u = ctx.empty()
    ctx.project_tgv(_dev(noise), cfg.noise_amp, u)
    u0 = initial_state(disc, noise, cfg.noise_amp)
    st = ctx.sdirk_step(u, cfg.dt())
    uo, sto = OS.SDIRK(disc, OS.SolverOpts(scheme=cfg.scheme)).step(u0, cfg.dt())
    ug = _host(u)
    print("tgv2d step counts", st["newton_its"], st["gmres_its"], flush=True)
    assert st["newton_its"] == [s.newton_its for s in sto]
    assert st["gmres_its"] == [s.gmres_its for s in sto]
    assert_step(ug, uo, "tgv2d 8x8 P=2 SDIRK2 CFL 20")


def test_residual_bitwise_repeatable_and_full_workload():
    """At the benchmark's full size (3D Taylor-Green, 16^3 hexahedra, P=3,
    the launch configuration bench.py times): residual and Jacobian-free
    matvec against the oracle, and two evaluations bitwise identical."""
    _case("full workload residual + matvec, 16^3 P=3")
    cfg = W.config(2)
    mesh = cfg.mesh()
    from oracle.dg import make_disc
    disc = make_disc(cfg, mesh)
    ctx = _ctx(cfg, mesh)
    noise = W.noise(disc.shape, cfg.seed)
    u = ctx.empty()
    ctx.project_tgv(_dev(noise), cfg.noise_amp, u)
    u0 = initial_state(disc, noise, cfg.noise_amp)
    R1, R2 = ctx.empty(), ctx.empty()
    ctx.residual(_dev(u0), R1)
    ctx.residual(_dev(u0), R2)
    r1, r2 = _host(R1), _host(R2)
    assert np.array_equal(r1, r2)
    Ro = disc.residual(u0)
    # At Ma 0.1 the single terms summed into R are of size U (c+|u|)(P+1)^2 2/h
    # with U up to the energy coefficient (c = 1/Ma), ~1e5 here, and cancel
    # down to |R| ~ 1..100: FP64 rounding of a few such terms bounds the
    # agreement, 1e-12 of |R_v| plus 2e-16 (one unit roundoff) of the largest term.
    h = mesh.elem_h.min()
    term = np.abs(u0).max() * (1.0 / cfg.Ma + 1.0) * (cfg.P + 1) ** 2 * 2.0 / h
    for v in range(disc.nv):
        err = np.abs(r1[:, v] - Ro[:, v]).max()
        assert err <= 1e-12 * np.abs(Ro[:, v]).max() + 2e-16 * term, (v, err, term)
    dt_a = cfg.dt() * 0.4358665215
    No = disc.stage_residual(u0, u0, dt_a)
    v = W.random_vector(mesh.n_elem, 3, cfg.P, seed=5)
    eps = OS.jfnk_eps(u0)
    Jv = ctx.empty()
    ctx.jfnk_matvec(_dev(u0), _dev(No), _dev(u0), dt_a, _dev(v), eps, Jv)
    Jo = OS.jfnk_matvec(disc, u0, No, u0, dt_a, v, eps)
    assert np.linalg.norm(_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)


def test_sdirk_step_parity_with_preconditioner_refresh():
    """The refresh rules (rebuild at S_m after a stage whose GMRES took more
    than pc_refresh_its iterations) taken on both sides: identical counts."""
    _case("sdirk step with refresh")
    cfg, mesh, disc = setup(2, (4, 3), 2, Ma=0.3, Re=40.0, scheme="sdirk3", pc_refresh_its=2)
    ctx = _ctx(cfg, mesh)
    u0 = W.random_state(mesh.n_elem, 2, 2, seed=43)
    du = _dev(u0)
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme="sdirk3", pc_refresh_its=2))
    uo = u0
    builds = 0
    for k in range(2):
        st = ctx.sdirk_step(du, 0.2)
        builds += st["pc_built"]
        uo, sto = stepper.step(uo, 0.2)
        assert st["newton_its"] == [s.newton_its for s in sto]
        assert st["gmres_its"] == [s.gmres_its for s in sto]
        assert_step(_host(du), uo, f"sdirk3 refresh step {k}")
    assert builds >= 2
