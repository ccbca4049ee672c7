"""Parity of the HIP path with the oracle on meshes with boundary faces:
1D characteristic far field and adiabatic no-slip walls (ghost states with
the interior gradient).  Tolerances as for the periodic parity tests:
residual 1e-12 relative per variable, matvec 1e-6, SDIRK steps 1e-12 per variable.
BRJ blocks 5e-6 and applies 1e-5: where a far-field face lies in the
inflow/outflow blend (|u_nb| below ~0.02 c_b) the forward difference of Eq.
31 divides the rounding of u_nb = (R+ + R-)/2 (|R+-| ~ 2c/(gamma-1)),
steepened by the blend's slope 1/(0.04 c_b), by chi (~1e-8 for the smallest
variable): both sides' blocks then differ by ~1e-6, and 7 sweeps compound
it."""
import dataclasses
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from oracle import solver as OS
from oracle.dg import Disc
from oracle.physics import Gas, BC_FARFIELD, BC_WALL
from tests.gpu_util import assert_step, rel_err_per_var


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _freestream(dim, Ma):
    gas = Gas(Ma=Ma)
    vel = np.zeros(dim)
    vel[0], vel[1] = 0.3, 0.1
    if dim == 3:
        vel[2] = 0.05     # every variable non-zero (the BRJ differencing step scales with its norm)
    p = 1.0 / (gas.gamma * Ma * Ma)
    return np.concatenate([[1.0], vel, [p / (gas.gamma - 1) + 0.5 * vel @ vel]])


def _setup(dim, cells, P, periodic, kinds, Ma=0.3, Re=40.0, **over):
    """(cfg, mesh, oracle disc, bc_kind, bc_state): face ids 2*axis+side."""
    base = W.config(1 if dim == 2 else 2)
    lengths = tuple(1.0 + 0.3 * i for i in range(dim))
    cfg = dataclasses.replace(base, dim=dim, ncells=tuple(cells), lengths=lengths, P=P, nq=P + 2, Ma=Ma, Re=Re,
                              **over)
    mesh = W.cartesian_mesh(cells, lengths, periodic=periodic, bc_ids=list(range(2 * dim)))
    Uinf = _freestream(dim, Ma)
    state = np.array([Uinf] * (2 * dim))
    kinds = np.array(kinds, dtype=np.int32)
    gas = Gas(gamma=cfg.gamma, Pr=cfg.Pr, Re=Re, Ma=Ma, visc_law=cfg.visc_law, T_ref_K=cfg.T_ref_K,
              flux_mode=cfg.flux_mode, riemann=cfg.riemann)
    disc = Disc(gas=gas, dim=dim, P=P, nq=P + 2, elem_origin=mesh.elem_origin, elem_h=mesh.elem_h,
                face_nbr=mesh.face_nbr, bc_kind=kinds, bc_state=state)
    return cfg, mesh, disc, kinds, state


def _ctx(cfg, mesh, kinds, state):
    from paper_2002_04222_amd import Context
    return Context(mesh, cfg, bc_kind=kinds, bc_state=state)


FF, WL = BC_FARFIELD, BC_WALL
CASES = [
    # dim, cells, P, periodic, kinds, flux_mode, riemann
    (2, (3, 3), 2, [False, False], [FF, FF, WL, WL], 0, 0),
    (2, (4, 3), 3, [False, True], [FF, FF, WL, WL], 0, 1),
    (2, (3, 2), 1, [False, False], [WL, FF, FF, WL], 1, 0),
    (3, (2, 3, 2), 2, [False, False, True], [FF, FF, WL, WL, FF, FF], 0, 0),
    (3, (2, 2, 2), 3, [False, True, False], [FF, FF, WL, WL, WL, WL], 0, 0),
]


@pytest.mark.parametrize("dim,cells,P,periodic,kinds,mode,riemann", CASES)
def test_bc_residual_parity(dim, cells, P, periodic, kinds, mode, riemann):
    _case(f"bc residual dim={dim} cells={cells} P={P} kinds={kinds} mode={mode} riemann={riemann}")
    cfg, mesh, disc, k, st = _setup(dim, cells, P, periodic, kinds, flux_mode=mode, riemann=riemann)
    ctx = _ctx(cfg, mesh, k, st)
    u = W.random_state(mesh.n_elem, dim, P, seed=200 + P, mean=st[0])
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    Ro = disc.residual(u)
    assert rel_err_per_var(_host(R), Ro) <= 1e-12


def test_bc_freestream_preserved():
    _case("bc freestream 3D P=3 far field")
    dim, P = 3, 3
    cfg, mesh, disc, k, st = _setup(dim, (2, 3, 2), P, [False] * 3, [FF] * 6)
    ctx = _ctx(cfg, mesh, k, st)
    u = np.zeros(disc.shape)
    u[:, :, 0] = st[0] * 2 ** (dim / 2)
    R = ctx.empty()
    ctx.residual(_dev(u), R)
    scale = np.abs(disc.residual(W.random_state(mesh.n_elem, dim, P, seed=1, mean=st[0]))).max()
    assert np.abs(_host(R)).max() <= 1e-12 * scale


def test_bc_matvec_and_precond_parity():
    _case("bc matvec + precond 2D P=2")
    cfg, mesh, disc, k, st = _setup(2, (3, 4), 2, [False, False], [FF, FF, WL, WL])
    ctx = _ctx(cfg, mesh, k, st)
    u = W.random_state(mesh.n_elem, 2, 2, seed=211, mean=st[0])
    S = 0.999 * u
    dt_a = 0.05
    No = disc.stage_residual(u, S, dt_a)
    v = W.random_vector(mesh.n_elem, 2, 2, seed=212)
    eps = OS.jfnk_eps(u)
    Jv = ctx.empty()
    ctx.jfnk_matvec(_dev(u), _dev(No), _dev(S), dt_a, _dev(v), eps, Jv)
    Jo = OS.jfnk_matvec(disc, u, No, S, dt_a, v, eps)
    assert np.linalg.norm(_host(Jv) - Jo) <= 1e-6 * np.linalg.norm(Jo)
    ctx.precond_build(_dev(u), dt_a)
    pc = OS.BRJ(disc, u, dt_a)
    nb = disc.nv * disc.ref.nm
    out = torch.empty((mesh.n_elem, nb, nb), dtype=torch.float64, device="cuda")
    ctx.precond_diag_inverse(out)
    Dg = _host(out)
    assert np.abs(Dg - pc.Dinv).max() <= 5e-6 * np.abs(pc.Dinv).max()
    q = W.random_vector(mesh.n_elem, 2, 2, seed=213)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    assert np.abs(_host(o) - ref).max() <= 1e-5 * np.abs(ref).max()


def test_bc_precond_parity_3d():
    _case("bc precond 3D P=2")
    cfg, mesh, disc, k, st = _setup(3, (2, 2, 3), 2, [False, True, False], [WL, FF, FF, FF, FF, WL])
    ctx = _ctx(cfg, mesh, k, st)
    u = W.random_state(mesh.n_elem, 3, 2, seed=221, mean=st[0])
    ctx.precond_build(_dev(u), 0.1)
    pc = OS.BRJ(disc, u, 0.1)
    q = W.random_vector(mesh.n_elem, 3, 2, seed=222)
    o = ctx.empty()
    ctx.precond_apply(_dev(q), o)
    ref = pc.apply(q)
    assert np.abs(_host(o) - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("scheme", ["sdirk2", "sdirk3"])
def test_bc_sdirk_step_parity(scheme):
    _case(f"bc sdirk step {scheme}")
    cfg, mesh, disc, k, st = _setup(2, (4, 3), 2, [False, False], [FF, FF, WL, WL], scheme=scheme)
    ctx = _ctx(cfg, mesh, k, st)
    u0 = W.random_state(mesh.n_elem, 2, 2, seed=231, mean=st[0])
    du = _dev(u0)
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme=scheme))
    uo = u0
    for k in range(2):
        s = ctx.sdirk_step(du, 0.1)
        uo, so = stepper.step(uo, 0.1)
        assert s["newton_its"] == [x.newton_its for x in so]
        assert s["gmres_its"] == [x.gmres_its for x in so]
        assert_step(_host(du), uo, f"walls + far field {scheme} step {k}")


def test_bc_create_rejects_bad_ids_and_kinds():
    _case("bc create errors")
    from paper_2002_04222_amd import DgjError
    cfg, mesh, disc, k, st = _setup(2, (3, 3), 2, [False, False], [FF, FF, WL, WL])
    with pytest.raises(DgjError) as ei:
        _ctx(cfg, mesh, k[:2], st[:2])       # ids 2 and 3 undefined
    assert ei.value.code == -1
    for kind in (8, -1):                      # kinds 0..7 exist
        bad = k.copy()
        bad[0] = kind
        with pytest.raises(DgjError):
            _ctx(cfg, mesh, bad, st)
    neg = st.copy()
    neg[0, 0] = -1.0
    with pytest.raises(DgjError):
        _ctx(cfg, mesh, k, neg)
    from paper_2002_04222_amd import Context
    with pytest.raises(DgjError):
        Context(mesh, cfg)                    # boundary faces but no boundary ids
