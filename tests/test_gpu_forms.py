"""The precision form (Sec. 4.2.2: the paper already stores the block
inverses in single precision) against the FP64 oracle: SDIRK steps whose
BRJ blocks are stored and applied in FP32 or BF16 (FP32 accumulation),
with the residual, the Frechet perturbation, GMRES and the Newton update in
FP64, compared with the oracle's plain FP64 step at the same Newton
tolerance (alpha = 1e-8 relative to ||N(S_m)||).  Both runs meet that
tolerance, so the states differ by at most about the Newton tolerance times
the conditioning of the stage system: the bar is 1e-8 per variable.  The
Newton and GMRES counts of both runs are printed (the reduced-precision
blocks may change the GMRES counts, not the Newton tolerance)."""
import dataclasses
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from oracle import solver as OS
from oracle.dg import initial_state, make_disc
from tests.gpu_util import assert_step

FORM_TOL = 1e-8


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _taylor_green(cfg, mesh, disc, prec):
    from paper_2002_04222_amd import Context
    ctx = Context(mesh, cfg, pc_precision=prec)
    noise = W.noise(disc.shape, cfg.seed)
    u = ctx.empty()
    ctx.project_tgv(_dev(noise), cfg.noise_amp, u)
    return ctx, u, initial_state(disc, noise, cfg.noise_amp)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_reduced_precision_step_tgv2d_workload(prec):
    """The 2D Taylor-Green workload (8x8, P=2, Re 100, Ma 0.1), one SDIRK2
    step at CFL 20."""
    _case(f"{prec} blocks: SDIRK2 step of tgv2d 8x8 P=2 vs the FP64 oracle")
    cfg = W.config(1)
    mesh = cfg.mesh()
    disc = make_disc(cfg, mesh)
    ctx, u, u0 = _taylor_green(cfg, mesh, disc, prec)
    st = ctx.sdirk_step(u, cfg.dt())
    uo, sto = OS.SDIRK(disc, OS.SolverOpts(scheme=cfg.scheme)).step(u0, cfg.dt())
    print(f"device {prec}: newton {st['newton_its']} gmres {st['gmres_its']}", flush=True)
    print(f"oracle f64: newton {[s.newton_its for s in sto]} gmres {[s.gmres_its for s in sto]}", flush=True)
    assert_step(_host(u), uo, f"{prec} blocks, tgv2d SDIRK2 step", FORM_TOL)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_reduced_precision_steps_tgv3d_p3(prec):
    """The 3D Taylor-Green problem on 3^3 hexahedra of the same cube at
    P = 3 (320 x 320 blocks), Re 1600, Ma 0.1, the benchmark's time step,
    two SDIRK3 steps; each step is compared with the oracle's FP64 step
    from the device's previous state."""
    _case(f"{prec} blocks: two SDIRK3 steps of tgv3d 3^3 P=3 vs the FP64 oracle")
    big = W.config(2)
    cfg = dataclasses.replace(big, ncells=(3, 3, 3))
    mesh = cfg.mesh()
    disc = make_disc(cfg, mesh)
    ctx, u, u0 = _taylor_green(cfg, mesh, disc, prec)
    dt = big.dt()
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme=cfg.scheme))
    uprev = u0
    for k in range(2):
        st = ctx.sdirk_step(u, dt)
        uo, sto = stepper.step(uprev, dt)
        print(f"step {k} device {prec}: newton {st['newton_its']} gmres {st['gmres_its']}", flush=True)
        print(f"step {k} oracle f64: newton {[s.newton_its for s in sto]} gmres {[s.gmres_its for s in sto]}",
              flush=True)
        ug = _host(u)
        assert_step(ug, uo, f"{prec} blocks, tgv3d 3^3 P=3 SDIRK3 step {k}", FORM_TOL)
        uprev = ug
