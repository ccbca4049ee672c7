"""The learned Newton guess on the GPU: MLP forward and gradient against
the FP64 oracle (BF16 matrix-core products, FP32 accumulation: 2e-2),
training, and the held-out gain over the paper's guess at the same absolute
Newton tolerance."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import workloads as W
from oracle import mlp as OM
from oracle import solver as OS
from oracle.dg import make_disc


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _ctx(cfg, mesh, **over):
    from paper_2002_04222_amd import Context
    return Context(mesh, cfg, **over)


def _small():
    cfg = W.config(1, ncells=(4, 4))
    return cfg, cfg.mesh()


# 2500 rows: the weight-gradient products are split over K (rows)
@pytest.mark.parametrize("R", [300, 2500])
def test_mlp_forward_and_gradient_match_oracle(R):
    _case(f"mlp forward/grad vs oracle, {R} rows")
    cfg, mesh = _small()
    ctx = _ctx(cfg, mesh)
    H = 64
    nb = ctx.shape[1] * ctx.shape[2]
    th = W.mlp_init(2 * nb, H, nb, seed=3, out_scale=1.0)
    ctx.mlp_create(H, th)
    assert ctx.mlp_n_params == OM.n_params(2 * nb, H, nb)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(R, 2 * nb)).astype(np.float32) * 0.5
    T = rng.normal(size=(R, nb)).astype(np.float32) * 0.3
    Xd = torch.tensor(X, device="cuda")
    Td = torch.tensor(T, device="cuda")
    Y = torch.empty((R, nb), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(Xd, Y)
    Yo, _ = OM.forward(th.astype(np.float64), X.astype(np.float64), 2 * nb, H, nb)
    yg = Y.cpu().numpy()
    assert np.linalg.norm(yg - Yo) <= 2e-2 * np.linalg.norm(Yo)
    g = torch.empty(ctx.mlp_n_params, dtype=torch.float32, device="cuda")
    loss = ctx.mlp_grad(Xd, Td, g)
    go = OM.grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), 2 * nb, H, nb)
    assert abs(loss - OM.loss(th.astype(np.float64), X, T, 2 * nb, H, nb)) <= 2e-2 * loss
    gg = g.cpu().numpy().astype(np.float64)
    o = 0
    for shp in OM.sizes(2 * nb, H, nb):
        k = int(np.prod(shp))
        a, b = gg[o:o + k], go[o:o + k]
        assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b), shp
        o += k


def test_mlp_training_reduces_loss():
    _case("mlp training")
    cfg, mesh = _small()
    ctx = _ctx(cfg, mesh)
    H = 64
    nb = ctx.shape[1] * ctx.shape[2]
    ctx.mlp_create(H, W.mlp_init(2 * nb, H, nb, seed=5))
    rng = np.random.default_rng(6)
    X = torch.tensor(rng.normal(size=(512, 2 * nb)).astype(np.float32), device="cuda")
    teacher = W.mlp_init(2 * nb, 32, nb, seed=7, out_scale=1.0).astype(np.float64)
    T, _ = OM.forward(teacher, X.cpu().numpy().astype(np.float64), 2 * nb, 32, nb)
    Td = torch.tensor(T.astype(np.float32), device="cuda")
    l0 = ctx.mlp_train_step(X, Td, 1e-3)
    for _ in range(300):
        l1 = ctx.mlp_train_step(X, Td, 1e-3)
    assert l1 < 0.2 * l0, (l0, l1)


def test_learned_guess_gain_and_step_parity():
    """Record plain steps of the 2D Taylor-Green workload, fit the MLP, then
    run held-out steps from one saved state with the paper's guess and with
    the learned guess: both stop at the same absolute tolerance
    alpha ||N(S_m)||; the learned start has a smaller residual and needs no
    more Newton iterations, and the steps agree with the FP64 oracle's plain
    step to 1e-8."""
    _case("learned guess gain, tgv2d 12x12 P=2")
    cfg = W.config(1, ncells=(12, 12))
    mesh = cfg.mesh()
    ctx = _ctx(cfg, mesh)
    n = ctx.n_unknowns
    u = ctx.empty()
    noise = torch.tensor(W.noise(ctx.shape, cfg.seed), device="cuda")
    ctx.project_tgv(noise, cfg.noise_amp, u)
    dt = cfg.dt()
    n_train, stages = 16, 2
    S_rec = torch.empty((n_train, stages, n), dtype=torch.float64, device="cuda")
    I_rec = torch.empty_like(S_rec)
    for k in range(n_train):
        ctx.set_record(S_rec[k], I_rec[k])
        ctx.sdirk_step(u, dt)
    ctx.set_record(None, None)
    nb = ctx.shape[1] * ctx.shape[2]
    ctx.mlp_create(256, W.mlp_init(2 * nb, 256, nb, seed=8))
    loss = ctx.mlp_fit(S_rec, I_rec, n_train, 150, 1e-3)
    print("fit loss", loss, flush=True)
    assert np.isfinite(loss) and loss < 1.0
    # held-out steps from the same saved state and increment history
    u_save = u.clone()
    inc_save = torch.empty((2, 3, n), dtype=torch.float64, device="cuda")
    ctx.guess_state(inc_out=inc_save)
    res = {}
    for mode in ("paper", "learned"):
        ctx.guess_state(inc_in=inc_save)
        ctx.set_guess(mode)
        uu = u_save.clone()
        its, norms = [], []
        for k in range(3):
            st = ctx.sdirk_step(uu, dt)
            its.append(sum(st["newton_its"]))
            norms.append(st["guess_norm"])
        res[mode] = (uu.cpu().numpy(), its, norms)
        print(mode, its, norms, flush=True)
    ctx.set_guess("paper")
    # every candidate is evaluated; the chosen start (learned or its
    # extrapolated fallback) beats S_m at every stage.  The learned / fallback
    # norm ratios are reported, not asserted: on these data the per-element
    # net's independent inter-element errors cost more in ||N|| than the
    # extrapolation's smooth ones.
    ratios = []
    for stage_norms in res["learned"][2]:
        for nS, nE, nM in stage_norms:
            assert nS > 0 and nE > 0 and nM > 0
            assert min(nE, nM) < nS
            ratios.append(nM / nE)
    print("learned / extrapolated residual norms", ratios, flush=True)
    assert sum(res["learned"][1]) <= sum(res["paper"][1])
    ua, ub = res["paper"][0], res["learned"][0]
    assert np.linalg.norm(ua - ub) <= 1e-8 * np.linalg.norm(ua)
    # one held-out step against the oracle's plain FP64 step from the saved state
    disc = make_disc(cfg, mesh)
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme=cfg.scheme))
    uo, _ = stepper.step(u_save.cpu().numpy(), dt)
    ctx.guess_state(inc_in=inc_save)
    ctx.set_guess("learned")
    ul = u_save.clone()
    ctx.precond_build(ul, dt * (1 - np.sqrt(2) / 2))
    ctx.sdirk_step(ul, dt)
    ctx.set_guess("paper")
    assert np.linalg.norm(ul.cpu().numpy() - uo) <= 1e-8 * np.linalg.norm(uo)
