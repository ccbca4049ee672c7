"""The learned Newton guess on the GPU: MLP forward and gradients (the
regression loss and the pooled blend loss) against the FP64 oracle (BF16
matrix-core products, FP32 accumulation: 2e-2), the features, training, and
the held-out gain over the paper's and the extrapolated guesses at the same
absolute Newton tolerance."""
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
    no = 2
    th = W.mlp_init(2 * nb, H, no, seed=3, out_scale=1.0)
    ctx.mlp_create(H, th)
    assert ctx.mlp_n_params == OM.n_params(2 * nb, H, no) and ctx.mlp_n_out == no
    rng = np.random.default_rng(4)
    X = rng.normal(size=(R, 2 * nb)).astype(np.float32) * 0.5
    T = rng.normal(size=(R, no)).astype(np.float32) * 0.3
    Xd = torch.tensor(X, device="cuda")
    Td = torch.tensor(T, device="cuda")
    Y = torch.empty((R, no), dtype=torch.float32, device="cuda")
    ctx.mlp_forward(Xd, Y)
    Yo, _ = OM.forward(th.astype(np.float64), X.astype(np.float64), 2 * nb, H, no)
    yg = Y.cpu().numpy()
    assert np.linalg.norm(yg - Yo) <= 2e-2 * np.linalg.norm(Yo)
    g = torch.empty(ctx.mlp_n_params, dtype=torch.float32, device="cuda")
    loss = ctx.mlp_grad(Xd, Td, g)
    go = OM.grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), 2 * nb, H, no)
    assert abs(loss - OM.loss(th.astype(np.float64), X, T, 2 * nb, H, no)) <= 2e-2 * loss
    gg = g.cpu().numpy().astype(np.float64)
    o = 0
    for shp in OM.sizes(2 * nb, H, no):
        k = int(np.prod(shp))
        a, b = gg[o:o + k], go[o:o + k]
        assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b), shp
        o += k


@pytest.mark.parametrize("E", [16, 2500])
def test_features_pool_and_pooled_gradient_match_oracle(E):
    """Features from three increment fields, the pooled blend (mean of the
    outputs over the elements, FP64 sums) and the parameter gradient of a
    loss of the blend (every row's output gradient dL/dc / E) against the
    oracle; 2500 elements take the split-K weight-gradient products."""
    _case(f"mlp features / pool / pooled gradient vs oracle, {E} elements")
    cfg = W.config(1, ncells=(E // 4 if E > 16 else 4, 4))
    mesh = cfg.mesh()
    ctx = _ctx(cfg, mesh)
    assert ctx.shape[0] == E
    H = 64
    nb = ctx.shape[1] * ctx.shape[2]
    th = W.mlp_init(2 * nb, H, 2, seed=9, out_scale=1.0)
    ctx.mlp_create(H, th)
    rng = np.random.default_rng(10)
    inc = [rng.normal(size=ctx.shape) * (1.0 + v) for v in range(3)]
    inc[1][:, 2, :] = inc[0][:, 2, :]          # a variable whose first difference is zero
    dev = [torch.tensor(x, device="cuda") for x in inc]
    X = torch.empty((E, 2 * nb), dtype=torch.float32, device="cuda")
    ctx.mlp_features(dev[0], dev[1], dev[2], X)
    Xo, so = OM.features(*inc)
    assert so[2] == 1.0
    assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6 * np.abs(Xo).max()
    c = ctx.mlp_pool(X)
    co = OM.pooled(th.astype(np.float64), X.cpu().numpy().astype(np.float64), 2 * nb, H, 2)
    assert np.linalg.norm(c - co) <= 2e-2 * np.linalg.norm(co)
    dLdc = np.array([0.7, -1.3])
    g = torch.empty(ctx.mlp_n_params, dtype=torch.float32, device="cuda")
    ctx.mlp_pool_backward(dLdc, g)
    go = OM.backprop(th.astype(np.float64), X.cpu().numpy().astype(np.float64), np.tile(dLdc / E, (E, 1)),
                     2 * nb, H, 2)
    gg = g.cpu().numpy().astype(np.float64)
    o = 0
    for shp in OM.sizes(2 * nb, H, 2):
        k = int(np.prod(shp))
        assert np.linalg.norm(gg[o:o + k] - go[o:o + k]) <= 3e-2 * np.linalg.norm(go[o:o + k]), shp
        o += k


def test_mlp_training_reduces_loss():
    _case("mlp training")
    cfg, mesh = _small()
    ctx = _ctx(cfg, mesh)
    H = 64
    nb = ctx.shape[1] * ctx.shape[2]
    ctx.mlp_create(H, W.mlp_init(2 * nb, H, 2, seed=5))
    rng = np.random.default_rng(6)
    X = torch.tensor(rng.normal(size=(512, 2 * nb)).astype(np.float32), device="cuda")
    teacher = W.mlp_init(2 * nb, 32, 2, seed=7, out_scale=1.0).astype(np.float64)
    T, _ = OM.forward(teacher, X.cpu().numpy().astype(np.float64), 2 * nb, 32, 2)
    Td = torch.tensor(T.astype(np.float32), device="cuda")
    l0 = ctx.mlp_train_step(X, Td, 1e-3)
    for _ in range(300):
        l1 = ctx.mlp_train_step(X, Td, 1e-3)
    assert l1 < 0.2 * l0, (l0, l1)


def test_learned_guess_gain_and_step_parity():
    """Record 24 plain steps of the 2D Taylor-Green workload on a 12 x 12
    mesh, fit the MLP on them, then run 6 held-out steps from one saved
    state and increment history with the paper's guess S_m, the
    extrapolated guess and the learned one, all stopping at the same
    absolute tolerance alpha ||N(S_m)||.  At every held-out stage the
    learned candidate's ||N|| is below the extrapolated one's, which is
    below ||N(S_m)||; the learned runs need no more Newton iterations than
    either; the fit's loss is below the zero network's (1: the extrapolated
    guess itself); the states agree with each other and one held-out step
    with the FP64 oracle's plain step to 1e-8."""
    _case("learned guess gain, tgv2d 12x12 P=2")
    cfg = W.config(1, ncells=(12, 12))
    mesh = cfg.mesh()
    ctx = _ctx(cfg, mesh)
    n = ctx.n_unknowns
    u = ctx.empty()
    noise = torch.tensor(W.noise(ctx.shape, cfg.seed), device="cuda")
    ctx.project_tgv(noise, cfg.noise_amp, u)
    dt = cfg.dt()
    n_train, stages, held = 24, 2, 6
    S_rec = torch.empty((n_train, stages, n), dtype=torch.float64, device="cuda")
    I_rec = torch.empty_like(S_rec)
    for k in range(n_train):
        ctx.set_record(S_rec[k], I_rec[k])
        ctx.sdirk_step(u, dt)
    ctx.set_record(None, None)
    nb = ctx.shape[1] * ctx.shape[2]
    ctx.mlp_create(64, W.mlp_init(2 * nb, 64, 2, seed=8))
    loss = ctx.mlp_fit(S_rec, I_rec, n_train, 200, 1e-3)
    print("fit loss", loss, flush=True)
    assert np.isfinite(loss) and loss < 0.9
    u_save = u.clone()
    inc_save = torch.empty((3, stages, n), dtype=torch.float64, device="cuda")
    ctx.guess_state(inc_out=inc_save)
    res = {}
    for mode in ("paper", "extrapolated", "learned"):
        ctx.guess_state(inc_in=inc_save)
        ctx.set_guess(mode)
        uu = u_save.clone()
        its, norms, blend = [], [], []
        for k in range(held):
            st = ctx.sdirk_step(uu, dt)
            its.append(sum(st["newton_its"]))
            norms.append(st["guess_norm"])
            blend.append(st["guess_blend"])
        res[mode] = (uu.cpu().numpy(), its, norms, blend)
        print(mode, "newton", its, flush=True)
    ctx.set_guess("paper")
    ratios = []
    for stage_norms, stage_blend in zip(res["learned"][2], res["learned"][3]):
        for (nS, nE, nM), c in zip(stage_norms, stage_blend):
            print(f"  ||N||: S_m {nS:.3e} extrapolated {nE:.3e} learned {nM:.3e}  blend {c}", flush=True)
            assert 0.0 < nM < nE < nS
            ratios.append(nM / nE)
    print("learned / extrapolated ||N||:", ["%.3f" % r for r in ratios], flush=True)
    assert sum(res["learned"][1]) <= sum(res["paper"][1])
    assert sum(res["learned"][1]) <= sum(res["extrapolated"][1])
    ua = res["paper"][0]
    for mode in ("extrapolated", "learned"):
        assert np.linalg.norm(res[mode][0] - ua) <= 1e-8 * np.linalg.norm(ua), mode
    # one held-out step against the oracle's plain FP64 step from the saved state
    disc = make_disc(cfg, mesh)
    stepper = OS.SDIRK(disc, OS.SolverOpts(scheme=cfg.scheme))
    uo, _ = stepper.step(u_save.cpu().numpy(), dt)
    ctx.guess_state(inc_in=inc_save)
    ctx.set_guess("learned")
    ul = u_save.clone()
    ctx.precond_build(ul, dt * (1 - np.sqrt(2) / 2))
    st = ctx.sdirk_step(ul, dt)
    ctx.set_guess("paper")
    assert st["guess_used"] == [2, 2]
    assert np.linalg.norm(ul.cpu().numpy() - uo) <= 1e-8 * np.linalg.norm(uo)
