"""Why the learned guess blends globally (the reading behind its design,
checked on the oracle): on recorded stages of the 2D Taylor-Green workload
the stage residual ||N|| of a corrected extrapolated guess depends far more
on how uniform the correction is than on how well it fits the converged
state.  The least-squares blend of the increments' first and second
differences fitted per element fits the state better than one blend for
all elements, yet its ||N|| is many times larger, also than the
extrapolated guess's (here, early in the run, the global least-squares blend
itself is not yet better than extrapolation: the state-space fit is not
the residual's, which is why the learned blend is judged by ||N|| and kept
only when it wins)."""
import numpy as np

import workloads as W
from oracle import solver as OS
from oracle.dg import initial_state, make_disc


def test_per_element_blend_fits_better_but_raises_the_stage_residual():
    cfg = W.config(1)
    mesh = cfg.mesh()
    disc = make_disc(cfg, mesh)
    u = initial_state(disc, W.noise(disc.shape, cfg.seed), cfg.noise_amp)
    dt = cfg.dt()
    st = OS.SDIRK(disc, OS.SolverOpts(scheme=cfg.scheme))
    A = st.A
    dta = dt * A[0, 0]
    rec = []
    for _ in range(10):
        st.ensure_pc(u, dta)
        Es, stages = [], []
        for m in range(A.shape[0]):
            S = u + sum(A[m, i] * Es[i] for i in range(m))
            um, _ = st.solve_stage(S, dt * A[m, m])
            Es.append((um - S) / A[m, m])
            stages.append((S, um))
        st.pc_age += 1
        u = u + sum(st.b[i] * Es[i] for i in range(len(Es)))
        rec.append(stages)
    n, m = 9, 0
    inc = [rec[k][m][1] - rec[k][m][0] for k in range(n + 1)]
    S, uh = rec[n][m]
    i1, i2, i3 = inc[n - 1], inc[n - 2], inc[n - 3]
    gE = S + 2 * i1 - i2
    r = uh - gE                                   # the extrapolated guess's error
    F = [i1 - i2, i1 - 2 * i2 + i3]               # the blend directions

    def blend_fit(axes):
        """least-squares (c0, c1) over the given axes, broadcast back"""
        G = np.array([[np.sum(a * b, axis=axes, keepdims=True) for b in F] for a in F])
        h = np.array([np.sum(a * r, axis=axes, keepdims=True) for a in F])
        Gm = np.moveaxis(G, (0, 1), (-2, -1))
        hm = np.moveaxis(h, 0, -1)
        c = np.linalg.solve(Gm, hm[..., None])[..., 0]
        return F[0] * c[..., 0] + F[1] * c[..., 1]

    glob = blend_fit((0, 1, 2))
    elem = blend_fit((1, 2))
    res = lambda g: np.linalg.norm(disc.stage_residual(g, S, dta))
    nE, nG, nP = res(gE), res(gE + glob), res(gE + elem)
    fit_glob, fit_elem = np.linalg.norm(glob - r), np.linalg.norm(elem - r)
    print(f"||N||: extrapolated {nE:.3e}, global blend {nG:.3e}, per-element blend {nP:.3e}; "
          f"state error: global {fit_glob:.3e}, per-element {fit_elem:.3e}")
    assert fit_elem < fit_glob                    # the per-element blend fits the state better
    assert nP > 5.0 * max(nG, nE)                 # but the per-element one costs in ||N||
