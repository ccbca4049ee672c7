"""dgj_precond_apply_static (the BRJ apply whose iterates live in the
library's static device array, for callers that cannot allocate) against
dgj_precond_apply through the C ABI: bitwise equal on two calls in a row,
the second on a smaller context (a curved mesh, which also uses the mass
product buffer), and a context above the array's size refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W
from tests.gpu_util import setup


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _apply_both(ctx, q):
    a, b = ctx.empty(), ctx.empty()
    ctx.precond_apply(q, a)
    ctx.precond_apply_static(q, b)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_static_apply_matches_apply_on_two_calls():
    from paper_2002_04222_amd import Context
    _case("static apply: 3D box 3x3x3 P=3 (8640 unknowns)")
    cfg, mesh, _ = setup(3, (3, 3, 3), 3, Ma=0.3, Re=40.0)
    ctx = Context(mesh, cfg)
    u = _dev(W.random_state(mesh.n_elem, 3, 3, seed=501))
    ctx.precond_build(u, 0.1)
    q = _dev(W.random_vector(mesh.n_elem, 3, 3, seed=502))
    a, b = _apply_both(ctx, q)
    assert np.array_equal(a, b)
    ctx.close()
    _case("static apply: curved 2D annulus 2x6 P=2 (smaller, mass product)")
    import dataclasses
    cfg2 = dataclasses.replace(W.config(4), dim=2, ncells=(2, 6), lengths=(1.0, 2 * np.pi), P=2, nq=4, r1=3.0,
                               Re=200.0)
    mesh2 = cfg2.mesh()
    k, st = cfg2.boundary()
    ctx2 = Context(mesh2, cfg2, bc_kind=k, bc_state=st)
    u2 = _dev(W.freestream_state(dataclasses.replace(cfg2, noise_amp=1e-2), mesh2.n_elem))
    ctx2.precond_build(u2, 0.05)
    q2 = _dev(W.random_vector(mesh2.n_elem, 2, 2, seed=503))
    assert ctx2.n_unknowns < 8640
    a2, b2 = _apply_both(ctx2, q2)
    assert np.array_equal(a2, b2)
    ctx2.close()


def test_static_apply_refuses_contexts_above_its_size():
    from paper_2002_04222_amd import Context, DgjError
    _case("static apply: 3D box 16x16x14 P=4 (2.24M unknowns) refused")
    cfg, mesh, _ = setup(3, (16, 16, 14), 4, Ma=0.3, Re=40.0)
    ctx = Context(mesh, cfg)
    assert ctx.n_unknowns > 1 << 21
    q, o = ctx.empty(), ctx.empty()
    with pytest.raises(DgjError) as e:
        ctx.precond_apply_static(q, o)
    assert "exceed the static scratch" in str(e.value)
    ctx.close()
