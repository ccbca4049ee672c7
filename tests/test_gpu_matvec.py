"""The Jacobian-free matvec of the library (Eq. 25) is exactly the forward
difference of its own stage residual (Eq. 20): Jv = (N(w) - N_u) / eps with
w = u + eps v rounded as a product and then a sum.  The device forms w in a
pass of its own and evaluates N inside the residual kernels; the test forms
w and the difference with torch from the library's stage residual at w and
requires bitwise equality, on affine and curved meshes, through the fused
kernel and the three-kernel path, and at a second eps (the buffer is
reused).  Oracle parity of the matvec is in test_gpu_parity.py; batches, whose
matvecs take per-instance eps, are equal bitwise to solo runs in
test_gpu_batch.py."""
import dataclasses
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W


def _case(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _mesh(kind, dim, P):
    if kind == "box":
        base = W.config(1 if dim == 2 else 2)
        cells = (3, 2) if dim == 2 else (2, 2, 3)
        lengths = tuple(1.0 + 0.3 * i for i in range(dim))
        cfg = dataclasses.replace(base, dim=dim, ncells=cells, lengths=lengths, P=P, nq=P + 2, Ma=0.3, Re=40.0)
        return cfg, W.cartesian_mesh(cells, lengths), None, None
    if kind == "curved":
        base = W.config(1 if dim == 2 else 2)
        cells = (3, 2) if dim == 2 else (2, 2, 2)
        lengths = tuple(1.0 + 0.3 * i for i in range(dim))
        cfg = dataclasses.replace(base, dim=dim, ncells=cells, lengths=lengths, P=P, nq=P + 2, Ma=0.3, Re=40.0)
        return cfg, W.curved_box_mesh(cells, lengths, geo_order=2, amp=0.15, seed=17), None, None
    base = W.config(4)
    cfg = dataclasses.replace(base, dim=dim, ncells=(2, 8) + ((2,) if dim == 3 else ()),
                              lengths=(1.0, 2 * np.pi) + ((1.0,) if dim == 3 else ()), P=P, nq=P + 2,
                              r1=3.0, Re=200.0)
    mesh = cfg.mesh()
    kinds, states = cfg.boundary()
    return cfg, mesh, kinds, states


CASES = [("box", 2, 3, True), ("box", 3, 2, True), ("box", 3, 2, False), ("curved", 2, 2, True),
         ("curved", 3, 3, True), ("curved", 3, 2, False), ("annulus", 3, 4, True)]


@pytest.mark.parametrize("kind,dim,P,fused", CASES)
def test_matvec_is_the_difference_of_stage_residuals(kind, dim, P, fused):
    _case(f"matvec vs stage residuals: {kind} dim={dim} P={P} fused={fused}")
    from paper_2002_04222_amd import Context
    cfg, mesh, kinds, states = _mesh(kind, dim, P)
    ctx = Context(mesh, cfg, bc_kind=kinds, bc_state=states) if kinds is not None else Context(mesh, cfg)
    ctx.set_residual_kernels(fused)
    if kind == "annulus":
        u = _dev(W.freestream_state(cfg, mesh.n_elem)).reshape(ctx.shape)
        u = u * (1.0 + 1e-3 * _dev(W.random_vector(mesh.n_elem, dim, P, seed=3)).reshape(ctx.shape))
    else:
        u = _dev(W.random_state(mesh.n_elem, dim, P, seed=21)).reshape(ctx.shape)
    S = 0.999 * u
    v = _dev(W.random_vector(mesh.n_elem, dim, P, seed=22)).reshape(ctx.shape)
    dt_a = 0.05
    Nu = ctx.empty()
    ctx.stage_residual(u, S, dt_a, Nu)
    for eps in (1.3e-7, 4.1e-9):
        Jv = ctx.empty()
        ctx.jfnk_matvec(u, Nu, S, dt_a, v, eps, Jv)
        w = u + (eps * v)          # the product, then the sum, each rounded
        Nw = ctx.empty()
        ctx.stage_residual(w, S, dt_a, Nw)
        # elementwise IEEE division (torch turns division by a Python scalar
        # into a product with its reciprocal)
        ref = (Nw - Nu) / torch.full_like(Nw, eps)
        torch.cuda.synchronize()
        assert torch.equal(Jv, ref), float((Jv - ref).abs().max())

