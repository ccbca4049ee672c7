"""ctypes binding of the dgj C ABI (include/dgj.h).  Argument marshalling
only: device arrays are torch tensors on the context's device, passed by
data pointer."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libdgj.so")

DGJ_OK = 0
DGJ_BEULER, DGJ_SDIRK2, DGJ_SDIRK3, DGJ_SDIRK4, DGJ_BDF2, DGJ_ERK2 = 1, 2, 3, 4, 12, 20
MAX_STAGES = 6
DGJ_PC_F64, DGJ_PC_F32, DGJ_PC_BF16 = 0, 1, 2
(DGJ_BC_FARFIELD, DGJ_BC_WALL, DGJ_BC_DIRICHLET, DGJ_BC_SLIP, DGJ_BC_ISOTHERMAL, DGJ_BC_EXTRAPOLATE,
 DGJ_BC_PRESSURE_OUT, DGJ_BC_PRESSURE_IN) = range(8)
STATUS = {0: "OK", -1: "EINVAL", -2: "EHIP", -3: "ENOMEM", -4: "ENOTCONV", -5: "ENAN", -6: "ESINGULAR",
          -7: "EUNSUPPORTED"}


class DgjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dgj status {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("P", C.c_int32), ("nq", C.c_int32), ("n_elem", C.c_int64),
                ("elem_origin", C.POINTER(C.c_double)), ("elem_h", C.POINTER(C.c_double)),
                ("face_nbr", C.POINTER(C.c_int32)), ("n_bc", C.c_int32), ("bc_kind", C.POINTER(C.c_int32)),
                ("bc_state", C.POINTER(C.c_double)), ("geo_order", C.c_int32), ("geo_nodes", C.POINTER(C.c_double))]


class Phys(C.Structure):
    _fields_ = [("gamma", C.c_double), ("Pr", C.c_double), ("Re", C.c_double), ("Ma", C.c_double),
                ("T_ref_K", C.c_double), ("visc_law", C.c_int32), ("flux_mode", C.c_int32),
                ("riemann", C.c_int32), ("viscous", C.c_int32)]


class Solver(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("newton_rtol", C.c_double), ("newton_max", C.c_int32),
                ("gmres_restart", C.c_int32), ("gmres_rtol", C.c_double), ("gmres_max", C.c_int32),
                ("brj_sweeps", C.c_int32), ("brj_omega", C.c_double), ("pc_precision", C.c_int32),
                ("pc_freeze", C.c_int32), ("pc_refresh_its", C.c_int32), ("ortho", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("stages", C.c_int32), ("newton_its", C.c_int32 * MAX_STAGES),
                ("gmres_its", (C.c_int32 * 64) * MAX_STAGES), ("nres", (C.c_double * 65) * MAX_STAGES),
                ("pc_built", C.c_int32), ("residual_evals", C.c_int32), ("status", C.c_int32),
                ("t_total_ms", C.c_double), ("t_pc_build_ms", C.c_double), ("guess_used", C.c_int32 * MAX_STAGES),
                ("guess_norm", (C.c_double * 3) * MAX_STAGES), ("guess_blend", (C.c_double * 2) * MAX_STAGES)]

    def to_dict(self):
        s = self.stages
        return {
            "stages": s,
            "newton_its": [self.newton_its[m] for m in range(s)],
            "gmres_its": [[self.gmres_its[m][i] for i in range(self.newton_its[m])] for m in range(s)],
            "nres": [[self.nres[m][i] for i in range(self.newton_its[m] + 1)] for m in range(s)],
            "pc_built": self.pc_built, "residual_evals": self.residual_evals, "status": self.status,
            "t_total_ms": self.t_total_ms, "t_pc_build_ms": self.t_pc_build_ms,
            "guess_used": [self.guess_used[m] for m in range(s)],
            "guess_norm": [[self.guess_norm[m][k] for k in range(3)] for m in range(s)],
            "guess_blend": [[self.guess_blend[m][k] for k in range(2)] for m in range(s)],
        }


_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"dgj HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    vp, dp, i64p, i32p = C.c_void_p, C.c_double, C.POINTER(C.c_int64), C.POINTER(C.c_int32)
    sig = {
        "dgj_create": ([C.POINTER(Mesh), C.POINTER(Phys), C.POINTER(Solver), vp, C.POINTER(vp)], C.c_int),
        "dgj_destroy": ([vp], None),
        "dgj_sizes": ([vp, i64p], C.c_int),
        "dgj_last_error": ([vp], C.c_char_p),
        "dgj_project_tgv": ([vp, vp, dp, vp], C.c_int),
        "dgj_residual": ([vp, vp, vp], C.c_int),
        "dgj_mass_inverse": ([vp, vp], C.c_int),
        "dgj_autotune": ([vp, vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)], C.c_int),
        "dgj_stage_residual": ([vp, vp, vp, dp, vp], C.c_int),
        "dgj_jfnk_matvec": ([vp, vp, vp, vp, dp, vp, dp, vp], C.c_int),
        "dgj_precond_build": ([vp, vp, dp], C.c_int),
        "dgj_precond_apply": ([vp, vp, vp], C.c_int),
        "dgj_precond_diag_inverse": ([vp, vp], C.c_int),
        "dgj_gmres": ([vp, vp, vp, vp, dp, dp, vp, vp, i32p], C.c_int),
        "dgj_newton": ([vp, vp, dp, vp, i32p, i32p], C.c_int),
        "dgj_sdirk_step": ([vp, vp, dp, C.POINTER(StepStats)], C.c_int),
        "dgj_set_guess": ([vp, C.c_int32], C.c_int),
        "dgj_set_pc_precision": ([vp, C.c_int32], C.c_int),
        "dgj_set_residual_kernels": ([vp, C.c_int32], C.c_int),
        "dgj_precond_apply_static": ([vp, vp, vp], C.c_int),
        "dgj_project": ([vp, vp, vp], C.c_int),
        "dgj_set_source": ([vp, vp], C.c_int),
        "dgj_set_bc_field": ([vp, vp], C.c_int),
        "dgj_reset_history": ([vp], C.c_int),
        "dgj_set_record": ([vp, vp, vp], C.c_int),
        "dgj_mlp_create": ([vp, C.c_int32, vp], C.c_int),
        "dgj_mlp_sizes": ([vp, i64p, i32p, i32p], C.c_int),
        "dgj_mlp_get_params": ([vp, vp], C.c_int),
        "dgj_mlp_set_params": ([vp, vp], C.c_int),
        "dgj_mlp_fit": ([vp, vp, vp, C.c_int32, C.c_int32, dp, C.POINTER(C.c_double)], C.c_int),
        "dgj_guess_state": ([vp, vp, vp], C.c_int),
        "dgj_mlp_features": ([vp, vp, vp, vp, vp], C.c_int),
        "dgj_mlp_pool": ([vp, vp, C.c_int64, vp], C.c_int),
        "dgj_mlp_pool_backward": ([vp, vp, vp], C.c_int),
        "dgj_mlp_forward": ([vp, vp, C.c_int64, vp], C.c_int),
        "dgj_mlp_grad": ([vp, vp, vp, C.c_int64, vp, C.POINTER(C.c_double)], C.c_int),
        "dgj_mlp_train_step": ([vp, vp, vp, C.c_int64, dp, C.POINTER(C.c_double)], C.c_int),
        "dgj_batch_create": ([C.c_int32, C.POINTER(Mesh), C.POINTER(Phys), C.POINTER(Solver), vp, C.POINTER(vp)],
                             C.c_int),
        "dgj_create_batch": ([C.c_int32, C.POINTER(Mesh), C.POINTER(Phys), C.POINTER(Solver), vp, C.POINTER(vp)],
                             C.c_int),
        "dgj_batch_destroy": ([vp], None),
        "dgj_batch_set_graphs": ([vp, C.c_int32], C.c_int),
        "dgj_batch_autotune": ([vp, vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
        "dgj_batch_last_error": ([vp], C.c_char_p),
        "dgj_batch_sizes": ([vp, i64p, i64p, i64p], C.c_int),
        "dgj_batch_project_tgv": ([vp, vp, dp, vp], C.c_int),
        "dgj_batch_residual": ([vp, vp, vp], C.c_int),
        "dgj_batch_sdirk_step": ([vp, vp, vp, i32p, i32p], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t, dtype: str = "torch.float64") -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or repr(t.dtype) != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor")
    return t.data_ptr()


def _fptr(t) -> Optional[int]:
    return _ptr(t, "torch.float32")


SCHEMES = {"beuler": DGJ_BEULER, "sdirk2": DGJ_SDIRK2, "sdirk3": DGJ_SDIRK3, "sdirk4": DGJ_SDIRK4,
           "bdf2": DGJ_BDF2, "erk2": DGJ_ERK2}
PRECISIONS = {"f64": DGJ_PC_F64, "f32": DGJ_PC_F32, "bf16": DGJ_PC_BF16}
VISCOUS = {"ip": 0, "ldg": 1}
ORTHO = {"mgs": 0, "cgs2": 1}


def _mesh_struct(mesh, cfg, keep, bc_kind=None, bc_state=None):
    """dgj_mesh over host copies held in keep; bc_kind[n_bc] and
    bc_state[n_bc][dim+2] describe the boundary ids of face_nbr < 0."""
    dp = C.POINTER(C.c_double)
    nbr = np.ascontiguousarray(mesh.face_nbr, dtype=np.int32)
    keep.append(nbr)
    m = Mesh(mesh.dim, cfg.P, cfg.nq, mesh.n_elem, dp(), dp(), nbr.ctypes.data_as(C.POINTER(C.c_int32)))
    if mesh.elem_h is not None:
        org = np.ascontiguousarray(mesh.elem_origin, dtype=np.float64)
        h = np.ascontiguousarray(mesh.elem_h, dtype=np.float64)
        keep.extend([org, h])
        m.elem_origin, m.elem_h = org.ctypes.data_as(dp), h.ctypes.data_as(dp)
    if getattr(mesh, "geo_nodes", None) is not None:
        nodes = np.ascontiguousarray(mesh.geo_nodes, dtype=np.float64)
        keep.append(nodes)
        m.geo_order = mesh.geo_order
        m.geo_nodes = nodes.ctypes.data_as(dp)
    if bc_kind is not None:
        kind = np.ascontiguousarray(bc_kind, dtype=np.int32).ravel()
        state = np.ascontiguousarray(bc_state, dtype=np.float64).reshape(len(kind), mesh.dim + 2)
        keep.extend([kind, state])
        m.n_bc = len(kind)
        m.bc_kind = kind.ctypes.data_as(C.POINTER(C.c_int32))
        m.bc_state = state.ctypes.data_as(C.POINTER(C.c_double))
    return m


def _phys_struct(cfg):
    return Phys(cfg.gamma, cfg.Pr, cfg.Re, cfg.Ma, cfg.T_ref_K, cfg.visc_law, cfg.flux_mode, cfg.riemann,
                VISCOUS[getattr(cfg, "viscous", "ip")])


def _solver_struct(cfg):
    return Solver(SCHEMES[cfg.scheme], cfg.newton_rtol, cfg.newton_max, cfg.gmres_restart, cfg.gmres_rtol,
                  cfg.gmres_max, cfg.brj_sweeps, cfg.brj_omega, PRECISIONS[cfg.pc_precision], cfg.pc_freeze,
                  cfg.pc_refresh_its, ORTHO[getattr(cfg, "ortho", "mgs")])


class Batch:
    """A batch of independent instances (see include/dgj.h, dgj_batch_*).
    cfgs: per-instance configurations (mesh size, P, gas parameters); the
    solver settings are the first one's."""

    def __init__(self, cfgs, stream=None):
        import torch
        self.lib = load_library()
        self._keep = []
        meshes = [c.mesh() for c in cfgs]
        n = len(cfgs)
        ms = (Mesh * n)(*[_mesh_struct(m, c, self._keep) for m, c in zip(meshes, cfgs)])
        ps = (Phys * n)(*[_phys_struct(c) for c in cfgs])
        sv = _solver_struct(cfgs[0])
        if stream is None:
            stream = torch.cuda.current_stream()
        h = C.c_void_p()
        rc = self.lib.dgj_batch_create(n, ms, ps, C.byref(sv), C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != DGJ_OK:
            raise DgjError(rc, "dgj_batch_create failed")
        self.h = h
        self.n = n
        tot = C.c_int64()
        off = (C.c_int64 * n)()
        cnt = (C.c_int64 * n)()
        self._check(self.lib.dgj_batch_sizes(self.h, C.byref(tot), off, cnt))
        self.n_total = tot.value
        self.offsets = [off[i] for i in range(n)]
        self.counts = [cnt[i] for i in range(n)]

    def _check(self, rc):
        if rc != DGJ_OK:
            raise DgjError(rc, self.lib.dgj_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dgj_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        import torch
        return torch.empty(self.n_total, dtype=torch.float64, device="cuda")

    def set_graphs(self, on):
        self._check(self.lib.dgj_batch_set_graphs(self.h, 1 if on else 0))

    def project_tgv(self, noise, amp, u):
        self._check(self.lib.dgj_batch_project_tgv(self.h, _ptr(noise), float(amp), _ptr(u)))

    def residual(self, u, R):
        self._check(self.lib.dgj_batch_residual(self.h, _ptr(u), _ptr(R)))

    def autotune(self, u, reps=20):
        """Residual workgroup sizes per order group; returns [[volume, face, lift], ...]."""
        ch = (C.c_int32 * (3 * self.n))()
        ng = C.c_int32()
        self._check(self.lib.dgj_batch_autotune(self.h, _ptr(u), int(reps), ch, C.byref(ng)))
        return [[ch[3 * g + k] for k in range(3)] for g in range(ng.value)]

    def sdirk_step(self, u, dt):
        dts = np.ascontiguousarray(dt, dtype=np.float64)
        nit = (C.c_int32 * (4 * self.n))()
        git = (C.c_int32 * (4 * self.n))()
        self._check(self.lib.dgj_batch_sdirk_step(self.h, _ptr(u), dts.ctypes.data, nit, git))
        return [[nit[4 * i + k] for k in range(4)] for i in range(self.n)], \
               [[git[4 * i + k] for k in range(4)] for i in range(self.n)]


class Context:
    """A dgj context for one mesh and set of options (see include/dgj.h)."""

    def __init__(self, mesh, cfg, stream=None, bc_kind=None, bc_state=None, **over):
        import torch
        self.lib = load_library()
        self.dim, self.P, self.nq = mesh.dim, cfg.P, cfg.nq
        self.n_elem = mesh.n_elem
        self._keep = []
        m = _mesh_struct(mesh, cfg, self._keep, bc_kind, bc_state)
        g = lambda k: over.get(k, getattr(cfg, k))
        ph = Phys(g("gamma"), g("Pr"), g("Re"), g("Ma"), g("T_ref_K"), g("visc_law"), g("flux_mode"), g("riemann"),
                  VISCOUS[over.get("viscous", getattr(cfg, "viscous", "ip"))])
        sv = Solver(SCHEMES[g("scheme")], g("newton_rtol"), g("newton_max"), g("gmres_restart"), g("gmres_rtol"),
                    g("gmres_max"), g("brj_sweeps"), g("brj_omega"), PRECISIONS[g("pc_precision")], g("pc_freeze"),
                    g("pc_refresh_its"), ORTHO[over.get("ortho", getattr(cfg, "ortho", "mgs"))])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = self.lib.dgj_create(C.byref(m), C.byref(ph), C.byref(sv), C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != DGJ_OK:
            raise DgjError(rc, "dgj_create failed")
        self.h = h
        n = C.c_int64()
        self._check(self.lib.dgj_sizes(self.h, C.byref(n)))
        self.n_unknowns = n.value
        self.shape = (mesh.n_elem, mesh.dim + 2, (cfg.P + 1) ** mesh.dim)

    def _check(self, rc):
        if rc != DGJ_OK:
            raise DgjError(rc, self.lib.dgj_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dgj_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        import torch
        return torch.empty(self.shape, dtype=torch.float64, device="cuda")

    def project_tgv(self, noise, amp, u):
        self._check(self.lib.dgj_project_tgv(self.h, _ptr(noise), float(amp), _ptr(u)))

    def residual(self, u, R):
        self._check(self.lib.dgj_residual(self.h, _ptr(u), _ptr(R)))

    def autotune(self, u, reps=20):
        """Workgroup sizes of the residual kernels chosen by timing; returns
        (chosen [volume, face, lift], times_ms [kernel][64, 128, 256])."""
        ch = (C.c_int32 * 3)()
        tm = (C.c_double * 9)()
        self._check(self.lib.dgj_autotune(self.h, _ptr(u), int(reps), ch, tm))
        return list(ch), [[tm[3 * k + i] for i in range(3)] for k in range(3)]

    def stage_residual(self, u, S, dt_a, N):
        self._check(self.lib.dgj_stage_residual(self.h, _ptr(u), _ptr(S), float(dt_a), _ptr(N)))

    def jfnk_matvec(self, u, N_u, S, dt_a, v, eps, Jv):
        self._check(self.lib.dgj_jfnk_matvec(self.h, _ptr(u), _ptr(N_u), _ptr(S), float(dt_a), _ptr(v),
                                             float(eps), _ptr(Jv)))

    def precond_build(self, u_p, dt_a):
        self._check(self.lib.dgj_precond_build(self.h, _ptr(u_p), float(dt_a)))

    def precond_apply(self, q, out):
        self._check(self.lib.dgj_precond_apply(self.h, _ptr(q), _ptr(out)))

    def mass_inverse(self, out):
        self._check(self.lib.dgj_mass_inverse(self.h, _ptr(out)))

    def precond_diag_inverse(self, out):
        self._check(self.lib.dgj_precond_diag_inverse(self.h, _ptr(out)))

    def gmres(self, u, N_u, S, dt_a, eps, b, x):
        it = C.c_int32()
        self._check(self.lib.dgj_gmres(self.h, _ptr(u), _ptr(N_u), _ptr(S), float(dt_a), float(eps), _ptr(b),
                                       _ptr(x), C.byref(it)))
        return it.value

    def newton(self, S, dt_a, u, newton_max=64):
        nit = C.c_int32()
        git = (C.c_int32 * max(64, newton_max))()
        self._check(self.lib.dgj_newton(self.h, _ptr(S), float(dt_a), _ptr(u), C.byref(nit), git))
        return nit.value, [git[i] for i in range(nit.value)]

    def sdirk_step(self, u, dt):
        st = StepStats()
        rc = self.lib.dgj_sdirk_step(self.h, _ptr(u), float(dt), C.byref(st))
        if rc != DGJ_OK:
            raise DgjError(rc, self.lib.dgj_last_error(self.h).decode())
        return st.to_dict()

    def project(self, f, u):
        """u = L2 projection of the values f[e][v][q] at the volume points."""
        self._check(self.lib.dgj_project(self.h, _ptr(f), _ptr(u)))

    def set_source(self, s):
        """Add s (modal, copied) to M^-1 L in every residual; None removes it."""
        self._check(self.lib.dgj_set_source(self.h, _ptr(s)))

    def set_bc_field(self, g):
        """Dirichlet ghost states g[e][f][v][p] at the face points (copied)."""
        self._check(self.lib.dgj_set_bc_field(self.h, _ptr(g)))

    def reset_history(self):
        self._check(self.lib.dgj_reset_history(self.h))

    # ---- Newton initial guess and the learned predictor
    GUESS = {"paper": 0, "extrapolated": 1, "learned": 2}

    def precond_apply_static(self, q, out):
        self._check(self.lib.dgj_precond_apply_static(self.h, _ptr(q), _ptr(out)))

    def set_residual_kernels(self, fused):
        self._check(self.lib.dgj_set_residual_kernels(self.h, 1 if fused else 0))

    def set_pc_precision(self, prec):
        self._check(self.lib.dgj_set_pc_precision(self.h, PRECISIONS[prec] if isinstance(prec, str) else int(prec)))

    def set_guess(self, mode):
        self._check(self.lib.dgj_set_guess(self.h, self.GUESS[mode] if isinstance(mode, str) else int(mode)))

    def set_record(self, S_rec, inc_rec):
        self._check(self.lib.dgj_set_record(self.h, _ptr(S_rec), _ptr(inc_rec)))

    def mlp_create(self, hidden, params=None):
        arr = None
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.dgj_mlp_create(self.h, int(hidden), arr.ctypes.data if arr is not None else None))
        npar, nin, nout = C.c_int64(), C.c_int32(), C.c_int32()
        self._check(self.lib.dgj_mlp_sizes(self.h, C.byref(npar), C.byref(nin), C.byref(nout)))
        self.mlp_n_params, self.mlp_n_in, self.mlp_n_out = npar.value, nin.value, nout.value

    def mlp_get_params(self, out):
        self._check(self.lib.dgj_mlp_get_params(self.h, _fptr(out)))

    def mlp_set_params(self, params):
        self._check(self.lib.dgj_mlp_set_params(self.h, _fptr(params)))

    def mlp_fit(self, S_rec, inc_rec, n_steps, epochs, lr):
        loss = C.c_double()
        self._check(self.lib.dgj_mlp_fit(self.h, _ptr(S_rec), _ptr(inc_rec), int(n_steps), int(epochs), float(lr),
                                         C.byref(loss)))
        return loss.value

    def guess_state(self, inc_out=None, inc_in=None):
        self._check(self.lib.dgj_guess_state(self.h, _ptr(inc_out), _ptr(inc_in)))

    def mlp_features(self, i1, i2, i3, X):
        self._check(self.lib.dgj_mlp_features(self.h, _ptr(i1), _ptr(i2), _ptr(i3), _fptr(X)))

    def mlp_pool(self, X):
        """Pooled forward pass: the mean over the rows of MLP(X) (numpy, n_out values)."""
        out = np.zeros(self.mlp_n_out)
        self._check(self.lib.dgj_mlp_pool(self.h, _fptr(X), X.shape[0], out.ctypes.data))
        return out

    def mlp_pool_backward(self, dLdc, grad=None):
        d = np.ascontiguousarray(dLdc, dtype=np.float64)
        self._check(self.lib.dgj_mlp_pool_backward(self.h, d.ctypes.data, _fptr(grad)))

    def mlp_forward(self, X, Y):
        self._check(self.lib.dgj_mlp_forward(self.h, _fptr(X), X.shape[0], _fptr(Y)))

    def mlp_grad(self, X, T, grad=None):
        loss = C.c_double()
        self._check(self.lib.dgj_mlp_grad(self.h, _fptr(X), _fptr(T), X.shape[0], _fptr(grad), C.byref(loss)))
        return loss.value

    def mlp_train_step(self, X, T, lr):
        loss = C.c_double()
        self._check(self.lib.dgj_mlp_train_step(self.h, _fptr(X), _fptr(T), X.shape[0], float(lr), C.byref(loss)))
        return loss.value
