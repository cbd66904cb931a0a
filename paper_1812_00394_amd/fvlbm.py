"""Python binding of libfvlbm.so (ctypes).  Argument marshalling only: every step of the method
runs in the library's HIP kernels; PyTorch provides the device workspace and the stream.

    mesh = Mesh(mesh_dict)                          # host preprocessing (FP64)
    st = State(mesh, params, precision="fp64", rho=..., u=..., k=..., omega=...)
    st.step(100); res = st.step(1, residual=True)
    m = st.moments()                                # dict of numpy arrays, user cell order
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import LIB

FVLBM_MAX_GROUPS = 16
FP64, FP32_DEV, FP32_DEV_GEO64 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32dev": FP32_DEV, "fp32dev_geo64": FP32_DEV_GEO64}
ORDERS = {"none": 0, "morton": 1, "rcm": 2, "tiles": 3}
STATUS = {0: "OK", -1: "EINVAL", -2: "EMESH", -3: "ENOMEM", -4: "EDEVICE", -5: "EDIVERGED", -6: "ESTATE"}

# k-omega SST constants as listed in Section 2 of the paper
SST_CONSTANTS = dict(a1=0.31, beta_star=0.09, kappa=0.41, sigma_k1=0.85, sigma_w1=0.5, beta1=0.075,
                     sigma_k2=1.0, sigma_w2=0.856, beta2=0.0828)


class FvlbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fvlbm {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("nu", C.c_double), ("dt", C.c_double), ("rho0", C.c_double),
                ("sst", C.c_int32), ("n_groups", C.c_int32),
                ("a1", C.c_double), ("beta_star", C.c_double), ("kappa", C.c_double),
                ("sigma_k1", C.c_double), ("sigma_w1", C.c_double), ("beta1", C.c_double),
                ("sigma_k2", C.c_double), ("sigma_w2", C.c_double), ("beta2", C.c_double),
                ("theta", C.c_double),
                ("group_u", (C.c_double * 2) * FVLBM_MAX_GROUPS),
                ("group_rho", C.c_double * FVLBM_MAX_GROUPS),
                ("group_k", C.c_double * FVLBM_MAX_GROUPS),
                ("group_w", C.c_double * FVLBM_MAX_GROUPS),
                ("bface_vals", C.POINTER(C.c_double)),
                ("jr_group", C.c_int32), ("limiter", C.c_int32),
                ("jr_xmin", C.c_double), ("eps_tau", C.c_double), ("sst_sweeps", C.c_int32)]


_lib = None

EXPORTS = ["fvlbm_mesh_create", "fvlbm_mesh_destroy", "fvlbm_mesh_counts", "fvlbm_mesh_geometry",
           "fvlbm_mesh_permutation", "fvlbm_state_bytes", "fvlbm_init", "fvlbm_set_state", "fvlbm_step",
           "fvlbm_moments", "fvlbm_get_f", "fvlbm_forces", "fvlbm_apply_advection", "fvlbm_state_destroy",
           "fvlbm_last_error", "fvlbm_mesh_max_dt", "fvlbm_timing", "fvlbm_timing_read",
           "fvlbm_apply_advection_adjoint", "fvlbm_adjoint_bytes", "fvlbm_record", "fvlbm_adjoint_step",
           "fvlbm_adjoint_state", "fvlbm_lift_drag", "fvlbm_step_explicit",
           "fvlbm_run_to_residual", "fvlbm_totals_noalloc", "fvlbm_adjoint_lift_drag"]
KERNELS = ["sst_a", "sst_b", "collide1", "grad", "sweep1", "sweep2", "sweep3", "sst", "explicit", "sst_jacobi", "face"]


def lib():
    """Loads the in-tree library; fails loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is missing: build it with `python -m paper_1812_00394_amd.build`")
    # torch first: its HIP runtime then satisfies the library's libamdhip64.so.7 dependency, so the
    # workspace, the stream and the library's kernels share one runtime
    import torch  # noqa: F401
    L = C.CDLL(LIB)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.fvlbm_mesh_create.argtypes = [I64, P, I64, P, P, I64, P, P, I32, P, P, I32, C.POINTER(C.c_void_p)]
    L.fvlbm_mesh_destroy.argtypes = [P]
    L.fvlbm_mesh_destroy.restype = None
    L.fvlbm_mesh_counts.argtypes = [P, P]
    L.fvlbm_mesh_geometry.argtypes = [P, P, P, P]
    L.fvlbm_mesh_permutation.argtypes = [P, P]
    L.fvlbm_state_bytes.argtypes = [P, I32, I32, C.POINTER(C.c_size_t)]
    L.fvlbm_init.argtypes = [P, C.POINTER(Params), I32, P, P, P, P, P, C.c_size_t, P, C.POINTER(C.c_void_p)]
    L.fvlbm_set_state.argtypes = [P, P, P, P]
    L.fvlbm_step.argtypes = [P, I32, P]
    L.fvlbm_step_explicit.argtypes = [P, I32, P]
    L.fvlbm_run_to_residual.argtypes = [P, I64, I32, C.c_double, P, P]
    L.fvlbm_moments.argtypes = [P, I32, P, P, P, P, P, P]
    L.fvlbm_get_f.argtypes = [P, I32, P]
    L.fvlbm_forces.argtypes = [P, C.c_uint64, P, P]
    L.fvlbm_lift_drag.argtypes = [P, C.c_uint64, C.c_double, C.c_double, P]
    L.fvlbm_totals_noalloc.argtypes = [P, P]
    L.fvlbm_adjoint_lift_drag.argtypes = [P, C.c_uint64, C.c_double, C.c_double, P, P, P]
    L.fvlbm_apply_advection.argtypes = [P, P, P]
    L.fvlbm_mesh_max_dt.argtypes = [P, P]
    L.fvlbm_timing.argtypes = [P, I32]
    L.fvlbm_timing_read.argtypes = [P, P, P]
    L.fvlbm_apply_advection_adjoint.argtypes = [P, P, P, P, P]
    L.fvlbm_adjoint_bytes.argtypes = [P, I32, I32, I32, C.POINTER(C.c_size_t)]
    L.fvlbm_record.argtypes = [P, I32, I32, P, C.c_size_t]
    L.fvlbm_adjoint_step.argtypes = [P, C.c_uint64, P, P]
    L.fvlbm_adjoint_state.argtypes = [P, P, P, P, P, P, P, P]
    L.fvlbm_state_destroy.argtypes = [P]
    L.fvlbm_state_destroy.restype = None
    L.fvlbm_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("fvlbm_mesh_destroy", "fvlbm_state_destroy", "fvlbm_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status):
    if status != 0:
        raise FvlbmError(status, lib().fvlbm_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Mesh:
    """Mesh preprocessed by the library (host, FP64); order: "tiles" (graph-grown tiles, the
    default), "morton", "rcm" or "none" (the fvlbm_mesh_create renumbering)."""

    def __init__(self, m, order="tiles"):
        L = lib()
        self._keep = dict(
            nodes=_f64(m["nodes"]),
            cell_ptr=np.ascontiguousarray(m["cell_ptr"], dtype=np.int64),
            cell_nodes=np.ascontiguousarray(m["cell_nodes"], dtype=np.int64),
            bface_nodes=np.ascontiguousarray(m["bface_nodes"], dtype=np.int64),
            bface_group=np.ascontiguousarray(m["bface_group"], dtype=np.int32),
            group_kind=np.ascontiguousarray(m["group_kind"], dtype=np.int32),
            periodic_shift=_f64(m["periodic_shift"]))
        k = self._keep
        self.n_groups = len(k["group_kind"])
        self.n_bfaces = len(k["bface_group"])
        h = C.c_void_p()
        _check(L.fvlbm_mesh_create(len(k["nodes"]), _ptr(k["nodes"]), len(k["cell_ptr"]) - 1, _ptr(k["cell_ptr"]),
                                   _ptr(k["cell_nodes"]), self.n_bfaces, _ptr(k["bface_nodes"]),
                                   _ptr(k["bface_group"]), self.n_groups, _ptr(k["group_kind"]),
                                   _ptr(k["periodic_shift"]), ORDERS[order], C.byref(h)))
        self.handle = h
        counts = np.zeros(4, dtype=np.int64)
        _check(L.fvlbm_mesh_counts(h, _ptr(counts)))
        self.n_cells, self.n_interior_edges, self.n_boundary_edges, self.max_faces = (int(x) for x in counts)

    def geometry(self):
        n = self.n_cells
        area, cen, wd = np.zeros(n), np.zeros((n, 2)), np.zeros(n)
        _check(lib().fvlbm_mesh_geometry(self.handle, _ptr(area), _ptr(cen), _ptr(wd)))
        return area, cen, wd

    def permutation(self):
        p = np.zeros(self.n_cells, dtype=np.int64)
        _check(lib().fvlbm_mesh_permutation(self.handle, _ptr(p)))
        return p

    def max_dt(self):
        """time step at advective Courant number 1"""
        d = np.zeros(1)
        _check(lib().fvlbm_mesh_max_dt(self.handle, _ptr(d)))
        return float(d[0])

    def state_bytes(self, precision="fp64", sst=False):
        b = C.c_size_t()
        _check(lib().fvlbm_state_bytes(self.handle, PRECISIONS[precision], int(bool(sst)), C.byref(b)))
        return b.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fvlbm_mesh_destroy(self.handle)
            self.handle = None


def make_params(p, n_groups, n_bfaces=None):
    """Builds the C parameter struct from a dictionary (keys as in the header)."""
    s = Params()
    s.nu, s.dt, s.rho0 = float(p["nu"]), float(p["dt"]), float(p.get("rho0", 1.0))
    s.sst = (2 if p.get("sst_stages") else 1) if p.get("sst", False) else 0
    s.n_groups = n_groups
    c = dict(SST_CONSTANTS)
    c.update({k: p[k] for k in SST_CONSTANTS if k in p})
    for k, v in c.items():
        setattr(s, k, float(v))
    s.theta = float(p.get("theta", 0.0))
    gu = p.get("group_u")
    gr = p.get("group_rho")
    gk = p.get("group_k")
    gw = p.get("group_w")
    for g in range(n_groups):
        if gu is not None:
            s.group_u[g][0], s.group_u[g][1] = float(gu[g][0]), float(gu[g][1])
        s.group_rho[g] = float(gr[g]) if gr is not None else s.rho0
        s.group_k[g] = float(gk[g]) if gk is not None else 0.0
        s.group_w[g] = float(gw[g]) if gw is not None else 1.0
    bv = p.get("bface_vals")
    keep = None
    if bv is not None:
        keep = _f64(bv, (n_bfaces, 5))
        s.bface_vals = keep.ctypes.data_as(C.POINTER(C.c_double))
    s.jr_group = int(p.get("jr_group", -1))
    s.limiter = int(p.get("limiter", 0))
    s.sst_sweeps = int(p.get("sst_sweeps", 0))
    s.jr_xmin = float(p.get("jr_xmin", 0.0))
    s.eps_tau = float(p.get("eps_tau", 1.0))
    return s, keep


class State:
    """One simulation state on the current HIP device (workspace = a torch uint8 tensor)."""

    def __init__(self, mesh: Mesh, params: dict, precision="fp64", rho=None, u=None, k=None, omega=None,
                 device="cuda", stream=None):
        import torch
        L = lib()
        self.mesh = mesh
        self.precision = precision
        self.sst = bool(params.get("sst", False))
        n = mesh.n_cells
        nbytes = mesh.state_bytes(precision, self.sst)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        if stream is None:
            stream = torch.cuda.current_stream(self.workspace.device)
        self.stream = stream
        self.params, self._keep_bv = make_params(params, mesh.n_groups, mesh.n_bfaces)
        rho = _f64(np.ones(n) if rho is None else rho, (n,))
        u = _f64(np.zeros((n, 2)) if u is None else u, (n, 2))
        kk = _f64(k, (n,)) if k is not None else None
        ww = _f64(omega, (n,)) if omega is not None else None
        h = C.c_void_p()
        _check(L.fvlbm_init(mesh.handle, C.byref(self.params), PRECISIONS[precision],
                            _ptr(rho), _ptr(u), _ptr(kk), _ptr(ww), C.c_void_p(self.workspace.data_ptr()),
                            nbytes, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.handle = h

    def step(self, n_steps=1, residual=False):
        r = C.c_double()
        _check(lib().fvlbm_step(self.handle, int(n_steps), C.byref(r) if residual else None))
        return r.value if residual else None

    def run_to_residual(self, tol, max_steps, check_every=1000):
        """Step until the velocity residual is below tol (checked every check_every steps) or
        max_steps steps were taken; returns (steps taken, last residual)."""
        n = C.c_int64()
        r = C.c_double()
        _check(lib().fvlbm_run_to_residual(self.handle, int(max_steps), int(check_every), float(tol),
                                           C.byref(n), C.byref(r)))
        return n.value, r.value

    def step_explicit(self, n_steps=1, residual=False):
        """n_steps of the explicit (forward Euler) scheme; stable for dt < 2 tau only."""
        r = C.c_double()
        _check(lib().fvlbm_step_explicit(self.handle, int(n_steps), C.byref(r) if residual else None))
        return r.value if residual else None

    def set_state(self, f=None, k=None, omega=None):
        n = self.mesh.n_cells
        f = _f64(f, (9, n)) if f is not None else None
        k = _f64(k, (n,)) if k is not None else None
        omega = _f64(omega, (n,)) if omega is not None else None
        _check(lib().fvlbm_set_state(self.handle, _ptr(f), _ptr(k), _ptr(omega)))

    def get_f(self):
        f = np.zeros((9, self.mesh.n_cells))
        _check(lib().fvlbm_get_f(self.handle, 0, _ptr(f)))
        return f

    def moments(self):
        n = self.mesh.n_cells
        out = dict(rho=np.zeros(n), u=np.zeros((n, 2)))
        if self.sst:
            out.update(k=np.zeros(n), omega=np.zeros(n), nu_t=np.zeros(n))
        tot = np.zeros(3)
        _check(lib().fvlbm_moments(self.handle, 0, _ptr(out["rho"]), _ptr(out["u"]), _ptr(out.get("k")),
                                   _ptr(out.get("omega")), _ptr(out.get("nu_t")), _ptr(tot)))
        out["totals"] = tot
        return out

    def forces(self, group_mask):
        F = np.zeros(2)
        jr = C.c_double()
        _check(lib().fvlbm_forces(self.handle, C.c_uint64(group_mask), _ptr(F), C.byref(jr)))
        return F, jr.value

    def totals_noalloc(self, out):
        """fvlbm_totals_noalloc: the totals into `out`, a torch float64 device tensor of 3 elements,
        enqueued on the state's stream (no synchronisation, no allocation in the library)."""
        import torch
        if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= 3 and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 device tensor of at least 3 elements")
        _check(lib().fvlbm_totals_noalloc(self.handle, C.c_void_p(out.data_ptr())))
        return out

    def lift_drag(self, group_mask, u_ref, chord=1.0):
        """(C_l, C_d) of the walls in group_mask: drag along the free stream (theta), lift normal to it."""
        c = np.zeros(2)
        _check(lib().fvlbm_lift_drag(self.handle, C.c_uint64(group_mask), float(u_ref), float(chord), _ptr(c)))
        return float(c[0]), float(c[1])

    def apply_advection(self, g):
        n = self.mesh.n_cells
        g = _f64(g, (9, n))
        out = np.zeros((9, n))
        _check(lib().fvlbm_apply_advection(self.handle, _ptr(g), _ptr(out)))
        return out

    def apply_advection_adjoint(self, g, lam):
        """(d Gamma^a(g)/dg)^T lam and d(lam . Gamma^a(g))/d theta"""
        n = self.mesh.n_cells
        g = _f64(g, (9, n))
        lam = _f64(lam, (9, n))
        out = np.zeros((9, n))
        dth = np.zeros(1)
        _check(lib().fvlbm_apply_advection_adjoint(self.handle, _ptr(g), _ptr(lam), _ptr(out), _ptr(dth)))
        return out, float(dth[0])

    # ---- adjoint ----
    def record(self, n_steps, ckpt_every=20):
        """advance n_steps steps, storing checkpoints for the adjoint"""
        import torch
        b = C.c_size_t()
        prec = PRECISIONS[self.precision]
        _check(lib().fvlbm_adjoint_bytes(self.mesh.handle, prec, int(n_steps), int(ckpt_every), C.byref(b)))
        self.adj_workspace = torch.empty(b.value, dtype=torch.uint8, device=self.workspace.device)
        _check(lib().fvlbm_record(self.handle, int(n_steps), int(ckpt_every),
                                  C.c_void_p(self.adj_workspace.data_ptr()), b.value))

    def adjoint(self, group_mask, seed):
        """dJ/d(theta, sigma_k1, sigma_w1, beta*, a1) for J = seed . (F_x, F_y, J_R) of the final state"""
        sd = _f64(seed, (3,))
        out = np.zeros(5)
        _check(lib().fvlbm_adjoint_step(self.handle, C.c_uint64(group_mask), _ptr(sd), _ptr(out)))
        return out

    def adjoint_lift_drag(self, group_mask, u_ref, chord, seed):
        """dJ/d(theta, sigma_k1, sigma_w1, beta*, a1) for J = seed . (C_l, C_d) of the final state;
        returns (gradient, (C_l, C_d))"""
        sd = _f64(seed, (2,))
        out = np.zeros(5)
        co = np.zeros(2)
        _check(lib().fvlbm_adjoint_lift_drag(self.handle, C.c_uint64(group_mask), float(u_ref), float(chord),
                                             _ptr(sd), _ptr(co), _ptr(out)))
        return out, (float(co[0]), float(co[1]))

    def adjoint_state(self, lam_f, lam_k=None, lam_w=None):
        n = self.mesh.n_cells
        lf = _f64(lam_f, (9, n))
        lk = _f64(lam_k, (n,)) if lam_k is not None else None
        lw = _f64(lam_w, (n,)) if lam_w is not None else None
        of, ok, ow = np.zeros((9, n)), np.zeros(n), np.zeros(n)
        dp = np.zeros(5)
        _check(lib().fvlbm_adjoint_state(self.handle, _ptr(lf), _ptr(lk), _ptr(lw), _ptr(of),
                                         _ptr(ok) if self.sst else None, _ptr(ow) if self.sst else None, _ptr(dp)))
        return of, ok, ow, dp

    def timing(self, enable=True):
        _check(lib().fvlbm_timing(self.handle, int(bool(enable))))

    def timing_read(self):
        """{kernel: (total ms, launches)} since timing was enabled"""
        ms = np.zeros(len(KERNELS))
        cnt = np.zeros(len(KERNELS), dtype=np.int64)
        _check(lib().fvlbm_timing_read(self.handle, _ptr(ms), _ptr(cnt)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNELS)}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.fvlbm_state_destroy(self.handle)
            self.handle = None
