"""ctypes binding of libibfsi.so (argument marshalling only).

Every computation happens in the HIP library; this module converts Python/NumPy
arguments to the C-ABI declared in ``include/ibfsi.h`` and raises on error codes.
PyTorch supplies device memory (through the allocator callbacks) and the stream.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libibfsi.so")

IB_FP64 = 0
IB_FP32_FLOW = 1
IB_FP32_FLOW_BF16_DST = 2
IB_SCHUR_AUTO = 0
IB_SCHUR_EXACT = 1
IB_SCHUR_SUBDOMAIN = 2
IB_DELTA_ROMA3 = 0
IB_DELTA_PESKIN4 = 1

(IB_OK, IB_ERR_ARG, IB_ERR_STATE, IB_ERR_OOM, IB_ERR_HIP, IB_ERR_NOT_CONVERGED,
 IB_ERR_OUT_OF_SUBDOMAIN, IB_ERR_NEAR_BOUNDARY, IB_ERR_NONFINITE, IB_ERR_CAPACITY, IB_ERR_BUDGET,
 IB_ERR_SCRATCH) = range(0, -12, -1)

STATUS = {
    0: "IB_OK", -1: "IB_ERR_ARG", -2: "IB_ERR_STATE", -3: "IB_ERR_OOM", -4: "IB_ERR_HIP",
    -5: "IB_ERR_NOT_CONVERGED", -6: "IB_ERR_OUT_OF_SUBDOMAIN", -7: "IB_ERR_NEAR_BOUNDARY",
    -8: "IB_ERR_NONFINITE", -9: "IB_ERR_CAPACITY", -10: "IB_ERR_BUDGET", -11: "IB_ERR_SCRATCH",
}


class IbError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


class IbConfig(ctypes.Structure):
    _fields_ = [
        ("n", c_int32), ("levels", c_int32), ("h", c_double), ("cx", c_double), ("cy", c_double),
        ("re", c_double), ("dt", c_double), ("u_inf", c_double * 2), ("precision", c_int32),
        ("schur_mode", c_int32), ("newton_tol", c_double), ("newton_max_iter", c_int32),
        ("newton_fixed_iter", c_int32), ("drop_tol", c_double), ("delta", c_int32),
        ("ny", c_int32),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
MOTION_FN = ctypes.CFUNCTYPE(None, c_double, POINTER(c_double), c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class IbAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", c_void_p)]


class IbStats(ctypes.Structure):
    _fields_ = [
        ("step", c_int64), ("newton_iters", c_int32), ("newton_iters_max", c_int32),
        ("newton_delta", c_double), ("subdomain_points", c_int64), ("subdomain_nnz", c_int64),
        ("prepare_seconds", c_double), ("refine_iters", c_int32), ("inverse_rebuilds", c_int32),
        ("refine_residual", c_double), ("operator_source", c_int32),
        ("graph_launches", c_int64), ("graph_captures", c_int64), ("fsi_resumes", c_int64),
        ("converged", c_int32), ("noslip_resid", c_double), ("force", c_double * 2),
        ("solve_fallbacks", c_int64), ("solve_by_lu", c_int32),
    ]


FLOW_VARIANTS = 9
IB_OPT_FSI_AHEAD, IB_OPT_GRAPHS, IB_OPT_REFRESH_EVERY_ITER, IB_OPT_TOP_AHEAD = 1, 2, 3, 4
IB_OPT_BARRIER_SPIN, IB_OPT_BARRIER_FORCE_TIMEOUT = 5, 6


class IbFlowTuning(ctypes.Structure):
    _fields_ = [
        ("n", c_int32), ("rhs_variant", c_int32), ("col_variant", c_int32),
        ("idst_variant", c_int32), ("rhs_us", c_double * FLOW_VARIANTS),
        ("col_us", c_double * FLOW_VARIANTS), ("idst_us", c_double * FLOW_VARIANTS),
    ]


class IbRequestInfo(ctypes.Structure):
    _fields_ = [
        ("ticket", c_int64), ("status", c_int32), ("steps_done", c_int32), ("arrival", c_double),
        ("admitted", c_double), ("started", c_double), ("finished", c_double), ("bytes", c_int64),
    ]


class IbBatchStats(ctypes.Structure):
    _fields_ = [
        ("steps", c_int64), ("member_steps_batched", c_int64), ("member_steps_alone", c_int64),
        ("launches", c_int64), ("fsi_resumes", c_int64),
    ]


_SIGS = {
    "ib_create": (c_int32, [POINTER(IbConfig), POINTER(IbAllocator), c_void_p, POINTER(c_void_p)]),
    "ib_add_rigid": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_double, POINTER(c_double),
                               POINTER(c_int32)]),
    "ib_add_torsional": (c_int32, [c_void_p, c_int32] + [c_double] * 9 + [POINTER(c_int32)]),
    "ib_add_moving_rigid": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_double, MOTION_FN,
                                      c_void_p, POINTER(c_int32)]),
    "ib_add_mounted_torsional": (c_int32, [c_void_p, c_int32, c_int32] + [c_double] * 11 +
                                 [POINTER(c_int32)]),
    "ib_add_deformable": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_double, c_double,
                                    c_double, POINTER(c_double), POINTER(c_double),
                                    POINTER(c_int32)]),
    "ib_set_subdomain": (c_int32, [c_void_p, c_double, c_double, c_double, c_double]),
    "ib_set_vorticity": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "ib_prepare": (c_int32, [c_void_p]),
    "ib_step": (c_int32, [c_void_p, c_int32]),
    "ib_sync": (c_int32, [c_void_p]),
    "ib_read_stresses": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int64]),
    "ib_read_deflection": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int64]),
    "ib_read_vorticity": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int64]),
    "ib_read_force": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int64]),
    "ib_read_streamfunction": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int64]),
    "ib_get_stats": (c_int32, [c_void_p, POINTER(IbStats)]),
    "ib_destroy": (c_int32, [c_void_p]),
    "ib_status_str": (ctypes.c_char_p, [c_int32]),
    "ib_op_solve": (c_int32, [c_int32, c_int32, c_double, c_void_p, c_void_p, c_int32, c_void_p]),
    "ib_op_solve_noalloc": (c_int32, [c_int32, c_int32, c_double, c_void_p, c_void_p, c_int32,
                                      c_void_p]),
    "ib_set_kernel_timing": (c_int32, [c_void_p, c_int32]),
    "ib_get_kernel_timing": (c_int32, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_double)]),
    "ib_set_stream": (c_int32, [c_void_p, c_void_p]),
    "ib_set_operator_cache": (c_int32, [c_int64]),
    "ib_export_operator": (c_int32, [c_void_p, c_void_p, c_int64, POINTER(c_int64)]),
    "ib_import_operator": (c_int32, [c_void_p, c_void_p, c_int64]),
    "ib_release": (c_int32, [c_void_p]),
    "ib_estimate_bytes": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    "ib_server_create": (c_int32, [c_int32, c_int64, c_int32, POINTER(c_void_p)]),
    "ib_server_submit": (c_int32, [c_void_p, c_void_p, c_int32, c_double, POINTER(c_int64)]),
    "ib_server_run": (c_int32, [c_void_p]),
    "ib_server_info": (c_int32, [c_void_p, c_int64, POINTER(IbRequestInfo)]),
    "ib_server_destroy": (c_int32, [c_void_p]),
    "ib_get_flow_tuning": (c_int32, [c_void_p, POINTER(IbFlowTuning)]),
    "ib_set_option": (c_int32, [c_void_p, c_int32, c_int64]),
    "ib_last_error": (ctypes.c_char_p, [c_void_p]),
    "ib_set_flow_variants": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "ib_flow_variant_info": (c_int32, [c_int32, c_int32, POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_int32)]),
    "ib_batch_create": (c_int32, [POINTER(c_void_p), c_int32, c_void_p, POINTER(c_void_p)]),
    "ib_batch_step": (c_int32, [c_void_p, c_int32]),
    "ib_batch_get_stats": (c_int32, [c_void_p, POINTER(IbBatchStats)]),
    "ib_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "ib_batch_destroy": (c_int32, [c_void_p]),
}

K_RHS_ROWDST, K_COL_SOLVE, K_ROW_IDST, K_FSI, K_CORRECT, K_RING = range(6)

_LIB = None


def load(path: str = LIB_PATH):
    """Load the built library; raises if it is missing (no fallback exists)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"libibfsi.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _check(code, what):
    if code != 0:
        raise IbError(code, what)


def _dptr(a):
    return a.ctypes.data_as(POINTER(c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class TorchAllocator:
    """Device memory from PyTorch's caching allocator, on the solver's stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream

        self.last_error = None

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception as e:  # reported to the library as out of memory
                self.last_error = e
                return None

        def _free(ptr, ctx):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch is gone, and so is its memory
                pass

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)
        self.struct = IbAllocator(self._alloc, self._free, None)


def flow_variant_info(kind, variant):
    """(width, threads, largest radix) of configuration `variant`; kind 0 rows, 1 columns."""
    w, t, r = c_int32(), c_int32(), c_int32()
    _check(load().ib_flow_variant_info(kind, variant, byref(w), byref(t), byref(r)),
           "ib_flow_variant_info")
    return w.value, t.value, r.value


def set_operator_cache(limit_bytes):
    _check(load().ib_set_operator_cache(int(limit_bytes)), "ib_set_operator_cache")


def op_solve(n, precision, alpha, in_ptr, out_ptr, pitch, stream=0):
    """[L (I + alpha L)]^{-1} on device arrays (see ib_op_solve)."""
    lib = load()
    _check(lib.ib_op_solve(n, precision, alpha, c_void_p(in_ptr), c_void_p(out_ptr), pitch,
                           c_void_p(stream)), "ib_op_solve")


def op_solve_noalloc(n, precision, alpha, in_ptr, out_ptr, pitch, stream=0):
    """ib_op_solve without device allocation (see ib_op_solve_noalloc)."""
    lib = load()
    _check(lib.ib_op_solve_noalloc(n, precision, alpha, c_void_p(in_ptr), c_void_p(out_ptr), pitch,
                                   c_void_p(stream)), "ib_op_solve_noalloc")


class Solver:
    """One solver instance built from a ``workloads.Problem``."""

    def __init__(self, problem, precision=IB_FP64, schur=IB_SCHUR_AUTO, newton_tol=1e-7,
                 newton_max=20, fixed_iters=0, drop_tol=0.007, torch_alloc=True, stream=None):
        import torch
        import workloads as W
        self.lib = load()
        self.problem = problem
        fl = problem.flow
        cfg = IbConfig()
        cfg.n, cfg.levels, cfg.h = fl.n, fl.levels, fl.h
        cfg.cx, cfg.cy, cfg.re, cfg.dt = fl.cx, fl.cy, fl.re, fl.dt
        cfg.u_inf[0], cfg.u_inf[1] = fl.u_inf
        cfg.precision, cfg.schur_mode = precision, schur
        cfg.newton_tol, cfg.newton_max_iter = newton_tol, newton_max
        cfg.newton_fixed_iter, cfg.drop_tol = fixed_iters, drop_tol
        cfg.delta = {"roma3": IB_DELTA_ROMA3, "peskin4": IB_DELTA_PESKIN4}[getattr(fl, "delta", "roma3")]
        cfg.ny = getattr(fl, "ny", 0) or 0
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._alloc = TorchAllocator(torch.cuda.current_device(), self.stream) if torch_alloc else None
        self.handle = c_void_p()
        _check(self.lib.ib_create(byref(cfg), byref(self._alloc.struct) if self._alloc else None,
                                  c_void_p(self.stream.cuda_stream if self.stream is not False else 0),
                                  byref(self.handle)), "ib_create")
        self.npts = []
        self._motion_cbs = []  # keep the callbacks alive as long as the solver
        for b in problem.bodies:
            bid = c_int32()
            if isinstance(b, W.MovingRigid):
                ref = _f64(b.xy_ref)

                def _cb(t, pose, ctx, body=b):
                    q = body.pose(t)
                    for k in range(6):
                        pose[k] = q[k]
                    if body.accel is not None:
                        acc = body.accelerations(t)
                        for k in range(3):
                            pose[6 + k] = acc[k]

                cb = MOTION_FN(_cb)
                self._motion_cbs.append(cb)
                _check(self.lib.ib_add_moving_rigid(self.handle, ref.shape[0], _dptr(ref), b.ds, cb,
                                                    None, byref(bid)), "ib_add_moving_rigid")
                self.npts.append(ref.shape[0])
            elif isinstance(b, W.Rigid):
                xy = _f64(b.xy)
                ub = None if b.u_b is None else _f64(b.u_b)
                _check(self.lib.ib_add_rigid(self.handle, xy.shape[0], _dptr(xy), b.ds,
                                             None if ub is None else _dptr(ub), byref(bid)),
                       "ib_add_rigid")
                self.npts.append(xy.shape[0])
            elif isinstance(b, W.MountedTorsional):
                _check(self.lib.ib_add_mounted_torsional(
                    self.handle, b.n, b.driver, b.hinge_body[0], b.hinge_body[1], b.theta_rel,
                    b.length, b.inertia, b.stiffness, b.damping, b.mass, b.cg, b.theta, b.phi,
                    byref(bid)), "ib_add_mounted_torsional")
                self.npts.append(b.n)
            elif isinstance(b, W.Torsional):
                _check(self.lib.ib_add_torsional(self.handle, b.n, b.hinge[0], b.hinge[1], b.length,
                                                 b.theta0, b.inertia, b.stiffness, b.damping,
                                                 b.theta, b.phi, byref(bid)), "ib_add_torsional")
                self.npts.append(b.n)
            else:
                xr, x0, r0 = _f64(b.xy_ref), _f64(b.xy0), _f64(b.rot0)
                _check(self.lib.ib_add_deformable(self.handle, xr.shape[0], _dptr(xr), b.mass, b.ei,
                                                  b.ea, _dptr(x0), _dptr(r0), byref(bid)),
                       "ib_add_deformable")
                self.npts.append(xr.shape[0])
        if problem.subdomain is not None:
            sd = problem.subdomain
            rects = [sd] if len(sd) == 4 and all(np.isscalar(v) for v in sd) else list(sd)
            for r in rects:
                _check(self.lib.ib_set_subdomain(self.handle, *r), "ib_set_subdomain")
        if problem.vorticity0 is not None:
            for g, w in enumerate(problem.vorticity0):
                if w is not None:
                    w = _f64(w)
                    _check(self.lib.ib_set_vorticity(self.handle, g, _dptr(w)), "ib_set_vorticity")

    def prepare(self):
        _check(self.lib.ib_prepare(self.handle), "ib_prepare")

    def step(self, n=1):
        _check(self.lib.ib_step(self.handle, n), "ib_step")

    def sync(self):
        _check(self.lib.ib_sync(self.handle), "ib_sync")

    def stresses(self, body):
        out = np.zeros(2 * self.npts[body])
        _check(self.lib.ib_read_stresses(self.handle, body, _dptr(out), out.size), "ib_read_stresses")
        return out

    def deflection(self, body):
        import workloads as W
        b = self.problem.bodies[body]
        size = 3 if isinstance(b, (W.Torsional, W.MountedTorsional)) else (3 if isinstance(b, W.Deformable) else 2) * self.npts[body]
        out = np.zeros(size)
        _check(self.lib.ib_read_deflection(self.handle, body, _dptr(out), out.size), "ib_read_deflection")
        return out

    def vorticity(self, level=0):
        nx, ny = self.problem.flow.nx_ny
        out = np.zeros((nx - 1) * (ny - 1))
        _check(self.lib.ib_read_vorticity(self.handle, level, _dptr(out), out.size), "ib_read_vorticity")
        return out.reshape(ny - 1, nx - 1)

    def streamfunction(self, level=0):
        nx, ny = self.problem.flow.nx_ny
        out = np.zeros((nx + 1) * (ny + 1))
        _check(self.lib.ib_read_streamfunction(self.handle, level, _dptr(out), out.size),
               "ib_read_streamfunction")
        return out.reshape(ny + 1, nx + 1)

    def stats(self):
        st = IbStats()
        _check(self.lib.ib_get_stats(self.handle, byref(st)), "ib_get_stats")
        out = {k: getattr(st, k) for k, _ in IbStats._fields_}
        out["force"] = (st.force[0], st.force[1])
        return out

    def force(self, body):
        out = np.zeros(2)
        _check(self.lib.ib_read_force(self.handle, body, _dptr(out), out.size), "ib_read_force")
        return out

    def set_kernel_timing(self, on=True):
        _check(self.lib.ib_set_kernel_timing(self.handle, 1 if on else 0), "ib_set_kernel_timing")

    def kernel_timing(self, cls):
        n, ms = c_int64(), c_double()
        _check(self.lib.ib_get_kernel_timing(self.handle, cls, byref(n), byref(ms)),
               "ib_get_kernel_timing")
        return n.value, ms.value

    def flow_tuning(self):
        """The measured transform-kernel configurations (see ib_get_flow_tuning)."""
        t = IbFlowTuning()
        _check(self.lib.ib_get_flow_tuning(self.handle, byref(t)), "ib_get_flow_tuning")
        return {"n": t.n, "rhs_variant": t.rhs_variant, "col_variant": t.col_variant,
                "idst_variant": t.idst_variant, "rhs_us": list(t.rhs_us),
                "col_us": list(t.col_us), "idst_us": list(t.idst_us)}

    def last_error(self):
        return self.lib.ib_last_error(self.handle).decode()

    def set_option(self, option, value):
        _check(self.lib.ib_set_option(self.handle, option, int(value)), "ib_set_option")

    def set_flow_variants(self, rhs=-1, col=-1, idst=-1):
        _check(self.lib.ib_set_flow_variants(self.handle, rhs, col, idst), "ib_set_flow_variants")

    def release(self):
        """Give the device memory back; stresses, deflections and level-0 vorticity stay readable."""
        _check(self.lib.ib_release(self.handle), "ib_release")

    def export_operator(self):
        """The offline operator as bytes (see ib_export_operator)."""
        used = c_int64()
        code = self.lib.ib_export_operator(self.handle, None, 0, byref(used))
        if code not in (0, -9):
            raise IbError(code, "ib_export_operator")
        buf = ctypes.create_string_buffer(used.value)
        _check(self.lib.ib_export_operator(self.handle, buf, used.value, byref(used)),
               "ib_export_operator")
        return buf.raw

    def import_operator(self, data):
        _check(self.lib.ib_import_operator(self.handle, data, len(data)), "ib_import_operator")

    def estimate_bytes(self):
        res, peak = c_int64(), c_int64()
        _check(self.lib.ib_estimate_bytes(self.handle, byref(res), byref(peak)), "ib_estimate_bytes")
        return res.value, peak.value

    def close(self):
        if self.handle:
            self.lib.ib_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many prepared solvers of one precision class stepped together, each kernel launch
    covering all members (ib_batch_*).  From construction on the members' work runs on
    ``stream`` (default: the current torch stream)."""

    def __init__(self, solvers, stream=None):
        import torch
        self.lib = load()
        self.solvers = list(solvers)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (c_void_p * len(self.solvers))(*[s.handle.value for s in self.solvers])
        self.handle = c_void_p()
        _check(self.lib.ib_batch_create(arr, len(self.solvers), c_void_p(self.stream.cuda_stream),
                                        byref(self.handle)), "ib_batch_create")
        for s in self.solvers:
            s.stream = self.stream

    def step(self, nsteps=1):
        code = self.lib.ib_batch_step(self.handle, nsteps)
        if code != 0:
            raise IbError(code, "ib_batch_step: " + self.last_error())

    def stats(self):
        r = IbBatchStats()
        _check(self.lib.ib_batch_get_stats(self.handle, byref(r)), "ib_batch_get_stats")
        return {k: getattr(r, k) for k, _ in IbBatchStats._fields_}

    def last_error(self):
        return self.lib.ib_batch_last_error(self.handle).decode()

    def close(self):
        if self.handle:
            self.lib.ib_batch_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching scheduler (ib_server_*): solvers built with torch_alloc=False and
    stream=False (the server gives each its own stream), submitted with step counts and
    arrival times, run to completion by ``run``."""

    def __init__(self, max_active, hbm_budget_bytes, chunk_steps=50):
        self.lib = load()
        self.handle = c_void_p()
        _check(self.lib.ib_server_create(max_active, int(hbm_budget_bytes), chunk_steps,
                                         byref(self.handle)), "ib_server_create")
        self.solvers = []

    def submit(self, solver, nsteps, arrival=0.0):
        t = c_int64()
        _check(self.lib.ib_server_submit(self.handle, solver.handle, nsteps, arrival, byref(t)),
               "ib_server_submit")
        self.solvers.append(solver)
        return t.value

    def run(self):
        _check(self.lib.ib_server_run(self.handle), "ib_server_run")

    def info(self, ticket):
        r = IbRequestInfo()
        _check(self.lib.ib_server_info(self.handle, ticket, byref(r)), "ib_server_info")
        return {k: getattr(r, k) for k, _ in IbRequestInfo._fields_}

    def close(self):
        if self.handle:
            self.lib.ib_server_destroy(self.handle)
            self.handle = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
