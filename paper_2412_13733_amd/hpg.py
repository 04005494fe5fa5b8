"""Thin ctypes binding of libhpg.so (argument marshalling only).

Every computation runs in the HIP library; this module converts Python/NumPy
/torch arguments to pointers and sizes and raises on non-OK statuses.  If the
library has not been built it raises immediately: there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpg.so")

OK, NOT_CONVERGED, PENDING = 0, 1, 2
ERR_INVALID_ARG, ERR_NOMEM, ERR_DEVICE, ERR_NUMERIC, ERR_BUDGET = -1, -2, -3, -4, -5
OBSTACLE, GRADIENT = 0, 1
FP64, MIXED = 0, 1
KRYLOV_MINRES = 0


class HpgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hpg status %d: %s" % (status, msg))
        self.status = status


class MeshInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("P", ctypes.c_int32), ("constraint", ctypes.c_int32),
                ("ncells", ctypes.c_int32 * 3), ("n_cells", ctypes.c_int64),
                ("n_u", ctypes.c_int64), ("n_psi", ctypes.c_int64), ("n_qp", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("alpha0", ctypes.c_double),
                ("alpha_factor", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("max_prox", ctypes.c_int32), ("prox_tol", ctypes.c_double),
                ("fixed_prox_steps", ctypes.c_int32), ("newton_tol", ctypes.c_double),
                ("stall_tol", ctypes.c_double), ("max_newton", ctypes.c_int32),
                ("krylov_rtol", ctypes.c_double), ("max_krylov", ctypes.c_int32),
                ("beta", ctypes.c_double), ("precision", ctypes.c_int32),
                ("krylov_chunk", ctypes.c_int32), ("inexact_newton", ctypes.c_int32),
                ("step_extension", ctypes.c_int32), ("q", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("warm_u", ctypes.c_void_p),
                ("warm_psi", ctypes.c_void_p), ("k0", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("prox_steps", ctypes.c_int32),
                ("newton_iters", ctypes.c_int32), ("line_search_halvings", ctypes.c_int32),
                ("krylov_iters", ctypes.c_int64), ("newton_error", ctypes.c_double),
                ("seconds", ctypes.c_double), ("alpha_last", ctypes.c_double),
                ("fp64_fallbacks", ctypes.c_int32), ("step_extensions", ctypes.c_int32),
                ("fp64_recomputations", ctypes.c_int32), ("complementarity", ctypes.c_double),
                ("complementarity_rel", ctypes.c_double), ("max_violation", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# every symbol include/hpg.h declares (checked by the CPU test-suite)
EXPORTS = ["hpg_last_error", "hpg_create_mesh", "hpg_destroy_mesh", "hpg_get_mesh_info",
           "hpg_quadrature_points", "hpg_create_problem", "hpg_destroy_problem",
           "hpg_set_forcing", "hpg_set_obstacle", "hpg_set_forcing_fn", "hpg_set_obstacle_fn",
           "hpg_default_opts", "hpg_solve",
           "hpg_solve_device", "hpg_op_setup", "hpg_op_apply_G", "hpg_op_apply_prec",
           "hpg_op_minres", "hpg_op_residual", "hpg_op_residual_noalloc", "hpg_l2_diff", "hpg_set_kernel_timing",
           "hpg_kernel_time", "hpg_problem_footprint", "hpg_server_create", "hpg_server_submit",
           "hpg_server_poll", "hpg_server_wait", "hpg_server_stats", "hpg_server_destroy",
           "hpg_create_batch", "hpg_destroy_batch", "hpg_batch_set_data", "hpg_batch_solve",
           "hpg_batch_op_setup", "hpg_batch_op_apply_G", "hpg_batch_set_kernel_timing",
           "hpg_batch_kernel_time"]


class RequestInfo(ctypes.Structure):
    _fields_ = [("queue_s", ctypes.c_double), ("run_s", ctypes.c_double),
                ("latency_s", ctypes.c_double), ("footprint", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServingStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("max_running", ctypes.c_int32),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_latency_s", ctypes.c_double), ("max_latency_s", ctypes.c_double),
                ("span_s", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("dof_krylov_per_s", ctypes.c_double), ("hbm_budget", ctypes.c_uint64),
                ("hbm_reserved", ctypes.c_uint64), ("hbm_peak_reserved", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

_lib = None

# double (*)(const double* x, void* ctx)
POINT_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhpg.so is not built (run paper_2412_13733_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                          ctypes.c_size_t)
    sig = {
        "hpg_last_error": ([], ctypes.c_char_p),
        "hpg_create_mesh": ([ctypes.c_int, P, P, P, I32, I32, P], ctypes.c_int),
        "hpg_destroy_mesh": ([P], None),
        "hpg_get_mesh_info": ([P, P], ctypes.c_int),
        "hpg_quadrature_points": ([P, P], ctypes.c_int),
        "hpg_create_problem": ([P, ctypes.c_int, P], ctypes.c_int),
        "hpg_destroy_problem": ([P], None),
        "hpg_set_forcing": ([P, P, SZ], ctypes.c_int),
        "hpg_set_obstacle": ([P, P, SZ], ctypes.c_int),
        "hpg_set_forcing_fn": ([P, POINT_FN, P], ctypes.c_int),
        "hpg_set_obstacle_fn": ([P, POINT_FN, P], ctypes.c_int),
        "hpg_default_opts": ([P], None),
        "hpg_solve": ([P, P, P, P, P, P], ctypes.c_int),
        "hpg_solve_device": ([P, P, P, P, P, P], ctypes.c_int),
        "hpg_op_setup": ([P, P, D, D, I32, P], ctypes.c_int),
        "hpg_op_apply_G": ([P, P, P, P], ctypes.c_int),
        "hpg_op_apply_prec": ([P, P, P, P], ctypes.c_int),
        "hpg_op_minres": ([P, P, P, D, I32, P, P], ctypes.c_int),
        "hpg_op_residual": ([P, P, P, P, D, P, P], ctypes.c_int),
        "hpg_op_residual_noalloc": ([P, P, P, P, D, P, P, P], ctypes.c_int),
        "hpg_l2_diff": ([P, P, P, P, P, P], ctypes.c_int),
        "hpg_set_kernel_timing": ([P, ctypes.c_char_p], ctypes.c_int),
        "hpg_kernel_time": ([P, ctypes.c_char_p, P, P], ctypes.c_int),
        "hpg_problem_footprint": ([P, I32, P], ctypes.c_int),
        "hpg_server_create": ([ctypes.c_int, ctypes.c_uint64, I32, P], ctypes.c_int),
        "hpg_server_submit": ([P, P, P, P, P, P], ctypes.c_int),
        "hpg_server_poll": ([P, ctypes.c_uint64, P, P, P, P], ctypes.c_int),
        "hpg_server_wait": ([P, ctypes.c_uint64, P, P, P, P], ctypes.c_int),
        "hpg_server_stats": ([P, P], ctypes.c_int),
        "hpg_server_destroy": ([P], None),
        "hpg_create_batch": ([P, I32, ctypes.c_int, P], ctypes.c_int),
        "hpg_destroy_batch": ([P], None),
        "hpg_batch_set_data": ([P, P, P, SZ], ctypes.c_int),
        "hpg_batch_solve": ([P, P, P, P, P, P], ctypes.c_int),
        "hpg_batch_op_setup": ([P, P, D, D, I32, P], ctypes.c_int),
        "hpg_batch_op_apply_G": ([P, P, P, P], ctypes.c_int),
        "hpg_batch_set_kernel_timing": ([P, ctypes.c_char_p], ctypes.c_int),
        "hpg_batch_kernel_time": ([P, ctypes.c_char_p, P, P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(st, allow=(OK,)):
    if st not in allow:
        raise HpgError(st, load().hpg_last_error().decode())
    return st


def _dptr(a, n=None):
    """Pointer of a contiguous NumPy array (host)."""
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _tptr(t):
    """Device pointer of a contiguous torch tensor."""
    assert t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def default_opts(**kw):
    o = SolveOpts()
    load().hpg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Mesh:
    """Tensor mesh; ``degree`` (one value per cell, direction 0 fastest)
    selects per-cell degrees (obstacle only; ``p`` is then ignored)."""

    def __init__(self, dim, ncells, p, constraint=OBSTACLE, breaks=None, degree=None):
        lib = load()
        vals = [int(v) for v in ncells] + [1] * max(0, 3 - len(ncells))
        nc = (ctypes.c_int32 * len(vals))(*vals)
        self._keep = []
        bp = None
        if breaks is not None:
            arrs = [np.ascontiguousarray(b, dtype=np.float64) for b in breaks]
            self._keep = arrs
            ptrs = (ctypes.c_void_p * 3)(*([a.ctypes.data for a in arrs] + [None] * (3 - len(arrs))))
            self._keep.append(ptrs)
            bp = ctypes.cast(ptrs, ctypes.c_void_p)
        dp = None
        if degree is not None:
            deg = np.ascontiguousarray(np.asarray(degree).reshape(-1), dtype=np.int32)
            self._keep.append(deg)
            dp = ctypes.c_void_p(deg.ctypes.data)
            p = 0
        h = ctypes.c_void_p()
        _check(lib.hpg_create_mesh(dim, ctypes.cast(nc, ctypes.c_void_p), bp, dp, p, constraint,
                                   ctypes.byref(h)))
        self.h = h
        inf = MeshInfo()
        _check(lib.hpg_get_mesh_info(h, ctypes.byref(inf)))
        self.info = inf
        self.dim, self.p, self.q, self.P = inf.dim, inf.p, inf.q, inf.P
        self.n_u, self.n_psi, self.n_qp, self.n_cells = inf.n_u, inf.n_psi, inf.n_qp, inf.n_cells

    def footprint(self, precision=FP64):
        """Upper estimate of the device bytes one solve on this mesh allocates."""
        b = ctypes.c_uint64(0)
        _check(load().hpg_problem_footprint(self.h, precision, ctypes.byref(b)))
        return b.value

    def quadrature_points(self):
        x = np.zeros((self.n_qp, self.dim))
        _check(load().hpg_quadrature_points(self.h, _dptr(x)))
        return x

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpg_destroy_mesh(self.h)
            self.h = None


class Problem:
    def __init__(self, mesh, device=0):
        self.mesh = mesh
        h = ctypes.c_void_p()
        _check(load().hpg_create_problem(mesh.h, device, ctypes.byref(h)))
        self.h = h

    def set_forcing(self, f_qp):
        f = np.ascontiguousarray(f_qp, dtype=np.float64).reshape(-1)
        _check(load().hpg_set_forcing(self.h, _dptr(f), f.size))

    def set_obstacle(self, phi_qp):
        f = np.ascontiguousarray(phi_qp, dtype=np.float64).reshape(-1)
        _check(load().hpg_set_obstacle(self.h, _dptr(f), f.size))

    def _point_fn(self, setter, fn):
        dim = self.mesh.dim

        def cb(x, ctx):
            return float(fn(np.ctypeslib.as_array(x, shape=(dim,)).copy()))

        c = POINT_FN(cb)
        _check(setter(self.h, c, None))

    def set_forcing_fn(self, fn):
        """f from a Python callable of one point (array of dim coordinates),
        evaluated by the library at every quadrature point."""
        self._point_fn(load().hpg_set_forcing_fn, fn)

    def set_obstacle_fn(self, fn):
        self._point_fn(load().hpg_set_obstacle_fn, fn)

    def solve(self, opts=None, want_lambda=False, warm=None):
        """warm = (u_k0, psi_k0, k0): resume after k0 proximal steps."""
        m = self.mesh
        u = np.zeros(m.n_u)
        psi = np.zeros(m.n_psi)
        lam = np.zeros(m.n_psi) if want_lambda else None
        st = SolveStats()
        o = opts if opts is not None else default_opts()
        keep = None
        if warm is not None:
            wu = np.ascontiguousarray(warm[0], dtype=np.float64)
            wp = np.ascontiguousarray(warm[1], dtype=np.float64)
            keep = (wu, wp)
            o = SolveOpts.from_buffer_copy(o)
            o.warm_u, o.warm_psi, o.k0 = wu.ctypes.data, wp.ctypes.data, int(warm[2])
        rc = load().hpg_solve(self.h, ctypes.byref(o), _dptr(u), _dptr(psi),
                              _dptr(lam) if lam is not None else None, ctypes.byref(st))
        del keep
        _check(rc, allow=(OK, NOT_CONVERGED))
        return u, psi, lam, st

    def solve_device(self, d_u, d_psi, opts=None, stream=None):
        st = SolveStats()
        o = opts if opts is not None else default_opts()
        rc = load().hpg_solve_device(self.h, ctypes.byref(o), _tptr(d_u), _tptr(d_psi),
                                     ctypes.c_void_p(stream) if stream else None, ctypes.byref(st))
        _check(rc, allow=(OK, NOT_CONVERGED))
        return st

    # operator-level calls on torch device tensors
    def op_setup(self, d_psi, alpha, beta=0.0, precision=FP64, stream=None):
        _check(load().hpg_op_setup(self.h, _tptr(d_psi), alpha, beta, precision,
                                   ctypes.c_void_p(stream) if stream else None))

    def op_apply_G(self, x, y, stream=None):
        _check(load().hpg_op_apply_G(self.h, _tptr(x), _tptr(y),
                                     ctypes.c_void_p(stream) if stream else None))

    def op_apply_prec(self, r, z, stream=None):
        _check(load().hpg_op_apply_prec(self.h, _tptr(r), _tptr(z),
                                        ctypes.c_void_p(stream) if stream else None))

    def op_minres(self, b, x, rtol, max_iters, stream=None):
        it = ctypes.c_int32(0)
        _check(load().hpg_op_minres(self.h, _tptr(b), _tptr(x), rtol, max_iters, ctypes.byref(it),
                                    ctypes.c_void_p(stream) if stream else None))
        return it.value

    def op_residual(self, u, psi, psi_prev, alpha, R, stream=None):
        _check(load().hpg_op_residual(self.h, _tptr(u), _tptr(psi), _tptr(psi_prev), alpha,
                                      _tptr(R), ctypes.c_void_p(stream) if stream else None))

    def op_residual_noalloc(self, u, psi, psi_prev, alpha, R, stream=None):
        """hpg_op_residual without allocation; returns (||R_u||^2, ||R_psi||^2)."""
        n2 = np.zeros(2)
        _check(load().hpg_op_residual_noalloc(self.h, _tptr(u), _tptr(psi), _tptr(psi_prev),
                                              alpha, _tptr(R), _dptr(n2),
                                              ctypes.c_void_p(stream) if stream else None))
        return float(n2[0]), float(n2[1])

    def l2_diff(self, a, b, stream=None):
        """(||a_h - b_h||_L2, ||b_h||_L2) for device u vectors a, b."""
        d = ctypes.c_double(0.0)
        nb = ctypes.c_double(0.0)
        _check(load().hpg_l2_diff(self.h, _tptr(a), _tptr(b), ctypes.byref(d), ctypes.byref(nb),
                                  ctypes.c_void_p(stream) if stream else None))
        return d.value, nb.value

    def set_kernel_timing(self, group):
        """group: None (off), "all", or one kernel group name."""
        _check(load().hpg_set_kernel_timing(self.h, group.encode() if group else None))

    def kernel_time(self, group):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(load().hpg_kernel_time(self.h, group.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpg_destroy_problem(self.h)
            self.h = None


class Batch:
    """Obstacle problems on one mesh solved together in nbatch slots
    (hpg_batch_*): every Krylov/Newton step of the requests in the slots is
    one launch, and a slot whose request finishes takes the next one."""

    def __init__(self, mesh, nbatch, device=0):
        self.mesh = mesh
        self.nb = int(nbatch)
        self.nreq = self.nb
        h = ctypes.c_void_p()
        _check(load().hpg_create_batch(mesh.h, self.nb, device, ctypes.byref(h)))
        self.h = h

    def set_data(self, f_qp, phi_qp):
        """f and phi of every request at the mesh's quadrature points,
        shape (nrequests, n_qp) (request-major; any number of requests)."""
        f = np.ascontiguousarray(f_qp, dtype=np.float64).reshape(-1)
        ph = np.ascontiguousarray(phi_qp, dtype=np.float64).reshape(-1)
        _check(load().hpg_batch_set_data(self.h, _dptr(f), _dptr(ph), f.size))
        self.nreq = f.size // self.mesh.n_qp

    def solve(self, opts=None, want_lambda=False):
        m, nb = self.mesh, self.nreq
        u = np.zeros((nb, m.n_u))
        psi = np.zeros((nb, m.n_psi))
        lam = np.zeros((nb, m.n_psi)) if want_lambda else None
        st = (SolveStats * nb)()
        o = opts if opts is not None else default_opts()
        rc = load().hpg_batch_solve(self.h, ctypes.byref(o), _dptr(u), _dptr(psi),
                                    _dptr(lam) if lam is not None else None,
                                    ctypes.cast(st, ctypes.c_void_p))
        _check(rc, allow=(OK, NOT_CONVERGED))
        return u, psi, lam, list(st)

    def op_setup(self, d_psi, alpha, beta=0.0, precision=FP64, stream=None):
        _check(load().hpg_batch_op_setup(self.h, _tptr(d_psi), alpha, beta, precision,
                                         ctypes.c_void_p(stream) if stream else None))

    def op_apply_G(self, x, y, stream=None):
        _check(load().hpg_batch_op_apply_G(self.h, _tptr(x), _tptr(y),
                                           ctypes.c_void_p(stream) if stream else None))

    def set_kernel_timing(self, group):
        _check(load().hpg_batch_set_kernel_timing(self.h, group.encode() if group else None))

    def kernel_time(self, group):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(load().hpg_batch_kernel_time(self.h, group.encode(), ctypes.byref(n),
                                            ctypes.byref(ms)))
        return n.value, ms.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpg_destroy_batch(self.h)
            self.h = None


class Server:
    """Continuous batching of independent solves on one device (hpg_server_*)."""

    def __init__(self, device=0, hbm_budget=0, max_slots=4):
        h = ctypes.c_void_p()
        _check(load().hpg_server_create(device, int(hbm_budget), max_slots, ctypes.byref(h)))
        self.h = h
        self._sizes = {}

    def submit(self, mesh, f_qp, phi_qp, opts=None):
        f = np.ascontiguousarray(f_qp, dtype=np.float64).reshape(-1)
        ph = np.ascontiguousarray(phi_qp, dtype=np.float64).reshape(-1)
        if f.size != mesh.n_qp or ph.size != mesh.n_qp:
            raise ValueError("f and phi must be given at the mesh's n_qp quadrature points")
        t = ctypes.c_uint64(0)
        o = opts if opts is not None else default_opts()
        _check(load().hpg_server_submit(self.h, mesh.h, _dptr(f), _dptr(ph), ctypes.byref(o),
                                        ctypes.byref(t)))
        self._sizes[t.value] = (mesh.n_u, mesh.n_psi)
        return t.value

    def _result(self, fn, ticket):
        sizes = self._sizes.get(ticket)
        u = np.zeros(sizes[0]) if sizes else None
        psi = np.zeros(sizes[1]) if sizes else None
        st = SolveStats()
        info = RequestInfo()
        rc = fn(self.h, ticket, _dptr(u) if sizes else None, _dptr(psi) if sizes else None,
                ctypes.byref(st), ctypes.byref(info))
        if rc == PENDING:
            return None
        self._sizes.pop(ticket, None)
        _check(rc, allow=(OK, NOT_CONVERGED))
        return u, psi, st, info

    def poll(self, ticket):
        """None while pending, else (u, psi, SolveStats, RequestInfo)."""
        return self._result(load().hpg_server_poll, ticket)

    def wait(self, ticket):
        return self._result(load().hpg_server_wait, ticket)

    def stats(self):
        s = ServingStats()
        _check(load().hpg_server_stats(self.h, ctypes.byref(s)))
        return s

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hpg_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
