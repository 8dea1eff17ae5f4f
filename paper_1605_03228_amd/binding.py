"""ctypes binding of the iHDG C ABI (include/ihdg.h): argument marshalling only.

PyTorch provides the device memory (workspace, scratch, coefficient arrays,
solution copies) and the stream; every computation runs in libihdg.so.  There
is no fallback: if the library is missing, every call raises.
"""
import ctypes as C
import os

import torch

TRANSPORT, SHALLOW_WATER, CD = 0, 1, 2
FP64, MIXED = 0, 1
_STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "workspace or scratch too small",
           4: "HIP error", 5: "singular local matrix", 6: "diverged", 7: "max iterations"}
OK, ERR_DIVERGED, ERR_MAXITER = 0, 6, 7


class IhdgError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"ihdg status {status} ({_STATUS.get(status, '?')}): {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class Sizes(C.Structure):
    _fields_ = [("n_el", C.c_int64), ("n_face", C.c_int64), ("np", C.c_int32), ("m", C.c_int32),
                ("n_loc", C.c_int32), ("nq", C.c_int32), ("nfq", C.c_int32), ("nfp", C.c_int32),
                ("n_in", C.c_int32), ("m_f", C.c_int32)]


class Coeffs(C.Structure):
    _fields_ = [("beta_q", C.c_void_p), ("divbeta_q", C.c_void_p), ("bn_fq", C.c_void_p),
                ("sigma_el", C.c_void_p), ("f_q", C.c_void_p), ("g_fq", C.c_void_p),
                ("beta_const", C.c_double * 3), ("sigma_const", C.c_double), ("kappa", C.c_double),
                ("nu", C.c_double), ("Phi", C.c_double), ("f0", C.c_double), ("gamma", C.c_double),
                ("mass_coef", C.c_double), ("tau_gamma", C.c_double)]


class Options(C.Structure):
    _fields_ = [("prec", C.c_int), ("check_every", C.c_int32), ("max_iters", C.c_int32),
                ("krylov_restart", C.c_int32), ("inner_rtol", C.c_double), ("use_graph", C.c_int32),
                ("force_per_element", C.c_int32), ("block_waves", C.c_int32), ("time_stepping", C.c_int32),
                ("transport_flux", C.c_int32), ("krylov_method", C.c_int32), ("mixed_period", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("fp64_sweeps", C.c_int64), ("fp32_sweeps", C.c_int64), ("outer_steps", C.c_int32),
                ("krylov_iters", C.c_int32), ("shared_operator", C.c_int32), ("kernel_waves", C.c_int32)]


_LIB = None


def library_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libihdg.so")


class BatchResult(C.Structure):
    _fields_ = [("tag", C.c_int64), ("status", C.c_int32), ("iters", C.c_int32), ("final_rel", C.c_double)]


EXPORTS = ["ihdg_sizes", "ihdg_quadrature_points", "ihdg_footprint", "ihdg_setup", "ihdg_sweep",
           "ihdg_solve", "ihdg_residual", "ihdg_get_solution", "ihdg_set_solution", "ihdg_set_stream",
           "ihdg_get_stats", "ihdg_last_error", "ihdg_status_string", "ihdg_destroy",
           "ihdg_batch_footprint", "ihdg_batch_create", "ihdg_batch_add", "ihdg_batch_round",
           "ihdg_batch_poll", "ihdg_batch_use_graphs", "ihdg_batch_destroy", "ihdg_batch_last_error",
           "ihdg_time_step", "ihdg_node_points", "ihdg_setup_noalloc", "ihdg_sweep32"]


def load():
    """Load libihdg.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.ihdg_sizes.argtypes = [P(Mesh), C.c_int32, C.c_int, P(Sizes)]
    lib.ihdg_quadrature_points.argtypes = [P(Mesh), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.ihdg_footprint.argtypes = [P(Mesh), C.c_int32, C.c_int, P(Coeffs), P(Options), P(C.c_size_t),
                                   P(C.c_size_t)]
    lib.ihdg_setup.argtypes = [P(Mesh), C.c_int32, C.c_int, P(Coeffs), P(Options), C.c_void_p, C.c_size_t,
                               C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]
    lib.ihdg_setup_noalloc.argtypes = [P(Mesh), C.c_int32, C.c_int, P(Coeffs), P(Options), C.c_void_p, C.c_size_t,
                                       C.c_void_p, P(C.c_void_p)]
    lib.ihdg_sweep.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
    lib.ihdg_sweep32.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
    lib.ihdg_solve.argtypes = [C.c_void_p, C.c_double, P(C.c_int32), P(C.c_double), P(C.c_double)]
    lib.ihdg_residual.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ihdg_get_solution.argtypes = [C.c_void_p, C.c_void_p]
    lib.ihdg_set_solution.argtypes = [C.c_void_p, C.c_void_p]
    lib.ihdg_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    lib.ihdg_get_stats.argtypes = [C.c_void_p, P(Stats)]
    lib.ihdg_last_error.argtypes = [C.c_void_p]
    lib.ihdg_last_error.restype = C.c_char_p
    lib.ihdg_status_string.argtypes = [C.c_int]
    lib.ihdg_status_string.restype = C.c_char_p
    lib.ihdg_destroy.argtypes = [C.c_void_p]
    lib.ihdg_destroy.restype = None
    lib.ihdg_batch_footprint.argtypes = [C.c_int32, C.c_int64, P(C.c_size_t)]
    lib.ihdg_batch_create.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]
    lib.ihdg_batch_add.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]
    lib.ihdg_batch_round.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32)]
    lib.ihdg_batch_poll.argtypes = [C.c_void_p, P(BatchResult), C.c_int32, P(C.c_int32)]
    lib.ihdg_batch_use_graphs.argtypes = [C.c_void_p, C.c_int32]
    lib.ihdg_time_step.argtypes = [C.c_void_p, C.c_int32]
    lib.ihdg_node_points.argtypes = [P(Mesh), C.c_int32, C.c_void_p, C.c_void_p]
    lib.ihdg_batch_destroy.argtypes = [C.c_void_p]
    lib.ihdg_batch_destroy.restype = None
    lib.ihdg_batch_last_error.argtypes = [C.c_void_p]
    lib.ihdg_batch_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("ihdg_last_error", "ihdg_status_string", "ihdg_destroy", "ihdg_batch_destroy",
                        "ihdg_batch_last_error"):
            getattr(lib, name).restype = C.c_int
    _LIB = lib
    return lib


def _mesh(n, lo=None, hi=None):
    m = Mesh()
    m.dim = len(n)
    for a in range(3):
        m.n[a] = int(n[a]) if a < len(n) else 1
        m.lo[a] = float(lo[a]) if lo is not None and a < len(n) else 0.0
        m.hi[a] = float(hi[a]) if hi is not None and a < len(n) else 1.0
    return m


def _check(st, ctx=None, batch=None):
    if st != OK:
        msg = load().ihdg_last_error(ctx).decode() if ctx else ""
        if batch:
            msg = load().ihdg_batch_last_error(batch).decode()
        raise IhdgError(st, msg)


def sizes(n, order, pde, lo=None, hi=None):
    s = Sizes()
    _check(load().ihdg_sizes(C.byref(_mesh(n, lo, hi)), order, pde, C.byref(s)))
    return {k: getattr(s, k) for k, _ in Sizes._fields_}


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def quadrature_points(n, order, lo=None, hi=None, device="cuda"):
    """(xq [n_el, nq, dim], xfq [n_face, nfq, dim]) as FP64 device tensors."""
    s = sizes(n, order, TRANSPORT if len(n) == 3 else TRANSPORT, lo, hi)
    dim = len(n)
    xq = torch.empty((s["n_el"], s["nq"], dim), dtype=torch.float64, device=device)
    xfq = torch.empty((s["n_face"], s["nfq"], dim), dtype=torch.float64, device=device)
    _check(load().ihdg_quadrature_points(C.byref(_mesh(n, lo, hi)), order, C.c_void_p(xq.data_ptr()),
                                         C.c_void_p(xfq.data_ptr()), _stream(device)))
    return xq, xfq


def node_points(n, order, lo=None, hi=None, device="cuda"):
    """GLL node coordinates of every element, [n_el, np, dim] FP64 on the device."""
    s = sizes(n, order, TRANSPORT, lo, hi)
    x = torch.empty((s["n_el"], s["np"], len(n)), dtype=torch.float64, device=device)
    _check(load().ihdg_node_points(C.byref(_mesh(n, lo, hi)), order, C.c_void_p(x.data_ptr()), _stream(device)))
    torch.cuda.current_stream(device).synchronize()
    return x


def _ptr(t):
    if t is None:
        return None
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _coeffs(c):
    cf = Coeffs()
    for k in ("beta_q", "divbeta_q", "bn_fq", "sigma_el", "f_q", "g_fq"):
        setattr(cf, k, _ptr(c.get(k)))
    bc = c.get("beta_const", (0.0, 0.0, 0.0))
    for a in range(3):
        cf.beta_const[a] = float(bc[a]) if a < len(bc) else 0.0
    for k in ("sigma_const", "kappa", "nu", "Phi", "f0", "gamma", "mass_coef", "tau_gamma"):
        setattr(cf, k, float(c.get(k, 0.0)))
    return cf


def _options(prec=FP64, check_every=16, max_iters=0, krylov_restart=0, inner_rtol=0.0, use_graph=True,
             force_per_element=False, block_waves=0, flux="upwind", time_stepping=False, krylov="gmres",
             mixed_period=0):
    """krylov = "gmres" (GMRES(krylov_restart) when krylov_restart > 0) or
    "bicgstab" (selects the Krylov solve by itself)."""
    o = Options()
    o.prec = prec
    o.check_every = check_every
    o.max_iters = max_iters
    o.krylov_method = {"gmres": 0, "bicgstab": 1}[krylov]
    o.krylov_restart = max(krylov_restart, 1) if krylov == "bicgstab" else krylov_restart
    o.inner_rtol = inner_rtol
    o.use_graph = 1 if use_graph else 0
    o.force_per_element = 1 if force_per_element else 0
    o.block_waves = block_waves
    o.transport_flux = {"upwind": 0, "npc": 1}[flux]
    o.time_stepping = 1 if time_stepping else 0
    o.mixed_period = mixed_period
    return o


def footprint(n, order, pde, coeffs=None, lo=None, hi=None, **opts):
    pb, sb = C.c_size_t(), C.c_size_t()
    cf = _coeffs(coeffs) if coeffs is not None else None
    _check(load().ihdg_footprint(C.byref(_mesh(n, lo, hi)), order, pde, C.byref(cf) if cf else None,
                                 C.byref(_options(**opts)), C.byref(pb), C.byref(sb)))
    return pb.value, sb.value


class Solver:
    """One iHDG problem resident on the GPU (owns its torch-allocated workspace)."""

    def __init__(self, n, order, pde, coeffs, lo=None, hi=None, device="cuda", noalloc=False, **opts):
        """noalloc: set up through ihdg_setup_noalloc (the library's own device
        scratch; only the workspace is allocated here)."""
        lib = load()
        self.lib, self.device = lib, torch.device(device)
        self.n, self.order, self.pde = tuple(n), order, pde
        self.sz = sizes(n, order, pde, lo, hi)
        mesh = _mesh(n, lo, hi)
        cf = _coeffs(coeffs)
        op = _options(**opts)
        pb, sb = C.c_size_t(), C.c_size_t()
        _check(lib.ihdg_footprint(C.byref(mesh), order, pde, C.byref(cf), C.byref(op), C.byref(pb), C.byref(sb)))
        self.workspace_bytes, self.scratch_bytes = pb.value, sb.value
        self.workspace = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        # the library works on a stream of its own (default priority); torch's
        # current stream has produced the coefficient arrays, so wait for it
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        ctx = C.c_void_p()
        if noalloc:
            st = lib.ihdg_setup_noalloc(C.byref(mesh), order, pde, C.byref(cf), C.byref(op),
                                        C.c_void_p(self.workspace.data_ptr()), pb.value,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        else:
            scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
            st = lib.ihdg_setup(C.byref(mesh), order, pde, C.byref(cf), C.byref(op),
                                C.c_void_p(self.workspace.data_ptr()), pb.value, C.c_void_p(scratch.data_ptr()),
                                sb.value, C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
            del scratch
        _check(st)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            self.lib.ihdg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1, norms=False):
        out = (C.c_double * 2)()
        _check(self.lib.ihdg_sweep(self.ctx, n, out if norms else None), self.ctx)
        return (out[0], out[1]) if norms else None

    def sweep32(self, n=1, norms=False):
        """n FP32 correction sweeps of a mixed-precision context (for timing)."""
        out = (C.c_double * 2)()
        _check(self.lib.ihdg_sweep32(self.ctx, n, out if norms else None), self.ctx)
        return (out[0], out[1]) if norms else None

    def solve(self, tol, raise_on_fail=False):
        it, inc, dfc = C.c_int32(), C.c_double(), C.c_double()
        st = self.lib.ihdg_solve(self.ctx, tol, C.byref(it), C.byref(inc), C.byref(dfc))
        if st not in (OK, ERR_DIVERGED, ERR_MAXITER) or (raise_on_fail and st != OK):
            _check(st, self.ctx)
        return {"status": st, "iters": it.value, "incr": inc.value, "defect": dfc.value, **self.stats()}

    def residual(self):
        out = (C.c_double * 2)()
        _check(self.lib.ihdg_residual(self.ctx, out), self.ctx)
        return out[0], out[1]

    def time_step(self, scheme="cn"):
        """Form the next implicit step's right-hand side from the current iterate
        (which stays as the warm start): scheme "be" or "cn"."""
        _check(self.lib.ihdg_time_step(self.ctx, {"be": 0, "cn": 1}[scheme]), self.ctx)

    def get_solution(self):
        u = torch.empty((self.sz["n_el"], self.sz["m"], self.sz["np"]), dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        _check(self.lib.ihdg_get_solution(self.ctx, C.c_void_p(u.data_ptr())), self.ctx)
        self.stream.synchronize()
        return u

    def set_solution(self, u):
        u = u.to(device=self.device, dtype=torch.float64).contiguous()
        torch.cuda.current_stream(self.device).synchronize()
        _check(self.lib.ihdg_set_solution(self.ctx, C.c_void_p(u.data_ptr())), self.ctx)
        self.stream.synchronize()

    def stats(self):
        s = Stats()
        _check(self.lib.ihdg_get_stats(self.ctx, C.byref(s)), self.ctx)
        return {k: getattr(s, k) for k, _ in Stats._fields_}


class Batch:
    """Continuous batching of Solver contexts (ihdg_batch_*): members join between
    rounds, every round advances each member by `sweeps` sweeps of its own solve
    with one launch per group of same-shaped members, finished members are
    reported by poll()."""

    def __init__(self, max_members=256, max_blocks=1 << 20, device="cuda", use_graphs=True):
        lib = load()
        self.lib, self.device = lib, torch.device(device)
        nb = C.c_size_t()
        _check(lib.ihdg_batch_footprint(max_members, max_blocks, C.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        _check(lib.ihdg_batch_create(max_members, max_blocks, C.c_void_p(self.workspace.data_ptr()), nb.value,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        _check(lib.ihdg_batch_use_graphs(h, 1 if use_graphs else 0))
        self.members = {}
        self.max_members = max_members

    def add(self, solver, tol, tag):
        solver.stream.synchronize()
        _check(self.lib.ihdg_batch_add(self.h, solver.ctx, tol, int(tag)))
        self.members[int(tag)] = solver

    def round(self, sweeps=16):
        n = C.c_int32()
        _check(self.lib.ihdg_batch_round(self.h, sweeps, C.byref(n)), batch=self.h)
        return n.value

    def poll(self):
        buf = (BatchResult * self.max_members)()
        n = C.c_int32()
        _check(self.lib.ihdg_batch_poll(self.h, buf, self.max_members, C.byref(n)))
        self.stream.synchronize()
        out = []
        for i in range(n.value):
            r = buf[i]
            out.append({"tag": r.tag, "status": r.status, "iters": r.iters, "final_rel": r.final_rel,
                        "solver": self.members.pop(r.tag, None)})
        return out

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()
            self.lib.ihdg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
