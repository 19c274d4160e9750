"""Python binding of libmgcut.so, the MI355X cut-cell multigrid library.

Argument marshalling only: every step of the solver runs in the HIP library.
Device arrays are torch tensors on the current HIP device (PyTorch supplies
device memory and the stream); importing fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgcut.so")

MG_OK = 0
STATUS = {0: "MG_OK", -1: "MG_ERR_INVALID_ARG", -2: "MG_ERR_GEOMETRY", -3: "MG_ERR_SINGULAR",
          -4: "MG_ERR_NO_CONVERGENCE", -5: "MG_ERR_DIVERGED", -6: "MG_ERR_OOM", -7: "MG_ERR_HIP",
          -8: "MG_ERR_UNSUPPORTED"}
BC = {"D": 0, "N": 1, "R": 2, "P": 3}
FP64, MIXED = 0, 1
CYCLE_V, CYCLE_FMG = 0, 1


class MGError(RuntimeError):
    def __init__(self, code, where, detail=""):
        super().__init__("%s failed: %s (%d) %s" % (where, STATUS.get(code, "?"), code, detail))
        self.code = code


class mg_segment(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_double * 8), ("bc", ctypes.c_int),
                ("alpha1", ctypes.c_double), ("alpha2", ctypes.c_double)]


class mg_curve(ctypes.Structure):
    _fields_ = [("n_seg", ctypes.c_int), ("seg", ctypes.POINTER(mg_segment))]


class mg_grid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("h", ctypes.c_double),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int)]


class mg_options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("omega", ctypes.c_double), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("n_levels", ctypes.c_int), ("min_coarse", ctypes.c_int),
                ("precision", ctypes.c_int), ("max_iters", ctypes.c_int), ("cycle", ctypes.c_int),
                ("degree", ctypes.c_int), ("w_min", ctypes.c_double), ("colouring", ctypes.c_int),
                ("split_cells", ctypes.c_longlong), ("small_cells", ctypes.c_longlong),
                ("split_b_sep", ctypes.c_int), ("seg_max", ctypes.c_int), ("seg_whole", ctypes.c_int),
                ("pair_sweeps", ctypes.c_int)]


class mg_info(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("nx", ctypes.c_int * 16), ("ny", ctypes.c_int * 16),
                ("n_active", ctypes.c_int * 16), ("n_plg", ctypes.c_int * 16), ("n_sep", ctypes.c_int * 16),
                ("sweep_words", ctypes.c_longlong * 16), ("n_sfv", ctypes.c_longlong * 16),
                ("n_face", ctypes.c_int), ("n_irr", ctypes.c_int), ("nnz_plg", ctypes.c_longlong),
                ("device_bytes", ctypes.c_longlong), ("setup_seconds", ctypes.c_double),
                ("cond_A22", ctypes.c_double * 16), ("setup_stage_seconds", ctypes.c_double * 6),
                ("n_pair_sfv", ctypes.c_longlong * 16)]


F_BATCH = ctypes.CFUNCTYPE(None, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)
G_BATCH = ctypes.CFUNCTYPE(None, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)
SMOOTH_JACOBI, SMOOTH_MULTICOLOUR = 0, 1


class mg_server_options(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int), ("hbm_budget", ctypes.c_longlong)]


class mg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("p50_solve_s", ctypes.c_double), ("p99_solve_s", ctypes.c_double),
                ("solves_per_s", ctypes.c_double), ("resident_bytes", ctypes.c_longlong),
                ("resident_problems", ctypes.c_int), ("evictions", ctypes.c_int), ("sweep_gbs", ctypes.c_double)]


def load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmgcut.so is not built (run __graft_entry__.build() or "
                          "python paper_2601_02975_amd/build.py)")
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it
    # first makes the dynamic loader reuse it for libmgcut.so, so one process
    # holds a single HIP runtime and torch tensors are valid device pointers.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    pI, pD, pLL = ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(LL)
    sig = {
        "mg_default_options": [ctypes.POINTER(mg_options)],
        "mg_setup": [ctypes.POINTER(mg_grid), I, ctypes.POINTER(mg_curve), D, D, D, ctypes.POINTER(mg_options), P,
                     ctypes.POINTER(P)],
        "mg_solve": [P, P, P, P, D, P, pI, pD],
        "mg_rhs": [P, P, P, P, P],
        "mg_vcycle": [P, P, P, P],
        "mg_smooth": [P, I, P, P, P],
        "mg_smooth32": [P, I, P, P, P],
        "mg_restrict": [P, I, I, P, P, P, P],
        "mg_prolong": [P, I, I, P, P, P],
        "mg_residual": [P, I, P, P, P, pD, P],
        "mg_query": [P, ctypes.POINTER(mg_info)],
        "mg_export_level": [P, I, pI, pI, pLL, pI, pI, pD, pD],
        "mg_cell_quadrature": [P, pI, pLL, pI, pLL, pD, pD, pD],
        "mg_boundary_quadrature": [P, pI, pLL, pLL, pD, pD, pD, pD, pD, pI, pD, pD],
        "mg_destroy": [P],
        "mg_project_rhs": [P, F_BATCH, G_BATCH, P, I, P, P, P],
        "mg_kernel_timing": [P, I, pI, pD],
        "mg_set_eager": [P, I],
        "mg_server_create": [ctypes.POINTER(mg_server_options), ctypes.POINTER(P)],
        "mg_server_add_problem": [P, ctypes.POINTER(mg_grid), I, ctypes.POINTER(mg_curve), D, D, D,
                                  ctypes.POINTER(mg_options), pI],
        "mg_server_submit": [P, I, P, P, P, D, ctypes.POINTER(ctypes.c_ulonglong)],
        "mg_server_poll": [P, ctypes.c_ulonglong, pI, pI, pI, pD, pD],
        "mg_server_wait": [P, ctypes.c_ulonglong, pI, pI, pD, pD],
        "mg_server_get_stats": [P, ctypes.POINTER(mg_server_stats)],
        "mg_server_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mg_error_string.argtypes = [ctypes.c_int]
    lib.mg_error_string.restype = ctypes.c_char_p
    lib.mg_last_error.argtypes = []
    lib.mg_last_error.restype = ctypes.c_char_p
    lib.mg_server_request_error.argtypes = [P, ctypes.c_ulonglong]
    lib.mg_server_request_error.restype = ctypes.c_char_p
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(code, where):
    if code != MG_OK:
        raise MGError(code, where, lib().mg_last_error().decode(errors="replace"))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong))


def _curves(curves):
    """mg_curve array for a list of curves of workloads.Segment; the segment
    arrays are returned too (they must outlive the call)."""
    keep = []
    carr = (mg_curve * len(curves))()
    for k, curve in enumerate(curves):
        segs = (mg_segment * len(curve))()
        for s, sg in enumerate(curve):
            segs[s].kind = {"line": 0, "arc": 1, "cubic": 2}[sg.kind]
            for t in range(8):
                segs[s].p[t] = float(sg.p[t]) if t < len(sg.p) else 0.0
            segs[s].bc = BC[sg.bc]
            segs[s].alpha1 = float(sg.alpha1)
            segs[s].alpha2 = float(sg.alpha2)
        keep.append(segs)
        carr[k].n_seg = len(curve)
        carr[k].seg = ctypes.cast(segs, ctypes.POINTER(mg_segment))
    return carr, keep


def _options(eps, omega, nu, n_levels, min_coarse, precision, max_iters, cycle=0, **extra):
    """mg_options from the library's defaults; extra: degree, w_min,
    colouring, split_cells, small_cells, split_b_sep."""
    opt = mg_options()
    lib().mg_default_options(ctypes.byref(opt))
    opt.eps, opt.omega, opt.nu1, opt.nu2 = eps, omega, nu[0], nu[1]
    opt.n_levels, opt.min_coarse, opt.precision, opt.max_iters = n_levels, min_coarse, precision, max_iters
    opt.cycle = cycle
    for k, v in extra.items():
        if v is not None:
            setattr(opt, k, v)
    return opt


class Solver:
    """A handle of the C library for one problem (grid, curves, a, b, c)."""

    def __init__(self, grid, curves, a, b, c, eps=0.08, omega=0.5, nu=(3, 3), n_levels=0, min_coarse=16,
                 precision=FP64, max_iters=100, cycle=0, **extra):
        L = lib()
        carr, self._segs = _curves(curves)
        g = mg_grid(grid.x0, grid.y0, grid.h, grid.nx, grid.ny)
        opt = _options(eps, omega, nu, n_levels, min_coarse, precision, max_iters, cycle, **extra)
        self.grid = grid
        self.curves = curves
        self.nx, self.ny = grid.nx, grid.ny
        h = ctypes.c_void_p()
        _check(L.mg_setup(ctypes.byref(g), len(curves), carr, a, b, c, ctypes.byref(opt), _stream(),
                          ctypes.byref(h)), "mg_setup")
        self.h = h
        self.info = self.query()

    def close(self):
        if getattr(self, "h", None):
            lib().mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout helpers ----------------------------------------------------------
    def padded_shape(self, level=0):
        return (self.info["ny"][level] + 4, self.info["nx"][level] + 4)

    def empty(self, level=0, dtype=None):
        import torch
        return torch.zeros(self.padded_shape(level), dtype=dtype or torch.float64, device="cuda")

    # -- entry points ------------------------------------------------------------
    def solve(self, f, g, u, tol=1e-10):
        it = ctypes.c_int()
        rel = ctypes.c_double()
        code = lib().mg_solve(self.h, _ptr(f), _ptr(g), _ptr(u), tol, _stream(), ctypes.byref(it), ctypes.byref(rel))
        if code not in (MG_OK, -4, -5):
            _check(code, "mg_solve")
        return it.value, rel.value, code

    def rhs(self, f, g, b):
        _check(lib().mg_rhs(self.h, _ptr(f), _ptr(g), _ptr(b), _stream()), "mg_rhs")

    def vcycle(self, b, u):
        _check(lib().mg_vcycle(self.h, _ptr(b), _ptr(u), _stream()), "mg_vcycle")

    def smooth(self, level, b, u):
        _check(lib().mg_smooth(self.h, level, _ptr(b), _ptr(u), _stream()), "mg_smooth")

    def smooth32(self, level, b, u):
        _check(lib().mg_smooth32(self.h, level, _ptr(b), _ptr(u), _stream()), "mg_smooth32")

    def restrict(self, level, b, u, bc):
        """bc (level + 1) = R (b - A u) (level); FP64 or FP32 tensors."""
        import torch
        prec = FP64 if b.dtype == torch.float64 else MIXED
        _check(lib().mg_restrict(self.h, level, prec, _ptr(b), _ptr(u), _ptr(bc), _stream()), "mg_restrict")

    def prolong(self, level, ec, u):
        """u (level) += P ec (level + 1); FP64 or FP32 tensors."""
        import torch
        prec = FP64 if u.dtype == torch.float64 else MIXED
        _check(lib().mg_prolong(self.h, level, prec, _ptr(ec), _ptr(u), _stream()), "mg_prolong")

    def residual(self, level, b, u, r=None):
        nrm = ctypes.c_double()
        _check(lib().mg_residual(self.h, level, _ptr(b), _ptr(u), _ptr(r), ctypes.byref(nrm), _stream()),
               "mg_residual")
        return nrm.value

    def query(self):
        inf = mg_info()
        _check(lib().mg_query(self.h, ctypes.byref(inf)), "mg_query")
        n = inf.n_levels
        return {"n_levels": n, "nx": list(inf.nx[:n]), "ny": list(inf.ny[:n]), "n_active": list(inf.n_active[:n]),
                "n_plg": list(inf.n_plg[:n]), "n_sep": list(inf.n_sep[:n]),
                "sweep_words": list(inf.sweep_words[:n]), "n_face": inf.n_face,
                "n_irr": inf.n_irr, "nnz_plg": inf.nnz_plg, "device_bytes": inf.device_bytes,
                "setup_seconds": inf.setup_seconds, "n_sfv": list(inf.n_sfv[:n]),
                "cond_A22": list(inf.cond_A22[:n]), "setup_stage_seconds": list(inf.setup_stage_seconds),
                "n_pair_sfv": list(inf.n_pair_sfv[:n])}

    def export_level(self, level):
        nx, ny = self.info["nx"][level], self.info["ny"][level]
        kind = np.zeros(nx * ny, np.int32)
        m = ctypes.c_int()
        nnz = ctypes.c_longlong()
        _check(lib().mg_export_level(self.h, level, _ip(kind), ctypes.byref(m), ctypes.byref(nnz), None, None, None,
                                     None), "mg_export_level")
        rp = np.zeros(m.value + 1, np.int32)
        col = np.zeros(max(nnz.value, 1), np.int32)
        val = np.zeros(max(nnz.value, 1))
        bb = np.zeros(max(m.value, 1))
        _check(lib().mg_export_level(self.h, level, None, None, None, _ip(rp), _ip(col), _dp(val), _dp(bb)),
               "mg_export_level")
        return kind.reshape(ny, nx), rp, col[:nnz.value], val[:nnz.value], bb[:m.value]

    def cell_quadrature(self):
        n = ctypes.c_int()
        nn = ctypes.c_longlong()
        _check(lib().mg_cell_quadrature(self.h, ctypes.byref(n), ctypes.byref(nn), None, None, None, None, None),
               "mg_cell_quadrature")
        cell = np.zeros(max(n.value, 1), np.int32)
        ptr = np.zeros(n.value + 1, np.int64)
        x, y, w = (np.zeros(max(nn.value, 1)) for _ in range(3))
        _check(lib().mg_cell_quadrature(self.h, ctypes.byref(n), ctypes.byref(nn), _ip(cell), _lp(ptr), _dp(x), _dp(y),
                                        _dp(w)), "mg_cell_quadrature")
        return cell[:n.value], ptr, x[:nn.value], y[:nn.value], w[:nn.value]

    def boundary_quadrature(self):
        n = ctypes.c_int()
        nn = ctypes.c_longlong()
        _check(lib().mg_boundary_quadrature(self.h, ctypes.byref(n), ctypes.byref(nn), None, None, None, None, None,
                                            None, None, None, None), "mg_boundary_quadrature")
        ptr = np.zeros(n.value + 1, np.int64)
        x, y, w, nxv, nyv, a1, a2 = (np.zeros(max(nn.value, 1)) for _ in range(7))
        bc = np.zeros(max(nn.value, 1), np.int32)
        _check(lib().mg_boundary_quadrature(self.h, ctypes.byref(n), ctypes.byref(nn), _lp(ptr), _dp(x), _dp(y),
                                            _dp(w), _dp(nxv), _dp(nyv), _ip(bc), _dp(a1), _dp(a2)),
               "mg_boundary_quadrature")
        k = nn.value
        return ptr, x[:k], y[:k], w[:k], nxv[:k], nyv[:k], bc[:k], a1[:k], a2[:k]

    def set_eager(self, eager):
        _check(lib().mg_set_eager(self.h, 1 if eager else 0), "mg_set_eager")

    def kernel_timing(self, enable):
        n = ctypes.c_int()
        avg = ctypes.c_double()
        _check(lib().mg_kernel_timing(self.h, 1 if enable else 0, ctypes.byref(n), ctypes.byref(avg)),
               "mg_kernel_timing")
        return n.value, avg.value

    # -- inputs ------------------------------------------------------------------
    def project_rhs(self, f, g, gauss_points=8):
        """Device tensors (f_dev, g_dev) from mg_project_rhs.  f(x, y) and
        g(x, y, curve, seg, nx, ny) evaluate NumPy arrays of points (g returns
        the boundary datum N u); the library chooses the points and forms the
        averages."""
        import torch

        def fcb(n, x, y, out, ctx):
            xv = np.ctypeslib.as_array(x, (n,))
            yv = np.ctypeslib.as_array(y, (n,))
            np.ctypeslib.as_array(out, (n,))[:] = f(xv, yv)

        def gcb(n, x, y, curve, seg, nx, ny, out, ctx):
            arr = lambda p, t=np.float64: np.ctypeslib.as_array(p, (n,))
            np.ctypeslib.as_array(out, (n,))[:] = g(arr(x), arr(y), arr(curve), arr(seg), arr(nx), arr(ny))

        fd = self.empty()
        gd = torch.zeros(max(self.info["n_face"] + self.info["n_irr"], 1), dtype=torch.float64, device="cuda")
        fc, gc = F_BATCH(fcb), G_BATCH(gcb)
        _check(lib().mg_project_rhs(self.h, fc, gc, None, int(gauss_points), _ptr(fd), _ptr(gd), _stream()),
               "mg_project_rhs")
        return fd, gd

    def project(self, sol, gauss_points=8):
        """Device tensors (f, g) for a manufactured solution sol (sol.f, sol.u
        and its gradient): the boundary datum of each segment is its boundary
        condition applied to sol.u."""
        kinds = [[(BC[sg.bc], float(sg.alpha1), float(sg.alpha2)) for sg in cv] for cv in self.curves]
        tab = {}
        for ci, cv in enumerate(kinds):
            for si, k in enumerate(cv):
                tab[(ci, si)] = k

        def g(x, y, curve, seg, nx, ny):
            key = curve.astype(np.int64) * 4096 + seg.astype(np.int64)
            bc = np.empty(len(x), np.int32)
            a1 = np.empty(len(x))
            a2 = np.empty(len(x))
            for kk in np.unique(key):
                sel = key == kk
                b0, b1, b2 = tab[(int(kk) // 4096, int(kk) % 4096)]
                bc[sel], a1[sel], a2[sel] = b0, b1, b2
            u = sol.u(x, y)
            dn = sol.ux(x, y) * nx + sol.uy(x, y) * ny
            return np.where(bc == 0, u, np.where(bc == 1, dn, np.where(bc == 3, 0.0, a1 * u + a2 * dn)))

        return self.project_rhs(sol.f, g, gauss_points)


def to_padded(grid_vals, nx, ny):
    out = np.zeros((ny + 4, nx + 4))
    out[2:ny + 2, 2:nx + 2] = grid_vals
    return out


def from_padded(p, nx, ny):
    return np.asarray(p)[2:ny + 2, 2:nx + 2]


class Server:
    """The library's solve server (mg_server_*): requests are admitted into
    max_active slots as slots and the device-memory budget free up, and the
    solves of different requests overlap on the device."""

    def __init__(self, max_active=4, hbm_budget=64 << 30):
        opt = mg_server_options(max_active, hbm_budget)
        h = ctypes.c_void_p()
        _check(lib().mg_server_create(ctypes.byref(opt), ctypes.byref(h)), "mg_server_create")
        self.h = h
        self._inflight = {}

    def add_problem(self, grid, curves, a, b, c, eps=0.08, omega=0.5, nu=(3, 3), n_levels=0, min_coarse=16,
                    precision=FP64, max_iters=100, cycle=0):
        carr, keep = _curves(curves)
        g = mg_grid(grid.x0, grid.y0, grid.h, grid.nx, grid.ny)
        opt = _options(eps, omega, nu, n_levels, min_coarse, precision, max_iters, cycle)
        pid = ctypes.c_int()
        _check(lib().mg_server_add_problem(self.h, ctypes.byref(g), len(curves), carr, a, b, c, ctypes.byref(opt),
                                           ctypes.byref(pid)), "mg_server_add_problem")
        return pid.value

    def submit(self, problem, f, g, u, tol):
        """Queues a solve; f, g, u are device tensors in the layouts of
        Solver.solve (u: initial guess, overwritten by the solution).  The
        caller's stream is synchronised first: the server runs on its own
        streams."""
        import torch
        torch.cuda.current_stream().synchronize()
        t = ctypes.c_ulonglong()
        _check(lib().mg_server_submit(self.h, problem, _ptr(f), _ptr(g), _ptr(u), tol, ctypes.byref(t)),
               "mg_server_submit")
        self._inflight[t.value] = (f, g, u)
        return t.value

    def _result(self, ticket, st, it, rel, lat):
        self._inflight.pop(ticket, None)
        err = lib().mg_server_request_error(self.h, ticket).decode(errors="replace") if st.value else ""
        return {"status": st.value, "iters": it.value, "rel_residual": rel.value, "latency_s": lat.value,
                "error": err}

    def poll(self, ticket):
        done, st, it = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rel, lat = ctypes.c_double(), ctypes.c_double()
        _check(lib().mg_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(it),
                                    ctypes.byref(rel), ctypes.byref(lat)), "mg_server_poll")
        return self._result(ticket, st, it, rel, lat) if done.value else None

    def wait(self, ticket):
        st, it = ctypes.c_int(), ctypes.c_int()
        rel, lat = ctypes.c_double(), ctypes.c_double()
        _check(lib().mg_server_wait(self.h, ticket, ctypes.byref(st), ctypes.byref(it), ctypes.byref(rel),
                                    ctypes.byref(lat)), "mg_server_wait")
        return self._result(ticket, st, it, rel, lat)

    def stats(self):
        s = mg_server_stats()
        _check(lib().mg_server_get_stats(self.h, ctypes.byref(s)), "mg_server_get_stats")
        return {k: getattr(s, k) for k, _ in mg_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().mg_server_destroy(self.h)
            self.h = None
            self._inflight.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
