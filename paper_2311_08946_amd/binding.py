"""ctypes binding of ``libpdd.so`` (include/pdd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (float64 CUDA tensors) and the
current HIP stream.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpdd.so")
_lib = None

PDD_OK, PDD_EINVAL, PDD_ECOVER, PDD_ENOMEM, PDD_EDEVICE, PDD_ENOCONV, PDD_EPATHCAP, PDD_EBREAKDOWN = range(8)
STATUS_NAMES = {0: "PDD_OK", 1: "PDD_EINVAL", 2: "PDD_ECOVER", 3: "PDD_ENOMEM", 4: "PDD_EDEVICE",
                5: "PDD_ENOCONV", 6: "PDD_EPATHCAP", 7: "PDD_EBREAKDOWN"}
ROW_SPECTRAL, ROW_MC, ROW_BOUNDARY = 0, 1, 2
MAX_TERMS = 16
MAX_HOLES = 4

EXPORTED = [
    "pdd_last_error", "pdd_eval_field", "pdd_build_cover", "pdd_cover_get_info", "pdd_cover_knots",
    "pdd_cover_pattern", "pdd_cover_nodes", "pdd_destroy_cover", "pdd_assemble_G",
    "pdd_system_copy", "pdd_system_get_stats", "pdd_solve_G", "pdd_assemble_G_backward",
    "pdd_destroy_system", "pdd_ras_build", "pdd_ras_get_parts", "pdd_ras_apply", "pdd_destroy_ras",
    "pdd_solve_gmres", "pdd_solve_G_noalloc", "pdd_system_csr", "pdd_release_cached_memory",
]


class PddError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Domain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_holes", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double),
                ("holes", (C.c_double * 3) * MAX_HOLES)]


class Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_terms", C.c_int32), ("clip_nonpos", C.c_int32),
                ("reserved", C.c_int32), ("base", C.c_double),
                ("a", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)),
                ("c", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double))]


class Problem(C.Structure):
    _fields_ = [("domain", Domain)] + [(n, Field) for n in
                                       ("axx", "axy", "ayy", "bx", "by", "c", "f", "g", "u")]


class CoverOpts(C.Structure):
    _fields_ = [("rule", C.c_int32), ("reserved", C.c_int32), ("rbf_c2", C.c_double)]


class CoverInfo(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("N", "nnz", "n_circles", "n_float", "n_perim",
                                         "n_spectral_rows", "n_mc_rows", "n_boundary_rows",
                                         "sum_n", "sum_n2")] + \
               [(n, C.c_int32) for n in ("max_n", "max_M", "max_arc", "n_buckets")]


class Samples(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("axx", "axy", "ayy", "bx", "by", "c", "f")]


class McOpts(C.Structure):
    _fields_ = [("paths", C.c_int64), ("h", C.c_double), ("seed", C.c_uint64),
                ("n_batches", C.c_int32), ("step_cap", C.c_int32),
                ("h_per_circle", C.POINTER(C.c_double)), ("scheme", C.c_int32), ("reserved", C.c_int32)]


class AssembleOpts(C.Structure):
    _fields_ = [("plan", C.c_int32), ("keep_factors", C.c_int32), ("hbm_budget_bytes", C.c_int64),
                ("mixed_buckets", C.c_int32), ("grid_cap", C.c_int32), ("use_graph", C.c_int32),
                ("no_lookahead", C.c_int32), ("mc_order", C.c_int32), ("reserved", C.c_int32)]


PLANS = {"batched": 0, "per_circle": 1, "autotuned": 2}
# the Monte Carlo rows beside the floating rows or after them (pdd_assemble_opts.mc_order)
MC_ORDERS = {"auto": 0, "beside": 1, "after": 2}


class SystemStats(C.Structure):
    _fields_ = [("path_steps", C.c_int64), ("paths", C.c_int64), ("capped_paths", C.c_int64),
                ("breakdowns", C.c_int32), ("n_launch_spectral", C.c_int32),
                ("n_launch_mc", C.c_int32)] + \
               [(n, C.c_float) for n in ("ms_sample", "ms_build", "ms_lu", "ms_solve", "ms_eval",
                                         "ms_mc", "ms_total")] + \
               [("factor_bytes", C.c_int64), ("recompute", C.c_int32), ("n_groups", C.c_int32),
                ("mixed_buckets", C.c_int32), ("grid_cap", C.c_int32), ("graph_replays", C.c_int32),
                ("ms_autotune", C.c_float), ("gamma_exits", C.c_int64), ("lu_lookahead", C.c_int32),
                ("mc_after_floating", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("use_guess", C.c_int32),
                ("method", C.c_int32), ("reserved", C.c_int32)]


SOLVE_METHODS = {"bicgstab": 0, "direct": 1}


class RasOpts(C.Structure):
    _fields_ = [("parts_x", C.c_int32), ("parts_y", C.c_int32), ("fp32_inverses", C.c_int32),
                ("reserved", C.c_int32)]


class GmresOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double)]


def lib():
    """Load libpdd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2311_08946_amd/build.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(_LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    dp = C.POINTER(C.c_double)
    L.pdd_last_error.restype = C.c_char_p
    L.pdd_release_cached_memory.argtypes = []
    L.pdd_release_cached_memory.restype = C.c_int64
    L.pdd_eval_field.argtypes = [C.POINTER(Problem), i32, vp, i64, vp, vp]
    L.pdd_build_cover.argtypes = [C.POINTER(Domain), i32, dp, dp, C.POINTER(i32), C.POINTER(i32),
                                  C.POINTER(i32), C.POINTER(CoverOpts), C.POINTER(vp)]
    L.pdd_cover_get_info.argtypes = [vp, C.POINTER(CoverInfo)]
    L.pdd_cover_knots.argtypes = [vp, dp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.pdd_cover_pattern.argtypes = [vp, C.POINTER(i64), C.POINTER(i32)]
    L.pdd_cover_nodes.argtypes = [vp, dp, C.POINTER(i64), C.POINTER(i32)]
    L.pdd_destroy_cover.argtypes = [vp]
    L.pdd_destroy_cover.restype = None
    L.pdd_assemble_G.argtypes = [vp, C.POINTER(Problem), C.POINTER(Samples), C.POINTER(McOpts),
                                 C.POINTER(AssembleOpts), vp, C.POINTER(vp)]
    L.pdd_system_copy.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pdd_system_csr.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.pdd_system_get_stats.argtypes = [vp, C.POINTER(SystemStats)]
    L.pdd_solve_G.argtypes = [vp, vp, vp, i32, C.POINTER(SolveOpts), vp, C.POINTER(SolveInfo)]
    L.pdd_solve_G_noalloc.argtypes = [vp, vp, vp, i32, C.POINTER(SolveOpts), vp, C.POINTER(SolveInfo)]
    L.pdd_assemble_G_backward.argtypes = [vp, vp, vp] + [vp] * 8 + [vp]
    L.pdd_destroy_system.argtypes = [vp]
    L.pdd_destroy_system.restype = None
    L.pdd_ras_build.argtypes = [vp, C.POINTER(RasOpts), vp, C.POINTER(vp)]
    L.pdd_ras_get_parts.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32)]
    L.pdd_ras_apply.argtypes = [vp, vp, vp, vp]
    L.pdd_destroy_ras.argtypes = [vp]
    L.pdd_destroy_ras.restype = None
    L.pdd_solve_gmres.argtypes = [vp, vp, vp, vp, C.POINTER(GmresOpts), vp, C.POINTER(SolveInfo)]
    for name in EXPORTED:
        if name not in ("pdd_last_error", "pdd_destroy_cover", "pdd_destroy_system", "pdd_destroy_ras",
                        "pdd_release_cached_memory"):
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def release_cached_memory():
    """Frees the library's cache of released device blocks; returns bytes."""
    return int(lib().pdd_release_cached_memory())


def _check(code, what=""):
    if code != PDD_OK:
        msg = lib().pdd_last_error().decode(errors="replace")
        raise PddError(code, f"{what}{msg}")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


# --------------------------------------------------------------- marshalling

def make_domain(dom):
    d = Domain()
    if dom["kind"] == "box":
        d.kind = 0
        d.x0, d.x1, d.y0, d.y1 = dom["x0"], dom["x1"], dom["y0"], dom["y1"]
    else:
        d.kind = 1
        d.cx, d.cy, d.R = dom["cx"], dom["cy"], dom["R"]
        holes = dom.get("holes", [])
        if len(holes) > MAX_HOLES:
            raise ValueError("at most 4 holes")
        d.n_holes = len(holes)
        for t, (hx, hy, hr) in enumerate(holes):
            d.holes[t][0], d.holes[t][1], d.holes[t][2] = hx, hy, hr
    return d


def _field(fd, keep):
    f = Field()
    kind = fd["kind"]
    if kind == "const":
        f.kind, f.base = 0, fd["value"]
    elif kind == "sinsum":
        arrs = [np.ascontiguousarray(fd[k], dtype=np.float64) for k in ("amp", "kx", "ky", "phase")]
        keep.extend(arrs)
        f.kind, f.n_terms, f.clip_nonpos, f.base = 1, len(arrs[0]), int(fd["clip_nonpos"]), fd["base"]
        f.a, f.b, f.c, f.d = (_dptr(a) for a in arrs)
    elif kind == "cpoly_re":
        arrs = [np.ascontiguousarray(fd[k], dtype=np.float64) for k in ("alpha", "beta")]
        keep.extend(arrs)
        f.kind, f.n_terms = 2, len(arrs[0])
        f.a, f.b = (_dptr(a) for a in arrs)
    elif kind == "derived_f":
        f.kind = 3
    elif kind == "eq46":
        f.kind = 4
    else:
        raise ValueError(kind)
    if f.n_terms > MAX_TERMS:
        raise ValueError("too many field terms")
    return f


def make_problem(prob):
    keep = []
    p = Problem()
    p.domain = make_domain(prob["domain"])
    for name in ("axx", "axy", "ayy", "bx", "by", "c", "f", "g"):
        setattr(p, name, _field(prob[name], keep))
    if prob["f"]["kind"] == "derived_f":
        p.u = _field(prob["f"]["u"], keep)
    else:
        p.u = _field({"kind": "const", "value": 0.0}, keep)
    return p, keep


WHICH = {"axx": 0, "axy": 1, "ayy": 2, "bx": 3, "by": 4, "c": 5, "f": 6, "g": 7, "u": 8}


def eval_field(problem, which, xy, stream=None):
    """Evaluate a field of the problem at points xy (float64 CUDA tensor (n, 2))."""
    import torch
    p, keep = make_problem(problem)
    if which == "u" and problem.get("u_exact") is not None:
        p.u = _field(problem["u_exact"], keep)
    xy = xy.contiguous()
    out = torch.empty(xy.shape[0], dtype=torch.float64, device=xy.device)
    _check(lib().pdd_eval_field(C.byref(p), WHICH[which], _tptr(xy), xy.shape[0], _tptr(out),
                                _stream_ptr(stream)), "eval_field: ")
    return out


# --------------------------------------------------------------------- cover

class Cover:
    """Geometry of the cover (host), see pdd_build_cover."""

    def __init__(self, domain, cover):
        L = lib()
        centres = np.ascontiguousarray(cover["centres"], dtype=np.float64).reshape(-1)
        radii = np.ascontiguousarray(cover["radii"], dtype=np.float64)
        M = np.ascontiguousarray(cover["M"], dtype=np.int32)
        Nt = np.ascontiguousarray(cover["Ntheta"], dtype=np.int32)
        Nr = np.ascontiguousarray(cover["Nr"], dtype=np.int32)
        opts = CoverOpts(int(cover.get("rule", 0)), 0, float(cover.get("rbf_c2", 0.0)))
        h = C.c_void_p()
        dom = make_domain(domain)
        _check(L.pdd_build_cover(C.byref(dom), len(radii), _dptr(centres), _dptr(radii), _iptr(M),
                                 _iptr(Nt), _iptr(Nr), C.byref(opts), C.byref(h)), "build_cover: ")
        self._h = h
        self.info = CoverInfo()
        _check(L.pdd_cover_get_info(h, C.byref(self.info)))
        self.N = int(self.info.N)
        self.nnz = int(self.info.nnz)

    @property
    def handle(self):
        return self._h

    def knots(self):
        N = self.N
        xy = np.zeros(2 * N)
        rc, asg, own = (np.zeros(N, dtype=np.int32) for _ in range(3))
        _check(lib().pdd_cover_knots(self._h, _dptr(xy), _iptr(rc), _iptr(asg), _iptr(own)))
        return xy.reshape(N, 2), rc, asg, own

    def pattern(self):
        rowptr = np.zeros(self.N + 1, dtype=np.int64)
        cols = np.zeros(self.nnz, dtype=np.int32)
        _check(lib().pdd_cover_pattern(self._h, rowptr.ctypes.data_as(C.POINTER(C.c_int64)), _iptr(cols)))
        return rowptr, cols

    def nodes(self):
        nf = int(self.info.n_float)
        xy = np.zeros(2 * int(self.info.sum_n))
        off = np.zeros(nf + 1, dtype=np.int64)
        ids = np.zeros(nf, dtype=np.int32)
        _check(lib().pdd_cover_nodes(self._h, _dptr(xy), off.ctypes.data_as(C.POINTER(C.c_int64)),
                                     _iptr(ids)))
        return xy.reshape(-1, 2), off, ids

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pdd_destroy_cover(h)
            self._h = None


# -------------------------------------------------------------------- system

def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _tptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class System:
    """Assembled C (CSR on the cover's pattern), r and standard errors, on the device."""

    def __init__(self, cover, problem, mc, samples=None, keep_factors=False, plan="batched",
                 hbm_budget_bytes=0, mixed_buckets=True, grid_cap=0, use_graph=False, lookahead=True,
                 mc_order="auto", stream=None):
        import torch
        L = lib()
        self.cover = cover
        p, keep = make_problem(problem)
        mo = McOpts()
        mo.paths, mo.h, mo.seed = int(mc["paths"]), float(mc["h"]), int(mc["seed"])
        mo.n_batches, mo.step_cap = int(mc["n_batches"]), int(mc["step_cap"])
        mo.scheme = int(mc.get("scheme", 0))
        if mc.get("h_per_circle") is not None:
            hpc = np.ascontiguousarray(mc["h_per_circle"], dtype=np.float64)
            keep.append(hpc)
            mo.h_per_circle = _dptr(hpc)
        ao = AssembleOpts(PLANS[plan], int(bool(keep_factors)), int(hbm_budget_bytes),
                          int(bool(mixed_buckets)), int(grid_cap), int(bool(use_graph)),
                          int(not lookahead), MC_ORDERS[mc_order], 0)
        sm = None
        if samples is not None:
            for k, v in samples.items():
                if v is not None and (v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous()):
                    raise ValueError(f"sample {k} must be a contiguous float64 CUDA tensor")
            sm = Samples(*[_tptr(samples.get(k)) for k in ("axx", "axy", "ayy", "bx", "by", "c", "f")])
        h = C.c_void_p()
        code = L.pdd_assemble_G(cover.handle, C.byref(p), C.byref(sm) if sm is not None else None,
                                C.byref(mo), C.byref(ao), _stream_ptr(stream), C.byref(h))
        self._h = h if h.value else None
        self._keep = keep
        _check(code, "assemble_G: ")
        self.stats = SystemStats()
        _check(L.pdd_system_get_stats(self._h, C.byref(self.stats)))

    @property
    def handle(self):
        return self._h

    def copy(self, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        val = torch.empty(self.cover.nnz, dtype=torch.float64, device=dev)
        se = torch.empty_like(val)
        b = torch.empty(self.cover.N, dtype=torch.float64, device=dev)
        se_b = torch.empty_like(b)
        _check(lib().pdd_system_copy(self._h, _tptr(val), _tptr(b), _tptr(se), _tptr(se_b),
                                     _stream_ptr(stream)))
        return val, b, se, se_b

    def csr(self, stream=None):
        """(rowptr, cols, val, b, se) of C and r on the device (pdd_system_csr)."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        rowptr = torch.empty(self.cover.N + 1, dtype=torch.int64, device=dev)
        cols = torch.empty(self.cover.nnz, dtype=torch.int32, device=dev)
        val = torch.empty(self.cover.nnz, dtype=torch.float64, device=dev)
        se = torch.empty_like(val)
        b = torch.empty(self.cover.N, dtype=torch.float64, device=dev)
        _check(lib().pdd_system_csr(self._h, _tptr(rowptr), _tptr(cols), _tptr(val), _tptr(b), _tptr(se),
                                    _stream_ptr(stream)))
        return rowptr, cols, val, b, se

    def solve(self, rhs=None, transpose=False, rtol=1e-12, max_iter=2000, guess=None, stream=None,
              method="bicgstab"):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        u = guess.clone() if guess is not None else torch.zeros(self.cover.N, dtype=torch.float64, device=dev)
        so = SolveOpts(rtol, max_iter, 1 if guess is not None else 0, SOLVE_METHODS[method], 0)
        info = SolveInfo()
        _check(lib().pdd_solve_G(self._h, _tptr(rhs), _tptr(u), int(bool(transpose)), C.byref(so),
                                 _stream_ptr(stream), C.byref(info)), "solve_G: ")
        return u, info

    def solve_gmres(self, ras=None, rhs=None, rtol=1e-12, max_iter=2000, restart=30, stream=None):
        """Restarted GMRES with the RAS preconditioner ``ras`` on the right (None: none)."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        u = torch.empty(self.cover.N, dtype=torch.float64, device=dev)
        go = GmresOpts(rtol, max_iter, restart)
        info = SolveInfo()
        _check(lib().pdd_solve_gmres(self._h, ras.handle if ras is not None else None, _tptr(rhs), _tptr(u),
                                     C.byref(go), _stream_ptr(stream), C.byref(info)), "solve_gmres: ")
        return u, info

    def backward(self, u, lam, stream=None, names=("axx", "axy", "ayy", "bx", "by", "c", "f")):
        """Gradients w.r.t. the node samples named in ``names``; "r" in names also
        returns dL/dr (= lam)."""
        import torch
        n = int(self.cover.info.sum_n)
        dev = u.device
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) if k in names else None
               for k in ("axx", "axy", "ayy", "bx", "by", "c", "f")}
        out["r"] = torch.empty(self.cover.N, dtype=torch.float64, device=dev) if "r" in names else None
        _check(lib().pdd_assemble_G_backward(self._h, _tptr(u), _tptr(lam),
                                             *[_tptr(out[k]) for k in ("axx", "axy", "ayy", "bx", "by", "c", "f",
                                                                       "r")],
                                             _stream_ptr(stream)), "assemble_G_backward: ")
        return {k: v for k, v in out.items() if v is not None}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pdd_destroy_system(h)
            self._h = None


class Ras:
    """One-level RAS preconditioner of an assembled system (eqs. 42-44)."""

    def __init__(self, system, parts_x, parts_y, fp32_inverses=False, stream=None):
        L = lib()
        self.system = system          # the preconditioner refers to the system
        h = C.c_void_p()
        opts = RasOpts(int(parts_x), int(parts_y), int(bool(fp32_inverses)), 0)
        code = L.pdd_ras_build(system.handle, C.byref(opts),
                               _stream_ptr(stream), C.byref(h))
        self._h = h if h.value else None
        _check(code, "ras_build: ")

    @property
    def handle(self):
        return self._h

    def parts(self):
        L = lib()
        P = C.c_int32()
        _check(L.pdd_ras_get_parts(self._h, C.byref(P), None, None))
        off = np.zeros(P.value + 1, dtype=np.int64)
        _check(L.pdd_ras_get_parts(self._h, None, off.ctypes.data_as(C.POINTER(C.c_int64)), None))
        knots = np.zeros(int(off[-1]), dtype=np.int32)
        _check(L.pdd_ras_get_parts(self._h, None, None, _iptr(knots)))
        return [knots[off[p]:off[p + 1]].astype(np.int64) for p in range(P.value)]

    def apply(self, x, stream=None):
        import torch
        y = torch.empty_like(x)
        _check(lib().pdd_ras_apply(self._h, _tptr(x), _tptr(y), _stream_ptr(stream)), "ras_apply: ")
        return y

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.pdd_destroy_ras(h)
            self._h = None
