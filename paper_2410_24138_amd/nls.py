"""ctypes binding of libnls (the C ABI declared in include/nls.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (tensors) and the stream.  The binding fails
loudly when libnls.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnls.so")

NLS_OK = 0
NLS_ENOCONV = 1
NLS_EINVAL = -1
NLS_EHIP = -2
NLS_ENOMEM = -3
NLS_EPARTITION = -4
NLS_ESINGULAR = -5
NLS_ELOCAL = -6
NLS_ENAN = -7
NLS_ESTATE = -8
NLS_ELIMIT = -9
NLS_EDETF = -10
NLS_GUESS_NOALLOC_ROWS = 4096

ELEM_P1_TRI = 3
ELEM_Q1_QUAD = 4
PROBLEM_DIFFUSION = 1
PROBLEM_NEOHOOKE = 2
PREC_FP64 = 0
PREC_FP32_IR = 1
PREC_BF16_IR = 2
ONE_LEVEL = 0
ADDITIVE = 1
HYBRID = 2
COARSE_NONE = 0
COARSE_GDSW = 1
COARSE_RGDSW = 2
MAX_OUTER = 64
FLAG_PROFILE = 1
FLAG_GRAPH = 2
FLAG_COARSE_CHORD = 4
FLAG_COARSE_LU_APPLY = 8
FLAG_AUTOTUNE = 16
FLAG_OVERLAP = 32
FLAG_TANGENT_SWEEP = 64

# every symbol include/nls.h declares
SYMBOLS = (
    "nls_default_options", "nls_create", "nls_destroy", "nls_set_mesh",
    "nls_set_mesh_structured",
    "nls_set_problem", "nls_set_dirichlet", "nls_set_partition",
    "nls_build_coarse", "nls_solve", "nls_eval_residual",
    "nls_eval_precond_residual", "nls_apply_tangent",
    "nls_get_inner_iterations", "nls_get_sizes", "nls_get_coarse_basis",
    "nls_eval_local", "nls_get_local_pattern",
    "nls_strerror", "nls_last_error", "nls_inspect_partition",
    "nls_inspect_coarse", "nls_set_load", "nls_guess_set_model",
    "nls_guess_get_model", "nls_guess_enable", "nls_guess_capture",
    "nls_guess_captured", "nls_guess_features", "nls_guess_lift",
    "nls_guess_predict", "nls_guess_predict_noalloc", "nls_guess_loss_grad",
    "nls_guess_train",
    "nls_get_tuning", "nls_set_nodal_load", "nls_solve_load_steps", "nls_solve_nks",
    "nls_solve_batch",
)

GUESS_PARAMS = 279552
GUESS_NORM = 1152
GUESS_IN = 320
GUESS_OUT = 256
TRAIN_FIT_NORM = 1
TRAIN_COSINE = 2
MAX_EPOCHS = 256


class Options(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int), ("stream", ctypes.c_void_p),
        ("precision", ctypes.c_int), ("coupling", ctypes.c_int),
        ("outer_rtol", ctypes.c_double), ("outer_maxit", ctypes.c_int),
        ("inner_rtol", ctypes.c_double), ("inner_eta", ctypes.c_double),
        ("stagnation", ctypes.c_double), ("inner_maxit", ctypes.c_int),
        ("gmres_rtol", ctypes.c_double), ("gmres_maxit", ctypes.c_int),
        ("gmres_restart", ctypes.c_int), ("flags", ctypes.c_int),
        ("lu_variant", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("converged", ctypes.c_int), ("outer_its", ctypes.c_int),
        ("gmres_its", ctypes.c_int * MAX_OUTER), ("gmres_its_total", ctypes.c_int),
        ("inner_its_total", ctypes.c_int64), ("inner_its_max", ctypes.c_int),
        ("local_solves", ctypes.c_int64), ("coarse_its_total", ctypes.c_int),
        ("failed_subdomain", ctypes.c_int), ("res0", ctypes.c_double),
        ("res_final", ctypes.c_double), ("ms_inner", ctypes.c_double),
        ("ms_coarse", ctypes.c_double), ("ms_gmres", ctypes.c_double),
        ("ms_other", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("n_local_launches", ctypes.c_int), ("ms_local_kernel", ctypes.c_double),
        ("n_tangent_launches", ctypes.c_int), ("ms_tangent_kernel", ctypes.c_double),
        ("guess_used", ctypes.c_int64), ("guess_fallback", ctypes.c_int64),
        ("ms_overlap", ctypes.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "gmres_its"}
        d["gmres_its"] = list(self.gmres_its[: self.outer_its])
        return d


class TrainOpts(ctypes.Structure):
    _fields_ = [
        ("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
        ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
        ("flags", ctypes.c_int),
    ]


class TrainStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64), ("final_loss", ctypes.c_double),
        ("epoch_loss", ctypes.c_double * MAX_EPOCHS), ("ms", ctypes.c_double),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libnls.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2410_24138_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "nls_default_options": ([ctypes.POINTER(Options)], ctypes.c_int),
        "nls_create": ([ctypes.POINTER(Options), ctypes.POINTER(P)], ctypes.c_int),
        "nls_destroy": ([P], ctypes.c_int),
        "nls_set_mesh": ([P, ctypes.c_int, i64, P, i64, P], ctypes.c_int),
        "nls_set_problem": ([P, ctypes.c_int, P, P, P], ctypes.c_int),
        "nls_set_dirichlet": ([P, i64, P, P], ctypes.c_int),
        "nls_set_partition": ([P, i32, P, i32], ctypes.c_int),
        "nls_set_mesh_structured": ([P, ctypes.c_int, i32, i32, dbl, dbl], ctypes.c_int),
        "nls_build_coarse": ([P, ctypes.c_int, P], ctypes.c_int),
        "nls_solve": ([P, P, ctypes.c_int, dbl, ctypes.POINTER(Stats)], ctypes.c_int),
        "nls_eval_residual": ([P, P, P], ctypes.c_int),
        "nls_eval_precond_residual": ([P, P, P], ctypes.c_int),
        "nls_apply_tangent": ([P, P, P], ctypes.c_int),
        "nls_get_inner_iterations": ([P, P], ctypes.c_int),
        "nls_eval_local": ([P, P, P, P], ctypes.c_int),
        "nls_get_local_pattern": ([P, P, P, P, P, P, P, P], ctypes.c_int),
        "nls_get_sizes": ([P, P, P, P], ctypes.c_int),
        "nls_get_coarse_basis": ([P, ctypes.POINTER(i64), P, P, P], ctypes.c_int),
        "nls_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "nls_inspect_partition": ([i64, i64, P, i32, P, i32, P, P, P, P, P, P, P, P],
                                  ctypes.c_int),
        "nls_inspect_coarse": ([i64, i64, P, i32, P, i64, P, P, P, P], ctypes.c_int),
        "nls_last_error": ([P], ctypes.c_char_p),
        "nls_set_load": ([P, P], ctypes.c_int),
        "nls_set_nodal_load": ([P, P], ctypes.c_int),
        "nls_solve_load_steps": ([P, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Stats)],
                                 ctypes.c_int),
        "nls_solve_nks": ([P, P, ctypes.c_int, ctypes.POINTER(Stats)], ctypes.c_int),
        "nls_solve_batch": ([P, ctypes.c_int, P, P, P, P], ctypes.c_int),
        "nls_get_tuning": ([P, P, P, P, P, P, P, P], ctypes.c_int),
        "nls_guess_set_model": ([P, P, i64, P], ctypes.c_int),
        "nls_guess_get_model": ([P, P, P], ctypes.c_int),
        "nls_guess_enable": ([P, ctypes.c_int], ctypes.c_int),
        "nls_guess_capture": ([P, i64], ctypes.c_int),
        "nls_guess_captured": ([P, P, P, i64, ctypes.POINTER(i64)], ctypes.c_int),
        "nls_guess_features": ([P, P, P], ctypes.c_int),
        "nls_guess_lift": ([P, P, P, P], ctypes.c_int),
        "nls_guess_predict": ([P, P, i64, P], ctypes.c_int),
        "nls_guess_predict_noalloc": ([P, P, i64, P], ctypes.c_int),
        "nls_guess_loss_grad": ([P, P, P, i64, P, ctypes.POINTER(dbl)], ctypes.c_int),
        "nls_guess_train": ([P, ctypes.POINTER(TrainOpts), P, P, i64, P,
                             ctypes.POINTER(TrainStats)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _ = dbl
    _lib = lib
    return lib


class NLSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libnls error {code}: {msg}")
        self.code = code


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def inspect_partition(case: dict):
    """Host-only: the subdomain maps libnls builds for a case (no device)."""
    lib = load()
    conn = np.ascontiguousarray(case["conn"], dtype=np.int32)
    part = np.ascontiguousarray(case["elem_part"], dtype=np.int32)
    N, E, ns, ov = len(case["xy"]), len(conn), int(case["n_sub"]), int(case["overlap"])
    cnt = np.zeros(2, dtype=np.int64)
    args = (N, E, _ptr(conn), ns, _ptr(part), ov)
    rc = lib.nls_inspect_partition(*args, _ptr(cnt), None, None, None, None, None, None, None)
    if rc:
        raise NLSError(rc, lib.nls_strerror(rc).decode())
    off_v = np.zeros(ns + 1, np.int32)
    off_g = np.zeros(ns + 1, np.int32)
    v = np.zeros(cnt[0], np.int32)
    g = np.zeros(cnt[1], np.int32)
    own = np.zeros(N, np.int32)
    kl = np.zeros(ns, np.int32)
    ku = np.zeros(ns, np.int32)
    rc = lib.nls_inspect_partition(*args, _ptr(cnt), _ptr(off_v), _ptr(v), _ptr(off_g),
                                   _ptr(g), _ptr(own), _ptr(kl), _ptr(ku))
    if rc:
        raise NLSError(rc, lib.nls_strerror(rc).decode())
    return {"off_v": off_v, "v": v, "off_g": off_g, "g": g, "own_pos": own,
            "kl": kl, "ku": ku}


def inspect_coarse(case: dict):
    """Host-only: the GDSW interface components libnls builds for a case."""
    lib = load()
    conn = np.ascontiguousarray(case["conn"], dtype=np.int32)
    part = np.ascontiguousarray(case["elem_part"], dtype=np.int32)
    dn = np.ascontiguousarray(case["dirichlet"], dtype=np.int64)
    N, E, ns = len(case["xy"]), len(conn), int(case["n_sub"])
    cnt = np.zeros(2, dtype=np.int64)
    args = (N, E, _ptr(conn), ns, _ptr(part), len(dn), _ptr(dn))
    rc = lib.nls_inspect_coarse(*args, _ptr(cnt), None, None)
    if rc:
        raise NLSError(rc, lib.nls_strerror(rc).decode())
    off = np.zeros(cnt[0] + 1, np.int32)
    nodes = np.zeros(cnt[1], np.int32)
    rc = lib.nls_inspect_coarse(*args, _ptr(cnt), _ptr(off), _ptr(nodes))
    if rc:
        raise NLSError(rc, lib.nls_strerror(rc).decode())
    return [nodes[off[k]:off[k + 1]] for k in range(cnt[0])]


def solve_batch(solvers, us=None):
    """nls_solve_batch over Solver objects (distinct handles; give each its
    own stream to let them run together).  us: float64 device tensors (the
    initial iterates, overwritten), default zeros.  Returns (us, per-instance
    stats, per-instance codes, rc)."""
    import torch
    lib = load()
    n = len(solvers)
    if us is None:
        us = [torch.zeros(s.N, dtype=torch.float64, device=s.device) for s in solvers]
    for s, u in zip(solvers, us):
        assert u.dtype == torch.float64 and u.is_cuda and u.is_contiguous() and u.numel() == s.N
    hs = (ctypes.c_void_p * n)(*[s.h.value for s in solvers])
    ups = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
    dev = (ctypes.c_int * n)(*([1] * n))
    sts = (Stats * n)()
    codes = (ctypes.c_int * n)()
    for s in solvers:
        torch.cuda.current_stream(s.device).synchronize()
    rc = lib.nls_solve_batch(hs, n, ups, dev, sts, codes)
    if rc == NLS_EINVAL:
        raise NLSError(rc, "nls_solve_batch: null or repeated handles")
    return us, [st.as_dict() for st in sts], list(codes), rc


def default_options() -> Options:
    o = Options()
    load().nls_default_options(ctypes.byref(o))
    return o


class Solver:
    """One libnls handle set up for an input case (see synth.diffusion_case).

    coupling: "one_level", "additive" or "hybrid"; precision: "fp64", "fp32_ir"
    or "bf16_ir" (the trial with bfloat16 operands in the LU's trailing updates).
    coarse_lin: linearisation point of the coarse basis extension (default 0);
    structured: (nx, ny, lx, ly) to let the library generate the case's
    structured grid (nls_set_mesh_structured) instead of passing it.
    Options not given keep the library defaults.
    """

    def __init__(self, case: dict, coupling: Optional[str] = None,
                 precision: str = "fp64", device: int = 0, stream=None,
                 coarse: str = "gdsw", coarse_lin=None, structured=None, **opts):
        import torch
        self.lib = load()
        self.torch = torch
        self.device = torch.device("cuda", device)
        o = default_options()
        o.device = device
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        o.stream = ctypes.c_void_p(int(stream))
        if coupling is None:
            coupling = "additive" if case.get("two_level") else "one_level"
        o.coupling = {"one_level": ONE_LEVEL, "additive": ADDITIVE, "hybrid": HYBRID}[coupling]
        o.precision = {"fp64": PREC_FP64, "fp32_ir": PREC_FP32_IR, "bf16_ir": PREC_BF16_IR}[precision]
        for k, v in opts.items():
            setattr(o, k, v)
        self.opts = o
        h = ctypes.c_void_p()
        self._check(self.lib.nls_create(ctypes.byref(o), ctypes.byref(h)), None)
        self.h = h
        self.case = case
        xy = np.ascontiguousarray(case["xy"], dtype=np.float64)
        conn = np.ascontiguousarray(case["conn"], dtype=np.int32)
        elastic = case.get("kind") == "neohooke"
        self.d = 2 if elastic else 1
        self.N = self.d * len(xy)
        kind_e = ELEM_Q1_QUAD if elastic else ELEM_P1_TRI
        if structured is not None:
            # (nx, ny, lx, ly): the library generates the case's grid itself
            nx, ny, lx, ly = structured
            self._check(self.lib.nls_set_mesh_structured(h, kind_e, int(nx), int(ny),
                                                         float(lx), float(ly)))
        else:
            self._check(self.lib.nls_set_mesh(h, kind_e, len(xy), _ptr(xy), len(conn), _ptr(conn)))
        if elastic:
            params = np.array([case["mu"], case["lam"]], dtype=np.float64)
            self._check(self.lib.nls_set_problem(h, PROBLEM_NEOHOOKE, _ptr(params), None, None))
        else:
            params = np.array([case.get("beta", 1.0)], dtype=np.float64)
            coef = case.get("elem_coef")
            load_ = case.get("elem_load")
            coef = None if coef is None else np.ascontiguousarray(coef, dtype=np.float64)
            load_ = None if load_ is None else np.ascontiguousarray(load_, dtype=np.float64)
            self._check(self.lib.nls_set_problem(
                h, PROBLEM_DIFFUSION, _ptr(params),
                None if coef is None else _ptr(coef),
                None if load_ is None else _ptr(load_)))
        dn = np.ascontiguousarray(case["dirichlet"], dtype=np.int64)
        dv = np.ascontiguousarray(case["dirichlet_vals"], dtype=np.float64)
        self._check(self.lib.nls_set_dirichlet(h, len(dn), _ptr(dn), _ptr(dv)))
        if elastic:
            self.set_nodal_load(case["nodal_force"])
        part = np.ascontiguousarray(case["elem_part"], dtype=np.int32)
        self._check(self.lib.nls_set_partition(h, int(case["n_sub"]), _ptr(part),
                                               int(case["overlap"])))
        if coupling in ("additive", "hybrid"):
            kind = {"gdsw": COARSE_GDSW, "rgdsw": COARSE_RGDSW}[coarse]
            ul = None
            if coarse_lin is not None:
                ul = np.ascontiguousarray(coarse_lin, dtype=np.float64)
                assert ul.size == self.N
            self._check(self.lib.nls_build_coarse(h, kind, None if ul is None else _ptr(ul)))

    def set_nodal_load(self, f):
        """Nodal forces (elasticity), n_nodes * 2 values in dof order."""
        a = np.ascontiguousarray(f, dtype=np.float64)
        assert a.size == self.N
        self._check(self.lib.nls_set_nodal_load(self.h, _ptr(a)))

    def _check(self, rc, h="self"):
        if rc < 0:
            hh = self.h if h == "self" else None
            msg = (self.lib.nls_last_error(hh) if hh else self.lib.nls_strerror(rc))
            raise NLSError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.nls_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, x):
        t = self.torch
        if isinstance(x, np.ndarray):
            x = t.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
        x = x.to(self.device, t.float64).contiguous()
        return x

    def _vp(self, t):
        return ctypes.c_void_p(t.data_ptr())

    # ---- entry points ------------------------------------------------------
    def solve(self, u0=None, load_factor=1.0):
        """Outer Newton from u0 (default 0) with the external load scaled by
        load_factor.  Returns (u tensor, stats, rc)."""
        t = self.torch
        u = t.zeros(self.N, dtype=t.float64, device=self.device) if u0 is None \
            else self._dev(u0).clone()
        st = Stats()
        rc = self._check(self.lib.nls_solve(self.h, self._vp(u), 1, float(load_factor),
                                            ctypes.byref(st)))
        return u, st.as_dict(), rc

    def solve_nks(self, u0=None):
        """Newton-Krylov-Schwarz comparator from u0 (default 0): Newton on
        F(u) = 0 with GMRES right-preconditioned by linear Schwarz.
        Returns (u tensor, stats, rc)."""
        t = self.torch
        u = t.zeros(self.N, dtype=t.float64, device=self.device) if u0 is None \
            else self._dev(u0).clone()
        st = Stats()
        rc = self._check(self.lib.nls_solve_nks(self.h, self._vp(u), 1, ctypes.byref(st)))
        return u, st.as_dict(), rc

    def solve_load_steps(self, n_steps, u0=None):
        """Load stepping from u0 (default 0) in n_steps equal increments.
        Returns (u tensor, per-step stats, rc)."""
        t = self.torch
        u = t.zeros(self.N, dtype=t.float64, device=self.device) if u0 is None \
            else self._dev(u0).clone()
        st = (Stats * int(n_steps))()
        rc = self._check(self.lib.nls_solve_load_steps(self.h, self._vp(u), 1, int(n_steps), st))
        return u, [s.as_dict() for s in st], rc

    def solve_(self, u):
        """Outer Newton in place on a float64 device tensor u; returns stats."""
        t = self.torch
        assert u.dtype == t.float64 and u.is_cuda and u.is_contiguous() and u.numel() == self.N
        st = Stats()
        self._check(self.lib.nls_solve(self.h, self._vp(u), 1, 1.0, ctypes.byref(st)))
        return st.as_dict()

    def solve_host(self, u: np.ndarray):
        """Same on a host array (updated in place)."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        st = Stats()
        rc = self._check(self.lib.nls_solve(self.h, _ptr(u), 0, 1.0, ctypes.byref(st)))
        return st.as_dict(), rc

    def residual(self, u):
        u = self._dev(u)
        F = self.torch.empty_like(u)
        self._check(self.lib.nls_eval_residual(self.h, self._vp(u), self._vp(F)))
        return F

    def precond_residual(self, u):
        u = self._dev(u)
        Fx = self.torch.empty_like(u)
        self._check(self.lib.nls_eval_precond_residual(self.h, self._vp(u), self._vp(Fx)))
        self._keep = u
        return Fx

    def tangent(self, v):
        v = self._dev(v)
        y = self.torch.empty_like(v)
        self._check(self.lib.nls_apply_tangent(self.h, self._vp(v), self._vp(y)))
        return y

    def local_pattern(self):
        """Packed row layout of the local problems and the CSR pattern of
        [J_ii | B_i] (numpy arrays, see nls_get_local_pattern)."""
        cnt = np.zeros(3, np.int64)
        self._check(self.lib.nls_get_local_pattern(self.h, _ptr(cnt), None, None, None, None,
                                                   None, None))
        ns = int(self.case["n_sub"])
        out = {"off_v": np.zeros(ns + 1, np.int32), "row_dof": np.zeros(cnt[0], np.int32),
               "off_g": np.zeros(ns + 1, np.int32), "gamma_dof": np.zeros(cnt[2], np.int32),
               "rowptr": np.zeros(cnt[0] + 1, np.int64), "col": np.zeros(cnt[1], np.int32)}
        self._check(self.lib.nls_get_local_pattern(
            self.h, _ptr(cnt), _ptr(out["off_v"]), _ptr(out["row_dof"]), _ptr(out["off_g"]),
            _ptr(out["gamma_dof"]), _ptr(out["rowptr"]), _ptr(out["col"])))
        return out

    def eval_local(self, u, jacobian=True, r=None, jval=None):
        """Standalone local assembly at x = R_i u: packed local residuals and
        (if jacobian) the CSR values of [J_ii | B_i].  Output tensors may be
        passed in (float64, on the device) to avoid allocation."""
        t = self.torch
        u = self._dev(u)
        if r is None or (jacobian and jval is None):
            cnt = np.zeros(3, np.int64)
            self._check(self.lib.nls_get_local_pattern(self.h, _ptr(cnt), None, None, None,
                                                       None, None, None))
            if r is None:
                r = t.empty(int(cnt[0]), dtype=t.float64, device=self.device)
            if jacobian and jval is None:
                jval = t.empty(int(cnt[1]), dtype=t.float64, device=self.device)
        self._check(self.lib.nls_eval_local(self.h, self._vp(u), self._vp(r),
                                            self._vp(jval) if jacobian else None))
        return r, jval

    def inner_iterations(self):
        n_sub, _, _ = self.sizes()
        its = np.zeros(n_sub, dtype=np.int32)
        self._check(self.lib.nls_get_inner_iterations(self.h, _ptr(its)))
        return its

    def sizes(self):
        ns = ctypes.c_int32()
        n0 = ctypes.c_int32()
        self._check(self.lib.nls_get_sizes(self.h, ctypes.byref(ns), ctypes.byref(n0), None))
        nv = np.zeros(ns.value, dtype=np.int32)
        self._check(self.lib.nls_get_sizes(self.h, None, None, _ptr(nv)))
        return ns.value, n0.value, nv

    def coarse_basis(self):
        import scipy.sparse as sp
        nnz = ctypes.c_int64(0)
        self._check(self.lib.nls_get_coarse_basis(self.h, ctypes.byref(nnz), None, None, None))
        rp = np.zeros(self.N + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        self._check(self.lib.nls_get_coarse_basis(self.h, ctypes.byref(nnz), _ptr(rp),
                                                  _ptr(col), _ptr(val)))
        _, n0, _ = self.sizes()
        return sp.csr_matrix((val, col, rp), shape=(self.N, n0))

    # ---- load and learned initial guess ------------------------------------
    def set_load(self, elem_load):
        """New load samples (E x 3, or None for f = 1) on the same partition."""
        if elem_load is None:
            self._check(self.lib.nls_set_load(self.h, None))
        else:
            a = np.ascontiguousarray(elem_load, dtype=np.float64)
            self._check(self.lib.nls_set_load(self.h, _ptr(a)))

    def _f32(self, x, cols):
        t = self.torch
        if isinstance(x, np.ndarray):
            x = t.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
        x = x.to(self.device, t.float32).contiguous()
        assert x.dim() == 2 and x.shape[1] == cols
        return x

    def guess_set_model(self, params, norm=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        assert nm is None or nm.size == GUESS_NORM
        self._check(self.lib.nls_guess_set_model(self.h, _ptr(p), p.size,
                                                 None if nm is None else _ptr(nm)))

    def guess_get_model(self):
        p = np.zeros(GUESS_PARAMS, dtype=np.float32)
        nm = np.zeros(GUESS_NORM, dtype=np.float32)
        self._check(self.lib.nls_guess_get_model(self.h, _ptr(p), _ptr(nm)))
        return p, nm

    def guess_enable(self, on=True):
        self._check(self.lib.nls_guess_enable(self.h, 1 if on else 0))

    def guess_capture(self, capacity):
        self._check(self.lib.nls_guess_capture(self.h, int(capacity)))

    def guess_count(self):
        """Rows captured so far."""
        n = ctypes.c_int64(0)
        self._check(self.lib.nls_guess_captured(self.h, None, None, 0, ctypes.byref(n)))
        return n.value

    def guess_captured(self):
        t = self.torch
        n = ctypes.c_int64(0)
        self._check(self.lib.nls_guess_captured(self.h, None, None, 0, ctypes.byref(n)))
        X = t.empty((n.value, GUESS_IN), dtype=t.float32, device=self.device)
        T = t.empty((n.value, GUESS_OUT), dtype=t.float32, device=self.device)
        if n.value:
            self._check(self.lib.nls_guess_captured(self.h, self._vp(X), self._vp(T),
                                                    n.value, ctypes.byref(n)))
        return X, T

    def guess_features(self, u):
        u = self._dev(u)
        ns, _, _ = self.sizes()
        X = self.torch.empty((ns, GUESS_IN), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.nls_guess_features(self.h, self._vp(u), self._vp(X)))
        return X

    def guess_lift(self, u, coef):
        u = self._dev(u)
        c = self._f32(coef, GUESS_OUT)
        _, _, nv = self.sizes()
        x = self.torch.empty(int(nv.sum()), dtype=self.torch.float64, device=self.device)
        self._check(self.lib.nls_guess_lift(self.h, self._vp(u), self._vp(c), self._vp(x)))
        return x

    def guess_predict(self, X):
        X = self._f32(X, GUESS_IN)
        Y = self.torch.empty((X.shape[0], GUESS_OUT), dtype=self.torch.float32,
                             device=self.device)
        self._check(self.lib.nls_guess_predict(self.h, self._vp(X), X.shape[0], self._vp(Y)))
        return Y

    def guess_predict_noalloc(self, X, Y):
        """nls_guess_predict_noalloc into the caller's Y (float32, rows x 256,
        on the device); enqueued on the handle's stream, not synchronised."""
        X = self._f32(X, GUESS_IN)
        assert Y.dtype == self.torch.float32 and Y.is_cuda and Y.is_contiguous()
        assert Y.shape == (X.shape[0], GUESS_OUT)
        self._check(self.lib.nls_guess_predict_noalloc(self.h, self._vp(X), X.shape[0],
                                                       self._vp(Y)))
        return Y

    def guess_loss_grad(self, X, T):
        X = self._f32(X, GUESS_IN)
        T = self._f32(T, GUESS_OUT)
        g = self.torch.empty(GUESS_PARAMS, dtype=self.torch.float32, device=self.device)
        loss = ctypes.c_double(0.0)
        self._check(self.lib.nls_guess_loss_grad(self.h, self._vp(X), self._vp(T), X.shape[0],
                                                 self._vp(g), ctypes.byref(loss)))
        return g, loss.value

    def guess_train(self, X, T, epochs, batch=256, lr=1e-3, order=None, fit_norm=True,
                    cosine=False, beta1=0.9, beta2=0.999, eps=1e-8):
        X = self._f32(X, GUESS_IN)
        T = self._f32(T, GUESS_OUT)
        o = TrainOpts(epochs=int(epochs), batch=int(batch), lr=float(lr), beta1=beta1,
                      beta2=beta2, eps=eps,
                      flags=(TRAIN_FIT_NORM if fit_norm else 0) | (TRAIN_COSINE if cosine else 0))
        ordt = None
        if order is not None:
            ordt = self.torch.as_tensor(np.ascontiguousarray(order, dtype=np.int32)).to(self.device)
            assert ordt.numel() == int(epochs) * X.shape[0]
        st = TrainStats()
        self._check(self.lib.nls_guess_train(self.h, ctypes.byref(o), self._vp(X), self._vp(T),
                                             X.shape[0], None if ordt is None else self._vp(ordt),
                                             ctypes.byref(st)))
        return {"steps": st.steps, "final_loss": st.final_loss, "ms": st.ms,
                "epoch_loss": list(st.epoch_loss[:min(int(epochs), MAX_EPOCHS)])}

    def tuning(self):
        """Bucket LU variants, LDS bytes and sizes; coarse apply strategy."""
        ns, _, _ = self.sizes()
        nb = ctypes.c_int32(0)
        var = np.zeros(ns, np.int32)
        lds = np.zeros(ns, np.int32)
        cnt = np.zeros(ns, np.int32)
        ci = ctypes.c_int32(0)
        cms = np.zeros(3, np.float64)
        prec = ctypes.c_int32(0)
        self._check(self.lib.nls_get_tuning(self.h, ctypes.byref(nb), _ptr(var), _ptr(lds),
                                            _ptr(cnt), ctypes.byref(ci), _ptr(cms),
                                            ctypes.byref(prec)))
        k = nb.value
        return {"lu_variant": var[:k].tolist(), "lds_bytes": lds[:k].tolist(),
                "n_sub": cnt[:k].tolist(), "coarse_inverse": bool(ci.value),
                "coarse_ms": cms.tolist(),
                "local_precision": {PREC_FP32_IR: "fp32_ir", PREC_BF16_IR: "bf16_ir"}.get(
                    prec.value, "fp64")}
