"""ctypes binding of the C ABI in include/sem.h (argument marshalling only).

Every computation runs in the HIP library libsemfd.so; torch provides device
memory and the current stream.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsemfd.so")

SEM_BC_DIRICHLET, SEM_BC_NEUMANN, SEM_BC_PERIODIC = 0, 1, 2
_BC = {"dirichlet": SEM_BC_DIRICHLET, "neumann": SEM_BC_NEUMANN, "periodic": SEM_BC_PERIODIC}
SEM_F64, SEM_F32, SEM_BF16, SEM_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"f64": SEM_F64, "f32": SEM_F32, "bf16": SEM_BF16, "bf16x3": SEM_BF16X3}
STATUS = {0: "SEM_OK", 1: "SEM_EINVAL", 2: "SEM_ENOMEM", 3: "SEM_EDEVICE", 4: "SEM_ESINGULAR",
          5: "SEM_ENOCONV", 6: "SEM_ENONFINITE"}


class SemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2310_00226_amd.build_lib)")
    lib = ctypes.CDLL(LIB_PATH)
    dp = POINTER(c_double)
    sig = {
        "sem_plan_create": (c_int, [c_int, POINTER(c_int), dp, c_double, c_int, POINTER(c_void_p)]),
        "sem_plan_create_mixed": (c_int, [c_int, POINTER(c_int), dp, c_double, POINTER(c_int), POINTER(c_void_p)]),
        "sem_plan_destroy": (None, [c_void_p]),
        "sem_plan_dims": (c_int, [c_void_p, POINTER(c_int)]),
        "sem_plan_nodes": (c_int, [c_void_p, c_int, dp]),
        "sem_plan_eigenvalues": (c_int, [c_void_p, c_int, dp]),
        "sem_plan_set_stream": (c_int, [c_void_p, c_void_p]),
        "sem_plan_workspace_bytes": (c_int, [c_void_p, c_int, POINTER(c_size_t)]),
        "sem_plan_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
        "sem_solve": (c_int, [c_void_p, c_void_p, c_void_p]),
        "sem_solve_noalloc": (c_int, [c_void_p, c_void_p, c_void_p]),
        "sem_mode_product": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p]),
        "sem_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
        "sem_lift_boundary": (c_int, [c_void_p, ctypes.POINTER(c_void_p), c_void_p]),
        "sem_solve_refined": (c_int, [c_void_p, c_int, c_double, c_int, c_void_p, c_void_p, POINTER(c_int),
                                      POINTER(c_double)]),
        "sem_solve_lowp": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
        "sem_plan_tune": (c_int, [c_void_p, c_int]),
        "sem_plan_tuning": (c_int, [c_void_p, c_int, POINTER(c_int), POINTER(c_int)]),
        "sem_plan_set_tuning": (c_int, [c_void_p, c_int, POINTER(c_int)]),
        "sem_tune_stats": (c_int, [POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
        "sem_lowp_pass": (c_int, [c_void_p, c_int, c_int, c_int]),
        "sem_apply_spectral": (c_int, [c_void_p, c_int, c_double, c_double, c_void_p, c_void_p]),
        "sem_pcg_workspace_bytes": (c_int, [c_void_p, POINTER(c_size_t)]),
        "sem_pcg_solve": (c_int, [c_void_p, c_void_p, c_double, c_int, c_double, c_int, c_void_p, c_void_p,
                                  c_void_p, c_size_t, POINTER(c_int), POINTER(c_double), POINTER(c_double)]),
        "sem_axis_host": (c_int, [c_int, c_int, c_double, c_double, c_int, POINTER(c_int), dp, dp, dp, dp, dp]),
        "sem_axis_fold_host": (c_int, [c_int, c_int, c_double, c_double, c_int, POINTER(c_int), POINTER(c_int), dp,
                                       dp, dp, dp]),
        "sem_batch_create": (c_int, [c_int, POINTER(c_void_p), POINTER(c_void_p)]),
        "sem_batch_destroy": (None, [c_void_p]),
        "sem_batch_set_stream": (c_int, [c_void_p, c_void_p]),
        "sem_batch_tile_rows": (c_int, [c_void_p, POINTER(c_int)]),
        "sem_batch_solve": (c_int, [c_void_p, c_int, c_double, c_int, POINTER(c_void_p), POINTER(c_void_p),
                                    POINTER(c_int)]),
        "sem_ch_create": (c_int, [c_int, POINTER(c_int), dp, c_double, c_double, c_double, c_int, c_int,
                                  POINTER(c_void_p)]),
        "sem_ch_destroy": (None, [c_void_p]),
        "sem_ch_dims": (c_int, [c_void_p, POINTER(c_int)]),
        "sem_ch_set_stream": (c_int, [c_void_p, c_void_p]),
        "sem_ch_tuning": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
        "sem_ch_set_forcing": (c_int, [c_void_p, c_void_p]),
        "sem_ch_set_graphs": (c_int, [c_void_p, c_int]),
        "sem_ch_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
        "sem_last_error": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int) -> None:
    if status != 0:
        raise SemError(status, lib.sem_last_error().decode())


def _dptr(arr):
    """ctypes double* for a contiguous float64 numpy array (or None)."""
    if arr is None:
        return None
    return arr.ctypes.data_as(POINTER(c_double))


def _dev_ptr(t, name, n=None, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA/HIP torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


def tune_stats():
    """Process-wide tuning-cache counters (sem_tune_stats): dict of hits, misses, entries."""
    h, m, e = c_int(0), c_int(0), c_int(0)
    check(lib.sem_tune_stats(ctypes.byref(h), ctypes.byref(m), ctypes.byref(e)))
    return {"hits": h.value, "misses": m.value, "entries": e.value}


def axis_fold_host(k: int, ne: int, a: float, b: float, bc: str):
    """Reflection-split form of one axis (host only): dict of nrep, nodd, lam_fold,
    ffold (n x nrep), bfold_sym (nrep x nrep), bfold_anti (nrep x nodd)."""
    import numpy as np
    bcv = _BC[bc]
    nr, no = c_int(0), c_int(0)
    check(lib.sem_axis_fold_host(k, ne, a, b, bcv, ctypes.byref(nr), ctypes.byref(no), None, None, None, None))
    nr, no = nr.value, no.value
    n = nr + no
    out = {"nrep": nr, "nodd": no, "lam_fold": np.empty(n), "ffold": np.empty((n, nr)),
           "bfold_sym": np.empty((nr, nr)), "bfold_anti": np.empty((nr, max(no, 0)))}
    check(lib.sem_axis_fold_host(k, ne, a, b, bcv, None, None, _dptr(out["lam_fold"]), _dptr(out["ffold"]),
                                 _dptr(out["bfold_sym"]), _dptr(out["bfold_anti"]) if no else None))
    return out


def axis_host(k: int, ne: int, a: float, b: float, bc: str):
    """1D operators of one axis as built by the plan (host only): dict of x, mass, lam, S, F."""
    import numpy as np
    bcv = _BC[bc]
    n = c_int(0)
    check(lib.sem_axis_host(k, ne, a, b, bcv, ctypes.byref(n), None, None, None, None, None))
    n = n.value
    out = {"x": np.empty(n), "mass": np.empty(n), "lam": np.empty(n), "S": np.empty((n, n)), "F": np.empty((n, n))}
    check(lib.sem_axis_host(k, ne, a, b, bcv, None, _dptr(out["x"]), _dptr(out["mass"]), _dptr(out["lam"]),
                            _dptr(out["S"]), _dptr(out["F"])))
    return out


class Plan:
    """A fast-diagonalisation plan for -Lap u + alpha u = f (sem_plan_create)."""

    def __init__(self, k: int, ne, box, alpha: float, bc: str = "dirichlet", device=None):
        import torch
        self._p = c_void_p(None)
        bcs = (bc,) * 3 if isinstance(bc, str) else tuple(bc)
        if len(bcs) != 3:
            raise ValueError("bc: one name or one per axis")
        bc_arr = (c_int * 3)(*[_BC[b] for b in bcs])
        ne_arr = (c_int * 3)(*[int(v) for v in ne])
        box_arr = (c_double * 6)(*[float(v) for v in box])
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            check(lib.sem_plan_create_mixed(int(k), ne_arr, box_arr, float(alpha), bc_arr, ctypes.byref(self._p)))
        self.k, self.ne, self.box, self.alpha, self.bc = int(k), tuple(ne), tuple(box), float(alpha), bc
        dims = (c_int * 3)()
        check(lib.sem_plan_dims(self._p, dims))
        self.shape = tuple(dims)
        self.numel = self.shape[0] * self.shape[1] * self.shape[2]
        self._ws = {}

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and p.value:
            lib.sem_plan_destroy(p)
            self._p = c_void_p(None)

    def close(self):
        self.__del__()

    def nodes(self, axis: int):
        import numpy as np
        x = np.empty(self.shape[axis])
        check(lib.sem_plan_nodes(self._p, axis, _dptr(x)))
        return x

    def eigenvalues(self, axis: int):
        import numpy as np
        x = np.empty(self.shape[axis])
        check(lib.sem_plan_eigenvalues(self._p, axis, _dptr(x)))
        return x

    def _prepare(self, prec: int):
        """Bind torch's current stream and a torch-allocated workspace."""
        import torch
        check(lib.sem_plan_set_stream(self._p, c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        need = c_size_t(0)
        check(lib.sem_plan_workspace_bytes(self._p, prec, ctypes.byref(need)))
        ws = self._ws.get("buf")
        if ws is None or ws.numel() < need.value:
            ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device=self.device)
            self._ws["buf"] = ws
            check(lib.sem_plan_set_workspace(self._p, c_void_p(ws.data_ptr()), ws.numel()))

    def solve(self, f, u=None):
        import torch
        if u is None:
            u = torch.empty_like(f)
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        up = _dev_ptr(u, "u", self.numel, torch.float64)
        self._prepare(SEM_F64)
        check(lib.sem_solve(self._p, fp, up))
        return u

    def solve_noalloc(self, f, u=None):
        """The FP64 solve with the library's fixed scratch array (sem_solve_noalloc):
        binds torch's current stream, installs no workspace, allocates nothing
        (except u when it is not given)."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        up = _dev_ptr(u, "u", self.numel, torch.float64)
        check(lib.sem_plan_set_stream(self._p, c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        check(lib.sem_solve_noalloc(self._p, fp, up))
        return u

    def solve_refined(self, f, u=None, prec: str = "bf16", tol: float = 1e-11, max_iter: int = 30,
                      raise_on_error: bool = True):
        """Mixed-precision solve with FP64 refinement (sem_solve_refined).

        Returns (u, iterations, last relative update, status)."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        up = _dev_ptr(u, "u", self.numel, torch.float64)
        self._prepare(pv)
        it = c_int(0)
        rel = c_double(0.0)
        st = lib.sem_solve_refined(self._p, pv, float(tol), int(max_iter), fp, up, ctypes.byref(it), ctypes.byref(rel))
        if raise_on_error:
            check(st)
        return u, it.value, rel.value, st

    def solve_lowp(self, f, u=None, prec: str = "bf16x3"):
        """One unrefined solve with low-precision mode products (sem_solve_lowp)."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        up = _dev_ptr(u, "u", self.numel, torch.float64)
        self._prepare(pv)
        check(lib.sem_solve_lowp(self._p, pv, fp, up))
        return u

    def tune(self, prec: str = "bf16x3"):
        """Tune the launch shapes of prec now (sem_plan_tune); returns tuning(prec)."""
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self._prepare(pv)
        check(lib.sem_plan_tune(self._p, pv))
        return self.tuning(pv)

    def tuning(self, prec: str = "bf16x3"):
        """The shapes of prec's six passes (sem_plan_tuning), or None before tuning."""
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        tuned = c_int(0)
        ch = (c_int * 6)()
        check(lib.sem_plan_tuning(self._p, pv, ctypes.byref(tuned), ch))
        return list(ch) if tuned.value else None

    def set_tuning(self, prec: str, choice):
        """Install the six pass shapes of prec without timing (sem_plan_set_tuning)."""
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        ch = (c_int * 6)(*[int(c) for c in choice])
        check(lib.sem_plan_set_tuning(self._p, pv, ch))

    def lowp_pass(self, prec: str, pass_index: int, reps: int = 1):
        """Launch one pass of prec's FD application reps times (sem_lowp_pass), for timing."""
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self._prepare(pv)
        check(lib.sem_lowp_pass(self._p, pv, int(pass_index), int(reps)))

    def apply_spectral(self, kind: str, a: float, param: float, f, u=None):
        """u = g(H_3 + a I) f with g(x) = exp(-param x) ("exp") or x^(-param) ("power")
        (sem_apply_spectral)."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        kv = {"exp": 1, "power": 2}[kind]
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        up = _dev_ptr(u, "u", self.numel, torch.float64)
        self._prepare(SEM_F64)
        check(lib.sem_apply_spectral(self._p, kv, float(a), float(param), fp, up))
        return u

    def pcg_solve(self, v, f, u=None, shift: float = None, prec: str = "f64", tol: float = 1e-12,
                  max_iter: int = 500, raise_on_error: bool = True):
        """alpha u - Lap u + V u = f by PCG with the FD solve of (shift I - Lap) as
        preconditioner (sem_pcg_solve); v is the potential at the nodes (>= 0),
        shift None lets the library take alpha + max(v)/2.  Returns (u, iterations,
        final relative residual, status); the shift used is kept in last_pcg_shift."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        vp = _dev_ptr(v, "v", self.numel, torch.float64)
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        up = _dev_ptr(u, "u", self.numel, torch.float64)
        self._prepare(pv)
        need = c_size_t(0)
        check(lib.sem_pcg_workspace_bytes(self._p, ctypes.byref(need)))
        work = self._ws.get("pcg")
        if work is None or work.numel() < need.value:
            work = torch.empty(need.value, dtype=torch.uint8, device=self.device)
            self._ws["pcg"] = work
        it = c_int(0)
        rel = c_double(0.0)
        used = c_double(0.0)
        st = lib.sem_pcg_solve(self._p, vp, 0.0 if shift is None else float(shift), pv, float(tol), int(max_iter),
                               fp, up, c_void_p(work.data_ptr()), work.numel(), ctypes.byref(it), ctypes.byref(rel),
                               ctypes.byref(used))
        self.last_pcg_shift = used.value
        if raise_on_error:
            check(st)
        return u, it.value, rel.value, st

    def mode_product(self, axis: int, inverse: bool, x, out=None):
        import torch
        if out is None:
            out = torch.empty_like(x)
        xp = _dev_ptr(x, "in", self.numel, torch.float64)
        op = _dev_ptr(out, "out", self.numel, torch.float64)
        self._prepare(SEM_F64)
        check(lib.sem_mode_product(self._p, int(axis), int(bool(inverse)), xp, op))
        return out

    def residual(self, u, f, r=None):
        import torch
        if r is None:
            r = torch.empty_like(u)
        a = _dev_ptr(u, "u", self.numel, torch.float64)
        b = _dev_ptr(f, "f", self.numel, torch.float64)
        c = _dev_ptr(r, "r", self.numel, torch.float64)
        self._prepare(SEM_F64)
        check(lib.sem_residual(self._p, a, b, c))
        return r

    def lift_boundary(self, faces, f):
        """Add the terms of non-homogeneous boundary data to the right-hand side f
        in place (sem_lift_boundary); faces: six tensors or None, face 2a / 2a+1 of
        the shape of the plan without axis a.  Returns f."""
        import torch
        if len(faces) != 6:
            raise ValueError("faces: expected six entries (x lower, x upper, y lower, ...)")
        fp = _dev_ptr(f, "f", self.numel, torch.float64)
        arr = (c_void_p * 6)()
        for i, g in enumerate(faces):
            if g is None:
                continue
            a = i // 2
            m = self.numel // self.shape[a]
            arr[i] = _dev_ptr(g, f"faces[{i}]", m, torch.float64).value
        check(lib.sem_plan_set_stream(self._p, c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        check(lib.sem_lift_boundary(self._p, arr, fp))
        return f


class CahnHilliard:
    """Cahn-Hilliard IMEX stepper (sem_ch_create / sem_ch_step), homogeneous Neumann."""

    def __init__(self, k: int, ne, box, eps: float, mob: float, dt: float, prec: str = "f32",
                 refine_sweeps: int = 2, graphs: bool = True, device=None):
        import torch
        self._c = c_void_p(None)
        ne_arr = (c_int * 3)(*[int(v) for v in ne])
        box_arr = (c_double * 6)(*[float(v) for v in box])
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            check(lib.sem_ch_create(int(k), ne_arr, box_arr, float(eps), float(mob), float(dt), pv,
                                    int(refine_sweeps), ctypes.byref(self._c)))
        dims = (c_int * 3)()
        check(lib.sem_ch_dims(self._c, dims))
        self.shape = tuple(dims)
        self.numel = self.shape[0] * self.shape[1] * self.shape[2]
        check(lib.sem_ch_set_graphs(self._c, 1 if graphs else 0))

    def __del__(self):
        c = getattr(self, "_c", None)
        if c is not None and c.value:
            lib.sem_ch_destroy(c)
            self._c = c_void_p(None)

    def close(self):
        self.__del__()

    def set_graphs(self, enable: bool):
        check(lib.sem_ch_set_graphs(self._c, 1 if enable else 0))

    def tuning(self):
        """Launch shapes of the stepper's six mode products (sem_ch_tuning), or None."""
        tuned = c_int(0)
        ch = (c_int * 6)()
        check(lib.sem_ch_tuning(self._c, ctypes.byref(tuned), ch))
        return list(ch) if tuned.value else None

    def set_forcing(self, s=None):
        """Source term read by every following step at the new time level (or None)."""
        import torch
        if s is None:
            self._forcing = None
            check(lib.sem_ch_set_forcing(self._c, c_void_p(None)))
            return
        ptr = _dev_ptr(s, "s", self.numel, torch.float64)
        self._forcing = s  # keep the array alive while the stepper may read it
        check(lib.sem_ch_set_forcing(self._c, ptr))

    def step(self, phi_n, phi_nm1, nsteps: int = 1):
        """Advance in place: on return phi_n, phi_nm1 hold phi_{n+nsteps}, phi_{n+nsteps-1}."""
        import torch
        a = _dev_ptr(phi_n, "phi_n", self.numel, torch.float64)
        b = _dev_ptr(phi_nm1, "phi_nm1", self.numel, torch.float64)
        check(lib.sem_ch_set_stream(self._c, c_void_p(torch.cuda.current_stream(self.device).cuda_stream)))
        check(lib.sem_ch_step(self._c, a, b, int(nsteps)))


class Batch:
    """Batched solves over several plans (sem_batch_create / sem_batch_solve)."""

    def __init__(self, plans):
        import torch
        self.plans = list(plans)  # keep the plans alive
        arr = (c_void_p * len(self.plans))(*[p._p.value for p in self.plans])
        self._b = c_void_p(None)
        with torch.cuda.device(self.plans[0].device):
            check(lib.sem_batch_create(len(self.plans), arr, ctypes.byref(self._b)))

    def __del__(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value:
            lib.sem_batch_destroy(b)
            self._b = c_void_p(None)

    def close(self):
        self.__del__()

    def tile_rows(self):
        rows = (c_int * 6)()
        check(lib.sem_batch_tile_rows(self._b, rows))
        return list(rows)

    def solve(self, fs, us, prec: str = "f32", tol: float = 1e-11, max_iter: int = 30,
              raise_on_error: bool = True):
        """Solve every problem; returns (per-problem iterations, status)."""
        import torch
        n = len(self.plans)
        if len(fs) != n or len(us) != n:
            raise ValueError("one right-hand side and one solution per plan")
        fp = (c_void_p * n)(*[_dev_ptr(f, f"f[{i}]", p.numel, torch.float64).value
                              for i, (f, p) in enumerate(zip(fs, self.plans))])
        up = (c_void_p * n)(*[_dev_ptr(u, f"u[{i}]", p.numel, torch.float64).value
                              for i, (u, p) in enumerate(zip(us, self.plans))])
        pv = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        its = (c_int * n)()
        check(lib.sem_batch_set_stream(self._b, c_void_p(torch.cuda.current_stream(self.plans[0].device).cuda_stream)))
        st = lib.sem_batch_solve(self._b, pv, float(tol), int(max_iter), fp, up, its)
        if raise_on_error:
            check(st)
        return list(its), st
