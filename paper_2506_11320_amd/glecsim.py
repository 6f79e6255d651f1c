"""Python binding of libglecsim.so (the gfx950 GL-ECSIM library).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  There is no
CPU fallback: if the library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglecsim.so")

GE_OK = 0
GE_ERR_ARG, GE_ERR_OOM, GE_ERR_HIP, GE_ERR_CFL, GE_ERR_NONFINITE, GE_ERR_STATE = -1, -2, -3, -4, -5, -6
GE_WARN_NOT_CONVERGED = 1
GE_FP64, GE_FP32 = 0, 1
GE_A_LIGHT, GE_A_BULK = 0, 1
GE_PC_NONE, GE_PC_JACOBI, GE_PC_CNN = 0, 1, 2
GE_LAG_EN, GE_PICARD1 = 0, 1
GE_HARVEST_SOLUTION, GE_HARVEST_KRYLOV = 1, 2
FIELDS = {
    "E": 0, "B": 1, "Eth": 2, "Bn": 3, "J_lab": 4, "J_eff": 5, "rho": 6, "mm": 7, "mass": 8, "u": 9,
    "EM": 10, "Mt": 11, "M0": 12, "kappa_E": 13, "kappa_B": 14, "rhs": 15, "psi": 16,
}
EXPORTS = [
    "ge_create", "ge_destroy", "ge_last_error", "ge_add_species", "ge_set_fields", "ge_deposit", "ge_solve_fields",
    "ge_push", "ge_update_fields", "ge_step", "ge_sync", "ge_gather", "ge_set", "ge_half_stencil",
    "ge_get_particles", "ge_apply_operator", "ge_diagnostics", "ge_timings", "ge_explicit_current", "ge_explicit_step",
    "ge_moves", "ge_diagnostics_noalloc", "ge_step_count", "ge_species_count", "ge_checkpoint", "ge_restore",
    "ge_inject",
    "ge_cnn_init", "ge_cnn_size", "ge_cnn_weights", "ge_cnn_apply", "ge_cnn_apply_scaled", "ge_cnn_harvest",
    "ge_cnn_add_pair",
    "ge_cnn_npairs", "ge_cnn_train", "ge_cnn_loss_grad",
]


GE_BC_PERIODIC, GE_BC_WALL, GE_BC_INFLOW = 0, 1, 2


class GEGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3)]


class GEParams(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("c", ctypes.c_double), ("dt", ctypes.c_double),
                ("lf_E", ctypes.c_int), ("lf_B", ctypes.c_int), ("beta_lim", ctypes.c_double),
                ("a_mode", ctypes.c_int), ("a_const", ctypes.c_double), ("comoving", ctypes.c_int),
                ("n_smooth_u", ctypes.c_int), ("phi_u", ctypes.c_double), ("precision", ctypes.c_int),
                ("ns_j", ctypes.c_int), ("dedner", ctypes.c_int), ("ch_frac", ctypes.c_double),
                ("dedner_damp", ctypes.c_double), ("ns_e", ctypes.c_int), ("limiter_lag", ctypes.c_int)]


class GESpecies(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double)]


class GESolveReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres", ctypes.c_double), ("bnorm", ctypes.c_double), ("seconds", ctypes.c_double),
                ("fallback", ctypes.c_int)]


class GETrainCfg(ctypes.Structure):
    _fields_ = [("crop", ctypes.c_int), ("batch", ctypes.c_int), ("iters", ctypes.c_int), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint32)]


class GETrainReport(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("pairs", ctypes.c_int), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("seconds", ctypes.c_double)]


class GEDiag(ctypes.Structure):
    _fields_ = [("W_E", ctypes.c_double), ("W_B", ctypes.c_double), ("K", ctypes.c_double * 4),
                ("P", (ctypes.c_double * 3) * 4), ("gauss", ctypes.c_double), ("nsp", ctypes.c_int)]


class GEMoveReport(ctypes.Structure):
    _fields_ = [("far_moves", ctypes.c_int64 * 4), ("max_move", ctypes.c_double * 4), ("resorts", ctypes.c_int),
                ("pushes", ctypes.c_int), ("gone", ctypes.c_int64 * 4), ("injected", ctypes.c_int64 * 4)]


class GlecsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"glecsim error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libglecsim.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2506_11320_amd/build.py (no CPU fallback)")
    L = ctypes.CDLL(path)
    vp, i64, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    L.ge_create.argtypes = [ctypes.POINTER(GEGrid), ctypes.POINTER(GEParams), vp, ctypes.POINTER(vp)]
    L.ge_destroy.argtypes = [vp]
    L.ge_destroy.restype = None
    L.ge_last_error.argtypes = [vp]
    L.ge_last_error.restype = ctypes.c_char_p
    L.ge_add_species.argtypes = [vp, ctypes.POINTER(GESpecies), i64, vp, vp, vp, vp]
    L.ge_set_fields.argtypes = [vp, vp, vp]
    for name in ["ge_deposit", "ge_push", "ge_update_fields", "ge_sync"]:
        getattr(L, name).argtypes = [vp]
    L.ge_solve_fields.argtypes = [vp, d, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(GESolveReport)]
    L.ge_step.argtypes = [vp, d, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(GESolveReport)]
    L.ge_gather.argtypes = [vp, ctypes.c_int, vp]
    L.ge_set.argtypes = [vp, ctypes.c_int, vp]
    L.ge_half_stencil.argtypes = [vp]
    L.ge_get_particles.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, vp]
    L.ge_apply_operator.argtypes = [vp, vp, vp]
    L.ge_explicit_current.argtypes = [vp, vp]
    L.ge_explicit_step.argtypes = [vp]
    L.ge_diagnostics.argtypes = [vp, ctypes.POINTER(GEDiag)]
    L.ge_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.ge_moves.argtypes = [vp, ctypes.POINTER(GEMoveReport)]
    L.ge_diagnostics_noalloc.argtypes = [vp, ctypes.POINTER(GEDiag)]
    L.ge_step_count.argtypes = [vp]
    L.ge_step_count.restype = ctypes.c_int64
    L.ge_inject.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, vp]
    L.ge_species_count.argtypes = [vp, ctypes.c_int]
    L.ge_species_count.restype = ctypes.c_int64
    L.ge_checkpoint.argtypes = [vp, ctypes.c_char_p]
    L.ge_restore.argtypes = [vp, ctypes.c_char_p]
    L.ge_cnn_init.argtypes = [vp, ctypes.c_uint32, ctypes.c_int]
    L.ge_cnn_size.argtypes = []
    L.ge_cnn_weights.argtypes = [vp, ctypes.c_int, vp]
    L.ge_cnn_apply.argtypes = [vp, vp, vp]
    L.ge_cnn_apply_scaled.argtypes = [vp, vp, vp, ctypes.c_double]
    L.ge_cnn_harvest.argtypes = [vp, ctypes.c_int]
    L.ge_cnn_add_pair.argtypes = [vp, vp, vp]
    L.ge_cnn_npairs.argtypes = [vp]
    L.ge_cnn_train.argtypes = [vp, ctypes.POINTER(GETrainCfg), ctypes.POINTER(GETrainReport)]
    L.ge_cnn_loss_grad.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
    _lib = L
    return L


def _require(ok: bool, msg: str) -> None:
    """Argument checks that guard the device pointers handed to the library
    (kept under python -O, unlike assert)."""
    if not ok:
        raise ValueError(msg)


def _ptr(t: torch.Tensor) -> int:
    _require(t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors")
    return t.data_ptr()


class Simulation:
    """One GL-ECSIM context on one GPU (see include/glecsim.h)."""

    def __init__(self, dim: int, n, dx, *, theta: float, dt: float, c: float = 1.0, lf_E: bool = True,
                 lf_B: bool = True, beta_lim: float = 1.0, a_mode: int = GE_A_BULK, a_const: float = 1.0,
                 comoving: bool = True, n_smooth_u: int = 5, phi_u: float = 0.5, fp32: bool = False,
                 ns_j: int = 0, dedner: bool = False, ch_frac: float = 0.8, dedner_damp: float = 0.1,
                 ns_e: int = 0, limiter_lag: int = GE_LAG_EN, bc=(GE_BC_PERIODIC, GE_BC_PERIODIC),
                 device: str = "cuda:0", stream: Optional[torch.cuda.Stream] = None):
        """bc: the x axis's (low, high) boundary kinds; with a wall the grid
        stores n[0] + 1 points along x (see ge_grid)."""
        if not torch.cuda.is_available():
            raise RuntimeError("glecsim needs a GPU (no CPU fallback)")
        self.L = load_library()
        self.device = torch.device(device)
        self.dim = dim
        self.n = tuple(int(n[d]) if d < dim else 1 for d in range(3))
        self.bc = (int(bc[0]), int(bc[1]))
        self.N = 1
        for d in range(dim):
            self.N *= self.n[d] + (1 if d == 0 and self.bc[0] != GE_BC_PERIODIC else 0)
        self.fp32 = fp32
        self.fdtype = torch.float32 if fp32 else torch.float64
        g = GEGrid()
        g.dim = dim
        for d in range(3):
            g.n[d] = self.n[d]
            g.dx[d] = float(dx[d]) if d < dim else 1.0
        g.bc_lo[0], g.bc_hi[0] = self.bc
        p = GEParams(theta, c, dt, int(lf_E), int(lf_B), beta_lim, a_mode, a_const, int(comoving), n_smooth_u,
                     phi_u, GE_FP32 if fp32 else GE_FP64, int(ns_j), int(dedner), ch_frac, dedner_damp,
                     int(ns_e), int(limiter_lag))
        self.params = p
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.L.ge_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(h))
        if rc != GE_OK:
            raise GlecsimError(rc, self.L.ge_last_error(None).decode())
        self.h = h
        self.nsp = 0
        self.counts = []

    # -------------------------------------------------------------- plumbing
    def _check(self, rc: int, allow_warn: bool = False) -> int:
        if rc < 0 or (rc > 0 and not allow_warn):
            raise GlecsimError(rc, self.L.ge_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.L.ge_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- setup
    def add_species(self, q: float, m: float, cell: torch.Tensor, off: torch.Tensor, v: torch.Tensor,
                    w: torch.Tensor):
        n = int(cell.numel())
        _require(cell.dtype == torch.int32, "cell must be int32")
        _require(off.dtype == v.dtype == w.dtype == self.fdtype, f"off, v and w must be {self.fdtype}")
        _require(off.shape == (3, n) and v.shape == (3, n) and w.shape == (n,), "off, v: [3, n]; w: [n]")
        sp = GESpecies(q, m)
        self._check(self.L.ge_add_species(self.h, ctypes.byref(sp), n, _ptr(cell), _ptr(off), _ptr(v), _ptr(w)))
        self.nsp += 1
        self.counts.append(n)

    def set_fields(self, E: torch.Tensor, B: torch.Tensor):
        _require(E.dtype == torch.float64 and B.dtype == torch.float64, "E and B must be float64")
        _require(E.shape == (3, self.N) and B.shape == (3, self.N), "E and B: [3, N]")
        self._check(self.L.ge_set_fields(self.h, _ptr(E), _ptr(B)))

    # -------------------------------------------------------------- step
    def deposit(self):
        self._check(self.L.ge_deposit(self.h))

    def solve(self, tol: float = 1e-8, maxit: int = 1000, restart: int = 30, precond: int = GE_PC_NONE) -> Dict:
        r = GESolveReport()
        rc = self._check(self.L.ge_solve_fields(self.h, tol, maxit, restart, precond, ctypes.byref(r)), True)
        return {"iterations": r.iterations, "restarts": r.restarts, "converged": bool(r.converged),
                "relres": r.relres, "bnorm": r.bnorm, "seconds": r.seconds, "fallback": bool(r.fallback), "rc": rc}

    def push(self):
        self._check(self.L.ge_push(self.h))

    def explicit_step(self):
        """One explicit PIC step with the explicit-form current (see glecsim.h)."""
        self._check(self.L.ge_explicit_step(self.h))

    def explicit_current(self) -> torch.Tensor:
        """Explicit-PIC current at the present particle state (see glecsim.h)."""
        J = torch.empty((3, self.N), dtype=torch.float64, device=self.device)
        self._check(self.L.ge_explicit_current(self.h, _ptr(J)))
        return J

    def update_fields(self):
        self._check(self.L.ge_update_fields(self.h))

    def step(self, tol: float = 1e-8, maxit: int = 1000, restart: int = 30, precond: int = GE_PC_NONE) -> Dict:
        r = GESolveReport()
        rc = self._check(self.L.ge_step(self.h, tol, maxit, restart, precond, ctypes.byref(r)), True)
        return {"iterations": r.iterations, "converged": bool(r.converged), "relres": r.relres, "rc": rc,
                "seconds": r.seconds, "fallback": bool(r.fallback)}

    def sync(self):
        self._check(self.L.ge_sync(self.h))

    def step_count(self) -> int:
        return int(self.L.ge_step_count(self.h))

    def checkpoint(self, path: str):
        self._check(self.L.ge_checkpoint(self.h, os.fsencode(path)))

    def restore(self, path: str):
        """Restore a checkpoint into this (species-less) context; the species
        counts come from the file."""
        self._check(self.L.ge_restore(self.h, os.fsencode(path)))
        d = GEDiag()
        self._check(self.L.ge_diagnostics(self.h, ctypes.byref(d)))
        self.nsp = d.nsp
        self.counts = [self._species_count(s) for s in range(self.nsp)]

    def _species_count(self, s: int) -> int:
        return int(self.L.ge_species_count(self.h, s))

    # -------------------------------------------------------------- data
    def half_stencil(self) -> int:
        return int(self.L.ge_half_stencil(self.h))

    def field_shape(self, what: str):
        N = self.N
        if what in ("rho",):
            return (self.nsp, N)
        if what in ("mass", "psi"):
            return (N,)
        if what in ("Mt", "M0"):
            return (self.half_stencil(), 9, N)
        if what in ("kappa_E", "kappa_B"):
            return (3, 3, N)
        return (3, N)

    def gather(self, what: str) -> torch.Tensor:
        out = torch.empty(self.field_shape(what), dtype=torch.float64, device=self.device)
        self._check(self.L.ge_gather(self.h, FIELDS[what], _ptr(out)))
        return out

    def set(self, what: str, src: torch.Tensor):
        src = src.to(device=self.device, dtype=torch.float64).contiguous()
        _require(tuple(src.shape) == self.field_shape(what), f"{what}: shape {self.field_shape(what)}")
        self._check(self.L.ge_set(self.h, FIELDS[what], _ptr(src)))
        self._keep = src  # keep alive until the stream has copied it

    def inject(self, s: int, cell: torch.Tensor, off: torch.Tensor, v: torch.Tensor, w: torch.Tensor):
        """Particles entering species s (see ge_inject)."""
        n = int(cell.numel())
        _require(cell.dtype == torch.int32, "cell must be int32")
        _require(off.dtype == v.dtype == w.dtype == self.fdtype, f"off, v and w must be {self.fdtype}")
        _require(off.shape == (3, n) and v.shape == (3, n) and w.shape == (n,), "off, v: [3, n]; w: [n]")
        if n == 0:
            return
        self._check(self.L.ge_inject(self.h, s, n, _ptr(cell), _ptr(off), _ptr(v), _ptr(w)))
        self._keep = (cell, off, v, w)  # alive until the stream has packed them

    def count(self, s: int) -> int:
        """Live particles of species s (settles the last push)."""
        self.sync()
        return int(self.L.ge_species_count(self.h, s))

    def particles(self, s: int) -> Dict[str, torch.Tensor]:
        n = self.count(s)
        cell = torch.empty(n, dtype=torch.int32, device=self.device)
        off = torch.empty((3, n), dtype=self.fdtype, device=self.device)
        v = torch.empty((3, n), dtype=self.fdtype, device=self.device)
        w = torch.empty(n, dtype=self.fdtype, device=self.device)
        self._check(self.L.ge_get_particles(self.h, s, n, _ptr(cell), _ptr(off), _ptr(v), _ptr(w)))
        return {"cell": cell, "off": off, "v": v, "w": w}

    def apply_operator(self, x: torch.Tensor) -> torch.Tensor:
        x = x.to(device=self.device, dtype=torch.float64).contiguous()
        y = torch.empty_like(x)
        self._check(self.L.ge_apply_operator(self.h, _ptr(x), _ptr(y)))
        return y

    def diagnostics(self, noalloc: bool = False) -> Dict:
        """FP64 energies, momenta and Gauss residual (ge_diagnostics, or its
        allocation-free variant ge_diagnostics_noalloc)."""
        dg = GEDiag()
        fn = self.L.ge_diagnostics_noalloc if noalloc else self.L.ge_diagnostics
        self._check(fn(self.h, ctypes.byref(dg)))
        return {"W_E": dg.W_E, "W_B": dg.W_B, "K": [dg.K[s] for s in range(self.nsp)],
                "P": [[dg.P[s][d] for d in range(3)] for s in range(self.nsp)], "gauss": dg.gauss}

    # -------------------------------------------------- learned preconditioner
    def cnn_init(self, seed: int = 0, max_pairs: int = 0):
        self._check(self.L.ge_cnn_init(self.h, seed, max_pairs))

    def cnn_size(self) -> int:
        return int(self.L.ge_cnn_size())

    def cnn_weights(self) -> "numpy.ndarray":
        import numpy as np
        w = np.empty(self.cnn_size(), dtype=np.float32)
        self._check(self.L.ge_cnn_weights(self.h, 0, w.ctypes.data))
        return w

    def cnn_set_weights(self, w) -> None:
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        _require(w.shape == (self.cnn_size(),), "weights: one vector of cnn_size() values")
        self._check(self.L.ge_cnn_weights(self.h, 1, w.ctypes.data))

    def cnn_apply(self, r: torch.Tensor) -> torch.Tensor:
        r = r.to(device=self.device, dtype=torch.float64).contiguous()
        _require(tuple(r.shape) == (3, self.N), "r: [3, N]")
        z = torch.empty_like(r)
        self._check(self.L.ge_cnn_apply(self.h, _ptr(r), _ptr(z)))
        return z

    def cnn_apply_scaled(self, r: torch.Tensor, scale: float, z: torch.Tensor = None) -> torch.Tensor:
        r = r.to(device=self.device, dtype=torch.float64).contiguous()
        _require(tuple(r.shape) == (3, self.N), "r: [3, N]")
        if z is None:
            z = torch.empty_like(r)
        _require(tuple(z.shape) == (3, self.N) and z.dtype == torch.float64 and z.is_contiguous(), "z: [3, N] float64")
        self._check(self.L.ge_cnn_apply_scaled(self.h, _ptr(r), _ptr(z), float(scale)))
        return z

    def cnn_harvest(self, flags: int = GE_HARVEST_SOLUTION):
        self._check(self.L.ge_cnn_harvest(self.h, int(flags)))

    def cnn_add_pair(self, r: torch.Tensor, e: torch.Tensor):
        r = r.to(device=self.device, dtype=torch.float64).contiguous()
        e = e.to(device=self.device, dtype=torch.float64).contiguous()
        _require(tuple(r.shape) == (3, self.N) and tuple(e.shape) == (3, self.N), "r and e: [3, N]")
        self._check(self.L.ge_cnn_add_pair(self.h, _ptr(r), _ptr(e)))

    def cnn_npairs(self) -> int:
        return int(self.L.ge_cnn_npairs(self.h))

    def cnn_train(self, crop: int = 16, batch: int = 8, iters: int = 200, lr: float = 1e-3, beta1: float = 0.9,
                  beta2: float = 0.999, eps: float = 1e-8, seed: int = 1) -> Dict:
        cfg = GETrainCfg(crop, batch, iters, lr, beta1, beta2, eps, seed)
        rep = GETrainReport()
        self._check(self.L.ge_cnn_train(self.h, ctypes.byref(cfg), ctypes.byref(rep)))
        return {"steps": rep.steps, "pairs": rep.pairs, "loss_first": rep.loss_first, "loss_last": rep.loss_last,
                "seconds": rep.seconds}

    def cnn_loss_grad(self, in_crops: torch.Tensor, tgt: torch.Tensor):
        """in_crops [B, (n+6)^3, 3], tgt [B, n^3, 3] (FP32, crop-local x-fastest order)."""
        in_crops = in_crops.to(device=self.device, dtype=torch.float32).contiguous()
        tgt = tgt.to(device=self.device, dtype=torch.float32).contiguous()
        B, v6 = in_crops.shape[0], in_crops.shape[1]
        n = round(v6 ** (1.0 / 3.0)) - 6
        _require((n + 6) ** 3 == v6 and tuple(tgt.shape) == (B, n ** 3, 3), "in_crops [B, (n+6)^3, 3], tgt [B, n^3, 3]")
        g = torch.empty(self.cnn_size(), dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._check(self.L.ge_cnn_loss_grad(self.h, B, n, _ptr(in_crops), _ptr(tgt), _ptr(g), ctypes.byref(loss)))
        return loss.value, g

    def moves(self) -> Dict:
        """Particle moves since the last call (see ge_moves)."""
        r = GEMoveReport()
        self._check(self.L.ge_moves(self.h, ctypes.byref(r)))
        return {"far_moves": [int(r.far_moves[s]) for s in range(self.nsp)],
                "max_move": [float(r.max_move[s]) for s in range(self.nsp)],
                "resorts": int(r.resorts), "pushes": int(r.pushes),
                "gone": [int(r.gone[s]) for s in range(self.nsp)],
                "injected": [int(r.injected[s]) for s in range(self.nsp)]}

    def timings(self):
        out = (ctypes.c_double * 8)()
        self._check(self.L.ge_timings(self.h, out))
        return list(out)
