"""FP64 CPU oracle of the GL-ECSIM particle pass and field step.

TEST INFRASTRUCTURE ONLY: plain, slow loops in double precision (C, in
``glecsim_oracle.c``, driven from here through ctypes), used by the tests,
the smoke check and the benchmark's CPU-baseline leg.  The product path never
imports it, and it shares no code with the GPU library.

Paper: Chen, Zhou & Toth, arXiv 2506.11320.  Section references are given
per function; readings of silent or garbled passages are listed in the C
source next to each function.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glecsim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_d = ctypes.c_double
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


BC_PERIODIC, BC_WALL, BC_INFLOW = 0, 1, 2


class Grid(ctypes.Structure):
    # bc_lo, bc_hi: the x axis's boundaries (see glecsim_oracle.h); a walled
    # grid stores n[0] = nx + 1 points along x (ghost cell nx)
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("bc_lo", ctypes.c_int), ("bc_hi", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("c", ctypes.c_double), ("dt", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        G = ctypes.POINTER(Grid)
        P = ctypes.POINTER(Params)
        L.or_limiter.restype = _d
        L.or_limiter.argtypes = [_d, _d, _d]
        L.or_alpha.argtypes = [_d, _p, _p]
        L.or_shape.restype = ctypes.c_int
        L.or_shape.argtypes = [G, _p, _p, _p]
        L.or_node_avg.argtypes = [G, _p, _p]
        L.or_deposit_species.argtypes = [G, _d, _d, _d, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.or_bulk_velocity.argtypes = [G, _p, _p, _p]
        L.or_filter_axis.argtypes = [G, _p, ctypes.c_int, _d, ctypes.c_int, ctypes.c_int]
        L.or_smooth.argtypes = [G, _p, ctypes.c_int, ctypes.c_int, _d]
        L.or_motional.argtypes = [G, _p, _p, _p]
        L.or_mass_apply.argtypes = [G, _p, _p, _p]
        L.or_current_eff.argtypes = [G, _p, _p, _p, _p]
        L.or_kappa_E.argtypes = [G, _p, _p, _d, _p]
        L.or_kappa_B.argtypes = [G, _p, _p, _d, _p]
        L.or_curl_nc.argtypes = [G, _p, _p]
        L.or_curl_cn.argtypes = [G, _p, _p]
        L.or_div_nc.argtypes = [G, _p, _p]
        L.or_gauss_sums.argtypes = [G, _p, _p, _p]
        L.or_diffusion.argtypes = [G, _p, _p, _p]
        L.or_apply_A.argtypes = [G, P, _p, _p, _p, _p]
        L.or_rhs.argtypes = [G, P, _p, _p, _p, _p]
        L.or_update_B.argtypes = [G, P, _p, _p, _p, _p]
        L.or_update_E.argtypes = [_i64, _d, _p, _p, _p]
        L.or_push_species.argtypes = [G, _d, _d, _i64, _p, _p, _p, _p, _p, _p, _p]
        L.or_gmres.restype = ctypes.c_int
        L.or_gmres.argtypes = [G, P, _p, _p, _p, _p, _d, ctypes.c_int, ctypes.c_int, _p]
        L.or_dense_A.argtypes = [G, P, _p, _p, _p]
        L.or_dense_solve.restype = ctypes.c_int
        L.or_dense_solve.argtypes = [_i64, _p, _p, _p]
        L.or_advect.argtypes = [ctypes.c_int, _p, _d, _d, ctypes.c_int, _d]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"] and a.dtype == np.float64, (a.dtype, a.flags)
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def grid(dim: int, n, dx, bc=(BC_PERIODIC, BC_PERIODIC)) -> Grid:
    """n: cells per axis; with walls on x (bc = (BC_WALL, BC_WALL or
    BC_INFLOW)) n[0] counts the physical cells and the grid stores n[0] + 1
    points along x."""
    g = Grid()
    g.dim = dim
    for d in range(3):
        g.n[d] = int(n[d]) if d < dim else 1
        g.dx[d] = float(dx[d]) if d < dim else 1.0
    g.bc_lo, g.bc_hi = int(bc[0]), int(bc[1])
    if g.bc_lo != BC_PERIODIC:
        g.n[0] += 1
    return g


def walled(G: Grid) -> bool:
    return G.bc_lo != BC_PERIODIC


def physical_cells(G: Grid) -> np.ndarray:
    """Mask of the physical cells of the storage grid (all but the ghost
    cell column of a walled grid)."""
    N = nnodes(G)
    if not walled(G):
        return np.ones(N, bool)
    return (np.arange(N) % G.n[0]) < G.n[0] - 1


def params(theta: float, dt: float, c: float = 1.0) -> Params:
    p = Params()
    p.theta, p.c, p.dt = theta, c, dt
    return p


def nnodes(G: Grid) -> int:
    return int(np.prod([G.n[d] for d in range(G.dim)]))


def cellvol(G: Grid) -> float:
    return float(np.prod([G.dx[d] for d in range(G.dim)]))


# ---------------------------------------------------------------- primitives
def limiter(num: float, den: float, beta: float) -> float:
    """Generalised MC limiter (Sec. 2.2)."""
    return lib().or_limiter(num, den, beta)


def alpha(beta: float, B) -> np.ndarray:
    """Rotation matrix alpha (Sec. 3.1), 3x3."""
    B = _f64(B)
    out = np.empty(9)
    lib().or_alpha(beta, _ptr(B), _ptr(out))
    return out.reshape(3, 3)


def shape(G: Grid, x):
    """Linear-shape nodes and weights of one particle."""
    x = _f64(x)
    nodes = np.empty(8, np.int64)
    W = np.empty(8)
    k = lib().or_shape(ctypes.byref(G), _ptr(x), nodes.ctypes.data, _ptr(W))
    return nodes[:k], W[:k]


def node_avg(G: Grid, Bc) -> np.ndarray:
    Bc = _f64(Bc)
    out = np.empty_like(Bc)
    lib().or_node_avg(ctypes.byref(G), _ptr(Bc), _ptr(out))
    return out


def global_positions(G: Grid, cell, off) -> np.ndarray:
    """x[p, d] = (i_d + f_d) dx_d from (linear cell, offset) pairs (FP64)."""
    cell = np.asarray(cell, np.int64)
    off = np.asarray(off, np.float64)
    x = np.zeros((cell.size, 3))
    rem = cell.copy()
    for d in range(G.dim):
        i = rem % G.n[d]
        rem //= G.n[d]
        x[:, d] = (i + off[d]) * G.dx[d]
    return x


def deposit_species(G: Grid, q: float, m: float, beta: float, x, v, w, Bn, u_node=None,
                    acc: Optional[Dict[str, np.ndarray]] = None) -> Dict[str, np.ndarray]:
    """Current, mass matrix and moments of one species (Sec. 3.1).

    x, v: [np, 3]; w: [np]; Bn: [3, N] node-averaged B.  Returns (or
    accumulates into acc) J [3,N], M [27,9,N], rho [N], mm [3,N], mass [N]."""
    N = nnodes(G)
    if acc is None:
        acc = {"J": np.zeros((3, N)), "M": np.zeros((27, 9, N)), "rho": np.zeros(N),
               "mm": np.zeros((3, N)), "mass": np.zeros(N)}
    x, v, w, Bn = _f64(x), _f64(v), _f64(w), _f64(Bn)
    un = None if u_node is None else _f64(u_node)
    lib().or_deposit_species(ctypes.byref(G), q, m, beta, int(w.size), _ptr(x), _ptr(v), _ptr(w), _ptr(Bn),
                             _ptr(un), _ptr(acc["J"]), _ptr(acc["M"]), _ptr(acc["rho"]), _ptr(acc["mm"]),
                             _ptr(acc["mass"]))
    return acc


def bulk_velocity(G: Grid, mm, mass) -> np.ndarray:
    mm, mass = _f64(mm), _f64(mass)
    u = np.empty_like(mm)
    lib().or_bulk_velocity(ctypes.byref(G), _ptr(mm), _ptr(mass), _ptr(u))
    return u


def filter_axis(G: Grid, f, phi: float, stride: int, axis: int) -> np.ndarray:
    f = _f64(f).copy()
    lib().or_filter_axis(ctypes.byref(G), _ptr(f), f.shape[0], phi, stride, axis)
    return f


def smooth(G: Grid, f, npass: int, phi: float = 0.5) -> np.ndarray:
    """npass digital-filter passes (Sec. 2.4 / Sec. 3.1), strides 1,2,1,2,..."""
    f = _f64(f).copy()
    lib().or_smooth(ctypes.byref(G), _ptr(f), f.shape[0], npass, phi)
    return f


def smooth_current(G: Grid, J, npass: int, phi: float = 0.5) -> np.ndarray:
    """Current smoothing (Sec. 3.2): npass passes of the digital filter of
    Sec. 2.4 at its default stride d = 1, each pass sweeping x, then y, then z
    (the sweep order is the reading used for the u smoothing as well)."""
    J = _f64(J).copy()
    for _ in range(npass):
        for axis in range(G.dim):
            J = filter_axis(G, J, phi, 1, axis)
    return J


def _cell_view(G: Grid, f):
    """[ncomp][N] (x fastest) -> [ncomp, nz, ny, nx] view."""
    f = np.asarray(f, dtype=np.float64)
    return f.reshape(f.shape[0], G.n[2], G.n[1], G.n[0])


def div_cc(G: Grid, Bc) -> np.ndarray:
    """Divergence of a cell-centred vector at the cell centres, central
    differences on the periodic mesh (READING for the divergence cleaning of
    Sec. 2.3, whose discretisation the paper takes from a reference that is
    not available): sum_d (B_d(c + e_d) - B_d(c - e_d)) / (2 dx_d)."""
    B = _cell_view(G, Bc)
    out = np.zeros(B.shape[1:])
    for d in range(G.dim):
        ax = 2 - d  # array axis of mesh axis d in [z, y, x]
        out += (np.roll(B[d], -1, axis=ax) - np.roll(B[d], 1, axis=ax)) / (2.0 * G.dx[d])
    return out.reshape(-1)


def grad_cc(G: Grid, psi) -> np.ndarray:
    """Gradient of a cell-centred scalar at the cell centres, central
    differences: the negative adjoint of div_cc on the periodic mesh."""
    f = np.asarray(psi, dtype=np.float64).reshape(G.n[2], G.n[1], G.n[0])
    out = np.zeros((3,) + f.shape)
    for d in range(G.dim):
        ax = 2 - d
        out[d] = (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) / (2.0 * G.dx[d])
    return out.reshape(3, -1)


def cleaning_speed(G: Grid, dt: float, ch_frac: float = 0.8) -> float:
    """c_h = ch_frac * dx / dt (Sec. 2.3 uses 0.8), dx the smallest active spacing."""
    return ch_frac * min(G.dx[d] for d in range(G.dim)) / dt


def dedner_psi(G: Grid, dt: float, psi, Bc, ch: float, damp: float = 0.1) -> np.ndarray:
    """One step of the cleaning scalar (Sec. 2.3): d psi/dt + c_h^2 div B =
    -(c_h^2/c_p^2) psi, READING: explicit in div B^n, then the damping term
    integrated exactly over the step, psi^{n+1} = (psi^n - dt c_h^2 div B^n)
    exp(-damp) with damp = dt c_h^2 / c_p^2 (0.1 in Sec. 2.3)."""
    psi = np.asarray(psi, dtype=np.float64).reshape(-1)
    return (psi - dt * ch * ch * div_cc(G, Bc)) * math.exp(-damp)


def motional(G: Grid, u, Bn) -> np.ndarray:
    u, Bn = _f64(u), _f64(Bn)
    out = np.empty_like(u)
    lib().or_motional(ctypes.byref(G), _ptr(u), _ptr(Bn), _ptr(out))
    return out


def mass_apply(G: Grid, M, x) -> np.ndarray:
    M, x = _f64(M), _f64(x)
    y = np.empty_like(x)
    lib().or_mass_apply(ctypes.byref(G), _ptr(M), _ptr(x), _ptr(y))
    return y


def current_eff(G: Grid, JC, Mt, EM) -> np.ndarray:
    JC, Mt, EM = _f64(JC), _f64(Mt), _f64(EM)
    out = np.empty_like(JC)
    lib().or_current_eff(ctypes.byref(G), _ptr(JC), _ptr(Mt), _ptr(EM), _ptr(out))
    return out


def kappa_E(G: Grid, E, a_node, beta: float) -> np.ndarray:
    E, a = _f64(E), _f64(a_node)
    out = np.empty((3, 3, nnodes(G)))
    lib().or_kappa_E(ctypes.byref(G), _ptr(E), _ptr(a), beta, _ptr(out))
    return out


def kappa_B(G: Grid, B, a_node, beta: float) -> np.ndarray:
    B, a = _f64(B), _f64(a_node)
    out = np.empty((3, 3, nnodes(G)))
    lib().or_kappa_B(ctypes.byref(G), _ptr(B), _ptr(a), beta, _ptr(out))
    return out


def _unary(fn, G, a, shape=None):
    a = _f64(a)
    out = np.empty(shape if shape is not None else a.shape)
    fn(ctypes.byref(G), _ptr(a), _ptr(out))
    return out


def curl_nc(G: Grid, E) -> np.ndarray:
    return _unary(lib().or_curl_nc, G, E)


def curl_cn(G: Grid, B) -> np.ndarray:
    return _unary(lib().or_curl_cn, G, B)


def div_nc(G: Grid, E) -> np.ndarray:
    return _unary(lib().or_div_nc, G, E, (nnodes(G),))


def gauss_residual(G: Grid, E, rho_s) -> float:
    """||div_NC E - 4 pi rho_c|| / ||4 pi rho_c|| with rho_c the cell mean of
    the node charge density summed over species (the absolute norm if there is
    no charge); see or_gauss_sums."""
    rho = _f64(np.sum(np.asarray(rho_s, np.float64).reshape(-1, nnodes(G)), axis=0))
    E = _f64(E)
    out = np.zeros(2)
    lib().or_gauss_sums(ctypes.byref(G), _ptr(E), _ptr(rho), _ptr(out))
    return float(math.sqrt(out[0] / out[1])) if out[1] > 0 else float(math.sqrt(out[0]))


def diffusion(G: Grid, kappa, F) -> np.ndarray:
    kappa, F = _f64(kappa), _f64(F)
    out = np.empty_like(F)
    lib().or_diffusion(ctypes.byref(G), _ptr(kappa), _ptr(F), _ptr(out))
    return out


def apply_A(G: Grid, P: Params, Mt, kE, x) -> np.ndarray:
    x = _f64(x)
    Mt = None if Mt is None else _f64(Mt)
    kE = None if kE is None else _f64(kE)
    y = np.empty_like(x)
    lib().or_apply_A(ctypes.byref(G), ctypes.byref(P), _ptr(Mt), _ptr(kE), _ptr(x), _ptr(y))
    return y


def rhs(G: Grid, P: Params, En, Bc, Jeff) -> np.ndarray:
    En, Bc, Jeff = _f64(En), _f64(Bc), _f64(Jeff)
    b = np.empty_like(En)
    lib().or_rhs(ctypes.byref(G), ctypes.byref(P), _ptr(En), _ptr(Bc), _ptr(Jeff), _ptr(b))
    return b


def update_B(G: Grid, P: Params, Bc, Eth, kB=None) -> np.ndarray:
    Bc, Eth = _f64(Bc), _f64(Eth)
    kB = None if kB is None else _f64(kB)
    out = np.empty_like(Bc)
    lib().or_update_B(ctypes.byref(G), ctypes.byref(P), _ptr(Bc), _ptr(Eth), _ptr(kB), _ptr(out))
    return out


def update_E(theta: float, En, Eth) -> np.ndarray:
    En, Eth = _f64(En), _f64(Eth)
    out = np.empty_like(En)
    lib().or_update_E(En.size, theta, _ptr(En), _ptr(Eth), _ptr(out))
    return out


def push_species(G: Grid, beta: float, dt: float, x, v, Eth, Bn, with_keep: bool = False):
    """Implicit mover (Sec. 3.1).  Returns (x_new, v_new), and with
    with_keep the mask of particles that stay in the domain (a walled grid
    with an inflow plane loses the particles that cross it)."""
    x, v = _f64(x), _f64(v)
    n = x.shape[0]
    xn = np.empty_like(x)
    vn = np.empty_like(v)
    keep = np.ones(n, np.int32)
    lib().or_push_species(ctypes.byref(G), beta, dt, n, _ptr(x), _ptr(v), _ptr(_f64(Eth)), _ptr(_f64(Bn)),
                          _ptr(xn), _ptr(vn), keep.ctypes.data)
    if with_keep:
        return xn, vn, keep.astype(bool)
    return xn, vn


def gmres(G: Grid, P: Params, Mt, kE, b, x0, tol: float = 1e-8, maxit: int = 1000, restart: int = 30):
    """Restarted GMRES (FP64, MGS).  Returns (x, iterations, relres)."""
    b = _f64(b)
    x = _f64(x0).copy()
    Mt = None if Mt is None else _f64(Mt)
    kE = None if kE is None else _f64(kE)
    rel = ctypes.c_double()
    it = lib().or_gmres(ctypes.byref(G), ctypes.byref(P), _ptr(Mt), _ptr(kE), _ptr(b), _ptr(x), tol, maxit,
                        restart, ctypes.addressof(rel))
    return x, it, rel.value


def dense_A(G: Grid, P: Params, Mt, kE) -> np.ndarray:
    n = 3 * nnodes(G)
    A = np.empty((n, n))
    Mt = None if Mt is None else _f64(Mt)
    kE = None if kE is None else _f64(kE)
    lib().or_dense_A(ctypes.byref(G), ctypes.byref(P), _ptr(Mt), _ptr(kE), _ptr(A))
    return A


def dense_solve(A, b) -> np.ndarray:
    A, b = _f64(A), _f64(b)
    x = np.empty_like(b)
    rc = lib().or_dense_solve(b.size, _ptr(A), _ptr(b), _ptr(x))
    assert rc == 0, "singular matrix"
    return x


def advect(u, nu: float, beta: float, nsteps: int, phi_override: float = -1.0) -> np.ndarray:
    """Scalar advection with the limited LF flux of Sec. 2.2 (c = a > 0)."""
    u = _f64(u).copy()
    lib().or_advect(u.size, _ptr(u), nu, beta, nsteps, phi_override)
    return u


def stable_cell_order(keys) -> np.ndarray:
    """Permutation that stable-sorts particles by cell (a library sort)."""
    return np.argsort(np.asarray(keys), kind="stable")


# ---------------------------------------------------------------- the step
# Offsets of the half stencil, in the order the GPU library stores them:
# offset 0 first, then every o != 0 whose last nonzero component (z, then y,
# then x) is +1, enumerated z-major.  Used only to compare layouts.
def half_offsets(dim: int) -> List[tuple]:
    out = [(0, 0, 0)]
    rng = [(-1, 0, 1) if d < dim else (0,) for d in range(3)]
    for oz in rng[2]:
        for oy in rng[1]:
            for ox in rng[0]:
                o = (ox, oy, oz)
                if o == (0, 0, 0):
                    continue
                last = oz if oz != 0 else (oy if oy != 0 else ox)
                if last > 0:
                    out.append(o)
    return out


def off27(o) -> int:
    return (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)


class Species:
    def __init__(self, q: float, m: float, x, v, w):
        self.q, self.m = float(q), float(m)
        self.x = _f64(x)
        self.v = _f64(v)
        self.w = _f64(w)


def beta_s(q: float, m: float, dt: float) -> float:
    """beta_s = (q_s/m_s)(dt/2) (Sec. 3.1)."""
    return q / m * dt / 2.0


def deposit(G: Grid, species: List[Species], dt: float, Bc, comoving: bool, n_smooth_u: int = 5,
            phi_u: float = 0.5, n_smooth_j: int = 0) -> Dict[str, np.ndarray]:
    """Particle-to-grid quantities of one step (Sec. 3.1).

    Returns J_lab, M_s (per species, 27-offset), Mt = sum beta_s M_s,
    M0 = sum M_s, rho_s, mm, mass, u (smoothed), EM, J_C and J_eff.
    n_smooth_j > 0 smooths the comoving-frame current J_C (the lab current when
    the comoving frame is off) before the E_M term is added (Sec. 3.2)."""
    N = nnodes(G)
    dV = cellvol(G)
    Bn = node_avg(G, Bc)
    out: Dict[str, np.ndarray] = {"Bn": Bn}
    tot = {"J": np.zeros((3, N)), "mm": np.zeros((3, N)), "mass": np.zeros(N)}
    Ms, rhos = [], []
    for sp in species:
        b = beta_s(sp.q, sp.m, dt)
        a = deposit_species(G, sp.q, sp.m, b, sp.x, sp.v, sp.w, Bn)
        tot["J"] += a["J"]
        tot["mm"] += a["mm"]
        tot["mass"] += a["mass"]
        Ms.append(a["M"])
        rhos.append(a["rho"])
    out["J_lab"] = tot["J"]
    out["mm"], out["mass"] = tot["mm"], tot["mass"]
    out["M_s"] = Ms
    out["rho_s"] = rhos
    out["Mt"] = sum(beta_s(sp.q, sp.m, dt) * M for sp, M in zip(species, Ms))
    out["M0"] = sum(Ms)
    u = bulk_velocity(G, tot["mm"], tot["mass"])
    u = smooth(G, u, n_smooth_u, phi_u)
    out["u"] = u
    out["EM"] = motional(G, u, Bn)
    if comoving:
        JC = np.zeros((3, N))
        for sp in species:
            b = beta_s(sp.q, sp.m, dt)
            a = deposit_species(G, sp.q, sp.m, b, sp.x, sp.v, sp.w, Bn, u_node=u)
            JC += a["J"]
        if n_smooth_j > 0:
            JC = smooth_current(G, JC, n_smooth_j, phi_u)
        out["J_C"] = JC
        out["J_eff"] = current_eff(G, JC, out["Mt"], out["EM"])
    else:
        JC = smooth_current(G, out["J_lab"], n_smooth_j, phi_u) if n_smooth_j > 0 else out["J_lab"]
        out["J_C"] = JC
        out["J_eff"] = JC
    return out


def explicit_current(G: Grid, species: List[Species], comoving: bool, n_smooth_u: int = 5, phi_u: float = 0.5,
                     n_smooth_j: int = 0) -> np.ndarray:
    """Current of an explicit PIC step (Sec. 3.1, explicit form): with the
    comoving frame, (1/dV) sum_{s,p} q w (v - u(x_p)) W(x_p - x_g), u the
    mass-weighted bulk velocity after n_smooth_u filter passes (strides 1, 2,
    ...) interpolated to x_p with the weights W; else the lab current
    (1/dV) sum q w v W.  Then n_smooth_j passes (Sec. 3.2).  The particle
    velocity enters unrotated, i.e. the deposit of this module with beta = 0,
    whose comoving branch deposits v - u(x_p) particle by particle."""
    N = nnodes(G)
    Bn = np.zeros((3, N))
    tot = {"J": np.zeros((3, N)), "M": np.zeros((27, 9, N)), "rho": np.zeros(N),
           "mm": np.zeros((3, N)), "mass": np.zeros(N)}
    for sp in species:
        deposit_species(G, sp.q, sp.m, 0.0, sp.x, sp.v, sp.w, Bn, acc=tot)
    J = tot["J"]
    if comoving:
        u = smooth(G, bulk_velocity(G, tot["mm"], tot["mass"]), n_smooth_u, phi_u)
        J = np.zeros((3, N))
        for sp in species:
            J += deposit_species(G, sp.q, sp.m, 0.0, sp.x, sp.v, sp.w, Bn, u_node=u)["J"]
    return smooth_current(G, J, n_smooth_j, phi_u) if n_smooth_j > 0 else J


def explicit_step(G: Grid, species: List[Species], E, Bc, *, dt: float, c: float = 1.0, comoving: bool = True,
                  n_smooth_u: int = 5, phi_u: float = 0.5, n_smooth_j: int = 0) -> Dict[str, object]:
    """One explicit PIC step with the current of Sec. 3.1's explicit form (the
    paper gives no explicit integrator; this is the leapfrog it writes for the
    1D Yee scheme in Sec. 2.1, on the node/cell mesh with the multi-D curls of
    the implicit path).  State: x^n, v^{n-1/2}, E^n at nodes, B^n at cells.
      1. v^{n+1/2} from v^{n-1/2} with E^n and the node-averaged B^n at x^n
         (push_species: its implicit-midpoint rotation is the Boris push),
         x^{n+1} = x^n + dt v^{n+1/2};
      2. J = explicit_current at (x^{n+1}, v^{n+1/2});
      3. B^{n+1/2} = B^n - (c dt/2) curl_NC E^n,
         E^{n+1} = E^n + c dt curl_CN B^{n+1/2} - 4 pi dt J,
         B^{n+1} = B^{n+1/2} - (c dt/2) curl_NC E^{n+1}."""
    Bn = node_avg(G, Bc)
    moved = []
    for sp in species:
        xn, vn = push_species(G, beta_s(sp.q, sp.m, dt), dt, sp.x, sp.v, E, Bn)
        moved.append(Species(sp.q, sp.m, xn, vn, sp.w))
    J = explicit_current(G, moved, comoving, n_smooth_u, phi_u, n_smooth_j)
    half = params(1.0, 0.5 * dt, c)
    Bh = update_B(G, half, Bc, E)
    En = rhs(G, params(1.0, dt, c), E, Bh, J)
    Bnew = update_B(G, half, Bh, En)
    return {"species": moved, "E": En, "B": Bnew, "J": J}


def diffusion_speed(G: Grid, u, a_mode: int, c: float = 1.0) -> np.ndarray:
    """a at nodes (Sec. 2.2): c (a_mode 0) or the bulk speed |u| (a_mode 1)."""
    N = nnodes(G)
    if a_mode == 0:
        return np.full(N, c)
    return np.sqrt((np.asarray(u) ** 2).sum(axis=0))


def node_weights(G: Grid) -> np.ndarray:
    """Control-volume weights of the nodes: 1, and 1/2 on the boundary node
    planes of a walled grid (the trapezoid rule of the mirror-doubled domain)."""
    N = nnodes(G)
    w = np.ones(N)
    if walled(G):
        i = np.arange(N) % G.n[0]
        w[(i == 0) | (i == G.n[0] - 1)] = 0.5
    return w


def diagnostics(G: Grid, species: List[Species], E, Bc, rho_s=None) -> Dict[str, object]:
    """Energies and momenta in FP64: W_E = sum |E|^2 dV / 8pi over nodes
    (half weight on the boundary planes of a walled grid), W_B over the
    physical cells, K_s = sum 1/2 m_s w |v|^2, P_s = sum m_s w v; with the
    node charge densities rho_s (per species) also the Gauss residual."""
    dV = cellvol(G)
    WE = float((node_weights(G) * (np.asarray(E) ** 2).sum(axis=0)).sum() * dV / (8 * math.pi))
    WB = float((np.asarray(Bc)[:, physical_cells(G)] ** 2).sum() * dV / (8 * math.pi))
    K = [float(0.5 * sp.m * (sp.w[:, None] * sp.v ** 2).sum()) for sp in species]
    P = [(sp.m * (sp.w[:, None] * sp.v).sum(axis=0)) for sp in species]
    out = {"W_E": WE, "W_B": WB, "K": K, "P": P}
    if rho_s is not None:
        out["gauss"] = gauss_residual(G, E, rho_s)
    return out


def step(G: Grid, species: List[Species], E, Bc, *, dt: float, theta: float, c: float = 1.0,
         comoving: bool = False, lf_E: bool = False, lf_B: bool = False, beta_lim: float = 1.0,
         a_mode: int = 1, n_smooth_u: int = 5, tol: float = 1e-12, restart: int = 30,
         solve: str = "gmres", n_smooth_j: int = 0, dedner: bool = False, ch_frac: float = 0.8,
         dedner_damp: float = 0.1, psi=None, n_smooth_e: int = 0, limiter_lag: str = "en",
         inject=None) -> Dict[str, object]:
    """One full GL-ECSIM step without the Gauss's-law correction:
    deposit -> implicit E solve -> B and E update -> particle push.
    With dedner, the cleaning scalar psi (cells, zero if None) is advanced
    from B^n first and B^{n+1} gets -dt grad psi^{n+1} (Sec. 2.3).
    n_smooth_e > 0 smooths E^{n+1} with that many filter passes (Sec. 2.4,
    strides 1, 2, 1, ...), the alternative to the LF diffusion of Sec. 4.1.
    The E limiter's smoothness ratio is taken from the unknown E^{n+theta} in
    Sec. 2.2, which makes the system nonlinear.  limiter_lag "en" takes it
    from E^n (one linear solve); "picard1" then takes one Picard step: the
    limiter from that first E^{n+theta}, and the system solved again from it.
    On a walled grid particles reflect on walls and leave through an inflow
    plane; inject (one (x, v, w) triple or None per species) appends
    particles after the push."""
    P = params(theta, dt, c)
    dep = deposit(G, species, dt, Bc, comoving, n_smooth_u, n_smooth_j=n_smooth_j)
    a_node = diffusion_speed(G, dep["u"], a_mode, c)
    kE = kappa_E(G, E, a_node, beta_lim) if lf_E else None
    kB = kappa_B(G, Bc, a_node, beta_lim) if lf_B else None
    b = rhs(G, P, E, Bc, dep["J_eff"])
    if limiter_lag not in ("en", "picard1"):
        raise ValueError(f"limiter_lag {limiter_lag!r}")

    def _solve(kE_, x0):
        if solve == "dense":
            return dense_solve(dense_A(G, P, dep["Mt"], kE_), b.ravel()).reshape(E.shape), 0, 0.0
        return gmres(G, P, dep["Mt"], kE_, b, x0, tol=tol, maxit=5000, restart=restart)

    Eth, its, rel = _solve(kE, E)
    if limiter_lag == "picard1" and lf_E:
        kE = kappa_E(G, Eth, a_node, beta_lim)
        Eth, its2, rel = _solve(kE, Eth)
        its += its2
    Bnew = update_B(G, P, Bc, Eth, kB)
    psi_new = None
    if dedner:
        psi0 = np.zeros(nnodes(G)) if psi is None else psi
        psi_new = dedner_psi(G, dt, psi0, Bc, cleaning_speed(G, dt, ch_frac), dedner_damp)
        Bnew = Bnew - dt * grad_cc(G, psi_new)
    Enew = update_E(theta, E, Eth)
    if n_smooth_e:
        Enew = smooth(G, Enew, n_smooth_e)
    new_species, kept = [], []
    for k, sp in enumerate(species):
        xn, vn, keep = push_species(G, beta_s(sp.q, sp.m, dt), dt, sp.x, sp.v, Eth, dep["Bn"], with_keep=True)
        x2, v2, w2 = xn[keep], vn[keep], sp.w[keep]
        if inject is not None and inject[k] is not None:
            xi, vi, wi = inject[k]
            x2 = np.concatenate([x2, _f64(xi).reshape(-1, 3)])
            v2 = np.concatenate([v2, _f64(vi).reshape(-1, 3)])
            w2 = np.concatenate([w2, _f64(wi).reshape(-1)])
        new_species.append(Species(sp.q, sp.m, x2, v2, w2))
        kept.append(keep)
    return {"dep": dep, "kE": kE, "kB": kB, "b": b, "Eth": Eth, "E": Enew, "B": Bnew,
            "species": new_species, "kept": kept, "iters": its, "relres": rel, "a_node": a_node, "psi": psi_new}
