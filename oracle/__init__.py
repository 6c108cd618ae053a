"""Python access to the FP64 CPU oracle (oracle/gks_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and
by the cpu_baseline leg of bench.py.  Nothing on the product path may import
this package.  The oracle is a literal, slow transcription of Pan & Xu,
arXiv:1412.4489 (see the header of gks_oracle.c); it shares no code with the
HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_CODES = {"periodic": 0, "outflow": 1, "reflect": 2, "noslip_iso": 3, "noslip_adia": 4,
            "inflow": 5, "dmr_bottom": 6, "dmr_top": 7}


def build(verbose=False):
    """Compile the oracle (gcc, FP64, no FMA contraction, OpenMP over rows)."""
    cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


class orc_problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("gamma", C.c_double), ("viscous", C.c_int), ("mu", C.c_double), ("prandtl", C.c_double),
        ("tau_eps", C.c_double), ("tau_c", C.c_double), ("cfl", C.c_double),
        ("weno_eps", C.c_double), ("weno_c", C.c_double), ("recon_vars", C.c_int),
        ("exact_c", C.c_int), ("bc_kind", C.c_int * 4), ("bc_state", (C.c_double * 4) * 4),
        ("bc_alt", (C.c_double * 4) * 4), ("bc_wall", (C.c_double * 3) * 4),
        ("obst_i0", C.c_int), ("obst_nj", C.c_int), ("admissibility", C.c_int),
        ("mesh", C.POINTER(C.c_double)), ("bc_omega", C.c_double * 4),
    ]


class orc_face_input(C.Structure):
    _fields_ = [(n, (C.c_double * 4) * 2) for n in ("W", "Wn", "Ws", "Wnn", "Wns", "Wss")] + [
        ("Ueq", ((C.c_double * 4) * 3) * 2), ("dn", C.c_double), ("ds", C.c_double),
        ("curv", C.c_int), ("G", C.c_double * 3)]


class orc_face_output(C.Structure):
    _fields_ = [("flux", C.c_double * 4), ("pv", (C.c_double * 4) * 2), ("W0", C.c_double * 4),
                ("q", (C.c_double * 4) * 5), ("tau", C.c_double), ("heat", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.orc_moment_tables.argtypes = [C.c_int, C.c_double, _D, C.c_int, _D, _D, _D, _D]
        L.orc_solve.argtypes = [C.c_int, C.c_double, _D, _D, _D]
        L.orc_coefficients.argtypes = [C.c_int, C.c_double, _D, _D, _D, _D, _D, _D, C.c_int, _D]
        L.orc_time_coefficients.argtypes = [C.c_double, C.c_double, C.c_int, _D]
        L.orc_time_integrals.argtypes = [C.c_double, C.c_double, C.c_int, _D]
        L.orc_face.argtypes = [C.POINTER(orc_problem), C.POINTER(orc_face_input), C.c_double,
                               C.POINTER(orc_face_output)]
        L.orc_f_assembled.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, C.c_double, _D, _D,
                                      C.c_double, C.c_double, C.c_int, _D, _D, _D, _D]
        L.orc_recon2d_scalar.argtypes = [C.c_double] * 17 + [_D]
        L.orc_euler_eigvec_2d.argtypes = [C.c_double, _D, C.c_int, _D]
        L.orc_recon2d_cell.argtypes = [C.c_int, C.c_double, _D, C.c_double, C.c_double, C.c_double,
                                       C.c_double, _D]
        L.orc_recon1d_scalar.argtypes = [C.c_double] * 8 + [_D]
        L.orc_equilibrium_poly.argtypes = [C.c_int, _D, _D, C.c_double, C.c_double, _D]
        L.orc_dt.argtypes = [C.POINTER(orc_problem), _D]
        L.orc_dt.restype = C.c_double
        L.orc_step.argtypes = [C.POINTER(orc_problem), _D, _D, _D, C.c_double, C.c_double]
        L.orc_run.argtypes = [C.POINTER(orc_problem), _D, _D, _D, C.c_int, C.c_double, C.c_double, _D]
        L.orc_last_fluxes.argtypes = [C.POINTER(orc_problem), _D, _D]
        L.orc_last_fallbacks.argtypes = []
        L.orc_last_fallbacks.restype = C.c_long
        L.orc_take_capped.argtypes = []
        L.orc_take_capped.restype = C.c_long
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None and a.size < n:
        a = np.concatenate([a.ravel(), np.zeros(n - a.size)])
    return a


def make_problem(prob, exact_c=False) -> orc_problem:
    P = orc_problem()
    P.dim, P.nx, P.ny = prob.dim, prob.nx, prob.ny
    P.x0, P.x1, P.y0, P.y1 = prob.x0, prob.x1, prob.y0, prob.y1
    P.gamma, P.viscous, P.mu, P.prandtl = prob.gamma, int(prob.viscous), prob.mu, prob.prandtl
    P.tau_eps, P.tau_c, P.cfl = prob.tau_eps, prob.tau_c, prob.cfl
    P.weno_eps, P.weno_c, P.recon_vars = prob.weno_eps, prob.weno_c, prob.recon_vars
    P.exact_c = int(exact_c)
    for s, bc in enumerate(prob.bc):
        P.bc_kind[s] = BC_CODES[bc.kind]
        for i in range(4):
            P.bc_state[s][i] = bc.state[i]
            P.bc_alt[s][i] = bc.alt[i]
        for i in range(3):
            P.bc_wall[s][i] = bc.wall[i]
        P.bc_omega[s] = getattr(bc, "omega", 0.0)
    P.obst_i0, P.obst_nj = prob.obstacle
    P.admissibility = prob.admissibility
    mesh = getattr(prob, "mesh", None)
    if mesh is not None:
        m = np.ascontiguousarray(mesh, dtype=np.float64)
        assert m.shape == (prob.ny + 1, prob.nx + 1, 2), m.shape
        P._mesh_keep = m  # the C side reads it during the call
        P.mesh = _p(m)
    return P


# --- building blocks ------------------------------------------------------

def moment_tables(dim, gamma, W, half=0):
    Mu, Mv, Mx, prim = np.zeros(16), np.zeros(16), np.zeros(8), np.zeros(4)
    W = _arr(W, 4)
    if lib().orc_moment_tables(dim, gamma, _p(W), half, _p(Mu), _p(Mv), _p(Mx), _p(prim)):
        raise ValueError("nonphysical state")
    return Mu, Mv, Mx, prim


def solve(dim, gamma, W, b):
    a = np.zeros(4)
    W, b = _arr(W, 4), _arr(b, 4)
    if lib().orc_solve(dim, gamma, _p(W), _p(b), _p(a)):
        raise ValueError("nonphysical state")
    return a[:dim + 2]


def coefficients(dim, gamma, W, Wx, Wy, Wxx, Wxy, Wyy, which=0):
    out = np.zeros((9, 4))
    args = [_arr(x, 4) for x in (W, Wx, Wy, Wxx, Wxy, Wyy)]
    if lib().orc_coefficients(dim, gamma, *[_p(a) for a in args], which, _p(out)):
        raise ValueError("nonphysical state")
    return out


def time_coefficients(tau, t, exact_c=False):
    out = np.zeros(10)
    lib().orc_time_coefficients(tau, t, int(exact_c), _p(out))
    return out


def time_integrals(tau, dt, exact_c=False):
    out = np.zeros(10)
    lib().orc_time_integrals(tau, dt, int(exact_c), _p(out))
    return out


def face(prob, inputs: dict, dt, exact_c=False):
    """inputs: W, Wn, Ws, Wnn, Wns, Wss -> arrays [2][nvar]; Ueq [2][3][nvar]; dn, ds."""
    fi = orc_face_input()
    for name in ("W", "Wn", "Ws", "Wnn", "Wns", "Wss"):
        a = np.zeros((2, 4))
        if name in inputs:
            v = np.asarray(inputs[name], dtype=np.float64)
            a[:, :v.shape[1]] = v
        getattr(fi, name)[0][:] = list(a[0])
        getattr(fi, name)[1][:] = list(a[1])
    U = np.zeros((2, 3, 4))
    v = np.asarray(inputs["Ueq"], dtype=np.float64)
    U[:, :, :v.shape[2]] = v
    for m in range(2):
        for n in range(3):
            fi.Ueq[m][n][:] = list(U[m, n])
    fi.dn, fi.ds = inputs["dn"], inputs.get("ds", 1.0)
    if "G" in inputs:  # an interface of a curvilinear grid: metric (G_nn, G_ns, G_ss)
        fi.curv = 1
        fi.G[:] = list(inputs["G"])
    fo = orc_face_output()
    P = make_problem(prob, exact_c)
    rc = lib().orc_face(C.byref(P), C.byref(fi), dt, C.byref(fo))
    if rc:
        raise ValueError(f"orc_face failed ({rc})")
    nv = prob.dim + 2
    return {"flux": np.array(fo.flux[:nv]), "pv": np.array([fo.pv[0][:nv], fo.pv[1][:nv]]),
            "W0": np.array(fo.W0[:nv]), "q": np.array([list(r)[:nv] for r in fo.q]),
            "tau": fo.tau, "heat": fo.heat}


def f_assembled(dim, gamma, viscous, exact_c, tau, prim, coef, y, t, u, v, xi2):
    """f at the interface for arrays of particle velocities (u, v, xi^2)."""
    prim = _arr(prim).reshape(3, 4)
    coef = _arr(coef).reshape(3, 9, 4)
    u, v, xi2 = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (u, v, xi2)))
    shape = u.shape
    u, v, xi2 = (np.ascontiguousarray(a.ravel()) for a in (u, v, xi2))
    out = np.zeros(u.size)
    lib().orc_f_assembled(dim, gamma, int(viscous), int(exact_c), tau, _p(prim), _p(coef), y, t,
                          u.size, _p(u), _p(v), _p(xi2), _p(out))
    return out.reshape(shape)


def recon2d_scalar(Uc, Ue, Uw, Un, Us, Ep, Em, Wp, Wm, Np, Nm, Sp, Sm, h, k, eps=1e-6, Cw=1.0):
    p = np.zeros(5)
    lib().orc_recon2d_scalar(Uc, Ue, Uw, Un, Us, Ep, Em, Wp, Wm, Np, Nm, Sp, Sm, h, k, eps, Cw, _p(p))
    return p


def euler_eigvec_2d(gamma, W, ax):
    """Right eigenvectors (columns) of the 2D Euler flux Jacobian along axis
    ax (0: x, 1: y) at the conservative state W."""
    R = np.zeros((4, 4))
    if lib().orc_euler_eigvec_2d(gamma, _p(_arr(W, 4)), ax, _p(R)):
        raise ValueError("nonphysical state")
    return R


def recon2d_cell(S, h, k, gamma=1.4, vars=0, eps=1e-6, Cw=1.0):
    """p2..p6 of the four components of one 2D cell from the stencil values
    S[13][4] (Uc, Ue, Uw, Un, Us, E+, E-, W+, W-, N+, N-, S+, S-)."""
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(13, 4)
    pc = np.zeros((4, 5))
    rc = lib().orc_recon2d_cell(vars, gamma, _p(S), h, k, eps, Cw, _p(pc))
    return pc, rc


def recon1d_scalar(Uc, Ue, Uw, Fp, Fm, h, eps=1e-6, Cw=1.0):
    p = np.zeros(2)
    lib().orc_recon1d_scalar(Uc, Ue, Uw, Fp, Fm, h, eps, Cw, _p(p))
    return p


def equilibrium_poly(dim, Ueq, U0, dn, ds):
    U = np.zeros((2, 3, 4))
    v = np.asarray(Ueq, dtype=np.float64)
    U[:, :, :v.shape[2]] = v
    q = np.zeros((5, 4))
    lib().orc_equilibrium_poly(dim, _p(U), _p(_arr(U0, 4)), dn, ds, _p(q))
    return q[:, :dim + 2]


# --- whole scheme -----------------------------------------------------------

def dt(prob, state):
    P = make_problem(prob)
    cell = np.ascontiguousarray(state.cell, dtype=np.float64)
    return lib().orc_dt(C.byref(P), _p(cell))


def step(prob, state, dt_, t=0.0, exact_c=False):
    """One step in place on a workloads.State; returns the fluxes (x, y)."""
    P = make_problem(prob, exact_c)
    for a in (state.cell, state.fx, state.fy):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    if lib().orc_step(C.byref(P), _p(state.cell), _p(state.fx), _p(state.fy), dt_, t):
        raise FloatingPointError("oracle step failed (nonphysical state)")
    nv, nx, ny = prob.nvar, prob.nx, prob.ny
    fxf = np.zeros((nv, ny, nx + 1))
    fyf = np.zeros((nv, ny + 1, nx))
    lib().orc_last_fluxes(C.byref(P), _p(fxf), _p(fyf))
    return fxf, fyf


def run(prob, state, nsteps=0, dt_fixed=0.0, t_end=0.0, t=0.0, exact_c=False):
    """Advance in place; returns (steps taken, final time)."""
    P = make_problem(prob, exact_c)
    tt = C.c_double(t)
    n = lib().orc_run(C.byref(P), _p(state.cell), _p(state.fx), _p(state.fy), nsteps, dt_fixed,
                      t_end, C.byref(tt))
    if n < 0:
        raise FloatingPointError("oracle run failed (nonphysical state)")
    return n, tt.value


def last_fallbacks():
    """Interior (gas) cells whose reconstruction fell back to the constant
    average in the last step (the admissibility reading)."""
    return int(lib().orc_last_fallbacks())


def take_capped():
    """Interface sides whose Chapman-Enskog correction was capped at cell
    Knudsen number one (the Knudsen reading of eq. dis2) since the last
    call; resets the count."""
    return int(lib().orc_take_capped())


def num_threads():
    return lib().orc_num_threads()
