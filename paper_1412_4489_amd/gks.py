"""Thin ctypes binding of the C ABI in include/gks.h (libgks.so, gfx950).

The functions keep the C names (gks_init, gks_init_device, gks_state_extent,
gks_step, gks_fetch, gks_destroy, gks_last_error, gks_profile, gks_kernel_time,
gks_tune, gks_block_size, gks_set_launch, gks_launch_shape, gks_fallbacks,
gks_step_noalloc) and only marshal arguments;
every step of the scheme runs in the HIP kernels of the library.  `Solver`
wraps a handle for numpy arrays laid out as in paper_1412_4489_amd.workloads.

There is no CPU fallback: if the library is not built or no HIP device is
present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libgks.so")

GKS_OK, GKS_EINVAL, GKS_ENOMEM, GKS_EDEVICE, GKS_ENONPHYS, GKS_ESTATE = 0, -1, -2, -3, -4, -5
GKS_FP64, GKS_FP32_MIXED = 0, 1
BC_CODES = {"periodic": 0, "outflow": 1, "reflect": 2, "noslip_iso": 3, "noslip_adia": 4,
            "inflow": 5, "dmr_bottom": 6, "dmr_top": 7}
KERNELS = {"ghost": 0, "dt": 1, "recon": 2, "interface": 3, "update": 4}
STATUS = {0: "GKS_OK", -1: "GKS_EINVAL", -2: "GKS_ENOMEM", -3: "GKS_EDEVICE", -4: "GKS_ENONPHYS",
          -5: "GKS_ESTATE"}


_D = C.POINTER(C.c_double)


class gks_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("state", C.c_double * 4), ("alt", C.c_double * 4),
                ("wall_u", C.c_double), ("wall_v", C.c_double), ("wall_T", C.c_double),
                ("wall_omega", C.c_double)]


class gks_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("gamma", C.c_double), ("viscous", C.c_int32), ("mu", C.c_double),
                ("prandtl", C.c_double), ("tau_eps", C.c_double), ("tau_c", C.c_double),
                ("cfl", C.c_double), ("weno_eps", C.c_double), ("weno_c", C.c_double),
                ("recon_vars", C.c_int32), ("precision", C.c_int32), ("bc", gks_bc * 4),
                ("t0", C.c_double), ("obstacle_i0", C.c_int32), ("obstacle_nj", C.c_int32),
                ("admissibility", C.c_int32), ("mesh", _D)]


class gks_noalloc_status(C.Structure):
    _fields_ = [("t", C.c_double), ("steps", C.c_int64), ("error", C.c_uint64), ("fallbacks", C.c_int64)]


class GKSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = C.c_void_p


def lib():
    """Load libgks.so (built by paper_1412_4489_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_1412_4489_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.gks_init.argtypes = [C.POINTER(_P), C.c_int32, C.POINTER(gks_problem), C.POINTER(_D), C.POINTER(_D),
                               C.POINTER(_D), _P]
        L.gks_init_device.argtypes = [C.POINTER(_P), C.c_int32, C.POINTER(gks_problem), C.POINTER(_P),
                                      C.POINTER(_P), C.POINTER(_P), _P]
        _I64 = C.POINTER(C.c_int64)
        L.gks_state_extent.argtypes = [C.POINTER(gks_problem), _I64, _I64, _I64, C.POINTER(C.c_int32)]
        L.gks_step.argtypes = [_P, C.c_int32, _D, _D]
        L.gks_fetch.argtypes = [_P, C.c_int32, _D, _D, _D, _D, C.POINTER(C.c_int64)]
        L.gks_destroy.argtypes = [_P]
        L.gks_last_error.argtypes = [_P]
        L.gks_last_error.restype = C.c_char_p
        L.gks_profile.argtypes = [_P, C.c_int32]
        L.gks_kernel_time.argtypes = [_P, C.c_int32, _D, C.POINTER(C.c_int64)]
        L.gks_tune.argtypes = [_P, C.c_int32]
        L.gks_block_size.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32)]
        L.gks_set_launch.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32]
        L.gks_launch_shape.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.gks_fallbacks.argtypes = [_P, C.c_int32, C.POINTER(C.c_int64)]
        L.gks_step_noalloc.argtypes = [C.POINTER(gks_problem), _P, _P, _P, C.c_int32, C.c_double, C.c_double, _P,
                                       _P]
        _lib = L
    return _lib


EXPORTED = ("gks_init", "gks_init_device", "gks_state_extent", "gks_step", "gks_fetch", "gks_destroy", "gks_last_error",
            "gks_profile", "gks_kernel_time", "gks_tune", "gks_block_size", "gks_set_launch", "gks_launch_shape",
            "gks_fallbacks", "gks_step_noalloc")


def to_c_problem(prob, precision=GKS_FP64, t0=0.0) -> gks_problem:
    P = gks_problem()
    P.t0 = t0
    P.dim, P.nx, P.ny = prob.dim, prob.nx, prob.ny
    P.x0, P.x1, P.y0, P.y1 = prob.x0, prob.x1, prob.y0, prob.y1
    P.gamma, P.viscous, P.mu, P.prandtl = prob.gamma, int(prob.viscous), prob.mu, prob.prandtl
    P.tau_eps, P.tau_c, P.cfl = prob.tau_eps, prob.tau_c, prob.cfl
    P.weno_eps, P.weno_c, P.recon_vars = prob.weno_eps, prob.weno_c, prob.recon_vars
    P.precision = precision
    P.obstacle_i0, P.obstacle_nj = prob.obstacle
    P.admissibility = prob.admissibility
    for s, bc in enumerate(prob.bc):
        P.bc[s].kind = BC_CODES[bc.kind]
        for i in range(4):
            P.bc[s].state[i] = bc.state[i]
            P.bc[s].alt[i] = bc.alt[i]
        P.bc[s].wall_u, P.bc[s].wall_v, P.bc[s].wall_T = bc.wall
        P.bc[s].wall_omega = getattr(bc, "omega", 0.0)
    mesh = getattr(prob, "mesh", None)
    if mesh is not None:
        m = np.ascontiguousarray(mesh, dtype=np.float64)
        if m.shape != (prob.ny + 1, prob.nx + 1, 2):
            raise ValueError(f"mesh must have shape {(prob.ny + 1, prob.nx + 1, 2)}, not {m.shape}")
        P._mesh_keep = m  # read by the library during the call
        P.mesh = m.ctypes.data_as(_D)
    return P


def _ptr(a):
    return a.ctypes.data_as(_D)


def gks_init(probs, states, precision=GKS_FP64, stream=None, t0=None):
    """probs: list of workloads.Problem; states: list of workloads.State;
    precision: one value or one per problem; t0: initial times (default 0).
    Returns an opaque handle (c_void_p)."""
    n = len(probs)
    t0 = [0.0] * n if t0 is None else list(np.broadcast_to(np.asarray(t0, dtype=np.float64), (n,)))
    prec = [int(x) for x in np.broadcast_to(np.asarray(precision, dtype=np.int64), (n,))]
    ps = [to_c_problem(p, q, t) for p, q, t in zip(probs, prec, t0)]  # (their meshes stay alive for the call)
    cp = (gks_problem * n)(*ps)
    keep = []
    cells, fxs, fys = (_D * n)(), (_D * n)(), (_D * n)()
    for k, (p, st) in enumerate(zip(probs, states)):
        c = np.ascontiguousarray(st.cell, dtype=np.float64)
        fx = np.ascontiguousarray(st.fx, dtype=np.float64)
        fy = np.ascontiguousarray(st.fy, dtype=np.float64)
        keep += [c, fx, fy]
        cells[k], fxs[k], fys[k] = _ptr(c), _ptr(fx), _ptr(fy)
    h = _P()
    rc = lib().gks_init(C.byref(h), n, cp, cells, fxs, fys, stream)
    if rc != GKS_OK:
        raise GKSError(rc, "gks_init: " + lib().gks_last_error(None).decode())
    return h


def gks_state_extent(prob, precision=GKS_FP64):
    """Element counts (cell, face_x, face_y) of the device buffers that
    gks_init_device takes for one problem, and the byte size of a face
    element (8 for GKS_FP64, 4 for GKS_FP32_MIXED).  Host-only."""
    cp = to_c_problem(prob, precision)
    n = [C.c_int64() for _ in range(3)]
    fb = C.c_int32()
    rc = lib().gks_state_extent(C.byref(cp), *[C.byref(x) for x in n], C.byref(fb))
    if rc != GKS_OK:
        raise GKSError(rc, "gks_state_extent: " + lib().gks_last_error(None).decode())
    return n[0].value, n[1].value, n[2].value, fb.value


def ghosted(prob, state, precision=GKS_FP64, fill=np.nan):
    """Host arrays in the ghosted device layouts of gks_init_device (cell
    averages double; point values double or float by precision), holding
    `state` (workloads.State layout) and `fill` in every ghost entry."""
    nv, nx, ny = prob.nvar, prob.nx, prob.ny
    ft = np.float32 if precision == GKS_FP32_MIXED else np.float64
    if prob.dim == 2:
        cell = np.full((4, ny + 4, nx + 4), fill)
        cell[:, 2:ny + 2, 2:nx + 2] = state.cell
        fx = np.full((2, 4, ny + 2, nx + 3), fill, dtype=ft)
        fx[:, :, 1:ny + 1, 1:nx + 2] = state.fx
        fy = np.full((2, 4, ny + 3, nx + 2), fill, dtype=ft)
        fy[:, :, 1:ny + 2, 1:nx + 1] = state.fy
        return cell, fx, fy
    cell = np.full((nv, nx + 4), fill)
    cell[:, 2:nx + 2] = state.cell.reshape(nv, nx)
    fx = np.full((nv, nx + 3), fill, dtype=ft)
    fx[:, 1:nx + 2] = state.fx.reshape(nv, nx + 1)
    return cell, fx, None


def unghosted(prob, cell, fx, fy=None):
    """workloads.State (float64 copies) of arrays in the ghosted layouts."""
    from .workloads import State
    nv, nx, ny = prob.nvar, prob.nx, prob.ny
    if prob.dim == 2:
        return State(np.array(cell[:, 2:ny + 2, 2:nx + 2], dtype=np.float64),
                     np.array(fx[:, :, 1:ny + 1, 1:nx + 2], dtype=np.float64),
                     np.array(fy[:, :, 1:ny + 2, 1:nx + 1], dtype=np.float64))
    return State(np.array(cell[:, 2:nx + 2], dtype=np.float64).reshape(nv, 1, nx),
                 np.array(fx[:, 1:nx + 2], dtype=np.float64).reshape(1, nv, 1, nx + 1),
                 np.zeros((2, nv, 2, nx)))


def _addr(x):
    """Device address of an int or of an object with data_ptr() (a tensor)."""
    if x is None:
        return None
    return int(x) if isinstance(x, int) else int(x.data_ptr())


def gks_init_device(probs, d_cell, d_face_x, d_face_y, precision=GKS_FP64, stream=None, t0=None):
    """Device-borrow form of gks_init: d_cell, d_face_x, d_face_y are lists
    (one entry per problem) of device buffers in the ghosted layouts of
    include/gks.h, as ints or tensors; d_face_y entries are None for 1D
    problems.  The library steps them in place; they must outlive the
    handle."""
    n = len(probs)
    t0 = [0.0] * n if t0 is None else list(np.broadcast_to(np.asarray(t0, dtype=np.float64), (n,)))
    prec = [int(x) for x in np.broadcast_to(np.asarray(precision, dtype=np.int64), (n,))]
    ps = [to_c_problem(p, q, t) for p, q, t in zip(probs, prec, t0)]  # (their meshes stay alive for the call)
    cp = (gks_problem * n)(*ps)
    for k, (p, q) in enumerate(zip(probs, prec)):
        ext = gks_state_extent(p, q)
        for x, elems, item, what in ((d_cell[k], ext[0], 8, "d_cell"), (d_face_x[k], ext[1], ext[3], "d_face_x"),
                                     (d_face_y[k], ext[2], ext[3], "d_face_y")):
            if x is None or isinstance(x, int) or not hasattr(x, "is_contiguous"):
                continue  # raw addresses: the library checks them
            if not (x.is_cuda and x.is_contiguous() and x.element_size() == item and x.is_floating_point()
                    and x.numel() >= elems):
                raise GKSError(GKS_EINVAL, f"gks_init_device: problem {k}: {what} must be a contiguous device "
                                           f"tensor of {elems} floating-point elements of {item} bytes")
    arrs = [(_P * n)(*[_addr(x) for x in lst]) for lst in (d_cell, d_face_x, d_face_y)]
    h = _P()
    rc = lib().gks_init_device(C.byref(h), n, cp, *arrs, stream)
    if rc != GKS_OK:
        raise GKSError(rc, "gks_init_device: " + lib().gks_last_error(None).decode())
    return h


def gks_step(h, nsteps, dt_fixed=None, t_end=None):
    d = None if dt_fixed is None else np.ascontiguousarray(dt_fixed, dtype=np.float64)
    e = None if t_end is None else np.ascontiguousarray(t_end, dtype=np.float64)
    rc = lib().gks_step(h, int(nsteps), None if d is None else _ptr(d), None if e is None else _ptr(e))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))


def gks_fetch(h, problem, prob, check=True):
    """Returns (State, t, steps) of one problem.  check=False: also return the
    state of a handle that reported a nonphysical state, as (State, t, steps,
    status)."""
    from .workloads import State
    nv = prob.nvar
    cell = np.zeros((nv, prob.ny, prob.nx))
    ng = 2 if prob.dim == 2 else 1
    fx = np.zeros((ng, nv, prob.ny, prob.nx + 1))
    fy = np.zeros((2, nv, prob.ny + 1, prob.nx))
    t = C.c_double()
    steps = C.c_int64()
    rc = lib().gks_fetch(h, int(problem), _ptr(cell), _ptr(fx), _ptr(fy) if prob.dim == 2 else None,
                         C.byref(t), C.byref(steps))
    if not check and rc in (GKS_OK, GKS_ENONPHYS):
        return State(cell, fx, fy), t.value, steps.value, rc
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))
    return State(cell, fx, fy), t.value, steps.value


def gks_destroy(h):
    lib().gks_destroy(h)


def gks_last_error(h):
    return lib().gks_last_error(h).decode()


def gks_profile(h, mode):
    rc = lib().gks_profile(h, int(mode))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))


def gks_kernel_time(h, kernel):
    ms = C.c_double()
    n = C.c_int64()
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    rc = lib().gks_kernel_time(h, k, C.byref(ms), C.byref(n))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))
    return ms.value, n.value


def gks_tune(h, steps=3):
    rc = lib().gks_tune(h, int(steps))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))


def gks_block_size(h, kernel):
    n = C.c_int32()
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    rc = lib().gks_block_size(h, k, C.byref(n))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))
    return n.value


def gks_set_launch(h, kernel, threads, grid=0):
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    rc = lib().gks_set_launch(h, k, int(threads), int(grid))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))


def gks_launch_shape(h, kernel):
    """(threads per block, persistent grid or 0) of a kernel class"""
    n, g = C.c_int32(), C.c_int32()
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    rc = lib().gks_launch_shape(h, k, C.byref(n), C.byref(g))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))
    return n.value, g.value


def gks_step_noalloc(prob, d_cell, d_face_x, d_face_y, nsteps, dt_fixed=0.0, t_end=0.0, d_status=None,
                     precision=GKS_FP64, stream=None, t0=0.0):
    """Allocation-free stepping of one problem on device buffers in the
    layouts of gks_init_device (ints or tensors; d_face_y None in 1D);
    d_status: None or a device buffer of 32 bytes (gks_noalloc_status).
    Enqueued on `stream` (None: the null stream); returns at once."""
    cp = to_c_problem(prob, precision, t0)
    rc = lib().gks_step_noalloc(C.byref(cp), _addr(d_cell), _addr(d_face_x), _addr(d_face_y), int(nsteps),
                                float(dt_fixed), float(t_end), _addr(d_status), stream)
    if rc != GKS_OK:
        raise GKSError(rc, "gks_step_noalloc: " + lib().gks_last_error(None).decode())


def gks_fallbacks(h, problem):
    """(interior cell, step) pairs of `problem` whose reconstruction fell back
    to the constant average since gks_init."""
    n = C.c_int64()
    rc = lib().gks_fallbacks(h, int(problem), C.byref(n))
    if rc != GKS_OK:
        raise GKSError(rc, gks_last_error(h))
    return n.value


class Solver:
    """A handle over one or more problems (context manager)."""

    def __init__(self, probs, states, precision=GKS_FP64, stream=None, t0=None):
        if not isinstance(probs, (list, tuple)):
            probs, states = [probs], [states]
        self.probs = list(probs)
        self.h = None
        self.h = gks_init(self.probs, states, precision, stream, t0)

    def step(self, nsteps=1, dt=None, t_end=None):
        n = len(self.probs)
        d = None if dt is None else np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).copy()
        e = None if t_end is None else np.broadcast_to(np.asarray(t_end, dtype=np.float64), (n,)).copy()
        gks_step(self.h, nsteps, d, e)

    def tune(self, steps=3):
        gks_tune(self.h, steps)
        return {k: gks_block_size(self.h, k) for k in KERNELS}

    def set_launch(self, kernel, threads, grid=0):
        gks_set_launch(self.h, kernel, threads, grid)

    def launch_shape(self, kernel):
        return gks_launch_shape(self.h, kernel)

    def fetch(self, k=0, check=True):
        return gks_fetch(self.h, k, self.probs[k], check)

    def fallbacks(self, k=0):
        return gks_fallbacks(self.h, k)

    def close(self):
        if self.h is not None:
            gks_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
