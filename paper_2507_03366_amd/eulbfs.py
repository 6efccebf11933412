"""Python binding of the C ABI in include/eulbfs.h (ctypes).

The functions keep the C names and only marshal arguments; every step of the
solver runs in the HIP kernels of libeulbfs.so.  PyTorch is used only to hold
device memory (the workspace) and to name the HIP stream.  There is no CPU
fallback: importing this module without a built libeulbfs.so raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeulbfs.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, EBUSY, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
KERNEL_FUSED, KERNEL_SPLIT, KERNEL_AUTO = 0, 1, 2
INIT_PRIMITIVE, INIT_CONSERVED, INIT_ANALYTIC = 0, 1, 2
ABI_VERSION = 6
FIELD = dict(H=0, P=1, MX=2, MY=3, C=4, FSDOT=5, T=6, FL=7, FS=8, RHO=9, U=10, V=11, MUC=12, W_ALL=13,
             W_GHOSTED=14)
SCALAR_DIAG = 100
NDIAG = 14
DIAG_NAMES = ("mass", "volume_C", "enthalpy", "solid", "umax", "nonfinite", "tip", "time", "steps", "dt",
              "c_min", "c_max", "wetted_length", "axis_height")


class EulbfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"eulbfs error {code}: {msg}")
        self.code = code


class eulbfs_bc(ct.Structure):
    _fields_ = [("periodic", ct.c_int32), ("flow", ct.c_int32), ("heat", ct.c_int32), ("reserved", ct.c_int32),
                ("T_w", ct.c_double), ("theta_deg", ct.c_double), ("theta_adv", ct.c_double),
                ("theta_rec", ct.c_double)]


class eulbfs_params(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_uint32), ("abi_version", ct.c_uint32),
        ("nx", ct.c_int32), ("ny", ct.c_int32), ("lattice_hg", ct.c_int32), ("precision", ct.c_int32),
        ("kernel", ct.c_int32), ("surf_model", ct.c_int32),
        ("dx", ct.c_double), ("delta_t", ct.c_double), ("dt", ct.c_double),
        ("rho", ct.c_double * 3), ("mu", ct.c_double * 3), ("lambda_", ct.c_double * 3), ("cp", ct.c_double * 3),
        ("latent", ct.c_double), ("T_s", ct.c_double), ("T_l", ct.c_double),
        ("sigma", ct.c_double), ("xi", ct.c_double), ("mobility", ct.c_double), ("Qg", ct.c_double),
        ("gx", ct.c_double), ("gy", ct.c_double),
        ("bc", eulbfs_bc * 4),
        ("tile_x", ct.c_int32), ("tile_y", ct.c_int32),
        ("x_width", ct.POINTER(ct.c_double)), ("y_width", ct.POINTER(ct.c_double)), ("c_source", ct.c_int32),
        ("reserved", ct.c_int32),
    ]


class eulbfs_shape(ct.Structure):
    _fields_ = [("profile", ct.c_int32), ("axis", ct.c_int32), ("c0", ct.c_double), ("h0", ct.c_double),
                ("x0", ct.c_double), ("y0", ct.c_double), ("r0", ct.c_double), ("t_out", ct.c_double),
                ("t_in", ct.c_double), ("t_amp", ct.c_double), ("seed", ct.c_uint64), ("fl0", ct.c_double),
                ("u_in", ct.c_double), ("v_in", ct.c_double)]


class eulbfs_init(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("on_device", ct.c_int32), ("planes", ct.POINTER(ct.c_double)),
                ("shape", ct.POINTER(eulbfs_shape))]


def shape_struct(sh) -> eulbfs_shape:
    """An eulbfs_shape from a problems.Shape (field for field)."""
    return eulbfs_shape(int(sh.profile), int(sh.axis), float(sh.c0), float(sh.h0), float(sh.x0), float(sh.y0),
                        float(sh.r0), float(sh.t_out), float(sh.t_in), float(sh.t_amp), int(sh.seed), float(sh.fl0),
                        float(sh.u_in), float(sh.v_in))


_lib = None


def lib():
    """Load libeulbfs.so (built in-tree by paper_2507_03366_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_03366_amd.build`")
        L = ct.CDLL(LIB_PATH)
        vp, dp, sz = ct.c_void_p, ct.POINTER(ct.c_double), ct.c_size_t
        pp = ct.POINTER(eulbfs_params)
        L.eulbfs_check_params.argtypes = [pp, ct.c_char_p, sz]
        L.eulbfs_workspace_bytes.argtypes = [pp]
        L.eulbfs_workspace_bytes.restype = sz
        L.eulbfs_create.argtypes = [pp, ct.POINTER(eulbfs_init), vp, sz, vp, ct.POINTER(vp)]
        L.eulbfs_step.argtypes = [vp, ct.c_int64]
        L.eulbfs_run.argtypes = [vp, ct.c_int64, ct.c_double]
        L.eulbfs_query.argtypes = [vp, ct.c_int32, vp, sz, ct.c_int32]
        L.eulbfs_set_field.argtypes = [vp, ct.c_int32, vp, sz, ct.c_int32]
        L.eulbfs_residual.argtypes = [vp, dp, dp, dp, ct.c_int32]
        L.eulbfs_residual_noalloc.argtypes = [vp, dp, dp, dp, ct.c_int32]
        L.eulbfs_destroy.argtypes = [vp]
        L.eulbfs_schedule.argtypes = [vp, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32)]
        L.eulbfs_last_error.argtypes = [vp]
        L.eulbfs_last_error.restype = ct.c_char_p
        for f in ("eulbfs_check_params", "eulbfs_create", "eulbfs_step", "eulbfs_run", "eulbfs_query",
                  "eulbfs_set_field", "eulbfs_residual", "eulbfs_residual_noalloc", "eulbfs_destroy"):
            getattr(L, f).restype = ct.c_int
        _lib = L
    return _lib


def _raise(rc, handle=None):
    if rc != OK:
        msg = lib().eulbfs_last_error(handle)
        raise EulbfsError(rc, msg.decode() if msg else "")


# ---------------------------------------------------------------------------
# Parameter marshalling
# ---------------------------------------------------------------------------
def params_from_problem(pr, precision: int = None, kernel: int = KERNEL_FUSED, tile=(0, 0)) -> eulbfs_params:
    P = eulbfs_params()
    P.struct_size = ct.sizeof(eulbfs_params)
    P.abi_version = ABI_VERSION
    P.nx, P.ny = pr.nx, pr.ny
    P.lattice_hg = pr.lattice_hg
    P.precision = pr.precision if precision is None else precision
    P.kernel = kernel
    P.surf_model = pr.surf_model
    P.c_source = pr.c_source
    P.dx, P.delta_t, P.dt = pr.dx, pr.delta_t, pr.dt
    P.rho[:] = list(pr.rho)
    P.mu[:] = list(pr.mu)
    P.lambda_[:] = list(pr.lam)
    P.cp[:] = list(pr.cp)
    P.latent, P.T_s, P.T_l = pr.latent, pr.T_s, pr.T_l
    P.sigma, P.xi, P.mobility, P.Qg = pr.sigma, pr.xi, pr.mobility, pr.Qg
    P.gx, P.gy = pr.gx, pr.gy
    for k, side in enumerate(("x-", "x+", "y-", "y+")):
        w = pr.wall(side)
        if w is None:
            P.bc[k].periodic = 1
            P.bc[k].theta_deg = 90.0
        else:
            P.bc[k].periodic = 0
            P.bc[k].flow, P.bc[k].heat = w.flow, w.heat
            P.bc[k].T_w, P.bc[k].theta_deg = w.T_w, w.theta_deg
            P.bc[k].theta_adv, P.bc[k].theta_rec = w.theta_adv, w.theta_rec
    P.tile_x, P.tile_y = tile
    # stretched mesh: host arrays, kept alive by the struct (the library copies them at create)
    P._widths = []
    for name, src, n in (("x_width", pr.x_width, pr.nx), ("y_width", pr.y_width, pr.ny)):
        if src is not None:
            a = np.ascontiguousarray(src, dtype=np.float64)
            if a.shape != (n,):
                raise ValueError(f"{name}: expected {n} widths, got shape {a.shape}")
            P._widths.append(a)
            setattr(P, name, a.ctypes.data_as(ct.POINTER(ct.c_double)))
    return P


# ---------------------------------------------------------------------------
# C-ABI functions (same names; argument marshalling only)
# ---------------------------------------------------------------------------
def eulbfs_check_params(P: eulbfs_params) -> str:
    buf = ct.create_string_buffer(256)
    rc = lib().eulbfs_check_params(ct.byref(P), buf, 256)
    return "" if rc == OK else buf.value.decode()


def eulbfs_workspace_bytes(P: eulbfs_params) -> int:
    return int(lib().eulbfs_workspace_bytes(ct.byref(P)))


def _init_of(init_planes, kind: int, shape):
    """The eulbfs_init for host or device planes, or for a problems.Shape
    (EULBFS_INIT_ANALYTIC); returns it with the objects it points to."""
    init = eulbfs_init()
    if shape is not None:
        sh = shape_struct(shape)
        init.kind, init.on_device = INIT_ANALYTIC, 0
        init.shape = ct.pointer(sh)
        return init, sh
    init.kind = kind
    if isinstance(init_planes, np.ndarray):
        arr = np.ascontiguousarray(init_planes, dtype=np.float64)
        init.on_device = 0
        init.planes = arr.ctypes.data_as(ct.POINTER(ct.c_double))
        return init, arr
    assert init_planes.dtype.itemsize == 8 and init_planes.is_contiguous()
    init.on_device = 1
    init.planes = ct.cast(ct.c_void_p(init_planes.data_ptr()), ct.POINTER(ct.c_double))
    return init, init_planes


def eulbfs_create(P: eulbfs_params, init_planes=None, kind: int = INIT_PRIMITIVE, workspace=None, stream=None,
                  shape=None):
    """init_planes: float64 array of 6 * nx * ny (host numpy or device torch tensor);
    or shape: a problems.Shape whose fields the library builds on the device.
    workspace: a torch uint8 CUDA tensor of >= eulbfs_workspace_bytes(P) (or None).
    stream: a torch.cuda.Stream (or None: the default stream).  Returns the handle."""
    init, _held = _init_of(init_planes, kind, shape)  # _held: what init points to, alive through the call
    ws_ptr = ct.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = ct.c_void_p(stream.cuda_stream) if stream is not None else None
    h = ct.c_void_p()
    _raise(lib().eulbfs_create(ct.byref(P), ct.byref(init), ws_ptr, ws_bytes, st, ct.byref(h)))
    return h


def eulbfs_step(h, nsteps: int) -> None:
    _raise(lib().eulbfs_step(h, int(nsteps)), h)


def eulbfs_run(h, nsteps: int, t_end: float = float("inf")) -> None:
    _raise(lib().eulbfs_run(h, int(nsteps), float(t_end)), h)


def eulbfs_query(h, what: int, nx: int, ny: int) -> np.ndarray:
    if what == SCALAR_DIAG:
        out = np.zeros(NDIAG)
    elif what == FIELD["W_ALL"]:
        out = np.zeros((6, ny, nx))
    elif what == FIELD["W_GHOSTED"]:
        out = np.zeros((5, ny + 6, nx + 6))
    else:
        out = np.zeros((ny, nx))
    _raise(lib().eulbfs_query(h, what, out.ctypes.data_as(ct.c_void_p), out.nbytes, 0), h)
    return out


def eulbfs_set_field(h, what: int, data: np.ndarray) -> None:
    arr = np.ascontiguousarray(data, dtype=np.float64)
    _raise(lib().eulbfs_set_field(h, what, arr.ctypes.data_as(ct.c_void_p), arr.nbytes, 0), h)


def eulbfs_residual(h, nx: int, ny: int):
    R = np.zeros((5, ny, nx))
    Fx = np.zeros((5, ny, nx + 1))
    Fy = np.zeros((5, ny + 1, nx))
    dp = ct.POINTER(ct.c_double)
    _raise(lib().eulbfs_residual(h, R.ctypes.data_as(dp), Fx.ctypes.data_as(dp), Fy.ctypes.data_as(dp), 0), h)
    return R, Fx, Fy


def eulbfs_residual_noalloc(h, nx: int, ny: int):
    R = np.zeros((5, ny, nx))
    Fx = np.zeros((5, ny, nx + 1))
    Fy = np.zeros((5, ny + 1, nx))
    dp = ct.POINTER(ct.c_double)
    _raise(lib().eulbfs_residual_noalloc(h, R.ctypes.data_as(dp), Fx.ctypes.data_as(dp), Fy.ctypes.data_as(dp), 0),
           h)
    return R, Fx, Fy


def eulbfs_schedule(h):
    """(kernel, tile_x, tile_y) the solver steps with."""
    k, tx, ty = ct.c_int32(), ct.c_int32(), ct.c_int32()
    _raise(lib().eulbfs_schedule(h, ct.byref(k), ct.byref(tx), ct.byref(ty)), h)
    return k.value, tx.value, ty.value


def eulbfs_destroy(h) -> None:
    lib().eulbfs_destroy(h)


def eulbfs_last_error(h=None) -> str:
    m = lib().eulbfs_last_error(h)
    return m.decode() if m else ""


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------
class Solver:
    """One grid on the GPU: workspace in a torch uint8 tensor, work on a torch stream."""

    def __init__(self, pr, state=None, *, precision=None, kernel=KERNEL_FUSED, tile=(0, 0), device="cuda:0",
                 stream=None, conserved=None, own_workspace=True, analytic=False):
        """analytic: build the initial fields on the device from state.shape
        (EULBFS_INIT_ANALYTIC) instead of copying the host planes."""
        import torch

        self.pr = pr
        self.P = params_from_problem(pr, precision=precision, kernel=kernel, tile=tile)
        msg = eulbfs_check_params(self.P)
        if msg:
            raise EulbfsError(EINVAL, msg)
        self.nx, self.ny = pr.nx, pr.ny
        self.device = torch.device(device)
        nbytes = eulbfs_workspace_bytes(self.P)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device) if own_workspace else None
        ws = None
        if self.workspace is not None:
            off = (-self.workspace.data_ptr()) % 256
            ws = self.workspace[off:off + nbytes]
        self.stream = stream
        if conserved is not None:
            self.h = eulbfs_create(self.P, np.ascontiguousarray(conserved, dtype=np.float64).ravel(),
                                   kind=INIT_CONSERVED, workspace=ws, stream=stream)
        elif analytic:
            if state.shape is None:
                raise ValueError("this initial state has no closed-form shape")
            self.h = eulbfs_create(self.P, workspace=ws, stream=stream, shape=state.shape)
        else:
            planes = np.concatenate([a.ravel() for a in state.planes()])
            self.h = eulbfs_create(self.P, planes, kind=INIT_PRIMITIVE, workspace=ws, stream=stream)

    def step(self, n: int):
        eulbfs_step(self.h, n)

    def run(self, n: int, t_end: float = float("inf")):
        eulbfs_run(self.h, n, t_end)

    def field(self, name: str) -> np.ndarray:
        return eulbfs_query(self.h, FIELD[name], self.nx, self.ny)

    def conserved(self) -> np.ndarray:
        """(6, ny, nx): H, p, Mx, My, C, dF_s/dt."""
        return eulbfs_query(self.h, FIELD["W_ALL"], self.nx, self.ny)

    def ghosted(self) -> np.ndarray:
        return eulbfs_query(self.h, FIELD["W_GHOSTED"], self.nx, self.ny)

    def diagnostics(self) -> dict:
        d = eulbfs_query(self.h, SCALAR_DIAG, self.nx, self.ny)
        return dict(zip(DIAG_NAMES, d))

    def residual(self):
        return eulbfs_residual(self.h, self.nx, self.ny)

    def schedule(self):
        """(kernel, tile_x, tile_y) in use (the tile is what KERNEL_AUTO picked)."""
        return eulbfs_schedule(self.h)

    def set_conserved(self, w6: np.ndarray):
        eulbfs_set_field(self.h, FIELD["W_ALL"], w6)

    def close(self):
        if self.h is not None:
            eulbfs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Batch API
# ---------------------------------------------------------------------------
def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        vp, sz = ct.c_void_p, ct.c_size_t
        pp = ct.POINTER(eulbfs_params)
        L.eulbfs_batch_create.argtypes = [sz, ct.c_int32, ct.c_int32, vp, sz, vp, ct.POINTER(vp)]
        L.eulbfs_batch_request_bytes.argtypes = [pp]
        L.eulbfs_batch_request_bytes.restype = sz
        L.eulbfs_batch_admit.argtypes = [vp, pp, ct.POINTER(eulbfs_init), ct.c_int64, ct.POINTER(ct.c_int32)]
        L.eulbfs_batch_tick.argtypes = [vp, ct.c_int32]
        L.eulbfs_batch_poll.argtypes = [vp, ct.POINTER(ct.c_int32), ct.c_int32, ct.POINTER(ct.c_int32)]
        L.eulbfs_batch_query.argtypes = [vp, ct.c_int32, ct.c_int32, vp, sz, ct.c_int32]
        L.eulbfs_batch_release.argtypes = [vp, ct.c_int32]
        L.eulbfs_batch_destroy.argtypes = [vp]
        L.eulbfs_batch_last_error.argtypes = [vp]
        L.eulbfs_batch_last_error.restype = ct.c_char_p
        L.eulbfs_batch_set_tile.argtypes = [vp, ct.c_int32]
        L.eulbfs_batch_schedule.argtypes = [vp, ct.POINTER(eulbfs_batch_sched)]
        for f in ("eulbfs_batch_create", "eulbfs_batch_admit", "eulbfs_batch_tick", "eulbfs_batch_poll",
                  "eulbfs_batch_query", "eulbfs_batch_release", "eulbfs_batch_destroy", "eulbfs_batch_set_tile",
                  "eulbfs_batch_schedule"):
            getattr(L, f).restype = ct.c_int
        L._batch_ready = True
    return L


def _braise(rc, b=None):
    if rc != OK:
        msg = _batch_lib().eulbfs_batch_last_error(b)
        raise EulbfsError(rc, msg.decode() if msg else "")


def eulbfs_batch_request_bytes(P: eulbfs_params) -> int:
    return int(_batch_lib().eulbfs_batch_request_bytes(ct.byref(P)))


def eulbfs_batch_create(hbm_budget: int, max_slots: int, precision: int, workspace=None, stream=None):
    ws = ct.c_void_p(workspace.data_ptr()) if workspace is not None else None
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = ct.c_void_p(stream.cuda_stream) if stream is not None else None
    b = ct.c_void_p()
    _braise(_batch_lib().eulbfs_batch_create(int(hbm_budget), int(max_slots), int(precision), ws, ws_bytes, st,
                                             ct.byref(b)))
    return b


def eulbfs_batch_admit(b, P: eulbfs_params, init_planes, nsteps: int, kind: int = INIT_PRIMITIVE, shape=None):
    """Host planes (or a problems.Shape, built on the device); returns the slot
    index, or None when the batch is full (EBUSY)."""
    init, _held = _init_of(init_planes, kind, shape)  # _held: what init points to, alive through the call
    slot = ct.c_int32(-1)
    rc = _batch_lib().eulbfs_batch_admit(b, ct.byref(P), ct.byref(init), int(nsteps), ct.byref(slot))
    if rc == EBUSY:
        return None
    _braise(rc, b)
    return slot.value


def eulbfs_batch_tick(b, steps: int) -> None:
    _braise(_batch_lib().eulbfs_batch_tick(b, int(steps)), b)


def eulbfs_batch_poll(b, cap: int = 4096):
    out = (ct.c_int32 * cap)()
    n = ct.c_int32(0)
    _braise(_batch_lib().eulbfs_batch_poll(b, out, cap, ct.byref(n)), b)
    return [out[k] for k in range(n.value)]


def eulbfs_batch_query(b, slot: int, what: int, nx: int, ny: int) -> np.ndarray:
    if what == SCALAR_DIAG:
        out = np.zeros(NDIAG)
    elif what == FIELD["W_ALL"]:
        out = np.zeros((6, ny, nx))
    else:
        out = np.zeros((ny, nx))
    _braise(_batch_lib().eulbfs_batch_query(b, slot, what, out.ctypes.data_as(ct.c_void_p), out.nbytes, 0), b)
    return out


BATCH_TILE_AUTO, BATCH_TILE_32x16, BATCH_TILE_64x8 = 0, 1, 2
BATCH_TILE_NAMES = {BATCH_TILE_32x16: "32x16", BATCH_TILE_64x8: "64x8"}


class eulbfs_batch_sched(ct.Structure):
    _fields_ = [("next_tile", ct.c_int32), ("reserved", ct.c_int32), ("ns_per_cell_step", ct.c_double * 2),
                ("ticks_timed", ct.c_int64 * 2), ("time_ratio", ct.c_double), ("pairs", ct.c_int64)]


def eulbfs_batch_set_tile(b, tile: int) -> None:
    _braise(_batch_lib().eulbfs_batch_set_tile(b, int(tile)), b)


def eulbfs_batch_schedule(b) -> dict:
    """What the batch's tile choice has measured: the next tick's tile, device
    ns per cell-step and timed ticks of each shape, the paired time ratio
    64x8 / 32x16 and the number of pairs."""
    s = eulbfs_batch_sched()
    _braise(_batch_lib().eulbfs_batch_schedule(b, ct.byref(s)), b)
    return {"next_tile": s.next_tile, "ns_per_cell_step": [s.ns_per_cell_step[0], s.ns_per_cell_step[1]],
            "ticks_timed": [s.ticks_timed[0], s.ticks_timed[1]], "time_ratio": s.time_ratio, "pairs": s.pairs}


def eulbfs_batch_release(b, slot: int) -> None:
    _braise(_batch_lib().eulbfs_batch_release(b, slot), b)


def eulbfs_batch_destroy(b) -> None:
    _batch_lib().eulbfs_batch_destroy(b)


def eulbfs_batch_last_error(b=None) -> str:
    m = _batch_lib().eulbfs_batch_last_error(b)
    return m.decode() if m else ""


class Batch:
    """Many grids resident in one device arena, advanced together."""

    def __init__(self, hbm_budget: int, max_slots: int, precision: int = FP32, device="cuda:0", stream=None):
        import torch

        self.device = torch.device(device)
        self.workspace = torch.empty(int(hbm_budget) + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.precision = precision
        self.stream = stream
        self.b = eulbfs_batch_create(hbm_budget, max_slots, precision, self.workspace[off:off + int(hbm_budget)],
                                     stream)
        self.shapes = {}

    def admit(self, pr, state, nsteps: int, analytic: bool = False):
        """analytic: the device builds the initial fields from state.shape."""
        P = params_from_problem(pr, precision=self.precision)
        if analytic:
            if state.shape is None:
                raise ValueError("this initial state has no closed-form shape")
            slot = eulbfs_batch_admit(self.b, P, None, nsteps, shape=state.shape)
        else:
            slot = eulbfs_batch_admit(self.b, P, np.concatenate([a.ravel() for a in state.planes()]), nsteps)
        if slot is not None:
            self.shapes[slot] = (pr.nx, pr.ny)
        return slot

    def tick(self, steps: int):
        eulbfs_batch_tick(self.b, steps)

    def poll(self):
        return eulbfs_batch_poll(self.b)

    def conserved(self, slot: int) -> np.ndarray:
        nx, ny = self.shapes[slot]
        return eulbfs_batch_query(self.b, slot, FIELD["W_ALL"], nx, ny)

    def diagnostics(self, slot: int) -> dict:
        nx, ny = self.shapes[slot]
        return dict(zip(DIAG_NAMES, eulbfs_batch_query(self.b, slot, SCALAR_DIAG, nx, ny)))

    def set_tile(self, tile: int):
        eulbfs_batch_set_tile(self.b, tile)

    def schedule(self):
        return eulbfs_batch_schedule(self.b)

    def release(self, slot: int):
        eulbfs_batch_release(self.b, slot)
        self.shapes.pop(slot, None)

    def close(self):
        if self.b is not None:
            eulbfs_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
