"""Python binding of libhts (MI355X hydrothermal FE time stepping).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch supplies device memory (through the caching allocator)
and the stream.  Importing this package does not load the library; call
``load()`` (done implicitly by every entry point), which raises if
``libhts.so`` has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhts.so")

PRESSURE, TEMPERATURE = 0, 1
FP64, FP32 = 0, 1
MODE_FP64, MODE_FP32_REFINED, MODE_LEARNED = 0, 1, 2
BC_DIRICHLET, BC_NEUMANN, BC_NONE = 0, 1, 2
LINE_HEAT, LINE_WELL = 0, 1

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_STATE", -3: "ERR_NOMEM", -4: "ERR_HIP",
          -5: "ERR_NOT_CONVERGED", -6: "ERR_BREAKDOWN", -7: "ERR_UNSUPPORTED"}

EXPORTS = [
    "hts_default_opts", "hts_create_mesh", "hts_destroy_mesh", "hts_set_materials",
    "hts_set_face_bc", "hts_set_volume_source", "hts_add_line_source",
    "hts_add_dirichlet_column", "hts_set_state", "hts_get_state", "hts_set_previous_state",
    "hts_get_previous_state", "hts_get_heat_spectrum", "hts_set_heat_spectrum", "hts_mesh_sizes",
    "hts_apply_operator", "hts_solve_steady_pressure", "hts_solve_step", "hts_advance",
    "hts_autotune", "hts_last_error", "hts_nn_create", "hts_nn_destroy", "hts_nn_harvest",
    "hts_nn_train", "hts_nn_save", "hts_nn_load", "hts_kernel_timing", "hts_nn_num_params",
    "hts_nn_set_params", "hts_nn_get_params", "hts_nn_eval", "hts_nn_conv3d", "hts_nn_adam", "hts_nn_time_forward",
    "hts_stream_copy", "hts_apply_operator_noalloc",
]


class HtsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


class TimeFn(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c0", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("cz", C.c_double), ("amp", C.c_double), ("period", C.c_double),
                ("phase", C.c_double)]

    @classmethod
    def of(cls, t) -> "TimeFn":
        kind, c0, cx, cy, cz, amp, period, phase = t
        return cls(int(kind), c0, cx, cy, cz, amp, period, phase)


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class MeshDesc(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("extent", C.c_double * 3), ("ncells", C.c_int32 * 3),
                ("degree", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p),
                ("alloc", Allocator), ("edges", C.c_void_p * 3), ("coords", C.c_void_p)]


class Materials(C.Structure):
    _fields_ = [("permeability", C.c_void_p), ("hydraulic_conductivity", C.c_void_p),
                ("porosity", C.c_void_p), ("lambda_solid", C.c_void_p), ("rhoc_solid", C.c_void_p),
                ("lambda_bulk", C.c_void_p), ("rhoc_bulk", C.c_void_p),
                ("rho_w", C.c_double), ("mu_w", C.c_double), ("c_w", C.c_double),
                ("lambda_w", C.c_double), ("g", C.c_double), ("B_poro", C.c_double)]


class SolverOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("rtol", C.c_double), ("max_iter", C.c_int32),
                ("gmres_restart", C.c_int32), ("cheb_degree", C.c_int32),
                ("mg_coarse_max", C.c_int32), ("heat_cheb_degree", C.c_int32),
                ("inner_rtol", C.c_double), ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("nn", C.c_void_p), ("verbose", C.c_int32), ("heat_precond", C.c_int32),
                ("extrapolate", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 2), ("outer", C.c_int32 * 2), ("relres", C.c_double * 2),
                ("fallbacks", C.c_int32), ("status", C.c_int32 * 2), ("time_ms", C.c_double * 2)]

    def as_dict(self):
        return {"iters": list(self.iters), "outer": list(self.outer),
                "relres": list(self.relres), "fallbacks": self.fallbacks,
                "status": list(self.status), "time_ms": list(self.time_ms)}


class NNDesc(C.Structure):
    _fields_ = [("levels", C.c_int32), ("channels", C.c_int32 * 4), ("device", C.c_int32),
                ("stream", C.c_void_p), ("seed", C.c_uint64)]


class TrainStats(C.Structure):
    _fields_ = [("epochs_done", C.c_int32), ("pairs", C.c_int32), ("loss_first", C.c_double),
                ("loss_last", C.c_double), ("val_loss", C.c_double)]


class KernelTimes(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


_lib = None


def load():
    """Load libhts.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhts.so not built: run __graft_entry__.build() or "
                          "python -m paper_2103_00081_amd.build")
    import torch  # noqa: F401  (maps the HIP runtime the library shares)
    L = C.CDLL(LIB_PATH)
    vp, i32, d, st = C.c_void_p, C.c_int32, C.c_double, C.c_int
    P = C.POINTER
    sig = {
        "hts_default_opts": (None, [P(SolverOpts)]),
        "hts_create_mesh": (st, [P(MeshDesc), P(vp)]),
        "hts_destroy_mesh": (None, [vp]),
        "hts_set_materials": (st, [vp, P(Materials)]),
        "hts_set_face_bc": (st, [vp, i32, i32, i32, P(TimeFn)]),
        "hts_set_volume_source": (st, [vp, vp]),
        "hts_add_line_source": (st, [vp, d, d, d, d, i32, P(TimeFn), d]),
        "hts_add_dirichlet_column": (st, [vp, i32, d, d, d, d, P(TimeFn)]),
        "hts_set_state": (st, [vp, i32, vp, d]),
        "hts_get_state": (st, [vp, i32, vp, P(d)]),
        "hts_set_previous_state": (st, [vp, i32, i32, vp, d]),
        "hts_get_heat_spectrum": (st, [vp, vp]),
        "hts_set_heat_spectrum": (st, [vp, vp]),
        "hts_get_previous_state": (st, [vp, i32, i32, vp, P(d)]),
        "hts_mesh_sizes": (st, [vp, P(C.c_int64), P(C.c_int64)]),
        "hts_apply_operator": (st, [vp, i32, i32, d, vp, vp]),
        "hts_solve_steady_pressure": (st, [vp, P(SolverOpts), P(StepStats)]),
        "hts_solve_step": (st, [vp, d, P(SolverOpts), P(StepStats)]),
        "hts_advance": (st, [P(vp), i32, i32, d, P(SolverOpts), P(StepStats)]),
        "hts_autotune": (st, [P(vp), i32]),
        "hts_last_error": (C.c_char_p, []),
        "hts_nn_create": (st, [P(NNDesc), P(vp)]),
        "hts_nn_destroy": (None, [vp]),
        "hts_nn_harvest": (st, [vp, P(vp), i32, i32, d, i32]),
        "hts_nn_train": (st, [vp, i32, d, i32, i32, P(TrainStats)]),
        "hts_nn_num_params": (st, [vp, P(C.c_int64)]),
        "hts_nn_set_params": (st, [vp, vp, C.c_int64]),
        "hts_nn_get_params": (st, [vp, vp, C.c_int64]),
        "hts_nn_eval": (st, [vp, P(i32), vp, vp, vp, vp, P(d), vp]),
        "hts_nn_conv3d": (st, [i32, i32, i32, i32, P(i32), vp, vp, vp, vp, vp, vp, vp]),
        "hts_nn_adam": (st, [C.c_int64, i32, d, d, vp, vp, vp, vp, vp, vp]),
        "hts_nn_time_forward": (st, [vp, P(i32), i32, P(d), P(d)]),
        "hts_stream_copy": (st, [vp, vp, C.c_int64, i32, vp, P(d)]),
        "hts_apply_operator_noalloc": (st, [vp, i32, i32, d, vp, vp]),
        "hts_nn_save": (st, [vp, C.c_char_p]),
        "hts_nn_load": (st, [vp, C.c_char_p]),
        "hts_kernel_timing": (st, [i32, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(code: int):
    if code != 0:
        msg = load().hts_last_error()
        raise HtsError(code, msg.decode() if msg else "")


def default_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    load().hts_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


# ------------------------------------------------------ torch plumbing
_keep = []


def _torch_allocator(device: int) -> Allocator:
    import torch

    def _alloc(nbytes, stream, ctx):
        s = stream if stream else None
        return torch.cuda.caching_allocator_alloc(int(nbytes), device, s)

    def _free(ptr, ctx):
        cuda = getattr(torch, "cuda", None)
        if cuda is not None:   # None once the interpreter is shutting down
            cuda.caching_allocator_delete(int(ptr))

    a = Allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
    _keep.append(a)
    return a


def _ptr(t) -> int:
    return int(t.data_ptr())


class Mesh:
    """Owner of one hts_mesh."""

    def __init__(self, origin, extent, ncells, degree=1, device=0, stream=None,
                 torch_allocator=True, edges=None, coords=None):
        L = load()
        import torch
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        desc = MeshDesc()
        for k in range(3):
            desc.origin[k] = float(origin[k])
            desc.extent[k] = float(extent[k])
            desc.ncells[k] = int(ncells[k])
        desc.degree = int(degree)
        desc.device = self.device
        keep = []
        if edges is not None:
            for k in range(3):
                if edges[k] is None:
                    continue
                e = np.ascontiguousarray(edges[k], dtype=np.float64)
                if e.size != int(ncells[k]) + 1:
                    raise ValueError("edges[%d] must have ncells + 1 values" % k)
                keep.append(e)
                desc.edges[k] = e.ctypes.data
        if coords is not None:
            xyz = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
            keep.append(xyz)
            desc.coords = xyz.ctypes.data
        desc.stream = C.c_void_p(int(stream)) if stream else None
        if torch_allocator:
            desc.alloc = _torch_allocator(self.device)
        h = C.c_void_p()
        _check(L.hts_create_mesh(C.byref(desc), C.byref(h)))
        self.h = h
        self.degree = int(degree)
        self.ncells = tuple(int(n) for n in ncells)
        nn, nc = C.c_int64(), C.c_int64()
        _check(L.hts_mesh_sizes(h, C.byref(nn), C.byref(nc)))
        self.nnode, self.ncell = nn.value, nc.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hts_destroy_mesh(self.h)
            self.h = None

    # ---------------------------------------------------------- setters
    def set_materials(self, permeability, porosity, lambda_solid, rhoc_solid, rho_w, mu_w, c_w,
                      lambda_w, g, B_poro, hydraulic_conductivity=None, lambda_bulk=None,
                      rhoc_bulk=None):
        arrs = {}

        def arr(name, a):
            if a is None:
                return None
            x = np.ascontiguousarray(a, dtype=np.float64)
            if x.size != self.ncell:
                raise ValueError("%s must have %d entries" % (name, self.ncell))
            arrs[name] = x
            return x.ctypes.data

        m = Materials(arr("k", permeability), arr("K", hydraulic_conductivity), arr("phi", porosity),
                      arr("ls", lambda_solid), arr("cs", rhoc_solid), arr("lb", lambda_bulk),
                      arr("cb", rhoc_bulk), rho_w, mu_w, c_w, lambda_w, g, B_poro)
        _check(load().hts_set_materials(self.h, C.byref(m)))

    def set_face_bc(self, field, face, kind, value=None):
        tf = TimeFn.of(value) if value is not None else None
        _check(load().hts_set_face_bc(self.h, field, face, kind, C.byref(tf) if tf else None))

    def set_volume_source(self, w):
        if w is None:
            _check(load().hts_set_volume_source(self.h, None))
            return
        x = np.ascontiguousarray(w, dtype=np.float64)
        _check(load().hts_set_volume_source(self.h, x.ctypes.data))

    def add_line_source(self, x, y, z0, z1, kind, rate, T_inj=0.0):
        tf = TimeFn.of(rate)
        _check(load().hts_add_line_source(self.h, x, y, z0, z1, kind, C.byref(tf), T_inj))

    def add_dirichlet_column(self, field, x, y, z0, z1, value):
        tf = TimeFn.of(value)
        _check(load().hts_add_dirichlet_column(self.h, field, x, y, z0, z1, C.byref(tf)))

    def set_state(self, field, values, t=0.0):
        x = np.ascontiguousarray(values, dtype=np.float64)
        if x.size != self.nnode:
            raise ValueError("state must have %d entries" % self.nnode)
        _check(load().hts_set_state(self.h, field, x.ctypes.data, t))

    def get_state(self, field):
        out = np.zeros(self.nnode)
        t = C.c_double()
        _check(load().hts_get_state(self.h, field, out.ctypes.data, C.byref(t)))
        return out, t.value

    def set_previous_state(self, field, values, dt_prev, level=1):
        """A previous time level of the field (level 1: before the last
        step, 2: before the one before) and the step size after it (dt_prev
        0 forgets it; values may then be None).  Set level 1 before 2."""
        if values is None:
            _check(load().hts_set_previous_state(self.h, field, level, None, dt_prev))
            return
        x = np.ascontiguousarray(values, dtype=np.float64)
        if x.size != self.nnode:
            raise ValueError("state must have %d entries" % self.nnode)
        _check(load().hts_set_previous_state(self.h, field, level, x.ctypes.data, dt_prev))

    def get_heat_spectrum(self):
        """(dt, lmax without convection, lmax with convection, imaginary
        extent) behind the heat preconditioner; dt 0 when none was made."""
        out = np.zeros(4)
        _check(load().hts_get_heat_spectrum(self.h, out.ctypes.data))
        return tuple(float(v) for v in out)

    def set_heat_spectrum(self, values):
        x = np.ascontiguousarray(values, dtype=np.float64)
        if x.size != 4:
            raise ValueError("4 values")
        _check(load().hts_set_heat_spectrum(self.h, x.ctypes.data))

    def get_previous_state(self, field, level=1):
        """(values, dt_prev) of a previous time level; values None when it
        is not known (dt_prev 0)."""
        out = np.zeros(self.nnode)
        dt = C.c_double()
        _check(load().hts_get_previous_state(self.h, field, level, out.ctypes.data, C.byref(dt)))
        return (out if dt.value > 0.0 else None), dt.value

    # --------------------------------------------------------- operators
    def apply_operator(self, field, prec, dt, x, y):
        """y = A x on device tensors (float64 for FP64, float32 for FP32)."""
        _check(load().hts_apply_operator(self.h, field, prec, dt, _ptr(x), _ptr(y)))

    def apply_operator_noalloc(self, field, prec, dt, x, y):
        """As apply_operator, through the allocation-free entry point."""
        _check(load().hts_apply_operator_noalloc(self.h, field, prec, dt, _ptr(x), _ptr(y)))

    def solve_steady_pressure(self, opts=None):
        st = StepStats()
        code = load().hts_solve_steady_pressure(self.h, C.byref(opts) if opts else None,
                                                C.byref(st))
        _check(code)
        return st.as_dict()

    def solve_step(self, dt, opts=None, raise_on_error=True):
        st = StepStats()
        code = load().hts_solve_step(self.h, dt, C.byref(opts) if opts else None, C.byref(st))
        if raise_on_error:
            _check(code)
        return code, st.as_dict()


def advance(meshes: Sequence[Mesh], n_steps: int, dt: float, opts=None, raise_on_error=True):
    n = len(meshes)
    arr = (C.c_void_p * n)(*[m.h.value for m in meshes])
    st = (StepStats * n)()
    code = load().hts_advance(arr, n, n_steps, dt, C.byref(opts) if opts else None, st)
    if raise_on_error:
        _check(code)
    return code, [s.as_dict() for s in st]


def kernel_timing_start():
    _check(load().hts_kernel_timing(1, None))


def kernel_timing_stop():
    """Totals per (field, precision) of the fine-level operator launches."""
    out = (KernelTimes * 4)()
    _check(load().hts_kernel_timing(0, C.cast(out, C.c_void_p)))
    res = {}
    for f in range(2):
        for p in range(2):
            k = out[2 * f + p]
            res[(f, p)] = {"launches": k.launches, "ms": k.ms, "bytes": k.bytes,
                           "flops": k.flops}
    return res


def autotune(meshes: Sequence[Mesh]):
    n = len(meshes)
    arr = (C.c_void_p * n)(*[m.h.value for m in meshes])
    _check(load().hts_autotune(arr, n))


# ------------------------------------------------- learned preconditioner
def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Net:
    """Owner of one hts_nn (the learned preconditioner network)."""

    def __init__(self, levels=4, channels=(16, 32, 48, 64), device=0, stream=None, seed=0):
        import torch
        ch = list(channels) + [0] * (4 - len(channels))
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        d = NNDesc(levels, (C.c_int32 * 4)(*ch), device, C.c_void_p(stream), seed)
        self.h = C.c_void_p()
        _check(load().hts_nn_create(C.byref(d), C.byref(self.h)))
        self.levels, self.channels = levels, tuple(channels[:levels])

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hts_nn_destroy(h)
            self.h = None

    def num_params(self) -> int:
        n = C.c_int64()
        _check(load().hts_nn_num_params(self.h, C.byref(n)))
        return n.value

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        _check(load().hts_nn_set_params(self.h, _np_ptr(th), th.size))

    def get_params(self):
        th = np.empty(self.num_params())
        _check(load().hts_nn_get_params(self.h, _np_ptr(th), th.size))
        return th

    def eval(self, dims, inp, target=None, mask=None, grad=False):
        """dims (NX, NY, NZ); inp [n][2] -> (out [n], loss, grad or None)."""
        n = int(np.prod(dims))
        x = np.ascontiguousarray(inp, dtype=np.float32).reshape(n, 2)
        t = None if target is None else np.ascontiguousarray(target, dtype=np.float32).reshape(n)
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(n)
        out = np.empty(n, dtype=np.float32)
        lv = C.c_double(0.0)
        g = np.empty(self.num_params()) if grad else None
        dd = (C.c_int32 * 3)(*dims)
        _check(load().hts_nn_eval(self.h, dd, _np_ptr(x), _np_ptr(t), _np_ptr(m), _np_ptr(out),
                                  C.byref(lv) if t is not None else None, _np_ptr(g)))
        return out, (lv.value if t is not None else None), g

    def harvest(self, meshes, n_steps, dt, pairs_per_solve):
        arr = (C.c_void_p * len(meshes))(*[mm.h.value for mm in meshes])
        _check(load().hts_nn_harvest(self.h, arr, len(meshes), n_steps, dt, pairs_per_solve))

    def train(self, epochs, lr, batch, val_draws):
        st = TrainStats()
        _check(load().hts_nn_train(self.h, epochs, lr, batch, val_draws, C.byref(st)))
        return {"epochs": st.epochs_done, "pairs": st.pairs, "loss_first": st.loss_first,
                "loss_last": st.loss_last, "val_loss": st.val_loss}

    def time_forward(self, dims, reps=5):
        """(ms per forward pass, flops per forward pass) on a dims grid."""
        ms, fl = C.c_double(), C.c_double()
        _check(load().hts_nn_time_forward(self.h, (C.c_int32 * 3)(*dims), reps, C.byref(ms), C.byref(fl)))
        return ms.value, fl.value

    def save(self, path):
        _check(load().hts_nn_save(self.h, str(path).encode()))

    def load(self, path):
        _check(load().hts_nn_load(self.h, str(path).encode()))


def conv3d(op, cin, cout, stride, din, x=None, w=None, bias=None, g=None):
    """One BF16 matrix-core convolution layer (verification entry point).
    x, g: uint16 BF16 bit patterns [voxel][channel]; w: uint16 [cout][cin][3][3][3]."""
    di = (C.c_int32 * 3)(*din)
    dout = [(n - 1) // stride + 1 for n in din]
    nin, nout = int(np.prod(din)), int(np.prod(dout))
    if op == 0:
        out = np.empty((nout, cout), dtype=np.float32)
    elif op == 1:
        out = np.empty((nin, cin), dtype=np.float32)
    else:
        out = np.empty((cout, cin, 3, 3, 3), dtype=np.float32)
    ob = np.empty(cout, dtype=np.float32) if op == 2 else None
    c = lambda a, dt: None if a is None else np.ascontiguousarray(a, dtype=dt)
    x, w, g, b = c(x, np.uint16), c(w, np.uint16), c(g, np.uint16), c(bias, np.float32)
    _check(load().hts_nn_conv3d(op, cin, cout, stride, di, _np_ptr(x), _np_ptr(w), _np_ptr(b),
                                _np_ptr(g), _np_ptr(out), _np_ptr(ob), None))
    return (out, ob) if op == 2 else out


def adam_step(step, lr, gscale, w, m, v, g):
    """One Adam update on the device (verification entry point).  Returns
    new copies (w, m, v, w as BF16 bit patterns); inputs are FP32."""
    c = lambda a: np.array(a, dtype=np.float32, copy=True, order="C")
    w, m, v, g = c(w), c(m), c(v), c(g)
    wbf = np.empty(w.size, dtype=np.uint16)
    _check(load().hts_nn_adam(w.size, int(step), float(lr), float(gscale), _np_ptr(w), _np_ptr(m), _np_ptr(v),
                              _np_ptr(g), _np_ptr(wbf), None))
    return w, m, v, wbf


def stream_copy(src, dst, reps=20):
    """Mean device time (ms) of one plain streaming copy src -> dst (device
    tensors of the same byte size) by the library's copy kernel."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb
    ms = C.c_double()
    _check(load().hts_stream_copy(_ptr(src), _ptr(dst), nb, reps, None, C.byref(ms)))
    return ms.value


# --------------------------------------------------- scenario marshalling
def _node_coords(scn):
    if getattr(scn, "coords", None) is not None:
        xyz = np.asarray(scn.coords, dtype=np.float64).reshape(-1, 3)
        return xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy()
    p = scn.degree
    edges = getattr(scn, "edges", None)
    ax = []
    for d in range(3):
        if edges is not None and edges[d] is not None:
            e = np.asarray(edges[d], dtype=np.float64)
            if p == 2:   # mid-edge nodes at the cell midpoints
                a = np.empty(2 * e.size - 1)
                a[0::2], a[1::2] = e, 0.5 * (e[:-1] + e[1:])
                e = a
            ax.append(e)
        else:
            ax.append(scn.origin[d] + np.arange(p * scn.ncells[d] + 1) * (scn.extent[d] / (p * scn.ncells[d])))
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


def _tf_at_nodes(tf, X, Y, Z):
    kind, c0, cx, cy, cz, amp, period, phase = tf
    if kind != 0:
        raise ValueError("initial states must be time independent")
    return c0 + cx * X + cy * Y + cz * Z


def from_scenario(scn, device=0, stream=None, initial=True, opts=None) -> Mesh:
    """Create and fill a Mesh from a synth.Scenario (same arrays the oracle
    receives).  With initial=True the state is set from the scenario's
    initial functions, and the steady pressure is solved when requested."""
    m = Mesh(scn.origin, scn.extent, scn.ncells, scn.degree, device, stream,
             edges=getattr(scn, "edges", None), coords=getattr(scn, "coords", None))
    m.set_materials(scn.permeability, scn.porosity, scn.lambda_solid, scn.rhoc_solid,
                    scn.rho_w, scn.mu_w, scn.c_w, scn.lambda_w, scn.g, scn.B_poro,
                    hydraulic_conductivity=getattr(scn, "hydraulic_conductivity", None),
                    lambda_bulk=getattr(scn, "lambda_bulk", None),
                    rhoc_bulk=getattr(scn, "rhoc_bulk", None))
    for bc in scn.bcs:
        m.set_face_bc(bc.field, bc.face, bc.kind, bc.value)
    if scn.heat_source is not None:
        m.set_volume_source(scn.heat_source)
    for ln in scn.lines:
        m.add_line_source(ln.x, ln.y, ln.z0, ln.z1, ln.kind, ln.rate, ln.T_inj)
    for c in scn.dir_columns:
        m.add_dirichlet_column(c.field, c.x, c.y, c.z0, c.z1, c.value)
    if initial:
        X, Y, Z = _node_coords(scn)
        m.set_state(PRESSURE, _tf_at_nodes(scn.P0, X, Y, Z), scn.t0)
        m.set_state(TEMPERATURE, _tf_at_nodes(scn.T0, X, Y, Z), scn.t0)
        if scn.P0_steady:
            m.solve_steady_pressure(opts)
    return m
