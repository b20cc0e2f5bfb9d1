"""Thin ctypes binding over libfdtd.so (the C ABI declared in include/fdtd.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  Host arrays are numpy float32; device buffers are torch CUDA
(HIP) tensors, passed by pointer with ``where=FDTD_DEVICE``.  PyTorch is used
for device memory and streams only.

The library is loaded from this package's directory; if it has not been
built, loading raises immediately (there is no fallback of any kind).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdtd.so")

FDTD_OK, FDTD_EINVAL, FDTD_ENOMEM, FDTD_EHIP, FDTD_ESTATE, FDTD_EUNSUPPORTED, FDTD_ETIMEOUT = \
    0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {0: "FDTD_OK", -1: "FDTD_EINVAL", -2: "FDTD_ENOMEM", -3: "FDTD_EHIP",
               -4: "FDTD_ESTATE", -5: "FDTD_EUNSUPPORTED", -6: "FDTD_ETIMEOUT"}
BC_PEC, BC_PERIODIC = 0, 1
SCHEME_PLAIN, SCHEME_SYSTOLIC, SCHEME_PLAIN_FUSED = 0, 1, 2
FP32, FP16_STORAGE = 0, 1
HOST, DEVICE = 0, 1
(OPT_SCHEME, OPT_BAND_STEPS, OPT_WORKGROUPS, OPT_SPIN_LIMIT, OPT_PROFILE, OPT_MATERIAL_IDS,
 OPT_GRAPHS, OPT_TILE_X, OPT_AUTOTUNE_PLAIN) = range(9)
KERNEL_PLAIN_E, KERNEL_PLAIN_H, KERNEL_SOURCES, KERNEL_SYSTOLIC, KERNEL_PLAIN_FUSED = range(5)
(INFO_SYSTOLIC_GRID, INFO_SYSTOLIC_BAND, INFO_SYSTOLIC_TICKETS, INFO_RING_SLOTS, INFO_TILE_X,
 INFO_TILE_Y, INFO_TILE_Z, INFO_MATERIALS, INFO_SCHEME) = range(9)
# fdtd_invariants sums, in order
INVARIANT_NAMES = ("energy", "e_energy", "h_energy", "div_e_l1", "div_e_l2sq", "div_h_l1",
                   "div_h_l2sq")
SCHEMES = {"plain": SCHEME_PLAIN, "systolic": SCHEME_SYSTOLIC, "plain_fused": SCHEME_PLAIN_FUSED}

# every symbol the header declares
EXPORTS = ("fdtd_create", "fdtd_destroy", "fdtd_set_materials", "fdtd_set_lossy_materials",
           "fdtd_set_fields",
           "fdtd_add_source", "fdtd_step", "fdtd_step_batch", "fdtd_read_fields", "fdtd_synchronize",
           "fdtd_current_step", "fdtd_last_error", "fdtd_adjoint", "fdtd_set_option",
           "fdtd_kernel_stats", "fdtd_get_info", "fdtd_set_field_scale", "fdtd_invariants",
           "fdtd_invariants_noalloc", "fdtd_autotune",
           "fdtd_prepare")


class FdtdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dt", ctypes.c_double), ("dx", ctypes.c_double),
                ("bc", ctypes.c_int32 * 3), ("scheme", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class AdjointSpec(ctypes.Structure):
    """fdtd_adjoint_spec: monitor and design boxes are [lo, hi) per axis."""
    _fields_ = [("struct_size", ctypes.c_uint32), ("mon_comp", ctypes.c_int32),
                ("mon_lo", ctypes.c_int32 * 3), ("mon_hi", ctypes.c_int32 * 3),
                ("des_lo", ctypes.c_int32 * 3), ("des_hi", ctypes.c_int32 * 3),
                ("checkpoint_every", ctypes.c_int32), ("omega", ctypes.c_double),
                ("nsteps", ctypes.c_int64), ("objective", ctypes.c_double),
                ("recomputed_steps", ctypes.c_int64), ("isotropic", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libfdtd.so and declare its signatures; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfdtd.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch carries a HIP runtime of its own beside the one the library links;
    # bringing torch's up first lets both share the device (brought up after
    # the library's, torch finds no GPU), so device tensors can be passed in
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    fp = ctypes.POINTER(ctypes.c_float)
    sig = {
        "fdtd_create": ([ctypes.POINTER(Config), ctypes.POINTER(vp)], ctypes.c_int),
        "fdtd_destroy": ([vp], ctypes.c_int),
        "fdtd_set_materials": ([vp, vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "fdtd_set_lossy_materials": ([vp] + [vp] * 6 + [ctypes.c_int], ctypes.c_int),
        "fdtd_set_fields": ([vp, u32, ctypes.POINTER(vp), ctypes.c_int], ctypes.c_int),
        "fdtd_add_source": ([vp, ctypes.c_int, i32, i32, i32, vp, i64, i64, ctypes.c_int],
                            ctypes.c_int),
        "fdtd_step": ([vp, i64], ctypes.c_int),
        "fdtd_step_batch": ([ctypes.POINTER(vp), ctypes.c_int, i64], ctypes.c_int),
        "fdtd_read_fields": ([vp, u32, ctypes.POINTER(vp), ctypes.c_int], ctypes.c_int),
        "fdtd_synchronize": ([vp], ctypes.c_int),
        "fdtd_current_step": ([vp], i64),
        "fdtd_last_error": ([vp], ctypes.c_char_p),
        "fdtd_adjoint": ([vp, ctypes.POINTER(AdjointSpec), vp, ctypes.c_int], ctypes.c_int),
        "fdtd_set_option": ([vp, ctypes.c_int, i64], ctypes.c_int),
        "fdtd_kernel_stats": ([vp, ctypes.c_int, ctypes.POINTER(i64),
                               ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "fdtd_get_info": ([vp, ctypes.c_int, ctypes.POINTER(i64)], ctypes.c_int),
        "fdtd_set_field_scale": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "fdtd_invariants": ([vp, vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "fdtd_invariants_noalloc": ([vp, vp, vp, vp], ctypes.c_int),
        "fdtd_autotune": ([vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "fdtd_prepare": ([vp, i64], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _pointer(a, ncell: int):
    """(pointer, where, keepalive) for a numpy array or a torch CUDA tensor."""
    if _is_torch(a):
        import torch
        if a.dtype != torch.float32 or a.numel() != ncell or not a.is_contiguous():
            raise ValueError("device arrays must be contiguous float32 with %d elements" % ncell)
        if not a.is_cuda:
            a = a.numpy()
        else:
            return ctypes.c_void_p(a.data_ptr()), DEVICE, a
    arr = np.ascontiguousarray(a, dtype=np.float32)
    if arr.size != ncell:
        raise ValueError("host arrays must have %d elements" % ncell)
    return ctypes.c_void_p(arr.ctypes.data), HOST, arr


class Simulation:
    """One FDTD context.  ``shape`` = (nx, ny, nz); ``bc`` per axis 0 = PEC, 1 = periodic;
    ``storage`` "fp32" or "fp16" (binary16 device arrays, FP32 arithmetic)."""

    def __init__(self, shape: Sequence[int], dt: float = 0.5, dx: float = 1.0,
                 bc: Sequence[int] = (0, 0, 0), scheme: str = "plain", device: int = 0,
                 stream: Optional[int] = None, storage: str = "fp32"):
        self._lib = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.ncell = self.shape[0] * self.shape[1] * self.shape[2]
        cfg = Config()
        cfg.struct_size = ctypes.sizeof(Config)
        cfg.nx, cfg.ny, cfg.nz = self.shape
        cfg.dt, cfg.dx = float(dt), float(dx)
        for a in range(3):
            cfg.bc[a] = int(bc[a])
        cfg.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        cfg.storage = {"fp32": FP32, "fp16": FP16_STORAGE}[storage] if isinstance(storage, str) \
            else int(storage)
        cfg.device = int(device)
        cfg.stream = ctypes.c_void_p(stream) if stream else None
        h = ctypes.c_void_p()
        rc = self._lib.fdtd_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != FDTD_OK:
            raise FdtdError(rc, self._lib.fdtd_last_error(None).decode())
        self._h = h
        self.adjoint_recomputed_steps = None

    # -- helpers ------------------------------------------------------------
    def _check(self, rc: int) -> int:
        if rc < 0:
            raise FdtdError(rc, self._lib.fdtd_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fdtd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- API ------------------------------------------------------------------
    def set_materials(self, eps_x, eps_y=None, eps_z=None, sigma=None):
        """Permittivity per component (one array for all three if only eps_x);
        with ``sigma`` (one array or three) the materials are conductive."""
        eps_y = eps_x if eps_y is None else eps_y
        eps_z = eps_x if eps_z is None else eps_z
        arrays = [eps_x, eps_y, eps_z]
        if sigma is not None:
            arrays += list(sigma) if isinstance(sigma, (list, tuple)) else [sigma] * 3
        ptrs = [_pointer(e, self.ncell) for e in arrays]
        wheres = {p[1] for p in ptrs}
        if len(wheres) != 1:
            raise ValueError("all material arrays must live on the same side")
        if sigma is None:
            self._check(self._lib.fdtd_set_materials(self._h, ptrs[0][0], ptrs[1][0], ptrs[2][0],
                                                     ptrs[0][1]))
        else:
            self._check(self._lib.fdtd_set_lossy_materials(self._h, *[q[0] for q in ptrs],
                                                           ptrs[0][1]))

    def set_field_scale(self, exp2):
        """FP16 storage: component c is stored as v * 2^-exp2[c]."""
        arr = (ctypes.c_int32 * 6)(*[int(e) for e in exp2])
        self._check(self._lib.fdtd_set_field_scale(self._h, arr))

    def set_fields(self, fields, mask: Optional[int] = None):
        """``fields``: six arrays (None entries skipped) in (Ex..Hz) order."""
        arr = (ctypes.c_void_p * 6)()
        keep, where, m = [], None, 0
        for c, f in enumerate(fields):
            if f is None:
                continue
            p, w, k = _pointer(f, self.ncell)
            if where is not None and w != where:
                raise ValueError("all field arrays must live on the same side")
            where = w
            arr[c] = p
            keep.append(k)
            m |= 1 << c
        if mask is not None:
            m &= mask
        self._check(self._lib.fdtd_set_fields(self._h, m, arr, HOST if where is None else where))

    def add_source(self, comp: int, i: int, j: int, k: int, waveform, first_step: int = 0) -> int:
        w = np.ascontiguousarray(waveform, dtype=np.float32)
        return self._check(self._lib.fdtd_add_source(self._h, int(comp), int(i), int(j), int(k),
                                                     ctypes.c_void_p(w.ctypes.data), int(w.size),
                                                     int(first_step), HOST))

    def step(self, nsteps: int):
        self._check(self._lib.fdtd_step(self._h, int(nsteps)))

    def prepare(self, nsteps: int):
        """Build and upload what a call of ``nsteps`` steps needs (fdtd_prepare)."""
        self._check(self._lib.fdtd_prepare(self._h, int(nsteps)))

    def read_fields(self, mask: int = 0x3F, out=None):
        """Return a tuple of six arrays (None where not selected).  With ``out``
        (six torch CUDA tensors) the copy is device-to-device in stream order."""
        arr = (ctypes.c_void_p * 6)()
        res = [None] * 6
        where = HOST
        for c in range(6):
            if not (mask >> c) & 1:
                continue
            if out is not None:
                p, where, k = _pointer(out[c], self.ncell)
                res[c] = out[c]
            else:
                k = np.empty(self.shape, dtype=np.float32)
                p = ctypes.c_void_p(k.ctypes.data)
                res[c] = k
            arr[c] = p
        self._check(self._lib.fdtd_read_fields(self._h, mask, arr, where))
        return tuple(res)

    def synchronize(self):
        self._check(self._lib.fdtd_synchronize(self._h))

    @property
    def current_step(self) -> int:
        return int(self._lib.fdtd_current_step(self._h))

    def set_option(self, option: int, value: int):
        self._check(self._lib.fdtd_set_option(self._h, int(option), int(value)))

    def kernel_stats(self, kernel: int):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        self._check(self._lib.fdtd_kernel_stats(self._h, int(kernel), ctypes.byref(n),
                                                ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def info(self, key: int) -> int:
        v = ctypes.c_int64()
        self._check(self._lib.fdtd_get_info(self._h, int(key), ctypes.byref(v)))
        return int(v.value)

    def invariants(self, per_cell: bool = False, device_out=None):
        """FP64 invariants of the current state (fdtd_invariants): a dict of the
        sums in INVARIANT_NAMES order; with ``per_cell`` also the per-node
        divergence of eps E and per-cell divergence of H as float64 arrays of
        the grid's shape.  ``device_out`` = (sums, div_e, div_h) torch float64
        CUDA tensors (div entries may be None) keeps every output on the device
        (stream-ordered); the tensors are returned as given."""
        if device_out is not None:
            sums, de, dh = device_out
            ptr = [ctypes.c_void_p(t.data_ptr()) if t is not None else None for t in (sums, de, dh)]
            self._check(self._lib.fdtd_invariants(self._h, ptr[0], ptr[1], ptr[2], DEVICE))
            return device_out
        sums = np.zeros(len(INVARIANT_NAMES), np.float64)
        de = np.empty(self.shape, np.float64) if per_cell else None
        dh = np.empty(self.shape, np.float64) if per_cell else None
        self._check(self._lib.fdtd_invariants(
            self._h, ctypes.c_void_p(sums.ctypes.data),
            ctypes.c_void_p(de.ctypes.data) if per_cell else None,
            ctypes.c_void_p(dh.ctypes.data) if per_cell else None, HOST))
        out = dict(zip(INVARIANT_NAMES, (float(v) for v in sums)))
        if per_cell:
            return out, de, dh
        return out

    def autotune(self, nsteps: int):
        """fdtd_autotune: time the systolic tile widths and band lengths for
        calls of ``nsteps`` steps and keep the fastest; returns (tile_x, band)."""
        w, k = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.fdtd_autotune(self._h, int(nsteps), ctypes.byref(w), ctypes.byref(k)))
        return int(w.value), int(k.value)

    def invariants_noalloc(self, sums, div_e=None, div_h=None):
        """fdtd_invariants_noalloc: the invariants into torch float64 CUDA
        tensors (sums of INVARIANT_NAMES length; div_e, div_h of the grid's
        cell count, or None), stream-ordered, with no allocation in the
        library.  Returns the tensors as given."""
        ptr = [ctypes.c_void_p(t.data_ptr()) if t is not None else None for t in (sums, div_e, div_h)]
        self._check(self._lib.fdtd_invariants_noalloc(self._h, ptr[0], ptr[1], ptr[2]))
        return sums, div_e, div_h

    def adjoint(self, nsteps: int, mon_comp: int, mon_lo, mon_hi, omega: float, des_lo, des_hi,
                checkpoint_every: int = 0, out=None, isotropic: bool = False):
        """Run ``nsteps`` forward with the monitor transform, then the reverse
        sweep.  Returns (J, grad) with grad of shape (3, *design box) holding
        dJ/deps_x, dJ/deps_y, dJ/deps_z (with ``isotropic``, shape (*design
        box): the derivative for one permittivity per cell, which the library
        sums over the components); with ``out`` (a torch CUDA tensor of that
        shape) the gradient is written there on the device.
        ``checkpoint_every`` is the segment length (0: automatic); the number
        of forward steps the sweep ran again is left in
        ``self.adjoint_recomputed_steps``."""
        spec = AdjointSpec()
        spec.struct_size = ctypes.sizeof(AdjointSpec)
        spec.mon_comp = int(mon_comp)
        for a in range(3):
            spec.mon_lo[a], spec.mon_hi[a] = int(mon_lo[a]), int(mon_hi[a])
            spec.des_lo[a], spec.des_hi[a] = int(des_lo[a]), int(des_hi[a])
        spec.checkpoint_every = int(checkpoint_every)
        spec.omega = float(omega)
        spec.nsteps = int(nsteps)
        spec.isotropic = int(isotropic)    # the library refuses anything but 0 and 1
        shape = (() if isotropic else (3,)) + tuple(int(des_hi[a]) - int(des_lo[a]) for a in range(3))
        if out is not None:
            if not _is_torch(out) or not out.is_cuda or tuple(out.shape) != shape or \
                    str(out.dtype) != "torch.float32" or not out.is_contiguous():
                raise ValueError("out must be a contiguous float32 CUDA tensor of shape %s" % (shape,))
            self._check(self._lib.fdtd_adjoint(self._h, ctypes.byref(spec),
                                               ctypes.c_void_p(out.data_ptr()), DEVICE))
            self.adjoint_recomputed_steps = int(spec.recomputed_steps)
            return spec.objective, out
        g = np.zeros(shape, np.float32)
        self._check(self._lib.fdtd_adjoint(self._h, ctypes.byref(spec),
                                           ctypes.c_void_p(g.ctypes.data), HOST))
        self.adjoint_recomputed_steps = int(spec.recomputed_steps)
        return spec.objective, g


class DesignProblem:
    """An inverse-design objective for :func:`design_objective`: a base
    permittivity map (numpy float32, all three components share it), the
    boundaries and step sizes, the sources, and the fdtd_adjoint arguments
    (monitor and design boxes, omega, nsteps, checkpoint_every).  An optional
    conductivity map ``sigma`` (shared by the three components, held fixed)
    makes the materials conductive.  Every evaluation starts from zero fields
    at step 0."""

    def __init__(self, eps, bc, dt, dx, sources, adjoint_args, device: int = 0, sigma=None):
        self.eps = np.ascontiguousarray(eps, dtype=np.float32)
        self.sigma = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.float32)
        self.bc, self.dt, self.dx = tuple(bc), float(dt), float(dx)
        self.sources = list(sources)
        self.args = dict(adjoint_args)
        self.device = int(device)

    def evaluate(self, eps_design: np.ndarray):
        """(J, dJ/deps over the design box) for the given design permittivity."""
        lo, hi = self.args["des_lo"], self.args["des_hi"]
        eps = self.eps.copy()
        eps[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = eps_design
        sim = Simulation(eps.shape, self.dt, self.dx, self.bc, scheme="plain", device=self.device)
        try:
            sim.set_materials(eps, sigma=self.sigma)
            for s in self.sources:
                sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"],
                               s.get("first_step", 0))
            # one permittivity per cell drives all three components
            J, g = sim.adjoint(**self.args, isotropic=True)
        finally:
            sim.close()
        return J, g


def design_objective(eps_design, problem: DesignProblem):
    """J(eps_design) as a differentiable torch scalar: the forward value and
    its gradient both come from one fdtd_adjoint call."""
    import torch

    class _Objective(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            J, g = problem.evaluate(x.detach().to("cpu", torch.float32).numpy())
            ctx.save_for_backward(torch.from_numpy(g).to(x.device, torch.float64))
            return torch.tensor(J, dtype=torch.float64, device=x.device)

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            return (gJ * g).to(eps_design.dtype)

    return _Objective.apply(eps_design)


def step_batch(sims: Sequence["Simulation"], nsteps: int):
    """Advance several Simulation objects by nsteps each in one persistent
    systolic launch (fdtd_step_batch)."""
    sims = list(sims)
    if not sims:
        raise ValueError("step_batch needs at least one simulation")
    lib = sims[0]._lib
    arr = (ctypes.c_void_p * len(sims))(*[s._h.value for s in sims])
    rc = lib.fdtd_step_batch(arr, len(sims), int(nsteps))
    if rc < 0:
        raise FdtdError(rc, lib.fdtd_last_error(sims[0]._h).decode())


def run_workload(w, scheme: str = "plain", nsteps: Optional[int] = None, device: int = 0,
                 options=None, storage: str = "fp32", field_exp2=None):
    """Run a workloads.Workload through the library and return the six fields (host)."""
    sim = Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, device=device, storage=storage)
    try:
        for k, v in (options or {}).items():
            sim.set_option(k, v)
        if field_exp2 is not None:
            sim.set_field_scale(field_exp2)
        sim.set_materials(w.eps)
        if w.fields is not None:
            sim.set_fields(w.fields)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"], s.get("first_step", 0))
        sim.step(w.nsteps if nsteps is None else nsteps)
        return sim.read_fields()
    finally:
        sim.close()
